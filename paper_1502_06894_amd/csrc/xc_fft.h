// Register/LDS Stockham FFT (forward, exp(-2 pi i k n / N), unnormalised).
//
// A group of T threads transforms one N-point frame.  Each thread holds
// E = N / T complex values in registers; a pass of radix R performs E / R
// radix-R butterflies per thread and exchanges through LDS (autosort
// Stockham indexing, so the output is in natural order without a bit-reversal
// pass).  Thread t owns input samples n = t + e T (e = 0 .. E-1) on entry and
// output bins k = j + r N / R_last on exit.
#pragma once

#include <hip/hip_runtime.h>

#include "xc_dev.h"

namespace xc {

__device__ inline float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ inline float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
// multiply by -i
__device__ inline float2 mul_mi(float2 a) { return make_float2(a.y, -a.x); }

template <int R>
struct Dft;

template <>
struct Dft<2> {
  __device__ static inline void run(float2* v) {
    const float2 a = v[0], b = v[1];
    v[0] = cadd(a, b);
    v[1] = csub(a, b);
  }
};

template <>
struct Dft<4> {
  __device__ static inline void run(float2* v) {
    const float2 t0 = cadd(v[0], v[2]), t1 = csub(v[0], v[2]);
    const float2 t2 = cadd(v[1], v[3]), t3 = mul_mi(csub(v[1], v[3]));
    v[0] = cadd(t0, t2);
    v[2] = csub(t0, t2);
    v[1] = cadd(t1, t3);
    v[3] = csub(t1, t3);
  }
};

template <>
struct Dft<8> {
  __device__ static inline void run(float2* v) {
    constexpr float c = 0.70710678118654752440f;
    float2 e[4] = {v[0], v[2], v[4], v[6]};
    float2 o[4] = {v[1], v[3], v[5], v[7]};
    Dft<4>::run(e);
    Dft<4>::run(o);
    // o[k] *= exp(-2 pi i k / 8)
    o[1] = make_float2(c * (o[1].x + o[1].y), c * (o[1].y - o[1].x));
    o[2] = mul_mi(o[2]);
    o[3] = make_float2(c * (o[3].y - o[3].x), -c * (o[3].x + o[3].y));
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      v[k] = cadd(e[k], o[k]);
      v[k + 4] = csub(e[k], o[k]);
    }
  }
};

template <>
struct Dft<16> {
  __device__ static inline void run(float2* v) {
    // exp(-2 pi i k / 16), k = 0..7
    constexpr float c1 = 0.92387953251128675613f, s1 = 0.38268343236508977173f;
    constexpr float c2 = 0.70710678118654752440f;
    float2 e[8], o[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      e[k] = v[2 * k];
      o[k] = v[2 * k + 1];
    }
    Dft<8>::run(e);
    Dft<8>::run(o);
    o[1] = cmul(o[1], make_float2(c1, -s1));
    o[2] = make_float2(c2 * (o[2].x + o[2].y), c2 * (o[2].y - o[2].x));
    o[3] = cmul(o[3], make_float2(s1, -c1));
    o[4] = mul_mi(o[4]);
    o[5] = cmul(o[5], make_float2(-s1, -c1));
    o[6] = make_float2(c2 * (o[6].y - o[6].x), -c2 * (o[6].x + o[6].y));
    o[7] = cmul(o[7], make_float2(-c1, -s1));
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      v[k] = cadd(e[k], o[k]);
      v[k + 8] = csub(e[k], o[k]);
    }
  }
};

// LDS index with padding: one float2 of padding every 32 entries.
__device__ inline int lds_pad(int i) { return i + (i >> 5); }

template <int N>
constexpr int lds_words() {
  return N + N / 32;
}

// Radix of the first pass for N = 2^L2: 16 when L2 is a multiple of 4, else 2^(L2 mod 4).
template <int N>
constexpr int first_radix() {
  return (__builtin_ctz(N) % 4) == 0 ? 16 : (1 << (__builtin_ctz(N) % 4));
}

// Twiddle sources for the Stockham passes.  Only radix-16 passes with
// sub-transform length Ns > 1 take twiddles: input r of butterfly j is
// multiplied by exp(-2 pi i k r / (16 Ns)), k = j mod Ns.
// TwGlobal reads them from the kTwiddleN-entry table in memory.
struct TwGlobal {
  const float2* __restrict__ tw;
  template <int R, int Ns>
  __device__ float2 get(int k, int r) const {
    return tw[k * r * (kTwiddleN / (Ns * R))];
  }
};

// TwLds reads them from per-pass tables staged in LDS: the pass with
// sub-transform length Ns (= R0, 16 R0, 256 R0, ...) owns 15 Ns entries from
// offset Ns - R0, entry (r - 1) Ns + k; a thread's 15 twiddles are one address
// plus compile-time offsets.  All passes together take N - R0 entries.
template <int N>
struct TwLds {
  const float2* tab;
  template <int R, int Ns>
  __device__ float2 get(int k, int r) const {
    return tab[(Ns - first_radix<N>()) + (r - 1) * Ns + k];
  }
};

template <int N>
constexpr int tw_lds_entries() {
  return N - first_radix<N>();
}

// Fill the TwLds tables of an N-point transform (threads tid, tid + nthr, ...).
template <int N>
__device__ inline void tw_lds_fill(float2* tab, const float2* __restrict__ tw, int tid, int nthr) {
  constexpr int R0 = first_radix<N>();
  for (int e = tid; e < tw_lds_entries<N>(); e += nthr) {
    int Ns = R0;
    while (e >= 16 * Ns - R0) Ns *= 16;
    const int e2 = e - (Ns - R0);
    const int r = e2 / Ns + 1, k = e2 - (r - 1) * Ns;
    tab[e] = tw[k * r * (kTwiddleN / (Ns * 16))];
  }
}

// TwSplit keeps the TwLds tables of every pass but the last, plus a 15 x 16
// table exp(-2 pi i kl r / N) (entry (r - 1) 16 + kl) after them.  The last
// pass (Ns = N / 16) forms its twiddle for k = 16 kh + kl as a product:
// exp(-2 pi i k r / N) = exp(-2 pi i kh r / Ns) exp(-2 pi i kl r / N), the
// first factor being the previous pass's entry (r - 1) Ns/16 + kh.  The
// tables shrink from N - R0 to N/16 - R0 + 240 entries for one complex
// multiply per last-pass twiddle.  Needs N >= 512 (a radix-16 pass with
// Ns > 1 before the last).
template <int N>
struct TwSplit {
  const float2* tab;
  template <int R, int Ns>
  __device__ float2 get(int k, int r) const {
    constexpr int R0 = first_radix<N>();
    if constexpr (Ns < N / 16) {
      return tab[(Ns - R0) + (r - 1) * Ns + k];
    } else {
      constexpr int Np = Ns / 16;
      static_assert(Np >= R0, "TwSplit needs a twiddled pass before the last");
      const float2 a = tab[(Np - R0) + (r - 1) * Np + (k >> 4)];
      const float2 b = tab[(N / 16 - R0) + (r - 1) * 16 + (k & 15)];
      return cmul(a, b);
    }
  }
};

template <int N>
constexpr int tw_split_entries() {
  return N / 16 - first_radix<N>() + 15 * 16;
}

template <int N>
__device__ inline void tw_split_fill(float2* tab, const float2* __restrict__ tw, int tid, int nthr) {
  constexpr int R0 = first_radix<N>();
  constexpr int base = N / 16 - R0;
  for (int e = tid; e < tw_split_entries<N>(); e += nthr) {
    if (e < base) {
      int Ns = R0;
      while (e >= 16 * Ns - R0) Ns *= 16;
      const int e2 = e - (Ns - R0);
      const int r = e2 / Ns + 1, k = e2 - (r - 1) * Ns;
      tab[e] = tw[k * r * (kTwiddleN / (Ns * 16))];
    } else {
      const int e2 = e - base;
      const int r = e2 / 16 + 1, kl = e2 % 16;
      tab[e] = tw[kl * r * (kTwiddleN / N)];
    }
  }
}

// For every pass and gather of the plans below, lds_pad(i + r S) =
// lds_pad(i) + r S + (r S) / 32: the stride S is a power of two and i's place
// in its 32-entry run plus (r S) mod 32 stays below 32 (S a multiple of 32; or
// i mod 32 < S with S R a multiple of 32; or a first pass whose R outputs start
// on a multiple of R), so adding r S carries no padding slot beyond (r S) / 32.
// Written as one padded base plus compile-time offsets, the compiler keeps one
// address per butterfly instead of one per output (R registers that the lean
// F-stage tasks would otherwise spill).
template <int S>
constexpr int pad_off(int r) {
  return r * S + (r * S) / 32;
}

// One Stockham pass of radix R with sub-transform length Ns over a frame of N
// points.  On entry v[b + r B] (B = E/R) is input r of butterfly j = t + b T;
// the outputs are written to lds; the caller synchronises.
template <int N, int T, int E, int R, int Ns, class TW>
__device__ inline void stockham_pass(float2 (&v)[E], float2* lds, const TW& tw, int t) {
  constexpr int B = E / R;
  static_assert(B * R == E, "radix must divide the per-thread count");
#pragma unroll
  for (int b = 0; b < B; ++b) {
    const int j = t + b * T;
    float2 u[R];
#pragma unroll
    for (int r = 0; r < R; ++r) u[r] = v[b + r * B];
    if constexpr (Ns > 1) {
      const int k = j % Ns;
#pragma unroll
      for (int r = 1; r < R; ++r) u[r] = cmul(u[r], tw.template get<R, Ns>(k, r));
    }
    Dft<R>::run(u);
    const int idx = (j / Ns) * Ns * R + (j % Ns);
    float2* o = lds + lds_pad(idx);
#pragma unroll
    for (int r = 0; r < R; ++r) o[pad_off<Ns>(r)] = u[r];
  }
}

// Gather the inputs of the next pass (radix R) from lds: v[b + r B] = x[j + r N / R].
template <int N, int T, int E, int R>
__device__ inline void stockham_gather(float2 (&v)[E], const float2* lds, int t) {
  constexpr int B = E / R;
#pragma unroll
  for (int b = 0; b < B; ++b) {
    const int j = t + b * T;
    const float2* x = lds + lds_pad(j);
#pragma unroll
    for (int r = 0; r < R; ++r) v[b + r * B] = x[pad_off<N / R>(r)];
  }
}

// Last pass: radix R with Ns = N / R; the butterfly outputs are final bins
// k = j + r N / R and stay in registers (v[b + r B]).
template <int N, int T, int E, int R, class TW>
__device__ inline void stockham_last(float2 (&v)[E], const TW& tw, int t) {
  constexpr int B = E / R;
  constexpr int Ns = N / R;
#pragma unroll
  for (int b = 0; b < B; ++b) {
    const int j = t + b * T;
    float2 u[R];
#pragma unroll
    for (int r = 0; r < R; ++r) u[r] = v[b + r * B];
    const int k = j % Ns;
#pragma unroll
    for (int r = 1; r < R; ++r) u[r] = cmul(u[r], tw.template get<R, Ns>(k, r));
    Dft<R>::run(u);
#pragma unroll
    for (int r = 0; r < R; ++r) v[b + r * B] = u[r];
  }
}

// Plan: radices for each N with T threads per frame and E values per thread.
template <int N>
struct FftPlan;

// N = 256: T = 16, E = 16: 16 x 16 (32..128: short transforms, e.g. over
// sub-integrations)
template <> struct FftPlan<32>    { static constexpr int T = 2,    E = 16; };
template <> struct FftPlan<64>    { static constexpr int T = 4,    E = 16; };
template <> struct FftPlan<128>   { static constexpr int T = 8,    E = 16; };
template <> struct FftPlan<256>   { static constexpr int T = 16,   E = 16; };
template <> struct FftPlan<512>   { static constexpr int T = 32,   E = 16; };
template <> struct FftPlan<1024>  { static constexpr int T = 64,   E = 16; };
template <> struct FftPlan<2048>  { static constexpr int T = 128,  E = 16; };
template <> struct FftPlan<4096>  { static constexpr int T = 256,  E = 16; };
template <> struct FftPlan<8192>  { static constexpr int T = 512,  E = 16; };
template <> struct FftPlan<16384> { static constexpr int T = 1024, E = 16; };

// Full transform, radix sequence: 32 = 2.16, 64 = 4.16, 128 = 8.16,
// 256 = 16.16, 512 = 2.16.16, 1024 = 4.16.16,
// 2048 = 8.16.16, 4096 = 16.16.16, 8192 = 2.16.16.16, 16384 = 4.16.16.16.
// On entry v[e] = x[t + e T]; on exit v[b + r B_last] = X[t + b T + r N / 16].
// `lds` holds lds_words<N>() float2; the group's threads synchronise with
// __syncthreads (the whole workgroup runs the same pass sequence).
template <int N, class TW>
__device__ inline void fft_forward(float2 (&v)[FftPlan<N>::E], float2* lds, const TW& tw, int t) {
  constexpr int T = FftPlan<N>::T, E = FftPlan<N>::E;
  constexpr int L2 = __builtin_ctz(N);
  // number of radix-16 passes after the first (mixed) pass
  constexpr int n16 = (L2 / 4) - ((L2 % 4) == 0 ? 1 : 0);
  constexpr int R0 = first_radix<N>();
  stockham_pass<N, T, E, R0, 1>(v, lds, tw, t);
  __syncthreads();
  stockham_gather<N, T, E, 16>(v, lds, t);
  if constexpr (n16 >= 2) {
    __syncthreads();
    stockham_pass<N, T, E, 16, R0>(v, lds, tw, t);
    __syncthreads();
    stockham_gather<N, T, E, 16>(v, lds, t);
  }
  if constexpr (n16 >= 3) {
    __syncthreads();
    stockham_pass<N, T, E, 16, R0 * 16>(v, lds, tw, t);
    __syncthreads();
    stockham_gather<N, T, E, 16>(v, lds, t);
  }
  static_assert(n16 <= 3, "plan supports up to 3 radix-16 passes after the first");
  stockham_last<N, T, E, 16>(v, tw, t);
}

}  // namespace xc
