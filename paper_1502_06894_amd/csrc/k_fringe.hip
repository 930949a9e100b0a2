// Delay-rate fringe search over stacked sub-integrations (the search behind
// the paper's first-fringe result, section 2): a zero-padded FFT over the
// channels of every (sub-integration, subband, baseline) row, then per
// (subband, baseline) a zero-padded FFT over sub-integrations of every delay
// column, the windowed peak and its parabolic refinement.
#include <math.h>

#include <atomic>

#include "xc_fft.h"
#include "xc_launch.h"
#include "xc_runtime.h"

namespace xc {

// Delay transform: rows q = (t, sb, bl) of vis [T][n_sb][nbl][n_chan], each
// zero-padded to D, into F [n_sb][nbl][T][D].  A workgroup runs kDelayIters
// groups of G rows (T threads a row, as in the F stage's FFT), with the
// twiddles in LDS tables filled once: the full per-pass tables up to D = 2048,
// the split ones above (less LDS, more resident workgroups).
constexpr int kDelayIters = 4;

template <int D>
struct RowGeom {
  static constexpr int T = FftPlan<D>::T;
  static constexpr int E = FftPlan<D>::E;
  static constexpr int G = T >= 256 ? 1 : 256 / T;
  static constexpr int WG = T * G;
  static constexpr bool split = D >= 4096;
  static constexpr int tw_entries = split ? tw_split_entries<D>() : tw_lds_entries<D>();
  static constexpr size_t lds_bytes =
      ((size_t)G * lds_words<D>() + (size_t)tw_entries) * sizeof(float2);
};

template <int D>
__global__ void __launch_bounds__(RowGeom<D>::WG)
    k_fringe_delay(const float2* __restrict__ vis, float2* __restrict__ F,
                   const float2* __restrict__ tw, int n_sub, int n_sb, int nbl, int n_chan) {
  using Gm = RowGeom<D>;
  constexpr int T = Gm::T, E = Gm::E, G = Gm::G;
  extern __shared__ float2 lds_all[];
  float2* tab = lds_all + G * lds_words<D>();
  if constexpr (Gm::split)
    tw_split_fill<D>(tab, tw, threadIdx.x, blockDim.x);
  else
    tw_lds_fill<D>(tab, tw, threadIdx.x, blockDim.x);
  const int g = threadIdx.x / T, t = threadIdx.x % T;
  const long n_rows = (long)n_sub * n_sb * nbl;
#pragma unroll 1
  for (int it = 0; it < kDelayIters; ++it) {
    __syncthreads();   // tables written / the previous group's exchange done
    const long q = ((long)blockIdx.x * kDelayIters + it) * G + g;
    // the row's indices (rows past the end transform zeros and store nothing)
    const bool live = q < n_rows;
    const long qq = live ? q : 0;
    const int bl = (int)(qq % nbl);
    const int sb = (int)((qq / nbl) % n_sb);
    const int ts = (int)(qq / ((long)nbl * n_sb));
    const float2* x = vis + qq * n_chan;
    float2 v[E];
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const int n = t + e * T;
      v[e] = live && n < n_chan ? x[n] : make_float2(0.f, 0.f);
    }
    if constexpr (Gm::split)
      fft_forward<D>(v, lds_all + g * lds_words<D>(), TwSplit<D>{tab}, t);
    else
      fft_forward<D>(v, lds_all + g * lds_words<D>(), TwLds<D>{tab}, t);
    if (!live) continue;
    float2* out = F + (((size_t)sb * nbl + bl) * n_sub + ts) * D;
    constexpr int B = E / 16;
#pragma unroll
    for (int b = 0; b < B; ++b)
#pragma unroll
      for (int r = 0; r < 16; ++r) out[t + b * T + r * (D / 16)] = v[b + r * B];
  }
}

// Rate transform, peak and refinement: one workgroup (256 threads) per
// (subband, baseline) map.  Each round takes GC delay columns; a column's
// R-point transform over sub-integrations (zero-padded from n_sub) runs on
// TR = R/16 threads of 16 values (the LDS Stockham FFT) for R >= 32, or in one
// thread's registers for R <= 16.  Thread (tl, c) = threadIdx tl GC + c, so a
// wave's loads of one sub-integration row are consecutive columns.
constexpr int kFringeThreads = 256;

template <int R>
struct RateGeom {
  static constexpr bool fft = R >= 32;
  static constexpr int TR = fft ? R / 16 : 1;       // threads per column
  static constexpr int E = fft ? 16 : R;            // values per thread
  static constexpr int GC = kFringeThreads / TR;    // columns per round
  static constexpr size_t lds_bytes =
      fft ? ((size_t)GC * lds_words<R>() + (size_t)tw_lds_entries<R>()) * sizeof(float2) : 0;
};

template <int R>
__device__ inline void small_dft(float2 (&v)[R]) {
  if constexpr (R > 1) Dft<R>::run(v);
}

// signed bin: [-n/2, n/2) for even n; a one-point axis has the single bin 0
__device__ inline int signed_bin(int b, int n) { return b >= (n + 1) / 2 ? b - n : b; }

// |G|^2 ordering with the tie rule: larger value first, then smaller index.
__device__ inline bool better(float a, int ia, float b, int ib) {
  return a > b || (a == b && ia < ib);
}

// G[r, d] by direct summation over sub-integrations (the refinement's
// neighbours), twiddles exp(-2 pi i m / R) from the global table
__device__ inline float2 rate_point(const float2* __restrict__ Fm, const float2* __restrict__ tw,
                                    int n_sub, int R, int D, int r, int d) {
  float2 acc = make_float2(0.f, 0.f);
  int m = 0;
  for (int ts = 0; ts < n_sub; ++ts) {
    const float2 f = Fm[(size_t)ts * D + d];
    const float2 w = tw[(size_t)m * (kTwiddleN / R)];
    acc.x = fmaf(f.x, w.x, fmaf(-f.y, w.y, acc.x));
    acc.y = fmaf(f.x, w.y, fmaf(f.y, w.x, acc.y));
    m = (m + r) & (R - 1);
  }
  return acc;
}

__device__ inline float parabola_off(float am, float a0, float ap) {
  const float den = am - 2.f * a0 + ap;
  return den == 0.f ? 0.f : (am - ap) / (2.f * den);
}

template <int R>
__global__ void __launch_bounds__(kFringeThreads)
    k_fringe_rate(const float2* __restrict__ F, const float2* __restrict__ tw,
                  xc_fringe_peak* __restrict__ peaks, float2* __restrict__ map, int n_sub, int D,
                  int n_chan, int delay_win, int rate_win, double dnu, double t_int) {
  using Rg = RateGeom<R>;
  constexpr int TR = Rg::TR, E = Rg::E, GC = Rg::GC;
  extern __shared__ float2 sh[];
  __shared__ float best_v[kFringeThreads];
  __shared__ int best_i[kFringeThreads];
  const int map_id = blockIdx.x;
  const float2* Fm = F + (size_t)map_id * n_sub * D;
  float2* tab = sh + GC * (Rg::fft ? lds_words<R>() : 0);
  if constexpr (Rg::fft) tw_lds_fill<R>(tab, tw, threadIdx.x, blockDim.x);
  const int c = threadIdx.x % GC, tl = threadIdx.x / GC;
  float bv = -1.f;
  int bi = 0x7fffffff;
  auto load = [&](float2 (&v)[E], int d) {
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const int ts = tl + e * TR;
      v[e] = ts < n_sub ? Fm[(size_t)ts * D + d] : make_float2(0.f, 0.f);
    }
  };
  auto search = [&](float2 (&v)[E], int d) {
    if constexpr (Rg::fft) {
      __syncthreads();   // tables written / the previous round's exchange done
      fft_forward<R>(v, sh + c * lds_words<R>(), TwLds<R>{tab}, tl);
    } else {
      small_dft<R>(v);
    }
    // v[j] = G[tl + j R/16, d] (FFT), G[j, d] (registers); r grows with j
    auto rate_of = [&](int j) { return Rg::fft ? tl + j * (R / 16) : j; };
    if (map) {
#pragma unroll
      for (int j = 0; j < E; ++j) map[((size_t)map_id * R + rate_of(j)) * D + d] = v[j];
    }
    // the round's largest |G|^2 (first j on ties: the smallest index r D + d),
    // then one comparison with the thread's best under the tie rule
    float m = -1.f;
    int mj = 0;
    if (delay_win <= 0 && rate_win <= 0) {
#pragma unroll
      for (int j = 0; j < E; ++j) {
        const float a2 = v[j].x * v[j].x + v[j].y * v[j].y;
        if (a2 > m) {
          m = a2;
          mj = j;
        }
      }
    } else {
      const int ds = signed_bin(d, D);
      const bool d_in = delay_win <= 0 || (ds <= delay_win && ds >= -delay_win);
#pragma unroll
      for (int j = 0; j < E; ++j) {
        const int rs = signed_bin(rate_of(j), R);
        const bool in = d_in && (rate_win <= 0 || (rs <= rate_win && rs >= -rate_win));
        const float a2 = v[j].x * v[j].x + v[j].y * v[j].y;
        if (in && a2 > m) {
          m = a2;
          mj = j;
        }
      }
    }
    const int idx = rate_of(mj) * D + d;
    if (m >= 0.f && better(m, idx, bv, bi)) {
      bv = m;
      bi = idx;
    }
  };
  // D >= 256 is a multiple of GC (<= 256): every round is full.  Two rounds'
  // columns are loaded together, so the second's loads overlap the first's
  // transform.
#pragma unroll 1
  for (int d0 = 0; d0 < D; d0 += 2 * GC) {
    const bool two = d0 + GC < D;
    float2 v0[E], v1[E];
    load(v0, d0 + c);
    if (two) load(v1, d0 + GC + c);
    search(v0, d0 + c);
    if (two) search(v1, d0 + GC + c);
  }
  best_v[threadIdx.x] = bv;
  best_i[threadIdx.x] = bi;
  __syncthreads();
  for (int w = kFringeThreads / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w &&
        better(best_v[threadIdx.x + w], best_i[threadIdx.x + w], best_v[threadIdx.x],
               best_i[threadIdx.x])) {
      best_v[threadIdx.x] = best_v[threadIdx.x + w];
      best_i[threadIdx.x] = best_i[threadIdx.x + w];
    }
    __syncthreads();
  }
  // the peak value and its four cyclic neighbours, recomputed from memory
  __shared__ float2 pts[5];
  const int pi = best_i[0];
  const int pr = pi / D, pd = pi - pr * D;
  if (threadIdx.x < 5) {
    const int k = threadIdx.x;
    const int rr = k == 3 ? (pr + R - 1) % R : k == 4 ? (pr + 1) % R : pr;
    const int dd = k == 1 ? (pd + D - 1) % D : k == 2 ? (pd + 1) % D : pd;
    pts[k] = rate_point(Fm, tw, n_sub, R, D, rr, dd);
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    auto mag = [](float2 z) { return sqrtf(z.x * z.x + z.y * z.y); };
    const float a0 = mag(pts[0]);
    const float od = parabola_off(mag(pts[1]), a0, mag(pts[2]));
    const float orr = parabola_off(mag(pts[3]), a0, mag(pts[4]));
    const int ds = signed_bin(pd, D), rs = signed_bin(pr, R);
    xc_fringe_peak p;
    p.delay_bin = ds;
    p.rate_bin = rs;
    p.amp = a0 / ((float)n_chan * (float)n_sub);
    p.phase = atan2f(pts[0].y, pts[0].x);
    p.delay_off = od;
    p.rate_off = orr;
    p.delay_s = ((double)ds + (double)od) / ((double)D * dnu);
    p.rate_hz = ((double)rs + (double)orr) / ((double)R * t_int);
    peaks[map_id] = p;
  }
}

// One attribute call per kernel and device (LDS above 64 KB).
template <class K>
static hipError_t allow_lds(K kernel, size_t bytes, std::atomic<bool> (&done)[64]) {
  if (bytes <= 65536) return hipSuccess;
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= 64) return hipErrorInvalidDevice;
  if (done[dev].load()) return hipSuccess;
  e = hipFuncSetAttribute((const void*)kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                          (int)bytes);
  if (e == hipSuccess) done[dev].store(true);
  return e;
}

template <int D>
static hipError_t launch_delay_d(const float2* vis, float2* F, const float2* tw, int n_sub,
                                 int n_sb, int nbl, int n_chan, hipStream_t s) {
  using Gm = RowGeom<D>;
  static std::atomic<bool> done[64];
  hipError_t e = allow_lds(k_fringe_delay<D>, Gm::lds_bytes, done);
  if (e != hipSuccess) return e;
  const long rows = (long)n_sub * n_sb * nbl;
  const long per_wg = (long)Gm::G * kDelayIters;
  hipLaunchKernelGGL(k_fringe_delay<D>, dim3((unsigned)((rows + per_wg - 1) / per_wg)),
                     dim3(Gm::WG), Gm::lds_bytes, s, vis, F, tw, n_sub, n_sb, nbl, n_chan);
  return hipGetLastError();
}

template <int R>
static hipError_t launch_rate_r(const xc_fringe_setup* fs, const float2* F, const float2* tw,
                                xc_fringe_peak* peaks, float2* map, hipStream_t s) {
  static std::atomic<bool> done[64];
  hipError_t e = allow_lds(k_fringe_rate<R>, RateGeom<R>::lds_bytes, done);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_fringe_rate<R>, dim3(fs->n_subbands * fs->n_baselines),
                     dim3(kFringeThreads), RateGeom<R>::lds_bytes, s, F, tw, peaks, map,
                     fs->n_subints, fs->delay_len, fs->n_chan, fs->delay_win, fs->rate_win,
                     fs->chan_width_hz, fs->t_int_s);
  return hipGetLastError();
}

hipError_t launch_fringe(const xc_fringe_setup* fs, const float2* vis, float2* F,
                         const float2* tw, xc_fringe_peak* peaks, float2* map, hipStream_t s) {
  hipError_t e;
  switch (fs->delay_len) {
#define XC_DCASE(DD)                                                                        \
  case DD:                                                                                  \
    e = launch_delay_d<DD>(vis, F, tw, fs->n_subints, fs->n_subbands, fs->n_baselines,      \
                           fs->n_chan, s);                                                  \
    break;
    XC_DCASE(256) XC_DCASE(512) XC_DCASE(1024) XC_DCASE(2048) XC_DCASE(4096) XC_DCASE(8192)
    XC_DCASE(16384)
#undef XC_DCASE
    default: return hipErrorInvalidValue;
  }
  if (e != hipSuccess) return e;
  switch (fs->rate_len) {
#define XC_RCASE(RR) \
  case RR: return launch_rate_r<RR>(fs, F, tw, peaks, map, s);
    XC_RCASE(1) XC_RCASE(2) XC_RCASE(4) XC_RCASE(8) XC_RCASE(16) XC_RCASE(32) XC_RCASE(64)
    XC_RCASE(128) XC_RCASE(256) XC_RCASE(512) XC_RCASE(1024)
#undef XC_RCASE
    default: return hipErrorInvalidValue;
  }
}

}  // namespace xc

using namespace xc;

namespace {

bool is_pow2(long x) { return x > 0 && (x & (x - 1)) == 0; }

int fringe_validate(xc_ctx* c, const xc_fringe_setup* fs) {
  if (!fs) return fail(c, XC_E_INVAL, "fringe setup is NULL");
  if (fs->n_subints < 1 || fs->n_subints > 256)
    return fail(c, XC_E_INVAL, "n_subints=%d outside 1..256", fs->n_subints);
  if (fs->n_subbands < 1 || fs->n_baselines < 1 || fs->n_chan < 1)
    return fail(c, XC_E_INVAL, "empty fringe search");
  if (!is_pow2(fs->delay_len) || fs->delay_len < 256 || fs->delay_len > 16384 ||
      fs->delay_len < fs->n_chan)
    return fail(c, XC_E_INVAL, "delay_len=%d: power of two in 256..16384 and >= n_chan",
                fs->delay_len);
  if (!is_pow2(fs->rate_len) || fs->rate_len < fs->n_subints || fs->rate_len > 1024)
    return fail(c, XC_E_INVAL, "rate_len=%d: power of two in n_subints..1024", fs->rate_len);
  if (fs->delay_win < 0 || fs->rate_win < 0) return fail(c, XC_E_INVAL, "negative window");
  if (!(fs->chan_width_hz > 0.0) || !(fs->t_int_s > 0.0))
    return fail(c, XC_E_INVAL, "chan_width_hz and t_int_s must be > 0");
  if ((long)fs->n_subbands * fs->n_baselines > 0x7fffffffL)
    return fail(c, XC_E_INVAL, "too many maps");
  return XC_OK;
}

size_t fringe_bytes(const xc_fringe_setup* fs) {
  return align_up((size_t)fs->n_subbands * fs->n_baselines * fs->n_subints * fs->delay_len *
                   sizeof(float2));
}

}  // namespace

extern "C" {

size_t xc_fringe_workspace_bytes(const xc_fringe_setup* fs) {
  if (fringe_validate(nullptr, fs) != XC_OK) return 0;
  return fringe_bytes(fs);
}

int xc_fringe_search(xc_ctx* c, const xc_fringe_setup* fs, const void* vis, void* peaks,
                     void* map, void* workspace, size_t ws_bytes, void* stream_) {
  if (!c) return XC_E_INVAL;
  int rc = fringe_validate(c, fs);
  if (rc != XC_OK) return rc;
  if (!vis || !peaks) return fail(c, XC_E_INVAL, "fringe search: vis or peaks is NULL");
  const size_t need = fringe_bytes(fs);
  if (!workspace || ws_bytes < need)
    return fail(c, XC_E_NOMEM, "workspace %zu bytes < %zu needed", ws_bytes, need);
  hipError_t e = hipSetDevice(c->device);
  if (e != hipSuccess) return hip_fail(c, e, "hipSetDevice");
  hipStream_t stream = (hipStream_t)stream_;
  e = timed(c, XC_K_FRINGE, stream, [&] {
    return launch_fringe(fs, static_cast<const float2*>(vis), static_cast<float2*>(workspace),
                         c->d_tw, static_cast<xc_fringe_peak*>(peaks),
                         static_cast<float2*>(map), stream);
  });
  return e == hipSuccess ? XC_OK : hip_fail(c, e, "fringe search");
}

}  // extern "C"
