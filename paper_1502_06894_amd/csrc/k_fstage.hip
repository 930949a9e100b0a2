// F stage (A2-A5): 2-bit unpack of the integer-shifted window, per-sample
// fringe rotation, FFT to channels and fractional-delay correction, fused in
// one kernel.  A workgroup holds G frames of one station (G groups of T
// threads); each group loads the payload words of its window once and reuses
// them for every input (subband, pol) of the station, since all recorded
// streams of a time sample share a word.
#include "xc_fft.h"
#include "xc_launch.h"

namespace xc {

template <int N>
struct FGeom {
  static constexpr int T = FftPlan<N>::T;
  static constexpr int E = FftPlan<N>::E;
  static constexpr int G = T >= 256 ? 1 : 256 / T;   // frames per workgroup
  static constexpr int WG = T * G;
  // Up to N = 4096 the twiddles are staged in LDS (their tables then cost no
  // registers); larger transforms read them from memory.
  static constexpr bool tw_in_lds = N <= 4096;
  // G FFT exchange buffers, the 8-entry level table, the twiddle tables
  static constexpr size_t lut_off = (size_t)G * lds_words<N>() * sizeof(float2);
  static constexpr size_t tw_off = lut_off + 8 * sizeof(float);
  static constexpr size_t lds_bytes =
      tw_off + (tw_in_lds ? (size_t)tw_lds_entries<N>() * sizeof(float2) : 0);
};

// Spectrum element written by the F stage: FP32 complex, or for the MFMA X
// path the power-of-two-scaled value as FP16 (Re, Im) or OCP e4m3 (Re, Im).
template <int OUT>
__device__ inline void put_spec(void* spec, size_t idx, float2 y, int e) {
  if constexpr (OUT == kOutF32) {
    static_cast<float2*>(spec)[idx] = y;
  } else if constexpr (OUT == kOutF16) {
    const float sx = ldexpf(y.x, e), sy = ldexpf(y.y, e);
    typedef _Float16 h2 __attribute__((ext_vector_type(2)));
    h2 h;
    h.x = (_Float16)sx;
    h.y = (_Float16)sy;
    static_cast<h2*>(spec)[idx] = h;
  } else {
    // the conversion maps overflow to NaN: saturate at the e4m3 maximum first
    const float sx = fminf(fmaxf(ldexpf(y.x, e), -448.f), 448.f);
    const float sy = fminf(fmaxf(ldexpf(y.y, e), -448.f), 448.f);
    const int pk = __builtin_amdgcn_cvt_pk_fp8_f32(sx, sy, 0, false);
    static_cast<uint16_t*>(spec)[idx] = (uint16_t)(pk & 0xffff);
  }
}

// W = 0: no occupancy request; W > 0: ask the compiler for W waves per SIMD
// (caps registers at 512 / W, trading spills for latency hiding).
// OUT: spectrum element type (kOutF32, kOutF16, kOutF8); for the low-precision
// outputs `scale_exp` [n_sb][M][n_chan] holds the power-of-two exponents.
template <int N, int W, int OUT>
__global__ void __attribute__((amdgpu_flat_work_group_size(1, FGeom<N>::WG),
                               amdgpu_waves_per_eu(W > 0 ? W : 1)))
    k_fstage(const DevJob* __restrict__ job, const DelayRec* __restrict__ drec,
             const PhaseRec* __restrict__ prec, const float2* __restrict__ tw,
             void* __restrict__ spec, const int8_t* __restrict__ scale_exp, int nf) {
  constexpr int T = FGeom<N>::T, E = FGeom<N>::E, G = FGeom<N>::G;
  extern __shared__ float2 lds_all[];
  const DevJob& J = *job;
  const int g = threadIdx.x / T, t = threadIdx.x % T;
  const int s = blockIdx.y;
  const int fl = blockIdx.x * G + g;
  const bool in_blk = fl < nf;
  DelayRec r;
  if (in_blk) {
    r = drec[(size_t)s * nf + fl];
  } else {
    r.valid = 0;
    r.d = 0.0;
    r.base = 0;
  }
  const bool valid = r.valid != 0;

  // payload words holding samples n = t + e T of this frame's window; T is a
  // multiple of 16, so all of a thread's samples share one field offset
  uint32_t wv[E];
  int sh0 = 0;
  if (valid) {
    const FrameCursor c = make_cursor(J, r.base);
    const uint32_t* words = J.st[s].words;
#pragma unroll
    for (int e = 0; e < E; ++e) wv[e] = *sample_word(J, words, c, t + e * T);
    sh0 = sample_shift(J, c, t);
  } else {
#pragma unroll
    for (int e = 0; e < E; ++e) wv[e] = 0u;
  }
  float2* lds = lds_all + g * lds_words<N>();
  // 2-bit code -> level (offset binary: -3.3359, -1, +1, +3.3359), and four
  // zeros that an invalid frame's lookups are pointed at
  unsigned char* lds_b = reinterpret_cast<unsigned char*>(lds_all);
  float* lut = reinterpret_cast<float*>(lds_b + FGeom<N>::lut_off);
  if (threadIdx.x < 8) {
    const float lv[4] = {-3.3359f, -1.0f, 1.0f, 3.3359f};
    lut[threadIdx.x] = threadIdx.x < 4 ? lv[threadIdx.x] : 0.0f;
  }
  float2* tw_tab = reinterpret_cast<float2*>(lds_b + FGeom<N>::tw_off);
  if constexpr (FGeom<N>::tw_in_lds) tw_lds_fill<N>(tw_tab, tw, threadIdx.x, blockDim.x);
  const float* lut_t = lut + (valid ? 0 : 4);
  __syncthreads();
  const int P = J.n_pols, M = J.M, n_chan = J.n_chan, n_sb = J.n_subbands;

  // fractional-delay phasors of this thread's output bins k = t + r N/16:
  // exp(2 pi i k d / N) = exp(2 pi i t d / N) * exp(2 pi i d / 16)^r
  float2 fd[8];
  {
    const float dd = (float)r.d;
    fd[0] = phasor_turns((float)t * dd * (1.0f / (float)N));
    const float2 st = phasor_turns(dd * (1.0f / 16.0f));
#pragma unroll
    for (int rr = 1; rr < 8; ++rr) fd[rr] = cmul(fd[rr - 1], st);
  }
  const double nc0 = (double)(t - N / 2);     // centred index of the thread's first sample
  constexpr double TD = (double)T;
  // With whole waves per frame (T >= 64) the frame index is wave-uniform: the
  // phase records then come in through scalar loads, which a wave does not
  // have to order behind its own outstanding spectrum stores.
  const int flu = T >= 64 ? __builtin_amdgcn_readfirstlane(fl) : fl;
  const bool in_blk_u = flu < nf;

  for (int in = 0; in < J.n_inputs; ++in) {
    const int sb = in / P, p = in - sb * P;
    const int sh = sh0 + 2 * J.stream_map[in];
    PhaseRec ph;
    if (in_blk_u) ph = prec[((size_t)s * n_sb + sb) * nf + flu];
    else ph.phi0 = ph.phi1 = ph.phi2 = 0.0;
    // fringe phasors z_e = exp(2 pi i phi(t + e T)) by the second-order recurrence
    // z_{e+1} = z_e w_e, w_{e+1} = w_e rho (w_e: phase step to the next sample,
    // rho: its constant change 2 phi2 T^2), restarted exactly every E/2 samples
    const float2 rho = phasor_turns(frac_f(2.0 * ph.phi2 * TD * TD));
    float2 v[E];
    float2 z = make_float2(1.f, 0.f), w = make_float2(1.f, 0.f);
#pragma unroll
    for (int e = 0; e < E; ++e) {
      if (e % (E / 2) == 0) {
        const double nc = nc0 + (double)e * TD;
        z = phasor_turns(frac_f(fma(fma(ph.phi2, nc, ph.phi1), nc, ph.phi0)));
        w = phasor_turns(frac_f(ph.phi1 * TD + ph.phi2 * TD * (2.0 * nc + TD)));
      } else {
        z = cmul(z, w);
        w = cmul(w, rho);
      }
      const float q = lut_t[(wv[e] >> sh) & 3u];
      v[e] = make_float2(q * z.x, q * z.y);
    }
    if constexpr (FGeom<N>::tw_in_lds) fft_forward<N>(v, lds, TwLds<N>{tw_tab}, t);
    else fft_forward<N>(v, lds, TwGlobal{tw}, t);
    if (in_blk) {
      const size_t row = ((size_t)(sb * nf + fl) * M + (s * P + p)) * n_chan;
      const int8_t* ex = OUT == kOutF32 ? nullptr
                                        : scale_exp + ((size_t)sb * M + (s * P + p)) * n_chan;
#pragma unroll
      for (int rr = 0; rr < 8; ++rr) {
        const int k = t + rr * (N / 16);
        const float2 y = valid ? cmul(v[rr], fd[rr]) : make_float2(0.f, 0.f);
        put_spec<OUT>(spec, row + k, y, OUT == kOutF32 ? 0 : (int)ex[k]);
      }
    }
    __syncthreads();   // the next input reuses lds
  }
}

template <int N, int W, int OUT>
static hipError_t launch_nw(const DevJob* job, int n_stations, const DelayRec* drec,
                            const PhaseRec* prec, const float2* tw, void* spec,
                            const int8_t* scale_exp, int nf, hipStream_t s) {
  using Gm = FGeom<N>;
  static bool attr_set = false;
  if (!attr_set) {
    hipError_t e = hipFuncSetAttribute((const void*)k_fstage<N, W, OUT>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)Gm::lds_bytes);
    if (e != hipSuccess) return e;
    attr_set = true;
  }
  dim3 grid((nf + Gm::G - 1) / Gm::G, n_stations);
  hipLaunchKernelGGL((k_fstage<N, W, OUT>), grid, dim3(Gm::WG), Gm::lds_bytes, s, job, drec, prec,
                     tw, spec, scale_exp, nf);
  return hipGetLastError();
}

template <int N>
static hipError_t launch_n(const DevJob* job, int n_stations, const DelayRec* drec,
                           const PhaseRec* prec, const float2* tw, void* spec,
                           const int8_t* scale_exp, int nf, int waves, int out, hipStream_t s) {
  if (out == kOutF16)
    return launch_nw<N, 0, kOutF16>(job, n_stations, drec, prec, tw, spec, scale_exp, nf, s);
  if (out == kOutF8)
    return launch_nw<N, 0, kOutF8>(job, n_stations, drec, prec, tw, spec, scale_exp, nf, s);
  switch (waves) {
    case 3: return launch_nw<N, 3, kOutF32>(job, n_stations, drec, prec, tw, spec, nullptr, nf, s);
    case 4: return launch_nw<N, 4, kOutF32>(job, n_stations, drec, prec, tw, spec, nullptr, nf, s);
    default:
      return launch_nw<N, 0, kOutF32>(job, n_stations, drec, prec, tw, spec, nullptr, nf, s);
  }
}

bool fstage_supported(int N) {
  switch (N) {
    case 256: case 512: case 1024: case 2048: case 4096: case 8192: case 16384: return true;
    default: return false;
  }
}

hipError_t launch_fstage(int N, const DevJob* job, int n_stations, const DelayRec* drec,
                         const PhaseRec* prec, const float2* tw, void* spec,
                         const int8_t* scale_exp, int nf, int waves, int out, hipStream_t s) {
  switch (N) {
#define XC_FCASE(NN)                                                                      \
  case NN:                                                                                \
    return launch_n<NN>(job, n_stations, drec, prec, tw, spec, scale_exp, nf, waves, out, s);
    XC_FCASE(256) XC_FCASE(512) XC_FCASE(1024) XC_FCASE(2048) XC_FCASE(4096) XC_FCASE(8192)
    XC_FCASE(16384)
#undef XC_FCASE
    default: return hipErrorInvalidValue;
  }
}

}  // namespace xc
