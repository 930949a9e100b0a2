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
  static constexpr size_t lds_bytes = (size_t)G * lds_words<N>() * sizeof(float2);
};

template <int N>
__global__ void __launch_bounds__(FGeom<N>::WG)
    k_fstage(const DevJob* __restrict__ job, const DelayRec* __restrict__ drec,
             const PhaseRec* __restrict__ prec, const float2* __restrict__ tw,
             float2* __restrict__ spec, int nf) {
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

  // payload words holding samples n = t + e T of this frame's window
  uint32_t wv[E];
  int sh0[E];
  if (valid) {
    const FrameCursor c = make_cursor(J, r.base);
    const uint32_t* words = J.st[s].words;
#pragma unroll
    for (int e = 0; e < E; ++e) wv[e] = *sample_word(J, words, c, t + e * T, sh0[e]);
  } else {
#pragma unroll
    for (int e = 0; e < E; ++e) {
      wv[e] = 0u;
      sh0[e] = 0;
    }
  }
  float2* lds = lds_all + g * lds_words<N>();
  const float dN = (float)(r.d / (double)N);
  const int P = J.n_pols, M = J.M, n_chan = J.n_chan, n_sb = J.n_subbands;

  for (int in = 0; in < J.n_inputs; ++in) {
    const int sb = in / P, p = in - sb * P;
    const int sh_stream = 2 * J.stream_map[in];
    PhaseRec ph;
    if (in_blk) ph = prec[((size_t)s * n_sb + sb) * nf + fl];
    else ph.phi0 = ph.phi1 = ph.phi2 = 0.0;
    float2 v[E];
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const int n = t + e * T;
      const float q = valid ? level_of((wv[e] >> (sh0[e] + sh_stream)) & 3u) : 0.0f;
      const double dn = (double)(n - N / 2);
      double x = fma(fma(ph.phi2, dn, ph.phi1), dn, ph.phi0);
      x -= floor(x);
      const float2 z = phasor_turns((float)x);
      v[e] = make_float2(q * z.x, q * z.y);
    }
    fft_forward<N>(v, lds, tw, t);
    if (in_blk) {
      float2* out = spec + ((size_t)(sb * nf + fl) * M + (s * P + p)) * n_chan;
#pragma unroll
      for (int rr = 0; rr < 8; ++rr) {
        const int k = t + rr * (N / 16);
        float2 y = v[rr];
        y = valid ? cmul(y, phasor_turns((float)k * dN)) : make_float2(0.f, 0.f);
        out[k] = y;
      }
    }
    __syncthreads();   // the next input reuses lds
  }
}

template <int N>
static hipError_t launch_n(const DevJob* job, int n_stations, const DelayRec* drec,
                           const PhaseRec* prec, const float2* tw, float2* spec, int nf,
                           hipStream_t s) {
  using Gm = FGeom<N>;
  static bool attr_set = false;
  if (!attr_set) {
    hipError_t e = hipFuncSetAttribute((const void*)k_fstage<N>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)Gm::lds_bytes);
    if (e != hipSuccess) return e;
    attr_set = true;
  }
  dim3 grid((nf + Gm::G - 1) / Gm::G, n_stations);
  hipLaunchKernelGGL(k_fstage<N>, grid, dim3(Gm::WG), Gm::lds_bytes, s, job, drec, prec, tw, spec,
                     nf);
  return hipGetLastError();
}

bool fstage_supported(int N) {
  switch (N) {
    case 256: case 512: case 1024: case 2048: case 4096: case 8192: case 16384: return true;
    default: return false;
  }
}

hipError_t launch_fstage(int N, const DevJob* job, int n_stations, const DelayRec* drec,
                         const PhaseRec* prec, const float2* tw, float2* spec, int nf,
                         hipStream_t s) {
  switch (N) {
    case 256: return launch_n<256>(job, n_stations, drec, prec, tw, spec, nf, s);
    case 512: return launch_n<512>(job, n_stations, drec, prec, tw, spec, nf, s);
    case 1024: return launch_n<1024>(job, n_stations, drec, prec, tw, spec, nf, s);
    case 2048: return launch_n<2048>(job, n_stations, drec, prec, tw, spec, nf, s);
    case 4096: return launch_n<4096>(job, n_stations, drec, prec, tw, spec, nf, s);
    case 8192: return launch_n<8192>(job, n_stations, drec, prec, tw, spec, nf, s);
    case 16384: return launch_n<16384>(job, n_stations, drec, prec, tw, spec, nf, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace xc
