// A7: X stage on the matrix cores for FP16 / FP8 spectra.
//
// Per channel, the block's spectra of the M <= 32 inputs form Z = [Re X; Im X]
// (2M x frames, each input scaled by a power of two before rounding).  The
// Hermitian product splits into real products over frames:
//   V_re = Re Re^T + Im Im^T,   V_im = Im Re^T - (Im Re^T)^T,
// so per channel two 32x32 MFMA accumulators in FP32 with K = frames: one
// takes both Re Re^T and Im Im^T (V_re directly), the other G21 = Im Re^T.
// A workgroup owns one 16-channel tile of one subband; the F stage writes the
// low-precision spectra channel-blocked ([frame][tile][input][16 channels]),
// so a frame of the tile is one contiguous run of M rows.  FP16 keeps the
// [frame][input][channel] order in LDS, rows padded to RW + 1 words
// and frames to 32 (RW + 1) + 1, so that both the row-wise stores
// (consecutive lanes, consecutive words) and each lane's operand gather (one
// word per frame, 32 lanes 32 inputs apart) hit distinct banks.  FP8 (half the
// words per row, twice the frames per operand) transposes into LDS as
// [channel word][input][frame], so that a lane's 8 frames are two 16-byte
// reads (measured faster there).  After the block, G21 is transposed through
// LDS, every element is unscaled by 2^-(e_i + e_j) and added to the FP64
// accumulator slot of the FP32 path.
#include <atomic>

#include "xc_launch.h"

namespace xc {

typedef _Float16 half4_t __attribute__((ext_vector_type(4)));
typedef float float16_t __attribute__((ext_vector_type(16)));

// Mean square of the four 2-bit levels for Gaussian data quantised at +-0.9816
// sigma (outer levels with probability 2 Phi(-0.9816) = 0.32630): the expected
// |Y[k]|^2 / N of an unnormalised FFT of such samples, whatever the rotation.
constexpr double kLevelPower = 4.304810;

// Valid pre-pass frames an input needs for its own per-channel scales: a mean
// |Y|^2 over fewer frames is too noisy (over 2 frames a channel's estimate is
// below 1/100 of its power with probability ~2e-4, which over 16384 channels
// would push a few channels 10x above the target level, into e4m3
// saturation); with 16 the estimate stays within a factor 4 in power.
constexpr int kMinScaleFrames = 16;

// Per (subband, input, channel; stored at scale_pos): the power-of-two exponent that brings the mean
// |Y|^2 over the pre-pass frames valid for the input's station to
// 2^(2 target_log2).  Invalid frames (zero spectra) are left out of the mean;
// an input with fewer than kMinScaleFrames valid pre-pass frames (all of them,
// when the pre-pass is shorter) takes the expected white-noise power
// N kLevelPower of 2-bit data.
__global__ void k_scales(const float2* __restrict__ spec, const DelayRec* __restrict__ drec,
                         int n_sb, int nf, int M, int P, int n_chan, int target_log2,
                         int8_t* __restrict__ scale_exp) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;   // (sb, m, k)
  const size_t total = (size_t)n_sb * M * n_chan;
  if (i >= total) return;
  const int k = (int)(i % n_chan);
  const int m = (int)((i / n_chan) % M);
  const int sb = (int)(i / ((size_t)n_chan * M));
  const DelayRec* rec = drec + (size_t)(m / P) * nf;
  double acc = 0.0;
  int n_valid = 0;
  for (int f = 0; f < nf; ++f) {
    if (!rec[f].valid) continue;
    const float2 y = spec[(((size_t)sb * nf + f) * M + m) * n_chan + k];
    acc += (double)y.x * y.x + (double)y.y * y.y;
    ++n_valid;
  }
  const bool own = n_valid > 0 && n_valid >= min(nf, kMinScaleFrames);
  const double power = own ? acc / n_valid : 2.0 * n_chan * kLevelPower;
  int e = 0;
  if (power > 0.0) {
    const double l2 = 0.5 * log2(power);                // log2 of the RMS magnitude
    e = (int)lrint((double)target_log2 - l2);
    e = e < -100 ? -100 : (e > 100 ? 100 : e);
  }
  scale_exp[i - k + scale_pos(k, n_chan)] = (int8_t)e;
}

hipError_t launch_scales(const float2* spec, const DelayRec* drec, int n_subbands, int nf, int M,
                         int P, int n_chan, int target_log2, int8_t* scale_exp, hipStream_t s) {
  const size_t total = (size_t)n_subbands * M * n_chan;
  hipLaunchKernelGGL(k_scales, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, spec,
                     drec, n_subbands, nf, M, P, n_chan, target_log2, scale_exp);
  return hipGetLastError();
}

__device__ inline int bl_of(int i, int j, int M) { return i * M - (i * (i - 1)) / 2 + (j - i); }

// OUT = kOutF16: element = 1 word (Re, Im halves), KC channels = KC words per row,
//       MFMA 32x32x8, a lane's operand = 4 frames.
// OUT = kOutF8:  element = 1 half-word (Re, Im bytes), KC channels = KC/2 words per
//       row, MFMA 32x32x16, a lane's operand = 8 frames.
// FB frames per LDS stage, CPW channels per wave.
template <int OUT, int KC, int CPW, int FB>
__global__ void __launch_bounds__(64 * (KC / CPW))
    k_xmfma(const DevJob* __restrict__ job, const uint32_t* __restrict__ spec,
            const int8_t* __restrict__ scale_exp, double2* __restrict__ vacc, int nf) {
  constexpr int NW = KC / CPW;                       // waves
  constexpr int NT = 64 * NW;
  constexpr int RW = OUT == kOutF16 ? KC : KC / 2;   // 32-bit words per (frame, input) row
  constexpr int RS = RW + 1;                         // FP16 LDS row stride (words)
  constexpr int FS = 32 * RS + 1;                    // FP16 LDS frame stride (words)
  constexpr int FP = FB + 4;                         // FP8 LDS frame stride (padding)
  constexpr int KSTEP = OUT == kOutF16 ? 8 : 16;     // frames per MFMA
  constexpr int OPF = KSTEP / 2;                     // frames per lane operand
  // 2 stages: FP16 [FB][32][RS] (+ padding), FP8 [RW][32][FP]
  extern __shared__ uint32_t lds[];
  constexpr int STAGE = OUT == kOutF16 ? FB * FS : RW * 32 * FP;
  const DevJob& J = *job;
  const int M = J.M, n_chan = J.n_chan, nbl = J.nbl;
  // XCD-aware tile order: workgroups are dealt to the 8 XCDs round-robin, so
  // workgroup b takes tile (b mod 8) (tiles / 8) + b / 8; each XCD then works
  // through a contiguous run of channel tiles, which in every frame are one
  // contiguous stretch of memory.
  const int n_tiles = gridDim.x * gridDim.y;
  const int b = blockIdx.x + gridDim.x * blockIdx.y;
  const int tile = n_tiles % 8 == 0 ? (b % 8) * (n_tiles / 8) + b / 8 : b;
  const int sb = tile / gridDim.x;
  const int k0 = (tile - sb * gridDim.x) * KC;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int m = lane & 31, g = lane >> 5;
  static_assert(KC == 16, "one channel tile of the blocked spectra per workgroup");
  // this tile's run in frame f: src + f * fstride, M rows of RW words
  const size_t fstride = (size_t)(n_chan / 16) * M * RW;
  const uint32_t* src = spec + ((size_t)sb * nf * (n_chan / 16) + k0 / 16) * M * RW;

  // inputs m >= M (and the padding) read zeros
  for (int q = threadIdx.x; q < 2 * STAGE; q += NT) lds[q] = 0u;

  float16_t accre[CPW], acc21[CPW];
#pragma unroll
  for (int c = 0; c < CPW; ++c) {
    accre[c] = (float16_t){};
    acc21[c] = (float16_t){};
  }

  // stage loader: FB frames x M inputs x RW words, each frame's M rows one
  // contiguous run, read in 16-byte pieces and stored word by word
  constexpr int VEC = 4;
  static_assert(RW % VEC == 0, "rows of whole 16-byte pieces");
  constexpr int RV = RW / VEC;                       // pieces per row
  constexpr int PER = (FB * 32 * RV + NT - 1) / NT;
  uint4 pre[PER];
  auto gload = [&](int f0) {
    const int nfb = min(FB, nf - f0);
#pragma unroll
    for (int i = 0; i < PER; ++i) {
      const int q = threadIdx.x + i * NT;
      const int w = (q % RV) * VEC, r = q / RV;      // r = fb * M + input
      const int fb = r / M, mm = r - fb * M;
      pre[i] = (r < FB * M && fb < nfb)
                   ? *reinterpret_cast<const uint4*>(src + (size_t)(f0 + fb) * fstride + mm * RW + w)
                   : make_uint4(0u, 0u, 0u, 0u);
    }
  };
  auto lstore = [&](int buf) {
#pragma unroll
    for (int i = 0; i < PER; ++i) {
      const int q = threadIdx.x + i * NT;
      const int w = (q % RV) * VEC, r = q / RV;
      const int fb = r / M, mm = r - fb * M;
      if (r < FB * M) {
        const uint32_t v4[VEC] = {pre[i].x, pre[i].y, pre[i].z, pre[i].w};
#pragma unroll
        for (int u = 0; u < VEC; ++u) {
          if constexpr (OUT == kOutF16)
            lds[buf * STAGE + fb * FS + mm * RS + w + u] = v4[u];
          else
            lds[buf * STAGE + ((w + u) * 32 + mm) * FP + fb] = v4[u];
        }
      }
    }
  };

  __syncthreads();
  gload(0);
  lstore(0);
  __syncthreads();
  int buf = 0;
  for (int f0 = 0; f0 < nf; f0 += FB) {
    const bool more = f0 + FB < nf;
    if (more) gload(f0 + FB);
    const uint32_t* st = lds + buf * STAGE;
#pragma unroll
    for (int c = 0; c < CPW; ++c) {
      const int ch = wave * CPW + c;                 // channel within the tile
#pragma unroll
      for (int ks = 0; ks < FB / KSTEP; ++ks) {
        const int fbase = ks * KSTEP + g * OPF;
        if constexpr (OUT == kOutF16) {
          // 4 frames of input m, channel word ch
          const uint32_t* p = st + fbase * FS + m * RS + ch;
          half4_t re, im;
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            const uint32_t w = p[e * FS];
            re[e] = __builtin_bit_cast(_Float16, (uint16_t)(w & 0xffffu));
            im[e] = __builtin_bit_cast(_Float16, (uint16_t)(w >> 16));
          }
          accre[c] = __builtin_amdgcn_mfma_f32_32x32x8f16(re, re, accre[c], 0, 0, 0);
          accre[c] = __builtin_amdgcn_mfma_f32_32x32x8f16(im, im, accre[c], 0, 0, 0);
          acc21[c] = __builtin_amdgcn_mfma_f32_32x32x8f16(im, re, acc21[c], 0, 0, 0);
        } else {
          // 8 frames of input m, channel ch: half-word (ch & 1) of word ch / 2
          const uint32_t* p = st + ((ch >> 1) * 32 + m) * FP + fbase;
          const uint4 w0 = *reinterpret_cast<const uint4*>(p);
          const uint4 w1 = *reinterpret_cast<const uint4*>(p + 4);
          const uint32_t ww[8] = {w0.x, w0.y, w0.z, w0.w, w1.x, w1.y, w1.z, w1.w};
          const int sh = (ch & 1) * 16;
          uint64_t re = 0, im = 0;
#pragma unroll
          for (int e = 0; e < 8; ++e) {
            const uint32_t h = (ww[e] >> sh) & 0xffffu;
            re |= (uint64_t)(h & 0xffu) << (8 * e);
            im |= (uint64_t)(h >> 8) << (8 * e);
          }
          accre[c] = __builtin_amdgcn_mfma_f32_32x32x16_fp8_fp8((long)re, (long)re, accre[c], 0, 0, 0);
          accre[c] = __builtin_amdgcn_mfma_f32_32x32x16_fp8_fp8((long)im, (long)im, accre[c], 0, 0, 0);
          acc21[c] = __builtin_amdgcn_mfma_f32_32x32x16_fp8_fp8((long)im, (long)re, acc21[c], 0, 0, 0);
        }
      }
    }
    if (more) lstore(buf ^ 1);
    __syncthreads();
    buf ^= 1;
  }

  // epilogue: transpose G21 through this wave's own 32 x 33 float scratch
  float* scr = reinterpret_cast<float*>(lds) + wave * (32 * 33);
  const int j = lane & 31;
#pragma unroll
  for (int c = 0; c < CPW; ++c) {
    const int k = k0 + wave * CPW + c;
#pragma unroll
    for (int v = 0; v < 16; ++v) {
      const int i = 8 * (v >> 2) + 4 * g + (v & 3);
      scr[i * 33 + j] = acc21[c][v];
    }
    __syncthreads();   // uniform: every wave runs CPW epilogue rounds
    const int kp = scale_pos(k, n_chan);
    const int ej = j < M ? scale_exp[((size_t)sb * M + j) * n_chan + kp] : 0;
#pragma unroll
    for (int v = 0; v < 16; ++v) {
      const int i = 8 * (v >> 2) + 4 * g + (v & 3);
      if (i <= j && j < M) {
        const int ei = scale_exp[((size_t)sb * M + i) * n_chan + kp];
        const double sc = ldexp(1.0, -(ei + ej));
        const double re = (double)accre[c][v] * sc;
        const double im = ((double)acc21[c][v] - (double)scr[j * 33 + i]) * sc;
        double2* o = vacc + ((size_t)sb * nbl + bl_of(i, j, M)) * n_chan + k;
        double2 a = *o;
        a.x += re;
        a.y += im;
        *o = a;
      }
    }
    __syncthreads();   // scratch is rewritten by the next round
  }
}

template <int OUT, int KC, int CPW, int FB>
static hipError_t launch_cfg(const DevJob* job, int n_chan, int n_subbands, const void* spec,
                             const int8_t* scale_exp, double2* vacc, int nf, hipStream_t s) {
  constexpr int NW = KC / CPW;
  constexpr int RW = OUT == kOutF16 ? KC : KC / 2;
  size_t lds = 2 * (OUT == kOutF16 ? (size_t)FB * (32 * (RW + 1) + 1)
                                    : (size_t)RW * 32 * (FB + 4)) * sizeof(uint32_t);
  const size_t scr = (size_t)NW * 32 * 33 * sizeof(float);
  if (scr > lds) lds = scr;
  static std::atomic<bool> attr_set[64];   // per device
  if (lds > 65536) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= 64) return hipErrorInvalidDevice;
    if (!attr_set[dev].load()) {
      e = hipFuncSetAttribute((const void*)k_xmfma<OUT, KC, CPW, FB>,
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
      if (e != hipSuccess) return e;
      attr_set[dev].store(true);
    }
  }
  dim3 grid(n_chan / KC, n_subbands);
  hipLaunchKernelGGL((k_xmfma<OUT, KC, CPW, FB>), grid, dim3(64 * NW), lds, s, job,
                     static_cast<const uint32_t*>(spec), scale_exp, vacc, nf);
  return hipGetLastError();
}

hipError_t launch_xmfma(const DevJob* job, int out, int M, int n_chan, int n_subbands,
                        const void* spec, const int8_t* scale_exp, double2* vacc,
                        size_t slot_stride, int nf, hipStream_t s) {
  (void)slot_stride;
  if (M > 32 || n_chan < 32) return hipErrorInvalidValue;
  // 16 channels per workgroup, one per wave (16 waves, 110 registers: four
  // waves per SIMD); 32 (FP16) / 64 (e4m3) frames per LDS stage, 139 KB of LDS,
  // one workgroup per CU.  Measured on a C4 step: 16-frame stages -> these,
  // FP16 5.33 -> 5.07 ms, e4m3 4.42 -> 3.86 ms; two channels per wave (8 waves)
  // -> one, 5.07 -> 4.87 and 3.88 -> 3.70 ms.
  if (out == kOutF16)
    return launch_cfg<kOutF16, 16, 1, 32>(job, n_chan, n_subbands, spec, scale_exp, vacc, nf, s);
  if (out == kOutF8)
    return launch_cfg<kOutF8, 16, 1, 64>(job, n_chan, n_subbands, spec, scale_exp, vacc, nf, s);
  return hipErrorInvalidValue;
}

}  // namespace xc
