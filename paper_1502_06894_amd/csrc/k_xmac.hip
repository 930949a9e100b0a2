// X stage (A6), FP32 vector path: for every subband and channel, accumulate
// Y_i[k] conj(Y_j[k]) over the block's frames for all input pairs i <= j.
//
// A workgroup owns KC consecutive channels of one subband.  Inputs are grouped
// four at a time; thread (channel c, tile (gi, gj)) accumulates the 4 x 4
// block of products between groups gi <= gj in FP32 registers over the block
// (at most 256 frames), then adds it to the FP64 accumulator in HBM, so each
// output has a single owner and the summation order is fixed.  Spectra are
// staged through LDS a few frames at a time, so every value is read from
// memory once per block.
#include "xc_launch.h"

namespace xc {

constexpr int kGroup = 4;

__device__ inline void tile_of(int tile, int ng, int& gi, int& gj) {
  // row-major enumeration of gi <= gj
  int row = 0, rem = tile;
  while (rem >= ng - row) {
    rem -= ng - row;
    ++row;
  }
  gi = row;
  gj = row + rem;
}

__device__ inline int bl_index(int i, int j, int M) { return i * M - (i * (i - 1)) / 2 + (j - i); }

template <int KC>
__global__ void k_xmac(const DevJob* __restrict__ job, const DelayRec* __restrict__ drec,
                       const float2* __restrict__ spec, double2* __restrict__ vacc,
                       double* __restrict__ wacc, int nf, int FB, int tiles_per_wg) {
  extern __shared__ float2 sh[];   // [FB][Mp][KC]
  const DevJob& J = *job;
  const int M = J.M, P = J.n_pols, n_chan = J.n_chan, nbl = J.nbl;
  const int Mp = (M + kGroup - 1) / kGroup * kGroup;
  const int ng = Mp / kGroup;
  const int ntiles = ng * (ng + 1) / 2;
  const int sb = blockIdx.y;
  const int k0 = blockIdx.x * KC;
  const int c = threadIdx.x % KC;
  const int tile = blockIdx.z * tiles_per_wg + threadIdx.x / KC;
  const bool active = (int)(threadIdx.x / KC) < tiles_per_wg && tile < ntiles;
  int gi = 0, gj = 0;
  if (active) tile_of(tile, ng, gi, gj);

  // zero the padding rows once
  for (int q = threadIdx.x; q < FB * (Mp - M) * KC; q += blockDim.x) {
    const int fb = q / ((Mp - M) * KC);
    const int rem = q - fb * (Mp - M) * KC;
    sh[(fb * Mp + M + rem / KC) * KC + rem % KC] = make_float2(0.f, 0.f);
  }

  float2 acc[kGroup][kGroup];
#pragma unroll
  for (int a = 0; a < kGroup; ++a)
#pragma unroll
    for (int b = 0; b < kGroup; ++b) acc[a][b] = make_float2(0.f, 0.f);

  const float2* src = spec + (size_t)sb * nf * M * n_chan + k0;
  for (int f0 = 0; f0 < nf; f0 += FB) {
    const int nfb = min(FB, nf - f0);
    __syncthreads();
    for (int q = threadIdx.x; q < nfb * M * KC; q += blockDim.x) {
      const int row = q / KC;                 // fb * M + m
      const int cc = q - row * KC;
      const int fb = row / M, m = row - fb * M;
      sh[(fb * Mp + m) * KC + cc] = src[((size_t)(f0 + fb) * M + m) * n_chan + cc];
    }
    __syncthreads();
    if (active) {
      for (int fb = 0; fb < nfb; ++fb) {
        float2 a[kGroup], b[kGroup];
#pragma unroll
        for (int x = 0; x < kGroup; ++x) {
          a[x] = sh[(fb * Mp + gi * kGroup + x) * KC + c];
          b[x] = sh[(fb * Mp + gj * kGroup + x) * KC + c];
        }
#pragma unroll
        for (int x = 0; x < kGroup; ++x)
#pragma unroll
          for (int y = 0; y < kGroup; ++y) {
            // a conj(b)
            acc[x][y].x = fmaf(a[x].x, b[y].x, fmaf(a[x].y, b[y].y, acc[x][y].x));
            acc[x][y].y = fmaf(a[x].y, b[y].x, fmaf(-a[x].x, b[y].y, acc[x][y].y));
          }
      }
    }
  }
  if (!active) return;
#pragma unroll
  for (int x = 0; x < kGroup; ++x)
#pragma unroll
    for (int y = 0; y < kGroup; ++y) {
      const int i = gi * kGroup + x, j = gj * kGroup + y;
      if (i <= j && j < M) {
        double2* o = vacc + ((size_t)sb * nbl + bl_index(i, j, M)) * n_chan + k0 + c;
        double2 v = *o;
        v.x += (double)acc[x][y].x;
        v.y += (double)acc[x][y].y;
        *o = v;
      }
    }
  // weights: frames valid for both stations (one channel lane per tile)
  if (blockIdx.x == 0 && c == 0) {
    for (int x = 0; x < kGroup; ++x)
      for (int y = 0; y < kGroup; ++y) {
        const int i = gi * kGroup + x, j = gj * kGroup + y;
        if (i > j || j >= M) continue;
        const int si = i / P, sj = j / P;
        int cnt = 0;
        for (int f = 0; f < nf; ++f)
          cnt += (drec[(size_t)si * nf + f].valid & drec[(size_t)sj * nf + f].valid);
        wacc[(size_t)sb * nbl + bl_index(i, j, M)] += (double)cnt;
      }
  }
}

hipError_t launch_xmac(const DevJob* job, int M, int n_chan, int n_subbands,
                       const DelayRec* drec, const float2* spec, double2* vacc, double* wacc,
                       int nf, int n_pols, hipStream_t s) {
  (void)n_pols;
  const int Mp = (M + kGroup - 1) / kGroup * kGroup;
  const int ng = Mp / kGroup;
  const int ntiles = ng * (ng + 1) / 2;
  int KC = ntiles <= 16 ? 64 : (ntiles <= 32 ? 32 : 16);
  if (KC > n_chan) KC = n_chan;
  int tiles_per_wg = 1024 / KC;
  if (tiles_per_wg > ntiles) tiles_per_wg = ntiles;
  const int zchunks = (ntiles + tiles_per_wg - 1) / tiles_per_wg;
  int FB = 8;
  while (FB > 1 && (size_t)FB * Mp * KC * sizeof(float2) > 65536) FB /= 2;
  const size_t lds = (size_t)FB * Mp * KC * sizeof(float2);
  dim3 grid(n_chan / KC, n_subbands, zchunks);
  dim3 block(KC * tiles_per_wg);
  switch (KC) {
    case 64:
      hipLaunchKernelGGL(k_xmac<64>, grid, block, lds, s, job, drec, spec, vacc, wacc, nf, FB,
                         tiles_per_wg);
      break;
    case 32:
      hipLaunchKernelGGL(k_xmac<32>, grid, block, lds, s, job, drec, spec, vacc, wacc, nf, FB,
                         tiles_per_wg);
      break;
    case 16:
      hipLaunchKernelGGL(k_xmac<16>, grid, block, lds, s, job, drec, spec, vacc, wacc, nf, FB,
                         tiles_per_wg);
      break;
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace xc
