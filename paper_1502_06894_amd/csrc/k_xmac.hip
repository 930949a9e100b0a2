// X stage (A6), FP32 vector path: for every subband and channel, accumulate
// Y_i[k] conj(Y_j[k]) over the block's frames for all input pairs i <= j.
//
// A workgroup owns KC consecutive channels of one subband and one slice of
// the block's frames (at most 256).  Inputs are grouped four at a time;
// thread (channel c, tile (gi, gj)) accumulates the 4 x 4 block of products
// between groups gi <= gj in FP32 registers over its frame slice, then adds it
// to the FP64 accumulator slot of that slice.  Every output element of a slot
// has a single owner, slots are summed in slot order by the finalise kernel,
// so results do not depend on scheduling.  Spectra are staged through LDS a
// few frames at a time, so every value is read from memory once.
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

// LDS row stride: KC channels plus one float2 so that rows start on different banks.
template <int KC>
__global__ void k_xmac(const DevJob* __restrict__ job, const float2* __restrict__ spec,
                       double2* __restrict__ vacc, int nf, int FB, int tiles_per_wg,
                       int zchunks, int frames_per_split, size_t slot_stride) {
  extern __shared__ float2 sh[];   // [FB][Mp][KC + 1]
  constexpr int RS = KC + 1;
  const DevJob& J = *job;
  const int M = J.M, n_chan = J.n_chan, nbl = J.nbl;
  const int Mp = (M + kGroup - 1) / kGroup * kGroup;
  const int ng = Mp / kGroup;
  const int ntiles = ng * (ng + 1) / 2;
  const int sb = blockIdx.y;
  const int k0 = blockIdx.x * KC;
  const int zc = blockIdx.z % zchunks, split = blockIdx.z / zchunks;
  const int fa = split * frames_per_split;
  const int fz = min(nf, fa + frames_per_split);
  const int c = threadIdx.x % KC;
  const int tile = zc * tiles_per_wg + threadIdx.x / KC;
  const bool active = (int)(threadIdx.x / KC) < tiles_per_wg && tile < ntiles;
  int gi = 0, gj = 0;
  if (active) tile_of(tile, ng, gi, gj);

  // zero the padding rows once
  const int pad_rows = Mp - M;
  for (int q = threadIdx.x; q < FB * pad_rows * KC; q += blockDim.x) {
    const int fb = q / (pad_rows * KC);
    const int rem = q - fb * pad_rows * KC;
    sh[(fb * Mp + M + rem / KC) * RS + rem % KC] = make_float2(0.f, 0.f);
  }

  float2 acc[kGroup][kGroup];
#pragma unroll
  for (int a = 0; a < kGroup; ++a)
#pragma unroll
    for (int b = 0; b < kGroup; ++b) acc[a][b] = make_float2(0.f, 0.f);

  const float2* src = spec + (size_t)sb * nf * M * n_chan + k0;
  for (int f0 = fa; f0 < fz; f0 += FB) {
    const int nfb = min(FB, fz - f0);
    __syncthreads();
    for (int q = threadIdx.x; q < nfb * M * KC; q += blockDim.x) {
      const int row = q / KC;                 // fb * M + m
      const int cc = q - row * KC;
      const int fb = row / M, m = row - fb * M;
      sh[(fb * Mp + m) * RS + cc] = src[((size_t)(f0 + fb) * M + m) * n_chan + cc];
    }
    __syncthreads();
    if (active) {
      for (int fb = 0; fb < nfb; ++fb) {
        float2 a[kGroup], b[kGroup];
#pragma unroll
        for (int x = 0; x < kGroup; ++x) {
          a[x] = sh[(fb * Mp + gi * kGroup + x) * RS + c];
          b[x] = sh[(fb * Mp + gj * kGroup + x) * RS + c];
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
  if (!active || fa >= fz) return;
  double2* slot = vacc + (size_t)split * slot_stride;
#pragma unroll
  for (int x = 0; x < kGroup; ++x)
#pragma unroll
    for (int y = 0; y < kGroup; ++y) {
      const int i = gi * kGroup + x, j = gj * kGroup + y;
      if (i <= j && j < M) {
        double2* o = slot + ((size_t)sb * nbl + bl_index(i, j, M)) * n_chan + k0 + c;
        double2 v = *o;
        v.x += (double)acc[x][y].x;
        v.y += (double)acc[x][y].y;
        *o = v;
      }
    }
}

int xmac_splits(int nf) { return (nf + kXmacFramesPerSplit - 1) / kXmacFramesPerSplit; }

hipError_t launch_xmac(const DevJob* job, int M, int n_chan, int n_subbands,
                       const float2* spec, double2* vacc, size_t slot_stride, int nf,
                       hipStream_t s) {
  const int Mp = (M + kGroup - 1) / kGroup * kGroup;
  const int ng = Mp / kGroup;
  const int ntiles = ng * (ng + 1) / 2;
  const int n_splits = xmac_splits(nf);
  const int fps = (nf + n_splits - 1) / n_splits;
  // widest channel tile that still gives a few workgroups per compute unit
  int KC = 16;
  for (int kc : {64, 32}) {
    int tpw = 1024 / kc < ntiles ? 1024 / kc : ntiles;
    long wgs = (long)(n_chan / kc) * n_subbands * ((ntiles + tpw - 1) / tpw) * n_splits;
    if (kc <= n_chan && wgs >= 1024) {
      KC = kc;
      break;
    }
  }
  int tiles_per_wg = 256 / KC > 1 ? 256 / KC : 1;    // 256-thread workgroups
  if (tiles_per_wg > ntiles) tiles_per_wg = ntiles;
  const int zchunks = (ntiles + tiles_per_wg - 1) / tiles_per_wg;
  int FB = 8;
  while (FB > 1 && (size_t)FB * Mp * (KC + 1) * sizeof(float2) > 32768) FB /= 2;
  const size_t lds = (size_t)FB * Mp * (KC + 1) * sizeof(float2);
  dim3 grid(n_chan / KC, n_subbands, zchunks * n_splits);
  dim3 block(KC * tiles_per_wg);
  switch (KC) {
    case 64:
      hipLaunchKernelGGL(k_xmac<64>, grid, block, lds, s, job, spec, vacc, nf, FB, tiles_per_wg,
                         zchunks, fps, slot_stride);
      break;
    case 32:
      hipLaunchKernelGGL(k_xmac<32>, grid, block, lds, s, job, spec, vacc, nf, FB, tiles_per_wg,
                         zchunks, fps, slot_stride);
      break;
    default:
      hipLaunchKernelGGL(k_xmac<16>, grid, block, lds, s, job, spec, vacc, nf, FB, tiles_per_wg,
                         zchunks, fps, slot_stride);
      break;
  }
  return hipGetLastError();
}

}  // namespace xc
