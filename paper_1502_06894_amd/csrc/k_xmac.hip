// X stage (A6), FP32 vector path: for every subband and channel, accumulate
// Y_i[k] conj(Y_j[k]) over the block's frames for all input pairs i <= j.
//
// A workgroup owns KC consecutive channels of one subband and one slice of
// the block's frames (at most 1024).  Inputs are grouped four at a time;
// thread (channel c, tile (gi, gj)) accumulates the 4 x 4 block of products
// between groups gi <= gj in FP32 registers over its frame slice, then adds it
// to the FP64 accumulator slot of that slice.  Every output element of a slot
// has a single owner, slots are summed in slot order by the finalise kernel,
// so results do not depend on scheduling.  Spectra are staged through LDS a
// few frames at a time, so every value is read from memory once.
#include <atomic>

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

// LDS layout per stage: [FB frames][Mp inputs][RS] float2 with RS = KC + 2, so
// rows start on different banks and stay 16-byte aligned.  Two stages are
// double-buffered: the global loads of stage s+1 are in flight (registers)
// while stage s is multiplied out of LDS.
template <int KC, int FB, int MAXL>
__global__ void __launch_bounds__(1024)
    k_xmac(const DevJob* __restrict__ job, const float2* __restrict__ spec,
           double2* __restrict__ vacc, int nf, int tiles_per_wg, int zchunks,
           int frames_per_split, size_t slot_stride) {
  extern __shared__ float4 sh4[];
  constexpr int RS = KC + 2;          // float2 per LDS row
  constexpr int RS4 = RS / 2;         // float4 per LDS row
  constexpr int KC4 = KC / 2;
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
  const int nthr = blockDim.x;
  const int stage4 = FB * Mp * RS4;   // float4 per stage buffer
  int gi = 0, gj = 0;
  if (active) tile_of(tile, ng, gi, gj);

  // zero both stages once (covers the padding rows Mp > M)
  for (int q = threadIdx.x; q < 2 * stage4; q += nthr) sh4[q] = make_float4(0.f, 0.f, 0.f, 0.f);

  float2 acc[kGroup][kGroup];
#pragma unroll
  for (int a = 0; a < kGroup; ++a)
#pragma unroll
    for (int b = 0; b < kGroup; ++b) acc[a][b] = make_float2(0.f, 0.f);

  const float4* src = reinterpret_cast<const float4*>(spec + (size_t)sb * nf * M * n_chan + k0);
  const int row4 = n_chan / 2;        // float4 per spectrum row
  float4 pre[MAXL];
  auto gload = [&](int f0) {
    const int nfb = min(FB, fz - f0);
    const int n = nfb * M * KC4;
#pragma unroll
    for (int i = 0; i < MAXL; ++i) {
      const int q = threadIdx.x + i * nthr;
      if (q < n) {
        const int row = q / KC4, cc = q - row * KC4;
        typedef float f4 __attribute__((ext_vector_type(4)));
        const f4 x = __builtin_nontemporal_load(
            reinterpret_cast<const f4*>(src) + (size_t)(f0 * M + row) * row4 + cc);
        pre[i] = make_float4(x.x, x.y, x.z, x.w);
      }
    }
  };
  auto lstore = [&](int f0, int buf) {
    const int nfb = min(FB, fz - f0);
    const int n = nfb * M * KC4;
#pragma unroll
    for (int i = 0; i < MAXL; ++i) {
      const int q = threadIdx.x + i * nthr;
      if (q < n) {
        const int row = q / KC4, cc = q - row * KC4;
        const int fb = row / M, m = row - fb * M;
        sh4[buf * stage4 + (fb * Mp + m) * RS4 + cc] = pre[i];
      }
    }
  };

  __syncthreads();
  if (fa < fz) {
    gload(fa);
    lstore(fa, 0);
  }
  __syncthreads();
  int buf = 0;
  for (int f0 = fa; f0 < fz; f0 += FB) {
    const int nfb = min(FB, fz - f0);
    const bool more = f0 + FB < fz;
    if (more) gload(f0 + FB);
    if (active) {
      const float2* shb = reinterpret_cast<const float2*>(sh4 + buf * stage4);
      for (int fb = 0; fb < nfb; ++fb) {
        float2 a[kGroup], b[kGroup];
#pragma unroll
        for (int x = 0; x < kGroup; ++x) {
          a[x] = shb[(fb * Mp + gi * kGroup + x) * RS + c];
          b[x] = shb[(fb * Mp + gj * kGroup + x) * RS + c];
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
    if (more) lstore(f0 + FB, buf ^ 1);
    __syncthreads();
    buf ^= 1;
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

// Barrier-free variant: each thread reads its 2 x 4 inputs of every frame
// straight from memory (the same workgroup's other tiles re-read them from L1),
// one frame ahead in registers.  A workgroup is all tiles of KC channels.
template <int KC>
__global__ void __launch_bounds__(1024)
    k_xmac_direct(const DevJob* __restrict__ job, const float2* __restrict__ spec,
                  double2* __restrict__ vacc, int nf, int tiles_per_wg, int zchunks,
                  int frames_per_split, size_t slot_stride) {
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
  if ((int)(threadIdx.x / KC) >= tiles_per_wg || tile >= ntiles || fa >= fz) return;
  int gi, gj;
  tile_of(tile, ng, gi, gj);
  // inputs beyond M read row M-1 (their products are never stored)
  int ra[kGroup], rb[kGroup];
#pragma unroll
  for (int x = 0; x < kGroup; ++x) {
    ra[x] = min(gi * kGroup + x, M - 1);
    rb[x] = min(gj * kGroup + x, M - 1);
  }
  const float2* src = spec + (size_t)sb * nf * M * n_chan + k0 + c;
  const size_t fstride = (size_t)M * n_chan;

  float2 acc[kGroup][kGroup];
#pragma unroll
  for (int a = 0; a < kGroup; ++a)
#pragma unroll
    for (int b = 0; b < kGroup; ++b) acc[a][b] = make_float2(0.f, 0.f);

  float2 a[kGroup], b[kGroup], an[kGroup], bn[kGroup];
  const float2* p = src + (size_t)fa * fstride;
#pragma unroll
  for (int x = 0; x < kGroup; ++x) {
    a[x] = p[(size_t)ra[x] * n_chan];
    b[x] = p[(size_t)rb[x] * n_chan];
  }
  for (int f = fa; f < fz; ++f) {
    if (f + 1 < fz) {
      const float2* q = p + fstride;
#pragma unroll
      for (int x = 0; x < kGroup; ++x) {
        an[x] = q[(size_t)ra[x] * n_chan];
        bn[x] = q[(size_t)rb[x] * n_chan];
      }
    }
#pragma unroll
    for (int x = 0; x < kGroup; ++x)
#pragma unroll
      for (int y = 0; y < kGroup; ++y) {
        acc[x][y].x = fmaf(a[x].x, b[y].x, fmaf(a[x].y, b[y].y, acc[x][y].x));
        acc[x][y].y = fmaf(a[x].y, b[y].x, fmaf(-a[x].x, b[y].y, acc[x][y].y));
      }
#pragma unroll
    for (int x = 0; x < kGroup; ++x) {
      a[x] = an[x];
      b[x] = bn[x];
    }
    p += fstride;
  }
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

// Ring variant (channel tile 64, at most 32 padded inputs).  Spectra go from
// memory straight into LDS (global_load_lds, no register staging) through a
// ring of kRing one-frame stages that runs kRing - 1 frames ahead of the
// multiply, so tens of KB per compute unit are in flight and memory latency
// is hidden.  One wave per 4 x 4 tile, one lane per channel: a wave reads one
// contiguous 512-byte LDS row per operand, free of bank conflicts.  A frame
// stage is MP rows of 64 float2; wave w loads rows 2w and 2w + 1 (1 KB, one
// instruction: LDS address = wave base + 16 * lane), so every wave issues
// exactly one load per frame and "frame j has landed" is a fixed
// outstanding-load count.  The ring stages are separate LDS variables so the
// compiler can tell the in-flight loads apart from the stage being read.
constexpr int kRing = 8;

typedef __attribute__((address_space(3))) void lds_void_t;
typedef __attribute__((address_space(1))) void glb_void_t;

// s_waitcnt immediates: at most n vector-memory operations of this wave
// outstanding, and with _lds also no LDS operation outstanding.
constexpr int waitcnt_vm(int n) { return (n & 15) | ((n >> 4) << 14) | (7 << 4) | (15 << 8); }
constexpr int waitcnt_vm_lds(int n) { return (n & 15) | ((n >> 4) << 14) | (7 << 4); }

// One ring step for frame j: wait for this wave's load of frame j + 1 (and
// its own LDS reads of frame j), barrier (frame j + 1's stage RD is complete
// everywhere; every wave holds frame j in registers, so stage RF, last used
// by frame j - 1, is free), refill RF with frame j + kRing - 1, read frame
// j + 1 from RD into registers NEXT, then multiply frame j from registers CUR:
// the LDS reads of the next frame are in flight during the multiply.
#define XC_RING_STEP(RD, RF, CUR_A, CUR_B, NEXT_A, NEXT_B)                            \
  {                                                                                  \
    __builtin_amdgcn_sched_barrier(0); /* the previous multiply stays before */      \
    __builtin_amdgcn_s_waitcnt(waitcnt_vm_lds(kRing - 3));                           \
    __asm__ volatile("" ::: "memory");                                               \
    __builtin_amdgcn_s_barrier();                                                    \
    __asm__ volatile("" ::: "memory");                                               \
    __builtin_amdgcn_sched_barrier(0);                                               \
    ring_load(gsrc + (size_t)min(j + kRing - 1, fz - 1) * fstride4 + loff, RF + lw * 64);\
    ring_read(reinterpret_cast<const float2*>(RD), gi, gj, lane, NEXT_A, NEXT_B);    \
    __builtin_amdgcn_sched_barrier(0); /* issue the reads before the multiply */     \
    ring_mac(CUR_A, CUR_B, acc);                                                     \
    ++j;                                                                             \
  }

// Cache policy 2 = non-temporal: the spectra stream through once (measured on
// MI355X: 4.5 -> 5.1 TB/s, a plain device copy's rate, together with the F
// stage's non-temporal stores).
__device__ __forceinline__ void ring_load(const float4* g, float4* l) {
  __builtin_amdgcn_global_load_lds((glb_void_t*)g, (lds_void_t*)l, 16, 0, 2);
}

// This lane's operands of one frame: rows gi*4 + x and gj*4 + x, its channel.
__device__ __forceinline__ void ring_read(const float2* shb, int gi, int gj, int lane,
                                          float2 (&a)[kGroup], float2 (&b)[kGroup]) {
#pragma unroll
  for (int x = 0; x < kGroup; ++x) {
    a[x] = shb[(gi * kGroup + x) * 64 + lane];
    b[x] = shb[(gj * kGroup + x) * 64 + lane];
  }
}

__device__ __forceinline__ void ring_mac(const float2 (&a)[kGroup], const float2 (&b)[kGroup],
                                         float2 (&acc)[kGroup][kGroup]) {
#pragma unroll
  for (int x = 0; x < kGroup; ++x)
#pragma unroll
    for (int y = 0; y < kGroup; ++y) {
      acc[x][y].x = fmaf(a[x].x, b[y].x, fmaf(a[x].y, b[y].y, acc[x][y].x));
      acc[x][y].y = fmaf(a[x].y, b[y].x, fmaf(-a[x].x, b[y].y, acc[x][y].y));
    }
}

template <int MP>
__global__ void __launch_bounds__(1024)
    k_xmac_ring(const DevJob* __restrict__ job, const float2* __restrict__ spec,
                double2* __restrict__ vacc, int nf, int tiles_per_wg, int zchunks,
                int frames_per_split, size_t slot_stride) {
  static_assert(MP % kGroup == 0 && MP <= 32, "ring stages hold at most 32 inputs");
  static_assert(kRing == 8, "one LDS variable per stage");
  constexpr int KC = 64;
  constexpr int F4 = MP * KC / 2;     // float4 per stage
  __shared__ float4 r0[F4], r1[F4], r2[F4], r3[F4], r4[F4], r5[F4], r6[F4], r7[F4];
  const int bx = blockIdx.x, by = blockIdx.y, bz = blockIdx.z;
  const DevJob& J = *job;
  const int M = J.M, n_chan = J.n_chan, nbl = J.nbl;
  constexpr int ng = MP / kGroup;
  constexpr int ntiles = ng * (ng + 1) / 2;
  const int sb = by;
  const int k0 = bx * KC;
  const int zc = bz % zchunks, split = bz / zchunks;
  const int fa = split * frames_per_split;
  const int fz = min(nf, fa + frames_per_split);
  if (fa >= fz) return;   // whole workgroup
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  const int tile = zc * tiles_per_wg + wave;
  const bool active = wave < tiles_per_wg && tile < ntiles;
  // The loop body has no branches (a branch would hide from the compiler which
  // stage an in-flight load writes, and it would then wait for all of them):
  // waves without a tile multiply tile 0 and store nothing, and waves beyond
  // the MP / 2 loaders load rows 0 and 1 again, to the same LDS place as wave 0
  // (identical bytes).
  int gi = 0, gj = 0;
  tile_of(active ? tile : 0, ng, gi, gj);
  const int lw = wave < MP / 2 ? wave : 0;

  // this lane's source: row 2 lw + lane / 32 (rows past M repeat row M - 1;
  // their products are never stored), float4 column lane % 32
  // (a wave-uniform frame base plus a loop-invariant 32-bit lane offset)
  const int lrow = min(2 * lw + (lane >> 5), M - 1);
  const float4* gsrc = reinterpret_cast<const float4*>(spec + (size_t)sb * nf * M * n_chan + k0);
  const int loff = lrow * (n_chan / 2) + (lane & 31);
  const size_t fstride4 = (size_t)M * n_chan / 2;

  float2 acc[kGroup][kGroup];
#pragma unroll
  for (int a = 0; a < kGroup; ++a)
#pragma unroll
    for (int b = 0; b < kGroup; ++b) acc[a][b] = make_float2(0.f, 0.f);

  int j = fa;
  // frames fa .. fa + kRing - 2 (past the slice: frame fz - 1 again); stage
  // of frame f: (f - fa) mod kRing
  ring_load(gsrc + (size_t)fa * fstride4 + loff, r0 + lw * 64);
  ring_load(gsrc + (size_t)min(fa + 1, fz - 1) * fstride4 + loff, r1 + lw * 64);
  ring_load(gsrc + (size_t)min(fa + 2, fz - 1) * fstride4 + loff, r2 + lw * 64);
  ring_load(gsrc + (size_t)min(fa + 3, fz - 1) * fstride4 + loff, r3 + lw * 64);
  ring_load(gsrc + (size_t)min(fa + 4, fz - 1) * fstride4 + loff, r4 + lw * 64);
  ring_load(gsrc + (size_t)min(fa + 5, fz - 1) * fstride4 + loff, r5 + lw * 64);
  ring_load(gsrc + (size_t)min(fa + 6, fz - 1) * fstride4 + loff, r6 + lw * 64);
  // frame fa into registers A
  float2 aA[kGroup], bA[kGroup], aB[kGroup], bB[kGroup];
  __builtin_amdgcn_s_waitcnt(waitcnt_vm_lds(kRing - 2));
  __asm__ volatile("" ::: "memory");
  __builtin_amdgcn_s_barrier();
  __asm__ volatile("" ::: "memory");
  ring_read(reinterpret_cast<const float2*>(r0), gi, gj, lane, aA, bA);
  // whole rounds of kRing frames, then the rest; no path leads back into the
  // steps with a different set of loads in flight.  Frame j is in registers A
  // at even steps of a round, B at odd ones.
  for (int round = (fz - fa) / kRing; round > 0; --round) {
    XC_RING_STEP(r1, r7, aA, bA, aB, bB) XC_RING_STEP(r2, r0, aB, bB, aA, bA)
    XC_RING_STEP(r3, r1, aA, bA, aB, bB) XC_RING_STEP(r4, r2, aB, bB, aA, bA)
    XC_RING_STEP(r5, r3, aA, bA, aB, bB) XC_RING_STEP(r6, r4, aB, bB, aA, bA)
    XC_RING_STEP(r7, r5, aA, bA, aB, bB) XC_RING_STEP(r0, r6, aB, bB, aA, bA)
  }
  do {
    if (j >= fz) break;
    XC_RING_STEP(r1, r7, aA, bA, aB, bB)
    if (j >= fz) break;
    XC_RING_STEP(r2, r0, aB, bB, aA, bA)
    if (j >= fz) break;
    XC_RING_STEP(r3, r1, aA, bA, aB, bB)
    if (j >= fz) break;
    XC_RING_STEP(r4, r2, aB, bB, aA, bA)
    if (j >= fz) break;
    XC_RING_STEP(r5, r3, aA, bA, aB, bB)
    if (j >= fz) break;
    XC_RING_STEP(r6, r4, aB, bB, aA, bA)
    if (j >= fz) break;
    XC_RING_STEP(r7, r5, aA, bA, aB, bB)
  } while (false);
  // no load may still be writing LDS when the workgroup ends
  __builtin_amdgcn_s_waitcnt(waitcnt_vm(0));
  if (!active) return;
  double2* slot = vacc + (size_t)split * slot_stride;
#pragma unroll
  for (int x = 0; x < kGroup; ++x)
#pragma unroll
    for (int y = 0; y < kGroup; ++y) {
      const int i = gi * kGroup + x, j = gj * kGroup + y;
      if (i <= j && j < M) {
        double2* o = slot + ((size_t)sb * nbl + bl_index(i, j, M)) * n_chan + k0 + lane;
        double2 v = *o;
        v.x += (double)acc[x][y].x;
        v.y += (double)acc[x][y].y;
        *o = v;
      }
    }
}
#undef XC_RING_STEP

static hipError_t launch_ring(const DevJob* job, int M, int n_chan, int n_subbands,
                              const float2* spec, double2* vacc, size_t slot_stride, int nf,
                              int fps_max, int tpw_req, hipStream_t s) {
  const int Mp = (M + kGroup - 1) / kGroup * kGroup;
  const int ng = Mp / kGroup;
  const int ntiles = ng * (ng + 1) / 2;
  if (Mp > 32 || n_chan % 64 != 0) return hipErrorInvalidValue;
  int n_splits, fps;
  xmac_splits(nf, fps_max, M, n_chan, n_subbands, n_splits, fps);
  int tiles_per_wg = tpw_req > 0 && tpw_req < 16 ? tpw_req : 16;
  if (tiles_per_wg > ntiles) tiles_per_wg = ntiles;
  const int zchunks = (ntiles + tiles_per_wg - 1) / tiles_per_wg;
  // every row pair of a stage needs a loading wave
  const int waves = tiles_per_wg > Mp / 2 ? tiles_per_wg : Mp / 2;
  dim3 grid(n_chan / 64, n_subbands, zchunks * n_splits);
  dim3 block(64 * waves);
#define XMAC_RING(MPV)                                                                    \
  case MPV:                                                                               \
    hipLaunchKernelGGL((k_xmac_ring<MPV>), grid, block, 0, s, job, spec, vacc, nf,        \
                       tiles_per_wg, zchunks, fps, slot_stride);                          \
    break;
  switch (Mp) {
    XMAC_RING(4) XMAC_RING(8) XMAC_RING(12) XMAC_RING(16) XMAC_RING(20) XMAC_RING(24)
    XMAC_RING(28) XMAC_RING(32)
    default: return hipErrorInvalidValue;
  }
#undef XMAC_RING
  return hipGetLastError();
}

bool xmac_fused_ok(int M, int n_chan) {
  const int Mp = (M + kGroup - 1) / kGroup * kGroup;
  return Mp <= 32 && n_chan % 64 == 0;
}

long ringm_resident(int Mp);

// Slice count for a block of nf frames: among ceil(nf / 1024) .. ceil(nf /
// fps_max) slices, the one whose workgroups take the least time per compute
// unit — (rounds of R resident workgroups, w per slice) x (frames per slice
// plus the slot update, which moves the bytes of slot_frames frames of
// spectra); the fewest slices among equals.  Without an occupancy figure
// (R = 0), ceil(nf / fps_max).
static int split_count(int nf, int fps_max, long w, long R, int slot_frames) {
  const int hi = (nf + fps_max - 1) / fps_max;
  if (R <= 0 || w <= 0) return hi;
  int best = hi;
  long best_cost = -1;
  for (int n = (nf + 1023) / 1024; n <= hi; ++n) {
    const long cost = ((n * w + R - 1) / R) * ((long)((nf + n - 1) / n) + slot_frames);
    if (best_cost < 0 || cost < best_cost) {
      best_cost = cost;
      best = n;
    }
  }
  return best;
}

void xmac_splits(int nf, int fps_max, int M, int n_chan, int n_subbands, int& n_splits,
                 int& fps) {
  // by the ring-fed matrix kernel's grid (64-channel tiles, one workgroup per
  // tile, subband and slice) for every X kernel, so that all of them slice a
  // block alike and give the same sums; a slice's slot update reads and
  // writes M (M + 1) / 2 FP64 products per channel, the bytes of 2 (M + 1)
  // frames of FP32 spectra
  const int Mp = (M + kGroup - 1) / kGroup * kGroup;
  const bool ringm = Mp <= 32 && n_chan % 64 == 0;
  n_splits = ringm ? split_count(nf, fps_max, (long)(n_chan / 64) * n_subbands, ringm_resident(Mp),
                                 2 * (M + 1))
                   : (nf + fps_max - 1) / fps_max;
  if (n_splits < 1) n_splits = 1;   // (an empty block: one empty slice)
  fps = (nf + n_splits - 1) / n_splits;
}

// Matrix-core variant: the same products on v_mfma_f32_4x4x1 (16 blocks of
// 4 x 4 outer products per instruction).  A wave owns 16 channels of one
// subband and one frame slice, and the 4 x 4 input tiles (gi <= gj) of one
// part of the subband's tiles (all of them up to 24 inputs, else half, so
// that the accumulators stay in registers at two waves per SIMD).
// Block b of the instruction is lanes 4b .. 4b + 3 = channel c0 + b; the A
// operand's row x and the B operand's column y of a block sit in lane 4b + x
// and 4b + y, and register x of the result holds row x, column lane % 4.  So
// lane 4b + r loads input 4g + r of every group g at its channel (four lanes
// read 16 channels of one input: one 128-byte run), and that one register is
// the A operand of the tiles in row g and the B operand of the tiles in
// column g.  Each block element is a fused multiply-add into the accumulator
// with one rounding, and the four real products of a complex one are issued
// in the vector kernels' order, so the sums are bit-identical to theirs.
// Operands come straight from memory, D frames ahead in registers (no LDS, no
// barrier): the matrix cores do a tile's 64 FMAs in 4 instructions, and the
// vector units only negate, address and load.
template <int MG>
struct MfmaTiles {
  static constexpr int NT = MG * (MG + 1) / 2;
  int gi[NT], gj[NT];
  constexpr MfmaTiles() : gi(), gj() {
    int t = 0;
    for (int a = 0; a < MG; ++a)
      for (int b = a; b < MG; ++b) {
        gi[t] = a;
        gj[t] = b;
        ++t;
      }
  }
};

typedef float xm_f4 __attribute__((ext_vector_type(4)));

// Tiles [PART * ceil(NT / S), ...) of MG groups over frames fa .. fz - 1,
// added to the FP64 slot.  Tile indices are compile-time constants, so every
// operand is a register.
template <int MG, int S, int PART, int D>
__device__ __forceinline__ void xmfma32_part(const float2* __restrict__ src,
                                             const int (&roff)[MG], size_t fstride, int fa,
                                             int fz, int M, int n_chan, int nbl, int sb, int c,
                                             int r, double2* __restrict__ slot) {
  constexpr MfmaTiles<MG> tiles{};
  constexpr int NT = MfmaTiles<MG>::NT;
  constexpr int NTW = (NT + S - 1) / S;
  constexpr int T0 = PART * NTW;
  constexpr int NTP = NT - T0 < NTW ? NT - T0 : NTW;   // tiles of this part
  xm_f4 accr[NTP], acci[NTP];
#pragma unroll
  for (int t = 0; t < NTP; ++t) {
    accr[t] = (xm_f4){0.f, 0.f, 0.f, 0.f};
    acci[t] = (xm_f4){0.f, 0.f, 0.f, 0.f};
  }
  typedef float f2v __attribute__((ext_vector_type(2)));
  auto load = [&](int f, float2 (&x)[MG]) {
    const f2v* p = reinterpret_cast<const f2v*>(src + (size_t)f * fstride);
#pragma unroll
    for (int g = 0; g < MG; ++g) {
      // one reader per value: stream it past the caches; with several parts
      // the block's other waves read it again, from cache
      const f2v v = S == 1 ? __builtin_nontemporal_load(p + roff[g]) : p[roff[g]];
      x[g] = make_float2(v.x, v.y);
    }
  };
  auto mac = [&](const float2 (&x)[MG]) {
#pragma unroll
    for (int t = 0; t < NTP; ++t) {
      const float2 a = x[tiles.gi[T0 + t]], b = x[tiles.gj[T0 + t]];
      // re: a.y b.y, then a.x b.x; im: -a.x b.y, then a.y b.x
      accr[t] = __builtin_amdgcn_mfma_f32_4x4x1f32(a.y, b.y, accr[t], 0, 0, 0);
      accr[t] = __builtin_amdgcn_mfma_f32_4x4x1f32(a.x, b.x, accr[t], 0, 0, 0);
      acci[t] = __builtin_amdgcn_mfma_f32_4x4x1f32(-a.x, b.y, acci[t], 0, 0, 0);
      acci[t] = __builtin_amdgcn_mfma_f32_4x4x1f32(a.y, b.x, acci[t], 0, 0, 0);
    }
  };
  // xb[d] holds frame f + d.  Whole rounds of D frames run without a branch,
  // each register set reloaded (D frames ahead; past the slice, frame fz - 1
  // again) as soon as its products are issued; the last fz - f < D frames
  // are already in xb[0 ..] when the rounds end.
  float2 xb[D][MG];
#pragma unroll
  for (int d = 0; d < D; ++d) load(min(fa + d, fz - 1), xb[d]);
  int f = fa;
  for (; f + D <= fz; f += D) {
#pragma unroll
    for (int d = 0; d < D; ++d) {
      mac(xb[d]);
      load(min(f + d + D, fz - 1), xb[d]);
      // keep the reload here: left to itself the scheduler sinks every load
      // of the round below the last products, and the next round then waits
      // for loads it has only just issued
      __builtin_amdgcn_sched_barrier(0);
    }
  }
#pragma unroll
  for (int d = 0; d < D - 1; ++d)
    if (f + d < fz) mac(xb[d]);
#pragma unroll
  for (int t = 0; t < NTP; ++t) {
    const int gi = tiles.gi[T0 + t], gj = tiles.gj[T0 + t];
#pragma unroll
    for (int x = 0; x < kGroup; ++x) {
      const int i = gi * kGroup + x, j = gj * kGroup + r;
      if (i <= j && j < M) {
        double2* o = slot + ((size_t)sb * nbl + bl_index(i, j, M)) * n_chan + c;
        double2 v = *o;
        v.x += (double)accr[t][x];
        v.y += (double)acci[t][x];
        *o = v;
      }
    }
  }
}

// Workgroup: 4 / S channel blocks of 16 (fewer when the subband has fewer
// channels), S waves (parts) per block.
template <int MG, int S, int D>
__global__ void __launch_bounds__(256)
    k_xmac_mfma(const DevJob* __restrict__ job, const float2* __restrict__ spec,
                double2* __restrict__ vacc, int nf, int frames_per_split, size_t slot_stride) {
  const DevJob& J = *job;
  const int M = J.M, n_chan = J.n_chan, nbl = J.nbl;
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int blocks = (int)(blockDim.x >> 6) / S;   // channel blocks per workgroup
  const int r = lane & 3;
  const int c = (blockIdx.x * blocks + wave / S) * 16 + (lane >> 2);
  const int sb = blockIdx.y, split = blockIdx.z;
  const int fa = split * frames_per_split;
  const int fz = min(nf, fa + frames_per_split);
  if (fa >= fz) return;
  // this lane's rows 4g + r (rows past M repeat row M - 1: their products are
  // never stored)
  const float2* src = spec + (size_t)sb * nf * M * n_chan + c;
  int roff[MG];
#pragma unroll
  for (int g = 0; g < MG; ++g) roff[g] = min(4 * g + r, M - 1) * n_chan;
  const size_t fstride = (size_t)M * n_chan;
  double2* slot = vacc + (size_t)split * slot_stride;
  static_assert(S >= 1 && S <= 3, "one to three parts per channel block");
  const int part = wave % S;
  if (part == 0)
    xmfma32_part<MG, S, 0, D>(src, roff, fstride, fa, fz, M, n_chan, nbl, sb, c, r, slot);
  if constexpr (S >= 2)
    if (part == 1)
      xmfma32_part<MG, S, 1, D>(src, roff, fstride, fa, fz, M, n_chan, nbl, sb, c, r, slot);
  if constexpr (S >= 3)
    if (part == 2)
      xmfma32_part<MG, S, 2, D>(src, roff, fstride, fa, fz, M, n_chan, nbl, sb, c, r, slot);
}

// Parts per channel block and frames in flight per wave for MG groups: the
// accumulators (8 registers per tile) and D frames of operands (2 MG
// registers each) within 256 VGPRs, two waves per SIMD.  Measured on
// C4-shaped jobs (4096 channels, 1024 frames): splitting the tiles of 6 or 8
// groups over more waves, each reading every input again from cache, is
// slower (24 inputs 0.82 -> 1.20 ms, 32 inputs 1.70 -> 2.36 ms over three
// parts), and more frames in flight gain at most 3 %.
constexpr int mfma_parts(int MG) { return MG <= 6 ? 1 : 2; }
constexpr int mfma_depth(int MG) { return MG <= 4 ? 8 : MG == 5 || MG == 7 ? 4 : 3; }

static hipError_t launch_mfma(const DevJob* job, int M, int n_chan, int n_subbands,
                              const float2* spec, double2* vacc, size_t slot_stride, int nf,
                              int fps_max, hipStream_t s) {
  const int ng = (M + kGroup - 1) / kGroup;
  if (ng > 8 || n_chan % 16 != 0) return hipErrorInvalidValue;
  int n_splits, fps;
  xmac_splits(nf, fps_max, M, n_chan, n_subbands, n_splits, fps);
  const int S = mfma_parts(ng);
  int blocks = 4 / S;   // channel blocks per workgroup
  if (blocks > n_chan / 16) blocks = n_chan / 16;
  dim3 grid(n_chan / (16 * blocks), n_subbands, n_splits);
  dim3 block(64 * S * blocks);
#define XMAC_MFMA(NG)                                                                     \
  case NG:                                                                                \
    hipLaunchKernelGGL((k_xmac_mfma<NG, mfma_parts(NG), mfma_depth(NG)>), grid, block, 0, s,\
                       job, spec, vacc, nf, fps, slot_stride);                            \
    break;
  switch (ng) {
    XMAC_MFMA(1) XMAC_MFMA(2) XMAC_MFMA(3) XMAC_MFMA(4) XMAC_MFMA(5) XMAC_MFMA(6)
    XMAC_MFMA(7) XMAC_MFMA(8)
    default: return hipErrorInvalidValue;
  }
#undef XMAC_MFMA
  return hipGetLastError();
}

// Matrix cores fed through the LDS ring: the ring kernel's loads (one 1 KB
// global_load_lds per wave and frame, kRing - 1 frames ahead, one barrier per
// frame), the matrix kernel's products.  Every input is loaded once per
// workgroup however many waves multiply it.  A workgroup owns 64 channels of
// one subband and one frame slice; wave w multiplies channel block w % 4 (16
// channels) over part w / 4 of the 4 x 4 tiles, and loads the row pair w.
// Rows are paired (8q + x, 8q + 4 + x) and pair (q, x) sits at byte
// q * kRingmQuad + x * kRingmPair of a stage, so row 4g + r of every group
// g starts 64 r bytes into a 256-byte bank window: the 32 lanes of a half-wave
// (8 channels x 4 rows) read 32 different 8-byte bank pairs of the 64 banks.
// (The compiler pairs two groups' reads, a multiple of 512 bytes apart, into
// one read2st64, whose two addresses of a lane then share a bank; the counters
// show those conflicts, and a layout that prevents the pairing measured no
// faster.)  A last, half-filled quad (MP % 8 == 4) loads its rows again into
// the unused halves.  Products are issued in the vector kernels' order, so the
// sums are bit-identical to theirs.
constexpr int kRingmPair = 1024 + 64;   // bytes: 64 r mod 256 for the pair at x = r
// bytes per quad: a multiple of 512 (one LDS base register serves every row of
// a stage: read2st64 offsets count 512-byte units)
constexpr int kRingmQuad = 9 * 512;
static_assert(4 * kRingmPair <= kRingmQuad && kRingmQuad % 512 == 0, "quad layout");

constexpr int ringm_parts(int MP) { return (MP + 7) / 8; }

// One ring step for frame j, as the ring kernel's: wait, barrier, refill RF
// with frame j + kRing - 1, read frame j + 1 from RD into NEXT, multiply CUR.
#define XC_RINGM_STEP(RD, RF, CUR, NEXT)                                               \
  {                                                                                  \
    __builtin_amdgcn_sched_barrier(0);                                               \
    __builtin_amdgcn_s_waitcnt(waitcnt_vm_lds(kRing - 3));                           \
    __asm__ volatile("" ::: "memory");                                               \
    __builtin_amdgcn_s_barrier();                                                    \
    __asm__ volatile("" ::: "memory");                                               \
    __builtin_amdgcn_sched_barrier(0);                                               \
    ring_load(gsrc + (size_t)min(j + kRing - 1, fz - 1) * fstride4 + loff, RF + wbase);\
    read(reinterpret_cast<const float2*>(RD), NEXT);                                 \
    __builtin_amdgcn_sched_barrier(0);                                               \
    mac(CUR);                                                                        \
    ++j;                                                                             \
  }

template <int MP, int S, int PART>
__device__ __forceinline__ void ringm_part(float4* r0, float4* r1, float4* r2, float4* r3,
                                          float4* r4, float4* r5, float4* r6, float4* r7,
                                          const float4* __restrict__ gsrc, int loff,
                                          size_t fstride4, int wbase, int rbase, int fa,
                                          int fz, int M, int n_chan, int nbl, int sb, int c,
                                          int r, double2* __restrict__ slot) {
  constexpr int MG = MP / kGroup;
  constexpr MfmaTiles<MG> tiles{};
  constexpr int NT = MfmaTiles<MG>::NT;
  constexpr int NTW = (NT + S - 1) / S;
  constexpr int T0 = PART * NTW;
  constexpr int NTP = NT - T0 < NTW ? NT - T0 : NTW;
  static_assert(NTP >= 1, "every part has a tile");
  xm_f4 accr[NTP], acci[NTP];
#pragma unroll
  for (int t = 0; t < NTP; ++t) {
    accr[t] = (xm_f4){0.f, 0.f, 0.f, 0.f};
    acci[t] = (xm_f4){0.f, 0.f, 0.f, 0.f};
  }
  // row 4g + r of a stage: pair (g / 2, r), half g % 2 (groups this part's
  // tiles never touch are not read)
  auto read = [&](const float2* st, float2 (&x)[MG]) {
#pragma unroll
    for (int g = 0; g < MG; ++g) x[g] = st[rbase + (g >> 1) * (kRingmQuad / 8) + (g & 1) * 64];
  };
  auto mac = [&](const float2 (&x)[MG]) {
#pragma unroll
    for (int t = 0; t < NTP; ++t) {
      const float2 a = x[tiles.gi[T0 + t]], b = x[tiles.gj[T0 + t]];
      // re: a.y b.y, then a.x b.x; im: -a.x b.y, then a.y b.x
      accr[t] = __builtin_amdgcn_mfma_f32_4x4x1f32(a.y, b.y, accr[t], 0, 0, 0);
      accr[t] = __builtin_amdgcn_mfma_f32_4x4x1f32(a.x, b.x, accr[t], 0, 0, 0);
      acci[t] = __builtin_amdgcn_mfma_f32_4x4x1f32(-a.x, b.y, acci[t], 0, 0, 0);
      acci[t] = __builtin_amdgcn_mfma_f32_4x4x1f32(a.y, b.x, acci[t], 0, 0, 0);
    }
  };
  int j = fa;
  ring_load(gsrc + (size_t)fa * fstride4 + loff, r0 + wbase);
  ring_load(gsrc + (size_t)min(fa + 1, fz - 1) * fstride4 + loff, r1 + wbase);
  ring_load(gsrc + (size_t)min(fa + 2, fz - 1) * fstride4 + loff, r2 + wbase);
  ring_load(gsrc + (size_t)min(fa + 3, fz - 1) * fstride4 + loff, r3 + wbase);
  ring_load(gsrc + (size_t)min(fa + 4, fz - 1) * fstride4 + loff, r4 + wbase);
  ring_load(gsrc + (size_t)min(fa + 5, fz - 1) * fstride4 + loff, r5 + wbase);
  ring_load(gsrc + (size_t)min(fa + 6, fz - 1) * fstride4 + loff, r6 + wbase);
  float2 xA[MG], xB[MG];
  __builtin_amdgcn_s_waitcnt(waitcnt_vm_lds(kRing - 2));
  __asm__ volatile("" ::: "memory");
  __builtin_amdgcn_s_barrier();
  __asm__ volatile("" ::: "memory");
  read(reinterpret_cast<const float2*>(r0), xA);
  for (int round = (fz - fa) / kRing; round > 0; --round) {
    XC_RINGM_STEP(r1, r7, xA, xB) XC_RINGM_STEP(r2, r0, xB, xA)
    XC_RINGM_STEP(r3, r1, xA, xB) XC_RINGM_STEP(r4, r2, xB, xA)
    XC_RINGM_STEP(r5, r3, xA, xB) XC_RINGM_STEP(r6, r4, xB, xA)
    XC_RINGM_STEP(r7, r5, xA, xB) XC_RINGM_STEP(r0, r6, xB, xA)
  }
  do {
    if (j >= fz) break;
    XC_RINGM_STEP(r1, r7, xA, xB)
    if (j >= fz) break;
    XC_RINGM_STEP(r2, r0, xB, xA)
    if (j >= fz) break;
    XC_RINGM_STEP(r3, r1, xA, xB)
    if (j >= fz) break;
    XC_RINGM_STEP(r4, r2, xB, xA)
    if (j >= fz) break;
    XC_RINGM_STEP(r5, r3, xA, xB)
    if (j >= fz) break;
    XC_RINGM_STEP(r6, r4, xB, xA)
    if (j >= fz) break;
    XC_RINGM_STEP(r7, r5, xA, xB)
  } while (false);
  // no load may still be writing LDS when the workgroup ends
  __builtin_amdgcn_s_waitcnt(waitcnt_vm(0));
  // the slot addresses are formed here, not before the loop (where the
  // compiler would otherwise hold them through it)
  __asm__ volatile("" : "+v"(c), "+v"(r));
#pragma unroll
  for (int t = 0; t < NTP; ++t) {
    const int gi = tiles.gi[T0 + t], gj = tiles.gj[T0 + t];
#pragma unroll
    for (int x = 0; x < kGroup; ++x) {
      const int i = gi * kGroup + x, jj = gj * kGroup + r;
      if (i <= jj && jj < M) {
        double2* o = slot + ((size_t)sb * nbl + bl_index(i, jj, M)) * n_chan + c;
        double2 v = *o;
        v.x += (double)accr[t][x];
        v.y += (double)acci[t][x];
        *o = v;
      }
    }
  }
}
#undef XC_RINGM_STEP

// FUSED: one launch over the blocks of many jobs (a fused batch round) whose
// inputs pad to the same MP: workgroup b belongs to the item whose xblk0 is
// the last at or below b, and b - xblk0 enumerates that item's (channel tile,
// subband, frame slice) as blockIdx (x, y, z) does otherwise.
template <int MP, bool FUSED>
__global__ void __launch_bounds__(1024)
    k_xmac_ringm(const DevJob* __restrict__ job, const float2* __restrict__ spec,
                 double2* __restrict__ vacc, int nf, int frames_per_split, size_t slot_stride,
                 const FusedItem* __restrict__ items, int n_items) {
  static_assert(MP % kGroup == 0 && MP <= 32, "ring stages hold at most 32 inputs");
  static_assert(kRing == 8, "one LDS variable per stage");
  constexpr int S = ringm_parts(MP);
  constexpr int F4 = S * kRingmQuad / 16;   // float4 per stage
  __shared__ float4 r0[F4], r1[F4], r2[F4], r3[F4], r4[F4], r5[F4], r6[F4], r7[F4];
  int bx = blockIdx.x, by = blockIdx.y, bz = blockIdx.z;
  if constexpr (FUSED) {
    // the item table and its job descriptors as constant data (scalar loads)
    const FusedItemsK ik = fused_const(items);
    const int it = fused_find(ik, n_items, (int)blockIdx.x,
                              [](const auto& I) { return I.xblk0; });
    job = (const DevJob*)&ik[it].jd;
    spec = ik[it].spec;
    vacc = ik[it].vacc;
    nf = ik[it].nf;
    frames_per_split = ik[it].fps;
    slot_stride = ik[it].slot_stride;
    const int n_ct = job->n_chan / 64;
    int local = (int)blockIdx.x - ik[it].xblk0;
    bx = local % n_ct;
    local /= n_ct;
    by = local % job->n_subbands;
    bz = local / job->n_subbands;
  }
  const DevJob& J = *job;
  const int M = J.M, n_chan = J.n_chan, nbl = J.nbl;
  const int sb = by, k0 = bx * 64;
  const int split = bz;
  const int fa = split * frames_per_split;
  const int fz = min(nf, fa + frames_per_split);
  if (fa >= fz) return;   // whole workgroup
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  // loads: row pair (q, x) = rows 8q + x and 8q + 4 + x (a row past MP: the
  // first again; rows past M repeat row M - 1, their products never stored),
  // float4 column lane % 32 of the 64-channel tile
  const int q = wave >> 2, x = wave & 3;
  const int lo = 8 * q + x, hi = lo + 4 < MP ? lo + 4 : lo;
  const int row = min((lane >> 5) ? hi : lo, M - 1);
  const float4* gsrc = reinterpret_cast<const float4*>(spec + (size_t)sb * nf * M * n_chan + k0);
  const int loff = row * (n_chan / 2) + (lane & 31);
  const size_t fstride4 = (size_t)M * n_chan / 2;
  const int wbase = (q * kRingmQuad + x * kRingmPair) / 16;
  // products: channel block wave % 4, part wave / 4; lane 4b + r holds row
  // 4g + r of each group g at channel 16 (wave % 4) + b
  const int cb = wave & 3, part = wave >> 2;
  const int r = lane & 3, b = lane >> 2;
  const int rbase = r * (kRingmPair / 8) + cb * 16 + b;
  const int c = k0 + cb * 16 + b;
  double2* slot = vacc + (size_t)split * slot_stride;
  static_assert(S >= 1 && S <= 4, "one to four parts");
  if (part == 0)
    ringm_part<MP, S, 0>(r0, r1, r2, r3, r4, r5, r6, r7, gsrc, loff, fstride4, wbase, rbase, fa,
                         fz, M, n_chan, nbl, sb, c, r, slot);
  if constexpr (S >= 2)
    if (part == 1)
      ringm_part<MP, S, 1>(r0, r1, r2, r3, r4, r5, r6, r7, gsrc, loff, fstride4, wbase, rbase,
                           fa, fz, M, n_chan, nbl, sb, c, r, slot);
  if constexpr (S >= 3)
    if (part == 2)
      ringm_part<MP, S, 2>(r0, r1, r2, r3, r4, r5, r6, r7, gsrc, loff, fstride4, wbase, rbase,
                           fa, fz, M, n_chan, nbl, sb, c, r, slot);
  if constexpr (S >= 4)
    if (part == 3)
      ringm_part<MP, S, 3>(r0, r1, r2, r3, r4, r5, r6, r7, gsrc, loff, fstride4, wbase, rbase,
                           fa, fz, M, n_chan, nbl, sb, c, r, slot);
}

// Workgroups of the ring-fed matrix kernel (inputs padded to Mp) resident on
// the current device at once: its occupancy per compute unit times the
// compute units (0 where the device cannot be queried).  Set once per device
// and Mp (host threads may race to store the same value).
long ringm_resident(int Mp) {
  static std::atomic<long> cache[64][9];
  int dev = 0;
  if (Mp < 4 || Mp > 32 || Mp % kGroup != 0 || hipGetDevice(&dev) != hipSuccess || dev < 0 ||
      dev >= 64)
    return 0;
  long v = cache[dev][Mp / kGroup].load();
  if (v != 0) return v > 0 ? v : 0;
  const int threads = 256 * ringm_parts(Mp);
  int per_cu = 0, n_cu = 0;
  hipError_t e = hipErrorInvalidValue;
#define XMAC_RINGM_OCC(MPV)                                                                  \
  case MPV:                                                                                  \
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_xmac_ringm<MPV, false>, threads, \
                                                     0);                                     \
    break;
  switch (Mp) {
    XMAC_RINGM_OCC(4) XMAC_RINGM_OCC(8) XMAC_RINGM_OCC(12) XMAC_RINGM_OCC(16) XMAC_RINGM_OCC(20)
    XMAC_RINGM_OCC(24) XMAC_RINGM_OCC(28) XMAC_RINGM_OCC(32)
    default: break;
  }
#undef XMAC_RINGM_OCC
  if (e == hipSuccess) e = hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev);
  v = e == hipSuccess && per_cu > 0 && n_cu > 0 ? (long)per_cu * n_cu : -1;
  cache[dev][Mp / kGroup].store(v);
  return v > 0 ? v : 0;
}

static hipError_t launch_ringm(const DevJob* job, int M, int n_chan, int n_subbands,
                               const float2* spec, double2* vacc, size_t slot_stride, int nf,
                               int fps_max, hipStream_t s) {
  const int Mp = (M + kGroup - 1) / kGroup * kGroup;
  if (Mp > 32 || n_chan % 64 != 0) return hipErrorInvalidValue;
  int n_splits, fps;
  xmac_splits(nf, fps_max, M, n_chan, n_subbands, n_splits, fps);
  dim3 grid(n_chan / 64, n_subbands, n_splits);
  dim3 block(256 * ringm_parts(Mp));
#define XMAC_RINGM(MPV)                                                                   \
  case MPV:                                                                               \
    hipLaunchKernelGGL((k_xmac_ringm<MPV, false>), grid, block, 0, s, job, spec, vacc, nf, \
                       fps, slot_stride, nullptr, 0);                                     \
    break;
  switch (Mp) {
    XMAC_RINGM(4) XMAC_RINGM(8) XMAC_RINGM(12) XMAC_RINGM(16) XMAC_RINGM(20) XMAC_RINGM(24)
    XMAC_RINGM(28) XMAC_RINGM(32)
    default: return hipErrorInvalidValue;
  }
#undef XMAC_RINGM
  return hipGetLastError();
}

// Fused batches: the ring-fed matrix-core kernel, one workgroup per channel
// tile, subband and frame slice of each item.
int xmac_fused_blocks(int M, int n_chan, int n_subbands, int n_splits) {
  (void)M;
  return n_chan / 64 * n_subbands * n_splits;
}

hipError_t launch_xmac_fused(int Mp, const FusedItem* items, int n_items, int n_blocks,
                             hipStream_t s) {
  if (n_blocks <= 0) return hipSuccess;
  if (Mp > 32 || Mp % kGroup != 0) return hipErrorInvalidValue;
  const dim3 grid(n_blocks), block(256 * ringm_parts(Mp));
#define XMAC_FUSED(MPV)                                                                   \
  case MPV:                                                                               \
    hipLaunchKernelGGL((k_xmac_ringm<MPV, true>), grid, block, 0, s, nullptr, nullptr,    \
                       nullptr, 0, 0, 0, items, n_items);                                 \
    break;
  switch (Mp) {
    XMAC_FUSED(4) XMAC_FUSED(8) XMAC_FUSED(12) XMAC_FUSED(16) XMAC_FUSED(20) XMAC_FUSED(24)
    XMAC_FUSED(28) XMAC_FUSED(32)
    default: return hipErrorInvalidValue;
  }
#undef XMAC_FUSED
  return hipGetLastError();
}

static hipError_t launch_direct(const DevJob* job, int M, int n_chan, int n_subbands,
                                const float2* spec, double2* vacc, size_t slot_stride, int nf,
                                int fps_max, int kc_req, int tpw_req, hipStream_t s) {
  const int Mp = (M + kGroup - 1) / kGroup * kGroup;
  const int ng = Mp / kGroup;
  const int ntiles = ng * (ng + 1) / 2;
  int n_splits, fps;
  xmac_splits(nf, fps_max, M, n_chan, n_subbands, n_splits, fps);
  int KC = (kc_req == 16 || kc_req == 32 || kc_req == 64) ? kc_req : 64;
  if (KC > n_chan) KC = n_chan;
  int tiles_per_wg = tpw_req > 0 ? tpw_req : 1024 / KC;
  if (tiles_per_wg > 1024 / KC) tiles_per_wg = 1024 / KC;
  if (tiles_per_wg > ntiles) tiles_per_wg = ntiles;
  const int zchunks = (ntiles + tiles_per_wg - 1) / tiles_per_wg;
  dim3 grid(n_chan / KC, n_subbands, zchunks * n_splits);
  dim3 block(KC * tiles_per_wg);
  switch (KC) {
    case 64:
      hipLaunchKernelGGL(k_xmac_direct<64>, grid, block, 0, s, job, spec, vacc, nf, tiles_per_wg,
                         zchunks, fps, slot_stride);
      break;
    case 32:
      hipLaunchKernelGGL(k_xmac_direct<32>, grid, block, 0, s, job, spec, vacc, nf, tiles_per_wg,
                         zchunks, fps, slot_stride);
      break;
    default:
      hipLaunchKernelGGL(k_xmac_direct<16>, grid, block, 0, s, job, spec, vacc, nf, tiles_per_wg,
                         zchunks, fps, slot_stride);
      break;
  }
  return hipGetLastError();
}

int xmac_frames_per_split(int T, int M, int n_chan, int n_subbands) {
  // Longer slices cut the FP64 slot traffic (one read and write of the slot
  // per slice).  1024-frame slices where the ring-fed matrix kernel's
  // workgroups still give at least three waves per SIMD (C2 with the vector
  // ring: X stage 16.2 -> 15.6 ms per step; whole 2048-frame blocks leave
  // half the CUs idle: 24.4 ms); else 512-frame slices where the 64-channel
  // tiles give at least 512 workgroups (two per compute unit); else 256.
  const int Mp = (M + kGroup - 1) / kGroup * kGroup;
  const int ng = Mp / kGroup;
  const int ntiles = ng * (ng + 1) / 2;
  const long zchunks = (ntiles + 15) / 16;
  if (Mp <= 32 && n_chan % 64 == 0) {
    const long wgs1k = (long)(n_chan / 64) * n_subbands * ((T + 1023) / 1024);
    if (wgs1k * 4 * ringm_parts(Mp) >= 3L * 1024) {
      // slices of at most 1024 frames that fill whole rounds of resident
      // workgroups (a C2 block of 13 107 frames: 14 slices, 7 rounds of 256,
      // instead of 13, six and a half), up to twice ceil(T / 1024) slices
      const long R = ringm_resident(Mp);
      if (R <= 0) return 1024;
      const int lo = (T + 1023) / 1024;
      const int n = split_count(T, (T + 2 * lo - 1) / (2 * lo), (long)(n_chan / 64) * n_subbands, R,
                                2 * (M + 1));
      return (T + n - 1) / n;
    }
  }
  const long wgs = (long)(n_chan / 64) * n_subbands * zchunks * ((T + 511) / 512);
  return wgs >= 512 ? 512 : 256;
}

template <int FB>
static hipError_t launch_fb(const DevJob* job, int M, int n_chan, int n_subbands,
                            const float2* spec, double2* vacc, size_t slot_stride, int nf,
                            int fps_max, int kc_req, int tpw_req, hipStream_t s) {
  const int Mp = (M + kGroup - 1) / kGroup * kGroup;
  const int ng = Mp / kGroup;
  const int ntiles = ng * (ng + 1) / 2;
  int n_splits, fps;
  xmac_splits(nf, fps_max, M, n_chan, n_subbands, n_splits, fps);
  auto lds_of = [&](int kc) { return 2 * (size_t)FB * Mp * (kc + 2) * sizeof(float2); };
  // widest channel tile that fits 64 KB of LDS and still gives a few
  // workgroups per compute unit; else the narrowest (unless one is requested)
  int KC = 16;
  if (kc_req == 16 || kc_req == 32 || kc_req == 64) {
    KC = kc_req <= n_chan ? kc_req : 16;
  } else {
    for (int kc : {64, 32}) {
      const int tpw = 1024 / kc < ntiles ? 1024 / kc : ntiles;
      const long wgs = (long)(n_chan / kc) * n_subbands * ((ntiles + tpw - 1) / tpw) * n_splits;
      if (kc <= n_chan && wgs >= 1024 && lds_of(kc) <= 65536) {
        KC = kc;
        break;
      }
    }
  }
  int tiles_per_wg = tpw_req > 0 && tpw_req < 1024 / KC ? tpw_req : 1024 / KC;
  // enough threads that each stages at most 16 float4 per LDS stage
  const int min_tpw = (FB * M * (KC / 2) + 16 * KC - 1) / (16 * KC);
  if (tiles_per_wg < min_tpw) tiles_per_wg = min_tpw;
  if (tiles_per_wg > ntiles) tiles_per_wg = ntiles;
  const int zchunks = (ntiles + tiles_per_wg - 1) / tiles_per_wg;
  const int nthr = KC * tiles_per_wg;
  const size_t lds = lds_of(KC);
  if (lds > 160 * 1024) return hipErrorInvalidValue;
  // float4 loads per thread per stage (the kernels hold up to MAXL in registers)
  const int per_thr = (FB * M * (KC / 2) + nthr - 1) / nthr;
  dim3 grid(n_chan / KC, n_subbands, zchunks * n_splits);
  dim3 block(nthr);
#define XMAC_LAUNCH(KCV, MAXLV)                                                                 \
  do {                                                                                         \
    auto kern = k_xmac<KCV, FB, MAXLV>;                                                        \
    if (lds > 65536) {                                                                         \
      hipError_t e = hipFuncSetAttribute((const void*)kern,                                    \
                                         hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);\
      if (e != hipSuccess) return e;                                                           \
    }                                                                                          \
    hipLaunchKernelGGL(kern, grid, block, lds, s, job, spec, vacc, nf, tiles_per_wg, zchunks,  \
                       fps, slot_stride);                                                      \
  } while (0)
  if (per_thr <= 4) {
    if (KC == 64) XMAC_LAUNCH(64, 4); else if (KC == 32) XMAC_LAUNCH(32, 4); else XMAC_LAUNCH(16, 4);
  } else if (per_thr <= 16) {
    if (KC == 64) XMAC_LAUNCH(64, 16); else if (KC == 32) XMAC_LAUNCH(32, 16); else XMAC_LAUNCH(16, 16);
  } else {
    return hipErrorInvalidValue;
  }
#undef XMAC_LAUNCH
  return hipGetLastError();
}

hipError_t launch_xmac(const DevJob* job, int M, int n_chan, int n_subbands,
                       const float2* spec, double2* vacc, size_t slot_stride, int nf, int fps,
                       int fb, int kc, int tpw, hipStream_t s) {
  if (fps < 1) return hipErrorInvalidValue;
  const int Mp = (M + kGroup - 1) / kGroup * kGroup;
  // default up to 32 inputs: the matrix cores fed through the LDS ring
  // (C4-shaped jobs of 1024 frames, against the vector ring: 32 inputs 0.76
  // vs 2.08 ms, 24: 0.57 vs 1.06, 20: 0.475 vs 0.485, 4: 0.086 vs 0.097, 8
  // and 16 equal within 2 %; the vector units are left free)
  if (fb == 0 && Mp <= 32 && kc == 0 && tpw == 0 && n_chan % 64 == 0) fb = kXmacMatrixRing;
  if ((fb == 0 || fb == kRing) && Mp <= 32 && (kc == 0 || kc == 64))
    return launch_ring(job, M, n_chan, n_subbands, spec, vacc, slot_stride, nf, fps, tpw, s);
  if (fb == kXmacMatrixRing && Mp <= 32 && n_chan % 64 == 0)
    return launch_ringm(job, M, n_chan, n_subbands, spec, vacc, slot_stride, nf, fps, s);
  if (fb == kXmacMatrix && Mp <= 32 && n_chan % 16 == 0)
    return launch_mfma(job, M, n_chan, n_subbands, spec, vacc, slot_stride, nf, fps, s);
  if (fb == 1)
    return launch_direct(job, M, n_chan, n_subbands, spec, vacc, slot_stride, nf, fps, kc, tpw,
                         s);
  if (fb == 4)
    return launch_fb<4>(job, M, n_chan, n_subbands, spec, vacc, slot_stride, nf, fps, kc, tpw, s);
  return launch_fb<2>(job, M, n_chan, n_subbands, spec, vacc, slot_stride, nf, fps, kc, tpw, s);
}

}  // namespace xc
