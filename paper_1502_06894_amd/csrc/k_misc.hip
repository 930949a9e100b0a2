// Small kernels: recording ingest (A0), delay/phase model per frame (A1),
// accumulator clearing, finalise (A8) and the unpack test tap.
#include "xc_launch.h"

namespace xc {

__global__ void k_ingest(const uint32_t* __restrict__ words, int64_t n_frames,
                         uint8_t* __restrict__ ok) {
  const int64_t f = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (f < n_frames) ok[f] = words[f * kFrameWords] == kSync ? 1 : 0;
}

hipError_t launch_ingest(const uint32_t* words, int64_t n_frames, uint8_t* frame_ok,
                         hipStream_t s) {
  if (n_frames <= 0) return hipSuccess;
  const int b = 256;
  const int64_t g = (n_frames + b - 1) / b;
  hipLaunchKernelGGL(k_ingest, dim3((unsigned)g), dim3(b), 0, s, words, n_frames, frame_ok);
  return hipGetLastError();
}

__global__ void k_zero(double* __restrict__ p, size_t n) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (size_t)gridDim.x * blockDim.x)
    p[i] = 0.0;
}

hipError_t launch_zero(double* p, size_t n, hipStream_t s) {
  if (n == 0) return hipSuccess;
  size_t g = (n + 255) / 256;
  if (g > 65536) g = 65536;
  hipLaunchKernelGGL(k_zero, dim3((unsigned)g), dim3(256), 0, s, p, n);
  return hipGetLastError();
}

// Delay record (subband 0 only) and phase record of frame fl of a block
// starting at frame f0, station s, subband sb.
__device__ inline void delay_phase_records(const DevJob& J, int s, int sb, int64_t f0, int fl,
                                           int nf, DelayRec* __restrict__ drec,
                                           PhaseRec* __restrict__ prec) {
  const DevStation& S = J.st[s];
  const int64_t f = f0 + fl;
  const int64_t num = J.sub_start + f * (int64_t)J.N + (int64_t)(J.N / 2);
  const double t = (double)num / J.fs;
  // one thread per (frame, station, subband): each writes its subband's phase
  // record, the subband-0 thread also the frame's delay record
  prec[((size_t)s * J.n_subbands + sb) * nf + fl] = frame_phase(S, J, sb, t);
  if (sb != 0) return;
  DelayRec r;
  frame_delay(S, J, f, &r.n_int, &r.d);
  r.base = J.sub_start + f * (int64_t)J.N + r.n_int - S.first_sample;
  const int64_t n_samples = S.n_frames_m5b * (int64_t)J.spf;
  bool ok = r.base >= 0 && r.base + J.N <= n_samples;
  if (ok) {
    const int64_t a = r.base / J.spf, b = (r.base + J.N - 1) / J.spf;
    for (int64_t m = a; m <= b; ++m) ok = ok && S.frame_ok[m] != 0;
  }
  r.valid = ok ? 1 : 0;
  double d1, d2;
  poly_derivs(S.delay_poly, S.poly_deg, t, d1, d2);
  r.rate = (float)d1;
  drec[(size_t)s * nf + fl] = r;
}

// One thread per (station, block frame, subband).  Writes the subband's fringe
// phase terms; the subband-0 thread also the integer/fractional delay, the
// validity and the delay rate of the frame.
__global__ void k_delays(const DevJob* __restrict__ job, int64_t f0, int nf,
                         DelayRec* __restrict__ drec, PhaseRec* __restrict__ prec,
                         unsigned* __restrict__ ctr) {
  const int fl = blockIdx.x * blockDim.x + threadIdx.x;
  const int s = blockIdx.y, sb = blockIdx.z;
  if (ctr && fl == 0 && s == 0 && sb == 0) {
    ctr[0] = 0u;   // the F stage's task counter
    ctr[1] = 0u;   // the drift-correction pass's
  }
  if (fl >= nf) return;
  delay_phase_records(*job, s, sb, f0, fl, nf, drec, prec);
}

hipError_t launch_delays(const DevJob* job, int n_stations, int n_subbands, int64_t f0, int nf,
                         DelayRec* drec, PhaseRec* prec, unsigned* ctr, hipStream_t s) {
  const int b = 64;
  dim3 grid((nf + b - 1) / b, n_stations, n_subbands);
  hipLaunchKernelGGL(k_delays, grid, dim3(b), 0, s, job, f0, nf, drec, prec, ctr);
  return hipGetLastError();
}

constexpr int kDelayThreads = 64;

int delays_fused_blocks(int nf, int n_stations, int n_subbands) {
  return (nf + kDelayThreads - 1) / kDelayThreads * n_stations * n_subbands;
}

// k_delays over the blocks of a fused round: workgroup -> (item, frame chunk,
// station, subband).
__global__ void __launch_bounds__(kDelayThreads)
    k_delays_fused(const FusedItem* __restrict__ items, int n_items, unsigned* __restrict__ ctr) {
  const int it = fused_find(items, n_items, (int)blockIdx.x,
                            [](const FusedItem& I) { return I.dblk0; });
  const FusedItem& I = items[it];
  const DevJob& J = I.jd;
  if (ctr && blockIdx.x == 0 && threadIdx.x == 0) {
    ctr[0] = 0u;
    ctr[1] = 0u;
  }
  const int nfb = (I.nf + kDelayThreads - 1) / kDelayThreads;
  int local = (int)blockIdx.x - I.dblk0;
  const int fb = local % nfb;
  local /= nfb;
  const int s = local % J.n_stations, sb = local / J.n_stations;
  const int fl = fb * kDelayThreads + (int)threadIdx.x;
  if (fl >= I.nf) return;
  delay_phase_records(J, s, sb, I.f0, fl, I.nf, I.drec, I.prec);
}

hipError_t launch_delays_fused(const FusedItem* items, int n_items, int n_blocks, unsigned* ctr,
                               hipStream_t s) {
  if (n_blocks <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_delays_fused, dim3(n_blocks), dim3(kDelayThreads), 0, s, items, n_items,
                     ctr);
  return hipGetLastError();
}

// One workgroup per station pair (si <= sj) and chunk of kWeightChunk frames:
// count the frames valid for both and add the count to the pair's total.  The
// counts are integers, exact in FP64 whatever order the chunks add in.
constexpr int kWeightChunk = 2048;

__device__ inline void pair_weights(const DelayRec* __restrict__ drec, int S, int nf,
                                    double* __restrict__ wst, int si, int sj, int chunk,
                                    int* part) {
  const int f0 = chunk * kWeightChunk;
  const int f1 = nf < f0 + kWeightChunk ? nf : f0 + kWeightChunk;
  int cnt = 0;
#pragma unroll 8
  for (int f = f0 + (int)threadIdx.x; f < f1; f += blockDim.x)
    cnt += drec[(size_t)si * nf + f].valid & drec[(size_t)sj * nf + f].valid;
  part[threadIdx.x] = cnt;
  __syncthreads();
  for (int w = blockDim.x / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) part[threadIdx.x] += part[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0 && part[0] != 0) atomicAdd(&wst[si * S + sj], (double)part[0]);
}

__global__ void k_weights(const DelayRec* __restrict__ drec, int S, int nf,
                          double* __restrict__ wst) {
  const int si = blockIdx.x, sj = blockIdx.y;
  if (sj < si) return;
  __shared__ int part[256];
  pair_weights(drec, S, nf, wst, si, sj, blockIdx.z, part);
}

int weights_fused_blocks(int nf, int n_stations) {
  return n_stations * n_stations * ((nf + kWeightChunk - 1) / kWeightChunk);
}

// k_weights over the blocks of a fused round: workgroup -> (item, si, sj, chunk).
__global__ void k_weights_fused(const FusedItem* __restrict__ items, int n_items) {
  const int it = fused_find(items, n_items, (int)blockIdx.x,
                            [](const FusedItem& I) { return I.wblk0; });
  const FusedItem& I = items[it];
  const int S = I.jd.n_stations;
  int local = (int)blockIdx.x - I.wblk0;
  const int si = local % S;
  local /= S;
  const int sj = local % S, chunk = local / S;
  if (sj < si) return;
  __shared__ int part[256];
  pair_weights(I.drec, S, I.nf, I.wst, si, sj, chunk, part);
}

hipError_t launch_weights_fused(const FusedItem* items, int n_items, int n_blocks, hipStream_t s) {
  if (n_blocks <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_weights_fused, dim3(n_blocks), dim3(256), 0, s, items, n_items);
  return hipGetLastError();
}

hipError_t launch_weights(const DelayRec* drec, int n_stations, int nf, double* wst,
                          hipStream_t s) {
  const dim3 grid(n_stations, n_stations, (nf + kWeightChunk - 1) / kWeightChunk);
  hipLaunchKernelGGL(k_weights, grid, dim3(256), 0, s, drec, n_stations, nf, wst);
  return hipGetLastError();
}

// Element e of a job's output: the sum of its n_slots FP64 slots over the
// weight of its station pair (W = 0 -> 0); the k = 0 element also writes W.
__device__ inline void finalise_elem(const double2* __restrict__ vacc, int n_slots,
                                     size_t slot_stride, const double* __restrict__ wst, int S,
                                     int P, int M, float2* __restrict__ vis,
                                     float* __restrict__ weight, int nbl, int n_chan, size_t e) {
  const size_t row = e / n_chan;          // sb * nbl + bl
  const int k = (int)(e - row * n_chan);
  const int bl = (int)(row % nbl);
  int i = 0, rem = bl;                    // bl -> (i, j), row-major upper triangle
  while (rem >= M - i) {
    rem -= M - i;
    ++i;
  }
  const int j = i + rem;
  const double w = wst[(i / P) * S + (j / P)];
  double2 a = vacc[e];
  // fixed slot order; the loads of eight slots are issued together (a job of
  // few channels and baselines can have over a hundred slots)
  int q = 1;
  for (; q + 8 <= n_slots; q += 8) {
    double2 b[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) b[u] = vacc[e + (size_t)(q + u) * slot_stride];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      a.x += b[u].x;
      a.y += b[u].y;
    }
  }
  for (; q < n_slots; ++q) {
    const double2 b = vacc[e + (size_t)q * slot_stride];
    a.x += b.x;
    a.y += b.y;
  }
  vis[e] = w > 0.0 ? make_float2((float)(a.x / w), (float)(a.y / w)) : make_float2(0.f, 0.f);
  if (k == 0) weight[row] = (float)w;
}

__global__ void k_finalise(const double2* __restrict__ vacc, int n_slots, size_t slot_stride,
                           const double* __restrict__ wst, int S, int P, int M,
                           float2* __restrict__ vis, float* __restrict__ weight, int nbl,
                           int n_chan, size_t total) {
  const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= total) return;
  finalise_elem(vacc, n_slots, slot_stride, wst, S, P, M, vis, weight, nbl, n_chan, e);
}

constexpr int kFinaliseThreads = 256;

int finalise_fused_blocks(int n_subbands, int M, int n_chan) {
  const size_t total = (size_t)n_subbands * (M * (M + 1) / 2) * n_chan;
  return (int)((total + kFinaliseThreads - 1) / kFinaliseThreads);
}

// k_finalise over the jobs of a fused batch: workgroup -> (job, element chunk).
__global__ void __launch_bounds__(kFinaliseThreads)
    k_finalise_fused(const FusedOut* __restrict__ outs, int n_outs) {
  int lo = 0, hi = n_outs - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (outs[mid].blk0 <= (int)blockIdx.x)
      lo = mid;
    else
      hi = mid - 1;
  }
  const FusedOut& O = outs[lo];
  const size_t total = (size_t)O.n_sb * O.nbl * O.n_chan;
  const size_t e = (size_t)((int)blockIdx.x - O.blk0) * kFinaliseThreads + threadIdx.x;
  if (e >= total) return;
  finalise_elem(O.vacc, O.n_slots, O.slot_stride, O.wst, O.S, O.P, O.M, O.vis, O.weight, O.nbl,
                O.n_chan, e);
}

hipError_t launch_finalise_fused(const FusedOut* outs, int n_outs, int n_blocks, hipStream_t s) {
  if (n_blocks <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_finalise_fused, dim3(n_blocks), dim3(kFinaliseThreads), 0, s, outs,
                     n_outs);
  return hipGetLastError();
}

// k_ingest over many recordings: workgroup -> (recording, frame chunk).
__global__ void k_ingest_fused(const FusedMask* __restrict__ masks, int n_masks) {
  int lo = 0, hi = n_masks - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (masks[mid].blk0 <= (int)blockIdx.x)
      lo = mid;
    else
      hi = mid - 1;
  }
  const FusedMask& K = masks[lo];
  const int64_t f = (int64_t)((int)blockIdx.x - K.blk0) * blockDim.x + threadIdx.x;
  if (f < K.n_frames) K.ok[f] = K.words[f * kFrameWords] == kSync ? 1 : 0;
}

int ingest_fused_blocks(int64_t n_frames) { return (int)((n_frames + 255) / 256); }

hipError_t launch_ingest_fused(const FusedMask* masks, int n_masks, int n_blocks, hipStream_t s) {
  if (n_blocks <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_ingest_fused, dim3(n_blocks), dim3(256), 0, s, masks, n_masks);
  return hipGetLastError();
}

hipError_t launch_finalise(const double2* vacc, int n_slots, size_t slot_stride,
                           const double* wst, int n_stations, int n_pols, float2* vis,
                           float* weight, int n_subbands, int M, int n_chan, hipStream_t s) {
  const int nbl = M * (M + 1) / 2;
  const size_t total = (size_t)n_subbands * nbl * n_chan;
  const size_t g = (total + 255) / 256;
  hipLaunchKernelGGL(k_finalise, dim3((unsigned)g), dim3(256), 0, s, vacc, n_slots, slot_stride,
                     wst, n_stations, n_pols, M, vis, weight, nbl, n_chan, total);
  return hipGetLastError();
}

// Unpack tap: the same addressing the F stage uses, one thread per sample.
__global__ void k_debug_unpack(const DevJob* __restrict__ job, const DelayRec* __restrict__ drec,
                               int nf, int station, int input, int fl, float* __restrict__ out) {
  const DevJob& J = *job;
  const int n = blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= J.N) return;
  const DelayRec r = drec[(size_t)station * nf + fl];
  if (!r.valid) {
    out[n] = 0.f;
    return;
  }
  const FrameCursor c = make_cursor(J, r.base);
  const uint32_t w = *sample_word(J, J.st[station].words, c, n);
  out[n] = level_of((w >> (sample_shift(J, c, n) + 2 * J.stream_map[input])) & 3u);
}

hipError_t launch_debug_unpack(const DevJob* job, const DelayRec* drec, int nf, int station,
                               int input, int fl, float* out, int N, hipStream_t s) {
  hipLaunchKernelGGL(k_debug_unpack, dim3((N + 255) / 256), dim3(256), 0, s, job, drec, nf,
                     station, input, fl, out);
  return hipGetLastError();
}

}  // namespace xc
