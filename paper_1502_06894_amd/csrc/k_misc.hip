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
  const DevJob& J = *job;
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

hipError_t launch_delays(const DevJob* job, int n_stations, int n_subbands, int64_t f0, int nf,
                         DelayRec* drec, PhaseRec* prec, unsigned* ctr, hipStream_t s) {
  const int b = 64;
  dim3 grid((nf + b - 1) / b, n_stations, n_subbands);
  hipLaunchKernelGGL(k_delays, grid, dim3(b), 0, s, job, f0, nf, drec, prec, ctr);
  return hipGetLastError();
}

// One workgroup per station pair (si <= sj) and chunk of kWeightChunk frames:
// count the frames valid for both and add the count to the pair's total.  The
// counts are integers, exact in FP64 whatever order the chunks add in.
constexpr int kWeightChunk = 2048;

__global__ void k_weights(const DelayRec* __restrict__ drec, int S, int nf,
                          double* __restrict__ wst) {
  const int si = blockIdx.x, sj = blockIdx.y;
  if (sj < si) return;
  const int f0 = blockIdx.z * kWeightChunk;
  const int f1 = nf < f0 + kWeightChunk ? nf : f0 + kWeightChunk;
  __shared__ int part[256];
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

hipError_t launch_weights(const DelayRec* drec, int n_stations, int nf, double* wst,
                          hipStream_t s) {
  const dim3 grid(n_stations, n_stations, (nf + kWeightChunk - 1) / kWeightChunk);
  hipLaunchKernelGGL(k_weights, grid, dim3(256), 0, s, drec, n_stations, nf, wst);
  return hipGetLastError();
}

__global__ void k_finalise(const double2* __restrict__ vacc, int n_slots, size_t slot_stride,
                           const double* __restrict__ wst, int S, int P, int M,
                           float2* __restrict__ vis, float* __restrict__ weight, int nbl,
                           int n_chan, size_t total) {
  const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= total) return;
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
