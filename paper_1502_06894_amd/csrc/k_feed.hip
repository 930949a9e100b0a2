// Feed-angle (parallactic-angle-equivalent) correction of dual-polarisation
// products (section 2's capability list; angles are inputs).  One workgroup per
// (sub-integration, subband, station pair a <= b, chunk of channels) rewrites
// the pair's three or four product rows in place.  The phasors depend only on
// the sub-integration and the pair: each wave evaluates them once in FP64 (one
// lane per angle) and broadcasts them; the channel loop is a plain HBM stream
// of 16-byte loads and stores (two channels a lane) when the rows allow it.
#include <math.h>
#include <stdint.h>

#include <algorithm>

#include "xc_launch.h"
#include "xc_runtime.h"

namespace xc {

namespace {

constexpr int kFeedUnroll = 2;  // vector units a thread keeps in flight per row

__device__ inline int pair_bl(int i, int j, int M) { return i * M - (i * (i - 1)) / 2 + (j - i); }

__device__ inline float2 cmulf(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

template <int V>
__device__ inline void ld(const float2* p, float2 (&o)[V]) {
  if constexpr (V == 2) {
    const float4 q = *reinterpret_cast<const float4*>(p);
    o[0] = make_float2(q.x, q.y);
    o[1] = make_float2(q.z, q.w);
  } else {
    o[0] = *p;
  }
}

template <int V>
__device__ inline void st(float2* p, const float2 (&o)[V]) {
  if constexpr (V == 2)
    *reinterpret_cast<float4*>(p) = make_float4(o[0].x, o[0].y, o[1].x, o[1].y);
  else
    *p = o[0];
}

// V channels per lane (2: 16-byte accesses, needs an even channel count and a
// 16-byte aligned buffer); the workgroup covers blockDim.x * V * kFeedUnroll
// channels of its chunk.
template <int FEED, int V>
__global__ __launch_bounds__(256) void k_feed(float2* __restrict__ vis,
                                               const double* __restrict__ angles, int n_sb, int S,
                                               int n_chan, int chunks) {
  constexpr int U = kFeedUnroll;
  const int M = 2 * S, npairs = S * (S + 1) / 2;
  const size_t nbl = (size_t)M * (M + 1) / 2;
  size_t g = blockIdx.x;
  const int chunk = (int)(g % chunks);
  g /= chunks;
  const int pr = (int)(g % npairs);
  g /= npairs;
  const int sb = (int)(g % n_sb);
  const size_t t = g / n_sb;
  // station pair pr -> (a, b), a <= b, row-major over the upper triangle
  int a = 0, rem = pr;
  while (rem >= S - a) {
    rem -= S - a;
    ++a;
  }
  const int b = a + rem;
  const bool full = a != b;  // a = b stores only (0,0), (0,1), (1,1)

  // Phasor terms, FP64 then rounded: circular needs exp(i(ca - cb)) and
  // exp(i(ca + cb)) (the other two are their conjugates, since the signs are
  // exact), linear needs the cosines and sines of ca and cb.
  const double ca = angles[t * S + a], cb = angles[t * S + b];
  const int lane = threadIdx.x & 63;
  const double x = FEED == XC_FEED_CIRCULAR ? (lane == 0 ? ca - cb : ca + cb) : (lane == 0 ? ca : cb);
  double sx, cx;
  sincos(x, &sx, &cx);
  const float c0 = __shfl((float)cx, 0), s0 = __shfl((float)sx, 0);
  const float c1 = __shfl((float)cx, 1), s1 = __shfl((float)sx, 1);

  float2* base = vis + ((size_t)t * n_sb + sb) * nbl * (size_t)n_chan;
  float2* row[4] = {base + (size_t)pair_bl(2 * a, 2 * b, M) * n_chan,
                    base + (size_t)pair_bl(2 * a, 2 * b + 1, M) * n_chan,
                    base + (size_t)(full ? pair_bl(2 * a + 1, 2 * b, M) : 0) * n_chan,
                    base + (size_t)pair_bl(2 * a + 1, 2 * b + 1, M) * n_chan};
  const int step = blockDim.x * V;
  const int k0 = chunk * step * U + threadIdx.x * V;

  float2 v[4][U][V];
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const int k = k0 + u * step;
    if (k < n_chan) {
      ld<V>(row[0] + k, v[0][u]);
      ld<V>(row[1] + k, v[1][u]);
      if (full) ld<V>(row[2] + k, v[2][u]);
      ld<V>(row[3] + k, v[3][u]);
    }
  }
#pragma unroll
  for (int u = 0; u < U; ++u)
#pragma unroll
    for (int e = 0; e < V; ++e) {
      if constexpr (FEED == XC_FEED_CIRCULAR) {
        // s_p ca - s_q cb with s_R = +1, s_L = -1
        v[0][u][e] = cmulf(v[0][u][e], make_float2(c0, s0));
        v[1][u][e] = cmulf(v[1][u][e], make_float2(c1, s1));
        v[2][u][e] = cmulf(v[2][u][e], make_float2(c1, -s1));
        v[3][u][e] = cmulf(v[3][u][e], make_float2(c0, -s0));
      } else {
        // V <- Rot(ca)^T V Rot(cb), Rot = [[c, s], [-s, c]]
        const float2 v00 = v[0][u][e], v01 = v[1][u][e], v11 = v[3][u][e];
        const float2 v10 = full ? v[2][u][e] : make_float2(v01.x, -v01.y);
        // U = Rot(ca)^T V with Rot(ca)^T = [[c0, -s0], [s0, c0]]
        const float2 u00 = make_float2(c0 * v00.x - s0 * v10.x, c0 * v00.y - s0 * v10.y);
        const float2 u01 = make_float2(c0 * v01.x - s0 * v11.x, c0 * v01.y - s0 * v11.y);
        const float2 u10 = make_float2(s0 * v00.x + c0 * v10.x, s0 * v00.y + c0 * v10.y);
        const float2 u11 = make_float2(s0 * v01.x + c0 * v11.x, s0 * v01.y + c0 * v11.y);
        // then U Rot(cb) with Rot(cb) = [[c1, s1], [-s1, c1]]
        v[0][u][e] = make_float2(c1 * u00.x - s1 * u01.x, c1 * u00.y - s1 * u01.y);
        v[1][u][e] = make_float2(s1 * u00.x + c1 * u01.x, s1 * u00.y + c1 * u01.y);
        v[2][u][e] = make_float2(c1 * u10.x - s1 * u11.x, c1 * u10.y - s1 * u11.y);
        v[3][u][e] = make_float2(s1 * u10.x + c1 * u11.x, s1 * u10.y + c1 * u11.y);
      }
    }
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const int k = k0 + u * step;
    if (k < n_chan) {
      st<V>(row[0] + k, v[0][u]);
      st<V>(row[1] + k, v[1][u]);
      if (full) st<V>(row[2] + k, v[2][u]);
      st<V>(row[3] + k, v[3][u]);
    }
  }
}

template <int FEED>
void launch_feed(float2* vis, const double* angles, int n_sb, int S, int n_chan, bool vec,
                 unsigned blocks, int threads, int chunks, hipStream_t s) {
  if (vec)
    hipLaunchKernelGGL((k_feed<FEED, 2>), dim3(blocks), dim3(threads), 0, s, vis, angles, n_sb, S,
                       n_chan, chunks);
  else
    hipLaunchKernelGGL((k_feed<FEED, 1>), dim3(blocks), dim3(threads), 0, s, vis, angles, n_sb, S,
                       n_chan, chunks);
}

}  // namespace

}  // namespace xc

using namespace xc;

extern "C" int xc_feed_correct(xc_ctx* c, const xc_feed_setup* fs, void* vis,
                               const double* angles, void* stream_) {
  if (!c) return XC_E_INVAL;
  if (!fs) return fail(c, XC_E_INVAL, "feed setup is NULL");
  if (!vis || !angles) return fail(c, XC_E_INVAL, "feed correction: vis or angles is NULL");
  if (fs->n_subints < 1 || fs->n_subbands < 1 || fs->n_stations < 1 || fs->n_chan < 1 ||
      fs->n_stations > XC_MAX_STATIONS)
    return fail(c, XC_E_INVAL, "feed correction: empty or oversized setup");
  if (fs->feed != XC_FEED_CIRCULAR && fs->feed != XC_FEED_LINEAR)
    return fail(c, XC_E_INVAL, "feed=%d is neither circular nor linear", fs->feed);
  hipError_t e = hipSetDevice(c->device);
  if (e != hipSuccess) return hip_fail(c, e, "hipSetDevice");
  const long npairs = (long)fs->n_stations * (fs->n_stations + 1) / 2;
  // two channels a lane where every row starts 16-byte aligned
  const bool vec = fs->n_chan % 2 == 0 && reinterpret_cast<uintptr_t>(vis) % 16 == 0;
  const int V = vec ? 2 : 1;
  const long units = ((long)fs->n_chan + V * kFeedUnroll - 1) / (V * kFeedUnroll);
  const int threads = (int)std::min<long>(256, (units + 63) / 64 * 64);
  const long chunks = ((long)fs->n_chan + (long)threads * V * kFeedUnroll - 1) /
                      ((long)threads * V * kFeedUnroll);
  const long blocks = (long)fs->n_subints * fs->n_subbands * npairs * chunks;
  if (blocks > 0x7fffffffL) return fail(c, XC_E_INVAL, "feed correction: too many products");
  hipStream_t stream = (hipStream_t)stream_;
  float2* v = static_cast<float2*>(vis);
  e = timed(c, XC_K_FEED, stream, [&] {
    if (fs->feed == XC_FEED_CIRCULAR)
      launch_feed<XC_FEED_CIRCULAR>(v, angles, fs->n_subbands, fs->n_stations, fs->n_chan, vec,
                                    (unsigned)blocks, threads, (int)chunks, stream);
    else
      launch_feed<XC_FEED_LINEAR>(v, angles, fs->n_subbands, fs->n_stations, fs->n_chan, vec,
                                  (unsigned)blocks, threads, (int)chunks, stream);
    return hipGetLastError();
  });
  return e == hipSuccess ? XC_OK : hip_fail(c, e, "feed correction");
}
