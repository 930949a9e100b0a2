// Feed-angle (parallactic-angle-equivalent) correction of dual-polarisation
// products (section 2's capability list; angles are inputs).  One thread per
// (sub-integration, subband, station pair a <= b, channel) rewrites the pair's
// products in place.
#include <math.h>

#include "xc_launch.h"
#include "xc_runtime.h"

namespace xc {

__device__ inline int pair_bl(int i, int j, int M) { return i * M - (i * (i - 1)) / 2 + (j - i); }

__device__ inline float2 cmulf(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

__global__ void k_feed(float2* __restrict__ vis, const double* __restrict__ angles, int n_sub,
                       int n_sb, int S, int n_chan, int feed) {
  const int M = 2 * S, nbl = M * (M + 1) / 2, npairs = S * (S + 1) / 2;
  const long gid = (long)blockIdx.x * blockDim.x + threadIdx.x;
  const long total = (long)n_sub * n_sb * npairs * n_chan;
  if (gid >= total) return;
  const int k = (int)(gid % n_chan);
  long rest = gid / n_chan;
  const int pr = (int)(rest % npairs);
  rest /= npairs;
  const int sb = (int)(rest % n_sb);
  const int t = (int)(rest / n_sb);
  // station pair pr -> (a, b), a <= b, row-major over the upper triangle
  int a = 0, rem = pr;
  while (rem >= S - a) {
    rem -= S - a;
    ++a;
  }
  const int b = a + rem;
  const double ca = angles[(size_t)t * S + a], cb = angles[(size_t)t * S + b];
  float2* base = vis + ((size_t)t * n_sb + sb) * nbl * (size_t)n_chan + k;
  auto at = [&](int p, int q) -> float2* {
    return base + (size_t)pair_bl(2 * a + p, 2 * b + q, M) * n_chan;
  };
  if (feed == XC_FEED_CIRCULAR) {
    const double s[2] = {1.0, -1.0};
    for (int p = 0; p < 2; ++p)
      for (int q = 0; q < 2; ++q) {
        if (a == b && p > q) continue;            // not stored (Hermitian partner)
        const double ang = s[p] * ca - s[q] * cb;
        const float2 w = make_float2((float)cos(ang), (float)sin(ang));
        float2* v = at(p, q);
        *v = cmulf(*v, w);
      }
    return;
  }
  // linear: V <- Rot(ca)^T V Rot(cb), Rot = [[c, s], [-s, c]]
  const float c1 = (float)cos(ca), s1 = (float)sin(ca), c2 = (float)cos(cb), s2 = (float)sin(cb);
  float2 v00 = *at(0, 0), v01 = *at(0, 1), v11 = *at(1, 1);
  float2 v10 = a == b ? make_float2(v01.x, -v01.y) : *at(1, 0);
  // Rot(ca)^T = [[c1, -s1], [s1, c1]]; first U = Rot(ca)^T V
  const float2 u00 = make_float2(c1 * v00.x - s1 * v10.x, c1 * v00.y - s1 * v10.y);
  const float2 u01 = make_float2(c1 * v01.x - s1 * v11.x, c1 * v01.y - s1 * v11.y);
  const float2 u10 = make_float2(s1 * v00.x + c1 * v10.x, s1 * v00.y + c1 * v10.y);
  const float2 u11 = make_float2(s1 * v01.x + c1 * v11.x, s1 * v01.y + c1 * v11.y);
  // then U Rot(cb) with Rot(cb) = [[c2, s2], [-s2, c2]]
  *at(0, 0) = make_float2(c2 * u00.x - s2 * u01.x, c2 * u00.y - s2 * u01.y);
  *at(0, 1) = make_float2(s2 * u00.x + c2 * u01.x, s2 * u00.y + c2 * u01.y);
  *at(1, 1) = make_float2(s2 * u10.x + c2 * u11.x, s2 * u10.y + c2 * u11.y);
  if (a != b) *at(1, 0) = make_float2(c2 * u10.x - s2 * u11.x, c2 * u10.y - s2 * u11.y);
}

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
  const long total = (long)fs->n_subints * fs->n_subbands * npairs * fs->n_chan;
  const int bs = 256;
  const long blocks = (total + bs - 1) / bs;
  if (blocks > 0x7fffffffL) return fail(c, XC_E_INVAL, "feed correction: too many products");
  hipStream_t stream = (hipStream_t)stream_;
  e = timed(c, XC_K_FEED, stream, [&] {
    hipLaunchKernelGGL(k_feed, dim3((unsigned)blocks), dim3(bs), 0, stream,
                       static_cast<float2*>(vis), angles, fs->n_subints, fs->n_subbands,
                       fs->n_stations, fs->n_chan, fs->feed);
    return hipGetLastError();
  });
  return e == hipSuccess ? XC_OK : hip_fail(c, e, "feed correction");
}
