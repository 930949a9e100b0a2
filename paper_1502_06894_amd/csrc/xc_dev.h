// Device-side job descriptors, delay/phase model and 2-bit sample addressing.
// Shared by every kernel of the library (never by the CPU oracle).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace xc {

constexpr int kMaxPolyDeg = 7;
constexpr int kMaxStations = 64;
constexpr int kMaxSubbands = 16;
constexpr int kMaxInputs = 32;
constexpr int kFrameWords = 2504;     // 16-byte header + 2500 payload words
constexpr int kHeaderWords = 4;
constexpr int kPayloadWords = 2500;
constexpr uint32_t kSync = 0xABADDEEDu;
constexpr int kTwiddleN = 32768;      // twiddle table length: exp(-2 pi i m / 32768)

struct DevStation {
  const uint32_t* words;      // recording, kFrameWords per frame
  const uint8_t* frame_ok;    // per recording frame: 1 = good sync
  int64_t n_frames_m5b;
  int64_t first_sample;
  int32_t poly_deg;
  int32_t has_phase;          // phase polynomials present for every subband
  int32_t rate_correct;       // correct the delay's drift inside each frame
  double delay_poly[kMaxPolyDeg + 1];
  const double* phase_poly;   // [n_subbands][kMaxPolyDeg + 1] or nullptr
};

struct DevJob {
  int32_t n_stations, n_subbands, n_pols, n_chan;
  int32_t N, C, M, n_inputs;  // n_inputs = n_subbands * n_pols (per station)
  int32_t nbl;                // M (M + 1) / 2
  int32_t spf;                // per-stream samples per recording frame = 40000 / C
  int32_t spw_log2;           // log2(16 / C): per-stream samples per word
  uint32_t spf_magic;         // ceil(2^32 / spf): exact quotient for numerators < 2^17
  double fs;
  int64_t sub_start, n_frames;
  int32_t stream_map[kMaxInputs];
  double lo_hz[kMaxSubbands];
  const DevStation* st;       // [n_stations]
};

// Per (station, block frame): integer delay, fractional delay, window start in
// the recording, validity.
struct DelayRec {
  int64_t n_int;
  double d;
  int64_t base;
  int32_t valid;
  float rate;     // delay rate tau' at the frame centre (s/s): the drift correction's rho
};

// Per (station, subband, block frame): fringe phase Taylor terms about the
// frame centre, in turns: phi(n) = phi0 + phi1 (n - N/2) + phi2 (n - N/2)^2.
struct PhaseRec {
  double phi0, phi1, phi2;
};

// ---------------------------------------------------------------- delay model
// Integer/fractional delay at the frame centre.  Evaluated with one rounding
// per IEEE operation (no contraction) so that it matches a plain FP64
// reference bit for bit: t_mid = (j0 + f N + N/2) / fs, tau by Horner,
// D = tau fs, n_int = floor(D + 1/2), d = D - n_int.
__device__ inline void frame_delay(const DevStation& s, const DevJob& j, int64_t f,
                                   int64_t* n_int, double* d) {
#pragma clang fp contract(off)
  const int64_t num = j.sub_start + f * (int64_t)j.N + (int64_t)(j.N / 2);
  const double t = (double)num / j.fs;
  double r = s.delay_poly[s.poly_deg];
  for (int k = s.poly_deg - 1; k >= 0; --k) {
    r = r * t;
    r = r + s.delay_poly[k];
  }
  const double D = r * j.fs;
  const double fl = floor(D + 0.5);
  *n_int = (int64_t)fl;
  *d = D - fl;
}

// Error-free transformations (Knuth two-sum, FMA two-product).
__device__ inline void two_sum(double a, double b, double& s, double& e) {
#pragma clang fp contract(off)
  s = a + b;
  const double z = s - a;
  e = (a - (s - z)) + (b - z);
}
__device__ inline void two_prod(double a, double b, double& p, double& e) {
#pragma clang fp contract(off)
  p = a * b;
  e = fma(a, b, -p);
}

// Compensated Horner (Graillat, Langlois & Louvet 2005): value of sum c_k t^k
// as hi + lo with about twice FP64's precision.
__device__ inline void comp_horner(const double* c, int deg, double t, double& hi, double& lo) {
#pragma clang fp contract(off)
  double s = c[deg], r = 0.0;
  for (int k = deg - 1; k >= 0; --k) {
    double p, pe, s2, se;
    two_prod(s, t, p, pe);
    two_sum(p, c[k], s2, se);
    r = r * t + (pe + se);
    s = s2;
  }
  hi = s;
  lo = r;
}

// First and second derivative of sum c_k t^k.
__device__ inline void poly_derivs(const double* c, int deg, double t, double& d1, double& d2) {
  double a = 0.0, b = 0.0;
  for (int k = deg; k >= 1; --k) a = a * t + (double)k * c[k];
  for (int k = deg; k >= 2; --k) b = b * t + (double)(k * (k - 1)) * c[k];
  d1 = a;
  d2 = b;
}

// Fractional part in [0, 1) of hi + lo (|lo| << 1).
__device__ inline double frac_dd(double hi, double lo) {
  const double f = (hi - floor(hi)) + lo;   // hi - floor(hi) is exact
  return f - floor(f);
}

// Fringe phase Taylor terms for station s, subband sb, about reference time t
// (the frame centre).  phi(t) = nu_sb tau(t) unless an explicit phase
// polynomial is given.  The frame-centre value is reduced to [0, 1) in
// double-double arithmetic so that a ~1e9-turn phase keeps ~1e-15 turns.
__device__ inline PhaseRec frame_phase(const DevStation& s, const DevJob& j, int sb, double t) {
  PhaseRec r;
  double hi, lo, d1, d2;
  if (s.has_phase) {
    const double* c = s.phase_poly + sb * (kMaxPolyDeg + 1);
    comp_horner(c, s.poly_deg, t, hi, lo);
    poly_derivs(c, s.poly_deg, t, d1, d2);
    r.phi0 = frac_dd(hi, lo);
  } else {
    const double nu = j.lo_hz[sb];
    comp_horner(s.delay_poly, s.poly_deg, t, hi, lo);
    poly_derivs(s.delay_poly, s.poly_deg, t, d1, d2);
    double p, pe;
    two_prod(nu, hi, p, pe);
    r.phi0 = frac_dd(p, pe + nu * lo);
    d1 *= nu;
    d2 *= nu;
  }
  r.phi1 = d1 / j.fs;
  r.phi2 = d2 / (2.0 * j.fs * j.fs);
  return r;
}

// ---------------------------------------------------------------- sample addressing
// Position of per-stream sample `base + n` of a recording: the payload word
// holding it and the bit offset of stream 0's field (stream c adds 2c).
struct FrameCursor {
  int64_t fm0;   // recording frame of the window start
  int32_t ip0;   // sample offset of the window start inside that frame
};

__device__ inline FrameCursor make_cursor(const DevJob& j, int64_t base) {
  FrameCursor c;
  c.fm0 = base / j.spf;
  c.ip0 = (int32_t)(base - c.fm0 * j.spf);
  return c;
}

// Payload word holding per-stream sample base + n (window start in cursor c).
__device__ inline const uint32_t* sample_word(const DevJob& j, const uint32_t* words,
                                              const FrameCursor& c, int n) {
  const uint32_t ip = (uint32_t)(c.ip0 + n);               // < spf + N <= 72768
  const uint32_t q = __umulhi(ip, j.spf_magic);            // ip / spf
  const uint32_t in = ip - q * (uint32_t)j.spf;
  return words + (c.fm0 + (int64_t)q) * kFrameWords + kHeaderWords + (in >> j.spw_log2);
}

// Bit offset of stream 0's field for sample base + n.  spf is a multiple of the
// samples per word, so the offset depends only on (ip0 + n) mod (16 / C).
__device__ inline int sample_shift(const DevJob& j, const FrameCursor& c, int n) {
  return (int)(2u * (((uint32_t)(c.ip0 + n)) & ((1u << j.spw_log2) - 1u)) * (uint32_t)j.C);
}

__device__ inline float level_of(uint32_t code) {
  // offset binary: 0 -> -3.3359, 1 -> -1, 2 -> +1, 3 -> +3.3359
  const float mag = (code == 0u || code == 3u) ? 3.3359f : 1.0f;
  return (code >= 2u) ? mag : -mag;
}

// exp(+2 pi i x) for x in turns, |x| <= 1: the hardware sine/cosine take
// their argument in revolutions.
__device__ inline float2 phasor_turns(float x) {
  return make_float2(__builtin_amdgcn_cosf(x), __builtin_amdgcn_sinf(x));
}

// x - floor(x) of a double, as float (in [0, 1]).
__device__ inline float frac_f(double x) { return (float)(x - floor(x)); }

// Complex product with its two fused multiply-adds written out, so that every
// kernel variant rounds it the same way (left to the compiler, the fusion
// depends on the surrounding code).
__device__ inline float2 cmul(float2 a, float2 b) {
  return make_float2(fmaf(a.x, b.x, -(a.y * b.y)), fmaf(a.x, b.y, a.y * b.x));
}

}  // namespace xc
