// C-ABI runtime: context, setup validation, workspace layout, descriptor
// upload and launch sequencing of the correlation path.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <string>
#include <vector>

#include "../../include/xcorr.h"
#include "xc_launch.h"

using namespace xc;

namespace {

constexpr int kSlots = 8;
constexpr size_t kSlotBytes = 256 * 1024;
constexpr size_t kAlign = 256;

size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

}  // namespace

struct Timed {
  int kind;
  hipEvent_t a, b;
};

struct xc_ctx {
  int device = 0;
  xc_tuning tune = {0, 0, 0, 0, 0};
  bool profiling = false;
  std::vector<Timed> prof;        // event pairs, reused across profile sessions
  size_t prof_used = 0;
  float2* d_tw = nullptr;                 // kTwiddleN entries
  unsigned char* h_stage = nullptr;       // kSlots x kSlotBytes pinned
  hipEvent_t ev[kSlots] = {};
  int next_slot = 0;
  std::string last_error;
};

namespace {

int fail(xc_ctx* c, int code, const char* fmt, ...) __attribute__((format(printf, 3, 4)));
int fail(xc_ctx* c, int code, const char* fmt, ...) {
  if (c) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    c->last_error = buf;
  }
  return code;
}

int hip_fail(xc_ctx* c, hipError_t e, const char* what) {
  return fail(c, XC_E_HIP, "%s: %s", what, hipGetErrorString(e));
}

bool pow2(int64_t x) { return x > 0 && (x & (x - 1)) == 0; }

int ilog2(int x) {
  int l = 0;
  while ((1 << l) < x) ++l;
  return l;
}

// Run a launcher, bracketed by an event pair when profiling is on.
template <class Fn>
hipError_t timed(xc_ctx* c, int kind, hipStream_t s, Fn&& fn) {
  if (!c->profiling || c->prof_used >= c->prof.size()) return fn();
  Timed& t = c->prof[c->prof_used++];
  t.kind = kind;
  hipError_t e = hipEventRecord(t.a, s);
  if (e != hipSuccess) return e;
  e = fn();
  if (e != hipSuccess) return e;
  return hipEventRecord(t.b, s);
}

// Workspace layout of one job.
struct Layout {
  size_t desc = 0, mask = 0, drec = 0, prec = 0, spec = 0, vacc = 0, wacc = 0, total = 0;
  size_t sexp = 0;                // int8 scale exponents [n_sb][M][n_chan] (MFMA path)
  int out = kOutF32;              // spectrum element type written by the F stage
  int n_scale = 0;                // frames of the scale pre-pass (MFMA path)
  size_t desc_bytes = 0;
  int n_slots = 1;                // FP64 accumulator slots of the X stage
  size_t slot_stride = 0;         // double2 elements per slot
  std::vector<size_t> mask_off;   // per station, SIZE_MAX if caller supplies frame_ok
  int T = 0;                      // frames per block
};

constexpr int kMaxBlockFrames = 2048;
constexpr int kScaleFrames = 64;          // frames that set the MFMA path's channel scales
constexpr int kF16TargetLog2 = 10;        // FP16: scaled RMS 2^10 (max 65504)
constexpr int kF8TargetLog2 = 5;          // e4m3: scaled RMS 2^5 (max 448)
constexpr int kDefaultBlockFrames = 2048;

int block_frames(const xc_setup* s, const xc_ctx* c) {
  int64_t T = s->frames_per_block > 0 ? s->frames_per_block
              : (c && c->tune.frames_per_block > 0) ? c->tune.frames_per_block
                                                     : kDefaultBlockFrames;
  if (T > s->n_frames) T = s->n_frames;
  return (int)T;
}

int validate(xc_ctx* c, const xc_setup* s, const xc_station* st) {
  if (!s) return fail(c, XC_E_INVAL, "setup is NULL");
  if (s->n_stations < 1 || s->n_stations > XC_MAX_STATIONS)
    return fail(c, XC_E_INVAL, "n_stations=%d outside 1..%d", s->n_stations, XC_MAX_STATIONS);
  if (s->n_subbands < 1 || s->n_subbands > XC_MAX_SUBBANDS)
    return fail(c, XC_E_INVAL, "n_subbands=%d outside 1..%d", s->n_subbands, XC_MAX_SUBBANDS);
  if (s->n_pols != 1 && s->n_pols != 2) return fail(c, XC_E_INVAL, "n_pols=%d", s->n_pols);
  if (s->n_subbands * s->n_pols > XC_MAX_INPUTS)
    return fail(c, XC_E_INVAL, "n_subbands*n_pols=%d > %d", s->n_subbands * s->n_pols,
                XC_MAX_INPUTS);
  if (!pow2(s->n_chan) || s->n_chan < XC_MIN_CHAN || s->n_chan > XC_MAX_CHAN)
    return fail(c, XC_E_INVAL, "n_chan=%d: power of two in %d..%d required", s->n_chan,
                XC_MIN_CHAN, XC_MAX_CHAN);
  if (!fstage_supported(2 * s->n_chan))
    return fail(c, XC_E_INVAL, "n_chan=%d not supported by this build", s->n_chan);
  const int C = s->n_streams_recorded;
  if (C != 1 && C != 2 && C != 4 && C != 8 && C != 16)
    return fail(c, XC_E_INVAL, "n_streams_recorded=%d not in {1,2,4,8,16}", C);
  if (!s->stream_map || !s->lo_hz) return fail(c, XC_E_INVAL, "stream_map/lo_hz is NULL");
  for (int i = 0; i < s->n_subbands * s->n_pols; ++i)
    if (s->stream_map[i] < 0 || s->stream_map[i] >= C)
      return fail(c, XC_E_INVAL, "stream_map[%d]=%d outside 0..%d", i, s->stream_map[i], C - 1);
  if (!(s->fs_hz > 0.0) || !isfinite(s->fs_hz)) return fail(c, XC_E_INVAL, "fs_hz invalid");
  if (s->n_frames < 1) return fail(c, XC_E_INVAL, "n_frames=%lld", (long long)s->n_frames);
  if (s->precision != XC_FP32 && s->precision != XC_FP16_MFMA && s->precision != XC_FP8_MFMA)
    return fail(c, XC_E_INVAL, "precision %d unknown", s->precision);
  if (s->precision != XC_FP32 && s->n_stations * s->n_pols > 32)
    return fail(c, XC_E_INVAL, "MFMA X stage takes at most 32 inputs per subband (M=%d)",
                s->n_stations * s->n_pols);
  if (s->frames_per_block < 0 || s->frames_per_block > kMaxBlockFrames)
    return fail(c, XC_E_INVAL, "frames_per_block=%d outside 0..%d", s->frames_per_block,
                kMaxBlockFrames);
  if (!st) return fail(c, XC_E_INVAL, "stations is NULL");
  const int N = 2 * s->n_chan;
  const double t0 = (double)s->sub_start / s->fs_hz;
  const double t1 = (double)(s->sub_start + s->n_frames * (int64_t)N) / s->fs_hz;
  for (int i = 0; i < s->n_stations; ++i) {
    const xc_station& x = st[i];
    if (!x.frames || x.n_frames_m5b < 1)
      return fail(c, XC_E_INVAL, "station %d: no recording", i);
    if (x.poly_deg < 0 || x.poly_deg > XC_MAX_POLY_DEG || !x.delay_poly)
      return fail(c, XC_E_INVAL, "station %d: poly_deg=%d", i, x.poly_deg);
    if (!(x.poly_t0 < x.poly_t1) || t0 < x.poly_t0 || t1 > x.poly_t1)
      return fail(c, XC_E_RANGE, "station %d: sub-int [%.6f, %.6f] s outside span [%.6f, %.6f]",
                  i, t0, t1, x.poly_t0, x.poly_t1);
    for (int k = 0; k <= x.poly_deg; ++k)
      if (!isfinite(x.delay_poly[k]))
        return fail(c, XC_E_INVAL, "station %d: delay_poly[%d] not finite", i, k);
  }
  return XC_OK;
}

Layout layout_of(const xc_setup* s, const xc_station* st, const xc_ctx* c) {
  Layout L;
  const int S = s->n_stations, nsb = s->n_subbands, M = S * s->n_pols;
  const size_t nbl = (size_t)M * (M + 1) / 2;
  L.T = block_frames(s, c);
  L.desc_bytes = sizeof(DevJob) + (size_t)S * sizeof(DevStation) +
                 (size_t)S * nsb * (kMaxPolyDeg + 1) * sizeof(double);
  size_t off = 0;
  L.desc = off;
  off += align_up(L.desc_bytes);
  L.mask = off;
  L.mask_off.assign(S, SIZE_MAX);
  for (int i = 0; i < S; ++i)
    if (!st[i].frame_ok) {
      L.mask_off[i] = off - L.mask;
      off += align_up((size_t)st[i].n_frames_m5b);
    }
  L.drec = off;
  off += align_up((size_t)S * L.T * sizeof(DelayRec));
  L.prec = off;
  off += align_up((size_t)S * nsb * L.T * sizeof(PhaseRec));
  L.out = s->precision == XC_FP16_MFMA ? kOutF16 : s->precision == XC_FP8_MFMA ? kOutF8 : kOutF32;
  L.spec = off;
  size_t spec_bytes = (size_t)nsb * L.T * M * s->n_chan * out_elem_bytes(L.out);
  if (L.out != kOutF32) {
    L.n_scale = L.T < kScaleFrames ? L.T : kScaleFrames;
    const size_t pre = (size_t)nsb * L.n_scale * M * s->n_chan * sizeof(float2);
    if (pre > spec_bytes) spec_bytes = pre;
  }
  off += align_up(spec_bytes);
  L.sexp = off;
  if (L.out != kOutF32) off += align_up((size_t)nsb * M * s->n_chan);
  L.n_slots = xmac_splits(L.T);
  L.slot_stride = (size_t)nsb * nbl * s->n_chan;
  L.vacc = off;
  off += (size_t)L.n_slots * L.slot_stride * sizeof(double2);   // wacc follows directly
  L.wacc = off;
  off += align_up((size_t)S * S * sizeof(double));
  L.total = off;
  return L;
}

// Build the job descriptor for device address `dev` into host memory `h`.
void build_desc(const xc_setup* s, const xc_station* st, const Layout& L, unsigned char* ws,
                unsigned char* h) {
  const int S = s->n_stations, nsb = s->n_subbands;
  DevJob* J = reinterpret_cast<DevJob*>(h);
  memset(h, 0, L.desc_bytes);
  J->n_stations = S;
  J->n_subbands = nsb;
  J->n_pols = s->n_pols;
  J->n_chan = s->n_chan;
  J->N = 2 * s->n_chan;
  J->C = s->n_streams_recorded;
  J->M = S * s->n_pols;
  J->n_inputs = nsb * s->n_pols;
  J->nbl = J->M * (J->M + 1) / 2;
  J->spf = kPayloadWords * 16 / J->C;
  J->spw_log2 = ilog2(16 / J->C);
  J->spf_magic = (uint32_t)((((uint64_t)1 << 32) + (uint64_t)J->spf - 1) / (uint64_t)J->spf);
  J->fs = s->fs_hz;
  J->sub_start = s->sub_start;
  J->n_frames = s->n_frames;
  for (int i = 0; i < J->n_inputs; ++i) J->stream_map[i] = s->stream_map[i];
  for (int b = 0; b < nsb; ++b) J->lo_hz[b] = s->lo_hz[b];
  unsigned char* dev = ws + L.desc;
  DevStation* hs = reinterpret_cast<DevStation*>(h + sizeof(DevJob));
  double* hp = reinterpret_cast<double*>(h + sizeof(DevJob) + (size_t)S * sizeof(DevStation));
  J->st = reinterpret_cast<const DevStation*>(dev + sizeof(DevJob));
  const double* dp =
      reinterpret_cast<const double*>(dev + sizeof(DevJob) + (size_t)S * sizeof(DevStation));
  for (int i = 0; i < S; ++i) {
    DevStation& d = hs[i];
    d.words = static_cast<const uint32_t*>(st[i].frames);
    d.frame_ok = st[i].frame_ok ? st[i].frame_ok
                                : reinterpret_cast<const uint8_t*>(ws + L.mask + L.mask_off[i]);
    d.n_frames_m5b = st[i].n_frames_m5b;
    d.first_sample = st[i].first_sample;
    d.poly_deg = st[i].poly_deg;
    for (int k = 0; k <= st[i].poly_deg; ++k) d.delay_poly[k] = st[i].delay_poly[k];
    d.has_phase = st[i].phase_poly ? 1 : 0;
    d.phase_poly = st[i].phase_poly ? dp + (size_t)i * nsb * (kMaxPolyDeg + 1) : nullptr;
    if (st[i].phase_poly)
      for (int b = 0; b < nsb; ++b)
        for (int k = 0; k <= st[i].poly_deg; ++k)
          hp[((size_t)i * nsb + b) * (kMaxPolyDeg + 1) + k] =
              st[i].phase_poly[b * (st[i].poly_deg + 1) + k];
  }
}

// Stage the descriptor through a pinned slot and copy it into the workspace.
int upload_desc(xc_ctx* c, const xc_setup* s, const xc_station* st, const Layout& L,
                unsigned char* ws, hipStream_t stream) {
  if (L.desc_bytes > kSlotBytes) return fail(c, XC_E_INVAL, "descriptor too large");
  const int k = c->next_slot;
  c->next_slot = (k + 1) % kSlots;
  hipError_t e = hipEventSynchronize(c->ev[k]);
  if (e != hipSuccess) return hip_fail(c, e, "hipEventSynchronize");
  unsigned char* h = c->h_stage + (size_t)k * kSlotBytes;
  build_desc(s, st, L, ws, h);
  e = hipMemcpyAsync(ws + L.desc, h, L.desc_bytes, hipMemcpyHostToDevice, stream);
  if (e != hipSuccess) return hip_fail(c, e, "descriptor upload");
  e = hipEventRecord(c->ev[k], stream);
  if (e != hipSuccess) return hip_fail(c, e, "hipEventRecord");
  return XC_OK;
}

// Common prologue: validate, lay out, check workspace, upload, ingest.
int prepare(xc_ctx* c, const xc_setup* s, const xc_station* st, void* workspace,
            size_t ws_bytes, hipStream_t stream, Layout& L) {
  if (!c) return XC_E_INVAL;
  int rc = validate(c, s, st);
  if (rc != XC_OK) return rc;
  L = layout_of(s, st, c);
  if (!workspace || ws_bytes < L.total)
    return fail(c, XC_E_NOMEM, "workspace %zu bytes < %zu needed", ws_bytes, L.total);
  hipError_t e = hipSetDevice(c->device);
  if (e != hipSuccess) return hip_fail(c, e, "hipSetDevice");
  unsigned char* ws = static_cast<unsigned char*>(workspace);
  rc = upload_desc(c, s, st, L, ws, stream);
  if (rc != XC_OK) return rc;
  for (int i = 0; i < s->n_stations; ++i)
    if (!st[i].frame_ok) {
      e = timed(c, XC_K_INGEST, stream, [&] {
        return launch_ingest(static_cast<const uint32_t*>(st[i].frames), st[i].n_frames_m5b,
                             reinterpret_cast<uint8_t*>(ws + L.mask + L.mask_off[i]), stream);
      });
      if (e != hipSuccess) return hip_fail(c, e, "ingest");
    }
  return XC_OK;
}

}  // namespace

extern "C" {

const char* xc_strerror(int code) {
  switch (code) {
    case XC_OK: return "ok";
    case XC_E_INVAL: return "invalid argument";
    case XC_E_RANGE: return "sub-integration outside the polynomial span";
    case XC_E_NOMEM: return "insufficient workspace or memory budget";
    case XC_E_HIP: return "HIP runtime error";
    case XC_E_CANCELLED: return "cancelled";
    case XC_E_TIMEOUT: return "timed out";
    default: return "unknown error";
  }
}

const char* xc_last_error(const xc_ctx* c) { return c ? c->last_error.c_str() : ""; }

int xc_create(xc_ctx** out, int hip_device) {
  if (!out) return XC_E_INVAL;
  *out = nullptr;
  int n = 0;
  if (hipGetDeviceCount(&n) != hipSuccess || hip_device < 0 || hip_device >= n) return XC_E_HIP;
  xc_ctx* c = new xc_ctx();
  c->device = hip_device;
  hipError_t e = hipSetDevice(hip_device);
  if (e == hipSuccess) e = hipMalloc(&c->d_tw, sizeof(float2) * kTwiddleN);
  std::vector<float2> tw(kTwiddleN);
  for (int m = 0; m < kTwiddleN; ++m) {
    const double a = 2.0 * M_PI * (double)m / (double)kTwiddleN;
    tw[m] = make_float2((float)cos(a), (float)-sin(a));
  }
  if (e == hipSuccess)
    e = hipMemcpy(c->d_tw, tw.data(), sizeof(float2) * kTwiddleN, hipMemcpyHostToDevice);
  if (e == hipSuccess)
    e = hipHostMalloc((void**)&c->h_stage, (size_t)kSlots * kSlotBytes, hipHostMallocDefault);
  for (int k = 0; k < kSlots && e == hipSuccess; ++k)
    e = hipEventCreateWithFlags(&c->ev[k], hipEventDisableTiming);
  if (e != hipSuccess) {
    xc_destroy(c);
    return XC_E_HIP;
  }
  *out = c;
  return XC_OK;
}

void xc_destroy(xc_ctx* c) {
  if (!c) return;
  hipSetDevice(c->device);
  for (Timed& t : c->prof) {
    hipEventSynchronize(t.b);
    hipEventDestroy(t.a);
    hipEventDestroy(t.b);
  }
  for (int k = 0; k < kSlots; ++k)
    if (c->ev[k]) {
      hipEventSynchronize(c->ev[k]);
      hipEventDestroy(c->ev[k]);
    }
  if (c->h_stage) hipHostFree(c->h_stage);
  if (c->d_tw) hipFree(c->d_tw);
  delete c;
}

int xc_ingest(xc_ctx* c, const void* frames, int64_t n_frames_m5b, uint8_t* frame_ok,
              void* stream) {
  if (!c) return XC_E_INVAL;
  if (!frames || !frame_ok || n_frames_m5b < 0)
    return fail(c, XC_E_INVAL, "ingest: bad arguments");
  hipError_t e = hipSetDevice(c->device);
  if (e == hipSuccess)
    e = launch_ingest(static_cast<const uint32_t*>(frames), n_frames_m5b, frame_ok,
                      (hipStream_t)stream);
  return e == hipSuccess ? XC_OK : hip_fail(c, e, "ingest");
}

int xc_validate(xc_ctx* c, const xc_setup* s, const xc_station* st) {
  return validate(c, s, st);
}

size_t xc_workspace_bytes(const xc_ctx* c, const xc_setup* s, const xc_station* st) {
  if (validate(const_cast<xc_ctx*>(c), s, st) != XC_OK) return 0;
  return layout_of(s, st, c).total;
}

int xc_correlate_subint(xc_ctx* c, const xc_setup* s, const xc_station* st, const xc_output* out,
                        void* workspace, size_t ws_bytes, void* stream_) {
  hipStream_t stream = (hipStream_t)stream_;
  Layout L;
  int rc = prepare(c, s, st, workspace, ws_bytes, stream, L);
  if (rc != XC_OK) return rc;
  if (!out || !out->vis || !out->weight) return fail(c, XC_E_INVAL, "output is NULL");
  unsigned char* ws = static_cast<unsigned char*>(workspace);
  const DevJob* dj = reinterpret_cast<const DevJob*>(ws + L.desc);
  DelayRec* drec = reinterpret_cast<DelayRec*>(ws + L.drec);
  PhaseRec* prec = reinterpret_cast<PhaseRec*>(ws + L.prec);
  float2* spec = reinterpret_cast<float2*>(ws + L.spec);
  double2* vacc = reinterpret_cast<double2*>(ws + L.vacc);
  double* wacc = reinterpret_cast<double*>(ws + L.wacc);
  const int S = s->n_stations, nsb = s->n_subbands, M = S * s->n_pols;
  const int N = 2 * s->n_chan;
  hipError_t e = timed(c, XC_K_ZERO, stream, [&] {
    return launch_zero(reinterpret_cast<double*>(vacc), (L.total - L.vacc) / sizeof(double),
                       stream);
  });
  if (e != hipSuccess) return hip_fail(c, e, "zero");
  int8_t* sexp = reinterpret_cast<int8_t*>(ws + L.sexp);
  if (L.out != kOutF32) {
    // channel scales from the first frames' FP32 spectra
    e = launch_delays(dj, S, nsb, 0, L.n_scale, drec, prec, stream);
    if (e == hipSuccess)
      e = timed(c, XC_K_FSTAGE, stream, [&] {
        return launch_fstage(N, dj, S, drec, prec, c->d_tw, spec, nullptr, L.n_scale, 0, kOutF32,
                             stream);
      });
    if (e == hipSuccess)
      e = launch_scales(spec, nsb, L.n_scale, M, s->n_chan,
                        L.out == kOutF16 ? kF16TargetLog2 : kF8TargetLog2, sexp, stream);
    if (e != hipSuccess) return hip_fail(c, e, "scales");
  }
  for (int64_t f0 = 0; f0 < s->n_frames; f0 += L.T) {
    const int nf = (int)((s->n_frames - f0) < L.T ? (s->n_frames - f0) : L.T);
    e = timed(c, XC_K_DELAYS, stream, [&] {
      hipError_t r = launch_delays(dj, S, nsb, f0, nf, drec, prec, stream);
      return r == hipSuccess ? launch_weights(drec, S, nf, wacc, stream) : r;
    });
    if (e != hipSuccess) return hip_fail(c, e, "delays");
    e = timed(c, XC_K_FSTAGE, stream, [&] {
      return launch_fstage(N, dj, S, drec, prec, c->d_tw, spec, sexp, nf,
                           c->tune.fstage_waves_per_simd, L.out, stream);
    });
    if (e != hipSuccess) return hip_fail(c, e, "fstage");
    if (L.out == kOutF32) {
      e = timed(c, XC_K_XMAC, stream, [&] {
        return launch_xmac(dj, M, s->n_chan, nsb, spec, vacc, L.slot_stride, nf,
                           c->tune.xmac_frames_per_stage, c->tune.xmac_channels_per_wg,
                           c->tune.xmac_tiles_per_wg, stream);
      });
    } else {
      e = timed(c, XC_K_XMFMA, stream, [&] {
        return launch_xmfma(dj, L.out, M, s->n_chan, nsb, spec, sexp, vacc, L.slot_stride, nf,
                            stream);
      });
    }
    if (e != hipSuccess) return hip_fail(c, e, "xmac");
  }
  e = timed(c, XC_K_FINALISE, stream, [&] {
    return launch_finalise(vacc, L.n_slots, L.slot_stride, wacc, S, s->n_pols,
                           static_cast<float2*>(out->vis), out->weight, nsb, M, s->n_chan,
                           stream);
  });
  if (e != hipSuccess) return hip_fail(c, e, "finalise");
  return XC_OK;
}

int xc_set_tuning(xc_ctx* c, const xc_tuning* t) {
  if (!c || !t) return XC_E_INVAL;
  const bool ok = t->fstage_waves_per_simd >= 0 && t->fstage_waves_per_simd <= 4 &&
                  (t->xmac_frames_per_stage >= 0 && t->xmac_frames_per_stage <= 4 &&
                   t->xmac_frames_per_stage != 3) &&
                  (t->xmac_channels_per_wg == 0 || t->xmac_channels_per_wg == 16 ||
                   t->xmac_channels_per_wg == 32 || t->xmac_channels_per_wg == 64) &&
                  t->frames_per_block >= 0 && t->frames_per_block <= kMaxBlockFrames &&
                  t->xmac_tiles_per_wg >= 0 && t->xmac_tiles_per_wg <= 64;
  if (!ok) return fail(c, XC_E_INVAL, "tuning value out of range");
  c->tune = *t;
  return XC_OK;
}

int xc_get_tuning(const xc_ctx* c, xc_tuning* t) {
  if (!c || !t) return XC_E_INVAL;
  *t = c->tune;
  return XC_OK;
}

int xc_profile_begin(xc_ctx* c, int32_t max_launches) {
  if (!c || max_launches < 1) return XC_E_INVAL;
  hipError_t e = hipSetDevice(c->device);
  while (e == hipSuccess && c->prof.size() < (size_t)max_launches) {
    Timed t{0, nullptr, nullptr};
    e = hipEventCreate(&t.a);
    if (e == hipSuccess) e = hipEventCreate(&t.b);
    if (e == hipSuccess) c->prof.push_back(t);
  }
  if (e != hipSuccess) return hip_fail(c, e, "profile_begin");
  c->prof_used = 0;
  c->profiling = true;
  return XC_OK;
}

int xc_profile_end(xc_ctx* c, double* ms_by_kind, int64_t* launches_by_kind) {
  if (!c) return XC_E_INVAL;
  c->profiling = false;
  for (int k = 0; k < XC_NKINDS; ++k) {
    if (ms_by_kind) ms_by_kind[k] = 0.0;
    if (launches_by_kind) launches_by_kind[k] = 0;
  }
  for (size_t i = 0; i < c->prof_used; ++i) {
    Timed& t = c->prof[i];
    hipError_t e = hipEventSynchronize(t.b);
    float ms = 0.f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, t.a, t.b);
    if (e != hipSuccess) return hip_fail(c, e, "profile_end");
    if (ms_by_kind) ms_by_kind[t.kind] += ms;
    if (launches_by_kind) launches_by_kind[t.kind] += 1;
  }
  c->prof_used = 0;
  return XC_OK;
}

int xc_debug_delays(xc_ctx* c, const xc_setup* s, const xc_station* st, int64_t* n_int,
                    double* d_frac, int32_t* valid, double* phi0, void* workspace,
                    size_t ws_bytes, void* stream_) {
  hipStream_t stream = (hipStream_t)stream_;
  Layout L;
  int rc = prepare(c, s, st, workspace, ws_bytes, stream, L);
  if (rc != XC_OK) return rc;
  unsigned char* ws = static_cast<unsigned char*>(workspace);
  const DevJob* dj = reinterpret_cast<const DevJob*>(ws + L.desc);
  DelayRec* drec = reinterpret_cast<DelayRec*>(ws + L.drec);
  PhaseRec* prec = reinterpret_cast<PhaseRec*>(ws + L.prec);
  const int S = s->n_stations, nsb = s->n_subbands;
  const int64_t F = s->n_frames;
  std::vector<DelayRec> hd((size_t)S * L.T);
  std::vector<PhaseRec> hp((size_t)S * nsb * L.T);
  for (int64_t f0 = 0; f0 < F; f0 += L.T) {
    const int nf = (int)((F - f0) < L.T ? (F - f0) : L.T);
    hipError_t e = launch_delays(dj, S, nsb, f0, nf, drec, prec, stream);
    if (e == hipSuccess)
      e = hipMemcpyAsync(hd.data(), drec, sizeof(DelayRec) * S * nf, hipMemcpyDeviceToHost,
                         stream);
    if (e == hipSuccess)
      e = hipMemcpyAsync(hp.data(), prec, sizeof(PhaseRec) * S * nsb * nf,
                         hipMemcpyDeviceToHost, stream);
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    if (e != hipSuccess) return hip_fail(c, e, "debug_delays");
    for (int i = 0; i < S; ++i)
      for (int fl = 0; fl < nf; ++fl) {
        const DelayRec& r = hd[(size_t)i * nf + fl];
        const size_t o = (size_t)i * F + f0 + fl;
        if (n_int) n_int[o] = r.n_int;
        if (d_frac) d_frac[o] = r.d;
        if (valid) valid[o] = r.valid;
        if (phi0)
          for (int b = 0; b < nsb; ++b)
            phi0[((size_t)i * nsb + b) * F + f0 + fl] = hp[((size_t)i * nsb + b) * nf + fl].phi0;
      }
  }
  return XC_OK;
}

int xc_debug_unpack(xc_ctx* c, const xc_setup* s, const xc_station* st, int32_t station,
                    int32_t input, int64_t frame, float* out, void* workspace, size_t ws_bytes,
                    void* stream_) {
  hipStream_t stream = (hipStream_t)stream_;
  Layout L;
  int rc = prepare(c, s, st, workspace, ws_bytes, stream, L);
  if (rc != XC_OK) return rc;
  if (station < 0 || station >= s->n_stations || input < 0 ||
      input >= s->n_subbands * s->n_pols || frame < 0 || frame >= s->n_frames || !out)
    return fail(c, XC_E_INVAL, "debug_unpack: index out of range");
  unsigned char* ws = static_cast<unsigned char*>(workspace);
  const DevJob* dj = reinterpret_cast<const DevJob*>(ws + L.desc);
  DelayRec* drec = reinterpret_cast<DelayRec*>(ws + L.drec);
  PhaseRec* prec = reinterpret_cast<PhaseRec*>(ws + L.prec);
  float* tmp = reinterpret_cast<float*>(ws + L.spec);
  const int N = 2 * s->n_chan;
  hipError_t e = launch_delays(dj, s->n_stations, s->n_subbands, frame, 1, drec, prec, stream);
  if (e == hipSuccess) e = launch_debug_unpack(dj, drec, 1, station, input, 0, tmp, N, stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(out, tmp, sizeof(float) * N, hipMemcpyDeviceToHost, stream);
  if (e == hipSuccess) e = hipStreamSynchronize(stream);
  return e == hipSuccess ? XC_OK : hip_fail(c, e, "debug_unpack");
}

int xc_debug_spectra(xc_ctx* c, const xc_setup* s, const xc_station* st, int64_t frame0,
                     int32_t n, void* spectra, void* workspace, size_t ws_bytes, void* stream_) {
  hipStream_t stream = (hipStream_t)stream_;
  Layout L;
  int rc = prepare(c, s, st, workspace, ws_bytes, stream, L);
  if (rc != XC_OK) return rc;
  if (n < 1 || n > L.T || frame0 < 0 || frame0 + n > s->n_frames || !spectra)
    return fail(c, XC_E_INVAL, "debug_spectra: frame range");
  unsigned char* ws = static_cast<unsigned char*>(workspace);
  const DevJob* dj = reinterpret_cast<const DevJob*>(ws + L.desc);
  DelayRec* drec = reinterpret_cast<DelayRec*>(ws + L.drec);
  PhaseRec* prec = reinterpret_cast<PhaseRec*>(ws + L.prec);
  hipError_t e = launch_delays(dj, s->n_stations, s->n_subbands, frame0, n, drec, prec, stream);
  if (e == hipSuccess)
    e = launch_fstage(2 * s->n_chan, dj, s->n_stations, drec, prec, c->d_tw, spectra, nullptr, n,
                      c->tune.fstage_waves_per_simd, kOutF32, stream);
  return e == hipSuccess ? XC_OK : hip_fail(c, e, "debug_spectra");
}

}  // extern "C"
