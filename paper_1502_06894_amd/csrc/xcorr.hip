// C-ABI runtime: context, setup validation, workspace layout, descriptor
// upload and launch sequencing of the correlation path.
#include <math.h>

#include <atomic>
#include <mutex>

#include "xc_runtime.h"

namespace xc {

// ---------------------------------------------------------------- allocation-free scratch
// Workspace of xc_correlate_subint_noalloc: a fixed array in the library's
// device code object, one copy per GPU, held until the process ends.  In host
// code `scratch` names a host-side stand-in, not device memory, so it is never
// handed to a kernel or a copy: xc_create looks up each device's address once
// (with that device current) and every use goes through that address.
constexpr size_t kScratchBytes = (size_t)256 << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];
constexpr int kScratchDevices = 64;
static std::atomic<unsigned char*> g_scratch_addr[kScratchDevices];
static std::mutex g_scratch_mu;

// The current device's address of `scratch` (caller has made `dev` current).
static hipError_t scratch_lookup(int dev) {
  if (dev < 0 || dev >= kScratchDevices) return hipErrorInvalidDevice;
  if (g_scratch_addr[dev].load()) return hipSuccess;
  std::lock_guard<std::mutex> g(g_scratch_mu);
  if (g_scratch_addr[dev].load()) return hipSuccess;
  void* p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e == hipSuccess && p) g_scratch_addr[dev].store(static_cast<unsigned char*>(p));
  return e != hipSuccess ? e : p ? hipSuccess : hipErrorInvalidSymbol;
}

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

namespace {

bool pow2(int64_t x) { return x > 0 && (x & (x - 1)) == 0; }

int ilog2(int x) {
  int l = 0;
  while ((1 << l) < x) ++l;
  return l;
}

}  // namespace

ShapeKey shape_key(const xc_setup* s) {
  return ShapeKey(2 * s->n_chan, s->n_stations * s->n_pols, s->n_subbands,
                  s->n_streams_recorded, s->precision);
}

xc_tuning effective_tuning(const xc_ctx* c, const xc_setup* s) {
  xc_tuning t = {0, 0, 0, 0, 0, 0};
  if (!c) return t;
  auto it = c->tuned.find(shape_key(s));
  if (it != c->tuned.end()) t = it->second;
  const xc_tuning& o = c->tune;
  if (o.fstage_waves_per_simd) t.fstage_waves_per_simd = o.fstage_waves_per_simd;
  if (o.xmac_frames_per_stage) t.xmac_frames_per_stage = o.xmac_frames_per_stage;
  if (o.xmac_channels_per_wg) t.xmac_channels_per_wg = o.xmac_channels_per_wg;
  if (o.frames_per_block) t.frames_per_block = o.frames_per_block;
  if (o.xmac_tiles_per_wg) t.xmac_tiles_per_wg = o.xmac_tiles_per_wg;
  if (o.block_overlap) t.block_overlap = o.block_overlap;
  return t;
}

static int block_frames(const xc_setup* s, const xc_tuning& tu) {
  int64_t T = s->frames_per_block > 0 ? s->frames_per_block : tu.frames_per_block;
  if (T <= 0) {
    const int eb = s->precision == XC_FP16_MFMA ? 4 : s->precision == XC_FP8_MFMA ? 2 : 8;
    const size_t per_frame =
        (size_t)s->n_subbands * s->n_stations * s->n_pols * s->n_chan * eb;
    const size_t fit = per_frame > 0 ? kDefaultBlockBytes / per_frame : kDefaultBlockFrames;
    T = fit > (size_t)kMaxBlockFrames ? kMaxBlockFrames
        : fit > (size_t)kDefaultBlockFrames ? (int64_t)fit
                                            : kDefaultBlockFrames;
  }
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
    if (x.rate_correct != 0 && x.rate_correct != 1)
      return fail(c, XC_E_INVAL, "station %d: rate_correct=%d", i, x.rate_correct);
    if (x.rate_correct && (s->precision != XC_FP32 || N > kMaxRateCorrectN))
      return fail(c, XC_E_INVAL,
                  "station %d: the drift correction needs the FP32 path and n_chan <= %d", i,
                  kMaxRateCorrectN / 2);
  }
  return XC_OK;
}

bool any_rate_correct(const xc_setup* s, const xc_station* st) {
  for (int i = 0; i < s->n_stations; ++i)
    if (st[i].rate_correct) return true;
  return false;
}

Layout layout_of(const xc_setup* s, const xc_station* st, const xc_tuning& tu, bool overlap) {
  Layout L;
  const int S = s->n_stations, nsb = s->n_subbands, M = S * s->n_pols;
  const size_t nbl = (size_t)M * (M + 1) / 2;
  L.T = block_frames(s, tu);
  L.desc_bytes = sizeof(DevJob) + (size_t)S * sizeof(DevStation) +
                 (size_t)S * nsb * (kMaxPolyDeg + 1) * sizeof(double);
  size_t off = 0;
  L.mask = off;
  L.mask_off.assign(S, SIZE_MAX);
  for (int i = 0; i < S; ++i)
    if (!st[i].frame_ok) {
      L.mask_off[i] = off - L.mask;
      off += align_up((size_t)st[i].n_frames_m5b);
    }
  L.nbuf = overlap && tu.block_overlap == 2 && s->n_frames > L.T ? 2 : 1;
  // each delay-record buffer ends with the F stage's task counter
  L.ctr_off = align_up((size_t)S * L.T * sizeof(DelayRec));
  L.drec_bytes = L.ctr_off + kAlign;
  L.drec = off;
  off += L.nbuf * L.drec_bytes;
  L.prec_bytes = align_up((size_t)S * nsb * L.T * sizeof(PhaseRec));
  L.prec = off;
  off += L.nbuf * L.prec_bytes;
  L.out = s->precision == XC_FP16_MFMA ? kOutF16 : s->precision == XC_FP8_MFMA ? kOutF8 : kOutF32;
  L.spec = off;
  size_t spec_bytes = (size_t)nsb * L.T * M * s->n_chan * out_elem_bytes(L.out);
  if (L.out != kOutF32) {
    L.n_scale = L.T < kScaleFrames ? L.T : kScaleFrames;
    const size_t pre = (size_t)nsb * L.n_scale * M * s->n_chan * sizeof(float2);
    if (pre > spec_bytes) spec_bytes = pre;
  }
  L.spec_bytes = align_up(spec_bytes);
  off += L.nbuf * L.spec_bytes;
  L.sexp = off;
  if (L.out != kOutF32) off += align_up((size_t)nsb * M * s->n_chan);
  L.scratch = off;
  off += align_up(fstage_scratch_bytes(2 * s->n_chan, S, nsb * s->n_pols, L.T, L.out));
  L.fps = xmac_frames_per_split(L.T, M, s->n_chan, nsb);
  L.n_slots = L.out == kOutF32 ? (L.T + L.fps - 1) / L.fps : 1;
  L.slot_stride = (size_t)nsb * nbl * s->n_chan;
  L.vacc = off;
  off += (size_t)L.n_slots * L.slot_stride * sizeof(double2);   // wacc follows directly
  L.wacc = off;
  off += align_up((size_t)S * S * sizeof(double));
  L.total = off;
  return L;
}

int shared_block_frames(const xc_setup& s, const Layout& L, size_t cap_bytes, int min_frames) {
  const size_t per_frame =
      (size_t)s.n_subbands * s.n_stations * s.n_pols * s.n_chan * out_elem_bytes(L.out);
  if ((size_t)L.T * per_frame <= cap_bytes) return L.T;
  int64_t T = (int64_t)(cap_bytes / per_frame);
  const int64_t amortize = (int64_t)kSlotAmortize * (s.n_stations * s.n_pols + 1);
  const int64_t floor_T = amortize < L.T ? amortize : L.T;
  if (T < floor_T) T = floor_T;
  if (T < min_frames) T = min_frames;
  if (T > L.T) T = L.T;
  return (int)T;
}

// Build the job descriptor for device address `dev` into host memory `h`.
void build_desc(const xc_setup* s, const xc_station* st, const Layout& L,
                const unsigned char* dev_desc, const unsigned char* arena, unsigned char* h) {
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
  const unsigned char* dev = dev_desc;
  DevStation* hs = reinterpret_cast<DevStation*>(h + sizeof(DevJob));
  double* hp = reinterpret_cast<double*>(h + sizeof(DevJob) + (size_t)S * sizeof(DevStation));
  J->st = reinterpret_cast<const DevStation*>(dev + sizeof(DevJob));
  const double* dp =
      reinterpret_cast<const double*>(dev + sizeof(DevJob) + (size_t)S * sizeof(DevStation));
  for (int i = 0; i < S; ++i) {
    DevStation& d = hs[i];
    d.words = static_cast<const uint32_t*>(st[i].frames);
    d.frame_ok = st[i].frame_ok ? st[i].frame_ok
                                : reinterpret_cast<const uint8_t*>(arena + L.mask + L.mask_off[i]);
    d.n_frames_m5b = st[i].n_frames_m5b;
    d.first_sample = st[i].first_sample;
    d.poly_deg = st[i].poly_deg;
    for (int k = 0; k <= st[i].poly_deg; ++k) d.delay_poly[k] = st[i].delay_poly[k];
    d.has_phase = st[i].phase_poly ? 1 : 0;
    d.rate_correct = st[i].rate_correct ? 1 : 0;
    d.phase_poly = st[i].phase_poly ? dp + (size_t)i * nsb * (kMaxPolyDeg + 1) : nullptr;
    if (st[i].phase_poly)
      for (int b = 0; b < nsb; ++b)
        for (int k = 0; k <= st[i].poly_deg; ++k)
          hp[((size_t)i * nsb + b) * (kMaxPolyDeg + 1) + k] =
              st[i].phase_poly[b * (st[i].poly_deg + 1) + k];
  }
}

int upload_desc(xc_ctx* c, const xc_setup* s, const xc_station* st, const Layout& L,
                unsigned char* dev_desc, const unsigned char* arena, hipStream_t stream) {
  if (L.desc_bytes > kSlotBytes) return fail(c, XC_E_INVAL, "descriptor too large");
  const int k = c->next_slot;
  c->next_slot = (k + 1) % kSlots;
  hipError_t e = hipEventSynchronize(c->ev[k]);
  if (e != hipSuccess) return hip_fail(c, e, "hipEventSynchronize");
  unsigned char* h = c->h_stage + (size_t)k * kSlotBytes;
  build_desc(s, st, L, dev_desc, arena, h);
  e = hipMemcpyAsync(dev_desc, h, L.desc_bytes, hipMemcpyHostToDevice, stream);
  if (e != hipSuccess) return hip_fail(c, e, "descriptor upload");
  e = hipEventRecord(c->ev[k], stream);
  if (e != hipSuccess) return hip_fail(c, e, "hipEventRecord");
  return XC_OK;
}

int enqueue_job(xc_ctx* c, const xc_setup* s, const xc_station* st, const xc_output* out,
                const DevJob* dj, unsigned char* arena, const Layout& L, const xc_tuning& tu,
                hipStream_t stream, hipStream_t xs) {
  DelayRec* drec = reinterpret_cast<DelayRec*>(arena + L.drec);
  PhaseRec* prec = reinterpret_cast<PhaseRec*>(arena + L.prec);
  void* spec = arena + L.spec;
  const bool overlap = L.nbuf == 2 && xs != nullptr;
  const bool rate_pass = any_rate_correct(s, st);
  double2* vacc = reinterpret_cast<double2*>(arena + L.vacc);
  double* wacc = reinterpret_cast<double*>(arena + L.wacc);
  int8_t* sexp = reinterpret_cast<int8_t*>(arena + L.sexp);
  const int S = s->n_stations, nsb = s->n_subbands, M = S * s->n_pols;
  const int N = 2 * s->n_chan;
  hipError_t e = hipSuccess;
  for (int i = 0; i < S && e == hipSuccess; ++i)
    if (!st[i].frame_ok)
      e = timed(c, XC_K_INGEST, stream, [&] {
        return launch_ingest(static_cast<const uint32_t*>(st[i].frames), st[i].n_frames_m5b,
                             reinterpret_cast<uint8_t*>(arena + L.mask + L.mask_off[i]), stream);
      });
  if (e != hipSuccess) return hip_fail(c, e, "ingest");
  e = timed(c, XC_K_ZERO, stream, [&] {
    return launch_zero(reinterpret_cast<double*>(vacc), (L.total - L.vacc) / sizeof(double),
                       stream);
  });
  if (e != hipSuccess) return hip_fail(c, e, "zero");
  if (L.out != kOutF32) {
    // channel scales from the first frames' FP32 spectra
    unsigned* ctr0 = reinterpret_cast<unsigned*>(arena + L.drec + L.ctr_off);
    e = launch_delays(dj, S, nsb, 0, L.n_scale, drec, prec, ctr0, stream);
    if (e == hipSuccess)
      e = timed(c, XC_K_FSTAGE, stream, [&] {
        return launch_fstage(N, dj, S, nsb * s->n_pols, drec, prec, c->d_tw, spec, nullptr,
                             L.n_scale, 0, kOutF32, ctr0,
                             reinterpret_cast<float2*>(arena + L.scratch), stream);
      });
    if (e == hipSuccess)
      e = launch_scales(static_cast<const float2*>(spec), drec, nsb, L.n_scale, M, s->n_pols,
                        s->n_chan, L.out == kOutF16 ? kF16TargetLog2 : kF8TargetLog2, sexp,
                        stream);
    if (e != hipSuccess) return hip_fail(c, e, "scales");
  }
  // Blocks of L.T frames.  Overlapped: block b uses buffer p = b mod 2; its F
  // stage (on `stream`) waits until the X stage of block b - 2 (on `xs`) has
  // read that buffer, and its X stage waits for its F stage.
  int64_t blk = 0;
  for (int64_t f0 = 0; f0 < s->n_frames; f0 += L.T, ++blk) {
    const int nf = (int)((s->n_frames - f0) < L.T ? (s->n_frames - f0) : L.T);
    const int p = overlap ? (int)(blk & 1) : 0;
    DelayRec* drec_p = reinterpret_cast<DelayRec*>(arena + L.drec + p * L.drec_bytes);
    PhaseRec* prec_p = reinterpret_cast<PhaseRec*>(arena + L.prec + p * L.prec_bytes);
    void* spec_p = arena + L.spec + p * L.spec_bytes;
    unsigned* ctr_p = reinterpret_cast<unsigned*>(arena + L.drec + p * L.drec_bytes + L.ctr_off);
    hipStream_t xstr = overlap ? xs : stream;
    if (overlap && blk >= 2) {
      e = hipStreamWaitEvent(stream, c->blk_x[p], 0);
      if (e != hipSuccess) return hip_fail(c, e, "block wait");
    }
    e = timed(c, XC_K_DELAYS, stream, [&] {
      hipError_t r = launch_delays(dj, S, nsb, f0, nf, drec_p, prec_p, ctr_p, stream);
      return r == hipSuccess ? launch_weights(drec_p, S, nf, wacc, stream) : r;
    });
    if (e != hipSuccess) return hip_fail(c, e, "delays");
    e = timed(c, XC_K_FSTAGE, stream, [&] {
      return launch_fstage(N, dj, S, nsb * s->n_pols, drec_p, prec_p, c->d_tw, spec_p, sexp, nf,
                           fstage_variant(tu.fstage_waves_per_simd, s->n_pols, s->n_chan, L.out),
                           L.out, ctr_p,
                           reinterpret_cast<float2*>(arena + L.scratch), stream);
    });
    if (e != hipSuccess) return hip_fail(c, e, "fstage");
    if (rate_pass) {
      e = timed(c, XC_K_FSTAGE, stream, [&] {
        return launch_fstage(N, dj, S, nsb * s->n_pols, drec_p, prec_p, c->d_tw, spec_p, sexp,
                             nf, kFstageRatePass, L.out, ctr_p + 1,
                             reinterpret_cast<float2*>(arena + L.scratch), stream);
      });
      if (e != hipSuccess) return hip_fail(c, e, "fstage drift correction");
    }
    if (overlap) {
      e = hipEventRecord(c->blk_f[p], stream);
      if (e == hipSuccess) e = hipStreamWaitEvent(xs, c->blk_f[p], 0);
      if (e != hipSuccess) return hip_fail(c, e, "block handoff");
    }
    if (L.out == kOutF32) {
      e = timed(c, XC_K_XMAC, xstr, [&] {
        return launch_xmac(dj, M, s->n_chan, nsb, static_cast<const float2*>(spec_p), vacc,
                           L.slot_stride, nf, L.fps, tu.xmac_frames_per_stage,
                           tu.xmac_channels_per_wg, tu.xmac_tiles_per_wg, xstr);
      });
    } else {
      e = timed(c, XC_K_XMFMA, xstr, [&] {
        return launch_xmfma(dj, L.out, M, s->n_chan, nsb, spec_p, sexp, vacc, L.slot_stride, nf,
                            xstr);
      });
    }
    if (e != hipSuccess) return hip_fail(c, e, "xmac");
    if (overlap) {
      e = hipEventRecord(c->blk_x[p], xs);
      if (e != hipSuccess) return hip_fail(c, e, "block record");
    }
  }
  if (overlap) {
    // X stages run in order on xs: the last one done means all are
    e = hipStreamWaitEvent(stream, c->blk_x[(blk - 1) & 1], 0);
    if (e != hipSuccess) return hip_fail(c, e, "block join");
  }
  e = timed(c, XC_K_FINALISE, stream, [&] {
    return launch_finalise(vacc, L.n_slots, L.slot_stride, wacc, S, s->n_pols,
                           static_cast<float2*>(out->vis), out->weight, nsb, M, s->n_chan,
                           stream);
  });
  if (e != hipSuccess) return hip_fail(c, e, "finalise");
  return XC_OK;
}

int ensure_xstream(xc_ctx* c) {
  if (c->xstream) return XC_OK;
  hipError_t e = hipStreamCreateWithFlags(&c->xstream, hipStreamNonBlocking);   // default priority
  for (int k = 0; k < 2 && e == hipSuccess; ++k) {
    e = hipEventCreateWithFlags(&c->blk_f[k], hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&c->blk_x[k], hipEventDisableTiming);
  }
  return e == hipSuccess ? XC_OK : hip_fail(c, e, "X-stage stream");
}

int ensure_lanes(xc_ctx* c, int n) {
  hipError_t e = hipSuccess;
  while (e == hipSuccess && (int)c->lanes.size() < n) {
    hipStream_t st;
    hipEvent_t ev;
    e = hipStreamCreateWithFlags(&st, hipStreamNonBlocking);   // default priority
    if (e == hipSuccess) e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
    if (e == hipSuccess) {
      c->lanes.push_back(st);
      c->lane_ev.push_back(ev);
    }
  }
  if (e == hipSuccess && !c->fork_ev) e = hipEventCreateWithFlags(&c->fork_ev, hipEventDisableTiming);
  return e == hipSuccess ? XC_OK : hip_fail(c, e, "lanes");
}

namespace {

// Single-job workspace: [descriptor][arena].
struct Prepared {
  Layout L;
  xc_tuning tu;
  unsigned char* desc;
  unsigned char* arena;
};

int prepare(xc_ctx* c, const xc_setup* s, const xc_station* st, void* workspace,
            size_t ws_bytes, hipStream_t stream, Prepared& p) {
  if (!c) return XC_E_INVAL;
  int rc = validate(c, s, st);
  if (rc != XC_OK) return rc;
  p.tu = effective_tuning(c, s);
  p.L = layout_of(s, st, p.tu, true);
  const size_t need = align_up(p.L.desc_bytes) + p.L.total;
  if (!workspace || ws_bytes < need)
    return fail(c, XC_E_NOMEM, "workspace %zu bytes < %zu needed", ws_bytes, need);
  hipError_t e = hipSetDevice(c->device);
  if (e != hipSuccess) return hip_fail(c, e, "hipSetDevice");
  p.desc = static_cast<unsigned char*>(workspace);
  p.arena = p.desc + align_up(p.L.desc_bytes);
  return upload_desc(c, s, st, p.L, p.desc, p.arena, stream);
}

// Ingest masks of stations without a caller-supplied frame_ok (taps only; the
// correlation path does this inside enqueue_job).
int ingest_missing(xc_ctx* c, const xc_setup* s, const xc_station* st, const Prepared& p,
                   hipStream_t stream) {
  for (int i = 0; i < s->n_stations; ++i)
    if (!st[i].frame_ok) {
      hipError_t e =
          launch_ingest(static_cast<const uint32_t*>(st[i].frames), st[i].n_frames_m5b,
                        reinterpret_cast<uint8_t*>(p.arena + p.L.mask + p.L.mask_off[i]), stream);
      if (e != hipSuccess) return hip_fail(c, e, "ingest");
    }
  return XC_OK;
}

}  // namespace
}  // namespace xc

using namespace xc;

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
  if (e == hipSuccess) c->scratch_rc = (int)scratch_lookup(hip_device);
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
  (void)hipSetDevice(c->device);
  for (Timed& t : c->prof) {
    (void)hipEventSynchronize(t.b);
    (void)hipEventDestroy(t.a);
    (void)hipEventDestroy(t.b);
  }
  for (int k = 0; k < kSlots; ++k)
    if (c->ev[k]) {
      (void)hipEventSynchronize(c->ev[k]);
      (void)hipEventDestroy(c->ev[k]);
    }
  for (auto& g : c->graphs) hipGraphExecDestroy(g.exec);
  for (size_t i = 0; i < c->lanes.size(); ++i) {
    (void)hipStreamSynchronize(c->lanes[i]);
    (void)hipStreamDestroy(c->lanes[i]);
    (void)hipEventDestroy(c->lane_ev[i]);
  }
  if (c->fork_ev) (void)hipEventDestroy(c->fork_ev);
  if (c->xstream) {
    (void)hipStreamSynchronize(c->xstream);
    (void)hipStreamDestroy(c->xstream);
  }
  for (int k = 0; k < 2; ++k) {
    if (c->blk_f[k]) (void)hipEventDestroy(c->blk_f[k]);
    if (c->blk_x[k]) (void)hipEventDestroy(c->blk_x[k]);
  }
  if (c->batch_ev) {
    (void)hipEventSynchronize(c->batch_ev);
    (void)hipEventDestroy(c->batch_ev);
  }
  if (c->h_batch) (void)hipHostFree(c->h_batch);
  if (c->h_stage) (void)hipHostFree(c->h_stage);
  if (c->d_tw) (void)hipFree(c->d_tw);
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
  const Layout L = layout_of(s, st, effective_tuning(c, s), true);
  return align_up(L.desc_bytes) + L.total;
}

int xc_correlate_subint(xc_ctx* c, const xc_setup* s, const xc_station* st, const xc_output* out,
                        void* workspace, size_t ws_bytes, void* stream_) {
  hipStream_t stream = (hipStream_t)stream_;
  if (c && (!out || !out->vis || !out->weight)) return fail(c, XC_E_INVAL, "output is NULL");
  Prepared p;
  int rc = prepare(c, s, st, workspace, ws_bytes, stream, p);
  if (rc != XC_OK) return rc;
  if (p.L.nbuf == 2) {
    rc = ensure_xstream(c);
    if (rc != XC_OK) return rc;
  }
  return enqueue_job(c, s, st, out, reinterpret_cast<const DevJob*>(p.desc), p.arena, p.L, p.tu,
                     stream, p.L.nbuf == 2 ? c->xstream : nullptr);
}

int xc_correlate_subint_noalloc(xc_ctx* c, const xc_setup* s, const xc_station* st,
                                const xc_output* out, void* stream_) {
  hipStream_t stream = (hipStream_t)stream_;
  if (!c) return XC_E_INVAL;
  if (!out || !out->vis || !out->weight) return fail(c, XC_E_INVAL, "output is NULL");
  int rc = validate(c, s, st);
  if (rc != XC_OK) return rc;
  unsigned char* base =
      c->device >= 0 && c->device < kScratchDevices ? g_scratch_addr[c->device].load() : nullptr;
  if (!base)
    return fail(c, XC_E_HIP, "allocation-free scratch unavailable on device %d: %s", c->device,
                hipGetErrorString((hipError_t)c->scratch_rc));
  xc_tuning tu = effective_tuning(c, s);
  tu.block_overlap = 1;   // one block buffer: no second stream, no second arena
  xc_setup q = *s;
  auto need = [&](const Layout& L) { return align_up(L.desc_bytes) + L.total; };
  Layout L = layout_of(&q, st, tu);
  if (need(L) > kScratchBytes) {
    if (s->frames_per_block > 0 || tu.frames_per_block > 0)
      return fail(c, XC_E_NOMEM,
                  "allocation-free call: %zu bytes needed at %d frames per block, the scratch "
                  "holds %zu",
                  need(L), L.T, kScratchBytes);
    // the largest block that fits: halve, then search between T and 2 T
    int hi = L.T, lo = 0;
    for (int T = L.T / 2; T >= 1; T /= 2) {
      q.frames_per_block = T;
      if (need(layout_of(&q, st, tu)) <= kScratchBytes) {
        lo = T;
        break;
      }
      hi = T;
    }
    if (lo == 0)
      return fail(c, XC_E_NOMEM,
                  "allocation-free call: even one frame per block needs more than the %zu-byte "
                  "scratch",
                  kScratchBytes);
    while (hi - lo > 1) {
      const int mid = lo + (hi - lo) / 2;
      q.frames_per_block = mid;
      if (need(layout_of(&q, st, tu)) <= kScratchBytes)
        lo = mid;
      else
        hi = mid;
    }
    q.frames_per_block = lo;
    L = layout_of(&q, st, tu);
  }
  hipError_t e = hipSetDevice(c->device);
  if (e != hipSuccess) return hip_fail(c, e, "hipSetDevice");
  unsigned char* desc = base;
  unsigned char* arena = base + align_up(L.desc_bytes);
  rc = upload_desc(c, &q, st, L, desc, arena, stream);
  if (rc != XC_OK) return rc;
  return enqueue_job(c, &q, st, out, reinterpret_cast<const DevJob*>(desc), arena, L, tu, stream);
}

size_t xc_noalloc_scratch_bytes(void) { return kScratchBytes; }

int xc_set_tuning(xc_ctx* c, const xc_tuning* t) {
  if (!c || !t) return XC_E_INVAL;
  const bool ok = t->fstage_waves_per_simd >= 0 &&
                  (t->fstage_waves_per_simd <= 5 || t->fstage_waves_per_simd == kFstageShare ||
                   t->fstage_waves_per_simd == kFstageLean) &&
                  (t->xmac_frames_per_stage == 0 || t->xmac_frames_per_stage == 1 ||
                   t->xmac_frames_per_stage == 2 || t->xmac_frames_per_stage == kXmacMatrix ||
                   t->xmac_frames_per_stage == 4 || t->xmac_frames_per_stage == kXmacMatrixRing || t->xmac_frames_per_stage == 8) &&
                  (t->xmac_channels_per_wg == 0 || t->xmac_channels_per_wg == 16 ||
                   t->xmac_channels_per_wg == 32 || t->xmac_channels_per_wg == 64) &&
                  t->frames_per_block >= 0 && t->frames_per_block <= kMaxBlockFrames &&
                  t->xmac_tiles_per_wg >= 0 && t->xmac_tiles_per_wg <= 64 &&
                  t->block_overlap >= 0 && t->block_overlap <= 2;
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
  Prepared p;
  int rc = prepare(c, s, st, workspace, ws_bytes, stream, p);
  if (rc == XC_OK) rc = ingest_missing(c, s, st, p, stream);
  if (rc != XC_OK) return rc;
  const Layout& L = p.L;
  const DevJob* dj = reinterpret_cast<const DevJob*>(p.desc);
  DelayRec* drec = reinterpret_cast<DelayRec*>(p.arena + L.drec);
  PhaseRec* prec = reinterpret_cast<PhaseRec*>(p.arena + L.prec);
  const int S = s->n_stations, nsb = s->n_subbands;
  const int64_t F = s->n_frames;
  std::vector<DelayRec> hd((size_t)S * L.T);
  std::vector<PhaseRec> hp((size_t)S * nsb * L.T);
  for (int64_t f0 = 0; f0 < F; f0 += L.T) {
    const int nf = (int)((F - f0) < L.T ? (F - f0) : L.T);
    hipError_t e = launch_delays(dj, S, nsb, f0, nf, drec, prec, nullptr, stream);
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
  Prepared p;
  int rc = prepare(c, s, st, workspace, ws_bytes, stream, p);
  if (rc == XC_OK) rc = ingest_missing(c, s, st, p, stream);
  if (rc != XC_OK) return rc;
  if (station < 0 || station >= s->n_stations || input < 0 ||
      input >= s->n_subbands * s->n_pols || frame < 0 || frame >= s->n_frames || !out)
    return fail(c, XC_E_INVAL, "debug_unpack: index out of range");
  const DevJob* dj = reinterpret_cast<const DevJob*>(p.desc);
  DelayRec* drec = reinterpret_cast<DelayRec*>(p.arena + p.L.drec);
  PhaseRec* prec = reinterpret_cast<PhaseRec*>(p.arena + p.L.prec);
  float* tmp = reinterpret_cast<float*>(p.arena + p.L.spec);
  const int N = 2 * s->n_chan;
  hipError_t e =
      launch_delays(dj, s->n_stations, s->n_subbands, frame, 1, drec, prec, nullptr, stream);
  if (e == hipSuccess) e = launch_debug_unpack(dj, drec, 1, station, input, 0, tmp, N, stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(out, tmp, sizeof(float) * N, hipMemcpyDeviceToHost, stream);
  if (e == hipSuccess) e = hipStreamSynchronize(stream);
  return e == hipSuccess ? XC_OK : hip_fail(c, e, "debug_unpack");
}

int xc_debug_spectra(xc_ctx* c, const xc_setup* s, const xc_station* st, int64_t frame0,
                     int32_t n, void* spectra, void* workspace, size_t ws_bytes, void* stream_) {
  hipStream_t stream = (hipStream_t)stream_;
  Prepared p;
  int rc = prepare(c, s, st, workspace, ws_bytes, stream, p);
  if (rc == XC_OK) rc = ingest_missing(c, s, st, p, stream);
  if (rc != XC_OK) return rc;
  if (n < 1 || n > p.L.T || frame0 < 0 || frame0 + n > s->n_frames || !spectra)
    return fail(c, XC_E_INVAL, "debug_spectra: frame range");
  const DevJob* dj = reinterpret_cast<const DevJob*>(p.desc);
  DelayRec* drec = reinterpret_cast<DelayRec*>(p.arena + p.L.drec);
  PhaseRec* prec = reinterpret_cast<PhaseRec*>(p.arena + p.L.prec);
  unsigned* ctr = reinterpret_cast<unsigned*>(p.arena + p.L.drec + p.L.ctr_off);
  hipError_t e = launch_delays(dj, s->n_stations, s->n_subbands, frame0, n, drec, prec, ctr, stream);
  if (e == hipSuccess)
    e = launch_fstage(2 * s->n_chan, dj, s->n_stations, s->n_subbands * s->n_pols, drec, prec,
                      c->d_tw, spectra, nullptr, n,
                      fstage_variant(p.tu.fstage_waves_per_simd, s->n_pols, s->n_chan, kOutF32),
                      kOutF32, ctr,
                      reinterpret_cast<float2*>(p.arena + p.L.scratch), stream);
  if (e == hipSuccess && any_rate_correct(s, st))
    e = launch_fstage(2 * s->n_chan, dj, s->n_stations, s->n_subbands * s->n_pols, drec, prec,
                      c->d_tw, spectra, nullptr, n, kFstageRatePass, kOutF32, ctr + 1,
                      reinterpret_cast<float2*>(p.arena + p.L.scratch), stream);
  return e == hipSuccess ? XC_OK : hip_fail(c, e, "debug_spectra");
}

}  // extern "C"
