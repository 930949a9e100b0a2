/*
 * xcorr.h -- C ABI of the MI355X (gfx950) FX correlator for space VLBI.
 *
 * The correlator implements the FX architecture the paper describes for the
 * DiFX software correlator (abstract: Fourier transform first, then
 * cross-multiply), extended as in section 2 for a space antenna: each
 * station's delay comes from a per-scan polynomial that already contains the
 * space-specific terms (arbitrary moving position and velocity, relativistic
 * corrections, and the spacecraft-to-tracking-station transmission delay),
 * and the station data arrive in a Mark5B-style recording (section 2, format
 * conversion paragraph).  Per station and FFT frame the library
 *   1. evaluates the delay polynomial in FP64 at the frame centre, splitting
 *      the delay into an integer sample shift and a fractional part,
 *   2. unpacks the 2-bit samples of the shifted window,
 *   3. rotates each sample by the fringe phase exp(+2 pi i phi(t_n)),
 *   4. FFTs the frame to channels (kept: DC .. Nyquist-1),
 *   5. corrects the fractional delay per channel, Y[k] *= exp(+2 pi i k d / N),
 * and then cross-multiplies every pair of inputs i <= j of a subband and
 * accumulates V_ij[k] = mean over frames of Y_i[k] conj(Y_j[k]).
 *
 * Conventions shared by every entry point:
 *   - Pointers documented as "device" must point to memory of the context's
 *     HIP device; "host" pointers are read during the call only.
 *   - The caller owns every input, output and workspace buffer.  The library
 *     owns only the context (and servers); it allocates device memory only in
 *     xc_create and xc_server_create, never on the correlation path.
 *   - Calls that take a stream are asynchronous on that stream (a HIP stream
 *     handle cast to void*, NULL for the default stream) unless stated.
 *   - Return codes: XC_OK (0) or a negative XC_E_* value; xc_last_error()
 *     gives a message for the last failure on the context.  Frames whose
 *     window leaves the recording or touches a recording frame with a bad sync
 *     word are not errors: they get weight 0 (see xc_output.weight).
 *   - A context is used by one host thread at a time.
 */
#ifndef XCORR_H
#define XCORR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---------------------------------------------------------------- codes */
#define XC_OK           0
#define XC_E_INVAL     -1   /* bad shape, non-power-of-two channels, stream map out of range */
#define XC_E_RANGE     -2   /* sub-integration outside a polynomial's validity span */
#define XC_E_NOMEM     -3   /* workspace too small, or a server cannot admit the job */
#define XC_E_HIP       -4   /* a HIP runtime call failed */
#define XC_E_CANCELLED -5
#define XC_E_TIMEOUT   -6

#define XC_FP32        0    /* FP32 fringe rotation, FFT and cross-multiply */
#define XC_FP16_MFMA   1    /* X step on MFMA, FP16 inputs, FP32 accumulate */
#define XC_FP8_MFMA    2    /* X step on MFMA, FP8 (e4m3) inputs, FP32 accumulate */

#define XC_MAX_POLY_DEG   7
#define XC_MAX_STATIONS   64
#define XC_MAX_SUBBANDS   16
#define XC_MAX_INPUTS     32   /* n_subbands * n_pols per station */
#define XC_MIN_CHAN       128
#define XC_MAX_CHAN       16384

/* Recording format: frames of 10016 bytes = 16-byte header (uint32 words:
 * 0xABADDEED sync, frame-in-second | station id << 16, integer second, 0)
 * + 2500 little-endian uint32 payload words.  With C recorded streams each
 * payload word holds 16 two-bit fields; field j (bits 2j..2j+1) is stream
 * j mod C at per-stream sample word*(16/C) + j/C, counting payload words from
 * the start of the recording.  Codes 0..3 are the levels -3.3359, -1, +1,
 * +3.3359 (offset binary). */
#define XC_FRAME_BYTES    10016
#define XC_SYNC_WORD      0xABADDEEDu

/* ---------------------------------------------------------------- context */
typedef struct xc_ctx xc_ctx;

/* Create a context on HIP device `hip_device`; uploads the FFT twiddle table.
 * Returns XC_OK and sets *out, or XC_E_HIP / XC_E_INVAL. */
int  xc_create(xc_ctx** out, int hip_device);
void xc_destroy(xc_ctx* ctx);
/* Static message for a return code. */
const char* xc_strerror(int code);
/* Detail of the last failure on this context (empty string if none). */
const char* xc_last_error(const xc_ctx* ctx);

/* ---------------------------------------------------------------- job description */
typedef struct {
  int32_t n_stations;          /* S, 1..XC_MAX_STATIONS */
  int32_t n_subbands;          /* 1..XC_MAX_SUBBANDS */
  int32_t n_pols;              /* P, 1 or 2; inputs are ordered i = s*P + p */
  int32_t n_chan;              /* channels kept; FFT length N = 2*n_chan, power of two */
  int32_t n_streams_recorded;  /* C in {1,2,4,8,16} */
  const int32_t* stream_map;   /* host [n_subbands*n_pols]: input (sb,p) -> recorded stream */
  double  fs_hz;               /* per-stream sample rate (twice the bandwidth, real sampling) */
  const double* lo_hz;         /* host [n_subbands]: sky frequency of each band's lower edge */
  int64_t sub_start;           /* reference-time sample index of the sub-integration start */
  int64_t n_frames;            /* FFT frames in the sub-integration (>= 1) */
  int32_t precision;           /* XC_FP32 | XC_FP16_MFMA | XC_FP8_MFMA */
  int32_t frames_per_block;    /* frames staged per F/X round, at most 65536; 0 = library
                                  default: 2048, or more (up to 65536) while the block's
                                  staged spectra stay within 16 GiB, so that a job runs
                                  in few, large rounds (the workspace grows with it:
                                  xc_workspace_bytes) */
} xc_setup;

typedef struct {
  const void*    frames;       /* device: the station's recording, n_frames_m5b frames */
  int64_t        n_frames_m5b;
  int64_t        first_sample; /* station-time sample index of the first payload sample */
  const uint8_t* frame_ok;     /* device [n_frames_m5b] from xc_ingest, or NULL (computed) */
  int32_t        poly_deg;     /* 0..XC_MAX_POLY_DEG */
  const double*  delay_poly;   /* host [poly_deg+1]: tau(t) in seconds, ascending powers,
                                  t = reference time in seconds since the polynomial epoch */
  const double*  phase_poly;   /* host [n_subbands][poly_deg+1] fringe phase in turns of the
                                  same t, or NULL: phase = lo_hz[sb] * tau(t) */
  double         poly_t0, poly_t1;  /* validity span of the polynomials (seconds) */
  int32_t        rate_correct; /* 1: correct the delay's drift inside each frame (the delay
                                  runs D_c + rho (n - N/2) samples across a frame, rho the
                                  delay rate at its centre): each kept spectrum becomes
                                  (1 - rho) Y(k) + (2 pi i rho k / N) Yr(k), Yr the spectrum
                                  of the ramp-weighted window -- first order in rho, for a
                                  spacecraft whose delay rate smears long frames.  FP32 path
                                  and n_chan <= 8192 only (XC_E_INVAL otherwise); 0: off */
} xc_station;

typedef struct {
  void*  vis;      /* device: complex float [n_subbands][M(M+1)/2][n_chan], M = S*P;
                      baselines (i,j), i <= j, packed row-major, diagonal = autos */
  float* weight;   /* device: float [n_subbands][M(M+1)/2], frames valid for both inputs */
} xc_output;

/* ---------------------------------------------------------------- ingest (A0) */
/* Per-frame validity of a recording: frame_ok[f] = 1 iff frame f's sync word is
 * 0xABADDEED.  frames: device, n_frames_m5b * 10016 bytes; frame_ok: device.  Async. */
int xc_ingest(xc_ctx* ctx, const void* frames, int64_t n_frames_m5b, uint8_t* frame_ok,
              void* stream);

/* ---------------------------------------------------------------- plain per-job path */
/* Check a job description without touching the GPU: XC_OK, XC_E_INVAL or
 * XC_E_RANGE (message in xc_last_error when ctx is not NULL). */
int xc_validate(xc_ctx* ctx, const xc_setup* setup, const xc_station* st);

/* Device workspace a correlate_subint call with this setup needs (0 on bad setup). */
size_t xc_workspace_bytes(const xc_ctx* ctx, const xc_setup* setup, const xc_station* st);

/* Correlate one sub-integration.  st: host [n_stations]; out: host struct of
 * device pointers; workspace: device, ws_bytes >= xc_workspace_bytes().  Async
 * on `stream`; results are complete when the stream reaches this point.
 * V = mean over valid frames (unnormalised FFT); W = 0 gives V = 0.  Frames
 * whose shifted window leaves a station's recording, or touches a recording
 * frame that fails its sync check, are not errors: they count 0 in W.  The
 * call returns before the GPU has judged any frame, so partial coverage is
 * reported by W (< n_frames), not by the return code. */
int xc_correlate_subint(xc_ctx* ctx, const xc_setup* setup, const xc_station* st,
                        const xc_output* out, void* workspace, size_t ws_bytes, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc): xc_correlate_subint
 * without a workspace argument.  The library's own fixed device scratch of
 * xc_noalloc_scratch_bytes() (256 MiB, one per GPU the library runs on,
 * held until the process ends) takes the workspace's place;
 * the call allocates nothing.  With frames_per_block = 0 (setup and tuning)
 * the library picks the largest block whose layout fits the scratch;
 * otherwise a layout that does not fit returns XC_E_NOMEM, as does a job
 * whose one-frame blocks do not fit.  Every call on a GPU shares that GPU's
 * scratch: calls in order on one stream are safe, calls that overlap on one
 * GPU (other streams, other threads, other contexts) race.  Results equal
 * xc_correlate_subint's at the same frames per block.  Async on `stream`.
 * Errors as for xc_correlate_subint. */
int xc_correlate_subint_noalloc(xc_ctx* ctx, const xc_setup* setup, const xc_station* st,
                                const xc_output* out, void* stream);
size_t xc_noalloc_scratch_bytes(void);

/* ---------------------------------------------------------------- test taps */
/* Same kernels as the correlation path, results copied to host; synchronous. */
/* Delay model per station and frame: n_int [S][F], d_frac [S][F], valid [S][F],
 * phi0 [S][n_subbands][F] (fringe phase at the frame centre, turns in [0,1)).
 * Any output pointer may be NULL. */
int xc_debug_delays(xc_ctx* ctx, const xc_setup* setup, const xc_station* st,
                    int64_t* n_int, double* d_frac, int32_t* valid, double* phi0,
                    void* workspace, size_t ws_bytes, void* stream);
/* Unpacked levels q[n] (float, host [N]) of input `input` (= sb*P + p) of
 * station `station` for frame `frame`, after the integer shift; all zero if
 * the frame is invalid. */
int xc_debug_unpack(xc_ctx* ctx, const xc_setup* setup, const xc_station* st,
                    int32_t station, int32_t input, int64_t frame, float* out,
                    void* workspace, size_t ws_bytes, void* stream);
/* Spectra after fractional-delay correction for frames frame0 .. frame0+n-1
 * (n <= frames_per_block of the setup): device complex float
 * [n_subbands][n][M][n_chan].  Async. */
int xc_debug_spectra(xc_ctx* ctx, const xc_setup* setup, const xc_station* st,
                     int64_t frame0, int32_t n, void* spectra, void* workspace,
                     size_t ws_bytes, void* stream);

/* ---------------------------------------------------------------- tuning */
/* Launch-shape parameters of the context (0 = library default / autotuned).
 * They change speed only: results are identical for every setting except
 * frames_per_block, which changes FP32 summation order, and F-stage variants 5
 * and 7, which at FFT lengths of 2048 and below round the last-pass twiddles
 * differently (results stay within the FP32 path's tolerance). */
typedef struct {
  int32_t fstage_waves_per_simd;   /* F-stage variant: 0 = default (FP32 spectra: 2 for
                                      dual-pol jobs with FFT lengths up to 4096, 7 for
                                      single-pol ones from 1024 to 4096; 7 for FFT lengths
                                      of 8192 and more; else 1); 1 = one task per station and
                                      frame group, the next task's window words loaded
                                      during the transforms; 2 = the pols of a subband
                                      share their fringe phasors (fewer operations, more
                                      registers); 3 or 4 = at least that many waves per
                                      SIMD requested (fewer registers); 5 = split twiddle
                                      tables (the last FFT pass multiplies two table
                                      entries: less LDS per workgroup, so more resident
                                      workgroups, for one complex multiply per twiddle);
                                      7 = lean tasks: one per station, frame group and
                                      group of up to four inputs, whose 2-bit codes are
                                      packed into one register per input before the
                                      transforms (split twiddles, 4 waves per SIMD; the
                                      window words are loaded once per group); 8 = as
                                      1, with the pols of a subband sharing their fringe
                                      phasors, no word prefetch and the fractional-delay
                                      phasors stepped at the store (bit-identical to 1).
                                      2-4 and 8 apply to FP32 spectra only. */
  int32_t xmac_frames_per_stage;   /* X-stage input staging: 8 = ring of 8 one-frame LDS
                                      stages filled by direct memory-to-LDS loads, products
                                      on the vector units (64-channel tiles, at most 32
                                      inputs per subband); 2 or 4 = double-buffered stages
                                      of that many frames through registers (the default
                                      above 32 inputs per subband);
                                      1 = no LDS staging (inputs read from memory, one frame
                                      ahead); 3 = the FP32 products on the matrix cores
                                      (v_mfma_f32_4x4x1: 16 channels per wave, inputs read
                                      from memory a few frames ahead, at most 32 inputs per
                                      subband, channels a multiple of 16); 5 = the same
                                      matrix-core products fed through the ring of 8 LDS
                                      stages (each input loaded once per 64-channel
                                      workgroup; at most 32 inputs per subband, channels a
                                      multiple of 64; the default where it applies, and the
                                      X stage of fused batches); 0 = default.
                                      Every staging gives bit-identical visibilities: the
                                      matrix cores' products are fused multiply-adds with
                                      one rounding, issued in the vector kernels' order */
  int32_t xmac_channels_per_wg;    /* X-stage channel tile: 0, 16, 32 or 64 */
  int32_t frames_per_block;        /* used when a setup says 0: 0 (= the library default)
                                      or 1..65536 */
  int32_t xmac_tiles_per_wg;       /* X-stage 4x4 input tiles per workgroup: 0 = all */
  int32_t block_overlap;           /* single-job calls over two or more blocks: 0 = default
                                      (off), 1 = off, 2 = on.  On: the F stage of block b + 1
                                      runs beside the X stage of block b on a second,
                                      library-owned stream (two block buffers in the
                                      workspace; identical results); the call stays
                                      asynchronous on the caller's stream */
} xc_tuning;

int xc_set_tuning(xc_ctx* ctx, const xc_tuning* t);
int xc_get_tuning(const xc_ctx* ctx, xc_tuning* t);

/* ---------------------------------------------------------------- batches */
/* A batch runs many sub-integrations of uneven shapes as one unit (the
 * batching of many sub-integrations in one persistent launch; abstract and
 * section 2 describe the correlator whose sub-integrations these are).
 * Default executor: short jobs (at most 4 blocks of frames_per_block frames)
 * of one FFT length form a group that runs in rounds; round r takes block r of
 * every job of the group and runs all of them as one delay launch, one
 * F-stage launch that is persistent over the tasks of every job's block, and
 * one X-stage launch per input-tile shape.  Groups of different FFT lengths run side by side on
 * n_lanes concurrent HIP streams ("lanes"); one ingest (each distinct
 * recording once), one clear of all accumulators and one finalise serve the
 * whole batch.  Long jobs (their own launches fill the GPU) and jobs the
 * fused kernels do not take (FP16 / FP8 precision, 16384 channels, drift
 * correction, or an X-stage tuning other than the default or the rings) run as
 * single jobs on the lanes, longest first.  XC_BATCH_LANES instead runs every
 * job as a single job, spread longest-first over the lanes.  Either way the
 * results are identical bit for bit to running each job alone with the
 * batch's block size: the library default, capped so that a job's staged
 * spectra stay within 1 GiB, except for a job the cap would cut into more than
 * four blocks, which keeps the default block and runs on the first lane, one
 * such job after another (so that it gives the same bits as a plain call).  With XC_BATCH_GRAPH the launches are captured
 * once as a hipGraph and a later call with an identical batch replays the
 * graph (one launch). */
typedef struct {
  xc_setup setup;
  const xc_station* st;        /* host [setup.n_stations] */
  xc_output out;
} xc_job;

#define XC_BATCH_GRAPH 1
#define XC_BATCH_LANES 2

/* Device workspace a batch needs with these flags (0 if a job is invalid). */
size_t xc_batch_workspace_bytes(xc_ctx* ctx, const xc_job* jobs, int32_t n_jobs,
                                int32_t n_lanes, int32_t flags);
/* Correlate jobs[0..n_jobs) (1 <= n_lanes <= 16).  Async on `stream`: all
 * results are complete when the stream reaches this point.  Error codes as
 * for xc_correlate_subint; the message names the failing job. */
int xc_correlate_batch(xc_ctx* ctx, const xc_job* jobs, int32_t n_jobs, int32_t n_lanes,
                       int32_t flags, void* workspace, size_t ws_bytes, void* stream);

/* ---------------------------------------------------------------- serving */
/* A server admits correlation requests continuously: each request needs a
 * slot (one of max_slots concurrent HIP streams) and its workspace footprint
 * from a device pool of hbm_budget_bytes allocated at creation; requests that
 * arrive while others run start as soon as a slot and memory are free, and
 * their work overlaps on the device.  Admission is first-in first-out, except
 * that a later request may start ahead of one that does not fit yet (at most
 * 8 times, then the earlier one blocks admission until it fits).  Results do
 * not depend on what else runs (a request's block is the library default,
 * capped so that its staged spectra stay within half the budget over the
 * slots, at least 1 GiB; never below 16 (M + 1) frames: the request run alone
 * at that block size gives the same bits).  Station recordings and outputs stay
 * caller-owned device memory and must stay valid until the request is done;
 * the job description (setup, stations, polynomials) is copied at submit. */
typedef struct xc_server xc_server;

typedef struct {
  double p50_ms, p99_ms, mean_ms;  /* latency: submit -> completion seen by the server */
  int64_t completed;               /* finished with XC_OK */
  int64_t failed, cancelled;
  int64_t queued, running;         /* now */
  double station_samples_per_s;    /* completed work / (last completion - first submit) */
} xc_server_stats;

int  xc_server_create(xc_server** out, int hip_device, size_t hbm_budget_bytes,
                      int32_t max_slots);
/* XC_E_NOMEM if the job's footprint exceeds the whole budget; XC_E_INVAL or
 * XC_E_RANGE for an invalid job; otherwise queues it and sets *ticket. */
int  xc_server_submit(xc_server* srv, const xc_job* job, uint64_t* ticket);
/* *done = 1 once the request finished; returns its result code then.  Once
 * poll or wait has reported a request finished, the server forgets its ticket:
 * later calls with it return XC_E_INVAL. */
int  xc_server_poll(xc_server* srv, uint64_t ticket, int32_t* done);
/* Block until done (returns its result code) or XC_E_TIMEOUT after timeout_ms (< 0: no limit). */
int  xc_server_wait(xc_server* srv, uint64_t ticket, int32_t timeout_ms);
/* A queued request is dropped; a running one completes on the device but
 * reports XC_E_CANCELLED.  XC_E_INVAL for an unknown or finished ticket. */
int  xc_server_cancel(xc_server* srv, uint64_t ticket);
int  xc_server_get_stats(xc_server* srv, xc_server_stats* out);
const char* xc_server_last_error(xc_server* srv);
/* Cancels queued requests, waits for running ones, frees the pool. */
void xc_server_destroy(xc_server* srv);

/* ---------------------------------------------------------------- autotuner */
/* Time candidate launch shapes (X-stage kernel, stage depth and channel tile;
 * frames per block only where the default does not fit the workspace) on this
 * job (its first 8192 frames) and remember the fastest for
 * every job of the same shape (FFT length, inputs, subbands, recorded
 * streams, precision) on this context.  Runs on `stream` and synchronises.
 * out/workspace as for xc_correlate_subint; candidates whose workspace does
 * not fit ws_bytes are skipped.  Frames per block: the library default (no
 * smaller block is faster over a whole job; a short probe repeated back to
 * back favours small ones through the cache), or, where it does not fit the
 * workspace, the largest power of two up to 2048 that does.  The library
 * default (the first candidate) stays
 * unless another candidate is more than 3 % faster.  best (host) may be NULL. */
int xc_autotune(xc_ctx* ctx, const xc_setup* setup, const xc_station* st, const xc_output* out,
                void* workspace, size_t ws_bytes, void* stream, xc_tuning* best);

/* ---------------------------------------------------------------- fringe search */
/* Delay-rate fringe search over T stacked sub-integrations: the search behind
 * the paper's first-fringe result (a single peak in residual delay and rate
 * inside a fringe-search window) and its wide search windows (section 2).
 * Per subband and baseline, with V_t[k] the visibility of sub-integration t,
 * channel k:
 *   F_t[d]  = sum_{k < n_chan} V_t[k] exp(-2 pi i k d / D)   (zero-padded to D)
 *   G[r, d] = sum_{t < T}      F_t[d] exp(-2 pi i t r / R)   (zero-padded to R)
 * Bins are signed, d in [-D/2, D/2) and r in [-R/2, R/2); the peak is the
 * largest |G| with |d| <= delay_win and |r| <= rate_win (0 = the whole axis),
 * ties going to the smallest r D + d of the unsigned bins; a parabola through
 * |G| at the peak and its two cyclic neighbours along each axis gives sub-bin
 * offsets.  FP32 arithmetic. */
typedef struct {
  int32_t n_subints;           /* T, 1..256 */
  int32_t n_subbands;          /* >= 1 */
  int32_t n_baselines;         /* >= 1 (e.g. M(M+1)/2 of a correlate output) */
  int32_t n_chan;              /* >= 1 */
  int32_t delay_len;           /* D: power of two, 256..16384, >= n_chan */
  int32_t rate_len;            /* R: power of two, T..1024 */
  int32_t delay_win;           /* search half-width in delay bins, 0 = whole axis */
  int32_t rate_win;            /* search half-width in rate bins, 0 = whole axis */
  double  chan_width_hz;       /* channel spacing dnu > 0 */
  double  t_int_s;             /* sub-integration spacing > 0 */
} xc_fringe_setup;

typedef struct {
  int32_t delay_bin;           /* signed peak bins */
  int32_t rate_bin;
  float   amp;                 /* |G| / (n_chan T): a unit-modulus fringe gives 1 */
  float   phase;               /* arg G at the peak, radians */
  float   delay_off;           /* parabolic sub-bin offsets */
  float   rate_off;
  double  delay_s;             /* (delay_bin + delay_off) / (D dnu) */
  double  rate_hz;             /* (rate_bin + rate_off) / (R t_int) */
} xc_fringe_peak;

/* Device workspace xc_fringe_search needs (0 if the setup is invalid). */
size_t xc_fringe_workspace_bytes(const xc_fringe_setup* fs);
/* vis: device complex float [T][n_subbands][n_baselines][n_chan] (for example
 * T correlate outputs, stacked); peaks: device xc_fringe_peak
 * [n_subbands][n_baselines]; map: NULL, or device complex float
 * [n_subbands][n_baselines][R][D] receiving G.  The caller owns every buffer.
 * Async on `stream`.  Errors: XC_E_INVAL (setup out of range or a NULL buffer),
 * XC_E_NOMEM (workspace smaller than xc_fringe_workspace_bytes), XC_E_HIP. */
int xc_fringe_search(xc_ctx* ctx, const xc_fringe_setup* fs, const void* vis, void* peaks,
                     void* map, void* workspace, size_t ws_bytes, void* stream);

/* ---------------------------------------------------------------- feed-angle correction */
/* The equivalent of the parallactic-angle correction for dual-polarisation
 * products (the paper lists it for the spaceborne antenna, computed from the
 * spacecraft orientation in its telemetry; section 2).  The angles are inputs.
 * A feed turned by chi gives, for linear feeds, X' = X cos chi + Y sin chi,
 * Y' = -X sin chi + Y cos chi; for circular feeds R' = exp(-i chi) R,
 * L' = exp(+i chi) L.  The correction restores the unturned feeds' products:
 * circular V_ij exp(+i (s_p chi_a - s_q chi_b)) with s_R = +1, s_L = -1;
 * linear, per station pair, V <- Rot(chi_a)^T V Rot(chi_b),
 * Rot = [[cos, sin], [-sin, cos]].  FP32 products, FP64 angles. */
#define XC_FEED_CIRCULAR 0      /* pol 0 = R, pol 1 = L */
#define XC_FEED_LINEAR   1      /* pol 0 = X, pol 1 = Y */

typedef struct {
  int32_t n_subints;           /* T >= 1 */
  int32_t n_subbands;          /* >= 1 */
  int32_t n_stations;          /* S >= 1: products of M = 2 S inputs, i = 2 s + p */
  int32_t n_chan;              /* >= 1 */
  int32_t feed;                /* XC_FEED_CIRCULAR or XC_FEED_LINEAR */
} xc_feed_setup;

/* In place on vis: device complex float [T][n_subbands][M(M+1)/2][n_chan]
 * (packed upper triangle i <= j, as xc_correlate_subint writes it, stacked over
 * T sub-integrations); angles: device double [T][S], radians.  Async on
 * `stream`.  Errors: XC_E_INVAL (setup out of range or a NULL pointer), XC_E_HIP. */
int xc_feed_correct(xc_ctx* ctx, const xc_feed_setup* fs, void* vis, const double* angles,
                    void* stream);

/* ---------------------------------------------------------------- kernel timing */
/* Kernel kinds for xc_profile_end. */
#define XC_K_INGEST    0
#define XC_K_DELAYS    1
#define XC_K_FSTAGE    2
#define XC_K_XMAC      3
#define XC_K_XMFMA     4
#define XC_K_FINALISE  5
#define XC_K_ZERO      6
#define XC_K_FRINGE    7
#define XC_K_FEED      8
#define XC_NKINDS      9

/* Start recording a HIP event pair around every kernel launch of this context
 * (on the launch's own stream), for at most max_launches launches. */
int xc_profile_begin(xc_ctx* ctx, int32_t max_launches);
/* Stop recording, wait for the recorded events and return, per kind, the
 * summed kernel time in ms and the launch count (host arrays [XC_NKINDS]).
 * Synchronous. */
int xc_profile_end(xc_ctx* ctx, double* ms_by_kind, int64_t* launches_by_kind);

#ifdef __cplusplus
}
#endif
#endif /* XCORR_H */
