// Host runtime shared by the C-ABI entry points: context, validation,
// per-job workspace arena layout, descriptor building and the launch sequence
// of one job.  Used by xcorr.hip (single jobs, taps), batch.hip (batches,
// autotuner) and server.hip (continuous-batching server).
#pragma once

#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <map>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/xcorr.h"
#include "xc_launch.h"

namespace xc {

constexpr int kSlots = 8;                 // pinned descriptor staging slots per context
constexpr size_t kSlotBytes = 256 * 1024;
constexpr size_t kAlign = 256;
constexpr int kMaxBlockFrames = 65536;
// Default frames per block: 2048, or more while the block's staged spectra
// stay within kDefaultBlockBytes.  A job alone on the device then runs in a
// few large rounds (a C2 sub-integration in 5 instead of 31): every round
// costs each kernel's ramp-up and drain and the X stage one read-modify-write
// of the FP64 accumulator slots, and a 16 GiB block is 6 % of the HBM.  Jobs
// that share the device (batches, served requests) cap their blocks lower.
constexpr int kDefaultBlockFrames = 2048;
constexpr size_t kDefaultBlockBytes = (size_t)16 << 30;
constexpr int kScaleFrames = 64;          // frames that set the MFMA path's channel scales
constexpr int kF16TargetLog2 = 10;        // FP16: scaled RMS 2^10 (max 65504)
constexpr int kF8TargetLog2 = 5;          // e4m3: scaled RMS 2^5 (max 448)
constexpr int kMaxLanes = 16;

inline size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

struct Timed {
  int kind;
  hipEvent_t a, b;
};

// Shape key of the autotune cache: FFT length, inputs, subbands, recorded streams, precision.
using ShapeKey = std::tuple<int, int, int, int, int>;

}  // namespace xc

struct xc_ctx {
  int device = 0;
  xc_tuning tune = {0, 0, 0, 0, 0, 0};       // explicit overrides (0 = auto)
  std::map<xc::ShapeKey, xc_tuning> tuned;   // autotuned shapes
  bool profiling = false;
  bool capturing = false;                    // inside a graph capture: no profiling events
  std::vector<xc::Timed> prof;
  size_t prof_used = 0;
  float2* d_tw = nullptr;                    // FFT twiddles, kTwiddleN entries
  int scratch_rc = 0;                        // lookup of the allocation-free scratch (hipError_t)
  unsigned char* h_stage = nullptr;          // kSlots x kSlotBytes pinned
  hipEvent_t ev[xc::kSlots] = {};
  int next_slot = 0;
  std::vector<hipStream_t> lanes;            // batch lanes (default priority)
  std::vector<hipEvent_t> lane_ev;           // join events, one per lane
  hipEvent_t fork_ev = nullptr;
  struct GraphEntry {
    uint64_t key;
    hipGraphExec_t exec;
  };
  std::vector<GraphEntry> graphs;            // captured batches, most recent last
  unsigned char* h_batch = nullptr;          // pinned descriptor blob of the last batch
  size_t h_batch_bytes = 0;
  hipEvent_t batch_ev = nullptr;             // the blob's upload has completed
  hipStream_t xstream = nullptr;             // X stage of overlapped single jobs
  hipEvent_t blk_f[2] = {}, blk_x[2] = {};   // block buffer p: F done / X done
  std::string last_error;
};

namespace xc {

int fail(xc_ctx* c, int code, const char* fmt, ...) __attribute__((format(printf, 3, 4)));
int hip_fail(xc_ctx* c, hipError_t e, const char* what);

// Run a launcher, bracketed by an event pair when profiling is on.
template <class Fn>
hipError_t timed(xc_ctx* c, int kind, hipStream_t s, Fn&& fn) {
  if (!c->profiling || c->capturing || c->prof_used >= c->prof.size()) return fn();
  Timed& t = c->prof[c->prof_used++];
  t.kind = kind;
  hipError_t e = hipEventRecord(t.a, s);
  if (e != hipSuccess) return e;
  e = fn();
  if (e != hipSuccess) return e;
  return hipEventRecord(t.b, s);
}

// Per-job arena: everything a job needs besides its descriptor.
struct Layout {
  size_t desc_bytes = 0;          // descriptor size (stored outside the arena)
  size_t mask = 0, drec = 0, prec = 0, spec = 0, sexp = 0, vacc = 0, wacc = 0, total = 0;
  std::vector<size_t> mask_off;   // per station, SIZE_MAX if the caller supplies frame_ok
  int T = 0;                      // frames per block
  int out = kOutF32;              // spectrum element type written by the F stage
  int n_scale = 0;                // frames of the scale pre-pass (MFMA path)
  int fps = 256;                  // X stage: frames per FP32 slice (xmac_frames_per_split)
  int n_slots = 1;                // FP64 accumulator slots of the X stage
  size_t slot_stride = 0;         // double2 elements per slot
  int nbuf = 1;                   // block buffers (2: F of block b+1 beside X of block b)
  size_t drec_bytes = 0, prec_bytes = 0, spec_bytes = 0;   // per block buffer
  size_t ctr_off = 0;             // F-stage task counter inside each delay-record buffer
  size_t scratch = 0;             // F-stage scratch (N = 32768 four-step FFT)
};

ShapeKey shape_key(const xc_setup* s);
// Launch shape for a job: explicit context overrides, else the autotuned
// entry for the job's shape, else built-in defaults (zeros).
xc_tuning effective_tuning(const xc_ctx* c, const xc_setup* s);
int validate(xc_ctx* c, const xc_setup* s, const xc_station* st);
// overlap: the caller can run blocks overlapped (single jobs); the layout then
// holds two block buffers when the tuning allows it and there are two blocks.
Layout layout_of(const xc_setup* s, const xc_station* st, const xc_tuning& tu,
                 bool overlap = false);
// Frames per block of a job that shares the device with others (a batch, a
// served request): its own block size L.T, with its staged spectra capped at
// cap_bytes, but never fewer than kSlotAmortize (M + 1) frames (nor than
// min_frames): the X stage reads and writes the job's FP64 accumulator, as
// large as M + 1 frames of spectra, once per block, so at 16 (M + 1) frames
// that traffic stays within 1/8 of the spectra's.  Returns L.T when it fits.
constexpr int kSlotAmortize = 16;
int shared_block_frames(const xc_setup& s, const Layout& L, size_t cap_bytes, int min_frames);
// Descriptor for device address `dev_desc`; stations' frame_ok default to the arena masks.
void build_desc(const xc_setup* s, const xc_station* st, const Layout& L,
                const unsigned char* dev_desc, const unsigned char* arena, unsigned char* h);
// Stage one descriptor through a pinned ring slot and copy it to dev_desc.
int upload_desc(xc_ctx* c, const xc_setup* s, const xc_station* st, const Layout& L,
                unsigned char* dev_desc, const unsigned char* arena, hipStream_t stream);
// Enqueue every kernel of one job (ingest .. finalise) on `stream`; with two
// block buffers and `xs` given, the X stages run on `xs` (joined back to
// `stream` before the finalise).
// Does any station ask for the drift correction inside frames?
bool any_rate_correct(const xc_setup* s, const xc_station* st);
int enqueue_job(xc_ctx* c, const xc_setup* s, const xc_station* st, const xc_output* out,
                const DevJob* dj, unsigned char* arena, const Layout& L, const xc_tuning& tu,
                hipStream_t stream, hipStream_t xs = nullptr);
int ensure_lanes(xc_ctx* c, int n);
// The context's X-stage stream and block events (created on first use).
int ensure_xstream(xc_ctx* c);

}  // namespace xc
