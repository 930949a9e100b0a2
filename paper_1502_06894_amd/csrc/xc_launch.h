// Host-side launchers of the library's kernels (one translation unit per
// kernel family; the runtime in xcorr.hip sequences them).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "xc_dev.h"

namespace xc {

// One job's block of frames in a round of a fused batch: a device table of
// these drives one delay, one weight, one F-stage and one X-stage launch per
// round over the blocks of many jobs (every job of the round has the same FFT
// length; an X launch takes the items of one input-tile shape).  Each launch
// numbers its workgroups (or the F stage its tasks) consecutively over the
// items; the *0 fields give the first number of each item.
struct FusedItem {
  DevJob jd;               // the job's descriptor, by value (read as constant data)
  const DevJob* job;       // the same descriptor in the workspace
  DelayRec* drec;          // [S][nf]
  PhaseRec* prec;          // [S][n_sb][nf]
  float2* spec;            // [n_sb][nf][M][n_chan]
  double2* vacc;           // the job's FP64 accumulator slots
  double* wst;             // the job's station-pair weights [S][S]
  size_t slot_stride;      // double2 elements per slot
  int64_t f0;              // first frame of the block
  int32_t nf;              // frames in the block
  int32_t fps;             // X stage: frames per FP32 slice
  int32_t task0;           // F stage: tasks before this item
  int32_t dblk0;           // delay kernel: workgroups before this item
  int32_t wblk0;           // weight kernel: workgroups before this item
  int32_t xblk0;           // X stage: workgroups before this item in its launch
};

// The item whose numbers start at or before `x` (first[i] ascending, first[0] = 0).
template <class P, class Get>
__device__ inline int fused_find(P items, int n, int x, Get first) {
  int lo = 0, hi = n - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (first(items[mid]) <= x)
      lo = mid;
    else
      hi = mid - 1;
  }
  return lo;
}
__device__ inline int fused_item_of(const FusedItem* items, int n, int task) {
  return fused_find(items, n, task, [](const FusedItem& I) { return I.task0; });
}
// The item table viewed as constant memory: the launches that read it never
// write it, and through this view the compiler keeps the item's fields (and
// its job's) in scalar registers, loaded with scalar loads.
typedef const __attribute__((address_space(4))) FusedItem* FusedItemsK;
__device__ inline FusedItemsK fused_const(const FusedItem* items) { return (FusedItemsK)items; }

// A0: frame_ok[f] = sync word of recording frame f is good.
hipError_t launch_ingest(const uint32_t* words, int64_t n_frames, uint8_t* frame_ok,
                         hipStream_t s);
// Zero n doubles.
hipError_t launch_zero(double* p, size_t n, hipStream_t s);
// A1: delay and phase records for frames f0 .. f0+nf-1 of every station; also
// zeroes the F stage's task counter *ctr when ctr is not null.
hipError_t launch_delays(const DevJob* job, int n_stations, int n_subbands, int64_t f0, int nf,
                         DelayRec* drec, PhaseRec* prec, unsigned* ctr, hipStream_t s);
// A2-A5: spectra [n_subbands][nf][M][n_chan] for the block's frames (FP32;
// the low-precision ones channel-blocked, see lp_index).
// Spectrum element types written by the F stage.
constexpr int kOutF32 = 0;   // float2
constexpr int kOutF16 = 1;   // (Re, Im) FP16, scaled by 2^scale_exp
constexpr int kOutF8 = 2;    // (Re, Im) OCP e4m3, scaled by 2^scale_exp, saturated at 448
inline int out_elem_bytes(int out) { return out == kOutF32 ? 8 : out == kOutF16 ? 4 : 2; }
// Low-precision spectra are channel-blocked, [n_subbands][nf][n_chan / 16][M][16]:
// a frame's 16-channel tile of all M inputs is one contiguous run (M x 64 B in
// FP16, M x 32 B in e4m3), the unit one MFMA X-stage workgroup reads.
// Element (subband-frame sf = sb nf + f, input m, channel k):
__host__ __device__ inline size_t lp_index(size_t sf, int m, int k, int M, int n_chan) {
  return (sf * (size_t)(n_chan >> 4) + (size_t)(k >> 4)) * (size_t)(M * 16) + (size_t)m * 16 +
         (size_t)(k & 15);
}
// The exponents of the low-precision outputs, int8 [n_subbands][M][n_chan / 8][8]:
// channel k of a row sits at byte scale_pos(k), so that F-stage thread t,
// whose kept bins are k = t + r n_chan / 8 (r < 8), finds its eight exponents
// in one aligned 8-byte word.
__host__ __device__ inline int scale_pos(int k, int n_chan) {
  const int q = n_chan >> 3;
  return (k & (q - 1)) * 8 + k / q;
}

// waves: F-stage variant (0 = default: kFstageLean for N >= kLeanMinN, else one task per
// station and frame group; 1 = the latter at every N; 2..5, 7, 8 as the tuning field
// describes; FP32 output only except 5 and 7).  The caller picks kFstageShare for dual-pol
// FP32 jobs (fstage_variant()).  kFstageLean: tasks of up to four inputs whose 2-bit
// codes are packed into one register each, so the window words are not held across the
// transforms (fewer registers, more resident waves, for reloading the words per group).
// kFstageRatePass: the drift-correction pass, run after the regular F stage on
// the stations that ask for it: it transforms the ramp-weighted window and rewrites their
// spectra in place as (1 - rho) Y + (2 pi i rho k / N) fd Yr (FP32 spectra, N <= 16384; it
// takes the next task counter, ctr + 1 of the regular pass).
constexpr int kFstageRatePass = 6;
constexpr int kFstageLean = 7;
// kFstageShare: the pols of a subband share their fringe phasors (held from the
// first pol to the second), with no word prefetch and the fractional-delay
// phasors stepped at the store to make room for them (bit-identical to
// variants 0-4; the fused batch kernels' form of variant 2).
constexpr int kFstageShare = 8;
constexpr int kShareMaxN = 4096;
constexpr int kLeanMinN = 8192;
constexpr int kLeanGroup = 4;   // inputs per lean task
// The F-stage variant a job runs: the tuned one, else for FP32 spectra up to
// N = kShareMaxN variant 2 for dual-pol jobs (pols share their fringe phasors,
// with the word prefetch and held fractional-delay phasors) and lean tasks
// for single-pol jobs from N = 1024; 0 otherwise (lean tasks from kLeanMinN).
// Measured on MI355X, F stage of 10-station, 2-subband jobs against the
// previous defaults: dual-pol N = 1024 / 2048 / 4096 -2 / -3 / -8 %,
// single-pol N = 1024 / 2048 / 4096 -7 / -9 / -3 %.
inline int fstage_variant(int tuned, int n_pols, int n_chan, int out) {
  if (tuned != 0) return tuned;
  const int N = 2 * n_chan;
  if (out != kOutF32 || N > kShareMaxN) return 0;
  if (n_pols == 2) return 2;
  return N >= 1024 ? kFstageLean : 0;
}
constexpr int kMaxRateCorrectN = 16384;   // the drift correction runs in the one-workgroup FFT
// ctr: task counter, zero at launch (launch_delays clears it), one per concurrent launch.
// scratch: fstage_scratch_bytes(...) of device memory (N = 32768 with FP16 / e4m3 spectra
// only; else unused).
hipError_t launch_fstage(int N, const DevJob* job, int n_stations, int n_inputs,
                         const DelayRec* drec, const PhaseRec* prec, const float2* tw,
                         void* spec, const int8_t* scale_exp, int nf, int waves, int out,
                         unsigned* ctr, float2* scratch, hipStream_t s);
// Scratch the F stage needs for nf frames (nonzero for N = 32768: its four-step
// FFT goes through memory).
size_t fstage_scratch_bytes(int N, int n_stations, int n_inputs, int nf, int out);
// Power-of-two exponents per (subband, input, channel) (at scale_pos) that bring the mean
// |Y|^2 of the first nf frames (FP32 spectra [n_sb][nf][M][n_chan]) to
// target_log2 (i.e. RMS 2^target_log2), averaged over the frames that drec
// ([n_stations][nf], input m = s P + p) marks valid; an input with no valid
// frame among them takes the expected power of white 2-bit data.
hipError_t launch_scales(const float2* spec, const DelayRec* drec, int n_subbands, int nf, int M,
                         int P, int n_chan, int target_log2, int8_t* scale_exp, hipStream_t s);
// A7: X stage on MFMA for the low-precision spectra (out = kOutF16 or kOutF8),
// M <= 32; accumulates into the same FP64 slots as the FP32 X stage.
hipError_t launch_xmfma(const DevJob* job, int out, int M, int n_chan, int n_subbands,
                        const void* spec, const int8_t* scale_exp, double2* vacc,
                        size_t slot_stride, int nf, hipStream_t s);
// Frames (at most) one X workgroup accumulates in FP32 before adding to its
// FP64 slot, for blocks of T frames of a job with M inputs per subband: up to
// 1024 (balanced so that the ring-fed matrix kernel's workgroups fill whole
// rounds of the GPU) or 512 when that still gives the GPU enough workgroups,
// else 256.  A block of nf frames uses at most ceil(nf / that) slots.
int xmac_frames_per_split(int T, int M, int n_chan, int n_subbands);
// A6: accumulate the block's spectra into the FP64 slots vacc[split][n_sb][nbl][n_chan]
// (double2), slot_stride elements apart; fps: xmac_frames_per_split of the job.
// fb: staging (8 = LDS ring, 2 or 4 = register-staged stages, 1 = none,
// kXmacMatrix = FP32 products on the matrix cores with operands loaded per
// wave, kXmacMatrixRing = the same products fed through the LDS ring, 0 =
// default); kc: channel
// tile (16/32/64, 0 = auto); tpw: 4x4 tiles per workgroup (0 = all that fit).
// Every staging gives bit-identical sums.
constexpr int kXmacMatrix = 3;
constexpr int kXmacMatrixRing = 5;
hipError_t launch_xmac(const DevJob* job, int M, int n_chan, int n_subbands,
                       const float2* spec, double2* vacc, size_t slot_stride, int nf, int fps,
                       int fb, int kc, int tpw, hipStream_t s);
// Frames of the block valid for both stations of each station pair: wst[si][sj] += count.
hipError_t launch_weights(const DelayRec* drec, int n_stations, int nf, double* wst,
                          hipStream_t s);
// A8: vis = (sum of the n_slots slots) / W (W = 0 -> 0), weight = W, with W of
// baseline (i, j) taken from wst[i / P][j / P].
hipError_t launch_finalise(const double2* vacc, int n_slots, size_t slot_stride,
                           const double* wst, int n_stations, int n_pols, float2* vis,
                           float* weight, int n_subbands, int M, int n_chan, hipStream_t s);
// Fused batches (FP32 spectra, the regular F-stage variants 0, kFstageLean and
// kFstageShare; no drift-correction pass).  `items` is a device table of
// n_items FusedItem; ctr a zeroed counter (launch_delays_fused clears it).
// Delay and phase records of every item's block (+ clears ctr[0], ctr[1]).
hipError_t launch_delays_fused(const FusedItem* items, int n_items, int n_blocks, unsigned* ctr,
                               hipStream_t s);
// Workgroups launch_delays_fused needs for an item of nf frames, S stations, n_sb subbands.
int delays_fused_blocks(int nf, int n_stations, int n_subbands);
// Station-pair weights of every item's block, added to the item's job's wst.
hipError_t launch_weights_fused(const FusedItem* items, int n_items, int n_blocks, hipStream_t s);
int weights_fused_blocks(int nf, int n_stations);
// F stage over every item's block (all items of FFT length N, variant `waves`).
hipError_t launch_fstage_fused(int N, int waves, const FusedItem* items, int n_items,
                               int n_tasks, const float2* tw, unsigned* ctr, hipStream_t s);
// F-stage tasks of an item (job with S stations and n_inputs inputs, nf frames).
int fstage_fused_tasks(int N, int waves, int n_stations, int n_inputs, int nf);
// The F-stage variant of a fused batch item: what the per-job path would run.
int fstage_fused_variant(int N, int n_pols, int n_chan);
// X stage over every item (all with inputs padded to Mp = MP, 64-channel tiles:
// the matrix cores fed through the LDS ring); workgroups of one item:
// xmac_fused_blocks.
hipError_t launch_xmac_fused(int Mp, const FusedItem* items, int n_items, int n_blocks,
                             hipStream_t s);
int xmac_fused_blocks(int M, int n_chan, int n_subbands, int n_splits);
// Frame slices of a block of nf frames (M inputs, n_chan channels, n_subbands)
// with at most fps_max frames each: their number and the (balanced) frames per
// slice, as every X kernel splits a block (where the ring-fed matrix kernel
// takes the job, the count within ceil(nf / 1024) .. ceil(nf / fps_max) whose
// workgroups fill the most whole rounds of the GPU).
void xmac_splits(int nf, int fps_max, int M, int n_chan, int n_subbands, int& n_splits, int& fps);
// Whether the fused X stage takes a job of M inputs and n_chan channels.
bool xmac_fused_ok(int M, int n_chan);

// One job of a fused batch's finalise (blk0: workgroups before it).
struct FusedOut {
  const double2* vacc;
  const double* wst;
  float2* vis;
  float* weight;
  size_t slot_stride;
  int32_t n_slots, S, P, M, nbl, n_chan, n_sb, blk0;
};
hipError_t launch_finalise_fused(const FusedOut* outs, int n_outs, int n_blocks, hipStream_t s);
int finalise_fused_blocks(int n_subbands, int M, int n_chan);
// One recording of a fused batch's ingest (blk0: workgroups before it).
struct FusedMask {
  const uint32_t* words;
  uint8_t* ok;
  int64_t n_frames;
  int32_t blk0;
};
hipError_t launch_ingest_fused(const FusedMask* masks, int n_masks, int n_blocks, hipStream_t s);
int ingest_fused_blocks(int64_t n_frames);

// Test tap: unpacked levels of one (station, input, block frame).
hipError_t launch_debug_unpack(const DevJob* job, const DelayRec* drec, int nf, int station,
                               int input, int fl, float* out, int N, hipStream_t s);

bool fstage_supported(int N);

}  // namespace xc
