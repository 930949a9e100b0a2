// Host-side launchers of the library's kernels (one translation unit per
// kernel family; the runtime in xcorr.hip sequences them).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "xc_dev.h"

namespace xc {

// A0: frame_ok[f] = sync word of recording frame f is good.
hipError_t launch_ingest(const uint32_t* words, int64_t n_frames, uint8_t* frame_ok,
                         hipStream_t s);
// Zero n doubles.
hipError_t launch_zero(double* p, size_t n, hipStream_t s);
// A1: delay and phase records for frames f0 .. f0+nf-1 of every station; also
// zeroes the F stage's task counter *ctr when ctr is not null.
hipError_t launch_delays(const DevJob* job, int n_stations, int n_subbands, int64_t f0, int nf,
                         DelayRec* drec, PhaseRec* prec, unsigned* ctr, hipStream_t s);
// A2-A5: spectra [n_subbands][nf][M][n_chan] for the block's frames.
// Spectrum element types written by the F stage.
constexpr int kOutF32 = 0;   // float2
constexpr int kOutF16 = 1;   // (Re, Im) FP16, scaled by 2^scale_exp
constexpr int kOutF8 = 2;    // (Re, Im) OCP e4m3, scaled by 2^scale_exp, saturated at 448
inline int out_elem_bytes(int out) { return out == kOutF32 ? 8 : out == kOutF16 ? 4 : 2; }

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
// phasors stepped at the store to make room for them; the default for dual-pol
// FP32 jobs up to kShareMaxN (measured on MI355X: a C2-shaped F stage 3.3 %
// faster; at N = 4096 the registers would cost a wave per SIMD).
constexpr int kFstageShare = 8;
constexpr int kShareMaxN = 2048;
constexpr int kLeanMinN = 8192;
constexpr int kLeanGroup = 4;   // inputs per lean task
// The F-stage variant a job runs: the tuned one, else kFstageShare where it pays.
inline int fstage_variant(int tuned, int n_pols, int n_chan, int out) {
  if (tuned != 0) return tuned;
  return n_pols == 2 && 2 * n_chan <= kShareMaxN && out == kOutF32 ? kFstageShare : 0;
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
// Power-of-two exponents per (subband, input, channel) that bring the mean
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
// FP64 slot, for blocks of T frames of a job with M inputs per subband: 512
// when that still gives the GPU enough workgroups, else 256.  A block of nf
// frames uses ceil(nf / that) slots.
int xmac_frames_per_split(int T, int M, int n_chan, int n_subbands);
// A6: accumulate the block's spectra into the FP64 slots vacc[split][n_sb][nbl][n_chan]
// (double2), slot_stride elements apart; fps: xmac_frames_per_split of the job.
// fb: staging (8 = LDS ring, 2 or 4 = register-staged stages, 1 = none, 0 = default);
// kc: channel tile (16/32/64, 0 = auto); tpw: 4x4 tiles per workgroup (0 = all that fit).
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
// Test tap: unpacked levels of one (station, input, block frame).
hipError_t launch_debug_unpack(const DevJob* job, const DelayRec* drec, int nf, int station,
                               int input, int fl, float* out, int N, hipStream_t s);

bool fstage_supported(int N);

}  // namespace xc
