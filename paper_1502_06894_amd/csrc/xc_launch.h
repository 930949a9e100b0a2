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
// A1: delay and phase records for frames f0 .. f0+nf-1 of every station.
hipError_t launch_delays(const DevJob* job, int n_stations, int n_subbands, int64_t f0, int nf,
                         DelayRec* drec, PhaseRec* prec, hipStream_t s);
// A2-A5: spectra [n_subbands][nf][M][n_chan] for the block's frames.
hipError_t launch_fstage(int N, const DevJob* job, int n_stations, const DelayRec* drec,
                         const PhaseRec* prec, const float2* tw, float2* spec, int nf,
                         hipStream_t s);
// A6: accumulate the block's spectra into vacc [n_sb][nbl][n_chan] (double2) and
// weights wacc [n_sb][nbl].
hipError_t launch_xmac(const DevJob* job, int M, int n_chan, int n_subbands,
                       const DelayRec* drec, const float2* spec, double2* vacc, double* wacc,
                       int nf, int n_pols, hipStream_t s);
// A8: vis = vacc / W (W = 0 -> 0), weight = W.
hipError_t launch_finalise(const double2* vacc, const double* wacc, float2* vis, float* weight,
                           int n_subbands, int nbl, int n_chan, hipStream_t s);
// Test tap: unpacked levels of one (station, input, block frame).
hipError_t launch_debug_unpack(const DevJob* job, const DelayRec* drec, int nf, int station,
                               int input, int fl, float* out, int N, hipStream_t s);

bool fstage_supported(int N);

}  // namespace xc
