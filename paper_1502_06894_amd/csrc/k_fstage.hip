// F stage (A2-A5): 2-bit unpack of the integer-shifted window, per-sample
// fringe rotation, FFT to channels and fractional-delay correction, fused in
// one kernel.  A workgroup holds G frames of one station (G groups of T
// threads); each group loads the payload words of its window once and reuses
// them for every input (subband, pol) of the station, since all recorded
// streams of a time sample share a word.
#include <atomic>

#include "xc_fft.h"
#include "xc_launch.h"

namespace xc {

// Twiddle tables of the F stage's FFT in LDS: the full per-pass tables
// (TwLds) or the split ones (TwSplit).
constexpr int kTwFull = 1, kTwSplit = 2;

template <int N>
constexpr int tw_default() {
  // The twiddles are staged in LDS (their tables then cost no registers).  The
  // split tables win where the full ones cost resident workgroups: N = 4096
  // (2 instead of 3 per CU) and N = 16384 (the full tables would not fit
  // beside the exchange buffer); measured on MI355X, the F stage takes 16 %
  // and 66 % less time there, and 4 % more at N = 2048 and 8192.
  return N == 4096 || N == 16384 ? kTwSplit : kTwFull;
}

template <int N, int TWM = tw_default<N>()>
struct FGeom {
  static constexpr int T = FftPlan<N>::T;
  static constexpr int E = FftPlan<N>::E;
  static constexpr int G = T >= 256 ? 1 : 256 / T;   // frames per workgroup
  static constexpr int WG = T * G;
  static constexpr int tw_mode = TWM;
  static constexpr int tw_entries = TWM == kTwFull ? tw_lds_entries<N>() : tw_split_entries<N>();
  // G FFT exchange buffers, the 8-entry level table, the twiddle tables
  static constexpr size_t lut_off = (size_t)G * lds_words<N>() * sizeof(float2);
  static constexpr size_t tw_off = lut_off + 8 * sizeof(float);
  static constexpr size_t lds_bytes = tw_off + (size_t)tw_entries * sizeof(float2);
};

// Twiddle source of k_fstage<N, W, ...>: W = 5 selects the split tables.
template <int N, int W>
constexpr int fstage_twm() {
  return (W == 5 || W == kFstageLean) && N >= 512 ? kTwSplit : tw_default<N>();
}

// Spectrum element written by the F stage: FP32 complex, or for the MFMA X
// path the power-of-two-scaled value as FP16 (Re, Im) or OCP e4m3 (Re, Im).
// NT: non-temporal stores, for a wave that writes whole lines (consecutive
// channels): a block's spectra (gigabytes) are read back by the X stage only
// after the whole block is written, so keeping them in the caches would only
// evict lines that are still useful (measured on MI355X: the X stage that
// follows runs 9 % faster).  Scattered stores (every 16th channel, the
// N = 32768 row kernel) stay ordinary so that the cache merges their lines.
template <typename V>
__device__ inline void store_spec(V* p, V v, bool nt) {
  if (nt)
    __builtin_nontemporal_store(v, p);
  else
    *p = v;
}

template <int OUT, bool NT = true>
__device__ inline void put_spec(void* spec, size_t idx, float2 y, int e) {
  if constexpr (OUT == kOutF32) {
    typedef float f2 __attribute__((ext_vector_type(2)));
    const f2 v = {y.x, y.y};
    store_spec(static_cast<f2*>(spec) + idx, v, NT);
  } else if constexpr (OUT == kOutF16) {
    const float sx = ldexpf(y.x, e), sy = ldexpf(y.y, e);
    typedef _Float16 h2 __attribute__((ext_vector_type(2)));
    h2 h;
    h.x = (_Float16)sx;
    h.y = (_Float16)sy;
    store_spec(static_cast<h2*>(spec) + idx, h, NT);
  } else {
    // the conversion maps overflow to NaN: saturate at the e4m3 maximum first
    const float sx = fminf(fmaxf(ldexpf(y.x, e), -448.f), 448.f);
    const float sy = fminf(fmaxf(ldexpf(y.y, e), -448.f), 448.f);
    const int pk = __builtin_amdgcn_cvt_pk_fp8_f32(sx, sy, 0, false);
    store_spec(static_cast<uint16_t*>(spec) + idx, (uint16_t)(pk & 0xffff), NT);
  }
}

// Window words of one station-frame: the payload words holding samples
// n = t + e T of the frame's window (T is a multiple of 16, so all of a
// thread's samples share one field offset, returned in sh0).
template <int N>
__device__ inline void load_window(const DevJob& J, int s, const DelayRec& r, int t,
                                   uint32_t (&wv)[FGeom<N>::E], int& sh0) {
  constexpr int T = FGeom<N>::T, E = FGeom<N>::E;
  if (r.valid) {
    const FrameCursor c = make_cursor(J, r.base);
    const uint32_t* words = J.st[s].words;
#pragma unroll
    for (int e = 0; e < E; ++e) wv[e] = *sample_word(J, words, c, t + e * T);
    sh0 = sample_shift(J, c, t);
  } else {
#pragma unroll
    for (int e = 0; e < E; ++e) wv[e] = 0u;
    sh0 = 0;
  }
}

// Compile-time shape of the F stage's tasks for variant W (see k_fstage).
template <int N, int W>
struct FTask {
  using Gm = FGeom<N, fstage_twm<N, W>()>;
  static constexpr int T = Gm::T, E = Gm::E, G = Gm::G;
  // last-pass butterflies per thread: the thread's bins are t + b T + r N/16
  // (b < BL, r < 16), the kept half r < 8
  static constexpr int BL = E / 16;
  static constexpr int kAnchor = E / 2 < 8 ? E / 2 : 8;   // exact phasor every kAnchor samples
  // W = 2: a subband's pols share one set of fringe phasors (both see the same
  // fringe phase), held in registers from the first pol to the second
  static constexpr bool kShare = W == 2 || W == kFstageShare;
  // W = kFstageRatePass: the drift-correction pass over the stations that ask
  // for it: the window is weighted by the ramp (n - N/2) before the transform,
  // and the stored spectrum Y (from the regular pass) becomes
  // (1 - rho) Y + (2 pi i rho k / N) fd Yr.  Its tasks are (flagged station,
  // frame group, input), finer than the regular (station, frame group), so
  // that the few flagged stations still spread evenly over the workgroups.
  static constexpr bool kRamp = W == kFstageRatePass;
  // W = kFstageLean: tasks (station, frame group, group of up to kLeanGroup
  // inputs); the group's codes are packed before the transforms, the words are
  // loaded per task (no prefetch) and the fractional-delay phasors are stepped
  // at the store instead of held in registers.  Asks for 4 waves per SIMD.
  static constexpr bool kLean = W == kFstageLean;
  // The next task's words are loaded while this task is transformed, except
  // for N = 16384 (1024 threads, 128 registers each: no room for them).
  static constexpr bool kPrefetch = N <= 8192 && !kLean && W != kFstageShare;
  // the fractional-delay phasors are stepped at the store instead of held
  static constexpr bool kFdStep = kLean || W == kFstageShare;
};

// Tasks per (station, frame group) of a job: one, or one per input (the
// drift-correction pass), or one per group of up to kLeanGroup inputs.
template <int N, int W>
__device__ __forceinline__ int fstage_igroups(const DevJob& J) {
  using F = FTask<N, W>;
  return F::kRamp ? J.n_inputs : F::kLean ? (J.n_inputs + kLeanGroup - 1) / kLeanGroup : 1;
}

// One F-stage task of a frame slot: for every input of the task, the fringe
// rotation of the window's samples (level lookups from `lut`), the FFT through
// `lds`, the fractional-delay correction and the spectrum store.  The window's
// payload words `wv` (field offset sh0) are loaded by the caller.  P, M, n_chan
// and n_sb are J's.
template <int N, int W, int OUT>
__device__ __forceinline__ void fstage_task(
    const DevJob& J, int P, int M, int n_chan, int n_sb, const PhaseRec* __restrict__ prec,
    void* __restrict__ spec, const int8_t* __restrict__ scale_exp, int nf, int s, int fl,
    int in_t, const DelayRec& r, const uint32_t (&wv)[FTask<N, W>::E], int sh0, float2* lds,
    const float* lut, const float2* tw_tab, int t) {
  using F = FTask<N, W>;
  using Gm = typename F::Gm;
  constexpr int T = F::T, E = F::E, BL = F::BL, kAnchor = F::kAnchor;
  constexpr bool kShare = F::kShare, kRamp = F::kRamp, kLean = F::kLean, kFdStep = F::kFdStep;
  const double nc0 = (double)(t - N / 2);     // centred index of the thread's first sample
  constexpr double TD = (double)T;
  // (one frame per task: every task's frame is in the block, and the spectra
  // epilogue is unconditional, so nothing it loads early sinks below the FFT)
  const bool in_blk = F::G == 1 || fl < nf;
  const bool valid = r.valid != 0;
  const float* lut_t = lut + (valid ? 0 : 4);
  // fractional-delay phasors of this thread's kept output bins
  // k = t + b T + r N/16 (b < BL, r < 8): exp(2 pi i k d / N) =
  // exp(2 pi i (t + b T) d / N) * exp(2 pi i d / 16)^r
  constexpr int FDK = kFdStep ? 1 : 8;
  float2 fd[BL][FDK];
  float2 fd_st;
  {
    const float dd = (float)r.d;
    fd_st = phasor_turns(dd * (1.0f / 16.0f));
#pragma unroll
    for (int b = 0; b < BL; ++b) {
      fd[b][0] = phasor_turns((float)(t + b * T) * dd * (1.0f / (float)N));
#pragma unroll
      for (int rr = 1; rr < FDK; ++rr) fd[b][rr] = cmul(fd[b][rr - 1], fd_st);
    }
  }

  // the fringe phasors of a subband, kept for its second pol when kShare
  float2 zs[E];
  // (a drift-correction task is one input, a lean task a group of inputs)
  const int in_lo = kRamp ? in_t : kLean ? in_t * kLeanGroup : 0;
  const int in_hi = kRamp ? in_t + 1
                          : kLean ? min(in_lo + kLeanGroup, J.n_inputs) : J.n_inputs;
  // lean: the group's 2-bit codes, 16 per input packed in one register, so
  // that the window words are not held across the transforms
  uint32_t codes[kLean ? kLeanGroup : 1];
  if constexpr (kLean) {
#pragma unroll
    for (int i = 0; i < kLeanGroup; ++i) {
      const int sh = sh0 + 2 * J.stream_map[min(in_lo + i, in_hi - 1)];
      uint32_t c = 0;
#pragma unroll
      for (int e = 0; e < E; ++e) c |= ((wv[e] >> sh) & 3u) << (2 * e);
      codes[i] = c;
    }
  }
  for (int in = in_lo; in < in_hi; ++in) {
    const int sb = in / P, p = in - sb * P;
    const int sh = sh0 + 2 * J.stream_map[in];
    uint32_t code_in = 0;
    if constexpr (kLean) {
      const int i = in - in_lo;
      code_in = codes[0];
#pragma unroll
      for (int j = 1; j < kLeanGroup; ++j) code_in = i == j ? codes[j] : code_in;
    }
    if (!kShare || p == 0) {
      PhaseRec ph;
      if (in_blk) ph = prec[((size_t)s * n_sb + sb) * nf + fl];
      else ph.phi0 = ph.phi1 = ph.phi2 = 0.0;
      // fringe phasors z_e = exp(2 pi i phi(t + e T)) by the second-order recurrence
      // z_{e+1} = z_e w_e, w_{e+1} = w_e rho (w_e: phase step to the next sample,
      // rho: its constant change 2 phi2 T^2), restarted exactly every kAnchor samples.
      // Keeping w fixed leaves out phi2 T^2 e (e - 1) turns at the e-th sample
      // after an anchor; where that stays below 1e-8 turns across all E of a
      // thread's samples (ground stations, a spacecraft away from perigee) one
      // anchor and the first-order recurrence serve them all (4 fewer
      // operations per sample, one anchor instead of E / kAnchor).  The test
      // is per (station, subband, frame), hence uniform across the wave.
      const bool quad = fabs(ph.phi2) * TD * TD * (double)(E * (E - 1)) > 1e-8;
      float2 w = make_float2(1.f, 0.f);
      if (quad) {
        const float2 rho = phasor_turns(frac_f(2.0 * ph.phi2 * TD * TD));
#pragma unroll
        for (int e = 0; e < E; ++e) {
          if (e % kAnchor == 0) {
            const double nc = nc0 + (double)e * TD;
            zs[e] = phasor_turns(frac_f(fma(fma(ph.phi2, nc, ph.phi1), nc, ph.phi0)));
            w = phasor_turns(frac_f(ph.phi1 * TD + ph.phi2 * TD * (2.0 * nc + TD)));
          } else {
            zs[e] = cmul(zs[e - 1], w);
            w = cmul(w, rho);
          }
        }
      } else {
        zs[0] = phasor_turns(frac_f(fma(fma(ph.phi2, nc0, ph.phi1), nc0, ph.phi0)));
        w = phasor_turns(frac_f(ph.phi1 * TD + ph.phi2 * TD * (2.0 * nc0 + TD)));
#pragma unroll
        for (int e = 1; e < E; ++e) zs[e] = cmul(zs[e - 1], w);
      }
    }
    float2 v[E];
#pragma unroll
    for (int e = 0; e < E; ++e) {
      float q = kLean ? lut_t[(code_in >> (2 * e)) & 3u] : lut_t[(wv[e] >> sh) & 3u];
      if constexpr (kRamp) q *= (float)(t + e * T - N / 2);
      v[e] = make_float2(q * zs[e].x, q * zs[e].y);
    }
    if constexpr (Gm::tw_mode == kTwFull) {
      fft_forward<N>(v, lds, TwLds<N>{tw_tab}, t);
    } else {
      fft_forward<N>(v, lds, TwSplit<N>{tw_tab}, t);
    }
    if (in_blk) {
      // FP32 row of this input; low precision: the input's place in the
      // frame's channel-blocked run (channel k adds (k / 16) 16 M + k mod 16)
      const size_t row = OUT == kOutF32 ? ((size_t)(sb * nf + fl) * M + (s * P + p)) * n_chan
                                        : (size_t)(sb * nf + fl) * M * n_chan + (s * P + p) * 16;
      // the exponents of this thread's eight output channels t + r n_chan / 8:
      // one 8-byte word (loaded after the transforms: held across them, its
      // two registers push the lean tasks' FFT addresses into scratch)
      uint2 ex8 = make_uint2(0u, 0u);
      if constexpr (OUT != kOutF32) {
        static_assert(BL == 1 && T * 8 == N / 2, "thread t keeps bins t + r T, r < 8");
        ex8 = *reinterpret_cast<const uint2*>(scale_exp + ((size_t)sb * M + (s * P + p)) * n_chan +
                                              (size_t)t * 8);
      }
#pragma unroll
      for (int b = 0; b < BL; ++b) {
        float2 fdr = fd[b][0];
#pragma unroll
        for (int rr = 0; rr < 8; ++rr) {
          const int k = t + b * T + rr * (N / 16);
          if constexpr (kFdStep) {
            if (rr > 0) fdr = cmul(fdr, fd_st);
          } else {
            fdr = fd[b][rr];
          }
          if constexpr (kRamp) {
            float2* sp = static_cast<float2*>(spec) + row + k;
            if (valid) {
              const float2 old = *sp;
              const float2 yr = cmul(v[b + rr * BL], fdr);
              const float rho = r.rate, a = 6.28318530717958648f * rho * (float)k / (float)N;
              *sp = make_float2((1.0f - rho) * old.x - a * yr.y, (1.0f - rho) * old.y + a * yr.x);
            }
          } else {
            const float2 y = valid ? cmul(v[b + rr * BL], fdr) : make_float2(0.f, 0.f);
            // byte rr of the exponent word, sign-extended
            const uint32_t ew = rr < 4 ? ex8.x : ex8.y;
            const int ek = (int)(ew << (24 - 8 * (rr & 3))) >> 24;
            put_spec<OUT>(spec, row + (OUT == kOutF32 ? k : (k >> 4) * 16 * M + (k & 15)), y,
                          OUT == kOutF32 ? 0 : ek);
          }
        }
      }
    }
    __syncthreads();   // the next input reuses lds
  }
}

// Per-workgroup set-up of the F stage: the 2-bit level table (offset binary:
// -3.3359, -1, +1, +3.3359, then four zeros that an invalid frame's lookups
// are pointed at) and the twiddle tables, in LDS after the G exchange buffers.
template <int N, int W>
__device__ __forceinline__ void fstage_setup(const float2* __restrict__ tw, float*& lut,
                                             float2*& tw_tab) {
  using Gm = typename FTask<N, W>::Gm;
  extern __shared__ float2 lds_all[];
  unsigned char* lds_b = reinterpret_cast<unsigned char*>(lds_all);
  lut = reinterpret_cast<float*>(lds_b + Gm::lut_off);
  if (threadIdx.x < 8) {
    const float lv[4] = {-3.3359f, -1.0f, 1.0f, 3.3359f};
    lut[threadIdx.x] = threadIdx.x < 4 ? lv[threadIdx.x] : 0.0f;
  }
  tw_tab = reinterpret_cast<float2*>(lds_b + Gm::tw_off);
  if constexpr (Gm::tw_mode == kTwFull)
    tw_lds_fill<N>(tw_tab, tw, threadIdx.x, blockDim.x);
  else
    tw_split_fill<N>(tw_tab, tw, threadIdx.x, blockDim.x);
  __syncthreads();
}

// A workgroup holds G frame slots of T threads and works through tasks
// (station, group of G frames): first task blockIdx.x, then gridDim.x + the
// next value of the shared counter *ctr (zero at launch), so workgroups that
// finish early take more.  The delay record and window words of the next task
// are loaded while the current one is transformed, and the level table and
// twiddles are set up once per workgroup.
// W = 0: default; W = 2: the pols of a subband share their fringe phasors;
// W = 3, 4: ask the compiler for W waves per SIMD (caps registers at 512 / W);
// W = 5: split twiddle tables (TwSplit) at every N >= 512 (the default at
// N = 4096 and 16384).
// OUT: spectrum element type (kOutF32, kOutF16, kOutF8); for the low-precision
// outputs `scale_exp` [n_sb][M][n_chan] holds the power-of-two exponents.
template <int N, int W, int OUT>
__global__ void __attribute__((amdgpu_flat_work_group_size(1, FGeom<N>::WG),
                               amdgpu_waves_per_eu(W == 3 || W == 4 ? W : W == kFstageLean ? 4 : 1)))
    k_fstage(const DevJob* __restrict__ job, const DelayRec* __restrict__ drec,
             const PhaseRec* __restrict__ prec, const float2* __restrict__ tw,
             void* __restrict__ spec, const int8_t* __restrict__ scale_exp, int nf,
             unsigned* __restrict__ ctr) {
  using F = FTask<N, W>;
  constexpr int T = F::T, E = F::E, G = F::G;
  constexpr bool kRamp = F::kRamp, kLean = F::kLean, kPrefetch = F::kPrefetch;
  static_assert(!kRamp || OUT == kOutF32, "the drift correction rewrites FP32 spectra");
  static_assert(!kLean || 2 * E <= 32, "a lean input's codes fit one 32-bit register");
  __shared__ int next_task;
  extern __shared__ float2 lds_all[];
  const DevJob& J = *job;
  const int g = threadIdx.x / T, t = threadIdx.x % T;
  const int P = J.n_pols, M = J.M, n_chan = J.n_chan, n_sb = J.n_subbands;
  const int n_groups = (nf + G - 1) / G;
  int n_flag = J.n_stations;
  if constexpr (kRamp) {
    n_flag = 0;
    for (int i = 0; i < J.n_stations; ++i) n_flag += J.st[i].rate_correct ? 1 : 0;
  }
  const int n_igroups = fstage_igroups<N, W>(J);
  const int per_station = n_groups * n_igroups;
  const int n_tasks = per_station * n_flag;

  float2* lds = lds_all + g * lds_words<N>();
  float* lut;
  float2* tw_tab;
  fstage_setup<N, W>(tw, lut, tw_tab);

  // With whole waves per frame (T >= 64) the frame index is wave-uniform: the
  // delay and phase records then come in through scalar loads, which a wave
  // does not have to order behind its own outstanding spectrum stores.
  auto frame_of = [&](int task, int& st, int& fl, int& in) {
    if (task >= n_tasks) {   // a workgroup beyond the tasks: an empty, invalid record
      st = 0;
      fl = nf;
      in = 0;
      return;
    }
    st = task / per_station;
    int grp = task - st * per_station;
    in = 0;
    if constexpr (kLean) {
      in = grp % n_igroups;
      grp /= n_igroups;
    }
    if constexpr (kRamp) {
      in = grp % J.n_inputs;
      grp /= J.n_inputs;
      // the st-th station that asks for the correction
      for (int i = 0, k = -1; i < J.n_stations; ++i) {
        k += J.st[i].rate_correct ? 1 : 0;
        if (k == st && J.st[i].rate_correct) {
          st = i;
          break;
        }
      }
    }
    fl = grp * G + g;
    if (T >= 64) fl = __builtin_amdgcn_readfirstlane(fl);
  };
  auto record_of = [&](int st, int fl) {
    DelayRec r;
    if (fl < nf) {
      r = drec[(size_t)st * nf + fl];
    } else {
      r.valid = 0;
      r.d = 0.0;
      r.base = 0;
    }
    return r;
  };

  int task = blockIdx.x;
  int s = 0, fl = 0, in_t = 0;
  frame_of(task, s, fl, in_t);
  DelayRec r = record_of(s, fl);
  uint32_t wv[E];
  int sh0;
  load_window<N>(J, s, r, t, wv, sh0);

  while (task < n_tasks) {
    if (threadIdx.x == 0) next_task = (int)gridDim.x + (int)atomicAdd(ctr, 1u);
    __syncthreads();
    const int task_n = next_task;   // rewritten only after the input loop's barriers
    int s_n = 0, fl_n = nf, in_n = 0;
    if (task_n < n_tasks) frame_of(task_n, s_n, fl_n, in_n);
    const DelayRec r_n = record_of(s_n, fl_n);
    uint32_t wv_n[kPrefetch ? E : 1];
    int sh0_n = 0;
    if constexpr (kPrefetch) load_window<N>(J, s_n, r_n, t, wv_n, sh0_n);

    fstage_task<N, W, OUT>(J, P, M, n_chan, n_sb, prec, spec, scale_exp, nf, s, fl, in_t, r, wv,
                           sh0, lds, lut, tw_tab, t);

    task = task_n;
    s = s_n;
    fl = fl_n;
    in_t = in_n;
    r = r_n;
    if constexpr (kPrefetch) {
      sh0 = sh0_n;
#pragma unroll
      for (int e = 0; e < E; ++e) wv[e] = wv_n[e];
    } else {
      load_window<N>(J, s, r, t, wv, sh0);
    }
  }
}

// ---------------------------------------------------------------- fused batches
// One F-stage launch over the blocks of many jobs of one FFT length (a round
// of a fused batch): the tasks of item i (one job's block) are numbered from
// items[i].task0, and a workgroup's next task may belong to any item.  Each
// task runs exactly as in k_fstage (same variant, same arithmetic), so a job's
// spectra do not depend on what else shares the launch.
template <int N, int W>
__global__ void __attribute__((amdgpu_flat_work_group_size(1, FGeom<N>::WG),
                               amdgpu_waves_per_eu(W == kFstageLean ? 4 : 1)))
    k_fstage_fused(const FusedItem* __restrict__ items_g, int n_items, int n_tasks,
                   const float2* __restrict__ tw, unsigned* __restrict__ ctr) {
  using F = FTask<N, W>;
  constexpr int T = F::T, E = F::E, G = F::G;
  constexpr bool kLean = F::kLean, kPrefetch = F::kPrefetch;
  static_assert(W == 0 || W == kFstageLean || W == kFstageShare, "fused F-stage variants");
  __shared__ int next_task;
  extern __shared__ float2 lds_all[];
  const FusedItemsK items = fused_const(items_g);
  const int g = threadIdx.x / T, t = threadIdx.x % T;
  float2* lds = lds_all + g * lds_words<N>();
  float* lut;
  float2* tw_tab;
  fstage_setup<N, W>(tw, lut, tw_tab);
  // item it's job descriptor (constant data)
  auto job_of = [&](int it) -> const DevJob& { return *(const DevJob*)&items[it].jd; };

  // task -> (item, station, frame, input group); beyond the tasks: item 0 with
  // an empty, invalid record
  auto locate = [&](int task, int& it, int& st, int& fl, int& in) {
    if (task >= n_tasks) {
      it = 0;
      st = 0;
      fl = items[0].nf;
      in = 0;
      return;
    }
    int lo = 0, hi = n_items - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (items[mid].task0 <= task)
        lo = mid;
      else
        hi = mid - 1;
    }
    it = lo;
    const int nf = items[it].nf;
    const int n_ig = fstage_igroups<N, W>(job_of(it));
    const int per_station = ((nf + G - 1) / G) * n_ig;
    const int local = task - items[it].task0;
    st = local / per_station;
    int grp = local - st * per_station;
    in = 0;
    if constexpr (kLean) {
      in = grp % n_ig;
      grp /= n_ig;
    }
    fl = grp * G + g;
    if (T >= 64) fl = __builtin_amdgcn_readfirstlane(fl);
  };
  auto record_of = [&](int it, int st, int fl) {
    DelayRec r;
    const int nf = items[it].nf;
    if (fl < nf) {
      r = items[it].drec[(size_t)st * nf + fl];
    } else {
      r.valid = 0;
      r.d = 0.0;
      r.base = 0;
    }
    return r;
  };

  int task = blockIdx.x;
  int it = 0, s = 0, fl = 0, in_t = 0;
  locate(task, it, s, fl, in_t);
  DelayRec r = record_of(it, s, fl);
  uint32_t wv[E];
  int sh0;
  load_window<N>(job_of(it), s, r, t, wv, sh0);

  while (task < n_tasks) {
    if (threadIdx.x == 0) next_task = (int)gridDim.x + (int)atomicAdd(ctr, 1u);
    __syncthreads();
    // the same value in every thread: kept in scalar registers, so that the
    // item lookup and the item's fields are scalar too
    const int task_n = __builtin_amdgcn_readfirstlane(next_task);
    int it_n = 0, s_n = 0, fl_n = 0, in_n = 0;
    locate(task_n, it_n, s_n, fl_n, in_n);
    const DelayRec r_n = record_of(it_n, s_n, fl_n);
    uint32_t wv_n[kPrefetch ? E : 1];
    int sh0_n = 0;
    if constexpr (kPrefetch) load_window<N>(job_of(it_n), s_n, r_n, t, wv_n, sh0_n);

    {
      const DevJob& J = job_of(it);
      fstage_task<N, W, kOutF32>(J, J.n_pols, J.M, J.n_chan, J.n_subbands, items[it].prec,
                                 items[it].spec, nullptr, items[it].nf, s, fl, in_t, r, wv, sh0,
                                 lds, lut, tw_tab, t);
    }

    task = task_n;
    it = it_n;
    s = s_n;
    fl = fl_n;
    in_t = in_n;
    r = r_n;
    if constexpr (kPrefetch) {
      sh0 = sh0_n;
#pragma unroll
      for (int e = 0; e < E; ++e) wv[e] = wv_n[e];
    } else {
      load_window<N>(job_of(it), s, r, t, wv, sh0);
    }
  }
}

template <int N, int W, int OUT>
static hipError_t launch_nw(const DevJob* job, int n_stations, const DelayRec* drec,
                            const PhaseRec* prec, const float2* tw, void* spec,
                            const int8_t* scale_exp, int nf, unsigned* ctr, hipStream_t s) {
  using Gm = FGeom<N, fstage_twm<N, W>()>;
  // per device: LDS attribute set, and how many workgroups fill the GPU (set
  // once; callers on several host threads may race to set the same value)
  static std::atomic<int> resident[64];
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= 64) return hipErrorInvalidDevice;
  int res = resident[dev].load();
  if (!res) {
    e = hipFuncSetAttribute((const void*)k_fstage<N, W, OUT>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)Gm::lds_bytes);
    int per_cu = 0, n_cu = 0;
    if (e == hipSuccess)
      e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_fstage<N, W, OUT>, Gm::WG,
                                                       Gm::lds_bytes);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess) return e;
    res = (per_cu > 0 ? per_cu : 1) * (n_cu > 0 ? n_cu : 1);
    resident[dev].store(res);
  }
  const long tasks = (long)((nf + Gm::G - 1) / Gm::G) * n_stations;
  const int grid = (int)(tasks < res ? tasks : res);
  hipLaunchKernelGGL((k_fstage<N, W, OUT>), dim3(grid), dim3(Gm::WG), Gm::lds_bytes, s, job, drec,
                     prec, tw, spec, scale_exp, nf, ctr);
  return hipGetLastError();
}

// Lean tasks per frame group: one per group of up to kLeanGroup inputs of each
// station (what launch_nw sizes the grid by in place of the station count).
static inline int lean_units(int n_stations, int n_inputs) {
  return n_stations * ((n_inputs + kLeanGroup - 1) / kLeanGroup);
}

template <int N, int OUT>
static hipError_t launch_lp(const DevJob* job, int n_stations, int n_inputs, const DelayRec* drec,
                            const PhaseRec* prec, const float2* tw, void* spec,
                            const int8_t* scale_exp, int nf, int waves, unsigned* ctr,
                            hipStream_t s) {
  if (waves == 5)
    return launch_nw<N, 5, OUT>(job, n_stations, drec, prec, tw, spec, scale_exp, nf, ctr, s);
  if (waves == kFstageLean)
    return launch_nw<N, kFstageLean, OUT>(job, lean_units(n_stations, n_inputs), drec, prec, tw,
                                          spec, scale_exp, nf, ctr, s);
  return launch_nw<N, 0, OUT>(job, n_stations, drec, prec, tw, spec, scale_exp, nf, ctr, s);
}

template <int N>
static hipError_t launch_n(const DevJob* job, int n_stations, int n_inputs, const DelayRec* drec,
                           const PhaseRec* prec, const float2* tw, void* spec,
                           const int8_t* scale_exp, int nf, int waves, int out, unsigned* ctr,
                           hipStream_t s) {
  // the default: lean tasks where the transform is large enough for them to pay
  // (measured on MI355X, F stage of C4-shaped jobs: -15 % at N = 8192, -13 % at
  // 16384; at 4096 -3 % there but +1.5 % over a mix of uneven jobs; +3 % at 2048)
  if (waves == 0 && N >= kLeanMinN) waves = kFstageLean;
  if (out == kOutF16)
    return launch_lp<N, kOutF16>(job, n_stations, n_inputs, drec, prec, tw, spec, scale_exp, nf,
                                 waves, ctr, s);
  if (out == kOutF8)
    return launch_lp<N, kOutF8>(job, n_stations, n_inputs, drec, prec, tw, spec, scale_exp, nf,
                                waves, ctr, s);
  switch (waves) {
    case 2:
      return launch_nw<N, 2, kOutF32>(job, n_stations, drec, prec, tw, spec, nullptr, nf, ctr, s);
    case 3:
      return launch_nw<N, 3, kOutF32>(job, n_stations, drec, prec, tw, spec, nullptr, nf, ctr, s);
    case 4:
      return launch_nw<N, 4, kOutF32>(job, n_stations, drec, prec, tw, spec, nullptr, nf, ctr, s);
    case 5:
      return launch_nw<N, 5, kOutF32>(job, n_stations, drec, prec, tw, spec, nullptr, nf, ctr, s);
    case kFstageShare:
      return launch_nw<N, kFstageShare, kOutF32>(job, n_stations, drec, prec, tw, spec, nullptr,
                                                 nf, ctr, s);
    case kFstageLean:
      return launch_nw<N, kFstageLean, kOutF32>(job, lean_units(n_stations, n_inputs), drec, prec,
                                                tw, spec, nullptr, nf, ctr, s);
    case kFstageRatePass:
      if constexpr (N <= kMaxRateCorrectN)
        return launch_nw<N, kFstageRatePass, kOutF32>(job, n_stations, drec, prec, tw, spec,
                                                      nullptr, nf, ctr, s);
      return hipErrorInvalidValue;
    default:
      return launch_nw<N, 0, kOutF32>(job, n_stations, drec, prec, tw, spec, nullptr, nf, ctr, s);
  }
}

// ---------------------------------------------------------------- N = 32768
// Too large for one workgroup's LDS, N = 32768 = 16 x 2048 runs as a
// four-step FFT through a scratch buffer Z.  Sample n = n2 + 2048 n1
// (n1 < 16, n2 < 2048); bin k = k1 + 16 k2.
//   A: per (station, frame, input) and n2: unpack, fringe rotation, the
//      16-point DFT over n1, times exp(-2 pi i n2 k1 / N), into Z row k1;
//   B: per row k1, the 2048-point FFT over n2 gives bins k1 + 16 k2; the kept
//      half (k2 < 1024) is multiplied by the fractional-delay phasor and stored.
constexpr int kBigN = 32768, kBigN2 = 2048, kBigChunk = 256;

__global__ void __launch_bounds__(kBigChunk)
    k_fbig_a(const DevJob* __restrict__ job, const DelayRec* __restrict__ drec,
             const PhaseRec* __restrict__ prec, const float2* __restrict__ tw,
             float2* __restrict__ Z, int nf) {
  const DevJob& J = *job;
  const int n2 = blockIdx.x * kBigChunk + threadIdx.x;
  const int fl = blockIdx.y, s = blockIdx.z;
  const DelayRec r = drec[(size_t)s * nf + fl];
  const bool valid = r.valid != 0;
  uint32_t wv[16];
  int sh0 = 0;
  if (valid) {
    const FrameCursor c = make_cursor(J, r.base);
    const uint32_t* words = J.st[s].words;
#pragma unroll
    for (int e = 0; e < 16; ++e) wv[e] = *sample_word(J, words, c, n2 + e * kBigN2);
    sh0 = sample_shift(J, c, n2);
  }
  const int P = J.n_pols, n_sb = J.n_subbands;
  const double nc0 = (double)(n2 - kBigN / 2);
  constexpr double TD = (double)kBigN2;
  float2* zrow0 = Z + (((size_t)s * nf + fl) * J.n_inputs) * kBigN;
  for (int in = 0; in < J.n_inputs; ++in) {
    const int sb = in / P;
    const int sh = sh0 + 2 * J.stream_map[in];
    const PhaseRec ph = prec[((size_t)s * n_sb + sb) * nf + fl];
    const float2 rho = phasor_turns(frac_f(2.0 * ph.phi2 * TD * TD));
    float2 v[16];
    float2 z = make_float2(1.f, 0.f), w = make_float2(1.f, 0.f);
#pragma unroll
    for (int e = 0; e < 16; ++e) {
      if (e % 8 == 0) {
        const double nc = nc0 + (double)e * TD;
        z = phasor_turns(frac_f(fma(fma(ph.phi2, nc, ph.phi1), nc, ph.phi0)));
        w = phasor_turns(frac_f(ph.phi1 * TD + ph.phi2 * TD * (2.0 * nc + TD)));
      } else {
        z = cmul(z, w);
        w = cmul(w, rho);
      }
      const float q = valid ? level_of((wv[e] >> sh) & 3u) : 0.0f;
      v[e] = make_float2(q * z.x, q * z.y);
    }
    Dft<16>::run(v);
    float2* zr = zrow0 + (size_t)in * kBigN;
#pragma unroll
    for (int k1 = 0; k1 < 16; ++k1) {
      const float2 y = k1 == 0 ? v[0] : cmul(v[k1], tw[n2 * k1]);   // n2 k1 < kTwiddleN
      zr[k1 * kBigN2 + n2] = y;
    }
  }
}

constexpr int kBigRowIters = 8;   // row groups per k_fbig_b workgroup

template <int OUT>
__global__ void __launch_bounds__(256)
    k_fbig_b(const DevJob* __restrict__ job, const DelayRec* __restrict__ drec,
             const float2* __restrict__ tw, const float2* __restrict__ Z,
             void* __restrict__ spec, const int8_t* __restrict__ scale_exp, int nf) {
  static_assert(OUT != kOutF32, "FP32 spectra at N = 32768 come from k_fhalf");
  constexpr int T = FftPlan<kBigN2>::T, E = FftPlan<kBigN2>::E;
  constexpr int G = 256 / T;
  extern __shared__ float2 lds_all[];
  // G exchange buffers, then the twiddle tables (filled once, used for
  // kBigRowIters groups of G rows)
  float2* tw_tab = lds_all + G * lds_words<kBigN2>();
  tw_lds_fill<kBigN2>(tw_tab, tw, threadIdx.x, blockDim.x);
  const DevJob& J = *job;
  const int g = threadIdx.x / T, t = threadIdx.x % T;
  const int P = J.n_pols, M = J.M, n_chan = J.n_chan;
  // row = ((s nf + fl) n_inputs + in) 16 + k1
  const long n_rows = (long)J.n_stations * nf * J.n_inputs * 16;
  for (int it = 0; it < kBigRowIters; ++it) {
    __syncthreads();   // tables written / the previous group's exchange done
    const long row = ((long)blockIdx.x * kBigRowIters + it) * G + g;
    const bool live = row < n_rows;
    const long rr = live ? row : 0;
    const int k1 = (int)(rr % 16);
    const int in = (int)((rr / 16) % J.n_inputs);
    const long sf = rr / (16L * J.n_inputs);
    const int fl = (int)(sf % nf), s = (int)(sf / nf);
    const float2* x = Z + rr * kBigN2;
    float2 v[E];
#pragma unroll
    for (int e = 0; e < E; ++e) v[e] = x[t + e * T];
    fft_forward<kBigN2>(v, lds_all + g * lds_words<kBigN2>(), TwLds<kBigN2>{tw_tab}, t);
    if (!live) continue;
    const DelayRec r = drec[(size_t)s * nf + fl];
    const bool valid = r.valid != 0;
    const float dd = (float)r.d;
    const int sb = in / P, p = in - sb * P;
    const int8_t* ex = scale_exp + ((size_t)sb * M + (s * P + p)) * n_chan;
    // v[r] = X[k1 + 16 k2] with k2 = t + r T; the kept half is k2 < 1024 (r < 8)
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int k = k1 + 16 * (t + q * T);
      const float2 fd = phasor_turns((float)k * dd * (1.0f / (float)kBigN));
      const float2 y = valid ? cmul(v[q], fd) : make_float2(0.f, 0.f);
      put_spec<OUT, false>(spec, lp_index((size_t)sb * nf + fl, s * P + p, k, M, n_chan), y,
                           (int)ex[scale_pos(k, n_chan)]);
    }
  }
}

// ---------------------------------------------------------------- N = 32768, two folded halves
// The kept half of a 32768-point frame (channels < 16384) without scratch
// memory, as two 16384-point transforms.  With W = exp(-2 pi i / 32768),
//   X[2k + h] = sum_{n < 16384} (y_h[n] + y_h[n + 16384]) exp(-2 pi i k n / 16384),
//   y_h[n] = x[n] W^(h n),
// and x[n] W^(h n) is the sample rotated by the fringe phase less h n / 32768
// turns: pass h (0, 1) rotates with phi0 - h / 2 and phi1 - h / 32768 (about the
// frame centre), folds the frame's two halves and transforms them in the
// one-workgroup FFT of N = 16384, whose kept bins k < 8192 are channels 2k + h.
// Tasks are (station, frame, group of up to kHalfGroup inputs), the group's
// codes packed as in the lean F stage (two registers per input).  FP32 spectra.
constexpr int kHalfN = kBigN / 2;
constexpr int kHalfGroup = kLeanGroup;   // inputs per task (2 or 1: hardly fewer spills)

__global__ void __attribute__((amdgpu_flat_work_group_size(1, FftPlan<kHalfN>::T)))
    k_fhalf(const DevJob* __restrict__ job, const DelayRec* __restrict__ drec,
            const PhaseRec* __restrict__ prec, const float2* __restrict__ tw,
            float2* __restrict__ spec, int nf, unsigned* __restrict__ ctr) {
  using Gm = FGeom<kHalfN, kTwSplit>;
  constexpr int T = Gm::T, E = Gm::E;
  static_assert(Gm::G == 1 && 2 * E <= 32, "one frame per workgroup, codes in 32 bits");
  __shared__ int next_task;
  extern __shared__ float2 lds_all[];
  const DevJob& J = *job;
  const int t = threadIdx.x;
  const int P = J.n_pols, M = J.M, n_chan = J.n_chan, n_sb = J.n_subbands;
  const int n_ig = (J.n_inputs + kHalfGroup - 1) / kHalfGroup;
  const int per_station = nf * n_ig;
  const int n_tasks = per_station * J.n_stations;
  unsigned char* lds_b = reinterpret_cast<unsigned char*>(lds_all);
  float* lut = reinterpret_cast<float*>(lds_b + Gm::lut_off);
  if (t < 8) {
    const float lv[4] = {-3.3359f, -1.0f, 1.0f, 3.3359f};
    lut[t] = t < 4 ? lv[t] : 0.0f;
  }
  float2* tw_tab = reinterpret_cast<float2*>(lds_b + Gm::tw_off);
  tw_split_fill<kHalfN>(tw_tab, tw, t, blockDim.x);
  __syncthreads();
  constexpr double TD = (double)T;

  int task = blockIdx.x;
  while (task < n_tasks) {
    const int s = task / per_station;
    const int rem = task - s * per_station;
    const int fl = __builtin_amdgcn_readfirstlane(rem / n_ig);
    const int in_lo = (rem - fl * n_ig) * kHalfGroup;
    const int in_hi = min(in_lo + kHalfGroup, J.n_inputs);
    const DelayRec r = drec[(size_t)s * nf + fl];
    const bool valid = r.valid != 0;
    const float* lut_t = lut + (valid ? 0 : 4);
    // the group's codes of samples t + e T (lo) and 16384 + t + e T (hi)
    uint32_t c_lo[kHalfGroup], c_hi[kHalfGroup];
    {
      // one half of the window at a time (16 words in flight)
      FrameCursor c;
      int sh0 = 0;
      if (valid) {
        c = make_cursor(J, r.base);
        sh0 = sample_shift(J, c, t);   // 16384 is a whole number of words
      }
      auto pack = [&](int off, uint32_t (&dst)[kHalfGroup]) {
        uint32_t w[E];
        if (valid) {
          const uint32_t* words = J.st[s].words;
#pragma unroll
          for (int e = 0; e < E; ++e) w[e] = *sample_word(J, words, c, off + t + e * T);
        } else {
#pragma unroll
          for (int e = 0; e < E; ++e) w[e] = 0u;
        }
#pragma unroll
        for (int i = 0; i < kHalfGroup; ++i) {
          const int sh = sh0 + 2 * J.stream_map[min(in_lo + i, in_hi - 1)];
          uint32_t a = 0;
#pragma unroll
          for (int e = 0; e < E; ++e) a |= ((w[e] >> sh) & 3u) << (2 * e);
          dst[i] = a;
        }
      };
      pack(0, c_lo);
      pack(kHalfN, c_hi);
    }
    const float dd = (float)r.d;
    const float2 fd_st = phasor_turns(dd * (1.0f / 16.0f));   // 2048 channels on
#pragma unroll 1
    for (int in = in_lo; in < in_hi; ++in) {
      const int sb = in / P, p = in - sb * P;
      const int i = in - in_lo;
      uint32_t cl = c_lo[0], ch = c_hi[0];
#pragma unroll
      for (int j = 1; j < kHalfGroup; ++j) {
        cl = i == j ? c_lo[j] : cl;
        ch = i == j ? c_hi[j] : ch;
      }
      const PhaseRec ph = prec[((size_t)s * n_sb + sb) * nf + fl];
      float2* row = spec + ((size_t)(sb * nf + fl) * M + (s * P + p)) * n_chan;
#pragma unroll 1
      for (int h = 0; h < 2; ++h) {
        const double phi0 = ph.phi0 - 0.5 * h, phi1 = ph.phi1 - (double)h / (double)kBigN;
        const double phi2 = ph.phi2;
        // centred index of sample n is n - 16384: t - 16384 + e T (lo), t + e T (hi);
        // exact phasors every 8 samples where the quadratic term matters, else once
        const bool quad = fabs(phi2) * TD * TD * (double)(E * (E - 1)) > 1e-8;
        // the thread index through an empty asm: the anchors' FP64 sample
        // positions below are recomputed here rather than hoisted out of the
        // loops and kept in scratch (the 1024-thread workgroup leaves 128
        // registers)
        int tq = t;
        __asm__ volatile("" : "+v"(tq));
        float2 v[E];
        auto anchor = [&](double nc, float2& z, float2& w) {
          z = phasor_turns(frac_f(fma(fma(phi2, nc, phi1), nc, phi0)));
          w = phasor_turns(frac_f(phi1 * TD + phi2 * TD * (2.0 * nc + TD)));
        };
        auto sample = [&](int e, float2 zl, float2 zh) {
          const float ql = lut_t[(cl >> (2 * e)) & 3u], qh = lut_t[(ch >> (2 * e)) & 3u];
          v[e] = make_float2(fmaf(ql, zl.x, qh * zh.x), fmaf(ql, zl.y, qh * zh.y));
        };
        float2 zl, wl, zh, wh;
        if (quad) {
          const float2 rho = phasor_turns(frac_f(2.0 * phi2 * TD * TD));
#pragma unroll
          for (int e = 0; e < E; ++e) {
            if (e % 8 == 0) {
              anchor((double)(tq - kHalfN) + (double)e * TD, zl, wl);
              anchor((double)tq + (double)e * TD, zh, wh);
            } else {
              zl = cmul(zl, wl);
              zh = cmul(zh, wh);
              wl = cmul(wl, rho);
              wh = cmul(wh, rho);
            }
            sample(e, zl, zh);
          }
        } else {
          anchor((double)(tq - kHalfN), zl, wl);
          anchor((double)tq, zh, wh);
#pragma unroll
          for (int e = 0; e < E; ++e) {
            if (e > 0) {
              zl = cmul(zl, wl);
              zh = cmul(zh, wh);
            }
            sample(e, zl, zh);
          }
        }
        fft_forward<kHalfN>(v, lds_all, TwSplit<kHalfN>{tw_tab}, t);
        // v[q] = bin t + q T of the folded transform; the kept bins (q < 8) are
        // channels 2 (t + q T) + h, whose fractional-delay phasor is
        // exp(2 pi i (2 (t + q T) + h) d / 32768)
        float2 fdr = phasor_turns((float)(2 * t + h) * dd * (1.0f / (float)kBigN));
#pragma unroll
        for (int q = 0; q < 8; ++q) {
          if (q > 0) fdr = cmul(fdr, fd_st);
          const float2 y = valid ? cmul(v[q], fdr) : make_float2(0.f, 0.f);
          put_spec<kOutF32, false>(row, (size_t)(2 * (t + q * T) + h), y, 0);
        }
        __syncthreads();   // the next pass reuses lds
      }
    }
    if (t == 0) next_task = (int)gridDim.x + (int)atomicAdd(ctr, 1u);
    __syncthreads();
    task = next_task;
  }
}

static hipError_t launch_half(const DevJob* job, int n_stations, int n_inputs,
                              const DelayRec* drec, const PhaseRec* prec, const float2* tw,
                              float2* spec, int nf, unsigned* ctr, hipStream_t s) {
  using Gm = FGeom<kHalfN, kTwSplit>;
  static std::atomic<int> resident[64];
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= 64) return hipErrorInvalidDevice;
  int res = resident[dev].load();
  if (!res) {
    e = hipFuncSetAttribute((const void*)k_fhalf, hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)Gm::lds_bytes);
    int per_cu = 0, n_cu = 0;
    if (e == hipSuccess)
      e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_fhalf, Gm::WG, Gm::lds_bytes);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess) return e;
    res = (per_cu > 0 ? per_cu : 1) * (n_cu > 0 ? n_cu : 1);
    resident[dev].store(res);
  }
  const long tasks = (long)nf * n_stations * ((n_inputs + kHalfGroup - 1) / kHalfGroup);
  const int grid = (int)(tasks < res ? tasks : res);
  hipLaunchKernelGGL(k_fhalf, dim3(grid), dim3(Gm::WG), Gm::lds_bytes, s, job, drec, prec, tw,
                     spec, nf, ctr);
  return hipGetLastError();
}

size_t fstage_scratch_bytes(int N, int n_stations, int n_inputs, int nf, int out) {
  // the four-step path's rows (the FP32 path folds its halves instead)
  return N == kBigN && out != kOutF32 ? (size_t)n_stations * nf * n_inputs * kBigN * sizeof(float2)
                                      : 0;
}

static hipError_t launch_big(const DevJob* job, int n_stations, int n_inputs,
                             const DelayRec* drec, const PhaseRec* prec, const float2* tw,
                             void* spec, const int8_t* scale_exp, int nf, int out, float2* Z,
                             hipStream_t s) {
  if (!Z) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_fbig_a, dim3(kBigN2 / kBigChunk, nf, n_stations), dim3(kBigChunk), 0, s,
                     job, drec, prec, tw, Z, nf);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  constexpr int G = 256 / FftPlan<kBigN2>::T;
  const size_t lds =
      ((size_t)G * lds_words<kBigN2>() + (size_t)tw_lds_entries<kBigN2>()) * sizeof(float2);
  const long rows = (long)n_stations * nf * n_inputs * 16;
  const long per_wg = (long)G * kBigRowIters;
  const dim3 grid((unsigned)((rows + per_wg - 1) / per_wg));
  if (out == kOutF16)
    hipLaunchKernelGGL(k_fbig_b<kOutF16>, grid, dim3(256), lds, s, job, drec, tw, Z, spec,
                       scale_exp, nf);
  else if (out == kOutF8)
    hipLaunchKernelGGL(k_fbig_b<kOutF8>, grid, dim3(256), lds, s, job, drec, tw, Z, spec,
                       scale_exp, nf);
  else
    return hipErrorInvalidValue;   // FP32 spectra fold the frame instead (k_fhalf)
  return hipGetLastError();
}

// ---------------------------------------------------------------- fused batch launchers
template <int N, int W>
static hipError_t launch_fused_nw(const FusedItem* items, int n_items, int n_tasks,
                                  const float2* tw, unsigned* ctr, hipStream_t s) {
  using Gm = typename FTask<N, W>::Gm;
  static std::atomic<int> resident[64];
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= 64) return hipErrorInvalidDevice;
  int res = resident[dev].load();
  if (!res) {
    e = hipFuncSetAttribute((const void*)k_fstage_fused<N, W>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)Gm::lds_bytes);
    int per_cu = 0, n_cu = 0;
    if (e == hipSuccess)
      e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_fstage_fused<N, W>, Gm::WG,
                                                       Gm::lds_bytes);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess) return e;
    res = (per_cu > 0 ? per_cu : 1) * (n_cu > 0 ? n_cu : 1);
    resident[dev].store(res);
  }
  if (n_tasks <= 0) return hipSuccess;
  const int grid = n_tasks < res ? n_tasks : res;
  hipLaunchKernelGGL((k_fstage_fused<N, W>), dim3(grid), dim3(Gm::WG), Gm::lds_bytes, s, items,
                     n_items, n_tasks, tw, ctr);
  return hipGetLastError();
}

template <int N>
static hipError_t launch_fused_n(int waves, const FusedItem* items, int n_items, int n_tasks,
                                 const float2* tw, unsigned* ctr, hipStream_t s) {
  if (waves == kFstageLean)
    return launch_fused_nw<N, kFstageLean>(items, n_items, n_tasks, tw, ctr, s);
  if (waves == kFstageShare)
    return launch_fused_nw<N, kFstageShare>(items, n_items, n_tasks, tw, ctr, s);
  if (waves == 0 && N < kLeanMinN)
    return launch_fused_nw<N, 0>(items, n_items, n_tasks, tw, ctr, s);
  return hipErrorInvalidValue;
}

int fstage_fused_variant(int N, int n_pols, int n_chan) {
  const int w = fstage_variant(0, n_pols, n_chan, kOutF32);
  // variant 2's fused form is kFstageShare (the same arithmetic)
  if (w == 2) return kFstageShare;
  return w == 0 && N >= kLeanMinN ? kFstageLean : w;
}

static_assert(FGeom<2048>::T == 2048 / 16 && FGeom<2048>::G == 2 && FGeom<8192>::G == 1,
              "fstage_fused_tasks mirrors FGeom");

int fstage_fused_tasks(int N, int waves, int n_stations, int n_inputs, int nf) {
  const int T = N / 16;                   // threads per frame (FftPlan<N>: 16 values each)
  const int G = T >= 256 ? 1 : 256 / T;   // frames per workgroup (FGeom<N>::G)
  const int groups = (nf + G - 1) / G;
  const int ig = waves == kFstageLean ? (n_inputs + kLeanGroup - 1) / kLeanGroup : 1;
  return n_stations * groups * ig;
}

hipError_t launch_fstage_fused(int N, int waves, const FusedItem* items, int n_items,
                               int n_tasks, const float2* tw, unsigned* ctr, hipStream_t s) {
  switch (N) {
#define XC_FFCASE(NN) \
  case NN: return launch_fused_n<NN>(waves, items, n_items, n_tasks, tw, ctr, s);
    XC_FFCASE(256) XC_FFCASE(512) XC_FFCASE(1024) XC_FFCASE(2048) XC_FFCASE(4096) XC_FFCASE(8192)
    XC_FFCASE(16384)
#undef XC_FFCASE
    default: return hipErrorInvalidValue;
  }
}

bool fstage_supported(int N) {
  switch (N) {
    case 256: case 512: case 1024: case 2048: case 4096: case 8192: case 16384: case 32768:
      return true;
    default: return false;
  }
}

hipError_t launch_fstage(int N, const DevJob* job, int n_stations, int n_inputs,
                         const DelayRec* drec, const PhaseRec* prec, const float2* tw,
                         void* spec, const int8_t* scale_exp, int nf, int waves, int out,
                         unsigned* ctr, float2* scratch, hipStream_t s) {
  if (N == kBigN) {
    if (out == kOutF32) {
      if (!ctr) return hipErrorInvalidValue;
      return launch_half(job, n_stations, n_inputs, drec, prec, tw, static_cast<float2*>(spec),
                         nf, ctr, s);
    }
    return launch_big(job, n_stations, n_inputs, drec, prec, tw, spec, scale_exp, nf, out,
                      scratch, s);
  }
  if (!ctr) return hipErrorInvalidValue;
  switch (N) {
#define XC_FCASE(NN)                                                                      \
  case NN:                                                                                \
    return launch_n<NN>(job, n_stations, n_inputs, drec, prec, tw, spec, scale_exp, nf, waves, \
                        out, ctr, s);
    XC_FCASE(256) XC_FCASE(512) XC_FCASE(1024) XC_FCASE(2048) XC_FCASE(4096) XC_FCASE(8192)
    XC_FCASE(16384)
#undef XC_FCASE
    default: return hipErrorInvalidValue;
  }
}

}  // namespace xc
