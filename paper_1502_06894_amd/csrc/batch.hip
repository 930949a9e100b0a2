// Batches (many uneven sub-integrations as one unit) and the autotuner.
#include <algorithm>
#include <map>
#include <numeric>

#include "xc_runtime.h"

using namespace xc;

namespace {

constexpr size_t kBatchSpecCap = (size_t)1 << 30;   // per-job staged spectra in a batch
// Jobs of more blocks than this run as single jobs: their own launches already
// fill the GPU block after block, and in rounds they would hold their group's
// lane for as many rounds as they have blocks.  Fusing pays for the short jobs,
// whose launches are too small to fill the GPU alone.
constexpr int kFusedMaxBlocks = 4;
constexpr int64_t kTuneFrames = 8192;               // frames an autotune candidate runs

struct Plan {
  std::vector<xc_setup> setups;          // job setups with the batch's block size
  std::vector<xc_tuning> tunes;
  std::vector<Layout> layouts;
  std::vector<size_t> desc_off;          // per job, in the descriptor region
  std::vector<int> lane_of;
  std::vector<std::vector<int>> order;   // per lane: jobs in launch order
  std::vector<size_t> arena_off;         // per lane
  std::vector<char> solo;                // per job: long, at the library's block size, lane 0
  size_t desc_bytes = 0, total = 0;
};

int64_t job_cost(const xc_setup& s) {
  return (int64_t)s.n_stations * s.n_subbands * s.n_pols * s.n_frames * 2 * s.n_chan;
}

int plan_batch(xc_ctx* c, const xc_job* jobs, int n, int lanes, Plan& P) {
  if (!jobs || n < 1) return fail(c, XC_E_INVAL, "batch: no jobs");
  if (lanes < 1 || lanes > kMaxLanes) return fail(c, XC_E_INVAL, "batch: n_lanes=%d", lanes);
  P.setups.resize(n);
  P.tunes.resize(n);
  P.layouts.resize(n);
  P.desc_off.resize(n);
  P.lane_of.assign(n, 0);
  P.solo.assign(n, 0);
  for (int j = 0; j < n; ++j) {
    int rc = validate(c, &jobs[j].setup, jobs[j].st);
    if (rc != XC_OK) {
      if (c) c->last_error = "job " + std::to_string(j) + ": " + c->last_error;
      return rc;
    }
    if (!jobs[j].out.vis || !jobs[j].out.weight)
      return fail(c, XC_E_INVAL, "job %d: output is NULL", j);
    xc_setup s = jobs[j].setup;
    xc_tuning tu = effective_tuning(c, &s);
    Layout L = layout_of(&s, jobs[j].st, tu);
    // bound each job's staged spectra so that many jobs fit in HBM together;
    // a job that the bound would cut into more than kFusedMaxBlocks blocks
    // keeps the library's (larger) default block instead and runs alone on
    // lane 0, after or before the other long jobs: it fills the GPU by itself,
    // and its rounds cost as little as when it runs outside a batch
    if (s.frames_per_block == 0) {
      const int T = shared_block_frames(s, L, kBatchSpecCap, 64);
      if (T != L.T) {
        if ((s.n_frames + T - 1) / T > kFusedMaxBlocks) {
          P.solo[j] = 1;
        } else {
          s.frames_per_block = T;
          L = layout_of(&s, jobs[j].st, tu);
        }
      }
    }
    P.setups[j] = s;
    P.tunes[j] = tu;
    P.layouts[j] = L;
    P.desc_off[j] = P.desc_bytes;
    P.desc_bytes += align_up(L.desc_bytes);
  }
  // longest processing time first: each job goes to the least loaded lane
  std::vector<int> idx(n);
  std::iota(idx.begin(), idx.end(), 0);
  std::stable_sort(idx.begin(), idx.end(), [&](int a, int b) {
    return job_cost(P.setups[a]) > job_cost(P.setups[b]);
  });
  std::vector<int64_t> load(lanes, 0);
  std::vector<size_t> arena(lanes, 0);
  P.order.assign(lanes, {});
  std::stable_partition(idx.begin(), idx.end(), [&](int j) { return P.solo[j] != 0; });
  for (int j : idx) {
    const int l = P.solo[j] ? 0 : (int)(std::min_element(load.begin(), load.end()) - load.begin());
    load[l] += job_cost(P.setups[j]);
    P.lane_of[j] = l;
    P.order[l].push_back(j);
    arena[l] = std::max(arena[l], align_up(P.layouts[j].total));
  }
  P.arena_off.resize(lanes);
  size_t off = align_up(P.desc_bytes);
  for (int l = 0; l < lanes; ++l) {
    P.arena_off[l] = off;
    off += arena[l];
  }
  P.total = off;
  return XC_OK;
}

uint64_t fnv(uint64_t h, const void* p, size_t n) {
  const unsigned char* b = static_cast<const unsigned char*>(p);
  for (size_t i = 0; i < n; ++i) h = (h ^ b[i]) * 0x100000001b3ull;
  return h;
}

// Everything a captured batch bakes in: shapes, pointers, lanes, tunings and
// descriptor contents.
uint64_t batch_key(const xc_job* jobs, int n, int lanes, const Plan& P, const void* ws) {
  uint64_t h = 0xcbf29ce484222325ull;
  h = fnv(h, &n, sizeof n);
  h = fnv(h, &lanes, sizeof lanes);
  h = fnv(h, &ws, sizeof ws);
  for (int j = 0; j < n; ++j) {
    const xc_setup& s = P.setups[j];
    h = fnv(h, &s.n_stations, 5 * sizeof(int32_t));
    h = fnv(h, s.stream_map, sizeof(int32_t) * s.n_subbands * s.n_pols);
    h = fnv(h, &s.fs_hz, sizeof s.fs_hz);
    h = fnv(h, s.lo_hz, sizeof(double) * s.n_subbands);
    h = fnv(h, &s.sub_start, 2 * sizeof(int64_t));
    h = fnv(h, &s.precision, 2 * sizeof(int32_t));
    h = fnv(h, &P.tunes[j], sizeof(xc_tuning));
    h = fnv(h, &jobs[j].out, sizeof(xc_output));
    for (int i = 0; i < s.n_stations; ++i) {
      const xc_station& st = jobs[j].st[i];
      h = fnv(h, &st.frames, sizeof st.frames);
      h = fnv(h, &st.n_frames_m5b, 2 * sizeof(int64_t));
      h = fnv(h, &st.frame_ok, sizeof st.frame_ok);
      h = fnv(h, &st.poly_deg, sizeof st.poly_deg);
      h = fnv(h, st.delay_poly, sizeof(double) * (st.poly_deg + 1));
      if (st.phase_poly)
        h = fnv(h, st.phase_poly, sizeof(double) * s.n_subbands * (st.poly_deg + 1));
    }
  }
  return h;
}

int upload_batch_desc(xc_ctx* c, const xc_job* jobs, int n, const Plan& P, unsigned char* ws,
                      hipStream_t stream) {
  hipError_t e = hipSuccess;
  if (!c->batch_ev) e = hipEventCreateWithFlags(&c->batch_ev, hipEventDisableTiming);
  if (e == hipSuccess) e = hipEventSynchronize(c->batch_ev);   // previous blob is uploaded
  if (e == hipSuccess && c->h_batch_bytes < P.desc_bytes) {
    if (c->h_batch) (void)hipHostFree(c->h_batch);
    c->h_batch = nullptr;
    c->h_batch_bytes = 0;
    e = hipHostMalloc((void**)&c->h_batch, P.desc_bytes, hipHostMallocDefault);
    if (e == hipSuccess) c->h_batch_bytes = P.desc_bytes;
  }
  if (e != hipSuccess) return hip_fail(c, e, "batch descriptors");
  for (int j = 0; j < n; ++j)
    build_desc(&P.setups[j], jobs[j].st, P.layouts[j], ws + P.desc_off[j],
               ws + P.arena_off[P.lane_of[j]], c->h_batch + P.desc_off[j]);
  e = hipMemcpyAsync(ws, c->h_batch, P.desc_bytes, hipMemcpyHostToDevice, stream);
  if (e == hipSuccess) e = hipEventRecord(c->batch_ev, stream);
  return e == hipSuccess ? XC_OK : hip_fail(c, e, "batch descriptor upload");
}

// Fork from `origin`, enqueue every lane's jobs, join back into `origin`.
int enqueue_batch(xc_ctx* c, const xc_job* jobs, const Plan& P, unsigned char* ws, int lanes,
                  hipStream_t origin) {
  hipError_t e = hipEventRecord(c->fork_ev, origin);
  for (int l = 0; l < lanes && e == hipSuccess; ++l) e = hipStreamWaitEvent(c->lanes[l], c->fork_ev, 0);
  if (e != hipSuccess) return hip_fail(c, e, "batch fork");
  for (int l = 0; l < lanes; ++l)
    for (int j : P.order[l]) {
      const DevJob* dj = reinterpret_cast<const DevJob*>(ws + P.desc_off[j]);
      int rc = enqueue_job(c, &P.setups[j], jobs[j].st, &jobs[j].out, dj, ws + P.arena_off[l],
                           P.layouts[j], P.tunes[j], c->lanes[l]);
      if (rc != XC_OK) {
        c->last_error = "job " + std::to_string(j) + ": " + c->last_error;
        return rc;
      }
    }
  for (int l = 0; l < lanes && e == hipSuccess; ++l) {
    e = hipEventRecord(c->lane_ev[l], c->lanes[l]);
    if (e == hipSuccess) e = hipStreamWaitEvent(origin, c->lane_ev[l], 0);
  }
  return e == hipSuccess ? XC_OK : hip_fail(c, e, "batch join");
}

// ---------------------------------------------------------------- fused executor
// Short jobs (at most kFusedMaxBlocks blocks) of one FFT length (and F-stage
// variant) form a group.  A group runs in rounds: round r takes block r of
// every job of the group that has one, and
// runs it as one delay, one weight, one F-stage launch (persistent over the
// tasks of all those blocks) and one X-stage launch per input-tile shape.  A
// job never has two blocks in one round, so every accumulator slot still has
// one writer per launch and a job's blocks add in block order: results are
// bit-identical to the job run alone with the same block size.  Groups run on
// lanes side by side with the long jobs and those the fused kernels do not
// take, which run as single jobs on the lanes.  One ingest (each distinct recording once), one clear of all
// accumulators and one finalise serve the whole batch.

struct XClass {
  int Mp, first, n, blocks;        // items [first, first + n) of the round, X workgroups
};

struct FRound {
  int first = 0, n = 0;            // items in the batch's item table
  int dblocks = 0, wblocks = 0, ntasks = 0;
  std::vector<XClass> xc;
};

struct FGroup {
  int N = 0, W = 0;
  std::vector<int> jobs;
  std::vector<FRound> rounds;
  size_t ctr_off = 0;              // two task counters in the workspace
  int64_t cost = 0;
};

struct FPlan {
  Plan P;                                   // setups (batch block sizes), tunings, descriptors
  std::vector<Layout> L;                    // per job: layout used by this executor
  std::vector<std::vector<xc_station>> st;  // per job: stations, frame_ok pointing at masks
  std::vector<int> group_of;                // per job: fused group, or -1 (single job)
  std::vector<FGroup> groups;
  std::vector<std::vector<int>> lane_groups, lane_jobs;
  std::vector<FusedItem> items;             // every round's items (pointers relative, see fill)
  std::vector<int> item_job;                // job of each item
  std::vector<FusedOut> outs;
  std::vector<int> out_job;
  std::vector<FusedMask> masks;
  std::vector<size_t> mask_off;             // per mask: offset of its bytes
  std::vector<std::vector<int>> st_mask;    // per job, station: mask index or -1 (caller's)
  size_t items_off = 0, outs_off = 0, masks_off = 0, blob_bytes = 0;
  size_t maskbytes_off = 0, acc_off = 0, acc_bytes = 0, ctr_off = 0;
  std::vector<size_t> vacc_off, wacc_off, blk_off, arena_off;
  int fin_blocks = 0, ingest_blocks = 0;
  size_t total = 0;
};

bool fused_job_ok(const xc_setup& s, const xc_station* st, const xc_tuning& tu, int T) {
  const int N = 2 * s.n_chan;
  if ((s.n_frames + T - 1) / T > kFusedMaxBlocks) return false;
  if (s.precision != XC_FP32 || N > 16384 || any_rate_correct(&s, st)) return false;
  if (tu.fstage_waves_per_simd != 0 || tu.xmac_tiles_per_wg != 0) return false;
  // the fused X stage is the matrix-core ring kernel, whose sums are bit-identical
  // to the vector ring's: a job tuned to either (or to the default) can join
  if (!(tu.xmac_frames_per_stage == 0 || tu.xmac_frames_per_stage == 8 ||
        tu.xmac_frames_per_stage == kXmacMatrixRing))
    return false;
  if (!(tu.xmac_channels_per_wg == 0 || tu.xmac_channels_per_wg == 64)) return false;
  return xmac_fused_ok(s.n_stations * s.n_pols, s.n_chan);
}

int plan_fused(xc_ctx* c, const xc_job* jobs, int n, int lanes, FPlan& F) {
  int rc = plan_batch(c, jobs, n, lanes, F.P);
  if (rc != XC_OK) return rc;
  const Plan& P = F.P;
  F.L.resize(n);
  F.st.resize(n);
  F.group_of.assign(n, -1);
  F.st_mask.resize(n);
  // distinct recordings without a caller mask: one mask each
  std::map<std::pair<const void*, int64_t>, int> mask_idx;
  size_t mbytes = 0;
  for (int j = 0; j < n; ++j) {
    const xc_setup& s = P.setups[j];
    F.st[j].assign(jobs[j].st, jobs[j].st + s.n_stations);
    F.st_mask[j].assign(s.n_stations, -1);
    if (P.solo[j] || !fused_job_ok(s, jobs[j].st, P.tunes[j], P.layouts[j].T)) continue;
    for (int i = 0; i < s.n_stations; ++i) {
      const xc_station& x = jobs[j].st[i];
      if (x.frame_ok) continue;
      auto key = std::make_pair(x.frames, x.n_frames_m5b);
      auto it = mask_idx.find(key);
      if (it == mask_idx.end()) {
        it = mask_idx.emplace(key, (int)F.masks.size()).first;
        FusedMask m{};
        m.words = static_cast<const uint32_t*>(x.frames);
        m.n_frames = x.n_frames_m5b;
        m.blk0 = F.ingest_blocks;
        F.ingest_blocks += ingest_fused_blocks(x.n_frames_m5b);
        F.masks.push_back(m);
        F.mask_off.push_back(mbytes);
        mbytes += align_up((size_t)x.n_frames_m5b);
      }
      F.st_mask[j][i] = it->second;
      F.st[j][i].frame_ok = reinterpret_cast<const uint8_t*>(1);   // sized as caller-supplied
    }
  }
  // groups by (FFT length, F-stage variant)
  std::map<std::pair<int, int>, int> gidx;
  for (int j = 0; j < n; ++j) {
    const xc_setup& s = P.setups[j];
    F.L[j] = layout_of(&s, F.st[j].data(), P.tunes[j]);
    if (P.solo[j] || !fused_job_ok(s, jobs[j].st, P.tunes[j], P.layouts[j].T)) continue;
    const int N = 2 * s.n_chan;
    const int W = fstage_fused_variant(N, s.n_pols, s.n_chan);
    auto key = std::make_pair(N, W);
    auto it = gidx.find(key);
    if (it == gidx.end()) {
      it = gidx.emplace(key, (int)F.groups.size()).first;
      F.groups.push_back(FGroup());
      F.groups.back().N = N;
      F.groups.back().W = W;
    }
    F.group_of[j] = it->second;
    F.groups[it->second].jobs.push_back(j);
    F.groups[it->second].cost += job_cost(s);
  }
  // A group whose work exceeds a lane's share is split (its jobs dealt
  // longest-first to the least loaded part), so that the lanes balance.
  {
    int64_t total = 0;
    for (const FGroup& g : F.groups) total += g.cost;
    for (int j = 0; j < n; ++j)
      if (F.group_of[j] < 0) total += job_cost(P.setups[j]);
    const int64_t share = (total + lanes - 1) / lanes;
    std::vector<FGroup> split;
    for (FGroup& g : F.groups) {
      const int parts = (int)std::min<int64_t>(
          (int64_t)g.jobs.size(), share > 0 ? (g.cost + share - 1) / share : 1);
      if (parts <= 1) {
        split.push_back(g);
        continue;
      }
      std::vector<int> js = g.jobs;
      std::stable_sort(js.begin(), js.end(),
                       [&](int a, int b) { return job_cost(P.setups[a]) > job_cost(P.setups[b]); });
      std::vector<FGroup> part(parts);
      for (FGroup& q : part) {
        q.N = g.N;
        q.W = g.W;
      }
      for (int j : js) {
        FGroup& q = *std::min_element(part.begin(), part.end(), [](const FGroup& a, const FGroup& b) {
          return a.cost < b.cost;
        });
        q.jobs.push_back(j);
        q.cost += job_cost(P.setups[j]);
      }
      for (FGroup& q : part) split.push_back(q);
    }
    F.groups.swap(split);
    for (size_t g = 0; g < F.groups.size(); ++g)
      for (int j : F.groups[g].jobs) F.group_of[j] = (int)g;
  }
  // workspace: [descriptors][tables][masks][accumulators][counters][blocks][single-job arenas]
  size_t off = align_up(P.desc_bytes);
  // rounds and items (tables are laid out once the item count is known)
  for (FGroup& g : F.groups) {
    // items of a round ordered by padded input count, so that each X launch
    // takes a contiguous run of them
    std::stable_sort(g.jobs.begin(), g.jobs.end(), [&](int a, int b) {
      const int ma = (P.setups[a].n_stations * P.setups[a].n_pols + 3) / 4;
      const int mb = (P.setups[b].n_stations * P.setups[b].n_pols + 3) / 4;
      return ma < mb;
    });
    for (int r = 0;; ++r) {
      FRound R;
      R.first = (int)F.items.size();
      for (int j : g.jobs) {
        const xc_setup& s = P.setups[j];
        const Layout& L = F.L[j];
        const int64_t f0 = (int64_t)r * L.T;
        if (f0 >= s.n_frames) continue;
        FusedItem it{};
        it.f0 = f0;
        it.nf = (int)(s.n_frames - f0 < L.T ? s.n_frames - f0 : L.T);
        const int M = s.n_stations * s.n_pols;
        int n_splits = 0, fps = 0;
        xmac_splits(it.nf, L.fps, M, s.n_chan, s.n_subbands, n_splits, fps);
        it.fps = fps;
        it.slot_stride = L.slot_stride;
        it.task0 = R.ntasks;
        R.ntasks += fstage_fused_tasks(g.N, g.W, s.n_stations, s.n_subbands * s.n_pols, it.nf);
        it.dblk0 = R.dblocks;
        R.dblocks += delays_fused_blocks(it.nf, s.n_stations, s.n_subbands);
        it.wblk0 = R.wblocks;
        R.wblocks += weights_fused_blocks(it.nf, s.n_stations);
        const int Mp = (M + 3) / 4 * 4;
        if (R.xc.empty() || R.xc.back().Mp != Mp)
          R.xc.push_back({Mp, (int)F.items.size() - R.first, 0, 0});
        XClass& X = R.xc.back();
        it.xblk0 = X.blocks;
        X.blocks += xmac_fused_blocks(M, s.n_chan, s.n_subbands, n_splits);
        ++X.n;
        F.items.push_back(it);
        F.item_job.push_back(j);
      }
      R.n = (int)F.items.size() - R.first;
      if (R.n == 0) break;
      g.rounds.push_back(R);
    }
  }
  for (int j = 0; j < n; ++j) {
    if (F.group_of[j] < 0) continue;
    const xc_setup& s = P.setups[j];
    FusedOut o{};
    o.n_slots = F.L[j].n_slots;
    o.slot_stride = F.L[j].slot_stride;
    o.S = s.n_stations;
    o.P = s.n_pols;
    o.M = s.n_stations * s.n_pols;
    o.nbl = o.M * (o.M + 1) / 2;
    o.n_chan = s.n_chan;
    o.n_sb = s.n_subbands;
    o.blk0 = F.fin_blocks;
    F.fin_blocks += finalise_fused_blocks(s.n_subbands, o.M, s.n_chan);
    F.outs.push_back(o);
    F.out_job.push_back(j);
  }
  F.items_off = off;
  off += align_up(F.items.size() * sizeof(FusedItem));
  F.outs_off = off;
  off += align_up(F.outs.size() * sizeof(FusedOut));
  F.masks_off = off;
  off += align_up(F.masks.size() * sizeof(FusedMask));
  F.blob_bytes = off;
  F.maskbytes_off = off;
  off += mbytes;
  F.acc_off = off;
  F.vacc_off.assign(n, 0);
  F.wacc_off.assign(n, 0);
  for (int j = 0; j < n; ++j) {
    if (F.group_of[j] < 0) continue;
    F.vacc_off[j] = off;
    off += (size_t)F.L[j].n_slots * F.L[j].slot_stride * sizeof(double2);
    F.wacc_off[j] = off;
    off += align_up((size_t)P.setups[j].n_stations * P.setups[j].n_stations * sizeof(double));
  }
  F.acc_bytes = off - F.acc_off;
  for (FGroup& g : F.groups) {
    g.ctr_off = off;
    off += kAlign;
  }
  F.blk_off.assign(n, 0);
  for (int j = 0; j < n; ++j) {
    if (F.group_of[j] < 0) continue;
    F.blk_off[j] = off;
    off += F.L[j].drec_bytes + F.L[j].prec_bytes + F.L[j].spec_bytes;
  }
  // lanes: the solo jobs on lane 0, then groups and single jobs, longest
  // first, each to the least loaded lane
  std::vector<std::pair<int64_t, int>> work;   // (cost, group g as -1 - g, or job j)
  for (size_t g = 0; g < F.groups.size(); ++g) work.push_back({F.groups[g].cost, -1 - (int)g});
  for (int j = 0; j < n; ++j)
    if (F.group_of[j] < 0) work.push_back({job_cost(P.setups[j]), j});
  std::stable_sort(work.begin(), work.end(),
                   [](const std::pair<int64_t, int>& a, const std::pair<int64_t, int>& b) {
                     return a.first > b.first;
                   });
  std::stable_partition(work.begin(), work.end(), [&](const std::pair<int64_t, int>& w) {
    return w.second >= 0 && P.solo[w.second];
  });
  std::vector<int64_t> load(lanes, 0);
  F.lane_groups.assign(lanes, {});
  F.lane_jobs.assign(lanes, {});
  std::vector<int> lane_of_job(n, 0);
  for (auto& w : work) {
    const bool solo = w.second >= 0 && P.solo[w.second];
    const int l = solo ? 0 : (int)(std::min_element(load.begin(), load.end()) - load.begin());
    load[l] += w.first;
    if (w.second < 0) {
      F.lane_groups[l].push_back(-1 - w.second);
    } else {
      F.lane_jobs[l].push_back(w.second);
      lane_of_job[w.second] = l;
    }
  }
  // single jobs run one after another on their lane, so a lane's single jobs
  // share one arena (its largest)
  std::vector<size_t> lane_arena(lanes, 0);
  for (int j = 0; j < n; ++j) {
    if (F.group_of[j] >= 0) continue;
    F.L[j] = layout_of(&P.setups[j], jobs[j].st, P.tunes[j]);   // its own masks
    lane_arena[lane_of_job[j]] = std::max(lane_arena[lane_of_job[j]], align_up(F.L[j].total));
  }
  std::vector<size_t> lane_off(lanes, 0);
  for (int l = 0; l < lanes; ++l) {
    lane_off[l] = off;
    off += lane_arena[l];
  }
  F.arena_off.assign(n, 0);
  for (int j = 0; j < n; ++j)
    if (F.group_of[j] < 0) F.arena_off[j] = lane_off[lane_of_job[j]];
  F.total = off;
  return XC_OK;
}

// Device pointers of the plan for workspace `ws`; host blob (descriptors and
// tables) into c->h_batch; upload it on `stream`.
int fill_and_upload_fused(xc_ctx* c, const xc_job* jobs, int n, FPlan& F, unsigned char* ws,
                          hipStream_t stream) {
  const Plan& P = F.P;
  for (size_t m = 0; m < F.masks.size(); ++m) F.masks[m].ok = ws + F.maskbytes_off + F.mask_off[m];
  for (int j = 0; j < n; ++j)
    for (size_t i = 0; i < F.st_mask[j].size(); ++i)
      if (F.st_mask[j][i] >= 0) F.st[j][i].frame_ok = F.masks[F.st_mask[j][i]].ok;
  for (size_t k = 0; k < F.items.size(); ++k) {
    const int j = F.item_job[k];
    const Layout& L = F.L[j];
    unsigned char* b = ws + F.blk_off[j];
    FusedItem& it = F.items[k];
    it.job = reinterpret_cast<const DevJob*>(ws + P.desc_off[j]);
    it.drec = reinterpret_cast<DelayRec*>(b);
    it.prec = reinterpret_cast<PhaseRec*>(b + L.drec_bytes);
    it.spec = reinterpret_cast<float2*>(b + L.drec_bytes + L.prec_bytes);
    it.vacc = reinterpret_cast<double2*>(ws + F.vacc_off[j]);
    it.wst = reinterpret_cast<double*>(ws + F.wacc_off[j]);
  }
  for (size_t k = 0; k < F.outs.size(); ++k) {
    const int j = F.out_job[k];
    FusedOut& o = F.outs[k];
    o.vacc = reinterpret_cast<const double2*>(ws + F.vacc_off[j]);
    o.wst = reinterpret_cast<const double*>(ws + F.wacc_off[j]);
    o.vis = static_cast<float2*>(jobs[j].out.vis);
    o.weight = jobs[j].out.weight;
  }
  hipError_t e = hipSuccess;
  if (!c->batch_ev) e = hipEventCreateWithFlags(&c->batch_ev, hipEventDisableTiming);
  if (e == hipSuccess) e = hipEventSynchronize(c->batch_ev);   // previous blob is uploaded
  if (e == hipSuccess && c->h_batch_bytes < F.blob_bytes) {
    if (c->h_batch) (void)hipHostFree(c->h_batch);
    c->h_batch = nullptr;
    c->h_batch_bytes = 0;
    e = hipHostMalloc((void**)&c->h_batch, F.blob_bytes, hipHostMallocDefault);
    if (e == hipSuccess) c->h_batch_bytes = F.blob_bytes;
  }
  if (e != hipSuccess) return hip_fail(c, e, "batch descriptors");
  memset(c->h_batch, 0, F.blob_bytes);
  for (int j = 0; j < n; ++j) {
    // single jobs keep their own masks in their own arena
    const bool fused = F.group_of[j] >= 0;
    build_desc(&P.setups[j], fused ? F.st[j].data() : jobs[j].st, F.L[j], ws + P.desc_off[j],
               fused ? nullptr : ws + F.arena_off[j], c->h_batch + P.desc_off[j]);
  }
  for (size_t k = 0; k < F.items.size(); ++k)
    F.items[k].jd = *reinterpret_cast<const DevJob*>(c->h_batch + P.desc_off[F.item_job[k]]);
  memcpy(c->h_batch + F.items_off, F.items.data(), F.items.size() * sizeof(FusedItem));
  memcpy(c->h_batch + F.outs_off, F.outs.data(), F.outs.size() * sizeof(FusedOut));
  memcpy(c->h_batch + F.masks_off, F.masks.data(), F.masks.size() * sizeof(FusedMask));
  e = hipMemcpyAsync(ws, c->h_batch, F.blob_bytes, hipMemcpyHostToDevice, stream);
  if (e == hipSuccess) e = hipEventRecord(c->batch_ev, stream);
  return e == hipSuccess ? XC_OK : hip_fail(c, e, "batch descriptor upload");
}

int enqueue_group(xc_ctx* c, const FPlan& F, const FGroup& g, unsigned char* ws, hipStream_t s) {
  const FusedItem* items = reinterpret_cast<const FusedItem*>(ws + F.items_off);
  unsigned* ctr = reinterpret_cast<unsigned*>(ws + g.ctr_off);
  for (const FRound& R : g.rounds) {
    const FusedItem* it = items + R.first;
    hipError_t e = timed(c, XC_K_DELAYS, s, [&] {
      hipError_t r = launch_delays_fused(it, R.n, R.dblocks, ctr, s);
      return r == hipSuccess ? launch_weights_fused(it, R.n, R.wblocks, s) : r;
    });
    if (e != hipSuccess) return hip_fail(c, e, "fused delays");
    e = timed(c, XC_K_FSTAGE, s, [&] {
      return launch_fstage_fused(g.N, g.W, it, R.n, R.ntasks, c->d_tw, ctr, s);
    });
    if (e != hipSuccess) return hip_fail(c, e, "fused F stage");
    for (const XClass& X : R.xc) {
      e = timed(c, XC_K_XMAC, s,
                [&] { return launch_xmac_fused(X.Mp, it + X.first, X.n, X.blocks, s); });
      if (e != hipSuccess) return hip_fail(c, e, "fused X stage");
    }
  }
  return XC_OK;
}

int enqueue_fused(xc_ctx* c, const xc_job* jobs, const FPlan& F, unsigned char* ws, int lanes,
                  hipStream_t origin) {
  const int n = (int)F.P.setups.size();
  hipError_t e = hipSuccess;
  if (!F.masks.empty())
    e = timed(c, XC_K_INGEST, origin, [&] {
      return launch_ingest_fused(reinterpret_cast<const FusedMask*>(ws + F.masks_off),
                                 (int)F.masks.size(), F.ingest_blocks, origin);
    });
  if (e == hipSuccess && F.acc_bytes)
    e = timed(c, XC_K_ZERO, origin, [&] {
      return launch_zero(reinterpret_cast<double*>(ws + F.acc_off), F.acc_bytes / sizeof(double),
                         origin);
    });
  if (e != hipSuccess) return hip_fail(c, e, "fused prologue");
  e = hipEventRecord(c->fork_ev, origin);
  for (int l = 0; l < lanes && e == hipSuccess; ++l) e = hipStreamWaitEvent(c->lanes[l], c->fork_ev, 0);
  if (e != hipSuccess) return hip_fail(c, e, "batch fork");
  for (int l = 0; l < lanes; ++l) {
    for (int g : F.lane_groups[l]) {
      const int rc = enqueue_group(c, F, F.groups[g], ws, c->lanes[l]);
      if (rc != XC_OK) return rc;
    }
    for (int j : F.lane_jobs[l]) {
      const DevJob* dj = reinterpret_cast<const DevJob*>(ws + F.P.desc_off[j]);
      const int rc = enqueue_job(c, &F.P.setups[j], jobs[j].st, &jobs[j].out, dj,
                                 ws + F.arena_off[j], F.L[j], F.P.tunes[j], c->lanes[l]);
      if (rc != XC_OK) {
        c->last_error = "job " + std::to_string(j) + ": " + c->last_error;
        return rc;
      }
    }
  }
  for (int l = 0; l < lanes && e == hipSuccess; ++l) {
    e = hipEventRecord(c->lane_ev[l], c->lanes[l]);
    if (e == hipSuccess) e = hipStreamWaitEvent(origin, c->lane_ev[l], 0);
  }
  if (e != hipSuccess) return hip_fail(c, e, "batch join");
  (void)n;
  if (!F.outs.empty())
    e = timed(c, XC_K_FINALISE, origin, [&] {
      return launch_finalise_fused(reinterpret_cast<const FusedOut*>(ws + F.outs_off),
                                   (int)F.outs.size(), F.fin_blocks, origin);
    });
  return e == hipSuccess ? XC_OK : hip_fail(c, e, "fused finalise");
}

}  // namespace

extern "C" {

size_t xc_batch_workspace_bytes(xc_ctx* c, const xc_job* jobs, int32_t n_jobs, int32_t n_lanes,
                                int32_t flags) {
  if (flags & XC_BATCH_LANES) {
    Plan P;
    if (plan_batch(c, jobs, n_jobs, n_lanes, P) != XC_OK) return 0;
    return P.total;
  }
  FPlan F;
  if (plan_fused(c, jobs, n_jobs, n_lanes, F) != XC_OK) return 0;
  return F.total;
}

int xc_correlate_batch(xc_ctx* c, const xc_job* jobs, int32_t n_jobs, int32_t n_lanes,
                       int32_t flags, void* workspace, size_t ws_bytes, void* stream_) {
  if (!c) return XC_E_INVAL;
  hipStream_t stream = (hipStream_t)stream_;
  const bool lanes_only = (flags & XC_BATCH_LANES) != 0;
  Plan P;
  FPlan F;
  int rc = lanes_only ? plan_batch(c, jobs, n_jobs, n_lanes, P)
                      : plan_fused(c, jobs, n_jobs, n_lanes, F);
  if (rc != XC_OK) return rc;
  const size_t need = lanes_only ? P.total : F.total;
  if (!workspace || ws_bytes < need)
    return fail(c, XC_E_NOMEM, "batch workspace %zu bytes < %zu needed", ws_bytes, need);
  hipError_t e = hipSetDevice(c->device);
  if (e != hipSuccess) return hip_fail(c, e, "hipSetDevice");
  // lanes 0..n-1 run jobs; lane n is the capture origin for graphs
  rc = ensure_lanes(c, n_lanes + 1);
  if (rc != XC_OK) return rc;
  unsigned char* ws = static_cast<unsigned char*>(workspace);
  rc = lanes_only ? upload_batch_desc(c, jobs, n_jobs, P, ws, stream)
                  : fill_and_upload_fused(c, jobs, n_jobs, F, ws, stream);
  if (rc != XC_OK) return rc;
  auto enqueue = [&](hipStream_t origin) {
    return lanes_only ? enqueue_batch(c, jobs, P, ws, n_lanes, origin)
                      : enqueue_fused(c, jobs, F, ws, n_lanes, origin);
  };
  if (!(flags & XC_BATCH_GRAPH)) return enqueue(stream);

  const uint64_t key =
      fnv(batch_key(jobs, n_jobs, n_lanes, lanes_only ? P : F.P, workspace), &flags, sizeof flags);
  for (auto& g : c->graphs)
    if (g.key == key) {
      e = hipGraphLaunch(g.exec, stream);
      return e == hipSuccess ? XC_OK : hip_fail(c, e, "hipGraphLaunch");
    }
  hipStream_t origin = c->lanes[n_lanes];
  e = hipStreamWaitEvent(origin, c->batch_ev, 0);   // (outside the capture)
  if (e == hipSuccess) e = hipStreamSynchronize(origin);
  if (e == hipSuccess) e = hipStreamBeginCapture(origin, hipStreamCaptureModeRelaxed);
  if (e != hipSuccess) return hip_fail(c, e, "hipStreamBeginCapture");
  c->capturing = true;
  rc = enqueue(origin);
  c->capturing = false;
  hipGraph_t graph = nullptr;
  e = hipStreamEndCapture(origin, &graph);
  if (rc != XC_OK) {
    if (graph) (void)hipGraphDestroy(graph);
    return rc;
  }
  if (e != hipSuccess) return hip_fail(c, e, "hipStreamEndCapture");
  hipGraphExec_t exec = nullptr;
  e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  if (e != hipSuccess) return hip_fail(c, e, "hipGraphInstantiate");
  if (c->graphs.size() >= 8) {
    (void)hipGraphExecDestroy(c->graphs.front().exec);
    c->graphs.erase(c->graphs.begin());
  }
  c->graphs.push_back({key, exec});
  e = hipGraphLaunch(exec, stream);
  return e == hipSuccess ? XC_OK : hip_fail(c, e, "hipGraphLaunch");
}

int xc_autotune(xc_ctx* c, const xc_setup* setup, const xc_station* st, const xc_output* out,
                void* workspace, size_t ws_bytes, void* stream_, xc_tuning* best_out) {
  if (!c || !setup) return XC_E_INVAL;
  int rc = validate(c, setup, st);
  if (rc != XC_OK) return rc;
  if (!out || !out->vis || !out->weight) return fail(c, XC_E_INVAL, "output is NULL");
  hipStream_t stream = (hipStream_t)stream_;
  hipError_t e = hipSetDevice(c->device);
  if (e != hipSuccess) return hip_fail(c, e, "hipSetDevice");
  xc_setup s = *setup;
  if (s.n_frames > kTuneFrames) s.n_frames = kTuneFrames;
  s.frames_per_block = 0;
  std::vector<xc_tuning> cands;
  // block size: the library default.  Every block costs each kernel's ramp-up
  // and drain, and no smaller block has been faster over a whole job; timed
  // here, a smaller block wins only by the probe's artefacts (a 512-frame block
  // that wins on 8192 frames runs a 4 s job in 122 blocks, the default in 5;
  // a short job repeated back to back finds its input in the cache, which a
  // run over many jobs does not).  Where the workspace is too small for the
  // default, the largest power of two up to 2048 that fits is tried as well.
  // The first candidate is the library default throughout.
  auto fits = [&](int fpb) {
    const xc_tuning tu = {0, 0, 0, fpb, 0, 1};
    const Layout L = layout_of(&s, st, tu);
    return align_up(L.desc_bytes) + L.total <= ws_bytes;
  };
  std::vector<int> fpbs = {0};
  if (!fits(0))
    for (int fpb = 2048; fpb >= 16; fpb /= 2)
      if (fits(fpb)) {
        fpbs.push_back(fpb);
        break;
      }
  for (int fpb : fpbs) {
    if (fpb > s.n_frames && fpb != 512) continue;
    if (s.precision == XC_FP32) {
      const int M = s.n_stations * s.n_pols;
      const int xs[][2] = {{0, 0}, {8, 0}, {kXmacMatrix, 0}, {kXmacMatrixRing, 0}, {2, 0}, {4, 0}, {2, 32}, {1, 0}};
      for (auto& x : xs) {
        // the ring and the matrix-core stage hold at most 32 inputs
        if ((x[0] == 8 || x[0] == kXmacMatrix || x[0] == kXmacMatrixRing) && M > 32) continue;
        if (x[0] == 0 && fpb != 0) continue;  // (the default X stage at other block sizes:
                                             //  ring, matrix or staged kernel, listed)
        cands.push_back({0, x[0], x[1], fpb, 0, 1});
      }
    } else {
      cands.push_back({0, 0, 0, fpb, 0, 1});
    }
  }
  hipEvent_t a = nullptr, b = nullptr;
  e = hipEventCreate(&a);
  if (e == hipSuccess) e = hipEventCreate(&b);
  if (e != hipSuccess) return hip_fail(c, e, "autotune events");
  const bool prof = c->profiling;
  c->profiling = false;
  float best_ms = 1e30f, default_ms = 1e30f;
  xc_tuning best = {0, 0, 0, 0, 0, 0};
  for (const xc_tuning& tu : cands) {
    const Layout L = layout_of(&s, st, tu);
    if (align_up(L.desc_bytes) + L.total > ws_bytes) continue;
    unsigned char* desc = static_cast<unsigned char*>(workspace);
    unsigned char* arena = desc + align_up(L.desc_bytes);
    rc = upload_desc(c, &s, st, L, desc, arena, stream);
    for (int rep = 0; rep < 3 && rc == XC_OK; ++rep) {
      if (rep == 1) e = hipEventRecord(a, stream);
      rc = enqueue_job(c, &s, st, out, reinterpret_cast<const DevJob*>(desc), arena, L, tu, stream);
    }
    if (rc != XC_OK) break;
    e = hipEventRecord(b, stream);
    if (e == hipSuccess) e = hipEventSynchronize(b);
    float ms = 0.f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, a, b);
    if (e != hipSuccess) {
      rc = hip_fail(c, e, "autotune timing");
      break;
    }
    // the library default (the first candidate) is kept unless another shape
    // is faster by more than the few per cent that runs of one shape differ
    const bool is_default = &tu == &cands.front();
    if (is_default) default_ms = ms;
    if (is_default ? ms < best_ms : ms < best_ms && ms < 0.97f * default_ms) {
      best_ms = ms;
      best = tu;
    }
  }
  c->profiling = prof;
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  if (rc != XC_OK) return rc;
  if (best_ms == 1e30f) return fail(c, XC_E_NOMEM, "autotune: no candidate fits the workspace");
  c->tuned[shape_key(setup)] = best;
  if (best_out) *best_out = best;
  return XC_OK;
}

}  // extern "C"
