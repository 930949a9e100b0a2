// Batches (many uneven sub-integrations as one unit) and the autotuner.
#include <algorithm>
#include <numeric>

#include "xc_runtime.h"

using namespace xc;

namespace {

constexpr size_t kBatchSpecCap = (size_t)1 << 30;   // per-job staged spectra in a batch
constexpr int64_t kTuneFrames = 8192;               // frames an autotune candidate runs

struct Plan {
  std::vector<xc_setup> setups;          // job setups with the batch's block size
  std::vector<xc_tuning> tunes;
  std::vector<Layout> layouts;
  std::vector<size_t> desc_off;          // per job, in the descriptor region
  std::vector<int> lane_of;
  std::vector<std::vector<int>> order;   // per lane: jobs in launch order
  std::vector<size_t> arena_off;         // per lane
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
    // bound each job's staged spectra so that many lanes fit in HBM together
    const size_t per_frame =
        (size_t)s.n_subbands * s.n_stations * s.n_pols * s.n_chan * out_elem_bytes(L.out);
    if ((size_t)L.T * per_frame > kBatchSpecCap && s.frames_per_block == 0) {
      int T = (int)(kBatchSpecCap / per_frame);
      T = T < 64 ? 64 : T;
      s.frames_per_block = T;
      L = layout_of(&s, jobs[j].st, tu);
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
  for (int j : idx) {
    const int l = (int)(std::min_element(load.begin(), load.end()) - load.begin());
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

}  // namespace

extern "C" {

size_t xc_batch_workspace_bytes(xc_ctx* c, const xc_job* jobs, int32_t n_jobs, int32_t n_lanes) {
  Plan P;
  if (plan_batch(c, jobs, n_jobs, n_lanes, P) != XC_OK) return 0;
  return P.total;
}

int xc_correlate_batch(xc_ctx* c, const xc_job* jobs, int32_t n_jobs, int32_t n_lanes,
                       int32_t flags, void* workspace, size_t ws_bytes, void* stream_) {
  if (!c) return XC_E_INVAL;
  hipStream_t stream = (hipStream_t)stream_;
  Plan P;
  int rc = plan_batch(c, jobs, n_jobs, n_lanes, P);
  if (rc != XC_OK) return rc;
  if (!workspace || ws_bytes < P.total)
    return fail(c, XC_E_NOMEM, "batch workspace %zu bytes < %zu needed", ws_bytes, P.total);
  hipError_t e = hipSetDevice(c->device);
  if (e != hipSuccess) return hip_fail(c, e, "hipSetDevice");
  // lanes 0..n-1 run jobs; lane n is the capture origin for graphs
  rc = ensure_lanes(c, n_lanes + 1);
  if (rc != XC_OK) return rc;
  unsigned char* ws = static_cast<unsigned char*>(workspace);
  rc = upload_batch_desc(c, jobs, n_jobs, P, ws, stream);
  if (rc != XC_OK) return rc;
  if (!(flags & XC_BATCH_GRAPH)) return enqueue_batch(c, jobs, P, ws, n_lanes, stream);

  const uint64_t key = batch_key(jobs, n_jobs, n_lanes, P, workspace);
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
  rc = enqueue_batch(c, jobs, P, ws, n_lanes, origin);
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
  const int fpbs[] = {512, 1024, 2048};
  for (int fpb : fpbs) {
    if (fpb > s.n_frames && fpb != 512) continue;
    if (s.precision == XC_FP32) {
      const int M = s.n_stations * s.n_pols;
      const int xs[][2] = {{8, 0}, {2, 0}, {4, 0}, {2, 32}, {1, 0}};
      for (auto& x : xs) {
        if (x[0] == 8 && M > 32) continue;   // the ring holds at most 32 inputs
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
  float best_ms = 1e30f;
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
    if (ms < best_ms) {
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
