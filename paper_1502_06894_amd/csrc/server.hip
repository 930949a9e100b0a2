// Continuous-batching correlation server: requests are admitted into
// concurrent lanes as lanes and device memory (a pool fixed at creation) free
// up; a scheduler thread launches them, detects completion with events and
// keeps latency statistics.
#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>

#include "xc_runtime.h"

using namespace xc;

namespace {

using Clock = std::chrono::steady_clock;
constexpr int kMaxBypass = 8;

// First-fit allocator over [0, size).
class Pool {
 public:
  explicit Pool(size_t size) { free_[0] = size; }
  bool alloc(size_t n, size_t& off) {
    n = align_up(n);
    for (auto it = free_.begin(); it != free_.end(); ++it)
      if (it->second >= n) {
        off = it->first;
        const size_t rest = it->second - n;
        free_.erase(it);
        if (rest) free_[off + n] = rest;
        return true;
      }
    return false;
  }
  void release(size_t off, size_t n) {
    n = align_up(n);
    auto it = free_.emplace(off, n).first;
    auto nx = std::next(it);
    if (nx != free_.end() && it->first + it->second == nx->first) {
      it->second += nx->second;
      free_.erase(nx);
    }
    if (it != free_.begin()) {
      auto pv = std::prev(it);
      if (pv->first + pv->second == it->first) {
        pv->second += it->second;
        free_.erase(it);
      }
    }
  }

 private:
  std::map<size_t, size_t> free_;
};

enum class State { Queued, Running, Done };

struct Request {
  uint64_t ticket = 0;
  xc_setup setup{};
  std::vector<int32_t> stream_map;
  std::vector<double> lo;
  std::vector<xc_station> st;
  std::vector<std::vector<double>> delay, phase;
  xc_output out{};
  Layout L;
  xc_tuning tu{};
  size_t footprint = 0, off = 0;
  int lane = -1, bypassed = 0;
  bool cancelled = false;
  State state = State::Queued;
  int rc = XC_OK;
  hipEvent_t done_ev = nullptr;
  Clock::time_point t_submit, t_end;
  double samples = 0;
};

}  // namespace

struct xc_server {
  xc_ctx* ctx = nullptr;
  unsigned char* pool_base = nullptr;
  std::unique_ptr<Pool> pool;
  size_t budget = 0;
  int slots = 0;
  std::vector<int> lane_busy;
  std::mutex mu;
  std::condition_variable cv_sched, cv_done;
  std::deque<std::shared_ptr<Request>> queue;
  std::vector<std::shared_ptr<Request>> running;
  std::map<uint64_t, std::shared_ptr<Request>> all;
  uint64_t next_ticket = 1;
  bool stop = false;
  std::thread th;
  std::vector<double> lat_ms;
  int64_t n_failed = 0, n_cancelled = 0;
  double done_samples = 0;
  bool have_first = false;
  Clock::time_point t_first, t_last;
  std::string last_error;

  void loop();
  void start(Request& r);
};

void xc_server::start(Request& r) {
  // caller holds mu
  int lane = -1;
  for (int i = 0; i < slots; ++i)
    if (!lane_busy[i]) {
      lane = i;
      break;
    }
  r.lane = lane;
  lane_busy[lane] = 1;
  r.state = State::Running;
  unsigned char* desc = pool_base + r.off;
  unsigned char* arena = desc + align_up(r.L.desc_bytes);
  hipStream_t s = ctx->lanes[lane];
  int rc = upload_desc(ctx, &r.setup, r.st.data(), r.L, desc, arena, s);
  if (rc == XC_OK)
    rc = enqueue_job(ctx, &r.setup, r.st.data(), &r.out, reinterpret_cast<const DevJob*>(desc),
                     arena, r.L, r.tu, s);
  if (rc == XC_OK && hipEventRecord(r.done_ev, s) != hipSuccess) rc = XC_E_HIP;
  r.rc = rc;
  if (rc != XC_OK) last_error = ctx->last_error;
  running.push_back(std::shared_ptr<Request>(all[r.ticket]));
}

void xc_server::loop() {
  (void)hipSetDevice(ctx->device);
  std::unique_lock<std::mutex> lk(mu);
  for (;;) {
    // completions
    for (size_t i = 0; i < running.size();) {
      Request& r = *running[i];
      const bool finished = r.rc != XC_OK || hipEventQuery(r.done_ev) == hipSuccess;
      if (!finished) {
        ++i;
        continue;
      }
      if (r.rc != XC_OK) (void)hipStreamSynchronize(ctx->lanes[r.lane]);   // drain a partial launch
      r.t_end = Clock::now();
      r.state = State::Done;
      pool->release(r.off, r.footprint);
      lane_busy[r.lane] = 0;
      if (r.cancelled) {
        r.rc = XC_E_CANCELLED;
        ++n_cancelled;
      } else if (r.rc != XC_OK) {
        ++n_failed;
      } else {
        lat_ms.push_back(std::chrono::duration<double, std::milli>(r.t_end - r.t_submit).count());
        done_samples += r.samples;
        t_last = r.t_end;
      }
      running.erase(running.begin() + i);
      cv_done.notify_all();
    }
    // admission: FIFO, but a later request may start ahead of earlier ones that
    // do not fit yet; each earlier one is passed at most kMaxBypass times
    for (size_t qi = 0; qi < queue.size() && (int)running.size() < slots;) {
      Request& r = *queue[qi];
      size_t off;
      if (!pool->alloc(r.footprint, off)) {
        if (r.bypassed >= kMaxBypass) break;   // nothing may pass it any more
        ++qi;
        continue;
      }
      for (size_t k = 0; k < qi; ++k) ++queue[k]->bypassed;
      r.off = off;
      std::shared_ptr<Request> keep = queue[qi];
      queue.erase(queue.begin() + qi);
      start(r);
    }
    if (stop && queue.empty() && running.empty()) break;
    if (running.empty())
      cv_sched.wait(lk, [&] { return stop || !queue.empty(); });
    else
      cv_sched.wait_for(lk, std::chrono::microseconds(100));
  }
}

extern "C" {

int xc_server_create(xc_server** out, int hip_device, size_t budget, int32_t max_slots) {
  if (!out || max_slots < 1 || max_slots > kMaxLanes || budget == 0) return XC_E_INVAL;
  *out = nullptr;
  xc_ctx* c = nullptr;
  int rc = xc_create(&c, hip_device);
  if (rc != XC_OK) return rc;
  xc_server* s = new xc_server();
  s->ctx = c;
  s->budget = budget;
  s->slots = max_slots;
  s->lane_busy.assign(max_slots, 0);
  rc = ensure_lanes(c, max_slots);
  if (rc == XC_OK && hipMalloc((void**)&s->pool_base, budget) != hipSuccess) rc = XC_E_NOMEM;
  if (rc != XC_OK) {
    if (s->pool_base) (void)hipFree(s->pool_base);
    xc_destroy(c);
    delete s;
    return rc;
  }
  s->pool.reset(new Pool(budget));
  s->th = std::thread([s] { s->loop(); });
  *out = s;
  return XC_OK;
}

int xc_server_submit(xc_server* s, const xc_job* job, uint64_t* ticket) {
  if (!s || !job || !ticket) return XC_E_INVAL;
  xc_ctx tmp;   // validation messages only (no device state)
  int rc = validate(&tmp, &job->setup, job->st);
  if (rc == XC_OK && (!job->out.vis || !job->out.weight)) rc = fail(&tmp, XC_E_INVAL, "output is NULL");
  if (rc != XC_OK) {
    std::lock_guard<std::mutex> g(s->mu);
    s->last_error = tmp.last_error;
    return rc;
  }
  auto r = std::make_shared<Request>();
  const xc_setup& js = job->setup;
  r->setup = js;
  r->stream_map.assign(js.stream_map, js.stream_map + js.n_subbands * js.n_pols);
  r->lo.assign(js.lo_hz, js.lo_hz + js.n_subbands);
  r->setup.stream_map = r->stream_map.data();
  r->setup.lo_hz = r->lo.data();
  r->st.assign(job->st, job->st + js.n_stations);
  r->delay.resize(js.n_stations);
  r->phase.resize(js.n_stations);
  for (int i = 0; i < js.n_stations; ++i) {
    const xc_station& x = job->st[i];
    r->delay[i].assign(x.delay_poly, x.delay_poly + x.poly_deg + 1);
    r->st[i].delay_poly = r->delay[i].data();
    if (x.phase_poly) {
      r->phase[i].assign(x.phase_poly, x.phase_poly + (size_t)js.n_subbands * (x.poly_deg + 1));
      r->st[i].phase_poly = r->phase[i].data();
    }
  }
  r->out = job->out;
  r->samples = (double)js.n_stations * js.n_subbands * js.n_pols * js.n_frames * 2.0 * js.n_chan;
  std::lock_guard<std::mutex> g(s->mu);
  r->tu = effective_tuning(s->ctx, &r->setup);
  r->L = layout_of(&r->setup, r->st.data(), r->tu);
  if (r->setup.frames_per_block == 0) {
    // bound each request's staged spectra (half the budget shared among the
    // slots, at least 1 GiB; or 16 (M + 1) frames where that is more) so that
    // several fit in the budget together
    const size_t cap = std::max((size_t)1 << 30, s->budget / (2 * (size_t)s->slots));
    const int T = shared_block_frames(r->setup, r->L, cap, 16);
    if (T != r->L.T) {
      r->setup.frames_per_block = T;
      r->L = layout_of(&r->setup, r->st.data(), r->tu);
    }
  }
  r->footprint = align_up(r->L.desc_bytes) + r->L.total;
  if (r->footprint > s->budget) {
    s->last_error = "request footprint " + std::to_string(r->footprint) + " exceeds the budget " +
                    std::to_string(s->budget);
    return XC_E_NOMEM;
  }
  if (hipEventCreateWithFlags(&r->done_ev, hipEventDisableTiming) != hipSuccess) return XC_E_HIP;
  r->ticket = s->next_ticket++;
  r->t_submit = Clock::now();
  if (!s->have_first) {
    s->have_first = true;
    s->t_first = r->t_submit;
  }
  s->all[r->ticket] = r;
  s->queue.push_back(r);
  *ticket = r->ticket;
  s->cv_sched.notify_one();
  return XC_OK;
}

// A finished request whose result has been reported: forget its ticket and
// release its event (caller holds mu).  Without this a long-running server
// would keep every request it ever served.
static int retire(xc_server* s, std::map<uint64_t, std::shared_ptr<Request>>::iterator it) {
  const int rc = it->second->rc;
  if (it->second->done_ev) (void)hipEventDestroy(it->second->done_ev);
  it->second->done_ev = nullptr;
  s->all.erase(it);
  return rc;
}

int xc_server_poll(xc_server* s, uint64_t ticket, int32_t* done) {
  if (!s || !done) return XC_E_INVAL;
  std::lock_guard<std::mutex> g(s->mu);
  auto it = s->all.find(ticket);
  if (it == s->all.end()) return XC_E_INVAL;
  *done = it->second->state == State::Done ? 1 : 0;
  return *done ? retire(s, it) : XC_OK;
}

int xc_server_wait(xc_server* s, uint64_t ticket, int32_t timeout_ms) {
  if (!s) return XC_E_INVAL;
  std::unique_lock<std::mutex> lk(s->mu);
  auto it = s->all.find(ticket);
  if (it == s->all.end()) return XC_E_INVAL;
  std::shared_ptr<Request> r = it->second;
  auto pred = [&] { return r->state == State::Done; };
  if (timeout_ms < 0)
    s->cv_done.wait(lk, pred);
  else if (!s->cv_done.wait_for(lk, std::chrono::milliseconds(timeout_ms), pred))
    return XC_E_TIMEOUT;
  // another thread may have retired the ticket while this one waited
  it = s->all.find(ticket);
  return it == s->all.end() ? r->rc : retire(s, it);
}

int xc_server_cancel(xc_server* s, uint64_t ticket) {
  if (!s) return XC_E_INVAL;
  std::lock_guard<std::mutex> g(s->mu);
  auto it = s->all.find(ticket);
  if (it == s->all.end() || it->second->state == State::Done) return XC_E_INVAL;
  Request& r = *it->second;
  r.cancelled = true;
  if (r.state == State::Queued) {
    s->queue.erase(std::find(s->queue.begin(), s->queue.end(), it->second));
    r.state = State::Done;
    r.rc = XC_E_CANCELLED;
    ++s->n_cancelled;
    s->cv_done.notify_all();
  }
  return XC_OK;
}

int xc_server_get_stats(xc_server* s, xc_server_stats* o) {
  if (!s || !o) return XC_E_INVAL;
  std::lock_guard<std::mutex> g(s->mu);
  std::vector<double> v = s->lat_ms;
  std::sort(v.begin(), v.end());
  auto pct = [&](double p) {
    if (v.empty()) return 0.0;
    const double x = p * (v.size() - 1);
    const size_t i = (size_t)x;
    return i + 1 < v.size() ? v[i] + (x - i) * (v[i + 1] - v[i]) : v.back();
  };
  o->p50_ms = pct(0.5);
  o->p99_ms = pct(0.99);
  double sum = 0;
  for (double x : v) sum += x;
  o->mean_ms = v.empty() ? 0.0 : sum / v.size();
  o->completed = (int64_t)v.size();
  o->failed = s->n_failed;
  o->cancelled = s->n_cancelled;
  o->queued = (int64_t)s->queue.size();
  o->running = (int64_t)s->running.size();
  const double span = v.empty() ? 0.0
                                : std::chrono::duration<double>(s->t_last - s->t_first).count();
  o->station_samples_per_s = span > 0 ? s->done_samples / span : 0.0;
  return XC_OK;
}

const char* xc_server_last_error(xc_server* s) { return s ? s->last_error.c_str() : ""; }

void xc_server_destroy(xc_server* s) {
  if (!s) return;
  {
    std::lock_guard<std::mutex> g(s->mu);
    for (auto& r : s->queue) {
      r->cancelled = true;
      r->state = State::Done;
      r->rc = XC_E_CANCELLED;
    }
    s->queue.clear();
    s->stop = true;
    s->cv_sched.notify_all();
    s->cv_done.notify_all();
  }
  s->th.join();
  for (auto& kv : s->all)
    if (kv.second->done_ev) (void)hipEventDestroy(kv.second->done_ev);
  (void)hipFree(s->pool_base);
  xc_destroy(s->ctx);
  delete s;
}

}  // extern "C"
