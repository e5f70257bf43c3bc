// gmc_server.cpp -- the served form: continuous batching of dose requests.
//
// A server thread owns up to max_slots slots, each a workspace with its own
// non-blocking stream.  Submitted requests wait in a FIFO; whenever a slot is
// free and the request's device footprint (queues and staging of its slot,
// K batch tallies and the dose/sigma outputs of its grid) fits beside what
// the other slots hold within the memory budget, the request starts on that
// slot: its rounds are captured in a graph that the server replays, reading
// the slot's control block through an event it polls, so requests that
// arrive while others run start at once and their kernels overlap on the
// device.  Phantoms and tables stay resident in the context; a request only
// references them.  A finished request's dose and sigma are finalized into a
// device buffer of the server's result pool and stay there until gmc_poll
// copies them out (device to device, or straight to host memory); pool
// buffers are reused by later requests, so finishing a request neither
// allocates pinned memory nor waits on a free.
//
// Every request is a single-beam job run by the same engine as gmc_run_beam,
// so its result is bit-identical to running it alone.
#include <algorithm>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <thread>

#include "gmc_host.hpp"

namespace gmc {

using Clock = std::chrono::steady_clock;

struct Request {
  uint64_t ticket = 0;
  int32_t pid = 0, tid = 0;
  gmc_source src{};
  std::vector<double> tab_e, tab_w;   // a tabulated spectrum's tables (src points at them)
  uint64_t n = 0, seed = 0;
  size_t nvox = 0;
  uint32_t K = 0;
  size_t need = 0;              // device bytes of its slot while it runs
  Clock::time_point t_submit, t_start, t_end;
  bool done = false;
  int rc = GMC_OK;
  std::string err;
  int res = -1;                 // result-pool buffer holding dose then sigma (nvox each), until polled
  std::vector<double> dose, sigma;   // the result in host memory instead (moved there when the server stops)
  gmc_run_stats stats{};
};

// A device buffer of the result pool: 2 x elems doubles.
struct ResultBuf {
  double* p = nullptr;
  size_t elems = 0;
  bool busy = false;
};

struct Slot {
  Workspace w;
  bool ready = false;
  std::shared_ptr<Request> req;
  int state = 0;                // 0 idle, 1 replaying, 2 finishing
  Engine E;
  hipGraphExec_t exec = nullptr;
  int nr = 0;
  uint64_t rounds = 0;
  const PhantomObj* P = nullptr;
  hipEvent_t ev_done = nullptr;
};

struct Server {
  gmc_context* c = nullptr;
  size_t budget = 0;
  int max_slots = 4;
  std::thread th;
  std::mutex mu;                    // pending, tickets, stopping
  std::condition_variable cv;       // work arrived, or stop
  std::condition_variable cv_done;  // a request finished
  std::deque<std::shared_ptr<Request>> pending;
  std::map<uint64_t, std::shared_ptr<Request>> tickets;
  std::vector<std::unique_ptr<Slot>> slots;
  std::vector<ResultBuf> results;   // guarded by mu (the caller's gmc_poll releases buffers)
  hipStream_t copy_stream = nullptr;  // the server thread's copies of results to host memory
  bool stopping = false;
  bool running = false;
  uint64_t next_ticket = 1;
  size_t slot_fixed = 0;            // queues + staging of one slot
};

namespace {

void release_refs(gmc_context* c, const Request& r) {
  std::lock_guard<std::mutex> lk(c->mu);
  if (--c->refs[r.pid] <= 0) c->refs.erase(r.pid);
  if (--c->refs[r.tid] <= 0) c->refs.erase(r.tid);
}

size_t result_bytes(const Server* s) {   // caller holds s->mu
  size_t b = 0;
  for (const ResultBuf& rb : s->results) b += 2 * rb.elems * sizeof(double);
  return b;
}

// Free the pool's idle buffers (hipFree waits for the device: only when the
// budget needs the room, or when the server stops).
void trim_results(Server* s) {
  std::vector<void*> idle;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    for (ResultBuf& rb : s->results)
      if (!rb.busy && rb.p) {
        idle.push_back(rb.p);
        rb.p = nullptr;
        rb.elems = 0;
      }
  }
  for (void* p : idle) (void)hipFree(p);   // outside the lock: a poll need not wait for the device
}

// A pool buffer of at least 2 x elems doubles for a finishing request: the
// smallest idle one that is large enough, else a new one.
int acquire_result(Server* s, Workspace* w, size_t elems, int* idx) {
  {
    std::lock_guard<std::mutex> lk(s->mu);
    int best = -1;
    for (int i = 0; i < (int)s->results.size(); ++i) {
      const ResultBuf& rb = s->results[i];
      if (!rb.busy && rb.p && rb.elems >= elems && (best < 0 || rb.elems < s->results[best].elems)) best = i;
    }
    if (best >= 0) {
      s->results[best].busy = true;
      *idx = best;
      return GMC_OK;
    }
  }
  void* p = nullptr;
  if (hipMalloc(&p, 2 * elems * sizeof(double)) != hipSuccess) {
    (void)hipGetLastError();
    trim_results(s);
    WS_TRY(w, hipMalloc(&p, 2 * elems * sizeof(double)));
  }
  std::lock_guard<std::mutex> lk(s->mu);
  int slot = -1;
  for (int i = 0; i < (int)s->results.size() && slot < 0; ++i)
    if (!s->results[i].p) slot = i;
  if (slot < 0) {
    slot = (int)s->results.size();
    s->results.emplace_back();
  }
  s->results[slot].p = static_cast<double*>(p);
  s->results[slot].elems = elems;
  s->results[slot].busy = true;
  *idx = slot;
  return GMC_OK;
}

void release_result(Server* s, Request& r) {   // caller holds s->mu
  if (r.res >= 0) s->results[r.res].busy = false;
  r.res = -1;
}

// Move the result of the oldest finished, unclaimed request from its pool
// buffer to host memory and free the buffer; false if there is none.
bool spill_oldest_result(Server* s) {
  void* freed = nullptr;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    Request* oldest = nullptr;
    for (auto& kv : s->tickets)   // ordered by ticket, i.e. by submission
      if (kv.second->done && kv.second->res >= 0) {
        oldest = kv.second.get();
        break;
      }
    if (!oldest) return false;
    Request& r = *oldest;
    ResultBuf& rb = s->results[r.res];
    r.dose.resize(r.nvox);
    r.sigma.resize(r.nvox);
    const size_t bytes = r.nvox * sizeof(double);
    hipError_t e = hipMemcpyAsync(r.dose.data(), rb.p, bytes, hipMemcpyDeviceToHost, s->copy_stream);
    if (e == hipSuccess)
      e = hipMemcpyAsync(r.sigma.data(), rb.p + r.nvox, bytes, hipMemcpyDeviceToHost, s->copy_stream);
    if (e == hipSuccess) e = hipStreamSynchronize(s->copy_stream);
    if (e != hipSuccess) {
      r.rc = GMC_EDEVICE;
      r.err = std::string("copy of a finished result to host memory: ") + hipGetErrorString(e);
    }
    freed = rb.p;
    rb.p = nullptr;
    rb.elems = 0;
    rb.busy = false;
    r.res = -1;
  }
  (void)hipFree(freed);
  return true;
}

void complete(Server* s, Slot& sl, int rc, const std::string& err) {
  std::shared_ptr<Request> r = sl.req;
  if (rc != GMC_OK && sl.w.stream) (void)hipStreamSynchronize(sl.w.stream);   // nothing of it still running
  if (sl.exec) (void)hipGraphExecDestroy(sl.exec);
  sl.exec = nullptr;
  sl.req.reset();
  sl.state = 0;
  r->t_end = Clock::now();
  release_refs(s->c, *r);
  {
    std::lock_guard<std::mutex> lk(s->mu);
    if (rc != GMC_OK) release_result(s, *r);
    r->rc = rc;
    r->err = err;
    r->done = true;
  }
  s->cv_done.notify_all();
}

// Enqueue the request's set-up, capture its rounds and launch the first
// replay with its control-block copy.
int start(Server* s, Slot& sl) {
  gmc_context* c = s->c;
  Request& r = *sl.req;
  Workspace* w = &sl.w;
  const PhantomObj* pp = nullptr;
  const TablesObj* tp = nullptr;
  gmc_tuning tun = default_tuning();
  {
    std::lock_guard<std::mutex> lk(c->mu);
    pp = c->phantoms.at(r.pid).get();
    tp = c->tables.at(r.tid).get();
    auto hit = c->tuned.find(job_class(*pp, *tp, &r.src, &r.n, 1));
    if (hit != c->tuned.end()) tun = hit->second;
  }
  const Tune tu = resolve_tuning(&tun);
  int rc = ws_ensure_tally(w, tally_vox(r.nvox) * r.K);
  if (rc) return rc;
  MajObj maj;
  rc = get_majorants(c, r.pid, r.tid, *pp, *tp, &maj, &w->err);
  if (rc) return rc;
  Job J;
  build_job(&J, w, *pp, *tp, maj, &r.src, &r.n, 1, r.seed, kCombined);
  sl.P = pp;
  sl.rounds = 0;
  WS_TRY(w, hipEventRecord(w->ev0, w->stream));
  WS_TRY(w, launch_fill_u64(w->d_tally, tally_vox(r.nvox) * r.K, 0ull, w->stream));
  rc = engine_setup(w, sl.E, J, tu);
  if (rc == GMC_OK) rc = engine_capture(sl.E, &sl.exec, &sl.nr);
  if (rc) return rc;
  WS_TRY(w, hipGraphLaunch(sl.exec, w->stream));
  sl.rounds += (uint64_t)sl.nr;
  rc = enqueue_control_copy(w);
  if (rc) return rc;
  sl.state = 1;
  return GMC_OK;
}

// The job is done: finalize into a result-pool buffer and copy the counters
// to pinned host memory, all behind one event.
int finish(Server* s, Slot& sl) {
  Workspace* w = &sl.w;
  Request& r = *sl.req;
  std::vector<double> nk;
  add_batch_sizes(nk, r.src.first_history, r.n, r.K);
  int idx = -1;
  int rc = acquire_result(s, w, r.nvox, &idx);
  if (rc) return rc;
  double* res = nullptr;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    r.res = idx;
    res = s->results[idx].p;
  }
  rc = finalize(w, *sl.P, w->d_tally, 1u, 0u, r.K, nk, r.n, res, res + r.nvox, true, false);
  if (rc) return rc;
  WS_TRY(w, hipMemcpyAsync(w->h_ctr, w->d_ctr, (size_t)C_COUNT * kCtrSlots * sizeof(unsigned long long),
                           hipMemcpyDeviceToHost, w->stream));
  WS_TRY(w, hipEventRecord(w->ev1, w->stream));
  WS_TRY(w, hipEventRecord(sl.ev_done, w->stream));
  sl.state = 2;
  return GMC_OK;
}

// Advance a slot whose outstanding device work has finished; returns
// whether anything happened.
bool progress(Server* s, Slot& sl) {
  Workspace* w = &sl.w;
  const hipError_t q = hipEventQuery(sl.state == 1 ? w->ev_ctl : sl.ev_done);
  if (q == hipErrorNotReady) return false;
  if (q != hipSuccess) {
    complete(s, sl, GMC_EDEVICE, std::string("device error: ") + hipGetErrorString(q));
    return true;
  }
  Request& r = *sl.req;
  int rc = GMC_OK;
  if (sl.state == 1) {
    bool done = false;
    rc = after_replay(sl.E, sl.nr, &done);
    if (rc == GMC_OK && !done) {
      const hipError_t e = hipGraphLaunch(sl.exec, w->stream);
      if (e != hipSuccess) rc = wfail(w, GMC_EDEVICE, std::string("graph launch: ") + hipGetErrorString(e));
      sl.rounds += (uint64_t)sl.nr;
      if (rc == GMC_OK) rc = enqueue_control_copy(w);
    } else if (rc == GMC_OK) {
      rc = finish(s, sl);
    }
    if (rc) complete(s, sl, rc, w->err);
    return true;
  }
  // finishing: results are in pinned memory
  float dev_ms = 0.0f;
  (void)hipEventElapsedTime(&dev_ms, w->ev0, w->ev1);
  const double t_total = std::chrono::duration<double>(Clock::now() - r.t_start).count();
  rc = stats_from_counters(w, w->h_ctr, &r.stats, r.n, sl.rounds, t_total, dev_ms * 1e-3);
  complete(s, sl, rc, rc ? w->err : std::string());
  return true;
}

// Device memory the server holds: its slots' workspaces and the result pool
// (finished requests not yet polled, and idle buffers kept for reuse).
size_t held_bytes(Server* s) {
  size_t b = 0;
  for (const auto& sl : s->slots) b += ws_device_bytes(sl->w);
  std::lock_guard<std::mutex> lk(s->mu);
  return b + result_bytes(s);
}

// Start pending requests, in order, on free slots while their footprint
// fits in the budget (idle slots give back their job buffers first).
void admit(Server* s) {
  for (auto& slp : s->slots) {
    Slot& sl = *slp;
    if (sl.req) continue;
    std::shared_ptr<Request> r;
    {
      std::lock_guard<std::mutex> lk(s->mu);
      if (s->pending.empty()) return;
      r = s->pending.front();
    }
    const size_t cur = ws_device_bytes(sl.w);
    size_t held = held_bytes(s);
    if (held - cur + std::max(cur, r->need) > s->budget) {
      for (auto& o : s->slots)
        if (!o->req) ws_trim(&o->w);
      trim_results(s);
      held = held_bytes(s);
      // results waiting to be polled give way to host memory, oldest first,
      // so that unpolled results never stop the queue
      while (held - ws_device_bytes(sl.w) + std::max(ws_device_bytes(sl.w), r->need) > s->budget &&
             spill_oldest_result(s))
        held = held_bytes(s);
      if (held - ws_device_bytes(sl.w) + std::max(ws_device_bytes(sl.w), r->need) > s->budget) return;
    }
    {
      std::lock_guard<std::mutex> lk(s->mu);
      s->pending.pop_front();
    }
    sl.req = r;
    r->t_start = Clock::now();
    int rc = GMC_OK;
    if (!sl.ready) {
      rc = ws_init(&sl.w, s->c->device, nullptr);
      if (rc == GMC_OK && hipEventCreateWithFlags(&sl.ev_done, hipEventDisableTiming) != hipSuccess)
        rc = wfail(&sl.w, GMC_EDEVICE, "event creation failed");
      sl.ready = rc == GMC_OK;
    }
    if (rc == GMC_OK) rc = start(s, sl);
    if (rc) complete(s, sl, rc, sl.w.err);
  }
}

void loop(Server* s) {
  (void)hipSetDevice(s->c->device);
  for (;;) {
    admit(s);
    bool active = false, did = false;
    for (auto& sl : s->slots)
      if (sl->req) {
        active = true;
        did |= progress(s, *sl);
      }
    std::unique_lock<std::mutex> lk(s->mu);
    if (s->stopping && s->pending.empty() && !active) break;
    if (did) continue;
    if (active) {
      lk.unlock();
      std::this_thread::sleep_for(std::chrono::microseconds(20));
    } else {
      s->cv.wait_for(lk, std::chrono::milliseconds(5), [&] { return s->stopping || !s->pending.empty(); });
    }
  }
  for (auto& sl : s->slots) {
    if (sl->ev_done) (void)hipEventDestroy(sl->ev_done);
    if (sl->ready) ws_free(&sl->w);
  }
  s->slots.clear();
  // finished requests not yet polled keep their results in host memory, so
  // that the device buffers can go
  while (spill_oldest_result(s)) {
  }
  trim_results(s);
}

}  // namespace

void server_destroy(gmc_context* c) {
  if (!c->server) return;
  Server* s = c->server;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stopping = true;
  }
  s->cv.notify_all();
  if (s->th.joinable()) s->th.join();
  for (ResultBuf& rb : s->results)
    if (rb.p) (void)hipFree(rb.p);
  if (s->copy_stream) (void)hipStreamDestroy(s->copy_stream);
  delete s;
  c->server = nullptr;
}

}  // namespace gmc

using namespace gmc;

extern "C" {

int gmc_server_start(gmc_context* c, const gmc_server_config* cfg) {
  if (!c) return GMC_EINVAL;
  if (c->server && c->server->running) return cfail(c, GMC_EBUSY, "the server is already running");
  server_destroy(c);
  auto s = std::make_unique<Server>();
  s->c = c;
  s->max_slots = cfg && cfg->max_slots > 0 ? std::min(cfg->max_slots, 16) : 4;
  (void)hipSetDevice(c->device);
  size_t free_b = 0, total_b = 0;
  if (hipMemGetInfo(&free_b, &total_b) != hipSuccess) return cfail(c, GMC_EDEVICE, "hipMemGetInfo failed");
  s->budget = cfg && cfg->hbm_budget_bytes > 0 ? (size_t)cfg->hbm_budget_bytes : free_b / 4 * 3;
  if (hipStreamCreateWithFlags(&s->copy_stream, hipStreamNonBlocking) != hipSuccess)
    return cfail(c, GMC_EDEVICE, "stream creation failed");
  // queues and staging of one slot at the default tuning
  Workspace probe;
  probe.device = c->device;
  uint32_t cap = 0, soft = 0, stg = 0;
  queue_sizes(&probe, resolve_tuning(nullptr), kMaxMat, &cap, &soft, &stg);
  s->slot_fixed = sizeof(uint32_t) * ((size_t)Q_FIELDS * 4ull * cap + (size_t)kStgFields * 2ull * stg);
  for (int i = 0; i < s->max_slots; ++i) s->slots.push_back(std::make_unique<Slot>());
  s->running = true;
  Server* sp = s.release();
  c->server = sp;
  sp->th = std::thread(loop, sp);
  return GMC_OK;
}

int gmc_server_stop(gmc_context* c) {
  if (!c) return GMC_EINVAL;
  if (!c->server || !c->server->running) return cfail(c, GMC_EINVAL, "no server is running");
  Server* s = c->server;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stopping = true;
  }
  s->cv.notify_all();
  if (s->th.joinable()) s->th.join();
  s->running = false;
  return GMC_OK;
}

int gmc_submit(gmc_context* c, int32_t phantom_id, int32_t tables_id, const gmc_source* src, uint64_t n_hist,
               uint64_t seed, uint64_t* ticket) {
  if (!c) return GMC_EINVAL;
  if (!ticket) return cfail(c, GMC_EINVAL, "ticket pointer is NULL");
  Server* s = c->server;
  if (!s || !s->running) return cfail(c, GMC_EINVAL, "no server is running");
  std::string err;
  if (check_source(&err, src)) return cfail(c, GMC_EINVAL, err);
  auto r = std::make_shared<Request>();
  {
    std::lock_guard<std::mutex> lk(c->mu);
    auto pi = c->phantoms.find(phantom_id);
    auto ti = c->tables.find(tables_id);
    if (pi == c->phantoms.end() || ti == c->tables.end())
      return cfail(c, GMC_ENOTFOUND, "unknown phantom or tables id");
    const PhantomObj& P = *pi->second;
    const TablesObj& T = *ti->second;
    if (P.max_mat >= T.host.n_mat) return cfail(c, GMC_EINVAL, "phantom uses a material index beyond the tables");
    r->K = (uint32_t)T.phys.n_batches;
    if (n_hist < r->K || n_hist >= (1ull << 32))
      return cfail(c, GMC_EINVAL, "histories must be in [n_batches, 2^32)");
    if (src->first_history + n_hist >= (1ull << 32))
      return cfail(c, GMC_EINVAL, "first_history + histories must stay below 2^32");
    const double e_max = source_emax(*src);
    if ((double)n_hist * (e_max * 134217728.0 + 1.0) >= 9.2e18)
      return cfail(c, GMC_EOVERFLOW, "histories x energy would overflow the 64-bit tallies");
    r->nvox = P.nvox();
    r->need = s->slot_fixed + tally_vox(r->nvox) * r->K * sizeof(unsigned long long) + 2 * r->nvox * sizeof(double);
    if (r->need > s->budget)
      return cfail(c, GMC_EBUSY, "the request's device footprint exceeds the server's memory budget");
    ++c->refs[phantom_id];
    ++c->refs[tables_id];
  }
  r->pid = phantom_id;
  r->tid = tables_id;
  r->src = *src;
  if (src->spectrum == GMC_TABULATED) {
    r->tab_e.assign(src->tab_e, src->tab_e + src->tab_n + 1);
    r->tab_w.assign(src->tab_w, src->tab_w + src->tab_n);
    r->src.tab_e = r->tab_e.data();
    r->src.tab_w = r->tab_w.data();
  }
  r->n = n_hist;
  r->seed = seed;
  r->t_submit = Clock::now();
  {
    std::lock_guard<std::mutex> lk(s->mu);
    r->ticket = s->next_ticket++;
    s->tickets[r->ticket] = r;
    s->pending.push_back(r);
  }
  s->cv.notify_all();
  *ticket = r->ticket;
  return GMC_OK;
}

int gmc_poll(gmc_context* c, uint64_t ticket, int wait, int* done, double* dose, double* sigma, int out_ptr_kind,
             gmc_request_stats* stats) {
  if (!c) return GMC_EINVAL;
  if (!done) return cfail(c, GMC_EINVAL, "done pointer is NULL");
  if (out_ptr_kind != GMC_HOST && out_ptr_kind != GMC_DEVICE) return cfail(c, GMC_EINVAL, "bad out_ptr_kind");
  Server* s = c->server;
  if (!s) return cfail(c, GMC_ENOTFOUND, "no server");
  std::shared_ptr<Request> r;
  const double* res_p = nullptr;
  {
    std::unique_lock<std::mutex> lk(s->mu);
    auto it = s->tickets.find(ticket);
    if (it == s->tickets.end()) return cfail(c, GMC_ENOTFOUND, "unknown ticket " + std::to_string(ticket));
    r = it->second;
    if (wait) s->cv_done.wait(lk, [&] { return r->done; });
    *done = r->done ? 1 : 0;
    if (!r->done) return GMC_OK;
    s->tickets.erase(it);   // claimed: the server no longer moves its result
    if (r->res >= 0) res_p = s->results[r->res].p;
  }
  if (stats) {
    stats->t_queue_s = std::chrono::duration<double>(r->t_start - r->t_submit).count();
    stats->t_run_s = std::chrono::duration<double>(r->t_end - r->t_start).count();
    stats->t_latency_s = std::chrono::duration<double>(r->t_end - r->t_submit).count();
    stats->run = r->stats;
  }
  if (r->rc) return cfail(c, r->rc, r->err);
  const size_t bytes = r->nvox * sizeof(double);
  int rc = GMC_OK;
  if (res_p) {
    // device-resident result: one copy to the caller's buffer (device to
    // device, or device to host), complete on return, then the buffer goes
    // back to the pool
    (void)hipSetDevice(c->device);
    const hipMemcpyKind kind = out_ptr_kind == GMC_HOST ? hipMemcpyDeviceToHost : hipMemcpyDeviceToDevice;
    hipStream_t st = c->ws.stream;   // the context stream, as the blocking forms' copies
    hipError_t e = hipSuccess;
    if (dose) e = hipMemcpyAsync(dose, res_p, bytes, kind, st);
    if (e == hipSuccess && sigma) e = hipMemcpyAsync(sigma, res_p + r->nvox, bytes, kind, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) rc = cfail(c, GMC_EDEVICE, std::string("copy of the result: ") + hipGetErrorString(e));
    std::lock_guard<std::mutex> lk(s->mu);
    release_result(s, *r);
  } else if (out_ptr_kind == GMC_HOST) {
    if (dose) std::memcpy(dose, r->dose.data(), bytes);
    if (sigma) std::memcpy(sigma, r->sigma.data(), bytes);
  } else {
    (void)hipSetDevice(c->device);
    if (dose && hipMemcpy(dose, r->dose.data(), bytes, hipMemcpyHostToDevice) != hipSuccess)
      return cfail(c, GMC_EDEVICE, "copy of the dose to device memory failed");
    if (sigma && hipMemcpy(sigma, r->sigma.data(), bytes, hipMemcpyHostToDevice) != hipSuccess)
      return cfail(c, GMC_EDEVICE, "copy of sigma to device memory failed");
  }
  return rc;
}

int gmc_server_status(gmc_context* c, gmc_server_status_t* st) {
  if (!c || !st) return GMC_EINVAL;
  Server* s = c->server;
  std::memset(st, 0, sizeof(*st));
  if (!s) return GMC_OK;
  std::lock_guard<std::mutex> lk(s->mu);
  st->running = s->running ? 1 : 0;
  st->pending = (int)s->pending.size();
  int done = 0;
  for (const auto& kv : s->tickets) done += kv.second->done ? 1 : 0;
  st->finished_unpolled = done;
  st->in_flight = (int)s->tickets.size() - done - st->pending;
  st->budget_bytes = s->budget;
  return GMC_OK;
}

}  // extern "C"
