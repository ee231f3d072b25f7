// Serving runtime: continuous batching of iFCTN completion requests on one GPU.
//
// A scheduler thread owns all device work of the server.  Requests wait in a
// FIFO queue and are admitted when a slot is free and the device pool (one
// allocation made at create time, sized by the HBM budget) has a contiguous
// range for the job's workspace.  Every resident job runs Algorithm 1 in
// rounds of a few sweeps on one of a small set of HIP streams; after each
// round the job's device stop flag (set by the stop test after every X step)
// is copied to pinned host memory and checked without blocking, so jobs
// admitted later overlap on the device with jobs already running.  A finished
// job writes X to the caller's buffer, returns its pool range and is reported
// by ifctn_server_poll.  The sweeps of a job are the same kernels in the same
// order as ifctn_complete's, so a result does not depend on what else runs.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "ifctn.h"
#include "ifctn_host.h"

using namespace ifctn;

namespace {

constexpr size_t kPoolAlign = 256;

// First-fit allocator over offsets of the device pool, with coalescing.
class PoolAlloc {
 public:
  void reset(size_t bytes) {
    free_.clear();
    if (bytes) free_[0] = bytes;
  }
  static size_t rounded(size_t bytes) { return (bytes + kPoolAlign - 1) & ~(kPoolAlign - 1); }
  bool alloc(size_t bytes, size_t* off) {
    bytes = rounded(bytes);
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second >= bytes) {
        *off = it->first;
        const size_t rest = it->second - bytes, at = it->first + bytes;
        free_.erase(it);
        if (rest) free_[at] = rest;
        return true;
      }
    }
    return false;
  }
  void release(size_t off, size_t bytes) {
    bytes = rounded(bytes);
    auto it = free_.emplace(off, bytes).first;
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

struct Pending {
  ifctn_request req;
  std::vector<double> G0;
  PlanOpts opts;   // the tuning options at submit: admission plans the job as it was sized
  size_t bytes;
  double t_submit;
};

// pinned host words a round's readback lands in
struct HostSlot {
  int flags[4];  // non-finite O, stop, sweeps counted by the stop test
  double stats[5];
};

enum Phase { PH_MAIN, PH_REFINE, PH_FINISH };

struct Resident {
  Pending p;
  ifctn_job* J = nullptr;
  size_t off = 0;
  int stream = 0, slot = 0;
  Phase phase = PH_MAIN;
  int t_main = 0, refine = 0;
  int issued_main = 0, issued_refine = 0;
  int main_done = 0;     // sweeps of the main phase that ran (the stop test may end it early)
  bool stopped = false;  // the stop test was met
  bool waiting = false;  // a round's readback is in flight
  bool finished = false;
  double t_admit = 0.0;
  hipEvent_t ev = nullptr;
};

}  // namespace

struct ifctn_server {
  ifctn_server_config cfg{};
  std::chrono::steady_clock::time_point t0;
  std::thread th;
  std::mutex mu;
  std::condition_variable cv_done, cv_work, cv_ready;
  std::deque<Pending> queue;
  std::vector<ifctn_completion> done;
  bool quit = false;
  bool ready = false;
  ifctn_status init_status = IFCTN_OK;
  std::string init_error;
  // owned by the scheduler thread
  unsigned char* pool = nullptr;
  PoolAlloc alloc;
  std::vector<hipStream_t> streams;
  HostSlot* host = nullptr;
  std::vector<int> free_slots;
  std::vector<Resident*> res;
  int next_stream = 0;

  double now() const { return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count(); }
  void run();
  ifctn_status setup();
  void teardown();
  bool admit();
  void step(Resident& r, bool* progressed);
  hipError_t issue(Resident& r);
  // drain: work of the job may still be queued (failure paths), so wait for
  // its stream before the pool range is handed to another job
  void finish(Resident& r, ifctn_status st, bool drain);
};

ifctn_status ifctn_server::setup() {
  if (hipSetDevice(cfg.device) != hipSuccess) return IFCTN_E_HIP;
  for (int q = 0; q < cfg.num_streams; ++q) {
    hipStream_t s;
    if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) return IFCTN_E_HIP;
    streams.push_back(s);
  }
  if (hipMalloc((void**)&pool, cfg.hbm_budget_bytes) != hipSuccess) {
    (void)hipGetLastError();
    pool = nullptr;
    return IFCTN_E_NOMEM;
  }
  if (hipHostMalloc((void**)&host, sizeof(HostSlot) * cfg.max_active, hipHostMallocDefault) != hipSuccess) {
    host = nullptr;
    return IFCTN_E_NOMEM;
  }
  alloc.reset(cfg.hbm_budget_bytes);
  for (int q = cfg.max_active - 1; q >= 0; --q) free_slots.push_back(q);
  return IFCTN_OK;
}

void ifctn_server::teardown() {
  for (hipStream_t s : streams) {
    (void)hipStreamSynchronize(s);
    (void)hipStreamDestroy(s);
  }
  streams.clear();
  if (pool) (void)hipFree(pool);
  if (host) (void)hipHostFree(host);
  pool = nullptr;
  host = nullptr;
}

// Report a job and give back its slot and pool range.
void ifctn_server::finish(Resident& r, ifctn_status st, bool drain) {
  ifctn_completion c;
  std::memset(&c, 0, sizeof(c));
  c.tag = r.p.req.tag;
  c.status = st;
  if (st == IFCTN_OK) {
    stats_from(host[r.slot].stats, r.main_done + r.issued_refine, &c.stats);
    c.stats.converged = r.stopped ? 1 : 0;
  }
  c.t_submit = r.p.t_submit;
  c.t_admit = r.t_admit;
  c.t_done = now();
  if (drain) (void)hipStreamSynchronize(streams[r.stream]);
  if (r.J) job_close(r.J);
  r.J = nullptr;
  alloc.release(r.off, r.p.bytes);
  free_slots.push_back(r.slot);
  if (r.ev) (void)hipEventDestroy(r.ev);
  r.ev = nullptr;
  r.finished = true;
  std::lock_guard<std::mutex> lk(mu);
  done.push_back(c);
  cv_done.notify_all();
}

// Admit queued requests (FIFO) while a slot and a pool range are free.
bool ifctn_server::admit() {
  bool any = false;
  for (;;) {
    Pending p;
    size_t off = 0;
    {
      std::lock_guard<std::mutex> lk(mu);
      if (queue.empty() || free_slots.empty() || quit) return any;
      if (!alloc.alloc(queue.front().bytes, &off)) return any;  // wait until memory frees up
      p = std::move(queue.front());
      queue.pop_front();
    }
    Resident* r = new Resident();
    r->p = std::move(p);
    r->off = off;
    r->slot = free_slots.back();
    free_slots.pop_back();
    r->stream = next_stream;
    next_stream = (next_stream + 1) % (int)streams.size();
    r->t_admit = now();
    res.push_back(r);
    any = true;
    const ifctn_request& q = r->p.req;
    ifctn_status st = take_injected_admit_failure()
                          ? set_error(IFCTN_E_NOMEM, "injected admission failure")
                          : job_open(&q.params, q.O_dev, q.mask_dev, r->p.G0.data(), streams[r->stream],
                                     pool + off, r->p.bytes, false, r->p.opts, &r->J);
    if (st != IFCTN_OK) {
      r->J = nullptr;
      finish(*r, st, true);
      continue;
    }
    if (hipEventCreateWithFlags(&r->ev, hipEventDisableTiming) != hipSuccess) {
      finish(*r, IFCTN_E_HIP, true);
      continue;
    }
    r->refine = job_is_bf16(r->J) ? std::min(job_refine_sweeps(r->J), q.t_max) : 0;
    r->t_main = q.t_max - r->refine;
    job_set_stop(r->J, q.eps);
    r->phase = r->t_main > 0 ? PH_MAIN : PH_REFINE;
    if (r->phase == PH_REFINE && job_is_bf16(r->J)) {
      job_set_stop(r->J, 0.0);
      if (job_promote(r->J) != hipSuccess) finish(*r, IFCTN_E_HIP, true);
    }
  }
}

// Enqueue the job's next round and the readback of its flags (or of its
// statistics and X, once it is done), then record the round's event.
hipError_t ifctn_server::issue(Resident& r) {
  ifctn_job* J = r.J;
  const hipStream_t s = streams[r.stream];
  hipError_t e = hipSuccess;
  const int spr = cfg.sweeps_per_round;
  if (r.phase == PH_MAIN) {
    const int n = std::min(spr, r.t_main - r.issued_main);
    e = job_sweeps(J, n);
    r.issued_main += n;
    if (e == hipSuccess && r.issued_main == r.t_main) e = job_x_step(J);
  } else if (r.phase == PH_REFINE) {
    const int n = std::min(spr, r.refine - r.issued_refine);
    e = job_sweeps(J, n);
    r.issued_refine += n;
    if (e == hipSuccess && r.issued_refine == r.refine) e = job_x_step(J);
  } else {
    e = job_x_step(J);
    if (e == hipSuccess) e = job_finalize(J);
    if (e == hipSuccess)
      e = hipMemcpyAsync(host[r.slot].stats, job_stats_dev(J), 5 * sizeof(double), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess && ifctn_reconstruct(J, r.p.req.X_out_dev, 1) != IFCTN_OK) e = hipErrorUnknown;
  }
  if (e == hipSuccess) e = hipMemcpyAsync(host[r.slot].flags, job_flags(J), 3 * sizeof(int), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipEventRecord(r.ev, s);
  if (e == hipSuccess) r.waiting = true;
  return e;
}

void ifctn_server::step(Resident& r, bool* progressed) {
  if (r.finished) return;   // failed at admission, or done: removed after this pass
  if (r.waiting) {
    const hipError_t q = hipEventQuery(r.ev);
    if (q == hipErrorNotReady) return;
    *progressed = true;
    r.waiting = false;
    if (q != hipSuccess) {
      finish(r, IFCTN_E_HIP, true);
      return;
    }
    const HostSlot& h = host[r.slot];
    if (h.flags[0]) {
      finish(r, IFCTN_E_INVAL, false);   // non-finite observed data
      return;
    }
    if (r.phase == PH_FINISH) {
      finish(r, IFCTN_OK, false);
      return;
    }
    if (r.phase == PH_MAIN && (h.flags[1] || r.issued_main >= r.t_main)) {
      r.stopped = h.flags[1] != 0;
      r.main_done = r.p.req.eps > 0.0 ? h.flags[2] : r.t_main;
      if (job_is_bf16(r.J)) {
        job_set_stop(r.J, 0.0);
        hipError_t e = job_promote(r.J);
        if (e == hipSuccess) e = job_reset_flags(r.J);  // the refinement always runs
        if (e != hipSuccess) {
          finish(r, IFCTN_E_HIP, true);
          return;
        }
      }
      r.phase = r.refine > 0 ? PH_REFINE : PH_FINISH;
    } else if (r.phase == PH_REFINE && r.issued_refine >= r.refine) {
      r.phase = PH_FINISH;
    }
  }
  if (!r.waiting) {
    *progressed = true;
    if (issue(r) != hipSuccess) finish(r, IFCTN_E_HIP, true);
  }
}

void ifctn_server::run() {
  ifctn_status st = setup();
  {
    std::lock_guard<std::mutex> lk(mu);
    init_status = st;
    ready = true;
  }
  cv_ready.notify_all();
  if (st != IFCTN_OK) {
    teardown();
    return;
  }
  for (;;) {
    bool progressed = admit();
    for (Resident* r : res) step(*r, &progressed);
    for (size_t q = 0; q < res.size();) {
      if (res[q]->finished) {
        delete res[q];
        res[q] = res.back();
        res.pop_back();
      } else {
        ++q;
      }
    }
    std::unique_lock<std::mutex> lk(mu);
    if (quit && res.empty()) break;
    if (!progressed) {
      if (res.empty()) {
        cv_work.wait(lk, [&] { return quit || !queue.empty(); });
      } else {
        lk.unlock();
        std::this_thread::sleep_for(std::chrono::microseconds(20));
      }
    }
  }
  teardown();
}

extern "C" {

ifctn_status ifctn_server_create(const ifctn_server_config* cfg, ifctn_server** out) {
  if (!out || !cfg) return set_error(IFCTN_E_INVAL, "config and out are required");
  *out = nullptr;
  if (cfg->hbm_budget_bytes < kPoolAlign) return set_error(IFCTN_E_INVAL, "hbm_budget_bytes too small");
  if (cfg->max_active < 1 || cfg->max_active > 1024) return set_error(IFCTN_E_INVAL, "max_active outside 1..1024");
  if (cfg->num_streams < 1 || cfg->num_streams > 16) return set_error(IFCTN_E_INVAL, "num_streams outside 1..16");
  if (cfg->sweeps_per_round < 1) return set_error(IFCTN_E_INVAL, "sweeps_per_round < 1");
  ifctn_server* S = new ifctn_server();
  S->cfg = *cfg;
  S->t0 = std::chrono::steady_clock::now();
  S->th = std::thread([S] { S->run(); });
  std::unique_lock<std::mutex> lk(S->mu);
  S->cv_ready.wait(lk, [&] { return S->ready; });
  const ifctn_status st = S->init_status;
  lk.unlock();
  if (st != IFCTN_OK) {
    S->th.join();
    delete S;
    return set_error(st, "server setup failed (device, streams, pool or pinned memory)");
  }
  *out = S;
  return IFCTN_OK;
}

ifctn_status ifctn_server_submit(ifctn_server* S, const ifctn_request* req) {
  if (!S || !req) return set_error(IFCTN_E_INVAL, "server and request are required");
  if (!req->O_dev || !req->mask_dev || !req->G0_host || !req->X_out_dev)
    return set_error(IFCTN_E_INVAL, "O_dev, mask_dev, G0_host and X_out_dev are required");
  if (req->t_max < 0) return set_error(IFCTN_E_INVAL, "t_max < 0");
  if (!(req->eps >= 0.0)) return set_error(IFCTN_E_INVAL, "eps < 0");
  PlanOpts opts = current_opts();
  // resident jobs already overlap one another on their own streams; a second
  // stream per job (Gamma_k beside the contraction) made the served mix about
  // 20% slower, so served jobs build Gamma_k in line
  opts.overlap = false;
  const size_t bytes = job_bytes(&req->params, opts);
  if (bytes == 0) return IFCTN_E_INVAL;  // message set by the params check
  if (PoolAlloc::rounded(bytes) > S->cfg.hbm_budget_bytes)
    return set_error(IFCTN_E_NOMEM, "the job needs more device memory than the server's whole budget");
  Pending p;
  p.req = *req;
  p.G0.assign(req->G0_host, req->G0_host + ifctn_num_factor_entries(&req->params));
  p.opts = opts;
  p.bytes = bytes;
  p.t_submit = S->now();
  {
    std::lock_guard<std::mutex> lk(S->mu);
    if (S->quit) return set_error(IFCTN_E_STATE, "server is shutting down");
    S->queue.push_back(std::move(p));
  }
  S->cv_work.notify_all();
  return IFCTN_OK;
}

ifctn_status ifctn_server_poll(ifctn_server* S, ifctn_completion* out, int32_t max, int32_t* n, int32_t wait_ms) {
  if (!S || !n || (max > 0 && !out)) return set_error(IFCTN_E_INVAL, "server, out and n are required");
  std::unique_lock<std::mutex> lk(S->mu);
  if (S->done.empty() && wait_ms > 0)
    S->cv_done.wait_for(lk, std::chrono::milliseconds(wait_ms), [&] { return !S->done.empty(); });
  const int32_t k = std::min<int32_t>(std::max<int32_t>(max, 0), (int32_t)S->done.size());
  for (int32_t q = 0; q < k; ++q) out[q] = S->done[q];
  S->done.erase(S->done.begin(), S->done.begin() + k);
  *n = k;
  return IFCTN_OK;
}

ifctn_status ifctn_server_queued(ifctn_server* S, int32_t* queued, int32_t* completed_unpolled) {
  if (!S || !queued || !completed_unpolled) return set_error(IFCTN_E_INVAL, "arguments are required");
  std::lock_guard<std::mutex> lk(S->mu);
  *queued = (int32_t)S->queue.size();
  *completed_unpolled = (int32_t)S->done.size();
  return IFCTN_OK;
}

ifctn_status ifctn_server_destroy(ifctn_server* S) {
  if (!S) return IFCTN_OK;
  {
    std::lock_guard<std::mutex> lk(S->mu);
    S->quit = true;
    S->queue.clear();
  }
  S->cv_work.notify_all();
  S->th.join();
  delete S;
  return IFCTN_OK;
}

}  // extern "C"
