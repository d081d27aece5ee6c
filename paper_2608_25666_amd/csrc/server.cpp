// Continuous-batching projection server: a worker thread admits queued
// requests into batched persistent launches while earlier launches still run,
// each launch on its own stream (declared in include/prism_server.h).
#include <hip/hip_runtime.h>
#include <time.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <mutex>
#include <new>
#include <thread>
#include <unordered_map>
#include <vector>

#include "prism_internal.h"
#include "prism_server.h"
#include "serve_sched.h"

using namespace prism;

namespace {

int64_t mono_ns() {
  timespec ts;
  clock_gettime(CLOCK_MONOTONIC, &ts);
  return (int64_t)ts.tv_sec * 1000000000ll + ts.tv_nsec;
}

struct Ticket {
  int ctrl = 0;
  int N = 0, iters = 0;
  const float* xin = nullptr;
  float* xout = nullptr;
  float* rp = nullptr;
  float* rd = nullptr;
  int* itout = nullptr;
  std::vector<double> q0, v0;
  int state = PRISM_SERVER_QUEUED;
  int error = 0;
  int warm = 0;
  int batch = 0;
  int64_t t_submit = 0, t_launch = 0, t_done = 0;
};

struct Ctrl {
  prism_proj_s* p;
  int max_N;
  size_t x_floats;   // max_N * H * nj
};

struct Slot {
  hipStream_t stream = nullptr;
  hipEvent_t done = nullptr;
  prism_batch_t staging = nullptr;
  std::vector<int64_t> jobs;
  bool busy = false;
};

}  // namespace

struct prism_server_s {
  explicit prism_server_s(const prism_server_config_t& c)
      : cfg(c), sched(c.hbm_budget, c.max_batch, (size_t)c.max_queue) {}
  int device = 0;
  prism_server_config_t cfg;
  char* pool = nullptr;
  serve::Scheduler sched;
  std::vector<Ctrl> ctrls;
  std::unordered_map<int64_t, Ticket> tickets;
  std::vector<Slot> slots;
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::thread worker;
  bool stop = false;
  int64_t next_ticket = 1;
  int64_t submitted = 0, completed = 0, failed = 0, launches = 0, running = 0, max_conc = 0;
};

namespace {

void finish_slot(prism_server_s* S, Slot& sl, prism_status_t st) {
  const int64_t t = mono_ns();
  for (int64_t id : sl.jobs) {
    auto it = S->tickets.find(id);
    if (it == S->tickets.end()) continue;
    Ticket& k = it->second;
    k.state = (st == PRISM_OK) ? PRISM_SERVER_DONE : PRISM_SERVER_FAILED;
    k.error = st;
    k.t_done = t;
    S->sched.complete(k.ctrl, st == PRISM_OK);
    if (st == PRISM_OK) ++S->completed;
    else ++S->failed;
    --S->running;
  }
  sl.jobs.clear();
  sl.busy = false;
  S->cv_done.notify_all();
}

// Called with the lock held; releases it around the HIP calls (only the worker
// touches the slots, and running tickets cannot be released or erased).
void launch(prism_server_s* S, Slot& sl, const std::vector<serve::Pick>& picks,
            std::unique_lock<std::mutex>& lk) {
  std::vector<BatchDesc> d;
  d.reserve(picks.size());
  const int64_t t = mono_ns();
  for (const serve::Pick& pk : picks) {
    Ticket& k = S->tickets[pk.ticket];
    const Ctrl& c = S->ctrls[pk.ctrl];
    float* xs = reinterpret_cast<float*>(S->pool + pk.state_off);
    float* qs = xs + c.x_floats;
    BatchDesc D{};
    D.p = c.p;
    D.xin = k.xin;
    D.xout = k.xout;
    D.xsave = xs;
    D.rp = k.rp;
    D.rd = k.rd;
    D.itout = k.itout;
    D.xw = pk.warm ? xs : nullptr;
    D.uw = pk.warm ? qs : nullptr;
    D.uout = qs;
    D.N = k.N;
    D.iters = k.iters;
    D.shift = pk.warm ? 1 : 0;
    D.q0 = k.q0.data();
    D.v0 = k.v0.data();
    d.push_back(D);
    k.state = PRISM_SERVER_RUNNING;
    k.warm = pk.warm ? 1 : 0;
    k.batch = (int)picks.size();
    k.t_launch = t;
    sl.jobs.push_back(pk.ticket);
    ++S->running;
  }
  const prism_options_t opts = S->cfg.opts;
  const int share = S->cfg.grid_share;
  lk.unlock();
  prism_status_t st = enqueue_batch(sl.staging, d.data(), (int)d.size(), opts, sl.stream, share);
  if (st == PRISM_OK && hipEventRecord(sl.done, sl.stream) != hipSuccess) st = PRISM_EDEVICE;
  lk.lock();
  if (st != PRISM_OK) {
    finish_slot(S, sl, st);
    return;
  }
  sl.busy = true;
  ++S->launches;
  int64_t conc = 0;
  for (const Slot& o : S->slots) conc += o.busy ? 1 : 0;
  S->max_conc = std::max(S->max_conc, conc);
}

void worker_main(prism_server_s* S) {
  (void)hipSetDevice(S->device);
  std::unique_lock<std::mutex> lk(S->mu);
  for (;;) {
    bool did = false, any_busy = false;
    for (Slot& sl : S->slots) {
      if (!sl.busy) continue;
      const hipError_t e = hipEventQuery(sl.done);
      if (e == hipErrorNotReady) {
        any_busy = true;
        continue;
      }
      finish_slot(S, sl, e == hipSuccess ? PRISM_OK : PRISM_EDEVICE);
      did = true;
    }
    if (S->stop && !any_busy) break;
    if (!S->stop) {
      for (Slot& sl : S->slots) {
        if (sl.busy) continue;
        if (S->sched.queued() == 0) break;
        const std::vector<serve::Pick> picks = S->sched.pick();
        if (picks.empty()) break;
        launch(S, sl, picks, lk);
        did = true;
        any_busy = any_busy || sl.busy;
      }
    }
    if (did) continue;
    if (any_busy) S->cv_work.wait_for(lk, std::chrono::microseconds(20));
    else if (!S->stop) S->cv_work.wait(lk);
  }
  // requests still queued at shutdown
  for (auto& kv : S->tickets)
    if (kv.second.state == PRISM_SERVER_QUEUED) {
      kv.second.state = PRISM_SERVER_FAILED;
      kv.second.error = PRISM_EDEVICE;
    }
  S->cv_done.notify_all();
}

void release_all(prism_server_s* S) {
  for (Slot& sl : S->slots) {
    if (sl.staging) prism_batch_destroy(sl.staging);
    if (sl.done) (void)hipEventDestroy(sl.done);
    if (sl.stream) (void)hipStreamDestroy(sl.stream);
  }
  S->slots.clear();
  if (S->pool) (void)hipFree(S->pool);
  S->pool = nullptr;
}

void fill_info(const Ticket& k, prism_ticket_info_t* info) {
  info->state = k.state;
  info->error = k.error;
  info->warm = k.warm;
  info->batch_size = k.batch;
  info->t_submit_ns = k.t_submit;
  info->t_launch_ns = k.t_launch;
  info->t_done_ns = k.t_done;
}

}  // namespace

extern "C" {

int64_t prism_server_now_ns(void) { return mono_ns(); }

void prism_server_config_default(prism_server_config_t* cfg) {
  if (!cfg) return;
  cfg->hbm_budget = (size_t)1 << 30;
  cfg->max_inflight = 2;
  cfg->max_batch = 64;
  cfg->max_queue = 65536;
  cfg->grid_share = 75;
  prism_options_default(&cfg->opts);
}

prism_status_t prism_server_create(const prism_server_config_t* cfg, prism_server_t* out) {
  if (!cfg || !out) return PRISM_EINVAL;
  *out = nullptr;
  if (cfg->hbm_budget < serve::kGranule || cfg->max_inflight < 1 || cfg->max_inflight > 4 ||
      cfg->max_batch < 1 || cfg->max_queue < 1 || cfg->grid_share < 1 || cfg->grid_share > 100)
    return PRISM_EINVAL;
  prism_status_t st = validate_options(&cfg->opts);
  if (st != PRISM_OK) return st;
  prism_server_s* S = new (std::nothrow) prism_server_s(*cfg);
  if (!S) return PRISM_ENOMEM;
  if (hipGetDevice(&S->device) != hipSuccess) {
    delete S;
    return PRISM_EDEVICE;
  }
  if (hipMalloc((void**)&S->pool, cfg->hbm_budget) != hipSuccess) {
    S->pool = nullptr;
    delete S;
    return PRISM_ENOMEM;
  }
  S->slots.resize((size_t)cfg->max_inflight);
  for (Slot& sl : S->slots) {
    if (hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&sl.done, hipEventDisableTiming) != hipSuccess ||
        prism_batch_create(&sl.staging) != PRISM_OK) {
      release_all(S);
      delete S;
      return PRISM_EDEVICE;
    }
  }
  S->worker = std::thread(worker_main, S);
  *out = S;
  return PRISM_OK;
}

void prism_server_destroy(prism_server_t S) {
  if (!S) return;
  {
    std::lock_guard<std::mutex> lk(S->mu);
    S->stop = true;
  }
  S->cv_work.notify_all();
  if (S->worker.joinable()) S->worker.join();
  release_all(S);
  delete S;
}

prism_status_t prism_server_add_controller(prism_server_t S, prism_proj_t proj, int32_t max_N,
                                           int32_t* ctrl_id) {
  if (!S || !proj || !ctrl_id || max_N < 1) return PRISM_EINVAL;
  if (proj->device != S->device) return PRISM_EDEVICE;
  const size_t xf = (size_t)max_N * proj->H * proj->nj;
  const size_t bytes = xf * sizeof(float) * 5;      // x [N][H][nj] + q [N][nj][4][H]
  std::lock_guard<std::mutex> lk(S->mu);
  const int id = S->sched.add_controller(bytes, max_N);
  if (id < 0) return PRISM_ENOMEM;
  S->ctrls.push_back(Ctrl{proj, max_N, xf});
  *ctrl_id = id;
  return PRISM_OK;
}

prism_status_t prism_server_submit(prism_server_t S, int32_t ctrl_id, const prism_serve_request_t* r,
                                   int64_t* ticket) {
  if (!S || !r || !ticket) return PRISM_EINVAL;
  Ctrl c;
  {
    std::lock_guard<std::mutex> lk(S->mu);
    if (ctrl_id < 0 || ctrl_id >= (int)S->ctrls.size()) return PRISM_EINVAL;
    c = S->ctrls[(size_t)ctrl_id];
  }
  if (r->N < 0 || r->N > c.max_N || r->iters < 0 || !r->q0 || !r->v0) return PRISM_EINVAL;
  if (r->N > 0 && (!r->v_samples || !r->v_out)) return PRISM_EINVAL;
  JointRowParams tmp[kMaxJoints];
  const prism_status_t st = fill_joint_params(c.p, r->q0, r->v0, tmp);
  if (st != PRISM_OK) return st;

  Ticket k;
  k.ctrl = ctrl_id;
  k.N = r->N;
  k.iters = r->iters;
  k.xin = r->v_samples;
  k.xout = r->v_out;
  k.rp = r->r_primal;
  k.rd = r->r_dual;
  k.itout = r->iters_out;
  k.q0.assign(r->q0, r->q0 + c.p->nj);
  k.v0.assign(r->v0, r->v0 + c.p->nj);
  k.t_submit = mono_ns();
  {
    std::lock_guard<std::mutex> lk(S->mu);
    if (S->stop) return PRISM_EDEVICE;
    const int64_t id = S->next_ticket;
    if (k.N == 0) {
      k.state = PRISM_SERVER_DONE;
      k.t_launch = k.t_done = k.t_submit;
    } else {
      const serve::SubmitResult sr = S->sched.submit(ctrl_id, id, k.N);
      if (sr == serve::kQueueFull) return PRISM_EBUSY;
      if (sr != serve::kQueued) return PRISM_EINVAL;
    }
    ++S->next_ticket;
    ++S->submitted;
    if (k.N == 0) ++S->completed;
    S->tickets.emplace(id, std::move(k));
    *ticket = id;
  }
  S->cv_work.notify_one();
  return PRISM_OK;
}

prism_status_t prism_server_poll(prism_server_t S, int64_t ticket, prism_ticket_info_t* info) {
  if (!S || !info) return PRISM_EINVAL;
  std::lock_guard<std::mutex> lk(S->mu);
  auto it = S->tickets.find(ticket);
  if (it == S->tickets.end()) return PRISM_EINVAL;
  fill_info(it->second, info);
  return PRISM_OK;
}

prism_status_t prism_server_wait(prism_server_t S, int64_t ticket, int64_t timeout_ms,
                                 prism_ticket_info_t* info) {
  if (!S || !info) return PRISM_EINVAL;
  std::unique_lock<std::mutex> lk(S->mu);
  auto finished = [&] {
    auto it = S->tickets.find(ticket);
    return it == S->tickets.end() || it->second.state == PRISM_SERVER_DONE ||
           it->second.state == PRISM_SERVER_FAILED;
  };
  if (timeout_ms < 0) S->cv_done.wait(lk, finished);
  else if (!S->cv_done.wait_for(lk, std::chrono::milliseconds(timeout_ms), finished))
    return PRISM_EBUSY;
  auto it = S->tickets.find(ticket);
  if (it == S->tickets.end()) return PRISM_EINVAL;
  fill_info(it->second, info);
  return PRISM_OK;
}

prism_status_t prism_server_release(prism_server_t S, int64_t ticket) {
  if (!S) return PRISM_EINVAL;
  std::lock_guard<std::mutex> lk(S->mu);
  auto it = S->tickets.find(ticket);
  if (it == S->tickets.end()) return PRISM_EINVAL;
  if (it->second.state == PRISM_SERVER_QUEUED || it->second.state == PRISM_SERVER_RUNNING)
    return PRISM_EBUSY;
  S->tickets.erase(it);
  return PRISM_OK;
}

prism_status_t prism_server_stats(prism_server_t S, prism_server_stats_t* out) {
  if (!S || !out) return PRISM_EINVAL;
  std::lock_guard<std::mutex> lk(S->mu);
  out->submitted = S->submitted;
  out->completed = S->completed;
  out->failed = S->failed;
  out->launches = S->launches;
  out->evictions = (int64_t)S->sched.evictions();
  out->queued = (int64_t)S->sched.queued();
  out->running = S->running;
  out->max_concurrent_launches = S->max_conc;
  out->pool_bytes = (int64_t)S->sched.pool().capacity();
  out->pool_used = (int64_t)S->sched.pool().used();
  return PRISM_OK;
}

}  // extern "C"
