// Flow server behind frg_submit / frg_poll.
//
// Admission: a submitted flow waits in a FIFO queue until a slot is free
// and its device footprint (its share of the staging buffer: U, dU/dt and
// the 7 Jacobian bands of one call) fits the context's HBM budget, so the
// staging buffer of any batch stays within the budget.
//
// Execution: every admitted flow runs the FP64 host stepper in its own
// thread.  Its right-hand-side calls are handed to one dispatcher thread,
// which takes ALL calls pending at that moment -- from any mix of flows,
// grid sizes and N -- and serves them with one batched LPA launch on the
// server's stream (continuous batching: flows join and leave at the
// granularity of a right-hand-side call, and calls that arrive while a batch
// is on the GPU form the next batch).  A flow's result does not depend on
// which flows shared its launches: the kernel evaluates each grid point of
// each flow independently, in a fixed order.
//
// Round trip of a batch: descriptors, the U of every flow and zeroed domain
// flags are packed into one pinned host buffer; the kernel reads them there
// and writes the flags and every flow's outputs back into it (zero copy, one
// launch and one synchronisation per batch; knob server_zero_copy), or the
// packed head goes up in one copy and the flags and outputs come back in
// one (a device mirror of the buffer).  The outputs are then written into
// the waiting flows' own buffers.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <vector>

#include "frg_ctx.h"

namespace frg {

int solve_flow(const frg_request &rq, frg_rhs_fn rhs, void *user, frg_result *res);

struct Server;

struct Flow {
  Server *srv = nullptr;
  uint64_t ticket = 0;
  frg_request req{};
  frg_result res{};
  int64_t n = 0;
  int64_t bytes = 0;
  // right-hand-side hand-off: the stepper's buffers, valid while it waits
  double t = 0.0;
  const double *U_src = nullptr;
  double *dUdt_dst = nullptr;
  double *jac_dst = nullptr;
  bool want_jac = false;
  bool ready = false;
  std::atomic<bool> ready_a{false};  // mirror of ready for waiting without the lock
  int rc = FRG_OK;
  bool done = false;
  std::condition_variable cv;
  std::thread th;
};

struct Server {
  Context *ctx = nullptr;
  hipStream_t stream = nullptr;
  char *h_stage = nullptr;   // pinned, mapped, coherent
  char *hd_stage = nullptr;  // its device address
  char *d_stage = nullptr;   // device mirror (copy mode)
  size_t stage_cap = 0;
  std::mutex m;
  std::condition_variable cv_disp;
  std::deque<Flow *> queue;
  std::vector<Flow *> pending;
  std::atomic<int> n_pending{0};  // size of pending, for waiting without the lock
  std::map<uint64_t, Flow *> flows;
  uint64_t next_ticket = 1;
  int active = 0;
  int max_active = 64;
  size_t max_queue = 65536;
  uint64_t budget = 0;
  uint64_t used = 0;
  bool stop = false;
  std::thread disp;
  int64_t flows_done = 0, launches = 0, batched = 0;

  int start();
  void shutdown();
  void dispatch_loop();
  void admit_locked();
  static int rhs_cb(void *user, double t, const double *U, int64_t n, double *dUdt, double *jac);
  void run_flow(Flow *f);
  bool grow_stage(size_t bytes);
};

// A right-hand side comes back, and the next call arrives, within tens of
// microseconds while flows run; the dispatcher and the steppers poll for
// that long before they sleep on their condition variables (a wake-up
// through the kernel costs about as much as the call itself).
constexpr double kSpinSeconds = 200e-6;

template <class Cond>
static bool spin_until(Cond cond) {
  const auto t0 = std::chrono::steady_clock::now();
  for (int i = 0;; ++i) {
    if (cond()) return true;
    if ((i & 63) == 63 && std::chrono::duration<double>(std::chrono::steady_clock::now() - t0)
                                  .count() > kSpinSeconds)
      return false;
  }
}

int Server::start() {
  if (hipStreamCreateWithFlags(&stream, hipStreamNonBlocking) != hipSuccess)
    return fail(FRG_E_DEVICE, "server stream");
  if (const char *e = std::getenv("FRG_SERVER_SLOTS")) max_active = std::max(1, std::atoi(e));
  disp = std::thread([this] { dispatch_loop(); });
  return FRG_OK;
}

void Server::shutdown() {
  {
    std::lock_guard<std::mutex> lk(m);
    stop = true;
    for (auto &kv : flows) kv.second->cv.notify_all();
  }
  cv_disp.notify_all();
  if (disp.joinable()) disp.join();
  // `flows` owns every flow that has not been polled, admitted or still
  // queued; `queue` only lists the queued ones, so it is cleared without
  // deleting anything
  for (auto &kv : flows) {
    if (kv.second->th.joinable()) kv.second->th.join();
    delete kv.second;
  }
  flows.clear();
  queue.clear();
  if (d_stage) hipFree(d_stage);
  if (h_stage) hipHostFree(h_stage);
  if (stream) hipStreamDestroy(stream);
}

// Dispatcher thread only (no batch in flight): make the staging buffer hold
// `bytes`.
bool Server::grow_stage(size_t bytes) {
  if (bytes <= stage_cap) return true;
  const size_t cap = std::max(bytes, 2 * stage_cap);
  if (d_stage) hipFree(d_stage);
  if (h_stage) hipHostFree(h_stage);
  d_stage = h_stage = hd_stage = nullptr;
  stage_cap = 0;
  if (hipMalloc((void **)&d_stage, cap) != hipSuccess) return false;
  if (hipHostMalloc((void **)&h_stage, cap, hipHostMallocMapped | hipHostMallocCoherent) !=
          hipSuccess ||
      hipHostGetDevicePointer((void **)&hd_stage, h_stage, 0) != hipSuccess) {
    if (h_stage) hipHostFree(h_stage);
    hipFree(d_stage);
    d_stage = h_stage = hd_stage = nullptr;
    return false;
  }
  stage_cap = cap;
  return true;
}

// Under m: start queued flows while slots and budget allow (strict FIFO).
void Server::admit_locked() {
  while (!queue.empty() && active < max_active && !stop) {
    Flow *f = queue.front();
    // the context's own device buffers count against the same budget (a flow
    // is always admitted when none runs: it fitted on its own at submission)
    if (active > 0 && used + (uint64_t)f->bytes + ctx->hbm.used.load() > budget) break;
    queue.pop_front();
    used += f->bytes;
    ++active;
    f->res.start_s = now_s();
    f->th = std::thread([this, f] { run_flow(f); });
  }
}

int Server::rhs_cb(void *user, double t, const double *U, int64_t n, double *dUdt, double *jac) {
  TraceRange trace_("frg_server_rhs");  // a flow thread's right-hand side, queued to its answer
  Flow *f = static_cast<Flow *>(user);
  Server *s = f->srv;
  if (n != f->n) return FRG_E_INVAL;
  {
    std::lock_guard<std::mutex> lk(s->m);
    if (s->stop) return FRG_E_DEVICE;
    f->t = t;
    f->U_src = U;
    f->dUdt_dst = dUdt;
    f->jac_dst = jac;
    f->want_jac = jac != nullptr;
    f->ready = false;
    f->ready_a.store(false, std::memory_order_relaxed);
    s->pending.push_back(f);
    s->n_pending.fetch_add(1, std::memory_order_release);
  }
  s->cv_disp.notify_one();
  if (!spin_until([&] { return f->ready_a.load(std::memory_order_acquire); })) {
    std::unique_lock<std::mutex> lk(s->m);
    f->cv.wait(lk, [&] { return f->ready || s->stop; });
    if (!f->ready) return FRG_E_DEVICE;
  }
  return f->rc;
}

void Server::run_flow(Flow *f) {
  frg_result r{};
  solve_flow(f->req, &Server::rhs_cb, f, &r);
  std::lock_guard<std::mutex> lk(m);
  f->res.status = r.status;
  f->res.steps = r.steps;
  f->res.rejected = r.rejected;
  f->res.rhs_calls = r.rhs_calls;
  f->res.t_reached = r.t_reached;
  f->res.done_s = now_s();
  f->done = true;
  used -= f->bytes;
  --active;
  ++flows_done;
  admit_locked();
}

void Server::dispatch_loop() {
  std::vector<Flow *> batch;
  std::vector<frg_lpa> lpas;
  std::vector<double> ts;
  std::vector<const double *> Us;
  std::vector<double *> Ds, Js;
  std::vector<LpaJob> jobs;
  std::vector<int64_t> start;
  std::vector<size_t> o_u, o_o;
  auto up8 = [](size_t x) { return (x + 7) & ~(size_t)7; };
  hipSetDevice(ctx->device);
  for (;;) {
    batch.clear();
    spin_until([&] { return n_pending.load(std::memory_order_acquire) > 0; });
    {
      std::unique_lock<std::mutex> lk(m);
      cv_disp.wait(lk, [&] { return !pending.empty() || stop; });
      if (stop) return;
      batch.swap(pending);
      n_pending.store(0, std::memory_order_relaxed);
    }
    TraceRange trace_("frg_server_batch");  // staging, one launch, its synchronisation
    const int nb = (int)batch.size();
    lpas.resize(nb);
    ts.resize(nb);
    Us.resize(nb);
    Ds.resize(nb);
    Js.resize(nb);
    jobs.resize(nb);
    start.resize(nb + 1);
    o_u.resize(nb);
    o_o.resize(nb);
    // staging layout: jobs | start | U of each flow | flags | outputs of each
    // flow (dU/dt, then the 7 bands when asked); [0, o_out) goes up,
    // [o_flags, end) comes back
    const size_t o_start = up8(nb * sizeof(LpaJob));
    const size_t o_U = up8(o_start + (nb + 1) * sizeof(int64_t));
    size_t cu = o_U;
    for (int i = 0; i < nb; ++i) {
      o_u[i] = cu;
      cu += batch[i]->n * sizeof(double);
    }
    const size_t o_flags = cu;
    size_t co = up8(o_flags + nb * sizeof(int));
    const size_t o_out = co;
    for (int i = 0; i < nb; ++i) {
      o_o[i] = co;
      co += (batch[i]->want_jac ? 8 : 1) * batch[i]->n * sizeof(double);
    }
    const size_t end = co;
    bool ok = grow_stage(end);
    int rc = ok ? FRG_OK : FRG_E_NOMEM;
    bool zero_copy = false;
    if (ok) {
      {
        std::lock_guard<std::mutex> lk(ctx->mu);
        zero_copy = ctx->tune.server_zero_copy != 0;
      }
      char *dev = zero_copy ? hd_stage : d_stage;  // where the kernel finds the buffer
      for (int i = 0; i < nb; ++i) {
        Flow *f = batch[i];
        lpas[i] = f->req.lpa;
        ts[i] = f->t;
        std::memcpy(h_stage + o_u[i], f->U_src, f->n * sizeof(double));
        Us[i] = (const double *)(dev + o_u[i]);
        Ds[i] = (double *)(dev + o_o[i]);
        Js[i] = f->want_jac ? Ds[i] + f->n : nullptr;
      }
      std::memset(h_stage + o_flags, 0, o_out - o_flags);
      {
        std::lock_guard<std::mutex> lk(ctx->mu);
        rc = ctx->lpa_job_table(nb, lpas.data(), ts.data(), Us.data(), Ds.data(), Js.data(),
                                (int *)(dev + o_flags), jobs.data(), start.data());
      }
      ok = rc == FRG_OK;
      if (ok) {
        std::memcpy(h_stage, jobs.data(), nb * sizeof(LpaJob));
        std::memcpy(h_stage + o_start, start.data(), (nb + 1) * sizeof(int64_t));
        if (zero_copy) {
          ok = launch_lpa((const LpaJob *)dev, (const int64_t *)(dev + o_start), nb, start[nb],
                          stream) == 0;
        } else {
          ok = hipMemcpyAsync(d_stage, h_stage, o_out, hipMemcpyHostToDevice, stream) ==
                   hipSuccess &&
               launch_lpa((const LpaJob *)dev, (const int64_t *)(dev + o_start), nb, start[nb],
                          stream) == 0 &&
               hipMemcpyAsync(h_stage + o_flags, d_stage + o_flags, end - o_flags,
                              hipMemcpyDeviceToHost, stream) == hipSuccess;
        }
        ok = hipStreamSynchronize(stream) == hipSuccess && ok;
        if (!ok) rc = FRG_E_DEVICE;
      }
    }
    if (ok) {
      for (int i = 0; i < nb; ++i) {
        Flow *f = batch[i];
        const double *o = (const double *)(h_stage + o_o[i]);
        std::memcpy(f->dUdt_dst, o, f->n * sizeof(double));
        if (f->want_jac) std::memcpy(f->jac_dst, o + f->n, 7 * f->n * sizeof(double));
      }
    }
    const int *flags = ok ? (const int *)(h_stage + o_flags) : nullptr;
    std::lock_guard<std::mutex> lk(m);
    ++launches;
    batched += nb;
    for (int i = 0; i < nb; ++i) {
      Flow *f = batch[i];
      f->rc = !ok ? rc : (flags[i] ? FRG_E_DOMAIN : FRG_OK);
      f->ready = true;
      f->ready_a.store(true, std::memory_order_release);
      f->cv.notify_one();
    }
  }
}

void Context::stop_server() {
  if (!server) return;
  server->shutdown();
  delete server;
  server = nullptr;
}

}  // namespace frg

using namespace frg;

extern "C" {

int frg_submit(frg_ctx *ctx, const frg_request *req, uint64_t *ticket) {
  frg::TraceRange trace_("frg_submit");
  if (!ctx || !req || !ticket) return fail(FRG_E_INVAL, "NULL argument");
  int rc = check_lpa(req->lpa);
  if (rc) return rc;
  if (!req->U_out) return fail(FRG_E_INVAL, "U_out is NULL");
  if (!std::isfinite(req->t_end) || req->t_end > 0.0) return fail(FRG_E_INVAL, "t_end must be <= 0");
  if (!std::isfinite(req->lambda) || !std::isfinite(req->rho0))
    return fail(FRG_E_INVAL, "bad initial potential");
  Server *s;
  {
    std::lock_guard<std::mutex> lk(ctx->mu);
    if (!ctx->server) {
      auto *ns = new Server();
      ns->ctx = ctx;
      ns->budget = ctx->hbm_budget;
      hipSetDevice(ctx->device);
      rc = ns->start();
      if (rc) {
        delete ns;
        return rc;
      }
      ctx->server = ns;
    }
    s = ctx->server;
  }
  const int64_t bytes = frg_flow_footprint(&req->lpa);
  std::lock_guard<std::mutex> lk(s->m);
  if ((uint64_t)bytes + ctx->hbm.used.load() > s->budget)
    return fail(FRG_E_NOMEM, "flow footprint %lld B and the context's buffers exceed the HBM budget",
                (long long)bytes);
  if (s->queue.size() >= s->max_queue) return fail(FRG_E_AGAIN, "submission queue full");
  Flow *f = new Flow();
  f->srv = s;
  f->ticket = s->next_ticket++;
  f->req = *req;
  f->n = req->lpa.n_grid;
  f->bytes = bytes;
  f->res.status = FRG_PENDING;
  f->res.submit_s = now_s();
  s->flows[f->ticket] = f;
  s->queue.push_back(f);
  s->admit_locked();
  *ticket = f->ticket;
  clear_error();
  return FRG_OK;
}

int frg_poll(frg_ctx *ctx, uint64_t ticket, frg_result *out) {
  if (!ctx || !out) return fail(FRG_E_INVAL, "NULL argument");
  Server *s = ctx->server;
  if (!s) return fail(FRG_E_NOTFOUND, "unknown ticket %llu", (unsigned long long)ticket);
  Flow *f;
  {
    std::lock_guard<std::mutex> lk(s->m);
    auto it = s->flows.find(ticket);
    if (it == s->flows.end()) return fail(FRG_E_NOTFOUND, "unknown ticket %llu", (unsigned long long)ticket);
    f = it->second;
    if (!f->done) {
      *out = f->res;
      out->status = FRG_PENDING;
      return FRG_PENDING;
    }
    s->flows.erase(it);
  }
  if (f->th.joinable()) f->th.join();
  *out = f->res;
  delete f;
  clear_error();
  return FRG_OK;
}

int frg_server_stats(frg_ctx *ctx, int64_t *flows_done, int64_t *launches, double *mean_batch) {
  if (!ctx) return fail(FRG_E_INVAL, "ctx is NULL");
  Server *s = ctx->server;
  int64_t d = 0, l = 0, b = 0;
  if (s) {
    std::lock_guard<std::mutex> lk(s->m);
    d = s->flows_done;
    l = s->launches;
    b = s->batched;
  }
  if (flows_done) *flows_done = d;
  if (launches) *launches = l;
  if (mean_batch) *mean_batch = l ? (double)b / (double)l : 0.0;
  return FRG_OK;
}

}  // extern "C"
