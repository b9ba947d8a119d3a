// Flow server behind frg_submit / frg_poll.
//
// Admission: a submitted flow waits in a FIFO queue until a slot is free
// and its device footprint (its share of a staging buffer: U, dU/dt and the
// 7 Jacobian bands of one call) fits the context's HBM budget, so the
// batches in flight, which never share a flow, stay within the budget
// together.
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
// launch and one event per batch; knob server_zero_copy), or the packed head
// goes up in one copy and the flags and outputs come back in one (a device
// mirror of the buffer).  The outputs are then written into the waiting
// flows' own buffers.  There are two such buffers: while one batch runs, the
// dispatcher stages and enqueues the next into the other, then waits for the
// running one and hands it back.
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

// One staging buffer: the batch's descriptors, inputs, flags and outputs.
struct Stage {
  char *h = nullptr;   // pinned, mapped, coherent
  char *hd = nullptr;  // its device address
  char *d = nullptr;   // device mirror (copy mode)
  size_t cap = 0;
  hipEvent_t done = nullptr;  // recorded after the batch's last operation
};

// A launched batch, until its outputs are handed back.
struct Batch {
  std::vector<Flow *> flows;
  std::vector<size_t> o_o;  // each flow's outputs in the staging buffer
  size_t o_flags = 0;
  int slot = 0;
  int rc = FRG_OK;
};

// With more running flows than spin_flows (environment FRG_SERVER_SPIN_FLOWS,
// default kSpinFlows), the steppers sleep on their condition variables at
// once: a spinning thread per flow would take the cores that the others'
// steppers need.
constexpr int kSpinFlows = 12;

struct Server {
  Context *ctx = nullptr;
  hipStream_t stream = nullptr;
  // two staging buffers: the next batch is staged and enqueued while the
  // previous one runs (at most two batches in flight, handed back in order)
  Stage stg[2];
  std::mutex m;
  std::condition_variable cv_disp;
  std::deque<Flow *> queue;
  std::vector<Flow *> pending;
  std::atomic<int> n_pending{0};  // size of pending, for waiting without the lock
  std::map<uint64_t, Flow *> flows;
  uint64_t next_ticket = 1;
  int active = 0;
  int max_active = 64;
  int spin_flows = kSpinFlows;
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
  bool grow_stage(Stage &g, size_t bytes);
  void launch_batch(Batch &b);
  void finish_batch(Batch &b);
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
  for (Stage &g : stg)
    if (hipEventCreateWithFlags(&g.done, hipEventDisableTiming) != hipSuccess)
      return fail(FRG_E_DEVICE, "server event");
  if (const char *e = std::getenv("FRG_SERVER_SLOTS")) max_active = std::max(1, std::atoi(e));
  if (const char *e = std::getenv("FRG_SERVER_SPIN_FLOWS")) spin_flows = std::max(0, std::atoi(e));
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
  if (stream) (void)hipStreamSynchronize(stream);
  for (Stage &g : stg) {
    if (g.d) (void)hipFree(g.d);
    if (g.h) (void)hipHostFree(g.h);
    if (g.done) (void)hipEventDestroy(g.done);
  }
  if (stream) (void)hipStreamDestroy(stream);
}

// Dispatcher thread only (no batch of this buffer in flight): make the
// staging buffer hold `bytes`.
bool Server::grow_stage(Stage &g, size_t bytes) {
  if (bytes <= g.cap) return true;
  const size_t cap = std::max(bytes, 2 * g.cap);
  if (g.d) (void)hipFree(g.d);
  if (g.h) (void)hipHostFree(g.h);
  g.d = g.h = g.hd = nullptr;
  g.cap = 0;
  if (hipMalloc((void **)&g.d, cap) != hipSuccess) return false;
  if (hipHostMalloc((void **)&g.h, cap, hipHostMallocMapped | hipHostMallocCoherent) !=
          hipSuccess ||
      hipHostGetDevicePointer((void **)&g.hd, g.h, 0) != hipSuccess) {
    if (g.h) (void)hipHostFree(g.h);
    (void)hipFree(g.d);
    g.d = g.h = g.hd = nullptr;
    return false;
  }
  g.cap = cap;
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
  bool spin;
  {
    std::lock_guard<std::mutex> lk(s->m);
    if (s->stop) return FRG_E_DEVICE;
    spin = s->active <= s->spin_flows;
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
  if (!spin || !spin_until([&] { return f->ready_a.load(std::memory_order_acquire); })) {
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

// Stage the batch's right-hand sides into its buffer and enqueue it on the
// server stream: the buffer's layout is jobs | start | U of each flow | flags
// | outputs of each flow (dU/dt, then the 7 bands when asked); [0, o_out)
// goes up and [o_flags, end) comes back (copy mode), or the kernel reads and
// writes the pinned buffer in place (zero copy).  Records the buffer's event.
void Server::launch_batch(Batch &b) {
  TraceRange trace_("frg_server_batch");  // staging and enqueueing one launch
  auto up8 = [](size_t x) { return (x + 7) & ~(size_t)7; };
  const int nb = (int)b.flows.size();
  std::vector<frg_lpa> lpas(nb);
  std::vector<double> ts(nb);
  std::vector<const double *> Us(nb);
  std::vector<double *> Ds(nb), Js(nb);
  std::vector<LpaJob> jobs(nb);
  std::vector<int64_t> start(nb + 1);
  std::vector<size_t> o_u(nb);
  b.o_o.resize(nb);
  const size_t o_start = up8(nb * sizeof(LpaJob));
  const size_t o_U = up8(o_start + (nb + 1) * sizeof(int64_t));
  size_t cu = o_U;
  for (int i = 0; i < nb; ++i) {
    o_u[i] = cu;
    cu += b.flows[i]->n * sizeof(double);
  }
  b.o_flags = cu;
  size_t co = up8(b.o_flags + nb * sizeof(int));
  const size_t o_out = co;
  for (int i = 0; i < nb; ++i) {
    b.o_o[i] = co;
    co += (b.flows[i]->want_jac ? 8 : 1) * b.flows[i]->n * sizeof(double);
  }
  const size_t end = co;
  Stage &g = stg[b.slot];
  if (!grow_stage(g, end)) {
    b.rc = FRG_E_NOMEM;
    return;
  }
  bool zero_copy;
  {
    std::lock_guard<std::mutex> lk(ctx->mu);
    zero_copy = ctx->tune.server_zero_copy != 0;
  }
  char *dev = zero_copy ? g.hd : g.d;  // where the kernel finds the buffer
  for (int i = 0; i < nb; ++i) {
    Flow *f = b.flows[i];
    lpas[i] = f->req.lpa;
    ts[i] = f->t;
    std::memcpy(g.h + o_u[i], f->U_src, f->n * sizeof(double));
    Us[i] = (const double *)(dev + o_u[i]);
    Ds[i] = (double *)(dev + b.o_o[i]);
    Js[i] = f->want_jac ? Ds[i] + f->n : nullptr;
  }
  std::memset(g.h + b.o_flags, 0, o_out - b.o_flags);
  {
    std::lock_guard<std::mutex> lk(ctx->mu);
    b.rc = ctx->lpa_job_table(nb, lpas.data(), ts.data(), Us.data(), Ds.data(), Js.data(),
                              (int *)(dev + b.o_flags), jobs.data(), start.data());
  }
  if (b.rc != FRG_OK) return;
  std::memcpy(g.h, jobs.data(), nb * sizeof(LpaJob));
  std::memcpy(g.h + o_start, start.data(), (nb + 1) * sizeof(int64_t));
  bool ok;
  if (zero_copy) {
    ok = launch_lpa((const LpaJob *)dev, (const int64_t *)(dev + o_start), nb, start[nb],
                    stream) == 0;
  } else {
    ok = hipMemcpyAsync(g.d, g.h, o_out, hipMemcpyHostToDevice, stream) == hipSuccess &&
         launch_lpa((const LpaJob *)dev, (const int64_t *)(dev + o_start), nb, start[nb],
                    stream) == 0 &&
         hipMemcpyAsync(g.h + b.o_flags, g.d + b.o_flags, end - b.o_flags,
                        hipMemcpyDeviceToHost, stream) == hipSuccess;
  }
  ok = ok && hipEventRecord(g.done, stream) == hipSuccess;
  if (!ok) b.rc = FRG_E_DEVICE;
}

// Wait for a launched batch and hand its outputs back to its flows.
void Server::finish_batch(Batch &b) {
  Stage &g = stg[b.slot];
  if (b.rc == FRG_OK && hipEventSynchronize(g.done) != hipSuccess) b.rc = FRG_E_DEVICE;
  const int nb = (int)b.flows.size();
  if (b.rc == FRG_OK) {
    for (int i = 0; i < nb; ++i) {
      Flow *f = b.flows[i];
      const double *o = (const double *)(g.h + b.o_o[i]);
      std::memcpy(f->dUdt_dst, o, f->n * sizeof(double));
      if (f->want_jac) std::memcpy(f->jac_dst, o + f->n, 7 * f->n * sizeof(double));
    }
  }
  const int *flags = b.rc == FRG_OK ? (const int *)(g.h + b.o_flags) : nullptr;
  std::lock_guard<std::mutex> lk(m);
  ++launches;
  batched += nb;
  for (int i = 0; i < nb; ++i) {
    Flow *f = b.flows[i];
    f->rc = b.rc != FRG_OK ? b.rc : (flags[i] ? FRG_E_DOMAIN : FRG_OK);
    f->ready = true;
    f->ready_a.store(true, std::memory_order_release);
    f->cv.notify_one();
  }
}

// Batches of the pending right-hand sides.  With no batch in flight the
// dispatcher waits for work; with one in flight it takes whatever is pending
// right away, stages and enqueues it (behind the running one, into the other
// buffer), and only then waits for the running one and hands it back.
void Server::dispatch_loop() {
  (void)hipSetDevice(ctx->device);
  Batch inflight;
  bool busy = false;
  for (;;) {
    Batch next;
    bool stopping = false;
    if (!busy) {
      spin_until([&] { return n_pending.load(std::memory_order_acquire) > 0; });
      std::unique_lock<std::mutex> lk(m);
      cv_disp.wait(lk, [&] { return !pending.empty() || stop; });
      stopping = stop;
      if (!stopping) {
        next.flows.swap(pending);
        n_pending.store(0, std::memory_order_relaxed);
      }
    } else if (n_pending.load(std::memory_order_acquire) > 0) {  // a stop is seen once idle
      std::lock_guard<std::mutex> lk(m);
      stopping = stop;
      if (!stopping) {
        next.flows.swap(pending);
        n_pending.store(0, std::memory_order_relaxed);
      }
    }
    if (stopping) {
      if (busy) finish_batch(inflight);
      return;
    }
    if (!next.flows.empty()) {
      next.slot = busy ? 1 - inflight.slot : 0;
      launch_batch(next);
    }
    if (busy) {
      finish_batch(inflight);
      busy = false;
    }
    if (!next.flows.empty()) {
      inflight = std::move(next);
      busy = true;
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
      (void)hipSetDevice(ctx->device);
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
