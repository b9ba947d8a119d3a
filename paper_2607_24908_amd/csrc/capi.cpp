// C ABI of libfrg: context, table cache, descriptor staging and the launch
// paths behind frg_integrate, frg_integrate_grid and frg_flow_rhs(_batch).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "device_exp.h"
#include "frg_ctx.h"

namespace frg {

static thread_local std::string g_err;

int fail(int code, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

int hip_fail(hipError_t e, const char *what) {
  return fail(FRG_E_DEVICE, "%s: %s", what, hipGetErrorString(e));
}

void clear_error() { g_err.clear(); }

double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

// ------------------------------------------------------------- DevBuf --
DevBuf::~DevBuf() { release(); }
void DevBuf::release() {
  if (ptr) {
    hipFree(ptr);
    if (acct) acct->used -= bytes;
  }
  ptr = nullptr;
  bytes = 0;
}
int DevBuf::reserve(size_t b) {
  if (b <= bytes) return FRG_OK;
  const size_t nb = std::max<size_t>(b, 256);
  if (acct && acct->used.load() - bytes + nb > acct->budget)
    return fail(FRG_E_NOMEM,
                "a buffer of %zu B would take the context's device buffers (%llu B) beyond its "
                "HBM budget (%llu B)",
                nb, (unsigned long long)acct->used.load(), (unsigned long long)acct->budget);
  release();
  hipError_t e = hipMalloc(&ptr, nb);
  if (e != hipSuccess) {
    ptr = nullptr;
    return fail(FRG_E_NOMEM, "hipMalloc(%zu): %s", nb, hipGetErrorString(e));
  }
  bytes = nb;
  if (acct) acct->used += nb;
  return FRG_OK;
}

// --------------------------------------------------------------- ring --
int DescRing::init(size_t slot_bytes_, int n_slots) {
  slot_bytes = slot_bytes_;
  slots.resize(n_slots);
  for (auto &s : slots) {
    if (hipHostMalloc(&s.host, slot_bytes, hipHostMallocDefault) != hipSuccess)
      return fail(FRG_E_NOMEM, "hipHostMalloc descriptor ring");
    if (hipMalloc(&s.dev, slot_bytes) != hipSuccess)
      return fail(FRG_E_NOMEM, "hipMalloc descriptor ring");
    if (hipEventCreateWithFlags(&s.done, hipEventDisableTiming) != hipSuccess)
      return fail(FRG_E_DEVICE, "hipEventCreate");
    s.used = false;
    s.cap = slot_bytes;
  }
  return FRG_OK;
}

void DescRing::destroy() {
  for (auto &s : slots) {
    if (s.used) hipEventSynchronize(s.done);
    if (s.host) hipHostFree(s.host);
    if (s.dev) hipFree(s.dev);
    if (s.done) hipEventDestroy(s.done);
    s = Slot{};
  }
  slots.clear();
}

// Copy `bytes` of host data into the next slot and enqueue the upload on
// `stream`; the returned device pointer stays valid until the slot comes
// round again, which first waits for the event recorded by release().
int DescRing::upload(const void *src, size_t bytes, hipStream_t stream, void **dev, int *slot_id) {
  Slot &s = slots[next];
  if (s.used) {
    hipError_t e = hipEventSynchronize(s.done);
    if (e != hipSuccess) return hip_fail(e, "hipEventSynchronize(ring)");
    s.used = false;
  }
  if (bytes > s.cap) {  // grow this slot (its previous use has completed)
    const size_t cap = std::max(bytes, 2 * s.cap);
    void *h = nullptr, *d = nullptr;
    if (hipHostMalloc(&h, cap, hipHostMallocDefault) != hipSuccess)
      return fail(FRG_E_NOMEM, "hipHostMalloc descriptor ring (%zu B)", cap);
    if (hipMalloc(&d, cap) != hipSuccess) {
      hipHostFree(h);
      return fail(FRG_E_NOMEM, "hipMalloc descriptor ring (%zu B)", cap);
    }
    hipHostFree(s.host);
    hipFree(s.dev);
    s.host = h;
    s.dev = d;
    s.cap = cap;
  }
  std::memcpy(s.host, src, bytes);
  hipError_t e = hipMemcpyAsync(s.dev, s.host, bytes, hipMemcpyHostToDevice, stream);
  if (e != hipSuccess) return hip_fail(e, "hipMemcpyAsync(descriptors)");
  *dev = s.dev;
  *slot_id = next;
  next = (next + 1) % (int)slots.size();
  return FRG_OK;
}

int DescRing::release(int slot_id, hipStream_t stream) {
  Slot &s = slots[slot_id];
  hipError_t e = hipEventRecord(s.done, stream);
  if (e != hipSuccess) return hip_fail(e, "hipEventRecord(ring)");
  s.used = true;
  return FRG_OK;
}

// ------------------------------------------------------------- tables --
static uint64_t dbits(double x) {
  uint64_t u;
  std::memcpy(&u, &x, 8);
  return u;
}

int Ctx::quad_table(const frg_quad &q, const double **dev, QuadTable *host_copy,
                    QuadTable **host_ref) {
  auto key = std::make_tuple(q.d, q.reg, dbits(q.k), dbits(q.q_max), q.n_radial, q.n_angular);
  auto it = qtabs.find(key);
  if (it == qtabs.end()) {
    QuadTable t = build_quad_table(q);
    auto buf = std::make_unique<DevBuf>(&hbm);
    int rc = buf->reserve(t.data.size() * sizeof(double));
    if (rc) return rc;
    hipError_t e = hipMemcpy(buf->ptr, t.data.data(), t.data.size() * sizeof(double),
                             hipMemcpyHostToDevice);
    if (e != hipSuccess) return hip_fail(e, "upload quadrature table");
    QEntry ent;
    ent.buf = std::move(buf);
    ent.host = std::move(t);
    it = qtabs.emplace(key, std::move(ent)).first;
  }
  *dev = (const double *)it->second.buf->ptr;
  if (host_copy) *host_copy = it->second.host;
  if (host_ref) *host_ref = &it->second.host;
  return FRG_OK;
}

int Ctx::lpa_table(int d, int reg, int n_r, double qmk, const double **dev, double *Cd) {
  auto key = std::make_tuple(d, reg, n_r, dbits(qmk));
  auto it = ltabs.find(key);
  if (it == ltabs.end()) {
    LpaTable t = build_lpa_table(d, reg, n_r, qmk);
    auto buf = std::make_unique<DevBuf>(&hbm);
    int rc = buf->reserve(t.data.size() * sizeof(double));
    if (rc) return rc;
    hipError_t e = hipMemcpy(buf->ptr, t.data.data(), t.data.size() * sizeof(double),
                             hipMemcpyHostToDevice);
    if (e != hipSuccess) return hip_fail(e, "upload LPA table");
    LEntry ent;
    ent.buf = std::move(buf);
    ent.Cd = t.Cd;
    it = ltabs.emplace(key, std::move(ent)).first;
  }
  *dev = (const double *)it->second.buf->ptr;
  *Cd = it->second.Cd;
  return FRG_OK;
}

// ------------------------------------------------------------ validation --
int check_quad(const frg_quad &q) {
  if (q.d < 3 || q.d > 8) return fail(FRG_E_INVAL, "quad.d=%d outside [3, 8]", q.d);
  if (q.reg != FRG_REG_EXP && q.reg != FRG_REG_LITIM)
    return fail(FRG_E_INVAL, "quad.reg=%d unknown", q.reg);
  if (!(q.k > 0.0) || !std::isfinite(q.k)) return fail(FRG_E_INVAL, "quad.k must be > 0");
  if (!(q.q_max > 0.0) || !std::isfinite(q.q_max))
    return fail(FRG_E_INVAL, "quad.q_max must be > 0");
  if (q.n_radial < 1 || q.n_radial > 1024)
    return fail(FRG_E_INVAL, "quad.n_radial=%d outside [1, 1024]", q.n_radial);
  if (q.n_angular < 1 || q.n_angular > 256)
    return fail(FRG_E_INVAL, "quad.n_angular=%d outside [1, 256]", q.n_angular);
  if (q.prec != FRG_PREC_FP64 && q.prec != FRG_PREC_FP32C)
    return fail(FRG_E_INVAL, "quad.prec=%d unknown", q.prec);
  if (q.reserved != 0) return fail(FRG_E_INVAL, "quad.reserved must be 0");
  return FRG_OK;
}

int check_lpa(const frg_lpa &l) {
  if (l.d < 2 || l.d > 8) return fail(FRG_E_INVAL, "lpa.d=%d outside [2, 8]", l.d);
  if (l.N < 1) return fail(FRG_E_INVAL, "lpa.N must be >= 1");
  if (l.reg != FRG_REG_EXP && l.reg != FRG_REG_LITIM) return fail(FRG_E_INVAL, "lpa.reg unknown");
  if (l.n_radial < 1 || l.n_radial > 1024) return fail(FRG_E_INVAL, "lpa.n_radial outside [1, 1024]");
  if (!(l.q_max_over_k > 0.0)) return fail(FRG_E_INVAL, "lpa.q_max_over_k must be > 0");
  if (!(l.Lambda > 0.0)) return fail(FRG_E_INVAL, "lpa.Lambda must be > 0");
  if (l.n_grid < 4 || l.n_grid > 65536) return fail(FRG_E_INVAL, "lpa.n_grid outside [4, 65536]");
  if (!(l.rho_max > 0.0) || !std::isfinite(l.rho_max)) return fail(FRG_E_INVAL, "lpa.rho_max must be > 0");
  return FRG_OK;
}

// ----------------------------------------------------------- integrate --
// Descriptor of set s with its quadrature table `h` at device address `tab`.
void Ctx::fill_setdev(const frg_set &s, const QuadTable &h, const double *tab, SetDev *out) {
  SetDev d{};
  d.p = s.p;
  d.m2 = s.m2;
  d.out = s.out;
  d.err = s.err_est;
  d.used64 = s.used_fp64;
  d.tab = tab;
  d.k2 = h.k2;
  d.inv_k2 = h.inv_k2;
  d.pref = h.pref;
  d.pref_k = h.pref * h.inv_k2;
  d.q_top = h.q_top;
  d.rmu_max = h.rmu_max;
  d.n_ext = s.n_ext;
  d.n_r = s.quad.n_radial;
  d.n_a = s.quad.n_angular;
  d.reg = s.quad.reg;
  d.prec = s.quad.prec;
  d.f32_flag = tune.fp32c_flag_ppb * 1e-9;
  d.f32_band = tune.fp32c_band_ppm * 1e-6;
  lane_split(d.n_r, d.n_a, &d.R, &d.J, &d.T, &d.U);
  *out = d;
}

int Ctx::replay_graph(const frg_set *sets, int n_sets, hipStream_t st) {
  for (auto &g : graphs) {
    if (g->stream != st || g->flag != d_flag || g->gen != tune_gen ||
        g->raw.size() != (size_t)n_sets ||
        (n_sets && std::memcmp(g->raw.data(), sets, n_sets * sizeof(frg_set)) != 0))
      continue;
    hipError_t e = hipGraphLaunch(g->exec, st);
    if (e == hipSuccess) e = hipEventRecord(g->done, st);
    if (e != hipSuccess) return hip_fail(e, "hipGraphLaunch");
    g->last_use = ++graph_clock;
    return 1;
  }
  return 0;
}

int Ctx::make_setdev(const frg_set &s, SetDev *out) {
  const double *tab;
  QuadTable *hp = nullptr;
  int rc = quad_table(s.quad, &tab, nullptr, &hp);
  if (rc) return rc;
  fill_setdev(s, *hp, tab, out);
  return FRG_OK;
}

// Device-side core: every pointer in `sets` is device memory.
int Ctx::integrate_device(const frg_set *sets, int n_sets, int flags, hipStream_t st) {
  if ((flags & FRG_PERSISTENT) && (flags & FRG_GRAPH)) {
    const int r = replay_graph(sets, n_sets, st);
    if (r) return r < 0 ? r : FRG_OK;
  }
  std::vector<SetDev> sd(n_sets);
  for (int i = 0; i < n_sets; ++i) {
    int rc = make_setdev(sets[i], &sd[i]);
    if (rc) return rc;
  }
  if (!(flags & FRG_PERSISTENT)) {
    for (int i = 0; i < n_sets; ++i) {
      if (sd[i].n_ext == 0) continue;
      int e = launch_points_plain(sd[i], plain_tile_for(sd[i], st), d_flag, st);
      if (e) return hip_fail((hipError_t)e, "points_plain_kernel launch");
    }
    return FRG_OK;
  }
  return persistent(sd, sets, n_sets, flags, st);
}

// Points per tile of a set: about tile_k * 1024 evaluations per tile (1..64
// points), so that tiles of every set cost about the same.
static int tile_points(const SetDev &s, int tile_k) {
  const double per = (double)s.n_r * s.n_a;
  const int tp = (int)std::floor((double)tile_k * 1024.0 / per);
  return std::max(1, std::min(64, tp));
}

// Work list, longest tile first (weight = per-point cost x points; ties in
// set order, then point order).  All full tiles of a set weigh the same, so
// a stable sort of runs -- the full tiles of a set, then its last partial
// tile -- gives the order of a stable sort of the tiles without sorting them
// one by one.
void build_tiles(const std::vector<SetDev> &sd, int tile_k, std::vector<Tile> *tiles) {
  struct Run {
    double w;
    int set, tp;
    int64_t start, count;  // tiles [start, start + count * tp) of `set`
  };
  std::vector<Run> runs;
  runs.reserve(2 * sd.size());
  int64_t n_tiles = 0;
  for (int i = 0; i < (int)sd.size(); ++i) {
    // cost per evaluation: exponential regulator about three times Litim (FP32C alike)
    const double w = sd[i].reg == FRG_REG_EXP ? 3.0 : 1.0;
    const double per = w * sd[i].n_r * sd[i].n_a;
    const int tp = tile_points(sd[i], tile_k);
    const int64_t full = sd[i].n_ext / tp, rem = sd[i].n_ext - full * tp;
    if (full) runs.push_back({per * tp, i, tp, 0, full});
    if (rem) runs.push_back({per * rem, i, tp, full * tp, 1});
    n_tiles += full + (rem ? 1 : 0);
  }
  std::stable_sort(runs.begin(), runs.end(), [](const Run &a, const Run &b) { return a.w > b.w; });
  tiles->resize(n_tiles);
  int64_t k = 0;
  for (const Run &r : runs) {
    for (int64_t c = 0; c < r.count; ++c) {
      Tile &t = (*tiles)[k++];
      t.set = r.set;
      t.start = r.start + c * r.tp;
      t.count = (int)std::min<int64_t>(r.tp, sd[r.set].n_ext - t.start);
    }
  }
}

bool any_fp32c(const std::vector<SetDev> &sd) {
  for (auto &s : sd)
    if (s.prec == FRG_PREC_FP32C) return true;
  return false;
}

// LDS bytes the persistent kernel needs for the largest tables of the batch
// (angular pairs and packed table; the launch adds the exponential table).
int max_table_bytes(const std::vector<SetDev> &sd) {
  size_t m = 0;
  for (auto &s : sd) {
    const size_t b = sizeof(double) * (2 * s.n_a + table_doubles(s.n_r, s.n_a));
    m = std::max(m, b);
  }
  return (int)m;
}

static bool same_sets(const std::vector<SetDev> &a, const std::vector<SetDev> &b) {
  return a.size() == b.size() &&
         (a.empty() || std::memcmp(a.data(), b.data(), a.size() * sizeof(SetDev)) == 0);
}

GraphEntry::~GraphEntry() {
  if (done) {
    hipEventSynchronize(done);
    hipEventDestroy(done);
  }
  if (exec) hipGraphExecDestroy(exec);
}

int Ctx::persistent(const std::vector<SetDev> &sd, const frg_set *sets, int n_sets, int flags,
                    hipStream_t st) {
  const bool graph = (flags & FRG_GRAPH) != 0;
  const PersistCfg pc = persist_cfg(sd, sd.empty() ? 0 : sd[0].prec, st);
  if (!graph) return persistent_eager(sd, pc, st);
  for (auto &g : graphs) {
    if (g->stream != st || g->flag != d_flag || g->pc.tile != pc.tile || g->pc.wpc != pc.wpc ||
        !same_sets(g->sd, sd))
      continue;
    hipError_t e = hipGraphLaunch(g->exec, st);
    if (e == hipSuccess) e = hipEventRecord(g->done, st);
    if (e != hipSuccess) return hip_fail(e, "hipGraphLaunch");
    g->last_use = ++graph_clock;
    g->raw.assign(sets, sets + n_sets);
    g->gen = tune_gen;
    return FRG_OK;
  }
  std::vector<Tile> tiles;
  build_tiles(sd, pc.tile, &tiles);
  if (tiles.empty()) return FRG_OK;
  const int lds = max_table_bytes(sd);
  if (lds > 60 * 1024) return fail(FRG_E_INVAL, "quadrature tables exceed 60 KiB of LDS");
  const int n_blocks = std::max(1, std::min<int>((int)tiles.size(), n_cu * pc.wpc));
  if (graphs.size() >= kMaxGraphs) {  // drop the least recently used capture
    auto lru = std::min_element(graphs.begin(), graphs.end(), [](const auto &x, const auto &y) {
      return x->last_use < y->last_use;
    });
    graphs.erase(lru);
  }
  auto g = std::make_unique<GraphEntry>();
  g->sets.acct = g->tiles.acct = g->counter.acct = &hbm;
  int rc = g->sets.reserve(sd.size() * sizeof(SetDev));
  if (!rc) rc = g->tiles.reserve(tiles.size() * sizeof(Tile));
  if (!rc) rc = g->counter.reserve(kCounterInts * sizeof(int));
  if (rc) return rc;
  hipError_t e = hipEventCreateWithFlags(&g->done, hipEventDisableTiming);
  if (e != hipSuccess) return hip_fail(e, "hipEventCreate(graph)");
  e = hipMemcpy(g->sets.ptr, sd.data(), sd.size() * sizeof(SetDev), hipMemcpyHostToDevice);
  if (e == hipSuccess)
    e = hipMemcpy(g->tiles.ptr, tiles.data(), tiles.size() * sizeof(Tile), hipMemcpyHostToDevice);
  if (e != hipSuccess) return hip_fail(e, "upload graph work list");
  e = hipStreamBeginCapture(cap_stream, hipStreamCaptureModeThreadLocal);
  if (e != hipSuccess) return hip_fail(e, "hipStreamBeginCapture");
  // the counters are cleared by a kernel inside the graph (no memset node)
  int e1 = launch_reset_counter((int *)g->counter.ptr, cap_stream);
  int e2 = launch_points_persistent((const SetDev *)g->sets.ptr, (const Tile *)g->tiles.ptr,
                                    (int)tiles.size(), (int *)g->counter.ptr, lds, n_blocks,
                                    any_fp32c(sd), d_flag, cap_stream);
  hipGraph_t graph_h = nullptr;
  e = hipStreamEndCapture(cap_stream, &graph_h);
  if (e1 || e2 || e != hipSuccess) {
    if (graph_h) hipGraphDestroy(graph_h);
    return fail(FRG_E_DEVICE, "graph capture of the persistent launch failed");
  }
  e = hipGraphInstantiate(&g->exec, graph_h, nullptr, nullptr, 0);
  hipGraphDestroy(graph_h);
  if (e != hipSuccess) return hip_fail(e, "hipGraphInstantiate");
  e = hipGraphLaunch(g->exec, st);
  if (e == hipSuccess) e = hipEventRecord(g->done, st);
  if (e != hipSuccess) return hip_fail(e, "hipGraphLaunch");
  g->stream = st;
  g->flag = d_flag;
  g->sd = sd;
  g->pc = pc;
  g->last_use = ++graph_clock;
  g->raw.assign(sets, sets + n_sets);
  g->gen = tune_gen;
  graphs.push_back(std::move(g));
  return FRG_OK;
}

// Eager persistent launch: work list, descriptors and zeroed work-list
// counters go through the ring, so every launch has its own counters (a ring
// slot is reused only after the launch that read it has completed).
int Ctx::persistent_eager(const std::vector<SetDev> &sd, const PersistCfg &pc, hipStream_t st) {
  std::vector<Tile> tiles;
  build_tiles(sd, pc.tile, &tiles);
  if (tiles.empty()) return FRG_OK;
  const int lds = max_table_bytes(sd);
  if (lds > 60 * 1024) return fail(FRG_E_INVAL, "quadrature tables exceed 60 KiB of LDS");
  const int n_blocks = std::max(1, std::min<int>((int)tiles.size(), n_cu * pc.wpc));
  const size_t o_tiles = sd.size() * sizeof(SetDev);
  const size_t o_counter = (o_tiles + tiles.size() * sizeof(Tile) + 255) & ~(size_t)255;
  std::vector<char> blob(o_counter + kCounterInts * sizeof(int), 0);
  std::memcpy(blob.data(), sd.data(), o_tiles);
  std::memcpy(blob.data() + o_tiles, tiles.data(), tiles.size() * sizeof(Tile));
  void *dev;
  int slot;
  int rc = ring.upload(blob.data(), blob.size(), st, &dev, &slot);
  if (rc) return rc;
  const SetDev *d_sets = (const SetDev *)dev;
  const Tile *d_tiles = (const Tile *)((char *)dev + o_tiles);
  int *d_counter = (int *)((char *)dev + o_counter);
  int e2 = launch_points_persistent(d_sets, d_tiles, (int)tiles.size(), d_counter, lds, n_blocks,
                                    any_fp32c(sd), d_flag, st);
  rc = ring.release(slot, st);
  if (e2) return fail(FRG_E_DEVICE, "persistent launch failed");
  return rc;
}

// Host-memory wrapper: stage inputs, run on the context stream, copy back.
int Ctx::integrate_host(const frg_set *sets, int n_sets, int flags) {
  size_t in_bytes = 0, out_bytes = 0, aux_bytes = 0;
  for (int i = 0; i < n_sets; ++i) {
    in_bytes += 2 * sets[i].n_ext * sizeof(double);
    out_bytes += sets[i].n_ext * sizeof(double);
    aux_bytes += sets[i].n_ext * (sizeof(double) + 1);
  }
  int rc = stage_in.reserve(in_bytes + 64);
  if (!rc) rc = stage_out.reserve(out_bytes + aux_bytes + 64);
  if (rc) return rc;
  std::vector<frg_set> dsets(sets, sets + n_sets);
  char *pin = (char *)stage_in.ptr;
  char *pout = (char *)stage_out.ptr;
  size_t oin = 0, oout = 0;
  for (int i = 0; i < n_sets; ++i) {
    const size_t nb = sets[i].n_ext * sizeof(double);
    dsets[i].p = (const double *)(pin + oin);
    hipMemcpyAsync(pin + oin, sets[i].p, nb, hipMemcpyHostToDevice, stream);
    oin += nb;
    dsets[i].m2 = (const double *)(pin + oin);
    hipMemcpyAsync(pin + oin, sets[i].m2, nb, hipMemcpyHostToDevice, stream);
    oin += nb;
    dsets[i].out = (double *)(pout + oout);
    oout += nb;
    if (sets[i].err_est) {
      dsets[i].err_est = (double *)(pout + oout);
      oout += nb;
    }
    if (sets[i].used_fp64) {
      dsets[i].used_fp64 = (uint8_t *)(pout + oout);
      oout += sets[i].n_ext;
      oout = (oout + 7) & ~(size_t)7;
    }
  }
  hipMemsetAsync(d_flag, 0, sizeof(int), stream);
  rc = integrate_device(dsets.data(), n_sets, flags & ~FRG_GRAPH, stream);
  if (rc) {
    hipStreamSynchronize(stream);
    return rc;
  }
  for (int i = 0; i < n_sets; ++i) {
    const size_t nb = sets[i].n_ext * sizeof(double);
    hipMemcpyAsync(sets[i].out, dsets[i].out, nb, hipMemcpyDeviceToHost, stream);
    if (sets[i].err_est) hipMemcpyAsync(sets[i].err_est, dsets[i].err_est, nb, hipMemcpyDeviceToHost, stream);
    if (sets[i].used_fp64)
      hipMemcpyAsync(sets[i].used_fp64, dsets[i].used_fp64, sets[i].n_ext, hipMemcpyDeviceToHost, stream);
  }
  int flag = 0;
  hipMemcpyAsync(&flag, d_flag, sizeof(int), hipMemcpyDeviceToHost, stream);
  hipError_t e = hipStreamSynchronize(stream);
  if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
  if (flag) return fail(FRG_E_DOMAIN, "some points have m^2 + k^2 <= 0 (or p < 0); their results are NaN");
  return FRG_OK;
}

// ---------------------------------------------------------------- grid --
// FRG_PREC_FP32C grids run the FP64 grid kernel and mark every result as
// FP64 (err 1e-14, used64 1): on this GPU an unpacked FP32 operation issues at
// the FP64 rate, and the FP64 grid form runs its power sums on the matrix
// cores, so no FP32 form of the grid is faster.
int Ctx::grid_device(const frg_quad &q_in, int64_t n_p, const double *p, int64_t n_m,
                     const double *m2, double *out, double *err, uint8_t *used, hipStream_t st) {
  frg_quad q = q_in;
  q.prec = FRG_PREC_FP64;
  const double *tab;
  QuadTable h;
  int rc = quad_table(q, &tab, &h);
  if (rc) return rc;
  GridArgs g{};
  g.p = p;
  g.m2 = m2;
  g.out = out;
  g.tab = tab;
  g.flag = d_flag;
  g.k2 = h.k2;
  g.inv_k2 = h.inv_k2;
  g.pref = h.pref;
  g.q_top = h.q_top;
  g.rmu_max = h.rmu_max;
  set_fold_scale(g, h);
  g.n_p = n_p;
  g.n_m = n_m;
  g.n_r = q.n_radial;
  g.n_a = q.n_angular;
  lane_split(g.n_r, g.n_a, &g.R, &g.J, &g.T, &g.U);
  g.chunk = std::max(8, tune.grid_lds_rows);
  g.form = tune.grid_form;
  if (grid_lds_bytes(g) > 64 * 1024) return fail(FRG_E_INVAL, "grid tables exceed 64 KiB of LDS");
  const GridCfg cfg = grid_cfg(q, g, st);
  rc = grid_launch(g, q.reg, cfg, st);
  if (rc || q_in.prec != FRG_PREC_FP32C) return rc;
  const int e = launch_fp64_marks(err, used, n_p * n_m, st);
  if (e) return hip_fail((hipError_t)e, "fp64_marks_kernel launch");
  return FRG_OK;
}

int Ctx::grid_launch(GridArgs g, int reg, const GridCfg &cfg_in, hipStream_t st) {
  const bool resident = grid_resident(g);
  GridCfg cfg = cfg_in;
  // coefficient form: tiles of 16 masses on the matrix cores, or at most 8
  // masses per wave on the vector units
  if (grid_uses_coef(g)) cfg.M = tune.grid_mfma ? 16 : std::min(cfg.M, 8);
  const int64_t per_wg_min = (int64_t)cfg.M * cfg.W;
  // mass blocks per wave: fewer workgroups per momentum, but keep at least
  // ~4 workgroups per CU in flight
  int mbk = resident ? std::max(1, cfg.MB) : 1;
  while (mbk > 1 && g.n_p * ((g.n_m + per_wg_min * mbk - 1) / (per_wg_min * mbk)) < 4LL * n_cu)
    mbk /= 2;
  if (grid_uses_coef(g))
    while (mbk > 1 && grid_coef_stage_bytes(mbk, cfg.W, cfg.M) > kGridCoefStageMax) mbk /= 2;
  g.mblocks = mbk;
  g.n_mb = (int)((g.n_m + per_wg_min * mbk - 1) / (per_wg_min * mbk));
  const int e = launch_grid(g, reg, cfg.M, cfg.W, st);
  if (e) return hip_fail((hipError_t)e, "grid_kernel launch");
  return FRG_OK;
}

// ------------------------------------------------------ tabulated G --
int Ctx::tab_device(const frg_quad &q, const frg_gtab &tb, int64_t n_p, const double *p,
                    double *out, hipStream_t st) {
  const double *tab;
  QuadTable h;
  int rc = quad_table(q, &tab, &h);
  if (rc) return rc;
  TabArgs a{};
  a.p = p;
  a.out = out;
  a.g = tb.g;
  a.tab = tab;
  a.flag = d_flag;
  a.pref = h.pref;
  a.k2 = h.k2;
  a.inv_h = (double)(tb.n_s - 1) / tb.s_max;
  a.t_last = (double)(tb.n_s - 1);
  a.n_p = n_p;
  a.n_rows = tb.n_rows;
  a.n_s = tb.n_s;
  a.os_p = tb.n_rows;
  a.os_r = 1;
  a.n_r = q.n_radial;
  a.n_a = q.n_angular;
  return tab_launch(a, q.reg, st);
}

// Launch shape of tab_kernel for the problem in `a` (p, out, g, tab, flag,
// pref, k2, inv_h, t_last, n_p, n_rows, n_s, os_p, os_r, n_r, n_a set by the
// caller).
int Ctx::tab_config(TabArgs &a, bool &lds_rows_out, int &W_out, int64_t &sblocks_out,
                    bool multi_rows) {
  const int64_t n_p = a.n_p;
  tab_lane_split(a.n_r, a.n_a, &a.R, &a.J, &a.T, &a.U);
  a.pairs = tune.tab_pairs ? 1 : 0;
  a.rb = 1;
  const bool lds_rows = a.n_s <= std::min<int64_t>(tune.tab_lds_nodes, tab_lds_max_nodes) &&
                        tab_lds_bytes(a, true) <= 150 * 1024;
  // rows in LDS: several rows per workgroup share every coordinate (knob
  // tab_rb; auto: two rows when there are two and the LDS holds them, which
  // measured fastest; four rows of plain values were no faster than two)
  if (lds_rows && multi_rows) {
    for (int rb : {4, 2}) {
      if (tune.tab_rb ? tune.tab_rb != rb : (rb != 2 || a.n_rows < rb)) continue;
      TabArgs b = a;
      b.rb = rb;
      if (tab_lds_bytes(b, true) <= 150 * 1024) {
        a.rb = rb;
        break;
      }
    }
  }
  const int W = a.rb > 1 ? std::max(1, std::min(16, tune.tab_rW))
                         : std::max(1, std::min(4, lds_rows ? tune.tab_W : tune.tab_sW));
  a.pw = std::max(1, std::min(64, lds_rows ? tune.tab_pw : tune.tab_spw));
  // streamed rows: tab_wpc workgroups per CU work through the rows of their
  // XCD one at a time; momentum blocks are made small enough that every
  // workgroup of an XCD has a share of each row
  const int64_t sblocks = (int64_t)n_cu * std::max(1, tune.tab_wpc);
  if (!lds_rows) {
    const int64_t slots = std::max<int64_t>(1, sblocks / 8);
    const int64_t fit = n_p / ((int64_t)W * slots);
    a.pw = (int)std::max<int64_t>(1, std::min<int64_t>(a.pw, fit));
  }
  a.n_pb = (int)((n_p + (int64_t)W * a.pw - 1) / ((int64_t)W * a.pw));
  // rows in LDS: small problems take fewer momenta per wave so that about
  // four workgroups per CU (one with several rows per workgroup) are in flight
  const int64_t n_groups = (a.n_rows + a.rb - 1) / a.rb;
  const int64_t want_wg = (a.rb > 1 ? 1LL : 4LL) * n_cu;
  while (lds_rows && a.pw > 1 && n_groups * a.n_pb < want_wg) {
    a.pw /= 2;
    a.n_pb = (int)((n_p + (int64_t)W * a.pw - 1) / ((int64_t)W * a.pw));
  }
  if (a.n_rows * a.n_pb > ((int64_t)1 << 31) - 1) return fail(FRG_E_INVAL, "tabulated problem too large");
  lds_rows_out = lds_rows;
  W_out = W;
  sblocks_out = sblocks;
  return FRG_OK;
}

int Ctx::tab_launch(TabArgs a, int reg, hipStream_t st) {
  bool lds_rows = false;
  int W = 1;
  int64_t sblocks = 0;
  int rc = tab_config(a, lds_rows, W, sblocks, true);
  if (rc) return rc;
  // knob tab_seg: 1 always, 2 (auto) when the table is larger than the
  // chip's memory-side cache: smaller tables are served from that cache and
  // the cache-streamed form is faster there (measured crossover: 2^20-node
  // rows, about 48 of them)
  const bool big = 8.0 * (double)a.n_rows * (double)a.n_s > kTabSegAutoBytes;
  if (!lds_rows && (tune.tab_seg == 1 || (tune.tab_seg == 2 && big))) {
    // segmented form, when its tables fit: LDS, superchunk count, term index
    // in 16 bits, counts in 32 bits, partial sums and term lists up to 1 GiB
    // each; in the auto mode also the HBM budget
    const TabSegShape s = tab_seg_shape(a, n_cu);
    const double part_bytes = 8.0 * s.n_super * (double)a.n_rows * (double)a.n_p;
    const double terms_bytes = 2.0 * (double)a.n_p * a.n_r * a.n_a;
    const double offs_bytes = 4.0 * (double)a.n_p * (s.n_seg + 1);
    const size_t scr_bytes = sizeof(unsigned) * (s.n_super + 64);
    bool fits = s.lds <= 160 * 1024 && s.n_super <= kTabSegMaxSuper && a.n_r * a.n_a <= 65536 &&
                (double)a.n_p * a.n_r * a.n_a < 4.0e9 && part_bytes <= (double)(1u << 30) &&
                terms_bytes <= (double)(1u << 30) && offs_bytes <= (double)(1u << 30);
    if (fits && tune.tab_seg == 2) {
      auto grow = [](const DevBuf &b, double need) {
        return need > (double)b.bytes ? std::max(need, 256.0) - (double)b.bytes : 0.0;
      };
      const double more = grow(tab_part, part_bytes) + grow(tab_terms, terms_bytes) +
                          grow(tab_offs, offs_bytes) + grow(tab_scr, (double)scr_bytes);
      fits = (double)hbm.used.load() + more <= (double)hbm.budget;
    }
    if (fits) {
      // the buffers are the context's: a launch on another stream waits for
      // the previous one (a reallocation waits for the device)
      if (!tab_done && hipEventCreateWithFlags(&tab_done, hipEventDisableTiming) != hipSuccess) {
        tab_done = nullptr;
        return fail(FRG_E_DEVICE, "hipEventCreate");
      }
      if (tab_part.bytes < (size_t)part_bytes || tab_terms.bytes < (size_t)terms_bytes ||
          tab_offs.bytes < (size_t)offs_bytes || tab_scr.bytes < scr_bytes)
        hipEventSynchronize(tab_done);
      rc = tab_part.reserve((size_t)part_bytes);
      if (!rc) rc = tab_terms.reserve((size_t)terms_bytes);
      if (!rc) rc = tab_offs.reserve((size_t)offs_bytes);
      if (!rc) rc = tab_scr.reserve(scr_bytes);
      if (rc) return rc;
      hipError_t he = hipStreamWaitEvent(st, tab_done, 0);
      if (he != hipSuccess) return hip_fail(he, "hipStreamWaitEvent");
      TabSegBufs bufs;
      bufs.part = (double *)tab_part.ptr;
      bufs.terms = (uint16_t *)tab_terms.ptr;
      bufs.offs = (int *)tab_offs.ptr;
      bufs.hist = (unsigned *)tab_scr.ptr;
      bufs.counter = (int *)(bufs.hist + s.n_super + 32);
      const int e = launch_tab_seg(a, s, bufs, n_cu, st);
      if (e) return hip_fail((hipError_t)e, "tab_seg_kernel launch");
      he = hipEventRecord(tab_done, st);
      if (he != hipSuccess) return hip_fail(he, "hipEventRecord");
      return FRG_OK;
    }
  }
  int e = launch_tab(a, reg, W, lds_rows, sblocks, st);
  if (e) return hip_fail((hipError_t)e, "tab_kernel launch");
  return FRG_OK;
}

// ----------------------------------------------------------------- LPA --
int Ctx::lpa_job_table(int n, const frg_lpa *lpa, const double *t, const double *const *U,
                       double *const *dUdt, double *const *jac, int *flags_dev, LpaJob *jobs,
                       int64_t *start) {
  int64_t total = 0;
  for (int f = 0; f < n; ++f) {
    const frg_lpa &l = lpa[f];
    const double *tab;
    double Cd;
    int rc = lpa_table(l.d, l.reg, l.n_radial, l.q_max_over_k, &tab, &Cd);
    if (rc) return rc;
    const double k = l.Lambda * std::exp(t[f]);
    LpaJob &j = jobs[f];
    j.U = U[f];
    j.dUdt = dUdt[f];
    j.jac = jac ? jac[f] : nullptr;
    j.tab = tab;
    j.flag = flags_dev ? flags_dev + f : d_flag;
    j.k2 = k * k;
    j.inv_k2 = 1.0 / j.k2;
    j.pre1 = Cd * std::pow(k, l.d);
    j.pre2 = Cd * std::pow(k, l.d - 2);
    j.dr = l.rho_max / (double)(l.n_grid - 1);
    j.Nm1 = (double)(l.N - 1);
    j.n = l.n_grid;
    j.n_r = l.n_radial;
    j.N = l.N;
    start[f] = total;
    total += l.n_grid;
  }
  start[n] = total;
  return FRG_OK;
}

int Ctx::lpa_jobs(int n, const frg_lpa *lpa, const double *t, const double *const *U,
                  double *const *dUdt, double *const *jac, int *flags_dev, hipStream_t st) {
  std::vector<LpaJob> jobs(n);
  std::vector<int64_t> start(n + 1);
  int rc = lpa_job_table(n, lpa, t, U, dUdt, jac, flags_dev, jobs.data(), start.data());
  if (rc) return rc;
  const int64_t total = start[n];
  const size_t jb = n * sizeof(LpaJob);
  std::vector<char> blob(jb + (n + 1) * sizeof(int64_t));
  std::memcpy(blob.data(), jobs.data(), jb);
  std::memcpy(blob.data() + jb, start.data(), (n + 1) * sizeof(int64_t));
  void *dev;
  int slot;
  rc = ring.upload(blob.data(), blob.size(), st, &dev, &slot);
  if (rc) return rc;
  int e = launch_lpa((const LpaJob *)dev, (const int64_t *)((char *)dev + jb), n, total, st);
  rc = ring.release(slot, st);
  if (e) return hip_fail((hipError_t)e, "lpa_kernel launch");
  return rc;
}

int Ctx::use_stream_flag(hipStream_t st) {
  auto it = stream_flags.find(st);
  if (it == stream_flags.end()) {
    int *f = nullptr;
    if (hipMalloc(&f, sizeof(int)) != hipSuccess) return fail(FRG_E_NOMEM, "hipMalloc(domain word)");
    if (hipMemset(f, 0, sizeof(int)) != hipSuccess) {
      hipFree(f);
      return fail(FRG_E_DEVICE, "hipMemset(domain word)");
    }
    it = stream_flags.emplace(st, f).first;
  }
  d_flag = it->second;
  return FRG_OK;
}

Context::~Context() {
  if (server) stop_server();
  if (stream) hipStreamSynchronize(stream);
  graphs.clear();
  ring.destroy();
  if (tab_done) {
    hipEventSynchronize(tab_done);
    hipEventDestroy(tab_done);
  }
  if (na_done) {
    hipEventSynchronize(na_done);
    hipEventDestroy(na_done);
  }
  if (na_stage) hipHostFree(na_stage);
  for (auto &kv : stream_flags) hipFree(kv.second);
  stream_flags.clear();
  if (stream) hipStreamDestroy(stream);
  if (cap_stream) hipStreamDestroy(cap_stream);
}

}  // namespace frg

using namespace frg;

// =================================================================== ABI ==
extern "C" {

const char *frg_last_error(void) { return g_err.c_str(); }

const char *frg_version(void) { return "frg-mi355x 0.1 (gfx950)"; }

int frg_create(frg_ctx **out, int hip_device, uint64_t hbm_budget_bytes) {
  if (!out) return fail(FRG_E_INVAL, "out is NULL");
  *out = nullptr;
  int ndev = 0;
  hipError_t e = hipGetDeviceCount(&ndev);
  if (e != hipSuccess || ndev == 0) return fail(FRG_E_DEVICE, "no HIP device available");
  if (hip_device < 0 || hip_device >= ndev) return fail(FRG_E_INVAL, "device %d out of range", hip_device);
  e = hipSetDevice(hip_device);
  if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
  auto c = std::make_unique<frg_ctx>();
  c->device = hip_device;
  hipDeviceProp_t prop;
  e = hipGetDeviceProperties(&prop, hip_device);
  if (e != hipSuccess) return hip_fail(e, "hipGetDeviceProperties");
  c->n_cu = prop.multiProcessorCount;
  c->arch = prop.gcnArchName;
  if (hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking) != hipSuccess ||
      hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking) != hipSuccess)
    return fail(FRG_E_DEVICE, "hipStreamCreate");
  int rc = c->use_stream_flag(c->stream);
  if (rc) return rc;
  rc = noalloc_init(hip_device, c.get());
  if (rc) return rc;
  rc = c->ring.init(1 << 20, 8);
  if (rc) return rc;
  size_t free_b = 0, total_b = 0;
  hipMemGetInfo(&free_b, &total_b);
  c->hbm_budget = hbm_budget_bytes ? hbm_budget_bytes : free_b / 2;
  c->hbm.budget = c->hbm_budget;
  c->tune.load_env();
  *out = c.release();
  clear_error();
  return FRG_OK;
}

void frg_destroy(frg_ctx *ctx) { delete ctx; }

int frg_integrate(frg_ctx *ctx, const frg_set *sets, int32_t n_sets, int32_t mem, int32_t flags,
                  void *hip_stream) {
  frg::TraceRange trace_("frg_integrate");
  if (!ctx) return fail(FRG_E_INVAL, "ctx is NULL");
  if (n_sets < 0 || (n_sets > 0 && !sets)) return fail(FRG_E_INVAL, "bad set array");
  if (mem != FRG_MEM_HOST && mem != FRG_MEM_DEVICE) return fail(FRG_E_INVAL, "mem must be FRG_MEM_HOST or FRG_MEM_DEVICE");
  if (flags & ~(FRG_PERSISTENT | FRG_GRAPH)) return fail(FRG_E_INVAL, "unknown flags 0x%x", flags);
  if ((flags & FRG_GRAPH) && !(flags & FRG_PERSISTENT)) return fail(FRG_E_INVAL, "FRG_GRAPH needs FRG_PERSISTENT");
  for (int i = 0; i < n_sets; ++i) {
    const frg_set &s = sets[i];
    int rc = check_quad(s.quad);
    if (rc) return rc;
    if (s.n_ext < 0) return fail(FRG_E_INVAL, "set %d: n_ext < 0", i);
    if (s.n_ext > 0 && (!s.p || !s.m2 || !s.out)) return fail(FRG_E_INVAL, "set %d: NULL array", i);
    if (s.n_ext > ((int64_t)1 << 40)) return fail(FRG_E_INVAL, "set %d: n_ext too large", i);
    if (mem == FRG_MEM_HOST)
      for (int64_t e = 0; e < s.n_ext; ++e)
        if (!(s.p[e] >= 0.0) || !std::isfinite(s.p[e]) || std::isnan(s.m2[e]))
          return fail(FRG_E_INVAL, "set %d point %lld: p must be finite and >= 0, m2 not NaN", i,
                      (long long)e);
  }
  std::lock_guard<std::mutex> lk(ctx->mu);
  hipSetDevice(ctx->device);
  clear_error();
  if (int rcf = ctx->use_stream_flag(mem == FRG_MEM_HOST ? ctx->stream : (hipStream_t)hip_stream))
    return rcf;
  if (mem == FRG_MEM_HOST) return ctx->integrate_host(sets, n_sets, flags);
  return ctx->integrate_device(sets, n_sets, flags, (hipStream_t)hip_stream);
}

int frg_integrate_grid(frg_ctx *ctx, const frg_quad *quad, int64_t n_p, const double *p,
                       int64_t n_m, const double *m2, double *out, double *err_est,
                       uint8_t *used_fp64, int32_t mem, void *hip_stream) {
  frg::TraceRange trace_("frg_integrate_grid");
  if (!ctx || !quad) return fail(FRG_E_INVAL, "NULL argument");
  int rc = check_quad(*quad);
  if (rc) return rc;
  if (n_p < 0 || n_m < 0) return fail(FRG_E_INVAL, "negative size");
  if (n_p * n_m > 0 && (!p || !m2 || !out)) return fail(FRG_E_INVAL, "NULL array");
  if (n_p > ((int64_t)1 << 30) || n_m > ((int64_t)1 << 30)) return fail(FRG_E_INVAL, "grid too large");
  if (mem != FRG_MEM_HOST && mem != FRG_MEM_DEVICE) return fail(FRG_E_INVAL, "bad mem");
  if (n_p == 0 || n_m == 0) return FRG_OK;
  std::lock_guard<std::mutex> lk(ctx->mu);
  hipSetDevice(ctx->device);
  clear_error();
  if (int rcf = ctx->use_stream_flag(mem == FRG_MEM_HOST ? ctx->stream : (hipStream_t)hip_stream))
    return rcf;
  if (mem == FRG_MEM_DEVICE)
    return ctx->grid_device(*quad, n_p, p, n_m, m2, out, err_est, used_fp64, (hipStream_t)hip_stream);
  for (int64_t a = 0; a < n_p; ++a)
    if (!(p[a] >= 0.0) || !std::isfinite(p[a])) return fail(FRG_E_INVAL, "p[%lld] must be finite and >= 0", (long long)a);
  const size_t nout = (size_t)(n_p * n_m);
  rc = ctx->stage_in.reserve((n_p + n_m) * sizeof(double) + 64);
  if (!rc) rc = ctx->stage_out.reserve(nout * (2 * sizeof(double) + 1) + 64);
  if (rc) return rc;
  double *dp = (double *)ctx->stage_in.ptr, *dm = dp + n_p;
  double *dout = (double *)ctx->stage_out.ptr, *derr = dout + nout;
  uint8_t *dused = (uint8_t *)(derr + nout);
  hipStream_t st = ctx->stream;
  hipMemcpyAsync(dp, p, n_p * sizeof(double), hipMemcpyHostToDevice, st);
  hipMemcpyAsync(dm, m2, n_m * sizeof(double), hipMemcpyHostToDevice, st);
  hipMemsetAsync(ctx->d_flag, 0, sizeof(int), st);
  rc = ctx->grid_device(*quad, n_p, dp, n_m, dm, dout, err_est ? derr : nullptr,
                        used_fp64 ? dused : nullptr, st);
  if (rc) {
    hipStreamSynchronize(st);
    return rc;
  }
  hipMemcpyAsync(out, dout, nout * sizeof(double), hipMemcpyDeviceToHost, st);
  if (err_est) hipMemcpyAsync(err_est, derr, nout * sizeof(double), hipMemcpyDeviceToHost, st);
  if (used_fp64) hipMemcpyAsync(used_fp64, dused, nout, hipMemcpyDeviceToHost, st);
  int flag = 0;
  hipMemcpyAsync(&flag, ctx->d_flag, sizeof(int), hipMemcpyDeviceToHost, st);
  hipError_t e = hipStreamSynchronize(st);
  if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
  if (flag) return fail(FRG_E_DOMAIN, "some masses have m^2 + k^2 <= 0; their results are NaN");
  return FRG_OK;
}

int frg_integrate_tab(frg_ctx *ctx, const frg_quad *quad, const frg_gtab *tab, int64_t n_p,
                      const double *p, double *out, int32_t mem, void *hip_stream) {
  frg::TraceRange trace_("frg_integrate_tab");
  if (!ctx || !quad || !tab) return fail(FRG_E_INVAL, "NULL argument");
  int rc = check_quad(*quad);
  if (rc) return rc;
  if (quad->prec != FRG_PREC_FP64) return fail(FRG_E_INVAL, "the tabulated variant is FP64 only");
  if (n_p < 0 || tab->n_rows < 0) return fail(FRG_E_INVAL, "negative size");
  if (tab->n_s < 2 || tab->n_s > ((int64_t)1 << 30)) return fail(FRG_E_INVAL, "tab.n_s outside [2, 2^30]");
  if (!(tab->s_max > 0.0) || !std::isfinite(tab->s_max)) return fail(FRG_E_INVAL, "tab.s_max must be finite and > 0");
  if (n_p > ((int64_t)1 << 30) || tab->n_rows > ((int64_t)1 << 24)) return fail(FRG_E_INVAL, "problem too large");
  if (mem != FRG_MEM_HOST && mem != FRG_MEM_DEVICE) return fail(FRG_E_INVAL, "bad mem");
  if (n_p == 0 || tab->n_rows == 0) return FRG_OK;
  if (!p || !out || !tab->g) return fail(FRG_E_INVAL, "NULL array");
  std::lock_guard<std::mutex> lk(ctx->mu);
  hipSetDevice(ctx->device);
  clear_error();
  if (int rcf = ctx->use_stream_flag(mem == FRG_MEM_HOST ? ctx->stream : (hipStream_t)hip_stream))
    return rcf;
  if (mem == FRG_MEM_DEVICE) return ctx->tab_device(*quad, *tab, n_p, p, out, (hipStream_t)hip_stream);
  const size_t gbytes = (size_t)(tab->n_rows * tab->n_s) * sizeof(double);
  const size_t nout = (size_t)(n_p * tab->n_rows);
  rc = ctx->stage_in.reserve(n_p * sizeof(double) + gbytes + 64);
  if (!rc) rc = ctx->stage_out.reserve(nout * sizeof(double) + 64);
  if (rc) return rc;
  double *dp = (double *)ctx->stage_in.ptr, *dg = dp + n_p;
  double *dout = (double *)ctx->stage_out.ptr;
  hipStream_t st = ctx->stream;
  hipMemcpyAsync(dp, p, n_p * sizeof(double), hipMemcpyHostToDevice, st);
  hipMemcpyAsync(dg, tab->g, gbytes, hipMemcpyHostToDevice, st);
  hipMemsetAsync(ctx->d_flag, 0, sizeof(int), st);
  frg_gtab dt = *tab;
  dt.g = dg;
  rc = ctx->tab_device(*quad, dt, n_p, dp, dout, st);
  if (rc) {
    hipStreamSynchronize(st);
    return rc;
  }
  hipMemcpyAsync(out, dout, nout * sizeof(double), hipMemcpyDeviceToHost, st);
  int flag = 0;
  hipMemcpyAsync(&flag, ctx->d_flag, sizeof(int), hipMemcpyDeviceToHost, st);
  hipError_t e = hipStreamSynchronize(st);
  if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
  if (flag) return fail(FRG_E_DOMAIN, "some momenta are negative; their results are NaN");
  return FRG_OK;
}

int frg_flow_rhs(frg_ctx *ctx, const frg_lpa *lpa, double t, const double *U, double *dUdt,
                 double *jac_bands, int32_t mem, void *hip_stream) {
  frg::TraceRange trace_("frg_flow_rhs");
  if (!ctx || !lpa || !U || !dUdt) return fail(FRG_E_INVAL, "NULL argument");
  int rc = check_lpa(*lpa);
  if (rc) return rc;
  if (!std::isfinite(t)) return fail(FRG_E_INVAL, "t must be finite");
  if (mem != FRG_MEM_HOST && mem != FRG_MEM_DEVICE) return fail(FRG_E_INVAL, "bad mem");
  std::lock_guard<std::mutex> lk(ctx->mu);
  hipSetDevice(ctx->device);
  clear_error();
  if (int rcf = ctx->use_stream_flag(mem == FRG_MEM_HOST ? ctx->stream : (hipStream_t)hip_stream))
    return rcf;
  if (mem == FRG_MEM_DEVICE) {
    const double *Up[1] = {U};
    double *Dp[1] = {dUdt};
    double *Jp[1] = {jac_bands};
    return ctx->lpa_jobs(1, lpa, &t, Up, Dp, Jp, nullptr, (hipStream_t)hip_stream);
  }
  const int64_t n = lpa->n_grid;
  rc = ctx->stage_in.reserve(n * sizeof(double));
  if (!rc) rc = ctx->stage_out.reserve(8 * n * sizeof(double));
  if (rc) return rc;
  hipStream_t st = ctx->stream;
  double *dU = (double *)ctx->stage_in.ptr;
  double *dD = (double *)ctx->stage_out.ptr;
  double *dJ = dD + n;
  hipMemcpyAsync(dU, U, n * sizeof(double), hipMemcpyHostToDevice, st);
  hipMemsetAsync(ctx->d_flag, 0, sizeof(int), st);
  const double *Up[1] = {dU};
  double *Dp[1] = {dD};
  double *Jp[1] = {jac_bands ? dJ : nullptr};
  rc = ctx->lpa_jobs(1, lpa, &t, Up, Dp, Jp, nullptr, st);
  if (rc) {
    hipStreamSynchronize(st);
    return rc;
  }
  hipMemcpyAsync(dUdt, dD, n * sizeof(double), hipMemcpyDeviceToHost, st);
  if (jac_bands) hipMemcpyAsync(jac_bands, dJ, 7 * n * sizeof(double), hipMemcpyDeviceToHost, st);
  int flag = 0;
  hipMemcpyAsync(&flag, ctx->d_flag, sizeof(int), hipMemcpyDeviceToHost, st);
  hipError_t e = hipStreamSynchronize(st);
  if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
  if (flag) return fail(FRG_E_DOMAIN, "a mass reached m^2 + k^2 <= 0");
  return FRG_OK;
}

int frg_flow_rhs_batch(frg_ctx *ctx, int32_t n_flows, const frg_lpa *lpa, const double *t,
                       const double *const *U, double *const *dUdt, double *const *jac_bands,
                       void *hip_stream) {
  frg::TraceRange trace_("frg_flow_rhs_batch");
  if (!ctx || n_flows < 0) return fail(FRG_E_INVAL, "bad arguments");
  if (n_flows == 0) return FRG_OK;
  if (!lpa || !t || !U || !dUdt) return fail(FRG_E_INVAL, "NULL argument");
  for (int f = 0; f < n_flows; ++f) {
    int rc = check_lpa(lpa[f]);
    if (rc) return rc;
    if (!U[f] || !dUdt[f]) return fail(FRG_E_INVAL, "flow %d: NULL buffer", f);
  }
  std::lock_guard<std::mutex> lk(ctx->mu);
  hipSetDevice(ctx->device);
  clear_error();
  if (int rcf = ctx->use_stream_flag((hipStream_t)hip_stream)) return rcf;
  return ctx->lpa_jobs(n_flows, lpa, t, U, dUdt, jac_bands, nullptr, (hipStream_t)hip_stream);
}

int frg_stream_status(frg_ctx *ctx, void *hip_stream) {
  if (!ctx) return fail(FRG_E_INVAL, "ctx is NULL");
  std::lock_guard<std::mutex> lk(ctx->mu);
  hipSetDevice(ctx->device);
  clear_error();
  hipStream_t st = (hipStream_t)hip_stream;
  if (int rc = ctx->use_stream_flag(st)) return rc;
  int flag = 0;
  hipError_t e = hipMemcpyAsync(&flag, ctx->d_flag, sizeof(int), hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipMemsetAsync(ctx->d_flag, 0, sizeof(int), st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) return hip_fail(e, "frg_stream_status");
  if (flag)
    return fail(FRG_E_DOMAIN, "a call on this stream met points with m^2 + k^2 <= 0 or p < 0; "
                              "their results are NaN");
  return FRG_OK;
}

int frg_gauss_legendre(int32_t n, double *x, double *w) {
  int rc = gauss_legendre_gw(n, x, w);
  if (rc) return fail(rc, "n must be in [1, 4096] and x, w non-NULL");
  return FRG_OK;
}

int frg_expneg(int64_t n, const double *y, double *out) {
  if (n < 0 || (n > 0 && (!y || !out))) return fail(FRG_E_INVAL, "bad arguments");
  for (int64_t i = 0; i < n; ++i) out[i] = exp_neg(y[i], kExp2Tab64);
  return FRG_OK;
}

int frg_expneg_fp32c(frg_ctx *ctx, int64_t n, const double *y, double *out, void *hip_stream) {
  if (!ctx) return fail(FRG_E_INVAL, "ctx is NULL");
  if (n < 0 || (n > 0 && (!y || !out))) return fail(FRG_E_INVAL, "bad arguments");
  std::lock_guard<std::mutex> lk(ctx->mu);
  hipSetDevice(ctx->device);
  clear_error();
  const int e = launch_expneg_fp32c(y, out, n, hip_stream);
  if (e) return hip_fail((hipError_t)e, "expneg_fp32c_kernel launch");
  return FRG_OK;
}

int64_t frg_flow_footprint(const frg_lpa *lpa) {
  if (!lpa || lpa->n_grid < 1) return -1;
  // the flow's share of the server's staging buffer: U, dUdt and 7 Jacobian
  // bands, plus a 4 KiB descriptor share
  return (int64_t)(9 * lpa->n_grid * sizeof(double)) + 4096;
}

}  // extern "C"
