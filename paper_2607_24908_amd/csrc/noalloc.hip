// frg_integrate_noalloc: the persistent point-list launch of frg_integrate
// (device memory, FRG_PERSISTENT) for callers that cannot allocate device
// memory.  Everything the launch needs beyond the caller's inputs and
// outputs -- work-list counters, a discarded domain word, set descriptors,
// the longest-first work list and the quadrature tables -- lives in
// `scratch`, a fixed array of kScratchBytes in device memory that every GPU
// the library runs on holds until the process ends.  The host writes the
// zeroed counters and the descriptors into the context's pinned staging
// buffer (allocated by frg_create) and copies it into the array with one
// hipMemcpyAsync on the caller's stream; the kernel is the one of
// frg_integrate, so the results are the same bits.
//
// Layout of one call in `scratch` (each part 256-byte aligned):
//   counters (kCounterInts ints, zero) | domain word (int) | SetDev[n_sets]
//   | Tile[n_tiles] | one packed quadrature table per distinct key.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <map>
#include <mutex>
#include <tuple>
#include <vector>

#include "frg_ctx.h"

namespace frg {

constexpr size_t kScratchBytes = (size_t)4 << 20;

static __device__ __align__(256) char scratch[kScratchBytes];

namespace {

constexpr int kMaxDevices = 64;
// Device address of `scratch` on each device (from hipGetSymbolAddress; the
// symbol's name is a host-side stand-in, never a device address).
char *g_scratch_dev[kMaxDevices];
std::once_flag g_scratch_once[kMaxDevices];
hipError_t g_scratch_err[kMaxDevices];

size_t up256(size_t x) { return (x + 255) & ~(size_t)255; }

uint64_t dbits(double x) {
  uint64_t u;
  std::memcpy(&u, &x, 8);
  return u;
}

}  // namespace

int noalloc_init(int device, Context *ctx) {
  if (device < 0 || device >= kMaxDevices)
    return fail(FRG_E_INVAL, "device %d beyond the %d devices of the scratch table", device,
                kMaxDevices);
  // once per device, with that device current (frg_create has set it)
  std::call_once(g_scratch_once[device], [device] {
    void *ptr = nullptr;
    g_scratch_err[device] = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    g_scratch_dev[device] = g_scratch_err[device] == hipSuccess ? (char *)ptr : nullptr;
  });
  if (g_scratch_err[device] != hipSuccess)
    return hip_fail(g_scratch_err[device], "hipGetSymbolAddress(scratch)");
  if (hipHostMalloc((void **)&ctx->na_stage, kScratchBytes, hipHostMallocDefault) != hipSuccess) {
    ctx->na_stage = nullptr;
    return fail(FRG_E_NOMEM, "hipHostMalloc(%zu) for the allocation-free staging", kScratchBytes);
  }
  hipError_t e = hipEventCreateWithFlags(&ctx->na_done, hipEventDisableTiming);
  if (e != hipSuccess) return hip_fail(e, "hipEventCreate(allocation-free call)");
  return FRG_OK;
}

const QuadTable &Context::host_quad_table(const frg_quad &q) {
  const auto key = std::make_tuple(q.d, q.reg, dbits(q.k), dbits(q.q_max), q.n_radial, q.n_angular);
  auto it = qtabs.find(key);
  if (it != qtabs.end()) return it->second.host;
  auto h = htabs.find(key);
  if (h == htabs.end()) h = htabs.emplace(key, build_quad_table(q)).first;
  return h->second;
}

}  // namespace frg

using namespace frg;

extern "C" int frg_integrate_noalloc(frg_ctx *ctx, const frg_set *sets, int32_t n_sets,
                                     int32_t *domain_flag, void *hip_stream) {
  if (!ctx) return fail(FRG_E_INVAL, "ctx is NULL");
  if (n_sets < 0 || (n_sets > 0 && !sets)) return fail(FRG_E_INVAL, "bad set array");
  for (int i = 0; i < n_sets; ++i) {
    const frg_set &s = sets[i];
    if (int rc = check_quad(s.quad)) return rc;
    if (s.n_ext < 0) return fail(FRG_E_INVAL, "set %d: n_ext < 0", i);
    if (s.n_ext > 0 && (!s.p || !s.m2 || !s.out)) return fail(FRG_E_INVAL, "set %d: NULL array", i);
    if (s.n_ext > ((int64_t)1 << 40)) return fail(FRG_E_INVAL, "set %d: n_ext too large", i);
  }
  std::lock_guard<std::mutex> lk(ctx->mu);
  if (ctx->device < 0 || ctx->device >= kMaxDevices || !g_scratch_dev[ctx->device] ||
      !ctx->na_stage)
    return fail(FRG_E_DEVICE, "the scratch area of device %d is not set up", ctx->device);
  hipSetDevice(ctx->device);
  clear_error();
  hipStream_t st = (hipStream_t)hip_stream;
  char *dev = g_scratch_dev[ctx->device];
  // distinct quadrature keys and the offsets of their tables
  using Key = std::tuple<int, int, uint64_t, uint64_t, int, int>;
  std::map<Key, size_t> tab_off;
  std::vector<const QuadTable *> hosts(n_sets);
  const size_t o_flag = up256(kCounterInts * sizeof(int));
  const size_t o_sets = o_flag + 256;
  const size_t o_tiles = up256(o_sets + (size_t)n_sets * sizeof(SetDev));
  std::vector<SetDev> sd(n_sets);
  for (int i = 0; i < n_sets; ++i) {
    hosts[i] = &ctx->host_quad_table(sets[i].quad);
    ctx->fill_setdev(sets[i], *hosts[i], nullptr, &sd[i]);
  }
  const PersistCfg pc = ctx->persist_cfg_cached(sd, sd.empty() ? 0 : sd[0].prec);
  std::vector<Tile> tiles;
  build_tiles(sd, pc.tile, &tiles);
  size_t off = up256(o_tiles + tiles.size() * sizeof(Tile));
  for (int i = 0; i < n_sets; ++i) {
    const frg_quad &q = sets[i].quad;
    const Key key{q.d, q.reg, dbits(q.k), dbits(q.q_max), q.n_radial, q.n_angular};
    auto it = tab_off.find(key);
    if (it == tab_off.end()) {
      it = tab_off.emplace(key, off).first;
      off = up256(off + hosts[i]->data.size() * sizeof(double));
    }
    sd[i].tab = (const double *)(dev + it->second);
  }
  if (off > kScratchBytes)
    return fail(FRG_E_INVAL,
                "the call needs %zu bytes of scratch (descriptors of %d sets, %zu tiles, %zu "
                "tables); the allocation-free area holds %zu",
                off, n_sets, tiles.size(), tab_off.size(), kScratchBytes);
  if (tiles.empty()) return FRG_OK;
  const int lds = max_table_bytes(sd);
  if (lds > 60 * 1024) return fail(FRG_E_INVAL, "quadrature tables exceed 60 KiB of LDS");
  // the previous call's copy must have left the staging buffer
  if (ctx->na_pending) {
    hipError_t e = hipEventSynchronize(ctx->na_done);
    if (e != hipSuccess) return hip_fail(e, "hipEventSynchronize(allocation-free call)");
    ctx->na_pending = false;
  }
  char *h = ctx->na_stage;
  std::memset(h, 0, o_sets);  // counters and domain word start at zero
  std::memcpy(h + o_sets, sd.data(), sd.size() * sizeof(SetDev));
  std::memcpy(h + o_tiles, tiles.data(), tiles.size() * sizeof(Tile));
  for (int i = 0; i < n_sets; ++i) {
    const size_t o = (const char *)sd[i].tab - dev;
    std::memcpy(h + o, hosts[i]->data.data(), hosts[i]->data.size() * sizeof(double));
  }
  // one copy, then the kernel of frg_integrate (FRG_PERSISTENT); the next
  // call waits for this one's event before it reuses the staging buffer
  hipError_t e = hipMemcpyAsync(dev, h, off, hipMemcpyHostToDevice, st);
  if (e != hipSuccess) return hip_fail(e, "hipMemcpyAsync(scratch)");
  const int n_blocks = std::max(1, std::min<int>((int)tiles.size(), ctx->n_cu * pc.wpc));
  int *flag = domain_flag ? domain_flag : (int *)(dev + o_flag);
  const int el = launch_points_persistent((const SetDev *)(dev + o_sets),
                                          (const Tile *)(dev + o_tiles), (int)tiles.size(),
                                          (int *)dev, lds, n_blocks, any_fp32c(sd), flag, st);
  e = hipEventRecord(ctx->na_done, st);
  ctx->na_pending = e == hipSuccess;
  if (el) return hip_fail((hipError_t)el, "points_persistent_kernel launch");
  if (e != hipSuccess) return hip_fail(e, "hipEventRecord(allocation-free call)");
  return FRG_OK;
}
