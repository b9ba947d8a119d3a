// Launch-shape autotuner.
//
// A key is (kernel family, regulator, n_radial, n_angular, precision, size
// class).  In tuning mode the first call with a new key times every
// candidate launch shape on that call's own inputs (HIP events on the
// caller's stream: one warm-up and two timed launches each) and keeps the
// fastest; later calls with the key reuse it.  Every kernel sums each result
// in an order fixed by (n_radial, n_angular), so the outputs of all
// candidates are bitwise identical and tuning never changes a result.
// Choices can be persisted in a small text file, one per line:
//   grid    <arch> <reg> <n_r> <n_a> <prec> <size> <M> <W> <MB>
//   plain   <arch> <reg> <n_r> <n_a> <prec> <size> <tile>
//   persist <arch> <prec> <size> <tile> <wpc>
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <functional>
#include <limits>
#include <sstream>

#include "frg_ctx.h"

namespace frg {

namespace {

int size_class(double work) { return work <= 1.0 ? 0 : (int)std::floor(std::log2(work) / 2.0); }

// Milliseconds per launch (two timed launches after one warm-up), or +inf
// if a launch fails.
double time_ms(hipStream_t st, const std::function<int()> &launch) {
  if (launch() != FRG_OK) return std::numeric_limits<double>::infinity();
  hipEvent_t a, b;
  hipEventCreate(&a);
  hipEventCreate(&b);
  hipEventRecord(a, st);
  int rc = launch();
  rc |= launch();
  hipEventRecord(b, st);
  hipEventSynchronize(b);
  float ms = 0.0f;
  hipEventElapsedTime(&ms, a, b);
  hipEventDestroy(a);
  hipEventDestroy(b);
  return rc == FRG_OK ? ms / 2.0 : std::numeric_limits<double>::infinity();
}

}  // namespace

void Tune::load_env() {
  if (const char *m = std::getenv("FRG_AUTOTUNE")) mode = std::atoi(m) ? 1 : 0;
  if (const char *p = std::getenv("FRG_AUTOTUNE_CACHE")) cache_path = p;
}

int Tune::load_file(const std::string &arch) {
  if (cache_path.empty()) return FRG_OK;
  std::ifstream f(cache_path);
  if (!f) return FRG_OK;  // no cache yet
  std::string line;
  while (std::getline(f, line)) {
    std::istringstream is(line);
    std::string kind, a;
    is >> kind >> a;
    if (a != arch) continue;
    if (kind == "grid") {
      int reg, nr, na, prec, sz;
      GridCfg c;
      if (is >> reg >> nr >> na >> prec >> sz >> c.M >> c.W >> c.MB)
        grid_best[ShapeKey{reg, nr, na, prec * 64 + sz}] = c;
    } else if (kind == "plain") {
      int reg, nr, na, prec, sz, tile;
      if (is >> reg >> nr >> na >> prec >> sz >> tile)
        plain_best[ShapeKey{reg, nr, na, prec * 64 + sz}] = tile;
    } else if (kind == "persist") {
      int prec, sz;
      PersistCfg c;
      if (is >> prec >> sz >> c.tile >> c.wpc) persist_best[prec * 64 + sz] = c;
    }
  }
  return FRG_OK;
}

int Tune::save_file(const std::string &arch) const {
  if (cache_path.empty()) return FRG_OK;
  std::ofstream f(cache_path);
  if (!f) return fail(FRG_E_INVAL, "cannot write autotune cache %s", cache_path.c_str());
  for (auto &kv : grid_best) {
    auto [reg, nr, na, ps] = kv.first;
    f << "grid " << arch << ' ' << reg << ' ' << nr << ' ' << na << ' ' << ps / 64 << ' ' << ps % 64
      << ' ' << kv.second.M << ' ' << kv.second.W << ' ' << kv.second.MB << '\n';
  }
  for (auto &kv : plain_best) {
    auto [reg, nr, na, ps] = kv.first;
    f << "plain " << arch << ' ' << reg << ' ' << nr << ' ' << na << ' ' << ps / 64 << ' '
      << ps % 64 << ' ' << kv.second << '\n';
  }
  for (auto &kv : persist_best)
    f << "persist " << arch << ' ' << kv.first / 64 << ' ' << kv.first % 64 << ' '
      << kv.second.tile << ' ' << kv.second.wpc << '\n';
  return FRG_OK;
}

GridCfg Context::grid_cfg(const frg_quad &q, const GridArgs &g, hipStream_t st) {
  const int sz = size_class((double)g.n_p * g.n_m * q.n_radial * q.n_angular);
  const ShapeKey key{q.reg, q.n_radial, q.n_angular, q.prec * 64 + sz};
  auto it = tune.grid_best.find(key);
  if (it != tune.grid_best.end()) return it->second;
  if (tune.mode != 1) return tune.grid;
  GridCfg best = tune.grid;
  double best_ms = std::numeric_limits<double>::infinity();
  for (int M : {4, 8, 16})
    for (int W : {2, 4, 8})
      for (int MB : {1, 2, 4, 8, 16}) {
        const GridCfg c{M, W, MB};
        const double ms = time_ms(st, [&] { return grid_launch(g, q.reg, c, st); });
        if (ms < best_ms) {
          best_ms = ms;
          best = c;
        }
      }
  tune.grid_best[key] = best;
  tune.save_file(arch);
  return best;
}

int Context::plain_tile_for(const SetDev &s, hipStream_t st) {
  const int sz = size_class((double)s.n_ext * s.n_r * s.n_a);
  const ShapeKey key{s.reg, s.n_r, s.n_a, s.prec * 64 + sz};
  auto it = tune.plain_best.find(key);
  if (it != tune.plain_best.end()) return it->second;
  if (tune.mode != 1) return tune.plain_tile;
  int best = tune.plain_tile;
  double best_ms = std::numeric_limits<double>::infinity();
  for (int tile : {1, 2, 4, 8, 16, 32, 64}) {
    const double ms = time_ms(st, [&] {
      return launch_points_plain(s, tile, d_flag, st) ? FRG_E_DEVICE : FRG_OK;
    });
    if (ms < best_ms) {
      best_ms = ms;
      best = tile;
    }
  }
  tune.plain_best[key] = best;
  tune.save_file(arch);
  return best;
}

PersistCfg Context::persist_cfg_cached(const std::vector<SetDev> &sd, int prec) const {
  double work = 0.0;
  for (auto &s : sd) work += (double)s.n_ext * s.n_r * s.n_a;
  auto it = tune.persist_best.find(prec * 64 + size_class(work));
  return it != tune.persist_best.end() ? it->second : tune.persist;
}

PersistCfg Context::persist_cfg(const std::vector<SetDev> &sd, int prec, hipStream_t st) {
  double work = 0.0;
  for (auto &s : sd) work += (double)s.n_ext * s.n_r * s.n_a;
  const int key = prec * 64 + size_class(work);
  auto it = tune.persist_best.find(key);
  if (it != tune.persist_best.end()) return it->second;
  if (tune.mode != 1) return tune.persist;
  PersistCfg best = tune.persist;
  double best_ms = std::numeric_limits<double>::infinity();
  for (int tile : {1, 2, 4, 8, 16, 32})
    for (int wpc : {4, 8, 16, 32}) {
      const PersistCfg c{tile, wpc};
      const double ms = time_ms(st, [&] { return persistent_eager(sd, c, st); });
      if (ms < best_ms) {
        best_ms = ms;
        best = c;
      }
    }
  tune.persist_best[key] = best;
  ++tune_gen;
  tune.save_file(arch);
  return best;
}

}  // namespace frg

using namespace frg;

extern "C" {

int frg_autotune(frg_ctx *ctx, int32_t mode, const char *cache_path) {
  frg::TraceRange trace_("frg_autotune");
  if (!ctx) return fail(FRG_E_INVAL, "ctx is NULL");
  if (mode != 0 && mode != 1) return fail(FRG_E_INVAL, "mode must be 0 or 1");
  std::lock_guard<std::mutex> lk(ctx->mu);
  ctx->tune.mode = mode;
  ++ctx->tune_gen;
  if (cache_path) {
    ctx->tune.cache_path = cache_path;
    int rc = ctx->tune.load_file(ctx->arch);
    if (rc) return rc;
  }
  clear_error();
  return FRG_OK;
}

static int *knob(frg_ctx *ctx, const char *key) {
  Tune &t = ctx->tune;
  if (!std::strcmp(key, "grid_M")) return &t.grid.M;
  if (!std::strcmp(key, "grid_W")) return &t.grid.W;
  if (!std::strcmp(key, "grid_MB")) return &t.grid.MB;
  if (!std::strcmp(key, "grid_lds_rows")) return &t.grid_lds_rows;
  if (!std::strcmp(key, "grid_form")) return &t.grid_form;
  if (!std::strcmp(key, "grid_mfma")) return &t.grid_mfma;
  if (!std::strcmp(key, "fv_persistent")) return &t.fv_persistent;
  if (!std::strcmp(key, "pflow_fused")) return &t.pflow_fused;
  if (!std::strcmp(key, "vertex_W")) return &t.vertex_W;
  if (!std::strcmp(key, "server_zero_copy")) return &t.server_zero_copy;
  if (!std::strcmp(key, "tab_W")) return &t.tab_W;
  if (!std::strcmp(key, "tab_pw")) return &t.tab_pw;
  if (!std::strcmp(key, "tab_lds_nodes")) return &t.tab_lds_nodes;
  if (!std::strcmp(key, "tab_wpc")) return &t.tab_wpc;
  if (!std::strcmp(key, "tab_sW")) return &t.tab_sW;
  if (!std::strcmp(key, "tab_spw")) return &t.tab_spw;
  if (!std::strcmp(key, "plain_tile")) return &t.plain_tile;
  if (!std::strcmp(key, "persist_tile")) return &t.persist.tile;
  if (!std::strcmp(key, "persist_wpc")) return &t.persist.wpc;
  if (!std::strcmp(key, "fp32c_flag_ppb")) return &t.fp32c_flag_ppb;
  if (!std::strcmp(key, "tab_pairs")) return &t.tab_pairs;
  if (!std::strcmp(key, "tab_rb")) return &t.tab_rb;
  if (!std::strcmp(key, "tab_rW")) return &t.tab_rW;
  if (!std::strcmp(key, "tab_seg")) return &t.tab_seg;
  if (!std::strcmp(key, "fp32c_band_ppm")) return &t.fp32c_band_ppm;
  return nullptr;
}

static bool knob_ok(const char *key, int v) {
  if (!std::strcmp(key, "grid_M")) return v == 4 || v == 8 || v == 16;
  if (!std::strcmp(key, "grid_W")) return v >= 1 && v <= 8;
  if (!std::strcmp(key, "grid_MB")) return v >= 1 && v <= 64;
  if (!std::strcmp(key, "grid_lds_rows")) return v >= 8 && v <= 96;
  if (!std::strcmp(key, "grid_form")) return v >= 0 && v <= 3;
  if (!std::strcmp(key, "grid_mfma") || !std::strcmp(key, "fv_persistent") ||
      !std::strcmp(key, "pflow_fused") || !std::strcmp(key, "server_zero_copy"))
    return v == 0 || v == 1;
  if (!std::strcmp(key, "vertex_W")) return v >= 1 && v <= 12;
  if (!std::strcmp(key, "tab_W")) return v >= 1 && v <= 4;
  if (!std::strcmp(key, "tab_pw")) return v >= 1 && v <= 64;
  if (!std::strcmp(key, "tab_lds_nodes")) return v >= 2 && v <= (int)tab_lds_max_nodes;
  if (!std::strcmp(key, "tab_wpc")) return v >= 1 && v <= 16;
  if (!std::strcmp(key, "tab_sW")) return v >= 1 && v <= 4;
  if (!std::strcmp(key, "tab_spw")) return v >= 1 && v <= 64;
  if (!std::strcmp(key, "tab_pairs")) return v == 0 || v == 1;
  if (!std::strcmp(key, "tab_rb")) return v == 0 || v == 1 || v == 2 || v == 4;
  if (!std::strcmp(key, "tab_rW")) return v >= 1 && v <= 16;
  if (!std::strcmp(key, "tab_seg")) return v >= 0 && v <= 2;
  if (!std::strcmp(key, "plain_tile") || !std::strcmp(key, "persist_tile")) return v >= 1 && v <= 64;
  if (!std::strcmp(key, "persist_wpc")) return v >= 1 && v <= 64;
  if (!std::strcmp(key, "fp32c_flag_ppb")) return v >= 0;
  if (!std::strcmp(key, "fp32c_band_ppm")) return v >= 0;
  return false;
}

int frg_tune_set(frg_ctx *ctx, const char *key, int32_t value) {
  if (!ctx || !key) return fail(FRG_E_INVAL, "NULL argument");
  std::lock_guard<std::mutex> lk(ctx->mu);
  int *k = knob(ctx, key);
  if (!k) return fail(FRG_E_INVAL, "unknown knob '%s'", key);
  if (!knob_ok(key, value)) return fail(FRG_E_INVAL, "value %d out of range for '%s'", value, key);
  *k = value;
  ++ctx->tune_gen;
  // explicit settings take effect for keys that were already tuned, too
  ctx->tune.grid_best.clear();
  ctx->tune.plain_best.clear();
  ctx->tune.persist_best.clear();
  clear_error();
  return FRG_OK;
}

int frg_tune_get(frg_ctx *ctx, const char *key, int32_t *value) {
  if (!ctx || !key || !value) return fail(FRG_E_INVAL, "NULL argument");
  std::lock_guard<std::mutex> lk(ctx->mu);
  int *k = knob(ctx, key);
  if (!k) return fail(FRG_E_INVAL, "unknown knob '%s'", key);
  *value = *k;
  return FRG_OK;
}

}  // extern "C"
