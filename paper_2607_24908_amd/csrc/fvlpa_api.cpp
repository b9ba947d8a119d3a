// Finite-volume LPA behind frg_fvlpa_rhs / frg_fvlpa_solve: argument checks,
// per-call device scratch (stream-ordered), and the SSP-RK3 stage loop, every
// stage launched on the caller's stream.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>

#include "frg_ctx.h"

namespace frg {

constexpr int64_t kFvStepsPerLaunch = 2048;

static int check_fvlpa(const frg_fvlpa &f, int64_t n_flows) {
  if (f.d < 2 || f.d > 8) return fail(FRG_E_INVAL, "fvlpa.d=%d outside [2, 8]", f.d);
  if (f.N < 1 || f.N > 64) return fail(FRG_E_INVAL, "fvlpa.N=%d outside [1, 64]", f.N);
  if (f.reg != FRG_REG_EXP && f.reg != FRG_REG_LITIM) return fail(FRG_E_INVAL, "fvlpa.reg unknown");
  if (f.n_radial < 1 || f.n_radial > 1024) return fail(FRG_E_INVAL, "fvlpa.n_radial outside [1, 1024]");
  if (!(f.lambda > 0.0) || !std::isfinite(f.lambda)) return fail(FRG_E_INVAL, "fvlpa.lambda must be finite and > 0");
  if (!(f.q_max_over_k > 0.0) || !std::isfinite(f.q_max_over_k))
    return fail(FRG_E_INVAL, "fvlpa.q_max_over_k must be finite and > 0");
  if (f.n_cells < 2 || f.n_cells > ((int64_t)1 << 24)) return fail(FRG_E_INVAL, "fvlpa.n_cells outside [2, 2^24]");
  if (!(f.sigma_max > 0.0) || !std::isfinite(f.sigma_max))
    return fail(FRG_E_INVAL, "fvlpa.sigma_max must be finite and > 0");
  if (n_flows < 0 || n_flows > ((int64_t)1 << 24)) return fail(FRG_E_INVAL, "n_flows outside [0, 2^24]");
  if (n_flows > 65535) return fail(FRG_E_INVAL, "n_flows outside [0, 65535]");
  if (n_flows * (f.n_cells + 1) > ((int64_t)1 << 31)) return fail(FRG_E_INVAL, "n_flows * n_cells too large");
  return FRG_OK;
}

int Ctx::fvlpa_device(const frg_fvlpa &f, int64_t n, double t_end, int64_t n_steps, double *u,
                      double *t_reached, double *dudt, double *dt_est, double t_rhs, int *flag,
                      hipStream_t st) {
  const double *tab;
  double Cd;
  int rc = lpa_table(f.d, f.reg, f.n_radial, f.q_max_over_k, &tab, &Cd);
  if (rc) return rc;
  const bool solve = dudt == nullptr;
  const int64_t m = n * f.n_cells, nq = n * (f.n_cells + 1);
  // scratch: Q | lam | [ys] | [t_reached] | alive
  const size_t nd = 2 * nq + (solve ? m : 0) + (t_reached ? 0 : n);
  void *buf = nullptr;
  hipError_t e = hipMallocAsync(&buf, nd * sizeof(double) + (size_t)n * sizeof(int) + 64, st);
  if (e != hipSuccess) return fail(FRG_E_NOMEM, "fvlpa scratch: %s", hipGetErrorString(e));
  double *d = (double *)buf;
  FvArgs a{};
  a.tab = tab;
  a.Q = d;
  d += nq;
  a.lam = d;
  d += nq;
  if (solve) {
    a.ys = d;
    d += m;
  }
  if (t_reached) {
    a.t_reached = t_reached;
  } else {
    a.t_reached = d;
    d += n;
  }
  a.alive = (int *)d;
  a.y0 = u;
  a.dudt = dudt;
  a.dt = dt_est;
  a.flag = flag;
  a.Cd = Cd;
  a.ds = f.sigma_max / (double)f.n_cells;
  a.inv_ds = (double)f.n_cells / f.sigma_max;
  a.n_rows = n;
  a.n = f.n_cells;
  a.n_r = f.n_radial;
  a.N = f.N;
  a.d = f.d;
  a.lambda = f.lambda;
  auto rhs_at = [&](double t, int stage, int first) -> int {
    a.t = t;  // the kernels form k = lambda e^t and its powers
    a.stage = stage;
    a.first = first;
    int r = launch_fv_flux(a, st);
    if (r) return hip_fail((hipError_t)r, "fv_flux_kernel launch");
    r = launch_fv_stage(a, st);
    if (r) return hip_fail((hipError_t)r, "fv_stage_kernel launch");
    return FRG_OK;
  };
  rc = launch_fv_init(a, solve ? t_end : t_rhs, st);
  if (rc) rc = hip_fail((hipError_t)rc, "fv_init_kernel launch");
  if (!rc && !solve) {
    a.t_n = t_rhs;
    rc = rhs_at(t_rhs, 3, 1);
    if (!rc && dt_est) {
      const int r = launch_fv_dt(a, st);
      if (r) rc = hip_fail((hipError_t)r, "fv_dt_kernel launch");
    }
  }
  if (!rc && solve) {
    const double hh = t_end / (double)n_steps;
    a.h = hh;
    if (tune.fv_persistent && fv_solve_lds_bytes(a) <= kFvSolveLdsMax) {
      // one workgroup per flow runs the steps with its state in LDS, in
      // launches of at most kFvStepsPerLaunch steps; the whole chip's
      // threads per flow while there are at most as many flows as CUs
      const int threads = n <= n_cu ? 1024 : n <= 2 * n_cu ? 512 : 256;
      for (int64_t s0 = 0; s0 < n_steps && !rc; s0 += kFvStepsPerLaunch) {
        const int r = launch_fv_solve(a, s0, std::min(kFvStepsPerLaunch, n_steps - s0), threads, st);
        if (r) rc = hip_fail((hipError_t)r, "fv_solve_kernel launch");
      }
    } else {
      const double cs[3] = {0.0, 1.0, 0.5};
      for (int64_t step = 0; step < n_steps && !rc; ++step) {
        const double tn = (double)step * hh;
        a.t_n = tn;
        for (int s = 0; s < 3 && !rc; ++s) rc = rhs_at(tn + cs[s] * hh, s, s == 0);
      }
    }
  }
  (void)hipFreeAsync(buf, st);
  return rc;
}

}  // namespace frg

using namespace frg;

extern "C" {

int frg_fvlpa_rhs(frg_ctx *ctx, const frg_fvlpa *fv, int64_t n_flows, double t, const double *u,
                  double *dudt, double *dt_est, int32_t mem, void *hip_stream) {
  frg::TraceRange trace_("frg_fvlpa_rhs");
  if (!ctx || !fv) return fail(FRG_E_INVAL, "NULL argument");
  int rc = check_fvlpa(*fv, n_flows);
  if (rc) return rc;
  if (!std::isfinite(t)) return fail(FRG_E_INVAL, "t must be finite");
  if (mem != FRG_MEM_HOST && mem != FRG_MEM_DEVICE) return fail(FRG_E_INVAL, "bad mem");
  if (n_flows == 0) return FRG_OK;
  if (!u || !dudt) return fail(FRG_E_INVAL, "NULL array");
  std::lock_guard<std::mutex> lk(ctx->mu);
  hipSetDevice(ctx->device);
  clear_error();
  const int64_t m = n_flows * fv->n_cells;
  if (mem == FRG_MEM_DEVICE) {
    hipStream_t st = (hipStream_t)hip_stream;
    int *flag = nullptr;
    if (hipMallocAsync((void **)&flag, sizeof(int), st) != hipSuccess)
      return fail(FRG_E_NOMEM, "fvlpa flag");
    rc = ctx->fvlpa_device(*fv, n_flows, 0.0, 1, const_cast<double *>(u), nullptr, dudt, dt_est,
                           t, flag, st);
    (void)hipFreeAsync(flag, st);
    return rc;
  }
  hipStream_t st = ctx->stream;
  double *buf = nullptr;
  const size_t nb = (size_t)(2 * m + n_flows) * sizeof(double) + 64;
  if (hipMallocAsync((void **)&buf, nb, st) != hipSuccess) return fail(FRG_E_NOMEM, "fvlpa staging");
  double *du = buf, *dd = du + m, *dt = dd + m;
  int *flag = (int *)(dt + n_flows);
  hipMemcpyAsync(du, u, m * sizeof(double), hipMemcpyHostToDevice, st);
  rc = ctx->fvlpa_device(*fv, n_flows, 0.0, 1, du, nullptr, dd, dt_est ? dt : nullptr, t, flag, st);
  int hflag = 0;
  if (!rc) {
    hipMemcpyAsync(dudt, dd, m * sizeof(double), hipMemcpyDeviceToHost, st);
    if (dt_est) hipMemcpyAsync(dt_est, dt, n_flows * sizeof(double), hipMemcpyDeviceToHost, st);
    hipMemcpyAsync(&hflag, flag, sizeof(int), hipMemcpyDeviceToHost, st);
  }
  (void)hipFreeAsync(buf, st);
  hipError_t e = hipStreamSynchronize(st);
  if (rc) return rc;
  if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
  if (hflag) return fail(FRG_E_DOMAIN, "some flows are outside the domain; their rows are NaN");
  return FRG_OK;
}

int frg_fvlpa_solve(frg_ctx *ctx, const frg_fvlpa *fv, int64_t n_flows, double t_end,
                    int64_t n_steps, double *u, double *t_reached, int32_t mem, void *hip_stream) {
  frg::TraceRange trace_("frg_fvlpa_solve");
  if (!ctx || !fv) return fail(FRG_E_INVAL, "NULL argument");
  int rc = check_fvlpa(*fv, n_flows);
  if (rc) return rc;
  if (!std::isfinite(t_end) || t_end > 0.0) return fail(FRG_E_INVAL, "t_end must be finite and <= 0");
  if (n_steps < 1 || n_steps > ((int64_t)1 << 26)) return fail(FRG_E_INVAL, "n_steps outside [1, 2^26]");
  if (mem != FRG_MEM_HOST && mem != FRG_MEM_DEVICE) return fail(FRG_E_INVAL, "bad mem");
  if (n_flows == 0) return FRG_OK;
  if (!u || !t_reached) return fail(FRG_E_INVAL, "NULL array");
  std::lock_guard<std::mutex> lk(ctx->mu);
  hipSetDevice(ctx->device);
  clear_error();
  const int64_t m = n_flows * fv->n_cells;
  if (mem == FRG_MEM_DEVICE) {
    hipStream_t st = (hipStream_t)hip_stream;
    int *flag = nullptr;
    if (hipMallocAsync((void **)&flag, sizeof(int), st) != hipSuccess)
      return fail(FRG_E_NOMEM, "fvlpa flag");
    rc = ctx->fvlpa_device(*fv, n_flows, t_end, n_steps, u, t_reached, nullptr, nullptr, 0.0, flag,
                           st);
    (void)hipFreeAsync(flag, st);
    return rc;
  }
  hipStream_t st = ctx->stream;
  double *buf = nullptr;
  const size_t nb = (size_t)(m + n_flows) * sizeof(double) + 64;
  if (hipMallocAsync((void **)&buf, nb, st) != hipSuccess) return fail(FRG_E_NOMEM, "fvlpa staging");
  double *du = buf, *dt = du + m;
  int *flag = (int *)(dt + n_flows);
  hipMemcpyAsync(du, u, m * sizeof(double), hipMemcpyHostToDevice, st);
  rc = ctx->fvlpa_device(*fv, n_flows, t_end, n_steps, du, dt, nullptr, nullptr, 0.0, flag, st);
  if (!rc) {
    hipMemcpyAsync(u, du, m * sizeof(double), hipMemcpyDeviceToHost, st);
    hipMemcpyAsync(t_reached, dt, n_flows * sizeof(double), hipMemcpyDeviceToHost, st);
  }
  (void)hipFreeAsync(buf, st);
  hipError_t e = hipStreamSynchronize(st);
  if (rc) return rc;
  if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
  return FRG_OK;
}

}  // extern "C"
