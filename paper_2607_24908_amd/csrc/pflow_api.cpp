// Momentum-dependent two-point flow behind frg_pflow_rhs / frg_pflow_solve:
// argument checks, per-call device scratch (stream-ordered allocations, so
// that calls on different streams never share it), and the stage loop of
// the RK4 integration, every stage launched on the caller's stream.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>

#include "frg_ctx.h"

namespace frg {

static int check_pflow(const frg_pflow &pf, int64_t n_flows) {
  if (pf.d < 3 || pf.d > 8) return fail(FRG_E_INVAL, "pflow.d=%d outside [3, 8]", pf.d);
  if (pf.reg != FRG_REG_EXP && pf.reg != FRG_REG_LITIM)
    return fail(FRG_E_INVAL, "pflow.reg=%d unknown", pf.reg);
  if (pf.n_radial < 1 || pf.n_radial > 1024) return fail(FRG_E_INVAL, "pflow.n_radial outside [1, 1024]");
  if (pf.n_angular < 1 || pf.n_angular > 256) return fail(FRG_E_INVAL, "pflow.n_angular outside [1, 256]");
  if (!(pf.lambda > 0.0) || !std::isfinite(pf.lambda)) return fail(FRG_E_INVAL, "pflow.lambda must be finite and > 0");
  if (!(pf.q_max_over_k > 0.0) || !std::isfinite(pf.q_max_over_k))
    return fail(FRG_E_INVAL, "pflow.q_max_over_k must be finite and > 0");
  if (pf.n_s < 2 || pf.n_s > ((int64_t)1 << 24)) return fail(FRG_E_INVAL, "pflow.n_s outside [2, 2^24]");
  if (!(pf.s_max > 0.0) || !std::isfinite(pf.s_max)) return fail(FRG_E_INVAL, "pflow.s_max must be finite and > 0");
  if (n_flows < 0 || n_flows > ((int64_t)1 << 24)) return fail(FRG_E_INVAL, "n_flows outside [0, 2^24]");
  if (n_flows * pf.n_s > ((int64_t)1 << 31)) return fail(FRG_E_INVAL, "n_flows * n_s too large");
  return FRG_OK;
}

int Ctx::pflow_device(const frg_pflow &pf, int64_t n, const double *lam3, const double *lam4,
                      double t_end, int64_t n_steps, double *sigma, double *t_reached,
                      double *dsdt, double t_rhs, int *flag, hipStream_t st) {
  frg_quad q{};
  q.d = pf.d;
  q.reg = pf.reg;
  q.k = 1.0;
  q.q_max = pf.q_max_over_k;
  q.n_radial = pf.n_radial;
  q.n_angular = pf.n_angular;
  q.prec = FRG_PREC_FP64;
  const double *base;
  QuadTable h;
  int rc = quad_table(q, &base, &h);
  if (rc) return rc;
  const int64_t ns = pf.n_s, nrs = n * ns;
  const bool solve = dsdt == nullptr;
  // scratch: tabk | p | g | J (2) | T (2) | [ys | acc (2) | y0 (one launch per
  // stage: the step-start state alternates between sigma and this one)] |
  // [t_reached] | alive (2)
  const size_t tabd = (size_t)table_doubles(pf.n_radial, pf.n_angular);
  const size_t nd = tabd + ns + 3 * nrs + 2 * n + (solve ? 4 * nrs : 0) + (t_reached ? 0 : n);
  void *buf = nullptr;
  hipError_t e = hipMallocAsync(&buf, nd * sizeof(double) + 2 * (size_t)n * sizeof(int) + 64, st);
  if (e != hipSuccess) return fail(FRG_E_NOMEM, "pflow scratch: %s", hipGetErrorString(e));
  double *d = (double *)buf;
  PflowArgs a{};
  a.base = base;
  a.tabk = d;
  d += tabd;
  a.p = d;
  d += ns;
  a.g = d;
  d += nrs;
  double *const Js = d;  // J of even / odd launches
  d += 2 * nrs;
  double *const Ts = d;
  d += 2 * n;
  double *accs = nullptr, *y0s = nullptr;
  if (solve) {
    a.ys = d;
    d += nrs;
    accs = d;
    d += 2 * nrs;
    y0s = d;
    d += nrs;
  }
  if (t_reached) {
    a.t_reached = t_reached;
  } else {
    a.t_reached = d;
    d += n;
  }
  int *const alives = (int *)d;
  a.J = Js;
  a.T = Ts;
  a.acc = accs;
  a.alive = alives;
  a.lam3 = lam3;
  a.lam4 = lam4;
  a.y0 = sigma;
  a.dsdt = dsdt;
  a.flag = flag;
  a.Cd = omega_sphere(pf.d) / std::pow(2.0 * M_PI, pf.d);
  a.h_s = pf.s_max / (double)(ns - 1);
  a.inv_h = (double)(ns - 1) / pf.s_max;
  a.t_last = (double)(ns - 1);
  a.n_rows = n;
  a.n_s = ns;
  a.n_r = pf.n_radial;
  a.n_a = pf.n_angular;
  TabArgs tb{};
  tb.p = a.p;
  tb.out = a.J;
  tb.g = a.g;
  tb.tab = a.tabk;
  tb.flag = flag;
  tb.pref = h.pref;
  tb.inv_h = a.inv_h;
  tb.t_last = a.t_last;
  tb.n_p = ns;
  tb.n_rows = n;
  tb.n_s = ns;
  tb.os_p = n;  // J[a * n_rows + r]; one launch per stage: J[r * n_s + a]
  tb.os_r = 1;
  tb.n_r = pf.n_radial;
  tb.n_a = pf.n_angular;
  bool lds_rows = false;
  int W = 1;
  int64_t sblocks = 0;
  rc = tab_config(tb, lds_rows, W, sblocks, true);
  const bool pull = tune.pflow_fused && lds_rows && pflow_pull_lds_bytes(tb) <= 150 * 1024;
  auto set_scale = [&](double t, double tn) {
    a.k = pf.lambda * std::exp(t);
    a.k2 = a.k * a.k;
    a.kd2 = std::pow(a.k, pf.d + 2);
    a.t_n = tn;
    tb.k2 = a.k2;
  };
  if (!rc) {
    rc = launch_pflow_init(a, solve ? t_end : t_rhs, st);
    if (rc) rc = hip_fail((hipError_t)rc, "pflow_init_kernel launch");
  }
  const double hh = solve ? t_end / (double)n_steps : 0.0;
  const double cs[4] = {0.0, 0.5, 0.5, 1.0};
  a.h = hh;
  if (!rc && pull) {
    // launch m (stage m of the solve, or the one right-hand side) reads the
    // arrays of parity (m - 1) mod 2 and writes those of parity m mod 2
    // (alive: reads m mod 2, writes (m + 1) mod 2); step s starts from
    // y0[s mod 2], y0[0] being the caller's state
    PflowPull u{};
    u.base = base;
    u.lam3 = lam3;
    u.lam4 = lam4;
    u.t_reached = a.t_reached;
    u.dsdt = dsdt;
    u.flag = flag;
    u.Cd = a.Cd;
    u.h_s = a.h_s;
    u.inv_h = a.inv_h;
    u.t_last = a.t_last;
    u.h = hh;
    u.n_rows = n;
    u.n_s = ns;
    u.n_r = pf.n_radial;
    u.n_a = pf.n_angular;
    tb.tab = base;
    tb.os_p = 1;
    tb.os_r = ns;
    double *const y0b[2] = {sigma, y0s};
    auto point = [&](int64_t m, int prev, int64_t step) {
      const int c = (int)(m & 1), o = c ^ 1;
      u.prev = prev;
      u.Jp = Js + o * nrs;
      u.Jn = Js + c * nrs;
      u.Tp = Ts + o * n;
      u.Tn = Ts + c * n;
      if (solve) {
        u.accp = accs + o * nrs;
        u.accn = accs + c * nrs;
        const bool new_step = prev == 3;
        u.y0p = y0b[(step + (new_step ? 1 : 0)) & 1];
        u.y0n = y0b[step & 1];
      } else {
        u.y0p = sigma;
        u.y0n = nullptr;
      }
      u.alivep = alives + c * n;
      u.aliven = alives + o * n;
    };
    auto stage = [&](int64_t m, int prev, int64_t step, double t, double tn) -> int {
      point(m, prev, step);
      set_scale(t, tn);
      u.k = a.k;
      u.k2 = a.k2;
      u.kd2 = a.kd2;
      u.t_n = tn;
      tb.out = u.Jn;
      const int r = launch_pflow_pull(tb, u, pf.reg, W, st);
      return r ? hip_fail((hipError_t)r, "pflow_pull_kernel launch") : FRG_OK;
    };
    int64_t m = 0;
    if (!solve) {
      rc = stage(0, -1, 0, t_rhs, t_rhs);
      m = 1;
    } else {
      for (int64_t step = 0; step < n_steps && !rc; ++step) {
        const double tn = (double)step * hh;
        for (int s = 0; s < 4 && !rc; ++s, ++m)
          rc = m == 0 ? stage(0, -1, 0, 0.0, 0.0)
                      : stage(m, (s + 3) % 4, step, tn + cs[s] * hh, tn);
      }
    }
    if (!rc) {
      // the update after the last stage: into the caller's state, or dsdt
      point(m, solve ? 3 : 4, solve ? n_steps : 0);
      if (solve) {
        u.y0p = y0b[(n_steps - 1) & 1];
        u.y0n = sigma;
      }
      const int r = launch_pflow_final(u, st);
      if (r) rc = hip_fail((hipError_t)r, "pflow_final_kernel launch");
    }
  } else if (!rc) {
    // prep of the first stage, then per stage: diagram, update (+ next prep)
    auto first_prep = [&](double t, double tn) -> int {
      set_scale(t, tn);
      int r = launch_pflow_prep(a, pf.reg, st);
      return r ? hip_fail((hipError_t)r, "pflow_prep_kernel launch") : FRG_OK;
    };
    auto stage_step = [&](int stage, bool prep_next, double t_next, double tn_next) -> int {
      int r = launch_tab(tb, pf.reg, W, lds_rows, sblocks, st);
      if (r) return hip_fail((hipError_t)r, "tab_kernel launch");
      a.stage = stage;
      a.prep = prep_next ? 1 : 0;
      if (prep_next) set_scale(t_next, tn_next);
      r = launch_pflow_stage(a, pf.reg, st);
      return r ? hip_fail((hipError_t)r, "pflow_stage_kernel launch") : FRG_OK;
    };
    if (!solve) {
      rc = first_prep(t_rhs, t_rhs);
      if (!rc) rc = stage_step(4, false, 0.0, 0.0);
    } else {
      rc = first_prep(0.0, 0.0);
      for (int64_t step = 0; step < n_steps && !rc; ++step) {
        const double tn = (double)step * hh;
        for (int s = 0; s < 4 && !rc; ++s) {
          // the stage after (step, s): (step, s + 1), or (step + 1, 0)
          const bool last = s == 3 && step + 1 == n_steps;
          const double tn_next = s < 3 ? tn : (double)(step + 1) * hh;
          const double t_next = s < 3 ? tn + cs[s + 1] * hh : tn_next;
          rc = stage_step(s, !last, t_next, tn_next);
        }
      }
    }
  }
  (void)hipFreeAsync(buf, st);
  return rc;
}

}  // namespace frg

using namespace frg;

extern "C" {

int frg_pflow_rhs(frg_ctx *ctx, const frg_pflow *pf, int64_t n_flows, const double *lam3,
                  const double *lam4, double t, const double *sigma, double *dsdt, int32_t mem,
                  void *hip_stream) {
  frg::TraceRange trace_("frg_pflow_rhs");
  if (!ctx || !pf) return fail(FRG_E_INVAL, "NULL argument");
  int rc = check_pflow(*pf, n_flows);
  if (rc) return rc;
  if (!std::isfinite(t)) return fail(FRG_E_INVAL, "t must be finite");
  if (mem != FRG_MEM_HOST && mem != FRG_MEM_DEVICE) return fail(FRG_E_INVAL, "bad mem");
  if (n_flows == 0) return FRG_OK;
  if (!lam3 || !lam4 || !sigma || !dsdt) return fail(FRG_E_INVAL, "NULL array");
  std::lock_guard<std::mutex> lk(ctx->mu);
  hipSetDevice(ctx->device);
  clear_error();
  const int64_t nrs = n_flows * pf->n_s;
  if (mem == FRG_MEM_DEVICE) {
    hipStream_t st = (hipStream_t)hip_stream;
    int *flag = nullptr;
    if (hipMallocAsync((void **)&flag, sizeof(int), st) != hipSuccess)
      return fail(FRG_E_NOMEM, "pflow flag");
    rc = ctx->pflow_device(*pf, n_flows, lam3, lam4, 0.0, 1, const_cast<double *>(sigma), nullptr,
                           dsdt, t, flag, st);
    (void)hipFreeAsync(flag, st);
    return rc;
  }
  hipStream_t st = ctx->stream;
  double *buf = nullptr;
  const size_t nb = (size_t)(2 * n_flows + 2 * nrs) * sizeof(double) + 64;
  if (hipMallocAsync((void **)&buf, nb, st) != hipSuccess) return fail(FRG_E_NOMEM, "pflow staging");
  double *d3 = buf, *d4 = d3 + n_flows, *ds = d4 + n_flows, *dd = ds + nrs;
  int *flag = (int *)(dd + nrs);
  hipMemcpyAsync(d3, lam3, n_flows * sizeof(double), hipMemcpyHostToDevice, st);
  hipMemcpyAsync(d4, lam4, n_flows * sizeof(double), hipMemcpyHostToDevice, st);
  hipMemcpyAsync(ds, sigma, nrs * sizeof(double), hipMemcpyHostToDevice, st);
  rc = ctx->pflow_device(*pf, n_flows, d3, d4, 0.0, 1, ds, nullptr, dd, t, flag, st);
  int hflag = 0;
  if (!rc) {
    hipMemcpyAsync(dsdt, dd, nrs * sizeof(double), hipMemcpyDeviceToHost, st);
    hipMemcpyAsync(&hflag, flag, sizeof(int), hipMemcpyDeviceToHost, st);
  }
  (void)hipFreeAsync(buf, st);
  hipError_t e = hipStreamSynchronize(st);
  if (rc) return rc;
  if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
  if (hflag) return fail(FRG_E_DOMAIN, "some flows are outside the domain; their rows are NaN");
  return FRG_OK;
}

int frg_pflow_solve(frg_ctx *ctx, const frg_pflow *pf, int64_t n_flows, const double *lam3,
                    const double *lam4, double t_end, int64_t n_steps, double *sigma,
                    double *t_reached, int32_t mem, void *hip_stream) {
  frg::TraceRange trace_("frg_pflow_solve");
  if (!ctx || !pf) return fail(FRG_E_INVAL, "NULL argument");
  int rc = check_pflow(*pf, n_flows);
  if (rc) return rc;
  if (!std::isfinite(t_end) || t_end > 0.0) return fail(FRG_E_INVAL, "t_end must be finite and <= 0");
  if (n_steps < 1 || n_steps > ((int64_t)1 << 24)) return fail(FRG_E_INVAL, "n_steps outside [1, 2^24]");
  if (mem != FRG_MEM_HOST && mem != FRG_MEM_DEVICE) return fail(FRG_E_INVAL, "bad mem");
  if (n_flows == 0) return FRG_OK;
  if (!lam3 || !lam4 || !sigma || !t_reached) return fail(FRG_E_INVAL, "NULL array");
  std::lock_guard<std::mutex> lk(ctx->mu);
  hipSetDevice(ctx->device);
  clear_error();
  const int64_t nrs = n_flows * pf->n_s;
  if (mem == FRG_MEM_DEVICE) {
    hipStream_t st = (hipStream_t)hip_stream;
    int *flag = nullptr;
    if (hipMallocAsync((void **)&flag, sizeof(int), st) != hipSuccess)
      return fail(FRG_E_NOMEM, "pflow flag");
    rc = ctx->pflow_device(*pf, n_flows, lam3, lam4, t_end, n_steps, sigma, t_reached, nullptr,
                           0.0, flag, st);
    (void)hipFreeAsync(flag, st);
    return rc;
  }
  hipStream_t st = ctx->stream;
  double *buf = nullptr;
  const size_t nb = (size_t)(3 * n_flows + nrs) * sizeof(double) + 64;
  if (hipMallocAsync((void **)&buf, nb, st) != hipSuccess) return fail(FRG_E_NOMEM, "pflow staging");
  double *d3 = buf, *d4 = d3 + n_flows, *dt = d4 + n_flows, *ds = dt + n_flows;
  int *flag = (int *)(ds + nrs);
  hipMemcpyAsync(d3, lam3, n_flows * sizeof(double), hipMemcpyHostToDevice, st);
  hipMemcpyAsync(d4, lam4, n_flows * sizeof(double), hipMemcpyHostToDevice, st);
  hipMemcpyAsync(ds, sigma, nrs * sizeof(double), hipMemcpyHostToDevice, st);
  rc = ctx->pflow_device(*pf, n_flows, d3, d4, t_end, n_steps, ds, dt, nullptr, 0.0, flag, st);
  if (!rc) {
    hipMemcpyAsync(sigma, ds, nrs * sizeof(double), hipMemcpyDeviceToHost, st);
    hipMemcpyAsync(t_reached, dt, n_flows * sizeof(double), hipMemcpyDeviceToHost, st);
  }
  (void)hipFreeAsync(buf, st);
  hipError_t e = hipStreamSynchronize(st);
  if (rc) return rc;
  if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
  return FRG_OK;
}

}  // extern "C"
