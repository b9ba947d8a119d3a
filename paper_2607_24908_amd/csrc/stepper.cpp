// Host FP64 implicit stepper for the LPA flow (method of lines in rho,
// integrated in RG time t from 0 to t_end < 0).
//
// Method: variable-step BDF of order 1 (first two steps) and 2, in the form
//   y_{n+1} - psi = gamma f(t_{n+1}, y_{n+1}),
// BDF2 with omega = h_n/h_{n-1}:
//   psi = ((1+omega)^2 y_n - omega^2 y_{n-1}) / (1 + 2 omega),
//   gamma = h_n (1+omega)/(1+2 omega).
// Newton on y - psi - gamma f(y) = 0 with the banded Jacobian returned by the
// right-hand side (7 bands), solved by banded LU with partial pivoting.
// Local error: BDF2 residual -gamma h_n (h_n + h_{n-1}) y'''/6 with y''' from
// the third divided difference over four solution points; BDF1 residual
// -h^2 y''/2 with y'' from the second divided difference.  Weighted RMS norm
// with weights atol + rtol max(|y_n|, |y_{n+1}|).  A right-hand side that
// reports a domain violation (a mass crossing the pole) rejects the step;
// when such rejections drive the step below 1e-8 |t_end| the flow has run
// into the singularity m^2 = -k^2 and ends with FRG_E_DOMAIN.  U_out always
// holds the last accepted state and t_reached its RG time.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <vector>

#include "frg_ctx.h"

namespace frg {

namespace {

constexpr int KL = 3, KU = 3, KV = KL + KU, LDAB = 2 * KL + KU + 1;

// Banded LU with partial pivoting; A(i,j) at ab[(KV + i - j) * n + j].
struct BandLU {
  int64_t n = 0;
  std::vector<double> ab;
  std::vector<int64_t> piv;
  double &A(int64_t i, int64_t j) { return ab[(KV + i - j) * n + j]; }

  // A = I - gamma J, J in the 7-band layout jac[(o+3)*n + j] = dF_j/dU_{j+o}
  void assemble(int64_t n_, double gamma, const double *jac) {
    n = n_;
    ab.assign((size_t)LDAB * n, 0.0);
    piv.assign(n, 0);
    for (int64_t i = 0; i < n; ++i)
      for (int o = -3; o <= 3; ++o) {
        const int64_t j = i + o;
        if (j < 0 || j >= n) continue;
        A(i, j) = (o == 0 ? 1.0 : 0.0) - gamma * jac[(o + 3) * n + i];
      }
  }

  bool factor() {
    int64_t ju = 0;
    for (int64_t j = 0; j < n; ++j) {
      const int64_t km = std::min<int64_t>(KL, n - 1 - j);
      int64_t jp = 0;
      double best = std::fabs(A(j, j));
      for (int64_t r = 1; r <= km; ++r)
        if (std::fabs(A(j + r, j)) > best) {
          best = std::fabs(A(j + r, j));
          jp = r;
        }
      piv[j] = j + jp;
      if (!(best > 0.0) || !std::isfinite(best)) return false;
      ju = std::max(ju, std::min<int64_t>(j + KU + jp, n - 1));
      if (jp)
        for (int64_t c = j; c <= ju; ++c) std::swap(A(j, c), A(j + jp, c));
      if (km > 0) {
        const double inv = 1.0 / A(j, j);
        for (int64_t r = 1; r <= km; ++r) A(j + r, j) *= inv;
        for (int64_t c = j + 1; c <= ju; ++c) {
          const double a = A(j, c);
          if (a != 0.0)
            for (int64_t r = 1; r <= km; ++r) A(j + r, c) -= A(j + r, j) * a;
        }
      }
    }
    return true;
  }

  void solve(double *b) {
    for (int64_t j = 0; j < n; ++j) {
      const int64_t km = std::min<int64_t>(KL, n - 1 - j);
      if (piv[j] != j) std::swap(b[j], b[piv[j]]);
      for (int64_t r = 1; r <= km; ++r) b[j + r] -= A(j + r, j) * b[j];
    }
    for (int64_t j = n - 1; j >= 0; --j) {
      b[j] /= A(j, j);
      const double x = b[j];
      for (int64_t i = std::max<int64_t>(0, j - KV); i < j; ++i) b[i] -= A(i, j) * x;
    }
  }
};

double wrms(const std::vector<double> &e, const std::vector<double> &ya,
            const std::vector<double> &yb, double rtol, double atol) {
  double s = 0.0;
  const size_t n = e.size();
  for (size_t i = 0; i < n; ++i) {
    const double w = atol + rtol * std::max(std::fabs(ya[i]), std::fabs(yb[i]));
    const double r = e[i] / w;
    s += r * r;
  }
  return std::sqrt(s / (double)n);
}

}  // namespace

int solve_flow(const frg_request &rq, frg_rhs_fn rhs, void *user, frg_result *res) {
  const frg_lpa &l = rq.lpa;
  const int64_t n = l.n_grid;
  const double t_end = rq.t_end;
  const double rtol = rq.rtol > 0 ? rq.rtol : 1e-6;
  const double atol = rq.atol > 0 ? rq.atol : 1e-9;
  res->steps = res->rejected = res->rhs_calls = 0;
  res->status = FRG_PENDING;
  const double dr = l.rho_max / (double)(n - 1);
  std::vector<double> y(n);
  for (int64_t j = 0; j < n; ++j) {
    const double rho = (double)j * dr;
    const double x = rho - rq.rho0;
    y[j] = (rq.lambda / 8.0) * (x * x);
  }
  if (!(t_end < 0.0)) {
    std::memcpy(rq.U_out, y.data(), n * sizeof(double));
    res->t_reached = 0.0;
    res->status = FRG_OK;
    return FRG_OK;
  }
  std::vector<double> f(n), jac(7 * n), ynew(n), g(n), dy(n), err(n);
  // history: most recent first
  std::vector<double> yh[3] = {y, y, y};
  double th[3] = {0.0, 0.0, 0.0};
  int nhist = 1;
  double hprev = 0.0, hprev2 = 0.0;
  // contraction rate of the Newton iteration, carried from step to step: an
  // iterate whose correction times this rate is below the convergence bar
  // is accepted (the next correction would be that small), which usually
  // saves the second right-hand side of a step.  Every kRateCheck steps so
  // accepted, a step iterates twice again so that the rate is measured anew.
  double crate = 1.0;
  constexpr int kRateCheck = 16;
  int unchecked = 0;

  auto call = [&](double t, const std::vector<double> &u, bool want_jac) -> int {
    res->rhs_calls++;
    return rhs(user, t, u.data(), n, f.data(), want_jac ? jac.data() : nullptr);
  };
  res->t_reached = 0.0;
  std::memcpy(rq.U_out, y.data(), n * sizeof(double));
  int rc = call(0.0, y, false);
  if (rc != FRG_OK) {
    res->status = rc;
    return rc;
  }
  // initial step from the size of the right-hand side
  double fn = 0.0, yn = 0.0;
  for (int64_t i = 0; i < n; ++i) {
    const double w = atol + rtol * std::fabs(y[i]);
    fn += (f[i] / w) * (f[i] / w);
    yn += (y[i] / w) * (y[i] / w);
  }
  fn = std::sqrt(fn / n);
  double h = -std::min(0.01 * std::fabs(t_end), fn > 0 ? 0.05 / fn : 0.01);
  h = std::min(h, -1e-10);
  std::vector<double> f0 = f;
  const double hmin = 1e-13 * std::fabs(t_end);
  const double hmin_pole = 1e-8 * std::fabs(t_end);
  double t = 0.0;
  BandLU lu;
  const bool dbg = std::getenv("FRG_STEPPER_DEBUG") != nullptr;
  while (t > t_end) {
    if (h < t_end - t) h = t_end - t;  // do not step past the end
    const int order = (nhist >= 3) ? 2 : 1;
    // --- predictor and BDF coefficients
    double gamma, omega = 0.0;
    std::vector<double> &y0 = yh[0];
    if (order == 2) {
      omega = h / hprev;
      const double den = 1.0 + 2.0 * omega;
      gamma = h * (1.0 + omega) / den;
      const double a = (1.0 + omega) * (1.0 + omega) / den, b = omega * omega / den;
      for (int64_t i = 0; i < n; ++i) {
        g[i] = a * y0[i] - b * yh[1][i];  // psi
        ynew[i] = y0[i] + omega * (y0[i] - yh[1][i]);
      }
    } else {
      gamma = h;
      for (int64_t i = 0; i < n; ++i) {
        g[i] = y0[i];
        ynew[i] = (nhist >= 2) ? y0[i] + (h / hprev) * (y0[i] - yh[1][i]) : y0[i] + h * f0[i];
      }
    }
    // --- Newton: the Jacobian bands and their factorisation at the first
    // iterate, reused by the later ones (a fresh pair only when the
    // iterates stop contracting)
    bool conv = false, domain = false, have_lu = false;
    double prev_norm = 0.0;
    for (int it = 0; it < 8; ++it) {
      const bool fresh = !have_lu;
      rc = call(t + h, ynew, fresh);
      if (rc == FRG_E_DOMAIN) {
        domain = true;
        break;
      }
      if (rc != FRG_OK) {
        res->status = rc;
        return rc;
      }
      for (int64_t i = 0; i < n; ++i) dy[i] = -(ynew[i] - g[i] - gamma * f[i]);
      if (fresh) {
        lu.assemble(n, gamma, jac.data());
        if (!lu.factor()) break;
        have_lu = true;
      }
      lu.solve(dy.data());
      bool finite = true;
      for (int64_t i = 0; i < n; ++i) {
        ynew[i] += dy[i];
        finite &= std::isfinite(ynew[i]);
      }
      if (!finite) break;
      const double nrm = wrms(dy, y0, ynew, rtol, atol);
      if (it > 0 && prev_norm > 0.0) {
        crate = std::max(0.3 * crate, nrm / prev_norm);
        unchecked = 0;
      }
      if (dbg)
        std::fprintf(stderr, "t=%.17g h=%.3e ord=%d it=%d nrm=%.3e crate=%.3e\n", t, h, order, it,
                     nrm, crate);
      const bool by_rate = it == 0 && unchecked < kRateCheck && nrm * std::min(1.0, crate) < 1e-3;
      if (nrm < 1e-3 || by_rate || (it > 0 && nrm < 0.05 && nrm < 0.2 * prev_norm)) {
        if (by_rate && !(nrm < 1e-3)) ++unchecked;
        conv = true;
        break;
      }
      if (it > 0 && nrm > 0.5 * prev_norm) {
        if (!fresh)
          have_lu = false;  // reused bands contract slowly: fresh ones next
        else if (it > 1 && nrm > 0.9 * prev_norm)
          break;  // fresh bands and still no contraction
      }
      prev_norm = nrm;
    }
    if (!conv) {
      if (dbg) std::fprintf(stderr, "reject newton t=%.17g h=%.3e domain=%d\n", t, h, (int)domain);
      res->rejected++;
      h *= domain ? 0.25 : 0.3;
      crate = 1.0;  // the rate no longer describes the iteration
      // a flow whose steps collapse on pole crossings has reached the
      // singularity m^2 = -k^2 of the propagator: it ends there
      const double floor = domain ? hmin_pole : hmin;
      if (std::fabs(h) < floor) {
        res->status = domain ? FRG_E_DOMAIN : FRG_E_STEP;
        return res->status;
      }
      continue;
    }
    // --- local error estimate
    double en;
    if (order == 2) {
      // third divided difference over (t+h, th0, th1, th2)
      const double t0 = t + h, t1 = th[0], t2 = th[1], t3 = th[2];
      for (int64_t i = 0; i < n; ++i) {
        const double d01 = (ynew[i] - yh[0][i]) / (t0 - t1);
        const double d12 = (yh[0][i] - yh[1][i]) / (t1 - t2);
        const double d23 = (yh[1][i] - yh[2][i]) / (t2 - t3);
        const double d012 = (d01 - d12) / (t0 - t2);
        const double d123 = (d12 - d23) / (t1 - t3);
        const double d3 = (d012 - d123) / (t0 - t3);  // y'''/6
        err[i] = gamma * h * (h + hprev) * d3;
      }
    } else if (nhist >= 2) {
      const double t0 = t + h, t1 = th[0], t2 = th[1];
      for (int64_t i = 0; i < n; ++i) {
        const double d01 = (ynew[i] - yh[0][i]) / (t0 - t1);
        const double d12 = (yh[0][i] - yh[1][i]) / (t1 - t2);
        err[i] = h * h * (d01 - d12) / (t0 - t2);  // h^2 y''/2
      }
    } else {
      for (int64_t i = 0; i < n; ++i) err[i] = (ynew[i] - y0[i]) - h * f0[i];
    }
    en = wrms(err, y0, ynew, rtol, atol);
    const double k = order + 1;
    double fac = 0.9 * std::pow(std::max(en, 1e-10), -1.0 / k);
    if (en > 1.0) {
      res->rejected++;
      h *= std::max(0.2, std::min(0.9, fac));
      crate = 1.0;  // after a rejection every iterate is checked again
      if (std::fabs(h) < hmin) {
        res->status = FRG_E_STEP;
        return FRG_E_STEP;
      }
      continue;
    }
    // --- accept
    t += h;
    res->steps++;
    res->t_reached = t;
    std::memcpy(rq.U_out, ynew.data(), n * sizeof(double));
    yh[2].swap(yh[1]);
    yh[1].swap(yh[0]);
    yh[0] = ynew;
    th[2] = th[1];
    th[1] = th[0];
    th[0] = t;
    nhist = std::min(nhist + 1, 3);
    hprev2 = hprev;
    hprev = h;
    double hn = h * std::min(2.0, std::max(0.5, fac));
    if (nhist >= 3) {
      // keep the BDF2 step ratio in a zero-stable range
      hn = std::max(hn, 2.0 * h);
      hn = std::min(hn, 0.3 * h);
    }
    h = hn;
  }
  (void)hprev2;
  res->status = FRG_OK;
  return FRG_OK;
}

}  // namespace frg

extern "C" int frg_flow_solve(const frg_request *req, frg_rhs_fn rhs, void *user, frg_result *out) {
  using namespace frg;
  if (!req || !rhs || !out || !req->U_out) return fail(FRG_E_INVAL, "NULL argument");
  int rc = check_lpa(req->lpa);
  if (rc) return rc;
  if (!std::isfinite(req->t_end) || req->t_end > 0.0) return fail(FRG_E_INVAL, "t_end must be <= 0");
  if (!std::isfinite(req->lambda) || !std::isfinite(req->rho0)) return fail(FRG_E_INVAL, "bad initial potential");
  std::memset(out, 0, sizeof *out);
  out->submit_s = out->start_s = now_s();
  rc = solve_flow(*req, rhs, user, out);
  out->done_s = now_s();
  if (rc != FRG_OK)
    return fail(rc, "flow stopped (status %d) at t = %.6g after %lld steps", rc, out->t_reached,
                (long long)out->steps);
  clear_error();
  return FRG_OK;
}
