// Host-side checks of libfrg's pure host code under AddressSanitizer and
// UndefinedBehaviorSanitizer (built with g++, no GPU): the Gauss-Legendre
// rule, the packed quadrature, LPA and vertex tables, the lane split, and the
// BDF(1,2) flow stepper (frg_flow_solve) with a host right-hand side.
//
// The library's error plumbing (fail, clear_error, now_s, check_lpa) lives
// in its device-side translation unit; the minimal stand-ins below are test
// plumbing only (the inputs here are valid, so check_lpa has nothing to
// reject).  Exit status 0 and the line "host checks ok" mean every check held.
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <vector>

#include "frg_internal.h"

namespace frg {
int fail(int code, const char *fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  std::vfprintf(stderr, fmt, ap);
  va_end(ap);
  std::fputc('\n', stderr);
  return code;
}
void clear_error() {}
double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}
int check_lpa(const frg_lpa &) { return 0; }
}  // namespace frg

static int failures = 0;
#define CHECK(c)                                                        \
  do {                                                                  \
    if (!(c)) {                                                         \
      std::fprintf(stderr, "check failed at line %d: %s\n", __LINE__, #c); \
      ++failures;                                                       \
    }                                                                   \
  } while (0)

// dU/dt = -c (U_{j-1} - 2 U_j + U_{j+1}) with U_{-1} = U_0, U_n = U_{n-1}:
// minus the discrete Neumann Laplacian, i.e. diffusion as t decreases (the
// flow runs from t = 0 to t_end < 0).  sum_j U_j is conserved by the ODE and
// by every BDF step up to the Newton iteration's residual.
struct Diffusion {
  double c;
};
static int diffusion_rhs(void *user, double, const double *U, int64_t n, double *dUdt,
                         double *jac) {
  const double c = static_cast<Diffusion *>(user)->c;
  for (int64_t j = 0; j < n; ++j) {
    const double l = U[j > 0 ? j - 1 : 0], r = U[j + 1 < n ? j + 1 : n - 1];
    dUdt[j] = -c * (l - 2.0 * U[j] + r);
  }
  if (jac) {
    for (int64_t k = 0; k < 7 * n; ++k) jac[k] = 0.0;
    for (int64_t j = 0; j < n; ++j) {
      double dm = -c, d0 = 2.0 * c, dp = -c;
      if (j == 0) { d0 += dm; dm = 0.0; }
      if (j == n - 1) { d0 += dp; dp = 0.0; }
      jac[(-1 + 3) * n + j] = dm;
      jac[(0 + 3) * n + j] = d0;
      jac[(1 + 3) * n + j] = dp;
    }
  }
  return FRG_OK;
}

int main() {
  // Gauss-Legendre: weights sum to 2, nodes ascend and are symmetric
  for (int n = 1; n <= 96; n += 5) {
    std::vector<double> x(n), w(n);
    CHECK(frg::gauss_legendre_gw(n, x.data(), w.data()) == 0);
    double sw = 0.0;
    for (int i = 0; i < n; ++i) {
      sw += w[i];
      CHECK(std::fabs(x[i] + x[n - 1 - i]) < 1e-14);
      if (i) CHECK(x[i] > x[i - 1]);
    }
    CHECK(std::fabs(sw - 2.0) < 1e-13);
  }
  // packed quadrature tables, both regulators, several shapes
  for (int reg : {FRG_REG_EXP, FRG_REG_LITIM})
    for (int d : {3, 4, 6})
      for (int nr : {1, 7, 64})
        for (int na : {1, 5, 32}) {
          frg_quad q{};
          q.d = d;
          q.reg = reg;
          q.k = 0.7;
          q.q_max = 6.0 * q.k;
          q.n_radial = nr;
          q.n_angular = na;
          const frg::QuadTable t = frg::build_quad_table(q);
          CHECK((int)t.data.size() == frg::table_doubles(nr, na));
          for (double v : t.data) CHECK(std::isfinite(v));
        }
  // LPA tables with their coefficient groups, and vertex angular tables
  for (int reg : {FRG_REG_EXP, FRG_REG_LITIM})
    for (int nr : {1, 8, 9, 64, 100}) {
      const frg::LpaTable t = frg::build_lpa_table(3, reg, nr, 6.0);
      CHECK((int)t.data.size() >= 2 * nr);
      for (double v : t.data) CHECK(std::isfinite(v));
    }
  for (int na : {1, 8}) {
    const std::vector<double> v = frg::build_vertex_table(3, na, 16);
    for (double e : v) CHECK(std::isfinite(e));
  }
  for (int nr : {1, 33, 128})
    for (int na : {1, 3, 32, 256}) {
      int R, J, T, U;
      frg::lane_split(nr, na, &R, &J, &T, &U);
      CHECK(R * J == frg::kWave && R * T >= nr && J * U >= na);
    }
  // the flow stepper on the Neumann diffusion: status OK, total conserved
  for (int64_t n : {4, 37, 256}) {
    std::vector<double> U(n);
    frg_request rq{};
    rq.lpa.d = 3;
    rq.lpa.N = 1;
    rq.lpa.reg = FRG_REG_LITIM;
    rq.lpa.n_radial = 8;
    rq.lpa.q_max_over_k = 6.0;
    rq.lpa.Lambda = 1.0;
    rq.lpa.n_grid = n;
    rq.lpa.rho_max = 1.0;
    rq.lambda = 8.0;
    rq.rho0 = 0.4;
    rq.t_end = -0.5;
    rq.rtol = 1e-8;
    rq.atol = 1e-10;
    rq.U_out = U.data();
    Diffusion df{0.05 * (double)((n - 1) * (n - 1))};
    frg_result res{};
    const int rc = frg_flow_solve(&rq, diffusion_rhs, &df, &res);
    CHECK(rc == FRG_OK && res.status == FRG_OK && res.steps > 0);
    // initial total: sum_j (lambda/8)(rho_j - rho0)^2 on rho_j = j rho_max/(n - 1)
    double s0 = 0.0, s1 = 0.0;
    for (int64_t j = 0; j < n; ++j) {
      const double rho = (double)j / (double)(n - 1) - rq.rho0;
      s0 += rho * rho;
      s1 += U[j];
      CHECK(std::isfinite(U[j]));
    }
    CHECK(std::fabs(s1 - s0) <= 1e-12 * s0);  // measured: below 1e-14
  }
  if (failures) {
    std::fprintf(stderr, "%d host checks failed\n", failures);
    return 1;
  }
  std::printf("host checks ok\n");
  return 0;
}
