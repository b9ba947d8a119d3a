// Host-side quadrature and regulator tables.
//
// The Gauss-Legendre rule comes from the Golub-Welsch construction: the
// nodes are the eigenvalues of the symmetric tridiagonal Jacobi matrix of
// the Legendre polynomials (zero diagonal, off-diagonal j/sqrt(4j^2-1)),
// found by the implicit QL iteration with Wilkinson-type shifts in 80-bit
// arithmetic and polished by Newton steps on P_n; the weights are
//   w = 2 / ((1 - x^2) P_n'(x)^2),  (1 - x^2) P_n'(x) = n (P_{n-1}(x) - x P_n(x)).
#include <algorithm>
#include <cmath>
#include <vector>

#include "frg_internal.h"

namespace frg {

int gauss_legendre_gw(int n, double *x, double *w) {
  if (n < 1 || n > 4096 || !x || !w) return FRG_E_INVAL;
  std::vector<long double> d(n, 0.0L), e(n, 0.0L);
  for (int j = 1; j < n; ++j) e[j - 1] = j / sqrtl(4.0L * j * j - 1.0L);
  // implicit QL on (d, e): e[i] couples i and i+1
  for (int l = 0; l < n; ++l) {
    for (int iter = 0; iter < 200; ++iter) {
      int m = l;
      for (; m < n - 1; ++m) {
        long double dd = fabsl(d[m]) + fabsl(d[m + 1]);
        if (fabsl(e[m]) + dd == dd) break;
      }
      if (m == l) break;
      long double g = (d[l + 1] - d[l]) / (2.0L * e[l]);
      long double r = hypotl(g, 1.0L);
      g = d[m] - d[l] + e[l] / (g + (g >= 0 ? r : -r));
      long double s = 1.0L, c = 1.0L, p = 0.0L;
      int i = m - 1;
      bool deflated = false;
      for (; i >= l; --i) {
        long double f = s * e[i], b = c * e[i];
        r = hypotl(f, g);
        e[i + 1] = r;
        if (r == 0.0L) {
          d[i + 1] -= p;
          e[m] = 0.0L;
          deflated = true;
          break;
        }
        s = f / r;
        c = g / r;
        g = d[i + 1] - p;
        r = (d[i] - g) * s + 2.0L * c * b;
        p = s * r;
        d[i + 1] = g + p;
        g = c * r - b;
      }
      if (deflated) continue;
      d[l] -= p;
      e[l] = g;
      e[m] = 0.0L;
    }
  }
  std::sort(d.begin(), d.end());
  for (int i = 0; i < n; ++i) {
    // symmetrise: the rule is exactly symmetric about 0
    long double xi = 0.5L * (d[i] - d[n - 1 - i]);
    if (2 * i + 1 == n) xi = 0.0L;
    // P_{n-1}(xi) and P_n(xi) by the three-term recurrence; two Newton
    // corrections of the eigenvalue on P_n remove the QL rounding that the
    // weight formula would amplify near the ends of [-1, 1].
    long double pm = 1.0L, pn = xi;  // P_{n-1}, P_n
    for (int pass = 0; pass < 3; ++pass) {
      long double p0 = 1.0L, p1 = xi;
      for (int j = 1; j < n; ++j) {
        long double p2 = ((2.0L * j + 1.0L) * xi * p1 - j * p0) / (j + 1.0L);
        p0 = p1;
        p1 = p2;
      }
      pm = (n == 1) ? 1.0L : p0;
      pn = (n == 1) ? xi : p1;
      if (pass == 2 || 2 * i + 1 == n) break;
      const long double dpn = n * (xi * pn - pm) / (xi * xi - 1.0L);
      xi -= pn / dpn;
    }
    // w = 2 / ((1 - x^2) P_n'(x)^2) with (1 - x^2) P_n' = n (P_{n-1} - x P_n)
    const long double omx2 = (1.0L - xi) * (1.0L + xi);
    const long double s = n * (pm - xi * pn);
    long double wi = 2.0L * omx2 / (s * s);
    x[i] = (double)xi;
    w[i] = (double)wi;
  }
  return FRG_OK;
}

double omega_sphere(int n) { return 2.0 * std::pow(M_PI, 0.5 * n) / std::tgamma(0.5 * n); }

// h(y) = y/(1 - e^{-y}) - 1, Bernoulli series below 0.1
double h_exp_host(double y) {
  if (y < 0.1) {
    const double y2 = y * y;
    return y * 0.5 + y2 * (1.0 / 12.0 + y2 * (-1.0 / 720.0 + y2 * (1.0 / 30240.0 +
                                  y2 * (-1.0 / 1209600.0 + y2 * (1.0 / 47900160.0)))));
  }
  return y / (-std::expm1(-y)) - 1.0;
}

static double bern(double z) { return z == 0.0 ? 1.0 : z / std::expm1(z); }

double dtR_over_k2_host(int reg, double y) {
  if (reg == FRG_REG_EXP) return 2.0 * bern(y) * bern(-y);
  return y < 1.0 ? 2.0 : 0.0;
}

static double angular_weight_factor(int d, double x) {
  const double z = (1.0 - x) * (1.0 + x);
  double f = 1.0;
  for (int i = 0; i < (d - 3) / 2; ++i) f *= z;
  if ((d - 3) % 2) f *= std::sqrt(z);
  return f;
}

QuadTable build_quad_table(const frg_quad &q) {
  QuadTable t;
  const int nr = q.n_radial, na = q.n_angular;
  t.n_r = nr;
  t.n_a = na;
  t.k2 = q.k * q.k;
  t.inv_k2 = 1.0 / t.k2;
  t.pref = omega_sphere(q.d - 1) / std::pow(2.0 * M_PI, q.d);
  t.q_top = q.q_max;
  t.rmu_max = 0.0;
  t.data.assign(table_doubles(nr, na), 0.0);
  std::vector<double> xr(nr), wr(nr), xa(na), wa(na);
  gauss_legendre_gw(nr, xr.data(), wr.data());
  gauss_legendre_gw(na, xa.data(), wa.data());
  const double Q = (q.reg == FRG_REG_LITIM) ? std::min(q.q_max, q.k) : q.q_max;
  for (int i = 0; i < nr; ++i) {
    const double qi = 0.5 * Q * (1.0 + xr[i]);
    const double wi = 0.5 * Q * wr[i];
    const double s = qi * qi, y = s / t.k2;
    double qp = 1.0;
    for (int e = 0; e < q.d - 1; ++e) qp *= qi;
    t.data[i] = qi;
    t.data[nr + i] = wi * qp * (t.k2 * dtR_over_k2_host(q.reg, y));
    t.data[2 * nr + i] =
        (q.reg == FRG_REG_EXP) ? t.k2 * h_exp_host(y) : std::max(s - t.k2, 0.0);
  }
  for (int j = 0; j < na; ++j) {
    t.data[3 * nr + j] = 1.0 + xa[j];
    const double mu = wa[j] * angular_weight_factor(q.d, xa[j]);
    t.data[3 * nr + na + j] = mu;
    t.data[3 * nr + 2 * na + j] = 1.0 / mu;
    t.rmu_max = std::max(t.rmu_max, 1.0 / mu);
  }
  return t;
}

LpaTable build_lpa_table(int d, int reg, int n_r, double q_max_over_k) {
  LpaTable t;
  t.n_r = n_r;
  t.Cd = omega_sphere(d) / std::pow(2.0 * M_PI, d);
  t.data.assign(2 * n_r, 0.0);
  std::vector<double> xr(n_r), wr(n_r);
  gauss_legendre_gw(n_r, xr.data(), wr.data());
  const double Q = (reg == FRG_REG_LITIM) ? std::min(q_max_over_k, 1.0) : q_max_over_k;
  for (int i = 0; i < n_r; ++i) {
    const double qi = 0.5 * Q * (1.0 + xr[i]);
    const double wi = 0.5 * Q * wr[i];
    const double y = qi * qi;
    double qp = 1.0;
    for (int e = 0; e < d - 1; ++e) qp *= qi;
    t.data[i] = wi * qp * dtR_over_k2_host(reg, y);
    t.data[n_r + i] = (reg == FRG_REG_EXP) ? h_exp_host(y) : std::max(y - 1.0, 0.0);
  }
  // coefficient groups (products in long double; all terms are >= 0)
  const int ng = fv_groups(n_r);
  t.data.resize(2 * (size_t)n_r + (size_t)kFvCoef * ng, 0.0);
  for (int g = 0; g < ng; ++g) {
    long double c[kFvGroup], h[kFvGroup];
    for (int l = 0; l < kFvGroup; ++l) {
      const int i = kFvGroup * g + l;
      c[l] = i < n_r ? t.data[i] : 0.0L;
      h[l] = i < n_r ? t.data[n_r + i] : 1.0L;
    }
    // poly *= (x + hl), coefficients from x^0 up
    auto mul_lin = [](std::vector<long double> &p, long double hl) {
      p.push_back(0.0L);
      for (size_t k = p.size() - 1; k > 0; --k) p[k] = p[k - 1] + hl * p[k];
      p[0] *= hl;
    };
    std::vector<long double> P{1.0L};
    for (int l = 0; l < kFvGroup; ++l) mul_lin(P, h[l]);
    std::vector<long double> N(kFvGroup, 0.0L), M(2 * kFvGroup - 1, 0.0L);
    for (int i = 0; i < kFvGroup; ++i) {
      std::vector<long double> Pi{1.0L};
      for (int l = 0; l < kFvGroup; ++l)
        if (l != i) mul_lin(Pi, h[l]);
      for (int k = 0; k < kFvGroup; ++k) N[k] += c[i] * Pi[k];
      for (int k = 0; k < kFvGroup; ++k)
        for (int k2 = 0; k2 < kFvGroup; ++k2) M[k + k2] += c[i] * Pi[k] * Pi[k2];
    }
    double *dst = t.data.data() + 2 * (size_t)n_r + (size_t)kFvCoef * g;
    for (int k = 0; k < kFvGroup; ++k) dst[k] = (double)P[k];
    for (int k = 0; k < kFvGroup; ++k) dst[kFvGroup + k] = (double)N[k];
    for (int k = 0; k < 2 * kFvGroup - 1; ++k) dst[2 * kFvGroup + k] = (double)M[k];
  }
  return t;
}

// Angular data of the vertex diagram: [x_j | sqrt(1 - x_j^2) | cos phi_l |
// nu_l], x_j the polar Gauss-Legendre nodes (as in build_quad_table),
// phi_l the Gauss-Legendre nodes on [0, pi] and nu_l = (pi/2) w_l sin^{d-3}(phi_l).
std::vector<double> build_vertex_table(int d, int n_a, int n_phi) {
  std::vector<double> xa(n_a), wa(n_a), xp(n_phi), wp(n_phi);
  gauss_legendre_gw(n_a, xa.data(), wa.data());
  gauss_legendre_gw(n_phi, xp.data(), wp.data());
  std::vector<double> t(2 * n_a + 2 * n_phi);
  for (int j = 0; j < n_a; ++j) {
    t[j] = xa[j];
    t[n_a + j] = std::sqrt((1.0 - xa[j]) * (1.0 + xa[j]));
  }
  for (int l = 0; l < n_phi; ++l) {
    const double f = 0.5 * M_PI * (1.0 + xp[l]);
    t[2 * n_a + l] = std::cos(f);
    t[2 * n_a + n_phi + l] = 0.5 * M_PI * wp[l] * std::pow(std::sin(f), d - 3);
  }
  return t;
}

void lane_split(int n_r, int n_a, int *R, int *J, int *T, int *U) {
  int r = 1;
  while (r * 2 <= n_r && r * 2 <= kWave) r *= 2;
  *R = r;
  *J = kWave / r;
  *T = (n_r + r - 1) / r;
  *U = (n_a + *J - 1) / *J;
}

}  // namespace frg
