/*
 * frg_oracle.c -- plain, slow FP64 CPU oracle for the FRG flow-diagram quadrature.
 *
 * TEST INFRASTRUCTURE ONLY.  Only tests/, the package's smoke check and the
 * benchmark's CPU-baseline leg may load this library.  It shares no code,
 * header, table or constant generator with the HIP library: it builds its own
 * Gauss-Legendre rules (Newton iteration on the Legendre three-term
 * recurrence), evaluates every integrand term from the definition, and sums
 * in natural order with an 80-bit accumulator.
 *
 * What is computed (textbook FRG; the paper's text has no FRG section, so the
 * definitions below are the standard Wetterich-equation ones, stated here in
 * full):
 *
 *   one-loop flow diagram, external momentum p, mass m^2, RG scale k,
 *   t = ln(k/Lambda), d_t = k d/dk:
 *     I(p, m^2) = int d^dq/(2pi)^d  d_tR_k(q^2) G(q^2)^2 G(|q+p|^2),
 *     G(s) = 1/(s + R_k(s) + m^2).
 *   With p along one axis and x = cos(angle(q,p)):
 *     d^dq/(2pi)^d = P_d q^{d-1} dq (1-x^2)^{(d-3)/2} dx,
 *     P_d = Omega_{d-1}/(2pi)^d,  Omega_n = 2 pi^{n/2}/Gamma(n/2).
 *   Discretisation: radial Gauss-Legendre on [0, Q], angular Gauss-Legendre
 *   in x on [-1, 1] with the weight multiplied by (1-x^2)^{(d-3)/2} at the
 *   nodes.  The result is the discrete double sum (this sum IS the method):
 *     I = P_d sum_i sum_j w_i q_i^{d-1} d_tR(q_i^2) G(q_i^2)^2 mu_j G(s_ij),
 *     s_ij = |q_i + p|^2 = (q_i - p)^2 + 2 q_i p (1 + x_j).
 *
 *   Regulators (y = s/k^2):
 *     exponential: R = s/(e^y - 1),  d_tR = 2 k^2 beta(y) beta(-y),
 *                  beta(z) = z/expm1(z);
 *     Litim:       R = (k^2 - s) theta(k^2 - s),  d_tR = 2 k^2 theta(k^2 - s).
 *   Propagator denominator written without cancellation at the pole
 *   m^2 -> -k^2 (delta = m^2 + k^2):
 *     exponential: s + R + m^2 = k^2 h(y) + delta,  h(y) = beta(-y) - 1,
 *                  h from its Bernoulli series below y = 0.1;
 *     Litim:       s + R + m^2 = max(s - k^2, 0) + delta.
 *   Radial domain Q = q_max (exponential), Q = min(q_max, k) (Litim: the
 *   support of d_tR).
 *
 *   Tabulated-propagator variant: the propagator of row r of a caller's
 *   table (a dressed propagator from an earlier solution, n_s values on the
 *   uniform grid s_k = k s_max/(n_s - 1)) replaces G in both places, the
 *   regulator insertion d_tR stays analytic:
 *     I(p, r) = P_d sum_i sum_j w_i q_i^{d-1} d_tR(q_i^2) G_r(q_i^2)^2 mu_j G_r(s_ij),
 *     G_r(s) = (1 - f) g_r[k] + f g_r[k+1],  t = s/h, k = floor(t), f = t - k,
 *   (piecewise-linear interpolation; s >= s_max takes g_r[n_s - 1]).
 *
 *   Two-external-momentum (vertex) diagram: momenta p1, p2 with cos th =
 *   p1.p2/(|p1||p2|), p1 along e1 and p2 in the (e1, e2) plane, q at polar
 *   cosine x to e1 and azimuth phi about e1 measured from the (e1, e2) plane:
 *     V(p1, p2, th, m^2) = int d^dq/(2pi)^d d_tR(q^2) G(q^2)^2 G(|q+p1|^2) G(|q+p2|^2),
 *     |q+p1|^2 = q^2 + p1^2 + 2 q p1 x,
 *     |q+p2|^2 = q^2 + p2^2 + 2 q p2 (x cos th + sqrt(1-x^2) cos phi sin th),
 *     d^dq = q^{d-1} dq (1-x^2)^{(d-3)/2} dx sin^{d-3}phi dphi dOmega_{d-2},
 *   phi in [0, pi], so the prefactor is Omega_{d-2}/(2pi)^d (Omega_1 = 2: the
 *   two half-planes of d = 3).  Discretisation: the radial and x rules of I,
 *   and Gauss-Legendre in phi on [0, pi] with the weight multiplied by
 *   sin^{d-3}(phi) at the nodes:
 *     V = Omega_{d-2}/(2pi)^d sum_i sum_j sum_l w_i q_i^{d-1} d_tR(q_i^2)
 *           G(q_i^2)^2 mu_j G(s1_ij) nu_l G(s2_ijl).
 *
 *   Momentum-dependent two-point flow (one loop, constant vertices): the
 *   two-point function Gamma2_k(p) = p^2 + Sigma_k(p) of a scalar with
 *   momentum-independent three- and four-point couplings lam3, lam4 flows by
 *   the second field derivative of the Wetterich equation,
 *     d_t Sigma(p) = lam3^2 J(p) - (lam4/2) T,
 *     J(p) = int d^dq/(2pi)^d d_tR(q^2) G(q^2)^2 G(|q+p|^2),
 *     T    = int d^dq/(2pi)^d d_tR(q^2) G(q^2)^2,
 *     G(s) = 1/(s + R_k(s) + Sigma(sqrt s)).
 *   Sigma lives on the nodes s_a = a s_max/(n_s - 1); at each RG time the
 *   table g[a] = 1/(s_a + R_k(s_a) + Sigma_a) is the propagator of the
 *   tabulated variant above (piecewise linear, constant beyond s_max), J is
 *   that variant at p_a = sqrt(s_a) and T its radial part with C_d:
 *     T = C_d sum_i w_i q_i^{d-1} d_tR(q_i^2) G(q_i^2)^2,
 *   with the quadrature at scale k = Lambda e^t and q_max = kappa k.  A
 *   non-positive table denominator ends the flow (domain).  Time stepping:
 *   classical fourth-order Runge-Kutta from t = 0 to t_end with n_steps equal
 *   steps h = t_end/n_steps, t_n = n h; a flow whose right-hand side meets the
 *   domain boundary at any stage of step n keeps its state at t_n and
 *   reports t_n as the time reached.
 *
 *   Finite-volume LPA (O(N), field amplitude sigma, u = dU/dsigma): with
 *   rho = sigma^2/2 the LPA flow below becomes the conservation law
 *     d_t u = d_sigma Q,  Q = 1/2 F_1(d_sigma u) + (N-1)/2 F_1(u/sigma).
 *   Cells i = 0..n-1 of width ds = sigma_max/n hold averages u_i; interface
 *   j = 0..n sits at sigma_j = j ds between cells j-1 and j; ghost cells
 *   u_{-1} = -u_0, u_{-2} = -u_1 (u odd in sigma) and u_n = 2 u_{n-1} - u_{n-2},
 *   u_{n+1} = 2 u_n - u_{n-1} (linear extrapolation).  Piecewise-linear
 *   reconstruction with minmod slopes, s_i = minmod(u_i - u_{i-1}, u_{i+1} - u_i)
 *   (minmod(a, b) = 0 if ab <= 0, else the one of smaller modulus), gives the
 *   states u-_j = u_{j-1} + s_{j-1}/2 and u+_j = u_j - s_j/2 at interface j.
 *   Interface fluxes:
 *     j = 0:  Q_0 = N/2 F_1(2 u_0/ds)  (sigma = 0: d_sigma u = u/sigma there),
 *     j >= 1: Q_j = 1/2 F_1((u_j - u_{j-1})/ds)
 *                   + 1/2 (f(u-_j) + f(u+_j)) - 1/2 a_j (u+_j - u-_j),
 *             f(u) = (N-1)/2 F_1(u/sigma_j)  (local Lax-Friedrichs flux),
 *             a_j = max |f'| over u-_j, u+_j,  f'(u) = -(N-1)/2 F_2(u/sigma_j)/sigma_j
 *   (the semi-discrete central scheme of Kurganov and Tadmor);
 *   d_t u_i = (Q_{i+1} - Q_i)/ds.  F_n at scale k = Lambda e^t with the radial
 *   rule on [0, kappa k].  A step estimate per flow: 1/max_j (2 D_j/ds^2 +
 *   a_j/ds) with D_0 = N/2 F_2(2 u_0/ds), D_j = 1/2 F_2((u_j - u_{j-1})/ds).
 *   Time stepping: three-stage strong-stability-preserving Runge-Kutta
 *   (Shu-Osher) in n_steps equal steps h = t_end/n_steps, stage times
 *   t_n, t_n + h, t_n + h/2; a flow whose right-hand side meets m^2 + k^2 <= 0
 *   stops at t_n with its state kept.
 *
 *   Threshold functions (radial only, LPA):
 *     F_n(m^2) = C_d sum_i w_i q_i^{d-1} d_tR(q_i^2) G(q_i^2)^n,
 *     C_d = Omega_d/(2pi)^d.
 *   LPA O(N) flow of the effective potential U(rho), rho = phi^2/2:
 *     d_t U = 1/2 [ F_1(U' + 2 rho U'') + (N-1) F_1(U') ],
 *   with U', U'' from second-order finite differences on a uniform grid.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

#define OR_REG_EXP 0
#define OR_REG_LITIM 1

#define OR_OK 0
#define OR_E_INVAL (-1)
#define OR_E_DOMAIN (-2)

/* ---------------------------------------------------------------- rules -- */

/* Gauss-Legendre rule on [-1,1], nodes ascending: Newton on P_n(x) with P_n
 * and P_n' from the three-term recurrence
 *   (j+1) P_{j+1} = (2j+1) x P_j - j P_{j-1},  P_n' = n (x P_n - P_{n-1})/(x^2-1),
 * weights 2/((1-x^2) P_n'(x)^2).  The recurrence runs in long double. */
int oracle_gauss_legendre(int n, double *x, double *w) {
  if (n < 1 || !x || !w) return OR_E_INVAL;
  const long double pi = 3.14159265358979323846264338327950288L;
  for (int i = 0; i < (n + 1) / 2; ++i) {
    long double z = cosl(pi * (i + 0.75L) / (n + 0.5L));
    long double dp = 1.0L;
    for (int it = 0; it < 100; ++it) {
      long double p0 = 1.0L, p1 = z;
      for (int j = 1; j < n; ++j) {
        long double p2 = ((2.0L * j + 1.0L) * z * p1 - j * p0) / (j + 1.0L);
        p0 = p1;
        p1 = p2;
      }
      if (n == 1) { p0 = 1.0L; p1 = z; }
      dp = n * (z * p1 - p0) / (z * z - 1.0L);
      long double dz = p1 / dp;
      z -= dz;
      if (fabsl(dz) < 1e-19L) break;
    }
    /* final derivative at the converged node */
    {
      long double p0 = 1.0L, p1 = z;
      for (int j = 1; j < n; ++j) {
        long double p2 = ((2.0L * j + 1.0L) * z * p1 - j * p0) / (j + 1.0L);
        p0 = p1;
        p1 = p2;
      }
      dp = n * (z * p1 - p0) / (z * z - 1.0L);
    }
    long double wt = 2.0L / ((1.0L - z * z) * dp * dp);
    x[n - 1 - i] = (double)z;
    x[i] = (double)(-z);
    w[i] = (double)wt;
    w[n - 1 - i] = (double)wt;
  }
  if (n % 2 == 1) x[n / 2] = 0.0;
  return OR_OK;
}

/* area of the unit sphere S^{n-1} in R^n */
static double omega(int n) {
  return 2.0 * pow(M_PI, 0.5 * n) / tgamma(0.5 * n);
}

/* angular measure prefactor P_d = Omega_{d-1}/(2pi)^d */
double oracle_Pd(int d) { return omega(d - 1) / pow(2.0 * M_PI, d); }

/* radial-only prefactor C_d = Omega_d/(2pi)^d */
double oracle_Cd(int d) { return omega(d) / pow(2.0 * M_PI, d); }

/* (1-x^2)^{(d-3)/2} */
static double angular_factor(int d, double x) {
  double z = (1.0 - x) * (1.0 + x);
  int e = d - 3;
  double f = 1.0;
  for (int i = 0; i < e / 2; ++i) f *= z;
  if (e % 2 == 1) f *= sqrt(z);
  return f;
}

static double ipow(double q, int e) {
  double r = 1.0;
  for (int i = 0; i < e; ++i) r *= q;
  return r;
}

/* ------------------------------------------------------------ regulators -- */

/* h(y) = beta(-y) - 1 = y/(1 - e^{-y}) - 1 for the exponential regulator */
static double h_exp(double y) {
  if (y < 0.1) {
    double y2 = y * y;
    return y / 2.0 + y2 / 12.0 - y2 * y2 / 720.0 + y2 * y2 * y2 / 30240.0 -
           y2 * y2 * y2 * y2 / 1209600.0 + y2 * y2 * y2 * y2 * y2 / 47900160.0;
  }
  return y / (-expm1(-y)) - 1.0;
}

/* beta(z) = z/expm1(z), beta(0) = 1 */
static double beta(double z) {
  if (z == 0.0) return 1.0;
  return z / expm1(z);
}

/* propagator denominator s + R(s) + m^2 in the stable form */
static double denom(int reg, double k2, double s, double delta) {
  if (reg == OR_REG_EXP) return k2 * h_exp(s / k2) + delta;
  return fmax(s - k2, 0.0) + delta;
}

/* d_t R(s) = k dR/dk */
static double dtR(int reg, double k2, double s) {
  if (reg == OR_REG_EXP) {
    double y = s / k2;
    return 2.0 * k2 * beta(y) * beta(-y);
  }
  return (s < k2) ? 2.0 * k2 : 0.0;
}

/* radial rule mapped to [0, Q] */
static int radial_rule(int reg, double k, double q_max, int n_r, double *q, double *w) {
  int rc = oracle_gauss_legendre(n_r, q, w);
  if (rc) return rc;
  double Q = (reg == OR_REG_LITIM) ? fmin(q_max, k) : q_max;
  for (int i = 0; i < n_r; ++i) {
    q[i] = 0.5 * Q * (1.0 + q[i]);
    w[i] = 0.5 * Q * w[i];
  }
  return OR_OK;
}

static int check_common(int d, int reg, double k, double q_max, int n_r) {
  if (d < 2 || d > 10) return OR_E_INVAL;
  if (reg != OR_REG_EXP && reg != OR_REG_LITIM) return OR_E_INVAL;
  if (!(k > 0.0) || !(q_max > 0.0) || n_r < 1) return OR_E_INVAL;
  return OR_OK;
}

/* ---------------------------------------------------------- integrals -- */

/* I(p_e, m2_e) for n_pts independent external points. */
int oracle_integrate(int d, int reg, double k, double q_max, int n_r, int n_a, long n_pts,
                     const double *p, const double *m2, double *out, int n_threads) {
  if (check_common(d, reg, k, q_max, n_r) || d < 3 || n_a < 1 || n_pts < 0) return OR_E_INVAL;
  if (n_pts > 0 && (!p || !m2 || !out)) return OR_E_INVAL;
  double *q = malloc(sizeof(double) * n_r), *w = malloc(sizeof(double) * n_r);
  double *x = malloc(sizeof(double) * n_a), *v = malloc(sizeof(double) * n_a);
  double *mu = malloc(sizeof(double) * n_a);
  radial_rule(reg, k, q_max, n_r, q, w);
  oracle_gauss_legendre(n_a, x, v);
  for (int j = 0; j < n_a; ++j) mu[j] = v[j] * angular_factor(d, x[j]);
  const double k2 = k * k;
  const double Pd = oracle_Pd(d);
  int domain = 0;
  if (n_threads < 1) n_threads = 1;
#pragma omp parallel for schedule(dynamic, 8) num_threads(n_threads) reduction(| : domain)
  for (long e = 0; e < n_pts; ++e) {
    double delta = m2[e] + k2;
    if (!(delta > 0.0) || !(p[e] >= 0.0)) {
      out[e] = NAN;
      domain |= 1;
      continue;
    }
    long double acc = 0.0L;
    for (int i = 0; i < n_r; ++i) {
      double qi = q[i];
      double Gq = 1.0 / denom(reg, k2, qi * qi, delta);
      double A = w[i] * ipow(qi, d - 1) * dtR(reg, k2, qi * qi) * Gq * Gq;
      for (int j = 0; j < n_a; ++j) {
        double s = (qi - p[e]) * (qi - p[e]) + 2.0 * qi * p[e] * (1.0 + x[j]);
        double G = 1.0 / denom(reg, k2, s, delta);
        acc += (long double)(A * mu[j] * G);
      }
    }
    out[e] = Pd * (double)acc;
  }
  free(q); free(w); free(x); free(v); free(mu);
  return domain ? OR_E_DOMAIN : OR_OK;
}

/* piecewise-linear interpolation of one table row at s (constant beyond s_max) */
static double interp_row(const double *g, long n_s, double s_max, double s) {
  double h = s_max / (double)(n_s - 1);
  double t = s / h;
  if (t >= (double)(n_s - 1)) return g[n_s - 1];
  if (t < 0.0) t = 0.0;
  long k = (long)floor(t);
  double f = t - (double)k;
  return (1.0 - f) * g[k] + f * g[k + 1];
}

/* Tabulated variant: out[a * n_rows + r] = I(p_a, row r). */
int oracle_integrate_tab(int d, int reg, double k, double q_max, int n_r, int n_a, long n_rows,
                         long n_s, double s_max, const double *G, long n_p, const double *p,
                         double *out, int n_threads) {
  if (check_common(d, reg, k, q_max, n_r) || d < 3 || n_a < 1 || n_p < 0 || n_rows < 0)
    return OR_E_INVAL;
  if (n_s < 2 || !(s_max > 0.0)) return OR_E_INVAL;
  if (n_p > 0 && n_rows > 0 && (!p || !G || !out)) return OR_E_INVAL;
  double *q = malloc(sizeof(double) * n_r), *w = malloc(sizeof(double) * n_r);
  double *x = malloc(sizeof(double) * n_a), *v = malloc(sizeof(double) * n_a);
  double *mu = malloc(sizeof(double) * n_a);
  radial_rule(reg, k, q_max, n_r, q, w);
  oracle_gauss_legendre(n_a, x, v);
  for (int j = 0; j < n_a; ++j) mu[j] = v[j] * angular_factor(d, x[j]);
  const double k2 = k * k;
  const double Pd = oracle_Pd(d);
  int domain = 0;
  if (n_threads < 1) n_threads = 1;
#pragma omp parallel for collapse(2) schedule(dynamic, 8) num_threads(n_threads) reduction(| : domain)
  for (long a = 0; a < n_p; ++a) {
    for (long r = 0; r < n_rows; ++r) {
      const double *g = G + r * n_s;
      if (!(p[a] >= 0.0)) {
        out[a * n_rows + r] = NAN;
        domain |= 1;
        continue;
      }
      long double acc = 0.0L;
      for (int i = 0; i < n_r; ++i) {
        double qi = q[i];
        double Gq = interp_row(g, n_s, s_max, qi * qi);
        double A = w[i] * ipow(qi, d - 1) * dtR(reg, k2, qi * qi) * Gq * Gq;
        for (int j = 0; j < n_a; ++j) {
          double s = (qi - p[a]) * (qi - p[a]) + 2.0 * qi * p[a] * (1.0 + x[j]);
          acc += (long double)(A * mu[j] * interp_row(g, n_s, s_max, s));
        }
      }
      out[a * n_rows + r] = Pd * (double)acc;
    }
  }
  free(q); free(w); free(x); free(v); free(mu);
  return domain ? OR_E_DOMAIN : OR_OK;
}

/* Sensitivity of a tabulated result to the evaluation coordinate (test
 * infrastructure: the tolerance of GPU-vs-oracle comparisons on rough rows).
 *
 * Two evaluations of the tabulated diagram on independent Gauss-Legendre
 * rules (nodes equal to about an ulp) and with different roundings in
 * forming t = s/h see coordinates that differ by |dt| <= 16 u ((q + p)^2/h + 1)
 * (u = 2^-53: the node differences |dq| <= 2u q and |d(1 + x)| <= 3u, three
 * roundings in s and two in t, with room to spare).  The piecewise-linear
 * G_r then moves by at most sigma(t) |dt| + 4u max(g_k, g_k+1), sigma(t) the
 * largest |g_{j+1} - g_j| over the intervals j = k-1, k, k+1 (k = floor(t),
 * intervals clamped to the table; 0 once t lies beyond the last node by more
 * than |dt|).  Every term c_i mu_j G(q_i^2)^2 G(s_ij) is positive, so the
 * relative deviation of a result is at most
 *   B = sum_ij c_i mu_j [G_q^2 dG_s + 2 G_q G_s dG_q] / sum_ij c_i mu_j G_q^2 G_s
 * plus the accumulation of roundings over the sum (taken as 1e-13).
 * out[a * n_rows + r] = B for the result of oracle_integrate_tab at (a, r). */
static double tab_dG(const double *g, long n_s, double h, double s, double qp2) {
  const double u = 1.1102230246251565e-16;
  const double t = s / h;
  const double dt = 16.0 * u * (qp2 / h + 1.0);
  const double last = (double)(n_s - 1);
  double tc = t < last ? t : last;
  long k = (long)floor(tc);
  if (k > n_s - 2) k = n_s - 2;
  double sig = 0.0;
  if (t <= last + dt) {
    for (long j = k - 1; j <= k + 1; ++j) {
      if (j < 0 || j > n_s - 2) continue;
      double dg = fabs(g[j + 1] - g[j]);
      if (dg > sig) sig = dg;
    }
  }
  double gm = g[k] > g[k + 1] ? g[k] : g[k + 1];
  return sig * dt + 4.0 * u * gm;
}

int oracle_integrate_tab_bound(int d, int reg, double k, double q_max, int n_r, int n_a,
                               long n_rows, long n_s, double s_max, const double *G, long n_p,
                               const double *p, double *out, int n_threads) {
  if (check_common(d, reg, k, q_max, n_r) || d < 3 || n_a < 1 || n_p < 0 || n_rows < 0)
    return OR_E_INVAL;
  if (n_s < 2 || !(s_max > 0.0)) return OR_E_INVAL;
  if (n_p > 0 && n_rows > 0 && (!p || !G || !out)) return OR_E_INVAL;
  double *q = malloc(sizeof(double) * n_r), *w = malloc(sizeof(double) * n_r);
  double *x = malloc(sizeof(double) * n_a), *v = malloc(sizeof(double) * n_a);
  double *mu = malloc(sizeof(double) * n_a);
  radial_rule(reg, k, q_max, n_r, q, w);
  oracle_gauss_legendre(n_a, x, v);
  for (int j = 0; j < n_a; ++j) mu[j] = v[j] * angular_factor(d, x[j]);
  const double k2 = k * k;
  const double h = s_max / (double)(n_s - 1);
  if (n_threads < 1) n_threads = 1;
#pragma omp parallel for collapse(2) schedule(dynamic, 8) num_threads(n_threads)
  for (long a = 0; a < n_p; ++a) {
    for (long r = 0; r < n_rows; ++r) {
      const double *g = G + r * n_s;
      if (!(p[a] >= 0.0)) {
        out[a * n_rows + r] = NAN;
        continue;
      }
      long double num = 0.0L, den = 0.0L;
      for (int i = 0; i < n_r; ++i) {
        double qi = q[i];
        double Gq = interp_row(g, n_s, s_max, qi * qi);
        double dGq = tab_dG(g, n_s, h, qi * qi, qi * qi);
        double c = w[i] * ipow(qi, d - 1) * dtR(reg, k2, qi * qi);
        double qp = qi + p[a];
        for (int j = 0; j < n_a; ++j) {
          double s = (qi - p[a]) * (qi - p[a]) + 2.0 * qi * p[a] * (1.0 + x[j]);
          double Gs = interp_row(g, n_s, s_max, s);
          double dGs = tab_dG(g, n_s, h, s, qp * qp);
          num += (long double)(c * mu[j] * (Gq * Gq * dGs + 2.0 * Gq * Gs * dGq));
          den += (long double)(c * mu[j] * Gq * Gq * Gs);
        }
      }
      out[a * n_rows + r] = (double)(num / den) + 1e-13;
    }
  }
  free(q); free(w); free(x); free(v); free(mu);
  return OR_OK;
}

/* F_n(m2_e), radial only */
int oracle_threshold(int d, int reg, double k, double q_max, int n_r, int n, long n_pts,
                     const double *m2, double *out) {
  if (check_common(d, reg, k, q_max, n_r) || n < 1 || n_pts < 0) return OR_E_INVAL;
  if (n_pts > 0 && (!m2 || !out)) return OR_E_INVAL;
  double *q = malloc(sizeof(double) * n_r), *w = malloc(sizeof(double) * n_r);
  radial_rule(reg, k, q_max, n_r, q, w);
  const double k2 = k * k, Cd = oracle_Cd(d);
  int domain = 0;
  for (long e = 0; e < n_pts; ++e) {
    double delta = m2[e] + k2;
    if (!(delta > 0.0)) {
      out[e] = NAN;
      domain = 1;
      continue;
    }
    long double acc = 0.0L;
    for (int i = 0; i < n_r; ++i) {
      double G = 1.0 / denom(reg, k2, q[i] * q[i], delta);
      acc += (long double)(w[i] * ipow(q[i], d - 1) * dtR(reg, k2, q[i] * q[i]) * ipow(G, n));
    }
    out[e] = Cd * (double)acc;
  }
  free(q); free(w);
  return domain ? OR_E_DOMAIN : OR_OK;
}

/* ------------------------------------------------------------------ LPA -- */

/* Finite differences on the uniform grid rho_j = j*dr, j = 0..n-1 (n >= 4):
 *   interior  U'  = (U[j+1] - U[j-1]) / (2 dr)
 *             U'' = ((U[j+1] - 2U[j]) + U[j-1]) / dr^2
 *   rho = 0   U'  = ((-3U[0] + 4U[1]) - U[2]) / (2 dr)
 *             U'' = (((2U[0] - 5U[1]) + 4U[2]) - U[3]) / dr^2
 *   rho_max   U'  = ((3U[n-1] - 4U[n-2]) + U[n-3]) / (2 dr)
 *             U'' = (((2U[n-1] - 5U[n-2]) + 4U[n-3]) - U[n-4]) / dr^2
 * and the coefficient of U[j+o] in U' (c1) and U'' (c2), o = -3..3, for the
 * Jacobian.  Grouping as written; no fused multiply-add. */
static void fd_stencil(const double *U, long n, long j, double dr, double *d1, double *d2,
                       double c1[7], double c2[7]) {
  for (int o = 0; o < 7; ++o) c1[o] = c2[o] = 0.0;
  const double i2 = 1.0 / (2.0 * dr), i1 = 1.0 / (dr * dr);
  if (j == 0) {
    *d1 = ((-3.0 * U[0] + 4.0 * U[1]) - U[2]) / (2.0 * dr);
    *d2 = (((2.0 * U[0] - 5.0 * U[1]) + 4.0 * U[2]) - U[3]) / (dr * dr);
    c1[3] = -3.0 * i2; c1[4] = 4.0 * i2; c1[5] = -1.0 * i2;
    c2[3] = 2.0 * i1; c2[4] = -5.0 * i1; c2[5] = 4.0 * i1; c2[6] = -1.0 * i1;
  } else if (j == n - 1) {
    *d1 = ((3.0 * U[n - 1] - 4.0 * U[n - 2]) + U[n - 3]) / (2.0 * dr);
    *d2 = (((2.0 * U[n - 1] - 5.0 * U[n - 2]) + 4.0 * U[n - 3]) - U[n - 4]) / (dr * dr);
    c1[3] = 3.0 * i2; c1[2] = -4.0 * i2; c1[1] = 1.0 * i2;
    c2[3] = 2.0 * i1; c2[2] = -5.0 * i1; c2[1] = 4.0 * i1; c2[0] = -1.0 * i1;
  } else {
    *d1 = (U[j + 1] - U[j - 1]) / (2.0 * dr);
    *d2 = ((U[j + 1] - 2.0 * U[j]) + U[j - 1]) / (dr * dr);
    c1[4] = i2; c1[2] = -i2;
    c2[4] = i1; c2[3] = -2.0 * i1; c2[2] = i1;
  }
}

/* dU/dt on the grid and, if jac != NULL, the Jacobian in 7 bands:
 * jac[(o+3)*n + j] = d(dUdt_j)/dU_{j+o}, o = -3..3, zero outside the grid.
 * The RG scale k is passed in (k = Lambda e^t is formed by the caller). */
int oracle_lpa_rhs(int d, int N, int reg, int n_r, double q_max_over_k, double k, long n,
                   double rho_max, const double *U, double *dUdt, double *jac) {
  if (check_common(d, reg, k, q_max_over_k * k, n_r) || N < 1 || n < 4 || !(rho_max > 0.0))
    return OR_E_INVAL;
  if (!U || !dUdt) return OR_E_INVAL;
  const double dr = rho_max / (double)(n - 1);
  int domain = 0;
  for (long j = 0; j < n; ++j) {
    double d1, d2, c1[7], c2[7];
    fd_stencil(U, n, j, dr, &d1, &d2, c1, c2);
    double rho = (double)j * dr;
    double m2s = d1 + (2.0 * rho) * d2;
    double m2p = d1;
    /* N = 1 has no Goldstone modes: the pion mass is neither used nor checked */
    double ms[2] = {m2s, m2p}, F1[2] = {0.0, 0.0}, F2[2] = {0.0, 0.0};
    long nm = (N > 1) ? 2 : 1;
    int r1 = oracle_threshold(d, reg, k, q_max_over_k * k, n_r, 1, nm, ms, F1);
    int r2 = oracle_threshold(d, reg, k, q_max_over_k * k, n_r, 2, nm, ms, F2);
    if (r1 == OR_E_DOMAIN || r2 == OR_E_DOMAIN) domain = 1;
    dUdt[j] = 0.5 * (F1[0] + (double)(N - 1) * F1[1]);
    if (jac) {
      for (int o = 0; o < 7; ++o) {
        double dms = c1[o] + (2.0 * rho) * c2[o];
        double dmp = c1[o];
        double v = -0.5 * (F2[0] * dms + (double)(N - 1) * F2[1] * dmp);
        long col = j + (o - 3);
        jac[(long)o * n + j] = (col >= 0 && col < n) ? v : 0.0;
      }
    }
  }
  return domain ? OR_E_DOMAIN : OR_OK;
}

/* ------------------------------------------- momentum-dependent flow -- */

/* Right-hand side of the two-point flow for n_rows flows at RG time t:
 * dSdt[r * n_s + a] = lam3[r]^2 J_r(p_a) - lam4[r]/2 T_r.  A flow with a
 * non-positive table denominator gets dead[r] = 1 and NaN in its row. */
int oracle_pflow_rhs(int d, int reg, double Lambda, double kappa, int n_r, int n_a, long n_rows,
                     long n_s, double s_max, const double *lam3, const double *lam4, double t,
                     const double *Sigma, double *dSdt, int *dead, int n_threads) {
  if (!(Lambda > 0.0) || !(kappa > 0.0) || n_s < 2 || !(s_max > 0.0) || n_rows < 0) return OR_E_INVAL;
  const double k = Lambda * exp(t), k2 = k * k;
  const double q_max = kappa * k;
  if (check_common(d, reg, k, q_max, n_r) || d < 3 || n_a < 1) return OR_E_INVAL;
  double *g = malloc(sizeof(double) * n_rows * n_s);
  double *p = malloc(sizeof(double) * n_s);
  double *J = malloc(sizeof(double) * n_s * (n_rows > 0 ? n_rows : 1));
  double *q = malloc(sizeof(double) * n_r), *w = malloc(sizeof(double) * n_r);
  const double h = s_max / (double)(n_s - 1);
  for (long a = 0; a < n_s; ++a) p[a] = sqrt((double)a * h);
  for (long r = 0; r < n_rows; ++r) {
    dead[r] = 0;
    for (long a = 0; a < n_s; ++a) {
      double s = (double)a * h;
      double den = denom(reg, k2, s, k2 + Sigma[r * n_s + a]);
      if (!(den > 0.0)) dead[r] = 1;
      g[r * n_s + a] = (den > 0.0) ? 1.0 / den : 0.0;
    }
  }
  int rc = oracle_integrate_tab(d, reg, k, q_max, n_r, n_a, n_rows, n_s, s_max, g, n_s, p, J,
                                n_threads);
  radial_rule(reg, k, q_max, n_r, q, w);
  const double Cd = oracle_Cd(d);
  for (long r = 0; r < n_rows && rc == OR_OK; ++r) {
    long double T = 0.0L;
    for (int i = 0; i < n_r; ++i) {
      double Gq = interp_row(g + r * n_s, n_s, s_max, q[i] * q[i]);
      T += (long double)(w[i] * ipow(q[i], d - 1) * dtR(reg, k2, q[i] * q[i]) * Gq * Gq);
    }
    const double Tr = Cd * (double)T;
    for (long a = 0; a < n_s; ++a)
      dSdt[r * n_s + a] = dead[r] ? NAN : lam3[r] * lam3[r] * J[a * n_rows + r] - 0.5 * lam4[r] * Tr;
  }
  free(g); free(p); free(J); free(q); free(w);
  if (rc != OR_OK) return rc;
  for (long r = 0; r < n_rows; ++r)
    if (dead[r]) return OR_E_DOMAIN;
  return OR_OK;
}

/* Classical RK4 from t = 0 to t_end in n_steps equal steps for every flow;
 * Sigma is updated in place, t_reached[r] = t_end or the start of the step
 * whose right-hand side met the domain boundary. */
int oracle_pflow_solve(int d, int reg, double Lambda, double kappa, int n_r, int n_a, long n_rows,
                       long n_s, double s_max, const double *lam3, const double *lam4,
                       double t_end, long n_steps, double *Sigma, double *t_reached, int n_threads) {
  if (!(t_end <= 0.0) || n_steps < 1 || n_rows < 0) return OR_E_INVAL;
  const long n = n_rows * n_s;
  double *y = malloc(sizeof(double) * n), *acc = malloc(sizeof(double) * n);
  double *kk = malloc(sizeof(double) * n);
  int *alive = malloc(sizeof(int) * (n_rows > 0 ? n_rows : 1));
  int *dead = malloc(sizeof(int) * (n_rows > 0 ? n_rows : 1));
  const double h = t_end / (double)n_steps;
  const double cs[4] = {0.0, 0.5, 0.5, 1.0};  /* stage times */
  const double bs[4] = {1.0, 2.0, 2.0, 1.0};  /* stage weights (times 1/6) */
  int rc = OR_OK;
  for (long r = 0; r < n_rows; ++r) {
    alive[r] = 1;
    t_reached[r] = t_end;
  }
  for (long step = 0; step < n_steps && rc != OR_E_INVAL; ++step) {
    const double tn = (double)step * h;
    for (long e = 0; e < n; ++e) {
      y[e] = Sigma[e];
      acc[e] = 0.0;
    }
    for (int st = 0; st < 4; ++st) {
      rc = oracle_pflow_rhs(d, reg, Lambda, kappa, n_r, n_a, n_rows, n_s, s_max, lam3, lam4,
                            tn + cs[st] * h, y, kk, dead, n_threads);
      if (rc == OR_E_INVAL) break;
      for (long r = 0; r < n_rows; ++r) {
        if (!alive[r]) continue;
        if (dead[r]) {
          alive[r] = 0;
          t_reached[r] = tn;
          continue;
        }
        for (long a = 0; a < n_s; ++a) {
          const long e = r * n_s + a;
          acc[e] += bs[st] * kk[e];
          if (st < 3) y[e] = Sigma[e] + cs[st + 1] * h * kk[e];
        }
      }
    }
    for (long r = 0; r < n_rows; ++r)
      if (alive[r])
        for (long a = 0; a < n_s; ++a) Sigma[r * n_s + a] += (h / 6.0) * acc[r * n_s + a];
  }
  free(y); free(acc); free(kk); free(alive); free(dead);
  return rc == OR_E_INVAL ? OR_E_INVAL : OR_OK;
}

/* -------------------------------------------------- vertex diagram -- */

/* V(p1_e, p2_e, th_e, m2_e) for n_pts points; c12[e] = cos th_e. */
int oracle_integrate_vertex(int d, int reg, double k, double q_max, int n_r, int n_a, int n_phi,
                            long n_pts, const double *p1, const double *p2, const double *c12,
                            const double *m2, double *out, int n_threads) {
  if (check_common(d, reg, k, q_max, n_r) || d < 3 || n_a < 1 || n_phi < 1 || n_pts < 0)
    return OR_E_INVAL;
  if (n_pts > 0 && (!p1 || !p2 || !c12 || !m2 || !out)) return OR_E_INVAL;
  double *q = malloc(sizeof(double) * n_r), *w = malloc(sizeof(double) * n_r);
  double *x = malloc(sizeof(double) * n_a), *v = malloc(sizeof(double) * n_a);
  double *mu = malloc(sizeof(double) * n_a);
  double *ph = malloc(sizeof(double) * n_phi), *pw = malloc(sizeof(double) * n_phi);
  double *nu = malloc(sizeof(double) * n_phi), *cph = malloc(sizeof(double) * n_phi);
  radial_rule(reg, k, q_max, n_r, q, w);
  oracle_gauss_legendre(n_a, x, v);
  for (int j = 0; j < n_a; ++j) mu[j] = v[j] * angular_factor(d, x[j]);
  oracle_gauss_legendre(n_phi, ph, pw);
  for (int l = 0; l < n_phi; ++l) {
    double f = 0.5 * M_PI * (1.0 + ph[l]); /* phi on [0, pi] */
    cph[l] = cos(f);
    nu[l] = 0.5 * M_PI * pw[l] * ipow(sin(f), d - 3);
  }
  const double k2 = k * k;
  const double pref = omega(d - 2) / pow(2.0 * M_PI, d);
  int domain = 0;
  if (n_threads < 1) n_threads = 1;
#pragma omp parallel for schedule(dynamic, 4) num_threads(n_threads) reduction(| : domain)
  for (long e = 0; e < n_pts; ++e) {
    double delta = m2[e] + k2;
    if (!(delta > 0.0) || !(p1[e] >= 0.0) || !(p2[e] >= 0.0) || !(c12[e] >= -1.0 && c12[e] <= 1.0)) {
      out[e] = NAN;
      domain |= 1;
      continue;
    }
    const double ct = c12[e], st = sqrt((1.0 - ct) * (1.0 + ct));
    long double acc = 0.0L;
    for (int i = 0; i < n_r; ++i) {
      double qi = q[i];
      double Gq = 1.0 / denom(reg, k2, qi * qi, delta);
      double A = w[i] * ipow(qi, d - 1) * dtR(reg, k2, qi * qi) * Gq * Gq;
      for (int j = 0; j < n_a; ++j) {
        double s1 = qi * qi + p1[e] * p1[e] + 2.0 * qi * p1[e] * x[j];
        double G1 = 1.0 / denom(reg, k2, fmax(s1, 0.0), delta);
        double sx = sqrt((1.0 - x[j]) * (1.0 + x[j]));
        for (int l = 0; l < n_phi; ++l) {
          double s2 = qi * qi + p2[e] * p2[e] + 2.0 * qi * p2[e] * (x[j] * ct + sx * cph[l] * st);
          double G2 = 1.0 / denom(reg, k2, fmax(s2, 0.0), delta);
          acc += (long double)(A * mu[j] * G1 * nu[l] * G2);
        }
      }
    }
    out[e] = pref * (double)acc;
  }
  free(q); free(w); free(x); free(v); free(mu); free(ph); free(pw); free(nu); free(cph);
  return domain ? OR_E_DOMAIN : OR_OK;
}

/* ------------------------------------------------ finite-volume LPA -- */

static double minmod(double a, double b) {
  if (a * b <= 0.0) return 0.0;
  return fabs(a) < fabs(b) ? a : b;
}

/* F_1 and F_2 at m^2 (radial rule q, w at scale k); 0 on the domain
 * boundary m^2 + k^2 <= 0 (flagged). */
static void fv_F12(int d, int reg, double k2, int n_r, const double *q, const double *w,
                   double Cd, double m2, double *F1, double *F2, int *bad) {
  const double delta = m2 + k2;
  if (!(delta > 0.0)) {
    *bad = 1;
    *F1 = *F2 = 0.0;
    return;
  }
  long double a1 = 0.0L, a2 = 0.0L;
  for (int i = 0; i < n_r; ++i) {
    double G = 1.0 / denom(reg, k2, q[i] * q[i], delta);
    double c = w[i] * ipow(q[i], d - 1) * dtR(reg, k2, q[i] * q[i]);
    a1 += (long double)(c * G);
    a2 += (long double)(c * G * G);
  }
  *F1 = Cd * (double)a1;
  *F2 = Cd * (double)a2;
}

/* Right-hand side of n_rows flows (u[r * n + i]) at RG time t; dt_est[r]
 * (may be NULL) the step estimate, dead[r] = 1 where the domain is left. */
int oracle_fvlpa_rhs(int d, int N, int reg, int n_r, double Lambda, double kappa, long n_rows,
                     long n, double sigma_max, double t, const double *u, double *dudt,
                     double *dt_est, int *dead) {
  if (!(Lambda > 0.0) || !(kappa > 0.0) || n < 2 || !(sigma_max > 0.0) || N < 1 || n_rows < 0)
    return OR_E_INVAL;
  const double k = Lambda * exp(t), k2 = k * k;
  if (check_common(d, reg, k, kappa * k, n_r)) return OR_E_INVAL;
  double *q = malloc(sizeof(double) * n_r), *w = malloc(sizeof(double) * n_r);
  double *Q = malloc(sizeof(double) * (n + 1));
  double *g = malloc(sizeof(double) * (n + 4)); /* u_{-2} .. u_{n+1} at g[i + 2] */
  radial_rule(reg, k, kappa * k, n_r, q, w);
  const double Cd = oracle_Cd(d), ds = sigma_max / (double)n;
  int any = 0;
  for (long r = 0; r < n_rows; ++r) {
    const double *ur = u + r * n;
    for (long i = 0; i < n; ++i) g[i + 2] = ur[i];
    g[1] = -ur[0];
    g[0] = -ur[1];
    g[n + 2] = 2.0 * ur[n - 1] - ur[n - 2];
    g[n + 3] = 2.0 * g[n + 2] - ur[n - 1];
    int bad = 0;
    double lam = 0.0;
    for (long j = 0; j <= n; ++j) {
      double F1, F2;
      if (j == 0) {
        fv_F12(d, reg, k2, n_r, q, w, Cd, 2.0 * ur[0] / ds, &F1, &F2, &bad);
        Q[0] = 0.5 * (double)N * F1;
        double l = 2.0 * (0.5 * (double)N * F2) / (ds * ds);
        lam = fmax(lam, l);
        continue;
      }
      const double uL = g[j + 1], uR = g[j + 2]; /* cells j-1 and j */
      const double sj = (double)j * ds;
      fv_F12(d, reg, k2, n_r, q, w, Cd, (uR - uL) / ds, &F1, &F2, &bad);
      const double sL = minmod(uL - g[j], uR - uL), sR = minmod(uR - uL, g[j + 3] - uR);
      const double um = uL + 0.5 * sL, up = uR - 0.5 * sR;
      double Qj = 0.5 * F1;
      double l = 2.0 * (0.5 * F2) / (ds * ds);
      if (N > 1) {
        double F1L, F2L, F1R, F2R;
        fv_F12(d, reg, k2, n_r, q, w, Cd, um / sj, &F1L, &F2L, &bad);
        fv_F12(d, reg, k2, n_r, q, w, Cd, up / sj, &F1R, &F2R, &bad);
        const double c = 0.5 * (double)(N - 1);
        const double a = fmax(c * F2L / sj, c * F2R / sj);
        Qj += 0.5 * (c * F1L + c * F1R) - 0.5 * a * (up - um);
        l += a / ds;
      }
      Q[j] = Qj;
      lam = fmax(lam, l);
    }
    dead[r] = bad;
    any |= bad;
    for (long i = 0; i < n; ++i) dudt[r * n + i] = bad ? NAN : (Q[i + 1] - Q[i]) / ds;
    if (dt_est) dt_est[r] = bad ? NAN : 1.0 / lam;
  }
  free(q); free(w); free(Q); free(g);
  return any ? OR_E_DOMAIN : OR_OK;
}

/* Three-stage SSP Runge-Kutta from t = 0 to t_end in n_steps equal steps;
 * u updated in place, t_reached[r] = t_end or the start of the step whose
 * right-hand side left the domain. */
int oracle_fvlpa_solve(int d, int N, int reg, int n_r, double Lambda, double kappa, long n_rows,
                       long n, double sigma_max, double t_end, long n_steps, double *u,
                       double *t_reached) {
  if (!(t_end <= 0.0) || n_steps < 1 || n_rows < 0) return OR_E_INVAL;
  const long m = n_rows * n;
  double *us = malloc(sizeof(double) * (m > 0 ? m : 1)), *L = malloc(sizeof(double) * (m > 0 ? m : 1));
  int *alive = malloc(sizeof(int) * (n_rows > 0 ? n_rows : 1));
  int *dead = malloc(sizeof(int) * (n_rows > 0 ? n_rows : 1));
  const double h = t_end / (double)n_steps;
  const double cs[3] = {0.0, 1.0, 0.5};
  int rc = OR_OK;
  for (long r = 0; r < n_rows; ++r) {
    alive[r] = 1;
    t_reached[r] = t_end;
  }
  for (long step = 0; step < n_steps && rc != OR_E_INVAL; ++step) {
    const double tn = (double)step * h;
    for (int st = 0; st < 3; ++st) {
      const double *state = (st == 0) ? u : us;
      rc = oracle_fvlpa_rhs(d, N, reg, n_r, Lambda, kappa, n_rows, n, sigma_max, tn + cs[st] * h,
                            state, L, NULL, dead);
      if (rc == OR_E_INVAL) break;
      for (long r = 0; r < n_rows; ++r) {
        if (!alive[r]) continue;
        if (dead[r]) {
          alive[r] = 0;
          t_reached[r] = tn;
          continue;
        }
        for (long i = 0; i < n; ++i) {
          const long e = r * n + i;
          if (st == 0)
            us[e] = u[e] + h * L[e];
          else if (st == 1)
            us[e] = 0.75 * u[e] + 0.25 * (us[e] + h * L[e]);
          else
            us[e] = u[e] / 3.0 + (2.0 / 3.0) * (us[e] + h * L[e]);
        }
      }
    }
    for (long r = 0; r < n_rows; ++r)
      if (alive[r])
        for (long i = 0; i < n; ++i) u[r * n + i] = us[r * n + i];
  }
  free(us); free(L); free(alive); free(dead);
  return rc == OR_E_INVAL ? OR_E_INVAL : OR_OK;
}
