/* The oracle (test infrastructure) under AddressSanitizer and
 * UndefinedBehaviorSanitizer, built with gcc on the CPU: every entry point on
 * small inputs that span its edge cases (one node, ragged shapes, p = 0,
 * points at the domain edge, flows that stop at the pole), one thread each.
 * Only memory and undefined-behaviour errors are looked for here; the values
 * are pinned by the Python tests.  Exit status 0 and "oracle checks ok" mean
 * no sanitizer report and no unexpected status. */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>

int oracle_gauss_legendre(int n, double *x, double *w);
int oracle_integrate(int d, int reg, double k, double q_max, int n_r, int n_a, long n_pts,
                     const double *p, const double *m2, double *out, int n_threads);
int oracle_integrate_tab(int d, int reg, double k, double q_max, int n_r, int n_a, long n_rows,
                         long n_s, double s_max, const double *G, long n_p, const double *p,
                         double *out, int n_threads);
int oracle_integrate_tab_bound(int d, int reg, double k, double q_max, int n_r, int n_a,
                               long n_rows, long n_s, double s_max, const double *G, long n_p,
                               const double *p, double *out, int n_threads);
int oracle_threshold(int d, int reg, double k, double q_max, int n_r, int n, long n_pts,
                     const double *m2, double *out);
int oracle_lpa_rhs(int d, int N, int reg, int n_r, double q_max_over_k, double k, long n,
                   double rho_max, const double *U, double *dUdt, double *jac);
int oracle_pflow_rhs(int d, int reg, double Lambda, double kappa, int n_r, int n_a, long n_rows,
                     long n_s, double s_max, const double *lam3, const double *lam4, double t,
                     const double *Sigma, double *dSdt, int *dead, int n_threads);
int oracle_pflow_solve(int d, int reg, double Lambda, double kappa, int n_r, int n_a, long n_rows,
                       long n_s, double s_max, const double *lam3, const double *lam4,
                       double t_end, long n_steps, double *Sigma, double *t_reached,
                       int n_threads);
int oracle_integrate_vertex(int d, int reg, double k, double q_max, int n_r, int n_a, int n_phi,
                            long n_pts, const double *p1, const double *p2, const double *c12,
                            const double *m2, double *out, int n_threads);
int oracle_fvlpa_rhs(int d, int N, int reg, int n_r, double Lambda, double kappa, long n_rows,
                     long n, double sigma_max, double t, const double *u, double *dudt,
                     double *dt_est, int *dead);
int oracle_fvlpa_solve(int d, int N, int reg, int n_r, double Lambda, double kappa, long n_rows,
                       long n, double sigma_max, double t_end, long n_steps, double *u,
                       double *t_reached);

static int failures = 0;
#define EXPECT(c)                                                                 \
  do {                                                                            \
    if (!(c)) {                                                                   \
      fprintf(stderr, "unexpected at line %d: %s\n", __LINE__, #c);               \
      ++failures;                                                                 \
    }                                                                             \
  } while (0)

/* status OK, or domain (-2) where the inputs reach the pole on purpose */
#define OK_OR_DOMAIN(rc) EXPECT((rc) == 0 || (rc) == -2)

int main(void) {
  enum { NP = 7 };
  const double p[NP] = {0.0, 0.3, 1.0, 2.5, 7.0, 0.01, 4.0};
  const double m2[NP] = {0.1, -0.5, 2.0, -0.999, 0.0, 5.0, -1.2};
  const double m2ok[NP] = {0.1, -0.5, 2.0, -0.9, 0.0, 5.0, 1e-6};  /* all above -k^2 = -1 */
  const double p2[NP] = {0.2, 0.0, 3.0, 1.0, 0.5, 6.0, 2.0};
  const double c12[NP] = {1.0, -1.0, 0.0, 0.5, -0.3, 0.99, -0.7};
  double out[NP * 4];
  for (int n = 1; n <= 40; n += 13) {
    double *x = malloc(sizeof(double) * n), *w = malloc(sizeof(double) * n);
    EXPECT(oracle_gauss_legendre(n, x, w) == 0);
    free(x);
    free(w);
  }
  for (int reg = 0; reg < 2; ++reg)
    for (int d = 3; d <= 5; ++d) {
      OK_OR_DOMAIN(oracle_integrate(d, reg, 1.0, 6.0, 9, 5, NP, p, m2, out, 1));
      OK_OR_DOMAIN(oracle_integrate(d, reg, 0.5, 3.0, 1, 1, NP, p, m2, out, 1));
      OK_OR_DOMAIN(oracle_threshold(d, reg, 1.0, 6.0, 11, 2, NP, m2, out));
      OK_OR_DOMAIN(oracle_integrate_vertex(d, reg, 1.0, 6.0, 5, 3, 4, NP, p, p2, c12, m2, out, 1));
      /* one point past the pole (m2 = -1.2 at k = 1) made those report the
       * domain; in the domain everywhere they return OK */
      EXPECT(oracle_integrate(d, reg, 1.0, 6.0, 9, 5, NP, p, m2ok, out, 1) == 0);
      EXPECT(oracle_threshold(d, reg, 1.0, 6.0, 11, 2, NP, m2ok, out) == 0);
      EXPECT(oracle_integrate_vertex(d, reg, 1.0, 6.0, 5, 3, 4, NP, p, p2, c12, m2ok, out, 1) == 0);
    }
  /* tabulated rows: two rows of 17 nodes, momenta past the table's end */
  {
    const long n_s = 17, n_rows = 2;
    double G[34];
    for (long i = 0; i < n_rows * n_s; ++i) G[i] = 1.0 / (1.0 + 0.1 * (double)i);
    for (int reg = 0; reg < 2; ++reg) {
      OK_OR_DOMAIN(oracle_integrate_tab(3, reg, 0.9, 5.4, 6, 4, n_rows, n_s, 30.0, G, NP, p, out, 1));
      OK_OR_DOMAIN(oracle_integrate_tab_bound(3, reg, 0.9, 5.4, 6, 4, n_rows, n_s, 30.0, G, NP, p,
                                              out, 1));
      OK_OR_DOMAIN(oracle_integrate_tab(4, reg, 0.9, 5.4, 1, 1, 1, 2, 1.0, G, NP, p, out, 1));
    }
  }
  /* LPA right-hand side with the bands, smallest grid and a ragged one */
  for (int N = 1; N <= 4; N += 3)
    for (long n = 4; n <= 23; n += 19) {
      double *U = malloc(sizeof(double) * n), *dU = malloc(sizeof(double) * n);
      double *jac = malloc(sizeof(double) * 7 * n);
      for (long j = 0; j < n; ++j) U[j] = 0.5 * (j / (double)(n - 1) - 0.3) * (j / (double)(n - 1) - 0.3);
      OK_OR_DOMAIN(oracle_lpa_rhs(3, N, 0, 16, 6.0, 1.0, n, 1.0, U, dU, jac));
      OK_OR_DOMAIN(oracle_lpa_rhs(4, N, 1, 16, 6.0, 0.7, n, 1.0, U, dU, NULL));
      free(U);
      free(dU);
      free(jac);
    }
  /* momentum flow: right-hand side and a few RK4 steps */
  {
    const long n_rows = 3, n_s = 9;
    const double lam3[3] = {0.5, 1.0, 3.0}, lam4[3] = {0.2, 1.0, 0.0};
    double S[27], dS[27], tr[3];
    int dead[3];
    for (long i = 0; i < n_rows * n_s; ++i) S[i] = 0.01 * (double)(i % 5);
    OK_OR_DOMAIN(oracle_pflow_rhs(3, 0, 1.0, 6.0, 5, 3, n_rows, n_s, 20.0, lam3, lam4, -0.1, S, dS,
                                  dead, 1));
    OK_OR_DOMAIN(oracle_pflow_solve(3, 1, 1.0, 6.0, 5, 3, n_rows, n_s, 20.0, lam3, lam4, -0.3, 4, S,
                                    tr, 1));
  }
  /* finite-volume LPA: right-hand side, step estimate, a short solve in the
   * broken phase (some flows stop at the pole) */
  for (int N = 1; N <= 4; N += 3) {
    const long n_rows = 2, n = 6;
    double u[12], du[12], dt[2], tr[2];
    int dead[2];
    for (long i = 0; i < n_rows * n; ++i) u[i] = (i < n ? 1.0 : -0.8) * ((i % n) * 0.2 - 0.3);
    OK_OR_DOMAIN(oracle_fvlpa_rhs(3, N, 0, 12, 1.0, 6.0, n_rows, n, 1.5, 0.0, u, du, dt, dead));
    OK_OR_DOMAIN(oracle_fvlpa_solve(3, N, 1, 12, 1.0, 6.0, n_rows, n, 1.5, -0.2, 5, u, tr));
  }
  if (failures) {
    fprintf(stderr, "%d oracle checks failed\n", failures);
    return 1;
  }
  printf("oracle checks ok\n");
  return 0;
}
