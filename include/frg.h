/*
 * frg.h -- C ABI of the MI355X (gfx950) library for batched FRG flow-diagram
 * quadrature.
 *
 * The operations follow the standard functional-renormalisation-group
 * definitions (Wetterich equation, one-loop flow diagrams with a regulator
 * R_k); the paper's text fixes none of them, so each entry point states the
 * formula it computes.
 *
 * Conventions shared by every call
 *   - RG time t = ln(k/Lambda), d_t = k d/dk.
 *   - Regulators (y = s/k^2, s a squared momentum):
 *       FRG_REG_EXP   R_k(s) = s/(e^y - 1)
 *       FRG_REG_LITIM R_k(s) = (k^2 - s) theta(k^2 - s)
 *   - Propagator G(s) = 1/(s + R_k(s) + m^2); a point is in the domain iff
 *     delta = m^2 + k^2 > 0 (then every denominator is >= delta > 0).
 *   - Quadrature: radial Gauss-Legendre on [0, Q] with Q = q_max (exponential)
 *     or Q = min(q_max, k) (Litim, the support of d_tR); angular
 *     Gauss-Legendre in x = cos(theta) on [-1, 1] with each weight multiplied
 *     by (1 - x^2)^{(d-3)/2}.  The discrete sum is the result; no
 *     extrapolation is applied.
 *   - Every function returns an frg_status (int).  No exception crosses the
 *     ABI.  On failure frg_last_error() returns a message for the calling
 *     thread.
 *   - Memory: the caller owns every input and output buffer.  `mem` says
 *     where ALL pointers of a call live (FRG_MEM_HOST or FRG_MEM_DEVICE); it
 *     is never guessed.  Device calls are asynchronous on `hip_stream` (a
 *     hipStream_t, NULL = the null stream; from PyTorch pass
 *     torch.cuda.current_stream().cuda_stream); host calls are synchronous.
 *   - A context serialises its synchronous calls internally; one context may
 *     be shared by threads.  frg_submit/frg_poll are thread-safe.
 */
#ifndef FRG_H
#define FRG_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes --------------------------------------------------------- */
#define FRG_OK 0
#define FRG_PENDING 1        /* frg_poll: the flow is not finished            */
#define FRG_E_INVAL (-1)     /* bad argument; nothing was written             */
#define FRG_E_DOMAIN (-2)    /* some point had m^2 + k^2 <= 0: its result is
                                NaN, every other result is valid              */
#define FRG_E_NOMEM (-3)     /* device memory or the HBM budget is exhausted  */
#define FRG_E_DEVICE (-4)    /* a HIP runtime call failed                     */
#define FRG_E_AGAIN (-5)     /* submission queue full; retry later            */
#define FRG_E_NOTFOUND (-6)  /* unknown ticket                                */
#define FRG_E_STEP (-7)      /* flow stepper failed (step size underflow)     */

/* ---- enumerations --------------------------------------------------------- */
#define FRG_REG_EXP 0
#define FRG_REG_LITIM 1

#define FRG_PREC_FP64 0   /* FP64 throughout                                   */
#define FRG_PREC_FP32C 1  /* relative error at most "fp32c_flag_ppb" (1e-7)
                             per result, by a stated bound: point lists of
                             the exponential regulator take e^{-y} from the
                             FP32 hardware exponential (corrected to first
                             order in FP64), everything else in FP64, with a
                             deterministic per-result error bound; points
                             whose bound exceeds the tolerance, points near
                             the pole (m^2 + k^2)/k^2 < "fp32c_band_ppm" 1e-6,
                             Litim points and tensor grids are evaluated in
                             FP64 (an unpacked FP32 operation costs what an
                             FP64 one does on this GPU, and the FP64 grid
                             form runs on the matrix cores)                   */

#define FRG_MEM_HOST 0
#define FRG_MEM_DEVICE 1

/* frg_integrate flags */
#define FRG_PLAIN 0       /* one ordinary launch per integral set              */
#define FRG_PERSISTENT 1  /* all sets in one persistent launch over a
                             longest-first work list                           */
#define FRG_GRAPH 2       /* with FRG_PERSISTENT: replay a captured HIP graph
                             when the same batch (same pointers and shapes) is
                             submitted again                                    */

typedef struct frg_ctx frg_ctx;

/* Create a context on HIP device `hip_device`.  `hbm_budget_bytes` bounds the
 * device memory the context holds (0 = 1/2 of the device's free memory at
 * creation): its working buffers (quadrature, LPA and vertex tables, staging
 * of host-memory calls, captured work lists, the segmented tabulated form's
 * buffers) and, beside them, the flow server's flow state.  A call whose
 * buffers would exceed it returns FRG_E_NOMEM without launching its kernels;
 * a flow that does not fit beside the context's buffers is refused at
 * submission.  Tables, work lists and staging buffers are owned by the
 * context and freed by frg_destroy. */
int frg_create(frg_ctx **out, int hip_device, uint64_t hbm_budget_bytes);

/* Finish or cancel all flows, free all device and host resources. */
void frg_destroy(frg_ctx *ctx);

/* Message of the last failed call on this thread ("" if none). */
const char *frg_last_error(void);

/* Library version string. */
const char *frg_version(void);

/* ---- quadrature description ---------------------------------------------- */
typedef struct {
  int32_t d;          /* space-time dimension, 3 <= d <= 8                     */
  int32_t reg;        /* FRG_REG_EXP or FRG_REG_LITIM                          */
  double k;           /* RG scale, > 0                                         */
  double q_max;       /* radial cut-off, > 0 (usually 6k)                      */
  int32_t n_radial;   /* radial Gauss-Legendre order, 1..1024                  */
  int32_t n_angular;  /* angular Gauss-Legendre order, 1..256                  */
  int32_t prec;       /* FRG_PREC_FP64 or FRG_PREC_FP32C                       */
  int32_t reserved;   /* must be 0                                             */
} frg_quad;

/* One integral set: n_ext independent external points (p[e], m2[e]).
 *   out[e] = P_d sum_i sum_j w_i q_i^{d-1} d_tR(q_i^2) G(q_i^2)^2 mu_j G(s_ij),
 *   s_ij = |q_i + p_e|^2 = q_i^2 + p_e^2 + 2 q_i p_e x_j,
 *   P_d = Omega_{d-1}/(2 pi)^d,  Omega_n = 2 pi^{n/2}/Gamma(n/2),
 * the radial x angular Gauss-Legendre form of
 *   int d^dq/(2 pi)^d d_tR_k(q^2) G(q^2)^2 G(|q+p|^2).
 * p[e] >= 0.  err_est (optional, FP32C only) receives a bound of the
 * relative error of out[e] (1e-14 for results evaluated in FP64); used_fp64
 * (optional, FP32C only) receives 1 where the point was evaluated in FP64.  Arrays are contiguous float64 / uint8. */
typedef struct {
  frg_quad quad;
  int64_t n_ext;
  const double *p;
  const double *m2;
  double *out;
  double *err_est;
  uint8_t *used_fp64;
} frg_set;

/* Evaluate n_sets integral sets.  flags: FRG_PLAIN, or FRG_PERSISTENT
 * (optionally | FRG_GRAPH).  Results are bitwise identical for every flag
 * and every tile choice: the summation order of each result depends only on
 * (n_radial, n_angular).  Returns FRG_E_DOMAIN if any point had
 * m^2 + k^2 <= 0 (host memory; device calls are asynchronous: they return
 * FRG_OK, leave NaN in out and record the violation for frg_stream_status). */
int frg_integrate(frg_ctx *ctx, const frg_set *sets, int32_t n_sets, int32_t mem, int32_t flags,
                  void *hip_stream);

/* Tensor grid of external points sharing one quadrature:
 *   out[a * n_m + b] = I(p[a], m2[b])   (same formula as frg_set).
 * The regulator part of G(|q+p|) depends on p only, so it is evaluated once
 * per (p, node) and reused for every mass.  err_est / used_fp64 as in
 * frg_set (n_p * n_m entries, optional). */
int frg_integrate_grid(frg_ctx *ctx, const frg_quad *quad, int64_t n_p, const double *p,
                       int64_t n_m, const double *m2, double *out, double *err_est,
                       uint8_t *used_fp64, int32_t mem, void *hip_stream);

/* ---- tabulated-propagator variant ---------------------------------------- */
/* A table of n_rows propagators G_r(s), s = q^2 (for instance dressed
 * propagators 1/(Gamma^(2)(q) + R_k(q)) from an earlier solution, one row per
 * field value), each sampled at n_s >= 2 points of the uniform grid
 * s_k = k s_max/(n_s - 1): g[r * n_s + k], contiguous float64.  Between nodes
 * G_r is the piecewise-linear interpolant, G_r(s) = g_r[k] + f (g_r[k+1] -
 * g_r[k]) with k = floor(s/h), f = s/h - k, h = s_max/(n_s - 1); beyond s_max
 * it is the last node g_r[n_s - 1]. */
typedef struct {
  int64_t n_rows;
  int64_t n_s;
  double s_max;
  const double *g;
} frg_gtab;

/* Flow diagram with tabulated propagators (the regulator insertion d_tR stays
 * analytic; quad.prec must be FRG_PREC_FP64):
 *   out[a * n_rows + r] = P_d sum_i sum_j w_i q_i^{d-1} d_tR(q_i^2)
 *                          G_r(q_i^2)^2 mu_j G_r(s_ij),
 *   s_ij = (q_i - p_a)^2 + 2 q_i p_a (1 + x_j)   (rules as for frg_set).
 * p[a] >= 0 (a negative p gives NaN in its row of out and FRG_E_DOMAIN as
 * for frg_integrate).  Rows that fit in LDS beside the quadrature tables (up
 * to 6144 nodes, knob "tab_lds_nodes") are staged there; longer rows are read
 * from HBM, either through the caches (each XCD working through its rows one
 * at a time so that the rows in flight stay in cache; the same bits as the
 * LDS form) or in the segmented form: segments of 2048 nodes of four rows at
 * a time are copied into LDS and every evaluation that falls in a segment is
 * done there, its coordinate shared by the four rows (terms sorted by segment
 * once per call); the sum of each result runs over segments in order and does
 * not depend on how the work is split; it agrees with the other forms to
 * rounding and keeps n_p * n_rows * ceil(n_s / 16384) doubles of partial sums
 * and n_p * n_r * n_a 16-bit term indices in context buffers.  Knob "tab_seg"
 * chooses: 2 (the default) the segmented form when the table (n_rows * n_s
 * doubles) exceeds 256 MiB and its buffers fit the context's HBM budget,
 * else the cache-streamed form; 1 the segmented form; 0 the cache-streamed
 * form.  mem says where p,
 * tab->g and out live; n_p * n_rows results. */
int frg_integrate_tab(frg_ctx *ctx, const frg_quad *quad, const frg_gtab *tab, int64_t n_p,
                      const double *p, double *out, int32_t mem, void *hip_stream);

/* ---- two-external-momentum (vertex) diagram -------------------------------- */
/* One-loop diagram with two external momenta p1, p2 at angle th:
 *   V(p1, p2, th, m^2) = int d^dq/(2pi)^d d_tR(q^2) G(q^2)^2 G(|q+p1|^2) G(|q+p2|^2),
 *   G(s) = 1/(s + R_k(s) + m^2),
 *   |q+p1|^2 = q^2 + p1^2 + 2 q p1 x,
 *   |q+p2|^2 = q^2 + p2^2 + 2 q p2 (x cos th + sqrt(1 - x^2) cos phi sin th),
 * with x the polar cosine of q to p1 and phi its azimuth about p1 measured
 * from the (p1, p2) plane.  Discretised as
 *   V = Omega_{d-2}/(2pi)^d sum_i sum_j sum_l w_i q_i^{d-1} d_tR(q_i^2) G(q_i^2)^2
 *         mu_j G(s1_ij) nu_l G(s2_ijl),
 * the radial and polar rules of frg_set (quad; FP64 only), and n_azimuth
 * Gauss-Legendre nodes phi_l on [0, pi] with nu_l = (pi/2) w_l sin^{d-3}(phi_l).
 * Tensor grid of configurations and masses:
 *   out[c * n_m + b] = V(p1[c], p2[c], acos(cos12[c]), m2[b]).
 * p1, p2 >= 0, -1 <= cos12 <= 1 and m2 + k^2 > 0, else NaN and FRG_E_DOMAIN
 * (host memory; device calls are asynchronous and return FRG_OK).  mem says
 * where p1, p2, cos12, m2 and out live. */
int frg_integrate_vertex(frg_ctx *ctx, const frg_quad *quad, int32_t n_azimuth, int64_t n_c,
                         const double *p1, const double *p2, const double *cos12, int64_t n_m,
                         const double *m2, double *out, int32_t mem, void *hip_stream);

/* ---- finite-volume LPA ----------------------------------------------------- */
/* The LPA O(N) flow of the potential (frg_lpa) written for u = dU/dsigma,
 * sigma the field amplitude (rho = sigma^2/2), as a conservation law
 *   d_t u = d_sigma Q,  Q = 1/2 F_1(d_sigma u) + (N-1)/2 F_1(u/sigma),
 * F_n(m^2) = C_d sum_i w_i q_i^{d-1} d_tR(q_i^2) G(q_i^2)^n at k = lambda e^t
 * (radial rule on [0, q_max_over_k k]; Litim: [0, k]).  Finite volumes:
 * n_cells cells of width ds = sigma_max/n_cells hold averages u_i (cell i
 * = [i ds, (i+1) ds]); interface j = 0..n_cells at sigma_j = j ds;
 *   d_t u_i = (Q_{i+1} - Q_i)/ds,
 *   Q_0 = N/2 F_1(2 u_0/ds)   (sigma = 0, where u/sigma = d_sigma u),
 *   Q_j = 1/2 F_1((u_j - u_{j-1})/ds) + 1/2 (f(u-) + f(u+)) - 1/2 a_j (u+ - u-),
 *   f(u) = (N-1)/2 F_1(u/sigma_j),  a_j = max(|f'(u-)|, |f'(u+)|),
 *   f'(u) = -(N-1)/2 F_2(u/sigma_j)/sigma_j   (local Lax-Friedrichs flux),
 *   u- = u_{j-1} + s_{j-1}/2, u+ = u_j - s_j/2, s_i = minmod(u_i - u_{i-1}, u_{i+1} - u_i)
 * (minmod(a, b) = 0 if ab <= 0, else the one of smaller modulus; the
 * semi-discrete central scheme of Kurganov and Tadmor), with ghost cells
 * u_{-1} = -u_0, u_{-2} = -u_1 (u odd) and u_n = 2u_{n-1} - u_{n-2},
 * u_{n+1} = 2u_n - u_{n-1} (linear extrapolation).  A flow leaves the domain
 * when a mass argument has m^2 + k^2 <= 0. */
typedef struct {
  int32_t d;            /* 2 <= d <= 8                                         */
  int32_t N;            /* O(N), 1..64                                         */
  int32_t reg;          /* FRG_REG_EXP or FRG_REG_LITIM                        */
  int32_t n_radial;     /* 1..1024                                             */
  double lambda;        /* UV scale, > 0: k = lambda e^t                       */
  double q_max_over_k;  /* > 0 (usually 6)                                     */
  int64_t n_cells;      /* 2..2^24                                             */
  double sigma_max;     /* > 0                                                 */
} frg_fvlpa;

/* One right-hand side at RG time t for n_flows (0..65535) flows: u and dudt hold
 * n_flows * n_cells values (row r = flow r).  dt_est (n_flows, may be NULL)
 * receives a step bound for explicit stepping, 1/max_j (2 D_j/ds^2 + a_j/ds)
 * with D_0 = N/2 F_2(2 u_0/ds), D_j = 1/2 F_2((u_j - u_{j-1})/ds).  A flow
 * outside the domain gets NaN (FRG_E_DOMAIN for host memory; device calls are
 * asynchronous and return FRG_OK).  mem says where all arrays live. */
int frg_fvlpa_rhs(frg_ctx *ctx, const frg_fvlpa *fv, int64_t n_flows, double t, const double *u,
                  double *dudt, double *dt_est, int32_t mem, void *hip_stream);

/* Integrate from t = 0 to t_end <= 0 with the three-stage strong-stability-
 * preserving Runge-Kutta method (Shu-Osher) in n_steps >= 1 equal steps h =
 * t_end/n_steps (stage times t_n, t_n + h, t_n + h/2), every stage on the
 * device; the step must respect the bound of frg_fvlpa_rhs (explicit
 * scheme).  u is updated in place; a flow whose right-hand side leaves the
 * domain at any stage of step n keeps its state at t_n and reports
 * t_reached = t_n, the others t_end.  Returns FRG_OK whether or not flows
 * stopped; device calls are asynchronous. */
int frg_fvlpa_solve(frg_ctx *ctx, const frg_fvlpa *fv, int64_t n_flows, double t_end,
                    int64_t n_steps, double *u, double *t_reached, int32_t mem, void *hip_stream);

/* ---- momentum-dependent two-point flow ------------------------------------ */
/* Flow of the momentum-dependent two-point function Gamma2_k(p) = p^2 +
 * Sigma_k(p) of one scalar with constant three- and four-point couplings
 * lam3, lam4: the second field derivative of the Wetterich equation, with the
 * one-loop flow diagram of frg_integrate_tab as its momentum-dependent part,
 *   d_t Sigma(p) = lam3^2 J(p) - (lam4/2) T,
 *   J(p) = int d^dq/(2pi)^d d_tR(q^2) G(q^2)^2 G(|q+p|^2),
 *   T    = int d^dq/(2pi)^d d_tR(q^2) G(q^2)^2,
 *   G(s) = 1/(s + R_k(s) + Sigma(sqrt s)),   k = lambda e^t.
 * Sigma of each flow lives on the n_s nodes s_a = a s_max/(n_s - 1) (p_a =
 * sqrt(s_a)); at each RG time the propagator table of the flow is
 * g[a] = 1/(s_a + R_k(s_a) + Sigma_a) (piecewise linear in s, the last node
 * beyond s_max, as in frg_gtab), J(p_a) is frg_integrate_tab of that row and
 * T = C_d sum_i w_i q_i^{d-1} d_tR(q_i^2) G(q_i^2)^2 its radial part, with the
 * quadrature rules at scale k (q_max = q_max_over_k k; Litim: min(q_max, k)).
 * A flow whose table has a denominator <= 0 has left the domain. */
typedef struct {
  int32_t d;            /* 3 <= d <= 8                                         */
  int32_t reg;          /* FRG_REG_EXP or FRG_REG_LITIM                        */
  int32_t n_radial;     /* 1..1024                                             */
  int32_t n_angular;    /* 1..256                                              */
  double lambda;        /* UV scale, > 0: k = lambda e^t                       */
  double q_max_over_k;  /* > 0 (usually 6)                                     */
  int64_t n_s;          /* momentum nodes, 2..2^24                             */
  double s_max;         /* > 0: last node                                      */
} frg_pflow;

/* One right-hand side at RG time t for n_flows flows:
 *   dsdt[r * n_s + a] = lam3[r]^2 J_r(p_a) - lam4[r]/2 T_r   given
 *   sigma[r * n_s + a] = Sigma_r(p_a);
 * lam3, lam4: n_flows each.  A flow outside the domain gets NaN in its row
 * (FRG_E_DOMAIN for host memory; device calls are asynchronous and return
 * FRG_OK).  mem says where all arrays live. */
int frg_pflow_rhs(frg_ctx *ctx, const frg_pflow *pf, int64_t n_flows, const double *lam3,
                  const double *lam4, double t, const double *sigma, double *dsdt, int32_t mem,
                  void *hip_stream);

/* Integrate n_flows flows from t = 0 to t_end <= 0 with the classical
 * fourth-order Runge-Kutta method in n_steps >= 1 equal steps h = t_end/n_steps
 * (stage times t_n + {0, h/2, h/2, h}, t_n = n h), every stage on the device.
 * sigma (n_flows * n_s, row r = flow r) holds Sigma at t = 0 on entry and at
 * t_reached[r] on return.  A flow whose right-hand side leaves the domain at
 * any stage of step n keeps its state at t_n and reports t_reached[r] = t_n;
 * the others report t_end (flows are independent: a batch gives the same
 * bits as each flow alone).  Returns FRG_OK whether or not flows stopped (the
 * stop is a result, read from t_reached); device calls are asynchronous. */
int frg_pflow_solve(frg_ctx *ctx, const frg_pflow *pf, int64_t n_flows, const double *lam3,
                    const double *lam4, double t_end, int64_t n_steps, double *sigma,
                    double *t_reached, int32_t mem, void *hip_stream);

/* ---- LPA O(N) flow -------------------------------------------------------- */
/* Local potential approximation of the O(N) model, effective potential U(rho)
 * with rho = phi^2/2 on the uniform grid rho_j = j rho_max/(n_grid-1):
 *   d_t U = 1/2 [ F_1(m_s^2) + (N-1) F_1(m_p^2) ],
 *   m_s^2 = U' + 2 rho U'',  m_p^2 = U',
 *   F_n(m^2) = C_d sum_i w_i q_i^{d-1} d_tR(q_i^2) G(q_i^2)^n,  C_d = Omega_d/(2 pi)^d,
 * radial rule on [0, q_max_over_k * k] (exponential) or [0, k] (Litim).
 * U', U'' by second-order differences, grouped exactly as
 *   interior  U'  = (U[j+1] - U[j-1]) / (2 dr)
 *             U'' = ((U[j+1] - 2U[j]) + U[j-1]) / dr^2
 *   rho = 0   U'  = ((-3U[0] + 4U[1]) - U[2]) / (2 dr)
 *             U'' = (((2U[0] - 5U[1]) + 4U[2]) - U[3]) / dr^2
 *   rho_max   U'  = ((3U[n-1] - 4U[n-2]) + U[n-3]) / (2 dr)
 *             U'' = (((2U[n-1] - 5U[n-2]) + 4U[n-3]) - U[n-4]) / dr^2
 * and m_s^2 = U' + (2 rho) U'' without fused multiply-add. */
typedef struct {
  int32_t d;             /* 2..8                                            */
  int32_t N;             /* O(N) components, >= 1 (N = 1: no Goldstones)    */
  int32_t reg;           /* FRG_REG_EXP or FRG_REG_LITIM                     */
  int32_t n_radial;      /* radial order, 1..1024                            */
  double q_max_over_k;   /* radial cut-off in units of k (usually 6)         */
  double Lambda;         /* UV scale, k = Lambda e^t                         */
  int64_t n_grid;        /* grid points, 4..65536                            */
  double rho_max;        /* grid end, > 0                                    */
} frg_lpa;

/* Right-hand side at RG time t (k = Lambda e^t).  U and dUdt: n_grid float64.
 * jac_bands (optional): 7*n_grid float64, jac_bands[(o+3)*n_grid + j] =
 * d(dUdt_j)/dU_{j+o} for o = -3..3 (zero where j+o is off the grid), built
 * from dF_1/dm^2 = -F_2.  FRG_E_DOMAIN (host memory) if some mass had
 * m^2 + k^2 <= 0; the affected entries are NaN. */
int frg_flow_rhs(frg_ctx *ctx, const frg_lpa *lpa, double t, const double *U, double *dUdt,
                 double *jac_bands, int32_t mem, void *hip_stream);

/* The same for n_flows independent flows in ONE launch (device memory only):
 * flow f uses lpa[f], t[f], U[f], dUdt[f], jac_bands[f] (jac_bands may be
 * NULL, or contain NULL entries).  Each flow's result is bitwise identical to
 * frg_flow_rhs on that flow alone. */
int frg_flow_rhs_batch(frg_ctx *ctx, int32_t n_flows, const frg_lpa *lpa, const double *t,
                       const double *const *U, double *const *dUdt, double *const *jac_bands,
                       void *hip_stream);

/* ---- flow integration on the host ------------------------------------------ */
/* One LPA flow request: U(t=0) = (lambda/8)(rho - rho0)^2, integrated from
 * t = 0 to t_end < 0 by the implicit variable-step BDF(1,2) stepper in FP64
 * (Newton with the banded Jacobian, formed and factorised at a step's first
 * iterate and reused by its later ones; an iterate is accepted when its
 * correction times the contraction rate seen on the previous steps is below
 * the bar, the rate being measured again every 16 such steps; local error
 * control with rtol/atol).
 * U_out (host, n_grid float64) receives U(t_end); it must stay valid until
 * frg_poll reports completion. */
typedef struct {
  frg_lpa lpa;
  double lambda;
  double rho0;
  double t_end;
  double rtol;
  double atol;
  double *U_out;
} frg_request;

typedef struct {
  int32_t status;     /* FRG_OK: reached t_end.  FRG_E_DOMAIN: ran into the
                         propagator pole m^2 = -k^2 at t_reached (with the
                         exponential regulator in d = 3 the threshold
                         function F_1 stays finite at the pole, so a flow in
                         the broken phase reaches it at finite RG time).
                         FRG_E_STEP: step-size underflow.  FRG_PENDING.    */
  int32_t reserved;
  int64_t steps;      /* accepted steps                                     */
  int64_t rejected;   /* rejected steps                                     */
  int64_t rhs_calls;  /* right-hand-side evaluations                        */
  double submit_s;    /* monotonic clock, seconds                           */
  double start_s;     /* admitted and started                               */
  double done_s;      /* finished                                           */
  double t_reached;   /* RG time of the last accepted step (U_out holds U
                         there, also when the flow stopped early)           */
} frg_result;

/* Host right-hand side used by frg_flow_solve: fill dUdt[n] and, if
 * jac_bands != NULL, the 7 bands as in frg_flow_rhs.  Return FRG_OK, or
 * FRG_E_DOMAIN to make the stepper reject the step. */
typedef int (*frg_rhs_fn)(void *user, double t, const double *U, int64_t n, double *dUdt,
                          double *jac_bands);

/* Integrate one request synchronously with a caller-supplied right-hand side
 * (host only; no GPU use).  The stepper is the one the flow server runs.
 * Returns the final status (also in out->status). */
int frg_flow_solve(const frg_request *req, frg_rhs_fn rhs, void *user, frg_result *out);

/* Submit a flow to the context's server (never blocks).  The server admits
 * a flow when a slot is free and its device footprint fits the HBM budget,
 * and batches the right-hand-side evaluations of all running flows into
 * shared launches (continuous batching), each reading and writing one packed
 * pinned buffer.  FRG_E_AGAIN if the queue is full.  Environment, read when
 * the server starts: FRG_SERVER_SLOTS (flows run at once, default 64) and
 * FRG_SERVER_SPIN_FLOWS (while at most this many run, a flow's stepper polls
 * briefly for each answer before it sleeps; default 12). */
int frg_submit(frg_ctx *ctx, const frg_request *req, uint64_t *ticket);

/* FRG_PENDING until the flow finishes; then the result (status inside) and
 * FRG_OK, and the ticket is released.  FRG_E_NOTFOUND for unknown tickets. */
int frg_poll(frg_ctx *ctx, uint64_t ticket, frg_result *out);

/* Server statistics: completed flows, batched launches and the mean number of
 * flows per launch since creation. */
int frg_server_stats(frg_ctx *ctx, int64_t *flows_done, int64_t *launches, double *mean_batch);

/* ---- launch shapes ------------------------------------------------------------- */
/* Launch-shape autotuning (points per wave, masses per wave, waves per
 * workgroup, tiles of the persistent work list).  mode 0: defaults and any
 * cached choice; mode 1: the first call with a new key (kernel, regulator,
 * n_radial, n_angular, precision, size class) times each candidate shape on
 * that call's own inputs with HIP events on its stream (that call then
 * synchronises the stream) and keeps the fastest.  cache_path (optional,
 * NULL = keep the current one) names a text file read now and rewritten
 * after each tuning.  The environment variables FRG_AUTOTUNE and
 * FRG_AUTOTUNE_CACHE set the same at frg_create.  The summation order of
 * every result is fixed by (n_radial, n_angular): no launch shape changes a
 * result. */
int frg_autotune(frg_ctx *ctx, int32_t mode, const char *cache_path);

/* Set / read one default launch-shape knob: "grid_M" (4, 8, 16), "grid_W"
 * (1..8), "grid_MB" (1..64) of the FP64 tensor-grid kernel,
 * "grid_form" (0: per-momentum Horner coefficients of one rational function
 * per lane, radial node and group of up to 32 angular terms, radial factor
 * included, when the table fits in LDS, the default; 1: eight-term running
 * fractions as in frg_integrate; 2 / 3: coefficients in groups of 8 / 16;
 * the forms agree to a few ulp), "grid_mfma" (coefficient form, 1: power
 * sums over tiles of 16 masses on the FP64 matrix cores, the default; 0:
 * nested evaluation on the vector units, at most 8 masses per wave; the two
 * agree to a few ulp), "fv_persistent" (finite-volume solves, 1: one
 * workgroup per flow runs the steps with its cells in LDS, the default where
 * 3 n_cells + 2 n_radial doubles fit in 64 KiB; 0: two launches per stage;
 * the same bits), "pflow_fused" (momentum-dependent flows with rows in LDS,
 * 1: one launch per RK4 stage, each workgroup redoing the previous stage's
 * update for its row, the default; 0: a diagram launch and a stage launch
 * per stage; the same bits), "vertex_W" (vertex diagrams whose coefficient
 * table takes over half the LDS: waves of the one workgroup per CU, 1..12,
 * default 12; above 8 only for the matrix-core form with groups of up to 16
 * azimuthal terms, else 8), "server_zero_copy" (flow server, 1: the LPA kernel reads
 * and writes the pinned batch buffer in place, the default; 0: one upload and
 * one download per batch; the same bits; two batch buffers, the next batch
 * staged while one runs), "grid_lds_rows" (8..96), "plain_tile" (points per
 * tile of a plain launch, 1..64), "persist_tile" (work of a tile of the persistent list, in
 * units of 1024 evaluations: 1..64 points of one set), "persist_wpc" (1..64), and of the
 * tabulated variant "tab_W" (1..4),
 * "tab_pw" (momenta per wave, 1..64), "tab_lds_nodes" (2..6144),
 * "tab_pairs" (1: rows in LDS as (value, slope) pairs, the default; 0: as
 * values; the same bits), "tab_rb" (rows in LDS per workgroup, sharing every
 * coordinate: 0 auto (two where there are two and they fit), 1, 2 or 4; the
 * same bits), "tab_rW" (waves of such a workgroup, 1..16, default 16),
 * "tab_seg" (rows that do not fit in LDS: 0 read
 * through the caches; 1 the segmented form; 2 the segmented form for tables
 * above 256 MiB, the default; the forms agree to rounding), and for cache-streamed rows "tab_wpc" (workgroups per
 * CU, 1..16), "tab_sW" (1..4), "tab_spw" (1..64).  Setting a knob drops the
 * tuned choices so that it takes effect.  Two knobs route FRG_PREC_FP32C
 * points to FP64 and do change results (within the FP32 tolerance):
 * "fp32c_flag_ppb" (error-bound threshold in units of 1e-9, default 100)
 * and "fp32c_band_ppm" (pole band on (m^2 + k^2)/k^2 in units of 1e-6,
 * default 10000). */
int frg_tune_set(frg_ctx *ctx, const char *key, int32_t value);
int frg_tune_get(frg_ctx *ctx, const char *key, int32_t *value);

/* ---- allocation-free variant ------------------------------------------------- */
/* For callers that cannot allocate device memory -- code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc:
 * frg_integrate(ctx, sets, n_sets, FRG_MEM_DEVICE, FRG_PERSISTENT, hip_stream),
 * the same kernel and the same bits, with its work-list counters, set
 * descriptors, longest-first work list and quadrature tables in a scratch
 * area of 4 MiB that the library keeps in device memory on every GPU it
 * runs on (a static device array, held until the process ends), filled by
 * one copy from a pinned buffer that frg_create allocated.  The call
 * allocates and frees no device memory (a quadrature key seen for the first
 * time costs host memory for its table only).  All pointers of `sets` are
 * device memory; results are asynchronous on hip_stream.
 * domain_flag (optional, device memory): set to 1 when a point has
 * m^2 + k^2 <= 0 or p < 0 (its result is NaN); the caller clears it.
 * Errors: FRG_E_INVAL for bad arguments and for a call whose descriptors,
 * work list and tables exceed the 4 MiB area (the message gives the bytes
 * needed: about 150 B per set, 16 B per tile of about 4096 evaluations and
 * 8 (3 n_radial + 3 n_angular) B per distinct quadrature); nothing is then
 * launched.
 * The area is shared by every call on one GPU and keeps the last call's
 * contents.  A call waits on the host for the previous call of its context
 * to finish before it overwrites the area, so the calls of one context never
 * overlap; calls from different contexts (or processes) on one GPU that
 * overlap in time race. */
int frg_integrate_noalloc(frg_ctx *ctx, const frg_set *sets, int32_t n_sets, int32_t *domain_flag,
                          void *hip_stream);

/* ---- domain status of device calls ----------------------------------------- */
/* Device-memory calls are asynchronous and return before their kernels run,
 * so a point outside the domain (m^2 + k^2 <= 0, p < 0, cos12 outside
 * [-1, 1]) cannot change their return value; the kernels record it in a word
 * kept per (context, stream).  frg_stream_status waits for hip_stream (as
 * hipStreamSynchronize) and returns FRG_E_DOMAIN if a device call of
 * frg_integrate, frg_integrate_grid, frg_integrate_tab, frg_integrate_vertex,
 * frg_flow_rhs or frg_flow_rhs_batch on that stream met such a point since
 * the previous frg_stream_status for the stream (the affected results are
 * NaN), else FRG_OK; the record is then cleared.  The flow solvers
 * (frg_pflow_solve, frg_fvlpa_solve) report per flow through t_reached. */
int frg_stream_status(frg_ctx *ctx, void *hip_stream);

/* ---- host-only helpers ------------------------------------------------------ */
/* Gauss-Legendre nodes (ascending) and weights on [-1, 1], n = 1..4096, by
 * the Golub-Welsch eigenvalue method (no GPU use). */
int frg_gauss_legendre(int32_t n, double *x, double *w);

/* e^{-y} for n arguments (0 <= y, not NaN), evaluated on the host by the
 * same operations, in the same order and rounding, as the point kernels use
 * for the exponential regulator: the table-driven method of Tang (ACM Trans.
 * Math. Softw. 15, 1989) with 64 entries 2^{j/64}, a Cody-Waite reduction and
 * a degree-5 polynomial; below 1.6 ulp where the result is normal, 0 above
 * y = 745.2.  y and out: n float64 each (host memory; no GPU use).
 * FRG_E_INVAL for n < 0 or NULL arrays with n > 0. */
int frg_expneg(int64_t n, const double *y, double *out);

/* e^{-y} for n arguments (y >= 0) on the GPU, by the operations the
 * FRG_PREC_FP32C point path uses: the FP32 hardware exp2 of
 * fl32(-y log2 e), corrected to first order by the FP64 residual
 * -y - fl32(-y log2 e) ln 2.  Its relative error (below 1.2e-7 where e^{-y}
 * is an FP32 normal, y < 87.3; absolute error below 2^-126 beyond) is the
 * premise of that path's error bound.  y and out: n float64 each in device
 * memory; asynchronous on hip_stream.  FRG_E_INVAL for a NULL ctx, n < 0 or
 * NULL arrays with n > 0. */
int frg_expneg_fp32c(frg_ctx *ctx, int64_t n, const double *y, double *out, void *hip_stream);

/* Bytes of device memory one flow of this shape takes in the server's staging
 * buffer during a batched call (what the server's HBM admission charges). */
int64_t frg_flow_footprint(const frg_lpa *lpa);

#ifdef __cplusplus
}
#endif

#endif /* FRG_H */
