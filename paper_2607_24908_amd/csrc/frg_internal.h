// Internal declarations shared by the host and device translation units of
// libfrg.  Nothing here is part of the public ABI (include/frg.h).
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include "frg.h"

namespace frg {

constexpr int kWave = 64;

// ---------------------------------------------------------------- tables --
// Gauss-Legendre rule on [-1, 1] (ascending nodes) by Golub-Welsch.
int gauss_legendre_gw(int n, double *x, double *w);

// Packed quadrature table of one (d, reg, k, q_max, n_r, n_a) key, float64:
//   [0, n_r)            q_i       radial node
//   [n_r, 2n_r)         c_i       w_i q_i^{d-1} d_tR(q_i^2)
//   [2n_r, 3n_r)        Hq_i      k^2 h(q_i^2/k^2)   (stable denominator part)
//   [3n_r, 3n_r+n_a)    opx_j     1 + x_j
//   [.., +n_a)          mu_j      v_j (1 - x_j^2)^{(d-3)/2}
//   [.., +n_a)          rmu_j     1 / mu_j
constexpr int table_doubles(int n_r, int n_a) { return 3 * n_r + 3 * n_a; }

struct QuadTable {
  std::vector<double> data;
  double k2, inv_k2, pref;  // pref = P_d
  double q_top;             // q_max: every radial node lies below it
  double rmu_max;           // max_j rmu_j
  int n_r, n_a;
};
QuadTable build_quad_table(const frg_quad &q);

// Scale-free radial table for the LPA threshold functions (unit k):
//   [0, n_r)       chat_i = what_i qhat_i^{d-1} 2 beta(y) beta(-y)   (exp)
//                          = what_i qhat_i^{d-1} 2                    (Litim)
//   [n_r, 2n_r)    hhat_i = h(qhat_i^2)
// so that F_n(m^2) = C_d k^{d+2-2n} sum_i chat_i / (hhat_i + delta/k^2)^n.
struct LpaTable {
  std::vector<double> data;  // chat (n_r) | hhat (n_r) | coefficient groups (fv_groups(n_r))
  double Cd;
  int n_r;
};
// Coefficient groups of the radial sums of the finite-volume flux: nodes
// 8g .. 8g + 7 (padded with c = 0, h = 1) form group g, stored as
// [a_0..a_7 | b_0..b_7 | m_0..m_14] with
//   P(x) = prod_l (x + h_l) = x^8 + sum_{k<8} a_k x^k,
//   N(x) = sum_i c_i prod_{l != i} (x + h_l) = sum_{k<8} b_k x^k,
//   M(x) = sum_i c_i prod_{l != i} (x + h_l)^2 = sum_{k<15} m_k x^k,
// so that sum_i c_i/(x + h_i) = N/P and sum_i c_i/(x + h_i)^2 = M/P^2 over the
// group.  Every coefficient is >= 0.
constexpr int kFvGroup = 8;
constexpr int kFvCoef = 31;
inline int fv_groups(int n_r) { return (n_r + kFvGroup - 1) / kFvGroup; }
LpaTable build_lpa_table(int d, int reg, int n_r, double q_max_over_k);

double omega_sphere(int n);  // area of S^{n-1}
double h_exp_host(double y);
double dtR_over_k2_host(int reg, double y);  // d_tR / k^2 at y = s/k^2

// ---------------------------------------------------------- device structs --
struct SetDev {
  const double *p;
  const double *m2;
  double *out;
  double *err;
  uint8_t *used64;
  const double *tab;  // device copy of QuadTable::data
  double k2, inv_k2, pref;
  double pref_k;  // pref / k^2: the point kernels sum in units of k^2
  int64_t n_ext;
  int32_t n_r, n_a, reg, prec;
  int32_t R, J;  // lanes along radial / angular nodes, R * J = 64
  int32_t T, U;  // ceil(n_r / R), ceil(n_a / J)
  double f32_flag;  // FP32C: error bound above which a point is evaluated in FP64
  double f32_band;  // FP32C: delta/k^2 below which a point is evaluated in FP64
  double q_top, rmu_max;  // range test of the grouped reciprocal sums
};

struct Tile {
  int32_t set;
  int32_t count;
  int64_t start;
};

// Work-list counters of the persistent point kernel (one per XCD of MI355X),
// kCounterStride ints apart (256 bytes: one cache line each); a launch needs
// kCounters * kCounterStride ints with the counters zero at its start.
constexpr int kCounters = 8;
constexpr int kCounterStride = 64;
constexpr int kCounterInts = kCounters * kCounterStride;

struct GridArgs {
  const double *p;
  const double *m2;
  double *out;
  const double *tab;
  int *flag;
  double k2, inv_k2, pref;
  double q_top, rmu_max;
  int64_t n_p, n_m;
  int32_t n_r, n_a, R, J, T, U;
  int32_t n_mb;     // workgroups per momentum
  int32_t chunk;    // (t, u) rows of the Hk table held in LDS at once
  int32_t mblocks;  // mass blocks per wave when the table is resident
  int32_t form;     // resident FP64 form: 0 coefficients (when they fit; group size from U),
                    // 1 running fractions, 2 / 3 coefficients in groups of 8 / 16
  double sig, kap, pref_c;  // coefficient form: scale of x and H, of c; pref kap^-1 sig^(E+1)
  // vertex diagram only: second momentum, cos of the angle, per-config;
  // vtab = [x_j | sqrt(1 - x_j^2) | cos phi_l | nu_l]
  const double *p2, *c12, *vtab;
  int32_t n_phi;
};


struct LpaJob {
  const double *U;
  double *dUdt;
  double *jac;      // may be null
  const double *tab;  // LpaTable::data on the device
  int *flag;        // set to 1 on a domain violation (may be null)
  double k2, inv_k2;
  double pre1, pre2;  // C_d k^d, C_d k^{d-2}
  double dr, Nm1;
  int64_t n;
  int32_t n_r, N;
};

void lane_split(int n_r, int n_a, int *R, int *J, int *T, int *U);

// Tabulated-propagator kernel arguments.  Lane map: J = largest power of two
// <= min(n_a, 8) angular lanes (neighbouring lanes read neighbouring table
// entries), R = 64 / J radial lanes.
struct TabArgs {
  const double *p;
  double *out;        // out[a * os_p + r * os_r] for momentum a of row r
  const double *g;    // table rows, g[r * n_s + k]
  const double *tab;  // QuadTable::data on the device
  int *flag;
  double pref, k2, inv_h, t_last;  // t_last = n_s - 1
  int64_t n_p, n_rows, n_s;
  int64_t os_p, os_r;
  int32_t n_r, n_a, R, J, T, U;
  int32_t pw;     // momenta per wave
  int32_t n_pb;   // momentum blocks per row (W * pw momenta each)
  int32_t pairs;  // rows in LDS as (value, slope) pairs
  int32_t rb;     // rows in LDS: rows per workgroup (1, 2 or 4; 0 means 1)
};
void tab_lane_split(int n_r, int n_a, int *R, int *J, int *T, int *U);

// Momentum-dependent two-point flow (pflow.hip).  State Sigma_r(s_a) of
// n_rows flows on the nodes s_a = a h_s.  A right-hand side at RG time t
// needs the propagator rows g_r[a] = 1/(s_a + R_k(s_a) + Sigma), the domain
// check, the tadpoles T_r and the quadrature table at scale k (prep), then
// the tabulated diagram J[a * n_rows + r] at p_a = sqrt(s_a) (tab_kernel),
// then rhs = lam3^2 J - lam4/2 T and the RK4 stage update (stage kernel,
// which also does the prep of the next stage).
struct PflowArgs {
  const double *base;  // QuadTable data at k = 1, q_max = kappa (device)
  double *tabk;        // the same table at scale k (written by the prep kernel)
  const double *lam3, *lam4;
  double *y0;          // state at the start of the step (n_rows * n_s)
  double *ys;          // stage state
  double *acc;         // RK4 accumulator
  double *g;           // propagator rows
  double *J;           // diagram, J[a * n_rows + r]
  double *T;           // tadpole per flow
  double *p;           // p_a = sqrt(s_a)
  int *alive;
  double *t_reached;
  double *dsdt;        // right-hand side only (stage = 4)
  int *flag;
  double k, k2, kd2, Cd;  // scale of the (next) prep, kd2 = k^(d+2)
  double h_s, inv_h, t_last;
  double t_n, h;        // start of the step of the (next) prep, step size
  int64_t n_rows, n_s;
  int32_t n_r, n_a;
  int32_t stage;        // update: 0..3 RK4 stages, 4: right-hand side only
  int32_t prep;         // stage kernel: also prepare the next stage (at k, t_n)
};
// Finite-volume LPA (fvlpa.hip): cell averages u[r * n + i] of u = dU/dsigma
// for n_rows flows; interface fluxes Q[r * (n + 1) + j] and their local rate
// bounds lam (same layout); F_n from the scale-free LPA table [chat | hhat].
struct FvArgs {
  const double *tab;   // LpaTable::data on the device
  double *y0;          // state at the start of the step
  double *ys;          // stage state
  double *Q, *lam;
  double *dudt;        // right-hand side only (stage = 3)
  double *dt;          // right-hand side only: step estimate per flow (may be null)
  int *alive;
  double *t_reached;
  int *flag;
  double Cd, lambda;    // k = lambda e^t
  double t;             // flux kernel: RG time of the stage
  double ds, inv_ds, h, t_n;
  int64_t n_rows, n;
  int32_t n_r, N, d;
  int32_t stage;       // 0..2 SSP-RK3 stages, 3: right-hand side only
  int32_t first;       // flux kernel: read y0 (first stage / rhs) instead of ys
};
int launch_fv_init(const FvArgs &a, double t_end, void *stream);
int launch_fv_flux(const FvArgs &a, void *stream);
int launch_fv_stage(const FvArgs &a, void *stream);
int launch_fv_dt(const FvArgs &a, void *stream);
// Steps [s0, s0 + n_st) of a solve, one workgroup of `threads` per flow with
// its state in LDS (fv_solve_lds_bytes); alive, t_reached and flag set up by
// launch_fv_init.
int64_t fv_solve_lds_bytes(const FvArgs &a);
constexpr int kFvSolveLdsMax = 160 * 1024;
int launch_fv_solve(const FvArgs &a, int64_t s0, int64_t n_st, int threads, void *stream);
int launch_pflow_init(const PflowArgs &a, double t_end, void *stream);
int launch_pflow_prep(const PflowArgs &a, int reg, void *stream);
int launch_pflow_stage(const PflowArgs &a, int reg, void *stream);
// One launch per stage (pflow_pull_kernel): the update of the previous
// stage, the prep and the diagram of this one.  Arrays "p" are the previous
// launch's, arrays "n" this launch's (stored by the workgroup with pb = 0);
// the two never alias, except y0p / y0n where only y0n is written.
struct PflowPull {
  const double *base;  // QuadTable data at k = 1, q_max = kappa (device)
  const double *lam3, *lam4;
  const double *Jp, *Tp, *accp, *y0p;  // J[r * n_s + a]; y0p: state at the start of the step
  const int *alivep;
  double *Jn, *Tn, *accn, *y0n;        // y0n: new step-start state (prev = 3)
  int *aliven;
  double *t_reached;
  double *dsdt;  // right-hand side only (final update, prev = 4)
  int *flag;
  double k, k2, kd2, Cd;  // scale of this stage, kd2 = k^(d+2)
  double h_s, inv_h, t_last;
  double t_n, h;  // start of this stage's step, step size
  int64_t n_rows, n_s;
  int32_t n_r, n_a;
  int32_t prev;  // stage of the previous launch (0..3), -1 none; final update: 3 or 4
};
int pflow_pull_lds_bytes(const TabArgs &t);
// t: the diagram (t.tab = the table at k = 1, t.out = a.Jn), rows in LDS, W waves
int launch_pflow_pull(const TabArgs &t, const PflowPull &a, int reg, int W, void *stream);
int launch_pflow_final(const PflowPull &a, void *stream);
constexpr int64_t tab_lds_max_nodes = 6144;  // rows up to this many nodes are staged in LDS

// Segmented form of the tabulated diagram (tab_seg.hip), for rows longer than
// the LDS: segments of kTabSegC nodes, kTabSegS per superchunk, batches of
// kTabSegRows rows, workgroups of kTabSegThreads threads (at most one
// momentum per thread in a work item).
constexpr int kTabSegC = 2048;
constexpr int kTabSegS = 8;
constexpr int kTabSegRows = 4;
constexpr int kTabSegThreads = 1024;
constexpr int kTabSegMaxSuper = 1024;  // superchunks per row at most (rows of ~16.7M nodes)
// knob tab_seg = 2: the segmented form for tables larger than the chip's
// 256 MiB memory-side cache
constexpr double kTabSegAutoBytes = 256.0 * 1024 * 1024;
struct TabSegShape {
  int n_seg, n_super, n_batch;
  int target;  // work items per row batch aimed at
  int lds;     // dynamic LDS bytes of the main kernel
};
TabSegShape tab_seg_shape(const TabArgs &t, int n_cu);
// Device buffers of one launch: part n_super * n_rows * n_p doubles, terms
// n_p * n_r * n_a uint16, offs n_p * (n_seg + 1) ints, hist n_super
// unsigned, counter one int.
struct TabSegBufs {
  double *part;
  uint16_t *terms;
  int *offs;
  unsigned *hist;
  int *counter;
};
int launch_tab_seg(const TabArgs &t, const TabSegShape &s, const TabSegBufs &b, int n_cu,
                   void *stream);



// -------------------------------------------------------------- launchers --
// All return hipError_t as int (0 = success).
// Plain launch over one set (FP64 or FP32C by s.prec).
int launch_points_plain(const SetDev &s, int tile_points, int *d_flag, void *stream);
int launch_points_persistent(const SetDev *d_sets, const Tile *d_tiles, int n_tiles,
                             int *d_counters /* kCounters ints, zero */, int lds_bytes, int n_blocks, bool with_f32,
                             int *d_flag, void *stream);
int launch_reset_counter(int *d_counters /* kCounters ints */, void *stream);
int launch_grid(const GridArgs &g, int reg, int M, int W, void *stream);
// err[i] = 1e-14, used64[i] = 1 for i < n (either may be null): the marks of
// FP32C results evaluated in FP64.
int launch_fp64_marks(double *err, uint8_t *used64, int64_t n, void *stream);
// out[i] = e^{-y[i]} by the FP32C point path's exponential (exp_neg32).
int launch_expneg_fp32c(const double *y, double *out, int64_t n, void *stream);
int grid_lds_bytes(const GridArgs &g);
// Resident coefficient form of the FP64 grid kernel: used when its table fits.
constexpr int kGridCoefLdsMax = 150 * 1024;
// staged masses and masks of one workgroup: MB W (16 + 8 M) bytes, at most
constexpr int kGridCoefStageMax = 8192;
int grid_coef_group(const GridArgs &g);
int grid_coef_lds_bytes(const GridArgs &g);  // with the largest staging area
int grid_coef_stage_bytes(int MB, int W, int M);
void set_fold_scale(GridArgs &g, const QuadTable &h, int E = 2);
// Vertex diagram (vertex_kernel): group size from n_phi, LDS bytes of the
// resident coefficient table (0 if it does not fit), launch.
int vertex_group(int n_phi);
// Largest waves per workgroup of vertex_kernel for tiles of M masses and
// groups of G terms: 12 for the matrix-core form with G <= 16, 8 else.
constexpr int vertex_max_waves(int M, int G) { return M == 16 && G <= 16 ? 12 : 8; }
int vertex_lds_bytes(const GridArgs &g, int M, int W, bool table);
int launch_vertex(const GridArgs &g, int reg, int M, int W, void *stream);
std::vector<double> build_vertex_table(int d, int n_a, int n_phi);
// Whether the FP64 grid kernel keeps its table resident, and in which form.
bool grid_uses_coef(const GridArgs &g);
bool grid_resident(const GridArgs &g);
// stream_blocks: workgroups of the streamed-row form (rounded up to a multiple of 8)
int launch_tab(const TabArgs &t, int reg, int W, bool lds_rows, int64_t stream_blocks,
               void *stream);
int tab_lds_bytes(const TabArgs &t, bool lds_rows);
int launch_lpa(const LpaJob *d_jobs, const int64_t *d_start, int n_jobs, int64_t total_points,
               void *stream);

}  // namespace frg
