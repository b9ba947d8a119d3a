// Momentum-dependent two-point flow on gfx950: the right-hand side
//   d_t Sigma_r(p_a) = lam3_r^2 J_r(p_a) - lam4_r/2 T_r
// of n_rows flows at once, and the classical RK4 stages, all on the device.
// J is the tabulated-propagator diagram (tab_kernel) with the row
// g_r[a] = 1/(s_a + R_k(s_a) + Sigma_r[a]); T_r = C_d sum_i c_i G_r(q_i^2)^2
// is its radial part.  The quadrature table at scale k follows from the one
// at k = 1 (q_max = kappa k): q_i -> k q_i, c_i -> k^(d+2) c_i, Hq_i -> k^2 Hq_i.
#include <hip/hip_runtime.h>

#include <type_traits>

#include <cmath>

#include "frg_internal.h"

#pragma clang fp contract(off)

#include "device_fp64.h"
#include "device_tab.h"

namespace frg {

namespace {

using namespace dev;

// alive = 1, t_reached = t_end, p_a = sqrt(s_a), domain flag cleared.
__global__ __launch_bounds__(256) void pflow_init_kernel(PflowArgs a, double t_end) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e == 0) *a.flag = 0;
  if (e < a.n_rows) {
    a.alive[e] = 1;
    a.t_reached[e] = t_end;
  }
  if (e < a.n_s) a.p[e] = sqrt((double)e * a.h_s);
}

// Table row, domain check and tadpole of flow r at scale a.k for the state
// `state` (all threads of the workgroup; alive is workgroup-uniform).
template <int REG>
__device__ __forceinline__ void prep_row(const PflowArgs &a, int64_t r, const double *state,
                                         bool alive) {
  const int n_r = a.n_r;
  double *row = a.g + r * a.n_s;
  const double inv_k2 = 1.0 / a.k2;
  bool bad = false;
  for (int64_t i = threadIdx.x; i < a.n_s; i += blockDim.x) {
    const double s = (double)i * a.h_s;
    const double den = (hk<REG>(s, a.k2, inv_k2) + a.k2) + state[i];
    const bool ok = den > 0.0;
    bad |= !ok;
    row[i] = (alive && ok) ? 1.0 / den : 0.0;
  }
  bad = __syncthreads_or(bad) && alive;
  if (bad) {
    // the flow ends at the start of this step with its state kept
    for (int64_t i = threadIdx.x; i < a.n_s; i += blockDim.x) row[i] = 0.0;
    if (threadIdx.x == 0) {
      a.alive[r] = 0;
      a.t_reached[r] = a.t_n;
      *a.flag = 1;
    }
    __syncthreads();
  }
  if (threadIdx.x < kWave) {
    const int lane = threadIdx.x;
    double acc = 0.0;
    for (int i = lane; i < n_r; i += kWave) {
      const double q = a.k * a.base[i];
      const double c = a.kd2 * a.base[n_r + i];
      const double G = interp(row, (q * q) * a.inv_h, a.t_last, (int)a.n_s - 2);
      acc = __builtin_fma((c * G), G, acc);
    }
    acc = wave_sum(acc);
    if (lane == 0) a.T[r] = a.Cd * acc;
  }
}

// The quadrature table at scale a.k for tab_kernel (workgroup 0).
__device__ __forceinline__ void scale_table(const PflowArgs &a) {
  const int n_r = a.n_r, n_a = a.n_a;
  for (int i = threadIdx.x; i < n_r; i += blockDim.x) {
    a.tabk[i] = a.k * a.base[i];
    a.tabk[n_r + i] = a.kd2 * a.base[n_r + i];
    a.tabk[2 * n_r + i] = a.k2 * a.base[2 * n_r + i];
  }
  for (int j = threadIdx.x; j < 3 * n_a; j += blockDim.x) a.tabk[3 * n_r + j] = a.base[3 * n_r + j];
}

// One workgroup per flow: table row, domain check and tadpole of the first
// stage (state y0), and the quadrature table at scale k.
template <int REG>
__global__ __launch_bounds__(256) void pflow_prep_kernel(PflowArgs a) {
  const int64_t r = blockIdx.x;
  if (r == 0) scale_table(a);
  prep_row<REG>(a, r, a.y0 + r * a.n_s, a.alive[r] != 0);
}

// Flow r (all threads of the workgroup): right-hand side rhs = lam3^2 J - lam4/2 T of the
// stage just evaluated and its RK4 update (stage 0..3; 4: rhs only), then,
// if a.prep, the table row, domain check and tadpole of the next stage (at
// a.k, step start a.t_n; state ys after stages 0..2, y0 after stage 3).
template <int REG>
__device__ __forceinline__ void stage_row(const PflowArgs &a, int64_t r) {
  const int64_t ns = a.n_s;
  const bool alive = a.alive[r] != 0;  // workgroup-uniform
  if (alive) {
    const double l3 = a.lam3[r];
    const double c4 = 0.5 * a.lam4[r] * a.T[r];
    for (int64_t i = threadIdx.x; i < ns; i += blockDim.x) {
      const int64_t e = r * ns + i;
      const double rhs = l3 * l3 * a.J[i * a.n_rows + r] - c4;
      switch (a.stage) {
        case 0:
          a.acc[e] = rhs;
          a.ys[e] = a.y0[e] + (0.5 * a.h) * rhs;
          break;
        case 1:
          a.acc[e] += 2.0 * rhs;
          a.ys[e] = a.y0[e] + (0.5 * a.h) * rhs;
          break;
        case 2:
          a.acc[e] += 2.0 * rhs;
          a.ys[e] = a.y0[e] + a.h * rhs;
          break;
        case 3:
          a.y0[e] += (a.h / 6.0) * (a.acc[e] + rhs);
          break;
        default:
          a.dsdt[e] = rhs;
          break;
      }
    }
  } else if (a.stage == 4) {
    for (int64_t i = threadIdx.x; i < ns; i += blockDim.x) a.dsdt[r * ns + i] = __builtin_nan("");
  }
  if (!a.prep) return;  // kernel-uniform
  __syncthreads();      // the row's new state is complete
  if (r == 0) scale_table(a);
  prep_row<REG>(a, r, (a.stage == 3 ? a.y0 : a.ys) + r * ns, alive);
}

template <int REG>
__global__ __launch_bounds__(256) void pflow_stage_kernel(PflowArgs a) {
  stage_row<REG>(a, blockIdx.x);
}

// ---- one launch per stage -------------------------------------------------
// Launch m of a solve evaluates the diagram of RK4 stage m.  Each of its
// workgroups (RB rows, momentum block pb) first redoes, for each whole row,
// the update that the stage kernel would do after stage m - 1 (from J, T, the
// accumulator and the step-start state of the previous launch), then the prep
// of stage m, with the propagator rows built in LDS.  Every workgroup of a row
// computes the same values; only the one with pb = 0 stores the new state,
// tadpole and flags, into buffers that no workgroup of the launch reads
// (read and written state alternate between launches), so a launch needs no
// communication between workgroups.  Same arithmetic, in the same order, as
// pflow_stage_kernel + prep_row + tab_kernel: the same bits.

// State of stage m at node i of row r (the previous stage's update): the
// state itself for the first launch; for a flow that has stopped, its
// step-start state (carried into the new step-start buffer after stage 3).
__device__ __forceinline__ double pull_state(const PflowPull &a, int64_t r, int64_t i, bool alive,
                                             double l3, double c4, bool writer) {
  const int64_t e = r * a.n_s + i;
  if (a.prev < 0) return a.y0p[e];
  if (!alive) {
    const double y = a.y0p[e];
    if (a.prev == 3 && writer) a.y0n[e] = y;
    return y;
  }
  const double rhs = l3 * l3 * a.Jp[e] - c4;
  switch (a.prev) {
    case 0:
      if (writer) a.accn[e] = rhs;
      return a.y0p[e] + (0.5 * a.h) * rhs;
    case 1:
      if (writer) a.accn[e] = a.accp[e] + 2.0 * rhs;
      return a.y0p[e] + (0.5 * a.h) * rhs;
    case 2:
      if (writer) a.accn[e] = a.accp[e] + 2.0 * rhs;
      return a.y0p[e] + a.h * rhs;
    default: {
      const double y = a.y0p[e] + (a.h / 6.0) * (a.accp[e] + rhs);
      if (writer) a.y0n[e] = y;
      return y;
    }
  }
}

// t: the diagram at scale a.k (t.tab = the table at k = 1, t.out = a.Jn,
// J[r * n_s + a]).  RB flows (rows) per workgroup, flows rg RB .. rg RB +
// nrb - 1: each flow's update and row as for one flow; the diagram of the
// rows shares every coordinate (tab_block_rows: each row's sums as alone).
// LDS: tab_lds's layout for RB rows, then (pairs) the rows as plain values.
template <int REG, int UR, bool PAIRS, int RB>
__global__ __launch_bounds__(RB > 1 ? 1024 : 256) void pflow_pull_kernel(TabArgs t, PflowPull a) {
  extern __shared__ double lds[];
  const int W = blockDim.x / kWave;
  const int wave = threadIdx.x / kWave;
  const int lane = threadIdx.x & (kWave - 1);
  const int n_r = a.n_r;
  const int n_s = (int)a.n_s;
  const int64_t rg = blockIdx.x / t.n_pb;
  const int64_t pb = blockIdx.x - rg * t.n_pb;
  const int64_t r0 = rg * RB;
  const int nrb = (int)min<int64_t>(RB, a.n_rows - r0);
  const bool writer = pb == 0;
  const TabLds l = tab_lds(t, lds, RB);
  const int len = PAIRS ? 2 * n_s : n_s;  // doubles of one staged row
  // the rows as plain values: after the pair rows, or the staged rows
  double *lv0 = PAIRS ? l.lg + RB * len : l.lg;
  const double inv_k2 = 1.0 / a.k2;
  for (int rr = 0; rr < nrb; ++rr) {
    const int64_t r = r0 + rr;
    double *lv = lv0 + rr * n_s;
    // update of the previous stage and the row of this one
    const bool alive = a.alivep[r] != 0;  // workgroup-uniform
    double l3 = 0.0, c4 = 0.0;
    if (alive && a.prev >= 0) {
      l3 = a.lam3[r];
      c4 = 0.5 * a.lam4[r] * a.Tp[r];
    }
    bool bad = false;
    for (int i = threadIdx.x; i < n_s; i += blockDim.x) {
      const double y = pull_state(a, r, i, alive, l3, c4, writer);
      const double s = (double)i * a.h_s;
      const double den = (hk<REG>(s, a.k2, inv_k2) + a.k2) + y;
      const bool ok = den > 0.0;
      bad |= !ok;
      lv[i] = (alive && ok) ? 1.0 / den : 0.0;
    }
    bad = __syncthreads_or(bad) && alive;
    if (bad) {
      // the flow ends at the start of this step with its state kept
      for (int i = threadIdx.x; i < n_s; i += blockDim.x) lv[i] = 0.0;
      if (writer && threadIdx.x == 0) {
        a.t_reached[r] = a.t_n;
        *a.flag = 1;
      }
      __syncthreads();
    }
    if (writer && threadIdx.x == 0) a.aliven[r] = alive && !bad;
    // the diagram's row as tab_rows_block stages it
    if constexpr (PAIRS) {
      double2 *lp = reinterpret_cast<double2 *>(l.lg) + rr * n_s;
      for (int k = threadIdx.x; k < n_s; k += blockDim.x) lp[k] = row_pair(lv, k, n_s);
    }
  }
  __syncthreads();
  using Row = typename std::conditional<PAIRS, PairRow, PlainRow>::type;
  const double2 *lp = reinterpret_cast<const double2 *>(l.lg);
  Row rows[RB];
#pragma unroll
  for (int rr = 0; rr < RB; ++rr) {
    const int rs = rr < nrb ? rr : nrb - 1;
    if constexpr (PAIRS)
      rows[rr] = PairRow{lp + rs * n_s};
    else
      rows[rr] = PlainRow{l.lg + rs * n_s};
  }
  // q_i and A_i of each row at scale k
  for (int x = threadIdx.x; x < nrb * n_r; x += blockDim.x) {
    const int rr = x / n_r, i = x - rr * n_r;
    const double q = a.k * a.base[i];
    double G;
    if constexpr (PAIRS)
      G = PairRow{lp + rr * n_s}((q * q) * t.inv_h, t.t_last, n_s - 2);
    else
      G = PlainRow{l.lg + rr * n_s}((q * q) * t.inv_h, t.t_last, n_s - 2);
    if (rr == 0) l.lrad[i * (1 + RB)] = q;
    l.lrad[i * (1 + RB) + 1 + rr] = ((a.kd2 * a.base[n_r + i]) * G) * G;
  }
  __syncthreads();
  tab_block_rows<UR, RB>(t, rows, nrb, l.lrad, l.lo, l.lm, r0, pb, W, wave, lane);
  // tadpole of this stage of each flow, as prep_row (wave 0 of the storing
  // workgroup)
  if (writer && threadIdx.x < kWave) {
    for (int rr = 0; rr < nrb; ++rr) {
      const double *lv = lv0 + rr * n_s;
      double acc = 0.0;
      for (int i = lane; i < n_r; i += kWave) {
        const double q = a.k * a.base[i];
        const double c = a.kd2 * a.base[n_r + i];
        const double G = interp(lv, (q * q) * a.inv_h, a.t_last, n_s - 2);
        acc = __builtin_fma((c * G), G, acc);
      }
      acc = wave_sum(acc);
      if (lane == 0) a.Tn[r0 + rr] = a.Cd * acc;
    }
  }
}

// The update after the last launch: the final state (a.prev = 3, a.y0n the
// caller's state) or the right-hand side (a.prev = 4: dsdt, NaN rows for
// flows outside the domain).  One workgroup per flow.
__global__ __launch_bounds__(256) void pflow_final_kernel(PflowPull a) {
  const int64_t r = blockIdx.x;
  const bool alive = a.alivep[r] != 0;
  double l3 = 0.0, c4 = 0.0;
  if (alive) {
    l3 = a.lam3[r];
    c4 = 0.5 * a.lam4[r] * a.Tp[r];
  }
  for (int64_t i = threadIdx.x; i < a.n_s; i += blockDim.x) {
    if (a.prev == 4)
      a.dsdt[r * a.n_s + i] = alive ? l3 * l3 * a.Jp[r * a.n_s + i] - c4 : __builtin_nan("");
    else
      (void)pull_state(a, r, i, alive, l3, c4, true);
  }
}
}  // namespace

int launch_pflow_init(const PflowArgs &a, double t_end, void *stream) {
  const int64_t n = a.n_rows > a.n_s ? a.n_rows : a.n_s;
  if (n <= 0) return 0;
  hipLaunchKernelGGL(pflow_init_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0,
                     (hipStream_t)stream, a, t_end);
  return (int)hipGetLastError();
}

int launch_pflow_prep(const PflowArgs &a, int reg, void *stream) {
  if (a.n_rows <= 0) return 0;
  if (reg == kExp)
    hipLaunchKernelGGL(pflow_prep_kernel<kExp>, dim3((unsigned)a.n_rows), dim3(256), 0,
                       (hipStream_t)stream, a);
  else
    hipLaunchKernelGGL(pflow_prep_kernel<kLitim>, dim3((unsigned)a.n_rows), dim3(256), 0,
                       (hipStream_t)stream, a);
  return (int)hipGetLastError();
}

int launch_pflow_stage(const PflowArgs &a, int reg, void *stream) {
  if (a.n_rows <= 0) return 0;
  if (reg == kExp)
    hipLaunchKernelGGL(pflow_stage_kernel<kExp>, dim3((unsigned)a.n_rows), dim3(256), 0,
                       (hipStream_t)stream, a);
  else
    hipLaunchKernelGGL(pflow_stage_kernel<kLitim>, dim3((unsigned)a.n_rows), dim3(256), 0,
                       (hipStream_t)stream, a);
  return (int)hipGetLastError();
}

int pflow_pull_lds_bytes(const TabArgs &t) {
  const int rb = t.rb > 1 ? t.rb : 1;
  return tab_lds_bytes(t, true) + (t.pairs ? (int)(sizeof(double) * rb * t.n_s) : 0);
}

// Dynamic LDS beyond 64 KiB (gfx950: 160 KiB per workgroup); a refusal where
// no opt-in is needed is cleared so that it cannot be taken for a launch error.
template <int REG, int UR, bool P, int RB>
static void pflow_pull_t(const TabArgs &t, const PflowPull &a, int W, hipStream_t st) {
  static const bool once = [] {
    (void)hipFuncSetAttribute((const void *)&pflow_pull_kernel<REG, UR, P, RB>,
                              hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    (void)hipGetLastError();
    return true;
  }();
  (void)once;
  const int64_t groups = (t.n_rows + RB - 1) / RB;
  hipLaunchKernelGGL((pflow_pull_kernel<REG, UR, P, RB>), dim3((unsigned)(groups * t.n_pb)),
                     dim3(kWave * W), pflow_pull_lds_bytes(t), st, t, a);
}

template <int REG, int RB>
static void pflow_pull_rows(const TabArgs &t, const PflowPull &a, int W, hipStream_t st) {
  const bool regs = t.U <= 4;
  if (t.pairs)
    regs ? pflow_pull_t<REG, 4, true, RB>(t, a, W, st) : pflow_pull_t<REG, 0, true, RB>(t, a, W, st);
  else
    regs ? pflow_pull_t<REG, 4, false, RB>(t, a, W, st) : pflow_pull_t<REG, 0, false, RB>(t, a, W, st);
}

template <int REG>
static void pflow_pull_reg(const TabArgs &t, const PflowPull &a, int W, hipStream_t st) {
  if (t.rb == 4)
    pflow_pull_rows<REG, 4>(t, a, W, st);
  else if (t.rb == 2)
    pflow_pull_rows<REG, 2>(t, a, W, st);
  else
    pflow_pull_rows<REG, 1>(t, a, W, st);
}

int launch_pflow_pull(const TabArgs &t, const PflowPull &a, int reg, int W, void *stream) {
  if (t.n_p <= 0 || t.n_rows <= 0) return 0;
  // RB rows per workgroup of at most 256 threads (one row) or 1024 (several),
  // the kernel's launch bounds
  const int rb = t.rb > 1 ? t.rb : 1;
  if (rb != 1 && rb != 2 && rb != 4) return (int)hipErrorInvalidValue;
  if (W < 1 || W * kWave > (rb > 1 ? 1024 : 256)) return (int)hipErrorInvalidValue;
  hipStream_t st = (hipStream_t)stream;
  if (reg == kExp)
    pflow_pull_reg<kExp>(t, a, W, st);
  else
    pflow_pull_reg<kLitim>(t, a, W, st);
  return (int)hipGetLastError();
}

int launch_pflow_final(const PflowPull &a, void *stream) {
  if (a.n_rows <= 0) return 0;
  hipLaunchKernelGGL(pflow_final_kernel, dim3((unsigned)a.n_rows), dim3(256), 0,
                     (hipStream_t)stream, a);
  return (int)hipGetLastError();
}

}  // namespace frg
