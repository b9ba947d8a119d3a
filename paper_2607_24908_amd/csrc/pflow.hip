// Momentum-dependent two-point flow on gfx950: the right-hand side
//   d_t Sigma_r(p_a) = lam3_r^2 J_r(p_a) - lam4_r/2 T_r
// of n_rows flows at once, and the classical RK4 stages, all on the device.
// J is the tabulated-propagator diagram (tab_kernel) with the row
// g_r[a] = 1/(s_a + R_k(s_a) + Sigma_r[a]); T_r = C_d sum_i c_i G_r(q_i^2)^2
// is its radial part.  The quadrature table at scale k follows from the one
// at k = 1 (q_max = kappa k): q_i -> k q_i, c_i -> k^(d+2) c_i, Hq_i -> k^2 Hq_i.
#include <hip/hip_runtime.h>

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

// One workgroup per flow: right-hand side rhs = lam3^2 J - lam4/2 T of the
// stage just evaluated and its RK4 update (stage 0..3; 4: rhs only), then,
// if a.prep, the table row, domain check and tadpole of the next stage (at
// a.k, step start a.t_n; state ys after stages 0..2, y0 after stage 3).
template <int REG>
__global__ __launch_bounds__(256) void pflow_stage_kernel(PflowArgs a) {
  const int64_t r = blockIdx.x;
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

}  // namespace frg
