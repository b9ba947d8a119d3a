// Tabulated-propagator flow diagram (gfx950): the propagator comes from a
// caller's table (one row per field value, piecewise-linear in s = q^2), the
// regulator insertion d_tR from the quadrature table.  A workgroup owns one
// table row and W * pw momenta; each wave evaluates its momenta one after
// another with the 64 lanes over the quadrature nodes (up to 8 angular lanes
// per radial node, so that neighbouring lanes read neighbouring table
// entries) and stores them together.  Rows of up to tab_lds_max_nodes nodes are staged in LDS;
// longer rows are read through the caches, with the workgroups of one row
// placed on one XCD.  Both forms do the same arithmetic in the same order.
#include <hip/hip_runtime.h>

#include <cmath>

#include "frg_internal.h"

#pragma clang fp contract(off)

#include "device_fp64.h"

namespace frg {

namespace {

using namespace dev;

// Interpolated propagator of one row at table coordinate t = s / h (t >= 0).
__device__ __forceinline__ double interp(const double *__restrict__ row, double t, double t_last,
                                         int k_last) {
  t = fmin(t, t_last);
  int k = (int)t;
  k = k < k_last ? k : k_last;
  const double f = t - (double)k;
  const double g0 = row[k], g1 = row[k + 1];
  return __builtin_fma(f, g1 - g0, g0);
}

// Block -> (row, momentum block), such that the blocks the hardware sends to
// one XCD (b mod 8) are consecutive in (row, block) order.
__device__ __forceinline__ int64_t xcd_order(int64_t b, int64_t total) {
  const int64_t x = b & 7, q = total >> 3, rem = total & 7;
  return x * q + (x < rem ? x : rem) + (b >> 3);
}

// UR > 0: every lane holds at most UR angular nodes (U <= UR), kept in
// registers; UR == 0: read from LDS.
template <bool LDS_ROW, int UR>
__global__ __launch_bounds__(256) void tab_kernel(TabArgs a) {
  extern __shared__ double lds[];
  const int W = blockDim.x / kWave;
  const int wave = threadIdx.x / kWave;
  const int lane = threadIdx.x & (kWave - 1);
  const int64_t total = a.n_rows * a.n_pb;
  const int64_t ord = LDS_ROW ? (int64_t)blockIdx.x : xcd_order(blockIdx.x, total);
  const int64_t r = ord / a.n_pb;
  const int64_t pb = ord - r * a.n_pb;
  const int n_r = a.n_r, n_a = a.n_a;
  const int k_last = (int)a.n_s - 2;
  double *lq = lds;           // q_i
  double *lA = lq + n_r;      // c_i G_r(q_i^2)^2
  double *lo = lA + n_r;      // 1 + x_j
  double *lm = lo + n_a;      // mu_j
  double *lg = lm + n_a;      // the row (LDS_ROW)
  const double *grow = a.g + r * a.n_s;
  if (LDS_ROW)
    for (int k = threadIdx.x; k < (int)a.n_s; k += blockDim.x) lg[k] = grow[k];
  for (int j = threadIdx.x; j < n_a; j += blockDim.x) {
    lo[j] = a.tab[3 * n_r + j];
    lm[j] = a.tab[3 * n_r + n_a + j];
  }
  __syncthreads();
  const double *row = LDS_ROW ? lg : grow;
  for (int i = threadIdx.x; i < n_r; i += blockDim.x) {
    const double q = a.tab[i];
    const double G = interp(row, (q * q) * a.inv_h, a.t_last, k_last);
    lq[i] = q;
    lA[i] = (a.tab[n_r + i] * G) * G;
  }
  __syncthreads();
  const int rho = lane & (a.R - 1);
  const int iota = lane / a.R;
  // this lane's angular nodes j = iota + J u (padded ones get mu = 0)
  double ro[UR > 0 ? UR : 1], rm[UR > 0 ? UR : 1];
  if (UR > 0) {
#pragma unroll
    for (int u = 0; u < UR; ++u) {
      const int j = iota + a.J * u;
      const bool vj = u < a.U && j < n_a;
      ro[u] = vj ? lo[j] : 1.0;
      rm[u] = vj ? lm[j] : 0.0;
    }
  }
  const int64_t p0 = (pb * W + wave) * a.pw;
  double res = 0.0;
  for (int e = 0; e < a.pw; ++e) {
    const int64_t ia = p0 + e;
    if (ia >= a.n_p) break;  // wave-uniform
    const double p = a.p[ia];
    double total_l = 0.0;
    if (p >= 0.0) {
      for (int t = 0; t < a.T; ++t) {
        const int i = rho + a.R * t;
        const bool vi = i < n_r;
        const double q = vi ? lq[i] : 0.0;
        const double A = vi ? lA[i] : 0.0;
        const double qm = q - p;
        const double ah = (qm * qm) * a.inv_h;
        const double bh = ((2.0 * q) * p) * a.inv_h;
        double inner = 0.0;
        if (UR > 0) {
#pragma unroll
          for (int u = 0; u < UR; ++u) {
            const double G = interp(row, __builtin_fma(bh, ro[u], ah), a.t_last, k_last);
            inner = __builtin_fma(rm[u], G, inner);
          }
        } else {
          for (int u = 0; u < a.U; ++u) {
            const int j = iota + a.J * u;
            if (j < n_a) {
              const double G = interp(row, __builtin_fma(bh, lo[j], ah), a.t_last, k_last);
              inner = __builtin_fma(lm[j], G, inner);
            }
          }
        }
        total_l = __builtin_fma(A, inner, total_l);
      }
    }
    const double v = a.pref * wave_sum(total_l);
    if (lane == e) res = p >= 0.0 ? v : __builtin_nan("");
    if (!(p >= 0.0) && lane == 0) *a.flag = 1;
  }
  const int64_t ia = p0 + lane;
  if (lane < a.pw && ia < a.n_p) a.out[ia * a.n_rows + r] = res;
}

}  // namespace

void tab_lane_split(int n_r, int n_a, int *R, int *J, int *T, int *U) {
  int j = 1;
  while (j * 2 <= n_a && j * 2 <= 8) j *= 2;
  *J = j;
  *R = kWave / j;
  *T = (n_r + *R - 1) / *R;
  *U = (n_a + j - 1) / j;
}

int tab_lds_bytes(const TabArgs &t, bool lds_rows) {
  return (int)(sizeof(double) * (2 * t.n_r + 2 * t.n_a + (lds_rows ? t.n_s : 0)));
}

template <bool L, int UR>
static void tab_launch_t(const TabArgs &t, int W, hipStream_t st) {
  const int64_t blocks = t.n_rows * t.n_pb;
  hipLaunchKernelGGL((tab_kernel<L, UR>), dim3((unsigned)blocks), dim3(kWave * W),
                     tab_lds_bytes(t, L), st, t);
}

int launch_tab(const TabArgs &t, int reg, int W, bool lds_rows, void *stream) {
  (void)reg;  // the regulator enters through the quadrature table only
  if (t.n_p <= 0 || t.n_rows <= 0) return 0;
  hipStream_t st = (hipStream_t)stream;
  const bool regs = t.U <= 4;
  if (lds_rows)
    regs ? tab_launch_t<true, 4>(t, W, st) : tab_launch_t<true, 0>(t, W, st);
  else
    regs ? tab_launch_t<false, 4>(t, W, st) : tab_launch_t<false, 0>(t, W, st);
  return (int)hipGetLastError();
}

}  // namespace frg
