// Piecewise-linear propagator tables (tabulated-propagator variant and the
// momentum-dependent flow built on it).
#pragma once

#include <hip/hip_runtime.h>

#include "device_fp64.h"
#include "frg_internal.h"

#pragma clang fp contract(off)

namespace frg {
namespace dev {

// Interpolated propagator of one row at table coordinate t = s / h (t >= 0):
// nodes k and k + 1 with f = t - k, and the last node beyond t_last = n_s - 1
// (k_last = n_s - 2).
__device__ __forceinline__ double interp(const double *__restrict__ row, double t, double t_last,
                                         int k_last) {
  t = fmin(t, t_last);
  int k = (int)t;
  k = k < k_last ? k : k_last;
  const double f = t - (double)k;
  const double g0 = row[k], g1 = row[k + 1];
  return __builtin_fma(f, g1 - g0, g0);
}

// A table row as plain values g_k (rows read from memory, or staged in LDS
// as they are) or as pairs (g_k, g_{k+1} - g_k) (rows staged in LDS): one
// 16-byte read per evaluation; both give the same bits.  locate(t, k, f)
// splits a clamped coordinate t <= t_last = n_s - 1 into a node and a
// fraction, fetch(k) = (g_k, g_{k+1} - g_k), and the value is
// g_k + f (g_{k+1} - g_k).  Plain rows clamp k to n_s - 2 (f = 1 at t_last);
// pair rows append the node (g_{n_s-2} + (g_{n_s-1} - g_{n_s-2}), 0), the
// value of that same expression, so they need no clamp: k = floor(t),
// f = t - k (exact).
struct PlainRow {
  const double *g;
  __device__ __forceinline__ double operator()(double t, double t_last, int k_last) const {
    return interp(g, t, t_last, k_last);
  }
  __device__ __forceinline__ void locate(double t, int k_last, int &k, double &f) const {
    const int kk = (int)t;
    k = kk < k_last ? kk : k_last;
    f = t - (double)k;
  }
  __device__ __forceinline__ double2 fetch(int k) const {
    const double g0 = g[k], g1 = g[k + 1];
    return make_double2(g0, g1 - g0);
  }
};
struct PairRow {
  const double2 *p;
  __device__ __forceinline__ double operator()(double t, double t_last, int) const {
    t = fmin(t, t_last);
    const double2 gd = p[(int)t];
    return __builtin_fma(__builtin_amdgcn_fract(t), gd.y, gd.x);
  }
  __device__ __forceinline__ void locate(double t, int, int &k, double &f) const {
    k = (int)t;                       // t >= 0: floor
    f = __builtin_amdgcn_fract(t);    // t - floor(t), exact
  }
  __device__ __forceinline__ double2 fetch(int k) const { return p[k]; }
};

// One (row, momentum block) of work: A_i of the row, then W * pw momenta.
// lq / lo / lm are staged; `row` is the LDS copy or the row in memory.
template <int UR, class Row>
__device__ __forceinline__ void tab_block(const TabArgs &a, const Row row, const double *lq,
                                          const double *lA, const double *lo, const double *lm,
                                          int64_t r, int64_t pb, int W, int wave, int lane) {
  const int n_a = a.n_a, n_r = a.n_r;
  const int k_last = (int)a.n_s - 2;
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
          // all table indices first, then all reads, then the sums (the
          // reads of the UR terms are in flight together)
          int kq[UR > 0 ? UR : 1];
          double fq[UR > 0 ? UR : 1];
#pragma unroll
          for (int u = 0; u < UR; ++u)
            row.locate(fmin(__builtin_fma(bh, ro[u], ah), a.t_last), k_last, kq[u], fq[u]);
          double2 gd[UR > 0 ? UR : 1];
#pragma unroll
          for (int u = 0; u < UR; ++u) gd[u] = row.fetch(kq[u]);
#pragma unroll
          for (int u = 0; u < UR; ++u)
            inner = __builtin_fma(rm[u], __builtin_fma(fq[u], gd[u].y, gd[u].x), inner);
        } else {
          for (int u = 0; u < a.U; ++u) {
            const int j = iota + a.J * u;
            if (j < n_a) {
              const double G = row(__builtin_fma(bh, lo[j], ah), a.t_last, k_last);
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
  if (lane < a.pw && ia < a.n_p) a.out[ia * a.os_p + r * a.os_r] = res;
}

// Stage the row-dependent factors A_i = c_i G_r(q_i^2)^2 (and q_i).
template <class Row>
__device__ __forceinline__ void tab_stage_A(const TabArgs &a, const Row row, double *lq,
                                            double *lA) {
  for (int i = threadIdx.x; i < a.n_r; i += blockDim.x) {
    const double q = a.tab[i];
    const double G = row((q * q) * a.inv_h, a.t_last, (int)a.n_s - 2);
    lq[i] = q;
    lA[i] = (a.tab[a.n_r + i] * G) * G;
  }
}


// LDS of the table kernels: q_i | A_i | 1 + x_j | mu_j | the row (rows
// staged in LDS: values, or (value, slope) pairs).  tab_lds also stages
// 1 + x_j and mu_j (all threads of the workgroup).
struct TabLds {
  double *lq, *lA, *lo, *lm, *lg;
};
__device__ __forceinline__ TabLds tab_lds(const TabArgs &a, double *lds) {
  const int n_r = a.n_r, n_a = a.n_a;
  TabLds l;
  l.lq = lds;
  l.lA = l.lq + n_r;
  l.lo = l.lA + n_r;
  l.lm = l.lo + n_a;
  l.lg = l.lm + n_a;
  for (int j = threadIdx.x; j < n_a; j += blockDim.x) {
    l.lo[j] = a.tab[3 * n_r + j];
    l.lm[j] = a.tab[3 * n_r + n_a + j];
  }
  return l;
}

// One (row, momentum block) with the row staged in LDS: the whole workgroup
// stages the row and the A_i, then each wave evaluates its momenta.
template <int UR, bool PAIRS>
__device__ __forceinline__ void tab_row_block(const TabArgs &a, const TabLds &l, int64_t r,
                                              int64_t pb, int W, int wave, int lane) {
  const double *grow = a.g + r * a.n_s;
  if constexpr (PAIRS) {
    double2 *lp = reinterpret_cast<double2 *>(l.lg);
    const int n_s = (int)a.n_s;
    for (int k = threadIdx.x; k < n_s; k += blockDim.x) {
      if (k + 1 < n_s) {
        const double g0 = grow[k];
        lp[k] = make_double2(g0, grow[k + 1] - g0);
      } else {
        const double g0 = grow[n_s - 2];
        lp[k] = make_double2(__builtin_fma(1.0, grow[n_s - 1] - g0, g0), 0.0);
      }
    }
    __syncthreads();
    const PairRow row{lp};
    tab_stage_A(a, row, l.lq, l.lA);
    __syncthreads();
    tab_block<UR>(a, row, l.lq, l.lA, l.lo, l.lm, r, pb, W, wave, lane);
  } else {
    for (int k = threadIdx.x; k < (int)a.n_s; k += blockDim.x) l.lg[k] = grow[k];
    __syncthreads();
    const PlainRow row{l.lg};
    tab_stage_A(a, row, l.lq, l.lA);
    __syncthreads();
    tab_block<UR>(a, row, l.lq, l.lA, l.lo, l.lm, r, pb, W, wave, lane);
  }
}

}  // namespace dev
}  // namespace frg
