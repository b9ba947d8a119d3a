// Piecewise-linear propagator tables (tabulated-propagator variant and the
// momentum-dependent flow built on it).
#pragma once

#include <hip/hip_runtime.h>

#include <type_traits>

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

// Pair k of a staged row: g_k and g_{k+1} - g_k, the last node
// (g_{n_s-2} + (g_{n_s-1} - g_{n_s-2}), 0); g is the row's plain values.
__device__ __forceinline__ double2 row_pair(const double *g, int k, int n_s) {
  if (k + 1 < n_s) {
    const double g0 = g[k];
    return make_double2(g0, g[k + 1] - g0);
  }
  const double g0 = g[n_s - 2];
  return make_double2(__builtin_fma(1.0, g[n_s - 1] - g0, g0), 0.0);
}

// Radial slots of the lane split: lane rho takes i = rho + R t (t < T), so
// q_i and A_i are staged for R T slots, the ones past n_r holding zeros (the
// values a guarded read would give), and the loop reads them unguarded.  A
// slot holds q_i then A_i of each of the rb rows staged together (stride
// 1 + rb doubles), so one address serves all of them.
__host__ __device__ __forceinline__ int tab_radial_slots(const TabArgs &a) { return a.R * a.T; }

// RB rows and one momentum block of work: A_i of the rows, then W * pw
// momenta.  rows[r] (r < nrb) are the rows (the others alias one of them and
// are not stored); lrad holds the radial slots (q_i, then
// A_i of rows 0 .. RB - 1); lo / lm are staged.  The rows share the lane's coordinates and node
// indices; the sum of every row is that of the row alone (same lanes, same
// order).
template <int UR, int RB, class Row>
__device__ __forceinline__ void tab_block_rows(const TabArgs &a, const Row *rows, int nrb,
                                               const double *lrad,
                                               const double *lo, const double *lm, int64_t r0,
                                               int64_t pb, int W, int wave, int lane) {
  constexpr int S = 1 + RB;  // doubles of a radial slot
  const int n_a = a.n_a;
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
  double res[RB];
#pragma unroll
  for (int r = 0; r < RB; ++r) res[r] = 0.0;
  for (int e = 0; e < a.pw; ++e) {
    const int64_t ia = p0 + e;
    if (ia >= a.n_p) break;  // wave-uniform
    const double p = a.p[ia];
    double total_l[RB];
#pragma unroll
    for (int r = 0; r < RB; ++r) total_l[r] = 0.0;
    if (p >= 0.0) {
      for (int t = 0; t < a.T; ++t) {
        const int i = rho + a.R * t;  // < R T: slots past n_r hold q = A = 0
        const double *slot = lrad + i * S;
        const double q = slot[0];
        double A[RB];
#pragma unroll
        for (int r = 0; r < RB; ++r) A[r] = slot[1 + r];
        const double qm = q - p;
        const double ah = (qm * qm) * a.inv_h;
        const double bh = ((2.0 * q) * p) * a.inv_h;
        double inner[RB];
#pragma unroll
        for (int r = 0; r < RB; ++r) inner[r] = 0.0;
        if (UR > 0) {
          // all table indices first, then each row's reads (the reads of its
          // UR terms in flight together), then its sums
          int kq[UR > 0 ? UR : 1];
          double fq[UR > 0 ? UR : 1];
#pragma unroll
          for (int u = 0; u < UR; ++u)
            rows[0].locate(fmin(__builtin_fma(bh, ro[u], ah), a.t_last), k_last, kq[u], fq[u]);
#pragma unroll
          for (int r = 0; r < RB; ++r) {
            double2 gd[UR > 0 ? UR : 1];
#pragma unroll
            for (int u = 0; u < UR; ++u) gd[u] = rows[r].fetch(kq[u]);
#pragma unroll
            for (int u = 0; u < UR; ++u)
              inner[r] = __builtin_fma(rm[u], __builtin_fma(fq[u], gd[u].y, gd[u].x), inner[r]);
          }
        } else {
          for (int u = 0; u < a.U; ++u) {
            const int j = iota + a.J * u;
            if (j < n_a) {
              const double tc = __builtin_fma(bh, lo[j], ah);
#pragma unroll
              for (int r = 0; r < RB; ++r)
                inner[r] = __builtin_fma(lm[j], rows[r](tc, a.t_last, k_last), inner[r]);
            }
          }
        }
#pragma unroll
        for (int r = 0; r < RB; ++r) total_l[r] = __builtin_fma(A[r], inner[r], total_l[r]);
      }
    }
#pragma unroll
    for (int r = 0; r < RB; ++r) {
      const double v = a.pref * wave_sum(total_l[r]);
      if (lane == e) res[r] = p >= 0.0 ? v : __builtin_nan("");
    }
    if (!(p >= 0.0) && lane == 0) *a.flag = 1;
  }
  const int64_t ia = p0 + lane;
  if (lane < a.pw && ia < a.n_p) {
#pragma unroll
    for (int r = 0; r < RB; ++r)
      if (r < nrb) a.out[ia * a.os_p + (r0 + r) * a.os_r] = res[r];
  }
}

// One (row, momentum block) of work: tab_block_rows with one row.
template <int UR, class Row>
__device__ __forceinline__ void tab_block(const TabArgs &a, const Row row, const double *lrad,
                                          const double *lo, const double *lm,
                                          int64_t r, int64_t pb, int W, int wave, int lane) {
  tab_block_rows<UR, 1>(a, &row, 1, lrad, lo, lm, r, pb, W, wave, lane);
}

// Stage the row-dependent factors A_i = c_i G_r(q_i^2)^2 and q_i of one row
// (radial slots of two doubles).
template <class Row>
__device__ __forceinline__ void tab_stage_A(const TabArgs &a, const Row row, double *lrad) {
  for (int i = threadIdx.x; i < a.n_r; i += blockDim.x) {
    const double q = a.tab[i];
    const double G = row((q * q) * a.inv_h, a.t_last, (int)a.n_s - 2);
    lrad[2 * i] = q;
    lrad[2 * i + 1] = (a.tab[a.n_r + i] * G) * G;
  }
}


// LDS of the table kernels: radial slots (q_i, A_i of rb rows) | 1 + x_j |
// mu_j | the rows (rows staged in LDS: values, or (value, slope) pairs).  tab_lds also stages 1 + x_j and mu_j and zeroes the slots past n_r
// (all threads of the workgroup), which the staging of q_i and A_i never
// writes.
struct TabLds {
  double *lrad, *lo, *lm, *lg;
};
__device__ __forceinline__ TabLds tab_lds(const TabArgs &a, double *lds, int rb = 1) {
  const int n_r = a.n_r, n_a = a.n_a, n_rp = tab_radial_slots(a);
  TabLds l;
  l.lrad = lds;
  l.lo = l.lrad + (1 + rb) * n_rp;
  l.lm = l.lo + n_a;
  l.lg = l.lm + n_a;
  for (int j = threadIdx.x; j < n_a; j += blockDim.x) {
    l.lo[j] = a.tab[3 * n_r + j];
    l.lm[j] = a.tab[3 * n_r + n_a + j];
  }
  for (int x = (1 + rb) * n_r + threadIdx.x; x < (1 + rb) * n_rp; x += blockDim.x)
    l.lrad[x] = 0.0;
  return l;
}

// RB rows (group rg) and one momentum block with the rows staged in LDS: the
// whole workgroup stages the rows and their A_i, then each wave evaluates its
// momenta for all of them.
template <int UR, bool PAIRS, int RB>
__device__ __forceinline__ void tab_rows_block(const TabArgs &a, const TabLds &l, int64_t rg,
                                               int64_t pb, int W, int wave, int lane) {
  const int64_t r0 = rg * RB;
  const int nrb = (int)min<int64_t>(RB, a.n_rows - r0);
  const int n_s = (int)a.n_s, n_r = a.n_r;
  // the rows one after another (pairs: n_s double2 each)
  double2 *lp = reinterpret_cast<double2 *>(l.lg);
  for (int r = 0; r < nrb; ++r) {
    const double *grow = a.g + (r0 + r) * a.n_s;
    if constexpr (PAIRS) {
      for (int k = threadIdx.x; k < n_s; k += blockDim.x) lp[r * n_s + k] = row_pair(grow, k, n_s);
    } else {
      double *dst = l.lg + r * n_s;
      for (int k = threadIdx.x; k < n_s; k += blockDim.x) dst[k] = grow[k];
    }
  }
  __syncthreads();
  using Row = typename std::conditional<PAIRS, PairRow, PlainRow>::type;
  Row rows[RB];
#pragma unroll
  for (int r = 0; r < RB; ++r) {
    const int rs = r < nrb ? r : nrb - 1;
    if constexpr (PAIRS)
      rows[r] = PairRow{lp + rs * n_s};
    else
      rows[r] = PlainRow{l.lg + rs * n_s};
  }
  // A_i = c_i G_r(q_i^2)^2 of each row (and q_i)
  for (int x = threadIdx.x; x < nrb * n_r; x += blockDim.x) {
    const int r = x / n_r, i = x - r * n_r;
    const double q = a.tab[i];
    double G;
    if constexpr (PAIRS)
      G = PairRow{lp + r * n_s}((q * q) * a.inv_h, a.t_last, n_s - 2);
    else
      G = PlainRow{l.lg + r * n_s}((q * q) * a.inv_h, a.t_last, n_s - 2);
    if (r == 0) l.lrad[i * (1 + RB)] = q;
    l.lrad[i * (1 + RB) + 1 + r] = (a.tab[n_r + i] * G) * G;
  }
  __syncthreads();
  tab_block_rows<UR, RB>(a, rows, nrb, l.lrad, l.lo, l.lm, r0, pb, W, wave, lane);
}

}  // namespace dev
}  // namespace frg
