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
#include "device_tab.h"

namespace frg {

namespace {

using namespace dev;

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
  if (lane < a.pw && ia < a.n_p) a.out[ia * a.n_rows + r] = res;
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

// LDS_ROW: one workgroup per (row, momentum block), the row staged in LDS.
// Otherwise a fixed grid of 8 * slots workgroups: workgroup b runs on XCD
// b mod 8 (round-robin dispatch) and works through the rows of that XCD one
// after another, taking momentum blocks slot, slot + slots, ... of each, so
// that each XCD streams one row at a time through its L2 and the rows in
// flight on the chip stay within the memory-side cache.
// UR > 0: every lane holds at most UR angular nodes (U <= UR), kept in
// registers; UR == 0: read from LDS.
template <bool LDS_ROW, int UR, bool PAIRS>
__global__ __launch_bounds__(256) void tab_kernel(TabArgs a) {
  extern __shared__ double lds[];
  const int W = blockDim.x / kWave;
  const int wave = threadIdx.x / kWave;
  const int lane = threadIdx.x & (kWave - 1);
  const int n_r = a.n_r, n_a = a.n_a;
  double *lq = lds;           // q_i
  double *lA = lq + n_r;      // c_i G_r(q_i^2)^2
  double *lo = lA + n_r;      // 1 + x_j
  double *lm = lo + n_a;      // mu_j
  double *lg = lm + n_a;      // the row (LDS_ROW): values, or (value, slope) pairs
  for (int j = threadIdx.x; j < n_a; j += blockDim.x) {
    lo[j] = a.tab[3 * n_r + j];
    lm[j] = a.tab[3 * n_r + n_a + j];
  }
  if constexpr (LDS_ROW) {
    const int64_t r = blockIdx.x / a.n_pb;
    const int64_t pb = blockIdx.x - r * a.n_pb;
    const double *grow = a.g + r * a.n_s;
    if constexpr (PAIRS) {
      double2 *lp = reinterpret_cast<double2 *>(lg);
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
      tab_stage_A(a, row, lq, lA);
      __syncthreads();
      tab_block<UR>(a, row, lq, lA, lo, lm, r, pb, W, wave, lane);
    } else {
      for (int k = threadIdx.x; k < (int)a.n_s; k += blockDim.x) lg[k] = grow[k];
      __syncthreads();
      const PlainRow row{lg};
      tab_stage_A(a, row, lq, lA);
      __syncthreads();
      tab_block<UR>(a, row, lq, lA, lo, lm, r, pb, W, wave, lane);
    }
  } else {
    const int x = blockIdx.x & 7;
    const int64_t slot = blockIdx.x >> 3, slots = gridDim.x >> 3;
    for (int64_t r = x; r < a.n_rows; r += 8) {
      const PlainRow grow{a.g + r * a.n_s};
      __syncthreads();  // the previous row's A_i are no longer read
      tab_stage_A(a, grow, lq, lA);
      __syncthreads();
      for (int64_t pb = slot; pb < a.n_pb; pb += slots)
        tab_block<UR>(a, grow, lq, lA, lo, lm, r, pb, W, wave, lane);
    }
  }
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
  const int row = !lds_rows ? 0 : t.pairs ? (int)(2 * t.n_s) : (int)t.n_s;
  return (int)(sizeof(double) * (2 * t.n_r + 2 * t.n_a + row));
}

// Dynamic LDS beyond 64 KiB (gfx950: 160 KiB per workgroup); a refusal where
// no opt-in is needed is cleared so that it cannot be taken for a launch error.
static void tab_allow_large_lds(const void *fn) {
  (void)hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
  (void)hipGetLastError();
}

template <bool L, int UR, bool P>
static void tab_launch_t(const TabArgs &t, int W, int64_t blocks, hipStream_t st) {
  static const bool once = (tab_allow_large_lds((const void *)&tab_kernel<L, UR, P>), true);
  (void)once;
  hipLaunchKernelGGL((tab_kernel<L, UR, P>), dim3((unsigned)blocks), dim3(kWave * W),
                     tab_lds_bytes(t, L), st, t);
}

int launch_tab(const TabArgs &t, int reg, int W, bool lds_rows, int64_t stream_blocks,
               void *stream) {
  (void)reg;  // the regulator enters through the quadrature table only
  if (t.n_p <= 0 || t.n_rows <= 0) return 0;
  hipStream_t st = (hipStream_t)stream;
  const bool regs = t.U <= 4;
  if (lds_rows) {
    const int64_t blocks = t.n_rows * t.n_pb;
    if (t.pairs)
      regs ? tab_launch_t<true, 4, true>(t, W, blocks, st) : tab_launch_t<true, 0, true>(t, W, blocks, st);
    else
      regs ? tab_launch_t<true, 4, false>(t, W, blocks, st) : tab_launch_t<true, 0, false>(t, W, blocks, st);
  } else {
    const int64_t blocks = 8 * ((stream_blocks + 7) / 8);
    regs ? tab_launch_t<false, 4, false>(t, W, blocks, st) : tab_launch_t<false, 0, false>(t, W, blocks, st);
  }
  return (int)hipGetLastError();
}

}  // namespace frg
