// Tensor-grid device routines shared by the FP64 grid kernel and the
// compensated-FP32 grid kernel (included by the .hip translation units only).
//
// A workgroup owns one momentum p; the table H'_ij = Hk(s_ij) rmu_j of that p
// sits in LDS, lane-major: row r = t U + u holds, in lane l = rho + R iota,
// the entry of radial node i = rho + R t and angular node j = iota + J u.
#pragma once

#include <hip/hip_runtime.h>

#include "device_fp64.h"
#include "frg_internal.h"

#pragma clang fp contract(off)

namespace frg {
namespace dev {

// Accumulate the rows [c0, c1) of the table for the M masses of one wave.
// `gmask` bit m: mass m takes the grouped form.
template <int M>
__device__ __forceinline__ void grid_rows(const GridArgs &g, const double *lH, const double *lc,
                                          const double *lq, const double *lr, int c0, int c1,
                                          int lane, const double *dm, unsigned gmask, int &t,
                                          int &u, double *A, double *in, double *tot) {
  const int rho = lane & (g.R - 1);
  const int iota = lane / g.R;
  const int n_r = g.n_r, n_a = g.n_a;
  const int G = grouped_u(n_a, g.J);
  const unsigned all = (M == 32) ? ~0u : ((1u << M) - 1u);
  int tu = c0;
  while (tu < c1) {
    if (u == 0) {
      const int i = rho + g.R * t;
      const bool vi = i < n_r;
      const double c = vi ? lc[i] : 0.0;
      const double Hq = vi ? lq[i] : 1.0;
#pragma unroll
      for (int m = 0; m < M; ++m) {
        const double Gq = rcp64(Hq + dm[m]);
        A[m] = (c * Gq) * Gq;
        in[m] = 0.0;
      }
    }
    if (u < G) {
      // a whole group lies in this chunk (chunk_end never splits one)
      double H[kGroup], r[kGroup];
#pragma unroll
      for (int k = 0; k < kGroup; ++k) {
        r[k] = lr[iota + g.J * (u + k)];
        H[k] = lH[(tu + k - c0) * kWave + lane];
      }
      if (gmask == all) {
        // common case: every mass takes the grouped form (no branches)
#pragma unroll
        for (int m = 0; m < M; ++m) {
          double Dp[kGroup];
#pragma unroll
          for (int k = 0; k < kGroup; ++k) Dp[k] = __builtin_fma(dm[m], r[k], H[k]);
          in[m] = chain_sum(Dp, in[m]);
        }
      } else {
#pragma unroll
        for (int m = 0; m < M; ++m) {
          double Dp[kGroup];
#pragma unroll
          for (int k = 0; k < kGroup; ++k) Dp[k] = __builtin_fma(dm[m], r[k], H[k]);
          if ((gmask >> m) & 1u) {
            in[m] = chain_sum(Dp, in[m]);
          } else {
#pragma unroll
            for (int k = 0; k < kGroup; ++k) in[m] = in[m] + rcp64(Dp[k]);
          }
        }
      }
      u += kGroup;
      tu += kGroup;
    } else {
      const int j = iota + g.J * u;
      if (j < n_a) {
        const double r = lr[j];
        const double H = lH[(tu - c0) * kWave + lane];
#pragma unroll
        for (int m = 0; m < M; ++m) in[m] = in[m] + rcp64(__builtin_fma(dm[m], r, H));
      }
      ++u;
      ++tu;
    }
    if (u == g.U) {
#pragma unroll
      for (int m = 0; m < M; ++m) tot[m] = __builtin_fma(A[m], in[m], tot[m]);
      u = 0;
      ++t;
    }
  }
}

// Resident table (all T U rows in LDS): the same visiting order and
// arithmetic as grid_rows, as plain nested loops.  Only the masses whose bit
// is set in `active` are computed (the others keep tot[m]); `gmask` bit m:
// mass m takes the grouped form.  ALL: every mass is active and grouped.
template <int M, bool ALL>
__device__ __forceinline__ void grid_resident(const GridArgs &g, const double *lH,
                                              const double *lc, const double *lq,
                                              const double *lr, int lane, const double *dm,
                                              unsigned active, unsigned gmask, double *tot) {
  const int rho = lane & (g.R - 1);
  const int iota = lane / g.R;
  const int G = grouped_u(g.n_a, g.J);
  for (int t = 0; t < g.T; ++t) {
    const int i = rho + g.R * t;
    const bool vi = i < g.n_r;
    const double c = vi ? lc[i] : 0.0;
    const double Hq = vi ? lq[i] : 1.0;
    double A[M], in[M];
#pragma unroll
    for (int m = 0; m < M; ++m) {
      if (!ALL && !((active >> m) & 1u)) continue;
      const double Gq = rcp64(Hq + dm[m]);
      A[m] = (c * Gq) * Gq;
      in[m] = 0.0;
    }
    const double *row = lH + (t * g.U) * kWave + lane;
    int u = 0;
    for (; u < G; u += kGroup) {
      double H[kGroup], r[kGroup];
#pragma unroll
      for (int k = 0; k < kGroup; ++k) {
        r[k] = lr[iota + g.J * (u + k)];
        H[k] = row[(u + k) * kWave];
      }
      if constexpr (ALL) {
        // masses in pairs: two independent chains in flight
#pragma unroll
        for (int m = 0; m < M; m += 2) {
          double Da[kGroup], Db[kGroup];
#pragma unroll
          for (int k = 0; k < kGroup; ++k) {
            Da[k] = __builtin_fma(dm[m], r[k], H[k]);
            Db[k] = __builtin_fma(dm[m + 1], r[k], H[k]);
          }
          chain_sum2(Da, Db, in[m], in[m + 1]);
        }
      } else {
#pragma unroll
        for (int m = 0; m < M; ++m) {
          if (!((active >> m) & 1u)) continue;
          double Dp[kGroup];
#pragma unroll
          for (int k = 0; k < kGroup; ++k) Dp[k] = __builtin_fma(dm[m], r[k], H[k]);
          if ((gmask >> m) & 1u) {
            in[m] = chain_sum(Dp, in[m]);
          } else {
#pragma unroll
            for (int k = 0; k < kGroup; ++k) in[m] = in[m] + rcp64(Dp[k]);
          }
        }
      }
    }
    for (; u < g.U; ++u) {
      const int j = iota + g.J * u;
      if (j < g.n_a) {
        const double r = lr[j];
        const double H = row[u * kWave];
#pragma unroll
        for (int m = 0; m < M; ++m) {
          if (!ALL && !((active >> m) & 1u)) continue;
          in[m] = in[m] + rcp64(__builtin_fma(dm[m], r, H));
        }
      }
    }
#pragma unroll
    for (int m = 0; m < M; ++m) {
      if (!ALL && !((active >> m) & 1u)) continue;
      tot[m] = __builtin_fma(A[m], in[m], tot[m]);
    }
  }
}

// End of the LDS chunk that starts at row c0: at most C rows, moved back to
// a group boundary so that no group is split (C >= kGroup).
__device__ __forceinline__ int chunk_end(const GridArgs &g, int c0, int C, int TU) {
  int c1 = c0 + C < TU ? c0 + C : TU;
  if (c1 < TU) {
    const int t1 = c1 / g.U, u1 = c1 - t1 * g.U;
    if (u1 < grouped_u(g.n_a, g.J)) c1 = t1 * g.U + (u1 - u1 % kGroup);
  }
  return c1;
}

// Fill rows [c0, c1) of the table of momentum p into lH and, when lH32 is
// non-null, its compensated-FP32 form lH32 = fl32(H' sig_j) (either may be
// null).
template <int REG>
__device__ __forceinline__ void grid_fill(const GridArgs &g, double *lH, int c0, int c1, double p,
                                          float *lH32 = nullptr, const double *sig = nullptr) {
  const double *tq = g.tab;
  const double *to = g.tab + 3 * g.n_r;
  const double *tr = to + 2 * g.n_a;
  const int l = threadIdx.x & (kWave - 1);
  const int rho = l & (g.R - 1), iota = l / g.R;
  // wave w fills rows c0 + w, c0 + w + W, ...; the row's (t, u) is stepped
  // without divisions (row, t and u are wave-uniform)
  const int W = blockDim.x / kWave;
  int row = c0 + __builtin_amdgcn_readfirstlane((int)(threadIdx.x / kWave));
  int tt = row / g.U, uu = row - tt * g.U;
  for (; row < c1; row += W) {
    const int i = rho + g.R * tt;
    const int j = iota + g.J * uu;
    double v = 1.0;
    if (j < g.n_a) {
      // padded radial lanes (i >= n_r) see q = 0, as in lane_point
      const double q = i < g.n_r ? tq[i] : 0.0;
      const double qm = q - p;
      const double aa = qm * qm;
      const double b = (2.0 * q) * p;
      v = hk<REG>(__builtin_fma(b, to[j], aa), g.k2, g.inv_k2) * tr[j];
    }
    if (lH) lH[(row - c0) * kWave + l] = v;
    if (lH32) lH32[(row - c0) * kWave + l] = (float)(v * (j < g.n_a ? sig[j] : 1.0));
    uu += W;
    while (uu >= g.U) {
      uu -= g.U;
      ++tt;
    }
  }
}

}  // namespace dev
}  // namespace frg
