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

namespace frg {
namespace dev {

// ------------------------------------------------ coefficient form --
// Resident tables of the FP64 grid kernel.  For a group of G angular terms
// of one lane (one radial node i; u = gi G .. gi G + G - 1), with
// H_k = Hk(s_ik) and weights mu_k,
//   sum_k mu_k / (delta + H_k) = N(delta) / P(delta),
//   P(delta) = prod_k (delta + H_k) = delta^G + sum_{m<G} c_m delta^m,
//   N(delta) = sum_k mu_k prod_{l != k} (delta + H_l) = sum_{m<G} d_m delta^m.
// The coefficients depend on the momentum only, so the workgroup builds them
// once (G^2 FMAs per group) and every mass evaluates two Horner chains
// (2G - 1 FMAs and one add) and one reciprocal per G terms.  Every H_k >= 0
// and mu_k > 0, so all coefficients are positive and both the expansion and
// the Horner sums add positive terms only (relative error O(G u)).
//
// Layout (lane-major, like the H' table): group (t, gi) occupies rows
// (t NG + gi) 2G + m, m < G holding c_m and m >= G holding d_{m-G}; the
// remaining angular terms of a row (u >= Gfull) hold H in rows
// T NG 2G + t UT + (u - Gfull).
template <int G>
struct CoefShape {
  int Gfull, NG, UT, rows;
  __host__ __device__ CoefShape(int n_a, int J, int T, int U) {
    const int umin = n_a / J;
    Gfull = umin - umin % G;
    NG = Gfull / G;
    UT = U - Gfull;
    rows = T * (2 * Gfull + UT);
  }
};

// Ranges where no coefficient, Horner partial sum or P over- or underflows:
// per momentum (q_max + p)^2 <= kCoefHi (bounds every H), per mass
// kCoefLo <= delta <= kCoefHi.
template <int G>
struct CoefRange;
template <>
struct CoefRange<8> {
  static constexpr double lo = 1e-36, hi = 1e36;
};
template <>
struct CoefRange<16> {
  static constexpr double lo = 1e-18, hi = 5e17;
};

template <int G>
__device__ __forceinline__ bool coef_p_ok(double p, double q_top) {
  const double qp = q_top + p;
  return qp * qp <= CoefRange<G>::hi;
}

template <int G>
__device__ __forceinline__ bool coef_m_ok(double delta) {
  return delta >= CoefRange<G>::lo && delta <= CoefRange<G>::hi;
}

// Build the coefficient table of momentum p (all threads of the workgroup).
template <int REG, int G>
__device__ void grid_fill_coef(const GridArgs &g, double *lC, double p, const CoefShape<G> &cs) {
  const double *tq = g.tab;
  const double *to = g.tab + 3 * g.n_r;
  const double *tm = to + g.n_a;
  const int n_group = kWave * g.T * cs.NG;
  const int n_tail = kWave * g.T * cs.UT;
  for (int task = threadIdx.x; task < n_group + n_tail; task += blockDim.x) {
    const int l = task & (kWave - 1);
    const int rho = l & (g.R - 1), iota = l / g.R;
    if (task < n_group) {
      const int rest = task / kWave;
      const int t = rest / cs.NG, gi = rest - t * cs.NG;
      const int i = rho + g.R * t;
      const double q = i < g.n_r ? tq[i] : 0.0;  // padded radial lanes: any finite value
      const double qm = q - p;
      const double a = qm * qm;
      const double b = (2.0 * q) * p;
      double P[G + 1], N[G];
#pragma unroll
      for (int m = 0; m <= G; ++m) P[m] = m == 0 ? 1.0 : 0.0;
#pragma unroll
      for (int m = 0; m < G; ++m) N[m] = 0.0;
#pragma unroll
      for (int k = 0; k < G; ++k) {
        const int j = iota + g.J * (gi * G + k);
        const double H = hk<REG>(__builtin_fma(b, to[j], a), g.k2, g.inv_k2);
        const double mu = tm[j];
        // N <- N (delta + H) + mu P, then P <- P (delta + H), on the old P.
        // Before term k, P has degree k with P[k] = 1 and N degree k - 1;
        // only those entries are touched (k is a compile-time index here).
        if (k == 0) {
          N[0] = mu;
          P[1] = 1.0;
          P[0] = H;
        } else {
          N[k] = __builtin_fma(mu, P[k], N[k - 1]);
#pragma unroll
          for (int m = G - 1; m >= 1; --m)
            if (m < k) N[m] = __builtin_fma(mu, P[m], __builtin_fma(H, N[m], N[m - 1]));
          N[0] = __builtin_fma(mu, P[0], H * N[0]);
          P[k + 1 <= G ? k + 1 : G] = 1.0;
#pragma unroll
          for (int m = G; m >= 1; --m)
            if (m <= k) P[m] = __builtin_fma(H, P[m], P[m - 1]);
          P[0] = H * P[0];
        }
      }
      double *dst = lC + ((t * cs.NG + gi) * 2 * G) * kWave + l;
#pragma unroll
      for (int m = 0; m < G; ++m) {
        dst[m * kWave] = P[m];
        dst[(G + m) * kWave] = N[m];
      }
    } else {
      const int rest = (task - n_group) / kWave;
      const int t = rest / cs.UT, ut = rest - t * cs.UT;
      const int i = rho + g.R * t;
      const int j = iota + g.J * (cs.Gfull + ut);
      double H = 1.0;
      if (j < g.n_a) {
        const double q = i < g.n_r ? tq[i] : 0.0;
        const double qm = q - p;
        H = hk<REG>(__builtin_fma((2.0 * q) * p, to[j], qm * qm), g.k2, g.inv_k2);
      }
      lC[(g.T * cs.NG * 2 * G + t * cs.UT + ut) * kWave + l] = H;
    }
  }
}

// Accumulate, for the masses set in `active`, the lane partials of the
// coefficient form into tot[m].  ALL: every mass active.
template <int M, int G, bool ALL>
__device__ __forceinline__ void grid_coef_rows(const GridArgs &g, const double *lC,
                                               const double *lc, const double *lq,
                                               const double *lm, int lane, const double *dm,
                                               unsigned active, const CoefShape<G> &cs,
                                               double *tot) {
  const int rho = lane & (g.R - 1);
  const int iota = lane / g.R;
  for (int t = 0; t < g.T; ++t) {
    const int i = rho + g.R * t;
    const bool vi = i < g.n_r;
    double in[M];
#pragma unroll
    for (int m = 0; m < M; ++m) in[m] = 0.0;
    for (int gi = 0; gi < cs.NG; ++gi) {
      const double *src = lC + ((t * cs.NG + gi) * 2 * G) * kWave + lane;
      double cc[G], dd[G];
#pragma unroll
      for (int m = 0; m < G; ++m) {
        cc[m] = src[m * kWave];
        dd[m] = src[(G + m) * kWave];
      }
      if constexpr (ALL) {
        // masses in pairs: four independent Horner chains in flight
#pragma unroll
        for (int m = 0; m < M; m += 2) {
          const double xa = dm[m], xb = dm[m + 1];
          double Pa = xa + cc[G - 1], Pb = xb + cc[G - 1];
          double Na = dd[G - 1], Nb = dd[G - 1];
#pragma unroll
          for (int k = G - 2; k >= 0; --k) {
            Pa = __builtin_fma(Pa, xa, cc[k]);
            Pb = __builtin_fma(Pb, xb, cc[k]);
            Na = __builtin_fma(Na, xa, dd[k]);
            Nb = __builtin_fma(Nb, xb, dd[k]);
            __builtin_amdgcn_sched_barrier(0);
          }
          in[m] = __builtin_fma(Na, rcp64(Pa), in[m]);
          in[m + 1] = __builtin_fma(Nb, rcp64(Pb), in[m + 1]);
        }
      } else {
#pragma unroll
        for (int m = 0; m < M; ++m) {
          if (!((active >> m) & 1u)) continue;
          const double x = dm[m];
          double P = x + cc[G - 1], N = dd[G - 1];
#pragma unroll
          for (int k = G - 2; k >= 0; --k) {
            P = __builtin_fma(P, x, cc[k]);
            N = __builtin_fma(N, x, dd[k]);
          }
          in[m] = __builtin_fma(N, rcp64(P), in[m]);
        }
      }
    }
    for (int ut = 0; ut < cs.UT; ++ut) {
      const int j = iota + g.J * (cs.Gfull + ut);
      if (j < g.n_a) {
        const double mu = lm[j];
        const double H = lC[(g.T * cs.NG * 2 * G + t * cs.UT + ut) * kWave + lane];
#pragma unroll
        for (int m = 0; m < M; ++m) {
          if (!ALL && !((active >> m) & 1u)) continue;
          in[m] = __builtin_fma(mu, rcp64(H + dm[m]), in[m]);
        }
      }
    }
    // radial factor A_i = c_i / (Hq_i + delta)^2, formed after the angular
    // sums so that it holds no registers during them
    const double c = vi ? lc[i] : 0.0;
    const double Hq = vi ? lq[i] : 1.0;
#pragma unroll
    for (int m = 0; m < M; ++m) {
      if (!ALL && !((active >> m) & 1u)) continue;
      const double Gq = rcp64(Hq + dm[m]);
      tot[m] = __builtin_fma((c * Gq) * Gq, in[m], tot[m]);
    }
  }
}

// Lane partial of one mass outside the coefficient range: every term on its
// own, the regulator evaluated again per term (rare: extreme masses or
// momenta).
template <int REG>
__device__ __forceinline__ double grid_single_mass(const GridArgs &g, const double *lc,
                                                const double *lq, const double *lm, int lane,
                                                double p, double delta) {
  const int rho = lane & (g.R - 1);
  const int iota = lane / g.R;
  const double *tq = g.tab;
  const double *to = g.tab + 3 * g.n_r;
  double total = 0.0;
  for (int t = 0; t < g.T; ++t) {
    const int i = rho + g.R * t;
    const bool vi = i < g.n_r;
    const double q = vi ? tq[i] : 0.0;
    const double c = vi ? lc[i] : 0.0;
    const double Hq = vi ? lq[i] : 1.0;
    const double Gq = rcp64(Hq + delta);
    const double A = (c * Gq) * Gq;
    const double qm = q - p;
    const double a = qm * qm;
    const double b = (2.0 * q) * p;
    double inner = 0.0;
    for (int u = 0; u < g.U; ++u) {
      const int j = iota + g.J * u;
      if (j < g.n_a) {
        const double H = hk<REG>(__builtin_fma(b, to[j], a), g.k2, g.inv_k2);
        inner = __builtin_fma(lm[j], rcp64(H + delta), inner);
      }
    }
    total = __builtin_fma(A, inner, total);
  }
  return total;
}

}  // namespace dev
}  // namespace frg
