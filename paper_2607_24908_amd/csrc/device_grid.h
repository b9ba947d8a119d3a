// Tensor-grid device routines of the FP64 grid kernels (included by the .hip
// translation units only).
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

// Fill rows [c0, c1) of the table of momentum p into lH.
template <int REG>
__device__ __forceinline__ void grid_fill(const GridArgs &g, double *lH, int c0, int c1, double p) {
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
    lH[(row - c0) * kWave + l] = v;
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
// Resident tables of the FP64 grid kernel.  Take one lane and one radial
// node i of it, and a group of G of the lane's angular terms k (weights
// mu_k, regulator values H_k = Hk(s_ik); terms past the end of the row are
// padding with mu = H = 0).  The group's part of the result at mass delta,
//   c_i / (Hq_i + delta)^2 * sum_k mu_k / (delta + H_k) = N(delta) / P(delta),
// is one rational function with
//   P(x) = (x + Hq_i)^2 prod_k (x + H_k)            (monic, degree G + 2),
//   N(x) = c_i sum_k mu_k prod_{l != k} (x + H_l)    (degree G - 1).
// Their coefficients depend on the momentum only: the workgroup builds them
// once, and every mass then costs two Horner sums (2G + 1 FMAs and one add),
// one reciprocal and one FMA per G terms, radial factor included.  Every
// H >= 0, mu >= 0 and c >= 0, so all coefficients are non-negative and both
// the expansion and the Horner sums add non-negative terms only (relative
// error O(G u), no cancellation).
//
// Scaling.  The coefficients are products of up to G + 2 factors, so they
// are formed in units where k^2 is about one: x = sig delta, H -> sig H,
// Hq -> sig Hq and c -> kap c, with sig and kap powers of two (exact), sig
// k^2 in [1, 2) and kap max_i c_i in [1/2, 1).  N/P then carries the factor
// kap / sig^3, which the host folds into the prefactor (pref_c).
//
// Range.  With X = sig (q_top + p)^2 (every sig H and sig Hq lies below it)
// and x in [lo, hi], X <= hi: every coefficient and Horner partial sum lies
// below (2 hi)^(G+2) <= 1e297 and P(x) >= x^(G+2) >= 1e-290, so nothing
// over- or underflows where it matters.  Masses outside the range, and every
// mass of a momentum outside it, take the per-term path (grid_single_mass).
//
// Layout (lane-major, like the H' table): group (t, gi), gi < NG, occupies
// 2G + 2 rows from (t NG + gi)(2G + 2): rows m < G + 2 hold the coefficient
// of x^m of P, rows G + 2 + m that of x^m of N.
// E = number of extra linear factors folded into P (2: (x + Hq)^2 of the
// two-point diagram; 3: also (x + H1) of the vertex diagram); a group takes
// 2G + E rows: G + E coefficients of the monic P, G of N.
template <int G, int E = 2>
struct FoldShape {
  int NG, rows;
  __host__ __device__ FoldShape(int U, int T) {
    NG = (U + G - 1) / G;
    rows = T * NG * (2 * G + E);
  }
};

// (lo, hi) with (2 hi)^(G+E) <= 1e297 and lo^(G+E) >= 1e-290.
template <int G, int E = 2>
struct FoldRange;
template <>
struct FoldRange<8, 2> {
  static constexpr double lo = 1e-29, hi = 2e29;
};
template <>
struct FoldRange<16, 2> {
  static constexpr double lo = 1e-16, hi = 1.5e16;
};
template <>
struct FoldRange<32, 2> {
  static constexpr double lo = 4e-9, hi = 2.5e8;
};
template <>
struct FoldRange<8, 3> {
  static constexpr double lo = 5e-27, hi = 4e26;
};
template <>
struct FoldRange<16, 3> {
  static constexpr double lo = 6e-16, hi = 2e15;
};
template <>
struct FoldRange<32, 3> {
  static constexpr double lo = 6e-9, hi = 1.5e8;
};

template <int G, int E = 2>
__device__ __forceinline__ bool fold_p_ok(double p, const GridArgs &g) {
  const double qp = g.q_top + p;
  return g.sig * (qp * qp) <= FoldRange<G, E>::hi;
}

template <int G, int E = 2>
__device__ __forceinline__ bool fold_m_ok(double x) {
  return x >= FoldRange<G, E>::lo && x <= FoldRange<G, E>::hi;
}

// Build the coefficient table of momentum p (all threads of the workgroup;
// lc, lq, lm: c_i, Hq_i and mu_j, lqn, lo: q_i and 1 + x_j, already staged in
// LDS).  Pass 1 spreads the regulator evaluations over all threads and parks
// the scaled H of each group in the group's own P rows; pass 2 expands one
// group per thread.  In pass 1 a thread keeps its lane (the stride is a
// multiple of 64 lanes) and steps the group row (t, gi, k) by the number of
// waves without divisions.
template <int REG, int G>
__device__ void grid_fill_fold(const GridArgs &g, double *lC, const double *lc, const double *lq,
                               const double *lm, const double *lqn, const double *lo, double p,
                               const FoldShape<G> &fs) {
  const int n_grp = g.T * fs.NG;
  {
    const int l = threadIdx.x & (kWave - 1);
    const int W = blockDim.x / kWave;
    const int rho = l & (g.R - 1), iota = l >> __builtin_ctz(g.R);  // R is a power of two
    int k = threadIdx.x / kWave, gi = 0, t = 0;
    while (k >= G) {
      k -= G;
      if (++gi == fs.NG) {
        gi = 0;
        ++t;
      }
    }
    for (int row = threadIdx.x / kWave; row < n_grp * G; row += W) {
      const int i = rho + g.R * t;
      const int j = iota + g.J * (gi * G + k);
      double H = 0.0;
      if (i < g.n_r && j < g.n_a) {
        const double q = lqn[i];
        const double qm = q - p;
        H = g.sig * hk<REG>(__builtin_fma((2.0 * q) * p, lo[j], qm * qm), g.k2, g.inv_k2);
      }
      lC[((t * fs.NG + gi) * (2 * G + 2) + k) * kWave + l] = H;
      k += W;
      while (k >= G) {
        k -= G;
        if (++gi == fs.NG) {
          gi = 0;
          ++t;
        }
      }
    }
  }
  __syncthreads();
  for (int task = threadIdx.x; task < kWave * n_grp; task += blockDim.x) {
    const int l = task & (kWave - 1);
    const int tg = task / kWave;
    const int t = tg / fs.NG, gi = tg - t * fs.NG;
    const int i = (l & (g.R - 1)) + g.R * t;
    const int j0 = l / g.R + g.J * gi * G;
    const bool vi = i < g.n_r;
    double *col = lC + tg * (2 * G + 2) * kWave + l;
    double P[G + 3], N[G];
#pragma unroll
    for (int m = 0; m < G + 3; ++m) P[m] = 0.0;
#pragma unroll
    for (int m = 0; m < G; ++m) N[m] = 0.0;
#pragma unroll
    for (int k = 0; k < G; ++k) {
      const double H = col[k * kWave];
      const int j = j0 + g.J * k;
      const double mu = (vi && j < g.n_a) ? lm[j] : 0.0;
      // N <- N (x + H) + mu P, then P <- P (x + H), on the old P.  Before
      // term k, P has degree k with P[k] = 1 and N degree k - 1; only those
      // entries are touched (k is a compile-time index here).
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
        P[k + 1] = 1.0;
#pragma unroll
        for (int m = G; m >= 1; --m)
          if (m <= k) P[m] = __builtin_fma(H, P[m], P[m - 1]);
        P[0] = H * P[0];
      }
    }
    // radial factor: P <- P (x + Hq)^2, N <- c N
    const double Hq = vi ? g.sig * lq[i] : 0.0;
    const double c = vi ? g.kap * lc[i] : 0.0;
#pragma unroll
    for (int r = 0; r < 2; ++r) {
      const int deg = G + r;  // P[deg] = 1
      P[deg + 1] = 1.0;
#pragma unroll
      for (int m = G + 1; m >= 1; --m)
        if (m <= deg) P[m] = __builtin_fma(Hq, P[m], P[m - 1]);
      P[0] = Hq * P[0];
    }
#pragma unroll
    for (int m = 0; m < G + 2; ++m) col[m * kWave] = P[m];
#pragma unroll
    for (int m = 0; m < G; ++m) col[(G + 2 + m) * kWave] = c * N[m];
  }
}

// Accumulate, for the masses set in `active`, the lane partials of the
// coefficient form into tot[m]; xs[m] = sig delta_m.  ALL: every mass active.
template <int M, int G, bool ALL, int E = 2>
__device__ __forceinline__ void grid_fold_rows(const GridArgs &g, const double *lC, int lane,
                                               const double *xs, unsigned active,
                                               const FoldShape<G, E> &fs, double *tot) {
  const int n_grp = g.T * fs.NG;
  for (int tg = 0; tg < n_grp; ++tg) {
    const double *src = lC + tg * (2 * G + E) * kWave + lane;
    double a[G + E], b[G];
#pragma unroll
    for (int m = 0; m < G + E; ++m) a[m] = src[m * kWave];
#pragma unroll
    for (int m = 0; m < G; ++m) b[m] = src[(G + E + m) * kWave];
    if constexpr (ALL) {
      // masses in pairs: four independent Horner chains in flight
#pragma unroll
      for (int m = 0; m < M; m += 2) {
        const double xa = xs[m], xb = xs[m + 1];
        double Pa = xa + a[G + E - 1], Pb = xb + a[G + E - 1];
        // P has E more coefficients than N: those steps first
#pragma unroll
        for (int k = G + E - 2; k >= G - 1; --k) {
          Pa = __builtin_fma(Pa, xa, a[k]);
          Pb = __builtin_fma(Pb, xb, a[k]);
        }
        double Na = b[G - 1], Nb = b[G - 1];
#pragma unroll
        for (int k = G - 2; k >= 0; --k) {
          Pa = __builtin_fma(Pa, xa, a[k]);
          Pb = __builtin_fma(Pb, xb, a[k]);
          Na = __builtin_fma(Na, xa, b[k]);
          Nb = __builtin_fma(Nb, xb, b[k]);
          __builtin_amdgcn_sched_barrier(0);
        }
        tot[m] = __builtin_fma(Na, rcp64(Pa), tot[m]);
        tot[m + 1] = __builtin_fma(Nb, rcp64(Pb), tot[m + 1]);
      }
    } else {
#pragma unroll
      for (int m = 0; m < M; ++m) {
        if (!((active >> m) & 1u)) continue;
        const double x = xs[m];
        double P = x + a[G + E - 1], N = b[G - 1];
#pragma unroll
        for (int k = G + E - 2; k >= G - 1; --k) P = __builtin_fma(P, x, a[k]);
#pragma unroll
        for (int k = G - 2; k >= 0; --k) {
          P = __builtin_fma(P, x, a[k]);
          N = __builtin_fma(N, x, b[k]);
        }
        tot[m] = __builtin_fma(N, rcp64(P), tot[m]);
      }
    }
  }
}

// ------------------------------------- coefficient form, matrix cores --
// For a tile of 16 masses x_j the values P_r(x_j) and N_r(x_j) of every lane
// row r of the table are the products A_P V and A_N V of the coefficient
// rows with the power matrix V[k][j] = x_j^k: dense contractions over k,
// taken four powers at a time by v_mfma_f64_16x16x4f64 on a 16-row slice of
// a 64-row group.  Operand layout of that instruction (A 16 x 4, B 4 x 16,
// D 16 x 16): lane l supplies A[l % 16][l / 16] and B[l / 16][l % 16] and
// holds D[4 e + l / 16][l % 16] in element e of the result.  Lane l thus
// ends with N/P of four rows of mass l % 16 and sums them in place.
// Every coefficient and every x_j^k is >= 0 (H >= 0, weights > 0, x > 0),
// so the power sums carry no cancellation and round like the nested form;
// each term is at most P(x) or N(x), inside the range of FoldRange.
typedef double dbl4 __attribute__((ext_vector_type(4)));

// P has G + E stored coefficients, then the monic 1 and zero padding to a
// multiple of four powers: G/4 + 1 slices of k (E = 2, 3).  N: G/4 slices.
template <int G, int E>
struct MfmaShape {
  static_assert(G % 4 == 0 && (E == 2 || E == 3), "G a multiple of 4, E 2 or 3");
  static constexpr int kP = G / 4 + 1, kN = G / 4;
};

// x^(4c + e) for c < kP, e = lane / 16: the lane's entries of V.  Powers
// above G + E (zero coefficients, padding) are set to 0, not computed: they
// lie outside the range of FoldRange (x^(G+3) overflows for G = 8 near hi),
// and 0 * inf would poison the sum.
template <int G, int E>
__device__ __forceinline__ void mfma_powers(double x, int lane, double *v) {
  constexpr int kP = MfmaShape<G, E>::kP;
  const int e = lane >> 4;
  const double x2 = x * x;
  const double x4 = x2 * x2;
  v[0] = e == 0 ? 1.0 : e == 1 ? x : e == 2 ? x2 : x2 * x;
#pragma unroll
  for (int c = 1; c < kP; ++c) v[c] = v[c - 1] * x4;
  if (e > E) v[kP - 1] = 0.0;
}

// Two 16-row slices (rows 16 s0 + ., 16 s1 + . of one group): four
// independent accumulator chains.
template <int G, int E>
__device__ __forceinline__ void mfma_slice_pair(const double *grp, int lane, const double *v,
                                                int s0, int s1, double &tot) {
  constexpr int kP = MfmaShape<G, E>::kP, kN = MfmaShape<G, E>::kN;
  const int e = lane >> 4;
  const double *a0 = grp + 16 * s0 + (lane & 15) + e * kWave;  // A[row][k] at grp[k 64 + row]
  const double *a1 = grp + 16 * s1 + (lane & 15) + e * kWave;
  const dbl4 z = {0.0, 0.0, 0.0, 0.0};
  dbl4 P0 = z, N0 = z, P1 = z, N1 = z;
#pragma unroll
  for (int c = 0; c < kN; ++c) {
    P0 = __builtin_amdgcn_mfma_f64_16x16x4f64(a0[4 * c * kWave], v[c], P0, 0, 0, 0);
    P1 = __builtin_amdgcn_mfma_f64_16x16x4f64(a1[4 * c * kWave], v[c], P1, 0, 0, 0);
    N0 = __builtin_amdgcn_mfma_f64_16x16x4f64(a0[(G + E + 4 * c) * kWave], v[c], N0, 0, 0, 0);
    N1 = __builtin_amdgcn_mfma_f64_16x16x4f64(a1[(G + E + 4 * c) * kWave], v[c], N1, 0, 0, 0);
  }
  // last slice of P: power G + e is stored for e < E, the monic 1 at e = E
  const double tail = e == E ? 1.0 : 0.0;
  const double l0 = e < E ? a0[4 * (kP - 1) * kWave] : tail;
  const double l1 = e < E ? a1[4 * (kP - 1) * kWave] : tail;
  P0 = __builtin_amdgcn_mfma_f64_16x16x4f64(l0, v[kP - 1], P0, 0, 0, 0);
  P1 = __builtin_amdgcn_mfma_f64_16x16x4f64(l1, v[kP - 1], P1, 0, 0, 0);
#pragma unroll
  for (int r = 0; r < 4; ++r) tot = __builtin_fma(N0[r], rcp64(P0[r]), tot);
#pragma unroll
  for (int r = 0; r < 4; ++r) tot = __builtin_fma(N1[r], rcp64(P1[r]), tot);
}

// Lane partial (four rows per 16-row slice, every slice of the table) of
// sum_r N_r(x)/P_r(x) for mass x = x_{lane % 16}; the whole wave takes part.
template <int G, int E>
__device__ __forceinline__ double mfma_fold_rows(const GridArgs &g, const double *lC, int lane,
                                                 double x, const FoldShape<G, E> &fs) {
  double v[MfmaShape<G, E>::kP];
  mfma_powers<G, E>(x, lane, v);
  double tot = 0.0;
  const int n_grp = g.T * fs.NG;
  for (int tg = 0; tg < n_grp; ++tg) {
    const double *grp = lC + tg * (2 * G + E) * kWave;
    mfma_slice_pair<G, E>(grp, lane, v, 0, 1, tot);
    mfma_slice_pair<G, E>(grp, lane, v, 2, 3, tot);
  }
  return tot;
}


// ------------------------------------------------ vertex diagram --
// Lane rows are (radial, polar) node pairs pi = lane + 64 t (i = pi / n_a,
// j = pi mod n_a); a group is G azimuthal nodes l of one pair, weights nu_l,
// H_l = Hk(s2_ijl); with H1 = Hk(s1_ij) the group's share of the result is
//   c_i mu_j/(Hq_i + x)^2/(H1 + x) sum_l nu_l/(x + H_l) = N(x)/P(x),
//   P = (x + Hq_i)^2 (x + H1) prod_l (x + H_l)  (monic, degree G + 3),
//   N = c_i mu_j sum_l nu_l prod_{l' != l}(x + H_l')  (degree G - 1),
// in the scaled units of the two-point form (N/P carries kap / sig^4).
template <int REG>
__device__ __forceinline__ double vertex_s2(double q, double p2, double x, double sx, double cph,
                                            double ct, double st) {
  return fmax((q * q + p2 * p2) + (2.0 * q) * p2 * (x * ct + (sx * cph) * st), 0.0);
}

template <int REG, int G>
__device__ void vertex_fill(const GridArgs &g, double *lC, const double *lc, const double *lq,
                            const double *lqn, const double *lx, const double *lm,
                            const double *lsx, const double *lcp, const double *lnu, double p1,
                            double p2, double ct, double st, const FoldShape<G, 3> &fs) {
  const int n_pairs = g.n_r * g.n_a;
  const int n_grp = g.T * fs.NG;
  {
    // as in grid_fill_fold: a thread keeps its lane and steps (t, gi, k);
    // its pair (i, j) changes with t only
    const int l = threadIdx.x & (kWave - 1);
    const int W = blockDim.x / kWave;
    int k = threadIdx.x / kWave, gi = 0, t = 0;
    while (k >= G) {
      k -= G;
      if (++gi == fs.NG) {
        gi = 0;
        ++t;
      }
    }
    int pi = l + kWave * t;
    int i = pi / g.n_a, j = pi - i * g.n_a;
    for (int row = threadIdx.x / kWave; row < n_grp * G; row += W) {
      const int az = gi * G + k;
      double H = 0.0;
      if (pi < n_pairs && az < g.n_phi) {
        const double s2 = vertex_s2<REG>(lqn[i], p2, lx[j], lsx[j], lcp[az], ct, st);
        H = g.sig * hk<REG>(s2, g.k2, g.inv_k2);
      }
      lC[((t * fs.NG + gi) * (2 * G + 3) + k) * kWave + l] = H;
      k += W;
      bool moved = false;
      while (k >= G) {
        k -= G;
        if (++gi == fs.NG) {
          gi = 0;
          ++t;
          moved = true;
        }
      }
      if (moved) {
        pi = l + kWave * t;
        i = pi / g.n_a;
        j = pi - i * g.n_a;
      }
    }
  }
  __syncthreads();
  for (int task = threadIdx.x; task < kWave * n_grp; task += blockDim.x) {
    const int l = task & (kWave - 1);
    const int tg = task / kWave;
    const int t = tg / fs.NG, gi = tg - t * fs.NG;
    const int pi = l + kWave * t;
    const bool vp = pi < n_pairs;
    const int i = vp ? pi / g.n_a : 0, j = vp ? pi - i * g.n_a : 0;
    double *col = lC + tg * (2 * G + 3) * kWave + l;
    double P[G + 4], N[G];
#pragma unroll
    for (int m = 0; m < G + 4; ++m) P[m] = 0.0;
#pragma unroll
    for (int m = 0; m < G; ++m) N[m] = 0.0;
#pragma unroll
    for (int k = 0; k < G; ++k) {
      const double H = col[k * kWave];
      const int az = gi * G + k;
      const double mu = (vp && az < g.n_phi) ? lnu[az] : 0.0;
      // N <- N (x + H) + mu P, then P <- P (x + H), as for the two-point form
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
        P[k + 1] = 1.0;
#pragma unroll
        for (int m = G; m >= 1; --m)
          if (m <= k) P[m] = __builtin_fma(H, P[m], P[m - 1]);
        P[0] = H * P[0];
      }
    }
    // P <- P (x + Hq)^2 (x + H1), N <- c_i mu_j N
    double q = 0.0, H1 = 0.0;
    if (vp) {
      q = lqn[i];
      const double s1 = fmax((q * q + p1 * p1) + (2.0 * q) * p1 * lx[j], 0.0);
      H1 = g.sig * hk<REG>(s1, g.k2, g.inv_k2);
    }
    const double Hq = vp ? g.sig * lq[i] : 0.0;
    const double c = vp ? (g.kap * lc[i]) * lm[j] : 0.0;
#pragma unroll
    for (int r = 0; r < 3; ++r) {
      const double f = r < 2 ? Hq : H1;
      const int deg = G + r;  // P[deg] = 1
      P[deg + 1] = 1.0;
#pragma unroll
      for (int m = G + 2; m >= 1; --m)
        if (m <= deg) P[m] = __builtin_fma(f, P[m], P[m - 1]);
      P[0] = f * P[0];
    }
#pragma unroll
    for (int m = 0; m < G + 3; ++m) col[m * kWave] = P[m];
#pragma unroll
    for (int m = 0; m < G; ++m) col[(G + 3 + m) * kWave] = c * N[m];
  }
}

// Lane partial of one vertex mass outside the coefficient range: every term
// on its own.
template <int REG>
__device__ __forceinline__ double vertex_single_mass(const GridArgs &g, const double *lc,
                                                  const double *lq, const double *lx,
                                                  const double *lm, const double *lsx,
                                                  const double *lcp, const double *lnu, int lane,
                                                  double p1, double p2, double ct, double st,
                                                  double delta) {
  const int n_pairs = g.n_r * g.n_a;
  double total = 0.0;
  for (int t = 0; t < g.T; ++t) {
    const int pi = lane + kWave * t;
    if (pi >= n_pairs) break;
    const int i = pi / g.n_a, j = pi - i * g.n_a;
    const double q = g.tab[i];
    const double Gq = rcp64(lq[i] + delta);
    const double A = (lc[i] * Gq) * Gq;
    const double s1 = fmax((q * q + p1 * p1) + (2.0 * q) * p1 * lx[j], 0.0);
    const double G1 = rcp64(hk<REG>(s1, g.k2, g.inv_k2) + delta);
    double inner = 0.0;
    for (int az = 0; az < g.n_phi; ++az) {
      const double s2 = vertex_s2<REG>(q, p2, lx[j], lsx[j], lcp[az], ct, st);
      inner = __builtin_fma(lnu[az], rcp64(hk<REG>(s2, g.k2, g.inv_k2) + delta), inner);
    }
    total = __builtin_fma((A * lm[j]) * G1, inner, total);
  }
  return total;
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
