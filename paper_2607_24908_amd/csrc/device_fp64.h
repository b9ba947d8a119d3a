// FP64 device routines shared by the kernels of libfrg (included by the
// .hip translation units only).
//
// Work per external point (p, m^2), delta = m^2 + k^2:
//   I = P_d sum_i A_i sum_j mu_j / D_ij,
//   A_i = c_i / (Hq_i + delta)^2,  c_i = w_i q_i^{d-1} d_tR(q_i^2),
//   D_ij = Hk(s_ij) + delta,  s_ij = (q_i - p)^2 + 2 q_i p (1 + x_j),
//   Hk(s) = k^2 h(s/k^2) (exponential regulator) or max(s - k^2, 0) (Litim).
//
// Lane map and summation order.  A wave of 64 lanes splits the nodes as
// R radial x J angular lanes (R = largest power of two <= min(n_r, 64),
// J = 64/R).  Lane (rho, iota) owns radial nodes i = rho + R t and angular
// nodes j = iota + J u (t < T, u < U, padded nodes contribute an exact 0).
// It accumulates  sum_t A_t (sum_u mu_u / D_tu)  in t and u order; the 64
// lane partials are then combined in a fixed order (the grid kernels'
// running-fraction form: the xor butterfly of wave_sum_split; the point
// kernels: wave_sum_fold).  The order thus depends only on (n_r, n_a): every
// launch form and tile choice of one kernel family gives bitwise-identical
// results for the same point.
//
// Reciprocal sums (grid kernels' running-fraction form, Litim point terms).
// With mu folded into the denominators, mu_j / D_ij = 1 / D'_ij,
// D'_ij = fma(delta, rmu_j, H'_ij),  H'_ij = fl(Hk(s_ij) rmu_j),
// rmu_j = 1/mu_j.  A lane takes its angular terms eight at a time by a running
// fraction N/P of positive numbers:
//   N <- 1, P <- D'_0;  then  N <- N D'_k + P,  P <- P D'_k  (k = 1..7),
// so sum_k 1/D'_k = N/P costs one multiply and one FMA per term plus one
// reciprocal per group.  The first G = 8 floor(floor(n_a/J)/8) values of u are
// grouped (every lane holds a real node there); the rest are taken one by one
// and padded nodes (j >= n_a) add nothing.  The grouped form is used when no
// product can leave the normal range: delta >= 1e-30 and
// ((q_top + p)^2 + delta) max_j rmu_j <= 1e37 (then 1e-243 < P, N < 1e297,
// because Hk(s) <= s <= (q_top + p)^2); otherwise every term gets its own
// reciprocal.  FP64 reciprocal: the hardware estimate (v_rcp_f64, relative
// error < 2^-24) and one Newton-Raphson step r <- r + r (1 - x r), relative
// error < 2.3e-15.
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>

#include "device_exp.h"
#include "frg_internal.h"

#pragma clang fp contract(off)

namespace frg {
namespace dev {

constexpr int kExp = FRG_REG_EXP;
constexpr int kLitim = FRG_REG_LITIM;

__device__ __forceinline__ double rcp64(double x) {
  const double r = __builtin_amdgcn_rcp(x);
  const double e = __builtin_fma(-x, r, 1.0);
  return __builtin_fma(r, e, r);
}

constexpr int kGroup = 8;
constexpr int kHalf = 4;  // terms computed together in the exponential groups

// Running fraction of one group: returns acc + sum_k 1/Dp[k].
__device__ __forceinline__ double chain_sum(const double *Dp, double acc) {
  double N = 1.0, P = Dp[0];
#pragma unroll
  for (int k = 1; k < kGroup; ++k) {
    N = __builtin_fma(N, Dp[k], P);
    P = P * Dp[k];
  }
  return __builtin_fma(N, rcp64(P), acc);
}

// Two running fractions in lockstep (the same operations as chain_sum on
// each; interleaving gives the FP64 pipeline two independent chains).
__device__ __forceinline__ void chain_sum2(const double *Da, const double *Db, double &acc_a,
                                           double &acc_b) {
  double Na = 1.0, Pa = Da[0], Nb = 1.0, Pb = Db[0];
#pragma unroll
  for (int k = 1; k < kGroup; ++k) {
    Na = __builtin_fma(Na, Da[k], Pa);
    Nb = __builtin_fma(Nb, Db[k], Pb);
    Pa = Pa * Da[k];
    Pb = Pb * Db[k];
    // keep the two chains interleaved (the scheduler would otherwise run
    // them one after the other)
    __builtin_amdgcn_sched_barrier(0);
  }
  const double ra = rcp64(Pa), rb = rcp64(Pb);
  acc_a = __builtin_fma(Na, ra, acc_a);
  acc_b = __builtin_fma(Nb, rb, acc_b);
}

// Whether the grouped form is safe for this point (same test in every kernel).
__device__ __forceinline__ bool chain_ok(double delta, double p, double q_top, double rmu_max) {
  const double qp = q_top + p;
  return delta >= 1e-30 && __builtin_fma(qp, qp, delta) * rmu_max <= 1e37;
}

// Number of grouped angular steps u (a multiple of kGroup, <= U).
__device__ __forceinline__ int grouped_u(int n_a, int J) {
  const int umin = n_a / J;
  return umin - umin % kGroup;
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, kWave);
  return v;
}

// wave_sum of M values at once (M a power of two, 1..64).  The first log2 M
// exchange steps halve the number of live values: at offset o a lane keeps
// the half of its values selected by its bit o and receives the partner's
// partial sums of that half; the remaining steps are the plain butterfly.
// Every partial sum is the one wave_sum forms (own + partner at offsets
// 32, 16, ..., 1), so lane l returns, bit for bit, wave_sum(v[l / (64/M)]).
template <int M>
__device__ __forceinline__ double wave_sum_split(const double *v, int lane) {
  constexpr int kSteps = (M >= 64) ? 6 : (M >= 32) ? 5 : (M >= 16) ? 4 : (M >= 8) ? 3
                                                        : (M >= 4) ? 2 : (M >= 2) ? 1 : 0;
  static_assert((1 << kSteps) == M, "M must be a power of two <= 64");
  double w[M];
#pragma unroll
  for (int m = 0; m < M; ++m) w[m] = v[m];
#pragma unroll
  for (int s = 0; s < kSteps; ++s) {
    const int off = 32 >> s;
    const int h = M >> (s + 1);
    const bool upper = (lane & off) != 0;
#pragma unroll
    for (int k = 0; k < h; ++k) {
      double lo = w[k], hi = w[h + k];
      // pin both values in registers: a select between two loads of w would
      // otherwise become one load at a lane-dependent index of w
      asm("" : "+v"(lo), "+v"(hi));
      const double keep = upper ? hi : lo;
      const double send = upper ? lo : hi;
      w[k] = keep + __shfl_xor(send, off, kWave);
    }
  }
  double x = w[0];
#pragma unroll
  for (int s = kSteps; s < 6; ++s) x += __shfl_xor(x, 32 >> s, kWave);
  return x;
}

// ------------------------------------------- cross-lane sums (gfx950) --
// Lane permutations of a double: DPP within rows of 16 lanes (CTRL: 0xB1
// swaps neighbours, 0x4E swaps pairs, 0x141 mirrors each half-row, 0x128
// rotates each row by 8) and the gfx950 lane swaps (half-waves, odd/even
// rows), each moving the two 32-bit halves separately.
template <int CTRL>
__device__ __forceinline__ double dpp_f64(double v) {
  const unsigned long long b = __builtin_bit_cast(unsigned long long, v);
  const int lo = __builtin_amdgcn_mov_dpp((int)(unsigned)b, CTRL, 0xf, 0xf, false);
  const int hi = __builtin_amdgcn_mov_dpp((int)(unsigned)(b >> 32), CTRL, 0xf, 0xf, false);
  return __builtin_bit_cast(double, ((unsigned long long)(unsigned)hi << 32) | (unsigned)lo);
}

// For values a, b in every lane, returns a' + b' where (a', b') is a and b
// with lanes [32, 64) of a exchanged with lanes [0, 32) of b (W32) or with
// rows 1 and 3 of a exchanged with rows 0 and 2 of b (W16): lane l gets
// a_l + a_{l+w} in the lower part of each 2w block and b_{l-w} + b_l in the
// upper part.
template <int W>
__device__ __forceinline__ double swap_add(double a, double b) {
  const unsigned long long ua = __builtin_bit_cast(unsigned long long, a);
  const unsigned long long ub = __builtin_bit_cast(unsigned long long, b);
  unsigned lo0, lo1, hi0, hi1;
  if constexpr (W == 32) {
    const auto rl = __builtin_amdgcn_permlane32_swap((unsigned)ua, (unsigned)ub, false, false);
    const auto rh = __builtin_amdgcn_permlane32_swap((unsigned)(ua >> 32), (unsigned)(ub >> 32), false, false);
    lo0 = rl[0]; lo1 = rl[1]; hi0 = rh[0]; hi1 = rh[1];
  } else {
    const auto rl = __builtin_amdgcn_permlane16_swap((unsigned)ua, (unsigned)ub, false, false);
    const auto rh = __builtin_amdgcn_permlane16_swap((unsigned)(ua >> 32), (unsigned)(ub >> 32), false, false);
    lo0 = rl[0]; lo1 = rl[1]; hi0 = rh[0]; hi1 = rh[1];
  }
  const double x = __builtin_bit_cast(double, ((unsigned long long)hi0 << 32) | lo0);
  const double y = __builtin_bit_cast(double, ((unsigned long long)hi1 << 32) | lo1);
  return x + y;
}

// Sums of M values (M = 1, 2, 4, 8) over the 64 lanes at once.  The pairing
// is the same for every M: lane offsets 32, 16, 8, then 1, 2 and 4 (as the
// half-row mirror, equivalent once each quad holds equal values), each step
// own + partner.  The first log2 M steps halve the number of live values (a
// lane keeps the half selected by the offset's bit of its index), so every
// lane ends with the total of one value, the same bits for every M: value
// fold_owner<M>(lane) = lane / (64/M); fold_leader<M>(lane) marks one lane
// per value.
template <int M>
__device__ __forceinline__ int fold_owner(int lane) {
  return lane / (64 / M);
}
template <int M>
__device__ __forceinline__ bool fold_leader(int lane) {
  return lane % (64 / M) == 0;
}

// Split step at offset 8 (DPP rotation by 8 within a row of 16): a lane
// keeps w[k] or w[h + k] by bit 3 of its index and adds the partner's copy
// of the same value.
template <int CTRL, int BIT>
__device__ __forceinline__ double split_dpp(double lo, double hi, int lane) {
  asm("" : "+v"(lo), "+v"(hi));
  const bool upper = (lane & BIT) != 0;
  const double keep = upper ? hi : lo;
  const double send = upper ? lo : hi;
  return keep + dpp_f64<CTRL>(send);
}

template <int M>
__device__ __forceinline__ double wave_sum_fold(const double *v, int lane) {
  static_assert(M == 1 || M == 2 || M == 4 || M == 8, "M must be 1, 2, 4 or 8");
  double w[M];
#pragma unroll
  for (int m = 0; m < M; ++m) w[m] = v[m];
  // offset 32
  if constexpr (M >= 2) {
#pragma unroll
    for (int k = 0; k < M / 2; ++k) w[k] = swap_add<32>(w[k], w[M / 2 + k]);
  } else {
    w[0] = swap_add<32>(w[0], w[0]);
  }
  // offset 16
  if constexpr (M >= 4) {
#pragma unroll
    for (int k = 0; k < M / 4; ++k) w[k] = swap_add<16>(w[k], w[M / 4 + k]);
  } else {
    w[0] = swap_add<16>(w[0], w[0]);
  }
  // offset 8 (rotation by 8 within a row of 16 is the exchange of offset 8)
  double x;
  if constexpr (M >= 8) {
#pragma unroll
    for (int k = 0; k < M / 8; ++k) w[k] = split_dpp<0x128, 8>(w[k], w[M / 8 + k], lane);
  } else {
    w[0] = w[0] + dpp_f64<0x128>(w[0]);
  }
  x = w[0] + dpp_f64<0xB1>(w[0]);  // offset 1
  x = x + dpp_f64<0x4E>(x);
  x = x + dpp_f64<0x141>(x);
  return x;
}

// h(y) = y/(1 - e^{-y}) - 1; Bernoulli series y/2 + y^2/12 - y^4/720 + ...
// below y = 0.1 (truncation < 1e-17 relative there).
__device__ __forceinline__ double h_exp(double y) {
  if (y < 0.1) {
    const double y2 = y * y;
    double t = __builtin_fma(y2, 1.0 / 47900160.0, -1.0 / 1209600.0);
    t = __builtin_fma(y2, t, 1.0 / 30240.0);
    t = __builtin_fma(y2, t, -1.0 / 720.0);
    t = __builtin_fma(y2, t, 1.0 / 12.0);
    return __builtin_fma(y2, t, 0.5 * y);
  }
  const double em = expm1(-y);  // in (-1, -0.095]
  return y * rcp64(-em) - 1.0;
}

template <int REG>
__device__ __forceinline__ double hk(double s, double k2, double inv_k2) {
  if constexpr (REG == kExp) {
    return k2 * h_exp(s * inv_k2);
  } else {
    return fmax(s - k2, 0.0);
  }
}

// ---------------------------------------------------- point kernels --
// Lane partial of one external point for the point-list kernels (plain and
// persistent, and the FP64 path of FRG_PREC_FP32C sets).  The sum is
// formed in units of k^2: with y = s/k^2 and dhat = delta/k^2,
//   mu_j / D_ij = (1/k^2) mu_j / (hh(y_ij) + dhat),   y_ij = ah_i + bh_i (1 + x_j),
//   ah_i = (q_i - p)^2 / k^2,  bh_i = 2 q_i p / k^2,
// hh(y) = h(y) (exponential) or max(y - 1, 0) (Litim); the factor 1/k^2 is in
// SetDev::pref_k.
//
// Exponential regulator.  Below y = kY0 the Bernoulli series of h.  Above,
// with E = e^{-y} (exp_neg, table-driven),
//   h(y) + dhat = num / (1 - E),   num = (y + dhat - 1) + E (1 - dhat),
// so that each term is a fraction a/b with a = mu_j (1 - E) and b = num: the
// division inside h joins the running fraction of the group, and no expm1 or
// reciprocal is spent per term.  num cancels at most by a factor
// (|y + dhat - 1| + E |1 - dhat|) / num <= 53 (at y = kY0, dhat -> 0), so a
// term keeps a relative error below ~60 u.
// The terms of a lane are taken eight at a time as a running fraction
//   N/P = sum_k a_k / b_k:  N <- a_0, P <- b_0;  N <- N b_k + a_k P,  P <- P b_k,
// (three operations per term, one reciprocal per eight), all of them
// positive.  The range test exp_chain_ok keeps every N and P normal
// (b >= min(dhat, 0.028), a >= mu_min (1 - e^{-kY0}), b <= y_top + dhat).
// Litim: b_k = (max(y - 1, 0) + dhat) / mu_j as before (two operations per
// term, mu in the denominator).
//
// Lane map and order: as at the top of this file (R radial x J angular lanes,
// (t, u) order within a lane); the cross-lane sum is wave_sum_fold, whose
// pairing is the same for tiles of 1, 2, 4 or 8 points, so every point
// kernel returns the same bits for the same point.
constexpr double kY0 = 0.25;

// h(y) for 0 <= y < kY0: y/2 + y^2/12 - y^4/720 + y^6/30240 - y^8/1209600
// + y^10/47900160, truncation < 3e-19 relative at y = kY0.
__device__ __forceinline__ double h_series(double y) {
  const double y2 = y * y;
  double t = __builtin_fma(y2, 1.0 / 47900160.0, -1.0 / 1209600.0);
  t = __builtin_fma(y2, t, 1.0 / 30240.0);
  t = __builtin_fma(y2, t, -1.0 / 720.0);
  t = __builtin_fma(y2, t, 1.0 / 12.0);
  return __builtin_fma(y2, t, 0.5 * y);
}

// The E-form of exp_frac alone (a valid fraction for y >= kY0; finite for
// any y >= 0, so that it can be computed for a whole group and replaced).
__device__ __forceinline__ void exp_frac_e(double y, double mu, double cm, double cp,
                                           const double *etab, double &a, double &b) {
  const double E = exp_neg(y, etab);
  b = __builtin_fma(E, cp, y + cm);
  a = __builtin_fma(-mu, E, mu);
}

// a/b = mu / (h(y) + dhat) (exponential regulator); cm = dhat - 1, cp = 1 - dhat.
__device__ __forceinline__ void exp_frac(double y, double mu, double dh, double cm, double cp,
                                         const double *etab, double &a, double &b) {
  if (y < kY0) {
    b = h_series(y) + dh;
    a = mu;
  } else {
    const double E = exp_neg(y, etab);
    b = __builtin_fma(E, cp, y + cm);
    a = __builtin_fma(-mu, E, mu);
  }
}

// Every N, P of the grouped forms stays normal: dhat >= 1e-30 and
// (y_top + dhat) (Litim: times max 1/mu) <= 1e37, y_top = (q_top + p)^2/k^2.
template <int REG>
__device__ __forceinline__ bool point_chain_ok(const SetDev &s, double p, double delta) {
  const double qp = s.q_top + p;
  const double top = __builtin_fma(qp, qp, delta) * s.inv_k2;
  const double dh = delta * s.inv_k2;
  return dh >= 1e-30 && (REG == kExp ? top : top * s.rmu_max) <= 1e37;
}

// LDS layout of the point kernels: kExp2Tab64 (kExpTab doubles), the
// angular pairs of the current set, then its packed table (table_doubles).
// Pair j is (1 + x_j, mu_j) for the exponential regulator and
// (1 + x_j, 1/mu_j) for Litim: one 16-byte read per term.
__device__ __forceinline__ int point_lds_doubles(int n_r, int n_a) {
  return kExpTab + 2 * n_a + table_doubles(n_r, n_a);
}

__device__ __forceinline__ void stage_pairs(const SetDev &s, double2 *ang, int tid, int nthreads) {
  const double *o = s.tab + 3 * s.n_r;
  const double *w = o + (s.reg == kExp ? s.n_a : 2 * s.n_a);
  for (int j = tid; j < s.n_a; j += nthreads) ang[j] = make_double2(o[j], w[j]);
}

// `tab`: the packed quadrature table, `ang`: the angular pairs, `etab`:
// kExp2Tab64, all in LDS.  JT: the lane split J when fixed at compile time
// (1 or 2), else 0 (J from the set).
template <int REG, int JT>
__device__ __forceinline__ double lane_point(const double *__restrict__ tab,
                                             const double2 *__restrict__ ang,
                                             const double *__restrict__ etab, const SetDev &s,
                                             int lane, double p, double delta) {
  const int n_r = s.n_r, n_a = s.n_a;
  const double *tq = tab;
  const double *tc = tab + n_r;
  const double *tH = tab + 2 * n_r;
  const int J = JT ? JT : s.J;
  const int rho = lane & (s.R - 1);
  const int iota = JT == 1 ? 0 : lane / s.R;
  const double2 *al = ang + iota;  // the lane's angular nodes: al[J u]
  const double dh = delta * s.inv_k2;
  const double cm = dh - 1.0, cp = 1.0 - dh;
  const int G = point_chain_ok<REG>(s, p, delta) ? grouped_u(n_a, J) : 0;
  double total = 0.0;
  for (int t = 0; t < s.T; ++t) {
    const int i = rho + s.R * t;
    const bool vi = i < n_r;
    const double q = vi ? tq[i] : 0.0;
    const double c = vi ? tc[i] : 0.0;
    const double Hq = vi ? tH[i] : 1.0;
    const double Gq = rcp64(Hq + delta);
    const double A = (c * Gq) * Gq;
    const double qm = q - p;
    const double ah = (qm * qm) * s.inv_k2;
    const double bh = ((2.0 * q) * p) * s.inv_k2;
    const double ah1 = ah - 1.0;
    double inner = 0.0;
    int u = 0;
    for (; u < G; u += kGroup) {
      const double2 *ag = al + J * u;
      if constexpr (REG == kExp) {
        // two halves of four terms (fewer live registers); the same
        // operations in the same order as one pass over eight
        double N = 0.0, P = 1.0;
#pragma unroll
        for (int h = 0; h < kGroup; h += kHalf) {
          double a[kHalf], b[kHalf], y[kHalf], mu[kHalf];
#pragma unroll
          for (int k = 0; k < kHalf; ++k) {
            const double2 w = ag[J * (h + k)];
            y[k] = __builtin_fma(bh, w.x, ah);
            mu[k] = w.y;
          }
#pragma unroll
          for (int k = 0; k < kHalf; ++k) exp_frac_e(y[k], mu[k], cm, cp, etab, a[k], b[k]);
          // the angular nodes ascend, so y[0] is the smallest y of the half;
          // lanes below kY0 (if any in the wave) take the series instead
          if (__builtin_amdgcn_ballot_w64(y[0] < kY0)) {
#pragma unroll
            for (int k = 0; k < kHalf; ++k) {
              const bool lo = y[k] < kY0;
              const double bs = h_series(y[k]) + dh;
              b[k] = lo ? bs : b[k];
              a[k] = lo ? mu[k] : a[k];
            }
          }
#pragma unroll
          for (int k = 0; k < kHalf; ++k) {
            if (h == 0 && k == 0) {
              N = a[0];
              P = b[0];
            } else {
              N = __builtin_fma(N, b[k], a[k] * P);
              P = P * b[k];
            }
          }
        }
        inner = __builtin_fma(N, rcp64(P), inner);
      } else {
        double2 w[kGroup];
#pragma unroll
        for (int k = 0; k < kGroup; ++k) w[k] = ag[J * k];
        double Dp[kGroup];
#pragma unroll
        for (int k = 0; k < kGroup; ++k) {
          const double H = fmax(__builtin_fma(bh, w[k].x, ah1), 0.0) * w[k].y;
          Dp[k] = __builtin_fma(dh, w[k].y, H);
        }
        inner = chain_sum(Dp, inner);
      }
    }
    for (; u < s.U; ++u) {
      const int j = iota + J * u;
      if (j < n_a) {
        const double2 w = al[J * u];
        if constexpr (REG == kExp) {
          double a, b;
          const double y = __builtin_fma(bh, w.x, ah);
          exp_frac(y, w.y, dh, cm, cp, etab, a, b);
          // b is +inf only for momenta beyond the grouped range: the term is 0
          inner = inner + (b < INFINITY ? a * rcp64(b) : 0.0);
        } else {
          const double H = fmax(__builtin_fma(bh, w.x, ah1), 0.0) * w.y;
          const double D = __builtin_fma(dh, w.y, H);
          inner = inner + (D < INFINITY ? rcp64(D) : 0.0);
        }
      }
    }
    total = __builtin_fma(A, inner, total);
  }
  return total;
}

// lane_point with the lane split of the set.
template <int REG>
__device__ __forceinline__ double point_partial(const SetDev &s, const double *tab,
                                                const double2 *ang, const double *etab, int lane,
                                                double p, double delta) {
  if (s.J == 1) return lane_point<REG, 1>(tab, ang, etab, s, lane, p, delta);
  if (s.J == 2) return lane_point<REG, 2>(tab, ang, etab, s, lane, p, delta);
  return lane_point<REG, 0>(tab, ang, etab, s, lane, p, delta);
}

}  // namespace dev
}  // namespace frg
