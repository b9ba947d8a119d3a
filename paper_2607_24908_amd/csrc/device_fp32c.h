// Compensated-FP32 point path (FRG_PREC_FP32C) of the flow-diagram
// quadrature.
//
// On gfx950 an unpacked FP32 FMA issues at the FP64 rate, so FP32 saves time
// only where one FP32 operation replaces a sequence of FP64 ones: the
// exponential of the exponential regulator (the table-driven e^{-y} of the
// FP64 point kernels costs about fifteen FP64 operations per term).  The FP32C
// point path is therefore the FP64 point path (device_fp64.h: the same lane
// map, E-form fraction, running fractions of eight, FP64 radial factors and
// cross-lane reduction) with e^{-y} taken from the FP32 hardware exp2 and
// corrected to first order in FP64 (exp_neg32), and with the Bernoulli series
// up to y = 1 (below it the E-form would magnify the FP32 error of E).
//
// Error bound.  Only E carries an FP32 error: |dE| <= eps E with
// eps = kExpRel, the hardware exp2's accuracy (1 ulp of FP32).  A term
// t = mu (1 - E)/num, num = (y - 1 + E) + dhat (1 - E), moves by
//   |dt| <= t |dE| (1/(1 - E) + |1 - dhat|/num) <= t eps E B1,
//   B1 = 1/(1 - e^{-1}) + |1 - dhat|/(e^{-1} + dhat (1 - e^{-1})),
// for y >= 1 (E <= e^{-1} and num increases with y).  The y of a lane's group
// ascend (ascending angular nodes), so the group's first E bounds all of its
// E-form terms (e^{-1} when the first term is a series term), and
//   |dI| / I <= eps B1 sum_rows A_i sum_groups Ebar_g g / I + kSerRel,
// with kSerRel covering the truncation of the FP64 series on [0, 1)
// (below 1e-9 relative per term) and the FP64 roundings.  The bound is
// deterministic (to first order in eps): a result is returned from this path
// only when it is at most the caller's tolerance f32_flag; otherwise the
// point is evaluated by the FP64 point path, as are points with
// dhat < f32_band and every point of the Litim regulator (whose terms have
// no transcendental to save).  FP64 results are the bits of the FP64 kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>

#include "device_fp64.h"
#include "frg_internal.h"

#pragma clang fp contract(off)

namespace frg {
namespace dev {

constexpr double kErr64 = 1e-14;  // reported for FP64 results
// Relative accuracy of v_exp_f32: 1 ulp of FP32 (<= 2^-23 relative), with a
// margin for the first-order correction (O(r^2), r <= 2^-24 1.5 y).
constexpr double kExpRel = 1.2e-7;
// Truncation of h_series on [0, 1) (B_12 y^12/12! / h(1) = 9.1e-10) and the
// FP64 roundings of a result.
constexpr double kSerRel = 1e-9 + 1e-13;
constexpr double kY1 = 1.0;                       // series below, E-form above
constexpr double kLog2E = 1.4426950408889634;     // log2(e)
constexpr double kLn2 = 0.6931471805599453;       // ln(2)
constexpr double kEm1 = 0.36787944117144233;      // e^{-1}

// e^{-y} (y >= 0) from the FP32 hardware exp2: xf = fl32(-y log2 e),
// e = 2^xf within 1 ulp; the residual r = -y - xf ln2 (exact to FP64
// rounding, |r| <= 2^-24 1.45 y) gives e^{-y} = e e^r = e (1 + r + O(r^2)).
// 0 (or an FP32 subnormal) beyond y = 87, where its absolute error is below
// 2^-126.
__device__ __forceinline__ double exp_neg32(double y) {
  const float xf = (float)(y * -kLog2E);
  const double e = (double)__builtin_amdgcn_exp2f(xf);
  const double r = __builtin_fma((double)xf, -kLn2, -y);
  return __builtin_fma(e, r, e);
}

// E-form of one term with the FP32 exponential: a/b = mu (1 - E)/num
// (valid for y >= kY1; finite for any y >= 0).
__device__ __forceinline__ void frac_e32(double y, double mu, double cm, double cp, double &a,
                                         double &b, double &E) {
  E = exp_neg32(y);
  b = __builtin_fma(E, cp, y + cm);
  a = __builtin_fma(-mu, E, mu);
}

// B1 of the bound for one point (dh = dhat); the reciprocals' relative
// errors (~1e-16) are covered by the margin of kExpRel.
__device__ __forceinline__ double bound_b1(double dh) {
  constexpr double kInv1mEm1 = 1.5819767068693265;  // 1/(1 - e^{-1})
  return __builtin_fma(fabs(1.0 - dh), rcp64(__builtin_fma(dh, 1.0 - kEm1, kEm1)), kInv1mEm1);
}

// Lane partial of one point of the exponential regulator with the FP32
// exponential: returns sum_t A_t inner_t and sets *ebar to
// sum_t A_t sum_g Ebar_g g (the bound's sum).  Tables as for lane_point.
template <int JT>
__device__ __forceinline__ double lane_point_e32(const double *__restrict__ tab,
                                                 const double2 *__restrict__ ang, const SetDev &s,
                                                 int lane, double p, double delta, double *ebar) {
  const int n_r = s.n_r, n_a = s.n_a;
  const double *tq = tab;
  const double *tc = tab + n_r;
  const double *tH = tab + 2 * n_r;
  const int J = JT ? JT : s.J;
  const int rho = lane & (s.R - 1);
  const int iota = JT == 1 ? 0 : lane / s.R;
  const double2 *al = ang + iota;
  const double dh = delta * s.inv_k2;
  const double cm = dh - 1.0, cp = 1.0 - dh;
  const int G = point_chain_ok<kExp>(s, p, delta) ? grouped_u(n_a, J) : 0;
  double total = 0.0, etot = 0.0;
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
    double inner = 0.0, einner = 0.0;
    int u = 0;
    for (; u < G; u += kGroup) {
      const double2 *ag = al + J * u;
      double N = 0.0, P = 1.0, E0 = kEm1;
#pragma unroll
      for (int h = 0; h < kGroup; h += kHalf) {
        double a[kHalf], b[kHalf], y[kHalf], mu[kHalf], E[kHalf];
#pragma unroll
        for (int k = 0; k < kHalf; ++k) {
          const double2 w = ag[J * (h + k)];
          y[k] = __builtin_fma(bh, w.x, ah);
          mu[k] = w.y;
        }
#pragma unroll
        for (int k = 0; k < kHalf; ++k) frac_e32(y[k], mu[k], cm, cp, a[k], b[k], E[k]);
        if (h == 0) E0 = y[0] < kY1 ? kEm1 : E[0];
        // y[0] is the smallest y of the half: lanes below kY1 (if any in the
        // wave) take the series
        if (__builtin_amdgcn_ballot_w64(y[0] < kY1)) {
#pragma unroll
          for (int k = 0; k < kHalf; ++k) {
            const bool lo = y[k] < kY1;
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
      const double g = N * rcp64(P);
      inner = inner + g;
      einner = __builtin_fma(E0, g, einner);
    }
    for (; u < s.U; ++u) {
      const int j = iota + J * u;
      if (j < n_a) {
        const double2 w = al[J * u];
        const double y = __builtin_fma(bh, w.x, ah);
        double a, b, E;
        if (y < kY1) {
          b = h_series(y) + dh;
          a = w.y;
          E = 0.0;
        } else {
          frac_e32(y, w.y, cm, cp, a, b, E);
        }
        // b is +inf only for momenta beyond the grouped range: the term is 0
        const double tv = b < INFINITY ? a * rcp64(b) : 0.0;
        inner = inner + tv;
        einner = __builtin_fma(E, tv, einner);
      }
    }
    total = __builtin_fma(A, inner, total);
    etot = __builtin_fma(A, einner, etot);
  }
  *ebar = etot;
  return total;
}

__device__ __forceinline__ double e32_partial(const double *tab, const double2 *ang,
                                              const SetDev &s, int lane, double p, double delta,
                                              double *ebar) {
  if (s.J == 1) return lane_point_e32<1>(tab, ang, s, lane, p, delta, ebar);
  if (s.J == 2) return lane_point_e32<2>(tab, ang, s, lane, p, delta, ebar);
  return lane_point_e32<0>(tab, ang, s, lane, p, delta, ebar);
}

// Lane l's value of a double, wave-uniform.
__device__ __forceinline__ double readlane64(double v, int l) {
  const unsigned long long b = __builtin_bit_cast(unsigned long long, v);
  const int lo = __builtin_amdgcn_readlane((int)(unsigned)b, l);
  const int hi = __builtin_amdgcn_readlane((int)(unsigned)(b >> 32), l);
  return __builtin_bit_cast(double, ((unsigned long long)(unsigned)hi << 32) | (unsigned)lo);
}

// One tile of `count` (<= 64) points of an FP32C set of the exponential
// regulator; lane e holds point e's inputs (pv, mv).  A point with
// dhat >= f32_band takes the FP32-exponential path; it is kept when its bound
// is at most f32_flag, else evaluated by the FP64 point path, as are the
// points near the pole.  Points go two at a time: their partials and bound
// sums are reduced together (wave_sum_fold<4>; a partial's bits are those of
// any other fold width, so an FP64 result has the bits of the FP64 kernels).
// Lane 0 stores out, err (the bound, or kErr64) and used64.
__device__ void fp32c_tile(const SetDev &s, const double *tab, const double2 *ang,
                           const double *etab, int64_t start, int count, double pv, double mv,
                           int lane, int *flag) {
  constexpr int F = 2;
  for (int e0 = 0; e0 < count; e0 += F) {
    const int nf = count - e0 < F ? count - e0 : F;
    double t0 = 0.0, t1 = 0.0, b0 = 0.0, b1 = 0.0;
    unsigned ok = 0, x32 = 0;
#pragma unroll 1
    for (int f = 0; f < nf; ++f) {
      const double p = readlane64(pv, e0 + f);
      const double delta = readlane64(mv, e0 + f) + s.k2;
      double part = 0.0, eb = 0.0;
      if (delta > 0.0 && p >= 0.0) {  // wave-uniform
        ok |= 1u << f;
        if (delta * s.inv_k2 >= s.f32_band) {
          part = e32_partial(tab, ang, s, lane, p, delta, &eb);
          x32 |= 1u << f;
        } else {
          part = point_partial<kExp>(s, tab, ang, etab, lane, p, delta);
        }
      } else if (lane == 0) {
        *flag = 1;
      }
      t0 = f == 0 ? part : t0;
      t1 = f == 1 ? part : t1;
      b0 = f == 0 ? eb : b0;
      b1 = f == 1 ? eb : b1;
    }
    // lanes 0-15: point e0, 16-31: point e0 + 1, 32-47 / 48-63: their bound sums
    const double v[4] = {t0, t1, b0, b1};
    const double r = wave_sum_fold<4>(v, lane);
#pragma unroll 1
    for (int f = 0; f < nf; ++f) {
      double tot = readlane64(r, 16 * f);
      double est = kErr64;
      bool used = true;
      if ((x32 >> f) & 1u) {
        const double dh = (readlane64(mv, e0 + f) + s.k2) * s.inv_k2;
        est = kExpRel * bound_b1(dh) * (readlane64(r, 32 + 16 * f) * rcp64(tot)) + kSerRel;
        used = !(est <= s.f32_flag);  // a NaN bound goes to FP64 too
        if (used) {
          const double p = readlane64(pv, e0 + f);
          const double delta = readlane64(mv, e0 + f) + s.k2;
          const double part = point_partial<kExp>(s, tab, ang, etab, lane, p, delta);
          tot = readlane64(wave_sum_fold<1>(&part, lane), 0);
          est = kErr64;
        }
      }
      if (lane == 0) {
        const int64_t o = start + e0 + f;
        const bool okf = (ok >> f) & 1u;
        s.out[o] = okf ? s.pref_k * tot : __builtin_nan("");
        if (s.err) s.err[o] = okf ? est : __builtin_nan("");
        if (s.used64) s.used64[o] = (uint8_t)(okf && used);
      }
    }
  }
}

}  // namespace dev
}  // namespace frg
