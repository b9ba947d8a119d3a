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
// It accumulates  sum_t A_t (sum_u mu_u / D_tu)  in t and u order, and the
// 64 lane partials are combined by a fixed xor butterfly.  The order thus
// depends only on (n_r, n_a): every kernel and tile choice below gives
// bitwise-identical results for the same point.
//
// Reciprocal sums: the angular terms of one lane are taken four at a time,
//   mu0/D0 + mu1/D1 + mu2/D2 + mu3/D3 = N/P,  P = (D0 D1)(D2 D3),
//   N = (mu0 D1 + mu1 D0)(D2 D3) + (mu2 D3 + mu3 D2)(D0 D1),
// so one reciprocal serves four terms (leftover u < U taken one by one).
// Every D >= delta > 0, so N and P are sums of positive products; the form is
// used when 1e-70 <= delta <= 1e70 (no over- or underflow of P), otherwise
// each term gets its own reciprocal.  FP64 reciprocal: the hardware estimate
// (v_rcp_f64, relative error < 2^-24) and one Newton-Raphson step
// r <- r + r (1 - x r), relative error < 2.3e-15.
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>

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

// mu/D for four terms with one reciprocal (see the header comment)
__device__ __forceinline__ double sum4(double D0, double D1, double D2, double D3, double m0,
                                       double m1, double m2, double m3, double acc) {
  const double P01 = D0 * D1, P23 = D2 * D3;
  const double N01 = __builtin_fma(m0, D1, m1 * D0);
  const double N23 = __builtin_fma(m2, D3, m3 * D2);
  const double P = P01 * P23;
  const double N = __builtin_fma(N01, P23, N23 * P01);
  return __builtin_fma(N, rcp64(P), acc);
}

__device__ __forceinline__ bool four_ok(double delta) { return delta >= 1e-70 && delta <= 1e70; }

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, kWave);
  return v;
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

// Lane partial of one point; `tab` is the packed table (LDS).
template <int REG>
__device__ __forceinline__ double lane_point(const double *__restrict__ tab, const SetDev &s,
                                             int lane, double p, double delta) {
  const int n_r = s.n_r, n_a = s.n_a;
  const double *tq = tab;
  const double *tc = tab + n_r;
  const double *tH = tab + 2 * n_r;
  const double *to = tab + 3 * n_r;
  const double *tm = to + n_a;
  const int rho = lane & (s.R - 1);
  const int iota = lane / s.R;
  const bool four = four_ok(delta);
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
    const double a = qm * qm;
    const double b = (2.0 * q) * p;
    double inner = 0.0;
    int u = 0;
    if (four) {
      for (; u + 4 <= s.U; u += 4) {
        double D[4], mu[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          const int j = iota + s.J * (u + k);
          const bool vj = j < n_a;
          mu[k] = vj ? tm[j] : 0.0;
          D[k] = hk<REG>(__builtin_fma(b, vj ? to[j] : 1.0, a), s.k2, s.inv_k2) + delta;
        }
        inner = sum4(D[0], D[1], D[2], D[3], mu[0], mu[1], mu[2], mu[3], inner);
      }
    }
    for (; u < s.U; ++u) {
      const int j = iota + s.J * u;
      const bool vj = j < n_a;
      const double opx = vj ? to[j] : 1.0;
      const double mu = vj ? tm[j] : 0.0;
      const double sij = __builtin_fma(b, opx, a);
      const double D = hk<REG>(sij, s.k2, s.inv_k2) + delta;
      inner = __builtin_fma(mu, rcp64(D), inner);
    }
    total = __builtin_fma(A, inner, total);
  }
  return total;
}

}  // namespace dev
}  // namespace frg
