// Compensated-FP32 path (FRG_PREC_FP32C) of the flow-diagram quadrature.
//
// Per external point the angular bulk  sum_j mu_j / D_ij  runs in FP32 and
// is accumulated with the two-sum (error-free addition) compensation; the
// per-radial-node factors A_i = c_i/(Hq_i + delta)^2, the sum over radial
// nodes and the cross-lane reduction are FP64.  The FP32 part is
// scale-free: with y = s/k^2 and dhat = delta/k^2,
//   D_ij / k^2 = h(y_ij) + dhat,   y_ij = a_i + b_i (1 + x_j),
//   a_i = (q_i - p)^2 / k^2,  b_i = 2 q_i p / k^2   (formed in FP64),
// and dhat and the angular weights mu_j enter as FP32 hi + lo pairs, so no
// rounding of an input is shared by all terms of a result.  For the Litim
// regulator every term with y <= 1 has D/k^2 = dhat exactly: those weights
// are summed apart and divided by dhat once in FP64.  Each term t carries independent rounding errors of
// order sigma_t = u (1 + y/D) relative (u = 2^-24; y/D is the sensitivity of
// D to the rounding of y, large for the Litim kink near y = 1); they add in
// quadrature, and err = kappa sqrt(sum (A t sigma_t)^2) / I + u/2 is the
// estimate returned for the result.  kappa = 3 and the floor u/2 were
// calibrated on MI355X against the FP64 oracle: over 11 216 points (d = 3, 4;
// both regulators; 8 x 4 to 128 x 32 nodes; dhat >= 1e-2) the estimate
// bounded 99.94 % of the observed errors, the largest of which was 7.1e-8.
// A point is evaluated in FP64 instead (bit-identical to the FP64 kernels)
// when it lies near the pole, dhat < f32_band (default 1e-2), or when err
// exceeds f32_flag (default 1e-7).
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>

#include "device_fp64.h"
#include "frg_internal.h"

#pragma clang fp contract(off)

namespace frg {
namespace dev {

constexpr float kU32 = 5.9604645e-08f;  // 2^-24
constexpr double kKappa = 3.0;          // multiplier of the statistical part
constexpr double kSys = 0.5 * 5.9604644775390625e-08;  // floor: coherent rounding, 0.5 u
constexpr double kErr64 = 1e-14;        // reported for FP64 results

__device__ __forceinline__ float rcp32(float x) {
  const float r = __builtin_amdgcn_rcpf(x);
  const float e = __builtin_fmaf(-x, r, 1.0f);
  return __builtin_fmaf(r, e, r);
}

// h(y) in FP32.  Exponential regulator: Bernoulli series below y = 1
// (truncation < 1e-10 relative), (y - 1 + e^{-y}) / (1 - e^{-y}) above,
// e^{-y} = 2^{-y log2 e} from the hardware exp2.  Litim: max(y - 1, 0).
template <int REG>
__device__ __forceinline__ float h32(float y) {
  if constexpr (REG == kExp) {
    if (y < 1.0f) {
      const float y2 = y * y;
      float t = __builtin_fmaf(y2, 1.0f / 47900160.0f, -1.0f / 1209600.0f);
      t = __builtin_fmaf(y2, t, 1.0f / 30240.0f);
      t = __builtin_fmaf(y2, t, -1.0f / 720.0f);
      t = __builtin_fmaf(y2, t, 1.0f / 12.0f);
      return __builtin_fmaf(y2, t, 0.5f * y);
    }
    const float e = __builtin_amdgcn_exp2f(-y * 1.44269504088896341f);
    return ((y - 1.0f) + e) * rcp32(1.0f - e);
  } else {
    return fmaxf(y - 1.0f, 0.0f);
  }
}

// s + t = s' + e exactly (Knuth); the error e is added to c.
__device__ __forceinline__ void two_sum(float &s, float t, float &c) {
  const float sN = s + t;
  const float bp = sN - s;
  c += (s - (sN - bp)) + (t - bp);
  s = sN;
}

// Lane partial of one point in compensated FP32: returns sum_t A'_t S_t in
// FP64 and accumulates the error variance.  tab: FP64 table in LDS;
// fo: 1 + x_j, fm / fl: mu_j as an FP32 hi + lo pair.
template <int REG>
__device__ __forceinline__ double lane_point_f32(const double *__restrict__ tab,
                                                 const float *__restrict__ fo,
                                                 const float *__restrict__ fm,
                                                 const float *__restrict__ fl, const SetDev &s,
                                                 int lane, double p, double delta, double *var) {
  const int n_r = s.n_r, n_a = s.n_a;
  const double *tq = tab;
  const double *tc = tab + n_r;
  const double *tH = tab + 2 * n_r;
  const int rho = lane & (s.R - 1);
  const int iota = lane / s.R;
  const double dhat = delta * s.inv_k2;
  const float dhi = (float)dhat;
  const float dlo = (float)(dhat - (double)dhi);
  const double rdhat = (REG == kLitim) ? 1.0 / dhat : 0.0;
  double total = 0.0, v64 = 0.0;
  for (int t = 0; t < s.T; ++t) {
    const int i = rho + s.R * t;
    const bool vi = i < n_r;
    const double q = vi ? tq[i] : 0.0;
    const double c = vi ? tc[i] : 0.0;
    const double Hq = vi ? tH[i] : 1.0;
    const double Gq = rcp64(Hq + delta);
    const double Ap = ((c * Gq) * Gq) * s.inv_k2;
    const double qm = q - p;
    const float ah = (float)((qm * qm) * s.inv_k2);
    const float bh = (float)(((2.0 * q) * p) * s.inv_k2);
    float S = 0.0f, C = 0.0f, V = 0.0f;
    float F = 0.0f, FC = 0.0f;  // Litim: sum of mu_j over the flat region y <= 1
    for (int u = 0; u < s.U; ++u) {
      const int j = iota + s.J * u;
      const bool vj = j < n_a;
      const float opx = vj ? fo[j] : 1.0f;
      const float mu = vj ? fm[j] : 0.0f;
      const float ml = vj ? fl[j] : 0.0f;
      const float y = __builtin_fmaf(bh, opx, ah);
      if (REG == kLitim && y <= 1.0f) {
        // D = dhat exactly: collect mu_j (hi + lo) and divide once in FP64
        two_sum(F, mu, FC);
        FC += ml;
        continue;
      }
      const float h = h32<REG>(y);
      const float D = (h + dlo) + dhi;
      const float r = rcp32(D);
      const float tt = __builtin_fmaf(ml, r, mu * r);
      two_sum(S, tt, C);
      const float sig = kU32 * __builtin_fmaf(y, r, 1.0f);
      const float et = tt * sig;
      V = __builtin_fmaf(et, et, V);
    }
    double inner = (double)S + (double)C;
    if (REG == kLitim) inner = __builtin_fma((double)F + (double)FC, rdhat, inner);
    total = __builtin_fma(Ap, inner, total);
    v64 = __builtin_fma(Ap * Ap, (double)V, v64);
  }
  *var = v64;
  return total;
}

template <int REG>
__device__ void fp32c_tile(const SetDev &s, const double *tab, const double2 *ang,
                           const double *etab, const float *fo, const float *fm, const float *fl,
                           int64_t start, int count, int64_t grid_nm, int lane, int *flag) {
  double res = 0.0, rerr = 0.0;
  int rused = 0;
  for (int e = 0; e < count; ++e) {
    const int64_t idx = start + e;
    const double p = grid_nm ? s.p[idx / grid_nm] : s.p[idx];
    const double m2 = grid_nm ? s.m2[idx % grid_nm] : s.m2[idx];
    const double delta = m2 + s.k2;
    double v, er;
    int used = 0;
    if (delta > 0.0 && p >= 0.0) {
      bool use64 = !(delta * s.inv_k2 >= s.f32_band);
      if (!use64) {
        double var;
        const double tot = wave_sum(lane_point_f32<REG>(tab, fo, fm, fl, s, lane, p, delta, &var));
        var = wave_sum(var);
        v = s.pref * tot;
        er = kKappa * sqrt(var) / tot + kSys;
        use64 = !(er <= s.f32_flag);
      }
      if (use64) {
        // the FP64 point-kernel path: the same bits as an FP64 set
        const double part = point_partial<REG>(s, tab, ang, etab, lane, p, delta);
        v = s.pref_k * wave_sum_fold<1>(&part, lane);
        er = kErr64;
        used = 1;
      }
    } else {
      v = __builtin_nan("");
      er = __builtin_nan("");
      if (lane == 0) *flag = 1;
    }
    if (lane == e) {
      res = v;
      rerr = er;
      rused = used;
    }
  }
  if (lane < count) {
    s.out[start + lane] = res;
    if (s.err) s.err[start + lane] = rerr;
    if (s.used64) s.used64[start + lane] = (uint8_t)rused;
  }
}

// Stage the FP64 table of set s and its FP32 angular tables (1 + x_j and
// mu_j as hi + lo) in LDS: the table (table_doubles) then fo, fm, fl.
__device__ __forceinline__ void stage_fp32c(const SetDev &s, double *tab, int tid, int nthreads) {
  const int ntab = table_doubles(s.n_r, s.n_a);
  float *fo = reinterpret_cast<float *>(tab + ntab);
  float *fm = fo + s.n_a;
  float *fl = fm + s.n_a;
  for (int i = tid; i < ntab; i += nthreads) tab[i] = s.tab[i];
  for (int j = tid; j < s.n_a; j += nthreads) {
    const double mu = s.tab[3 * s.n_r + s.n_a + j];
    fo[j] = (float)s.tab[3 * s.n_r + j];
    fm[j] = (float)mu;
    fl[j] = (float)(mu - (double)(float)mu);
  }
}

__host__ __device__ inline size_t fp32c_lds_bytes(int n_r, int n_a) {
  return sizeof(double) * table_doubles(n_r, n_a) + sizeof(float) * 3 * n_a;
}

}  // namespace dev
}  // namespace frg
