// e^{-y} for the exponential regulator, on the device and on the host (the
// host copy backs frg_expneg, through which tests compare it with the C
// library's exp).
//
// Method: the table-driven exponential of P. T. P. Tang ("Table-driven
// implementation of the exponential function in IEEE floating-point
// arithmetic", ACM Trans. Math. Softw. 15 (1989) 144-157) with 64 table
// entries.  For x = -y:
//   N = rint(x 64/ln2) = 64 m + j  (0 <= j < 64),   r = x - N ln2/64,
//   e^x = 2^m 2^{j/64} e^r,   |r| <= ln2/128 < 0.0055.
//   - N: one FMA against the shift 1.5 2^52 rounds x 64/ln2 to an integer,
//     which the low word of the result holds in two's complement.
//   - r: Cody-Waite reduction with ln2/64 = L_hi + L_lo, L_hi carrying 32
//     significant bits, so that N L_hi is exact for |N| < 2^21 and
//     x - N L_hi is exact (Sterbenz); r = (x - N L_hi) - N L_lo in one more FMA.
//   - e^r - 1 = r (1 + r/2 + r^2/6 + r^3/24 + r^4/120), Taylor, truncation
//     < r^6/720 < 3.5e-17 relative.
//   - e^x = 2^m (T_j + T_j (e^r - 1)), T_j = 2^{j/64} rounded to double.
// Error: T_j (<= 0.5 ulp of T_j, up to 1 ulp of the result when j = 0 and
// r < 0 put the result just below a power of two), truncation and the
// rounding of the polynomial (<= 0.1 ulp together, |e^r - 1| < 0.0056) and
// the final FMA (0.5 ulp): below 1.6 ulp wherever the result is normal.
// Arguments above 746 are clamped there (e^{-746} lies below half the
// smallest subnormal: the result is 0).
// Cost: 14 FP64/integer vector instructions and one table read.
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>

namespace frg {

// 2^{j/64}, j = 0..63, rounded to the nearest double (from 40-digit values).
constexpr double kExp2Tab64[64] = {
    0x1.0000000000000p+0, 0x1.02c9a3e778061p+0, 0x1.059b0d3158574p+0, 0x1.0874518759bc8p+0,
    0x1.0b5586cf9890fp+0, 0x1.0e3ec32d3d1a2p+0, 0x1.11301d0125b51p+0, 0x1.1429aaea92de0p+0,
    0x1.172b83c7d517bp+0, 0x1.1a35beb6fcb75p+0, 0x1.1d4873168b9aap+0, 0x1.2063b88628cd6p+0,
    0x1.2387a6e756238p+0, 0x1.26b4565e27cddp+0, 0x1.29e9df51fdee1p+0, 0x1.2d285a6e4030bp+0,
    0x1.306fe0a31b715p+0, 0x1.33c08b26416ffp+0, 0x1.371a7373aa9cbp+0, 0x1.3a7db34e59ff7p+0,
    0x1.3dea64c123422p+0, 0x1.4160a21f72e2ap+0, 0x1.44e086061892dp+0, 0x1.486a2b5c13cd0p+0,
    0x1.4bfdad5362a27p+0, 0x1.4f9b2769d2ca7p+0, 0x1.5342b569d4f82p+0, 0x1.56f4736b527dap+0,
    0x1.5ab07dd485429p+0, 0x1.5e76f15ad2148p+0, 0x1.6247eb03a5585p+0, 0x1.6623882552225p+0,
    0x1.6a09e667f3bcdp+0, 0x1.6dfb23c651a2fp+0, 0x1.71f75e8ec5f74p+0, 0x1.75feb564267c9p+0,
    0x1.7a11473eb0187p+0, 0x1.7e2f336cf4e62p+0, 0x1.82589994cce13p+0, 0x1.868d99b4492edp+0,
    0x1.8ace5422aa0dbp+0, 0x1.8f1ae99157736p+0, 0x1.93737b0cdc5e5p+0, 0x1.97d829fde4e50p+0,
    0x1.9c49182a3f090p+0, 0x1.a0c667b5de565p+0, 0x1.a5503b23e255dp+0, 0x1.a9e6b5579fdbfp+0,
    0x1.ae89f995ad3adp+0, 0x1.b33a2b84f15fbp+0, 0x1.b7f76f2fb5e47p+0, 0x1.bcc1e904bc1d2p+0,
    0x1.c199bdd85529cp+0, 0x1.c67f12e57d14bp+0, 0x1.cb720dcef9069p+0, 0x1.d072d4a07897cp+0,
    0x1.d5818dcfba487p+0, 0x1.da9e603db3285p+0, 0x1.dfc97337b9b5fp+0, 0x1.e502ee78b3ff6p+0,
    0x1.ea4afa2a490dap+0, 0x1.efa1bee615a27p+0, 0x1.f50765b6e4540p+0, 0x1.fa7c1819e90d8p+0,
};
constexpr int kExpTab = 64;

constexpr double kExpInvL = 0x1.71547652b82fep+6;  // 64/ln2
constexpr double kExpShift = 0x1.8p52;             // 1.5 2^52
constexpr double kExpLhi = 0x1.62e42fee00000p-7;   // ln2/64, 32 significant bits
constexpr double kExpLlo = 0x1.a39ef35793c76p-39;  // ln2/64 - kExpLhi
constexpr double kExpClamp = 746.0;

// e^{-y}; `tab` holds kExp2Tab64 (in LDS on the device).
__host__ __device__ __forceinline__ double exp_neg(double y, const double *tab) {
  const double x = -fmin(y, kExpClamp);
  const double t = __builtin_fma(x, kExpInvL, kExpShift);
  const double nd = t - kExpShift;
  const int n = (int)(unsigned)__builtin_bit_cast(unsigned long long, t);
  double r = __builtin_fma(-nd, kExpLhi, x);
  r = __builtin_fma(-nd, kExpLlo, r);
  double q = __builtin_fma(r, 1.0 / 120.0, 1.0 / 24.0);
  q = __builtin_fma(r, q, 1.0 / 6.0);
  q = __builtin_fma(r, q, 0.5);
  q = __builtin_fma(r, q, 1.0);
  const double em1 = r * q;
  const double T = tab[n & (kExpTab - 1)];
  return ldexp(__builtin_fma(T, em1, T), n >> 6);
}

}  // namespace frg
