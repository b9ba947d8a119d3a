// Compensated-FP32 kernel (FRG_PREC_FP32C) for plain launches and tensor
// grids; the per-point arithmetic is in device_fp32c.h.
#include <hip/hip_runtime.h>

#include <cmath>

#include "frg_internal.h"

#pragma clang fp contract(off)

#include "device_fp32c.h"
#include "device_grid.h"

namespace frg {

namespace {

using namespace dev;

// 4 waves per workgroup share the staged tables; each wave takes one tile.
// grid_nm > 0: point e is (p[e / grid_nm], m2[e % grid_nm]).
template <int REG>
__global__ __launch_bounds__(256) void fp32c_kernel(SetDev s, int tile_points, int64_t n_tiles,
                                                    int64_t grid_nm, int *flag) {
  extern __shared__ double lds[];
  double *etab = lds;  // kExp2Tab64 and the angular pairs for the FP64 path
  double2 *ang = reinterpret_cast<double2 *>(lds + kExpTab);
  double *tab = lds + kExpTab + 2 * s.n_a;
  const int ntab = table_doubles(s.n_r, s.n_a);
  const float *fo = reinterpret_cast<const float *>(tab + ntab);
  const float *fm = fo + s.n_a;
  const float *fl = fm + s.n_a;
  for (int i = threadIdx.x; i < kExpTab; i += blockDim.x) etab[i] = kExp2Tab64[i];
  stage_pairs(s, ang, threadIdx.x, blockDim.x);
  stage_fp32c(s, tab, threadIdx.x, blockDim.x);
  __syncthreads();
  const int lane = threadIdx.x & (kWave - 1);
  const int64_t tile = (int64_t)blockIdx.x * (blockDim.x / kWave) + (threadIdx.x / kWave);
  if (tile >= n_tiles) return;
  const int64_t start = tile * tile_points;
  const int64_t left = s.n_ext - start;
  const int count = left < tile_points ? (int)left : tile_points;
  fp32c_tile<REG>(s, tab, ang, etab, fo, fm, fl, start, count, grid_nm, lane, flag);
}

// ------------------------------------------------------ tensor grid --
// Compensated-FP32 tensor grid (exponential regulator).  The workgroup layout
// and the fill are those of the FP64 grid kernel; LDS holds the FP32 table
// H''_ij = fl32(H'_ij sig_j) = fl32((Hk(s_ij)/k^2) rho_j).  Each mass of a wave
// is FP32 (dhat >= band and the running fraction stays in the FP32 normal
// range) or FP64.  FP32 masses take, per group of eight angular terms, N/P
// over D''_k = fma(dhat, rho_k, H''_k) in FP32 (one FMA, one FMA and one
// multiply per term, one hardware reciprocal per group), scaled by gam_g and
// accumulated in FP64.  Per result the estimate
//   err = kKappa * kSigma32 * sqrt(sum_i A_i^2 sum_g g^2) / |I|
//         + |fl32(dhat) - dhat| / dhat + erho
// (statistical rounding of the group sums g, rounding of dhat shared by all
// terms, and the largest weight error |gam/rho_j - mu_j| / mu_j) decides
// whether the FP32 value is returned.  Masses above f32_flag and the FP64
// masses are marked used64 = 1 and computed by the FP64 grid kernel in redo
// mode (bit for bit its ordinary results), launched right after.

constexpr double kSigma32 = 1.3 * 5.9604644775390625e-08;  // rms rounding of a group sum, relative

template <int M, bool ALL>
__device__ __forceinline__ void grid32_resident(const GridArgs &g, const double *lc,
                                                const double *lq, const float *lH32,
                                                const float *lrho, const double *lgam, int lane,
                                                const double *dm, const float *dh,
                                                unsigned active, double *tot, double *var) {
  const int rho_l = lane & (g.R - 1);
  const int iota = lane / g.R;
  const int G = grouped_u(g.n_a, g.J);
  // this lane's angular data, u-major: rb[u] = rho_j, gb[u] = gam_j, j = iota + J u
  const float *rb = lrho + iota * g.U;
  const double *gb = lgam + iota * g.U;
  for (int t = 0; t < g.T; ++t) {
    const int i = rho_l + g.R * t;
    const bool vi = i < g.n_r;
    const double c = vi ? lc[i] : 0.0;
    const double Hq = vi ? lq[i] : 1.0;
    double A[M], in[M];
    float V[M];
#pragma unroll
    for (int m = 0; m < M; ++m) {
      if (!ALL && !((active >> m) & 1u)) continue;
      const double Gq = rcp64(Hq + dm[m]);
      A[m] = (c * Gq) * Gq;
      in[m] = 0.0;
      V[m] = 0.0f;
    }
    const float *row = lH32 + (t * g.U) * kWave + lane;
    int u = 0;
    for (; u < G; u += kGroup) {
      float H[kGroup], r[kGroup];
#pragma unroll
      for (int k = 0; k < kGroup; ++k) {
        r[k] = rb[u + k];
        H[k] = row[(u + k) * kWave];
      }
      const double gam = gb[u];
      const float gam32 = (float)gam;
      // masses four at a time (ALL) or one by one: four independent chains
      // in flight cover the latency of the FP32 pipeline
      constexpr int S = ALL ? (M >= 4 ? 4 : M) : 1;
#pragma unroll
      for (int m = 0; m < M; m += S) {
        if (!ALL && !((active >> m) & 1u)) continue;
        float N[S], P[S];
#pragma unroll
        for (int x = 0; x < S; ++x) {
          N[x] = 1.0f;
          P[x] = __builtin_fmaf(dh[m + x], r[0], H[0]);
        }
#pragma unroll
        for (int k = 1; k < kGroup; ++k) {
          float D[S];
#pragma unroll
          for (int x = 0; x < S; ++x) D[x] = __builtin_fmaf(dh[m + x], r[k], H[k]);
#pragma unroll
          for (int x = 0; x < S; ++x) N[x] = __builtin_fmaf(N[x], D[x], P[x]);
#pragma unroll
          for (int x = 0; x < S; ++x) P[x] = P[x] * D[x];
          // keep the chains interleaved (the scheduler would otherwise run
          // them one after the other)
          if (S > 1) __builtin_amdgcn_sched_barrier(0);
        }
#pragma unroll
        for (int x = 0; x < S; ++x) {
          const float q = N[x] * __builtin_amdgcn_rcpf(P[x]);
          const float gs = q * gam32;
          V[m + x] = __builtin_fmaf(gs, gs, V[m + x]);
          in[m + x] = __builtin_fma((double)q, gam, in[m + x]);
        }
      }
    }
    for (; u < g.U; ++u) {
      const int j = iota + g.J * u;
      if (j < g.n_a) {
        const float r = rb[u];
        const float H = row[u * kWave];
        const double gam = gb[u];
        const float gam32 = (float)gam;
#pragma unroll
        for (int m = 0; m < M; ++m) {
          if (!ALL && !((active >> m) & 1u)) continue;
          const float q = __builtin_amdgcn_rcpf(__builtin_fmaf(dh[m], r, H));
          const float gs = q * gam32;
          V[m] = __builtin_fmaf(gs, gs, V[m]);
          in[m] = __builtin_fma((double)q, gam, in[m]);
        }
      }
    }
#pragma unroll
    for (int m = 0; m < M; ++m) {
      if (!ALL && !((active >> m) & 1u)) continue;
      tot[m] = __builtin_fma(A[m], in[m], tot[m]);
      var[m] = __builtin_fma(A[m] * A[m], (double)V[m], var[m]);
    }
  }
}

// The FP32 running fraction of a group stays in the normal range when every
// D'' lies in [3.2e-5, 4e4] (then 1e-36 < P and N < 1e37).
__device__ __forceinline__ bool range32_ok(const GridArgs &g, double dhat, double p) {
  const double qp = g.q_top + p;
  return dhat * g.f32_rmin >= 3.2e-5 && __builtin_fma(qp * qp, g.inv_k2, dhat) * g.f32_rmax <= 4e4;
}

template <int REG, int M>
__global__ __launch_bounds__(512) void grid32_kernel(GridArgs g) {
  extern __shared__ double lds[];
  const int W = blockDim.x / kWave;
  const int wave = threadIdx.x / kWave;
  const int lane = threadIdx.x & (kWave - 1);
  const int64_t a = blockIdx.x / g.n_mb;
  const int mb = (int)(blockIdx.x - a * g.n_mb);
  const double p = g.p[a];
  const int n_r = g.n_r, n_a = g.n_a;
  const int TU = g.T * g.U;
  double *lc = lds;
  double *lq = lc + n_r;
  double *lgam = lq + n_r;
  float *lH32 = reinterpret_cast<float *>(lgam + g.J * g.U);
  float *lrho = lH32 + TU * kWave;
  const double *gsig = g.tab32 + n_a;
  const float *grho = reinterpret_cast<const float *>(g.tab32 + 2 * n_a);
  for (int idx = threadIdx.x; idx < n_r; idx += blockDim.x) {
    lc[idx] = g.tab[n_r + idx];
    lq[idx] = g.tab[2 * n_r + idx];
  }
  for (int idx = threadIdx.x; idx < g.J * g.U; idx += blockDim.x) {
    // lane-major copies: entry (iota, u) holds angular node j = iota + J u
    const int iota = idx / g.U, u = idx - iota * g.U;
    const int j = iota + g.J * u;
    lgam[idx] = j < n_a ? g.tab32[j] : 0.0;
    lrho[idx] = j < n_a ? grho[j] : 1.0f;
  }
  grid_fill<REG>(g, nullptr, 0, TU, p, lH32, gsig);
  __syncthreads();
  const bool p_ok = p >= 0.0;
  const unsigned all = (M == 32) ? ~0u : ((1u << M) - 1u);
  for (int rep = 0; rep < g.mblocks; ++rep) {
    const int64_t m0 = (((int64_t)mb * g.mblocks + rep) * W + wave) * M;
    if (m0 >= g.n_m) break;  // wave-uniform
    double dm[M], edel[M];
    float dh[M];
    unsigned okm = 0, m32 = 0;
#pragma unroll
    for (int m = 0; m < M; ++m) {
      const int64_t idx = m0 + m;
      const bool valid = idx < g.n_m;
      const double d = valid ? g.m2[idx] + g.k2 : 1.0;
      const bool ok = valid && p_ok && d > 0.0;
      dm[m] = ok ? d : 1.0;
      const double dhat = dm[m] * g.inv_k2;
      dh[m] = (float)dhat;
      edel[m] = fabs((double)dh[m] - dhat) * __builtin_amdgcn_rcp(dhat);  // a bound: few digits
      okm |= ok ? (1u << m) : 0u;
      m32 |= (ok && dhat >= g.f32_band && range32_ok(g, dhat, p)) ? (1u << m) : 0u;
    }
    // the masses are the same in every lane: make the choices wave-uniform
    okm = __builtin_amdgcn_readfirstlane(okm);
    m32 = __builtin_amdgcn_readfirstlane(m32);
    const int mine = fold_owner<M>(lane);
    const bool leader = fold_leader<M>(lane);
    double s32 = 0.0, err32 = 0.0;
    unsigned flagged = 0;
    if (m32) {
      double tot[M], var[M];
#pragma unroll
      for (int m = 0; m < M; ++m) tot[m] = var[m] = 0.0;
      if (m32 == all)
        grid32_resident<M, true>(g, lc, lq, lH32, lrho, lgam, lane, dm, dh, m32, tot, var);
      else
        grid32_resident<M, false>(g, lc, lq, lH32, lrho, lgam, lane, dm, dh, m32, tot, var);
      s32 = wave_sum_fold<M>(tot, lane);
      const double v32 = wave_sum_fold<M>(var, lane);
      double ed = 0.0;
#pragma unroll
      for (int m = 0; m < M; ++m) ed = (m == mine) ? edel[m] : ed;
      // the estimate needs few digits: hardware reciprocal and FP32 root
      const float rel2 = (float)(v32 * __builtin_amdgcn_rcp(s32 * s32));
      err32 = kKappa * kSigma32 * (double)__builtin_sqrtf(rel2) + ed + g.f32_erho;
      const bool bad = ((m32 >> mine) & 1u) && !(err32 <= g.f32_flag);
      const uint64_t b = __ballot(leader && bad);
#pragma unroll
      for (int m = 0; m < M; ++m) flagged |= ((b >> (m * (kWave / M))) & 1ull) ? (1u << m) : 0u;
    }
    const unsigned m64 = (okm & ~m32) | flagged;
    bool badm = false;
#pragma unroll
    for (int m = 0; m < M; ++m) badm |= (m0 + m < g.n_m) && !((okm >> m) & 1u);
    if (badm && lane == 0) *g.flag = 1;
    // FP64 masses are marked used64 = 1 here and computed by the FP64 grid
    // kernel in redo mode, launched next on the same stream
    if (leader && m0 + mine < g.n_m) {
      const int64_t o = a * g.n_m + m0 + mine;
      if (!((okm >> mine) & 1u)) {
        g.out[o] = __builtin_nan("");
        if (g.err) g.err[o] = __builtin_nan("");
        g.used64[o] = 0;
      } else if ((m64 >> mine) & 1u) {
        g.used64[o] = 1;
      } else {
        g.out[o] = (g.pref * g.inv_k2) * s32;
        if (g.err) g.err[o] = err32;
        g.used64[o] = 0;
      }
    }
  }
}

}  // namespace

int launch_fp32c(const SetDev &s, int tile_points, int64_t grid_nm, int *d_flag, void *stream) {
  if (s.n_ext <= 0) return 0;
  const int64_t n_tiles = (s.n_ext + tile_points - 1) / tile_points;
  const int waves = 4;
  const int64_t blocks = (n_tiles + waves - 1) / waves;
  const size_t lds = sizeof(double) * (kExpTab + 2 * s.n_a) + fp32c_lds_bytes(s.n_r, s.n_a);
  hipStream_t st = (hipStream_t)stream;
  if (s.reg == kExp)
    hipLaunchKernelGGL(fp32c_kernel<kExp>, dim3((unsigned)blocks), dim3(64 * waves), lds, st, s,
                       tile_points, n_tiles, grid_nm, d_flag);
  else
    hipLaunchKernelGGL(fp32c_kernel<kLitim>, dim3((unsigned)blocks), dim3(64 * waves), lds, st, s,
                       tile_points, n_tiles, grid_nm, d_flag);
  return (int)hipGetLastError();
}

int grid32_lds_bytes(const GridArgs &g) {
  const int TU = g.T * g.U;
  return (int)(sizeof(double) * (2 * g.n_r + g.J * g.U) + sizeof(float) * (TU * kWave + g.J * g.U));
}

template <int REG, int M>
static void grid32_launch_t(const GridArgs &g, int W, hipStream_t st) {
  const int64_t blocks = g.n_p * g.n_mb;
  hipLaunchKernelGGL((grid32_kernel<REG, M>), dim3((unsigned)blocks), dim3(kWave * W),
                     grid32_lds_bytes(g), st, g);
}

int launch_grid32(const GridArgs &g, int reg, int M, int W, void *stream) {
  if (g.n_p <= 0 || g.n_m <= 0) return 0;
  hipStream_t st = (hipStream_t)stream;
  if (M != 4 && M != 8) return (int)hipErrorInvalidValue;  // the host passes M <= 8
  if (reg == kExp)
    M == 8 ? grid32_launch_t<kExp, 8>(g, W, st) : grid32_launch_t<kExp, 4>(g, W, st);
  else
    M == 8 ? grid32_launch_t<kLitim, 8>(g, W, st) : grid32_launch_t<kLitim, 4>(g, W, st);
  return (int)hipGetLastError();
}

}  // namespace frg
