// HIP kernels (gfx950) for the FRG flow-diagram quadrature.
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
// FP64 reciprocal: the hardware estimate (v_rcp_f64) refined by two
// Newton-Raphson steps r <- r + r (1 - x r).
#include <hip/hip_runtime.h>

#include <cmath>

#include "frg_internal.h"

#pragma clang fp contract(off)

namespace frg {

namespace {

constexpr int kExp = FRG_REG_EXP;
constexpr int kLitim = FRG_REG_LITIM;

__device__ __forceinline__ double rcp64(double x) {
  double r = __builtin_amdgcn_rcp(x);
  double e = __builtin_fma(-x, r, 1.0);
  r = __builtin_fma(r, e, r);
  e = __builtin_fma(-x, r, 1.0);
  r = __builtin_fma(r, e, r);
  return r;
}

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
    for (int u = 0; u < s.U; ++u) {
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

// One tile: `count` (<= 64) consecutive points of set s, one after another;
// lane e keeps the result of point e, stored coalesced at the end.
template <int REG>
__device__ void do_tile(const SetDev &s, const double *tab, int64_t start, int count, int lane,
                        int *flag) {
  double res = 0.0;
  for (int e = 0; e < count; ++e) {
    const double p = s.p[start + e];
    const double delta = s.m2[start + e] + s.k2;
    double v;
    if (delta > 0.0 && p >= 0.0) {
      v = s.pref * wave_sum(lane_point<REG>(tab, s, lane, p, delta));
    } else {
      v = __builtin_nan("");
      if (lane == 0) *flag = 1;
    }
    if (lane == e) res = v;
  }
  if (lane < count) s.out[start + lane] = res;
}

__device__ __forceinline__ void stage_table(const SetDev &s, double *lds, int tid, int nthreads) {
  const int ntab = 3 * s.n_r + 2 * s.n_a;
  for (int i = tid; i < ntab; i += nthreads) lds[i] = s.tab[i];
}

// Plain launch over one set: 4 waves per workgroup share the staged table,
// each wave takes one tile of `tile_points` points.
template <int REG>
__global__ __launch_bounds__(256) void points_plain_kernel(SetDev s, int tile_points, int64_t n_tiles,
                                                           int *flag) {
  extern __shared__ double lds[];
  stage_table(s, lds, threadIdx.x, blockDim.x);
  __syncthreads();
  const int lane = threadIdx.x & (kWave - 1);
  const int64_t tile = (int64_t)blockIdx.x * (blockDim.x / kWave) + (threadIdx.x / kWave);
  if (tile >= n_tiles) return;
  const int64_t start = tile * tile_points;
  const int64_t left = s.n_ext - start;
  const int count = left < tile_points ? (int)left : tile_points;
  do_tile<REG>(s, lds, start, count, lane, flag);
}

// Persistent launch over many sets: one wave per workgroup; waves pull
// tiles (longest first) from an atomic counter until the list is drained.
__global__ __launch_bounds__(64) void points_persistent_kernel(const SetDev *__restrict__ sets,
                                                               const Tile *__restrict__ tiles,
                                                               int n_tiles, int *counter,
                                                               int *flag) {
  extern __shared__ double lds[];
  const int lane = threadIdx.x;
  int cur = -1;
  for (;;) {
    int t = 0;
    if (lane == 0) t = atomicAdd(counter, 1);
    t = __shfl(t, 0, kWave);
    if (t >= n_tiles) break;
    const Tile tl = tiles[t];
    const SetDev s = sets[tl.set];
    if (tl.set != cur) {
      __syncthreads();
      stage_table(s, lds, lane, kWave);
      __syncthreads();
      cur = tl.set;
    }
    if (s.reg == kExp)
      do_tile<kExp>(s, lds, tl.start, tl.count, lane, flag);
    else
      do_tile<kLitim>(s, lds, tl.start, tl.count, lane, flag);
  }
}

__global__ void reset_counter_kernel(int *c) {
  if (threadIdx.x == 0) *c = 0;
}

// Tensor grid: workgroup = W waves sharing one momentum p[a]; wave w owns
// M consecutive masses.  The table Hk(s_ij) of this p is built in LDS
// (lane-major, conflict-free) in chunks of g.chunk (t, u) rows and each
// entry is reused for the M masses of every wave.  Rows are visited in the
// same (t, u) order as lane_point, so results match the point kernel bit
// for bit.
template <int REG, int M>
__global__ __launch_bounds__(512) void grid_kernel(GridArgs g) {
  extern __shared__ double lds[];
  const int W = blockDim.x / kWave;
  const int wave = threadIdx.x / kWave;
  const int lane = threadIdx.x & (kWave - 1);
  const int64_t a = blockIdx.x / g.n_mb;
  const int mb = (int)(blockIdx.x - a * g.n_mb);
  const double p = g.p[a];
  const int n_r = g.n_r, n_a = g.n_a;
  const double *tq = g.tab;
  const double *tc = g.tab + n_r;
  const double *tH = g.tab + 2 * n_r;
  const double *to = g.tab + 3 * n_r;
  const double *tm = to + n_a;
  const int TU = g.T * g.U;
  const int C = g.chunk < TU ? g.chunk : TU;
  double *lH = lds;
  double *lc = lH + C * kWave;
  double *lq = lc + n_r;
  double *lm = lq + n_r;
  for (int idx = threadIdx.x; idx < n_r; idx += blockDim.x) {
    lc[idx] = tc[idx];
    lq[idx] = tH[idx];
  }
  for (int idx = threadIdx.x; idx < n_a; idx += blockDim.x) lm[idx] = tm[idx];

  const int64_t m0 = ((int64_t)mb * W + wave) * M;
  const bool p_ok = p >= 0.0;
  double dm[M];
  bool ok[M];
#pragma unroll
  for (int m = 0; m < M; ++m) {
    const int64_t idx = m0 + m;
    const bool valid = idx < g.n_m;
    const double d = valid ? g.m2[idx] + g.k2 : 1.0;
    ok[m] = valid && p_ok && d > 0.0;
    dm[m] = ok[m] ? d : 1.0;
  }
  const int rho = lane & (g.R - 1);
  const int iota = lane / g.R;
  double tot[M], A[M], in[M];
#pragma unroll
  for (int m = 0; m < M; ++m) tot[m] = A[m] = in[m] = 0.0;
  int t = 0, u = 0;
  for (int c0 = 0; c0 < TU; c0 += C) {
    const int c1 = (c0 + C < TU) ? c0 + C : TU;
    if (c0 > 0) __syncthreads();  // all waves are done with the previous chunk
    for (int idx = threadIdx.x; idx < (c1 - c0) * kWave; idx += blockDim.x) {
      const int l = idx & (kWave - 1);
      const int tu = c0 + idx / kWave;
      const int tt = tu / g.U, uu = tu - tt * g.U;
      const int i = (l & (g.R - 1)) + g.R * tt;
      const int j = (l / g.R) + g.J * uu;
      double v = 1.0;
      if (i < n_r && j < n_a) {
        const double q = tq[i];
        const double qm = q - p;
        const double aa = qm * qm;
        const double b = (2.0 * q) * p;
        v = hk<REG>(__builtin_fma(b, to[j], aa), g.k2, g.inv_k2);
      }
      lH[idx] = v;
    }
    __syncthreads();
    for (int tu = c0; tu < c1; ++tu) {
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
      const int j = iota + g.J * u;
      const double mu = j < n_a ? lm[j] : 0.0;
      const double H = lH[(tu - c0) * kWave + lane];
#pragma unroll
      for (int m = 0; m < M; ++m) in[m] = __builtin_fma(mu, rcp64(H + dm[m]), in[m]);
      if (++u == g.U) {
#pragma unroll
        for (int m = 0; m < M; ++m) tot[m] = __builtin_fma(A[m], in[m], tot[m]);
        u = 0;
        ++t;
      }
    }
  }
  double res = 0.0;
  bool bad = false;
#pragma unroll
  for (int m = 0; m < M; ++m) {
    const double v = g.pref * wave_sum(tot[m]);
    const bool valid = m0 + m < g.n_m;
    if (lane == m) res = ok[m] ? v : __builtin_nan("");
    bad |= valid && !ok[m];
  }
  if (bad && lane == 0) *g.flag = 1;
  if (lane < M && m0 + lane < g.n_m) g.out[a * g.n_m + m0 + lane] = res;
}

// Coefficient of U[j+o] in U' (c1) and U'' (c2) of the difference formulas.
__device__ __forceinline__ void fd_coef(int64_t j, int64_t n, int o, double i2, double i1,
                                        double *c1, double *c2) {
  double a = 0.0, b = 0.0;
  if (j == 0) {
    if (o == 0) { a = -3.0 * i2; b = 2.0 * i1; }
    else if (o == 1) { a = 4.0 * i2; b = -5.0 * i1; }
    else if (o == 2) { a = -1.0 * i2; b = 4.0 * i1; }
    else if (o == 3) { b = -1.0 * i1; }
  } else if (j == n - 1) {
    if (o == 0) { a = 3.0 * i2; b = 2.0 * i1; }
    else if (o == -1) { a = -4.0 * i2; b = -5.0 * i1; }
    else if (o == -2) { a = 1.0 * i2; b = 4.0 * i1; }
    else if (o == -3) { b = -1.0 * i1; }
  } else {
    if (o == 1) { a = i2; b = i1; }
    else if (o == 0) { b = -2.0 * i1; }
    else if (o == -1) { a = -i2; b = i1; }
  }
  *c1 = a;
  *c2 = b;
}

// LPA right-hand side for a batch of flows: one wave per grid point, lanes
// over radial nodes; F_1 and F_2 at the sigma and pion masses.
__global__ __launch_bounds__(256) void lpa_kernel(const LpaJob *__restrict__ jobs,
                                                  const int64_t *__restrict__ start, int n_jobs,
                                                  int64_t total) {
  const int lane = threadIdx.x & (kWave - 1);
  const int64_t gid = (int64_t)blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave;
  if (gid >= total) return;
  int lo = 0, hi = n_jobs - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (start[mid] <= gid) lo = mid; else hi = mid - 1;
  }
  const LpaJob jb = jobs[lo];
  const int64_t j = gid - start[lo];
  const int64_t n = jb.n;
  const double *U = jb.U;
  const double dr = jb.dr;
  double d1, d2;
  if (j == 0) {
    d1 = ((-3.0 * U[0] + 4.0 * U[1]) - U[2]) / (2.0 * dr);
    d2 = (((2.0 * U[0] - 5.0 * U[1]) + 4.0 * U[2]) - U[3]) / (dr * dr);
  } else if (j == n - 1) {
    d1 = ((3.0 * U[n - 1] - 4.0 * U[n - 2]) + U[n - 3]) / (2.0 * dr);
    d2 = (((2.0 * U[n - 1] - 5.0 * U[n - 2]) + 4.0 * U[n - 3]) - U[n - 4]) / (dr * dr);
  } else {
    d1 = (U[j + 1] - U[j - 1]) / (2.0 * dr);
    d2 = ((U[j + 1] - 2.0 * U[j]) + U[j - 1]) / (dr * dr);
  }
  const double rho = (double)j * dr;
  const double ms = d1 + (2.0 * rho) * d2;
  const double mp = d1;
  const double ds = ms + jb.k2;
  const double dp = mp + jb.k2;
  const bool pion = jb.N > 1;
  const bool ok = ds > 0.0 && (!pion || dp > 0.0);
  const double dsh = (ok ? ds : jb.k2) * jb.inv_k2;
  const double dph = ((ok && pion) ? dp : jb.k2) * jb.inv_k2;
  const double *chat = jb.tab;
  const double *hhat = jb.tab + jb.n_r;
  double f1s = 0.0, f2s = 0.0, f1p = 0.0, f2p = 0.0;
  for (int i = lane; i < jb.n_r; i += kWave) {
    const double c = chat[i], h = hhat[i];
    const double gs = rcp64(h + dsh);
    const double gp = rcp64(h + dph);
    const double cs = c * gs, cp = c * gp;
    f1s += cs;
    f2s = __builtin_fma(cs, gs, f2s);
    f1p += cp;
    f2p = __builtin_fma(cp, gp, f2p);
  }
  const double F1s = jb.pre1 * wave_sum(f1s);
  const double F2s = jb.pre2 * wave_sum(f2s);
  const double F1p = pion ? jb.pre1 * wave_sum(f1p) : 0.0;
  const double F2p = pion ? jb.pre2 * wave_sum(f2p) : 0.0;
  const double nan = __builtin_nan("");
  if (lane == 0) {
    jb.dUdt[j] = ok ? 0.5 * (F1s + jb.Nm1 * F1p) : nan;
    if (!ok && jb.flag) *jb.flag = 1;
  }
  if (jb.jac && lane < 7) {
    const int o = lane - 3;
    double c1, c2;
    fd_coef(j, n, o, 1.0 / (2.0 * dr), 1.0 / (dr * dr), &c1, &c2);
    const double dms = c1 + (2.0 * rho) * c2;
    const double v = -0.5 * (F2s * dms + (jb.Nm1 * F2p) * c1);
    const int64_t col = j + o;
    jb.jac[(int64_t)lane * n + j] = ok ? ((col >= 0 && col < n) ? v : 0.0) : nan;
  }
}

}  // namespace

// ------------------------------------------------------------------ host --

int launch_points_plain(const SetDev &s, int tile_points, int *d_flag, void *stream) {
  if (s.n_ext <= 0) return 0;
  const int64_t n_tiles = (s.n_ext + tile_points - 1) / tile_points;
  const int waves = 4;
  const int64_t blocks = (n_tiles + waves - 1) / waves;
  const size_t lds = sizeof(double) * (3 * s.n_r + 2 * s.n_a);
  hipStream_t st = (hipStream_t)stream;
  if (s.reg == kExp)
    hipLaunchKernelGGL(points_plain_kernel<kExp>, dim3((unsigned)blocks), dim3(64 * waves), lds, st,
                       s, tile_points, n_tiles, d_flag);
  else
    hipLaunchKernelGGL(points_plain_kernel<kLitim>, dim3((unsigned)blocks), dim3(64 * waves), lds,
                       st, s, tile_points, n_tiles, d_flag);
  return (int)hipGetLastError();
}

int launch_reset_counter(int *d_counter, void *stream) {
  hipLaunchKernelGGL(reset_counter_kernel, dim3(1), dim3(64), 0, (hipStream_t)stream, d_counter);
  return (int)hipGetLastError();
}

int launch_points_persistent(const SetDev *d_sets, const Tile *d_tiles, int n_tiles, int *d_counter,
                             int lds_doubles, int n_blocks, int *d_flag, void *stream) {
  if (n_tiles <= 0) return 0;
  hipLaunchKernelGGL(points_persistent_kernel, dim3(n_blocks), dim3(64),
                     sizeof(double) * lds_doubles, (hipStream_t)stream, d_sets, d_tiles, n_tiles,
                     d_counter, d_flag);
  return (int)hipGetLastError();
}

int grid_lds_bytes(const GridArgs &g) {
  const int TU = g.T * g.U;
  const int C = g.chunk < TU ? g.chunk : TU;
  return (int)sizeof(double) * (C * kWave + 2 * g.n_r + g.n_a);
}

template <int REG, int M>
static void grid_launch_t(const GridArgs &g, int W, hipStream_t st) {
  const int64_t blocks = g.n_p * g.n_mb;
  hipLaunchKernelGGL((grid_kernel<REG, M>), dim3((unsigned)blocks), dim3(kWave * W),
                     grid_lds_bytes(g), st, g);
}

int launch_grid(const GridArgs &g, int reg, int M, int W, void *stream) {
  if (g.n_p <= 0 || g.n_m <= 0) return 0;
  hipStream_t st = (hipStream_t)stream;
  if (reg == kExp) {
    switch (M) {
      case 4: grid_launch_t<kExp, 4>(g, W, st); break;
      case 8: grid_launch_t<kExp, 8>(g, W, st); break;
      default: grid_launch_t<kExp, 16>(g, W, st); break;
    }
  } else {
    switch (M) {
      case 4: grid_launch_t<kLitim, 4>(g, W, st); break;
      case 8: grid_launch_t<kLitim, 8>(g, W, st); break;
      default: grid_launch_t<kLitim, 16>(g, W, st); break;
    }
  }
  return (int)hipGetLastError();
}

int launch_lpa(const LpaJob *d_jobs, const int64_t *d_start, int n_jobs, int64_t total_points,
               void *stream) {
  if (total_points <= 0) return 0;
  const int waves = 4;
  const int64_t blocks = (total_points + waves - 1) / waves;
  hipLaunchKernelGGL(lpa_kernel, dim3((unsigned)blocks), dim3(64 * waves), 0, (hipStream_t)stream,
                     d_jobs, d_start, n_jobs, total_points);
  return (int)hipGetLastError();
}

}  // namespace frg
