// FP64 kernels (gfx950) of the FRG flow-diagram quadrature: the point-list
// kernel (plain and persistent launches), the tensor-grid kernel and the
// batched LPA right-hand side.  The per-point arithmetic, lane map and
// summation order are in device_fp64.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>

#include "frg_internal.h"

#pragma clang fp contract(off)

#include "device_fp32c.h"
#include "device_fp64.h"
#include "device_grid.h"

namespace frg {

namespace {

using namespace dev;

// Lane l's value of a double, as a wave-uniform (scalar) value.
__device__ __forceinline__ double readlane_f64(double v, int l) {
  const unsigned long long b = __builtin_bit_cast(unsigned long long, v);
  const int lo = __builtin_amdgcn_readlane((int)(unsigned)b, l);
  const int hi = __builtin_amdgcn_readlane((int)(unsigned)(b >> 32), l);
  return __builtin_bit_cast(double, ((unsigned long long)(unsigned)hi << 32) | (unsigned)lo);
}

// One tile: `count` (<= 64) consecutive points of set s.  Lane e loads point
// e, so the tile's inputs arrive with one memory latency; the points are
// then taken one after another (wave-uniform p, delta) and four at a time
// summed over the wave (wave_sum_fold<4>: lane l ends with the total of
// point l/16, the same bits as for any other number of points per fold);
// lanes 0, 16, 32, 48 store.
// Lane e's inputs of a tile (0 beyond count).
__device__ __forceinline__ void load_tile(const SetDev &s, int64_t start, int count, int lane,
                                          double &pv, double &mv) {
  pv = lane < count ? s.p[start + lane] : 0.0;
  mv = lane < count ? s.m2[start + lane] : 0.0;
}

// MARK: the set is FRG_PREC_FP32C evaluated in FP64 (Litim): also store
// err = kErr64 and used64 = 1 (NaN and 0 for points outside the domain).
template <int REG, bool MARK>
__device__ void do_tile(const SetDev &s, const double *tab, const double2 *ang, const double *etab,
                        int64_t start, int count, double pv, double mv, int lane, int *flag) {
  constexpr int F = 4;
  for (int e0 = 0; e0 < count; e0 += F) {
    const int nf = count - e0 < F ? count - e0 : F;
    double v0 = 0.0, v1 = 0.0, v2 = 0.0, v3 = 0.0;
    unsigned ok = 0;
    // one copy of the point code: the partials go to v0..v3 by selects on
    // the wave-uniform f
#pragma unroll 1
    for (int f = 0; f < nf; ++f) {
      const double p = readlane_f64(pv, e0 + f);
      const double delta = readlane_f64(mv, e0 + f) + s.k2;
      double part = 0.0;
      if (delta > 0.0 && p >= 0.0) {
        part = point_partial<REG>(s, tab, ang, etab, lane, p, delta);
        ok |= 1u << f;
      } else if (lane == 0) {
        *flag = 1;
      }
      v0 = f == 0 ? part : v0;
      v1 = f == 1 ? part : v1;
      v2 = f == 2 ? part : v2;
      v3 = f == 3 ? part : v3;
    }
    const double v[F] = {v0, v1, v2, v3};
    const double tot = wave_sum_fold<F>(v, lane);
    const int mine = fold_owner<F>(lane);
    if (fold_leader<F>(lane) && mine < nf) {
      const int64_t o = start + e0 + mine;
      const bool okm = (ok >> mine) & 1u;
      s.out[o] = okm ? s.pref_k * tot : __builtin_nan("");
      if (MARK) {
        if (s.err) s.err[o] = okm ? kErr64 : __builtin_nan("");
        if (s.used64) s.used64[o] = (uint8_t)okm;
      }
    }
  }
}

__device__ __forceinline__ void stage_exp_table(double *etab, int tid, int nthreads) {
  for (int i = tid; i < kExpTab; i += nthreads) etab[i] = kExp2Tab64[i];
}

__device__ __forceinline__ void stage_table(const SetDev &s, double *lds, int tid, int nthreads) {
  const int ntab = table_doubles(s.n_r, s.n_a);
  for (int i = tid; i < ntab; i += nthreads) lds[i] = s.tab[i];
}

// Plain launch over one set: 4 waves per workgroup share the staged tables
// (LDS layout of point_lds_doubles), each wave takes one tile of
// `tile_points` points.  F32: the set is FRG_PREC_FP32C (fp32c_tile).
template <int REG, bool F32>
__global__ __launch_bounds__(256) void points_plain_kernel(SetDev s, int tile_points, int64_t n_tiles,
                                                           int *flag) {
  extern __shared__ double lds[];
  double *etab = lds;
  double2 *ang = reinterpret_cast<double2 *>(lds + kExpTab);
  double *tab = lds + kExpTab + 2 * s.n_a;
  stage_exp_table(etab, threadIdx.x, blockDim.x);
  stage_pairs(s, ang, threadIdx.x, blockDim.x);
  stage_table(s, tab, threadIdx.x, blockDim.x);
  __syncthreads();
  const int lane = threadIdx.x & (kWave - 1);
  const int64_t tile = (int64_t)blockIdx.x * (blockDim.x / kWave) + (threadIdx.x / kWave);
  if (tile >= n_tiles) return;
  const int64_t start = tile * tile_points;
  const int64_t left = s.n_ext - start;
  const int count = left < tile_points ? (int)left : tile_points;
  double pv, mv;
  load_tile(s, start, count, lane, pv, mv);
  if (F32 && REG == kExp)
    fp32c_tile(s, tab, ang, etab, start, count, pv, mv, lane, flag);
  else
    do_tile<REG, F32>(s, tab, ang, etab, start, count, pv, mv, lane, flag);
}

// Persistent launch over many sets (FP64 and FP32C mixed): one wave per
// workgroup; waves pull tiles from kCounters counters until the list is
// drained.  Sub-list x holds tiles x, x + kCounters, ... of the longest-first
// list (an equal share of every cost class) and is served by workgroups
// b = x mod kCounters (with round-robin dispatch, the workgroups of one
// XCD); the counters lie kCounterStride ints apart, on different cache
// lines, so the claims spread over kCounters atomic units.  A wave ends at
// its first empty claim; the launch has at least min(n_tiles, kCounters)
// workgroups, so every non-empty sub-list is served.  At most 128 VGPRs, so
// that four waves share each SIMD (the FP32C variant needs the bound).
template <bool WITH_F32>
__global__ __launch_bounds__(64, 4) void points_persistent_kernel(const SetDev *__restrict__ sets,
                                                               const Tile *__restrict__ tiles,
                                                               int n_tiles, int *counters,
                                                               int *flag) {
  extern __shared__ double lds[];
  double *etab = lds;
  const int lane = threadIdx.x;
  stage_exp_table(etab, lane, kWave);
  int cur = -1;
  // lane 0 claims tiles; the claim of the next tile is issued while the
  // current one is processed, so its latency is hidden.  Tile indices are
  // made wave-uniform (scalar registers), and the tile and set descriptors
  // read with them are scalar loads.
  const int x = (int)(blockIdx.x % kCounters);
  int *ctr = counters + x * kCounterStride;
  auto claim = [&]() -> int {
    int c = 0;
    if (lane == 0) c = atomicAdd(ctr, 1);
    return c;
  };
  int c = __builtin_amdgcn_readfirstlane(claim());
  for (;;) {
    const int64_t tt = (int64_t)x + (int64_t)kCounters * c;
    if (tt >= n_tiles) break;
    const int t = (int)tt;
    const Tile tl = tiles[t];
    const SetDev s = sets[tl.set];
    const bool f32 = WITH_F32 && s.prec == FRG_PREC_FP32C;
    double pv, mv;
    load_tile(s, tl.start, tl.count, lane, pv, mv);
    double2 *ang = reinterpret_cast<double2 *>(lds + kExpTab);
    double *tab = lds + kExpTab + 2 * s.n_a;
    if (tl.set != cur) {
      __syncthreads();
      stage_pairs(s, ang, lane, kWave);
      stage_table(s, tab, lane, kWave);
      __syncthreads();
      cur = tl.set;
    }
    // claim the next tile after this tile's loads, so that waiting for them
    // does not wait for the claim
    const int cn = claim();
    if (s.reg == kExp) {
      if (f32)
        fp32c_tile(s, tab, ang, etab, tl.start, tl.count, pv, mv, lane, flag);
      else
        do_tile<kExp, false>(s, tab, ang, etab, tl.start, tl.count, pv, mv, lane, flag);
    } else if (f32) {
      do_tile<kLitim, true>(s, tab, ang, etab, tl.start, tl.count, pv, mv, lane, flag);
    } else {
      do_tile<kLitim, false>(s, tab, ang, etab, tl.start, tl.count, pv, mv, lane, flag);
    }
    c = __builtin_amdgcn_readfirstlane(cn);
  }
}

__global__ void fp64_marks_kernel(double *err, uint8_t *used64, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  if (err) err[i] = kErr64;
  if (used64) used64[i] = 1;
}

__global__ void expneg_fp32c_kernel(const double *y, double *out, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = exp_neg32(y[i]);
}

__global__ void reset_counter_kernel(int *c) {
  if (threadIdx.x < kCounters) c[threadIdx.x * kCounterStride] = 0;
}

// Tensor grid.  A workgroup of W waves owns one momentum p[a] and
// W * M * MB consecutive masses; wave w takes mass blocks w, w + W, ... of M
// masses each.  The table H'_ij = Hk(s_ij) rmu_j of this p lives in LDS
// (lane-major, conflict-free) and serves every mass block; tables larger than
// g.chunk rows are streamed through LDS in chunks (then MB = 1).  The (t, u)
// visiting order, the grouping and the arithmetic are those of lane_point, so
// results match the point kernel bit for bit.

// RESIDENT: the whole table fits in g.chunk rows (host-checked).
template <int REG, int M, bool RESIDENT>
__global__ __launch_bounds__(512) void grid_kernel(GridArgs g) {
  extern __shared__ double lds[];
  const int W = blockDim.x / kWave;
  const int wave = threadIdx.x / kWave;
  const int lane = threadIdx.x & (kWave - 1);
  const int64_t a = blockIdx.x / g.n_mb;
  const int mb = (int)(blockIdx.x - a * g.n_mb);
  const double p = g.p[a];
  const int n_r = g.n_r, n_a = g.n_a;
  const int TU = g.T * g.U;
  constexpr bool resident = RESIDENT;
  const int C = resident ? TU : g.chunk;
  const int MB = resident ? g.mblocks : 1;
  double *lH = lds;
  double *lc = lH + C * kWave;
  double *lq = lc + n_r;
  double *lr = lq + n_r;
  for (int idx = threadIdx.x; idx < n_r; idx += blockDim.x) {
    lc[idx] = g.tab[n_r + idx];
    lq[idx] = g.tab[2 * n_r + idx];
  }
  for (int idx = threadIdx.x; idx < n_a; idx += blockDim.x) lr[idx] = g.tab[3 * n_r + 2 * n_a + idx];
  if (resident) {
    grid_fill<REG>(g, lH, 0, TU, p);
    __syncthreads();
  }
  const bool p_ok = p >= 0.0;
  const unsigned all = (M == 32) ? ~0u : ((1u << M) - 1u);
  for (int rep = 0; rep < MB; ++rep) {
    const int64_t m0 = (((int64_t)mb * MB + rep) * W + wave) * M;
    if (m0 >= g.n_m && resident) break;  // wave-uniform
    double dm[M];
    bool ok[M];
    unsigned mask = 0;
    const unsigned act = all;
#pragma unroll
    for (int m = 0; m < M; ++m) {
      const int64_t idx = m0 + m;
      const bool valid = idx < g.n_m;
      const double d = valid ? g.m2[idx] + g.k2 : 1.0;
      ok[m] = valid && p_ok && d > 0.0;
      dm[m] = ok[m] ? d : 1.0;
      mask |= chain_ok(dm[m], p, g.q_top, g.rmu_max) ? (1u << m) : 0u;
    }
    // the masses are the same in every lane: make the choices wave-uniform
    const unsigned gmask = __builtin_amdgcn_readfirstlane(mask);
    double tot[M];
#pragma unroll
    for (int m = 0; m < M; ++m) tot[m] = 0.0;
    if constexpr (RESIDENT) {
      if (act == all && gmask == all)
        grid_resident<M, true>(g, lH, lc, lq, lr, lane, dm, act, gmask, tot);
      else
        grid_resident<M, false>(g, lH, lc, lq, lr, lane, dm, act, gmask, tot);
    } else {
      double A[M], in[M];
#pragma unroll
      for (int m = 0; m < M; ++m) A[m] = in[m] = 0.0;
      int t = 0, u = 0;
      for (int c0 = 0; c0 < TU;) {
        const int c1 = chunk_end(g, c0, C, TU);
        __syncthreads();  // previous chunk consumed; also orders the small tables
        grid_fill<REG>(g, lH, c0, c1, p);
        __syncthreads();
        grid_rows<M>(g, lH, lc, lq, lr, c0, c1, lane, dm, gmask, t, u, A, in, tot);
        c0 = c1;
      }
    }
    // lane l ends with the total of mass l / (64 / M)
    const double v = g.pref * wave_sum_split<M>(tot, lane);
    const int mine = lane / (kWave / M);
    unsigned okbits = 0;
    bool bad = false;
#pragma unroll
    for (int m = 0; m < M; ++m) {
      okbits |= ok[m] ? (1u << m) : 0u;
      bad |= (m0 + m < g.n_m) && !ok[m];
    }
    const bool okm = (okbits >> mine) & 1u;
    if (bad && lane == 0) *g.flag = 1;
    if (lane % (kWave / M) == 0 && m0 + mine < g.n_m)
      g.out[a * g.n_m + m0 + mine] = okm ? v : __builtin_nan("");
  }
}

// Stage the masses of one workgroup (blocks of M) in LDS with their masks:
// lmask[4b..4b+2] = valid, ok (domain), coefficient form (4b + 3 pads a
// block's masks to 16 bytes), ldm[bM + m] = delta.
template <int M, int G, int E>
__device__ __forceinline__ void stage_masses(const GridArgs &g, int64_t wg_m0, int nblk, bool p_ok,
                                             bool table, unsigned *lmask, double *ldm) {
  for (int b = threadIdx.x; b < nblk; b += blockDim.x) {
    unsigned vb = 0, okb = 0, cmb = 0;
#pragma unroll
    for (int m = 0; m < M; ++m) {
      const int64_t idx = wg_m0 + (int64_t)b * M + m;
      const bool valid = idx < g.n_m;
      const double d = valid ? g.m2[idx] + g.k2 : 1.0;
      const bool ok = valid && p_ok && d > 0.0;
      const double dd = ok ? d : 1.0;
      ldm[b * M + m] = dd;
      vb |= valid ? (1u << m) : 0u;
      okb |= ok ? (1u << m) : 0u;
      cmb |= (table && fold_m_ok<G, E>(g.sig * dd)) ? (1u << m) : 0u;
    }
    lmask[4 * b] = vb;
    lmask[4 * b + 1] = okb;
    lmask[4 * b + 2] = cmb;
  }
}

// The mass blocks of one wave: coefficient form for the masses in range,
// single(delta) (per-term lane partial) for the others, reduction, store.
template <int M, int G, int E, class Single>
__device__ __forceinline__ void coef_blocks(const GridArgs &g, const double *lC,
                                            const unsigned *lmask, const double *ldm, int64_t a,
                                            int64_t wg_m0, int MB, int W, int wave, int lane,
                                            const FoldShape<G, E> &fs, Single single) {
  const unsigned all = (1u << M) - 1u;
  for (int rep = 0; rep < MB; ++rep) {
    const int b = rep * W + wave;
    const int64_t m0 = wg_m0 + (int64_t)b * M;
    if (m0 >= g.n_m) break;  // wave-uniform
    // the masses are the same in every lane: the choices are wave-uniform
    const unsigned validbits = __builtin_amdgcn_readfirstlane(lmask[4 * b]);
    const unsigned okbits = __builtin_amdgcn_readfirstlane(lmask[4 * b + 1]);
    const unsigned cmask = __builtin_amdgcn_readfirstlane(lmask[4 * b + 2]);
    double dm[M], xs[M];
#pragma unroll
    for (int m = 0; m < M; ++m) {
      dm[m] = ldm[b * M + m];
      xs[m] = g.sig * dm[m];
    }
    double tot[M];
#pragma unroll
    for (int m = 0; m < M; ++m) tot[m] = 0.0;
    const unsigned cm = cmask;
    if (cm == all)
      grid_fold_rows<M, G, true, E>(g, lC, lane, xs, cm, fs, tot);
    else if (cm)
      grid_fold_rows<M, G, false, E>(g, lC, lane, xs, cm, fs, tot);
    const unsigned sm = all & ~cmask;
    if (sm) {
#pragma unroll
      for (int m = 0; m < M; ++m)
        if ((sm >> m) & 1u) tot[m] = single(dm[m]);
    }
    // lane l ends with the total of mass fold_owner(l); the coefficient form
    // carries the factor kap / sig^(E+1) (folded into pref_c)
    const double s = wave_sum_fold<M>(tot, lane);
    const int mine = fold_owner<M>(lane);
    const double v = (((cmask >> mine) & 1u) ? g.pref_c : g.pref) * s;
    const bool okm = (okbits >> mine) & 1u;
    const bool mine_out = fold_leader<M>(lane) && ((validbits >> mine) & 1u);
    if ((validbits & ~okbits) && lane == 0) *g.flag = 1;
    if (mine_out) g.out[a * g.n_m + m0 + mine] = okm ? v : __builtin_nan("");
  }
}

// The 16-mass tiles of one wave on the matrix cores (mfma_fold_rows): lane l
// carries mass l % 16; the four lanes of a mass add their partials (offsets
// 32 and 16, the same order in each of them).  Masses outside the range of
// the coefficient form are evaluated at x = 1 there (in range, result
// dropped) and take single(delta) with a full-wave sum.  The value of a mass
// depends on its own column only: tile composition, W and MB change nothing.
template <int G, int E, class Single>
__device__ __forceinline__ void mfma_blocks(const GridArgs &g, const double *lC,
                                            const unsigned *lmask, const double *ldm, int64_t a,
                                            int64_t wg_m0, int MB, int W, int wave, int lane,
                                            const FoldShape<G, E> &fs, Single single) {
  constexpr int M = 16;
  const int mine = lane & (M - 1);
  for (int rep = 0; rep < MB; ++rep) {
    const int b = rep * W + wave;
    const int64_t m0 = wg_m0 + (int64_t)b * M;
    if (m0 >= g.n_m) break;  // wave-uniform
    const unsigned validbits = __builtin_amdgcn_readfirstlane(lmask[4 * b]);
    const unsigned okbits = __builtin_amdgcn_readfirstlane(lmask[4 * b + 1]);
    const unsigned cmask = __builtin_amdgcn_readfirstlane(lmask[4 * b + 2]);
    const unsigned cm = cmask;
    double s = 0.0;
    if (cm) {
      const double x = ((cm >> mine) & 1u) ? g.sig * ldm[b * M + mine] : 1.0;
      s = mfma_fold_rows<G, E>(g, lC, lane, x, fs);
      s = swap_add<32>(s, s);
      s = swap_add<16>(s, s);
    }
    unsigned sm = ((1u << M) - 1u) & ~cmask;
    while (sm) {  // wave-uniform
      const int m = __builtin_ctz(sm);
      sm &= sm - 1u;
      const double one = single(ldm[b * M + m]);
      const double t = wave_sum_fold<1>(&one, lane);
      if (mine == m) s = t;
    }
    const double v = (((cmask >> mine) & 1u) ? g.pref_c : g.pref) * s;
    const bool okm = (okbits >> mine) & 1u;
    const bool mine_out = lane < M && ((validbits >> mine) & 1u);
    if ((validbits & ~okbits) && lane == 0) *g.flag = 1;
    if (mine_out) g.out[a * g.n_m + m0 + mine] = okm ? v : __builtin_nan("");
  }
}

// Tensor grid, resident coefficient form (device_grid.h): a workgroup owns
// one momentum and W * M * MB masses; it builds the per-group coefficients of
// its momentum once in LDS and every mass evaluates them by Horner.
template <int REG, int M, int G>
__global__ __launch_bounds__(512) void grid_coef_kernel(GridArgs g) {
  extern __shared__ double lds[];
  const int W = blockDim.x / kWave;
  const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x / kWave));
  const int lane = threadIdx.x & (kWave - 1);
  const int64_t a = blockIdx.x / g.n_mb;
  const int mb = (int)(blockIdx.x - a * g.n_mb);
  const double p = g.p[a];
  const int n_r = g.n_r, n_a = g.n_a;
  const int MB = g.mblocks;
  const int nblk = MB * W;  // mass blocks of M masses in this workgroup
  const int64_t wg_m0 = (int64_t)mb * nblk * M;
  // LDS: coefficients | per-block masks | masses delta | c_i | Hq_i | mu_j |
  // q_i | 1 + x_j
  const FoldShape<G> fs(g.U, g.T);
  double *lC = lds;
  unsigned *lmask = reinterpret_cast<unsigned *>(lC + fs.rows * kWave);
  double *ldm = reinterpret_cast<double *>(lmask + 4 * nblk);
  double *lc = ldm + nblk * M;
  double *lq = lc + n_r;
  double *lm = lq + n_r;
  double *lqn = lm + n_a;
  double *lo = lqn + n_r;
  for (int idx = threadIdx.x; idx < n_r; idx += blockDim.x) {
    lc[idx] = g.tab[n_r + idx];
    lq[idx] = g.tab[2 * n_r + idx];
    lqn[idx] = g.tab[idx];
  }
  for (int idx = threadIdx.x; idx < n_a; idx += blockDim.x) {
    lm[idx] = g.tab[3 * n_r + n_a + idx];
    lo[idx] = g.tab[3 * n_r + idx];
  }
  const bool p_ok = p >= 0.0;
  const bool table = p_ok && fold_p_ok<G>(p, g);  // workgroup-uniform
  stage_masses<M, G, 2>(g, wg_m0, nblk, p_ok, table, lmask, ldm);
  __syncthreads();
  if (table) grid_fill_fold<REG, G>(g, lC, lc, lq, lm, lqn, lo, p, fs);
  __syncthreads();
  auto single = [&](double delta) {
    return grid_single_mass<REG>(g, lc, lq, lm, lane, p, delta);
  };
  if constexpr (M == 16)
    mfma_blocks<G, 2>(g, lC, lmask, ldm, a, wg_m0, MB, W, wave, lane, fs, single);
  else
    coef_blocks<M, G, 2>(g, lC, lmask, ldm, a, wg_m0, MB, W, wave, lane, fs, single);
}

// Vertex diagram on a tensor grid (configurations x masses): a workgroup owns
// one configuration (p1, p2, cos th) and W * M * MB masses.  Lane rows are
// (radial, polar) node pairs, groups are azimuthal nodes; P carries the
// extra factor (x + H1) of G(|q + p1|) (device_grid.h, vertex section).
// g.form == 1: no coefficient table (every mass per term).
// MAXT: 768 (12 waves, three per SIMD) for the matrix-core form with groups
// of up to 16 terms, whose registers allow three waves per SIMD; 512 else.
template <int REG, int M, int G, int MAXT>
__global__ __launch_bounds__(MAXT) void vertex_kernel(GridArgs g) {
  extern __shared__ double lds[];
  const int W = blockDim.x / kWave;
  const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x / kWave));
  const int lane = threadIdx.x & (kWave - 1);
  const int64_t a = blockIdx.x / g.n_mb;
  const int mb = (int)(blockIdx.x - a * g.n_mb);
  const double p1 = g.p[a], p2 = g.p2[a], ct = g.c12[a];
  const int n_r = g.n_r, n_a = g.n_a, n_phi = g.n_phi;
  const int MB = g.mblocks;
  const int nblk = MB * W;
  const int64_t wg_m0 = (int64_t)mb * nblk * M;
  const FoldShape<G, 3> fs(g.U, g.T);
  const bool table_form = g.form != 1;
  double *lC = lds;
  unsigned *lmask = reinterpret_cast<unsigned *>(lC + (table_form ? fs.rows * kWave : 0));
  double *ldm = reinterpret_cast<double *>(lmask + 4 * nblk);
  double *lc = ldm + nblk * M;  // c_i
  double *lq = lc + n_r;        // Hq_i
  double *lx = lq + n_r;        // x_j
  double *lm = lx + n_a;        // mu_j
  double *lsx = lm + n_a;       // sqrt(1 - x_j^2)
  double *lcp = lsx + n_a;      // cos phi_l
  double *lnu = lcp + n_phi;    // nu_l
  double *lqn = lnu + n_phi;    // q_i
  for (int idx = threadIdx.x; idx < n_r; idx += blockDim.x) {
    lc[idx] = g.tab[n_r + idx];
    lq[idx] = g.tab[2 * n_r + idx];
    lqn[idx] = g.tab[idx];
  }
  for (int idx = threadIdx.x; idx < n_a; idx += blockDim.x) {
    lx[idx] = g.vtab[idx];
    lm[idx] = g.tab[3 * n_r + n_a + idx];
    lsx[idx] = g.vtab[n_a + idx];
  }
  for (int idx = threadIdx.x; idx < n_phi; idx += blockDim.x) {
    lcp[idx] = g.vtab[2 * n_a + idx];
    lnu[idx] = g.vtab[2 * n_a + n_phi + idx];
  }
  const bool p_ok = p1 >= 0.0 && p2 >= 0.0 && ct >= -1.0 && ct <= 1.0;
  const double st = p_ok ? sqrt((1.0 - ct) * (1.0 + ct)) : 0.0;
  const bool table = table_form && p_ok && fold_p_ok<G, 3>(fmax(p1, p2), g);
  stage_masses<M, G, 3>(g, wg_m0, nblk, p_ok, table, lmask, ldm);
  __syncthreads();
  if (table) vertex_fill<REG, G>(g, lC, lc, lq, lqn, lx, lm, lsx, lcp, lnu, p1, p2, ct, st, fs);
  __syncthreads();
  auto single = [&](double delta) {
    return vertex_single_mass<REG>(g, lc, lq, lx, lm, lsx, lcp, lnu, lane, p1, p2, ct, st, delta);
  };
  if constexpr (M == 16)
    mfma_blocks<G, 3>(g, lC, lmask, ldm, a, wg_m0, MB, W, wave, lane, fs, single);
  else
    coef_blocks<M, G, 3>(g, lC, lmask, ldm, a, wg_m0, MB, W, wave, lane, fs, single);
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
  const size_t lds = sizeof(double) * (kExpTab + 2 * s.n_a + table_doubles(s.n_r, s.n_a));
  hipStream_t st = (hipStream_t)stream;
  const dim3 grid((unsigned)blocks), block(64 * waves);
  if (s.prec == FRG_PREC_FP32C) {
    if (s.reg == kExp)
      hipLaunchKernelGGL((points_plain_kernel<kExp, true>), grid, block, lds, st, s, tile_points,
                         n_tiles, d_flag);
    else
      hipLaunchKernelGGL((points_plain_kernel<kLitim, true>), grid, block, lds, st, s, tile_points,
                         n_tiles, d_flag);
  } else if (s.reg == kExp) {
    hipLaunchKernelGGL((points_plain_kernel<kExp, false>), grid, block, lds, st, s, tile_points,
                       n_tiles, d_flag);
  } else {
    hipLaunchKernelGGL((points_plain_kernel<kLitim, false>), grid, block, lds, st, s, tile_points,
                       n_tiles, d_flag);
  }
  return (int)hipGetLastError();
}

int launch_fp64_marks(double *err, uint8_t *used64, int64_t n, void *stream) {
  if (n <= 0 || (!err && !used64)) return 0;
  hipLaunchKernelGGL(fp64_marks_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0,
                     (hipStream_t)stream, err, used64, n);
  return (int)hipGetLastError();
}

int launch_expneg_fp32c(const double *y, double *out, int64_t n, void *stream) {
  if (n <= 0) return 0;
  hipLaunchKernelGGL(expneg_fp32c_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0,
                     (hipStream_t)stream, y, out, n);
  return (int)hipGetLastError();
}

int launch_reset_counter(int *d_counter, void *stream) {
  hipLaunchKernelGGL(reset_counter_kernel, dim3(1), dim3(64), 0, (hipStream_t)stream, d_counter);
  return (int)hipGetLastError();
}

int launch_points_persistent(const SetDev *d_sets, const Tile *d_tiles, int n_tiles, int *d_counter,
                             int lds_bytes, int n_blocks, bool with_f32, int *d_flag,
                             void *stream) {
  if (n_tiles <= 0) return 0;
  // every non-empty sub-list needs a workgroup of its own
  if (n_blocks < kCounters) n_blocks = n_tiles < kCounters ? n_tiles : kCounters;
  lds_bytes += (int)sizeof(double) * kExpTab;  // kExp2Tab64 ahead of the set's tables
  if (with_f32)
    hipLaunchKernelGGL(points_persistent_kernel<true>, dim3(n_blocks), dim3(64), (size_t)lds_bytes,
                       (hipStream_t)stream, d_sets, d_tiles, n_tiles, d_counter, d_flag);
  else
    hipLaunchKernelGGL(points_persistent_kernel<false>, dim3(n_blocks), dim3(64), (size_t)lds_bytes,
                       (hipStream_t)stream, d_sets, d_tiles, n_tiles, d_counter, d_flag);
  return (int)hipGetLastError();
}

int grid_lds_bytes(const GridArgs &g) {
  const int TU = g.T * g.U;
  const int C = g.chunk < TU ? g.chunk : TU;
  return (int)sizeof(double) * (C * kWave + 2 * g.n_r + g.n_a);
}

int grid_coef_group(const GridArgs &g) {
  if (g.form == 2) return 8;
  if (g.form == 3) return 16;
  return g.U <= 8 ? 8 : g.U <= 16 ? 16 : 32;
}

int grid_coef_lds_bytes(const GridArgs &g) {
  const int G = grid_coef_group(g);
  const int rows = G == 32   ? FoldShape<32>(g.U, g.T).rows
                   : G == 16 ? FoldShape<16>(g.U, g.T).rows
                             : FoldShape<8>(g.U, g.T).rows;
  return (int)sizeof(double) * (rows * kWave + 3 * g.n_r + 2 * g.n_a) + kGridCoefStageMax;
}

int grid_coef_stage_bytes(int MB, int W, int M) { return MB * W * (16 + 8 * M); }

void set_fold_scale(GridArgs &g, const QuadTable &h, int E) {
  int e_k, e_c;
  (void)std::frexp(h.k2, &e_k);  // k2 = f 2^e_k, f in [1/2, 1)
  double cmax = 0.0;
  for (int i = 0; i < h.n_r; ++i) cmax = std::max(cmax, h.data[h.n_r + i]);
  if (cmax > 0.0)
    (void)std::frexp(cmax, &e_c);
  else
    e_c = 0;
  g.sig = std::ldexp(1.0, 1 - e_k);
  g.kap = std::ldexp(1.0, -e_c);
  // N/P carries kap / sig^(E+1) (g.pref: the prefactor of the diagram)
  g.pref_c = std::ldexp(g.pref, (E + 1) * (1 - e_k) + e_c);
}



// Ask for dynamic LDS beyond 64 KiB for one kernel (gfx950: 160 KiB per
// workgroup).  The runtime may refuse the request where no opt-in is needed;
// that status is cleared so that it cannot be taken for a launch error.
static void allow_large_lds(const void *fn) {
  (void)hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
  (void)hipGetLastError();
}

int vertex_group(int n_phi) { return n_phi <= 8 ? 8 : n_phi <= 16 ? 16 : 32; }

static int vertex_rows(const GridArgs &g) {
  const int G = vertex_group(g.n_phi);
  return G == 32 ? FoldShape<32, 3>(g.U, g.T).rows
                 : G == 16 ? FoldShape<16, 3>(g.U, g.T).rows : FoldShape<8, 3>(g.U, g.T).rows;
}

// LDS of vertex_kernel: coefficient table (if resident) | masks and masses |
// c, Hq | x, mu, sqrt(1 - x^2) | cos phi, nu | q.
int vertex_lds_bytes(const GridArgs &g, int M, int W, bool table) {
  return (int)sizeof(double) * ((table ? vertex_rows(g) * kWave : 0) + 3 * g.n_r + 3 * g.n_a +
                                2 * g.n_phi) +
         grid_coef_stage_bytes(g.mblocks, W, M);
}

template <int REG, int M, int G, int MAXT>
static void vertex_launch_b(const GridArgs &g, int W, hipStream_t st) {
  static const bool once = (allow_large_lds((const void *)&vertex_kernel<REG, M, G, MAXT>), true);
  (void)once;
  hipLaunchKernelGGL((vertex_kernel<REG, M, G, MAXT>), dim3((unsigned)(g.n_p * g.n_mb)),
                     dim3(kWave * W), vertex_lds_bytes(g, M, W, g.form != 1), st, g);
}

template <int REG, int M, int G>
static void vertex_launch_t(const GridArgs &g, int W, hipStream_t st) {
  if constexpr (vertex_max_waves(M, G) > 8) {
    if (W > 8) {
      vertex_launch_b<REG, M, G, 64 * vertex_max_waves(M, G)>(g, W, st);
      return;
    }
  }
  vertex_launch_b<REG, M, G, 512>(g, W, st);
}

template <int REG, int M>
static void vertex_launch_m(const GridArgs &g, int W, hipStream_t st) {
  const int G = vertex_group(g.n_phi);
  if (G == 32)
    vertex_launch_t<REG, M, 32>(g, W, st);
  else if (G == 16)
    vertex_launch_t<REG, M, 16>(g, W, st);
  else
    vertex_launch_t<REG, M, 8>(g, W, st);
}

// M = 16: tiles of 16 masses on the matrix cores; M = 4, 8: vector units.
int launch_vertex(const GridArgs &g, int reg, int M, int W, void *stream) {
  if (g.n_p <= 0 || g.n_m <= 0) return 0;
  hipStream_t st = (hipStream_t)stream;
  if (M != 4 && M != 8 && M != 16) return (int)hipErrorInvalidValue;
  if (W < 1 || W > vertex_max_waves(M, vertex_group(g.n_phi))) return (int)hipErrorInvalidValue;
  if (reg == kExp) {
    if (M == 16) vertex_launch_m<kExp, 16>(g, W, st);
    else if (M == 8) vertex_launch_m<kExp, 8>(g, W, st);
    else vertex_launch_m<kExp, 4>(g, W, st);
  } else {
    if (M == 16) vertex_launch_m<kLitim, 16>(g, W, st);
    else if (M == 8) vertex_launch_m<kLitim, 8>(g, W, st);
    else vertex_launch_m<kLitim, 4>(g, W, st);
  }
  return (int)hipGetLastError();
}

template <int REG, int M, int G>
static void coef_launch_t(const GridArgs &g, int W, hipStream_t st) {
  static const bool once = (allow_large_lds((const void *)&grid_coef_kernel<REG, M, G>), true);
  (void)once;
  const int64_t blocks = g.n_p * g.n_mb;
  const int lds = grid_coef_lds_bytes(g) - kGridCoefStageMax + grid_coef_stage_bytes(g.mblocks, W, M);
  hipLaunchKernelGGL((grid_coef_kernel<REG, M, G>), dim3((unsigned)blocks), dim3(kWave * W), lds,
                     st, g);
}

bool grid_uses_coef(const GridArgs &g) {
  return g.form != 1 && std::isnormal(g.pref_c) && std::isnormal(g.sig) &&
         grid_coef_lds_bytes(g) <= kGridCoefLdsMax;
}

bool grid_resident(const GridArgs &g) { return grid_uses_coef(g) || g.T * g.U <= g.chunk; }

template <int REG, int M>
static void grid_launch_t(const GridArgs &g, int W, hipStream_t st) {
  if (grid_uses_coef(g)) {
    // M = 16: tiles of 16 masses on the matrix cores; M <= 8: vector units
    const int G = grid_coef_group(g);
    if (G == 32)
      coef_launch_t<REG, M, 32>(g, W, st);
    else if (G == 16)
      coef_launch_t<REG, M, 16>(g, W, st);
    else
      coef_launch_t<REG, M, 8>(g, W, st);
    return;
  }
  const int64_t blocks = g.n_p * g.n_mb;
  if (g.T * g.U <= g.chunk) {
    // resident table, running-fraction form
    hipLaunchKernelGGL((grid_kernel<REG, M, true>), dim3((unsigned)blocks), dim3(kWave * W),
                       grid_lds_bytes(g), st, g);
    return;
  }
  // tables too large for LDS: streamed in chunks (running-fraction form)
  hipLaunchKernelGGL((grid_kernel<REG, M, false>), dim3((unsigned)blocks), dim3(kWave * W),
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
