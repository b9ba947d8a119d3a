// Finite-volume LPA on gfx950: the semi-discrete central scheme of Kurganov
// and Tadmor for d_t u = d_sigma Q, Q = 1/2 F_1(d_sigma u) + (N-1)/2 F_1(u/sigma),
// u = dU/dsigma, with the local Lax-Friedrichs flux on the Goldstone part and
// minmod-limited piecewise-linear states, for n_rows flows at once; the
// three-stage strong-stability-preserving Runge-Kutta stages on the device.
//
// Cells i = 0..n-1 of width ds; interface j = 0..n at sigma_j = j ds between
// cells j-1 and j; ghost cells u_{-1} = -u_0, u_{-2} = -u_1 (u odd in sigma),
// u_n = 2u_{n-1} - u_{n-2}, u_{n+1} = 2u_n - u_{n-1}.  Interface 0 carries the
// flux N/2 F_1(2u_0/ds) (at sigma = 0 the Goldstone mass u/sigma equals
// d_sigma u); interface j >= 1 carries
//   1/2 F_1((u_j - u_{j-1})/ds) + 1/2 (f(u-) + f(u+)) - 1/2 a (u+ - u-),
//   f(u) = (N-1)/2 F_1(u/sigma_j), a = max |f'(u-)|, |f'(u+)|,
//   f'(u) = -(N-1)/2 F_2(u/sigma_j)/sigma_j,
// with u- = u_{j-1} + s_{j-1}/2, u+ = u_j - s_j/2, s_i = minmod(u_i - u_{i-1},
// u_{i+1} - u_i).  F_n(m^2) = C_d k^(d+2-2n) sum_i chat_i/(hhat_i + delta/k^2)^n,
// delta = m^2 + k^2 > 0 (else the flow has left the domain).
#include <hip/hip_runtime.h>

#include <cmath>

#include "frg_internal.h"

#pragma clang fp contract(off)

#include "device_fp64.h"

namespace frg {

namespace {

using namespace dev;

__device__ __forceinline__ double minmod(double a, double b) {
  if (a * b <= 0.0) return 0.0;
  return fabs(a) < fabs(b) ? a : b;
}

// alive = 1, t_reached = t_end, domain flag cleared.
__global__ __launch_bounds__(256) void fv_init_kernel(FvArgs a, double t_end) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e == 0) *a.flag = 0;
  if (e < a.n_rows) {
    a.alive[e] = 1;
    a.t_reached[e] = t_end;
  }
}

// Scales of the stage at RG time t: k = lambda e^t, k^2, 1/k^2, k^d, k^(d-2)
// (integer powers by products).  Every kernel forms them the same way.
struct FvScale {
  double k2, inv_k2, kd, kdm2;
};
__device__ __forceinline__ FvScale fv_scale(const FvArgs &a, double t) {
  const double k = a.lambda * exp(t);
  FvScale sc;
  sc.k2 = k * k;
  sc.inv_k2 = 1.0 / sc.k2;
  double p = 1.0;
  for (int i = 0; i < a.d - 2; ++i) p *= k;
  sc.kdm2 = p;
  sc.kd = p * sc.k2;
  return sc;
}

// The masses of interface j of one flow with cell values u[0..n) (global
// memory or LDS): d_sigma u and, on the Goldstone part (j > 0, N > 1), the
// limited states u-/sigma_j and u+/sigma_j (nm masses).  dh[m] =
// (m^2 + k^2)/k^2 for the masses in the domain (1 elsewhere); bad: one of them
// has left it.  The four neighbouring cells are loaded at clamped indices
// (issued together) and the ghost rules applied afterwards.
struct FvIface {
  double dh[3];
  double um, up, isj;
  int nm;
  bool bad;
};
__device__ __forceinline__ FvIface fv_prep(const FvArgs &a, const FvScale &sc, const double *u,
                                           int j) {
  const int n = (int)a.n;  // at most 2^24 cells
  const double ids = a.inv_ds;
  const int nm1 = n - 1;
  auto cl = [&](int i) { return i < 0 ? 0 : (i > nm1 ? nm1 : i); };
  const double v0 = u[cl(j - 2)], v1 = u[cl(j - 1)], v2 = u[cl(j)], v3 = u[cl(j + 1)];
  const double e0 = u[0], e1 = u[1], f1 = u[nm1], f2 = u[n - 2];
  const double gn = 2.0 * f1 - f2, gn1 = 2.0 * gn - f1;
  auto cell = [&](int i, double v) {
    return i == -1 ? -e0 : i == -2 ? -e1 : i == n ? gn : i == n + 1 ? gn1 : v;
  };
  FvIface f;
  f.nm = (j > 0 && a.N > 1) ? 3 : 1;
  f.um = 0.0;
  f.up = 0.0;
  f.isj = 0.0;
  double ms;
  if (j == 0) {
    ms = 2.0 * e0 * ids;
  } else {
    const double uLL = cell(j - 2, v0), uL = cell(j - 1, v1), uR = cell(j, v2),
                 uRR = cell(j + 1, v3);
    ms = (uR - uL) * ids;
    const double sL = minmod(uL - uLL, uR - uL);
    const double sR = minmod(uR - uL, uRR - uR);
    f.um = uL + 0.5 * sL;
    f.up = uR - 0.5 * sR;
    f.isj = ids / (double)j;  // 1/sigma_j
  }
  const double m2[3] = {ms, f.um * f.isj, f.up * f.isj};
  f.bad = false;
#pragma unroll
  for (int m = 0; m < 3; ++m) {
    const double delta = m2[m] + sc.k2;
    f.bad |= m < f.nm && !(delta > 0.0);
    f.dh[m] = (m < f.nm && delta > 0.0) ? delta * sc.inv_k2 : 1.0;
  }
  return f;
}

// s1 = sum_i chat_i/(hhat_i + x) and s2 = sum_i chat_i/(hhat_i + x)^2 over
// all radial nodes, in one lane.  For x in [kFvXMin, kFvXMax] the table's
// coefficient groups in order: N/P and M/P^2 by Horner with one reciprocal per
// group of eight nodes (the powers of x and the products stay inside the
// FP64 range there); term by term outside it.  Every term and coefficient is
// positive and x > 0, so neither form cancels.
constexpr double kFvXMin = 1e-20, kFvXMax = 1e20;

// fma(a, b, c) with c wave-uniform, taken from a scalar register: written out
// so that the compiler does not copy c into a vector register first (its
// two-address form wants the addend there), which cost two moves per
// coefficient.
__device__ __forceinline__ double fma_su(double a, double b, double c) {
  double r;
  asm("v_fma_f64 %0, %1, %2, %3" : "=v"(r) : "v"(a), "v"(b), "s"(c));
  return r;
}
__device__ __forceinline__ double fma_vu(double a, double b, double c) {
  return __builtin_fma(a, b, c);
}

// One coefficient group c at x: N, r = 1/P and M r, whose terms enter the
// sums as s1 = fma(N, r, s1), s2 = fma(M r, r, s2).  UNIFORM: c is the same
// in every lane (scalar operands); else per lane (the same operations).
template <bool UNIFORM>
__device__ __forceinline__ void fv_group(double x, const double *c, double &N, double &r,
                                         double &Mr) {
  auto fm = [](double u, double v, double w) {
    if constexpr (UNIFORM)
      return fma_su(u, v, w);
    else
      return fma_vu(u, v, w);
  };
  double P = x + c[7];
#pragma unroll
  for (int k = 6; k >= 0; --k) P = fm(P, x, c[k]);
  N = c[15];
#pragma unroll
  for (int k = 14; k >= 8; --k) N = fm(N, x, c[k]);
  double M = c[30];
#pragma unroll
  for (int k = 29; k >= 16; --k) M = fm(M, x, c[k]);
  r = rcp64(P);
  Mr = M * r;
}

__device__ __forceinline__ bool fv_coef_range(double x) { return x >= kFvXMin && x <= kFvXMax; }

__device__ __forceinline__ void fv_radial(const FvArgs &a, const double *tab,
                                          const double *__restrict__ cf, double x, double &s1,
                                          double &s2) {
  s1 = 0.0;
  s2 = 0.0;
  if (fv_coef_range(x)) {
    const int ng = (a.n_r + kFvGroup - 1) / kFvGroup;
    for (int g = 0; g < ng; ++g) {
      double N, r, Mr;
      fv_group<true>(x, cf + kFvCoef * g, N, r, Mr);
      s1 = __builtin_fma(N, r, s1);
      s2 = __builtin_fma(Mr, r, s2);
    }
  } else {
    for (int i = 0; i < a.n_r; ++i) {
      const double G = rcp64(tab[a.n_r + i] + x);
      const double cg = tab[i] * G;
      s1 += cg;
      s2 = __builtin_fma(cg, G, s2);
    }
  }
}

// F_1 = C_d k^d s1 and F_2 = C_d k^(d-2) s2 from the radial sums.
__device__ __forceinline__ void fv_scale_sums(const FvArgs &a, const FvScale &sc, double s1,
                                              double s2, double &F1, double &F2) {
  F1 = a.Cd * sc.kd * s1;
  F2 = a.Cd * sc.kdm2 * s2;
}

// F_1 and F_2 at dh = x.
__device__ __forceinline__ void fv_mass(const FvArgs &a, const FvScale &sc, const double *tab,
                                        const double *__restrict__ cf, double x, double &F1,
                                        double &F2) {
  double s1, s2;
  fv_radial(a, tab, cf, x, s1, s2);
  fv_scale_sums(a, sc, s1, s2, F1, F2);
}

// Flux Q and the local bound lam of the step estimate at interface j from
// its masses and F1[m], F2[m] at them.
__device__ __forceinline__ void fv_flux(const FvArgs &a, const FvIface &f, int j,
                                        const double *F1, const double *F2, double &Q,
                                        double &lam) {
  const double ids = a.inv_ds;
  if (j == 0) {
    Q = 0.5 * (double)a.N * F1[0];
    lam = 2.0 * (0.5 * (double)a.N * F2[0]) * (ids * ids);
  } else {
    Q = 0.5 * F1[0];
    lam = 2.0 * (0.5 * F2[0]) * (ids * ids);
    if (f.nm == 3) {
      const double c = 0.5 * (double)(a.N - 1);
      const double am = fmax(c * F2[1] * f.isj, c * F2[2] * f.isj);
      Q += 0.5 * (c * F1[1] + c * F1[2]) - 0.5 * am * (f.up - f.um);
      lam += am * ids;
    }
  }
}

// SSP-RK3 stage `stage` (0..2) of one cell with right-hand side L.
__device__ __forceinline__ void fv_update(int stage, double L, double h, double &y0, double &ys) {
  switch (stage) {
    case 0:
      ys = y0 + h * L;
      break;
    case 1:
      ys = 0.75 * y0 + 0.25 * (ys + h * L);
      break;
    default:
      y0 = y0 / 3.0 + (2.0 / 3.0) * (ys + h * L);
      break;
  }
}

// Grid (blocks of 4 kFvPerWave interfaces, flows) at the stage time a.t:
// lane 3 i + m of a wave computes mass m of the wave's interface i
// (fv_mass), lane 3 i gathers the three and stores Q, lam (lane 63 idles).
constexpr int kFvPerWave = kWave / 3;
__global__ __launch_bounds__(256) void fv_flux_kernel(FvArgs a, const double *__restrict__ cf) {
  const int lane = threadIdx.x & (kWave - 1);
  const int wave = threadIdx.x / kWave;
  const int64_t r = blockIdx.y;
  const int64_t n = a.n, nq = n + 1;
  const int il = lane / 3, m = lane - 3 * il;
  const int64_t j = ((int64_t)blockIdx.x * (blockDim.x / kWave) + wave) * kFvPerWave + il;
  const bool live = il < kFvPerWave && j < nq;
  const int64_t o = r * nq + j;
  if (!a.alive[r]) {  // workgroup-uniform
    if (live && m == 0) {
      a.Q[o] = 0.0;
      a.lam[o] = 0.0;
    }
    return;
  }
  const double *u = (a.first ? a.y0 : a.ys) + r * n;
  const FvScale sc = fv_scale(a, a.t);
  const FvIface f = fv_prep(a, sc, u, (int)(live ? j : n));
  double F1 = 0.0, F2 = 0.0;
  const double x = m == 0 ? f.dh[0] : (m == 1 ? f.dh[1] : f.dh[2]);
  if (live && m < f.nm) fv_mass(a, sc, a.tab, cf, x, F1, F2);
  double G1[3], G2[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {  // every lane takes part
    G1[k] = __shfl(F1, lane - m + k, kWave);
    G2[k] = __shfl(F2, lane - m + k, kWave);
  }
  if (!live || m != 0) return;
  if (f.bad) {
    // the flow ends at the start of this step with its state kept
    a.alive[r] = 0;
    a.t_reached[r] = a.t_n;
    *a.flag = 1;
    a.Q[o] = 0.0;
    a.lam[o] = 0.0;
    return;
  }
  double Q, lam;
  fv_flux(a, f, (int)j, G1, G2, Q, lam);
  a.Q[o] = Q;
  a.lam[o] = lam;
}

// Grid (cell blocks, flows): d_t u_i = (Q_{i+1} - Q_i)/ds and the stage.
__global__ __launch_bounds__(256) void fv_stage_kernel(FvArgs a) {
  const int64_t r = blockIdx.y;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= a.n) return;
  const int64_t e = r * a.n + i;
  if (!a.alive[r]) {
    if (a.stage == 3) a.dudt[e] = __builtin_nan("");
    return;
  }
  const double *Q = a.Q + r * (a.n + 1);
  const double L = (Q[i + 1] - Q[i]) * a.inv_ds;
  if (a.stage == 3) {
    a.dudt[e] = L;
  } else {
    double y0 = a.y0[e], ys = a.stage == 0 ? 0.0 : a.ys[e];
    fv_update(a.stage, L, a.h, y0, ys);
    if (a.stage == 2)
      a.y0[e] = y0;
    else
      a.ys[e] = ys;
  }
}

// Steps [s0, s0 + n_st) of one flow per workgroup: state, stage state,
// fluxes, the radial table and per interface its masses, F_1 and F_2 in LDS
// (the coefficient groups, the same for every lane, through the scalar
// cache).  Per stage: one thread per interface forms its masses (fv_prep), a
// barrier; thread t takes mass t % 3 of interface t / 3 (fv_mass), a barrier;
// one thread per interface forms the flux (fv_flux), a barrier; the cell
// updates, a barrier.  The per-mass, per-interface and per-cell arithmetic is
// that of the flux and stage kernels (same bits); no launch per stage.  A
// flow whose masses leave the domain in a stage ends with the state of the
// start of that step.
__global__ __launch_bounds__(1024) void fv_solve_kernel(FvArgs a, const double *__restrict__ cf,
                                                       int64_t s0, int64_t n_st) {
  extern __shared__ double lds[];
  const int64_t r = blockIdx.x;
  if (!a.alive[r]) return;  // workgroup-uniform
  const int n = (int)a.n, nq = n + 1;
  const int tid = threadIdx.x, bs = blockDim.x;
  double *y0 = lds;
  double *ys = y0 + n;
  double *Q = ys + n;
  double *tab = Q + nq;            // chat | hhat
  double *lP = tab + 2 * a.n_r;    // [n + 1][6]: dh (then F_1) of the masses, um, up, 1/sigma_j
  double *lF2 = lP + 6 * nq;       // [n + 1][3]: F_2 of the masses
  int *lN = reinterpret_cast<int *>(lF2 + 3 * nq);  // [n + 1]: number of masses
  int *bad_flag = lN + nq;
  for (int i = tid; i < n; i += bs) y0[i] = a.y0[r * n + i];
  for (int i = tid; i < 2 * a.n_r; i += bs) tab[i] = a.tab[i];
  if (tid == 0) *bad_flag = 0;
  __syncthreads();
  const double cs[3] = {0.0, 1.0, 0.5};
  const int ng = (a.n_r + kFvGroup - 1) / kFvGroup;  // coefficient groups
  for (int64_t st = 0; st < n_st; ++st) {
    const double tn = (double)(s0 + st) * a.h;
    for (int s = 0; s < 3; ++s) {
      const FvScale sc = fv_scale(a, tn + cs[s] * a.h);
      const double *u = s == 0 ? y0 : ys;
      bool bad = false;
      for (int j = tid; j < nq; j += bs) {
        const FvIface f = fv_prep(a, sc, u, j);
        double *P = lP + 6 * j;
        P[0] = f.dh[0];
        P[1] = f.dh[1];
        P[2] = f.dh[2];
        P[3] = f.um;
        P[4] = f.up;
        P[5] = f.isj;
        lN[j] = f.nm;
        bad |= f.bad;
      }
      if (bad) *bad_flag = 1;
      __syncthreads();
      if (*bad_flag) {  // workgroup-uniform
        if (tid == 0) {
          a.alive[r] = 0;
          a.t_reached[r] = tn;
          *a.flag = 1;
        }
        for (int i = tid; i < n; i += bs) a.y0[r * n + i] = y0[i];
        return;
      }
      // radial sums, one lane per (interface, mass) task.  When the tasks
      // leave a few in a last wave (3 (n + 1) = 64 w + tail), that wave
      // splits each of its tail tasks over the coefficient groups, one lane
      // per group, and the task's first lane folds the groups' terms in
      // order: the operations of one lane alone (the same bits), in the time
      // of one group instead of all of them, so the SIMD that holds that wave
      // is not left with one more whole radial sum than the others.
      const int T = 3 * nq, tail = T % kWave, t_full = T - tail;
      const bool split = tail > 0 && T <= bs && tail * ng <= kWave;  // workgroup-uniform
      for (int t = tid; t < (split ? t_full : T); t += bs) {
        const int j = t / 3, m = t - 3 * j;
        if (m < lN[j]) {
          double F1, F2;
          fv_mass(a, sc, tab, cf, lP[6 * j + m], F1, F2);
          lP[6 * j + m] = F1;
          lF2[3 * j + m] = F2;
        }
      }
      if (split && tid >= t_full && tid < t_full + kWave) {  // wave-uniform: the last wave
        const int l = tid - t_full;
        const int k = l / ng, g = l - k * ng;  // tail task k, group g
        const int tk = t_full + (k < tail ? k : 0);
        const int j = tk / 3, m = tk - 3 * j;
        const bool real = k < tail && m < lN[j];
        const double x = real ? lP[6 * j + m] : 1.0;
        double Nv = 0.0, rv = 0.0, Mr = 0.0;
        if (real && fv_coef_range(x)) fv_group<false>(x, cf + kFvCoef * g, Nv, rv, Mr);
        double s1 = 0.0, s2 = 0.0;
        for (int gg = 0; gg < ng; ++gg) {  // every lane of the wave takes part
          const int src = min(k * ng + gg, kWave - 1);
          const double n_ = __shfl(Nv, src, kWave), r_ = __shfl(rv, src, kWave);
          const double m_ = __shfl(Mr, src, kWave);
          s1 = __builtin_fma(n_, r_, s1);
          s2 = __builtin_fma(m_, r_, s2);
        }
        if (real && g == 0) {
          if (!fv_coef_range(x)) fv_radial(a, tab, cf, x, s1, s2);  // term by term
          double F1, F2;
          fv_scale_sums(a, sc, s1, s2, F1, F2);
          lP[6 * j + m] = F1;
          lF2[3 * j + m] = F2;
        }
      }
      __syncthreads();
      for (int j = tid; j < nq; j += bs) {
        const double *P = lP + 6 * j;
        FvIface f;
        f.nm = lN[j];
        f.um = P[3];
        f.up = P[4];
        f.isj = P[5];
        double q, lam;
        fv_flux(a, f, j, P, lF2 + 3 * j, q, lam);
        Q[j] = q;
      }
      __syncthreads();
      for (int i = tid; i < n; i += bs) {
        const double L = (Q[i + 1] - Q[i]) * a.inv_ds;
        fv_update(s, L, a.h, y0[i], ys[i]);
      }
      __syncthreads();
    }
  }
  for (int i = tid; i < n; i += bs) a.y0[r * n + i] = y0[i];
}

// One workgroup per flow: step estimate 1 / max_j lam_j.
__global__ __launch_bounds__(256) void fv_dt_kernel(FvArgs a) {
  __shared__ double red[256];
  const int64_t r = blockIdx.x;
  double m = 0.0;
  for (int64_t j = threadIdx.x; j <= a.n; j += blockDim.x) m = fmax(m, a.lam[r * (a.n + 1) + j]);
  red[threadIdx.x] = m;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + s]);
    __syncthreads();
  }
  if (threadIdx.x == 0) a.dt[r] = a.alive[r] ? 1.0 / red[0] : __builtin_nan("");
}

}  // namespace

int launch_fv_init(const FvArgs &a, double t_end, void *stream) {
  const int64_t n = a.n_rows > 1 ? a.n_rows : 1;
  hipLaunchKernelGGL(fv_init_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0,
                     (hipStream_t)stream, a, t_end);
  return (int)hipGetLastError();
}

int launch_fv_flux(const FvArgs &a, void *stream) {
  if (a.n_rows <= 0) return 0;
  const int64_t per_block = 4 * kFvPerWave;
  hipLaunchKernelGGL(fv_flux_kernel,
                     dim3((unsigned)((a.n + 1 + per_block - 1) / per_block), (unsigned)a.n_rows),
                     dim3(256), 0, (hipStream_t)stream, a, a.tab + 2 * a.n_r);
  return (int)hipGetLastError();
}

int launch_fv_stage(const FvArgs &a, void *stream) {
  if (a.n_rows <= 0) return 0;
  hipLaunchKernelGGL(fv_stage_kernel, dim3((unsigned)((a.n + 255) / 256), (unsigned)a.n_rows),
                     dim3(256), 0, (hipStream_t)stream, a);
  return (int)hipGetLastError();
}

int64_t fv_solve_lds_bytes(const FvArgs &a) {
  return (int64_t)sizeof(double) * (3 * a.n + 1 + 2 * (int64_t)a.n_r + 9 * (a.n + 1)) +
         (int64_t)sizeof(int) * (a.n + 1) + 16;
}

int launch_fv_solve(const FvArgs &a, int64_t s0, int64_t n_st, int threads, void *stream) {
  if (a.n_rows <= 0 || n_st <= 0) return 0;
  if (threads < 64 || threads > 1024 || threads % 64) return (int)hipErrorInvalidValue;
  if (fv_solve_lds_bytes(a) > kFvSolveLdsMax) return (int)hipErrorInvalidValue;
  static const bool once =
      ((void)hipFuncSetAttribute((const void *)&fv_solve_kernel,
                                 hipFuncAttributeMaxDynamicSharedMemorySize, kFvSolveLdsMax),
       (void)hipGetLastError(), true);
  (void)once;
  hipLaunchKernelGGL(fv_solve_kernel, dim3((unsigned)a.n_rows), dim3(threads),
                     (size_t)fv_solve_lds_bytes(a), (hipStream_t)stream, a, a.tab + 2 * a.n_r,
                     s0, n_st);
  return (int)hipGetLastError();
}

int launch_fv_dt(const FvArgs &a, void *stream) {
  if (a.n_rows <= 0) return 0;
  hipLaunchKernelGGL(fv_dt_kernel, dim3((unsigned)a.n_rows), dim3(256), 0, (hipStream_t)stream, a);
  return (int)hipGetLastError();
}

}  // namespace frg
