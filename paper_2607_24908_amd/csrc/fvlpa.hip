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

// Sum over the 8 lanes of an aligned group (xor 1, xor 2, then the mirror
// of the 8 lanes, equivalent to xor 4 once each quad holds equal values).
__device__ __forceinline__ double group8_sum(double x) {
  x = x + dpp_f64<0xB1>(x);
  x = x + dpp_f64<0x4E>(x);
  return x + dpp_f64<0x141>(x);
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

// Flux Q and the local bound lam of the step estimate at interface j of one
// flow with cell values u[0..n) (global memory or LDS) and radial table tab
// (chat | hhat, global memory or LDS); the eight lanes of an aligned group
// (sub = 0..7) take radial nodes sub, sub + 8, ... of F_1, F_2 at up to three
// masses (d_sigma u and the two Goldstone states) and meet in group8_sum, so
// every lane of the group returns the same Q, lam.  bad: a mass of a live
// interface has left the domain.  Interfaces past n (not live) load clamped
// cells; their results are not used.
__device__ __forceinline__ void fv_interface(const FvArgs &a, const FvScale &sc, const double *u,
                                             const double *tab, int64_t j, int sub, bool live,
                                             double &Q, double &lam, bool &bad) {
  const int64_t n = a.n;
  const double ids = a.inv_ds;
  // cells j-2 .. j+1 with the ghost cells: loads at clamped indices first
  // (issued together), the ghost rules after
  const int64_t nm1 = n - 1;
  auto cl = [&](int64_t i) { return i < 0 ? (int64_t)0 : (i > nm1 ? nm1 : i); };
  const double v0 = u[cl(j - 2)], v1 = u[cl(j - 1)], v2 = u[cl(j)], v3 = u[cl(j + 1)];
  const double e0 = u[0], e1 = u[1], f1 = u[nm1], f2 = u[n - 2];
  const double gn = 2.0 * f1 - f2, gn1 = 2.0 * gn - f1;
  auto cell = [&](int64_t i, double v) {
    return i == -1 ? -e0 : i == -2 ? -e1 : i == n ? gn : i == n + 1 ? gn1 : v;
  };
  const bool gold = j > 0 && a.N > 1;
  double ms, um = 0.0, up = 0.0, isj = 0.0;
  if (j == 0) {
    ms = 2.0 * e0 * ids;
  } else {
    const double uLL = cell(j - 2, v0), uL = cell(j - 1, v1), uR = cell(j, v2),
                 uRR = cell(j + 1, v3);
    ms = (uR - uL) * ids;
    const double sL = minmod(uL - uLL, uR - uL);
    const double sR = minmod(uR - uL, uRR - uR);
    um = uL + 0.5 * sL;
    up = uR - 0.5 * sR;
    isj = ids / (double)j;  // 1/sigma_j
  }
  const double m2[3] = {ms, um * isj, up * isj};
  const int nm = gold ? 3 : 1;
  bad = false;
  double dh[3];
#pragma unroll
  for (int m = 0; m < 3; ++m) {
    const double delta = m2[m] + sc.k2;
    bad |= live && m < nm && !(delta > 0.0);
    dh[m] = (m < nm && delta > 0.0) ? delta * sc.inv_k2 : 1.0;
  }
  double s1[3] = {0.0, 0.0, 0.0}, s2[3] = {0.0, 0.0, 0.0};
  for (int i = sub; i < a.n_r; i += 8) {
    const double c = tab[i], hh = tab[a.n_r + i];
#pragma unroll
    for (int m = 0; m < 3; ++m) {
      if (m >= nm) break;
      const double G = rcp64(hh + dh[m]);
      const double cg = c * G;
      s1[m] += cg;
      s2[m] = __builtin_fma(cg, G, s2[m]);
    }
  }
  double F1[3], F2[3];
#pragma unroll
  for (int m = 0; m < 3; ++m) {
    F1[m] = a.Cd * sc.kd * group8_sum(s1[m]);
    F2[m] = a.Cd * sc.kdm2 * group8_sum(s2[m]);
  }
  if (j == 0) {
    Q = 0.5 * (double)a.N * F1[0];
    lam = 2.0 * (0.5 * (double)a.N * F2[0]) * (ids * ids);
  } else {
    Q = 0.5 * F1[0];
    lam = 2.0 * (0.5 * F2[0]) * (ids * ids);
    if (gold) {
      const double c = 0.5 * (double)(a.N - 1);
      const double am = fmax(c * F2[1] * isj, c * F2[2] * isj);
      Q += 0.5 * (c * F1[1] + c * F1[2]) - 0.5 * am * (up - um);
      lam += am * ids;
    }
  }
}

// Interface 0 (flux N/2 F_1(2 u_0/ds), one mass) by a whole wave: lane l
// takes radial nodes l, l + 64, ..., then the fixed-order wave sum, so every
// lane returns the same Q, lam, bad.  The fused solve and the flux kernel
// both take interface 0 this way (the same bits); a group of eight lanes
// would need eight times as long, and in the fused solve with n a multiple
// of the group count it is the one interface of a third round.
__device__ __forceinline__ void fv_interface0(const FvArgs &a, const FvScale &sc, const double *u,
                                              const double *tab, int lane, double &Q, double &lam,
                                              bool &bad) {
  const double ids = a.inv_ds;
  const double delta = 2.0 * u[0] * ids + sc.k2;
  bad = !(delta > 0.0);
  const double dh = delta > 0.0 ? delta * sc.inv_k2 : 1.0;
  double s1 = 0.0, s2 = 0.0;
  for (int i = lane; i < a.n_r; i += kWave) {
    const double c = tab[i], hh = tab[a.n_r + i];
    const double G = rcp64(hh + dh);
    const double cg = c * G;
    s1 += cg;
    s2 = __builtin_fma(cg, G, s2);
  }
  const double F1 = a.Cd * sc.kd * wave_sum_fold<1>(&s1, lane);
  const double F2 = a.Cd * sc.kdm2 * wave_sum_fold<1>(&s2, lane);
  Q = 0.5 * (double)a.N * F1;
  lam = 2.0 * (0.5 * (double)a.N * F2) * (ids * ids);
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

// Grid (blocks of 32 interfaces, flows): eight interfaces per wave, eight
// lanes per interface (fv_interface) at the stage time a.t.
__global__ __launch_bounds__(256) void fv_flux_kernel(FvArgs a) {
  const int lane = threadIdx.x & (kWave - 1);
  const int wave = threadIdx.x / kWave;
  const int sub = lane & 7;
  const int64_t r = blockIdx.y;
  const int64_t n = a.n, nq = n + 1;
  const int64_t j = ((int64_t)blockIdx.x * (blockDim.x / kWave) + wave) * 8 + (lane >> 3);
  const bool live = j < nq;  // every lane takes part in the group sums
  const int64_t o = r * nq + j;
  if (!a.alive[r]) {  // workgroup-uniform
    if (live && sub == 0) {
      a.Q[o] = 0.0;
      a.lam[o] = 0.0;
    }
    return;
  }
  const double *u = (a.first ? a.y0 : a.ys) + r * n;
  const FvScale sc = fv_scale(a, a.t);
  double Q, lam;
  bool bad;
  fv_interface(a, sc, u, a.tab, j, sub, live, Q, lam, bad);
  if (blockIdx.x == 0 && wave == 0) {  // the wave of interface 0
    double q0, l0;
    bool b0;
    fv_interface0(a, sc, u, a.tab, lane, q0, l0, b0);
    if (j == 0) {
      Q = q0;
      lam = l0;
      bad = b0;
    }
  }
  if (!live || sub != 0) return;
  if (bad) {
    // the flow ends at the start of this step with its state kept
    a.alive[r] = 0;
    a.t_reached[r] = a.t_n;
    *a.flag = 1;
    a.Q[o] = 0.0;
    a.lam[o] = 0.0;
    return;
  }
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
// fluxes and the radial table in LDS; per stage the fluxes of all n + 1
// interfaces (groups of eight lanes over interfaces 1..n, interface 0 by one
// wave), a barrier, the cell updates, a barrier.  The per-interface and per-cell arithmetic is that of the flux
// and stage kernels (same bits); no launch per stage.  A flow whose masses
// leave the domain in a stage ends with the state of the start of that step.
__global__ __launch_bounds__(1024) void fv_solve_kernel(FvArgs a, int64_t s0, int64_t n_st) {
  extern __shared__ double lds[];
  const int64_t r = blockIdx.x;
  if (!a.alive[r]) return;  // workgroup-uniform
  const int64_t n = a.n;
  const int tid = threadIdx.x, bs = blockDim.x;
  double *y0 = lds;
  double *ys = y0 + n;
  double *Q = ys + n;
  double *tab = Q + n + 1;
  int *bad_flag = reinterpret_cast<int *>(tab + 2 * a.n_r);
  for (int64_t i = tid; i < n; i += bs) y0[i] = a.y0[r * n + i];
  for (int i = tid; i < 2 * a.n_r; i += bs) tab[i] = a.tab[i];
  if (tid == 0) *bad_flag = 0;
  __syncthreads();
  const int G = bs / 8, grp = tid / 8, sub = tid & 7;
  // interface 0 by a wave whose groups hold one interface fewer than the
  // first groups (groups n % G and up), or wave 0 when all hold as many
  int wave0 = ((int)(n % G) + 7) / 8;
  if (wave0 >= G / 8) wave0 = 0;
  const double cs[3] = {0.0, 1.0, 0.5};
  for (int64_t st = 0; st < n_st; ++st) {
    const double tn = (double)(s0 + st) * a.h;
    for (int s = 0; s < 3; ++s) {
      const FvScale sc = fv_scale(a, tn + cs[s] * a.h);
      const double *u = s == 0 ? y0 : ys;
      bool bad = false;
      for (int64_t j = 1 + grp; j <= n; j += G) {
        double q, lam;
        bool b;
        fv_interface(a, sc, u, tab, j, sub, true, q, lam, b);
        if (sub == 0) Q[j] = q;
        bad |= b;
      }
      if (tid / kWave == wave0) {  // wave-uniform
        double q, lam;
        bool b;
        fv_interface0(a, sc, u, tab, tid & (kWave - 1), q, lam, b);
        if ((tid & (kWave - 1)) == 0) Q[0] = q;
        bad |= b;
      }
      if (bad) *bad_flag = 1;
      __syncthreads();
      if (*bad_flag) {  // workgroup-uniform
        if (tid == 0) {
          a.alive[r] = 0;
          a.t_reached[r] = tn;
          *a.flag = 1;
        }
        for (int64_t i = tid; i < n; i += bs) a.y0[r * n + i] = y0[i];
        return;
      }
      for (int64_t i = tid; i < n; i += bs) {
        const double L = (Q[i + 1] - Q[i]) * a.inv_ds;
        fv_update(s, L, a.h, y0[i], ys[i]);
      }
      __syncthreads();
    }
  }
  for (int64_t i = tid; i < n; i += bs) a.y0[r * n + i] = y0[i];
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
  hipLaunchKernelGGL(fv_flux_kernel, dim3((unsigned)((a.n + 1 + 31) / 32), (unsigned)a.n_rows),
                     dim3(256), 0, (hipStream_t)stream, a);
  return (int)hipGetLastError();
}

int launch_fv_stage(const FvArgs &a, void *stream) {
  if (a.n_rows <= 0) return 0;
  hipLaunchKernelGGL(fv_stage_kernel, dim3((unsigned)((a.n + 255) / 256), (unsigned)a.n_rows),
                     dim3(256), 0, (hipStream_t)stream, a);
  return (int)hipGetLastError();
}

int fv_solve_lds_bytes(const FvArgs &a) {
  return (int)(sizeof(double) * (3 * a.n + 1 + 2 * (int64_t)a.n_r) + 16);
}

int launch_fv_solve(const FvArgs &a, int64_t s0, int64_t n_st, int threads, void *stream) {
  if (a.n_rows <= 0 || n_st <= 0) return 0;
  if (threads < 64 || threads > 1024 || threads % 64) return (int)hipErrorInvalidValue;
  hipLaunchKernelGGL(fv_solve_kernel, dim3((unsigned)a.n_rows), dim3(threads),
                     fv_solve_lds_bytes(a), (hipStream_t)stream, a, s0, n_st);
  return (int)hipGetLastError();
}

int launch_fv_dt(const FvArgs &a, void *stream) {
  if (a.n_rows <= 0) return 0;
  hipLaunchKernelGGL(fv_dt_kernel, dim3((unsigned)a.n_rows), dim3(256), 0, (hipStream_t)stream, a);
  return (int)hipGetLastError();
}

}  // namespace frg
