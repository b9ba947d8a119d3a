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

// Cell average i in [-2, n + 1] with the ghost cells (wave-uniform).
__device__ __forceinline__ double cell(const double *u, int64_t n, int64_t i) {
  if (i < 0) return -u[-i - 1];
  if (i < n) return u[i];
  const double gn = 2.0 * u[n - 1] - u[n - 2];
  return i == n ? gn : 2.0 * gn - u[n - 1];
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

// One wave per (flow, interface); lanes over the radial nodes of F_1, F_2 at
// up to three masses (d_sigma u and the two Goldstone states).
__global__ __launch_bounds__(256) void fv_flux_kernel(FvArgs a) {
  const int lane = threadIdx.x & (kWave - 1);
  const int64_t gid = (int64_t)blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave;
  const int64_t n = a.n, nq = n + 1;
  if (gid >= a.n_rows * nq) return;  // wave-uniform
  const int64_t r = gid / nq, j = gid - r * nq;
  const int64_t o = r * nq + j;
  if (!a.alive[r]) {
    a.Q[o] = 0.0;
    a.lam[o] = 0.0;
    return;
  }
  const double *u = (a.first ? a.y0 : a.ys) + r * n;
  const double ds = a.ds;
  const bool gold = j > 0 && a.N > 1;
  double ms, um = 0.0, up = 0.0, sj = 0.0;
  if (j == 0) {
    ms = 2.0 * u[0] / ds;
  } else {
    const double uL = cell(u, n, j - 1), uR = cell(u, n, j);
    ms = (uR - uL) / ds;
    const double sL = minmod(uL - cell(u, n, j - 2), uR - uL);
    const double sR = minmod(uR - uL, cell(u, n, j + 1) - uR);
    um = uL + 0.5 * sL;
    up = uR - 0.5 * sR;
    sj = (double)j * ds;
  }
  const double m2[3] = {ms, gold ? um / sj : 0.0, gold ? up / sj : 0.0};
  const int nm = gold ? 3 : 1;
  bool bad = false;
  double dh[3];
#pragma unroll
  for (int m = 0; m < 3; ++m) {
    const double delta = m2[m] + a.k2;
    bad |= m < nm && !(delta > 0.0);
    dh[m] = (m < nm && delta > 0.0) ? delta * a.inv_k2 : 1.0;
  }
  double s1[3] = {0.0, 0.0, 0.0}, s2[3] = {0.0, 0.0, 0.0};
  for (int i = lane; i < a.n_r; i += kWave) {
    const double c = a.tab[i], hh = a.tab[a.n_r + i];
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
    F1[m] = m < nm ? a.Cd * a.kd * wave_sum(s1[m]) : 0.0;
    F2[m] = m < nm ? a.Cd * a.kdm2 * wave_sum(s2[m]) : 0.0;
  }
  if (lane != 0) return;
  if (bad) {
    // the flow ends at the start of this step with its state kept
    a.alive[r] = 0;
    a.t_reached[r] = a.t_n;
    *a.flag = 1;
    a.Q[o] = 0.0;
    a.lam[o] = 0.0;
    return;
  }
  double Q, lam;
  if (j == 0) {
    Q = 0.5 * (double)a.N * F1[0];
    lam = 2.0 * (0.5 * (double)a.N * F2[0]) / (ds * ds);
  } else {
    Q = 0.5 * F1[0];
    lam = 2.0 * (0.5 * F2[0]) / (ds * ds);
    if (gold) {
      const double c = 0.5 * (double)(a.N - 1);
      const double am = fmax(c * F2[1] / sj, c * F2[2] / sj);
      Q += 0.5 * (c * F1[1] + c * F1[2]) - 0.5 * am * (up - um);
      lam += am / ds;
    }
  }
  a.Q[o] = Q;
  a.lam[o] = lam;
}

// One thread per (flow, cell): d_t u_i = (Q_{i+1} - Q_i)/ds and the stage.
__global__ __launch_bounds__(256) void fv_stage_kernel(FvArgs a) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= a.n_rows * a.n) return;
  const int64_t r = e / a.n, i = e - r * a.n;
  if (!a.alive[r]) {
    if (a.stage == 3) a.dudt[e] = __builtin_nan("");
    return;
  }
  const double *Q = a.Q + r * (a.n + 1);
  const double L = (Q[i + 1] - Q[i]) / a.ds;
  switch (a.stage) {
    case 0:
      a.ys[e] = a.y0[e] + a.h * L;
      break;
    case 1:
      a.ys[e] = 0.75 * a.y0[e] + 0.25 * (a.ys[e] + a.h * L);
      break;
    case 2:
      a.y0[e] = a.y0[e] / 3.0 + (2.0 / 3.0) * (a.ys[e] + a.h * L);
      break;
    default:
      a.dudt[e] = L;
      break;
  }
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
  const int64_t waves = a.n_rows * (a.n + 1);
  if (waves <= 0) return 0;
  hipLaunchKernelGGL(fv_flux_kernel, dim3((unsigned)((waves + 3) / 4)), dim3(256), 0,
                     (hipStream_t)stream, a);
  return (int)hipGetLastError();
}

int launch_fv_stage(const FvArgs &a, void *stream) {
  const int64_t m = a.n_rows * a.n;
  if (m <= 0) return 0;
  hipLaunchKernelGGL(fv_stage_kernel, dim3((unsigned)((m + 255) / 256)), dim3(256), 0,
                     (hipStream_t)stream, a);
  return (int)hipGetLastError();
}

int launch_fv_dt(const FvArgs &a, void *stream) {
  if (a.n_rows <= 0) return 0;
  hipLaunchKernelGGL(fv_dt_kernel, dim3((unsigned)a.n_rows), dim3(256), 0, (hipStream_t)stream, a);
  return (int)hipGetLastError();
}

}  // namespace frg
