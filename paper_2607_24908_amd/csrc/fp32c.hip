// Compensated-FP32 kernel (FRG_PREC_FP32C) for plain launches and tensor
// grids; the per-point arithmetic is in device_fp32c.h.
#include <hip/hip_runtime.h>

#include <cmath>

#include "frg_internal.h"

#pragma clang fp contract(off)

#include "device_fp32c.h"

namespace frg {

namespace {

using namespace dev;

// 4 waves per workgroup share the staged tables; each wave takes one tile.
// grid_nm > 0: point e is (p[e / grid_nm], m2[e % grid_nm]).
template <int REG>
__global__ __launch_bounds__(256) void fp32c_kernel(SetDev s, int tile_points, int64_t n_tiles,
                                                    int64_t grid_nm, int *flag) {
  extern __shared__ double lds[];
  const int ntab = table_doubles(s.n_r, s.n_a);
  const float *fo = reinterpret_cast<const float *>(lds + ntab);
  const float *fm = fo + s.n_a;
  const float *fl = fm + s.n_a;
  stage_fp32c(s, lds, threadIdx.x, blockDim.x);
  __syncthreads();
  const int lane = threadIdx.x & (kWave - 1);
  const int64_t tile = (int64_t)blockIdx.x * (blockDim.x / kWave) + (threadIdx.x / kWave);
  if (tile >= n_tiles) return;
  const int64_t start = tile * tile_points;
  const int64_t left = s.n_ext - start;
  const int count = left < tile_points ? (int)left : tile_points;
  fp32c_tile<REG>(s, lds, fo, fm, fl, start, count, grid_nm, lane, flag);
}

}  // namespace

int launch_fp32c(const SetDev &s, int tile_points, int64_t grid_nm, int *d_flag, void *stream) {
  if (s.n_ext <= 0) return 0;
  const int64_t n_tiles = (s.n_ext + tile_points - 1) / tile_points;
  const int waves = 4;
  const int64_t blocks = (n_tiles + waves - 1) / waves;
  const size_t lds = fp32c_lds_bytes(s.n_r, s.n_a);
  hipStream_t st = (hipStream_t)stream;
  if (s.reg == kExp)
    hipLaunchKernelGGL(fp32c_kernel<kExp>, dim3((unsigned)blocks), dim3(64 * waves), lds, st, s,
                       tile_points, n_tiles, grid_nm, d_flag);
  else
    hipLaunchKernelGGL(fp32c_kernel<kLitim>, dim3((unsigned)blocks), dim3(64 * waves), lds, st, s,
                       tile_points, n_tiles, grid_nm, d_flag);
  return (int)hipGetLastError();
}

}  // namespace frg
