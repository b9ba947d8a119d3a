// Tabulated-propagator flow diagram (gfx950): the propagator comes from a
// caller's table (one row per field value, piecewise-linear in s = q^2), the
// regulator insertion d_tR from the quadrature table.  A workgroup owns one
// table row (or, with rows in LDS, RB rows that share every coordinate) and
// W * pw momenta; each wave evaluates its momenta one after another with the
// 64 lanes over the quadrature nodes (up to 8 angular lanes per radial node,
// so that neighbouring lanes read neighbouring table entries) and stores
// them together.  Rows of up to tab_lds_max_nodes nodes are staged in LDS;
// longer rows are read through the caches, with the workgroups of one row
// placed on one XCD.  All forms do the same arithmetic in the same order.
#include <hip/hip_runtime.h>

#include <cmath>

#include "frg_internal.h"

#pragma clang fp contract(off)

#include "device_fp64.h"
#include "device_tab.h"

namespace frg {

namespace {

using namespace dev;

// LDS_ROW: one workgroup per (group of RB rows, momentum block), the rows
// staged in LDS.
// Otherwise a fixed grid of 8 * slots workgroups: workgroup b runs on XCD
// b mod 8 (round-robin dispatch) and works through the rows of that XCD one
// after another, taking momentum blocks slot, slot + slots, ... of each, so
// that each XCD streams one row at a time through its L2 and the rows in
// flight on the chip stay within the memory-side cache.
// UR > 0: every lane holds at most UR angular nodes (U <= UR), kept in
// registers; UR == 0: read from LDS.  RB rows per workgroup (rows in LDS):
// the rows share every coordinate and node index, each row's sums are those
// of the row alone.
template <bool LDS_ROW, int UR, bool PAIRS, int RB>
__global__ __launch_bounds__(RB > 1 ? 1024 : 256) void tab_kernel(TabArgs a) {
  extern __shared__ double lds[];
  const int W = blockDim.x / kWave;
  const int wave = threadIdx.x / kWave;
  const int lane = threadIdx.x & (kWave - 1);
  const TabLds l = tab_lds(a, lds, RB);
  if constexpr (LDS_ROW) {
    const int64_t rg = blockIdx.x / a.n_pb;
    tab_rows_block<UR, PAIRS, RB>(a, l, rg, blockIdx.x - rg * a.n_pb, W, wave, lane);
  } else {
    const int x = blockIdx.x & 7;
    const int64_t slot = blockIdx.x >> 3, slots = gridDim.x >> 3;
    for (int64_t r = x; r < a.n_rows; r += 8) {
      const PlainRow grow{a.g + r * a.n_s};
      __syncthreads();  // the previous row's A_i are no longer read
      tab_stage_A(a, grow, l.lrad);
      __syncthreads();
      for (int64_t pb = slot; pb < a.n_pb; pb += slots)
        tab_block<UR>(a, grow, l.lrad, l.lo, l.lm, r, pb, W, wave, lane);
    }
  }
}

}  // namespace

void tab_lane_split(int n_r, int n_a, int *R, int *J, int *T, int *U) {
  int j = 1;
  while (j * 2 <= n_a && j * 2 <= 8) j *= 2;
  *J = j;
  *R = kWave / j;
  *T = (n_r + *R - 1) / *R;
  *U = (n_a + j - 1) / j;
}

int tab_lds_bytes(const TabArgs &t, bool lds_rows) {
  const int rb = lds_rows && t.rb > 1 ? t.rb : 1;
  const int row = !lds_rows ? 0 : t.pairs ? (int)(2 * t.n_s) : (int)t.n_s;
  int R, J, T, U;
  tab_lane_split(t.n_r, t.n_a, &R, &J, &T, &U);
  return (int)(sizeof(double) * ((1 + rb) * R * T + 2 * t.n_a + rb * row));
}

// Dynamic LDS beyond 64 KiB (gfx950: 160 KiB per workgroup); a refusal where
// no opt-in is needed is cleared so that it cannot be taken for a launch error.
static void tab_allow_large_lds(const void *fn) {
  (void)hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
  (void)hipGetLastError();
}

template <bool L, int UR, bool P, int RB = 1>
static void tab_launch_t(const TabArgs &t, int W, int64_t blocks, hipStream_t st) {
  static const bool once = (tab_allow_large_lds((const void *)&tab_kernel<L, UR, P, RB>), true);
  (void)once;
  hipLaunchKernelGGL((tab_kernel<L, UR, P, RB>), dim3((unsigned)blocks), dim3(kWave * W),
                     tab_lds_bytes(t, L), st, t);
}

template <bool P, int RB>
static void tab_launch_rows(const TabArgs &t, bool regs, int W, int64_t blocks, hipStream_t st) {
  regs ? tab_launch_t<true, 4, P, RB>(t, W, blocks, st)
       : tab_launch_t<true, 0, P, RB>(t, W, blocks, st);
}

int launch_tab(const TabArgs &t, int reg, int W, bool lds_rows, int64_t stream_blocks,
               void *stream) {
  (void)reg;  // the regulator enters through the quadrature table only
  if (t.n_p <= 0 || t.n_rows <= 0) return 0;
  hipStream_t st = (hipStream_t)stream;
  const bool regs = t.U <= 4;
  if (lds_rows) {
    const int rb = t.rb > 1 ? t.rb : 1;
    if (rb != 1 && rb != 2 && rb != 4) return (int)hipErrorInvalidValue;
    if (W < 1 || W * kWave > (rb > 1 ? 1024 : 256)) return (int)hipErrorInvalidValue;
    const int64_t blocks = ((t.n_rows + rb - 1) / rb) * t.n_pb;
    if (rb == 4)
      t.pairs ? tab_launch_rows<true, 4>(t, regs, W, blocks, st)
              : tab_launch_rows<false, 4>(t, regs, W, blocks, st);
    else if (rb == 2)
      t.pairs ? tab_launch_rows<true, 2>(t, regs, W, blocks, st)
              : tab_launch_rows<false, 2>(t, regs, W, blocks, st);
    else
      t.pairs ? tab_launch_rows<true, 1>(t, regs, W, blocks, st)
              : tab_launch_rows<false, 1>(t, regs, W, blocks, st);
  } else {
    const int64_t blocks = 8 * ((stream_blocks + 7) / 8);
    regs ? tab_launch_t<false, 4, false>(t, W, blocks, st) : tab_launch_t<false, 0, false>(t, W, blocks, st);
  }
  return (int)hipGetLastError();
}

}  // namespace frg
