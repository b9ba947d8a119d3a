// Tabulated-propagator flow diagram, rows too long for LDS (segmented form).
//
// Every row shares the interpolation coordinates t_e(p) = s_e / h of the
// terms e = (i, j): only the table values differ.  A row is cut into segments
// of kTabSegC nodes and kTabSegS consecutive segments form a superchunk.
//  1. tab_seg_sort_kernel, once per call: for each momentum, its terms sorted
//     by (segment of their node index, e) -- a list of e (16 bits) and the
//     offset of every segment in it, by a counting sort; term counts per
//     superchunk.
//  2. tab_seg_kernel: a work item is (batch of kTabSegRows rows, superchunk,
//     range of momenta).  Its workgroup copies the superchunk's segments of
//     its rows into LDS (two buffers: the next segment is copied straight from
//     memory while the current one is used); for each momentum the terms of
//     the segment are a run of its list, evaluated from LDS for all rows of
//     the batch with one coordinate.  Items are balanced on the term counts
//     (hot superchunks are split by momenta) and taken from a work counter.
//  3. tab_seg_reduce_kernel: the superchunks' partial sums, in order.
//
// Mapping: a momentum's run of a segment is taken by one wave, the 64 lanes
// on consecutive terms, and folded over the wave (wave_sum_fold).  The sum of
// one result is fixed by the shapes: per segment, the run's terms split over
// the lanes by position, each lane's terms in order, the fixed fold; the
// segments of a superchunk added in order into part[superchunk][row][momentum];
// the superchunks in order.  How momenta are split into items changes no bit.
#include <hip/hip_runtime.h>

#include <cmath>

#include "frg_internal.h"

#pragma clang fp contract(off)

#include "device_fp64.h"

namespace frg {

namespace {

using namespace dev;

constexpr int kC = kTabSegC;
constexpr int kS = kTabSegS;
constexpr int kRB = kTabSegRows;
static_assert(kRB == 4, "the run fold leaves one row per group of 16 lanes");
constexpr int kNT = kTabSegThreads;
constexpr int kRowLds = kC + 1;           // a segment's nodes and its right neighbour
constexpr int kBufD = kRB * kRowLds;      // doubles of one segment buffer

// Node index of an evaluation: k = min(floor(min(t, t_last)), k_last),
// t = fma(bh, 1 + x_j, ah) (the node and fraction of the piecewise-linear
// interpolant, as in the other tabulated kernels).
__device__ __forceinline__ int node_of(double t, double t_last, int k_last) {
  const int k = (int)fmin(t, t_last);
  return k < k_last ? k : k_last;
}

// A term e = (i, j) is stored as (i << 8) | j when both node counts fit a
// byte, else as i n_a + j; either way the terms of a segment keep the order
// (i, j), so the sums do not depend on the encoding.
__host__ __device__ __forceinline__ bool term_packed(const TabArgs &a) {
  return a.n_r <= 256 && a.n_a <= 256;
}

// Lane l's value of v (l wave-uniform).
__device__ __forceinline__ double readlane_d(double v, int l) {
  const unsigned long long b = __builtin_bit_cast(unsigned long long, v);
  const int lo = __builtin_amdgcn_readlane((int)(unsigned)b, l);
  const int hi = __builtin_amdgcn_readlane((int)(unsigned)(b >> 32), l);
  return __builtin_bit_cast(double, ((unsigned long long)(unsigned)hi << 32) | (unsigned)lo);
}

// Term counts per superchunk (hist) and the work counter, zeroed.
__global__ void tab_seg_zero_kernel(unsigned *hist, int n_super, int *counter) {
  for (int i = threadIdx.x + blockIdx.x * blockDim.x; i < n_super; i += blockDim.x * gridDim.x)
    hist[i] = 0u;
  if (blockIdx.x == 0 && threadIdx.x == 0) *counter = 0;
}

// Four waves per momentum: its terms e = i n_a + j sorted by (segment, e), a
// counting sort that uses the structure of the coordinates: for a fixed i
// the node index grows with j (the angular nodes ascend), so the j of one i
// that fall in one segment form a chunk of consecutive lanes.  Wave w takes
// the w-th quarter of the radial nodes.
//  1. counts per wave and segment: each chunk's head adds the chunk's size;
//  2. offs[p][s] = first position of segment >= s (exclusive scan over the
//     segments), and per wave and segment a cursor: the segment's start plus
//     the counts of the waves before it, so the quarters keep their order;
//     term counts per superchunk go to hist;
//  3. i in order within each wave: each chunk's head takes its position
//     from its wave's cursor and advances it; the chunk's lanes write their e.
// The order within a segment is ascending e.  Momenta outside the domain get
// empty runs.
constexpr int kSortW = 4;
static_assert(kS <= kWave && kWave % kS == 0, "superchunk sums within a wave's block");

__global__ __launch_bounds__(kSortW * kWave) void tab_seg_sort_kernel(TabArgs a, uint16_t *terms,
                                                                      int *offs, unsigned *hist,
                                                                      int n_seg) {
  extern __shared__ int cnt[];  // [kSortW][n_seg]: counts, then cursors
  const int64_t ip = blockIdx.x;
  const int tid = threadIdx.x, lane = tid % kWave, w = tid / kWave;
  const int n_r = a.n_r, n_a = a.n_a;
  const int E = n_r * n_a;
  int *po = offs + ip * (n_seg + 1);
  const double p = a.p[ip];
  if (!(p >= 0.0)) {  // uniform over the workgroup
    for (int x = tid; x <= n_seg; x += kSortW * kWave) po[x] = 0;
    return;
  }
  const int k_last = (int)a.n_s - 2;
  const double *opx = a.tab + 3 * n_r;
  for (int x = tid; x < kSortW * n_seg; x += kSortW * kWave) cnt[x] = 0;
  __syncthreads();
  int *mine = cnt + w * n_seg;
  const int i_lo = (int)((int64_t)w * n_r / kSortW), i_hi = (int)((int64_t)(w + 1) * n_r / kSortW);
  // segment of term (i, jb + lane) (q = q_i, oj = 1 + x_{jb + lane}) and the
  // chunk structure of this block of up to 64 j: head lanes (first lane or
  // segment change), chunk sizes, the last head at or before each lane
  auto chunk = [&](double q, double oj, int jb, int &sg, bool &head, int &size, int &hl) {
    const bool valid = jb + lane < n_a;
    sg = -1;
    if (valid) {
      const double qm = q - p;
      const double ah = (qm * qm) * a.inv_h;
      const double bh = ((2.0 * q) * p) * a.inv_h;
      sg = node_of(__builtin_fma(bh, oj, ah), a.t_last, k_last) / kC;
    }
    const int prev = __shfl_up(sg, 1, kWave);
    head = valid && (lane == 0 || prev != sg);
    const unsigned long long hm = __builtin_amdgcn_ballot_w64(head);
    const int nv = min(kWave, n_a - jb);  // valid lanes of the block
    const unsigned long long above = lane == 63 ? 0ull : hm >> (lane + 1);
    const int next = above ? lane + 1 + __builtin_ctzll(above) : nv;
    size = next - lane;
    const unsigned long long upto = hm & (lane == 63 ? ~0ull : ((2ull << lane) - 1ull));
    hl = 63 - __builtin_clzll(upto | 1ull);
  };
  // radial nodes 64 at a time in a register (q_i by readlane), the first 64
  // angular nodes in a register
  const double o0 = lane < n_a ? opx[lane] : 0.0;
  auto oj_of = [&](int jb) { return jb == 0 ? o0 : (jb + lane < n_a ? opx[jb + lane] : 0.0); };
  for (int i0 = i_lo; i0 < i_hi; i0 += kWave) {
    const double qv = i0 + lane < i_hi ? a.tab[i0 + lane] : 0.0;
    const int ni = min(kWave, i_hi - i0);
    for (int ii = 0; ii < ni; ++ii) {
      const double q = readlane_d(qv, ii);
      for (int jb = 0; jb < n_a; jb += kWave) {
        int sg, size, hl;
        bool head;
        chunk(q, oj_of(jb), jb, sg, head, size, hl);
        if (head) atomicAdd(&mine[sg], size);
      }
    }
  }
  __syncthreads();
  if (w == 0) {
    // exclusive scan over the segments, blocks of 64
    int carry = 0;
    for (int x0 = 0; x0 < n_seg; x0 += kWave) {
      const int x = x0 + lane;
      int c[kSortW], tot = 0;
#pragma unroll
      for (int v = 0; v < kSortW; ++v) {
        c[v] = x < n_seg ? cnt[v * n_seg + x] : 0;
        tot += c[v];
      }
      int incl = tot;
#pragma unroll
      for (int d = 1; d < kWave; d <<= 1) {
        const int t = __shfl_up(incl, d, kWave);
        if (lane >= d) incl += t;
      }
      int run = carry + incl - tot;
      if (x < n_seg) {
        po[x] = run;
#pragma unroll
        for (int v = 0; v < kSortW; ++v) {
          cnt[v * n_seg + x] = run;
          run += c[v];
        }
      }
      // terms of each superchunk of this block (kS lanes each)
      int hs = tot;
#pragma unroll
      for (int d = 1; d < kS; d <<= 1) hs += __shfl_xor(hs, d, kWave);
      if (lane % kS == 0 && x < n_seg && hs) atomicAdd(&hist[x / kS], (unsigned)hs);
      carry += __shfl(incl, kWave - 1, kWave);
    }
    if (lane == 0) po[n_seg] = carry;  // = E
  }
  __syncthreads();
  uint16_t *pt = terms + ip * E;
  for (int i0 = i_lo; i0 < i_hi; i0 += kWave) {
    const double qv = i0 + lane < i_hi ? a.tab[i0 + lane] : 0.0;
    const int ni = min(kWave, i_hi - i0);
    for (int ii = 0; ii < ni; ++ii) {
      const double q = readlane_d(qv, ii);
      const int i = i0 + ii;
      for (int jb = 0; jb < n_a; jb += kWave) {
        int sg, size, hl;
        bool head;
        chunk(q, oj_of(jb), jb, sg, head, size, hl);
        int base = 0;
        if (head) {
          base = mine[sg];
          mine[sg] = base + size;
        }
        base = __shfl(base, hl, kWave);
        const int j = jb + lane;
        if (j < n_a) pt[base + (lane - hl)] = (uint16_t)(term_packed(a) ? (i << 8) | j : i * n_a + j);
      }
    }
  }
}

// Momenta split of superchunk c: between ceil(n_p / kItemMax) items and
// ceil(n_p / kItemMin), in proportion to its cost (terms + kNodeW * nodes,
// the copy of a node for the batch weighed against a term's work).
constexpr double kNodeW = 8.0;
constexpr int kWaves = kNT / kWave;
constexpr int kItemMax = kNT;     // momenta per item: one per lane
constexpr int kItemMin = kWaves;  // one per wave

__device__ __forceinline__ double super_nodes(const TabArgs &a, int c, int n_seg) {
  const int s0 = c * kS, s1 = min(s0 + kS, n_seg);
  const int64_t k0 = (int64_t)s0 * kC;
  const int64_t k1 = min((int64_t)s1 * kC, a.n_s - 1);
  return (double)(k1 - k0);
}

// Work items from the counter until the list is drained.  Momentum ip of an
// item is owned by lane l of wave w with ip = p_lo + w + kWaves l; for each
// segment a wave takes the non-empty runs of its momenta one after another,
// all 64 lanes on one run (lane l: positions o + l, o + l + 64, ...), and the
// four row sums of the run are folded over the wave and added by the owner.
template <bool PACKED>
__global__ __launch_bounds__(kNT) void tab_seg_kernel(TabArgs a, const unsigned *hist,
                                                      const uint16_t *__restrict__ terms,
                                                      const int *__restrict__ offs, int *counter,
                                                      double *part, int n_seg, int n_super,
                                                      int n_batch, int target) {
  extern __shared__ double lds[];
  const int n_r = a.n_r, n_a = a.n_a;
  const int tid = threadIdx.x;
  double *lg0 = lds;                      // two segment buffers [kRB][kRowLds]
  // radial slots [n_r][1 + kRB]: q_i, then A_i of the batch's rows; angular
  // slots [n_a][2]: 1 + x_j, mu_j (one address per node)
  constexpr int kRS = 1 + kRB;
  double *lrad = lg0 + 2 * kBufD;
  double *lang = lrad + kRS * n_r;
  int *ns = reinterpret_cast<int *>(lang + 2 * n_a);  // splits per superchunk
  int *ord = ns + n_super;                       // superchunks, costliest first
  long long *pre = reinterpret_cast<long long *>(ord + n_super);  // item prefix (8-byte aligned)
  int *claim = reinterpret_cast<int *>(pre + n_super + 1);
  for (int i = tid; i < n_r; i += kNT) lrad[i * kRS] = a.tab[i];
  for (int j = tid; j < n_a; j += kNT) {
    lang[2 * j] = a.tab[3 * n_r + j];
    lang[2 * j + 1] = a.tab[3 * n_r + n_a + j];
  }
  // the plan (the same in every workgroup)
  const int smin = (int)((a.n_p + kItemMax - 1) / kItemMax);
  const int smax = (int)((a.n_p + kItemMin - 1) / kItemMin);
  double total = 0.0;
  for (int c = 0; c < n_super; ++c) total += (double)hist[c] + kNodeW * super_nodes(a, c, n_seg);
  const double budget = total / (double)target;
  for (int c = tid; c < n_super; c += kNT) {
    const double cost = (double)hist[c] + kNodeW * super_nodes(a, c, n_seg);
    int s = (int)ceil(cost / budget);
    s = s < smin ? smin : (s > smax ? smax : s);
    ns[c] = s;
    // rank: costlier first, ties by index
    int rank = 0;
    for (int d = 0; d < n_super; ++d) {
      const double cd = (double)hist[d] + kNodeW * super_nodes(a, d, n_seg);
      rank += (cd > cost || (cd == cost && d < c)) ? 1 : 0;
    }
    ord[rank] = c;
  }
  __syncthreads();
  if (tid == 0) {
    long long acc = 0;
    for (int r = 0; r < n_super; ++r) {
      pre[r] = acc;
      acc += (long long)ns[ord[r]] * n_batch;
    }
    pre[n_super] = acc;
  }
  __syncthreads();
  const long long n_items = pre[n_super];
  const int k_last = (int)a.n_s - 2;
  const int E = n_r * n_a;
  const float inv_na = 1.0f / (float)n_a;
  const int wave = tid / kWave, lane = tid % kWave;
  for (;;) {
    if (tid == 0) *claim = atomicAdd(counter, 1);
    __syncthreads();
    const long long item = *claim;
    __syncthreads();  // every thread has read the claim
    if (item >= n_items) break;
    // decode: rank (superchunk), then batch, then momentum split
    int ra = 0, rb = n_super;
    while (rb - ra > 1) {
      const int m = (ra + rb) >> 1;
      if (pre[m] <= item) ra = m; else rb = m;
    }
    const int c = ord[ra];
    const int nsc = ns[c];
    const long long off = item - pre[ra];
    const int b = (int)(off / nsc), msp = (int)(off % nsc);
    const int64_t p_lo = (int64_t)msp * a.n_p / nsc, p_hi = (int64_t)(msp + 1) * a.n_p / nsc;
    const int64_t r0 = (int64_t)b * kRB;
    const int nrb = (int)min<int64_t>(kRB, a.n_rows - r0);
    // A_i = c_i G_r(q_i^2)^2 of the batch's rows
    for (int x = tid; x < kRB * n_r; x += kNT) {
      const int r = x / n_r, i = x - r * n_r;
      double A = 0.0;
      if (r < nrb) {
        const double *row = a.g + (r0 + r) * a.n_s;
        const double q = lrad[i * kRS];
        const double t = fmin((q * q) * a.inv_h, a.t_last);
        int k = (int)t;
        k = k < k_last ? k : k_last;
        const double f = t - (double)k;
        const double g0 = row[k], g1 = row[k + 1];
        const double G = __builtin_fma(f, g1 - g0, g0);
        A = (a.tab[n_r + i] * G) * G;
      }
      lrad[i * kRS + 1 + r] = A;
    }
    // this lane's momentum
    const int64_t my = p_lo + wave + (int64_t)kWaves * lane;
    const bool mine = my < p_hi;
    const double pv = mine ? a.p[my] : -1.0;
    const bool live = pv >= 0.0;  // NaN and p < 0 have no terms
    const int *pof = offs + (mine ? my : 0) * (int64_t)(n_seg + 1);
    // accumulators: lane L = 16 r + s holds row r of the wave's momenta
    // l = s, s + 16, s + 32, s + 48 (acc[l / 16]), where the fold below
    // leaves the row sums of a run
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    const int sg0 = c * kS, sg1 = min(sg0 + kS, n_seg);
    // copy segment sg of the batch's rows into buffer d: waves w, w + kRB, ...
    // take row w % kRB, 4 bytes per lane and 256 contiguous bytes of LDS per
    // wave instruction; words beyond the table are left unwritten (never read)
    const int lrow = wave % kRB;
    const unsigned *grow32 = reinterpret_cast<const unsigned *>(a.g + (r0 + lrow) * a.n_s);
    const int64_t words = 2 * a.n_s;  // 4-byte words of a row
    auto load = [&](int sg, int d) {
      if (lrow >= nrb) return;  // wave-uniform: no such row in the batch
      const int64_t w0 = 2 * (int64_t)sg * kC;
      unsigned *dst = reinterpret_cast<unsigned *>(lg0 + d * kBufD + lrow * kRowLds);
      for (int m = wave / kRB; m * kWave < 2 * kRowLds; m += kWaves / kRB) {  // wave-uniform
        const int x = m * kWave + lane;
        if (x < 2 * kRowLds && w0 + x < words)
          __builtin_amdgcn_global_load_lds(
              grow32 + w0 + x, (__attribute__((address_space(3))) void *)(dst + m * kWave), 4, 0,
              0);
      }
    };
    load(sg0, 0);
    // run bounds of this lane's momentum: segment sg, and sg + 1 ahead
    int o_cur = live ? pof[sg0] : 0;
    int o_nxt = live ? pof[sg0 + 1] : 0;
    for (int sg = sg0; sg < sg1; ++sg) {
      const int cur = (sg - sg0) & 1;
      const int o_after = (live && sg + 2 <= n_seg) ? pof[sg + 2] : 0;
      // this wave's copies of segment sg have landed; after the barrier every
      // wave's have, and every wave is done with the other buffer
      __builtin_amdgcn_s_waitcnt(0);
      __syncthreads();
      if (sg + 1 < sg1) load(sg + 1, cur ^ 1);
      const double *lg = lg0 + cur * kBufD;
      const int T0 = sg * kC;
      unsigned long long todo = __builtin_amdgcn_ballot_w64(live && o_nxt > o_cur);
      while (todo) {  // wave-uniform: the momenta with terms in this segment
        const int l = __builtin_ctzll(todo);
        todo &= todo - 1ull;
        const int ra0 = __builtin_amdgcn_readlane(o_cur, l);
        const int ra1 = __builtin_amdgcn_readlane(o_nxt, l);
        const double p = readlane_d(pv, l);
        const int64_t ip = p_lo + wave + (int64_t)kWaves * l;
        const uint16_t *pt = terms + ip * E;
        double in[kRB];
#pragma unroll
        for (int r = 0; r < kRB; ++r) in[r] = 0.0;
        for (int pos = ra0 + lane; pos < ra1; pos += kWave) {
          const unsigned e = pt[pos];
          int i, j;
          if constexpr (PACKED) {
            i = (int)(e >> 8);
            j = (int)(e & 255u);
          } else {
            // e = i n_a + j (exact: e < 2^16, and e + 1/2 is at least
            // 1/(2 n_a) away from a multiple of n_a)
            i = (int)(((float)e + 0.5f) * inv_na);
            j = (int)e - i * n_a;
          }
          const double *rad = lrad + i * kRS;
          const double q = rad[0];
          const double qm = q - p;
          const double ah = (qm * qm) * a.inv_h;
          const double bh = ((2.0 * q) * p) * a.inv_h;
          const double t = fmin(__builtin_fma(bh, lang[2 * j], ah), a.t_last);
          int k = (int)t;
          k = k < k_last ? k : k_last;
          const double f = t - (double)k;
          const double mu = lang[2 * j + 1];
          // k lies in the segment by construction; the clamp only keeps the
          // LDS index in bounds
          int x = k - T0;
          x = x < 0 ? 0 : (x > kC - 1 ? kC - 1 : x);
#pragma unroll
          for (int r = 0; r < kRB; ++r) {
            const double g0 = lg[r * kRowLds + x], g1 = lg[r * kRowLds + x + 1];
            in[r] = __builtin_fma(rad[1 + r] * mu, __builtin_fma(f, g1 - g0, g0), in[r]);
          }
        }
        // lane groups of 16 end with the sums of rows 0..3
        const double rs = wave_sum_fold<kRB>(in, lane);
        if ((lane & 15) == (l & 15)) {
          switch (l >> 4) {  // wave-uniform: one add, not four selected ones
            case 0: acc[0] += rs; break;
            case 1: acc[1] += rs; break;
            case 2: acc[2] += rs; break;
            default: acc[3] += rs; break;
          }
        }
      }
      o_cur = o_nxt;
      o_nxt = o_after;
    }
    {
      const int r = lane >> 4;
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const int64_t ip = p_lo + wave + (int64_t)kWaves * ((lane & 15) + 16 * k);
        if (r < nrb && ip < p_hi) part[((int64_t)c * a.n_rows + r0 + r) * a.n_p + ip] = acc[k];
      }
    }
  }
}

// out[a, r] = pref sum_c part[c][r][a] (superchunks in order); NaN and the
// domain flag for p < 0.
__global__ void tab_seg_reduce_kernel(TabArgs a, const double *part, int n_super) {
  const int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (x >= a.n_p * a.n_rows) return;
  const int64_t r = x / a.n_p, ip = x - r * a.n_p;
  const double p = a.p[ip];
  double v;
  if (p >= 0.0) {
    double s = 0.0;
    for (int c = 0; c < n_super; ++c) s = s + part[((int64_t)c * a.n_rows + r) * a.n_p + ip];
    v = a.pref * s;
  } else {
    v = __builtin_nan("");
    if (r == 0) *a.flag = 1;
  }
  a.out[ip * a.os_p + r * a.os_r] = v;
}

}  // namespace

TabSegShape tab_seg_shape(const TabArgs &t, int n_cu) {
  TabSegShape s;
  s.n_seg = (int)((t.n_s - 1 + kC - 1) / kC);
  s.n_super = (s.n_seg + kS - 1) / kS;
  s.n_batch = (int)((t.n_rows + kRB - 1) / kRB);
  const int64_t want = 4LL * n_cu;
  s.target = (int)std::max<int64_t>(s.n_super, (want + s.n_batch - 1) / s.n_batch);
  s.lds = (int)(sizeof(double) * (2 * kBufD + t.n_r + kRB * t.n_r + 2 * t.n_a) +
                sizeof(int) * 2 * s.n_super + sizeof(long long) * (s.n_super + 1) + sizeof(int));
  return s;
}

int launch_tab_seg(const TabArgs &t, const TabSegShape &s, const TabSegBufs &b, int n_cu,
                   void *stream) {
  if (t.n_p <= 0 || t.n_rows <= 0) return 0;
  hipStream_t st = (hipStream_t)stream;
  static const bool once =
      ((void)hipFuncSetAttribute((const void *)&tab_seg_kernel<true>,
                                 hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024),
       (void)hipFuncSetAttribute((const void *)&tab_seg_kernel<false>,
                                 hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024),
       (void)hipFuncSetAttribute((const void *)&tab_seg_sort_kernel,
                                 hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024),
       (void)hipGetLastError(), true);
  (void)once;
  hipLaunchKernelGGL(tab_seg_zero_kernel, dim3(1), dim3(256), 0, st, b.hist, s.n_super, b.counter);
  hipLaunchKernelGGL(tab_seg_sort_kernel, dim3((unsigned)t.n_p), dim3(kSortW * kWave),
                     sizeof(int) * kSortW * s.n_seg, st, t, b.terms, b.offs, b.hist, s.n_seg);
  if (term_packed(t))
    hipLaunchKernelGGL(tab_seg_kernel<true>, dim3((unsigned)n_cu), dim3(kNT), (size_t)s.lds, st, t,
                       (const unsigned *)b.hist, (const uint16_t *)b.terms, (const int *)b.offs,
                       b.counter, b.part, s.n_seg, s.n_super, s.n_batch, s.target);
  else
    hipLaunchKernelGGL(tab_seg_kernel<false>, dim3((unsigned)n_cu), dim3(kNT), (size_t)s.lds, st,
                       t, (const unsigned *)b.hist, (const uint16_t *)b.terms,
                       (const int *)b.offs, b.counter, b.part, s.n_seg, s.n_super, s.n_batch,
                       s.target);
  const int64_t n = t.n_p * t.n_rows;
  hipLaunchKernelGGL(tab_seg_reduce_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, t,
                     (const double *)b.part, s.n_super);
  return (int)hipGetLastError();
}

}  // namespace frg
