// The context object behind the opaque frg_ctx handle (host side only).
#pragma once

#include <hip/hip_runtime.h>
#include <rocprofiler-sdk-roctx/roctx.h>

#include <atomic>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "frg_internal.h"

namespace frg {

// A named roctx range over a scope (entry points, server batches): shown by
// rocprofv3 --marker-trace, a few nanoseconds when no tool is attached.
struct TraceRange {
  explicit TraceRange(const char *name) { roctxRangePush(name); }
  ~TraceRange() { roctxRangePop(); }
  TraceRange(const TraceRange &) = delete;
  TraceRange &operator=(const TraceRange &) = delete;
};

int fail(int code, const char *fmt, ...);
int hip_fail(hipError_t e, const char *what);
void clear_error();
double now_s();
int check_quad(const frg_quad &q);
int check_lpa(const frg_lpa &l);
struct Context;
// noalloc.hip: once per device (that device current), the device address of
// the scratch area; and the context's pinned staging buffer
int noalloc_init(int device, Context *ctx);
void build_tiles(const std::vector<SetDev> &sd, int tile, std::vector<Tile> *tiles);
int max_table_bytes(const std::vector<SetDev> &sd);
bool any_fp32c(const std::vector<SetDev> &sd);

// Bytes of device memory held by a context's working buffers, checked
// against its HBM budget.
struct HbmAccount {
  std::atomic<uint64_t> used{0};
  uint64_t budget = ~0ull;
};

// Grow-only device allocation, charged to an account when it has one.
struct DevBuf {
  void *ptr = nullptr;
  size_t bytes = 0;
  HbmAccount *acct = nullptr;
  DevBuf() = default;
  explicit DevBuf(HbmAccount *a) : acct(a) {}
  DevBuf(const DevBuf &) = delete;
  DevBuf &operator=(const DevBuf &) = delete;
  ~DevBuf();
  int reserve(size_t b);
  void release();
};

// Pinned host + device slots for per-launch descriptor uploads.
struct DescRing {
  struct Slot {
    void *host = nullptr;
    void *dev = nullptr;
    hipEvent_t done = nullptr;
    bool used = false;
    size_t cap = 0;
  };
  std::vector<Slot> slots;
  size_t slot_bytes = 0;
  int next = 0;
  int init(size_t slot_bytes, int n_slots);
  void destroy();
  int upload(const void *src, size_t bytes, hipStream_t stream, void **dev, int *slot_id);
  int release(int slot_id, hipStream_t stream);
};

// Launch shapes.  Defaults below; the autotuner (autotune.cpp) replaces
// them per key with measured choices.  No launch shape changes a result.
struct GridCfg {
  int M = 8;    // masses per wave
  int W = 4;    // waves per workgroup
  int MB = 16;  // mass blocks per wave while the table is resident
};
struct PersistCfg {
  int tile = 4;  // work per tile of the persistent list, in units of 1024 evaluations
  int wpc = 24;  // resident one-wave workgroups per CU
};
using ShapeKey = std::tuple<int, int, int, int>;  // (regulator, n_r, n_a, precision)

struct Tune {
  GridCfg grid;
  int plain_tile = 8;
  int tab_W = 4;           // tabulated variant: waves per workgroup
  int tab_pw = 16;         // tabulated variant: momenta per wave
  int tab_lds_nodes = 6144;  // tabulated variant: rows up to this many nodes staged in LDS
  int tab_wpc = 8;         // tabulated variant, streamed rows: workgroups per CU
  int tab_sW = 2;          // tabulated variant, streamed rows: waves per workgroup
  int tab_spw = 1;         // tabulated variant, streamed rows: momenta per wave (at most)
  int tab_pairs = 1;       // tabulated variant: rows in LDS as (value, slope) pairs
  int tab_rb = 0;          // tabulated variant, rows in LDS: rows per workgroup (0: auto)
  int tab_rW = 16;         // tabulated variant, several rows per workgroup: waves per workgroup
  int tab_seg = 2;         // tabulated variant, rows longer than the LDS: segmented form (2: auto)
  PersistCfg persist;
  int grid_lds_rows = 64;  // (t, u) rows of 64 doubles staged per LDS chunk
  int grid_form = 0;       // resident FP64 grid: 0 per-momentum coefficients, 1 running fractions
  int grid_mfma = 1;       // coefficient form: 1 tiles of 16 masses on the matrix cores, 0 vector units
  int vertex_W = 12;       // vertex diagram, table over half the LDS: waves per workgroup (capped at 8 where registers need it)
  int pflow_fused = 1;     // momentum flow, rows in LDS: 1 one launch per stage; 0 diagram + stage launches
  int fv_persistent = 1;   // finite-volume solves: 1 one workgroup per flow, state in LDS; 0 launches per stage
  int server_zero_copy = 1;  // flow server: 1 kernel reads/writes the pinned batch buffer; 0 two copies
  int fp32c_flag_ppb = 100;    // FP32C: FP64 above this error bound (1e-9 units)
  int fp32c_band_ppm = 10000;  // FP32C: FP64 below this delta/k^2 (1e-6 units)
  int mode = 0;            // 0: defaults and cached choices, 1: tune new keys
  std::string cache_path;
  std::map<ShapeKey, GridCfg> grid_best;
  std::map<ShapeKey, int> plain_best;
  std::map<int, PersistCfg> persist_best;  // by precision
  void load_env();
  int load_file(const std::string &arch);
  int save_file(const std::string &arch) const;
};

// A captured persistent launch (FRG_GRAPH).  It is replayed only for the
// same stream and the same set descriptors (pointers, shapes, tables and the
// FP32C routing knobs) and launch shape; its work-list counter is its own,
// and replays on one stream run in order.
struct GraphEntry {
  DevBuf sets, tiles, counter;
  hipGraphExec_t exec = nullptr;
  hipEvent_t done = nullptr;  // recorded after every replay
  hipStream_t stream = nullptr;
  int *flag = nullptr;
  std::vector<SetDev> sd;
  PersistCfg pc;
  uint64_t last_use = 0;
  // the caller's set array of the last call that replayed this capture, and
  // the knob generation then: a call with the same bytes, stream and
  // generation replays it without rebuilding the descriptors
  std::vector<frg_set> raw;
  uint64_t gen = 0;
  GraphEntry() = default;
  GraphEntry(const GraphEntry &) = delete;
  GraphEntry &operator=(const GraphEntry &) = delete;
  ~GraphEntry();  // waits for the last replay
};
constexpr size_t kMaxGraphs = 32;  // least recently used entries are dropped beyond this

struct Server;

struct Context {
  int device = 0;
  int n_cu = 256;
  std::string arch;
  hipStream_t stream = nullptr;      // host-memory calls
  hipStream_t cap_stream = nullptr;  // graph capture
  std::mutex mu;
  // Domain word of the call in progress: the word of its stream (set at the
  // entry of every call that can meet a point outside the domain).  Each
  // stream has its own word, so calls on different streams never share one;
  // frg_stream_status reads and clears it.
  int *d_flag = nullptr;
  std::map<hipStream_t, int *> stream_flags;
  int use_stream_flag(hipStream_t st);
  frg::DescRing ring;
  frg::HbmAccount hbm;  // the working buffers below, the tables and captured work lists
  frg::DevBuf stage_in{&hbm}, stage_out{&hbm};
  // segmented tabulated form: partial sums, sorted term lists, their segment
  // offsets, counts + work counter
  frg::DevBuf tab_part{&hbm}, tab_terms{&hbm}, tab_offs{&hbm}, tab_scr{&hbm};
  hipEvent_t tab_done = nullptr;   // after the last segmented launch (which used them)
  frg::Tune tune;
  uint64_t tune_gen = 1;  // advanced whenever a knob or a tuned choice changes
  uint64_t hbm_budget = 0;

  struct QEntry {
    std::unique_ptr<frg::DevBuf> buf;
    frg::QuadTable host;
  };
  struct LEntry {
    std::unique_ptr<frg::DevBuf> buf;
    double Cd = 0.0;
  };
  std::map<std::tuple<int, int, uint64_t, uint64_t, int, int>, QEntry> qtabs;
  std::map<std::tuple<int, int, int, uint64_t>, LEntry> ltabs;
  std::vector<std::unique_ptr<frg::GraphEntry>> graphs;
  uint64_t graph_clock = 0;
  std::map<std::tuple<int, int, int>, std::unique_ptr<frg::DevBuf>> vtabs;  // (d, n_a, n_phi)
  frg::Server *server = nullptr;

  virtual ~Context();
  int quad_table(const frg_quad &q, const double **dev, frg::QuadTable *host_copy,
                 frg::QuadTable **host_ref = nullptr);
  int lpa_table(int d, int reg, int n_r, double qmk, const double **dev, double *Cd);
  int make_setdev(const frg_set &s, frg::SetDev *out);
  void fill_setdev(const frg_set &s, const frg::QuadTable &h, const double *tab, frg::SetDev *out);
  // noalloc.hip: pinned staging of the allocation-free call (filled and
  // copied to the device scratch area), the event after its last kernel, and
  // host-only quadrature tables of keys not in qtabs
  char *na_stage = nullptr;
  hipEvent_t na_done = nullptr;
  bool na_pending = false;
  std::map<std::tuple<int, int, uint64_t, uint64_t, int, int>, frg::QuadTable> htabs;
  const frg::QuadTable &host_quad_table(const frg_quad &q);
  int integrate_device(const frg_set *sets, int n_sets, int flags, hipStream_t st);
  // FRG_GRAPH: replay the capture made for exactly this set array, stream
  // and knob generation (1 if replayed, 0 if none matched, < 0 on error)
  int replay_graph(const frg_set *sets, int n_sets, hipStream_t st);
  int integrate_host(const frg_set *sets, int n_sets, int flags);
  int persistent(const std::vector<frg::SetDev> &sd, const frg_set *sets, int n_sets, int flags,
                 hipStream_t st);
  int tab_device(const frg_quad &q, const frg_gtab &tab, int64_t n_p, const double *p, double *out,
                 hipStream_t st);
  // Launch shape of the table kernel for a (fills R, J, T, U, pairs, pw and
  // n_pb of a): rows in LDS or streamed, waves per workgroup, streaming grid.
  // launch shape of the tabulated diagram; several rows per workgroup only
  // where the caller's kernel takes them
  int tab_config(frg::TabArgs &a, bool &lds_rows, int &W, int64_t &sblocks, bool multi_rows);
  int tab_launch(frg::TabArgs a, int reg, hipStream_t st);
  // pflow_api.cpp: momentum-dependent flow; dsdt != nullptr: one right-hand side
  // at t_rhs, else RK4 from 0 to t_end (all arrays on the device)
  int pflow_device(const frg_pflow &pf, int64_t n_flows, const double *lam3, const double *lam4,
                   double t_end, int64_t n_steps, double *sigma, double *t_reached,
                   double *dsdt, double t_rhs, int *flag, hipStream_t st);
  int grid_device(const frg_quad &q, int64_t n_p, const double *p, int64_t n_m, const double *m2,
                  double *out, double *err, uint8_t *used, hipStream_t st);
  int lpa_jobs(int n, const frg_lpa *lpa, const double *t, const double *const *U,
               double *const *dUdt, double *const *jac, int *flags_dev, hipStream_t st);
  // Descriptors of n LPA jobs (device pointers given) and their grid offsets
  // start[0..n]; no GPU work except building missing LPA tables.
  int lpa_job_table(int n, const frg_lpa *lpa, const double *t, const double *const *U,
                    double *const *dUdt, double *const *jac, int *flags_dev, LpaJob *jobs,
                    int64_t *start);
  void stop_server();
  // fvlpa_api.cpp: finite-volume LPA; dudt != nullptr: one right-hand side
  // at t_rhs (and dt_est if not null), else SSP-RK3 from 0 to t_end
  int fvlpa_device(const frg_fvlpa &f, int64_t n_flows, double t_end, int64_t n_steps, double *u,
                   double *t_reached, double *dudt, double *dt_est, double t_rhs, int *flag,
                   hipStream_t st);
  // vertex_api.cpp: two-external-momentum diagram on a (configuration x mass) grid
  int vertex_device(const frg_quad &q, int n_phi, int64_t n_c, const double *p1,
                    const double *p2, const double *c12, int64_t n_m, const double *m2,
                    double *out, hipStream_t st);
  // autotune.cpp
  int grid_launch(GridArgs g, int reg, const GridCfg &cfg, hipStream_t st);
  GridCfg grid_cfg(const frg_quad &q, const GridArgs &g, hipStream_t st);
  int plain_tile_for(const SetDev &s, hipStream_t st);
  PersistCfg persist_cfg(const std::vector<SetDev> &sd, int prec, hipStream_t st);
  // the tuned or default shape, never timing candidates
  PersistCfg persist_cfg_cached(const std::vector<SetDev> &sd, int prec) const;
  int persistent_eager(const std::vector<SetDev> &sd, const PersistCfg &pc, hipStream_t st);
};

using Ctx = Context;

}  // namespace frg

// The opaque handle of the C ABI.
struct frg_ctx : frg::Context {};
