// Two-external-momentum (vertex) diagram behind frg_integrate_vertex:
// argument checks, the angular table of the azimuthal rule (cached per
// (d, n_a, n_phi)), and the launch shape of vertex_kernel.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>

#include "frg_ctx.h"

namespace frg {

int Ctx::vertex_device(const frg_quad &q, int n_phi, int64_t n_c, const double *p1,
                       const double *p2, const double *c12, int64_t n_m, const double *m2,
                       double *out, hipStream_t st) {
  const double *tab;
  QuadTable h;
  int rc = quad_table(q, &tab, &h);
  if (rc) return rc;
  auto key = std::make_tuple(q.d, q.n_angular, n_phi);
  auto it = vtabs.find(key);
  if (it == vtabs.end()) {
    const std::vector<double> t = build_vertex_table(q.d, q.n_angular, n_phi);
    auto buf = std::make_unique<DevBuf>(&hbm);
    rc = buf->reserve(t.size() * sizeof(double));
    if (rc) return rc;
    hipError_t e = hipMemcpy(buf->ptr, t.data(), t.size() * sizeof(double), hipMemcpyHostToDevice);
    if (e != hipSuccess) return hip_fail(e, "upload vertex table");
    it = vtabs.emplace(key, std::move(buf)).first;
  }
  GridArgs g{};
  g.p = p1;
  g.p2 = p2;
  g.c12 = c12;
  g.vtab = (const double *)it->second->ptr;
  g.m2 = m2;
  g.out = out;
  g.tab = tab;
  g.flag = d_flag;
  g.k2 = h.k2;
  g.inv_k2 = h.inv_k2;
  g.pref = omega_sphere(q.d - 2) / std::pow(2.0 * M_PI, q.d);
  g.q_top = h.q_top;
  g.n_p = n_c;
  g.n_m = n_m;
  g.n_r = q.n_radial;
  g.n_a = q.n_angular;
  g.n_phi = n_phi;
  g.T = (q.n_radial * q.n_angular + kWave - 1) / kWave;  // (radial, polar) pairs per lane
  g.U = n_phi;
  set_fold_scale(g, h, 3);
  // launch shape: the grid kernel's (tiles of 16 masses on the matrix cores,
  // or M <= 8 on the vector units); mass blocks so that about four
  // workgroups per CU are in flight -- or one, when the table takes more than
  // half the LDS (one workgroup per CU can be resident; it gets vertex_W
  // waves, up to three per SIMD where the registers allow, and splitting a
  // configuration's masses over more workgroups would only repeat its table
  // build)
  GridCfg cfg = tune.grid;
  cfg.M = tune.grid_mfma ? 16 : std::min(cfg.M, 8);
  g.mblocks = 1;
  const bool big = vertex_lds_bytes(g, cfg.M, cfg.W, true) > 80 * 1024;
  if (big) cfg.W = std::min(tune.vertex_W, vertex_max_waves(cfg.M, vertex_group(n_phi)));
  const int64_t per_wg = (int64_t)cfg.M * cfg.W;
  const int64_t want_wgs = (big ? 1LL : 4LL) * n_cu;
  int mbk = std::max(1, cfg.MB);
  while (mbk > 1 && (n_c * ((n_m + per_wg * mbk - 1) / (per_wg * mbk)) < want_wgs ||
                     grid_coef_stage_bytes(mbk, cfg.W, cfg.M) > kGridCoefStageMax))
    mbk /= 2;
  g.mblocks = mbk;
  g.n_mb = (int)((n_m + per_wg * mbk - 1) / (per_wg * mbk));
  const bool fits = std::isnormal(g.pref_c) && std::isnormal(g.sig) && tune.grid_form != 1 &&
                    vertex_lds_bytes(g, cfg.M, cfg.W, true) <= kGridCoefLdsMax;
  g.form = fits ? 0 : 1;  // 1: no resident table, every mass per term
  if (!fits && vertex_lds_bytes(g, cfg.M, cfg.W, false) > 64 * 1024)
    return fail(FRG_E_INVAL, "vertex tables exceed the LDS");
  const int e = launch_vertex(g, q.reg, cfg.M, cfg.W, st);
  if (e) return hip_fail((hipError_t)e, "vertex_kernel launch");
  return FRG_OK;
}

}  // namespace frg

using namespace frg;

extern "C" {

int frg_integrate_vertex(frg_ctx *ctx, const frg_quad *quad, int32_t n_azimuth, int64_t n_c,
                         const double *p1, const double *p2, const double *cos12, int64_t n_m,
                         const double *m2, double *out, int32_t mem, void *hip_stream) {
  frg::TraceRange trace_("frg_integrate_vertex");
  if (!ctx || !quad) return fail(FRG_E_INVAL, "NULL argument");
  int rc = check_quad(*quad);
  if (rc) return rc;
  if (quad->prec != FRG_PREC_FP64) return fail(FRG_E_INVAL, "the vertex diagram is FP64 only");
  if (n_azimuth < 1 || n_azimuth > 64) return fail(FRG_E_INVAL, "n_azimuth outside [1, 64]");
  if (n_c < 0 || n_m < 0) return fail(FRG_E_INVAL, "negative size");
  if (n_c > ((int64_t)1 << 30) || n_m > ((int64_t)1 << 30) || n_c * n_m > ((int64_t)1 << 40))
    return fail(FRG_E_INVAL, "problem too large");
  if (mem != FRG_MEM_HOST && mem != FRG_MEM_DEVICE) return fail(FRG_E_INVAL, "bad mem");
  if (n_c == 0 || n_m == 0) return FRG_OK;
  if (!p1 || !p2 || !cos12 || !m2 || !out) return fail(FRG_E_INVAL, "NULL array");
  std::lock_guard<std::mutex> lk(ctx->mu);
  hipSetDevice(ctx->device);
  clear_error();
  if (int rcf = ctx->use_stream_flag(mem == FRG_MEM_HOST ? ctx->stream : (hipStream_t)hip_stream))
    return rcf;
  if (mem == FRG_MEM_DEVICE)
    return ctx->vertex_device(*quad, n_azimuth, n_c, p1, p2, cos12, n_m, m2, out,
                              (hipStream_t)hip_stream);
  hipStream_t st = ctx->stream;
  const size_t nout = (size_t)(n_c * n_m);
  rc = ctx->stage_in.reserve((3 * n_c + n_m) * sizeof(double) + 64);
  if (!rc) rc = ctx->stage_out.reserve(nout * sizeof(double) + 64);
  if (rc) return rc;
  double *d1 = (double *)ctx->stage_in.ptr, *d2 = d1 + n_c, *dc = d2 + n_c, *dm = dc + n_c;
  double *dout = (double *)ctx->stage_out.ptr;
  hipMemcpyAsync(d1, p1, n_c * sizeof(double), hipMemcpyHostToDevice, st);
  hipMemcpyAsync(d2, p2, n_c * sizeof(double), hipMemcpyHostToDevice, st);
  hipMemcpyAsync(dc, cos12, n_c * sizeof(double), hipMemcpyHostToDevice, st);
  hipMemcpyAsync(dm, m2, n_m * sizeof(double), hipMemcpyHostToDevice, st);
  hipMemsetAsync(ctx->d_flag, 0, sizeof(int), st);
  rc = ctx->vertex_device(*quad, n_azimuth, n_c, d1, d2, dc, n_m, dm, dout, st);
  if (rc) {
    hipStreamSynchronize(st);
    return rc;
  }
  hipMemcpyAsync(out, dout, nout * sizeof(double), hipMemcpyDeviceToHost, st);
  int flag = 0;
  hipMemcpyAsync(&flag, ctx->d_flag, sizeof(int), hipMemcpyDeviceToHost, st);
  hipError_t e = hipStreamSynchronize(st);
  if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
  if (flag)
    return fail(FRG_E_DOMAIN, "some points have m^2 + k^2 <= 0, a negative momentum or |cos| > 1; "
                              "their results are NaN");
  return FRG_OK;
}

}  // extern "C"
