"""Thin ctypes binding of libfrg (include/frg.h).

Argument marshalling only: every step of the computation runs in the HIP
library.  Functions keep the C names; device buffers are passed as torch
tensors (their data pointers) or raw integer addresses, host buffers as numpy
arrays.  Importing this module loads ``libfrg.so`` and raises if it is
missing -- there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libfrg.so")

FRG_OK, FRG_PENDING = 0, 1
FRG_E_INVAL, FRG_E_DOMAIN, FRG_E_NOMEM, FRG_E_DEVICE = -1, -2, -3, -4
FRG_E_AGAIN, FRG_E_NOTFOUND, FRG_E_STEP = -5, -6, -7
FRG_REG_EXP, FRG_REG_LITIM = 0, 1
FRG_PREC_FP64, FRG_PREC_FP32C = 0, 1
FRG_MEM_HOST, FRG_MEM_DEVICE = 0, 1
FRG_PLAIN, FRG_PERSISTENT, FRG_GRAPH = 0, 1, 2

STATUS_NAMES = {0: "FRG_OK", 1: "FRG_PENDING", -1: "FRG_E_INVAL", -2: "FRG_E_DOMAIN",
                -3: "FRG_E_NOMEM", -4: "FRG_E_DEVICE", -5: "FRG_E_AGAIN",
                -6: "FRG_E_NOTFOUND", -7: "FRG_E_STEP"}

EXPORTS = ["frg_create", "frg_destroy", "frg_last_error", "frg_version", "frg_integrate",
           "frg_integrate_grid", "frg_integrate_tab", "frg_integrate_vertex", "frg_pflow_rhs",
           "frg_pflow_solve", "frg_fvlpa_rhs", "frg_fvlpa_solve",
           "frg_flow_rhs", "frg_flow_rhs_batch", "frg_flow_solve",
           "frg_submit", "frg_poll", "frg_server_stats", "frg_gauss_legendre",
           "frg_flow_footprint", "frg_autotune", "frg_tune_set", "frg_tune_get", "frg_expneg",
           "frg_stream_status", "frg_integrate_noalloc", "frg_expneg_fp32c"]


class frg_quad(ctypes.Structure):
    _fields_ = [("d", ctypes.c_int32), ("reg", ctypes.c_int32), ("k", ctypes.c_double),
                ("q_max", ctypes.c_double), ("n_radial", ctypes.c_int32),
                ("n_angular", ctypes.c_int32), ("prec", ctypes.c_int32),
                ("reserved", ctypes.c_int32)]


class frg_set(ctypes.Structure):
    _fields_ = [("quad", frg_quad), ("n_ext", ctypes.c_int64), ("p", ctypes.c_void_p),
                ("m2", ctypes.c_void_p), ("out", ctypes.c_void_p), ("err_est", ctypes.c_void_p),
                ("used_fp64", ctypes.c_void_p)]


class frg_gtab(ctypes.Structure):
    _fields_ = [("n_rows", ctypes.c_int64), ("n_s", ctypes.c_int64), ("s_max", ctypes.c_double),
                ("g", ctypes.c_void_p)]


class frg_fvlpa(ctypes.Structure):
    _fields_ = [("d", ctypes.c_int32), ("N", ctypes.c_int32), ("reg", ctypes.c_int32),
                ("n_radial", ctypes.c_int32), ("lambda_", ctypes.c_double),
                ("q_max_over_k", ctypes.c_double), ("n_cells", ctypes.c_int64),
                ("sigma_max", ctypes.c_double)]


class frg_pflow(ctypes.Structure):
    _fields_ = [("d", ctypes.c_int32), ("reg", ctypes.c_int32), ("n_radial", ctypes.c_int32),
                ("n_angular", ctypes.c_int32), ("lambda_", ctypes.c_double),
                ("q_max_over_k", ctypes.c_double), ("n_s", ctypes.c_int64),
                ("s_max", ctypes.c_double)]


class frg_lpa(ctypes.Structure):
    _fields_ = [("d", ctypes.c_int32), ("N", ctypes.c_int32), ("reg", ctypes.c_int32),
                ("n_radial", ctypes.c_int32), ("q_max_over_k", ctypes.c_double),
                ("Lambda", ctypes.c_double), ("n_grid", ctypes.c_int64),
                ("rho_max", ctypes.c_double)]


class frg_request(ctypes.Structure):
    _fields_ = [("lpa", frg_lpa), ("lambda_", ctypes.c_double), ("rho0", ctypes.c_double),
                ("t_end", ctypes.c_double), ("rtol", ctypes.c_double), ("atol", ctypes.c_double),
                ("U_out", ctypes.c_void_p)]


class frg_result(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("steps", ctypes.c_int64), ("rejected", ctypes.c_int64),
                ("rhs_calls", ctypes.c_int64), ("submit_s", ctypes.c_double),
                ("start_s", ctypes.c_double), ("done_s", ctypes.c_double),
                ("t_reached", ctypes.c_double)]


RHS_FN = ctypes.CFUNCTYPE(ctypes.c_int, ctypes.c_void_p, ctypes.c_double,
                          ctypes.POINTER(ctypes.c_double), ctypes.c_int64,
                          ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double))


class FrgError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{STATUS_NAMES.get(code, code)}: {msg}")
        self.code = code


def _load():
    # PyTorch ships its own HIP runtime under the same soname
    # (libamdhip64.so.7).  Loading torch first makes the dynamic loader bind
    # libfrg to that already-loaded runtime, so a process holds one HIP
    # runtime and device pointers and streams are shared with torch.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is not built; run `python -m paper_2607_24908_amd.build` "
                           "(there is no non-HIP fallback)")
    L = ctypes.CDLL(LIB_PATH)
    vp, i32, i64, dbl = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    L.frg_create.argtypes = [ctypes.POINTER(vp), ctypes.c_int, ctypes.c_uint64]
    L.frg_destroy.argtypes = [vp]
    L.frg_destroy.restype = None
    L.frg_last_error.restype = ctypes.c_char_p
    L.frg_version.restype = ctypes.c_char_p
    L.frg_integrate.argtypes = [vp, ctypes.POINTER(frg_set), i32, i32, i32, vp]
    L.frg_integrate_grid.argtypes = [vp, ctypes.POINTER(frg_quad), i64, vp, i64, vp, vp, vp, vp,
                                     i32, vp]
    L.frg_integrate_tab.argtypes = [vp, ctypes.POINTER(frg_quad), ctypes.POINTER(frg_gtab), i64,
                                    vp, vp, i32, vp]
    L.frg_integrate_vertex.argtypes = [vp, ctypes.POINTER(frg_quad), i32, i64, vp, vp, vp, i64,
                                       vp, vp, i32, vp]
    L.frg_fvlpa_rhs.argtypes = [vp, ctypes.POINTER(frg_fvlpa), i64, dbl, vp, vp, vp, i32, vp]
    L.frg_fvlpa_solve.argtypes = [vp, ctypes.POINTER(frg_fvlpa), i64, dbl, i64, vp, vp, i32, vp]
    L.frg_pflow_rhs.argtypes = [vp, ctypes.POINTER(frg_pflow), i64, vp, vp, dbl, vp, vp, i32, vp]
    L.frg_pflow_solve.argtypes = [vp, ctypes.POINTER(frg_pflow), i64, vp, vp, dbl, i64, vp, vp,
                                  i32, vp]
    L.frg_flow_rhs.argtypes = [vp, ctypes.POINTER(frg_lpa), dbl, vp, vp, vp, i32, vp]
    L.frg_flow_rhs_batch.argtypes = [vp, i32, ctypes.POINTER(frg_lpa), ctypes.POINTER(dbl),
                                     ctypes.POINTER(vp), ctypes.POINTER(vp), ctypes.POINTER(vp), vp]
    L.frg_flow_solve.argtypes = [ctypes.POINTER(frg_request), RHS_FN, vp, ctypes.POINTER(frg_result)]
    L.frg_submit.argtypes = [vp, ctypes.POINTER(frg_request), ctypes.POINTER(ctypes.c_uint64)]
    L.frg_poll.argtypes = [vp, ctypes.c_uint64, ctypes.POINTER(frg_result)]
    L.frg_server_stats.argtypes = [vp, ctypes.POINTER(i64), ctypes.POINTER(i64),
                                   ctypes.POINTER(dbl)]
    L.frg_gauss_legendre.argtypes = [i32, vp, vp]
    L.frg_expneg.argtypes = [i64, vp, vp]
    L.frg_expneg_fp32c.argtypes = [vp, i64, vp, vp, vp]
    L.frg_stream_status.argtypes = [vp, vp]
    L.frg_integrate_noalloc.argtypes = [vp, ctypes.POINTER(frg_set), i32, vp, vp]
    L.frg_flow_footprint.argtypes = [ctypes.POINTER(frg_lpa)]
    L.frg_flow_footprint.restype = i64
    L.frg_autotune.argtypes = [vp, i32, ctypes.c_char_p]
    L.frg_tune_set.argtypes = [vp, ctypes.c_char_p, i32]
    L.frg_tune_get.argtypes = [vp, ctypes.c_char_p, ctypes.POINTER(i32)]
    return L


lib = _load()


def last_error() -> str:
    return lib.frg_last_error().decode()


def _check(rc, allow=()):
    if rc != FRG_OK and rc not in allow:
        raise FrgError(rc, last_error())
    return rc


def _addr(x):
    """Address of a torch tensor, numpy array or integer (None -> NULL)."""
    if x is None:
        return None
    if isinstance(x, int):
        return x
    if isinstance(x, np.ndarray):
        if not x.flags["C_CONTIGUOUS"]:
            raise ValueError("numpy array must be C-contiguous")
        return x.ctypes.data
    if hasattr(x, "data_ptr"):
        if not x.is_contiguous():
            raise ValueError("tensor must be contiguous")
        return x.data_ptr()
    raise TypeError(f"cannot take the address of {type(x)}")


def _stream(s):
    if s is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    if isinstance(s, int):
        return s
    return s.cuda_stream


def make_quad(d, reg, k, q_max, n_radial, n_angular, prec=FRG_PREC_FP64) -> frg_quad:
    return frg_quad(d, reg, float(k), float(q_max), n_radial, n_angular, prec, 0)


# ------------------------------------------------------------ C names --
def frg_version() -> str:
    return lib.frg_version().decode()


def frg_create(device: int = 0, hbm_budget_bytes: int = 0) -> int:
    h = ctypes.c_void_p()
    _check(lib.frg_create(ctypes.byref(h), device, hbm_budget_bytes))
    return h.value


def frg_destroy(ctx: int) -> None:
    lib.frg_destroy(ctx)


def make_set_array(sets):
    """The frg_set array of a list of dicts {quad, p, m2, out, [err_est],
    [used_fp64]} (tensors/arrays; the caller keeps them alive)."""
    arr = (frg_set * max(1, len(sets)))()
    for i, s in enumerate(sets):
        n = int(s["p"].numel() if hasattr(s["p"], "numel") else s["p"].size)
        arr[i] = frg_set(s["quad"], n, _addr(s["p"]), _addr(s["m2"]), _addr(s["out"]),
                         _addr(s.get("err_est")), _addr(s.get("used_fp64")))
    return arr


def frg_integrate(ctx, sets, mem=FRG_MEM_DEVICE, flags=FRG_PLAIN, stream=None, allow_domain=False):
    """sets: list of dicts {quad, p, m2, out, [err_est], [used_fp64]} with tensors/arrays."""
    arr = make_set_array(sets)
    st = 0 if mem == FRG_MEM_HOST else _stream(stream)
    return _check(lib.frg_integrate(ctx, arr, len(sets), mem, flags, st),
                  (FRG_E_DOMAIN,) if allow_domain else ())


def frg_integrate_noalloc(ctx, sets, domain_flag=None, stream=None):
    """Allocation-free persistent launch over device-memory sets (the dicts of
    frg_integrate); domain_flag: optional device int32 tensor set to 1 on a
    domain violation."""
    arr = make_set_array(sets)
    return _check(lib.frg_integrate_noalloc(ctx, arr, len(sets), _addr(domain_flag),
                                            _stream(stream)))


def frg_integrate_array(ctx, arr, n_sets, mem=FRG_MEM_DEVICE, flags=FRG_PLAIN, stream=None,
                        allow_domain=False):
    """frg_integrate on a set array from make_set_array (no per-call marshalling)."""
    st = 0 if mem == FRG_MEM_HOST else _stream(stream)
    return _check(lib.frg_integrate(ctx, arr, n_sets, mem, flags, st),
                  (FRG_E_DOMAIN,) if allow_domain else ())


def frg_stream_status(ctx, stream=None, allow_domain=False):
    """Wait for the stream; FRG_E_DOMAIN if a device call on it met a point
    outside the domain since the last query (raises unless allow_domain)."""
    return _check(lib.frg_stream_status(ctx, _stream(stream)),
                  (FRG_E_DOMAIN,) if allow_domain else ())


def frg_integrate_grid(ctx, quad, p, m2, out, err_est=None, used_fp64=None, mem=FRG_MEM_DEVICE,
                       stream=None, allow_domain=False):
    n_p = int(p.numel() if hasattr(p, "numel") else p.size)
    n_m = int(m2.numel() if hasattr(m2, "numel") else m2.size)
    st = 0 if mem == FRG_MEM_HOST else _stream(stream)
    return _check(lib.frg_integrate_grid(ctx, ctypes.byref(quad), n_p, _addr(p), n_m, _addr(m2),
                                         _addr(out), _addr(err_est), _addr(used_fp64), mem, st),
                  (FRG_E_DOMAIN,) if allow_domain else ())


def frg_integrate_tab(ctx, quad, g, s_max, p, out, mem=FRG_MEM_DEVICE, stream=None,
                      allow_domain=False):
    """g: (n_rows, n_s) float64 table (torch tensor or numpy array, contiguous),
    out: n_p * n_rows results, out[a * n_rows + r]."""
    shape = tuple(g.shape)
    if len(shape) != 2:
        raise ValueError("g must be (n_rows, n_s)")
    tab = frg_gtab(shape[0], shape[1], float(s_max), _addr(g))
    n_p = int(p.numel() if hasattr(p, "numel") else p.size)
    st = 0 if mem == FRG_MEM_HOST else _stream(stream)
    return _check(lib.frg_integrate_tab(ctx, ctypes.byref(quad), ctypes.byref(tab), n_p, _addr(p),
                                        _addr(out), mem, st),
                  (FRG_E_DOMAIN,) if allow_domain else ())


def frg_integrate_vertex(ctx, quad, n_azimuth, p1, p2, cos12, m2, out, mem=FRG_MEM_DEVICE,
                         stream=None, allow_domain=False):
    """out[c * n_m + b] = V(p1[c], p2[c], acos(cos12[c]), m2[b])."""
    n_c = int(p1.numel() if hasattr(p1, "numel") else p1.size)
    n_m = int(m2.numel() if hasattr(m2, "numel") else m2.size)
    st = 0 if mem == FRG_MEM_HOST else _stream(stream)
    return _check(lib.frg_integrate_vertex(ctx, ctypes.byref(quad), int(n_azimuth), n_c,
                                           _addr(p1), _addr(p2), _addr(cos12), n_m, _addr(m2),
                                           _addr(out), mem, st),
                  (FRG_E_DOMAIN,) if allow_domain else ())


def make_fvlpa(d, N, reg, n_radial, lam, q_max_over_k, n_cells, sigma_max):
    return frg_fvlpa(int(d), int(N), int(reg), int(n_radial), float(lam), float(q_max_over_k),
                     int(n_cells), float(sigma_max))


def frg_fvlpa_rhs(ctx, fv, t, u, dudt, dt_est=None, mem=FRG_MEM_DEVICE, stream=None,
                  allow_domain=False):
    """u, dudt: n_flows * n_cells values (row r = flow r); dt_est: n_flows or None."""
    n = int((u.numel() if hasattr(u, "numel") else u.size) // fv.n_cells)
    st = 0 if mem == FRG_MEM_HOST else _stream(stream)
    return _check(lib.frg_fvlpa_rhs(ctx, ctypes.byref(fv), n, float(t), _addr(u), _addr(dudt),
                                    _addr(dt_est), mem, st),
                  (FRG_E_DOMAIN,) if allow_domain else ())


def frg_fvlpa_solve(ctx, fv, t_end, n_steps, u, t_reached, mem=FRG_MEM_DEVICE, stream=None):
    n = int((u.numel() if hasattr(u, "numel") else u.size) // fv.n_cells)
    st = 0 if mem == FRG_MEM_HOST else _stream(stream)
    return _check(lib.frg_fvlpa_solve(ctx, ctypes.byref(fv), n, float(t_end), int(n_steps),
                                      _addr(u), _addr(t_reached), mem, st))


def make_pflow(d, reg, n_radial, n_angular, lam, q_max_over_k, n_s, s_max):
    return frg_pflow(int(d), int(reg), int(n_radial), int(n_angular), float(lam),
                     float(q_max_over_k), int(n_s), float(s_max))


def frg_pflow_rhs(ctx, pf, lam3, lam4, t, sigma, dsdt, mem=FRG_MEM_DEVICE, stream=None,
                  allow_domain=False):
    """sigma, dsdt: n_flows * n_s values, row r = flow r; lam3, lam4: n_flows."""
    n = int(lam3.numel() if hasattr(lam3, "numel") else np.asarray(lam3).size)
    st = 0 if mem == FRG_MEM_HOST else _stream(stream)
    return _check(lib.frg_pflow_rhs(ctx, ctypes.byref(pf), n, _addr(lam3), _addr(lam4), float(t),
                                    _addr(sigma), _addr(dsdt), mem, st),
                  (FRG_E_DOMAIN,) if allow_domain else ())


def frg_pflow_solve(ctx, pf, lam3, lam4, t_end, n_steps, sigma, t_reached, mem=FRG_MEM_DEVICE,
                    stream=None):
    """RK4 from t = 0 to t_end; sigma (n_flows * n_s) is updated in place,
    t_reached (n_flows) receives where each flow stopped."""
    n = int(lam3.numel() if hasattr(lam3, "numel") else np.asarray(lam3).size)
    st = 0 if mem == FRG_MEM_HOST else _stream(stream)
    return _check(lib.frg_pflow_solve(ctx, ctypes.byref(pf), n, _addr(lam3), _addr(lam4),
                                      float(t_end), int(n_steps), _addr(sigma), _addr(t_reached),
                                      mem, st))


def frg_flow_rhs(ctx, lpa, t, U, dUdt, jac_bands=None, mem=FRG_MEM_DEVICE, stream=None,
                 allow_domain=False):
    st = 0 if mem == FRG_MEM_HOST else _stream(stream)
    return _check(lib.frg_flow_rhs(ctx, ctypes.byref(lpa), float(t), _addr(U), _addr(dUdt),
                                   _addr(jac_bands), mem, st),
                  (FRG_E_DOMAIN,) if allow_domain else ())


def frg_flow_rhs_batch(ctx, lpas, ts, Us, dUdts, jacs=None, stream=None):
    n = len(lpas)
    la = (frg_lpa * n)(*lpas)
    ta = (ctypes.c_double * n)(*[float(t) for t in ts])
    ua = (ctypes.c_void_p * n)(*[_addr(u) for u in Us])
    da = (ctypes.c_void_p * n)(*[_addr(u) for u in dUdts])
    ja = (ctypes.c_void_p * n)(*[_addr(u) for u in jacs]) if jacs is not None else None
    return _check(lib.frg_flow_rhs_batch(ctx, n, la, ta, ua, da, ja, _stream(stream)))


def frg_flow_solve(request: frg_request, rhs_callable):
    """Run the host stepper with a Python right-hand side
    rhs_callable(t, U: ndarray) -> (dUdt, jac_bands or None, status)."""
    res = frg_result()

    def cb(user, t, U, n, dUdt, jac):
        u = np.ctypeslib.as_array(U, shape=(n,)).copy()
        f, J, rc = rhs_callable(t, u)
        np.ctypeslib.as_array(dUdt, shape=(n,))[:] = f
        if jac and J is not None:
            np.ctypeslib.as_array(jac, shape=(7 * n,))[:] = np.asarray(J).ravel()
        return int(rc)

    fn = RHS_FN(cb)
    rc = lib.frg_flow_solve(ctypes.byref(request), fn, None, ctypes.byref(res))
    return rc, res


def frg_submit(ctx, request: frg_request) -> int:
    t = ctypes.c_uint64()
    _check(lib.frg_submit(ctx, ctypes.byref(request), ctypes.byref(t)))
    return t.value


def frg_poll(ctx, ticket: int):
    res = frg_result()
    rc = lib.frg_poll(ctx, ticket, ctypes.byref(res))
    if rc not in (FRG_OK, FRG_PENDING):
        raise FrgError(rc, last_error())
    return rc, res


def frg_server_stats(ctx):
    a, b, c = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_double()
    _check(lib.frg_server_stats(ctx, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c)))
    return a.value, b.value, c.value


def frg_gauss_legendre(n: int):
    x = np.empty(n)
    w = np.empty(n)
    _check(lib.frg_gauss_legendre(n, _addr(x), _addr(w)))
    return x, w


def frg_expneg(y: np.ndarray) -> np.ndarray:
    y = np.ascontiguousarray(y, dtype=np.float64)
    out = np.empty_like(y)
    _check(lib.frg_expneg(y.size, _addr(y), _addr(out)))
    return out


def frg_expneg_fp32c(ctx, y, out, stream=None):
    """e^{-y} on the GPU by the FP32C point path's exponential (device tensors)."""
    return _check(lib.frg_expneg_fp32c(ctx, int(y.numel()), _addr(y), _addr(out), _stream(stream)))


def frg_flow_footprint(lpa: frg_lpa) -> int:
    return int(lib.frg_flow_footprint(ctypes.byref(lpa)))


def frg_autotune(ctx, mode: int, cache_path: str | None = None):
    return _check(lib.frg_autotune(ctx, mode, cache_path.encode() if cache_path else None))


def frg_tune_set(ctx, key: str, value: int):
    return _check(lib.frg_tune_set(ctx, key.encode(), int(value)))


def frg_tune_get(ctx, key: str) -> int:
    v = ctypes.c_int32()
    _check(lib.frg_tune_get(ctx, key.encode(), ctypes.byref(v)))
    return v.value


def make_lpa(d=3, N=1, reg=FRG_REG_EXP, n_radial=64, q_max_over_k=6.0, Lambda=1.0, n_grid=128,
             rho_max=0.5) -> frg_lpa:
    return frg_lpa(d, N, reg, n_radial, float(q_max_over_k), float(Lambda), int(n_grid),
                   float(rho_max))


def make_request(lpa: frg_lpa, lam, rho0, t_end, rtol, atol, U_out: np.ndarray) -> frg_request:
    return frg_request(lpa, float(lam), float(rho0), float(t_end), float(rtol), float(atol),
                       _addr(U_out))
