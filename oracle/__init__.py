"""FP64 CPU oracle for the FRG flow-diagram quadrature (test infrastructure).

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  It loads ``liboracle.so`` built from
``frg_oracle.c`` (plain C, no code shared with the HIP library) and exposes
numpy-facing wrappers.  Every function states the definition it follows; the
definitions themselves are written out in the header comment of
``frg_oracle.c``.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "frg_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

REG_EXP = 0
REG_LITIM = 1
OK, E_INVAL, E_DOMAIN = 0, -1, -2


def build(force: bool = True) -> str:
    """Compile ``liboracle.so`` with gcc, strict IEEE (no fast-math, no contraction)."""
    if force or not os.path.exists(_LIB):
        cmd = ["gcc", "-O2", "-fno-fast-math", "-ffp-contract=off", "-fopenmp", "-std=c11",
               "-D_GNU_SOURCE", "-shared", "-fPIC", "-o", _LIB + ".tmp", _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(_LIB + ".tmp", _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        L = ctypes.CDLL(_LIB)
        dp = ctypes.POINTER(ctypes.c_double)
        L.oracle_gauss_legendre.argtypes = [ctypes.c_int, dp, dp]
        L.oracle_Pd.argtypes = [ctypes.c_int]
        L.oracle_Pd.restype = ctypes.c_double
        L.oracle_Cd.argtypes = [ctypes.c_int]
        L.oracle_Cd.restype = ctypes.c_double
        L.oracle_integrate.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_double,
                                       ctypes.c_double, ctypes.c_int, ctypes.c_int,
                                       ctypes.c_long, dp, dp, dp, ctypes.c_int]
        L.oracle_threshold.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_double,
                                       ctypes.c_double, ctypes.c_int, ctypes.c_int,
                                       ctypes.c_long, dp, dp]
        L.oracle_integrate_tab.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_double,
                                           ctypes.c_double, ctypes.c_int, ctypes.c_int,
                                           ctypes.c_long, ctypes.c_long, ctypes.c_double, dp,
                                           ctypes.c_long, dp, dp, ctypes.c_int]
        L.oracle_integrate_tab_bound.argtypes = L.oracle_integrate_tab.argtypes
        L.oracle_lpa_rhs.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                     ctypes.c_double, ctypes.c_double, ctypes.c_long,
                                     ctypes.c_double, dp, dp, dp]
        L.oracle_integrate_vertex.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_double,
                                              ctypes.c_double, ctypes.c_int, ctypes.c_int,
                                              ctypes.c_int, ctypes.c_long, dp, dp, dp, dp, dp,
                                              ctypes.c_int]
        ip = ctypes.POINTER(ctypes.c_int)
        L.oracle_fvlpa_rhs.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                       ctypes.c_double, ctypes.c_double, ctypes.c_long,
                                       ctypes.c_long, ctypes.c_double, ctypes.c_double, dp, dp,
                                       dp, ip]
        L.oracle_fvlpa_solve.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                         ctypes.c_double, ctypes.c_double, ctypes.c_long,
                                         ctypes.c_long, ctypes.c_double, ctypes.c_double,
                                         ctypes.c_long, dp, dp]
        L.oracle_pflow_rhs.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_double,
                                       ctypes.c_double, ctypes.c_int, ctypes.c_int,
                                       ctypes.c_long, ctypes.c_long, ctypes.c_double, dp, dp,
                                       ctypes.c_double, dp, dp, ip, ctypes.c_int]
        L.oracle_pflow_solve.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_double,
                                         ctypes.c_double, ctypes.c_int, ctypes.c_int,
                                         ctypes.c_long, ctypes.c_long, ctypes.c_double, dp, dp,
                                         ctypes.c_double, ctypes.c_long, dp, dp, ctypes.c_int]
        _lib = L
    return _lib


def _ptr(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _f64(a):
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


def gauss_legendre(n: int):
    """Gauss-Legendre nodes (ascending) and weights on [-1, 1]."""
    x = np.empty(n)
    w = np.empty(n)
    rc = lib().oracle_gauss_legendre(n, _ptr(x), _ptr(w))
    if rc != OK:
        raise ValueError(f"oracle_gauss_legendre rc={rc}")
    return x, w


def Pd(d: int) -> float:
    """Angular-measure prefactor Omega_{d-1}/(2 pi)^d."""
    return lib().oracle_Pd(d)


def Cd(d: int) -> float:
    """Radial-only prefactor Omega_d/(2 pi)^d."""
    return lib().oracle_Cd(d)


def integrate(d, reg, k, q_max, n_r, n_a, p, m2, threads=1, allow_domain=False):
    """One-loop flow-diagram integral I(p, m^2) for each (p[e], m2[e]) pair.

    I = P_d sum_ij w_i q_i^{d-1} d_tR(q_i^2) G(q_i^2)^2 mu_j G(|q_i+p|^2), the
    radial x angular Gauss-Legendre discretisation of
    int d^dq/(2pi)^d d_tR G(q)^2 G(q+p).  Returns a float64 array (NaN where
    m^2 + k^2 <= 0)."""
    p = _f64(p).ravel()
    m2 = _f64(m2).ravel()
    if p.shape != m2.shape:
        raise ValueError("p and m2 must have the same length")
    out = np.empty_like(p)
    rc = lib().oracle_integrate(int(d), int(reg), float(k), float(q_max), int(n_r), int(n_a),
                                p.size, _ptr(p), _ptr(m2), _ptr(out), int(threads))
    if rc == E_INVAL or (rc == E_DOMAIN and not allow_domain):
        raise ValueError(f"oracle_integrate rc={rc}")
    return out


def integrate_grid(d, reg, k, q_max, n_r, n_a, p, m2, threads=1):
    """Tensor grid: out[a, b] = I(p[a], m2[b])."""
    p = _f64(p).ravel()
    m2 = _f64(m2).ravel()
    P = np.repeat(p, m2.size)
    M = np.tile(m2, p.size)
    return integrate(d, reg, k, q_max, n_r, n_a, P, M, threads).reshape(p.size, m2.size)


def integrate_tab(d, reg, k, q_max, n_r, n_a, G, s_max, p, threads=1, allow_domain=False):
    """Tabulated-propagator variant: out[a, r] = I(p[a], row r) with the
    propagator taken from row r of G (shape (n_rows, n_s)) by piecewise-linear
    interpolation on the uniform grid s_k = k s_max/(n_s - 1) (constant beyond
    s_max), in both G(q_i^2) and G(s_ij); d_tR stays analytic."""
    G = np.ascontiguousarray(np.asarray(G, dtype=np.float64))
    if G.ndim != 2:
        raise ValueError("G must be (n_rows, n_s)")
    p = _f64(p).ravel()
    out = np.empty((p.size, G.shape[0]))
    rc = lib().oracle_integrate_tab(int(d), int(reg), float(k), float(q_max), int(n_r), int(n_a),
                                    G.shape[0], G.shape[1], float(s_max), _ptr(G), p.size, _ptr(p),
                                    _ptr(out), int(threads))
    if rc == E_INVAL or (rc == E_DOMAIN and not allow_domain):
        raise ValueError(f"oracle_integrate_tab rc={rc}")
    return out


def integrate_tab_bound(d, reg, k, q_max, n_r, n_a, G, s_max, p, threads=1):
    """Relative deviation that the evaluation coordinate can cause in each
    result of integrate_tab between two implementations whose rules agree to
    about an ulp (see oracle_integrate_tab_bound): the tolerance of GPU
    comparisons on rough tables, not a pinned value."""
    G = np.ascontiguousarray(np.asarray(G, dtype=np.float64))
    p = _f64(p).ravel()
    out = np.empty((p.size, G.shape[0]))
    rc = lib().oracle_integrate_tab_bound(int(d), int(reg), float(k), float(q_max), int(n_r),
                                          int(n_a), G.shape[0], G.shape[1], float(s_max), _ptr(G),
                                          p.size, _ptr(p), _ptr(out), int(threads))
    if rc == E_INVAL:
        raise ValueError(f"oracle_integrate_tab_bound rc={rc}")
    return out


def threshold(d, reg, k, q_max, n_r, n, m2, allow_domain=False):
    """Threshold function F_n(m^2) = C_d sum_i w_i q_i^{d-1} d_tR(q_i^2) G(q_i^2)^n."""
    m2 = _f64(m2).ravel()
    out = np.empty_like(m2)
    rc = lib().oracle_threshold(int(d), int(reg), float(k), float(q_max), int(n_r), int(n),
                                m2.size, _ptr(m2), _ptr(out))
    if rc == E_INVAL or (rc == E_DOMAIN and not allow_domain):
        raise ValueError(f"oracle_threshold rc={rc}")
    return out


def lpa_rhs(d, N, reg, n_r, q_max_over_k, k, rho_max, U, jacobian=True, allow_domain=False):
    """LPA O(N) right-hand side d_tU = 1/2 [F_1(U'+2 rho U'') + (N-1) F_1(U')]
    on the uniform grid rho_j = j rho_max/(n-1), with its 7-band Jacobian
    jac[o+3, j] = d(d_tU_j)/dU_{j+o}.  Returns (dUdt, jac or None, rc)."""
    U = _f64(U).ravel()
    n = U.size
    dUdt = np.empty(n)
    jac = np.zeros((7, n)) if jacobian else None
    rc = lib().oracle_lpa_rhs(int(d), int(N), int(reg), int(n_r), float(q_max_over_k),
                              float(k), n, float(rho_max), _ptr(U), _ptr(dUdt),
                              _ptr(jac) if jacobian else None)
    if rc == E_INVAL or (rc == E_DOMAIN and not allow_domain):
        raise ValueError(f"oracle_lpa_rhs rc={rc}")
    return dUdt, jac, rc


def integrate_vertex(d, reg, k, q_max, n_r, n_a, n_phi, p1, p2, c12, m2, threads=1,
                     allow_domain=False):
    """Vertex diagram V(p1, p2, th, m^2) = int d^dq/(2pi)^d d_tR G(q^2)^2
    G(|q+p1|^2) G(|q+p2|^2) for independent points (p1[e], p2[e], c12[e] =
    cos th, m2[e]): radial and polar rules as for I, Gauss-Legendre in the
    azimuth phi on [0, pi] with weight sin^{d-3} phi, prefactor
    Omega_{d-2}/(2pi)^d."""
    p1 = _f64(p1).ravel()
    p2 = _f64(p2).ravel()
    c12 = _f64(c12).ravel()
    m2 = _f64(m2).ravel()
    out = np.empty_like(p1)
    rc = lib().oracle_integrate_vertex(int(d), int(reg), float(k), float(q_max), int(n_r),
                                       int(n_a), int(n_phi), p1.size, _ptr(p1), _ptr(p2),
                                       _ptr(c12), _ptr(m2), _ptr(out), int(threads))
    if rc == E_INVAL or (rc == E_DOMAIN and not allow_domain):
        raise ValueError(f"oracle_integrate_vertex rc={rc}")
    return out


def pflow_rhs(d, reg, Lam, kappa, n_r, n_a, s_max, lam3, lam4, t, Sigma, threads=1,
              allow_domain=False):
    """Right-hand side of the momentum-dependent two-point flow (constant
    vertices): dSigma_r(p_a)/dt = lam3_r^2 J_r(p_a) - lam4_r/2 T_r with the
    propagator table g_r[a] = 1/(s_a + R_k(s_a) + Sigma_r[a]) on the nodes
    s_a = a s_max/(n_s - 1), p_a = sqrt(s_a), k = Lam e^t, q_max = kappa k;
    J is the tabulated diagram, T = C_d sum_i w_i q_i^{d-1} d_tR G(q_i^2)^2.
    Sigma has shape (n_flows, n_s).  Returns (dSdt, dead)."""
    S = np.ascontiguousarray(np.asarray(Sigma, dtype=np.float64))
    if S.ndim != 2:
        raise ValueError("Sigma must be (n_flows, n_s)")
    l3 = _f64(lam3).ravel()
    l4 = _f64(lam4).ravel()
    out = np.empty_like(S)
    dead = np.zeros(S.shape[0], dtype=np.int32)
    rc = lib().oracle_pflow_rhs(int(d), int(reg), float(Lam), float(kappa), int(n_r), int(n_a),
                                S.shape[0], S.shape[1], float(s_max), _ptr(l3), _ptr(l4),
                                float(t), _ptr(S), _ptr(out),
                                dead.ctypes.data_as(ctypes.POINTER(ctypes.c_int)), int(threads))
    if rc == E_INVAL or (rc == E_DOMAIN and not allow_domain):
        raise ValueError(f"oracle_pflow_rhs rc={rc}")
    return out, dead


def pflow_solve(d, reg, Lam, kappa, n_r, n_a, s_max, lam3, lam4, t_end, n_steps, Sigma0,
                threads=1):
    """The two-point flow integrated by classical RK4 from t = 0 to t_end in
    n_steps equal steps (see pflow_rhs).  Returns (Sigma(t_end), t_reached);
    a flow that meets the domain boundary keeps the state at the start of
    that step and reports that time."""
    S = np.array(Sigma0, dtype=np.float64, copy=True, order="C")
    l3 = _f64(lam3).ravel()
    l4 = _f64(lam4).ravel()
    t_reached = np.empty(S.shape[0])
    rc = lib().oracle_pflow_solve(int(d), int(reg), float(Lam), float(kappa), int(n_r), int(n_a),
                                  S.shape[0], S.shape[1], float(s_max), _ptr(l3), _ptr(l4),
                                  float(t_end), int(n_steps), _ptr(S), _ptr(t_reached),
                                  int(threads))
    if rc == E_INVAL:
        raise ValueError("oracle_pflow_solve: invalid arguments")
    return S, t_reached


def fvlpa_rhs(d, N, reg, n_r, Lam, kappa, sigma_max, t, u, allow_domain=False):
    """Finite-volume LPA right-hand side d_t u_i = (Q_{i+1} - Q_i)/ds for
    u = dU/dsigma cell averages of shape (n_flows, n) (flux definitions in
    frg_oracle.c).  Returns (dudt, dt_estimate, dead)."""
    U = np.ascontiguousarray(np.asarray(u, dtype=np.float64))
    if U.ndim != 2:
        raise ValueError("u must be (n_flows, n)")
    out = np.empty_like(U)
    dt = np.empty(U.shape[0])
    dead = np.zeros(U.shape[0], dtype=np.int32)
    rc = lib().oracle_fvlpa_rhs(int(d), int(N), int(reg), int(n_r), float(Lam), float(kappa),
                                U.shape[0], U.shape[1], float(sigma_max), float(t), _ptr(U),
                                _ptr(out), _ptr(dt),
                                dead.ctypes.data_as(ctypes.POINTER(ctypes.c_int)))
    if rc == E_INVAL or (rc == E_DOMAIN and not allow_domain):
        raise ValueError(f"oracle_fvlpa_rhs rc={rc}")
    return out, dt, dead


def fvlpa_solve(d, N, reg, n_r, Lam, kappa, sigma_max, t_end, n_steps, u0):
    """Three-stage SSP Runge-Kutta integration of the finite-volume LPA from
    t = 0 to t_end; returns (u(t_end), t_reached)."""
    U = np.array(u0, dtype=np.float64, copy=True, order="C")
    tr = np.empty(U.shape[0])
    rc = lib().oracle_fvlpa_solve(int(d), int(N), int(reg), int(n_r), float(Lam), float(kappa),
                                  U.shape[0], U.shape[1], float(sigma_max), float(t_end),
                                  int(n_steps), _ptr(U), _ptr(tr))
    if rc == E_INVAL:
        raise ValueError("oracle_fvlpa_solve: invalid arguments")
    return U, tr


def Omega(n: int) -> float:
    """Area of the unit sphere S^{n-1} in R^n (plain Python, for the pins)."""
    return 2.0 * math.pi ** (n / 2) / math.gamma(n / 2)
