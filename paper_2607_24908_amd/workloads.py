"""Seeded synthetic inputs for the FRG quadrature workloads.

This module holds no arithmetic of the method: it only draws or lays out
external points, quadrature orders and flow requests.  Both the HIP path and
the CPU oracle are fed from here, so that their inputs are identical.

Workloads (k = 1 throughout; radial domain [0, 6k] for the exponential
regulator):

* ``plain_d4``  -- d = 4, exponential regulator, 64 momenta p log-spaced in
  [1e-3, 10] x 32 masses m^2 uniform in [-0.5, 5], 64 radial x 16 angular
  Gauss-Legendre nodes: 2048 integrals.
* ``scaleup_d3`` -- d = 3, exponential regulator, 4096 momenta log-spaced in
  [1e-4, 20] x 512 masses uniform in [-0.9, 10], 128 radial x 32 angular
  nodes: 2 097 152 integrals, 8.59e9 integrand evaluations.
* ``uneven_sets`` -- 256 independent integral sets: points per set uniform in
  [16, 1024], radial order in {32, 64, 128, 256}, angular order in {8, 16, 32},
  d in {3, 4}, regulator in {exponential, Litim}; per point p log-uniform in
  [1e-3, 10] and m^2 uniform in [-0.5, 5].
* ``precision_d4`` -- the plain_d4 shape with half of the masses close to the
  pole, m^2 = -k^2 + 10^U(-8,-1), and half uniform in [-0.9, 10].
* ``tabulated_d3`` -- the tabulated-propagator variant: d = 3, exponential
  regulator insertion, 1024 momenta log-spaced in [1e-4, 20], 64 table rows
  (field values) of n_s nodes on s in [0, 676] = [0, (q_max + p_max)^2],
  128 radial x 32 angular nodes.  Row r holds the smooth positive function
  g_r(s) = (1 + 0.1/(1 + s))/(s + M_r), M_r evenly spaced in [0.1, 11] (an input
  standing in for a dressed propagator; nothing of the method is computed).
  n_s = 4096 (rows staged in LDS) and 2^20 (8 MB rows read through the caches).
* ``vertex_d3`` -- two-external-momentum diagram: d = 3, exponential regulator,
  k = 1, q_max = 6, 48 radial x 8 polar x 16 azimuthal nodes; 256 momentum
  configurations (128 at the symmetric point p1 = p2 log-spaced in [1e-3, 10]
  with cos th = -1/2, 128 with p1, p2 log-uniform in [1e-3, 10] and cos th
  uniform in [-1, 1]) x 512 masses uniform in [-0.9, 10].
* ``fvlpa_d3`` -- finite-volume LPA, O(4), d = 3, exponential regulator, 64
  radial nodes, 128 flows of 256 cells on sigma in [0, 2] starting from the
  cell averages of U = lam/8 sigma^4 + m^2/2 sigma^2 with lam uniform in
  [1, 20], m^2 uniform in [0.05, 0.5]; RG time 0 -> -0.5 in 2000 SSP-RK3 steps
  (inside the explicit step bound at t = 0).
* ``pflow_d3`` -- momentum-dependent two-point flows: d = 3, exponential
  regulator, Lambda = 1, q_max = 6k, 128 radial x 32 angular nodes, Sigma on
  256 nodes of s in [0, 49] (p up to 7 Lambda), 64 flows with lam3 uniform in
  [0.5, 2.5], lam4 uniform in [0, 8], Sigma(t = 0) = m^2 uniform in [0.2, 1]
  (Gamma2 = p^2 + m^2), RG time 0 -> -4 in 100 RK4 steps.
* ``lpa_requests`` -- a Poisson stream (rate 50/s) of LPA O(N) flow requests:
  N in {1, 2, 4}, d = 3, exponential regulator, grid of 128..1024 points on
  rho in [0, 0.5], initial U = lambda/8 (rho - rho0)^2 with lambda ~ U(1, 20),
  rho0 ~ U(0, 0.2), RG time 0 -> -9, 64 radial nodes; stepper tolerances
  rtol 1e-8, atol 1e-10.

All random draws use numpy's PCG64 with an explicit seed.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

REG_EXP = 0
REG_LITIM = 1


@dataclass
class Quad:
    d: int
    reg: int
    k: float
    q_max: float
    n_r: int
    n_a: int


@dataclass
class GridWorkload:
    """Tensor grid of external points: out[a, b] = I(p[a], m2[b])."""
    name: str
    quad: Quad
    p: np.ndarray
    m2: np.ndarray

    @property
    def n_integrals(self) -> int:
        return self.p.size * self.m2.size

    @property
    def n_evals(self) -> int:
        return self.n_integrals * self.quad.n_r * self.quad.n_a


@dataclass
class PointSet:
    """An integral set of independent (p, m^2) points sharing one quadrature."""
    quad: Quad
    p: np.ndarray
    m2: np.ndarray

    @property
    def n_evals(self) -> int:
        return self.p.size * self.quad.n_r * self.quad.n_a


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def plain_d4() -> GridWorkload:
    q = Quad(d=4, reg=REG_EXP, k=1.0, q_max=6.0, n_r=64, n_a=16)
    return GridWorkload("plain_d4_exp_64x32_64r16a", q,
                        np.logspace(-3.0, 1.0, 64), np.linspace(-0.5, 5.0, 32))


def scaleup_d3(n_p: int = 4096, n_m: int = 512) -> GridWorkload:
    q = Quad(d=3, reg=REG_EXP, k=1.0, q_max=6.0, n_r=128, n_a=32)
    return GridWorkload(f"scaleup_d3_exp_{n_p}x{n_m}_128r32a", q,
                        np.logspace(-4.0, np.log10(20.0), n_p), np.linspace(-0.9, 10.0, n_m))


def scaleup_d3_litim_p0(n_m: int = 512) -> GridWorkload:
    """Litim regulator at p = 0 over the scale-up masses (closed-form check)."""
    q = Quad(d=3, reg=REG_LITIM, k=1.0, q_max=6.0, n_r=128, n_a=32)
    return GridWorkload(f"scaleup_d3_litim_p0_{n_m}", q, np.zeros(1),
                        np.linspace(-0.9, 10.0, n_m))


def uneven_sets(seed: int = 0, n_sets: int = 256, max_points: int = 1024) -> list[PointSet]:
    rng = _rng(seed)
    sets = []
    for _ in range(n_sets):
        n_ext = int(rng.integers(16, max_points + 1))
        n_r = int(rng.choice([32, 64, 128, 256]))
        n_a = int(rng.choice([8, 16, 32]))
        d = int(rng.choice([3, 4]))
        reg = int(rng.choice([REG_EXP, REG_LITIM]))
        p = 10.0 ** rng.uniform(-3.0, 1.0, n_ext)
        m2 = rng.uniform(-0.5, 5.0, n_ext)
        sets.append(PointSet(Quad(d, reg, 1.0, 6.0, n_r, n_a), p, m2))
    return sets


def precision_d4(seed: int = 0) -> GridWorkload:
    rng = _rng(seed)
    near = -1.0 + 10.0 ** rng.uniform(-8.0, -1.0, 16)
    far = rng.uniform(-0.9, 10.0, 16)
    q = Quad(d=4, reg=REG_EXP, k=1.0, q_max=6.0, n_r=64, n_a=16)
    return GridWorkload(f"precision_d4_seed{seed}", q, np.logspace(-3.0, 1.0, 64),
                        np.concatenate([np.sort(near), np.sort(far)]))


@dataclass
class TabWorkload:
    name: str
    quad: Quad
    p: np.ndarray
    g: np.ndarray      # (n_rows, n_s)
    s_max: float

    @property
    def n_integrals(self) -> int:
        return self.p.size * self.g.shape[0]

    @property
    def n_evals(self) -> int:
        return self.n_integrals * self.quad.n_r * self.quad.n_a


def tab_rows(n_rows: int, n_s: int, s_max: float, m_lo: float = 0.1, m_hi: float = 11.0) -> np.ndarray:
    """Rows g_r(s_k) = (1 + 0.1/(1 + s_k))/(s_k + M_r) on s_k = k s_max/(n_s - 1)."""
    s = np.linspace(0.0, s_max, n_s)
    M = np.linspace(m_lo, m_hi, n_rows)
    return (1.0 + 0.1 / (1.0 + s))[None, :] / (s[None, :] + M[:, None])


def tabulated_d3(n_s: int = 4096, n_p: int = 1024, n_rows: int = 64) -> TabWorkload:
    q = Quad(d=3, reg=REG_EXP, k=1.0, q_max=6.0, n_r=128, n_a=32)
    p = np.logspace(-4.0, np.log10(20.0), n_p)
    s_max = (q.q_max + 20.0) ** 2
    return TabWorkload(f"tabulated_d3_{n_p}p_{n_rows}rows_{n_s}s_128r32a", q, p,
                       tab_rows(n_rows, n_s, s_max), s_max)


@dataclass
class VertexWorkload:
    name: str
    quad: Quad
    n_phi: int
    p1: np.ndarray
    p2: np.ndarray
    c12: np.ndarray
    m2: np.ndarray

    @property
    def n_integrals(self) -> int:
        return self.p1.size * self.m2.size

    @property
    def n_evals(self) -> int:
        return self.n_integrals * self.quad.n_r * self.quad.n_a * self.n_phi


def vertex_d3(seed: int = 0, n_sym: int = 128, n_rand: int = 128, n_m: int = 512) -> VertexWorkload:
    rng = _rng(seed)
    p_sym = np.logspace(-3.0, 1.0, n_sym)
    p1 = np.concatenate([p_sym, 10.0 ** rng.uniform(-3.0, 1.0, n_rand)])
    p2 = np.concatenate([p_sym, 10.0 ** rng.uniform(-3.0, 1.0, n_rand)])
    c12 = np.concatenate([np.full(n_sym, -0.5), rng.uniform(-1.0, 1.0, n_rand)])
    q = Quad(d=3, reg=REG_EXP, k=1.0, q_max=6.0, n_r=48, n_a=8)
    return VertexWorkload(f"vertex_d3_exp_{p1.size}c_{n_m}m_48r8x16phi", q, 16, p1, p2, c12,
                          np.linspace(-0.9, 10.0, n_m))


@dataclass
class FvlpaWorkload:
    name: str
    d: int
    N: int
    reg: int
    n_r: int
    lam: float
    kappa: float
    n_cells: int
    sigma_max: float
    u0: np.ndarray      # (n_flows, n_cells) cell averages of dU/dsigma
    t_end: float
    n_steps: int

    @property
    def n_flows(self) -> int:
        return self.u0.shape[0]


def quartic_cell_averages(coef4: np.ndarray, coef2: np.ndarray, n_cells: int,
                          sigma_max: float) -> np.ndarray:
    """Exact cell averages of u = dU/dsigma for U = coef4/8 sigma^4 + coef2/2 sigma^2
    (one row per (coef4, coef2)): (U(right face) - U(left face))/ds."""
    ds = sigma_max / n_cells
    f = np.arange(n_cells + 1) * ds
    U = coef4[:, None] / 8.0 * f[None, :] ** 4 + coef2[:, None] / 2.0 * f[None, :] ** 2
    return (U[:, 1:] - U[:, :-1]) / ds


def fvlpa_d3(seed: int = 0, n_flows: int = 128, n_cells: int = 256, n_steps: int = 2000,
             t_end: float = -0.5) -> FvlpaWorkload:
    rng = _rng(seed)
    lam = rng.uniform(1.0, 20.0, n_flows)
    m2 = rng.uniform(0.05, 0.5, n_flows)
    u0 = quartic_cell_averages(lam, m2, n_cells, 2.0)
    return FvlpaWorkload(f"fvlpa_d3_O4_exp_{n_flows}flows_{n_cells}cells_{n_steps}steps", 3, 4,
                         REG_EXP, 64, 1.0, 6.0, n_cells, 2.0, u0, t_end, n_steps)


@dataclass
class PflowWorkload:
    name: str
    d: int
    reg: int
    n_r: int
    n_a: int
    lam: float          # UV scale
    kappa: float        # q_max / k
    n_s: int
    s_max: float
    lam3: np.ndarray    # (n_flows,)
    lam4: np.ndarray    # (n_flows,)
    sigma0: np.ndarray  # (n_flows, n_s)
    t_end: float
    n_steps: int

    @property
    def n_flows(self) -> int:
        return self.lam3.size

    @property
    def evals_per_rhs(self) -> int:
        return self.n_flows * self.n_s * self.n_r * self.n_a

    @property
    def n_evals(self) -> int:
        return 4 * self.n_steps * self.evals_per_rhs


def pflow_d3(seed: int = 0, n_flows: int = 64, n_s: int = 256, n_steps: int = 100,
             n_r: int = 128, n_a: int = 32) -> PflowWorkload:
    rng = _rng(seed)
    lam3 = rng.uniform(0.5, 2.5, n_flows)
    lam4 = rng.uniform(0.0, 8.0, n_flows)
    m2 = rng.uniform(0.2, 1.0, n_flows)
    sigma0 = np.repeat(m2[:, None], n_s, axis=1)
    return PflowWorkload(f"pflow_d3_exp_{n_flows}flows_{n_s}s_{n_r}r{n_a}a_{n_steps}steps", 3,
                         REG_EXP, n_r, n_a, 1.0, 6.0, n_s, 49.0, lam3, lam4, sigma0, -4.0, n_steps)


@dataclass
class FlowRequest:
    N: int
    d: int
    reg: int
    n_grid: int
    rho_max: float
    lam: float
    rho0: float
    t_end: float = -9.0
    n_r: int = 64
    q_max_over_k: float = 6.0
    Lambda: float = 1.0
    arrival_s: float = 0.0
    rtol: float = 1e-8
    atol: float = 1e-10

    def rho(self) -> np.ndarray:
        return np.linspace(0.0, self.rho_max, self.n_grid)

    def U0(self) -> np.ndarray:
        """Initial potential (lambda/8) (rho - rho0)^2 on the grid."""
        r = self.rho()
        return (self.lam / 8.0) * (r - self.rho0) ** 2


def lpa_requests(seed: int = 0, n: int = 100, rate: float = 50.0,
                 grid_lo: int = 128, grid_hi: int = 1024) -> list[FlowRequest]:
    rng = _rng(seed)
    gaps = rng.exponential(1.0 / rate, n)
    arrivals = np.cumsum(gaps) - gaps[0]
    reqs = []
    for i in range(n):
        reqs.append(FlowRequest(
            N=int(rng.choice([1, 2, 4])), d=3, reg=REG_EXP,
            n_grid=int(rng.integers(grid_lo, grid_hi + 1)), rho_max=0.5,
            lam=float(rng.uniform(1.0, 20.0)), rho0=float(rng.uniform(0.0, 0.2)),
            arrival_s=float(arrivals[i])))
    return reqs
