"""Pins of the FP64 oracle to facts fixed by mathematics, not by the oracle itself.

Each test names the identity it checks.  Together they are chosen so that a
plausible slip in the oracle -- a wrong measure prefactor, a wrong power of G,
a dropped factor in d_tR, a wrong |q+p|, a bad quadrature rule, a lost digit
near the pole -- fails at least one of them:

* Gauss-Legendre rules: numpy's leggauss (a library routine) and exactness on
  monomials up to degree 2n-1.
* Litim regulator at p = 0: closed form C_d 2 k^{d+2}/(d delta^3) (the
  discrete rule is exact there, every propagator equals 1/delta).
* Exponential regulator, large m^2: m^6 I -> P_d (sum mu) k^{d+2}
  Gamma(d/2+2) zeta(d/2+1), from int y^s e^y/(e^y-1)^2 dy = Gamma(s+1) zeta(s).
* Continuum integral by adaptive quadrature (scipy) in a different
  parametrisation (over s = |q+p|^2 instead of cos theta), with R and d_tR
  written from their definitions, against the converged discrete rule.
* The discrete rule evaluated in 40-digit arithmetic (mpmath) on tiny inputs.
* p -> 0 behaviour (quadratic in p), positivity and monotonicity in m^2.
* LPA: Litim threshold functions in closed form, exponential F_1(0) and its
  large-mass limit in terms of zeta, finite-difference exactness on
  quadratics, and the Jacobian against numerical differentiation.
"""
import math

import numpy as np
import pytest
from scipy import integrate, special

import oracle
from oracle import REG_EXP, REG_LITIM

PI = math.pi


def closed_Pd(d):
    return {3: 1.0 / (4 * PI ** 2), 4: 1.0 / (4 * PI ** 3)}[d]


def closed_Cd(d):
    return {3: 1.0 / (2 * PI ** 2), 4: 1.0 / (8 * PI ** 2), 5: 1.0 / (12 * PI ** 3)}[d]


def mu_sum(d, n_a):
    """sum_j v_j (1-x_j^2)^{(d-3)/2} with numpy's own Gauss-Legendre rule."""
    x, v = np.polynomial.legendre.leggauss(n_a)
    return float(np.sum(v * (1 - x * x) ** ((d - 3) / 2)))


# ---------------------------------------------------------------- rules --

@pytest.mark.parametrize("n", [1, 2, 3, 4, 5, 8, 16, 31, 32, 64, 128, 256])
def test_gauss_legendre_library_and_moments(n):
    x, w = oracle.gauss_legendre(n)
    xr, wr = np.polynomial.legendre.leggauss(n)
    assert np.all(np.diff(x) > 0)
    assert np.max(np.abs(x - xr)) < 2e-15
    assert np.max(np.abs(w - wr)) < 5e-14  # numpy's own weights carry ~1e-14 absolute
    assert abs(w.sum() - 2.0) < 1e-14
    for deg in range(0, min(2 * n, 48)):
        exact = 2.0 / (deg + 1) if deg % 2 == 0 else 0.0
        assert abs(np.dot(w, x ** deg) - exact) < 2e-14, (n, deg)


@pytest.mark.parametrize("n", [7, 64, 128])
def test_gauss_legendre_40_digits(n):
    """Nodes and weights against roots of P_n found in 40-digit arithmetic."""
    import mpmath as mp
    mp.mp.dps = 40
    x, w = oracle.gauss_legendre(n)
    xs, ws = _mp_rule(n)
    for i in range(0, n, max(1, n // 9)):
        assert abs(x[i] - float(xs[i])) < 1e-16
        assert abs(w[i] / float(ws[i]) - 1) < 1e-15
    mp.mp.dps = 15


def test_prefactors_closed_form():
    for d in (3, 4):
        assert oracle.Pd(d) == pytest.approx(closed_Pd(d), rel=1e-15)
        assert oracle.Cd(d) == pytest.approx(closed_Cd(d), rel=1e-15)


# ------------------------------------------------------- Litim at p = 0 --

@pytest.mark.parametrize("d", [3, 4])
@pytest.mark.parametrize("k", [1.0, 0.7, 2.5])
def test_litim_p0_closed_form(d, k):
    k2 = k * k
    m2 = np.array([-0.9, -0.5, -1.0 + 1e-8, 0.0, 3.0]) * k2
    delta = m2 + k2
    n_a = 16
    got = oracle.integrate(d, REG_LITIM, k, 6 * k, 32, n_a, np.zeros_like(m2), m2)
    want = closed_Pd(d) * mu_sum(d, n_a) * 2 * k ** (d + 2) / (d * delta ** 3)
    np.testing.assert_allclose(got, want, rtol=2e-14, atol=0)
    if d == 3:  # continuum value k^5/(3 pi^2 delta^3): the d=3 angular rule is exact
        np.testing.assert_allclose(got, k ** 5 / (3 * PI ** 2 * delta ** 3), rtol=2e-14)


# -------------------------------------------------- exp, large mass limit --

@pytest.mark.parametrize("d", [3, 4])
def test_exp_large_mass_limit(d):
    """m^6 I(m^2) -> P_d (sum mu) k^{d+2} Gamma(d/2+2) zeta(d/2+1), Richardson in 1/m^2."""
    k, n_a = 1.3, 16
    p = np.array([0.4])

    def f(M):
        return M ** 3 * oracle.integrate(d, REG_EXP, k, 8 * k, 64, n_a, p, np.array([M]))[0]

    M = 1e5
    r1 = 2 * f(2 * M) - f(M)
    r2 = 2 * f(4 * M) - f(2 * M)
    lim = (4 * r2 - r1) / 3
    want = closed_Pd(d) * mu_sum(d, n_a) * k ** (d + 2) * special.gamma(d / 2 + 2) * special.zeta(d / 2 + 1)
    assert lim == pytest.approx(want, rel=1e-11)
    # without Richardson the leading correction is O(1/m^2) and negative
    assert f(M) < want


# ------------------------------------------------- continuum, scipy quad --

def _continuum(d, reg, k, Q, p, m2):
    """int d^dq/(2pi)^d d_tR G(q)^2 G(q+p) truncated at |q| <= Q, by adaptive
    quadrature.  R, d_tR = k dR/dk and G are written from their definitions;
    the angular integral runs over s = |q+p|^2 (d = 3) or over x with the
    algebraic weight (1-x^2)^{1/2} handled by QUADPACK (d = 4)."""
    k2 = k * k

    def R(s):
        if reg == REG_EXP:
            return s / math.expm1(s / k2) if s > 0 else k2
        return max(k2 - s, 0.0)

    def dtR(s):
        if reg == REG_EXP:
            y = s / k2
            # k d/dk [s/(e^{s/k^2}-1)] = 2 s^2 e^y / (k^2 (e^y - 1)^2)
            return 2.0 * s * s * math.exp(y) / (k2 * math.expm1(y) ** 2) if y > 0 else 2 * k2
        return 2.0 * k2 if s < k2 else 0.0

    def G(s):
        return 1.0 / (s + R(s) + m2)

    kinks = [k2] if reg == REG_LITIM else []

    def inner(q):
        if d == 3:
            lo, hi = (q - p) ** 2, (q + p) ** 2
            pts = [s for s in kinks if lo < s < hi]
            v = integrate.quad(G, lo, hi, points=pts or None, epsabs=0, epsrel=1e-13, limit=200)[0]
            return v / (2 * q * p)
        # d = 4: x-form with weight (1+x)^{1/2} (1-x)^{1/2}
        g = lambda x: G(q * q + p * p + 2 * q * p * x)
        return integrate.quad(g, -1.0, 1.0, weight="alg", wvar=(0.5, 0.5), epsabs=0,
                              epsrel=1e-13, limit=200)[0]

    def outer(q):
        s = q * q
        return q ** (d - 1) * dtR(s) * G(s) ** 2 * inner(q)

    pts = []
    if reg == REG_LITIM:
        pts = [x for x in (abs(k - p), k + p) if 0 < x < Q]
    val = integrate.quad(outer, 0.0, Q, points=pts or None, epsabs=0, epsrel=1e-13, limit=400)[0]
    return oracle.Omega(d - 1) / (2 * PI) ** d * val


@pytest.mark.parametrize("p,m2", [(0.3, -0.5), (1.0, 0.0), (3.0, 2.0), (0.05, 0.7)])
def test_exp_d3_continuum(p, m2):
    got = oracle.integrate(3, REG_EXP, 1.0, 6.0, 128, 64, [p], [m2])[0]
    want = _continuum(3, REG_EXP, 1.0, 6.0, p, m2)
    assert got == pytest.approx(want, rel=1e-11)


@pytest.mark.parametrize("p,m2", [(0.3, -0.5), (2.0, 1.0)])
def test_exp_d4_continuum_and_rate(p, m2):
    """The literal d = 4 rule (GL weights times sqrt(1-x^2)) converges to the
    continuum algebraically, ~ n_a^-3."""
    want = _continuum(4, REG_EXP, 1.0, 6.0, p, m2)
    errs = [abs(oracle.integrate(4, REG_EXP, 1.0, 6.0, 96, n, [p], [m2])[0] / want - 1)
            for n in (32, 64, 128)]
    assert errs[0] / errs[1] == pytest.approx(8.0, rel=0.15)
    assert errs[1] / errs[2] == pytest.approx(8.0, rel=0.15)
    big = oracle.integrate(4, REG_EXP, 1.0, 6.0, 96, 1024, [p], [m2])[0]
    assert big == pytest.approx(want, rel=2e-9)


@pytest.mark.parametrize("p,m2", [(0.4, -0.3), (1.7, 0.5)])
def test_litim_d3_continuum(p, m2):
    """Litim, p > 0: the kink at |q+p| = k limits the rule to algebraic convergence."""
    want = _continuum(3, REG_LITIM, 1.0, 6.0, p, m2)
    got = oracle.integrate(3, REG_LITIM, 1.0, 6.0, 256, 2048, [p], [m2])[0]
    assert got == pytest.approx(want, rel=2e-5)
    coarse = oracle.integrate(3, REG_LITIM, 1.0, 6.0, 32, 32, [p], [m2])[0]
    assert abs(got / want - 1) < abs(coarse / want - 1)


# ------------------------------------------ discrete rule, 40 digits ---

def _mp_rule(n):
    """Gauss-Legendre rule from mpmath's Legendre function (hypergeometric
    evaluation, 100 working digits), roots polished from numpy's nodes."""
    import mpmath as mp
    xr, _ = np.polynomial.legendre.leggauss(n)
    xs, ws = [], []
    with mp.workdps(100):
        for x0 in xr:
            x = mp.findroot(lambda t: mp.legendre(n, t), mp.mpf(x0), tol=mp.mpf(10) ** -80)
            dp = mp.diff(lambda t: mp.legendre(n, t), x)
            xs.append(x)
            ws.append(2 / ((1 - x * x) * dp * dp))
    return xs, ws


def _mp_discrete(d, reg, k, q_max, n_r, n_a, p, m2):
    import mpmath as mp
    k, p, m2 = mp.mpf(k), mp.mpf(p), mp.mpf(m2)
    k2 = k * k
    Q = min(mp.mpf(q_max), k) if reg == REG_LITIM else mp.mpf(q_max)
    xi, om = _mp_rule(n_r)
    xa, va = _mp_rule(n_a)

    def R(s):
        if reg == REG_EXP:
            return s / mp.expm1(s / k2)
        return max(k2 - s, mp.mpf(0))

    def dtR(s):
        if reg == REG_EXP:
            y = s / k2
            return 2 * s * s * mp.exp(y) / (k2 * mp.expm1(y) ** 2)
        return 2 * k2 if s < k2 else mp.mpf(0)

    G = lambda s: 1 / (s + R(s) + m2)
    tot = mp.mpf(0)
    for i in range(n_r):
        q = Q * (1 + xi[i]) / 2
        w = Q * om[i] / 2
        A = w * q ** (d - 1) * dtR(q * q) * G(q * q) ** 2
        for j in range(n_a):
            mu = va[j] * (1 - xa[j] ** 2) ** (mp.mpf(d - 3) / 2)
            tot += A * mu * G(q * q + p * p + 2 * q * p * xa[j])
    Pd = 2 * mp.pi ** (mp.mpf(d - 1) / 2) / mp.gamma(mp.mpf(d - 1) / 2) / (2 * mp.pi) ** d
    return Pd * tot


@pytest.mark.parametrize("d,reg", [(3, REG_EXP), (4, REG_EXP), (3, REG_LITIM), (4, REG_LITIM)])
def test_discrete_rule_extended_precision(d, reg):
    import mpmath as mp
    mp.mp.dps = 40
    pts = [(1e-3, -0.5), (0.37, 0.0), (1.9, -0.95), (5.0, 4.0), (0.8, -1.0 + 1e-6)]
    for p, m2 in pts:
        want = _mp_discrete(d, reg, 1.0, 6.0, 12, 6, p, m2)
        got = oracle.integrate(d, reg, 1.0, 6.0, 12, 6, [p], [m2])[0]
        assert abs(got / float(want) - 1) < 3e-15, (p, m2, got, want)
    mp.mp.dps = 15


# ------------------------------------------------ limits and invariants --

def test_p_to_zero_is_quadratic():
    """(I(p) - I(0))/I(0) = c2 p^2 + O(p^4): the symmetric angular rule keeps odd moments at zero."""
    p = np.array([0.0, 1e-2, 1e-3, 1e-4])
    I = oracle.integrate(3, REG_EXP, 1.0, 6.0, 64, 16, p, np.full(4, 0.3))
    c = (I[1:] - I[0]) / I[0] / p[1:] ** 2
    assert c[0] == pytest.approx(c[1], rel=1e-3)
    assert c[1] == pytest.approx(c[2], rel=1e-4)


@pytest.mark.parametrize("d,reg", [(3, REG_EXP), (4, REG_EXP), (3, REG_LITIM), (4, REG_LITIM)])
def test_positive_and_decreasing_in_mass(d, reg):
    m2 = np.linspace(-0.99, 10.0, 40)
    for p in (1e-3, 0.5, 4.0):
        I = oracle.integrate(d, reg, 1.0, 6.0, 32, 8, np.full_like(m2, p), m2)
        assert np.all(I > 0)
        assert np.all(np.diff(I) < 0)


def test_domain_violation_gives_nan():
    out = oracle.integrate(3, REG_EXP, 1.0, 6.0, 16, 8, [0.5, 0.5, 0.5], [-1.0, -1.5, 0.0],
                           allow_domain=True)
    assert np.isnan(out[0]) and np.isnan(out[1]) and np.isfinite(out[2])
    with pytest.raises(ValueError):
        oracle.integrate(3, REG_EXP, 1.0, 6.0, 16, 8, [0.5], [-1.0])


# ------------------------------------------------------------------- LPA --

@pytest.mark.parametrize("d", [3, 4])
@pytest.mark.parametrize("n", [1, 2])
def test_litim_threshold_closed_form(d, n):
    k = 0.8
    m2 = np.array([-0.9, -0.3, 0.0, 2.0]) * k * k
    got = oracle.threshold(d, REG_LITIM, k, 6 * k, 16, n, m2)
    want = closed_Cd(d) * 2 * k ** (d + 2) / (d * (m2 + k * k) ** n)
    np.testing.assert_allclose(got, want, rtol=1e-14)


@pytest.mark.parametrize("d", [3, 4])
def test_exp_threshold_zeta_forms(d):
    k = 1.4
    # F_1(0) = C_d k^d Gamma(d/2+1) zeta(d/2+1)
    f0 = oracle.threshold(d, REG_EXP, k, 8 * k, 64, 1, [0.0])[0]
    assert f0 == pytest.approx(closed_Cd(d) * k ** d * special.gamma(d / 2 + 1) * special.zeta(d / 2 + 1),
                               rel=1e-13)
    # m^2 F_1(m^2) -> C_d k^{d+2} Gamma(d/2+2) zeta(d/2+1)
    f = lambda M: M * oracle.threshold(d, REG_EXP, k, 8 * k, 64, 1, [M])[0]
    M = 1e5
    r1, r2 = 2 * f(2 * M) - f(M), 2 * f(4 * M) - f(2 * M)
    assert (4 * r2 - r1) / 3 == pytest.approx(
        closed_Cd(d) * k ** (d + 2) * special.gamma(d / 2 + 2) * special.zeta(d / 2 + 1), rel=1e-11)


@pytest.mark.parametrize("N", [1, 2, 4])
def test_lpa_rhs_quadratic_potential_litim(N):
    """U = a + b rho + c rho^2: the difference formulas are exact, so
    m_sigma^2 = b + 6 c rho, m_pi^2 = b + 2 c rho, and with the Litim closed
    form d_tU = C_d k^{d+2}/d [1/(m_s^2+k^2) + (N-1)/(m_p^2+k^2)]."""
    d, k, n, rho_max = 3, 0.9, 64, 0.5
    a, b, c = 0.1, -0.2, 1.5
    rho = np.linspace(0, rho_max, n)
    U = a + b * rho + c * rho ** 2
    dUdt, _, rc = oracle.lpa_rhs(d, N, REG_LITIM, 32, 6.0, k, rho_max, U)
    ms, mp_ = b + 6 * c * rho, b + 2 * c * rho
    want = closed_Cd(d) * k ** (d + 2) / d * (1 / (ms + k * k) + (N - 1) / (mp_ + k * k))
    np.testing.assert_allclose(dUdt, want, rtol=1e-11)


@pytest.mark.parametrize("N", [1, 4])
def test_lpa_jacobian_matches_numerical_derivative(N):
    d, k, n, rho_max = 3, 0.6, 24, 0.5
    rho = np.linspace(0, rho_max, n)
    U = 5.0 / 8 * (rho - 0.1) ** 2 + 0.02 * np.sin(7 * rho)
    _, jac, _ = oracle.lpa_rhs(d, N, REG_EXP, 64, 6.0, k, rho_max, U)
    eps = 1e-8
    num = np.zeros((n, n))
    for l in range(n):
        Up, Um = U.copy(), U.copy()
        Up[l] += eps
        Um[l] -= eps
        num[:, l] = (oracle.lpa_rhs(d, N, REG_EXP, 64, 6.0, k, rho_max, Up, False)[0]
                     - oracle.lpa_rhs(d, N, REG_EXP, 64, 6.0, k, rho_max, Um, False)[0]) / (2 * eps)
    dense = np.zeros((n, n))
    for o in range(-3, 4):
        for j in range(n):
            if 0 <= j + o < n:
                dense[j, j + o] = jac[o + 3, j]
    scale = np.max(np.abs(num))
    assert np.max(np.abs(dense - num)) < 1e-6 * scale
    # nothing outside the 7 bands
    for j in range(n):
        for l in range(n):
            if abs(l - j) > 3:
                assert abs(num[j, l]) < 1e-9 * scale


# ------------------------------------------- tabulated-propagator variant --

def test_tab_constant_table_closed_form():
    """G_r(s) = g_r constant: I = P_d g^3 (sum mu) sum_i w_i q_i^{d-1} d_tR; Litim,
    d = 3: 2k^2 k^3/3 for the radial sum (GL exact), sum mu = 2."""
    k = 0.7
    g = np.array([0.3, 1.0, 2.5])
    G = np.repeat(g[:, None], 5, axis=1)
    p = np.array([0.0, 0.2, 3.0])
    got = oracle.integrate_tab(3, REG_LITIM, k, 6 * k, 16, 8, G, 4.0, p)
    want = closed_Pd(3) * g[None, :] ** 3 * 2 * k * k * k ** 3 / 3 * 2
    np.testing.assert_allclose(got, np.broadcast_to(want, got.shape), rtol=2e-15)


@pytest.mark.parametrize("p", [0.0, 0.35, 1.7])
def test_tab_linear_table_is_exact_polynomial(p):
    """G(s) = a + b s tabulated over a range covering every s: the interpolation
    is exact, sum_j mu_j s_ij = 2(q^2 + p^2) for the symmetric d = 3 rule, and
    I = P_3 2k^2 int_0^k q^2 (a + b q^2)^2 2(a + b(q^2 + p^2)) dq exactly
    (polynomial of degree 8; 16 radial nodes integrate it exactly)."""
    k, a, b = 0.9, 0.8, -0.15
    s_max = (k + p) ** 2 * 1.01 + 1.0
    n_s = 33
    s_nodes = np.linspace(0.0, s_max, n_s)
    G = (a + b * s_nodes)[None, :]
    got = oracle.integrate_tab(3, REG_LITIM, k, 6 * k, 16, 12, G, s_max, [p])[0, 0]
    poly = np.polynomial.Polynomial
    q = poly([0, 1])
    f = q ** 2 * (a + b * q ** 2) ** 2 * 2 * (a + b * (q ** 2 + p * p))
    F = f.integ()
    want = closed_Pd(3) * 2 * k * k * (F(k) - F(0))
    assert abs(got - want) <= 1e-14 * abs(want)


def test_tab_clamps_beyond_the_table():
    """Every s above s_max takes the last node: a two-node table with a tiny
    s_max reduces to the constant-table closed form with g = last node."""
    k = 1.1
    G = np.array([[7.0, 0.6]])
    got = oracle.integrate_tab(3, REG_LITIM, k, 6 * k, 12, 6, G, 1e-300, [0.5])
    want = closed_Pd(3) * 0.6 ** 3 * 2 * k * k * k ** 3 / 3 * 2
    np.testing.assert_allclose(got[0, 0], want, rtol=2e-15)


@pytest.mark.parametrize("d", [3, 4])
def test_tab_converges_to_analytic_propagator(d):
    """Tabulating the exponential-regulator propagator 1/(s + R(s) + m^2) (R
    written here from its definition) on finer grids approaches the analytic
    quadrature at the O(h^2) rate of linear interpolation."""
    k, m2 = 1.0, 0.4
    p = np.array([0.0, 0.3, 2.0])
    n_r, n_a = 48, 12
    want = oracle.integrate(d, REG_EXP, k, 6 * k, n_r, n_a, p, np.full(3, m2))
    s_max = (6 * k + p.max()) ** 2

    def table(n_s):
        s = np.linspace(0.0, s_max, n_s)
        R = np.where(s > 0, s / np.expm1(np.where(s > 0, s, 1.0) / k ** 2), k ** 2)
        return (1.0 / (s + R + m2))[None, :]

    errs = []
    for n_s in (2001, 4001, 8001, 16001):
        got = oracle.integrate_tab(d, REG_EXP, k, 6 * k, n_r, n_a, table(n_s), s_max, p)[:, 0]
        errs.append(np.max(np.abs(got - want) / want))
    assert errs[-1] < 1e-6
    # the quadrature nodes sample the interpolation error at scattered positions
    # in their cells, so single halvings of h scatter around 4; over an 8-fold
    # refinement the reduction is close to 64
    for e1, e2 in zip(errs, errs[1:]):
        assert 2.5 < e1 / e2 < 7.0
    assert 40 < errs[0] / errs[-1] < 100


def test_tab_domain_and_arguments():
    G = np.ones((2, 4))
    out = oracle.integrate_tab(3, REG_EXP, 1.0, 6.0, 8, 4, G, 10.0, [-1.0, 0.5], allow_domain=True)
    assert np.all(np.isnan(out[0])) and np.all(np.isfinite(out[1]))
    with pytest.raises(ValueError):
        oracle.integrate_tab(3, REG_EXP, 1.0, 6.0, 8, 4, np.ones((2, 1)), 10.0, [0.5])
    with pytest.raises(ValueError):
        oracle.integrate_tab(3, REG_EXP, 1.0, 6.0, 8, 4, G, 0.0, [0.5])


# ------------------------------------------- momentum-dependent flow (f2) --

@pytest.mark.parametrize("d", [3, 5])
@pytest.mark.parametrize("t", [0.0, math.log(0.5)])
def test_pflow_rhs_litim_p0_closed_form(d, t):
    """Litim regulator, uniform Sigma = m^2, k^2 on a node of the table
    (h = 1/4; k^2 = 1 at t = 0, 1/4 at t = ln 1/2): below k^2 every node holds
    1/(k^2 + m^2), so at p = 0 the diagram is closed-form,
    J(0) = C_d (2/d) k^(d+2) / (k^2 + m^2)^3 and T = C_d (2/d) k^(d+2) / (k^2 + m^2)^2
    (d = 3, 5: the angular weight (1 - x^2)^((d-3)/2) is a polynomial, so the
    angular rule is exact and P_d sum_j mu_j = C_d)."""
    k = math.exp(t)
    lam3 = np.array([1.0, 0.0, 2.5, 0.7])
    lam4 = np.array([0.0, 1.0, 3.0, -2.0])
    m2 = np.array([0.3, -0.1, 2.0, 0.05]) * k * k
    Sigma = np.repeat(m2[:, None], 17, axis=1)
    rhs, dead = oracle.pflow_rhs(d, REG_LITIM, 1.0, 6.0, 12, 6, 4.0, lam3, lam4, t, Sigma)
    assert not dead.any()
    base = closed_Cd(d) * (2.0 / d) * k ** (d + 2)
    want = base * (lam3 ** 2 / (k * k + m2) ** 3 - 0.5 * lam4 / (k * k + m2) ** 2)
    np.testing.assert_allclose(rhs[:, 0], want, rtol=1e-13, atol=1e-15 * base)


def test_pflow_rhs_is_linear_in_the_couplings():
    """d_t Sigma = lam3^2 J - lam4/2 T: the right-hand side for (lam3, lam4)
    is lam3^2 times that for (1, 0) plus lam4 times that for (0, 1)."""
    rng = np.random.Generator(np.random.PCG64(3))
    Sigma = rng.uniform(0.1, 1.0, (1, 21))
    args = (3, REG_EXP, 1.0, 6.0, 16, 8, 9.0)
    a, _ = oracle.pflow_rhs(*args, [1.0], [0.0], -0.3, Sigma)
    b, _ = oracle.pflow_rhs(*args, [0.0], [1.0], -0.3, Sigma)
    c, _ = oracle.pflow_rhs(*args, [1.7], [-2.3], -0.3, Sigma)
    np.testing.assert_allclose(c, 1.7 ** 2 * a - 2.3 * b, rtol=1e-13, atol=1e-16)
    assert np.all(a > 0) and np.all(b < 0)  # J > 0, T > 0


def test_pflow_without_cubic_coupling_stays_uniform():
    """With lam3 = 0 the right-hand side is the same at every momentum, so a
    uniform Sigma stays uniform (to the bit) under the RK4 steps."""
    S0 = np.full((2, 33), 0.4)
    S, tr = oracle.pflow_solve(4, REG_EXP, 1.0, 6.0, 24, 8, 16.0, [0.0, 0.0], [1.5, -3.0],
                               -1.5, 30, S0)
    assert np.all(tr == -1.5)
    for r in range(2):
        assert np.all(S[r] == S[r, 0])
    assert S[0, 0] > 0.4 and S[1, 0] < 0.4  # -lam4/2 T dt with dt < 0


@pytest.mark.parametrize("d", [3, 4])
def test_pflow_matches_the_continuum_mass_flow(d):
    """lam3 = 0, Litim: Sigma stays uniform, m^2(t), and the radial rule is
    exact for the Litim integrand; once the table is fine enough that no
    radial node falls in the cell across the kink of R at s = k^2, the
    interpolation is exact too and the discrete flow is the continuum ODE
    d_t m^2 = -(lam4/2) C_d (2/d) k^(d+2) / (k^2 + m^2)^2, k = e^t (integrated
    here by scipy at tight tolerance) up to the RK4 error.  On a coarse table
    the kink cell costs a visible but bounded error."""
    lam4, m20, t_end = 4.0, 0.2, -1.0
    Cd = closed_Cd(d)

    def f(t, y):
        k = math.exp(t)
        return [-0.5 * lam4 * Cd * (2.0 / d) * k ** (d + 2) / (k * k + y[0]) ** 2]

    ref = integrate.solve_ivp(f, (0.0, t_end), [m20], method="DOP853", rtol=1e-13,
                              atol=1e-15).y[0, -1]
    errs = {}
    for n_s in (65, 1025):
        S, tr = oracle.pflow_solve(d, REG_LITIM, 1.0, 6.0, 8, 4, 1.0, [0.0], [lam4], t_end, 200,
                                   np.full((1, n_s), m20))
        assert tr[0] == t_end
        errs[n_s] = abs(S[0, 0] - ref) / abs(ref - m20)
    assert errs[1025] < 1e-10
    assert 1e-7 < errs[65] < 1e-3


def test_pflow_rk4_is_fourth_order():
    """Halving the step divides the error of the final state by ~16 (a
    table clamped beyond a tiny s_max makes the right-hand side smooth in t:
    G = 1/(s_max + R_k(s_max) + Sigma), the same at every node)."""
    args = (3, REG_EXP, 1.0, 6.0, 16, 8, 1e-6, [2.0], [1.0], -1.0)
    S0 = np.full((1, 3), 0.5)
    ref, _ = oracle.pflow_solve(*args, 512, S0)
    errs = [np.max(np.abs(oracle.pflow_solve(*args, n, S0)[0] - ref)) for n in (4, 8, 16, 32)]
    assert abs(ref[0, 0] - 0.5) > 0.1
    for e1, e2 in zip(errs, errs[1:]):
        assert 11.0 < e1 / e2 < 17.0


def test_pflow_domain_stops():
    """A flow whose table denominator s + R_k(s) + Sigma is not positive stops
    at the start of that step with its state kept; the other flows of the
    batch are unaffected (rows are independent)."""
    args = (3, REG_EXP, 1.0, 6.0, 16, 8, 4.0)
    S0 = np.vstack([np.full(17, -1.5), np.full(17, 0.5), np.full(17, -0.5)])
    lam3, lam4 = [1.0, 1.0, 2.0], [0.0, 0.0, 0.0]
    S, tr = oracle.pflow_solve(*args, lam3, lam4, -2.0, 40, S0)
    assert tr[0] == 0.0 and np.all(S[0] == -1.5)  # k^2 - 1.5 < 0 at p = 0
    assert tr[1] == -2.0
    assert tr[2] == 3 * (-2.0 / 40)  # driven to the pole during the fourth step
    assert np.all(np.isfinite(S[2])) and np.all(S[2] < -0.5)
    alone, tr1 = oracle.pflow_solve(*args, lam3[1:2], lam4[1:2], -2.0, 40, S0[1:2])
    assert np.array_equal(alone[0], S[1]) and tr1[0] == -2.0
    _, dead = oracle.pflow_rhs(*args, lam3, lam4, 0.0, S0, allow_domain=True)
    assert list(dead) == [1, 0, 0]


# ------------------------------------------------------- vertex diagram (f3) --

def _exp_parts(k, m2):
    """Continuum integrand pieces written from the regulator's definition
    (R = s/(e^{s/k^2} - 1), d_tR = k dR/dk), independent of the oracle."""
    def dtR(s):
        y = s / k ** 2
        if y == 0.0:
            return 2.0 * k * k
        return 2.0 * s * math.exp(y) * y / math.expm1(y) ** 2

    def G(s):
        y = s / k ** 2
        R = s / math.expm1(y) if y > 0 else k * k
        return 1.0 / (s + R + m2)
    return dtR, G


@pytest.mark.parametrize("d,n_ang,rtol", [(3, 4, 1e-14), (5, 24, 1e-12)])
def test_vertex_litim_zero_momenta_closed_form(d, n_ang, rtol):
    """Litim, p1 = p2 = 0: every propagator is 1/(k^2 + m^2) inside the
    support, V = C_d (2/d) k^(d+2)/(k^2 + m^2)^4 (d = 3: both angular weights
    are 1, the rule is exact; d = 5: (1 - x^2) is exact, sin^2 phi converges)."""
    k, m2 = 1.3, np.array([0.2, -0.5, 4.0])
    v = oracle.integrate_vertex(d, REG_LITIM, k, 6 * k, 8, n_ang, n_ang, np.zeros(3), np.zeros(3),
                                [0.3, -1.0, 1.0], m2)
    want = closed_Cd(d) * (2.0 / d) * k ** (d + 2) / (k * k + m2) ** 4
    np.testing.assert_allclose(v, want, rtol=rtol)


@pytest.mark.parametrize("p1,p2,ct", [(0.7, 1.3, 0.25), (2.0, 0.5, -0.8), (1.1, 1.1, -0.5)])
def test_vertex_matches_continuum_d3(p1, p2, ct):
    """d = 3, exponential regulator, generic configurations: the product
    rule converges spectrally to the continuum integral over (q, x, phi)
    (scipy tplquad of the integrand written from the definitions)."""
    k, m2 = 1.0, 0.3
    dtR, G = _exp_parts(k, m2)
    st = math.sqrt(1 - ct * ct)

    def f(phi, x, q):
        s1 = q * q + p1 * p1 + 2 * q * p1 * x
        s2 = q * q + p2 * p2 + 2 * q * p2 * (x * ct + math.sqrt(1 - x * x) * math.cos(phi) * st)
        return q * q * dtR(q * q) * G(q * q) ** 2 * G(s1) * G(s2)

    val, _ = integrate.tplquad(f, 0, 6 * k, -1, 1, 0, PI, epsabs=1e-14, epsrel=1e-12)
    want = 2.0 / (2 * PI) ** 3 * val
    got = oracle.integrate_vertex(3, REG_EXP, k, 6 * k, 64, 32, 32, [p1], [p2], [ct], [m2])[0]
    assert abs(got - want) <= 1e-11 * want


def test_vertex_d4_converges_at_third_order():
    """d = 4: the polar weight sqrt(1 - x^2) taken literally (as for I) gives
    O(n^-3) convergence to the continuum (scipy tplquad with weights
    sqrt(1 - x^2) sin phi and prefactor 2 pi/(2 pi)^4)."""
    k, m2, p1, p2, ct = 1.0, 0.3, 0.7, 1.3, 0.25
    dtR, G = _exp_parts(k, m2)
    st = math.sqrt(1 - ct * ct)

    def f(phi, x, q):
        s1 = q * q + p1 * p1 + 2 * q * p1 * x
        s2 = q * q + p2 * p2 + 2 * q * p2 * (x * ct + math.sqrt(1 - x * x) * math.cos(phi) * st)
        return (q ** 3 * math.sqrt(1 - x * x) * math.sin(phi) * dtR(q * q) * G(q * q) ** 2 * G(s1)
                * G(s2))

    val, _ = integrate.tplquad(f, 0, 6 * k, -1, 1, 0, PI, epsabs=1e-14, epsrel=1e-11)
    want = 2 * PI / (2 * PI) ** 4 * val
    errs = [abs(oracle.integrate_vertex(4, REG_EXP, k, 6 * k, 48, n, n, [p1], [p2], [ct], [m2])[0]
                - want) / want for n in (16, 32, 64)]
    for e1, e2 in zip(errs, errs[1:]):
        assert 6.0 < e1 / e2 < 10.0
    assert errs[-1] < 3e-6


def test_vertex_symmetries():
    """Swapping p1 and p2 (same angle) is a symmetry of the integral; the rule
    (tied to p1's axis) reproduces it to rounding once converged.  With
    p2 = 0 the angle does not enter: the same bits for every cos th."""
    k, m2 = 1.0, 0.4
    a = oracle.integrate_vertex(3, REG_EXP, k, 6 * k, 48, 24, 24, [0.7, 1.9], [1.9, 0.7],
                                [0.1, 0.1], [m2, m2])
    assert abs(a[0] - a[1]) <= 1e-13 * a[0]
    v = oracle.integrate_vertex(4, REG_LITIM, k, 6 * k, 16, 8, 8, np.full(3, 0.9), np.zeros(3),
                                [-1.0, 0.2, 1.0], np.full(3, m2))
    assert v[0] == v[1] == v[2]


def test_vertex_domain():
    v = oracle.integrate_vertex(3, REG_EXP, 1.0, 6.0, 8, 4, 4, [0.5, -0.1, 0.5, 0.5],
                                [0.5, 0.5, 0.5, 0.5], [0.2, 0.2, 1.5, 0.2], [0.1, 0.1, 0.1, -1.0],
                                allow_domain=True)
    assert np.isfinite(v[0]) and np.all(np.isnan(v[1:]))
    with pytest.raises(ValueError):
        oracle.integrate_vertex(3, REG_EXP, 1.0, 6.0, 8, 4, 0, [0.5], [0.5], [0.2], [0.1])


# ------------------------------------------------- finite-volume LPA (f4) --

def _litim_F(n_, m2, d, k=1.0):
    """Litim threshold functions in closed form, C_d (2/d) k^(d+2)/(k^2 + m^2)^n."""
    return closed_Cd(d) * (2.0 / d) * k ** (d + 2) / (k * k + m2) ** n_


def _quartic(n, smax, lam=1.0, s02=0.5):
    """Exact cell averages of u = U' for U = lam/8 (sigma^2 - s02)^2, and the
    exact cell averages of the continuum right-hand side d_sigma Q, i.e. the
    continuum flux Q(sigma) = 1/2 F_1(u') + (N-1)/2 F_1(u/sigma) differenced
    over each cell (Litim closed forms)."""
    U = lambda s: lam / 8 * (s * s - s02) ** 2
    u = lambda s: lam / 2 * s * (s * s - s02)
    up = lambda s: lam / 2 * (3 * s * s - s02)
    ds = smax / n
    f = np.arange(n + 1) * ds
    ubar = (U(f[1:]) - U(f[:-1])) / ds

    def rhs(N, d):
        gold = np.empty_like(f)
        gold[0] = up(0.0)
        gold[1:] = u(f[1:]) / f[1:]
        Q = 0.5 * _litim_F(1, up(f), d) + 0.5 * (N - 1) * _litim_F(1, gold, d)
        return (Q[1:] - Q[:-1]) / ds
    return ubar, rhs


@pytest.mark.parametrize("reg", [REG_EXP, REG_LITIM])
@pytest.mark.parametrize("N", [1, 2, 4])
def test_fvlpa_linear_u_is_stationary(N, reg):
    """A quadratic potential (u = m^2 sigma, linear) has a constant continuum
    flux N/2 F_1(m^2): the reconstruction is exact on linear data, every
    interface state has u/sigma = m^2, and the right-hand side vanishes to
    rounding in every cell (N = 1, 2, 4)."""
    n, smax = 48, 2.0
    s = (np.arange(n) + 0.5) * smax / n
    u = np.vstack([0.3 * s, -0.2 * s, 4.0 * s])
    r, dt, dead = oracle.fvlpa_rhs(3, N, reg, 24, 1.0, 6.0, smax, -0.4, u)
    assert not dead.any() and np.all(dt > 0)
    scale = _litim_F(1, 0.0, 3) / (smax / n)
    assert np.abs(r).max() < 1e-13 * scale


@pytest.mark.parametrize("d", [3, 4])
def test_fvlpa_converges_to_the_continuum(d):
    """Litim, quartic potential with a minimum at sigma^2 = 1/2: against the
    exact cell averages of the continuum right-hand side, N = 1 converges at
    second order in every cell but the two at the extrapolated edge; N = 4 at
    second order away from sigma = 0, the extremum of u (minmod clipping)
    and the edge, and at first order including them."""
    smax = 1.5
    e1, e4, e4s = [], [], []
    for n in (64, 128, 256):
        ubar, rhs = _quartic(n, smax)
        ds = smax / n
        g1, _, _ = oracle.fvlpa_rhs(d, 1, REG_LITIM, 8, 1.0, 6.0, smax, 0.0, ubar[None, :])
        g4, _, _ = oracle.fvlpa_rhs(d, 4, REG_LITIM, 8, 1.0, 6.0, smax, 0.0, ubar[None, :])
        e1.append(np.abs(g1[0] - rhs(1, d))[:-2].max())
        err4 = np.abs(g4[0] - rhs(4, d))[:-2]
        e4.append(err4.sum() * ds)
        centers = (np.arange(n - 2) + 0.5) * ds
        smooth = (centers > 0.1) & (np.abs(centers - math.sqrt(0.5 / 3)) > 0.1)
        e4s.append(err4[smooth].max())
    for a, b in zip(e1, e1[1:]):
        assert 3.5 < a / b < 4.5
    for a, b in zip(e4s, e4s[1:]):
        assert a / b > 3.5
    for a, b in zip(e4, e4[1:]):
        assert a / b > 1.8


@pytest.mark.parametrize("N", [1, 4])
def test_fvlpa_ssp_rk3_is_third_order(N):
    """Fixed steps well inside the stability bound: halving the step divides
    the error of the final state by ~8."""
    ubar, _ = _quartic(16, 1.5)
    args = (3, N, REG_EXP, 16, 1.0, 6.0, 1.5, -0.5)
    ref, _ = oracle.fvlpa_solve(*args, 2048, ubar[None, :])
    errs = [np.abs(oracle.fvlpa_solve(*args, m, ubar[None, :])[0] - ref).max() for m in (64, 128, 256)]
    for a, b in zip(errs, errs[1:]):
        assert 7.0 < a / b < 9.0


def test_fvlpa_step_estimate_and_domain_stop():
    """The step estimate follows the diffusive bound ds^2/(2D) (a quarter
    when the cells halve, N = 1), and it separates stable from unstable
    steps: a sawtooth of 1e-6 on a symmetric-phase potential does not grow
    over three steps of 0.8 of it and grows over three steps of four times
    it.  A state outside the domain stops at t = 0 with the state kept."""
    dts = {}
    for n in (16, 32):
        smax = 1.5
        ds = smax / n
        f = np.arange(n + 1) * ds
        U = lambda x: x ** 4 / 8 + 0.25 * x * x
        u0 = ((U(f[1:]) - U(f[:-1])) / ds)[None, :]
        _, dt, _ = oracle.fvlpa_rhs(3, 1, REG_EXP, 16, 1.0, 6.0, smax, 0.0, u0)
        dts[n] = dt[0]
    assert 0.24 < dts[32] / dts[16] < 0.26
    saw = 1e-6 * (-1.0) ** np.arange(32)
    growth = {}
    for fac in (0.8, 4.0):
        h = fac * dts[32]
        ref, _ = oracle.fvlpa_solve(3, 1, REG_EXP, 16, 1.0, 6.0, 1.5, -3 * h, 3, u0)
        S, tr = oracle.fvlpa_solve(3, 1, REG_EXP, 16, 1.0, 6.0, 1.5, -3 * h, 3, u0 + saw)
        assert tr[0] == -3 * h
        growth[fac] = np.abs(S - ref).max() / 1e-6
    assert growth[0.8] < 1.01 and growth[4.0] > 2.0
    bad = u0.copy()
    bad[0, 3] = -5.0
    S, tr = oracle.fvlpa_solve(3, 1, REG_EXP, 16, 1.0, 6.0, 1.5, -0.5, 20, bad)
    assert tr[0] == 0.0 and np.array_equal(S, bad)
    _, _, dead = oracle.fvlpa_rhs(3, 1, REG_EXP, 16, 1.0, 6.0, 1.5, 0.0, np.vstack([bad, u0]),
                                  allow_domain=True)
    assert list(dead) == [1, 0]


@pytest.mark.parametrize("n_s", [4097, 65537])
def test_tab_coordinate_bound_covers_ulp_perturbations(n_s):
    """The per-result tolerance for rough tables (oracle.integrate_tab_bound)
    covers the oracle's own response to ulp-level changes of the evaluation
    coordinate: s_max and p moved by 4 ulp shift every t by about 4u t, the
    kind of difference two implementations with ulp-close rules show."""
    rng = np.random.default_rng(11)
    g = 10.0 ** rng.uniform(-1.0, 1.0, (4, n_s))  # rough positive rows, two decades
    s_max = 676.0
    p = np.array([1e-3, 0.37, 2.0, 7.5])
    args = (3, REG_EXP, 1.0, 6.0, 48, 12)
    base = oracle.integrate_tab(*args, g, s_max, p)
    bound = oracle.integrate_tab_bound(*args, g, s_max, p)
    u = 2.0 ** -53
    seen = 0.0
    for sm, pp in ((s_max * (1 + 4 * u), p), (s_max * (1 - 4 * u), p),
                   (s_max, p * (1 + 4 * u)), (s_max, p * (1 - 4 * u))):
        moved = oracle.integrate_tab(*args, g, sm, pp)
        rel = np.abs(moved - base) / base
        assert np.all(rel <= bound), (rel / bound).max()
        seen = max(seen, float((rel / bound).max()))
    # the perturbation is visible and the bound not vacuous
    assert seen > 1e-3
    # smooth rows: the bound is the 1e-13 floor plus a few ulp
    sg = np.linspace(0.0, s_max, n_s)
    gs = (1.0 + 0.1 / (1.0 + sg))[None, :] / (sg[None, :] + np.array([0.1, 1.0, 4.0, 11.0])[:, None])
    assert oracle.integrate_tab_bound(*args, gs, s_max, p).max() < 3e-13
