"""Two-external-momentum (vertex) diagram on the GPU against the oracle:
ragged shapes, both regulators, the resident coefficient form and the
per-term form, range boundaries, domain, launch shapes, host memory, the
bench workload."""
import numpy as np
import pytest

import oracle
from paper_2607_24908_amd import frg, workloads

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

EXP, LIT = frg.FRG_REG_EXP, frg.FRG_REG_LITIM
RTOL = 1e-12
XTOL = 1e-13  # coefficient form vs per-term form: different rounding paths


@pytest.fixture(scope="module")
def ctx():
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    h = frg.frg_create(0)
    yield h
    torch.cuda.synchronize()
    frg.frg_destroy(h)


def dev(a):
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


def run(ctx, quad, n_phi, p1, p2, c12, m2):
    out = torch.full((len(p1) * len(m2),), float("nan"), dtype=torch.float64, device="cuda")
    frg.frg_integrate_vertex(ctx, quad, n_phi, dev(p1), dev(p2), dev(c12), dev(m2), out)
    torch.cuda.synchronize()
    return out.cpu().numpy()


def want(d, reg, k, n_r, n_a, n_phi, p1, p2, c12, m2):
    P1, P2, C = (np.repeat(np.asarray(v, dtype=np.float64), len(m2)) for v in (p1, p2, c12))
    M = np.tile(np.asarray(m2, dtype=np.float64), len(p1))
    return oracle.integrate_vertex(d, reg, k, 6 * k, n_r, n_a, n_phi, P1, P2, C, M, threads=8,
                                   allow_domain=True)


def configs(rng, n):
    p1 = np.concatenate([[0.0, 0.0, 1.3, 0.5], 10 ** rng.uniform(-3, 1, n)])
    p2 = np.concatenate([[0.0, 0.8, 0.0, 0.5], 10 ** rng.uniform(-3, 1, n)])
    c12 = np.concatenate([[0.3, 1.0, -1.0, 1.0], rng.uniform(-1, 1, n)])
    return p1, p2, c12


# (d, reg, n_r, n_a, n_phi): group sizes 8, 16, 32 (with padding), several
# pairs per lane, and a table too large for LDS (every mass per term)
SHAPES = [(3, EXP, 32, 8, 16), (4, LIT, 24, 6, 8), (3, EXP, 48, 8, 16), (5, EXP, 16, 5, 24),
          (3, LIT, 20, 3, 5), (4, EXP, 64, 16, 8), (3, EXP, 7, 2, 33)]


@pytest.mark.parametrize("d,reg,n_r,n_a,n_phi", SHAPES)
def test_vertex_matches_oracle(ctx, d, reg, n_r, n_a, n_phi):
    print(f"[case] vertex d={d} reg={reg} {n_r}x{n_a}x{n_phi}", flush=True)
    rng = np.random.Generator(np.random.PCG64(n_r * 100 + n_a * 10 + n_phi))
    k = 0.9
    p1, p2, c12 = configs(rng, 13)
    m2 = np.concatenate([[-k * k + 1e-6, 0.0], rng.uniform(-0.9 * k * k, 9.0, 21)])
    quad = frg.make_quad(d, reg, k, 6 * k, n_r, n_a)
    got = run(ctx, quad, n_phi, p1, p2, c12, m2)
    w = want(d, reg, k, n_r, n_a, n_phi, p1, p2, c12, m2)
    err = np.abs(got - w) / np.abs(w)
    print(f"  max rel err {err.max():.3e}")
    assert np.all(np.isfinite(got)) and err.max() < RTOL


def test_vertex_forms_agree(ctx):
    """The per-term form (grid_form = 1) and the coefficient form, as power
    sums on the matrix cores (grid_mfma = 1) and nested on the vector units
    (grid_mfma = 0), agree with each other and with the oracle."""
    rng = np.random.Generator(np.random.PCG64(4))
    p1, p2, c12 = configs(rng, 9)
    m2 = rng.uniform(-0.5, 6.0, 17)
    quad = frg.make_quad(3, EXP, 1.0, 6.0, 32, 8)
    w = want(3, EXP, 1.0, 32, 8, 16, p1, p2, c12, m2)
    default = frg.frg_tune_get(ctx, "grid_form")
    default_mfma = frg.frg_tune_get(ctx, "grid_mfma")
    outs = []
    try:
        for form, mfma in ((0, 1), (0, 0), (1, 1), (1, 0)):
            frg.frg_tune_set(ctx, "grid_form", form)
            frg.frg_tune_set(ctx, "grid_mfma", mfma)
            got = run(ctx, quad, 16, p1, p2, c12, m2)
            assert np.max(np.abs(got - w) / np.abs(w)) < RTOL, (form, mfma)
            outs.append(got)
    finally:
        frg.frg_tune_set(ctx, "grid_form", default)
        frg.frg_tune_set(ctx, "grid_mfma", default_mfma)
    for alt in outs[1:]:
        assert np.all(np.abs(alt - outs[0]) <= XTOL * np.abs(outs[0]))


def test_vertex_range_boundaries(ctx):
    """Masses and momenta on both sides of the bounds of the coefficient form
    (x = sig delta in [lo, hi] and sig (q_top + max(p1, p2))^2 <= hi, sig k^2 =
    1.15 here; G = 16: lo 6e-16, hi 2e15; G = 8: lo 5e-27, hi 4e26), in one
    grid: every form matches the oracle."""
    k = 1e-9
    kk = k * k
    cases = [(16, np.array([0.0, 1e-6, 4e-2, 4.3e-2]), np.array([1e-3, 1e-9, 0.0, 4.1e-2]),
              np.array([0.0, 1e-3, 1.5e-3, 2e-3, -kk + 1e-20, 1e-15])),
             (8, np.array([0.0, 1.0, 1.8e4, 1.9e4]), np.array([2.0, 0.0, 1.0, 1.9e4]),
              np.array([0.0, 1e8, 3e8, 4e8, -kk + 1e-25, 1e-3]))]
    for n_phi, p1, p2, m2 in cases:
        c12 = np.array([0.1, -0.7, 1.0, 0.4])
        for d, reg, n_r, n_a in [(3, EXP, 24, 6), (4, LIT, 16, 4)]:
            print(f"[case] vertex bounds n_phi={n_phi} d={d} reg={reg}", flush=True)
            quad = frg.make_quad(d, reg, k, 6 * k, n_r, n_a)
            got = run(ctx, quad, n_phi, p1, p2, c12, m2)
            w = want(d, reg, k, n_r, n_a, n_phi, p1, p2, c12, m2)
            err = np.abs(got - w) / np.abs(w)
            print(f"  max rel err {err.max():.3e}")
            assert np.all(np.isfinite(got)) and err.max() < RTOL


def test_vertex_launch_shapes_bitwise(ctx):
    rng = np.random.Generator(np.random.PCG64(8))
    p1, p2, c12 = configs(rng, 7)
    m2 = rng.uniform(-0.5, 6.0, 75)
    quad = frg.make_quad(4, EXP, 1.0, 6.0, 24, 6)
    keys = ("grid_M", "grid_W", "grid_MB", "grid_mfma")
    defaults = {key: frg.frg_tune_get(ctx, key) for key in keys}
    try:
        for mfma in (1, 0):
            ref = None
            for M, W, MB in [(8, 4, 16), (4, 2, 1), (16, 8, 4), (4, 8, 8), (8, 1, 3)]:
                for key, v in zip(keys, (M, W, MB, mfma)):
                    frg.frg_tune_set(ctx, key, v)
                got = run(ctx, quad, 8, p1, p2, c12, m2)
                if ref is None:
                    ref = got
                assert np.array_equal(got, ref), (mfma, M, W, MB)
    finally:
        for key, v in defaults.items():
            frg.frg_tune_set(ctx, key, v)


def test_vertex_domain_and_host_memory(ctx):
    quad = frg.make_quad(3, EXP, 1.0, 6.0, 16, 4)
    p1 = np.array([0.5, -0.1, 0.5, 0.7])
    p2 = np.array([0.5, 0.5, 0.5, 0.2])
    c12 = np.array([0.2, 0.2, 1.5, -0.3])
    m2 = np.array([0.1, -1.0, 2.0])
    d_out = run(ctx, quad, 8, p1, p2, c12, m2).reshape(4, 3)
    assert np.all(np.isnan(d_out[1])) and np.all(np.isnan(d_out[2])) and np.all(np.isnan(d_out[:, 1]))
    good = np.isfinite(d_out)
    assert good.sum() == 4
    h_out = np.empty(12)
    with pytest.raises(frg.FrgError):
        frg.frg_integrate_vertex(ctx, quad, 8, p1, p2, c12, m2, h_out, mem=frg.FRG_MEM_HOST)
    frg.frg_integrate_vertex(ctx, quad, 8, p1, p2, c12, m2, h_out, mem=frg.FRG_MEM_HOST,
                             allow_domain=True)
    assert np.array_equal(h_out.reshape(4, 3)[good], d_out[good])
    w = want(3, EXP, 1.0, 16, 4, 8, p1, p2, c12, m2).reshape(4, 3)
    assert np.all(np.abs(d_out[good] - w[good]) <= RTOL * np.abs(w[good]))
    with pytest.raises(frg.FrgError):
        frg.frg_integrate_vertex(ctx, quad, 0, p1, p2, c12, m2, h_out, mem=frg.FRG_MEM_HOST)
    with pytest.raises(frg.FrgError):
        frg.frg_integrate_vertex(ctx, frg.make_quad(3, EXP, 1.0, 6.0, 16, 4, frg.FRG_PREC_FP32C), 8,
                                 p1, p2, c12, m2, h_out, mem=frg.FRG_MEM_HOST)


def test_vertex_bench_workload_sampled(ctx):
    w = workloads.vertex_d3()
    q = w.quad
    print(f"[case] {w.name}", flush=True)
    quad = frg.make_quad(q.d, q.reg, q.k, q.q_max, q.n_r, q.n_a)
    got = run(ctx, quad, w.n_phi, w.p1, w.p2, w.c12, w.m2).reshape(w.p1.size, w.m2.size)
    rng = np.random.Generator(np.random.PCG64(3))
    ia = np.concatenate([rng.integers(0, w.p1.size, 300), [0, w.p1.size - 1]])
    ib = np.concatenate([rng.integers(0, w.m2.size, 300), [0, w.m2.size - 1]])
    ref = oracle.integrate_vertex(q.d, q.reg, q.k, q.q_max, q.n_r, q.n_a, w.n_phi, w.p1[ia],
                                  w.p2[ia], w.c12[ia], w.m2[ib], threads=8)
    err = np.abs(got[ia, ib] - ref) / np.abs(ref)
    print(f"  max rel err {err.max():.3e}")
    assert err.max() < RTOL
