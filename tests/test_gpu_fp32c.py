"""Compensated-FP32 path (FRG_PREC_FP32C) against the FP64 oracle.

The bar: every returned result within 1e-7 relative of the oracle, by a
stated bound.  A result of the FP32-exponential point path (used_fp64 = 0)
carries a deterministic first-order bound err_est <= fp32c_flag_ppb 1e-9;
its distance to the oracle must not exceed that bound (plus the FP64 level
1e-13) for any result.  Results evaluated in FP64 (near the pole, bound above
the tolerance, Litim, tensor grids) carry 1e-14 and equal the FP64 kernels
bit for bit.  The premise of the bound, the accuracy of the GPU exponential,
is checked on its own."""
import numpy as np
import pytest

import oracle
from paper_2607_24908_amd import frg, workloads

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL32 = 1e-7
EXP_REL = 1.2e-7  # the bound's premise: relative error of the GPU exponential


@pytest.fixture(scope="module")
def ctx():
    assert torch.cuda.is_available()
    h = frg.frg_create(0)
    yield h
    torch.cuda.synchronize()
    frg.frg_destroy(h)


def dev(a):
    return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64), device="cuda")


def points(ctx, sets, prec, flags=frg.FRG_PERSISTENT):
    """Run point sets [(Quad, p, m2)] in one call; returns [(out, err, used)]."""
    ds = []
    for q, p, m2 in sets:
        n = p.size
        ds.append(dict(quad=frg.make_quad(q.d, q.reg, q.k, q.q_max, q.n_r, q.n_a, prec),
                       p=dev(p), m2=dev(m2),
                       out=torch.full((n,), float("nan"), dtype=torch.float64, device="cuda"),
                       err_est=torch.full((n,), float("nan"), dtype=torch.float64, device="cuda"),
                       used_fp64=torch.full((n,), 7, dtype=torch.uint8, device="cuda")))
    frg.frg_integrate(ctx, ds, flags=flags)
    torch.cuda.synchronize()
    return [(d["out"].cpu().numpy(), d["err_est"].cpu().numpy(), d["used_fp64"].cpu().numpy())
            for d in ds]


def histogram(rel):
    edges = 10.0 ** np.arange(-17, -5)
    h, _ = np.histogram(np.clip(rel, 1e-17, 1e-6), bins=edges)
    return " ".join(f"[1e{int(np.log10(a))}:{c}]" for a, c in zip(edges[:-1], h) if c)


def check_against_oracle(q, p, m2, got, err, used, tag):
    want = oracle.integrate(q.d, q.reg, q.k, q.q_max, q.n_r, q.n_a, p, m2)
    rel = np.abs(got - want) / np.abs(want)
    f32 = used == 0
    assert set(np.unique(used)) <= {0, 1}, tag
    assert np.all(err[~f32] == 1e-14), tag
    assert np.all(err[f32] <= TOL32), tag
    # the bound holds for every FP32 result (oracle and FP64 kernels agree to ~1e-15)
    assert np.all(rel[f32] <= err[f32] + 1e-13), (tag, np.max(rel[f32] - err[f32]))
    assert rel.max() < TOL32, tag
    return rel, f32


def test_gpu_exponential_within_premise(ctx):
    """exp_neg32 on the GPU over y in [0, 87.3) (FP32-normal results): the
    relative error stays below 1.2e-7, the premise of the bound; beyond, the
    absolute error is below 2^-126."""
    print("[case] fp32c exponential", flush=True)
    rng = np.random.Generator(np.random.PCG64(11))
    y = np.concatenate([np.linspace(0.0, 87.3, 1 << 22, endpoint=False),
                        rng.uniform(0.0, 87.3, 1 << 20), 10.0 ** rng.uniform(-12, 0, 1 << 16),
                        np.linspace(87.3, 120.0, 4096)])
    out = torch.empty(y.size, dtype=torch.float64, device="cuda")
    frg.frg_expneg_fp32c(ctx, dev(y), out)
    torch.cuda.synchronize()
    got = out.cpu().numpy()
    want = np.exp(-y)
    normal = y < 87.3
    rel = np.abs(got[normal] - want[normal]) / want[normal]
    print(f"max rel err {rel.max():.3e} = {rel.max() / 2.0 ** -24:.3f} u32")
    assert rel.max() <= EXP_REL
    assert np.all(np.abs(got[~normal] - want[~normal]) <= 2.0 ** -126)


@pytest.mark.parametrize("seed", [0, 1, 2, 3])
def test_uneven_exp_points_bound_holds(ctx, seed):
    """Uneven sets of the exponential regulator (sizes and rules of the
    batched workload): the bound holds for every FP32 result, the FP64
    results equal the FP64 kernels bit for bit, and the FP32 path carries
    most of the work."""
    sets = [s for s in workloads.uneven_sets(seed=seed, n_sets=48, max_points=256)
            if s.quad.reg == workloads.REG_EXP]
    print(f"[case] fp32c uneven exp seed={seed} ({len(sets)} sets)", flush=True)
    trip = [(s.quad, s.p, s.m2) for s in sets]
    got = points(ctx, trip, frg.FRG_PREC_FP32C)
    ref = points(ctx, trip, frg.FRG_PREC_FP64)
    work = work32 = 0
    rels = []
    for (q, p, m2), (o, e, u), (o64, _, _) in zip(trip, got, ref):
        rel, f32 = check_against_oracle(q, p, m2, o, e, u, f"seed {seed} {q}")
        assert np.array_equal(o[~f32], o64[~f32])
        work += p.size * q.n_r * q.n_a
        work32 += f32.sum() * q.n_r * q.n_a
        rels.append(rel)
    rel = np.concatenate(rels)
    print(f"FP32 share of the work {work32 / work:.3f}; max rel {rel.max():.3e}")
    print("  histogram:", histogram(rel))
    assert work32 > 0.9 * work


def test_precision_points_near_pole(ctx):
    """The C4 precision workload (d = 4, masses down to 1e-8 above the pole)
    as point lists: points within the band are FP64, the others keep the
    bound."""
    for seed in (0, 1, 2):
        w = workloads.precision_d4(seed)
        q = w.quad
        P = np.repeat(w.p, w.m2.size)
        M = np.tile(w.m2, w.p.size)
        print(f"[case] fp32c {w.name} as points", flush=True)
        (o, e, u), = points(ctx, [(q, P, M)], frg.FRG_PREC_FP32C, flags=frg.FRG_PLAIN)
        rel, f32 = check_against_oracle(q, P, M, o, e, u, w.name)
        dhat = (M + q.k ** 2) / q.k ** 2
        assert np.all(u[dhat < 1e-2] == 1)
        print(f"{w.name}: FP32 {f32.sum()}/{rel.size}, max rel {rel.max():.3e}")
        print("  histogram:", histogram(rel))


@pytest.mark.parametrize("d,n_r,n_a", [(3, 128, 32), (3, 100, 12), (4, 64, 16), (5, 24, 40),
                                       (3, 7, 3)])
def test_other_rules_and_lane_splits(ctx, d, n_r, n_a):
    """Rules whose lane split has 1, 2 or more angular lanes, ragged radial
    rows and ungrouped angular terms."""
    rng = np.random.Generator(np.random.PCG64(n_r + n_a + d))
    p = 10 ** rng.uniform(-3, 1.3, 300)
    m2 = rng.uniform(-0.95, 10.0, 300)
    q = workloads.Quad(d, workloads.REG_EXP, 1.3, 7.8, n_r, n_a)
    print(f"[case] fp32c rule d={d} {n_r}x{n_a}", flush=True)
    for flags in (frg.FRG_PLAIN, frg.FRG_PERSISTENT):
        (o, e, u), = points(ctx, [(q, p, m2)], frg.FRG_PREC_FP32C, flags=flags)
        rel, f32 = check_against_oracle(q, p, m2, o, e, u, f"{d} {n_r}x{n_a}")
        print(f"flags {flags}: FP32 share {f32.mean():.2f}, max rel {rel.max():.3e}")


def test_tolerance_knob_routes_to_fp64(ctx):
    """A tolerance below every bound sends every point to FP64: the results
    are the FP64 kernels' bits."""
    s = workloads.uneven_sets(seed=5, n_sets=6)
    trip = [(x.quad, x.p, x.m2) for x in s]
    old = frg.frg_tune_get(ctx, "fp32c_flag_ppb")
    try:
        frg.frg_tune_set(ctx, "fp32c_flag_ppb", 0)
        got = points(ctx, trip, frg.FRG_PREC_FP32C)
    finally:
        frg.frg_tune_set(ctx, "fp32c_flag_ppb", old)
    ref = points(ctx, trip, frg.FRG_PREC_FP64)
    for (o, e, u), (o64, _, _) in zip(got, ref):
        assert np.all(u == 1) and np.all(e == 1e-14)
        assert np.array_equal(o, o64)


def test_litim_points_and_grids_are_fp64(ctx):
    """Litim FP32C points and every FP32C tensor grid are evaluated in FP64:
    the FP64 kernels' bits, err 1e-14, used_fp64 1."""
    q = workloads.Quad(3, workloads.REG_LITIM, 1.0, 6.0, 64, 16)
    rng = np.random.Generator(np.random.PCG64(4))
    p, m2 = 10 ** rng.uniform(-3, 1, 200), rng.uniform(-0.9, 5.0, 200)
    (o, e, u), = points(ctx, [(q, p, m2)], frg.FRG_PREC_FP32C)
    (o64, _, _), = points(ctx, [(q, p, m2)], frg.FRG_PREC_FP64)
    assert np.all(u == 1) and np.all(e == 1e-14) and np.array_equal(o, o64)
    for w in (workloads.precision_d4(0), workloads.plain_d4()):
        q = w.quad
        outs = {}
        for prec in (frg.FRG_PREC_FP64, frg.FRG_PREC_FP32C):
            quad = frg.make_quad(q.d, q.reg, q.k, q.q_max, q.n_r, q.n_a, prec)
            n = w.p.size * w.m2.size
            out = torch.full((n,), float("nan"), dtype=torch.float64, device="cuda")
            err = torch.full((n,), float("nan"), dtype=torch.float64, device="cuda")
            used = torch.full((n,), 7, dtype=torch.uint8, device="cuda")
            frg.frg_integrate_grid(ctx, quad, dev(w.p), dev(w.m2), out, err, used)
            torch.cuda.synchronize()
            outs[prec] = (out.cpu().numpy(), err.cpu().numpy(), used.cpu().numpy())
        g, ge, gu = outs[frg.FRG_PREC_FP32C]
        assert np.array_equal(g, outs[frg.FRG_PREC_FP64][0])
        assert np.all(ge == 1e-14) and np.all(gu == 1)


def test_mixed_precision_sets_in_one_call(ctx):
    sets = workloads.uneven_sets(seed=3, n_sets=12)
    ds = []
    for i, s in enumerate(sets):
        q = s.quad
        prec = frg.FRG_PREC_FP32C if i % 2 else frg.FRG_PREC_FP64
        ds.append(dict(quad=frg.make_quad(q.d, q.reg, q.k, q.q_max, q.n_r, q.n_a, prec),
                       p=dev(s.p), m2=dev(s.m2),
                       out=torch.zeros(s.p.size, dtype=torch.float64, device="cuda")))
    frg.frg_integrate(ctx, ds, flags=frg.FRG_PERSISTENT)
    torch.cuda.synchronize()
    for i, (s, d) in enumerate(zip(sets, ds)):
        q = s.quad
        want = oracle.integrate(q.d, q.reg, q.k, q.q_max, q.n_r, q.n_a, s.p, s.m2)
        rel = np.abs(d["out"].cpu().numpy() - want) / want
        assert rel.max() < (TOL32 if i % 2 else 1e-12), (i, rel.max())
