"""Momentum-dependent two-point flow on the GPU against the oracle: one
right-hand side, RK4 solves, domain stops, batching and host memory."""
import numpy as np
import pytest

import oracle
from paper_2607_24908_amd import frg, workloads

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

EXP, LIT = frg.FRG_REG_EXP, frg.FRG_REG_LITIM
# FP64 bar: every right-hand side within 1e-12 of the scale of its two
# parts (lam3^2 |J| + |lam4/2| T: the parts can cancel), every final state
# within 1e-12 of its magnitude.
RTOL = 1e-12


@pytest.fixture(scope="module")
def ctx():
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    h = frg.frg_create(0)
    yield h
    torch.cuda.synchronize()
    frg.frg_destroy(h)


def dev(a):
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


def gpu_rhs(ctx, pf, lam3, lam4, t, S):
    out = torch.full(S.shape, float("nan"), dtype=torch.float64, device="cuda")
    frg.frg_pflow_rhs(ctx, pf, dev(lam3), dev(lam4), t, dev(S), out)
    torch.cuda.synchronize()
    return out.cpu().numpy()


def gpu_solve(ctx, pf, lam3, lam4, t_end, n_steps, S0):
    S = dev(S0)
    tr = torch.full((len(lam3),), float("nan"), dtype=torch.float64, device="cuda")
    frg.frg_pflow_solve(ctx, pf, dev(lam3), dev(lam4), t_end, n_steps, S, tr)
    torch.cuda.synchronize()
    return S.cpu().numpy(), tr.cpu().numpy()


def initial(rng, n_flows, n_s, s_max):
    """Sigma(t = 0): a mass plus a smooth momentum dependence."""
    s = np.linspace(0.0, s_max, n_s)
    m2 = rng.uniform(0.05, 1.0, n_flows)
    b = rng.uniform(-0.2, 0.2, n_flows)
    return m2[:, None] + b[:, None] * s[None, :] / (1.0 + s[None, :])


SHAPES = [(3, EXP, 32, 8, 33, 9.0), (4, LIT, 24, 6, 17, 4.0), (3, EXP, 64, 16, 129, 49.0),
          (5, EXP, 16, 5, 2, 1.0), (3, LIT, 100, 12, 300, 30.0)]


@pytest.mark.parametrize("d,reg,n_r,n_a,n_s,s_max", SHAPES)
def test_rhs_matches_oracle(ctx, d, reg, n_r, n_a, n_s, s_max):
    print(f"[case] pflow rhs d={d} reg={reg} {n_r}x{n_a} n_s={n_s}", flush=True)
    rng = np.random.Generator(np.random.PCG64(n_s * 7 + n_r))
    n = 5
    lam3 = rng.uniform(0.2, 3.0, n)
    lam4 = rng.uniform(-4.0, 8.0, n)
    S = initial(rng, n, n_s, s_max)
    pf = frg.make_pflow(d, reg, n_r, n_a, 1.3, 6.0, n_s, s_max)
    for t in (0.0, -0.7):
        got = gpu_rhs(ctx, pf, lam3, lam4, t, S)
        args = (d, reg, 1.3, 6.0, n_r, n_a, s_max)
        want, dead = oracle.pflow_rhs(*args, lam3, lam4, t, S)
        a, _ = oracle.pflow_rhs(*args, lam3, np.zeros(n), t, S)
        b, _ = oracle.pflow_rhs(*args, np.zeros(n), lam4, t, S)
        scale = np.abs(a) + np.abs(b)
        assert not dead.any()
        err = np.abs(got - want) / scale
        print(f"  t={t}: max scaled err {err.max():.3e}")
        assert err.max() < RTOL


@pytest.mark.parametrize("d,reg,n_r,n_a,n_s,s_max", SHAPES[:3])
def test_solve_matches_oracle(ctx, d, reg, n_r, n_a, n_s, s_max):
    print(f"[case] pflow solve d={d} reg={reg} {n_r}x{n_a} n_s={n_s}", flush=True)
    rng = np.random.Generator(np.random.PCG64(n_s * 11 + n_a))
    n = 4
    lam3 = rng.uniform(0.2, 2.0, n)
    lam4 = rng.uniform(0.0, 6.0, n)
    S0 = initial(rng, n, n_s, s_max) + 0.3
    pf = frg.make_pflow(d, reg, n_r, n_a, 1.0, 6.0, n_s, s_max)
    got, tr = gpu_solve(ctx, pf, lam3, lam4, -2.0, 12, S0)
    want, tr_w = oracle.pflow_solve(d, reg, 1.0, 6.0, n_r, n_a, s_max, lam3, lam4, -2.0, 12, S0,
                                    threads=8)
    assert np.array_equal(tr, tr_w) and np.all(tr == -2.0)
    err = np.abs(got - want).max(axis=1) / np.abs(want).max(axis=1)
    print(f"  max rel err {err.max():.3e}; max |change| {np.abs(want - S0).max():.3e}")
    assert err.max() < RTOL


def test_domain_stops_match_oracle(ctx):
    """Flows outside the domain at t = 0, driven to the pole, and regular
    ones in one batch: the same stops (to the step) and states."""
    args = (3, EXP, 16, 8, 17, 4.0)
    S0 = np.vstack([np.full(17, -1.5), np.full(17, 0.5), np.full(17, -0.5), np.full(17, -0.2)])
    lam3 = np.array([1.0, 1.0, 2.0, 1.5])
    lam4 = np.zeros(4)
    pf = frg.make_pflow(args[0], args[1], args[2], args[3], 1.0, 6.0, args[4], args[5])
    got, tr = gpu_solve(ctx, pf, lam3, lam4, -2.0, 40, S0)
    want, tr_w = oracle.pflow_solve(args[0], args[1], 1.0, 6.0, args[2], args[3], args[5], lam3,
                                    lam4, -2.0, 40, S0)
    print("t_reached", tr, tr_w)
    assert np.array_equal(tr, tr_w)
    assert tr[0] == 0.0 and tr[1] == -2.0 and -2.0 < tr[2] < 0.0
    assert np.array_equal(got[0], S0[0])
    err = np.abs(got - want).max(axis=1) / np.abs(want).max(axis=1)
    assert err.max() < RTOL
    # the right-hand side of a flow outside the domain is NaN, the others finite
    out = gpu_rhs(ctx, pf, lam3, lam4, 0.0, S0)
    assert np.all(np.isnan(out[0])) and np.all(np.isfinite(out[1:]))


def test_batch_equals_each_flow_alone_bitwise(ctx):
    rng = np.random.Generator(np.random.PCG64(5))
    n_s, s_max = 65, 16.0
    pf = frg.make_pflow(3, EXP, 48, 12, 1.0, 6.0, n_s, s_max)
    lam3 = rng.uniform(0.2, 2.0, 6)
    lam4 = rng.uniform(0.0, 6.0, 6)
    S0 = initial(rng, 6, n_s, s_max) + 0.2
    S, tr = gpu_solve(ctx, pf, lam3, lam4, -1.5, 10, S0)
    for r in (0, 3, 5):
        Sa, tra = gpu_solve(ctx, pf, lam3[r:r + 1], lam4[r:r + 1], -1.5, 10, S0[r:r + 1])
        assert np.array_equal(Sa[0], S[r]) and tra[0] == tr[r]


def test_host_memory_equals_device_bitwise(ctx):
    rng = np.random.Generator(np.random.PCG64(9))
    n_s, s_max = 40, 9.0
    pf = frg.make_pflow(4, LIT, 32, 8, 1.0, 6.0, n_s, s_max)
    lam3 = rng.uniform(0.2, 2.0, 3)
    lam4 = rng.uniform(0.0, 6.0, 3)
    S0 = initial(rng, 3, n_s, s_max) + 0.2
    S_d, tr_d = gpu_solve(ctx, pf, lam3, lam4, -1.0, 8, S0)
    S_h = S0.copy()
    tr_h = np.empty(3)
    frg.frg_pflow_solve(ctx, pf, lam3, lam4, -1.0, 8, S_h, tr_h, mem=frg.FRG_MEM_HOST)
    assert np.array_equal(S_h, S_d) and np.array_equal(tr_h, tr_d)
    r_d = gpu_rhs(ctx, pf, lam3, lam4, -0.4, S0)
    r_h = np.empty_like(S0)
    frg.frg_pflow_rhs(ctx, pf, lam3, lam4, -0.4, S0, r_h, mem=frg.FRG_MEM_HOST)
    assert np.array_equal(r_h, r_d)
    bad = S0.copy()
    bad[1] = -5.0
    with pytest.raises(frg.FrgError):
        frg.frg_pflow_rhs(ctx, pf, lam3, lam4, 0.0, bad, r_h, mem=frg.FRG_MEM_HOST)
    r_h2 = np.empty_like(S0)
    frg.frg_pflow_rhs(ctx, pf, lam3, lam4, 0.0, bad, r_h2, mem=frg.FRG_MEM_HOST, allow_domain=True)
    assert np.all(np.isnan(r_h2[1])) and np.all(np.isfinite(r_h2[[0, 2]]))


def test_bench_workload_two_steps(ctx):
    """The bench shape (64 flows, 256 nodes, 128 x 32 rule) for two RK4 steps,
    four flows checked against the oracle."""
    w = workloads.pflow_d3()
    print(f"[case] {w.name}, 2 steps", flush=True)
    pf = frg.make_pflow(w.d, w.reg, w.n_r, w.n_a, w.lam, w.kappa, w.n_s, w.s_max)
    h = w.t_end / w.n_steps
    got, tr = gpu_solve(ctx, pf, w.lam3, w.lam4, 2 * h, 2, w.sigma0)
    assert np.all(tr == 2 * h)
    sel = [0, 17, 40, 63]
    want, _ = oracle.pflow_solve(w.d, w.reg, w.lam, w.kappa, w.n_r, w.n_a, w.s_max, w.lam3[sel],
                                 w.lam4[sel], 2 * h, 2, w.sigma0[sel], threads=8)
    err = np.abs(got[sel] - want).max(axis=1) / np.abs(want).max(axis=1)
    print(f"  max rel err {err.max():.3e}")
    assert err.max() < RTOL


def test_bad_arguments(ctx):
    pf = frg.make_pflow(3, EXP, 16, 8, 1.0, 6.0, 17, 4.0)
    lam = np.ones(2)
    S = np.ones((2, 17))
    tr = np.empty(2)
    for bad in (frg.make_pflow(2, EXP, 16, 8, 1.0, 6.0, 17, 4.0),
                frg.make_pflow(3, EXP, 16, 8, 0.0, 6.0, 17, 4.0),
                frg.make_pflow(3, EXP, 16, 8, 1.0, 6.0, 1, 4.0),
                frg.make_pflow(3, EXP, 16, 8, 1.0, 6.0, 17, -1.0)):
        with pytest.raises(frg.FrgError):
            frg.frg_pflow_solve(ctx, bad, lam, lam, -1.0, 4, S, tr, mem=frg.FRG_MEM_HOST)
    with pytest.raises(frg.FrgError):
        frg.frg_pflow_solve(ctx, pf, lam, lam, 0.5, 4, S, tr, mem=frg.FRG_MEM_HOST)
    with pytest.raises(frg.FrgError):
        frg.frg_pflow_solve(ctx, pf, lam, lam, -1.0, 0, S, tr, mem=frg.FRG_MEM_HOST)


# 40 angular nodes (five per lane: angular nodes read from LDS, not registers);
# rows near the LDS limit: 6000 nodes (one launch per stage with 145 KB of LDS)
# and 6144 nodes with a 512 x 64 rule (too large for it: two launches, rows in LDS)
LDS_EDGE = [(3, EXP, 24, 40, 64, 9.0), (3, EXP, 32, 8, 6000, 50.0), (3, LIT, 512, 64, 6144, 60.0)]


@pytest.mark.parametrize("case", range(len(SHAPES) + 1 + len(LDS_EDGE)))
def test_fused_and_two_launch_stages_same_bits(ctx, case):
    """One launch per stage (every workgroup of a row redoes the previous
    stage's RK4 update and the prep for its row, state buffers alternating
    between launches), a diagram and a stage launch per stage, rows streamed
    from memory instead of LDS (two launches), and one, two (the default) or
    four flows per workgroup: the same bits, for solves with flows that stop
    at the domain boundary and for one right-hand side."""
    rng = np.random.Generator(np.random.PCG64(100 + case))
    steps = 12
    if case < len(SHAPES):
        d, reg, n_r, n_a, n_s, s_max = SHAPES[case]
        n_flows = 9
    elif case > len(SHAPES):
        d, reg, n_r, n_a, n_s, s_max = LDS_EDGE[case - len(SHAPES) - 1]
        n_flows, steps = 3, 2
    else:
        w = workloads.pflow_d3()
        d, reg, n_r, n_a, n_s, s_max = w.d, w.reg, w.n_r, w.n_a, w.n_s, w.s_max
        n_flows = 64
    print(f"[case] pflow fused vs two launches d={d} n_r={n_r} n_a={n_a} n_s={n_s} "
          f"flows={n_flows}", flush=True)
    pf = frg.make_pflow(d, reg, n_r, n_a, 1.0, 6.0, n_s, s_max)
    lam3 = rng.uniform(0.2, 2.5, n_flows)
    lam4 = rng.uniform(0.0, 6.0, n_flows)
    S0 = initial(rng, n_flows, n_s, s_max)
    S0[0] -= 2.0        # outside the domain at t = 0
    lam3[1] = 4.0       # driven towards the pole
    keys = ("pflow_fused", "tab_lds_nodes", "tab_rb")
    default = {k: frg.frg_tune_get(ctx, k) for k in keys}
    outs = []
    nodes = default["tab_lds_nodes"]
    try:
        # fused with the default rows per workgroup, two launches, streamed
        # rows, fused with one and with four flows per workgroup
        for fused, lds_nodes, rb in ((1, nodes, 0), (0, nodes, 0), (1, 2, 0), (1, nodes, 1),
                                     (1, nodes, 4)):
            frg.frg_tune_set(ctx, "pflow_fused", fused)
            frg.frg_tune_set(ctx, "tab_lds_nodes", lds_nodes)
            frg.frg_tune_set(ctx, "tab_rb", rb)
            S, tr = gpu_solve(ctx, pf, lam3, lam4, -0.1 * steps, steps, S0)
            r = np.empty_like(S0)
            frg.frg_pflow_rhs(ctx, pf, lam3, lam4, -0.3, S0, r, mem=frg.FRG_MEM_HOST,
                              allow_domain=True)
            outs.append((S, tr, r))
    finally:
        for k in keys:
            frg.frg_tune_set(ctx, k, default[k])
    print("  t_reached", outs[0][1][:4], f"{np.sum(outs[0][1] == -0.1 * steps)}/{n_flows} to t_end")
    assert outs[0][1][0] == 0.0
    for S, tr, r in outs[1:]:
        assert np.array_equal(tr, outs[0][1])
        assert np.array_equal(S, outs[0][0])
        assert np.array_equal(r, outs[0][2], equal_nan=True)
