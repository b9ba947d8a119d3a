"""Boundary behaviour of the C ABI on the GPU: the domain status of
asynchronous device calls, concurrent persistent launches on two streams,
graph replays keyed on the full set descriptors, tearing down a context
with flows still waiting for admission, and the HBM budget of synchronous
calls."""
import numpy as np
import pytest

import oracle
from paper_2607_24908_amd import frg, workloads

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    h = frg.frg_create(0)
    yield h
    torch.cuda.synchronize()
    frg.frg_destroy(h)


def dev(a):
    return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64), device="cuda")


def sets_on_device(sets, prec=frg.FRG_PREC_FP64):
    return [dict(quad=frg.make_quad(s.quad.d, s.quad.reg, s.quad.k, s.quad.q_max, s.quad.n_r,
                                    s.quad.n_a, prec),
                 p=dev(s.p), m2=dev(s.m2),
                 out=torch.full((s.p.size,), float("nan"), dtype=torch.float64, device="cuda"))
            for s in sets]


def test_device_domain_status_per_stream(ctx):
    """A device call with points outside the domain returns FRG_OK (it is
    asynchronous); frg_stream_status of its stream reports FRG_E_DOMAIN once,
    another stream reports nothing, and the good points match the oracle."""
    print("[case] device domain status", flush=True)
    quad = frg.make_quad(3, frg.FRG_REG_EXP, 1.0, 6.0, 64, 16)
    p = np.array([0.5, 0.7, 0.5, 2.0, 0.1])
    m2 = np.array([0.1, -1.0, -2.0, 0.3, 1.0])
    s1 = torch.cuda.Stream()
    s2 = torch.cuda.Stream()
    assert frg.frg_stream_status(ctx, s1) == frg.FRG_OK
    assert frg.frg_stream_status(ctx, s2) == frg.FRG_OK
    with torch.cuda.stream(s1):
        P, M = dev(p), dev(m2)
        out = torch.zeros(5, dtype=torch.float64, device="cuda")
        assert frg.frg_integrate(ctx, [dict(quad=quad, p=P, m2=M, out=out)], stream=s1,
                                 flags=frg.FRG_PERSISTENT) == frg.FRG_OK
    assert frg.frg_stream_status(ctx, s2) == frg.FRG_OK
    assert frg.frg_stream_status(ctx, s1, allow_domain=True) == frg.FRG_E_DOMAIN
    assert frg.frg_stream_status(ctx, s1) == frg.FRG_OK  # cleared
    o = out.cpu().numpy()
    assert np.isnan(o[1]) and np.isnan(o[2])
    want = oracle.integrate(3, 0, 1.0, 6.0, 64, 16, p[[0, 3, 4]], m2[[0, 3, 4]])
    assert np.max(np.abs(o[[0, 3, 4]] - want) / want) < 1e-12
    # tensor grid on the device: the same record
    g = torch.zeros(5, dtype=torch.float64, device="cuda")
    with torch.cuda.stream(s2):
        frg.frg_integrate_grid(ctx, quad, dev(p[:1]), dev(m2), g, stream=s2)
    assert frg.frg_stream_status(ctx, s2, allow_domain=True) == frg.FRG_E_DOMAIN
    assert frg.frg_stream_status(ctx, s1) == frg.FRG_OK


def test_two_streams_persistent_equal_serial(ctx):
    """Two persistent launches in flight on different streams (each with its
    own work-list counter) give the bits of the same launches run one after
    the other."""
    print("[case] two streams persistent", flush=True)
    sa = workloads.uneven_sets(seed=3, n_sets=48)
    sb = workloads.uneven_sets(seed=4, n_sets=48)
    ref_a, ref_b = sets_on_device(sa), sets_on_device(sb)
    frg.frg_integrate(ctx, ref_a, flags=frg.FRG_PERSISTENT)
    frg.frg_integrate(ctx, ref_b, flags=frg.FRG_PERSISTENT)
    torch.cuda.synchronize()
    s1 = torch.cuda.Stream()
    s2 = torch.cuda.Stream()
    for flags in (frg.FRG_PERSISTENT, frg.FRG_PERSISTENT | frg.FRG_GRAPH):
        for rep in range(3):
            a, b = sets_on_device(sa), sets_on_device(sb)
            torch.cuda.synchronize()
            for _ in range(2):  # queue several launches on both streams
                frg.frg_integrate(ctx, a, flags=flags, stream=s1)
                frg.frg_integrate(ctx, b, flags=flags, stream=s2)
            torch.cuda.synchronize()
            for x, y in zip(a, ref_a):
                assert torch.equal(x["out"], y["out"]), f"stream 1, flags {flags}, rep {rep}"
            for x, y in zip(b, ref_b):
                assert torch.equal(x["out"], y["out"]), f"stream 2, flags {flags}, rep {rep}"


def test_graph_follows_fp32c_knobs(ctx):
    """A graph replay after frg_tune_set of the FP32C routing knobs equals the
    eager call with the new knobs (the capture is keyed on the descriptors)."""
    print("[case] graph vs fp32c knob", flush=True)
    sets = workloads.uneven_sets(seed=5, n_sets=24, max_points=256)
    old = frg.frg_tune_get(ctx, "fp32c_flag_ppb")
    try:
        outs = []
        for ppb in (100, 0, 100):
            frg.frg_tune_set(ctx, "fp32c_flag_ppb", ppb)
            g = sets_on_device(sets, frg.FRG_PREC_FP32C)
            e = sets_on_device(sets, frg.FRG_PREC_FP32C)
            frg.frg_integrate(ctx, g, flags=frg.FRG_PERSISTENT | frg.FRG_GRAPH)
            frg.frg_integrate(ctx, g, flags=frg.FRG_PERSISTENT | frg.FRG_GRAPH)
            frg.frg_integrate(ctx, e, flags=frg.FRG_PERSISTENT)
            torch.cuda.synchronize()
            for x, y in zip(g, e):
                assert torch.equal(x["out"], y["out"]), f"ppb {ppb}"
            outs.append(torch.cat([x["out"] for x in g]))
        # threshold 0 sends every point to FP64: the results differ from FP32
        assert not torch.equal(outs[0], outs[1])
        assert torch.equal(outs[0], outs[2])
    finally:
        frg.frg_tune_set(ctx, "fp32c_flag_ppb", old)


def test_graph_cache_is_bounded(ctx):
    """More distinct batches than the graph cache holds: every replay still
    equals the eager result (least recently used captures are dropped)."""
    print("[case] graph cache bound", flush=True)
    base = workloads.uneven_sets(seed=6, n_sets=4, max_points=64)
    ref = sets_on_device(base)
    frg.frg_integrate(ctx, ref, flags=frg.FRG_PERSISTENT)
    torch.cuda.synchronize()
    for rep in range(2):
        for i in range(40):  # distinct output pointers: distinct captures
            d = sets_on_device(base)
            frg.frg_integrate(ctx, d, flags=frg.FRG_PERSISTENT | frg.FRG_GRAPH)
            torch.cuda.synchronize()
            for x, y in zip(d, ref):
                assert torch.equal(x["out"], y["out"]), f"rep {rep} batch {i}"


def test_destroy_with_flows_waiting_for_admission():
    """frg_destroy while flows wait in the queue (one slot, budget for one
    flow at a time) returns cleanly; a later context works."""
    import os
    print("[case] destroy with queued flows", flush=True)
    lpa = frg.make_lpa(d=3, N=2, n_grid=256)
    old = os.environ.get("FRG_SERVER_SLOTS")
    os.environ["FRG_SERVER_SLOTS"] = "1"
    try:
        for budget in (0, frg.frg_flow_footprint(lpa) + 16):
            c = frg.frg_create(0, budget)
            outs = [np.zeros(256) for _ in range(12)]
            for o in outs:
                frg.frg_submit(c, frg.make_request(lpa, 6.0, 0.05, -9.0, 1e-8, 1e-10, o))
            frg.frg_destroy(c)
    finally:
        if old is None:
            os.environ.pop("FRG_SERVER_SLOTS", None)
        else:
            os.environ["FRG_SERVER_SLOTS"] = old
    c = frg.frg_create(0)
    U = np.zeros(256)
    t = frg.frg_submit(c, frg.make_request(lpa, 6.0, 0.05, -1.0, 1e-8, 1e-10, U))
    import time
    for _ in range(20000):
        rc, res = frg.frg_poll(c, t)
        if rc == frg.FRG_OK:
            break
        time.sleep(0.001)
    assert rc == frg.FRG_OK and res.status == frg.FRG_OK
    frg.frg_destroy(c)


def test_hbm_budget_bounds_synchronous_calls(ctx):
    """A context created with a 1 MiB budget: a host-memory call whose staging
    needs more returns FRG_E_NOMEM and leaves its output untouched; calls that
    fit run and equal those of an unlimited context bit for bit."""
    print("[case] hbm budget of synchronous calls", flush=True)
    quad = frg.make_quad(3, frg.FRG_REG_EXP, 1.0, 6.0, 32, 8)
    rng = np.random.Generator(np.random.PCG64(8))
    small = frg.frg_create(0, 1 << 20)
    try:
        n_big = 100_000  # p, m2 in, out back: 2.4 MB of staging
        p = rng.uniform(0.0, 3.0, n_big)
        m2 = rng.uniform(-0.5, 2.0, n_big)
        out = np.full(n_big, 7.0)
        with pytest.raises(frg.FrgError) as ei:
            frg.frg_integrate(small, [dict(quad=quad, p=p, m2=m2, out=out)], mem=frg.FRG_MEM_HOST)
        assert ei.value.code == frg.FRG_E_NOMEM
        assert np.all(out == 7.0)
        # a call that fits, on the same context, and the same call unlimited
        got = np.zeros(2000)
        want = np.zeros(2000)
        frg.frg_integrate(small, [dict(quad=quad, p=p[:2000], m2=m2[:2000], out=got)],
                          mem=frg.FRG_MEM_HOST)
        frg.frg_integrate(ctx, [dict(quad=quad, p=p[:2000], m2=m2[:2000], out=want)],
                          mem=frg.FRG_MEM_HOST)
        assert np.array_equal(got, want)
    finally:
        frg.frg_destroy(small)
