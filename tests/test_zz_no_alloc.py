"""The allocation-free variant of the persistent point-list launch
(frg_integrate_noalloc) against frg_integrate with FRG_PERSISTENT: the same
bits on two calls in a row (the second smaller), with FP64 and compensated
FP32 sets, its domain word, and the size limit of its scratch area."""
import numpy as np
import pytest

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


def sets_on_device(sets, prec=frg.FRG_PREC_FP64):
    return [dict(quad=frg.make_quad(s.quad.d, s.quad.reg, s.quad.k, s.quad.q_max, s.quad.n_r,
                                    s.quad.n_a, prec),
                 p=torch.as_tensor(s.p, device="cuda"), m2=torch.as_tensor(s.m2, device="cuda"),
                 out=torch.full((s.p.size,), float("nan"), dtype=torch.float64, device="cuda"),
                 err_est=(torch.zeros(s.p.size, dtype=torch.float64, device="cuda")
                          if prec == frg.FRG_PREC_FP32C else None))
            for s in sets]


@pytest.mark.parametrize("prec", [frg.FRG_PREC_FP64, frg.FRG_PREC_FP32C])
def test_noalloc_equals_persistent_two_calls(ctx, prec):
    for seed, n_sets, max_points in ((0, 256, 1024), (2, 40, 128)):
        print(f"[case] noalloc prec={prec} seed={seed} n_sets={n_sets}", flush=True)
        sets = workloads.uneven_sets(seed=seed, n_sets=n_sets, max_points=max_points)
        ref = sets_on_device(sets, prec)
        got = sets_on_device(sets, prec)
        frg.frg_integrate(ctx, ref, flags=frg.FRG_PERSISTENT)
        flag = torch.zeros(1, dtype=torch.int32, device="cuda")
        frg.frg_integrate_noalloc(ctx, got, domain_flag=flag)
        torch.cuda.synchronize()
        assert int(flag.item()) == 0
        for a, b in zip(got, ref):
            assert torch.equal(a["out"], b["out"]), f"seed {seed}"
            if prec == frg.FRG_PREC_FP32C:
                assert torch.equal(a["err_est"], b["err_est"]), f"seed {seed}"


def test_noalloc_domain_word_and_nan(ctx):
    print("[case] noalloc domain word", flush=True)
    quad = frg.make_quad(3, frg.FRG_REG_EXP, 1.0, 6.0, 64, 16)
    p = torch.tensor([0.5, 0.5, 1.0], dtype=torch.float64, device="cuda")
    m2 = torch.tensor([0.2, -1.5, 0.4], dtype=torch.float64, device="cuda")
    out = torch.zeros(3, dtype=torch.float64, device="cuda")
    ref = torch.zeros(3, dtype=torch.float64, device="cuda")
    flag = torch.zeros(1, dtype=torch.int32, device="cuda")
    frg.frg_integrate_noalloc(ctx, [dict(quad=quad, p=p, m2=m2, out=out)], domain_flag=flag)
    frg.frg_integrate(ctx, [dict(quad=quad, p=p, m2=m2, out=ref)], flags=frg.FRG_PERSISTENT)
    torch.cuda.synchronize()
    assert int(flag.item()) == 1
    o = out.cpu().numpy()
    assert np.isnan(o[1]) and np.isfinite(o[0]) and np.isfinite(o[2])
    assert torch.equal(out[[0, 2]], ref[[0, 2]])


def test_noalloc_rejects_calls_beyond_its_scratch(ctx):
    print("[case] noalloc size limit", flush=True)
    quad = frg.make_quad(3, frg.FRG_REG_LITIM, 1.0, 6.0, 32, 8)
    p = torch.full((1,), 0.5, dtype=torch.float64, device="cuda")
    m2 = torch.full((1,), 0.5, dtype=torch.float64, device="cuda")
    out = torch.zeros(1, dtype=torch.float64, device="cuda")
    many = [dict(quad=quad, p=p, m2=m2, out=out)] * 30000  # ~5 MB of descriptors
    with pytest.raises(frg.FrgError) as ei:
        frg.frg_integrate_noalloc(ctx, many)
    assert ei.value.code == frg.FRG_E_INVAL
    assert "scratch" in str(ei.value)
    # the library still works afterwards
    few = [dict(quad=quad, p=p, m2=m2, out=out)]
    frg.frg_integrate_noalloc(ctx, few)
    torch.cuda.synchronize()
    assert np.isfinite(out.item())
