"""The project's launch-shape autotuner on the GPU: tuning the persistent
uneven-set launch and two tensor grids changes no bit of any result, the
choices are written to the cache file, a second call with a tuned key does
not time candidates again, and a fresh context reloads the file."""
import os
import time

import numpy as np
import pytest

from paper_2607_24908_amd import frg, workloads

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def sets_on_device(sets):
    return [dict(quad=frg.make_quad(s.quad.d, s.quad.reg, s.quad.k, s.quad.q_max, s.quad.n_r,
                                    s.quad.n_a),
                 p=torch.as_tensor(s.p, device="cuda"), m2=torch.as_tensor(s.m2, device="cuda"),
                 out=torch.full((s.p.size,), float("nan"), dtype=torch.float64, device="cuda"))
            for s in sets]


GRIDS = [workloads.plain_d4(), workloads.scaleup_d3(n_p=256, n_m=512)]


def run_grids(ctx):
    outs = []
    for w in GRIDS:
        q = w.quad
        quad = frg.make_quad(q.d, q.reg, q.k, q.q_max, q.n_r, q.n_a)
        out = torch.full((w.n_integrals,), float("nan"), dtype=torch.float64, device="cuda")
        frg.frg_integrate_grid(ctx, quad, torch.as_tensor(w.p, device="cuda"),
                               torch.as_tensor(w.m2, device="cuda"), out)
        outs.append(out)
    torch.cuda.synchronize()
    return outs


def run_uneven(ctx, sets):
    d = sets_on_device(sets)
    t0 = time.perf_counter()
    frg.frg_integrate(ctx, d, flags=frg.FRG_PERSISTENT)
    torch.cuda.synchronize()
    return d, time.perf_counter() - t0


def test_autotuner_bitwise_cached_and_reloaded(tmp_path):
    print("[case] autotune uneven sets + two grids", flush=True)
    path = str(tmp_path / "frg_tune.txt")
    sets = workloads.uneven_sets(seed=0, n_sets=96)
    ctx = frg.frg_create(0)
    try:
        ref, _ = run_uneven(ctx, sets)  # default shapes
        ref_g = run_grids(ctx)
        frg.frg_autotune(ctx, 1, path)
        tuned, t_first = run_uneven(ctx, sets)  # times the candidates of this key
        for a, b in zip(tuned, ref):
            assert torch.equal(a["out"], b["out"])
        text = open(path).read()
        assert "persist " in text, text
        for a, b in zip(run_grids(ctx), ref_g):  # times the grid candidates
            assert torch.equal(a, b)
        text = open(path).read()
        assert text.count("\ngrid ") + text.startswith("grid ") >= 2, text
        stamp = os.stat(path).st_mtime_ns
        again, t_second = run_uneven(ctx, sets)  # tuned key: no timing
        for a, b in zip(again, ref):
            assert torch.equal(a["out"], b["out"])
        run_grids(ctx)
        assert os.stat(path).st_mtime_ns == stamp and open(path).read() == text
        print(f"first tuned call {t_first * 1e3:.1f} ms, second {t_second * 1e3:.1f} ms")
        assert t_second < t_first / 3
    finally:
        frg.frg_destroy(ctx)
    # a fresh context in tuning mode finds every key in the file: nothing is
    # timed or rewritten, and the results are the same bits
    ctx2 = frg.frg_create(0)
    try:
        frg.frg_autotune(ctx2, 1, path)
        got, t_fresh = run_uneven(ctx2, sets)
        for a, b in zip(got, ref):
            assert torch.equal(a["out"], b["out"])
        for a, b in zip(run_grids(ctx2), ref_g):
            assert torch.equal(a, b)
        assert os.stat(path).st_mtime_ns == stamp
        print(f"fresh context call {t_fresh * 1e3:.1f} ms")
    finally:
        frg.frg_destroy(ctx2)
