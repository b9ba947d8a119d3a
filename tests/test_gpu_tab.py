"""Tabulated-propagator variant (frg_integrate_tab) against the FP64 oracle.

Bar: 1e-12 relative per result on smooth tables; on rough tables the
per-result bound of oracle.integrate_tab_bound.  A piecewise-linear row is
sensitive to its evaluation coordinate t = s/h: the kernel and the oracle
build their quadrature rules independently (nodes equal to about an ulp) and
round t differently, so t differs by about u t and a result moves by up to
u t |g_{k+1} - g_k| / G relative -- about 1e-10 for random rows of 2^20
nodes, whatever the formula; the bound sums that sensitivity over the terms
of each result.  The LDS-row and cache-streamed forms of the kernel do the
same arithmetic in the same order and must agree bit for bit; the segmented
form (long rows cut into LDS segments shared by four rows) sums each result
segment by segment: it agrees with them to rounding, and its bits do not
depend on how its work is split (which follows the momenta of the call)."""
import numpy as np
import pytest

import oracle
from paper_2607_24908_amd import frg, workloads

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

RTOL = 1e-12


@pytest.fixture(scope="module")
def ctx():
    assert torch.cuda.is_available()
    h = frg.frg_create(0)
    yield h
    torch.cuda.synchronize()
    frg.frg_destroy(h)


def dev(a):
    return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64), device="cuda")


def run_tab(ctx, q, g, s_max, p, lds_nodes=6144, pw=16, W=4, pairs=1, seg=0, rb=0, rW=16):
    frg.frg_tune_set(ctx, "tab_pairs", pairs)
    frg.frg_tune_set(ctx, "tab_seg", seg)
    frg.frg_tune_set(ctx, "tab_rb", rb)
    frg.frg_tune_set(ctx, "tab_rW", rW)
    frg.frg_tune_set(ctx, "tab_lds_nodes", lds_nodes)
    frg.frg_tune_set(ctx, "tab_pw", pw)
    frg.frg_tune_set(ctx, "tab_W", W)
    frg.frg_tune_set(ctx, "tab_spw", pw)
    frg.frg_tune_set(ctx, "tab_sW", W)
    quad = frg.make_quad(q.d, q.reg, q.k, q.q_max, q.n_r, q.n_a)
    out = torch.full((len(p) * g.shape[0],), float("nan"), dtype=torch.float64, device="cuda")
    frg.frg_integrate_tab(ctx, quad, dev(g), s_max, dev(p), out)
    torch.cuda.synchronize()
    return out.cpu().numpy().reshape(len(p), g.shape[0])


def want_of(q, g, s_max, p):
    return oracle.integrate_tab(q.d, q.reg, q.k, q.q_max, q.n_r, q.n_a, g, s_max, p, threads=8)


SHAPES = [(3, 0, 48, 12), (4, 1, 33, 5), (3, 0, 128, 32), (4, 0, 64, 16), (3, 1, 1, 1),
          (3, 0, 17, 40), (4, 0, 200, 3)]


@pytest.mark.parametrize("d,reg,n_r,n_a", SHAPES)
def test_tab_matches_oracle_and_forms_agree(ctx, d, reg, n_r, n_a):
    print(f"[case] tab d={d} reg={reg} {n_r}x{n_a}", flush=True)
    q = workloads.Quad(d, reg, 0.9, 5.4, n_r, n_a)
    rng = np.random.Generator(np.random.PCG64(n_r * 100 + n_a))
    p = np.concatenate([[0.0, 1e-9], 10 ** rng.uniform(-3, 1.2, 37)])
    s_max = 40.0   # momenta up to ~16: many s beyond the table (constant tail)
    g = workloads.tab_rows(7, 1537, s_max)
    got = run_tab(ctx, q, g, s_max, p)
    want = want_of(q, g, s_max, p)
    err = np.abs(got - want) / np.abs(want)
    print(f"max rel err {err.max():.3e}")
    assert err.max() < RTOL
    streamed = run_tab(ctx, q, g, s_max, p, lds_nodes=2, pw=5, W=3)
    assert np.array_equal(streamed, got)
    values = run_tab(ctx, q, g, s_max, p, pairs=0)  # rows in LDS as values
    assert np.array_equal(values, got)
    # one, two or four rows per workgroup (7 rows: ragged last groups)
    for pairs in (1, 0):
        for rb, rW in ((1, 16), (2, 16), (2, 3), (4, 8)):
            rows = run_tab(ctx, q, g, s_max, p, pairs=pairs, rb=rb, rW=rW)
            assert np.array_equal(rows, got), (pairs, rb, rW)
    segmented = run_tab(ctx, q, g, s_max, p, lds_nodes=2, seg=1)
    assert np.max(np.abs(segmented - want) / np.abs(want)) < RTOL
    assert np.all(np.abs(segmented - got) <= 1e-13 * np.abs(got))


@pytest.mark.parametrize("d,reg,n_r,n_a", [(3, 0, 1, 130), (4, 1, 3, 65), (3, 0, 5, 256),
                                           (5, 0, 70, 200), (3, 1, 9, 64), (4, 1, 260, 64),
                                           (4, 0, 300, 256)])
def test_tab_segmented_sort_shapes(ctx, d, reg, n_r, n_a):
    """The segmented form's term sort over rules whose angular nodes span one
    to four blocks of 64 lanes and whose radial nodes are fewer than, equal
    to or more than its four waves, on rows of 11 segments (the last one
    ragged): against the oracle, and within 1e-13 of the cache-streamed form.
    Terms are stored as byte pairs (i, j) up to 256 nodes each way, else as
    i n_a + j (260 radial nodes).  300 x 256 terms exceed its 16-bit term
    index: the call takes the cache-streamed form (the same bits)."""
    print(f"[case] segmented sort d={d} reg={reg} {n_r}x{n_a}", flush=True)
    q = workloads.Quad(d, reg, 0.9, 5.4, n_r, n_a)
    rng = np.random.Generator(np.random.PCG64(7 * n_r + n_a))
    p = np.concatenate([[0.0, 1e-9], 10 ** rng.uniform(-3, 1.2, 29)])
    s_max = 40.0
    g = workloads.tab_rows(5, 20483, s_max)
    seg = run_tab(ctx, q, g, s_max, p, lds_nodes=2, seg=1)
    cache = run_tab(ctx, q, g, s_max, p, lds_nodes=2, seg=0)
    want = want_of(q, g, s_max, p)
    err = np.abs(seg - want) / np.abs(want)
    print(f"max rel err {err.max():.3e}")
    assert err.max() < RTOL
    assert np.all(np.abs(seg - cache) <= 1e-13 * np.abs(cache))
    if n_r * n_a > 65536:
        assert np.array_equal(seg, cache)
    frg.frg_tune_set(ctx, "tab_seg", 0)


@pytest.mark.parametrize("n_rows,n_p", [(1, 1), (1, 3), (5, 17), (3, 1030)])
def test_tab_segmented_few_rows_and_momenta(ctx, n_rows, n_p):
    """The segmented form with one row (a batch of four holding one), a ragged
    batch, a single momentum (one lane of one wave) and more momenta than
    the lanes of a workgroup: against the oracle and the cache-streamed
    form."""
    print(f"[case] segmented rows={n_rows} momenta={n_p}", flush=True)
    q = workloads.Quad(3, 0, 1.0, 6.0, 48, 16)
    rng = np.random.Generator(np.random.PCG64(31 * n_rows + n_p))
    p = 10 ** rng.uniform(-3, np.log10(20.0), n_p)
    s_max = 676.0
    g = workloads.tab_rows(n_rows, 40961, s_max)
    seg = run_tab(ctx, q, g, s_max, p, lds_nodes=2, seg=1)
    cache = run_tab(ctx, q, g, s_max, p, lds_nodes=2, seg=0)
    sel = np.arange(0, n_p, max(1, n_p // 40))
    want = want_of(q, g, s_max, p[sel])
    err = np.abs(seg[sel] - want) / np.abs(want)
    print(f"max rel err {err.max():.3e}")
    assert err.max() < RTOL
    assert np.all(np.abs(seg - cache) <= 1e-13 * np.abs(cache))
    frg.frg_tune_set(ctx, "tab_seg", 0)


@pytest.mark.parametrize("n_s,form", [(4097, "lds"), (4097, "cache"), (4097, "seg"),
                                      (40961, "seg"), (1 << 20, "seg"), (1 << 20, "cache")])
def test_tab_rough_rows_within_coordinate_bound(ctx, n_s, form):
    """Seeded random positive rows (two decades, no smoothness) in LDS,
    cache-streamed and segmented, including rows of 2^20 nodes: every result
    within its bound."""
    print(f"[case] rough rows n_s={n_s} form={form}", flush=True)
    lds = form == "lds"
    rng = np.random.Generator(np.random.PCG64(n_s + lds))
    n_rows = 6 if n_s < 100000 else 2
    g = 10.0 ** rng.uniform(-1.0, 1.0, (n_rows, n_s))
    s_max = 676.0
    q = workloads.Quad(3, 0, 1.0, 6.0, 128, 32)
    p = np.concatenate([[0.0, 1e-6], 10 ** rng.uniform(-3.0, np.log10(20.0), 22)])
    got = run_tab(ctx, q, g, s_max, p, lds_nodes=6144 if lds else 2, seg=int(form == "seg"))
    want = want_of(q, g, s_max, p)
    bound = oracle.integrate_tab_bound(q.d, q.reg, q.k, q.q_max, q.n_r, q.n_a, g, s_max, p,
                                       threads=8)
    rel = np.abs(got - want) / want
    print(f"max rel err {rel.max():.3e}, max bound {bound.max():.3e}, "
          f"max err/bound {(rel / bound).max():.3f}")
    assert np.all(rel <= bound)


@pytest.mark.parametrize("seg", [0, 1])
def test_tab_long_rows_sampled(ctx, seg):
    """Rows of 2^20 nodes (8 MB each; read through the caches, or the
    segmented form) at the sizes of the bench workload, checked on a sample
    of momenta and rows."""
    w = workloads.tabulated_d3(n_s=1 << 20, n_p=64, n_rows=8)
    print(f"[case] {w.name} seg={seg}", flush=True)
    got = run_tab(ctx, w.quad, w.g, w.s_max, w.p, seg=seg)
    sel = np.arange(0, w.p.size, 7)
    want = want_of(w.quad, w.g, w.s_max, w.p[sel])
    err = np.abs(got[sel] - want) / want
    print(f"max rel err {err.max():.3e}")
    assert err.max() < RTOL


def test_tab_segmented_bits_independent_of_the_split(ctx):
    """The segmented form balances its work from the momenta of the call; a
    momentum's result must not depend on that: results for a subset of the
    momenta (a different split) equal those of the full call bit for bit, and
    the full bench-size call is checked against the oracle on a sample."""
    w = workloads.tabulated_d3(n_s=1 << 20, n_p=1024, n_rows=16)
    print(f"[case] segmented split independence {w.name}", flush=True)
    full = run_tab(ctx, w.quad, w.g, w.s_max, w.p, seg=1)
    for sel in (np.arange(0, w.p.size, 7), np.arange(w.p.size - 100, w.p.size), np.array([5])):
        part = run_tab(ctx, w.quad, w.g, w.s_max, w.p[sel], seg=1)
        assert np.array_equal(part, full[sel]), sel[:3]
    sel = np.arange(1, w.p.size, 61)
    want = want_of(w.quad, w.g, w.s_max, w.p[sel])
    err = np.abs(full[sel] - want) / want
    print(f"max rel err {err.max():.3e}")
    assert err.max() < RTOL
    # a momentum outside the domain: NaN in its row, FRG_E_DOMAIN on the host path
    p = np.array([0.3, -2.0, 7.0])
    frg.frg_tune_set(ctx, "tab_seg", 1)
    quad = frg.make_quad(w.quad.d, w.quad.reg, w.quad.k, w.quad.q_max, w.quad.n_r, w.quad.n_a)
    out = np.zeros(p.size * 2)
    rc = frg.frg_integrate_tab(ctx, quad, np.ascontiguousarray(w.g[:2]), w.s_max, p, out,
                               mem=frg.FRG_MEM_HOST, allow_domain=True)
    assert rc == frg.FRG_E_DOMAIN
    out = out.reshape(3, 2)
    assert np.all(np.isnan(out[1])) and np.all(np.isfinite(out[[0, 2]]))
    assert np.array_equal(out[[0, 2]], run_tab(ctx, w.quad, w.g[:2], w.s_max, p[[0, 2]], seg=1))
    frg.frg_tune_set(ctx, "tab_seg", 0)


def test_tab_auto_mode_picks_by_table_size(ctx):
    """Knob tab_seg = 2, the default: a table above 256 MiB takes the
    segmented form, a smaller one the cache-streamed form (the bits of
    tab_seg = 1 and 0); a context whose HBM budget cannot hold the segmented
    form's buffers takes the cache-streamed form instead of failing."""
    fresh = frg.frg_create(0)
    small = frg.frg_create(0, 1 << 20)
    try:
        assert frg.frg_tune_get(fresh, "tab_seg") == 2
        w = workloads.tabulated_d3(n_s=1 << 20, n_p=256, n_rows=36)  # 288 MiB
        print(f"[case] tabulated auto mode {w.name}", flush=True)
        seg = run_tab(ctx, w.quad, w.g, w.s_max, w.p, seg=1)
        cache = run_tab(ctx, w.quad, w.g, w.s_max, w.p, seg=0)
        assert not np.array_equal(seg, cache)  # the forms round differently
        assert np.array_equal(run_tab(ctx, w.quad, w.g, w.s_max, w.p, seg=2), seg)
        assert np.array_equal(run_tab(small, w.quad, w.g, w.s_max, w.p, seg=2), cache)
        # 30 rows: 240 MiB
        assert np.array_equal(run_tab(ctx, w.quad, w.g[:30], w.s_max, w.p, seg=2), cache[:, :30])
    finally:
        frg.frg_destroy(small)
        frg.frg_destroy(fresh)
        frg.frg_tune_set(ctx, "tab_seg", 0)


def test_tab_bench_shape_sampled(ctx):
    """The LDS-row bench workload (1024 momenta x 64 rows of 4096 nodes) on
    a sample of momenta against the oracle."""
    w = workloads.tabulated_d3()
    got = run_tab(ctx, w.quad, w.g, w.s_max, w.p)
    sel = np.arange(3, w.p.size, 97)
    want = want_of(w.quad, w.g, w.s_max, w.p[sel])
    assert np.max(np.abs(got[sel] - want) / want) < RTOL
    assert np.all(got > 0)


def test_tab_host_memory_and_domain(ctx):
    frg.frg_tune_set(ctx, "tab_lds_nodes", 6144)
    q = workloads.Quad(3, 0, 1.0, 6.0, 32, 8)
    quad = frg.make_quad(q.d, q.reg, q.k, q.q_max, q.n_r, q.n_a)
    g = workloads.tab_rows(3, 100, 50.0)
    p = np.array([0.1, -1.0, 2.0])
    out = np.zeros(p.size * 3)
    rc = frg.frg_integrate_tab(ctx, quad, g, 50.0, p, out, mem=frg.FRG_MEM_HOST, allow_domain=True)
    assert rc == frg.FRG_E_DOMAIN
    out = out.reshape(3, 3)
    assert np.all(np.isnan(out[1])) and np.all(np.isfinite(out[[0, 2]]))
    want = want_of(q, g, 50.0, p[[0, 2]])
    assert np.max(np.abs(out[[0, 2]] - want) / want) < RTOL
    dout = torch.zeros(9, dtype=torch.float64, device="cuda")
    frg.frg_integrate_tab(ctx, quad, dev(g), 50.0, dev(p), dout)
    torch.cuda.synchronize()
    assert np.array_equal(dout.cpu().numpy().reshape(3, 3)[[0, 2]], out[[0, 2]])


def test_tab_bad_arguments(ctx):
    q = frg.make_quad(3, 0, 1.0, 6.0, 16, 8)
    p = np.array([0.5])
    out = np.zeros(4)
    for g, s_max in [(np.ones((4, 1)), 1.0), (np.ones((4, 3)), 0.0), (np.ones((4, 3)), np.inf)]:
        with pytest.raises(frg.FrgError) as ei:
            frg.frg_integrate_tab(ctx, q, g, s_max, p, out, mem=frg.FRG_MEM_HOST)
        assert ei.value.code == frg.FRG_E_INVAL
    q32 = frg.make_quad(3, 0, 1.0, 6.0, 16, 8, frg.FRG_PREC_FP32C)
    with pytest.raises(frg.FrgError):
        frg.frg_integrate_tab(ctx, q32, np.ones((4, 3)), 1.0, p, out, mem=frg.FRG_MEM_HOST)
    # empty problems are no-ops
    frg.frg_integrate_tab(ctx, q, np.ones((0, 3)), 1.0, p, out, mem=frg.FRG_MEM_HOST)
