"""Early merges of the private LDS histograms (Sect. 4.1's per-thread
histograms, summed into the shared result).  A wavefront empties its
workgroup's LDS counts and exact weighted limbs into the global accumulators
once it has claimed 2^flush_log2 candidate pairs since it last did; the
default (2^26) guards the 32-bit LDS counters and fires only on the largest
counts.  Lowering flush_log2 makes every launch take that path: the counts
and weighted sums must still equal the oracle's, and equal the default
launch bit for bit, for single counts, batches and pair lists."""
import numpy as np
import pytest

from paper_2301_12557_amd import synth
from helpers import check_case, gpu_count, note, oracle_count, assert_same, to_dev

pytestmark = pytest.mark.gpu

# merge once a wavefront has claimed 4 pairs: every work item of 4 or more
# pairs triggers one (sparse catalogues have items of only a few pairs)
FLUSH = 2


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2301_12557_amd import fcfc
    fcfc.load()


@pytest.mark.parametrize("weighted", [False, True])
def test_merges_smu_periodic(weighted):
    """(s, mu), line of sight z, periodic clustered box (C2 shape at 30k points)."""
    n = 30000
    x = synth.lognormal_box(n, 2000.0, synth.config_seed(2), ngrid=64)
    w1 = synth.uniform_weights(n, 0.5, 1.5, 77) if weighted else None
    kw = dict(kind="smu", edges1=synth.linear_edges(0, 200, 40), edges2=synth.mu_edges(100), box=2000.0, w1=w1)
    g, gw, st = check_case(f"merge smu w={weighted}", x, flush_log2=FLUSH, method="grid", **kw)
    note(f"flushes {st['flushes']} candidates {st['candidates']}")
    assert st["flushes"] > 0
    g0, gw0, st0 = gpu_count(x, **kw)
    assert st0["flushes"] == 0
    assert np.array_equal(g, g0)
    if weighted:
        assert np.array_equal(gw, gw0)


@pytest.mark.parametrize("weighted", [False, True])
def test_merges_spi_midpoint(weighted):
    """(s_perp, pi), mid-point line of sight, open survey shell (C3 shape): DD and DR."""
    d = synth.survey_shell(3000, 11)
    r = synth.survey_shell(6000, 12)
    wd = synth.uniform_weights(len(d), 0.5, 2.0, 13) if weighted else None
    wr = synth.uniform_weights(len(r), 0.5, 2.0, 14) if weighted else None
    e = synth.linear_edges(0, 200, 40)
    kw = dict(kind="spi", los="mid", edges1=e, edges2=e, box=0.0)
    _, _, st = check_case("merge C3-DD", d, w1=wd, flush_log2=FLUSH, **kw)
    assert st["flushes"] > 0
    _, _, st = check_case("merge C3-DR", d, r, w1=wd, w2=wr, flush_log2=FLUSH, **kw)
    assert st["flushes"] > 0


def test_merges_s_log_bins_and_histogram_copies():
    """s bins (log, hybrid table), periodic, with 2 and 4 LDS histogram copies:
    an early merge empties every copy."""
    n = 40000
    x = synth.lognormal_box(n, 3000.0, synth.config_seed(5), ngrid=64)
    kw = dict(kind="s", edges1=synth.log_edges(0.1, 50.0, 50), box=3000.0)
    o, _ = oracle_count(x, method="grid", **kw)
    for copies in (1, 2, 4):
        g, _, st = gpu_count(x, flush_log2=FLUSH, hist_copies=copies, **kw)
        assert st["flushes"] > 0
        assert_same(g, o, what=f"merge s copies={copies}")


def test_merges_smu_midpoint_open():
    """(s, mu) with the mid-point line of sight in an open box, weighted."""
    a = synth.survey_shell(2500, 21, rmin=300.0, rmax=700.0)
    wa = synth.uniform_weights(len(a), 0.5, 2.0, 22)
    _, _, st = check_case("merge smu mid", a, kind="smu", los="mid", edges1=synth.linear_edges(0, 100, 10),
                          edges2=synth.mu_edges(10), box=0.0, w1=wa, flush_log2=FLUSH)
    assert st["flushes"] > 0


@pytest.mark.parametrize("weighted", [False, True])
def test_merges_batched_mocks(weighted):
    """A batch of mocks of uneven size (C4 shape, scaled), replayed from a HIP
    graph: every histogram equals the oracle's, and the launch merged early."""
    import torch
    from paper_2301_12557_amd import fcfc
    L = 500.0
    sizes = [3000, 9000, 1500, 6000]
    xs = [synth.lognormal_box(n, L, 900 + i, ngrid=32) for i, n in enumerate(sizes)]
    ws = [synth.uniform_weights(n, 0.5, 1.5, 950 + i) for i, n in enumerate(sizes)] if weighted else None
    e1 = synth.linear_edges(0, 100, 20)
    e2 = synth.mu_edges(10)
    plan = fcfc.Plan("smu", e1, e2, box=L, n_hint=5000, flush_log2=FLUSH)
    dx = [to_dev(x) for x in xs]
    dw = [to_dev(w) for w in ws] if weighted else [None] * len(xs)
    note(f"merge batch sizes {sizes} weighted={weighted}")
    b = fcfc.Batch(plan, list(zip(dx, dw)))
    nb = plan.n1 * plan.n2
    out = torch.empty(len(xs) * nb, dtype=torch.int64, device="cuda")
    wout = torch.empty(len(xs) * nb, dtype=torch.float64, device="cuda") if weighted else None
    refs = [oracle_count(x, kind="smu", edges1=e1, edges2=e2, box=L, w1=ws[i] if weighted else None)
            for i, x in enumerate(xs)]
    for rep in range(3):
        out.fill_(-1)
        b.run(out, wout, use_graph=True)
        b.check()
        st = b.stats()
        assert st["flushes"] > 0, st
        got = out.cpu().numpy().reshape(len(xs), *plan.shape)
        gw = wout.cpu().numpy().reshape(len(xs), *plan.shape) if weighted else None
        for i, (o, ow) in enumerate(refs):
            assert_same(got[i], o, gw[i] if weighted else None, ow, what=f"merge batch mock {i} replay {rep}")
        torch.cuda.synchronize()
        _ = (dx[0] * 2.0).sum().item()
    b.close()
    plan.close()


def test_merges_pair_list():
    """DD, DR and RR of a survey patch in one weighted pair-list launch (the
    multi-tracer configuration), merging early: every histogram equals the oracle's."""
    import torch
    from paper_2301_12557_amd import fcfc
    d = synth.survey_shell(2500, 61)
    r = synth.survey_shell(5000, 62)
    wd = synth.uniform_weights(len(d), 0.5, 2.0, 63)
    wr = synth.uniform_weights(len(r), 0.5, 2.0, 64)
    e = synth.linear_edges(0, 120, 6)
    plan = fcfc.Plan("spi", e, e, los="mid", box=0.0, n_hint=5000, flush_log2=FLUSH)
    dd, dr = to_dev(d), to_dev(r)
    plan.fit_bounds([(dd, None), (dr, None)])
    pairs = [(0, 0), (0, 1), (1, 1)]
    b = fcfc.Batch(plan, [(dd, to_dev(wd)), (dr, to_dev(wr))], pairs=pairs)
    nb = plan.n1 * plan.n2
    out = torch.empty(3 * nb, dtype=torch.int64, device="cuda")
    wout = torch.empty(3 * nb, dtype=torch.float64, device="cuda")
    b.run(out, wout, use_graph=False)
    b.check()
    assert b.stats()["flushes"] > 0
    got = out.cpu().numpy().reshape(3, *plan.shape)
    gw = wout.cpu().numpy().reshape(3, *plan.shape)
    kw = dict(kind="spi", los="mid", edges1=e, edges2=e, box=0.0)
    refs = [oracle_count(d, w1=wd, **kw), oracle_count(d, r, w1=wd, w2=wr, **kw), oracle_count(r, w1=wr, **kw)]
    for q, (o, ow) in enumerate(refs):
        assert_same(got[q], o, gw[q], ow, what=f"merge pair list {pairs[q]}")
    b.close()
    plan.close()


def test_merges_full_size_c2_weighted():
    """C2 at full size (1,000,000 clustered points, weighted (s, mu) 40 x 100), the
    benchmark's count: with a merge every 2^14 claimed pairs the counts and the
    exact weighted sums are bit-identical to the default launch."""
    w = synth.workload(2, weighted=True)
    kw = dict(kind="smu", edges1=w["edges1"], edges2=w["edges2"], box=w["box"], w1=w["w1"])
    note("C2 full weighted, default merges")
    g0, gw0, st0 = gpu_count(w["x1"], **kw)
    note("C2 full weighted, merge every 2^14 pairs")
    g1, gw1, st1 = gpu_count(w["x1"], flush_log2=14, **kw)
    note(f"flushes {st1['flushes']}")
    assert st1["flushes"] > 1000
    assert np.array_equal(g0, g1)
    assert np.array_equal(gw0, gw1)
