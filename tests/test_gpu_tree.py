"""The k-d tree variant (Sect. 2.2, counted through the dual-tree work list of
Sect. 3.1) against the oracle: every separation kind and line of sight on
open survey-like boxes, auto and cross, weighted and not, leaf sizes 32..128,
ragged and degenerate catalogues, and bit-for-bit equality with the grid on
larger catalogues (counts and exact weighted sums)."""
import numpy as np
import pytest

from paper_2301_12557_amd import synth
from helpers import check_case, gpu_count, note, assert_same, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2301_12557_amd import fcfc
    fcfc.load()


E40 = synth.linear_edges(0, 200, 40)


@pytest.mark.parametrize("leaf", [32, 77, 128])
@pytest.mark.parametrize("weighted", [False, True])
def test_tree_c3_shape_dd_dr(leaf, weighted):
    """(s_perp, pi) 40 x 40, mid-point line of sight, survey shell (C3 shape): DD and DR."""
    d = synth.survey_shell(3000, 31)
    r = synth.survey_shell(7000, 32)
    wd = synth.uniform_weights(len(d), 0.5, 2.0, 33) if weighted else None
    wr = synth.uniform_weights(len(r), 0.5, 2.0, 34) if weighted else None
    kw = dict(kind="spi", los="mid", edges1=E40, edges2=E40, box=0.0, tree_leaf=leaf)
    _, _, st = check_case(f"tree C3 DD leaf={leaf}", d, w1=wd, **kw)
    assert st["cells"] == -(-len(d) // leaf)
    check_case(f"tree C3 DR leaf={leaf}", d, r, w1=wd, w2=wr, **kw)


@pytest.mark.parametrize("kind,los", [("s", "z"), ("smu", "z"), ("smu", "mid"), ("spi", "z")])
def test_tree_other_kinds(kind, los):
    """s, (s, mu) along z and mid-point, (s_perp, pi) along z, on a shell patch."""
    a = synth.survey_shell(2500, 41, rmin=300.0, rmax=700.0)
    b = synth.survey_shell(4000, 42, rmin=300.0, rmax=700.0)
    wa = synth.uniform_weights(len(a), 0.5, 2.0, 43)
    wb = synth.uniform_weights(len(b), 0.5, 2.0, 44)
    e1 = synth.linear_edges(0, 120, 12)
    e2 = synth.mu_edges(10) if kind == "smu" else (synth.linear_edges(0, 80, 8) if kind == "spi" else None)
    kw = dict(kind=kind, los=los, edges1=e1, edges2=e2, box=0.0, tree_leaf=128)
    check_case(f"tree {kind} {los} auto", a, w1=wa, **kw)
    check_case(f"tree {kind} {los} cross", a, b, w1=wa, w2=wb, **kw)


def test_tree_log_bins_clustered():
    """log s bins (several edges per table entry near s = 0) on a clustered box
    counted as an open catalogue."""
    x = synth.lognormal_box(20000, 500.0, 51, ngrid=32) + 10.0
    check_case("tree s log", x, kind="s", edges1=synth.log_edges(0.1, 40.0, 30), box=0.0, tree_leaf=64)


def test_tree_degenerate_catalogues():
    """Empty, single, fewer points than a leaf, one more than a leaf, and many
    coincident points (FP32 sort keys all equal)."""
    rng = np.random.default_rng(61)
    kw = dict(kind="spi", los="mid", edges1=E40, edges2=E40, box=0.0, tree_leaf=64)
    base = synth.survey_shell(500, 62)
    for n in (1, 63, 64, 65, 129):
        check_case(f"tree n={n}", base[:n], **kw)
    dup = np.repeat(base[:5], 40, axis=0)
    dup[::7] += rng.normal(0, 1e-3, (len(dup[::7]), 3))
    check_case("tree duplicates", dup, base[:100], **kw)
    g, _, _ = gpu_count(base[:0], base, **kw)
    assert g.sum() == 0


def test_tree_sparse_leaves_widen_the_bands():
    """A catalogue so sparse that leaves span hundreds of Mpc: the FP32 bands are
    rebuilt for the leaf extent and the counts stay exact."""
    rng = np.random.default_rng(71)
    x = rng.uniform(1000.0, 3000.0, (600, 3))
    x[:300] = synth.survey_shell(300, 72)
    e = synth.linear_edges(0, 300, 30)
    _, _, st = check_case("tree sparse", x, kind="spi", los="mid", edges1=e, edges2=e, box=0.0, tree_leaf=128)
    note(f"band {st['band_d2_rel']:.3g}")


def test_tree_midpoint_knife_edges():
    """The constructed mid-point knife-edge pairs of the grid test, through the tree."""
    from test_gpu_parity import _midpoint_pairs
    e = synth.linear_edges(0, 200, 40)
    a, b = _midpoint_pairs(e, e, 16, 5)
    check_case("tree mid knife spi", a, b, kind="spi", los="mid", edges1=e, edges2=e, box=0.0, tree_leaf=128)
    check_case("tree mid knife smu", a, b, kind="smu", los="mid", edges1=synth.linear_edges(0, 282, 47),
               edges2=synth.mu_edges(20), box=0.0, tree_leaf=32)


@pytest.mark.parametrize("weighted", [False, True])
def test_tree_equals_grid_c3_scaled(weighted):
    """C3 at 1/20 (100,000 data, 400,000 randoms; weighted (s_perp, pi) 40 x 40,
    mid-point): DD and DR through the tree equal the grid's bit for bit."""
    w = synth.workload(3, scale=0.05, weighted=weighted)
    d, r = w["x1"], w["x2"][:400_000]
    wd = w["w1"]
    wr = w["w2"][:400_000] if weighted else None
    kw = dict(kind="spi", los="mid", edges1=w["edges1"], edges2=w["edges2"], box=0.0)
    for name, args in (("DD", (d, None, wd, None)), ("DR", (d, r, wd, wr))):
        x1, x2, w1, w2 = args
        gg, gw, sg = gpu_count(x1, x2, w1=w1, w2=w2, **kw)
        tg, tw, stt = gpu_count(x1, x2, w1=w1, w2=w2, tree_leaf=128, **kw)
        note(f"C3/20 {name}: grid {sg['kernel_ms']:.2f} ms {sg['candidates']} cand, "
             f"tree {stt['kernel_ms']:.2f} ms {stt['candidates']} cand, {stt['items']} items")
        assert np.array_equal(gg, tg), name
        if weighted:
            assert np.array_equal(gw, tw), name


def test_tree_refusals():
    """Trees are for open boxes; batches and triangle counts take grid plans."""
    from paper_2301_12557_amd import fcfc
    with pytest.raises(fcfc.FcfcError):
        fcfc.Plan("s", E40, box=1000.0, tree_leaf=128)
    plan = fcfc.Plan("s", synth.linear_edges(0, 30, 3), box=0.0, tree_leaf=64)
    x = to_dev(synth.survey_shell(300, 81))
    plan.fit_bounds([(x, None)])
    with pytest.raises(fcfc.FcfcError):
        fcfc.Batch(plan, [(x, None)])
    c = plan.build_cells(x)
    with pytest.raises(fcfc.FcfcError):
        plan.count_triplets(c)
    c.close()
    plan.close()
