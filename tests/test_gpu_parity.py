"""GPU parity: the HIP library against the FP64 CPU oracle, bin by bin.

Integer counts must match bit for bit; weighted counts within 1e-12 relative
(the exact fixed-point accumulation gives identical FP64 values)."""
import itertools
import json
import os

import numpy as np
import pytest

from paper_2301_12557_amd import synth
from helpers import check_case, gpu_count, note, oracle_count, assert_same, to_dev

pytestmark = pytest.mark.gpu
HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2301_12557_amd import fcfc
    fcfc.load()


def _hand_cases():
    with open(os.path.join(HERE, "golden", "hand_cases.json")) as f:
        return json.load(f)["cases"]


@pytest.mark.parametrize("case", _hand_cases(), ids=lambda c: c["name"])
def test_hand_cases_gpu(case):
    e2 = case.get("edges2")
    if e2 == "mu100":
        e2 = synth.mu_edges(100)
    x1 = np.array(case["x1"], dtype=np.float64)
    x2 = np.array(case["x2"], dtype=np.float64) if "x2" in case else None
    w1 = np.array(case["w1"]) if "w1" in case else None
    rmax = float(case["edges1"][-1]) if case["kind"] != "spi" else float(np.hypot(case["edges1"][-1], e2[-1]))
    if case["box"] > 0 and rmax > case["box"] / 2:
        # the library requires the prune radius to be at most L/2 (the minimum image is then the
        # only image in range); such a plan is rejected with FCFC_ERANGE
        from paper_2301_12557_amd import fcfc
        with pytest.raises(fcfc.FcfcError) as ei:
            gpu_count(x1, x2, kind=case["kind"], los=case["los"], box=case["box"], edges1=case["edges1"], edges2=e2)
        assert ei.value.name == "FCFC_ERANGE"
        return
    check_case(case["name"], x1, x2, kind=case["kind"], los=case["los"], box=case["box"],
               edges1=case["edges1"], edges2=e2, w1=w1, w2=(w1 if (w1 is not None and x2 is not None) else None))


def _lattice(n, a):
    g = np.arange(n) * a
    return np.array(list(itertools.product(g, g, g)), dtype=np.float64)


@pytest.mark.parametrize("a", [1.0, 0.3, 0.1])
def test_lattice_knife_edges(a):
    """Lattice pairs sit exactly on (a = 1) or within rounding of (a = 0.3, 0.1) the bin edges:
    the FP64 recheck must reproduce the oracle."""
    n = 9
    x = _lattice(n, a)
    L = n * a
    x = np.minimum(x, np.nextafter(L, 0))
    e = np.arange(0, 5) * a
    check_case(f"lattice s a={a}", x, kind="s", edges1=e, box=L)
    check_case(f"lattice smu a={a}", x, kind="smu", edges1=e, edges2=synth.mu_edges(8), box=L)
    check_case(f"lattice spi a={a}", x, kind="spi", edges1=e[:4], edges2=e[:4], box=L)


@pytest.mark.parametrize("weighted", [False, True])
def test_c1_full_size(weighted):
    """Config C1 at full size: 20,000 uniform points, L = 1000, 40 linear s bins."""
    w = synth.workload(1, weighted=weighted)
    check_case("C1", w["x1"], kind="s", edges1=w["edges1"], box=w["box"], w1=w["w1"])


@pytest.mark.parametrize("weighted", [False, True])
def test_c2_scaled(weighted):
    """Config C2 shape (lognormal, (s,mu) 40 x 100, LOS z, periodic L = 2000) at 30k points."""
    n = 30000
    x = synth.lognormal_box(n, 2000.0, synth.config_seed(2), ngrid=64)
    w1 = synth.uniform_weights(n, 0.5, 1.5, 77) if weighted else None
    check_case("C2-30k", x, kind="smu", edges1=synth.linear_edges(0, 200, 40), edges2=synth.mu_edges(100),
               box=2000.0, w1=w1)


@pytest.mark.parametrize("weighted", [False, True])
def test_c3_scaled(weighted):
    """Config C3 shape (survey shell, (s_perp,pi) 40 x 40, mid-point LOS, open box): DD, DR, RR."""
    nd, nr = 3000, 6000
    d = synth.survey_shell(nd, 11)
    r = synth.survey_shell(nr, 12)
    wd = synth.uniform_weights(nd, 0.5, 2.0, 13) if weighted else None
    wr = synth.uniform_weights(nr, 0.5, 2.0, 14) if weighted else None
    e = synth.linear_edges(0, 200, 40)
    kw = dict(kind="spi", los="mid", edges1=e, edges2=e, box=0.0)
    check_case("C3-DD", d, w1=wd, **kw)
    check_case("C3-DR", d, r, w1=wd, w2=wr, **kw)
    check_case("C3-RR", r, w1=wr, **kw)


def test_c5_scaled():
    """Config C5 shape: log s bins [0.1, 50) (hybrid table), periodic L = 3000, clustered."""
    n = 60000
    x = synth.lognormal_box(n, 3000.0, synth.config_seed(5), ngrid=64)
    check_case("C5-60k", x, kind="s", edges1=synth.log_edges(0.1, 50.0, 50), box=3000.0)


@pytest.mark.parametrize("kind,los,box", [("s", "z", 0.0), ("smu", "z", 0.0), ("smu", "mid", 0.0),
                                          ("spi", "z", 0.0), ("spi", "z", 130.0), ("smu", "z", 120.0)])
def test_cross_counts(kind, los, box):
    rng = np.random.default_rng(3)
    if box > 0:
        a = rng.random((1500, 3)) * box
        b = rng.random((1100, 3)) * box
    else:
        a = synth.survey_shell(1500, 5, rmin=200.0, rmax=320.0)
        b = synth.survey_shell(1100, 6, rmin=200.0, rmax=320.0)
    e1 = np.array([0.0, 3.0, 7.5, 12.0, 20.0, 31.0, 45.0])
    e2 = synth.mu_edges(10) if kind == "smu" else (np.array([0.0, 4.0, 10.0, 25.0, 40.0]) if kind == "spi" else None)
    w1 = synth.uniform_weights(len(a), 0.5, 1.5, 1)
    w2 = synth.uniform_weights(len(b), 0.5, 1.5, 2)
    check_case(f"cross {kind}/{los}/{box}", a, b, kind=kind, los=los, box=box, edges1=e1, edges2=e2, w1=w1, w2=w2)


@pytest.mark.parametrize("sa,sb", [(1e300, 1e-300), (1e-300, 1e300), (3.0, 0.25)])
def test_cross_weights_far_from_one(sa, sb):
    """Weights of very different magnitudes (pair weights near 1): with A weights
    near 1e300 the kernel must not pre-scale them by 2^S (that would overflow)
    and still sum exactly; with B weights near 1e300 it may."""
    rng = np.random.default_rng(8)
    a = rng.random((1200, 3)) * 120.0
    b = rng.random((900, 3)) * 120.0
    e1 = np.array([0.0, 3.0, 7.5, 12.0, 20.0, 31.0, 45.0])
    w1 = sa * synth.uniform_weights(len(a), 1.0, 2.0, 3)
    w2 = sb * synth.uniform_weights(len(b), 1.0, 2.0, 4)
    check_case(f"cross weights {sa:g}/{sb:g}", a, b, kind="smu", los="z", box=120.0, edges1=e1,
               edges2=synth.mu_edges(10), w1=w1, w2=w2)


def test_weighted_sums_bit_exact():
    """Both sides round the same exact sum of FP64 pair weights once, so the
    weighted histograms agree bit for bit (not just within 1e-12)."""
    w = synth.workload(1, weighted=True)
    g, gw, _ = gpu_count(w["x1"], kind="s", edges1=w["edges1"], box=w["box"], w1=w["w1"])
    o, ow = oracle_count(w["x1"], kind="s", edges1=w["edges1"], box=w["box"], w1=w["w1"])
    assert np.array_equal(g, o) and np.array_equal(gw, ow)
    rng = np.random.default_rng(9)
    a = synth.survey_shell(1500, 11, rmin=200.0, rmax=320.0)
    b = synth.survey_shell(1200, 12, rmin=200.0, rmax=320.0)
    wa = 1e300 * rng.uniform(1.0, 2.0, len(a))
    wb = 1e-300 * rng.uniform(1.0, 2.0, len(b))
    kw = dict(kind="spi", los="mid", edges1=np.array([0.0, 4.0, 9.0, 20.0, 33.0]),
              edges2=np.array([0.0, 5.0, 12.0, 30.0]), box=0.0)
    g, gw, _ = gpu_count(a, b, w1=wa, w2=wb, **kw)
    o, ow = oracle_count(a, b, w1=wa, w2=wb, **kw)
    assert np.array_equal(g, o) and np.array_equal(gw, ow)


def test_empty_and_tiny():
    e = np.array([0.0, 1.0, 2.0, 5.0])
    for n in (0, 1, 2, 3):
        x = np.random.default_rng(n).random((n, 3)) * 4.0
        check_case(f"tiny n={n}", x, kind="s", edges1=e, box=10.0)
        check_case(f"tiny open n={n}", x, kind="smu", edges1=e, edges2=synth.mu_edges(4), box=0.0)
    y = np.random.default_rng(9).random((5, 3)) * 4.0
    check_case("cross with empty", np.zeros((0, 3)), y, kind="s", edges1=e, box=10.0)


def test_degenerate_catalogues():
    """Coincident points (d = 0: s-bin 0, mu = 0, every pair through the FP64 recheck
    of tiny separations), and one dense clump inside a single cell (tiles within a
    cell, B pieces split by b_chunk, the same-row rule inside one cell)."""
    rng = np.random.default_rng(31)
    x = np.concatenate([np.full((600, 3), 7.25), rng.random((900, 3)) * 20.0])
    e = np.array([0.0, 0.5, 2.0, 4.0, 6.0])
    check_case("coincident smu", x, kind="smu", edges1=e, edges2=synth.mu_edges(5), box=20.0)
    check_case("coincident s open", x, kind="s", edges1=e, box=0.0)
    clump = 50.0 + rng.normal(0.0, 0.3, (12000, 3))
    bg = rng.random((3000, 3)) * 100.0
    y = np.concatenate([clump, bg])
    e2 = np.array([0.0, 0.2, 0.5, 1.0, 3.0, 8.0])
    check_case("dense clump", y, kind="smu", edges1=e2, edges2=synth.mu_edges(4), box=100.0, method="grid")
    check_case("dense clump small chunks", y, kind="s", edges1=e2, box=100.0, method="grid", b_chunk=300)


def test_histogram_size_limits():
    """The largest unweighted histogram the LDS holds counts exactly; a weighted one
    too large for the LDS limbs is refused with FCFC_ERANGE (nothing is counted)."""
    from paper_2301_12557_amd import fcfc
    x = np.random.default_rng(4).random((3000, 3)) * 60.0
    e1 = synth.linear_edges(0, 20, 240)
    check_case("24000 bins", x, kind="smu", edges1=e1, edges2=synth.mu_edges(100), box=60.0)
    w = np.random.default_rng(5).uniform(0.5, 1.5, len(x))
    with pytest.raises(fcfc.FcfcError) as ei:
        gpu_count(x, kind="smu", edges1=e1, edges2=synth.mu_edges(100), box=60.0, w1=w)
    assert ei.value.name == "FCFC_ERANGE"


def test_tuning_sweep_small():
    """Random small problems under many tuning settings: all must match the oracle."""
    rng = np.random.default_rng(2024)
    for t in range(24):
        n = int(rng.integers(50, 600))
        kind = ["s", "smu", "spi"][t % 3]
        periodic = bool(rng.integers(0, 2))
        L = float(rng.uniform(20, 60))
        if periodic:
            x = rng.random((n, 3)) * L
        else:
            x = rng.normal(size=(n, 3)) * L / 4 + (np.array([3 * L, 0, 0]) if kind != "s" else 0)
        smax = L * float(rng.uniform(0.15, 0.45 if kind != "spi" else 0.34))
        nb = int(rng.integers(1, 12))
        e1 = np.sort(rng.uniform(0, smax, nb + 1))
        if rng.random() < 0.5:
            e1[0] = 0.0
        e2 = synth.mu_edges(int(rng.integers(1, 9))) if kind == "smu" else np.sort(rng.uniform(0, smax * 0.7, 4))
        los = "mid" if (not periodic and kind != "s" and rng.random() < 0.5) else "z"
        tuning = dict(cells_per_rmax=int(rng.integers(1, 6)), tile_points=int(rng.choice([64, 128])),
                      seg_cells=int(rng.integers(1, 5)), b_chunk=int(rng.choice([256, 1024, 16384])),
                      hist_copies=int(rng.choice([1, 2, 4])), order=str(rng.choice(["built", "heuristic"])))
        w = synth.uniform_weights(n, 0.5, 2.0, t) if rng.random() < 0.3 else None
        check_case(f"sweep {t}", x, kind=kind, los=los, box=L if periodic else 0.0, edges1=e1,
                   edges2=None if kind == "s" else e2, w1=w, **tuning)


def test_invariance_under_tuning_c2_shape():
    """Counts do not depend on the cell size, tile, segment, chunk, histogram copies or order."""
    n = 40000
    x = synth.lognormal_box(n, 2000.0, 99, ngrid=64)
    kw = dict(kind="smu", edges1=synth.linear_edges(0, 200, 40), edges2=synth.mu_edges(100), box=2000.0)
    ref = None
    for tune in [dict(), dict(cells_per_rmax=1), dict(cells_per_rmax=4, tile_points=64),
                 dict(cells_per_rmax=3, seg_cells=3, b_chunk=512, hist_copies=2, order="built")]:
        note(f"invariance {tune}")
        g, _, _ = gpu_count(x, **kw, **tune)
        if ref is None:
            ref = g
        assert np.array_equal(g, ref), tune
    perm = np.random.default_rng(1).permutation(n)
    g, _, _ = gpu_count(x[perm], **kw)
    assert np.array_equal(g, ref)


def test_c2_full_size_sampled():
    """C2 at full size (1,000,000 clustered points): the total equals the sum over a partition of
    the catalogue into pieces counted as autos and crosses on the GPU, and one piece is checked
    against the oracle (cross of a 2,000-point sample with the whole catalogue)."""
    w = synth.workload(2)
    x = w["x1"]
    kw = dict(kind="smu", edges1=w["edges1"], edges2=w["edges2"], box=w["box"])
    note("C2 full auto")
    full, _, st = gpu_count(x, **kw)
    assert full.sum() == st["in_range"]
    # additivity: auto(A u B) = auto(A) + auto(B) + cross(A, B)
    h = len(x) // 2
    a, b = x[:h], x[h:]
    note("C2 halves")
    aa, _, _ = gpu_count(a, **kw)
    bb, _, _ = gpu_count(b, **kw)
    ab, _, _ = gpu_count(a, b, **kw)
    assert np.array_equal(aa + bb + ab, full)
    # sampled cross against the oracle (cell list)
    idx = np.random.default_rng(5).choice(len(x), 2000, replace=False)
    s = x[idx]
    note("C2 sample x full")
    g, _, _ = gpu_count(s, x, **kw)
    o, _ = oracle_count(s, x, method="grid", **kw)
    assert_same(g, o, what="C2 sample x full")


def test_c2_full_size_weighted_sampled():
    """C2 weighted at full size, as the benchmark counts it: a 2,000-point sample crossed with
    the whole catalogue, counts and FP64 weighted sums, against the oracle."""
    w = synth.workload(2, weighted=True)
    x, wt = w["x1"], w["w1"]
    kw = dict(kind="smu", edges1=w["edges1"], edges2=w["edges2"], box=w["box"])
    idx = np.random.default_rng(6).choice(len(x), 2000, replace=False)
    note("C2 weighted sample x full")
    g, gw, _ = gpu_count(x[idx], x, w1=wt[idx], w2=wt, **kw)
    o, ow = oracle_count(x[idx], x, method="grid", w1=wt[idx], w2=wt, **kw)
    assert_same(g, o, gw, ow, what="C2 weighted sample x full")


def test_c3_full_size_sampled():
    """C3 at full size (2,000,000 data, 40,000,000 randoms, open box, mid-point line of sight,
    weights): DD of the whole data set satisfies additivity over two halves, and samples of
    DD and DR (1,000 data points against all data; 40 against all randoms) match the oracle."""
    w = synth.workload(3, weighted=True)
    d, r, wd, wr = w["x1"], w["x2"], w["w1"], w["w2"]
    kw = dict(kind="spi", los="mid", edges1=w["edges1"], edges2=w["edges2"], box=0.0)
    note("C3 DD full")
    full, fw, st = gpu_count(d, w1=wd, **kw)
    assert full.sum() == st["in_range"]
    h = len(d) // 2
    note("C3 DD halves")
    aa, aw, _ = gpu_count(d[:h], w1=wd[:h], **kw)
    bb, bw, _ = gpu_count(d[h:], w1=wd[h:], **kw)
    ab, abw, _ = gpu_count(d[:h], d[h:], w1=wd[:h], w2=wd[h:], **kw)
    assert np.array_equal(aa + bb + ab, full)
    # each weighted bin is its exact sum rounded once: the three parts add up to
    # the whole within a few roundings
    assert np.all(np.abs((aw + bw + abw) - fw) <= 4e-16 * np.abs(fw))
    # merging the LDS histograms every 2^16 claimed pairs changes nothing
    note("C3 DD full, early merges")
    fm, fwm, stm = gpu_count(d, w1=wd, flush_log2=16, **kw)
    assert stm["flushes"] > 0
    assert np.array_equal(fm, full) and np.array_equal(fwm, fw)
    rng = np.random.default_rng(7)
    idx = rng.choice(len(d), 1000, replace=False)
    note("C3 DD sample x full data")
    g, gw, _ = gpu_count(d[idx], d, w1=wd[idx], w2=wd, **kw)
    o, ow = oracle_count(d[idx], d, method="grid", w1=wd[idx], w2=wd, **kw)
    assert_same(g, o, gw, ow, what="C3 DD sample")
    idx = rng.choice(len(d), 40, replace=False)
    note("C3 DR sample x full randoms")
    g, gw, _ = gpu_count(d[idx], r, w1=wd[idx], w2=wr, **kw)
    o, ow = oracle_count(d[idx], r, method="grid", w1=wd[idx], w2=wr, **kw)
    assert_same(g, o, gw, ow, what="C3 DR sample")


def test_c5_full_size_sampled():
    """C5 at full size (10,000,000 clustered points, log bins down to s = 0.1): additivity over
    two halves and a 3,000-point sample against the whole catalogue, checked by the oracle."""
    w = synth.workload(5)
    x = w["x1"]
    kw = dict(kind="s", edges1=w["edges1"], box=w["box"])
    note("C5 full auto")
    full, _, st = gpu_count(x, **kw)
    assert full.sum() == st["in_range"]
    h = len(x) // 2
    note("C5 halves")
    aa, _, _ = gpu_count(x[:h], **kw)
    bb, _, _ = gpu_count(x[h:], **kw)
    ab, _, _ = gpu_count(x[:h], x[h:], **kw)
    assert np.array_equal(aa + bb + ab, full)
    idx = np.random.default_rng(8).choice(len(x), 3000, replace=False)
    note("C5 sample x full")
    g, _, _ = gpu_count(x[idx], x, **kw)
    o, _ = oracle_count(x[idx], x, method="grid", **kw)
    assert_same(g, o, what="C5 sample x full")


def test_errors_on_device_data():
    import torch
    from paper_2301_12557_amd import fcfc
    e = np.array([0.0, 1.0, 2.0])
    x = np.random.default_rng(0).random((100, 3)) * 10.0
    bad = x.copy()
    bad[5, 1] = np.nan
    with pytest.raises(fcfc.FcfcError) as ei:
        fcfc.count_pairs(torch.from_numpy(bad).cuda(), kind="s", edges1=e, box=10.0)
    assert ei.value.name == "FCFC_ENONFINITE"
    out = x.copy()
    out[7, 2] = 10.0
    with pytest.raises(fcfc.FcfcError) as ei:
        fcfc.count_pairs(torch.from_numpy(out).cuda(), kind="s", edges1=e, box=10.0)
    assert ei.value.name == "FCFC_EBOX"
    p1 = fcfc.Plan("s", e, box=10.0)
    p2 = fcfc.Plan("s", e, box=10.0)
    c1 = p1.build_cells(torch.from_numpy(x).cuda())
    with pytest.raises(fcfc.FcfcError) as ei:
        p2.count(c1)
    assert ei.value.name == "FCFC_EGRID"


def test_hardware_rsq_rcp_within_band_bound():
    """The FP32 mu and mid-point pi bands assume a relative error bound for the
    hardware rsq and rcp; measured over every FP32 input in [2^-64, 2^64)."""
    from paper_2301_12557_amd import fcfc
    rs, rc, bound = fcfc.diag_transcendental()
    note(f"max rel error rsq {rs:.3e} rcp {rc:.3e} (bands assume {bound:.3e})")
    assert 0 < rs <= bound and 0 < rc <= bound


def test_roofline_microbenchmarks_are_plausible():
    """The measured FP32 FMA, LDS atomic and copy rates the bench reports beside the
    published peaks: positive, and not above the published figures."""
    from paper_2301_12557_amd import fcfc
    pk = fcfc.diag_peaks()
    note(f"peaks {pk}")
    assert 10.0 < pk["fma_tflops"] <= 157.3 * 1.05
    assert pk["lds_u32_per_s"] > 1e12 and pk["lds_u64_per_s"] > 1e11
    assert 100.0 < pk["copy_gbps"] <= 8000.0 * 1.1


def test_shards_sum_to_the_whole_count():
    """The work-list shards (ordered items i % G == g) of G GPUs, each counted on its
    own: the G histograms sum bit-exactly to the whole count, weighted sums to 1e-12."""
    w = synth.workload(2, scale=0.03, weighted=True)
    kw = dict(kind="smu", edges1=w["edges1"], edges2=w["edges2"], box=w["box"], w1=w["w1"])
    whole, wwhole, st = gpu_count(w["x1"], **kw)
    for G in (2, 3, 8):
        tot = np.zeros_like(whole)
        wtot = np.zeros_like(wwhole)
        cand = 0
        for g in range(G):
            c, wc, sg = gpu_count(w["x1"], shard_count=G, shard_index=g, **kw)
            tot += c
            wtot += wc
            cand += sg["candidates"]
        assert np.array_equal(tot, whole), G
        assert cand == st["candidates"]
        assert np.allclose(wtot, wwhole, rtol=1e-12, atol=0)


def _midpoint_pairs(edges_sp, edges_pi, n_per, seed, rmin=1000.0, rmax=2000.0):
    """Pairs (a_i, b_i) of a survey shell placed so that the FP64 mid-point pi^2
    or s_perp^2 of the pair lies at a chosen relative offset (1e-11 .. 1e-1, both
    signs) from an edge.  b = a + pi l_hat + s_perp p_hat, with l_hat the
    mid-point line of sight of the pair itself, found by fixed-point iteration."""
    rng = np.random.default_rng(seed)
    offs = np.concatenate([-np.logspace(-11, -1, 21), np.logspace(-11, -1, 21)])
    A, B = [], []

    def place(pi_t, sp_t):
        a = synth.survey_shell(1, int(rng.integers(1 << 30)), rmin=rmin + 300.0, rmax=rmax - 300.0)[0]
        t = rng.normal(size=3)
        lh = a / np.linalg.norm(a)
        for _ in range(60):
            p = t - (t @ lh) * lh
            p /= np.linalg.norm(p)
            b = a + pi_t * lh + sp_t * p
            l2 = (a + b) / np.linalg.norm(a + b)
            if np.allclose(l2, lh, rtol=0, atol=1e-17):
                break
            lh = l2
        A.append(a)
        B.append(b)

    for k, e in enumerate(edges_pi[1:], 1):
        for d in offs[rng.permutation(len(offs))[:n_per]]:
            place(np.sqrt(e * e * (1.0 + d)), rng.uniform(0.0, edges_sp[-1] * 0.9))
    for k, e in enumerate(edges_sp[1:], 1):
        for d in offs[rng.permutation(len(offs))[:n_per]]:
            place(rng.uniform(0.0, edges_pi[-1] * 0.9) * rng.choice([-1.0, 1.0]), np.sqrt(e * e * (1.0 + d)))
    return np.array(A), np.array(B)


def test_midpoint_knife_edges():
    """Pairs at every distance from 1e-11 to 1e-1 (relative, both sides) of each
    pi and s_perp edge, mid-point line of sight: the FP32 bands must send every
    pair whose FP32 value could fall on the wrong side to the FP64 recheck, so the
    counts equal the oracle's bit for bit."""
    e = synth.linear_edges(0, 200, 40)
    a, b = _midpoint_pairs(e, e, 16, 5)
    note(f"mid-point knife edges: {len(a)} constructed pairs")
    check_case("mid knife spi", a, b, kind="spi", los="mid", edges1=e, edges2=e, box=0.0)
    # (s, mu) with the same pairs: mu edges meet pairs at every angle
    check_case("mid knife smu", a, b, kind="smu", los="mid", edges1=synth.linear_edges(0, 282, 47),
               edges2=synth.mu_edges(20), box=0.0)


def test_c4_full_size_batch_sampled():
    """C4 at full size, as the benchmark counts it (batched pipeline replayed from
    a HIP graph): six mocks of the 200 (the largest, the smallest and four
    others, 100k-500k points, L = 1000, (s, mu) 40 x 100).  Each batched histogram
    equals that mock counted alone, bit for bit, and a sampled cross of each mock
    equals the oracle's."""
    import torch
    from paper_2301_12557_amd import fcfc
    sizes = synth.mock_sizes(200)
    pick = sorted({int(np.argmax(sizes)), int(np.argmin(sizes)), 3, 50, 120, 199})
    e1 = synth.linear_edges(0, 200, 40)
    e2 = synth.mu_edges(100)
    xs = [synth.lognormal_box_torch(int(sizes[m]), 1000.0, synth.MOCK_SEED_BASE + m, device="cuda") for m in pick]
    note(f"C4 batch of mocks {pick}, sizes {[int(sizes[m]) for m in pick]}")
    plan = fcfc.Plan("smu", e1, e2, box=1000.0, n_hint=int(np.median(sizes)))
    b = fcfc.Batch(plan, [(x, None) for x in xs])
    nb = 40 * 100
    out = torch.empty(len(xs) * nb, dtype=torch.int64, device="cuda")
    for _ in range(2):
        b.run(out, use_graph=True)
        b.check()
    got = out.cpu().numpy().reshape(len(xs), nb)
    rng = np.random.default_rng(17)
    for i, x in enumerate(xs):
        c = plan.build_cells(x)
        alone, _ = plan.count(c)
        c.close()
        assert np.array_equal(got[i], alone.cpu().numpy().reshape(-1)), f"mock {pick[i]}"
        xh = x.cpu().numpy()
        s = xh[rng.choice(len(xh), 1000, replace=False)]
        g, _, _ = gpu_count(s, xh, kind="smu", edges1=e1, edges2=e2, box=1000.0)
        o, _ = oracle_count(s, xh, kind="smu", edges1=e1, edges2=e2, box=1000.0, method="grid")
        assert_same(g, o, what=f"C4 mock {pick[i]} sample x full")
    b.close()
    plan.close()


@pytest.mark.parametrize("wlo,whi", [(1e-200, 1.0), (1e-160, 1e-160)])
def test_weight_products_underflow_refused(wlo, whi):
    """Weights whose smallest pair product underflows FP64 (zero, or subnormal)
    cannot be summed exactly: the pair count, the batched pipeline and the
    triangle count refuse them with FCFC_ERANGE, as the oracle refuses them,
    and the outputs are left untouched."""
    import oracle
    import torch
    from paper_2301_12557_amd import fcfc
    rng = np.random.default_rng(12)
    x = rng.random((300, 3)) * 50.0
    w = np.where(rng.random(300) < 0.5, wlo, whi)
    w[0], w[1] = wlo, whi
    e = synth.linear_edges(0, 10, 5)
    with pytest.raises(oracle.OracleError):
        oracle_count(x, kind="s", edges1=e, box=50.0, w1=w)
    with pytest.raises(fcfc.FcfcError) as ei:
        gpu_count(x, kind="s", edges1=e, box=50.0, w1=w)
    assert ei.value.name == "FCFC_ERANGE"
    plan = fcfc.Plan("s", e, box=50.0)
    dx, dw = to_dev(x), to_dev(w)
    with pytest.raises(fcfc.FcfcError) as ei:
        fcfc.Batch(plan, [(dx, dw), (dx, dw)])
    assert ei.value.name == "FCFC_ERANGE"
    cells = plan.build_cells(dx, dw)
    out = torch.full((5,), -7, dtype=torch.int64, device="cuda")
    wout = torch.full((5,), -7.0, dtype=torch.float64, device="cuda")
    with pytest.raises(fcfc.FcfcError) as ei:
        plan.count(cells, weighted=True, out=out, wout=wout)
    assert ei.value.name == "FCFC_ERANGE"
    assert int(out.sum()) == -35 and float(wout.sum()) == -35.0
    with pytest.raises(fcfc.FcfcError) as ei:
        fcfc.count_triplets(dx, edges=e, box=50.0, w=dw)
    assert ei.value.name == "FCFC_ERANGE"
    cells.close()
    plan.close()


# ---------------------------------------------------------------------------
# Full-size histograms against the oracle's cell list, bin for bin: the
# benchmark's own counts (definitions of Sect. 2.5, each unordered pair once
# as in Sect. 3.1).  The cell list is pinned to the brute-force loop on the
# same shapes by the CPU tests.
# ---------------------------------------------------------------------------
def test_c2_full_size_weighted_vs_oracle():
    """C2, the headline count, in full: all 1,000,000 clustered points, weighted
    (s, mu) 40 x 100, line of sight z, periodic L = 2000.  Counts and exact
    weighted sums equal the oracle's in every bin."""
    w = synth.workload(2, weighted=True)
    kw = dict(kind="smu", edges1=w["edges1"], edges2=w["edges2"], box=w["box"], w1=w["w1"])
    note("C2 full weighted, GPU")
    g, gw, st = gpu_count(w["x1"], **kw)
    note(f"C2 full weighted, oracle ({st['in_range']} pairs)")
    o, ow = oracle_count(w["x1"], method="grid", **kw)
    assert_same(g, o, gw, ow, what="C2 full weighted")
    assert np.array_equal(gw, ow)


def test_c5_full_size_vs_oracle():
    """C5 in full, as the benchmark draws it on the GPU: 10,000,000 clustered
    points, periodic L = 3000, 50 log s bins over [0.1, 50) (hybrid table)."""
    import torch
    x = synth.lognormal_box_torch(10_000_000, 3000.0, synth.config_seed(5), device="cuda")
    e1 = synth.log_edges(0.1, 50.0, 50)
    note("C5 full, GPU")
    from paper_2301_12557_amd import fcfc
    c, _, st = fcfc.count_pairs(x, kind="s", edges1=e1, box=3000.0, return_stats=True)
    torch.cuda.synchronize()
    g = c.cpu().numpy()
    xh = x.cpu().numpy()
    del x
    note(f"C5 full, oracle ({st['in_range']} pairs)")
    o, _ = oracle_count(xh, kind="s", edges1=e1, box=3000.0, method="grid")
    assert_same(g, o, what="C5 full")


def test_c4_smallest_mocks_batched_vs_oracle():
    """C4 through the batched pipeline replayed from a HIP graph, as the
    benchmark runs it: the 20 smallest of the 200 mocks (L = 1000, (s, mu)
    40 x 100), each histogram equal to the oracle's in every bin."""
    import torch
    from paper_2301_12557_amd import fcfc
    sizes = synth.mock_sizes(200)
    pick = [int(m) for m in np.argsort(sizes, kind="stable")[:20]]
    e1 = synth.linear_edges(0, 200, 40)
    e2 = synth.mu_edges(100)
    xs = [synth.lognormal_box_torch(int(sizes[m]), 1000.0, synth.MOCK_SEED_BASE + m, device="cuda") for m in pick]
    note(f"C4 batch of the 20 smallest mocks, {int(sizes[pick].sum())} points")
    plan = fcfc.Plan("smu", e1, e2, box=1000.0, n_hint=int(np.median(sizes)))
    b = fcfc.Batch(plan, [(x, None) for x in xs])
    nb = 40 * 100
    out = torch.empty(len(xs) * nb, dtype=torch.int64, device="cuda")
    for _ in range(2):
        b.run(out, use_graph=True)
        b.check()
    got = out.cpu().numpy().reshape(len(xs), 40, 100)
    b.close()
    plan.close()
    for i, x in enumerate(xs):
        o, _ = oracle_count(x.cpu().numpy(), kind="smu", edges1=e1, edges2=e2, box=1000.0, method="grid")
        assert_same(got[i], o, what=f"C4 mock {pick[i]}")


def test_c3_rr_additivity_and_sample():
    """C3's RR (randoms x randoms, open survey shell, weighted (s_perp, pi), mid-point
    line of sight) at a quarter of the randoms' density (10,000,000 points): the
    whole auto count equals the sum over two halves counted as autos and a cross
    (counts exactly, weighted sums within rounding), and 40 randoms crossed with
    all of them match the oracle."""
    w = synth.workload(3, weighted=True, scale=0.25)
    r, wr = w["x2"], w["w2"]
    kw = dict(kind="spi", los="mid", edges1=w["edges1"], edges2=w["edges2"], box=0.0)
    note(f"C3 RR at {len(r)} randoms")
    full, fw, st = gpu_count(r, w1=wr, **kw)
    assert full.sum() == st["in_range"] and st["candidates"] > full.sum()
    h = len(r) // 2
    aa, aw, _ = gpu_count(r[:h], w1=wr[:h], **kw)
    bb, bw, _ = gpu_count(r[h:], w1=wr[h:], **kw)
    ab, abw, _ = gpu_count(r[:h], r[h:], w1=wr[:h], w2=wr[h:], **kw)
    assert np.array_equal(aa + bb + ab, full)
    assert np.all(np.abs((aw + bw + abw) - fw) <= 4e-16 * np.abs(fw))
    idx = np.random.default_rng(33).choice(len(r), 40, replace=False)
    note("C3 RR sample x all randoms")
    g, gw, _ = gpu_count(r[idx], r, w1=wr[idx], w2=wr, **kw)
    o, ow = oracle_count(r[idx], r, method="grid", w1=wr[idx], w2=wr, **kw)
    assert_same(g, o, gw, ow, what="C3 RR sample")
