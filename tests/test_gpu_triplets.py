"""Triangle counts on the GPU (fcfc_count_triplets) against the oracle, bit for
bit: the cubic-lattice closed forms, uniform periodic and open boxes, clustered
points whose neighbour lists exceed one LDS region (chunked lists), several
grid sizes, and tiny catalogues."""
import numpy as np
import pytest

import oracle
from helpers import note, to_dev, assert_same

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _gpu_tri(x, edges, box, **tuning):
    import torch
    from paper_2301_12557_amd import fcfc
    c, st = fcfc.count_triplets(to_dev(x), edges=edges, box=box, return_stats=True, **tuning)
    torch.cuda.synchronize()
    return c.cpu().numpy(), st


def test_cubic_lattice():
    g = np.arange(6, dtype=np.float64)
    x = np.stack(np.meshgrid(g, g, g, indexing="ij"), -1).reshape(-1, 3)
    N = len(x)
    e = [0.5, 1.2, 1.5, 1.8, 2.1]
    note("triplets: cubic lattice 6^3, periodic")
    got, st = _gpu_tri(x, e, 6.0)
    assert got[0, 0, 1] == 12 * N and got[1, 1, 1] == 8 * N and got[0, 1, 2] == 24 * N
    assert got[0, 0, 3] == 3 * N and got[1, 1, 3] == 12 * N and got[2, 2, 3] == 12 * N
    assert_same(got, oracle.triplets(x, edges=e, box=6.0, method="brute"), what="lattice")
    assert st["in_range"] == got.sum()


@pytest.mark.parametrize("box", [100.0, 0.0])
def test_uniform_box(box):
    rng = np.random.default_rng(11)
    x = rng.uniform(0, 100, (3000, 3))
    e = np.linspace(1.0, 10.0, 10)
    note(f"triplets: uniform 3000 in 100^3, box {box}")
    got, st = _gpu_tri(x, e, box)
    ref = oracle.triplets(x, edges=e, box=box)
    assert ref.sum() > 10000
    assert_same(got, ref, what=f"uniform box {box}")


@pytest.mark.parametrize("box", [100.0, 0.0])
def test_clustered_long_lists(box):
    """Tight Gaussian blobs: hundreds of neighbours per point, so the lists are
    taken in chunks of 128 (chunk against itself and every later chunk)."""
    rng = np.random.default_rng(12)
    cen = rng.uniform(10, 90, (6, 3))
    x = cen[rng.integers(0, 6, 3000)] + rng.normal(0, 1.2, (3000, 3))
    x = np.concatenate([x, rng.uniform(0, 100, (1000, 3))])
    x = np.clip(x, 0, np.nextafter(100.0, 0))
    e = np.concatenate([[0.05], np.geomspace(0.2, 6.0, 12)])
    note(f"triplets: clustered 4000, box {box}")
    got, st = _gpu_tri(x, e, box)
    ref = oracle.triplets(x, edges=e, box=box)
    assert ref.sum() > 1e6
    assert_same(got, ref, what=f"clustered box {box}")


def test_grid_sizes_agree():
    rng = np.random.default_rng(13)
    x = rng.uniform(0, 50, (2000, 3))
    e = np.linspace(0.0, 6.0, 7)
    ref = oracle.triplets(x, edges=e, box=50.0)
    for k in (1, 2, 3, 4):
        note(f"triplets: cells_per_rmax {k}")
        got, _ = _gpu_tri(x, e, 50.0, cells_per_rmax=k)
        assert_same(got, ref, what=f"k={k}")


def test_vertex_order_ties_and_many_stencil_rows():
    """A triangle is found from its first vertex in the order of the stored
    coordinates (z, y, x, then index): an open lattice puts many points on
    one z plane, one y line and one spot (duplicates), so every tie-break of
    that order decides.  Clustered points with 4 cells per r_max give more
    than 32 stencil rows (the gather fetches them 32 at a time) and chunked
    lists, with ordered counters (13 bins) and sorted ones (20 bins)."""
    g = np.arange(5, dtype=np.float64)
    lat = np.stack(np.meshgrid(g, g, g, indexing="ij"), -1).reshape(-1, 3)
    lat = np.concatenate([lat, lat[::7]])  # duplicated points
    e = [0.0, 0.5, 1.2, 1.5, 1.8, 2.1, 3.1]
    note("triplets: open lattice 5^3 with duplicates")
    got, _ = _gpu_tri(lat, e, 0.0)
    assert_same(got, oracle.triplets(lat, edges=e, box=0.0, method="brute"), what="open lattice")
    rng = np.random.default_rng(21)
    cen = rng.uniform(10, 40, (4, 3))
    x = cen[rng.integers(0, 4, 1500)] + rng.normal(0, 1.0, (1500, 3))
    x = np.concatenate([x, rng.uniform(0, 50, (500, 3))])
    for nb in (13, 20):
        e = np.linspace(0.0, 5.0, nb + 1)
        ref = oracle.triplets(x, edges=e, box=0.0)
        note(f"triplets: clustered open box, 4 cells per r_max, {nb} bins")
        got, st = _gpu_tri(x, e, 0.0, cells_per_rmax=4)
        assert_same(got, ref, what=f"clustered k=4 nb={nb}")


def test_tiny_catalogues():
    rng = np.random.default_rng(14)
    e = [0.0, 1.0, 2.0, 3.0]
    for n in (0, 1, 2, 3, 7):
        x = rng.uniform(0, 2, (n, 3)) if n else np.zeros((0, 3))
        got, _ = _gpu_tri(x, e, 10.0)
        assert_same(got, oracle.triplets(x, edges=e, box=10.0, method="brute"), what=f"n={n}")


def test_full_size_invariances():
    """The bench workload (2e6 uniform points, periodic box 1000, 15 bins to 30),
    in the launch the bench times: the counts do not change with the grid (1 or
    2 cells per r_max: other stencils, scan orders and list chunks) or with the
    order of the input points, and the total matches the stats."""
    import torch
    from paper_2301_12557_amd import fcfc, synth
    n, L = 2_000_000, 1000.0
    x = torch.from_numpy(synth.uniform_box(n, L, synth.config_seed(7))).cuda()
    e = synth.linear_edges(0, 30.0, 15)
    note("triplets: full size, default grid")
    a, st = fcfc.count_triplets(x, edges=e, box=L, return_stats=True)
    assert a.sum().item() == st["in_range"] > 7e9
    note("triplets: full size, 2 cells per r_max")
    b = fcfc.count_triplets(x, edges=e, box=L, cells_per_rmax=2)
    assert torch.equal(a, b)
    note("triplets: full size, permuted input")
    perm = torch.randperm(n, generator=torch.Generator().manual_seed(5)).cuda()
    c = fcfc.count_triplets(x[perm].contiguous(), edges=e, box=L)
    assert torch.equal(a, c)
    # sorted-bin structure: nothing below the diagonal
    idx = torch.nonzero(a)
    assert bool((idx[:, 0] <= idx[:, 1]).all() and (idx[:, 1] <= idx[:, 2]).all())


def _gpu_tri_w(x, w, edges, box, **tuning):
    import torch
    from paper_2301_12557_amd import fcfc
    (c, wc), st = fcfc.count_triplets(to_dev(x), edges=edges, box=box, w=to_dev(w), return_stats=True, **tuning)
    torch.cuda.synchronize()
    return c.cpu().numpy(), wc.cpu().numpy(), st


@pytest.mark.parametrize("box", [100.0, 0.0])
def test_weighted_match_oracle(box):
    """Weighted triangles (weights sorted by value, fl(fl(a b) c), exact sums
    rounded once): uniform points with mixed-sign weights, and clustered points
    whose lists are chunked; counts bit for bit, weighted sums within 1e-12."""
    rng = np.random.default_rng(31)
    x = rng.uniform(0, 100, (3000, 3))
    w = rng.uniform(0.5, 2.0, len(x)) * rng.choice([-1.0, 1.0], len(x))
    e = np.linspace(1.0, 10.0, 10)
    note(f"triplets weighted: uniform 3000, box {box}")
    c, wc, _ = _gpu_tri_w(x, w, e, box)
    rc, rw = oracle.triplets(x, edges=e, box=box, w=w)
    assert_same(c, rc, wc, rw, what=f"weighted uniform box {box}")
    cen = rng.uniform(10, 90, (6, 3))
    x = cen[rng.integers(0, 6, 3000)] + rng.normal(0, 1.2, (3000, 3))
    x = np.clip(np.concatenate([x, rng.uniform(0, 100, (1000, 3))]), 0, np.nextafter(100.0, 0))
    w = rng.uniform(0.6, 1.8, len(x))
    e = np.concatenate([[0.05], np.geomspace(0.2, 6.0, 12)])
    note(f"triplets weighted: clustered 4000, box {box}")
    c, wc, _ = _gpu_tri_w(x, w, e, box)
    rc, rw = oracle.triplets(x, edges=e, box=box, w=w)
    assert_same(c, rc, wc, rw, what=f"weighted clustered box {box}")


def test_weighted_closed_forms():
    rng = np.random.default_rng(32)
    x = rng.uniform(0, 50, (2000, 3))
    e = np.linspace(0.0, 6.0, 7)
    c1, w1, _ = _gpu_tri_w(x, np.ones(len(x)), e, 50.0)
    assert np.array_equal(w1, c1.astype(np.float64))
    c2, w2, _ = _gpu_tri_w(x, np.full(len(x), 2.0), e, 50.0)
    assert np.array_equal(c2, c1) and np.array_equal(w2, 8.0 * c1)


def test_cross_catalogue_terms_from_weighted_counts():
    """Data weight 1 and randoms weight t on the merged catalogue give
    DDD + t DDR + t^2 DRR + t^3 RRR per bin, exactly for small integers t; with
    t = 2 and t = -1 and DDD, RRR counted alone, DDR and DRR follow exactly.
    Checked against an enumeration of typed triples."""
    from itertools import combinations
    rng = np.random.default_rng(33)
    L = 10.0
    d = rng.uniform(0, L, (150, 3))
    r = rng.uniform(0, L, (150, 3))
    e = [0.5, 1.5, 2.5, 3.5]
    x = np.concatenate([d, r])
    ddd, _, _ = _gpu_tri_w(d, np.ones(len(d)), e, L)
    rrr, _, _ = _gpu_tri_w(r, np.ones(len(r)), e, L)
    _, w2, _ = _gpu_tri_w(x, np.r_[np.ones(len(d)), np.full(len(r), 2.0)], e, L)
    _, wm, _ = _gpu_tri_w(x, np.r_[np.ones(len(d)), np.full(len(r), -1.0)], e, L)
    A = w2 - ddd - 8.0 * rrr
    B = wm - ddd + rrr
    ddr = (A - 4.0 * B) / 6.0
    drr = (A + 2.0 * B) / 6.0
    # typed enumeration
    dv = x[None, :, :] - x[:, None, :]
    dv = dv - L * np.round(dv / L)
    s = np.sqrt((dv * dv).sum(-1))
    E = np.asarray(e)
    b = np.searchsorted(E, s, side="right") - 1
    b[(s < E[0]) | (s >= E[-1])] = -1
    nb = len(e) - 1
    nd = len(d)
    tr = np.array(list(combinations(range(len(x)), 3)))
    sides = np.stack([b[tr[:, 0], tr[:, 1]], b[tr[:, 0], tr[:, 2]], b[tr[:, 1], tr[:, 2]]], axis=1)
    nr = (tr >= nd).sum(1)
    ok = (sides >= 0).all(1)
    sides = np.sort(sides, axis=1)
    ref = {}
    for kind in (1, 2):
        sel = ok & (nr == kind)
        h = np.zeros(nb ** 3)
        np.add.at(h, (sides[sel, 0] * nb + sides[sel, 1]) * nb + sides[sel, 2], 1)
        ref[kind] = h.reshape(nb, nb, nb)
    assert ref[1].sum() > 1000 and ref[2].sum() > 1000
    assert np.array_equal(ddr, ref[1]) and np.array_equal(drr, ref[2])


def test_most_bins():
    """32 bins (the most; 5984 counters leave fewer waves per workgroup), and
    20 bins weighted, exact; 32 bins weighted do not fit the LDS and are
    refused."""
    from paper_2301_12557_amd import fcfc
    rng = np.random.default_rng(34)
    x = rng.uniform(0, 40, (3000, 3))
    e32 = np.linspace(0.2, 6.6, 33)
    note("triplets: 32 bins")
    got, st = _gpu_tri(x, e32, 40.0)
    assert_same(got, oracle.triplets(x, edges=e32, box=40.0), what="32 bins")
    w = rng.uniform(0.5, 2.0, len(x))
    e20 = np.linspace(0.2, 6.2, 21)
    note("triplets: 20 bins weighted")
    c, wc, _ = _gpu_tri_w(x, w, e20, 40.0)
    rc, rw = oracle.triplets(x, edges=e20, box=40.0, w=w)
    assert_same(c, rc, wc, rw, what="20 bins weighted")
    with pytest.raises(fcfc.FcfcError):
        _gpu_tri_w(x, w, e32, 40.0)
