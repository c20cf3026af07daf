"""Pins of the triangle-count oracle (oracle.triplets): closed forms on a
periodic cubic lattice, an independent numpy enumeration of all triples, every
triple of a compact set, and invariance under permutation, translation and
scaling."""
from itertools import combinations
from math import comb

import numpy as np
import pytest

import oracle


def _enumerate(x, edges, box):
    """All triples by numpy: minimum-image side lengths, searchsorted bins,
    sorted bin triples counted."""
    x = np.asarray(x, dtype=np.float64)
    n = len(x)
    d = x[None, :, :] - x[:, None, :]
    if box > 0:
        d = d - box * np.round(d / box)
    s = np.sqrt((d * d).sum(-1))
    e = np.asarray(edges, dtype=np.float64)
    b = np.searchsorted(e, s, side="right") - 1
    b[(s < e[0]) | (s >= e[-1])] = -1
    t = np.array(list(combinations(range(n), 3)))
    sides = np.stack([b[t[:, 0], t[:, 1]], b[t[:, 0], t[:, 2]], b[t[:, 1], t[:, 2]]], axis=1)
    ok = (sides >= 0).all(1)
    sides = np.sort(sides[ok], axis=1)
    nb = len(e) - 1
    h = np.zeros(nb ** 3, dtype=np.int64)
    np.add.at(h, (sides[:, 0] * nb + sides[:, 1]) * nb + sides[:, 2], 1)
    return h.reshape(nb, nb, nb)


def _lattice(m):
    g = np.arange(m, dtype=np.float64)
    return np.stack(np.meshgrid(g, g, g, indexing="ij"), -1).reshape(-1, 3)


def test_cubic_lattice_closed_forms():
    """Unit lattice, periodic box of 6: bins isolate sides 1, sqrt2, sqrt3, 2.
    Per point: 12 right triangles (1, 1, sqrt2) at their right angle; 8
    equilateral (sqrt2)^3 per unit cube; 24 (1, sqrt2, sqrt3) (6 per body
    diagonal, 4 diagonals per point); 3 collinear (1, 1, 2) by their middle
    point; 12 (sqrt2, sqrt2, 2) and 12 (sqrt3, sqrt3, 2) over the 3 pairs at
    distance 2 per point, with 4 apexes each."""
    x = _lattice(6)
    N = len(x)
    e = [0.5, 1.2, 1.5, 1.8, 2.1]
    for method in ("brute", "list"):
        h = oracle.triplets(x, edges=e, box=6.0, method=method)
        assert h[0, 0, 1] == 12 * N
        assert h[1, 1, 1] == 8 * N
        assert h[0, 1, 2] == 24 * N
        assert h[0, 0, 3] == 3 * N
        assert h[1, 1, 3] == 12 * N
        assert h[2, 2, 3] == 12 * N
        # only sorted bin triples are filled
        a, b, c = np.nonzero(h)
        assert np.all(a <= b) and np.all(b <= c)
    assert np.array_equal(h, _enumerate(x, e, 6.0))


@pytest.mark.parametrize("box", [0.0, 10.0])
def test_random_points_agree_with_enumeration(box):
    rng = np.random.default_rng(3 if box else 4)
    x = rng.uniform(0, 10, (120, 3))
    e = [0.3, 1.0, 2.0, 3.5, 4.9]
    ref = _enumerate(x, e, box)
    assert ref.sum() > 1000
    for method in ("brute", "list"):
        assert np.array_equal(oracle.triplets(x, edges=e, box=box, method=method), ref)


def test_every_triple_of_a_compact_set():
    rng = np.random.default_rng(5)
    x = rng.normal(50, 0.5, (50, 3))
    x = x[np.linalg.norm(x - 50, axis=1) < 1.0]
    h = oracle.triplets(x, edges=[0.0, 10.0], box=0.0)
    assert h[0, 0, 0] == comb(len(x), 3)
    h2 = oracle.triplets(x, edges=[0.0, 10.0], box=100.0)
    assert h2[0, 0, 0] == comb(len(x), 3)


def test_invariances():
    rng = np.random.default_rng(6)
    L = 20.0
    x = rng.uniform(0, L, (400, 3))
    e = np.linspace(0.5, 3.0, 6)
    ref = oracle.triplets(x, edges=e, box=L)
    assert ref.sum() > 500
    assert np.array_equal(oracle.triplets(x[rng.permutation(len(x))], edges=e, box=L), ref)
    shifted = np.mod(x + np.array([7.25, 13.5, 2.125]), L)
    assert np.array_equal(oracle.triplets(shifted, edges=e, box=L), ref)
    assert np.array_equal(oracle.triplets(2 * x, edges=2 * e, box=2 * L), ref)


def test_weighted_closed_forms_and_exact_sums():
    """Weighted triangles: unit weights give the counts, weights of 2 give 8x
    the counts exactly; with mixed-sign random weights every bin equals the
    exact rational sum (fractions) of fl(fl(a b) c) over its triangles, weights
    sorted a <= b <= c, rounded once."""
    from fractions import Fraction
    rng = np.random.default_rng(21)
    L = 10.0
    x = rng.uniform(0, L, (150, 3))
    e = [0.5, 1.0, 2.0, 3.0]
    c0 = oracle.triplets(x, edges=e, box=L)
    c1, w1 = oracle.triplets(x, edges=e, box=L, w=np.ones(len(x)))
    assert np.array_equal(c1, c0) and np.array_equal(w1, c0.astype(np.float64))
    _, w2 = oracle.triplets(x, edges=e, box=L, w=np.full(len(x), 2.0))
    assert np.array_equal(w2, 8.0 * c0)
    w = rng.uniform(0.5, 2.0, len(x)) * rng.choice([-1.0, 1.0], len(x))
    c, wc = oracle.triplets(x, edges=e, box=L, w=w)
    assert np.array_equal(c, c0)
    # independent: enumerate the triples with numpy, sum the products exactly
    d = x[None, :, :] - x[:, None, :]
    d = d - L * np.round(d / L)
    s = np.sqrt((d * d).sum(-1))
    E = np.asarray(e)
    b = np.searchsorted(E, s, side="right") - 1
    b[(s < E[0]) | (s >= E[-1])] = -1
    nb = len(e) - 1
    ref = {}
    for i, j, k in combinations(range(len(x)), 3):
        t = (b[i, j], b[i, k], b[j, k])
        if min(t) < 0:
            continue
        a1, a2, a3 = sorted((w[i], w[j], w[k]))
        key = tuple(sorted(t))
        ref[key] = ref.get(key, Fraction(0)) + Fraction((a1 * a2) * a3)
    expect = np.zeros((nb, nb, nb))
    for key, v in ref.items():
        expect[key] = float(v)
    assert np.array_equal(wc, expect)
