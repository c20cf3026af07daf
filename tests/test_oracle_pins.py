"""Pins of the CPU oracle against facts that do not come from the oracle itself.

Each test names what fixes the expected value: hand-worked cases, lattice
closed forms (sums of three squares), exact counting identities, the uniform
periodic-box expectation with its exact variance, an independent library
neighbour counter, and exactly rounded sums.
"""
import itertools
import json
import math
import os
from fractions import Fraction

import numpy as np
import pytest

import oracle
from paper_2301_12557_amd import synth

HERE = os.path.dirname(os.path.abspath(__file__))


def _hand_cases():
    with open(os.path.join(HERE, "golden", "hand_cases.json")) as f:
        return json.load(f)["cases"]


@pytest.mark.parametrize("case", _hand_cases(), ids=lambda c: c["name"])
def test_hand_cases(case):
    e2 = case.get("edges2")
    if e2 == "mu100":
        e2 = synth.mu_edges(100)
    x1 = np.array(case["x1"], dtype=np.float64)
    x2 = np.array(case["x2"], dtype=np.float64) if "x2" in case else None
    w1 = np.array(case["w1"]) if "w1" in case else None
    for method in ("brute", "grid"):
        c, wc = oracle.count(x1, x2, kind=case["kind"], los=case["los"], box=case["box"],
                             edges1=case["edges1"], edges2=e2, w1=w1, method=method)
        if "expect" in case:
            assert c.ravel().tolist() == case["expect"]
        else:
            exp = np.zeros_like(c)
            for (i, j) in case["expect_bins"]:
                exp[i, j] += 1
            assert (c == exp).all(), (np.argwhere(c), case["expect_bins"])
        if "expect_w" in case:
            assert wc.ravel().tolist() == case["expect_w"]


def r3_table(mmax):
    """Number of integer vectors v with |v|^2 = m, by enumeration."""
    r = [0] * (mmax + 1)
    b = int(math.isqrt(mmax)) + 1
    for v in itertools.product(range(-b, b + 1), repeat=3):
        m = v[0] * v[0] + v[1] * v[1] + v[2] * v[2]
        if m <= mmax:
            r[m] += 1
    return r


def test_r3_textbook_values():
    # sums of three squares: r3(1..7) = 6, 12, 8, 6, 24, 24, 0 (7 = 8*0+7 is not a sum of three squares)
    assert r3_table(7)[1:] == [6, 12, 8, 6, 24, 24, 0]


def _lattice(n, a=1.0):
    g = np.arange(n) * a
    return np.array(list(itertools.product(g, g, g)), dtype=np.float64)


@pytest.mark.parametrize("method", ["brute", "grid"])
def test_lattice_shells(method):
    """n^3 periodic lattice (n odd, spacing 1): pairs at d^2 = m number N r3(m)/2 for sqrt(m) < L/2."""
    n = 7
    x = _lattice(n)
    N = len(x)
    M = 11
    edges = np.sqrt(np.arange(M + 1) + 0.5)       # bin k holds d^2 = k + 1 only
    r3 = r3_table(M + 1)
    c, _ = oracle.count(x, kind="s", edges1=edges, box=float(n), method=method)
    expect = [N * r3[k + 1] // 2 for k in range(M)]
    assert c.tolist() == expect


@pytest.mark.parametrize("method", ["brute", "grid"])
def test_lattice_integer_edges(method):
    """Integer edges put many lattice pairs exactly on an edge: half-open bins decide."""
    n = 7
    x = _lattice(n)
    N = len(x)
    r3 = r3_table(9)
    c, _ = oracle.count(x, kind="s", edges1=[0, 1, 2, 3], box=float(n), method=method)
    expect = [0, N * sum(r3[1:4]) // 2, N * sum(r3[4:9]) // 2]
    assert c.tolist() == expect


def test_lattice_mu_along_axes():
    """Nearest lattice neighbours: 2 of the 6 unit vectors lie along z (mu = 1), 4 across (mu = 0)."""
    n = 7
    x = _lattice(n)
    N = len(x)
    c, _ = oracle.count(x, kind="smu", edges1=[0.5, 1.2], edges2=synth.mu_edges(4), box=float(n))
    assert c[0].tolist() == [N * 4 // 2, 0, 0, N * 2 // 2]


@pytest.mark.parametrize("kind", ["s", "smu", "spi"])
@pytest.mark.parametrize("box", [0.0, 10.0])
def test_total_count_all_pairs(kind, box):
    """Bins covering every separation give N(N-1)/2 (auto) and N1*N2 (cross)."""
    rng = np.random.default_rng(3)
    x = rng.random((300, 3)) * 10.0
    y = rng.random((211, 3)) * 10.0
    big = 20.0  # > sqrt(3) * 10
    e2 = synth.mu_edges(7) if kind == "smu" else ([0, 3, 7, big] if kind == "spi" else None)
    e1 = [0, 1.5, 4, big]
    c, _ = oracle.count(x, kind=kind, edges1=e1, edges2=e2, box=box)
    assert c.sum() == 300 * 299 // 2
    c, _ = oracle.count(x, y, kind=kind, edges1=e1, edges2=e2, box=box)
    assert c.sum() == 300 * 211


def _binom2(n):
    return n * (n - 1) // 2


def test_uniform_periodic_expectation_s():
    """E[DD_k] = C(N,2) V_k/L^3 (Eq. npair_valid per shell); i.i.d. uniform points in a periodic
    box make pair indicators pairwise independent, so Var = C(N,2) p (1-p) exactly."""
    N, L = 4000, 100.0
    x = synth.uniform_box(N, L, 11)
    e = np.linspace(0, 25, 11)
    c, _ = oracle.count(x, kind="s", edges1=e, box=L)
    p = 4.0 * np.pi / 3.0 * (e[1:] ** 3 - e[:-1] ** 3) / L ** 3
    mean = _binom2(N) * p
    sd = np.sqrt(_binom2(N) * p * (1 - p))
    z = (c - mean) / sd
    assert np.all(np.abs(z) < 5.0), z


def test_uniform_periodic_expectation_smu():
    """Isotropy: each of n_mu equal mu bins of shell k holds V_k/n_mu of the volume."""
    N, L = 4000, 100.0
    x = synth.uniform_box(N, L, 12)
    e = np.linspace(0, 25, 6)
    nm = 5
    c, _ = oracle.count(x, kind="smu", edges1=e, edges2=synth.mu_edges(nm), box=L)
    p = (4.0 * np.pi / 3.0 * (e[1:] ** 3 - e[:-1] ** 3) / L ** 3)[:, None] / nm * np.ones((1, nm))
    mean = _binom2(N) * p
    sd = np.sqrt(_binom2(N) * p * (1 - p))
    z = (c - mean) / sd
    assert np.all(np.abs(z) < 5.0), z


def test_uniform_periodic_expectation_sigma_pi_zlos():
    """Line of sight z: the (sigma,pi) cell is a cylindrical ring of volume
    pi (sb^2 - sa^2) * 2 (pb - pa) (both signs of dz)."""
    N, L = 4000, 100.0
    x = synth.uniform_box(N, L, 13)
    es = np.linspace(0, 20, 5)
    ep = np.linspace(0, 20, 5)
    c, _ = oracle.count(x, kind="spi", los="z", edges1=es, edges2=ep, box=L)
    vs = np.pi * (es[1:] ** 2 - es[:-1] ** 2)
    vp = 2.0 * (ep[1:] - ep[:-1])
    p = vs[:, None] * vp[None, :] / L ** 3
    mean = _binom2(N) * p
    sd = np.sqrt(_binom2(N) * p * (1 - p))
    z = (c - mean) / sd
    assert np.all(np.abs(z) < 5.0), z


def test_midpoint_sphere_points_have_zero_pi():
    """Points on a sphere about the observer: (s2-s1).(s2+s1) = |s2|^2-|s1|^2 = 0, so pi = 0 and
    sigma = s.  Integer points with |v|^2 = 50 make every product exact."""
    pts = [v for v in itertools.product(range(-8, 9), repeat=3) if v[0] ** 2 + v[1] ** 2 + v[2] ** 2 == 50]
    x = np.array(pts, dtype=np.float64) + 0.0
    es = [0, 2, 4, 6, 8, 10, 12, 14, 16]
    c, _ = oracle.count(x, kind="spi", los="mid", edges1=es, edges2=[0, 1, 2])
    cs, _ = oracle.count(x, kind="s", edges1=es)
    assert (c[:, 1] == 0).all()
    assert (c[:, 0] == cs).all()
    assert c.sum() == len(x) * (len(x) - 1) // 2 - 0  # every pair within 2*sqrt(50) < 16


def test_midpoint_collinear_points_have_zero_sigma():
    """Points k*(1,2,2) on a ray from the observer: l is parallel to s, so pi = s = 3|k2-k1|, sigma = 0."""
    k = np.arange(1, 21)
    x = np.stack([k * 1.0, k * 2.0, k * 2.0], axis=1)
    ep = np.arange(0, 61, 3) - 0.5
    ep[0] = 0.0
    c, _ = oracle.count(x, kind="spi", los="mid", edges1=[0, 0.5, 10], edges2=ep)
    assert (c[1:] == 0).all()
    # pi = 3 m lies in bin m (edges 3m - 0.5 .. 3m + 2.5)
    expect = np.zeros(len(ep) - 1, dtype=np.int64)
    for m in range(1, 20):
        expect[m] = 20 - m
    assert c[0].tolist() == expect.tolist()


@pytest.mark.parametrize("kind,los,box", [("s", "z", 50.0), ("smu", "z", 50.0), ("spi", "z", 50.0),
                                          ("spi", "mid", 0.0), ("smu", "mid", 0.0), ("s", "z", 0.0)])
def test_exact_identities(kind, los, box):
    """Bit-exact identities: cross symmetry, cross(A,A) = 2 auto(A) + self pairs,
    auto(A u B) = auto(A) + auto(B) + cross(A,B), permutation invariance."""
    rng = np.random.default_rng(5)
    if box > 0:
        A = rng.random((250, 3)) * box
        B = rng.random((180, 3)) * box
    else:
        A = synth.survey_shell(250, 21, rmin=100.0, rmax=140.0)
        B = synth.survey_shell(180, 22, rmin=100.0, rmax=140.0)
    e1 = [0, 2, 5, 9, 14, 20]
    e2 = synth.mu_edges(6) if kind == "smu" else ([0, 3, 8, 15] if kind == "spi" else None)
    kw = dict(kind=kind, los=los, box=box, edges1=e1, edges2=e2)
    ab, _ = oracle.count(A, B, **kw)
    ba, _ = oracle.count(B, A, **kw)
    assert (ab == ba).all()
    aa_auto, _ = oracle.count(A, **kw)
    aa_cross, _ = oracle.count(A, A, **kw)
    self_pairs = np.zeros_like(aa_auto)
    self_pairs.ravel()[0] = len(A)   # s = 0 (and mu = 0, sigma = pi = 0) lands in the first bin
    assert (aa_cross == 2 * aa_auto + self_pairs).all()
    bb_auto, _ = oracle.count(B, **kw)
    u_auto, _ = oracle.count(np.concatenate([A, B]), **kw)
    assert (u_auto == aa_auto + bb_auto + ab).all()
    perm = rng.permutation(len(A))
    pa, _ = oracle.count(A[perm], **kw)
    assert (pa == aa_auto).all()


def test_marginal_and_nested_bins():
    """Summing (s,mu) over mu gives the s histogram; 5 fine linear bins sum to 1 coarse bin
    (squared edges 25k^2 and k^2 are exact integers)."""
    x = synth.uniform_box(1500, 200.0, 17)
    smu, _ = oracle.count(x, kind="smu", edges1=np.linspace(0, 60, 13), edges2=synth.mu_edges(10), box=200.0)
    s, _ = oracle.count(x, kind="s", edges1=np.linspace(0, 60, 13), box=200.0)
    assert (smu.sum(axis=1) == s).all()
    fine, _ = oracle.count(x, kind="s", edges1=np.arange(0, 61.0), box=200.0)
    assert (fine.reshape(12, 5).sum(axis=1) == s).all()


def test_scipy_kdtree_cumulative_counts():
    """Independent library: scipy cKDTree.count_neighbors counts pairs with d <= r; radii are
    chosen where no pair separation lies within 1e-9, so <= and < agree."""
    from scipy.spatial import cKDTree
    L = 100.0
    x = synth.uniform_box(1200, L, 19)
    e = np.array([0.0, 3.1, 7.7, 12.3, 18.9, 24.4])
    # no pair may sit on a radius
    d = x[:, None, :] - x[None, :, :]
    d = d - L * np.round(d / L)
    dist = np.sqrt((d ** 2).sum(-1))
    for r in e[1:]:
        assert np.abs(dist - r).min() > 1e-9
    c, _ = oracle.count(x, kind="s", edges1=e, box=L)
    t = cKDTree(x, boxsize=L)
    cum = (t.count_neighbors(t, e[1:]) - len(x)) // 2
    assert np.cumsum(c).tolist() == cum.tolist()
    # cross, open box
    y = synth.uniform_box(900, L, 20)
    c2, _ = oracle.count(x, y, kind="s", edges1=e)
    t1, t2 = cKDTree(x), cKDTree(y)
    assert np.cumsum(c2).tolist() == t1.count_neighbors(t2, e[1:]).tolist()


def test_weights_unit_and_powers_of_two():
    """Unit weights reproduce the counts; weights 2^a give bin sums that exact rational
    arithmetic fixes."""
    rng = np.random.default_rng(23)
    x = rng.random((400, 3)) * 30.0
    e = [0, 3, 6, 9, 12]
    c, wc = oracle.count(x, kind="s", edges1=e, box=30.0, w1=np.ones(400))
    assert (wc == c).all()
    a = rng.integers(-3, 4, size=400)
    w = np.ldexp(1.0, a)
    c, wc = oracle.count(x, kind="s", edges1=e, box=30.0, w1=w)
    exact = [Fraction(0)] * 4
    for i in range(400):
        for j in range(i + 1, 400):
            b = oracle.classify_pair(x[i], x[j], kind="s", edges1=e, box=30.0)
            if b >= 0:
                exact[b] += Fraction(2) ** int(a[i] + a[j])
    assert [float(v) for v in exact] == wc.tolist()


def test_weights_exactly_rounded_sum():
    """Each bin's weighted count equals math.fsum (a correctly rounded sum) of the FP64
    pair products; pins the 128-bit accumulation and its final rounding."""
    rng = np.random.default_rng(29)
    x = rng.random((300, 3)) * 20.0
    y = rng.random((250, 3)) * 20.0
    w = synth.uniform_weights(300, 0.5, 1.5, 1)
    v = synth.uniform_weights(250, 0.5, 2.0, 2)
    e = [0, 2, 5, 9, 14]
    c, wc = oracle.count(x, y, kind="s", edges1=e, box=20.0, w1=w, w2=v)
    terms = [[] for _ in range(4)]
    for i in range(300):
        for j in range(250):
            b = oracle.classify_pair(x[i], y[j], kind="s", edges1=e, box=20.0)
            if b >= 0:
                terms[b].append(float(w[i]) * float(v[j]))
    assert [len(t) for t in terms] == c.tolist()
    assert [math.fsum(t) for t in terms] == wc.tolist()


def test_no_fused_multiply_add():
    """A pair whose d^2 rounds differently with a fused multiply-add: the oracle must give the
    unfused IEEE result (the evaluation order written in its header)."""
    # search a pair where fma(dx,dx, dy*dy) != dx*dx + dy*dy and the unfused d2 is an edge
    rng = np.random.default_rng(31)
    for _ in range(100000):
        dx, dy = rng.random(2) * 10.0
        unfused = dx * dx + dy * dy
        fused = float(Fraction(dx) * Fraction(dx) + Fraction(dy * dy))
        fused = float(np.float64(fused))
        if fused != unfused:
            break
    else:
        pytest.skip("no witness found")
    edge = math.sqrt(unfused)
    # use E = unfused exactly as an edge: pick e with e*e == unfused if possible
    if edge * edge != unfused:
        pytest.skip("edge not representable")
    p1 = np.array([0.0, 0.0, 0.0])
    p2 = np.array([dx, dy, 0.0])
    b = oracle.classify_pair(p1, p2, kind="s", edges1=[0.0, edge, 2 * edge + 1.0])
    assert b == 1          # unfused d2 == edge^2 -> upper bin
