"""Pins of the histogram-update oracle (oracle/histogram.py): closed forms on
integer edges, the half-open rule at the edges themselves, a brute-force walk
over the edges, binning by the separation itself, and the s^2 law of the
benchmark input (App. C)."""
import numpy as np

from oracle import histogram as H
from paper_2301_12557_amd import synth


def test_integer_lattice_closed_form():
    """Edges e_k = 5 k have exact squares 25 k^2; the integers 0 .. 25 n^2 + 99
    put 25 ((i+1)^2 - i^2) = 25 (2 i + 1) values in bin i and none past the top."""
    n = 40
    v = np.arange(25 * n * n + 100, dtype=np.float64)
    h = H.bin_squared(v, synth.linear_edges(0, 5 * n, n), chunk=1000)
    assert h.dtype == np.int64
    assert np.array_equal(h, 25 * (2 * np.arange(n) + 1))
    assert h.sum() == 25 * n * n


def test_half_open_edges_and_special_values():
    e = np.array([0.0, 1.0, 2.5, 7.0, 200.0])
    E = e * e
    below = np.nextafter(E, -np.inf)
    vals = np.concatenate([E, below[1:], [np.nan, -1.0, -1e-300, np.inf, -0.0, 1e300]])
    b = H.bin_index_brute(vals, e)
    # each squared edge opens its own bin; the top edge closes the range
    assert list(b[:5]) == [0, 1, 2, 3, -1]
    # one ulp below an edge is still in the bin underneath
    assert list(b[5:9]) == [0, 1, 2, 3]
    # NaN, negatives, infinity and huge values land nowhere; -0.0 compares equal to 0
    assert list(b[9:]) == [-1, -1, -1, -1, 0, -1]
    h = H.bin_squared(vals, e)
    assert np.array_equal(h, np.bincount(b[b >= 0], minlength=4))
    assert list(h) == [3, 2, 2, 2]


def test_matches_brute_walk_on_random_values():
    rng = np.random.default_rng(5)
    for edges in (synth.linear_edges(0, 200, 20), synth.log_edges(0.1, 200, 20), [3.0, 3.5, 80.0]):
        v = np.concatenate([rng.uniform(-10, 41000, 3000), np.asarray(edges) ** 2])
        b = H.bin_index_brute(v, edges)
        n = len(edges) - 1
        assert np.array_equal(H.bin_squared(v, edges, chunk=777), np.bincount(b[b >= 0], minlength=n))


def test_agrees_with_binning_the_separation_itself():
    """Away from rounding distance of an edge, binning s^2 against e^2 is
    binning s against e (numpy's histogram of the square roots)."""
    v = synth.s2_samples(200000, 200.0, 11)
    for edges in (synth.linear_edges(0, 200, 200), synth.log_edges(0.1, 200, 200)):
        E = np.asarray(edges) ** 2
        gap = np.min(np.abs(v[:, None] - E[None, :]) / E[None, :].clip(1e-300), axis=1)
        assert gap.min() > 1e-12
        ref, _ = np.histogram(np.sqrt(v), bins=np.asarray(edges))
        assert np.array_equal(H.bin_squared(v, edges), ref)


def test_benchmark_input_follows_s_squared_law():
    """s^2 = x^(2/3) R^2 with x uniform gives P(s < t) = (t / R)^3: the count of
    bin [a, b) has mean N (b^3 - a^3) / R^3 and binomial spread; every bin of
    the linear and logarithmic layouts within 5 sigma."""
    N, R = 2_000_000, 200.0
    v = synth.s2_samples(N, R, 7)
    for edges in (synth.linear_edges(0, R, 20), synth.log_edges(0.1, R, 20), synth.linear_edges(0, R, 200)):
        e = np.asarray(edges)
        p = (e[1:] ** 3 - e[:-1] ** 3) / R ** 3
        h = H.bin_squared(v, e)
        sd = np.sqrt(N * p * (1 - p))
        assert np.all(np.abs(h - N * p) <= 5 * sd + 1)
