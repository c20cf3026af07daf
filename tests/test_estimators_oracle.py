"""Pins of the estimator oracle (oracle/estimators.py) by hand values, closed
forms and the counting oracle on uniform boxes."""
import numpy as np
import pytest

import oracle
from oracle import estimators as E
from paper_2301_12557_amd import synth


def test_linear_estimators_by_hand():
    dd, dr, rr = np.array([30.0, 10.0]), np.array([50.0, 40.0]), np.array([40.0, 0.0])
    n = [10.0, 20.0, 40.0]
    # LS by hand: (30/10 - 2*50/20 + 40/40) / (40/40) = 3 - 5 + 1 = -1; second bin: zero RR -> NaN
    ls = E.xi_linear([dd, dr, rr], [1, -2, 1], n, 2)
    assert ls[0] == -1.0 and np.isnan(ls[1])
    # PH by hand: (30/10) / (40/40) - 1 = 2
    assert E.xi_linear([dd, rr], [1, -1], [10.0, 40.0], 1)[0] == 2.0
    # counts in proportion to their pair numbers give xi = 0
    assert E.xi_linear([rr * 0.25, rr * 0.5, rr], [1, -2, 1], [10.0, 20.0, 40.0], 2)[0] == 0.0


def test_bin_volumes_closed_forms():
    e = np.array([0.0, 1.0, 2.0, 3.5])
    v = E.bin_volumes("s", e)
    assert v.sum() == pytest.approx(4.0 / 3.0 * np.pi * 3.5 ** 3, rel=1e-15)
    vmu = E.bin_volumes("smu", e, synth.mu_edges(7))
    assert np.allclose(vmu.sum(axis=1), v, rtol=1e-15)           # mu bins partition the sphere
    vp = E.bin_volumes("spi", e, np.array([0.0, 0.5, 2.0]))
    assert vp.sum() == pytest.approx(np.pi * 3.5 ** 2 * 2 * 2.0, rel=1e-15)   # cylinder of height 2 pi_max


@pytest.mark.parametrize("kind", ["s", "smu", "spi"])
def test_analytic_rr_matches_uniform_box_counts(kind):
    """The oracle's counts of uniform periodic points lie within 5 sigma of the
    analytic RR (variance C(N,2) p (1 - p) for i.i.d. uniform points)."""
    n, L = 4000, 100.0
    x = synth.uniform_box(n, L, 77)
    e1 = synth.linear_edges(0, 12, 6)
    e2 = synth.mu_edges(4) if kind == "smu" else (synth.linear_edges(0, 10, 5) if kind == "spi" else None)
    c, _ = oracle.count(x, kind=kind, edges1=e1, edges2=e2, box=L)
    npairs = n * (n - 1) / 2.0
    rr = E.analytic_rr(kind, e1, e2, L, npairs)
    p = rr / npairs
    sig = np.sqrt(npairs * p * (1 - p))
    assert np.all(np.abs(c - rr) <= 5 * sig + 1e-9), np.max(np.abs(c - rr) / sig)


def test_multipoles_closed_forms():
    mu = synth.mu_edges(200)
    const = np.full((3, 200), 2.5)
    m = E.multipoles(const, mu, (0, 2, 4))
    assert np.allclose(m[0], 2.5, rtol=1e-14) and np.all(np.abs(m[1:]) < 1e-12)
    # bin averages of P_2: xi_0 = 0 exactly (P_2 integrates to 0), xi_2 -> 1 as bins shrink
    p2 = E.legendre_bin_integrals(2, mu) / np.diff(mu)
    m = E.multipoles(p2[None, :], mu, (0, 2, 4))
    assert abs(m[0, 0]) < 1e-14 and m[1, 0] == pytest.approx(1.0, abs=1e-4) and abs(m[2, 0]) < 1e-4
    # P_2 by hand: (3 mu^2 - 1) / 2 integrates over [0, 1/2] to (1/8 - 1/2) / 2 = -3/16
    assert E.legendre_bin_integrals(2, [0.0, 0.5])[0] == pytest.approx(-3.0 / 16.0, rel=1e-15)


def test_wp_closed_form():
    pe = np.array([0.0, 3.0, 10.0, 40.0])
    assert np.allclose(E.wp(np.full((2, 3), 0.7), pe), 2 * 0.7 * 40.0, rtol=1e-15)
    x = np.array([[1.0, 2.0, 3.0]])
    assert E.wp(x, pe)[0] == 2 * (1 * 3 + 2 * 7 + 3 * 30)
