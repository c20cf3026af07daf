"""Pins of the angular oracle (oracle/angular.py) against closed forms and an
independent angle-based count."""
import numpy as np

from oracle import angular as A


def test_unit_vectors_and_chords():
    u = A.radec_to_unit([0.0, 90.0, 45.0, 123.0], [0.0, 0.0, 90.0, -30.0])
    assert np.allclose(np.linalg.norm(u, axis=1), 1.0, atol=1e-15)
    assert np.allclose(u[0], [1, 0, 0], atol=1e-15) and np.allclose(u[1], [0, 1, 0], atol=1e-15)
    assert np.allclose(u[2], [0, 0, 1], atol=1e-15)
    # 123 deg east, 30 deg south: spherical to Cartesian by hand
    assert np.allclose(u[3], [np.cos(np.pi / 6) * np.cos(123 * np.pi / 180),
                              np.cos(np.pi / 6) * np.sin(123 * np.pi / 180), -0.5], atol=1e-15)
    c = A.chord_edges([0.0, 60.0, 90.0, 180.0])
    assert np.allclose(c, [0.0, 1.0, np.sqrt(2.0), 2.0], rtol=1e-15, atol=0)


def _sphere(n, seed):
    rng = np.random.default_rng(seed)
    ra = rng.uniform(0.0, 360.0, n)
    dec = np.rad2deg(np.arcsin(rng.uniform(-1.0, 1.0, n)))
    return ra, dec


def test_uniform_sky_matches_cap_areas():
    """Uniform points on the sphere: a pair's angle falls in [t1, t2) with
    probability (cos t1 - cos t2) / 2 (area of a spherical zone over 4 pi);
    pairs sharing a point are independent for uniform points, so the variance
    is C(N,2) p (1 - p): every bin within 5 sigma."""
    ra, dec = _sphere(3000, 4)
    u = A.radec_to_unit(ra, dec)
    th = np.array([0.0, 2.0, 5.0, 10.0, 20.0, 45.0, 90.0, 135.0, 180.0])
    c, _ = A.angular_count(u, chord=A.chord_edges(th))
    npair = len(u) * (len(u) - 1) / 2
    p = (np.cos(np.deg2rad(th[:-1])) - np.cos(np.deg2rad(th[1:]))) / 2.0
    mu = npair * p
    sd = np.sqrt(npair * p * (1 - p))
    assert c.sum() == npair
    assert np.all(np.abs(c - mu) <= 5 * sd), (c, mu, sd)


def test_chord_bins_equal_angle_bins():
    """The chord-binned count equals the count binned by the angle itself
    (arccos of the dot product) on random points, where no pair falls within
    rounding of an edge."""
    ra, dec = _sphere(800, 7)
    u = A.radec_to_unit(ra, dec)
    th = np.linspace(0.0, 180.0, 37)
    c, _ = A.angular_count(u, chord=A.chord_edges(th))
    assert np.array_equal(c, A.angle_bins_brute(u, th))


def test_hand_pairs():
    """Points at known angles: 1, 30 and 120 degrees apart along the equator."""
    u = A.radec_to_unit([0.0, 1.0, 31.0, 151.0], [0.0, 0.0, 0.0, 0.0])
    th = np.array([0.0, 0.5, 1.5, 29.5, 30.5, 119.5, 120.5, 180.0])
    c, _ = A.angular_count(u, chord=A.chord_edges(th))
    # pairs: 1 (0-1), 31 (0-31), 151 (0-151), 30 (1-31), 150 (1-151), 120 (31-151)
    assert list(c) == [0, 1, 0, 1, 1, 1, 2]
