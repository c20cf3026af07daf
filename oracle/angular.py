"""Angular pair counts -- TEST INFRASTRUCTURE ONLY (oracle of the angular
extension: the dual-tree method applies to angular pairs directly, Sect. 3.1;
angular statistics are the future work of Sect. 6).

Definitions, in FP64:
* a position on the sky (right ascension alpha, declination delta, degrees)
  is the unit vector (cos delta cos alpha, cos delta sin alpha, sin delta);
* the angle theta between two such points maps one to one onto the chord
  c = |u - v| = 2 sin(theta / 2) on [0, 180] degrees, so an angular bin
  [theta_k, theta_k+1) is the chord bin [2 sin(theta_k / 2), 2 sin(theta_k+1 / 2)).
  The chord bins of the unit vectors are the counted quantity (the squared
  chord against squared chord edges, as every separation here).
"""
import numpy as np

from . import count as _count


def radec_to_unit(ra_deg, dec_deg):
    """Unit vectors of sky positions (degrees), FP64, N x 3."""
    a = np.deg2rad(np.asarray(ra_deg, dtype=np.float64))
    d = np.deg2rad(np.asarray(dec_deg, dtype=np.float64))
    cd = np.cos(d)
    return np.stack([cd * np.cos(a), cd * np.sin(a), np.sin(d)], axis=1)


def chord_edges(theta_deg):
    """Chord lengths 2 sin(theta / 2) of angular edges in degrees."""
    t = np.asarray(theta_deg, dtype=np.float64)
    return 2.0 * np.sin(np.deg2rad(t) / 2.0)


def angular_count(u1, u2=None, *, chord, w1=None, w2=None):
    """Pair counts of unit vectors in the chord bins `chord` (auto when u2 is None)."""
    return _count(u1, u2, kind="s", edges1=chord, box=0.0, w1=w1, w2=w2)


def angle_bins_brute(u1, theta_deg):
    """Auto-pair counts binned by the angle itself (arccos of the dot product),
    for the tests: equal to the chord bins except for pairs within rounding of
    an edge."""
    u1 = np.asarray(u1, dtype=np.float64)
    n = len(u1)
    i, j = np.triu_indices(n, 1)
    c = np.clip((u1[i] * u1[j]).sum(1), -1.0, 1.0)
    th = np.rad2deg(np.arccos(c))
    h, _ = np.histogram(th, bins=np.asarray(theta_deg, dtype=np.float64))
    return h
