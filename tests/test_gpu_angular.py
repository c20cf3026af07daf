"""Angular pair counts on the GPU: sky positions to unit vectors (within two
ulps of the FP64 formula), then chord-binned counts equal to the oracle's on
the same unit vectors, bit for bit, and the closed form of a uniform sky."""
import numpy as np
import pytest

from oracle import angular as A
from helpers import note, to_dev, assert_same

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _sky(n, seed, dec_lo=-90.0, dec_hi=90.0, ra_hi=360.0):
    rng = np.random.default_rng(seed)
    s0, s1 = np.sin(np.deg2rad(dec_lo)), np.sin(np.deg2rad(dec_hi))
    return rng.uniform(0.0, ra_hi, n), np.rad2deg(np.arcsin(rng.uniform(s0, s1, n)))


def test_radec_to_unit():
    from paper_2301_12557_amd import fcfc
    ra, dec = _sky(100000, 1)
    ra[:4] = [0.0, 90.0, 180.0, 359.999]
    dec[:4] = [0.0, 90.0, -90.0, 45.0]
    u = fcfc.radec_to_unit(to_dev(ra), to_dev(dec)).cpu().numpy()
    ref = A.radec_to_unit(ra, dec)
    assert np.max(np.abs(u - ref)) <= 4.5e-16
    assert np.max(np.abs(np.linalg.norm(u, axis=1) - 1.0)) <= 1e-15


@pytest.mark.parametrize("weighted", [False, True])
def test_angular_counts_match_oracle(weighted):
    """Auto and cross counts of a survey-like patch, small and large angles."""
    import torch
    from paper_2301_12557_amd import fcfc
    ra1, dec1 = _sky(6000, 2, dec_lo=-10.0, dec_hi=30.0, ra_hi=80.0)
    ra2, dec2 = _sky(9000, 3, dec_lo=-10.0, dec_hi=30.0, ra_hi=80.0)
    u1 = fcfc.radec_to_unit(to_dev(ra1), to_dev(dec1))
    u2 = fcfc.radec_to_unit(to_dev(ra2), to_dev(dec2))
    w1 = A_w = None
    if weighted:
        rng = np.random.default_rng(5)
        A_w = (rng.uniform(0.5, 2.0, len(ra1)), rng.uniform(0.5, 2.0, len(ra2)))
    th = np.concatenate([[0.0], np.logspace(-2, 1, 16)])
    for cross in (False, True):
        note(f"angular weighted={weighted} cross={cross}")
        kw = dict(w1=to_dev(A_w[0]) if weighted else None, w2=to_dev(A_w[1]) if (weighted and cross) else None)
        c, wc, chord = fcfc.angular_count(u1, u2 if cross else None, theta_deg=th, **kw)
        o, ow = A.angular_count(u1.cpu().numpy(), u2.cpu().numpy() if cross else None, chord=chord,
                                w1=A_w[0] if weighted else None, w2=A_w[1] if (weighted and cross) else None)
        assert_same(c.cpu().numpy(), o, wc.cpu().numpy() if weighted else None, ow, what=f"angular cross={cross}")
        assert int(c.sum()) > 1000


def test_uniform_sky_closed_form():
    """Uniform points over the whole sky: each zone [t1, t2) holds C(N,2)(cos t1 -
    cos t2)/2 pairs on average with variance C(N,2) p (1 - p); 5 sigma."""
    from paper_2301_12557_amd import fcfc
    ra, dec = _sky(200000, 9)
    u = fcfc.radec_to_unit(to_dev(ra), to_dev(dec))
    th = np.array([0.0, 0.1, 0.3, 1.0, 2.0, 4.0])
    c, _, _ = fcfc.angular_count(u, theta_deg=th)
    c = c.cpu().numpy()
    npair = len(ra) * (len(ra) - 1) / 2
    p = (np.cos(np.deg2rad(th[:-1])) - np.cos(np.deg2rad(th[1:]))) / 2.0
    mu, sd = npair * p, np.sqrt(npair * p * (1 - p))
    note(f"uniform sky: {c} vs {mu.round()}")
    assert np.all(np.abs(c - mu) <= 5 * sd)
