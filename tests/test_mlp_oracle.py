"""Pins of the cost-model oracle (oracle/mlp.py) against facts that do not come
from the oracle itself: finite differences of its own forward pass, networks
built so that the output follows by index chasing, and closed forms of the
Adam update."""
import numpy as np
import pytest

from oracle import mlp as M


def _rand_params(seed, scale=0.3):
    rng = np.random.default_rng(seed)
    return rng.normal(0.0, scale, M.NPARAM)


def _norm(seed):
    rng = np.random.default_rng(seed)
    return np.concatenate([rng.normal(0, 2, 4), rng.uniform(0.5, 3, 4), [rng.normal()], [rng.uniform(0.5, 2)]])


def test_layout_size():
    # 4*64 + 64 + 2*(64*64 + 64) + 64 + 1
    assert M.NPARAM == 8705
    p = np.arange(M.NPARAM, dtype=np.float64)
    P = M.unpack(p)
    assert P["W1"][0, 1] == 1 and P["W1"][1, 0] == 4          # row-major [out][in]
    assert P["b1"][0] == 256 and P["W2"][0, 0] == 320
    assert P["b4"] == M.NPARAM - 1
    assert np.array_equal(M.pack(P), p)


def test_gradient_matches_central_differences():
    """Every parameter group: analytic gradient = (L(p+h) - L(p-h)) / 2h."""
    rng = np.random.default_rng(5)
    p = _rand_params(1)
    nrm = _norm(2)
    feat = rng.normal(0, 2, (23, 4))
    tgt = rng.normal(0, 1, 23)
    loss, g = M.loss_and_grad(p, nrm, feat, tgt)
    offs = np.cumsum([0] + [int(np.prod(s)) for _, s in M.SIZES])
    idx = []
    for a, b in zip(offs[:-1], offs[1:]):
        idx += list(rng.choice(np.arange(a, b), size=min(12, b - a), replace=False))
    h = 1e-6
    for i in idx:
        pp = p.copy(); pp[i] += h
        pm = p.copy(); pm[i] -= h
        fd = (M.loss_and_grad(pp, nrm, feat, tgt)[0] - M.loss_and_grad(pm, nrm, feat, tgt)[0]) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(g[i])), (i, fd, g[i])
    # the loss itself: 0.5 * sum of squared standardised residuals
    y = M.predict(p, nrm, feat)
    assert loss == pytest.approx(0.5 * np.sum(((y - tgt) / nrm[9]) ** 2), rel=1e-12)


def test_forward_by_index_chasing():
    """W1 picks feature f(o) with sign, W2 and W3 permute units, W4 selects one
    unit: the output is one input feature (or 0), found without any product."""
    rng = np.random.default_rng(3)
    P = {k: np.zeros(s) for k, s in M.SIZES}
    f_of = rng.integers(0, 4, 64)
    sign = np.where(rng.random(64) < 0.5, -1.0, 1.0)
    for o in range(64):
        P["W1"][o, f_of[o]] = sign[o]
    perm2 = rng.permutation(64)   # h2[o] = h1[perm2[o]]
    perm3 = rng.permutation(64)   # h3[o] = h2[perm3[o]]
    for o in range(64):
        P["W2"][o, perm2[o]] = 1.0
        P["W3"][o, perm3[o]] = 1.0
    j = 17
    P["W4"][j] = 2.5
    P["b4"] = -1.25
    p = M.pack(P)
    x = rng.normal(0, 1, (50, 4))
    y, _ = M.forward(p, x)
    u = perm2[perm3[j]]            # h3[j] = h2[perm3[j]] = h1[perm2[perm3[j]]]
    want = 2.5 * np.maximum(sign[u] * x[:, f_of[u]], 0.0) - 1.25
    assert np.array_equal(y, want)
    # the test tells the wiring apart: transposed W2, W3 select another unit
    inv2, inv3 = np.argsort(perm2), np.argsort(perm3)
    assert inv2[inv3[j]] != u
    Pt = dict(P)
    Pt["W2"], Pt["W3"] = P["W2"].T.copy(), P["W3"].T.copy()
    yt, _ = M.forward(M.pack(Pt), x)
    assert not np.array_equal(yt, want)


def test_zero_network_and_dead_relus():
    P = {k: np.zeros(s) for k, s in M.SIZES}
    P["b4"] = 0.75
    P["b1"][:] = -5.0               # every first-layer unit dead for |x| < 1
    rng = np.random.default_rng(0)
    P["W1"] = rng.uniform(-1, 1, (64, 4)) / 4.0
    p = M.pack(P)
    nrm = np.array([0, 0, 0, 0, 1, 1, 1, 1, 0, 1.0])
    x = rng.uniform(-1, 1, (10, 4))
    t = rng.normal(0, 1, 10)
    loss, g = M.loss_and_grad(p, nrm, x, t)
    assert np.all(M.predict(p, nrm, x) == 0.75)
    G = M.unpack(g)
    assert G["b4"] == pytest.approx(np.sum(0.75 - t), rel=1e-14)
    for k in ("W1", "b1", "W2", "b2", "W3", "b3", "W4"):
        assert np.all(G[k] == 0), k


def test_standardisation():
    nrm = np.array([1.0, 2.0, 3.0, 4.0, 2.0, 4.0, 8.0, 16.0, 10.0, 3.0])
    P = {k: np.zeros(s) for k, s in M.SIZES}
    P["W1"][0, 2] = 1.0             # h1[0] = relu((x2 - 3) / 8)
    P["W2"][0, 0] = 1.0
    P["W3"][0, 0] = 1.0
    P["W4"][0] = 1.0
    feat = np.array([[0.0, 0.0, 19.0, 0.0], [0.0, 0.0, -5.0, 0.0]])
    y = M.predict(M.pack(P), nrm, feat)
    assert np.array_equal(y, [3.0 * 2.0 + 10.0, 10.0])


def test_adam_closed_forms():
    """First step moves each parameter by lr * sign(g) (|g| >> eps); with a
    constant gradient every later step does too (bias corrections cancel)."""
    rng = np.random.default_rng(1)
    p = rng.normal(0, 1, 50)
    g = rng.choice([-1.0, 1.0], 50) * rng.uniform(0.5, 2.0, 50)
    m1 = np.zeros(50)
    m2 = np.zeros(50)
    q = p.copy()
    for t in range(1, 6):
        q, m1, m2 = M.adam_step(q, g, m1, m2, t, lr=0.01)
        step = np.abs(p - q) / t
        assert np.allclose(step, 0.01, rtol=1e-6)
    assert np.array_equal(np.sign(p - q), np.sign(g))
    # moments after one step from zero
    _, a, b = M.adam_step(p, g, np.zeros(50), np.zeros(50), 1, lr=0.1)
    assert np.allclose(a, 0.1 * g, rtol=1e-15) and np.allclose(b, 0.001 * g * g, rtol=1e-13)


def test_fit_norm():
    f = np.array([[1.0, 2, 3, 4], [3.0, 2, 5, 8]])
    n = M.fit_norm(f, np.array([0.0, 2.0]))
    assert np.allclose(n, [2, 2, 4, 6, 1, 1e-3, 1, 2, 1, 1])
