"""The learned cost model on the GPU: forward, gradient and Adam kernels against
the float64 CPU oracle (oracle/mlp.py), training, the learned work order (which
must leave every count unchanged) and the cell-size chooser.

Tolerances (FP32 kernels vs FP64 oracle):
* forward: each layer is a 64-term FP32 dot product; with u = 2^-24 the error
  is below ~64 u times the sum of |terms|, so for three hidden layers and the
  output we allow 3e-5 times A, where A is the output of the same network with
  |W|, |b| and |x| (an upper bound of every sum of |terms|), in target units;
* gradient: sums over up to m samples accumulated with FP32 atomics in any
  order: 1e-3 of the largest |component| of the same parameter group;
* one Adam step: the step is lr * g / (|g| + eps), i.e. +-lr wherever |g| is
  well above the rounding of g; compared there to 1e-3 lr, elsewhere bounded by lr.
"""
import ctypes

import numpy as np
import pytest

from oracle import mlp as M
from paper_2301_12557_amd import synth
from helpers import note, to_dev, oracle_count, assert_same

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _params(seed, scale=0.25):
    rng = np.random.default_rng(seed)
    return rng.normal(0.0, scale, M.NPARAM).astype(np.float32)


def _norm():
    return np.array([1.0, -2.0, 0.5, 3.0, 2.0, 1.5, 0.7, 1.2, 4.0, 2.5], dtype=np.float32)


def _abs_bound(params, norm, feat):
    """Output scale bound: the network with absolute weights on |standardised x|."""
    P = M.unpack(params)
    x = np.abs(M.standardise(feat, norm))
    h = np.abs(P["b1"]) + x @ np.abs(P["W1"]).T
    h = np.abs(P["b2"]) + h @ np.abs(P["W2"]).T
    h = np.abs(P["b3"]) + h @ np.abs(P["W3"]).T
    return (np.abs(P["b4"]) + h @ np.abs(P["W4"])) * float(norm[9])


def test_forward_matches_oracle():
    import torch
    from paper_2301_12557_amd import fcfc
    rng = np.random.default_rng(1)
    for m in (1, 63, 1000, 4097):
        p = _params(10 + m)
        nrm = _norm()
        feat = rng.normal(0, 2, (m, 4)).astype(np.float32)
        note(f"mlp forward m={m}")
        md = fcfc.Model(seed=1)
        md.set(p, nrm)
        y = md.predict(torch.from_numpy(feat).cuda()).cpu().numpy().astype(np.float64)
        ref = M.predict(p.astype(np.float64), nrm.astype(np.float64), feat.astype(np.float64))
        tol = 3e-5 * _abs_bound(p.astype(np.float64), nrm.astype(np.float64), feat.astype(np.float64)) + 1e-6
        assert np.all(np.abs(y - ref) <= tol), np.max(np.abs(y - ref) / tol)
        md.close()


def test_gradient_matches_oracle():
    import torch
    from paper_2301_12557_amd import fcfc
    rng = np.random.default_rng(2)
    offs = np.cumsum([0] + [int(np.prod(s)) for _, s in M.SIZES])
    for m in (64, 777):
        p = _params(20 + m)
        nrm = _norm()
        feat = rng.normal(0, 2, (m, 4)).astype(np.float32)
        tgt = rng.normal(4, 3, m).astype(np.float32)
        note(f"mlp grad m={m}")
        md = fcfc.Model(seed=2)
        md.set(p, nrm)
        g, loss = md.grad(torch.from_numpy(feat).cuda(), torch.from_numpy(tgt).cuda())
        rl, rg = M.loss_and_grad(p.astype(np.float64), nrm.astype(np.float64), feat.astype(np.float64),
                                 tgt.astype(np.float64))
        assert loss == pytest.approx(rl, rel=1e-4)
        for (name, _), a, b in zip(M.SIZES, offs[:-1], offs[1:]):
            scale = np.max(np.abs(rg[a:b]))
            err = np.max(np.abs(g[a:b].astype(np.float64) - rg[a:b]))
            assert err <= 1e-3 * scale + 1e-6, (name, err, scale)
        md.close()


def test_one_adam_step_matches_oracle():
    """train(epochs=1, batch=m): normalisation from the data, then exactly one
    Adam step on the mean gradient of all m samples."""
    import torch
    from paper_2301_12557_amd import fcfc
    rng = np.random.default_rng(3)
    m, lr = 500, 1e-2
    feat = rng.normal(0, 2, (m, 4)).astype(np.float32)
    tgt = (feat[:, 0] - 0.5 * feat[:, 1] + rng.normal(0, 0.1, m)).astype(np.float32)
    md = fcfc.Model(seed=77)
    p0, _ = md.get()
    md.train(torch.from_numpy(feat).cuda(), torch.from_numpy(tgt).cuda(), epochs=1, batch=m, lr=lr, seed=5)
    p1, nrm = md.get()
    ref_norm = M.fit_norm(feat.astype(np.float64), tgt.astype(np.float64))
    assert np.allclose(nrm, ref_norm, rtol=1e-5, atol=1e-6)
    _, g = M.loss_and_grad(p0.astype(np.float64), nrm.astype(np.float64), feat.astype(np.float64),
                           tgt.astype(np.float64))
    g /= m
    ref, _, _ = M.adam_step(p0.astype(np.float64), g, np.zeros_like(g), np.zeros_like(g), 1, lr)
    d = p1.astype(np.float64) - p0
    dref = ref - p0
    big = np.abs(g) > 1e-3 * np.max(np.abs(g))
    assert np.all(np.abs(d[big] - dref[big]) <= 1e-3 * lr + 1e-7)
    assert np.all(np.abs(d) <= lr * (1 + 1e-5) + 1e-7)
    md.close()


def test_training_fits_a_smooth_target():
    import torch
    from paper_2301_12557_amd import fcfc
    rng = np.random.default_rng(4)
    m = 20000
    na = rng.integers(1, 129, m)
    nb = rng.integers(1, 4096, m)
    sep = rng.uniform(0, 4, m)
    k = rng.integers(1, 6, m)
    feat = np.stack([np.log2(1 + na), np.log2(1 + nb), sep, k], axis=1).astype(np.float32)
    tgt = (np.log2(1 + na * nb * (1 - 0.1 * sep)) + 0.2 * k).astype(np.float32)
    md = fcfc.Model(seed=3)
    loss = md.train(torch.from_numpy(feat).cuda(), torch.from_numpy(tgt).cuda(), epochs=30, batch=256, lr=2e-3,
                    seed=1)
    note(f"final mean loss {loss}")
    # a constant predictor has mean loss 0.5 in standardised units
    assert loss < 0.01
    pred = md.predict(torch.from_numpy(feat).cuda()).cpu().numpy()
    assert np.corrcoef(pred, tgt)[0, 1] > 0.99
    md.close()


def test_save_load_roundtrip(tmp_path):
    from paper_2301_12557_amd import fcfc
    md = fcfc.Model(seed=9)
    md.set(_params(9), _norm())
    f = tmp_path / "m.bin"
    md.save(str(f))
    m2 = fcfc.Model(path=str(f))
    a, na = md.get()
    b, nb = m2.get()
    assert np.array_equal(a, b) and np.array_equal(na, nb)
    md.close()
    m2.close()


def _catalogue(n=30000, L=500.0, seed=12):
    return synth.lognormal_box(n, L, seed, ngrid=64)


def _trained_model(plan, cells, epochs=20):
    from paper_2301_12557_amd import fcfc
    plan.count(cells)
    feat, logt = plan.timings()
    md = fcfc.Model(seed=5)
    md.train(feat, logt, epochs=epochs, batch=256, lr=2e-3, seed=2)
    return md, feat, logt


def test_timings_and_learned_order_keep_counts():
    """Timings are recorded per item; ordering by the trained model leaves the
    counts bit-exact (they equal the oracle's) and the stats say which order ran."""
    import torch
    from paper_2301_12557_amd import fcfc
    L = 500.0
    x = _catalogue(L=L)
    e1 = synth.linear_edges(0, 40, 20)
    e2 = synth.mu_edges(10)
    dx = to_dev(x)
    plan = fcfc.Plan("smu", e1, e2, box=L, n_hint=len(x), record_timing=1)
    c = plan.build_cells(dx)
    md, feat, logt = _trained_model(plan, c)
    st = plan.stats()
    assert feat.shape == (st["items"], 4) and logt.shape == (st["items"],)
    f = feat.cpu().numpy()
    t = logt.cpu().numpy()
    assert np.all(np.isfinite(f)) and np.all(t > 0)
    assert np.all(f[:, 3] == np.float32(plan_kcells(st, e1)))
    assert np.all(f[:, 0] <= np.log2(129.0) + 1e-6)
    pred = md.predict(feat).cpu().numpy()
    note(f"items {len(t)} corr(pred, log t) = {np.corrcoef(pred, t)[0, 1]:.3f}")
    assert np.corrcoef(pred, t)[0, 1] > 0.5

    ref, _ = oracle_count(x, kind="smu", edges1=e1, edges2=e2, box=L)
    for order, model, want in (("built", None, "built"), ("heuristic", None, "heuristic"),
                               ("learned", md, "learned"), ("learned", None, "heuristic")):
        p2 = fcfc.Plan("smu", e1, e2, box=L, n_hint=len(x), order=order)
        p2.set_model(model)
        c2 = p2.build_cells(dx)
        got, _ = p2.count(c2)
        assert_same(got.cpu().numpy(), ref, what=f"order {order}")
        assert p2.stats()["order_used"] == want
        c2.close()
        p2.close()
    # a model whose predictions are not finite falls back to the heuristic key
    bad = fcfc.Model(seed=1)
    pb, nb = md.get()
    pb[-1] = np.nan
    bad.set(pb, nb)
    p3 = fcfc.Plan("smu", e1, e2, box=L, n_hint=len(x), order="learned")
    p3.set_model(bad)
    c3 = p3.build_cells(dx)
    got, _ = p3.count(c3)
    assert_same(got.cpu().numpy(), ref, what="nan model")
    assert p3.stats()["order_used"] == "heuristic"
    c.close()
    plan.close()


def plan_kcells(st, e1):
    return float(e1[-1]) / st["cell_side"]


def test_predict_and_choose_cells():
    import torch
    from paper_2301_12557_amd import fcfc
    L = 500.0
    x = _catalogue(L=L)
    e1 = synth.linear_edges(0, 40, 20)
    e2 = synth.mu_edges(10)
    dx = to_dev(x)
    plan = fcfc.Plan("smu", e1, e2, box=L, n_hint=len(x), record_timing=1)
    c = plan.build_cells(dx)
    md, _, _ = _trained_model(plan, c)
    st = plan.stats()
    ms, n = plan.predict(md, c)
    note(f"predicted {ms:.3f} ms, measured {st['kernel_ms']:.3f} ms, items {n}")
    assert n == st["items"] and np.isfinite(ms) and ms > 0
    k, pred = fcfc.choose_cells(dx, model=md, kind="smu", edges1=e1, edges2=e2, box=L)
    note(f"learned k={k} predictions {pred}")
    assert 1 <= k <= 6 and np.isfinite(pred[k - 1]) and pred[k - 1] == min(v for v in pred if np.isfinite(v))
    k0, pred0 = fcfc.choose_cells(dx, model=None, kind="smu", edges1=e1, edges2=e2, box=L)
    assert k0 == st["cells_per_rmax"] and all(np.isnan(v) for v in pred0)
    # the chosen k counts exactly like any other
    ref, _ = oracle_count(x, kind="smu", edges1=e1, edges2=e2, box=L)
    got, _ = fcfc.count_pairs(dx, kind="smu", edges1=e1, edges2=e2, box=L, cells_per_rmax=k)
    assert_same(got.cpu().numpy(), ref, what=f"k={k}")
    c.close()
    plan.close()
