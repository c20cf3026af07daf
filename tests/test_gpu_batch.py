"""Batched pipeline: many periodic catalogues counted in one launch (optionally a HIP
graph) must give, catalogue by catalogue, the oracle's histograms."""
import numpy as np
import pytest

from paper_2301_12557_amd import synth
from helpers import note, oracle_count, assert_same, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _mocks(ncat, L, seed, lo=300, hi=2500, weighted=False):
    rng = np.random.default_rng(seed)
    sizes = rng.integers(lo, hi + 1, size=ncat)
    xs = [synth.lognormal_box(int(n), L, seed * 1000 + m, ngrid=32) for m, n in enumerate(sizes)]
    ws = [synth.uniform_weights(int(n), 0.5, 1.5, seed * 1000 + 500 + m) for m, n in enumerate(sizes)] if weighted else None
    return xs, ws


@pytest.mark.parametrize("kind,weighted", [("smu", False), ("s", True), ("spi", False), ("smu", True)])
def test_batch_matches_oracle(kind, weighted):
    import torch
    from paper_2301_12557_amd import fcfc
    L = 150.0
    xs, ws = _mocks(9, L, 3 + (kind == "s"), weighted=weighted)
    e1 = synth.linear_edges(0, 30, 10)
    e2 = synth.mu_edges(8) if kind == "smu" else (synth.linear_edges(0, 30, 6) if kind == "spi" else None)
    if kind == "spi":
        e1 = synth.linear_edges(0, 25, 5)
    plan = fcfc.Plan(kind, e1, e2, box=L, n_hint=1500)
    dx = [to_dev(x) for x in xs]
    dw = [to_dev(w) for w in ws] if weighted else [None] * len(xs)
    note(f"batch {kind} weighted={weighted} sizes={[len(x) for x in xs]}")
    b = fcfc.Batch(plan, list(zip(dx, dw)))
    nb = plan.n1 * plan.n2
    out = torch.empty(len(xs) * nb, dtype=torch.int64, device="cuda")
    wout = torch.empty(len(xs) * nb, dtype=torch.float64, device="cuda") if weighted else None
    for use_graph in (False, True, True):
        out.fill_(-1)
        b.run(out, wout, use_graph=use_graph)
        n_items, ms = b.check()
        assert n_items > 0
        got = out.cpu().numpy().reshape(len(xs), *plan.shape)
        gw = wout.cpu().numpy().reshape(len(xs), *plan.shape) if weighted else None
        for m, x in enumerate(xs):
            o, ow = oracle_count(x, kind=kind, edges1=e1, edges2=e2, box=L, w1=ws[m] if weighted else None)
            assert_same(got[m], o, gw[m] if weighted else None, ow, what=f"mock {m} graph={use_graph}")
        # eager work between replays
        torch.cuda.synchronize()
        _ = (dx[0] * 2.0).sum().item()
    b.close()


def test_batch_graph_replays_equal_individual_counts():
    """Replays of the captured graph give the same histograms as per-catalogue counts."""
    import torch
    from paper_2301_12557_amd import fcfc
    L = 300.0
    xs, _ = _mocks(16, L, 11, lo=1000, hi=6000)
    e1 = synth.linear_edges(0, 60, 12)
    e2 = synth.mu_edges(10)
    plan = fcfc.Plan("smu", e1, e2, box=L, n_hint=3000)
    dx = [to_dev(x) for x in xs]
    ref = []
    for x in dx:
        c = plan.build_cells(x)
        r, _ = plan.count(c)
        ref.append(r.clone())
        c.close()
    ref = torch.stack(ref).reshape(len(xs), -1)
    b = fcfc.Batch(plan, [(x, None) for x in dx])
    out = torch.empty_like(ref).reshape(-1)
    for r in range(4):
        out.zero_()
        b.run(out, use_graph=True)
        b.check()
        assert torch.equal(out.reshape(len(xs), -1), ref), f"replay {r}"
        torch.cuda.synchronize()
    b.close()


def test_batch_rejects_open_plan_without_bounds():
    from paper_2301_12557_amd import fcfc
    plan = fcfc.Plan("s", [0.0, 1.0, 2.0], box=0.0)
    x = to_dev(np.random.default_rng(0).random((10, 3)))
    with pytest.raises(fcfc.FcfcError) as ei:
        fcfc.Batch(plan, [(x, None)])
    assert ei.value.name == "FCFC_ESTATE"


def test_batch_learned_order_keeps_counts():
    """A batch whose plan runs the learned order (a trained model attached)
    gives the same histograms as the heuristic order, bit for bit; so does a
    model whose predictions are not finite (the heuristic key takes over), and
    retraining the model after the batch was made changes nothing."""
    import torch
    from paper_2301_12557_amd import fcfc
    L = 300.0
    xs, _ = _mocks(12, L, 21, lo=2000, hi=8000)
    e1 = synth.linear_edges(0, 60, 12)
    e2 = synth.mu_edges(10)
    dx = [to_dev(x) for x in xs]
    plan = fcfc.Plan("smu", e1, e2, box=L, n_hint=5000, record_timing=1)
    c = plan.build_cells(dx[0])
    plan.count(c)
    feat, logt = plan.timings()
    c.close()
    md = fcfc.Model(seed=4)
    md.train(feat, logt, epochs=10, batch=128, lr=2e-3, seed=1)
    nb = plan.n1 * plan.n2
    ref = torch.empty(len(xs) * nb, dtype=torch.int64, device="cuda")
    bh = fcfc.Batch(fcfc.Plan("smu", e1, e2, box=L, n_hint=5000), [(x, None) for x in dx])
    bh.run(ref, use_graph=True)
    bh.check()
    for name, model in (("trained", md), ("nan", None)):
        if model is None:
            model = fcfc.Model(seed=5)
            p, n = md.get()
            p[-1] = np.nan
            model.set(p, n)
        pl = fcfc.Plan("smu", e1, e2, box=L, n_hint=5000, order="learned")
        pl.set_model(model)
        b = fcfc.Batch(pl, [(x, None) for x in dx])
        out = torch.empty_like(ref)
        for use_graph in (False, True, True):
            out.fill_(-1)
            b.run(out, use_graph=use_graph)
            b.check()
            assert torch.equal(out, ref), f"{name} graph={use_graph}"
            if name == "trained" and use_graph:
                md.train(feat, logt, epochs=1, batch=128, lr=2e-3, seed=2)  # the batch holds its own copy
        b.close()
        pl.close()
    bh.close()
