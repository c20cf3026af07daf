"""Batches over lists of catalogue pairs (auto and cross counts of several
tracers sharing one cell build and one counting launch, the multi-tracer
configuration of App. D): every histogram must equal the oracle's count of its
pair, periodic or open, z or mid-point line of sight, weighted or not, on eager
runs and on graph replays."""
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


def _run_and_check(plan, xs, ws, pairs, kind, e1, e2, los, box, what):
    import torch
    from paper_2301_12557_amd import fcfc
    weighted = ws is not None
    dx = [to_dev(x) for x in xs]
    dw = [to_dev(w) for w in ws] if weighted else [None] * len(xs)
    note(f"{what}: sizes {[len(x) for x in xs]} pairs {pairs} weighted={weighted}")
    b = fcfc.Batch(plan, list(zip(dx, dw)), pairs=pairs)
    nb = plan.n1 * plan.n2
    out = torch.empty(len(pairs) * nb, dtype=torch.int64, device="cuda")
    wout = torch.empty(len(pairs) * nb, dtype=torch.float64, device="cuda") if weighted else None
    refs = []
    for (a, c) in pairs:
        if a == c:
            refs.append(oracle_count(xs[a], kind=kind, edges1=e1, edges2=e2, los=los, box=box,
                                     w1=ws[a] if weighted else None))
        else:
            refs.append(oracle_count(xs[a], xs[c], kind=kind, edges1=e1, edges2=e2, los=los, box=box,
                                     w1=ws[a] if weighted else None, w2=ws[c] if weighted else None))
    for use_graph in (False, True, True):
        out.fill_(-1)
        if weighted:
            wout.fill_(np.nan)
        b.run(out, wout, use_graph=use_graph)
        n_items, _ = b.check()
        got = out.cpu().numpy().reshape(len(pairs), *plan.shape)
        gw = wout.cpu().numpy().reshape(len(pairs), *plan.shape) if weighted else None
        for q, (o, ow) in enumerate(refs):
            assert_same(got[q], o, gw[q] if weighted else None, ow, what=f"{what} pair {pairs[q]} graph={use_graph}")
        # the program's own eager work between replays
        torch.cuda.synchronize()
        _ = (dx[0] * 2.0).sum().item()
    b.close()
    return got, gw


@pytest.mark.parametrize("weighted", [False, True])
def test_pairs_periodic_smu(weighted):
    """Data, randoms and a second tracer in a periodic box: every auto and cross
    pair, both orders of a cross pair, and a repeated pair."""
    from paper_2301_12557_amd import fcfc
    L = 200.0
    xs = [synth.lognormal_box(2500, L, 41, ngrid=32), synth.uniform_box(4000, L, 42),
          synth.lognormal_box(1500, L, 43, ngrid=32)]
    ws = [synth.uniform_weights(len(x), 0.5, 1.5, 50 + i) for i, x in enumerate(xs)] if weighted else None
    e1 = synth.linear_edges(0, 40, 10)
    e2 = synth.mu_edges(8)
    pairs = [(0, 0), (0, 1), (1, 1), (1, 0), (0, 2), (2, 2), (2, 1), (0, 1)]
    plan = fcfc.Plan("smu", e1, e2, box=L, n_hint=3000)
    got, gw = _run_and_check(plan, xs, ws, pairs, "smu", e1, e2, "z", L, "periodic smu")
    # cross counts are symmetric under swapping the catalogues, bit for bit
    assert np.array_equal(got[1], got[3]) and np.array_equal(got[1], got[7])
    if weighted:
        assert np.array_equal(gw[1], gw[3])
    plan.close()


@pytest.mark.parametrize("kind,los", [("spi", "mid"), ("smu", "mid"), ("s", "z"), ("spi", "z")])
def test_pairs_open_survey(kind, los):
    """A survey patch (open box): data and randoms, DD, DR and RR in one launch,
    weighted, with the plan bounds fitted over both catalogues."""
    from paper_2301_12557_amd import fcfc
    d = synth.survey_shell(2500, 61)
    r = synth.survey_shell(5000, 62)
    wd = synth.uniform_weights(len(d), 0.5, 2.0, 63)
    wr = synth.uniform_weights(len(r), 0.5, 2.0, 64)
    if kind == "spi":
        e1 = synth.linear_edges(0, 120, 6)
        e2 = synth.linear_edges(0, 120, 6)
    elif kind == "smu":
        e1 = synth.linear_edges(0, 150, 6)
        e2 = synth.mu_edges(5)
    else:
        e1 = synth.linear_edges(0, 150, 10)
        e2 = None
    plan = fcfc.Plan(kind, e1, e2, los=los, box=0.0, n_hint=5000)
    plan.fit_bounds([(to_dev(d), None), (to_dev(r), None)])
    _run_and_check(plan, [d, r], [wd, wr], [(0, 0), (0, 1), (1, 1)], kind, e1, e2, los, 0.0,
                   f"open {kind} {los}")
    plan.close()


def test_pairs_match_individual_counts_and_empty_catalogue():
    """Histograms of a pair batch equal fcfc_count_pairs on the same plan bit
    for bit (counts and exact weighted sums); an empty catalogue gives zeros."""
    import torch
    from paper_2301_12557_amd import fcfc
    L = 300.0
    xs = [synth.lognormal_box(6000, L, 71, ngrid=32), synth.uniform_box(9000, L, 72), np.zeros((0, 3))]
    ws = [synth.uniform_weights(len(x), 0.5, 1.5, 73 + i) for i, x in enumerate(xs)]
    e1 = synth.linear_edges(0, 60, 12)
    e2 = synth.linear_edges(0, 60, 6)
    plan = fcfc.Plan("spi", e1, e2, box=L, n_hint=8000)
    dx = [to_dev(x) for x in xs]
    dw = [to_dev(w) for w in ws]
    pairs = [(1, 0), (0, 0), (2, 2), (0, 2), (2, 1), (1, 1)]
    note(f"pairs vs individual counts: {pairs}")
    b = fcfc.Batch(plan, list(zip(dx, dw)), pairs=pairs)
    nb = plan.n1 * plan.n2
    out = torch.empty(len(pairs) * nb, dtype=torch.int64, device="cuda")
    wout = torch.empty(len(pairs) * nb, dtype=torch.float64, device="cuda")
    b.run(out, wout, use_graph=True)
    b.check()
    cells = [plan.build_cells(x, w) for x, w in zip(dx, dw)]
    for q, (a, c) in enumerate(pairs):
        r, rw = plan.count(cells[a], None if a == c else cells[c], weighted=True)
        assert torch.equal(out[q * nb:(q + 1) * nb], r.reshape(-1)), pairs[q]
        assert torch.equal(wout[q * nb:(q + 1) * nb], rw.reshape(-1)), pairs[q]
        if 2 in (a, c):
            assert int(out[q * nb:(q + 1) * nb].sum()) == 0
    for c in cells:
        c.close()
    b.close()
    plan.close()
