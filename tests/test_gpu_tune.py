"""The autotuner: measured tuning choices (with and without the learned cost
model proposing cell sizes), its cache, and counts that stay exact under every
tuning it returns."""
import time

import numpy as np
import pytest

from paper_2301_12557_amd import synth
from helpers import note, to_dev, oracle_count, assert_same

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


L = 500.0
E1 = synth.linear_edges(0, 40, 20)
E2 = synth.mu_edges(10)


def _plan_kw(t):
    return {k: v for k, v in t.items() if k != "record_timing"}


def test_autotune_exact_counts_and_cache(tmp_path):
    from paper_2301_12557_amd import fcfc
    x = synth.lognormal_box(30000, L, 21, ngrid=64)
    dx = to_dev(x)
    cache = str(tmp_path / "tune.txt")
    t, best, heur, n = fcfc.autotune(dx, kind="smu", edges1=E1, edges2=E2, box=L, cache=cache)
    note(f"tuned {t} best {best:.3f} ms analytic {heur:.3f} ms trials {n}")
    assert n >= 3 and np.isfinite(best) and best <= heur
    assert 1 <= t["cells_per_rmax"] <= 6 and t["tile_points"] in (64, 128) and t["hist_copies"] in (1, 2, 4)
    ref, _ = oracle_count(x, kind="smu", edges1=E1, edges2=E2, box=L)
    got, _ = fcfc.count_pairs(dx, kind="smu", edges1=E1, edges2=E2, box=L, **_plan_kw(t))
    assert_same(got.cpu().numpy(), ref, what=f"tuned {t}")
    # a cache hit returns the stored tuning without timing anything
    t2, best2, heur2, n2 = fcfc.autotune(dx, kind="smu", edges1=E1, edges2=E2, box=L, cache=cache)
    assert n2 == 0 and t2 == t and best2 == pytest.approx(best, rel=1e-5) and np.isnan(heur2)
    # other bins: another signature, tuned again
    e1b = synth.linear_edges(0, 30, 15)
    _, _, _, n3 = fcfc.autotune(dx, kind="smu", edges1=e1b, edges2=E2, box=L, cache=cache)
    assert n3 >= 3
    assert len(open(cache).read().splitlines()) == 2


def test_autotune_weighted_and_open_box():
    from paper_2301_12557_amd import fcfc
    rng = np.random.default_rng(3)
    d = synth.survey_shell(4000, 5)
    r = synth.survey_shell(8000, 6)
    wd = rng.uniform(0.5, 2.0, len(d))
    wr = rng.uniform(0.5, 2.0, len(r))
    e1 = synth.linear_edges(0, 40, 8)
    e2 = synth.linear_edges(0, 40, 8)
    dd, dr, wdd, wdr = to_dev(d), to_dev(r), to_dev(wd), to_dev(wr)
    t, best, heur, n = fcfc.autotune(dd, dr, kind="spi", edges1=e1, edges2=e2, los="mid", box=0.0, w1=wdd, w2=wdr)
    note(f"tuned DR {t} {best:.3f} ms (analytic {heur:.3f}) trials {n}")
    assert n >= 3 and best <= heur
    ref, wref = oracle_count(d, r, kind="spi", edges1=e1, edges2=e2, los="mid", box=0.0, w1=wd, w2=wr)
    got, wgot = fcfc.count_pairs(dd, dr, kind="spi", edges1=e1, edges2=e2, los="mid", box=0.0, w1=wdd, w2=wdr,
                                 **_plan_kw(t))
    assert_same(got.cpu().numpy(), ref, wgot.cpu().numpy(), wref, what=f"tuned {t}")


def _blobs(n, nblob, rad, frac, seed):
    """Clustered catalogue: a fraction of the points in Gaussian blobs, the rest uniform."""
    rng = np.random.default_rng(seed)
    nb = int(n * frac)
    cen = rng.uniform(rad * 3, L - rad * 3, (nblob, 3))
    x = cen[rng.integers(0, nblob, nb)] + rng.normal(0, rad, (nb, 3))
    x = np.concatenate([x, rng.uniform(0, L, (n - nb, 3))])
    return np.clip(x, 0, np.nextafter(L, 0))


def _time_count(fcfc, dx, reps=3, model=None, **tune):
    import torch
    tune.setdefault("n_hint", len(dx))
    plan = fcfc.Plan("smu", E1, E2, box=L, **tune)
    if model is not None:
        plan.set_model(model)
    best = np.inf
    for _ in range(reps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        c = plan.build_cells(dx)
        plan.count(c)
        torch.cuda.synchronize()
        best = min(best, time.perf_counter() - t0)
        c.close()
    plan.close()
    return best * 1e3


def test_learned_tuning_gain_over_analytic():
    """Train the cost model on timings of lognormal boxes, then tune a held-out
    clustered catalogue with it: the tuned count is measured again, afresh,
    against the analytic tuning, and must not be slower (5 % timing noise)."""
    import torch
    from paper_2301_12557_amd import fcfc
    feats, ts = [], []
    for i, n in enumerate((50000, 200000)):
        x = synth.lognormal_box_torch(n, L, 100 + i, device="cuda", ngrid=128)
        for k in (1, 2, 3, 4):
            plan = fcfc.Plan("smu", E1, E2, box=L, n_hint=n, cells_per_rmax=k, record_timing=1)
            c = plan.build_cells(x)
            plan.count(c)
            f, t = plan.timings()
            feats.append(f)
            ts.append(t)
            c.close()
            plan.close()
    md = fcfc.Model(seed=1)
    loss = md.train(torch.cat(feats), torch.cat(ts), epochs=10, batch=512, lr=2e-3, seed=1)
    dx = to_dev(_blobs(300000, 30, 15.0, 0.8, 8))
    t, best, heur, n = fcfc.autotune(dx, model=md, kind="smu", edges1=E1, edges2=E2, box=L)
    tuned = _time_count(fcfc, dx, model=md, **_plan_kw(t))
    analytic = _time_count(fcfc, dx)
    note(f"model loss {loss:.3f}; tuned {t}: {tuned:.2f} ms, analytic {analytic:.2f} ms, "
         f"gain x{analytic / tuned:.2f} ({n} trials)")
    assert tuned <= 1.05 * analytic
