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
    return synth.blobs_box(n, L, nblob, rad, frac, seed)


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


def _train_model(fcfc, torch):
    """Cost model trained on per-item timings of two lognormal boxes at k = 1..4."""
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
    return md, loss


@pytest.mark.parametrize("blobs", [(30, 15.0, 0.8, 8), (10, 5.0, 0.9, 9)], ids=["blobs30", "blobs10"])
def test_tuning_gain_on_clustered_catalogue(blobs):
    """Held-out catalogues far more clustered than the analytic cell-size rule
    assumes (80-90 % of 300,000 points in a few Gaussian blobs): the tuning
    found with the learned model proposing cell sizes, measured again afresh,
    must beat the analytic tuning by at least 1.25x (on MI355X: 2.1x and
    1.8x).  The model only adds cell sizes to the model-free search, so its
    result must not be slower than that search's by more than timing noise
    and the other knobs' descent from another start (10 %); the gain the
    model adds on its own is printed."""
    import torch
    from paper_2301_12557_amd import fcfc
    md, loss = _train_model(fcfc, torch)
    nblob, rad, frac, seed = blobs
    dx = to_dev(_blobs(300000, nblob, rad, frac, seed))
    t0, _, _, n0 = fcfc.autotune(dx, kind="smu", edges1=E1, edges2=E2, box=L)
    t1, _, _, n1 = fcfc.autotune(dx, model=md, kind="smu", edges1=E1, edges2=E2, box=L)
    analytic = min(_time_count(fcfc, dx) for _ in range(2))
    free = min(_time_count(fcfc, dx, **_plan_kw(t0)) for _ in range(2))
    tuned = min(_time_count(fcfc, dx, model=md, **_plan_kw(t1)) for _ in range(2))
    note(f"model loss {loss:.3f}; analytic {analytic:.2f} ms; model-free search ({n0} trials, "
         f"k={t0['cells_per_rmax']}) {free:.2f} ms; with the model ({n1} trials, k={t1['cells_per_rmax']}) "
         f"{tuned:.2f} ms: gain x{analytic / tuned:.2f} over analytic, x{free / tuned:.2f} from the model")
    assert n1 >= n0
    assert analytic >= 1.25 * tuned
    assert tuned <= 1.10 * free
