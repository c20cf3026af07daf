"""The histogram update routine on its own (fcfc_bin_squared): counts of given
squared separations equal the oracle's bit for bit, for the benchmark's four
bin layouts (20 and 200 bins, linear on [0, 200) and logarithmic on
[0.1, 200)), every look-up table size, values planted on and next to every
edge, special values, unaligned and tiny inputs; and at the benchmark's full
size of 6.4e9 values, in the launch the benchmark times, by properties that
hold at any size."""
import numpy as np
import pytest

from oracle import histogram as H
from paper_2301_12557_amd import synth
from helpers import note, to_dev, assert_same

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


R = 200.0
LAYOUTS = {
    "lin20": synth.linear_edges(0, R, 20),
    "lin200": synth.linear_edges(0, R, 200),
    "log20": synth.log_edges(0.1, R, 20),
    "log200": synth.log_edges(0.1, R, 200),
}


def _values(n, edges, seed):
    """The App. C input with planted values: every squared edge, one ulp either
    side of it, points a few 1e-8 away (inside the FP32 bands), and special values."""
    rng = np.random.default_rng(seed)
    v = synth.s2_samples(n, R, seed)
    E = np.asarray(edges, dtype=np.float64) ** 2
    plant = np.concatenate([E, np.nextafter(E, -np.inf), np.nextafter(E, np.inf), E * (1 + 3e-8), E * (1 - 3e-8),
                            [np.nan, -1.0, -1e-300, np.inf, -np.inf, -0.0, 0.0, 1e300, 5e-324]])
    pos = rng.choice(n, size=len(plant), replace=False)
    v[pos] = plant
    return v


def _gpu_bins(fcfc, plan, v):
    import torch
    out = plan.bin_squared(v)
    torch.cuda.synchronize()
    return out.cpu().numpy()


@pytest.mark.parametrize("name", list(LAYOUTS))
def test_layouts_match_oracle(name):
    from paper_2301_12557_amd import fcfc
    edges = LAYOUTS[name]
    n = 3_000_001  # odd: a tail value after the 16-byte pairs
    v = _values(n, edges, 31)
    note(f"bin_squared {name}: n={n}")
    ref = H.bin_squared(v, edges)
    plan = fcfc.Plan("s", edges, box=4 * R)
    dv = to_dev(v)
    got = _gpu_bins(fcfc, plan, dv)
    assert_same(got, ref, what=name)
    st = plan.stats()
    assert st["candidates"] == n and st["in_range"] == ref.sum()
    assert st["rechecks"] > 0  # the planted values inside the bands took the FP64 path
    # an 8-byte (not 16-byte) aligned start: one head value before the pairs
    got1 = plan.bin_squared(dv[1:]).cpu().numpy()
    assert_same(got1, H.bin_squared(v[1:], edges), what=name + " unaligned")
    plan.close()


@pytest.mark.parametrize("lut_log2", [8, 10, 12, 14])
def test_table_sizes_agree(lut_log2):
    """Fewer table entries mean more entries that meet a band: the bands and
    the FP64 path keep the counts exact at every size."""
    from paper_2301_12557_amd import fcfc
    for name in ("lin200", "log200"):
        edges = LAYOUTS[name]
        v = _values(1_000_000, edges, 40 + lut_log2)
        plan = fcfc.Plan("s", edges, box=4 * R, lut_log2=lut_log2)
        note(f"bin_squared {name} lut_log2={lut_log2}")
        assert_same(_gpu_bins(fcfc, plan, to_dev(v)), H.bin_squared(v, edges), what=f"{name} 2^{lut_log2}")
        plan.close()


def test_tiny_and_empty_inputs():
    import torch
    from paper_2301_12557_amd import fcfc
    edges = LAYOUTS["lin20"]
    plan = fcfc.Plan("s", edges, box=4 * R)
    base = to_dev(_values(512, edges, 3))
    for start in (0, 1):
        for n in (0, 1, 2, 3, 5, 17):
            v = base[start:start + n]
            got = plan.bin_squared(v).cpu().numpy()
            assert_same(got, H.bin_squared(v.cpu().numpy(), edges), what=f"start {start} n {n}")
    empty = torch.empty(0, dtype=torch.float64, device="cuda")
    assert plan.bin_squared(empty).cpu().numpy().sum() == 0
    plan.close()


def test_periodic_and_open_plans_give_the_same_bins():
    """The bins are those of the plan's edges whatever its box: an open-box
    plan, before and after its bounds are set, counts the same values
    identically."""
    import torch
    from paper_2301_12557_amd import fcfc
    edges = LAYOUTS["log20"]
    v = _values(500_000, edges, 9)
    dv = to_dev(v)
    p1 = fcfc.Plan("s", edges, box=4 * R)
    p2 = fcfc.Plan("s", edges, box=0.0)
    b0 = p2.bin_squared(dv).cpu().numpy()  # the table depends on the edges alone
    p2.set_bounds([0, 0, 0], [3000, 2000, 1000])
    a = p1.bin_squared(dv).cpu().numpy()
    b = p2.bin_squared(dv).cpu().numpy()
    torch.cuda.synchronize()
    assert_same(a, H.bin_squared(v, edges), what="periodic")
    assert_same(b0, a, what="open, no bounds")
    assert_same(b, a, what="open")
    p1.close()
    p2.close()


N_FULL = 6_400_000_000


@pytest.mark.parametrize("name", ["lin20", "log200"])
def test_full_size_properties(name):
    """6.4e9 values of the App. C law in one call (the launch the benchmark
    times): the counts equal, bin by bin, those of torch.bucketize on the same
    squared edges (an independent definition of the half-open bins), and equal
    the sum of three separate calls over a partition; one part of 8e6 values is
    checked against the oracle."""
    import torch
    from paper_2301_12557_amd import fcfc
    edges = LAYOUTS[name]
    note(f"bin_squared full size {name}: generating {N_FULL} values")
    v = synth.s2_samples_torch(N_FULL, R, 2301125579)
    plan = fcfc.Plan("s", edges, box=4 * R)
    whole = plan.bin_squared(v)
    torch.cuda.synchronize()
    note(f"bin_squared full size {name}: kernel {plan.stats()['kernel_ms']:.3f} ms")
    E = torch.tensor(np.asarray(edges) ** 2, dtype=torch.float64, device="cuda")
    ref = torch.zeros(len(edges) + 1, dtype=torch.int64, device="cuda")
    step = 1 << 28
    for lo in range(0, N_FULL, step):
        idx = torch.bucketize(v[lo:lo + step], E, right=True)  # number of edges <= v
        ref += torch.bincount(idx, minlength=len(edges) + 1)
        del idx
    ref = ref[1:len(edges)].cpu().numpy()
    assert_same(whole.cpu().numpy(), ref, what=f"{name} full size vs bucketize")
    a, b = 1_000_000_007, 4_000_000_001
    parts = [plan.bin_squared(v[s:e]).cpu().numpy() for s, e in ((0, a), (a, b), (b, N_FULL))]
    assert_same(whole.cpu().numpy(), parts[0] + parts[1] + parts[2], what=f"{name} partition")
    m = 3_123_456_789
    sample = v[m:m + 8_000_000]
    assert_same(plan.bin_squared(sample).cpu().numpy(), H.bin_squared(sample.cpu().numpy(), edges),
                what=f"{name} sampled part vs oracle")
    plan.close()
    del v
    torch.cuda.empty_cache()


def test_any_plan_bins_its_first_axis():
    """An (s, mu) or (s_perp, pi) plan bins given values by its first-axis edges,
    exactly as the s plan of the same edges and the oracle do."""
    from paper_2301_12557_amd import fcfc
    edges = LAYOUTS["lin20"]
    v = _values(400_000, edges, 17)
    dv = to_dev(v)
    ref = H.bin_squared(v, edges)
    for kind, e2, box in (("s", None, 4 * R), ("smu", synth.mu_edges(10), 4 * R), ("spi", synth.linear_edges(0, 50, 5), 0.0)):
        plan = fcfc.Plan(kind, edges, e2, box=box)
        note(f"bin_squared with a {kind} plan")
        assert_same(_gpu_bins(fcfc, plan, dv), ref, what=f"{kind} plan")
        plan.close()


@pytest.mark.parametrize("layout,nb", [("log", 1000), ("linear", 2000)])
def test_many_bins_few_copies(layout, nb):
    """1000 or 2000 bins leave room for only 16 or 8 LDS histogram copies per
    workgroup (lanes share copies, and each bin's copies are summed by one
    thread): still exact.  Far more bins than the LDS holds are refused."""
    from paper_2301_12557_amd import fcfc
    edges = synth.log_edges(0.1, R, nb) if layout == "log" else synth.linear_edges(0, R, nb)
    v = _values(2_000_001, edges, 50 + nb)
    plan = fcfc.Plan("s", edges, box=4 * R)
    note(f"bin_squared {layout}{nb}")
    assert_same(_gpu_bins(fcfc, plan, to_dev(v)), H.bin_squared(v, edges), what=f"{layout}{nb}")
    plan.close()


def test_too_many_bins_refused():
    from paper_2301_12557_amd import fcfc
    edges = synth.linear_edges(0, R, 12000)
    plan = fcfc.Plan("s", edges, box=4 * R)
    with pytest.raises(fcfc.FcfcError):
        plan.bin_squared(to_dev(np.ones(16)))
    plan.close()


@pytest.mark.parametrize("box", [500.0, 0.0])
def test_binning_all_pair_separations_equals_pair_counts(box):
    """The two exact routines agree: every pair's squared separation, formed in
    FP64 by numpy with the pair definition (minimum image, (dx^2 + dy^2) + dz^2),
    binned by fcfc_bin_squared, gives the s counts of fcfc_count_pairs."""
    from paper_2301_12557_amd import fcfc
    x = synth.lognormal_box(3000, 500.0, 61, ngrid=32)
    edges = synth.log_edges(0.5, 60.0, 25)
    i, j = np.triu_indices(len(x), 1)
    d = x[j] - x[i]
    if box > 0:
        h = box * 0.5
        d = np.where(d > h, d - box, np.where(d < -h, d + box, d))
    s2 = (d[:, 0] * d[:, 0] + d[:, 1] * d[:, 1]) + d[:, 2] * d[:, 2]
    plan = fcfc.Plan("s", edges, box=box)
    binned = _gpu_bins(fcfc, plan, to_dev(s2))
    plan.close()
    counts, _ = fcfc.count_pairs(to_dev(x), kind="s", edges1=edges, box=box)
    assert_same(binned, counts.cpu().numpy(), what=f"box {box}")
    assert_same(binned, H.bin_squared(s2, edges), what=f"box {box} oracle")
