"""fcfc_count_pairs_noalloc, the pair count for callers that cannot allocate
device memory: through the C ABI, its histograms equal fcfc_count_pairs's bit
for bit (counts and exact weighted sums) on two calls in a row, the second
with a smaller input, and a count whose scratch does not fit the library's
fixed array is refused with the outputs untouched."""
import ctypes

import numpy as np
import pytest

from paper_2301_12557_amd import synth
from helpers import note, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _counts(lib, fn, plan, c1, c2, nb, weighted):
    import torch
    from paper_2301_12557_amd import fcfc
    out = torch.full((nb,), -3, dtype=torch.int64, device="cuda")
    wout = torch.full((nb,), -3.0, dtype=torch.float64, device="cuda") if weighted else None
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    rc = getattr(lib, fn)(plan.h, c1.h, c2.h if c2 is not None else None, ctypes.c_void_p(out.data_ptr()),
                          ctypes.c_void_p(wout.data_ptr()) if weighted else None, stream)
    if rc != 0:
        raise fcfc.FcfcError(rc, lib.fcfc_last_error().decode())
    torch.cuda.synchronize()
    return out.cpu().numpy(), (wout.cpu().numpy() if weighted else None)


@pytest.mark.parametrize("kind,weighted,cross", [("smu", True, False), ("s", False, False),
                                                 ("spi", True, True)])
def test_noalloc_matches_allocating_count_twice(kind, weighted, cross):
    from paper_2301_12557_amd import fcfc
    lib = fcfc.load()
    assert lib.fcfc_noalloc_scratch_bytes() == 64 << 20
    L = 1000.0
    e1 = synth.linear_edges(0, 200, 40)
    e2 = {"smu": synth.mu_edges(100), "spi": synth.linear_edges(0, 120, 24), "s": None}[kind]
    if kind == "spi":
        e1 = synth.linear_edges(0, 120, 24)
    plan = fcfc.Plan(kind, e1, e2, box=L, n_hint=20000)
    nb = plan.n1 * plan.n2
    # the second call has a smaller input: the array keeps the first call's
    # contents, and whatever must start at zero is cleared again
    for n in (20000, 6000):
        x = synth.uniform_box(n, L, 100 + n)
        w = synth.uniform_weights(n, 0.5, 1.5, 200 + n) if weighted else None
        y = synth.lognormal_box(n // 2, L, 300 + n, ngrid=32) if cross else None
        wy = synth.uniform_weights(n // 2, 0.5, 1.5, 400 + n) if (cross and weighted) else None
        note(f"noalloc {kind} weighted={weighted} cross={cross} n={n}")
        c1 = plan.build_cells(to_dev(x), to_dev(w))
        c2 = plan.build_cells(to_dev(y), to_dev(wy)) if cross else None
        got, gw = _counts(lib, "fcfc_count_pairs_noalloc", plan, c1, c2, nb, weighted)
        ref, rw = _counts(lib, "fcfc_count_pairs", plan, c1, c2, nb, weighted)
        assert got.sum() > 0
        assert np.array_equal(got, ref)
        if weighted:
            assert np.array_equal(gw, rw)
        c1.close()
        if c2 is not None:
            c2.close()
    plan.close()


def test_noalloc_stats_and_oversized_refusal():
    """Without an earlier allocating count the plan keeps no statistics
    (FCFC_ESTATE); after one it does.  A count needing more scratch than the
    array holds is FCFC_ERANGE and leaves the outputs untouched."""
    import torch
    from paper_2301_12557_amd import fcfc
    lib = fcfc.load()
    L = 1000.0
    e1 = synth.linear_edges(0, 100, 20)
    plan = fcfc.Plan("s", e1, box=L, n_hint=5000)
    x = to_dev(synth.uniform_box(5000, L, 7))
    c = plan.build_cells(x)
    got, _ = _counts(lib, "fcfc_count_pairs_noalloc", plan, c, None, 20, False)
    st = fcfc.Stats()
    assert lib.fcfc_plan_stats(plan.h, ctypes.byref(st)) == -10
    ref, _ = _counts(lib, "fcfc_count_pairs", plan, c, None, 20, False)
    assert np.array_equal(got, ref)
    got2, _ = _counts(lib, "fcfc_count_pairs_noalloc", plan, c, None, 20, False)
    assert np.array_equal(got2, ref)
    assert lib.fcfc_plan_stats(plan.h, ctypes.byref(st)) == 0
    assert st.in_range == int(ref.sum()) and st.candidates >= st.in_range
    c.close()
    plan.close()
    # 1,000,000 points on a grid of 10^6 cells (s_max = 10, one cell per
    # radius), one tile per cell: about 5 million work items (some 400 MB of
    # scratch), far beyond the 64 MiB array
    big = fcfc.Plan("s", synth.linear_edges(0, 10, 4), box=L, cells_per_rmax=1, tile_points=64, seg_cells=1,
                    b_chunk=256)
    xb = to_dev(synth.uniform_box(1000000, L, 8))
    cb = big.build_cells(xb)
    out = torch.full((4,), -3, dtype=torch.int64, device="cuda")
    rc = lib.fcfc_count_pairs_noalloc(big.h, cb.h, None, ctypes.c_void_p(out.data_ptr()), None,
                                      ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    note(f"oversized: rc {rc}: {lib.fcfc_last_error().decode()}")
    assert rc == -5
    torch.cuda.synchronize()
    assert out.cpu().tolist() == [-3] * 4
    cb.close()
    big.close()
