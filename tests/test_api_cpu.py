"""Host-side checks of the C ABI: the library loads, exports every declared entry
point, and rejects bad plans with the documented status codes (no GPU needed)."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_2301_12557_amd import fcfc

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    names = set()
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if fn.endswith(".h"):
            txt = open(os.path.join(ROOT, "include", fn)).read()
            names |= set(re.findall(r"\b(fcfc_[a-z0-9_]+)\s*\(", txt))
    return names


def test_library_exports_every_declared_symbol():
    lib = fcfc.load()
    names = _declared()
    assert "fcfc_count_pairs" in names and "fcfc_build_cells" in names
    missing = [n for n in sorted(names) if not hasattr(lib, n)]
    assert not missing, missing
    bound = {s[0] for s in fcfc.SIGNATURES}
    assert names <= bound, sorted(names - bound)


def test_version_and_status_strings():
    lib = fcfc.load()
    assert lib.fcfc_version() >= 1
    assert lib.fcfc_status_str(0) == b"ok"
    assert lib.fcfc_status_str(-6) == b"invalid bin edges"


def _create(kind=0, los=0, e1=(0, 1, 2), e2=None, L=10.0, tune=None):
    lib = fcfc.load()
    e1 = np.asarray(e1, dtype=np.float64)
    e2a = None if e2 is None else np.asarray(e2, dtype=np.float64)
    h = ctypes.c_void_p()
    rc = lib.fcfc_plan_create(kind, los, e1.ctypes.data_as(ctypes.c_void_p), len(e1) - 1,
                              None if e2a is None else e2a.ctypes.data_as(ctypes.c_void_p),
                              0 if e2a is None else len(e2a) - 1, float(L),
                              ctypes.byref(tune) if tune is not None else None, ctypes.byref(h))
    if rc == 0:
        lib.fcfc_plan_free(h)
    return rc


def test_plan_ok():
    assert _create() == 0
    assert _create(kind=1, e2=np.arange(11) / 10.0) == 0
    assert _create(kind=2, e1=[0, 1, 2], e2=[0, 1, 3]) == 0
    assert _create(kind=2, los=1, e1=[0, 1, 2], e2=[0, 1, 3], L=0.0) == 0


@pytest.mark.parametrize("e1", [(0, 2, 1), (1, 1, 2), (-1, 0, 1), (0, np.nan, 1), (0, np.inf)])
def test_plan_bad_edges(e1):
    assert _create(e1=e1) == -6


def test_plan_prune_radius_beyond_half_box():
    assert _create(e1=(0, 6), L=10.0) == -5
    assert _create(e1=(0, 5), L=10.0) == 0
    # (s_perp, pi) prunes on sqrt(s_perp^2 + pi^2)
    assert _create(kind=2, e1=(0, 4), e2=(0, 4), L=10.0) == -5


def test_plan_midpoint_needs_open_box():
    assert _create(kind=2, los=1, e1=(0, 1), e2=(0, 1), L=10.0) == -1


def test_plan_mu_edges_must_be_uniform():
    assert _create(kind=1, e2=[0, 0.3, 1.0]) == -6
    assert _create(kind=1, e2=[0, 0.5, 1.0]) == 0


def test_plan_bad_args():
    lib = fcfc.load()
    h = ctypes.c_void_p()
    e = np.array([0.0, 1.0])
    assert lib.fcfc_plan_create(0, 0, None, 1, None, 0, 10.0, None, ctypes.byref(h)) == -1
    assert lib.fcfc_plan_create(7, 0, e.ctypes.data_as(ctypes.c_void_p), 1, None, 0, 10.0, None,
                                ctypes.byref(h)) == -1
    assert lib.fcfc_plan_create(0, 0, e.ctypes.data_as(ctypes.c_void_p), 1, None, 0, -1.0, None,
                                ctypes.byref(h)) == -1
    assert lib.fcfc_plan_create(1, 0, e.ctypes.data_as(ctypes.c_void_p), 1, None, 0, 10.0, None,
                                ctypes.byref(h)) == -1
    assert b"edges2" in lib.fcfc_last_error()


def test_plan_too_many_bins():
    e1 = np.linspace(0, 4, 301)
    assert _create(kind=1, e1=e1, e2=np.arange(101) / 100.0) == -5


def test_open_plan_bounds_state():
    lib = fcfc.load()
    e = np.array([0.0, 1.0, 2.0])
    h = ctypes.c_void_p()
    assert lib.fcfc_plan_create(0, 0, e.ctypes.data_as(ctypes.c_void_p), 2, None, 0, 0.0, None,
                                ctypes.byref(h)) == 0
    lo = np.zeros(3)
    hi = np.array([10.0, 5.0, 1.0])
    bad = np.array([-1.0, 5.0, 1.0])
    assert lib.fcfc_plan_set_bounds(h, lo.ctypes.data_as(ctypes.c_void_p), bad.ctypes.data_as(ctypes.c_void_p)) == -1
    assert lib.fcfc_plan_set_bounds(h, lo.ctypes.data_as(ctypes.c_void_p), hi.ctypes.data_as(ctypes.c_void_p)) == 0
    assert lib.fcfc_plan_set_bounds(h, lo.ctypes.data_as(ctypes.c_void_p), hi.ctypes.data_as(ctypes.c_void_p)) == -10
    lib.fcfc_plan_free(h)


def test_midpoint_observer_inside_box_rejected():
    lib = fcfc.load()
    e = np.array([0.0, 1.0, 2.0])
    h = ctypes.c_void_p()
    assert lib.fcfc_plan_create(2, 1, e.ctypes.data_as(ctypes.c_void_p), 2, e.ctypes.data_as(ctypes.c_void_p), 2,
                                0.0, None, ctypes.byref(h)) == 0
    lo = np.array([-5.0, -5.0, -5.0])
    hi = np.array([5.0, 5.0, 5.0])
    assert lib.fcfc_plan_set_bounds(h, lo.ctypes.data_as(ctypes.c_void_p), hi.ctypes.data_as(ctypes.c_void_p)) == -5
    lib.fcfc_plan_free(h)


def test_model_file_errors(tmp_path):
    """A missing, foreign or truncated model file is FCFC_EMODEL (checked before any GPU work)."""
    lib = fcfc.load()
    assert lib.fcfc_model_nparams() == 8705
    h = ctypes.c_void_p()
    assert lib.fcfc_model_load(os.fsencode(str(tmp_path / "none.bin")), ctypes.byref(h)) == -9
    bad = tmp_path / "bad.bin"
    bad.write_bytes(b"NOTAMODEL" + bytes(100))
    assert lib.fcfc_model_load(os.fsencode(str(bad)), ctypes.byref(h)) == -9
    short = tmp_path / "short.bin"
    short.write_bytes(b"FCFCMLP1" + np.int32(8705).tobytes() + bytes(40) + bytes(400))
    assert lib.fcfc_model_load(os.fsencode(str(short)), ctypes.byref(h)) == -9
    wrong = tmp_path / "wrong.bin"
    wrong.write_bytes(b"FCFCMLP1" + np.int32(100).tobytes() + bytes(40 + 400))
    assert lib.fcfc_model_load(os.fsencode(str(wrong)), ctypes.byref(h)) == -9
    assert not h.value


def test_model_entry_points_reject_nulls():
    lib = fcfc.load()
    assert lib.fcfc_model_create(0, None) == -1
    assert lib.fcfc_plan_set_model(None, None) == -1
    assert lib.fcfc_model_predict(None, None, 0, None, None) == -1
    assert lib.fcfc_model_train(None, None, None, 0, 1, 64, ctypes.c_float(1e-3), 0, None, None) == -1
    k = ctypes.c_int32()
    assert lib.fcfc_choose_cells(None, 0, 0, None, 0, None, 0, 10.0, None, None, None, None,
                                 ctypes.byref(k), None) == -1


def test_plan_timings_before_any_count():
    lib = fcfc.load()
    e1 = np.asarray([0.0, 1.0, 2.0])
    p = ctypes.c_void_p()
    assert lib.fcfc_plan_create(0, 0, e1.ctypes.data_as(ctypes.c_void_p), 2, None, 0, 10.0, None,
                                ctypes.byref(p)) == 0
    n = ctypes.c_int64()
    assert lib.fcfc_plan_timings(p, None, None, 0, ctypes.byref(n), None) == -10
    assert lib.fcfc_plan_set_model(p, None) == 0
    lib.fcfc_plan_free(p)


def test_binding_rejects_host_tensors_and_bad_outputs():
    """The binding refuses inputs and outputs the library could not use, before any GPU work."""
    torch = pytest.importorskip("torch")
    x = torch.zeros((10, 3), dtype=torch.float64)
    with pytest.raises(ValueError):
        fcfc._catalog(x)                      # host tensor
    with pytest.raises(ValueError):
        fcfc._out_tensor(torch.zeros(5, dtype=torch.int64), 5, torch.int64, "out")   # host tensor
    with pytest.raises(ValueError):
        fcfc._out_tensor(torch.zeros(5, dtype=torch.float64), 5, torch.int64, "out")  # wrong dtype


def test_plan_rejects_bad_shard():
    t = fcfc.Tuning()
    t.shard_count = 4
    t.shard_index = 4
    assert _create(tune=t) == -1
    t.shard_index = 3
    assert _create(tune=t) == 0
    t.shard_count = -1
    t.shard_index = 0
    assert _create(tune=t) == -1


def test_build_cells_rejects_oversized_catalogue():
    """Catalogues hold at most 2^31 points (32-bit point indices in the work
    list); beyond that, or with a negative size, build_cells refuses on the host."""
    lib = fcfc.load()
    e1 = np.asarray([0.0, 1.0, 2.0])
    p = ctypes.c_void_p()
    assert lib.fcfc_plan_create(0, 0, e1.ctypes.data_as(ctypes.c_void_p), 2, None, 0, 10.0, None,
                                ctypes.byref(p)) == 0
    out = ctypes.c_void_p()
    for n in ((1 << 31) + 1, -1):
        cat = fcfc.Catalog()
        cat.xyz = ctypes.c_void_p(16)    # never dereferenced: the size check comes first
        cat.w = None
        cat.n = n
        assert lib.fcfc_build_cells(p, ctypes.byref(cat), None, ctypes.byref(out)) == -1
        assert b"2^31" in lib.fcfc_last_error()
    assert not out.value
    lib.fcfc_plan_free(p)


def test_batch_pairs_rejected_on_the_host():
    """A pair naming a catalogue outside [0, ncat), or an empty pair list, is
    FCFC_EINVAL before any GPU work."""
    lib = fcfc.load()
    e1 = np.asarray([0.0, 1.0, 2.0])
    p = ctypes.c_void_p()
    assert lib.fcfc_plan_create(0, 0, e1.ctypes.data_as(ctypes.c_void_p), 2, None, 0, 10.0, None,
                                ctypes.byref(p)) == 0
    cats = (fcfc.Catalog * 2)()
    for c in cats:
        c.xyz = ctypes.c_void_p(16)    # never dereferenced: the checks come first
        c.w = None
        c.n = 10
    out = ctypes.c_void_p()
    for pairs in ([0, 2], [-1, 0], [1, 0, 0, 5]):
        pr = np.asarray(pairs, dtype=np.int32)
        assert lib.fcfc_batch_create_pairs(p, cats, 2, pr.ctypes.data_as(ctypes.c_void_p), len(pr) // 2, None,
                                           ctypes.byref(out)) == -1, pairs
        assert b"pair" in lib.fcfc_last_error()
    pr = np.asarray([0, 0], dtype=np.int32)
    assert lib.fcfc_batch_create_pairs(p, cats, 2, pr.ctypes.data_as(ctypes.c_void_p), 0, None,
                                       ctypes.byref(out)) == -1
    assert lib.fcfc_batch_create_pairs(p, cats, 2, None, 1, None, ctypes.byref(out)) == -1
    assert not out.value
    lib.fcfc_plan_free(p)


def test_angular_plan_on_the_host():
    """fcfc_angular_plan returns the FP64 chord edges 2 sin(theta/2) it counts with
    (within an ulp of the oracle's), and refuses edges outside [0, 180] degrees."""
    from oracle import angular as A
    lib = fcfc.load()
    th = np.array([0.0, 0.5, 1.0, 10.0, 60.0, 179.0])
    chord = np.empty(len(th))
    h = ctypes.c_void_p()
    assert lib.fcfc_angular_plan(th.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), len(th) - 1, None,
                                 chord.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), ctypes.byref(h)) == 0
    assert np.allclose(chord, A.chord_edges(th), rtol=2.3e-16, atol=0)
    lib.fcfc_plan_free(h)
    for bad in ([0.0, 10.0, 190.0], [0.0, -1.0, 5.0], [0.0, 5.0, 5.0]):
        b = np.asarray(bad)
        assert lib.fcfc_angular_plan(b.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), 2, None, None,
                                     ctypes.byref(h)) == -6, bad


def test_bin_and_triplet_arguments_rejected_on_the_host():
    """fcfc_bin_squared and fcfc_count_triplets refuse bad arguments before any
    GPU work: null pointers, negative or oversized counts, unaligned values,
    plans that are not s plans, and more than 32 triangle bins."""
    lib = fcfc.load()
    e = np.asarray([0.0, 1.0, 2.0, 3.0])
    p = ctypes.c_void_p()
    assert lib.fcfc_plan_create(0, 0, e.ctypes.data_as(ctypes.c_void_p), 3, None, 0, 10.0, None,
                                ctypes.byref(p)) == 0
    fake = ctypes.c_void_p(1 << 20)  # never dereferenced: the checks come first
    assert lib.fcfc_bin_squared(None, fake, 10, fake, None) == -1
    assert lib.fcfc_bin_squared(p, fake, -1, fake, None) == -1
    assert lib.fcfc_bin_squared(p, fake, 10, None, None) == -1
    assert lib.fcfc_bin_squared(p, None, 10, fake, None) == -1
    assert lib.fcfc_bin_squared(p, fake, (1 << 61) + 1, fake, None) == -1
    assert lib.fcfc_bin_squared(p, ctypes.c_void_p((1 << 20) + 4), 10, fake, None) == -1
    assert b"aligned" in lib.fcfc_last_error()
    assert lib.fcfc_count_triplets(None, None, fake, None, None) == -1
    assert lib.fcfc_count_triplets(p, None, fake, None, None) == -1
    assert lib.fcfc_count_triplets(p, fake, None, None, None) == -1
    lib.fcfc_plan_free(p)
    m = np.linspace(0.0, 1.0, 5)
    assert lib.fcfc_plan_create(1, 0, e.ctypes.data_as(ctypes.c_void_p), 3, m.ctypes.data_as(ctypes.c_void_p), 4,
                                10.0, None, ctypes.byref(p)) == 0
    assert lib.fcfc_count_triplets(p, fake, fake, None, None) == -1
    assert b"s plan" in lib.fcfc_last_error()
    lib.fcfc_plan_free(p)
    e40 = np.linspace(0.0, 2.0, 41)
    assert lib.fcfc_plan_create(0, 0, e40.ctypes.data_as(ctypes.c_void_p), 40, None, 0, 10.0, None,
                                ctypes.byref(p)) == 0
    assert lib.fcfc_count_triplets(p, fake, fake, None, None) == -5
    assert b"32" in lib.fcfc_last_error()
    lib.fcfc_plan_free(p)


def test_plan_rejects_bad_chunk_and_flush():
    """b_chunk bounds the pairs of one work item and flush_log2 the pairs a
    wavefront claims between two merges of the 32-bit LDS counters; values that
    could overflow them are refused."""
    for chunk, rc in ((0, 0), (256, 0), (1 << 19, 0), (255, -1), ((1 << 19) + 1, -1), (-5, -1)):
        t = fcfc.Tuning()
        t.b_chunk = chunk
        assert _create(tune=t) == rc, chunk
    for fl, rc in ((0, 0), (1, 0), (26, 0), (27, -1), (-1, -1)):
        t = fcfc.Tuning()
        t.flush_log2 = fl
        assert _create(tune=t) == rc, fl


def _oracle_refuses(w1, w2):
    """The oracle's answer for a weighted cross count of two points with these weights."""
    import oracle
    x = np.array([[1.0, 1.0, 1.0]])
    y = np.array([[1.5, 1.0, 1.0]])
    try:
        oracle.count(x, y, kind="s", edges1=[0.0, 1.0], w1=np.array([w1]), w2=np.array([w2]))
    except oracle.OracleError:
        return True
    return False


@pytest.mark.parametrize("wmin,wmax,ok", [
    (1e-200, 1.0, False),      # the smallest product 1e-400 underflows to zero
    (1e-160, 1e-160, False),   # the smallest product 1e-320 is subnormal
    (1e-150, 1e-150, False),   # 1e-300 is normal but needs a scale 2^1049 beyond FP64
    (0.5, 2.0, True),
    (0.5, 1.5, True),
    (1e-100, 1e-100, True),
    (1.0, 1e3, False),         # max/min product 1e6: beyond 2^62 / 2^53
])
def test_weight_scale_refuses_underflowing_products(wmin, wmax, ok):
    """The exact weighted sums need every pair product w_i*w_j to be an FP64
    multiple of one power of two that fits: products that underflow (zero or
    subnormal), a scale 2^S beyond FP64, or a range too wide are FCFC_ERANGE,
    and the oracle refuses the same weights."""
    if ok:
        S = fcfc.weight_scale(wmin, wmax)
        p = wmin * wmin
        assert 2.0 ** 52 <= p * 2.0 ** S < 2.0 ** 53
        assert wmax * wmax * 2.0 ** S < 2.0 ** 62
    else:
        with pytest.raises(fcfc.FcfcError) as ei:
            fcfc.weight_scale(wmin, wmax)
        assert ei.value.name == "FCFC_ERANGE"
    if wmax / wmin < 100:
        assert _oracle_refuses(wmin, wmin) == (not ok)


def test_weight_scale_cross_and_triangles():
    """Cross counts combine the ranges of both catalogues; triangles take the
    cube of one catalogue's range (fl(fl(a b) c))."""
    assert fcfc.weight_scale(1e300, 2e300, 1e-300, 2e-300) >= 0
    with pytest.raises(fcfc.FcfcError):
        fcfc.weight_scale(1e-200, 1.0, 1e-200, 1.0)
    assert _oracle_refuses(1e-200, 1e-200)
    S = fcfc.weight_scale(0.5, 2.0, nfactors=3)
    assert 2.0 ** 52 <= 0.125 * 2.0 ** S < 2.0 ** 53
    with pytest.raises(fcfc.FcfcError) as ei:
        fcfc.weight_scale(1e-110, 1e-110, nfactors=3)  # 1e-330: subnormal
    assert ei.value.name == "FCFC_ERANGE"
    with pytest.raises(fcfc.FcfcError) as ei:
        fcfc.weight_scale(1e200, 1e200)  # the largest product overflows
    assert ei.value.name == "FCFC_ERANGE"
    # all-zero weights: every product is zero, nothing to scale
    assert fcfc.weight_scale(0.0, 0.0, 0.5, 1.0) == 0
    lib = fcfc.load()
    S = ctypes.c_int32()
    assert lib.fcfc_weight_scale(1.0, 1.0, 1.0, 1.0, 4, ctypes.byref(S)) == -1
    assert lib.fcfc_weight_scale(-1.0, 1.0, 1.0, 1.0, 2, ctypes.byref(S)) == -1
    assert lib.fcfc_weight_scale(float("nan"), 1.0, 1.0, 1.0, 2, ctypes.byref(S)) == -1
    assert lib.fcfc_weight_scale(1.0, 1.0, 1.0, 1.0, 2, None) == -1


def test_pair_norm_exact():
    """Pairs behind a count, formed exactly and rounded once (host only)."""
    assert fcfc.pair_norm(4) == 6.0 and fcfc.pair_norm(3, 5) == 15.0 and fcfc.pair_norm(1) == 0.0
    for n in (2_000_000, 40_000_000, 3_000_000_007, 2 ** 31 + 11):
        assert fcfc.pair_norm(n) == float(n * (n - 1) // 2)
        assert fcfc.pair_norm(n, n + 3) == float(n * (n + 3))
    lib = fcfc.load()
    out = ctypes.c_double()
    assert lib.fcfc_pair_norm(-1, -1, ctypes.byref(out)) == -1
    assert lib.fcfc_pair_norm(5, -1, None) == -1
    # too few points: refused before anything touches a device
    assert lib.fcfc_landy_szalay(None, None, None, 10, 10, 4, None, None) == -1


def test_tree_plan_validation():
    """Tree plans: leaves of 32..128 points, open boxes only (host checks)."""
    t = fcfc.Tuning()
    for leaf, box, rc in ((128, 0.0, 0), (32, 0.0, 0), (31, 0.0, -1), (129, 0.0, -1), (64, 1000.0, -1)):
        t.tree_leaf = leaf
        assert _create(kind=2, los=1, e1=[0, 1, 2], e2=[0, 1, 3], L=box, tune=t) == rc, (leaf, box)
    p = fcfc.Plan("spi", [0.0, 10.0, 20.0], [0.0, 10.0, 20.0], los="mid", box=0.0, tree_leaf=64)
    p.set_bounds([500.0, 0.0, -100.0], [900.0, 400.0, 100.0])
    assert p.numerics()["nx"] > 0
    p.close()
