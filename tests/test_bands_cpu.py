"""The counting kernel's FP32 decisions, replayed on the CPU.

The kernel forms separations in FP32 and bins a pair there only when its
value lies outside every band around a bin edge; inside a band the pair is
binned again in FP64 (the single-precision evaluation of Sect. 2.5 made exact
for the squared-edge bins of Sect. 3.2.1, through the look-up tables of
Sect. 3.2.3).  Two checks, neither needing a GPU:

* every entry of every look-up table against the plan's FP64 squared edges
  and FP32 bands (a clean entry's whole value range lies between the bands of
  its bin's edges, a hot entry names the first band it meets, and so on);
* the kernel's FP32 arithmetic emulated operation by operation in numpy
  (cell-local coordinates, the explicit fma chains rounded once, the table
  look-up, the mu and mid-point line-of-sight steps with the hardware
  reciprocal square root and reciprocal at both ends of their error bound),
  over more than 10^7 pairs per workload geometry, many of them within a few
  FP32 ulps of an edge and some exactly on one: every pair the emulation bins
  without the FP64 recheck must land in the oracle's bin, and every pair it
  drops must be out of range for the oracle too.
"""
from fractions import Fraction

import numpy as np
import pytest

import oracle
from paper_2301_12557_amd import fcfc, synth

F32 = np.float32
F64 = np.float64
N_FULL = 10_200_000   # pairs for the C2, C3 mid-point and C5 geometries
N_SHORT = 2_000_000   # for the other shapes
CHUNK = 1_700_000


# ---------------------------------------------------------------------------
# exact FP32 arithmetic
# ---------------------------------------------------------------------------

def fma32(a, b, c):
    """Single-rounded FP32 a*b + c of FP32 arrays.  a*b is exact in FP64 and
    TwoSum gives the exact p + c as s + err; s rounds to FP32 as p + c does
    unless s is a midpoint between two FP32 numbers (a midpoint is an FP64
    number, so the nearest FP64 value of anything closer to it is the
    midpoint itself), and there the sign of err decides."""
    p = a.astype(F64) * b.astype(F64)
    c64 = c.astype(F64)
    s = p + c64
    bb = s - p
    err = (p - (s - bb)) + (c64 - bb)
    r = s.astype(F32)
    r64 = r.astype(F64)
    toward = np.where(s > r64, F32(np.inf), F32(-np.inf)).astype(F32)
    other = np.nextafter(r, toward)
    mid = (r64 + other.astype(F64)) * 0.5
    tie = (s == mid) & (s != r64) & (err != 0)
    hi = np.maximum(r, other)
    lo = np.minimum(r, other)
    return np.where(tie & (err > 0), hi, np.where(tie & (err < 0), lo, r))


def _round32_exact(q):
    """Fraction -> nearest FP32 (ties to even), for the fma32 pin."""
    f = F32(float(q))  # within one FP32 ulp of q (float(q) is nearest FP64)
    best = None
    for cand in (np.nextafter(f, F32(-np.inf)), f, np.nextafter(f, F32(np.inf))):
        d = abs(Fraction(float(cand)) - q)
        key = (d, int(np.frombuffer(F32(cand).tobytes(), np.uint32)[0]) & 1)
        if best is None or key < best[0]:
            best = (key, cand)
    return best[1]


def test_fma32_matches_rational_arithmetic():
    """fma32 against exact rational arithmetic, on random operands and on
    constructed ties where FP64 rounding of the sum would mislead."""
    rng = np.random.default_rng(5)
    a = (rng.standard_normal(3000) * 10.0 ** rng.integers(-3, 4, 3000)).astype(F32)
    b = (rng.standard_normal(3000) * 10.0 ** rng.integers(-3, 4, 3000)).astype(F32)
    c = (rng.standard_normal(3000) * 10.0 ** rng.integers(-6, 6, 3000)).astype(F32)
    # ties: c = 1 and a*b half an FP32 ulp of 1 plus or minus a tiny amount
    a_t = np.array([1.0, 1.0 + 2.0 ** -23, 1.0 - 2.0 ** -24, 3.0, -1.0], dtype=F32)
    b_t = np.array([2.0 ** -24, 2.0 ** -24, 2.0 ** -24, 2.0 ** -25, 2.0 ** -25], dtype=F32)
    c_t = np.array([1.0, 1.0, 1.0, 1.0, 1.0], dtype=F32)
    a, b, c = np.concatenate([a, a_t]), np.concatenate([b, b_t]), np.concatenate([c, c_t])
    got = fma32(a, b, c)
    for i in range(len(a)):
        q = Fraction(float(a[i])) * Fraction(float(b[i])) + Fraction(float(c[i]))
        want = _round32_exact(q)
        assert got[i] == want, (i, a[i], b[i], c[i], got[i], want)
    # the constructed ties: 1 + 2^-24 (exact tie) rounds to even (1); slightly
    # more rounds up; 3 * 2^-25 = 1.5 half-ulps rounds up
    assert got[-5] == F32(1.0) and got[-4] == F32(1.0 + 2.0 ** -23) and got[-2] == F32(1.0 + 2.0 ** -23)


# ---------------------------------------------------------------------------
# the look-up tables, entry by entry
# ---------------------------------------------------------------------------

def _geometries():
    """(name, kind, los, box, edges1, edges2, n_hint, bounds) of the workload shapes."""
    lin = synth.linear_edges(0, 200, 40)
    shell_lo, shell_hi = [400.0, -10.0, -560.0], [2010.0, 1760.0, 560.0]
    return [
        ("C1 s", "s", "z", 1000.0, lin, None, 20_000, None),
        ("C2 smu", "smu", "z", 2000.0, lin, synth.mu_edges(100), 1_000_000, None),
        ("C2 spi z", "spi", "z", 2000.0, lin, lin, 1_000_000, None),
        ("C3 spi mid", "spi", "mid", 0.0, lin, lin, 2_000_000, (shell_lo, shell_hi)),
        ("C3 smu mid", "smu", "mid", 0.0, lin, synth.mu_edges(100), 2_000_000, (shell_lo, shell_hi)),
        ("C5 s log", "s", "z", 3000.0, synth.log_edges(0.1, 50.0, 50), None, 10_000_000, None),
    ]


def _plan(g):
    name, kind, los, box, e1, e2, n_hint, bounds = g
    p = fcfc.Plan(kind, e1, e2, los=los, box=box, n_hint=n_hint)
    if bounds is not None:
        p.set_bounds(*bounds)
    return p


def _tables(p):
    """[(label, first-axis table, second-axis table or None)]: the default and the
    doubled tables, as the kernel may take either."""
    two = p.kind == "spi"
    out = [("default", p.table(0), p.table(1) if two else None)]
    if p.numerics()["has_big"]:
        out.append(("doubled", p.table(2), p.table(3) if two else None))
    return out


def _check_table(t, edges, what):
    E, lo, hi, tab = t["E"], t["lo"].astype(F64), t["hi"].astype(F64), t["tab"].astype(np.int64)
    n = len(E) - 1
    e = np.asarray(edges, dtype=F64)
    assert np.array_equal(E, e * e), what
    scale = float(t["scale"])
    m, _ = np.frexp(scale)
    assert m == 0.5, f"{what}: scale {scale} is not a power of two"
    assert t["vmax"] == t["hi"][n], what
    # the largest FP32 value below vmax still indexes the table
    below = float(np.nextafter(t["vmax"], F32(0)))
    assert int(np.floor(below * scale)) < len(tab), what
    # every non-empty band holds its edge; bands are ordered
    pos = E > 0
    assert np.all(lo[pos] <= E[pos]) and np.all(E[pos] <= hi[pos]) and np.all(lo[pos] < hi[pos]), what
    assert np.all(lo[~pos] == 0) and np.all(hi[~pos] == 0), what
    assert np.all(np.diff(lo) >= 0) and np.all(np.diff(hi) >= 0), what
    j = np.arange(len(tab), dtype=F64)
    a = j / scale
    b = (j + 1) / scale
    nonempty = hi > lo
    meets = (lo[None, :] < b[:, None]) & (hi[None, :] > a[:, None]) & nonempty[None, :]
    first = np.where(meets.any(axis=1), meets.argmax(axis=1), -1)
    hot = tab <= -2
    # a hot entry names the first band meeting it, and every edge below that one
    # is certainly at or below the entry (band end <= a)
    assert np.array_equal(-2 - tab[hot], first[hot]), what
    for jj in np.nonzero(hot)[0][:: max(1, hot.sum() // 2000)]:
        k = first[jj]
        assert np.all(hi[:k] <= a[jj]), (what, jj)
    # a clean entry is met by no band
    assert np.all(first[~hot] == -1), what
    clean = (tab >= 0)
    c = tab[clean]
    assert np.all(c <= n - 1), what
    # its whole value range lies at or above its lower edge's band and below
    # its upper edge's band
    assert np.all(hi[c] <= a[clean]) and np.all(b[clean] <= lo[c + 1]), what
    none = tab == -1
    assert np.all((b[none] <= lo[0]) | (a[none] >= hi[n])), what
    assert np.all(hot | clean | none), what
    return int(hot.sum()), len(tab)


def test_every_table_entry_against_fp64_edges():
    for g in _geometries():
        p = _plan(g)
        try:
            for label, t1, t2 in _tables(p):
                nh, nt = _check_table(t1, g[4], f"{g[0]} {label} axis 1")
                if t2 is not None:
                    _check_table(t2, g[5], f"{g[0]} {label} axis 2")
                assert nh < 0.1 * nt
        finally:
            p.close()


# ---------------------------------------------------------------------------
# the kernel's arithmetic, pair by pair
# ---------------------------------------------------------------------------

def _cells(x, num, box):
    """Cell index per axis (FP64 floor of (x - lo) / side, clamped) and the cell
    origin lo + c * side, as the cell build forms them."""
    lo = np.asarray(num["lo"], dtype=F64)
    n = np.array([num["nx"], num["ny"], num["nz"]])
    c = np.floor((x - lo) / num["side"])
    c = np.clip(c, 0, n - 1).astype(np.int64)
    return c, lo + c.astype(F64) * num["side"]


def _displacement32(A, B, num, box):
    """FP32 displacement B - A exactly as the counting kernel forms it."""
    cA, oA = _cells(A, num, box)
    cB, oB = _cells(B, num, box)
    a32 = (A - oA).astype(F32)
    b32 = (B - oB).astype(F32)
    dc = cB - cA
    if box > 0:
        n = np.array([num["nx"], num["ny"], num["nz"]])
        dc = dc - n * np.round(dc / n).astype(np.int64)
    D = dc.astype(F32) * F32(num["side32"])
    return b32 - (a32 - D)


def _lookup(t, v):
    """Bin (>= 0), -1 (out of range) or -2 (recheck) of FP32 values v < vmax."""
    tab = t["tab"]
    j = np.floor(v.astype(F64) * float(t["scale"])).astype(np.int64)
    r = tab[j].astype(np.int64)
    hot = np.nonzero(r <= -2)[0]
    if len(hot):
        lo, hi = t["lo"], t["hi"]
        n = len(lo) - 1
        vv = v[hot]
        k = -2 - r[hot]
        c = k.copy()
        res = np.full(len(hot), -3, dtype=np.int64)
        active = np.ones(len(hot), dtype=bool)
        while active.any():
            kk = np.minimum(k, n)
            past = active & (k <= n) & (vv >= hi[kk])
            inband = active & (k <= n) & ~(vv >= hi[kk]) & (vv >= lo[kk])
            res[inband] = -2
            c[past] = k[past] + 1
            stop = active & ~past
            active = active & past
            k = k + 1
            done = stop & ~inband
            res[done] = np.where((c[done] >= 1) & (c[done] <= n), c[done] - 1, -1)
        r[hot] = res
    return r


def _rsq(x, delta):
    return (1.0 / np.sqrt(x.astype(F64)) * (1.0 + delta)).astype(F32)


def _rcp(x, delta):
    return (1.0 / x.astype(F64) * (1.0 + delta)).astype(F32)


def _values(kind, los, num, n2, d, A, deltas, vmax):
    """The kernel's FP32 values per pair (they do not depend on which table is
    used): the candidate mask and the squared separations, mu * n2 and its band."""
    with np.errstate(divide="ignore", invalid="ignore"):
        dx, dy, dz = d[:, 0], d[:, 1], d[:, 2]
        v = {}
        if kind == "spi" and los == "z":
            v1 = fma32(dy, dy, dx * dx)
            v2 = dz * dz
            idx = np.nonzero((v1 < vmax[0]) & (v2 < vmax[1]))[0]
            v["sp2"], v["pi2"] = v1[idx], v2[idx]
        else:
            d2 = fma32(dz, dz, fma32(dy, dy, dx * dx))
            idx = np.nonzero(d2 < F32(num["r2prune32"]))[0]
            v["d2"] = d2[idx]
        v["idx"] = idx
        if kind == "s" or (kind == "spi" and los == "z"):
            return v
        if los == "mid":
            q = 2.0 * A[idx].astype(F32)
            l = q + d[idx]
            lx, ly, lz = l[:, 0], l[:, 1], l[:, 2]
            ex, ey, ez = dx[idx], dy[idx], dz[idx]
            dot = fma32(ez, lz, fma32(ey, ly, ex * lx))
            ll = fma32(lz, lz, fma32(ly, ly, lx * lx))
        if kind == "smu":
            mu_n = F32(n2)
            if los == "z":
                proj_n = np.abs(dz[idx]) * mu_n
            else:
                proj_n = np.abs(dot) * (_rsq(ll, deltas[1]) * mu_n)
            rs = _rsq(v["d2"], deltas[0])
            mun = proj_n * rs
            tolA = F32(num["mu_tolA"]) if n2 > 1 else F32(0)
            tolC = F32(num["mu_tolC"]) if n2 > 1 else F32(0)
            cr = np.clip(np.rint(mun), F32(1), F32(max(n2 - 1, 1))).astype(F32)
            tol = fma32(np.full_like(rs, tolA), rs, np.full_like(rs, tolC))
            v["mun"], v["tol"] = mun, tol
            v["mb"] = np.minimum(np.nan_to_num(np.floor(mun), nan=0.0).astype(np.int64), n2 - 1)
            v["mu_band"] = (np.abs(mun - cr) < tol) | (v["d2"] < F32(num["d2small"]))
            return v
        pi2 = (dot * dot) * _rcp(ll, deltas[0])
        v["pi2"] = pi2
        v["sp2"] = np.maximum(v["d2"] - pi2, F32(0))
        return v


def _classify(kind, n2, v, t1, t2, npairs):
    """The kernel's decision per pair from its FP32 values and a table: flat bin,
    -1 (dropped) or -2 (binned again in FP64)."""
    out = np.full(npairs, -1, dtype=np.int64)
    idx = v["idx"]
    if kind == "s":
        out[idx] = _lookup(t1, v["d2"])
    elif kind == "smu":
        sb = _lookup(t1, v["d2"])
        rm = (sb == -2) | v["mu_band"]
        out[idx] = np.where(rm, -2, np.where(sb >= 0, sb * n2 + v["mb"], -1))
    else:
        sp2, pi2 = v["sp2"], v["pi2"]
        inm = (sp2 < t1["vmax"]) & (pi2 < t2["vmax"])
        b1 = _lookup(t1, np.where(inm, sp2, F32(0)))
        b2 = _lookup(t2, np.where(inm, pi2, F32(0)))
        rm = ((b1 == -2) | (b2 == -2)) & inm
        out[idx] = np.where(rm, -2, np.where(inm & (b1 >= 0) & (b2 >= 0), b1 * n2 + b2, -1))
    return out


def _exact_values(kind, los, box, n2, A, B):
    """FP64 values of the quantities the FP32 ones stand for: d2 (or s_perp^2 and
    pi^2) and mu * n2, by the definitions of Sect. 2.5 (minimum image in a
    periodic box; mid-point line of sight along x_a + x_b)."""
    d = B - A
    if box > 0:
        d = d - box * np.round(d / box)
    d2 = (d[:, 0] * d[:, 0] + d[:, 1] * d[:, 1]) + d[:, 2] * d[:, 2]
    if kind == "s":
        return {"v1": d2}
    if los == "z":
        par2 = d[:, 2] * d[:, 2]
    else:
        l = A + B
        dot = (d * l).sum(axis=1)
        par2 = dot * dot / (l * l).sum(axis=1)
    if kind == "smu":
        with np.errstate(invalid="ignore", divide="ignore"):
            return {"v1": d2, "mun": np.sqrt(par2 / d2) * n2}
    sp2 = d2 - par2 if los == "mid" else d[:, 0] * d[:, 0] + d[:, 1] * d[:, 1]
    return {"v1": np.maximum(sp2, 0.0), "v2": par2}


def _band_use(v32, V, t):
    """Largest |v32 - V| over the half-width of the band of the nearest edge, for
    values V within a half-width of that edge (where the band decides)."""
    E, lo, hi = t["E"], t["lo"].astype(F64), t["hi"].astype(F64)
    k = np.clip(np.searchsorted(E, V), 1, len(E) - 1)
    k = np.where(np.abs(V - E[k - 1]) < np.abs(V - E[k]), k - 1, k)
    hw = np.minimum(E[k] - lo[k], hi[k] - E[k])
    near = (hw > 0) & (np.abs(V - E[k]) <= hw)
    if not near.any():
        return 0.0
    return float(np.max(np.abs(v32[near].astype(F64) - V[near]) / hw[near]))


def _unit(rng, m):
    v = rng.standard_normal((m, 3))
    return v / np.linalg.norm(v, axis=1)[:, None]


def _from_perp_par(A, perp, par, los, rng):
    """Displacements with the given components across and along the line of
    sight (z, or the mid-point direction, which itself depends on d)."""
    phi = rng.random(len(perp)) * 2 * np.pi
    if los == "z":
        return np.stack([perp * np.cos(phi), perp * np.sin(phi), par], axis=1)
    d = np.zeros((len(perp), 3))
    for _ in range(4):
        lh = 2.0 * A + d
        lh /= np.linalg.norm(lh, axis=1)[:, None]
        t1 = np.cross(lh, [0.0, 0.0, 1.0])
        t1 /= np.linalg.norm(t1, axis=1)[:, None]
        t2 = np.cross(lh, t1)
        d = par[:, None] * lh + perp[:, None] * (np.cos(phi)[:, None] * t1 + np.sin(phi)[:, None] * t2)
    return d


def _pairs(g, m, rng, bounds_box):
    """m pairs (A, B) of the geometry: A from the workload's point distribution
    (uniform in a periodic box, the survey shell in an open one); B at a
    separation that is volume-uniform out to just past the largest edge (a
    third of the pairs), with the first binned coordinate (s or s_perp) close
    to one of its edges (a third), or the second (mu or pi) close to one of its
    edges (a third)."""
    name, kind, los, box, e1, e2, _, bounds = g
    if box > 0:
        A = rng.random((m, 3)) * box
    else:
        A = synth.survey_shell(m, int(rng.integers(1 << 30)))
    top = e1[-1] if kind != "spi" else np.hypot(e1[-1], e2[-1])
    case = rng.integers(0, 3, m)
    # relative offsets from an edge spread from 1e-9 to 1e-3, so that pairs
    # fall deep inside every band, near its ends and just outside it
    eps = rng.choice([-1.0, 1.0], m) * 10.0 ** rng.uniform(-9.0, -3.0, m)
    d = _unit(rng, m) * (top * 1.02 * np.cbrt(rng.random(m)))[:, None]
    lo1 = 1 if e1[0] == 0 else 0
    for c in (1, 2):
        sel = np.nonzero(case == c)[0]
        k = len(sel)
        if k == 0 or (kind == "s" and c == 2):
            continue
        sgn = rng.choice([-1.0, 1.0], k)
        if kind == "spi":
            if c == 1:
                perp = e1[rng.integers(lo1, len(e1), k)] * (1.0 + eps[sel])
                par = rng.uniform(-1.02, 1.02, k) * e2[-1]
            else:
                perp = e1[-1] * 1.02 * np.sqrt(rng.random(k))
                par = e2[rng.integers(0, len(e2), k)] * (1.0 + eps[sel]) * sgn
            d[sel] = _from_perp_par(A[sel], perp, par, los, rng)
        elif c == 1:
            d[sel] = _unit(rng, k) * (e1[rng.integers(lo1, len(e1), k)] * (1.0 + eps[sel]))[:, None]
        else:
            mu = np.clip(e2[rng.integers(0, len(e2), k)] * (1.0 + eps[sel]), 0.0, 1.0)
            r = top * 1.02 * np.cbrt(rng.random(k))
            d[sel] = _from_perp_par(A[sel], np.sqrt(1.0 - mu * mu) * r, mu * r * sgn, los, rng)
    B = A + d
    if box > 0:
        B = np.minimum(np.mod(B, box), np.nextafter(box, 0))
    else:
        lo, hi = bounds_box
        ok = np.all((B >= lo) & (B <= hi), axis=1)
        A, B, case = A[ok], B[ok], case[ok]
    return A, B, case


def _knife_pairs(g, rng):
    """Pairs on or next to an edge in FP64, in a periodic box: points on a 1/128
    lattice displaced by a Pythagorean triple scaled to a first-axis edge (an
    exact edge where the scale is exact) or to a multiple of 1/8 (mu exactly
    0, 0.28, 0.6, 0.64, 0.8, 0.96 or 1 with s between edges); every coordinate
    exact, so the pairs the oracle sees are the ones constructed."""
    name, kind, los, box, e1, e2, _, _ = g
    if box <= 0:
        return np.zeros((0, 3)), np.zeros((0, 3)), np.zeros(0, dtype=np.int64)
    m = 20000
    A = np.floor(rng.random((m, 3)) * box * 128) / 128
    trip = np.array([[0, 3, 4, 5], [0, 4, 3, 5], [0, 7, 24, 25], [0, 24, 7, 25], [9, 12, 20, 25],
                     [12, 15, 16, 25], [0, 0, 1, 1], [0, 1, 0, 1], [1, 0, 0, 1]], dtype=F64)
    t = trip[rng.integers(0, len(trip), m)]
    ek = e1[rng.integers(0, len(e1), m)]
    onedge = rng.random(m) < 0.5
    scale = np.where(onedge, ek / t[:, 3], np.floor(rng.random(m) * e1[-1] * 8) / 8 / t[:, 3])
    scale = np.round(scale * 2.0 ** 20) / 2.0 ** 20
    d = t[:, :3] * scale[:, None] * rng.choice([-1.0, 1.0], (m, 3))
    B = np.mod(A + d, box)
    return A, B, np.full(m, 3)


@pytest.mark.parametrize("gi", range(6), ids=[g[0] for g in _geometries()])
def test_kernel_fp32_decisions_match_the_oracle(gi):
    g = _geometries()[gi]
    name, kind, los, box, e1, e2, _, bounds = g
    p = _plan(g)
    try:
        num = p.numerics()
        tabs = _tables(p)
    finally:
        p.close()
    n2 = 1 if kind == "s" else len(e2) - 1
    ok_kw = dict(kind=kind, edges1=e1, edges2=e2, los=los, box=box)
    if kind == "smu" and los == "mid":
        deltas_set = [(-1, -1), (0, 0), (1, 1), (-1, 1), (1, -1)]
    elif kind == "s" or (kind != "s" and los == "z" and kind == "spi"):
        deltas_set = [(0, 0)]
    else:
        deltas_set = [(-1, 0), (0, 0), (1, 0)]
    tr = float(num["trans_rel"])
    rng = np.random.default_rng(1000 + gi)
    bbox = (np.asarray(bounds[0]), np.asarray(bounds[1])) if bounds else None
    total = checked = rechecked = binned = 0
    u_in = u_rechecked = 0
    use = {}
    chunks = []
    A, B, case = _knife_pairs(g, rng)
    if len(A):
        chunks.append((A, B, case))
    want = N_FULL if name in ("C2 smu", "C3 spi mid", "C5 s log") else N_SHORT
    while total < want:
        A, B, case = _pairs(g, CHUNK, rng, bbox)
        chunks.append((A, B, case))
        total += len(A)
    total = 0
    for A, B, case in chunks:
        ref = oracle.classify_pairs(A, B, **ok_kw)
        d = _displacement32(A, B, num, box)
        for dl in deltas_set:
            vals = _values(kind, los, num, n2, d, A, (dl[0] * tr, dl[1] * tr),
                           (tabs[0][1]["vmax"], tabs[0][2]["vmax"] if tabs[0][2] is not None else None))
            if dl == (0, 0):
                ex = _exact_values(kind, los, box, n2, A[vals["idx"]], B[vals["idx"]])
                t1, t2 = tabs[0][1], tabs[0][2]
                if kind == "spi":
                    use["axis 1"] = max(use.get("axis 1", 0.0), _band_use(vals["sp2"], ex["v1"], t1))
                    use["axis 2"] = max(use.get("axis 2", 0.0), _band_use(vals["pi2"], ex["v2"], t2))
                else:
                    use["d2"] = max(use.get("d2", 0.0), _band_use(vals["d2"], ex["v1"], t1))
                if kind == "smu":
                    mun, tol, V = vals["mun"].astype(F64), vals["tol"].astype(F64), ex["mun"]
                    near = (np.abs(V - np.rint(V)) <= tol) & (np.rint(V) >= 1) & (np.rint(V) <= n2 - 1) & \
                           (vals["d2"] >= F32(num["d2small"]))
                    if near.any():
                        use["mu"] = max(use.get("mu", 0.0), float(np.max(np.abs(mun[near] - V[near]) / tol[near])))
            for label, t1, t2 in tabs:
                got = _classify(kind, n2, vals, t1, t2, len(A))
                clean = got >= 0
                bad = np.nonzero(clean & (got != ref))[0]
                assert len(bad) == 0, (name, label, dl, A[bad[:3]], B[bad[:3]], got[bad[:3]], ref[bad[:3]])
                dropped = np.nonzero((got == -1) & (ref >= 0))[0]
                assert len(dropped) == 0, (name, label, dl, A[dropped[:3]], B[dropped[:3]], ref[dropped[:3]])
                checked += len(got)
                rechecked += int((got == -2).sum())
                binned += int(clean.sum())
                uni = (case == 0) & (ref >= 0)
                u_in += int(uni.sum())
                u_rechecked += int((uni & (got == -2)).sum())
        total += len(A)
    assert total >= min(want, 10_000_000)
    u_rate = u_rechecked / max(u_in, 1)
    print(f"[bands] {name}: {total} pairs x {len(tabs)} tables x {len(deltas_set)} rsq/rcp ends; "
          f"binned in FP32 {binned / checked:.3f}, rechecked {rechecked / checked:.4f}; "
          f"volume-uniform pairs in range rechecked {u_rate:.5f}; largest share of a band the FP32 error "
          f"takes: " + ", ".join(f"{k} {v:.3f}" for k, v in use.items()))
    assert all(v < 1.0 for v in use.values()), use
    # two thirds of the pairs are built within a few ulps of an edge and are
    # mostly rechecked; pairs at the workload's own separations rarely are
    assert u_rate < 0.02


# ---------------------------------------------------------------------------
# triangle sides
# ---------------------------------------------------------------------------

U32 = 2.0 ** -24
U64 = 2.0 ** -53


def _min_image(d, box):
    if box <= 0:
        return d
    h = 0.5 * box
    return np.where(d > h, d - box, np.where(d < -h, d + box, d))


@pytest.mark.parametrize("box,r,scale", [(1000.0, 30.0, 1000.0), (120.0, 30.0, 120.0), (0.0, 30.0, 2000.0)])
def test_triangle_side_fp32_error_within_the_band_model(box, r, scale):
    """The triangle kernel bins the side between two neighbours p, q of a
    primary from their FP32 displacements (each the FP64 displacement of the
    definition, minimum image in a periodic box, rounded to FP32): the FP32
    difference per axis and the fma chain of its squares.  Its table bands are
    built from |Q32 - Q64| <= 2 sqrt3 e sqrt(Q) + 3 e^2 + 3.3 u Q with e twice
    the per-axis error 4 u r' + 4 u64 (L + r').  Checked here against the FP64
    side of the definition formed directly from the stored positions, over
    random and adversarial triples: neighbours at the reach in every axis,
    across the periodic faces, and far from the origin of an open box."""
    rng = np.random.default_rng(int(box) + 7)
    n = 400_000
    rr = r * (1.0 + 1e-6) + 1e-9 * max(box, 0.0)
    e = 2.0 * (4.0 * U32 * rr + 4.0 * 2.0 ** -52 * (max(box, 0.0) + rr))
    hi = box if box > 0 else scale
    P = rng.uniform(0.0, hi, (n, 3))
    # neighbour offsets: uniform in the ball, or on the reach along the axes
    off = []
    for _ in range(2):
        v = rng.normal(size=(n, 3))
        v /= np.linalg.norm(v, axis=1)[:, None]
        rad = r * rng.uniform(0, 1, n) ** (1 / 3)
        edge = rng.random(n) < 0.3
        rad[edge] = r * (1 - rng.uniform(0, 1e-6, edge.sum()))
        axis = rng.random(n) < 0.2
        v[axis] = np.sign(rng.normal(size=(axis.sum(), 3))) / np.sqrt(3.0)
        off.append(v * rad[:, None])
    if box > 0:
        # primaries within r of a face, so that neighbours wrap
        face = rng.random(n) < 0.5
        P[face, 0] = rng.uniform(0, r, face.sum())
    Q1 = P + off[0]
    Q2 = P + off[1]
    if box > 0:
        Q1 = np.mod(Q1, box)
        Q2 = np.mod(Q2, box)
    # the kernel: FP64 displacements from the primary, rounded to FP32
    d1 = _min_image(Q1 - P, box).astype(F32)
    d2 = _min_image(Q2 - P, box).astype(F32)
    ex = d2 - d1
    v32 = fma32(ex[:, 2], ex[:, 2], fma32(ex[:, 1], ex[:, 1], ex[:, 0] * ex[:, 0])).astype(F64)
    # the definition, from the stored positions
    D = _min_image(Q2 - Q1, box)
    V = (D[:, 0] * D[:, 0] + D[:, 1] * D[:, 1]) + D[:, 2] * D[:, 2]
    bound = 2.0 * np.sqrt(3.0) * e * np.sqrt(V) + 3.0 * e * e + (3.3 * U32 + 1e-15) * V
    err = np.abs(v32 - V)
    share = float(np.max(err / bound))
    print(f"[bands] triangle sides, box {box}, r {r}: {n} pairs, largest share of the bound used {share:.3f}")
    assert share < 1.0
    # the bound is not loose by orders of magnitude (it would then send many
    # sides to the FP64 recheck for nothing)
    assert share > 0.05
