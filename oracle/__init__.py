"""CPU oracle for exact pair counting -- TEST INFRASTRUCTURE ONLY.

Only the test suite, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The product library never does; it
shares no code with it.  The counting rules (separation definitions of
Sect. 2.5, half-open squared-edge bins of Sect. 3.2, auto pairs counted once as
in Sect. 3.1) are written out in ``fcfc_oracle.c``.
"""
import ctypes
import os

import numpy as np

from . import build as _build

KIND = {"s": 0, "smu": 1, "spi": 2}
LOS = {"z": 0, "mid": 1}

_lib = None


def _load():
    global _lib
    if _lib is None:
        path = _build.LIB
        if not os.path.exists(path) or os.path.getmtime(path) < os.path.getmtime(_build.SRC):
            _build.build(force=True)
        lib = ctypes.CDLL(path)
        P = ctypes.c_void_p
        i64 = ctypes.c_int64
        ci = ctypes.c_int
        cd = ctypes.c_double
        lib.oracle_count_brute.argtypes = [P, P, i64, P, P, i64, ci, ci, ci, cd, P, ci, P, ci, P, P, ci]
        lib.oracle_count_brute.restype = ci
        lib.oracle_count_grid.argtypes = [P, P, i64, P, P, i64, ci, ci, ci, cd, P, ci, P, ci, cd, P, P, ci]
        lib.oracle_count_grid.restype = ci
        lib.oracle_classify_pair.argtypes = [P, P, ci, ci, cd, P, ci, P, ci]
        lib.oracle_classify_pair.restype = ctypes.c_long
        lib.oracle_classify_pairs.argtypes = [P, P, i64, ci, ci, cd, P, ci, P, ci, P]
        lib.oracle_classify_pairs.restype = ci
        lib.oracle_triplets_brute.argtypes = [P, i64, cd, P, ci, P, ci]
        lib.oracle_triplets_brute.restype = ci
        lib.oracle_triplets_list.argtypes = [P, i64, cd, P, ci, P, ci]
        lib.oracle_triplets_list.restype = ci
        lib.oracle_triplets_list_w.argtypes = [P, P, i64, cd, P, ci, P, P, ci]
        lib.oracle_triplets_list_w.restype = ci
        lib.oracle_version.restype = ci
        _lib = lib
    return _lib


def _f64(a, shape_last=None):
    a = np.ascontiguousarray(np.asarray(a, dtype=np.float64))
    if shape_last is not None:
        a = a.reshape(-1, shape_last)
    return a


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


class OracleError(RuntimeError):
    pass


def count(x1, x2=None, *, kind="s", edges1, edges2=None, los="z", box=0.0,
          w1=None, w2=None, method="brute", cell=None, threads=0):
    """Exact pair counts.

    x1, x2: (N,3) float64 positions.  x2=None -> auto count (pairs i<j of x1).
    kind: "s", "smu" or "spi";  los: "z" or "mid";  box: L>0 periodic, 0 open.
    edges1: s (or sigma) edges; edges2: mu (or pi) edges.
    Weighted when w1 (and w2 for a cross count) are given.
    Returns (counts int64 [n1, n2] (or [n1] for "s"), wcounts float64 or None).
    """
    lib = _load()
    x1 = _f64(x1, 3)
    auto = x2 is None
    x2a = x1 if auto else _f64(x2, 3)
    e1 = _f64(edges1)
    n1 = len(e1) - 1
    if kind == "s":
        e2 = np.array([0.0, 1.0])
        n2 = 1
    else:
        e2 = _f64(edges2)
        n2 = len(e2) - 1
    weighted = w1 is not None
    w1a = _f64(w1) if weighted else None
    w2a = (w1a if auto else _f64(w2)) if weighted else None
    counts = np.zeros(n1 * n2, dtype=np.int64)
    wcounts = np.zeros(n1 * n2, dtype=np.float64) if weighted else None
    if method == "brute":
        rc = lib.oracle_count_brute(_ptr(x1), _ptr(w1a), len(x1), _ptr(x2a), _ptr(w2a), len(x2a),
                                    int(auto), KIND[kind], LOS[los], float(box), _ptr(e1), n1,
                                    _ptr(e2), n2, _ptr(counts), _ptr(wcounts), int(threads))
    elif method == "grid":
        if cell is None:
            rmax = float(e1[-1]) if kind != "spi" else float(np.hypot(e1[-1], e2[-1]))
            cell = rmax / 2.0
        rc = lib.oracle_count_grid(_ptr(x1), _ptr(w1a), len(x1), _ptr(x2a), _ptr(w2a), len(x2a),
                                   int(auto), KIND[kind], LOS[los], float(box), _ptr(e1), n1,
                                   _ptr(e2), n2, float(cell), _ptr(counts), _ptr(wcounts), int(threads))
    else:
        raise ValueError(method)
    if rc != 0:
        raise OracleError(f"oracle returned {rc}")
    shape = (n1,) if kind == "s" else (n1, n2)
    return counts.reshape(shape), (wcounts.reshape(shape) if weighted else None)


def triplets(x, *, edges, box=0.0, method="list", w=None, threads=0):
    """Triangle counts of the points x ((N,3) float64): every set of three
    distinct points once, when its three sides lie in [edges[0], edges[-1]),
    binned by the sorted side bins (a <= b <= c) into an int64 [n, n, n]
    histogram (zero where a > b or b > c).  method "brute" (triple loop) or
    "list" (neighbour lists from each point's lowest-index triangles).
    With weights w (list method): returns (counts, weighted counts), a
    triangle weighing fl(fl(a*b)*c) for its weights sorted a <= b <= c, each
    bin the exact sum rounded once."""
    lib = _load()
    x = _f64(x, 3)
    e = _f64(edges)
    nb = len(e) - 1
    counts = np.zeros(nb * nb * nb, dtype=np.int64)
    if w is not None:
        wa = _f64(w)
        wc = np.zeros(nb * nb * nb, dtype=np.float64)
        rc = lib.oracle_triplets_list_w(_ptr(x), _ptr(wa), len(x), float(box), _ptr(e), nb, _ptr(counts),
                                        _ptr(wc), int(threads))
        if rc != 0:
            raise OracleError(f"oracle returned {rc}")
        return counts.reshape(nb, nb, nb), wc.reshape(nb, nb, nb)
    fn = {"brute": lib.oracle_triplets_brute, "list": lib.oracle_triplets_list}[method]
    rc = fn(_ptr(x), len(x), float(box), _ptr(e), nb, _ptr(counts), int(threads))
    if rc != 0:
        raise OracleError(f"oracle returned {rc}")
    return counts.reshape(nb, nb, nb)


def classify_pair(p1, p2, *, kind="s", edges1, edges2=None, los="z", box=0.0):
    """Flat bin index of one pair (p1 from catalogue 1, p2 from catalogue 2), or -1."""
    lib = _load()
    a = _f64(p1)
    b = _f64(p2)
    e1 = _f64(edges1)
    e2 = np.array([0.0, 1.0]) if kind == "s" else _f64(edges2)
    r = lib.oracle_classify_pair(_ptr(a), _ptr(b), KIND[kind], LOS[los], float(box), _ptr(e1),
                                 len(e1) - 1, _ptr(e2), len(e2) - 1)
    if r == -2:
        raise OracleError("bad specification")
    return int(r)


def classify_pairs(p1, p2, *, kind="s", edges1, edges2=None, los="z", box=0.0):
    """Flat bin index (int64, -1 out of range) of each pair (p1[i], p2[i]), (n, 3) arrays."""
    lib = _load()
    a = _f64(p1, 3)
    b = _f64(p2, 3)
    if a.shape != b.shape:
        raise ValueError("p1 and p2 must have the same shape")
    e1 = _f64(edges1)
    e2 = np.array([0.0, 1.0]) if kind == "s" else _f64(edges2)
    out = np.empty(len(a), dtype=np.int64)
    r = lib.oracle_classify_pairs(_ptr(a), _ptr(b), len(a), KIND[kind], LOS[los], float(box), _ptr(e1),
                                  len(e1) - 1, _ptr(e2), len(e2) - 1, _ptr(out))
    if r == -2:
        raise OracleError("bad specification")
    return out
