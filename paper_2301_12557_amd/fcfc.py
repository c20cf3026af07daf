"""ctypes binding of libfcfc.so (include/fcfc.h) -- argument marshalling only.

Every step of the pair count runs in the HIP library; this module turns torch
device tensors into pointers and sizes and checks return codes.  If the
library is missing it raises: there is no fallback.
"""
import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "_lib", "libfcfc.so")

FCFC_OK = 0
STATUS = {0: "FCFC_OK", -1: "FCFC_EINVAL", -2: "FCFC_ENOMEM", -3: "FCFC_EBOX", -4: "FCFC_ENONFINITE",
          -5: "FCFC_ERANGE", -6: "FCFC_EEDGES", -7: "FCFC_EGRID", -8: "FCFC_EHIP", -9: "FCFC_EMODEL",
          -10: "FCFC_ESTATE"}
KIND = {"s": 0, "smu": 1, "spi": 2}
LOS = {"z": 0, "mid": 1}
ORDER = {"heuristic": 0, "built": 1, "learned": 2}


class FcfcError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{STATUS.get(code, code)}: {msg}")
        self.code = code
        self.name = STATUS.get(code, str(code))


class Catalog(ctypes.Structure):
    _fields_ = [("xyz", ctypes.c_void_p), ("w", ctypes.c_void_p), ("n", ctypes.c_int64)]


class Tuning(ctypes.Structure):
    _fields_ = [("cells_per_rmax", ctypes.c_int32), ("tile_points", ctypes.c_int32),
                ("seg_cells", ctypes.c_int32), ("b_chunk", ctypes.c_int32),
                ("hist_copies", ctypes.c_int32), ("order", ctypes.c_int32),
                ("record_timing", ctypes.c_int32), ("n_hint", ctypes.c_int32),
                ("lut_log2", ctypes.c_int32), ("group_waves", ctypes.c_int32),
                ("shard_count", ctypes.c_int32), ("shard_index", ctypes.c_int32),
                ("batch_chunk", ctypes.c_int32), ("flush_log2", ctypes.c_int32),
                ("tree_leaf", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class Stats(ctypes.Structure):
    _fields_ = [("items", ctypes.c_int64), ("candidates", ctypes.c_int64), ("rechecks", ctypes.c_int64),
                ("in_range", ctypes.c_int64), ("cells", ctypes.c_int64), ("grid", ctypes.c_int32 * 3),
                ("cells_per_rmax", ctypes.c_int32), ("cell_side", ctypes.c_double),
                ("kernel_ms", ctypes.c_double), ("band_d2_rel", ctypes.c_double),
                ("lut_entries", ctypes.c_int32), ("wg_per_cu", ctypes.c_int32),
                ("order_used", ctypes.c_int32), ("group_waves", ctypes.c_int32),
                ("flushes", ctypes.c_int64)]

    def as_dict(self):
        d = {k: getattr(self, k) for k, _ in self._fields_}
        d["grid"] = list(self.grid)
        d["order_used"] = {v: k for k, v in ORDER.items()}.get(self.order_used, self.order_used)
        return d


class Numerics(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
                ("cells_per_rmax", ctypes.c_int32), ("lo", ctypes.c_double * 3), ("side", ctypes.c_double),
                ("e_axis", ctypes.c_double), ("side32", ctypes.c_float), ("r2prune32", ctypes.c_float),
                ("d2small", ctypes.c_float), ("mu_tolA", ctypes.c_float), ("mu_tolC", ctypes.c_float),
                ("trans_rel", ctypes.c_float), ("has_big", ctypes.c_int32), ("reserved", ctypes.c_int32)]


# (name, restype, argtypes) of every exported entry point of include/fcfc.h
_P = ctypes.c_void_p
_I32 = ctypes.c_int32
_I64 = ctypes.c_int64
_D = ctypes.c_double
SIGNATURES = [
    ("fcfc_plan_create", _I32, [_I32, _I32, _P, _I32, _P, _I32, _D, ctypes.POINTER(Tuning), ctypes.POINTER(_P)]),
    ("fcfc_plan_fit_bounds", _I32, [_P, ctypes.POINTER(Catalog), _I32, _P]),
    ("fcfc_plan_set_bounds", _I32, [_P, _P, _P]),
    ("fcfc_build_cells", _I32, [_P, ctypes.POINTER(Catalog), _P, ctypes.POINTER(_P)]),
    ("fcfc_count_pairs", _I32, [_P, _P, _P, _P, _P, _P]),
    ("fcfc_count_pairs_noalloc", _I32, [_P, _P, _P, _P, _P, _P]),
    ("fcfc_noalloc_scratch_bytes", _I64, []),
    ("fcfc_plan_stats", _I32, [_P, ctypes.POINTER(Stats)]),
    ("fcfc_plan_numerics", _I32, [_P, ctypes.POINTER(Numerics)]),
    ("fcfc_plan_table", _I32, [_P, _I32, _P, _P, _P, _P, _I64, ctypes.POINTER(_I64), ctypes.POINTER(ctypes.c_float),
                               ctypes.POINTER(ctypes.c_float)]),
    ("fcfc_weight_scale", _I32, [_D, _D, _D, _D, _I32, ctypes.POINTER(_I32)]),
    ("fcfc_batch_create", _I32, [_P, ctypes.POINTER(Catalog), _I32, _P, ctypes.POINTER(_P)]),
    ("fcfc_batch_create_pairs", _I32, [_P, ctypes.POINTER(Catalog), _I32, _P, _I32, _P, ctypes.POINTER(_P)]),
    ("fcfc_batch_run", _I32, [_P, _P, _P, _I32, _P]),
    ("fcfc_batch_check", _I32, [_P, _P, ctypes.POINTER(ctypes.c_uint32), ctypes.POINTER(ctypes.c_float)]),
    ("fcfc_batch_stats", _I32, [_P, _P, ctypes.POINTER(_I64)]),
    ("fcfc_batch_free", None, [_P]),
    ("fcfc_cells_free", None, [_P]),
    ("fcfc_plan_free", None, [_P]),
    ("fcfc_cells_info", _I32, [_P, ctypes.POINTER(_I64), ctypes.POINTER(_I64)]),
    ("fcfc_model_nparams", _I32, []),
    ("fcfc_model_create", _I32, [ctypes.c_uint64, ctypes.POINTER(_P)]),
    ("fcfc_model_free", None, [_P]),
    ("fcfc_model_get", _I32, [_P, _P, _P]),
    ("fcfc_model_set", _I32, [_P, _P, _P]),
    ("fcfc_model_predict", _I32, [_P, _P, _I64, _P, _P]),
    ("fcfc_model_grad", _I32, [_P, _P, _P, _I64, _P, ctypes.POINTER(ctypes.c_float), _P]),
    ("fcfc_model_train", _I32, [_P, _P, _P, _I64, _I32, _I32, ctypes.c_float, ctypes.c_uint64, _P,
                                ctypes.POINTER(ctypes.c_float)]),
    ("fcfc_model_save", _I32, [_P, ctypes.c_char_p]),
    ("fcfc_model_load", _I32, [ctypes.c_char_p, ctypes.POINTER(_P)]),
    ("fcfc_plan_timings", _I32, [_P, _P, _P, _I64, ctypes.POINTER(_I64), _P]),
    ("fcfc_plan_set_model", _I32, [_P, _P]),
    ("fcfc_plan_predict", _I32, [_P, _P, _P, _P, _P, ctypes.POINTER(_D), ctypes.POINTER(_I64)]),
    ("fcfc_choose_cells", _I32, [_P, _I32, _I32, _P, _I32, _P, _I32, _D, ctypes.POINTER(Tuning),
                                 ctypes.POINTER(Catalog), ctypes.POINTER(Catalog), _P, ctypes.POINTER(_I32),
                                 ctypes.POINTER(_D)]),
    ("fcfc_autotune", _I32, [_P, _I32, _I32, _P, _I32, _P, _I32, _D, ctypes.POINTER(Tuning),
                             ctypes.POINTER(Catalog), ctypes.POINTER(Catalog), _I32, ctypes.c_char_p, _P,
                             ctypes.POINTER(Tuning), ctypes.POINTER(_D), ctypes.POINTER(_D),
                             ctypes.POINTER(_I32)]),
    ("fcfc_diag_transcendental", _I32, [ctypes.POINTER(_D), ctypes.POINTER(_D), ctypes.POINTER(_D), _P]),
    ("fcfc_diag_peaks", _I32, [ctypes.POINTER(_D), ctypes.POINTER(_D), ctypes.POINTER(_D), ctypes.POINTER(_D), _P]),
    ("fcfc_xi", _I32, [_I32, ctypes.POINTER(_P), ctypes.POINTER(_D), ctypes.POINTER(_D), _I32, _I64, _P, _P]),
    ("fcfc_analytic_rr", _I32, [_P, _D, _P, _P]),
    ("fcfc_pair_norm", _I32, [_I64, _I64, ctypes.POINTER(_D)]),
    ("fcfc_landy_szalay", _I32, [_P, _P, _P, _I64, _I64, _I64, _P, _P]),
    ("fcfc_multipoles", _I32, [_P, _I32, ctypes.POINTER(_D), _I32, ctypes.POINTER(_I32), _I32, _P, _P]),
    ("fcfc_wp", _I32, [_P, _I32, ctypes.POINTER(_D), _I32, _P, _P]),
    ("fcfc_radec_to_unit", _I32, [_P, _P, _I64, _P, _P]),
    ("fcfc_angular_plan", _I32, [ctypes.POINTER(_D), _I32, ctypes.POINTER(Tuning), ctypes.POINTER(_D),
                                 ctypes.POINTER(_P)]),
    ("fcfc_bin_squared", _I32, [_P, _P, _I64, _P, _P]),
    ("fcfc_count_triplets", _I32, [_P, _P, _P, _P, _P]),
    ("fcfc_status_str", ctypes.c_char_p, [_I32]),
    ("fcfc_last_error", ctypes.c_char_p, []),
    ("fcfc_version", _I32, []),
]

_lib = None


def load():
    """Load libfcfc.so; raise if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: run __graft_entry__.build() "
                              "(or python paper_2301_12557_amd/build_lib.py) first")
        lib = ctypes.CDLL(LIB_PATH)
        for name, res, args in SIGNATURES:
            f = getattr(lib, name)
            f.restype = res
            f.argtypes = args
        _lib = lib
    return _lib


def check(code):
    if code != FCFC_OK:
        msg = load().fcfc_last_error().decode()
        raise FcfcError(code, msg)


def _stream_ptr(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _catalog(xyz, w=None):
    import torch
    if not (isinstance(xyz, torch.Tensor) and xyz.is_cuda and xyz.dtype == torch.float64
            and xyz.dim() == 2 and xyz.shape[1] == 3 and xyz.is_contiguous()):
        raise ValueError("positions must be a contiguous CUDA float64 tensor of shape (N, 3)")
    if w is not None and not (isinstance(w, torch.Tensor) and w.is_cuda and w.dtype == torch.float64
                              and w.dim() == 1 and w.shape[0] == xyz.shape[0] and w.is_contiguous()):
        raise ValueError("weights must be a contiguous CUDA float64 tensor of shape (N,)")
    return Catalog(xyz.data_ptr() if xyz.numel() else None, (w.data_ptr() if (w is not None and w.numel()) else None),
                   xyz.shape[0])


def _out_tensor(t, n, dtype, name):
    """Check a caller-provided device output: contiguous, on the GPU, of the right type and size."""
    import torch
    if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == dtype and t.is_contiguous()
            and t.numel() == n):
        raise ValueError(f"{name} must be a contiguous CUDA {dtype} tensor with {n} elements")
    return t


def weight_scale(wmin1, wmax1, wmin2=None, wmax2=None, nfactors=2):
    """Fixed-point scale exponent S of the exact weighted sums for weights whose
    smallest non-zero and largest magnitudes are given (fcfc_weight_scale);
    raises FcfcError (FCFC_ERANGE) for weights the exact sums cannot hold."""
    if wmin2 is None:
        wmin2, wmax2 = wmin1, wmax1
    S = ctypes.c_int32()
    check(load().fcfc_weight_scale(float(wmin1), float(wmax1), float(wmin2), float(wmax2), int(nfactors),
                                   ctypes.byref(S)))
    return S.value


def make_tuning(**kw):
    t = Tuning()
    for k, v in kw.items():
        if k == "order" and isinstance(v, str):
            v = ORDER[v]
        setattr(t, k, int(v))
    return t


class Plan:
    """Owns an fcfc_plan_t."""

    def __init__(self, kind, edges1, edges2=None, los="z", box=0.0, **tuning):
        lib = load()
        e1 = np.ascontiguousarray(np.asarray(edges1, dtype=np.float64))
        self.kind = kind
        self.n1 = len(e1) - 1
        if kind == "s":
            e2 = None
            self.n2 = 1
        else:
            e2 = np.ascontiguousarray(np.asarray(edges2, dtype=np.float64))
            self.n2 = len(e2) - 1
        self._e1, self._e2 = e1, e2
        self.tuning = make_tuning(**tuning)
        h = ctypes.c_void_p()
        check(lib.fcfc_plan_create(KIND[kind], LOS[los], e1.ctypes.data_as(_P), self.n1,
                                   e2.ctypes.data_as(_P) if e2 is not None else None,
                                   self.n2 if e2 is not None else 0, float(box), ctypes.byref(self.tuning),
                                   ctypes.byref(h)))
        self.h = h

    @classmethod
    def _wrap(cls, h, kind, e1, e2, tuning):
        """A Plan object owning an fcfc_plan_t made by another entry point."""
        self = cls.__new__(cls)
        self.kind = kind
        self._e1 = np.ascontiguousarray(e1, dtype=np.float64)
        self._e2 = None if e2 is None else np.ascontiguousarray(e2, dtype=np.float64)
        self.n1 = len(self._e1) - 1
        self.n2 = 1 if e2 is None else len(self._e2) - 1
        self.tuning = tuning
        self.h = h
        return self

    @property
    def shape(self):
        return (self.n1,) if self.kind == "s" else (self.n1, self.n2)

    def fit_bounds(self, catalogs, stream=None):
        arr = (Catalog * len(catalogs))(*[_catalog(x, w) for (x, w) in catalogs])
        check(load().fcfc_plan_fit_bounds(self.h, arr, len(catalogs), _stream_ptr(stream)))

    def set_bounds(self, lo, hi):
        lo = np.ascontiguousarray(np.asarray(lo, dtype=np.float64))
        hi = np.ascontiguousarray(np.asarray(hi, dtype=np.float64))
        check(load().fcfc_plan_set_bounds(self.h, lo.ctypes.data_as(_P), hi.ctypes.data_as(_P)))

    def build_cells(self, xyz, w=None, stream=None):
        return Cells(self, xyz, w, stream)

    def count(self, c1, c2=None, weighted=False, out=None, wout=None, stream=None):
        import torch
        nb = self.n1 * self.n2
        dev = c1.device
        if out is None:
            out = torch.empty(nb, dtype=torch.int64, device=dev)
        _out_tensor(out, nb, torch.int64, "out")
        if weighted and wout is None:
            wout = torch.empty(nb, dtype=torch.float64, device=dev)
        if weighted:
            _out_tensor(wout, nb, torch.float64, "wout")
        check(load().fcfc_count_pairs(self.h, c1.h, c2.h if c2 is not None else None, out.data_ptr(),
                                      wout.data_ptr() if weighted else None, _stream_ptr(stream)))
        return out.view(self.shape), (wout.view(self.shape) if weighted else None)

    def bin_squared(self, s2, out=None, stream=None):
        """Counts (int64, n1 bins of the first axis) of the squared separations s2
        (1-D CUDA float64 tensor): s2 in [edges[i]^2, edges[i+1]^2) counts in bin i."""
        import torch
        if not (isinstance(s2, torch.Tensor) and s2.is_cuda and s2.dtype == torch.float64 and s2.dim() == 1
                and s2.is_contiguous()):
            raise ValueError("s2 must be a contiguous 1-D CUDA float64 tensor")
        if out is None:
            out = torch.empty(self.n1, dtype=torch.int64, device=s2.device)
        _out_tensor(out, self.n1, torch.int64, "out")
        check(load().fcfc_bin_squared(self.h, s2.data_ptr(), int(s2.shape[0]), out.data_ptr(), _stream_ptr(stream)))
        return out

    def count_triplets(self, cells, weighted=False, out=None, wout=None, stream=None):
        """Triangle counts (int64 [n1, n1, n1], sorted side bins a <= b <= c) of a
        cell set, and the weighted counts (float64, or None)."""
        import torch
        nb = self.n1
        if out is None:
            out = torch.empty(nb ** 3, dtype=torch.int64, device=cells.device)
        _out_tensor(out, nb ** 3, torch.int64, "out")
        if weighted and wout is None:
            wout = torch.empty(nb ** 3, dtype=torch.float64, device=cells.device)
        if weighted:
            _out_tensor(wout, nb ** 3, torch.float64, "wout")
        check(load().fcfc_count_triplets(self.h, cells.h, out.data_ptr(), wout.data_ptr() if weighted else None,
                                         _stream_ptr(stream)))
        return out.view(nb, nb, nb), (wout.view(nb, nb, nb) if weighted else None)

    def stats(self):
        s = Stats()
        check(load().fcfc_plan_stats(self.h, ctypes.byref(s)))
        return s.as_dict()

    def numerics(self):
        """The FP32 constants a count of this plan uses (fcfc_plan_numerics), as a dict."""
        n = Numerics()
        check(load().fcfc_plan_numerics(self.h, ctypes.byref(n)))
        d = {k: getattr(n, k) for k, _ in Numerics._fields_ if k != "reserved"}
        d["lo"] = list(n.lo)
        return d

    def table(self, which):
        """Look-up table `which` (0: s or s_perp, 1: pi, 2 and 3: the same with twice
        the entries) as a dict of numpy arrays E (FP64), lo, hi (FP32), tab (int16)
        and the FP32 scale and vmax (fcfc_plan_table)."""
        lib = load()
        nt = _I64()
        check(lib.fcfc_plan_table(self.h, int(which), None, None, None, None, 0, ctypes.byref(nt), None, None))
        nb = self.n2 if which in (1, 3) else self.n1
        E = np.empty(nb + 1, dtype=np.float64)
        lo = np.empty(nb + 1, dtype=np.float32)
        hi = np.empty(nb + 1, dtype=np.float32)
        tab = np.empty(nt.value, dtype=np.int16)
        sc = ctypes.c_float()
        vm = ctypes.c_float()
        check(lib.fcfc_plan_table(self.h, int(which), E.ctypes.data, lo.ctypes.data, hi.ctypes.data, tab.ctypes.data,
                                  nt.value, ctypes.byref(nt), ctypes.byref(sc), ctypes.byref(vm)))
        return {"E": E, "lo": lo, "hi": hi, "tab": tab, "scale": np.float32(sc.value), "vmax": np.float32(vm.value)}

    def set_model(self, model):
        """Attach a Model for order="learned" (None detaches); the plan keeps a reference."""
        self._model = model
        check(load().fcfc_plan_set_model(self.h, model.h if model is not None else None))

    def timings(self, stream=None):
        """(features (n, 4), log2(1 + ticks) (n,)) float32 device tensors of the last
        count recorded with record_timing=1."""
        import torch
        lib = load()
        n = ctypes.c_int64()
        check(lib.fcfc_plan_timings(self.h, None, None, 0, ctypes.byref(n), _stream_ptr(stream)))
        feat = torch.empty((n.value, 4), dtype=torch.float32, device="cuda")
        logt = torch.empty(n.value, dtype=torch.float32, device="cuda")
        check(lib.fcfc_plan_timings(self.h, feat.data_ptr(), logt.data_ptr(), n.value, ctypes.byref(n),
                                    _stream_ptr(stream)))
        return feat, logt

    def predict(self, model, c1, c2=None, stream=None):
        """(predicted counting ms, work items) of count(c1, c2) under `model`."""
        ms = ctypes.c_double()
        n = ctypes.c_int64()
        check(load().fcfc_plan_predict(self.h, c1.h, c2.h if c2 is not None else None, model.h,
                                       _stream_ptr(stream), ctypes.byref(ms), ctypes.byref(n)))
        return ms.value, n.value

    def close(self):
        if getattr(self, "h", None):
            load().fcfc_plan_free(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Cells:
    """Owns an fcfc_cells_t built on a plan."""

    def __init__(self, plan, xyz, w=None, stream=None):
        cat = _catalog(xyz, w)
        h = ctypes.c_void_p()
        check(load().fcfc_build_cells(plan.h, ctypes.byref(cat), _stream_ptr(stream), ctypes.byref(h)))
        self.h = h
        self.device = xyz.device
        self.plan = plan

    def info(self):
        n = ctypes.c_int64()
        c = ctypes.c_int64()
        check(load().fcfc_cells_info(self.h, ctypes.byref(n), ctypes.byref(c)))
        return n.value, c.value

    def close(self):
        if getattr(self, "h", None):
            load().fcfc_cells_free(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """Owns an fcfc_batch_t: counts of many catalogues in one pipeline.

    catalogs: list of (xyz, w or None) device tensors.  pairs: None for the
    auto count of every catalogue, else a list of (a, b) catalogue indices,
    a == b for the auto count of a and a != b for the cross count of a with b;
    run() writes one histogram per pair, in the order given."""

    def __init__(self, plan, catalogs, pairs=None, stream=None):
        self._keep = catalogs
        arr = (Catalog * len(catalogs))(*[_catalog(x, w) for (x, w) in catalogs])
        h = ctypes.c_void_p()
        if pairs is None:
            check(load().fcfc_batch_create(plan.h, arr, len(catalogs), _stream_ptr(stream), ctypes.byref(h)))
            self.nhist = len(catalogs)
        else:
            pr = np.ascontiguousarray(np.asarray(pairs, dtype=np.int32).reshape(-1, 2))
            check(load().fcfc_batch_create_pairs(plan.h, arr, len(catalogs), pr.ctypes.data_as(_P), len(pr),
                                                 _stream_ptr(stream), ctypes.byref(h)))
            self.nhist = len(pr)
        self.h = h
        self.plan = plan
        self.ncat = len(catalogs)

    def run(self, out, wout=None, use_graph=True, stream=None):
        import torch
        nb = self.nhist * self.plan.n1 * self.plan.n2
        _out_tensor(out, nb, torch.int64, "out")
        if wout is not None:
            _out_tensor(wout, nb, torch.float64, "wout")
        check(load().fcfc_batch_run(self.h, out.data_ptr(), wout.data_ptr() if wout is not None else None,
                                    int(bool(use_graph)), _stream_ptr(stream)))
        return out

    def check(self, stream=None):
        """Wait, then return (work items, GPU ms of the last run); raises if the work list overflowed."""
        n = ctypes.c_uint32()
        ms = ctypes.c_float()
        check(load().fcfc_batch_check(self.h, _stream_ptr(stream), ctypes.byref(n), ctypes.byref(ms)))
        return n.value, ms.value

    def stats(self, stream=None):
        """Wait, then return the counting launch of the last run: candidates, rechecks and
        early LDS merges (flushes)."""
        v = (ctypes.c_int64 * 3)()
        check(load().fcfc_batch_stats(self.h, _stream_ptr(stream), v))
        return {"candidates": v[0], "rechecks": v[1], "flushes": v[2]}

    def close(self):
        if getattr(self, "h", None):
            load().fcfc_batch_free(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Model:
    """Owns an fcfc_model_t: the learned work-item cost model (4 -> 64 -> 64 -> 64 -> 1)."""

    def __init__(self, seed=0, path=None):
        h = ctypes.c_void_p()
        if path is not None:
            check(load().fcfc_model_load(os.fsencode(path), ctypes.byref(h)))
        else:
            check(load().fcfc_model_create(int(seed), ctypes.byref(h)))
        self.h = h

    @staticmethod
    def nparams():
        return int(load().fcfc_model_nparams())

    def get(self):
        p = np.empty(self.nparams(), dtype=np.float32)
        nrm = np.empty(10, dtype=np.float32)
        check(load().fcfc_model_get(self.h, p.ctypes.data_as(_P), nrm.ctypes.data_as(_P)))
        return p, nrm

    def set(self, params=None, norm=None):
        p = None if params is None else np.ascontiguousarray(params, dtype=np.float32)
        n = None if norm is None else np.ascontiguousarray(norm, dtype=np.float32)
        if p is not None and p.size != self.nparams():
            raise ValueError(f"params must have {self.nparams()} values")
        if n is not None and n.size != 10:
            raise ValueError("norm must have 10 values")
        check(load().fcfc_model_set(self.h, p.ctypes.data_as(_P) if p is not None else None,
                                    n.ctypes.data_as(_P) if n is not None else None))

    @staticmethod
    def _feat(x):
        import torch
        if not (isinstance(x, torch.Tensor) and x.is_cuda and x.dtype == torch.float32 and x.dim() == 2
                and x.shape[1] == 4 and x.is_contiguous()):
            raise ValueError("features must be a contiguous CUDA float32 tensor of shape (M, 4)")
        return x

    def predict(self, feat, stream=None):
        import torch
        feat = self._feat(feat)
        out = torch.empty(feat.shape[0], dtype=torch.float32, device=feat.device)
        check(load().fcfc_model_predict(self.h, feat.data_ptr(), feat.shape[0], out.data_ptr(), _stream_ptr(stream)))
        return out

    def _target(self, target, m):
        import torch
        return _out_tensor(target, m, torch.float32, "target")

    def grad(self, feat, target, stream=None):
        feat = self._feat(feat)
        target = self._target(target, feat.shape[0])
        g = np.empty(self.nparams(), dtype=np.float32)
        loss = ctypes.c_float()
        check(load().fcfc_model_grad(self.h, feat.data_ptr(), target.data_ptr(), feat.shape[0],
                                     g.ctypes.data_as(_P), ctypes.byref(loss), _stream_ptr(stream)))
        return g, loss.value

    def train(self, feat, target, epochs=30, batch=256, lr=1e-3, seed=0, stream=None):
        feat = self._feat(feat)
        target = self._target(target, feat.shape[0])
        loss = ctypes.c_float()
        check(load().fcfc_model_train(self.h, feat.data_ptr(), target.data_ptr(), feat.shape[0],
                                      int(epochs), int(batch), float(lr), int(seed), _stream_ptr(stream),
                                      ctypes.byref(loss)))
        return loss.value

    def save(self, path):
        check(load().fcfc_model_save(self.h, os.fsencode(path)))

    def close(self):
        if getattr(self, "h", None):
            load().fcfc_model_free(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def choose_cells(x1, x2=None, *, model=None, kind="s", edges1, edges2=None, los="z", box=0.0, stream=None,
                 **tuning):
    """(best cells per prune radius, predicted ms for k = 1..6) from the library's chooser."""
    e1 = np.ascontiguousarray(np.asarray(edges1, dtype=np.float64))
    e2 = None if kind == "s" else np.ascontiguousarray(np.asarray(edges2, dtype=np.float64))
    t = make_tuning(**tuning)
    c1 = _catalog(x1)
    c2 = _catalog(x2) if x2 is not None else None
    k = ctypes.c_int32()
    pred = (ctypes.c_double * 6)()
    check(load().fcfc_choose_cells(model.h if model is not None else None, KIND[kind], LOS[los],
                                   e1.ctypes.data_as(_P), len(e1) - 1,
                                   e2.ctypes.data_as(_P) if e2 is not None else None,
                                   len(e2) - 1 if e2 is not None else 0, float(box), ctypes.byref(t),
                                   ctypes.byref(c1), ctypes.byref(c2) if c2 is not None else None,
                                   _stream_ptr(stream), ctypes.byref(k), pred))
    return k.value, list(pred)


def diag_transcendental(stream=None):
    """(measured max relative error of rsq, of rcp, the bound the error bands assume)."""
    a, b, c = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
    check(load().fcfc_diag_transcendental(ctypes.byref(a), ctypes.byref(b), ctypes.byref(c), _stream_ptr(stream)))
    return a.value, b.value, c.value


def diag_peaks(stream=None):
    """Measured device rates: dict with fma_tflops, lds_u32_per_s, lds_u64_per_s, copy_gbps."""
    v = [ctypes.c_double() for _ in range(4)]
    check(load().fcfc_diag_peaks(*[ctypes.byref(x) for x in v], _stream_ptr(stream)))
    return dict(zip(("fma_tflops", "lds_u32_per_s", "lds_u64_per_s", "copy_gbps"), (x.value for x in v)))


def _f64_dev(t, name):
    import torch
    if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.float64 and t.is_contiguous()):
        raise ValueError(f"{name} must be a contiguous CUDA float64 tensor")
    return t


def xi(terms, coef, norm, den, stream=None):
    """Linear estimator: (sum_t coef_t X_t / norm_t) / (X_den / norm_den); terms are CUDA float64
    tensors of one shape (counts: .double())."""
    import torch
    terms = [_f64_dev(t, "term") for t in terms]
    n = terms[0].numel()
    if any(t.numel() != n for t in terms):
        raise ValueError("all terms need the same number of bins")
    out = torch.empty_like(terms[0])
    ptrs = (_P * len(terms))(*[t.data_ptr() for t in terms])
    c = (_D * len(terms))(*[float(v) for v in coef])
    nm = (_D * len(terms))(*[float(v) for v in norm])
    check(load().fcfc_xi(len(terms), ptrs, c, nm, int(den), n, out.data_ptr(), _stream_ptr(stream)))
    return out


def pair_norm(n1, n2=None):
    """Pairs behind a count: n1 (n1 - 1) / 2 (auto, n2 None) or n1 n2 (fcfc_pair_norm)."""
    out = _D()
    check(load().fcfc_pair_norm(int(n1), -1 if n2 is None else int(n2), ctypes.byref(out)))
    return out.value


def landy_szalay(dd, dr, rr, n_d, n_r, stream=None):
    """LS estimator (fcfc_landy_szalay) of auto counts DD, RR and the cross DR of
    n_d data and n_r random points; the result has DD's shape."""
    import torch
    t = [_f64_dev(x.double().contiguous(), name) for x, name in ((dd, "dd"), (dr, "dr"), (rr, "rr"))]
    n = t[0].numel()
    if any(x.numel() != n for x in t):
        raise ValueError("DD, DR and RR need the same number of bins")
    out = torch.empty(n, dtype=torch.float64, device=t[0].device)
    check(load().fcfc_landy_szalay(t[0].data_ptr(), t[1].data_ptr(), t[2].data_ptr(), int(n_d), int(n_r), n,
                                   out.data_ptr(), _stream_ptr(stream)))
    return out.view(dd.shape)


def analytic_rr(plan, npairs, stream=None):
    """Uniform periodic-box pair counts for the plan's bins (npairs = N (N - 1) / 2 for an auto count)."""
    import torch
    out = torch.empty(plan.n1 * plan.n2, dtype=torch.float64, device="cuda")
    check(load().fcfc_analytic_rr(plan.h, float(npairs), out.data_ptr(), _stream_ptr(stream)))
    return out.view(plan.shape)


def multipoles(xi_smu, mu_edges, ells=(0, 2, 4), stream=None):
    """Legendre multipoles of xi(s, mu) (shape (ns, nmu)): tensor (len(ells), ns)."""
    import torch
    x = _f64_dev(xi_smu, "xi")
    ns, nmu = x.shape
    mu = np.ascontiguousarray(np.asarray(mu_edges, dtype=np.float64))
    if mu.size != nmu + 1:
        raise ValueError("mu_edges needs nmu + 1 values")
    ls = np.ascontiguousarray(np.asarray(ells, dtype=np.int32))
    out = torch.empty((len(ls), ns), dtype=torch.float64, device=x.device)
    check(load().fcfc_multipoles(x.data_ptr(), ns, mu.ctypes.data_as(ctypes.POINTER(_D)), nmu,
                                 ls.ctypes.data_as(ctypes.POINTER(_I32)), len(ls), out.data_ptr(),
                                 _stream_ptr(stream)))
    return out


def wp(xi_spi, pi_edges, stream=None):
    """Projected correlation function of xi(s_perp, pi) (shape (nsp, npi))."""
    import torch
    x = _f64_dev(xi_spi, "xi")
    nsp, npi = x.shape
    pe = np.ascontiguousarray(np.asarray(pi_edges, dtype=np.float64))
    if pe.size != npi + 1:
        raise ValueError("pi_edges needs npi + 1 values")
    out = torch.empty(nsp, dtype=torch.float64, device=x.device)
    check(load().fcfc_wp(x.data_ptr(), nsp, pe.ctypes.data_as(ctypes.POINTER(_D)), npi, out.data_ptr(),
                         _stream_ptr(stream)))
    return out


TUNING_KEYS = ("cells_per_rmax", "tile_points", "seg_cells", "b_chunk", "hist_copies", "order",
               "record_timing", "n_hint", "lut_log2", "group_waves", "shard_count", "shard_index", "batch_chunk",
               "flush_log2", "tree_leaf")


def autotune(x1, x2=None, *, model=None, kind="s", edges1, edges2=None, los="z", box=0.0, w1=None, w2=None,
             cache=None, stream=None, **tuning):
    """Time candidate tunings on these catalogues (see fcfc_autotune).

    Returns (tuning dict, best ms, analytic-tuning ms, configurations timed)."""
    e1 = np.ascontiguousarray(np.asarray(edges1, dtype=np.float64))
    e2 = None if kind == "s" else np.ascontiguousarray(np.asarray(edges2, dtype=np.float64))
    t = make_tuning(**tuning)
    weighted = w1 is not None
    c1 = _catalog(x1, w1)
    c2 = _catalog(x2, w2) if x2 is not None else None
    best = Tuning()
    bms = ctypes.c_double()
    hms = ctypes.c_double()
    ntr = ctypes.c_int32()
    check(load().fcfc_autotune(model.h if model is not None else None, KIND[kind], LOS[los],
                               e1.ctypes.data_as(_P), len(e1) - 1,
                               e2.ctypes.data_as(_P) if e2 is not None else None,
                               len(e2) - 1 if e2 is not None else 0, float(box), ctypes.byref(t),
                               ctypes.byref(c1), ctypes.byref(c2) if c2 is not None else None, int(weighted),
                               os.fsencode(cache) if cache else None, _stream_ptr(stream), ctypes.byref(best),
                               ctypes.byref(bms), ctypes.byref(hms), ctypes.byref(ntr)))
    return {k: int(getattr(best, k)) for k in TUNING_KEYS}, bms.value, hms.value, ntr.value


def radec_to_unit(ra_deg, dec_deg, out=None, stream=None):
    """Unit vectors (N x 3 CUDA float64) of sky positions in degrees (CUDA float64 tensors)."""
    import torch
    for t, name in ((ra_deg, "ra"), (dec_deg, "dec")):
        if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.float64 and t.dim() == 1
                and t.is_contiguous()):
            raise ValueError(f"{name} must be a contiguous 1-D CUDA float64 tensor")
    if ra_deg.shape != dec_deg.shape:
        raise ValueError("ra and dec must have the same length")
    n = int(ra_deg.shape[0])
    if out is None:
        out = torch.empty((n, 3), dtype=torch.float64, device=ra_deg.device)
    _out_tensor(out, 3 * n, torch.float64, "out")
    check(load().fcfc_radec_to_unit(ra_deg.data_ptr(), dec_deg.data_ptr(), n, out.data_ptr(), _stream_ptr(stream)))
    return out


def angular_plan(theta_deg, **tuning):
    """Plan of angular bins (degrees) over unit vectors; returns (Plan, chord edges used)."""
    th = np.ascontiguousarray(np.asarray(theta_deg, dtype=np.float64))
    chord = np.empty(len(th), dtype=np.float64)
    t = make_tuning(**tuning)
    h = ctypes.c_void_p()
    check(load().fcfc_angular_plan(th.ctypes.data_as(ctypes.POINTER(_D)), len(th) - 1, ctypes.byref(t),
                                   chord.ctypes.data_as(ctypes.POINTER(_D)), ctypes.byref(h)))
    return Plan._wrap(h, "s", chord, None, t), chord


def angular_count(u1, u2=None, *, theta_deg, w1=None, w2=None, stream=None, **tuning):
    """Angular pair counts of unit vectors (CUDA float64 N x 3): auto when u2 is None.
    Returns (counts, wcounts or None, chord edges used)."""
    weighted = w1 is not None
    if "n_hint" not in tuning:
        tuning["n_hint"] = int(max(u1.shape[0], 0 if u2 is None else u2.shape[0]))
    plan, chord = angular_plan(theta_deg, **tuning)
    try:
        c1 = plan.build_cells(u1, w1 if weighted else None, stream)
        c2 = plan.build_cells(u2, w2 if weighted else None, stream) if u2 is not None else None
        counts, wcounts = plan.count(c1, c2, weighted=weighted, stream=stream)
        c1.close()
        if c2 is not None:
            c2.close()
    finally:
        plan.close()
    return counts, wcounts, chord


def bin_squared(s2, edges, *, stream=None, **tuning):
    """Histogram of squared separations s2 (1-D CUDA float64 tensor) in the
    separation bins `edges`: value v counts in bin i when edges[i]^2 <= v <
    edges[i+1]^2.  Returns (int64 counts, plan stats)."""
    e = np.asarray(edges, dtype=np.float64)
    plan = Plan("s", e, box=0.0, **tuning)
    try:
        out = plan.bin_squared(s2, stream=stream)
        st = plan.stats()
    finally:
        plan.close()
    return out, st


def count_triplets(x, *, edges, box=0.0, w=None, stream=None, return_stats=False, **tuning):
    """Triangle counts of a device catalogue (CUDA float64 N x 3): every set of
    three distinct points once when its sides lie in [edges[0], edges[-1]),
    binned by the sorted side bins into an int64 [n, n, n] tensor.  With
    weights w: returns (counts, weighted counts)."""
    if "n_hint" not in tuning:
        tuning["n_hint"] = int(x.shape[0])
    plan = Plan("s", edges, box=box, **tuning)
    try:
        if box == 0.0:
            plan.fit_bounds([(x, None)], stream)
        c = plan.build_cells(x, w, stream)
        counts, wcounts = plan.count_triplets(c, weighted=w is not None, stream=stream)
        st = plan.stats() if return_stats else None
        c.close()
    finally:
        plan.close()
    res = counts if w is None else (counts, wcounts)
    return (res, st) if return_stats else res


def count_pairs(x1, x2=None, *, kind="s", edges1, edges2=None, los="z", box=0.0, w1=None, w2=None,
                stream=None, return_stats=False, **tuning):
    """Pair counts of device catalogues (torch float64 CUDA tensors).

    x2=None: auto count of x1.  Weighted when w1 (and w2 for a cross count) are given.
    Returns (counts int64 tensor, wcounts float64 tensor or None[, stats dict]).
    """
    weighted = w1 is not None
    if "n_hint" not in tuning:
        tuning["n_hint"] = int(max(x1.shape[0], 0 if x2 is None else x2.shape[0]))
    plan = Plan(kind, edges1, edges2, los=los, box=box, **tuning)
    try:
        if box == 0.0:
            cats = [(x1, None)] + ([(x2, None)] if x2 is not None else [])
            plan.fit_bounds(cats, stream)
        c1 = plan.build_cells(x1, w1 if weighted else None, stream)
        c2 = plan.build_cells(x2, w2 if weighted else None, stream) if x2 is not None else None
        counts, wcounts = plan.count(c1, c2, weighted=weighted, stream=stream)
        st = plan.stats() if return_stats else None
        c1.close()
        if c2 is not None:
            c2.close()
    finally:
        plan.close()
    if return_stats:
        return counts, wcounts, st
    return counts, wcounts
