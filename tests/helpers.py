"""Shared helpers of the GPU tests: run a case through the HIP library and the oracle."""
import sys

import numpy as np

import oracle
from paper_2301_12557_amd import fcfc

WREL = 1e-12   # relative tolerance of weighted counts (exact accumulation gives 0)


def note(msg):
    print(f"[case] {msg}", flush=True)
    sys.stdout.flush()


def to_dev(a):
    import torch
    if a is None:
        return None
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def gpu_count(x1, x2=None, *, kind, edges1, edges2=None, los="z", box=0.0, w1=None, w2=None, **tuning):
    import torch
    c, wc, st = fcfc.count_pairs(to_dev(x1), to_dev(x2), kind=kind, edges1=edges1, edges2=edges2, los=los,
                                 box=box, w1=to_dev(w1), w2=to_dev(w2), return_stats=True, **tuning)
    torch.cuda.synchronize()
    return c.cpu().numpy(), (wc.cpu().numpy() if wc is not None else None), st


def oracle_count(x1, x2=None, *, kind, edges1, edges2=None, los="z", box=0.0, w1=None, w2=None,
                 method="brute", cell=None):
    return oracle.count(x1, x2, kind=kind, edges1=edges1, edges2=edges2, los=los, box=box, w1=w1,
                        w2=w2, method=method, cell=cell)


def assert_same(g, o, gw=None, ow=None, what=""):
    g = np.asarray(g)
    o = np.asarray(o)
    assert g.shape == o.shape, (g.shape, o.shape)
    if not np.array_equal(g, o):
        bad = np.argwhere(g != o)
        msg = [f"{what}: {len(bad)} bins differ; total gpu {g.sum()} oracle {o.sum()}"]
        for b in bad[:10]:
            b = tuple(b)
            msg.append(f"  bin {b}: gpu {g[b]} oracle {o[b]}")
        raise AssertionError("\n".join(msg))
    if ow is not None:
        assert gw is not None
        denom = np.maximum(np.abs(ow), 1e-300)
        rel = np.abs(gw - ow) / denom
        assert np.all(rel <= WREL), f"{what}: weighted rel err {rel.max()}"


def check_case(name, x1, x2=None, *, method="brute", cell=None, **kw):
    tuning = {k: kw.pop(k) for k in list(kw) if k in fcfc.TUNING_KEYS}
    note(f"{name}: n1={len(x1)} n2={None if x2 is None else len(x2)} kind={kw.get('kind')} "
         f"los={kw.get('los', 'z')} box={kw.get('box', 0.0)} w={kw.get('w1') is not None} tuning={tuning}")
    g, gw, st = gpu_count(x1, x2, **kw, **tuning)
    o, ow = oracle_count(x1, x2, method=method, cell=cell, **kw)
    assert_same(g, o, gw, ow, what=name)
    return g, gw, st
