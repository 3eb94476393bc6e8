"""Helpers for mixed batches in the tests: the oracle run over many one-input
workloads (grouped by program into one oracle call each), and flattening of
per-kernel results into the layout of one library job."""
import numpy as np

from oracle import oracle as O
from paper_2601_01048_amd.gen import workloads as W


def group(kernels):
    """One multi-input Workload holding one-input workloads that share a program
    (tables stacked; data lists concatenated with their references shifted)."""
    ir = kernels[0].ir
    launch = np.concatenate([k.launch for k in kernels])
    scalars = np.concatenate([k.scalars for k in kernels])
    tabs, data = [], []
    for k in kernels:
        t = np.array(k.tables[0], W.ALLOC_DTYPE)
        refs = t["data"].astype(np.int64)
        t["data"] = np.where(refs > 0, refs + len(data), 0).astype(np.uint64)
        tabs.append(t)
        data.extend(k.data)
    tables = np.stack(tabs)
    return W.Workload("group", ir, launch, scalars, tables, np.arange(len(kernels), dtype=np.uint32), data,
                      kernels[0].mode, kernels[0].cap_log2)


def oracle_mixed(mb, idx=None, nthreads=1, maps=True):
    """Oracle results of kernels ``idx`` (default all) of mixed batch ``mb``:
    list of dict(records [n_acc], maps [65536] or None, status)."""
    idx = list(range(mb.n_kernels)) if idx is None else list(idx)
    by_ir = {}
    for i in idx:
        by_ir.setdefault(mb.kernels[i].ir, []).append(i)
    out = {}
    for ir, members in by_ir.items():
        res = O.check(group([mb.kernels[i] for i in members]), nthreads=nthreads, maps=maps)
        for j, i in enumerate(members):
            out[i] = dict(records=res["records"][j], maps=None if res["maps"] is None else res["maps"][j],
                          status=res["status"][j])
    return [out[i] for i in idx]


def same(a, b, what, maps=True):
    """Byte equality of two per-kernel result dicts (records, maps, status)."""
    for f in ("first_key", "count", "kinds", "index", "first_kind"):
        assert np.array_equal(a["records"][f], b["records"][f]), (what, f, a["records"], b["records"])
    for f in ("lanes", "accesses_checked", "hang_lanes", "arith_faults"):
        assert a["status"][f] == b["status"][f], (what, f, a["status"], b["status"])
    if maps:
        assert np.array_equal(a["maps"], b["maps"]), (what, "maps")
