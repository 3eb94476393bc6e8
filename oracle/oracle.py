"""ctypes wrapper of the reference checker in ``ckc_oracle.c``.

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the benchmark's
CPU-baseline leg call this; the library never does.  The C file is compiled
with gcc into ``oracle/libckc_oracle.so`` on first use (or by ``build()``).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "ckc_oracle.c")
LIB = os.path.join(HERE, "libckc_oracle.so")

RECORD_DTYPE = np.dtype([("first_key", "<u8"), ("index", "<i8"), ("count", "<u8"),
                         ("kinds", "<u4"), ("first_kind", "<u4")])
STATUS_DTYPE = np.dtype([("lanes", "<u8"), ("accesses_checked", "<u8"), ("hang_lanes", "<u8"),
                         ("arith_faults", "<u8"), ("flags", "<u4"), ("pad", "<u4")])
KIND_OVER, KIND_UNDER, KIND_FREED, KIND_NULL = 1, 2, 4, 8

_lock = threading.Lock()
_lib = None


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (plain -O2, no tuning)."""
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        tmp = LIB + f".tmp{os.getpid()}"
        subprocess.check_call(["gcc", "-O2", "-std=gnu11", "-Wall", "-shared", "-fPIC", "-pthread",
                               SRC, "-o", tmp, "-lm"])
        os.replace(tmp, LIB)
    return LIB


def _load():
    global _lib
    with _lock:
        if _lib is None:
            build()
            lib = ctypes.CDLL(LIB)
            p = ctypes.c_void_p
            lib.ckco_check.argtypes = [p, ctypes.c_size_t, ctypes.c_uint32, p, p, p, p, p,
                                       ctypes.c_uint32, ctypes.c_uint32, p, p, p, p, p, ctypes.c_int, p]
            lib.ckco_check.restype = ctypes.c_int
            lib.ckco_validate.argtypes = [p, ctypes.c_size_t, p]
            lib.ckco_validate.restype = ctypes.c_int
            lib.ckco_fuzz.argtypes = [p, ctypes.c_size_t, p, p, p, ctypes.c_uint32, ctypes.c_uint32,
                                      ctypes.c_uint32, p, p, p, p, p, p, p, p, p, p, ctypes.c_int]
            lib.ckco_fuzz.restype = ctypes.c_int
            lib.ckco_fuzz_rand.argtypes = [ctypes.c_uint64, ctypes.c_uint64]
            lib.ckco_fuzz_rand.restype = ctypes.c_uint64
            lib.ckco_ir_exp.argtypes = [ctypes.c_double]
            lib.ckco_ir_exp.restype = ctypes.c_double
            lib.ckco_fuzz_class.argtypes = [ctypes.c_uint32]
            lib.ckco_fuzz_class.restype = ctypes.c_uint32
            _lib = lib
    return _lib


class OracleError(RuntimeError):
    def __init__(self, code):
        super().__init__(f"oracle returned {code}")
        self.code = code


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p) if a.size else None


def validate(ir: bytes):
    """Decode-only check: returns (n_accesses, n_sites, max_depth, n_slots) or raises."""
    lib = _load()
    out = np.zeros(4, np.int32)
    buf = ctypes.create_string_buffer(ir, len(ir))
    rc = lib.ckco_validate(buf, len(ir), _ptr(out))
    if rc:
        raise OracleError(rc)
    return tuple(int(v) for v in out)


def check(wl, mode: int | None = None, cap_log2=None, nthreads: int = 1, maps: bool = True,
          detector: int | None = None, executed: bool = False):
    """Run the oracle over every input of workload ``wl`` (``detector``: 0
    exact bounds, 1 the tripwire model; default the workload's).

    Returns dict(records [n, n_acc] RECORD_DTYPE, counts [n, n_sites] uint64,
    maps [n, 65536] uint8 or None, status [n] STATUS_DTYPE)."""
    lib = _load()
    n_acc, n_sites, _, n_slots = validate(wl.ir)
    n = wl.n_inputs
    mode = wl.mode if mode is None else mode
    detector = getattr(wl, "detector", 0) if detector is None else detector
    cap = np.asarray(wl.cap_log2 if cap_log2 is None else cap_log2, np.uint32)
    launch = np.ascontiguousarray(wl.launch, np.uint32)
    scalars = np.ascontiguousarray(wl.scalars, np.int64)
    # per-input tables with host addresses of the data arrays
    data = [np.ascontiguousarray(d) for d in wl.data]
    tabs = wl.tables.copy()
    refs = tabs["data"].astype(np.int64)
    addr = np.zeros_like(tabs["data"])
    for k, d in enumerate(data):
        addr[refs == k + 1] = d.ctypes.data
    tabs["data"] = addr
    n_tab_slots = tabs.shape[1]
    flat = np.ascontiguousarray(tabs.reshape(-1))
    table_off = (np.asarray(wl.table_idx, np.uint64) * np.uint64(n_tab_slots)).astype(np.uint64)
    table_len = np.full(n, n_tab_slots, np.uint32)
    recs = np.zeros((n, n_acc), RECORD_DTYPE)
    counts = np.zeros((n, n_sites), np.uint64)
    mp = np.zeros((n, 65536), np.uint8) if maps else None
    st = np.zeros(n, STATUS_DTYPE)
    ex = np.zeros((n, 2), np.uint64) if executed else None
    buf = ctypes.create_string_buffer(wl.ir, len(wl.ir))
    rc = lib.ckco_check(buf, len(wl.ir), n, _ptr(launch), _ptr(scalars), _ptr(flat),
                        _ptr(table_off), _ptr(table_len), int(mode), int(detector), _ptr(cap),
                        _ptr(recs), _ptr(counts), _ptr(mp) if maps else None, _ptr(st),
                        int(nthreads), _ptr(ex) if executed else None)
    if rc:
        raise OracleError(rc)
    del data
    out = dict(records=recs, counts=counts, maps=mp, status=st)
    if executed:
        out["executed"] = ex  # [n, 2]: instruction executions of the program as written / as pruned
    return out


MUT_LAUNCH, MUT_SCALAR, MUT_DATA = 1, 2, 4
NO_SLOT = 0xFFFFFFFF


def fuzz_rand(seed: int, k: int) -> int:
    """Output k of the campaign's SplitMix64 generator started at ``seed``."""
    return int(_load().ckco_fuzz_rand(seed, k))


def ir_exp(x: float) -> float:
    """e^x by the IR's fixed method (the FEXP operation)."""
    return float(_load().ckco_ir_exp(x))


def fuzz_class(v: int) -> int:
    """The hit-count class the campaign gives a map byte."""
    return int(_load().ckco_fuzz_class(v))


def fuzz(wl, generations: int, batch: int, max_stack: int = 4, max_threads: int = 1 << 20,
         max_block: int = 1024, corpus_cap: int = 256, data_slot: int = NO_SLOT,
         ops: int = MUT_LAUNCH | MUT_SCALAR, seed: int = 0, nthreads: int = 1, mode: int | None = None,
         detector: int | None = None):
    """A fuzzing campaign from input 0 of workload ``wl`` (its launch,
    scalars and table; data slots resolved to host arrays).  Returns dict(
    launch [size, 6], scalars [size, 16], data [size, n_elems] or None, gen
    [size], virgin [65536], sigs [n_accesses, 4], stats dict)."""
    lib = _load()
    n_acc, _, _, _ = validate(wl.ir)
    mode = wl.mode if mode is None else mode
    detector = getattr(wl, "detector", 0) if detector is None else detector
    cap = np.asarray(wl.cap_log2, np.uint32)
    data = [np.ascontiguousarray(d) for d in wl.data]
    tab = np.array(wl.tables[wl.table_idx[0]], copy=True)
    refs = tab["data"].astype(np.int64)
    addr = np.zeros_like(tab["data"])
    for k, d in enumerate(data):
        addr[refs == k + 1] = d.ctypes.data
    tab["data"] = addr
    tab = np.ascontiguousarray(tab)
    launch = np.ascontiguousarray(wl.launch[0], np.uint32)
    sc = np.zeros(16, np.int64)
    sc[: wl.scalars.shape[1]] = wl.scalars[0]
    n_elems = int(tab[data_slot]["size_bytes"]) // 4 if data_slot < len(tab) else 0
    cfg = np.array([batch, max_stack, max_threads, max_block, corpus_cap, data_slot, ops, seed, generations],
                   np.uint64)
    c_launch = np.zeros((corpus_cap, 6), np.uint32)
    c_scalars = np.zeros((corpus_cap, 16), np.int64)
    c_data = np.zeros((corpus_cap, max(1, n_elems)), np.int32)
    c_gen = np.zeros(corpus_cap, np.uint32)
    c_size = np.zeros(1, np.uint32)
    virgin = np.zeros(65536, np.uint8)
    sigs = np.zeros((max(1, n_acc), 4), np.uint64)
    stats = np.zeros(4, np.uint64)
    buf = ctypes.create_string_buffer(wl.ir, len(wl.ir))
    rc = lib.ckco_fuzz(buf, len(wl.ir), _ptr(launch), _ptr(sc), _ptr(tab), len(tab), int(mode), int(detector),
                       _ptr(cap), _ptr(cfg), _ptr(c_launch), _ptr(c_scalars), _ptr(c_data), _ptr(c_gen),
                       _ptr(c_size), _ptr(virgin), _ptr(sigs), _ptr(stats), int(nthreads))
    if rc:
        raise OracleError(rc)
    n = int(c_size[0])
    del data
    return dict(launch=c_launch[:n], scalars=c_scalars[:n], data=c_data[:n] if n_elems else None,
                gen=c_gen[:n], virgin=virgin, sigs=sigs[:n_acc],
                stats=dict(execs=int(stats[0]), novel=int(stats[1]), crashes=int(stats[2]),
                           generations=int(stats[3])))
