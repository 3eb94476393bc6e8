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
                               SRC, "-o", tmp])
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
                                       ctypes.c_uint32, ctypes.c_uint32, p, p, p, p, p, ctypes.c_int]
            lib.ckco_check.restype = ctypes.c_int
            lib.ckco_validate.argtypes = [p, ctypes.c_size_t, p]
            lib.ckco_validate.restype = ctypes.c_int
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
          detector: int | None = None):
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
    buf = ctypes.create_string_buffer(wl.ir, len(wl.ir))
    rc = lib.ckco_check(buf, len(wl.ir), n, _ptr(launch), _ptr(scalars), _ptr(flat),
                        _ptr(table_off), _ptr(table_len), int(mode), int(detector), _ptr(cap),
                        _ptr(recs), _ptr(counts), _ptr(mp) if maps else None, _ptr(st),
                        int(nthreads))
    if rc:
        raise OracleError(rc)
    del data
    return dict(records=recs, counts=counts, maps=mp, status=st)
