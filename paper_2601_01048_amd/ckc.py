"""Python binding of libckc (include/ckc.h) over ctypes.

Argument marshalling only: every step of a check runs in the library's HIP
kernels.  Loading fails loudly when ``libckc.so`` has not been built; there is
no fallback path.  PyTorch is used (by ``run_workload``) only to place input
data in device memory.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "libckc.so")

OK, NOT_READY = 0, 1
FULL, REP_CORNERS, REP_BOUNDARY = 0, 1, 2
DENSE_MAP = 2
WAIT, DST_DEVICE = 1, 2
CLS = dict(AFFINE=1, GUARDED=2, INDIRECT=4, I64=8, UNIFORM=16, EXPANDED=32)

RECORD_DTYPE = np.dtype([("first_key", "<u8"), ("index", "<i8"), ("count", "<u8"),
                         ("kinds", "<u4"), ("first_kind", "<u4")])
STATUS_DTYPE = np.dtype([("lanes", "<u8"), ("accesses_checked", "<u8"), ("hang_lanes", "<u8"),
                         ("arith_faults", "<u8"), ("flags", "<u4"), ("pad", "<u4")])
ALLOC_DTYPE = np.dtype([("base", "<u8"), ("size_bytes", "<u8"), ("data", "<u8"),
                        ("flags", "<u4"), ("pad", "<u4")])


class ProgInfo(ctypes.Structure):
    _fields_ = [(n, ctypes.c_uint32) for n in
                ("n_accesses", "n_sites", "n_slots", "n_scalars", "max_loop_depth", "cls",
                 "n_instr_live", "n_regs_phys")]


class AccessInfo(ctypes.Structure):
    _fields_ = [(n, ctypes.c_uint32) for n in
                ("access_id", "slot", "log2_elem", "width", "affine", "guarded", "indirect",
                 "loop_depth")] + [("coef", ctypes.c_uint64 * 7)]


class Batch(ctypes.Structure):
    _fields_ = [("prog_id", ctypes.c_uint32), ("n_inputs", ctypes.c_uint32),
                ("launch", ctypes.c_void_p), ("scalars", ctypes.c_void_p),
                ("table_ids", ctypes.c_void_p), ("mode", ctypes.c_uint32),
                ("flags", ctypes.c_uint32), ("loop_cap_log2", ctypes.c_uint32 * 2)]


class LaunchOpts(ctypes.Structure):
    _fields_ = [("tile", ctypes.c_uint32), ("wg_size", ctypes.c_uint32), ("n_wg", ctypes.c_uint32),
                ("force_generic", ctypes.c_uint32), ("hip_stream", ctypes.c_void_p)]


class CkcError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"ckc error {code}: {msg}")
        self.code = code


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            raise RuntimeError(f"{LIB} is missing: build it with python -m paper_2601_01048_amd.build")
        L = ctypes.CDLL(LIB)
        vp, u32, u64, sz = ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_size_t
        L.ckc_last_error.restype = ctypes.c_char_p
        L.ckc_init.argtypes = [ctypes.c_int, ctypes.POINTER(vp)]
        L.ckc_shutdown.argtypes = [vp]
        L.ckc_shutdown.restype = None
        L.ckc_analyze_ir.argtypes = [vp, sz, vp, vp, u32]
        L.ckc_load_program.argtypes = [vp, vp, sz, ctypes.POINTER(u32), vp]
        L.ckc_unload_program.argtypes = [vp, u32]
        L.ckc_put_alloc_table.argtypes = [vp, vp, u32, ctypes.POINTER(u32)]
        L.ckc_free_alloc_table.argtypes = [vp, u32]
        L.ckc_check_batch.argtypes = [vp, vp, u32, vp, ctypes.POINTER(u64)]
        L.ckc_read_results.argtypes = [vp, u64, vp, vp, vp, u32]
        L.ckc_job_sizes.argtypes = [vp, u64, ctypes.POINTER(u64), ctypes.POINTER(u64)]
        L.ckc_job_timing.argtypes = [vp, u64, vp]
        for f in ("ckc_init", "ckc_analyze_ir", "ckc_load_program", "ckc_unload_program",
                  "ckc_put_alloc_table", "ckc_free_alloc_table", "ckc_check_batch",
                  "ckc_read_results", "ckc_job_sizes", "ckc_job_timing"):
            getattr(L, f).restype = ctypes.c_int
        _lib = L
    return _lib


def _check(rc):
    if rc < 0:
        raise CkcError(rc, lib().ckc_last_error().decode())
    return rc


def _p(a: np.ndarray):
    return a.ctypes.data if a is not None and a.size else None


def analyze(ir: bytes):
    """Host-only analysis: (info dict, list of per-access dicts)."""
    info = ProgInfo()
    buf = ctypes.create_string_buffer(ir, len(ir))
    _check(lib().ckc_analyze_ir(buf, len(ir), ctypes.byref(info), None, 0))
    accs = (AccessInfo * max(1, info.n_accesses))()
    _check(lib().ckc_analyze_ir(buf, len(ir), None, accs, info.n_accesses))
    out = []
    for a in accs[: info.n_accesses]:
        d = {f: getattr(a, f) for f, _ in AccessInfo._fields_ if f != "coef"}
        d["coef"] = [(int(c) >> 32, int(c) & 0xFFFFFFFF) for c in a.coef]
        out.append(d)
    return {f: getattr(info, f) for f, _ in ProgInfo._fields_}, out


class Context:
    """One library context on one HIP device."""

    def __init__(self, device: int = 0):
        h = ctypes.c_void_p()
        _check(lib().ckc_init(device, ctypes.byref(h)))
        self.h = h

    def close(self):
        if self.h:
            lib().ckc_shutdown(self.h)
            self.h = None

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def load_program(self, ir: bytes):
        pid = ctypes.c_uint32()
        info = ProgInfo()
        buf = ctypes.create_string_buffer(ir, len(ir))
        _check(lib().ckc_load_program(self.h, buf, len(ir), ctypes.byref(pid), ctypes.byref(info)))
        return pid.value, {f: getattr(info, f) for f, _ in ProgInfo._fields_}

    def unload_program(self, pid: int):
        _check(lib().ckc_unload_program(self.h, pid))

    def put_table(self, entries: np.ndarray) -> int:
        """entries: ALLOC_DTYPE array whose ``data`` fields are device addresses."""
        e = np.ascontiguousarray(entries, ALLOC_DTYPE)
        tid = ctypes.c_uint32()
        _check(lib().ckc_put_alloc_table(self.h, _p(e), len(e), ctypes.byref(tid)))
        return tid.value

    def free_table(self, tid: int):
        _check(lib().ckc_free_alloc_table(self.h, tid))

    def check(self, descs, force_generic=False, n_wg=0, stream=None) -> int:
        """descs: list of dict(prog, launch [n,6], scalars [n,k], table_ids [n],
        mode, flags, cap_log2)."""
        keep = []
        arr = (Batch * len(descs))()
        for b, d in zip(arr, descs):
            launch = np.ascontiguousarray(d["launch"], np.uint32)
            sc = np.ascontiguousarray(d.get("scalars", np.zeros((len(launch), 0))), np.int64)
            tids = np.ascontiguousarray(d["table_ids"], np.uint32)
            keep += [launch, sc, tids]
            b.prog_id = d["prog"]
            b.n_inputs = len(launch)
            b.launch, b.scalars, b.table_ids = _p(launch), _p(sc), _p(tids)
            b.mode = d.get("mode", FULL)
            b.flags = d.get("flags", 0)
            cap = d.get("cap_log2", (20, 12))
            b.loop_cap_log2[0], b.loop_cap_log2[1] = cap
        opts = LaunchOpts(0, 0, n_wg, 1 if force_generic else 0, stream)
        job = ctypes.c_uint64()
        _check(lib().ckc_check_batch(self.h, arr, len(descs), ctypes.byref(opts), ctypes.byref(job)))
        return job.value

    def sizes(self, job: int):
        ni, nr = ctypes.c_uint64(), ctypes.c_uint64()
        _check(lib().ckc_job_sizes(self.h, job, ctypes.byref(ni), ctypes.byref(nr)))
        return ni.value, nr.value

    def timing(self, job: int):
        ms = (ctypes.c_float * 4)()
        _check(lib().ckc_job_timing(self.h, job, ms))
        return list(ms)

    def read(self, job: int, maps: bool = True, wait: bool = True):
        """Host copies of (records [inputs*accesses], maps [inputs, 65536], status)."""
        ni, nr = self.sizes(job)
        recs = np.zeros(nr, RECORD_DTYPE)
        mp = np.zeros((ni, 65536), np.uint8) if maps else None
        st = np.zeros(ni, STATUS_DTYPE)
        rc = _check(lib().ckc_read_results(self.h, job, _p(recs), _p(mp) if maps else None, _p(st),
                                           WAIT if wait else 0))
        if rc == NOT_READY:
            return None
        return recs, mp, st

    def read_device(self, job: int, recs_ptr: int, maps_ptr: int | None, st_ptr: int | None):
        _check(lib().ckc_read_results(self.h, job, recs_ptr, maps_ptr, st_ptr, WAIT | DST_DEVICE))


class DeviceWorkload:
    """A workload's data arrays, allocation tables and program placed on the
    device once (kept resident across checks)."""

    def __init__(self, ctx: Context, wl, device: str = "cuda"):
        import torch
        self.ctx, self.wl = ctx, wl
        self.tensors = [torch.from_numpy(np.ascontiguousarray(d)).to(device) for d in wl.data]
        self.prog, self.info = ctx.load_program(wl.ir)
        self.table_ids = []
        for t in wl.tables:
            e = np.array(t, ALLOC_DTYPE)
            refs = e["data"].astype(np.int64)
            e["data"] = [self.tensors[r - 1].data_ptr() if r else 0 for r in refs]
            self.table_ids.append(ctx.put_table(e))
        self.table_ids = np.array(self.table_ids, np.uint32)

    def desc(self, mode=None, dense=True, cap_log2=None, idx=None):
        wl = self.wl
        sel = slice(None) if idx is None else idx
        return dict(prog=self.prog, launch=wl.launch[sel], scalars=wl.scalars[sel],
                    table_ids=self.table_ids[wl.table_idx[sel]],
                    mode=wl.mode if mode is None else mode, flags=DENSE_MAP if dense else 0,
                    cap_log2=wl.cap_log2 if cap_log2 is None else cap_log2)

    def close(self):
        for t in self.table_ids:
            self.ctx.free_table(int(t))
        self.ctx.unload_program(self.prog)
        self.tensors = []


def run_workload(ctx: Context, wl, mode=None, force_generic=False, maps=True, cap_log2=None):
    """Check every input of a workload; returns the oracle-shaped result dict
    (records [n, n_acc], maps [n, 65536] or None, status [n])."""
    dw = DeviceWorkload(ctx, wl)
    try:
        job = ctx.check([dw.desc(mode, maps, cap_log2)], force_generic=force_generic)
        recs, mp, st = ctx.read(job, maps=maps)
    finally:
        dw.close()
    n = wl.n_inputs
    return dict(records=recs.reshape(n, -1), maps=mp, status=st, info=dw.info)
