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
FULL, REP_CORNERS, REP_BOUNDARY, REP_PREX, FULL_ENDPOINTS = 0, 1, 2, 3, 4
ST_VERTEX_EXACT = 1
SCHED_DEFAULT, SCHED_BLOCKED, SCHED_CYCLIC, SCHED_DYNAMIC, SCHED_LPT = 0, 1, 2, 3, 4
SCHED_NAMES = {0: "default", 1: "blocked", 2: "cyclic", 3: "dynamic", 4: "lpt"}
DENSE_MAP = 2
LOAD_NO_PRUNE = 1
TRIPWIRE = 4
SPACE_GLOBAL, SPACE_SHARED, SPACE_LOCAL = 0, 1, 2
WAIT, DST_DEVICE, ENQUEUE = 1, 2, 4
CLS = dict(AFFINE=1, GUARDED=2, INDIRECT=4, I64=8, UNIFORM=16, EXPANDED=32, GATHER=64, BARRIER=128)

RECORD_DTYPE = np.dtype([("first_key", "<u8"), ("index", "<i8"), ("count", "<u8"),
                         ("kinds", "<u4"), ("first_kind", "<u4")])
STATUS_DTYPE = np.dtype([("lanes", "<u8"), ("accesses_checked", "<u8"), ("hang_lanes", "<u8"),
                         ("arith_faults", "<u8"), ("flags", "<u4"), ("pad", "<u4")])
ALLOC_DTYPE = np.dtype([("base", "<u8"), ("size_bytes", "<u8"), ("data", "<u8"),
                        ("flags", "<u4"), ("redzone", "<u4")])


class ProgInfo(ctypes.Structure):
    _fields_ = [(n, ctypes.c_uint32) for n in
                ("n_accesses", "n_sites", "n_slots", "n_scalars", "max_loop_depth", "cls",
                 "n_instr_live", "n_regs_phys", "rows_form")]


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
    _fields_ = [("schedule", ctypes.c_uint32), ("chunk", ctypes.c_uint32), ("wg_per_cu", ctypes.c_uint32),
                ("force_generic", ctypes.c_uint32), ("use_graph", ctypes.c_uint32), ("pad", ctypes.c_uint32),
                ("hip_stream", ctypes.c_void_p)]

    def as_dict(self):
        return dict(schedule=SCHED_NAMES.get(self.schedule, self.schedule), chunk=self.chunk,
                    wg_per_cu=self.wg_per_cu, use_graph=self.use_graph)


class TuneEntry(ctypes.Structure):
    _fields_ = [("opts", LaunchOpts), ("ms", ctypes.c_float), ("pad", ctypes.c_uint32)]


class ServerConfig(ctypes.Structure):
    _fields_ = [("n_streams", ctypes.c_uint32), ("max_batch_jobs", ctypes.c_uint32),
                ("hbm_cap_bytes", ctypes.c_uint64), ("opts", LaunchOpts)]


class JobStats(ctypes.Structure):
    _fields_ = [("t_arrival_ns", ctypes.c_uint64), ("t_admit_ns", ctypes.c_uint64),
                ("t_done_ns", ctypes.c_uint64), ("ws_bytes", ctypes.c_uint64),
                ("batch_jobs", ctypes.c_uint32), ("status", ctypes.c_int32)]


class ServerStats(ctypes.Structure):
    _fields_ = [(n, ctypes.c_uint64) for n in ("submitted", "completed", "rejected", "batches",
                                                "max_inflight_bytes", "max_inflight_jobs")]


MUT_LAUNCH, MUT_SCALAR, MUT_DATA = 1, 2, 4
FUZZ_NO_SLOT = 0xFFFFFFFF


class FuzzConfig(ctypes.Structure):
    _fields_ = [("prog_id", ctypes.c_uint32), ("table_id", ctypes.c_uint32), ("launch", ctypes.c_uint32 * 6),
                ("scalars", ctypes.c_int64 * 16), ("mode", ctypes.c_uint32), ("flags", ctypes.c_uint32),
                ("loop_cap_log2", ctypes.c_uint32 * 2), ("batch", ctypes.c_uint32), ("max_stack", ctypes.c_uint32),
                ("max_block", ctypes.c_uint32), ("corpus_cap", ctypes.c_uint32), ("max_threads", ctypes.c_uint64),
                ("data_slot", ctypes.c_uint32), ("ops", ctypes.c_uint32), ("seed", ctypes.c_uint64)]


class FuzzStats(ctypes.Structure):
    _fields_ = [(n, ctypes.c_uint64) for n in ("generations", "execs", "novel", "crashes", "corpus", "map_bits")]


def launch_opts(schedule=0, chunk=0, wg_per_cu=0, force_generic=False, use_graph=False, stream=None):
    return LaunchOpts(schedule, chunk, wg_per_cu, 1 if force_generic else 0, 1 if use_graph else 0, 0, stream)


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
        L.ckc_load_program_ex.argtypes = [vp, vp, sz, u32, ctypes.POINTER(u32), vp]
        L.ckc_unload_program.argtypes = [vp, u32]
        L.ckc_put_alloc_table.argtypes = [vp, vp, u32, ctypes.POINTER(u32)]
        L.ckc_free_alloc_table.argtypes = [vp, u32]
        L.ckc_check_batch.argtypes = [vp, vp, u32, vp, ctypes.POINTER(u64)]
        L.ckc_check_batch_noalloc.argtypes = [vp, vp, u32, vp, vp, vp, vp]
        L.ckc_read_results.argtypes = [vp, u64, vp, vp, vp, u32]
        L.ckc_job_sizes.argtypes = [vp, u64, ctypes.POINTER(u64), ctypes.POINTER(u64)]
        L.ckc_job_timing.argtypes = [vp, u64, vp]
        L.ckc_job_elapsed.argtypes = [vp, u64, ctypes.POINTER(ctypes.c_float)]
        L.ckc_autotune.argtypes = [vp, vp, u32, vp, u32, vp, vp, u32, ctypes.POINTER(u32)]
        L.ckc_server_create.argtypes = [vp, vp, ctypes.POINTER(vp)]
        L.ckc_server_destroy.argtypes = [vp]
        L.ckc_server_destroy.restype = None
        L.ckc_server_submit.argtypes = [vp, vp, u64, ctypes.POINTER(u64)]
        L.ckc_server_result.argtypes = [vp, u64, vp, vp, vp, vp, u32]
        L.ckc_server_get_stats.argtypes = [vp, vp]
        L.ckc_fuzz_create.argtypes = [vp, vp, ctypes.POINTER(vp)]
        L.ckc_fuzz_run.argtypes = [vp, u32]
        L.ckc_fuzz_get_stats.argtypes = [vp, vp]
        L.ckc_fuzz_read.argtypes = [vp, vp, vp, vp, vp, vp, vp]
        L.ckc_fuzz_destroy.argtypes = [vp]
        L.ckc_fuzz_destroy.restype = None
        for f in ("ckc_init", "ckc_analyze_ir", "ckc_load_program", "ckc_load_program_ex", "ckc_unload_program",
                  "ckc_put_alloc_table", "ckc_free_alloc_table", "ckc_check_batch", "ckc_check_batch_noalloc",
                  "ckc_read_results", "ckc_job_sizes", "ckc_job_timing", "ckc_job_elapsed",
                  "ckc_autotune", "ckc_server_create", "ckc_server_submit", "ckc_server_result",
                  "ckc_server_get_stats", "ckc_fuzz_create", "ckc_fuzz_run", "ckc_fuzz_get_stats",
                  "ckc_fuzz_read"):
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

    def load_program(self, ir: bytes, no_prune: bool = False):
        """(program id, info dict); ``no_prune`` keeps every instruction (the
        unpruned baseline of the pruning measurement)."""
        pid = ctypes.c_uint32()
        info = ProgInfo()
        buf = ctypes.create_string_buffer(ir, len(ir))
        _check(lib().ckc_load_program_ex(self.h, buf, len(ir), LOAD_NO_PRUNE if no_prune else 0,
                                         ctypes.byref(pid), ctypes.byref(info)))
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

    @staticmethod
    def prepare(descs):
        """ctypes descriptor array for ``descs`` (list of dict(prog, launch [n,6],
        scalars [n,k], table_ids [n], mode, flags, cap_log2)); reusable."""
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
        return (arr, keep)

    def check(self, descs, force_generic=False, stream=None, opts: LaunchOpts | None = None) -> int:
        """Queues one job over ``descs`` (a list of descriptor dicts or the
        result of ``prepare``); returns the job id."""
        arr, keep = descs if isinstance(descs, tuple) else self.prepare(descs)
        if opts is None:
            opts = launch_opts(force_generic=force_generic, stream=stream)
        job = ctypes.c_uint64()
        _check(lib().ckc_check_batch(self.h, arr, len(arr), ctypes.byref(opts), ctypes.byref(job)))
        del keep
        return job.value

    def check_noalloc(self, descs, recs_ptr: int, maps_ptr: int | None, st_ptr: int,
                      opts: LaunchOpts | None = None):
        """ckc_check_batch_noalloc: queues the check of ``descs`` with results
        written to the given device buffers; allocates nothing.  The results
        are valid once the context's stream (or the device) is synchronized."""
        arr, keep = descs if isinstance(descs, tuple) else self.prepare(descs)
        _check(lib().ckc_check_batch_noalloc(self.h, arr, len(arr), ctypes.byref(opts) if opts else None,
                                             recs_ptr, maps_ptr, st_ptr))
        del keep

    def elapsed(self, job: int) -> float:
        ms = ctypes.c_float()
        _check(lib().ckc_job_elapsed(self.h, job, ctypes.byref(ms)))
        return ms.value

    def release(self, job: int):
        """Waits for a job and drops its results."""
        _check(lib().ckc_read_results(self.h, job, None, None, None, WAIT))

    def autotune(self, descs, reps: int = 2, base: LaunchOpts | None = None, log_cap: int = 128):
        """Native autotuner: (best LaunchOpts, [(opts dict, ms), ...])."""
        arr, keep = descs if isinstance(descs, tuple) else self.prepare(descs)
        best = LaunchOpts()
        log = (TuneEntry * log_cap)()
        n = ctypes.c_uint32()
        _check(lib().ckc_autotune(self.h, arr, len(arr), ctypes.byref(base) if base else None, reps,
                                  ctypes.byref(best), log, log_cap, ctypes.byref(n)))
        del keep
        return best, [(log[k].opts.as_dict(), log[k].ms) for k in range(n.value)]

    def sizes(self, job: int):
        ni, nr = ctypes.c_uint64(), ctypes.c_uint64()
        _check(lib().ckc_job_sizes(self.h, job, ctypes.byref(ni), ctypes.byref(nr)))
        return ni.value, nr.value

    def timing(self, job: int):
        """[plan, trace evaluators, interpreter, body passes, finishing] in ms."""
        ms = (ctypes.c_float * 5)()
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

    def read_device(self, job: int, recs_ptr: int, maps_ptr: int | None, st_ptr: int | None,
                    enqueue: bool = False):
        """Device-to-device readback; with enqueue the copies are only queued
        behind the job (synchronize the device before using the results)."""
        flags = WAIT | DST_DEVICE | (ENQUEUE if enqueue else 0)
        _check(lib().ckc_read_results(self.h, job, recs_ptr, maps_ptr, st_ptr, flags))


class DeviceWorkload:
    """A workload's data arrays, allocation tables and program placed on the
    device once (kept resident across checks)."""

    def __init__(self, ctx: Context, wl, device: str = "cuda", no_prune: bool = False):
        import torch
        self.ctx, self.wl = ctx, wl
        self.tensors = [torch.from_numpy(np.ascontiguousarray(d)).to(device) for d in wl.data]
        self.prog, self.info = ctx.load_program(wl.ir, no_prune=no_prune)
        self.table_ids = []
        for t in wl.tables:
            e = np.array(t, ALLOC_DTYPE)
            refs = e["data"].astype(np.int64)
            e["data"] = [self.tensors[r - 1].data_ptr() if r else 0 for r in refs]
            self.table_ids.append(ctx.put_table(e))
        self.table_ids = np.array(self.table_ids, np.uint32)

    def desc(self, mode=None, dense=True, cap_log2=None, idx=None, detector=None):
        """Descriptor dict of the workload (inputs ``idx``, default all);
        ``detector`` overrides the workload's detector model (0 exact, 1
        tripwire)."""
        wl = self.wl
        sel = slice(None) if idx is None else idx
        det = getattr(wl, "detector", 0) if detector is None else detector
        flags = (DENSE_MAP if dense else 0) | (TRIPWIRE if det else 0)
        return dict(prog=self.prog, launch=wl.launch[sel], scalars=wl.scalars[sel],
                    table_ids=self.table_ids[wl.table_idx[sel]],
                    mode=wl.mode if mode is None else mode, flags=flags,
                    cap_log2=wl.cap_log2 if cap_log2 is None else cap_log2)

    def close(self):
        for t in self.table_ids:
            self.ctx.free_table(int(t))
        self.ctx.unload_program(self.prog)
        self.tensors = []


def run_workload(ctx: Context, wl, mode=None, force_generic=False, maps=True, cap_log2=None,
                 opts: LaunchOpts | None = None, no_prune: bool = False):
    """Check every input of a workload; returns the oracle-shaped result dict
    (records [n, n_acc], maps [n, 65536] or None, status [n]).  ``opts``
    (launch_opts) overrides force_generic."""
    dw = DeviceWorkload(ctx, wl, no_prune=no_prune)
    try:
        job = ctx.check([dw.desc(mode, maps, cap_log2)], force_generic=force_generic, opts=opts)
        recs, mp, st = ctx.read(job, maps=maps)
    finally:
        dw.close()
    n = wl.n_inputs
    return dict(records=recs.reshape(n, -1), maps=mp, status=st, info=dw.info)


class DeviceBatch:
    """A mixed batch (one-input workloads with their own programs, tables and
    data) placed on the device once: each distinct program is loaded once,
    every data array sits in one int32 device buffer, one table per kernel."""

    def __init__(self, ctx: Context, mb, device: str = "cuda"):
        import torch
        self.ctx, self.mb = ctx, mb
        self.progs, self.infos = {}, {}
        for k in mb.kernels:
            if k.ir not in self.progs:
                self.progs[k.ir], self.infos[k.ir] = ctx.load_program(k.ir)
        # one flat buffer for every data array (all int32), 256-byte aligned offsets
        offs, total = [], 0
        for k in mb.kernels:
            o = []
            for d in k.data:
                o.append(total)
                total += (d.nbytes + 255) // 256 * 256
            offs.append(o)
        flat = np.zeros(max(total, 256) // 4, np.int32)
        for k, o in zip(mb.kernels, offs):
            for d, off in zip(k.data, o):
                flat[off // 4: off // 4 + d.size] = np.ascontiguousarray(d, np.int32).reshape(-1)
        self.buf = torch.from_numpy(flat).to(device)
        base = self.buf.data_ptr()
        self.table_ids = []
        for k, o in zip(mb.kernels, offs):
            e = np.array(k.tables[0], ALLOC_DTYPE)
            refs = e["data"].astype(np.int64)
            e["data"] = [base + o[r - 1] if r else 0 for r in refs]
            self.table_ids.append(ctx.put_table(e))

    def descs(self, idx=None, dense=True):
        """One descriptor per kernel (kernels ``idx``, default all), in order."""
        ks = range(len(self.mb.kernels)) if idx is None else idx
        out = []
        for i in ks:
            k = self.mb.kernels[i]
            out.append(dict(prog=self.progs[k.ir], launch=k.launch, scalars=k.scalars,
                            table_ids=np.array([self.table_ids[i]], np.uint32), mode=k.mode,
                            flags=DENSE_MAP if dense else 0, cap_log2=k.cap_log2))
        return out

    def n_accesses(self, i):
        return self.infos[self.mb.kernels[i].ir]["n_accesses"]

    def close(self):
        for t in self.table_ids:
            self.ctx.free_table(int(t))
        for pid in self.progs.values():
            self.ctx.unload_program(pid)
        self.table_ids, self.progs, self.buf = [], {}, None


def split_results(recs, maps, st, counts):
    """Per-input views of a job's flat records given each input's access count."""
    out, r = [], 0
    for i, n in enumerate(counts):
        out.append(dict(records=recs[r:r + n], maps=None if maps is None else maps[i], status=st[i]))
        r += n
    return out


class Server:
    """The library's request loop (ckc_server_*) on a context: continuous
    batching of submitted jobs over ``n_streams`` streams under an HBM
    working-set cap.  While it exists, the context is used only through it."""

    def __init__(self, ctx: Context, n_streams=4, max_batch_jobs=0, hbm_cap_bytes=0,
                 opts: LaunchOpts | None = None):
        cfg = ServerConfig(n_streams, max_batch_jobs, hbm_cap_bytes, opts if opts is not None else LaunchOpts())
        h = ctypes.c_void_p()
        _check(lib().ckc_server_create(ctx.h, ctypes.byref(cfg), ctypes.byref(h)))
        self.h = h

    def submit(self, desc, arrival_ns: int = 0) -> int:
        """desc: a descriptor dict or a ``Context.prepare([desc])`` result."""
        arr, keep = desc if isinstance(desc, tuple) else Context.prepare([desc])
        t = ctypes.c_uint64()
        _check(lib().ckc_server_submit(self.h, arr, arrival_ns, ctypes.byref(t)))
        del keep
        return t.value

    def result(self, ticket: int, n_inputs: int, n_acc: int, maps: bool = True, wait: bool = True):
        """(code, records [n_inputs*n_acc], maps [n_inputs, 65536] or None, status, stats dict);
        code is CKC_OK or the job's error (e.g. -4 for a job above the cap); None if not ready."""
        recs = np.zeros(n_inputs * n_acc, RECORD_DTYPE)
        mp = np.zeros((n_inputs, 65536), np.uint8) if maps else None
        st = np.zeros(n_inputs, STATUS_DTYPE)
        js = JobStats()
        rc = lib().ckc_server_result(self.h, ticket, _p(recs), _p(mp) if maps else None, _p(st),
                                     ctypes.byref(js), WAIT if wait else 0)
        if rc == NOT_READY:
            return None
        stats = {f: getattr(js, f) for f, _ in JobStats._fields_}
        return rc, recs, mp, st, stats

    def stats(self):
        out = ServerStats()
        _check(lib().ckc_server_get_stats(self.h, ctypes.byref(out)))
        return {f: getattr(out, f) for f, _ in ServerStats._fields_}

    def close(self):
        if self.h:
            lib().ckc_server_destroy(self.h)
            self.h = None

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()


class DeviceStream:
    """A served stream's programs, resident CSR pool (one device buffer) and
    one allocation table per job, placed on the device before serving."""

    def __init__(self, ctx: Context, ss, device: str = "cuda"):
        import torch
        self.ctx, self.ss = ctx, ss
        self.progs, self.infos = {}, {}
        for k in ss.jobs:
            if k.ir not in self.progs:
                self.progs[k.ir], self.infos[k.ir] = ctx.load_program(k.ir)
        offs, total = [], 0
        for d in ss.pool:
            offs.append(total)
            total += (d.nbytes + 255) // 256 * 256
        flat = np.zeros(max(total, 256) // 4, np.int32)
        for d, off in zip(ss.pool, offs):
            flat[off // 4: off // 4 + d.size] = np.ascontiguousarray(d, np.int32).reshape(-1)
        self.buf = torch.from_numpy(flat).to(device)
        base = self.buf.data_ptr()
        self.table_ids = []
        for k in ss.jobs:
            e = np.array(k.tables[0], ALLOC_DTYPE)
            refs = e["data"].astype(np.int64)
            e["data"] = [base + offs[r - 1] if r else 0 for r in refs]
            self.table_ids.append(ctx.put_table(e))

    def desc(self, j: int, dense: bool = True):
        k = self.ss.jobs[j]
        return dict(prog=self.progs[k.ir], launch=k.launch, scalars=k.scalars,
                    table_ids=np.array([self.table_ids[j]], np.uint32), mode=k.mode,
                    flags=DENSE_MAP if dense else 0, cap_log2=k.cap_log2)

    def n_accesses(self, j: int) -> int:
        return self.infos[self.ss.jobs[j].ir]["n_accesses"]

    def close(self):
        for t in self.table_ids:
            self.ctx.free_table(int(t))
        for pid in self.progs.values():
            self.ctx.unload_program(pid)
        self.table_ids, self.progs, self.buf = [], {}, None


class Fuzz:
    """A fuzzing campaign on the device (ckc_fuzz_*) seeded with input
    ``idx`` of a DeviceWorkload."""

    def __init__(self, ctx: Context, dw: DeviceWorkload, batch: int, max_stack: int = 4,
                 max_threads: int = 1 << 20, max_block: int = 1024, corpus_cap: int = 256,
                 data_slot: int = FUZZ_NO_SLOT, ops: int = MUT_LAUNCH | MUT_SCALAR, seed: int = 0,
                 mode=None, idx: int = 0):
        wl = dw.wl
        cfg = FuzzConfig()
        cfg.prog_id = dw.prog
        cfg.table_id = int(dw.table_ids[wl.table_idx[idx]])
        for q in range(6):
            cfg.launch[q] = int(wl.launch[idx][q])
        for q in range(wl.scalars.shape[1]):
            cfg.scalars[q] = int(wl.scalars[idx][q])
        cfg.mode = wl.mode if mode is None else mode
        cfg.flags = TRIPWIRE if getattr(wl, "detector", 0) else 0
        cfg.loop_cap_log2[0], cfg.loop_cap_log2[1] = wl.cap_log2
        cfg.batch, cfg.max_stack, cfg.max_block, cfg.corpus_cap = batch, max_stack, max_block, corpus_cap
        cfg.max_threads, cfg.data_slot, cfg.ops, cfg.seed = max_threads, data_slot, ops, seed
        self.cfg, self.dw = cfg, dw
        self.n_elems = 0
        tab = wl.tables[wl.table_idx[idx]]
        if data_slot != FUZZ_NO_SLOT and data_slot < len(tab):
            self.n_elems = int(tab[data_slot]["size_bytes"]) // 4
        h = ctypes.c_void_p()
        _check(lib().ckc_fuzz_create(ctx.h, ctypes.byref(cfg), ctypes.byref(h)))
        self.h = h

    def run(self, generations: int):
        _check(lib().ckc_fuzz_run(self.h, generations))

    def stats(self):
        st = FuzzStats()
        _check(lib().ckc_fuzz_get_stats(self.h, ctypes.byref(st)))
        return {f: int(getattr(st, f)) for f, _ in FuzzStats._fields_}

    def read(self):
        """dict(launch [size, 6], scalars [size, 16], data [size, n_elems] or
        None, gen [size], virgin [65536], sigs [n_accesses, 4], stats)."""
        st = self.stats()
        cap, n = self.cfg.corpus_cap, st["corpus"]
        n_acc = self.dw.info["n_accesses"]
        launch = np.zeros((cap, 6), np.uint32)
        scal = np.zeros((cap, 16), np.int64)
        data = np.zeros((cap, max(1, self.n_elems)), np.int32)
        gen = np.zeros(cap, np.uint32)
        virgin = np.zeros(65536, np.uint8)
        sigs = np.zeros((max(1, n_acc), 4), np.uint64)
        _check(lib().ckc_fuzz_read(self.h, _p(launch), _p(scal), _p(data) if self.n_elems else None, _p(gen),
                                   _p(virgin), _p(sigs)))
        return dict(launch=launch[:n], scalars=scal[:n], data=data[:n] if self.n_elems else None, gen=gen[:n],
                    virgin=virgin, sigs=sigs[:n_acc], stats=st)

    def close(self):
        if self.h:
            lib().ckc_fuzz_destroy(self.h)
            self.h = None

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()
