#!/usr/bin/env python3
"""Throughput of the checking hot path on one MI355X.

Workload: the 2-D 9-point stencil configuration -- 4096 seeded inputs, each a
grid of (128 +- 3)^2 blocks of 16 x 16 threads over an (2048 +- 3)^2 int32-indexed
pair of allocations, halo radius 1 or 2 -- checked over the whole grid (every
thread of every input).  One step = one ckc_check_batch (thread sets and
traces, evaluation, first-violation replay, dense 64 KiB maps) plus
ckc_read_results into device buffers; program and allocation tables are
resident before the timed region.

Prints one JSON line: checked thread-accesses/s (value), inputs/s, the
roofline of the dominant kernel (timed with HIP events on the job's stream)
and the oracle's throughput on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

from paper_2601_01048_amd import ckc  # noqa: E402
from paper_2601_01048_amd.gen import workloads as W  # noqa: E402

# MI355X: 256 CUs x 64 int32 lanes per clock x 2.4 GHz
PEAK_INT_OPS = 256 * 64 * 2.4e9
# algorithmic work of one checked access on the affine path: form the index
# (per-thread base + per-access offset) and one unsigned bound compare
OPS_PER_ACCESS = 2
# sources of the trace evaluator (its counters stay valid while these are unchanged)
TRACE_SOURCES = ("dev_common.h", "dev_plan.h", "dev_trace.h", "dformat.h", "kernels.h")


# sources of the interpreter's body passes (the CSR gather kernel)
INTERP_SOURCES = ("dev_common.h", "dev_plan.h", "dev_interp.h", "dformat.h", "kernels.h")


def source_hash(files=TRACE_SOURCES) -> str:
    import hashlib
    h = hashlib.sha256()
    for f in files:
        h.update(open(os.path.join(ROOT, "paper_2601_01048_amd", "csrc", f), "rb").read())
    return h.hexdigest()[:16]


def recorded_traffic(kernel: str, files) -> float | None:
    """HBM bytes per launch from the committed counter runs, valid only for the
    kernel sources they were taken on."""
    try:
        rec = json.load(open(os.path.join(ROOT, "profiles", "traffic.json")))[kernel]
        return rec["traffic_bytes"] if source_hash(files) == rec["source_sha256_16"] else None
    except (OSError, KeyError, ValueError):
        return None


def progress(msg: str):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def kernel_ms(kern) -> dict:
    """Mean per-stage device times (HIP events on the job's stream)."""
    names = ("plan", "eval_trace", "interpreter", "body_passes", "finish")
    return {k: float(kern[:, q].mean()) for q, k in enumerate(names)}


def copy_probe():
    """One 1 GiB device-to-device copy: the reference for HBM byte counters."""
    import torch
    src = torch.ones(1 << 28, dtype=torch.int32, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    del src, dst


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-rep", action="store_true", help="skip the representative-thread line")
    ap.add_argument("--cpu-sample", type=int, default=16, help="inputs in the oracle sample")
    ap.add_argument("--copy-probe", action="store_true",
                    help="also run one 1 GiB device-to-device copy (reference for HBM byte counters)")
    ap.add_argument("--no-batched", action="store_true", help="skip the batched sub-result")
    ap.add_argument("--no-served", action="store_true", help="skip the served sub-result")
    ap.add_argument("--served-seconds", type=float, default=35.0,
                    help="length of the served stream (the first 5 s are warm-up)")
    ap.add_argument("--workload", default="stencil", choices=["stencil", "csr", "affine1d", "batched", "served"],
                    help="stencil: the benchmark batch; csr / affine1d: the other plain configurations; "
                         "batched: 10,000 mixed kernels in one job vs one job per kernel")
    return ap.parse_args()


HBM_PEAK = 8.0e12  # bytes/s


def bench_other(args):
    """The CSR gather (64 inputs, 2^20 rows) or the 1-D affine batch (256
    inputs): same step definition, one JSON line."""
    import torch
    if args.workload == "csr":
        wl = W.config3()
        desc_w = "CSR SpMV gather, 64 inputs, 2^20 rows, power-law rows (mean 16 nnz), 0.1% corrupted col_idx"
    else:
        wl = W.config1()
        desc_w = "1-D affine kernel, 256 inputs, 32-80 blocks of 256, 4 accesses per thread"
    n = wl.n_inputs
    if args.copy_probe:
        copy_probe()
    with ckc.Context(0) as ctx:
        dw = ckc.DeviceWorkload(ctx, wl)
        n_acc = dw.info["n_accesses"]
        out = dict(recs=torch.empty(n * n_acc * 32, dtype=torch.uint8, device="cuda"),
                   maps=torch.empty(n * 65536, dtype=torch.uint8, device="cuda"),
                   st=torch.empty(n * 40, dtype=torch.uint8, device="cuda"))
        run_steps(ctx, dw, out, W.MODE_FULL, args.warmup)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        tim = run_steps(ctx, dw, out, W.MODE_FULL, args.steps)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        st = np.frombuffer(out["st"].cpu().numpy().tobytes(), ckc.STATUS_DTYPE)
        dw.close()
    accesses = int(st["accesses_checked"].sum())
    step_s = (t1 - t0) / args.steps
    kern = np.array(tim)
    res = {"metric": "checked thread-accesses/sec", "value": accesses / step_s, "unit": "accesses/s",
           "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": step_s * 1e3,
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "int32",
           "data": "synthetic", "config": {"workload": desc_w, "inputs": n, "accesses_per_batch": accesses},
           "inputs_per_s": n / step_s, "kernel_ms": kernel_ms(kern)}
    if args.workload == "csr":
        # the body pass reads col_idx once per nonzero (4 B); val and x are
        # address-only; row_ptr is read by the whole-thread pass
        nnz = wl.meta["nnz"]
        alg = n * 4 * nnz
        ms = float(kern[:, 3].mean())
        res["roofline"] = {"bound": "hbm", "kernel": "eval_gather_kernel", "achieved": alg / (ms * 1e-3) / 1e9,
                           "peak": HBM_PEAK / 1e9, "unit": "GB/s", "frac": alg / (ms * 1e-3) / HBM_PEAK,
                           "traffic": recorded_traffic("eval_gather_kernel", INTERP_SOURCES)}
    else:
        ms = float(kern[:, 1].mean())
        ach = OPS_PER_ACCESS * accesses / (ms * 1e-3)
        res["roofline"] = {"bound": "alu", "kernel": "eval_trace_kernel", "achieved": ach / 1e12,
                           "peak": PEAK_INT_OPS / 1e12, "unit": "Tops/s (int32)", "frac": ach / PEAK_INT_OPS,
                           "traffic": None}
    print(json.dumps(res))


def bench_batched(args):
    """10,000 mixed kernels (F1/F2/F3, int32/int64, 1..65536 threads each) in
    one job with autotuned launch options and one graph, against one job
    (seven kernel launches) per kernel."""
    import torch
    t_gen = time.perf_counter()
    mb = W.config4()
    t_gen = time.perf_counter() - t_gen
    with ckc.Context(0) as ctx:
        db = ckc.DeviceBatch(ctx, mb)
        descs = db.descs()
        prep = ckc.Context.prepare(descs)
        n_rec = sum(db.n_accesses(i) for i in range(mb.n_kernels))
        n = mb.n_kernels
        out = dict(recs=torch.empty(n_rec * 32, dtype=torch.uint8, device="cuda"),
                   maps=torch.empty(n * 65536, dtype=torch.uint8, device="cuda"),
                   st=torch.empty(n * 40, dtype=torch.uint8, device="cuda"))
        progress("batched: generated and uploaded")
        t_tune = time.perf_counter()
        best, log = ctx.autotune(prep, reps=1)
        t_tune = time.perf_counter() - t_tune
        best.use_graph = 1
        # per-kernel split of the tuned options (events need the non-graph form)
        split_opts = ckc.launch_opts(best.schedule, best.chunk, best.wg_per_cu)
        job = ctx.check(prep, opts=split_opts)
        split = ctx.timing(job)
        ctx.release(job)

        def step():
            j = ctx.check(prep, opts=best)
            ctx.read_device(j, out["recs"].data_ptr(), out["maps"].data_ptr(), out["st"].data_ptr(), enqueue=True)

        for _ in range(args.warmup):
            step()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            step()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        st = np.frombuffer(out["st"].cpu().numpy().tobytes(), ckc.STATUS_DTYPE)
        accesses = int(st["accesses_checked"].sum())
        step_s = (t1 - t0) / args.steps
        # one job per kernel: all queued, then each read back into the same buffers
        singles = [ckc.Context.prepare([d]) for d in descs]
        rec_off = np.concatenate([[0], np.cumsum([db.n_accesses(i) for i in range(n)])])
        for rep in range(2):  # the first pass fills the buffer pool
            torch.cuda.synchronize()
            p0 = time.perf_counter()
            jobs = [ctx.check(sp) for sp in singles]
            for i, j in enumerate(jobs):
                ctx.read_device(j, out["recs"].data_ptr() + 32 * int(rec_off[i]),
                                out["maps"].data_ptr() + 65536 * i, out["st"].data_ptr() + 40 * i)
            torch.cuda.synchronize()
            p1 = time.perf_counter()
        st2 = np.frombuffer(out["st"].cpu().numpy().tobytes(), ckc.STATUS_DTYPE)
        assert int(st2["accesses_checked"].sum()) == accesses
        db.close()
    per_kernel_s = p1 - p0
    fam = mb.meta["family"]
    res = {"metric": "checked thread-accesses/sec", "value": accesses / step_s, "unit": "accesses/s",
           "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": step_s * 1e3,
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "int32+int64",
           "data": "synthetic",
           "config": {"workload": "batched: 10,000 mixed kernels (F1 1-D affine, F2 stencil, F3 CSR; int32 and "
                                  "int64), threads per kernel log-uniform in [1, 65536], one job, one graph",
                      "kernels": n, "threads": int(st["lanes"].sum()), "accesses_per_batch": accesses,
                      "family_counts": [int((fam == f).sum()) for f in range(3)], "seed": 1004},
           "kernels_per_s": n / step_s,
           "per_kernel_launches": {"ms_total": per_kernel_s * 1e3, "kernels_per_s": n / per_kernel_s,
                                   "accesses_per_s": accesses / per_kernel_s,
                                   "launches": int(sum(8 + (8 if k.meta["family"] == "F3" else 0)
                                                       for k in mb.kernels))},
           "speedup_vs_per_kernel": per_kernel_s / step_s,
           "autotune": {"best": best.as_dict(), "candidates": len(log), "seconds": t_tune,
                        "best_ms": min(ms for _, ms in log), "worst_ms": max(ms for _, ms in log),
                        "default_ms": [ms for d, ms in log
                                       if d["schedule"] == "blocked" and d["wg_per_cu"] == 0][0]},
           "kernel_ms_tuned_no_graph": kernel_ms(np.array([split])),
           "generator_s": t_gen}
    return res


def bench_served(args):
    """Poisson stream of check jobs (2000/s, 1e3..1e7 thread-accesses each,
    F1/F2/F3 mix, int32/int64) replayed open-loop through the library's
    request loop (4 streams, continuous batching, 64 GB admission cap)."""
    from paper_2601_01048_amd import serve
    warm = 5.0
    ss = W.config5(duration_s=args.served_seconds)
    with ckc.Context(0) as ctx:
        t0 = time.perf_counter()
        ds = ckc.DeviceStream(ctx, ss)
        t_setup = time.perf_counter() - t0
        progress(f"served: {ss.n_jobs} jobs staged, replaying")
        with ckc.Server(ctx, n_streams=4) as srv:
            res, lag = serve.replay(srv, ds)
            st = srv.stats()
        ds.close()
    summ = serve.summarize(res, t_from_s=min(warm, args.served_seconds / 2), arrivals=ss.arrivals)
    offered = float(ss.meta["A"].mean() * ss.meta["rate"])
    return {"metric": "checked thread-accesses/sec (served) and p50/p99 job latency",
            "value": summ["accesses_per_s"], "unit": "accesses/s",
            "p50_ms": summ["p50_ms"], "p99_ms": summ["p99_ms"], "mean_ms": summ["mean_ms"],
            "max_ms": summ["max_ms"], "jobs_per_s": summ["jobs_per_s"],
            "config": {"workload": "served: Poisson 2000 jobs/s, sizes log-uniform in [1e3, 1e7] thread-accesses, "
                                   "F1/F2/F3 x int32/int64, resident CSR pool 2^4..2^18 rows, dense maps, "
                                   "4 streams, 64 GB admission cap",
                       "jobs": ss.n_jobs, "seconds": args.served_seconds, "warmup_s": warm, "seed": 1005},
            "offered_accesses_per_s": offered, "window": summ, "server": st, "submit_lag": lag,
            "setup_s": t_setup}


def run_steps(ctx, dw, out, mode, steps):
    """Runs `steps` checks back to back on the context's stream: each job is
    queued before the previous one's stage timing is read, and every job's
    results are copied to the device buffers behind it on the same stream
    (CKC_ENQUEUE), so the device never waits for the host.  Returns the
    per-step stage timings."""
    timings, prev = [], None

    def retire(job):
        timings.append(ctx.timing(job))
        ctx.read_device(job, out["recs"].data_ptr(), out["maps"].data_ptr(), out["st"].data_ptr(), enqueue=True)

    for _ in range(steps):
        job = ctx.check([dw.desc(mode=mode, dense=True)])
        if prev is not None:
            retire(prev)
        prev = job
    if prev is not None:
        retire(prev)
    return timings


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported (the workload shards by "
              "input with no communication; see the design notes).", file=sys.stderr)
        sys.exit(2)
    import torch

    assert torch.cuda.is_available(), "bench.py needs a HIP device"
    torch.cuda.set_device(0)
    if args.workload == "batched":
        print(json.dumps(bench_batched(args)))
        return
    if args.workload == "served":
        print(json.dumps(bench_served(args)))
        return
    if args.workload != "stencil":
        bench_other(args)
        return
    if args.copy_probe:
        copy_probe()
    wl = W.config2(mode=W.MODE_FULL)
    n = wl.n_inputs
    with ckc.Context(0) as ctx:
        dw = ckc.DeviceWorkload(ctx, wl)
        n_acc = dw.info["n_accesses"]
        out = dict(recs=torch.empty(n * n_acc * 32, dtype=torch.uint8, device="cuda"),
                   maps=torch.empty(n * 65536, dtype=torch.uint8, device="cuda"),
                   st=torch.empty(n * 40, dtype=torch.uint8, device="cuda"))
        run_steps(ctx, dw, out, W.MODE_FULL, args.warmup)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        tim = run_steps(ctx, dw, out, W.MODE_FULL, args.steps)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        st = np.frombuffer(out["st"].cpu().numpy().tobytes(), ckc.STATUS_DTYPE)
        accesses = int(st["accesses_checked"].sum())
        step_s = (t1 - t0) / args.steps
        kern = np.array(tim)  # [steps, 5] ms per stage
        eval_ms = float(kern[:, 1].mean())
        result = {
            "metric": "checked thread-accesses/sec",
            "value": accesses / step_s,
            "unit": "accesses/s",
            "n_gpus": 1,
            "steps": args.steps,
            "warmup": args.warmup,
            "ms_per_step": step_s * 1e3,
            "higher_is_better": True,
            "scaling": "weak",
            "vs_baseline": None,
            "dtype": "int32",
            "data": "synthetic",
            "config": {
                "workload": "2-D 9-point stencil, 4096 inputs, grid (128+-3)^2 x 16x16 threads, "
                            "(2048+-3)^2 allocations, radius 1-2, whole grid (FULL)",
                "inputs": n,
                "threads_per_batch": int(st["lanes"].sum()),
                "accesses_per_batch": accesses,
                "seed": 1002,
            },
            "inputs_per_s": n / step_s,
            "kernel_ms": kernel_ms(kern),
        }
        achieved = OPS_PER_ACCESS * accesses / (eval_ms * 1e-3)
        # HBM bytes per launch from the committed counter runs
        traffic = recorded_traffic("eval_trace_kernel", TRACE_SOURCES)
        result["roofline"] = {
            "bound": "alu",
            "kernel": "eval_trace_kernel",
            "achieved": achieved / 1e12,
            "peak": PEAK_INT_OPS / 1e12,
            "unit": "Tops/s (int32)",
            "frac": achieved / PEAK_INT_OPS,
            "traffic": traffic,
        }
        # the same batch decided by the end indices of row progressions:
        # identical results, most indices never formed -> inputs/s only
        run_steps(ctx, dw, out, W.MODE_ENDPOINTS, 1)
        torch.cuda.synchronize()
        e0 = time.perf_counter()
        et = run_steps(ctx, dw, out, W.MODE_ENDPOINTS, max(2, args.steps // 2))
        torch.cuda.synchronize()
        e1 = time.perf_counter()
        es = (e1 - e0) / len(et)
        result["full_endpoints"] = {"inputs_per_s": n / es, "ms_per_step": es * 1e3,
                                    "speedup_inputs_per_s_vs_full": step_s / es,
                                    "kernel_ms": kernel_ms(np.array(et))}
        if not args.no_rep:
            run_steps(ctx, dw, out, W.MODE_BOUNDARY, 1)
            torch.cuda.synchronize()
            r0 = time.perf_counter()
            rt = run_steps(ctx, dw, out, W.MODE_BOUNDARY, max(2, args.steps // 2))
            torch.cuda.synchronize()
            r1 = time.perf_counter()
            rst = np.frombuffer(out["st"].cpu().numpy().tobytes(), ckc.STATUS_DTYPE)
            rs = (r1 - r0) / len(rt)
            result["rep_boundary"] = {"inputs_per_s": n / rs, "ms_per_step": rs * 1e3,
                                      "accesses_per_s": int(rst["accesses_checked"].sum()) / rs,
                                      "lanes_per_batch": int(rst["lanes"].sum()),
                                      "speedup_inputs_per_s_vs_full": step_s / rs,
                                      "kernel_ms": kernel_ms(np.array(rt))}
        dw.close()
    progress("stencil done")
    if not args.no_batched:
        b = bench_batched(args)
        progress("batched done")
        result["batched"] = {k: b[k] for k in ("value", "unit", "ms_per_step", "kernels_per_s",
                                                "per_kernel_launches", "speedup_vs_per_kernel", "autotune",
                                                "kernel_ms_tuned_no_graph", "config")}
    if not args.no_served:
        sv = bench_served(args)
        progress("served done")
        result["served"] = {k: sv[k] for k in ("value", "unit", "p50_ms", "p99_ms", "mean_ms", "jobs_per_s",
                                                "offered_accesses_per_s", "config", "server")}
    if not args.no_cpu_baseline:
        from oracle import oracle as O
        k = min(args.cpu_sample, n)
        cores = min(16, os.cpu_count() or 1)
        sub = wl.subset(np.arange(k))
        c0 = time.perf_counter()
        o = O.check(sub, nthreads=cores, maps=False)
        c1 = time.perf_counter()
        acc_cpu = int(o["status"]["accesses_checked"].sum())
        result["cpu_baseline"] = {"value": acc_cpu / (c1 - c0), "unit": "accesses/s", "cores": cores,
                                  "kind": "oracle",
                                  "sample": f"first {k} of {n} inputs of the same workload (FULL), "
                                            f"{acc_cpu} accesses in {c1 - c0:.2f} s"}
    print(json.dumps(result))


if __name__ == "__main__":
    main()
