"""Open-loop replay of a served stream through the library's request loop:
each job is submitted at its arrival time (whether or not earlier jobs have
finished), a collector thread takes results as they complete, and the
per-job stats (arrival, admission, results readable) give the latency
distribution.  Marshalling and timing only; the checking runs in libckc."""
from __future__ import annotations

import gc
import threading
import time

import numpy as np

from . import ckc


def replay(server: ckc.Server, ds: ckc.DeviceStream, jobs=None, time_scale: float = 1.0, maps: bool = True,
           keep_results: bool = False):
    """Submits ``jobs`` (default all) of ``ds.ss`` at their arrival times
    (scaled by ``time_scale``; 0 submits back to back) and collects them.
    Returns (list of per-job dicts with stats [and results], submit lag stats)."""
    ss = ds.ss
    idx = list(range(ss.n_jobs)) if jobs is None else list(jobs)
    prepared = [ckc.Context.prepare([ds.desc(j, dense=maps)]) for j in idx]
    n_acc = [ds.n_accesses(j) for j in idx]
    out = [None] * len(idx)
    tickets = [None] * len(idx)
    ready = threading.Semaphore(0)

    def collect():
        for q in range(len(idx)):
            ready.acquire()
            code, recs, mp, st, stats = server.result(tickets[q], 1, n_acc[q], maps=maps, wait=True)
            d = dict(job=idx[q], code=code, stats=stats, accesses=int(st["accesses_checked"].sum()))
            if keep_results:
                d.update(records=recs, maps=None if mp is None else mp[0], status=st[0])
            out[q] = d

    # the load generator must not pause: Python's cyclic garbage collector
    # (a full collection over the replay's objects takes hundreds of ms) is
    # off while jobs are submitted, and the objects made so far are frozen
    gc_was = gc.isenabled()
    gc.collect()
    gc.freeze()
    gc.disable()
    th = threading.Thread(target=collect)
    th.start()
    t0 = time.monotonic_ns() + 20_000_000  # start 20 ms from now
    lags = []
    try:
        for q, j in enumerate(idx):
            due = t0 + int(ss.arrivals[j] * time_scale * 1e9)
            while True:
                now = time.monotonic_ns()
                if now >= due:
                    break
                if due - now > 200_000:
                    time.sleep((due - now - 100_000) / 1e9)
            lags.append(time.monotonic_ns() - due)
            tickets[q] = server.submit(prepared[q], arrival_ns=due)
            ready.release()
    finally:
        th.join()
        gc.unfreeze()
        if gc_was:
            gc.enable()
    lags = np.array(lags) / 1e3
    for q, d in enumerate(out):
        d["submit_lag_us"] = float(lags[q])
    return out, dict(submit_lag_us_p50=float(np.percentile(lags, 50)),
                     submit_lag_us_p99=float(np.percentile(lags, 99)),
                     submit_lag_us_max=float(lags.max()) if len(lags) else 0.0,
                     late_over_1ms=int((lags > 1000).sum()), t0_ns=t0)


def summarize(res, t_from_s: float = 0.0, t0_ns: int = 0, arrivals=None):
    """Latency percentiles (ms) and sustained accesses/s over the jobs that
    arrived at or after ``t_from_s``."""
    sel = [r for r in res if arrivals is None or arrivals[r["job"]] >= t_from_s]
    ok = [r for r in sel if r["code"] == 0]
    lat = np.array([(r["stats"]["t_done_ns"] - r["stats"]["t_arrival_ns"]) / 1e6 for r in ok])
    first = min(r["stats"]["t_arrival_ns"] for r in ok)
    last = max(r["stats"]["t_done_ns"] for r in ok)
    acc = sum(r["accesses"] for r in ok)
    span = (last - first) / 1e9
    batch = np.array([r["stats"]["batch_jobs"] for r in ok])
    return dict(jobs=len(sel), completed_ok=len(ok), p50_ms=float(np.percentile(lat, 50)),
                p99_ms=float(np.percentile(lat, 99)), p999_ms=float(np.percentile(lat, 99.9)),
                mean_ms=float(lat.mean()), max_ms=float(lat.max()),
                accesses=acc, window_s=span, accesses_per_s=acc / span, jobs_per_s=len(ok) / span,
                mean_batch_jobs=float(batch.mean()), max_batch_jobs=int(batch.max()))
