"""The served form: the library's request loop admits jobs from an open-loop
Poisson stream under an HBM working-set cap and runs them in overlapping
batches on several streams.  Each job's result must be byte-identical to the
same job checked alone (zero tolerance: every reduction is order-free) and to
the oracle; the cap must hold at all times."""
import os

import numpy as np
import pytest

from oracle import oracle as O
from paper_2601_01048_amd import ckc, serve
from paper_2601_01048_amd.gen import workloads as W

pytestmark = pytest.mark.gpu

NCPU = max(1, min(16, os.cpu_count() or 1))


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    c = ckc.Context(0)
    yield c
    c.close()


@pytest.fixture(scope="module")
def stream(ctx):
    ss = W.config5(seed=1005, rate=20000.0, duration_s=0.05, a_range=(1e3, 3e5), log2_range=(4, 12))
    ds = ckc.DeviceStream(ctx, ss)
    yield ss, ds
    ds.close()


def alone(ctx, ds, j):
    job = ctx.check([ds.desc(j)])
    recs, mp, st = ctx.read(job)
    return dict(records=recs, maps=mp[0], status=st[0])


def same(a, b, what):
    for f in ("first_key", "count", "kinds", "index", "first_kind"):
        assert np.array_equal(a["records"][f], b["records"][f]), (what, f)
    for f in ("lanes", "accesses_checked", "hang_lanes", "arith_faults"):
        assert int(a["status"][f]) == int(b["status"][f]), (what, f)
    assert np.array_equal(a["maps"], b["maps"]), (what, "maps")


def oracle_job(ss, j):
    k = ss.jobs[j]
    wl = W.Workload(k.name, k.ir, k.launch, k.scalars, k.tables, k.table_idx, ss.pool, k.mode, k.cap_log2)
    o = O.check(wl, nthreads=NCPU)
    return dict(records=o["records"][0], maps=o["maps"][0], status=o["status"][0])


def test_served_equals_alone_and_oracle(ctx, stream):
    ss, ds = stream
    print(f"[case] served stream of {ss.n_jobs} jobs", flush=True)
    with ckc.Server(ctx, n_streams=4) as srv:
        res, lag = serve.replay(srv, ds, keep_results=True)
        st = srv.stats()
    assert st["submitted"] == st["completed"] == ss.n_jobs and st["rejected"] == 0
    assert all(r["code"] == 0 for r in res)
    # continuous batching happened: several jobs per batch and batches in flight together
    assert max(r["stats"]["batch_jobs"] for r in res) > 1
    assert st["max_inflight_jobs"] > 1
    for r in res:
        s = r["stats"]
        assert s["t_arrival_ns"] <= s["t_admit_ns"] <= s["t_done_ns"]
    for r in res:
        same(r, alone(ctx, ds, r["job"]), f"job {r['job']} alone")
    for j in np.random.default_rng(3).choice(ss.n_jobs, size=40, replace=False):
        same(res[int(j)], oracle_job(ss, int(j)), f"job {j} oracle")


def test_admission_cap_1mib(ctx):
    """All jobs at once under a 1 MiB cap: the cap binds (at most a few jobs with
    their 64 KiB maps in flight), jobs above it alone end with CKC_E_NOMEM, the
    rest equal their results alone."""
    ss = W.config5(seed=77, rate=20000.0, duration_s=0.012, a_range=(1e3, 5e6), log2_range=(4, 16))
    ds = ckc.DeviceStream(ctx, ss)
    cap = 1 << 20
    print(f"[case] served stream of {ss.n_jobs} jobs under a 1 MiB cap", flush=True)
    try:
        with ckc.Server(ctx, n_streams=4, hbm_cap_bytes=cap) as srv:
            res, _ = serve.replay(srv, ds, time_scale=0.0, keep_results=True)
            st = srv.stats()
        _check_cap(ctx, ds, res, st, cap)
    finally:
        ds.close()


def _check_cap(ctx, ds, res, st, cap):
    assert 0 < st["max_inflight_bytes"] <= cap
    big = [r for r in res if r["stats"]["ws_bytes"] > cap]
    assert big, "the stream should hold jobs above 1 MiB"
    assert st["rejected"] == len(big)
    for r in res:
        if r["stats"]["ws_bytes"] > cap:
            assert r["code"] == -4
        else:
            assert r["code"] == 0
            same(r, alone(ctx, ds, r["job"]), f"job {r['job']} under cap")


def test_server_rejects_bad_descriptor(ctx, stream):
    ss, ds = stream
    with ckc.Server(ctx, n_streams=2) as srv:
        d = ds.desc(0)
        d["prog"] = 999999
        with pytest.raises(ckc.CkcError):
            srv.submit(d)
        t = srv.submit(ds.desc(0))
        code, recs, mp, st, stats = srv.result(t, 1, ds.n_accesses(0))
        assert code == 0 and stats["batch_jobs"] >= 1
