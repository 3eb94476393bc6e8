"""The batched form: thousands of small kernels of the three families, int32
and int64, checked in one job (one persistent launch per evaluator, or one
graph).  Every kernel's result must equal the oracle's and its own result when
checked alone, for every schedule, chunk, occupancy and with or without the
graph; the autotuner must return one of its candidates."""
import os

import numpy as np
import pytest

import batch_util as B
from paper_2601_01048_amd import ckc
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
def mini(ctx):
    mb = W.config4(seed=1004, n_kernels=160, t_max=4096)
    db = ckc.DeviceBatch(ctx, mb)
    yield mb, db
    db.close()


def run_batch(ctx, db, idx=None, opts=None):
    descs = db.descs(idx)
    job = ctx.check(descs, opts=opts)
    recs, maps, st = ctx.read(job, maps=True)
    idx = list(range(db.mb.n_kernels)) if idx is None else list(idx)
    return ckc.split_results(recs, maps, st, [db.n_accesses(i) for i in idx])


def test_mixed_batch_matches_oracle(ctx, mini):
    mb, db = mini
    print(f"[case] mixed batch of {mb.n_kernels} kernels vs oracle", flush=True)
    g = run_batch(ctx, db)
    o = B.oracle_mixed(mb, nthreads=NCPU)
    fams = set()
    for i in range(mb.n_kernels):
        B.same(g[i], o[i], f"kernel {i} ({mb.kernels[i].name}, T={mb.kernels[i].meta['T']})")
        fams.add(mb.kernels[i].name)
    assert fams == {"f1_i32", "f1_i64", "f2_i32", "f2_i64", "f3_i32", "f3_i64"}


@pytest.mark.parametrize("use_graph", [False, True])
@pytest.mark.parametrize("sched,chunk,wg", [(ckc.SCHED_BLOCKED, 1, 0), (ckc.SCHED_CYCLIC, 1, 2),
                                            (ckc.SCHED_CYCLIC, 3, 0), (ckc.SCHED_DYNAMIC, 1, 4),
                                            (ckc.SCHED_DYNAMIC, 5, 1), (ckc.SCHED_LPT, 1, 0),
                                            (ckc.SCHED_LPT, 16, 8)])
def test_launch_options_do_not_change_results(ctx, mini, sched, chunk, wg, use_graph):
    mb, db = mini
    print(f"[case] schedule {sched} chunk {chunk} wg/cu {wg} graph {use_graph}", flush=True)
    ref = run_batch(ctx, db)
    for rep in range(2):  # a cached graph is replayed on the second pass
        g = run_batch(ctx, db, opts=ckc.launch_opts(sched, chunk, wg, use_graph=use_graph))
        for i in range(mb.n_kernels):
            B.same(g[i], ref[i], f"kernel {i} sched {sched} chunk {chunk} rep {rep}")


def test_alone_equals_in_batch(ctx, mini):
    mb, db = mini
    print("[case] alone vs in batch", flush=True)
    full = run_batch(ctx, db)
    rng = np.random.default_rng(5)
    for i in rng.choice(mb.n_kernels, size=16, replace=False):
        alone = run_batch(ctx, db, idx=[int(i)])[0]
        B.same(alone, full[int(i)], f"kernel {i} alone")


def test_enqueued_readback_equals_waiting_readback(ctx, mini):
    """Results read with CKC_ENQUEUE (copies queued behind the job, no host
    wait) equal a waiting readback, also when later jobs reuse the pool while
    earlier copies may still run."""
    import torch
    mb, db = mini
    print("[case] enqueued readback, 3 jobs in flight", flush=True)
    ref = run_batch(ctx, db)
    n = mb.n_kernels
    n_rec = sum(db.n_accesses(i) for i in range(n))
    outs = []
    for rep in range(3):
        o = dict(recs=torch.zeros(n_rec * 32, dtype=torch.uint8, device="cuda"),
                 maps=torch.zeros(n * 65536, dtype=torch.uint8, device="cuda"),
                 st=torch.zeros(n * 40, dtype=torch.uint8, device="cuda"))
        job = ctx.check(db.descs(), opts=ckc.launch_opts(use_graph=rep == 1))
        ctx.read_device(job, o["recs"].data_ptr(), o["maps"].data_ptr(), o["st"].data_ptr(), enqueue=True)
        outs.append(o)
    torch.cuda.synchronize()
    for rep, o in enumerate(outs):
        recs = np.frombuffer(o["recs"].cpu().numpy().tobytes(), ckc.RECORD_DTYPE)
        maps = o["maps"].cpu().numpy().reshape(n, 65536)
        st = np.frombuffer(o["st"].cpu().numpy().tobytes(), ckc.STATUS_DTYPE)
        g = ckc.split_results(recs, maps, st, [db.n_accesses(i) for i in range(n)])
        for i in range(n):
            B.same(g[i], ref[i], f"kernel {i} enqueued rep {rep}")


def test_enqueue_needs_device_destination(ctx, mini):
    """CKC_ENQUEUE with host destinations is rejected and leaves the job
    readable."""
    import ctypes
    mb, db = mini
    job = ctx.check(db.descs([0, 1]))
    ni, nr = ctx.sizes(job)
    recs = np.zeros(nr, ckc.RECORD_DTYPE)
    st = np.zeros(ni, ckc.STATUS_DTYPE)
    rc = ckc.lib().ckc_read_results(ctx.h, job, recs.ctypes.data_as(ctypes.c_void_p), None,
                                    st.ctypes.data_as(ctypes.c_void_p), ckc.WAIT | ckc.ENQUEUE)
    assert rc == -1
    out = ctx.read(job, maps=False)
    assert out is not None and int(out[2]["lanes"].sum()) > 0


def test_graph_timing_and_elapsed(ctx, mini):
    mb, db = mini
    job = ctx.check(db.descs(), opts=ckc.launch_opts(use_graph=True))
    assert ctx.timing(job) == [-1.0] * 5
    assert ctx.elapsed(job) > 0
    ctx.release(job)
    job = ctx.check(db.descs())
    t = ctx.timing(job)
    assert all(x >= 0 for x in t) and ctx.elapsed(job) >= max(t)
    ctx.release(job)


def test_autotune(ctx, mini):
    mb, db = mini
    print("[case] autotune", flush=True)
    prep = ckc.Context.prepare(db.descs())
    best, log = ctx.autotune(prep, reps=1)
    assert len(log) == 50
    assert all(ms > 0 for _, ms in log)
    assert best.as_dict() in [d for d, _ in log]
    assert min(ms for _, ms in log) == [ms for d, ms in log if d == best.as_dict()][0]
    ref = run_batch(ctx, db)
    g = run_batch(ctx, db, opts=best)
    for i in range(mb.n_kernels):
        B.same(g[i], ref[i], f"kernel {i} tuned")


def test_full_config4_sampled(ctx):
    """The full batch (10,000 kernels, ~59 M threads) in one job; the oracle
    checks a sample of 300 kernels, every kernel's thread count is checked."""
    mb = W.config4()
    print(f"[case] config4 full, {mb.n_kernels} kernels", flush=True)
    db = ckc.DeviceBatch(ctx, mb)
    try:
        g = run_batch(ctx, db, opts=ckc.launch_opts(use_graph=True))
    finally:
        db.close()
    lanes = np.array([int(np.prod(k.launch[0].astype(np.int64))) for k in mb.kernels])
    np.testing.assert_array_equal(np.array([int(r["status"]["lanes"]) for r in g]), lanes)
    idx = np.random.default_rng(7).choice(mb.n_kernels, size=300, replace=False)
    o = B.oracle_mixed(mb, idx=idx, nthreads=NCPU)
    for j, i in enumerate(idx):
        B.same(g[int(i)], o[j], f"kernel {i}")
