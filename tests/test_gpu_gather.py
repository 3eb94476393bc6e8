"""GPU parity of expanded loops evaluated as gathers (entries built once per
input) and of their near misses (interpreted), against the oracle."""
import numpy as np
import pytest

import gatherprog as G
from oracle import oracle as O
from paper_2601_01048_amd import ckc

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    c = ckc.Context(0)
    yield c
    c.close()


@pytest.mark.parametrize("seed", range(4))
def test_random_gather_bodies(ctx, seed):
    from test_gpu_parity import compare
    rng = np.random.default_rng(500 + seed)
    n_gather = 0
    for k in range(30):
        ir = G.gather_program(rng, near_miss=(k % 5 == 4))
        info, _ = ckc.analyze(ir)
        n_gather += bool(info["cls"] & ckc.CLS["GATHER"])
        wl = G.gather_workload(rng, ir)
        print(f"[case] seed {seed} prog {k} cls {info['cls']}", flush=True)
        g = ckc.run_workload(ctx, wl)
        o = O.check(wl)
        compare(g, o, what=f"gather seed {seed} prog {k} ir {ir.hex()}")
    assert n_gather > 0


@pytest.mark.parametrize("schedule,wg,log2_rows", [(ckc.SCHED_DEFAULT, 1, 15), (ckc.SCHED_DEFAULT, 0, 15),
                                                   (ckc.SCHED_DYNAMIC, 1, 15), (ckc.SCHED_CYCLIC, 2, 15),
                                                   (ckc.SCHED_DEFAULT, 1, 13)])
def test_gather_tile_runs(ctx, schedule, wg, log2_rows):
    """Runs of chained contiguous tiles in the gather pass: broken chains,
    empty tiles, tiles that are not contiguous, violations in late tiles of a
    run; few workgroups, so that each takes many pieces.  Inputs of 128 tiles
    take the gather pass with 16-chunk rounds, inputs of 32 tiles the one
    without."""
    from test_gpu_parity import compare
    wl = G.csr_runs_workload(11, log2_rows=log2_rows)
    print(f"[case] csr runs schedule {schedule} wg_per_cu {wg} rows 2^{log2_rows}", flush=True)
    g = ckc.run_workload(ctx, wl, opts=ckc.launch_opts(schedule=schedule, wg_per_cu=wg))
    o = O.check(wl, nthreads=4)
    compare(g, o, what=f"csr runs schedule {schedule} wg {wg}")
    assert (o["records"]["count"][:, 3] > 0).all() and (o["records"]["count"][:, 4] > 100).all()


@pytest.mark.parametrize("col_short", [1, 5000])
def test_gather_runs_loaded_index_out_of_bounds(ctx, col_short):
    """Runs of chained tiles whose loaded array (col_idx) ends before the last
    nonzeros: the rounds that reach its end cannot stream it unchecked (the
    next round's loads are issued early only while every index of the run's
    whole rounds is in bounds), and its out-of-bounds indices are violations
    with nothing loaded."""
    from test_gpu_parity import compare
    wl = G.csr_runs_workload(13, log2_rows=15, col_short=col_short)
    print(f"[case] csr runs col_short {col_short}", flush=True)
    g = ckc.run_workload(ctx, wl)
    o = O.check(wl, nthreads=4)
    compare(g, o, what=f"csr runs col_short {col_short}")
    assert (o["records"]["count"][:, 2] == col_short).all()  # the last col_short nonzeros


@pytest.mark.parametrize("big", [False, True])
@pytest.mark.parametrize("seed", range(3))
def test_long_gather_rounds(ctx, seed, big):
    """Whole rounds of the contiguous form over random 32-bit gather bodies:
    loads of int32 and int64 data by the counter (in bounds for the whole
    round or not), by a loaded value or a constant, second loads, checks of
    freed and NULL slots.  Inputs of 2 tiles take the gather kernel with
    8-chunk rounds, inputs of 64 tiles the one with 16-chunk rounds; one
    workgroup per compute unit gives each workgroup several pieces."""
    from test_gpu_parity import compare
    rng = np.random.default_rng(900 + seed + 10 * big)
    for k in range(8):
        ir = G.long_gather_program(rng)
        info, _ = ckc.analyze(ir)
        assert info["cls"] & ckc.CLS["GATHER"]
        wl = G.long_gather_workload(rng, ir, blocks=64 if big else 2, L_range=(16, 24) if big else (40, 100))
        o = O.check(wl, nthreads=4)
        for wg in (1, 0):
            print(f"[case] long gather seed {seed} big {big} prog {k} wg_per_cu {wg}", flush=True)
            g = ckc.run_workload(ctx, wl, opts=ckc.launch_opts(wg_per_cu=wg))
            compare(g, o, what=f"long gather seed {seed} big {big} prog {k} wg {wg} ir {ir.hex()}")
