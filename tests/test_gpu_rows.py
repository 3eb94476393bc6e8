"""The whole-thread pass's rows form (the part of a program around an
expanded gather loop reduced per input to affine forms and run with no
instruction dispatch) against the oracle on random programs of that shape:
affine thread-coordinate forms at both widths, one level of IF guards with
every comparison, loads feeding the loop bounds and other indices, steps of
1, 2 and -1, loops over the trip cap (hangs), accesses before and after the
loop, two-dimensional blocks, and near misses the device walk hands back to
the interpreter.  Records, dense maps and status byte for byte, in the whole
grid, the boundary set and the corner set."""
import os

import numpy as np
import pytest

import rowsprog as RP
from oracle import oracle as O
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


def check_same(ctx, wl, mode=None, what=""):
    print(f"[case] rows {what} mode={wl.mode if mode is None else mode} inputs={wl.n_inputs}", flush=True)
    g = ckc.run_workload(ctx, wl, mode=mode)
    o = O.check(wl, mode=mode, nthreads=NCPU)
    for f in ("first_key", "index", "count", "kinds", "first_kind"):
        assert np.array_equal(g["records"][f], o["records"][f]), (what, f)
    assert np.array_equal(g["maps"], o["maps"]), what
    for f in ("lanes", "accesses_checked", "hang_lanes", "arith_faults", "flags"):
        assert np.array_equal(g["status"][f], o["status"][f]), (what, f)
    return g, o


@pytest.mark.parametrize("seed", range(12))
def test_random_rows_programs(ctx, seed):
    rng = np.random.default_rng(4000 + seed)
    for k in range(4):
        near = k == 3
        ir = RP.rows_program(rng, near_miss=near)
        cap = (2, 12) if (seed + k) % 3 == 0 else (20, 12)
        wl = RP.rows_workload(rng, ir, cap=cap)
        for mode in (W.MODE_FULL, W.MODE_BOUNDARY, W.MODE_CORNERS):
            check_same(ctx, wl, mode=mode, what=f"{seed}.{k}{' near' if near else ''} cap={cap[0]}")


def test_csr_batch_rows_form(ctx):
    """The CSR configuration's program (guard, two row-pointer loads, the
    gather loop, y[r]) at both widths, whole grid."""
    for w in (32, 64):
        check_same(ctx, W.mini("config3", w=w), what=f"csr i{w}")


@pytest.mark.parametrize("cap", [(20, 12), (4, 12)])
def test_rows_32bit_extremes(ctx, cap):
    """The 32-bit evaluation of the rows form at the ends of the int32 range:
    loop bounds loaded near INT32_MIN and INT32_MAX (short spans there, spans
    across the whole range that exceed the trip cap, reversed bounds), and an
    index that wraps modulo 2^32 to either sign.  The program is all 32-bit,
    so the rows kernel takes its 32-bit path; checked against the oracle in the
    whole grid and the boundary set."""
    rng = np.random.default_rng(77 + cap[0])
    ir = RP.extreme_rows_program()
    wl = RP.extreme_rows_workload(rng, ir)
    wl.cap_log2 = cap
    for mode in (W.MODE_FULL, W.MODE_BOUNDARY):
        g, o = check_same(ctx, wl, mode=mode, what=f"extremes cap={cap[0]}")
        assert int(o["status"]["hang_lanes"].sum()) > 0
        assert int(o["records"]["count"].sum()) > 0


def test_mixed_width_rows_batch(ctx):
    """One job of two programs that both take the rows form, one all 32-bit
    (the CSR program) and one with 64-bit entries: the job runs the general
    rows kernel, which evaluates the first in 32-bit arithmetic and the
    second in 64-bit.  Each workload's records, maps and status against the
    oracle."""
    rng = np.random.default_rng(4100)
    ir64 = None
    for _ in range(400):
        ir = RP.rows_program(rng)
        if ckc.analyze(ir)[0]["rows_form"] == 1:
            ir64 = ir
            break
    assert ir64 is not None
    wls = [W.mini("config3", w=32), RP.rows_workload(rng, ir64)]
    assert ckc.analyze(wls[0].ir)[0]["rows_form"] == 2
    print(f"[case] rows mixed widths inputs={[wl.n_inputs for wl in wls]}", flush=True)
    dws = [ckc.DeviceWorkload(ctx, wl) for wl in wls]
    try:
        job = ctx.check([dw.desc() for dw in dws])
        recs, mp, st = ctx.read(job)
        n_acc = [dw.info["n_accesses"] for dw in dws]
    finally:
        for dw in dws:
            dw.close()
    r0 = i0 = 0
    for k, (wl, na) in enumerate(zip(wls, n_acc)):
        n = wl.n_inputs
        o = O.check(wl, nthreads=NCPU)
        g = recs[r0:r0 + n * na].reshape(n, na)
        for f in ("first_key", "index", "count", "kinds", "first_kind"):
            assert np.array_equal(g[f], o["records"][f]), (k, f)
        assert np.array_equal(mp[i0:i0 + n], o["maps"]), k
        for f in ("lanes", "accesses_checked", "hang_lanes", "arith_faults", "flags"):
            assert np.array_equal(st[i0:i0 + n][f], o["status"][f]), (k, f)
        r0 += n * na
        i0 += n
