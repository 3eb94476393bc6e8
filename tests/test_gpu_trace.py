"""GPU parity of the block-major trace evaluator in its two whole-grid forms:
CKC_FULL (every index formed and compared) and CKC_FULL_ENDPOINTS (rows of
blocks decided by the end indices of their progressions), against the
oracle's whole-grid result, bit for bit; plus 3-D grids, row segments of
jobs at and past the 2^31 span guard, and violations at interior segment
ends."""
import os

import numpy as np
import pytest

import randprog as R
from oracle import oracle as O
from paper_2601_01048_amd import ckc
from paper_2601_01048_amd.gen import workloads as W
from test_gpu_parity import compare

pytestmark = pytest.mark.gpu

NCPU = max(1, min(16, os.cpu_count() or 1))
WHOLE = (W.MODE_FULL, W.MODE_ENDPOINTS)


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    c = ckc.Context(0)
    yield c
    c.close()


def check(ctx, wl, mode, what):
    print(f"[case] {what} mode={mode} n={wl.n_inputs}", flush=True)
    g = ckc.run_workload(ctx, wl, mode=mode)
    o = O.check(wl, mode=W.MODE_FULL if mode == W.MODE_ENDPOINTS else mode, nthreads=NCPU)
    compare(g, o, what=f"{what} mode {mode}")
    return g


@pytest.mark.parametrize("name,w", [("config1", 32), ("config1", 64), ("config2", 32), ("config2", 64),
                                    ("config3", 32)])
def test_endpoints_mini_configs(ctx, name, w):
    wl = W.mini(name, w=w)
    check(ctx, wl, W.MODE_ENDPOINTS, f"mini {name} i{w}")


@pytest.mark.parametrize("mode", WHOLE)
@pytest.mark.parametrize("k_bx", R.GRID_STEPS)
def test_affine_grid_groups_both(ctx, k_bx, mode):
    rng = np.random.default_rng(4000 + R.GRID_STEPS.index(k_bx))
    for k in range(3):
        ir = R.affine_grid_program(rng, k_bx)
        wl = R.affine_grid_workload(rng, ir, k_bx)
        check(ctx, wl, mode, f"affine grid k_bx {k_bx} prog {k}")


SEG_STEPS = [1, 16, -16, 4096, (1 << 31) // 126, (1 << 31) // 126 + 1, -((1 << 31) // 126) - 1,
             (1 << 31) // 69 + 1]


@pytest.mark.parametrize("mode", WHOLE)
@pytest.mark.parametrize("k_bx", SEG_STEPS)
def test_row_segments(ctx, k_bx, mode):
    """Jobs of 256 blocks over rows of 70..127 blocks: 3 or 4 row segments per
    job, segment spans at and past 2^31, bounds that put the only violations
    at a row end inside a job."""
    rng = np.random.default_rng(5000 + SEG_STEPS.index(k_bx))
    for k_by in (0, -(abs(k_bx) * 64), 3 * abs(k_bx) + 1):
        ir = R.segment_program(k_bx, k_by)
        wl = R.segment_workload(rng, ir, k_bx, k_by)
        g = check(ctx, wl, mode, f"segments k_bx {k_bx} k_by {k_by}")
        assert g["records"]["count"].sum() >= 0


@pytest.mark.parametrize("mode", WHOLE + (W.MODE_BOUNDARY, W.MODE_CORNERS))
def test_grid3d(ctx, mode):
    """One coefficient class over 3-D grids and 16x2x2 blocks (tid.z and bid.z
    coefficients nonzero): the block-major walk across x, y and z wraps."""
    rng = np.random.default_rng(6000)
    for k in range(4):
        ir = R.grid3d_program(rng)
        wl = R.grid3d_workload(rng, ir)
        check(ctx, wl, mode, f"grid3d prog {k}")


def test_endpoints_config2_equals_full(ctx):
    """The benchmark batch: both whole-grid forms give identical bytes."""
    wl = W.config2(mode=W.MODE_FULL)
    a = ckc.run_workload(ctx, wl, mode=W.MODE_FULL)
    b = ckc.run_workload(ctx, wl, mode=W.MODE_ENDPOINTS)
    for f in ("first_key", "index", "count", "kinds", "first_kind"):
        np.testing.assert_array_equal(a["records"][f], b["records"][f], err_msg=f)
    np.testing.assert_array_equal(a["maps"], b["maps"])
    for f in ("lanes", "accesses_checked", "hang_lanes", "arith_faults", "flags"):
        np.testing.assert_array_equal(a["status"][f], b["status"][f], err_msg=f)
