"""GPU parity: the HIP library against the oracle, element by element (records,
dense coverage maps, per-input status), through the C-ABI.  Integer work, so
the bar is bit-exact."""
import os

import numpy as np
import pytest

import kernels as K
import randprog as R
from oracle import oracle as O
from paper_2601_01048_amd import ckc
from paper_2601_01048_amd.gen import workloads as W
from paper_2601_01048_amd.gen.ir import Program

pytestmark = pytest.mark.gpu

NCPU = max(1, min(16, os.cpu_count() or 1))


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    c = ckc.Context(0)
    yield c
    c.close()


def compare(gpu, ora, n=None, maps=True, what=""):
    n = gpu["records"].shape[0] if n is None else n
    g, o = gpu["records"][:n], ora["records"][:n]
    for f in ("first_key", "count", "kinds", "index", "first_kind"):
        bad = np.nonzero(g[f] != o[f])
        if bad[0].size:
            i, a = int(bad[0][0]), int(bad[1][0])
            raise AssertionError(f"{what}: field {f} differs at {bad[0].size} records; first "
                                 f"(input {i}, access {a}): gpu {g[i, a]} oracle {o[i, a]}")
    for f in ("lanes", "accesses_checked", "hang_lanes", "arith_faults", "flags"):
        np.testing.assert_array_equal(gpu["status"][f][:n], ora["status"][f][:n], err_msg=f"{what} {f}")
    if maps:
        bad = np.nonzero(gpu["maps"][:n] != ora["maps"][:n])
        assert bad[0].size == 0, (what, "maps", bad[0][:5], bad[1][:5])


def both(ctx, wl, mode=None, force_generic=False, cap=None, nthreads=NCPU):
    print(f"[case] {wl.name} mode={mode} generic={force_generic} n={wl.n_inputs}", flush=True)
    g = ckc.run_workload(ctx, wl, mode=mode, force_generic=force_generic, cap_log2=cap)
    o = O.check(wl, mode=mode, cap_log2=cap, nthreads=nthreads)
    return g, o


@pytest.mark.parametrize("generic", [False, True])
@pytest.mark.parametrize("mode", [W.MODE_FULL, W.MODE_CORNERS, W.MODE_BOUNDARY])
@pytest.mark.parametrize("name,w", [("config1", 32), ("config1", 64), ("config2", 32), ("config2", 64),
                                    ("config3", 32), ("config3", 64)])
def test_mini_configs(ctx, name, w, mode, generic):
    wl = W.mini(name, w=w)
    g, o = both(ctx, wl, mode, generic)
    compare(g, o, what=f"{name} i{w} mode {mode} generic {generic}")


@pytest.mark.parametrize("generic", [False, True])
def test_listings(ctx, generic):
    LB = W.LOGICAL_BASE
    for N, bs in ((1023, 256), (1000, 256), (77, 8)):
        grid = -(-N // bs)
        wl = K.simple_workload(K.listing3_program(), [[grid, 1, 1, bs, 1, 1]], [[(LB, N * 4, 0, 0, 0)] * 3],
                               scalars=[[N]])
        g, o = both(ctx, wl, None, generic)
        compare(g, o, what=f"listing3 N={N}")
        assert list(g["records"]["first_key"][0]) == [N - 1] * 3
    ir = K.listing1_program()
    for n_el in (40, 39):
        tables = [[(LB, 32, 0, 0, 0), (LB, 32, 0, 0, 0)] + [(LB, n_el * 4, 0, 0, 0)] * 3]
        wl = K.simple_workload(ir, [[5, 1, 1, 8, 1, 1]], tables)
        g, o = both(ctx, wl, None, generic)
        compare(g, o, what="listing1")


@pytest.mark.parametrize("generic", [False, True])
def test_integer_semantics(ctx, generic):
    from test_oracle import OPS
    vals = [0, 1, -1, 3, -7, 31, 32, 63, 64, -(1 << 31), (1 << 31) - 1, -(1 << 63), (1 << 63) - 1, 1 << 40]
    for op in OPS:  # one program per op keeps each within the IR limits
        p = Program(n_scalars=0, n_slots=1)
        for w in (32, 64):
            for a in vals:
                for b in vals[::3]:
                    p.access(0, p.op(op, p.const(a, w), p.const(b, w), w), w=64, site=False)
        wl = K.simple_workload(p.to_bytes(), [[1, 1, 1, 2, 1, 1]], [[(0, 0, 0, 0, 0)]])
        g, o = both(ctx, wl, None, generic)
        compare(g, o, what=f"alu {op}")


@pytest.mark.parametrize("generic", [False, True])
def test_thread_dependent_alu(ctx, generic):
    """Every op on thread-dependent operands (generic path; exposes values as
    NULL-slot indices, one record per op, first key = thread 0)."""
    from test_oracle import OPS
    p = Program(n_scalars=1, n_slots=2)
    t = p.special("tid.x")
    b = p.special("bid.y")
    s = p.scalar(0, 64)
    for w in (32, 64):
        x = p.sub(p.mul(t, p.const(0x12345679, w), w), s, w)
        y = p.add(b, p.const(-3, w), w)
        for op in OPS:
            p.access(0, p.op(op, x, y, w), w=64)
            p.access(1, p.op(op, y, x, w), w=w)
    wl = K.simple_workload(p.to_bytes(), [[1, 3, 1, 64, 1, 1], [2, 2, 1, 33, 1, 1]],
                           [[(0, 0, 0, 0, 0), (W.LOGICAL_BASE, 400, 0, 0, 0)]] * 2,
                           scalars=[[7], [-(1 << 35)]])
    g, o = both(ctx, wl, None, generic)
    compare(g, o, what="alu-varying")


def test_loops_and_caps(ctx):
    p = Program(n_scalars=4, n_slots=1)
    s0, e0, st0, e1 = (p.scalar(k, 32) for k in range(4))
    with p.loop(s0, e0, st0, w=32) as i:
        with p.loop(0, e1, 1, w=32) as j:
            p.access(0, p.add(p.mul(i, p.const(100, 32), 32), j, 32), w=32)
    cases = [(0, 10, 3, 2), (10, 0, -3, 1), (5, 5, 1, 3), (-7, 7, 4, 0), (2, -(1 << 31), -(1 << 30), 1),
             (0, 1 << 30, 1, 2), (0, 5, 0, 1)]
    wl = K.simple_workload(p.to_bytes(), [[2, 1, 1, 3, 1, 1]] * len(cases), [[(W.LOGICAL_BASE, 64, 0, 0, 0)]] * len(cases),
                           scalars=np.array(cases, np.int64), cap=(6, 4))
    for generic in (False, True):
        g, o = both(ctx, wl, None, generic)
        compare(g, o, what=f"loops generic={generic}")


def test_special_registers(ctx):
    p = Program(n_scalars=0, n_slots=1)
    for nm in R.SPECIALS:
        p.access(0, p.special(nm), w=64)
    wl = K.simple_workload(p.to_bytes(), [[2, 3, 4, 5, 2, 3], [1, 1, 1, 1, 1, 1], [3, 1, 2, 7, 1, 1]],
                           [[(W.LOGICAL_BASE, 8, 0, 0, 0)]] * 3)
    for mode in (W.MODE_FULL, W.MODE_CORNERS, W.MODE_BOUNDARY):
        for generic in (False, True):
            g, o = both(ctx, wl, mode, generic)
            compare(g, o, what=f"specials {mode} {generic}")


def test_boundary_shapes(ctx):
    """Boundary thread sets over many 3-D grid shapes (degenerate dimensions
    included), for block sizes that take the block-major and the lane-tiled
    trace layouts and for the interpreter."""
    rng = np.random.default_rng(7)
    p = Program(n_scalars=0, n_slots=2)
    for nm in R.SPECIALS[:6]:
        p.access(0, p.special(nm), w=64)
    g = p.add(p.mul(p.special("bid.x"), p.special("bdim.x"), 32), p.special("tid.x"), 32)
    p.access(1, p.add(g, p.mul(p.special("bid.y"), 3, 32), 32))
    ir = p.to_bytes()
    launches = []
    for blk in ((64, 1, 1), (16, 4, 1), (8, 2, 1), (32, 2, 2), (3, 1, 1)):
        for _ in range(6):
            launches.append([int(v) for v in rng.integers(1, 6, size=3)] + list(blk))
    tables = [[(W.LOGICAL_BASE, 8, 0, 0, 0), (W.LOGICAL_BASE, 4 * 200, 0, 0, 0)]] * len(launches)
    wl = K.simple_workload(ir, launches, tables, mode=W.MODE_BOUNDARY)
    for mode in (W.MODE_BOUNDARY, W.MODE_FULL, W.MODE_CORNERS):
        for generic in (False, True):
            gg, o = both(ctx, wl, mode, generic)
            compare(gg, o, what=f"boundary shapes mode {mode} generic {generic}")


def test_empty_and_degenerate(ctx):
    wl = K.simple_workload(K.listing3_program(), [[0, 1, 1, 32, 1, 1], [1, 1, 1, 1, 1, 1], [3, 0, 1, 4, 1, 1]],
                           [[(W.LOGICAL_BASE, 4, 0, 0, 0)] * 3] * 3, scalars=[[5], [5], [5]])
    for generic in (False, True):
        g, o = both(ctx, wl, None, generic)
        compare(g, o, what="empty")


@pytest.mark.parametrize("seed", range(6))
def test_random_programs(ctx, seed):
    rng = np.random.default_rng(100 + seed)
    for k in range(25):
        ir = R.random_program(rng, uniform_only=(k % 3 == 0))
        for mode in (W.MODE_FULL, W.MODE_CORNERS, W.MODE_BOUNDARY):
            wl = R.random_workload(rng, ir, mode=mode)
            for generic in (False, True):
                g = ckc.run_workload(ctx, wl, force_generic=generic)
                o = O.check(wl)
                compare(g, o, what=f"seed {seed} prog {k} mode {mode} generic {generic} ir {ir.hex()}")


# ---------------------------------------------------------------------------
# full sizes (the configurations the benchmark times)
# ---------------------------------------------------------------------------
def test_config1_full(ctx):
    wl = W.config1()
    g, o = both(ctx, wl)
    compare(g, o, what="config1 full")


@pytest.mark.parametrize("mode", [W.MODE_FULL, W.MODE_BOUNDARY])
def test_config2_full_sampled(ctx, mode):
    """All 4096 inputs on the GPU in one job; the oracle recomputes a spread
    sample of inputs one by one."""
    wl = W.config2(mode=mode)
    print("[case] config2 full on GPU", flush=True)
    g = ckc.run_workload(ctx, wl)
    sample = np.array([0, 1, 777, 2048, 3001, 4095])
    o = O.check(wl.subset(sample), nthreads=NCPU)
    sub = dict(records=g["records"][sample], maps=g["maps"][sample], status=g["status"][sample])
    compare(sub, o, what="config2 sample")
    # properties at every input: 10 accesses per thread in the thread set
    lanes = g["status"]["lanes"].astype(np.int64)
    np.testing.assert_array_equal(g["status"]["accesses_checked"], 10 * lanes)
    if mode == W.MODE_FULL:
        np.testing.assert_array_equal(lanes, wl.launch[:, 0].astype(np.int64) * wl.launch[:, 1] * 256)


def test_config3_full_sampled(ctx):
    wl = W.config3(n_inputs=8)
    print("[case] config3 full (8 inputs) on GPU", flush=True)
    g = ckc.run_workload(ctx, wl)
    from test_oracle import f3_numpy
    for i in range(wl.n_inputs):
        cnt, fk, fi, kinds = f3_numpy(wl, i)
        r = g["records"][i, 4]
        assert (int(r["count"]), int(r["first_key"]), int(r["kinds"])) == (cnt, fk, kinds), i
        if cnt:
            assert int(r["index"]) == fi
    o = O.check(wl.subset([0, 7]), nthreads=2)
    sub = dict(records=g["records"][[0, 7]], maps=g["maps"][[0, 7]], status=g["status"][[0, 7]])
    compare(sub, o, what="config3 sample")


@pytest.mark.parametrize("k_bx", R.GRID_STEPS)
def test_affine_grid_groups(ctx, k_bx):
    """Block-major trace evaluator over grids of 16 to 70 blocks per row: whole
    groups of 16 blocks in one row whose block bases step by k_bx (the
    two-end test applies while 15*|k_bx| < 2^31, the largest such step and
    the next are both here), groups across rows, a short last group, bounds
    anywhere in the index range, freed and NULL slots; every record, map and
    status against the oracle."""
    rng = np.random.default_rng(4000 + R.GRID_STEPS.index(k_bx))
    for k in range(3):
        ir = R.affine_grid_program(rng, k_bx)
        wl = R.affine_grid_workload(rng, ir, k_bx)
        g, o = both(ctx, wl)
        compare(g, o, what=f"affine grid k_bx {k_bx} prog {k} ir {ir.hex()}")
