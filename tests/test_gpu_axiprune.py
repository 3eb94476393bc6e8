"""Pruned programs (the paper's AXIPrune, Section 5.2) on the GPU against the
oracle, which runs every program as written: kernels with shared memory and
barriers run block by block in the interpreter (blocks of a tile share their
instance in LDS), first violations whose indices read shared memory come from
the capture pass, data math no index reads is dropped.  Every kernel is also
loaded unpruned, which must give the same bytes.  Records, dense maps and
status are compared byte for byte; refusals of launches the blockwise
evaluation cannot take are checked too."""
import os

import numpy as np
import pytest

import sharedprog as SP
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


def check_same(ctx, wl, mode=None, no_prune=False, what=""):
    print(f"[case] axiprune {what} mode={wl.mode if mode is None else mode} no_prune={no_prune} "
          f"inputs={wl.n_inputs}", flush=True)
    g = ckc.run_workload(ctx, wl, mode=mode, no_prune=no_prune)
    o = O.check(wl, mode=mode, nthreads=NCPU)
    for f in ("first_key", "index", "count", "kinds", "first_kind"):
        assert np.array_equal(g["records"][f], o["records"][f]), (what, f)
    assert np.array_equal(g["maps"], o["maps"]), what
    for f in ("lanes", "accesses_checked", "hang_lanes", "arith_faults", "flags"):
        assert np.array_equal(g["status"][f], o["status"][f]), (what, f)
    return g, o


SHARED = {"rotate": SP.rotate, "rotate3d": lambda: SP.rotate(dims=3), "rotate_neg": lambda: SP.rotate(k=-5, c=40),
          "racing_max": SP.racing_max, "phases": SP.phases, "shared_divisor": SP.shared_divisor,
          "bounds": SP.bounds, "bounds_up": lambda: SP.bounds(off=2), "tile_gather": SP.tile_gather,
          "prefix_max": SP.prefix_max, "hist_like": SP.hist_like}
BLOCKS_1D = [(1, 1, 1), (8, 1, 1), (32, 1, 1), (64, 1, 1), (128, 1, 1), (256, 1, 1)]
BLOCKS_3D = [(2, 2, 2), (4, 4, 2), (8, 4, 2), (8, 8, 4)]
GRIDS = [(1, 1, 1), (5, 1, 1), (3, 2, 1), (40, 1, 1), (2, 2, 3)]


def shared_workload(name, rng, mode=W.MODE_FULL):
    """The kernel over every block shape and grid, with shared arrays that
    fit the tile (a tile of 256 threads holds 256 / bs blocks, 12 bytes of
    LDS per element of each) and are sometimes smaller than the block."""
    case = SHARED[name]()
    blocks = BLOCKS_3D if name == "rotate3d" else BLOCKS_1D
    if name == "prefix_max":
        blocks = [b for b in blocks if b[0] >= 32]
    launches, tables = [], []
    for bs in blocks:
        n = bs[0] * bs[1] * bs[2]
        cap = 16 * n  # elements per block that fit the tile's LDS
        for g in GRIDS:
            launches.append(list(g) + list(bs))
            na = int(rng.integers(20, 700))
            lo = 8 if name != "prefix_max" else 256
            ns = int(rng.integers(min(lo, cap), min(cap, 600) + 1))
            tab = [(SP.LB + 4096, 4 * na, 0, 0, 0), (SP.SH_BASE, 4 * ns, 0, 0, 0)]
            if len(case.spaces) > 2:
                tab.append((SP.LB + (1 << 24), 4 * 8192, 1, 0, 0))
            tables.append(tab)
    data = [SP.data_array(rng)]
    return case, SP.workload(case, launches, tables, data=data, mode=mode)


@pytest.mark.parametrize("name", list(SHARED))
@pytest.mark.parametrize("no_prune", [False, True])
def test_shared_kernels(ctx, name, no_prune):
    rng = np.random.default_rng(100 + list(SHARED).index(name))
    for mode in (W.MODE_FULL, W.MODE_BOUNDARY):
        case, wl = shared_workload(name, rng, mode)
        g, o = check_same(ctx, wl, no_prune=no_prune, what=name)
    if name in ("rotate", "racing_max", "phases", "bounds", "prefix_max"):
        assert int(o["records"]["count"].sum()) > 0


def test_large_grid_capture(ctx):
    """4096 blocks of 256 threads whose indices read shared memory: the
    first violations (found by the capture pass) and every count."""
    case = SP.rotate(k=3, c=-7)
    launches = [[4096, 1, 1, 256, 1, 1], [1000, 3, 1, 64, 1, 1]]
    tables = [[(SP.LB + 4096, 4 * 700, 0, 0, 0), (SP.SH_BASE, 4 * 256, 0, 0, 0)],
              [(SP.LB + 4096, 4 * 150, 0, 0, 0), (SP.SH_BASE, 4 * 60, 0, 0, 0)]]
    check_same(ctx, SP.workload(case, launches, tables), what="rotate large")


@pytest.mark.parametrize("no_prune", [False, True])
def test_fp_kernels(ctx, no_prune):
    """ep-like (an FP chain no index reads, an index through FP) and
    FP arithmetic into indices, over large grids; FTOI's special values."""
    ep = SP.ep_like()
    launches = [[2048, 1, 1, 256, 1, 1], [37, 1, 1, 96, 1, 1]]
    tables = [[(SP.LB + 4096, 4 * 190000, 0, 0, 0), (SP.LB + (1 << 24), 4 * 500000, 0, 0, 0)]] * 2
    check_same(ctx, SP.workload(ep, launches, tables), no_prune=no_prune, what="ep_like")
    fa = SP.fp_arith()
    check_same(ctx, SP.workload(fa, [[64, 1, 1, 128, 1, 1]], [[(SP.LB + 4096, 4 * 300, 0, 0, 0)]]),
               no_prune=no_prune, what="fp_arith")
    consts = [float("nan"), float("inf"), -float("inf"), 1e20, -1e20, 2147483647.5, 2147483648.0,
              -2147483648.5, -2147483649.0, 9.3e18, -9.3e18, -2.9, 2.9, -0.0, 5e-324, 17.999999999]
    fi = SP.fp_index(consts)
    check_same(ctx, SP.workload(fi, [[1, 1, 1, 2, 1, 1]], [[(SP.LB + 4096, 64, 0, 0, 0)]],
                                scalars=[[SP.f2bits(c) for c in consts]]), no_prune=no_prune, what="ftoi")


def test_fexp_bits(ctx):
    """FEXP gives the oracle's bits on the device over the whole range
    (subnormal results included): e^x is scaled by powers of two (exact) to
    about [2^61, 2^62) and converted to an int64 index, which holds every bit of the
    result; slot A is NULL, so every index is recorded."""
    import math

    import kernels as K
    from paper_2601_01048_amd.gen.ir import Program
    rng = np.random.default_rng(11)
    xs = np.concatenate([rng.uniform(-745.0, 709.78, 1500), rng.uniform(-2, 2, 1500),
                         rng.uniform(-745.13, -708.0, 500)])
    p = Program(n_scalars=3, n_slots=1)
    y = p.fop("FMUL", p.fop("FMUL", p.fop("FEXP", p.scalar(0, 64)), p.scalar(1, 64)), p.scalar(2, 64))
    p.access(0, p.ftoi(y, 64), w=64, elem=1)
    scal = []
    for v in xs:
        e = 61 - math.floor(float(v) / math.log(2))
        e1 = min(e, 1000)
        scal.append([SP.f2bits(float(v)), SP.f2bits(2.0 ** e1), SP.f2bits(2.0 ** (e - e1))])
    n = len(xs)
    wl = K.simple_workload(p.to_bytes(), [[1, 1, 1, 1, 1, 1]] * n, [[(0, 1 << 20, 0, 0, 0)]] * n, scalars=scal)
    g, o = check_same(ctx, wl, what="fexp")
    assert np.all(o["records"]["count"] == 1)
    idx = o["records"]["index"][:, 0].astype(np.int64)
    assert np.all((idx >= 1 << 59) & (idx < (1 << 63) - 1))  # at least 59 bits: every bit of the double


def test_prex_and_corners(ctx):
    """PREX runs kernels that run block by block when their indices do not
    read shared memory (shared_divisor); a kernel that needs no block (the
    histogram, pruned) takes the corner threads and PREX; unpruned it needs its
    blocks and the corner set is refused, as is PREX when indices read shared
    memory."""
    rng = np.random.default_rng(5)
    for name, mode in (("shared_divisor", W.MODE_PREX), ("hist_like", W.MODE_CORNERS), ("hist_like", W.MODE_PREX)):
        case, wl = shared_workload(name, rng, mode)
        check_same(ctx, wl, what=name)
    _, wl = shared_workload("hist_like", rng, W.MODE_CORNERS)
    with pytest.raises(ckc.CkcError) as e:
        ckc.run_workload(ctx, wl, no_prune=True)
    assert e.value.code == -1
    _, wl = shared_workload("rotate", rng, W.MODE_PREX)
    with pytest.raises(ckc.CkcError) as e:
        ckc.run_workload(ctx, wl)
    assert e.value.code == -1


def test_blockwise_launch_refusals(ctx):
    """Blocks that do not divide the 256-thread tile, and shared memory of
    one tile's blocks above 48 KiB, are refused with CKC_E_INVALID."""
    case = SP.rotate()
    for launch, sh in (([2, 1, 1, 48, 1, 1], 64), ([2, 1, 1, 512, 1, 1], 64), ([4, 1, 1, 16, 1, 1], 300)):
        wl = SP.workload(case, [launch], [[(SP.LB + 4096, 400, 0, 0, 0), (SP.SH_BASE, 4 * sh, 0, 0, 0)]])
        with pytest.raises(ckc.CkcError) as e:
            ckc.run_workload(ctx, wl)
        assert e.value.code == -1, launch


def test_unpruned_load_keeps_everything(ctx):
    """The live count of the unpruned load is the program's length; pruned,
    the ep-like chain goes."""
    ep = SP.ep_like()
    pid, info = ctx.load_program(ep.ir, no_prune=True)
    ctx.unload_program(pid)
    assert info["n_instr_live"] == ep.n_instr
    pid, info = ctx.load_program(ep.ir)
    ctx.unload_program(pid)
    assert info["n_instr_live"] == ep.n_instr - ep.n_data


def test_mixed_job(ctx):
    """One job with a kernel run block by block, a capture kernel and plain
    FP kernels: tiles of different kinds side by side in one launch."""
    rng = np.random.default_rng(9)
    parts = [shared_workload("phases", rng)[1], shared_workload("shared_divisor", rng)[1],
             SP.workload(SP.fp_arith(), [[64, 1, 1, 128, 1, 1]], [[(SP.LB + 4096, 4 * 300, 0, 0, 0)]])]
    dws = [ckc.DeviceWorkload(ctx, wl) for wl in parts]
    try:
        print("[case] axiprune mixed job", flush=True)
        job = ctx.check([d.desc() for d in dws])
        recs, mp, st = ctx.read(job, maps=True)
        r0, m0 = 0, 0
        for wl in parts:
            o = O.check(wl, nthreads=NCPU)
            n, na = wl.n_inputs, o["records"].shape[1]
            r = recs[r0:r0 + n * na].reshape(n, na)
            for f in ("first_key", "index", "count", "kinds", "first_kind"):
                assert np.array_equal(r[f], o["records"][f]), f
            assert np.array_equal(mp[m0:m0 + n], o["maps"])
            for f in ("lanes", "accesses_checked", "arith_faults", "flags"):
                assert np.array_equal(st[m0:m0 + n][f], o["status"][f]), f
            r0 += n * na
            m0 += n
    finally:
        for d in dws:
            d.close()


def test_blockwise_without_allocation(ctx):
    """The entry point that allocates nothing runs kernels block by block and
    the capture pass too."""
    import torch
    rng = np.random.default_rng(21)
    _, wl = shared_workload("rotate", rng)
    dw = ckc.DeviceWorkload(ctx, wl)
    try:
        n, na = wl.n_inputs, dw.info["n_accesses"]
        recs = torch.zeros(n * na * 32, dtype=torch.uint8, device="cuda")
        maps = torch.zeros(n * 65536, dtype=torch.uint8, device="cuda")
        st = torch.zeros(n * 40, dtype=torch.uint8, device="cuda")
        torch.cuda.synchronize()
        print("[case] axiprune noalloc", flush=True)
        ctx.check_noalloc([dw.desc(dense=True)], recs.data_ptr(), maps.data_ptr(), st.data_ptr())
        torch.cuda.synchronize()
        r = np.frombuffer(recs.cpu().numpy().tobytes(), ckc.RECORD_DTYPE).reshape(n, na)
        o = O.check(wl, nthreads=NCPU)
        for f in ("first_key", "index", "count", "kinds", "first_kind"):
            assert np.array_equal(r[f], o["records"][f]), f
        assert np.array_equal(maps.cpu().numpy().reshape(n, 65536), o["maps"])
    finally:
        dw.close()


def test_blockwise_tripwire(ctx):
    """Shared-memory kernels under the tripwire model: A with redzones, the
    shared window's end caught."""
    rng = np.random.default_rng(31)
    _, wl = shared_workload("bounds_up", rng)
    tabs = wl.tables.copy()
    tabs["redzone"][:, 0] = 16
    wl.tables = tabs
    wl.detector = W.DETECT_TRIPWIRE
    check_same(ctx, wl, what="bounds tripwire")
