"""The tripwire (redzone) detector model and memory spaces on the GPU,
against the oracle: records, dense maps and status byte for byte.

Allocations are laid out next to each other with per-allocation redzones,
so overflows of every distance occur: into the own redzone (caught), over it
into the neighbour (missed), into freed memory (caught).  Programs that
normally run on the trace or gather paths run on the interpreter under this
model; the thread sets, the PREX sweep and the entry point that allocates
nothing are covered too."""
import os

import numpy as np
import pytest

import randprog as RP
from oracle import oracle as O
from paper_2601_01048_amd import ckc
from paper_2601_01048_amd.gen import workloads as W
from paper_2601_01048_amd.gen.ir import Program

pytestmark = pytest.mark.gpu

NCPU = max(1, min(16, os.cpu_count() or 1))
LB = W.LOGICAL_BASE


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    c = ckc.Context(0)
    yield c
    c.close()


def relayout(wl, rng, rz_choices=(0, 4, 8, 16, 64, 256), gap_choices=(0, 0, 4, 100), freed_p=0.0,
             keep_data=True):
    """The workload with every table's live allocations placed one after the
    other (in slot order) with random redzones and gaps; a fraction of the
    non-data slots freed.  One table per input."""
    n = wl.n_inputs
    src = wl.tables[wl.table_idx]
    tabs = np.zeros_like(src)
    for i in range(n):
        cur = LB + 4096
        for s in range(src.shape[1]):
            e = src[i, s].copy()
            if e["base"] != 0:
                rz = int(rng.choice(rz_choices))
                cur += rz + int(rng.choice(gap_choices))
                e["base"] = cur
                e["redzone"] = rz
                cur += int(e["size_bytes"]) + rz
                if freed_p and e["data"] == 0 and rng.random() < freed_p:
                    e["flags"] |= W.ALLOC_FREED
            tabs[i, s] = e
    out = wl.subset(np.arange(n))
    out.tables = tabs
    out.table_idx = np.arange(n, dtype=np.uint32)
    out.detector = W.DETECT_TRIPWIRE
    return out


def check_same(ctx, wl, mode=None, what=""):
    print(f"[case] tripwire {what} mode={wl.mode if mode is None else mode} inputs={wl.n_inputs}", flush=True)
    g = ckc.run_workload(ctx, wl, mode=mode)
    o = O.check(wl, mode=mode, nthreads=NCPU)
    for f in ("first_key", "index", "count", "kinds", "first_kind"):
        assert np.array_equal(g["records"][f], o["records"][f]), (what, f)
    assert np.array_equal(g["maps"], o["maps"]), what
    for f in ("lanes", "accesses_checked", "hang_lanes", "arith_faults", "flags"):
        assert np.array_equal(g["status"][f], o["status"][f]), (what, f)
    return g, o


@pytest.mark.parametrize("seed", range(3))
def test_affine1d_layouts(ctx, seed):
    rng = np.random.default_rng(500 + seed)
    wl = relayout(W.mini("config1", n_inputs=32, seed=20 + seed), rng, freed_p=0.2)
    g, o = check_same(ctx, wl, what="1-D")
    ex = O.check(wl, detector=W.DETECT_EXACT)
    # the model reports fewer violations than exact bounds, never more
    assert int(g["records"]["count"].sum()) <= int(ex["records"]["count"].sum())


@pytest.mark.parametrize("mode", [W.MODE_FULL, W.MODE_BOUNDARY, W.MODE_CORNERS, W.MODE_PREX])
def test_stencil_layouts_every_thread_set(ctx, mode):
    rng = np.random.default_rng(600 + mode)
    wl = relayout(W.mini("config2"), rng, rz_choices=(0, 8, 64, 4096), freed_p=0.25)
    check_same(ctx, wl, mode=mode, what="stencil")


@pytest.mark.parametrize("w", [32, 64])
def test_csr_gather_layouts(ctx, w):
    """CSR rows with corrupted columns: x[col] overflows up to 64 elements
    past either end, so some land in x's redzone and some beyond it."""
    rng = np.random.default_rng(700 + w)
    wl = relayout(W.mini("config3", w=w), rng, rz_choices=(16, 64, 128), gap_choices=(0, 8))
    g, o = check_same(ctx, wl, what=f"csr i{w}")
    ex = O.check(wl, detector=W.DETECT_EXACT)
    caught, total = int(g["records"]["count"][:, 4].sum()), int(ex["records"]["count"][:, 4].sum())
    assert 0 < caught < total, (caught, total)


@pytest.mark.parametrize("seed", range(8))
def test_random_programs_spaces_and_redzones(ctx, seed):
    rng = np.random.default_rng(800 + seed)
    ir = RP.random_program(rng)
    wl = RP.random_workload(rng, ir)
    wl = relayout(wl, rng, rz_choices=(0, 4, 16, 64), freed_p=0.15)
    # slots 1 and 2 in shared / local memory when the program does not load them
    spaces = [0, int(rng.integers(0, 3)), int(rng.integers(0, 3))]
    hdr = bytearray(wl.ir)
    sp = spaces[0] | spaces[1] << 2 | spaces[2] << 4
    hdr[20:24] = int(sp).to_bytes(4, "little")
    try:
        O.validate(bytes(hdr))
        wl.ir = bytes(hdr)
    except O.OracleError:
        pass  # a LOAD reads slot 1 or 2: keep them global
    for mode in (W.MODE_FULL, W.MODE_BOUNDARY):
        check_same(ctx, wl, mode=mode, what=f"random {seed}")


def test_table1_split_and_shared_window(ctx):
    """Table 1's global-memory split (overflow into the redzone caught, a jump
    into the neighbouring buffer missed) and a shared window, one thread per
    index value."""
    n, rz = 64, 16
    a = LB + 4096
    p = Program(n_scalars=1, n_slots=4, spaces=[0, 0, 1, 1])
    i = p.scalar(0, 32)
    p.access(0, i, elem=4)
    p.access(2, i, elem=4)
    ir = p.to_bytes()
    tab = np.array([(a, 4 * n, 0, 0, rz), (a + 4 * n + 2 * rz, 4 * n, 0, 0, rz),
                    (0x100, 64, 0, 0, 0), (0x140, 32, 0, 0, 0)], W.ALLOC_DTYPE)
    idx = np.array([n, n + 11, -1, -5, n + 3, n + 4, 16, 23, 24, -65, -1 << 31, (1 << 31) - 1], np.int64)
    launch = np.tile(np.array([[1, 1, 1, 1, 1, 1]], np.uint32), (len(idx), 1))
    wl = W.Workload("t1", ir, launch, idx.reshape(-1, 1), tab.reshape(1, -1), np.zeros(len(idx), np.uint32),
                    [], W.MODE_FULL, detector=W.DETECT_TRIPWIRE)
    g, o = check_same(ctx, wl, what="table 1")
    assert [int(c) for c in g["records"]["count"][:, 0][:6]] == [1, 0, 1, 0, 1, 1]
    assert [int(c) for c in g["records"]["count"][:, 1][6:10]] == [0, 0, 1, 1]


def test_tripwire_without_allocation(ctx):
    """The entry point that allocates nothing runs the same model."""
    import torch
    rng = np.random.default_rng(900)
    wl = relayout(W.mini("config3"), rng, rz_choices=(16, 64))
    dw = ckc.DeviceWorkload(ctx, wl)
    try:
        desc = [dw.desc(dense=True)]
        n, na = wl.n_inputs, dw.info["n_accesses"]
        recs = torch.zeros(n * na * 32, dtype=torch.uint8, device="cuda")
        maps = torch.zeros(n * 65536, dtype=torch.uint8, device="cuda")
        st = torch.zeros(n * 40, dtype=torch.uint8, device="cuda")
        torch.cuda.synchronize()
        ctx.check_noalloc(desc, recs.data_ptr(), maps.data_ptr(), st.data_ptr())
        torch.cuda.synchronize()
        r = np.frombuffer(recs.cpu().numpy().tobytes(), ckc.RECORD_DTYPE).reshape(n, na)
        o = O.check(wl, nthreads=NCPU)
        for f in ("first_key", "index", "count", "kinds", "first_kind"):
            assert np.array_equal(r[f], o["records"][f]), f
        assert np.array_equal(maps.cpu().numpy().reshape(n, 65536), o["maps"])
    finally:
        dw.close()


def test_tripwire_layout_rejected(ctx):
    """An allocation whose left redzone would start below address 0 is refused
    under the tripwire model and accepted under exact bounds."""
    ir = W.f1_program(32)
    tab = np.array([(16, 64, 0, 0, 32), (LB, 64, 0, 0, 0)], W.ALLOC_DTYPE)
    wl = W.Workload("bad", ir, np.array([[1, 1, 1, 8, 1, 1]], np.uint32), np.zeros((1, 0), np.int64),
                    tab.reshape(1, -1), np.zeros(1, np.uint32), [], W.MODE_FULL)
    ckc.run_workload(ctx, wl)
    wl.detector = W.DETECT_TRIPWIRE
    with pytest.raises(ckc.CkcError) as e:
        ckc.run_workload(ctx, wl)
    assert e.value.code == -1
