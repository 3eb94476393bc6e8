"""Pins of the oracle's memory spaces and tripwire (redzone) detector model.

The paper contrasts two kinds of detectors (Section 7.1, Table 1):
address sanitizers that poison only redzones around allocations ("tripwires")
catch linear buffer overflows (BO) but miss out-of-bounds reads/writes that
jump over a redzone into other memory (RW), while base-and-bounds checkers
catch both.  The pins here: a byte-level shadow-memory model written from
that description (``brute.shadow``: sets of poisoned byte addresses, as a
sanitizer's shadow memory holds them) on small grids and several layouts;
special cases that reduce to the exact model (redzones wider than any
overflow) or to nothing (no redzones); the Table 1 global-memory split; the
window of shared memory; the subset property against exact bounds."""
import numpy as np
import pytest

import brute
import kernels as K
import randprog as RP
from oracle import oracle as O
from paper_2601_01048_amd.gen import workloads as W
from paper_2601_01048_amd.gen.ir import Program

LB = W.LOGICAL_BASE
EXACT, TRIP = W.DETECT_EXACT, W.DETECT_TRIPWIRE


def f1_layout(n, rz_a, rz_b, gap=0, b_flags=0, a_base=LB + 4096):
    """A (n int32) then B (n int32) right after A's right redzone, B's left
    redzone and `gap` more bytes."""
    b_base = a_base + 4 * n + rz_a + rz_b + gap
    return [(a_base, 4 * n, 0, 0, rz_a), (b_base, 4 * n, 0, b_flags, rz_b)]


def run_both(ir, launches, tables, model, n_acc, n_sites, spaces=(), scalars=None, L=(0, 0)):
    wl = K.simple_workload(ir, launches, tables, scalars=scalars)
    wl.detector = TRIP
    got = O.check(wl)
    exp = brute.run(model, [np.asarray(l, np.uint32) for l in launches], tables, n_acc, n_sites,
                    tripwire=True, spaces=spaces, scalars=None if scalars is None else np.asarray(scalars), L=L)
    brute.assert_matches(got, exp)
    return got


@pytest.mark.parametrize("rz_a,rz_b,gap,b_flags", [
    (0, 0, 0, 0), (4, 0, 0, 0), (8, 8, 0, 0), (16, 4, 12, 0), (64, 64, 0, 0),
    (3, 5, 1, 0), (8, 0, 0, W.ALLOC_FREED), (0, 0, 40, W.ALLOC_FREED), (0, 8, 0, W.ALLOC_FREED)])
def test_f1_shadow_brute_force(rz_a, rz_b, gap, b_flags):
    """A[gid-1], A[gid], B[gid+1], B[gid+2] over grids past the arrays' ends:
    underflow of A at gid 0, overflows of A into its redzone, B's redzone and
    B itself, overflows of B past its own redzone; B freed in three layouts
    (in the last, A's overflow lands in the freed B's redzone)."""
    ir = W.f1_program(32)
    launches, tables = [], []
    for G, bs, n in ((1, 32, 20), (2, 32, 50), (3, 64, 100), (4, 16, 30)):
        launches.append([G, 1, 1, bs, 1, 1])
        tables.append(f1_layout(n, rz_a, rz_b, gap, b_flags))
    run_both(ir, launches, tables, K.f1_model(32), 4, 4)


def test_f2_shadow_brute_force():
    """2-D stencil over a small image with in/out adjacent and 8-byte
    redzones: row overflows of one row land in the next row (in bounds),
    overflows past the last row hit the redzone only within 8 bytes."""
    ir = W.f2_program(32)
    launches, tables, scalars = [], [], []
    for (gx, gy, H, Wd, r) in ((2, 2, 30, 30, 1), (3, 2, 40, 44, 2), (2, 3, 35, 30, 2)):
        launches.append([gx, gy, 1, 16, 16, 1])
        size = 4 * H * Wd
        a = LB + 1024
        tables.append([(a, size, 0, 0, 8), (a + size + 16, size, 0, 0, 8)])
        scalars.append([Wd, r])
    run_both(ir, launches, tables, K.f2_model(32), 3, 5, scalars=scalars, L=(20, 0))


def test_redzones_wider_than_any_overflow_equal_exact():
    """With redzones wider than the farthest overflow every exact violation
    touches a redzone: the tripwire model reduces to exact bounds."""
    wl = W.mini("config1")
    tabs = wl.tables.copy()
    tabs["redzone"] = 1 << 20
    wl.tables = tabs
    ex = O.check(wl, detector=EXACT)
    tw = O.check(wl, detector=TRIP)
    assert ex["records"].tobytes() == tw["records"].tobytes()
    assert int(ex["records"]["count"].sum()) > 0


def test_no_redzones_report_only_null_and_freed_bytes():
    """Without redzones nothing is poisoned but freed memory: live overflows
    all go unreported; a NULL slot is always reported; accesses inside a freed
    allocation are reported as FREED and those outside it are not."""
    ir = W.f1_program(32)
    n = 40
    launch = [[2, 1, 1, 32, 1, 1]]
    tw_live = O.check(K.simple_workload(ir, launch, [f1_layout(n, 0, 0, gap=64)]), detector=TRIP)
    assert int(tw_live["records"]["count"].sum()) == 0
    ex_live = O.check(K.simple_workload(ir, launch, [f1_layout(n, 0, 0, gap=64)]), detector=EXACT)
    assert int(ex_live["records"]["count"].sum()) > 0
    # B freed: B[gid+1], B[gid+2] are reported exactly for the indices inside
    # B (0 <= gid+off < n), i.e. n - 1 and n - 2 threads of the 64
    tw_freed = O.check(K.simple_workload(ir, launch, [f1_layout(n, 0, 0, gap=200, b_flags=W.ALLOC_FREED)]),
                       detector=TRIP)
    rec = tw_freed["records"][0]
    assert [int(c) for c in rec["count"]] == [0, 0, n - 1, n - 2]
    assert int(rec[2]["first_kind"]) == brute.KIND_FREED and int(rec[2]["first_key"]) == 0
    # A at base 0 (NULL): every access to A reported as NULL under both models
    null_tab = [[(0, 4 * n, 0, 0, 0), (LB + 8192, 4 * n, 0, 0, 0)]]
    tw_null = O.check(K.simple_workload(ir, launch, null_tab), detector=TRIP)
    assert [int(c) for c in tw_null["records"][0]["count"]][:2] == [64, 64]
    assert int(tw_null["records"][0][0]["kinds"]) == brute.KIND_NULL


def test_table1_global_overflow_versus_arbitrary_access():
    """Table 1, global memory: a tripwire detector catches the buffer
    overflow (one element past the end, inside the redzone) and misses the
    out-of-bounds access that lands in the neighbouring buffer; exact bounds
    catch both."""
    n, rz = 64, 16
    a = LB + 4096
    b = a + 4 * n + 2 * rz
    p = Program(n_scalars=1, n_slots=2)
    i = p.scalar(0, 32)
    p.access(0, i, elem=4)
    ir = p.to_bytes()
    tab = [(a, 4 * n, 0, 0, rz), (b, 4 * n, 0, 0, rz)]
    # index n: BO (first byte past A, in A's redzone); index n + (2*rz)/4 + 3:
    # lands inside B (RW); index -1: BO below A; index -(rz/4) - 1: left of
    # A's left redzone, nothing there (RW)
    cases = [(n, True), (n + 2 * rz // 4 + 3, False), (-1, True), (-(rz // 4) - 1, False),
             (n + rz // 4 - 1, True), (n + rz // 4, True)]
    launches = [[1, 1, 1, 1, 1, 1]] * len(cases)
    wl = K.simple_workload(ir, launches, [tab] * len(cases), scalars=[[c] for c, _ in cases])
    ex = O.check(wl, detector=EXACT)
    tw = O.check(wl, detector=TRIP)
    for k, (idx, caught) in enumerate(cases):
        assert int(ex["records"][k, 0]["count"]) == 1, idx
        assert int(tw["records"][k, 0]["count"]) == int(caught), idx
        if caught:
            assert int(tw["records"][k, 0]["index"]) == idx


def test_shared_window_and_neighbour():
    """Two per-block shared buffers without redzones: an access past the end
    of the shared window is caught (a detector that knows the shared region,
    Section 7.2.1), one that lands in the other buffer is not, and a global
    buffer at the same logical addresses does not affect either."""
    p = Program(n_scalars=1, n_slots=3, spaces=[1, 1, 0])
    i = p.scalar(0, 32)
    p.access(0, i, elem=4)
    ir = p.to_bytes()
    s0, s1 = 0x100, 0x100 + 64
    tab = [(s0, 64, 0, 0, 0), (s1, 32, 0, 0, 0), (0x100 + 96, 4096, 0, 0, 16)]
    cases = [(16, False),   # first element of the second shared buffer
             (23, False),   # its last element
             (24, True),    # first byte past the shared window (0x100 + 96)
             (-1, False),   # below the first buffer, still inside the window
             (-65, True)]   # below address 0 of the window
    launches = [[1, 1, 1, 1, 1, 1]] * len(cases)
    wl = K.simple_workload(ir, launches, [tab] * len(cases), scalars=[[c] for c, _ in cases])
    tw = O.check(wl, detector=TRIP)
    exp = brute.run(lambda tid, bid, launch, sc: [("acc", 0, 0, int(sc[0]), 4, 0, 0)],
                    [np.asarray(l, np.uint32) for l in launches], [tab] * len(cases), 1, 0, tripwire=True,
                    spaces=[1, 1, 0], scalars=np.array([[c] for c, _ in cases]))
    for k, (idx, caught) in enumerate(cases):
        assert int(tw["records"][k, 0]["count"]) == int(caught), idx
        assert int(tw["records"][k, 0]["count"]) == exp[0][k][0]["count"], idx


@pytest.mark.parametrize("seed", range(6))
def test_tripwire_is_subset_of_exact_on_random_programs(seed):
    """Every record of the tripwire model is contained in the exact one:
    counts at most, kinds a subset, first keys not earlier; same status."""
    rng = np.random.default_rng(9000 + seed)
    ir = RP.random_program(rng)
    wl = RP.random_workload(rng, ir)
    tabs = wl.tables.copy()
    tabs["redzone"] = rng.integers(0, 64, size=tabs.shape)
    live = tabs["base"] != 0
    tabs["base"][live] += 4096  # room for left redzones
    wl.tables = tabs
    ex = O.check(wl, detector=EXACT)
    tw = O.check(wl, detector=TRIP)
    e, t = ex["records"], tw["records"]
    assert np.all(t["count"] <= e["count"])
    assert np.all((t["kinds"] & ~e["kinds"]) == 0)
    has = t["count"] > 0
    assert np.all(t["first_key"][has] >= e["first_key"][has])
    for f in ("lanes", "accesses_checked", "hang_lanes", "arith_faults"):
        assert np.array_equal(ex["status"][f], tw["status"][f])
    assert np.array_equal(ex["counts"], tw["counts"])


def test_tripwire_layout_and_space_validation():
    """A live allocation whose left redzone would start below address 0 is
    refused under the tripwire model (and accepted under exact bounds);
    slot spaces other than global/shared/local, spaces on slots the program
    does not have, and LOADs from local slots are malformed IR (LOADs from
    shared slots read shared memory back)."""
    ir = W.f1_program(32)
    tab = [[(16, 64, 0, 0, 32), (LB, 64, 0, 0, 0)]]
    wl = K.simple_workload(ir, [[1, 1, 1, 8, 1, 1]], tab)
    O.check(wl, detector=EXACT)
    with pytest.raises(O.OracleError) as e:
        O.check(wl, detector=TRIP)
    assert e.value.code == -1
    for spaces in ([3, 0], [0, 0, 1]):
        p = Program(n_slots=2, spaces=spaces)
        p.access(0, p.const(0, 32), elem=4)
        with pytest.raises(O.OracleError):
            O.validate(p.to_bytes())
    p = Program(n_slots=2, spaces=[0, 2])
    p.load(1, p.const(0, 32), elem=4)
    with pytest.raises(O.OracleError):
        O.validate(p.to_bytes())
    p = Program(n_slots=2, spaces=[0, 1])
    p.load(1, p.const(0, 32), elem=4)
    O.validate(p.to_bytes())
    p = Program(n_slots=2, spaces=[2, 1])
    p.access(0, p.const(0, 32), elem=4)
    p.access(1, p.const(0, 32), elem=4)
    O.validate(p.to_bytes())
