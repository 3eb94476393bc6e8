"""Pins of the oracle against what the paper and plain mathematics fix:
brute force from kernel formulas on tiny grids, closed forms at full size,
the paper's worked examples (Listing 1, Listing 3), the PREX Theorem's
subset/equality property, Algorithm 1's stop rule, and integer semantics
checked against Python's exact integers."""
import numpy as np
import pytest

import brute
import kernels as K
from oracle import oracle as O
from paper_2601_01048_amd.gen import workloads as W
from paper_2601_01048_amd.gen.ir import Program

LB = W.LOGICAL_BASE


# --------------------------------------------------------------------------
# brute force on small grids
# --------------------------------------------------------------------------
def test_f1_brute_force_mini():
    wl = W.mini("config1")
    out = O.check(wl)
    exp = brute.run(K.f1_model(), wl.launch, [t for t in wl.tables], 4, 4)
    brute.assert_matches(out, exp)


@pytest.mark.parametrize("mode", ["full", "corners", "boundary"])
def test_f2_brute_force_tiny(mode):
    wl = W.config2(seed=7, n_inputs=3, g0=3, hw0=30, delta=1, block=(8, 4),
                   mode={"full": 0, "corners": 1, "boundary": 2}[mode])
    out = O.check(wl)
    exp = brute.run(K.f2_model(), wl.launch, list(wl.tables), 3, 5, mode=mode, L=(20, 0),
                    scalars=wl.scalars)
    brute.assert_matches(out, exp)


def test_f2_i64_brute_force_tiny():
    wl = W.config2(seed=8, n_inputs=2, g0=3, hw0=30, delta=1, block=(8, 4), w=64)
    out = O.check(wl)
    exp = brute.run(K.f2_model(w=64), wl.launch, list(wl.tables), 3, 5, L=(20, 0),
                    scalars=wl.scalars)
    brute.assert_matches(out, exp)


@pytest.mark.parametrize("w", [32, 64])
def test_f3_brute_force_tiny(w):
    wl = W.config3(seed=11, n_inputs=3, log2_rows=6, mean=4, frac=0.05, block=32, w=w)
    out = O.check(wl)
    model, bind = K.f3_model(list(wl.tables), wl.data, w=w)
    recs, counts, status = [], [], []
    for i in range(wl.n_inputs):
        bind(i)
        r, c, s = brute.run(model, wl.launch[i:i + 1], [wl.tables[i]], 6, 10, L=(20, 0),
                            scalars=wl.scalars[i:i + 1])
        recs += r; counts += c; status += s
    brute.assert_matches(out, (recs, counts, status))
    assert out["records"]["count"][:, 4].sum() > 0  # corrupted col_idx reached x[]


def test_f3_hang_cap_brute_force():
    wl = W.config3(seed=12, n_inputs=2, log2_rows=6, mean=6, frac=0.0, block=32)
    cap = 3  # rows longer than 8 nonzeros hang
    out = O.check(wl, cap_log2=(cap, 12))
    model, bind = K.f3_model(list(wl.tables), wl.data, cap=1 << cap)
    recs, counts, status = [], [], []
    for i in range(wl.n_inputs):
        bind(i)
        r, c, s = brute.run(model, wl.launch[i:i + 1], [wl.tables[i]], 6, 10, L=(cap, 0),
                            scalars=wl.scalars[i:i + 1])
        recs += r; counts += c; status += s
    brute.assert_matches(out, (recs, counts, status))
    assert out["status"]["hang_lanes"].sum() > 0


def test_null_and_freed_kinds():
    ir = K.listing3_program()
    launch = [[2, 1, 1, 4, 1, 1]]
    tables = [[(0, 64, 0, 0, 0), (LB, 64, 0, 1, 0), (LB, 16, 0, 0, 0)]]
    wl = K.simple_workload(ir, launch, tables, scalars=[[8]])
    out = O.check(wl)
    exp = brute.run(K.listing3_model, wl.launch, list(wl.tables), 3, 5, scalars=wl.scalars)
    brute.assert_matches(out, exp)
    r = out["records"][0]
    assert r[0]["kinds"] == O.KIND_NULL and r[0]["count"] == 8
    assert r[1]["kinds"] == O.KIND_FREED and r[1]["count"] == 8
    assert r[2]["kinds"] == O.KIND_OVER and r[2]["count"] == 5  # c has 4 elements; ids 3..7 write 4..8


# --------------------------------------------------------------------------
# the paper's worked examples
# --------------------------------------------------------------------------
def test_listing1_seven_accesses():
    """Listing 1 has seven memory accesses over two distinct indices
    (Section 5.1.1); with N = gridSize*blockSize nothing is out of bounds and
    with one element less, exactly the last thread overflows a, b and c."""
    ir = K.listing1_program()
    assert O.validate(ir)[0] == 7
    bs, gs = 8, 5
    N = bs * gs
    for n_elems, expect_bad in ((N, False), (N - 1, True)):
        tables = [[(LB, bs * 4), (LB, bs * 4), (LB, n_elems * 4), (LB, n_elems * 4), (LB, n_elems * 4)]]
        wl = K.simple_workload(ir, [[gs, 1, 1, bs, 1, 1]], [[t + (0, 0, 0) for t in tables[0]]])
        out = O.check(wl)
        exp = brute.run(K.listing1_model, wl.launch, list(wl.tables), 7, 7)
        brute.assert_matches(out, exp)
        bad = out["records"]["count"][0]
        if expect_bad:
            assert list(bad) == [1, 0, 1, 0, 0, 0, 1]
            assert out["records"]["first_key"][0][0] == N - 1
        else:
            assert bad.sum() == 0


@pytest.mark.parametrize("N,bs", [(1023, 256), (1000, 256), (77, 8)])
def test_listing3_worked_bug(N, bs):
    """Listing 3: with ceil(N/blockSize) blocks and the guard id < N, the only
    thread that goes out of bounds is id = N-1, once on each of a, b, c.  When
    N mod blockSize = blockSize-1 that thread is (block ceil(N/bs)-1, thread
    bs-2), the coordinates given in Section 5.1.2."""
    grid = -(-N // bs)
    tables = [[(LB, N * 4, 0, 0, 0)] * 3]
    wl = K.simple_workload(K.listing3_program(), [[grid, 1, 1, bs, 1, 1]], tables, scalars=[[N]])
    out = O.check(wl)
    rec = out["records"][0]
    assert list(rec["count"]) == [1, 1, 1]
    assert list(rec["first_key"]) == [N - 1] * 3
    assert list(rec["index"]) == [N] * 3
    assert list(rec["first_kind"]) == [O.KIND_OVER] * 3
    gtid = int(rec["first_key"][0])
    if N % bs == bs - 1:
        assert (gtid // bs, gtid % bs) == (grid - 1, bs - 2)
    exp = brute.run(K.listing3_model, wl.launch, list(wl.tables), 3, 5, scalars=wl.scalars)
    brute.assert_matches(out, exp)


# --------------------------------------------------------------------------
# closed forms at full size
# --------------------------------------------------------------------------
def f1_closed_form(wl):
    """Access k with offset o over T = 256*G threads and n elements:
    UNDER count max(0, min(T, -o)); OVER count max(0, T-n+o); first key 0 if
    o < 0 else n-o; map min(255, T) at each of the four sites."""
    G, n = wl.meta["G"].astype(np.int64), wl.meta["n"].astype(np.int64)
    T = G * wl.meta["block"]
    exp = {}
    for a, o in enumerate((-1, 0, 1, 2)):
        under = np.maximum(0, np.minimum(T, -o))
        over = np.maximum(0, T - n + o)
        key = np.where(o < 0, 0, n - o)
        exp[a] = (under + over, key, np.where(o < 0, -1, n))
    return T, exp


def test_f1_closed_form_full_size():
    wl = W.config1()
    out = O.check(wl, nthreads=8)
    T, exp = f1_closed_form(wl)
    for a in range(4):
        cnt, key, idx = exp[a]
        np.testing.assert_array_equal(out["records"]["count"][:, a], cnt)
        has = cnt > 0
        np.testing.assert_array_equal(out["records"]["first_key"][has, a], key[has])
        np.testing.assert_array_equal(out["records"]["index"][has, a], idx[has])
    np.testing.assert_array_equal(out["status"]["lanes"], T)
    np.testing.assert_array_equal(out["status"]["accesses_checked"], 4 * T)
    for s in range(4):
        np.testing.assert_array_equal(out["maps"][:, s], np.minimum(255, T))
    # the reading of the configuration: every input underflows at gid 0 and
    # most inputs overflow at offset +2 (see the design notes)
    assert (out["records"]["kinds"][:, 0] & O.KIND_UNDER).all()


def f2_numpy(wl, i):
    """Vectorised enumeration of config-2 indices for input i over the
    (bx, by, tx, ty) box: returns (count, first_key, index, kinds) per access."""
    gx, gy, _, bx, by, _ = (int(v) for v in wl.launch[i])
    S, r = int(wl.scalars[i, 0]), int(wl.scalars[i, 1])
    n_el = int(wl.tables[wl.table_idx[i]][0]["size_bytes"]) // 4
    BY, BX, TY, TX = np.meshgrid(np.arange(gy), np.arange(gx), np.arange(by), np.arange(bx), indexing="ij")
    blin = BX + gx * BY
    gtid = (blin * (bx * by) + TX + bx * TY).ravel().astype(np.int64)
    x = (BX * bx + TX).ravel().astype(np.int64)
    y = (BY * by + TY).ravel().astype(np.int64)
    base = y * S + x
    res = []
    for a, offs in ((0, [0]), (1, None), (2, [0])):
        if offs is None:
            offs = []
            for k in range(8):
                j = k + (k > 3)
                offs.append((j // 3 - 1) * r * S + (j % 3 - 1) * r)
        cnt, fk, fi, kinds = 0, (1 << 64) - 1, 0, 0
        for it, o in enumerate(offs):
            idx = base + o
            bad = (idx < 0) | (idx >= n_el)
            cnt += int(bad.sum())
            if bad.any():
                kinds |= (1 if (idx >= n_el).any() else 0) | (2 if (idx < 0).any() else 0)
                keys = (gtid[bad] << 20) | (it if a == 1 else 0)
                m = int(keys.argmin())
                if int(keys[m]) < fk:
                    fk, fi = int(keys[m]), int(idx[bad][m])
        res.append((cnt, fk, fi, kinds))
    return res


def test_f2_numpy_mini():
    wl = W.mini("config2")
    out = O.check(wl)
    for i in range(wl.n_inputs):
        for a, (cnt, fk, fi, kinds) in enumerate(f2_numpy(wl, i)):
            rec = out["records"][i, a]
            assert (int(rec["count"]), int(rec["first_key"]), int(rec["kinds"])) == (cnt, fk, kinds)
            if cnt:
                assert int(rec["index"]) == fi


@pytest.mark.slow
def test_f2_numpy_full_size_two_inputs():
    wl = W.config2().subset([0, 4095])
    out = O.check(wl, nthreads=2)
    for i in range(2):
        for a, (cnt, fk, fi, kinds) in enumerate(f2_numpy(wl, i)):
            rec = out["records"][i, a]
            assert (int(rec["count"]), int(rec["first_key"]), int(rec["kinds"])) == (cnt, fk, kinds)
    lanes = wl.launch[:, 0].astype(np.int64) * wl.launch[:, 1] * 256
    np.testing.assert_array_equal(out["status"]["accesses_checked"], 10 * lanes)


def f3_numpy(wl, i):
    """Config 3 closed form: only x[col] can be out of bounds (row_ptr, col_idx,
    val and y are in bounds by construction); rows are contiguous in j, so the
    first bad j gives the first key (row << 20 | j - row_ptr[row])."""
    row_ptr = wl.data[0].astype(np.int64)
    col = wl.data[1 + i].astype(np.int64)
    ncols = wl.meta["ncols"]
    bad = (col < 0) | (col >= ncols)
    if not bad.any():
        return 0, (1 << 64) - 1, 0, 0
    j = int(np.nonzero(bad)[0][0])
    row = int(np.searchsorted(row_ptr, j, side="right") - 1)
    kinds = (1 if (col >= ncols).any() else 0) | (2 if (col < 0).any() else 0)
    return int(bad.sum()), (row << 20) | (j - int(row_ptr[row])), int(col[j]), kinds


def test_f3_numpy_mini():
    wl = W.mini("config3")
    out = O.check(wl)
    nnz = wl.meta["nnz"]
    for i in range(wl.n_inputs):
        cnt, fk, fi, kinds = f3_numpy(wl, i)
        rec = out["records"][i]
        assert (int(rec[4]["count"]), int(rec[4]["first_key"]), int(rec[4]["kinds"])) == (cnt, fk, kinds)
        if cnt:
            assert int(rec[4]["index"]) == fi
        for a in (0, 1, 2, 3, 5):
            assert int(rec[a]["count"]) == 0
        nrows = wl.meta["nrows"]
        assert int(out["status"][i]["accesses_checked"]) == 3 * nrows + 3 * nnz


# --------------------------------------------------------------------------
# the PREX Theorem and Algorithm 1
# --------------------------------------------------------------------------
def flagged(out):
    return {(i, a, k) for i in range(out["records"].shape[0]) for a in range(out["records"].shape[1])
            for k in (1, 2, 4, 8) if out["records"]["kinds"][i, a] & k}


def assert_subset(rep, full):
    r, f = rep["records"], full["records"]
    assert (r["count"] <= f["count"]).all()
    assert ((r["kinds"] & ~f["kinds"]) == 0).all()
    has = r["count"] > 0
    assert (r["first_key"][has] >= f["first_key"][has]).all()
    assert (rep["maps"] <= full["maps"]).all()


@pytest.mark.parametrize("name", ["config1", "config2"])
@pytest.mark.parametrize("mode", [W.MODE_CORNERS, W.MODE_BOUNDARY])
def test_theorem_equality_on_affine_unguarded(name, mode):
    """For an affine-access kernel with no guarded access, the corner threads
    flag exactly the violations the whole grid flags (Theorem, Section 5.1.1);
    every superset of the corners does too."""
    wl = W.mini(name)
    full = O.check(wl, mode=W.MODE_FULL)
    rep = O.check(wl, mode=mode)
    assert (rep["status"]["flags"] & 1).all()  # no vertex wraps: the Theorem's premise holds
    assert_subset(rep, full)
    assert flagged(rep) == flagged(full)
    assert ((rep["records"]["count"] > 0) == (full["records"]["count"] > 0)).all()
    assert ((rep["maps"] > 0) == (full["maps"] > 0)).all()


@pytest.mark.parametrize("mode", [W.MODE_CORNERS, W.MODE_BOUNDARY, W.MODE_PREX])
def test_representative_sets_are_subsets(mode):
    wl = W.mini("config3")
    assert_subset(O.check(wl, mode=mode), O.check(wl, mode=W.MODE_FULL))


def test_boundary_set_sizes():
    """The boundary set is the perimeter of the grid in the dimensions it spans
    plus its middle block: a 128 x 128 grid gives 128*4 - 4 + 1 = 509 blocks;
    a grid of extent 1 or 2 in every spanned dimension is all boundary."""
    p = Program(n_scalars=0, n_slots=1)
    p.access(0, p.special("tid.x"), w=64)
    ir = p.to_bytes()
    for g, blocks in (((128, 128, 1), 509), ((1, 1, 1), 1), ((5, 1, 1), 3), ((2, 2, 2), 8),
                      ((4, 4, 4), 4 * 4 * 4 - 2 * 2 * 2 + 1), ((3, 1, 7), 3 * 7 - 1 * 5 + 1)):
        wl = K.simple_workload(ir, [list(g) + [2, 1, 1]], [[(LB, 8, 0, 0, 0)]], mode=W.MODE_BOUNDARY)
        assert int(O.check(wl)["status"]["lanes"][0]) == 2 * blocks, g
        assert len(brute.threads(wl.launch[0], "boundary")) == 2 * blocks, g


def test_corners_miss_guarded_bug():
    """Listing 3 is why the Theorem needs unguarded accesses: the corner
    threads miss the bug at id = N-1 unless it is a corner."""
    N, bs = 1000, 256
    wl = K.simple_workload(K.listing3_program(), [[4, 1, 1, bs, 1, 1]], [[(LB, N * 4, 0, 0, 0)] * 3],
                           scalars=[[N]])
    assert O.check(wl, mode=W.MODE_CORNERS)["records"]["count"].sum() == 0
    assert O.check(wl, mode=W.MODE_FULL)["records"]["count"].sum() == 3


def test_prex_runtime_stop_rules():
    """Algorithm 1 on Listing 3: the first head/tail pair (blocks 0 and 3)
    already holds the bug, so the sweep stops after two blocks; with no bug it
    continues until every access instruction has executed."""
    N, bs = 1000, 256
    wl = K.simple_workload(K.listing3_program(), [[4, 1, 1, bs, 1, 1]], [[(LB, N * 4, 0, 0, 0)] * 3],
                           scalars=[[N]], mode=W.MODE_PREX)
    out = O.check(wl)
    assert int(out["status"][0]["lanes"]) == 2 * bs
    assert list(out["records"]["count"][0]) == [1, 1, 1]
    # bug-free: arrays large enough; the accesses all run in the first pair
    wl2 = K.simple_workload(K.listing3_program(), [[4, 1, 1, bs, 1, 1]], [[(LB, 2 * N * 4, 0, 0, 0)] * 3],
                            scalars=[[N]], mode=W.MODE_PREX)
    out2 = O.check(wl2)
    assert int(out2["status"][0]["lanes"]) == 2 * bs and out2["records"]["count"].sum() == 0
    # guard false everywhere (N = 0): accesses never run, the sweep covers all
    # blocks, an odd count runs its middle block once
    wl3 = K.simple_workload(K.listing3_program(), [[5, 1, 1, bs, 1, 1]], [[(LB, 4, 0, 0, 0)] * 3],
                            scalars=[[0]], mode=W.MODE_PREX)
    assert int(O.check(wl3)["status"][0]["lanes"]) == 5 * bs


# --------------------------------------------------------------------------
# integer semantics, observed through the index of a NULL-slot violation
# --------------------------------------------------------------------------
def _probe(cases):
    """One thread; each case computes a value and exposes it as the index of
    an access to a NULL allocation (every access violates, index recorded)."""
    p = Program(n_scalars=0, n_slots=1)
    for op, w, a, b in cases:
        ra, rb = p.const(a, w), p.const(b, w)
        r = p.op(op, ra, rb, w)
        p.access(0, r, w=64)
    wl = K.simple_workload(p.to_bytes(), [[1, 1, 1, 1, 1, 1]], [[(0, 0, 0, 0, 0)]])
    out = O.check(wl)
    return [int(v) for v in out["records"]["index"][0]], int(out["status"][0]["arith_faults"])


def _trunc_div(a, b):
    q = abs(a) // abs(b)
    return q if (a >= 0) == (b >= 0) else -q


def _expect(op, w, a, b):
    a, b = K.wrap(a, w), K.wrap(b, w)
    ua, ub = a % (1 << w), b % (1 << w)
    mn = -(1 << (w - 1))
    sh = ub % w
    fault = 0
    if op == "ADD": r = a + b
    elif op == "SUB": r = a - b
    elif op == "MUL": r = a * b
    elif op == "DIVS":
        if b == 0: r, fault = 0, 1
        elif a == mn and b == -1: r = mn
        else: r = _trunc_div(a, b)
    elif op == "REMS":
        if b == 0: r, fault = 0, 1
        elif a == mn and b == -1: r = 0
        else: r = a - b * _trunc_div(a, b)
    elif op == "DIVU": r, fault = (ua // ub, 0) if ub else (0, 1)
    elif op == "REMU": r, fault = (ua % ub, 0) if ub else (0, 1)
    elif op == "AND": r = ua & ub
    elif op == "OR": r = ua | ub
    elif op == "XOR": r = ua ^ ub
    elif op == "SHL": r = ua << sh
    elif op == "SHRA": r = a >> sh
    elif op == "SHRL": r = ua >> sh
    elif op == "MINS": r = min(a, b)
    elif op == "MAXS": r = max(a, b)
    elif op == "MINU": r = min(ua, ub)
    elif op == "MAXU": r = max(ua, ub)
    elif op == "CMPEQ": r = int(a == b)
    elif op == "CMPNE": r = int(a != b)
    elif op == "CMPLTS": r = int(a < b)
    elif op == "CMPLES": r = int(a <= b)
    elif op == "CMPLTU": r = int(ua < ub)
    elif op == "CMPLEU": r = int(ua <= ub)
    return K.wrap(r, w), fault


OPS = ("ADD SUB MUL DIVS REMS DIVU REMU AND OR XOR SHL SHRA SHRL MINS MAXS MINU MAXU "
       "CMPEQ CMPNE CMPLTS CMPLES CMPLTU CMPLEU").split()


@pytest.mark.parametrize("w", [32, 64])
def test_integer_semantics(w):
    mn, mx = -(1 << (w - 1)), (1 << (w - 1)) - 1
    vals = [0, 1, -1, 2, 3, -3, 7, -7, mn, mx, w - 1, w, w + 1, 123456789, -987654321, (1 << 40) + 5]
    rng = np.random.default_rng(5)
    vals += [int(v) for v in rng.integers(-(1 << 62), 1 << 62, size=4)]
    for op in OPS:
        cases, exp, faults = [], [], 0
        for a in vals:
            for b in vals:
                cases.append((op, w, a, b))
                r, f = _expect(op, w, a, b)
                exp.append(r)
                faults += f
        got, got_faults = _probe(cases)
        assert got == exp, op
        assert got_faults == faults, op


def test_conversions_and_select():
    p = Program(n_scalars=0, n_slots=1)
    big = p.const(0x1_8000_0001, 64)
    p.access(0, p.sext(big), w=64)      # low 32 = 0x80000001 -> negative
    p.access(0, p.zext(big), w=64)
    p.access(0, p.trunc(big), w=64)
    p.access(0, p.const(0x1_8000_0001, 32), w=64)  # CONST at width 32 keeps the low half
    c1, c0 = p.const(5, 64), p.const(0, 64)
    p.access(0, p.select(c1, p.const(11, 64), p.const(22, 64)), w=64)
    p.access(0, p.select(c0, p.const(11, 64), p.const(22, 64)), w=64)
    p.access(0, big, w=32)              # index read at width 32
    wl = K.simple_workload(p.to_bytes(), [[1, 1, 1, 1, 1, 1]], [[(0, 0, 0, 0, 0)]])
    got = [int(v) for v in O.check(wl)["records"]["index"][0]]
    assert got == [K.wrap(0x80000001, 32), 0x80000001, K.wrap(0x80000001, 32),
                   K.wrap(0x80000001, 32), 11, 22, K.wrap(0x80000001, 32)]


def test_special_registers_3d():
    """tid/bid/bdim/gdim of a 3-D launch, exposed per thread: index =
    packed coordinates; the first violation per access is thread 0's and the
    last thread's values are checked through a bounded allocation."""
    p = Program(n_scalars=0, n_slots=1)
    names = ["tid.x", "tid.y", "tid.z", "bid.x", "bid.y", "bid.z", "bdim.x", "bdim.y", "bdim.z",
             "gdim.x", "gdim.y", "gdim.z"]
    for nm in names:
        p.access(0, p.special(nm), w=64)
    launch = [2, 3, 4, 5, 2, 3]
    # size 0 with a live base: every index >= 0 is OVER, so each access counts
    # every thread and index at first key = value at gtid 0
    wl = K.simple_workload(p.to_bytes(), [launch], [[(LB, 0, 0, 0, 0)]])
    out = O.check(wl)
    nthr = 2 * 3 * 4 * 5 * 2 * 3
    assert (out["records"]["count"][0] == nthr).all()
    assert [int(v) for v in out["records"]["index"][0]] == [0] * 6 + launch[3:] + launch[:3]


# --------------------------------------------------------------------------
# loops: trip counts, caps, nesting and keys
# --------------------------------------------------------------------------
def test_loop_trip_counts_and_nested_keys():
    """Nested loops with signed steps; the key carries (gtid, i1, i2)."""
    p = Program(n_scalars=4, n_slots=1)
    s0, e0, st0, e1 = (p.scalar(k, 32) for k in range(4))
    with p.loop(s0, e0, st0, w=32) as i:
        with p.loop(0, e1, 1, w=32) as j:
            p.access(0, p.add(p.mul(i, p.const(100, 32), 32), j, 32), w=32)
    ir = p.to_bytes()
    cases = [(0, 10, 3, 2), (10, 0, -3, 1), (5, 5, 1, 3), (-7, 7, 4, 0), (2, -(1 << 31), -(1 << 30), 1)]
    sc = np.array(cases, np.int64)
    launch = [[1, 1, 1, 2, 1, 1]] * len(cases)
    wl = K.simple_workload(ir, launch, [[(LB, 0, 0, 0, 0)]] * len(cases), scalars=sc, cap=(6, 4))
    out = O.check(wl)
    for n, (s, e, st, e1v) in enumerate(cases):
        outer = list(range(s, e, st))
        inner = list(range(0, e1v))
        assert int(out["records"]["count"][n, 0]) == 2 * len(outer) * len(inner)
        if outer and inner:
            assert int(out["records"]["first_key"][n, 0]) == 0
            assert int(out["records"]["index"][n, 0]) == K.wrap(outer[0] * 100, 32)
        # sites: LOOP iter/exit (outer 0,1), inner 2,3, access 4
        assert list(out["counts"][n]) == [2 * len(outer), 2, 2 * len(outer) * len(inner),
                                          2 * len(outer), 2 * len(outer) * len(inner)]


def test_loop_cap_hang_stops_thread():
    p = Program(n_scalars=1, n_slots=1)
    n = p.scalar(0, 64)
    with p.loop(0, n, 1, w=64) as k:
        p.access(0, k, w=64)
    p.access(0, p.const(-1, 64), w=64)
    ir = p.to_bytes()
    wl = K.simple_workload(ir, [[1, 1, 1, 3, 1, 1]] * 3, [[(LB, 4 * 4, 0, 0, 0)]] * 3,
                           scalars=[[4], [5], [1 << 62]], cap=(2, 0))
    out = O.check(wl)
    st = out["status"]
    assert list(st["hang_lanes"]) == [0, 3, 3]
    assert list(st["accesses_checked"]) == [3 * 5, 3 * 4, 3 * 4]
    assert list(out["records"]["count"][:, 1]) == [3, 0, 0]
    # keys carry the iteration ordinal in L1 = 2 bits: thread 1 is 1 << 2
    assert int(out["records"]["first_key"][0, 1]) == 0


def test_zero_step_loop_never_ends():
    p = Program(n_scalars=0, n_slots=1)
    with p.loop(0, 5, 0, w=32) as k:
        p.access(0, k)
    wl = K.simple_workload(p.to_bytes(), [[1, 1, 1, 1, 1, 1]], [[(LB, 64, 0, 0, 0)]], cap=(3, 0))
    out = O.check(wl)
    assert int(out["status"][0]["hang_lanes"]) == 1
    assert int(out["status"][0]["accesses_checked"]) == 8


# --------------------------------------------------------------------------
# errors
# --------------------------------------------------------------------------
def test_malformed_ir_rejected():
    ir = W.f3_program()
    with pytest.raises(O.OracleError) as e:
        O.validate(ir[:-1])
    assert e.value.code == -2
    bad = bytearray(ir)
    bad[0] ^= 1
    with pytest.raises(O.OracleError):
        O.validate(bytes(bad))
    # use of a register defined inside a loop body after the loop
    p = Program(n_scalars=0, n_slots=1)
    with p.loop(0, 4, 1) as k:
        v = p.add(k, 1)
    p.access(0, v)
    with pytest.raises(O.OracleError):
        O.validate(p.to_bytes())


def test_mutated_ir_never_crashes():
    rng = np.random.default_rng(3)
    base = bytearray(W.f3_program())
    for _ in range(300):
        b = bytearray(base)
        for _ in range(int(rng.integers(1, 6))):
            b[int(rng.integers(0, len(b)))] = int(rng.integers(0, 256))
        try:
            O.validate(bytes(b))
        except O.OracleError as e:
            assert e.code == -2


def test_key_range_rejected():
    p = Program(n_scalars=0, n_slots=1)
    with p.loop(0, 4, 1) as k:
        with p.loop(0, 4, 1) as j:
            p.access(0, p.add(k, j))
    # 2^20 blocks x 1024 threads = 2^30 threads; 2^30 << (32+4) > 2^64
    wl = K.simple_workload(p.to_bytes(), [[1 << 20, 1, 1, 1024, 1, 1]], [[(LB, 64, 0, 0, 0)]], cap=(32, 4))
    with pytest.raises(O.OracleError) as e:
        O.check(wl)
    assert e.value.code == -3


def test_empty_grid():
    wl = K.simple_workload(K.listing3_program(), [[0, 1, 1, 32, 1, 1]], [[(LB, 4, 0, 0, 0)] * 3],
                           scalars=[[5]])
    out = O.check(wl)
    assert int(out["status"][0]["lanes"]) == 0 and out["records"]["count"].sum() == 0
