"""Random programs whose part outside an expanded gather loop has the shapes
the whole-thread pass's rows form takes (affine forms of the thread
coordinates, loads, one level of IF guards, the loop's bounds from loads or
forms), plus near misses the device walk must hand back to the interpreter
(products of varying values, bit operations on them, a 32-bit value used at
64 bits).  For differential tests of the library against the oracle."""
from __future__ import annotations

import numpy as np

from paper_2601_01048_amd.gen import workloads as W
from paper_2601_01048_amd.gen.ir import Program

LB = W.LOGICAL_BASE


def rows_program(rng, near_miss: bool = False):
    """Slots: 0 P (int32 data: row-pointer-like, loaded), 1 C (int32 data,
    loaded in the body), 2 and 3 address-only.  Scalars: 0 a bound, 1 and 2
    uniform coefficients."""
    p = Program(n_scalars=3, n_slots=4)
    w = int(rng.choice([32, 64]))
    dims = rng.random() < 0.3
    tx, bx = p.special("tid.x"), p.special("bid.x")
    r = p.add(p.mul(bx, p.special("bdim.x"), w), tx, w)
    if dims:  # a second coordinate term
        r = p.add(r, p.mul(p.special("tid.y"), p.const(int(rng.integers(-3, 4)), w), w), w)
    k = rng.random()
    if k < 0.2:
        r = p.sub(r, p.scalar(1, w), w)
    elif k < 0.3:
        r = p.shl(r, p.const(1, w), w)
    elif k < 0.4:
        r = p.mul(r, p.const(int(rng.choice([-1, 2, 3])), w), w)
    elif k < 0.5 and w == 64:
        r = p.trunc(r)
        w = 32
    if near_miss:
        kind = int(rng.integers(3))
        if kind == 0:
            r = p.mul(r, p.special("tid.x"), w)        # product of two varying values
        elif kind == 1:
            r = p.op("AND", r, p.const(0xFFF, w), w)   # bit operation on a varying value
        elif w == 32:
            r = p.add(r, p.const(0, 64), 64)           # a 32-bit form read at 64 bits
        else:
            r = p.op("XOR", r, p.const(5, w), w)
    guard = rng.random()
    opened = False
    if guard < 0.7:
        bound = p.scalar(0, w)
        op = str(rng.choice(["CMPLTS", "CMPLTU", "CMPLES", "CMPLEU", "CMPNE", "CMPEQ"]))
        if op == "CMPEQ":
            pred = p.op(op, p.op("SUB", r, r, w) if rng.random() < 0.2 else r, bound, w)
        else:
            pred = p.op(op, r, bound, w)
        p._emit("IF", 0, 0xFFFF, pred.idx, 0, 0, 0, p._site_arg(True), p._site_arg(True))
        p._open.append("IF")
        opened = True
    elif guard < 0.8:
        p._emit("IF", 0, 0xFFFF, r.idx, 0, 0, 0, p._site_arg(True), p._site_arg(True))  # value != 0
        p._open.append("IF")
        opened = True
    if rng.random() < 0.3:
        p.access(2, p.add(r, p.const(int(rng.integers(-2, 3)), w), w), w=w)
    s = p.load(0, r, elem=4, w=w)
    if rng.random() < 0.7:
        e = p.load(0, p.add(r, p.const(1, w), w), elem=4, w=w)
    else:
        e = p.add(s, p.const(int(rng.integers(0, 5)), 32), 32)
    if rng.random() < 0.2:  # an index from a loaded value
        s2 = p.load(0, p.add(s, p.scalar(2, 32), 32), elem=4, w=32)
        p.access(3, s2, w=32)
    lw = 32
    step = p.const(int(rng.choice([1, 1, 1, 2, -1])), lw)
    with p.loop(s, e, step, w=lw, site_iter=True, site_exit=True) as j:
        c = p.load(1, j, elem=4, w=lw)
        p.access(2, j, w=lw)
        p.access(3, c, w=lw)
    p.access(3, r, w=w)
    if opened:
        assert p._open.pop() == "IF"
        p._emit("ENDIF")
    if rng.random() < 0.5:
        p.access(2, r, w=w)
    return p.to_bytes()


def rows_workload(rng, ir, n_inputs=6, mode=W.MODE_FULL, cap=(20, 12)):
    """Inputs of several launch shapes; P holds nondecreasing row starts with
    some corrupted entries (negative or past C), C column indices with some
    out of range."""
    n_rows = 3000
    lens = rng.integers(0, 6, size=n_rows)
    P = np.concatenate([[0], np.cumsum(lens)]).astype(np.int32)
    bad = rng.choice(n_rows, size=6, replace=False)
    P[bad] = rng.integers(-40, int(P[-1]) + 80, size=6)
    nnz = int(P[-1])
    C = rng.integers(-3, 2200, size=max(nnz, 1) + 64).astype(np.int32)
    launches, tabs, scal = [], [], []
    for i in range(n_inputs):
        bs = int(rng.choice([32, 64, 96, 256]))
        by = int(rng.choice([1, 1, 2]))
        g = int(rng.integers(1, 3000 // (bs * by) + 2))
        launches.append([g, 1, 1, bs, by, 1])
        tabs.append([(LB, 4 * (n_rows + 1 - int(rng.integers(0, 40))), 1, 0, 0),
                     (LB + (1 << 30), 4 * (nnz + int(rng.integers(-20, 20))), 2, 0, 0),
                     (LB + (2 << 30), 4 * int(rng.integers(1000, 3000)), 0, 0, 0),
                     (LB + (3 << 30), 4 * 2048, 0, 0, 0)])
        scal.append([int(rng.integers(n_rows // 2, n_rows + 50)), int(rng.integers(-3, 4)),
                     int(rng.integers(-5, 5))])
    launches = np.array(launches, np.uint32)
    tables = np.zeros((n_inputs, 4), W.ALLOC_DTYPE)
    for i in range(n_inputs):
        tables[i] = tabs[i]
    return W.Workload("rows", ir, launches, np.array(scal, np.int64), tables,
                      np.arange(n_inputs, dtype=np.uint32), [P, C], mode, cap)


def extreme_rows_program():
    """A 32-bit rows-form program whose loop bounds come from loaded values
    near the ends of the int32 range and whose last index is the row times a
    scalar (wrapping modulo 2^32): r = bid.x * bdim.x + tid.x; if r < s0:
    [s, e) = P[r], P[r + 1]; for j in [s, e): X[C[j]]; Y[r * s1]."""
    p = Program(n_scalars=2, n_slots=4)
    w = 32
    r = p.add(p.mul(p.special("bid.x"), p.special("bdim.x"), w), p.special("tid.x"), w)
    pred = p.op("CMPLTS", r, p.scalar(0, w), w)
    p._emit("IF", 0, 0xFFFF, pred.idx, 0, 0, 0, p._site_arg(True), p._site_arg(True))
    p._open.append("IF")
    s = p.load(0, r, elem=4, w=w)
    e = p.load(0, p.add(r, p.const(1, w), w), elem=4, w=w)
    with p.loop(s, e, p.const(1, w), w=w, site_iter=True, site_exit=True) as j:
        c = p.load(1, j, elem=4, w=w)
        p.access(2, c, w=w)
    p.access(3, p.mul(r, p.scalar(1, w), w), w=w)
    assert p._open.pop() == "IF"
    p._emit("ENDIF")
    return p.to_bytes()


def extreme_rows_workload(rng, ir, n_inputs=4):
    """Row pointers with ordinary rows and rows whose bounds sit near
    INT32_MIN and INT32_MAX (spans of a few iterations there, spans over the
    trip cap across the range, bounds in both orders); multipliers of the last
    index that wrap it to either sign."""
    n_rows = 2000
    lens = rng.integers(0, 5, size=n_rows)
    P = np.concatenate([[0], np.cumsum(lens)]).astype(np.int64)
    i32min, i32max = -(1 << 31), (1 << 31) - 1
    for r in rng.choice(n_rows - 1, size=40, replace=False):
        k = int(rng.integers(5))
        if k == 0:
            P[r], P[r + 1] = i32max - int(rng.integers(1, 9)), i32max
        elif k == 1:
            P[r], P[r + 1] = i32min, i32min + int(rng.integers(1, 9))
        elif k == 2:
            P[r], P[r + 1] = i32min + int(rng.integers(0, 9)), i32max - int(rng.integers(0, 9))
        elif k == 3:
            P[r], P[r + 1] = i32max, i32min
        else:
            P[r], P[r + 1] = -int(rng.integers(1, 50)), int(rng.integers(1, 50))
    P = P.astype(np.int32)
    nnz = int(lens.sum()) + 64
    C = rng.integers(-5, 1200, size=nnz).astype(np.int32)
    launches, tabs, scal = [], [], []
    mults = [0x40000003, -0x3FFFFFFD, 7, 0x7FFFFFFF]
    for i in range(n_inputs):
        bs = int(rng.choice([64, 256]))
        launches.append([(n_rows + bs - 1) // bs, 1, 1, bs, 1, 1])
        tabs.append([(LB, 4 * (n_rows + 1), 1, 0, 0), (LB + (1 << 30), 4 * nnz, 2, 0, 0),
                     (LB + (2 << 30), 4 * 1024, 0, 0, 0), (LB + (3 << 30), 4 * 4096, 0, 0, 0)])
        scal.append([n_rows - int(rng.integers(0, 3)), mults[i % len(mults)]])
    tables = np.zeros((n_inputs, 4), W.ALLOC_DTYPE)
    for i in range(n_inputs):
        tables[i] = tabs[i]
    return W.Workload("rows_extreme", ir, np.array(launches, np.uint32), np.array(scal, np.int64), tables,
                      np.arange(n_inputs, dtype=np.uint32), [P, C], W.MODE_FULL, (20, 12))
