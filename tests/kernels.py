"""Test kernels written twice: as IR (through the builder) and as a plain
Python model of one thread taken from the kernel's formula.  The Python model
feeds ``brute.run``; it never reads the IR."""
from __future__ import annotations

import numpy as np

from paper_2601_01048_amd.gen.ir import Program
from paper_2601_01048_amd.gen import workloads as W


def wrap(v: int, w: int) -> int:
    v &= (1 << w) - 1
    return v - (1 << w) if v >> (w - 1) else v


# ---- F1 ------------------------------------------------------------------
def f1_model(w=32, base_off=0):
    def k(tid, bid, launch, sc):
        gid = wrap(bid[0] * int(launch[3]) + tid[0], w) + base_off
        ev = []
        for a, (slot, off) in enumerate(((0, -1), (0, 0), (1, 1), (1, 2))):
            ev.append(("site", a))
            ev.append(("acc", a, slot, wrap(gid + off, w), 4, 0, 0))
        return ev
    return k


# ---- F2 ------------------------------------------------------------------
def f2_model(w=32, cap=1 << 20):
    def k(tid, bid, launch, sc):
        S, r = int(sc[0]), int(sc[1])
        off = int(sc[2]) if w == 64 else 0
        x = bid[0] * int(launch[3]) + tid[0]
        y = bid[1] * int(launch[4]) + tid[1]
        base = wrap(y * S + x + off, w)
        ev = [("site", 0), ("acc", 0, 0, base, 4, 0, 0)]
        for kk in range(8):
            if kk >= cap:
                ev.append(("hang",))
                return ev
            ev.append(("site", 1))
            j = kk + (1 if kk > 3 else 0)
            dy, dx = (j // 3 - 1) * r, (j % 3 - 1) * r
            ev += [("site", 3), ("acc", 1, 0, wrap(base + dy * S + dx, w), 4, kk, 0)]
        ev += [("site", 2), ("site", 4), ("acc", 2, 1, base, 4, 0, 0)]
        return ev
    return k


# ---- F3 ------------------------------------------------------------------
def f3_model(tables, data, w=32, cap=1 << 20):
    """tables[i] rows give (base, size, data_ref, flags); data[ref-1] arrays."""
    state = {}

    def k(tid, bid, launch, sc):
        nrows = int(sc[0])
        off = int(sc[1]) if w == 64 else 0
        tab = state["tab"]
        row_ptr = data[int(tab[0][2]) - 1]
        col = data[int(tab[1][2]) - 1]
        r = bid[0] * int(launch[3]) + tid[0]
        ev = []
        if not (r < nrows):
            return [("site", 1)]
        ev.append(("site", 0))

        def load(slot, arr, idx, acc, site, i1):
            from brute import kind_of
            ev.append(("site", site))
            ev.append(("acc", acc, slot, idx, 4, i1, 0))
            return 0 if kind_of(tab[slot], idx, 4) else int(arr[idx])

        rp0 = load(0, row_ptr, r, 0, 2, 0)
        rp1 = load(0, row_ptr, r + 1, 1, 3, 0)
        n = max(0, rp1 - rp0)
        for kk in range(min(n, cap)):
            j = rp0 + kk
            ev.append(("site", 4))
            c = load(1, col, j, 2, 6, kk)
            ev += [("site", 7), ("acc", 3, 2, j + off, 4, kk, 0)]
            ev += [("site", 8), ("acc", 4, 3, c + off, 4, kk, 0)]
        if n > cap:
            ev.append(("hang",))
            return ev
        ev += [("site", 5), ("site", 9), ("acc", 5, 4, r + off, 4, 0, 0)]
        return ev

    def bind(i):
        state["tab"] = tables[i]
    return k, bind


# ---- Listing 1: vecAdd with two shared arrays ------------------------------
def listing1_program():
    """Listing 1 as an index program.  Slots: 0 s_a, 1 s_b (blockSize ints,
    per block), 2 a, 3 b, 4 c.  Accesses in evaluation order:
    0 a[id] R, 1 s_a[tx] W, 2 b[id] R, 3 s_b[tx] W, 4 s_a[tx] R, 5 s_b[tx] R,
    6 c[id] W  (seven accesses; the barrier carries no index)."""
    p = Program(n_scalars=0, n_slots=5)
    tx = p.special("tid.x")
    tx32 = p.add(tx, p.const(0, 32), 32)
    idv = p.add(p.mul(p.special("bid.x"), p.special("bdim.x"), 32), tx32, 32)
    p.access(2, idv)
    p.access(0, tx32, write=True)
    p.access(3, idv)
    p.access(1, tx32, write=True)
    p.access(0, tx32)
    p.access(1, tx32)
    p.access(4, idv, write=True)
    return p.to_bytes()


def listing1_model(tid, bid, launch, sc):
    tx = tid[0]
    i = bid[0] * int(launch[3]) + tx
    order = ((2, i), (0, tx), (3, i), (1, tx), (0, tx), (1, tx), (4, i))
    ev = []
    for a, (slot, idx) in enumerate(order):
        ev += [("site", a), ("acc", a, slot, idx, 4, 0, 0)]
    return ev


# ---- Listing 3: guarded vecAdd ------------------------------------------------
def listing3_program():
    """``if (id < N) c[id+1] = a[id+1] + b[id+1]``.  Slots 0 a, 1 b, 2 c;
    scalar 0 = N.  Accesses: 0 a[id+1] R, 1 b[id+1] R, 2 c[id+1] W.
    Sites: 0 guard true, 1 guard false, 2..4 the accesses."""
    p = Program(n_scalars=1, n_slots=3)
    idv = p.add(p.mul(p.special("bid.x"), p.special("bdim.x"), 32), p.special("tid.x"), 32)
    n = p.scalar(0, 32)
    with p.if_(p.cmplts(idv, n, 32)):
        i1 = p.add(idv, p.const(1, 32), 32)
        p.access(0, i1)
        p.access(1, i1)
        p.access(2, i1, write=True)
    return p.to_bytes()


def listing3_model(tid, bid, launch, sc):
    i = bid[0] * int(launch[3]) + tid[0]
    if not (i < int(sc[0])):
        return [("site", 1)]
    ev = [("site", 0)]
    for a in range(3):
        ev += [("site", 2 + a), ("acc", a, a, i + 1, 4, 0, 0)]
    return ev


def simple_workload(ir, launches, tables, scalars=None, mode=W.MODE_FULL, cap=(20, 12), data=()):
    launches = np.asarray(launches, np.uint32).reshape(-1, 6)
    n = launches.shape[0]
    tabs = np.zeros((n, len(tables[0])), W.ALLOC_DTYPE)
    for i in range(n):
        tabs[i] = [tuple(t) + (0,) * (5 - len(t)) if len(t) < 5 else tuple(t) for t in tables[i]]
    if scalars is None:
        scalars = np.zeros((n, 0), np.int64)
    scalars = np.asarray(scalars, np.int64).reshape(n, -1)
    return W.Workload("t", ir, launches, scalars, tabs, np.arange(n, dtype=np.uint32),
                      list(data), mode, tuple(cap))
