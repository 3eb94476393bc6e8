"""Random programs whose expandable loop body has the shape of an indirect
gather (loads feeding indices, indices built from the counter and loaded
values with uniform coefficients), plus near misses that must stay on the
interpreter.  For differential tests of the library against the oracle."""
from __future__ import annotations

import numpy as np

from paper_2601_01048_amd.gen.ir import Program
from paper_2601_01048_amd.gen import workloads as W

LB = W.LOGICAL_BASE


def gather_program(rng, near_miss: bool = False):
    """Slots: 0 data D (int32, loaded), 1 data E (int64, loaded), 2 and 3
    address-only.  Scalars: 0..2 uniform coefficients (any width)."""
    p = Program(n_scalars=3, n_slots=4)
    lw = int(rng.choice([32, 64]))
    t = p.special("tid.x")
    b = p.special("bid.x")
    # varying trip count: 0..6 per thread, start from a load or a uniform value
    trips = p.remu(p.add(t, p.mul(b, p.const(3, 32), 32), 32), p.const(7, 32), 32)
    if rng.random() < 0.5:
        start = p.load(0, p.remu(t, p.const(16, 32), 32), elem=4, w=32)
    else:
        start = p.scalar(0, lw)
    end = p.add(start, trips, lw)
    step = p.const(int(rng.choice([1, 1, 2, -1])), lw)
    if int(step.idx) >= 0 and rng.random() < 0.2:
        end = p.sub(start, trips, lw)  # zero trips for positive steps
    with p.loop(start, end, step, w=lw) as j:
        vals = [j]  # varying values available in the body
        n_ops = int(rng.integers(2, 7))
        for _ in range(n_ops):
            x = vals[int(rng.integers(len(vals)))]
            w = int(rng.choice([32, 64, lw, lw]))
            r = rng.random()
            u = p.scalar(int(rng.integers(3)), w) if rng.random() < 0.5 else p.const(int(rng.integers(-5, 6)), w)
            if r < 0.2:
                y = p.add(x, u, w)
            elif r < 0.3:
                y = p.sub(u, x, w)
            elif r < 0.4:
                y = p.mul(x, u, w)
            elif r < 0.45:
                y = p.shl(x, p.const(int(rng.integers(0, 3)), w), w)
            elif r < 0.55 and len(vals) > 1:
                y = p.add(x, x, w)
            elif r < 0.7:
                y = p.load(0, x, elem=4, w=w)
            elif r < 0.8:
                y = p.load(1, x, elem=8, w=w)
            else:
                p.access(int(rng.integers(2, 4)), x, elem=int(rng.choice([4, 8])), w=w)
                continue
            vals.append(y)
        # uniform work inside the body, including a division by a scalar that may be 0
        q = p.divs(p.scalar(1, 64), p.scalar(2, 64), 64)
        p.access(2, p.add(vals[-1], q, 64), elem=4, w=64)
        if near_miss:
            kind = int(rng.integers(4))
            if kind == 0:
                p.access(3, p.add(vals[-1], t, 32), w=32)          # thread coordinate in the body
            elif kind == 1:
                c = p.load(0, j, elem=4, w=lw)
                p.access(3, p.add(j, c, lw), w=lw)                   # two variables
            elif kind == 2:
                with p.if_(p.cmplts(j, p.const(2, lw), lw)):         # control flow in the body
                    p.access(3, j, w=lw)
            else:
                c = p.load(0, j, elem=4, w=lw)
                p.access(3, p.mul(j, c, lw), w=lw)                   # product of varying values
        p.access(3, vals[int(rng.integers(len(vals)))], w=int(rng.choice([32, 64])))
    p.access(3, trips, w=32)
    return p.to_bytes()


def gather_workload(rng, ir, n_inputs=4):
    D = rng.integers(-20, 60, size=64).astype(np.int32)
    E = rng.integers(-20, 60, size=32).astype(np.int64)
    launches, tables, scalars = [], [], []
    for i in range(n_inputs):
        launches.append([int(rng.integers(1, 4)), 1, 1, int(rng.choice([5, 64, 100])), 1, 1])
        dead = int(rng.integers(4))
        s2 = (0, 0, 0, 0) if dead == 0 else ((LB, 160, 0, 1) if dead == 1 else (LB, int(rng.integers(0, 400)), 0, 0))
        tables.append([(LB, 4 * 64, 1, 0), (LB + (1 << 36), 8 * 32, 2, 0), s2,
                       (LB + (3 << 36), int(rng.integers(8, 600)), 0, 0)])
        scalars.append([int(rng.integers(-8, 9)), int(rng.integers(-50, 50)), int(rng.choice([0, 1, 3, -2]))])
    launches = np.asarray(launches, np.uint32)
    tabs = np.zeros((n_inputs, 4), W.ALLOC_DTYPE)
    for i in range(n_inputs):
        tabs[i] = [t + (0,) for t in tables[i]]
    return W.Workload("gather", ir, launches, np.asarray(scalars, np.int64), tabs,
                      np.arange(n_inputs, dtype=np.uint32), [D, E], W.MODE_FULL, (20, 12))


def csr_runs_workload(seed: int, log2_rows: int = 15, n_inputs: int = 4, col_short: int = 0):
    """CSR gathers (the F3 program) whose row pointers exercise how the gather
    pass joins consecutive contiguous tiles of 256 rows into one run:
    input 0 a plain matrix (every tile continues the one before); input 1
    tile boundaries where the last row of a tile runs backwards, so the next
    tile restarts below the previous end (each tile contiguous, the chain
    broken); input 2 whole tiles of empty rows and a short last tile; input 3
    rows running backwards inside tiles (tiles not contiguous).  Every input
    has its own corrupted col_idx, a val allocation that ends before the last
    nonzeros (violations in late tiles of long runs) and an x allocation short
    of ncols (violations spread over every tile).  col_short > 0 also ends the
    col_idx allocation that many elements before the last nonzero (the loaded
    index runs out of bounds inside the last run)."""
    rng = np.random.default_rng(seed)
    data, tables, launch, scalars = [], [], [], []
    for i in range(n_inputs):
        nrows = (1 << log2_rows) - (77 if i == 2 else 0)
        ncols = 1 << log2_rows
        L = W.powerlaw_row_lengths(rng, nrows, ncols, 16)
        if i == 2:  # empty tiles
            for t in rng.choice(nrows // 256 - 1, size=12, replace=False):
                L[256 * t:256 * (t + 1)] = 0
        rp = np.zeros(nrows + 1, np.int64)
        np.cumsum(L, out=rp[1:])
        if i == 1:  # backward last rows at tile boundaries
            for t in rng.choice(np.arange(1, nrows // 256), size=20, replace=False):
                rp[256 * t] = rp[256 * t - 1] - int(rng.integers(1, 9))
        if i == 3:  # backward rows inside tiles
            for r in rng.choice(nrows - 2, size=15, replace=False) + 1:
                rp[r] = max(0, rp[r - 1] - int(rng.integers(1, 9)))
        nnz = int(rp.max())
        col = rng.integers(0, ncols, size=nnz, dtype=np.int64).astype(np.int32)
        col = W.corrupt_copy(rng, col, ncols, 0.002)
        data += [rp.astype(np.int32), col]
        val_len = nnz - int(rng.integers(1, 2000))
        tables.append([W.alloc((nrows + 1) * 4, len(data) - 1, W.LOGICAL_BASE),
                       W.alloc((nnz - col_short) * 4, len(data), W.LOGICAL_BASE + (1 << 36)),
                       W.alloc(val_len * 4, 0, W.LOGICAL_BASE + (2 << 36)),
                       W.alloc((ncols - int(rng.integers(100, 1000))) * 4, 0, W.LOGICAL_BASE + (3 << 36)),
                       W.alloc(nrows * 4, 0, W.LOGICAL_BASE + (4 << 36))])
        launch.append([(nrows + 255) // 256, 1, 1, 256, 1, 1])
        scalars.append([nrows])
    return W.Workload("csr_runs", W.f3_program(32), np.array(launch, np.uint32), np.array(scalars, np.int64),
                      np.array([[tuple(a) for a in t] for t in tables], dtype=W.ALLOC_DTYPE),
                      np.arange(n_inputs, dtype=np.uint32), data, W.MODE_FULL)


def long_gather_program(rng):
    """Contiguous 32-bit gathers over long ranges: thread gid of the grid runs
    j over [gid*L + s, gid*L + s + L) (scalar 0 = s, scalar 1 = L), so every
    tile is contiguous and whole rounds of the contiguous form occur.  The body
    has two to four entries of width 32: loads from D (int32, slot 0) or E
    (int64, slot 1) and address-only accesses (slots 2, 3), indexed by the
    counter or a loaded value (coefficient 1 or 2, constant or scalar offsets)
    or by a constant."""
    p = Program(n_scalars=3, n_slots=4)
    gid = p.add(p.mul(p.special("bid.x"), p.special("bdim.x"), 32), p.special("tid.x"), 32)
    L = p.scalar(1, 32)
    start = p.add(p.mul(gid, L, 32), p.scalar(0, 32), 32)
    with p.loop(start, p.add(start, L, 32), 1, w=32) as j:
        vals, n_load = [j], 0
        for _ in range(int(rng.integers(2, 5))):
            src = vals[int(rng.integers(len(vals)))]
            k = rng.random()
            if k < 0.3:
                idx = src
            elif k < 0.55:
                idx = p.add(src, p.const(int(rng.integers(-3, 4)), 32), 32)
            elif k < 0.7:
                idx = p.mul(src, p.const(2, 32), 32)
            elif k < 0.85:
                idx = p.add(src, p.scalar(2, 32), 32)
            else:
                idx = p.const(int(rng.integers(0, 40)), 32)
            if n_load < 2 and rng.random() < 0.5:
                slot, elem = (0, 4) if rng.random() < 0.6 else (1, 8)
                vals.append(p.load(slot, idx, elem=elem, w=32))
                n_load += 1
            else:
                p.access(int(rng.integers(2, 4)), idx, elem=int(rng.choice([4, 8])), w=32)
    return p.to_bytes()


def long_gather_workload(rng, ir, n_inputs=4, blocks=2, L_range=(40, 100)):
    """Inputs of long_gather_program: `blocks` blocks of 256 threads, L drawn
    from L_range, start offsets that may be negative, loaded allocations that
    cover the whole counter range or end inside it, address-only allocations
    of any size, freed or NULL."""
    span = blocks * 256 * L_range[1] + 256
    n = 2 * span + 64
    D = rng.integers(-40, span + 40, size=n).astype(np.int32)
    E = rng.integers(-40, span + 40, size=n).astype(np.int64)
    launches, tables, scalars = [], [], []
    for i in range(n_inputs):
        launches.append([blocks, 1, 1, 256, 1, 1])
        L = int(rng.integers(L_range[0], L_range[1] + 1))
        s = int(rng.choice([0, 0, int(rng.integers(-50, 0)), int(rng.integers(1, 200))]))
        scalars.append([s, L, int(rng.integers(-8, 9))])
        used = blocks * 256 * L + max(s, 0) + 8

        def loaded(elem):
            return n * elem if rng.random() < 0.5 else int(rng.integers(used // 2, used)) * elem

        def addr_only():
            r = rng.random()
            if r < 0.15:
                return (0, 64, 0, 0)  # NULL
            if r < 0.3:
                return (LB + (2 << 36), 4 * used, 0, W.ALLOC_FREED)
            return (LB + (2 << 36), int(rng.integers(0, 8 * used)), 0, 0)
        tables.append([(LB, loaded(4), 1, 0), (LB + (1 << 36), loaded(8), 2, 0), addr_only(), addr_only()])
    tabs = np.zeros((n_inputs, 4), W.ALLOC_DTYPE)
    for i in range(n_inputs):
        tabs[i] = [t + (0,) for t in tables[i]]
    return W.Workload("long_gather", ir, np.asarray(launches, np.uint32), np.asarray(scalars, np.int64), tabs,
                      np.arange(n_inputs, dtype=np.uint32), [D, E], W.MODE_FULL, (20, 12))
