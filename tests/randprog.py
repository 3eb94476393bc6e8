"""Random well-formed index programs for differential tests (GPU library vs
oracle).  Programs mix every opcode, both widths, guards, nested loops with
small or huge trip counts, and loads from a small data array, so that guarded,
indirect, capped and faulting paths are all exercised."""
from __future__ import annotations

import numpy as np

from paper_2601_01048_amd.gen.ir import BINARY, Program
from paper_2601_01048_amd.gen import workloads as W

SPECIALS = ["tid.x", "tid.y", "tid.z", "bid.x", "bid.y", "bid.z", "bdim.x", "bdim.y", "bdim.z",
            "gdim.x", "gdim.y", "gdim.z"]


class _Gen:
    def __init__(self, rng, n_scalars, n_slots, budget, loads=True, uniform_only=False):
        self.rng = rng
        self.p = Program(n_scalars=n_scalars, n_slots=n_slots)
        self.scopes = [[]]
        self.budget = budget
        self.loads = loads
        self.uniform_only = uniform_only
        self.n_scalars = n_scalars
        self.n_slots = n_slots

    def vis(self):
        return [r for s in self.scopes for r in s]

    def val(self):
        v = self.vis()
        if not v or self.rng.random() < 0.2:
            return self.leaf()
        return v[int(self.rng.integers(len(v)))]

    def leaf(self):
        r = self.rng.random()
        p = self.p
        if r < 0.35:
            names = SPECIALS[6:] if self.uniform_only else SPECIALS
            x = p.special(names[int(self.rng.integers(len(names)))])
        elif r < 0.6 and self.n_scalars:
            x = p.scalar(int(self.rng.integers(self.n_scalars)), int(self.rng.choice([32, 64])))
        else:
            c = int(self.rng.choice([0, 1, -1, 2, 3, 5, 7, 31, 32, 63, 64, -(1 << 31), (1 << 31) - 1,
                                     1 << 33, -(1 << 63), int(self.rng.integers(-100, 100))]))
            x = p.const(c, int(self.rng.choice([32, 64])))
        self.scopes[-1].append(x)
        return x

    def stmt(self, loop_depth, nest):
        rng, p = self.rng, self.p
        self.budget -= 1
        r = rng.random()
        w = int(rng.choice([32, 64]))
        if r < 0.45:
            op = BINARY[int(rng.integers(len(BINARY)))]
            if self.uniform_only and op in ("MUL", "SHL"):
                op = "ADD"
            x = p.op(op, self.val(), self.val(), w)
        elif r < 0.5:
            x = p.select(self.val(), self.val(), self.val(), w)
        elif r < 0.55:
            x = [p.sext, p.zext, p.trunc][int(rng.integers(3))](self.val())
        elif r < 0.75:
            slot = int(rng.integers(self.n_slots))
            p.access(slot, self.val(), elem=int(rng.choice([1, 2, 4, 8])), write=bool(rng.random() < 0.5),
                     w=w, site=bool(rng.random() < 0.9))
            return
        elif r < 0.82 and self.loads:
            idx = p.op("REMU", self.val(), p.const(int(rng.integers(40, 90)), w), w)
            x = p.load(0, idx, elem=4, w=w)
        elif r < 0.9 and nest < 4:
            with p.if_(self.val(), site_t=bool(rng.random() < 0.9), site_f=bool(rng.random() < 0.9)):
                self.scopes.append([])
                self.block(loop_depth, nest + 1, int(rng.integers(1, 5)))
                self.scopes.pop()
                if rng.random() < 0.4:
                    p.else_()
                    self.scopes.append([])
                    self.block(loop_depth, nest + 1, int(rng.integers(1, 4)))
                    self.scopes.pop()
            return
        elif loop_depth < 2 and nest < 4:
            start = self.val()
            if rng.random() < 0.8:
                end = p.op("ADD", start, p.const(int(rng.integers(-2, 7)), w), w)
            else:
                end = self.val()  # arbitrary: may be huge (capped) or empty
            step = p.const(int(rng.choice([1, 1, 2, -1, 3])), w)
            with p.loop(start, end, step, w=w, site_iter=bool(rng.random() < 0.9),
                        site_exit=bool(rng.random() < 0.9)) as k:
                self.scopes.append([k])
                self.block(loop_depth + 1, nest + 1, int(rng.integers(1, 5)))
                self.scopes.pop()
            return
        else:
            x = self.leaf()
            return
        self.scopes[-1].append(x)

    def block(self, loop_depth, nest, n):
        for _ in range(n):
            if self.budget <= 0:
                break
            self.stmt(loop_depth, nest)


def random_program(rng, n_scalars=2, n_slots=3, budget=40, loads=True, uniform_only=False) -> bytes:
    g = _Gen(rng, n_scalars, n_slots, budget, loads, uniform_only)
    g.block(0, 0, budget)
    # at least one access so the program checks something
    g.p.access(int(rng.integers(n_slots)), g.val(), elem=4)
    return g.p.to_bytes()


def random_workload(rng, ir: bytes, n_inputs=4, n_scalars=2, n_slots=3, mode=W.MODE_FULL,
                    cap=(4, 3)) -> W.Workload:
    launch = np.zeros((n_inputs, 6), np.uint32)
    for i in range(n_inputs):
        launch[i] = [rng.integers(1, 4), rng.integers(1, 3), rng.integers(1, 3),
                     rng.integers(1, 9), rng.integers(1, 4), rng.integers(1, 3)]
    scalars = rng.integers(-5, 40, size=(n_inputs, n_scalars)).astype(np.int64)
    scalars[rng.random(scalars.shape) < 0.1] = (1 << 40) + 3
    data = [rng.integers(-10, 70, size=64).astype(np.int32)]
    tables = np.zeros((n_inputs, n_slots), W.ALLOC_DTYPE)
    for i in range(n_inputs):
        for s in range(n_slots):
            base = W.LOGICAL_BASE + (s << 36)
            flags = 0
            u = rng.random()
            if s > 0 and u < 0.08:
                base = 0
            elif s > 0 and u < 0.16:
                flags = W.ALLOC_FREED
            size = 64 * 4 if s == 0 else int(rng.integers(0, 200))
            tables[i, s] = (base, size, 1 if s == 0 else 0, flags, 0)
    return W.Workload("rand", ir, launch, scalars, tables, np.arange(n_inputs, dtype=np.uint32), data,
                      mode, tuple(cap))


# block-x coefficients around the largest step whose 16-block progressions
# cannot wrap (0x7FFFFFFF // 15 = 143165576), and ordinary ones
GRID_STEPS = [1, 16, 256, -1, -16, 4096, 143165576, 143165577, -143165576, -143165577, 1 << 30, -(1 << 30)]


def affine_grid_program(rng, k_bx: int, n_acc: int = 4) -> bytes:
    """Width-32 accesses sharing one linear part in the thread and block
    coordinates (k_bx per block along x, random small coefficients
    elsewhere, scalar 0 added) at different constant offsets: the shape the
    block-major trace evaluator takes, over grids wide enough for whole
    groups of 16 blocks in one row."""
    p = Program(n_scalars=1, n_slots=2)
    tx, bx, by = p.special("tid.x"), p.special("bid.x"), p.special("bid.y")
    base = p.add(p.mul(bx, p.const(k_bx, 32), 32), p.mul(tx, p.const(int(rng.choice([1, 2, -1])), 32), 32), 32)
    base = p.add(base, p.mul(by, p.const(int(rng.choice([0, 1000, 5000, -3000])), 32), 32), 32)
    base = p.add(base, p.scalar(0, 32), 32)
    for _ in range(n_acc):
        p.access(int(rng.integers(2)), p.add(base, p.const(int(rng.integers(-70, 70)), 32), 32), elem=4)
    return p.to_bytes()


def affine_grid_workload(rng, ir: bytes, k_bx: int, n_inputs: int = 6) -> W.Workload:
    """Grids of 16 to 70 blocks along x (1 or 2 rows) of 64 threads; scalar 0
    and the allocation sizes put the bounds anywhere in the index range, so
    some groups are clean, some cross a bound at one end, and inputs with a
    freed or NULL slot take the general path."""
    launch = np.zeros((n_inputs, 6), np.uint32)
    scalars = np.zeros((n_inputs, 1), np.int64)
    tables = np.zeros((n_inputs, 2), W.ALLOC_DTYPE)
    for i in range(n_inputs):
        gx, gy = int(rng.integers(16, 71)), int(rng.integers(1, 3))
        launch[i] = [gx, gy, 1, 64, 1, 1]
        span = abs(k_bx) * gx + 64 * 2 + 6000 * gy
        s0 = int(rng.choice([0, 100, -50, abs(k_bx) * gx // 2 if k_bx < 0 else 0, (1 << 31) - 10]))
        scalars[i, 0] = s0 if s0 < (1 << 31) else s0 - (1 << 32)
        for s in range(2):
            u = rng.random()
            if u < 0.5:
                size = (1 << 31) - 1  # every non-negative 32-bit index
            elif u < 0.8:
                size = int(rng.integers(1, min(span, 1 << 31)))
            else:
                size = int(rng.integers(1, 5000))
            base, flags = W.LOGICAL_BASE + (s << 36), 0
            u = rng.random()
            if s == 1 and u < 0.1:
                base = 0
            elif s == 1 and u < 0.2:
                flags = W.ALLOC_FREED
            tables[i, s] = (base, 4 * size, 0, flags, 0)
    return W.Workload("affine_grid", ir, launch, scalars, tables, np.arange(n_inputs, dtype=np.uint32), [],
                      W.MODE_FULL, (4, 3))


def grid3d_program(rng, n_acc: int = 5) -> bytes:
    """Width-32 accesses sharing one linear part in all six coordinates
    (nonzero tid.z and bid.z coefficients) at different constant offsets: one
    coefficient class, so 64-thread blocks take the block-major trace layout
    with the z parts of the thread and block walks in use."""
    p = Program(n_scalars=1, n_slots=2)
    coef = [int(rng.choice(v)) for v in ((1, 2, -1), (16, 40, -16), (32, 100, -70), (64, 3, -64),
                                          (2048, 700, -999), (65536, 9000, -40000))]
    names = ("tid.x", "tid.y", "tid.z", "bid.x", "bid.y", "bid.z")
    base = p.scalar(0, 32)
    for nm, k in zip(names, coef):
        base = p.add(base, p.mul(p.special(nm), p.const(k, 32), 32), 32)
    for _ in range(n_acc):
        p.access(int(rng.integers(2)), p.add(base, p.const(int(rng.integers(-90, 90)), 32), 32), elem=4)
    return p.to_bytes()


def grid3d_workload(rng, ir: bytes, n_inputs: int = 8) -> W.Workload:
    """3-D grids (gx 16..40, gy 1..3, gz 2..4) of 16x2x2 blocks: jobs cross
    x, y and z wraps; scalar 0 and the allocation sizes put bounds inside
    the grid's index range, so some blocks violate and most do not."""
    launch = np.zeros((n_inputs, 6), np.uint32)
    scalars = np.zeros((n_inputs, 1), np.int64)
    tables = np.zeros((n_inputs, 2), W.ALLOC_DTYPE)
    for i in range(n_inputs):
        launch[i] = [int(rng.integers(16, 41)), int(rng.integers(1, 4)), int(rng.integers(2, 5)), 16, 2, 2]
        scalars[i, 0] = int(rng.choice([0, 50, 200000, 400000]))
        for s in range(2):
            u = rng.random()
            size = (1 << 31) - 1 if u < 0.3 else int(rng.integers(1, 600000))
            tables[i, s] = (W.LOGICAL_BASE + (s << 36), 4 * size, 0, 0, 0)
    return W.Workload("grid3d", ir, launch, scalars, tables, np.arange(n_inputs, dtype=np.uint32), [],
                      W.MODE_FULL, (4, 3))


def segment_program(k_bx: int, k_by: int, offsets=(-3, 0, 5, 70)) -> bytes:
    """idx = k_bx*bid.x + k_by*bid.y + tid.x + s0 + off (width 32): the block
    bases of a grid row form one arithmetic progression with step k_bx."""
    p = Program(n_scalars=1, n_slots=2)
    base = p.add(p.mul(p.special("bid.x"), p.const(k_bx, 32), 32), p.special("tid.x"), 32)
    base = p.add(base, p.mul(p.special("bid.y"), p.const(k_by, 32), 32), 32)
    base = p.add(base, p.scalar(0, 32), 32)
    for k, off in enumerate(offsets):
        p.access(k % 2, p.add(base, p.const(off, 32), 32), elem=4)
    return p.to_bytes()


def segment_workload(rng, ir: bytes, k_bx: int, k_by: int, offsets=(-3, 0, 5, 70),
                     n_inputs: int = 8) -> W.Workload:
    """Whole grids of 64-thread blocks with 70..127 blocks per row and 3..7
    rows, so a job of 256 blocks covers 3 or 4 row segments (partial first
    row, whole rows, partial last row).  Bounds are set from the index at a
    chosen block that ends a row inside a job (x = gx-1 or x = 0, not the
    job's first or last block), so the only violations sit at interior
    segment ends and next to them."""
    def idx(bx, by, tx, s0, off):
        v = (k_bx * bx + k_by * by + tx + s0 + off) & 0xFFFFFFFF
        return v - (1 << 32) if v >= (1 << 31) else v

    launch = np.zeros((n_inputs, 6), np.uint32)
    scalars = np.zeros((n_inputs, 1), np.int64)
    tables = np.zeros((n_inputs, 2), W.ALLOC_DTYPE)
    for i in range(n_inputs):
        gx, gy = int(rng.integers(70, 128)), int(rng.integers(3, 8))
        launch[i] = [gx, gy, 1, 64, 1, 1]
        s0 = int(rng.choice([0, 7, 1 << 20]))
        scalars[i, 0] = s0
        # a row end strictly inside the first job (blocks 0..255)
        row = int(rng.integers(0, min(gy, 256 // gx)))
        bx = gx - 1 if k_bx >= 0 else 0
        if row * gx + bx in (0, 255) or row * gx + bx > 255:
            row, bx = 0, gx - 1 if k_bx >= 0 else 1
        for s in range(2):
            offs = [o for k, o in enumerate(offsets) if k % 2 == s]
            hi = max(idx(bx, row, 63, s0, o) for o in offs)
            u = rng.random()
            if u < 0.6 and 0 < hi < (1 << 31) - 1:
                size = hi  # exactly the largest index at that block is out of bounds
            elif u < 0.8:
                size = (1 << 31) - 1
            else:
                size = int(rng.integers(1, 1 << 31))
            tables[i, s] = (W.LOGICAL_BASE + (s << 36), 4 * size, 0, 0, 0)
    return W.Workload("segments", ir, launch, scalars, tables, np.arange(n_inputs, dtype=np.uint32), [],
                      W.MODE_FULL, (4, 3))
