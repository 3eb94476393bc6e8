"""Kernels with shared memory, barriers and floating-point data math, each
with a block-level model written from the kernel's own formula.

The IR's shared-memory semantics (``include/ckc_ir.h``): each block has its
own instance of every shared slot, all zero at the start; a LOAD sees the
instance as at the start of the current phase (phases are separated by
BARRIERs); at the end of a phase every element written in it takes the
largest value written to it.  ``BlockSim`` holds that state; the models call
it in the kernel's own order.  Nothing here reads the IR, so the models pin
the oracle's block runner, and through it the device.

Slots: 0 = A (global int32 array, the accesses whose indices are checked),
1 = sh (shared int32 array), 2 = G (global int32 data, where a kernel reads
data).  Every access instruction has its own coverage site, in program order.
"""
from __future__ import annotations

import math
import struct

import numpy as np

import brute
from paper_2601_01048_amd.gen import workloads as W
from paper_2601_01048_amd.gen.ir import Program

LB = W.LOGICAL_BASE
SH_BASE = 0x100


def w32(v: int) -> int:
    v &= 0xFFFFFFFF
    return v - (1 << 32) if v >> 31 else v


def f2bits(x: float) -> int:
    return struct.unpack("<q", struct.pack("<d", x))[0]


def ftoi(x: float, w: int) -> int:
    """Truncation toward zero, NaN 0, out-of-range values saturated."""
    lo, hi = -(1 << (w - 1)), (1 << (w - 1)) - 1
    if x != x:
        return 0
    if x <= lo:
        return lo
    if x >= hi + 1:
        return hi
    return int(x)  # int() truncates toward zero


class BlockSim:
    """Shared memory of one block."""

    def __init__(self, table, spaces):
        self.cur, self.pend = {}, {}
        for s, e in enumerate(table):
            if s < len(spaces) and spaces[s] == 1 and int(e[0]) != 0:
                self.cur[s] = [0] * (int(e[1]) // 4)
                self.pend[s] = {}

    def store(self, slot, idx, val):
        v = w32(val)
        p = self.pend[slot]
        p[idx] = max(p.get(idx, v), v)

    def load(self, slot, idx):
        return self.cur[slot][idx]

    def barrier(self):
        for s, p in self.pend.items():
            for i, v in p.items():
                self.cur[s][i] = v
            p.clear()


class Thr:
    """One thread's events; accesses are checked by the definition."""

    def __init__(self, tl, tid, bid, table, data, sim):
        self.tl, self.tid, self.bid = tl, tid, bid
        self.table, self.data, self.sim = table, data, sim
        self.ev = []

    def acc(self, a, slot, idx, site, i1=0):
        self.ev += [("site", site), ("acc", a, slot, idx, 4, i1, 0)]
        return brute.kind_of(self.table[slot], idx, 4)

    def store(self, a, slot, idx, val, site, i1=0):
        if self.acc(a, slot, idx, site, i1) == 0 and slot in self.sim.cur:
            self.sim.store(slot, idx, val)

    def load(self, a, slot, idx, site, i1=0):
        if self.acc(a, slot, idx, site, i1):
            return 0
        if slot in self.sim.cur:
            return self.sim.load(slot, idx)
        ref = int(self.table[slot][2])
        return int(self.data[ref - 1][idx])

    def divs(self, x, y):
        """Signed 32-bit division: by zero 0 and an arithmetic fault."""
        x, y = w32(x), w32(y)
        if y == 0:
            self.ev.append(("fault",))
            return 0
        if x == -(1 << 31) and y == -1:
            return x
        q = abs(x) // abs(y)
        return q if (x < 0) == (y < 0) else -q


def block_threads(launch, blin):
    gx, gy, gz, bx, by, bz = (int(v) for v in launch)
    bid = (blin % gx, (blin // gx) % gy, blin // (gx * gy))
    bs = bx * by * bz
    return [(t, (t % bx, (t // bx) % by, t // (bx * by)), bid) for t in range(bs)]


def expected(case, launches, tables, scalars=None, data=(), mode="full"):
    """Brute-force records, counts and status of a block model over whole
    blocks (modes "full" and "boundary")."""
    out = ([], [], [])
    for i, launch in enumerate(launches):
        memo = {}
        sc = None if scalars is None else scalars[i]
        tab = tables[i]

        def kernel(tid, bid, launch, sc, tab=tab, memo=memo):
            gx, gy = int(launch[0]), int(launch[1])
            blin = bid[0] + gx * (bid[1] + gy * bid[2])
            if blin not in memo:
                sim = BlockSim(tab, case.spaces)
                T = [Thr(tl, t, b, tab, data, sim) for tl, t, b in block_threads(launch, blin)]
                case.model(sim, T, launch, sc)
                memo[blin] = {t.tid: t.ev for t in T}
            return memo[blin][tuple(tid)]

        r, c, s = brute.run(kernel, [launch], [tab], case.n_acc, case.n_sites, mode=mode, L=case.L,
                            scalars=None if sc is None else [sc])
        out[0].append(r[0])
        out[1].append(c[0])
        out[2].append(s[0])
    return out


class Case:
    def __init__(self, name, p: Program, model, n_scalars=0):
        self.name, self.model = name, model
        self.spaces = list(p.spaces)
        self.ir = p.to_bytes()
        self.n_acc = p.n_accesses
        self.n_sites = len(p.site_ids)
        self.n_instr = len(p.instrs)
        self.n_scalars = n_scalars
        self.L = (0, 0)  # key bits of loop iterations (depth-1 programs: 20, 0)


def _tl(p: Program, dims: int):
    """Linear thread index in the block (32-bit)."""
    tx = p.trunc(p.special("tid.x"))
    if dims == 1:
        return tx
    bx = p.trunc(p.special("bdim.x"))
    by = p.trunc(p.special("bdim.y"))
    ty = p.trunc(p.special("tid.y"))
    tz = p.trunc(p.special("tid.z"))
    return p.add(tx, p.mul(bx, p.add(ty, p.mul(by, tz))))


def _bs(p: Program, dims: int):
    b = p.trunc(p.special("bdim.x"))
    if dims == 1:
        return b
    return p.mul(b, p.mul(p.trunc(p.special("bdim.y")), p.trunc(p.special("bdim.z"))))


def _bsize(launch):
    return int(launch[3]) * int(launch[4]) * int(launch[5])


# ---- the kernels --------------------------------------------------------------

def rotate(k=3, c=-7, dims=1):
    """sh[t] = t*k + c; barrier; A[sh[(t + 1) mod bs]]."""
    p = Program(n_slots=2, spaces=[0, 1])
    t = _tl(p, dims)
    p.store(1, t, p.add(p.mul(t, k), c))
    p.barrier()
    u = p.load(1, p.remu(p.add(t, 1), _bs(p, dims)))
    p.access(0, u)

    def model(B, T, launch, sc):
        bs = _bsize(launch)
        for x in T:
            x.store(0, 1, x.tl, x.tl * k + c, 0)
        B.barrier()
        for x in T:
            u = x.load(1, 1, (x.tl + 1) % bs, 1)
            x.acc(2, 0, u, 2)
    return Case(f"rotate{dims}d", p, model)


def racing_max(d=5):
    """All threads write sh[0] = t - d and sh[1] = 5 - 3t; barrier;
    A[sh[0]], A[sh[1]]: the largest value of each, signed."""
    p = Program(n_slots=2, spaces=[0, 1])
    t = _tl(p, 1)
    z, one = p.const(0, 32), p.const(1, 32)
    p.store(1, z, p.sub(t, d))
    p.store(1, one, p.sub(p.const(5, 32), p.mul(t, 3)))
    p.barrier()
    a = p.load(1, z)
    b = p.load(1, one)
    p.access(0, a)
    p.access(0, b)

    def model(B, T, launch, sc):
        for x in T:
            x.store(0, 1, 0, x.tl - d, 0)
            x.store(1, 1, 1, 5 - 3 * x.tl, 1)
        B.barrier()
        for x in T:
            a = x.load(2, 1, 0, 2)
            b = x.load(3, 1, 1, 3)
            x.acc(4, 0, a, 4)
            x.acc(5, 0, b, 5)
    return Case("racing_max", p, model)


def phases():
    """A load sees its phase's start; unwritten elements keep their value:
    sh[t] = t + 100; A[sh[t]] (0); barrier; even t: sh[t] = 2t + 1;
    b = sh[t] (t + 100); barrier; c = sh[t]; A[b]; A[c]."""
    p = Program(n_slots=2, spaces=[0, 1])
    t = _tl(p, 1)
    p.store(1, t, p.add(t, 100))
    a = p.load(1, t)
    p.access(0, a)
    p.barrier()
    with p.if_(p.cmpeq(p.op("AND", t, 1), 0), site_t=False, site_f=False):
        p.store(1, t, p.add(p.mul(t, 2), 1))
    b = p.load(1, t)
    p.barrier()
    c = p.load(1, t)
    p.access(0, b)
    p.access(0, c)

    def model(B, T, launch, sc):
        for x in T:
            x.store(0, 1, x.tl, x.tl + 100, 0)
            x.acc(2, 0, x.load(1, 1, x.tl, 1), 2)
        B.barrier()
        bv = {}
        for x in T:
            if x.tl % 2 == 0:
                x.store(3, 1, x.tl, 2 * x.tl + 1, 3)
            bv[x.tl] = x.load(4, 1, x.tl, 4)
        B.barrier()
        for x in T:
            c = x.load(5, 1, x.tl, 5)
            x.acc(6, 0, bv[x.tl], 6)
            x.acc(7, 0, c, 7)
    return Case("phases", p, model)


def shared_divisor():
    """sh[t] = t mod 3; barrier; q = 60 / sh[(t + 1) mod bs] (a fault when
    0); A[t]: the shared value reaches only a division."""
    p = Program(n_slots=2, spaces=[0, 1])
    t = _tl(p, 1)
    p.store(1, t, p.remu(t, 3))
    p.barrier()
    v = p.load(1, p.remu(p.add(t, 1), _bs(p, 1)))
    p.divs(p.const(60, 32), v)
    p.access(0, t)

    def model(B, T, launch, sc):
        bs = _bsize(launch)
        for x in T:
            x.store(0, 1, x.tl, x.tl % 3, 0)
        B.barrier()
        for x in T:
            v = x.load(1, 1, (x.tl + 1) % bs, 1)
            x.divs(60, v)
            x.acc(2, 0, x.tl, 2)
    return Case("shared_divisor", p, model)


def bounds(off=-3):
    """sh[t + off] = 7 (some out of bounds: reported, nothing written);
    barrier; v = sh[t - 2] (0 below the start); A[v + t]."""
    p = Program(n_slots=2, spaces=[0, 1])
    t = _tl(p, 1)
    p.store(1, p.add(t, off), p.const(7, 32))
    p.barrier()
    v = p.load(1, p.sub(t, 2))
    p.access(0, p.add(v, t))

    def model(B, T, launch, sc):
        for x in T:
            x.store(0, 1, x.tl + off, 7, 0)
        B.barrier()
        for x in T:
            v = x.load(1, 1, x.tl - 2, 1)
            x.acc(2, 0, v + x.tl, 2)
    return Case(f"bounds{off}", p, model)


def tile_gather():
    """A tile of data into shared memory, then used as indices: sh[t] = G[b*bs
    + t]; barrier; A[sh[bs - 1 - t]] (the data-dependent indices a kernel
    reads from a shared tile)."""
    p = Program(n_slots=3, spaces=[0, 1, 0])
    t = _tl(p, 1)
    bs = _bs(p, 1)
    g = p.add(p.mul(p.trunc(p.special("bid.x")), bs), t)
    p.store(1, t, p.load(2, g))
    p.barrier()
    p.access(0, p.load(1, p.sub(p.sub(bs, 1), t)))

    def model(B, T, launch, sc):
        bs = _bsize(launch)
        for x in T:
            v = x.load(0, 2, x.bid[0] * bs + x.tl, 0)
            x.store(1, 1, x.tl, v, 1)
        B.barrier()
        for x in T:
            x.acc(3, 0, x.load(2, 1, bs - 1 - x.tl, 2), 3)
    return Case("tile_gather", p, model)


def prefix_max():
    """sh[t] = (7t mod 13) + 1; barrier; for j < t: m[t] = sh[j] (the writes
    of one phase keep the largest, so m[t] is the largest of sh[0..t)); barrier;
    A[m[t]]: a kept barrier around a loop of shared loads and stores (m is sh
    from element 256 on)."""
    p = Program(n_slots=2, spaces=[0, 1])
    t = _tl(p, 1)
    p.store(1, t, p.add(p.remu(p.mul(t, 7), 13), 1))
    p.barrier()
    m = p.add(p.const(256, 32), t)
    with p.loop(0, t, site_iter=False, site_exit=False) as j:
        p.store(1, m, p.load(1, j))
    p.barrier()
    p.access(0, p.load(1, m))

    def model(B, T, launch, sc):
        for x in T:
            x.store(0, 1, x.tl, (7 * x.tl) % 13 + 1, 0)
        B.barrier()
        for x in T:
            for j in range(x.tl):
                x.store(2, 1, 256 + x.tl, x.load(1, 1, j, 1, i1=j), 2, i1=j)
        B.barrier()
        for x in T:
            x.acc(4, 0, x.load(3, 1, 256 + x.tl, 3), 4)
    c = Case("prefix_max", p, model)
    c.L = (20, 0)
    return c


def hist_like(nbins=16):
    """A block histogram whose counts no index reads: x = G[b*bs + t];
    sh[x mod nbins] = sh[x mod nbins] + 1; barrier; the counts are written
    out (to A[b*nbins + t] for t < nbins).  The pruned program drops the
    increment and the barrier; the accesses stay."""
    p = Program(n_slots=3, spaces=[0, 1, 0])
    t = _tl(p, 1)
    g = p.add(p.mul(p.trunc(p.special("bid.x")), _bs(p, 1)), t)
    b = p.remu(p.load(2, g), nbins)
    v = p.load(1, b)
    n0 = len(p.instrs)
    inc = p.add(v, 1)
    p.store(1, b, inc)
    p.barrier()
    n_drop = 3  # CONST 1, ADD, BARRIER
    assert len(p.instrs) - n0 == 4
    with p.if_(p.cmpltu(t, nbins), site_t=False, site_f=False):
        c = p.load(1, t)
        p.store(0, p.add(p.mul(p.trunc(p.special("bid.x")), nbins), t), c)

    def model(B, T, launch, sc):
        bs = _bsize(launch)
        for x in T:
            xv = x.load(0, 2, x.bid[0] * bs + x.tl, 0)
            bb = (xv & 0xFFFFFFFF) % nbins
            x.load(1, 1, bb, 1)
            x.store(2, 1, bb, 0, 2)
        for x in T:
            if x.tl < nbins:
                x.load(3, 1, x.tl, 3)
                x.acc(4, 0, x.bid[0] * nbins + x.tl, 4)
    c = Case("hist_like", p, model)
    c.n_drop = n_drop
    c.values_free = True  # the model does not track shared values (no index reads them)
    return c


def ep_like(n_fp=12, scale=0.37, off=-3.3):
    """Data math the indices do not need (a chain of FP operations whose
    result is only written out) next to an index computed through FP:
    i = b*bs + t; A[FTOI(ITOF(i) * scale + off)]; the chain ends in a STORE
    to A[i]."""
    p = Program(n_slots=2, spaces=[0, 0])
    t = _tl(p, 1)
    i = p.add(p.mul(p.trunc(p.special("bid.x")), _bs(p, 1)), t)
    fi = p.itof(i)
    k = p.ftoi(p.fop("FADD", p.fop("FMUL", fi, p.const(f2bits(scale), 64)), p.const(f2bits(off), 64)))
    p.access(0, k)
    n0 = len(p.instrs)
    x = p.fop("FMUL", fi, p.const(f2bits(1e-3), 64))
    for q in range(n_fp):
        x = p.fop("FEXP" if q % 3 == 0 else ("FSUB" if q % 3 == 1 else "FMUL"), x,
                  None if q % 3 == 0 else p.const(f2bits(0.5 + q), 64))
    v = p.ftoi(x)
    n_data = len(p.instrs) - n0
    p.store(1, i, v)

    def model(B, T, launch, sc):
        bs = _bsize(launch)
        for th in T:
            ii = th.bid[0] * bs + th.tl
            th.acc(0, 0, ftoi(float(ii) * scale + off, 32), 0)
            th.acc(1, 1, ii, 1)
    c = Case("ep_like", p, model)
    c.n_data = n_data  # instructions the pruned program drops
    return c


def fp_index(consts):
    """A[FTOI_w(c)] for double constants c given as scalars (bit patterns):
    width 32 and 64 conversions, NaN, infinities, saturation, truncation."""
    p = Program(n_scalars=len(consts), n_slots=1)
    for k in range(len(consts)):
        x = p.scalar(k, 64)
        p.access(0, p.ftoi(x, 32))
        p.access(0, p.ftoi(x, 64), w=64)

    def model(B, T, launch, sc):
        for th in T:
            for k, c in enumerate(consts):
                th.acc(2 * k, 0, ftoi(c, 32), 2 * k)
                th.acc(2 * k + 1, 0, ftoi(c, 64), 2 * k + 1)
    return Case("fp_index", p, model, n_scalars=len(consts))


def fp_arith(a=-2.75, b=1e-3):
    """A[FTOI(ITOF(t - 9) * a - b + (t * 0.1))]: ITOF of negative values,
    FMUL, FSUB, FADD in order, each rounded on its own."""
    p = Program(n_slots=1)
    t = _tl(p, 1)
    x = p.fop("FSUB", p.fop("FMUL", p.itof(p.sub(t, 9)), p.const(f2bits(a), 64)), p.const(f2bits(b), 64))
    y = p.fop("FMUL", p.itof(t), p.const(f2bits(0.1), 64))
    p.access(0, p.ftoi(p.fop("FADD", x, y)))

    def model(B, T, launch, sc):
        for th in T:
            v = (float(th.tl - 9) * a - b) + float(th.tl) * 0.1
            th.acc(0, 0, ftoi(v, 32), 0)
    return Case("fp_arith", p, model)


ALL = [rotate, racing_max, phases, shared_divisor, bounds, tile_gather, prefix_max, hist_like, ep_like,
       fp_arith]


def tables_for(case, rng, n, a_elems=(40, 300), sh_elems=None):
    """n tables: A of a random size, sh of ``sh_elems`` (or a random size
    up to 512 + 64 elements), G with data reference 1."""
    out = []
    for _ in range(n):
        na = int(rng.integers(*a_elems))
        ns = int(sh_elems if sh_elems is not None else rng.integers(8, 600))
        tab = [(LB + 4096, 4 * na, 0, 0, 0)]
        if len(case.spaces) > 1:
            tab.append((SH_BASE, 4 * ns, 0, 0, 0) if case.spaces[1] == 1 else (LB + (1 << 20), 4 * 4096, 0, 0, 0))
        if len(case.spaces) > 2:
            tab.append((LB + (1 << 24), 4 * 8192, 1, 0, 0))
        out.append(tab)
    return out


def workload(case, launches, tables, scalars=None, data=(), mode=W.MODE_FULL):
    import kernels as K
    return K.simple_workload(case.ir, launches, tables, scalars=scalars, mode=mode, data=data)


def exp_ulps(x: float, ref: float) -> float:
    """|x - ref| in units of ref's last place (subnormal spacing below 2^-1022)."""
    if math.isinf(ref) or ref == 0.0:
        return 0.0 if x == ref else math.inf
    return abs(x - ref) / math.ulp(ref)


def data_array(rng, n=8192, lo=-20, hi=600):
    return rng.integers(lo, hi, size=n).astype(np.int32)
