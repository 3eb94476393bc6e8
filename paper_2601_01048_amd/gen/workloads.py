"""Seeded synthetic workloads: index programs plus per-input launch shapes,
scalars and allocation tables.

The paper measures on third-party CUDA benchmark suites and on its own
memory-safety benchmark (Section 7.1); none of them is available here, so these
generators stand in for them with the access *shapes* the paper discusses:
affine kernels such as vector addition (Listing 1, Listing 3) and stencils, and
indirect kernels whose indices come from loaded index arrays (the paper's
graph kernels, for which PREX falls back to the whole grid, Section 7.3).

Families (each in an int32 and an int64 form):
  F1  1-D affine kernel: four accesses A[gid-1], A[gid], B[gid+1], B[gid+2]
  F2  2-D 9-point stencil: centre read, an 8-iteration neighbour loop with a
      halo radius and a row-stride scalar, centre write
  F3  CSR SpMV gather: guarded row, two row_ptr loads, a loop over the row's
      nonzeros loading col_idx[j] and touching val[j] and x[col], then y[row]

and three kernels with data math, shared memory and barriers, the shapes the
paper's pruning (Section 5.2; Section 7.4's ep and hist) is measured on: an
EP-like kernel (a chain of exponentials no index reads), a block histogram
(shared counts no index reads, a barrier) and a tile gather (a data tile in
shared memory read back as indices: the barrier stays).

Only numpy's PCG64 generator is used; nothing here performs the checking
arithmetic.  A workload is a plain record of arrays that both the oracle
wrapper and the GPU binding consume.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from .ir import Program

# allocation-table entry (32 bytes; layout shared by the C-ABI's ckc_alloc):
# the ``data`` field holds a 1-based index into ``Workload.data`` here (0 = no
# data); consumers replace it with a host or device address.
ALLOC_DTYPE = np.dtype([("base", "<u8"), ("size_bytes", "<u8"), ("data", "<u8"),
                        ("flags", "<u4"), ("redzone", "<u4")])
ALLOC_FREED = 1
DETECT_EXACT, DETECT_TRIPWIRE = 0, 1

MODE_FULL, MODE_CORNERS, MODE_BOUNDARY, MODE_PREX, MODE_ENDPOINTS = 0, 1, 2, 3, 4
DEFAULT_CAP_LOG2 = (20, 12)
I64_BASE = 1 << 32  # base offset of the int64 variants (no memory behind it)
LOGICAL_BASE = 0x7F00_0000_0000  # nonzero logical base for live allocations


@dataclass
class Workload:
    name: str
    ir: bytes
    launch: np.ndarray          # [n, 6] uint32: gx gy gz bx by bz
    scalars: np.ndarray         # [n, n_scalars] int64
    tables: np.ndarray          # [n_tables, n_slots] ALLOC_DTYPE
    table_idx: np.ndarray       # [n] uint32: table of each input
    data: list = field(default_factory=list)  # arrays referenced by tables["data"]
    mode: int = MODE_FULL
    cap_log2: tuple = DEFAULT_CAP_LOG2
    meta: dict = field(default_factory=dict)
    detector: int = DETECT_EXACT  # exact bounds, or the tripwire (redzone) model

    @property
    def n_inputs(self) -> int:
        return int(self.launch.shape[0])

    def subset(self, idx) -> "Workload":
        """The same workload restricted to inputs ``idx`` (tables kept whole)."""
        idx = np.asarray(idx)
        return Workload(self.name, self.ir, self.launch[idx].copy(), self.scalars[idx].copy(),
                        self.tables, self.table_idx[idx].copy(), self.data, self.mode,
                        self.cap_log2, dict(self.meta), self.detector)


def alloc(size_bytes: int, data_ref: int = 0, base: int = LOGICAL_BASE, flags: int = 0, redzone: int = 0):
    return (base, size_bytes, data_ref, flags, redzone)


# ---------------------------------------------------------------------------
# programs
# ---------------------------------------------------------------------------
def _gid_x(p: Program, w: int):
    return p.add(p.mul(p.special("bid.x"), p.special("bdim.x"), w), p.special("tid.x"), w)


def f1_program(w: int = 32) -> bytes:
    """F1: gid = bid.x*bdim.x + tid.x; reads A[gid-1], A[gid]; writes B[gid+1],
    B[gid+2] (the index form of the vector kernels of Listings 1 and 3).  The
    int64 form adds scalar 0 (a base offset) to every index."""
    p = Program(n_scalars=1 if w == 64 else 0, n_slots=2)
    gid = _gid_x(p, w)
    if w == 64:
        gid = p.add(gid, p.scalar(0, 64), 64)
    for slot, off, write in ((0, -1, False), (0, 0, False), (1, 1, True), (1, 2, True)):
        p.access(slot, p.add(gid, p.const(off, w), w), elem=4, write=write)
    return p.to_bytes()


def f2_program(w: int = 32) -> bytes:
    """F2: 2-D 9-point stencil.  Scalars: 0 = row stride S, 1 = radius r
    (2 = base offset in the int64 form).  base = y*S + x; read in[base];
    for k in 0..7: j = k + (k > 3); read in[base + ((j/3)-1)*r*S + ((j%3)-1)*r];
    write out[base]."""
    p = Program(n_scalars=3 if w == 64 else 2, n_slots=2)
    x = p.add(p.mul(p.special("bid.x"), p.special("bdim.x"), w), p.special("tid.x"), w)
    y = p.add(p.mul(p.special("bid.y"), p.special("bdim.y"), w), p.special("tid.y"), w)
    S = p.scalar(0, w)
    r = p.scalar(1, w)
    base = p.add(p.mul(y, S, w), x, w)
    if w == 64:
        base = p.add(base, p.scalar(2, 64), 64)
    p.access(0, base, elem=4)
    with p.loop(0, 8, 1, w=w) as k:
        j = p.add(k, p.cmplts(p.const(3, w), k, w), w)
        dy = p.mul(p.sub(p.divs(j, p.const(3, w), w), p.const(1, w), w), r, w)
        dx = p.mul(p.sub(p.rems(j, p.const(3, w), w), p.const(1, w), w), r, w)
        p.access(0, p.add(base, p.add(p.mul(dy, S, w), dx, w), w), elem=4)
    p.access(1, base, elem=4, write=True)
    return p.to_bytes()


def f3_program(w: int = 32) -> bytes:
    """F3: CSR SpMV gather.  Slots 0 row_ptr, 1 col_idx (int32, real data),
    2 val, 3 x, 4 y (fp32, addresses only).  Scalar 0 = nrows (1 = base offset
    added to the val/x/y indices in the int64 form)."""
    p = Program(n_scalars=2 if w == 64 else 1, n_slots=5)
    r = _gid_x(p, w)
    nrows = p.scalar(0, w)
    with p.if_(p.cmplts(r, nrows, w)):
        rp0 = p.load(0, r, elem=4, w=w)
        rp1 = p.load(0, p.add(r, p.const(1, w), w), elem=4, w=w)
        off = p.scalar(1, 64) if w == 64 else None
        with p.loop(rp0, rp1, 1, w=w) as j:
            c = p.load(1, j, elem=4, w=w)
            jj = p.add(j, off, 64) if w == 64 else j
            cc = p.add(c, off, 64) if w == 64 else c
            p.access(2, jj, elem=4, w=w)
            p.access(3, cc, elem=4, w=w)
        rr = p.add(r, off, 64) if w == 64 else r
        p.access(4, rr, elem=4, write=True, w=w)
    return p.to_bytes()


PROGRAMS = {("F1", 32): f1_program, ("F1", 64): f1_program, ("F2", 32): f2_program,
            ("F2", 64): f2_program, ("F3", 32): f3_program, ("F3", 64): f3_program}


def program(family: str, w: int) -> bytes:
    return PROGRAMS[(family, w)](w)


# ---------------------------------------------------------------------------
# CSR generator (power-law row lengths, corrupted copies of col_idx)
# ---------------------------------------------------------------------------
def powerlaw_row_lengths(rng, nrows: int, ncols: int, mean: int = 16, alpha: float = 2.1):
    """Row lengths L = min(ncols, max(1, floor(s*w))) with w = (1-u)^(-1/(alpha-1))
    (a Pareto law with density exponent alpha); s is bisected to the largest
    value with sum(L) <= mean*nrows (at most nrows*ncols) and the remaining
    deficit is added one nonzero at a time to the first rows below ncols."""
    u = rng.random(nrows)
    w = (1.0 - u) ** (-1.0 / (alpha - 1.0))
    target = min(mean * nrows, nrows * ncols)  # a matrix smaller than mean x nrows is full

    def total(s):
        return int(np.minimum(ncols, np.maximum(1, np.floor(s * w))).sum())

    lo, hi = 0.0, float(mean) * 4
    while total(hi) < target:
        hi *= 2
    for _ in range(100):
        mid = 0.5 * (lo + hi)
        if total(mid) <= target:
            lo = mid
        else:
            hi = mid
    L = np.minimum(ncols, np.maximum(1, np.floor(lo * w))).astype(np.int64)
    deficit = target - int(L.sum())
    if deficit > 0:
        open_rows = np.nonzero(L < ncols)[0][:deficit]
        L[open_rows] += 1
    assert int(L.sum()) == target
    return L


def csr_structure(seed: int, nrows: int, ncols: int, mean: int = 16):
    rng = np.random.default_rng(seed)
    L = powerlaw_row_lengths(rng, nrows, ncols, mean)
    row_ptr = np.zeros(nrows + 1, dtype=np.int64)
    np.cumsum(L, out=row_ptr[1:])
    assert row_ptr[-1] < 2**31
    col = rng.integers(0, ncols, size=int(row_ptr[-1]), dtype=np.int64).astype(np.int32)
    return rng, row_ptr.astype(np.int32), col


def corrupt_copy(rng, col: np.ndarray, ncols: int, frac: float = 0.001):
    """A copy of ``col`` with round(frac*nnz) positions (without replacement)
    replaced by values uniform in [-64, ncols+64)."""
    out = col.copy()
    k = int(round(frac * col.size))
    if k:
        pos = rng.choice(col.size, size=k, replace=False)
        out[pos] = rng.integers(-64, ncols + 64, size=k, dtype=np.int64).astype(np.int32)
    return out


# ---------------------------------------------------------------------------
# configurations
# ---------------------------------------------------------------------------
def config1(seed: int = 1001, n_inputs: int = 256, g_range=(32, 80), block: int = 256,
            n_range=(8192, 16384), w: int = 32) -> Workload:
    """Plain 1-D affine check: G ~ U{g_range} blocks of ``block`` threads,
    n ~ U{n_range} int32 elements per allocation."""
    rng = np.random.default_rng(seed)
    G = rng.integers(g_range[0], g_range[1] + 1, size=n_inputs)
    n = rng.integers(n_range[0], n_range[1] + 1, size=n_inputs)
    launch = np.zeros((n_inputs, 6), np.uint32)
    launch[:, 0] = G
    launch[:, 1:3] = 1
    launch[:, 3] = block
    launch[:, 4:6] = 1
    extra = I64_BASE if w == 64 else 0
    tables = np.zeros((n_inputs, 2), ALLOC_DTYPE)
    for i in range(n_inputs):
        sz = (int(n[i]) + extra) * 4
        tables[i] = [alloc(sz), alloc(sz, base=LOGICAL_BASE + (1 << 36))]
    scalars = np.full((n_inputs, 1), extra, np.int64) if w == 64 else np.zeros((n_inputs, 0), np.int64)
    return Workload(f"config1_f1_i{w}", f1_program(w), launch, scalars, tables,
                    np.arange(n_inputs, dtype=np.uint32), [], MODE_FULL,
                    meta=dict(seed=seed, G=G, n=n, block=block))


def config2(seed: int = 1002, n_inputs: int = 4096, g0: int = 128, hw0: int = 2048,
            delta: int = 3, block=(16, 16), mode: int = MODE_FULL, w: int = 32) -> Workload:
    """2-D 9-point stencil: grid (g0+d1) x (g0+d2) blocks of 16x16 threads over
    an H x W fp32 pair of allocations with H = hw0+d3, W = hw0+d4 (d ~ U{-delta..delta}),
    radius r ~ U{1, 2}, row stride S = W."""
    rng = np.random.default_rng(seed)
    d = rng.integers(-delta, delta + 1, size=(n_inputs, 4))
    r = rng.integers(1, 3, size=n_inputs)
    gx, gy = g0 + d[:, 0], g0 + d[:, 1]
    H, W = hw0 + d[:, 2], hw0 + d[:, 3]
    launch = np.zeros((n_inputs, 6), np.uint32)
    launch[:, 0], launch[:, 1], launch[:, 2] = gx, gy, 1
    launch[:, 3], launch[:, 4], launch[:, 5] = block[0], block[1], 1
    extra = I64_BASE if w == 64 else 0
    ns = 3 if w == 64 else 2
    scalars = np.zeros((n_inputs, ns), np.int64)
    scalars[:, 0], scalars[:, 1] = W, r
    if w == 64:
        scalars[:, 2] = extra
    tables = np.zeros((n_inputs, 2), ALLOC_DTYPE)
    for i in range(n_inputs):
        sz = (int(H[i]) * int(W[i]) + extra) * 4
        tables[i] = [alloc(sz), alloc(sz, base=LOGICAL_BASE + (1 << 36))]
    return Workload(f"config2_f2_i{w}", f2_program(w), launch, scalars, tables,
                    np.arange(n_inputs, dtype=np.uint32), [], mode,
                    meta=dict(seed=seed, H=H, W=W, r=r, gx=gx, gy=gy))


def config3(seed: int = 1003, n_inputs: int = 64, log2_rows: int = 20, mean: int = 16,
            frac: float = 0.001, block: int = 256, w: int = 32) -> Workload:
    """CSR gather: nrows = ncols = 2^log2_rows, power-law rows with mean
    ``mean`` nonzeros, one corrupted copy of col_idx per input."""
    nrows = ncols = 1 << log2_rows
    rng, row_ptr, col = csr_structure(seed, nrows, ncols, mean)
    nnz = int(row_ptr[-1])
    data = [row_ptr]
    for _ in range(n_inputs):
        data.append(corrupt_copy(rng, col, ncols, frac))
    launch = np.zeros((n_inputs, 6), np.uint32)
    launch[:, 0] = (nrows + block - 1) // block
    launch[:, 1:3] = 1
    launch[:, 3] = block
    launch[:, 4:6] = 1
    extra = I64_BASE if w == 64 else 0
    ns = 2 if w == 64 else 1
    scalars = np.zeros((n_inputs, ns), np.int64)
    scalars[:, 0] = nrows
    if w == 64:
        scalars[:, 1] = extra
    tables = np.zeros((n_inputs, 5), ALLOC_DTYPE)
    for i in range(n_inputs):
        tables[i] = [alloc((nrows + 1) * 4, 1, LOGICAL_BASE),
                     alloc(nnz * 4, 2 + i, LOGICAL_BASE + (1 << 36)),
                     alloc((nnz + extra) * 4, 0, LOGICAL_BASE + (2 << 36)),
                     alloc((ncols + extra) * 4, 0, LOGICAL_BASE + (3 << 36)),
                     alloc((nrows + extra) * 4, 0, LOGICAL_BASE + (4 << 36))]
    return Workload(f"config3_f3_i{w}", f3_program(w), launch, scalars, tables,
                    np.arange(n_inputs, dtype=np.uint32), data, MODE_FULL,
                    meta=dict(seed=seed, nrows=nrows, ncols=ncols, nnz=nnz))


def _f2bits(x: float) -> int:
    import struct
    return struct.unpack("<q", struct.pack("<d", x))[0]


def ep_program(n_exp: int = 8) -> bytes:
    """EP-like: i = bid*bs + tid; A[i] is read; a chain of n_exp rounds of
    x = e^(-x/2) * 1.0001 + 0.25 starting from x = i * 2^-20 (the kernel's
    data math) ends in a write of FTOI(1000 x) to B[i].  No index reads x."""
    p = Program(n_slots=2)
    t = p.trunc(p.special("tid.x"))
    i = p.add(p.mul(p.trunc(p.special("bid.x")), p.trunc(p.special("bdim.x"))), t)
    p.access(0, i)
    x = p.fop("FMUL", p.itof(i), p.const(_f2bits(2.0 ** -20), 64))
    for _ in range(n_exp):
        x = p.fop("FEXP", p.fop("FMUL", x, p.const(_f2bits(-0.5), 64)))
        x = p.fop("FADD", p.fop("FMUL", x, p.const(_f2bits(1.0001), 64)), p.const(_f2bits(0.25), 64))
    p.store(1, i, p.ftoi(p.fop("FMUL", x, p.const(_f2bits(1000.0), 64))))
    return p.to_bytes()


def hist_program(nbins: int = 256) -> bytes:
    """Block histogram: x = G[bid*bs + tid]; the count of bin x mod nbins in
    shared memory is read and written back incremented; a barrier; threads
    below nbins write their bin's count to H[bid*nbins + tid].  The counts
    reach no index (slots: 0 G data, 1 bins shared, 2 H)."""
    p = Program(n_slots=3, spaces=[0, 1, 0])
    t = p.trunc(p.special("tid.x"))
    b = p.trunc(p.special("bid.x"))
    g = p.add(p.mul(b, p.trunc(p.special("bdim.x"))), t)
    k = p.remu(p.load(0, g), nbins)
    p.store(1, k, p.add(p.load(1, k), 1))
    p.barrier()
    with p.if_(p.cmpltu(t, nbins)):
        p.store(2, p.add(p.mul(b, nbins), t), p.load(1, t))
    return p.to_bytes()


def tile_gather_program() -> bytes:
    """Tile gather: sh[tid] = G[bid*bs + tid]; a barrier; A[sh[bs - 1 - tid]]:
    indices read back from shared memory, so the barrier stays (slots: 0 A,
    1 tile shared, 2 G data)."""
    p = Program(n_slots=3, spaces=[0, 1, 0])
    t = p.trunc(p.special("tid.x"))
    bs = p.trunc(p.special("bdim.x"))
    g = p.add(p.mul(p.trunc(p.special("bid.x")), bs), t)
    p.store(1, t, p.load(2, g))
    p.barrier()
    p.access(0, p.load(1, p.sub(p.sub(bs, 1), t)))
    return p.to_bytes()


def pruning_config(kind: str, seed: int = 1010, n_inputs: int = 256, g_range=(48, 80), block: int = 256,
                   n_range=(12000, 20000)) -> Workload:
    """Inputs of one of the three pruning kernels ("ep", "hist", "tile"):
    G ~ U{g_range} blocks of ``block`` threads; arrays of n ~ U{n_range}
    int32 elements (so the last blocks run past some of them); G's data are
    seeded values in [-64, 40000) shared by every input."""
    rng = np.random.default_rng(seed)
    G = rng.integers(g_range[0], g_range[1] + 1, size=n_inputs)
    n = rng.integers(n_range[0], n_range[1] + 1, size=n_inputs)
    launch = np.zeros((n_inputs, 6), np.uint32)
    launch[:, 0], launch[:, 1:3], launch[:, 3], launch[:, 4:6] = G, 1, block, 1
    nd = int(g_range[1]) * block
    data = [rng.integers(-64, 40000, size=nd).astype(np.int32)]
    tables = np.zeros((n_inputs, 3 if kind != "ep" else 2), ALLOC_DTYPE)
    for i in range(n_inputs):
        a = alloc(4 * int(n[i]))
        if kind == "ep":
            tables[i] = [a, alloc(4 * int(n[i]), base=LOGICAL_BASE + (1 << 36))]
        elif kind == "hist":
            tables[i] = [alloc(4 * nd, 1, base=LOGICAL_BASE + (1 << 40)), alloc(4 * 256, base=0x100),
                         alloc(4 * 256 * int(G[i]) - 4 * int(rng.integers(0, 512)), base=LOGICAL_BASE)]
        else:
            tables[i] = [a, alloc(4 * block, base=0x100), alloc(4 * nd, 1, base=LOGICAL_BASE + (1 << 40))]
    ir = {"ep": ep_program, "hist": hist_program, "tile": tile_gather_program}[kind]()
    return Workload(f"pruning_{kind}", ir, launch, np.zeros((n_inputs, 0), np.int64), tables,
                    np.arange(n_inputs, dtype=np.uint32), data, MODE_FULL,
                    meta=dict(seed=seed, G=G, n=n, block=block))


def adjacent_layout(wl: Workload, redzone: int, gap: int = 0) -> Workload:
    """The workload under the tripwire detector model with each input's live
    allocations placed one after the other in slot order, each with
    ``redzone`` bytes on both sides and ``gap`` bytes between neighbours (how
    a sanitizer's allocator packs buffers), so that overflows can land in a
    redzone or in the next buffer.  One table per input."""
    n = wl.n_inputs
    src = wl.tables[wl.table_idx]
    tabs = src.copy()
    for i in range(n):
        cur = LOGICAL_BASE + 4096
        for s in range(src.shape[1]):
            if src[i, s]["base"] != 0:
                cur += redzone + gap
                tabs[i, s]["base"] = cur
                tabs[i, s]["redzone"] = redzone
                cur += int(src[i, s]["size_bytes"]) + redzone
    return Workload(wl.name + "_tripwire", wl.ir, wl.launch.copy(), wl.scalars.copy(), tabs,
                    np.arange(n, dtype=np.uint32), wl.data, wl.mode, wl.cap_log2, dict(wl.meta),
                    DETECT_TRIPWIRE)


def mini(name: str, **kw) -> Workload:
    """Reduced forms of the configurations: small enough for the oracle to
    finish in seconds, still spanning many tiles and a ragged tail."""
    if name == "config1":
        base = dict(n_inputs=24, g_range=(2, 9), block=64, n_range=(100, 600))
        base.update(kw)
        return config1(**base)
    if name == "config2":
        base = dict(n_inputs=12, g0=6, hw0=90, delta=3, block=(16, 16))
        base.update(kw)
        return config2(**base)
    if name == "config3":
        base = dict(n_inputs=6, log2_rows=11, mean=16, frac=0.01)
        base.update(kw)
        return config3(**base)
    raise KeyError(name)


# ---------------------------------------------------------------------------
# mixed batches (many small kernels of the three families)
# ---------------------------------------------------------------------------
@dataclass
class MixedBatch:
    """A list of one-input workloads checked together.  ``kernels[k]`` is a
    Workload with one input; programs are shared by (family, width)."""
    name: str
    kernels: list
    meta: dict = field(default_factory=dict)

    @property
    def n_kernels(self) -> int:
        return len(self.kernels)


def _f1_kernel(rng, T: int, w: int) -> Workload:
    block = min(256, T)
    grid = -(-T // block)
    n = int(rng.integers(-(-9 * T // 10), -(-11 * T // 10) + 1))
    extra = I64_BASE if w == 64 else 0
    launch = np.array([[grid, 1, 1, block, 1, 1]], np.uint32)
    sz = (n + extra) * 4
    tables = np.array([[alloc(sz), alloc(sz, base=LOGICAL_BASE + (1 << 36))]], ALLOC_DTYPE)
    scalars = np.full((1, 1), extra, np.int64) if w == 64 else np.zeros((1, 0), np.int64)
    return Workload(f"f1_i{w}", f1_program(w), launch, scalars, tables, np.zeros(1, np.uint32),
                    [], MODE_FULL, meta=dict(family="F1", T=T, n=n))


def _f2_kernel(rng, T: int, w: int) -> Workload:
    side = int(np.ceil(np.sqrt(T)))
    b = min(16, side)
    g = -(-side // b)
    H = side + int(rng.integers(-3, 4))
    W = side + int(rng.integers(-3, 4))
    H, W = max(H, 1), max(W, 1)
    r = int(rng.integers(1, 3))
    extra = I64_BASE if w == 64 else 0
    launch = np.array([[g, g, 1, b, b, 1]], np.uint32)
    sc = [W, r] + ([extra] if w == 64 else [])
    scalars = np.array([sc], np.int64)
    sz = (H * W + extra) * 4
    tables = np.array([[alloc(sz), alloc(sz, base=LOGICAL_BASE + (1 << 36))]], ALLOC_DTYPE)
    return Workload(f"f2_i{w}", f2_program(w), launch, scalars, tables, np.zeros(1, np.uint32),
                    [], MODE_FULL, meta=dict(family="F2", T=T, H=H, W=W, r=r))


def _f3_kernel(seed: int, T: int, w: int, frac: float = 0.001, block: int = 256) -> Workload:
    nrows = ncols = T
    rng, row_ptr, col = csr_structure(seed, nrows, ncols, 16)
    nnz = int(row_ptr[-1])
    col = corrupt_copy(rng, col, ncols, frac)
    bs = min(block, nrows)
    extra = I64_BASE if w == 64 else 0
    launch = np.array([[-(-nrows // bs), 1, 1, bs, 1, 1]], np.uint32)
    scalars = np.array([[nrows] + ([extra] if w == 64 else [])], np.int64)
    tables = np.array([[alloc((nrows + 1) * 4, 1, LOGICAL_BASE),
                        alloc(nnz * 4, 2, LOGICAL_BASE + (1 << 36)),
                        alloc((nnz + extra) * 4, 0, LOGICAL_BASE + (2 << 36)),
                        alloc((ncols + extra) * 4, 0, LOGICAL_BASE + (3 << 36)),
                        alloc((nrows + extra) * 4, 0, LOGICAL_BASE + (4 << 36))]], ALLOC_DTYPE)
    return Workload(f"f3_i{w}", f3_program(w), launch, scalars, tables, np.zeros(1, np.uint32),
                    [row_ptr, col], MODE_FULL, meta=dict(family="F3", T=T, nnz=nnz))


def config4(seed: int = 1004, n_kernels: int = 10000, t_max: int = 65536) -> MixedBatch:
    """Batched mix: family ~ U{F1, F2, F3}, width ~ U{32, 64}, total threads
    T = floor(exp(U[0, ln t_max])) per kernel.  F1: block min(256, T), grid
    ceil(T/block), n ~ U{ceil(0.9T)..ceil(1.1T)} elements.  F2: side ceil(sqrt T),
    block min(16, side)^2, grid ceil(side/b)^2, H, W = side + U{-3..3}, r ~ U{1, 2}.
    F3: nrows = ncols = T, power-law rows of mean 16 capped at T, 0.1% of col_idx
    corrupted.  Width-64 kernels add the base offset 2^32 to their indices."""
    rng = np.random.default_rng(seed)
    fam = rng.integers(0, 3, size=n_kernels)
    wid = np.where(rng.integers(0, 2, size=n_kernels) == 1, 64, 32)
    T = np.floor(np.exp(rng.uniform(0.0, np.log(t_max), size=n_kernels))).astype(np.int64)
    T = np.maximum(T, 1)
    seeds = rng.integers(0, 2**62, size=n_kernels)
    ks = []
    for k in range(n_kernels):
        sub = np.random.default_rng(int(seeds[k]))
        t, w = int(T[k]), int(wid[k])
        if fam[k] == 0:
            ks.append(_f1_kernel(sub, t, w))
        elif fam[k] == 1:
            ks.append(_f2_kernel(sub, t, w))
        else:
            ks.append(_f3_kernel(int(seeds[k]), t, w))
    return MixedBatch("config4_mixed", ks, meta=dict(seed=seed, T=T, family=fam, width=wid))


# ---------------------------------------------------------------------------
# served stream (open-loop arrivals of check jobs)
# ---------------------------------------------------------------------------
ACCESSES_PER_THREAD = {"F1": 4, "F2": 10, "F3": 51}  # F3: per row, 3 + 3 x mean 16 nonzeros


@dataclass
class ServedStream:
    """Jobs with arrival times.  ``jobs[k]`` is a one-input Workload whose
    data references (``tables["data"]``) index ``pool`` (1-based), the
    resident CSR arrays shared by every F3 job."""
    name: str
    arrivals: np.ndarray   # seconds from the start, increasing
    jobs: list
    pool: list
    meta: dict = field(default_factory=dict)

    @property
    def n_jobs(self) -> int:
        return len(self.jobs)


def csr_pool(seed: int, log2_range=(4, 18), frac: float = 0.001):
    """Pre-corrupted CSR matrices with 2^k rows (= columns) for k in
    log2_range; returns (data list [row_ptr_k, col_k, ...], {k: (ref of
    row_ptr, ref of col, nrows, nnz)}) with 1-based references."""
    data, index = [], {}
    for k in range(log2_range[0], log2_range[1] + 1):
        n = 1 << k
        rng, row_ptr, col = csr_structure(seed + k, n, n, 16)
        col = corrupt_copy(rng, col, n, frac)
        data += [row_ptr, col]
        index[k] = (len(data) - 1, len(data), n, int(row_ptr[-1]))
    return data, index


def config5(seed: int = 1005, rate: float = 2000.0, duration_s: float = 35.0, a_range=(1e3, 1e7),
            log2_range=(4, 18), dense: bool = True) -> ServedStream:
    """Served stream: Poisson arrivals at ``rate`` jobs/s over ``duration_s``
    seconds (exponential gaps); size A = exp(U[ln a_min, ln a_max]) thread-
    accesses; family ~ U{F1, F2, F3}, width ~ U{32, 64}; T = ceil(A / a_f)
    threads (a_f = 4, 10, 51).  F1 and F2 shapes as in the batched mix.  F3
    jobs take the pool matrix of 2^k rows with k = round(log2 T) clamped to
    log2_range, and an x vector of ncols + U{-64..64} elements."""
    rng = np.random.default_rng(seed)
    n = int(rate * duration_s * 1.2) + 16
    gaps = rng.exponential(1.0 / rate, size=n)
    arr = np.cumsum(gaps)
    arr = arr[arr < duration_s]
    n = arr.size
    fam = rng.integers(0, 3, size=n)
    wid = np.where(rng.integers(0, 2, size=n) == 1, 64, 32)
    A = np.exp(rng.uniform(np.log(a_range[0]), np.log(a_range[1]), size=n))
    seeds = rng.integers(0, 2**62, size=n)
    pool, index = csr_pool(seed, log2_range)
    jobs = []
    for j in range(n):
        sub = np.random.default_rng(int(seeds[j]))
        w = int(wid[j])
        if fam[j] == 0:
            T = int(np.ceil(A[j] / ACCESSES_PER_THREAD["F1"]))
            k = _f1_kernel(sub, T, w)
        elif fam[j] == 1:
            T = int(np.ceil(A[j] / ACCESSES_PER_THREAD["F2"]))
            k = _f2_kernel(sub, T, w)
        else:
            T = int(np.ceil(A[j] / ACCESSES_PER_THREAD["F3"]))
            lg = int(min(max(round(np.log2(max(T, 1))), log2_range[0]), log2_range[1]))
            r_rp, r_col, nr, nnz = index[lg]
            xs = nr + int(sub.integers(-64, 65))
            extra = I64_BASE if w == 64 else 0
            bs = min(256, nr)
            launch = np.array([[-(-nr // bs), 1, 1, bs, 1, 1]], np.uint32)
            scalars = np.array([[nr] + ([extra] if w == 64 else [])], np.int64)
            tables = np.array([[alloc((nr + 1) * 4, r_rp, LOGICAL_BASE),
                                alloc(nnz * 4, r_col, LOGICAL_BASE + (1 << 36)),
                                alloc((nnz + extra) * 4, 0, LOGICAL_BASE + (2 << 36)),
                                alloc((max(xs, 0) + extra) * 4, 0, LOGICAL_BASE + (3 << 36)),
                                alloc((nr + extra) * 4, 0, LOGICAL_BASE + (4 << 36))]], ALLOC_DTYPE)
            k = Workload(f"f3_i{w}", f3_program(w), launch, scalars, tables, np.zeros(1, np.uint32),
                         [], MODE_FULL, meta=dict(family="F3", T=nr, nnz=nnz, x=xs, log2_rows=lg))
        k.meta["A"] = float(A[j])
        jobs.append(k)
    return ServedStream("config5_served", arr, jobs, pool,
                        meta=dict(seed=seed, rate=rate, duration_s=duration_s, family=fam, width=wid, A=A,
                                  dense=dense))
