"""Pins of the oracle's rep-exact status flag (the exact-integer premise of
the Section 5.1.1 Theorem): an independent Python model of straight-line
affine chains evaluated in exact integers at every vertex of the (grid x
block) box, worked cases of divergent control and of the loop budget, and the
Theorem's equality property gated on the flag, with a case where a wrap at a
vertex hides an interior violation from the representative set."""
import itertools

import numpy as np
import pytest

import kernels as K
from oracle import oracle as O
from paper_2601_01048_amd.gen import workloads as W
from paper_2601_01048_amd.gen.ir import Program

LB = W.LOGICAL_BASE
NAMES = ("tid.x", "tid.y", "tid.z", "bid.x", "bid.y", "bid.z")
I32 = (-(1 << 31), 1 << 31)
I64 = (-(1 << 63), 1 << 63)


def _wrap(v, w):
    v &= (1 << w) - 1
    return v - (1 << w) if v >> (w - 1) else v


def _in(v, w):
    lo, hi = I32 if w == 32 else I64
    return lo <= v < hi


def model_flag(spec, launch, scalars):
    """Exact-integer model of the flag for a straight-line chain: True when no
    operation wraps at any vertex thread.  Registers hold the container value
    (a width-32 result sign-extended)."""
    gx, gy, gz, bx, by, bz = (int(v) for v in launch)
    ext = (bx, by, bz, gx, gy, gz)  # tid.xyz, bid.xyz extents
    for corner in itertools.product(*[(0, e - 1) if e > 1 else (0,) for e in ext]):
        vals = []
        for op in spec:
            kind = op[0]
            if kind == "special":
                vals.append(corner[NAMES.index(op[1])])
            elif kind == "scalar":
                vals.append(_wrap(int(scalars[op[1]]), op[2]))
            elif kind == "const":
                vals.append(_wrap(op[1], op[2]))
            elif kind in ("add", "sub", "mul", "shl"):
                x, y, w = vals[op[1]], vals[op[2]], op[3]
                if w == 32 and not (_in(x, 32) and _in(y, 32)):
                    return False
                sx, sy = _wrap(x, w), _wrap(y, w)
                r = {"add": sx + sy, "sub": sx - sy, "mul": sx * sy,
                     "shl": sx * (1 << (sy % w))}[kind]
                if not _in(r, w):
                    return False
                vals.append(r)
            elif kind in ("sext", "trunc"):
                if not _in(vals[op[1]], 32):
                    return False
                vals.append(vals[op[1]])
            elif kind == "zext":
                if not (0 <= vals[op[1]] < (1 << 31)):
                    return False
                vals.append(vals[op[1]])
            elif kind == "access":
                if op[2] == 32 and not _in(vals[op[1]], 32):
                    return False
                vals.append(None)
    return True


def build(spec, n_scalars):
    p = Program(n_scalars=n_scalars, n_slots=1)
    regs = []
    for op in spec:
        kind = op[0]
        if kind == "special":
            regs.append(p.special(op[1]))
        elif kind == "scalar":
            regs.append(p.scalar(op[1], op[2]))
        elif kind == "const":
            regs.append(p.const(op[1], op[2]))
        elif kind in ("add", "sub", "mul", "shl"):
            regs.append(p.op(kind.upper(), regs[op[1]], regs[op[2]], op[3]))
        elif kind in ("sext", "zext", "trunc"):
            regs.append(getattr(p, kind)(regs[op[1]]))
        elif kind == "access":
            p.access(0, regs[op[1]], w=op[2])
            regs.append(None)
    return p


def random_chain(rng, n_ops=12):
    """An affine chain: coordinates and uniform values combined by add/sub,
    multiplied or shifted by uniform values; every value ends in an access."""
    spec = []
    uniform = []
    for nm in rng.choice(NAMES, size=3, replace=False):
        spec.append(("special", str(nm)))
    for _ in range(3):
        if rng.random() < 0.5:
            spec.append(("scalar", int(rng.integers(2)), int(rng.choice([32, 64]))))
        else:
            c = int(rng.choice([1, -1, 3, 1000, 1 << 20, 1 << 29, (1 << 31) - 1, 1 << 33, -(1 << 40), 7]))
            spec.append(("const", c, int(rng.choice([32, 64]))))
        uniform.append(len(spec) - 1)
    for _ in range(n_ops):
        w = int(rng.choice([32, 64]))
        kind = str(rng.choice(["add", "sub", "mul", "shl", "sext", "zext", "trunc"]))
        vals = [k for k, o in enumerate(spec) if o[0] != "access"]
        if kind in ("add", "sub"):
            spec.append((kind, int(rng.choice(vals)), int(rng.choice(vals)), w))
        elif kind in ("mul", "shl"):
            spec.append((kind, int(rng.choice(vals)), int(rng.choice(uniform)), w))
        else:
            spec.append((kind, int(rng.choice(vals))))
    n = len(spec)
    for k in range(n):
        if spec[k][0] != "access":
            spec.append(("access", k, int(rng.choice([32, 64]))))
    return spec


@pytest.mark.parametrize("seed", range(4))
def test_vertex_flag_matches_exact_model(seed):
    rng = np.random.default_rng(900 + seed)
    agree = {True: 0, False: 0}
    for _ in range(40):
        spec = random_chain(rng)
        ir = build(spec, 2).to_bytes()
        launches, scal = [], []
        for _ in range(6):
            launches.append([int(rng.integers(1, 5)), int(rng.integers(1, 3)), int(rng.integers(1, 3)),
                             int(rng.integers(1, 9)), int(rng.integers(1, 4)), int(rng.integers(1, 3))])
            scal.append([int(rng.choice([0, 5, -9, 1 << 31, 1 << 40, (1 << 62) + 3])) for _ in range(2)])
        wl = K.simple_workload(ir, launches, [[(0, 0, 0, 0, 0)]] * 6, scalars=scal)
        for mode in (W.MODE_CORNERS, W.MODE_BOUNDARY, W.MODE_PREX):
            flags = O.check(wl, mode=mode, maps=False)["status"]["flags"]
            for i in range(6):
                exp = model_flag(spec, wl.launch[i], wl.scalars[i])
                assert bool(flags[i] & 1) == exp, (spec, wl.launch[i].tolist(), wl.scalars[i].tolist(), mode)
                agree[exp] += 1
        assert (O.check(wl, mode=W.MODE_FULL, maps=False)["status"]["flags"] == 0).all()
    assert agree[True] > 0 and agree[False] > 0  # both outcomes exercised


def test_dead_wraps_do_not_count():
    """Only operations an index, predicate or bound depends on count."""
    p = Program(n_scalars=0, n_slots=1)
    t = p.special("tid.x")
    p.op("MUL", p.const(1 << 40, 64), p.const(1 << 40, 64), 64)  # wraps, feeds nothing
    p.op("MUL", p.mul(t, p.const(1 << 30, 32), 32), p.const(8, 32), 32)  # wraps at tid 1, feeds nothing
    p.access(0, p.add(t, p.const(1, 32), 32))
    wl = K.simple_workload(p.to_bytes(), [[3, 1, 1, 4, 1, 1]], [[(LB, 16, 0, 0, 0)]])
    assert O.check(wl, mode=W.MODE_CORNERS)["status"]["flags"][0] == 1


def test_wrap_hides_interior_violation():
    """idx = tid.x * 1.5*2^30 at width 32 over 4 threads: 0, 1.5*2^30, then
    3*2^30 wraps to -2^30 (an UNDER at the interior thread 2), then 4.5*2^30
    wraps to 2^29 (in bounds).  The corner threads 0 and 3 see nothing wrong;
    the flag is clear because the product wraps at vertex 3."""
    p = Program(n_scalars=0, n_slots=1)
    p.access(0, p.mul(p.special("tid.x"), p.const(3 << 29, 32), 32))
    wl = K.simple_workload(p.to_bytes(), [[1, 1, 1, 4, 1, 1]], [[(LB, 4 * ((1 << 31) - 1), 0, 0, 0)]])
    full = O.check(wl, mode=W.MODE_FULL)
    rep = O.check(wl, mode=W.MODE_CORNERS)
    assert int(full["records"]["count"][0, 0]) == 1 and int(full["records"]["kinds"][0, 0]) == O.KIND_UNDER
    assert int(rep["records"]["count"][0, 0]) == 0
    assert rep["status"]["flags"][0] == 0
    # one thread fewer: no wrap at any vertex, and then nothing is hidden
    wl3 = K.simple_workload(p.to_bytes(), [[1, 1, 1, 2, 1, 1]], [[(LB, 4 * ((1 << 31) - 1), 0, 0, 0)]])
    assert O.check(wl3, mode=W.MODE_CORNERS)["status"]["flags"][0] == 1


def test_divergent_control_clears_flag():
    """Listing 3 (access guarded by id < N): the vertex threads take different
    branches when N cuts the grid between its first and last thread."""
    bs, g = 256, 4
    for N, exp in ((g * bs - 1, 0), (g * bs, 1), (1000, 0), (0, 1)):
        wl = K.simple_workload(K.listing3_program(), [[g, 1, 1, bs, 1, 1]], [[(LB, 4 << 20, 0, 0, 0)] * 3],
                               scalars=[[N]])
        for mode in (W.MODE_CORNERS, W.MODE_BOUNDARY):
            assert int(O.check(wl, mode=mode)["status"]["flags"][0]) == exp, (N, mode)


def test_loop_budget():
    """One uniform loop of n iterations costs 1 + n against the 2^16 budget."""
    p = Program(n_scalars=1, n_slots=1)
    with p.loop(0, p.scalar(0, 32), 1, w=32) as i:
        p.access(0, p.add(i, p.special("tid.x"), 32))
    ir = p.to_bytes()
    for n, exp in ((65535, 1), (65536, 0), (10, 1)):
        wl = K.simple_workload(ir, [[1, 1, 1, 2, 1, 1]], [[(LB, 4 << 20, 0, 0, 0)]], scalars=[[n]], cap=(20, 12))
        assert int(O.check(wl, mode=W.MODE_CORNERS, maps=False)["status"]["flags"][0]) == exp, n


def test_loop_counter_and_index_wrap():
    """Counters of a loop stay between start and end (exact trip counts), so
    they never wrap themselves; an index formed from a counter near 2^31 - 1
    does, at the vertex thread with the largest tid.x."""
    p = Program(n_scalars=2, n_slots=1)
    with p.loop(p.scalar(0, 32), p.scalar(1, 32), 1 << 30, w=32) as i:
        p.access(0, p.add(i, p.special("tid.x"), 32), w=32)
    ir = p.to_bytes()
    top = (1 << 31) - 1
    for s, e, bdx, exp in ((0, 100, 2, 1), (top - 5, -(1 << 31), 2, 1), (-(1 << 31), top, 2, 1),
                           (top - 2, top, 3, 1), (top - 1, top, 2, 1), (top - 1, top, 3, 0)):
        wl = K.simple_workload(ir, [[1, 1, 1, bdx, 1, 1]], [[(LB, 4 << 20, 0, 0, 0)]], scalars=[[s, e]])
        got = int(O.check(wl, mode=W.MODE_CORNERS, maps=False)["status"]["flags"][0])
        assert got == exp, (s, e, bdx)


@pytest.mark.parametrize("name", ["config1", "config2"])
@pytest.mark.parametrize("mode", [W.MODE_CORNERS, W.MODE_BOUNDARY])
def test_theorem_equality_gated(name, mode):
    """Affine, unguarded kernels whose vertices do not wrap (flag set): the
    representative set flags exactly what the whole grid flags."""
    wl = W.mini(name)
    full = O.check(wl, mode=W.MODE_FULL)
    rep = O.check(wl, mode=mode)
    ok = (rep["status"]["flags"] & 1) == 1
    assert ok.all()
    r, f = rep["records"], full["records"]
    assert ((r["kinds"] == f["kinds"]) | ~ok[:, None]).all()
    assert (((r["count"] > 0) == (f["count"] > 0)) | ~ok[:, None]).all()
