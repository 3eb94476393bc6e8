"""GPU parity of the PREX runtime sweep (Algorithm 1, mode CKC_REP_PREX)
against the oracle's sweep: block pairs from both ends inward, a stop before
a round once every access instruction has executed or a violation has been
seen, a single middle block once.  Bit-exact records, maps and status."""
import numpy as np
import pytest

import kernels as K
from oracle import oracle as O
from paper_2601_01048_amd import ckc
from paper_2601_01048_amd.gen import workloads as W
from paper_2601_01048_amd.gen.ir import Program, with_op_helpers
from test_gpu_parity import NCPU, compare

pytestmark = pytest.mark.gpu
with_op_helpers()

LB = W.LOGICAL_BASE


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    c = ckc.Context(0)
    yield c
    c.close()


def both(ctx, wl, generic=False, maps=True):
    print(f"[case] prex {wl.name} generic={generic} n={wl.n_inputs}", flush=True)
    g = ckc.run_workload(ctx, wl, mode=W.MODE_PREX, force_generic=generic, maps=maps)
    o = O.check(wl, mode=W.MODE_PREX, nthreads=NCPU, maps=maps)
    return g, o


def rounds_run(st, launch):
    """Rounds each input ran, from its lane count (every round but a lone
    middle block runs two whole blocks)."""
    bs = launch[:, 3] * launch[:, 4] * launch[:, 5]
    return st["lanes"] // bs


@pytest.mark.parametrize("generic", [False, True])
@pytest.mark.parametrize("name,w", [("config1", 32), ("config1", 64), ("config2", 32), ("config2", 64),
                                    ("config3", 32), ("config3", 64)])
def test_mini_configs(ctx, name, w, generic):
    wl = W.mini(name, w=w)
    g, o = both(ctx, wl, generic)
    compare(g, o, what=f"prex {name} i{w} generic {generic}")


@pytest.mark.parametrize("generic", [False, True])
def test_listing3(ctx, generic):
    """The guarded kernel of Listing 3: the first pair holds the violating
    thread id N-1 (and covers every access), so one round runs."""
    for N, bs in ((1023, 256), (1000, 256), (77, 8), (5000, 64)):
        grid = -(-N // bs)
        wl = K.simple_workload(K.listing3_program(), [[grid, 1, 1, bs, 1, 1]], [[(LB, N * 4, 0, 0, 0)] * 3],
                               scalars=[[N]])
        g, o = both(ctx, wl, generic)
        compare(g, o, what=f"listing3 N={N}")
        assert list(g["records"]["first_key"][0]) == [N - 1] * 3
        assert g["status"]["lanes"][0] == (2 if grid > 1 else 1) * bs


def middle_program():
    """acc 0 everywhere (in bounds); acc 1 only in block x == s0; acc 2 only
    in block x == s1 with index s2 (out of bounds when s2 >= 64); acc 3 never
    has a site of its own (an internal site decides its coverage)."""
    p = Program(n_scalars=4, n_slots=2)
    bx = p.special("bid.x")
    t = p.special("tid.x")
    p.access(0, p.add(t, p.const(0, 64), 64), w=64)
    with p.if_(p.cmpeq(bx, p.scalar(0, 64), 64)):
        p.access(0, t, w=64)
    with p.if_(p.cmpeq(bx, p.scalar(1, 64), 64)):
        p.access(1, p.scalar(2, 64), elem=8, w=64)
    with p.if_(p.cmpeq(bx, p.scalar(3, 64), 64), site_t=False, site_f=False):
        p.access(1, t, elem=8, w=64, site=False)
    return p.to_bytes()


@pytest.mark.parametrize("generic", [False, True])
def test_stop_rules(ctx, generic):
    """Coverage and bug stops at every position of the doubling windows,
    odd and even block counts, one-block grids, and sweeps that never stop
    early (the whole grid)."""
    ir = middle_program()
    launches, scal = [], []
    for gx in (1, 2, 3, 7, 8, 40, 41, 130):
        bs = 32
        for s0, s1, s2, s3 in ((gx // 2, gx // 2, 5, gx // 2), (gx // 2, gx // 2, 99, gx // 2),
                               (3, 2, 99, 1), (-1, -1, 0, -1), (gx - 1, 6, 70, 0), (5, 9, 1, 13),
                               (gx // 3, -1, 0, gx // 3)):
            launches.append([gx, 1, 1, bs, 1, 1])
            scal.append([s0, s1, s2, s3])
    n = len(launches)
    wl = K.simple_workload(ir, launches, [[(LB, 64 * 4, 0, 0, 0), (LB, 64 * 8, 0, 0, 0)]] * n, scalars=scal)
    g, o = both(ctx, wl, generic)
    compare(g, o, what="stop rules")
    r = rounds_run(g["status"], np.asarray(launches))
    assert r.max() > 30  # some sweeps ran to the middle


def test_never_covered_equals_full(ctx):
    """An access no thread reaches keeps the sweep going to the middle: the
    sweep is then the whole grid, and every result but the vertex flag is the
    whole grid's."""
    ir = middle_program()
    launches = [[gx, gy, 1, bx, by, 1] for gx, gy, bx, by in
                ((33, 1, 64, 1), (16, 3, 8, 4), (5, 5, 7, 3), (1, 9, 64, 2), (128, 2, 16, 1))]
    n = len(launches)
    wl = K.simple_workload(ir, launches, [[(LB, 300 * 4, 0, 0, 0), (LB, 64 * 8, 0, 0, 0)]] * n,
                           scalars=[[-1, -1, 0, -1]] * n)
    g = ckc.run_workload(ctx, wl, mode=W.MODE_PREX)
    f = ckc.run_workload(ctx, wl, mode=W.MODE_FULL)
    o = O.check(wl, mode=W.MODE_PREX, nthreads=NCPU)
    compare(g, o, what="never covered")
    for fld in ("first_key", "index", "count", "kinds", "first_kind"):
        np.testing.assert_array_equal(g["records"][fld], f["records"][fld])
    np.testing.assert_array_equal(g["maps"], f["maps"])
    for fld in ("lanes", "accesses_checked", "hang_lanes", "arith_faults"):
        np.testing.assert_array_equal(g["status"][fld], f["status"][fld])


def test_window_limits(ctx):
    """More (input, round) pairs than one window holds: the sweep splits a
    pass over the inputs into several windows."""
    ir = middle_program()
    n = 1500
    gx = 1024  # 512 rounds each; the 256-round pass holds 384,000 pairs
    wl = K.simple_workload(ir, [[gx, 1, 1, 1, 1, 1]] * n, [[(LB, 64 * 4, 0, 0, 0), (LB, 64 * 8, 0, 0, 0)]] * n,
                           scalars=[[-1, (k * 7) % gx, 3, -1] for k in range(n)])
    g, o = both(ctx, wl, maps=False)
    compare(g, o, maps=False, what="window limits")


def guarded_stencil_program():
    """The stencil of the 2-D workload under a Listing-3-style guard
    (x < W and y < H around every access).  Scalars: 0 = S (= W), 1 = r,
    2 = H."""
    p = Program(n_scalars=3, n_slots=2)
    x = p.add(p.mul(p.special("bid.x"), p.special("bdim.x"), 32), p.special("tid.x"), 32)
    y = p.add(p.mul(p.special("bid.y"), p.special("bdim.y"), 32), p.special("tid.y"), 32)
    S, r, H = p.scalar(0, 32), p.scalar(1, 32), p.scalar(2, 32)
    with p.if_(p.op("AND", p.cmplts(x, S, 32), p.cmplts(y, H, 32), 32)):
        base = p.add(p.mul(y, S, 32), x, 32)
        p.access(0, base)
        with p.loop(0, 8, 1, w=32) as k:
            j = p.add(k, p.cmplts(p.const(3, 32), k, 32), 32)
            dy = p.mul(p.sub(p.divs(j, p.const(3, 32), 32), p.const(1, 32), 32), r, 32)
            dx = p.mul(p.sub(p.rems(j, p.const(3, 32), 32), p.const(1, 32), 32), r, 32)
            p.access(0, p.add(base, p.add(p.mul(dy, S, 32), dx, 32), 32))
        p.access(1, base, write=True)
    return p.to_bytes()


@pytest.mark.parametrize("generic", [False, True])
def test_guarded_stencil(ctx, generic):
    """The guarded stencil over grids that overhang the allocation: the
    first pair covers every access and holds the halo overflow."""
    import dataclasses
    wl = W.mini("config2")
    sc = np.concatenate([wl.scalars[:, :2], np.asarray(wl.meta["H"], np.int64).reshape(-1, 1)], axis=1)
    wl = dataclasses.replace(wl, ir=guarded_stencil_program(), scalars=sc)
    g, o = both(ctx, wl, generic)
    compare(g, o, what="guarded stencil")
    assert (g["status"]["lanes"] == 2 * 256).all()


def test_mixed_with_other_modes_rejected(ctx):
    wl = W.mini("config1")
    dw = ckc.DeviceWorkload(ctx, wl)
    try:
        with pytest.raises(ckc.CkcError):
            ctx.check([dw.desc(mode=W.MODE_PREX), dw.desc(mode=W.MODE_FULL)])
    finally:
        dw.close()
