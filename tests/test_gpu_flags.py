"""GPU parity of the vertex-exact status flag (status bit 0 of the
representative modes) against the oracle: random affine chains at random
launch shapes, dead wrapping operations, a wrap that hides an interior
violation, divergent guards, the loop budget and indices wrapping next to a
loop counter; every record, map and status field compared."""
import numpy as np
import pytest

import kernels as K
import test_oracle_flags as F
from oracle import oracle as O
from paper_2601_01048_amd import ckc
from paper_2601_01048_amd.gen import workloads as W
from paper_2601_01048_amd.gen.ir import Program
from test_gpu_parity import compare

pytestmark = pytest.mark.gpu
LB = W.LOGICAL_BASE
REP = (W.MODE_CORNERS, W.MODE_BOUNDARY)


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    c = ckc.Context(0)
    yield c
    c.close()


def both(ctx, wl, mode, generic=False, what=""):
    print(f"[case] {what} mode={mode} generic={generic}", flush=True)
    g = ckc.run_workload(ctx, wl, mode=mode, force_generic=generic)
    o = O.check(wl, mode=mode)
    compare(g, o, what=f"{what} mode {mode} generic {generic}")
    return g


@pytest.mark.parametrize("seed", range(3))
def test_random_chains(ctx, seed):
    rng = np.random.default_rng(900 + seed)
    seen = set()
    for k in range(20):
        spec = F.random_chain(rng)
        ir = F.build(spec, 2).to_bytes()
        launches, scal = [], []
        for _ in range(6):
            launches.append([int(rng.integers(1, 5)), int(rng.integers(1, 3)), int(rng.integers(1, 3)),
                             int(rng.integers(1, 9)), int(rng.integers(1, 4)), int(rng.integers(1, 3))])
            scal.append([int(rng.choice([0, 5, -9, 1 << 31, 1 << 40, (1 << 62) + 3])) for _ in range(2)])
        wl = K.simple_workload(ir, launches, [[(0, 0, 0, 0, 0)]] * 6, scalars=scal)
        for mode in REP:
            for generic in (False, True):
                g = both(ctx, wl, mode, generic, f"chain {seed}/{k}")
                seen |= set(int(v) for v in g["status"]["flags"])
    assert seen == {0, 1}


def test_worked_cases(ctx):
    p = Program(n_scalars=0, n_slots=1)
    p.access(0, p.mul(p.special("tid.x"), p.const(3 << 29, 32), 32))
    for bdx in (4, 2):
        wl = K.simple_workload(p.to_bytes(), [[1, 1, 1, bdx, 1, 1]], [[(LB, 4 * ((1 << 31) - 1), 0, 0, 0)]])
        for mode in REP:
            both(ctx, wl, mode, False, f"hidden UNDER bdx {bdx}")
    bs, g = 256, 4
    for N in (g * bs - 1, g * bs, 1000, 0):
        wl = K.simple_workload(K.listing3_program(), [[g, 1, 1, bs, 1, 1]], [[(LB, 4 << 20, 0, 0, 0)] * 3],
                               scalars=[[N]])
        for mode in REP:
            for generic in (False, True):
                both(ctx, wl, mode, generic, f"listing3 N={N}")
    p = Program(n_scalars=1, n_slots=1)
    with p.loop(0, p.scalar(0, 32), 1, w=32) as i:
        p.access(0, p.add(i, p.special("tid.x"), 32))
    for n in (65535, 65536, 10):
        wl = K.simple_workload(p.to_bytes(), [[1, 1, 1, 2, 1, 1]], [[(LB, 4 << 20, 0, 0, 0)]], scalars=[[n]],
                               cap=(20, 12))
        both(ctx, wl, W.MODE_CORNERS, False, f"budget n={n}")
    p = Program(n_scalars=2, n_slots=1)
    with p.loop(p.scalar(0, 32), p.scalar(1, 32), 1 << 30, w=32) as i:
        p.access(0, p.add(i, p.special("tid.x"), 32), w=32)
    top = (1 << 31) - 1
    for s, e, bdx in ((0, 100, 2), (top - 2, top, 3), (top - 1, top, 3)):
        wl = K.simple_workload(p.to_bytes(), [[1, 1, 1, bdx, 1, 1]], [[(LB, 4 << 20, 0, 0, 0)]], scalars=[[s, e]])
        both(ctx, wl, W.MODE_CORNERS, False, f"counter index s={s} e={e} bdx={bdx}")
