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
