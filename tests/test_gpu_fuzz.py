"""Fuzzing campaigns on the device (ckc_fuzz_*) against the oracle's
campaign loop: corpus (launch, scalars, elements, generation of each entry),
virgin map, crash signatures and counters identical after every number of
generations, for launch/scalar mutation, data mutation, the tripwire model
and a representative thread set."""
import os

import numpy as np
import pytest

import kernels as K
from oracle import oracle as O
from paper_2601_01048_amd import ckc
from paper_2601_01048_amd.gen import workloads as W

pytestmark = pytest.mark.gpu

NCPU = max(1, min(16, os.cpu_count() or 1))
LB = W.LOGICAL_BASE


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    c = ckc.Context(0)
    yield c
    c.close()


def listing3_seed(N=100, alloc=200, grid=1, bs=64):
    return K.simple_workload(K.listing3_program(), [[grid, 1, 1, bs, 1, 1]], [[(LB, alloc * 4, 0, 0, 0)] * 3],
                             scalars=[[N]])


CASES = {
    "listing3": (lambda: listing3_seed(), dict(ops=ckc.MUT_LAUNCH | ckc.MUT_SCALAR, max_threads=1 << 12,
                                               max_block=256, batch=64)),
    "stencil": (lambda: W.mini("config2", n_inputs=1, g0=3, hw0=40),
                dict(ops=ckc.MUT_LAUNCH | ckc.MUT_SCALAR, max_threads=1 << 13, max_block=256, batch=48)),
    "stencil_boundary": (lambda: W.mini("config2", n_inputs=1, g0=4, hw0=60, mode=W.MODE_BOUNDARY),
                         dict(ops=ckc.MUT_LAUNCH | ckc.MUT_SCALAR, max_threads=1 << 14, max_block=256, batch=40)),
    "csr_data": (lambda: W.mini("config3", n_inputs=1, log2_rows=8),
                 dict(ops=ckc.MUT_DATA | ckc.MUT_LAUNCH, data_slot=1, max_threads=1 << 12, max_block=256,
                      batch=64)),
    "csr_i64_tripwire": (lambda: W.adjacent_layout(W.mini("config3", n_inputs=1, log2_rows=8, w=64), 32),
                         dict(ops=ckc.MUT_DATA | ckc.MUT_LAUNCH | ckc.MUT_SCALAR, data_slot=1,
                              max_threads=1 << 12, max_block=256, batch=32, max_stack=8)),
    "affine1d": (lambda: W.mini("config1", n_inputs=1),
                 dict(ops=ckc.MUT_LAUNCH, max_threads=1 << 13, max_block=512, batch=128)),
}


def same(g, o, what):
    for f in ("launch", "scalars", "gen", "virgin", "sigs"):
        assert np.array_equal(g[f], o[f]), (what, f)
    if o["data"] is not None:
        assert np.array_equal(g["data"], o["data"]), (what, "data")
    for f in ("execs", "novel", "crashes", "generations"):
        assert g["stats"][f] == o["stats"][f], (what, f, g["stats"][f], o["stats"][f])
    assert g["stats"]["corpus"] == len(o["gen"])


@pytest.mark.parametrize("name", sorted(CASES))
def test_campaign_matches_oracle(ctx, name):
    make, kw = CASES[name]
    wl = make()
    kw = dict(kw)
    batch = kw.pop("batch")
    seed = 1000 + len(name)
    dw = ckc.DeviceWorkload(ctx, wl)
    try:
        with ckc.Fuzz(ctx, dw, batch=batch, seed=seed, corpus_cap=128, **kw) as fz:
            done = 0
            for G in (1, 2, 5):  # run in pieces: 1, then 1 more, then 3 more
                print(f"[case] fuzz {name} generations={G} batch={batch}", flush=True)
                fz.run(G - done)
                done = G
                g = fz.read()
                o = O.fuzz(wl, generations=G, batch=batch, seed=seed, corpus_cap=128, nthreads=NCPU, **kw)
                same(g, o, f"{name} after {G}")
            assert g["stats"]["execs"] == 5 * batch
    finally:
        dw.close()


def test_listing3_bug_found(ctx):
    """From a bug-free seed the device campaign reports OVER on all three
    accesses of Listing 3 (the oracle pins the same campaign)."""
    wl = listing3_seed()
    dw = ckc.DeviceWorkload(ctx, wl)
    try:
        with ckc.Fuzz(ctx, dw, batch=64, seed=7, max_threads=1 << 14) as fz:
            fz.run(8)
            g = fz.read()
        assert g["stats"]["crashes"] > 0
        assert all(int(g["sigs"][a, 0]) != 2 ** 64 - 1 for a in range(3))
    finally:
        dw.close()


def test_campaign_rejections(ctx):
    wl = listing3_seed()
    dw = ckc.DeviceWorkload(ctx, wl)
    try:
        for kw in (dict(batch=0), dict(batch=8, max_stack=16), dict(batch=8, max_block=32),
                   dict(batch=8, mode=W.MODE_PREX), dict(batch=8, data_slot=5)):
            with pytest.raises(ckc.CkcError):
                ckc.Fuzz(ctx, dw, **kw)
        # the program and table are released when a campaign ends
        with ckc.Fuzz(ctx, dw, batch=8) as fz:
            fz.run(1)
    finally:
        dw.close()
