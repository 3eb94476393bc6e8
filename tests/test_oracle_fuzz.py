"""Pins of the oracle's closed-loop fuzzing campaign (Section 2.1: pick an
input from the corpus, mutate it, execute it, keep it when it reaches new
coverage, report inputs that trigger a memory bug).

What fixes it from outside: the generator's published first outputs
(SplitMix64 from seed 0), AFL's documented hit-count buckets, the worked bug
of Listing 3 (a guarded vecAdd whose bug appears once the grid covers
id = N-1) found from a bug-free seed, and properties any such campaign has:
a campaign of G generations is a prefix of one of G+1; every input a
generation adds to the corpus, checked again alone, reaches a bucket the
virgin map still had before that generation; the virgin map only loses
bits; children respect the campaign's bounds; results do not depend on the
oracle's thread count."""
import numpy as np
import pytest

import kernels as K
from oracle import oracle as O
from paper_2601_01048_amd.gen import workloads as W

LB = W.LOGICAL_BASE


def test_generator_known_answers():
    """SplitMix64 started from seed 0: its first three outputs as published
    with the generator (Steele, Lea and Flood; the reference code by Vigna)."""
    assert [O.fuzz_rand(0, k) for k in range(3)] == [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4,
                                                       0x06C45D188009454F]


def test_hit_count_buckets():
    """AFL's buckets of hit counts: 0 | 1 | 2 | 3 | 4-7 | 8-15 | 16-31 |
    32-127 | 128+, one bit each in increasing order."""
    ranges = [(1, 1), (2, 2), (3, 3), (4, 7), (8, 15), (16, 31), (32, 127), (128, 255)]
    assert O.fuzz_class(0) == 0
    for b, (lo, hi) in enumerate(ranges):
        for v in range(lo, hi + 1):
            assert O.fuzz_class(v) == 1 << b, v


def bucket(m):
    return np.array([O.fuzz_class(int(v)) for v in range(256)], np.uint8)[m]


def listing3_seed(N=100, alloc=200, grid=1, bs=64):
    return K.simple_workload(K.listing3_program(), [[grid, 1, 1, bs, 1, 1]], [[(LB, alloc * 4, 0, 0, 0)] * 3],
                             scalars=[[N]])


def test_listing3_bug_found_from_bug_free_seed():
    """The seed covers ids 0..63 < N = 100 of 200-element arrays: no bug.  The
    campaign, mutating the launch and N, reaches a child whose grid covers an
    id at or past the arrays' ends and reports OVER on all three accesses."""
    wl = listing3_seed()
    assert int(O.check(wl)["records"]["count"].sum()) == 0
    out = O.fuzz(wl, generations=8, batch=64, seed=7, max_threads=1 << 14)
    assert out["stats"]["crashes"] > 0
    for a in range(3):
        assert out["sigs"][a, 0] != np.uint64(2 ** 64 - 1), a   # OVER seen on every access
    assert np.all(out["sigs"][:, 1:3] == np.uint64(2 ** 64 - 1))  # nothing UNDER/FREED here
    assert out["stats"]["execs"] == 8 * 64 and out["stats"]["generations"] == 8


@pytest.mark.parametrize("name,kw", [
    ("listing3", dict(ops=O.MUT_LAUNCH | O.MUT_SCALAR, max_threads=1 << 12, max_block=256)),
    ("stencil", dict(ops=O.MUT_LAUNCH | O.MUT_SCALAR, max_threads=1 << 13, max_block=256)),
    ("csr", dict(ops=O.MUT_DATA | O.MUT_LAUNCH, data_slot=1, max_threads=1 << 12, max_block=256)),
])
def test_campaign_prefix_novelty_and_bounds(name, kw):
    if name == "listing3":
        wl = listing3_seed()
    elif name == "stencil":
        wl = W.mini("config2", n_inputs=1, g0=3, hw0=40)
    else:
        wl = W.mini("config3", n_inputs=1, log2_rows=8)
    G, B = 4, 24
    a = O.fuzz(wl, generations=G, batch=B, seed=11, corpus_cap=64, **kw)
    b = O.fuzz(wl, generations=G + 1, batch=B, seed=11, corpus_cap=64, **kw)
    n = len(a["gen"])
    # prefix
    for f in ("launch", "scalars", "gen"):
        assert np.array_equal(b[f][:n], a[f]), f
    if a["data"] is not None:
        assert np.array_equal(b["data"][:n], a["data"])
    # the virgin map only loses bits
    assert np.all((b["virgin"] & ~a["virgin"]) == 0)
    assert b["stats"]["execs"] == a["stats"]["execs"] + B
    def alone(k):
        one = wl.subset([0])
        one.launch = b["launch"][k: k + 1].copy()
        one.scalars = b["scalars"][k: k + 1, : wl.scalars.shape[1]].copy()
        if b["data"] is not None:
            one.data = list(wl.data)
            ref = int(wl.tables[wl.table_idx[0]][kw["data_slot"]]["data"])
            one.data[ref - 1] = b["data"][k].copy()
        return bucket(O.check(one)["maps"][0])

    # each input added by the last generation reaches a bucket still virgin
    added = np.nonzero(b["gen"] == G)[0]
    assert b["stats"]["novel"] - a["stats"]["novel"] >= len(added)
    for k in added:
        assert np.any(alone(k) & a["virgin"]), k
    # every input the campaign executed and kept has left no bucket virgin
    for k in range(1, len(b["gen"])):
        assert not np.any(alone(k) & b["virgin"]), k
    # bounds of every corpus input
    for L in b["launch"]:
        bs = int(L[3]) * int(L[4]) * int(L[5])
        assert 1 <= bs <= kw["max_block"] and bs * int(L[0]) * int(L[1]) * int(L[2]) <= kw["max_threads"]
    assert np.all(np.diff(b["gen"].astype(np.int64)) >= 0)
    assert len(b["gen"]) > 1  # the campaign found something new


def test_thread_count_and_seed():
    wl = W.mini("config3", n_inputs=1, log2_rows=8)
    kw = dict(generations=3, batch=16, ops=O.MUT_DATA, data_slot=1, max_threads=1 << 12)
    a = O.fuzz(wl, seed=5, nthreads=1, **kw)
    b = O.fuzz(wl, seed=5, nthreads=4, **kw)
    c = O.fuzz(wl, seed=6, nthreads=4, **kw)
    for f in ("launch", "scalars", "data", "gen", "virgin", "sigs"):
        assert np.array_equal(a[f], b[f]), f
    assert a["stats"] == b["stats"]
    assert not (np.array_equal(a["virgin"], c["virgin"]) and len(a["gen"]) == len(c["gen"])
                and np.array_equal(a["data"], c["data"]))


def test_corpus_cap_and_invalid_campaigns():
    wl = listing3_seed()
    out = O.fuzz(wl, generations=6, batch=64, seed=3, corpus_cap=3)
    assert len(out["gen"]) <= 3
    with pytest.raises(O.OracleError):
        O.fuzz(wl, generations=1, batch=0)
    with pytest.raises(O.OracleError):
        O.fuzz(wl, generations=1, batch=4, mode=W.MODE_PREX)
    with pytest.raises(O.OracleError):  # the seed's block above max_block
        O.fuzz(wl, generations=1, batch=4, max_block=32)
    with pytest.raises(O.OracleError):
        O.fuzz(wl, generations=1, batch=4, max_stack=16)
