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
oracle's thread count.  And the loop itself, replayed generation by
generation in plain Python from its definition in ``include/ckc.h`` (parent
choice, mutation count, operators, kinds and values, novelty against the
virgin map as at the generation's start, append order, the corpus cap, the
least tag per violated access and kind), with every generation's children
executed by the oracle's check (pinned on its own) and the generator pinned
by its known answers."""
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


SPECIAL = [0, 1, -1, 2, 7, 8, 15, 16, 31, 32, 63, 64, 127, 128, 255, 256, 1023, 1024, 4095, 4096, 65535, 65536,
           2 ** 31 - 1, -2 ** 31, 2 ** 32 - 1, 2 ** 32, -2 ** 63, 2 ** 63 - 1]
AFL_RANGES = [(1, 1), (2, 2), (3, 3), (4, 7), (8, 15), (16, 31), (32, 127), (128, 255)]


def _s64(v):
    v &= (1 << 64) - 1
    return v - (1 << 64) if v >> 63 else v


def _s32(v):
    v &= (1 << 32) - 1
    return v - (1 << 32) if v >> 31 else v


def _mutate(L, S, D, n_scalars, ops, max_block, max_threads, u0, u1, u2):
    """One mutation as the header defines it."""
    avail = [o for o, ok in ((O.MUT_LAUNCH, True), (O.MUT_SCALAR, n_scalars > 0), (O.MUT_DATA, D is not None))
             if ops & o and ok]
    if not avail:
        return
    op = avail[u0 % len(avail)]
    kind = (u1 >> 8) % 4
    if op == O.MUT_LAUNCH:
        d = u1 % 6
        v = L[d]
        v = [v + 1 + u2 % 8, v - (1 + u2 % 8) if v > 1 + u2 % 8 else 1, 1 << (u2 % 11), 1 + u2 % 256][kind]
        M = list(L)
        M[d] = v
        bs, nb = M[3] * M[4] * M[5], M[0] * M[1] * M[2]
        if 1 <= v <= 2 ** 32 - 1 and bs <= max_block and nb <= 2 ** 32 - 1 and nb * bs <= max_threads:
            L[d] = v
    elif op == O.MUT_SCALAR:
        k = u1 % n_scalars
        S[k] = _s64([S[k] ^ (1 << (u2 % 64)), S[k] + (u2 % 33) - 16, SPECIAL[u2 % 28], u2][kind])
    else:
        e = u1 % len(D)
        D[e] = _s32([int(D[e]) + (u2 % 33) - 16, SPECIAL[u2 % 28], u2, int(D[e]) ^ (1 << (u2 % 32))][kind])


def py_campaign(wl, generations, batch, max_stack, max_threads, max_block, corpus_cap, ops, seed,
                data_slot=O.NO_SLOT):
    """The campaign replayed: returns corpus (launch, scalars, data, gen),
    virgin map, sigs and stats like O.fuzz."""
    lut = np.zeros(256, np.uint8)
    for b, (lo, hi) in enumerate(AFL_RANGES):
        lut[lo: hi + 1] = 1 << b
    tab = wl.tables[wl.table_idx[0]]
    ns = wl.scalars.shape[1]
    ref = int(tab[data_slot]["data"]) if data_slot < len(tab) else 0
    d0 = np.array(wl.data[ref - 1], np.int32).ravel() if ref else None
    corpus = [([int(v) for v in wl.launch[0]], [int(v) for v in wl.scalars[0]], d0, 0)]
    virgin = np.full(65536, 0xFF, np.uint8)
    n_acc = O.validate(wl.ir)[0]
    sigs = np.full((n_acc, 4), 2 ** 64 - 1, np.uint64)
    stats = dict(execs=0, novel=0, crashes=0, generations=0)
    for g in range(generations):
        size = len(corpus)
        kids = []
        for c in range(batch):
            base = (g * batch + c) * 64
            r = lambda k: O.fuzz_rand(seed, base + k)  # noqa: E731
            L, S, D, _ = corpus[r(0) % size]
            L, S, D = list(L), list(S), None if D is None else D.copy()
            for j in range(1 + r(1) % max_stack):
                _mutate(L, S, D, ns, ops, max_block, max_threads, r(2 + 4 * j), r(3 + 4 * j), r(4 + 4 * j))
            kids.append((L, S, D))
        # the generation's children, checked together
        tabs = np.repeat(tab[None, :], batch, axis=0)
        data = list(wl.data)
        if ref:
            for c in range(batch):
                data.append(kids[c][2])
                tabs[c, data_slot]["data"] = len(data)
        kw = W.Workload("kids", wl.ir, np.array([k[0] for k in kids], np.uint32),
                        np.array([k[1] for k in kids], np.int64).reshape(batch, ns), tabs,
                        np.arange(batch, dtype=np.uint32), data, wl.mode, wl.cap_log2)
        o = O.check(kw)
        buckets = lut[o["maps"]]
        seen = np.bitwise_or.reduce(buckets, axis=0)
        for c in range(batch):
            nv = bool(np.any(buckets[c] & virgin))
            stats["novel"] += nv
            rec = o["records"][c]
            stats["crashes"] += bool(np.any(rec["count"] > 0))
            for a in range(n_acc):
                for k in range(4):
                    if rec[a]["kinds"] & (1 << k):
                        sigs[a, k] = min(int(sigs[a, k]), (g << 32) | c)
            kids[c] = kids[c] + (nv,)
        virgin &= ~seen
        for c in range(batch):
            if kids[c][3] and len(corpus) < corpus_cap:
                corpus.append((kids[c][0], kids[c][1], kids[c][2], g))
        stats["execs"] += batch
        stats["generations"] += 1
    return corpus, virgin, sigs, stats


@pytest.mark.parametrize("name", ["listing3", "stencil", "csr"])
def test_campaign_replayed_from_its_definition(name):
    if name == "listing3":
        wl = listing3_seed()
        kw = dict(ops=O.MUT_LAUNCH | O.MUT_SCALAR, max_threads=1 << 12, max_block=256)
    elif name == "stencil":
        wl = W.mini("config2", n_inputs=1, g0=3, hw0=40)
        kw = dict(ops=O.MUT_LAUNCH | O.MUT_SCALAR, max_threads=1 << 13, max_block=256)
    else:
        wl = W.mini("config3", n_inputs=1, log2_rows=8)
        kw = dict(ops=O.MUT_DATA | O.MUT_LAUNCH | O.MUT_SCALAR, data_slot=1, max_threads=1 << 12, max_block=256)
    common = dict(generations=4, batch=12, max_stack=5, corpus_cap=20, seed=23, **kw)
    got = O.fuzz(wl, **common)
    corpus, virgin, sigs, stats = py_campaign(wl, **common)
    assert len(got["gen"]) == len(corpus)
    ns = wl.scalars.shape[1]
    for k, (L, S, D, g) in enumerate(corpus):
        assert [int(v) for v in got["launch"][k]] == L, k
        assert [int(v) for v in got["scalars"][k][:ns]] == S, k
        assert int(got["gen"][k]) == g, k
        if D is not None:
            assert np.array_equal(got["data"][k], D), k
    assert np.array_equal(got["virgin"], virgin)
    assert np.array_equal(got["sigs"], sigs)
    assert got["stats"] == stats
    assert len(corpus) > 2


def test_identical_children_all_novel_in_their_generation():
    """With no mutation operator enabled every child is a copy of the seed
    (which is never executed by itself): all children of generation 0 are
    novel (judged against the map as at the generation's start), none later."""
    wl = listing3_seed()
    out = O.fuzz(wl, generations=3, batch=5, ops=0, corpus_cap=64, seed=1)
    assert out["stats"]["novel"] == 5
    assert list(out["gen"]) == [0, 0, 0, 0, 0, 0]
