"""Pins of the oracle's shared memory, barriers and floating-point data math,
and of the pruning (the paper's AXIPrune, Section 5.2, Algorithm 2: slicing
the index computations, removing the data math that reaches no index and the
barriers when no index reads shared memory).

The oracle runs every program as written (nothing pruned): its results are
the definition, which the pruned device program must reproduce.  Pins:
block-level models of kernels with shared memory written from their formulas
(``sharedprog``), against records, counts and status; FP conversions and
operations against Python's IEEE doubles; FEXP against the C library's exp
within a few units in the last place; and the pruned live set -- the loader's
(the library, on the host) against what each kernel marks as droppable while
it is built, and against the oracle's count of executed instructions."""
import math

import numpy as np
import pytest

import brute
import sharedprog as SP
from oracle import oracle as O
from paper_2601_01048_amd import ckc
from paper_2601_01048_amd.gen import workloads as W


def run_case(case, launches, tables, mode="full", scalars=None, data=()):
    wl = SP.workload(case, launches, tables, scalars=scalars, data=data,
                     mode={"full": W.MODE_FULL, "boundary": W.MODE_BOUNDARY}[mode])
    got = O.check(wl)
    exp = SP.expected(case, launches, tables, scalars=scalars, data=data, mode=mode)
    brute.assert_matches(got, exp)
    return got


def test_ir_exp_within_ulps_of_libm():
    """FEXP's fixed method is within 2 units in the last place of the C
    library's exp over the whole finite range (subnormal results included),
    exact at 0, and follows the special cases of the IR definition."""
    rng = np.random.default_rng(1)
    xs = np.concatenate([rng.uniform(-745.0, 709.78, 20000), rng.uniform(-1, 1, 5000),
                         rng.uniform(-745.13, -708.4, 3000), [0.0, -0.0, 1.0, -1.0, 0.5, 709.78, -745.13]])
    worst = 0.0
    for x in xs:
        x = float(x)
        got, ref = O.ir_exp(x), math.exp(x)
        worst = max(worst, SP.exp_ulps(got, ref))
    assert worst <= 2.0, worst
    assert O.ir_exp(0.0) == 1.0
    assert math.isnan(O.ir_exp(float("nan")))
    assert O.ir_exp(float("inf")) == math.inf and O.ir_exp(-math.inf) == 0.0
    assert O.ir_exp(709.79) == math.inf and math.isfinite(O.ir_exp(709.782712893384))
    assert O.ir_exp(-745.14) == 0.0 and O.ir_exp(-745.13) > 0.0


FP_CONSTS = [float("nan"), math.inf, -math.inf, 1e20, -1e20, 2147483647.5, 2147483648.0, -2147483648.5,
             -2147483649.0, 9.3e18, -9.3e18, -2.9, 2.9, -0.0, 5e-324, 2.0 ** 63, -(2.0 ** 63), 17.999999999]


def test_ftoi_special_values():
    """FTOI at widths 32 and 64: truncation toward zero, NaN 0, saturation
    at both ends, exactly at and beyond 2^31 and 2^63."""
    for part in (FP_CONSTS[:9], FP_CONSTS[9:]):  # at most 16 scalars a program
        case = SP.fp_index(part)
        sc = [[SP.f2bits(c) for c in part]]
        run_case(case, [[1, 1, 1, 2, 1, 1]], [[(SP.LB + 4096, 4 * 16, 0, 0, 0)]], scalars=sc)


@pytest.mark.parametrize("launch", [[2, 1, 1, 16, 1, 1], [3, 1, 1, 64, 1, 1]])
def test_fp_arith_and_data_math(launch):
    """ITOF of negative values, FMUL/FSUB/FADD rounded one by one, and the
    ep-like kernel (an index through FP next to a chain that no index reads)."""
    run_case(SP.fp_arith(), [launch], [[(SP.LB + 4096, 4 * 20, 0, 0, 0)]])
    run_case(SP.ep_like(), [launch], [[(SP.LB + 4096, 4 * 30, 0, 0, 0), (SP.LB + 65536, 4 * 100, 0, 0, 0)]])


SHARED = [SP.rotate, lambda: SP.rotate(dims=3), lambda: SP.rotate(k=-5, c=40), SP.racing_max, SP.phases,
          SP.shared_divisor, SP.bounds, lambda: SP.bounds(off=2), SP.tile_gather, SP.prefix_max, SP.hist_like]


@pytest.mark.parametrize("k", range(len(SHARED)))
@pytest.mark.parametrize("mode", ["full", "boundary"])
def test_shared_kernels_against_block_models(k, mode):
    """Each kernel over grids of several block shapes (the shared array
    smaller than the block in some tables, so stores and loads leave it)."""
    case = SHARED[k]()
    rng = np.random.default_rng(40 + k)
    data = [SP.data_array(rng)]
    dims3 = case.name == "rotate3d"
    launches = []
    for bs in ((4, 3, 2), (2, 2, 2), (5, 1, 3)) if dims3 else ((1, 1, 1), (7, 1, 1), (32, 1, 1), (40, 1, 1)):
        for g in ((1, 1, 1), (3, 1, 1), (2, 3, 1)):
            launches.append(list(g) + list(bs))
    tables = SP.tables_for(case, rng, len(launches), sh_elems=None)
    got = run_case(case, launches, tables, mode=mode, data=data)
    if case.name in ("rotate1d", "racing_max", "phases", "bounds-3", "prefix_max"):
        assert int(got["records"]["count"].sum()) > 0  # violations that depend on shared values


def test_racing_writes_keep_the_signed_maximum():
    """All threads of a 40-thread block write sh[1] = 5 - 3t: the largest is
    5 (thread 0) as a signed value, which A[5] accepts; the most negative
    value (the largest unsigned one) would underflow A."""
    case = SP.racing_max(d=5)
    got = run_case(case, [[1, 1, 1, 40, 1, 1]], [[(SP.LB + 4096, 4 * 36, 0, 0, 0), (SP.SH_BASE, 8, 0, 0, 0)]])
    assert int(got["records"][0, 5]["count"]) == 0
    # sh[0] ends as 39 - 5 = 34 < 36: in bounds too
    assert int(got["records"][0, 4]["count"]) == 0
    got = run_case(case, [[1, 1, 1, 45, 1, 1]], [[(SP.LB + 4096, 4 * 36, 0, 0, 0), (SP.SH_BASE, 8, 0, 0, 0)]])
    assert int(got["records"][0, 4]["count"]) == 45 and int(got["records"][0, 4]["index"]) == 39


def test_loads_see_the_phase_start():
    """phases: the load right after the first store reads 0 (the phase's
    start), the next phase's load reads t + 100 for every t, the last one
    2t + 1 for even t; A of 120 elements separates the three."""
    case = SP.phases()
    bs = 32
    got = run_case(case, [[1, 1, 1, bs, 1, 1]], [[(SP.LB + 4096, 4 * 120, 0, 0, 0), (SP.SH_BASE, 4 * bs, 0, 0, 0)]])
    r = got["records"][0]
    assert int(r[2]["count"]) == 0                                            # A[0]
    assert int(r[6]["count"]) == sum(1 for t in range(bs) if t + 100 >= 120)  # A[t + 100]
    assert int(r[7]["count"]) == sum(1 for t in range(bs) if (2 * t + 1 if t % 2 == 0 else t + 100) >= 120)


def test_division_by_shared_values_counts_faults():
    """shared_divisor: t mod 3 is 0 for ceil(bs / 3) threads of every block,
    so that many divisions by zero (read back from the neighbour's element)."""
    case = SP.shared_divisor()
    for bs, nb in ((30, 2), (31, 3), (1, 4)):
        got = run_case(case, [[nb, 1, 1, bs, 1, 1]], [[(SP.LB + 4096, 4 * 64, 0, 0, 0), (SP.SH_BASE, 4 * bs, 0, 0, 0)]])
        assert int(got["status"][0]["arith_faults"]) == nb * ((bs + 2) // 3)


def _live(ir):
    info, _ = ckc.analyze(ir)
    return info


def test_pruned_live_set():
    """The loader's live instruction count: the ep-like kernel drops its FP
    chain, the histogram its increment and barrier (no index reads shared
    memory), kernels whose indices read shared memory keep everything (the
    unpruned load, which keeps everything, needs a device context: a GPU
    test); the class bit of index-related shared memory is set exactly when
    an index reads it."""
    ep = SP.ep_like()
    info = _live(ep.ir)
    assert info["n_instr_live"] == ep.n_instr - ep.n_data
    h = SP.hist_like()
    info = _live(h.ir)
    assert info["n_instr_live"] == h.n_instr - h.n_drop
    assert not info["cls"] & ckc.CLS["BARRIER"]
    for mk in (SP.rotate, SP.racing_max, SP.phases, SP.tile_gather, SP.prefix_max, SP.bounds):
        c = mk()
        info = _live(c.ir)
        assert info["n_instr_live"] == c.n_instr, c.name
        assert info["cls"] & ckc.CLS["BARRIER"], c.name
    # the shared value reaches a division only: the barrier stays (the
    # division's faults depend on it), indices do not read shared memory
    d = SP.shared_divisor()
    info = _live(d.ir)
    assert info["n_instr_live"] == d.n_instr
    assert not info["cls"] & ckc.CLS["BARRIER"]


@pytest.mark.parametrize("mk", [SP.ep_like, SP.hist_like, SP.shared_divisor, SP.rotate, SP.fp_arith])
def test_executed_counts_match_the_live_set(mk):
    """Straight-line kernels (hist_like: its IF aside) execute every
    instruction once per thread; the oracle's count of executed instructions
    of the pruned program is the loader's live count per thread.  ENDIF,
    ELSE and ENDLOOP only mark where a region ends: they are not counted."""
    case = mk()
    rng = np.random.default_rng(7)
    launches = [[3, 1, 1, 32, 1, 1], [2, 1, 1, 8, 1, 1]]
    tables = SP.tables_for(case, rng, 2, sh_elems=64)
    wl = SP.workload(case, launches, tables, data=[SP.data_array(rng)])
    ex = O.check(wl, executed=True)["executed"]
    live = _live(case.ir)["n_instr_live"]
    for i, l in enumerate(launches):
        lanes = l[0] * l[3]
        if case.name == "hist_like":
            # the IF region (7 instructions, all kept) runs in threads t < 16
            inside = min(l[3], 16)
            assert int(ex[i, 0]) == lanes * (case.n_instr - 8) + l[0] * inside * 7
            assert int(ex[i, 1]) == lanes * (live - 8) + l[0] * inside * 7
        else:
            assert int(ex[i, 0]) == lanes * case.n_instr
            assert int(ex[i, 1]) == lanes * live
