"""Host-side tests of the library (no GPU): the C-ABI loads and exports every
declared symbol, the load-time analysis classifies programs and reproduces the
paper's affine decomposition of Listing 1, pruning removes instructions that
feed no index, and malformed IR is rejected without crashing, in agreement with
the oracle's own decoder."""
import os
import re

import numpy as np
import pytest

import kernels as K
from oracle import oracle as O
from paper_2601_01048_amd import ckc
from paper_2601_01048_amd.gen import workloads as W
from paper_2601_01048_amd.gen.ir import Program

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _have_lib():
    return os.path.exists(ckc.LIB)


pytestmark = pytest.mark.skipif(not _have_lib(), reason="libckc.so not built")


def test_exports_every_declared_symbol():
    decl = set()
    for h in ("ckc.h",):
        txt = open(os.path.join(ROOT, "include", h)).read()
        decl |= set(re.findall(r"\b(ckc_[a-z_]+)\s*\(", txt))
    lib = ckc.lib()
    assert decl, "no declarations found"
    for name in sorted(decl):
        assert hasattr(lib, name), name


def test_listing1_affine_decomposition():
    """Section 5.1.1: the seven accesses of Listing 1 use two indices,
    threadIdx.x and blockIdx.x*blockDim.x + threadIdx.x, with
    T = [[1, 0], [1, blockDim.x]] over (threadIdx.x, blockIdx.x) and b = 0."""
    info, acc = ckc.analyze(K.listing1_program())
    assert info["n_accesses"] == 7
    assert info["cls"] & ckc.CLS["AFFINE"] and not info["cls"] & ckc.CLS["GUARDED"]
    bdim_reg = 4  # register defined by SPECIAL bdim.x in listing1_program
    rows = set()
    for a in acc:
        assert a["affine"] and not a["guarded"] and not a["indirect"]
        c = a["coef"]
        assert c[0] == (1, 1)                      # tid.x coefficient 1
        assert c[1] == c[2] == c[4] == c[5] == (0, 0)
        assert c[6] == (1, 0)                      # b = 0
        rows.add(c[3])
    assert rows == {(0, 0), (2, bdim_reg)}          # bid.x: 0 or blockDim.x


def test_program_classes():
    def cls(ir):
        return {k for k, v in ckc.CLS.items() if ckc.analyze(ir)[0]["cls"] & v}
    assert cls(W.f1_program()) == {"AFFINE", "UNIFORM"}
    assert cls(W.f2_program(64)) == {"AFFINE", "UNIFORM", "I64"}
    assert cls(W.f3_program()) == {"GUARDED", "INDIRECT", "EXPANDED", "GATHER"}
    assert cls(W.f3_program(64)) == {"GUARDED", "INDIRECT", "I64", "EXPANDED", "GATHER"}
    assert cls(K.listing3_program()) == {"AFFINE", "GUARDED"}
    # thread-dependent product: not affine
    p = Program(n_scalars=0, n_slots=1)
    t = p.special("tid.x")
    p.access(0, p.mul(t, t, 32))
    assert "AFFINE" not in cls(p.to_bytes())
    # sign extension of a thread-dependent 32-bit value into a 64-bit index
    p = Program(n_scalars=0, n_slots=1)
    g = p.add(p.special("tid.x"), p.const(5, 32), 32)
    p.access(0, p.sext(g), w=64)
    assert "AFFINE" not in cls(p.to_bytes())


def test_pruning_keeps_only_index_slice():
    """Arithmetic that feeds no index, guard or loop bound is removed
    (MathElimination of Algorithm 2); divisions stay because they count
    arithmetic faults."""
    p = Program(n_scalars=1, n_slots=1)
    t = p.special("tid.x")
    junk = p.mul(p.add(t, 3, 32), p.const(7, 32), 32)
    p.xor(junk, t, 32)                         # dead
    p.divs(t, p.scalar(0, 32), 32)              # dead value, kept for faults
    p.access(0, p.add(t, 1, 32))
    info, _ = ckc.analyze(p.to_bytes())
    # live: tid.x, scalar, divs, const 1, add, access
    assert info["n_instr_live"] == 6


def _pressure_program(k):
    """tid.x, then k values tid.x + c_j that all stay live until a final sum:
    the pressure peaks at k + 1 (the last constant, the k - 1 earlier sums'
    operands, tid.x and the constant itself)."""
    p = Program(n_scalars=0, n_slots=1)
    t = p.special("tid.x")
    vs = [p.add(t, p.const(j, 32), 32) for j in range(k)]
    acc = vs[0]
    for v in vs[1:]:
        acc = p.add(acc, v, 32)
    p.access(0, acc)
    return p.to_bytes()


def test_register_limit_at_and_over():
    """The live-register rule of ckc_ir.h (CKC_IR_MAX_LIVE_REGS = 32): the
    library and the oracle accept a program at the limit and both reject one
    register over it."""
    p = Program(n_scalars=0, n_slots=1)
    t = p.special("tid.x")
    for k in range(40):  # each value dies at its access: registers are reused
        p.access(0, p.add(t, p.const(k, 32), 32))
    ckc.analyze(p.to_bytes())
    O.validate(p.to_bytes())
    at, over = _pressure_program(31), _pressure_program(32)
    info, _ = ckc.analyze(at)
    assert info["n_regs_phys"] <= 32
    O.validate(at)
    with pytest.raises(ckc.CkcError) as e:
        ckc.analyze(over)
    assert e.value.code == -2
    with pytest.raises(O.OracleError):
        O.validate(over)


def test_register_rule_agrees_with_oracle_on_random_programs():
    """Random programs around the limit (loops keep values live to their end):
    the library accepts exactly what the oracle accepts."""
    import randprog as R
    rng = np.random.default_rng(31)
    verdicts = set()
    for k in range(300):
        ir = R.random_program(rng, budget=int(rng.integers(20, 140)))
        try:
            O.validate(ir)
            ok_o = True
        except O.OracleError:
            ok_o = False
        try:
            ckc.analyze(ir)
            ok_l = True
        except ckc.CkcError:
            ok_l = False
        assert ok_o == ok_l, ir.hex()
        verdicts.add(ok_o)
    assert verdicts == {True, False}


def test_malformed_ir_agrees_with_oracle():
    rng = np.random.default_rng(9)
    for base in (W.f3_program(), W.f2_program(), K.listing3_program()):
        for _ in range(400):
            b = bytearray(base)
            for _ in range(int(rng.integers(1, 4))):
                b[int(rng.integers(32, len(b)))] = int(rng.integers(0, 256))
            b = bytes(b)
            try:
                O.validate(b)
                ok_oracle = True
            except O.OracleError:
                ok_oracle = False
            try:
                ckc.analyze(b)
                ok_lib = True
            except ckc.CkcError as e:
                assert e.code == -2
                ok_lib = False
            assert ok_oracle == ok_lib, b.hex()


def test_truncated_and_garbage_ir():
    for b in (b"", b"\x00" * 8, W.f1_program()[:-16], b"CKC1" + b"\xff" * 60):
        with pytest.raises(ckc.CkcError):
            ckc.analyze(b)


def test_gather_classification():
    """Expanded bodies with a thread coordinate, two varying operands in one
    index, control flow or a product of varying values stay interpreted; the
    plain gather shapes are recognised."""
    import gatherprog as G
    rng = np.random.default_rng(3)
    n_gather = 0
    for k in range(80):
        near = k % 2 == 1
        info, _ = ckc.analyze(G.gather_program(rng, near_miss=near))
        assert info["cls"] & ckc.CLS["EXPANDED"]
        if near:
            assert not info["cls"] & ckc.CLS["GATHER"], k
        n_gather += bool(info["cls"] & ckc.CLS["GATHER"])
    assert n_gather >= 10


def test_slot_spaces_agree_with_oracle():
    """The header's slot-space word (2 bits per slot: global, shared, local):
    every value of each field, fields beyond n_slots, and LOADs from global,
    shared (allowed: shared memory is read back) and local slots (refused),
    accepted or refused alike by the loader and the oracle's decoder."""
    from paper_2601_01048_amd.gen.ir import Program
    cases = []
    for spaces in ([0, 0], [1, 2], [2, 0], [3, 0], [0, 3], [1, 1, 1], [0, 0, 2]):
        p = Program(n_slots=2, spaces=spaces)
        p.access(0, p.const(0, 32), elem=4)
        p.access(1, p.const(1, 32), elem=4)
        cases.append(p.to_bytes())
    for sp in (0, 1, 2):
        p = Program(n_slots=2, spaces=[0, sp])
        p.load(1, p.const(0, 32), elem=4)
        cases.append(p.to_bytes())
    results = []
    for b in cases:
        try:
            O.validate(b)
            ok_oracle = True
        except O.OracleError:
            ok_oracle = False
        try:
            ckc.analyze(b)
            ok_lib = True
        except ckc.CkcError as e:
            assert e.code == -2
            ok_lib = False
        assert ok_oracle == ok_lib, b[:32].hex()
        results.append(ok_lib)
    assert results == [True, True, True, False, False, False, False, True, True, False]


def test_rows_form_flag():
    """The loader's rows-form decision, which picks the whole-thread kernel:
    the CSR program (guard, two row-pointer loads, the gather loop, y[r]) is
    all 32-bit at width 32 (2), and its int64 form is not a rows form (0);
    the all-32-bit program of the int32-range test is 2; the CSR shape at
    width 32 with one 64-bit access after the loop is 1; a program with no
    expanded loop (F1) is 0."""
    import rowsprog as RP
    assert ckc.analyze(W.f3_program(32))[0]["rows_form"] == 2
    assert ckc.analyze(W.f3_program(64))[0]["rows_form"] == 0
    assert ckc.analyze(RP.extreme_rows_program())[0]["rows_form"] == 2
    assert ckc.analyze(W.f1_program(32))[0]["rows_form"] == 0
    p = Program(n_scalars=1, n_slots=5)
    r = p.add(p.mul(p.special("bid.x"), p.special("bdim.x"), 32), p.special("tid.x"), 32)
    r64 = p.add(p.mul(p.special("bid.x"), p.special("bdim.x"), 64), p.special("tid.x"), 64)
    with p.if_(p.cmplts(r, p.scalar(0, 32), 32)):
        rp0 = p.load(0, r, elem=4, w=32)
        rp1 = p.load(0, p.add(r, p.const(1, 32), 32), elem=4, w=32)
        with p.loop(rp0, rp1, 1, w=32) as j:
            c = p.load(1, j, elem=4, w=32)
            p.access(2, j, elem=4, w=32)
            p.access(3, c, elem=4, w=32)
        p.access(4, r64, elem=4, write=True, w=64)
    assert ckc.analyze(p.to_bytes())[0]["rows_form"] == 1
