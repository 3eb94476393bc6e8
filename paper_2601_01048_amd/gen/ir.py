"""Builder and serialiser for the index-program IR (the byte format that
``ckc_load_program`` accepts; the format is specified in ``include/ckc_ir.h``).

An index program is a kernel reduced to what decides its memory accesses: the
integer index arithmetic, the branches and loops around the accesses, and the
loads that feed other indices -- the part the paper's AXIPrune keeps
(Section 5.2, Algorithm 2) and its affine-access analysis reads (Section 5.1.1).

This module only writes bytes: it performs none of the checking arithmetic.
It is shared by the workload generators, the tests and the benchmark as the
source of inputs for both the oracle and the GPU library.
"""
from __future__ import annotations

import struct
from contextlib import contextmanager
from dataclasses import dataclass

MAGIC = 0x31434B43
VERSION = 1
NO_SITE = 0xFFFF
NO_REG = 0xFFFF

OP = dict(
    NOP=0, CONST=1, SCALAR=2, SPECIAL=3,
    ADD=8, SUB=9, MUL=10, DIVS=11, DIVU=12, REMS=13, REMU=14,
    AND=15, OR=16, XOR=17, SHL=18, SHRA=19, SHRL=20,
    MINS=21, MAXS=22, MINU=23, MAXU=24,
    CMPEQ=25, CMPNE=26, CMPLTS=27, CMPLES=28, CMPLTU=29, CMPLEU=30,
    SELECT=31, SEXT=32, ZEXT=33, TRUNC=34,
    FADD=40, FSUB=41, FMUL=42, FEXP=43, ITOF=44, FTOI=45,
    ACCESS=48, LOAD=49, STORE=50, IF=56, ELSE=57, ENDIF=58, LOOP=59, ENDLOOP=60, BARRIER=61,
)
BINARY = ("ADD SUB MUL DIVS DIVU REMS REMU AND OR XOR SHL SHRA SHRL MINS MAXS "
          "MINU MAXU CMPEQ CMPNE CMPLTS CMPLES CMPLTU CMPLEU").split()
SPECIALS = ["tid.x", "tid.y", "tid.z", "bid.x", "bid.y", "bid.z",
            "bdim.x", "bdim.y", "bdim.z", "gdim.x", "gdim.y", "gdim.z"]

INSTR = struct.Struct("<BBHHHHHHH")   # op, w, dst, a, b, c, d, s0, s1  (16 bytes)
HEADER = struct.Struct("<IHHHHHHHHI8x")  # ... n_regs, slot_spaces, reserved
SPACE = dict(global_=0, shared=1, local=2)


@dataclass(frozen=True)
class Reg:
    idx: int
    w: int  # width the value was produced at (32 or 64)


class Program:
    """Incremental builder.  Methods append one instruction and return the
    defined register (or the access id for ACCESS).  Sites are numbered in
    creation order; their coverage-map ids default to ``site_base + index``."""

    def __init__(self, n_scalars: int = 0, n_slots: int = 1, site_base: int = 0,
                 site_stride: int = 1, spaces=None):
        self.n_scalars = n_scalars
        self.n_slots = n_slots
        # memory space per slot: 0 global, 1 shared (per block), 2 local (per thread)
        self.spaces = list(spaces) if spaces is not None else [0] * n_slots
        self.instrs: list[tuple] = []
        self.consts: list[int] = []
        self.site_ids: list[int] = []
        self.n_regs = 0
        self.n_accesses = 0
        self._site_base = site_base
        self._site_stride = site_stride
        self._open: list[str] = []

    # -- helpers -------------------------------------------------------------
    def _new(self, w: int) -> Reg:
        r = Reg(self.n_regs, w)
        self.n_regs += 1
        return r

    def site(self, site_id: int | None = None) -> int:
        """Allocate a coverage site; returns its index."""
        if site_id is None:
            site_id = (self._site_base + len(self.site_ids) * self._site_stride) & 0xFFFF
        self.site_ids.append(site_id)
        return len(self.site_ids) - 1

    def _site_arg(self, s) -> int:
        if s is None or s is False:
            return NO_SITE
        if s is True:
            return self.site()
        return int(s)

    def _emit(self, op, w=0, dst=NO_REG, a=0, b=0, c=0, d=0, s0=NO_SITE, s1=NO_SITE):
        self.instrs.append((OP[op], w, dst, a, b, c, d, s0, s1))

    # -- sources -------------------------------------------------------------
    def const(self, value: int, w: int = 32) -> Reg:
        value = int(value)
        if value not in self.consts:
            self.consts.append(value)
        r = self._new(w)
        self._emit("CONST", w, r.idx, self.consts.index(value))
        return r

    def scalar(self, k: int, w: int = 64) -> Reg:
        r = self._new(w)
        self._emit("SCALAR", w, r.idx, k)
        return r

    def special(self, name: str) -> Reg:
        r = self._new(64)
        self._emit("SPECIAL", 64, r.idx, SPECIALS.index(name))
        return r

    # -- arithmetic ----------------------------------------------------------
    def _as_reg(self, v, w):
        return v if isinstance(v, Reg) else self.const(v, w)

    def op(self, name: str, a, b, w: int | None = None) -> Reg:
        if w is None:
            w = a.w if isinstance(a, Reg) else b.w
        a = self._as_reg(a, w)
        b = self._as_reg(b, w)
        r = self._new(w)
        self._emit(name, w, r.idx, a.idx, b.idx)
        return r

    def select(self, cond: Reg, t, f, w: int | None = None) -> Reg:
        if w is None:
            w = t.w if isinstance(t, Reg) else f.w
        t = self._as_reg(t, w)
        f = self._as_reg(f, w)
        r = self._new(w)
        self._emit("SELECT", w, r.idx, cond.idx, t.idx, f.idx)
        return r

    def sext(self, a: Reg) -> Reg:
        r = self._new(64)
        self._emit("SEXT", 64, r.idx, a.idx)
        return r

    def zext(self, a: Reg) -> Reg:
        r = self._new(64)
        self._emit("ZEXT", 64, r.idx, a.idx)
        return r

    def trunc(self, a: Reg) -> Reg:
        r = self._new(32)
        self._emit("TRUNC", 32, r.idx, a.idx)
        return r

    # -- memory --------------------------------------------------------------
    def access(self, slot: int, idx: Reg, elem: int = 4, write: bool = False,
               w: int | None = None, site=True) -> int:
        w = idx.w if w is None else w
        acc = self.n_accesses
        self.n_accesses += 1
        flags = (elem.bit_length() - 1) | (4 if write else 0)
        self._emit("ACCESS", w, NO_REG, idx.idx, acc, slot, flags, self._site_arg(site))
        return acc

    def store(self, slot: int, idx: Reg, value: Reg, elem: int = 4, w: int | None = None,
              site=True) -> int:
        """Checked write of ``value`` (a STORE: kept as data only for shared
        slots read back by a LOAD)."""
        w = idx.w if w is None else w
        acc = self.n_accesses
        self.n_accesses += 1
        self._emit("STORE", w, value.idx, idx.idx, acc, slot, elem.bit_length() - 1, self._site_arg(site))
        return acc

    def barrier(self):
        """__syncthreads (top level only)."""
        self._emit("BARRIER")

    def fop(self, name: str, a: Reg, b: Reg | None = None) -> Reg:
        """FADD / FSUB / FMUL (a, b) or FEXP (a): binary64 bit patterns."""
        r = self._new(64)
        self._emit(name, 64, r.idx, a.idx, 0 if b is None else b.idx)
        return r

    def itof(self, a: Reg) -> Reg:
        r = self._new(64)
        self._emit("ITOF", 32, r.idx, a.idx)
        return r

    def ftoi(self, a: Reg, w: int = 32) -> Reg:
        r = self._new(w)
        self._emit("FTOI", w, r.idx, a.idx)
        return r

    def load(self, slot: int, idx: Reg, elem: int = 4, w: int | None = None,
             site=True) -> Reg:
        w = idx.w if w is None else w
        acc = self.n_accesses
        self.n_accesses += 1
        r = self._new(64 if elem == 8 else 32)
        self._emit("LOAD", w, r.idx, idx.idx, acc, slot, elem.bit_length() - 1,
                   self._site_arg(site))
        return r

    # -- control flow --------------------------------------------------------
    @contextmanager
    def if_(self, pred: Reg, site_t=True, site_f=True):
        self._emit("IF", 0, NO_REG, pred.idx, 0, 0, 0, self._site_arg(site_t),
                   self._site_arg(site_f))
        self._open.append("IF")
        yield
        assert self._open.pop() == "IF"
        self._emit("ENDIF")

    def else_(self):
        """Call inside an ``if_`` block to start its false arm."""
        assert self._open and self._open[-1] == "IF"
        self._emit("ELSE")

    @contextmanager
    def loop(self, start, end, step=1, w: int = 32, site_iter=True, site_exit=True):
        start = self._as_reg(start, w)
        end = self._as_reg(end, w)
        step = self._as_reg(step, w)
        ctr = self._new(w)
        self._emit("LOOP", w, ctr.idx, start.idx, end.idx, step.idx, 0,
                   self._site_arg(site_iter), self._site_arg(site_exit))
        self._open.append("LOOP")
        yield ctr
        assert self._open.pop() == "LOOP"
        self._emit("ENDLOOP")

    # -- output --------------------------------------------------------------
    def to_bytes(self) -> bytes:
        assert not self._open, "unclosed IF/LOOP"
        spaces = 0
        for k, sp in enumerate(self.spaces):
            spaces |= (sp & 3) << (2 * k)
        out = bytearray(HEADER.pack(MAGIC, VERSION, len(self.instrs), len(self.consts),
                                    self.n_scalars, self.n_slots, self.n_accesses,
                                    len(self.site_ids), self.n_regs, spaces))
        for c in self.consts:
            out += struct.pack("<q", c)
        sites = struct.pack(f"<{len(self.site_ids)}H", *self.site_ids)
        sites += b"\0" * (-len(sites) % 8)
        out += sites
        for ins in self.instrs:
            out += INSTR.pack(*ins)
        return bytes(out)


def with_op_helpers():
    """Attach ``add``/``sub``/... shorthands for every binary op."""
    for name in BINARY:
        def f(self, a, b, w=None, _n=name):
            return self.op(_n, a, b, w)
        setattr(Program, name.lower(), f)


with_op_helpers()


def header_of(ir: bytes) -> dict:
    """Decode only the header (for generators and harness bookkeeping)."""
    f = HEADER.unpack_from(ir, 0)
    keys = ["magic", "version", "n_instr", "n_consts", "n_scalars", "n_slots",
            "n_accesses", "n_sites", "n_regs", "slot_spaces"]
    return dict(zip(keys, f))
