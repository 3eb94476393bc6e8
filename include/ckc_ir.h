/*
 * ckc_ir.h — binary format of the index-program IR accepted by ckc_load_program().
 *
 * An index program is the part of a GPU kernel that decides which memory it
 * touches: the integer index computations of its memory accesses, the
 * branches and loops that guard them, and the loads whose values feed other
 * indices.  It is what remains of a kernel after the paper's AXIPrune pass has
 * removed every instruction that feeds no index and no branch (Section 5.2,
 * Algorithm 2, MathElimination), written down directly instead of extracted
 * from NVVM IR.  Everything here is integer: the arithmetic the paper's
 * affine-access analysis reasons about (Section 5.1.1) plus the control flow
 * its PREX runtime has to respect (Section 5.1.2, Listing 3).
 *
 * ------------------------------------------------------------------------
 * Layout (little-endian, no padding except where stated)
 *
 *   ckc_ir_header                        32 bytes
 *   int64_t  consts[n_consts]            constant pool
 *   uint16_t site_ids[n_sites]           coverage-map position of each site,
 *                                        padded with zeros to a multiple of 8 bytes
 *   ckc_ir_instr instrs[n_instr]         16 bytes each
 *
 * The byte count handed to ckc_load_program must equal this layout exactly.
 *
 * ------------------------------------------------------------------------
 * Values and registers
 *
 * Registers are SSA virtual registers 0..n_regs-1, each defined by exactly one
 * instruction.  Every register is a 64-bit container.  A value of width 32 is
 * kept sign-extended from its low 32 bits; an operation of width w reads the
 * low w bits of each operand (sign-extended when w = 32) and wraps its result
 * modulo 2^w.  A register defined inside an IF/ELSE arm or a LOOP body is
 * visible only up to the end of that arm or body; a LOOP counter is visible
 * only inside its body.  There are no phi nodes (SELECT gives conditional
 * values), so the only state carried from one loop iteration to the next is the
 * counter.
 *
 * Special sources (SPECIAL, operand a): 0..2 tid.x/y/z, 3..5 bid.x/y/z,
 * 6..8 bdim.x/y/z, 9..11 gdim.x/y/z; each is a u32 zero-extended into the
 * container.
 *
 * Integer semantics (width w in {32, 64}):
 *   ADD SUB MUL           wrap modulo 2^w
 *   DIVS REMS             truncate toward zero; x/0 = x%0 = 0 and counts an
 *                         arithmetic fault; INT_MIN/-1 = INT_MIN, INT_MIN%-1 = 0
 *                         (no fault)
 *   DIVU REMU             unsigned; x/0 = x%0 = 0 with a fault
 *   AND OR XOR
 *   SHL SHRA SHRL         shift amount taken modulo w
 *   MINS MAXS MINU MAXU
 *   CMPEQ CMPNE CMPLTS CMPLES CMPLTU CMPLEU     result 0 or 1
 *   SELECT                dst = (a != 0) ? b : c, the condition register a
 *                         tested as a whole 64-bit container; the chosen
 *                         value is then narrowed to width w
 *   SEXT ZEXT             low 32 bits of a, sign-/zero-extended to 64
 *   TRUNC                 low 32 bits of a, as a width-32 value
 *
 * ------------------------------------------------------------------------
 * Memory accesses and the allocation table
 *
 * ACCESS and LOAD name an allocation slot 0..n_slots-1 of the input's
 * allocation table, an element size 2^log2_elem bytes and an index register
 * read at width w.  Each is checked against that one allocation, record and
 * continue:
 *     kind = NULL  if the slot's base is 0
 *          = FREED if the slot carries the FREED flag
 *          = UNDER if index < 0
 *          = OVER  if index >= floor(size_bytes / 2^log2_elem)
 *          = none  otherwise
 * LOAD then reads the element (4 bytes sign-extended, or 8 bytes) from the
 * slot's data; a LOAD outside those bounds reads 0 and the lane continues.
 * Slots live in a memory space declared in the header (global, per-block
 * shared, per-thread local); LOAD reads global and shared slots.
 *
 * STORE is a checked write like ACCESS that also carries a value register.
 * A STORE of 4-byte elements to a shared slot, within bounds, writes the
 * value's low 32 bits into the block's instance of the slot; every other
 * STORE only checks (global memory holds the host's data; local memory is
 * not modelled).  Shared memory works in phases: BARRIER (the kernel's
 * __syncthreads, written at the top level only) ends a phase.  Every element
 * of a shared instance starts at 0; a LOAD from a shared slot (4-byte
 * elements) reads the element as it was at the start of the phase; at the end
 * of a phase each element written in it takes the largest (signed) value
 * stored to it in the phase.  For a kernel without racing writes this is the
 * value of its one write.
 *
 * Non-index arithmetic (the data math of a kernel, what the paper's
 * MathElimination removes when their values reach no index): FADD FSUB FMUL on
 * IEEE binary64 bit patterns in 64-bit registers (round to nearest even);
 * FEXP e^x by one fixed method, so that every implementation gives the same
 * bits: k = floor(x * (1/ln 2) + 1/2), r = (x - k * ln2_hi) - k * ln2_lo with
 * ln2_hi = 0x1.62e42ffp-1 (ln 2 rounded to 29 significant bits) and ln2_lo =
 * -0x1.718432a1b0e26p-35, the Taylor polynomial sum r^i / i! (i = 0..13,
 * coefficients rounded to binary64) in Horner form, times 2^k (for k below
 * -1022: times 2^(k+1000), then 2^-1000; for k = 1024: 2^1023, then 2);
 * NaN stays NaN, x > 709.782712893384 gives +inf, x < -745.1332191019412
 * gives 0; every operation rounded on its own (no fused multiply-add).  ITOF
 * converts an int32 (w = 32) exactly; FTOI truncates toward zero to width w,
 * NaN giving 0 and values out of range the nearest representable one.
 *
 * ------------------------------------------------------------------------
 * Control flow (structured; matching is by nesting, not by stored targets)
 *
 *   IF p ... [ELSE ...] ENDIF    arm taken when register p != 0; visits site s0
 *                                on the true outcome, s1 on the false one
 *   LOOP ctr, start, end, step ... ENDLOOP
 *        For step >= 0 the trip count is n = ceil((end-start)/step) if
 *        start < end, else 0 (step = 0 with start < end never ends); for
 *        step < 0 it is ceil((start-end)/-step) if start > end, else 0.  The
 *        quantities are exact integers of the width-w operands.  Iteration k
 *        sets ctr = start + k*step (mod 2^w) and visits site s0 first.  After
 *        a normal exit the loop visits s1.  Loops nest at most 2 deep.  When n
 *        exceeds the batch's trip cap for that depth the loop runs cap
 *        iterations and then the thread stops (a hang): it visits no further
 *        site and checks no further access.
 *   IF and LOOP blocks nest at most 16 deep in total.
 *
 * Site index 0xFFFF means "no site".  Every site index and every access id is
 * used by at most one instruction; every access id 0..n_accesses-1 is used.
 */
#ifndef CKC_IR_H
#define CKC_IR_H

#include <stdint.h>

#define CKC_IR_MAGIC 0x31434B43u /* "CKC1" */
#define CKC_IR_VERSION 1u

#define CKC_IR_MAX_INSTR 4096u
#define CKC_IR_MAX_CONSTS 4096u
#define CKC_IR_MAX_SCALARS 16u
#define CKC_IR_MAX_SLOTS 16u
#define CKC_IR_MAX_ACCESSES 1024u
#define CKC_IR_MAX_SITES 4096u
#define CKC_IR_MAX_LOOP_DEPTH 2u
#define CKC_IR_MAX_NEST 16u /* IF and LOOP nesting together */
/* Register pressure.  A register is live from the instruction that defines
 * it to its last use; a use inside a LOOP body that does not contain the
 * definition keeps the register live to the ENDLOOP of the outermost such
 * LOOP, and a loop counter stays live to its ENDLOOP.  At every instruction
 * that defines a register, the registers defined before it that are still
 * live after it, plus the one it defines, must number at most
 * CKC_IR_MAX_LIVE_REGS.  The rule applies to the program as written, before
 * any unused instruction is removed. */
#define CKC_IR_MAX_LIVE_REGS 32u
#define CKC_IR_NO_SITE 0xFFFFu
#define CKC_IR_NO_REG 0xFFFFu

typedef struct ckc_ir_header {
  uint32_t magic;
  uint16_t version;
  uint16_t n_instr;
  uint16_t n_consts;
  uint16_t n_scalars;
  uint16_t n_slots;
  uint16_t n_accesses;
  uint16_t n_sites;
  uint16_t n_regs;
  uint32_t slot_spaces; /* memory space of slot k in bits 2k..2k+1 (ckc_ir_space);
                           0 for slots k >= n_slots */
  uint32_t reserved[2]; /* must be zero */
} ckc_ir_header;        /* 32 bytes */

/* Memory space of an allocation slot (the CUDA memory spaces of the paper's
 * Section 6.1): global memory has one instance per input; shared memory one
 * per block of the launch; local memory one per thread.  Bounds are the same
 * for every instance (the slot's size); under the tripwire detector each
 * space is its own address window (see ckc.h, CKC_TRIPWIRE).  Only global
 * and shared slots may be read by LOAD. */
enum ckc_ir_space { CKC_SPACE_GLOBAL = 0, CKC_SPACE_SHARED = 1, CKC_SPACE_LOCAL = 2 };

typedef struct ckc_ir_instr {
  uint8_t op;   /* ckc_ir_op */
  uint8_t w;    /* 32 or 64 where the op has a width, else 0 */
  uint16_t dst; /* defined register, CKC_IR_NO_REG if none */
  uint16_t a, b, c, d;
  uint16_t s0, s1; /* site indices */
} ckc_ir_instr;    /* 16 bytes */

/* Operand use per op:
 *   CONST    dst, a = pool index            (w: 32 keeps the low 32 bits)
 *   SCALAR   dst, a = scalar index          (w as CONST)
 *   SPECIAL  dst, a = source 0..11          (w = 64)
 *   binary   dst, a, b
 *   SEXT/ZEXT/TRUNC  dst, a
 *   SELECT   dst, a = condition, b = value if true, c = value if false
 *   ACCESS   a = index reg, b = access id, c = slot, d = log2_elem (bits 0..1) | write (bit 2), s0 = site
 *   LOAD     dst, a = index reg, b = access id, c = slot, d = log2_elem (2 or 3), s0 = site
 *   STORE    dst = VALUE register (read, not defined), a = index reg, b = access id, c = slot,
 *            d = log2_elem (0..3), s0 = site
 *   FADD FSUB FMUL  dst, a, b (w = 64);  FEXP  dst, a (w = 64)
 *   ITOF     dst, a (w = 32: the operand's width);  FTOI  dst, a (w: the result's width)
 *   BARRIER  no operands; top level only
 *   IF       a = predicate, s0 = true-site, s1 = false-site
 *   LOOP     dst = counter, a = start, b = end, c = step, s0 = iteration site, s1 = exit site
 *   ELSE ENDIF ENDLOOP   no operands */
enum ckc_ir_op {
  CKC_OP_NOP = 0,
  CKC_OP_CONST = 1,
  CKC_OP_SCALAR = 2,
  CKC_OP_SPECIAL = 3,
  CKC_OP_ADD = 8,
  CKC_OP_SUB = 9,
  CKC_OP_MUL = 10,
  CKC_OP_DIVS = 11,
  CKC_OP_DIVU = 12,
  CKC_OP_REMS = 13,
  CKC_OP_REMU = 14,
  CKC_OP_AND = 15,
  CKC_OP_OR = 16,
  CKC_OP_XOR = 17,
  CKC_OP_SHL = 18,
  CKC_OP_SHRA = 19,
  CKC_OP_SHRL = 20,
  CKC_OP_MINS = 21,
  CKC_OP_MAXS = 22,
  CKC_OP_MINU = 23,
  CKC_OP_MAXU = 24,
  CKC_OP_CMPEQ = 25,
  CKC_OP_CMPNE = 26,
  CKC_OP_CMPLTS = 27,
  CKC_OP_CMPLES = 28,
  CKC_OP_CMPLTU = 29,
  CKC_OP_CMPLEU = 30,
  CKC_OP_SELECT = 31,
  CKC_OP_SEXT = 32,
  CKC_OP_ZEXT = 33,
  CKC_OP_TRUNC = 34,
  CKC_OP_FADD = 40,
  CKC_OP_FSUB = 41,
  CKC_OP_FMUL = 42,
  CKC_OP_FEXP = 43,
  CKC_OP_ITOF = 44,
  CKC_OP_FTOI = 45,
  CKC_OP_ACCESS = 48,
  CKC_OP_LOAD = 49,
  CKC_OP_STORE = 50,
  CKC_OP_IF = 56,
  CKC_OP_ELSE = 57,
  CKC_OP_ENDIF = 58,
  CKC_OP_LOOP = 59,
  CKC_OP_ENDLOOP = 60,
  CKC_OP_BARRIER = 61
};

enum ckc_special {
  CKC_SP_TID_X = 0, CKC_SP_TID_Y, CKC_SP_TID_Z,
  CKC_SP_BID_X, CKC_SP_BID_Y, CKC_SP_BID_Z,
  CKC_SP_BDIM_X, CKC_SP_BDIM_Y, CKC_SP_BDIM_Z,
  CKC_SP_GDIM_X, CKC_SP_GDIM_Y, CKC_SP_GDIM_Z
};

#endif /* CKC_IR_H */
