// loader.cpp — host-side loading of index programs: validation, pruning,
// uniformity and affine-access analysis, register allocation and lowering to
// the device form of dformat.h.  Pure host code (no HIP calls), so it is
// tested on machines without a GPU through ckc_analyze_ir().
//
// The analysis follows the paper's compile-time passes, applied to the IR:
//   * pruning keeps only what feeds an index, a branch or a loop bound
//     (AXIPrune's MathElimination, Section 5.2, Algorithm 2);
//   * an access is affine when its index is sum_d T_d * coord_d + b with
//     thread-invariant T and b (the affine-access definition of Section 5.1.1);
//     the coefficient vector reported per access is a row of the paper's T.
#include <cstdint>
#include <algorithm>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/ckc.h"
#include "dformat.h"
#include "loader.h"

namespace ckc {
namespace {

struct Ins {
  uint8_t op, w;
  uint16_t dst, a, b, c, d, s0, s1;
  int alt = -1, end = -1, depth = 0;  // IF: ELSE; IF/ELSE: ENDIF; LOOP<->ENDLOOP
  int parent = -1;                    // innermost enclosing IF/ELSE/LOOP pc
  bool live = false;
  bool store_val = false;             // STORE: its value is kept (shared memory read back)
};

bool is_binary(int op) { return op >= CKC_OP_ADD && op <= CKC_OP_CMPLEU; }
bool is_float(int op) { return op >= CKC_OP_FADD && op <= CKC_OP_FTOI; }
// The instruction defines its dst register.
bool defines_op(int op) {
  return !(op == CKC_OP_ACCESS || op == CKC_OP_STORE || op == CKC_OP_IF || op == CKC_OP_ELSE ||
           op == CKC_OP_ENDIF || op == CKC_OP_ENDLOOP || op == CKC_OP_BARRIER);
}
// Registers an instruction reads (a STORE's value only when `with_value`).
int reads(const Ins& I, uint16_t r[3], bool with_value) {
  switch (I.op) {
    case CKC_OP_CONST: case CKC_OP_SCALAR: case CKC_OP_SPECIAL: case CKC_OP_ELSE: case CKC_OP_ENDIF:
    case CKC_OP_ENDLOOP: case CKC_OP_BARRIER:
      return 0;
    case CKC_OP_SELECT: case CKC_OP_LOOP: r[0] = I.a; r[1] = I.b; r[2] = I.c; return 3;
    case CKC_OP_SEXT: case CKC_OP_ZEXT: case CKC_OP_TRUNC: case CKC_OP_ACCESS: case CKC_OP_LOAD:
    case CKC_OP_IF: case CKC_OP_FEXP: case CKC_OP_ITOF: case CKC_OP_FTOI:
      r[0] = I.a; return 1;
    case CKC_OP_STORE:
      r[0] = I.a;
      if (!with_value) return 1;
      r[1] = I.dst;
      return 2;
    default: r[0] = I.a; r[1] = I.b; return 2;  // integer and floating-point binary ops
  }
}
bool is_divrem(int op) {
  return op == CKC_OP_DIVS || op == CKC_OP_DIVU || op == CKC_OP_REMS || op == CKC_OP_REMU;
}

// Symbolic component of an affine form: zero, a known constant, a uniform IR
// register, or some other thread-invariant expression.
struct Comp {
  uint8_t kind = 0;  // 0 zero, 1 const, 2 reg, 3 expr
  int64_t v = 0;
};
struct Form {
  bool affine = false;
  int k = 0;  // valid modulo 2^k (0 = exact integer)
  Comp c[7];
};

int64_t wrapw(int64_t v, int w) { return w == 32 ? (int64_t)(int32_t)(uint32_t)(uint64_t)v : v; }

Comp cadd(Comp x, Comp y, int w) {
  if (x.kind == 0) return y;
  if (y.kind == 0) return x;
  if (x.kind == 1 && y.kind == 1) return Comp{1, wrapw((int64_t)((uint64_t)x.v + (uint64_t)y.v), w)};
  return Comp{3, 0};
}
Comp cneg(Comp x, int w) {
  if (x.kind == 0) return x;
  if (x.kind == 1) return Comp{1, wrapw((int64_t)(0 - (uint64_t)x.v), w)};
  return Comp{3, 0};
}
Comp cmul(Comp x, Comp u, int w) {  // u: the uniform factor
  if (x.kind == 0 || u.kind == 0) return Comp{};
  if (x.kind == 1 && x.v == 1) return u;
  if (u.kind == 1 && u.v == 1) return x;
  if (x.kind == 1 && u.kind == 1) return Comp{1, wrapw((int64_t)((uint64_t)x.v * (uint64_t)u.v), w)};
  return Comp{3, 0};
}

struct Analyzer {
  std::string err;
  const uint8_t* ir = nullptr;
  size_t n = 0;
  int n_instr = 0, n_consts = 0, n_scalars = 0, n_slots = 0, n_accesses = 0, n_sites = 0,
      n_regs = 0;
  uint32_t slot_spaces = 0;
  std::vector<int64_t> consts;
  std::vector<uint16_t> site_ids;
  std::vector<Ins> ins;
  std::vector<int> def_pc;      // per virtual register
  std::vector<char> uni;        // uniform register
  std::vector<char> ctrl_var;   // per pc: under thread-dependent control
  std::vector<Form> form;
  std::vector<char> indirect;
  int max_depth = 0;
  bool no_prune = false;     // keep every instruction (the unpruned program)
  bool has_barrier = false;  // some BARRIER
  uint32_t shared_idx = 0;   // shared slots some LOAD of which feeds the slice
  uint32_t shared_live = 0;  // shared slots read back into the pruned program

  uint32_t space_of(int slot) const { return slot < 16 ? (slot_spaces >> (2 * slot)) & 3u : 0u; }

  bool fail(int pc, const char* what) {
    err = pc >= 0 ? ("instruction " + std::to_string(pc) + ": " + what) : std::string(what);
    return false;
  }

  static uint16_t rd16(const uint8_t* p) { return (uint16_t)(p[0] | (p[1] << 8)); }

  bool decode() {
    if (!ir || n < sizeof(ckc_ir_header)) return fail(-1, "IR shorter than its header");
    ckc_ir_header h;
    std::memcpy(&h, ir, sizeof h);
    if (h.magic != CKC_IR_MAGIC) return fail(-1, "bad magic");
    if (h.version != CKC_IR_VERSION) return fail(-1, "unsupported IR version");
    if (h.reserved[0] || h.reserved[1]) return fail(-1, "reserved header bytes not zero");
    n_instr = h.n_instr; n_consts = h.n_consts; n_scalars = h.n_scalars; n_slots = h.n_slots;
    n_accesses = h.n_accesses; n_sites = h.n_sites; n_regs = h.n_regs;
    slot_spaces = h.slot_spaces;
    for (int k = 0; k < 16; k++) {
      const uint32_t sp = (slot_spaces >> (2 * k)) & 3u;
      if (sp > CKC_SPACE_LOCAL || (k >= n_slots && k < 16 && sp != 0))
        return fail(-1, "bad memory space of an allocation slot");
    }
    if (n_instr > (int)CKC_IR_MAX_INSTR || n_consts > (int)CKC_IR_MAX_CONSTS ||
        n_scalars > (int)CKC_IR_MAX_SCALARS || n_slots > (int)CKC_IR_MAX_SLOTS ||
        n_accesses > (int)CKC_IR_MAX_ACCESSES || n_sites > (int)CKC_IR_MAX_SITES)
      return fail(-1, "header count above the supported limit");
    size_t site_bytes = ((size_t)n_sites * 2 + 7) / 8 * 8;
    size_t need = sizeof(ckc_ir_header) + (size_t)n_consts * 8 + site_bytes + (size_t)n_instr * 16;
    if (need != n) return fail(-1, "byte count does not match the header");
    const uint8_t* p = ir + sizeof(ckc_ir_header);
    consts.resize(n_consts);
    for (int i = 0; i < n_consts; i++) std::memcpy(&consts[i], p + 8 * i, 8);
    p += 8 * (size_t)n_consts;
    site_ids.resize(n_sites);
    for (int i = 0; i < n_sites; i++) site_ids[i] = rd16(p + 2 * i);
    p += site_bytes;
    ins.resize(n_instr);
    for (int i = 0; i < n_instr; i++) {
      const uint8_t* q = p + 16 * (size_t)i;
      Ins& I = ins[i];
      I.op = q[0]; I.w = q[1];
      I.dst = rd16(q + 2); I.a = rd16(q + 4); I.b = rd16(q + 6); I.c = rd16(q + 8);
      I.d = rd16(q + 10); I.s0 = rd16(q + 12); I.s1 = rd16(q + 14);
    }
    return true;
  }

  // Structure, SSA and scoping rules of ckc_ir.h.
  bool validate() {
    std::vector<char> id_seen(65536, 0), site_used(n_sites, 0), acc_used(n_accesses, 0);
    for (int i = 0; i < n_sites; i++) {
      if (id_seen[site_ids[i]]) return fail(-1, "duplicate coverage-map id");
      id_seen[site_ids[i]] = 1;
    }
    def_pc.assign(n_regs, -1);
    std::vector<int> def_scope(n_regs, -1);
    std::vector<char> scope_open(1, 1);
    std::vector<int> scope_stack{0}, ctl;
    int loop_depth = 0;
    auto use = [&](int pc, unsigned r) {
      if ((int)r >= n_regs || def_scope[r] < 0 || !scope_open[def_scope[r]])
        return fail(pc, "register used before definition or outside its scope");
      return true;
    };
    auto def = [&](int pc, unsigned r) {
      if ((int)r >= n_regs || def_scope[r] != -1) return fail(pc, "register defined twice or out of range");
      def_scope[r] = scope_stack.back();
      def_pc[r] = pc;
      return true;
    };
    auto site = [&](int pc, unsigned s) {
      if (s == CKC_IR_NO_SITE) return true;
      if ((int)s >= n_sites || site_used[s]) return fail(pc, "site index out of range or reused");
      site_used[s] = 1;
      return true;
    };
    auto width = [&](int pc, int w) { return (w == 32 || w == 64) ? true : fail(pc, "width must be 32 or 64"); };
    auto open_scope = [&]() {
      scope_open.push_back(1);
      scope_stack.push_back((int)scope_open.size() - 1);
    };
    auto close_scope = [&]() {
      scope_open[scope_stack.back()] = 0;
      scope_stack.pop_back();
    };
    for (int i = 0; i < n_instr; i++) {
      Ins& I = ins[i];
      I.depth = loop_depth;
      I.parent = ctl.empty() ? -1 : ctl.back();
      switch (I.op) {
        case CKC_OP_CONST:
          if (!width(i, I.w)) return false;
          if (I.a >= n_consts) return fail(i, "constant index out of range");
          if (!def(i, I.dst)) return false;
          break;
        case CKC_OP_SCALAR:
          if (!width(i, I.w)) return false;
          if (I.a >= n_scalars) return fail(i, "scalar index out of range");
          if (!def(i, I.dst)) return false;
          break;
        case CKC_OP_SPECIAL:
          if (I.a > 11) return fail(i, "unknown special source");
          if (!def(i, I.dst)) return false;
          break;
        case CKC_OP_SELECT:
          if (!width(i, I.w) || !use(i, I.a) || !use(i, I.b) || !use(i, I.c) || !def(i, I.dst)) return false;
          break;
        case CKC_OP_SEXT: case CKC_OP_ZEXT: case CKC_OP_TRUNC:
          if (!use(i, I.a) || !def(i, I.dst)) return false;
          break;
        case CKC_OP_ACCESS:
        case CKC_OP_STORE:
        case CKC_OP_LOAD:
          if (!width(i, I.w) || !use(i, I.a)) return false;
          if (I.op == CKC_OP_STORE && !use(i, I.dst)) return false;
          if (I.b >= n_accesses || acc_used[I.b]) return fail(i, "access id out of range or reused");
          acc_used[I.b] = 1;
          if (I.c >= n_slots) return fail(i, "allocation slot out of range");
          if (I.op == CKC_OP_ACCESS) {
            if (I.d > 7) return fail(i, "bad ACCESS flags");
          } else if (I.op == CKC_OP_STORE) {
            if (I.d > 3) return fail(i, "bad STORE element size");
          } else {
            if (I.d != 2 && I.d != 3) return fail(i, "LOAD element must be 4 or 8 bytes");
            if (space_of(I.c) == CKC_SPACE_LOCAL) return fail(i, "LOAD reads global or shared slots only");
            if (space_of(I.c) == CKC_SPACE_SHARED && I.d != 2) return fail(i, "shared LOAD element must be 4 bytes");
            if (!def(i, I.dst)) return false;
          }
          if (!site(i, I.s0)) return false;
          break;
        case CKC_OP_FADD: case CKC_OP_FSUB: case CKC_OP_FMUL:
          if (I.w != 64) return fail(i, "floating-point operations have width 64");
          if (!use(i, I.a) || !use(i, I.b) || !def(i, I.dst)) return false;
          break;
        case CKC_OP_FEXP:
          if (I.w != 64) return fail(i, "floating-point operations have width 64");
          if (!use(i, I.a) || !def(i, I.dst)) return false;
          break;
        case CKC_OP_ITOF:
          if (I.w != 32) return fail(i, "ITOF converts a width-32 value");
          if (!use(i, I.a) || !def(i, I.dst)) return false;
          break;
        case CKC_OP_FTOI:
          if (!width(i, I.w) || !use(i, I.a) || !def(i, I.dst)) return false;
          break;
        case CKC_OP_BARRIER:
          if (!ctl.empty()) return fail(i, "BARRIER inside IF or LOOP");
          has_barrier = true;
          break;
        case CKC_OP_IF:
          if (!use(i, I.a) || !site(i, I.s0) || !site(i, I.s1)) return false;
          if (ctl.size() >= CKC_IR_MAX_NEST) return fail(i, "nesting deeper than 16");
          ctl.push_back(i);
          open_scope();
          break;
        case CKC_OP_ELSE:
          if (ctl.empty() || ins[ctl.back()].op != CKC_OP_IF || ins[ctl.back()].alt >= 0)
            return fail(i, "ELSE without an open IF");
          ins[ctl.back()].alt = i;
          I.parent = ctl.back();
          close_scope();
          open_scope();
          ctl.back() = i;  // else-arm instructions hang off the ELSE
          break;
        case CKC_OP_ENDIF: {
          if (ctl.empty() || (ins[ctl.back()].op != CKC_OP_IF && ins[ctl.back()].op != CKC_OP_ELSE))
            return fail(i, "ENDIF without an open IF");
          int t = ctl.back();
          ctl.pop_back();
          int f = ins[t].op == CKC_OP_ELSE ? ins[t].parent : t;
          ins[f].end = i;
          if (ins[f].alt >= 0) ins[ins[f].alt].end = i;
          I.parent = f;
          close_scope();
          break;
        }
        case CKC_OP_LOOP:
          if (!width(i, I.w) || !use(i, I.a) || !use(i, I.b) || !use(i, I.c)) return false;
          if (!site(i, I.s0) || !site(i, I.s1)) return false;
          if (ctl.size() >= CKC_IR_MAX_NEST) return fail(i, "nesting deeper than 16");
          if (loop_depth >= (int)CKC_IR_MAX_LOOP_DEPTH) return fail(i, "loops nested deeper than 2");
          ctl.push_back(i);
          loop_depth++;
          if (loop_depth > max_depth) max_depth = loop_depth;
          open_scope();
          if (!def(i, I.dst)) return false;
          break;
        case CKC_OP_ENDLOOP: {
          if (ctl.empty() || ins[ctl.back()].op != CKC_OP_LOOP) return fail(i, "ENDLOOP without an open LOOP");
          int f = ctl.back();
          ctl.pop_back();
          ins[f].end = i;
          I.end = f;
          I.parent = f;
          loop_depth--;
          close_scope();
          break;
        }
        default:
          if (!is_binary(I.op)) return fail(i, "unknown opcode");
          if (!width(i, I.w) || !use(i, I.a) || !use(i, I.b) || !def(i, I.dst)) return false;
          break;
      }
    }
    if (!ctl.empty()) return fail(-1, "unclosed IF or LOOP");
    for (int a = 0; a < n_accesses; a++)
      if (!acc_used[a]) return fail(-1, "an access id is never used");
    return pressure_ok();
  }

  // The live-register rule of ckc_ir.h (CKC_IR_MAX_LIVE_REGS) over the program
  // as written.  Pruning only shortens live ranges, so the allocation of the
  // pruned program then needs at most as many registers.
  bool pressure_ok() {
    std::vector<int> end(n_regs, -1);
    auto touch = [&](int r, int pc) {
      if (r >= n_regs) return;
      int e = pc;
      for (int p = ins[pc].parent; p >= 0; p = ins[p].parent)
        if (ins[p].op == CKC_OP_LOOP && def_pc[r] < p) e = std::max(e, ins[p].end);
      end[r] = std::max(end[r], e);
    };
    for (int i = 0; i < n_instr; i++) {
      const Ins& I = ins[i];
      uint16_t rr[3];
      const int nr = reads(I, rr, true);
      for (int q = 0; q < nr; q++) touch(rr[q], i);
      if (I.op == CKC_OP_LOOP) end[I.dst] = std::max(end[I.dst], I.end);
    }
    // live after instruction i: registers r with def_pc[r] < i < end[r]
    std::vector<int> diff(n_instr + 2, 0);
    for (int r = 0; r < n_regs; r++)
      if (def_pc[r] >= 0 && end[r] > def_pc[r]) {
        diff[def_pc[r] + 1]++;
        diff[end[r]]--;
      }
    int cur = 0;
    for (int i = 0; i < n_instr; i++) {
      cur += diff[i];
      const Ins& I = ins[i];
      if (defines_op(I.op) && cur + 1 > (int)CKC_IR_MAX_LIVE_REGS)
        return fail(i, "more than CKC_IR_MAX_LIVE_REGS (32) registers live");
    }
    return true;
  }

  // Pruning, the paper's AXIPrune (Algorithm 2).  slice_pass walks
  // backwards (every definition precedes its uses) from the accesses, IF
  // predicates and loop bounds and, with `divs`, the divisions (they count
  // arithmetic faults, so their operands stay exact), marking every
  // instruction whose result a marked one reads; a STORE's value is read
  // when its slot is in xs.  It returns the shared slots some LOAD of which
  // has its result needed.  The fixpoint over xs (the set only grows) gives
  // without divisions the index-related shared variables and the slice, whose
  // wraps at the vertex threads clear the vertex-exact flag; with divisions
  // the shared slots read back into the pruned program.  MathElimination keeps
  // only that live set and the control structure; BarrierElimination removes
  // every BARRIER unless some shared slot is read back (all or none, as the
  // algorithm is written).  With no_prune everything is kept.
  std::vector<char> slice;
  uint32_t slice_pass(uint32_t xs, bool divs, std::vector<char>& need, std::vector<char>& mark) const {
    std::fill(need.begin(), need.end(), 0);
    mark.assign(n_instr, 0);
    for (int i = n_instr - 1; i >= 0; i--) {
      const Ins& I = ins[i];
      const bool root = I.op == CKC_OP_ACCESS || I.op == CKC_OP_LOAD || I.op == CKC_OP_STORE ||
                        I.op == CKC_OP_IF || I.op == CKC_OP_LOOP || (divs && is_divrem(I.op));
      if (!(root || (defines_op(I.op) && I.op != CKC_OP_LOOP && I.dst < n_regs && need[I.dst]))) continue;
      mark[i] = 1;
      uint16_t rr[3];
      const int nr = reads(I, rr, I.op == CKC_OP_STORE && ((xs >> I.c) & 1u));
      for (int q = 0; q < nr; q++)
        if (rr[q] < n_regs) need[rr[q]] = 1;
    }
    uint32_t nxs = 0;
    for (int i = 0; i < n_instr; i++) {
      const Ins& I = ins[i];
      if (I.op == CKC_OP_LOAD && space_of(I.c) == CKC_SPACE_SHARED && need[I.dst]) nxs |= 1u << I.c;
    }
    return nxs;
  }
  uint32_t slice_fixpoint(bool divs, std::vector<char>& mark) const {
    std::vector<char> need(n_regs, 0);
    uint32_t xs = 0;
    for (;;) {
      const uint32_t nxs = slice_pass(xs, divs, need, mark);
      if (nxs == xs) return xs;
      xs = nxs;
    }
  }
  bool prune() {
    shared_idx = slice_fixpoint(false, slice);
    std::vector<char> live;
    shared_live = slice_fixpoint(true, live);
    for (int i = 0; i < n_instr; i++) {
      Ins& I = ins[i];
      const bool structure = I.op == CKC_OP_ELSE || I.op == CKC_OP_ENDIF || I.op == CKC_OP_ENDLOOP;
      I.live = no_prune || live[i] || structure || (I.op == CKC_OP_BARRIER && shared_live != 0);
      I.store_val = I.op == CKC_OP_STORE && (no_prune || ((shared_live >> I.c) & 1u));
    }
    return true;
  }

  // The program needs its blocks run together (shared memory read back, or
  // barriers executed).
  bool blockwise() const {
    for (int i = 0; i < n_instr; i++) {
      const Ins& I = ins[i];
      if (!I.live) continue;
      if (I.op == CKC_OP_BARRIER) return true;
      // a shared LOAD whose result nothing kept reads may return anything
      if (I.op == CKC_OP_LOAD && space_of(I.c) == CKC_SPACE_SHARED && (no_prune || ((shared_live >> I.c) & 1u)))
        return true;
    }
    return false;
  }

  // The whole-thread part of a program whose expanded loop has a gather body
  // (everything outside that body) runs without instruction dispatch, in the
  // rows form, when the device's symbolic walk (build_rows) reduces it to
  // affine forms: every value a constant, an affine form of the thread
  // coordinates or of one loaded value (at most 4 loads), exact at the width
  // it is used at; IF regions without ELSE, not nested, whose predicate is a
  // comparison just before or a value; the loop's bounds forms, its step and
  // live-ins uniform; at most 16 entries.  The walk's decisions depend only on
  // kinds and widths, not on values, so they are replayed here: a program
  // flagged PF_ROWS always passes the walk.  *w32 (when given): every entry
  // the walk makes, ENDIF's aside, is 32 bits wide.
  bool rows_form(bool* w32 = nullptr) const {
    if (expand_pc < 0 || !body_gather || blockwise()) return false;
    const int body_end = ins[expand_pc].end;
    enum { UNI = 0, COORD = 1, PRED = 2, LOAD0 = 3 };  // LOAD0 + k: the k-th load
    std::vector<int> kind(n_regs, UNI), wd(n_regs, 64);
    auto fits = [&](int r, int w) { return kind[r] == UNI || (kind[r] != PRED && wd[r] >= w); };
    int n = 0, n_load = 0, preg = -1, open_if = 0, pw = 64;
    bool all32 = true;
    for (int i = 0; i < n_instr; i++) {
      const Ins& I = ins[i];
      if (!I.live || (i > expand_pc && i < body_end)) continue;
      const int op = I.op, w = I.w;
      switch (op) {
        case CKC_OP_CONST: case CKC_OP_SCALAR: kind[I.dst] = UNI; wd[I.dst] = 64; break;
        case CKC_OP_SPECIAL: kind[I.dst] = I.a < 6 ? COORD : UNI; wd[I.dst] = 64; break;
        case CKC_OP_ADD: case CKC_OP_SUB: case CKC_OP_MUL: case CKC_OP_SHL: {
          const int ka = kind[I.a], kb = kind[I.b];
          if (!fits(I.a, w) || !fits(I.b, w)) return false;
          if (op == CKC_OP_SHL && kb != UNI) return false;
          if (op == CKC_OP_MUL && ka != UNI && kb != UNI) return false;
          if ((op == CKC_OP_ADD || op == CKC_OP_SUB) && ka != UNI && kb != UNI && ka != kb) return false;
          kind[I.dst] = ka != UNI ? ka : kb;
          wd[I.dst] = kind[I.dst] == UNI ? 64 : w;
          break;
        }
        case CKC_OP_TRUNC:
          if (!fits(I.a, 32)) return false;
          kind[I.dst] = kind[I.a];
          wd[I.dst] = kind[I.dst] == UNI ? 64 : 32;
          break;
        case CKC_OP_SEXT: case CKC_OP_ZEXT:
          if (kind[I.a] != UNI) return false;
          kind[I.dst] = UNI; wd[I.dst] = 64;
          break;
        case CKC_OP_SELECT:
          if (kind[I.a] != UNI || kind[I.b] != UNI || kind[I.c] != UNI) return false;
          kind[I.dst] = UNI; wd[I.dst] = 64;
          break;
        case CKC_OP_ACCESS: case CKC_OP_STORE: case CKC_OP_LOAD:
          if (op == CKC_OP_STORE && I.store_val) return false;
          if (op == CKC_OP_LOAD && (space_of(I.c) != CKC_SPACE_GLOBAL || n_load >= 4)) return false;
          if (n >= 16 || !fits(I.a, w)) return false;
          n++;
          all32 &= w == 32;
          if (op == CKC_OP_LOAD) { kind[I.dst] = LOAD0 + n_load++; wd[I.dst] = 64; }
          break;
        case CKC_OP_IF:
          if (open_if++ || n >= 16 || (kind[I.a] == PRED && I.a != preg)) return false;
          n++;
          // a comparison's guard has its width; a value's tests the width its form is exact at
          all32 &= (kind[I.a] == PRED ? pw : kind[I.a] == UNI ? 64 : wd[I.a]) == 32;
          break;
        case CKC_OP_ENDIF:
          open_if--;
          if (n >= 16) return false;
          n++;
          break;
        case CKC_OP_LOOP:
          if (i != expand_pc || n >= 16 || !fits(I.a, w) || !fits(I.b, w) || kind[I.c] != UNI) return false;
          for (int r : livein)
            if (kind[r] != UNI) return false;
          n++;
          all32 &= w == 32;
          i = body_end;  // continue after ENDLOOP
          break;
        default:
          if (op >= CKC_OP_CMPEQ && op <= CKC_OP_CMPLEU && (kind[I.a] != UNI || kind[I.b] != UNI)) {
            if (!fits(I.a, w) || !fits(I.b, w)) return false;
            kind[I.dst] = PRED;
            preg = I.dst;
            pw = w;
            break;
          }
          if (op < CKC_OP_ADD || op > CKC_OP_CMPLEU || is_divrem(op)) return false;
          if (kind[I.a] != UNI || kind[I.b] != UNI) return false;
          kind[I.dst] = UNI; wd[I.dst] = 64;
          break;
      }
    }
    if (w32) *w32 = all32;
    return true;
  }

  bool reg_used(int r) const {
    for (int i = def_pc[r] + 1; i < n_instr; i++) {
      const Ins& I = ins[i];
      if (!I.live) continue;
      uint16_t rr[3];
      const int nr = reads(I, rr, I.store_val);
      for (int q = 0; q < nr; q++)
        if (rr[q] == r) return true;
    }
    return false;
  }

  // Uniformity (thread-invariance) of values and control, and the affine
  // form of every value over (tid.xyz, bid.xyz).
  void classify() {
    uni.assign(n_regs, 0);
    indirect.assign(n_regs, 0);
    form.assign(n_regs, Form{});
    ctrl_var.assign(n_instr, 0);
    std::vector<char> cvar_stack{0};
    auto uform = [&](int r, int pc) {  // form of a uniform register
      Form f;
      f.affine = true;
      f.k = 0;
      const Ins& I = ins[pc];
      if (I.op == CKC_OP_CONST) f.c[6] = Comp{1, wrapw(consts[I.a], I.w)};
      else if (I.op == CKC_OP_SCALAR || I.op == CKC_OP_SPECIAL) f.c[6] = Comp{2, r};
      else f.c[6] = Comp{3, 0};
      return f;
    };
    auto usable = [&](int r, int w) {
      const Form& f = form[r];
      return f.affine && (uni[r] || f.k == 0 || f.k >= w);
    };
    for (int i = 0; i < n_instr; i++) {
      Ins& I = ins[i];
      // control context of this instruction
      ctrl_var[i] = cvar_stack.back();
      if (I.op == CKC_OP_ELSE || I.op == CKC_OP_ENDIF || I.op == CKC_OP_ENDLOOP) {
        cvar_stack.pop_back();
        if (I.op == CKC_OP_ELSE) cvar_stack.push_back(cvar_stack.back() || !uni[ins[I.parent].a]);
        ctrl_var[i] = cvar_stack.back();
        continue;
      }
      if (I.op == CKC_OP_IF) {
        cvar_stack.push_back(cvar_stack.back() || !uni[I.a]);
        continue;
      }
      if (I.op == CKC_OP_STORE || I.op == CKC_OP_BARRIER) continue;
      int r = I.dst;
      switch (I.op) {
        case CKC_OP_CONST: case CKC_OP_SCALAR:
          uni[r] = 1; form[r] = uform(r, i);
          break;
        case CKC_OP_SPECIAL:
          if (I.a >= 6) { uni[r] = 1; form[r] = uform(r, i); }
          else {
            Form f; f.affine = true; f.k = 0; f.c[I.a] = Comp{1, 1};
            form[r] = f;
          }
          break;
        case CKC_OP_LOAD:
          // shared memory differs from block to block and phase to phase
          uni[r] = uni[I.a] && space_of(I.c) != CKC_SPACE_SHARED;
          if (uni[r]) form[r] = uform(r, i);
          else indirect[r] = 1;
          break;
        case CKC_OP_FADD: case CKC_OP_FSUB: case CKC_OP_FMUL: case CKC_OP_FEXP: case CKC_OP_ITOF:
        case CKC_OP_FTOI: {
          const bool unary = I.op == CKC_OP_FEXP || I.op == CKC_OP_ITOF || I.op == CKC_OP_FTOI;
          uni[r] = uni[I.a] && (unary || uni[I.b]);
          indirect[r] = indirect[I.a] || (!unary && indirect[I.b]);
          form[r] = Form{};  // never affine (not modular integer arithmetic)
          break;
        }
        case CKC_OP_LOOP: {
          bool u = uni[I.a] && uni[I.b] && uni[I.c];
          uni[r] = u;
          if (u) form[r] = uform(r, i);
          cvar_stack.push_back(cvar_stack.back() || !u);
          break;
        }
        case CKC_OP_ACCESS:
          break;
        default: {
          bool u = uni[I.a] && (I.op == CKC_OP_SEXT || I.op == CKC_OP_ZEXT || I.op == CKC_OP_TRUNC ||
                                (uni[I.b] && (I.op != CKC_OP_SELECT || uni[I.c])));
          uni[r] = u;
          indirect[r] = indirect[I.a] || (I.op != CKC_OP_SEXT && I.op != CKC_OP_ZEXT &&
                                          I.op != CKC_OP_TRUNC && indirect[I.b]) ||
                        (I.op == CKC_OP_SELECT && indirect[I.c]);
          if (u) { form[r] = uform(r, i); break; }
          Form f;
          int w = I.w;
          if ((I.op == CKC_OP_ADD || I.op == CKC_OP_SUB) && usable(I.a, w) && usable(I.b, w)) {
            f.affine = true; f.k = w;
            for (int d = 0; d < 7; d++)
              f.c[d] = cadd(form[I.a].c[d], I.op == CKC_OP_SUB ? cneg(form[I.b].c[d], w) : form[I.b].c[d], w);
          } else if ((I.op == CKC_OP_MUL || I.op == CKC_OP_SHL) && usable(I.a, w) && usable(I.b, w) &&
                     (uni[I.a] || uni[I.b])) {
            int v = uni[I.b] ? I.a : I.b, u2 = uni[I.b] ? I.b : I.a;
            if (I.op == CKC_OP_SHL && !uni[I.b]) { form[r] = f; break; }  // varying shift amount
            Comp factor = form[u2].c[6];
            if (I.op == CKC_OP_SHL)
              factor = factor.kind == 1 ? Comp{1, wrapw((int64_t)(1ull << ((uint64_t)factor.v & (w - 1))), w)}
                                        : Comp{3, 0};
            f.affine = true; f.k = w;
            for (int d = 0; d < 7; d++) f.c[d] = cmul(form[v].c[d], factor, w);
          } else if (I.op == CKC_OP_TRUNC && form[I.a].affine) {
            f = form[I.a];
            f.k = 32;
          }
          form[r] = f;
        }
      }
    }
  }

  // ------------------------------------------------------------------------
  // register allocation (linear scan over live values)
  std::vector<int> phys;  // per virtual register, -1 if none
  int n_phys = 0;

  bool allocate() {
    std::vector<int> last(n_regs, -1);
    auto touch = [&](int r, int pc) {
      if (r >= n_regs) return;
      // a use inside loops that do not contain the definition keeps the value
      // alive to the end of the outermost such loop
      int end = pc;
      for (int p = ins[pc].parent; p >= 0; p = ins[p].parent) {
        const Ins& P = ins[p];
        if (P.op == CKC_OP_LOOP && def_pc[r] < p) end = std::max(end, P.end);
      }
      last[r] = std::max(last[r], end);
    };
    for (int i = 0; i < n_instr; i++) {
      const Ins& I = ins[i];
      if (!I.live) continue;
      uint16_t rr[3];
      const int nr = reads(I, rr, I.store_val);
      for (int q = 0; q < nr; q++) touch(rr[q], i);
    }
    // a loop counter lives through its whole body
    for (int i = 0; i < n_instr; i++)
      if (ins[i].live && ins[i].op == CKC_OP_LOOP) last[ins[i].dst] = std::max(last[ins[i].dst], ins[i].end);
    phys.assign(n_regs, -1);
    std::vector<int> busy_until(NREG, -1);
    for (int i = 0; i < n_instr; i++) {
      const Ins& I = ins[i];
      if (!I.live) continue;
      if (!defines_op(I.op) || I.dst >= n_regs) continue;
      int r = I.dst;
      int end = last[r] < 0 ? i : last[r];
      int got = -1;
      for (int p = 0; p < NREG; p++)
        if (busy_until[p] < i) { got = p; break; }
      // operands whose interval ends exactly here may share the register
      if (got < 0) {
        for (int p = 0; p < NREG; p++)
          if (busy_until[p] == i) { got = p; break; }
      }
      if (got < 0) return fail(i, "program needs more than 32 live registers");
      phys[r] = got;
      busy_until[got] = end;
      n_phys = std::max(n_phys, got + 1);
    }
    return true;
  }

  // ------------------------------------------------------------------------
  // lowering
  int expand_pc = -1;
  std::vector<int> livein;

  bool body_has_loop(int lp) const {
    for (int i = lp + 1; i < ins[lp].end; i++)
      if (ins[i].live && ins[i].op == CKC_OP_LOOP) return true;
    return false;
  }

  void choose_expansion(bool uniform_prog) {
    if (uniform_prog || blockwise()) return;  // a blockwise program's threads stay in their block
    for (int i = 0; i < n_instr; i++) {
      const Ins& I = ins[i];
      if (!I.live || I.op != CKC_OP_LOOP || I.depth != 0) continue;
      if (uni[I.dst]) continue;  // uniform trip count: nothing to balance
      if (body_has_loop(i)) continue;
      // registers read by the body and defined before the loop
      std::vector<int> li;
      for (int j = i + 1; j < I.end; j++) {
        const Ins& J = ins[j];
        if (!J.live) continue;
        uint16_t ops[3] = {CKC_IR_NO_REG, CKC_IR_NO_REG, CKC_IR_NO_REG};
        reads(J, ops, J.store_val);
        for (uint16_t r : ops) {
          if (r >= n_regs || r == I.dst || def_pc[r] >= i) continue;
          int p = phys[r];
          bool have = false;
          for (int q : li) have |= q == p;
          if (!have) li.push_back(p);
        }
      }
      if ((int)li.size() > MAX_LIVEIN) continue;
      expand_pc = i;
      livein = li;
      return;
    }
  }

  // The expanded body as a gather: straight-line code whose live-ins are
  // uniform and whose every varying value is affine in one variable (the loop
  // counter or one loaded value) with uniform coefficients, valid modulo 2^w
  // for each access of width w that uses it.  Such a body is evaluated from a
  // per-input list of (coefficient, offset, variable) entries instead of being
  // interpreted.
  bool body_gather = false;

  void check_gather() {
    if (expand_pc < 0) return;
    const Ins& L = ins[expand_pc];
    std::vector<int> var(n_regs, -1), valid(n_regs, 64);
    var[L.dst] = 0;
    int n_load = 0, n_ent = 0;
    auto operand_ok = [&](int r) {  // live-ins must be uniform
      if (r >= n_regs) return true;
      if (def_pc[r] < expand_pc && r != L.dst) return (bool)uni[r];
      return true;
    };
    auto v_of = [&](int r) { return r < n_regs ? var[r] : -1; };
    auto k_of = [&](int r) { return r < n_regs ? valid[r] : 64; };
    for (int i = expand_pc + 1; i < L.end; i++) {
      const Ins& I = ins[i];
      if (!I.live) continue;
      const int op = I.op, w = I.w;
      switch (op) {
        case CKC_OP_CONST: case CKC_OP_SCALAR: var[I.dst] = -1; break;
        case CKC_OP_SPECIAL:
          if (I.a < 6) return;  // thread coordinates: keep the interpreter
          var[I.dst] = -1;
          break;
        case CKC_OP_STORE:
          if (I.store_val) return;  // a value written back: keep the interpreter
          [[fallthrough]];
        case CKC_OP_ACCESS: case CKC_OP_LOAD: {
          if (!operand_ok(I.a)) return;
          if (v_of(I.a) >= 0 && k_of(I.a) < w) return;
          if (++n_ent > 32) return;
          if (op == CKC_OP_LOAD) {
            if (++n_load > 7) return;
            var[I.dst] = n_load;
            valid[I.dst] = 64;
          }
          break;
        }
        case CKC_OP_SEXT: case CKC_OP_ZEXT: case CKC_OP_TRUNC:
          if (!operand_ok(I.a) || v_of(I.a) >= 0) return;
          var[I.dst] = -1;
          break;
        case CKC_OP_SELECT:
          if (!operand_ok(I.a) || !operand_ok(I.b) || !operand_ok(I.c)) return;
          if (v_of(I.a) >= 0 || v_of(I.b) >= 0 || v_of(I.c) >= 0) return;
          var[I.dst] = -1;
          break;
        default: {
          if (!is_binary(op)) return;  // control flow inside the body
          if (!operand_ok(I.a) || !operand_ok(I.b)) return;
          const int va = v_of(I.a), vb = v_of(I.b);
          if (va < 0 && vb < 0) { var[I.dst] = -1; break; }
          int v, k;
          if (op == CKC_OP_ADD || op == CKC_OP_SUB) {
            if (va >= 0 && vb >= 0 && va != vb) return;
            v = va >= 0 ? va : vb;
            k = std::min({va >= 0 ? k_of(I.a) : 64, vb >= 0 ? k_of(I.b) : 64, w});
          } else if (op == CKC_OP_MUL) {
            if (va >= 0 && vb >= 0) return;
            v = va >= 0 ? va : vb;
            k = std::min(va >= 0 ? k_of(I.a) : k_of(I.b), w);
          } else if (op == CKC_OP_SHL) {
            if (vb >= 0) return;
            v = va;
            k = std::min(k_of(I.a), w);
          } else {
            return;
          }
          var[I.dst] = v;
          valid[I.dst] = k;
          break;
        }
      }
    }
    body_gather = true;
  }

  std::vector<uint8_t> lower(uint32_t cls, uint32_t trace_cap, int* n_live_out) {
    std::vector<int> newpc(n_instr, -1);
    int m = 0;
    for (int i = 0; i < n_instr; i++)
      if (ins[i].live) newpc[i] = m++;
    *n_live_out = m;
    std::vector<int> cmap(n_consts, -1);
    std::vector<int64_t> dconsts;
    std::vector<dins> out(m);
    std::vector<daccess> acc(n_accesses);
    int n_internal = 0;
    // IFs enclosing the expanded loop are never skipped
    std::vector<char> noskip(n_instr, 0);
    if (expand_pc >= 0)
      for (int p = ins[expand_pc].parent; p >= 0; p = ins[p].parent) {
        noskip[p] = 1;
        if (ins[p].op == CKC_OP_ELSE) noskip[ins[p].parent] = 1;
      }
    for (int i = 0; i < n_instr; i++) {
      const Ins& I = ins[i];
      if (!I.live) continue;
      dins D;
      std::memset(&D, 0, sizeof D);
      D.op = I.op;
      D.w = I.w;
      D.s0 = I.s0; D.s1 = I.s1;
      if ((I.op == CKC_OP_ACCESS || I.op == CKC_OP_LOAD || I.op == CKC_OP_STORE) && I.s0 == CKC_IR_NO_SITE)
        D.s0 = (uint16_t)(n_sites + n_internal++);  // internal site: counted, never mapped
      auto P = [&](uint16_t r) -> uint8_t { return r < n_regs && phys[r] >= 0 ? (uint8_t)phys[r] : 0; };
      switch (I.op) {
        case CKC_OP_CONST: {
          if (cmap[I.a] < 0) { cmap[I.a] = (int)dconsts.size(); dconsts.push_back(consts[I.a]); }
          D.dst = P(I.dst); D.x = (uint16_t)cmap[I.a];
          break;
        }
        case CKC_OP_SCALAR: case CKC_OP_SPECIAL: D.dst = P(I.dst); D.x = I.a; D.w = I.op == CKC_OP_SPECIAL ? 64 : I.w; break;
        case CKC_OP_SELECT: D.dst = P(I.dst); D.a = P(I.a); D.b = P(I.b); D.c = P(I.c); break;
        case CKC_OP_SEXT: case CKC_OP_ZEXT: case CKC_OP_TRUNC: D.dst = P(I.dst); D.a = P(I.a); break;
        case CKC_OP_ACCESS: case CKC_OP_LOAD: case CKC_OP_STORE: {
          D.a = P(I.a); D.slot = (uint8_t)I.c; D.x = I.b;
          D.fl = (uint8_t)(I.op == CKC_OP_LOAD ? I.d : (I.d & 3));
          D.dst = I.op == CKC_OP_LOAD ? P(I.dst) : 0;
          // a STORE whose value nothing reads back is a checked write
          if (I.op == CKC_OP_STORE) {
            if (I.store_val) D.b = P(I.dst);
            else D.op = CKC_OP_ACCESS;
          }
          daccess& A = acc[I.b];
          A.pc = (uint16_t)newpc[i];
          A.depth = (uint16_t)I.depth;
          A.loop_pc[0] = A.loop_pc[1] = -1;
          int lv = I.depth;
          for (int p = I.parent; p >= 0; p = ins[p].parent)
            if (ins[p].op == CKC_OP_LOOP) A.loop_pc[--lv] = (int16_t)newpc[p];
          break;
        }
        case CKC_OP_IF:
          D.a = P(I.a);
          D.jmp = (uint16_t)newpc[I.alt >= 0 ? I.alt : I.end];
          D.fl = (uint8_t)((noskip[i] ? DI_NOSKIP : 0) | (I.alt >= 0 ? DI_HASELSE : 0));
          break;
        case CKC_OP_ELSE: D.jmp = (uint16_t)newpc[I.end]; D.fl = noskip[I.parent] ? DI_NOSKIP : 0; break;
        case CKC_OP_ENDIF: break;
        case CKC_OP_LOOP:
          D.dst = P(I.dst); D.a = P(I.a); D.b = P(I.b); D.c = P(I.c);
          D.x = (uint16_t)I.depth;
          D.jmp = (uint16_t)newpc[I.end];
          D.fl = (uint8_t)(i == expand_pc ? (DI_EXPAND | DI_NOSKIP) : 0);
          break;
        case CKC_OP_ENDLOOP: D.jmp = (uint16_t)newpc[I.end]; D.x = (uint16_t)ins[I.end].depth; break;
        case CKC_OP_BARRIER: break;
        case CKC_OP_FEXP: case CKC_OP_ITOF: case CKC_OP_FTOI: D.dst = P(I.dst); D.a = P(I.a); break;
        default: D.dst = P(I.dst); D.a = P(I.a); D.b = P(I.b); break;
      }
      if (slice[i] && I.op < CKC_OP_ACCESS) D.fl |= DI_SLICE;
      out[newpc[i]] = D;
    }
    auto al = [](uint32_t v) { return (v + 15u) & ~15u; };
    dprog h;
    std::memset(&h, 0, sizeof h);
    h.n_instr = (uint32_t)m;
    h.n_consts = (uint32_t)dconsts.size();
    h.n_accesses = (uint32_t)n_accesses;
    h.n_sites = (uint32_t)(n_sites + n_internal);
    h.n_map_sites = (uint32_t)n_sites;
    h.n_slots = (uint32_t)n_slots;
    h.n_scalars = (uint32_t)n_scalars;
    h.max_depth = (uint32_t)max_depth;
    h.cls = cls;
    h.n_regs = (uint32_t)n_phys;
    h.expand_pc = expand_pc >= 0 ? newpc[expand_pc] : -1;
    h.n_livein = (uint32_t)livein.size();
    if (expand_pc >= 0)
      for (int i = expand_pc + 1; i < ins[expand_pc].end; i++)
        if (ins[i].live && ins[i].op == CKC_OP_SPECIAL && ins[i].a < 6) h.body_special = 1;
    h.body_gather = body_gather ? 1u : 0u;
    h.slot_spaces = slot_spaces;
    bool w32 = false;
    const bool rows = rows_form(&w32);
    h.pflags = (uint32_t)((blockwise() ? PF_BLOCKWISE : 0) | (shared_idx ? PF_CAPTURE : 0) | (rows ? PF_ROWS : 0) |
                          (rows && w32 ? PF_ROWS32 : 0));
    for (size_t k = 0; k < livein.size(); k++) h.livein[k] = (uint8_t)livein[k];
    h.trace_cap = trace_cap;
    h.off_instr = al(sizeof(dprog));
    h.off_consts = al(h.off_instr + 16u * m);
    h.off_access = al(h.off_consts + 8u * h.n_consts);
    h.off_sites = al(h.off_access + (uint32_t)sizeof(daccess) * n_accesses);
    h.total_bytes = al(h.off_sites + 2u * n_sites);
    std::vector<uint8_t> blob(h.total_bytes, 0);
    std::memcpy(blob.data(), &h, sizeof h);
    if (m) std::memcpy(blob.data() + h.off_instr, out.data(), 16u * m);
    if (!dconsts.empty()) std::memcpy(blob.data() + h.off_consts, dconsts.data(), 8u * dconsts.size());
    if (n_accesses) std::memcpy(blob.data() + h.off_access, acc.data(), sizeof(daccess) * n_accesses);
    if (n_sites) std::memcpy(blob.data() + h.off_sites, site_ids.data(), 2u * n_sites);
    return blob;
  }

  // Static upper bound of the per-thread access count of a uniform program,
  // when every loop around an access has constant bounds; else 0 (unknown).
  uint64_t static_trace_len() const {
    auto cval = [&](uint16_t r, int w, int64_t* v) {
      int p = def_pc[r];
      if (p < 0 || ins[p].op != CKC_OP_CONST) return false;
      *v = wrapw(consts[ins[p].a], w);
      return true;
    };
    uint64_t total = 0;
    for (int i = 0; i < n_instr; i++) {
      const Ins& I = ins[i];
      // every checked access is a trace entry: a STORE too (lowered to an ACCESS)
      if (!I.live || (I.op != CKC_OP_ACCESS && I.op != CKC_OP_LOAD && I.op != CKC_OP_STORE)) continue;
      uint64_t mult = 1;
      for (int p = I.parent; p >= 0; p = ins[p].parent) {
        const Ins& L = ins[p];
        if (L.op != CKC_OP_LOOP) continue;
        int64_t s, e, st;
        if (!cval(L.a, L.w, &s) || !cval(L.b, L.w, &e) || !cval(L.c, L.w, &st)) return 0;
        uint64_t n = 0;
        if (st > 0 && s < e) n = ((uint64_t)e - (uint64_t)s + (uint64_t)st - 1) / (uint64_t)st;
        else if (st < 0 && s > e) n = ((uint64_t)s - (uint64_t)e + (0 - (uint64_t)st) - 1) / (0 - (uint64_t)st);
        else if (st == 0 && s < e) return 0;
        mult *= n;
        if (mult > (1u << 20)) return 0;
      }
      total += mult;
      if (total > (1u << 20)) return 0;
    }
    return total;
  }
};

}  // namespace

int analyze_program(const void* ir, size_t ir_bytes, Loaded* out, bool no_prune) {
  Analyzer A;
  A.ir = (const uint8_t*)ir;
  A.n = ir_bytes;
  A.no_prune = no_prune;
  if (!A.decode() || !A.validate() || !A.prune()) {
    out->err = A.err;
    return CKC_E_IR;
  }
  A.classify();
  if (!A.allocate()) {
    out->err = A.err;
    return CKC_E_IR;
  }
  // per-access facts and the program class
  out->acc.assign(A.n_accesses, ckc_access_info{});
  bool all_affine = true, any_guard = false, any_ind = false, any64 = false;
  for (int i = 0; i < A.n_instr; i++) {
    const Ins& I = A.ins[i];
    if (I.op != CKC_OP_ACCESS && I.op != CKC_OP_LOAD && I.op != CKC_OP_STORE) continue;
    ckc_access_info& ai = out->acc[I.b];
    ai.access_id = I.b;
    ai.slot = I.c;
    ai.log2_elem = I.op == CKC_OP_LOAD ? I.d : (I.d & 3u);
    ai.width = I.w;
    const Form& f = A.form[I.a];
    bool aff = f.affine && (A.uni[I.a] || f.k == 0 || f.k >= I.w);
    ai.affine = aff;
    ai.guarded = A.ctrl_var[i];
    ai.indirect = A.indirect[I.a];
    ai.loop_depth = I.depth;
    for (int d = 0; d < 7; d++)
      ai.coef[d] = aff ? ((uint64_t)f.c[d].kind << 32) | (uint32_t)f.c[d].v : (3ull << 32);
    all_affine &= aff;
    any_guard |= (bool)ai.guarded;
    any_ind |= (bool)ai.indirect;
    any64 |= I.w == 64;
  }
  // uniform-trace eligibility: thread-invariant control, affine indices, and
  // every live thread-dependent value that is used is affine
  bool any_var_ctrl = false, var_ok = true;
  for (int i = 0; i < A.n_instr; i++) {
    const Ins& I = A.ins[i];
    if (!I.live) continue;
    if (I.op == CKC_OP_IF && !A.uni[I.a]) any_var_ctrl = true;
    if (I.op == CKC_OP_LOOP && !A.uni[I.dst]) any_var_ctrl = true;
    if (is_float(I.op) || I.store_val || I.op == CKC_OP_BARRIER) var_ok = false;  // not on the trace path
    if (defines_op(I.op) && I.op != CKC_OP_LOOP && I.dst < A.n_regs && !A.uni[I.dst]) {
      if (is_divrem(I.op)) var_ok = false;
      else if (!A.form[I.dst].affine && A.reg_used(I.dst)) var_ok = false;
    }
  }
  bool uniform_prog = all_affine && !any_var_ctrl && var_ok && !A.blockwise() && !no_prune;
  uint32_t cls = (all_affine ? CKC_CLS_AFFINE : 0) | (any_guard ? CKC_CLS_GUARDED : 0) |
                 (any_ind ? CKC_CLS_INDIRECT : 0) | (any64 ? CKC_CLS_I64 : 0) |
                 (uniform_prog ? CKC_CLS_UNIFORM : 0) | (A.shared_idx ? CKC_CLS_BARRIER : 0);
  A.choose_expansion(uniform_prog);
  A.check_gather();
  if (A.expand_pc >= 0) cls |= CKC_CLS_EXPANDED;
  if (A.body_gather) cls |= CKC_CLS_GATHER;
  uint32_t trace_cap = 0;
  if (uniform_prog) {
    uint64_t s = A.static_trace_len();
    trace_cap = s ? (uint32_t)std::min<uint64_t>(s, 4096) : 256;
    if (trace_cap == 0) trace_cap = 1;
  }
  int n_live = 0;
  out->blob = A.lower(cls, trace_cap, &n_live);
  std::memset(&out->info, 0, sizeof out->info);
  out->info.n_accesses = A.n_accesses;
  out->info.n_sites = A.n_sites;
  out->info.n_slots = A.n_slots;
  out->info.n_scalars = A.n_scalars;
  out->info.max_loop_depth = A.max_depth;
  out->info.cls = cls;
  out->info.n_instr_live = n_live;
  out->info.n_regs_phys = A.n_phys;
  const uint32_t pf = ((const dprog*)out->blob.data())->pflags;
  out->info.rows_form = (pf & PF_ROWS32) ? 2u : (pf & PF_ROWS) ? 1u : 0u;
  out->load_slots = 0;
  for (int i = 0; i < A.n_instr; i++)
    if (A.ins[i].op == CKC_OP_LOAD && A.space_of(A.ins[i].c) == CKC_SPACE_GLOBAL)
      out->load_slots |= 1u << A.ins[i].c;
  return CKC_OK;
}

}  // namespace ckc
