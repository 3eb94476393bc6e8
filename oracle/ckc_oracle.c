/*
 * ckc_oracle.c — the reference checker for index programs.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the oracle that the GPU library is
 * compared against; it is used by the tests, by the smoke check and by the
 * benchmark's CPU-baseline leg, and by nothing else.  It shares no code,
 * header, table or helper with the library: it decodes the IR bytes itself and
 * defines its own constants.
 *
 * What it computes is the plain definition of the result the paper's fuzzing
 * pipeline produces for one kernel launch under AddressSanitizer and AFL++
 * coverage (Section 4: the kernel is translated so that every GPU thread runs
 * on the CPU and every memory access is checked; Section 2.1: a coverage map
 * is filled while the program runs):
 *
 *   for every input, in order
 *     for every thread of the chosen thread set, in global-thread-id order
 *       run the program sequentially, check every access against the
 *       allocation it names, count every site visit.
 *
 * The thread sets are the whole grid (what the paper runs for kernels that
 * are not affine-access, Section 5.1), the corner threads of the PREX Theorem
 * (Section 5.1.1), the boundary-blocks-plus-one-interior set, and the block
 * order of the PREX runtime algorithm (Section 5.1.2, Algorithm 1).
 *
 * Readings where the paper is silent (each one is listed with its reason in
 * the design notes of the repository):
 *   - bounds are exact per allocation (the paper contrasts redzone tripwires
 *     with base-and-bounds checking in Section 7.1); a violation is recorded
 *     and execution continues (record-and-continue, so that "first violation
 *     per access" is defined);
 *   - a violating LOAD reads 0;
 *   - integer arithmetic wraps at its width; division by zero gives 0 and is
 *     counted as an arithmetic fault; INT_MIN / -1 = INT_MIN;
 *   - the first violation of an access is the one with the smallest
 *     (global thread id, outer iteration, inner iteration), packed into a
 *     64-bit key;
 *   - coverage is one saturating (at 255) hit counter per program site,
 *     the LLVM-PCGuard style the paper fuzzes with (Section 7.1).
 *
 * Build: gcc -O2 -shared -fPIC -pthread ckc_oracle.c -o libckc_oracle.so
 */
#include <limits.h>
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ---- IR constants, decoded independently of the library ---------------- */
enum {
  O_CONST = 1, O_SCALAR = 2, O_SPECIAL = 3,
  O_ADD = 8, O_SUB, O_MUL, O_DIVS, O_DIVU, O_REMS, O_REMU, O_AND, O_OR, O_XOR,
  O_SHL, O_SHRA, O_SHRL, O_MINS, O_MAXS, O_MINU, O_MAXU,
  O_CMPEQ, O_CMPNE, O_CMPLTS, O_CMPLES, O_CMPLTU, O_CMPLEU,
  O_SELECT = 31, O_SEXT = 32, O_ZEXT = 33, O_TRUNC = 34,
  O_FADD = 40, O_FSUB = 41, O_FMUL = 42, O_FEXP = 43, O_ITOF = 44, O_FTOI = 45,
  O_ACCESS = 48, O_LOAD = 49, O_STORE = 50,
  O_IF = 56, O_ELSE = 57, O_ENDIF = 58, O_LOOP = 59, O_ENDLOOP = 60, O_BARRIER = 61
};
#define NOSITE 0xFFFFu
#define NOREG 0xFFFFu

/* violation kinds */
#define K_OVER 1u
#define K_UNDER 2u
#define K_FREED 4u
#define K_NULL 8u
#define A_FREED 1u

/* memory spaces of allocation slots (2 bits per slot in the IR header) */
#define SP_GLOBAL 0u
#define SP_SHARED 1u
#define SP_LOCAL 2u

/* detector models */
#define DET_EXACT 0u
#define DET_TRIPWIRE 1u

/* thread-set modes */
#define M_FULL 0u
#define M_CORNERS 1u
#define M_BOUNDARY 2u
#define M_PREX 3u

#define E_OK 0
#define E_INVALID (-1)
#define E_IR (-2)
#define E_RANGE (-3)

typedef struct { uint64_t base, size_bytes; const void* data; uint32_t flags, redzone; } or_alloc;
typedef struct { uint64_t first_key; int64_t index; uint64_t count; uint32_t kinds, first_kind; } or_record;
typedef struct { uint64_t lanes, accesses_checked, hang_lanes, arith_faults; uint32_t flags, pad; } or_status;

typedef struct {
  uint8_t op, w;
  uint16_t dst, a, b, c, d, s0, s1;
  int32_t alt;  /* IF: its ELSE (or -1); */
  int32_t end;  /* IF/ELSE: its ENDIF; LOOP: its ENDLOOP */
  int32_t depth; /* loop depth of the instruction itself (LOOP: depth it opens) */
} or_ins;

typedef struct {
  int n_instr, n_consts, n_scalars, n_slots, n_accesses, n_sites, n_regs;
  const int64_t* consts; /* points into a private copy */
  uint16_t* site_ids;
  or_ins* ins;
  int max_depth;
  uint8_t* load_slot; /* slot used by some LOAD */
  int64_t* const_copy;
  uint8_t* in_slice;  /* [n_instr]: an index, IF predicate or loop bound depends on it */
  uint8_t space[16];  /* memory space of each slot */
  int has_barrier;     /* some BARRIER */
  int block_sync;      /* some LOAD reads shared memory: blocks run phase by phase */
  uint32_t shared_idx; /* shared slots some LOAD of which feeds the slice (bit per slot):
                          the index-related shared variables of the paper's Algorithm 2 */
  uint32_t shared_live; /* shared slots read back into the pruned program (indices,
                           control or divisions): BARRIERs are kept when nonzero */
  uint8_t* kept;       /* [n_instr]: what the pruned program keeps (for counting) */
} or_prog;

static uint16_t rd16(const uint8_t* p) { return (uint16_t)(p[0] | (p[1] << 8)); }
static uint32_t rd32(const uint8_t* p) { return (uint32_t)rd16(p) | ((uint32_t)rd16(p + 2) << 16); }
static int64_t rd64(const uint8_t* p) { return (int64_t)((uint64_t)rd32(p) | ((uint64_t)rd32(p + 4) << 32)); }

static void prog_free(or_prog* P) {
  free(P->site_ids); free(P->ins); free(P->load_slot); free(P->const_copy); free(P->in_slice); free(P->kept);
  memset(P, 0, sizeof *P);
}

static int is_binary(int op) { return op >= O_ADD && op <= O_CMPLEU; }
static int is_fbinary(int op) { return op == O_FADD || op == O_FSUB || op == O_FMUL; }
static int is_funary(int op) { return op == O_FEXP || op == O_ITOF || op == O_FTOI; }
/* ops that define no register */
static int defines_nothing(int op) {
  return op == O_ACCESS || op == O_STORE || op == O_IF || op == O_ELSE || op == O_ENDIF || op == O_ENDLOOP ||
         op == O_BARRIER;
}

/* The live-register rule of the IR description: a register lives from its
 * definition to its last use, a use inside a loop that does not contain the
 * definition extends it to that loop's end (the outermost such loop), a loop
 * counter lives to its ENDLOOP; at each defining instruction, the registers
 * defined earlier and live beyond it, plus one, are at most 32.  Needs the
 * loop ends (I->end) filled in. */
static int pressure_ok(const or_prog* P) {
  int n = P->n_instr, nr = P->n_regs, ok = 1;
  int* def_at = (int*)malloc(sizeof(int) * (nr + 1));
  int* endr = (int*)malloc(sizeof(int) * (nr + 1));
  int* diff = (int*)calloc(n + 2, sizeof(int));
  for (int r = 0; r < nr; r++) { def_at[r] = -1; endr[r] = -1; }
  for (int i = 0; i < n; i++) {
    const or_ins* I = &P->ins[i];
    int op = I->op;
    if (!defines_nothing(op)) def_at[I->dst] = i;
  }
  int loops[4], nl = 0; /* open LOOPs, outermost first */
  for (int u = 0; u < n; u++) {
    const or_ins* I = &P->ins[u];
    int op = I->op, uses[3], nu = 0;
    if (op == O_ENDLOOP) { nl--; continue; }
    if (op == O_SELECT || op == O_LOOP) { uses[nu++] = I->a; uses[nu++] = I->b; uses[nu++] = I->c; }
    else if (op == O_SEXT || op == O_ZEXT || op == O_TRUNC || op == O_ACCESS || op == O_LOAD || op == O_IF ||
             is_funary(op)) uses[nu++] = I->a;
    else if (op == O_STORE) { uses[nu++] = I->a; uses[nu++] = I->dst; }
    else if (is_binary(op) || is_fbinary(op)) { uses[nu++] = I->a; uses[nu++] = I->b; }
    for (int k = 0; k < nu; k++) {
      int r = uses[k], e = u;
      for (int q = 0; q < nl; q++)
        if (loops[q] > def_at[r]) { if (P->ins[loops[q]].end > e) e = P->ins[loops[q]].end; break; }
      if (e > endr[r]) endr[r] = e;
    }
    if (op == O_LOOP) {
      if (I->end > endr[I->dst]) endr[I->dst] = I->end;
      loops[nl++] = u;
    }
  }
  for (int r = 0; r < nr; r++)
    if (def_at[r] >= 0 && endr[r] > def_at[r]) { diff[def_at[r] + 1]++; diff[endr[r]]--; }
  int cur = 0;
  for (int i = 0; i < n && ok; i++) {
    cur += diff[i];
    int op = P->ins[i].op;
    if (!defines_nothing(op) && cur + 1 > 32) ok = 0;
  }
  free(def_at); free(endr); free(diff);
  return ok;
}

/* Decode and validate the byte format (include/ckc_ir.h describes it; this is
 * an independent reading of that description). */
/* One backward pass (every definition precedes its uses) from the roots:
 * the accesses (a STORE's value too when its slot is in xs), IF predicates
 * and loop bounds and, with `divs`, the divisions and remainders (they count
 * arithmetic faults, so their operands must be exact); every instruction whose
 * result a marked instruction reads is marked.  Returns the shared slots some
 * LOAD of which has its result needed. */
static uint32_t slice_pass(const or_prog* P, uint32_t xs, int divs, uint8_t* need, uint8_t* mark) {
  memset(need, 0, P->n_regs + 1);
  memset(mark, 0, P->n_instr + 1);
  for (int i = P->n_instr - 1; i >= 0; i--) {
    const or_ins* I = &P->ins[i];
    int op = I->op;
    int div = op == O_DIVS || op == O_DIVU || op == O_REMS || op == O_REMU;
    int root = op == O_ACCESS || op == O_LOAD || op == O_STORE || op == O_IF || op == O_LOOP || (divs && div);
    int keep = root || (!defines_nothing(op) && op != O_LOOP && I->dst < P->n_regs && need[I->dst]);
    if (!keep) continue;
    mark[i] = 1;
    if (op == O_CONST || op == O_SCALAR || op == O_SPECIAL) continue;
    need[I->a] = 1;
    if (op == O_LOOP || op == O_SELECT) { need[I->b] = 1; need[I->c] = 1; }
    else if (is_binary(op) || is_fbinary(op)) need[I->b] = 1;
    else if (op == O_STORE && ((xs >> I->c) & 1u)) need[I->dst] = 1;
  }
  uint32_t nxs = 0;
  for (int i = 0; i < P->n_instr; i++) {
    const or_ins* I = &P->ins[i];
    if (I->op == O_LOAD && P->space[I->c] == SP_SHARED && need[I->dst]) nxs |= 1u << I->c;
  }
  return nxs;
}

/* Shared slots read back into the pass's result (the index-related shared
 * variables of Algorithm 2 when `divs` is 0): a shared slot is one when some
 * LOAD from it has its result needed; then the values STOREd to it are
 * needed too, which may bring in more loads.  Repeated until nothing changes
 * (the set only grows); mark[] holds the last pass. */
static uint32_t slice_fixpoint(const or_prog* P, int divs, uint8_t* need, uint8_t* mark) {
  uint32_t xs = 0;
  for (;;) {
    uint32_t nxs = slice_pass(P, xs, divs, need, mark);
    if (nxs == xs) return xs;
    xs = nxs;
  }
}

static int prog_decode(const uint8_t* ir, size_t n, or_prog* P) {
  memset(P, 0, sizeof *P);
  if (!ir || n < 32) return E_IR;
  if (rd32(ir) != 0x31434B43u || rd16(ir + 4) != 1) return E_IR;
  P->n_instr = rd16(ir + 6); P->n_consts = rd16(ir + 8); P->n_scalars = rd16(ir + 10);
  P->n_slots = rd16(ir + 12); P->n_accesses = rd16(ir + 14); P->n_sites = rd16(ir + 16);
  P->n_regs = rd16(ir + 18);
  for (int i = 24; i < 32; i++) if (ir[i]) return E_IR;
  if (P->n_scalars > 16 || P->n_slots > 16 || P->n_accesses > 1024 || P->n_sites > 4096 ||
      P->n_instr > 4096 || P->n_consts > 4096) return E_IR;
  /* slot spaces: two bits per slot, global / shared / local; none for slots
   * the program does not have */
  {
    uint32_t spaces = rd32(ir + 20);
    for (int s = 0; s < 16; s++) {
      uint32_t v = (spaces >> (2 * s)) & 3u;
      if (v > SP_LOCAL || (s >= P->n_slots && v != 0)) return E_IR;
      P->space[s] = (uint8_t)v;
    }
  }
  size_t site_bytes = ((size_t)P->n_sites * 2 + 7) / 8 * 8;
  size_t need = 32 + (size_t)P->n_consts * 8 + site_bytes + (size_t)P->n_instr * 16;
  if (need != n) return E_IR;
  const uint8_t* pc = ir + 32;
  P->const_copy = (int64_t*)calloc(P->n_consts + 1, 8);
  for (int i = 0; i < P->n_consts; i++) P->const_copy[i] = rd64(pc + 8 * i);
  P->consts = P->const_copy;
  const uint8_t* ps = pc + 8 * P->n_consts;
  P->site_ids = (uint16_t*)calloc(P->n_sites + 1, 2);
  for (int i = 0; i < P->n_sites; i++) P->site_ids[i] = rd16(ps + 2 * i);
  const uint8_t* pi = ps + site_bytes;
  P->ins = (or_ins*)calloc(P->n_instr + 1, sizeof(or_ins));
  P->load_slot = (uint8_t*)calloc(17, 1);
  for (int i = 0; i < P->n_instr; i++) {
    const uint8_t* q = pi + 16 * i;
    or_ins* I = &P->ins[i];
    I->op = q[0]; I->w = q[1]; I->dst = rd16(q + 2); I->a = rd16(q + 4); I->b = rd16(q + 6);
    I->c = rd16(q + 8); I->d = rd16(q + 10); I->s0 = rd16(q + 12); I->s1 = rd16(q + 14);
    I->alt = -1; I->end = -1;
  }

  /* site ids unique; every site index and access id used at most once */
  int rc = E_IR;
  uint8_t* seen_id = (uint8_t*)calloc(65536, 1);
  uint8_t* site_used = (uint8_t*)calloc(P->n_sites + 1, 1);
  uint8_t* acc_used = (uint8_t*)calloc(P->n_accesses + 1, 1);
  int32_t* def_scope = (int32_t*)malloc(sizeof(int32_t) * (P->n_regs + 1));
  uint8_t* scope_open = (uint8_t*)calloc(P->n_instr + 2, 1);
  int32_t stack[64]; int sp = 0; int loop_depth = 0; int n_scopes = 1;
  for (int r = 0; r < P->n_regs; r++) def_scope[r] = -1;
  for (int i = 0; i < P->n_sites; i++) { if (seen_id[P->site_ids[i]]) goto out; seen_id[P->site_ids[i]] = 1; }
  scope_open[0] = 1;
  int32_t scope_stack[64]; int ssp = 0; scope_stack[ssp++] = 0;

#define USE(r) do { if ((r) >= P->n_regs || def_scope[(r)] < 0 || !scope_open[def_scope[(r)]]) goto out; } while (0)
#define DEF(r) do { if ((r) >= P->n_regs || def_scope[(r)] != -1) goto out; def_scope[(r)] = scope_stack[ssp - 1]; } while (0)
#define SITE(s) do { if ((s) != NOSITE) { if ((s) >= P->n_sites || site_used[(s)]) goto out; site_used[(s)] = 1; } } while (0)
#define WIDTH(wv) do { if ((wv) != 32 && (wv) != 64) goto out; } while (0)

  for (int i = 0; i < P->n_instr; i++) {
    or_ins* I = &P->ins[i];
    I->depth = loop_depth;
    switch (I->op) {
      case O_CONST: WIDTH(I->w); if (I->a >= P->n_consts) goto out; DEF(I->dst); break;
      case O_SCALAR: WIDTH(I->w); if (I->a >= P->n_scalars) goto out; DEF(I->dst); break;
      case O_SPECIAL: if (I->a > 11) goto out; DEF(I->dst); break;
      case O_SELECT: WIDTH(I->w); USE(I->a); USE(I->b); USE(I->c); DEF(I->dst); break;
      case O_SEXT: case O_ZEXT: case O_TRUNC: USE(I->a); DEF(I->dst); break;
      case O_ACCESS:
      case O_LOAD:
        WIDTH(I->w); USE(I->a);
        if (I->b >= P->n_accesses || acc_used[I->b]) goto out;
        acc_used[I->b] = 1;
        if (I->c >= P->n_slots) goto out;
        if (I->op == O_ACCESS) { if (I->d > 7) goto out; }
        else {
          /* loads read global memory (the host's data) or shared memory
           * (4-byte elements written by the block's STOREs); local memory is
           * not modelled */
          if ((I->d != 2 && I->d != 3) || P->space[I->c] == SP_LOCAL) goto out;
          if (P->space[I->c] == SP_SHARED && I->d != 2) goto out;
          if (P->space[I->c] == SP_GLOBAL) P->load_slot[I->c] = 1;
          else P->block_sync = 1;
          DEF(I->dst);
        }
        SITE(I->s0);
        break;
      case O_STORE:
        WIDTH(I->w); USE(I->a); USE(I->dst);
        if (I->b >= P->n_accesses || acc_used[I->b]) goto out;
        acc_used[I->b] = 1;
        if (I->c >= P->n_slots || I->d > 3) goto out;
        SITE(I->s0);
        break;
      case O_FADD: case O_FSUB: case O_FMUL:
        if (I->w != 64) goto out;
        USE(I->a); USE(I->b); DEF(I->dst);
        break;
      case O_FEXP:
        if (I->w != 64) goto out;
        USE(I->a); DEF(I->dst);
        break;
      case O_ITOF:
        if (I->w != 32) goto out;
        USE(I->a); DEF(I->dst);
        break;
      case O_FTOI:
        WIDTH(I->w); USE(I->a); DEF(I->dst);
        break;
      case O_BARRIER:
        if (sp != 0) goto out; /* __syncthreads at the top level only */
        P->has_barrier = 1;
        break;
      case O_IF:
        USE(I->a); SITE(I->s0); SITE(I->s1);
        if (sp >= 16) goto out;
        stack[sp++] = i;
        scope_open[n_scopes] = 1; scope_stack[ssp++] = n_scopes++;
        break;
      case O_ELSE:
        if (sp == 0 || P->ins[stack[sp - 1]].op != O_IF || P->ins[stack[sp - 1]].alt >= 0) goto out;
        P->ins[stack[sp - 1]].alt = i;
        scope_open[scope_stack[--ssp]] = 0;
        scope_open[n_scopes] = 1; scope_stack[ssp++] = n_scopes++;
        break;
      case O_ENDIF: {
        if (sp == 0 || P->ins[stack[sp - 1]].op != O_IF) goto out;
        int f = stack[--sp];
        P->ins[f].end = i;
        if (P->ins[f].alt >= 0) P->ins[P->ins[f].alt].end = i;
        scope_open[scope_stack[--ssp]] = 0;
        break;
      }
      case O_LOOP:
        WIDTH(I->w); USE(I->a); USE(I->b); USE(I->c); SITE(I->s0); SITE(I->s1);
        if (sp >= 16 || loop_depth >= 2) goto out;
        stack[sp++] = i; loop_depth++;
        if (loop_depth > P->max_depth) P->max_depth = loop_depth;
        scope_open[n_scopes] = 1; scope_stack[ssp++] = n_scopes++;
        DEF(I->dst);
        break;
      case O_ENDLOOP: {
        if (sp == 0 || P->ins[stack[sp - 1]].op != O_LOOP) goto out;
        int f = stack[--sp];
        P->ins[f].end = i; I->end = f; loop_depth--;
        scope_open[scope_stack[--ssp]] = 0;
        break;
      }
      default:
        if (!is_binary(I->op)) goto out;
        WIDTH(I->w); USE(I->a); USE(I->b); DEF(I->dst);
        break;
    }
    if (ssp > 60) goto out;
  }
  if (sp != 0) goto out;
  for (int a = 0; a < P->n_accesses; a++) if (!acc_used[a]) goto out;
  if (!pressure_ok(P)) goto out;
  /* The slice of the indices, IF predicates and loop bounds, and the live
   * set of the pruned program (Algorithm 2); see slice_fixpoint. */
  {
    uint8_t* need = (uint8_t*)calloc(P->n_regs + 1, 1);
    uint8_t* live = (uint8_t*)calloc(P->n_instr + 1, 1);
    P->in_slice = (uint8_t*)calloc(P->n_instr + 1, 1);
    P->shared_idx = slice_fixpoint(P, 0, need, P->in_slice);
    const uint32_t xl = slice_fixpoint(P, 1, need, live);
    P->shared_live = xl;
    /* what the pruned program keeps (MathElimination): the live set, the
     * structure of IF and LOOP and, when some shared variable is read back
     * into it, every BARRIER (BarrierElimination is all or none) */
    P->kept = (uint8_t*)calloc(P->n_instr + 1, 1);
    for (int i = 0; i < P->n_instr; i++) {
      int op = P->ins[i].op;
      P->kept[i] = live[i] || op == O_ELSE || op == O_ENDIF || op == O_ENDLOOP || (op == O_BARRIER && xl != 0);
    }
    free(need); free(live);
  }
  rc = E_OK;
out:
#undef USE
#undef DEF
#undef SITE
#undef WIDTH
  free(seen_id); free(site_used); free(acc_used); free(def_scope); free(scope_open);
  if (rc != E_OK) prog_free(P);
  return rc;
}

/* ---- integer semantics (wrap at width w; see the IR description) -------- */
static uint64_t narrow(uint64_t v, int w) { return w == 32 ? (uint64_t)(int64_t)(int32_t)(uint32_t)v : v; }

static uint64_t alu(int op, int w, uint64_t x, uint64_t y, uint64_t* faults) {
  x = narrow(x, w); y = narrow(y, w);
  uint64_t mask = w == 32 ? 0xFFFFFFFFull : ~0ull;
  uint64_t ux = x & mask, uy = y & mask; /* unsigned views */
  int64_t sx = (int64_t)x, sy = (int64_t)y; /* signed views (already sign-extended) */
  int64_t smin = w == 32 ? (int64_t)INT32_MIN : INT64_MIN;
  unsigned sh = (unsigned)(uy & (uint64_t)(w - 1));
  uint64_t r = 0;
  switch (op) {
    case O_ADD: r = ux + uy; break;
    case O_SUB: r = ux - uy; break;
    case O_MUL: r = ux * uy; break;
    case O_DIVS:
      if (sy == 0) { (*faults)++; r = 0; }
      else if (sx == smin && sy == -1) r = (uint64_t)smin;
      else r = (uint64_t)(sx / sy);
      break;
    case O_REMS:
      if (sy == 0) { (*faults)++; r = 0; }
      else if (sx == smin && sy == -1) r = 0;
      else r = (uint64_t)(sx % sy);
      break;
    case O_DIVU: if (uy == 0) { (*faults)++; r = 0; } else r = ux / uy; break;
    case O_REMU: if (uy == 0) { (*faults)++; r = 0; } else r = ux % uy; break;
    case O_AND: r = ux & uy; break;
    case O_OR: r = ux | uy; break;
    case O_XOR: r = ux ^ uy; break;
    case O_SHL: r = ux << sh; break;
    case O_SHRA: r = (uint64_t)(sx >> sh); break;
    case O_SHRL: r = ux >> sh; break;
    case O_MINS: r = (uint64_t)(sx < sy ? sx : sy); break;
    case O_MAXS: r = (uint64_t)(sx > sy ? sx : sy); break;
    case O_MINU: r = ux < uy ? ux : uy; break;
    case O_MAXU: r = ux > uy ? ux : uy; break;
    case O_CMPEQ: r = ux == uy; break;
    case O_CMPNE: r = ux != uy; break;
    case O_CMPLTS: r = sx < sy; break;
    case O_CMPLES: r = sx <= sy; break;
    case O_CMPLTU: r = ux < uy; break;
    case O_CMPLEU: r = ux <= uy; break;
  }
  return narrow(r, w);
}

/* Trip count of LOOP start,end,step at width w, as an exact integer,
 * saturated at UINT64_MAX ("never ends"). */
static uint64_t trip_count(int64_t s, int64_t e, int64_t step) {
  if (step >= 0) {
    if (!(s < e)) return 0;
    if (step == 0) return UINT64_MAX;
    uint64_t span = (uint64_t)e - (uint64_t)s; /* exact: e > s */
    return span / (uint64_t)step + (span % (uint64_t)step != 0);
  } else {
    if (!(s > e)) return 0;
    uint64_t span = (uint64_t)s - (uint64_t)e;
    uint64_t mag = (uint64_t)0 - (uint64_t)step;
    return span / mag + (span % mag != 0);
  }
}

/* e^x as the IR defines FEXP: k = floor(x / ln 2 + 1/2), r = (x - k ln2_hi)
 * - k ln2_lo with ln 2 split into a part of 29 significant bits (k times it
 * is exact) and the rest, the Taylor polynomial of e^r to degree 13 in Horner
 * form, times 2^k (in two
 * steps below 2^-1022); NaN stays NaN, x above 709.782712893384 gives +inf,
 * below -745.1332191019412 gives 0.  Plain IEEE binary64 operations, each
 * rounded on its own, so that any two implementations agree bit for bit. */
static double ir_exp(double x) {
  static const double C[14] = {
      0x1.0000000000000p+0, 0x1.0000000000000p+0, 0x1.0000000000000p-1, 0x1.5555555555555p-3,
      0x1.5555555555555p-5, 0x1.1111111111111p-7, 0x1.6c16c16c16c17p-10, 0x1.a01a01a01a01ap-13,
      0x1.a01a01a01a01ap-16, 0x1.71de3a556c734p-19, 0x1.27e4fb7789f5cp-22, 0x1.ae64567f544e4p-26,
      0x1.1eed8eff8d898p-29, 0x1.6124613a86d09p-33};
  if (x != x) return x;
  if (x > 709.782712893384) return INFINITY;
  if (x < -745.1332191019412) return 0.0;
  volatile double t = x * 0x1.71547652b82fep+0;
  const double k = floor(t + 0.5);
  volatile double kh = k * 0x1.62e42ff000000p-1;
  volatile double r0 = x - kh;
  volatile double kl = k * -0x1.718432a1b0e26p-35;
  const double r = r0 - kl;
  double p = C[13];
  for (int i = 12; i >= 0; i--) {
    volatile double pr = p * r;
    p = pr + C[i];
  }
  const int ki = (int)k;
  uint64_t b;
  double s;
  if (ki > 1023) {
    b = (uint64_t)(1023 + 1023) << 52;
    memcpy(&s, &b, 8);
    volatile double q = p * s;
    return q * 2.0;
  }
  if (ki >= -1022) {
    b = (uint64_t)(ki + 1023) << 52;
    memcpy(&s, &b, 8);
    return p * s;
  }
  b = (uint64_t)(ki + 1000 + 1023) << 52;
  memcpy(&s, &b, 8);
  volatile double q = p * s;
  b = (uint64_t)(-1000 + 1023) << 52;
  memcpy(&s, &b, 8);
  return q * s;
}

/* ---- one thread --------------------------------------------------------- */
typedef struct {
  const or_prog* P;
  const int64_t* scalars;
  const uint32_t* launch; /* gx gy gz bx by bz */
  const or_alloc* table;
  uint32_t table_n;   /* entries of this input's table */
  uint32_t detector;  /* DET_EXACT or DET_TRIPWIRE */
  /* shared memory of the block being run: per slot its elements as at the
   * start of the phase, and the phase's writes (0 = none, else 2^32 | the
   * value's bits with the sign bit flipped, so that the maximum is the
   * largest value) */
  int32_t* sh_cur[16];
  uint64_t* sh_next[16];
  uint64_t sh_n[16];
  uint64_t* executed;  /* this input's [all, kept] instruction executions, or NULL */
  uint32_t tid[3], bid[3];
  uint64_t gtid;
  unsigned L1, L2;
  uint64_t cap[2];
  uint64_t* regs;
  uint64_t iter[2];
  int stopped;
  or_record* rec;  /* this input's records [n_accesses] */
  uint64_t* cnt;   /* this input's site counters [n_sites] */
  or_status* st;
  uint8_t* acc_seen; /* [n_accesses]: executed at least once in this input */
  /* vertex run (rep-exact flag): no records, visits or status updates; wraps
   * of slice instructions and the control decisions are observed instead */
  int dry;
  int wrapped;        /* some slice operation wrapped */
  int abort_run;      /* control path differs from vertex 0, or budget exceeded */
  uint64_t budget;    /* IF and LOOP executions plus loop iterations so far */
  uint64_t* dec;      /* decisions of vertex 0 (IF outcome, LOOP trip count) */
  size_t ndec, pos;
  int recording;
  uint64_t dummy_faults;
} thr;

#define VERTEX_BUDGET 65536u

/* One control decision of a vertex run: vertex 0 records it, the others must
 * repeat it; the budget counts it. */
static void decide(thr* t, uint64_t v) {
  if (++t->budget > VERTEX_BUDGET) { t->abort_run = 1; t->stopped = 1; return; }
  if (t->recording) { t->dec[t->ndec++] = v; return; }
  if (t->pos >= t->ndec || t->dec[t->pos] != v) { t->abort_run = 1; t->stopped = 1; return; }
  t->pos++;
}

/* Exact-integer checks of the vertex run.  fits(v, w): the signed value v is
 * representable at width w. */
static int fits(__int128 v, int w) {
  __int128 lo = w == 32 ? -((__int128)1 << 31) : -((__int128)1 << 63);
  __int128 hi = w == 32 ? ((__int128)1 << 31) : ((__int128)1 << 63);
  return v >= lo && v < hi;
}
/* A register read at width 32 must already hold an int32 value. */
static int read32_ok(uint64_t c) { return fits((__int128)(int64_t)c, 32); }

static void check_wrap(thr* t, const or_ins* I, uint64_t x, uint64_t y) {
  int w = I->w, op = I->op;
  if (w == 32 && (!read32_ok(x) || (is_binary(op) && !read32_ok(y)))) { t->wrapped = 1; return; }
  int64_t sx = (int64_t)narrow(x, w), sy = (int64_t)narrow(y, w);
  __int128 r;
  switch (op) {
    case O_ADD: r = (__int128)sx + sy; break;
    case O_SUB: r = (__int128)sx - sy; break;
    case O_MUL: r = (__int128)sx * sy; break;
    case O_SHL: r = (__int128)sx * ((__int128)1 << ((uint64_t)sy & (uint64_t)(w - 1))); break;
    case O_DIVS: r = (sy == -1 && sx == (w == 32 ? (int64_t)INT32_MIN : INT64_MIN)) ? -(__int128)sx : 0; break;
    default: return;
  }
  if (!fits(r, w)) t->wrapped = 1;
}

static void visit(thr* t, uint16_t s) { if (s != NOSITE && !t->dry) t->cnt[s]++; }

/* Check one access (the allocation-table check of an ASan-style detector). */
static uint32_t check_kind(const or_alloc* a, int64_t idx, unsigned log2e) {
  if (a->base == 0) return K_NULL;
  if (a->flags & A_FREED) return K_FREED;
  if (idx < 0) return K_UNDER;
  uint64_t n_elems = a->size_bytes >> log2e;
  if ((uint64_t)idx >= n_elems) return K_OVER;
  return 0;
}

/* The tripwire (redzone) detector of the address sanitizers the paper
 * contrasts with base-and-bounds checkers (Section 7.1, Table 1): memory is
 * poisoned only around allocations, so an access is caught when one of its
 * bytes falls in a redzone or in freed memory, and missed when it jumps over
 * the redzone into other memory.  Allocation k of the access's memory space
 * occupies [base, base + size); its redzones are the `redzone` bytes on each
 * side; a freed allocation is poisoned whole, redzones included.  A shared or
 * local slot lives in its block's or thread's own window, which ends at the
 * largest allocation end (redzone included) of that space: bytes beyond it
 * are caught too.  Addresses are exact integers (base + index * element
 * size), not wrapped.  Only called for an access that is out of exact bounds
 * on a non-NULL slot; returns 1 if the detector reports it. */
static int overlaps(__int128 a, __int128 b, __int128 x, __int128 y) { return x < y && a < y && x < b; }

static int tripwire_catches(const thr* t, int slot, int64_t idx, unsigned log2e) {
  const or_alloc* T = t->table;
  const int sp = t->P->space[slot];
  const __int128 a = (__int128)T[slot].base + (__int128)idx * ((__int128)1 << log2e);
  const __int128 b = a + ((__int128)1 << log2e); /* one past the last byte */
  __int128 window = 0;
  for (uint32_t k = 0; k < t->table_n; k++) {
    const or_alloc* A = &T[k];
    int ksp = k < 16 ? t->P->space[k] : (int)SP_GLOBAL;
    if (A->base == 0 || ksp != sp) continue;
    const __int128 lo = (__int128)A->base - A->redzone;
    const __int128 end = (__int128)A->base + A->size_bytes;
    const __int128 hi = end + A->redzone;
    if (hi > window) window = hi;
    if (A->flags & A_FREED) {
      if (overlaps(a, b, lo, hi)) return 1;
    } else if (overlaps(a, b, lo, (__int128)A->base) || overlaps(a, b, end, hi)) {
      return 1; /* a redzone */
    }
  }
  if (sp != SP_GLOBAL && (a < 0 || b > window)) return 1;
  return 0;
}

static void record(thr* t, int acc, uint32_t kind, int64_t idx) {
  if (t->dry) return;
  or_record* R = &t->rec[acc];
  uint64_t key = (t->gtid << (t->L1 + t->L2)) | (t->iter[0] << t->L2) | t->iter[1];
  R->count++;
  R->kinds |= kind;
  if (key < R->first_key) { R->first_key = key; R->index = idx; R->first_kind = kind; }
}

static void exec_range(thr* t, int pc, int end);

static void exec_one_loop(thr* t, int pc) {
  const or_ins* I = &t->P->ins[pc];
  int w = I->w;
  int64_t s = (int64_t)narrow(t->regs[I->a], w);
  int64_t e = (int64_t)narrow(t->regs[I->b], w);
  int64_t st = (int64_t)narrow(t->regs[I->c], w);
  uint64_t n = trip_count(s, e, st);
  int d = I->depth; /* 0 for a depth-1 loop */
  uint64_t cap = t->cap[d];
  uint64_t run = n < cap ? n : cap;
  if (t->dry) {
    if (w == 32 && (!read32_ok(t->regs[I->a]) || !read32_ok(t->regs[I->b]) || !read32_ok(t->regs[I->c])))
      t->wrapped = 1;
    decide(t, n);
    if (t->stopped) return;
  }
  for (uint64_t k = 0; k < run && !t->stopped; k++) {
    if (t->dry) {
      if (!fits((__int128)s + (__int128)k * st, w)) t->wrapped = 1;
      if (++t->budget > VERTEX_BUDGET) { t->abort_run = 1; t->stopped = 1; break; }
    }
    t->regs[I->dst] = narrow((uint64_t)s + k * (uint64_t)st, w);
    t->iter[d] = k;
    visit(t, I->s0);
    exec_range(t, pc + 1, I->end);
  }
  t->iter[d] = 0;
  if (t->stopped) return;
  if (n > cap) { t->stopped = 1; if (!t->dry) t->st->hang_lanes++; return; }
  visit(t, I->s1);
}

static void exec_range(thr* t, int pc, int end) {
  const or_prog* P = t->P;
  uint64_t* R = t->regs;
  while (pc < end && !t->stopped) {
    const or_ins* I = &P->ins[pc];
    if (t->executed && !t->dry) {
      t->executed[0]++;
      if (P->kept[pc]) t->executed[1]++;
    }
    switch (I->op) {
      case O_CONST: R[I->dst] = narrow((uint64_t)P->consts[I->a], I->w); break;
      case O_SCALAR: R[I->dst] = narrow((uint64_t)t->scalars[I->a], I->w); break;
      case O_SPECIAL: {
        uint32_t v;
        int k = I->a;
        if (k < 3) v = t->tid[k];
        else if (k < 6) v = t->bid[k - 3];
        else if (k < 9) v = t->launch[3 + (k - 6)];
        else v = t->launch[k - 9];
        R[I->dst] = (uint64_t)v;
        break;
      }
      case O_SELECT: {
        uint64_t v = R[I->a] != 0 ? R[I->b] : R[I->c];
        if (t->dry && P->in_slice[pc] && I->w == 32 && !read32_ok(v)) t->wrapped = 1;
        R[I->dst] = narrow(v, I->w);
        break;
      }
      case O_SEXT: case O_TRUNC:
        if (t->dry && P->in_slice[pc] && !read32_ok(R[I->a])) t->wrapped = 1;
        R[I->dst] = narrow(R[I->a], 32);
        break;
      case O_ZEXT:
        if (t->dry && P->in_slice[pc] && !(read32_ok(R[I->a]) && (int64_t)R[I->a] >= 0)) t->wrapped = 1;
        R[I->dst] = R[I->a] & 0xFFFFFFFFull;
        break;
      case O_FADD: case O_FSUB: case O_FMUL: {
        double x, y, r;
        memcpy(&x, &R[I->a], 8);
        memcpy(&y, &R[I->b], 8);
        r = I->op == O_FADD ? x + y : I->op == O_FSUB ? x - y : x * y;
        memcpy(&R[I->dst], &r, 8);
        break;
      }
      case O_FEXP: {
        double x, r;
        memcpy(&x, &R[I->a], 8);
        r = ir_exp(x);
        memcpy(&R[I->dst], &r, 8);
        break;
      }
      case O_ITOF: {
        double r = (double)(int32_t)(uint32_t)R[I->a];
        memcpy(&R[I->dst], &r, 8);
        break;
      }
      case O_FTOI: {
        double x;
        memcpy(&x, &R[I->a], 8);
        const int w = I->w;
        const double lo = w == 32 ? -2147483648.0 : -9223372036854775808.0;
        const double hi = w == 32 ? 2147483648.0 : 9223372036854775808.0; /* first value above the range */
        int64_t v;
        if (x != x) v = 0;
        else if (x <= lo) v = w == 32 ? (int64_t)INT32_MIN : INT64_MIN;
        else if (x >= hi) v = w == 32 ? (int64_t)INT32_MAX : INT64_MAX;
        else v = (int64_t)x; /* truncation toward zero */
        R[I->dst] = narrow((uint64_t)v, w);
        break;
      }
      case O_BARRIER:
        break; /* phases are driven by run_block */
      case O_ACCESS:
      case O_STORE:
      case O_LOAD: {
        if (t->dry && I->w == 32 && !read32_ok(R[I->a])) t->wrapped = 1;
        int64_t idx = (int64_t)narrow(R[I->a], I->w);
        unsigned log2e = I->op == O_LOAD ? I->d : (I->d & 3u);
        const or_alloc* A = &t->table[I->c];
        uint32_t kind = check_kind(A, idx, log2e);
        /* the tripwire model reports a subset of the exact violations; a
         * LOAD outside exact bounds reads 0 under either model */
        int reported = kind != 0 && (t->detector == DET_EXACT || kind == K_NULL ||
                                     tripwire_catches(t, I->c, idx, log2e));
        if (!t->dry) {
          t->st->accesses_checked++;
          t->acc_seen[I->b] = 1;
        }
        visit(t, I->s0);
        if (reported) record(t, I->b, kind, idx);
        const int shared = P->space[I->c] == SP_SHARED;
        if (I->op == O_LOAD) {
          uint64_t v = 0;
          if (!kind && shared) {
            /* the block's instance as at the start of the phase (0 in a
             * vertex run, which has no block) */
            if (!t->dry && t->sh_cur[I->c] && (uint64_t)idx < t->sh_n[I->c])
              v = (uint64_t)(int64_t)t->sh_cur[I->c][idx];
          } else if (!kind) {
            if (log2e == 2) v = (uint64_t)(int64_t)((const int32_t*)A->data)[idx];
            else v = (uint64_t)((const int64_t*)A->data)[idx];
          }
          R[I->dst] = v;
        } else if (I->op == O_STORE && !kind && shared && log2e == 2 && !t->dry && t->sh_next[I->c] &&
                   (uint64_t)idx < t->sh_n[I->c]) {
          const uint64_t packed = (1ull << 32) | (uint32_t)((uint32_t)R[I->dst] ^ 0x80000000u);
          if (packed > t->sh_next[I->c][idx]) t->sh_next[I->c][idx] = packed;
        }
        break;
      }
      case O_IF: {
        int taken = R[I->a] != 0;
        if (t->dry) {
          decide(t, (uint64_t)taken);
          if (t->stopped) return;
        }
        if (taken) {
          visit(t, I->s0);
          exec_range(t, pc + 1, I->alt >= 0 ? I->alt : I->end);
        } else {
          visit(t, I->s1);
          if (I->alt >= 0) exec_range(t, I->alt + 1, I->end);
        }
        pc = I->end; /* continue after ENDIF */
        break;
      }
      case O_LOOP:
        exec_one_loop(t, pc);
        pc = I->end;
        break;
      case O_ELSE: case O_ENDIF: case O_ENDLOOP:
        break; /* reached only as range ends */
      default:
        if (t->dry && P->in_slice[pc]) check_wrap(t, I, R[I->a], R[I->b]);
        R[I->dst] = alu(I->op, I->w, R[I->a], R[I->b], t->dry ? &t->dummy_faults : &t->st->arith_faults);
        break;
    }
    pc++;
  }
}

/* Coordinates of thread (blin, tlin) of the launch. */
static void thread_coords(thr* t, uint64_t blin, uint32_t tlin) {
  const uint32_t* L = t->launch;
  uint32_t gx = L[0], gy = L[1], bx = L[3], by = L[4];
  uint64_t bsize = (uint64_t)L[3] * L[4] * L[5];
  t->bid[0] = (uint32_t)(blin % gx);
  t->bid[1] = (uint32_t)((blin / gx) % gy);
  t->bid[2] = (uint32_t)(blin / ((uint64_t)gx * gy));
  t->tid[0] = tlin % bx;
  t->tid[1] = (tlin / bx) % by;
  t->tid[2] = tlin / (bx * by);
  t->gtid = blin * bsize + tlin;
}

/* Sets up thread (blin, tlin): coordinates, zero registers, a new lane. */
static void thread_begin(thr* t, uint64_t blin, uint32_t tlin) {
  thread_coords(t, blin, tlin);
  memset(t->regs, 0, sizeof(uint64_t) * (t->P->n_regs + 1));
  t->iter[0] = t->iter[1] = 0;
  t->stopped = 0;
  if (!t->dry) t->st->lanes++;
}

static void run_thread(thr* t, uint64_t blin, uint32_t tlin) {
  thread_begin(t, blin, tlin);
  exec_range(t, 0, t->P->n_instr);
}

/* The threads tl[0..n) of block blin run together, phase by phase: every
 * thread runs the program up to the next BARRIER (or the end), in thread
 * order, before any thread goes on; the block's shared memory starts at 0,
 * loads see it as at the start of the phase, and at the end of the phase each
 * element written takes the largest value stored to it (the IR's shared
 * memory semantics). */
static void run_block(thr* t, uint64_t blin, const uint32_t* tl, uint32_t n) {
  const or_prog* P = t->P;
  const size_t nr = (size_t)P->n_regs + 1;
  uint64_t* saved = (uint64_t*)calloc((size_t)n * nr, 8);
  uint8_t* stopped = (uint8_t*)calloc(n, 1);
  for (int s = 0; s < 16; s++) {
    t->sh_cur[s] = NULL; t->sh_next[s] = NULL; t->sh_n[s] = 0;
    if (s < P->n_slots && P->space[s] == SP_SHARED && t->table[s].base != 0) {
      t->sh_n[s] = t->table[s].size_bytes / 4;
      t->sh_cur[s] = (int32_t*)calloc(t->sh_n[s] + 1, 4);
      t->sh_next[s] = (uint64_t*)calloc(t->sh_n[s] + 1, 8);
    }
  }
  for (uint32_t k = 0; k < n; k++) thread_begin(t, blin, tl[k]); /* lanes; registers start at 0 */
  int pc = 0;
  for (;;) {
    int end = pc;
    while (end < P->n_instr && P->ins[end].op != O_BARRIER) end++;
    for (uint32_t k = 0; k < n; k++) {
      thread_coords(t, blin, tl[k]);
      memcpy(t->regs, saved + k * nr, nr * 8);
      t->iter[0] = t->iter[1] = 0;
      t->stopped = stopped[k];
      exec_range(t, pc, end);
      if (end < P->n_instr && !t->stopped && t->executed) { /* the BARRIER itself */
        t->executed[0]++;
        if (P->kept[end]) t->executed[1]++;
      }
      memcpy(saved + k * nr, t->regs, nr * 8);
      stopped[k] = (uint8_t)t->stopped;
    }
    for (int s = 0; s < 16; s++)
      for (uint64_t e = 0; e < t->sh_n[s]; e++)
        if (t->sh_next[s][e]) {
          t->sh_cur[s][e] = (int32_t)((uint32_t)t->sh_next[s][e] ^ 0x80000000u);
          t->sh_next[s][e] = 0;
        }
    if (end >= P->n_instr) break;
    pc = end + 1;
  }
  for (int s = 0; s < 16; s++) {
    free(t->sh_cur[s]); free(t->sh_next[s]);
    t->sh_cur[s] = NULL; t->sh_next[s] = NULL; t->sh_n[s] = 0;
  }
  free(saved); free(stopped);
}

/* All threads of block blin. */
static void run_whole_block(thr* t, uint64_t blin, uint32_t bsize) {
  if (!t->P->block_sync) {
    for (uint32_t tl = 0; tl < bsize; tl++) run_thread(t, blin, tl);
    return;
  }
  uint32_t* tl = (uint32_t*)malloc(sizeof(uint32_t) * bsize);
  for (uint32_t k = 0; k < bsize; k++) tl[k] = k;
  run_block(t, blin, tl, bsize);
  free(tl);
}

/* A block is a boundary block when, along some grid dimension of extent at
 * least 2, its coordinate is the first or the last one.  A dimension of extent
 * 1 has no boundary of its own (otherwise every block of a 2-D grid would be a
 * boundary block): the set is the perimeter of the grid in the dimensions it
 * actually spans. */
static int is_boundary_block(const uint32_t* L, uint64_t blin) {
  uint32_t gx = L[0], gy = L[1], gz = L[2];
  uint32_t x = (uint32_t)(blin % gx), y = (uint32_t)((blin / gx) % gy), z = (uint32_t)(blin / ((uint64_t)gx * gy));
  return (gx >= 2 && (x == 0 || x == gx - 1)) || (gy >= 2 && (y == 0 || y == gy - 1)) ||
         (gz >= 2 && (z == 0 || z == gz - 1));
}

/* Vertices of the box of block and thread coordinates: per dimension the
 * first and the last coordinate (one when the extent is 1). */
static int n_vertices(const uint32_t* L) {
  int tot = 1;
  for (int d = 0; d < 6; d++) tot *= L[d] == 1 ? 1 : 2;
  return tot;
}
/* Vertex v in global-thread-id order: block coordinates outermost (z, y, x),
 * then thread coordinates (z, y, x). */
static void vertex(const uint32_t* L, int tot, int v, uint64_t* blin, uint32_t* tlin) {
  uint32_t c[6];
  int rem = v, div = tot;
  const int order[6] = {2, 1, 0, 5, 4, 3}; /* bz by bx tz ty tx (gx..gz = 0..2, bx..bz = 3..5) */
  for (int o = 0; o < 6; o++) {
    int d = order[o];
    int cnt = L[d] == 1 ? 1 : 2;
    div /= cnt;
    int digit = rem / div;
    rem %= div;
    c[d] = digit ? L[d] - 1 : 0;
  }
  *blin = c[0] + (uint64_t)L[0] * (c[1] + (uint64_t)L[1] * c[2]);
  *tlin = c[3] + L[3] * (c[4] + L[4] * c[5]);
}

/* The rep-exact flag of a representative mode (the reading of the Theorem's
 * exact-integer premise, Section 5.1.1): run every vertex thread without
 * recording anything; the flag holds when they all take vertex 0's control
 * decisions within the budget and no slice operation wraps at any of them.
 * Then every intermediate of an affine index is affine over the whole box in
 * exact integers (an affine function on a box is extremal at a vertex), so no
 * interior thread wraps either. */
static uint32_t vertex_exact(thr* t) {
  const uint32_t* L = t->launch;
  if ((uint64_t)L[0] * L[1] * L[2] == 0 || (uint64_t)L[3] * L[4] * L[5] == 0) return 0;
  /* indices that depend on other threads' shared-memory writes: no vertex
   * argument applies */
  if (t->P->shared_idx) return 0;
  int tot = n_vertices(L);
  t->dry = 1; t->wrapped = 0; t->abort_run = 0;
  t->dec = (uint64_t*)malloc(sizeof(uint64_t) * (VERTEX_BUDGET + 1));
  t->ndec = 0;
  for (int v = 0; v < tot && !t->abort_run && !t->wrapped; v++) {
    uint64_t blin; uint32_t tlin;
    vertex(L, tot, v, &blin, &tlin);
    t->recording = v == 0;
    t->pos = 0;
    t->budget = 0;
    run_thread(t, blin, tlin);
    if (v > 0 && t->pos != t->ndec) t->abort_run = 1;
  }
  uint32_t ok = !t->abort_run && !t->wrapped;
  free(t->dec); t->dec = NULL;
  t->dry = 0;
  return ok;
}

/* One input under the chosen thread set. */
static void run_input(thr* t, uint32_t mode) {
  const uint32_t* L = t->launch;
  uint64_t nblocks = (uint64_t)L[0] * L[1] * L[2];
  uint32_t bsize = L[3] * L[4] * L[5];
  if (nblocks == 0 || bsize == 0) return;
  if (mode == M_FULL) {
    /* The whole grid: what the paper executes for kernels that are not
     * affine-access (Section 5.1, fall-back to all blocks and threads). */
    for (uint64_t b = 0; b < nblocks; b++) run_whole_block(t, b, bsize);
  } else if (mode == M_CORNERS) {
    /* The PREX Theorem's representative threads {first, last thread} x
     * {first, last block} (Section 5.1.1), taken per dimension: every vertex
     * of the box of block and thread coordinates. */
    int tot = n_vertices(L);
    if (!t->P->block_sync) {
      for (int v = 0; v < tot; v++) {
        uint64_t blin; uint32_t tlin;
        vertex(L, tot, v, &blin, &tlin);
        run_thread(t, blin, tlin);
      }
    } else {
      /* vertices of one block are consecutive: they run together */
      uint32_t tl[64];
      uint64_t cur = 0;
      uint32_t n = 0;
      for (int v = 0; v < tot; v++) {
        uint64_t blin; uint32_t tlin;
        vertex(L, tot, v, &blin, &tlin);
        if (n && blin != cur) { run_block(t, cur, tl, n); n = 0; }
        cur = blin;
        tl[n++] = tlin;
      }
      if (n) run_block(t, cur, tl, n);
    }
  } else if (mode == M_BOUNDARY) {
    /* Every block on the faces of the grid plus the middle block, all of
     * their threads (the blocks the PREX runtime prioritises, Section 5.1.2,
     * plus one interior representative). */
    uint64_t centre = (uint64_t)(L[0] / 2) + (uint64_t)L[0] * ((L[1] / 2) + (uint64_t)L[1] * (L[2] / 2));
    for (uint64_t b = 0; b < nblocks; b++)
      if (is_boundary_block(L, b) || b == centre) run_whole_block(t, b, bsize);
  } else if (mode == M_PREX) {
    /* Algorithm 1 (PREX runtime): blocks are taken from both ends of the
     * block order inward, head then tail, and the sweep stops before a new
     * pair once every memory-access instruction of the program has executed
     * (the runtime's "coverage is 100%") or a violation has been seen.  A
     * single middle block (head == tail) runs once. */
    uint64_t head = 0, tail = nblocks - 1;
    for (;;) {
      if (head > tail) break;
      int covered = 1, bug = 0;
      for (int a = 0; a < t->P->n_accesses; a++) if (!t->acc_seen[a]) { covered = 0; break; }
      for (int a = 0; a < t->P->n_accesses; a++) if (t->rec[a].count) { bug = 1; break; }
      if (covered || bug) break;
      run_whole_block(t, head, bsize);
      if (tail != head) run_whole_block(t, tail, bsize);
      head++;
      if (tail == 0) break;
      tail--;
    }
  }
}

/* ---- batch driver ------------------------------------------------------- */
typedef struct {
  const or_prog* P;
  uint32_t n_inputs;
  const uint32_t* launch;
  const int64_t* scalars;
  const or_alloc* tables;     /* concatenated */
  const uint64_t* table_off;  /* [n_inputs] first entry of each input's table */
  const uint32_t* table_len;  /* [n_inputs] entries of each input's table */
  uint32_t mode, detector;
  unsigned L1, L2;
  uint64_t cap[2];
  or_record* recs;
  uint64_t* counts;
  or_status* st;
  uint64_t* executed; /* [n_inputs][2] or NULL */
  int nthreads, me;
} job_t;

static void* worker(void* arg) {
  job_t* J = (job_t*)arg;
  const or_prog* P = J->P;
  thr t;
  memset(&t, 0, sizeof t);
  t.P = P;
  t.regs = (uint64_t*)calloc(P->n_regs + 1, 8);
  t.acc_seen = (uint8_t*)calloc(P->n_accesses + 1, 1);
  t.L1 = J->L1; t.L2 = J->L2; t.cap[0] = J->cap[0]; t.cap[1] = J->cap[1];
  int64_t zero_scalars[16] = {0};
  for (uint32_t i = (uint32_t)J->me; i < J->n_inputs; i += (uint32_t)J->nthreads) {
    t.launch = J->launch + 6 * (size_t)i;
    t.scalars = P->n_scalars ? J->scalars + (size_t)P->n_scalars * i : zero_scalars;
    t.table = J->tables + J->table_off[i];
    t.table_n = J->table_len[i];
    t.executed = J->executed ? J->executed + 2 * (size_t)i : NULL;
    t.detector = J->detector;
    t.rec = J->recs + (size_t)P->n_accesses * i;
    t.cnt = J->counts + (size_t)P->n_sites * i;
    t.st = J->st + i;
    memset(t.acc_seen, 0, P->n_accesses + 1);
    if (J->mode != M_FULL) t.st->flags = vertex_exact(&t) ? 1u : 0u;
    run_input(&t, J->mode);
  }
  free(t.regs);
  free(t.acc_seen);
  return NULL;
}

/* Public entry: check n_inputs inputs of one program.
 *   launch   [n_inputs][6]  gx gy gz bx by bz
 *   scalars  [n_inputs][n_scalars]
 *   tables   concatenated allocation tables; input i's table starts at
 *            table_off[i] and has table_len[i] >= n_slots entries
 *   mode     0 whole grid, 1 corner threads, 2 boundary blocks, 3 PREX sweep
 *   detector 0 exact bounds, 1 tripwire (redzones)
 *   cap_log2 trip caps 2^cap_log2[d] for loops at depth d+1
 *   recs     [n_inputs][n_accesses] out; counts [n_inputs][n_sites] out (u64);
 *   maps     [n_inputs][65536] out or NULL; st [n_inputs] out
 * Returns 0, or a negative code (-1 invalid arguments, -2 bad IR, -3 key range). */
int ckco_check(const uint8_t* ir, size_t ir_bytes, uint32_t n_inputs, const uint32_t* launch,
               const int64_t* scalars, const or_alloc* tables, const uint64_t* table_off,
               const uint32_t* table_len, uint32_t mode, uint32_t detector, const uint32_t* cap_log2,
               or_record* recs, uint64_t* counts, uint8_t* maps, or_status* st, int nthreads,
               uint64_t* executed) {
  or_prog P;
  int rc = prog_decode(ir, ir_bytes, &P);
  if (rc) return rc;
  if (mode > M_PREX || detector > DET_TRIPWIRE || cap_log2[0] > 32 || cap_log2[1] > 32) {
    prog_free(&P);
    return E_INVALID;
  }
  unsigned L1 = P.max_depth >= 1 ? cap_log2[0] : 0;
  unsigned L2 = P.max_depth >= 2 ? cap_log2[1] : 0;
  for (uint32_t i = 0; i < n_inputs; i++) {
    const uint32_t* L = launch + 6 * (size_t)i;
    if (table_len[i] < (uint32_t)P.n_slots) { prog_free(&P); return E_INVALID; }
    for (int s = 0; s < P.n_slots; s++) {
      const or_alloc* A = tables + table_off[i] + s;
      if (P.load_slot[s] && A->base != 0 && !(A->flags & A_FREED) && A->data == NULL && A->size_bytes > 0) {
        prog_free(&P); return E_INVALID;
      }
    }
    /* the tripwire model needs every allocation with its redzones inside
     * [0, 2^63] */
    if (detector == DET_TRIPWIRE)
      for (uint32_t k = 0; k < table_len[i]; k++) {
        const or_alloc* A = tables + table_off[i] + k;
        if (A->base == 0) continue;
        if (A->base < A->redzone ||
            (unsigned __int128)A->base + A->size_bytes + A->redzone > ((unsigned __int128)1 << 63)) {
          prog_free(&P);
          return E_INVALID;
        }
      }
    unsigned __int128 nthr = (unsigned __int128)L[0] * L[1] * L[2] * ((uint64_t)L[3] * L[4] * L[5]);
    if ((uint64_t)L[3] * L[4] * L[5] > 1024 || (uint64_t)L[0] * L[1] * L[2] > 0xFFFFFFFFull) { prog_free(&P); return E_INVALID; }
    if (nthr > 0 && L1 + L2 > 0) {
      unsigned __int128 lim = (unsigned __int128)1 << (64 - L1 - L2);
      if (nthr > lim) { prog_free(&P); return E_RANGE; }
    }
  }
  for (size_t k = 0; k < (size_t)n_inputs * P.n_accesses; k++) {
    recs[k].first_key = UINT64_MAX; recs[k].index = 0; recs[k].count = 0; recs[k].kinds = 0; recs[k].first_kind = 0;
  }
  memset(counts, 0, sizeof(uint64_t) * (size_t)n_inputs * P.n_sites);
  memset(st, 0, sizeof(or_status) * n_inputs);
  if (executed) memset(executed, 0, sizeof(uint64_t) * 2 * n_inputs);
  if (nthreads < 1) nthreads = 1;
  if ((uint32_t)nthreads > n_inputs && n_inputs > 0) nthreads = (int)n_inputs;
  job_t* jobs = (job_t*)calloc(nthreads, sizeof(job_t));
  pthread_t* th = (pthread_t*)calloc(nthreads, sizeof(pthread_t));
  for (int k = 0; k < nthreads; k++) {
    job_t* J = &jobs[k];
    J->P = &P; J->n_inputs = n_inputs; J->launch = launch; J->scalars = scalars;
    J->tables = tables; J->table_off = table_off; J->table_len = table_len; J->mode = mode;
    J->detector = detector; J->L1 = L1; J->L2 = L2; J->executed = executed;
    J->cap[0] = 1ull << cap_log2[0]; J->cap[1] = 1ull << cap_log2[1];
    J->recs = recs; J->counts = counts; J->st = st; J->nthreads = nthreads; J->me = k;
  }
  if (nthreads == 1) worker(&jobs[0]);
  else {
    for (int k = 0; k < nthreads; k++) pthread_create(&th[k], NULL, worker, &jobs[k]);
    for (int k = 0; k < nthreads; k++) pthread_join(th[k], NULL);
  }
  if (maps) {
    memset(maps, 0, (size_t)n_inputs * 65536);
    for (uint32_t i = 0; i < n_inputs; i++)
      for (int s = 0; s < P.n_sites; s++) {
        uint64_t c = counts[(size_t)i * P.n_sites + s];
        maps[(size_t)i * 65536 + P.site_ids[s]] = (uint8_t)(c > 255 ? 255 : c);
      }
  }
  free(jobs); free(th);
  prog_free(&P);
  return E_OK;
}

/* Decode-only entry: 0 if the IR is well formed, else -2.  Fills
 * n_accesses/n_sites/max_depth when out != NULL. */
int ckco_validate(const uint8_t* ir, size_t ir_bytes, int32_t* out) {
  or_prog P;
  int rc = prog_decode(ir, ir_bytes, &P);
  if (rc) return rc;
  if (out) { out[0] = P.n_accesses; out[1] = P.n_sites; out[2] = P.max_depth; out[3] = P.n_slots; }
  prog_free(&P);
  return E_OK;
}

/* ---- closed-loop fuzzing ------------------------------------------------
 * The campaign loop of a coverage-guided fuzzer (Section 2.1): take an input
 * from the corpus, mutate it, execute it, keep it when it reaches coverage
 * not seen before, and note the inputs that trigger a memory bug.  Readings
 * (listed in the design notes):
 *   - one generation checks `batch` children; child c of generation g draws
 *     its random numbers from SplitMix64 in counter form,
 *     r(k) = mix(seed + (((g * batch + c) * 64 + k) + 1) * 0x9E3779B97F4A7C15);
 *   - the child copies corpus entry r(0) mod |corpus| (corpus as at the
 *     generation's start) and applies 1 + r(1) mod max_stack mutations, the
 *     j-th drawing r(2+4j) .. r(5+4j);
 *   - coverage maps are bucketed by hit count as AFL does (1, 2, 3, 4-7,
 *     8-15, 16-31, 32-127, 128+ -> one bit each); a child is novel when its
 *     bucketed map shares a bit with the virgin map as it was at the start of
 *     the generation; afterwards every bit of every child's bucketed map is
 *     cleared from the virgin map, and novel children join the corpus in child
 *     order while it has room;
 *   - a child "crashes" when any of its records has a violation; for each
 *     (access, kind) the first (generation, child) that reported it is kept. */
#define FZ_GOLDEN 0x9E3779B97F4A7C15ull
#define MUT_LAUNCH 1u
#define MUT_SCALAR 2u
#define MUT_DATA 4u

/* SplitMix64 (Steele, Lea and Flood, 2014): output k of the generator
 * started at `seed`. */
static uint64_t fz_rand(uint64_t seed, uint64_t k) {
  uint64_t z = seed + (k + 1) * FZ_GOLDEN;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

/* the values a mutation may substitute for a scalar or an element: zero, one,
 * minus one and the edges of power-of-two ranges */
static const int64_t FZ_SPECIAL[28] = {
  0, 1, -1, 2, 7, 8, 15, 16, 31, 32, 63, 64, 127, 128, 255, 256, 1023, 1024, 4095, 4096,
  65535, 65536, 2147483647, -2147483647 - 1, 4294967295ll, 4294967296ll, INT64_MIN, INT64_MAX};

/* AFL's hit-count classes */
static uint8_t fz_class(uint8_t v) {
  if (v == 0) return 0;
  if (v == 1) return 1;
  if (v == 2) return 2;
  if (v == 3) return 4;
  if (v <= 7) return 8;
  if (v <= 15) return 16;
  if (v <= 31) return 32;
  if (v <= 127) return 64;
  return 128;
}

typedef struct {
  uint32_t batch, max_stack, max_block, corpus_cap, data_slot, ops, n_scalars;
  uint64_t max_threads, seed;
  uint64_t n_elems; /* int32 elements of the mutated data slot (0: none) */
} fz_cfg;

/* One mutation of a child (launch[6], scalars[16], data[n_elems]). */
static void fz_mutate(const fz_cfg* C, uint32_t* L, int64_t* S, int32_t* D, uint64_t u0, uint64_t u1, uint64_t u2) {
  uint32_t ops[3], n = 0;
  if (C->ops & MUT_LAUNCH) ops[n++] = MUT_LAUNCH;
  if ((C->ops & MUT_SCALAR) && C->n_scalars) ops[n++] = MUT_SCALAR;
  if ((C->ops & MUT_DATA) && C->n_elems) ops[n++] = MUT_DATA;
  if (n == 0) return;
  const uint32_t op = ops[u0 % n];
  const uint32_t kind = (uint32_t)((u1 >> 8) % 4);
  if (op == MUT_LAUNCH) {
    const uint32_t d = (uint32_t)(u1 % 6);
    uint64_t v = L[d];
    switch (kind) {
      case 0: v = v + 1 + u2 % 8; break;
      case 1: { uint64_t dv = 1 + u2 % 8; v = v > dv ? v - dv : 1; break; }
      case 2: v = 1ull << (u2 % 11); break;
      default: v = 1 + u2 % 256; break;
    }
    uint32_t M[6];
    memcpy(M, L, sizeof M);
    M[d] = (uint32_t)v;
    const uint64_t bs = (uint64_t)M[3] * M[4] * M[5], nb = (uint64_t)M[0] * M[1] * M[2];
    /* a child stays inside the campaign's bounds, else the mutation is void */
    if (v >= 1 && v <= 0xFFFFFFFFull && bs <= C->max_block && nb <= 0xFFFFFFFFull &&
        (unsigned __int128)nb * bs <= C->max_threads)
      L[d] = (uint32_t)v;
  } else if (op == MUT_SCALAR) {
    const uint32_t k = (uint32_t)(u1 % C->n_scalars);
    switch (kind) {
      case 0: S[k] = (int64_t)((uint64_t)S[k] ^ (1ull << (u2 % 64))); break;
      case 1: S[k] = (int64_t)((uint64_t)S[k] + (uint64_t)((int64_t)(u2 % 33) - 16)); break;
      case 2: S[k] = FZ_SPECIAL[u2 % 28]; break;
      default: S[k] = (int64_t)u2; break;
    }
  } else {
    const uint64_t e = u1 % C->n_elems;
    switch (kind) {
      case 0: D[e] = (int32_t)(uint32_t)((uint32_t)D[e] + (uint32_t)((int32_t)(u2 % 33) - 16)); break;
      case 1: D[e] = (int32_t)(uint32_t)(uint64_t)FZ_SPECIAL[u2 % 28]; break;
      case 2: D[e] = (int32_t)(uint32_t)u2; break;
      default: D[e] = (int32_t)((uint32_t)D[e] ^ (1u << (u2 % 32))); break;
    }
  }
}

/* A fuzzing campaign of `generations` generations from one seed input.
 *   cfg      batch, max_stack, max_threads, max_block, corpus_cap, data_slot
 *            (>= 16: none), ops (MUT_* bits), seed, generations
 *   corpus   out: c_launch [corpus_cap][6], c_scalars [corpus_cap][16],
 *            c_data [corpus_cap][n_elems] (when a data slot is mutated),
 *            c_gen [corpus_cap] (generation that added it; the seed: 0 with
 *            c_size counting it), c_size [1]
 *   virgin   out [65536]; sigs out [n_accesses][4] (generation << 32 | child,
 *            UINT64_MAX if never); stats out [4]: execs, novel children, crashing
 *            children, generations
 * Returns 0 or a negative code. */
int ckco_fuzz(const uint8_t* ir, size_t ir_bytes, const uint32_t* seed_launch, const int64_t* seed_scalars,
              const or_alloc* table, uint32_t table_len, uint32_t mode, uint32_t detector,
              const uint32_t* cap_log2, const uint64_t* cfg, uint32_t* c_launch, int64_t* c_scalars,
              int32_t* c_data, uint32_t* c_gen, uint32_t* c_size, uint8_t* virgin, uint64_t* sigs,
              uint64_t* stats, int nthreads) {
  or_prog P;
  int rc = prog_decode(ir, ir_bytes, &P);
  if (rc) return rc;
  fz_cfg C;
  C.batch = (uint32_t)cfg[0]; C.max_stack = (uint32_t)cfg[1]; C.max_threads = cfg[2];
  C.max_block = (uint32_t)cfg[3]; C.corpus_cap = (uint32_t)cfg[4]; C.data_slot = (uint32_t)cfg[5];
  C.ops = (uint32_t)cfg[6]; C.seed = cfg[7];
  const uint64_t G = cfg[8];
  C.n_scalars = (uint32_t)P.n_scalars;
  C.n_elems = C.data_slot < table_len && table[C.data_slot].data ? table[C.data_slot].size_bytes / 4 : 0;
  const int n_acc = P.n_accesses, n_sites = P.n_sites;
  prog_free(&P);
  if (C.batch == 0 || C.max_stack == 0 || C.corpus_cap == 0 || C.max_block == 0 || C.max_block > 1024 ||
      table_len == 0 || table_len > 16 || mode > M_BOUNDARY)
    return E_INVALID;
  {
    const uint64_t bs = (uint64_t)seed_launch[3] * seed_launch[4] * seed_launch[5];
    const uint64_t nb = (uint64_t)seed_launch[0] * seed_launch[1] * seed_launch[2];
    if (C.max_stack > 15 || bs == 0 || nb == 0 || bs > C.max_block || (unsigned __int128)nb * bs > C.max_threads)
      return E_INVALID; /* the seed itself must respect the campaign's bounds */
  }
  const uint64_t ne = C.n_elems;
  /* corpus: the seed input */
  memcpy(c_launch, seed_launch, 6 * sizeof(uint32_t));
  memset(c_scalars, 0, 16 * sizeof(int64_t) * (size_t)C.corpus_cap);
  for (uint32_t s = 0; s < C.n_scalars; s++) c_scalars[s] = seed_scalars[s];
  if (ne) memcpy(c_data, table[C.data_slot].data, ne * 4);
  c_gen[0] = 0;
  uint32_t size = 1;
  memset(virgin, 0xFF, 65536);
  for (int k = 0; k < n_acc * 4; k++) sigs[k] = UINT64_MAX;
  memset(stats, 0, 4 * sizeof(uint64_t));
  /* children of one generation */
  const uint32_t B = C.batch;
  uint32_t* launch = (uint32_t*)malloc(sizeof(uint32_t) * 6 * B);
  int64_t* scal = (int64_t*)calloc((size_t)B * (C.n_scalars ? C.n_scalars : 1), sizeof(int64_t));
  int32_t* data = (int32_t*)malloc(4 * (ne ? ne : 1) * B);
  or_alloc* tabs = (or_alloc*)malloc(sizeof(or_alloc) * table_len * B);
  uint64_t* toff = (uint64_t*)malloc(sizeof(uint64_t) * B);
  uint32_t* tlen = (uint32_t*)malloc(sizeof(uint32_t) * B);
  or_record* recs = (or_record*)malloc(sizeof(or_record) * (size_t)B * (n_acc ? n_acc : 1));
  uint64_t* counts = (uint64_t*)malloc(sizeof(uint64_t) * (size_t)B * (n_sites ? n_sites : 1));
  uint8_t* maps = (uint8_t*)malloc((size_t)B * 65536);
  or_status* st = (or_status*)malloc(sizeof(or_status) * B);
  uint8_t* novel = (uint8_t*)malloc(B);
  uint8_t* seen = (uint8_t*)malloc(65536);
  int64_t S[16];
  rc = E_OK;
  for (uint64_t g = 0; g < G && rc == E_OK; g++) {
    for (uint32_t c = 0; c < B; c++) {
      const uint64_t base = ((g * B + c) * 64);
      const uint32_t p = (uint32_t)(fz_rand(C.seed, base + 0) % size);
      uint32_t* L = launch + 6 * (size_t)c;
      memcpy(L, c_launch + 6 * (size_t)p, 6 * sizeof(uint32_t));
      memcpy(S, c_scalars + 16 * (size_t)p, sizeof S);
      int32_t* D = data + ne * c;
      if (ne) memcpy(D, c_data + ne * p, ne * 4);
      const uint32_t m = 1 + (uint32_t)(fz_rand(C.seed, base + 1) % C.max_stack);
      for (uint32_t j = 0; j < m; j++)
        fz_mutate(&C, L, S, D, fz_rand(C.seed, base + 2 + 4 * j), fz_rand(C.seed, base + 3 + 4 * j),
                  fz_rand(C.seed, base + 4 + 4 * j));
      for (uint32_t s = 0; s < C.n_scalars; s++) scal[(size_t)c * C.n_scalars + s] = S[s];
      memcpy(tabs + (size_t)c * table_len, table, sizeof(or_alloc) * table_len);
      if (ne) tabs[(size_t)c * table_len + C.data_slot].data = D;
      toff[c] = (uint64_t)c * table_len;
      tlen[c] = table_len;
    }
    rc = ckco_check(ir, ir_bytes, B, launch, scal, tabs, toff, tlen, mode, detector, cap_log2, recs, counts, maps,
                    st, nthreads, NULL);
    if (rc) break;
    /* novelty against the virgin map as at the generation's start */
    memset(seen, 0, 65536);
    for (uint32_t c = 0; c < B; c++) {
      const uint8_t* M = maps + (size_t)c * 65536;
      int nv = 0;
      for (int i = 0; i < 65536; i++) {
        const uint8_t b = fz_class(M[i]);
        if (b & virgin[i]) nv = 1;
        seen[i] |= b;
      }
      novel[c] = (uint8_t)nv;
      int crash = 0;
      for (int a = 0; a < n_acc; a++) {
        const or_record* R = &recs[(size_t)c * n_acc + a];
        if (!R->count) continue;
        crash = 1;
        for (int k = 0; k < 4; k++)
          if (R->kinds & (1u << k)) {
            const uint64_t tag = (g << 32) | c;
            if (tag < sigs[a * 4 + k]) sigs[a * 4 + k] = tag;
          }
      }
      stats[1] += nv;
      stats[2] += crash;
    }
    for (int i = 0; i < 65536; i++) virgin[i] &= (uint8_t)~seen[i];
    for (uint32_t c = 0; c < B && size < C.corpus_cap; c++) {
      if (!novel[c]) continue;
      memcpy(c_launch + 6 * (size_t)size, launch + 6 * (size_t)c, 6 * sizeof(uint32_t));
      for (uint32_t s = 0; s < 16; s++)
        c_scalars[16 * (size_t)size + s] = s < C.n_scalars ? scal[(size_t)c * C.n_scalars + s] : 0;
      if (ne) memcpy(c_data + ne * size, data + ne * c, ne * 4);
      c_gen[size] = (uint32_t)g;
      size++;
    }
    stats[0] += B;
    stats[3]++;
  }
  *c_size = size;
  free(launch); free(scal); free(data); free(tabs); free(toff); free(tlen); free(recs); free(counts);
  free(maps); free(st); free(novel); free(seen);
  return rc;
}

/* Output k of the campaign's generator for `seed` (for tests). */
uint64_t ckco_fuzz_rand(uint64_t seed, uint64_t k) { return fz_rand(seed, k); }

/* The hit-count class of a map byte (for tests). */
uint32_t ckco_fuzz_class(uint32_t v) { return fz_class((uint8_t)v); }

/* FEXP as the IR defines it (for tests). */
double ckco_ir_exp(double x) { return ir_exp(x); }
