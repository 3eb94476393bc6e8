// dev_plan.h — planning (thread sets, per-input traces, tile scan), work schedules, finishing (totals, dense maps).
// Part of the device code of libckc; included by kernels.hip only (one
// translation unit, no relocatable device code).
#pragma once

namespace ckc {

// ---------------------------------------------------------------------------
// plan: thread-set sizes and per-input traces of uniform-control programs
// ---------------------------------------------------------------------------
__device__ __forceinline__ const dins* prog_ins(const dprog* p) {
  return (const dins*)((const uint8_t*)p + p->off_instr);
}
__device__ __forceinline__ const int64_t* prog_consts(const dprog* p) {
  return (const int64_t*)((const uint8_t*)p + p->off_consts);
}
__device__ __forceinline__ const daccess* prog_access(const dprog* p) {
  return (const daccess*)((const uint8_t*)p + p->off_access);
}
__device__ __forceinline__ const uint16_t* prog_sites(const dprog* p) {
  return (const uint16_t*)((const uint8_t*)p + p->off_sites);
}

// Symbolic register file of the planning wavefront in LDS: register r of
// lane j is RG[r * 64 + j] (64 bits).
#define RGET64(i) RG[(uint32_t)(i) * 64u + j]
#define RSET(i, v) (RG[(uint32_t)(i) * 64u + j] = (uint64_t)(v))

__device__ __forceinline__ uint64_t readlane64(uint64_t v, int l) {
  const uint32_t h = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(v >> 32), l);
  const uint32_t w = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v, l);
  return ((uint64_t)h << 32) | w;
}

// Symbolic evaluation of a uniform-control program for one input.  Lane j of
// the wavefront holds coefficient j (tid.x, tid.y, tid.z, bid.x, bid.y, bid.z)
// and lane 6 the thread-invariant part of every register.  Sites, accesses and
// faults are counted per thread (every thread performs the same sequence).
__device__ void build_trace(const dprog* P, const dinput& in, const int64_t* sc, const ckc_alloc* tab,
                            dtrace_head* th, dtrace_entry* te, uint32_t* visits,
                            ckc_input_status* st, uint64_t* RG) {
  const uint32_t j = lane_id();
  const dins* I = prog_ins(P);
  const int64_t* K = prog_consts(P);
  for (uint32_t r = 0; r < P->n_regs; r++) RSET(r, 0ull);
  uint32_t n_ent = 0, n_cls = 0, overflow = 0, hang = 0, any_dead = 0;
  uint64_t acc_per_thread = 0, faults_per_thread = 0;
  __shared__ int64_t cls_coef[MAX_CLASSES][6];
  __shared__ uint32_t cls_w[MAX_CLASSES];
  uint64_t k[2] = {0, 0}, run[2] = {0, 0}, lstart[2] = {0, 0}, lstep[2] = {0, 0};
  uint32_t lhang[2] = {0, 0};
  const uint32_t L2 = in.L2;
  const uint32_t n = P->n_instr;
  const uint32_t cap_log2_0 = in.cap_log2[0], cap_log2_1 = in.cap_log2[1];
  uint32_t pc = 0;
  auto visit = [&](uint32_t s) {
    if (s != NOSITE && j == 0 && visits[s] < 255u) visits[s] += 1;  // only min(255, .) is observable
  };
  while (pc < n && !hang && !overflow) {
    const dins D = I[pc];
    const uint32_t op = D.op, w = D.w;
    switch (op) {
      case CKC_OP_CONST: RSET(D.dst, j == 6 ? narrow((uint64_t)K[D.x], w) : 0ull); break;
      case CKC_OP_SCALAR: RSET(D.dst, j == 6 ? narrow((uint64_t)sc[D.x], w) : 0ull); break;
      case CKC_OP_SPECIAL: {
        uint64_t v = 0;
        if (D.x < 6) v = (j == D.x) ? 1ull : 0ull;
        else if (j == 6) v = D.x < 9 ? in.launch[3 + (D.x - 6)] : in.launch[D.x - 9];
        RSET(D.dst, v);
        break;
      }
      case CKC_OP_ADD: case CKC_OP_SUB: {
        uint64_t a = RGET64(D.a), b = RGET64(D.b);
        RSET(D.dst, narrow(op == CKC_OP_ADD ? a + b : a - b, w));
        break;
      }
      case CKC_OP_MUL: case CKC_OP_SHL: {
        uint64_t a = RGET64(D.a), b = RGET64(D.b);
        bool b_uni = __ballot(j < 6 && b != 0) == 0;
        uint64_t r;
        if (op == CKC_OP_SHL) {
          uint64_t amt = readlane64(b, 6) & (uint64_t)(w - 1);
          r = a << amt;
        } else if (b_uni) {
          r = a * readlane64(b, 6);
        } else {
          r = b * readlane64(a, 6);
        }
        RSET(D.dst, narrow(r, w));
        break;
      }
      case CKC_OP_TRUNC: RSET(D.dst, narrow(RGET64(D.a), 32)); break;
      case CKC_OP_SEXT: RSET(D.dst, j == 6 ? narrow(RGET64(D.a), 32) : 0ull); break;
      case CKC_OP_ZEXT: RSET(D.dst, j == 6 ? (RGET64(D.a) & 0xFFFFFFFFull) : 0ull); break;
      case CKC_OP_SELECT: {
        uint64_t c = readlane64(RGET64(D.a), 6);
        RSET(D.dst, narrow(c != 0 ? RGET64(D.b) : RGET64(D.c), w));
        break;
      }
      case CKC_OP_ACCESS: case CKC_OP_LOAD: {
        uint64_t v = RGET64(D.a);
        const ckc_alloc A = tab[D.slot];
        uint32_t lg = D.fl & 3u;
        // coefficient vector of this index (wrapped to the access width)
        uint64_t cw = narrow(v, w);
        int64_t coef[6];
#pragma unroll
        for (int d = 0; d < 6; d++) coef[d] = (int64_t)readlane64(cw, d);
        int64_t off = (int64_t)readlane64(cw, 6);
        int cls = -1;
        for (uint32_t c = 0; c < n_cls; c++) {
          bool same = cls_w[c] == w;
          for (int d = 0; d < 6; d++) same = same && cls_coef[c][d] == coef[d];
          if (same) { cls = (int)c; break; }
        }
        if (cls < 0) {
          if (n_cls == MAX_CLASSES) { overflow = 1; break; }
          cls = (int)n_cls++;
          for (int d = 0; d < 6; d++) cls_coef[cls][d] = coef[d];
          cls_w[cls] = w;
        }
        if (n_ent >= P->trace_cap) { overflow = 1; break; }
        if (j == 0) {
          const uint32_t cap8 = (P->trace_cap + 7u) & ~7u;
          int64_t* h64 = (int64_t*)(th + 1);
          uint32_t* h32 = (uint32_t*)(h64 + 2 * (size_t)cap8);
          dtrace_entry E;
          E.off = off;
          E.keylo = (k[0] << L2) | k[1];
          uint64_t lim = w == 32 ? (1ull << 31) : (1ull << 63);
          uint64_t nel = A.size_bytes >> lg;
          E.bound = nel < lim ? nel : lim;
          E.acc = D.x;
          E.cls = (uint8_t)cls;
          E.w = (uint8_t)w;
          E.dead_kind = A.base == 0 ? CKC_KIND_NULL : ((A.flags & CKC_ALLOC_FREED) ? CKC_KIND_FREED : 0);
          E.pad = 0;
          te[n_ent] = E;
          h64[2 * n_ent] = off;
          h64[2 * n_ent + 1] = (int64_t)E.bound;
          h32[2 * n_ent] = (uint32_t)off;
          h32[2 * n_ent + 1] = (uint32_t)E.bound;
          if (E.dead_kind) any_dead = 1;
        }
        n_ent++;
        acc_per_thread++;
        visit(D.s0);
        if (op == CKC_OP_LOAD) {
          // a LOAD whose value is used has a thread-invariant index here
          uint64_t val = 0;
          uint32_t kd = kind_of(A.base, A.size_bytes, A.flags, off, lg);
          bool uni_idx = __ballot(j < 6 && v != 0) == 0;
          if (!kd && uni_idx && A.data) {
            val = lg == 2 ? (uint64_t)(int64_t)((const int32_t*)A.data)[off]
                          : (uint64_t)((const int64_t*)A.data)[off];
          }
          RSET(D.dst, j == 6 ? val : 0ull);
        }
        break;
      }
      case CKC_OP_IF: {
        uint64_t c = readlane64(RGET64(D.a), 6);
        if (c != 0) {
          visit(D.s0);
        } else {
          visit(D.s1);
          pc = D.jmp;  // ELSE (its arm follows) or ENDIF
        }
        break;
      }
      case CKC_OP_ELSE: pc = D.jmp; break;  // end of the taken arm: skip to ENDIF
      case CKC_OP_ENDIF: break;
      case CKC_OP_LOOP: {
        uint32_t d = D.x;
        int64_t s = (int64_t)narrow(readlane64(RGET64(D.a), 6), w);
        int64_t e = (int64_t)narrow(readlane64(RGET64(D.b), 6), w);
        int64_t stp = (int64_t)narrow(readlane64(RGET64(D.c), 6), w);
        uint64_t nt = trip_count(s, e, stp);
        uint64_t cap = 1ull << (d == 0 ? cap_log2_0 : cap_log2_1);
        uint64_t rn = nt < cap ? nt : cap;
        if (d == 0) { run[0] = rn; lstart[0] = (uint64_t)s; lstep[0] = (uint64_t)stp; lhang[0] = nt > cap; k[0] = 0; }
        else { run[1] = rn; lstart[1] = (uint64_t)s; lstep[1] = (uint64_t)stp; lhang[1] = nt > cap; k[1] = 0; }
        if (rn == 0) {
          if (nt > cap) { hang = 1; break; }  // cap 2^k >= 1, unreachable
          visit(D.s1);
          pc = D.jmp;  // ENDLOOP; continue after it
          break;
        }
        RSET(D.dst, j == 6 ? narrow((uint64_t)s, w) : 0ull);
        visit(D.s0);
        break;
      }
      case CKC_OP_ENDLOOP: {
        uint32_t d = D.x;
        const dins Lp = I[D.jmp];
        uint64_t kk = (d == 0 ? k[0] : k[1]) + 1;
        uint64_t rn = d == 0 ? run[0] : run[1];
        if (kk < rn) {
          if (d == 0) k[0] = kk; else k[1] = kk;
          uint64_t s0 = d == 0 ? lstart[0] : lstart[1], st0 = d == 0 ? lstep[0] : lstep[1];
          RSET(Lp.dst, j == 6 ? narrow(s0 + kk * st0, Lp.w) : 0ull);
          visit(Lp.s0);
          pc = D.jmp;  // back to the LOOP; body follows
        } else {
          if (d == 0) k[0] = 0; else k[1] = 0;
          if (d == 0 ? lhang[0] : lhang[1]) { hang = 1; break; }
          visit(Lp.s1);
        }
        break;
      }
      default: {
        // remaining ops only see thread-invariant operands here
        uint32_t f = 0;
        uint64_t r = alu(op, w, readlane64(RGET64(D.a), 6), readlane64(RGET64(D.b), 6), f);
        faults_per_thread += f;
        RSET(D.dst, j == 6 ? r : 0ull);
        break;
      }
    }
    pc++;
  }
  if (j == 0) {
    th->n_entries = n_ent;
    th->n_classes = n_cls;
    th->overflow = overflow;
    th->hang = hang;
    th->any_dead = any_dead;
    th->cap8 = (P->trace_cap + 7u) & ~7u;
    for (uint32_t c = 0; c < n_cls; c++) {
      for (int d = 0; d < 6; d++) th->coef[c][d] = cls_coef[c][d];
      th->cls_w[c] = (uint8_t)cls_w[c];
    }
    st->accesses_checked = acc_per_thread;
    st->arith_faults = faults_per_thread;
    st->hang_lanes = hang;
  }
}

// ---------------------------------------------------------------------------
// Vertex-exact flag of the representative modes (the exact-integer premise
// of the Section 5.1.1 Theorem): the vertex threads of the (grid x block) box
// run the lowered program in lockstep, one lane each, with concrete values in
// the LDS register file.  The flag is set when they take the same control
// decisions (IF outcomes, exact loop trip counts; at most 2^16 decisions and
// iterations in all) and no slice operation wraps at any of them.
// ---------------------------------------------------------------------------
constexpr uint32_t VERTEX_BUDGET = 65536;

__device__ __forceinline__ bool fits32(uint64_t c) { return (uint64_t)((int64_t)c + (1ll << 31)) < (1ull << 32); }

// Exact signed result of ADD/SUB/MUL/SHL/DIVS at width w outside its range,
// or a width-32 operand outside int32.
__device__ __forceinline__ bool op_wraps(uint32_t op, uint32_t w, uint64_t x, uint64_t y) {
  const bool bin = op >= CKC_OP_ADD && op <= CKC_OP_CMPLEU;
  if (w == 32 && (!fits32(x) || (bin && !fits32(y)))) return true;
  const int64_t sx = (int64_t)narrow(x, w), sy = (int64_t)narrow(y, w);
  if (w == 32) {
    int64_t r;
    switch (op) {
      case CKC_OP_ADD: r = sx + sy; break;
      case CKC_OP_SUB: r = sx - sy; break;
      case CKC_OP_MUL: r = sx * sy; break;  // |operands| <= 2^31: no 64-bit overflow
      case CKC_OP_SHL: r = sx * (int64_t)(1ll << ((uint32_t)sy & 31u)); break;  // |r| < 2^62
      case CKC_OP_DIVS: return sx == INT32_MIN && sy == -1;
      default: return false;
    }
    return !fits32((uint64_t)r);
  }
  switch (op) {
    case CKC_OP_ADD: { int64_t r; return __builtin_add_overflow(sx, sy, &r); }
    case CKC_OP_SUB: { int64_t r; return __builtin_sub_overflow(sx, sy, &r); }
    case CKC_OP_MUL: { int64_t r; return __builtin_mul_overflow(sx, sy, &r); }
    case CKC_OP_SHL: {
      const uint32_t sh = (uint32_t)sy & 63u;
      if (sx == 0 || sh == 0) return false;
      // exact x * 2^sh fits in int64 iff the top sh+1 bits of x are all equal
      const int64_t t = sx >> (63 - sh);
      return !(t == 0 || t == -1);
    }
    case CKC_OP_DIVS: return sx == INT64_MIN && sy == -1;
    default: return false;
  }
}

__device__ uint32_t vertex_flag(const dprog* P, const dinput& in, const int64_t* sc, const ckc_alloc* tab,
                                uint64_t* RG) {
  const uint32_t j = lane_id();
  const uint32_t* L = in.launch;
  uint32_t nv = 1;
  for (int d = 0; d < 6; d++) nv *= L[d] >= 2 ? 2u : 1u;
  if ((uint64_t)L[0] * L[1] * L[2] == 0 || (uint64_t)L[3] * L[4] * L[5] == 0) return 0;
  // indices that depend on other threads' shared-memory writes: no vertex
  // argument applies
  if (P->pflags & PF_CAPTURE) return 0;
  // lanes past the vertex count run vertex 0 again (a duplicate changes
  // nothing and keeps every lane's control decisions equal)
  // coordinates of vertex j: tid.xyz then bid.xyz, each first or last
  uint32_t crd[6];
  {
    uint32_t v = j < nv ? j : 0u;
    const int ord[6] = {3, 4, 5, 0, 1, 2};  // launch index of tid.x .. bid.z
#pragma unroll
    for (int d = 0; d < 6; d++) {
      const uint32_t e = L[ord[d]];
      if (e >= 2) {
        crd[d] = (v & 1u) ? e - 1 : 0u;
        v >>= 1;
      } else {
        crd[d] = 0;
      }
    }
  }
  const dins* I = prog_ins(P);
  const int64_t* K = prog_consts(P);
  for (uint32_t r = 0; r < P->n_regs; r++) RSET(r, 0ull);
  uint64_t k[2] = {0, 0}, run[2] = {0, 0}, lstart[2] = {0, 0}, lstep[2] = {0, 0};
  uint32_t lhang[2] = {0, 0}, lw[2] = {32, 32};
  uint32_t budget = 0;
  bool wrapped = false, abort_run = false;
  const uint32_t n = P->n_instr;
  uint32_t pc = 0;
  auto decide = [&](uint64_t v) {
    if (++budget > VERTEX_BUDGET) { abort_run = true; return; }
    const uint64_t lo = wave_min64(v), hi = ~wave_min64(~v);
    if (lo != hi) abort_run = true;
  };
  while (pc < n && !abort_run) {
    const dins D = I[pc];
    const uint32_t op = D.op, w = D.w;
    const bool sl = (D.fl & DI_SLICE) != 0;
    switch (op) {
      case CKC_OP_CONST: RSET(D.dst, narrow((uint64_t)K[D.x], w)); break;
      case CKC_OP_SCALAR: RSET(D.dst, narrow((uint64_t)sc[D.x], w)); break;
      case CKC_OP_SPECIAL:
        RSET(D.dst, (uint64_t)(D.x < 6 ? crd[D.x] : D.x < 9 ? L[3 + (D.x - 6)] : L[D.x - 9]));
        break;
      case CKC_OP_TRUNC: case CKC_OP_SEXT: {
        const uint64_t x = RGET64(D.a);
        if (sl && !fits32(x)) wrapped = true;
        RSET(D.dst, narrow(x, 32));
        break;
      }
      case CKC_OP_ZEXT: {
        const uint64_t x = RGET64(D.a);
        if (sl && !(fits32(x) && (int64_t)x >= 0)) wrapped = true;
        RSET(D.dst, x & 0xFFFFFFFFull);
        break;
      }
      case CKC_OP_SELECT: {
        const uint64_t v = RGET64(D.a) != 0 ? RGET64(D.b) : RGET64(D.c);
        if (sl && w == 32 && !fits32(v)) wrapped = true;
        RSET(D.dst, narrow(v, w));
        break;
      }
      case CKC_OP_FADD: case CKC_OP_FSUB: case CKC_OP_FMUL: case CKC_OP_FEXP: case CKC_OP_ITOF:
      case CKC_OP_FTOI:
        RSET(D.dst, float_op(op, w, RGET64(D.a), RGET64(D.b)));
        break;
      case CKC_OP_BARRIER: break;
      case CKC_OP_ACCESS: case CKC_OP_LOAD: case CKC_OP_STORE: {
        const uint64_t x = RGET64(D.a);
        if (w == 32 && !fits32(x)) wrapped = true;
        // shared memory holds nothing in a vertex run (no block runs)
        if (op == CKC_OP_LOAD && ((P->slot_spaces >> (2 * D.slot)) & 3u) == CKC_SPACE_SHARED) {
          RSET(D.dst, 0ull);
        } else if (op == CKC_OP_LOAD) {
          const ckc_alloc A = tab[D.slot];
          const uint32_t lg = D.fl & 3u;
          const int64_t idx = (int64_t)narrow(x, w);
          const uint32_t kd = kind_of(A.base, A.size_bytes, A.flags, idx, lg);
          uint64_t val = 0;
          if (!kd)
            val = lg == 2 ? (uint64_t)(int64_t)((const int32_t*)A.data)[idx] : (uint64_t)((const int64_t*)A.data)[idx];
          RSET(D.dst, val);
        }
        break;
      }
      case CKC_OP_IF: {
        const bool taken = RGET64(D.a) != 0;
        decide(taken ? 1ull : 0ull);
        if (abort_run) break;
        if (!__ballot(taken)) pc = D.jmp;  // ELSE (its arm follows) or ENDIF
        break;
      }
      case CKC_OP_ELSE: pc = D.jmp; break;
      case CKC_OP_ENDIF: break;
      case CKC_OP_LOOP: {
        const uint32_t d = D.x;
        const uint64_t xa = RGET64(D.a), xb = RGET64(D.b), xc = RGET64(D.c);
        if (w == 32 && (!fits32(xa) || !fits32(xb) || !fits32(xc))) wrapped = true;
        const int64_t s0 = (int64_t)narrow(xa, w), e0 = (int64_t)narrow(xb, w), st0 = (int64_t)narrow(xc, w);
        const uint64_t nt0 = trip_count(s0, e0, st0);
        decide(nt0);
        if (abort_run) break;
        const uint64_t nt = ufirst64(nt0);  // equal in every lane once decided
        const uint64_t cap = 1ull << (d == 0 ? in.cap_log2[0] : in.cap_log2[1]);
        const uint64_t rn = nt < cap ? nt : cap;
        run[d & 1] = rn; lstart[d & 1] = (uint64_t)s0; lstep[d & 1] = (uint64_t)st0;
        lhang[d & 1] = nt > cap; k[d & 1] = 0; lw[d & 1] = w;
        if (rn == 0) {
          pc = D.jmp;  // ENDLOOP; continue after it
          break;
        }
        if (++budget > VERTEX_BUDGET) { abort_run = true; break; }
        RSET(D.dst, narrow((uint64_t)s0, w));
        break;
      }
      case CKC_OP_ENDLOOP: {
        const uint32_t d = D.x & 1u;
        const dins Lp = I[D.jmp];
        const uint64_t kk = k[d] + 1;
        if (kk < run[d]) {
          if (++budget > VERTEX_BUDGET) { abort_run = true; break; }
          k[d] = kk;
          // the counter lies between start and end for every iteration below
          // the exact trip count, so it cannot leave the width's range
          RSET(Lp.dst, narrow(lstart[d] + kk * lstep[d], lw[d]));
          pc = D.jmp;
        } else {
          k[d] = 0;
          if (lhang[d]) pc = n;  // every vertex thread stops here
        }
        break;
      }
      default: {
        const uint64_t x = RGET64(D.a), y = RGET64(D.b);
        if (sl && op_wraps(op, w, x, y)) wrapped = true;
        uint32_t f = 0;
        RSET(D.dst, alu(op, w, x, y, f));
        break;
      }
    }
    if (pc >= n) break;
    pc++;
  }
  const bool bad = abort_run || __ballot(wrapped) != 0;
  return bad ? 0u : 1u;
}

__device__ __forceinline__ bool is_div_op(uint32_t op) {
  return op == CKC_OP_DIVS || op == CKC_OP_DIVU || op == CKC_OP_REMS || op == CKC_OP_REMU;
}

// State of the rows form's symbolic walk: each register's form (lane j < 7
// of the wavefront holds component j: the constant part, then the
// coefficients), the kind of its form and the width it is exact at, the last
// comparison of varying forms.
struct RowWalk {
  uint64_t sym[NREG][8];
  uint8_t var[NREG], wd[NREG];
  RForm pa, pb;
  uint32_t pop, pw;
};

// The symbolic walk of the rows form (one wavefront, once per input): lane 0
// holds a register's constant part, lanes 1..6 its coordinate coefficients
// (or lane 1 the coefficient of its loaded value).  A form is exact modulo
// 2^wd of the width of the operation that made it; it may feed operations
// and accesses of width at most wd.  G.ok is cleared when the part outside
// the loop body takes anything else (the loader flags PF_ROWS only for
// programs whose walk succeeds).
__device__ void build_rows(drows& G, RowWalk& Wk, const dprog* P, const int64_t* sc, const uint32_t* launch) {
  const uint32_t j = lane_id();
  const dins* I = prog_ins(P);
  const int64_t* K = prog_consts(P);
  auto rg = [&](uint32_t r) -> uint64_t& { return Wk.sym[r][j]; };  // lanes j < 7 only
  for (uint32_t r = j; r < NREG; r += 64) { Wk.var[r] = RV_UNI; Wk.wd[r] = 64; }
  uint32_t n = 0, n_load = 0, ok = P->expand_pc >= 0 ? 1u : 0u, preg = 0xFFu;
  auto form_of = [&](RForm& f, uint32_t r) {  // copy register r's form (lanes 0..6 write)
    const uint64_t v = j < 7 ? rg(r) : 0ull;
    if (j == 0) { f.off = (int64_t)v; f.var = Wk.var[r]; }
    else if (j < 7) f.c[j - 1] = (int64_t)v;
  };
  // a varying form may feed an operation of width w only if exact at w
  auto fits = [&](uint32_t r, uint32_t w) { return Wk.var[r] == RV_UNI || (Wk.var[r] != RV_PRED && Wk.wd[r] >= w); };
  const uint32_t npc = P->n_instr;
  for (uint32_t pc = 0; pc < npc && ok; pc++) {
    const dins D = I[pc];
    const uint32_t op = D.op, w = D.w;
    const uint32_t da = ufirst(D.a), db = ufirst(D.b), dc = ufirst(D.c), dd = ufirst(D.dst);
    const uint64_t a = j < 7 ? rg(da) : 0, b = j < 7 ? rg(db) : 0;
    const uint32_t va = Wk.var[da], vb = Wk.var[db];
    uint64_t r = 0;
    uint32_t rv = RV_UNI, rw = 64;
    bool wr = true;
    switch (op) {
      case CKC_OP_CONST: r = j == 0 ? narrow((uint64_t)K[D.x], w) : 0; break;
      case CKC_OP_SCALAR: r = j == 0 ? narrow((uint64_t)sc[D.x], w) : 0; break;
      case CKC_OP_SPECIAL:
        if (D.x < 6) {
          r = j == 1u + D.x ? 1ull : 0ull;
          rv = RV_COORD;
        } else {
          r = j == 0 ? (uint64_t)(D.x < 9 ? launch[3 + D.x - 6] : launch[D.x - 9]) : 0;
        }
        break;
      case CKC_OP_ADD: case CKC_OP_SUB:
        if ((va != RV_UNI && vb != RV_UNI && va != vb) || !fits(da, w) || !fits(db, w)) { ok = 0; break; }
        r = narrow(op == CKC_OP_ADD ? a + b : a - b, w);
        rv = va != RV_UNI ? va : vb;
        rw = rv == RV_UNI ? 64 : w;
        if (rv == RV_UNI && j != 0) r = 0;
        break;
      case CKC_OP_MUL:
        if ((va != RV_UNI && vb != RV_UNI) || !fits(da, w) || !fits(db, w)) { ok = 0; break; }
        r = narrow(va != RV_UNI ? a * readlane64(b, 0) : b * readlane64(a, 0), w);
        rv = va != RV_UNI ? va : vb;
        rw = rv == RV_UNI ? 64 : w;
        if (rv == RV_UNI) r = j == 0 ? narrow(readlane64(a, 0) * readlane64(b, 0), w) : 0;
        break;
      case CKC_OP_SHL:
        if (vb != RV_UNI || !fits(da, w)) { ok = 0; break; }
        r = narrow(a << (readlane64(b, 0) & (uint64_t)(w - 1)), w);
        rv = va;
        rw = rv == RV_UNI ? 64 : w;
        if (rv == RV_UNI && j != 0) r = 0;
        break;
      case CKC_OP_TRUNC:
        if (!fits(da, 32)) { ok = 0; break; }
        r = narrow(a, 32);
        rv = va;
        rw = rv == RV_UNI ? 64 : 32;
        if (rv == RV_UNI && j != 0) r = 0;
        break;
      case CKC_OP_SEXT:
        if (va != RV_UNI) { ok = 0; break; }
        r = j == 0 ? narrow(readlane64(a, 0), 32) : 0;
        break;
      case CKC_OP_ZEXT:
        if (va != RV_UNI) { ok = 0; break; }
        r = j == 0 ? (readlane64(a, 0) & 0xFFFFFFFFull) : 0;
        break;
      case CKC_OP_SELECT:
        if (va != RV_UNI || vb != RV_UNI || Wk.var[dc] != RV_UNI) { ok = 0; break; }
        r = j == 0 ? narrow(readlane64(a, 0) != 0 ? readlane64(b, 0) : readlane64(rg(dc), 0), w) : 0;
        break;
      case CKC_OP_ACCESS:
      case CKC_OP_LOAD: {
        if (n >= MAX_RENT || !fits(da, w) || (op == CKC_OP_LOAD && n_load >= RV_MAXLOAD)) { ok = 0; break; }
        REnt& E = G.e[n];
        form_of(E.a, da);
        if (j == 0) {
          E.kind = op == CKC_OP_LOAD ? RE_LOAD : RE_ACCESS;
          E.w = (uint8_t)w;
          E.acc = D.x;
          E.s0 = D.s0;
          E.slot = D.slot;
          E.lg = D.fl & 3u;
          E.dst = op == CKC_OP_LOAD ? (uint8_t)(n_load + 1) : 0;
        }
        n++;
        if (op == CKC_OP_LOAD) {
          n_load++;
          r = j == 1 ? 1ull : 0ull;
          rv = n_load;
        } else {
          wr = false;
        }
        break;
      }
      case CKC_OP_IF: {
        if (n >= MAX_RENT) { ok = 0; break; }
        REnt& E = G.e[n];
        if (va == RV_PRED) {
          if (da != preg) { ok = 0; break; }
          if (j == 0) { E.a = Wk.pa; E.b = Wk.pb; E.op = (uint8_t)Wk.pop; E.w = (uint8_t)Wk.pw; }
        } else {
          // IF tests the register's 64-bit value: a form exact at wd is
          // nonzero exactly when its value modulo 2^wd is
          form_of(E.a, da);
          if (j == 0) {
            E.b.off = 0;
            E.b.var = RV_UNI;
            E.op = CKC_OP_CMPNE;
            E.w = (uint8_t)(va == RV_UNI ? 64u : Wk.wd[da]);
          }
        }
        if (j == 0) { E.kind = RE_GUARD; E.s0 = D.s0; E.s1 = D.s1; }
        n++;
        wr = false;
        break;
      }
      case CKC_OP_ENDIF:
        if (n >= MAX_RENT) { ok = 0; break; }
        if (j == 0) G.e[n].kind = RE_ENDG;
        n++;
        wr = false;
        break;
      case CKC_OP_LOOP: {
        const uint32_t nl = P->n_livein;
        if (n >= MAX_RENT || (int32_t)pc != P->expand_pc || !fits(da, w) || !fits(db, w) ||
            Wk.var[dc] != RV_UNI) { ok = 0; break; }
        for (uint32_t q = 0; q < nl; q++)
          if (Wk.var[ufirst(P->livein[q])] != RV_UNI) ok = 0;
        if (!ok) break;
        REnt& E = G.e[n];
        form_of(E.a, da);
        form_of(E.b, db);
        const uint64_t stp = narrow(readlane64(rg(dc), 0), w);
        for (uint32_t q = 0; q < nl; q++) {
          const uint64_t v = readlane64(rg(ufirst(P->livein[q])), 0);
          if (j == 0) G.livein[q] = v;
        }
        if (j == 0) {
          E.kind = RE_LOOP;
          E.w = (uint8_t)w;
          E.step = stp;
          E.s1 = D.s1;
        }
        n++;
        wr = false;
        pc = D.jmp;  // the body is the gather pass's; continue after ENDLOOP
        break;
      }
      default: {
        if (op >= CKC_OP_CMPEQ && op <= CKC_OP_CMPLEU && (va != RV_UNI || vb != RV_UNI)) {
          // a comparison of varying forms: only an IF may read it
          if (!fits(da, w) || !fits(db, w)) { ok = 0; break; }
          form_of(Wk.pa, da);
          form_of(Wk.pb, db);
          if (j == 0) { Wk.pop = op; Wk.pw = w; }
          preg = dd;
          rv = RV_PRED;
          r = 0;
          break;
        }
        if (op < CKC_OP_ADD || op > CKC_OP_CMPLEU || is_div_op(op) || va != RV_UNI || vb != RV_UNI) {
          ok = 0;
          break;
        }
        uint32_t f = 0;
        const uint64_t v = alu(op, w, readlane64(a, 0), readlane64(b, 0), f);
        r = j == 0 ? v : 0;
        break;
      }
    }
    if (ok && wr) {
      if (j < 7) rg(dd) = r;
      if (j == 0) { Wk.var[dd] = (uint8_t)rv; Wk.wd[dd] = (uint8_t)rw; }
    }
    // lanes exchange values through LDS: keep the order of the iterations
    __builtin_amdgcn_wave_barrier();
  }
  if (j == 0) {
    // coordinate classes: equal coefficient vectors share one per-lane sum
    uint32_t ncls = 0;
    for (uint32_t q = 0; q < n; q++) {
      RForm* fs[2] = {&G.e[q].a, &G.e[q].b};
      const uint32_t nf = G.e[q].kind == RE_GUARD || G.e[q].kind == RE_LOOP ? 2u : 1u;
      for (uint32_t h = 0; h < nf; h++) {
        RForm& f = *fs[h];
        f.cls = RCLS_NONE;
        if (f.var != RV_COORD) continue;
        for (uint32_t k = 0; k < ncls && f.cls == RCLS_NONE; k++) {
          bool same = true;
          for (int d = 0; d < 6; d++) same = same && G.cc[k][d] == f.c[d];
          if (same) f.cls = (uint8_t)k;
        }
        if (f.cls == RCLS_NONE && ncls < MAX_RCLS) {
          for (int d = 0; d < 6; d++) G.cc[ncls][d] = f.c[d];
          f.cls = (uint8_t)ncls++;
        }
      }
    }
    G.ncls = ncls;
    uint32_t all32 = 1;
    for (uint32_t q = 0; q < n; q++)
      if (G.e[q].kind != RE_ENDG && G.e[q].w != 32) all32 = 0;
    G.all32 = all32;
    G.n = n;
    G.ok = ok;
  }
}

__global__ void __launch_bounds__(64, 4) plan_kernel(KArgs a) {
  extern __shared__ uint64_t RG[];  // [max_regs][64]: symbolic registers of build_trace
  __shared__ RowWalk rw;            // the rows form's walk
  __shared__ drows rf;
  const uint32_t i = blockIdx.x;
  if (i >= a.n_inputs) return;
  dinput& in = a.inputs[i];
  const dprog* P = (const dprog*)in.prog;
  const uint32_t j = threadIdx.x;
  // records: no violation yet
  ckc_record* rec = a.recs + in.rec_base;
  for (uint32_t r = j; r < P->n_accesses; r += 64) {
    ckc_record z;
    z.first_key = ~0ull; z.index = 0; z.count = 0; z.kinds = 0; z.first_kind = 0;
    rec[r] = z;
  }
  uint32_t* cnt = a.counts + in.cnt_base;
  for (uint32_t s = j; s < P->n_sites; s += 64) cnt[s] = 0;
  if (in.xstate)  // expanded tiles start with no iterations
    for (uint64_t q = j; q < in.n_xt; q += 64) {
      a.xtot[in.xt_begin + q] = 0;
      a.xpb[in.xt_begin + q] = 0;
      a.xpg[in.xt_begin + q] = 0;
    }
  uint64_t lanes = set_lanes(in.mode, in.launch, in.aux);
  bool trace = (P->cls & CKC_CLS_UNIFORM) && !a.force_generic && in.trace != 0 && lanes > 0 && !in.detector;
  __syncthreads();
  ckc_input_status* st = a.status + i;
  if (j == 0) {
    st->lanes = lanes; st->accesses_checked = 0; st->hang_lanes = 0; st->arith_faults = 0;
    st->flags = 0; st->pad = 0;
  }
  // the flag of the representative modes; a PREX sweep takes it from its
  // first round
  if (in.mode == CKC_REP_CORNERS || in.mode == CKC_REP_BOUNDARY || (in.mode == MODE_PAIR && in.aux == 0)) {
    const uint32_t f = vertex_flag(P, in, a.scalars + (size_t)i * MAX_SCALARS, (const ckc_alloc*)in.table, RG);
    if (j == 0) st->flags = f;
    __syncthreads();
  }
  uint32_t path = 1;
  if (trace) {
    dtrace_head* th = (dtrace_head*)in.trace;
    const uint32_t cap8 = (P->trace_cap + 7u) & ~7u;
    dtrace_entry* te = (dtrace_entry*)((uint8_t*)(th + 1) + (size_t)cap8 * 24);
    build_trace(P, in, a.scalars + (size_t)i * MAX_SCALARS, (const ckc_alloc*)in.table, th, te, cnt, st, RG);
    __syncthreads();
    path = th->overflow ? 1 : 0;
    if (path == 1) {  // fall back: undo the per-thread counts
      for (uint32_t s = j; s < P->n_sites; s += 64) cnt[s] = 0;
      if (j == 0) { st->accesses_checked = 0; st->arith_faults = 0; st->hang_lanes = 0; }
    }
  }
  if ((P->pflags & PF_ROWS) && !(P->cls & CKC_CLS_UNIFORM) && in.trace != 0 && !in.detector && lanes > 0) {
    // the rows form of the input's whole-thread part, once for all its tiles
    build_rows(rf, rw, P, a.scalars + (size_t)i * MAX_SCALARS, in.launch);
    __syncthreads();
    uint4* dst = (uint4*)in.trace;
    const uint4* src = (const uint4*)&rf;
    for (uint32_t q = j; q < sizeof(drows) / 16; q += 64) dst[q] = src[q];
  }
  if (j == 0) {
    uint64_t tiles = (lanes + TILE - 1) / TILE;
    const uint32_t bs = in.launch[3] * in.launch[4] * in.launch[5];
    if (path == 0) {
      if ((in.mode == CKC_FULL || in.mode == CKC_REP_BOUNDARY) && bs % 64u == 0 &&
          ((const dtrace_head*)in.trace)->n_classes == 1) {
        // block-major jobs: (64-thread slice position, ngj groups of LPB set blocks)
        const uint64_t nsb = in.mode == CKC_FULL ? (uint64_t)in.launch[0] * in.launch[1] * in.launch[2]
                                                 : bset_size(in.launch);
        const uint64_t ngroups = (nsb + LPB - 1) / LPB;
        const uint32_t ngj = in.mode == CKC_FULL ? NGJ_FULL : NGJ_SET;
        const uint64_t jobs = (uint64_t)(bs / 64u) * ((ngroups + ngj - 1) / ngj);
        tiles = (jobs + 3) / 4;
        path = PATH_BLOCKS;
        dtrace_head* th = (dtrace_head*)in.trace;
        dblk& B = th->blk;
        for (int q = 0; q < 6; q++) B.L[q] = in.launch[q];
        const uint32_t L0 = in.launch[0], L1 = in.launch[1], L3 = in.launch[3], L4 = in.launch[4];
        B.mode = in.mode;
        B.ngj = ngj;
        B.bs = bs;
        B.gxy = L0 * L1;
        B.bxy = L3 * L4;
        B.nsb = (uint32_t)nsb;
        B.ngroups = (uint32_t)ngroups;
        B.spb = bs / 64u;
        B.ne = th->n_entries;
        B.any_dead = th->any_dead;
        B.w = th->cls_w[0];
        B.Lsum = in.L1 + in.L2;
        B.n_acc = P->n_accesses;
        UDiv u = udiv_make(L0);
        B.m_gx = u.m; B.s_gx = u.s;
        u = udiv_make(L0 * L1);
        B.m_gxy = u.m; B.s_gxy = u.s;
        u = udiv_make(L3);
        B.m_bx = u.m; B.s_bx = u.s;
        u = udiv_make(L3 * L4);
        B.m_bxy = u.m; B.s_bxy = u.s;
        u = udiv_make(bs / 64u);
        B.m_spb = u.m; B.s_spb = u.s;
        B.proof = in.mode == CKC_FULL && in.aux == 1u ? 1u : 0u;
        for (int q = 0; q < 2; q++) B.pad[q] = 0;
        for (int q = 0; q < 6; q++) B.k[q] = th->coef[0][q];
        const uint64_t k3 = (uint64_t)B.k[3], k4 = (uint64_t)B.k[4], k5 = (uint64_t)B.k[5];
        B.d1 = k3;
        B.dy = k4 - k3 * (uint64_t)(L0 - 1);
        B.dz = k5 - k3 * (uint64_t)(L0 - 1) - k4 * (uint64_t)(L1 - 1);
        B.rec = (uint64_t)(a.recs + in.rec_base);
      } else {
        path = PATH_LANES;
      }
    }
    in.lanes = lanes;
    in.path = path;
    for (uint32_t q = 0; q < 3; q++) in.n_tiles[q] = q == path ? (uint32_t)tiles : 0u;
  }
}

// Exclusive prefix of per-input tile counts for the three evaluators, taken in
// tile-space order (a.order: position -> input).
__global__ void __launch_bounds__(1024) scan_kernel(KArgs a) {
  __shared__ unsigned long long part[3][1024 / 64];
  __shared__ unsigned long long carry[3];
  const uint32_t t = threadIdx.x;
  if (t < 3) carry[t] = 0;
  __syncthreads();
  for (uint32_t base = 0; base < a.n_inputs; base += 1024) {
    const uint32_t pos = base + t;
    const uint32_t i = pos < a.n_inputs ? a.order[pos] : 0u;
    uint64_t v[3], sc[3];
    for (int p = 0; p < 3; p++) {
      v[p] = pos < a.n_inputs ? a.inputs[i].n_tiles[p] : 0;
      sc[p] = v[p];
    }
    for (int o = 1; o < 64; o <<= 1)  // inclusive wavefront scan
      for (int p = 0; p < 3; p++) {
        const uint64_t u = __shfl_up((unsigned long long)sc[p], o, 64);
        if ((int)lane_id() >= o) sc[p] += u;
      }
    if (lane_id() == 63)
      for (int p = 0; p < 3; p++) part[p][t / 64] = sc[p];
    __syncthreads();
    uint64_t w[3] = {0, 0, 0}, c[3];
    for (int p = 0; p < 3; p++) {
      for (uint32_t q = 0; q < t / 64; q++) w[p] += part[p][q];
      c[p] = carry[p];
    }
    if (pos < a.n_inputs)
      for (int p = 0; p < 3; p++) a.inputs[i].tile_begin[p] = c[p] + w[p] + sc[p] - v[p];
    __syncthreads();
    if (t == 1023)
      for (int p = 0; p < 3; p++) carry[p] = c[p] + w[p] + sc[p];
    __syncthreads();
  }
  if (t < 3) {
    a.js->total_tiles[t] = carry[t];
    a.js->next_tile[t] = 0;
  }
}

// Position p (into a.order) of the input whose tiles hold t (t < total): the
// largest p with tile_begin[path] of input order[p] <= t, which always has
// tiles since the next position starts after t.
__device__ __forceinline__ uint32_t find_pos(const dinput* in, const uint32_t* order, uint32_t n, uint32_t path,
                                             uint64_t t) {
  uint32_t lo = 0, hi = n - 1;
  while (lo < hi) {
    uint32_t mid = lo + (hi - lo + 1) / 2;
    if (in[order[mid]].tile_begin[path] <= t) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

// Work distribution of a persistent evaluator over its `total` tiles: work
// items are runs of `chunk` consecutive tiles.  BLOCKED: workgroup g takes
// tiles [total*g/G, total*(g+1)/G); CYCLIC: items g, g+G, g+2G, ...;
// DYNAMIC and LPT: items from an atomic counter (LPT's tile space lists the
// inputs largest first).  sched_next is called by the whole workgroup and
// returns the same tile in every lane, ~0 when the workgroup is done.
template <uint32_t SK>
struct Sched {
  uint32_t chunk;
  uint64_t total, cur, end, item;
};
template <uint32_t SK>
__device__ __forceinline__ void sched_init(Sched<SK>& s, const KArgs& a, uint64_t total) {
  s.chunk = a.chunk ? a.chunk : 1u;
  s.total = total;
  const uint64_t G = gridDim.x, g = blockIdx.x;
  if (SK == CKC_SCHED_BLOCKED) {
    s.cur = total * g / G;
    s.end = total * (g + 1) / G;
  } else if (SK == CKC_SCHED_CYCLIC) {
    s.item = g;
    s.cur = g * s.chunk;
    s.end = s.cur + s.chunk < total ? s.cur + s.chunk : total;
  } else {
    s.cur = s.end = 0;
  }
}
template <uint32_t SK>
__device__ __forceinline__ uint64_t sched_next(Sched<SK>& s, unsigned long long* counter, unsigned long long* slot) {
  if (s.cur < s.end) return s.cur++;
  if (SK == CKC_SCHED_BLOCKED) return ~0ull;
  uint64_t item;
  if (SK == CKC_SCHED_CYCLIC) {
    s.item += gridDim.x;
    item = s.item;
  } else {
    __syncthreads();  // every wavefront has read the previous item
    if (threadIdx.x == 0) *slot = atomicAdd(counter, 1ull);
    __syncthreads();
    item = *slot;
  }
  const uint64_t b = item * s.chunk;
  if (b >= s.total) {
    s.cur = s.end = 0;
    return ~0ull;
  }
  s.cur = b + 1;
  s.end = b + s.chunk < s.total ? b + s.chunk : s.total;
  return b;
}
// The schedule a kernel instantiation is compiled for (LPT runs DYNAMIC over
// its own tile order).
constexpr uint32_t sched_impl(uint32_t k) {
  return k == CKC_SCHED_BLOCKED ? CKC_SCHED_BLOCKED : k == CKC_SCHED_CYCLIC ? CKC_SCHED_CYCLIC : CKC_SCHED_DYNAMIC;
}

// ---------------------------------------------------------------------------
// Per input: trace-path totals from per-thread counts, then the dense map.
__global__ void __launch_bounds__(256) finish_kernel(KArgs a) {
  const uint32_t i = blockIdx.x;
  if (i >= a.n_inputs) return;
  const dinput& in = a.inputs[i];
  const dprog* P = (const dprog*)in.prog;
  uint32_t* cnt = a.counts + in.cnt_base;
  const uint64_t lanes = in.lanes;
  if (in.path != PATH_GENERIC) {
    for (uint32_t s = threadIdx.x; s < P->n_sites; s += blockDim.x) {
      uint64_t v = (uint64_t)cnt[s] * lanes;
      cnt[s] = v > 255 ? 255u : (uint32_t)v;
    }
    if (threadIdx.x == 0) {
      ckc_input_status* st = a.status + i;
      st->accesses_checked *= lanes;
      st->arith_faults *= lanes;
      st->hang_lanes = st->hang_lanes ? lanes : 0;
    }
  }
  __syncthreads();
  if (a.maps) {
    uint4* m = (uint4*)(a.maps + (size_t)i * 65536);
    const uint4 z = {0, 0, 0, 0};
    for (uint32_t q = threadIdx.x; q < 65536 / 16; q += blockDim.x) m[q] = z;
    __syncthreads();
    const uint16_t* ids = prog_sites(P);
    uint8_t* mb = a.maps + (size_t)i * 65536;
    for (uint32_t s = threadIdx.x; s < P->n_map_sites; s += blockDim.x) {
      uint32_t c = cnt[s];
      mb[ids[s]] = (uint8_t)(c > 255 ? 255 : c);
    }
  }
}

// ---------------------------------------------------------------------------
// PREX sweep (Algorithm 1): initial state and the fold of one window of rounds
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(64) prex_init_kernel(PrexArgs p) {
  const uint32_t i = blockIdx.x;
  if (i >= p.n_real) return;
  const dinput& in = p.real_in[i];
  const dprog* P = (const dprog*)in.prog;
  const uint32_t j = threadIdx.x;
  ckc_record* rec = p.real_recs + in.rec_base;
  for (uint32_t r = j; r < P->n_accesses; r += 64) {
    ckc_record z;
    z.first_key = ~0ull; z.index = 0; z.count = 0; z.kinds = 0; z.first_kind = 0;
    rec[r] = z;
  }
  uint32_t* cnt = p.real_counts + in.cnt_base;
  for (uint32_t s = j; s < P->n_sites; s += 64) cnt[s] = 0;
  if (j == 0) {
    ckc_input_status* st = p.real_status + i;
    st->lanes = 0; st->accesses_checked = 0; st->hang_lanes = 0; st->arith_faults = 0;
    st->flags = 0; st->pad = 0;
    p.stopped[i] = 0;
  }
}

// One workgroup per item: the input's rounds of this window in round order.
// Before each round, the test of Algorithm 1: the sweep stops once every
// ACCESS/LOAD instruction has executed at least once (its site counter is
// nonzero; every access has a site, internal if the program gave none) or
// some access has violated.  A round's results are then added: counters as
// saturating sums (a trace-path round counts per thread, times its lanes),
// records by least first key, summed counts and OR of kinds (index and kind
// at the least key are filled afterwards by replaying that thread), status
// by sums.  The first round also carries the vertex flag.
__global__ void __launch_bounds__(256) prex_merge_kernel(PrexArgs p) {
  const uint32_t it = blockIdx.x;
  if (it >= p.n_items) return;
  const prex_item X = p.items[it];
  const dinput& in = p.real_in[X.real];
  const dprog* P = (const dprog*)in.prog;
  const dins* I = prog_ins(P);
  const daccess* A = prog_access(P);
  ckc_record* rr = p.real_recs + in.rec_base;
  uint32_t* rc = p.real_counts + in.cnt_base;
  ckc_input_status* rs = p.real_status + X.real;
  const uint32_t tid = threadIdx.x;
  __shared__ uint32_t stop;
  if (tid == 0) {
    stop = p.stopped[X.real];
    if (X.r0 == 0) rs->flags = p.vstatus[X.vbeg].flags;
  }
  __syncthreads();
  for (uint32_t k = 0; k < X.vcnt; k++) {
    if (stop) break;  // read after a barrier: the same in every lane
    int miss = 0, bug = 0;
    for (uint32_t q = tid; q < P->n_accesses; q += blockDim.x) {
      if (rc[I[A[q].pc].s0] == 0) miss = 1;
      if (rr[q].count != 0) bug = 1;
    }
    miss = __syncthreads_or(miss);
    bug = __syncthreads_or(bug);
    if (!miss || bug) {
      if (tid == 0) stop = 1;
      break;
    }
    const dinput& V = p.vin[X.vbeg + k];
    const bool per_thread = V.path != PATH_GENERIC;
    const uint64_t lanes = V.lanes;
    const uint32_t* vc = p.vcounts + V.cnt_base;
    for (uint32_t s = tid; s < P->n_sites; s += blockDim.x) {
      uint64_t c = vc[s];
      if (per_thread) c *= lanes;
      const uint64_t t = (uint64_t)rc[s] + (c < 255 ? c : 255);
      rc[s] = t < 255 ? (uint32_t)t : 255u;
    }
    const ckc_record* vr = p.vrecs + V.rec_base;
    for (uint32_t q = tid; q < P->n_accesses; q += blockDim.x) {
      const ckc_record v = vr[q];
      if (v.count == 0) continue;
      if (v.first_key < rr[q].first_key) rr[q].first_key = v.first_key;
      rr[q].count += v.count;
      rr[q].kinds |= v.kinds;
    }
    if (tid == 0) {
      const ckc_input_status& vs = p.vstatus[X.vbeg + k];
      rs->lanes += lanes;
      rs->accesses_checked += per_thread ? vs.accesses_checked * lanes : vs.accesses_checked;
      rs->arith_faults += per_thread ? vs.arith_faults * lanes : vs.arith_faults;
      rs->hang_lanes += per_thread ? (vs.hang_lanes ? lanes : 0ull) : vs.hang_lanes;
      if (X.r0 + k == X.last) stop = 1;  // every block has run
    }
    __syncthreads();  // the next round's test reads what this one wrote
  }
  __syncthreads();
  if (tid == 0) p.stopped[X.real] = stop;
}

}  // namespace ckc
