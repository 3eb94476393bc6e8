// dev_common.h — integer semantics of the IR, wavefront reductions, multiply-shift division, thread-set decoding.
// Part of the device code of libckc; included by kernels.hip only (one
// translation unit, no relocatable device code).
#pragma once

namespace ckc {

// ---------------------------------------------------------------------------
// integer semantics of the IR (ckc_ir.h)
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint64_t narrow(uint64_t v, uint32_t w) {
  return w == 32 ? (uint64_t)(int64_t)(int32_t)(uint32_t)v : v;
}

// Width 32 in 32-bit arithmetic: the low 32 bits of every result depend only
// on the low 32 bits of the operands, and a 32-bit signed quotient cannot
// overflow once INT32_MIN / -1 is taken apart; the result is sign-extended as
// every 32-bit value in a register is.
__device__ __forceinline__ uint64_t alu32(uint32_t op, uint32_t a, uint32_t b, uint32_t& faults) {
  const int32_t sa = (int32_t)a, sb = (int32_t)b;
  uint32_t r;
  switch (op) {
    case CKC_OP_ADD: r = a + b; break;
    case CKC_OP_SUB: r = a - b; break;
    case CKC_OP_MUL: r = a * b; break;
    case CKC_OP_DIVS:
      if (sb == 0) { faults++; r = 0; }
      else if (sa == INT32_MIN && sb == -1) r = (uint32_t)INT32_MIN;
      else r = (uint32_t)(sa / sb);
      break;
    case CKC_OP_REMS:
      if (sb == 0) { faults++; r = 0; }
      else if (sa == INT32_MIN && sb == -1) r = 0;
      else r = (uint32_t)(sa % sb);
      break;
    case CKC_OP_DIVU: if (b == 0) { faults++; r = 0; } else r = a / b; break;
    case CKC_OP_REMU: if (b == 0) { faults++; r = 0; } else r = a % b; break;
    case CKC_OP_AND: r = a & b; break;
    case CKC_OP_OR: r = a | b; break;
    case CKC_OP_XOR: r = a ^ b; break;
    case CKC_OP_SHL: r = a << (b & 31u); break;
    case CKC_OP_SHRA: r = (uint32_t)(sa >> (b & 31u)); break;
    case CKC_OP_SHRL: r = a >> (b & 31u); break;
    case CKC_OP_MINS: r = (uint32_t)(sa < sb ? sa : sb); break;
    case CKC_OP_MAXS: r = (uint32_t)(sa > sb ? sa : sb); break;
    case CKC_OP_MINU: r = a < b ? a : b; break;
    case CKC_OP_MAXU: r = a > b ? a : b; break;
    case CKC_OP_CMPEQ: r = a == b; break;
    case CKC_OP_CMPNE: r = a != b; break;
    case CKC_OP_CMPLTS: r = sa < sb; break;
    case CKC_OP_CMPLES: r = sa <= sb; break;
    case CKC_OP_CMPLTU: r = a < b; break;
    case CKC_OP_CMPLEU: r = a <= b; break;
    default: r = 0; break;
  }
  return (uint64_t)(int64_t)(int32_t)r;
}

__device__ __forceinline__ uint64_t alu(uint32_t op, uint32_t w, uint64_t x, uint64_t y, uint32_t& faults) {
  if (w == 32) return alu32(op, (uint32_t)x, (uint32_t)y, faults);
  const bool n32 = (w == 32);
  const uint64_t ux = n32 ? (uint64_t)(uint32_t)x : x;
  const uint64_t uy = n32 ? (uint64_t)(uint32_t)y : y;
  const int64_t sx = n32 ? (int64_t)(int32_t)(uint32_t)x : (int64_t)x;
  const int64_t sy = n32 ? (int64_t)(int32_t)(uint32_t)y : (int64_t)y;
  const int64_t smin = n32 ? (int64_t)INT32_MIN : INT64_MIN;
  const uint32_t sh = (uint32_t)(uy & (uint64_t)(w - 1));
  uint64_t r;
  switch (op) {
    case CKC_OP_ADD: r = ux + uy; break;
    case CKC_OP_SUB: r = ux - uy; break;
    case CKC_OP_MUL: r = ux * uy; break;
    case CKC_OP_DIVS:
      if (sy == 0) { faults++; r = 0; }
      else if (sx == smin && sy == -1) r = (uint64_t)smin;
      else r = (uint64_t)(sx / sy);
      break;
    case CKC_OP_REMS:
      if (sy == 0) { faults++; r = 0; }
      else if (sx == smin && sy == -1) r = 0;
      else r = (uint64_t)(sx % sy);
      break;
    case CKC_OP_DIVU: if (uy == 0) { faults++; r = 0; } else r = ux / uy; break;
    case CKC_OP_REMU: if (uy == 0) { faults++; r = 0; } else r = ux % uy; break;
    case CKC_OP_AND: r = ux & uy; break;
    case CKC_OP_OR: r = ux | uy; break;
    case CKC_OP_XOR: r = ux ^ uy; break;
    case CKC_OP_SHL: r = ux << sh; break;
    case CKC_OP_SHRA: r = (uint64_t)(sx >> sh); break;
    case CKC_OP_SHRL: r = ux >> sh; break;
    case CKC_OP_MINS: r = (uint64_t)(sx < sy ? sx : sy); break;
    case CKC_OP_MAXS: r = (uint64_t)(sx > sy ? sx : sy); break;
    case CKC_OP_MINU: r = ux < uy ? ux : uy; break;
    case CKC_OP_MAXU: r = ux > uy ? ux : uy; break;
    case CKC_OP_CMPEQ: r = ux == uy; break;
    case CKC_OP_CMPNE: r = ux != uy; break;
    case CKC_OP_CMPLTS: r = sx < sy; break;
    case CKC_OP_CMPLES: r = sx <= sy; break;
    case CKC_OP_CMPLTU: r = ux < uy; break;
    case CKC_OP_CMPLEU: r = ux <= uy; break;
    default: r = 0; break;
  }
  return narrow(r, w);
}

// Exact trip count of LOOP start,end,step (saturated at UINT64_MAX).
__device__ __forceinline__ uint64_t trip_count(int64_t s, int64_t e, int64_t st) {
  if (st >= 0) {
    if (!(s < e)) return 0;
    if (st == 0) return ~0ull;
    uint64_t span = (uint64_t)e - (uint64_t)s;
    if (st == 1) return span;  // the common unit step: no 64-bit division
    return span / (uint64_t)st + (span % (uint64_t)st != 0);
  }
  if (!(s > e)) return 0;
  uint64_t span = (uint64_t)s - (uint64_t)e, mag = 0ull - (uint64_t)st;
  return span / mag + (span % mag != 0);
}

// Kind of one access against its allocation (ASan-style exact bounds).
__device__ __forceinline__ uint32_t kind_of(uint64_t base, uint64_t size, uint32_t flags, int64_t idx,
                                            uint32_t lg) {
  if (base == 0) return CKC_KIND_NULL;
  if (flags & CKC_ALLOC_FREED) return CKC_KIND_FREED;
  if (idx < 0) return CKC_KIND_UNDER;
  return (uint64_t)idx >= (size >> lg) ? CKC_KIND_OVER : 0u;
}

// e^x by the IR's definition of FEXP: reduction by ln 2 split into a part
// of 29 significant bits (k times it is exact) and the rest (k = floor(x /
// ln 2 + 1/2)), the degree-13 Taylor polynomial of e^r in Horner form,
// scaling by 2^k (two steps below 2^-1022); each operation rounded on its own (no fused multiply-add), so
// the result is the same bit pattern on any IEEE binary64 machine.
__device__ __noinline__ double ir_exp(double x) {
#pragma clang fp contract(off)
  const double C[14] = {
      0x1.0000000000000p+0, 0x1.0000000000000p+0, 0x1.0000000000000p-1, 0x1.5555555555555p-3,
      0x1.5555555555555p-5, 0x1.1111111111111p-7, 0x1.6c16c16c16c17p-10, 0x1.a01a01a01a01ap-13,
      0x1.a01a01a01a01ap-16, 0x1.71de3a556c734p-19, 0x1.27e4fb7789f5cp-22, 0x1.ae64567f544e4p-26,
      0x1.1eed8eff8d898p-29, 0x1.6124613a86d09p-33};
  if (x != x) return x;
  if (x > 709.782712893384) return __longlong_as_double(0x7FF0000000000000ll);
  if (x < -745.1332191019412) return 0.0;
  const double k = floor(x * 0x1.71547652b82fep+0 + 0.5);
  const double r = (x - k * 0x1.62e42ff000000p-1) - k * -0x1.718432a1b0e26p-35;
  double p = C[13];
  for (int i = 12; i >= 0; i--) p = p * r + C[i];
  const int ki = (int)k;
  if (ki > 1023) return (p * __longlong_as_double((long long)(1023 + 1023) << 52)) * 2.0;
  if (ki >= -1022) return p * __longlong_as_double((long long)(ki + 1023) << 52);
  return (p * __longlong_as_double((long long)(ki + 1000 + 1023) << 52)) *
         __longlong_as_double((long long)(-1000 + 1023) << 52);
}

// Non-index arithmetic: FADD FSUB FMUL FEXP on IEEE binary64 bit patterns
// (round to nearest even; FEXP as ir_exp), ITOF of
// a width-32 value (exact), FTOI truncating toward zero to width w (NaN 0,
// out-of-range values saturated).
__device__ __forceinline__ uint64_t float_op(uint32_t op, uint32_t w, uint64_t x, uint64_t y) {
  const double a = __longlong_as_double((long long)x), b = __longlong_as_double((long long)y);
  switch (op) {
    case CKC_OP_FADD: return (uint64_t)__double_as_longlong(a + b);
    case CKC_OP_FSUB: return (uint64_t)__double_as_longlong(a - b);
    case CKC_OP_FMUL: return (uint64_t)__double_as_longlong(a * b);
    case CKC_OP_FEXP: return (uint64_t)__double_as_longlong(ir_exp(a));
    case CKC_OP_ITOF: return (uint64_t)__double_as_longlong((double)(int32_t)(uint32_t)x);
    default: {  // FTOI
      const double lo = w == 32 ? -2147483648.0 : -9223372036854775808.0;
      const double hi = w == 32 ? 2147483648.0 : 9223372036854775808.0;
      int64_t v;
      if (a != a) v = 0;
      else if (a <= lo) v = w == 32 ? (int64_t)INT32_MIN : INT64_MIN;
      else if (a >= hi) v = w == 32 ? (int64_t)INT32_MAX : INT64_MAX;
      else v = (int64_t)a;
      return w == 32 ? (uint64_t)(int64_t)(int32_t)(uint32_t)v : (uint64_t)v;
    }
  }
}

// The tripwire (redzone) detector model (CKC_TRIPWIRE), for an access out of
// its slot's exact bounds on a non-NULL slot: caught when one of its bytes
// falls in a redzone of a live allocation or in a freed allocation (with its
// redzones) of the slot's memory space, or, for shared and local slots, when
// it leaves that space's window [0, largest allocation end plus redzone).
// The byte address base + idx * 2^lg is an exact integer; every allocation and
// redzone lies in [0, 2^63] (checked at submission), so addresses are held
// plus 8 and clamped to [-8, 2^63] + 8 in 64 bits: below -8 or above 2^63
// nothing changes (no poisoned byte, outside every window).  T: the input's
// table of MAX_SLOTS entries (unused ones have base 0).
template <class TAB>
__device__ bool tripwire_catches(TAB* T, uint32_t spaces, uint32_t slot, int64_t idx, uint32_t lg) {
  constexpr uint64_t TOP = 1ull << 63;
  const uint32_t sp = (spaces >> (2 * slot)) & 3u;
  const uint64_t base = T[slot].base, e = 1ull << lg;
  uint64_t a8;  // address + 8, clamped
  if (idx < 0) {
    const uint64_t mag = 0ull - (uint64_t)idx;
    a8 = mag > ((base + 8) >> lg) ? 0ull : base + 8 - (mag << lg);
  } else {
    const uint64_t u = (uint64_t)idx;
    a8 = (u > (TOP >> lg) || (u << lg) > TOP - base) ? TOP + 8 : base + (u << lg) + 8;
  }
  const uint64_t b8 = a8 + e;
  uint64_t win8 = 8;
  for (uint32_t k = 0; k < MAX_SLOTS; k++) {
    const uint64_t kb = T[k].base;
    if (kb == 0 || ((spaces >> (2 * k)) & 3u) != sp) continue;
    const uint64_t rz = T[k].redzone, lo8 = kb - rz + 8, end8 = kb + T[k].size_bytes + 8, hi8 = end8 + rz;
    win8 = hi8 > win8 ? hi8 : win8;
    if (T[k].flags & CKC_ALLOC_FREED) {
      if (lo8 < hi8 && a8 < hi8 && lo8 < b8) return true;
    } else if ((lo8 < kb + 8 && a8 < kb + 8 && lo8 < b8) || (end8 < hi8 && a8 < hi8 && end8 < b8)) {
      return true;
    }
  }
  return sp != CKC_SPACE_GLOBAL && (a8 < 8 || b8 > win8);
}

// ---------------------------------------------------------------------------
// wavefront reductions
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint64_t shfl_xor64(uint64_t v, int m) {
  uint32_t lo = (uint32_t)v, hi = (uint32_t)(v >> 32);
  lo = __shfl_xor(lo, m, 64);
  hi = __shfl_xor(hi, m, 64);
  return ((uint64_t)hi << 32) | lo;
}
__device__ __forceinline__ uint64_t wave_min64(uint64_t v) {
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) {
    uint64_t o = shfl_xor64(v, m);
    v = o < v ? o : v;
  }
  return v;
}
__device__ __forceinline__ uint64_t wave_sum64(uint64_t v) {
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) v += shfl_xor64(v, m);
  return v;
}
__device__ __forceinline__ uint32_t lane_id() { return __lane_id(); }
__device__ __forceinline__ uint32_t ufirst(uint32_t v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ uint64_t ufirst64(uint64_t v) {
  return ((uint64_t)ufirst((uint32_t)(v >> 32)) << 32) | ufirst((uint32_t)v);
}

// Merge this wavefront's violations of one access into its record.  `bad` is
// the lane's kind (0 = none), `key` its first-violation key.
__device__ __forceinline__ void merge_violation(ckc_record* rec, uint32_t bad, uint64_t key) {
  uint64_t mask = __ballot(bad != 0);
  if (mask == 0) return;
  uint64_t k = wave_min64(bad ? key : ~0ull);
  uint32_t kinds = 0;
  if (__ballot(bad & CKC_KIND_OVER)) kinds |= CKC_KIND_OVER;
  if (__ballot(bad & CKC_KIND_UNDER)) kinds |= CKC_KIND_UNDER;
  if (__ballot(bad & CKC_KIND_FREED)) kinds |= CKC_KIND_FREED;
  if (__ballot(bad & CKC_KIND_NULL)) kinds |= CKC_KIND_NULL;
  uint32_t leader = __ffsll((unsigned long long)mask) - 1;
  if (lane_id() == leader) {
    atomicMin((unsigned long long*)&rec->first_key, (unsigned long long)k);
    atomicAdd((unsigned long long*)&rec->count, (unsigned long long)__popcll(mask));
    atomicOr(&rec->kinds, kinds);
  }
}

// Unsigned 32-bit division by a runtime divisor d >= 1 with a precomputed
// multiplier (Granlund and Montgomery, "Division by invariant integers using
// multiplication", 1994): m = floor(2^32 (2^s - d) / d) + 1, s = ceil(log2 d),
// q = (mulhi(n, m) + n) >> s, the sum taken in 64 bits.
struct UDiv {
  uint32_t m, s;
};
__device__ __forceinline__ UDiv udiv_make(uint32_t d) {
  const uint32_t s = 32u - (uint32_t)__clz((int)(d - 1u));
  const uint64_t m = ((1ull << 32) * ((1ull << s) - d)) / d + 1ull;
  return UDiv{(uint32_t)m, s};
}
__device__ __forceinline__ uint32_t udiv(uint32_t n, UDiv D) {
  return (uint32_t)(((uint64_t)__umulhi(n, D.m) + n) >> D.s);
}

// ---------------------------------------------------------------------------
// thread sets (CKC_FULL, CKC_REP_CORNERS, CKC_REP_BOUNDARY, and MODE_PAIR: one
// round of the PREX sweep)
// ---------------------------------------------------------------------------
struct Thr {
  uint32_t t[3], b[3];
  uint64_t gtid;
};

__device__ __forceinline__ void thr_from(const uint32_t* L, uint64_t blin, uint32_t tlin, Thr& th) {
  uint32_t gx = L[0], gy = L[1], bx = L[3], by = L[4];
  uint32_t bsz = L[3] * L[4] * L[5];
  uint64_t gxy = (uint64_t)gx * gy;
  th.b[2] = (uint32_t)(blin / gxy);
  uint32_t r = (uint32_t)(blin - (uint64_t)th.b[2] * gxy);
  th.b[1] = r / gx;
  th.b[0] = r - th.b[1] * gx;
  uint32_t bxy = bx * by;
  th.t[2] = tlin / bxy;
  uint32_t q = tlin - th.t[2] * bxy;
  th.t[1] = q / bx;
  th.t[0] = q - th.t[1] * bx;
  th.gtid = blin * bsz + tlin;
}

// Divisors of the whole-grid decode of one input, as multiply-shift pairs.
struct Dec {
  UDiv dbs, dgxy, dgx, dbxy, dbx;
  uint32_t bs, gxy, gx, bxy, bx;
  uint32_t one_d;  // one-dimensional grid of one-dimensional blocks
};
__device__ __forceinline__ void dec_make(Dec& d, const uint32_t* L) {
  d.one_d = L[1] == 1 && L[2] == 1 && L[4] == 1 && L[5] == 1;
  d.gx = L[0];
  d.gxy = L[0] * L[1];
  d.bx = L[3];
  d.bxy = L[3] * L[4];
  d.bs = d.bxy * L[5];
  d.dbs = udiv_make(d.bs);
  d.dgxy = udiv_make(d.gxy);
  d.dgx = udiv_make(d.gx);
  d.dbxy = udiv_make(d.bxy);
  d.dbx = udiv_make(d.bx);
}
// Whole-grid lane l: the lane index is the global thread id.
__device__ __forceinline__ void decode_full(const Dec& d, uint64_t l, Thr& th) {
  if (d.one_d && l < (1ull << 32)) {  // block and thread x only: one division
    const uint32_t b = udiv((uint32_t)l, d.dbs);
    th.b[0] = b;
    th.t[0] = (uint32_t)l - b * d.bs;
    th.b[1] = th.b[2] = th.t[1] = th.t[2] = 0;
    th.gtid = l;
    return;
  }
  uint32_t blin, tlin;
  if (l < (1ull << 32)) {
    blin = udiv((uint32_t)l, d.dbs);
    tlin = (uint32_t)l - blin * d.bs;
  } else {
    const uint64_t q = l / d.bs;
    blin = (uint32_t)q;
    tlin = (uint32_t)(l - q * d.bs);
  }
  th.b[2] = udiv(blin, d.dgxy);
  const uint32_t r = blin - th.b[2] * d.gxy;
  th.b[1] = udiv(r, d.dgx);
  th.b[0] = r - th.b[1] * d.gx;
  th.t[2] = udiv(tlin, d.dbxy);
  const uint32_t q = tlin - th.t[2] * d.bxy;
  th.t[1] = udiv(q, d.dbx);
  th.t[0] = q - th.t[1] * d.bx;
  th.gtid = l;
}

// The boundary thread set: every block that, along some grid dimension of
// extent >= 2, sits at the first or last coordinate, plus the middle block
// (gx/2, gy/2, gz/2) when it is not such a block; all threads of those blocks.
// Blocks are taken in block order.  Structure used below: the set is made of
// whole "face" slabs (z first/last), and in the other slabs of whole face rows
// (y first/last) and, in the other rows, the first and last block (x) -- plus
// the middle block in its own slab and row.
struct BSet {
  uint32_t gx, gy, gz, cx, cy, cz;
  uint32_t centre;      // 1 if the middle block is interior (an extra member)
  uint32_t per_row;     // set blocks of a non-face row without the middle block
  uint32_t face_rows;   // face rows of a non-face slab
  uint64_t gxy;
  uint64_t mbase;       // set blocks of a non-face slab without the middle block
};
__device__ __forceinline__ BSet bset(const uint32_t* L) {
  BSet s;
  s.gx = L[0]; s.gy = L[1]; s.gz = L[2];
  s.cx = s.gx / 2; s.cy = s.gy / 2; s.cz = s.gz / 2;
  s.centre = (s.gx == 1 || s.gx >= 3) && (s.gy == 1 || s.gy >= 3) && (s.gz == 1 || s.gz >= 3);
  s.per_row = s.gx >= 2 ? 2u : 0u;
  s.face_rows = s.gy >= 2 ? 2u : 0u;
  s.gxy = (uint64_t)s.gx * s.gy;
  s.mbase = (uint64_t)s.face_rows * s.gx + (uint64_t)(s.gy - s.face_rows) * s.per_row;
  return s;
}
__device__ __forceinline__ uint64_t bset_size(const uint32_t* L) {
  const uint64_t nb = (uint64_t)L[0] * L[1] * L[2];
  uint64_t inner = 1;
  for (int d = 0; d < 3; d++) inner *= L[d] >= 2 ? (uint64_t)(L[d] - 2) : 1ull;
  const BSet s = bset(L);
  return nb - inner + s.centre;
}
// Position k (0-based) of a middle-section list in which each of `n` groups
// holds `per` items, except group `cg` (if has_c) which holds one more.
// Returns the group and the index inside it.
__device__ __forceinline__ void split_groups(uint64_t k, uint64_t per, uint32_t n, bool has_c, uint32_t cg,
                                             uint32_t& grp, uint64_t& idx) {
  if (!has_c) {
    grp = per ? (uint32_t)(k / per) : 0u;
    idx = per ? k - (uint64_t)grp * per : k;
    return;
  }
  const uint64_t before = (uint64_t)cg * per;
  if (k < before) { grp = (uint32_t)(k / per); idx = k - (uint64_t)grp * per; return; }
  if (k < before + per + 1) { grp = cg; idx = k - before; return; }
  const uint64_t k2 = k - before - per - 1;
  const uint32_t g2 = per ? (uint32_t)(k2 / per) : 0u;
  grp = cg + 1 + g2;
  idx = per ? k2 - (uint64_t)g2 * per : k2;
  (void)n;
}
// Block index of the k-th member of the boundary set (k < bset_size).
__device__ __forceinline__ uint64_t bset_block(const uint32_t* L, uint64_t k) {
  const BSet s = bset(L);
  const bool zf = s.gz >= 2;
  if (zf && k < s.gxy) return k;  // first face slab
  const uint64_t k1 = zf ? k - s.gxy : k;
  const uint32_t zoff = zf ? 1u : 0u;
  const uint32_t nmid = zf ? s.gz - 2 : 1u;
  const uint64_t mid_total = (uint64_t)nmid * s.mbase + s.centre;
  if (k1 >= mid_total) return (uint64_t)(s.gz - 1) * s.gxy + (k1 - mid_total);  // last face slab
  uint32_t zi;
  uint64_t r;
  split_groups(k1, s.mbase, nmid, s.centre != 0, s.cz - zoff, zi, r);
  const uint32_t z = zoff + zi;
  const bool cslab = s.centre && z == s.cz;
  const bool yf = s.gy >= 2;
  const uint64_t zbase = (uint64_t)z * s.gxy;
  if (yf && r < s.gx) return zbase + r;  // first face row
  const uint64_t r1 = yf ? r - s.gx : r;
  const uint32_t yoff = yf ? 1u : 0u;
  const uint32_t nmid_rows = yf ? s.gy - 2 : 1u;
  const uint64_t mid_rows_total = (uint64_t)nmid_rows * s.per_row + (cslab ? 1 : 0);
  if (r1 >= mid_rows_total) return zbase + (uint64_t)(s.gy - 1) * s.gx + (r1 - mid_rows_total);
  uint32_t yi;
  uint64_t rr;
  split_groups(r1, s.per_row, nmid_rows, cslab, s.cy - yoff, yi, rr);
  const uint32_t y = yoff + yi;
  const bool crow = cslab && y == s.cy;
  uint32_t x;
  if (s.gx >= 2) x = rr == 0 ? 0u : (crow && rr == 1) ? s.cx : s.gx - 1;
  else x = 0;  // only the middle block
  return zbase + (uint64_t)y * s.gx + x;
}

// `aux` is the round r of a MODE_PAIR thread set (r <= nblocks-1-r) and is
// unused otherwise.
__device__ __forceinline__ uint64_t set_lanes(uint32_t mode, const uint32_t* L, uint32_t aux) {
  uint64_t nb = (uint64_t)L[0] * L[1] * L[2];
  uint64_t bs = (uint64_t)L[3] * L[4] * L[5];
  if (nb == 0 || bs == 0) return 0;
  if (mode == CKC_FULL) return nb * bs;
  if (mode == MODE_PAIR) return (nb - 1 - aux == aux ? 1ull : 2ull) * bs;
  if (mode == CKC_REP_CORNERS) {
    uint64_t n = 1;
    for (int d = 0; d < 6; d++) n *= L[d] == 1 ? 1 : 2;
    return n;
  }
  return bset_size(L) * bs;
}

// Thread of lane `l` (< set_lanes) of the input's thread set.  A MODE_PAIR
// set (round r = aux) holds block r, then block nblocks-1-r, each with all of
// its threads in thread order, so lanes run in increasing global thread id as
// in every other set.
__device__ __forceinline__ void decode_lane(uint32_t mode, const uint32_t* L, uint32_t aux, uint64_t l, Thr& th) {
  uint32_t bs = L[3] * L[4] * L[5];
  if (mode == MODE_PAIR) {
    const uint64_t nb = (uint64_t)L[0] * L[1] * L[2];
    const uint32_t half = l >= bs ? 1u : 0u;
    thr_from(L, half ? nb - 1 - aux : (uint64_t)aux, (uint32_t)(l - (uint64_t)half * bs), th);
    return;
  }
  if (mode == CKC_REP_CORNERS) {
    uint32_t c[6];
    uint32_t v = (uint32_t)l;
#pragma unroll
    for (int d = 3; d < 6; d++) {  // thread dims least significant
      uint32_t two = L[d] == 1 ? 1u : 2u;
      c[d] = (v % two) ? L[d] - 1 : 0;
      v /= two;
    }
#pragma unroll
    for (int d = 0; d < 3; d++) {
      uint32_t two = L[d] == 1 ? 1u : 2u;
      c[d] = (v % two) ? L[d] - 1 : 0;
      v /= two;
    }
    uint64_t blin = c[0] + (uint64_t)L[0] * (c[1] + (uint64_t)L[1] * c[2]);
    uint32_t tlin = c[3] + L[3] * (c[4] + L[4] * c[5]);
    thr_from(L, blin, tlin, th);
    return;
  }
  uint64_t q = l / bs;
  uint32_t tlin = (uint32_t)(l - q * bs);
  uint64_t blin = mode == CKC_FULL ? q : bset_block(L, q);
  thr_from(L, blin, tlin, th);
}


}  // namespace ckc
