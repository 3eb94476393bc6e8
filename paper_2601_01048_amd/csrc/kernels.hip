// kernels.hip — device side of libckc for gfx950 (MI355X, CDNA4).
//
// One lane per (input, thread of the thread set).  Kernels of a job:
//   plan      one wavefront per input: thread-set size, and for programs whose
//             control flow is thread-invariant the per-input access trace
//             (affine forms of every index, evaluated once per input);
//   scan      tile offsets of both evaluators over the inputs;
//   eval_trace  persistent: per lane, base[class] + offset for every trace
//             entry and one unsigned compare against the bound;
//   eval_generic persistent: a wavefront-uniform interpreter of the lowered
//             bytecode staged in LDS, with one loop per program evaluated one
//             lane per iteration across the workgroup;
//   fixup     one wavefront per violated record: replays the winning thread to
//             fill the index and kind at the first key;
//   finish    per input: coverage counts -> saturating dense map, status.
//
// Violations are reduced per wavefront (ballot, min, or) and merged with one
// 64-bit atomicMin / atomicAdd / atomicOr per (wavefront, access).  Every merge
// is order-independent, so results do not depend on scheduling.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

#include "../../include/ckc.h"
#include "dformat.h"
#include "kernels.h"

#include <cstring>

namespace ckc {

// ---------------------------------------------------------------------------
// integer semantics of the IR (ckc_ir.h)
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint64_t narrow(uint64_t v, uint32_t w) {
  return w == 32 ? (uint64_t)(int64_t)(int32_t)(uint32_t)v : v;
}

__device__ __forceinline__ uint64_t alu(uint32_t op, uint32_t w, uint64_t x, uint64_t y, uint32_t& faults) {
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
// thread sets (CKC_FULL, CKC_REP_CORNERS, CKC_REP_BOUNDARY)
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
};
__device__ __forceinline__ void dec_make(Dec& d, const uint32_t* L) {
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

__device__ __forceinline__ uint64_t set_lanes(uint32_t mode, const uint32_t* L) {
  uint64_t nb = (uint64_t)L[0] * L[1] * L[2];
  uint64_t bs = (uint64_t)L[3] * L[4] * L[5];
  if (nb == 0 || bs == 0) return 0;
  if (mode == CKC_FULL) return nb * bs;
  if (mode == CKC_REP_CORNERS) {
    uint64_t n = 1;
    for (int d = 0; d < 6; d++) n *= L[d] == 1 ? 1 : 2;
    return n;
  }
  return bset_size(L) * bs;
}

// Thread of lane `l` (< set_lanes) of the input's thread set.
__device__ __forceinline__ void decode_lane(uint32_t mode, const uint32_t* L, uint64_t l, Thr& th) {
  uint32_t bs = L[3] * L[4] * L[5];
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

__device__ __forceinline__ uint64_t rget(const uint32_t* lo, const uint32_t* hi, uint32_t i) {
  return ((uint64_t)hi[i] << 32) | lo[i];
}
#define RSET(i, v)                      \
  do {                                  \
    uint64_t _v = (v);                  \
    lo[(i)] = (uint32_t)_v;             \
    hi[(i)] = (uint32_t)(_v >> 32);     \
  } while (0)

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
                            ckc_input_status* st) {
  const uint32_t j = lane_id();
  const dins* I = prog_ins(P);
  const int64_t* K = prog_consts(P);
  uint32_t lo[NREG], hi[NREG];
#pragma unroll
  for (int r = 0; r < NREG; r++) { lo[r] = 0; hi[r] = 0; }
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
        uint64_t a = rget(lo, hi, D.a), b = rget(lo, hi, D.b);
        RSET(D.dst, narrow(op == CKC_OP_ADD ? a + b : a - b, w));
        break;
      }
      case CKC_OP_MUL: case CKC_OP_SHL: {
        uint64_t a = rget(lo, hi, D.a), b = rget(lo, hi, D.b);
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
      case CKC_OP_TRUNC: RSET(D.dst, narrow(rget(lo, hi, D.a), 32)); break;
      case CKC_OP_SEXT: RSET(D.dst, j == 6 ? narrow(rget(lo, hi, D.a), 32) : 0ull); break;
      case CKC_OP_ZEXT: RSET(D.dst, j == 6 ? (rget(lo, hi, D.a) & 0xFFFFFFFFull) : 0ull); break;
      case CKC_OP_SELECT: {
        uint64_t c = readlane64(rget(lo, hi, D.a), 6);
        RSET(D.dst, narrow(c != 0 ? rget(lo, hi, D.b) : rget(lo, hi, D.c), w));
        break;
      }
      case CKC_OP_ACCESS: case CKC_OP_LOAD: {
        uint64_t v = rget(lo, hi, D.a);
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
        uint64_t c = readlane64(rget(lo, hi, D.a), 6);
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
        int64_t s = (int64_t)narrow(readlane64(rget(lo, hi, D.a), 6), w);
        int64_t e = (int64_t)narrow(readlane64(rget(lo, hi, D.b), 6), w);
        int64_t stp = (int64_t)narrow(readlane64(rget(lo, hi, D.c), 6), w);
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
        uint64_t r = alu(op, w, readlane64(rget(lo, hi, D.a), 6), readlane64(rget(lo, hi, D.b), 6), f);
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

__global__ void __launch_bounds__(64) plan_kernel(KArgs a) {
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
    }
  uint64_t lanes = set_lanes(in.mode, in.launch);
  bool trace = (P->cls & CKC_CLS_UNIFORM) && !a.force_generic && in.trace != 0 && lanes > 0;
  __syncthreads();
  ckc_input_status* st = a.status + i;
  if (j == 0) {
    st->lanes = lanes; st->accesses_checked = 0; st->hang_lanes = 0; st->arith_faults = 0;
    st->flags = 0; st->pad = 0;
  }
  uint32_t path = 1;
  if (trace) {
    dtrace_head* th = (dtrace_head*)in.trace;
    const uint32_t cap8 = (P->trace_cap + 7u) & ~7u;
    dtrace_entry* te = (dtrace_entry*)((uint8_t*)(th + 1) + (size_t)cap8 * 24);
    build_trace(P, in, a.scalars + (size_t)i * MAX_SCALARS, (const ckc_alloc*)in.table, th, te, cnt, st);
    __syncthreads();
    path = th->overflow ? 1 : 0;
    if (path == 1) {  // fall back: undo the per-thread counts
      for (uint32_t s = j; s < P->n_sites; s += 64) cnt[s] = 0;
      if (j == 0) { st->accesses_checked = 0; st->arith_faults = 0; st->hang_lanes = 0; }
    }
  }
  if (j == 0) {
    uint64_t tiles = (lanes + TILE - 1) / TILE;
    const uint32_t bs = in.launch[3] * in.launch[4] * in.launch[5];
    if (path == 0) {
      if (in.mode != CKC_REP_CORNERS && bs % 64u == 0 && ((const dtrace_head*)in.trace)->n_classes == 1) {
        // block-major jobs: (64-thread slice position, group of LPB set blocks)
        const uint64_t nsb = in.mode == CKC_FULL ? (uint64_t)in.launch[0] * in.launch[1] * in.launch[2]
                                                 : bset_size(in.launch);
        const uint64_t jobs = (uint64_t)(bs / 64u) * ((nsb + LPB - 1) / LPB);
        tiles = (jobs + 3) / 4;
        path = PATH_BLOCKS;
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
// trace evaluator
// ---------------------------------------------------------------------------
// Read-only job data is read through the constant address space so that
// wavefront-uniform loads become scalar loads.
typedef const __attribute__((address_space(4))) dtrace_entry c_entry;
typedef const __attribute__((address_space(4))) dtrace_head c_head;
typedef const __attribute__((address_space(4))) dinput c_input;
typedef const __attribute__((address_space(4))) jobstate c_jobstate;
typedef const __attribute__((address_space(4))) uint32_t c_u32;

__device__ __forceinline__ uint32_t find_pos_c(c_input* in, c_u32* order, uint32_t n, uint32_t path, uint64_t t) {
  uint32_t lo = 0, hi = n - 1;
  while (lo < hi) {
    uint32_t mid = lo + (hi - lo + 1) / 2;
    if (in[order[mid]].tile_begin[path] <= t) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

// Position of the input holding tile t: the next one or two positions are
// tried first (consecutive tiles of one workgroup), then a binary search.
__device__ __forceinline__ uint32_t pos_of_tile(c_input* ins, c_u32* order, uint32_t n, uint32_t path,
                                                uint32_t pos, uint64_t cur_end, uint64_t t) {
  if (pos != 0xFFFFFFFFu && t >= cur_end) {
    for (uint32_t q = pos + 1; q < n && q <= pos + 2; q++) {
      const uint32_t i = order[q];
      if (t >= ins[i].tile_begin[path] && t < ins[i].tile_begin[path] + ins[i].n_tiles[path]) return q;
    }
  }
  return find_pos_c(ins, order, n, path, t);
}

// Violations found by the trace evaluator are merged per workgroup in LDS (first
// key, count, kinds per access of the current input) and flushed into the job's
// records once per input.  Every thread-set decode of this evaluator is
// increasing in the global thread id along the lanes of a wavefront, and the
// blocks of a wavefront job are increasing too, so the first violation of a
// wavefront is its lowest violating lane.
constexpr uint32_t TR_ACC_LDS = 256;
struct TraceLds {
  unsigned long long fk[TR_ACC_LDS];
  unsigned long long cnt[TR_ACC_LDS];
  uint32_t kinds[TR_ACC_LDS];
};

__device__ __forceinline__ void tr_note(TraceLds& S, ckc_record* rec, uint32_t acc, bool lds, uint64_t key,
                                        uint64_t cnt, uint32_t kinds) {
  if (lane_id() == 0) {
    if (lds) {
      atomicMin(&S.fk[acc], (unsigned long long)key);
      atomicAdd(&S.cnt[acc], (unsigned long long)cnt);
      atomicOr(&S.kinds[acc], kinds);
    } else {
      atomicMin((unsigned long long*)&rec[acc].first_key, (unsigned long long)key);
      atomicAdd((unsigned long long*)&rec[acc].count, (unsigned long long)cnt);
      atomicOr(&rec[acc].kinds, kinds);
    }
  }
}

__device__ void tr_flush(TraceLds& S, ckc_record* rec, uint32_t n_acc) {
  __syncthreads();
  for (uint32_t q = threadIdx.x; q < n_acc && q < TR_ACC_LDS; q += TILE) {
    if (S.cnt[q]) {
      atomicMin((unsigned long long*)&rec[q].first_key, S.fk[q]);
      atomicAdd((unsigned long long*)&rec[q].count, S.cnt[q]);
      atomicOr(&rec[q].kinds, S.kinds[q]);
      S.fk[q] = ~0ull;
      S.cnt[q] = 0;
      S.kinds[q] = 0;
    }
  }
  __syncthreads();
}

// Out-of-line boundary-set decode (keeps its divisions off the FULL path).
__device__ __forceinline__ uint64_t bset_block_call(uint32_t gx, uint32_t gy, uint32_t gz, uint64_t k) {
  const uint32_t L[3] = {gx, gy, gz};
  return bset_block(L, k);
}

typedef const __attribute__((address_space(4))) int64_t c_i64;
typedef const __attribute__((address_space(4))) dprog c_dprog;

// Violation path of entry e in a block-major job (rare): per block, the mask
// of violating lanes and of negative indices; the first block with a
// violation gives the first key at its lowest violating lane.
template <int W, class BT>
__device__ __forceinline__ void blocks_violation(TraceLds& S, c_entry* te, uint32_t e, uint64_t tpart,
                                                 const BT* bp, const uint32_t* Lg, uint64_t g, uint32_t bs,
                                                 uint32_t nvalid, uint32_t tlin_lane0, ckc_record* rec,
                                                 bool lds, uint32_t Lsum) {
  const int64_t off = te[e].off;
  const uint64_t bound = te[e].bound;
  const uint32_t dead = te[e].dead_kind;
  uint64_t fk = ~0ull, cnt = 0;
  uint32_t kinds = 0;
  for (uint32_t j = 0; j < nvalid; j++) {
    uint64_t badm, underm;
    if (W == 32) {
      const uint32_t v = (uint32_t)tpart + (uint32_t)off + (uint32_t)bp[j];
      badm = __ballot(v >= (uint32_t)bound);
      underm = __ballot((int32_t)v < 0);
    } else {
      const uint64_t v = tpart + (uint64_t)off + (uint64_t)bp[j];
      badm = __ballot(v >= bound);
      underm = __ballot((int64_t)v < 0);
    }
    if (dead) {
      badm = ~0ull;
      kinds |= dead;
    } else {
      underm &= badm;
      kinds |= (underm ? CKC_KIND_UNDER : 0u) | ((badm & ~underm) ? CKC_KIND_OVER : 0u);
    }
    if (badm) {
      if (fk == ~0ull) {
        // block of member g*LPB + j of the thread set (Lg[6] holds the mode)
        const uint64_t k = g * LPB + j;
        const uint64_t blin = Lg[6] == CKC_FULL ? k : bset_block(Lg, k);
        fk = ((blin * bs + tlin_lane0 + (uint64_t)(__ffsll((unsigned long long)badm) - 1)) << Lsum) |
             te[e].keylo;
      }
      cnt += (uint64_t)__popcll(badm);
    }
  }
  if (cnt) tr_note(S, rec, te[e].acc, lds, fk, cnt, kinds);
}

// Block-major checks of one wavefront job: this lane's thread position in up to
// LPB set blocks; tpart is the thread part of the index base, bp[j] the block
// parts (wavefront-uniform).  Entries come as packed (offset, bound) pairs
// through scalar loads.  Width 32: an index is in bounds iff its unsigned
// value is below the bound (clamped to 2^31), so one entry is clean for all
// blocks iff the unsigned maximum over the blocks is below the bound -- one
// add per block, a max tree and one compare.
template <int W, bool ALL, class BT>
__device__ __forceinline__ bool entry_bad(uint64_t tpart, uint64_t off, uint64_t bnd, const BT* bp,
                                          uint32_t nvalid) {
  if (W == 32) {
    const uint32_t t = (uint32_t)tpart + (uint32_t)off;
    uint32_t mx = 0;
#pragma unroll
    for (uint32_t j = 0; j < LPB; j++) {
      const uint32_t v = t + (uint32_t)bp[j];
      if (ALL || j < nvalid) mx = v > mx ? v : mx;
    }
    return mx >= (uint32_t)bnd;
  } else {
    const uint64_t t = tpart + off;
    bool x = false;
#pragma unroll
    for (uint32_t j = 0; j < LPB; j++)
      if (ALL || j < nvalid) x |= (t + (uint64_t)bp[j]) >= bnd;
    return x;
  }
}

template <int W, bool ALL, bool DEADS, class BT>
__device__ __forceinline__ void trace_blocks(TraceLds& S, c_entry* te, c_i64* h64, c_u32* h32, uint32_t ne,
                                             uint64_t tpart, const BT* bp, const uint32_t* Lg, uint64_t g,
                                             uint32_t bs, uint32_t nvalid, uint32_t tlin_lane0,
                                             ckc_record* rec, bool lds, uint32_t Lsum) {
  constexpr uint32_t EB = W == 32 ? 8 : 4;  // entries per scalar-load batch
  uint32_t e = 0;  // first entry that needs the violation path
  if (!DEADS) {
    // fast scan: stop at the first entry with a violating lane
    const uint32_t neb = ne - ne % EB;
    bool hit = false;
    for (uint32_t e0 = 0; e0 < neb && !hit; e0 += EB) {
      uint64_t off[EB], bnd[EB];
#pragma unroll
      for (uint32_t k = 0; k < EB; k++) {
        if (W == 32) {
          off[k] = h32[2 * (e0 + k)];
          bnd[k] = h32[2 * (e0 + k) + 1];
        } else {
          off[k] = (uint64_t)h64[2 * (e0 + k)];
          bnd[k] = (uint64_t)h64[2 * (e0 + k) + 1];
        }
      }
#pragma unroll
      for (uint32_t k = 0; k < EB; k++) {
        if (!hit && __ballot(entry_bad<W, ALL>(tpart, off[k], bnd[k], bp, nvalid))) {
          hit = true;
          e = e0 + k;
        }
      }
      if (!hit) e = e0 + EB;
    }
    if (!hit) {
      for (; e < ne; e++) {
        uint64_t off, bnd;
        if (W == 32) {
          off = h32[2 * e];
          bnd = h32[2 * e + 1];
        } else {
          off = (uint64_t)h64[2 * e];
          bnd = (uint64_t)h64[2 * e + 1];
        }
        if (__ballot(entry_bad<W, ALL>(tpart, off, bnd, bp, nvalid))) break;
      }
    }
    if (e >= ne) return;
  }
  // violation path: the remaining entries one by one (one copy of this code)
  for (; e < ne; e++) {
    uint64_t off, bnd;
    if (W == 32) {
      off = h32[2 * e];
      bnd = h32[2 * e + 1];
    } else {
      off = (uint64_t)h64[2 * e];
      bnd = (uint64_t)h64[2 * e + 1];
    }
    if (DEADS || __ballot(entry_bad<W, false>(tpart, off, bnd, bp, nvalid)))
      blocks_violation<W>(S, te, e, tpart, bp, Lg, g, bs, nvalid, tlin_lane0, rec, lds, Lsum);
  }
}

// Per-input state of the trace evaluator (wavefront-uniform).
struct TrIn {
  uint32_t L[7];  // launch dims, then the thread-set mode
  uint32_t bs, gxy, bxy, mode, Lsum, ne, n_acc;
  UDiv dgx, dgxy, dbx, dbxy, dspb;
  uint64_t nsb;
  c_head* th;     // coefficients are re-read per job (scalar loads)
  uint32_t any_dead;
  bool lds;
  c_entry* te;
  c_i64* h64;
  c_u32* h32;
  ckc_record* rec;
};

// One block-major wavefront job: slice position o (64 threads) of the blocks
// g*LPB .. g*LPB+LPB-1 of the set.
template <int W>
__device__ __forceinline__ void block_job(TraceLds& S, const TrIn& I, uint64_t g, uint32_t o) {
  typedef typename std::conditional<W == 32, uint32_t, uint64_t>::type BT;
  const uint32_t tlin = o * 64u + (threadIdx.x & 63u);
  const uint32_t tz = udiv(tlin, I.dbxy), tr = tlin - tz * I.bxy;
  const uint32_t ty = udiv(tr, I.dbx);
  const uint32_t tx = tr - ty * I.L[3];
  const int64_t k0 = I.th->coef[0][0], k1 = I.th->coef[0][1], k2 = I.th->coef[0][2];
  const int64_t k3 = I.th->coef[0][3], k4 = I.th->coef[0][4], k5 = I.th->coef[0][5];
  uint64_t tpart = 0;
  if (k0 == 1) tpart += tx; else if (k0 != 0) tpart += (uint64_t)k0 * tx;
  if (k1 == 1) tpart += ty; else if (k1 != 0) tpart += (uint64_t)k1 * ty;
  if (k2 == 1) tpart += tz; else if (k2 != 0) tpart += (uint64_t)k2 * tz;
  BT bp[LPB];
  const uint64_t left = I.nsb - g * LPB;
  const uint32_t nvalid = left < LPB ? (uint32_t)left : LPB;
  if (I.mode == CKC_FULL) {
    // blocks g*LPB ..: walk x with carries from the first one
    const uint32_t b0 = (uint32_t)(g * LPB);
    uint32_t bz = udiv(b0, I.dgxy), brem = b0 - bz * I.gxy;
    uint32_t by = udiv(brem, I.dgx), bx = brem - by * I.L[0];
#pragma unroll
    for (uint32_t jj = 0; jj < LPB; jj++) {
      bp[jj] = (BT)((uint64_t)k3 * bx + (uint64_t)k4 * by + (uint64_t)k5 * bz);
      if (++bx == I.L[0]) {
        bx = 0;
        if (++by == I.L[1]) { by = 0; ++bz; }
      }
    }
  } else {
    for (uint32_t jj = 0; jj < LPB; jj++) {
      const uint32_t blin = jj < nvalid ? (uint32_t)bset_block_call(I.L[0], I.L[1], I.L[2], g * LPB + jj) : 0u;
      const uint32_t bz = udiv(blin, I.dgxy), brem = blin - bz * I.gxy;
      const uint32_t by = udiv(brem, I.dgx), bx = brem - by * I.L[0];
      bp[jj] = (BT)((uint64_t)k3 * bx + (uint64_t)k4 * by + (uint64_t)k5 * bz);
    }
  }
  const uint32_t t0 = o * 64u;
  if (I.any_dead) {
    trace_blocks<W, false, true>(S, I.te, I.h64, I.h32, I.ne, tpart, bp, I.L, g, I.bs, nvalid, t0, I.rec, I.lds, I.Lsum);
  } else if (nvalid == LPB) {
    trace_blocks<W, true, false>(S, I.te, I.h64, I.h32, I.ne, tpart, bp, I.L, g, I.bs, nvalid, t0, I.rec, I.lds, I.Lsum);
  } else {
    trace_blocks<W, false, false>(S, I.te, I.h64, I.h32, I.ne, tpart, bp, I.L, g, I.bs, nvalid, t0, I.rec, I.lds, I.Lsum);
  }
}

// Per-lane checks of one lane tile (thread sets without the block-major
// layout).  The lowest violating lane has the smallest key.
__device__ __forceinline__ void lanes_violation(TraceLds& S, c_entry* te, uint32_t e, uint64_t v, bool act,
                                                uint64_t gtid, ckc_record* rec, bool lds, uint32_t Lsum) {
  const uint32_t w = te[e].w;
  const uint64_t bound = te[e].bound;
  const uint32_t dead = te[e].dead_kind;
  uint64_t badm, underm;
  if (w == 32) {
    badm = __ballot(act && (uint32_t)v >= (uint32_t)bound);
    underm = __ballot(act && (int32_t)(uint32_t)v < 0);
  } else {
    badm = __ballot(act && v >= bound);
    underm = __ballot(act && (int64_t)v < 0);
  }
  uint32_t kinds;
  if (dead) {
    badm = __ballot(act);
    kinds = dead;
  } else {
    underm &= badm;
    kinds = (underm ? CKC_KIND_UNDER : 0u) | ((badm & ~underm) ? CKC_KIND_OVER : 0u);
  }
  if (!badm) return;
  const int first = __ffsll((unsigned long long)badm) - 1;
  const uint64_t key = (readlane64(gtid, first) << Lsum) | te[e].keylo;
  tr_note(S, rec, te[e].acc, lds, key, (uint64_t)__popcll(badm), kinds);
}

// Loads the per-input state of the trace evaluator.
__device__ __forceinline__ void tr_load(TrIn& I, c_input* ins, uint32_t i, ckc_record* recs, uint64_t& tb,
                                        uint32_t path, uint32_t& ncls, uint32_t& w0, c_head*& th) {
  for (int q = 0; q < 6; q++) I.L[q] = ins[i].launch[q];
  I.L[6] = ins[i].mode;
  I.bs = I.L[3] * I.L[4] * I.L[5];
  I.gxy = I.L[0] * I.L[1];
  I.bxy = I.L[3] * I.L[4];
  I.dgx = udiv_make(I.L[0]);
  I.dgxy = udiv_make(I.gxy);
  I.dbx = udiv_make(I.L[3]);
  I.dbxy = udiv_make(I.bxy);
  I.dspb = udiv_make(I.bs >= 64 ? I.bs / 64u : 1u);
  I.mode = ins[i].mode;
  I.Lsum = ins[i].L1 + ins[i].L2;
  I.n_acc = ((c_dprog*)ins[i].prog)->n_accesses;
  I.lds = I.n_acc <= TR_ACC_LDS;
  th = (c_head*)ins[i].trace;
  const uint32_t cap8 = th->cap8;
  I.h64 = (c_i64*)(th + 1);
  I.h32 = (c_u32*)(I.h64 + 2 * (size_t)cap8);
  I.te = (c_entry*)(I.h32 + 2 * (size_t)cap8);
  I.any_dead = th->any_dead;
  I.rec = recs + ins[i].rec_base;
  I.ne = th->n_entries;
  ncls = th->n_classes;
  w0 = th->cls_w[0];
  I.nsb = I.mode == CKC_FULL ? (uint64_t)I.L[0] * I.L[1] * I.L[2] : bset_size(I.L);
  I.th = th;
  tb = ins[i].tile_begin[path];
}

// Trace evaluator, block-major layout: persistent workgroups over the tile
// space of PATH_BLOCKS under the job's schedule; a tile is four wavefront jobs.
template <uint32_t SK>
__global__ void __launch_bounds__(TILE) eval_trace_kernel(KArgs a) {
  __shared__ TraceLds S;
  __shared__ unsigned long long item_slot;
  c_jobstate* js = (c_jobstate*)a.js;
  c_input* ins = (c_input*)a.inputs;
  c_u32* order = (c_u32*)a.order;
  const uint64_t total = js->total_tiles[PATH_BLOCKS];
  if (total == 0) return;
  Sched<SK> sc;
  sched_init(sc, a, total);
  if (SK == CKC_SCHED_BLOCKED && sc.cur >= sc.end) return;
  const uint32_t tid = threadIdx.x;
  for (uint32_t q = tid; q < TR_ACC_LDS; q += TILE) {
    S.fk[q] = ~0ull;
    S.cnt[q] = 0;
    S.kinds[q] = 0;
  }
  __syncthreads();
  uint32_t pos = 0xFFFFFFFFu, ncls = 0, w0 = 32;
  uint64_t tb = 0, cur_end = 0;
  c_head* th = nullptr;
  TrIn I;
  for (;;) {
    const uint64_t t = sched_next(sc, &a.js->next_tile[PATH_BLOCKS], &item_slot);
    if (t == ~0ull) break;
    if (pos == 0xFFFFFFFFu || t < tb || t >= cur_end) {
      const uint32_t np = pos_of_tile(ins, order, a.n_inputs, PATH_BLOCKS, pos, cur_end, t);
      if (pos != 0xFFFFFFFFu && I.lds) tr_flush(S, I.rec, I.n_acc);
      pos = np;
      const uint32_t i = order[pos];
      tr_load(I, ins, i, a.recs, tb, PATH_BLOCKS, ncls, w0, th);
      cur_end = tb + ins[i].n_tiles[PATH_BLOCKS];
    }
    const uint32_t wv = ufirst(tid >> 6);
    const uint64_t job = (t - tb) * 4 + wv;
    const uint32_t spb = I.bs / 64u;
    const uint64_t g = job < (1ull << 32) ? (uint64_t)udiv((uint32_t)job, I.dspb) : job / spb;
    const uint32_t o = (uint32_t)(job - g * spb);
    if (g * LPB >= I.nsb) continue;  // past the last group (whole wavefront)
    if (w0 == 32) block_job<32>(S, I, g, o);
    else block_job<64>(S, I, g, o);
  }
  if (pos != 0xFFFFFFFFu && I.lds) tr_flush(S, I.rec, I.n_acc);
}

// Trace evaluator over lane tiles (thread sets or traces the block-major
// layout does not cover): TILE consecutive lanes of the thread set per tile.
template <uint32_t SK>
__global__ void __launch_bounds__(TILE) eval_trace_lanes_kernel(KArgs a) {
  __shared__ TraceLds S;
  __shared__ unsigned long long item_slot;
  c_jobstate* js = (c_jobstate*)a.js;
  c_input* ins = (c_input*)a.inputs;
  c_u32* order = (c_u32*)a.order;
  const uint64_t total = js->total_tiles[PATH_LANES];
  if (total == 0) return;
  Sched<SK> sc;
  sched_init(sc, a, total);
  if (SK == CKC_SCHED_BLOCKED && sc.cur >= sc.end) return;
  const uint32_t tid = threadIdx.x;
  for (uint32_t q = tid; q < TR_ACC_LDS; q += TILE) {
    S.fk[q] = ~0ull;
    S.cnt[q] = 0;
    S.kinds[q] = 0;
  }
  __syncthreads();
  uint32_t pos = 0xFFFFFFFFu, ncls = 0, w0 = 32;
  uint64_t tb = 0, cur_end = 0, lanes = 0;
  c_head* th = nullptr;
  TrIn I;
  for (;;) {
    const uint64_t t = sched_next(sc, &a.js->next_tile[PATH_LANES], &item_slot);
    if (t == ~0ull) break;
    if (pos == 0xFFFFFFFFu || t < tb || t >= cur_end) {
      const uint32_t np = pos_of_tile(ins, order, a.n_inputs, PATH_LANES, pos, cur_end, t);
      if (pos != 0xFFFFFFFFu && I.lds) tr_flush(S, I.rec, I.n_acc);
      pos = np;
      const uint32_t i = order[pos];
      tr_load(I, ins, i, a.recs, tb, PATH_LANES, ncls, w0, th);
      cur_end = tb + ins[i].n_tiles[PATH_LANES];
      lanes = ins[i].lanes;
    }
    const uint64_t l = (t - tb) * TILE + tid;
    const bool act = l < lanes;
    Thr T;
    decode_lane(I.mode, I.L, act ? l : 0, T);
    const uint32_t c6[6] = {T.t[0], T.t[1], T.t[2], T.b[0], T.b[1], T.b[2]};
    // base of each coefficient class: sum of coefficient x coordinate,
    // skipping zero coefficients (uniform branches)
    uint64_t base[MAX_CLASSES];
#pragma unroll
    for (int c = 0; c < MAX_CLASSES; c++) {
      uint64_t b = 0;
      if ((uint32_t)c < ncls) {
#pragma unroll
        for (int d = 0; d < 6; d++) {
          const int64_t k = th->coef[c][d];
          if (k == 1) b += c6[d];
          else if (k != 0) b += (uint64_t)k * c6[d];
        }
      }
      base[c] = b;
    }
    c_entry* te = I.te;
    for (uint32_t e = 0; e < I.ne; e++) {
      const uint32_t c = te[e].cls;
      const uint64_t b = c == 0 ? base[0] : c == 1 ? base[1] : c == 2 ? base[2] : base[3];
      const uint64_t v = b + (uint64_t)te[e].off;
      bool x;
      if (te[e].w == 32) x = (uint32_t)v >= (uint32_t)te[e].bound;
      else x = v >= te[e].bound;
      if (__ballot(act && x) || te[e].dead_kind) lanes_violation(S, te, e, v, act, T.gtid, I.rec, I.lds, I.Lsum);
    }
  }
  if (pos != 0xFFFFFFFFu && I.lds) tr_flush(S, I.rec, I.n_acc);
}

// ---------------------------------------------------------------------------
// generic interpreter
// ---------------------------------------------------------------------------
// The register file lives in LDS (dynamic shared memory): register r of lane t
// is R[r * TILE + t], 64 bits, so operands are addressed by wavefront-uniform
// register numbers without any per-lane indexing.  The lowered bytecode and
// its constants are read through the scalar cache (constant address space):
// every instruction field arrives in scalar registers.
typedef const __attribute__((address_space(4))) dins c_dins;
typedef const __attribute__((address_space(4))) daccess c_daccess;

// One 16-byte instruction through four scalar loads.
__device__ __forceinline__ dins ld_ins(c_dins* I, uint32_t pc) {
  c_u32* p = (c_u32*)(I + pc);
  const uint32_t w[4] = {p[0], p[1], p[2], p[3]};
  dins d;
  __builtin_memcpy(&d, w, sizeof d);
  return d;
}

typedef const __attribute__((address_space(4))) ckc_alloc c_alloc;

struct GenLds {
  uint32_t sites[MAX_SITES_LDS];
  unsigned long long wsum[TILE / 64];
  unsigned long long acc_checked, hangs, faults;
  unsigned long long pref[TILE + 1];  // trip-count prefix of the tile's threads (expanded loop)
};

// Modes of the interpreter: M_MAIN runs whole threads (an expanded loop is
// only recorded), M_BODY runs one iteration of the expanded loop's body per
// lane, M_FIX replays one thread (lane 0) up to a target access.
enum { M_MAIN = 0, M_FIX = 1, M_BODY = 2 };

struct Lane {
  uint32_t dis;            // 0 = active; >0 disabled depth; >= DEAD stopped
  uint64_t k0, k1;         // iteration ordinals at depth 0 / 1
  uint64_t run0, run1;     // iterations to run
  uint64_t st0, st1;       // loop start
  uint64_t sp0, sp1;       // loop step
  uint32_t hangp;          // bit d: the loop at depth d exceeds its cap
  uint64_t gtid;
  uint32_t faults, hangs;
  uint32_t acc;            // ACCESS and LOAD executions
};

struct Ctx {
  const dinput* in;
  c_dprog* P;
  c_dins* I;
  c_i64* K;
  const int64_t* sc;
  c_alloc* tab;            // this input's allocation table (scalar loads)
  ckc_record* rec;
  uint32_t* gcnt;          // global site counters (sites beyond the LDS range)
  uint32_t Lsum, L2;
  uint64_t cap0, cap1;
  uint32_t t0, t1, t2, b0, b1, b2;  // thread coordinates (this lane)
  // expanded loop: this input's thread-state arrays (pref, start, step,
  // live-ins; xn entries each), the tile's first lane and expanded tile
  uint64_t* xs;
  uint64_t xn, lane0, xt;
  unsigned long long *xtot, *xpb;
  uint32_t* xin;
  uint32_t input;
  // fix-up target
  uint32_t tacc;
  uint64_t tk0, tk1;
  int32_t tloop0, tloop1;
  ckc_record* trec;
};

// Coverage of site s by the lanes of `mask`: one LDS add per wavefront.  `sat`
// (wavefront-uniform) marks sites below 64 whose workgroup count has reached
// the saturation value 255, after which counting them changes nothing.
__device__ __forceinline__ void count_site(GenLds& S, const Ctx& C, uint64_t& sat, uint32_t s, uint64_t mask) {
  if (s == NOSITE || mask == 0) return;
  if (s < 64 && ((sat >> s) & 1u)) return;
  const uint32_t leader = (uint32_t)(__ffsll((unsigned long long)mask) - 1);
  const uint32_t c = (uint32_t)__popcll(mask);
  if (s < MAX_SITES_LDS) {
    uint32_t old = 0;
    if (lane_id() == leader) old = atomicAdd(&S.sites[s], c);
    old = __builtin_amdgcn_readlane(old, leader);
    if (s < 64 && old + c >= 255u) sat |= 1ull << s;
  } else if (lane_id() == leader && C.gcnt[s] < 255u) {
    atomicAdd(&C.gcnt[s], c);
  }
}

// Register file in LDS (dynamic shared memory): register r of lane t is
// R[r * TILE + t], 64 bits, addressed by wavefront-uniform register numbers.
#define RGET(i) R[(uint32_t)(i) * TILE + threadIdx.x]
#define RPUT(i, v) (R[(uint32_t)(i) * TILE + threadIdx.x] = (v))

// Iterations of an expanded loop per work item of the body pass.
constexpr uint32_t PIECE = 2048;

// Runs the program for the wavefront from pc0 until pc_end (exclusive) or the
// end.  M_MAIN: whole threads; at the expanded loop each lane's trip count,
// start, step and live-ins are stored with the tile's prefix of trip counts
// and the loop is left at once (its iterations run in the body pass).  M_BODY:
// registers hold the live-ins and the counter of iteration ln.k0; runs the body.
// M_FIX: replays lane 0 towards the target access and stops there.
template <int MODE>
__device__ void run_program(GenLds& S, uint64_t* R, Ctx& C, Lane& ln, uint64_t& sat, uint32_t pc0,
                            uint32_t pc_end) {
  c_dprog* P = C.P;
  c_dins* I = C.I;
  if (MODE == M_BODY) {
    // live-ins of the owner thread, counter of this iteration
    const uint64_t l = C.lane0;  // lane index of the owner (set per lane)
    const uint32_t nl = P->n_livein;
    for (uint32_t q = 0; q < nl; q++) RPUT(ufirst(P->livein[q]), C.xs[(3 + q) * C.xn + l]);
    const dins L = ld_ins(I, pc0 - 1);
    RPUT(ufirst(L.dst), narrow(C.xs[C.xn + l] + ln.k0 * C.xs[2 * C.xn + l], L.w));
  }
  uint32_t pc = pc0;
  while (pc < pc_end) {
    const dins D = ld_ins(I, pc);
    const uint32_t op = D.op, w = D.w;
    const uint32_t da = ufirst(D.a), db = ufirst(D.b), dc = ufirst(D.c), dd = ufirst(D.dst);
    // operands: a for every op that reads registers, b for binary ops, SELECT
    // and LOOP, c for SELECT and LOOP (uniform tests, no lane reads otherwise)
    const bool rd_a = op >= CKC_OP_ADD && op != CKC_OP_ELSE && op != CKC_OP_ENDIF && op != CKC_OP_ENDLOOP;
    const bool rd_b = (op >= CKC_OP_ADD && op <= CKC_OP_SELECT) || op == CKC_OP_LOOP;
    const bool rd_c = op == CKC_OP_SELECT || op == CKC_OP_LOOP;
    const uint64_t va = rd_a ? RGET(da) : 0, vb = rd_b ? RGET(db) : 0, vc = rd_c ? RGET(dc) : 0;
    const bool act = ln.dis == 0;
    uint64_t r = 0;
    uint32_t wreg = 0xFFu;   // register written after the switch
    uint32_t npc = pc + 1;
    switch (op) {
      case CKC_OP_CONST: r = narrow((uint64_t)C.K[D.x], w); wreg = dd; break;
      case CKC_OP_SCALAR: r = narrow((uint64_t)C.sc[D.x], w); wreg = dd; break;
      case CKC_OP_SPECIAL: {
        const uint32_t x = D.x;
        uint32_t v;
        switch (x) {
          case 0: v = C.t0; break;
          case 1: v = C.t1; break;
          case 2: v = C.t2; break;
          case 3: v = C.b0; break;
          case 4: v = C.b1; break;
          case 5: v = C.b2; break;
          default: v = x < 9 ? C.in->launch[3 + x - 6] : C.in->launch[x - 9]; break;
        }
        r = v;
        wreg = dd;
        break;
      }
      case CKC_OP_SELECT: r = narrow(va != 0 ? vb : vc, w); wreg = dd; break;
      case CKC_OP_SEXT: case CKC_OP_TRUNC: r = narrow(va, 32); wreg = dd; break;
      case CKC_OP_ZEXT: r = va & 0xFFFFFFFFull; wreg = dd; break;
      case CKC_OP_ACCESS:
      case CKC_OP_LOAD: {
        const uint32_t slot = D.slot, lg = D.fl & 3u, acc = D.x;
        const int64_t idx = (int64_t)narrow(va, w);
        c_alloc& A = C.tab[slot];
        const uint32_t kd = act ? kind_of(A.base, A.size_bytes, A.flags, idx, lg) : 0u;
        if (MODE != M_FIX) {
          ln.acc += act ? 1u : 0u;
          count_site(S, C, sat, D.s0, __ballot(act));
          if (__ballot(kd != 0)) {
            const uint64_t key = (ln.gtid << C.Lsum) | (ln.k0 << C.L2) | ln.k1;
            merge_violation(C.rec + acc, kd, key);
          }
        } else if (acc == C.tacc) {
          if (lane_id() == 0) { C.trec->index = idx; C.trec->first_kind = kd; }
          return;
        }
        if (op == CKC_OP_LOAD) {
          uint64_t v = 0;
          if (act && kd == 0)
            v = lg == 2 ? (uint64_t)(int64_t)((const int32_t*)A.data)[idx] : (uint64_t)((const int64_t*)A.data)[idx];
          r = v;
          wreg = dd;
        }
        break;
      }
      case CKC_OP_IF: {
        const bool p = va != 0;
        if (MODE != M_FIX) {
          count_site(S, C, sat, D.s0, __ballot(act && p));
          count_site(S, C, sat, D.s1, __ballot(act && !p));
        }
        ln.dis = act ? (p ? 0u : 1u) : ln.dis + 1;
        if (!(D.fl & DI_NOSKIP) && __ballot(ln.dis == 0) == 0) npc = D.jmp;  // ELSE / ENDIF handle it
        break;
      }
      case CKC_OP_ELSE:
        ln.dis = ln.dis == 1 ? 0u : (ln.dis == 0 ? 1u : ln.dis);
        if (!(D.fl & DI_NOSKIP) && __ballot(ln.dis == 0) == 0) npc = D.jmp;
        break;
      case CKC_OP_ENDIF: ln.dis = ln.dis > 0 ? ln.dis - 1 : 0u; break;
      case CKC_OP_LOOP: {
        const uint32_t d = D.x, fl = D.fl, endpc = D.jmp;
        const int64_t s0 = (int64_t)narrow(va, w), e0 = (int64_t)narrow(vb, w), stp = (int64_t)narrow(vc, w);
        if (MODE == M_FIX) {
          const int32_t me = (int32_t)pc;
          if (me != C.tloop0 && me != C.tloop1) { npc = endpc + 1; break; }
          const uint64_t kk = me == C.tloop0 ? C.tk0 : C.tk1;
          r = narrow((uint64_t)s0 + kk * (uint64_t)stp, w);
          wreg = dd;
          if (d == 0) ln.k0 = kk; else ln.k1 = kk;
          break;  // into the body for exactly the target iteration
        }
        const uint64_t nt = act ? trip_count(s0, e0, stp) : 0;
        const uint64_t cap = d == 0 ? C.cap0 : C.cap1;
        const uint64_t rn = nt < cap ? nt : cap;
        const bool hg = act && nt > cap;
        if (MODE == M_MAIN && (fl & DI_EXPAND) && C.xs != nullptr) {
          // every wavefront of the workgroup arrives here exactly once per tile:
          // prefix of the trip counts over the tile, thread state to memory
          const uint32_t tid = threadIdx.x;
          const uint64_t cnt = act ? rn : 0;
          uint64_t incl = cnt;
          for (int o = 1; o < 64; o <<= 1) {
            const uint64_t u = __shfl_up((unsigned long long)incl, o, 64);
            if ((int)lane_id() >= o) incl += u;
          }
          if (lane_id() == 63) S.wsum[tid / 64] = incl;
          __syncthreads();
          uint64_t wpre = 0;
          for (uint32_t q = 0; q < tid / 64; q++) wpre += S.wsum[q];
          const uint64_t pre = wpre + incl - cnt;
          const uint64_t l = C.lane0 + tid;
          C.xs[l] = pre;
          if (cnt) {
            C.xs[C.xn + l] = (uint64_t)s0;
            C.xs[2 * C.xn + l] = (uint64_t)stp;
            const uint32_t nl = P->n_livein;
            for (uint32_t q = 0; q < nl; q++) C.xs[(3 + q) * C.xn + l] = RGET(ufirst(P->livein[q]));
          }
          if (tid == TILE - 1) {
            const uint64_t tot = pre + cnt;
            C.xtot[C.xt] = tot;
            C.xpb[C.xt] = (tot + PIECE - 1) / PIECE;
            C.xin[C.xt] = C.input;
          }
          __syncthreads();
          // the loop is left at once: lanes that run it to the end pass its
          // exit, lanes over the cap stop
          count_site(S, C, sat, D.s1, __ballot(act && !hg));
          if (hg) { ln.dis = DEAD; ln.hangs++; }
          npc = endpc + 1;
          break;
        }
        if (d == 0) { ln.run0 = rn; ln.st0 = (uint64_t)s0; ln.sp0 = (uint64_t)stp; ln.k0 = 0; }
        else { ln.run1 = rn; ln.st1 = (uint64_t)s0; ln.sp1 = (uint64_t)stp; ln.k1 = 0; }
        ln.hangp = (ln.hangp & ~(1u << d)) | (hg ? (1u << d) : 0u);
        ln.dis = act ? (rn > 0 ? 0u : 1u) : ln.dis + 1;
        if (__ballot(ln.dis == 0) == 0) { npc = endpc; break; }  // ENDLOOP: exit handling
        r = narrow((uint64_t)s0, w);
        wreg = dd;
        count_site(S, C, sat, D.s0, __ballot(ln.dis == 0));
        break;
      }
      case CKC_OP_ENDLOOP: {
        if (MODE == M_FIX) return;  // target not reached in this iteration
        const uint32_t d = D.x, lpc = D.jmp;
        const dins Lp = ld_ins(I, lpc);
        if (ln.dis == 0) {
          const uint64_t kk = (d == 0 ? ln.k0 : ln.k1) + 1;
          if (d == 0) ln.k0 = kk; else ln.k1 = kk;
          if (kk == (d == 0 ? ln.run0 : ln.run1)) ln.dis = 1;  // done at this level
        }
        if (__ballot(ln.dis == 0)) {
          const uint64_t kk = d == 0 ? ln.k0 : ln.k1;
          const uint64_t sa = d == 0 ? ln.st0 : ln.st1, sp = d == 0 ? ln.sp0 : ln.sp1;
          wreg = ufirst(Lp.dst);
          // lanes that left the loop keep their value
          r = ln.dis == 0 ? narrow(sa + kk * sp, Lp.w) : RGET(wreg);
          count_site(S, C, sat, Lp.s0, __ballot(ln.dis == 0));
          npc = lpc + 1;
          break;
        }
        // exit: lanes that ran this loop leave it; a capped loop stops its lane
        const bool mine = ln.dis == 1;
        const bool hg = mine && ((ln.hangp >> d) & 1u);
        count_site(S, C, sat, Lp.s1, __ballot(mine && !hg));
        if (mine) {
          if (hg) { ln.dis = DEAD; ln.hangs++; }
          else ln.dis = 0;
        } else if (ln.dis > 1) {
          ln.dis--;
        }
        if (d == 0) ln.k0 = 0; else ln.k1 = 0;
        break;
      }
      default: {
        uint32_t f = 0;
        r = alu(op, w, va, vb, f);
        if (act) ln.faults += f;
        wreg = dd;
        break;
      }
    }
    if (wreg != 0xFFu) RPUT(wreg, r);
    pc = npc;
  }
}

__device__ void flush_input(GenLds& S, const KArgs& a, uint32_t input, uint32_t n_sites) {
  __syncthreads();
  const dinput& in = a.inputs[input];
  uint32_t* cnt = a.counts + in.cnt_base;
  const uint32_t ns = n_sites < (uint32_t)MAX_SITES_LDS ? n_sites : (uint32_t)MAX_SITES_LDS;
  for (uint32_t s = threadIdx.x; s < ns; s += TILE) {
    uint32_t c = S.sites[s];
    if (c) {
      if (cnt[s] < 255u) atomicAdd(&cnt[s], c < 255u ? c : 255u);
      S.sites[s] = 0;
    }
  }
  if (threadIdx.x == 0) {
    ckc_input_status* st = a.status + input;
    if (S.acc_checked) atomicAdd((unsigned long long*)&st->accesses_checked, S.acc_checked);
    if (S.hangs) atomicAdd((unsigned long long*)&st->hang_lanes, S.hangs);
    if (S.faults) atomicAdd((unsigned long long*)&st->arith_faults, S.faults);
    S.acc_checked = 0; S.hangs = 0; S.faults = 0;
  }
  __syncthreads();
}

__device__ __forceinline__ void ctx_init(Ctx& C, const KArgs& a, const dinput& in, uint32_t i, const Thr& T) {
  C.in = &in;
  C.P = (c_dprog*)in.prog;
  C.I = (c_dins*)((const uint8_t*)in.prog + C.P->off_instr);
  C.K = (c_i64*)((const uint8_t*)in.prog + C.P->off_consts);
  C.sc = a.scalars + (size_t)i * MAX_SCALARS;
  C.tab = (c_alloc*)in.table;
  C.rec = a.recs + in.rec_base;
  C.gcnt = a.counts + in.cnt_base;
  C.Lsum = in.L1 + in.L2;
  C.L2 = in.L2;
  C.cap0 = 1ull << in.cap_log2[0];
  C.cap1 = 1ull << in.cap_log2[1];
  C.t0 = T.t[0]; C.t1 = T.t[1]; C.t2 = T.t[2]; C.b0 = T.b[0]; C.b1 = T.b[1]; C.b2 = T.b[2];
  C.xs = (uint64_t*)in.xstate;
  C.xn = in.xn;
  C.xtot = a.xtot;
  C.xpb = a.xpb;
  C.xin = a.xin;
  C.input = i;
  C.lane0 = 0;
  C.xt = 0;
}

__device__ __forceinline__ void lane_init(Lane& ln, bool act, uint64_t gtid) {
  ln.dis = act ? 0u : DEAD;
  ln.k0 = ln.k1 = ln.run0 = ln.run1 = ln.st0 = ln.st1 = ln.sp0 = ln.sp1 = 0;
  ln.hangp = 0;
  ln.gtid = gtid;
  ln.faults = 0;
  ln.hangs = 0;
  ln.acc = 0;
}

__device__ __forceinline__ void add_lane_totals(GenLds& S, const Lane& ln) {
  const uint64_t f = wave_sum64(ln.faults), h = wave_sum64(ln.hangs), n = wave_sum64(ln.acc);
  if (lane_id() == 0) {
    if (f) atomicAdd(&S.faults, (unsigned long long)f);
    if (h) atomicAdd(&S.hangs, (unsigned long long)h);
    if (n) atomicAdd(&S.acc_checked, (unsigned long long)n);
  }
}

// The interpreter over whole threads: one lane per thread of the thread set.
template <uint32_t SK>
__global__ void __launch_bounds__(TILE) eval_generic_kernel(KArgs a) {
  __shared__ GenLds S;
  extern __shared__ uint64_t R[];  // [n_regs][TILE]
  __shared__ unsigned long long item_slot;
  const uint32_t tid = threadIdx.x;
  const uint64_t total = a.js->total_tiles[PATH_GENERIC];
  if (total == 0) return;
  Sched<SK> sc;
  sched_init(sc, a, total);
  if (SK == CKC_SCHED_BLOCKED && sc.cur >= sc.end) return;
  c_input* ins = (c_input*)a.inputs;
  c_u32* order = (c_u32*)a.order;
  for (uint32_t s = tid; s < MAX_SITES_LDS; s += TILE) S.sites[s] = 0;
  if (tid == 0) { S.acc_checked = 0; S.hangs = 0; S.faults = 0; }
  uint32_t pos = 0xFFFFFFFFu, cur = 0xFFFFFFFFu, cur_sites = 0;
  uint64_t tb = 0, cur_end = 0, sat = 0;
  Dec dec;
  for (;;) {
    __syncthreads();
    const uint64_t t = sched_next(sc, &a.js->next_tile[PATH_GENERIC], &item_slot);
    if (t == ~0ull) break;
    if (pos == 0xFFFFFFFFu || t < tb || t >= cur_end) {
      pos = pos_of_tile(ins, order, a.n_inputs, PATH_GENERIC, pos, cur_end, t);
      const uint32_t i = order[pos];
      if (cur != 0xFFFFFFFFu) flush_input(S, a, cur, cur_sites);
      sat = 0;
      cur = i;
      cur_sites = ((c_dprog*)a.inputs[i].prog)->n_sites;
      tb = ins[i].tile_begin[PATH_GENERIC];
      cur_end = tb + ins[i].n_tiles[PATH_GENERIC];
      const uint32_t L6[6] = {ins[i].launch[0], ins[i].launch[1], ins[i].launch[2],
                              ins[i].launch[3], ins[i].launch[4], ins[i].launch[5]};
      dec_make(dec, L6);
    }
    const uint32_t i = cur;
    const dinput& in = a.inputs[i];
    const uint64_t l = (t - tb) * TILE + tid;
    const bool act = l < in.lanes;
    Thr T;
    if (in.mode == CKC_FULL) decode_full(dec, act ? l : 0, T);
    else decode_lane(in.mode, in.launch, act ? l : 0, T);
    Ctx C;
    ctx_init(C, a, in, i, T);
    C.lane0 = (t - tb) * TILE;
    C.xt = in.xt_begin + (t - tb);
    Lane ln;
    lane_init(ln, act, T.gtid);
    run_program<M_MAIN>(S, R, C, ln, sat, 0, C.P->n_instr);
    add_lane_totals(S, ln);
  }
  if (cur != 0xFFFFFFFFu) flush_input(S, a, cur, cur_sites);
}

// Exclusive scan, in place, of the per-tile piece counts of expanded loops
// (a.xpb, a.n_xtiles entries) in three steps: per-block sums of XSB entries,
// a scan of the block sums (which also stores the total), per-block rescans.
constexpr uint32_t XSB = 4096;
__global__ void __launch_bounds__(256) xscan_sums_kernel(KArgs a) {
  __shared__ unsigned long long part[4];
  const uint64_t b0 = (uint64_t)blockIdx.x * XSB;
  unsigned long long v = 0;
  for (uint32_t q = threadIdx.x; q < XSB; q += 256)
    if (b0 + q < a.n_xtiles) v += a.xpb[b0 + q];
  v = wave_sum64(v);
  if (lane_id() == 0) part[threadIdx.x / 64] = v;
  __syncthreads();
  if (threadIdx.x == 0) a.xbsum[blockIdx.x] = part[0] + part[1] + part[2] + part[3];
}
__global__ void __launch_bounds__(1024) xscan_blocks_kernel(KArgs a, uint32_t n_blocks) {
  __shared__ unsigned long long part[16];
  __shared__ unsigned long long carry;
  const uint32_t t = threadIdx.x;
  if (t == 0) carry = 0;
  __syncthreads();
  for (uint32_t base = 0; base < n_blocks; base += 1024) {
    const uint32_t i = base + t;
    const uint64_t v = i < n_blocks ? a.xbsum[i] : 0;
    uint64_t sc = v;
    for (int o = 1; o < 64; o <<= 1) {
      const uint64_t u = __shfl_up((unsigned long long)sc, o, 64);
      if ((int)lane_id() >= o) sc += u;
    }
    if (lane_id() == 63) part[t / 64] = sc;
    __syncthreads();
    uint64_t w = 0;
    for (uint32_t q = 0; q < t / 64; q++) w += part[q];
    const uint64_t c = carry;
    if (i < n_blocks) a.xbsum[i] = c + w + sc - v;
    __syncthreads();
    if (t == 1023) carry = c + w + sc;
    __syncthreads();
  }
  if (t == 0) {
    a.js->total_pieces = carry;
    a.js->next_piece = 0;
  }
}
__global__ void __launch_bounds__(256) xscan_apply_kernel(KArgs a) {
  __shared__ unsigned long long part[4];
  __shared__ unsigned long long carry;
  const uint64_t b0 = (uint64_t)blockIdx.x * XSB;
  if (threadIdx.x == 0) carry = a.xbsum[blockIdx.x];
  __syncthreads();
  for (uint32_t base = 0; base < XSB; base += 256) {
    const uint64_t e = b0 + base + threadIdx.x;
    const uint64_t v = e < a.n_xtiles ? a.xpb[e] : 0;
    uint64_t sc = v;
    for (int o = 1; o < 64; o <<= 1) {
      const uint64_t u = __shfl_up((unsigned long long)sc, o, 64);
      if ((int)lane_id() >= o) sc += u;
    }
    if (lane_id() == 63) part[threadIdx.x / 64] = sc;
    __syncthreads();
    uint64_t w = 0;
    for (uint32_t q = 0; q < threadIdx.x / 64; q++) w += part[q];
    const uint64_t c = carry;
    if (e < a.n_xtiles) a.xpb[e] = c + w + sc - v;
    __syncthreads();
    if (threadIdx.x == 255) carry = c + w + sc;
    __syncthreads();
  }
}

// Expanded tile of piece p: the largest xt with xpb[xt] <= p (it has pieces,
// since the next tile starts after p).
__device__ __forceinline__ uint64_t find_xtile(const unsigned long long* xpb, uint64_t n, uint64_t p) {
  uint64_t lo = 0, hi = n - 1;
  while (lo < hi) {
    const uint64_t mid = lo + (hi - lo + 1) / 2;
    if (xpb[mid] <= p) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

// The body pass of expanded loops: work items are pieces of PIECE consecutive
// iterations of one tile's flattened iteration space; each lane runs one
// iteration (owner thread by binary search in the tile's prefix).
template <uint32_t SK>
__global__ void __launch_bounds__(TILE) eval_body_kernel(KArgs a) {
  __shared__ GenLds S;
  extern __shared__ uint64_t R[];  // [n_regs][TILE]
  __shared__ unsigned long long item_slot;
  const uint32_t tid = threadIdx.x;
  const uint64_t total = a.js->total_pieces;
  if (total == 0) return;
  Sched<SK> sc;
  sched_init(sc, a, total);
  if (SK == CKC_SCHED_BLOCKED && sc.cur >= sc.end) return;
  for (uint32_t s = tid; s < MAX_SITES_LDS; s += TILE) S.sites[s] = 0;
  if (tid == 0) { S.acc_checked = 0; S.hangs = 0; S.faults = 0; }
  uint32_t cur = 0xFFFFFFFFu, cur_sites = 0;
  uint64_t cur_xt = ~0ull, sat = 0;
  Dec dec;
  for (;;) {
    __syncthreads();
    const uint64_t p = sched_next(sc, &a.js->next_piece, &item_slot);
    if (p == ~0ull) break;
    const uint64_t xt = ufirst64(find_xtile(a.xpb, a.n_xtiles, p));
    const uint32_t i = ufirst(a.xin[xt]);
    const dinput& in = a.inputs[i];
    if (i != cur) {
      if (cur != 0xFFFFFFFFu) flush_input(S, a, cur, cur_sites);
      sat = 0;
      cur = i;
      cur_sites = ((c_dprog*)in.prog)->n_sites;
      const uint32_t L6[6] = {in.launch[0], in.launch[1], in.launch[2], in.launch[3], in.launch[4], in.launch[5]};
      dec_make(dec, L6);
    }
    const uint64_t lane0 = (xt - in.xt_begin) * TILE;
    const uint64_t* xs = (const uint64_t*)in.xstate;
    if (xt != cur_xt) {
      S.pref[tid] = xs[lane0 + tid];
      if (tid == 0) S.pref[TILE] = a.xtot[xt];
      cur_xt = xt;
      __syncthreads();
    }
    const uint64_t it0 = (p - a.xpb[xt]) * PIECE;
    const uint64_t tot = S.pref[TILE];
    const uint64_t it1 = it0 + PIECE < tot ? it0 + PIECE : tot;
    c_dprog* P = (c_dprog*)in.prog;
    const uint32_t lpc = (uint32_t)P->expand_pc;
    const uint32_t endpc = ld_ins((c_dins*)((const uint8_t*)in.prog + P->off_instr), lpc).jmp;
    for (uint64_t base = it0; base < it1; base += TILE) {
      const uint64_t g = base + tid;
      const bool ga = g < it1;
      uint32_t o = 0;
      if (ga) {
        uint32_t l2 = 0, h2 = TILE - 1;
        while (l2 < h2) {
          const uint32_t m = (l2 + h2 + 1) >> 1;
          if (S.pref[m] <= g) l2 = m;
          else h2 = m - 1;
        }
        o = l2;
      }
      const uint64_t l = lane0 + o;
      Thr T;
      if (in.mode != CKC_FULL) {
        decode_lane(in.mode, in.launch, l, T);
      } else if (P->body_special) {
        decode_full(dec, l, T);
      } else {  // the body reads no thread coordinate
        T.t[0] = T.t[1] = T.t[2] = T.b[0] = T.b[1] = T.b[2] = 0;
        T.gtid = l;
      }
      Ctx C;
      ctx_init(C, a, in, i, T);
      C.lane0 = l;
      Lane ln;
      lane_init(ln, ga, T.gtid);
      ln.k0 = ga ? g - S.pref[o] : 0;
      count_site(S, C, sat, ld_ins(C.I, lpc).s0, __ballot(ga));
      run_program<M_BODY>(S, R, C, ln, sat, lpc + 1, endpc);
      add_lane_totals(S, ln);
    }
  }
  if (cur != 0xFFFFFFFFu) flush_input(S, a, cur, cur_sites);
}

// One wavefront per record: replays the thread of first_key up to the access
// and stores the index and kind there.
__global__ void __launch_bounds__(64) fixup_kernel(KArgs a, uint64_t n_records) {
  __shared__ GenLds S;
  extern __shared__ uint64_t R[];  // [n_regs][TILE], lanes 0..63 used
  const uint64_t r = blockIdx.x;
  if (r >= n_records) return;
  ckc_record* rec = a.recs + r;
  if (rec->count == 0) return;
  // input owning record r
  uint32_t lo_i = 0, hi_i = a.n_inputs - 1;
  while (lo_i < hi_i) {
    uint32_t mid = (lo_i + hi_i + 1) / 2;
    if (a.inputs[mid].rec_base <= r) lo_i = mid; else hi_i = mid - 1;
  }
  const dinput& in = a.inputs[lo_i];
  const dprog* P = (const dprog*)in.prog;
  const uint32_t acc = (uint32_t)(r - in.rec_base);
  const uint64_t key = rec->first_key;
  const uint32_t Lsum = in.L1 + in.L2;
  const uint64_t gtid = Lsum >= 64 ? 0 : key >> Lsum;
  const uint64_t i1 = in.L1 ? (key >> in.L2) & ((1ull << in.L1) - 1) : 0;
  const uint64_t i2 = in.L2 ? key & ((1ull << in.L2) - 1) : 0;
  const uint32_t bs = in.launch[3] * in.launch[4] * in.launch[5];
  Thr T;
  thr_from(in.launch, gtid / bs, (uint32_t)(gtid % bs), T);
  const daccess A = prog_access(P)[acc];
  Ctx C;
  ctx_init(C, a, in, lo_i, T);
  C.tacc = acc;
  C.tk0 = i1;
  C.tk1 = i2;
  C.tloop0 = A.loop_pc[0];
  C.tloop1 = A.loop_pc[1];
  C.trec = rec;
  Lane ln;
  lane_init(ln, lane_id() == 0, gtid);
  uint64_t sat = 0;
  run_program<M_FIX>(S, R, C, ln, sat, 0, C.P->n_instr);
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
    for (uint32_t s = threadIdx.x; s < P->n_sites; s += blockDim.x) {
      uint32_t c = cnt[s];
      mb[ids[s]] = (uint8_t)(c > 255 ? 255 : c);
    }
  }
}

// ---------------------------------------------------------------------------
// host-callable launchers
// ---------------------------------------------------------------------------
hipError_t launch_plan(const KArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(plan_kernel, dim3(a.n_inputs), dim3(64), 0, s, a);
  return hipGetLastError();
}
hipError_t launch_scan(const KArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(scan_kernel, dim3(1), dim3(1024), 0, s, a);
  return hipGetLastError();
}
namespace {
KArgs with_sched(const KArgs& a, const EvalGrid& eg, uint32_t path) {
  KArgs k = a;
  k.sched = eg.sched[path];
  return k;
}
// Kernel of evaluator `path` compiled for schedule `sk`.
void* eval_fn(uint32_t path, uint32_t sk) {
  const uint32_t s = sched_impl(sk);
  if (path == PATH_BLOCKS)
    return s == CKC_SCHED_BLOCKED ? (void*)eval_trace_kernel<CKC_SCHED_BLOCKED>
         : s == CKC_SCHED_CYCLIC  ? (void*)eval_trace_kernel<CKC_SCHED_CYCLIC>
                                  : (void*)eval_trace_kernel<CKC_SCHED_DYNAMIC>;
  if (path == PATH_LANES)
    return s == CKC_SCHED_BLOCKED ? (void*)eval_trace_lanes_kernel<CKC_SCHED_BLOCKED>
         : s == CKC_SCHED_CYCLIC  ? (void*)eval_trace_lanes_kernel<CKC_SCHED_CYCLIC>
                                  : (void*)eval_trace_lanes_kernel<CKC_SCHED_DYNAMIC>;
  return s == CKC_SCHED_BLOCKED ? (void*)eval_generic_kernel<CKC_SCHED_BLOCKED>
       : s == CKC_SCHED_CYCLIC  ? (void*)eval_generic_kernel<CKC_SCHED_CYCLIC>
                                : (void*)eval_generic_kernel<CKC_SCHED_DYNAMIC>;
}
hipError_t launch_eval(const KArgs& a, const EvalGrid& eg, uint32_t path, hipStream_t s) {
  KArgs k = with_sched(a, eg, path);
  void* args[] = {&k};
  return hipLaunchKernel(eval_fn(path, eg.sched[path]), dim3(eg.n_wg[path]), dim3(TILE), args,
                         path == PATH_GENERIC ? regfile_bytes(a) : 0, s);
}
}  // namespace

hipError_t launch_eval_trace(const KArgs& a, const EvalGrid& eg, hipStream_t s) {
  return launch_eval(a, eg, PATH_BLOCKS, s);
}
hipError_t launch_eval_trace_lanes(const KArgs& a, const EvalGrid& eg, hipStream_t s) {
  return launch_eval(a, eg, PATH_LANES, s);
}
hipError_t launch_eval_generic(const KArgs& a, const EvalGrid& eg, hipStream_t s) {
  return launch_eval(a, eg, PATH_GENERIC, s);
}
static void* body_fn(uint32_t sk) {
  const uint32_t s = sched_impl(sk);
  return s == CKC_SCHED_BLOCKED ? (void*)eval_body_kernel<CKC_SCHED_BLOCKED>
       : s == CKC_SCHED_CYCLIC  ? (void*)eval_body_kernel<CKC_SCHED_CYCLIC>
                                : (void*)eval_body_kernel<CKC_SCHED_DYNAMIC>;
}
static uint32_t xscan_blocks(const KArgs& a) { return (uint32_t)((a.n_xtiles + XSB - 1) / XSB); }

hipError_t launch_expand(const KArgs& a, const EvalGrid& eg, hipStream_t s) {
  if (a.n_xtiles == 0) return hipSuccess;
  const uint32_t nb = xscan_blocks(a);
  hipLaunchKernelGGL(xscan_sums_kernel, dim3(nb), dim3(256), 0, s, a);
  hipLaunchKernelGGL(xscan_blocks_kernel, dim3(1), dim3(1024), 0, s, a, nb);
  hipLaunchKernelGGL(xscan_apply_kernel, dim3(nb), dim3(256), 0, s, a);
  KArgs k = with_sched(a, eg, PATH_GENERIC);
  void* args[] = {&k};
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  return hipLaunchKernel(body_fn(eg.sched[PATH_GENERIC]), dim3(eg.n_wg[PATH_GENERIC]), dim3(TILE), args,
                         regfile_bytes(a), s);
}

hipError_t launch_fixup(const KArgs& a, uint64_t n_records, hipStream_t s) {
  if (n_records == 0) return hipSuccess;
  hipLaunchKernelGGL(fixup_kernel, dim3((uint32_t)n_records), dim3(64), regfile_bytes(a), s, a, n_records);
  return hipGetLastError();
}
hipError_t launch_finish(const KArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(finish_kernel, dim3(a.n_inputs), dim3(256), 0, s, a);
  return hipGetLastError();
}

namespace {
hipError_t add_node(hipGraph_t g, hipGraphNode_t* node, const hipGraphNode_t* deps, size_t n_deps, void* fn,
                    uint32_t grid, uint32_t block, void** args, uint32_t smem = 0) {
  hipKernelNodeParams p;
  std::memset(&p, 0, sizeof p);
  p.func = fn;
  p.gridDim = dim3(grid);
  p.blockDim = dim3(block);
  p.sharedMemBytes = smem;
  p.kernelParams = args;
  p.extra = nullptr;
  return hipGraphAddKernelNode(node, g, deps, n_deps, &p);
}
}  // namespace

hipError_t build_job_graph(hipGraph_t g, const KArgs& a, const EvalGrid& eg, uint64_t n_records) {
  KArgs ka = a;
  KArgs kp[3] = {with_sched(a, eg, 0), with_sched(a, eg, 1), with_sched(a, eg, 2)};
  uint64_t nr = n_records;
  void* args1[] = {&ka};
  void* args2[] = {&ka, &nr};
  void* argsp[3][1] = {{&kp[0]}, {&kp[1]}, {&kp[2]}};
  hipGraphNode_t plan, scan, ev[3], fix, fin;
  hipError_t e = add_node(g, &plan, nullptr, 0, (void*)plan_kernel, a.n_inputs, 64, args1);
  if (e == hipSuccess) e = add_node(g, &scan, &plan, 1, (void*)scan_kernel, 1, 1024, args1);
  if (e == hipSuccess)
    e = add_node(g, &ev[0], &scan, 1, eval_fn(PATH_BLOCKS, eg.sched[PATH_BLOCKS]), eg.n_wg[PATH_BLOCKS], TILE,
                 argsp[PATH_BLOCKS]);
  if (e == hipSuccess)
    e = add_node(g, &ev[1], &scan, 1, eval_fn(PATH_GENERIC, eg.sched[PATH_GENERIC]), eg.n_wg[PATH_GENERIC], TILE,
                 argsp[PATH_GENERIC], regfile_bytes(a));
  if (e == hipSuccess)
    e = add_node(g, &ev[2], &scan, 1, eval_fn(PATH_LANES, eg.sched[PATH_LANES]), eg.n_wg[PATH_LANES], TILE,
                 argsp[PATH_LANES]);
  if (e != hipSuccess) return e;
  if (a.n_xtiles) {  // generic -> scan of pieces -> body pass
    uint32_t nb = xscan_blocks(a);
    void* argsb[] = {&ka, &nb};
    hipGraphNode_t x1, x2, x3, xb;
    e = add_node(g, &x1, &ev[1], 1, (void*)xscan_sums_kernel, nb, 256, args1);
    if (e == hipSuccess) e = add_node(g, &x2, &x1, 1, (void*)xscan_blocks_kernel, 1, 1024, argsb);
    if (e == hipSuccess) e = add_node(g, &x3, &x2, 1, (void*)xscan_apply_kernel, nb, 256, args1);
    if (e == hipSuccess)
      e = add_node(g, &xb, &x3, 1, body_fn(eg.sched[PATH_GENERIC]), eg.n_wg[PATH_GENERIC], TILE, argsp[PATH_GENERIC],
                   regfile_bytes(a));
    if (e != hipSuccess) return e;
    ev[1] = xb;
  }
  hipGraphNode_t last = nullptr;
  if (n_records) {
    e = add_node(g, &fix, ev, 3, (void*)fixup_kernel, (uint32_t)n_records, 64, args2, regfile_bytes(a));
    last = fix;
  }
  if (e == hipSuccess)
    e = add_node(g, &fin, last ? &last : ev, last ? 1 : 3, (void*)finish_kernel, a.n_inputs, 256, args1);
  return e;
}

}  // namespace ckc
