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

#include "../../include/ckc.h"
#include "dformat.h"
#include "kernels.h"

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
  uint32_t n_ent = 0, n_cls = 0, overflow = 0, hang = 0;
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
    dtrace_entry* te = (dtrace_entry*)(th + 1);
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
    uint32_t tv = 0;
    const uint32_t bs = in.launch[3] * in.launch[4] * in.launch[5];
    if (path == 0 && in.mode != CKC_REP_CORNERS && bs % 64u == 0 &&
        ((const dtrace_head*)in.trace)->n_classes == 1) {
      // block-major jobs: (64-thread slice position, group of LPB set blocks)
      const uint64_t nsb = in.mode == CKC_FULL ? (uint64_t)in.launch[0] * in.launch[1] * in.launch[2]
                                               : bset_size(in.launch);
      const uint64_t jobs = (uint64_t)(bs / 64u) * ((nsb + LPB - 1) / LPB);
      tiles = (jobs + 3) / 4;
      tv = 1;
    }
    in.lanes = lanes;
    in.path = path;
    in.tv = tv;
    in.n_tiles[0] = path == 0 ? (uint32_t)tiles : 0;
    in.n_tiles[1] = path == 1 ? (uint32_t)tiles : 0;
  }
}

// Exclusive prefix of per-input tile counts for both evaluators.
__global__ void __launch_bounds__(1024) scan_kernel(KArgs a) {
  __shared__ unsigned long long part[2][1024 / 64];
  __shared__ unsigned long long carry[2];
  const uint32_t t = threadIdx.x;
  if (t < 2) carry[t] = 0;
  __syncthreads();
  for (uint32_t base = 0; base < a.n_inputs; base += 1024) {
    uint32_t i = base + t;
    uint64_t v0 = i < a.n_inputs ? a.inputs[i].n_tiles[0] : 0;
    uint64_t v1 = i < a.n_inputs ? a.inputs[i].n_tiles[1] : 0;
    // inclusive wave scan
    uint64_t s0 = v0, s1 = v1;
    for (int o = 1; o < 64; o <<= 1) {
      uint64_t u0 = __shfl_up((unsigned long long)s0, o, 64);
      uint64_t u1 = __shfl_up((unsigned long long)s1, o, 64);
      if ((int)lane_id() >= o) { s0 += u0; s1 += u1; }
    }
    if (lane_id() == 63) { part[0][t / 64] = s0; part[1][t / 64] = s1; }
    __syncthreads();
    uint64_t w0 = 0, w1 = 0;
    for (uint32_t q = 0; q < t / 64; q++) { w0 += part[0][q]; w1 += part[1][q]; }
    uint64_t c0 = carry[0], c1 = carry[1];
    if (i < a.n_inputs) {
      a.inputs[i].tile_begin[0] = c0 + w0 + s0 - v0;
      a.inputs[i].tile_begin[1] = c1 + w1 + s1 - v1;
    }
    __syncthreads();
    if (t == 1023) { carry[0] = c0 + w0 + s0; carry[1] = c1 + w1 + s1; }
    __syncthreads();
  }
  if (t == 0) {
    a.js->total_tiles[0] = carry[0];
    a.js->total_tiles[1] = carry[1];
    a.js->next_tile[0] = 0;
    a.js->next_tile[1] = 0;
  }
}

// Largest input index i with tile_begin[path][i] <= t (t < total).
__device__ __forceinline__ uint32_t find_input(const dinput* in, uint32_t n, uint32_t path, uint64_t t) {
  uint32_t lo = 0, hi = n - 1;
  while (lo < hi) {
    uint32_t mid = lo + (hi - lo + 1) / 2;
    if (in[mid].tile_begin[path] <= t) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

// ---------------------------------------------------------------------------
// trace evaluator
// ---------------------------------------------------------------------------
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

// Read-only job data is read through the constant address space so that
// wavefront-uniform loads become scalar loads.
typedef const __attribute__((address_space(4))) dtrace_entry c_entry;
typedef const __attribute__((address_space(4))) dtrace_head c_head;
typedef const __attribute__((address_space(4))) dinput c_input;
typedef const __attribute__((address_space(4))) jobstate c_jobstate;

__device__ __forceinline__ uint32_t find_input_c(c_input* in, uint32_t n, uint32_t path, uint64_t t) {
  uint32_t lo = 0, hi = n - 1;
  while (lo < hi) {
    uint32_t mid = lo + (hi - lo + 1) / 2;
    if (in[mid].tile_begin[path] <= t) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

// Rare path of one trace entry: some lane of the wavefront violates.
__device__ __noinline__ void trace_violation(ckc_record* rec, uint32_t bad, uint64_t gtid, uint32_t Lsum,
                                             uint64_t keylo) {
  merge_violation(rec, bad, (gtid << Lsum) | keylo);
}

// Checks of a trace whose entries all use one coefficient class of width W:
// per entry one add and one unsigned compare against the clamped bound.
template <int W>
__device__ __forceinline__ void trace_entries_1(c_entry* te, uint32_t ne, uint64_t base, bool act,
                                                ckc_record* rec, uint64_t gtid, uint32_t Lsum) {
  for (uint32_t e = 0; e < ne; e++) {
    const int64_t off = te[e].off;
    const uint64_t bound = te[e].bound;
    const uint32_t dead = te[e].dead_kind;
    uint32_t bad;
    if (W == 32) {
      const uint32_t v = (uint32_t)base + (uint32_t)off;
      bad = v >= (uint32_t)bound ? (((int32_t)v < 0) ? CKC_KIND_UNDER : CKC_KIND_OVER) : 0u;
    } else {
      const uint64_t v = base + (uint64_t)off;
      bad = v >= bound ? (((int64_t)v < 0) ? CKC_KIND_UNDER : CKC_KIND_OVER) : 0u;
    }
    if (dead) bad = dead;
    bad = act ? bad : 0u;
    if (__ballot(bad != 0)) trace_violation(rec + te[e].acc, bad, gtid, Lsum, te[e].keylo);
  }
}

// Block-major checks of one wavefront job: this lane's thread position
// (tlin) in up to LPB set blocks; tpart is the thread part of the index base,
// bp[j] the block parts (wavefront-uniform).  Per entry: one add for the
// thread part, then one add and one compare per block.
template <int W>
__device__ __forceinline__ void trace_blocks(c_entry* te, uint32_t ne, uint64_t tpart, const uint64_t* bp,
                                             const uint64_t* gb, uint32_t nvalid, uint32_t tlin,
                                             ckc_record* rec, uint32_t Lsum) {
  for (uint32_t e = 0; e < ne; e++) {
    const int64_t off = te[e].off;
    const uint64_t bound = te[e].bound;
    const uint32_t dead = te[e].dead_kind;
    uint64_t m = 0;
    uint32_t bad[LPB];
#pragma unroll
    for (uint32_t j = 0; j < LPB; j++) {
      if (W == 32) {
        const uint32_t v = (uint32_t)tpart + (uint32_t)off + (uint32_t)bp[j];
        bad[j] = v >= (uint32_t)bound ? (((int32_t)v < 0) ? CKC_KIND_UNDER : CKC_KIND_OVER) : 0u;
      } else {
        const uint64_t v = tpart + (uint64_t)off + bp[j];
        bad[j] = v >= bound ? (((int64_t)v < 0) ? CKC_KIND_UNDER : CKC_KIND_OVER) : 0u;
      }
      if (dead) bad[j] = dead;
      if (j >= nvalid) bad[j] = 0;
      m |= __ballot(bad[j] != 0);
    }
    if (m) {
      const uint32_t acc = te[e].acc;
      const uint64_t keylo = te[e].keylo;
#pragma unroll
      for (uint32_t j = 0; j < LPB; j++)
        if (__ballot(bad[j] != 0)) trace_violation(rec + acc, bad[j], gb[j] + tlin, Lsum, keylo);
    }
  }
}

__global__ void __launch_bounds__(TILE) eval_trace_kernel(KArgs a) {
  c_jobstate* js = (c_jobstate*)a.js;
  c_input* ins = (c_input*)a.inputs;
  const uint64_t total = js->total_tiles[0];
  if (total == 0) return;
  const uint64_t G = gridDim.x;
  const uint64_t t_begin = total * blockIdx.x / G, t_end = total * (blockIdx.x + 1) / G;
  if (t_begin >= t_end) return;
  const uint32_t tid = threadIdx.x;
  uint32_t i = find_input_c(ins, a.n_inputs, 0, t_begin);
  uint32_t cur = 0xFFFFFFFFu;
  // per-input state (wavefront-uniform)
  uint32_t L[6] = {0, 0, 0, 0, 0, 0};
  uint32_t bs = 1, gxy = 1, bxy = 1, mode = 0, Lsum = 0, ncls = 0, ne = 0, w0 = 32;
  UDiv dbs{1, 0}, dgx{1, 0}, dgxy{1, 0}, dbx{1, 0}, dbxy{1, 0}, dspb{1, 0};
  uint64_t lanes = 0, tb = 0, blin0 = 0, nsb = 0;
  uint32_t tlin0 = 0, tv = 0;
  int64_t k0 = 0, k1 = 0, k2 = 0, k3 = 0, k4 = 0, k5 = 0;
  c_head* th = nullptr;
  c_entry* te = nullptr;
  ckc_record* rec = nullptr;
  uint64_t cur_end = 0;
  for (uint64_t t = t_begin; t < t_end; t++) {
    if (t >= cur_end || cur == 0xFFFFFFFFu) {
      while (ins[i].n_tiles[0] == 0 || t >= ins[i].tile_begin[0] + ins[i].n_tiles[0]) i++;
      cur_end = ins[i].tile_begin[0] + ins[i].n_tiles[0];
    }
    if (i != cur) {
      cur = i;
      for (int q = 0; q < 6; q++) L[q] = ins[i].launch[q];
      bs = L[3] * L[4] * L[5];
      gxy = L[0] * L[1];
      bxy = L[3] * L[4];
      dbs = udiv_make(bs); dgx = udiv_make(L[0]); dgxy = udiv_make(gxy);
      dbx = udiv_make(L[3]); dbxy = udiv_make(bxy);
      dspb = udiv_make(bs >= 64 ? bs / 64u : 1u);
      mode = ins[i].mode;
      Lsum = ins[i].L1 + ins[i].L2;
      lanes = ins[i].lanes;
      tb = ins[i].tile_begin[0];
      th = (c_head*)ins[i].trace;
      te = (c_entry*)(th + 1);
      rec = a.recs + ins[i].rec_base;
      ncls = th->n_classes;
      ne = th->n_entries;
      w0 = th->cls_w[0];
      tv = ins[i].tv;
      nsb = mode == CKC_FULL ? (uint64_t)L[0] * L[1] * L[2] : bset_size(L);
      k0 = th->coef[0][0]; k1 = th->coef[0][1]; k2 = th->coef[0][2];
      k3 = th->coef[0][3]; k4 = th->coef[0][4]; k5 = th->coef[0][5];
      const uint64_t l0 = (t - tb) * TILE;
      blin0 = l0 / bs;
      tlin0 = (uint32_t)(l0 - blin0 * bs);
    }
    if (tv == 1) {
      // ---- block-major wavefront job ----
      const uint32_t wv = ufirst(tid >> 6);
      const uint64_t job = (t - tb) * 4 + wv;
      const uint32_t spb = bs / 64u;
      const uint64_t g = job < (1ull << 32) ? (uint64_t)udiv((uint32_t)job, dspb) : job / spb;
      const uint32_t o = (uint32_t)(job - g * spb);
      if (g * LPB >= nsb) continue;  // past the last group (whole wavefront)
      const uint32_t tlin = o * 64u + (tid & 63u);
      const uint32_t tz = udiv(tlin, dbxy), tr = tlin - tz * bxy;
      const uint32_t ty = udiv(tr, dbx);
      const uint32_t tx = tr - ty * L[3];
      uint64_t tpart = 0;
      if (k0 == 1) tpart += tx; else if (k0 != 0) tpart += (uint64_t)k0 * tx;
      if (k1 == 1) tpart += ty; else if (k1 != 0) tpart += (uint64_t)k1 * ty;
      if (k2 == 1) tpart += tz; else if (k2 != 0) tpart += (uint64_t)k2 * tz;
      uint64_t bp[LPB], gb[LPB];
      const uint64_t left = nsb - g * LPB;
      const uint32_t nvalid = left < LPB ? (uint32_t)left : LPB;
#pragma unroll
      for (uint32_t jj = 0; jj < LPB; jj++) {
        const uint64_t k = g * LPB + jj;
        const uint32_t blin = jj < nvalid ? (uint32_t)(mode == CKC_FULL ? k : bset_block(L, k)) : 0u;
        const uint32_t bz = udiv(blin, dgxy), brem = blin - bz * gxy;
        const uint32_t by = udiv(brem, dgx), bx = brem - by * L[0];
        bp[jj] = (uint64_t)k3 * bx + (uint64_t)k4 * by + (uint64_t)k5 * bz;
        gb[jj] = (uint64_t)blin * bs;
      }
      if (w0 == 32) trace_blocks<32>(te, ne, tpart, bp, gb, nvalid, tlin, rec, Lsum);
      else trace_blocks<64>(te, ne, tpart, bp, gb, nvalid, tlin, rec, Lsum);
      continue;
    }
    const uint64_t l = (t - tb) * TILE + tid;
    const bool act = l < lanes;
    uint32_t c6[6];
    uint64_t gtid;
    if (mode == CKC_FULL) {
      // consecutive lanes are consecutive threads: block carry by division
      const uint32_t u = tlin0 + tid;
      const uint32_t q = udiv(u, dbs);
      const uint32_t tlin = u - q * bs;
      uint32_t blin = (uint32_t)blin0 + q;
      if (bs % 64u == 0) blin = ufirst(blin);  // one block per wavefront
      const uint32_t z = udiv(blin, dgxy), r = blin - z * gxy;
      const uint32_t y = udiv(r, dgx);
      c6[3] = r - y * L[0]; c6[4] = y; c6[5] = z;
      const uint32_t tz = udiv(tlin, dbxy), tr = tlin - tz * bxy;
      const uint32_t ty = udiv(tr, dbx);
      c6[0] = tr - ty * L[3]; c6[1] = ty; c6[2] = tz;
      gtid = (uint64_t)blin * bs + tlin;
      // next tile
      tlin0 += TILE;
      const uint32_t qn = udiv(tlin0, dbs);
      blin0 += qn;
      tlin0 -= qn * bs;
    } else {
      Thr T;
      decode_lane(mode, L, act ? l : 0, T);
      c6[0] = T.t[0]; c6[1] = T.t[1]; c6[2] = T.t[2]; c6[3] = T.b[0]; c6[4] = T.b[1]; c6[5] = T.b[2];
      gtid = T.gtid;
    }
    // base of each coefficient class: sum of coefficient x coordinate, skipping
    // zero coefficients (uniform branches)
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
    if (ncls == 1) {
      if (w0 == 32) trace_entries_1<32>(te, ne, base[0], act, rec, gtid, Lsum);
      else trace_entries_1<64>(te, ne, base[0], act, rec, gtid, Lsum);
    } else {
      for (uint32_t e = 0; e < ne; e++) {
        const uint32_t c = te[e].cls;
        const uint64_t b = c == 0 ? base[0] : c == 1 ? base[1] : c == 2 ? base[2] : base[3];
        const uint64_t v = b + (uint64_t)te[e].off;
        uint32_t bad;
        if (te[e].w == 32) {
          const uint32_t v32 = (uint32_t)v;
          bad = v32 >= (uint32_t)te[e].bound ? (((int32_t)v32 < 0) ? CKC_KIND_UNDER : CKC_KIND_OVER) : 0u;
        } else {
          bad = v >= te[e].bound ? (((int64_t)v < 0) ? CKC_KIND_UNDER : CKC_KIND_OVER) : 0u;
        }
        if (te[e].dead_kind) bad = te[e].dead_kind;
        bad = act ? bad : 0u;
        if (__ballot(bad != 0)) trace_violation(rec + te[e].acc, bad, gtid, Lsum, te[e].keylo);
      }
    }
  }
}

// ---------------------------------------------------------------------------
// generic interpreter
// ---------------------------------------------------------------------------
struct GenLds {
  dins ins[MAX_DINSTR];
  int64_t consts[MAX_DCONST];
  ckc_alloc tab[MAX_SLOTS];
  uint32_t sites[MAX_SITES_LDS];
  // expanded loop: one entry per lane of the workgroup
  unsigned long long x_pref[TILE + 1];
  uint64_t x_start[TILE], x_step[TILE], x_gtid[TILE];
  uint64_t x_live[MAX_LIVEIN][TILE];
  unsigned long long wsum[TILE / 64];
  unsigned long long acc_checked, hangs, faults;
  uint64_t tile;
  uint32_t input;
  uint32_t n_instr;
};

enum { M_MAIN = 0, M_FIX = 1 };

struct Lane {
  uint32_t dis;            // 0 = active; >0 disabled depth; >= DEAD stopped
  uint64_t k0, k1;         // iteration ordinals at depth 0 / 1
  uint64_t run0, run1;     // iterations to run
  uint64_t st0, st1;       // loop start
  uint64_t sp0, sp1;       // loop step
  uint32_t hangp;          // bit d: the loop at depth d exceeds its cap
  uint64_t gtid;
  uint32_t faults, hangs;
};

struct Ctx {
  const dinput* in;
  const int64_t* sc;
  ckc_record* rec;
  uint32_t* gcnt;          // global site counters (sites beyond the LDS range)
  uint32_t Lsum, L2;
  uint64_t cap0, cap1;
  uint32_t t0, t1, t2, b0, b1, b2;  // thread coordinates (this lane)
  // fix-up target
  uint32_t tacc;
  uint64_t tk0, tk1;
  int32_t tloop0, tloop1;
  ckc_record* trec;
};

__device__ __forceinline__ void count_site(GenLds& S, const Ctx& C, uint32_t s, uint64_t mask) {
  if (s == NOSITE || mask == 0) return;
  if (lane_id() == (uint32_t)(__ffsll((unsigned long long)mask) - 1)) {
    uint32_t c = (uint32_t)__popcll(mask);
    if (s < MAX_SITES_LDS) {
      if (S.sites[s] < 255u) atomicAdd(&S.sites[s], c);
    } else if (C.gcnt[s] < 255u) {
      atomicAdd(&C.gcnt[s], c);
    }
  }
}

// Runs instructions [pc, pc_end) for the wavefront.  MODE M_MAIN checks,
// counts and records; M_FIX replays one thread (lane 0) towards the target
// access and stops there.  EXPAND allows the workgroup-wide expanded loop.
template <int MODE>
__device__ void run_program(GenLds& S, Ctx& C, Lane& ln, uint32_t* lo, uint32_t* hi, uint32_t n_instr) {
  // state of the expanded loop (one lane per iteration across the workgroup)
  bool in_x = false;
  uint64_t x_base = 0, x_total = 0;
  uint32_t x_lpc = 0, x_own_dis = 0, x_hang = 0, x_act = 0, x_nlive = 0;
  uint64_t x_own_gtid = 0;
  const dprog* P = (const dprog*)C.in->prog;
  uint32_t pc = 0;
  // Prepares chunk x_base of the expanded loop at LOOP pc `lpc`: every lane takes
  // one iteration of some thread of the workgroup ("owner" o).
  auto x_chunk = [&](uint32_t lpc) {
    const dins L = S.ins[lpc];
    const uint32_t tid = threadIdx.x;
    const uint64_t g = x_base + tid;
    const bool ga = g < x_total;
    uint32_t o = 0;
    if (ga) {  // last o with pref[o] <= g
      uint32_t l2 = 0, h2 = TILE - 1;
      while (l2 < h2) {
        uint32_t m = (l2 + h2 + 1) >> 1;
        if (S.x_pref[m] <= g) l2 = m; else h2 = m - 1;
      }
      o = l2;
    }
    const uint64_t kk = ga ? g - S.x_pref[o] : 0;
    for (uint32_t q = 0; q < x_nlive; q++) RSET(P->livein[q], S.x_live[q][o]);
    RSET(ufirst(L.dst), narrow(S.x_start[o] + kk * S.x_step[o], ufirst(L.w)));
    ln.dis = ga ? 0u : 1u;
    ln.gtid = S.x_gtid[o];
    ln.k0 = kk;
    ln.k1 = 0;
    count_site(S, C, ufirst(L.s0), __ballot(ga));
  };
  while (pc < n_instr) {
    const dins D = S.ins[pc];
    const uint32_t op = ufirst(D.op);
    const uint32_t w = ufirst(D.w);
    const uint32_t da = ufirst(D.a), db = ufirst(D.b), dc = ufirst(D.c), dd = ufirst(D.dst);
    const bool act = ln.dis == 0;
    switch (op) {
      case CKC_OP_CONST: RSET(dd, narrow((uint64_t)S.consts[ufirst(D.x)], w)); break;
      case CKC_OP_SCALAR: RSET(dd, narrow((uint64_t)C.sc[ufirst(D.x)], w)); break;
      case CKC_OP_SPECIAL: {
        const uint32_t x = ufirst(D.x);
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
        RSET(dd, (uint64_t)v);
        break;
      }
      case CKC_OP_SELECT: RSET(dd, narrow(rget(lo, hi, da) != 0 ? rget(lo, hi, db) : rget(lo, hi, dc), w)); break;
      case CKC_OP_SEXT: case CKC_OP_TRUNC: RSET(dd, narrow(rget(lo, hi, da), 32)); break;
      case CKC_OP_ZEXT: RSET(dd, rget(lo, hi, da) & 0xFFFFFFFFull); break;
      case CKC_OP_ACCESS:
      case CKC_OP_LOAD: {
        const uint32_t slot = ufirst(D.slot), lg = ufirst(D.fl) & 3u, acc = ufirst(D.x);
        const int64_t idx = (int64_t)narrow(rget(lo, hi, da), w);
        const ckc_alloc& A = S.tab[slot];
        uint32_t kd = act ? kind_of(A.base, A.size_bytes, A.flags, idx, lg) : 0u;
        if (MODE == M_MAIN) {
          uint64_t am = __ballot(act);
          if (lane_id() == 0 && am) atomicAdd(&S.acc_checked, (unsigned long long)__popcll(am));
          count_site(S, C, ufirst(D.s0), am);
          if (__ballot(kd != 0)) {
            uint64_t key = (ln.gtid << C.Lsum) | (ln.k0 << C.L2) | ln.k1;
            merge_violation(C.rec + acc, kd, key);
          }
        } else if (acc == C.tacc) {
          if (lane_id() == 0) { C.trec->index = idx; C.trec->first_kind = kd; }
          return;
        }
        if (op == CKC_OP_LOAD) {
          uint64_t v = 0;
          if (act && kd == 0) {
            v = lg == 2 ? (uint64_t)(int64_t)((const int32_t*)A.data)[idx]
                        : (uint64_t)((const int64_t*)A.data)[idx];
          }
          RSET(dd, v);
        }
        break;
      }
      case CKC_OP_IF: {
        const bool p = rget(lo, hi, da) != 0;
        const uint32_t fl = ufirst(D.fl);
        if (MODE == M_MAIN) {
          count_site(S, C, ufirst(D.s0), __ballot(act && p));
          count_site(S, C, ufirst(D.s1), __ballot(act && !p));
        }
        ln.dis = act ? (p ? 0u : 1u) : ln.dis + 1;
        if (!(fl & DI_NOSKIP) && __ballot(ln.dis == 0) == 0) {
          pc = ufirst(D.jmp);  // ELSE or ENDIF: handled there
          continue;
        }
        break;
      }
      case CKC_OP_ELSE: {
        ln.dis = ln.dis == 1 ? 0u : (ln.dis == 0 ? 1u : ln.dis);
        if (!(ufirst(D.fl) & DI_NOSKIP) && __ballot(ln.dis == 0) == 0) {
          pc = ufirst(D.jmp);
          continue;
        }
        break;
      }
      case CKC_OP_ENDIF: ln.dis = ln.dis > 0 ? ln.dis - 1 : 0u; break;
      case CKC_OP_LOOP: {
        const uint32_t d = ufirst(D.x), fl = ufirst(D.fl);
        const uint32_t endpc = ufirst(D.jmp);
        const int64_t s = (int64_t)narrow(rget(lo, hi, da), w);
        const int64_t e = (int64_t)narrow(rget(lo, hi, db), w);
        const int64_t stp = (int64_t)narrow(rget(lo, hi, dc), w);
        if (MODE == M_FIX) {
          const int32_t me = (int32_t)pc;
          if (me != C.tloop0 && me != C.tloop1) { pc = endpc + 1; continue; }
          const uint64_t kk = me == C.tloop0 ? C.tk0 : C.tk1;
          RSET(dd, narrow((uint64_t)s + kk * (uint64_t)stp, w));
          if (d == 0) ln.k0 = kk; else ln.k1 = kk;
          break;  // into the body for exactly the target iteration
        }
        const uint64_t nt = act ? trip_count(s, e, stp) : 0;
        const uint64_t cap = d == 0 ? C.cap0 : C.cap1;
        const uint64_t rn = nt < cap ? nt : cap;
        const bool hg = act && nt > cap;
        if (fl & DI_EXPAND) {
          // every wavefront of the workgroup arrives here exactly once per tile
          const uint32_t tid = threadIdx.x;
          x_nlive = ufirst(P->n_livein);
          S.x_start[tid] = (uint64_t)s;
          S.x_step[tid] = (uint64_t)stp;
          S.x_gtid[tid] = ln.gtid;
          for (uint32_t q = 0; q < x_nlive; q++) S.x_live[q][tid] = rget(lo, hi, P->livein[q]);
          const uint64_t v = act ? rn : 0;
          uint64_t incl = v;
          for (int o = 1; o < 64; o <<= 1) {
            uint64_t u = __shfl_up((unsigned long long)incl, o, 64);
            if ((int)lane_id() >= o) incl += u;
          }
          if (lane_id() == 63) S.wsum[tid / 64] = incl;
          __syncthreads();
          uint64_t wpre = 0;
          for (uint32_t q = 0; q < tid / 64; q++) wpre += S.wsum[q];
          S.x_pref[tid] = wpre + incl - v;
          if (tid == TILE - 1) S.x_pref[TILE] = wpre + incl;
          __syncthreads();
          x_total = S.x_pref[TILE];
          x_base = 0;
          x_lpc = pc;
          x_own_dis = ln.dis;
          x_own_gtid = ln.gtid;
          x_hang = hg;
          x_act = act;
          if (x_total == 0) {
            pc = endpc;  // ENDLOOP finishes the expansion
            in_x = true;
            continue;
          }
          in_x = true;
          x_chunk(pc);
          break;  // body follows
        }
        if (d == 0) { ln.run0 = rn; ln.st0 = (uint64_t)s; ln.sp0 = (uint64_t)stp; ln.k0 = 0; }
        else { ln.run1 = rn; ln.st1 = (uint64_t)s; ln.sp1 = (uint64_t)stp; ln.k1 = 0; }
        ln.hangp = (ln.hangp & ~(1u << d)) | (hg ? (1u << d) : 0u);
        ln.dis = act ? (rn > 0 ? 0u : 1u) : ln.dis + 1;
        if (__ballot(ln.dis == 0) == 0) {
          pc = endpc;  // ENDLOOP: exit handling
          continue;
        }
        RSET(dd, narrow((uint64_t)s, w));
        if (MODE == M_MAIN) count_site(S, C, ufirst(D.s0), __ballot(ln.dis == 0));
        break;
      }
      case CKC_OP_ENDLOOP: {
        if (MODE == M_FIX) return;  // target not reached in this iteration
        const uint32_t d = ufirst(D.x);
        const uint32_t lpc = ufirst(D.jmp);
        if (in_x && lpc == x_lpc) {
          x_base += TILE;
          if (x_base < x_total) {
            x_chunk(lpc);
            pc = lpc + 1;
            continue;
          }
          // expansion done: back to this lane's own thread
          in_x = false;
          for (uint32_t q = 0; q < x_nlive; q++) RSET(P->livein[q], S.x_live[q][threadIdx.x]);
          ln.gtid = x_own_gtid;
          ln.k0 = 0;
          ln.k1 = 0;
          ln.dis = x_own_dis;
          if (x_hang) { ln.dis = DEAD; ln.hangs++; }
          count_site(S, C, ufirst(S.ins[lpc].s1), __ballot(x_act && !x_hang));
          __syncthreads();
          break;
        }
        const dins Lp = S.ins[lpc];
        const uint32_t lw = ufirst(Lp.w), ldst = ufirst(Lp.dst);
        if (ln.dis == 0) {
          uint64_t kk = (d == 0 ? ln.k0 : ln.k1) + 1;
          if (d == 0) ln.k0 = kk; else ln.k1 = kk;
          if (kk == (d == 0 ? ln.run0 : ln.run1)) ln.dis = 1;  // done at this level
        }
        if (__ballot(ln.dis == 0)) {
          const uint64_t kk = d == 0 ? ln.k0 : ln.k1;
          const uint64_t s0 = d == 0 ? ln.st0 : ln.st1, sp = d == 0 ? ln.sp0 : ln.sp1;
          if (ln.dis == 0) RSET(ldst, narrow(s0 + kk * sp, lw));
          if (MODE == M_MAIN) count_site(S, C, ufirst(Lp.s0), __ballot(ln.dis == 0));
          pc = lpc + 1;
          continue;
        }
        // exit: lanes that ran this loop leave it; a capped loop stops its lane
        const bool mine = ln.dis == 1;
        const bool hg = mine && ((ln.hangp >> d) & 1u);
        if (MODE == M_MAIN) count_site(S, C, ufirst(Lp.s1), __ballot(mine && !hg));
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
        uint64_t r = alu(op, w, rget(lo, hi, da), rget(lo, hi, db), f);
        if (act) ln.faults += f;
        RSET(dd, r);
        break;
      }
    }
    pc++;
  }
}

__device__ void flush_input(GenLds& S, const KArgs& a, uint32_t input, const dprog* P) {
  __syncthreads();
  const dinput& in = a.inputs[input];
  uint32_t* cnt = a.counts + in.cnt_base;
  uint32_t ns = P->n_sites < (uint32_t)MAX_SITES_LDS ? P->n_sites : (uint32_t)MAX_SITES_LDS;
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

__global__ void __launch_bounds__(TILE) eval_generic_kernel(KArgs a) {
  __shared__ GenLds S;
  const uint32_t tid = threadIdx.x;
  const uint64_t total = a.js->total_tiles[1];
  if (total == 0) return;
  for (uint32_t s = tid; s < MAX_SITES_LDS; s += TILE) S.sites[s] = 0;
  if (tid == 0) { S.acc_checked = 0; S.hangs = 0; S.faults = 0; }
  uint32_t cur = 0xFFFFFFFFu;
  uint64_t cur_prog = 0;
  for (;;) {
    __syncthreads();
    if (tid == 0) S.tile = atomicAdd((unsigned long long*)&a.js->next_tile[1], 1ull);
    __syncthreads();
    const uint64_t t = S.tile;
    if (t >= total) break;
    const uint32_t i = find_input(a.inputs, a.n_inputs, 1, t);
    const dinput& in = a.inputs[i];
    const dprog* P = (const dprog*)in.prog;
    if (i != cur) {
      if (cur != 0xFFFFFFFFu) flush_input(S, a, cur, (const dprog*)a.inputs[cur].prog);
      if (in.prog != cur_prog) {
        const dins* src = prog_ins(P);
        for (uint32_t q = tid; q < P->n_instr; q += TILE) S.ins[q] = src[q];
        const int64_t* k = prog_consts(P);
        for (uint32_t q = tid; q < P->n_consts; q += TILE) S.consts[q] = k[q];
        cur_prog = in.prog;
      }
      const ckc_alloc* tab = (const ckc_alloc*)in.table;
      if (tid < P->n_slots) S.tab[tid] = tab[tid];
      cur = i;
      __syncthreads();
    }
    const uint64_t l = (t - in.tile_begin[1]) * TILE + tid;
    const bool act = l < in.lanes;
    Thr T;
    decode_lane(in.mode, in.launch, act ? l : 0, T);
    Ctx C;
    C.in = &in;
    C.sc = a.scalars + (size_t)i * MAX_SCALARS;
    C.rec = a.recs + in.rec_base;
    C.gcnt = a.counts + in.cnt_base;
    C.Lsum = in.L1 + in.L2;
    C.L2 = in.L2;
    C.cap0 = 1ull << in.cap_log2[0];
    C.cap1 = 1ull << in.cap_log2[1];
    C.t0 = T.t[0]; C.t1 = T.t[1]; C.t2 = T.t[2]; C.b0 = T.b[0]; C.b1 = T.b[1]; C.b2 = T.b[2];
    Lane ln;
    ln.dis = act ? 0u : DEAD;
    ln.k0 = ln.k1 = ln.run0 = ln.run1 = ln.st0 = ln.st1 = ln.sp0 = ln.sp1 = 0;
    ln.hangp = 0;
    ln.gtid = T.gtid;
    ln.faults = 0;
    ln.hangs = 0;
    uint32_t lo[NREG], hi[NREG];
#pragma unroll
    for (int r = 0; r < NREG; r++) { lo[r] = 0; hi[r] = 0; }
    run_program<M_MAIN>(S, C, ln, lo, hi, P->n_instr);
    uint64_t f = wave_sum64(ln.faults), h = wave_sum64(ln.hangs);
    if (lane_id() == 0) {
      if (f) atomicAdd(&S.faults, (unsigned long long)f);
      if (h) atomicAdd(&S.hangs, (unsigned long long)h);
    }
  }
  if (cur != 0xFFFFFFFFu) flush_input(S, a, cur, (const dprog*)a.inputs[cur].prog);
}

// One wavefront per record: replays the thread of first_key up to the access
// and stores the index and kind there.
__global__ void __launch_bounds__(64) fixup_kernel(KArgs a, uint64_t n_records) {
  __shared__ GenLds S;
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
  const dins* src = prog_ins(P);
  for (uint32_t q = threadIdx.x; q < P->n_instr; q += 64) S.ins[q] = src[q];
  const int64_t* k = prog_consts(P);
  for (uint32_t q = threadIdx.x; q < P->n_consts; q += 64) S.consts[q] = k[q];
  const ckc_alloc* tab = (const ckc_alloc*)in.table;
  if (threadIdx.x < P->n_slots) S.tab[threadIdx.x] = tab[threadIdx.x];
  __syncthreads();
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
  C.in = &in;
  C.sc = a.scalars + (size_t)lo_i * MAX_SCALARS;
  C.rec = a.recs + in.rec_base;
  C.gcnt = a.counts + in.cnt_base;
  C.Lsum = Lsum;
  C.L2 = in.L2;
  C.cap0 = 1ull << in.cap_log2[0];
  C.cap1 = 1ull << in.cap_log2[1];
  C.t0 = T.t[0]; C.t1 = T.t[1]; C.t2 = T.t[2]; C.b0 = T.b[0]; C.b1 = T.b[1]; C.b2 = T.b[2];
  C.tacc = acc;
  C.tk0 = i1;
  C.tk1 = i2;
  C.tloop0 = A.loop_pc[0];
  C.tloop1 = A.loop_pc[1];
  C.trec = rec;
  Lane ln;
  ln.dis = lane_id() == 0 ? 0u : DEAD;
  ln.k0 = ln.k1 = ln.run0 = ln.run1 = ln.st0 = ln.st1 = ln.sp0 = ln.sp1 = 0;
  ln.hangp = 0;
  ln.gtid = gtid;
  ln.faults = 0;
  ln.hangs = 0;
  uint32_t lo[NREG], hi[NREG];
#pragma unroll
  for (int q = 0; q < NREG; q++) { lo[q] = 0; hi[q] = 0; }
  run_program<M_FIX>(S, C, ln, lo, hi, P->n_instr);
}

// Per input: trace-path totals from per-thread counts, then the dense map.
__global__ void __launch_bounds__(256) finish_kernel(KArgs a) {
  const uint32_t i = blockIdx.x;
  if (i >= a.n_inputs) return;
  const dinput& in = a.inputs[i];
  const dprog* P = (const dprog*)in.prog;
  uint32_t* cnt = a.counts + in.cnt_base;
  const uint64_t lanes = in.lanes;
  if (in.path == 0) {
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
hipError_t launch_eval_trace(const KArgs& a, uint32_t n_wg, hipStream_t s) {
  hipLaunchKernelGGL(eval_trace_kernel, dim3(n_wg), dim3(TILE), 0, s, a);
  return hipGetLastError();
}
hipError_t launch_eval_generic(const KArgs& a, uint32_t n_wg, hipStream_t s) {
  hipLaunchKernelGGL(eval_generic_kernel, dim3(n_wg), dim3(TILE), 0, s, a);
  return hipGetLastError();
}
hipError_t launch_fixup(const KArgs& a, uint64_t n_records, hipStream_t s) {
  if (n_records == 0) return hipSuccess;
  hipLaunchKernelGGL(fixup_kernel, dim3((uint32_t)n_records), dim3(64), 0, s, a, n_records);
  return hipGetLastError();
}
hipError_t launch_finish(const KArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(finish_kernel, dim3(a.n_inputs), dim3(256), 0, s, a);
  return hipGetLastError();
}

}  // namespace ckc
