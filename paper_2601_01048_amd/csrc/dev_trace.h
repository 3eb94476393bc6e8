// dev_trace.h — the trace evaluator (uniform-control programs with affine indices).
// Part of the device code of libckc; included by kernels.hip only (one
// translation unit, no relocatable device code).
#pragma once

namespace ckc {

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

typedef const __attribute__((address_space(4))) int64_t c_i64;
typedef const __attribute__((address_space(4))) dprog c_dprog;
typedef const __attribute__((address_space(4))) dblk c_blk;

// An opaque copy of p: loads through it cannot be hoisted out of the loop the
// copy is made in, so such per-input values are reloaded with scalar loads
// where they are used instead of being held in registers across the loop.
template <class T>
__device__ __forceinline__ T* fresh(T* p) {
  asm volatile("" : "+s"(p));
  return p;
}

__device__ __forceinline__ c_i64* trace_hot64(c_head* th) { return (c_i64*)(th + 1); }
__device__ __forceinline__ c_u32* trace_hot32(c_head* th) {
  return (c_u32*)(trace_hot64(th) + 2 * (size_t)th->cap8);
}
__device__ __forceinline__ c_entry* trace_entries(c_head* th) {
  return (c_entry*)(trace_hot32(th) + 2 * (size_t)th->cap8);
}

// Violation path of entry e in group g of a block-major job (rare): per
// block, the mask of violating lanes and of negative indices; the first block
// with a violation gives the first key at its lowest violating lane.  w[j] is
// this lane's index base (thread part + block part) in block j of the group.
template <int W, class BT>
__device__ __forceinline__ void blocks_violation(TraceLds& S, c_head* th, uint32_t e, const BT* w, uint32_t g,
                                              uint32_t nvalid, uint32_t t0) {
  c_blk* B = &th->blk;
  c_entry* te = trace_entries(th);
  const int64_t off = te[e].off;
  const uint64_t bound = te[e].bound;
  const uint32_t dead = te[e].dead_kind;
  uint64_t fk = ~0ull, cnt = 0;
  uint32_t kinds = 0;
  for (uint32_t j = 0; j < nvalid; j++) {
    uint64_t badm, underm;
    if (W == 32) {
      const uint32_t v = (uint32_t)w[j] + (uint32_t)off;
      badm = __ballot(v >= (uint32_t)bound);
      underm = __ballot((int32_t)v < 0);
    } else {
      const uint64_t v = (uint64_t)w[j] + (uint64_t)off;
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
        // block of member g*LPB + j of the thread set
        const uint64_t k = (uint64_t)g * LPB + j;
        uint32_t L[6];
        for (int q = 0; q < 6; q++) L[q] = B->L[q];
        const uint64_t blin = B->mode == CKC_FULL ? k : bset_block(L, k);
        fk = ((blin * B->bs + t0 + (uint64_t)(__ffsll((unsigned long long)badm) - 1)) << B->Lsum) |
             te[e].keylo;
      }
      cnt += (uint64_t)__popcll(badm);
    }
  }
  if (cnt) tr_note(S, (ckc_record*)B->rec, te[e].acc, B->n_acc <= TR_ACC_LDS, fk, cnt, kinds);
}

// Block-major checks of one group: w[j] is this lane's index base in block j
// of the group (thread part + block part, wrapped at the index width); a
// group with fewer than LPB blocks repeats its first block's base in the
// unused slots.  Entries come as packed (offset, bound) pairs through scalar
// loads.  Width 32: an index is in bounds iff its unsigned value is below the
// bound (clamped to 2^31), so one entry is clean for all blocks iff the
// unsigned maximum over the blocks is below the bound -- one add per block, a
// max tree and one compare.
template <int W, class BT>
__device__ __forceinline__ bool entry_bad(uint64_t off, uint64_t bnd, const BT* w) {
  if (W == 32) {
    uint32_t mx = 0;
#pragma unroll
    for (uint32_t j = 0; j < LPB; j++) {
      const uint32_t v = (uint32_t)w[j] + (uint32_t)off;
      mx = v > mx ? v : mx;
    }
    return mx >= (uint32_t)bnd;
  } else {
    bool x = false;
#pragma unroll
    for (uint32_t j = 0; j < LPB; j++) x |= ((uint64_t)w[j] + off) >= bnd;
    return x;
  }
}

// Width 32, LIN groups: the bases are an arithmetic progression
// w[j] = w[0] + j*s (mod 2^32) over all LPB blocks with (LPB-1)*|s| < 2^31.
// Then every index of the entry is in bounds iff both end indices are: if
// both are below the bound (at most 2^31), the progression between them
// spans less than 2^32 from a value below 2^31, so it does not wrap and
// every term lies between the ends.  Exact, with two adds, one max and one
// compare for the LPB indices.
template <class BT>
__device__ __forceinline__ bool entry_bad_lin(uint64_t off, uint64_t bnd, const BT* w) {
  const uint32_t a = (uint32_t)w[0] + (uint32_t)off, b = (uint32_t)w[LPB - 1] + (uint32_t)off;
  return (a > b ? a : b) >= (uint32_t)bnd;
}

// LIN: only w[0] and w[LPB-1] are formed by the caller; the rest are filled
// from the step before the violation path needs them.
// Width 32: true if some lane has an access offset out of bounds somewhere in
// the progression from v0 to v1 (bases of consecutive blocks of one row, the
// span below 2^31, as for entry_bad_lin); one test per batch of 8 offsets.
template <class BT>
__device__ __forceinline__ bool span_bad(c_head* th, BT v0, BT v1) {
  const uint32_t ne = th->blk.ne;
  c_u32* h32 = trace_hot32(th);
  for (uint32_t e = 0; e < ne; e += 8) {
    uint32_t off[8], bnd[8];
#pragma unroll
    for (uint32_t k = 0; k < 8; k++) {
      off[k] = h32[2 * (e + k)];
      bnd[k] = h32[2 * (e + k) + 1];
    }
    uint64_t badm = 0;
#pragma unroll
    for (uint32_t k = 0; k < 8; k++) {
      if (e + k < ne) {
        const uint32_t a = (uint32_t)v0 + off[k], b = (uint32_t)v1 + off[k];
        badm |= __ballot((a > b ? a : b) >= bnd[k]);
      }
    }
    if (badm) return true;
  }
  return false;
}

// Width 32: as span_bad over up to 4 progressions at once (the row segments
// of a job), nseg of them in use.
template <class BT>
__device__ __forceinline__ bool segs_bad(c_head* th, const BT* v0, const BT* v1, uint32_t nseg) {
  const uint32_t ne = th->blk.ne;
  c_u32* h32 = trace_hot32(th);
  for (uint32_t e = 0; e < ne; e += 8) {
    uint32_t off[8], bnd[8];
#pragma unroll
    for (uint32_t k = 0; k < 8; k++) {
      off[k] = h32[2 * (e + k)];
      bnd[k] = h32[2 * (e + k) + 1];
    }
    uint64_t badm = 0;
#pragma unroll
    for (uint32_t k = 0; k < 8; k++) {
      if (e + k < ne) {
        bool b = false;
#pragma unroll
        for (uint32_t q = 0; q < 4; q++) {
          if (q < nseg) {
            const uint32_t a = (uint32_t)v0[q] + off[k], c = (uint32_t)v1[q] + off[k];
            b |= (a > c ? a : c) >= bnd[k];
          }
        }
        badm |= __ballot(b);
      }
    }
    if (badm) return true;
  }
  return false;
}

template <int W, bool DEADS, bool LIN, class BT>
__device__ __forceinline__ void trace_blocks(TraceLds& S, c_head* th, BT* w, uint32_t g, uint32_t nvalid,
                                             uint32_t t0, BT step) {
  constexpr uint32_t EB = W == 32 ? 8 : 4;  // entries per scalar-load batch
  const uint32_t ne = th->blk.ne;
  c_i64* h64 = trace_hot64(th);
  c_u32* h32 = trace_hot32(th);
  uint32_t e = 0;  // first entry that needs the violation path
  if (!DEADS) {
    // fast scan: one test per batch of EB entries (the OR of their lane
    // masks); a batch with a violating lane goes to the violation path whole.
    // The trace arrays hold a multiple of 8 entries, so the last batch load
    // stays inside them; its entries past the end are not tested.
    bool hit = false;
    for (; e < ne; e += EB) {
      uint64_t off[EB], bnd[EB];
#pragma unroll
      for (uint32_t k = 0; k < EB; k++) {
        if (W == 32) {
          off[k] = h32[2 * (e + k)];
          bnd[k] = h32[2 * (e + k) + 1];
        } else {
          off[k] = (uint64_t)h64[2 * (e + k)];
          bnd[k] = (uint64_t)h64[2 * (e + k) + 1];
        }
      }
      uint64_t badm = 0;
      if (e + EB <= ne) {
#pragma unroll
        for (uint32_t k = 0; k < EB; k++)
          badm |= __ballot(LIN ? entry_bad_lin(off[k], bnd[k], w) : entry_bad<W>(off[k], bnd[k], w));
      } else {
        const uint32_t r = ne - e;
#pragma unroll
        for (uint32_t k = 0; k < EB - 1; k++)
          if (k < r) badm |= __ballot(LIN ? entry_bad_lin(off[k], bnd[k], w) : entry_bad<W>(off[k], bnd[k], w));
      }
      if (badm) {
        hit = true;
        break;
      }
    }
    if (!hit) return;
  }
  if (LIN) {
#pragma unroll
    for (uint32_t jj = 1; jj < LPB - 1; jj++) w[jj] = w[0] + (BT)jj * step;
  }
  // violation path: the remaining entries one by one
  for (; e < ne; e++) {
    uint64_t off, bnd;
    if (W == 32) {
      off = h32[2 * e];
      bnd = h32[2 * e + 1];
    } else {
      off = (uint64_t)h64[2 * e];
      bnd = (uint64_t)h64[2 * e + 1];
    }
    if (DEADS || __ballot(entry_bad<W>(off, bnd, w))) blocks_violation<W>(S, th, e, w, g, nvalid, t0);
  }
}

// Per-input state of the trace evaluator over lane tiles (wavefront-uniform).
struct TrIn {
  uint32_t L[6];  // launch dims
  uint32_t mode, aux, Lsum, ne, n_acc;  // thread-set mode, its PREX round
  bool lds;
  c_entry* te;
  ckc_record* rec;
};

// One block-major wavefront job: slice position o (64 threads) of the groups
// gs*ngj .. gs*ngj+ngj-1 (LPB set blocks each; ngj from the plan).  The thread part of the index
// base is formed once per job; in the whole-grid modes the block coordinates
// are walked from group to group, and a group that stays inside one grid row
// forms its block parts by adding the x coefficient.
//
// PROOF = false (CKC_FULL): every index of every thread is formed (one add
// per access) and compared against its bound (a max tree over the 16 blocks
// of a group, one compare per tree).
// PROOF = true (CKC_FULL_ENDPOINTS, width 32): the whole grid is decided by
// the end-point argument of the affine-access Theorem (Section 5.1.1) applied
// to row progressions of block bases: a progression whose span stays below
// 2^31 is in bounds exactly when its two end indices are, so most indices are
// never formed.  Results are identical; the work is not per access.
template <int W, bool FULL, bool PROOF>
__device__ __forceinline__ void block_job(TraceLds& S, c_head* th, uint32_t gs, uint32_t o) {
  typedef typename std::conditional<W == 32, uint32_t, uint64_t>::type BT;
  c_blk* B = &th->blk;
  const uint32_t tlin = o * 64u + (threadIdx.x & 63u);
  const uint32_t tz = udiv(tlin, UDiv{B->m_bxy, B->s_bxy}), tr = tlin - tz * B->bxy;
  const uint32_t ty = udiv(tr, UDiv{B->m_bx, B->s_bx});
  const uint32_t tx = tr - ty * B->L[3];
  const int64_t k0 = B->k[0], k1 = B->k[1], k2 = B->k[2];
  // thread part at the index width (wrapping there is the index semantics)
  BT tp = 0;
  if (k0 == 1) tp += (BT)tx; else if (k0 != 0) tp += (BT)k0 * (BT)tx;
  if (k1 == 1) tp += (BT)ty; else if (k1 != 0) tp += (BT)k1 * (BT)ty;
  if (k2 == 1) tp += (BT)tz; else if (k2 != 0) tp += (BT)k2 * (BT)tz;
  const uint32_t t0 = o * 64u;
  const uint32_t ngj = B->ngj;
  uint32_t g = gs * ngj;
  const uint32_t gend = g + ngj < B->ngroups ? g + ngj : B->ngroups;
  // whole grid: coordinates and block part of the group's first block
  uint32_t bx = 0, by = 0, bz = 0;
  BT cur = 0;
  if (FULL) {
    const uint32_t b0 = g * LPB;
    bz = udiv(b0, UDiv{B->m_gxy, B->s_gxy});
    const uint32_t brem = b0 - bz * B->gxy;
    by = udiv(brem, UDiv{B->m_gx, B->s_gx});
    bx = brem - by * B->L[0];
    cur = (BT)B->k[3] * (BT)bx + (BT)B->k[4] * (BT)by + (BT)B->k[5] * (BT)bz;
    if (PROOF && W == 32 && !B->any_dead) {
      // the job's blocks split at row ends into at most 4 row segments, each
      // a progression of block bases: when every segment's span stays below
      // 2^31 and no offset is out of bounds at the ends of any segment, the
      // whole job is clean
      const uint32_t gx = B->L[0], gy = B->L[1];
      const uint32_t bend = gend * LPB < B->nsb ? gend * LPB : B->nsb;
      const uint32_t sd = (uint32_t)B->d1, ad = (int32_t)sd < 0 ? 0u - sd : sd;
      const BT d1 = (BT)B->d1, dy = (BT)B->dy, dz = (BT)B->dz;
      uint32_t left = bend - g * LPB, sx = bx, sy = by, nseg = 0;
      BT sc = cur, v0[4], v1[4];
      bool ok = true;
#pragma unroll
      for (uint32_t q = 0; q < 4; q++) {
        if (left != 0 && ok) {
          const uint32_t len = gx - sx < left ? gx - sx : left;
          if ((uint64_t)ad * (len - 1) > 0x7FFFFFFFull) {
            ok = false;
          } else {
            v0[q] = tp + sc;
            v1[q] = v0[q] + (BT)(len - 1) * d1;
            nseg = q + 1;
            left -= len;
            sx += len;
            sc += (BT)len * d1;
            if (sx == gx) {
              sx = 0;
              if (++sy == gy) {
                sy = 0;
                sc += dz;
              } else {
                sc += dy;
              }
              sc -= d1;
            }
          }
        }
      }
      if (ok && left == 0 && !segs_bad(th, v0, v1, nseg)) return;
    }
  }
#pragma unroll 1
  for (; g < gend; g++) {
    c_head* tg = fresh(th);
    c_blk* Bg = &tg->blk;
    if (FULL && PROOF && W == 32 && !Bg->any_dead) {
      // the whole groups of the job from g on that lie in the current row
      // form one progression of block bases: when its span stays below 2^31
      // and no offset is out of bounds at either end, they are all clean
      const uint32_t gx = Bg->L[0], full_groups = Bg->nsb / LPB;
      uint32_t k = (gx - bx) / LPB;
      const uint32_t glim = gend < full_groups ? gend : full_groups;
      k = g < glim ? (k < glim - g ? k : glim - g) : 0u;
      const uint32_t sd = (uint32_t)Bg->d1, ad = (int32_t)sd < 0 ? 0u - sd : sd;
      if (k >= 2 && (uint64_t)ad * (LPB * k - 1) <= 0x7FFFFFFFull) {
        const BT d1 = (BT)Bg->d1;
        const BT v0 = tp + cur;
        if (!span_bad(tg, v0, v0 + (BT)(LPB * k - 1) * d1)) {
          bx += LPB * k;
          cur += (BT)(LPB * k) * d1;
          if (bx == gx) {
            bx = 0;
            if (++by == Bg->L[1]) {
              by = 0;
              ++bz;
              cur += (BT)Bg->dz;
            } else {
              cur += (BT)Bg->dy;
            }
            cur -= d1;
          }
          g += k - 1;
          continue;
        }
      }
    }
    BT w[LPB];
    const uint32_t left = Bg->nsb - g * LPB;
    const uint32_t nvalid = left < LPB ? left : LPB;
    bool lin = false;  // w is an arithmetic progression with a small step (width 32)
    if (FULL) {
      // the block part moves by d1 per block, by dy when x wraps and by dz
      // when y wraps as well
      const uint32_t gx = Bg->L[0];
      const BT d1 = (BT)Bg->d1;
      if (bx + LPB <= gx) {
        // the group stays in one row
        if (PROOF && W == 32 && nvalid == LPB && !Bg->any_dead) {
          const uint32_t sd = (uint32_t)d1, ad = (int32_t)sd < 0 ? 0u - sd : sd;
          lin = ad <= 0x7FFFFFFFu / (LPB - 1);
        }
        BT v = tp + cur;
        if (lin) {
          w[0] = v;
          w[LPB - 1] = v + (BT)(LPB - 1) * d1;
        } else {
#pragma unroll
          for (uint32_t jj = 0; jj < LPB; jj++) {
            w[jj] = v;
            v += d1;
          }
        }
        bx += LPB;
        cur += (BT)LPB * d1;
        if (bx == gx) {
          bx = 0;
          if (++by == Bg->L[1]) {
            by = 0;
            ++bz;
            cur += (BT)Bg->dz;
          } else {
            cur += (BT)Bg->dy;
          }
          cur -= d1;
        }
      } else {
        const uint32_t gy = Bg->L[1];
        const BT dy = (BT)Bg->dy, dz = (BT)Bg->dz;
#pragma unroll
        for (uint32_t jj = 0; jj < LPB; jj++) {
          w[jj] = tp + cur;
          if (++bx == gx) {
            bx = 0;
            if (++by == gy) {
              by = 0;
              ++bz;
              cur += dz;
            } else {
              cur += dy;
            }
          } else {
            cur += d1;
          }
        }
      }
    } else {
      uint32_t L[6];
      for (int q = 0; q < 6; q++) L[q] = Bg->L[q];
      const UDiv dgx{Bg->m_gx, Bg->s_gx}, dgxy{Bg->m_gxy, Bg->s_gxy};
      const uint32_t gxy = Bg->gxy;
      const int64_t k3 = Bg->k[3], k4 = Bg->k[4], k5 = Bg->k[5];
      // lane jj of the wavefront decodes member g*LPB + jj of the set (the
      // decodes of the group run side by side), then each block part is
      // broadcast from its lane
      const uint32_t jl = lane_id() & (LPB - 1);
      const uint32_t blin = jl < nvalid ? (uint32_t)bset_block(L, (uint64_t)g * LPB + jl) : 0u;
      const uint32_t cz = udiv(blin, dgxy), crem = blin - cz * gxy;
      const uint32_t cy = udiv(crem, dgx), cx = crem - cy * L[0];
      const uint64_t part = (uint64_t)k3 * cx + (uint64_t)k4 * cy + (uint64_t)k5 * cz;
#pragma unroll
      for (uint32_t jj = 0; jj < LPB; jj++) w[jj] = tp + (BT)readlane64(part, (int)jj);
    }
    if (nvalid < LPB) {
      // the last group of the set: unused slots repeat the first block
#pragma unroll
      for (uint32_t jj = 1; jj < LPB; jj++)
        if (jj >= nvalid) w[jj] = w[0];
    }
    if (Bg->any_dead) trace_blocks<W, true, false>(S, tg, w, g, nvalid, t0, (BT)0);
    else if (lin) trace_blocks<W, false, true>(S, tg, w, g, nvalid, t0, (BT)Bg->d1);
    else trace_blocks<W, false, false>(S, tg, w, g, nvalid, t0, (BT)0);
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

// Loads the per-input state of the trace evaluator over lane tiles.
__device__ __forceinline__ void tr_load(TrIn& I, c_input* ins, uint32_t i, ckc_record* recs, uint64_t& tb,
                                        uint32_t path, uint32_t& ncls, c_head*& th) {
  for (int q = 0; q < 6; q++) I.L[q] = ins[i].launch[q];
  I.mode = ins[i].mode;
  I.aux = ins[i].aux;
  I.Lsum = ins[i].L1 + ins[i].L2;
  I.n_acc = ((c_dprog*)ins[i].prog)->n_accesses;
  I.lds = I.n_acc <= TR_ACC_LDS;
  th = (c_head*)ins[i].trace;
  I.te = trace_entries(th);
  I.rec = recs + ins[i].rec_base;
  I.ne = th->n_entries;
  ncls = th->n_classes;
  tb = ins[i].tile_begin[path];
}

// Trace evaluator, block-major layout: persistent workgroups over the tile
// space of PATH_BLOCKS under the job's schedule; a tile is four wavefront jobs.
template <uint32_t SK>
__global__ void __launch_bounds__(TILE, 7) eval_trace_kernel(KArgs a) {
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
  const uint32_t wv = ufirst(tid >> 6);
  uint32_t pos = 0xFFFFFFFFu;
  uint64_t tb = 0, cur_end = 0;
  c_head* th = nullptr;
  for (;;) {
    const uint64_t t = sched_next(sc, &a.js->next_tile[PATH_BLOCKS], &item_slot);
    if (t == ~0ull) break;
    if (pos == 0xFFFFFFFFu || t < tb || t >= cur_end) {
      const uint32_t np = pos_of_tile(ins, order, a.n_inputs, PATH_BLOCKS, pos, cur_end, t);
      if (pos != 0xFFFFFFFFu && th->blk.n_acc <= TR_ACC_LDS)
        tr_flush(S, (ckc_record*)th->blk.rec, th->blk.n_acc);
      pos = np;
      const uint32_t i = order[pos];
      th = (c_head*)ins[i].trace;
      tb = ins[i].tile_begin[PATH_BLOCKS];
      cur_end = tb + ins[i].n_tiles[PATH_BLOCKS];
    }
    c_head* tj = fresh(th);
    c_blk* B = &tj->blk;
    const uint64_t job = (t - tb) * 4 + wv;
    const uint64_t gs = job < (1ull << 32) ? (uint64_t)udiv((uint32_t)job, UDiv{B->m_spb, B->s_spb}) : job / B->spb;
    const uint32_t o = (uint32_t)(job - gs * B->spb);
    if (gs * B->ngj >= B->ngroups) continue;  // past the last group (whole wavefront)
    const bool full = B->mode == CKC_FULL;
    if (B->w == 32) {
      if (full) {
        if (B->proof) block_job<32, true, true>(S, tj, (uint32_t)gs, o);
        else block_job<32, true, false>(S, tj, (uint32_t)gs, o);
      } else {
        block_job<32, false, false>(S, tj, (uint32_t)gs, o);
      }
    } else {
      if (full) block_job<64, true, false>(S, tj, (uint32_t)gs, o);
      else block_job<64, false, false>(S, tj, (uint32_t)gs, o);
    }
  }
  if (pos != 0xFFFFFFFFu && th->blk.n_acc <= TR_ACC_LDS) tr_flush(S, (ckc_record*)th->blk.rec, th->blk.n_acc);
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
  uint32_t pos = 0xFFFFFFFFu, ncls = 0;
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
      tr_load(I, ins, i, a.recs, tb, PATH_LANES, ncls, th);
      cur_end = tb + ins[i].n_tiles[PATH_LANES];
      lanes = ins[i].lanes;
    }
    const uint64_t l = (t - tb) * TILE + tid;
    const bool act = l < lanes;
    Thr T;
    decode_lane(I.mode, I.L, I.aux, act ? l : 0, T);
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


}  // namespace ckc
