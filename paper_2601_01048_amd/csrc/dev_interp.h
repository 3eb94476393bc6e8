// dev_interp.h — the interpreter (whole threads, the body pass of expanded loops, first-violation replay).
// Part of the device code of libckc; included by kernels.hip only (one
// translation unit, no relocatable device code).
#pragma once

namespace ckc {

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
// The rows form of an input, read through scalar loads.
typedef const __attribute__((address_space(4))) drows c_drows;
typedef const __attribute__((address_space(4))) REnt c_rent;
typedef const __attribute__((address_space(4))) RForm c_rform;
// Loaded data through the global address space (global rather than flat loads).
typedef const __attribute__((address_space(1))) int32_t g_i32;
typedef const __attribute__((address_space(1))) int64_t g_i64;
typedef __attribute__((address_space(1))) uint64_t g_u64w;  // written global memory

// Iterations of an expanded loop per work item of the body pass (also the
// length of the owner map staged in LDS).
constexpr uint32_t PIECE_LDS = 2048;

// One access of a gather body: index = narrow(off + coef * X[var], w) with
// X[0] the loop counter and X[k] (k >= 1) the value of the k-th LOAD of the
// body (var 0xFF: a uniform index `off`).
constexpr uint32_t MAX_GENT = 32;
// tiles after the first that one run of the gather pass may take
constexpr uint32_t RUN_TILES = 64;
struct GEnt {
  int64_t coef, off;
  uint64_t bound;       // elements of the slot's allocation (size >> lg)
  const void* data;     // the slot's data (LOAD)
  uint32_t acc;
  uint16_t site;
  uint8_t slot, lg;
  uint8_t w, var, dst;  // dst: variable a LOAD defines (0 for ACCESS)
  uint8_t dead;         // NULL or FREED kind of the slot, else 0
  uint8_t pad[4];
};
static_assert(sizeof(GEnt) == 48, "gather entry layout");
struct GBody {
  GEnt e[MAX_GENT];
  uint32_t n, ok, faults;  // entries, usable, division faults per iteration
  uint8_t var[NREG];       // symbolic walk: variable of each register (0xFF uniform)
};

// LDS of the whole-thread pass (and what every pass counts into): coverage
// counters of the current input, its status totals, the expanded loop's
// per-wavefront sums and contiguity (the least and greatest start minus prefix
// of the wavefront's threads with iterations, flags 1: some thread has
// iterations, 2: some step is not 1), the tile's shared-memory layout (words
// per block instance, blocks per tile, offset of each shared slot).
struct WtLds {
  uint32_t sites[MAX_SITES_LDS];
  unsigned long long wsum[TILE / 64];
  unsigned long long acc_checked, hangs, faults;
  unsigned long long wemin[TILE / 64], wemax[TILE / 64];
  uint32_t wflag[TILE / 64];
  uint32_t sh_w, sh_nbt, sh_off[MAX_SLOTS];
};
// The interpreter's passes add the state of the expanded loops' body passes.
struct GenLds : WtLds {
  unsigned long long pref[TILE + 1];  // trip-count prefix of the tile's threads (expanded loop)
  GBody gb;                           // gather entries of the current input (body pass)
  unsigned long long xstart[TILE], xstep[TILE];  // loop start and step of the tile's threads (gather pass)
  uint16_t own[PIECE_LDS];            // owner thread of each iteration of the current piece
  uint16_t omax[TILE / 64];           // owner-map scan: per-wavefront maxima
  // gather pass: the violations of the current input's gather entries,
  // merged here and flushed per input
  unsigned long long vfk[MAX_GENT], vcnt[MAX_GENT];
  uint32_t vkinds[MAX_GENT];
  // gather pass over a run of chained contiguous tiles (iterations numbered
  // from the run's first tile on): per gather entry the least violating
  // iteration, the start of each tile after the first, the number of those
  // tiles, the run's end and its piece end
  unsigned long long rmin[MAX_GENT];
  unsigned long long rstart[RUN_TILES + 1];
  unsigned long long rend, rpend;
  uint32_t rn;
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
  // totals of this lane since the last flush (several threads or iterations)
  uint64_t faults, acc;    // divisions by zero; ACCESS and LOAD executions
  uint32_t hangs;          // threads stopped by a trip cap
};

struct Ctx {
  c_input* in;             // read through scalar loads
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
  unsigned long long *xtot, *xpb, *xpg, *xd;
  uint32_t* xin;
  uint32_t input;
  uint32_t tw;              // the input runs under the tripwire detector model
  uint32_t spaces;          // memory space of each slot (2 bits per slot)
  uint32_t capture;         // capture pass: only the first violation's index and kind
  // shared memory of the tile's blocks (blockwise programs in the whole-thread
  // pass; null elsewhere): the instances as at the phase start and the
  // phase's writes, the lane's instance offset and each slot's offset in it
  int32_t* shcur;
  unsigned long long* shnext;
  uint32_t sh_q;
  // fix-up target
  uint32_t tacc;
  uint64_t tk0, tk1;
  int32_t tloop0, tloop1;
  ckc_record* trec;
};

// Coverage of site s by the lanes of `mask`: one LDS add per wavefront.  `sat`
// (wavefront-uniform) marks sites below 64 whose workgroup count has reached
// the saturation value 255, after which counting them changes nothing.
__device__ __forceinline__ void count_site(WtLds& S, const Ctx& C, uint64_t& sat, uint32_t s, uint64_t mask) {
  if (s == NOSITE || mask == 0 || C.capture) return;
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

constexpr uint32_t PIECE = PIECE_LDS;

// The whole-thread pass at an expanded loop: every thread of the workgroup
// calls this exactly once per tile, with its capped trip count (0 for lanes
// that do not reach the loop), start and step.  Stores the prefix of the trip
// counts over the tile and the thread's loop state, and per tile the total,
// the pieces, the input and whether the tile is contiguous (every thread with
// iterations has step 1 and the same start minus prefix d: iteration g of the
// tile then has counter d + g).  `liv(q)` gives the thread's live-in q.
template <class LIV>
__device__ __forceinline__ void expand_record(WtLds& S, const Ctx& C, uint64_t cnt, uint64_t s0, uint64_t stp,
                                              LIV liv) {
  c_dprog* P = C.P;
  const uint32_t tid = threadIdx.x, wv = tid / 64;
  uint64_t incl = cnt;
  for (int o = 1; o < 64; o <<= 1) {
    const uint64_t u = __shfl_up((unsigned long long)incl, o, 64);
    if ((int)lane_id() >= o) incl += u;
  }
  // per wavefront, start minus the prefix within the wavefront
  const uint64_t e = s0 - (incl - cnt);
  const uint64_t emin = wave_min64(cnt ? e : ~0ull), emax = ~wave_min64(cnt ? ~e : ~0ull);
  const uint64_t has = __ballot(cnt != 0), nonunit = __ballot(cnt != 0 && stp != 1);
  if (lane_id() == 63) {
    S.wsum[wv] = incl;
    S.wemin[wv] = emin;
    S.wemax[wv] = emax;
    S.wflag[wv] = (has ? 1u : 0u) | (nonunit ? 2u : 0u);
  }
  __syncthreads();
  uint64_t wpre = 0;
  for (uint32_t q = 0; q < wv; q++) wpre += S.wsum[q];
  const uint64_t pre = wpre + incl - cnt;
  bool contig = true, any = false;
  uint64_t dref = 0, sum = 0;
  for (uint32_t q = 0; q < TILE / 64; q++) {
    const uint32_t f = S.wflag[q];
    if (f & 1u) {
      const uint64_t dq = S.wemin[q] - sum;
      if ((f & 2u) || S.wemin[q] != S.wemax[q] || (any && dq != dref)) contig = false;
      dref = dq;
      any = true;
    }
    sum += S.wsum[q];
  }
  contig = contig && any;
  const uint64_t l = C.lane0 + tid;
  C.xs[l] = pre;
  if (cnt) {
    // gather bodies of contiguous tiles keep no start and step (the gather
    // pass forms them from d)
    if (!(contig && P->body_gather && !C.tw)) {
      C.xs[C.xn + l] = s0;
      C.xs[2 * C.xn + l] = stp;
    }
    const uint32_t nl = P->n_livein;
    for (uint32_t q = 0; q < nl; q++) C.xs[(3 + q) * C.xn + l] = liv(q);
  }
  if (tid == TILE - 1) {
    const uint64_t tot = pre + cnt;
    C.xtot[C.xt] = tot;
    // the tripwire model is checked by the interpreted body form
    (P->body_gather && !C.tw ? C.xpg : C.xpb)[C.xt] = (tot + PIECE - 1) / PIECE;
    C.xin[C.xt] = C.input;
    C.xd[2 * C.xt] = dref;
    C.xd[2 * C.xt + 1] = contig ? 1ull : 0ull;
  }
  __syncthreads();
}

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
    const bool rd_b = (op >= CKC_OP_ADD && op <= CKC_OP_SELECT) || op == CKC_OP_LOOP || op == CKC_OP_FADD ||
                      op == CKC_OP_FSUB || op == CKC_OP_FMUL || op == CKC_OP_STORE;
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
      case CKC_OP_FADD: case CKC_OP_FSUB: case CKC_OP_FMUL: case CKC_OP_FEXP: case CKC_OP_ITOF:
      case CKC_OP_FTOI:
        r = float_op(op, w, va, vb);
        wreg = dd;
        break;
      case CKC_OP_BARRIER:
        // end of a phase: every wavefront of the workgroup is here (top
        // level); the phase's writes become the blocks' shared memory
        if (MODE == M_MAIN && C.shcur) {
          __syncthreads();
          const uint32_t tot = S.sh_nbt * S.sh_w;
          for (uint32_t e = threadIdx.x; e < tot; e += TILE) {
            const unsigned long long nx = C.shnext[e];
            if (nx) {
              C.shcur[e] = (int32_t)((uint32_t)nx ^ 0x80000000u);
              C.shnext[e] = 0;
            }
          }
          __syncthreads();
        }
        break;
      case CKC_OP_ACCESS:
      case CKC_OP_STORE:
      case CKC_OP_LOAD: {
        const uint32_t slot = D.slot, lg = D.fl & 3u, acc = D.x;
        const int64_t idx = (int64_t)narrow(va, w);
        c_alloc& A = C.tab[slot];
        // kx: exact kind (decides what a LOAD reads and a STORE writes); kd:
        // the kind reported under the input's detector model
        const uint32_t kx = act ? kind_of(A.base, A.size_bytes, A.flags, idx, lg) : 0u;
        uint32_t kd = kx;
        if (C.tw && kx != 0 && kx != CKC_KIND_NULL && !tripwire_catches(C.tab, C.spaces, slot, idx, lg)) kd = 0;
        const bool shared = ((C.spaces >> (2 * slot)) & 3u) == CKC_SPACE_SHARED;
        if (MODE != M_FIX) {
          const uint64_t key = (ln.gtid << C.Lsum) | (ln.k0 << C.L2) | ln.k1;
          if (C.capture) {
            // keys are unique per access: one lane writes
            if (kd != 0 && key == C.rec[acc].first_key) {
              C.rec[acc].index = idx;
              C.rec[acc].first_kind = kd;
            }
          } else {
            ln.acc += act ? 1u : 0u;
            count_site(S, C, sat, D.s0, __ballot(act));
            if (__ballot(kd != 0)) merge_violation(C.rec + acc, kd, key);
          }
        } else if (acc == C.tacc) {
          if (lane_id() == 0) { C.trec->index = idx; C.trec->first_kind = kd; }
          return;
        }
        if (op == CKC_OP_LOAD) {
          uint64_t v = 0;
          if (act && kx == 0) {
            if (shared)  // the block's instance as at the phase start (0 outside the whole-thread pass)
              v = C.shcur ? (uint64_t)(int64_t)C.shcur[C.sh_q + S.sh_off[slot] + (uint64_t)idx] : 0ull;
            else
              v = lg == 2 ? (uint64_t)(int64_t)((g_i32*)A.data)[idx] : (uint64_t)((g_i64*)A.data)[idx];
          }
          r = v;
          wreg = dd;
        } else if (op == CKC_OP_STORE && act && kx == 0 && shared && lg == 2 && C.shnext) {
          // racing writes of a phase keep the largest value: compare as
          // unsigned with the sign bit flipped, bit 32 marks "written"
          const unsigned long long packed = (1ull << 32) | (uint32_t)((uint32_t)vb ^ 0x80000000u);
          atomicMax(&C.shnext[C.sh_q + S.sh_off[slot] + (uint64_t)idx], packed);
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
          expand_record(S, C, act ? rn : 0, (uint64_t)s0, (uint64_t)stp,
                        [&](uint32_t q) { return RGET(ufirst(C.P->livein[q])); });
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

__device__ __forceinline__ void flush_input(WtLds& S, const KArgs& a, uint32_t input, uint32_t n_sites) {
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

__device__ __forceinline__ void ctx_init(Ctx& C, const KArgs& a, c_input& in, uint32_t i, const Thr& T) {
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
  C.xpg = a.xpg;
  C.xin = a.xin;
  C.xd = a.xd;
  C.input = i;
  C.lane0 = 0;
  C.xt = 0;
  C.tw = in.detector;
  C.spaces = C.P->slot_spaces;
  C.capture = a.capture;
  C.shcur = nullptr;
  C.shnext = nullptr;
  C.sh_q = 0;
}

// Per-thread state of a lane (its totals are kept).
__device__ __forceinline__ void lane_init(Lane& ln, bool act, uint64_t gtid) {
  ln.dis = act ? 0u : DEAD;
  ln.k0 = ln.k1 = ln.run0 = ln.run1 = ln.st0 = ln.st1 = ln.sp0 = ln.sp1 = 0;
  ln.hangp = 0;
  ln.gtid = gtid;
}
__device__ __forceinline__ void lane_zero_totals(Lane& ln) {
  ln.faults = 0;
  ln.acc = 0;
  ln.hangs = 0;
}
// Adds the wavefront's totals to the workgroup's and clears them (called by
// the whole workgroup before a flush).
__device__ __forceinline__ void add_lane_totals(WtLds& S, Lane& ln) {
  const uint64_t f = wave_sum64(ln.faults), h = wave_sum64(ln.hangs), n = wave_sum64(ln.acc);
  if (lane_id() == 0) {
    if (f) atomicAdd(&S.faults, (unsigned long long)f);
    if (h) atomicAdd(&S.hangs, (unsigned long long)h);
    if (n) atomicAdd(&S.acc_checked, (unsigned long long)n);
  }
  lane_zero_totals(ln);
}

// The interpreter over whole threads: one lane per thread of the thread set.
template <uint32_t SK>
__global__ void __launch_bounds__(TILE, 4) eval_generic_kernel(KArgs a) {
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
  uint32_t pos = 0xFFFFFFFFu, cur = 0xFFFFFFFFu, cur_sites = 0, cur_mode = 0;
  uint64_t tb = 0, cur_end = 0, sat = 0, cur_lanes = 0;
  uint32_t cur_L[7] = {0, 0, 0, 0, 0, 0, 0};  // launch dims, then the PREX round
  Dec dec;
  Lane ln;
  lane_zero_totals(ln);
  for (;;) {
    __syncthreads();
    const uint64_t t = sched_next(sc, &a.js->next_tile[PATH_GENERIC], &item_slot);
    if (t == ~0ull) break;
    if (pos == 0xFFFFFFFFu || t < tb || t >= cur_end) {
      pos = pos_of_tile(ins, order, a.n_inputs, PATH_GENERIC, pos, cur_end, t);
      const uint32_t i = order[pos];
      if (cur != 0xFFFFFFFFu && !a.capture) {  // the capture pass counts nothing
        add_lane_totals(S, ln);
        flush_input(S, a, cur, cur_sites);
      }
      sat = 0;
      cur = i;
      cur_sites = ((c_dprog*)a.inputs[i].prog)->n_sites;
      tb = ins[i].tile_begin[PATH_GENERIC];
      cur_end = tb + ins[i].n_tiles[PATH_GENERIC];
      for (int q = 0; q < 6; q++) cur_L[q] = ins[i].launch[q];
      cur_L[6] = ins[i].aux;
      cur_mode = ins[i].mode;
      cur_lanes = ins[i].lanes;
      dec_make(dec, cur_L);
    }
    const uint32_t i = cur;
    c_input& in = ins[i];
    const uint64_t l = (t - tb) * TILE + tid;
    const bool act = l < cur_lanes;
    c_dprog* Pi = (c_dprog*)in.prog;
    const uint32_t pfl = Pi->pflags;
    if (a.capture) {
      // the capture pass runs only the tiles that hold the thread of some
      // first violation (lanes are in thread order in every thread set, and
      // a tile holds whole blocks); every lane decides alike
      if (!(pfl & PF_CAPTURE)) continue;
      const uint64_t l0 = (t - tb) * TILE;
      const uint64_t l1 = (l0 + TILE < cur_lanes ? l0 + TILE : cur_lanes) - 1;
      Thr T0, T1;
      if (cur_mode == CKC_FULL) { decode_full(dec, l0, T0); decode_full(dec, l1, T1); }
      else { decode_lane(cur_mode, cur_L, cur_L[6], l0, T0); decode_lane(cur_mode, cur_L, cur_L[6], l1, T1); }
      const ckc_record* rec = a.recs + in.rec_base;
      const uint32_t ls = in.L1 + in.L2;
      bool hit = false;
      for (uint32_t q = 0; q < Pi->n_accesses && !hit; q++) {
        if (rec[q].count == 0) continue;
        const uint64_t g = rec[q].first_key >> ls;
        hit = g >= T0.gtid && g <= T1.gtid;
      }
      if (!hit) continue;
    }
    Thr T;
    if (cur_mode == CKC_FULL) decode_full(dec, act ? l : 0, T);
    else decode_lane(cur_mode, cur_L, cur_L[6], act ? l : 0, T);
    Ctx C;
    ctx_init(C, a, in, i, T);
    C.lane0 = (t - tb) * TILE;
    C.xt = in.xt_begin + (t - tb);
    if (pfl & PF_BLOCKWISE) {
      // the tile holds whole blocks (block size divides TILE, checked at
      // submission): block tid / bs of the tile gets its own shared instance,
      // all zero at the start
      const uint32_t bs = cur_L[3] * cur_L[4] * cur_L[5];
      if (tid == 0) {
        uint32_t wsum = 0;
        c_alloc* tab = (c_alloc*)in.table;
        for (uint32_t s = 0; s < (uint32_t)MAX_SLOTS; s++) {
          S.sh_off[s] = wsum;
          if (s < Pi->n_slots && ((Pi->slot_spaces >> (2 * s)) & 3u) == CKC_SPACE_SHARED && tab[s].base != 0)
            wsum += (uint32_t)(tab[s].size_bytes / 4);
        }
        S.sh_w = wsum;
        S.sh_nbt = TILE / bs;
      }
      __syncthreads();
      const uint32_t rows = a.max_regs > 8u ? a.max_regs : 8u;
      unsigned long long* nx = (unsigned long long*)(R + (size_t)rows * TILE);
      int32_t* cu = (int32_t*)(nx + (size_t)S.sh_nbt * S.sh_w);
      for (uint32_t e = tid; e < S.sh_nbt * S.sh_w; e += TILE) {
        nx[e] = 0;
        cu[e] = 0;
      }
      __syncthreads();
      C.shcur = cu;
      C.shnext = nx;
      C.sh_q = (tid / bs) * S.sh_w;
    }
    lane_init(ln, act, T.gtid);
    run_program<M_MAIN>(S, R, C, ln, sat, 0, C.P->n_instr);
  }
  if (cur != 0xFFFFFFFFu && !a.capture) {
    add_lane_totals(S, ln);
    flush_input(S, a, cur, cur_sites);
  }
}

// ---------------------------------------------------------------------------
// The rows-form kernel: the whole-thread pass of jobs whose programs all take
// the rows form (PF_ROWS; the plan kernel has reduced each input's part
// outside the expanded loop's body to a list of entries, read here through
// scalar loads).  One lane per thread, tiles of 256 threads as in the
// interpreter, with no register file and no instruction dispatch.
struct RowsLds {
  uint32_t sites[MAX_SITES_LDS];       // coverage of the current input
  unsigned long long wsum[TILE / 64];  // expanded loop: per wavefront, its trip-count total,
  unsigned long long wd[TILE / 64];    // the start minus prefix d of its threads with iterations,
  uint32_t wflag[TILE / 64];           // 1: some thread has iterations, 2: they are not contiguous
  unsigned long long acc_checked, hangs;
  unsigned long long item_slot;
};

// Per-thread values: the coordinate-class sums and the loaded values X[1..4].
struct RSlice {
  uint64_t base[MAX_RCLS];
  uint64_t x[RV_MAXLOAD];
};
__device__ __forceinline__ uint64_t rsel4(const uint64_t* v, uint32_t k) {
  return k == 0 ? v[0] : k == 1 ? v[1] : k == 2 ? v[2] : v[3];
}
__device__ __forceinline__ void rset4(uint64_t* v, uint32_t k, uint64_t x) {
  if (k == 0) v[0] = x;
  else if (k == 1) v[1] = x;
  else if (k == 2) v[2] = x;
  else v[3] = x;
}
__device__ __forceinline__ uint64_t coord(const Thr& T, int d) {
  return d < 3 ? (uint64_t)T.t[d] : (uint64_t)T.b[d - 3];
}

// A form of the rows form for one thread at width w (fields uniform: scalar
// loads); a coordinate form outside the classes (more distinct coefficient
// vectors than classes) is summed from the thread's coordinates.
__device__ __forceinline__ uint64_t rform(c_rform& f, const RSlice& X, const Thr& T, uint32_t w) {
  const uint32_t var = f.var;
  uint64_t v = (uint64_t)f.off;
  if (var == RV_COORD) {
    const uint32_t cls = f.cls;
    if (cls != RCLS_NONE) {
      v += rsel4(X.base, cls);
    } else {
      for (int d = 0; d < 6; d++) v += (uint64_t)f.c[d] * coord(T, d);
    }
  } else if (var != RV_UNI) {
    v += (uint64_t)f.c[0] * rsel4(X.x, var - 1);
  }
  return narrow(v, w);
}

// The comparisons a rows-form guard takes (CMPEQ..CMPLEU at width w).
__device__ __forceinline__ bool rcmp(uint32_t op, uint32_t w, uint64_t x, uint64_t y) {
  x = narrow(x, w);
  y = narrow(y, w);
  const uint64_t m = w == 32 ? 0xFFFFFFFFull : ~0ull;
  const uint64_t ux = x & m, uy = y & m;
  const int64_t sx = (int64_t)x, sy = (int64_t)y;
  switch (op) {
    case CKC_OP_CMPEQ: return ux == uy;
    case CKC_OP_CMPNE: return ux != uy;
    case CKC_OP_CMPLTS: return sx < sy;
    case CKC_OP_CMPLES: return sx <= sy;
    case CKC_OP_CMPLTU: return ux < uy;
    default: return ux <= uy;  // CMPLEU
  }
}
// Trip counts of steps other than 1 (64-bit division, out of line).
__device__ __noinline__ uint64_t trip_count_div(int64_t s, int64_t e, int64_t st) { return trip_count(s, e, st); }
__device__ __forceinline__ uint64_t rtrips(int64_t s, int64_t e, int64_t st) {
  if (st == 1) return s < e ? (uint64_t)e - (uint64_t)s : 0;
  return trip_count_div(s, e, st);
}

// Visits of the entries' sites are counted per wavefront in one register
// (lane 2q: site s0 of entry q, lane 2q + 1: its s1) and moved to the
// workgroup's counters when the input changes.
__device__ __forceinline__ void rsite(uint32_t& sv, uint32_t slot, uint64_t mask) {
  const uint32_t c = (uint32_t)__popcll(mask);
  if (lane_id() == slot) sv += c;
}
__device__ __forceinline__ void rsite_flush(RowsLds& S, uint32_t& sv, c_drows& G, uint32_t* gcnt) {
  const uint32_t j = lane_id();
  if (sv != 0 && j < 2 * MAX_RENT) {
    const uint32_t s = (j & 1u) ? G.e[j >> 1].s1 : G.e[j >> 1].s0;
    if (s != NOSITE) {
      if (s < MAX_SITES_LDS) atomicAdd(&S.sites[s], sv);
      else if (gcnt[s] < 255u) atomicAdd(&gcnt[s], sv < 255u ? sv : 255u);
    }
  }
  sv = 0;
}

// Inclusive prefix sum over the wavefront (32-bit values).
__device__ __forceinline__ uint32_t wave_incl32(uint32_t v) {
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const uint32_t u = __shfl_up(v, o, 64);
    if ((int)lane_id() >= o) v += u;
  }
  return v;
}

// The expanded loop of one tile (every thread of the workgroup, once): the
// tile's prefix of the capped trip counts, the threads' loop state, and per
// tile the total, the pieces, the input and whether the tile is contiguous
// (every thread with iterations has step 1 and the same start minus prefix d:
// iteration g of the tile then has counter d + g).  Caps below 2^24 keep the
// tile's sums in 32 bits.
__device__ __forceinline__ void rows_expand(RowsLds& S, const Ctx& C, c_drows& G, uint64_t cnt, uint64_t s0,
                                            uint64_t stp) {
  c_dprog* P = C.P;
  const uint32_t tid = threadIdx.x, wv = tid / 64;
  uint64_t incl;
  if (C.cap0 < (1ull << 24)) incl = wave_incl32((uint32_t)cnt);
  else {
    incl = cnt;
    for (int o = 1; o < 64; o <<= 1) {
      const uint64_t u = __shfl_up((unsigned long long)incl, o, 64);
      if ((int)lane_id() >= o) incl += u;
    }
  }
  const uint64_t has = __ballot(cnt != 0);
  // d of the wavefront: its first thread with iterations; every other one
  // must agree
  const uint64_t e = s0 - (incl - cnt);
  uint64_t dw = 0;
  bool split = stp != 1;
  if (has) {
    dw = readlane64(e, (int)(__ffsll((unsigned long long)has) - 1));
    split = split || __ballot(cnt != 0 && e != dw) != 0;
  }
  if (lane_id() == 63) {
    S.wsum[wv] = incl;
    S.wd[wv] = dw;
    S.wflag[wv] = (has ? 1u : 0u) | (split ? 2u : 0u);
  }
  __syncthreads();
  uint64_t wpre = 0, tot = 0, dref = 0;
  bool contig = true, any = false;
  for (uint32_t q = 0; q < TILE / 64; q++) {
    const uint32_t f = S.wflag[q];
    if (q == wv) wpre = tot;
    if (f & 1u) {
      const uint64_t dq = S.wd[q] - tot;
      if ((f & 2u) || (any && dq != dref)) contig = false;
      dref = dq;
      any = true;
    }
    tot += S.wsum[q];
  }
  contig = contig && any;
  const uint64_t pre = wpre + incl - cnt;
  // the tile's rows of the state arrays (workgroup-uniform bases, indexed by
  // the thread)
  g_u64w* x0 = (g_u64w*)ufirst64((uint64_t)(uintptr_t)(C.xs + C.lane0));
  x0[tid] = pre;
  if (cnt) {
    if (!(contig && P->body_gather)) {
      x0[C.xn + tid] = s0;
      x0[2 * C.xn + tid] = stp;
    }
    // the live-ins are uniform over the input: the gather pass reads them
    // from the tile's first thread with iterations only
    if (pre == 0) {
      const uint32_t nl = P->n_livein;
      for (uint32_t q = 0; q < nl; q++) x0[(3 + q) * C.xn + tid] = G.livein[q];
    }
  }
  if (tid == TILE - 1) {
    C.xtot[C.xt] = tot;
    (P->body_gather ? C.xpg : C.xpb)[C.xt] = (tot + PIECE - 1) / PIECE;
    C.xin[C.xt] = C.input;
    C.xd[2 * C.xt] = dref;
    C.xd[2 * C.xt + 1] = contig ? 1ull : 0ull;
  }
  __syncthreads();
}

// One thread in the rows form: the same sites, records, status and
// expanded-loop state as the interpreter's whole-thread pass.
__device__ __forceinline__ void rows_thread(RowsLds& S, const Ctx& C, c_drows& G, const Thr& T, bool act,
                                            uint64_t& acc, uint64_t& hangs, uint32_t& sv) {
  RSlice X;
  const uint32_t ncls = G.ncls;
#pragma unroll
  for (uint32_t c = 0; c < MAX_RCLS; c++) {
    uint64_t v = 0;
    if (c < ncls)
#pragma unroll
      for (int d = 0; d < 6; d++) {
        const uint64_t cf = (uint64_t)G.cc[c][d];
        if (cf) v += cf * coord(T, d);
      }
    X.base[c] = v;
  }
#pragma unroll
  for (uint32_t q = 0; q < RV_MAXLOAD; q++) X.x[q] = 0;
  const uint64_t key = T.gtid << C.Lsum;
  bool on = act, alive = act;
  const uint32_t n = G.n;
  for (uint32_t q = 0; q < n; q++) {
    c_rent& E = G.e[q];
    const uint32_t kind = E.kind, w = E.w;
    if (kind == RE_GUARD) {
      const bool p = on && rcmp(E.op, w, rform(E.a, X, T, w), rform(E.b, X, T, w));
      rsite(sv, 2 * q, __ballot(p));
      rsite(sv, 2 * q + 1, __ballot(on && !p));
      on = p;
    } else if (kind == RE_ENDG) {
      on = alive;
    } else if (kind == RE_LOOP) {
      const uint64_t stp = E.step;
      const uint64_t s0 = rform(E.a, X, T, w);
      const int64_t e0 = (int64_t)rform(E.b, X, T, w);
      const uint64_t nt = on ? rtrips((int64_t)s0, e0, (int64_t)stp) : 0;
      const bool hg = on && nt > C.cap0;
      rows_expand(S, C, G, on ? (nt < C.cap0 ? nt : C.cap0) : 0, s0, stp);
      rsite(sv, 2 * q + 1, __ballot(on && !hg));
      if (hg) {
        on = alive = false;
        hangs++;
      }
    } else {  // ACCESS, LOAD
      const uint32_t lg = E.lg, dst = E.dst;
      c_alloc& A = C.tab[E.slot];
      const int64_t idx = (int64_t)rform(E.a, X, T, w);
      const uint32_t kd = on ? kind_of(A.base, A.size_bytes, A.flags, idx, lg) : 0u;
      acc += on ? 1u : 0u;
      rsite(sv, 2 * q, __ballot(on));
      if (__ballot(kd != 0)) merge_violation(C.rec + E.acc, kd, key);
      if (dst) {
        uint64_t v = 0;
        if (on && kd == 0)
          v = lg == 2 ? (uint64_t)(int64_t)((g_i32*)A.data)[idx] : (uint64_t)((g_i64*)A.data)[idx];
        rset4(X.x, dst - 1, v);
      }
    }
  }
}

// The rows form of an input whose entries are all 32 bits wide, in 32-bit
// arithmetic: a form at width 32 is its value modulo 2^32 (sign-extended
// where a 64-bit value is needed), and the low 32 bits of sums and products
// depend only on the low 32 bits of their operands.  An index is in bounds iff
// its unsigned value is below the slot's element count clamped to 2^31.
struct RSlice32 {
  uint32_t base[MAX_RCLS];
  uint32_t x[RV_MAXLOAD];
};
__device__ __forceinline__ uint32_t rsel4_32(const uint32_t* v, uint32_t k) {
  return k == 0 ? v[0] : k == 1 ? v[1] : k == 2 ? v[2] : v[3];
}
__device__ __forceinline__ void rset4_32(uint32_t* v, uint32_t k, uint32_t x) {
  if (k == 0) v[0] = x;
  else if (k == 1) v[1] = x;
  else if (k == 2) v[2] = x;
  else v[3] = x;
}
__device__ __forceinline__ uint32_t rform32(c_rform& f, const RSlice32& X, const Thr& T) {
  const uint32_t var = f.var;
  uint32_t v = (uint32_t)f.off;
  if (var == RV_COORD) {
    const uint32_t cls = f.cls;
    if (cls != RCLS_NONE) {
      v += rsel4_32(X.base, cls);
    } else {
#pragma unroll
      for (int d = 0; d < 6; d++) v += (uint32_t)f.c[d] * (uint32_t)coord(T, d);
    }
  } else if (var != RV_UNI) {
    v += (uint32_t)f.c[0] * rsel4_32(X.x, var - 1);
  }
  return v;
}
__device__ __forceinline__ bool rcmp32(uint32_t op, uint32_t x, uint32_t y) {
  switch (op) {
    case CKC_OP_CMPEQ: return x == y;
    case CKC_OP_CMPNE: return x != y;
    case CKC_OP_CMPLTS: return (int32_t)x < (int32_t)y;
    case CKC_OP_CMPLES: return (int32_t)x <= (int32_t)y;
    case CKC_OP_CMPLTU: return x < y;
    default: return x <= y;  // CMPLEU
  }
}
__device__ __forceinline__ void rows_thread32(RowsLds& S, const Ctx& C, c_drows& G, const Thr& T, bool act,
                                              uint64_t& acc, uint64_t& hangs, uint32_t& sv) {
  RSlice32 X;
  const uint32_t ncls = G.ncls;
#pragma unroll
  for (uint32_t c = 0; c < MAX_RCLS; c++) {
    uint32_t v = 0;
    if (c < ncls)
#pragma unroll
      for (int d = 0; d < 6; d++) {
        const uint32_t cf = (uint32_t)G.cc[c][d];
        if (cf) v += cf * (uint32_t)coord(T, d);
      }
    X.base[c] = v;
  }
#pragma unroll
  for (uint32_t q = 0; q < RV_MAXLOAD; q++) X.x[q] = 0;
  const uint64_t key = T.gtid << C.Lsum;
  bool on = act, alive = act;
  const uint32_t n = G.n;
  for (uint32_t q = 0; q < n; q++) {
    c_rent& E = G.e[q];
    const uint32_t kind = E.kind;
    if (kind == RE_GUARD) {
      const bool p = on && rcmp32(E.op, rform32(E.a, X, T), rform32(E.b, X, T));
      rsite(sv, 2 * q, __ballot(p));
      rsite(sv, 2 * q + 1, __ballot(on && !p));
      on = p;
    } else if (kind == RE_ENDG) {
      on = alive;
    } else if (kind == RE_LOOP) {
      const uint64_t stp = E.step;
      const int32_t s0 = (int32_t)rform32(E.a, X, T), e0 = (int32_t)rform32(E.b, X, T);
      uint64_t nt = 0;
      if (on)
        nt = stp == 1 ? (s0 < e0 ? (uint64_t)((uint32_t)e0 - (uint32_t)s0) : 0) : trip_count_div(s0, e0, (int64_t)stp);
      const bool hg = on && nt > C.cap0;
      rows_expand(S, C, G, on ? (nt < C.cap0 ? nt : C.cap0) : 0, (uint64_t)(int64_t)s0, stp);
      rsite(sv, 2 * q + 1, __ballot(on && !hg));
      if (hg) {
        on = alive = false;
        hangs++;
      }
    } else {  // ACCESS, LOAD
      const uint32_t lg = E.lg, dst = E.dst;
      c_alloc& A = C.tab[E.slot];
      const uint64_t ne = A.size_bytes >> lg;
      const uint32_t bnd = ne > 0x80000000ull ? 0x80000000u : (uint32_t)ne;
      const uint32_t dk = A.base == 0 ? CKC_KIND_NULL : (A.flags & CKC_ALLOC_FREED) ? CKC_KIND_FREED : 0u;
      const uint32_t v = rform32(E.a, X, T);
      const uint32_t kd = !on ? 0u : dk ? dk : (int32_t)v < 0 ? CKC_KIND_UNDER : v >= bnd ? CKC_KIND_OVER : 0u;
      acc += on ? 1u : 0u;
      rsite(sv, 2 * q, __ballot(on));
      if (__ballot(kd != 0)) merge_violation(C.rec + E.acc, kd, key);
      if (dst) {
        uint32_t x = 0;
        if (on && kd == 0) x = lg == 2 ? (uint32_t)((g_i32*)A.data)[v] : (uint32_t)((g_i64*)A.data)[v];
        rset4_32(X.x, dst - 1, x);
      }
    }
  }
}

// Coverage and status of the current input into its global counters (the
// whole workgroup).
__device__ void flush_rows(RowsLds& S, const KArgs& a, uint32_t input, uint32_t n_sites, uint64_t& acc,
                           uint64_t& hangs, uint32_t& sv) {
  const dinput& in = a.inputs[input];
  uint32_t* cnt = a.counts + in.cnt_base;
  rsite_flush(S, sv, *(c_drows*)in.trace, cnt);
  const uint64_t n = wave_sum64(acc), h = wave_sum64(hangs);
  if (lane_id() == 0) {
    if (n) atomicAdd(&S.acc_checked, (unsigned long long)n);
    if (h) atomicAdd(&S.hangs, (unsigned long long)h);
  }
  acc = 0;
  hangs = 0;
  __syncthreads();
  const uint32_t ns = n_sites < (uint32_t)MAX_SITES_LDS ? n_sites : (uint32_t)MAX_SITES_LDS;
  for (uint32_t s = threadIdx.x; s < ns; s += TILE) {
    const uint32_t c = S.sites[s];
    if (c) {
      if (cnt[s] < 255u) atomicAdd(&cnt[s], c < 255u ? c : 255u);
      S.sites[s] = 0;
    }
  }
  if (threadIdx.x == 0) {
    ckc_input_status* st = a.status + input;
    if (S.acc_checked) atomicAdd((unsigned long long*)&st->accesses_checked, S.acc_checked);
    if (S.hangs) atomicAdd((unsigned long long*)&st->hang_lanes, S.hangs);
    S.acc_checked = 0;
    S.hangs = 0;
  }
  __syncthreads();
}

// W32: the instantiation for batches whose rows forms are all 32 bits wide
// (the loader's PF_ROWS32), without the 64-bit evaluation and its registers.
template <uint32_t SK, bool W32>
__global__ void __launch_bounds__(TILE, W32 ? 7 : 6) eval_rows_kernel(KArgs a) {
  __shared__ RowsLds S;
  const uint32_t tid = threadIdx.x;
  const uint64_t total = a.js->total_tiles[PATH_GENERIC];
  if (total == 0) return;
  Sched<SK> sc;
  sched_init(sc, a, total);
  if (SK == CKC_SCHED_BLOCKED && sc.cur >= sc.end) return;
  c_input* ins = (c_input*)a.inputs;
  c_u32* order = (c_u32*)a.order;
  for (uint32_t s = tid; s < MAX_SITES_LDS; s += TILE) S.sites[s] = 0;
  if (tid == 0) { S.acc_checked = 0; S.hangs = 0; }
  uint32_t pos = 0xFFFFFFFFu, cur = 0xFFFFFFFFu, cur_sites = 0, cur_mode = 0, sv = 0;
  uint64_t tb = 0, cur_end = 0, cur_lanes = 0, acc = 0, hangs = 0;
  uint32_t cur_L[7] = {0, 0, 0, 0, 0, 0, 0};
  Dec dec;
  for (;;) {
    __syncthreads();
    const uint64_t t = sched_next(sc, &a.js->next_tile[PATH_GENERIC], &S.item_slot);
    if (t == ~0ull) break;
    if (pos == 0xFFFFFFFFu || t < tb || t >= cur_end) {
      pos = pos_of_tile(ins, order, a.n_inputs, PATH_GENERIC, pos, cur_end, t);
      const uint32_t i = order[pos];
      if (cur != 0xFFFFFFFFu) flush_rows(S, a, cur, cur_sites, acc, hangs, sv);
      cur = i;
      cur_sites = ((c_dprog*)a.inputs[i].prog)->n_sites;
      tb = ins[i].tile_begin[PATH_GENERIC];
      cur_end = tb + ins[i].n_tiles[PATH_GENERIC];
      for (int q = 0; q < 6; q++) cur_L[q] = ins[i].launch[q];
      cur_L[6] = ins[i].aux;
      cur_mode = ins[i].mode;
      cur_lanes = ins[i].lanes;
      dec_make(dec, cur_L);
    }
    const uint32_t i = cur;
    c_input& in = ins[i];
    c_dprog* Pi = (c_dprog*)in.prog;
    c_drows* G = (c_drows*)in.trace;
    if (!(Pi->pflags & PF_ROWS) || in.detector || in.xstate == 0 || in.trace == 0 || !G->ok) {
      // not reached: the host takes this kernel only when every program passes
      // the walk; the input's status says so rather than a silent gap
      if (tid == 0) atomicOr(&a.status[i].flags, (uint32_t)CKC_ST_INTERNAL);
      continue;
    }
    const uint64_t l = (t - tb) * TILE + tid;
    const bool act = l < cur_lanes;
    Thr T;
    if (cur_mode == CKC_FULL) decode_full(dec, act ? l : 0, T);
    else decode_lane(cur_mode, cur_L, cur_L[6], act ? l : 0, T);
    Ctx C;
    ctx_init(C, a, in, i, T);
    C.lane0 = (t - tb) * TILE;
    C.xt = in.xt_begin + (t - tb);
    if (W32 || G->all32) {
      // W32 with a form wider than 32 bits is not reached (the loader's flag
      // and the plan kernel's walk agree): every thread of the tile would be
      // inactive, the tile empty, and the input's status says so
      if (!G->all32 && tid == 0) atomicOr(&a.status[i].flags, (uint32_t)CKC_ST_INTERNAL);
      rows_thread32(S, C, *G, T, act && G->all32, acc, hangs, sv);
    } else {
      rows_thread(S, C, *G, T, act, acc, hangs, sv);
    }
  }
  if (cur != 0xFFFFFFFFu) flush_rows(S, a, cur, cur_sites, acc, hangs, sv);
}

// Exclusive scan, in place, of the per-tile piece counts of expanded loops
// (a.xpb, a.n_xtiles entries) in three steps: per-block sums of XSB entries,
// a scan of the block sums (which also stores the total), per-block rescans.
constexpr uint32_t XSB = 4096;
__global__ void __launch_bounds__(256) xscan_sums_kernel(KArgs a, uint32_t which) {
  __shared__ unsigned long long part[4];
  unsigned long long* xp = which ? a.xpg : a.xpb;
  unsigned long long* bsum = a.xbsum + which * gridDim.x;
  const uint64_t b0 = (uint64_t)blockIdx.x * XSB;
  unsigned long long v = 0;
  for (uint32_t q = threadIdx.x; q < XSB; q += 256)
    if (b0 + q < a.n_xtiles) v += xp[b0 + q];
  v = wave_sum64(v);
  if (lane_id() == 0) part[threadIdx.x / 64] = v;
  __syncthreads();
  if (threadIdx.x == 0) bsum[blockIdx.x] = part[0] + part[1] + part[2] + part[3];
}
__global__ void __launch_bounds__(1024) xscan_blocks_kernel(KArgs a, uint32_t n_blocks, uint32_t which) {
  __shared__ unsigned long long part[16];
  __shared__ unsigned long long carry;
  unsigned long long* bsum = a.xbsum + which * n_blocks;
  const uint32_t t = threadIdx.x;
  if (t == 0) carry = 0;
  __syncthreads();
  for (uint32_t base = 0; base < n_blocks; base += 1024) {
    const uint32_t i = base + t;
    const uint64_t v = i < n_blocks ? bsum[i] : 0;
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
    if (i < n_blocks) bsum[i] = c + w + sc - v;
    __syncthreads();
    if (t == 1023) carry = c + w + sc;
    __syncthreads();
  }
  if (t == 0) {
    a.js->total_pieces[which] = carry;
    a.js->next_piece[which] = 0;
  }
}
__global__ void __launch_bounds__(256) xscan_apply_kernel(KArgs a, uint32_t which) {
  __shared__ unsigned long long part[4];
  __shared__ unsigned long long carry;
  unsigned long long* xp = which ? a.xpg : a.xpb;
  const uint64_t b0 = (uint64_t)blockIdx.x * XSB;
  if (threadIdx.x == 0) carry = a.xbsum[which * gridDim.x + blockIdx.x];
  __syncthreads();
  for (uint32_t base = 0; base < XSB; base += 256) {
    const uint64_t e = b0 + base + threadIdx.x;
    const uint64_t v = e < a.n_xtiles ? xp[e] : 0;
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
    if (e < a.n_xtiles) xp[e] = c + w + sc - v;
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

// Builds the gather entries of the expanded body for the current input
// (wavefront 0; lane 0 holds the constant part of each register, lane 1 its
// coefficient of the register's variable).  `live` is the owner thread's lane
// whose stored live-ins are used (they are uniform over the input).
__device__ __forceinline__ void build_gather(GenLds& S, uint64_t* R, const Ctx& C, uint32_t lpc, uint32_t endpc, uint64_t live) {
  const uint32_t j = lane_id();
  c_dprog* P = C.P;
  c_dins* I = C.I;
  GBody& G = S.gb;
  auto rg = [&](uint32_t r) -> uint64_t& { return R[r * TILE + j]; };
  // one wavefront: its LDS accesses are performed in program order
  if (j == 0) { G.n = 0; G.ok = 1; G.faults = 0; }
  for (uint32_t r = j; r < NREG; r += 64) G.var[r] = 0xFF;
  const uint32_t nl = P->n_livein;
  for (uint32_t q = 0; q < nl; q++) {
    const uint32_t r = ufirst(P->livein[q]);
    if (j < 2) rg(r) = j == 0 ? C.xs[(3 + q) * C.xn + live] : 0ull;
  }
  const dins L = ld_ins(I, lpc);
  const uint32_t ctr = ufirst(L.dst);
  if (j < 2) rg(ctr) = j == 0 ? 0ull : 1ull;
  if (j == 0) G.var[ctr] = 0;
  uint32_t n_load = 0, ok = 1, n = 0, faults = 0;
  for (uint32_t pc = lpc + 1; pc < endpc && ok; pc++) {
    const dins D = ld_ins(I, pc);
    const uint32_t op = D.op, w = D.w;
    const uint32_t da = ufirst(D.a), db = ufirst(D.b), dc = ufirst(D.c), dd = ufirst(D.dst);
    const uint64_t a = j < 2 ? rg(da) : 0, b = j < 2 ? rg(db) : 0, c = j < 2 ? rg(dc) : 0;
    const uint32_t va = G.var[da], vb = G.var[db];
    uint64_t r = 0;
    uint32_t rv = 0xFF;
    bool wr = true;
    switch (op) {
      case CKC_OP_CONST: r = j == 0 ? narrow((uint64_t)C.K[D.x], w) : 0; break;
      case CKC_OP_SCALAR: r = j == 0 ? narrow((uint64_t)C.sc[D.x], w) : 0; break;
      case CKC_OP_SPECIAL:
        if (D.x < 6) { ok = 0; break; }
        r = j == 0 ? (D.x < 9 ? C.in->launch[3 + D.x - 6] : C.in->launch[D.x - 9]) : 0;
        break;
      case CKC_OP_ACCESS:
      case CKC_OP_LOAD: {
        if (n >= MAX_GENT) { ok = 0; break; }
        const uint64_t off = readlane64(a, 0), coef = readlane64(a, 1);
        if (j == 0) {
          GEnt& E = G.e[n];
          E.coef = va == 0xFF ? 0 : (int64_t)coef;
          E.off = (int64_t)off;
          E.acc = D.x;
          E.site = D.s0;
          E.slot = D.slot;
          E.lg = D.fl & 3u;
          E.w = (uint8_t)w;
          E.var = (uint8_t)va;
          E.dst = op == CKC_OP_LOAD ? (uint8_t)(n_load + 1) : 0;
          c_alloc& A = C.tab[D.slot];
          E.bound = A.size_bytes >> E.lg;
          E.data = A.data;
          E.dead = A.base == 0 ? CKC_KIND_NULL : ((A.flags & CKC_ALLOC_FREED) ? CKC_KIND_FREED : 0);
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
      case CKC_OP_ADD: case CKC_OP_SUB:
        if (va != 0xFF && vb != 0xFF && va != vb) { ok = 0; break; }
        r = narrow(op == CKC_OP_ADD ? a + b : a - b, w);
        rv = va != 0xFF ? va : vb;
        break;
      case CKC_OP_MUL:
        if (va != 0xFF && vb != 0xFF) { ok = 0; break; }
        r = narrow(va != 0xFF ? a * readlane64(b, 0) : b * readlane64(a, 0), w);
        rv = va != 0xFF ? va : vb;
        if (va == 0xFF && vb == 0xFF) r = j == 0 ? narrow(readlane64(a, 0) * readlane64(b, 0), w) : 0;
        break;
      case CKC_OP_SHL:
        if (vb != 0xFF) { ok = 0; break; }
        r = narrow(a << (readlane64(b, 0) & (uint64_t)(w - 1)), w);
        rv = va;
        break;
      case CKC_OP_SELECT:
        if (va != 0xFF || vb != 0xFF || G.var[dc] != 0xFF) { ok = 0; break; }
        r = j == 0 ? narrow(readlane64(a, 0) != 0 ? readlane64(b, 0) : readlane64(c, 0), w) : 0;
        break;
      case CKC_OP_SEXT: case CKC_OP_TRUNC:
        if (va != 0xFF) { ok = 0; break; }
        r = j == 0 ? narrow(readlane64(a, 0), 32) : 0;
        break;
      case CKC_OP_ZEXT:
        if (va != 0xFF) { ok = 0; break; }
        r = j == 0 ? (readlane64(a, 0) & 0xFFFFFFFFull) : 0;
        break;
      default: {
        if (op < CKC_OP_ADD || op > CKC_OP_CMPLEU || va != 0xFF || vb != 0xFF) { ok = 0; break; }
        uint32_t f = 0;
        const uint64_t v = alu(op, w, readlane64(a, 0), readlane64(b, 0), f);
        faults += f;
        r = j == 0 ? v : 0;
        break;
      }
    }
    if (ok && wr) {
      if (j < 2) rg(dd) = r;
      if (j == 0) G.var[dd] = (uint8_t)rv;
    }
  }
  if (j == 0) { G.n = n; G.ok = ok; G.faults = faults; }
}

// Evaluates one chunk of a gather body: X lives in the register file rows
// 0..7 of the lane.  `k` is the lane's iteration, `ctr` the counter value.
__device__ __forceinline__ void run_gather(GenLds& S, uint64_t* R, const Ctx& C, Lane& ln, uint64_t& sat,
                                           uint64_t ctr) {
  const bool act = ln.dis == 0;
  R[threadIdx.x] = ctr;
  const uint32_t n = S.gb.n;
  const uint64_t key = (ln.gtid << C.Lsum) | (ln.k0 << C.L2);
  const uint64_t am = __ballot(act);
  for (uint32_t e = 0; e < n; e++) {
    const GEnt& E = S.gb.e[e];
    const uint32_t var = ufirst(E.var), slot = ufirst(E.slot), lg = ufirst(E.lg), w = ufirst(E.w);
    const uint64_t coef = ufirst64((uint64_t)E.coef), off = ufirst64((uint64_t)E.off);
    uint64_t v = off;
    if (var != 0xFF) {
      const uint64_t x = R[var * TILE + threadIdx.x];
      v = coef == 1 ? off + x : off + coef * x;
    }
    const int64_t idx = (int64_t)narrow(v, w);
    c_alloc& A = C.tab[slot];
    const uint32_t kd = act ? kind_of(A.base, A.size_bytes, A.flags, idx, lg) : 0u;
    count_site(S, C, sat, ufirst(E.site), am);
    if (__ballot(kd != 0)) merge_violation(C.rec + ufirst(E.acc), kd, key);
    const uint32_t dst = ufirst(E.dst);
    if (dst) {
      uint64_t x = 0;
      if (act && kd == 0)
        x = lg == 2 ? (uint64_t)(int64_t)((g_i32*)A.data)[idx] : (uint64_t)((g_i64*)A.data)[idx];
      R[dst * TILE + threadIdx.x] = x;
    }
  }
  if (act) {
    ln.acc += n;
    ln.faults += S.gb.faults;
  }
}

// Kind of index idx of a live-or-dead slot with `bound` elements (the same
// precedence as kind_of: NULL > FREED > UNDER > OVER).
__device__ __forceinline__ uint32_t kind_bound(uint32_t dead, uint64_t bound, int64_t idx) {
  if (dead) return dead;
  if (idx < 0) return CKC_KIND_UNDER;
  return (uint64_t)idx >= bound ? CKC_KIND_OVER : 0u;
}

// Owner of iteration g in a tile: the largest o with pref[o] <= g.
__device__ __forceinline__ uint32_t owner_of(const GenLds& S, uint64_t g) {
  uint32_t l2 = 0, h2 = TILE - 1;
  while (l2 < h2) {
    const uint32_t m = (l2 + h2 + 1) >> 1;
    if (S.pref[m] <= g) l2 = m;
    else h2 = m - 1;
  }
  return l2;
}

// Adds c visits of site s for the wavefront (lane 0 updates the counter); the
// wavefront is converged.
__device__ __forceinline__ void count_site_n(GenLds& S, const Ctx& C, uint64_t& sat, uint32_t s, uint32_t c) {
  if (s == NOSITE || c == 0) return;
  if (s < 64 && ((sat >> s) & 1u)) return;
  if (s < MAX_SITES_LDS) {
    uint32_t old = 0;
    if (lane_id() == 0) old = atomicAdd(&S.sites[s], c);
    old = __builtin_amdgcn_readlane(old, 0);
    if (s < 64 && old + c >= 255u) sat |= 1ull << s;
  } else if (lane_id() == 0 && C.gcnt[s] < 255u) {
    atomicAdd(&C.gcnt[s], c);
  }
}

// Entries of a gather body evaluated by the piece evaluator (larger bodies go
// through run_gather).
constexpr uint32_t GREG = 4;

// Evaluates the iterations [it0, it1) of a piece of a gather body with at most
// GREG entries.  A lane takes U iterations at a time (one per chunk of TILE),
// forms each counter from its owner's start and step, and evaluates each entry
// for all U before the next entry, so that the U loads of an entry are in
// flight together.  The loaded value of LOAD number d (1-based) for chunk q
// lives in R row (d-1)*U + q, so the body's loads need U rows each.  A
// violation (rare) is recorded by recomputing that chunk's key and index.
// TS: the input's thread set -- launch dims, then the PREX round (MODE_PAIR).
template <uint32_t U>
__device__ __forceinline__ void gather_piece(GenLds& S, uint64_t* R, const Ctx& C, Lane& ln, uint64_t& sat,
                                             uint64_t it0, uint64_t it1, uint64_t lane0, uint32_t mode,
                                             const uint32_t* TS, uint32_t site_iter, uint32_t ctr_w) {
  const uint32_t tid = threadIdx.x;
  const uint32_t n = S.gb.n;
  const uint32_t faults = S.gb.faults;
  for (uint64_t base = it0; base < it1; base += (uint64_t)TILE * U) {
    uint64_t ctr[U];
    bool act[U];
    uint32_t nact = 0, mine = 0;
#pragma unroll
    for (uint32_t q = 0; q < U; q++) {
      const uint64_t g = base + q * TILE + tid;
      act[q] = g < it1;
      const uint32_t o = act[q] ? (uint32_t)S.own[g - it0] : 0u;
      const uint64_t k = act[q] ? g - S.pref[o] : 0;
      ctr[q] = narrow(S.xstart[o] + k * S.xstep[o], ctr_w);
      nact += (uint32_t)__popcll(__ballot(act[q]));
      mine += act[q] ? 1u : 0u;
    }
    count_site_n(S, C, sat, site_iter, nact);
    for (uint32_t e = 0; e < n; e++) {
      const GEnt& E = S.gb.e[e];
      const uint32_t var = ufirst(E.var), dst = ufirst(E.dst), lg = ufirst(E.lg), w64 = ufirst(E.w) == 64;
      const uint32_t dead = ufirst(E.dead);
      const uint64_t coef = ufirst64((uint64_t)E.coef), off = ufirst64((uint64_t)E.off);
      const uint64_t bound = ufirst64(E.bound);
      const void* data = (const void*)ufirst64((uint64_t)E.data);
      uint32_t vio = 0;
#pragma unroll
      for (uint32_t q = 0; q < U; q++) {
        uint64_t v = off;
        if (var != 0xFF) {
          const uint64_t x = var == 0 ? ctr[q] : R[((var - 1) * U + q) * TILE + tid];
          v = coef == 1 ? v + x : v + coef * x;
        }
        const int64_t idx = w64 ? (int64_t)v : (int64_t)(int32_t)(uint32_t)v;
        const uint32_t kd = act[q] ? kind_bound(dead, bound, idx) : 0u;
        if (__ballot(kd != 0)) vio |= 1u << q;
        if (dst) {
          uint64_t x = 0;
          if (act[q] && kd == 0)
            x = lg == 2 ? (uint64_t)(int64_t)((g_i32*)data)[idx] : (uint64_t)((g_i64*)data)[idx];
          R[((dst - 1) * U + q) * TILE + tid] = x;
        }
      }
      count_site_n(S, C, sat, ufirst(E.site), nact);
      for (uint32_t q = 0; q < U; q++) {
        if (!((vio >> q) & 1u)) continue;
        const uint64_t g = base + q * TILE + tid;
        const bool a = g < it1;
        const uint32_t o = a ? (uint32_t)S.own[g - it0] : 0u;
        const uint64_t k = a ? g - S.pref[o] : 0;
        const uint64_t l = lane0 + o;
        uint64_t gtid = l;
        if (mode != CKC_FULL) {
          Thr T;
          decode_lane(mode, TS, TS[6], l, T);
          gtid = T.gtid;
        }
        uint64_t v = off;
        if (var != 0xFF) {
          const uint64_t x = var == 0 ? narrow(S.xstart[o] + k * S.xstep[o], ctr_w) : R[((var - 1) * U + q) * TILE + tid];
          v = coef == 1 ? v + x : v + coef * x;
        }
        const int64_t idx = w64 ? (int64_t)v : (int64_t)(int32_t)(uint32_t)v;
        const uint32_t kd = a ? kind_bound(dead, bound, idx) : 0u;
        merge_violation(C.rec + ufirst(E.acc), kd, (gtid << C.Lsum) | (k << C.L2));
      }
    }
    ln.acc += (uint64_t)n * mine;
    ln.faults += (uint64_t)faults * mine;
  }
}

// Merges this wavefront's violations of gather entry e into the workgroup's
// per-entry record in LDS.
__device__ __forceinline__ void merge_vio_lds(GenLds& S, uint32_t e, uint32_t kd, uint64_t key) {
  const uint64_t mask = __ballot(kd != 0);
  if (mask == 0) return;
  const uint64_t k = wave_min64(kd ? key : ~0ull);
  uint32_t kinds = 0;
  if (__ballot(kd & CKC_KIND_OVER)) kinds |= CKC_KIND_OVER;
  if (__ballot(kd & CKC_KIND_UNDER)) kinds |= CKC_KIND_UNDER;
  if (__ballot(kd & CKC_KIND_FREED)) kinds |= CKC_KIND_FREED;
  if (__ballot(kd & CKC_KIND_NULL)) kinds |= CKC_KIND_NULL;
  const uint32_t leader = (uint32_t)(__ffsll((unsigned long long)mask) - 1);
  if (lane_id() == leader) {
    atomicMin(&S.vfk[e], (unsigned long long)k);
    atomicAdd(&S.vcnt[e], (unsigned long long)__popcll(mask));
    atomicOr(&S.vkinds[e], kinds);
  }
}

// As merge_vio_lds, for a run of chained tiles: the wavefront's least
// violating iteration goes to S.rmin (its owner is found once, at the end of
// the run); count and kinds go to the records directly.
__device__ __forceinline__ void merge_vio_run(GenLds& S, uint32_t e, uint32_t kd, uint64_t g) {
  const uint64_t mask = __ballot(kd != 0);
  if (mask == 0) return;
  const uint64_t gm = wave_min64(kd ? g : ~0ull);
  uint32_t kinds = 0;
  if (__ballot(kd & CKC_KIND_OVER)) kinds |= CKC_KIND_OVER;
  if (__ballot(kd & CKC_KIND_UNDER)) kinds |= CKC_KIND_UNDER;
  if (__ballot(kd & CKC_KIND_FREED)) kinds |= CKC_KIND_FREED;
  if (__ballot(kd & CKC_KIND_NULL)) kinds |= CKC_KIND_NULL;
  const uint32_t leader = (uint32_t)(__ffsll((unsigned long long)mask) - 1);
  if (lane_id() == leader) {
    atomicMin(&S.rmin[e], (unsigned long long)gm);
    atomicAdd(&S.vcnt[e], (unsigned long long)__popcll(mask));
    atomicOr(&S.vkinds[e], kinds);
  }
}

// Flushes the per-entry violation records of the current gather body into the
// input's records (workgroup-converged; S.gb still holds that body).
__device__ __forceinline__ void flush_vio_lds(GenLds& S, ckc_record* rec) {
  const uint32_t e = threadIdx.x;
  if (e < MAX_GENT && e < S.gb.n && S.vcnt[e]) {
    ckc_record* r = rec + S.gb.e[e].acc;
    atomicMin((unsigned long long*)&r->first_key, S.vfk[e]);
    atomicAdd((unsigned long long*)&r->count, S.vcnt[e]);
    atomicOr(&r->kinds, S.vkinds[e]);
  }
  if (e < MAX_GENT) {
    S.vfk[e] = ~0ull;
    S.vcnt[e] = 0;
    S.vkinds[e] = 0;
  }
}

// Gather bodies of at most GREG entries whose entries and counter are all of
// width 32, with at most two loads, over a contiguous tile (every owner's
// counter is start + k with start - prefix the same d for all owners): the
// counter of iteration g is d + g, so no owner map is needed, and all index
// arithmetic is 32-bit (the low 32 bits of an index depend only on the low 32
// bits of its operands).  A lane takes U iterations at a time, one per chunk
// of TILE, and evaluates each entry for all U before the next one, so that
// the U loads of an entry are in flight together.  The body is straight-line,
// so every site of it is visited once per iteration: the visits are counted
// once at the end.  A violating chunk of an entry keeps its index values in
// R32 (row q of TILE lanes, 32 bits; the dynamic LDS holds at least 16 such
// rows) and, right after the entry (rare), finds each lane's owner by binary
// search and merges into the workgroup's per-entry records.  Rounds wholly
// inside the range drop the per-lane range tests, and an entry indexed by the
// counter with coefficient 1 whose indices in the round all lie in bounds
// (one uniform test) is loaded, or passed over, with no per-lane check.
// One entry of the contiguous form over U chunks: XV selects the index
// variable (-1 none, 0 the counter, 1 or 2 the first or second loaded value),
// DV the loaded value the entry defines (0 none), FULL that every iteration
// of the round is in range (act unused).  The counter of chunk q is
// c0 + q * TILE.  Loads land directly in their variable, so the U loads are in
// flight together; a lane with nothing to load reads element 0 (valid: the
// caller passes DV = 0 when no index can be in bounds) and keeps 0.  Returns
// the chunks with a violating lane; their index values go to R32.
template <uint32_t U, int XV, int DV, bool FULL>
__device__ __forceinline__ uint32_t c32_entry(uint32_t c0, uint32_t* l1, uint32_t* l2, const bool* act,
                                              uint32_t off, uint32_t coef, bool c1, uint32_t bnd, bool dead,
                                              uint32_t sh, const void* data, uint32_t* R32, uint32_t tid) {
  uint32_t vio = 0;
#pragma unroll
  for (uint32_t q = 0; q < U; q++) {
    uint32_t vv = off;
    if (XV >= 0) {
      const uint32_t x = XV == 0 ? c0 + q * TILE : XV == 1 ? l1[q] : l2[q];
      if (c1) vv += x;
      else vv += coef * x;
    }
    const bool on = FULL || act[q];
    const bool bad = on && (dead || vv >= bnd);
    if (__ballot(bad)) {
      vio |= 1u << q;
      R32[q * TILE + tid] = vv;
    }
    if (DV != 0) {
      const bool ld = on && !bad;
      const uint32_t ix = ld ? vv : 0u;
      uint32_t val = (uint32_t) * (g_i32*)((const __attribute__((address_space(1))) uint8_t*)data + ((uint64_t)ix << sh));
      val = ld ? val : 0u;
      if (DV == 1) l1[q] = val;
      else l2[q] = val;
    }
  }
  return vio;
}

// Loads of an entry whose U * TILE indices of the round are the consecutive
// values i0, i0 + 1, ..., all in bounds: no check, and the address of chunk q
// is a uniform base plus the lane and an immediate.
template <uint32_t U, bool W32>
__device__ __forceinline__ void c32_stream(uint32_t* l, const void* data, uint32_t i0, uint32_t tid) {
  if (W32) {
    const g_i32* p = (const g_i32*)data + i0;
#pragma unroll
    for (uint32_t q = 0; q < U; q++) l[q] = (uint32_t)p[q * TILE + tid];
  } else {
    const g_i64* p = (const g_i64*)data + i0;
#pragma unroll
    for (uint32_t q = 0; q < U; q++) l[q] = (uint32_t)p[q * TILE + tid];
  }
}

// One round of the contiguous form: U chunks of TILE iterations from base.
// FULL: the whole round lies before it1.  An entry indexed by the counter with
// coefficient 1 whose round of indices lies inside its allocation (one
// uniform comparison) takes no per-iteration check.  NL: the body's loads
// (one or two; with one, the second loaded value's registers do not exist).
// PRE: entry 0 is the body's one load, streamed by the caller into pre.
template <uint32_t U, bool FULL, uint32_t NL, bool PRE = false>
__device__ __forceinline__ void c32_round(GenLds& S, uint32_t* R32, const Ctx& C, uint64_t base, uint64_t it0,
                                          uint64_t it1, uint32_t d32, uint32_t n, uint64_t lane0, uint32_t mode,
                                          const uint32_t* TS, bool run, uint32_t& mine, uint64_t& visits,
                                          const uint32_t* pre = nullptr) {
  const uint32_t tid = threadIdx.x;
  uint32_t l1[U], l2[U];
  bool act[U];
  const uint32_t c0 = d32 + (uint32_t)(base + tid);
#pragma unroll
  for (uint32_t q = 0; q < U; q++) {
    act[q] = FULL || base + q * TILE + tid < it1;
    l1[q] = PRE ? pre[q] : 0u;
    l2[q] = 0;
    if (!FULL) {
      mine += act[q] ? 1u : 0u;
      visits += (uint64_t)__popcll(__ballot(act[q]));  // this wavefront's iterations
    }
  }
  if (FULL) {
    mine += U;
    visits += (uint64_t)U * 64;
  }
  for (uint32_t e = PRE ? 1u : 0u; e < n; e++) {
    const GEnt& E = S.gb.e[e];
    const uint32_t meta = ufirst((uint32_t)E.var | ((uint32_t)E.dst << 8) | ((uint32_t)E.lg << 16) |
                                 ((uint32_t)(E.coef == 1) << 24) | ((uint32_t)(E.dead != 0) << 25));
    const uint32_t var = meta & 0xFFu, dst = (meta >> 8) & 0xFFu;
    const bool lg2 = ((meta >> 16) & 0xFFu) == 2, c1 = (meta >> 24) & 1u, dead = (meta >> 25) & 1u;
    const uint32_t off = ufirst((uint32_t)E.off), coef = (uint32_t)E.coef;
    const uint64_t b64 = ufirst64(E.bound);
    const uint32_t bnd = b64 > 0x80000000ull ? 0x80000000u : (uint32_t)b64;
    const void* data = (const void*)ufirst64((uint64_t)E.data);
    if (FULL && var == 0 && c1 && !dead && dst != 2) {
      const uint32_t i0 = ufirst(off + d32 + (uint32_t)base);  // index of the round's first iteration
      if ((uint64_t)i0 + (uint64_t)U * TILE <= bnd) {
        if (dst == 1) {
          if (lg2) c32_stream<U, true>(l1, data, i0, tid);
          else c32_stream<U, false>(l1, data, i0, tid);
        }
        continue;
      }
    }
    // no index of the entry can be in bounds: nothing to load, values 0
    const bool none = dead || bnd == 0;
    uint32_t vio;
#define C32E(XV, DV) \
  vio = c32_entry<U, XV, DV, FULL>(c0, l1, l2, act, off, coef, c1, bnd, dead, lg2 ? 2u : 3u, data, R32, tid)
#define C32D(XV)                  \
  if (dst == 0 || none) C32E(XV, 0); \
  else if (NL == 1 || dst == 1) C32E(XV, 1); \
  else C32E(XV, 2)
    if (var == 0xFF) { C32D(-1); }
    else if (var == 0) { C32D(0); }
    else if (NL == 1 || var == 1) { C32D(1); }
    else { C32D(2); }
#undef C32D
#undef C32E
    if (dst != 0 && none) {
#pragma unroll
      for (uint32_t q = 0; q < U; q++) {
        if (dst == 1) l1[q] = 0;
        else l2[q] = 0;
      }
    }
    for (uint32_t bits = vio; bits; bits &= bits - 1) {
      const uint32_t q = (uint32_t)__ffs((int)bits) - 1;
      const uint32_t vv = R32[q * TILE + tid];
      const uint64_t g = base + q * TILE + tid;
      const bool bad = g < it1 && (dead || vv >= bnd);
      const uint32_t kd = !bad ? 0u : dead ? ufirst(E.dead) : ((int32_t)vv < 0 ? CKC_KIND_UNDER : CKC_KIND_OVER);
      if (run) {
        merge_vio_run(S, e, kd, g);
        continue;
      }
      const uint32_t o = owner_of(S, g < it1 ? g : it0);
      const uint64_t k = g < it1 ? g - S.pref[o] : 0;
      const uint64_t l = lane0 + o;
      uint64_t gtid = l;
      if (mode != CKC_FULL) {
        Thr T;
        decode_lane(mode, TS, TS[6], l, T);
        gtid = T.gtid;
      }
      merge_vio_lds(S, e, kd, (gtid << C.Lsum) | (k << C.L2));
    }
  }
}

// With BIG, long ranges go in rounds of 16 chunks (more loads in flight), the
// rest in rounds of 8 (a piece of PIECE iterations is one round); the larger
// rounds cost registers that the per-piece state of jobs of many small inputs
// then spills.  run: [it0, it1)
// spans a run of chained tiles (full thread set only): a violation's owner is
// not looked up here, merge_vio_run keeps the least violating iteration per
// entry instead.
template <bool BIG, uint32_t NL>
__device__ __forceinline__ void gather_c32(GenLds& S, uint32_t* R32, const Ctx& C, Lane& ln, uint64_t& sat,
                                           uint64_t it0, uint64_t it1, uint64_t lane0, uint32_t mode,
                                           const uint32_t* TS, uint32_t site_iter, uint32_t d32, bool run) {
  // R32 rows: UL (the launch gives large-round jobs at least 32 rows)
  constexpr uint32_t UL = NL == 1 ? 32 : 16, US = 8;
  const uint32_t n = S.gb.n, faults = S.gb.faults;
  uint64_t visits = 0;
  uint32_t mine = 0;
  uint64_t base = it0;
  if (BIG && NL == 1 && it1 - it0 >= 2ull * TILE * UL) {
    // entry 0 the body's only load, of 32-bit elements at the counter, every
    // index of the whole rounds in bounds: the next round's loads are issued
    // before the current round is checked (twice the loads in flight)
    const GEnt& E0 = S.gb.e[0];
    const uint32_t m0 = ufirst((uint32_t)E0.var | ((uint32_t)E0.dst << 8) | ((uint32_t)E0.lg << 16) |
                               ((uint32_t)(E0.coef == 1) << 24) | ((uint32_t)(E0.dead != 0) << 25));
    const uint64_t nr = (it1 - it0) / ((uint64_t)TILE * UL);  // whole rounds
    const uint32_t i0 = ufirst((uint32_t)E0.off + d32 + (uint32_t)it0);
    const uint64_t b64 = ufirst64(E0.bound);
    const uint64_t bnd = b64 > 0x80000000ull ? 0x80000000ull : b64;
    if (m0 == ((0u) | (1u << 8) | (2u << 16) | (1u << 24)) && (uint64_t)i0 + nr * TILE * UL <= bnd) {
      const void* data0 = (const void*)ufirst64((uint64_t)E0.data);
      uint32_t la[UL], lb[UL];
#pragma unroll
      for (uint32_t q = 0; q < UL; q++) lb[q] = 0;  // the last round loads no next one
      c32_stream<UL, true>(la, data0, i0, threadIdx.x);
      for (uint64_t r = 0; r < nr; r++, base += (uint64_t)TILE * UL) {
        if (r + 1 < nr) c32_stream<UL, true>(lb, data0, i0 + (uint32_t)((r + 1) * TILE * UL), threadIdx.x);
        c32_round<UL, true, NL, true>(S, R32, C, base, it0, it1, d32, n, lane0, mode, TS, run, mine, visits, la);
#pragma unroll
        for (uint32_t q = 0; q < UL; q++) la[q] = lb[q];
      }
    }
  }
  if (BIG)
    for (; base + (uint64_t)TILE * UL <= it1; base += (uint64_t)TILE * UL)
      c32_round<UL, true, NL>(S, R32, C, base, it0, it1, d32, n, lane0, mode, TS, run, mine, visits);
  for (; base + (uint64_t)TILE * US <= it1; base += (uint64_t)TILE * US)
    c32_round<US, true, NL>(S, R32, C, base, it0, it1, d32, n, lane0, mode, TS, run, mine, visits);
  if (base < it1) c32_round<US, false, NL>(S, R32, C, base, it0, it1, d32, n, lane0, mode, TS, run, mine, visits);
  // visits of the counter's site and of every entry's site
  const uint32_t vc = (uint32_t)(visits < 0xFFFFFFFFull ? visits : 0xFFFFFFFFull);
  count_site_n(S, C, sat, site_iter, vc);
  for (uint32_t e = 0; e < n; e++) count_site_n(S, C, sat, ufirst(S.gb.e[e].site), vc);
  ln.acc += (uint64_t)n * mine;
  ln.faults += (uint64_t)faults * mine;
}

// Ends a run of chained tiles (workgroup-converged): for each gather entry
// with a violation in the run, the owner of its least violating iteration is
// found in the prefix of the tile that holds it (the first tile's in LDS, a
// later one's in memory), and the entry's key is merged.  lane0 is the first
// tile's first lane.
__device__ __forceinline__ void end_run(GenLds& S, const Ctx& C, const uint64_t* xs, uint64_t lane0, uint32_t n) {
  __syncthreads();
  const uint32_t e = threadIdx.x;
  if (e < n && S.rmin[e] != ~0ull) {
    const uint64_t g = S.rmin[e];
    uint32_t lo = 0, hi = S.rn;
    while (lo < hi) {
      const uint32_t m = (lo + hi + 1) >> 1;
      if (S.rstart[m] <= g) lo = m;
      else hi = m - 1;
    }
    const uint64_t gl = g - S.rstart[lo];
    const uint64_t l0 = lane0 + (uint64_t)lo * TILE;
    uint32_t o;
    uint64_t pre;
    if (lo == 0) {
      o = owner_of(S, gl);
      pre = S.pref[o];
    } else {
      uint32_t l2 = 0, h2 = TILE - 1;
      while (l2 < h2) {
        const uint32_t m = (l2 + h2 + 1) >> 1;
        if (xs[l0 + m] <= gl) l2 = m;
        else h2 = m - 1;
      }
      o = l2;
      pre = xs[l0 + o];
    }
    atomicMin(&S.vfk[e], (unsigned long long)(((l0 + o) << C.Lsum) | ((gl - pre) << C.L2)));
    S.rmin[e] = ~0ull;
  }
}

// Owner map of the iterations [it0, it1) of a piece: S.own[g - it0] is the
// tile thread that owns iteration g.  Every thread of the tile whose iteration
// range starts inside the piece marks its start; a workgroup max-scan over the
// marks (owners increase with the iteration) fills the rest, the piece's
// first iteration taking the owner found by one binary search.
__device__ __forceinline__ void build_owner_map(GenLds& S, uint64_t it0, uint64_t it1) {
  const uint32_t tid = threadIdx.x;
  constexpr uint32_t PER = PIECE_LDS / TILE;  // entries per thread
  for (uint32_t q = 0; q < PER; q++) S.own[tid * PER + q] = 0;
  const uint32_t o0 = owner_of(S, it0);
  __syncthreads();
  {
    const uint64_t st = S.pref[tid], en = S.pref[tid + 1];
    if (en > st && st > it0 && st < it1) S.own[st - it0] = (uint16_t)tid;
    if (tid == 0) S.own[0] = (uint16_t)o0;
  }
  __syncthreads();
  // max-scan: PER entries per thread, then across threads
  uint32_t m = 0;
  for (uint32_t q = 0; q < PER; q++) {
    const uint32_t v = S.own[tid * PER + q];
    m = v > m ? v : m;
  }
  uint32_t incl = m;
  for (int o = 1; o < 64; o <<= 1) {
    const uint32_t u = __shfl_up(incl, o, 64);
    if ((int)lane_id() >= o) incl = u > incl ? u : incl;
  }
  if (lane_id() == 63) S.omax[tid / 64] = (uint16_t)incl;
  __syncthreads();
  uint32_t before = 0;
  for (uint32_t w = 0; w < tid / 64; w++) before = S.omax[w] > before ? S.omax[w] : before;
  uint32_t prev = __shfl_up(incl, 1, 64);
  if (lane_id() == 0) prev = 0;
  uint32_t run = prev > before ? prev : before;
  for (uint32_t q = 0; q < PER; q++) {
    const uint32_t v = S.own[tid * PER + q];
    run = v > run ? v : run;
    S.own[tid * PER + q] = (uint16_t)run;
  }
  __syncthreads();
}

// Pieces per work item of the body passes: a workgroup takes runs of
// consecutive pieces, so that finding a piece's tile is a step forward from
// the previous piece's tile rather than a search.
constexpr uint32_t PIECE_RUN = 8;

// Piece p of body pass `which` (0 interpreted, 1 gather): its expanded tile
// and input.  `xt` holds the previous piece's tile (~0 for none); the next two
// tiles are tried before a binary search.  Uniform.
__device__ __forceinline__ void piece_tile(const KArgs& a, uint32_t which, uint64_t p, uint64_t& xt, uint32_t& i) {
  typedef const __attribute__((address_space(4))) unsigned long long c_u64;
  c_u64* xp = (c_u64*)(which ? a.xpg : a.xpb);
  const uint64_t n = a.n_xtiles;
  uint64_t t = ~0ull;
  if (xt != ~0ull) {
    for (uint64_t q = xt; q < n && q <= xt + 2; q++) {
      const uint64_t b = xp[q], e = q + 1 < n ? xp[q + 1] : ~0ull;
      if (p >= b && p < e) { t = q; break; }
    }
  }
  if (t == ~0ull) t = find_xtile(which ? a.xpg : a.xpb, n, p);
  xt = ufirst64(t);
  i = ufirst(a.xin[xt]);
}

// The body pass of interpreted expanded loops: work items are pieces of PIECE
// consecutive iterations of one tile's flattened iteration space; each lane
// runs one iteration (owner thread by binary search in the tile's prefix).
template <uint32_t SK>
__global__ void __launch_bounds__(TILE, 4) eval_body_kernel(KArgs a) {
  __shared__ GenLds S;
  extern __shared__ uint64_t R[];  // [n_regs][TILE]
  __shared__ unsigned long long item_slot;
  const uint32_t tid = threadIdx.x;
  const uint64_t total = a.js->total_pieces[0];
  if (total == 0) return;
  Sched<SK> sc;
  KArgs ar = a;
  ar.chunk = PIECE_RUN;
  sched_init(sc, ar, total);
  if (SK == CKC_SCHED_BLOCKED && sc.cur >= sc.end) return;
  for (uint32_t s = tid; s < MAX_SITES_LDS; s += TILE) S.sites[s] = 0;
  if (tid == 0) { S.acc_checked = 0; S.hangs = 0; S.faults = 0; }
  uint32_t cur = 0xFFFFFFFFu, cur_sites = 0, cur_mode = 0;
  uint32_t cur_L[7] = {0, 0, 0, 0, 0, 0, 0};  // launch dims, then the PREX round
  uint64_t cur_xt = ~0ull, sat = 0, cur_xt_hint = ~0ull;
  Dec dec;
  Lane ln;
  lane_zero_totals(ln);
  for (;;) {
    __syncthreads();
    const uint64_t p = sched_next(sc, &a.js->next_piece[0], &item_slot);
    if (p == ~0ull) break;
    uint64_t xt = cur_xt_hint;
    uint32_t i;
    piece_tile(a, 0, p, xt, i);
    cur_xt_hint = xt;
    c_input& in = ((c_input*)a.inputs)[i];
    if (i != cur) {
      if (cur != 0xFFFFFFFFu) {
        add_lane_totals(S, ln);
        flush_input(S, a, cur, cur_sites);
      }
      sat = 0;
      cur = i;
      cur_sites = ((c_dprog*)in.prog)->n_sites;
      for (int q = 0; q < 6; q++) cur_L[q] = in.launch[q];
      cur_L[6] = in.aux;
      cur_mode = in.mode;
      dec_make(dec, cur_L);
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
    Thr T0;
    T0.t[0] = T0.t[1] = T0.t[2] = T0.b[0] = T0.b[1] = T0.b[2] = 0;
    T0.gtid = 0;
    Ctx C;
    ctx_init(C, a, in, i, T0);
    const uint32_t site_iter = ld_ins(C.I, lpc).s0;
    const uint32_t body_special = P->body_special;
    build_owner_map(S, it0, it1);
    for (uint64_t base = it0; base < it1; base += TILE) {
      const uint64_t g = base + tid;
      const bool ga = g < it1;
      const uint32_t o = ga ? (uint32_t)S.own[g - it0] : 0u;
      const uint64_t l = lane0 + o;
      Thr T;
      if (cur_mode != CKC_FULL) {
        decode_lane(cur_mode, cur_L, cur_L[6], l, T);
      } else if (body_special) {
        decode_full(dec, l, T);
      } else {  // the body reads no thread coordinate
        T.t[0] = T.t[1] = T.t[2] = T.b[0] = T.b[1] = T.b[2] = 0;
        T.gtid = l;
      }
      C.t0 = T.t[0]; C.t1 = T.t[1]; C.t2 = T.t[2]; C.b0 = T.b[0]; C.b1 = T.b[1]; C.b2 = T.b[2];
      C.lane0 = l;
      ln.dis = ga ? 0u : DEAD;
      ln.k0 = ga ? g - S.pref[o] : 0;
      ln.k1 = 0;
      ln.gtid = T.gtid;
      count_site(S, C, sat, site_iter, __ballot(ga));
      run_program<M_BODY>(S, R, C, ln, sat, lpc + 1, endpc);
    }
  }
  if (cur != 0xFFFFFFFFu) {
    add_lane_totals(S, ln);
    flush_input(S, a, cur, cur_sites);
  }
}

// The body pass of gather bodies: as above, but each input's body is first
// reduced to its gather entries, and every lane evaluates the entries of its
// iteration (no instruction dispatch).  The owners' start and step are staged
// in LDS with the tile's prefix, so an iteration costs one memory round trip
// per dependent load of the body.
template <uint32_t SK, bool BIG>
__global__ void __launch_bounds__(TILE, BIG ? 2 : 3) eval_gather_kernel(KArgs a) {
  __shared__ GenLds S;
  extern __shared__ uint64_t R[];  // rows: counter and loaded values per lane; the build uses [n_regs]
  __shared__ unsigned long long item_slot;
  const uint32_t tid = threadIdx.x;
  const uint64_t total = a.js->total_pieces[1];
  if (total == 0) return;
  Sched<SK> sc;
  KArgs ar = a;
  ar.chunk = PIECE_RUN;
  sched_init(sc, ar, total);
  if (SK == CKC_SCHED_BLOCKED && sc.cur >= sc.end) return;
  for (uint32_t s = tid; s < MAX_SITES_LDS; s += TILE) S.sites[s] = 0;
  if (tid == 0) { S.acc_checked = 0; S.hangs = 0; S.faults = 0; }
  if (tid < MAX_GENT) {
    S.vfk[tid] = ~0ull;
    S.vcnt[tid] = 0;
    S.vkinds[tid] = 0;
    S.rmin[tid] = ~0ull;
  }
  uint32_t cur = 0xFFFFFFFFu, cur_sites = 0, built = 0, ok = 0, fast = 0, cur_mode = 0, cont = 0;
  uint32_t cur_L[7] = {0, 0, 0, 0, 0, 0, 0};  // launch dims, then the PREX round
  uint64_t cur_xt = ~0ull, sat = 0, xd = 0;
  uint64_t pb = 0, pe = 0;  // pieces of the current tile
  // the next tile of the same input, loaded while the current one runs:
  // its index, this lane's prefix, its total, piece end, d and contiguity
  uint64_t nx = ~0ull, nx_pref = 0, nx_tot = 0, nx_pe = 0, nx_d = 0, nx_c = 0;
  Lane ln;
  lane_zero_totals(ln);
  for (;;) {
    __syncthreads();
    const uint64_t p = sched_next(sc, &a.js->next_piece[1], &item_slot);
    if (p == ~0ull) break;
    uint64_t xt = cur_xt;
    uint32_t i = cur;
    if (cur_xt == ~0ull || p < pb || p >= pe) {
      const uint64_t npe = ufirst64(nx_pe);
      if (nx != ~0ull && p >= pe && p < npe) {
        xt = nx;
        pb = pe;
        pe = npe;
      } else {
        piece_tile(a, 1, p, xt, i);
        pb = a.xpg[xt];
        pe = xt + 1 < a.n_xtiles ? a.xpg[xt + 1] : ~0ull;
      }
    }
    c_input& in = ((c_input*)a.inputs)[i];
    if (i != cur) {
      if (cur != 0xFFFFFFFFu) {
        add_lane_totals(S, ln);
        flush_input(S, a, cur, cur_sites);
        flush_vio_lds(S, a.recs + ((c_input*)a.inputs)[cur].rec_base);
      }
      sat = 0;
      cur = i;
      built = 0;
      cur_sites = ((c_dprog*)in.prog)->n_sites;
      for (int q = 0; q < 6; q++) cur_L[q] = in.launch[q];
      cur_L[6] = in.aux;
      cur_mode = in.mode;
    }
    const uint64_t lane0 = (xt - in.xt_begin) * TILE;
    const uint64_t* xs = (const uint64_t*)in.xstate;
    const uint64_t xn = in.xn;
    if (xt != cur_xt) {
      // the tile's d and contiguity come from the whole-thread pass; a
      // contiguous tile of a gather body keeps no start and step in memory:
      // start = prefix + d, step 1
      uint64_t pv;
      if (xt == nx) {
        pv = nx_pref;
        xd = ufirst64(nx_d);
        cont = (uint32_t)ufirst64(nx_c);
        if (tid == 0) S.pref[TILE] = ufirst64(nx_tot);
      } else {
        typedef const __attribute__((address_space(4))) unsigned long long c_u64;
        pv = xs[lane0 + tid];
        xd = ((c_u64*)a.xd)[2 * xt];
        cont = (uint32_t)((c_u64*)a.xd)[2 * xt + 1];
        if (tid == 0) S.pref[TILE] = a.xtot[xt];
      }
      S.pref[tid] = pv;
      if (cont) {
        S.xstart[tid] = pv + xd;
        S.xstep[tid] = 1;
      } else {
        S.xstart[tid] = xs[xn + lane0 + tid];
        S.xstep[tid] = xs[2 * xn + lane0 + tid];
      }
      cur_xt = xt;
      if (xt + 1 < in.xt_begin + in.n_xt) {
        nx = xt + 1;
        typedef const __attribute__((address_space(4))) unsigned long long c_u64;
        nx_pref = xs[lane0 + TILE + tid];
        nx_tot = ((c_u64*)a.xtot)[nx];
        nx_pe = nx + 1 < a.n_xtiles ? ((c_u64*)a.xpg)[nx + 1] : ~0ull;
        nx_d = ((c_u64*)a.xd)[2 * nx];
        nx_c = ((c_u64*)a.xd)[2 * nx + 1];
      } else {
        nx = ~0ull;
      }
      __syncthreads();
    }
    const uint64_t it0 = (p - pb) * PIECE;
    const uint64_t tot = S.pref[TILE];
    const uint64_t it1 = it0 + PIECE < tot ? it0 + PIECE : tot;
    c_dprog* P = (c_dprog*)in.prog;
    const uint32_t lpc = (uint32_t)P->expand_pc;
    c_dins* I = (c_dins*)((const uint8_t*)in.prog + P->off_instr);
    const dins Lx = ld_ins(I, lpc);
    Thr T0;
    T0.t[0] = T0.t[1] = T0.t[2] = T0.b[0] = T0.b[1] = T0.b[2] = 0;
    T0.gtid = 0;
    Ctx C;
    ctx_init(C, a, in, i, T0);
    if (!built) {
      // live-ins are uniform over the input: take them from the tile's first
      // thread with iterations (the one thread the rows form stores them for)
      const uint32_t o0 = ufirst(owner_of(S, 0));
      if (tid < 64) build_gather(S, R, C, lpc, Lx.jmp, lane0 + o0);
      __syncthreads();
      built = 1;
      ok = S.gb.ok;
      // all-32-bit bodies with at most two loads take the contiguous form
      // fast: 1 or 2 for bodies of at most one or two loads, 0 otherwise
      fast = S.gb.n >= 1 && S.gb.n <= GREG && Lx.w == 32;
      uint32_t nl = 1;
      for (uint32_t e = 0; e < S.gb.n && e < GREG; e++) {
        const GEnt& E = S.gb.e[e];
        if (E.w != 32 || (E.var != 0xFF && E.var > 2) || E.dst > 2) fast = 0;
        nl = E.dst > nl ? E.dst : nl;
      }
      fast = ufirst(fast ? nl : 0u);
    }
    if (!ok) continue;  // cannot happen for a body the loader accepted
    if (fast && cont) {
      // the rest of this tile's pieces in the workgroup's current range go
      // with this one (no owner map bounds the length)
      const uint64_t lim = pe < sc.end ? pe : sc.end;
      uint64_t iend = it1;
      bool run = false;
      if (lim > p + 1) {
        const uint64_t e1 = (lim - pb) * PIECE;
        iend = e1 < tot ? e1 : tot;
        sc.cur = lim;
      }
      // The tile ends inside the workgroup's range: the following tiles of
      // the input that are contiguous, continue the counter where the one
      // before ends and start inside the range form one run with this one
      // (empty tiles are passed over).  Wavefront 0 reads one tile per lane.
      if (cur_mode == CKC_FULL && pe < sc.end) {
        if (tid < 64) {
          const uint64_t tl = xt + 1 + tid;
          const bool valid = tl < in.xt_begin + in.n_xt;
          uint64_t tt = 0, dd = 0, cc = 0, tb = ~0ull, te = ~0ull;
          if (valid) {
            tt = a.xtot[tl];
            dd = a.xd[2 * tl];
            cc = a.xd[2 * tl + 1];
            tb = a.xpg[tl];
            te = tl + 1 < a.n_xtiles ? a.xpg[tl + 1] : ~0ull;
          }
          uint64_t incl = tt;
          for (int o = 1; o < 64; o <<= 1) {
            const uint64_t u = __shfl_up((unsigned long long)incl, o, 64);
            if ((int)lane_id() >= o) incl += u;
          }
          const uint64_t F = tot + incl - tt;  // the tile's first iteration in the run
          const bool link = valid && tb < sc.end && (tt == 0 || (cc && (uint32_t)dd == (uint32_t)(xd + F)));
          const uint64_t broken = __ballot(!link);
          const uint32_t m = broken ? (uint32_t)__ffsll((unsigned long long)broken) - 1 : 64u;
          if (tid < m) S.rstart[tid + 1] = F;
          if (m != 0 && tid == m - 1) {
            const uint64_t pend = te < sc.end ? te : sc.end;
            const uint64_t span = (pend - tb) * PIECE;
            S.rend = F + (span < tt ? span : tt);
            S.rpend = pend;
          }
          if (tid == 0) {
            S.rn = m;
            S.rstart[0] = 0;
          }
        }
        __syncthreads();
        if (S.rn != 0) {
          iend = S.rend;
          sc.cur = S.rpend;
          run = true;
        }
      }
      if (fast == 1)
        gather_c32<BIG, 1>(S, (uint32_t*)R, C, ln, sat, it0, iend, lane0, cur_mode, cur_L, Lx.s0, (uint32_t)xd, run);
      else
        gather_c32<BIG, 2>(S, (uint32_t*)R, C, ln, sat, it0, iend, lane0, cur_mode, cur_L, Lx.s0, (uint32_t)xd, run);
      if (run) {
        end_run(S, C, xs, lane0, S.gb.n);
        cur_xt = ~0ull;  // the next piece sets its tile up afresh
        nx = ~0ull;
      }
      continue;
    }
    build_owner_map(S, it0, it1);
    if (S.gb.n <= GREG) {
      gather_piece<1>(S, R, C, ln, sat, it0, it1, lane0, cur_mode, cur_L, Lx.s0, Lx.w);
      continue;
    }
    for (uint64_t base = it0; base < it1; base += TILE) {
      const uint64_t g = base + tid;
      const bool ga = g < it1;
      const uint32_t o = ga ? (uint32_t)S.own[g - it0] : 0u;
      const uint64_t l = lane0 + o;
      uint64_t gtid = l;
      if (cur_mode != CKC_FULL) {
        Thr T;
        decode_lane(cur_mode, cur_L, cur_L[6], l, T);
        gtid = T.gtid;
      }
      ln.dis = ga ? 0u : DEAD;
      ln.k0 = ga ? g - S.pref[o] : 0;
      ln.gtid = gtid;
      count_site(S, C, sat, Lx.s0, __ballot(ga));
      const uint64_t ctr = narrow(S.xstart[o] + ln.k0 * S.xstep[o], Lx.w);
      run_gather(S, R, C, ln, sat, ctr);
    }
  }
  if (cur != 0xFFFFFFFFu) {
    add_lane_totals(S, ln);
    flush_input(S, a, cur, cur_sites);
    flush_vio_lds(S, a.recs + ((c_input*)a.inputs)[cur].rec_base);
  }
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
  c_input& in = ((c_input*)a.inputs)[lo_i];
  const dprog* P = (const dprog*)in.prog;
  if (P->pflags & PF_CAPTURE) return;  // filled by the capture pass
  const uint32_t acc = (uint32_t)(r - in.rec_base);
  const uint64_t key = rec->first_key;
  const uint32_t Lsum = in.L1 + in.L2;
  const uint64_t gtid = Lsum >= 64 ? 0 : key >> Lsum;
  const uint64_t i1 = in.L1 ? (key >> in.L2) & ((1ull << in.L1) - 1) : 0;
  const uint64_t i2 = in.L2 ? key & ((1ull << in.L2) - 1) : 0;
  const uint32_t L6[6] = {in.launch[0], in.launch[1], in.launch[2], in.launch[3], in.launch[4], in.launch[5]};
  const uint32_t bs = L6[3] * L6[4] * L6[5];
  Thr T;
  thr_from(L6, gtid / bs, (uint32_t)(gtid % bs), T);
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
  lane_zero_totals(ln);
  uint64_t sat = 0;
  run_program<M_FIX>(S, R, C, ln, sat, 0, C.P->n_instr);
}


}  // namespace ckc
