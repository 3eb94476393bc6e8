// dformat.h — the lowered (device) form of a loaded index program and the
// per-job descriptors the evaluation kernels read.  Shared by the host runtime
// and the HIP kernels of libckc; plain C layout, no HIP types.
#pragma once
#include <stdint.h>

namespace ckc {

constexpr int NREG = 32;          // physical registers per lane (64-bit each)
constexpr int MAX_SLOTS = 16;
constexpr int MAX_CLASSES = 4;    // distinct coefficient vectors in a trace
constexpr int MAX_LIVEIN = 6;     // registers carried into an expanded loop body
constexpr int MAX_SITES_LDS = 1024; // sites counted in LDS by the interpreter
constexpr uint32_t NOSITE = 0xFFFFu;
constexpr uint32_t DEAD = 0x40000000u;  // "disabled depth" of a stopped lane

// Lowered instruction (16 bytes).  Register fields are physical registers.
struct dins {
  uint8_t op;     // IR opcode (ckc_ir_op numbering)
  uint8_t w;      // 32 / 64
  uint8_t dst, a;
  uint8_t b, c;
  uint8_t slot;   // ACCESS/LOAD: slot
  uint8_t fl;     // ACCESS/LOAD: log2_elem; IF/LOOP: DI_* flags
  uint16_t s0, s1;
  uint16_t x;     // CONST: const index; SCALAR: scalar; SPECIAL: source;
                  // ACCESS/LOAD: access id; LOOP: depth (0/1)
  uint16_t jmp;   // IF: ELSE or ENDIF; ELSE: ENDIF; LOOP: ENDLOOP; ENDLOOP: LOOP
};
static_assert(sizeof(dins) == 16, "dins layout");

// Program flags (dprog.pflags).
enum : uint8_t {
  PF_BLOCKWISE = 1,  // blocks run together: BARRIERs executed, shared memory read back
  PF_CAPTURE = 2,    // indices depend on shared memory: the first-violation index and
                     // kind come from a second evaluation pass (no one-thread replay)
  PF_ROWS = 4,       // the whole-thread part around an expanded gather loop may run
                     // in the rows form (no instruction dispatch; decided per input)
  PF_ROWS32 = 8      // PF_ROWS, and every entry of that form is 32 bits wide (decided,
                     // like PF_ROWS, from the kinds and widths alone)
};

enum : uint8_t {
  DI_NOSKIP = 1,    // IF/LOOP: never skip the region (holds the expanded loop)
  DI_EXPAND = 2,    // LOOP: evaluated one lane per iteration
  DI_HASELSE = 4,   // IF: jmp points at an ELSE
  DI_SLICE = 0x80   // value op that an index, IF predicate or loop bound depends on
};

// Per-access facts used by the fix-up pass.
struct daccess {
  uint16_t pc;        // instruction index
  uint16_t depth;     // enclosing loops
  int16_t loop_pc[2]; // pcs of the enclosing LOOPs, outermost first (-1 if none)
};

// Program blob header; followed in memory by dins[n_instr], int64 consts,
// daccess[n_accesses], uint16 site_ids[n_sites] (each region 16-byte aligned).
struct dprog {
  uint32_t n_instr, n_consts, n_accesses, n_sites;
  uint32_t n_slots, n_scalars, max_depth, cls;
  uint32_t n_regs;
  int32_t expand_pc;          // LOOP lowered with DI_EXPAND, or -1
  uint32_t n_livein;
  uint32_t trace_cap;         // entries reserved per input for the trace path (0 = none)
  uint8_t livein[MAX_LIVEIN]; // physical registers read by the expanded body
  uint8_t pad[2];
  // flags the kernels test per work item are whole dwords (scalar loads)
  uint32_t pflags;            // PF_* bits
  uint32_t body_special;      // the expanded body reads tid or bid
  uint32_t off_instr, off_consts, off_access, off_sites;  // byte offsets from the header
  uint32_t total_bytes;
  uint32_t body_gather;       // the expanded body is evaluated as a gather (entries)
  uint32_t n_map_sites;       // sites 0..n_map_sites-1 have a coverage-map position
                              // (site_ids); sites n_map_sites..n_sites-1 are internal:
                              // one per ACCESS/LOAD written without a site, so that
                              // every access instruction's execution is counted
  uint32_t slot_spaces;       // memory space of slot k in bits 2k..2k+1 (ckc_ir_space)
};

// One input of a job (the global input list concatenates the descriptors).
struct dinput {
  uint64_t prog;          // device address of the dprog blob
  uint64_t table;         // device address of the ckc_alloc[] table
  uint64_t lanes;         // threads in the thread set
  uint64_t tile_begin[3]; // first tile in each evaluator's tile space (see path)
  uint64_t rec_base;      // first record of this input
  uint64_t cnt_base;      // first site counter of this input
  uint64_t trace;         // device address of this input's trace (0 = none)
  uint32_t launch[6];
  uint32_t mode;
  uint32_t L1, L2;        // key bits of depth-1 / depth-2 iteration ordinals
  uint32_t cap_log2[2];
  uint32_t path;          // evaluator, set by planning: PATH_BLOCKS, PATH_GENERIC, PATH_LANES
  uint32_t n_tiles[3];
  uint32_t aux;           // mode CKC_FULL: 1 = decide row progressions by their end indices
                          // (CKC_FULL_ENDPOINTS); mode MODE_PAIR: the round r
  // expanded loop (interpreter path): per-thread state arrays and this
  // input's range of expanded tiles
  uint64_t xstate;        // device address of xn x (3 + n_livein) uint64: trip-count
                          // prefix within the tile, start, step, live-ins (0 = none)
  uint64_t xt_begin;      // first expanded tile of this input
  uint64_t xn;            // entries per state array (tiles x TILE, >= lanes)
  uint64_t n_xt;          // expanded tiles reserved for this input
  uint32_t detector;      // 0 exact bounds, 1 the tripwire model (CKC_TRIPWIRE)
  uint32_t pad2;
};
static_assert(sizeof(dinput) == 176, "dinput layout");
// Internal thread-set mode of one round of the PREX sweep (Algorithm 1): the
// blocks r and nblocks-1-r (one block when they coincide), all their threads,
// in block order.  Never seen at the C-ABI.
constexpr uint32_t MODE_PAIR = 8;

// Evaluators of an input: the trace evaluator in block-major wavefront jobs,
// the general interpreter, or the trace evaluator over lane tiles.
enum : uint32_t { PATH_BLOCKS = 0, PATH_GENERIC = 1, PATH_LANES = 2 };

// Rows form of the whole-thread part of a program (PF_ROWS): per input, the
// plan kernel reduces every value outside the expanded loop's body to an
// affine form over the thread coordinates, or over one loaded value (the
// symbolic walk), and the whole-thread pass runs a short list of entries with
// no instruction dispatch.  A form: off + sum c[d] * coord[d] (var RV_COORD;
// the coefficient vector is one of the input's classes, whose per-lane sums
// are formed once per tile), off + c[0] * X[var] (var 1..RV_MAXLOAD: the value
// of the var-th LOAD), or off (RV_UNI); it is evaluated modulo 2^w at its
// entry's width w.
constexpr uint32_t RV_UNI = 0xFF, RV_COORD = 0xFE, RV_PRED = 0xFD, RV_MAXLOAD = 4;
constexpr uint32_t MAX_RENT = 16, MAX_RCLS = 4, RCLS_NONE = 0xFF;
// Every field of the rows form is at least 32 bits wide: the kernels read
// them as uniform values through scalar loads, which move whole dwords
// (narrower fields would be read by vector loads, each a memory round trip).
struct RForm {
  int64_t off;
  int64_t c[6];
  uint32_t var, cls;  // cls: coordinate class of a RV_COORD form (RCLS_NONE: evaluate c directly)
};
enum : uint32_t { RE_GUARD = 0, RE_ENDG = 1, RE_ACCESS = 2, RE_LOAD = 3, RE_LOOP = 4 };
struct REnt {
  RForm a, b;           // GUARD: the compared forms; ACCESS/LOAD: a = index; LOOP: start, end
  uint64_t step;        // LOOP: the (uniform) step
  uint32_t acc;         // ACCESS/LOAD: access id
  uint32_t s0, s1;      // sites: access / IF taken, IF not taken / loop exit
  uint32_t kind, w, op; // op: GUARD comparison opcode
  uint32_t slot, lg, dst, pad;
};
static_assert(sizeof(RForm) == 64 && sizeof(REnt) % 16 == 0, "rows form layout");
// One input's rows form (in the input's `trace` buffer, which programs with
// an expanded loop never use for a trace).
struct drows {
  REnt e[MAX_RENT];
  int64_t cc[MAX_RCLS][6];      // coefficient vectors of the coordinate classes
  uint64_t livein[MAX_LIVEIN];  // the loop's live-ins (uniform)
  uint32_t n, ok, ncls;
  uint32_t all32;  // every entry is 32 bits wide: the rows kernel evaluates in 32-bit arithmetic
};
static_assert(sizeof(drows) % 16 == 0, "rows form alignment");

constexpr int MAX_SCALARS = 16;
constexpr uint32_t LPB = 16;  // blocks per group of the block-major trace path
// groups per wavefront job of the block-major trace path: the whole grid
// (jobs of many groups amortize the job's set-up), and a thread set of
// boundary blocks (fewer groups per input: more jobs to spread)
constexpr uint32_t NGJ_FULL = 16, NGJ_SET = 4;

// Trace of a uniform-control program for one input: every thread performs the
// same access sequence; each access index is base[class](thread) + off.
struct dtrace_entry {
  int64_t off;          // constant part (wrapped at the access width)
  uint64_t keylo;       // i1 << L2 | i2 of this dynamic access
  uint64_t bound;       // element count, clamped to 2^63 (2^31 for width 32)
  uint32_t acc;         // access id
  uint8_t cls;          // coefficient class
  uint8_t w;            // 32 / 64
  uint8_t dead_kind;    // NULL/FREED kind when the slot is dead, else 0
  uint8_t pad;
};
static_assert(sizeof(dtrace_entry) == 32, "trace entry layout");

// Block-major parameters of an input on the trace path PATH_BLOCKS, formed by
// the plan kernel once per input; the evaluator reloads them with scalar loads
// where it uses them.  Divisors come as multiply-shift pairs (m, s).
struct dblk {
  uint32_t L[6];        // gx gy gz bx by bz
  uint32_t mode, bs, gxy, bxy, nsb, ngroups, spb, ne;
  uint32_t any_dead, w, Lsum, n_acc;
  uint32_t m_gx, s_gx, m_gxy, s_gxy, m_bx, s_bx, m_bxy, s_bxy, m_spb, s_spb, ngj;
  uint32_t proof;       // whole grid decided by the end indices of row progressions
  uint32_t pad[2];
  int64_t k[6];         // coefficients of the one class: tid.xyz, bid.xyz
  uint64_t d1, dy, dz;  // block-part steps: next x, x wrap, x and y wrap
  uint64_t rec;         // the input's records
};
static_assert(sizeof(dblk) % 16 == 0, "block-major parameters alignment");

struct dtrace_head {
  uint32_t n_entries;
  uint32_t n_classes;
  uint32_t overflow;    // 1 if the trace did not fit (input falls back)
  uint32_t hang;        // 1 if every thread stops at the end of the trace
  int64_t coef[MAX_CLASSES][6];  // per class: tid.xyz, bid.xyz coefficients
  uint8_t cls_w[MAX_CLASSES];
  uint32_t any_dead;    // some entry names a NULL or FREED slot
  uint32_t cap8;        // entry capacity rounded up to a multiple of 8
  uint32_t pad;
  dblk blk;             // set when the input takes the block-major path
};
static_assert(sizeof(dtrace_head) % 16 == 0, "trace head alignment");
// Followed by three arrays of cap8 entries each:
//   int64 hot64[cap8][2]   (offset, bound) for width-64 checks
//   uint32 hot32[cap8][2]  (offset, bound) low halves for width-32 checks
//   dtrace_entry entries[cap8]
constexpr uint64_t trace_bytes(uint32_t cap) {
  return sizeof(dtrace_head) + (uint64_t)((cap + 7u) & ~7u) * (16 + 8 + sizeof(dtrace_entry));
}

}  // namespace ckc
