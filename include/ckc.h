/*
 * ckc.h — C-ABI of libckc: GPU-native checking of index programs on AMD
 * MI355X (gfx950).
 *
 * The library runs the hot path of coverage-guided kernel fuzzing with an
 * address sanitizer (the method of the paper, Sections 4 and 5): for many
 * inputs of one or more kernels it evaluates every memory-access index of
 * every thread of the launch grid (or of a representative subset of threads,
 * the PREX idea of Section 5.1), checks each index against the allocation it
 * names, records the first violation of every (input, access), and builds a
 * 64 KiB saturating coverage map per input (the AFL++ map of Section 2.1).
 * Programs are given in the index-program IR of ckc_ir.h.
 *
 * Conventions for every entry point:
 *   - the return value is CKC_OK (0), CKC_NOT_READY (1) or a negative error;
 *     no call aborts, and no C++ exception crosses the ABI;
 *   - ckc_last_error() returns a message for the calling thread's last failed
 *     call (valid until that thread's next call);
 *   - a context may be used by one thread at a time;
 *   - "host" pointers are ordinary CPU memory, "device" pointers are HIP
 *     device memory of the context's device.
 */
#ifndef CKC_H
#define CKC_H

#include <stddef.h>
#include <stdint.h>

#include "ckc_ir.h"

#ifdef __cplusplus
extern "C" {
#endif

enum ckc_status_code {
  CKC_OK = 0,
  CKC_NOT_READY = 1,   /* results not yet available (ckc_read_results without CKC_WAIT) */
  CKC_E_INVALID = -1,  /* bad argument, id, size or combination */
  CKC_E_IR = -2,       /* IR bytes malformed or outside the supported limits */
  CKC_E_RANGE = -3,    /* a first-violation key would not fit in 64 bits */
  CKC_E_NOMEM = -4,    /* device or host allocation failed */
  CKC_E_HIP = -5,      /* a HIP runtime call failed */
  CKC_E_BUSY = -6      /* object still referenced by unread jobs */
};

/* thread-set modes (ckc_batch.mode) */
enum ckc_mode {
  CKC_FULL = 0,         /* every thread of the grid (Section 5.1: the fall-back for
                           kernels that are not affine-access); every index of every
                           thread is formed and compared against its bound */
  CKC_REP_CORNERS = 1,  /* the vertices of the (grid x block) coordinate box: the
                           first/last thread of the first/last block of the PREX
                           Theorem (Section 5.1.1), per dimension */
  CKC_REP_BOUNDARY = 2, /* every block with a coordinate first or last along its grid
                           dimension, plus the middle block, all of their threads */
  CKC_REP_PREX = 3,     /* the PREX runtime sweep (Section 5.1.2, Algorithm 1): rounds
                           of block pairs (r, nblocks-1-r), r = 0, 1, ..., all their
                           threads; an input stops before its next round once every
                           ACCESS/LOAD instruction of the program has executed at
                           least once or some access has violated (a single middle
                           block runs once).  ckc_check_batch returns only after
                           every input has stopped (the round decisions need the
                           device's results); a job holds PREX descriptors only */
  CKC_FULL_ENDPOINTS = 4 /* the whole grid, with results identical to CKC_FULL, but
                           programs on the trace path at width 32 are decided by the
                           end-point argument of the Section 5.1.1 Theorem applied to
                           rows of blocks: the block bases of consecutive blocks in a
                           grid row form an arithmetic progression, and a progression
                           spanning less than 2^31 is in bounds exactly when its two
                           end indices are, so most indices are never formed.
                           Report it in inputs/s, not per access */
};

/* ckc_input_status.flags bits */
enum ckc_status_flags {
  /* REP modes: the vertex threads of the (grid x block) coordinate box (the
   * CKC_REP_CORNERS set) all follow one control path (same IF outcomes, same
   * loop trip counts, at most 2^16 loop iterations in all) and no operation
   * that an index, an IF predicate or a loop bound depends on wraps at any of
   * them: no ADD/SUB/MUL/SHL whose exact signed result leaves its width's
   * range, no DIVS of the minimum by -1, no LOOP counter start + k*step
   * outside the range, and no 64-bit value outside the int32 range read at
   * width 32 (an operand of a width-32 operation, a width-32 index or
   * loop bound, SEXT/TRUNC/ZEXT or a width-32 SELECT; ZEXT of a negative
   * value also counts).  Each intermediate of an affine index is then affine
   * over the box in exact integers and extremal at a vertex, which is the
   * condition under which the Section 5.1.1 Theorem makes a representative set
   * flag exactly the (access, kind) pairs of the whole grid for affine,
   * unguarded programs.  Never set in CKC_FULL / CKC_FULL_ENDPOINTS. */
  CKC_ST_VERTEX_EXACT = 1,
  /* The library skipped part of this input's evaluation (an internal
   * inconsistency; never expected): its results are incomplete. */
  CKC_ST_INTERNAL = 0x80000000u
};

/* violation kinds (ckc_record.kinds / first_kind) */
enum ckc_kind { CKC_KIND_OVER = 1, CKC_KIND_UNDER = 2, CKC_KIND_FREED = 4, CKC_KIND_NULL = 8 };

/* program classes (ckc_prog_info.cls), from the load-time analysis */
enum ckc_prog_class {
  CKC_CLS_AFFINE = 1,     /* every access index is affine in the thread and block
                             coordinates with thread-invariant coefficients
                             (Section 5.1.1's affine-access definition) */
  CKC_CLS_GUARDED = 2,    /* some access sits under thread-dependent control flow */
  CKC_CLS_INDIRECT = 4,   /* some index depends on a loaded value */
  CKC_CLS_I64 = 8,        /* some access index has width 64 */
  CKC_CLS_UNIFORM = 16,   /* control flow is thread-invariant and every index is
                             affine: evaluated as a per-input access trace */
  CKC_CLS_EXPANDED = 32,  /* one loop is evaluated one lane per iteration */
  CKC_CLS_GATHER = 64,    /* that loop's body is straight-line with indices affine in
                             the counter or in one loaded value (an indirect gather),
                             evaluated from per-input entries rather than interpreted */
  CKC_CLS_BARRIER = 128   /* some index depends on a value loaded from shared memory (an
                             index-related shared variable of Algorithm 2): BARRIERs are
                             kept and each block runs phase by phase */
};

typedef struct ckc_ctx_s* ckc_ctx;

/* One context per HIP device: the counterpart of the runtime library the
 * paper links every translated program with, whose thread pool runs the
 * kernel's blocks (Section 4).  Creates the context's stream-independent
 * state; no kernel runs.  Errors: CKC_E_INVALID (no such device), CKC_E_HIP. */
int ckc_init(int hip_device, ckc_ctx* out);
/* Waits for outstanding work, frees every program, table and job. */
void ckc_shutdown(ckc_ctx ctx);
/* Message of the calling thread's last failed call ("" if none). */
const char* ckc_last_error(void);

/* ---- programs (Section 5.1.1 affine analysis, Section 5.2 pruning) ------ */
typedef struct ckc_prog_info {
  uint32_t n_accesses, n_sites, n_slots, n_scalars;
  uint32_t max_loop_depth;
  uint32_t cls;            /* ckc_prog_class bits */
  uint32_t n_instr_live;   /* instructions left after removing those that feed no
                              index, guard or loop bound */
  uint32_t n_regs_phys;    /* registers after allocation */
  uint32_t rows_form;      /* 1: the whole-thread part around an expanded gather loop
                              may run in the rows form (affine forms, no instruction
                              dispatch; the plan decides per input); 2: and every entry
                              of that form is 32 bits wide (32-bit evaluation); 0: no */
} ckc_prog_info;

/* Per-access result of the load-time analysis.  coef[] describes the index
 * as sum_d coef[d]*coord[d] + coef[6] over coord = (tid.x, tid.y, tid.z,
 * bid.x, bid.y, bid.z) when the access is affine: each entry is encoded as
 * kind << 32 | value with kind 0 = zero, 1 = the constant `value`, 2 = the
 * uniform IR register `value` (a SPECIAL, SCALAR or CONST result), 3 = a
 * thread-invariant expression. */
typedef struct ckc_access_info {
  uint32_t access_id, slot, log2_elem, width;
  uint32_t affine;        /* 1 if the index is affine in the coordinates */
  uint32_t guarded;       /* 1 if under thread-dependent control flow */
  uint32_t indirect;      /* 1 if the index depends on a loaded value */
  uint32_t loop_depth;
  uint64_t coef[7];
} ckc_access_info;        /* 88 bytes */

/* Host-only analysis of IR bytes (no device needed): validation, pruning of
 * instructions that feed no index (Section 5.2, Algorithm 2), and the
 * affine-access classification of every access (Section 5.1.1: an index is
 * affine when it is a linear function of the thread and block indices with
 * thread-invariant coefficients, the rows of the paper's matrix T).  info and acc (n_accesses entries) may be NULL.
 * Errors: CKC_E_IR with a message naming the offending instruction. */
int ckc_analyze_ir(const void* ir, size_t ir_bytes, ckc_prog_info* info, ckc_access_info* acc,
                   uint32_t acc_capacity);

/* Validates, analyses and lowers the program, and uploads its device form
 * once: the compile-time half of the paper's flow (Section 4: the kernel
 * translator's AXIPrune pass, then the PREX analysis, then the lowering that
 * decides how threads are executed, Section 4.1).  ir: host bytes in the ckc_ir.h layout (copied).  *prog_id receives a
 * nonzero id.  info may be NULL.  Errors: CKC_E_IR, CKC_E_NOMEM, CKC_E_HIP. */
int ckc_load_program(ckc_ctx ctx, const void* ir, size_t ir_bytes, uint32_t* prog_id,
                     ckc_prog_info* info);
/* ckc_load_program with flags: CKC_LOAD_NO_PRUNE keeps every instruction of
 * the program as written (the data math, every BARRIER, every STORE value):
 * the unpruned baseline of the paper's AXIPrune measurement (Section 7.4.2);
 * results are identical, only the work differs.  Such a program always runs
 * on the interpreter.  Errors as ckc_load_program, CKC_E_INVALID for unknown
 * flags. */
enum ckc_load_flags { CKC_LOAD_NO_PRUNE = 1 };
int ckc_load_program_ex(ckc_ctx ctx, const void* ir, size_t ir_bytes, uint32_t flags, uint32_t* prog_id,
                        ckc_prog_info* info);
/* CKC_E_BUSY while an unread job uses the program. */
int ckc_unload_program(ckc_ctx ctx, uint32_t prog_id);

/* ---- allocation tables (the analogue of the heap the paper's translated
 *      kernels run against, Section 4.1) -------------------------------- */
#define CKC_ALLOC_FREED 1u
typedef struct ckc_alloc {
  uint64_t base;        /* logical address; 0 = NULL allocation.  Slots of the
                           shared and local spaces (ckc_ir_space) take addresses
                           within their block's or thread's own window */
  uint64_t size_bytes;  /* bounds; metadata only unless data != NULL */
  const void* data;     /* device pointer to size_bytes bytes; required for slots
                           read by LOAD; borrowed: must stay valid until every job
                           using the table has been read */
  uint32_t flags;       /* CKC_ALLOC_FREED */
  uint32_t redzone;     /* bytes poisoned on each side of the allocation under the
                           tripwire detector (CKC_TRIPWIRE); ignored otherwise */
} ckc_alloc;            /* 32 bytes */

/* Copies n (1..16) host entries into a device-resident table.  Each entry
 * is one buffer of the kernel's global memory with its exact base and size:
 * the base-and-bounds metadata that the exact detectors of Section 7.1 keep
 * (GPUShield, CuCatch, No-Fat), here per allocation slot; the FREED flag is
 * the dangling-pointer case of Section 2.2 (temporal errors, Section 7.2.2).  *table_id
 * receives a nonzero id.  Errors: CKC_E_INVALID, CKC_E_NOMEM. */
int ckc_put_alloc_table(ckc_ctx ctx, const ckc_alloc* entries, uint32_t n, uint32_t* table_id);
/* CKC_E_BUSY while an unread job uses the table. */
int ckc_free_alloc_table(ckc_ctx ctx, uint32_t table_id);

/* ---- checking ----------------------------------------------------------- */
enum ckc_batch_flags {
  CKC_DENSE_MAP = 2,  /* also build the dense 64 KiB maps */
  /* Detector model of the redzone ("tripwire") address sanitizers that the
   * paper contrasts with base-and-bounds checkers (Section 7.1, Table 1;
   * the memory spaces of Section 6.1) instead of exact bounds: an access that
   * is out of its slot's exact bounds is reported only when its slot is NULL,
   * when one of its bytes (base + index * element size, an exact integer)
   * falls in a redzone of an allocation of its own memory space (the
   * `redzone` bytes on each side of a live allocation) or in a freed
   * allocation of that space (its bytes and redzones), or, for a shared or
   * local slot, when it leaves that space's window [0, the largest allocation
   * end plus redzone of the space).  Linear overflows into a redzone are
   * caught; accesses that jump over it into other memory are not.  Reported
   * records carry the exact kind and index; a LOAD out of exact bounds reads 0
   * either way.  Every allocation with a nonzero base must satisfy base >=
   * redzone and base + size_bytes + redzone <= 2^63 (else CKC_E_INVALID).
   * Inputs run on the interpreter path. */
  CKC_TRIPWIRE = 4
};

typedef struct ckc_batch {
  uint32_t prog_id;
  uint32_t n_inputs;
  const uint32_t* launch;    /* host [n_inputs][6]: gx gy gz bx by bz (copied) */
  const int64_t* scalars;    /* host [n_inputs][n_scalars] (copied); NULL if n_scalars = 0 */
  const uint32_t* table_ids; /* host [n_inputs] (copied) */
  uint32_t mode;             /* ckc_mode */
  uint32_t flags;            /* ckc_batch_flags */
  uint32_t loop_cap_log2[2]; /* trip caps 2^k for loops at depth 1 and 2 (k <= 32);
                                0,0 selects the defaults 20, 12 */
} ckc_batch;

/* How the persistent evaluators hand out their work items (runs of `chunk`
 * consecutive 256-lane tiles) to workgroups. */
enum ckc_schedule {
  CKC_SCHED_DEFAULT = 0,  /* BLOCKED for the trace evaluators, DYNAMIC for the interpreter */
  CKC_SCHED_BLOCKED = 1,  /* workgroup g takes one contiguous range of tiles */
  CKC_SCHED_CYCLIC = 2,   /* workgroup g takes items g, g+G, g+2G, ... */
  CKC_SCHED_DYNAMIC = 3,  /* items from an atomic counter */
  CKC_SCHED_LPT = 4       /* DYNAMIC over a tile space that lists the largest inputs first */
};

typedef struct ckc_launch_opts {
  uint32_t schedule;      /* ckc_schedule */
  uint32_t chunk;         /* tiles per work item (1..256); 0 = per-evaluator defaults (1 for
                             the trace evaluators, 4 for the interpreter); the body pass of
                             expanded loops always takes runs of 8 pieces */
  uint32_t wg_per_cu;     /* persistent workgroups per compute unit for every evaluator
                             (1..32); 0 = per-evaluator defaults (8 trace, 2 interpreter) */
  uint32_t force_generic; /* 1: evaluate every program with the general interpreter */
  uint32_t use_graph;     /* 1: run the job's kernels as one HIP graph (the evaluators as
                             parallel branches); per-kernel timing is then unavailable */
  uint32_t pad;
  void* hip_stream;       /* hipStream_t; NULL = the context's own stream */
} ckc_launch_opts;        /* 32 bytes; all zeros = defaults */

/* One fuzzing execution per input, for every input of every descriptor, in
 * one job: the thread set of the chosen mode (Section 5.1, Algorithm 1 for
 * CKC_REP_PREX) runs the program, every ACCESS/LOAD is checked against its
 * allocation as an address sanitizer would (Section 2.1, exact bounds of
 * Section 7.1), and every instrumented site counts into the input's coverage
 * map (Section 2.1, the LLVM-PCGuard mode of Section 7.1).  One planning pass
 * and one persistent evaluation cover all inputs.  Host arrays are copied before
 * the call returns; the work is queued on the stream and the call returns
 * without waiting.  Launch limits: block <= 1024 threads, grid < 2^32 blocks.
 * Errors: CKC_E_INVALID (ids, sizes, missing LOAD data), CKC_E_RANGE (key
 * bits: log2(threads per input) + cap bits of the depths used > 64),
 * CKC_E_NOMEM, CKC_E_HIP. */
int ckc_check_batch(ckc_ctx ctx, const ckc_batch* descs, uint32_t n_descs,
                    const ckc_launch_opts* opts, uint64_t* job);

/* What the address sanitizer reports for one (input, access): a spatial
 * violation (out of bounds below or above, Section 2.2) or a temporal one
 * (NULL or freed allocation), here recorded and continued rather than aborted
 * at, with the first one in sequential thread order. */
typedef struct ckc_record {
  uint64_t first_key;   /* smallest (gtid << (L1+L2) | i1 << L2 | i2) that violated;
                           UINT64_MAX if none */
  int64_t index;        /* index value at first_key */
  uint64_t count;       /* violating executions */
  uint32_t kinds;       /* OR of ckc_kind bits */
  uint32_t first_kind;  /* kind at first_key */
} ckc_record;           /* 32 bytes */

/* Per-input counters.  hang_lanes is the per-thread form of the paper's
 * hang timeout (Section 7.1); arith_faults counts the division-by-zero kernel
 * errors of Section 2.3.2. */
typedef struct ckc_input_status {
  uint64_t lanes;            /* threads executed */
  uint64_t accesses_checked; /* ACCESS and LOAD executions */
  uint64_t hang_lanes;       /* threads stopped by a loop trip cap */
  uint64_t arith_faults;     /* divisions by zero */
  uint32_t flags, pad;
} ckc_input_status;          /* 40 bytes */

enum ckc_read_flags { CKC_WAIT = 1, CKC_DST_DEVICE = 2, CKC_ENQUEUE = 4 };

/* Copies a job's results out and releases the job: the step at which a
 * fuzzer reads the coverage data and the sanitizer's reports after each
 * execution (Section 2.1).  The dense map is AFL's 64 KiB map.  Inputs are numbered in
 * descriptor order.  recs: [sum over inputs of n_accesses]; maps: [inputs][65536]
 * or NULL (requires CKC_DENSE_MAP); st: [inputs] or NULL.  With CKC_DST_DEVICE
 * the three pointers are device pointers (device-to-device copies on the
 * job's stream).  Without CKC_WAIT returns CKC_NOT_READY while the job runs.
 * CKC_ENQUEUE (with CKC_DST_DEVICE only) queues the copies behind the job on
 * its stream and returns at once, CKC_WAIT or not: the destination is valid
 * once that stream (or the device) has been synchronized, and the job's
 * buffers are reused by later jobs only after the copies have completed.
 * The job's programs and tables count as in use until then.
 * Errors: CKC_E_INVALID (unknown job, CKC_ENQUEUE without CKC_DST_DEVICE),
 * CKC_E_HIP. */
int ckc_read_results(ckc_ctx ctx, uint64_t job, ckc_record* recs, uint8_t* maps,
                     ckc_input_status* st, uint32_t flags);

/* Number of inputs and records of a job (for sizing result buffers;
 * records are [inputs][accesses] as in ckc_read_results). */
int ckc_job_sizes(ckc_ctx ctx, uint64_t job, uint64_t* n_inputs, uint64_t* n_records);

/* Device timing of the job's stages in milliseconds (the paper measures
 * throughput as executions per second, Section 7.1; this splits one job's
 * device time) (HIP events on the job's
 * stream; waits for the job): [0] planning (thread sets, traces, tile scan),
 * [1] trace evaluators, [2] interpreter over whole threads, [3] body passes of
 * expanded loops (piece scans, interpreted bodies, gather bodies), [4]
 * finishing (first-violation replay, status, dense maps).  Jobs run as a
 * graph report -1 in all five.  Call before ckc_read_results releases the job. */
int ckc_job_timing(ckc_ctx ctx, uint64_t job, float* ms5);
/* Device time of the whole job (first kernel start to last kernel end), in
 * milliseconds; waits for the job.  Errors: CKC_E_INVALID (unknown job). */
int ckc_job_elapsed(ckc_ctx ctx, uint64_t job, float* ms);

/* ---- checking without allocation ------------------------------------------
 * For callers that cannot allocate device memory: code that runs under HIP
 * graph capture, tight serving loops, and harnesses that forbid hipMalloc. */
#define CKC_NOALLOC_SCRATCH_BYTES (64u << 20) /* static scratch of the library, per device */
#define CKC_NOALLOC_MAX_INPUTS 4096u          /* inputs per call, over all descriptors */

/* The work of ckc_check_batch followed by ckc_read_results with
 * CKC_DST_DEVICE, in one call that allocates nothing: no hipMalloc or
 * hipFree, no pooled job buffer, no event, no graph, no host heap (host
 * staging arrays are reserved by ckc_init).  The job's internal buffers (input
 * descriptors, scalars, per-site counters, access traces, the loop state of
 * expanded loops) are consecutive pieces of one static device array of
 * CKC_NOALLOC_SCRATCH_BYTES, held by every device the library runs on until
 * the process ends; records, maps and status are written straight into the
 * caller's device buffers.  Results are identical to ckc_check_batch's.
 *   recs: device [sum over inputs of n_accesses] records (required);
 *   maps: device [inputs][65536] when some descriptor has CKC_DENSE_MAP, else
 *         NULL;
 *   st:   device [inputs] status (required).
 * The work is queued on opts->hip_stream (NULL: the context's stream) and the
 * call returns without waiting; the outputs are valid once that stream has
 * completed it.  Every call on a device shares that device's scratch, which
 * keeps the last call's contents: calls queued on one stream run in order,
 * but calls that overlap on one device (other streams, other contexts of the
 * same device) race and their results are undefined.  Programs and tables
 * are not marked in use: keep them loaded until the stream has completed.
 * Not available here: CKC_REP_PREX (its sweep reads stop flags back between
 * rounds) and use_graph.
 * Errors: as ckc_check_batch, plus CKC_E_INVALID (more than
 * CKC_NOALLOC_MAX_INPUTS inputs, recs or st NULL, maps NULL with dense maps
 * requested or given without, CKC_REP_PREX, use_graph) and CKC_E_NOMEM when
 * the batch's buffers do not fit in the scratch; nothing is queued then. */
int ckc_check_batch_noalloc(ckc_ctx ctx, const ckc_batch* descs, uint32_t n_descs, const ckc_launch_opts* opts,
                            ckc_record* recs, uint8_t* maps, ckc_input_status* st);

/* ---- closed-loop fuzzing on the device ---------------------------------------
 * The loop the paper's fuzzer runs around every execution (Section 2.1, the
 * AFL++ campaign of Section 7.1): take an input from the corpus, mutate it,
 * execute it under the sanitizer with coverage, keep it when it reaches
 * coverage not seen before, note it when it triggers a memory bug.  Here a
 * generation is a batch of children checked together, and the whole loop
 * stays on the device: corpus, virgin map and crash signatures never leave it
 * between generations.
 *
 * Generation g, child c (both sides of every test compute exactly this):
 *   r(k) = SplitMix64 output (g * batch + c) * 64 + k of the seed, the
 *          counter form mix(seed + (n + 1) * 0x9E3779B97F4A7C15) (Steele,
 *          Lea and Flood, 2014);
 *   the child copies corpus entry r(0) mod |corpus| (corpus as at the start of
 *   the generation) and applies 1 + r(1) mod max_stack mutations, mutation j
 *   drawing u0, u1, u2 = r(2+4j), r(3+4j), r(4+4j): an operator among the
 *   enabled ones (launch, scalar, data, in that order, each only if it has
 *   something to mutate) by u0, a target (launch dimension u1 mod 6, scalar
 *   u1 mod n_scalars, element u1 mod n_elems) and a kind ((u1 >> 8) mod 4) by
 *   u1, a value by u2:
 *     launch: + (1 + u2 mod 8), - (1 + u2 mod 8) (at least 1), 2^(u2 mod 11),
 *             1 + u2 mod 256; void when the dimension would exceed 2^32 - 1,
 *             the child's block max_block, its grid 2^32 - 1 blocks or grid x
 *             block max_threads;
 *     scalar: flip bit u2 mod 64, add (u2 mod 33) - 16, special value
 *             number u2 mod 28, the 64 bits of u2;
 *     data (int32 elements): add (u2 mod 33) - 16, the low 32 bits of special
 *             value number u2 mod 28, the low 32 bits of u2, flip bit u2 mod 32;
 *   (kinds in the order listed, all arithmetic wrapping at the element's
 *   width; the 28 special values in order: 0, 1, -1, 2, 7, 8, 15, 16, 31, 32,
 *   63, 64, 127, 128, 255, 256, 1023, 1024, 4095, 4096, 65535, 65536,
 *   2^31-1, -2^31, 2^32-1, 2^32, -2^63, 2^63-1);
 *   the children are checked as one job (mode, detector and caps of the
 *   campaign); a child is novel when its coverage map, bucketed by hit count
 *   as AFL buckets it (1, 2, 3, 4-7, 8-15, 16-31, 32-127, 128+: one bit each),
 *   shares a bit with the virgin map as at the start of the generation; then
 *   every child's buckets are cleared from the virgin map, novel children
 *   join the corpus in child order while it has room, and every violated
 *   (access, kind) keeps its least (generation << 32 | child). */
enum ckc_mutation_ops { CKC_MUT_LAUNCH = 1, CKC_MUT_SCALAR = 2, CKC_MUT_DATA = 4 };
#define CKC_FUZZ_NO_SLOT 0xFFFFFFFFu

typedef struct ckc_fuzz_config {
  uint32_t prog_id;
  uint32_t table_id;        /* allocation table of the seed input (resident) */
  uint32_t launch[6];       /* seed input: gx gy gz bx by bz */
  int64_t scalars[16];      /* seed input: the program's scalars (the rest ignored) */
  uint32_t mode;            /* CKC_FULL, CKC_REP_CORNERS or CKC_REP_BOUNDARY */
  uint32_t flags;           /* 0 or CKC_TRIPWIRE */
  uint32_t loop_cap_log2[2];/* as in ckc_batch */
  uint32_t batch;           /* children per generation, 1..65536 */
  uint32_t max_stack;       /* mutations per child drawn from 1..max_stack, max_stack 1..15 */
  uint32_t max_block;       /* bound on a child's block, 1..1024 */
  uint32_t corpus_cap;      /* corpus entries kept, 1..2^20 */
  uint64_t max_threads;     /* bound on a child's threads (grid x block) */
  uint32_t data_slot;       /* slot whose data is mutated as int32 elements (each child and
                               corpus entry gets its own copy), or CKC_FUZZ_NO_SLOT */
  uint32_t ops;             /* ckc_mutation_ops bits */
  uint64_t seed;            /* generator seed */
} ckc_fuzz_config;

typedef struct ckc_fuzz_stats {
  uint64_t generations, execs;  /* generations run, children checked */
  uint64_t novel;               /* novel children (kept or not: the corpus may be full) */
  uint64_t crashes;             /* children with a reported violation */
  uint64_t corpus;              /* corpus entries, the seed included */
  uint64_t map_bits;            /* bucket bits cleared from the virgin map */
} ckc_fuzz_stats;

typedef struct ckc_fuzz_s* ckc_fuzz;

/* Creates a campaign whose corpus holds the seed input: validates it like a
 * one-input batch (errors as ckc_check_batch), stages the children's job once
 * (buffers for batch inputs of up to max_threads threads each) and places the
 * corpus, virgin map and signatures in device memory.  The program and table
 * stay in use until ckc_fuzz_destroy.  The campaign runs on the context's
 * stream; while it exists, use the context from one thread.
 * Errors: CKC_E_INVALID (limits, the seed outside the bounds, a data slot
 * without data), CKC_E_RANGE (key bits of max_threads), CKC_E_NOMEM, CKC_E_HIP. */
int ckc_fuzz_create(ckc_ctx ctx, const ckc_fuzz_config* cfg, ckc_fuzz* out);
/* Queues `generations` generations and returns without waiting. */
int ckc_fuzz_run(ckc_fuzz f, uint32_t generations);
/* Waits for the queued generations; the campaign's counters. */
int ckc_fuzz_get_stats(ckc_fuzz f, ckc_fuzz_stats* st);
/* Waits; copies the campaign out to host memory (any pointer may be NULL):
 * launch [corpus_cap][6], scalars [corpus_cap][16], data [corpus_cap][n_elems]
 * (n_elems = size_bytes / 4 of the data slot), gen [corpus_cap] (generation
 * that added each entry; 0 for the seed), virgin [65536], sigs
 * [n_accesses][4] (kinds OVER, UNDER, FREED, NULL in bit order; UINT64_MAX if
 * never).  Entries past the corpus size are unspecified. */
int ckc_fuzz_read(ckc_fuzz f, uint32_t* launch, int64_t* scalars, int32_t* data, uint32_t* gen,
                  uint8_t* virgin, uint64_t* sigs);
/* Waits, frees the campaign and releases its program and table. */
void ckc_fuzz_destroy(ckc_fuzz f);

/* ---- autotuning of the persistent launch ---------------------------------- */
typedef struct ckc_tune_entry {
  ckc_launch_opts opts;   /* candidate (hip_stream as passed in base) */
  float ms;               /* best device time over the repetitions */
  uint32_t pad;
} ckc_tune_entry;         /* 40 bytes */

/* The paper maps blocks to CPU threads with a fixed thread pool
 * (Section 4.1); on the GPU the equivalent choice is how persistent
 * workgroups take tiles.  Times candidate launch options on the batch given
 * (pass a batch other than the one to be measured to keep tuning and
 * measurement apart) and returns the fastest
 * in *best.  Candidates: every schedule (BLOCKED, CYCLIC, DYNAMIC, LPT) x
 * chunk {1, 4, 16} x wg_per_cu {defaults, 2, 4, 8, 16}; `base` supplies
 * force_generic, use_graph and the stream (NULL = defaults).  Each candidate
 * runs `reps` (>= 1) complete jobs whose results are discarded; results do
 * not depend on the options, so any candidate may be used.  log (may be
 * NULL) receives up to log_cap entries in trial order, *n_log their count.
 * Errors: as ckc_check_batch. */
int ckc_autotune(ckc_ctx ctx, const ckc_batch* descs, uint32_t n_descs, const ckc_launch_opts* base,
                 uint32_t reps, ckc_launch_opts* best, ckc_tune_entry* log, uint32_t log_cap,
                 uint32_t* n_log);

/* ---- serving: a request loop with continuous batching ---------------------
 * The paper's fuzzer runs one execution after another as a child process
 * (Section 2.1) against a service that processes untrusted inputs
 * (Section 3); here executions arrive as independent check jobs.
 * A server owns a worker thread that admits submitted check jobs in arrival
 * order while their device working set fits under a cap, packs the admitted
 * jobs into one batched check per free stream (jobs that arrive while others
 * run join the next batch on the next free stream, so batches overlap on the
 * device), and copies each batch's results to host memory as it completes.
 * While a server exists, its context must not be used by any other thread
 * except through the ckc_server_* calls; load programs and put tables first. */
typedef struct ckc_server_s* ckc_server;

typedef struct ckc_server_config {
  uint32_t n_streams;       /* concurrent batches (1..16); 0 = 4 */
  uint32_t max_batch_jobs;  /* jobs per batch (1..65536); 0 = 1024 */
  uint64_t hbm_cap_bytes;   /* device working set of admitted, unfinished jobs; 0 = 64 GB */
  ckc_launch_opts opts;     /* launch options of every batch (hip_stream ignored) */
} ckc_server_config;

typedef struct ckc_job_stats {
  uint64_t t_arrival_ns;    /* CLOCK_MONOTONIC times: arrival (as submitted), */
  uint64_t t_admit_ns;      /* admission into a batch (its launch), */
  uint64_t t_done_ns;       /* results copied to host memory (readable) */
  uint64_t ws_bytes;        /* working-set estimate used for admission */
  uint32_t batch_jobs;      /* jobs in the batch that ran this one */
  int32_t status;           /* CKC_OK or the error that ended the job */
} ckc_job_stats;            /* 40 bytes */

typedef struct ckc_server_stats {
  uint64_t submitted, completed, rejected, batches;
  uint64_t max_inflight_bytes;  /* largest admitted working set at any time */
  uint64_t max_inflight_jobs;
} ckc_server_stats;             /* 48 bytes */

/* Starts a server on ctx.  Errors: CKC_E_INVALID (limits), CKC_E_HIP. */
int ckc_server_create(ckc_ctx ctx, const ckc_server_config* cfg, ckc_server* out);
/* Drains every submitted job, stops the worker, frees the server (unread
 * results are dropped). */
void ckc_server_destroy(ckc_server srv);
/* Queues one job: the inputs of one descriptor (host arrays copied before
 * return; CKC_DENSE_MAP in desc->flags asks for maps).  arrival_ns: the
 * job's arrival on CLOCK_MONOTONIC (0 = now).  The descriptor is validated
 * here (errors as ckc_check_batch).  A job whose working set alone exceeds
 * the cap is accepted and ends with CKC_E_NOMEM.  Thread-safe. */
int ckc_server_submit(ckc_server srv, const ckc_batch* desc, uint64_t arrival_ns, uint64_t* ticket);
/* Results of a job, then the job is forgotten.  recs: [n_inputs][n_accesses],
 * maps: [n_inputs][65536] or NULL (requires CKC_DENSE_MAP), st: [n_inputs] or
 * NULL, stats: may be NULL; all host pointers.  Without CKC_WAIT returns
 * CKC_NOT_READY while the job is unfinished.  Returns the job's status
 * (CKC_OK, or e.g. CKC_E_NOMEM for a job above the cap).  Thread-safe. */
int ckc_server_result(ckc_server srv, uint64_t ticket, ckc_record* recs, uint8_t* maps, ckc_input_status* st,
                      ckc_job_stats* stats, uint32_t flags);
/* Counters since creation.  Thread-safe. */
int ckc_server_get_stats(ckc_server srv, ckc_server_stats* out);

#ifdef __cplusplus
}
#endif
#endif /* CKC_H */
