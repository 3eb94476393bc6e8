// kernels.h — launch interface between the host runtime and kernels.hip.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/ckc.h"
#include "dformat.h"

namespace ckc {

constexpr int TILE = 256;  // lanes per tile = threads per evaluation workgroup
// LDS for the shared-memory instances of one tile's blocks (blockwise programs)
constexpr uint64_t SHARED_LDS_MAX = 48 * 1024;

struct jobstate {
  unsigned long long total_tiles[3];  // tile space of each evaluator (dinput.path)
  unsigned long long next_tile[3];    // dynamic schedule counters
  unsigned long long total_pieces[2];  // work items of the expanded-loop body passes
  unsigned long long next_piece[2];    // [0] interpreted bodies, [1] gather bodies
};

struct KArgs {
  dinput* inputs;
  const int64_t* scalars;   // [n_inputs][MAX_SCALARS]
  uint32_t n_inputs;
  uint32_t force_generic;
  ckc_record* recs;
  uint32_t* counts;         // per (input, site), saturating near 255
  ckc_input_status* status;
  uint8_t* maps;            // [n_inputs][65536] or null
  jobstate* js;
  const uint32_t* order;    // [n_inputs]: tile-space position -> input index
  uint32_t sched;           // ckc_schedule of the evaluator being launched (set per launch)
  uint32_t chunk;           // tiles per work item
  // expanded loops: per expanded tile the trip-count total, the piece count
  // (scanned in place into the first piece), the input; block sums of the scan
  unsigned long long* xtot;
  unsigned long long* xpb;    // pieces of interpreted bodies
  unsigned long long* xpg;    // pieces of gather bodies
  uint32_t* xin;
  unsigned long long* xd;     // [2 per expanded tile]: start - prefix (d), contiguous (1) or not
  unsigned long long* xbsum;  // [2][blocks]
  uint64_t n_xtiles;
  uint32_t max_regs;        // interpreter registers (LDS rows of TILE lanes) of the job's programs
  uint32_t capture;         // this launch of the interpreter is the capture pass
  uint32_t sh_bytes;        // LDS of the tile's shared-memory instances (blockwise programs)
  uint32_t rows_only;       // 1: every input's program takes the rows form (the lean whole-thread
                            // kernel); 2: and every rows form is 32 bits wide (its 32-bit instantiation)
};
// LDS bytes of the interpreter's register file for a job.
// At least 8 rows: the gather evaluation of expanded bodies keeps the counter
// and up to 7 loaded values there.
inline uint32_t regfile_bytes(const KArgs& a) { return (a.max_regs > 8u ? a.max_regs : 8u) * TILE * 8u; }
// Dynamic LDS of the gather pass: the register file, and for the variant with
// large rounds at least 32 rows of TILE 32-bit index values.
inline uint32_t body_lds_bytes(const KArgs& a, uint32_t big) {
  const uint32_t r = regfile_bytes(a);
  return big && r < 32u * TILE * 4u ? 32u * TILE * 4u : r;
}
// LDS bytes of the planning wavefront's symbolic register file.
inline uint32_t plan_lds_bytes(const KArgs& a) { return (a.max_regs > 1u ? a.max_regs : 1u) * 64u * 8u; }

// Workgroups and schedule of each evaluator (index PATH_*).
struct EvalGrid {
  uint32_t n_wg[3];
  uint32_t sched[3];
  uint32_t chunk[3];
  uint32_t n_wg_body;   // workgroups of the body passes of expanded loops (the gather pass: n_wg_gather)
  uint32_t n_wg_gather;
  uint32_t sched_body;  // schedule of the body passes
  uint32_t big_body;    // gather pass with large rounds (inputs of many tiles)
  uint32_t body_kinds;  // body passes with work: bit 0 interpreted bodies, bit 1 gather bodies
  uint32_t no_trace;    // 1: no input can take a trace path (the trace evaluators are not launched)
};

// The PREX sweep (Algorithm 1) runs in windows of rounds.  A window is an
// ordinary job whose inputs are (input, round r) pairs of thread set MODE_PAIR
// with their own records, counters and status; after it, prex_merge folds each
// input's rounds into the input's own results in round order, applying the
// stop test of Algorithm 1 before every round.
struct prex_item {
  uint32_t real;   // index of the input (into PrexArgs.real_in)
  uint32_t vbeg;   // its first round's input in the window's input list
  uint32_t vcnt;   // consecutive rounds of the input in this window
  uint32_t r0;     // round of vbeg
  uint32_t last;   // last round of the whole sweep: ceil(nblocks / 2) - 1
  uint32_t pad;
};
struct PrexArgs {
  const dinput* real_in;
  uint32_t n_real, n_items;
  ckc_record* real_recs;
  uint32_t* real_counts;
  ckc_input_status* real_status;
  uint32_t* stopped;          // per input: 1 once the sweep has stopped
  const prex_item* items;     // [n_items]
  const dinput* vin;          // the window's inputs
  const ckc_record* vrecs;
  const uint32_t* vcounts;
  const ckc_input_status* vstatus;
};
// Clears the inputs' records, counters, status and stop flags.
hipError_t launch_prex_init(const PrexArgs& p, hipStream_t s);
// Folds one window into the inputs' results (one workgroup per item).
hipError_t launch_prex_merge(const PrexArgs& p, hipStream_t s);

// Capture pass of programs whose indices depend on shared memory: the
// interpreter runs their inputs again, and the lane whose key is a record's
// first key writes the record's index and kind.
hipError_t launch_capture(const KArgs& a, const EvalGrid& eg, hipStream_t s);

hipError_t launch_plan(const KArgs& a, hipStream_t s);
hipError_t launch_scan(const KArgs& a, hipStream_t s);
hipError_t launch_eval_trace(const KArgs& a, const EvalGrid& eg, hipStream_t s);
hipError_t launch_eval_trace_lanes(const KArgs& a, const EvalGrid& eg, hipStream_t s);
hipError_t launch_eval_generic(const KArgs& a, const EvalGrid& eg, hipStream_t s);
hipError_t launch_fixup(const KArgs& a, uint64_t n_records, hipStream_t s);
// Body pass of expanded loops: scan of the piece counts, then the pass itself
// (nothing is launched when the job has no expanded tiles).
hipError_t launch_expand(const KArgs& a, const EvalGrid& eg, hipStream_t s);
hipError_t launch_finish(const KArgs& a, hipStream_t s);
// The whole job as one graph: plan -> scan -> the three evaluators (parallel
// branches) -> first-violation replay -> finishing.
hipError_t build_job_graph(hipGraph_t g, const KArgs& a, const EvalGrid& eg, uint64_t n_records);

// A fuzzing campaign on the device: its counters, and the buffers its
// generation kernels use (the children are the inputs of a staged job).
struct FzState {
  uint32_t size, pad;         // corpus entries
  uint64_t execs, novel, crashes, generations;
};
struct FzArgs {
  dinput* in;                 // the job's inputs: one per child
  int64_t* sc;                // the job's scalars [batch][MAX_SCALARS]
  const ckc_record* recs;     // the job's records
  const uint32_t* counts;     // the job's per-site counts
  uint32_t batch, n_scalars, max_stack, max_block, cap, ops;
  uint64_t max_threads, seed, n_elems;
  int32_t* child_data;        // [batch][n_elems]: the children's mutated elements
  uint32_t* c_launch;         // corpus [cap][6]
  int64_t* c_scalars;         // corpus [cap][MAX_SCALARS]
  int32_t* c_data;            // corpus [cap][n_elems]
  uint32_t* c_gen;            // corpus [cap]: generation that added the entry
  uint8_t* virgin;            // [65536]: bucket bits not yet seen
  uint32_t* seen;             // [65536 / 4]: buckets seen by the current generation
  unsigned long long* sigs;   // [n_accesses][4]: least (generation << 32 | child) per kind
  uint32_t* novel;            // [batch]
  uint32_t* pos;              // [batch]: corpus position of an appended child, or ~0
  FzState* st;
};
// Builds the children of generation g from the corpus.
hipError_t launch_fuzz_mutate(const FzArgs& f, uint64_t g, hipStream_t s);
// Classifies the checked children of generation g, updates the virgin map,
// appends novel children to the corpus.
hipError_t launch_fuzz_update(const FzArgs& f, uint64_t g, hipStream_t s);

// Device address of the static scratch array (CKC_NOALLOC_SCRATCH_BYTES) on
// device dev, which must be the current device; looked up once per device.
hipError_t scratch_address(int dev, void** out);

}  // namespace ckc
