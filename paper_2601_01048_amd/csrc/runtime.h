// runtime.h — internal state of libckc's host runtime (contexts, programs,
// tables, jobs), shared by the C-ABI implementation and the request server.
#pragma once
#include <hip/hip_runtime.h>

#include <algorithm>
#include <map>
#include <string>
#include <utility>
#include <vector>

#include "../../include/ckc.h"
#include "dformat.h"
#include "kernels.h"
#include "loader.h"

namespace ckc {
namespace rt {

constexpr int NEV = 6;  // plan | trace evaluators | interpreter | body passes | finishing

struct Program {
  void* dblob = nullptr;
  Loaded L;
  int busy = 0;
};

struct Table {
  void* dptr = nullptr;
  std::vector<ckc_alloc> host;
  int busy = 0;
};

struct Job {
  hipStream_t stream = nullptr;
  std::vector<std::pair<size_t, void*>> bufs;  // (bytes, device pointer)
  dinput* d_inputs = nullptr;
  ckc_record* d_recs = nullptr;
  uint32_t* d_counts = nullptr;
  ckc_input_status* d_status = nullptr;
  uint8_t* d_maps = nullptr;
  uint64_t n_inputs = 0, n_records = 0;
  std::vector<uint32_t> progs, tables;
  hipEvent_t ev[NEV] = {};  // job start, then the end of each timed stage
  bool dense = false;
  bool graph = false;  // ran as one graph: only the first and last events are meaningful
};

// Inputs of one launch sequence (a job, or one window of a PREX sweep) staged
// on the host: their descriptors with buffer offsets, scalars, work estimates,
// the tile-space order, and the sizes of the device buffers they need.
struct Stage {
  std::vector<dinput> hin;
  std::vector<int64_t> hsc;
  std::vector<uint64_t> est;     // estimated work per input (LPT order)
  std::vector<uint32_t> order;   // tile-space position -> input (filled when uploaded)
  uint64_t n_xtiles = 0, xstate_bytes = 0, n_xin = 0;  // expanded loops: tiles, bytes, inputs
  uint32_t max_regs = 1;                               // interpreter register file rows
  uint64_t gen_tiles = 0;  // interpreter tiles (estimate from the launch shapes)
  uint64_t n_records = 0, n_counts = 0, trace_bytes = 0;
  uint32_t sh_bytes = 0;  // LDS of the shared-memory instances of a tile (blockwise programs)
  bool capture = false;   // some input needs the capture pass
  bool all_rows = true;   // every input's program takes the rows form (PF_ROWS, exact bounds)
  bool all_rows32 = true;  // ... and every rows form is 32 bits wide (PF_ROWS32)
  uint32_t body_kinds = 0;  // expanded loops: bit 0 some interpreted body, bit 1 some gather body
  bool any_uniform = false;  // some input's program may take a trace path (uniform, not forced generic)

  // Notes an input of a blockwise program (PF_BLOCKWISE): each tile holds
  // TILE / bs of its blocks, each with one instance of every shared slot (a
  // 32-bit current word and a 64-bit phase-write word per element).
  void note_blockwise(const dprog* h, const ckc_alloc* tab, uint32_t n_tab, const uint32_t* L) {
    if (!(h->pflags & PF_BLOCKWISE)) return;
    const uint64_t bs = (uint64_t)L[3] * L[4] * L[5];
    uint64_t words = 0;
    for (uint32_t s = 0; s < h->n_slots && s < n_tab; s++)
      if (((h->slot_spaces >> (2 * s)) & 3u) == CKC_SPACE_SHARED && tab[s].base != 0) words += tab[s].size_bytes / 4;
    const uint64_t need = bs ? (TILE / bs) * words * 12 : 0;
    if (need > sh_bytes) sh_bytes = (uint32_t)need;
    capture |= (h->pflags & PF_CAPTURE) != 0;
  }

  // Room for n inputs, so that staging up to n allocates no host memory.
  void reserve(size_t n) {
    hin.reserve(n);
    hsc.reserve(n * MAX_SCALARS);
    est.reserve(n);
    order.reserve(n);
  }
  // Empties the stage and keeps the reserved room.
  void clear() {
    hin.clear();
    hsc.clear();
    est.clear();
    order.clear();
    n_xtiles = xstate_bytes = n_xin = 0;
    max_regs = 1;
    gen_tiles = 0;
    n_records = n_counts = trace_bytes = 0;
    sh_bytes = 0;
    capture = false;
    all_rows = true;
    all_rows32 = true;
    body_kinds = 0;
    any_uniform = false;
  }

  // d: prog, table, launch, mode, aux, L1, L2 and caps set by the caller;
  // lanes_max: most lanes of its thread set; sc: the program's scalars.
  void add(const dprog* h, dinput d, const int64_t* sc, uint64_t lanes_max, bool force_generic) {
    max_regs = std::max(max_regs, h->n_regs);
    d.rec_base = n_records;
    d.cnt_base = n_counts;
    n_records += h->n_accesses;
    n_counts += h->n_sites;
    const bool uniform = (h->cls & CKC_CLS_UNIFORM) && !force_generic;
    any_uniform |= uniform;
    if (uniform) {
      d.trace = trace_bytes + 1;  // offset + 1 for now; rebased after allocation
      trace_bytes += ckc::trace_bytes(h->trace_cap);
    } else if ((h->pflags & PF_ROWS) && !d.detector && lanes_max > 0) {
      d.trace = trace_bytes + 1;  // the input's rows form
      trace_bytes += sizeof(drows);
    }
    if (h->expand_pc >= 0 && !uniform && lanes_max > 0) {
      // expanded loop: thread-state arrays over at most lanes_max lanes
      const uint64_t n_xt = (lanes_max + TILE - 1) / TILE;
      d.xstate = xstate_bytes + 1;  // rebased after allocation
      d.xt_begin = n_xtiles;
      d.xn = n_xt * TILE;
      d.n_xt = n_xt;
      n_xtiles += n_xt;
      n_xin++;
      xstate_bytes += d.xn * 8 * (3 + (uint64_t)h->n_livein);
      body_kinds |= h->body_gather && !d.detector ? 2u : 1u;
    }
    if (!(h->pflags & PF_ROWS) || d.detector) all_rows = false;
    if (!(h->pflags & PF_ROWS32) || d.detector) all_rows32 = false;
    hin.push_back(d);
    est.push_back(lanes_max * (1 + h->n_accesses));
    if (!uniform) gen_tiles += (lanes_max + TILE - 1) / TILE;
    for (uint32_t s = 0; s < MAX_SCALARS; s++) hsc.push_back(s < h->n_scalars ? sc[s] : 0);
  }
};

}  // namespace rt
}  // namespace ckc

struct ckc_ctx_s {
  int dev = 0;
  hipStream_t stream = nullptr;
  uint32_t next_prog = 1, next_table = 1;
  uint64_t next_job = 1;
  std::map<uint32_t, ckc::rt::Program> progs;
  std::map<uint32_t, ckc::rt::Table> tables;
  std::map<uint64_t, ckc::rt::Job> jobs;
  int n_cu = 256;
  // device buffers of finished jobs, reused by later jobs of similar size
  std::multimap<size_t, void*> pool;
  size_t pool_bytes = 0;
  // instantiated job graphs keyed by their launch parameters (kernel
  // arguments hold the job's buffers, so a key is never shared by two
  // unread jobs)
  std::map<std::string, hipGraphExec_t> graphs;
  // jobs read with CKC_ENQUEUE whose copies may still run: released (buffers
  // back to the pool) once their event has completed
  std::vector<std::pair<hipEvent_t, ckc::rt::Job>> retiring;
  // ckc_check_batch_noalloc: the device address of the library's static
  // scratch array on this context's device (looked up once per device), and
  // host staging arrays reserved at creation for CKC_NOALLOC_MAX_INPUTS inputs
  void* scratch = nullptr;
  ckc::rt::Stage na_stage;
};


namespace ckc {
namespace rt {
// Sets the calling thread's error message; returns code.
int fail(int code, const std::string& msg);
// Checks descriptor k of a batch against the context (ids, arrays, modes,
// caps, launch limits, LOAD data); on success *ws_bytes (may be NULL) is the
// device working set of its inputs: the job's own buffers plus the bytes of
// every allocation its program reads with LOAD.
int validate_desc(ckc_ctx c, const ckc_batch& B, uint32_t k, bool force_generic, uint64_t* ws_bytes);
// Completion event of an unread job (nullptr if unknown).
hipEvent_t job_done_event(ckc_ctx c, uint64_t job);
// Device buffers of a staged input list (default launch options), in J.
int stage_new_job(ckc_ctx c, Job& J, Stage& S, bool dense, KArgs& a, EvalGrid& eg);
// The job input of input i of descriptor B (program, table, launch, caps).
dinput make_input(const Program& P, const Table& T, const ckc_batch& B, uint32_t i);
// Planning and every evaluator of a staged job, queued on s.
hipError_t run_evaluation(const KArgs& a, const EvalGrid& eg, hipStream_t s);
// Returns a job's buffers to the context's pool.
void release_job(ckc_ctx c, Job& J);
// Bits needed for the values 0..n-1.
unsigned index_bits(uint64_t n);
}  // namespace rt
}  // namespace ckc
