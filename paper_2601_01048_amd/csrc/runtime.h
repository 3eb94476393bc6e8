// runtime.h — internal state of libckc's host runtime (contexts, programs,
// tables, jobs), shared by the C-ABI implementation and the request server.
#pragma once
#include <hip/hip_runtime.h>

#include <map>
#include <string>
#include <utility>
#include <vector>

#include "../../include/ckc.h"
#include "dformat.h"
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
}  // namespace rt
}  // namespace ckc
