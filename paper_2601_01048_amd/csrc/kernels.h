// kernels.h — launch interface between the host runtime and kernels.hip.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/ckc.h"
#include "dformat.h"

namespace ckc {

constexpr int TILE = 256;  // lanes per tile = threads per evaluation workgroup

struct jobstate {
  unsigned long long total_tiles[3];  // tile space of each evaluator (dinput.path)
  unsigned long long next_tile[3];    // dynamic schedule counters
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
};

hipError_t launch_plan(const KArgs& a, hipStream_t s);
hipError_t launch_scan(const KArgs& a, hipStream_t s);
hipError_t launch_eval_trace(const KArgs& a, uint32_t n_wg, hipStream_t s);
hipError_t launch_eval_trace_lanes(const KArgs& a, uint32_t n_wg, hipStream_t s);
hipError_t launch_eval_generic(const KArgs& a, uint32_t n_wg, uint32_t n_regs, hipStream_t s);
hipError_t launch_fixup(const KArgs& a, uint64_t n_records, uint32_t n_regs, hipStream_t s);
hipError_t launch_finish(const KArgs& a, hipStream_t s);

}  // namespace ckc
