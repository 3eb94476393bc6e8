// kernels.hip — device side of libckc for gfx950 (MI355X, CDNA4): the one
// translation unit that holds every kernel (dev_*.h) and their host-callable
// launchers.
//
// One lane per (input, thread of the thread set).  Kernels of a job:
//   plan       one wavefront per input: thread-set size, and for programs whose
//              control flow is thread-invariant the per-input access trace
//              (affine forms of every index, evaluated once per input);
//   scan       tile offsets of the three evaluators over the inputs;
//   eval_trace, eval_trace_lanes
//              persistent: every index formed with one add of the thread's
//              base and the access offset, checked 16 at a time by an
//              unsigned maximum and one compare (block-major wavefront jobs,
//              or lane tiles); the end-point mode instead decides the blocks
//              a job has in one grid row by the two end indices of the row;
//   eval_generic
//              persistent: a wavefront-uniform interpreter of the lowered
//              bytecode, one lane per thread; the program's expandable loop is
//              only recorded (trip counts, start, step, live-ins per thread);
//   xscan_*    prefix of the expanded loops' work pieces;
//   eval_body  persistent: one lane per iteration of the expanded loops;
//   fixup      one wavefront per violated record: replays the winning thread to
//              fill the index and kind at the first key;
//   finish     per input: coverage counts -> saturating dense map, status.
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
#include <mutex>

#include "dev_common.h"
#include "dev_plan.h"
#include "dev_trace.h"
#include "dev_interp.h"
#include "dev_fuzz.h"

// Buffers of ckc_check_batch_noalloc: one static array per device, held until
// the process ends.  Host code never passes `scratch` itself to a kernel (on
// the host it names a stand-in, not device memory): it uses the address that
// scratch_address looked up for the device.
static __device__ __align__(256) uint8_t scratch[CKC_NOALLOC_SCRATCH_BYTES];

namespace ckc {

namespace {
constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[MAX_DEVICES];
}  // namespace

hipError_t scratch_address(int dev, void** out) {
  if (dev < 0 || dev >= MAX_DEVICES) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return hipSuccess;
}

// ---------------------------------------------------------------------------
// host-callable launchers
// ---------------------------------------------------------------------------
hipError_t launch_prex_init(const PrexArgs& p, hipStream_t s) {
  if (p.n_real == 0) return hipSuccess;
  hipLaunchKernelGGL(prex_init_kernel, dim3(p.n_real), dim3(64), 0, s, p);
  return hipGetLastError();
}
hipError_t launch_prex_merge(const PrexArgs& p, hipStream_t s) {
  if (p.n_items == 0) return hipSuccess;
  hipLaunchKernelGGL(prex_merge_kernel, dim3(p.n_items), dim3(256), 0, s, p);
  return hipGetLastError();
}
hipError_t launch_plan(const KArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(plan_kernel, dim3(a.n_inputs), dim3(64), plan_lds_bytes(a), s, a);
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
  k.chunk = eg.chunk[path];
  return k;
}
// Kernel of evaluator `path` compiled for schedule `sk` (the whole-thread
// pass: the rows-form kernel when `rows` is 1, its 32-bit instantiation when 2).
void* eval_fn(uint32_t path, uint32_t sk, uint32_t rows = 0) {
  const uint32_t s = sched_impl(sk);
  if (path == PATH_BLOCKS)
    return s == CKC_SCHED_BLOCKED ? (void*)eval_trace_kernel<CKC_SCHED_BLOCKED>
         : s == CKC_SCHED_CYCLIC  ? (void*)eval_trace_kernel<CKC_SCHED_CYCLIC>
                                  : (void*)eval_trace_kernel<CKC_SCHED_DYNAMIC>;
  if (path == PATH_LANES)
    return s == CKC_SCHED_BLOCKED ? (void*)eval_trace_lanes_kernel<CKC_SCHED_BLOCKED>
         : s == CKC_SCHED_CYCLIC  ? (void*)eval_trace_lanes_kernel<CKC_SCHED_CYCLIC>
                                  : (void*)eval_trace_lanes_kernel<CKC_SCHED_DYNAMIC>;
  if (rows == 2)
    return s == CKC_SCHED_BLOCKED ? (void*)eval_rows_kernel<CKC_SCHED_BLOCKED, true>
         : s == CKC_SCHED_CYCLIC  ? (void*)eval_rows_kernel<CKC_SCHED_CYCLIC, true>
                                  : (void*)eval_rows_kernel<CKC_SCHED_DYNAMIC, true>;
  if (rows)
    return s == CKC_SCHED_BLOCKED ? (void*)eval_rows_kernel<CKC_SCHED_BLOCKED, false>
         : s == CKC_SCHED_CYCLIC  ? (void*)eval_rows_kernel<CKC_SCHED_CYCLIC, false>
                                  : (void*)eval_rows_kernel<CKC_SCHED_DYNAMIC, false>;
  return s == CKC_SCHED_BLOCKED ? (void*)eval_generic_kernel<CKC_SCHED_BLOCKED>
       : s == CKC_SCHED_CYCLIC  ? (void*)eval_generic_kernel<CKC_SCHED_CYCLIC>
                                : (void*)eval_generic_kernel<CKC_SCHED_DYNAMIC>;
}
// Dynamic LDS of evaluator `path` (the interpreter's register file and
// shared-memory instances; the rows-form kernel has none).
uint32_t eval_lds(const KArgs& a, uint32_t path) {
  return path == PATH_GENERIC && !a.rows_only ? regfile_bytes(a) + a.sh_bytes : 0u;
}
hipError_t launch_eval(const KArgs& a, const EvalGrid& eg, uint32_t path, hipStream_t s) {
  KArgs k = with_sched(a, eg, path);
  void* args[] = {&k};
  const uint32_t rows = path == PATH_GENERIC ? a.rows_only : 0u;
  return hipLaunchKernel(eval_fn(path, eg.sched[path], rows), dim3(eg.n_wg[path]), dim3(TILE), args,
                         eval_lds(a, path), s);
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
hipError_t launch_capture(const KArgs& a, const EvalGrid& eg, hipStream_t s) {
  KArgs k = a;
  k.capture = 1;
  k.sched = CKC_SCHED_BLOCKED;  // no schedule counter to reset
  k.chunk = 1;
  void* args[] = {&k};
  return hipLaunchKernel((void*)eval_generic_kernel<CKC_SCHED_BLOCKED>, dim3(eg.n_wg[PATH_GENERIC]), dim3(TILE),
                         args, regfile_bytes(a) + a.sh_bytes, s);
}
static void* body_fn(uint32_t sk, uint32_t which, uint32_t big) {
  const uint32_t s = sched_impl(sk);
  if (which && big)
    return s == CKC_SCHED_BLOCKED ? (void*)eval_gather_kernel<CKC_SCHED_BLOCKED, true>
         : s == CKC_SCHED_CYCLIC  ? (void*)eval_gather_kernel<CKC_SCHED_CYCLIC, true>
                                  : (void*)eval_gather_kernel<CKC_SCHED_DYNAMIC, true>;
  if (which)
    return s == CKC_SCHED_BLOCKED ? (void*)eval_gather_kernel<CKC_SCHED_BLOCKED, false>
         : s == CKC_SCHED_CYCLIC  ? (void*)eval_gather_kernel<CKC_SCHED_CYCLIC, false>
                                  : (void*)eval_gather_kernel<CKC_SCHED_DYNAMIC, false>;
  return s == CKC_SCHED_BLOCKED ? (void*)eval_body_kernel<CKC_SCHED_BLOCKED>
       : s == CKC_SCHED_CYCLIC  ? (void*)eval_body_kernel<CKC_SCHED_CYCLIC>
                                : (void*)eval_body_kernel<CKC_SCHED_DYNAMIC>;
}
static uint32_t xscan_blocks(const KArgs& a) { return (uint32_t)((a.n_xtiles + XSB - 1) / XSB); }

hipError_t launch_expand(const KArgs& a, const EvalGrid& eg, hipStream_t s) {
  if (a.n_xtiles == 0) return hipSuccess;
  const uint32_t nb = xscan_blocks(a);
  KArgs k = with_sched(a, eg, PATH_GENERIC);
  void* args[] = {&k};
  for (uint32_t which = 0; which < 2; which++) {
    if (!((eg.body_kinds >> which) & 1u)) continue;  // no body of this kind in the job
    hipLaunchKernelGGL(xscan_sums_kernel, dim3(nb), dim3(256), 0, s, a, which);
    hipLaunchKernelGGL(xscan_blocks_kernel, dim3(1), dim3(1024), 0, s, a, nb, which);
    hipLaunchKernelGGL(xscan_apply_kernel, dim3(nb), dim3(256), 0, s, a, which);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess)
      e = hipLaunchKernel(body_fn(eg.sched_body, which, eg.big_body), dim3(which ? eg.n_wg_gather : eg.n_wg_body),
                          dim3(TILE), args, body_lds_bytes(a, which == 1 && eg.big_body), s);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_fuzz_mutate(const FzArgs& f, uint64_t g, hipStream_t s) {
  hipLaunchKernelGGL(fuzz_mutate_kernel, dim3(f.batch), dim3(256), 0, s, f, g);
  return hipGetLastError();
}
hipError_t launch_fuzz_update(const FzArgs& f, uint64_t g, hipStream_t s) {
  hipLaunchKernelGGL(fuzz_classify_kernel, dim3(f.batch), dim3(256), 0, s, f, g);
  hipLaunchKernelGGL(fuzz_virgin_kernel, dim3(65536 / 4 / 256), dim3(256), 0, s, f);
  hipLaunchKernelGGL(fuzz_append_kernel, dim3(1), dim3(1024), 0, s, f, g);
  hipLaunchKernelGGL(fuzz_copy_kernel, dim3(f.batch), dim3(256), 0, s, f);
  return hipGetLastError();
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
  hipError_t e = add_node(g, &plan, nullptr, 0, (void*)plan_kernel, a.n_inputs, 64, args1, plan_lds_bytes(a));
  if (e == hipSuccess) e = add_node(g, &scan, &plan, 1, (void*)scan_kernel, 1, 1024, args1);
  if (e == hipSuccess)
    e = add_node(g, &ev[0], &scan, 1, eval_fn(PATH_BLOCKS, eg.sched[PATH_BLOCKS]), eg.n_wg[PATH_BLOCKS], TILE,
                 argsp[PATH_BLOCKS]);
  if (e == hipSuccess)
    e = add_node(g, &ev[1], &scan, 1, eval_fn(PATH_GENERIC, eg.sched[PATH_GENERIC], a.rows_only),
                 eg.n_wg[PATH_GENERIC], TILE, argsp[PATH_GENERIC], eval_lds(a, PATH_GENERIC));
  if (e == hipSuccess)
    e = add_node(g, &ev[2], &scan, 1, eval_fn(PATH_LANES, eg.sched[PATH_LANES]), eg.n_wg[PATH_LANES], TILE,
                 argsp[PATH_LANES]);
  if (e != hipSuccess) return e;
  if (a.n_xtiles) {  // generic -> (scan of pieces -> body pass) for both kinds of bodies, in parallel
    uint32_t nb = xscan_blocks(a);
    uint32_t wh[2] = {0, 1};
    void* argsw[2][2] = {{&ka, &wh[0]}, {&ka, &wh[1]}};
    void* argsb[2][3] = {{&ka, &nb, &wh[0]}, {&ka, &nb, &wh[1]}};
    hipGraphNode_t xb[2];
    uint32_t nxb = 0;
    for (uint32_t which = 0; which < 2 && e == hipSuccess; which++) {
      if (!((eg.body_kinds >> which) & 1u)) continue;  // no body of this kind in the job
      hipGraphNode_t x1, x2, x3;
      e = add_node(g, &x1, &ev[1], 1, (void*)xscan_sums_kernel, nb, 256, argsw[which]);
      if (e == hipSuccess) e = add_node(g, &x2, &x1, 1, (void*)xscan_blocks_kernel, 1, 1024, argsb[which]);
      if (e == hipSuccess) e = add_node(g, &x3, &x2, 1, (void*)xscan_apply_kernel, nb, 256, argsw[which]);
      if (e == hipSuccess)
        e = add_node(g, &xb[nxb++], &x3, 1, body_fn(eg.sched_body, which, eg.big_body),
                     which ? eg.n_wg_gather : eg.n_wg_body, TILE, argsp[PATH_GENERIC],
                     body_lds_bytes(a, which == 1 && eg.big_body));
    }
    if (e != hipSuccess) return e;
    // the replay waits for both body passes
    hipGraphNode_t join;
    e = hipGraphAddEmptyNode(&join, g, xb, nxb);
    if (e != hipSuccess) return e;
    ev[1] = join;
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
