// runtime.cpp — the C-ABI of libckc (include/ckc.h): contexts, programs,
// allocation tables, jobs.  Host code; every step of a check runs in the
// kernels of kernels.hip, queued on one HIP stream per job.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "../../include/ckc.h"
#include "dformat.h"
#include "kernels.h"
#include "loader.h"
#include "runtime.h"

using namespace ckc;
using ckc::rt::Job;
using ckc::rt::Program;
using ckc::rt::Stage;
using ckc::rt::Table;
using ckc::rt::fail;

namespace {
thread_local std::string g_err;
}  // namespace

int ckc::rt::fail(int code, const std::string& msg) {
  g_err = msg;
  return code;
}

namespace {

#define HIPCHECK(expr)                                                                   \
  do {                                                                                   \
    hipError_t _e = (expr);                                                              \
    if (_e != hipSuccess)                                                                \
      return fail(CKC_E_HIP, std::string(#expr) + ": " + hipGetErrorString(_e));         \
  } while (0)

}  // namespace

namespace {

int set_device(ckc_ctx c) {
  HIPCHECK(hipSetDevice(c->dev));
  return CKC_OK;
}

constexpr size_t POOL_LIMIT = 16ull << 30;  // bytes kept for reuse per context

void free_job(ckc_ctx c, Job& J) {
  for (auto& b : J.bufs) {
    if (c->pool_bytes + b.first <= POOL_LIMIT) {
      c->pool.emplace(b.first, b.second);
      c->pool_bytes += b.first;
    } else {
      (void)hipFree(b.second);
    }
  }
  J.bufs.clear();
  for (auto& e : J.ev)
    if (e) (void)hipEventDestroy(e);
  for (uint32_t p : J.progs) {
    auto it = c->progs.find(p);
    if (it != c->progs.end()) it->second.busy--;
  }
  for (uint32_t t : J.tables) {
    auto it = c->tables.find(t);
    if (it != c->tables.end()) it->second.busy--;
  }
}

// Releases the retiring jobs whose copies have completed (all of them, waiting,
// with wait).
void reap(ckc_ctx c, bool wait) {
  auto& R = c->retiring;
  size_t k = 0;
  for (size_t q = 0; q < R.size(); q++) {
    hipEvent_t ev = R[q].first;
    const bool done = wait ? ((void)hipEventSynchronize(ev), true) : hipEventQuery(ev) != hipErrorNotReady;
    if (done) {
      (void)hipEventDestroy(ev);
      free_job(c, R[q].second);
    } else {
      if (k != q) R[k] = std::move(R[q]);
      k++;
    }
  }
  R.resize(k);
}

template <class T>
int dalloc(ckc_ctx c, Job& J, T** out, size_t count) {
  size_t bytes = std::max<size_t>(count * sizeof(T), 256);
  bytes = (bytes + 255) & ~(size_t)255;
  void* p = nullptr;
  auto it = c->pool.lower_bound(bytes);
  if (it != c->pool.end() && it->first <= 2 * bytes) {
    bytes = it->first;
    p = it->second;
    c->pool_bytes -= bytes;
    c->pool.erase(it);
  } else {
    hipError_t e = hipMalloc(&p, bytes);
    if (e != hipSuccess) {  // release retiring jobs and pooled buffers, retry once
      reap(c, true);
      for (auto& kv : c->pool) (void)hipFree(kv.second);
      c->pool.clear();
      c->pool_bytes = 0;
      e = hipMalloc(&p, bytes);
    }
    if (e != hipSuccess) return fail(CKC_E_NOMEM, std::string("hipMalloc: ") + hipGetErrorString(e));
  }
  J.bufs.emplace_back(bytes, p);
  *out = (T*)p;
  return CKC_OK;
}

unsigned bits_of(uint64_t n) {  // bits needed for values 0..n-1
  unsigned b = 0;
  while (b < 64 && (n - 1) >> b) b++;
  return b;
}


// Launches the job's kernels as one graph; the executable graph is cached by
// its launch parameters and reused when a later job has the same ones.
hipError_t launch_graph(ckc_ctx c, const KArgs& a, const EvalGrid& eg, uint64_t n_records, hipStream_t s) {
  std::string key((const char*)&a, sizeof a);
  key.append((const char*)&eg, sizeof eg);
  key.append((const char*)&n_records, sizeof n_records);
  auto it = c->graphs.find(key);
  if (it == c->graphs.end()) {
    hipGraph_t g = nullptr;
    hipError_t e = hipGraphCreate(&g, 0);
    if (e != hipSuccess) return e;
    e = build_job_graph(g, a, eg, n_records);
    hipGraphExec_t x = nullptr;
    if (e == hipSuccess) e = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) return e;
    if (c->graphs.size() >= 32) {  // keep the cache small
      (void)hipGraphExecDestroy(c->graphs.begin()->second);
      c->graphs.erase(c->graphs.begin());
    }
    it = c->graphs.emplace(key, x).first;
  }
  return hipGraphLaunch(it->second, s);
}

}  // namespace

int ckc::rt::validate_desc(ckc_ctx c, const ckc_batch& B, uint32_t k, bool force_generic, uint64_t* ws_bytes) {
  // messages are built only on failure (a valid batch allocates nothing here)
  auto dk = [&]() { return "descriptor " + std::to_string(k) + ": "; };
  auto pit = c->progs.find(B.prog_id);
  if (pit == c->progs.end()) return fail(CKC_E_INVALID, dk() + "unknown program");
  if (B.n_inputs && (!B.launch || !B.table_ids)) return fail(CKC_E_INVALID, dk() + "arrays missing");
  const Program& P = pit->second;
  const dprog* h = (const dprog*)P.L.blob.data();
  if (h->n_scalars && B.n_inputs && !B.scalars) return fail(CKC_E_INVALID, dk() + "scalars missing");
  if (B.mode > CKC_FULL_ENDPOINTS) return fail(CKC_E_INVALID, dk() + "unknown mode");
  if (B.flags & ~(uint32_t)(CKC_DENSE_MAP | CKC_TRIPWIRE)) return fail(CKC_E_INVALID, dk() + "unknown flags");
  const bool tripwire = (B.flags & CKC_TRIPWIRE) != 0;
  uint32_t c0 = B.loop_cap_log2[0], c1 = B.loop_cap_log2[1];
  if (c0 == 0 && c1 == 0) { c0 = 20; c1 = 12; }
  if (c0 > 32 || c1 > 32) return fail(CKC_E_INVALID, dk() + "loop cap above 2^32");
  unsigned L1 = h->max_depth >= 1 ? c0 : 0, L2 = h->max_depth >= 2 ? c1 : 0;
  uint64_t ws = 0;
  for (uint32_t i = 0; i < B.n_inputs; i++) {
    auto di = [&]() { return dk() + "input " + std::to_string(i) + ": "; };
    const uint32_t* L = B.launch + 6 * (size_t)i;
    uint64_t nb = (uint64_t)L[0] * L[1] * L[2], bs = (uint64_t)L[3] * L[4] * L[5];
    if (bs > 1024) return fail(CKC_E_INVALID, di() + "block above 1024 threads");
    if (nb > 0xFFFFFFFFull) return fail(CKC_E_INVALID, di() + "grid of 2^32 blocks or more");
    uint64_t nthr = nb * bs;
    if (nthr > 1 && bits_of(nthr) + L1 + L2 > 64)
      return fail(CKC_E_RANGE, di() + "first-violation key needs more than 64 bits");
    auto tit = c->tables.find(B.table_ids[i]);
    if (tit == c->tables.end()) return fail(CKC_E_INVALID, di() + "unknown table");
    const Table& T = tit->second;
    if (T.host.size() < h->n_slots) return fail(CKC_E_INVALID, di() + "table has fewer slots than the program");
    if (h->pflags & PF_BLOCKWISE) {
      // a tile of the interpreter holds whole blocks, whose shared memory fits in LDS
      if (bs > (uint64_t)TILE || TILE % bs != 0)
        return fail(CKC_E_INVALID, di() + "blocks of a program with barriers or shared loads must divide 256 threads");
      if (B.mode == CKC_REP_CORNERS)
        return fail(CKC_E_INVALID, di() + "the corner thread set splits blocks that share memory");
      if ((h->pflags & PF_CAPTURE) && B.mode == CKC_REP_PREX)
        return fail(CKC_E_INVALID, di() + "PREX sweep of a program with index-related shared memory");
      uint64_t words = 0;  // each slot capped, so that the sum cannot wrap
      for (uint32_t s = 0; s < h->n_slots; s++)
        if (((h->slot_spaces >> (2 * s)) & 3u) == CKC_SPACE_SHARED && T.host[s].base != 0)
          words += std::min<uint64_t>(T.host[s].size_bytes / 4, SHARED_LDS_MAX);
      if ((TILE / bs) * words * 12 > SHARED_LDS_MAX)
        return fail(CKC_E_INVALID, di() + "shared memory of the blocks of one tile above 48 KiB");
    }
    if (tripwire)  // every allocation with its redzones inside [0, 2^63]
      for (size_t s = 0; s < T.host.size(); s++) {
        const ckc_alloc& A = T.host[s];
        if (A.base != 0 && (A.base < A.redzone || A.base > (1ull << 63) ||
                            A.size_bytes > (1ull << 63) - A.base ||
                            A.redzone > (1ull << 63) - A.base - A.size_bytes))
          return fail(CKC_E_INVALID, di() + "slot " + std::to_string(s) +
                                         ": allocation and redzones leave [0, 2^63] (tripwire detector)");
      }
    for (uint32_t s = 0; s < h->n_slots; s++) {
      const ckc_alloc& A = T.host[s];
      const bool live = A.base != 0 && !(A.flags & CKC_ALLOC_FREED) && A.size_bytes > 0;
      if ((P.L.load_slots >> s & 1u) && live) {
        if (A.data == nullptr) return fail(CKC_E_INVALID, di() + "slot " + std::to_string(s) + " is loaded but has no data");
        ws += A.size_bytes;
      }
    }
    ws += sizeof(dinput) + 8 * MAX_SCALARS + 4 + sizeof(ckc_input_status) + (uint64_t)h->n_accesses * sizeof(ckc_record) +
          (uint64_t)h->n_sites * 4;
    if ((h->cls & CKC_CLS_UNIFORM) && !force_generic && !tripwire) ws += ckc::trace_bytes(h->trace_cap);
    else if ((h->pflags & PF_ROWS) && !tripwire) ws += sizeof(drows);
    if (B.flags & CKC_DENSE_MAP) ws += 65536;
  }
  if (ws_bytes) *ws_bytes = ws;
  return CKC_OK;
}

hipEvent_t ckc::rt::job_done_event(ckc_ctx c, uint64_t job) {
  auto it = c->jobs.find(job);
  return it == c->jobs.end() ? nullptr : it->second.ev[ckc::rt::NEV - 1];
}

namespace {

// Where the device buffers of a staged launch sequence come from.
struct BufSource {
  virtual int get(size_t bytes, void** out) = 0;
};

// A job's buffers: the context's pool, else hipMalloc (kept in J.bufs).
struct JobBufs : BufSource {
  ckc_ctx c;
  Job& J;
  JobBufs(ckc_ctx c_, Job& J_) : c(c_), J(J_) {}
  int get(size_t bytes, void** out) override { return dalloc(c, J, (uint8_t**)out, bytes); }
};

// Consecutive pieces of the library's static scratch array (no allocation).
struct ScratchBufs : BufSource {
  uint8_t* base;
  size_t cap, used = 0;
  ScratchBufs(void* b, size_t n) : base((uint8_t*)b), cap(n) {}
  int get(size_t bytes, void** out) override {
    if (bytes > cap - used)
      return fail(CKC_E_NOMEM, "the batch needs more than the " + std::to_string(cap >> 20) +
                                   " MiB scratch of the no-allocation entry point (at least " +
                                   std::to_string((used + bytes) >> 20) + " MiB so far)");
    *out = base + used;
    used += bytes;
    return CKC_OK;
  }
};

// count elements of T, in 256-byte units
template <class T>
int take(BufSource& B, T** out, size_t count) {
  size_t bytes = std::max<size_t>(count * sizeof(T), 256);
  bytes = (bytes + 255) & ~(size_t)255;
  void* p = nullptr;
  int rc = B.get(bytes, &p);
  if (rc != CKC_OK) return rc;
  *out = (T*)p;
  return CKC_OK;
}

// Result buffers a caller brings (all NULL: take them from the source).
struct ExtOut {
  ckc_record* recs = nullptr;
  ckc_input_status* st = nullptr;
  uint8_t* maps = nullptr;
};

// Takes S's buffers from B (records, status and maps from ext when given),
// queues the copies of the inputs on stream s and fills a (kernel arguments)
// and eg (evaluator grid).  Every buffer is initialised by the kernels
// themselves, so none needs clearing here.
int stage_upload(ckc_ctx c, BufSource& B, hipStream_t s, Stage& S, const ckc_launch_opts& O, bool dense,
                 const ExtOut& ext, KArgs& a, EvalGrid& eg) {
  const uint64_t n_inputs = S.hin.size();
  // tile-space order of the inputs: as given, or largest first for LPT
  S.order.resize(n_inputs);
  for (uint64_t i = 0; i < n_inputs; i++) S.order[i] = (uint32_t)i;
  if (O.schedule == CKC_SCHED_LPT)
    std::stable_sort(S.order.begin(), S.order.end(), [&](uint32_t x, uint32_t y) { return S.est[x] > S.est[y]; });
  int rc;
  const uint64_t nx = S.n_xtiles;
  dinput* d_in = nullptr;
  int64_t* sc = nullptr;
  jobstate* js = nullptr;
  uint8_t *tr = nullptr, *xs = nullptr;
  uint32_t *order = nullptr, *xin = nullptr, *counts = nullptr;
  unsigned long long *xtot = nullptr, *xpb = nullptr, *xpg = nullptr, *xbsum = nullptr, *xd = nullptr;
  ckc_record* recs = ext.recs;
  ckc_input_status* st = ext.st;
  uint8_t* maps = ext.maps;
  if ((rc = take(B, &d_in, n_inputs)) || (rc = take(B, &sc, S.hsc.size())) || (rc = take(B, &order, n_inputs)) ||
      (nx && ((rc = take(B, &xs, S.xstate_bytes)) || (rc = take(B, &xtot, nx)) || (rc = take(B, &xpb, nx)) ||
              (rc = take(B, &xpg, nx)) || (rc = take(B, &xin, nx)) || (rc = take(B, &xd, 2 * nx)) ||
              (rc = take(B, &xbsum, 2 * ((nx + 4095) / 4096))))) ||
      (!recs && (rc = take(B, &recs, S.n_records))) || (rc = take(B, &counts, S.n_counts)) ||
      (!st && (rc = take(B, &st, n_inputs))) || (rc = take(B, &js, 1)) || (rc = take(B, &tr, S.trace_bytes)) ||
      (dense && !maps && (rc = take(B, &maps, n_inputs * 65536))))
    return rc;
  for (auto& d : S.hin) {
    if (d.trace) d.trace = (uint64_t)(uintptr_t)(tr + (d.trace - 1));
    if (d.xstate) d.xstate = (uint64_t)(uintptr_t)(xs + (d.xstate - 1));
  }
  // pageable copies are staged before hipMemcpyAsync returns, so S may be
  // reused afterwards
  hipError_t e = hipMemcpyAsync(d_in, S.hin.data(), sizeof(dinput) * n_inputs, hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipMemcpyAsync(sc, S.hsc.data(), sizeof(int64_t) * S.hsc.size(), hipMemcpyHostToDevice, s);
  if (e == hipSuccess)
    e = hipMemcpyAsync(order, S.order.data(), sizeof(uint32_t) * n_inputs, hipMemcpyHostToDevice, s);
  if (e != hipSuccess) return fail(CKC_E_HIP, std::string("staging: ") + hipGetErrorString(e));
  a.inputs = d_in;
  a.scalars = sc;
  a.n_inputs = (uint32_t)n_inputs;
  a.force_generic = O.force_generic;
  a.recs = recs;
  a.counts = counts;
  a.status = st;
  a.maps = dense ? maps : nullptr;
  a.js = js;
  a.order = order;
  a.xtot = xtot;
  a.xpb = xpb;
  a.xpg = xpg;
  a.xin = xin;
  a.xd = xd;
  a.xbsum = xbsum;
  a.n_xtiles = nx;
  a.max_regs = S.max_regs;
  a.capture = 0;
  a.sh_bytes = S.sh_bytes;
  a.rows_only = S.all_rows && !S.hin.empty() ? (S.all_rows32 ? 2u : 1u) : 0u;
  a.sched = CKC_SCHED_DYNAMIC;
  a.chunk = O.chunk ? O.chunk : 1u;
  // PATH_BLOCKS, PATH_GENERIC, PATH_LANES; the rows-form kernel keeps 6
  // wavefronts per SIMD, 7 in its 32-bit instantiation
  const uint32_t defwg[3] = {8, a.rows_only == 2 ? 7u : a.rows_only ? 6u : 4u, 2};
  for (int p = 0; p < 3; p++) {
    eg.n_wg[p] = (uint32_t)c->n_cu * (O.wg_per_cu ? O.wg_per_cu : defwg[p]);
    eg.sched[p] = O.schedule ? O.schedule : (p == PATH_GENERIC ? CKC_SCHED_DYNAMIC : CKC_SCHED_BLOCKED);
    // interpreter tiles: by default several per work item when there are
    // plenty (each item costs a schedule step and a lookup of its input)
    // (16 for the rows-form kernel, whose tiles cost less)
    eg.chunk[p] = O.chunk ? O.chunk
                          : (p == PATH_GENERIC && S.gen_tiles >= 16ull * eg.n_wg[p] ? (a.rows_only ? 16u : 4u) : 1u);
  }
  // body passes: pieces are near-equal work, and a workgroup walking one
  // contiguous range of them finds each piece's tile by a step from the last
  eg.sched_body = O.schedule ? O.schedule : CKC_SCHED_BLOCKED;
  // long gather ranges (inputs of 64 tiles or more on average) take the
  // variant with larger rounds (2 wavefronts per SIMD: the registers hold a
  // round's loads and the next round's), one workgroup per resident slot (a
  // second wave of workgroups costs more than it balances)
  eg.big_body = S.n_xin != 0 && S.n_xtiles >= 64 * S.n_xin ? 1u : 0u;
  eg.body_kinds = S.body_kinds;
  // the planner sends only uniform programs to the trace paths
  eg.no_trace = S.any_uniform ? 0u : 1u;
  eg.n_wg_body = (uint32_t)c->n_cu * (O.wg_per_cu ? O.wg_per_cu : 8u);
  eg.n_wg_gather = (uint32_t)c->n_cu * (O.wg_per_cu ? O.wg_per_cu : eg.big_body ? 2u : 8u);
  return CKC_OK;
}

// A job's buffers from the pool, recorded in J.
int stage_job(ckc_ctx c, Job& J, Stage& S, const ckc_launch_opts& O, bool dense, KArgs& a, EvalGrid& eg) {
  JobBufs B(c, J);
  int rc = stage_upload(c, B, J.stream, S, O, dense, ExtOut(), a, eg);
  if (rc != CKC_OK) return rc;
  J.d_inputs = a.inputs;
  J.d_recs = a.recs;
  J.d_counts = a.counts;
  J.d_status = a.status;
  J.d_maps = a.maps;
  return CKC_OK;
}

// Planning and every evaluator of a staged launch sequence (no replay, no
// finishing), with the stage events ev[1..3] when ev is given.
hipError_t launch_evaluation(const KArgs& a, const EvalGrid& eg, hipStream_t s, hipEvent_t* ev) {
  hipError_t e = launch_plan(a, s);
  if (e == hipSuccess) e = launch_scan(a, s);
  if (e == hipSuccess && ev) e = hipEventRecord(ev[1], s);
  if (e == hipSuccess && !eg.no_trace) e = launch_eval_trace(a, eg, s);
  if (e == hipSuccess && !eg.no_trace) e = launch_eval_trace_lanes(a, eg, s);
  if (e == hipSuccess && ev) e = hipEventRecord(ev[2], s);
  if (e == hipSuccess) e = launch_eval_generic(a, eg, s);
  if (e == hipSuccess && ev) e = hipEventRecord(ev[3], s);
  if (e == hipSuccess) e = launch_expand(a, eg, s);
  return e;
}

// Key bits of the loop depths a program uses, from a descriptor's caps.
void key_bits(const ckc_batch& B, const dprog* h, uint32_t& c0, uint32_t& c1, unsigned& L1, unsigned& L2) {
  c0 = B.loop_cap_log2[0];
  c1 = B.loop_cap_log2[1];
  if (c0 == 0 && c1 == 0) { c0 = 20; c1 = 12; }
  L1 = h->max_depth >= 1 ? c0 : 0;
  L2 = h->max_depth >= 2 ? c1 : 0;
}

dinput input_of(const Program& P, const Table& T, const ckc_batch& B, uint32_t i) {
  const dprog* h = (const dprog*)P.L.blob.data();
  dinput d;
  std::memset(&d, 0, sizeof d);
  d.prog = (uint64_t)(uintptr_t)P.dblob;
  d.table = (uint64_t)(uintptr_t)T.dptr;
  for (int q = 0; q < 6; q++) d.launch[q] = B.launch[6 * (size_t)i + q];
  uint32_t c0, c1;
  unsigned L1, L2;
  key_bits(B, h, c0, c1, L1, L2);
  d.L1 = L1;
  d.L2 = L2;
  d.cap_log2[0] = c0;
  d.cap_log2[1] = c1;
  return d;
}

// Every input of every (validated, non-PREX) descriptor, in order.
void stage_inputs(ckc_ctx c, const ckc_batch* descs, uint32_t n_descs, const ckc_launch_opts& O, Stage& S) {
  for (uint32_t k = 0; k < n_descs; k++) {
    const ckc_batch& B = descs[k];
    const Program& P = c->progs.find(B.prog_id)->second;
    const dprog* h = (const dprog*)P.L.blob.data();
    for (uint32_t i = 0; i < B.n_inputs; i++) {
      const Table& T = c->tables.find(B.table_ids[i])->second;
      dinput d = input_of(P, T, B, i);
      d.mode = B.mode == CKC_FULL_ENDPOINTS ? CKC_FULL : B.mode;
      d.aux = B.mode == CKC_FULL_ENDPOINTS ? 1u : 0u;
      d.detector = (B.flags & CKC_TRIPWIRE) ? 1u : 0u;
      const uint32_t* L = d.launch;
      const uint64_t nthr = (uint64_t)L[0] * L[1] * L[2] * ((uint64_t)L[3] * L[4] * L[5]);
      // most lanes of the thread set (the corner set has at most 64)
      const uint64_t lanes_max = B.mode == CKC_REP_CORNERS ? std::min<uint64_t>(nthr, 64) : nthr;
      // tripwire inputs take the interpreter: no trace of their own
      S.add(h, d, B.scalars ? B.scalars + (size_t)i * h->n_scalars : nullptr, lanes_max,
            O.force_generic != 0 || d.detector != 0);
      S.note_blockwise(h, T.host.data(), (uint32_t)T.host.size(), d.launch);
    }
  }
}

void mark_busy(ckc_ctx c, Job& J, const ckc_batch* descs, uint32_t n_descs) {
  for (uint32_t k = 0; k < n_descs; k++) {
    J.progs.push_back(descs[k].prog_id);
    c->progs[descs[k].prog_id].busy++;
    for (uint32_t i = 0; i < descs[k].n_inputs; i++) {
      J.tables.push_back(descs[k].table_ids[i]);
      c->tables[descs[k].table_ids[i]].busy++;
    }
  }
}

// Most (input, round) pairs and most lanes in one window of a PREX sweep.
constexpr uint64_t PREX_WINDOW_PAIRS = 1ull << 18;
constexpr uint64_t PREX_WINDOW_LANES = 1ull << 30;

// CKC_REP_PREX: the sweep of Algorithm 1 over every input, in windows of
// rounds (1, then 1, 2, 4, ... rounds per input), each an evaluation of
// (input, round) pairs followed by the fold; the stop flags are read back
// after each window to decide the next one.  Then the replay of first
// violations and the finishing pass over the inputs themselves.
int check_prex(ckc_ctx c, const ckc_batch* descs, uint32_t n_descs, const ckc_launch_opts& O, uint64_t* job) {
  Stage R;  // the inputs themselves
  std::vector<uint32_t> rounds;  // ceil(nblocks / 2) per input (0: empty grid)
  std::vector<const dprog*> heads;
  std::vector<const ckc_alloc*> tabs_host;  // each input's table (host copy) and its entries
  std::vector<uint32_t> tabs_n;
  for (uint32_t k = 0; k < n_descs; k++) {
    const ckc_batch& B = descs[k];
    const Program& P = c->progs.find(B.prog_id)->second;
    const dprog* h = (const dprog*)P.L.blob.data();
    for (uint32_t i = 0; i < B.n_inputs; i++) {
      const Table& T = c->tables.find(B.table_ids[i])->second;
      dinput d = input_of(P, T, B, i);
      d.mode = CKC_REP_PREX;
      d.detector = (B.flags & CKC_TRIPWIRE) ? 1u : 0u;
      d.path = PATH_GENERIC;  // results arrive folded: the finishing pass only builds maps
      const uint32_t* L = d.launch;
      const uint64_t nb = (uint64_t)L[0] * L[1] * L[2], bs = (uint64_t)L[3] * L[4] * L[5];
      rounds.push_back(nb == 0 || bs == 0 ? 0u : (uint32_t)((nb + 1) / 2));
      heads.push_back(h);
      tabs_host.push_back(T.host.data());
      tabs_n.push_back((uint32_t)T.host.size());
      // the inputs need no trace or loop state of their own
      R.add(h, d, B.scalars ? B.scalars + (size_t)i * h->n_scalars : nullptr, 0, true);
    }
  }
  const uint64_t n_inputs = R.hin.size();
  if (n_inputs == 0) return fail(CKC_E_INVALID, "no inputs");
  if (n_inputs > 0xFFFFFFFFull) return fail(CKC_E_INVALID, "too many inputs");
  int rc;
  if ((rc = set_device(c))) return rc;
  reap(c, false);
  Job J;
  J.n_inputs = n_inputs;
  J.n_records = R.n_records;
  J.stream = O.hip_stream ? (hipStream_t)O.hip_stream : c->stream;
  J.dense = false;
  for (uint32_t k = 0; k < n_descs; k++) J.dense |= (descs[k].flags & CKC_DENSE_MAP) != 0;
  auto bail = [&](int code) {
    (void)hipStreamSynchronize(J.stream);
    free_job(c, J);
    return code;
  };
  KArgs a;
  EvalGrid eg;
  uint32_t* d_stop = nullptr;
  prex_item* d_items = nullptr;
  if ((rc = stage_job(c, J, R, O, J.dense, a, eg)) || (rc = dalloc(c, J, &d_stop, n_inputs)) ||
      (rc = dalloc(c, J, &d_items, std::min<uint64_t>(n_inputs, PREX_WINDOW_PAIRS))))
    return bail(rc);
  std::vector<uint32_t> h_stop(n_inputs, 0);
  hipError_t e = hipSuccess;
  for (int q = 0; q < ckc::rt::NEV && e == hipSuccess; q++) e = hipEventCreate(&J.ev[q]);
  if (e != hipSuccess) return bail(fail(CKC_E_HIP, std::string("events: ") + hipGetErrorString(e)));
  PrexArgs p;
  std::memset(&p, 0, sizeof p);
  p.real_in = a.inputs;
  p.n_real = (uint32_t)n_inputs;
  p.real_recs = a.recs;
  p.real_counts = a.counts;
  p.real_status = a.status;
  p.stopped = d_stop;
  p.items = d_items;
  e = hipEventRecord(J.ev[0], J.stream);
  if (e == hipSuccess) e = launch_prex_init(p, J.stream);
  if (e == hipSuccess) e = hipEventRecord(J.ev[1], J.stream);
  if (e != hipSuccess) return bail(fail(CKC_E_HIP, std::string("launch: ") + hipGetErrorString(e)));
  // inputs whose sweep goes on, and the next round of each
  std::vector<uint32_t> active, next(n_inputs, 0);
  for (uint64_t i = 0; i < n_inputs; i++)
    if (rounds[i]) active.push_back((uint32_t)i);
  ckc_launch_opts WO = O;
  WO.use_graph = 0;
  uint64_t per = 1;   // rounds per input in the current pass over the active inputs
  size_t cursor = 0;  // first active input of the next window
  while (!active.empty()) {
    Stage W;
    std::vector<prex_item> items;
    uint64_t lanes = 0;
    size_t end = cursor;
    for (; end < active.size(); end++) {
      const uint32_t i = active[end];
      const dinput& d = R.hin[i];
      const uint64_t bs2 = 2ull * d.launch[3] * d.launch[4] * d.launch[5];
      // window limits; every window takes at least one round of one input
      const uint64_t room = std::min<uint64_t>(PREX_WINDOW_PAIRS - W.hin.size(),
                                               lanes < PREX_WINDOW_LANES ? (PREX_WINDOW_LANES - lanes) / bs2 : 0);
      if (room == 0 && !items.empty()) break;
      const uint64_t n = std::max<uint64_t>(1, std::min<uint64_t>({per, (uint64_t)(rounds[i] - next[i]), room}));
      prex_item X;
      X.real = i;
      X.vbeg = (uint32_t)W.hin.size();
      X.vcnt = (uint32_t)n;
      X.r0 = next[i];
      X.last = rounds[i] - 1;
      X.pad = 0;
      items.push_back(X);
      const int64_t* sc = &R.hsc[(size_t)i * MAX_SCALARS];
      for (uint64_t r = 0; r < n; r++) {
        dinput v = d;
        v.rec_base = v.cnt_base = 0;
        v.trace = v.xstate = v.xt_begin = v.xn = v.n_xt = 0;
        v.mode = MODE_PAIR;
        v.aux = next[i] + (uint32_t)r;
        v.path = 0;
        W.add(heads[i], v, sc, bs2, O.force_generic != 0 || v.detector != 0);
        W.note_blockwise(heads[i], (const ckc_alloc*)tabs_host[i], tabs_n[i], v.launch);
        lanes += bs2;
      }
    }
    // the window's buffers live until its stop flags have been read back
    Job WJ;
    WJ.stream = J.stream;
    KArgs wa;
    EvalGrid weg;
    if ((rc = stage_job(c, WJ, W, WO, false, wa, weg))) {
      free_job(c, WJ);
      return bail(rc);
    }
    p.n_items = (uint32_t)items.size();
    p.vin = wa.inputs;
    p.vrecs = wa.recs;
    p.vcounts = wa.counts;
    p.vstatus = wa.status;
    e = hipMemcpyAsync(d_items, items.data(), sizeof(prex_item) * items.size(), hipMemcpyHostToDevice, J.stream);
    if (e == hipSuccess) e = launch_evaluation(wa, weg, J.stream, nullptr);
    if (e == hipSuccess) e = launch_prex_merge(p, J.stream);
    if (e == hipSuccess)
      e = hipMemcpyAsync(h_stop.data(), d_stop, sizeof(uint32_t) * n_inputs, hipMemcpyDeviceToHost, J.stream);
    if (e == hipSuccess) e = hipStreamSynchronize(J.stream);
    free_job(c, WJ);
    if (e != hipSuccess) return bail(fail(CKC_E_HIP, std::string("PREX window: ") + hipGetErrorString(e)));
    // inputs of this window move on or drop out; the others wait their turn
    for (const prex_item& X : items) next[X.real] += X.vcnt;
    std::vector<uint32_t> still;
    size_t new_cursor = 0;
    for (size_t q = 0; q < active.size(); q++) {
      const uint32_t i = active[q];
      if (q == end) new_cursor = still.size();
      if (q >= cursor && q < end && (h_stop[i] || next[i] >= rounds[i])) continue;
      still.push_back(i);
    }
    if (end == active.size()) {  // a whole pass: the next one takes twice the rounds
      cursor = 0;
      per *= 2;
    } else {
      cursor = new_cursor;
    }
    active.swap(still);
  }
  e = hipEventRecord(J.ev[2], J.stream);
  if (e == hipSuccess) e = hipEventRecord(J.ev[3], J.stream);
  if (e == hipSuccess) e = hipEventRecord(J.ev[4], J.stream);
  if (e == hipSuccess) e = launch_fixup(a, R.n_records, J.stream);
  if (e == hipSuccess) e = launch_finish(a, J.stream);
  if (e == hipSuccess) e = hipEventRecord(J.ev[ckc::rt::NEV - 1], J.stream);
  if (e != hipSuccess) return bail(fail(CKC_E_HIP, std::string("launch: ") + hipGetErrorString(e)));
  mark_busy(c, J, descs, n_descs);
  uint64_t id = c->next_job++;
  c->jobs.emplace(id, std::move(J));
  *job = id;
  return CKC_OK;
}

}  // namespace

int ckc::rt::stage_new_job(ckc_ctx c, Job& J, Stage& S, bool dense, KArgs& a, EvalGrid& eg) {
  ckc_launch_opts O;
  std::memset(&O, 0, sizeof O);
  return stage_job(c, J, S, O, dense, a, eg);
}
dinput ckc::rt::make_input(const Program& P, const Table& T, const ckc_batch& B, uint32_t i) {
  return input_of(P, T, B, i);
}
hipError_t ckc::rt::run_evaluation(const KArgs& a, const EvalGrid& eg, hipStream_t s) {
  return launch_evaluation(a, eg, s, nullptr);
}
void ckc::rt::release_job(ckc_ctx c, Job& J) { free_job(c, J); }
unsigned ckc::rt::index_bits(uint64_t n) { return bits_of(n); }

extern "C" {

const char* ckc_last_error(void) { return g_err.c_str(); }

int ckc_init(int hip_device, ckc_ctx* out) {
  if (!out) return fail(CKC_E_INVALID, "out is NULL");
  int n = 0;
  if (hipGetDeviceCount(&n) != hipSuccess || hip_device < 0 || hip_device >= n)
    return fail(CKC_E_INVALID, "no such HIP device");
  ckc_ctx c = new (std::nothrow) ckc_ctx_s;
  if (!c) return fail(CKC_E_NOMEM, "context");
  c->dev = hip_device;
  hipError_t e = hipSetDevice(hip_device);
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking);
  if (e != hipSuccess) {
    delete c;
    return fail(CKC_E_HIP, std::string("context stream: ") + hipGetErrorString(e));
  }
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, hip_device) == hipSuccess) c->n_cu = prop.multiProcessorCount;
  // the no-allocation entry point: the scratch address on this device (the
  // device is current) and host staging room for its largest call
  e = ckc::scratch_address(hip_device, &c->scratch);
  if (e != hipSuccess) {
    (void)hipStreamDestroy(c->stream);
    delete c;
    return fail(CKC_E_HIP, std::string("scratch address: ") + hipGetErrorString(e));
  }
  try {
    c->na_stage.reserve(CKC_NOALLOC_MAX_INPUTS);
  } catch (const std::bad_alloc&) {
    (void)hipStreamDestroy(c->stream);
    delete c;
    return fail(CKC_E_NOMEM, "context staging arrays");
  }
  *out = c;
  return CKC_OK;
}

void ckc_shutdown(ckc_ctx c) {
  if (!c) return;
  (void)hipSetDevice(c->dev);
  reap(c, true);
  for (auto& kv : c->jobs) {
    if (kv.second.stream) (void)hipStreamSynchronize(kv.second.stream);
    free_job(c, kv.second);
  }
  c->jobs.clear();
  for (auto& kv : c->progs) (void)hipFree(kv.second.dblob);
  for (auto& kv : c->tables) (void)hipFree(kv.second.dptr);
  for (auto& kv : c->pool) (void)hipFree(kv.second);
  for (auto& kv : c->graphs) (void)hipGraphExecDestroy(kv.second);
  if (c->stream) (void)hipStreamDestroy(c->stream);
  delete c;
}

int ckc_analyze_ir(const void* ir, size_t ir_bytes, ckc_prog_info* info, ckc_access_info* acc,
                   uint32_t acc_capacity) {
  Loaded L;
  int rc = analyze_program(ir, ir_bytes, &L);
  if (rc != CKC_OK) return fail(rc, L.err);
  if (info) *info = L.info;
  if (acc) {
    uint32_t n = std::min<uint32_t>(acc_capacity, (uint32_t)L.acc.size());
    std::memcpy(acc, L.acc.data(), n * sizeof(ckc_access_info));
  }
  return CKC_OK;
}

int ckc_load_program(ckc_ctx c, const void* ir, size_t ir_bytes, uint32_t* prog_id, ckc_prog_info* info) {
  if (!c || !prog_id) return fail(CKC_E_INVALID, "NULL argument");
  Program P;
  int rc = analyze_program(ir, ir_bytes, &P.L);
  if (rc != CKC_OK) return fail(rc, P.L.err);
  if ((rc = set_device(c))) return rc;
  hipError_t e = hipMalloc(&P.dblob, P.L.blob.size());
  if (e != hipSuccess) return fail(CKC_E_NOMEM, "program upload");
  e = hipMemcpy(P.dblob, P.L.blob.data(), P.L.blob.size(), hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    (void)hipFree(P.dblob);
    return fail(CKC_E_HIP, std::string("program upload: ") + hipGetErrorString(e));
  }
  uint32_t id = c->next_prog++;
  if (info) *info = P.L.info;
  c->progs.emplace(id, std::move(P));
  *prog_id = id;
  return CKC_OK;
}

int ckc_load_program_ex(ckc_ctx c, const void* ir, size_t ir_bytes, uint32_t flags, uint32_t* prog_id,
                        ckc_prog_info* info) {
  if (!c || !prog_id) return fail(CKC_E_INVALID, "NULL argument");
  if (flags & ~(uint32_t)CKC_LOAD_NO_PRUNE) return fail(CKC_E_INVALID, "unknown load flags");
  Program P;
  int rc = analyze_program(ir, ir_bytes, &P.L, (flags & CKC_LOAD_NO_PRUNE) != 0);
  if (rc != CKC_OK) return fail(rc, P.L.err);
  if ((rc = set_device(c))) return rc;
  hipError_t e = hipMalloc(&P.dblob, P.L.blob.size());
  if (e != hipSuccess) return fail(CKC_E_NOMEM, "program upload");
  e = hipMemcpy(P.dblob, P.L.blob.data(), P.L.blob.size(), hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    (void)hipFree(P.dblob);
    return fail(CKC_E_HIP, std::string("program upload: ") + hipGetErrorString(e));
  }
  uint32_t id = c->next_prog++;
  if (info) *info = P.L.info;
  c->progs.emplace(id, std::move(P));
  *prog_id = id;
  return CKC_OK;
}

int ckc_unload_program(ckc_ctx c, uint32_t prog_id) {
  if (!c) return fail(CKC_E_INVALID, "NULL context");
  auto it = c->progs.find(prog_id);
  if (it == c->progs.end()) return fail(CKC_E_INVALID, "unknown program id");
  if (it->second.busy) reap(c, true);
  if (it->second.busy) return fail(CKC_E_BUSY, "program used by an unread job");
  set_device(c);
  (void)hipFree(it->second.dblob);
  c->progs.erase(it);
  return CKC_OK;
}

int ckc_put_alloc_table(ckc_ctx c, const ckc_alloc* entries, uint32_t n, uint32_t* table_id) {
  if (!c || !entries || !table_id) return fail(CKC_E_INVALID, "NULL argument");
  if (n == 0 || n > CKC_IR_MAX_SLOTS) return fail(CKC_E_INVALID, "a table holds 1..16 entries");
  int rc;
  if ((rc = set_device(c))) return rc;
  Table T;
  T.host.assign(entries, entries + n);
  T.host.resize(MAX_SLOTS, ckc_alloc{0, 0, nullptr, 0, 0});
  hipError_t e = hipMalloc(&T.dptr, sizeof(ckc_alloc) * MAX_SLOTS);
  if (e != hipSuccess) return fail(CKC_E_NOMEM, "table");
  e = hipMemcpy(T.dptr, T.host.data(), sizeof(ckc_alloc) * MAX_SLOTS, hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    (void)hipFree(T.dptr);
    return fail(CKC_E_HIP, std::string("table upload: ") + hipGetErrorString(e));
  }
  T.host.resize(n);
  uint32_t id = c->next_table++;
  c->tables.emplace(id, std::move(T));
  *table_id = id;
  return CKC_OK;
}

int ckc_free_alloc_table(ckc_ctx c, uint32_t table_id) {
  if (!c) return fail(CKC_E_INVALID, "NULL context");
  auto it = c->tables.find(table_id);
  if (it == c->tables.end()) return fail(CKC_E_INVALID, "unknown table id");
  if (it->second.busy) reap(c, true);
  if (it->second.busy) return fail(CKC_E_BUSY, "table used by an unread job");
  set_device(c);
  (void)hipFree(it->second.dptr);
  c->tables.erase(it);
  return CKC_OK;
}

int ckc_check_batch(ckc_ctx c, const ckc_batch* descs, uint32_t n_descs, const ckc_launch_opts* opts,
                    uint64_t* job) {
  if (!c || !descs || !job || n_descs == 0) return fail(CKC_E_INVALID, "NULL argument or no descriptor");
  ckc_launch_opts O;
  std::memset(&O, 0, sizeof O);
  if (opts) O = *opts;
  if (O.schedule > CKC_SCHED_LPT) return fail(CKC_E_INVALID, "unknown schedule");
  if (O.chunk > 256) return fail(CKC_E_INVALID, "chunk above 256 tiles");
  if (O.wg_per_cu > 32) return fail(CKC_E_INVALID, "wg_per_cu above 32");
  // ---- validate and build the input list on the host (copies only) ----
  uint32_t n_prex = 0;
  for (uint32_t k = 0; k < n_descs; k++) {
    int vr = ckc::rt::validate_desc(c, descs[k], k, O.force_generic != 0, nullptr);
    if (vr != CKC_OK) return vr;
    n_prex += descs[k].mode == CKC_REP_PREX;
  }
  if (n_prex && n_prex != n_descs)
    return fail(CKC_E_INVALID, "a job holds CKC_REP_PREX descriptors only, or none");
  if (n_prex) return check_prex(c, descs, n_descs, O, job);
  Stage S;
  stage_inputs(c, descs, n_descs, O, S);
  const uint64_t n_inputs = S.hin.size();
  if (n_inputs == 0) return fail(CKC_E_INVALID, "no inputs");
  if (n_inputs > 0xFFFFFFFFull) return fail(CKC_E_INVALID, "too many inputs");
  int rc;
  if ((rc = set_device(c))) return rc;
  reap(c, false);
  Job J;
  J.n_inputs = n_inputs;
  J.n_records = S.n_records;
  J.stream = O.hip_stream ? (hipStream_t)O.hip_stream : c->stream;
  J.dense = false;
  for (uint32_t k = 0; k < n_descs; k++) J.dense |= (descs[k].flags & CKC_DENSE_MAP) != 0;
  auto bail = [&](int code) {
    (void)hipStreamSynchronize(J.stream);
    free_job(c, J);
    return code;
  };
  KArgs a;
  EvalGrid eg;
  if ((rc = stage_job(c, J, S, O, J.dense, a, eg))) return bail(rc);
  hipError_t e = hipSuccess;
  for (int q = 0; q < ckc::rt::NEV && e == hipSuccess; q++) e = hipEventCreate(&J.ev[q]);
  if (e != hipSuccess) return bail(fail(CKC_E_HIP, std::string("staging: ") + hipGetErrorString(e)));
  J.graph = O.use_graph != 0 && !S.capture;  // the capture pass runs outside graphs
  e = hipEventRecord(J.ev[0], J.stream);
  if (J.graph) {
    if (e == hipSuccess) e = launch_graph(c, a, eg, S.n_records, J.stream);
    for (int q = 1; q < ckc::rt::NEV - 1 && e == hipSuccess; q++) e = hipEventRecord(J.ev[q], J.stream);
  } else {
    if (e == hipSuccess) e = launch_evaluation(a, eg, J.stream, J.ev);
    if (e == hipSuccess && S.capture) e = launch_capture(a, eg, J.stream);
    if (e == hipSuccess) e = hipEventRecord(J.ev[4], J.stream);
    if (e == hipSuccess) e = launch_fixup(a, S.n_records, J.stream);
    if (e == hipSuccess) e = launch_finish(a, J.stream);
  }
  if (e == hipSuccess) e = hipEventRecord(J.ev[ckc::rt::NEV - 1], J.stream);
  if (e != hipSuccess) return bail(fail(CKC_E_HIP, std::string("launch: ") + hipGetErrorString(e)));
  mark_busy(c, J, descs, n_descs);
  uint64_t id = c->next_job++;
  c->jobs.emplace(id, std::move(J));
  *job = id;
  return CKC_OK;
}

int ckc_check_batch_noalloc(ckc_ctx c, const ckc_batch* descs, uint32_t n_descs, const ckc_launch_opts* opts,
                            ckc_record* recs, uint8_t* maps, ckc_input_status* st) {
  if (!c || !descs || n_descs == 0) return fail(CKC_E_INVALID, "NULL argument or no descriptor");
  if (!recs || !st) return fail(CKC_E_INVALID, "records and status buffers are required");
  if (!c->scratch) return fail(CKC_E_HIP, "no scratch address on this device");
  ckc_launch_opts O;
  std::memset(&O, 0, sizeof O);
  if (opts) O = *opts;
  if (O.schedule > CKC_SCHED_LPT) return fail(CKC_E_INVALID, "unknown schedule");
  if (O.chunk > 256) return fail(CKC_E_INVALID, "chunk above 256 tiles");
  if (O.wg_per_cu > 32) return fail(CKC_E_INVALID, "wg_per_cu above 32");
  if (O.use_graph) return fail(CKC_E_INVALID, "use_graph is not available without allocation");
  uint64_t n_inputs = 0;
  bool dense = false;
  for (uint32_t k = 0; k < n_descs; k++) {
    int vr = ckc::rt::validate_desc(c, descs[k], k, O.force_generic != 0, nullptr);
    if (vr != CKC_OK) return vr;
    if (descs[k].mode == CKC_REP_PREX)
      return fail(CKC_E_INVALID, "CKC_REP_PREX is not available without allocation");
    n_inputs += descs[k].n_inputs;
    dense |= (descs[k].flags & CKC_DENSE_MAP) != 0;
  }
  if (n_inputs == 0) return fail(CKC_E_INVALID, "no inputs");
  if (n_inputs > CKC_NOALLOC_MAX_INPUTS)
    return fail(CKC_E_INVALID, "more than " + std::to_string(CKC_NOALLOC_MAX_INPUTS) +
                                   " inputs in one call without allocation");
  if (dense != (maps != nullptr))
    return fail(CKC_E_INVALID, dense ? "dense maps requested but maps is NULL"
                                     : "maps given but no descriptor has CKC_DENSE_MAP");
  Stage& S = c->na_stage;  // reserved for CKC_NOALLOC_MAX_INPUTS inputs by ckc_init
  S.clear();
  stage_inputs(c, descs, n_descs, O, S);
  int rc;
  if ((rc = set_device(c))) return rc;
  const hipStream_t s = O.hip_stream ? (hipStream_t)O.hip_stream : c->stream;
  ScratchBufs B(c->scratch, CKC_NOALLOC_SCRATCH_BYTES);
  ExtOut ext;
  ext.recs = recs;
  ext.st = st;
  ext.maps = maps;
  KArgs a;
  EvalGrid eg;
  if ((rc = stage_upload(c, B, s, S, O, dense, ext, a, eg))) return rc;
  hipError_t e = launch_evaluation(a, eg, s, nullptr);
  if (e == hipSuccess && S.capture) e = launch_capture(a, eg, s);
  if (e == hipSuccess) e = launch_fixup(a, S.n_records, s);
  if (e == hipSuccess) e = launch_finish(a, s);
  if (e != hipSuccess) return fail(CKC_E_HIP, std::string("launch: ") + hipGetErrorString(e));
  return CKC_OK;
}

int ckc_job_sizes(ckc_ctx c, uint64_t job, uint64_t* n_inputs, uint64_t* n_records) {
  if (!c) return fail(CKC_E_INVALID, "NULL context");
  auto it = c->jobs.find(job);
  if (it == c->jobs.end()) return fail(CKC_E_INVALID, "unknown job");
  if (n_inputs) *n_inputs = it->second.n_inputs;
  if (n_records) *n_records = it->second.n_records;
  return CKC_OK;
}

int ckc_job_timing(ckc_ctx c, uint64_t job, float* ms5) {
  if (!c || !ms5) return fail(CKC_E_INVALID, "NULL argument");
  auto it = c->jobs.find(job);
  if (it == c->jobs.end()) return fail(CKC_E_INVALID, "unknown job");
  Job& J = it->second;
  set_device(c);
  HIPCHECK(hipEventSynchronize(J.ev[ckc::rt::NEV - 1]));
  if (J.graph) {
    for (int q = 0; q < ckc::rt::NEV - 1; q++) ms5[q] = -1.0f;
    return CKC_OK;
  }
  for (int q = 0; q < ckc::rt::NEV - 1; q++) HIPCHECK(hipEventElapsedTime(&ms5[q], J.ev[q], J.ev[q + 1]));
  return CKC_OK;
}

int ckc_job_elapsed(ckc_ctx c, uint64_t job, float* ms) {
  if (!c || !ms) return fail(CKC_E_INVALID, "NULL argument");
  auto it = c->jobs.find(job);
  if (it == c->jobs.end()) return fail(CKC_E_INVALID, "unknown job");
  Job& J = it->second;
  set_device(c);
  HIPCHECK(hipEventSynchronize(J.ev[ckc::rt::NEV - 1]));
  HIPCHECK(hipEventElapsedTime(ms, J.ev[0], J.ev[ckc::rt::NEV - 1]));
  return CKC_OK;
}

int ckc_read_results(ckc_ctx c, uint64_t job, ckc_record* recs, uint8_t* maps, ckc_input_status* st,
                     uint32_t flags) {
  if (!c) return fail(CKC_E_INVALID, "NULL context");
  auto it = c->jobs.find(job);
  if (it == c->jobs.end()) return fail(CKC_E_INVALID, "unknown job");
  Job& J = it->second;
  int rc;
  if ((rc = set_device(c))) return rc;
  if (!(flags & CKC_WAIT)) {
    hipError_t q = hipEventQuery(J.ev[ckc::rt::NEV - 1]);
    if (q == hipErrorNotReady) return CKC_NOT_READY;
    if (q != hipSuccess) return fail(CKC_E_HIP, std::string("job: ") + hipGetErrorString(q));
  }
  if (maps && !J.dense) return fail(CKC_E_INVALID, "maps requested but the job was not run with CKC_DENSE_MAP");
  const bool enq = (flags & CKC_ENQUEUE) != 0;
  if (enq && !(flags & CKC_DST_DEVICE)) return fail(CKC_E_INVALID, "CKC_ENQUEUE needs CKC_DST_DEVICE");
  hipMemcpyKind kind = (flags & CKC_DST_DEVICE) ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
  hipError_t e = hipSuccess;
  if (recs) e = hipMemcpyAsync(recs, J.d_recs, sizeof(ckc_record) * J.n_records, kind, J.stream);
  if (e == hipSuccess && maps) e = hipMemcpyAsync(maps, J.d_maps, J.n_inputs * 65536, kind, J.stream);
  if (e == hipSuccess && st) e = hipMemcpyAsync(st, J.d_status, sizeof(ckc_input_status) * J.n_inputs, kind, J.stream);
  if (enq && e == hipSuccess) {
    hipEvent_t done = nullptr;
    e = hipEventCreateWithFlags(&done, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventRecord(done, J.stream);
    if (e == hipSuccess) {
      c->retiring.emplace_back(done, std::move(J));
      c->jobs.erase(it);
      return CKC_OK;
    }
    if (done) (void)hipEventDestroy(done);
  }
  if (e == hipSuccess) e = hipStreamSynchronize(J.stream);
  if (e != hipSuccess) return fail(CKC_E_HIP, std::string("readback: ") + hipGetErrorString(e));
  free_job(c, J);
  c->jobs.erase(it);
  return CKC_OK;
}

int ckc_autotune(ckc_ctx c, const ckc_batch* descs, uint32_t n_descs, const ckc_launch_opts* base,
                 uint32_t reps, ckc_launch_opts* best, ckc_tune_entry* log, uint32_t log_cap,
                 uint32_t* n_log) {
  if (!c || !descs || !best || n_descs == 0) return fail(CKC_E_INVALID, "NULL argument or no descriptor");
  ckc_launch_opts B;
  std::memset(&B, 0, sizeof B);
  if (base) B = *base;
  if (reps == 0) reps = 1;
  const uint32_t scheds[4] = {CKC_SCHED_BLOCKED, CKC_SCHED_CYCLIC, CKC_SCHED_DYNAMIC, CKC_SCHED_LPT};
  const uint32_t chunks[3] = {1, 4, 16};
  const uint32_t wgs[5] = {0, 2, 4, 8, 16};
  float best_ms = -1.0f;
  uint32_t n = 0;
  for (uint32_t sc : scheds)
    for (uint32_t ch : chunks) {
      if (sc == CKC_SCHED_BLOCKED && ch != 1) continue;  // one range per workgroup: chunk unused
      for (uint32_t wg : wgs) {
        ckc_launch_opts O = B;
        O.schedule = sc;
        O.chunk = ch;
        O.wg_per_cu = wg;
        float t_min = -1.0f;
        for (uint32_t r = 0; r < reps; r++) {
          uint64_t job = 0;
          int rc = ckc_check_batch(c, descs, n_descs, &O, &job);
          if (rc != CKC_OK) return rc;
          float ms = 0;
          rc = ckc_job_elapsed(c, job, &ms);
          int rc2 = ckc_read_results(c, job, nullptr, nullptr, nullptr, CKC_WAIT);
          if (rc != CKC_OK) return rc;
          if (rc2 != CKC_OK) return rc2;
          if (t_min < 0 || ms < t_min) t_min = ms;
        }
        if (log && n < log_cap) {
          log[n].opts = O;
          log[n].ms = t_min;
          log[n].pad = 0;
        }
        n++;
        if (best_ms < 0 || t_min < best_ms) {
          best_ms = t_min;
          *best = O;
        }
      }
    }
  if (n_log) *n_log = n < log_cap ? n : log_cap;
  return CKC_OK;
}

}  // extern "C"
