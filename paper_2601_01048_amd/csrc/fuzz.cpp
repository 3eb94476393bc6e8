// fuzz.cpp — closed-loop fuzzing campaigns on the device (include/ckc.h,
// ckc_fuzz_*): the children of a generation are the inputs of one job staged
// once at creation; every generation is mutation, the job's evaluation, and
// the campaign update, all queued on the context's stream.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "../../include/ckc.h"
#include "dformat.h"
#include "kernels.h"
#include "runtime.h"

using namespace ckc;
using ckc::rt::fail;

struct ckc_fuzz_s {
  ckc_ctx c = nullptr;
  ckc_fuzz_config cfg{};
  uint32_t n_acc = 0;
  uint64_t n_records = 0;
  uint64_t gen = 0;  // generations queued so far
  bool capture = false;  // the children's program needs the capture pass
  rt::Job J;         // the children's job buffers (from the context's pool)
  KArgs a{};
  EvalGrid eg{};
  FzArgs f{};
  std::vector<void*> own;  // the campaign's own device buffers
};

namespace {

template <class T>
int own_alloc(ckc_fuzz F, T** out, size_t count) {
  void* p = nullptr;
  const size_t bytes = std::max<size_t>(count * sizeof(T), 256);
  if (hipMalloc(&p, bytes) != hipSuccess) return fail(CKC_E_NOMEM, "fuzzing campaign buffers");
  F->own.push_back(p);
  *out = (T*)p;
  return CKC_OK;
}

void release(ckc_fuzz F) {
  ckc_ctx c = F->c;
  (void)hipSetDevice(c->dev);
  (void)hipStreamSynchronize(c->stream);
  rt::release_job(c, F->J);
  for (void* p : F->own) (void)hipFree(p);
  F->own.clear();
  auto pit = c->progs.find(F->cfg.prog_id);
  if (pit != c->progs.end()) pit->second.busy--;
  auto tit = c->tables.find(F->cfg.table_id);
  if (tit != c->tables.end()) tit->second.busy--;
}

}  // namespace

extern "C" {

int ckc_fuzz_create(ckc_ctx c, const ckc_fuzz_config* cfg, ckc_fuzz* out) {
  if (!c || !cfg || !out) return fail(CKC_E_INVALID, "NULL argument");
  const ckc_fuzz_config C = *cfg;
  if (C.batch == 0 || C.batch > 65536) return fail(CKC_E_INVALID, "batch outside 1..65536");
  if (C.max_stack == 0 || C.max_stack > 15) return fail(CKC_E_INVALID, "max_stack outside 1..15");
  if (C.max_block == 0 || C.max_block > 1024) return fail(CKC_E_INVALID, "max_block outside 1..1024");
  if (C.corpus_cap == 0 || C.corpus_cap > (1u << 20)) return fail(CKC_E_INVALID, "corpus_cap outside 1..2^20");
  if (C.mode > CKC_REP_BOUNDARY) return fail(CKC_E_INVALID, "campaign mode must be FULL, REP_CORNERS or REP_BOUNDARY");
  if (C.flags & ~(uint32_t)CKC_TRIPWIRE) return fail(CKC_E_INVALID, "campaign flags: CKC_TRIPWIRE only");
  if (C.ops & ~(uint32_t)(CKC_MUT_LAUNCH | CKC_MUT_SCALAR | CKC_MUT_DATA))
    return fail(CKC_E_INVALID, "unknown mutation operators");
  auto pit = c->progs.find(C.prog_id);
  if (pit == c->progs.end()) return fail(CKC_E_INVALID, "unknown program");
  auto tit = c->tables.find(C.table_id);
  if (tit == c->tables.end()) return fail(CKC_E_INVALID, "unknown table");
  const rt::Program& P = pit->second;
  const rt::Table& T = tit->second;
  const dprog* h = (const dprog*)P.L.blob.data();
  // the seed validated as a one-input batch
  ckc_batch B;
  std::memset(&B, 0, sizeof B);
  B.prog_id = C.prog_id;
  B.n_inputs = 1;
  B.launch = C.launch;
  B.scalars = C.scalars;
  B.table_ids = &C.table_id;
  B.mode = C.mode;
  B.flags = C.flags;
  B.loop_cap_log2[0] = C.loop_cap_log2[0];
  B.loop_cap_log2[1] = C.loop_cap_log2[1];
  int rc = rt::validate_desc(c, B, 0, false, nullptr);
  if (rc != CKC_OK) return rc;
  const uint64_t bs = (uint64_t)C.launch[3] * C.launch[4] * C.launch[5];
  const uint64_t nb = (uint64_t)C.launch[0] * C.launch[1] * C.launch[2];
  if (bs > C.max_block || nb * bs > C.max_threads || nb * bs == 0)
    return fail(CKC_E_INVALID, "the seed input is empty or outside max_block / max_threads");
  uint32_t c0 = C.loop_cap_log2[0], c1 = C.loop_cap_log2[1];
  if (c0 == 0 && c1 == 0) { c0 = 20; c1 = 12; }
  const unsigned L1 = h->max_depth >= 1 ? c0 : 0, L2 = h->max_depth >= 2 ? c1 : 0;
  if (C.max_threads > 1 && rt::index_bits(C.max_threads) + L1 + L2 > 64)
    return fail(CKC_E_RANGE, "first-violation keys of max_threads threads need more than 64 bits");
  uint64_t n_elems = 0;
  if (C.data_slot != CKC_FUZZ_NO_SLOT) {
    if (C.data_slot >= T.host.size()) return fail(CKC_E_INVALID, "data slot outside the table");
    const ckc_alloc& A = T.host[C.data_slot];
    if (!A.data || A.size_bytes < 4) return fail(CKC_E_INVALID, "data slot without data");
    n_elems = A.size_bytes / 4;
  }
  int e0 = (int)hipSetDevice(c->dev);
  if (e0 != hipSuccess) return fail(CKC_E_HIP, "hipSetDevice");
  ckc_fuzz F = new (std::nothrow) ckc_fuzz_s;
  if (!F) return fail(CKC_E_NOMEM, "campaign");
  F->c = c;
  F->cfg = C;
  F->n_acc = h->n_accesses;
  F->J.stream = c->stream;
  auto bail = [&](int code) {
    for (void* p : F->own) (void)hipFree(p);
    rt::release_job(c, F->J);
    delete F;
    return code;
  };
  FzArgs& f = F->f;
  const uint32_t Bn = C.batch;
  ckc_alloc* tabs = nullptr;
  if ((rc = own_alloc(F, &tabs, (size_t)Bn * MAX_SLOTS)) || (rc = own_alloc(F, &f.child_data, Bn * std::max<uint64_t>(n_elems, 1))) ||
      (rc = own_alloc(F, &f.c_launch, (size_t)C.corpus_cap * 6)) ||
      (rc = own_alloc(F, &f.c_scalars, (size_t)C.corpus_cap * MAX_SCALARS)) ||
      (rc = own_alloc(F, &f.c_data, (size_t)C.corpus_cap * std::max<uint64_t>(n_elems, 1))) ||
      (rc = own_alloc(F, &f.c_gen, C.corpus_cap)) || (rc = own_alloc(F, &f.virgin, 65536)) ||
      (rc = own_alloc(F, &f.seen, 65536 / 4)) || (rc = own_alloc(F, &f.sigs, (size_t)std::max(F->n_acc, 1u) * 4)) ||
      (rc = own_alloc(F, &f.novel, Bn)) || (rc = own_alloc(F, &f.pos, Bn)) || (rc = own_alloc(F, &f.st, 1)))
    return bail(rc);
  // one table per child: the seed's, with the data slot pointing at the
  // child's own elements
  std::vector<ckc_alloc> ht((size_t)Bn * MAX_SLOTS);
  for (uint32_t k = 0; k < Bn; k++)
    for (uint32_t s = 0; s < (uint32_t)MAX_SLOTS; s++) {
      ckc_alloc A = s < T.host.size() ? T.host[s] : ckc_alloc{0, 0, nullptr, 0, 0};
      if (n_elems && s == C.data_slot) A.data = f.child_data + n_elems * k;
      ht[(size_t)k * MAX_SLOTS + s] = A;
    }
  // the children's job: batch inputs of at most max_threads threads each
  rt::Stage S;
  S.reserve(Bn);
  const bool tripwire = (C.flags & CKC_TRIPWIRE) != 0;
  const uint64_t lanes_max = C.mode == CKC_REP_CORNERS ? std::min<uint64_t>(C.max_threads, 64) : C.max_threads;
  for (uint32_t k = 0; k < Bn; k++) {
    dinput d = rt::make_input(P, T, B, 0);
    d.table = (uint64_t)(uintptr_t)(tabs + (size_t)k * MAX_SLOTS);
    d.mode = C.mode;
    d.detector = tripwire ? 1u : 0u;
    S.add(h, d, C.scalars, lanes_max, tripwire);
    S.note_blockwise(h, T.host.data(), (uint32_t)T.host.size(), d.launch);
  }
  F->capture = S.capture;
  if ((rc = rt::stage_new_job(c, F->J, S, false, F->a, F->eg))) return bail(rc);
  F->n_records = S.n_records;
  f.in = F->a.inputs;
  f.sc = const_cast<int64_t*>(F->a.scalars);
  f.recs = F->a.recs;
  f.counts = F->a.counts;
  f.batch = Bn;
  f.n_scalars = h->n_scalars;
  f.max_stack = C.max_stack;
  f.max_block = C.max_block;
  f.cap = C.corpus_cap;
  f.ops = C.ops;
  f.max_threads = C.max_threads;
  f.seed = C.seed;
  f.n_elems = n_elems;
  // corpus = the seed; every bucket virgin; no signature yet
  int64_t sc16[MAX_SCALARS] = {0};
  for (uint32_t s = 0; s < h->n_scalars; s++) sc16[s] = C.scalars[s];
  FzState st0;
  std::memset(&st0, 0, sizeof st0);
  st0.size = 1;
  const uint32_t g0 = 0;
  hipStream_t s = c->stream;
  hipError_t e = hipMemcpyAsync(tabs, ht.data(), sizeof(ckc_alloc) * ht.size(), hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipMemcpyAsync(f.c_launch, C.launch, 6 * sizeof(uint32_t), hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipMemcpyAsync(f.c_scalars, sc16, sizeof sc16, hipMemcpyHostToDevice, s);
  if (e == hipSuccess && n_elems)
    e = hipMemcpyAsync(f.c_data, T.host[C.data_slot].data, n_elems * 4, hipMemcpyDeviceToDevice, s);
  if (e == hipSuccess) e = hipMemcpyAsync(f.c_gen, &g0, sizeof g0, hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipMemcpyAsync(f.st, &st0, sizeof st0, hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipMemsetAsync(f.virgin, 0xFF, 65536, s);
  if (e == hipSuccess) e = hipMemsetAsync(f.seen, 0, 65536, s);
  if (e == hipSuccess) e = hipMemsetAsync(f.sigs, 0xFF, sizeof(unsigned long long) * std::max(F->n_acc, 1u) * 4, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);  // the host arrays above are locals
  if (e != hipSuccess) return bail(fail(CKC_E_HIP, std::string("campaign set-up: ") + hipGetErrorString(e)));
  c->progs[C.prog_id].busy++;
  c->tables[C.table_id].busy++;
  *out = F;
  return CKC_OK;
}

int ckc_fuzz_run(ckc_fuzz F, uint32_t generations) {
  if (!F) return fail(CKC_E_INVALID, "NULL campaign");
  if (F->gen + generations > 0xFFFFFFFFull) return fail(CKC_E_RANGE, "more than 2^32 generations");
  if (hipSetDevice(F->c->dev) != hipSuccess) return fail(CKC_E_HIP, "hipSetDevice");
  const hipStream_t s = F->c->stream;
  for (uint32_t k = 0; k < generations; k++) {
    const uint64_t g = F->gen;
    hipError_t e = launch_fuzz_mutate(F->f, g, s);
    if (e == hipSuccess) e = rt::run_evaluation(F->a, F->eg, s);
    if (e == hipSuccess && F->capture) e = launch_capture(F->a, F->eg, s);
    if (e == hipSuccess) e = launch_fixup(F->a, F->n_records, s);
    if (e == hipSuccess) e = launch_finish(F->a, s);
    if (e == hipSuccess) e = launch_fuzz_update(F->f, g, s);
    if (e != hipSuccess) return fail(CKC_E_HIP, std::string("generation launch: ") + hipGetErrorString(e));
    F->gen++;
  }
  return CKC_OK;
}

int ckc_fuzz_get_stats(ckc_fuzz F, ckc_fuzz_stats* out) {
  if (!F || !out) return fail(CKC_E_INVALID, "NULL argument");
  if (hipSetDevice(F->c->dev) != hipSuccess) return fail(CKC_E_HIP, "hipSetDevice");
  FzState st;
  std::vector<uint8_t> v(65536);
  hipError_t e = hipMemcpyAsync(&st, F->f.st, sizeof st, hipMemcpyDeviceToHost, F->c->stream);
  if (e == hipSuccess) e = hipMemcpyAsync(v.data(), F->f.virgin, 65536, hipMemcpyDeviceToHost, F->c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(F->c->stream);
  if (e != hipSuccess) return fail(CKC_E_HIP, std::string("campaign stats: ") + hipGetErrorString(e));
  uint64_t bits = 0;
  for (uint8_t b : v) bits += (uint64_t)__builtin_popcount((uint8_t)~b);
  out->generations = st.generations;
  out->execs = st.execs;
  out->novel = st.novel;
  out->crashes = st.crashes;
  out->corpus = st.size;
  out->map_bits = bits;
  return CKC_OK;
}

int ckc_fuzz_read(ckc_fuzz F, uint32_t* launch, int64_t* scalars, int32_t* data, uint32_t* gen, uint8_t* virgin,
                  uint64_t* sigs) {
  if (!F) return fail(CKC_E_INVALID, "NULL campaign");
  if (hipSetDevice(F->c->dev) != hipSuccess) return fail(CKC_E_HIP, "hipSetDevice");
  const hipStream_t s = F->c->stream;
  const size_t cap = F->cfg.corpus_cap;
  const auto D2H = hipMemcpyDeviceToHost;
  hipError_t e = hipSuccess;
  if (launch) e = hipMemcpyAsync(launch, F->f.c_launch, cap * 6 * sizeof(uint32_t), D2H, s);
  if (e == hipSuccess && scalars) e = hipMemcpyAsync(scalars, F->f.c_scalars, cap * MAX_SCALARS * 8, D2H, s);
  if (e == hipSuccess && data && F->f.n_elems)
    e = hipMemcpyAsync(data, F->f.c_data, cap * F->f.n_elems * 4, D2H, s);
  if (e == hipSuccess && gen) e = hipMemcpyAsync(gen, F->f.c_gen, cap * 4, D2H, s);
  if (e == hipSuccess && virgin) e = hipMemcpyAsync(virgin, F->f.virgin, 65536, D2H, s);
  if (e == hipSuccess && sigs && F->n_acc) e = hipMemcpyAsync(sigs, F->f.sigs, (size_t)F->n_acc * 4 * 8, D2H, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return fail(CKC_E_HIP, std::string("campaign read: ") + hipGetErrorString(e));
  return CKC_OK;
}

void ckc_fuzz_destroy(ckc_fuzz F) {
  if (!F) return;
  release(F);
  delete F;
}

}  // extern "C"
