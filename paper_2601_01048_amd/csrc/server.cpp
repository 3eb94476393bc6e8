// server.cpp — the serving form of libckc (include/ckc.h, ckc_server_*): a
// worker thread admits check jobs in arrival order under a device working-set
// cap and runs them as batched checks on several streams, so that batches
// overlap on the device and jobs that arrive meanwhile join the next batch
// (continuous batching).  Host code only; each batch is one ckc_check_batch.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <mutex>
#include <new>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "../../include/ckc.h"
#include "runtime.h"

namespace {

uint64_t now_ns() {
  return (uint64_t)std::chrono::duration_cast<std::chrono::nanoseconds>(
             std::chrono::steady_clock::now().time_since_epoch())
      .count();
}

struct SJob {
  ckc_batch desc;
  std::vector<uint32_t> launch, tids;
  std::vector<int64_t> scalars;
  uint32_t n_acc = 0;
  ckc_job_stats st{};
  bool done = false;
  std::vector<ckc_record> recs;
  std::vector<uint8_t> maps;
  std::vector<ckc_input_status> status;
};

struct Slot {
  hipStream_t stream = nullptr;
  bool busy = false;
  uint64_t job = 0;                 // library job of the running batch
  hipEvent_t done = nullptr;
  std::vector<uint64_t> tickets;    // jobs of the batch, in input order
  uint64_t bytes = 0;
};

}  // namespace

struct ckc_server_s {
  ckc_ctx c = nullptr;
  ckc_server_config cfg{};
  std::thread worker;
  std::mutex ctx_mu;                // every use of the context
  std::mutex mu;                    // queues, jobs, counters
  std::condition_variable cv_work;  // submissions, shutdown
  std::condition_variable cv_done;  // completions
  std::deque<uint64_t> pending;
  std::unordered_map<uint64_t, SJob> jobs;
  std::vector<Slot> slots;
  uint64_t next_ticket = 1;
  uint64_t inflight_bytes = 0, inflight_jobs = 0;
  bool stop = false;
  ckc_server_stats stats{};
};

namespace {

// Copies a finished batch's results into its jobs (called with ctx_mu held).
void finish_slot(ckc_server s, Slot& sl) {
  uint64_t n_in = 0, n_rec = 0;
  int rc = ckc_job_sizes(s->c, sl.job, &n_in, &n_rec);
  std::vector<ckc_record> recs(rc == CKC_OK ? n_rec : 0);
  std::vector<ckc_input_status> st(rc == CKC_OK ? n_in : 0);
  bool want_maps = false;
  {
    std::lock_guard<std::mutex> g(s->mu);
    for (uint64_t t : sl.tickets) want_maps |= (s->jobs[t].desc.flags & CKC_DENSE_MAP) != 0;
  }
  std::vector<uint8_t> maps(rc == CKC_OK && want_maps ? n_in * 65536 : 0);
  if (rc == CKC_OK)
    rc = ckc_read_results(s->c, sl.job, recs.data(), want_maps ? maps.data() : nullptr, st.data(), CKC_WAIT);
  const uint64_t t_done = now_ns();
  std::lock_guard<std::mutex> g(s->mu);
  uint64_t in_off = 0, rec_off = 0;
  for (uint64_t t : sl.tickets) {
    SJob& J = s->jobs[t];
    const uint32_t n = J.desc.n_inputs;
    if (rc == CKC_OK) {
      J.recs.assign(recs.begin() + rec_off, recs.begin() + rec_off + (uint64_t)n * J.n_acc);
      J.status.assign(st.begin() + in_off, st.begin() + in_off + n);
      if (J.desc.flags & CKC_DENSE_MAP)
        J.maps.assign(maps.begin() + in_off * 65536, maps.begin() + (in_off + n) * 65536);
    }
    in_off += n;
    rec_off += (uint64_t)n * J.n_acc;
    J.st.t_done_ns = t_done;
    J.st.status = rc;
    J.done = true;
    s->stats.completed++;
  }
  s->inflight_bytes -= sl.bytes;
  s->inflight_jobs -= sl.tickets.size();
  sl.busy = false;
  sl.tickets.clear();
  sl.bytes = 0;
  s->cv_done.notify_all();
}

// Takes jobs from the head of the queue while they fit; launches them as one
// batch on slot sl.  Returns true if anything happened.
bool admit(ckc_server s, Slot& sl) {
  std::vector<uint64_t> take;
  uint64_t bytes = 0;
  {
    std::lock_guard<std::mutex> g(s->mu);
    while (!s->pending.empty() && take.size() < s->cfg.max_batch_jobs) {
      const uint64_t t = s->pending.front();
      SJob& J = s->jobs[t];
      if (J.st.ws_bytes > s->cfg.hbm_cap_bytes) {  // can never be admitted
        s->pending.pop_front();
        J.st.t_admit_ns = J.st.t_done_ns = now_ns();
        J.st.status = CKC_E_NOMEM;
        J.done = true;
        s->stats.rejected++;
        s->stats.completed++;
        s->cv_done.notify_all();
        continue;
      }
      if (s->inflight_bytes + bytes + J.st.ws_bytes > s->cfg.hbm_cap_bytes) break;
      bytes += J.st.ws_bytes;
      take.push_back(t);
      s->pending.pop_front();
    }
    if (take.empty()) return false;
    s->inflight_bytes += bytes;
    s->inflight_jobs += take.size();
    s->stats.max_inflight_bytes = std::max(s->stats.max_inflight_bytes, s->inflight_bytes);
    s->stats.max_inflight_jobs = std::max(s->stats.max_inflight_jobs, s->inflight_jobs);
    s->stats.batches++;
  }
  std::vector<ckc_batch> descs;
  descs.reserve(take.size());
  {
    std::lock_guard<std::mutex> g(s->mu);
    for (uint64_t t : take) descs.push_back(s->jobs[t].desc);
  }
  ckc_launch_opts O = s->cfg.opts;
  O.hip_stream = sl.stream;
  uint64_t job = 0;
  const uint64_t t_admit = now_ns();
  int rc = ckc_check_batch(s->c, descs.data(), (uint32_t)descs.size(), &O, &job);
  sl.tickets = take;
  sl.bytes = bytes;
  {
    std::lock_guard<std::mutex> g(s->mu);
    for (uint64_t t : take) {
      s->jobs[t].st.t_admit_ns = t_admit;
      s->jobs[t].st.batch_jobs = (uint32_t)take.size();
    }
  }
  if (rc != CKC_OK) {  // the whole batch ends with the launch error
    std::lock_guard<std::mutex> g(s->mu);
    for (uint64_t t : take) {
      SJob& J = s->jobs[t];
      J.st.t_done_ns = now_ns();
      J.st.status = rc;
      J.done = true;
      s->stats.completed++;
    }
    s->inflight_bytes -= bytes;
    s->inflight_jobs -= take.size();
    sl.tickets.clear();
    sl.bytes = 0;
    s->cv_done.notify_all();
    return true;
  }
  sl.busy = true;
  sl.job = job;
  sl.done = ckc::rt::job_done_event(s->c, job);
  return true;
}

void worker_main(ckc_server s) {
  (void)hipSetDevice(s->c->dev);
  for (;;) {
    bool progress = false, busy = false;
    {
      std::lock_guard<std::mutex> g(s->ctx_mu);
      for (Slot& sl : s->slots) {
        if (!sl.busy) continue;
        if (hipEventQuery(sl.done) == hipErrorNotReady) {
          busy = true;
          continue;
        }
        finish_slot(s, sl);
        progress = true;
      }
      // with nothing in flight the queue head is always admitted or rejected
      for (Slot& sl : s->slots) {
        if (sl.busy) continue;
        if (!admit(s, sl)) break;
        progress = true;
        busy |= sl.busy;
      }
    }
    std::unique_lock<std::mutex> lk(s->mu);
    if (progress) continue;
    if (s->stop && s->pending.empty() && !busy) return;
    if (busy)  // poll for completions; a submission wakes the worker early
      s->cv_work.wait_for(lk, std::chrono::microseconds(20));
    else
      s->cv_work.wait(lk, [&] { return !s->pending.empty() || s->stop; });
  }
}

}  // namespace

extern "C" {

int ckc_server_create(ckc_ctx c, const ckc_server_config* cfg, ckc_server* out) {
  if (!c || !out) return ckc::rt::fail(CKC_E_INVALID, "NULL argument");
  ckc_server_config C;
  std::memset(&C, 0, sizeof C);
  if (cfg) C = *cfg;
  if (C.n_streams == 0) C.n_streams = 4;
  if (C.max_batch_jobs == 0) C.max_batch_jobs = 1024;
  if (C.hbm_cap_bytes == 0) C.hbm_cap_bytes = 64ull * 1000 * 1000 * 1000;
  if (C.n_streams > 16) return ckc::rt::fail(CKC_E_INVALID, "n_streams above 16");
  if (C.max_batch_jobs > 65536) return ckc::rt::fail(CKC_E_INVALID, "max_batch_jobs above 65536");
  ckc_server s = new (std::nothrow) ckc_server_s;
  if (!s) return ckc::rt::fail(CKC_E_NOMEM, "server");
  s->c = c;
  s->cfg = C;
  s->slots.resize(C.n_streams);
  hipError_t e = hipSetDevice(c->dev);
  for (Slot& sl : s->slots)
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking);
  if (e != hipSuccess) {
    for (Slot& sl : s->slots)
      if (sl.stream) (void)hipStreamDestroy(sl.stream);
    delete s;
    return ckc::rt::fail(CKC_E_HIP, std::string("server streams: ") + hipGetErrorString(e));
  }
  try {
    s->worker = std::thread(worker_main, s);
  } catch (...) {
    for (Slot& sl : s->slots) (void)hipStreamDestroy(sl.stream);
    delete s;
    return ckc::rt::fail(CKC_E_INVALID, "cannot start the worker thread");
  }
  *out = s;
  return CKC_OK;
}

void ckc_server_destroy(ckc_server s) {
  if (!s) return;
  {
    std::lock_guard<std::mutex> g(s->mu);
    s->stop = true;
  }
  s->cv_work.notify_all();
  if (s->worker.joinable()) s->worker.join();
  (void)hipSetDevice(s->c->dev);
  for (Slot& sl : s->slots)
    if (sl.stream) (void)hipStreamDestroy(sl.stream);
  delete s;
}

int ckc_server_submit(ckc_server s, const ckc_batch* desc, uint64_t arrival_ns, uint64_t* ticket) {
  if (!s || !desc || !ticket) return ckc::rt::fail(CKC_E_INVALID, "NULL argument");
  if (desc->n_inputs == 0) return ckc::rt::fail(CKC_E_INVALID, "no inputs");
  // the sweep decides its rounds on the host between windows, which would
  // hold the worker: served jobs use the other thread sets
  if (desc->mode == CKC_REP_PREX) return ckc::rt::fail(CKC_E_INVALID, "CKC_REP_PREX jobs are not served");
  SJob J;
  uint64_t ws = 0;
  {
    std::lock_guard<std::mutex> g(s->ctx_mu);
    int rc = ckc::rt::validate_desc(s->c, *desc, 0, s->cfg.opts.force_generic != 0, &ws);
    if (rc != CKC_OK) return rc;
    J.n_acc = s->c->progs.find(desc->prog_id)->second.L.info.n_accesses;
  }
  const uint32_t n = desc->n_inputs;
  J.desc = *desc;
  J.launch.assign(desc->launch, desc->launch + 6 * (size_t)n);
  J.tids.assign(desc->table_ids, desc->table_ids + n);
  uint32_t n_sc = 0;
  {
    std::lock_guard<std::mutex> g(s->ctx_mu);
    n_sc = ((const ckc::dprog*)s->c->progs.find(desc->prog_id)->second.L.blob.data())->n_scalars;
  }
  if (n_sc) J.scalars.assign(desc->scalars, desc->scalars + (size_t)n * n_sc);
  J.desc.launch = J.launch.data();
  J.desc.table_ids = J.tids.data();
  J.desc.scalars = n_sc ? J.scalars.data() : nullptr;
  J.st.t_arrival_ns = arrival_ns ? arrival_ns : now_ns();
  J.st.ws_bytes = ws;
  {
    std::lock_guard<std::mutex> g(s->mu);
    const uint64_t t = s->next_ticket++;
    auto it = s->jobs.emplace(t, std::move(J)).first;
    SJob& K = it->second;  // re-point the descriptor at the moved vectors
    K.desc.launch = K.launch.data();
    K.desc.table_ids = K.tids.data();
    K.desc.scalars = n_sc ? K.scalars.data() : nullptr;
    s->pending.push_back(t);
    s->stats.submitted++;
    *ticket = t;
  }
  s->cv_work.notify_one();
  return CKC_OK;
}

int ckc_server_result(ckc_server s, uint64_t ticket, ckc_record* recs, uint8_t* maps, ckc_input_status* st,
                      ckc_job_stats* stats, uint32_t flags) {
  if (!s) return ckc::rt::fail(CKC_E_INVALID, "NULL server");
  std::unique_lock<std::mutex> lk(s->mu);
  auto it = s->jobs.find(ticket);
  if (it == s->jobs.end()) return ckc::rt::fail(CKC_E_INVALID, "unknown ticket");
  if (!it->second.done) {
    if (!(flags & CKC_WAIT)) return CKC_NOT_READY;
    s->cv_done.wait(lk, [&] { return it->second.done; });
  }
  SJob& J = it->second;
  if (maps && !(J.desc.flags & CKC_DENSE_MAP) && J.st.status == CKC_OK)
    return ckc::rt::fail(CKC_E_INVALID, "maps requested but the job was submitted without CKC_DENSE_MAP");
  if (stats) *stats = J.st;
  const int status = J.st.status;
  if (status == CKC_OK) {
    if (recs && !J.recs.empty()) std::memcpy(recs, J.recs.data(), J.recs.size() * sizeof(ckc_record));
    if (st) std::memcpy(st, J.status.data(), J.status.size() * sizeof(ckc_input_status));
    if (maps) std::memcpy(maps, J.maps.data(), J.maps.size());
  }
  s->jobs.erase(it);
  if (status != CKC_OK && status != CKC_E_NOMEM)
    return ckc::rt::fail(status, "job failed at launch or readback");
  if (status == CKC_E_NOMEM) return ckc::rt::fail(status, "job's working set exceeds the admission cap");
  return CKC_OK;
}

int ckc_server_get_stats(ckc_server s, ckc_server_stats* out) {
  if (!s || !out) return ckc::rt::fail(CKC_E_INVALID, "NULL argument");
  std::lock_guard<std::mutex> g(s->mu);
  *out = s->stats;
  return CKC_OK;
}

}  // extern "C"
