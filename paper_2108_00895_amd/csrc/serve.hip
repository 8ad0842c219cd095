// Request server of libskm: continuous batching of assign-new-rows requests
// against one resident context, and small clustering jobs run beside them
// (declared in include/skm.h).
//
// Requests.  Client threads submit host CSR requests; a worker thread owns
// n_slots batch slots, each a HIP stream with pinned staging buffers and device
// buffers sized for slot_rows rows and slot_nnz non-zeros.  Whenever a slot is
// free the worker packs the requests at the head of the queue into it (in
// arrival order, as many as fit its rows and non-zeros), copies them in on the
// slot's stream, runs the exact new-row pipeline (low-precision scoring +
// certification + FP64 tier + FP64 scores) and copies the answers back; a
// completed slot's answers are stored in the requests themselves and their
// waiters are woken.  Different slots run on different streams, so batches
// overlap on the device.  With use_graphs, each slot's compute pipeline is
// captured once into a HIP graph sized for the slot's capacity; a batch then
// costs the copies plus one graph launch, and the kernels read the batch's row
// count from the device.
//
// Jobs.  A clustering job (rows, a configuration) waits in a queue until the
// server's memory budget, less the slots, holds its estimated device memory
// (skm_context_bytes); a job thread then builds its context (own stream) and
// runs the admitted jobs round robin, one iteration (assign, stop test, update,
// stop test) per turn, so that jobs of any size share the device with each
// other and with the request batches.  A finished job's assignment (and, when
// asked for, its FP64 centroids) is copied into the job and its context freed,
// which admits the next job.
//
// Answers are copied into the caller's buffers by skm_server_wait itself, so
// nothing is written to them after a time-out or a cancellation.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "host_checks.h"
#include "internal.h"

using namespace skm;

namespace {

using Clock = std::chrono::steady_clock;

struct Request {
  int64_t id = 0;
  bool is_job = false;
  int64_t n_rows = 0, nnz = 0, n_cols = 0;
  std::vector<int64_t> indptr;
  std::vector<int32_t> indices;
  std::vector<float> values;
  // caller's buffers, written only by skm_server_wait
  int32_t *out_a = nullptr;
  double *out_s = nullptr;           // request: scores; job: centroids (may be null)
  skm_job_info *out_info = nullptr;  // job only (may be null)
  // answers, owned by the request until the wait copies them out
  std::vector<int32_t> res_a;
  std::vector<double> res_s;
  // job
  skm_config cfg{};
  std::vector<int32_t> init_rows;
  size_t need = 0;                   // admitted device bytes
  skm_ctx *ctx = nullptr;
  skm_job_info info{};
  Clock::time_point t_submit;
  bool done = false;
  bool cancelled = false;
  int waiters = 0;
  skm_status status = SKM_OK;
};

struct Slot {
  hipStream_t stream = nullptr;
  hipEvent_t done_ev = nullptr;
  int64_t *h_indptr = nullptr;
  int32_t *h_indices = nullptr;
  float *h_values = nullptr;
  int32_t *h_a = nullptr;
  double *h_s = nullptr;
  NewRows d{};
  int64_t *d_indptr = nullptr;
  int32_t *d_indices = nullptr;
  float *d_values = nullptr;
  double *d_xl1 = nullptr;
  int64_t *h_n = nullptr;            // rows of the current batch (pinned)
  int64_t *d_n = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  std::vector<std::shared_ptr<Request>> reqs;
  int64_t rows = 0;
  bool busy = false;
};

size_t slot_device_bytes(const skm_ctx *c, int64_t rows, int64_t nnz) {
  const int64_t nch = (c->k + kChunk - 1) / kChunk;
  return (size_t)(rows + 1) * 8 + (size_t)nnz * 8 + (size_t)rows * 8 /*xl1*/ +
         (size_t)nch * rows * sizeof(Partial) + (size_t)rows * (4 + 8 + 8 + 4 + 8 + 1 + 8) + 32 + 128;
}

// The CSR conventions of skm.h on a host copy (host_checks.cpp; the
// certificate of the low-precision scores assumes positive values and
// ascending terms).
skm_status check_host_rows(const std::vector<int64_t> &ip, const std::vector<int32_t> &ix,
                           const std::vector<float> &v, int64_t n, int64_t z, int64_t D) {
  std::string why;
  if (!host::rows_ok(ip.data(), ix.data(), v.data(), n, z, D, &why))
    return set_error(SKM_E_INVALID, why);
  return SKM_OK;
}

}  // namespace

struct skm_server {
  skm_ctx *c = nullptr;
  skm_server_config cfg{};
  std::vector<Slot> slots;
  std::vector<void *> dev_allocs, host_allocs;
  size_t hbm = 0;                    // slots
  size_t job_hbm = 0;                // admitted jobs
  std::mutex mu;
  std::condition_variable cv_work, cv_done, cv_jobs;
  std::deque<std::shared_ptr<Request>> queue;
  std::deque<std::shared_ptr<Request>> job_queue;
  std::vector<std::shared_ptr<Request>> running;
  std::unordered_map<int64_t, std::shared_ptr<Request>> live;
  int64_t next_id = 1;
  bool stopping = false;
  int n_waiters = 0;                 // threads inside skm_server_wait
  std::thread worker, job_worker;
  // statistics
  std::vector<double> lat_ms;
  int64_t rows_done = 0, batches = 0;
  int64_t jobs_done = 0, job_iterations = 0;
  int32_t max_depth = 0;
  bool any_submit = false;
  Clock::time_point t_first, t_last;
  hipError_t dev_error = hipSuccess;
};

namespace {

template <typename T>
bool dev_alloc(skm_server *s, T **p, size_t count) {
  void *q = nullptr;
  const size_t bytes = std::max<size_t>(count * sizeof(T), 1);
  if (hipMalloc(&q, bytes) != hipSuccess) {
    (void)hipGetLastError();
    return false;
  }
  s->dev_allocs.push_back(q);
  s->hbm += bytes;
  *p = static_cast<T *>(q);
  return true;
}

template <typename T>
bool host_alloc(skm_server *s, T **p, size_t count) {
  void *q = nullptr;
  if (hipHostMalloc(&q, std::max<size_t>(count * sizeof(T), 1), hipHostMallocDefault) != hipSuccess) {
    (void)hipGetLastError();
    return false;
  }
  s->host_allocs.push_back(q);
  *p = static_cast<T *>(q);
  return true;
}

void release(skm_server *s) {
  for (Slot &sl : s->slots) {
    if (sl.stream) (void)hipStreamSynchronize(sl.stream);
    if (sl.exec) (void)hipGraphExecDestroy(sl.exec);
    if (sl.graph) (void)hipGraphDestroy(sl.graph);
    if (sl.done_ev) (void)hipEventDestroy(sl.done_ev);
    if (sl.stream) (void)hipStreamDestroy(sl.stream);
  }
  for (void *p : s->dev_allocs) (void)hipFree(p);
  for (void *p : s->host_allocs) (void)hipHostFree(p);
  (void)hipGetLastError();
}

bool make_slot(skm_server *s, Slot &sl) {
  const int64_t R = s->cfg.slot_rows, Z = s->cfg.slot_nnz;
  const int64_t nch = (s->c->k + kChunk - 1) / kChunk;
  if (hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking) != hipSuccess) return false;
  if (hipEventCreateWithFlags(&sl.done_ev, hipEventDisableTiming) != hipSuccess) return false;
  bool ok = host_alloc(s, &sl.h_indptr, R + 1) && host_alloc(s, &sl.h_indices, Z) &&
            host_alloc(s, &sl.h_values, Z) && host_alloc(s, &sl.h_a, R) && host_alloc(s, &sl.h_s, R);
  ok = ok && dev_alloc(s, &sl.d_indptr, R + 1) && dev_alloc(s, &sl.d_indices, Z) &&
       dev_alloc(s, &sl.d_values, Z) && dev_alloc(s, &sl.d_xl1, R) &&
       dev_alloc(s, &sl.d.part, (size_t)(nch * R)) && dev_alloc(s, &sl.d.a, R) &&
       dev_alloc(s, &sl.d.lo, R) && dev_alloc(s, &sl.d.hi, R) && dev_alloc(s, &sl.d.flag_rows, R) &&
       dev_alloc(s, &sl.d.flag_L, R) && dev_alloc(s, &sl.d.flag_mode, R) &&
       dev_alloc(s, &sl.d.counters, 8) && dev_alloc(s, &sl.d.stat, 16) &&
       dev_alloc(s, &sl.d.score, R) && host_alloc(s, &sl.h_n, 1) && dev_alloc(s, &sl.d_n, 1);
  sl.d.indptr = sl.d_indptr;
  sl.d.indices = sl.d_indices;
  sl.d.values = sl.d_values;
  sl.d.xl1 = sl.d_xl1;
  if (!ok || !s->cfg.use_graphs) return ok;
  // capture the compute pipeline for R rows of capacity; the row count is read
  // from d_n, which each batch copies in before the replay
  hipStream_t st = sl.stream;
  if (hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal) != hipSuccess) return false;
  hipError_t e = launch_row_stats_only(sl.d_indptr, sl.d_indices, sl.d_values, R, sl.d_xl1, st, sl.d_n);
  if (e == hipSuccess) e = launch_new_rows(s->c, sl.d, R, st, sl.d_n);
  const hipError_t e2 = hipStreamEndCapture(st, &sl.graph);
  if (e != hipSuccess || e2 != hipSuccess) {
    (void)hipGetLastError();
    return false;
  }
  if (hipGraphInstantiate(&sl.exec, sl.graph, nullptr, nullptr, 0) != hipSuccess) {
    (void)hipGetLastError();
    return false;
  }
  return true;
}

// Packs the requests at the head of the queue into a free slot and launches
// it.  Called with the lock held; the host copies are made under the lock
// (they are memcpys of already-validated host arrays).
void launch_slot(skm_server *s, Slot &sl) {
  int64_t rows = 0, nnz = 0;
  sl.reqs.clear();
  sl.h_indptr[0] = 0;
  while (!s->queue.empty()) {
    const auto &r = s->queue.front();
    if (rows + r->n_rows > s->cfg.slot_rows || nnz + r->nnz > s->cfg.slot_nnz) break;
    std::memcpy(sl.h_indices + nnz, r->indices.data(), sizeof(int32_t) * r->nnz);
    std::memcpy(sl.h_values + nnz, r->values.data(), sizeof(float) * r->nnz);
    for (int64_t i = 0; i < r->n_rows; ++i) sl.h_indptr[rows + i + 1] = nnz + r->indptr[i + 1];
    rows += r->n_rows;
    nnz += r->nnz;
    sl.reqs.push_back(r);
    s->queue.pop_front();
  }
  sl.rows = rows;
  hipStream_t st = sl.stream;
  hipError_t e = hipMemcpyAsync(sl.d_indptr, sl.h_indptr, 8 * (rows + 1), hipMemcpyHostToDevice, st);
  if (e == hipSuccess && nnz > 0)
    e = hipMemcpyAsync(sl.d_indices, sl.h_indices, 4 * nnz, hipMemcpyHostToDevice, st);
  if (e == hipSuccess && nnz > 0)
    e = hipMemcpyAsync(sl.d_values, sl.h_values, 4 * nnz, hipMemcpyHostToDevice, st);
  if (sl.exec) {
    *sl.h_n = rows;
    if (e == hipSuccess) e = hipMemcpyAsync(sl.d_n, sl.h_n, 8, hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipGraphLaunch(sl.exec, st);
  } else {
    if (e == hipSuccess)
      e = launch_row_stats_only(sl.d_indptr, sl.d_indices, sl.d_values, rows, sl.d_xl1, st);
    if (e == hipSuccess) e = launch_new_rows(s->c, sl.d, rows, st);
  }
  if (e == hipSuccess) e = hipMemcpyAsync(sl.h_a, sl.d.a, 4 * rows, hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipMemcpyAsync(sl.h_s, sl.d.score, 8 * rows, hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipEventRecord(sl.done_ev, st);
  if (e != hipSuccess) s->dev_error = e;
  sl.busy = true;
  s->batches += 1;
}

// A cancelled request keeps only its ticket (for the wait that reports the
// cancellation): its rows and answers are released.
void drop_payload(skm_server *, const std::shared_ptr<Request> &r) {
  if (!r->cancelled) return;
  std::vector<int64_t>().swap(r->indptr);
  std::vector<int32_t>().swap(r->indices);
  std::vector<float>().swap(r->values);
  std::vector<int32_t>().swap(r->res_a);
  std::vector<double>().swap(r->res_s);
}

// Stores a finished slot's answers in its requests (lock held).
void finish_slot(skm_server *s, Slot &sl, hipError_t e) {
  int64_t row = 0;
  const auto now = Clock::now();
  for (auto &r : sl.reqs) {
    if (r->cancelled) {
      r->status = SKM_E_CANCELLED;   // answers dropped
    } else if (e == hipSuccess) {
      r->res_a.assign(sl.h_a + row, sl.h_a + row + r->n_rows);
      r->res_s.assign(sl.h_s + row, sl.h_s + row + r->n_rows);
      r->status = SKM_OK;
    } else {
      r->status = SKM_E_DEVICE;
    }
    row += r->n_rows;
    r->done = true;
    s->lat_ms.push_back(std::chrono::duration<double, std::milli>(now - r->t_submit).count());
    s->rows_done += r->n_rows;
    drop_payload(s, r);
  }
  s->t_last = now;
  sl.reqs.clear();
  sl.busy = false;
}

void worker_loop(skm_server *s) {
  (void)hipSetDevice(s->c->device);
  std::unique_lock<std::mutex> lk(s->mu);
  Clock::time_point partial_since{};
  bool partial_waiting = false;
  for (;;) {
    bool progressed = false;
    // completions
    for (Slot &sl : s->slots) {
      if (!sl.busy) continue;
      const hipError_t q = hipEventQuery(sl.done_ev);
      if (q == hipErrorNotReady) continue;
      if (q != hipSuccess) s->dev_error = q;
      finish_slot(s, sl, s->dev_error);
      progressed = true;
    }
    if (progressed) s->cv_done.notify_all();
    // launches: fill free slots from the queue head
    int busy = 0;
    for (Slot &sl : s->slots) busy += sl.busy;
    for (Slot &sl : s->slots) {
      if (sl.busy || s->queue.empty()) continue;
      // a partly filled batch waits a little for more rows, but only while
      // nothing is running (otherwise running batches already hide the wait)
      int64_t queued_rows = 0;
      for (auto &r : s->queue) queued_rows += r->n_rows;
      const bool full = queued_rows >= s->cfg.slot_rows;
      if (!full && busy == 0 && !s->stopping && s->cfg.max_wait_us > 0) {
        if (!partial_waiting) {
          partial_waiting = true;
          partial_since = Clock::now();
        }
        if (Clock::now() - partial_since < std::chrono::microseconds(s->cfg.max_wait_us)) break;
      }
      partial_waiting = false;
      launch_slot(s, sl);
      busy += 1;
      progressed = true;
    }
    if (s->stopping && s->queue.empty() && busy == 0) break;
    if (!progressed) {
      // nothing finished and nothing launched: sleep briefly (new requests or
      // a shorter deadline wake us), then poll the running slots again
      s->cv_work.wait_for(lk, std::chrono::microseconds(busy ? 20 : 200));
    }
  }
}

// Device bytes the server may give to jobs (0 = no limit).
size_t job_budget(const skm_server *s) {
  if (!s->cfg.hbm_budget_bytes) return 0;
  return s->cfg.hbm_budget_bytes > s->hbm ? s->cfg.hbm_budget_bytes - s->hbm : 1;
}

// A finished job's answers, fetched without the server lock (they wait on
// the job's own stream); the context is freed.
struct JobResult {
  skm_status status = SKM_OK;
  std::vector<int32_t> a;
  std::vector<double> c;
};

JobResult collect_job(skm_ctx *ctx, int64_t n_rows, int64_t k, int64_t n_cols, bool centroids,
                      skm_status st, bool fetch) {
  JobResult out;
  out.status = st;
  if (ctx && fetch && st == SKM_OK) {
    out.a.resize(n_rows);
    out.status = skm_get_assignments(ctx, out.a.data(), 0);
    if (out.status == SKM_OK && centroids) {
      out.c.resize((size_t)k * (size_t)n_cols);
      out.status = skm_get_centroids(ctx, out.c.data(), 0);
    }
  }
  if (ctx) skm_destroy(ctx);
  return out;
}

// Completes a job (lock held): its answers or status into the request, its
// memory returned to the budget, its waiters woken.  The context must be
// freed already (r->ctx null), except when the server stops.
void finish_job(skm_server *s, const std::shared_ptr<Request> &r, JobResult res) {
  if (r->ctx) {
    skm_destroy(r->ctx);
    r->ctx = nullptr;
  }
  s->job_hbm -= r->need;
  r->info.hbm_bytes = r->need;
  r->need = 0;
  if (r->cancelled) {
    r->status = SKM_E_CANCELLED;
  } else {
    r->status = res.status;
    r->res_a = std::move(res.a);
    r->res_s = std::move(res.c);
  }
  r->done = true;
  s->jobs_done += 1;
  s->running.erase(std::remove(s->running.begin(), s->running.end(), r), s->running.end());
  drop_payload(s, r);
  s->cv_done.notify_all();
  s->cv_jobs.notify_all();
}

JobResult status_only(skm_status st) {
  JobResult r;
  r.status = st;
  return r;
}

void job_loop(skm_server *s) {
  (void)hipSetDevice(s->c->device);
  std::unique_lock<std::mutex> lk(s->mu);
  size_t turn = 0;
  for (;;) {
    // admission: jobs in arrival order while their memory fits the budget
    while (!s->job_queue.empty() && !s->stopping &&
           (int32_t)s->running.size() < s->cfg.max_jobs) {
      auto r = s->job_queue.front();
      const size_t cap = job_budget(s);
      if (cap && s->job_hbm + r->need > cap) break;
      s->job_queue.pop_front();
      s->job_hbm += r->need;
      s->running.push_back(r);
      // the context is built outside the lock (it copies the rows to HBM)
      skm_csr d{r->n_rows, r->n_cols, r->nnz, r->indptr.data(), r->indices.data(),
                r->values.data(), 0};
      skm_config cf = r->cfg;
      cf.init_rows = r->init_rows.data();
      cf.init_centroids = nullptr;
      cf.stream = nullptr;
      cf.hbm_budget_bytes = 0;
      lk.unlock();
      skm_ctx *ctx = nullptr;
      const skm_status st = skm_init(&d, &cf, &ctx);
      lk.lock();
      r->ctx = ctx;
      if (st != SKM_OK) finish_job(s, r, status_only(st));
    }
    if (s->stopping) {
      // queued and running jobs end as cancelled
      while (!s->job_queue.empty()) {
        auto r = s->job_queue.front();
        s->job_queue.pop_front();
        r->cancelled = true;
        s->job_hbm += r->need;   // finish_job gives it back
        finish_job(s, r, status_only(SKM_E_CANCELLED));
      }
      while (!s->running.empty()) {
        auto r = s->running.front();
        r->cancelled = true;
        finish_job(s, r, status_only(SKM_E_CANCELLED));
      }
      break;
    }
    if (s->running.empty()) {
      s->cv_jobs.wait(lk);
      continue;
    }
    // one iteration of the next running job, outside the lock
    auto r = s->running[turn++ % s->running.size()];
    const bool cancel = r->cancelled;
    skm_ctx *ctx = r->ctx;
    r->ctx = nullptr;   // owned by this turn; collect_job frees it when the job ends
    lk.unlock();
    skm_iter_stats st{};
    int32_t n = 0, conv = 0;
    skm_status rc = SKM_OK;
    bool end = cancel;
    if (!cancel) {
      rc = skm_iterate(ctx, 1, &st, &n, &conv);
      end = rc != SKM_OK || conv || r->info.iterations + n >= r->cfg.max_iter;
    }
    JobResult res;
    if (end) {
      res = collect_job(ctx, r->n_rows, r->cfg.k, r->n_cols, r->out_s != nullptr, rc, !cancel);
      ctx = nullptr;
    }
    lk.lock();
    r->ctx = ctx;
    s->job_iterations += n;
    r->info.iterations += n;
    if (st.objective_update >= 0.0) r->info.objective = st.objective_update;
    if (end) {
      r->info.converged = conv;
      finish_job(s, r, std::move(res));
    }
  }
}

}  // namespace

extern "C" {

void skm_server_config_default(skm_server_config *cfg) {
  if (!cfg) return;
  cfg->n_slots = 4;
  cfg->slot_rows = 16384;
  cfg->slot_nnz = 4 * 1024 * 1024;
  cfg->hbm_budget_bytes = 0;
  cfg->max_wait_us = 100;
  cfg->use_graphs = 1;
  cfg->max_jobs = 2;
}

skm_status skm_server_start(skm_ctx *c, const skm_server_config *cfg, skm_server **out) {
  if (!c || !out) return set_error(SKM_E_INVALID, "context or out is NULL");
  *out = nullptr;
  if (c->poisoned) return set_error(SKM_E_DEVICE, "context is poisoned");
  if (c->server_attached) return set_error(SKM_E_BUSY, "a server is already attached");
  skm_server_config cf;
  skm_server_config_default(&cf);
  if (cfg) cf = *cfg;
  if (cf.n_slots < 1 || cf.slot_rows < 1 || cf.slot_nnz < 1 || cf.max_wait_us < 0 ||
      cf.max_jobs < 0)
    return set_error(SKM_E_INVALID, "bad server config");
  const size_t per = slot_device_bytes(c, cf.slot_rows, cf.slot_nnz);
  if (cf.hbm_budget_bytes) {
    const int64_t fit = (int64_t)(cf.hbm_budget_bytes / per);
    if (fit < 1) return set_error(SKM_E_NOMEM, "HBM budget below one batch slot");
    cf.n_slots = (int32_t)std::min<int64_t>(cf.n_slots, fit);
  }
  auto *s = new (std::nothrow) skm_server();
  if (!s) return set_error(SKM_E_NOMEM, "host allocation failed");
  s->c = c;
  s->cfg = cf;
  s->slots.resize(cf.n_slots);
  for (Slot &sl : s->slots) {
    if (!make_slot(s, sl)) {
      release(s);
      delete s;
      return set_error(SKM_E_NOMEM, "allocating a batch slot failed");
    }
  }
  c->server_attached = 1;
  s->worker = std::thread(worker_loop, s);
  s->job_worker = std::thread(job_loop, s);
  *out = s;
  return SKM_OK;
}

skm_status skm_server_submit(skm_server *s, const skm_csr *docs, int32_t *out_assign,
                             double *out_score, int64_t *ticket) {
  if (!s || !docs || !ticket) return set_error(SKM_E_INVALID, "NULL argument");
  if (docs->on_device) return set_error(SKM_E_INVALID, "server requests are host CSR");
  const int64_t n = docs->n_rows, z = docs->nnz;
  if (n < 0 || z < 0 || docs->n_cols > s->c->D || docs->n_cols < 1)
    return set_error(SKM_E_INVALID, "bad CSR sizes");
  if (n > 0 && (!out_assign || !out_score || !docs->indptr || (z > 0 && (!docs->indices || !docs->values))))
    return set_error(SKM_E_INVALID, "NULL array");
  if (n > s->cfg.slot_rows || z > s->cfg.slot_nnz)
    return set_error(SKM_E_INVALID, "request larger than a batch slot");
  auto r = std::make_shared<Request>();
  r->n_rows = n;
  r->nnz = z;
  if (n > 0) {
    r->indptr.assign(docs->indptr, docs->indptr + n + 1);
    r->indices.assign(docs->indices, docs->indices + z);
    r->values.assign(docs->values, docs->values + z);
    const skm_status st = check_host_rows(r->indptr, r->indices, r->values, n, z, s->c->D);
    if (st != SKM_OK) return st;
  }
  r->out_a = out_assign;
  r->out_s = out_score;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->stopping) return set_error(SKM_E_STATE, "server is stopping");
    r->id = s->next_id++;
    r->t_submit = Clock::now();
    if (!s->any_submit) {
      s->any_submit = true;
      s->t_first = r->t_submit;
    }
    if (n == 0) {
      r->done = true;
    } else {
      s->queue.push_back(r);
      s->max_depth = std::max<int32_t>(s->max_depth, (int32_t)s->queue.size());
    }
    s->live[r->id] = r;
    *ticket = r->id;
  }
  s->cv_work.notify_one();
  return SKM_OK;
}

skm_status skm_server_submit_job(skm_server *s, const skm_csr *docs, const skm_config *cfg,
                                 int32_t *out_assign, double *out_centroids,
                                 skm_job_info *out_info, int64_t *ticket) {
  if (!s || !docs || !cfg || !ticket || !out_assign) return set_error(SKM_E_INVALID, "NULL argument");
  if (docs->on_device) return set_error(SKM_E_INVALID, "jobs are host CSR");
  const int64_t n = docs->n_rows, z = docs->nnz;
  if (n < 1 || z < 0 || docs->n_cols < 1 || !docs->indptr || (z > 0 && (!docs->indices || !docs->values)))
    return set_error(SKM_E_INVALID, "bad CSR");
  if (!cfg->init_rows) return set_error(SKM_E_INVALID, "a job needs init_rows");
  if (cfg->k < 1 || cfg->k > n) return set_error(SKM_E_INVALID, "k must be in [1, n_rows]");
  if (cfg->max_iter < 1) return set_error(SKM_E_INVALID, "a job needs max_iter >= 1");
  auto r = std::make_shared<Request>();
  r->is_job = true;
  r->n_rows = n;
  r->nnz = z;
  r->n_cols = docs->n_cols;
  r->indptr.assign(docs->indptr, docs->indptr + n + 1);
  if (r->indptr[0] != 0 || r->indptr[n] != z) return set_error(SKM_E_INVALID, "bad indptr");
  for (int64_t i = 0; i < n; ++i)
    if (r->indptr[i + 1] < r->indptr[i]) return set_error(SKM_E_INVALID, "indptr decreases");
  r->indices.assign(docs->indices, docs->indices + z);
  r->values.assign(docs->values, docs->values + z);
  r->cfg = *cfg;
  r->init_rows.assign(cfg->init_rows, cfg->init_rows + cfg->k);
  r->need = skm_context_bytes(docs, cfg);
  if (r->need == 0) return set_error(SKM_E_INVALID, "bad job configuration");
  r->out_a = out_assign;
  r->out_s = out_centroids;
  r->out_info = out_info;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->stopping) return set_error(SKM_E_STATE, "server is stopping");
    const size_t cap = job_budget(s);
    if (cap && r->need > cap)
      return set_error(SKM_E_NOMEM, "job needs " + std::to_string(r->need) +
                                        " device bytes, more than the server's budget leaves (" +
                                        std::to_string(cap) + ")");
    r->id = s->next_id++;
    r->t_submit = Clock::now();
    s->job_queue.push_back(r);
    s->live[r->id] = r;
    *ticket = r->id;
  }
  s->cv_jobs.notify_all();
  return SKM_OK;
}

skm_status skm_server_wait(skm_server *s, int64_t ticket, double timeout_s) {
  if (!s) return set_error(SKM_E_INVALID, "server is NULL");
  std::unique_lock<std::mutex> lk(s->mu);
  auto it = s->live.find(ticket);
  if (it == s->live.end()) return set_error(SKM_E_INVALID, "unknown ticket");
  auto r = it->second;
  auto ready = [&] { return r->done; };
  r->waiters += 1;
  s->n_waiters += 1;
  bool ok = true;
  if (timeout_s < 0) {
    s->cv_done.wait(lk, ready);
  } else {
    ok = s->cv_done.wait_for(lk, std::chrono::duration<double>(timeout_s), ready);
  }
  r->waiters -= 1;
  s->n_waiters -= 1;
  if (!ok) {
    s->cv_done.notify_all();   // a stopping server may wait for waiters to leave
    return set_error(SKM_E_TIMEOUT, "request not answered yet");
  }
  s->live.erase(ticket);
  const skm_status st = r->status;
  if (st == SKM_OK) {
    // the answers are copied out here, by the waiting caller
    if (!r->res_a.empty()) std::memcpy(r->out_a, r->res_a.data(), sizeof(int32_t) * r->res_a.size());
    if (r->out_s && !r->res_s.empty())
      std::memcpy(r->out_s, r->res_s.data(), sizeof(double) * r->res_s.size());
    if (r->is_job && r->out_info) *r->out_info = r->info;
  }
  s->cv_done.notify_all();
  if (st == SKM_E_CANCELLED) return set_error(st, "request was cancelled");
  if (st != SKM_OK) return set_error(st, r->is_job ? "clustering job failed" : "device error while serving");
  return SKM_OK;
}

skm_status skm_server_cancel(skm_server *s, int64_t ticket) {
  if (!s) return set_error(SKM_E_INVALID, "server is NULL");
  {
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->live.find(ticket);
    if (it == s->live.end()) return set_error(SKM_E_INVALID, "unknown ticket");
    auto r = it->second;
    r->cancelled = true;
    r->res_a.clear();   // answers not collected yet are dropped
    r->res_s.clear();
    auto drop = [&](std::deque<std::shared_ptr<Request>> &q) {
      auto p = std::find(q.begin(), q.end(), r);
      if (p == q.end()) return false;
      q.erase(p);
      return true;
    };
    // still queued or already answered: complete as cancelled now; in a
    // running batch, finish_slot completes it without answers; a running job
    // is ended by the job thread at its next turn
    if ((r->is_job ? drop(s->job_queue) : drop(s->queue)) || r->done) {
      r->done = true;
      r->status = SKM_E_CANCELLED;
      drop_payload(s, r);
    }
  }
  s->cv_done.notify_all();
  s->cv_jobs.notify_all();
  return SKM_OK;
}

skm_status skm_server_get_stats(skm_server *s, skm_server_stats *out) {
  if (!s || !out) return set_error(SKM_E_INVALID, "NULL argument");
  std::lock_guard<std::mutex> lk(s->mu);
  std::memset(out, 0, sizeof(*out));
  out->requests_done = (int64_t)s->lat_ms.size();
  out->rows_done = s->rows_done;
  out->batches = s->batches;
  out->slots = (int32_t)s->slots.size();
  out->max_queue_depth = s->max_depth;
  out->hbm_bytes = s->hbm + s->job_hbm;
  out->jobs_done = s->jobs_done;
  out->job_iterations = s->job_iterations;
  out->jobs_running = (int32_t)s->running.size();
  out->jobs_queued = (int32_t)s->job_queue.size();
  if (!s->lat_ms.empty()) {
    std::vector<double> v = s->lat_ms;
    std::sort(v.begin(), v.end());
    auto pct = [&](double p) {
      const size_t i = (size_t)std::min<double>(v.size() - 1, std::floor(p * (double)(v.size() - 1) + 0.5));
      return v[i];
    };
    out->p50_ms = pct(0.50);
    out->p99_ms = pct(0.99);
    out->max_ms = v.back();
    double sum = 0;
    for (double x : v) sum += x;
    out->mean_ms = sum / (double)v.size();
    const double span = std::chrono::duration<double>(s->t_last - s->t_first).count();
    out->rows_per_s = span > 0 ? (double)s->rows_done / span : 0.0;
  }
  return SKM_OK;
}

skm_status skm_server_stop(skm_server *s) {
  if (!s) return set_error(SKM_E_INVALID, "server is NULL");
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stopping = true;
  }
  s->cv_work.notify_all();
  s->cv_jobs.notify_all();
  if (s->worker.joinable()) s->worker.join();
  if (s->job_worker.joinable()) s->job_worker.join();
  {
    // every request is answered now; threads still inside skm_server_wait
    // leave before the server is freed
    std::unique_lock<std::mutex> lk(s->mu);
    s->cv_done.notify_all();
    s->cv_done.wait(lk, [&] { return s->n_waiters == 0; });
  }
  const bool dev_err = s->dev_error != hipSuccess;
  s->c->server_attached = 0;
  if (dev_err) s->c->poisoned = true;
  release(s);
  delete s;
  return dev_err ? set_error(SKM_E_DEVICE, "device error while serving") : SKM_OK;
}

}  // extern "C"
