// server.hip -- served partition jobs with continuous batching.
//
// A worker thread owns a context of its own (scratch, stream).  A submitted
// job is charged its device footprint against the HBM budget (submission
// waits until it fits beside the queued and running jobs), copied to device
// memory owned by the server and queued.  Between executor steps the worker
// admits queued jobs in arrival order up to max_active, then advances every
// admitted job by one step: one fused LP round over all jobs at an LP stage,
// their contractions, initial partitions and finishing.  A job's charge is
// returned when it completes.
// Jobs that arrive while others run therefore share the following launches.
// Every step is exact per job, so a served result equals the same job run
// alone.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "engine.h"

using namespace sclap;

namespace sclap {
int setup_partition_job(Ctx* c, Job* j, const sclap_csr* g, int32_t k, int64_t eps_num, int64_t eps_den,
                        const sclap_ml_params* p, int32_t* part_out, hipStream_t st);
}

namespace {

struct ServedJob {
  uint64_t ticket = 0;
  Job job;
  // device copy of the input, owned by the server
  int64_t* rp = nullptr;
  int32_t* col = nullptr;
  int32_t* ew = nullptr;
  void* nw = nullptr;
  sclap_csr g{};
  int32_t k = 2;
  int64_t eps_num = 3, eps_den = 100;
  sclap_ml_params params{};
  int32_t* part_out = nullptr;
  int64_t footprint = 0;
  double t_submit = 0, t_admit = 0, t_done = 0;
  bool done = false;
  sclap_job_result res{};
};

}  // namespace

namespace sclap {
// Device bytes of a job's input copy.
int64_t input_bytes_of(const sclap_csr& g) {
  const int64_t n = g.n, m = g.m;
  return 8 * (n + 1) + 4 * m + (g.ew ? 4 * m : 0) + (g.nw ? (int64_t)g.nw_bytes * n : 0);
}

// Device bytes a job may hold at once, as an upper bound:
//   - its input copy;
//   - the hierarchy: at most two weighted copies of the input (every level
//     has at most the nodes and entries of the one below it, and each
//     contraction shrinks the node count by at least 5%, so the levels above
//     level 1 sum to less than another copy): 8 (n + 1) + 8 m + 8 n + 4 n each;
//   - the LP state of a level: labels, desires, admitted flags, label or
//     block weights and incoming sums, the two rated-set bitmaps (48 B per
//     node), and the block connections of refinement (n x k int32 for
//     k <= kConnMaxK);
//   - its share of the context scratch that every fused round sizes by the
//     total node count of the round: kRoundBytesPerNode per node (degree
//     bins and rows, rated list, movers, contended keys, hub rows, tile
//     admission) and kRoundBytesPerEntry per stored entry (the staged
//     (label, sum) pairs of hub rows);
//   - the temporaries of a contraction: kContractBytesPerEntry per stored
//     entry of the contracted level (two key arrays, sums, sort space,
//     mirror) and the initial-partition scratch (16 B per node);
//   - level 0, the input without its degree-0 nodes: row offsets, renumbered
//     columns, node weights, input ids and the renumbering scratch;
//   - with the Section 4 extensions: the best partition of iterated cycles
//     (4 B per node), the level without the cut edges that a later cycle's
//     clustering rates (8 (n + 1) + 8 m) and its filter scratch (2 B per
//     entry), the degree classes of sub-rounds (1 B per node), and an
//     ensemble's overlay with its sort and scans (48 B per node).
int64_t footprint_of(const sclap_csr& g, int32_t k, const sclap_ml_params* p) {
  const int64_t n = g.n, m = g.m;
  const int64_t hierarchy = 2 * (8 * (n + 1) + 8 * m + 8 * n + 4 * n);
  const int64_t conn = k <= kConnMaxK ? 4 * n * (int64_t)k : 0;
  const int64_t scratch = kRoundBytesPerNode * n + kRoundBytesPerEntry * m;
  const int64_t contraction = kContractBytesPerEntry * m + 16 * n;
  // the input without its degree-0 nodes (level 0) and its renumbering
  int64_t ext = 8 * (n + 1) + 4 * m + 8 * n + 12 * n;
  if (p && p->vcycles > 1) ext += 4 * n + 8 * (n + 1) + 8 * m + 2 * m + 4096;
  if (p && p->subrounds > 1) ext += n;
  if (p && p->ensemble > 1) ext += 48 * n;
  return input_bytes_of(g) + hierarchy + 48 * n + conn + scratch + contraction + ext + 65536;
}
}  // namespace sclap

namespace {

void free_input(ServedJob* sj, hipStream_t st) {
  dfree(sj->rp, st);
  dfree(sj->col, st);
  dfree(sj->ew, st);
  dfree(sj->nw, st);
  sj->rp = nullptr;
  sj->col = nullptr;
  sj->ew = nullptr;
  sj->nw = nullptr;
}

}  // namespace

struct sclap_server {
  Ctx ctx;
  int device = 0;
  hipStream_t stream = nullptr;   // worker
  hipStream_t upload = nullptr;   // submissions
  int64_t budget = 0;
  int64_t in_use = 0;
  int64_t peak = 0;
  int32_t max_active = 64;
  int64_t peak_active = 0;        // most jobs on the device at once (under mu)
  std::mutex mu;
  std::mutex upload_mu;
  std::condition_variable work_cv;
  std::condition_variable done_cv;
  std::deque<ServedJob*> queue;
  std::vector<ServedJob*> active;
  std::unordered_map<uint64_t, ServedJob*> jobs;
  std::vector<double> latencies;
  uint64_t next_ticket = 1;
  bool stop = false;
  bool hold = false;              // admission held: queued jobs wait (under mu)
  std::thread worker;
  double t_first_submit = -1;
  double t_last_done = 0;
  int64_t completed = 0;

  void run();
};

void sclap_server::run() {
  (void)hipSetDevice(device);
  CtxScope scope(&ctx);
  for (;;) {
    std::vector<ServedJob*> admit;
    {
      std::unique_lock<std::mutex> lk(mu);
      work_cv.wait(lk, [&] { return stop || (!hold && !queue.empty()) || !active.empty(); });
      if (stop && queue.empty() && active.empty()) break;
      // every queued job's footprint is charged from its submission on, so
      // admission only waits for a free slot
      while (!hold && !queue.empty() && (int32_t)(active.size() + admit.size()) < max_active) {
        admit.push_back(queue.front());
        queue.pop_front();
      }
    }
    for (ServedJob* sj : admit) {
      sj->t_admit = now_ms();
      sj->job = Job();
      const int rc = setup_partition_job(&ctx, &sj->job, &sj->g, sj->k, sj->eps_num, sj->eps_den, &sj->params,
                                         sj->part_out, stream);
      if (rc != SCLAP_OK) {
        sj->job.stage = ST_ERROR;
        sj->job.status = rc;
      }
      active.push_back(sj);
    }
    {
      std::lock_guard<std::mutex> lk(mu);
      peak_active = std::max<int64_t>(peak_active, (int64_t)active.size());
    }
    std::vector<Job*> js;
    for (ServedJob* sj : active) js.push_back(&sj->job);
    bool all_done = false;
    int rc = SCLAP_OK;
    if (!js.empty()) {
      ctx.bin_sig_valid = false;  // the job set changes between steps
      rc = step_jobs(&ctx, js, stream, &all_done);
    }
    if (rc != SCLAP_OK) {
      for (ServedJob* sj : active)
        if (sj->job.stage != ST_DONE) {
          sj->job.stage = ST_ERROR;
          sj->job.status = rc;
        }
    }
    // retire finished jobs
    std::vector<ServedJob*> still;
    std::vector<ServedJob*> finished;
    for (ServedJob* sj : active) {
      if (sj->job.stage == ST_DONE || sj->job.stage == ST_ERROR) finished.push_back(sj);
      else still.push_back(sj);
    }
    if (!finished.empty()) {
      for (ServedJob* sj : finished) {
        job_release_lp(&sj->job, stream, false);
        job_release_levels(&sj->job, stream);
        free_input(sj, stream);
      }
      (void)hipStreamSynchronize(stream);
      // freed blocks beyond the context's cache limit go back to HIP; the
      // cache is outside the budget, so it is kept small
      if (ctx.cache_bytes > ctx.cache_limit / 2) ctx_trim(&ctx);
      const double t = now_ms();
      std::lock_guard<std::mutex> lk(mu);
      for (ServedJob* sj : finished) {
        sj->t_done = t;
        sj->res.status = sj->job.stage == ST_DONE ? SCLAP_OK : (sj->job.status ? sj->job.status : SCLAP_EHIP);
        sj->res.cut = sj->job.st.cut;
        sj->res.max_block = sj->job.st.max_block;
        sj->res.latency_ms = sj->t_done - sj->t_submit;
        sj->res.queue_ms = sj->t_admit - sj->t_submit;
        sj->done = true;
        in_use -= sj->footprint;
        latencies.push_back(sj->res.latency_ms);
        ++completed;
        t_last_done = t;
      }
      done_cv.notify_all();
    }
    active.swap(still);
  }
}

extern "C" {

int sclap_server_create(sclap_ctx* ctx, int64_t hbm_budget_bytes, int32_t max_active, sclap_server** out) {
  if (!ctx || !out || hbm_budget_bytes <= 0 || max_active < 1) return fail(SCLAP_EINVAL, "bad server argument");
  *out = nullptr;
  int dev = 0;
  SCLAP_HIP(hipGetDevice(&dev));
  sclap_server* s = new sclap_server();
  s->device = dev;
  s->budget = hbm_budget_bytes;
  s->max_active = max_active;
  s->ctx.device = dev;
  // freed device blocks cached by the worker are not part of any job's
  // footprint: at most 1/16 of the budget (and 8 GiB)
  s->ctx.cache_limit = (size_t)std::min<int64_t>(hbm_budget_bytes / 16, (int64_t)8 << 30);
  if (hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking) != hipSuccess ||
      hipStreamCreateWithFlags(&s->upload, hipStreamNonBlocking) != hipSuccess) {
    delete s;
    return fail(SCLAP_EHIP, "stream creation failed");
  }
  for (auto& e : s->ctx.ev) (void)hipEventCreate(&e);
  s->worker = std::thread([s] { s->run(); });
  *out = s;
  return SCLAP_OK;
}

int sclap_server_submit(sclap_server* srv, const sclap_job* job, uint64_t* ticket) {
  if (!srv || !job || !ticket) return fail(SCLAP_EINVAL, "NULL argument");
  const sclap_csr& g = job->graph;
  if (g.n < 0 || g.m < 0 || !g.row_ptr || (g.m > 0 && !g.col) || (g.n > 0 && !job->part_out) || job->k < 1)
    return fail(SCLAP_EINVAL, "bad job");
  if (g.nw && g.nw_bytes != 4 && g.nw_bytes != 8) return fail(SCLAP_EINVAL, "nw_bytes must be 4 or 8");
  ServedJob* sj = new ServedJob();
  sj->footprint = footprint_of(g, job->k, &job->params);
  if (sj->footprint > srv->budget) {
    delete sj;
    return fail(SCLAP_EBUDGET, "job larger than the server's memory budget");
  }
  {
    // the job's whole footprint counts against the budget from now on (its
    // input copy is made here): wait while it does not fit beside the jobs
    // queued and running; a job alone always fits
    std::unique_lock<std::mutex> lk(srv->mu);
    srv->done_cv.wait(lk, [&] { return srv->in_use + sj->footprint <= srv->budget; });
    srv->in_use += sj->footprint;
    srv->peak = std::max(srv->peak, srv->in_use);
  }
  sj->k = job->k;
  sj->eps_num = job->eps_num;
  sj->eps_den = job->eps_den;
  sj->params = job->params;
  sj->part_out = job->part_out;
  {
    std::lock_guard<std::mutex> ul(srv->upload_mu);
    (void)hipSetDevice(srv->device);
    hipStream_t st = srv->upload;
    int rc = dalloc_t(&sj->rp, (size_t)g.n + 1, st);
    if (rc == SCLAP_OK) rc = dalloc_t(&sj->col, (size_t)std::max<int64_t>(g.m, 1), st);
    if (rc == SCLAP_OK && g.ew) rc = dalloc_t(&sj->ew, (size_t)std::max<int64_t>(g.m, 1), st);
    if (rc == SCLAP_OK && g.nw) rc = dalloc(&sj->nw, (size_t)g.nw_bytes * std::max<int64_t>(g.n, 1), st);
    if (rc == SCLAP_OK && hipMemcpyAsync(sj->rp, g.row_ptr, (size_t)(g.n + 1) * 8, hipMemcpyDeviceToDevice, st))
      rc = SCLAP_EHIP;
    if (rc == SCLAP_OK && g.m > 0 &&
        hipMemcpyAsync(sj->col, g.col, (size_t)g.m * 4, hipMemcpyDeviceToDevice, st) != hipSuccess)
      rc = SCLAP_EHIP;
    if (rc == SCLAP_OK && g.ew && g.m > 0 &&
        hipMemcpyAsync(sj->ew, g.ew, (size_t)g.m * 4, hipMemcpyDeviceToDevice, st) != hipSuccess)
      rc = SCLAP_EHIP;
    if (rc == SCLAP_OK && g.nw && g.n > 0 &&
        hipMemcpyAsync(sj->nw, g.nw, (size_t)g.n * g.nw_bytes, hipMemcpyDeviceToDevice, st) != hipSuccess)
      rc = SCLAP_EHIP;
    if (hipStreamSynchronize(st) != hipSuccess && rc == SCLAP_OK) rc = SCLAP_EHIP;
    if (rc != SCLAP_OK) {
      free_input(sj, st);
      (void)hipStreamSynchronize(st);
      {
        std::lock_guard<std::mutex> lk(srv->mu);
        srv->in_use -= sj->footprint;
      }
      srv->done_cv.notify_all();
      delete sj;
      return fail(rc, "copying the job's graph failed");
    }
  }
  sj->g = g;
  sj->g.row_ptr = sj->rp;
  sj->g.col = sj->col;
  sj->g.ew = sj->ew;
  sj->g.nw = sj->nw;
  {
    std::lock_guard<std::mutex> lk(srv->mu);
    sj->ticket = srv->next_ticket++;
    sj->t_submit = now_ms();
    if (srv->t_first_submit < 0) srv->t_first_submit = sj->t_submit;
    srv->jobs[sj->ticket] = sj;
    srv->queue.push_back(sj);
    *ticket = sj->ticket;
  }
  srv->work_cv.notify_one();
  return SCLAP_OK;
}

static int take_result(sclap_server* srv, uint64_t ticket, sclap_job_result* res, bool wait) {
  std::unique_lock<std::mutex> lk(srv->mu);
  auto it = srv->jobs.find(ticket);
  if (it == srv->jobs.end()) return fail(SCLAP_ENOTFOUND, "unknown ticket");
  ServedJob* sj = it->second;
  if (!sj->done) {
    if (!wait) return SCLAP_EAGAIN;
    srv->done_cv.wait(lk, [&] { return sj->done; });
  }
  if (res) *res = sj->res;
  srv->jobs.erase(it);
  delete sj;
  return SCLAP_OK;
}

int sclap_server_poll(sclap_server* srv, uint64_t ticket, sclap_job_result* res) {
  if (!srv) return fail(SCLAP_EINVAL, "NULL server");
  return take_result(srv, ticket, res, false);
}

int sclap_server_wait(sclap_server* srv, uint64_t ticket, sclap_job_result* res) {
  if (!srv) return fail(SCLAP_EINVAL, "NULL server");
  return take_result(srv, ticket, res, true);
}

int sclap_submit(sclap_server* srv, const sclap_job* job, uint64_t* ticket) {
  return sclap_server_submit(srv, job, ticket);
}
int sclap_poll(sclap_server* srv, uint64_t ticket, sclap_job_result* res) {
  return sclap_server_poll(srv, ticket, res);
}
int sclap_wait(sclap_server* srv, uint64_t ticket, sclap_job_result* res) {
  return sclap_server_wait(srv, ticket, res);
}

int sclap_server_footprint(const sclap_csr* g, int32_t k, const sclap_ml_params* p, int64_t* input_bytes,
                           int64_t* footprint_bytes) {
  if (!g || k < 1 || g->n < 0 || g->m < 0) return fail(SCLAP_EINVAL, "bad argument");
  if (input_bytes) *input_bytes = input_bytes_of(*g);
  if (footprint_bytes) *footprint_bytes = footprint_of(*g, k, p);
  return SCLAP_OK;
}

int sclap_server_path_counters(sclap_server* srv, int32_t count, int64_t* out) {
  if (!srv || count < 0 || (count > 0 && !out)) return fail(SCLAP_EINVAL, "bad argument");
  for (int i = 0; i < count && i < kPathCounters; ++i) out[i] = srv->ctx.path_ctr[i].load(std::memory_order_relaxed);
  return SCLAP_OK;
}

int sclap_server_stats(sclap_server* srv, double* p50_ms, double* p99_ms, double* jobs_per_s, int64_t* completed,
                       int64_t* peak_bytes, int64_t* peak_active) {
  if (!srv) return fail(SCLAP_EINVAL, "NULL server");
  std::lock_guard<std::mutex> lk(srv->mu);
  std::vector<double> l = srv->latencies;
  std::sort(l.begin(), l.end());
  auto pct = [&](double q) {
    if (l.empty()) return 0.0;
    size_t i = (size_t)(q * (double)(l.size() - 1) + 0.5);
    return l[std::min(i, l.size() - 1)];
  };
  if (p50_ms) *p50_ms = pct(0.50);
  if (p99_ms) *p99_ms = pct(0.99);
  const double span = srv->t_last_done - srv->t_first_submit;
  if (jobs_per_s) *jobs_per_s = (srv->completed > 0 && span > 0) ? srv->completed / (span * 1e-3) : 0.0;
  if (completed) *completed = srv->completed;
  if (peak_bytes) *peak_bytes = srv->peak;
  if (peak_active) *peak_active = srv->peak_active;
  return SCLAP_OK;
}

int sclap_server_hold(sclap_server* srv, int32_t hold) {
  if (!srv) return fail(SCLAP_EINVAL, "NULL server");
  {
    std::lock_guard<std::mutex> lk(srv->mu);
    srv->hold = hold != 0;
  }
  srv->work_cv.notify_all();
  return SCLAP_OK;
}

int sclap_server_destroy(sclap_server* srv) {
  if (!srv) return SCLAP_OK;
  {
    std::lock_guard<std::mutex> lk(srv->mu);
    srv->stop = true;
  }
  srv->work_cv.notify_all();
  if (srv->worker.joinable()) srv->worker.join();
  (void)hipSetDevice(srv->device);
  for (auto& kv : srv->jobs) {
    free_input(kv.second, srv->stream);
    delete kv.second;
  }
  (void)hipStreamSynchronize(srv->stream);
  ctx_release(&srv->ctx, srv->stream);
  (void)hipStreamDestroy(srv->stream);
  (void)hipStreamDestroy(srv->upload);
  delete srv;
  return SCLAP_OK;
}

}  // extern "C"
