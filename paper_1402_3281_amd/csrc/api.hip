// api.hip -- the C ABI declared in include/sclap.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cstring>
#include <memory>
#include <string>
#include <vector>

#include "engine.h"
#include "ext.h"

namespace sclap {
const char* last_error_cstr();
int noalloc_setup(int device);
}

using namespace sclap;

struct sclap_ctx {
  Ctx c;
};

struct sclap_graph {
  Level L;
};

static hipStream_t as_stream(void* s) { return (hipStream_t)s; }

static int check_csr(const sclap_csr* g) {
  if (!g) return fail(SCLAP_EINVAL, "graph is NULL");
  if (g->n < 0 || g->m < 0) return fail(SCLAP_EINVAL, "negative n or m");
  if (g->n >= ((int64_t)1 << 31) - 1) return fail(SCLAP_EINVAL, "n must be below 2^31 - 1");
  if (!g->row_ptr) return fail(SCLAP_EINVAL, "row_ptr is NULL");
  if (g->m > 0 && !g->col) return fail(SCLAP_EINVAL, "col is NULL");
  if (g->nw && g->nw_bytes != 4 && g->nw_bytes != 8) return fail(SCLAP_EINVAL, "nw_bytes must be 4 or 8");
  return SCLAP_OK;
}

static int check_lp(const sclap_lp_params* p) {
  if (!p) return fail(SCLAP_EINVAL, "params are NULL");
  if (p->max_rounds < 1 || p->max_rounds > SCLAP_MAX_ROUNDS) return fail(SCLAP_EINVAL, "max_rounds out of range");
  if (p->stop_rule != 0 && p->stop_rule != 1) return fail(SCLAP_EINVAL, "stop_rule must be 0 or 1");
  if (p->subrounds < 0 || p->subrounds > SCLAP_MAX_SUBROUNDS) return fail(SCLAP_EINVAL, "subrounds out of range");
  return SCLAP_OK;
}

static int bounds_impl(int64_t total_w, int64_t max_w, int32_t k, int64_t eps_num, int64_t eps_den, int32_t f,
                       int64_t* lmax, int64_t* W, int64_t* U) {
  if (k < 1 || eps_num < 0 || eps_den < 1 || f < 1 || total_w < 0 || max_w < 0)
    return fail(SCLAP_EINVAL, "bounds: k >= 1, eps_num >= 0, eps_den >= 1, f >= 1 required");
  const int64_t per = total_w / k + (total_w % k != 0);
  const __int128 num = (__int128)(eps_den + eps_num) * per;
  const __int128 l = num / eps_den;
  const __int128 w = num / ((__int128)eps_den * f);
  if (l > INT64_MAX / 2) return fail(SCLAP_EOVERFLOW, "L_max overflows");
  *lmax = (int64_t)l;
  *W = (int64_t)w;
  *U = max_w > *W ? max_w : *W;
  return SCLAP_OK;
}

// Total undirected edge weight must stay below 2^31 so that every rating and
// coarse edge weight fits int32.
static int check_edge_total(Ctx* c, const sclap_csr* g, hipStream_t st) {
  if (!g->ew) {
    if (g->m / 2 >= ((int64_t)1 << 31)) return fail(SCLAP_EOVERFLOW, "more than 2^31 edges");
    return SCLAP_OK;
  }
  // sum of edge weights: reuse graph_totals on a view with ew as weights
  SCLAP_TRY(c->small.ensure(256, st));
  unsigned long long* d = (unsigned long long*)c->small.p;
  // treat ew as node weights of a graph with m nodes and empty rows
  int64_t* zero_rp = nullptr;
  int64_t* w64 = nullptr;
  SCLAP_TRY(dalloc_t(&zero_rp, (size_t)g->m + 1, st));
  SCLAP_TRY(dalloc_t(&w64, (size_t)std::max<int64_t>(g->m, 1), st));
  SCLAP_TRY(fill_i64(zero_rp, g->m + 1, 0, st));
  SCLAP_TRY(widen_nw(g->ew, 4, g->m, w64, st));
  SCLAP_TRY(graph_totals(zero_rp, w64, g->m, 1, d, st));
  SCLAP_TRY(ctx_ensure_pin(c, 64));
  SCLAP_HIP(hipMemcpyAsync(c->pin, d, 16, hipMemcpyDeviceToHost, st));
  SCLAP_HIP(hipStreamSynchronize(st));
  dfree(zero_rp, st);
  dfree(w64, st);
  if (c->pin[0] / 2 >= ((int64_t)1 << 31)) return fail(SCLAP_EOVERFLOW, "total edge weight reaches 2^31");
  return SCLAP_OK;
}

namespace sclap {

// Set up a partition job: bounds from the whole input, level 0, first stage.
int setup_partition_job(Ctx* c, Job* j, const sclap_csr* g, int32_t k, int64_t eps_num, int64_t eps_den,
                               const sclap_ml_params* p, int32_t* part_out, hipStream_t st) {
  SCLAP_TRY(check_csr(g));
  if (!p) return fail(SCLAP_EINVAL, "params are NULL");
  if (k < 1) return fail(SCLAP_EINVAL, "k must be >= 1");
  if (p->lp_rounds < 1 || p->lp_rounds > SCLAP_MAX_ROUNDS || p->refine_rounds < 0 ||
      p->refine_rounds > SCLAP_MAX_ROUNDS)
    return fail(SCLAP_EINVAL, "rounds out of range");
  if (p->vcycles < 0 || p->vcycles > SCLAP_MAX_CYCLES) return fail(SCLAP_EINVAL, "vcycles out of range");
  if (p->subrounds < 0 || p->subrounds > SCLAP_MAX_SUBROUNDS) return fail(SCLAP_EINVAL, "subrounds out of range");
  if (p->ensemble < 0 || p->ensemble > SCLAP_MAX_ENSEMBLE) return fail(SCLAP_EINVAL, "ensemble out of range");
  if (p->delta_num < 0 || (p->delta_num > 0 && p->delta_den < 1))
    return fail(SCLAP_EINVAL, "extra imbalance: delta_num >= 0 and delta_den >= 1 required");
  if (g->n > 0 && !part_out) return fail(SCLAP_EINVAL, "part_out is NULL");
  j->t_start = now_ms();
  j->vcycles = std::max<int32_t>(p->vcycles, 1);
  j->subrounds = p->subrounds;
  j->members = std::max<int32_t>(p->ensemble, 1);
  j->delta_num = p->delta_num;
  j->delta_den = p->delta_num > 0 ? p->delta_den : 1;
  j->eps_num = eps_num;
  j->eps_den = eps_den;
  j->kind = JOB_PARTITION;
  j->k = k;
  j->lp_rounds = p->lp_rounds;
  j->ref_rounds = p->refine_rounds;
  j->dir_rule = p->direction_rule;
  j->stop_rule = 1;
  j->part_out = part_out;
  std::memset(&j->st, 0, sizeof(j->st));
  if (g->n == 0) {
    // an empty graph is done at once, with no launch: one level, no
    // clustering (0 nodes are below any threshold), and the refinement
    // rounds that the stop rule gives when nothing moves (two)
    SCLAP_TRY(bounds_impl(0, 0, k, eps_num, eps_den, p->f, &j->lmax, &j->W, &j->U));
    j->threshold = p->threshold > 0 ? p->threshold : 60 * (int64_t)k;
    j->st.lmax = j->lmax;
    j->st.W = j->W;
    j->st.U = j->U;
    j->st.threshold = j->threshold;
    j->st.levels = 1;
    j->st.rounds_r[0] = std::min<int32_t>(j->ref_rounds, 2);
    // every cycle of an empty graph is the same: the first is kept
    j->st.cycles = 1;
    j->st.cycle_levels[0] = 1;
    j->st.ms_total = now_ms() - j->t_start;
    j->stage = ST_DONE;
    return SCLAP_OK;
  }
  SCLAP_TRY(check_edge_total(c, g, st));
  SCLAP_TRY(job_set_input(c, j, g, st));
  int64_t C = 0, maxc = 0;
  SCLAP_TRY(level_totals(c, j, &j->lv[0], &C, &maxc, st));
  if (C > 0 && (__int128)C * k >= ((__int128)1 << 62)) return fail(SCLAP_EOVERFLOW, "k * c(V) overflows");
  SCLAP_TRY(bounds_impl(C, maxc, k, eps_num, eps_den, p->f, &j->lmax, &j->W, &j->U));
  j->total_w = C;
  if (p->threshold > 0) {
    j->threshold = p->threshold;
  } else {
    const int64_t a = 60 * (int64_t)k, b = g->n / (60 * (int64_t)k);
    j->threshold = a > b ? a : b;
  }
  // level 0: the input without its degree-0 nodes
  SCLAP_TRY(job_compact_input(c, j, st));
  Level& L = j->lv[0];
  j->st.lmax = j->lmax;
  j->st.W = j->W;
  j->st.U = j->U;
  j->st.threshold = j->threshold;
  j->st.n_isolated = g->n - L.n_active;
  j->st.levels = 1;
  j->st.n_level[0] = L.n_active;
  j->st.m_level[0] = L.m;
  j->cur = 0;
  if (L.n_active > j->threshold) return job_begin_cluster(c, j, st);
  j->stage = ST_IP;
  return SCLAP_OK;
}

}  // namespace sclap

extern "C" {

const char* sclap_last_error(const sclap_ctx* ctx) {
  (void)ctx;  // the message is kept per thread
  return last_error_cstr();
}

int sclap_trim(sclap_ctx* ctx) {
  if (!ctx) return fail(SCLAP_EINVAL, "ctx is NULL");
  SCLAP_HIP(hipSetDevice(ctx->c.device));
  ctx_trim(&ctx->c);
  return SCLAP_OK;
}

int sclap_create(sclap_ctx** out, int device) {
  if (!out) return fail(SCLAP_EINVAL, "out is NULL");
  *out = nullptr;
  int ndev = 0;
  SCLAP_HIP(hipGetDeviceCount(&ndev));
  if (device < 0 || device >= ndev) return fail(SCLAP_EINVAL, "no such device");
  SCLAP_HIP(hipSetDevice(device));
  std::unique_ptr<sclap_ctx> x(new sclap_ctx());
  x->c.device = device;
  int cus = 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) == hipSuccess && cus > 0)
    x->c.cu_count = cus;
  hipMemPool_t pool;
  if (hipDeviceGetDefaultMemPool(&pool, device) == hipSuccess) {
    uint64_t thr = UINT64_MAX;
    (void)hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &thr);
  }
  for (auto& e : x->c.ev) SCLAP_HIP(hipEventCreate(&e));
  // the allocation-free entry point's fixed scratch on this device
  SCLAP_TRY(noalloc_setup(device));
  *out = x.release();
  return SCLAP_OK;
}

int sclap_destroy(sclap_ctx* ctx) {
  if (!ctx) return SCLAP_OK;
  Ctx& c = ctx->c;
  (void)hipSetDevice(c.device);
  (void)hipDeviceSynchronize();
  ctx_release(&c, nullptr);
  delete ctx;
  return SCLAP_OK;
}

int sclap_bounds(int64_t total_w, int64_t max_w, int32_t k, int64_t eps_num, int64_t eps_den, int32_t f,
                 int64_t* lmax, int64_t* W, int64_t* U) {
  if (!lmax || !W || !U) return fail(SCLAP_EINVAL, "NULL output");
  return bounds_impl(total_w, max_w, k, eps_num, eps_den, f, lmax, W, U);
}

int sclap_validate(sclap_ctx* ctx, const sclap_csr* g, void* stream) {
  if (!ctx) return fail(SCLAP_EINVAL, "ctx is NULL");
  SCLAP_TRY(check_csr(g));
  Ctx* c = &ctx->c;
  CtxScope scope(c);
  hipStream_t st = as_stream(stream);
  const int64_t n = g->n, m = g->m;
  const size_t mz = (size_t)std::max<int64_t>(m, 1);
  uint64_t *fk = nullptr, *rk = nullptr, *fk2 = nullptr, *rk2 = nullptr;
  int32_t *fw = nullptr, *fw2 = nullptr, *rw2 = nullptr;
  SCLAP_TRY(dalloc_t(&fk, mz, st));
  SCLAP_TRY(dalloc_t(&rk, mz, st));
  SCLAP_TRY(dalloc_t(&fk2, mz, st));
  SCLAP_TRY(dalloc_t(&rk2, mz, st));
  SCLAP_TRY(dalloc_t(&fw, mz, st));
  SCLAP_TRY(dalloc_t(&fw2, mz, st));
  SCLAP_TRY(dalloc_t(&rw2, mz, st));
  SCLAP_TRY(c->small.ensure(256, st));
  unsigned* bad = (unsigned*)((char*)c->small.p + 192);
  SCLAP_TRY(fill_u32(bad, 1, 0, st));
  const int bits = bits_for(n);
  if (n > 0) SCLAP_TRY(validate_keys(g->row_ptr, g->col, g->ew, n, m, bits, fk, rk, fw, bad, st));
  SCLAP_TRY(validate_nw(g->nw, g->nw_bytes, n, bad, st));
  const size_t tb = prim_sort_pairs_bytes(mz);
  SCLAP_TRY(c->prim.ensure(tb, st));
  SCLAP_TRY(prim_sort_pairs(c->prim.p, tb, fk, fk2, fw, fw2, (size_t)m, 2 * bits, st));
  SCLAP_TRY(prim_sort_pairs(c->prim.p, tb, rk, rk2, fw, rw2, (size_t)m, 2 * bits, st));
  SCLAP_TRY(validate_cmp(fk2, rk2, fw2, rw2, m, bad, st));
  SCLAP_TRY(ctx_ensure_pin(c, 64));
  SCLAP_HIP(hipMemcpyAsync(c->pin, bad, 4, hipMemcpyDeviceToHost, st));
  SCLAP_HIP(hipStreamSynchronize(st));
  const unsigned b = *(unsigned*)c->pin;
  for (void* p : {(void*)fk, (void*)rk, (void*)fk2, (void*)rk2, (void*)fw, (void*)fw2, (void*)rw2}) dfree(p, st);
  if (b & 2u) return fail(SCLAP_EINVAL, "neighbour id, row offset or weight out of range");
  if (b & 1u) return fail(SCLAP_ENOTSYM, "CSR is not symmetric, has a self-loop or repeats a neighbour");
  return SCLAP_OK;
}

static int cluster_impl(sclap_ctx* ctx, const sclap_csr* g, int64_t U, const sclap_lp_params* p,
                        const int32_t* blocks, int32_t member, int32_t* labels_out, int64_t* n_clusters,
                        sclap_round_stats* rs, void* stream);

int sclap_cluster(sclap_ctx* ctx, const sclap_csr* g, int64_t U, const sclap_lp_params* p, int32_t* labels_out,
                  int64_t* n_clusters, sclap_round_stats* rs, void* stream) {
  return cluster_impl(ctx, g, U, p, nullptr, 0, labels_out, n_clusters, rs, stream);
}

int sclap_cluster_ext(sclap_ctx* ctx, const sclap_csr* g, int64_t U, const sclap_lp_params* p,
                      const int32_t* blocks, int32_t member, int32_t* labels_out, int64_t* n_clusters,
                      sclap_round_stats* rs, void* stream) {
  if (member < 0) return fail(SCLAP_EINVAL, "member must be >= 0");
  return cluster_impl(ctx, g, U, p, blocks, member, labels_out, n_clusters, rs, stream);
}

int sclap_overlay(sclap_ctx* ctx, int64_t n, int32_t* overlay_inout, const int32_t* labels, int64_t* n_clusters,
                  void* stream) {
  if (!ctx) return fail(SCLAP_EINVAL, "ctx is NULL");
  if (n < 0 || n >= ((int64_t)1 << 31)) return fail(SCLAP_EINVAL, "n out of range");
  if (n > 0 && (!overlay_inout || !labels)) return fail(SCLAP_EINVAL, "NULL labels");
  Ctx* c = &ctx->c;
  CtxScope scope(c);
  hipStream_t st = as_stream(stream);
  int64_t cnt = 0;
  int rc = overlay_labels(c, overlay_inout, labels, n, &cnt, st);
  if (rc == SCLAP_OK && n_clusters) *n_clusters = cnt;
  (void)hipStreamSynchronize(st);
  return rc;
}

static int cluster_impl(sclap_ctx* ctx, const sclap_csr* g, int64_t U, const sclap_lp_params* p,
                        const int32_t* blocks, int32_t member, int32_t* labels_out, int64_t* n_clusters,
                        sclap_round_stats* rs, void* stream) {
  if (!ctx) return fail(SCLAP_EINVAL, "ctx is NULL");
  SCLAP_TRY(check_csr(g));
  SCLAP_TRY(check_lp(p));
  if (g->n > 0 && !labels_out) return fail(SCLAP_EINVAL, "labels_out is NULL");
  if (g->n == 0) {
    // an empty graph, with no launch: no clusters; the 5% rule never holds
    // for 0 nodes, so every round runs (and moves nothing)
    if (n_clusters) *n_clusters = 0;
    if (rs) {
      std::memset(rs, 0, sizeof(*rs));
      rs->rounds = p->max_rounds;
    }
    return SCLAP_OK;
  }
  Ctx* c = &ctx->c;
  CtxScope scope(c);
  hipStream_t st = as_stream(stream);
  SCLAP_TRY(check_edge_total(c, g, st));
  Job j;
  j.kind = JOB_CLUSTER;
  j.U = U;
  j.k = 1;
  j.lp_rounds = p->max_rounds;
  j.stop_rule = p->stop_rule;
  j.dir_rule = p->direction_rule;
  j.subrounds = p->subrounds;
  j.member = member;
  j.part_out = labels_out;
  j.t_start = now_ms();
  std::memset(&j.rst, 0, sizeof(j.rst));
  int rc = job_set_input(c, &j, g, st);
  j.lv[0].blk = const_cast<int32_t*>(blocks);  // the caller's; not owned
  if (rc == SCLAP_OK) rc = level_totals(c, &j, &j.lv[0], nullptr, nullptr, st);
  if (rc == SCLAP_OK) rc = job_begin_cluster(c, &j, st);
  if (rc == SCLAP_OK) {
    std::vector<Job*> jobs{&j};
    rc = run_jobs(c, jobs, st);
  }
  if (rc == SCLAP_OK && n_clusters) {
    int32_t *used = nullptr, *cid = nullptr;
    const int64_t n = g->n;
    *n_clusters = 0;
    if (n > 0) {
      rc = dalloc_t(&used, (size_t)n, st);
      if (rc == SCLAP_OK) rc = dalloc_t(&cid, (size_t)n, st);
      if (rc == SCLAP_OK) rc = contract_flag(labels_out, g->row_ptr, n, 0, used, st);
      const size_t sb = prim_exscan_i32_bytes((size_t)n);
      if (rc == SCLAP_OK) rc = c->prim.ensure(sb, st);
      if (rc == SCLAP_OK) rc = prim_exscan_i32(c->prim.p, sb, used, cid, (size_t)n, st);
      if (rc == SCLAP_OK) rc = ctx_ensure_pin(c, 64);
      if (rc == SCLAP_OK) {
        int32_t* h = (int32_t*)c->pin;
        (void)hipMemcpyAsync(h, cid + n - 1, 4, hipMemcpyDeviceToHost, st);
        (void)hipMemcpyAsync(h + 1, used + n - 1, 4, hipMemcpyDeviceToHost, st);
        if (hipStreamSynchronize(st) != hipSuccess) rc = fail(SCLAP_EHIP, "sync");
        *n_clusters = (int64_t)h[0] + h[1];
      }
      dfree(used, st);
      dfree(cid, st);
    }
  }
  if (rs) *rs = j.rst;
  job_release_lp(&j, st, true);
  job_release_levels(&j, st);
  (void)hipStreamSynchronize(st);
  return rc;
}

int sclap_contract(sclap_ctx* ctx, const sclap_csr* g, const int32_t* labels, int32_t drop_isolated,
                   int32_t* coarse_of_out, sclap_graph** coarse_out, void* stream) {
  if (!ctx || !coarse_out) return fail(SCLAP_EINVAL, "NULL argument");
  *coarse_out = nullptr;
  SCLAP_TRY(check_csr(g));
  if (g->n > 0 && (!labels || !coarse_of_out)) return fail(SCLAP_EINVAL, "NULL labels or coarse_of_out");
  Ctx* c = &ctx->c;
  CtxScope scope(c);
  hipStream_t st = as_stream(stream);
  if (g->n == 0) {
    // an empty graph contracts to an empty graph: row_ptr = {0}
    Level L;
    SCLAP_TRY(dalloc_t(&L.own_rp, 1, st));
    int rc = fill_i64(L.own_rp, 1, 0, st);
    if (rc == SCLAP_OK) rc = hipStreamSynchronize(st) == hipSuccess ? SCLAP_OK : fail(SCLAP_EHIP, "sync");
    if (rc != SCLAP_OK) {
      dfree(L.own_rp, st);
      return rc;
    }
    L.rp = L.own_rp;
    L.rows_sorted = 1;
    sclap_graph* out = new sclap_graph();
    out->L = L;
    *coarse_out = out;
    return SCLAP_OK;
  }
  SCLAP_TRY(check_edge_total(c, g, st));
  Job j;
  j.kind = JOB_CLUSTER;
  int rc = job_set_input(c, &j, g, st);
  j.lab = const_cast<int32_t*>(labels);
  if (rc == SCLAP_OK) rc = contract_level(c, &j, 0, drop_isolated ? 1 : 0, st);
  if (rc == SCLAP_OK || rc == SCLAP_EOVERFLOW) {
    if (rc == SCLAP_OK) {
      if (g->n > 0) rc = copy_i32(j.lv[0].coarse_of, coarse_of_out, g->n, st);
      sclap_graph* out = new sclap_graph();
      out->L = j.lv[1];
      j.lv[1] = Level();
      *coarse_out = out;
    }
  }
  j.lab = nullptr;
  job_release_levels(&j, st);
  SCLAP_HIP(hipStreamSynchronize(st));
  return rc;
}

int sclap_graph_view(const sclap_graph* cg, sclap_csr* view) {
  if (!cg || !view) return fail(SCLAP_EINVAL, "NULL argument");
  view->n = cg->L.n;
  view->m = cg->L.m;
  view->row_ptr = cg->L.rp;
  view->col = cg->L.col;
  view->ew = cg->L.ew;
  view->nw = cg->L.nw;
  view->nw_bytes = 8;
  view->rows_sorted = 1;
  return SCLAP_OK;
}

int sclap_graph_copy(const sclap_graph* cg, int64_t* row_ptr, int32_t* col, int32_t* ew, int64_t* nw,
                     void* stream) {
  if (!cg || !row_ptr || (cg->L.m > 0 && (!col || !ew)) || (cg->L.n > 0 && !nw))
    return fail(SCLAP_EINVAL, "NULL argument");
  hipStream_t st = as_stream(stream);
  const Level& L = cg->L;
  SCLAP_HIP(hipMemcpyAsync(row_ptr, L.rp, (size_t)(L.n + 1) * 8, hipMemcpyDeviceToDevice, st));
  if (L.m > 0) {
    SCLAP_HIP(hipMemcpyAsync(col, L.col, (size_t)L.m * 4, hipMemcpyDeviceToDevice, st));
    SCLAP_HIP(hipMemcpyAsync(ew, L.ew, (size_t)L.m * 4, hipMemcpyDeviceToDevice, st));
  }
  if (L.n > 0) SCLAP_HIP(hipMemcpyAsync(nw, L.nw, (size_t)L.n * 8, hipMemcpyDeviceToDevice, st));
  return SCLAP_OK;
}

int sclap_graph_free(sclap_graph* cg) {
  if (!cg) return SCLAP_OK;
  (void)hipDeviceSynchronize();
  {
    Level& L = cg->L;
    dfree(L.own_rp, nullptr);
    dfree(L.own_col, nullptr);
    dfree(L.own_ew, nullptr);
    dfree(L.own_nw, nullptr);
    dfree(L.coarse_of, nullptr);
  }
  (void)hipDeviceSynchronize();
  delete cg;
  return SCLAP_OK;
}

int sclap_initial_partition(sclap_ctx* ctx, const sclap_csr* g, int32_t k, int32_t skip_isolated, int32_t* part_out,
                            void* stream) {
  if (!ctx) return fail(SCLAP_EINVAL, "ctx is NULL");
  SCLAP_TRY(check_csr(g));
  if (k < 1) return fail(SCLAP_EINVAL, "k must be >= 1");
  if (g->n > 0 && !part_out) return fail(SCLAP_EINVAL, "part_out is NULL");
  if (g->n == 0) return SCLAP_OK;  // an empty graph: nothing to place, no launch
  Ctx* c = &ctx->c;
  CtxScope scope(c);
  hipStream_t st = as_stream(stream);
  Job j;
  j.kind = skip_isolated ? JOB_PARTITION : JOB_REFINE;  // selects skip_isolated on level 0
  j.k = k;
  int rc = job_set_input(c, &j, g, st);
  int64_t C = 0;
  if (rc == SCLAP_OK) rc = level_totals(c, &j, &j.lv[0], &C, nullptr, st);
  if (rc == SCLAP_OK && C > 0 && (__int128)C * k >= ((__int128)1 << 62)) rc = fail(SCLAP_EOVERFLOW, "k * c(V)");
  if (rc == SCLAP_OK) {
    std::vector<Job*> jobs{&j};
    std::vector<int32_t*> parts{part_out};
    rc = ip_jobs(c, jobs, parts, st);
  }
  job_release_levels(&j, st);
  (void)hipStreamSynchronize(st);
  return rc;
}

int sclap_refine(sclap_ctx* ctx, const sclap_csr* g, int32_t k, int64_t lmax, const sclap_lp_params* p,
                 int32_t* part_inout, sclap_round_stats* rs, void* stream) {
  if (!ctx) return fail(SCLAP_EINVAL, "ctx is NULL");
  SCLAP_TRY(check_csr(g));
  SCLAP_TRY(check_lp(p));
  if (k < 1) return fail(SCLAP_EINVAL, "k must be >= 1");
  if (g->n > 0 && !part_inout) return fail(SCLAP_EINVAL, "part_inout is NULL");
  if (g->n == 0) {
    // an empty graph, with no launch: nothing moves, and the stop rule ends
    // the refinement after two such rounds
    if (rs) {
      std::memset(rs, 0, sizeof(*rs));
      rs->rounds = std::min<int32_t>(p->max_rounds, 2);
    }
    return SCLAP_OK;
  }
  Ctx* c = &ctx->c;
  CtxScope scope(c);
  hipStream_t st = as_stream(stream);
  SCLAP_TRY(check_edge_total(c, g, st));
  Job j;
  j.kind = JOB_REFINE;
  j.k = k;
  j.lmax = lmax;
  j.ref_rounds = p->max_rounds;
  j.dir_rule = p->direction_rule;
  j.t_start = now_ms();
  std::memset(&j.rst, 0, sizeof(j.rst));
  int rc = job_set_input(c, &j, g, st);
  if (rc == SCLAP_OK) rc = level_totals(c, &j, &j.lv[0], nullptr, nullptr, st);
  if (rc == SCLAP_OK) rc = job_begin_refine(c, &j, part_inout, false, st);
  if (rc == SCLAP_OK) {
    std::vector<Job*> jobs{&j};
    rc = run_jobs(c, jobs, st);
  }
  if (rs) *rs = j.rst;
  job_release_lp(&j, st, true);
  job_release_levels(&j, st);
  (void)hipStreamSynchronize(st);
  return rc;
}

int sclap_cut(sclap_ctx* ctx, const sclap_csr* g, const int32_t* part, int32_t k, int64_t* cut_out,
              int64_t* block_w_out, void* stream) {
  if (!ctx || !cut_out) return fail(SCLAP_EINVAL, "NULL argument");
  SCLAP_TRY(check_csr(g));
  if (k < 1) return fail(SCLAP_EINVAL, "k must be >= 1");
  Ctx* c = &ctx->c;
  CtxScope scope(c);
  hipStream_t st = as_stream(stream);
  SCLAP_TRY(c->small.ensure(256, st));
  unsigned long long* d = (unsigned long long*)((char*)c->small.p + 128);
  SCLAP_TRY(c->cutbuf.ensure((size_t)cut_partials(g->m) * 8, st));
  const int32_t* trow = nullptr;
  SCLAP_TRY(ctx_tile_rows(c, g->row_ptr, g->n, g->m, &trow, st));
  SCLAP_TRY(cut_edges(g->row_ptr, g->col, g->ew, part, g->n, g->m, d, (int64_t*)c->cutbuf.p, st, trow));
  SCLAP_TRY(ctx_ensure_pin(c, 64 + (size_t)k * 8));
  SCLAP_HIP(hipMemcpyAsync(c->pin, d, 8, hipMemcpyDeviceToHost, st));
  SCLAP_HIP(hipStreamSynchronize(st));
  *cut_out = c->pin[0];
  if (block_w_out) {
    int64_t *nw = nullptr, *B = nullptr;
    SCLAP_TRY(dalloc_t(&nw, (size_t)std::max<int64_t>(g->n, 1), st));
    SCLAP_TRY(dalloc_t(&B, (size_t)k, st));
    SCLAP_TRY(widen_nw(g->nw, g->nw_bytes, g->n, nw, st));
    SCLAP_TRY(block_weights(part, nw, g->n, k, B, st));
    SCLAP_HIP(hipMemcpyAsync(c->pin, B, (size_t)k * 8, hipMemcpyDeviceToHost, st));
    SCLAP_HIP(hipStreamSynchronize(st));
    std::memcpy(block_w_out, c->pin, (size_t)k * 8);
    dfree(nw, st);
    dfree(B, st);
  }
  return SCLAP_OK;
}

int sclap_partition(sclap_ctx* ctx, const sclap_csr* g, int32_t k, int64_t eps_num, int64_t eps_den,
                    const sclap_ml_params* p, int32_t* part_out, sclap_stats* stats, void* stream) {
  if (!ctx) return fail(SCLAP_EINVAL, "ctx is NULL");
  Ctx* c = &ctx->c;
  CtxScope scope(c);
  hipStream_t st = as_stream(stream);
  Job j;
  int rc = setup_partition_job(c, &j, g, k, eps_num, eps_den, p, part_out, st);
  if (rc == SCLAP_OK && j.stage != ST_DONE) {
    std::vector<Job*> jobs{&j};
    rc = run_jobs(c, jobs, st);
    if (rc == SCLAP_OK && j.stage == ST_ERROR) rc = j.status;
  }
  if (stats) *stats = j.st;
  job_release_lp(&j, st, false);
  job_release_levels(&j, st);
  (void)hipStreamSynchronize(st);
  return rc;
}

int sclap_partition_batch(sclap_ctx* ctx, int32_t count, const sclap_csr* gs, const int32_t* ks, int64_t eps_num,
                          int64_t eps_den, const sclap_ml_params* p, int32_t* const* parts_out, sclap_stats* sts,
                          void* stream) {
  if (!ctx || count < 0 || (count > 0 && (!gs || !ks || !parts_out))) return fail(SCLAP_EINVAL, "NULL argument");
  Ctx* c = &ctx->c;
  CtxScope scope(c);
  hipStream_t st = as_stream(stream);
  std::vector<Job> jobs((size_t)count);
  std::vector<Job*> ptrs;
  int rc = SCLAP_OK;
  for (int32_t i = 0; i < count && rc == SCLAP_OK; ++i) {
    rc = setup_partition_job(c, &jobs[i], &gs[i], ks[i], eps_num, eps_den, p, parts_out[i], st);
    ptrs.push_back(&jobs[i]);
  }
  if (rc == SCLAP_OK) rc = run_jobs(c, ptrs, st);
  for (int32_t i = 0; i < count; ++i) {
    if (rc == SCLAP_OK && jobs[i].stage == ST_ERROR) rc = jobs[i].status;
    if (sts) sts[i] = jobs[i].st;
    job_release_lp(&jobs[i], st, false);
    job_release_levels(&jobs[i], st);
  }
  (void)hipStreamSynchronize(st);
  return rc;
}

// Profiling of the rating step (used by the benchmark).
int sclap_profile_enable(sclap_ctx* ctx, int32_t on) {
  if (!ctx) return fail(SCLAP_EINVAL, "ctx is NULL");
  ctx->c.profile = on != 0;
  ctx->c.prof_rate_ms = 0;
  ctx->c.prof_rate_launches = 0;
  ctx->c.prof_rate_visits = 0;
  ctx->c.prof_rate_nodes = 0;
  ctx->c.prof_round_ms = 0;
  ctx->c.prof_rounds = 0;
  ctx->c.prof_k_launches = 0;
  for (int b = 0; b < kBins; ++b) {
    ctx->c.prof_k_ms[b] = 0;
    ctx->c.prof_k_bytes[b] = 0;
    ctx->c.prof_k_visits[b] = 0;
    ctx->c.prof_k_nodes[b] = 0;
    ctx->c.prof_k_group_launches[b] = 0;
  }
  return SCLAP_OK;
}

int sclap_profile_kernels(sclap_ctx* ctx, int32_t count, double* ms, double* bytes, int64_t* visits, int64_t* nodes,
                          int64_t* launches, int64_t* rounds) {
  if (!ctx || count < 0) return fail(SCLAP_EINVAL, "bad argument");
  const Ctx& c = ctx->c;
  for (int b = 0; b < count && b < kBins; ++b) {
    if (ms) ms[b] = c.prof_k_ms[b];
    if (bytes) bytes[b] = c.prof_k_bytes[b];
    if (visits) visits[b] = c.prof_k_visits[b];
    if (nodes) nodes[b] = c.prof_k_nodes[b];
    if (launches) launches[b] = c.prof_k_group_launches[b];
  }
  if (rounds) *rounds = c.prof_k_launches;
  return SCLAP_OK;
}

static bool valid_bin_bounds(const int32_t* hi) {
  int32_t lo = 32;
  for (int q = 0; q < 4; ++q) {
    if (hi[q] < lo || hi[q] > kBinHiCap[q]) return false;
    lo = hi[q];
  }
  return true;
}

int sclap_set_bin_bounds(sclap_ctx* ctx, const int32_t* hi) {
  if (!ctx || !hi) return fail(SCLAP_EINVAL, "NULL argument");
  if (!valid_bin_bounds(hi)) return fail(SCLAP_EINVAL, "bin bounds must rise from 32 and stay within 64/128/512/1024");
  for (int q = 0; q < 4; ++q) ctx->c.tune_hi[q] = hi[q];
  return SCLAP_OK;
}

int sclap_get_bin_bounds(sclap_ctx* ctx, int32_t* hi) {
  if (!ctx || !hi) return fail(SCLAP_EINVAL, "NULL argument");
  for (int q = 0; q < 4; ++q) hi[q] = ctx->c.tune_hi[q];
  return SCLAP_OK;
}

int sclap_autotune(sclap_ctx* ctx, const sclap_csr* g, int64_t U, int32_t rounds, int32_t* hi_out, double* best_ms,
                   double* default_ms, void* stream) {
  if (!ctx) return fail(SCLAP_EINVAL, "ctx is NULL");
  SCLAP_TRY(check_csr(g));
  if (rounds < 1 || rounds > SCLAP_MAX_ROUNDS) return fail(SCLAP_EINVAL, "rounds out of range");
  Ctx* c = &ctx->c;
  int32_t* lab = nullptr;
  {
    CtxScope scope(c);
    SCLAP_TRY(dalloc_t(&lab, (size_t)std::max<int64_t>(g->n, 1), as_stream(stream)));
  }
  // candidate bounds of bins 3..6: each bin may start where the one below
  // ends; the kernels' capacities cap them
  std::vector<std::array<int32_t, 4>> cand;
  for (int32_t h0 : {32, 64})
    for (int32_t h1 : {64, 128})
      for (int32_t h2 : {128, 256, 512})
        for (int32_t h3 : {512, 1024, 2048})
          if (h1 >= h0 && h2 >= h1 && h3 >= h2) cand.push_back({h0, h1, h2, h3});
  sclap_lp_params p{rounds, 0, 1, 0};
  const std::array<int32_t, 4> saved{c->tune_hi[0], c->tune_hi[1], c->tune_hi[2], c->tune_hi[3]};
  auto time_it = [&](const std::array<int32_t, 4>& hi, double* ms) -> int {
    for (int q = 0; q < 4; ++q) c->tune_hi[q] = hi[q];
    double best = 1e300;
    for (int rep = 0; rep < 2; ++rep) {
      const double t0 = now_ms();
      SCLAP_TRY(cluster_impl(ctx, g, U, &p, nullptr, 0, lab, nullptr, nullptr, stream));
      best = std::min(best, now_ms() - t0);
    }
    *ms = best;
    return SCLAP_OK;
  };
  int rc = SCLAP_OK;
  double dms = 0, bms = 1e300;
  std::array<int32_t, 4> best{kBinHiDefault[0], kBinHiDefault[1], kBinHiDefault[2], kBinHiDefault[3]};
  rc = time_it(best, &dms);
  bms = dms;
  for (size_t i = 0; rc == SCLAP_OK && i < cand.size(); ++i) {
    double ms = 0;
    rc = time_it(cand[i], &ms);
    if (rc == SCLAP_OK && ms < bms) {
      bms = ms;
      best = cand[i];
    }
  }
  {
    CtxScope scope(c);
    dfree(lab, as_stream(stream));
    (void)hipStreamSynchronize(as_stream(stream));
  }
  if (rc != SCLAP_OK) {
    for (int q = 0; q < 4; ++q) c->tune_hi[q] = saved[q];
    return rc;
  }
  for (int q = 0; q < 4; ++q) c->tune_hi[q] = best[q];
  if (hi_out)
    for (int q = 0; q < 4; ++q) hi_out[q] = best[q];
  if (best_ms) *best_ms = bms;
  if (default_ms) *default_ms = dms;
  return SCLAP_OK;
}

int sclap_path_counters(sclap_ctx* ctx, int32_t count, int64_t* out) {
  if (!ctx || count < 0 || (count > 0 && !out)) return fail(SCLAP_EINVAL, "bad argument");
  for (int i = 0; i < count && i < kPathCounters; ++i) out[i] = ctx->c.path_ctr[i].load(std::memory_order_relaxed);
  return SCLAP_OK;
}

int sclap_profile_read(sclap_ctx* ctx, double* rate_ms, int64_t* rate_launches, int64_t* visits, int64_t* nodes,
                       double* round_ms, int64_t* rounds) {
  if (!ctx) return fail(SCLAP_EINVAL, "ctx is NULL");
  const Ctx& c = ctx->c;
  if (rate_ms) *rate_ms = c.prof_rate_ms;
  if (rate_launches) *rate_launches = c.prof_rate_launches;
  if (visits) *visits = c.prof_rate_visits;
  if (nodes) *nodes = c.prof_rate_nodes;
  if (round_ms) *round_ms = c.prof_round_ms;
  if (rounds) *rounds = c.prof_rounds;
  return SCLAP_OK;
}

}  // extern "C"
