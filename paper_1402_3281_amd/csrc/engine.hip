// engine.hip -- host executor of the multilevel scheme (Section 1, Figure 1;
// Section 3.1): coarsening by size-constrained label propagation and cluster
// contraction, initial partition of the coarsest level, projection and label
// propagation local search on every level.  Every step fuses all jobs that are
// at that step into one set of launches.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <climits>
#include <cstring>
#include <string>

#include <mutex>
#include <unordered_map>

#include "engine.h"
#include "ext.h"

namespace sclap {

static thread_local std::string g_err;
void set_error(const std::string& msg) { g_err = msg; }
int fail(int code, const std::string& msg) {
  g_err = msg;
  return code;
}
const char* last_error_cstr() { return g_err.c_str(); }

double now_ms() {
  return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

int bits_for(int64_t count) {
  if (count <= 2) return 1;
  return 64 - __builtin_clzll((unsigned long long)(count - 1));
}

namespace {
thread_local Ctx* tls_ctx = nullptr;
std::mutex g_size_mu;
struct BlockInfo {
  size_t bytes;
  int device;
};
std::unordered_map<void*, BlockInfo> g_size;  // every live dalloc block

// Allocation classes: powers of two up to 1 MiB, then eighths of an octave.
size_t alloc_class(size_t bytes) {
  if (bytes <= 256) return 256;
  if (bytes <= (1u << 20)) {
    size_t c = 256;
    while (c < bytes) c <<= 1;
    return c;
  }
  const int lg = 63 - __builtin_clzll((unsigned long long)bytes);
  const size_t step = (size_t)1 << (lg - 3);
  return (bytes + step - 1) / step * step;
}
}  // namespace

CtxScope::CtxScope(Ctx* c) : prev(tls_ctx) { tls_ctx = c; }
CtxScope::~CtxScope() { tls_ctx = prev; }

void ctx_trim(Ctx* c) {
  if (c->cache.empty()) return;
  // a cached block may still be read by work queued before its release
  (void)hipDeviceSynchronize();
  for (const CachedBlock& b : c->cache) {
    (void)hipFree(b.p);
    std::lock_guard<std::mutex> lk(g_size_mu);
    g_size.erase(b.p);
  }
  c->cache.clear();
  c->cache_bytes = 0;
}

int dalloc(void** p, size_t bytes, hipStream_t st) {
  *p = nullptr;
  const size_t need = alloc_class(bytes == 0 ? 256 : bytes);
  Ctx* c = tls_ctx;
  if (c) {
    // best fit among cached blocks of this stream, at most 1/4 larger
    int best = -1;
    for (int i = 0; i < (int)c->cache.size(); ++i) {
      const CachedBlock& b = c->cache[i];
      if (b.st == st && b.bytes >= need && b.bytes <= need + need / 4 &&
          (best < 0 || b.bytes < c->cache[best].bytes))
        best = i;
    }
    if (best >= 0) {
      *p = c->cache[best].p;
      c->cache_bytes -= c->cache[best].bytes;
      c->cache[best] = c->cache.back();
      c->cache.pop_back();
      return SCLAP_OK;
    }
  }
  hipError_t e = hipMallocAsync(p, need, st);
  if (e == hipErrorOutOfMemory && c && !c->cache.empty()) {
    (void)hipGetLastError();
    ctx_trim(c);
    e = hipMallocAsync(p, need, st);
  }
  if (e != hipSuccess) {
    *p = nullptr;
    return fail(e == hipErrorOutOfMemory ? SCLAP_ENOMEM : SCLAP_EHIP,
                std::string("device allocation of ") + std::to_string(bytes) + " bytes: " + hipGetErrorString(e));
  }
  int dev = 0;
  (void)hipGetDevice(&dev);
  std::lock_guard<std::mutex> lk(g_size_mu);
  g_size[*p] = BlockInfo{need, dev};
  return SCLAP_OK;
}

void dfree(void* p, hipStream_t st) {
  if (!p) return;
  Ctx* c = tls_ctx;
  size_t bytes = 0;
  {
    std::lock_guard<std::mutex> lk(g_size_mu);
    auto it = g_size.find(p);
    if (it != g_size.end()) {
      bytes = it->second.bytes;
      if (c && it->second.device != c->device) c = nullptr;
      if (!c || c->cache_bytes + bytes > c->cache_limit) g_size.erase(it);
    }
  }
  if (c && bytes && c->cache_bytes + bytes <= c->cache_limit) {
    c->cache.push_back({p, bytes, st});
    c->cache_bytes += bytes;
    return;
  }
  (void)hipFreeAsync(p, st);
}

int Scratch::ensure(size_t need, hipStream_t st) {
  if (need <= bytes && p) return SCLAP_OK;
  release(st);
  size_t nb = need + need / 4 + 4096;
  SCLAP_TRY(dalloc(&p, nb, st));
  bytes = nb;
  return SCLAP_OK;
}

void Scratch::release(hipStream_t st) {
  dfree(p, st);
  p = nullptr;
  bytes = 0;
}

int ctx_ensure_pin(Ctx* c, size_t bytes) {
  if (bytes <= c->pin_bytes) return SCLAP_OK;
  if (c->pin) (void)hipHostFree(c->pin);
  c->pin = nullptr;
  size_t nb = std::max<size_t>(bytes, 1 << 16);
  SCLAP_HIP(hipHostMalloc((void**)&c->pin, nb, hipHostMallocDefault));
  c->pin_bytes = nb;
  return SCLAP_OK;
}

int ctx_tile_rows(Ctx* c, const int64_t* rp, int64_t n, int64_t m, const int32_t** out, hipStream_t st) {
  *out = nullptr;
  if (n <= 0 || m <= 0) return SCLAP_OK;
  SCLAP_TRY(c->trows.ensure((size_t)tile_rows_len(m) * sizeof(int32_t), st));
  SCLAP_TRY(tile_rows(rp, n, m, (int32_t*)c->trows.p, st));
  *out = (const int32_t*)c->trows.p;
  return SCLAP_OK;
}

void ctx_release(Ctx* c, hipStream_t st) {
  ctx_trim(c);
  Scratch* all[] = {&c->bins, &c->ckeys, &c->ckeys2, &c->tkey, &c->wv, &c->prefix, &c->prim, &c->hub_chunk,
                    &c->hub_tab, &c->hub_own, &c->hub_gkeys, &c->step_ctr, &c->small,
                    &c->slots_dev, &c->ip_slots, &c->hub_slice, &c->hub_best, &c->movers, &c->binfo,
                    &c->hub_maps, &c->binmeta, &c->hub_P, &c->hub_mat,
                    &c->binscr, &c->cutbuf, &c->tadm, &c->hub_keep, &c->trows, &c->part8, &c->lab8};
  for (Scratch* s : all) s->release(st);
  (void)hipStreamSynchronize(st);
  if (c->pin) (void)hipHostFree(c->pin);
  if (c->pin_slots) (void)hipHostFree(c->pin_slots);
  c->pin = nullptr;
  c->pin_slots = nullptr;
  c->pin_bytes = c->pin_slots_cap = 0;
  for (auto& ev : c->ev) (void)hipEventDestroy(ev);
}

int ctx_ensure_slots(Ctx* c, size_t count) {
  if (count <= c->pin_slots_cap) return SCLAP_OK;
  if (c->pin_slots) (void)hipHostFree(c->pin_slots);
  c->pin_slots = nullptr;
  size_t nc = std::max<size_t>(count, 64);
  SCLAP_HIP(hipHostMalloc((void**)&c->pin_slots, nc * sizeof(DevSlot), hipHostMallocDefault));
  c->pin_slots_cap = nc;
  return SCLAP_OK;
}

// ---------------------------------------------------------------------------
// Levels and jobs.
// ---------------------------------------------------------------------------
int job_set_input(Ctx* c, Job* j, const sclap_csr* g, hipStream_t st) {
  (void)c;
  j->lv.clear();
  j->lv.emplace_back();
  Level& L = j->lv[0];
  L.n = g->n;
  L.m = g->m;
  L.rp = g->row_ptr;
  L.col = g->col;
  L.ew = g->ew;
  L.rows_sorted = g->rows_sorted;
  SCLAP_TRY(dalloc_t(&L.own_nw, (size_t)std::max<int64_t>(g->n, 1), st));
  SCLAP_TRY(widen_nw(g->nw, g->nw_bytes, g->n, L.own_nw, st));
  L.nw = L.own_nw;
  return SCLAP_OK;
}

int job_compact_input(Ctx* c, Job* j, hipStream_t st) {
  Level& L = j->lv[0];
  const int64_t n = L.n, m = L.m, n0 = L.n_active;
  if (n0 == n || n0 == 0) return SCLAP_OK;
  const int64_t W = (n + 63) / 64;
  uint64_t* words = nullptr;
  int32_t *wcnt = nullptr, *wpre = nullptr;
  SCLAP_TRY(dalloc_t(&words, (size_t)W, st));
  SCLAP_TRY(dalloc_t(&wcnt, (size_t)W, st));
  SCLAP_TRY(dalloc_t(&wpre, (size_t)W, st));
  SCLAP_TRY(active_words(L.rp, n, words, wcnt, st));
  const size_t sb = prim_exscan_i32_bytes((size_t)W);
  SCLAP_TRY(c->prim.ensure(sb, st));
  SCLAP_TRY(prim_exscan_i32(c->prim.p, sb, wcnt, wpre, (size_t)W, st));
  dfree(wcnt, st);
  Level C;
  C.n = n0;
  C.m = m;
  C.rows_sorted = L.rows_sorted;
  SCLAP_TRY(dalloc_t(&C.own_rp, (size_t)n0 + 1, st));
  SCLAP_TRY(dalloc_t(&C.own_col, (size_t)std::max<int64_t>(m, 1), st));
  SCLAP_TRY(dalloc_t(&C.own_nw, (size_t)n0, st));
  SCLAP_TRY(dalloc_t(&j->act, (size_t)n0, st));
  uint8_t* rec = nullptr;
  SCLAP_TRY(dalloc_t(&rec, (size_t)compact_rec_bytes(n), st));
  SCLAP_TRY(compact_graph(L.rp, L.col, L.nw, words, wpre, n, m, n0, C.own_rp, C.own_col, C.own_nw, j->act, rec, st));
  dfree(words, st);
  dfree(wpre, st);
  dfree(rec, st);
  C.rp = C.own_rp;
  C.col = C.own_col;
  C.ew = L.ew;  // entries keep their places
  C.nw = C.own_nw;
  // the totals carry over (no sync): degrees are unchanged, and a node's
  // degree never exceeds n0 - 1, so the hub layout sizes are the same; the
  // largest weight may only shrink, which keeps the input's a valid bound
  C.n_active = n0;
  C.max_deg = L.max_deg;
  C.max_w = L.max_w;
  C.hubs = L.hubs;
  C.hub_stage = L.hub_stage;
  C.hub_parts_c = L.hub_parts_c;
  C.hub_mat_c = L.hub_mat_c;
  C.hub_parts_r = L.hub_parts_r;
  C.hub_mat_r = L.hub_mat_r;
  j->input = L;
  j->lv[0] = C;
  j->compact = true;
  return SCLAP_OK;
}

int level_totals(Ctx* c, Job* j, Level* L, int64_t* sum_w, int64_t* max_w, hipStream_t st) {
  SCLAP_TRY(c->small.ensure(256, st));
  unsigned long long* d = (unsigned long long*)c->small.p;
  SCLAP_TRY(graph_totals(L->rp, L->nw, L->n, std::max<int64_t>(j->k, 1), d, st));
  SCLAP_TRY(ctx_ensure_pin(c, 128));
  SCLAP_HIP(hipMemcpyAsync(c->pin, d, kGraphTotals * sizeof(int64_t), hipMemcpyDeviceToHost, st));
  SCLAP_HIP(hipStreamSynchronize(st));
  if (sum_w) *sum_w = c->pin[0];
  if (max_w) *max_w = c->pin[1];
  L->n_active = c->pin[2];
  L->hub_stage = c->pin[3];
  L->hubs = c->pin[4];
  L->hub_parts_c = c->pin[5];
  L->hub_mat_c = c->pin[6];
  L->hub_parts_r = c->pin[7];
  L->hub_mat_r = c->pin[8];
  L->max_deg = c->pin[9];
  L->max_w = c->pin[1];
  return SCLAP_OK;
}

void job_release_lp(Job* j, hipStream_t st, bool keep_lab) {
  if (!keep_lab && j->lab_owned) dfree(j->lab, st);
  if (!keep_lab) j->lab = nullptr;
  j->lab_owned = false;
  dfree(j->desire, st);
  dfree(j->adm, st);
  dfree(j->Wt, st);
  dfree(j->inc, st);
  dfree(j->fcur, st);
  dfree(j->fnext, st);
  dfree(j->conn, st);
  j->conn = nullptr;
  j->desire = nullptr;
  j->adm = nullptr;
  j->Wt = nullptr;
  j->inc = nullptr;
  j->fcur = nullptr;
  j->fnext = nullptr;
}

static void level_free(Level& L, hipStream_t st) {
  dfree(L.own_rp, st);
  dfree(L.own_col, st);
  dfree(L.own_ew, st);
  dfree(L.own_nw, st);
  dfree(L.coarse_of, st);
  if (L.blk_owned) dfree(L.blk, st);
  L.own_rp = nullptr;
  L.own_col = nullptr;
  L.own_ew = nullptr;
  L.own_nw = nullptr;
  L.coarse_of = nullptr;
  L.blk = nullptr;
  L.blk_owned = false;
}

void job_release_ext(Job* j, hipStream_t st) {
  if (j->flt_on) level_free(j->flt, st);
  j->flt = Level();
  j->flt_on = false;
  dfree(j->cls, st);
  j->cls = nullptr;
}

void job_release_levels(Job* j, hipStream_t st) {
  for (auto& L : j->lv) level_free(L, st);
  level_free(j->input, st);
  dfree(j->act, st);
  j->act = nullptr;
  job_release_ext(j, st);
  dfree(j->ovl, st);
  j->ovl = nullptr;
  dfree(j->best, st);
  j->best = nullptr;
}

int job_begin_cluster(Ctx* c, Job* j, hipStream_t st) {
  Level& L = j->lv[j->cur];
  const int64_t n = L.n;
  const size_t nn = (size_t)std::max<int64_t>(n, 1);
  if (L.blk && !j->flt_on) {
    // clustering that respects the level's blocks rates the level without
    // its cut edges (built once per level, shared by the ensemble members)
    SCLAP_TRY(build_respect_graph(c, L, L.blk, &j->flt, st));
    j->flt_on = true;
    SCLAP_TRY(level_totals(c, j, &j->flt, nullptr, nullptr, st));
  }
  if (j->subrounds > 1 && !j->cls) {
    SCLAP_TRY(dalloc_t(&j->cls, nn, st));
    SCLAP_TRY(degree_classes(L.rp, n, j->subrounds, j->cls, st));
  }
  if (j->kind == JOB_CLUSTER) {
    j->lab = j->part_out;
    j->lab_owned = false;
  } else {
    SCLAP_TRY(dalloc_t(&j->lab, nn, st));
    j->lab_owned = true;
  }
  SCLAP_TRY(dalloc_t(&j->desire, nn, st));
  SCLAP_TRY(dalloc_t(&j->adm, nn, st));
  SCLAP_TRY(dalloc_t(&j->Wt, nn, st));
  SCLAP_TRY(dalloc_t(&j->inc, nn, st));
  SCLAP_TRY(fill_i64(j->inc, n, 0, st));
  if (j->member == 0) SCLAP_TRY(init_cluster(j->lab, j->desire, j->Wt, L.nw, n, st));
  else SCLAP_TRY(begin_member_labels(c, j, st));
  j->nlabels = n;
  j->round = 1;
  j->sub = 0;
  j->sub_moved = 0;
  j->sub_visits = 0;
  j->lp_gen += 1;
  j->wt_clusters = true;
  j->moved_prev = 0;
  j->n_stop = (j->cur == 0 && j->kind == JOB_PARTITION) ? L.n_active : L.n;
  j->stage = ST_COARSEN;
  return SCLAP_OK;
}

int job_begin_refine(Ctx* c, Job* j, int32_t* part, bool owned, hipStream_t st) {
  (void)c;
  Level& L = j->lv[j->cur];
  const int64_t n = L.n;
  const size_t nn = (size_t)std::max<int64_t>(n, 1);
  const size_t kk = (size_t)std::max<int32_t>(j->k, 1);
  j->lab = part;
  j->lab_owned = owned;
  SCLAP_TRY(dalloc_t(&j->desire, nn, st));
  SCLAP_TRY(dalloc_t(&j->adm, nn, st));
  SCLAP_TRY(dalloc_t(&j->Wt, kk, st));
  SCLAP_TRY(dalloc_t(&j->inc, kk, st));
  SCLAP_TRY(dalloc_t(&j->fcur, nn, st));
  SCLAP_TRY(dalloc_t(&j->fnext, nn, st));
  SCLAP_TRY(fill_i64(j->inc, j->k, 0, st));
  j->conn_stale = false;
  if (j->k <= kConnMaxK && n > 0) {
    // block connections: built in the first round, kept by every move
    SCLAP_TRY(dalloc_t(&j->conn, (size_t)n * kk, st));
    SCLAP_TRY(fill_i32(j->conn, n * (int64_t)j->k, 0, st));
  }
  SCLAP_TRY(fill_u8(j->fnext, n, 0, st));
  SCLAP_TRY(fill_u8(j->fcur, n, 0, st));
  SCLAP_TRY(copy_i32(part, j->desire, n, st));
  SCLAP_TRY(block_weights(part, L.nw, n, j->k, j->Wt, st));
  // extra imbalance on the coarse levels of the first cycle (Section 4)
  j->lmax_cur = j->kind == JOB_PARTITION && j->cycle == 0
                    ? level_lmax(j->total_w, j->k, j->eps_num, j->eps_den, j->delta_num, j->delta_den,
                                 j->st.levels, j->cur, j->lmax)
                    : j->lmax;
  j->nlabels = j->k;
  j->round = 1;
  j->lp_gen += 1;
  j->zero_streak = 0;
  j->stage = ST_REFINE;
  return SCLAP_OK;
}

// ---------------------------------------------------------------------------
// One fused LP round.
// ---------------------------------------------------------------------------
int lp_round(Ctx* c, std::vector<Job*>& jobs, hipStream_t st) {
  const int ns = (int)jobs.size();
  if (ns == 0) return SCLAP_OK;
  SCLAP_TRY(ctx_ensure_slots(c, (size_t)ns));
  int64_t N = 0, Lt = 0, T_bin = 0, hub_stage = 0, hub_parts = 0, hub_mat = 0, max_tiles = 0;
  int64_t bin_max_deg = 0;  // largest degree of a slot whose nodes go to the bins
  int32_t lo5 = kBinHiCap[1], lo7 = kBinHiCap[3];  // smallest lower bounds of bins 5 and 7 over the slots
  bool hubs_ident = true;   // every slot with hubs is in its first clustering round
  bool tiny_graph = false;  // a binned slot with fewer than 32 entries (degree <= 64 in the 64-lane bin)
  SCLAP_TRY(c->small.ensure(512 + (size_t)ns * CTR_N * sizeof(int64_t) + 4096, st));
  int64_t* ctr = (int64_t*)((char*)c->small.p + 512);
  uint32_t* table_err = (uint32_t*)((char*)c->small.p + 256) + 17;
  bool any_build = false, any_cached = false, any_tile = false, any_other = false, any_binned = false;
  bool any_plain = false;  // a slot rated from the bins (no block connections)
  int tile_kmax = 0;
  for (int s = 0; s < ns; ++s) {
    Job* j = jobs[s];
    const bool refine = j->stage == ST_REFINE;
    // a clustering that respects a partition rates the level without its cut edges
    const Level& L = !refine && j->flt_on ? j->flt : j->lv[j->cur];
    DevSlot& d = c->pin_slots[s];
    std::memset(&d, 0, sizeof(d));
    d.rp = L.rp;
    d.col = L.col;
    d.ew = L.ew;
    d.nw = L.nw;
    d.lab = j->lab;
    d.desire = j->desire;
    d.adm = j->adm;
    d.W = j->Wt;
    d.inc = j->inc;
    d.flag_cur = j->fcur;
    d.flag_next = j->fnext;
    d.ctr = ctr + (size_t)s * CTR_N;
    d.err = table_err;
    d.n = L.n;
    d.m = L.m;
    d.nbase = N;
    d.tbase = T_bin;
    d.nlabels = j->nlabels;
    d.lbase = Lt;
    d.cap = refine ? j->lmax_cur : j->U;
    d.round = j->round;
    d.mode = refine ? MODE_REFINE : MODE_CLUSTER;
    // clustering starts from lab(v) = v (ensemble member 0, before any move)
    d.ident = !refine && j->round == 1 && j->sub == 0 && j->member == 0 ? 1 : 0;
    // in that round W(t) = c(t), so with 2 max c <= U no candidate is ineligible
    d.all_elig = d.ident && 2 * L.max_w <= j->U ? 1 : 0;
    // degree-ordered sub-rounds rate the nodes of one degree class
    d.cls = !refine && j->subrounds > 1 ? j->cls : nullptr;
    d.sub = j->sub;
    // degree bins: tuned bounds for clustering, the defaults for refinement
    const int32_t* hi = refine ? kBinHiDefault : c->tune_hi;
    for (int q = 0; q < 4; ++q) d.bin_hi[q] = hi[q];
    lo5 = std::min(lo5, d.bin_hi[1]);
    lo7 = std::min(lo7, d.bin_hi[3]);
    if (L.hubs > 0 && !d.ident) hubs_ident = false;
    d.dir_rule = j->dir_rule;
    d.use_flags = refine && j->round > 1;
    d.conn = refine ? j->conn : nullptr;
    d.conn_k = j->k;
    d.conn_mode = d.conn ? (j->round == 1 || j->conn_stale ? CONN_BUILD : CONN_RATE) : CONN_NONE;
    d.last_round = j->round >= (refine ? j->ref_rounds : j->lp_rounds);
    any_build = any_build || d.conn_mode == CONN_BUILD;
    any_cached = any_cached || d.conn_mode == CONN_RATE;
    any_binned = any_binned || d.conn_mode != CONN_RATE;
    any_plain = any_plain || d.conn_mode == CONN_NONE;
    // refinement slots with few blocks are admitted by tiles
    if (refine && j->nlabels <= kConnMaxK) {
      any_tile = true;
      tile_kmax = std::max<int>(tile_kmax, (int)j->nlabels);
    } else {
      any_other = true;
    }
    N += L.n;
    T_bin += bin_tiles(L.n);
    max_tiles = std::max<int64_t>(max_tiles, bin_tiles(L.n));
    Lt += j->nlabels;
    if (d.conn_mode != CONN_RATE) {  // nodes rated from block connections skip the bins
      bin_max_deg = std::max<int64_t>(bin_max_deg, L.max_deg);
      tiny_graph = tiny_graph || L.m < 32;
      hub_stage += L.hub_stage;
      hub_parts += refine ? L.hub_parts_r : L.hub_parts_c;
      hub_mat += refine ? L.hub_mat_r : L.hub_mat_c;
    }
  }
  if (N >= ((int64_t)1 << 31) || Lt >= ((int64_t)1 << 32))
    return fail(SCLAP_EINVAL, "fused round larger than 2^31 nodes");
  // slots of at least kLab8Nodes nodes that build block connections gather
  // their neighbours' blocks from a byte copy of the blocks (a quarter of the
  // bytes to cache); smaller levels' blocks stay in the caches anyway, and a
  // batch of many small graphs would pay a launch per slot
  constexpr int64_t kLab8Nodes = (int64_t)1 << 20;
  auto wants_lab8 = [&](const DevSlot& d) { return d.conn_mode == CONN_BUILD && d.n >= kLab8Nodes; };
  bool any_lab8 = false;
  for (int s = 0; s < ns; ++s) any_lab8 = any_lab8 || wants_lab8(c->pin_slots[s]);
  if (any_lab8) {
    int64_t bytes = 0;
    for (int s = 0; s < ns; ++s)
      if (wants_lab8(c->pin_slots[s])) bytes += (c->pin_slots[s].n + 255) / 256 * 256;
    SCLAP_TRY(c->lab8.ensure((size_t)std::max<int64_t>(bytes, 256), st));
    int64_t off = 0;
    for (int s = 0; s < ns; ++s) {
      DevSlot& d = c->pin_slots[s];
      if (!wants_lab8(d)) continue;
      uint8_t* b = (uint8_t*)c->lab8.p + off;
      SCLAP_TRY(narrow_u8(d.lab, d.n, b, st));
      d.lab8 = b;
      off += (d.n + 255) / 256 * 256;
    }
  }
  const size_t Nz = (size_t)std::max<int64_t>(N, 1);
  SCLAP_TRY(c->bins.ensure(kBins * Nz * sizeof(int32_t), st));
  SCLAP_TRY(c->binfo.ensure(kBins * Nz * sizeof(uint64_t), st));
  // hub rating path (see HubLayout): per hub, per chunk and per label part
  const bool hubs = hub_stage > 0;
  const size_t map_cap = (size_t)std::max<int64_t>(hub_stage / kHubChunk, hub_parts) + 64;
  if (hubs) {
    SCLAP_TRY(c->hub_chunk.ensure((Nz + 1) * sizeof(uint32_t), st));
    SCLAP_TRY(c->hub_slice.ensure((Nz + 1) * sizeof(uint32_t), st));
    SCLAP_TRY(c->hub_tab.ensure((Nz + 1) * sizeof(int64_t), st));
    SCLAP_TRY(c->hub_P.ensure(Nz * sizeof(uint32_t), st));
    SCLAP_TRY(c->hub_maps.ensure(2 * map_cap * sizeof(uint32_t), st));
    SCLAP_TRY(c->hub_mat.ensure((size_t)std::max<int64_t>(hub_mat, 1) * sizeof(uint32_t), st));
    SCLAP_TRY(c->hub_gkeys.ensure((size_t)hub_stage * sizeof(int2), st));
  }
  if (c->hub_own.bytes < Nz * sizeof(int64_t) || !c->hub_own.p) {
    SCLAP_TRY(c->hub_own.ensure(Nz * sizeof(int64_t), st));
    SCLAP_TRY(fill_i64((int64_t*)c->hub_own.p, (int64_t)(c->hub_own.bytes / 8), 0, st));
  }
  if (c->hub_best.bytes < Nz * sizeof(int64_t) || !c->hub_best.p) {
    SCLAP_TRY(c->hub_best.ensure(Nz * sizeof(int64_t), st));
    SCLAP_TRY(fill_i64((int64_t*)c->hub_best.p, (int64_t)(c->hub_best.bytes / 8), 0, st));
  }
  // rated list, old blocks of the movers by rated position, big movers
  SCLAP_TRY(c->movers.ensure(3 * Nz * sizeof(int32_t), st));
  int32_t* rated = (int32_t*)c->movers.p;
  int32_t* mold = rated + Nz;
  int32_t* bigm = mold + Nz;
  SCLAP_TRY(c->ckeys.ensure(Nz * 8, st));
  SCLAP_TRY(c->slots_dev.ensure((size_t)ns * sizeof(DevSlot), st));
  DevSlot* S = (DevSlot*)c->slots_dev.p;
  // Per-round counters (zeroed together with the slot counters after them):
  // u32 [9] contended, [10] hub overflow, [11..12] hub chunks and label
  // parts, [13] refinement movers, [15] big movers, [16] contended set too
  // large for the one-workgroup path, [17] an LDS hash table filled up,
  // [18] movers with rows above 65536 entries, [20..21] mover entries
  // walked (u64, measurement only).  The binning results live in c->binmeta:
  // u32 [0..8] bin counts, [14] rated; u64 at byte 128: visits per bin.
  // Clustering rounds of the same jobs on the same levels rate the same
  // nodes, so their bins are reused.
  uint32_t* small = (uint32_t*)((char*)c->small.p + 256);
  SCLAP_TRY(c->binmeta.ensure(256, st));
  uint32_t* meta = (uint32_t*)c->binmeta.p;
  unsigned long long* bin_vis = (unsigned long long*)((char*)meta + 128);
  SCLAP_TRY(round_begin(c->pin_slots, ns, S, small, 64 + (int64_t)ns * CTR_N * 2, st));
  int32_t* bins = (int32_t*)c->bins.p;
  const int64_t bin_cap = (int64_t)Nz;
  std::vector<std::pair<const void*, int>> sig;
  bool all_cluster = true;
  for (int s = 0; s < ns; ++s) {
    sig.emplace_back(jobs[s], (int)jobs[s]->lp_gen);
    all_cluster = all_cluster && jobs[s]->stage == ST_COARSEN;
  }
  const bool reuse_bins = all_cluster && c->bin_sig_valid && sig == c->bin_sig && c->bin_cap_used == bin_cap;

  if (c->profile) SCLAP_HIP(hipEventRecord(c->ev[kRateGroups + 1], st));
  c->path_ctr[0].fetch_add(1, std::memory_order_relaxed);
  if (ns > 1) c->path_ctr[1].fetch_add(1, std::memory_order_relaxed);
  if (!reuse_bins && bin_scan_device_wide(T_bin)) c->path_ctr[2].fetch_add(1, std::memory_order_relaxed);
  if (hubs) c->path_ctr[4].fetch_add(1, std::memory_order_relaxed);
  uint64_t* binfo = (uint64_t*)c->binfo.p;
  if (!reuse_bins) {
    const size_t bsb = bin_scratch_bytes(T_bin);
    SCLAP_TRY(c->binscr.ensure(bsb, st));
    SCLAP_TRY(launch_bin(S, ns, T_bin, bins, binfo, bin_cap, meta, bin_vis, rated, meta + 14, c->binscr.p,
                         c->binscr.bytes, st));
    c->bin_sig = sig;
    c->bin_sig_valid = all_cluster;
    c->bin_cap_used = bin_cap;
  }
  HubLayout hub{};
  if (hubs) {
    hub.chunk_off = (uint32_t*)c->hub_chunk.p;
    hub.part_off = (uint32_t*)c->hub_slice.p;
    hub.mat_off = (int64_t*)c->hub_tab.p;
    hub.hub_P = (uint32_t*)c->hub_P.p;
    hub.chunk_hub = (uint32_t*)c->hub_maps.p;
    hub.part_hub = hub.chunk_hub + map_cap;
    hub.map_cap = (int64_t)map_cap;
    SCLAP_TRY(c->hub_keep.ensure(64, st));
    hub.totals = small + 11;
    hub.totals_kept = (uint32_t*)c->hub_keep.p;
    hub.parts_cap = hub_parts;
    hub.mat = (uint32_t*)c->hub_mat.p;
    hub.mat_cap = hub_mat;
    hub.stage = (int2*)c->hub_gkeys.p;
    hub.stage_cap = hub_stage;
    hub.own = (int64_t*)c->hub_own.p;
    hub.best = (unsigned long long*)c->hub_best.p;
    hub.overflow = small + 10;
  }
  bool unit_weights = true;
  for (int s = 0; s < ns; ++s) unit_weights = unit_weights && c->pin_slots[s].ew == nullptr;
  // rounds whose every slot rates from block connections leave the bins empty
  unsigned groups = 0;  // rating launch groups that ran
  if (any_plain) {
    // (binned nodes of CONN_BUILD slots are rated here too, and again, with
    // the same result, from their new rows below)
    SCLAP_TRY(launch_rate(S, ns, bins, binfo, bin_cap, meta, hub, N, hubs, unit_weights,
                          tiny_graph ? std::max<int64_t>(bin_max_deg, 64) : bin_max_deg, lo5, lo7, hubs_ident,
                          reuse_bins && c->hub_keep_valid, st,
                          c->profile ? c->ev : nullptr, &groups));
    c->hub_keep_valid = hubs;
  } else {
    // every binned slot builds its block connections and is rated from them
    if (any_binned && hubs) SCLAP_TRY(launch_hub_prep(S, ns, bins, bin_cap, meta, hub, st));
    c->hub_keep_valid = false;
    if (c->profile)
      for (int e = 0; e <= kRateGroups; ++e) SCLAP_HIP(hipEventRecord(c->ev[e], st));
  }
  if (any_build) SCLAP_TRY(launch_conn_build(S, ns, bins, binfo, bin_cap, meta, hub, N, hubs, st));
  if (any_cached || any_build) SCLAP_TRY(launch_rate_cached(S, ns, N, rated, meta + 14, st));
  const int node_bits = bits_for(N);
  const int lab_bits = bits_for(Lt);
  if (any_other) {
    SCLAP_TRY(launch_incoming_decide(S, ns, N, Lt, rated, meta + 14, (uint64_t*)c->ckeys.p, small + 9, node_bits,
                                     st));
    SCLAP_TRY(launch_contended_small(S, ns, (const uint64_t*)c->ckeys.p, small + 9, node_bits, small + 16, st));
  }
  if (any_tile) {
    // the binning scratch still holds this round's rated-list offsets
    const size_t tb = tile_adm_bytes(T_bin, tile_kmax);
    SCLAP_TRY(c->tadm.ensure(tb, st));
    SCLAP_TRY(launch_tile_admission(S, ns, rated, bin_rated_offsets(c->binscr.p, T_bin), T_bin, tile_kmax, max_tiles,
                                    c->tadm.p, c->tadm.bytes, mold, st));
  }
  bool any_refine = false, any_big = false;
  for (int s = 0; s < ns; ++s) {
    const bool r = c->pin_slots[s].mode == MODE_REFINE;
    any_refine = any_refine || r;
    any_big = any_big || (r && jobs[s]->lv[jobs[s]->cur].hubs > 0);  // rows above 4096 entries
  }
  int32_t* big = any_big ? bigm : nullptr;
  // measurement of the marking kernels: events around them, and the mover
  // entries they walk (u64 at words 20..21 of the round counters)
  unsigned long long* mark_entries = c->profile ? (unsigned long long*)(small + 20) : nullptr;
  hipEvent_t* mark_ev = c->profile ? c->ev + kRateGroups + 3 : nullptr;
  SCLAP_TRY(launch_apply(S, ns, N, rated, meta + 14, mold, big, small + 15, small + 18, (int64_t)Nz, any_other,
                         any_refine, small + 16, st, mark_ev, mark_entries));
  const size_t rd = 256 + (size_t)ns * CTR_N * sizeof(int64_t);
  SCLAP_TRY(ctx_ensure_pin(c, rd + 512));
  SCLAP_HIP(hipMemcpyAsync(c->pin, small, rd, hipMemcpyDeviceToHost, st));
  SCLAP_HIP(hipStreamSynchronize(st));
  const uint32_t* hs = (const uint32_t*)c->pin;
  if (hs[10] || hs[17]) {
    // a hub label part beyond its LDS table, a layout beyond its sizes, or a
    // hash table that filled up: the counters that are kept zero between
    // rounds may be left nonzero, so they are cleared before the error
    SCLAP_TRY(fill_i64((int64_t*)c->hub_own.p, (int64_t)(c->hub_own.bytes / 8), 0, st));
    SCLAP_TRY(fill_i64((int64_t*)c->hub_best.p, (int64_t)(c->hub_best.bytes / 8), 0, st));
    (void)hipStreamSynchronize(st);
    return fail(SCLAP_EHIP, hs[10] ? "hub rating: a label part exceeds its table"
                                   : "rating or admission: an LDS hash table filled up");
  }
  if (hs[16]) {
    // contended set too large for one workgroup: device-wide sort and scan,
    // then the apply step that was skipped
    c->path_ctr[3].fetch_add(1, std::memory_order_relaxed);
    const uint32_t cc = hs[9];
    SCLAP_TRY(c->ckeys2.ensure((size_t)cc * 8, st));
    SCLAP_TRY(c->tkey.ensure((size_t)cc * 4, st));
    SCLAP_TRY(c->wv.ensure((size_t)cc * 8, st));
    SCLAP_TRY(c->prefix.ensure((size_t)cc * 8, st));
    const size_t tb = std::max(prim_sort_keys_bytes(cc), prim_scan_by_key_bytes(cc));
    SCLAP_TRY(c->prim.ensure(tb, st));
    SCLAP_TRY(prim_sort_keys(c->prim.p, tb, (const uint64_t*)c->ckeys.p, (uint64_t*)c->ckeys2.p, cc,
                             node_bits + lab_bits, st));
    SCLAP_TRY(launch_contended_split(S, ns, (const uint64_t*)c->ckeys2.p, cc, node_bits, (uint32_t*)c->tkey.p,
                                     (int64_t*)c->wv.p, st));
    SCLAP_TRY(prim_scan_by_key(c->prim.p, tb, (const uint32_t*)c->tkey.p, (const int64_t*)c->wv.p,
                               (int64_t*)c->prefix.p, cc, st));
    SCLAP_TRY(launch_contended_mark(S, ns, (const uint64_t*)c->ckeys2.p, cc, node_bits,
                                    (const int64_t*)c->prefix.p, st));
    SCLAP_TRY(launch_contended_add(S, ns, (const uint64_t*)c->ckeys2.p, cc, node_bits,
                                   (const int64_t*)c->prefix.p, st));
    SCLAP_TRY(launch_apply(S, ns, N, rated, meta + 14, mold, big, small + 15, small + 18, (int64_t)Nz, any_other,
                           any_refine, nullptr, st, mark_ev, mark_entries));
    SCLAP_HIP(hipMemcpyAsync(c->pin, small, rd, hipMemcpyDeviceToHost, st));
    SCLAP_HIP(hipStreamSynchronize(st));
  }
  if (c->profile) SCLAP_HIP(hipEventRecord(c->ev[kRateGroups + 2], st));
  // slot counters follow the lp counters: expose them at c->pin for the caller
  const int64_t* sctr = (const int64_t*)((const char*)c->pin + 256);
  if (c->profile) {
    SCLAP_HIP(hipStreamSynchronize(st));
    uint32_t* hm = (uint32_t*)((char*)c->pin + rd);
    SCLAP_HIP(hipMemcpyAsync(hm, meta, 256, hipMemcpyDeviceToHost, st));
    SCLAP_HIP(hipStreamSynchronize(st));
    const unsigned long long* hv = (const unsigned long long*)((const char*)hm + 128);
    bool weighted = false, gather = false;  // gather: some slot reads its neighbours' labels
    for (int s = 0; s < ns; ++s) {
      weighted = weighted || c->pin_slots[s].ew != nullptr;
      gather = gather || !c->pin_slots[s].ident;
    }
    const int group_of[kBins] = {0, 0, 0, 1, 1, 2, 2, 3, 4};
    for (int g = 0; g < kRateGroups; ++g) {
      float ms = 0;
      SCLAP_HIP(hipEventElapsedTime(&ms, c->ev[g], c->ev[g + 1]));
      c->prof_k_ms[g] += ms;
      if ((groups >> g) & 1u) c->prof_k_group_launches[g] += 1;
    }
    for (int b = 0; b < kBins; ++b) {
      const int g = group_of[b];
      if (!((groups >> g) & 1u)) continue;  // binned for the block connections only
      c->prof_k_visits[g] += (int64_t)hv[b];
      c->prof_k_nodes[g] += hm[b];
      c->prof_k_bytes[g] += (double)hv[b] * (4.0 + (weighted ? 4.0 : 0.0) + (gather ? 4.0 : 0.0)) + (double)hm[b] * 32.0;
      c->prof_rate_nodes += hm[b];
    }
    float a = 0, b2 = 0;
    SCLAP_HIP(hipEventElapsedTime(&a, c->ev[0], c->ev[kRateGroups]));
    SCLAP_HIP(hipEventElapsedTime(&b2, c->ev[kRateGroups + 1], c->ev[kRateGroups + 2]));
    c->prof_rate_ms += a;
    c->prof_rate_launches += 1;
    c->prof_k_launches += 1;
    c->prof_round_ms += b2;
    c->prof_rounds += 1;
    for (int s = 0; s < ns; ++s) c->prof_rate_visits += sctr[(size_t)s * CTR_N + CTR_VISITS];
    if (any_refine) {
      // marking group (kMarkGroup): per rated position its id and old block
      // (8 B); per mover its row offsets and new block (20 B); per entry of
      // a mover's row the neighbour id and its rated-set flag (5 B), and,
      // when the round's moves are added to the block connections, the
      // edge weight (weighted levels) and two 4-byte read-modify-writes
      float mm = 0;
      SCLAP_HIP(hipEventElapsedTime(&mm, c->ev[kRateGroups + 3], c->ev[kRateGroups + 4]));
      const uint64_t ent = *(const unsigned long long*)((const char*)c->pin + 80);
      int64_t movers = 0;
      bool push = false;
      for (int s = 0; s < ns; ++s) {
        const DevSlot& d = c->pin_slots[s];
        if (d.mode != MODE_REFINE) continue;
        const int64_t mv = sctr[(size_t)s * CTR_N + CTR_MOVED];
        movers += mv;
        push = push || (d.conn && !d.last_round && mv * kConnPushDiv <= d.n);
      }
      c->prof_k_ms[kMarkGroup] += mm;
      c->prof_k_group_launches[kMarkGroup] += 1;
      c->prof_k_nodes[kMarkGroup] += movers;
      c->prof_k_visits[kMarkGroup] += (int64_t)ent;
      c->prof_k_bytes[kMarkGroup] += 8.0 * hm[14] + 20.0 * (double)movers +
                                     (double)ent * (5.0 + (push ? 16.0 + (weighted ? 4.0 : 0.0) : 0.0));
    }
  }
  // move the slot counters to the front of the staging buffer; a clustering
  // round rates every node of degree > 0, so its edge visits are the level's m
  std::memmove(c->pin, sctr, (size_t)ns * CTR_N * sizeof(int64_t));
  for (int s = 0; s < ns; ++s) {
    const Job* j = jobs[s];
    if (j->stage == ST_COARSEN && j->subrounds <= 1)
      c->pin[(size_t)s * CTR_N + CTR_VISITS] = j->flt_on ? j->flt.m : j->lv[j->cur].m;
  }
  return SCLAP_OK;
}

// ---------------------------------------------------------------------------
// Contraction of level i into level i + 1 (Section 3.1, Figure 2).
// ---------------------------------------------------------------------------
int contract_level(Ctx* c, Job* j, int i, int drop, hipStream_t st) {
  Level& F = j->lv[i];
  const int64_t n = F.n;
  const size_t nn = (size_t)std::max<int64_t>(n, 1);
  int32_t *used = nullptr, *cid = nullptr;
  SCLAP_TRY(dalloc_t(&used, nn, st));
  SCLAP_TRY(dalloc_t(&cid, nn, st));
  SCLAP_TRY(contract_flag(j->lab, F.rp, n, drop, used, st));
  const size_t sb = prim_exscan_i32_bytes(nn);
  SCLAP_TRY(c->prim.ensure(sb, st));
  SCLAP_TRY(prim_exscan_i32(c->prim.p, sb, used, cid, (size_t)n, st));
  SCLAP_TRY(ctx_ensure_pin(c, 64));
  int64_t nc = 0;
  if (n > 0) {
    int32_t* h = (int32_t*)c->pin;
    SCLAP_HIP(hipMemcpyAsync(h, cid + n - 1, 4, hipMemcpyDeviceToHost, st));
    SCLAP_HIP(hipMemcpyAsync(h + 1, used + n - 1, 4, hipMemcpyDeviceToHost, st));
    SCLAP_HIP(hipStreamSynchronize(st));
    nc = (int64_t)h[0] + h[1];
  }
  Level C;
  C.n = nc;
  C.rows_sorted = 1;
  SCLAP_TRY(dalloc_t(&F.coarse_of, nn, st));
  SCLAP_TRY(dalloc_t(&C.own_nw, (size_t)std::max<int64_t>(nc, 1), st));
  // after a clustering of this level, the label weights are the cluster weights
  const int64_t* Wl = (j->wt_clusters && j->Wt && j->nlabels == n && j->kind == JOB_PARTITION) ? j->Wt : nullptr;
  SCLAP_TRY(contract_coarse_of(j->lab, F.rp, F.nw, n, drop, cid, F.coarse_of, C.own_nw, nc, used, Wl, st));
  dfree(used, st);
  dfree(cid, st);
  const int bits = bits_for(nc);
  SCLAP_TRY(c->small.ensure(256, st));
  // unit edge weights: the sums are the run lengths of the sorted keys;
  // weighted keys of at most kPackedKeyBits bits carry their weight in the
  // low half of one 64-bit item (one key-only sort instead of key-value pairs)
  const bool unit = F.ew == nullptr;
  const bool packed = !unit && 2 * bits <= kPackedKeyBits;
  // the cross entries (one per undirected edge, at most m/2 of the m
  // entries of a symmetric graph; room for m), then their count
  const size_t cz = (size_t)std::max<int64_t>(F.m, 1);
  uint64_t *k1 = nullptr, *k2 = nullptr;
  int32_t *v1 = nullptr, *v2 = nullptr;
  SCLAP_TRY(dalloc_t(&k1, cz, st));
  if (!unit && !packed) SCLAP_TRY(dalloc_t(&v1, cz, st));
  unsigned long long* cursor = (unsigned long long*)((char*)c->small.p + 96);
  const int32_t* trow = nullptr;
  SCLAP_TRY(ctx_tile_rows(c, F.rp, n, F.m, &trow, st));
  SCLAP_TRY(contract_cross(F.rp, F.col, F.ew, F.coarse_of, n, F.m, bits, cursor, k1, v1, packed ? 1 : 0, trow, st));
  SCLAP_HIP(hipMemcpyAsync(c->pin, cursor, 8, hipMemcpyDeviceToHost, st));
  SCLAP_HIP(hipStreamSynchronize(st));
  const int64_t mx = c->pin[0];
  if (mx < 0 || mx > F.m) return fail(SCLAP_EHIP, "contraction: cross entry count out of range");
  const size_t mz = (size_t)std::max<int64_t>(mx, 1);
  SCLAP_TRY(dalloc_t(&k2, mz, st));
  if (!unit && !packed) SCLAP_TRY(dalloc_t(&v2, mz, st));
  const size_t tb = unit     ? std::max(prim_sort_keys_bytes(mz), prim_rle_bytes(mz))
                    : packed ? std::max(prim_sort_keys_bytes(mz), prim_reduce_packed_bytes(mz))
                             : std::max(prim_sort_pairs_bytes(mz), prim_reduce_by_key_bytes(mz));
  SCLAP_TRY(c->prim.ensure(tb, st));
  if (unit) SCLAP_TRY(prim_sort_keys(c->prim.p, tb, k1, k2, (size_t)mx, 2 * bits, st));
  else if (packed) SCLAP_TRY(prim_sort_keys(c->prim.p, tb, k1, k2, (size_t)mx, 32 + 2 * bits, st, 32));
  else SCLAP_TRY(prim_sort_pairs(c->prim.p, tb, k1, k2, v1, v2, (size_t)mx, 2 * bits, st));
  // reduce equal (x, y) keys: unique keys into k1, sums into an int64 buffer
  int64_t* aggs = nullptr;
  SCLAP_TRY(dalloc_t(&aggs, mz, st));
  uint32_t* ucount = (uint32_t*)((char*)c->small.p + 64);
  SCLAP_TRY(fill_u32(ucount, 2, 0, st));
  if (mx > 0) {
    if (unit) SCLAP_TRY(prim_rle(c->prim.p, tb, k2, k1, aggs, ucount, (size_t)mx, st));
    else if (packed) SCLAP_TRY(prim_reduce_packed(c->prim.p, tb, k2, k1, aggs, ucount, (size_t)mx, st));
    else SCLAP_TRY(prim_reduce_by_key(c->prim.p, tb, k2, v2, k1, aggs, ucount, (size_t)mx, st));
  }
  SCLAP_HIP(hipMemcpyAsync(c->pin, ucount, 4, hipMemcpyDeviceToHost, st));
  SCLAP_HIP(hipStreamSynchronize(st));
  // k1[0, mh): the coarse edges x < y with their weights; the mirror (y, x)
  // is sorted on its own and the two halves are placed row by row
  const int64_t mh = (int64_t)((uint32_t*)c->pin)[0];
  const int64_t mc = 2 * mh;
  C.m = mc;
  dfree(k2, st);
  k2 = nullptr;
  dfree(v2, st);
  v2 = nullptr;
  const bool mpacked = 2 * bits <= kPackedKeyBits;
  const size_t hz = (size_t)std::max<int64_t>(mh, 1);
  uint64_t *mk = nullptr, *mks = nullptr;
  int32_t *mw = nullptr, *mws = nullptr;
  SCLAP_TRY(dalloc_t(&mk, hz, st));
  SCLAP_TRY(dalloc_t(&mks, hz, st));
  if (!mpacked) {
    SCLAP_TRY(dalloc_t(&mw, hz, st));
    SCLAP_TRY(dalloc_t(&mws, hz, st));
  }
  unsigned* ovf = (unsigned*)ucount + 1;
  SCLAP_TRY(contract_mirror(k1, aggs, mh, bits, mpacked ? 1 : 0, mk, mw, ovf, st));
  if (mh > 0) {
    const size_t tb2 = mpacked ? prim_sort_keys_bytes(hz) : prim_sort_pairs_bytes(hz);
    SCLAP_TRY(c->prim.ensure(tb2, st));
    // the mirror keys y * 2^bits + x come in ascending (x, y) order, so a
    // stable sort by y alone leaves every row's x ascending
    if (mpacked) SCLAP_TRY(prim_sort_keys(c->prim.p, tb2, mk, mks, (size_t)mh, 32 + 2 * bits, st, 32 + bits));
    else SCLAP_TRY(prim_sort_pairs(c->prim.p, tb2, mk, mks, mw, mws, (size_t)mh, 2 * bits, st, bits));
  }
  dfree(mk, st);
  dfree(mw, st);
  int64_t *ru = nullptr, *rl = nullptr;
  SCLAP_TRY(dalloc_t(&ru, (size_t)nc + 1, st));
  SCLAP_TRY(dalloc_t(&rl, (size_t)nc + 1, st));
  SCLAP_TRY(dalloc_t(&C.own_rp, (size_t)nc + 1, st));
  SCLAP_TRY(dalloc_t(&C.own_col, (size_t)std::max<int64_t>(mc, 1), st));
  SCLAP_TRY(dalloc_t(&C.own_ew, (size_t)std::max<int64_t>(mc, 1), st));
  SCLAP_TRY(contract_finish2(k1, aggs, mh, mks, mws, mh, bits, mpacked ? 1 : 0, nc, ru, rl, C.own_rp, C.own_col,
                             C.own_ew, st));
  SCLAP_HIP(hipMemcpyAsync(c->pin, ovf, 4, hipMemcpyDeviceToHost, st));
  SCLAP_HIP(hipStreamSynchronize(st));
  const unsigned overflow = ((uint32_t*)c->pin)[0];
  dfree(ru, st);
  dfree(rl, st);
  dfree(mks, st);
  dfree(mws, st);
  dfree(k1, st);
  dfree(v1, st);
  dfree(aggs, st);
  C.rp = C.own_rp;
  C.col = C.own_col;
  C.ew = C.own_ew;
  C.nw = C.own_nw;
  if (F.blk) {
    // a coarse node takes the block its members share
    SCLAP_TRY(dalloc_t(&C.blk, (size_t)std::max<int64_t>(nc, 1), st));
    C.blk_owned = true;
    SCLAP_TRY(blocks_up(F.coarse_of, F.blk, n, C.blk, st));
  }
  j->lv.push_back(C);
  if (overflow) return fail(SCLAP_EOVERFLOW, "coarse edge weight exceeds int32");
  return SCLAP_OK;
}

// ---------------------------------------------------------------------------
// Fused initial partition: one workgroup per job.
// ---------------------------------------------------------------------------
constexpr int64_t kIpBigLevel = 1 << 18;  // entries of a BFS level expanded grid-wide

// Expand yielded BFS levels of one slot with grid-wide kernels until the
// workgroup kernel finishes.
static int ip_single_loop(Ctx* c, IpSlot* dslot, int64_t n, int64_t* dstate, hipStream_t st) {
  int64_t *deg = nullptr, *dpre = nullptr;
  int32_t *flags = nullptr, *fpos = nullptr;
  SCLAP_TRY(ctx_ensure_pin(c, 256));
  for (int iter = 0;; ++iter) {
    SCLAP_TRY(initial_partition(dslot, 1, n, 1, kIpBigLevel, st));
    SCLAP_HIP(hipMemcpyAsync(c->pin, dstate, 4 * sizeof(int64_t), hipMemcpyDeviceToHost, st));
    SCLAP_HIP(hipStreamSynchronize(st));
    if (c->pin[3] == 0) break;
    const int64_t head = c->pin[0], tail = c->pin[1], next = c->pin[2];
    const int64_t F = tail - head;
    // frontier degrees -> exclusive prefix (F + 1 entries, the last = E)
    SCLAP_TRY(dalloc_t(&deg, (size_t)F + 1, st));
    SCLAP_TRY(dalloc_t(&dpre, (size_t)F + 1, st));
    SCLAP_TRY(ip_level_deg(dslot, head, F, deg, st));
    size_t sb = prim_exscan_i64_bytes((size_t)F + 1);
    SCLAP_TRY(c->prim.ensure(sb, st));
    SCLAP_TRY(prim_exscan_i64(c->prim.p, sb, deg, dpre, (size_t)F + 1, st));
    SCLAP_HIP(hipMemcpyAsync(c->pin, dpre + F, 8, hipMemcpyDeviceToHost, st));
    SCLAP_HIP(hipStreamSynchronize(st));
    const int64_t E = c->pin[0];
    SCLAP_TRY(dalloc_t(&flags, (size_t)std::max<int64_t>(E, 1), st));
    SCLAP_TRY(dalloc_t(&fpos, (size_t)std::max<int64_t>(E, 1), st));
    SCLAP_TRY(ip_level_entries(dslot, head, F, dpre, E, 0, nullptr, st));
    SCLAP_TRY(ip_level_entries(dslot, head, F, dpre, E, 1, flags, st));
    sb = prim_exscan_i32_bytes((size_t)std::max<int64_t>(E, 1));
    SCLAP_TRY(c->prim.ensure(sb, st));
    SCLAP_TRY(prim_exscan_i32(c->prim.p, sb, flags, fpos, (size_t)E, st));
    int64_t T = 0;
    if (E > 0) {
      int32_t* h = (int32_t*)c->pin;
      SCLAP_HIP(hipMemcpyAsync(h, fpos + E - 1, 4, hipMemcpyDeviceToHost, st));
      SCLAP_HIP(hipMemcpyAsync(h + 1, flags + E - 1, 4, hipMemcpyDeviceToHost, st));
      SCLAP_HIP(hipStreamSynchronize(st));
      T = (int64_t)h[0] + h[1];
    }
    SCLAP_TRY(ip_level_emit(dslot, head, tail, F, dpre, E, flags, fpos, T, st));
    dfree(deg, st);
    dfree(dpre, st);
    dfree(flags, st);
    dfree(fpos, st);
    deg = nullptr;
    dpre = nullptr;
    flags = fpos = nullptr;
    c->pin[0] = tail;
    c->pin[1] = tail + T;
    c->pin[2] = next;
    c->pin[3] = 0;
    SCLAP_HIP(hipMemcpyAsync(dstate, c->pin, 4 * sizeof(int64_t), hipMemcpyHostToDevice, st));
    SCLAP_HIP(hipStreamSynchronize(st));
  }
  return SCLAP_OK;
}

int ip_jobs(Ctx* c, std::vector<Job*>& jobs, std::vector<int32_t*>& parts, hipStream_t st) {
  const int cnt = (int)jobs.size();
  if (cnt == 0) return SCLAP_OK;
  std::vector<IpSlot> hs(cnt);
  std::vector<int32_t*> scratch(cnt, nullptr);
  int64_t* states = nullptr;
  // 4 words of search state per slot, then the claim-table error flag
  SCLAP_TRY(dalloc_t(&states, (size_t)cnt * 4 + 1, st));
  SCLAP_TRY(fill_i64(states, (int64_t)cnt * 4 + 1, 0, st));
  uint32_t* ip_err = (uint32_t*)(states + (size_t)cnt * 4);
  for (int s = 0; s < cnt; ++s) {
    Job* j = jobs[s];
    const Level& L = j->lv[j->cur];
    const int64_t n = L.n;
    const size_t nn = (size_t)std::max<int64_t>(n, 1);
    SCLAP_TRY(dalloc_t(&scratch[s], 4 * nn, st));
    IpSlot& x = hs[s];
    x.rp = L.rp;
    x.col = L.col;
    x.nw = L.nw;
    x.n = n;
    x.k = j->k;
    x.skip_isolated = (j->cur == 0 && j->kind == JOB_PARTITION) ? 1 : 0;
    x.rows_sorted = L.rows_sorted;
    x.part = parts[s];
    x.order = scratch[s];
    x.pos = scratch[s] + nn;
    x.claim = scratch[s] + 2 * nn;
    x.cnt = scratch[s] + 3 * nn;
    x.state = states + 4 * s;
    x.err = ip_err;
    SCLAP_TRY(fill_i32(x.part, n, -1, st));
    SCLAP_TRY(fill_i32(x.pos, n, -1, st));
    SCLAP_TRY(fill_i32(x.claim, n, INT32_MAX, st));
  }
  SCLAP_TRY(c->ip_slots.ensure((size_t)cnt * sizeof(IpSlot), st));
  SCLAP_TRY(ctx_ensure_pin(c, (size_t)cnt * sizeof(IpSlot)));
  std::memcpy(c->pin, hs.data(), (size_t)cnt * sizeof(IpSlot));
  SCLAP_HIP(hipMemcpyAsync(c->ip_slots.p, c->pin, (size_t)cnt * sizeof(IpSlot), hipMemcpyHostToDevice, st));
  SCLAP_HIP(hipStreamSynchronize(st));  // pinned staging is reused right after
  const Level& L0 = jobs[0]->lv[jobs[0]->cur];
  int64_t max_n = 0;
  for (int s = 0; s < cnt; ++s) max_n = std::max<int64_t>(max_n, hs[s].n);
  if (cnt == 1 && L0.rows_sorted && L0.m > kIpBigLevel) {
    SCLAP_TRY(ip_single_loop(c, (IpSlot*)c->ip_slots.p, L0.n, states, st));
  } else {
    SCLAP_TRY(initial_partition((const IpSlot*)c->ip_slots.p, cnt, max_n, 0, 0, st));
  }
  SCLAP_TRY(ctx_ensure_pin(c, 64));
  SCLAP_HIP(hipMemcpyAsync(c->pin, ip_err, 4, hipMemcpyDeviceToHost, st));
  SCLAP_HIP(hipStreamSynchronize(st));
  const uint32_t err = *(const uint32_t*)c->pin;
  for (int s = 0; s < cnt; ++s) dfree(scratch[s], st);
  dfree(states, st);
  if (err) return fail(SCLAP_EHIP, "initial partition: the LDS claim table filled up");
  return SCLAP_OK;
}

// ---------------------------------------------------------------------------
// Executor.
// ---------------------------------------------------------------------------
static int64_t read_cut(Ctx* c, const Level& L, const int32_t* part, int32_t k, hipStream_t st) {
  if (c->small.ensure(256, st) != SCLAP_OK) return -1;
  unsigned long long* d = (unsigned long long*)((char*)c->small.p + 128);
  if (c->cutbuf.ensure((size_t)cut_partials(L.m) * 8, st) != SCLAP_OK) return -1;
  const int32_t* trow = nullptr;
  if (ctx_tile_rows(c, L.rp, L.n, L.m, &trow, st) != SCLAP_OK) return -1;
  // with k <= 256 the blocks are gathered from a byte copy of the partition
  const uint8_t* part8 = nullptr;
  if (k <= 256 && L.n > 0 && L.m > 0) {
    if (c->part8.ensure((size_t)L.n, st) != SCLAP_OK) return -1;
    if (narrow_u8(part, L.n, (uint8_t*)c->part8.p, st) != SCLAP_OK) return -1;
    part8 = (const uint8_t*)c->part8.p;
  }
  if (cut_edges(L.rp, L.col, L.ew, part, L.n, L.m, d, (int64_t*)c->cutbuf.p, st, trow, part8) != SCLAP_OK) return -1;
  if (ctx_ensure_pin(c, 64) != SCLAP_OK) return -1;
  if (hipMemcpyAsync(c->pin, d, 8, hipMemcpyDeviceToHost, st) != hipSuccess) return -1;
  if (hipStreamSynchronize(st) != hipSuccess) return -1;
  return c->pin[0];
}

// Allocate the block array of level i (level 0 writes the caller's buffer,
// unless level 0 is the input without its degree-0 nodes).
static int alloc_part(Job* j, int i, int32_t** out, bool* owned, hipStream_t st) {
  if (i == 0 && j->part_out && !j->compact) {
    *out = j->part_out;
    *owned = false;
    return SCLAP_OK;
  }
  *owned = true;
  return dalloc_t(out, (size_t)std::max<int64_t>(j->lv[i].n, 1), st);
}

static int finish_partition(Ctx* c, Job* j, hipStream_t st) {
  // the caller's graph: level 0, or the input that level 0 compacts
  Level& L = j->compact ? j->input : j->lv[0];
  int32_t* part = j->part_out;
  const int64_t k = j->k;
  if (j->compact) {
    // level 0's blocks go to their input nodes; the degree-0 nodes wait
    SCLAP_TRY(fill_i32(part, L.n, -1, st));
    SCLAP_TRY(scatter_i32(j->act, j->lab, j->lv[0].n, part, st));
    dfree(j->lab, st);
    j->lab = nullptr;
  }
  int64_t* B = nullptr;
  SCLAP_TRY(dalloc_t(&B, (size_t)k, st));
  if (j->st.n_isolated > 0) {
    SCLAP_TRY(block_weights(part, L.nw, L.n, j->k, B, st));
    int64_t *tw = nullptr, *tp = nullptr, *ends = nullptr;
    int32_t* last = nullptr;
    SCLAP_TRY(dalloc_t(&tw, (size_t)L.n, st));
    SCLAP_TRY(dalloc_t(&tp, (size_t)L.n, st));
    SCLAP_TRY(dalloc_t(&ends, (size_t)k, st));
    SCLAP_TRY(dalloc_t(&last, 1, st));
    const size_t sb = prim_exscan_i64_bytes((size_t)L.n);
    SCLAP_TRY(c->prim.ensure(sb, st));
    SCLAP_TRY(place_isolated(L.rp, L.nw, L.n, B, j->k, part, tw, tp, ends, last, c->prim.p, sb, st));
    dfree(tw, st);
    dfree(tp, st);
    dfree(ends, st);
    dfree(last, st);
  }
  SCLAP_TRY(block_weights(part, L.nw, L.n, j->k, B, st));
  const int64_t cut = read_cut(c, L, part, j->k, st);
  if (cut < 0) return fail(SCLAP_EHIP, "cut");
  SCLAP_TRY(ctx_ensure_pin(c, (size_t)k * 8));
  SCLAP_HIP(hipMemcpyAsync(c->pin, B, (size_t)k * 8, hipMemcpyDeviceToHost, st));
  SCLAP_HIP(hipStreamSynchronize(st));
  int64_t mb = 0;
  for (int64_t b = 0; b < k; ++b) mb = std::max(mb, c->pin[b]);
  dfree(B, st);
  j->st.cut = cut;
  j->st.max_block = mb;
  return SCLAP_OK;
}

// After the refinement of level cur: project to the next finer level or
// finish.
static int after_refine_level(Ctx* c, Job* j, hipStream_t st) {
  if (j->kind == JOB_REFINE) {
    job_release_lp(j, st, true);
    j->stage = ST_DONE;
    return SCLAP_OK;
  }
  if (j->cur == 0) {
    job_release_lp(j, st, true);
    j->stage = ST_FINISH;
    return SCLAP_OK;
  }
  const int fine = j->cur - 1;
  int32_t* pf = nullptr;
  bool owned = false;
  SCLAP_TRY(alloc_part(j, fine, &pf, &owned, st));
  SCLAP_TRY(project(j->lv[fine].coarse_of, j->lab, j->lv[fine].n, pf, st));
  job_release_lp(j, st, false);
  // the coarse level is no longer needed
  level_free(j->lv[j->cur], st);
  j->cur = fine;
  if (j->ref_rounds <= 0) {
    j->lab = pf;
    j->lab_owned = owned;
    return after_refine_level(c, j, st);
  }
  return job_begin_refine(c, j, pf, owned, st);
}

// Later cycles (Section 4, iterated multilevel algorithms): the coarsest
// level keeps the blocks of the cycle's start partition (same cut and block
// weights), with no initial partitioning.
static int start_from_blocks(Ctx* c, Job* j, hipStream_t st) {
  Level& L = j->lv[j->cur];
  int32_t* part = nullptr;
  bool owned = false;
  SCLAP_TRY(alloc_part(j, j->cur, &part, &owned, st));
  SCLAP_TRY(copy_i32(L.blk, part, L.n, st));
  j->st.ip_cut = read_cut(c, L, part, j->k, st);
  if (j->ref_rounds > 0) return job_begin_refine(c, j, part, owned, st);
  j->lab = part;
  j->lab_owned = owned;
  return after_refine_level(c, j, st);
}

static int start_ip_or_refine(Ctx* c, Job* j, std::vector<Job*>& ipq, hipStream_t st) {
  if (j->cycle > 0) return start_from_blocks(c, j, st);
  j->stage = ST_IP;
  ipq.push_back(j);
  return SCLAP_OK;
}

// After a clustering of the current level: the next ensemble member, or the
// contraction of the members' overlay (Section 4, ensemble clusterings).
static int after_member(Ctx* c, Job* j, hipStream_t st) {
  if (j->members <= 1) {
    j->stage = ST_CONTRACT;
    return SCLAP_OK;
  }
  const int64_t n = j->lv[j->cur].n;
  if (j->member == 0) {
    j->ovl = j->lab;  // the overlay starts as the first member's clustering
    j->lab = nullptr;
    j->lab_owned = false;
  } else {
    SCLAP_TRY(overlay_labels(c, j->ovl, j->lab, n, nullptr, st));
  }
  job_release_lp(j, st, false);
  if (j->member + 1 < j->members) {
    j->member += 1;
    return job_begin_cluster(c, j, st);
  }
  j->lab = j->ovl;
  j->lab_owned = true;
  j->ovl = nullptr;
  j->wt_clusters = false;  // the overlay's cluster weights are summed by the contraction
  j->member = 0;
  j->stage = ST_CONTRACT;
  return SCLAP_OK;
}

static int after_contract(Ctx* c, Job* j, std::vector<Job*>& ipq, hipStream_t st) {
  // level cur was just contracted into cur + 1
  const int64_t n_prev = j->cur == 0 ? j->lv[0].n_active : j->lv[j->cur].n;
  job_release_lp(j, st, false);
  job_release_ext(j, st);
  j->cur += 1;
  Level& L = j->lv[j->cur];
  SCLAP_TRY(level_totals(c, j, &L, nullptr, nullptr, st));
  j->st.levels = j->cur + 1;
  j->st.n_level[j->cur] = L.n;
  j->st.m_level[j->cur] = L.m;
  const bool stall = 20 * (n_prev - L.n) < n_prev;
  if (L.n > j->threshold && !stall && j->cur + 1 < SCLAP_MAX_LEVELS) return job_begin_cluster(c, j, st);
  return start_ip_or_refine(c, j, ipq, st);
}

// Iterated multilevel algorithms (Section 4; Appendix B.1): the next cycle
// starts from the best partition so far, clustering every level within its
// blocks.  Per-level statistics describe the last cycle.
static int begin_next_cycle(Ctx* c, Job* j, hipStream_t st) {
  j->cycle += 1;
  sclap_stats& S = j->st;
  S.levels = 1;
  for (int i = 1; i < SCLAP_MAX_LEVELS; ++i) {
    S.n_level[i] = 0;
    S.m_level[i] = 0;
  }
  std::memset(S.rounds_c, 0, sizeof(S.rounds_c));
  std::memset(S.rounds_r, 0, sizeof(S.rounds_r));
  std::memset(S.moved_c, 0, sizeof(S.moved_c));
  std::memset(S.moved_r, 0, sizeof(S.moved_r));
  std::memset(S.visits_c, 0, sizeof(S.visits_c));
  std::memset(S.visits_r, 0, sizeof(S.visits_r));
  S.ip_cut = 0;
  // the coarse levels of the last cycle are gone; level 0 is contracted anew
  for (size_t i = 1; i < j->lv.size(); ++i) level_free(j->lv[i], st);
  j->lv.resize(1);
  Level& L0 = j->lv[0];
  dfree(L0.coarse_of, st);
  L0.coarse_of = nullptr;
  if (j->compact) {
    // level 0 numbers only the input's nodes of degree > 0
    if (!L0.blk_owned) {
      SCLAP_TRY(dalloc_t(&L0.blk, (size_t)L0.n, st));
      L0.blk_owned = true;
    }
    SCLAP_TRY(gather_i32(j->act, j->best, L0.n, L0.blk, st));
  } else {
    L0.blk = j->best;
    L0.blk_owned = false;
  }
  j->cur = 0;
  j->member = 0;
  if (L0.n_active > j->threshold) return job_begin_cluster(c, j, st);
  return start_from_blocks(c, j, st);
}

// After the cut of a cycle's partition (part_out): keep it if it is the best
// so far (blocks within L_max first, then the smaller cut; ties keep the
// earlier cycle), then start the next cycle or finish with the best.
static int after_cycle(Ctx* c, Job* j, hipStream_t st) {
  sclap_stats& S = j->st;
  const int cy = j->cycle;
  int64_t vis = 0;
  for (int i = 0; i < S.levels; ++i) vis += S.visits_c[i] + S.visits_r[i];
  const int64_t cut = S.cut, mb = S.max_block;
  if (cy < SCLAP_MAX_CYCLES) {
    S.cycle_cut[cy] = cut;
    S.cycle_max_block[cy] = mb;
    S.cycle_visits[cy] = vis;
    S.cycle_levels[cy] = S.levels;
  }
  S.cycles = cy + 1;
  const int64_t over = mb > j->lmax ? 1 : 0;
  if (cy == 0 || over < j->best_over || (over == j->best_over && cut < j->best_cut)) {
    j->best_over = over;
    j->best_cut = cut;
    j->best_cycle = cy;
    if (j->vcycles > 1) {
      const int64_t n = j->compact ? j->input.n : j->lv[0].n;
      if (!j->best) SCLAP_TRY(dalloc_t(&j->best, (size_t)std::max<int64_t>(n, 1), st));
      SCLAP_TRY(copy_i32(j->part_out, j->best, n, st));
    }
  }
  S.best_cycle = j->best_cycle;
  S.cut = j->best_cut;
  S.max_block = S.cycle_max_block[j->best_cycle];
  if (cy + 1 < j->vcycles) return begin_next_cycle(c, j, st);
  const int64_t n_in = j->compact ? j->input.n : j->lv[0].n;
  if (j->best_cycle != cy) SCLAP_TRY(copy_i32(j->best, j->part_out, n_in, st));
  dfree(j->best, st);
  j->best = nullptr;
  if (j->lv[0].blk_owned) dfree(j->lv[0].blk, st);
  j->lv[0].blk = nullptr;
  j->lv[0].blk_owned = false;
  j->stage = ST_DONE;
  return SCLAP_OK;
}

// One step of the executor: one fused LP round over every job at an LP
// stage, then contractions, initial partitions and finishing.  Jobs whose
// stage is ST_IP on entry are partitioned in this step.  *all_done is set
// when every job is done or failed.
int step_jobs(Ctx* c, std::vector<Job*>& jobs, hipStream_t st, bool* all_done_out) {
  std::vector<Job*> ipq;
  for (Job* j : jobs)
    if (j->stage == ST_IP) ipq.push_back(j);
  // 1. LP rounds
  std::vector<Job*> lp;
  for (Job* j : jobs)
    if (j->stage == ST_COARSEN || j->stage == ST_REFINE) lp.push_back(j);
  if (!lp.empty()) {
    const double t0 = now_ms();
    SCLAP_TRY(lp_round(c, lp, st));
    const double dt = now_ms() - t0;
    for (size_t s = 0; s < lp.size(); ++s) {
      Job* j = lp[s];
      const int64_t moved = c->pin[s * CTR_N + CTR_MOVED];
      const int64_t visits = c->pin[s * CTR_N + CTR_VISITS];
      const int r = j->round;
      if (j->stage == ST_COARSEN) {
        j->st.ms_cluster += dt;
        j->rst.ms += dt;
        int64_t mv = moved, vs = visits;
        if (j->subrounds > 1) {
          // a round is its sub-rounds, one degree class each (Section 4 node order)
          j->sub_moved += moved;
          j->sub_visits += visits;
          j->lp_gen += 1;
          if (j->sub + 1 < j->subrounds) {
            j->sub += 1;
            continue;
          }
          mv = j->sub_moved;
          vs = j->sub_visits;
          j->sub = 0;
          j->sub_moved = 0;
          j->sub_visits = 0;
        }
        // ensemble members add up per round (moves) and per level (visits)
        j->st.moved_c[j->cur][r - 1] += mv;
        j->st.visits_c[j->cur] += vs;
        j->rst.moved[r - 1] = mv;
        j->rst.visits += vs;
        bool done = r >= j->lp_rounds;
        if (j->stop_rule == 1 && r >= 2 && 20 * (mv + j->moved_prev) < j->n_stop) done = true;
        j->moved_prev = mv;
        if (done) {
          j->st.rounds_c[j->cur] = std::max(j->st.rounds_c[j->cur], r);
          j->rst.rounds = r;
          if (j->kind == JOB_CLUSTER) {
            j->stage = ST_DONE;
            job_release_lp(j, st, true);
            job_release_ext(j, st);
          } else {
            SCLAP_TRY(after_member(c, j, st));
          }
        } else {
          j->round = r + 1;
        }
      } else {
        j->st.ms_refine += dt;
        j->st.moved_r[j->cur][r - 1] = moved;
        j->st.visits_r[j->cur] += visits;
        j->rst.moved[r - 1] = moved;
        j->rst.visits += visits;
        j->rst.ms += dt;
        j->zero_streak = moved == 0 ? j->zero_streak + 1 : 0;
        j->conn_stale = c->pin[s * CTR_N + CTR_STALE] != 0;
        const bool done = r >= j->ref_rounds || j->zero_streak >= 2;
        if (done) {
          j->st.rounds_r[j->cur] = r;
          j->rst.rounds = r;
          SCLAP_TRY(after_refine_level(c, j, st));
        } else {
          std::swap(j->fcur, j->fnext);  // the binning kernel clears the new fnext
          j->round = r + 1;
        }
      }
    }
  }
  // 2. contractions
  for (Job* j : jobs) {
    if (j->stage != ST_CONTRACT) continue;
    const double t0 = now_ms();
    int rc = contract_level(c, j, j->cur, j->cur == 0 ? 1 : 0, st);
    if (rc == SCLAP_EOVERFLOW) {
      j->status = rc;
      j->stage = ST_ERROR;
      job_release_lp(j, st, false);
      continue;
    }
    SCLAP_TRY(rc);
    SCLAP_TRY(after_contract(c, j, ipq, st));
    j->st.ms_contract += now_ms() - t0;
  }
  // 3. initial partitions
  if (!ipq.empty()) {
    const double t0 = now_ms();
    std::vector<int32_t*> parts(ipq.size());
    std::vector<bool> owned(ipq.size());
    for (size_t s = 0; s < ipq.size(); ++s) {
      bool o = false;
      SCLAP_TRY(alloc_part(ipq[s], ipq[s]->cur, &parts[s], &o, st));
      owned[s] = o;
    }
    SCLAP_TRY(ip_jobs(c, ipq, parts, st));
    const double dt = now_ms() - t0;
    for (size_t s = 0; s < ipq.size(); ++s) {
      Job* j = ipq[s];
      j->st.ms_initial += dt;
      j->st.ip_cut = read_cut(c, j->lv[j->cur], parts[s], j->k, st);
      if (j->ref_rounds > 0) {
        SCLAP_TRY(job_begin_refine(c, j, parts[s], owned[s], st));
      } else {
        j->lab = parts[s];
        j->lab_owned = owned[s];
        SCLAP_TRY(after_refine_level(c, j, st));
      }
    }
    ipq.clear();
  }
  // 4. finish
  bool all_done = true;
  for (Job* j : jobs) {
    if (j->stage == ST_FINISH) {
      SCLAP_TRY(finish_partition(c, j, st));
      SCLAP_TRY(after_cycle(c, j, st));
    }
    if (j->stage == ST_DONE && j->st.ms_total == 0) j->st.ms_total = now_ms() - j->t_start;
    if (j->stage != ST_DONE && j->stage != ST_ERROR) all_done = false;
  }
  *all_done_out = all_done;
  return SCLAP_OK;
}

int run_jobs(Ctx* c, std::vector<Job*>& jobs, hipStream_t st) {
  // cached bins are keyed by job addresses, which other calls may reuse
  c->bin_sig_valid = false;
  for (;;) {
    bool done = false;
    SCLAP_TRY(step_jobs(c, jobs, st, &done));
    if (done) break;
  }
  c->bin_sig_valid = false;
  return SCLAP_OK;
}

}  // namespace sclap
