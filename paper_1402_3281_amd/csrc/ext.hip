// ext.hip -- executor steps of the Section 4 extensions: the graph that a
// partition-respecting clustering rates (Appendix B.1), the overlay of
// ensemble members, and the coarse-level bounds with extra imbalance.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "edges.h"
#include "engine.h"
#include "ext.h"
#include "lp.h"
#include "misc.h"

namespace sclap {

int build_respect_graph(Ctx* c, const Level& L, const int32_t* blk, Level* F, hipStream_t st) {
  *F = Level();
  F->n = L.n;
  F->nw = L.nw;
  F->rows_sorted = L.rows_sorted;
  const int64_t n = L.n, m = L.m;
  const int64_t T = filter_tiles(m);
  const size_t words = (size_t)std::max<int64_t>(T * (kEpb / kWave), 1);
  uint64_t* kw = nullptr;
  uint32_t* wpre = nullptr;
  int64_t *tcnt = nullptr, *toff = nullptr;
  SCLAP_TRY(dalloc_t(&kw, words, st));
  SCLAP_TRY(dalloc_t(&wpre, words, st));
  SCLAP_TRY(dalloc_t(&tcnt, (size_t)T + 1, st));
  SCLAP_TRY(dalloc_t(&toff, (size_t)T + 1, st));
  SCLAP_TRY(fill_i64(tcnt + T, 1, 0, st));
  const int32_t* trow = nullptr;
  SCLAP_TRY(ctx_tile_rows(c, L.rp, n, m, &trow, st));
  SCLAP_TRY(filter_mark(L.rp, L.col, blk, n, m, kw, wpre, tcnt, trow, st));
  const size_t sb = prim_exscan_i64_bytes((size_t)T + 1);
  SCLAP_TRY(c->prim.ensure(sb, st));
  SCLAP_TRY(prim_exscan_i64(c->prim.p, sb, tcnt, toff, (size_t)T + 1, st));
  SCLAP_TRY(ctx_ensure_pin(c, 64));
  SCLAP_HIP(hipMemcpyAsync(c->pin, toff + T, 8, hipMemcpyDeviceToHost, st));
  SCLAP_HIP(hipStreamSynchronize(st));
  const int64_t m2 = c->pin[0];
  const size_t mz = (size_t)std::max<int64_t>(m2, 1);
  SCLAP_TRY(dalloc_t(&F->own_rp, (size_t)n + 1, st));
  SCLAP_TRY(dalloc_t(&F->own_col, mz, st));
  if (L.ew) SCLAP_TRY(dalloc_t(&F->own_ew, mz, st));
  SCLAP_TRY(filter_place(L.col, L.ew, m, kw, wpre, toff, F->own_col, F->own_ew, st));
  SCLAP_TRY(filter_rows(L.rp, n, m, kw, wpre, toff, T, F->own_rp, st));
  dfree(kw, st);
  dfree(wpre, st);
  dfree(tcnt, st);
  dfree(toff, st);
  F->m = m2;
  F->rp = F->own_rp;
  F->col = F->own_col;
  F->ew = L.ew ? F->own_ew : nullptr;
  return SCLAP_OK;
}

int begin_member_labels(Ctx* c, Job* j, hipStream_t st) {
  (void)c;
  // a partition's level 0 already numbers only the input's nodes of degree > 0
  const Level& L = j->lv[j->cur];
  return init_member(j->lab, j->desire, j->Wt, L.nw, L.n, j->member, st);
}

int overlay_labels(Ctx* c, int32_t* O, const int32_t* C, int64_t n, int64_t* count, hipStream_t st) {
  if (count) *count = 0;
  if (n <= 0) return SCLAP_OK;
  const size_t nz = (size_t)n;
  const int bits = bits_for(n);
  uint64_t *k1 = nullptr, *k2 = nullptr;
  int32_t *v1 = nullptr, *v2 = nullptr, *head = nullptr, *hx = nullptr, *segmin = nullptr, *first = nullptr,
          *rank = nullptr;
  SCLAP_TRY(dalloc_t(&k1, nz, st));
  SCLAP_TRY(dalloc_t(&k2, nz, st));
  SCLAP_TRY(dalloc_t(&v1, nz, st));
  SCLAP_TRY(dalloc_t(&v2, nz, st));
  SCLAP_TRY(overlay_keys(O, C, n, bits, k1, v1, st));
  const size_t tb = std::max(prim_sort_pairs_bytes(nz), prim_exscan_i32_bytes(nz));
  SCLAP_TRY(c->prim.ensure(tb, st));
  SCLAP_TRY(prim_sort_pairs(c->prim.p, tb, k1, k2, v1, v2, nz, 2 * bits, st));
  dfree(k1, st);
  dfree(v1, st);
  SCLAP_TRY(dalloc_t(&head, nz, st));
  SCLAP_TRY(dalloc_t(&hx, nz, st));
  SCLAP_TRY(overlay_heads(k2, n, head, st));
  dfree(k2, st);
  SCLAP_TRY(prim_exscan_i32(c->prim.p, tb, head, hx, nz, st));
  SCLAP_TRY(dalloc_t(&segmin, nz, st));
  SCLAP_TRY(dalloc_t(&first, nz, st));
  SCLAP_TRY(dalloc_t(&rank, nz, st));
  SCLAP_TRY(fill_i32(first, n, 0, st));
  SCLAP_TRY(overlay_first(v2, head, hx, n, segmin, first, st));
  SCLAP_TRY(prim_exscan_i32(c->prim.p, tb, first, rank, nz, st));
  SCLAP_TRY(overlay_assign(v2, head, hx, segmin, rank, n, O, st));
  if (count) {
    SCLAP_TRY(ctx_ensure_pin(c, 64));
    int32_t* h = (int32_t*)c->pin;
    SCLAP_HIP(hipMemcpyAsync(h, hx + n - 1, 4, hipMemcpyDeviceToHost, st));
    SCLAP_HIP(hipMemcpyAsync(h + 1, head + n - 1, 4, hipMemcpyDeviceToHost, st));
    SCLAP_HIP(hipStreamSynchronize(st));
    *count = (int64_t)h[0] + h[1];
  }
  dfree(v2, st);
  dfree(head, st);
  dfree(hx, st);
  dfree(segmin, st);
  dfree(first, st);
  dfree(rank, st);
  return SCLAP_OK;
}

int64_t level_lmax(int64_t C, int32_t k, int64_t eps_num, int64_t eps_den, int64_t dnum, int64_t dden, int32_t q,
                   int32_t i, int64_t lmax) {
  if (i <= 0 || dnum <= 0 || dden <= 0 || q - i <= 0) return lmax;
  const __int128 ck = (C + k - 1) / k;
  const __int128 span = q - i;
  const __int128 num = ck * ((__int128)(eps_den + eps_num) * dden * span + (__int128)dnum * eps_den);
  const __int128 den = (__int128)eps_den * dden * span;
  return (int64_t)(num / den);
}

}  // namespace sclap
