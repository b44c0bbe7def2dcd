/*
 * seq_sclap.c -- the paper's sequential size-constrained label propagation,
 * used only as a QUALITY reference for the synchronous oracle (test
 * infrastructure; never on the product path).
 *
 * Section 3.1: nodes are visited one at a time and each moves at once to the
 * eligible cluster with the strongest connection, against the current
 * cluster weights.  Section 4 (node ordering): nodes are visited in
 * increasing degree.  Random tie breaking is replaced by the smallest label.
 * As local search (Section 3.1, last paragraph) the cap is L_max and a node
 * of an overloaded block ignores its own block; the active-nodes scheme of
 * Section 4 / Appendix B.2 (two FIFO queues and two bit vectors) picks the
 * nodes of later rounds.
 */
#include <stdlib.h>
#include <string.h>

#include "sclap_oracle.h"

static inline int64_t nwt(const orc_graph* g, int64_t v) { return g->nw ? g->nw[v] : 1; }
static inline int64_t ewt(const orc_graph* g, int64_t e) { return g->ew ? (int64_t)g->ew[e] : 1; }

static const orc_graph* g_sort;
static int cmp_deg(const void* a, const void* b) {
  int32_t x = *(const int32_t*)a, y = *(const int32_t*)b;
  int64_t dx = g_sort->rp[x + 1] - g_sort->rp[x], dy = g_sort->rp[y + 1] - g_sort->rp[y];
  if (dx != dy) return dx < dy ? -1 : 1;
  return (x > y) - (x < y);
}

static int32_t* degree_order(const orc_graph* g) {
  int32_t* ord = (int32_t*)malloc(sizeof(int32_t) * (size_t)(g->n > 0 ? g->n : 1));
  for (int64_t v = 0; v < g->n; ++v) ord[v] = (int32_t)v;
  g_sort = g;
  qsort(ord, (size_t)g->n, sizeof(int32_t), cmp_deg);
  return ord;
}

/* Visit v: move to the best eligible label; returns 1 if it moved. */
static int visit(const orc_graph* g, int32_t v, int32_t* lab, int64_t* Wt, int64_t cap, int refine,
                 int64_t* conn, int32_t* touched) {
  int32_t own = lab[v];
  int64_t nt = 0;
  for (int64_t e = g->rp[v]; e < g->rp[v + 1]; ++e) {
    int32_t t = lab[g->col[e]];
    if (conn[t] == 0) touched[nt++] = t;
    conn[t] += ewt(g, e);
  }
  int32_t best_t = -1;
  int64_t best_c = -1;
  if (!(refine && Wt[own] > cap)) {
    best_t = own;
    best_c = conn[own];
  }
  for (int64_t i = 0; i < nt; ++i) {
    int32_t t = touched[i];
    if (t == own || Wt[t] + nwt(g, v) > cap) continue;
    if (conn[t] > best_c || (conn[t] == best_c && t < best_t)) {
      best_c = conn[t];
      best_t = t;
    }
  }
  for (int64_t i = 0; i < nt; ++i) conn[touched[i]] = 0;
  if (best_t < 0 || best_t == own) return 0;
  Wt[own] -= nwt(g, v);
  Wt[best_t] += nwt(g, v);
  lab[v] = best_t;
  return 1;
}

/* Sequential size-constrained clustering: at most max_rounds rounds in
 * increasing-degree order, stopping when fewer than 5% of the nodes moved. */
int32_t seq_cluster(const orc_graph* g, int64_t U, int32_t max_rounds, int32_t* lab) {
  int64_t n = g->n;
  int64_t* Wt = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
  int64_t* conn = (int64_t*)calloc((size_t)(n > 0 ? n : 1), sizeof(int64_t));
  int32_t* touched = (int32_t*)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
  int32_t* ord = degree_order(g);
  for (int64_t v = 0; v < n; ++v) {
    lab[v] = (int32_t)v;
    Wt[v] = nwt(g, v);
  }
  int32_t r;
  for (r = 1; r <= max_rounds; ++r) {
    int64_t moved = 0;
    for (int64_t i = 0; i < n; ++i) moved += visit(g, ord[i], lab, Wt, U, 0, conn, touched);
    if (20 * moved < n) break;
  }
  free(Wt);
  free(conn);
  free(touched);
  free(ord);
  return r > max_rounds ? max_rounds : r;
}

/* Sequential label propagation local search with active nodes. */
static int32_t seq_refine(const orc_graph* g, int32_t k, int64_t lmax, int32_t max_rounds, int32_t* part) {
  int64_t n = g->n;
  int64_t* Wb = (int64_t*)calloc((size_t)k, sizeof(int64_t));
  int64_t* conn = (int64_t*)calloc((size_t)k, sizeof(int64_t));
  int32_t* touched = (int32_t*)malloc(sizeof(int32_t) * (size_t)(k > 0 ? k : 1));
  int32_t* q[2];
  uint8_t* inq[2];
  for (int i = 0; i < 2; ++i) {
    q[i] = (int32_t*)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    inq[i] = (uint8_t*)calloc((size_t)(n > 0 ? n : 1), 1);
  }
  for (int64_t v = 0; v < n; ++v) Wb[part[v]] += nwt(g, v);
  int32_t* ord = degree_order(g);
  int64_t qn[2] = {n, 0};
  memcpy(q[0], ord, sizeof(int32_t) * (size_t)n);
  memset(inq[0], 1, (size_t)n);
  free(ord);
  int32_t r, cur = 0;
  for (r = 1; r <= max_rounds && qn[cur] > 0; ++r) {
    int nx = 1 - cur;
    int64_t moved = 0;
    for (int64_t i = 0; i < qn[cur]; ++i) {
      int32_t v = q[cur][i];
      inq[cur][v] = 0;
      if (visit(g, v, part, Wb, lmax, 1, conn, touched)) {
        ++moved;
        for (int64_t e = g->rp[v]; e < g->rp[v + 1]; ++e) {
          int32_t u = g->col[e];
          if (!inq[nx][u]) {
            inq[nx][u] = 1;
            q[nx][qn[nx]++] = u;
          }
        }
      }
    }
    qn[cur] = 0;
    cur = nx;
    if (moved == 0) break;
  }
  free(Wb);
  free(conn);
  free(touched);
  for (int i = 0; i < 2; ++i) {
    free(q[i]);
    free(inq[i]);
  }
  return r > max_rounds ? max_rounds : r;
}

/* Same multilevel driver as the oracle's, with the sequential steps. */
int seq_partition(const orc_graph* in, int32_t k, int64_t eps_num, int64_t eps_den, int32_t f,
                  int32_t lp_rounds, int32_t ref_rounds, int64_t threshold, int32_t* part_out,
                  orc_stats* st) {
  memset(st, 0, sizeof(*st));
  int64_t n = in->n, C = 0, maxc = 0;
  for (int64_t v = 0; v < n; ++v) {
    C += nwt(in, v);
    if (nwt(in, v) > maxc) maxc = nwt(in, v);
  }
  int64_t lmax, W, U;
  int rc = orc_bounds(C, maxc, k, eps_num, eps_den, f, &lmax, &W, &U);
  if (rc) return rc;
  if (threshold <= 0) {
    int64_t a = 60 * (int64_t)k, b = n / (60 * (int64_t)k);
    threshold = a > b ? a : b;
  }
  st->lmax = lmax;
  st->W = W;
  st->U = U;
  st->threshold = threshold;
  uint8_t* iso = (uint8_t*)calloc((size_t)(n > 0 ? n : 1), 1);
  int32_t* newid = (int32_t*)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
  int64_t n0 = 0;
  for (int64_t v = 0; v < n; ++v) {
    iso[v] = in->rp[v + 1] == in->rp[v];
    newid[v] = iso[v] ? -1 : (int32_t)(n0++);
  }
  st->n_isolated = n - n0;
  orc_owned lv[ORC_MAXLEV];
  int32_t* cof[ORC_MAXLEV];
  memset(lv, 0, sizeof(lv));
  memset(cof, 0, sizeof(cof));
  lv[0].n = n0;
  lv[0].m = in->m;
  lv[0].rp = (int64_t*)calloc((size_t)n0 + 1, sizeof(int64_t));
  lv[0].col = (int32_t*)malloc(sizeof(int32_t) * (size_t)(in->m > 0 ? in->m : 1));
  lv[0].ew = (int32_t*)malloc(sizeof(int32_t) * (size_t)(in->m > 0 ? in->m : 1));
  lv[0].nw = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n0 > 0 ? n0 : 1));
  for (int64_t v = 0, i = 0, e0 = 0; v < n; ++v) {
    if (iso[v]) continue;
    for (int64_t e = in->rp[v]; e < in->rp[v + 1]; ++e) {
      lv[0].col[e0] = newid[in->col[e]];
      lv[0].ew[e0] = in->ew ? in->ew[e] : 1;
      ++e0;
    }
    lv[0].nw[i] = nwt(in, v);
    lv[0].rp[i + 1] = e0;
    ++i;
  }
  int L = 0;
  while (lv[L].n > threshold && L + 1 < ORC_MAXLEV) {
    orc_graph g = {lv[L].n, lv[L].m, lv[L].rp, lv[L].col, lv[L].ew, lv[L].nw};
    int32_t* lab = (int32_t*)malloc(sizeof(int32_t) * (size_t)g.n);
    st->rounds_c[L] = seq_cluster(&g, U, lp_rounds, lab);
    cof[L] = (int32_t*)malloc(sizeof(int32_t) * (size_t)g.n);
    rc = orc_contract(&g, lab, 0, cof[L], &lv[L + 1]);
    free(lab);
    if (rc) goto done;
    ++L;
    if (20 * (lv[L - 1].n - lv[L].n) < lv[L - 1].n) break;
  }
  st->levels = L + 1;
  for (int i = 0; i <= L; ++i) {
    st->n_level[i] = lv[i].n;
    st->m_level[i] = lv[i].m;
  }
  {
    int32_t* part = (int32_t*)malloc(sizeof(int32_t) * (size_t)(lv[L].n > 0 ? lv[L].n : 1));
    orc_graph gq = {lv[L].n, lv[L].m, lv[L].rp, lv[L].col, lv[L].ew, lv[L].nw};
    orc_initial_partition(&gq, k, 0, part);
    st->ip_cut = orc_cut(&gq, part, k, NULL);
    for (int i = L; i >= 0; --i) {
      orc_graph g = {lv[i].n, lv[i].m, lv[i].rp, lv[i].col, lv[i].ew, lv[i].nw};
      if (i < L) {
        int32_t* fine = (int32_t*)malloc(sizeof(int32_t) * (size_t)(g.n > 0 ? g.n : 1));
        for (int64_t v = 0; v < g.n; ++v) fine[v] = part[cof[i][v]];
        free(part);
        part = fine;
      }
      if (ref_rounds > 0) st->rounds_r[i] = seq_refine(&g, k, lmax, ref_rounds, part);
    }
    int64_t* B = (int64_t*)calloc((size_t)k, sizeof(int64_t));
    for (int64_t v = 0; v < n; ++v) {
      if (iso[v]) continue;
      part_out[v] = part[newid[v]];
      B[part_out[v]] += nwt(in, v);
    }
    free(part);
    orc_place_isolated(in->nw, n, iso, k, B, part_out);
    free(B);
    int64_t* bw = (int64_t*)calloc((size_t)k, sizeof(int64_t));
    st->cut = orc_cut(in, part_out, k, bw);
    for (int32_t b = 0; b < k; ++b)
      if (bw[b] > st->max_block) st->max_block = bw[b];
    free(bw);
  }
done:
  for (int i = 0; i < ORC_MAXLEV; ++i) {
    orc_owned_free(&lv[i]);
    free(cof[i]);
  }
  free(iso);
  free(newid);
  return rc;
}
