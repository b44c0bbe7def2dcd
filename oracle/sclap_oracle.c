/*
 * sclap_oracle.c -- plain, slow, single-threaded CPU oracle of synchronous
 * size-constrained label propagation (SCLaP), cluster contraction and the
 * multilevel partitioner built on them.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the package smoke check and
 * the benchmark's CPU-baseline leg may load this library.  It shares no code,
 * header or helper with the device library; the two only read the same
 * generated input graphs.
 *
 * Paper: Meyerhenke, Sanders, Schulz, "Partitioning Complex Networks via
 * Size-constrained Clustering" (2014).  Citations below name its sections.
 *
 * The paper's label propagation is sequential (nodes visited one at a time,
 * random ties).  This oracle computes the synchronous, deterministic reading
 * of it that the device path implements:
 *   - every node rates clusters from the previous round's labels and weights;
 *   - ties go to the smallest label, the own label included in the tie set;
 *   - odd rounds only allow moves to smaller labels, even rounds only to
 *     larger ones (without this rule two adjacent singletons swap forever);
 *   - moves into a cluster are admitted in increasing node id while the
 *     cluster's previous weight plus the inclusive prefix of admitted weight
 *     stays within the cap.
 * Every reading of a point the paper leaves open is listed with its reason
 * in the design notes of the repository.
 *
 * All arithmetic is integer.  Node weights are int64, edge weights int32
 * (NULL means unit), ratings accumulate in int64.
 */
#include <stdlib.h>
#include <string.h>

#include "sclap_oracle.h"

static inline int64_t node_w(const orc_graph* g, int64_t v) { return g->nw ? g->nw[v] : 1; }
static inline int64_t edge_w(const orc_graph* g, int64_t e) { return g->ew ? (int64_t)g->ew[e] : 1; }

/* ------------------------------------------------------------------------ */
/* Bounds (Section 2.1 balance constraint; Section 3.1 cluster bound U).     */
/* ------------------------------------------------------------------------ */

/*
 * L_max = (1 + eps) * ceil(c(V) / k) with eps = eps_num / eps_den, and the
 * cluster bound W = L_max / f, both floored: for integer weights w <= x iff
 * w <= floor(x), and floor(floor(x) / f) == floor(x / f), so the floors are
 * exact.  U = max(max_v c(v), W).
 */
int orc_bounds(int64_t total_w, int64_t max_w, int32_t k, int64_t eps_num, int64_t eps_den,
               int32_t f, int64_t* lmax, int64_t* W, int64_t* U) {
  if (k < 1 || eps_num < 0 || eps_den < 1 || f < 1 || total_w < 0) return ORC_EINVAL;
  int64_t per = (total_w + k - 1) / k;
  __int128 num = (__int128)(eps_den + eps_num) * per;
  *lmax = (int64_t)(num / eps_den);
  *W = (int64_t)(num / ((__int128)eps_den * f));
  *U = max_w > *W ? max_w : *W;
  return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* One rating step (Section 3.1: move to the eligible block with the         */
/* strongest connection; local-search variant for overloaded blocks).       */
/* ------------------------------------------------------------------------ */

/*
 * For every node v, from labels `lab` and label weights `Wt` of the previous
 * round:
 *   conn(v, t) = sum of w(v, u) over neighbours u with lab(u) == t;
 *   candidates = {lab(v)} and the labels of v's neighbours;
 *   a foreign label t is kept only if Wt(t) + c(v) <= cap (eligible) and,
 *   with the direction rule, t < lab(v) in odd rounds, t > lab(v) in even;
 *   in refinement mode the own label is dropped when Wt(lab(v)) > cap;
 *   desire(v) = candidate with largest conn, ties to the smallest label;
 *   no candidate left -> desire(v) = lab(v).
 */
void orc_rate(const orc_graph* g, const int32_t* lab, const int64_t* Wt, int64_t nlabels,
              int64_t cap, int32_t round, int32_t dir_rule, int32_t refine, int32_t* desire) {
  int64_t* conn = (int64_t*)calloc((size_t)(nlabels > 0 ? nlabels : 1), sizeof(int64_t));
  int32_t* touched = (int32_t*)malloc(sizeof(int32_t) * (size_t)(g->n > 0 ? g->n : 1));
  for (int64_t v = 0; v < g->n; ++v) {
    const int32_t own = lab[v];
    int64_t nt = 0;
    for (int64_t e = g->rp[v]; e < g->rp[v + 1]; ++e) {
      int32_t t = lab[g->col[e]];
      if (conn[t] == 0) touched[nt++] = t;   /* edge weights are >= 1 */
      conn[t] += edge_w(g, e);
    }
    int32_t best_t = -1;
    int64_t best_c = -1;
    int own_allowed = !(refine && Wt[own] > cap);
    if (own_allowed) {
      best_t = own;
      best_c = conn[own];
    }
    for (int64_t i = 0; i < nt; ++i) {
      int32_t t = touched[i];
      if (t == own) continue;
      if (dir_rule) {
        if ((round & 1) && t > own) continue;
        if (!(round & 1) && t < own) continue;
      }
      if (Wt[t] + node_w(g, v) > cap) continue;
      int64_t c = conn[t];
      if (c > best_c || (c == best_c && t < best_t)) {
        best_c = c;
        best_t = t;
      }
    }
    desire[v] = best_t < 0 ? own : best_t;
    for (int64_t i = 0; i < nt; ++i) conn[touched[i]] = 0;
  }
  free(conn);
  free(touched);
}

/*
 * Admission and apply.  A mover is v with desire(v) != lab(v).  For each
 * target t the movers into t are taken in increasing node id; v is admitted
 * iff Wt(t) + (sum of c over movers into t with id <= v) <= cap, where Wt is
 * the weight before the round (departures are not subtracted).  This keeps
 * every cluster within the cap (Section 3.1: a move never overloads the
 * target).  Admitted movers take their target label; Wt is then recomputed
 * from scratch.  Returns the number of admitted movers.
 */
int64_t orc_admit_apply(const orc_graph* g, const int32_t* desire, int32_t* lab, int64_t* Wt,
                        int64_t nlabels, int64_t cap, uint8_t* admitted_out) {
  int64_t* acc = (int64_t*)calloc((size_t)(nlabels > 0 ? nlabels : 1), sizeof(int64_t));
  uint8_t* adm = (uint8_t*)calloc((size_t)(g->n > 0 ? g->n : 1), 1);
  for (int64_t v = 0; v < g->n; ++v) {
    int32_t t = desire[v];
    if (t == lab[v]) continue;
    acc[t] += node_w(g, v);
    adm[v] = (Wt[t] + acc[t] <= cap);
  }
  int64_t moved = 0;
  for (int64_t v = 0; v < g->n; ++v) {
    if (adm[v]) {
      lab[v] = desire[v];
      ++moved;
    }
  }
  for (int64_t t = 0; t < nlabels; ++t) Wt[t] = 0;
  for (int64_t v = 0; v < g->n; ++v) Wt[lab[v]] += node_w(g, v);
  if (admitted_out) memcpy(admitted_out, adm, (size_t)g->n);
  free(acc);
  free(adm);
  return moved;
}

/* ------------------------------------------------------------------------ */
/* Size-constrained clustering (Section 3.1).                                */
/* ------------------------------------------------------------------------ */

/*
 * Labels start as node ids (each node its own cluster), cluster weights as
 * node weights.  Up to max_rounds rounds of rate + admit.  stop_rule 0: run
 * exactly max_rounds rounds.  stop_rule 1: after round r >= 2 stop when
 * fewer than 5% of the nodes moved over the last two rounds (one downward
 * and one upward round under the direction rule), i.e.
 * 20 * (moved_r + moved_{r-1}) < n.  Edge visits of a round are the sum of
 * the degrees of all rated nodes, here every node.  Returns the rounds run.
 */
int32_t orc_cluster(const orc_graph* g, int64_t U, int32_t max_rounds, int32_t stop_rule,
                    int32_t dir_rule, int32_t* lab, int64_t* moved_out, int64_t* visits_out) {
  int64_t n = g->n;
  int64_t* Wt = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
  int32_t* desire = (int32_t*)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
  for (int64_t v = 0; v < n; ++v) {
    lab[v] = (int32_t)v;
    Wt[v] = node_w(g, v);
  }
  int64_t visits = 0, prev = 0;
  int32_t r;
  for (r = 1; r <= max_rounds; ++r) {
    orc_rate(g, lab, Wt, n, U, r, dir_rule, 0, desire);
    int64_t moved = orc_admit_apply(g, desire, lab, Wt, n, U, NULL);
    visits += g->m;
    if (moved_out) moved_out[r - 1] = moved;
    if (stop_rule == 1 && r >= 2 && 20 * (moved + prev) < n) break;
    prev = moved;
  }
  if (r > max_rounds) r = max_rounds;
  if (visits_out) *visits_out = visits;
  free(Wt);
  free(desire);
  return r;
}

/* ------------------------------------------------------------------------ */
/* Cluster contraction (Section 3.1, Figure 2).                              */
/* ------------------------------------------------------------------------ */

typedef struct { int32_t x, y; int64_t w; } orc_ent;

static int cmp_ent(const void* a, const void* b) {
  const orc_ent* p = (const orc_ent*)a;
  const orc_ent* q = (const orc_ent*)b;
  if (p->x != q->x) return p->x < q->x ? -1 : 1;
  return (p->y > q->y) - (p->y < q->y);
}

/*
 * Each cluster becomes one node; coarse ids rank the labels in use by
 * value.  The coarse node weight is the sum of its members' weights.  Two
 * coarse nodes are adjacent iff their clusters are joined by an edge; the
 * coarse edge weight is the sum of those edges' weights, intra-cluster edges
 * vanish.  Rows are in coarse id order with neighbours ascending, both
 * directions stored.  With drop_isolated, nodes of degree 0 belong to no
 * coarse node (coarse_of = -1).  Returns ORC_EOVERFLOW if a coarse edge
 * weight exceeds int32.
 */
int orc_contract(const orc_graph* g, const int32_t* lab, int32_t drop_isolated,
                 int32_t* coarse_of, orc_owned* out) {
  int64_t n = g->n;
  int32_t* cid = (int32_t*)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
  uint8_t* used = (uint8_t*)calloc((size_t)(n > 0 ? n : 1), 1);
  for (int64_t v = 0; v < n; ++v) {
    if (drop_isolated && g->rp[v + 1] == g->rp[v]) continue;
    used[lab[v]] = 1;
  }
  int64_t nc = 0;
  for (int64_t t = 0; t < n; ++t) cid[t] = used[t] ? (int32_t)(nc++) : -1;
  int64_t* nw = (int64_t*)calloc((size_t)(nc > 0 ? nc : 1), sizeof(int64_t));
  for (int64_t v = 0; v < n; ++v) {
    if (drop_isolated && g->rp[v + 1] == g->rp[v]) { coarse_of[v] = -1; continue; }
    coarse_of[v] = cid[lab[v]];
    nw[coarse_of[v]] += node_w(g, v);
  }
  int64_t ne = 0;
  for (int64_t u = 0; u < n; ++u)
    for (int64_t e = g->rp[u]; e < g->rp[u + 1]; ++e)
      if (coarse_of[u] != coarse_of[g->col[e]]) ++ne;
  orc_ent* ent = (orc_ent*)malloc(sizeof(orc_ent) * (size_t)(ne > 0 ? ne : 1));
  int64_t i = 0;
  for (int64_t u = 0; u < n; ++u)
    for (int64_t e = g->rp[u]; e < g->rp[u + 1]; ++e) {
      int32_t x = coarse_of[u], y = coarse_of[g->col[e]];
      if (x != y) {
        ent[i].x = x;
        ent[i].y = y;
        ent[i].w = edge_w(g, e);
        ++i;
      }
    }
  qsort(ent, (size_t)ne, sizeof(orc_ent), cmp_ent);
  int64_t mc = 0;
  for (int64_t j = 0; j < ne; ++j) {
    if (mc > 0 && ent[mc - 1].x == ent[j].x && ent[mc - 1].y == ent[j].y) ent[mc - 1].w += ent[j].w;
    else ent[mc++] = ent[j];
  }
  int64_t* rp = (int64_t*)calloc((size_t)nc + 1, sizeof(int64_t));
  int32_t* col = (int32_t*)malloc(sizeof(int32_t) * (size_t)(mc > 0 ? mc : 1));
  int32_t* ew = (int32_t*)malloc(sizeof(int32_t) * (size_t)(mc > 0 ? mc : 1));
  int rc = ORC_OK;
  for (int64_t j = 0; j < mc; ++j) {
    rp[ent[j].x + 1]++;
    col[j] = ent[j].y;
    if (ent[j].w > INT32_MAX) rc = ORC_EOVERFLOW;
    ew[j] = (int32_t)ent[j].w;
  }
  for (int64_t x = 0; x < nc; ++x) rp[x + 1] += rp[x];
  free(ent);
  free(cid);
  free(used);
  out->n = nc;
  out->m = mc;
  out->rp = rp;
  out->col = col;
  out->ew = ew;
  out->nw = nw;
  return rc;
}

void orc_owned_free(orc_owned* o) {
  free(o->rp);
  free(o->col);
  free(o->ew);
  free(o->nw);
  memset(o, 0, sizeof(*o));
}

/* ------------------------------------------------------------------------ */
/* Initial partition of the coarsest graph: BFS order cut into k chunks.     */
/* (Replaces the paper's KaHIP recursive bisection, Section 3.1.)            */
/* ------------------------------------------------------------------------ */

static int cmp_i32(const void* a, const void* b) {
  int32_t x = *(const int32_t*)a, y = *(const int32_t*)b;
  return (x > y) - (x < y);
}

/*
 * Breadth-first order: a new search starts from the smallest unvisited id;
 * a node's unvisited neighbours are appended in ascending id.  With P(v) the
 * total weight of the nodes before v in that order and C the total weight,
 * block(v) = min(k - 1, floor(k P(v) / C)).  With skip_isolated, nodes of
 * degree 0 are left out (block -1) and excluded from C.
 */
void orc_initial_partition(const orc_graph* g, int32_t k, int32_t skip_isolated, int32_t* part) {
  int64_t n = g->n;
  int32_t* order = (int32_t*)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
  uint8_t* seen = (uint8_t*)calloc((size_t)(n > 0 ? n : 1), 1);
  int64_t maxdeg = 0;
  for (int64_t v = 0; v < n; ++v)
    if (g->rp[v + 1] - g->rp[v] > maxdeg) maxdeg = g->rp[v + 1] - g->rp[v];
  int32_t* buf = (int32_t*)malloc(sizeof(int32_t) * (size_t)(maxdeg > 0 ? maxdeg : 1));
  int64_t head = 0, tail = 0;
  for (int64_t s = 0; s < n; ++s) {
    if (seen[s]) continue;
    if (skip_isolated && g->rp[s + 1] == g->rp[s]) { part[s] = -1; continue; }
    seen[s] = 1;
    order[tail++] = (int32_t)s;
    while (head < tail) {
      int32_t f = order[head++];
      int64_t d = g->rp[f + 1] - g->rp[f];
      memcpy(buf, g->col + g->rp[f], sizeof(int32_t) * (size_t)d);
      qsort(buf, (size_t)d, sizeof(int32_t), cmp_i32);
      for (int64_t i = 0; i < d; ++i)
        if (!seen[buf[i]]) {
          seen[buf[i]] = 1;
          order[tail++] = buf[i];
        }
    }
  }
  int64_t C = 0;
  for (int64_t i = 0; i < tail; ++i) C += node_w(g, order[i]);
  int64_t P = 0;
  for (int64_t i = 0; i < tail; ++i) {
    int32_t v = order[i];
    int64_t b = C > 0 ? (int64_t)(((__int128)k * P) / C) : 0;
    part[v] = (int32_t)(b < k - 1 ? b : k - 1);
    P += node_w(g, v);
  }
  free(order);
  free(seen);
  free(buf);
}

/* ------------------------------------------------------------------------ */
/* Cut and block weights (Section 2.1).                                      */
/* ------------------------------------------------------------------------ */

/* cut = sum over edges {u, v} with block(u) != block(v) of w(u, v); nodes
 * with block -1 are ignored in the block weights. */
int64_t orc_cut(const orc_graph* g, const int32_t* part, int32_t k, int64_t* block_w) {
  int64_t twice = 0;
  for (int64_t u = 0; u < g->n; ++u)
    for (int64_t e = g->rp[u]; e < g->rp[u + 1]; ++e)
      if (part[u] != part[g->col[e]]) twice += edge_w(g, e);
  if (block_w) {
    for (int32_t b = 0; b < k; ++b) block_w[b] = 0;
    for (int64_t v = 0; v < g->n; ++v)
      if (part[v] >= 0) block_w[part[v]] += node_w(g, v);
  }
  return twice / 2;
}

/* ------------------------------------------------------------------------ */
/* Label propagation as local search (Section 3.1, last paragraph; active    */
/* nodes, Section 4).                                                        */
/* ------------------------------------------------------------------------ */

/*
 * Rounds of rate + admit with labels = block ids, cap = L_max and the own
 * block dropped from the candidates while it is overloaded.  Stops after
 * max_rounds rounds or after two consecutive rounds without a move (under
 * the direction rule one round without moves is not yet a fixed point).
 *
 * Only boundary nodes can move (an interior node's only candidate is its own
 * block), so the rated set of round r + 1 is the boundary nodes found in
 * round r plus the neighbours of the nodes that moved in round r; round 1
 * rates every node.  The oracle rates every node each round and checks
 * that no node outside that set wants to move; the set only defines the
 * edge visits counted (sum of degrees of the rated nodes).  Nodes with
 * block -1 take no part.  Returns the rounds run, or -1 if the check fails.
 */
int32_t orc_refine(const orc_graph* g, int32_t k, int64_t lmax, int32_t max_rounds, int32_t dir_rule,
                   int32_t* part, int64_t* moved_out, int64_t* visits_out) {
  int64_t n = g->n;
  int64_t* Wb = (int64_t*)calloc((size_t)(k > 0 ? k : 1), sizeof(int64_t));
  int32_t* desire = (int32_t*)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
  uint8_t* rated = (uint8_t*)malloc((size_t)(n > 0 ? n : 1));
  uint8_t* nxt = (uint8_t*)malloc((size_t)(n > 0 ? n : 1));
  uint8_t* adm = (uint8_t*)malloc((size_t)(n > 0 ? n : 1));
  int32_t* lab = (int32_t*)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
  orc_graph sub = *g;
  for (int64_t v = 0; v < n; ++v) {
    rated[v] = part[v] >= 0;
    if (part[v] >= 0) Wb[part[v]] += node_w(g, v);
  }
  /* Nodes with block -1 have degree 0 and never move; give them a harmless
   * label so the generic steps can run over all nodes. */
  int64_t visits = 0;
  int32_t zero_streak = 0, r, ok = 1;
  for (r = 1; r <= max_rounds; ++r) {
    for (int64_t v = 0; v < n; ++v) {
      lab[v] = part[v] >= 0 ? part[v] : 0;
      if (rated[v]) visits += g->rp[v + 1] - g->rp[v];
    }
    /* block weights must not count the -1 nodes: rate against Wb */
    orc_rate(&sub, lab, Wb, k, lmax, r, dir_rule, 1, desire);
    for (int64_t v = 0; v < n; ++v) {
      if (part[v] < 0) desire[v] = lab[v];
      if (!rated[v] && desire[v] != lab[v]) ok = 0;
    }
    /* admission against Wb over participating nodes only */
    int64_t* acc = (int64_t*)calloc((size_t)(k > 0 ? k : 1), sizeof(int64_t));
    for (int64_t v = 0; v < n; ++v) {
      adm[v] = 0;
      int32_t t = desire[v];
      if (part[v] < 0 || t == lab[v]) continue;
      acc[t] += node_w(g, v);
      adm[v] = (Wb[t] + acc[t] <= lmax);
    }
    free(acc);
    int64_t moved = 0;
    memset(nxt, 0, (size_t)n);
    for (int64_t v = 0; v < n; ++v) {
      if (!rated[v]) continue;
      for (int64_t e = g->rp[v]; e < g->rp[v + 1]; ++e)
        if (part[g->col[e]] != part[v]) { nxt[v] = 1; break; }
    }
    for (int64_t v = 0; v < n; ++v) {
      if (!adm[v]) continue;
      part[v] = desire[v];
      ++moved;
      for (int64_t e = g->rp[v]; e < g->rp[v + 1]; ++e) nxt[g->col[e]] = 1;
    }
    for (int32_t b = 0; b < k; ++b) Wb[b] = 0;
    for (int64_t v = 0; v < n; ++v)
      if (part[v] >= 0) Wb[part[v]] += node_w(g, v);
    memcpy(rated, nxt, (size_t)n);
    if (moved_out) moved_out[r - 1] = moved;
    zero_streak = moved == 0 ? zero_streak + 1 : 0;
    if (zero_streak >= 2) break;
  }
  if (r > max_rounds) r = max_rounds;
  if (visits_out) *visits_out = visits;
  free(Wb);
  free(desire);
  free(rated);
  free(nxt);
  free(adm);
  free(lab);
  return ok ? r : -1;
}

/* ------------------------------------------------------------------------ */
/* Isolated nodes: placed after refinement by filling the blocks up to a     */
/* common level, in increasing node id (the paper does not treat them).      */
/* ------------------------------------------------------------------------ */

/*
 * B(b) = block weights without the isolated nodes, C_I their total weight.
 * lambda = smallest integer >= min_b B(b) with D(lambda) =
 * sum_b max(0, lambda - B(b)) >= C_I; block b receives the interval
 * [D_b, D_b + d_b) of the isolated weight, d_b = max(0, lambda - B(b)),
 * D_b = sum of d over blocks before b.  Isolated node i, with P_i the weight
 * of the isolated nodes before it, goes to the first block whose interval
 * end exceeds P_i; if none does (only zero-weight nodes at the end), to the
 * last block with d_b > 0, else block 0.
 */
void orc_place_isolated(const int64_t* nw, int64_t n, const uint8_t* isolated, int32_t k,
                        const int64_t* B, int32_t* part) {
  int64_t CI = 0, lo = INT64_MAX, hi = INT64_MIN;
  for (int64_t v = 0; v < n; ++v)
    if (isolated[v]) CI += nw ? nw[v] : 1;
  for (int32_t b = 0; b < k; ++b) {
    if (B[b] < lo) lo = B[b];
    if (B[b] > hi) hi = B[b];
  }
  /* D(lo) = 0 and D(hi + CI) >= CI: binary search the smallest lambda */
  int64_t a = lo, z = hi + CI;
  while (a < z) {
    int64_t mid = a + (z - a) / 2;
    int64_t D = 0;
    for (int32_t b = 0; b < k; ++b)
      if (mid > B[b]) D += mid - B[b];
    if (D >= CI) z = mid;
    else a = mid + 1;
  }
  int64_t lambda = a;
  int64_t* end = (int64_t*)malloc(sizeof(int64_t) * (size_t)k);
  int64_t D = 0;
  int32_t last_pos = 0;
  for (int32_t b = 0; b < k; ++b) {
    int64_t d = lambda > B[b] ? lambda - B[b] : 0;
    D += d;
    end[b] = D;
    if (d > 0) last_pos = b;
  }
  int64_t P = 0;
  for (int64_t v = 0; v < n; ++v) {
    if (!isolated[v]) continue;
    int32_t blk = -1;
    for (int32_t b = 0; b < k; ++b)
      if (end[b] > P) { blk = b; break; }
    part[v] = blk >= 0 ? blk : last_pos;
    P += nw ? nw[v] : 1;
  }
  free(end);
}

/* ------------------------------------------------------------------------ */
/* Multilevel partitioner (Section 1 multilevel scheme; Section 3.1).        */
/* ------------------------------------------------------------------------ */

/*
 * 1. Bounds from the whole input: L_max, W, U.
 * 2. Isolated nodes are removed; the rest, renumbered in id order, is level 0.
 * 3. While the current level has more than `threshold` nodes: cluster it
 *    (stop rule 1) and contract; the new level is kept; stop after it if it
 *    shrank by less than 5% (20 (n - n') < n).  threshold <= 0 selects the
 *    paper's rule max(60 k, n / (60 k)) on the input n.
 * 4. Initial partition of the coarsest level (BFS chunks).
 * 5. From the coarsest level to level 0: project (a fine node takes its
 *    coarse node's block), then refine.
 * 6. Isolated nodes are placed; the cut is recomputed on the input.
 */
int orc_partition(const orc_graph* in, int32_t k, int64_t eps_num, int64_t eps_den, int32_t f,
                  int32_t lp_rounds, int32_t ref_rounds, int64_t threshold, int32_t dir_rule,
                  int32_t* part_out, orc_stats* st) {
  if (k < 1 || lp_rounds < 1 || lp_rounds > ORC_MAXR || ref_rounds < 0 || ref_rounds > ORC_MAXR)
    return ORC_EINVAL;
  memset(st, 0, sizeof(*st));
  int64_t n = in->n;
  int64_t C = 0, maxc = 0;
  for (int64_t v = 0; v < n; ++v) {
    C += node_w(in, v);
    if (node_w(in, v) > maxc) maxc = node_w(in, v);
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

  /* level 0: induced subgraph on the nodes of degree > 0 */
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
    lv[0].nw[i] = node_w(in, v);
    lv[0].rp[i + 1] = e0;
    ++i;
  }

  int L = 0;   /* index of the coarsest level */
  while (lv[L].n > threshold && L + 1 < ORC_MAXLEV) {
    orc_graph g = {lv[L].n, lv[L].m, lv[L].rp, lv[L].col, lv[L].ew, lv[L].nw};
    int32_t* lab = (int32_t*)malloc(sizeof(int32_t) * (size_t)g.n);
    st->rounds_c[L] = orc_cluster(&g, U, lp_rounds, 1, dir_rule, lab, st->moved_c[L], &st->visits_c[L]);
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
      if (ref_rounds > 0) {
        int32_t rr = orc_refine(&g, k, lmax, ref_rounds, dir_rule, part, st->moved_r[i], &st->visits_r[i]);
        if (rr < 0) { rc = ORC_EINVAL; free(part); goto done; }
        st->rounds_r[i] = rr;
      }
    }
    /* back to input ids, then place the isolated nodes */
    int64_t* B = (int64_t*)calloc((size_t)k, sizeof(int64_t));
    for (int64_t v = 0; v < n; ++v) {
      if (iso[v]) continue;
      part_out[v] = part[newid[v]];
      B[part_out[v]] += node_w(in, v);
    }
    free(part);
    orc_place_isolated(in->nw, n, iso, k, B, part_out);
    free(B);
    int64_t* bw = (int64_t*)calloc((size_t)k, sizeof(int64_t));
    st->cut = orc_cut(in, part_out, k, bw);
    st->max_block = 0;
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
