/*
 * sclap_extensions.c -- CPU oracle of the algorithmic extensions of
 * Section 4 of the paper, built on the plain oracle (sclap_oracle.c):
 *   - clustering that respects an input partition, and iterated V-cycles
 *     (Section 4, "Iterated Multilevel Algorithms"; Appendix B.1);
 *   - extra imbalance on the coarse levels of the first cycle (Section 4,
 *     "Allowing Larger Imbalances on Coarse Levels");
 *   - degree-ordered sub-rounds, a synchronous reading of the increasing
 *     degree order of the label propagation (Section 4, "Node Ordering for
 *     Label Propagation");
 *   - ensemble clusterings combined by their overlay (Section 4, "Ensemble
 *     Clusterings").
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the package smoke check and
 * the benchmark's CPU-baseline leg may load this library.  It shares no code,
 * header or helper with the device library.
 *
 * The synchronous round semantics are those of the plain oracle (ratings from
 * the previous round, ties to the smallest label, the direction rule,
 * admission in increasing node id against the previous weights).  The
 * readings taken where the paper leaves a point open are stated at each
 * function and listed in the design notes.
 */
#include <stdlib.h>
#include <string.h>

#include "sclap_oracle.h"

static inline int64_t xnode_w(const orc_graph* g, int64_t v) { return g->nw ? g->nw[v] : 1; }
static inline int64_t xedge_w(const orc_graph* g, int64_t e) { return g->ew ? (int64_t)g->ew[e] : 1; }

/* ------------------------------------------------------------------------ */
/* Rating with the extensions' filters.                                      */
/* ------------------------------------------------------------------------ */

/*
 * The clustering rating of the plain oracle (conn(v, t) summed over the
 * neighbours with label t; foreign candidates eligible when Wt(t) + c(v) <=
 * cap and allowed by the direction rule; the largest conn wins, ties to the
 * smallest label, the own label in the tie set), with two additions:
 *
 *   vblk, lblk (Appendix B.1): when vblk is given, v may only move to a
 *     cluster that lies inside its own block vblk(v) of the input partition;
 *     lblk(t) is the block of the nodes of cluster t (a cluster only ever
 *     holds nodes of one block, which is checked: the own cluster must lie in
 *     v's block).  The edge visits of v are then its neighbours in its own
 *     block: the others can never carry a candidate.
 *   active: when given, only nodes with active(v) != 0 are rated; the others
 *     keep their label (desire = own) and visit nothing.
 *
 * Returns the edge visits, or -1 if a cluster was found outside its block.
 */
int64_t orc_rate_ext(const orc_graph* g, const int32_t* lab, const int64_t* Wt, int64_t nlabels, int64_t cap,
                     int32_t round, int32_t dir_rule, const int32_t* vblk, const int32_t* lblk,
                     const uint8_t* active, int32_t* desire) {
  int64_t* conn = (int64_t*)calloc((size_t)(nlabels > 0 ? nlabels : 1), sizeof(int64_t));
  int32_t* touched = (int32_t*)malloc(sizeof(int32_t) * (size_t)(g->n > 0 ? g->n : 1));
  int64_t visits = 0;
  int bad = 0;
  for (int64_t v = 0; v < g->n; ++v) {
    const int32_t own = lab[v];
    desire[v] = own;
    if (active && !active[v]) continue;
    if (vblk && lblk[own] != vblk[v]) bad = 1;
    int64_t nt = 0;
    for (int64_t e = g->rp[v]; e < g->rp[v + 1]; ++e) {
      const int32_t u = g->col[e];
      if (!vblk || vblk[u] == vblk[v]) ++visits;
      const int32_t t = lab[u];
      if (conn[t] == 0) touched[nt++] = t;
      conn[t] += xedge_w(g, e);
    }
    int32_t best_t = own;
    int64_t best_c = conn[own];
    for (int64_t i = 0; i < nt; ++i) {
      const int32_t t = touched[i];
      if (t == own) continue;
      if (vblk && lblk[t] != vblk[v]) continue;        /* cluster t lies in another block */
      if (dir_rule) {
        if ((round & 1) && t > own) continue;
        if (!(round & 1) && t < own) continue;
      }
      if (Wt[t] + xnode_w(g, v) > cap) continue;
      const int64_t c = conn[t];
      if (c > best_c || (c == best_c && t < best_t)) {
        best_c = c;
        best_t = t;
      }
    }
    desire[v] = best_t;
    for (int64_t i = 0; i < nt; ++i) conn[touched[i]] = 0;
  }
  free(conn);
  free(touched);
  return bad ? -1 : visits;
}

/*
 * Degree class of v for S sub-rounds (Section 4 orders the nodes by
 * increasing degree; the synchronous reading splits a round into S
 * sub-rounds by degree class): 0 below degree 4, else floor(log4(degree)),
 * at most S - 1.
 */
static int32_t deg_class(const orc_graph* g, int64_t v, int32_t S) {
  int64_t d = g->rp[v + 1] - g->rp[v];
  int32_t c = 0;
  while (d >= 4 && c < S - 1) {
    d >>= 2;
    ++c;
  }
  return c;
}

/* ------------------------------------------------------------------------ */
/* Clustering with the extensions.                                           */
/* ------------------------------------------------------------------------ */

/*
 * Size-constrained clustering as in the plain oracle, with:
 *   lab0: initial labels (a permutation of [0, n)); NULL: node ids.  Cluster
 *     weights start as Wt(lab0(v)) = c(v).
 *   vblk: the input partition to respect (Appendix B.1); the block of the
 *     cluster that starts as {v} is vblk(v).
 *   subrounds S >= 2: every round is S sub-rounds; sub-round s rates the
 *     nodes of degree class s from the labels and weights after sub-round
 *     s - 1, and admits and applies their moves as a round does.  The
 *     direction rule follows the round number; a round's moves and visits
 *     are the sums over its sub-rounds, and the 5% rule looks at rounds.
 * Returns the rounds run, or -1 if a cluster left its block.
 */
int32_t orc_cluster_ext(const orc_graph* g, int64_t U, int32_t max_rounds, int32_t stop_rule, int32_t dir_rule,
                        const int32_t* vblk, int32_t subrounds, const int32_t* lab0, int32_t* lab,
                        int64_t* moved_out, int64_t* visits_out) {
  const int64_t n = g->n;
  const size_t nz = (size_t)(n > 0 ? n : 1);
  const int32_t S = subrounds > 1 ? subrounds : 1;
  int64_t* Wt = (int64_t*)calloc(nz, sizeof(int64_t));
  int32_t* desire = (int32_t*)malloc(sizeof(int32_t) * nz);
  int32_t* lblk = vblk ? (int32_t*)malloc(sizeof(int32_t) * nz) : NULL;
  uint8_t* active = S > 1 ? (uint8_t*)malloc(nz) : NULL;
  for (int64_t v = 0; v < n; ++v) {
    lab[v] = lab0 ? lab0[v] : (int32_t)v;
    Wt[lab[v]] += xnode_w(g, v);
    if (lblk) lblk[lab[v]] = vblk[v];
  }
  int64_t visits = 0, prev = 0;
  int32_t r, bad = 0;
  for (r = 1; r <= max_rounds; ++r) {
    int64_t moved = 0;
    for (int32_t s = 0; s < S; ++s) {
      if (active)
        for (int64_t v = 0; v < n; ++v) active[v] = deg_class(g, v, S) == s;
      const int64_t vis = orc_rate_ext(g, lab, Wt, n, U, r, dir_rule, vblk, lblk, active, desire);
      if (vis < 0) bad = 1;
      else visits += vis;
      moved += orc_admit_apply(g, desire, lab, Wt, n, U, NULL);
    }
    if (moved_out) moved_out[r - 1] = moved;
    if (stop_rule == 1 && r >= 2 && 20 * (moved + prev) < n) break;
    prev = moved;
  }
  if (r > max_rounds) r = max_rounds;
  if (visits_out) *visits_out = visits;
  free(Wt);
  free(desire);
  free(lblk);
  free(active);
  return bad ? -1 : r;
}

/* ------------------------------------------------------------------------ */
/* Ensemble clusterings and their overlay (Section 4, "Ensemble             */
/* Clusterings").                                                            */
/* ------------------------------------------------------------------------ */

static int64_t gcd64(int64_t a, int64_t b) {
  while (b) {
    const int64_t t = a % b;
    a = b;
    b = t;
  }
  return a;
}

/*
 * Initial labels of ensemble member e (the paper varies its members by
 * random seeds; this reading varies them deterministically): member 0 starts
 * from the node ids, member e >= 1 from the permutation
 *   pi_e(v) = (a_e v + b_e) mod n,
 * with a_e the first value from (2654435761 e) mod n upward (cyclically,
 * skipping 0) that is coprime to n, and b_e = (2246822519 e) mod n.  The
 * label order then differs per member, and with it the ties and the
 * direction rule.
 */
void orc_member_labels(int64_t n, int32_t e, int32_t* lab0) {
  if (e == 0 || n <= 1) {
    for (int64_t v = 0; v < n; ++v) lab0[v] = (int32_t)v;
    return;
  }
  int64_t a = (int64_t)(((unsigned __int128)2654435761u * (uint64_t)e) % (uint64_t)n);
  for (;;) {
    if (a == 0) a = 1;
    if (gcd64(a, n) == 1) break;
    a = (a + 1) % n;
  }
  const int64_t b = (int64_t)(((unsigned __int128)2246822519u * (uint64_t)e) % (uint64_t)n);
  for (int64_t v = 0; v < n; ++v) lab0[v] = (int32_t)(((unsigned __int128)a * (uint64_t)v + (uint64_t)b) % (uint64_t)n);
}

/*
 * Overlay of the current overlay O with clustering C (Section 4): nodes are
 * taken in increasing id; the pair (O[v], C[v]) gets the next number of a
 * counter the first time it is seen, and O[v] becomes that number.  Two
 * nodes share a cluster of the result iff they shared one in O and in C.
 * Returns the number of clusters.  The pairs are kept in an open-addressing
 * hash map.
 */
int64_t orc_overlay(int64_t n, int32_t* O, const int32_t* C) {
  size_t cap = 16;
  while (cap < 2 * (size_t)(n > 0 ? n : 1)) cap <<= 1;
  uint64_t* keys = (uint64_t*)malloc(cap * sizeof(uint64_t));
  int32_t* vals = (int32_t*)malloc(cap * sizeof(int32_t));
  uint8_t* used = (uint8_t*)calloc(cap, 1);
  int32_t c = 0;
  for (int64_t v = 0; v < n; ++v) {
    const uint64_t key = ((uint64_t)(uint32_t)O[v] << 32) | (uint32_t)C[v];
    size_t h = (size_t)((key * 0x9E3779B97F4A7C15ull) >> 20) & (cap - 1);
    while (used[h] && keys[h] != key) h = (h + 1) & (cap - 1);
    if (!used[h]) {
      used[h] = 1;
      keys[h] = key;
      vals[h] = c++;
    }
    O[v] = vals[h];
  }
  free(keys);
  free(vals);
  free(used);
  return c;
}

/*
 * Ensemble clustering of one level: `members` clusterings (orc_cluster_ext
 * with member e's initial labels) overlaid in member order.  With one
 * member this is the plain clustering and its labels.  Statistics: rounds =
 * the largest member's rounds, moved[r] = the sum over members of the moves
 * of round r, visits = the sum over members.  Returns the rounds, or -1.
 */
int32_t orc_ensemble(const orc_graph* g, int64_t U, int32_t max_rounds, int32_t stop_rule, int32_t dir_rule,
                     int32_t members, const int32_t* vblk, int32_t subrounds, int32_t* lab, int64_t* moved_out,
                     int64_t* visits_out) {
  const int64_t n = g->n;
  const size_t nz = (size_t)(n > 0 ? n : 1);
  if (members < 1) members = 1;
  int32_t* lab0 = (int32_t*)malloc(sizeof(int32_t) * nz);
  int32_t* C = (int32_t*)malloc(sizeof(int32_t) * nz);
  int64_t mv[ORC_MAXR];
  int64_t visits = 0;
  int32_t rounds = 0;
  if (moved_out) memset(moved_out, 0, sizeof(int64_t) * (size_t)(max_rounds > 0 ? max_rounds : 1));
  for (int32_t e = 0; e < members; ++e) {
    orc_member_labels(n, e, lab0);
    int64_t vis = 0;
    memset(mv, 0, sizeof(mv));
    const int32_t r = orc_cluster_ext(g, U, max_rounds, stop_rule, dir_rule, vblk, subrounds, lab0,
                                      e == 0 ? lab : C, mv, &vis);
    if (r < 0) {
      rounds = -1;
      break;
    }
    if (r > rounds) rounds = r;
    visits += vis;
    if (moved_out)
      for (int32_t i = 0; i < r; ++i) moved_out[i] += mv[i];
    if (e > 0) orc_overlay(n, lab, C);
  }
  if (visits_out) *visits_out = visits;
  free(lab0);
  free(C);
  return rounds;
}

/* ------------------------------------------------------------------------ */
/* Multilevel partitioner with V-cycles and the extensions.                  */
/* ------------------------------------------------------------------------ */

/*
 * L_max on level i of a hierarchy of q levels (level 0 = the input) with
 * extra imbalance delta (Section 4): (1 + eps + delta / (q - i)) ceil(C / k),
 * floored, for 1 <= i <= q - 1; the plain L_max on level 0.  With levels
 * numbered from 1 at the input as in the paper, delta / (q - i) is the
 * paper's delta / (q - l + 1) for l = i + 1.
 */
int64_t orc_level_lmax(int64_t C, int32_t k, int64_t eps_num, int64_t eps_den, int64_t dnum, int64_t dden,
                          int32_t q, int32_t i, int64_t lmax) {
  if (i == 0 || dnum <= 0) return lmax;
  const __int128 ck = (C + k - 1) / k;
  const __int128 span = q - i;
  const __int128 num = ck * ((__int128)(eps_den + eps_num) * dden * span + (__int128)dnum * eps_den);
  const __int128 den = (__int128)eps_den * dden * span;
  return (int64_t)(num / den);
}

/*
 * Iterated multilevel partitioning (V-cycles, Section 4 and Appendix B.1),
 * with the plain scheme of orc_partition as its first cycle, except that the
 * clustering of every level is orc_ensemble (x->ensemble members, x->subrounds
 * sub-rounds) and that refinement on a coarse level i of the first cycle uses
 * the bound orc_level_lmax (x->delta_num / x->delta_den; none on level 0 and in
 * later cycles).  Cycle c >= 2 starts from the best partition P found so far:
 *   - coarsening clusters every level respecting the blocks of P on it (the
 *     blocks of level 0 are P's; a coarse node takes the block of its
 *     members, which all share one), so no cut edge of P is contracted;
 *   - the coarsest level's partition is P's blocks on it (same cut and block
 *     weights as P), with no initial partitioning;
 *   - uncoarsening projects and refines as in the first cycle.
 * The coarsening stop rules are the first cycle's.  Isolated nodes are set
 * aside and placed after refinement in every cycle.  "Best" (the returned
 * partition and the next cycle's start): the cycles whose largest block is
 * within L_max before the others, then the smaller cut; ties keep the
 * earlier cycle.  st describes the last cycle's hierarchy, with cut and
 * max_block of the returned partition; cy gets every cycle's results.
 */
int orc_partition_ext(const orc_graph* in, int32_t k, int64_t eps_num, int64_t eps_den, int32_t f,
                      int32_t lp_rounds, int32_t ref_rounds, int64_t threshold, int32_t dir_rule,
                      const orc_mlx* x, int32_t* part_out, orc_stats* st, orc_cycles* cy) {
  const int32_t cycles = x && x->vcycles > 1 ? x->vcycles : 1;
  if (k < 1 || lp_rounds < 1 || lp_rounds > ORC_MAXR || ref_rounds < 0 || ref_rounds > ORC_MAXR ||
      cycles > ORC_MAXCYC)
    return ORC_EINVAL;
  if (x && x->delta_num > 0 && x->delta_den <= 0) return ORC_EINVAL;
  const int32_t S = x ? x->subrounds : 0;
  const int32_t E = x && x->ensemble > 1 ? x->ensemble : 1;
  const int64_t dnum = x ? x->delta_num : 0, dden = x ? x->delta_den : 1;
  memset(st, 0, sizeof(*st));
  memset(cy, 0, sizeof(*cy));
  const int64_t n = in->n;
  const size_t nz = (size_t)(n > 0 ? n : 1);
  int64_t C = 0, maxc = 0;
  for (int64_t v = 0; v < n; ++v) {
    C += xnode_w(in, v);
    if (xnode_w(in, v) > maxc) maxc = xnode_w(in, v);
  }
  int64_t lmax, W, U;
  int rc = orc_bounds(C, maxc, k, eps_num, eps_den, f, &lmax, &W, &U);
  if (rc) return rc;
  if (threshold <= 0) {
    const int64_t a = 60 * (int64_t)k, b = n / (60 * (int64_t)k);
    threshold = a > b ? a : b;
  }

  /* level 0: the induced subgraph on the nodes of degree > 0, in id order */
  uint8_t* iso = (uint8_t*)calloc(nz, 1);
  int32_t* newid = (int32_t*)malloc(sizeof(int32_t) * nz);
  int64_t n0 = 0;
  for (int64_t v = 0; v < n; ++v) {
    iso[v] = in->rp[v + 1] == in->rp[v];
    newid[v] = iso[v] ? -1 : (int32_t)(n0++);
  }
  orc_owned lv[ORC_MAXLEV];
  int32_t* cof[ORC_MAXLEV];
  int32_t* blk[ORC_MAXLEV];
  memset(lv, 0, sizeof(lv));
  memset(cof, 0, sizeof(cof));
  memset(blk, 0, sizeof(blk));
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
    lv[0].nw[i] = xnode_w(in, v);
    lv[0].rp[i + 1] = e0;
    ++i;
  }

  int32_t* pc = (int32_t*)malloc(sizeof(int32_t) * nz);  /* this cycle's partition of the input */
  int64_t* bw = (int64_t*)calloc((size_t)k, sizeof(int64_t));
  int64_t best_cut = 0, best_over = 0;
  for (int32_t cyc = 0; cyc < cycles && rc == ORC_OK; ++cyc) {
    orc_stats cs;
    memset(&cs, 0, sizeof(cs));
    if (cyc > 0) {
      blk[0] = (int32_t*)malloc(sizeof(int32_t) * (size_t)(n0 > 0 ? n0 : 1));
      for (int64_t v = 0; v < n; ++v)
        if (!iso[v]) blk[0][newid[v]] = part_out[v];
    }
    int L = 0;
    while (lv[L].n > threshold && L + 1 < ORC_MAXLEV) {
      orc_graph g = {lv[L].n, lv[L].m, lv[L].rp, lv[L].col, lv[L].ew, lv[L].nw};
      int32_t* lab = (int32_t*)malloc(sizeof(int32_t) * (size_t)(g.n > 0 ? g.n : 1));
      cs.rounds_c[L] = orc_ensemble(&g, U, lp_rounds, 1, dir_rule, E, blk[L], S, lab, cs.moved_c[L],
                                    &cs.visits_c[L]);
      if (cs.rounds_c[L] < 0) {
        free(lab);
        rc = ORC_EINVAL;
        break;
      }
      cof[L] = (int32_t*)malloc(sizeof(int32_t) * (size_t)(g.n > 0 ? g.n : 1));
      rc = orc_contract(&g, lab, 0, cof[L], &lv[L + 1]);
      free(lab);
      if (rc) break;
      if (blk[L]) {
        blk[L + 1] = (int32_t*)malloc(sizeof(int32_t) * (size_t)(lv[L + 1].n > 0 ? lv[L + 1].n : 1));
        for (int64_t v = 0; v < g.n; ++v) blk[L + 1][cof[L][v]] = blk[L][v];
      }
      ++L;
      if (20 * (lv[L - 1].n - lv[L].n) < lv[L - 1].n) break;
    }
    if (rc) break;
    cs.levels = L + 1;
    for (int i = 0; i <= L; ++i) {
      cs.n_level[i] = lv[i].n;
      cs.m_level[i] = lv[i].m;
    }
    int32_t* part = (int32_t*)malloc(sizeof(int32_t) * (size_t)(lv[L].n > 0 ? lv[L].n : 1));
    orc_graph gq = {lv[L].n, lv[L].m, lv[L].rp, lv[L].col, lv[L].ew, lv[L].nw};
    if (cyc == 0) orc_initial_partition(&gq, k, 0, part);
    else memcpy(part, blk[L], sizeof(int32_t) * (size_t)lv[L].n);
    cs.ip_cut = orc_cut(&gq, part, k, NULL);
    for (int i = L; i >= 0 && rc == ORC_OK; --i) {
      orc_graph g = {lv[i].n, lv[i].m, lv[i].rp, lv[i].col, lv[i].ew, lv[i].nw};
      if (i < L) {
        int32_t* fine = (int32_t*)malloc(sizeof(int32_t) * (size_t)(g.n > 0 ? g.n : 1));
        for (int64_t v = 0; v < g.n; ++v) fine[v] = part[cof[i][v]];
        free(part);
        part = fine;
      }
      if (ref_rounds > 0) {
        const int64_t li = cyc == 0 ? orc_level_lmax(C, k, eps_num, eps_den, dnum, dden, L + 1, i, lmax) : lmax;
        cy->lmax[cyc][i] = li;
        const int32_t rr = orc_refine(&g, k, li, ref_rounds, dir_rule, part, cs.moved_r[i], &cs.visits_r[i]);
        if (rr < 0) rc = ORC_EINVAL;
        cs.rounds_r[i] = rr;
      }
    }
    if (rc) {
      free(part);
      break;
    }
    /* back to input ids, then place the isolated nodes */
    for (int32_t b = 0; b < k; ++b) bw[b] = 0;
    for (int64_t v = 0; v < n; ++v) {
      if (iso[v]) continue;
      pc[v] = part[newid[v]];
      bw[pc[v]] += xnode_w(in, v);
    }
    free(part);
    orc_place_isolated(in->nw, n, iso, k, bw, pc);
    const int64_t cut = orc_cut(in, pc, k, bw);
    int64_t mb = 0;
    for (int32_t b = 0; b < k; ++b)
      if (bw[b] > mb) mb = bw[b];
    cy->cut[cyc] = cut;
    cy->max_block[cyc] = mb;
    cy->levels[cyc] = cs.levels;
    int64_t vis = 0;
    for (int i = 0; i < cs.levels; ++i) vis += cs.visits_c[i] + cs.visits_r[i];
    cy->visits[cyc] = vis;
    cy->cycles = cyc + 1;
    const int64_t over = mb > lmax;
    if (cyc == 0 || over < best_over || (over == best_over && cut < best_cut)) {
      best_over = over;
      best_cut = cut;
      cy->best = cyc;
      memcpy(part_out, pc, sizeof(int32_t) * (size_t)n);
    }
    *st = cs;
    /* this cycle's hierarchy is not needed by the next one */
    for (int i = 0; i < ORC_MAXLEV; ++i) {
      if (i > 0) orc_owned_free(&lv[i]);
      free(cof[i]);
      free(blk[i]);
      cof[i] = NULL;
      blk[i] = NULL;
    }
  }
  if (rc == ORC_OK) {
    st->lmax = lmax;
    st->W = W;
    st->U = U;
    st->threshold = threshold;
    st->n_isolated = n - n0;
    st->cut = best_cut;
    st->max_block = cy->max_block[cy->best];
  }
  for (int i = 0; i < ORC_MAXLEV; ++i) {
    orc_owned_free(&lv[i]);
    free(cof[i]);
    free(blk[i]);
  }
  free(pc);
  free(bw);
  free(iso);
  free(newid);
  return rc;
}
