/*
 * sclap_oracle.h -- types and entry points of the plain CPU oracle.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the package smoke check and
 * the benchmark's CPU-baseline leg may load the oracle library.  It shares
 * no code, header or helper with the device library.
 */
#ifndef SCLAP_ORACLE_H
#define SCLAP_ORACLE_H

#include <stdint.h>

#define ORC_MAXLEV 64
#define ORC_MAXR 64
#define ORC_MAXCYC 16

enum { ORC_OK = 0, ORC_EINVAL = -1, ORC_ENOMEM = -2, ORC_EOVERFLOW = -3 };

typedef struct orc_graph {
  int64_t n;
  int64_t m;            /* directed entries */
  const int64_t* rp;    /* n + 1 */
  const int32_t* col;   /* m */
  const int32_t* ew;    /* m, or NULL for unit edge weights */
  const int64_t* nw;    /* n, or NULL for unit node weights */
} orc_graph;

typedef struct orc_owned {
  int64_t n, m;
  int64_t* rp;
  int32_t* col;
  int32_t* ew;
  int64_t* nw;
} orc_owned;

typedef struct orc_stats {
  int32_t levels;                       /* graphs in the hierarchy, level 0 = input without isolated nodes */
  int32_t pad;
  int64_t n_level[ORC_MAXLEV];
  int64_t m_level[ORC_MAXLEV];
  int32_t rounds_c[ORC_MAXLEV];         /* clustering rounds run on level i */
  int32_t rounds_r[ORC_MAXLEV];         /* refinement rounds run on level i */
  int64_t moved_c[ORC_MAXLEV][ORC_MAXR];
  int64_t moved_r[ORC_MAXLEV][ORC_MAXR];
  int64_t visits_c[ORC_MAXLEV];         /* coarsening edge visits on level i */
  int64_t visits_r[ORC_MAXLEV];         /* refinement edge visits on level i */
  int64_t lmax, W, U, threshold;
  int64_t n_isolated;
  int64_t ip_cut;                       /* cut of the initial partition (coarsest level) */
  int64_t cut;
  int64_t max_block;
} orc_stats;

/* The extensions of Section 4 (all zero: the plain multilevel scheme). */
typedef struct orc_mlx {
  int32_t vcycles;      /* multilevel iterations; <= 1: one */
  int32_t subrounds;    /* degree-ordered sub-rounds per clustering round; <= 1: synchronous rounds */
  int32_t ensemble;     /* clusterings overlaid per coarsening level; <= 1: one */
  int32_t pad;
  int64_t delta_num;    /* extra imbalance delta = num / den on coarse levels of the first cycle; */
  int64_t delta_den;    /* num 0: none */
} orc_mlx;

/* Per-cycle results of an iterated multilevel run. */
typedef struct orc_cycles {
  int32_t cycles;       /* cycles run */
  int32_t best;         /* index of the returned partition */
  int64_t cut[ORC_MAXCYC];
  int64_t max_block[ORC_MAXCYC];
  int64_t visits[ORC_MAXCYC];   /* clustering + refinement edge visits of the cycle */
  int32_t levels[ORC_MAXCYC];
  int64_t lmax[ORC_MAXCYC][ORC_MAXLEV];  /* refinement bound used on each level of each cycle */
} orc_cycles;

int orc_bounds(int64_t total_w, int64_t max_w, int32_t k, int64_t eps_num, int64_t eps_den, int32_t f,
               int64_t* lmax, int64_t* W, int64_t* U);
void orc_rate(const orc_graph* g, const int32_t* lab, const int64_t* Wt, int64_t nlabels, int64_t cap,
              int32_t round, int32_t dir_rule, int32_t refine, int32_t* desire);
int64_t orc_admit_apply(const orc_graph* g, const int32_t* desire, int32_t* lab, int64_t* Wt, int64_t nlabels,
                        int64_t cap, uint8_t* admitted_out);
int32_t orc_cluster(const orc_graph* g, int64_t U, int32_t max_rounds, int32_t stop_rule, int32_t dir_rule,
                    int32_t* lab, int64_t* moved_out, int64_t* visits_out);
int orc_contract(const orc_graph* g, const int32_t* lab, int32_t drop_isolated, int32_t* coarse_of,
                 orc_owned* out);
void orc_owned_free(orc_owned* o);
void orc_initial_partition(const orc_graph* g, int32_t k, int32_t skip_isolated, int32_t* part);
int64_t orc_cut(const orc_graph* g, const int32_t* part, int32_t k, int64_t* block_w);
int32_t orc_refine(const orc_graph* g, int32_t k, int64_t lmax, int32_t max_rounds, int32_t dir_rule,
                   int32_t* part, int64_t* moved_out, int64_t* visits_out);
void orc_place_isolated(const int64_t* nw, int64_t n, const uint8_t* isolated, int32_t k, const int64_t* B,
                        int32_t* part);
int orc_partition(const orc_graph* in, int32_t k, int64_t eps_num, int64_t eps_den, int32_t f, int32_t lp_rounds,
                  int32_t ref_rounds, int64_t threshold, int32_t dir_rule, int32_t* part_out, orc_stats* st);

#endif
