/*
 * sclap.h -- C ABI of the MI355X (gfx950) size-constrained label propagation
 * library: SCLaP clustering, cluster contraction, SCLaP local search, cut,
 * and the multilevel partitioner built from them, for one graph, a batch of
 * graphs, or a served stream of partition jobs.
 *
 * Paper: Meyerhenke, Sanders, Schulz, "Partitioning Complex Networks via
 * Size-constrained Clustering" (2014).  Each entry point names the passage
 * that defines what it computes.
 *
 * Conventions for every call:
 *  - Graphs are symmetric CSR in DEVICE memory owned by the caller: row
 *    offsets int64[n+1], neighbour ids int32[m], edge weights int32[m] (NULL
 *    = all 1), node weights int32 or int64[n] (NULL = all 1).  Each
 *    undirected edge is stored in both rows, with equal weights; no
 *    self-loops, no repeated neighbour in a row; edge weights >= 1, node
 *    weights >= 0 (Section 2.1).  Row order is free: results do not depend
 *    on the order of neighbours inside a row.
 *  - Label, partition and coarse-id arrays are int32 DEVICE arrays owned by
 *    the caller.  Scalars and statistics are HOST memory.
 *  - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *    Calls are stream-ordered; calls that return host results synchronize
 *    the stream before returning.
 *  - An empty graph (n = 0) is valid input: every call returns its trivial
 *    result (no labels, an empty coarse graph, cut 0) without a launch, and
 *    round statistics count the rounds the stop rules give when nothing
 *    moves (clustering: all max_rounds; refinement: two).
 *  - Every call returns SCLAP_OK (0) or a negative SCLAP_E* code and never
 *    throws.  sclap_last_error() returns a description of the last failure
 *    on the calling thread.
 *  - Semantics are synchronous and deterministic: rounds read the previous
 *    round's labels and weights; ties go to the smallest label; odd rounds
 *    only move to smaller labels and even rounds only to larger ones
 *    (direction_rule = 1); moves into a cluster are admitted in increasing
 *    node id while the cluster's weight before the round plus the admitted
 *    weight stays within the cap.  All arithmetic is integer, so results are
 *    bit-identical run to run and across batch compositions.
 */
#ifndef SCLAP_H
#define SCLAP_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SCLAP_OK 0
#define SCLAP_EINVAL (-1)     /* bad argument or precondition */
#define SCLAP_ENOTSYM (-2)    /* sclap_validate: CSR not symmetric / self-loop / repeat */
#define SCLAP_EOVERFLOW (-3)  /* an edge weight sum or k * c(V) would overflow */
#define SCLAP_ENOMEM (-4)     /* device allocation failed */
#define SCLAP_EHIP (-5)       /* a HIP runtime call failed */
#define SCLAP_EBUDGET (-6)    /* job larger than the server's memory budget */
#define SCLAP_ENOTFOUND (-7)  /* unknown ticket */
#define SCLAP_EAGAIN (-8)     /* result not ready yet */

#define SCLAP_MAX_LEVELS 64
#define SCLAP_MAX_ROUNDS 64
#define SCLAP_MAX_CYCLES 16
#define SCLAP_MAX_SUBROUNDS 16
#define SCLAP_MAX_ENSEMBLE 64

typedef struct sclap_ctx sclap_ctx;
typedef struct sclap_graph sclap_graph;
typedef struct sclap_server sclap_server;

/* A CSR graph in device memory (see conventions above). */
typedef struct sclap_csr {
  int64_t n;              /* nodes */
  int64_t m;              /* stored (directed) entries = 2 |E| */
  const int64_t* row_ptr; /* device, n + 1 */
  const int32_t* col;     /* device, m */
  const int32_t* ew;      /* device, m, or NULL for unit edge weights */
  const void* nw;         /* device, n, or NULL for unit node weights */
  int32_t nw_bytes;       /* 4 (int32) or 8 (int64) when nw != NULL */
  int32_t rows_sorted;    /* 1 if every row is ascending (speeds up the initial partition) */
} sclap_csr;

/* Label propagation parameters (Section 3.1: at most l rounds, stop when
 * fewer than 5% of the nodes moved). */
typedef struct sclap_lp_params {
  int32_t max_rounds;     /* l, 1..SCLAP_MAX_ROUNDS */
  int32_t stop_rule;      /* 0: exactly max_rounds rounds; 1: stop after round r >= 2 when
                             20 * (moved_r + moved_{r-1}) < n */
  int32_t direction_rule; /* 1: odd rounds move down, even rounds up (default); 0: no rule */
  int32_t subrounds;      /* Section 4 node ordering by increasing degree: with S >= 2, every round
                             is S sub-rounds; sub-round s rates the nodes of degree class s (0 below
                             degree 4, else floor(log4 degree), at most S - 1) from the labels and
                             weights the previous sub-round left, and admits their moves; the
                             direction rule follows the round.  0 or 1: synchronous rounds.
                             At most SCLAP_MAX_SUBROUNDS. */
} sclap_lp_params;

/* Per-call round statistics (edge visits = sum of the degrees of the nodes
 * rated in each round). */
typedef struct sclap_round_stats {
  int32_t rounds;
  int32_t reserved;
  int64_t visits;
  int64_t moved[SCLAP_MAX_ROUNDS];
  double ms;               /* device time of the rounds (HIP events) */
} sclap_round_stats;

/* Multilevel parameters (Section 3.1; Section 5 parameter values). */
typedef struct sclap_ml_params {
  int32_t f;               /* cap divisor: W = L_max / f */
  int32_t lp_rounds;       /* l during coarsening */
  int32_t refine_rounds;   /* l during uncoarsening (0 = no refinement) */
  int32_t direction_rule;  /* as in sclap_lp_params */
  int64_t threshold;       /* stop coarsening at <= threshold nodes; <= 0: max(60k, n/(60k)) */
  /* Section 4 extensions; all zero gives the plain scheme. */
  int32_t vcycles;         /* iterated multilevel cycles (Section 4; Appendix B.1), 0 or 1: one;
                              cycle c >= 2 starts from the best partition so far, clusters every
                              level within its blocks (no cut edge is contracted) and takes those
                              blocks on its coarsest level instead of an initial partition.  The
                              result is the best cycle's partition: blocks within L_max first,
                              then the smaller cut, ties to the earlier cycle.  <= SCLAP_MAX_CYCLES */
  int32_t subrounds;       /* degree-ordered sub-rounds of every clustering round (see
                              sclap_lp_params); 0 or 1: none */
  int32_t ensemble;        /* clusterings overlaid on every coarsening level (Section 4, ensemble
                              clusterings), 0 or 1: one.  Member e >= 1 starts from the labels
                              (a_e v + b_e) mod n (sclap_cluster_ext); the overlay puts two nodes
                              together iff every member does.  <= SCLAP_MAX_ENSEMBLE */
  int32_t reserved;
  int64_t delta_num;       /* extra imbalance delta = delta_num / delta_den on the coarse levels of */
  int64_t delta_den;       /* the first cycle (Section 4): level i of q refines against
                              floor((1 + eps + delta / (q - i)) ceil(c(V) / k)); 0: none */
} sclap_ml_params;

/* Multilevel statistics.  Level 0 is the input without its degree-0 nodes. */
typedef struct sclap_stats {
  int32_t levels;
  int32_t reserved;
  int64_t n_level[SCLAP_MAX_LEVELS];
  int64_t m_level[SCLAP_MAX_LEVELS];
  int32_t rounds_c[SCLAP_MAX_LEVELS];                 /* clustering rounds on level i */
  int32_t rounds_r[SCLAP_MAX_LEVELS];                 /* refinement rounds on level i */
  int64_t moved_c[SCLAP_MAX_LEVELS][SCLAP_MAX_ROUNDS];
  int64_t moved_r[SCLAP_MAX_LEVELS][SCLAP_MAX_ROUNDS];
  int64_t visits_c[SCLAP_MAX_LEVELS];
  int64_t visits_r[SCLAP_MAX_LEVELS];
  int64_t lmax, W, U, threshold;
  int64_t n_isolated;
  int64_t ip_cut;          /* cut of the initial partition on the coarsest level */
  int64_t cut;
  int64_t max_block;
  double ms_cluster;       /* device time in clustering rounds */
  double ms_contract;
  double ms_initial;
  double ms_refine;
  double ms_total;         /* wall time of the call */
  /* iterated cycles: the per-level fields above describe the last cycle;
     cut and max_block are the returned (best) partition's */
  int32_t cycles;
  int32_t best_cycle;
  int64_t cycle_cut[SCLAP_MAX_CYCLES];
  int64_t cycle_max_block[SCLAP_MAX_CYCLES];
  int64_t cycle_visits[SCLAP_MAX_CYCLES];  /* clustering + refinement edge visits of the cycle */
  int32_t cycle_levels[SCLAP_MAX_CYCLES];
} sclap_stats;

/* ---- context ------------------------------------------------------------ */

/* Create a context on HIP device `device`.  The context owns scratch
 * memory and tuning state; one context may be used by one thread at a
 * time. */
int sclap_create(sclap_ctx** out, int device);
int sclap_destroy(sclap_ctx* ctx);
/* Description of the last failure on the calling thread (the text is kept
 * per thread, so ctx may be NULL). */
const char* sclap_last_error(const sclap_ctx* ctx);
/* Return the device blocks that the context keeps cached for reuse to HIP
 * (synchronises the device first).  Other contexts and servers on the same
 * device can then allocate that memory. */
int sclap_trim(sclap_ctx* ctx);

/* Check the CSR preconditions (symmetry with equal weights, no self-loops,
 * no repeated neighbours, weights in range) on the device.  Returns
 * SCLAP_OK, SCLAP_ENOTSYM or SCLAP_EINVAL. */
int sclap_validate(sclap_ctx* ctx, const sclap_csr* g, void* stream);

/* ---- bounds (Section 2.1 balance constraint; Section 3.1 bound U) -------- */

/* L_max = floor((1 + eps) * ceil(total_w / k)) with eps = eps_num / eps_den,
 * W = floor(L_max_real / f), U = max(max_w, W).  Pure host integer math. */
int sclap_bounds(int64_t total_w, int64_t max_w, int32_t k, int64_t eps_num, int64_t eps_den,
                 int32_t f, int64_t* lmax, int64_t* W, int64_t* U);

/* ---- size-constrained label propagation (Section 3.1) -------------------- */

/* Cluster g under cap U: labels start as node ids; rounds as described in
 * the conventions.  labels_out (device, n) receives the final labels;
 * *n_clusters the number of distinct labels; st (may be NULL) the rounds. */
int sclap_cluster(sclap_ctx* ctx, const sclap_csr* g, int64_t U, const sclap_lp_params* p,
                  int32_t* labels_out, int64_t* n_clusters, sclap_round_stats* st, void* stream);

/* Clustering with the Section 4 extensions.
 * blocks (device, n, or NULL): a partition to respect (Appendix B.1): a node
 *   only joins clusters that lie inside its own block, so no cluster takes
 *   nodes of two blocks and contracting keeps every cut edge of the
 *   partition.  Edge visits count each node's neighbours in its own block.
 * member (>= 0): the ensemble member whose initial labels are used: member 0
 *   starts from the node ids, member e >= 1 from (a_e v + b_e) mod n, where
 *   a_e is the first value from (2654435761 e) mod n upward (cyclically,
 *   skipping 0) that is coprime to n, and b_e = (2246822519 e) mod n.
 * p->subrounds: degree-ordered sub-rounds (see sclap_lp_params).
 * Otherwise as sclap_cluster. */
int sclap_cluster_ext(sclap_ctx* ctx, const sclap_csr* g, int64_t U, const sclap_lp_params* p,
                      const int32_t* blocks, int32_t member, int32_t* labels_out, int64_t* n_clusters,
                      sclap_round_stats* st, void* stream);

/* Overlay of two clusterings (Section 4, ensemble clusterings): nodes u, v
 * share a cluster of the result iff overlay_inout(u) == overlay_inout(v) and
 * labels(u) == labels(v).  Clusters are numbered 0, 1, ... in the order in
 * which a pass over the nodes in increasing id first meets them.
 * overlay_inout and labels: device, n, values in [0, n).  *n_clusters (may be
 * NULL) receives the cluster count. */
int sclap_overlay(sclap_ctx* ctx, int64_t n, int32_t* overlay_inout, const int32_t* labels,
                  int64_t* n_clusters, void* stream);

/* ---- cluster contraction (Section 3.1, Figure 2) -------------------------- */

/* Contract clusters `labels` (device, n, values in [0, n)) into one node
 * each.  Coarse ids rank the labels in use by value; coarse node weight =
 * sum of members; coarse edge weight = sum of the edges between the two
 * clusters; intra-cluster edges vanish; rows ascending.  With
 * drop_isolated, degree-0 nodes join no coarse node (coarse_of = -1).
 * coarse_of_out (device, n) is caller-owned; the coarse graph is allocated
 * by the library and released with sclap_graph_free.  Returns
 * SCLAP_EOVERFLOW if a coarse edge weight exceeds int32. */
int sclap_contract(sclap_ctx* ctx, const sclap_csr* g, const int32_t* labels, int32_t drop_isolated,
                   int32_t* coarse_of_out, sclap_graph** coarse_out, void* stream);
/* View of a library-owned graph (int64 node weights, rows ascending). */
int sclap_graph_view(const sclap_graph* cg, sclap_csr* view);
int sclap_graph_free(sclap_graph* cg);
/* Copy a library-owned graph into caller-owned device arrays: row_ptr
 * int64[n+1], col int32[m], ew int32[m], nw int64[n] (stream-ordered). */
int sclap_graph_copy(const sclap_graph* cg, int64_t* row_ptr, int32_t* col, int32_t* ew, int64_t* nw,
                     void* stream);

/* ---- initial partition (replaces the paper's KaHIP step, Section 3.1) ---- */

/* Breadth-first order (searches start at the smallest unvisited id,
 * neighbours appended in ascending id), cut into k consecutive chunks:
 * block(v) = min(k-1, floor(k P(v) / C)), P(v) = weight before v.  With
 * skip_isolated, degree-0 nodes get block -1 and are not counted in C. */
int sclap_initial_partition(sclap_ctx* ctx, const sclap_csr* g, int32_t k, int32_t skip_isolated,
                            int32_t* part_out, void* stream);

/* ---- SCLaP as local search (Section 3.1 last paragraph; Section 4) -------- */

/* Refine part_inout (device, n, blocks in [0,k), or -1 for degree-0 nodes
 * that take no part) with label propagation under cap lmax; a node of an
 * overloaded block ignores its own block.  Only boundary nodes are rated
 * after round 1 (exact: an interior node cannot move).  Stops after
 * p->max_rounds rounds or two consecutive rounds without a move.
 * For k <= 64 the library keeps every node's connection to every block
 * (n x k int32 of device memory while a level is refined) and rates later
 * rounds from it; the result is the same. */
int sclap_refine(sclap_ctx* ctx, const sclap_csr* g, int32_t k, int64_t lmax, const sclap_lp_params* p,
                 int32_t* part_inout, sclap_round_stats* st, void* stream);

/* ---- cut (Section 2.1) --------------------------------------------------- */

/* *cut_out = sum of weights of edges whose ends lie in different blocks;
 * block_w_out (HOST, k entries, may be NULL) = block weights (nodes with
 * block -1 are not counted). */
int sclap_cut(sclap_ctx* ctx, const sclap_csr* g, const int32_t* part, int32_t k, int64_t* cut_out,
              int64_t* block_w_out, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): the cut
 * and, if block_w_out is not NULL, the block weights of sclap_cut, written
 * to DEVICE memory the caller owns (cut_out: 1 int64, block_w_out: k int64)
 * on `stream`, with no host synchronisation and no allocation of any kind.
 * The cut's per-workgroup partial sums use a fixed device array of the
 * library (64 KiB, 8192 entries, enough for any edge count; one copy per
 * GPU, kept until the process ends, its address looked up by sclap_create
 * or by the first call on a device).  k is at most 4096 when block weights
 * are asked for (SCLAP_EINVAL otherwise).  Calls that overlap on one GPU
 * (on different streams, or from several threads) share that array and
 * race; calls in order on one stream do not.  Node weights are read as
 * given (nw_bytes 4 or 8, NULL for unit weights). */
int sclap_cut_noalloc(const sclap_csr* g, const int32_t* part, int32_t k, int64_t* cut_out, int64_t* block_w_out,
                      void* stream);

/* ---- multilevel partition (Section 1 scheme; Section 3.1) ----------------- */

/* Bounds from the whole input; degree-0 nodes set aside; coarsen by
 * SCLaP (cap U, stop rule 1) + contraction while the level has more than
 * the threshold nodes, stopping after a level that shrank by less than 5%;
 * initial partition of the coarsest level; project and refine (cap L_max)
 * on every level from the coarsest to the finest; place the degree-0 nodes
 * into the lightest blocks up to a common level in increasing id; cut.
 * part_out (device, n) is caller-owned. */
int sclap_partition(sclap_ctx* ctx, const sclap_csr* g, int32_t k, int64_t eps_num, int64_t eps_den,
                    const sclap_ml_params* p, int32_t* part_out, sclap_stats* st, void* stream);

/* ---- batched partition ----------------------------------------------------- */

/* Partition `count` independent graphs together: every step (rating,
 * admission, contraction, initial partition, refinement) is one fused launch
 * over all graphs still at that step.  Each result equals sclap_partition on
 * that graph alone.  parts_out[i] (device, gs[i].n) and sts (HOST, count
 * entries, may be NULL) are caller-owned. */
int sclap_partition_batch(sclap_ctx* ctx, int32_t count, const sclap_csr* gs, const int32_t* ks,
                          int64_t eps_num, int64_t eps_den, const sclap_ml_params* p,
                          int32_t* const* parts_out, sclap_stats* sts, void* stream);

/* ---- served partition jobs (continuous batching) --------------------------- */

typedef struct sclap_job {
  sclap_csr graph;         /* device memory; copied by submit, caller may free after */
  int32_t k;
  int32_t reserved;
  int64_t eps_num, eps_den;
  sclap_ml_params params;
  int32_t* part_out;       /* device, graph.n; written when the job completes */
} sclap_job;

typedef struct sclap_job_result {
  int32_t status;          /* SCLAP_OK or an error code */
  int32_t reserved;
  int64_t cut;
  int64_t max_block;
  double latency_ms;       /* submit -> completion */
  double queue_ms;         /* submit -> admission */
} sclap_job_result;

/* A server owns a worker thread that keeps the sum of the device footprints
 * of its queued and running jobs within hbm_budget_bytes, admits up to
 * max_active queued jobs to the device in arrival order, keeps each admitted
 * job's graph hierarchy resident on the device, and advances all admitted
 * jobs together step by step, so that jobs admitted while others run share
 * their launches.  A job's result equals sclap_partition on it alone. */
int sclap_server_create(sclap_ctx* ctx, int64_t hbm_budget_bytes, int32_t max_active, sclap_server** out);
/* Copies job->graph (device memory that must be complete: the caller has
 * synchronised the stream that wrote it) and queues the job.  SCLAP_EBUDGET
 * if the job's footprint alone exceeds the budget.  Blocks while the job's
 * footprint does not fit in the budget beside the queued and running jobs.
 * part_out stays owned by the caller and must stay allocated until the
 * job's result was taken. */
int sclap_server_submit(sclap_server* srv, const sclap_job* job, uint64_t* ticket);
/* SCLAP_OK with *res filled once done (part_out is then complete on the
 * device), after which the ticket is forgotten; SCLAP_EAGAIN while pending;
 * SCLAP_ENOTFOUND for an unknown or already taken ticket. */
int sclap_server_poll(sclap_server* srv, uint64_t ticket, sclap_job_result* res);
int sclap_server_wait(sclap_server* srv, uint64_t ticket, sclap_job_result* res);
/* The same calls under the names of the served-job interface: submit,
 * poll and wait a job of the server. */
int sclap_submit(sclap_server* srv, const sclap_job* job, uint64_t* ticket);
int sclap_poll(sclap_server* srv, uint64_t ticket, sclap_job_result* res);
int sclap_wait(sclap_server* srv, uint64_t ticket, sclap_job_result* res);
/* The device bytes a server charges against its budget for a job on graph
 * g with k blocks, from submission (when the input is copied) to completion
 * (host math, no device access): input_bytes of the copy, and the footprint,
 * which bounds everything the job holds at once: the input copy, two
 * weighted copies of the hierarchy, the LP state of a level with the block
 * connections of refinement, its share of the context scratch of the fused
 * rounds, and the temporaries of a contraction, plus what the Section 4
 * extensions of p (may be NULL: none) add: the best partition and the level
 * without cut edges of iterated cycles, the degree classes of sub-rounds, the
 * overlay of an ensemble. */
int sclap_server_footprint(const sclap_csr* g, int32_t k, const sclap_ml_params* p, int64_t* input_bytes,
                           int64_t* footprint_bytes);
/* Latency percentiles over completed jobs and throughput since creation;
 * peak_bytes: the most footprint bytes charged at once; peak_active: the most
 * jobs admitted to the device at once.  Any output may be NULL. */
int sclap_server_stats(sclap_server* srv, double* p50_ms, double* p99_ms, double* jobs_per_s,
                       int64_t* completed, int64_t* peak_bytes, int64_t* peak_active);
/* Finishes every queued and running job, then frees the server. */
/* Hold (hold != 0) or release admission: while held, submitted jobs queue
 * (their footprints are charged) and no queued job is admitted to the
 * device; jobs already admitted run on.  Releasing admits queued jobs up to
 * max_active at once, for callers that submit a group of requests together. */
int sclap_server_hold(sclap_server* srv, int32_t hold);
int sclap_server_destroy(sclap_server* srv);

/* ---- measurement ------------------------------------------------------------ */

/* Time the rating step (degree binning excluded) and whole LP rounds of every
 * following call with HIP events on the call's stream.  Enabling resets the
 * accumulators. */
int sclap_profile_enable(sclap_ctx* ctx, int32_t on);
/* Accumulated since enabling: rating-step device ms and launches, edge
 * visits and nodes rated, whole-round device ms and rounds. */
int sclap_profile_read(sclap_ctx* ctx, double* rate_ms, int64_t* rate_launches, int64_t* visits, int64_t* nodes,
                       double* round_ms, int64_t* rounds);
/* Per launch group (0: rating, degree 1-32, one thread per node; 1: degree
 * 33-128, 64 lanes per node or one wave with an LDS table; 2: degree
 * 129-1024; 3: degree 1025-4096, one workgroup with an LDS table; 4: the
 * multi-workgroup hub path; 5: the refinement marking kernels, which add the
 * neighbours of moved nodes to the next rated set and move their edge
 * weights between block connections), `count` entries each (any pointer may
 * be NULL): device ms; algorithmic bytes (rating: 4 B neighbour id + 4 B
 * neighbour label, not read in the first clustering round of a level, where
 * labels are node ids [+ 4 B edge weight] per visit, 32 B per rated node;
 * marking: 8 B per rated position, 20 B per mover, per entry of a mover's
 * row 5 B, plus 16 B of block-connection updates [+ 4 B edge weight] in
 * rounds that update them); edge visits (marking: mover entries) and nodes
 * (marking: movers), summed over rounds; and launches = rounds in which the
 * group's kernels ran.  *rounds = LP rounds profiled. */
int sclap_profile_kernels(sclap_ctx* ctx, int32_t count, double* ms, double* bytes, int64_t* visits, int64_t* nodes,
                          int64_t* launches, int64_t* rounds);

/* ---- tuning of the degree bins (clustering rounds) ------------------------ */

/* Nodes of degree 1..32 are rated one thread per node (unit weights) and
 * nodes of degree above 4096 by the hub path; degrees in between go to bins
 * 3..7, whose kernels are: bin 3 one wave with a 128-slot LDS table, bin 4
 * one wave with 256 slots, bin 5 one wave with 1024, bin 6 one workgroup of
 * 256 threads with up to 4096, bin 7 one workgroup of 512 with up to 8192.
 * hi[0..3] are the largest degrees of bins 3..6: 32 <= hi[0] <= 64,
 * hi[0] <= hi[1] <= 128, hi[1] <= hi[2] <= 512, hi[2] <= hi[3] <= 2048
 * (default 64, 128, 512, 1024).  The bounds change
 * only which kernel rates a node, never the result; they apply to the
 * clustering rounds of the context's later calls. */
int sclap_set_bin_bounds(sclap_ctx* ctx, const int32_t* hi);
int sclap_get_bin_bounds(sclap_ctx* ctx, int32_t* hi);
/* Autotuner: times `rounds` clustering rounds of g under cap U (no stop
 * rule; the best of two runs) with the default bounds and with each of a
 * grid of candidate bounds (hi[0] in {32, 64}, hi[1] in {64, 128}, hi[2] in
 * {128, 256, 512}, hi[3] in {512, 1024, 2048}, rising), keeps the fastest in the
 * context and returns it in hi_out (4 entries, may be NULL) with its time
 * and the default bounds' time in ms (may be NULL).  Synchronous. */
int sclap_autotune(sclap_ctx* ctx, const sclap_csr* g, int64_t U, int32_t rounds, int32_t* hi_out, double* best_ms,
                   double* default_ms, void* stream);

/* Counts of the paths the LP rounds of a context (or of a server's context)
 * took since it was created, always kept: out[0] rounds, out[1] rounds fused
 * over more than one job, out[2] binning scans done device-wide (more than
 * one workgroup's worth of tiles), out[3] device-wide contended admissions
 * (more contended movers than one workgroup sorts), out[4] rounds with rows
 * above 4096 entries (the hub path).  count: entries wanted (at most 5). */
int sclap_path_counters(sclap_ctx* ctx, int32_t count, int64_t* out);
int sclap_server_path_counters(sclap_server* srv, int32_t count, int64_t* out);

#ifdef __cplusplus
}
#endif
#endif /* SCLAP_H */
