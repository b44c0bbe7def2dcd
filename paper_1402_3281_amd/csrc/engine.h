// engine.h -- host-side executor of the multilevel scheme over a set of jobs.
//
// A job is one graph's partition (or a single clustering / refinement run).
// The executor advances all jobs step by step; every step fuses the work of
// all jobs that are at that step into one set of launches:
//   LP round   (clustering rounds and refinement rounds together)
//   contract   (jobs whose clustering of a level finished)
//   initial    (jobs that reached their coarsest level)
//   finish     (jobs whose finest level is refined)
#pragma once

#include <hip/hip_runtime.h>

#include <atomic>
#include <vector>

#include "common.h"
#include "lp.h"
#include "misc.h"

namespace sclap {

struct Level {
  int64_t n = 0, m = 0;
  const int64_t* rp = nullptr;
  const int32_t* col = nullptr;
  const int32_t* ew = nullptr;
  const int64_t* nw = nullptr;
  // owned storage (coarse levels; widened node weights of the input)
  int64_t* own_rp = nullptr;
  int32_t* own_col = nullptr;
  int32_t* own_ew = nullptr;
  int64_t* own_nw = nullptr;
  int32_t* coarse_of = nullptr;  // n: map to the next coarser level
  int32_t* blk = nullptr;        // n: blocks of the partition the clustering respects, or nullptr
  bool blk_owned = false;
  int rows_sorted = 0;
  int64_t n_active = 0;          // nodes of degree > 0
  int64_t max_deg = 0;
  int64_t max_w = 0;             // largest node weight
  // sizes of the hub rating path on this level (degree > kBinBlock)
  int64_t hubs = 0;
  int64_t hub_stage = 0;         // staged pair slots
  int64_t hub_parts_c = 0, hub_mat_c = 0;  // label parts, matrix entries: clustering
  int64_t hub_parts_r = 0, hub_mat_r = 0;  // ... refinement
};

enum Stage : int { ST_COARSEN, ST_CONTRACT, ST_IP, ST_REFINE, ST_FINISH, ST_DONE, ST_ERROR };
enum Kind : int { JOB_PARTITION, JOB_CLUSTER, JOB_REFINE };

struct Job {
  Kind kind = JOB_PARTITION;
  Stage stage = ST_COARSEN;
  int status = SCLAP_OK;
  // parameters
  int32_t k = 2;
  int64_t lmax = 0, U = 0, W = 0, threshold = 0;
  int32_t lp_rounds = 10, ref_rounds = 10, dir_rule = 1, stop_rule = 1;
  int64_t total_w = 0;
  std::vector<Level> lv;
  int cur = 0;
  // LP state of the current stage
  int32_t round = 0;
  int64_t moved_prev = 0;
  int32_t zero_streak = 0;
  int64_t n_stop = 0;              // node count of the 5% rule
  int32_t* lab = nullptr;          // labels (cluster) or blocks (refine)
  bool lab_owned = false;
  int32_t* desire = nullptr;
  uint8_t* adm = nullptr;
  int64_t* Wt = nullptr;
  int64_t* inc = nullptr;
  uint8_t* fcur = nullptr;
  uint8_t* fnext = nullptr;
  int32_t* conn = nullptr;         // refine: n x k block connections (k <= kConnMaxK)
  bool conn_stale = false;         // the last round's moves were not added to conn
  int64_t nlabels = 0;
  // extensions (Section 4)
  int32_t vcycles = 1, cycle = 0;        // iterated multilevel cycles; the current one
  int32_t subrounds = 0, sub = 0;        // degree-ordered sub-rounds per round; the current one
  int64_t sub_moved = 0, sub_visits = 0; // sums over the sub-rounds of the current round
  int32_t members = 1, member = 0;       // ensemble clusterings per level; the current one
  int64_t delta_num = 0, delta_den = 1;  // extra imbalance on coarse levels of the first cycle
  int64_t eps_num = 3, eps_den = 100;
  int64_t lmax_cur = 0;                  // refinement bound of the level being refined
  uint8_t* cls = nullptr;                // degree classes of the level being clustered (subrounds >= 2)
  Level flt;                             // that level without the cut edges of its blocks
  bool flt_on = false;
  int32_t* ovl = nullptr;                // overlay of the members clustered so far
  bool wt_clusters = true;               // Wt holds the weights of the clusters of lab
  int32_t* best = nullptr;               // best partition of the input so far (several cycles)
  int64_t best_cut = 0, best_over = 0;
  int32_t best_cycle = 0;
  int64_t lp_gen = 0;                    // changes whenever the rated node set may change
  // Partitions of inputs with degree-0 nodes work on the input without them
  // (level 0, its nodes numbered in id order); `input` is the caller's graph
  // (with widened node weights) and act maps level-0 nodes to input ids.
  bool compact = false;
  Level input;
  int32_t* act = nullptr;
  // outputs
  int32_t* part_out = nullptr;     // caller buffer (level-0 blocks / labels)
  sclap_stats st{};
  sclap_round_stats rst{};         // single clustering / refinement runs
  double t_start = 0;
};

// Device blocks that a context keeps for reuse instead of returning them to
// the HIP memory pool (whose frees of large blocks take milliseconds).
struct CachedBlock {
  void* p;
  size_t bytes;
  hipStream_t st;
};

struct Ctx {
  int device = 0;
  int cu_count = 256;
  // upper degree bounds of bins 3..6 for clustering rounds (sclap_autotune)
  int32_t tune_hi[4] = {kBinHiDefault[0], kBinHiDefault[1], kBinHiDefault[2], kBinHiDefault[3]};
  // freed device blocks kept for later allocations on the same stream
  std::vector<CachedBlock> cache;
  size_t cache_bytes = 0;
  size_t cache_limit = (size_t)96 << 30;  // bytes kept cached at most
  // scratch reused by every step
  Scratch bins, ckeys, ckeys2, tkey, wv, prefix, prim, hub_chunk, hub_tab, hub_own, hub_gkeys;
  Scratch step_ctr, small, slots_dev, ip_slots, hub_slice, hub_best, movers, binfo, hub_maps, binmeta;
  Scratch hub_P, hub_mat, binscr, cutbuf, tadm, hub_keep, trows, part8, lab8;
  // jobs and levels whose nodes the current bins hold (clustering rounds only)
  std::vector<std::pair<const void*, int>> bin_sig;
  bool bin_sig_valid = false;
  int64_t bin_cap_used = 0;
  bool hub_keep_valid = false;     // the hub layout buffers hold the last clustering round's layout
  // pinned host staging
  int64_t* pin = nullptr;
  size_t pin_bytes = 0;
  DevSlot* pin_slots = nullptr;
  size_t pin_slots_cap = 0;
  // optional timing of the rating kernels (per degree bin) and LP rounds
  bool profile = false;
  // [0..kRateGroups] rating launch groups, [kRateGroups+1], [kRateGroups+2]
  // the whole round, [kRateGroups+3], [kRateGroups+4] the marking kernels
  hipEvent_t ev[kBins + 3];
  double prof_rate_ms = 0;         // sum over rounds of the whole rating step
  int64_t prof_rate_launches = 0;
  int64_t prof_rate_visits = 0;
  int64_t prof_rate_nodes = 0;
  double prof_round_ms = 0;        // whole LP rounds
  int64_t prof_rounds = 0;
  double prof_k_ms[kBins] = {};    // per rating launch group (kRateGroups used)
  double prof_k_bytes[kBins] = {}; // algorithmic bytes moved by that kernel
  int64_t prof_k_visits[kBins] = {};
  int64_t prof_k_nodes[kBins] = {};
  int64_t prof_k_launches = 0;     // rounds profiled
  int64_t prof_k_group_launches[kBins] = {};  // rounds in which the group's kernels ran
  // Which paths the LP rounds took (kept always, read by sclap_path_counters):
  // [0] rounds, [1] rounds over more than one job, [2] device-wide binning
  // scans, [3] device-wide contended admissions, [4] rounds with a hub row
  std::atomic<int64_t> path_ctr[kPathCounters] = {};
};

int ctx_ensure_pin(Ctx* c, size_t bytes);
// While a CtxScope for c is alive on a thread, dalloc and dfree on that
// thread take blocks from and return blocks to c's cache.
struct CtxScope {
  Ctx* prev;
  explicit CtxScope(Ctx* c);
  ~CtxScope();
};
// Returns every cached block of c to HIP (synchronises the device first).
void ctx_trim(Ctx* c);
// Frees every scratch buffer, the pinned staging and the events of c.
void ctx_release(Ctx* c, hipStream_t st);
// The tile-row table (misc.h) of a graph, built in the context's scratch;
// *out stays NULL for an empty graph.  Valid until the next call on c.
int ctx_tile_rows(Ctx* c, const int64_t* rp, int64_t n, int64_t m, const int32_t** out, hipStream_t st);
int ctx_ensure_slots(Ctx* c, size_t count);

// Prepare a job's level 0 from the caller's CSR (widens node weights).
int job_set_input(Ctx* c, Job* j, const sclap_csr* g, hipStream_t st);
// Partitions: make level 0 the input without its degree-0 nodes (after
// level_totals of the input; nothing to do without such nodes).
int job_compact_input(Ctx* c, Job* j, hipStream_t st);
// Compute per-level totals (n_active, hub table needs); returns via sync.
int level_totals(Ctx* c, Job* j, Level* L, int64_t* sum_w, int64_t* max_w, hipStream_t st);
// Start clustering on level cur (labels = node ids).
int job_begin_cluster(Ctx* c, Job* j, hipStream_t st);
// Start refinement on level cur with blocks in `part` (owned by the job).
int job_begin_refine(Ctx* c, Job* j, int32_t* part, bool owned, hipStream_t st);
void job_release_lp(Job* j, hipStream_t st, bool keep_lab);
// Frees the respect graph and degree classes of the level being clustered.
void job_release_ext(Job* j, hipStream_t st);
void job_release_levels(Job* j, hipStream_t st);

// One fused LP round over the given jobs (all in ST_COARSEN or ST_REFINE).
int lp_round(Ctx* c, std::vector<Job*>& jobs, hipStream_t st);

// Upper bounds of the context scratch a fused round sizes by its total node
// count and by its slots' stored entries, with the 1/4 growth margin of
// Scratch::ensure: degree bins (4 B) and their rows (8 B) for each of kBins
// bins, hub own/best rows (16 B), rated list, old blocks and big movers
// (12 B), contended keys (8 B) and their sort/scan buffers (28 B, plus sort
// space), hub layout rows (20 B), binning and tile-admission scans; per
// stored entry the staged (label, sum) pairs of hub rows (8 B per pair, room
// for a whole chunk of pairs per chunk of entries) and the hub chunk x part
// matrix.
constexpr int64_t kRoundBytesPerNode = 320;
constexpr int64_t kRoundBytesPerEntry = 40;
// Temporaries of contracting a level, per stored entry: the cross keys as
// emitted (room for every entry, 8 B, and 4 B weights), their sorted copy
// and sums (at most one per undirected edge, 8 B each, weights 4 B), sort
// space, and the sorted mirror of the coarse edges.
constexpr int64_t kContractBytesPerEntry = 48;

// Served jobs: device bytes of a job's input copy, and an upper bound of
// everything the job holds at once on the device (see server.hip).
int64_t input_bytes_of(const sclap_csr& g);
int64_t footprint_of(const sclap_csr& g, int32_t k, const sclap_ml_params* p);
// Contract level cur of a job into level cur + 1.
int contract_level(Ctx* c, Job* j, int i, int drop_isolated, hipStream_t st);
// Fused initial partition of the jobs' current (coarsest) levels.
int ip_jobs(Ctx* c, std::vector<Job*>& jobs, std::vector<int32_t*>& parts, hipStream_t st);

// One executor step over the jobs (see engine.hip); run_jobs loops it.
int step_jobs(Ctx* c, std::vector<Job*>& jobs, hipStream_t st, bool* all_done);
int run_jobs(Ctx* c, std::vector<Job*>& jobs, hipStream_t st);

double now_ms();
int bits_for(int64_t count);

}  // namespace sclap
