// misc.h -- launchers of the contraction, initial-partition, projection, cut,
// block-weight, placement and validation kernels.
#pragma once

#include "common.h"

namespace sclap {

int fill_i32(int32_t* p, int64_t n, int32_t v, hipStream_t st);
int fill_i64(int64_t* p, int64_t n, int64_t v, hipStream_t st);
int fill_u8(uint8_t* p, int64_t n, uint8_t v, hipStream_t st);
int fill_u32(uint32_t* p, int64_t n, uint32_t v, hipStream_t st);

// out (device, kGraphTotals entries): sum c, max c, nodes of degree > 0,
// the hub rating path sizes (see k_graph_totals), and the largest degree.
constexpr int kGraphTotals = 10;
int graph_totals(const int64_t* rp, const int64_t* nw, int64_t n, int64_t k, unsigned long long* out,
                 hipStream_t st);
int widen_nw(const void* src, int bytes, int64_t n, int64_t* dst, hipStream_t st);
int init_cluster(int32_t* lab, int32_t* desire, int64_t* W, const int64_t* nw, int64_t n, hipStream_t st);
int copy_i32(const int32_t* a, int32_t* b, int64_t n, hipStream_t st);
// The nodes of degree > 0 as one 64-bit mask per 64 ids (words, ceil(n/64))
// and the masks' popcounts (wcnt); wpre below is the exclusive scan of wcnt.
int active_words(const int64_t* rp, int64_t n, uint64_t* words, int32_t* wcnt, hipStream_t st);
// The input without its degree-0 nodes (n0 of the n nodes have degree > 0):
// row offsets rp0 (n0 + 1), columns col0 (m, renumbered), node weights nw0
// (n0) and act (n0: input id of each compacted node).  Entries keep their
// order, so edge weights are shared.
// rec: compact_rec_bytes(n) bytes of scratch (16-byte aligned).
int64_t compact_rec_bytes(int64_t n);
int compact_graph(const int64_t* rp, const int32_t* col, const int64_t* nw, const uint64_t* words,
                  const int32_t* wpre, int64_t n, int64_t m, int64_t n0, int64_t* rp0, int32_t* col0, int64_t* nw0,
                  int32_t* act, void* rec, hipStream_t st);
// dst(i) = src(idx(i)) and dst(idx(i)) = src(i), i < n.
int gather_i32(const int32_t* idx, const int32_t* src, int64_t n, int32_t* dst, hipStream_t st);
int scatter_i32(const int32_t* idx, const int32_t* src, int64_t n, int32_t* dst, hipStream_t st);
int block_weights(const int32_t* part, const int64_t* nw, int64_t n, int32_t k, int64_t* W, hipStream_t st);
// Block weights from node weights as the caller gives them (nw_bytes 4 or 8,
// nw NULL for unit weights) into W (k entries, zeroed here by a kernel);
// k at most kBlockWeightsLdsK.  Allocates nothing.
constexpr int32_t kBlockWeightsLdsK = 4096;
int block_weights_raw(const int32_t* part, const void* nw, int nw_bytes, int64_t n, int32_t k, int64_t* W,
                      hipStream_t st);
// Workgroup partial sums cut_edges needs for m entries.
int cut_partials(int64_t m);
// *out = the cut: sum of w over the undirected edges (entries u < v of the
// symmetric graph) joining different blocks.
int cut_edges(const int64_t* rp, const int32_t* col, const int32_t* ew, const int32_t* part, int64_t n, int64_t m,
              unsigned long long* out, int64_t* partial, hipStream_t st, const int32_t* trow = nullptr,
              const uint8_t* part8 = nullptr);
// b(v) = a(v) as one byte (blocks of a partition with k <= 256): the cut
// then gathers the blocks from a quarter of the bytes (part8 above, used
// instead of part when not NULL).
int narrow_u8(const int32_t* a, int64_t n, uint8_t* b, hipStream_t st);
// The tile-row table of the edge-centric kernels (tile_rows_len(m) int32
// entries): entry t is the row holding entry t * 2048 of the graph, the last
// is n - 1.  The edge-centric launchers take it as trow; without it (NULL)
// every tile searches the row offsets for its rows.
int64_t tile_rows_len(int64_t m);
int tile_rows(const int64_t* rp, int64_t n, int64_t m, int32_t* trow, hipStream_t st);

int contract_flag(const int32_t* lab, const int64_t* rp, int64_t n, int drop, int32_t* used, hipStream_t st);
// coarse_of and coarse node weights; with W (label weights of the labels in
// [0, n), as kept by the clustering) the weights are copied, else summed.
int contract_coarse_of(const int32_t* lab, const int64_t* rp, const int64_t* nw, int64_t n, int drop,
                       const int32_t* cid, int32_t* cof, int64_t* cnw, int64_t nc, const int32_t* used,
                       const int64_t* W, hipStream_t st);
// The entries (u, v) with u < v whose ends lie in coarse nodes x != y (one
// per undirected edge of the symmetric graph) as keys
// min(x, y) * 2^bits + max(x, y), with their weights in vals (NULL: not
// written), in no particular order; *cursor (device, zeroed here) ends as
// their count, and keys/vals need room for every entry with u < v (at most
// m); packed (2 bits <= 32): keys hold key << 32 | weight.
int contract_cross(const int64_t* rp, const int32_t* col, const int32_t* ew, const int32_t* cof, int64_t n,
                   int64_t m, int bits, unsigned long long* cursor, uint64_t* keys, int32_t* vals, int packed,
                   const int32_t* trow, hipStream_t st);
// The reduced upper entries (ukeys x * 2^bits + y with x < y, ascending; aggs
// their weights, m of them) mirrored to keys y * 2^bits + x with int32
// weights in mw (packed: key << 32 | weight in mkeys, mw unused); *overflow
// set if a weight exceeds int32.
int contract_mirror(const uint64_t* ukeys, const int64_t* aggs, int64_t m, int bits, int packed, uint64_t* mkeys,
                    int32_t* mw, unsigned* overflow, hipStream_t st);
// Coarse CSR from the upper entries (mu) and the sorted mirror (ml, lkeys/lw
// as from contract_mirror, sorted): rows ascending, lower neighbours first.
// ru, rl: nc + 1 scratch entries each; rp: nc + 1.
int contract_finish2(const uint64_t* ukeys, const int64_t* aggs, int64_t mu, const uint64_t* lkeys, const int32_t* lw,
                     int64_t ml, int bits, int packed, int64_t nc, int64_t* ru, int64_t* rl, int64_t* rp,
                     int32_t* col, int32_t* ew, hipStream_t st);
int project(const int32_t* cof, const int32_t* pc, int64_t n, int32_t* pf, hipStream_t st);

// One graph of a fused initial-partition launch.
struct IpSlot {
  const int64_t* rp;
  const int32_t* col;
  const int64_t* nw;
  int64_t n;
  int32_t k;
  int32_t skip_isolated;
  int32_t rows_sorted;
  int32_t pad;
  int32_t* part;   // n, pre-filled with -1
  int32_t* order;  // n scratch
  int32_t* pos;    // n scratch, pre-filled with -1
  int32_t* claim;  // n scratch, pre-filled with INT32_MAX
  int32_t* cnt;    // n scratch
  int64_t* state;  // 4: head, tail, next seed, yielded (zero before the first launch)
  uint32_t* err;   // set nonzero if the LDS claim table filled up (the partition fails)
};
// One workgroup per slot; see k_ip_bfs for allow_yield / big_entries.
// max_n: the largest n over the slots (graphs of up to 2^18 nodes keep
// their search state in LDS).
int initial_partition(const IpSlot* dev_slots, int count, int64_t max_n, int allow_yield, int64_t big_entries,
                      hipStream_t st);
// Grid-wide expansion of one level of the BFS of a single slot.
int ip_level_deg(const IpSlot* slot, int64_t head, int64_t F, int64_t* deg, hipStream_t st);
int ip_level_entries(const IpSlot* slot, int64_t head, int64_t F, const int64_t* dpre, int64_t E, int mode,
                     int32_t* flags, hipStream_t st);
int ip_level_emit(const IpSlot* slot, int64_t head, int64_t tail, int64_t F, const int64_t* dpre, int64_t E,
                  const int32_t* flags, const int32_t* fpos, int64_t T, hipStream_t st);

int place_isolated(const int64_t* rp, const int64_t* nw, int64_t n, const int64_t* B, int32_t k, int32_t* part,
                   int64_t* tmp_w, int64_t* tmp_pre, int64_t* ends, int32_t* last, void* scan_tmp, size_t scan_bytes,
                   hipStream_t st);

int validate_keys(const int64_t* rp, const int32_t* col, const int32_t* ew, int64_t n, int64_t m, int bits,
                  uint64_t* fk, uint64_t* rk, int32_t* fw, unsigned* bad, hipStream_t st);
int validate_cmp(const uint64_t* fk, const uint64_t* rk, const int32_t* fw, const int32_t* rw, int64_t m,
                 unsigned* bad, hipStream_t st);
int validate_nw(const void* nw, int bytes, int64_t n, unsigned* bad, hipStream_t st);

}  // namespace sclap
