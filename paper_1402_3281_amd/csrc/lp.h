// lp.h -- launchers of the label-propagation round kernels.
#pragma once

#include "common.h"

namespace sclap {

// Device layout of the hub rating path (degree > kBinBlock); see
// lp_kernels.hip.  Arrays marked "kept 0" are zero between rounds.
struct HubLayout {
  uint32_t* chunk_off;    // hubs + 1: first chunk of every hub
  uint32_t* part_off;     // hubs + 1: first label part of every hub
  int64_t* mat_off;       // hubs + 1: first entry of every hub's chunk x part matrix
  uint32_t* hub_P;        // hubs: label parts of every hub
  uint32_t* chunk_hub;    // map_cap: hub of every chunk
  uint32_t* part_hub;     // map_cap: hub of every part
  int64_t map_cap;
  uint32_t* totals;       // 2: chunks, parts
  uint32_t* totals_kept;  // 2: the same, kept between rounds (the layout is reused with the bins)
  int64_t parts_cap;      // the most label parts a layout may hold
  uint32_t* mat;          // mat_cap: per chunk, the first staged pair of each part (P + 1)
  int64_t mat_cap;
  int2* stage;            // stage_cap: (label, weight sum) pairs, kHubChunk per chunk, grouped by part
  int64_t stage_cap;
  int64_t* own;           // hubs: own-label connection (kept 0)
  unsigned long long* best;  // hubs: best foreign candidate key (kept 0)
  uint32_t* overflow;     // 1
};

// Bins the rated nodes; also lists them all in `rated` (rated_cnt) and sets
// every slot's CTR_VISITS.  T = total tiles (bin_tiles per slot, summed; the
// tiles of slot s start at S[s].tbase); scratch holds bin_scratch_bytes(T).
// binfo receives first entry | degree << 40 of every binned node except hubs.
// Stores the round's slot descriptors (host_slots, ns entries; pinned or
// pageable host memory, free for reuse on return) in S and zeroes zero[0,
// nzero) on stream st, in one launch when ns is small.
// Whether binning T tiles scans device-wide (rocPRIM) instead of in one workgroup.
bool bin_scan_device_wide(int64_t T);

int round_begin(const DevSlot* host_slots, int ns, DevSlot* S, uint32_t* zero, int64_t nzero, hipStream_t st);
int64_t bin_tiles(int64_t n);
size_t bin_scratch_bytes(int64_t T);
int launch_bin(const DevSlot* S, int ns, int64_t T, int32_t* bins, uint64_t* binfo, int64_t bin_cap,
               uint32_t* bin_cnt, unsigned long long* bin_visits, int32_t* rated, uint32_t* rated_cnt,
               void* scratch, size_t scratch_bytes, hipStream_t st);
// Rating launches: bins 0-4 (k_rate_small), 5-6 (k_rate_mid), 7 (k_rate_large),
// 8 (hub kernels, only if `hubs`).  evs (may be NULL): 5 events around them.
constexpr int kRateGroups = 5;
// Measurement group of the refinement marking kernels (k_mark, k_mark_big),
// after the rating groups in the profile arrays.
constexpr int kMarkGroup = kRateGroups;
// max_deg: no binned node has a larger degree (the launches of bins above
// it are left out).  *groups (may be NULL): bit g set when launch group g
// (the intervals between evs[g] and evs[g + 1]) ran a kernel.
int launch_rate(const DevSlot* S, int ns, const int32_t* bins, const uint64_t* binfo, int64_t bin_cap,
                const uint32_t* bin_cnt, const HubLayout& hub, int64_t n_hint, bool hubs, bool unit_weights,
                int64_t max_deg, int32_t lo5, int32_t lo7, bool hubs_ident, bool hub_layout_kept, hipStream_t st,
                hipEvent_t* evs, unsigned* groups);
// Small contended sets resolved on the device (admission, then the admitted
// weight added to each target's W); sets *big_flag if too large.
int launch_contended_small(const DevSlot* S, int ns, const uint64_t* keys, const uint32_t* ccnt, int node_bits,
                           uint32_t* big_flag, hipStream_t st);
// Incoming weight per target, the fast admission of targets that take all
// their movers (adm = 2; their arrivals go to W at once, and inc is cleared
// for all labels: Lt = the labels of all slots), contended keys for the rest.
int launch_incoming_decide(const DevSlot* S, int ns, int64_t N, int64_t Lt, const int32_t* rated,
                           const uint32_t* rcnt, uint64_t* ckeys, uint32_t* ccnt, int node_bits, hipStream_t st);
int launch_contended_split(const DevSlot* S, int ns, const uint64_t* keys, uint32_t cnt, int node_bits,
                           uint32_t* tkey, int64_t* wv, hipStream_t st);
int launch_contended_mark(const DevSlot* S, int ns, const uint64_t* keys, uint32_t cnt, int node_bits,
                          const int64_t* prefix, hipStream_t st);
// After launch_contended_mark: W(t) += the admitted weight of every target.
int launch_contended_add(const DevSlot* S, int ns, const uint64_t* keys, uint32_t cnt, int node_bits,
                         const int64_t* prefix, hipStream_t st);
// movers (N entries) and mcnt (zeroed) collect the moved nodes of refinement slots.
// skip (may be NULL): when *skip != 0 the launch does nothing.
// Refinement with block connections: build them for CONN_BUILD slots from
// this round's bins (after launch_rate, which laid out the hub chunks), and
// rate the rated nodes of CONN_RATE slots from them.
int launch_conn_build(const DevSlot* S, int ns, const int32_t* bins, const uint64_t* binfo, int64_t bin_cap,
                      const uint32_t* bin_cnt, const HubLayout& hub, int64_t n_hint, bool hubs, hipStream_t st);
// The hub chunk layout alone (what launch_conn_build needs from launch_rate
// when no binned node is rated by the bins).
int launch_hub_prep(const DevSlot* S, int ns, const int32_t* bins, int64_t bin_cap, const uint32_t* bin_cnt,
                    const HubLayout& hub, hipStream_t st);
// Rates the rated nodes of slots with block connections (CONN_RATE, and
// CONN_BUILD after launch_conn_build) from their rows.
int launch_rate_cached(const DevSlot* S, int ns, int64_t N, const int32_t* rated, const uint32_t* rcnt,
                       hipStream_t st);
// Applies admitted moves of the slots not admitted by tiles (run_apply); in
// refinement writes the old block of every admitted mover by rated position
// (mold, -1: stayed) and then marks the movers' neighbours (updating block
// connections) for every refinement slot.  big == NULL: no row has more than
// 4096 entries (no walk of long rows is launched); else big (big_cap entries)
// lists the movers with longer rows, counted by big_cnt from its front and,
// above 65536 entries, by huge_cnt from its back.
// mark_ev (may be NULL): two events recorded around the marking kernels;
// mark_entries (may be NULL): receives the number of mover entries walked.
int launch_apply(const DevSlot* S, int ns, int64_t N, const int32_t* rated, const uint32_t* rcnt, int32_t* mold,
                 int32_t* big, uint32_t* big_cnt, uint32_t* huge_cnt, int64_t big_cap, bool run_apply,
                 bool any_refine, const uint32_t* skip, hipStream_t st, hipEvent_t* mark_ev = nullptr,
                 unsigned long long* mark_entries = nullptr);
// Admission and application of the moves of refinement slots with at most
// kConnMaxK blocks, by binning tiles (roff: the rated-list offsets of the
// tiles from launch_bin's scratch, see bin_rated_offsets; kmax: the largest
// block count of those slots; scratch: tile_adm_bytes(T, kmax)).  Writes mold
// for their rated positions, updates W and the moved counters.
struct TileAdm {
  const uint32_t* roff;  // T + 1: rated-list offsets of the tiles (relative to roff[0])
  int64_t T;
  int kmax;              // rows of the matrices below
  int64_t* tsum;         // kmax x T: movers' weight per target block and tile
  int64_t* tpre;         // kmax x T: inclusive scan of tsum per (block, slot)
  int64_t* dW;           // kmax x T: per tile, the change of every block weight
  int64_t* tmoved;       // T: admitted movers per tile
  uint32_t* keys;        // kmax x T: scan segments (block x slot)
};
size_t tile_adm_bytes(int64_t T, int kmax);
// max_slot_tiles: the largest tile count of one slot (small ones are scanned
// by one workgroup per block and slot).
int launch_tile_admission(const DevSlot* S, int ns, const int32_t* rated, const uint32_t* roff, int64_t T, int kmax,
                          int64_t max_slot_tiles, void* scratch, size_t scratch_bytes, int32_t* mold,
                          hipStream_t st);
const uint32_t* bin_rated_offsets(void* scratch, int64_t T);

// Library primitives (rocPRIM) used as steps: sorts, scans, reductions.
//
// The radix sort sorts 1024 < n <= 2^20 keys by block sorts and merges, and
// its merge comparison masks bits [begin_bit, end_bit) with a shift by
// end_bit that is undefined at 64 (on the device the mask then covers the
// low 32 bits, and the merged keys come out unsorted).  Sorts over a range
// that starts above bit 0 must therefore end below bit 64: packed items
// (key << 32 | weight, sorted by bits [32, 32 + key bits)) take keys of at
// most kPackedKeyBits bits, and prim_sort_keys rejects such a range.
constexpr int kPackedKeyBits = 30;
size_t prim_sort_keys_bytes(size_t n);
// Sort by bits [begin_bit, end_bit) of the 64-bit keys (end_bit < 64 when
// begin_bit > 0).
int prim_sort_keys(void* tmp, size_t tmp_bytes, const uint64_t* in, uint64_t* out, size_t n, int end_bit,
                   hipStream_t st, int begin_bit = 0);
size_t prim_sort_pairs_bytes(size_t n);
// Stable by the keys' bits [begin_bit, end_bit) (end_bit < 64 when begin_bit > 0).
int prim_sort_pairs(void* tmp, size_t tmp_bytes, const uint64_t* kin, uint64_t* kout, const int32_t* vin,
                    int32_t* vout, size_t n, int end_bit, hipStream_t st, int begin_bit = 0);
size_t prim_scan_by_key_bytes(size_t n);
int prim_scan_by_key(void* tmp, size_t tmp_bytes, const uint32_t* keys, const int64_t* in, int64_t* out, size_t n,
                     hipStream_t st);
size_t prim_exscan_i32_bytes(size_t n);
int prim_exscan_i32(void* tmp, size_t tmp_bytes, const int32_t* in, int32_t* out, size_t n, hipStream_t st);
size_t prim_exscan_i64_bytes(size_t n);
int prim_exscan_i64(void* tmp, size_t tmp_bytes, const int64_t* in, int64_t* out, size_t n, hipStream_t st);
// Runs of equal keys (sorted input): the keys and their lengths (n < 2^32).
size_t prim_rle_bytes(size_t n);
int prim_rle(void* tmp, size_t tmp_bytes, const uint64_t* keys, uint64_t* ukeys, int64_t* counts, uint32_t* runs,
             size_t n, hipStream_t st);
// Sorted items key << 32 | weight (weight < 2^32): unique keys (as 64-bit
// values) and the sum of their weights.
size_t prim_reduce_packed_bytes(size_t n);
int prim_reduce_packed(void* tmp, size_t tmp_bytes, const uint64_t* items, uint64_t* ukeys, int64_t* sums,
                       uint32_t* count, size_t n, hipStream_t st);
size_t prim_reduce_by_key_bytes(size_t n);
int prim_reduce_by_key(void* tmp, size_t tmp_bytes, const uint64_t* keys, const int32_t* vals, uint64_t* ukeys,
                       int64_t* aggs, uint32_t* count, size_t n, hipStream_t st);

}  // namespace sclap
