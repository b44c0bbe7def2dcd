// lp.h -- launchers of the label-propagation round kernels.
#pragma once

#include "common.h"

namespace sclap {

struct RateHubScratch {
  uint32_t* chunk_off;  // bin capacity + 1
  uint32_t* slice_off;  // bin capacity + 1
  uint32_t* chunk_hub;  // map_cap: hub of each chunk
  uint32_t* slice_hub;  // map_cap: hub of each table slice
  uint32_t map_cap;
  unsigned long long* best;  // bin capacity, kept at 0 between rounds
  int64_t* tab_off;     // bin capacity
  uint32_t* totals;     // 2: chunks, slices
  int32_t* gkeys;       // tab_cap, kept at -1 between rounds
  int32_t* gvals;       // tab_cap, kept at 0 between rounds
  int64_t* own;         // bin capacity, kept at 0 between rounds
  uint32_t* overflow;   // 1
  int64_t tab_cap;
};

// Bins the rated nodes; also lists them all in `rated` (rated_cnt).
// binfo receives first entry | degree << 40 of every binned node except hubs.
int launch_bin(const DevSlot* S, int ns, int64_t N, int32_t* bins, uint64_t* binfo, int64_t bin_cap,
               uint32_t* bin_cnt, unsigned long long* bin_visits, int32_t* rated, uint32_t* rated_cnt,
               hipStream_t st);
// Rating launches: bins 0-4 (k_rate_small), 5-6 (k_rate_mid), 7 (k_rate_large),
// 8 (hub kernels, only if `hubs`).  evs (may be NULL): 5 events around them.
constexpr int kRateGroups = 5;
int launch_rate(const DevSlot* S, int ns, const int32_t* bins, const uint64_t* binfo, int64_t bin_cap,
                const uint32_t* bin_cnt, const RateHubScratch& hub, int64_t n_hint, bool hubs, bool unit_weights,
                hipStream_t st, hipEvent_t* evs);
// Small contended sets resolved on the device; sets *big_flag if too large.
int launch_contended_small(const DevSlot* S, int ns, const uint64_t* keys, const uint32_t* ccnt, int node_bits,
                           uint32_t* big_flag, hipStream_t st);
int launch_incoming_decide(const DevSlot* S, int ns, int64_t N, const int32_t* rated, const uint32_t* rcnt,
                           uint64_t* ckeys, uint32_t* ccnt, int node_bits, hipStream_t st);
int launch_contended_split(const DevSlot* S, int ns, const uint64_t* keys, uint32_t cnt, int node_bits,
                           uint32_t* tkey, int64_t* wv, hipStream_t st);
int launch_contended_mark(const DevSlot* S, int ns, const uint64_t* keys, uint32_t cnt, int node_bits,
                          const int64_t* prefix, hipStream_t st);
// movers (N entries) and mcnt (zeroed) collect the moved nodes of refinement slots.
// skip (may be NULL): when *skip != 0 the launch does nothing.
int launch_apply(const DevSlot* S, int ns, int64_t N, const int32_t* rated, const uint32_t* rcnt, int32_t* movers,
                 uint32_t* mcnt, int32_t* big, uint32_t* big_cnt, bool any_refine, const uint32_t* skip,
                 hipStream_t st);

// Library primitives (rocPRIM) used as steps: sorts, scans, reductions.
size_t prim_sort_keys_bytes(size_t n);
int prim_sort_keys(void* tmp, size_t tmp_bytes, const uint64_t* in, uint64_t* out, size_t n, int end_bit,
                   hipStream_t st);
size_t prim_sort_pairs_bytes(size_t n);
int prim_sort_pairs(void* tmp, size_t tmp_bytes, const uint64_t* kin, uint64_t* kout, const int32_t* vin,
                    int32_t* vout, size_t n, int end_bit, hipStream_t st);
size_t prim_scan_by_key_bytes(size_t n);
int prim_scan_by_key(void* tmp, size_t tmp_bytes, const uint32_t* keys, const int64_t* in, int64_t* out, size_t n,
                     hipStream_t st);
size_t prim_exscan_i32_bytes(size_t n);
int prim_exscan_i32(void* tmp, size_t tmp_bytes, const int32_t* in, int32_t* out, size_t n, hipStream_t st);
size_t prim_exscan_i64_bytes(size_t n);
int prim_exscan_i64(void* tmp, size_t tmp_bytes, const int64_t* in, int64_t* out, size_t n, hipStream_t st);
size_t prim_reduce_by_key_bytes(size_t n);
int prim_reduce_by_key(void* tmp, size_t tmp_bytes, const uint64_t* keys, const int32_t* vals, uint64_t* ukeys,
                       int64_t* aggs, uint32_t* count, size_t n, hipStream_t st);

}  // namespace sclap
