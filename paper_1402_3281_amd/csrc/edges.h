// edges.h -- edge-centric traversal shared by the graph-wide kernels.
#pragma once

#include "common.h"

namespace sclap {

// ---------------------------------------------------------------------------
// Edge-centric traversal: a workgroup takes kEpb consecutive stored entries;
// the rows they belong to are found by binary search over an LDS copy of
// the row offsets of that range, so neighbour ids are read coalesced.
// ---------------------------------------------------------------------------
constexpr int kItems = 8;
constexpr int kEpb = 256 * kItems;
constexpr int kRpLds = kEpb + 1;

// largest u in [lo, hi] with rp[u] <= e (the row holding entry e)
__device__ __forceinline__ int64_t row_search(const int64_t* __restrict__ rp, int64_t lo, int64_t hi, int64_t e) {
  while (lo < hi) {
    const int64_t mid = (lo + hi + 1) >> 1;
    if (rp[mid] <= e) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

struct EdgeRange {
  int64_t e0, e1, ulo, uhi;
  bool lds;
};

// Tile rows (built by tile_rows in misc_kernels.hip): trow[t] is the row
// holding entry t * kEpb (t < T, the number of tiles) and trow[T] = n - 1,
// so rows trow[t] .. trow[t + 1] hold every entry of tile t.
// All threads: set up the entry range [E0, E0 + kEpb) of this workgroup.
// With a tile-row table the range's rows are read from it; without one
// (callers that may not allocate it) thread 0 searches the row offsets.
__device__ __forceinline__ EdgeRange edge_range(const int64_t* __restrict__ rp, int64_t n, int64_t m, int64_t E0,
                                                int64_t* s_rp, int64_t* s_bounds,
                                                const int32_t* __restrict__ trow = nullptr) {
  __syncthreads();
  EdgeRange r;
  r.e0 = E0;
  if (trow) {
    const int64_t t = E0 / kEpb;
    r.e1 = E0 + kEpb < m ? E0 + kEpb : m;
    r.ulo = trow[t];
    r.uhi = trow[t + 1];
  } else {
    if (threadIdx.x == 0) {
      const int64_t E1 = E0 + kEpb < m ? E0 + kEpb : m;
      const int64_t ulo = row_search(rp, 0, n - 1, E0);
      const int64_t uhi = row_search(rp, ulo, n - 1, E1 - 1);
      s_bounds[0] = E1;
      s_bounds[1] = ulo;
      s_bounds[2] = uhi;
    }
    __syncthreads();
    r.e1 = s_bounds[0];
    r.ulo = s_bounds[1];
    r.uhi = s_bounds[2];
  }
  r.lds = r.uhi - r.ulo + 2 <= kRpLds;
  if (r.lds)
    for (int64_t i = threadIdx.x; i <= r.uhi - r.ulo + 1; i += blockDim.x) s_rp[i] = rp[r.ulo + i];
  __syncthreads();
  return r;
}

__device__ __forceinline__ int64_t edge_row(const int64_t* __restrict__ rp, const EdgeRange& r,
                                            const int64_t* s_rp, int64_t e) {
  if (r.lds) {
    int64_t lo = 0, hi = r.uhi - r.ulo;
    while (lo < hi) {
      const int64_t mid = (lo + hi + 1) >> 1;
      if (s_rp[mid] <= e) lo = mid;
      else hi = mid - 1;
    }
    return r.ulo + lo;
  }
  return row_search(rp, r.ulo, r.uhi, e);
}

}  // namespace sclap
