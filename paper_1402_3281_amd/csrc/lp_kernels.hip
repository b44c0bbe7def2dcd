// lp_kernels.hip -- one synchronous size-constrained label propagation round
// (Section 3.1) over a set of graphs ("slots"), as gfx950 kernels:
//
//   bin      nodes to rate -> seven degree bins, edge visits per slot
//   rate     per-node neighbour-cluster rating: conn(v, t) = sum of w(v, u)
//            over neighbours u with label t; candidates = own label and
//            neighbour labels in the allowed direction; eligible if
//            W(t) + c(v) <= cap; argmax with ties to the smallest label.
//   admit    movers into a target are admitted in increasing node id while
//            W(t) + inclusive prefix of their weights <= cap: targets whose
//            total incoming weight fits admit everyone; the others sort
//            their movers by (target, node) and scan.
//   apply    labels, label weights, moved counts, and in refinement the
//            rated set of the next round.
//
// Every result is a pure function of the previous round's state: integer
// atomics only ever sum or take maxima, so the order of execution does not
// change any value.  Sums that many threads add to the same address are
// first combined per workgroup in LDS.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <type_traits>

#include "common.h"
#include "lp.h"
#include "misc.h"

namespace sclap {

__device__ __forceinline__ uint32_t lane_id() { return __lane_id(); }

// Slot of global node u.  Kernels are instantiated for a single slot (ONE),
// where the descriptor address is uniform and its fields use scalar loads.
#define SLOT(u) (ONE ? 0 : slot_of(S, ns, (u)))

__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
  __builtin_amdgcn_wave_barrier();
}

// Graphs with fewer stored entries than this rate their nodes of degree <= 32
// in the 64-lane bin: the one-thread-per-node bins read a window of up to 32
// entries from the row start.
constexpr int64_t kThreadMinM = 32;

// Degree bin of a node: fixed bounds up to 32 and from 4097 on; between them
// the slot's bounds hi[0..3] (at most the kernels' capacities kBinHiCap,
// each at least the one before) split degrees 33..4096 into bins 3..7.
__device__ __forceinline__ int bin_of(int64_t d, int64_t m, const int32_t* hi) {
  if (m < kThreadMinM && d <= 64) return 3;
  return d <= 8 ? 0 : d <= 16 ? 1 : d <= 32 ? 2 : d <= hi[0] ? 3 : d <= hi[1] ? 4 : d <= hi[2] ? 5 : d <= hi[3] ? 6
       : d <= kBinBlock ? 7 : 8;
}

// ---------------------------------------------------------------------------
// Binning: every node of an active slot with degree > 0 (and, in refinement
// after round 1, in the rated set) goes to its degree bin and to the rated
// list (nodes rated from block connections go to the rated list only, and
// their edge visits are counted in its row).  The nodes of every slot are split into tiles of kBinTile; a tile
// belongs to one slot.  bin_count writes per tile and bin the node count and
// edge visits; an exclusive scan of those (bin-major) gives every tile its
// place in each bin, so no counter is shared between workgroups.
// ---------------------------------------------------------------------------
constexpr int kBinTile = 256;
constexpr int kBinRows = kBins + 1;  // the bins and the rated list

// Slot of tile t (tiles of slot s start at S[s].tbase).
__device__ __forceinline__ int slot_of_tile(const DevSlot* __restrict__ S, int ns, int64_t t) {
  int lo = 0, hi = ns - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (S[mid].tbase <= t) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

// Bin of the node at lane position; take = rated this round.
struct BinOf {
  bool take;
  int b;
  int64_t e0, d, v;
};

template <bool ONE>
__device__ __forceinline__ BinOf bin_node(const DevSlot& sl, int64_t v) {
  BinOf r{false, 0, 0, 0, v};
  if (v < sl.n && sl.round > 0 && (!sl.use_flags || gld(sl.flag_cur, v)) &&
      (!sl.cls || (int32_t)gld(sl.cls, v) == sl.sub)) {
    r.e0 = gld(sl.rp, v);
    r.d = gld(sl.rp, v + 1) - r.e0;
    r.take = r.d > 0;
    // rated from the block connections: the rated list only
    r.b = sl.conn_mode == CONN_RATE ? kBins : bin_of(r.d, sl.m, sl.bin_hi);
  }
  return r;
}

template <bool ONE>
__global__ void __launch_bounds__(kBinTile) k_bin_count(const DevSlot* __restrict__ S, int ns, int64_t T,
                                                        uint32_t* __restrict__ cnt, int64_t* __restrict__ vis) {
  __shared__ uint32_t s_c[4][kBinRows];
  __shared__ int64_t s_v[4][kBinRows];
  const int w = threadIdx.x / kWave;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    // the entry after the last tile: the scans' totals land there
    cnt[(int64_t)kBinRows * T] = 0;
    vis[(int64_t)kBinRows * T] = 0;
  }
  for (int64_t t = blockIdx.x; t < T; t += gridDim.x) {
    const int s = ONE ? 0 : slot_of_tile(S, ns, t);
    const DevSlot& sl = S[s];
    const int64_t v = (t - sl.tbase) * kBinTile + threadIdx.x;
    const BinOf r = bin_node<ONE>(sl, v);
    // the rated set of the next round is rebuilt from scratch
    if (v < sl.n && sl.round > 0 && sl.mode == MODE_REFINE) gst(sl.flag_next, v, (uint8_t)0);
#pragma unroll
    for (int j = 0; j < kBins; ++j) {
      const bool in = r.take && r.b == j;
      const uint64_t m = __ballot(in);
      // visits of the bin in this wave (only bins present; below the hub bin
      // the degrees are at most kBinBlock, so 32 bits hold the wave's sum)
      int64_t dv = 0;
      if (m) {
        if (j < kBins - 1) {
          uint32_t d32 = in ? (uint32_t)r.d : 0u;
          for (int off = 32; off > 0; off >>= 1) d32 += __shfl_xor(d32, off);
          dv = d32;
        } else {
          dv = in ? r.d : 0;
          for (int off = 32; off > 0; off >>= 1) dv += __shfl_xor(dv, off);
        }
      }
      if (lane_id() == 0) {
        s_c[w][j] = (uint32_t)__popcll(m);
        s_v[w][j] = dv;
      }
    }
    {
      const uint64_t m = __ballot(r.take);
      // visits of the nodes outside the bins (rated from block connections)
      const bool cn = r.take && r.b == kBins;
      int64_t dv = 0;
      if (__ballot(cn)) {
        dv = cn ? r.d : 0;
        for (int off = 32; off > 0; off >>= 1) dv += __shfl_xor(dv, off);
      }
      if (lane_id() == 0) {
        s_c[w][kBins] = (uint32_t)__popcll(m);
        s_v[w][kBins] = dv;
      }
    }
    __syncthreads();
    if (threadIdx.x < kBinRows) {
      const int j = threadIdx.x;
      cnt[(int64_t)j * T + t] = s_c[0][j] + s_c[1][j] + s_c[2][j] + s_c[3][j];
      vis[(int64_t)j * T + t] = s_v[0][j] + s_v[1][j] + s_v[2][j] + s_v[3][j];
    }
    __syncthreads();
  }
}

// off: exclusive scan of cnt (bin-major), off[kBinRows * T] = total.
template <bool ONE>
__global__ void __launch_bounds__(kBinTile) k_bin_write(const DevSlot* __restrict__ S, int ns, int64_t T,
                                                        const uint32_t* __restrict__ off,
                                                        int32_t* __restrict__ bins, uint64_t* __restrict__ binfo,
                                                        int64_t bin_cap, int32_t* __restrict__ rated) {
  __shared__ uint32_t s_c[4][kBinRows];
  const int w = threadIdx.x / kWave;
  const uint64_t lt = (1ull << lane_id()) - 1ull;
  for (int64_t t = blockIdx.x; t < T; t += gridDim.x) {
    const int s = ONE ? 0 : slot_of_tile(S, ns, t);
    const DevSlot& sl = S[s];
    const int64_t v = (t - sl.tbase) * kBinTile + threadIdx.x;
    const BinOf r = bin_node<ONE>(sl, v);
    uint32_t rank = 0, rrank = 0;
#pragma unroll
    for (int j = 0; j < kBins; ++j) {
      const bool in = r.take && r.b == j;
      const uint64_t m = __ballot(in);
      if (in) rank = (uint32_t)__popcll(m & lt);
      if (lane_id() == 0) s_c[w][j] = (uint32_t)__popcll(m);
    }
    {
      const uint64_t m = __ballot(r.take);
      rrank = (uint32_t)__popcll(m & lt);
      if (lane_id() == 0) s_c[w][kBins] = (uint32_t)__popcll(m);
    }
    __syncthreads();
    if (r.take) {
      uint32_t before = 0, rbefore = 0;
      for (int k = 0; k < w; ++k) {
        before += r.b < kBins ? s_c[k][r.b] : 0u;
        rbefore += s_c[k][kBins];
      }
      const int64_t u = sl.nbase + v;
      if (r.b < kBins) {
        const int64_t pos =
            (int64_t)r.b * bin_cap + (off[(int64_t)r.b * T + t] - off[(int64_t)r.b * T]) + before + rank;
        bins[pos] = (int32_t)u;
        if (r.b < kBins - 1) binfo[pos] = (uint64_t)r.e0 | ((uint64_t)r.d << 40);
      }
      rated[(off[(int64_t)kBins * T + t] - off[(int64_t)kBins * T]) + rbefore + rrank] = (int32_t)u;
    }
    __syncthreads();
  }
}

// Exclusive scans of cnt and vis (rows entries, the last one 0) in one
// workgroup of kScan1Threads threads, for small tile counts (one launch
// instead of the device-wide scans).
constexpr int kScan1Threads = 1024;
constexpr int64_t kScan1Rows = 64 * kScan1Threads;

bool bin_scan_device_wide(int64_t T) { return T > 0 && (int64_t)kBinRows * T + 1 > kScan1Rows; }

__device__ void bin_totals(const DevSlot* __restrict__ S, int ns, int64_t T, const uint32_t* __restrict__ off,
                           const int64_t* __restrict__ voff, uint32_t* __restrict__ bin_cnt,
                           unsigned long long* __restrict__ bin_visits, uint32_t* __restrict__ rated_cnt);

__global__ void __launch_bounds__(kScan1Threads) k_bin_scan1(const uint32_t* __restrict__ cnt,
                                                            const int64_t* __restrict__ vis, int64_t rows,
                                                            uint32_t* __restrict__ off, int64_t* __restrict__ voff,
                                                            const DevSlot* __restrict__ S, int ns, int64_t T,
                                                            uint32_t* __restrict__ bin_cnt,
                                                            unsigned long long* __restrict__ bin_visits,
                                                            uint32_t* __restrict__ rated_cnt) {
  __shared__ uint32_t sc[kScan1Threads / kWave];
  __shared__ int64_t sv[kScan1Threads / kWave];
  const int64_t per = (rows + kScan1Threads - 1) / kScan1Threads;
  const int64_t b = threadIdx.x * per, e = b + per < rows ? b + per : rows;
  uint32_t c = 0;
  int64_t v = 0;
  for (int64_t i = b; i < e; ++i) {
    c += cnt[i];
    v += vis[i];
  }
  // exclusive scan of the thread sums
  uint32_t ci = c;
  int64_t vi = v;
  for (int o = 1; o < kWave; o <<= 1) {
    const uint32_t c2 = __shfl_up(ci, o);
    const int64_t v2 = __shfl_up(vi, o);
    if ((int)lane_id() >= o) {
      ci += c2;
      vi += v2;
    }
  }
  const int w = threadIdx.x / kWave;
  if (lane_id() == kWave - 1) {
    sc[w] = ci;
    sv[w] = vi;
  }
  __syncthreads();
  uint32_t cb = 0;
  int64_t vb = 0;
  for (int q = 0; q < w; ++q) {
    cb += sc[q];
    vb += sv[q];
  }
  cb += ci - c;
  vb += vi - v;
  for (int64_t i = b; i < e; ++i) {
    off[i] = cb;
    voff[i] = vb;
    cb += cnt[i];
    vb += vis[i];
  }
  // then the totals (the scans are complete in this workgroup)
  __syncthreads();
  bin_totals(S, ns, T, off, voff, bin_cnt, bin_visits, rated_cnt);
}

// Totals: node count and visits per bin, rated count, edge visits per slot.
__device__ void bin_totals(const DevSlot* __restrict__ S, int ns, int64_t T, const uint32_t* __restrict__ off,
                           const int64_t* __restrict__ voff, uint32_t* __restrict__ bin_cnt,
                           unsigned long long* __restrict__ bin_visits, uint32_t* __restrict__ rated_cnt) {
  if (threadIdx.x < kBinRows) {
    const int j = threadIdx.x;
    const uint32_t c = off[(int64_t)(j + 1) * T] - off[(int64_t)j * T];
    if (j < kBins) {
      bin_cnt[j] = c;
      bin_visits[j] = (unsigned long long)(voff[(int64_t)(j + 1) * T] - voff[(int64_t)j * T]);
    } else {
      *rated_cnt = c;
    }
  }
  // per slot: the visits of its tiles over all bins
  for (int s = threadIdx.x; s < ns; s += blockDim.x) {
    const int64_t t0 = S[s].tbase, t1 = s + 1 < ns ? S[s + 1].tbase : T;
    int64_t sum = 0;
    for (int j = 0; j < kBinRows; ++j) sum += voff[(int64_t)j * T + t1] - voff[(int64_t)j * T + t0];
    gst(S[s].ctr, CTR_VISITS, sum);
  }
}

__global__ void __launch_bounds__(256) k_bin_totals(const DevSlot* __restrict__ S, int ns, int64_t T,
                                                    const uint32_t* __restrict__ off,
                                                    const int64_t* __restrict__ voff, uint32_t* __restrict__ bin_cnt,
                                                    unsigned long long* __restrict__ bin_visits,
                                                    uint32_t* __restrict__ rated_cnt) {
  bin_totals(S, ns, T, off, voff, bin_cnt, bin_visits, rated_cnt);
}

// ---------------------------------------------------------------------------
// Choice of a node from its aggregated candidates.
// ---------------------------------------------------------------------------
__device__ __forceinline__ bool own_allowed(const DevSlot& sl, int32_t own) {
  return !(sl.mode == MODE_REFINE && gld(sl.W, own) > sl.cap);
}

// Foreign candidate t with connection c: its key if it can win and is
// eligible (W(t) + c(v) <= cap), else 0.  A candidate that cannot beat the
// own label is not looked up (the own label is always in the set then).
__device__ __forceinline__ uint64_t cand_key(const DevSlot& sl, bool own_ok, int64_t conn_own, int32_t own,
                                             int64_t cv, int32_t t, int64_t c) {
  const bool beats = !own_ok || c > conn_own || (c == conn_own && t < own);
  if (beats && gld(sl.W, t) + cv <= sl.cap) return pack_key(c, t);
  return 0;
}

__device__ __forceinline__ bool dir_blocked(const DevSlot& sl, int32_t t, int32_t own) {
  return sl.dir_rule && ((sl.round & 1) ? t > own : t < own);
}

// Refinement slots with at most kConnMaxK blocks are admitted by tiles
// (k_ta_*), without global atomics on their few targets; the other slots go
// through k_incoming / k_decide / k_apply.
__device__ __forceinline__ bool tile_admission(const DevSlot& sl) {
  return sl.mode == MODE_REFINE && sl.nlabels <= kConnMaxK;
}

// Row of a binned node: first entry | degree << 40.
__device__ __forceinline__ int64_t info_e0(uint64_t x) { return (int64_t)(x & ((1ull << 40) - 1ull)); }
__device__ __forceinline__ int info_d(uint64_t x) { return (int)(x >> 40); }

// ---------------------------------------------------------------------------
// Rating, G lanes per node (degree <= G).  Each iteration handles two sets of
// nodes whose loads are issued together; the pairwise loop runs over the
// wave's largest degree only.
// ---------------------------------------------------------------------------
template <int G, bool ONE>
__device__ __forceinline__ void rate_group_body(const DevSlot* __restrict__ S, int ns, const int32_t* __restrict__ list,
                                                const uint64_t* __restrict__ info, uint32_t cnt, uint32_t bid,
                                                uint32_t nblk) {
  constexpr int R = 2;
  const int lane = (int)lane_id();
  const int gl = lane & (G - 1);
  const int gbase = lane & ~(G - 1);
  const uint32_t per_block = blockDim.x / G;
  for (uint32_t base = bid * per_block * R; base < cnt; base += nblk * per_block * R) {
    // Every load is issued from a clamped, always valid index and masked
    // afterwards, so the loads of all R node sets are in flight at once.
    bool valid[R];
    uint32_t ic[R];
    uint64_t x[R];
    int64_t u[R], e0[R], v[R], cv[R];
    int d[R];
    int32_t own[R], nb[R], w[R], t[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const uint32_t i = base + r * per_block + threadIdx.x / G;
      valid[r] = i < cnt;
      ic[r] = valid[r] ? i : cnt - 1;
    }
#pragma unroll
    for (int r = 0; r < R; ++r) u[r] = gld(list, ic[r]);
#pragma unroll
    for (int r = 0; r < R; ++r) x[r] = gld(info, ic[r]);
#pragma unroll
    for (int r = 0; r < R; ++r) {
      e0[r] = info_e0(x[r]);
      d[r] = info_d(x[r]);
    }
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const DevSlot& sl = S[SLOT(u[r])];
      v[r] = u[r] - sl.nbase;
      own[r] = gld(sl.lab, v[r]);
      cv[r] = gld(sl.nw, v[r]);
      const int64_t e = e0[r] + (gl < d[r] ? gl : d[r] - 1);
      nb[r] = gld(sl.col, e);
      w[r] = sl.ew ? gld(sl.ew, e) : 1;
    }
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const DevSlot& sl = S[SLOT(u[r])];
      const int32_t tl = sl.ident ? nb[r] : gld(sl.lab, nb[r]);
      t[r] = gl < d[r] ? tl : -1;
      w[r] = gl < d[r] ? w[r] : 0;
    }
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const DevSlot& sl = S[SLOT(u[r])];
      // largest degree in the wave (every degree here is at most G <= 64)
      const int dv = valid[r] ? d[r] : 0;
      int dm = 0;
#pragma unroll
      for (int b = 6; b >= 0; --b) {
        const int c = dm | (1 << b);
        if (__ballot(dv >= c)) dm = c;
      }
      const int dlim = dm < G ? dm : G;
      const bool foreign = t[r] >= 0 && t[r] != own[r];
      const uint64_t fmask = __ballot(foreign);
      const bool boundary = ((fmask >> gbase) & (G == 64 ? ~0ull : ((1ull << (G & 63)) - 1ull))) != 0;
      const int32_t te = (foreign && dir_blocked(sl, t[r], own[r])) ? -1 : t[r];
      int64_t conn = 0, conn_own = 0;
      bool leader = te >= 0;
      for (int j = 0; j < dlim; ++j) {
        int32_t tj, wj;
        if (G == 64) {
          tj = __builtin_amdgcn_readlane(te, j);
          wj = __builtin_amdgcn_readlane(w[r], j);
        } else {
          tj = __shfl(te, gbase + j);
          wj = __shfl(w[r], gbase + j);
        }
        if (tj == te) {
          conn += wj;
          if (j < gl) leader = false;
        }
        if (tj == own[r]) conn_own += wj;
      }
      uint64_t key = 0;
      bool own_ok = true;
      if (valid[r]) {
        own_ok = own_allowed(sl, own[r]);
        if (leader && te != own[r]) key = cand_key(sl, own_ok, conn_own, own[r], cv[r], te, conn);
      }
#pragma unroll
      for (int off = G / 2; off > 0; off >>= 1) {
        const uint64_t o = __shfl_xor(key, off);
        key = key > o ? key : o;
      }
      if (valid[r] && gl == 0) {
        if (own_ok) {
          const uint64_t ok = pack_key(conn_own, own[r]);
          key = key > ok ? key : ok;
        }
        gst(sl.desire, v[r], key ? key_label(key) : own[r]);
        if (sl.mode == MODE_REFINE && boundary) gst(sl.flag_next, v[r], (uint8_t)1);
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Rating, one thread per node (degree <= D): the node's neighbour labels are
// sorted in registers by a bitonic network, so that equal labels form runs
// whose weight sums are the connections; the best run that beats the own
// label and is eligible wins.  Nothing crosses lanes.
// ---------------------------------------------------------------------------
constexpr int32_t kNoLabel = 0x7FFFFFFF;  // sorts after every label
// Word 3 of a raw 32-bit buffer resource on gfx9-family GPUs (data format 32).
constexpr int kBufferConfig = 0x00020000;

template <int D, bool WEIGHTED>
__device__ __forceinline__ void sort_labels(int32_t (&t)[D], int32_t (&w)[D]) {
#pragma unroll
  for (int k = 2; k <= D; k <<= 1) {
#pragma unroll
    for (int j = k >> 1; j > 0; j >>= 1) {
#pragma unroll
      for (int i = 0; i < D; ++i) {
        const int l = i ^ j;
        if (l > i) {
          const bool up = (i & k) == 0;
          const int32_t a = t[i], b = t[l];
          if (WEIGHTED) {
            const bool sw = up ? a > b : a < b;
            const int32_t wa = w[i], wb = w[l];
            t[i] = sw ? b : a;
            t[l] = sw ? a : b;
            w[i] = sw ? wb : wa;
            w[l] = sw ? wa : wb;
          } else {
            t[i] = up ? min(a, b) : max(a, b);
            t[l] = up ? max(a, b) : min(a, b);
          }
        }
      }
    }
  }
}

// Largest candidate key below `limit` among the runs of the sorted labels
// that beat the own label (0 if none); branch-free over the unrolled runs.
template <int D, bool WEIGHTED>
__device__ __forceinline__ uint64_t best_run(const int32_t (&t)[D], const int32_t (&w)[D], bool own_ok,
                                             int64_t conn_own, int32_t own, uint64_t limit) {
  using Acc = typename std::conditional<WEIGHTED, int64_t, int32_t>::type;
  uint64_t best = 0;
  Acc acc = 0;
#pragma unroll
  for (int q = 0; q < D; ++q) {
    acc += WEIGHTED ? (Acc)w[q] : (Acc)1;
    const int32_t tq = t[q];
    const bool end = q == D - 1 || t[q + 1 < D ? q + 1 : q] != tq;
    const bool beats = !own_ok || (int64_t)acc > conn_own || ((int64_t)acc == conn_own && tq < own);
    const uint64_t k = pack_key((int64_t)acc, tq);
    const bool take = end && tq != kNoLabel && beats && k < limit && k > best;
    best = take ? k : best;
    acc = end ? (Acc)0 : acc;
  }
  return best;
}

template <int D, bool ONE, bool WEIGHTED>
__device__ __forceinline__ void rate_thread_body(const DevSlot* __restrict__ S, int ns,
                                                 const int32_t* __restrict__ list, const uint64_t* __restrict__ info,
                                                 uint32_t cnt, uint32_t bid, uint32_t nblk) {
  for (uint32_t base = bid * blockDim.x; base < cnt; base += nblk * blockDim.x) {
    const uint32_t i = base + threadIdx.x;
    const bool valid = i < cnt;
    const uint32_t ic = valid ? i : cnt - 1;
    const int64_t u = gld(list, ic);
    const uint64_t x = gld(info, ic);
    const int64_t e0 = info_e0(x);
    const int d = info_d(x);
    const DevSlot& sl = S[SLOT(u)];
    const int64_t v = u - sl.nbase;
    const int32_t own = gld(sl.lab, v);
    const int64_t cv = gld(sl.nw, v);
    // A window of D consecutive entries holding the row, so that every load
    // has the same base and a constant offset: it starts at the row unless
    // the row is among the last D entries of the graph (then it ends there;
    // graphs with fewer than kThreadMinM entries are binned elsewhere).
    int32_t t[D], w[D];
    const int64_t eb = e0 + D <= sl.m ? e0 : sl.m - D;
    const int sh = (int)(e0 - eb);
    {
      const int32_t* cb = sl.col + eb;
      const int32_t* wb = WEIGHTED && sl.ew ? sl.ew + eb : nullptr;
#pragma unroll
      for (int q = 0; q < D; ++q) {
        t[q] = gld(cb, q);
        w[q] = wb ? gld(wb, q) : 1;
      }
    }
    if (sl.ident) {
      // labels are node ids: the neighbour ids are the labels
    } else if (ONE && sl.n < ((int64_t)1 << 30)) {
      // one slot: the label gathers go through a buffer resource (scalar
      // base, 32-bit offsets, range-checked by the hardware)
      const __amdgpu_buffer_rsrc_t rs =
          __builtin_amdgcn_make_buffer_rsrc((void*)sl.lab, (short)0, (int)(sl.n * 4), kBufferConfig);
#pragma unroll
      for (int q = 0; q < D; ++q) t[q] = __builtin_amdgcn_raw_buffer_load_b32(rs, t[q] * 4, 0, 0);
    } else {
#pragma unroll
      for (int q = 0; q < D; ++q) t[q] = gld(sl.lab, t[q]);
    }
    // own connection, boundary flag, and the labels that may be chosen
    // (direction rule: odd rounds only smaller labels, even rounds larger)
    // as the interval [lo, hi] of labels that may be chosen
    const bool down = sl.dir_rule && (sl.round & 1), up = sl.dir_rule && !(sl.round & 1);
    const int32_t lo = up ? own + 1 : INT32_MIN, hi = down ? own - 1 : INT32_MAX;
    int64_t conn_own = 0;
    bool foreign = false;
#pragma unroll
    for (int q = 0; q < D; ++q) {
      const bool in = q >= sh && q < sh + d;
      const int32_t tq = t[q];
      const bool mine = in && tq == own;
      conn_own += mine ? (WEIGHTED ? (int64_t)w[q] : (int64_t)1) : (int64_t)0;
      const bool f = in && tq != own;
      foreign = foreign || f;
      t[q] = (f && tq >= lo && tq <= hi) ? tq : kNoLabel;
      if (WEIGHTED) w[q] = in ? w[q] : 0;
    }
    sort_labels<D, WEIGHTED>(t, w);
    const bool own_ok = own_allowed(sl, own);
    uint64_t limit = ~0ull, key = 0;
    for (;;) {
      const uint64_t k = best_run<D, WEIGHTED>(t, w, own_ok, conn_own, own, limit);
      if (!k) break;
      if (gld(sl.W, key_label(k)) + cv <= sl.cap) {
        key = k;
        break;
      }
      limit = k;  // ineligible: look for the next best run
    }
    if (valid) {
      if (own_ok) {
        const uint64_t ok = pack_key(conn_own, own);
        key = key > ok ? key : ok;
      }
      gst(sl.desire, v, key ? key_label(key) : own);
      if (sl.mode == MODE_REFINE && foreign) gst(sl.flag_next, v, (uint8_t)1);
    }
  }
}

// Degree <= D: one thread per node on unit-weight levels, D lanes per node
// (rate_group_body) on weighted ones.
template <int D, bool ONE>
__device__ __forceinline__ void rate_upto(const DevSlot* __restrict__ S, int ns, const int32_t* __restrict__ list,
                                          const uint64_t* __restrict__ info, uint32_t cnt, uint32_t bid,
                                          uint32_t nblk, int unit_weights) {
  if (unit_weights) rate_thread_body<D, ONE, false>(S, ns, list, info, cnt, bid, nblk);
  else rate_group_body<D, ONE>(S, ns, list, info, cnt, bid, nblk);
}

// Insert (t, w) into an open-addressing table (keys -1 = empty).  Tables
// are sized for twice the distinct keys they can receive, so the probe ends
// well before it has seen every slot; if it ever did, *err is set (the round
// fails) instead of probing forever.
__device__ __forceinline__ void table_add(int32_t* keys, int32_t* vals, uint32_t mask, int32_t t, int32_t w,
                                          uint32_t* err) {
  uint32_t h = hash32((uint32_t)t) & mask;
  for (uint32_t probes = 0; probes <= mask; ++probes) {
    const int32_t prev = atomicCAS(&keys[h], -1, t);
    if (prev == -1 || prev == t) {
      atomicAdd(&vals[h], w);
      return;
    }
    h = (h + 1) & mask;
  }
  atomicOr(err, 1u);
}

__device__ __forceinline__ uint32_t table_size(int64_t d, int64_t nlabels) {
  const int64_t distinct = d < nlabels ? d : nlabels;
  uint32_t tsz = 64;
  while (tsz < 2 * distinct) tsz <<= 1;
  return tsz;
}

// Loads of a binned node that its iteration needs first: the list entry and
// row (issued one node ahead), then the own label and weight and the first B
// entries of the row for this thread (issued while the node before is being
// finished), so that a node starts with its label gathers.
template <int B>
struct NodePre {
  int64_t u;
  uint64_t x;
  int32_t own;
  int64_t cv;
  int32_t nb[B], wt[B];
};

template <int B, bool ONE>
__device__ __forceinline__ void pre_row(NodePre<B>& p, const DevSlot* __restrict__ S, int ns, int first, int step) {
  const DevSlot& sl = S[SLOT(p.u)];
  const int64_t v = p.u - sl.nbase;
  const int64_t e0 = info_e0(p.x);
  const int d = info_d(p.x);
  p.own = gld(sl.lab, v);
  p.cv = gld(sl.nw, v);
#pragma unroll
  for (int q = 0; q < B; ++q) {
    const int ee = first + q * step;
    const int64_t ec = e0 + (ee < d ? ee : d - 1);
    p.nb[q] = gld(sl.col, ec);
    p.wt[q] = sl.ew ? gld(sl.ew, ec) : 1;
  }
}

// Aggregate the d entries of a row into the table: this thread takes entries
// first, first + step, ..., B at a time, the first B already loaded (nb, wt).
// The next B entries are loaded before the current ones are inserted.  Labels
// outside [lo, hi] (the direction rule) are not inserted; the own label's
// connection and whether a foreign label was seen are accumulated.  lab may
// be null: the labels are the node ids.
template <int B>
__device__ __forceinline__ void table_fill(const int32_t* __restrict__ col, const int32_t* __restrict__ ew,
                                           const int32_t* __restrict__ lab, int64_t row0, int first, int d, int step,
                                           int32_t own, int32_t lo, int32_t hi, int32_t* keys, int32_t* vals,
                                           uint32_t mask, int32_t (&nb)[B], int32_t (&wt)[B], int64_t& my_own,
                                           bool& foreign, uint32_t* err) {
  for (int base = 0; base < d; base += step * B) {
    int32_t tt[B], cw[B];
#pragma unroll
    for (int q = 0; q < B; ++q) {
      tt[q] = lab ? gld(lab, nb[q]) : nb[q];
      cw[q] = wt[q];
    }
    const int nbase = base + step * B;
    if (nbase < d) {
#pragma unroll
      for (int q = 0; q < B; ++q) {
        const int ee = nbase + first + q * step;
        const int64_t ec = row0 + (ee < d ? ee : d - 1);
        nb[q] = gld(col, ec);
        wt[q] = ew ? gld(ew, ec) : 1;
      }
    }
#pragma unroll
    for (int q = 0; q < B; ++q) {
      const int32_t tq = tt[q];
      if (base + first + q * step >= d) continue;
      if (tq == own) {
        my_own += cw[q];
        continue;
      }
      foreign = true;
      if (tq < lo || tq > hi) continue;
      table_add(keys, vals, mask, tq, cw[q], err);
    }
  }
}

// Labels that the direction rule lets a node with label own choose, as an
// interval: odd rounds only smaller labels, even rounds only larger ones.
__device__ __forceinline__ void dir_interval(const DevSlot& sl, int32_t own, int32_t& lo, int32_t& hi) {
  const bool down = sl.dir_rule && (sl.round & 1), up = sl.dir_rule && !(sl.round & 1);
  lo = up ? own + 1 : INT32_MIN;
  hi = down ? own - 1 : INT32_MAX;
}

// First clustering round of a level (labels = node ids, weights W(t) = c(t)):
// no row repeats a neighbour, so conn(v, u) = w(v, u) for each neighbour u,
// and no neighbour carries the own label (conn 0).  The best candidate is the
// direction-allowed eligible neighbour of largest weight, ties to the
// smallest id: a maximum of pack_key(w, u) over the row, with no table.  This
// thread takes entries first, first + step, ..., B at a time, the first B
// already loaded (nb, wt).  W(u) is read only when the slot's level does not
// make every candidate eligible.
template <int B>
__device__ __forceinline__ uint64_t ident_best(const DevSlot& sl, int64_t row0, int first, int d, int step,
                                               int32_t lo, int32_t hi, int64_t cv, int32_t (&nb)[B],
                                               int32_t (&wt)[B]) {
  uint64_t best = 0;
  for (int base = 0; base < d; base += step * B) {
    int32_t t[B], w[B];
    bool in[B];
    int64_t wu[B];
#pragma unroll
    for (int q = 0; q < B; ++q) {
      t[q] = nb[q];
      w[q] = wt[q];
      in[q] = base + first + q * step < d && t[q] >= lo && t[q] <= hi;
      wu[q] = (in[q] && !sl.all_elig) ? gld(sl.W, t[q]) : 0;
    }
    const int nbase = base + step * B;
    if (nbase < d) {
#pragma unroll
      for (int q = 0; q < B; ++q) {
        const int ee = nbase + first + q * step;
        const int64_t ec = row0 + (ee < d ? ee : d - 1);
        nb[q] = gld(sl.col, ec);
        wt[q] = sl.ew ? gld(sl.ew, ec) : 1;
      }
    }
#pragma unroll
    for (int q = 0; q < B; ++q) {
      const uint64_t k = (in[q] && (sl.all_elig || wu[q] + cv <= sl.cap)) ? pack_key(w[q], t[q]) : 0ull;
      best = best > k ? best : k;
    }
  }
  return best;
}

// Best eligible candidate among the table slots first, first + step, ...
// below tsz (keys -1 = empty).  C slots per thread are read at a time and
// their W lookups are issued together, so that a thread waits for one round
// of gathers per C slots rather than one per candidate.  A slot that cannot
// beat the own label reads W(own) instead (always a valid label).
template <int C>
__device__ __forceinline__ uint64_t scan_table(const DevSlot& sl, const int32_t* keys, const int32_t* vals,
                                               uint32_t tsz, uint32_t first, uint32_t step, bool own_ok,
                                               int64_t conn_own, int32_t own, int64_t cv) {
  uint64_t best = 0;
  for (uint32_t j0 = first; j0 < tsz; j0 += step * C) {
    int32_t t[C], c[C];
    int64_t wt[C];
    bool b[C];
#pragma unroll
    for (int q = 0; q < C; ++q) {
      const uint32_t j = j0 + (uint32_t)q * step;
      const uint32_t jc = j < tsz ? j : tsz - 1;
      t[q] = j < tsz ? keys[jc] : -1;
      c[q] = vals[jc];
    }
#pragma unroll
    for (int q = 0; q < C; ++q) {
      const int64_t cq = c[q];
      b[q] = t[q] >= 0 && (!own_ok || cq > conn_own || (cq == conn_own && t[q] < own));
      wt[q] = gld(sl.W, b[q] ? t[q] : own);
    }
#pragma unroll
    for (int q = 0; q < C; ++q) {
      const uint64_t k = (b[q] && wt[q] + cv <= sl.cap) ? pack_key(c[q], t[q]) : 0ull;
      best = best > k ? best : k;
    }
  }
  return best;
}

// ---------------------------------------------------------------------------
// Rating, one wave per node (degree <= TS / 2), wave-private LDS table.
// ---------------------------------------------------------------------------
template <int TS, bool ONE>
__device__ __forceinline__ void rate_wave_body(const DevSlot* __restrict__ S, int ns, const int32_t* __restrict__ list,
                                               const uint64_t* __restrict__ info, uint32_t cnt, uint32_t bid,
                                               uint32_t nblk, int32_t* lds) {
  constexpr int B = 4;
  const int w = threadIdx.x / kWave;
  int32_t* keys = lds + w * TS;
  int32_t* vals = lds + 4 * TS + w * TS;
  const int lane = (int)lane_id();
  const uint32_t stride = nblk * 4;
  uint32_t i = __builtin_amdgcn_readfirstlane(bid * 4 + w);
  if (i >= cnt) return;
  NodePre<B> p;
  p.u = gld(list, i);
  p.x = gld(info, i);
  pre_row<B, ONE>(p, S, ns, lane, kWave);
  for (; i < cnt; i += stride) {
    const bool has_next = i + stride < cnt;
    const uint32_t in = has_next ? i + stride : i;
    const int64_t un = gld(list, in);
    const uint64_t xn = gld(info, in);
    const int64_t u = p.u;
    const DevSlot& sl = S[SLOT(u)];
    const int64_t v = u - sl.nbase;
    const int64_t e0 = info_e0(p.x);
    const int d = info_d(p.x);
    const int32_t own = __builtin_amdgcn_readfirstlane(p.own);
    const int64_t cv = p.cv;
    int32_t lo, hi;
    dir_interval(sl, own, lo, hi);
    if (sl.ident) {
      // first clustering round: a maximum over the row, no table
      uint64_t best = ident_best<B>(sl, e0, lane, d, kWave, lo, hi, cv, p.nb, p.wt);
      p.u = un;
      p.x = xn;
      if (has_next) pre_row<B, ONE>(p, S, ns, lane, kWave);
      for (int off = 32; off > 0; off >>= 1) {
        const uint64_t o = __shfl_xor(best, off);
        best = best > o ? best : o;
      }
      if (lane == 0) gst(sl.desire, v, best ? key_label(best) : own);
      continue;
    }
    const uint32_t tsz = table_size(d, sl.nlabels);
    for (uint32_t j = lane; j < tsz; j += kWave) {
      keys[j] = -1;
      vals[j] = 0;
    }
    wave_sync();
    int64_t my_own = 0;
    bool foreign = false;
    table_fill<B>(sl.col, sl.ew, sl.lab, e0, lane, d, kWave, own, lo, hi, keys, vals, tsz - 1, p.nb, p.wt, my_own,
                  foreign, sl.err);
    for (int off = 32; off > 0; off >>= 1) my_own += __shfl_xor(my_own, off);
    const bool boundary = __ballot(foreign) != 0;
    wave_sync();
    const bool own_ok = own_allowed(sl, own);
    uint64_t best = scan_table<TS / kWave < 8 ? TS / kWave : 8>(sl, keys, vals, tsz, lane, kWave, own_ok, my_own,
                                                                 own, cv);
    p.u = un;
    p.x = xn;
    if (has_next) pre_row<B, ONE>(p, S, ns, lane, kWave);
    for (int off = 32; off > 0; off >>= 1) {
      const uint64_t o = __shfl_xor(best, off);
      best = best > o ? best : o;
    }
    if (lane == 0) {
      if (own_ok) {
        const uint64_t ok = pack_key(my_own, own);
        best = best > ok ? best : ok;
      }
      gst(sl.desire, v, best ? key_label(best) : own);
      if (sl.mode == MODE_REFINE && boundary) gst(sl.flag_next, v, (uint8_t)1);
    }
    wave_sync();
  }
}

// Block-wide reductions (up to 8 waves; sh has 8 entries).
template <class T, class Op>
__device__ __forceinline__ T block_reduce(T x, T* sh, Op op) {
  for (int off = 32; off > 0; off >>= 1) x = op(x, __shfl_xor(x, off));
  const int w = threadIdx.x / kWave;
  __syncthreads();
  if (lane_id() == 0) sh[w] = x;
  __syncthreads();
  T r = sh[0];
  for (int i = 1; i < (int)(blockDim.x / kWave); ++i) r = op(r, sh[i]);
  return r;
}

struct OpMax64 {
  __device__ uint64_t operator()(uint64_t a, uint64_t b) const { return a > b ? a : b; }
};
struct OpAdd64 {
  __device__ int64_t operator()(int64_t a, int64_t b) const { return a + b; }
};
struct OpOr {
  __device__ int operator()(int a, int b) const { return a | b; }
};

// ---------------------------------------------------------------------------
// Rating, one workgroup per node (degree <= TS / 2), LDS hash table.
// ---------------------------------------------------------------------------
// LDS scratch of its block reductions (up to 8 waves); the caller places it,
// so that a kernel whose table array has room to spare adds no LDS for it.
struct BlockRed {
  uint64_t best[8];
  int64_t conn[8];
  int flag[8];
};

template <int TS, int NT, bool ONE>
__device__ __forceinline__ void rate_block_body(const DevSlot* __restrict__ S, int ns, const int32_t* __restrict__ list,
                                                const uint64_t* __restrict__ info, uint32_t cnt, uint32_t bid,
                                                uint32_t nblk, int32_t* lds, BlockRed* red) {
  constexpr int B = 4;
  int32_t* keys = lds;
  int32_t* vals = lds + TS;
  uint32_t i = bid;
  if (i >= cnt) return;
  NodePre<B> p;
  p.u = gld(list, i);
  p.x = gld(info, i);
  pre_row<B, ONE>(p, S, ns, threadIdx.x, NT);
  for (; i < cnt; i += nblk) {
    const bool has_next = i + nblk < cnt;
    const uint32_t in = has_next ? i + nblk : i;
    const int64_t un = gld(list, in);
    const uint64_t xn = gld(info, in);
    const int64_t u = p.u;
    const DevSlot& sl = S[SLOT(u)];
    const int64_t v = u - sl.nbase;
    const int64_t e0 = info_e0(p.x);
    const int d = info_d(p.x);
    const int32_t own = __builtin_amdgcn_readfirstlane(p.own);
    const int64_t cv = p.cv;
    int32_t lo, hi;
    dir_interval(sl, own, lo, hi);
    if (sl.ident) {
      // first clustering round: a maximum over the row, no table
      uint64_t best = ident_best<B>(sl, e0, threadIdx.x, d, NT, lo, hi, cv, p.nb, p.wt);
      p.u = un;
      p.x = xn;
      if (has_next) pre_row<B, ONE>(p, S, ns, threadIdx.x, NT);
      best = block_reduce(best, red->best, OpMax64());
      if (threadIdx.x == 0) gst(sl.desire, v, best ? key_label(best) : own);
      __syncthreads();
      continue;
    }
    const uint32_t tsz = table_size(d, sl.nlabels);
    const uint32_t mask = tsz - 1;
    for (uint32_t j = threadIdx.x; j < tsz; j += NT) {
      keys[j] = -1;
      vals[j] = 0;
    }
    __syncthreads();
    int64_t my_own = 0;
    bool foreign = false;
    table_fill<B>(sl.col, sl.ew, sl.lab, e0, threadIdx.x, d, NT, own, lo, hi, keys, vals, mask, p.nb, p.wt, my_own,
                  foreign, sl.err);
    const int64_t conn_own = block_reduce(my_own, red->conn, OpAdd64());
    const int boundary = block_reduce(foreign ? 1 : 0, red->flag, OpOr());
    const bool own_ok = own_allowed(sl, own);
    uint64_t best = scan_table<8>(sl, keys, vals, tsz, threadIdx.x, NT, own_ok, conn_own, own, cv);
    p.u = un;
    p.x = xn;
    if (has_next) pre_row<B, ONE>(p, S, ns, threadIdx.x, NT);
    best = block_reduce(best, red->best, OpMax64());
    if (threadIdx.x == 0) {
      if (own_ok) {
        const uint64_t ok = pack_key(conn_own, own);
        best = best > ok ? best : ok;
      }
      gst(sl.desire, v, best ? key_label(best) : own);
      if (sl.mode == MODE_REFINE && boundary) gst(sl.flag_next, v, (uint8_t)1);
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// Fused launches: blocks [b * nblk, (b + 1) * nblk) serve bin `first + b`.
// ---------------------------------------------------------------------------
template <bool ONE>
__global__ void __launch_bounds__(256) k_rate_tiny(const DevSlot* __restrict__ S, int ns,
                                                   const int32_t* __restrict__ bins,
                                                   const uint64_t* __restrict__ binfo, int64_t bin_cap,
                                                   const uint32_t* __restrict__ bin_cnt, uint32_t nblk,
                                                   int unit_weights) {
  const uint32_t b = blockIdx.x / nblk, bid = blockIdx.x % nblk;
  const int32_t* list = bins + b * bin_cap;
  const uint64_t* info = binfo + b * bin_cap;
  const uint32_t cnt = bin_cnt[b];
  if (b == 0) rate_upto<8, ONE>(S, ns, list, info, cnt, bid, nblk, unit_weights);
  else rate_upto<16, ONE>(S, ns, list, info, cnt, bid, nblk, unit_weights);
}

template <bool ONE>
__global__ void __launch_bounds__(256) k_rate_b32(const DevSlot* __restrict__ S, int ns,
                                                  const int32_t* __restrict__ list,
                                                  const uint64_t* __restrict__ info,
                                                  const uint32_t* __restrict__ cnt_ptr, int unit_weights) {
  rate_upto<32, ONE>(S, ns, list, info, *cnt_ptr, blockIdx.x, gridDim.x, unit_weights);
}

template <bool ONE>
__global__ void __launch_bounds__(256) k_rate_small(const DevSlot* __restrict__ S, int ns,
                                                    const int32_t* __restrict__ bins,
                                                    const uint64_t* __restrict__ binfo, int64_t bin_cap,
                                                    const uint32_t* __restrict__ bin_cnt, uint32_t nblk) {
  __shared__ int32_t lds[8 * 256];
  const uint32_t b = 3 + blockIdx.x / nblk, bid = blockIdx.x % nblk;
  const int32_t* list = bins + b * bin_cap;
  const uint64_t* info = binfo + b * bin_cap;
  const uint32_t cnt = bin_cnt[b];
  if (b == 3) rate_wave_body<128, ONE>(S, ns, list, info, cnt, bid, nblk, lds);
  else rate_wave_body<256, ONE>(S, ns, list, info, cnt, bid, nblk, lds);
}

template <bool ONE>
__global__ void __launch_bounds__(256) k_rate_mid(const DevSlot* __restrict__ S, int ns,
                                                  const int32_t* __restrict__ bins,
                                                  const uint64_t* __restrict__ binfo, int64_t bin_cap,
                                                  const uint32_t* __restrict__ bin_cnt, uint32_t nblk) {
  // bin 5: four wave tables of 2 x 1024; bin 6: one table of 2 x 4096 and
  // the reduction scratch after it (32.9 KB in all: four workgroups per CU)
  __shared__ __align__(16) int32_t lds[8 * 1024 + sizeof(BlockRed) / sizeof(int32_t)];
  const uint32_t b = 5 + blockIdx.x / nblk, bid = blockIdx.x % nblk;
  const int32_t* list = bins + b * bin_cap;
  const uint64_t* info = binfo + b * bin_cap;
  const uint32_t cnt = bin_cnt[b];
  if (b == 5) rate_wave_body<1024, ONE>(S, ns, list, info, cnt, bid, nblk, lds);
  else rate_block_body<4096, 256, ONE>(S, ns, list, info, cnt, bid, nblk, lds,
                                        reinterpret_cast<BlockRed*>(lds + 2 * 4096));
}

template <bool ONE>
__global__ void __launch_bounds__(512) k_rate_large(const DevSlot* __restrict__ S, int ns,
                                                    const int32_t* __restrict__ list,
                                                    const uint64_t* __restrict__ info,
                                                    const uint32_t* __restrict__ cnt_ptr) {
  __shared__ int32_t lds[2 * 8192];
  __shared__ BlockRed red;
  rate_block_body<8192, 512, ONE>(S, ns, list, info, *cnt_ptr, blockIdx.x, gridDim.x, lds, &red);
}

// ---------------------------------------------------------------------------
// Rating of hubs (degree > kBinBlock), without global hash tables:
//   prep     per hub: chunks of kHubChunk entries, label parts (a power of
//            two, about kHubPartLabels distinct labels each), offsets
//   chunk    per chunk: labels aggregated in an LDS table; the chunk's
//            (label, sum) pairs are staged grouped by part, each part's
//            first pair noted in the hub's chunk x part matrix
//   part     per part: the part's pairs, counted from the matrix and read
//            from every chunk of its hub, aggregated in LDS; the best
//            eligible label of the part,
//            combined per hub with an integer maximum
//   final    per hub: the own label against the best foreign one.
// Every label of a hub falls in exactly one part, so the per-part sums are
// the node's connections.
// ---------------------------------------------------------------------------
constexpr int kHubTable = 2 * kHubChunk;   // LDS table entries of a chunk
constexpr int kHubPartTable = 4096;        // LDS table entries of a label part
constexpr int kHubPartFill = kHubPartTable - kHubPartTable / 8;  // distinct labels one part may hold

// Part of label t among P parts (bits independent of the LDS table slot).
__device__ __forceinline__ uint32_t hub_part_of(int32_t t, uint32_t P) {
  return (hash32((uint32_t)t) >> 19) & (P - 1);
}

// One workgroup: per hub chunk, part and matrix offsets (exclusive scans).
template <bool ONE>
__global__ void __launch_bounds__(1024) k_hub_prep(const DevSlot* __restrict__ S, int ns,
                                                   const int32_t* __restrict__ list,
                                                   const uint32_t* __restrict__ cnt_ptr, HubLayout L) {
  constexpr int NW = 1024 / kWave;
  __shared__ uint32_t wc[NW], wp[NW];
  __shared__ int64_t wm[NW];
  __shared__ uint32_t carry_c, carry_p;
  __shared__ int64_t carry_m;
  const uint32_t cnt = *cnt_ptr;
  const uint32_t lane = lane_id(), w = threadIdx.x / kWave;
  if (threadIdx.x == 0) {
    carry_c = 0;
    carry_p = 0;
    carry_m = 0;
  }
  __syncthreads();
  for (uint32_t base = 0; base < cnt; base += blockDim.x) {
    const uint32_t i = base + threadIdx.x;
    uint32_t nc = 0, np = 0;
    int64_t nm = 0;
    if (i < cnt) {
      const int64_t u = list[i];
      const DevSlot& sl = S[SLOT(u)];
      const int64_t v = u - sl.nbase;
      const int64_t d = gld(sl.rp, v + 1) - gld(sl.rp, v);
      nc = (uint32_t)((d + kHubChunk - 1) / kHubChunk);
      np = hub_parts(d, sl.nlabels);
      nm = (int64_t)nc * (np + 1);
      L.hub_P[i] = np;
    }
    // inclusive scans within the wave, then over the waves' totals
    uint32_t ic = nc, ip = np;
    int64_t im = nm;
    for (int off = 1; off < kWave; off <<= 1) {
      const uint32_t oc = __shfl_up(ic, off), op = __shfl_up(ip, off);
      const uint32_t mlo = __shfl_up((uint32_t)im, off), mhi = __shfl_up((uint32_t)((uint64_t)im >> 32), off);
      if ((int)lane >= off) {
        ic += oc;
        ip += op;
        im += (int64_t)(((uint64_t)mhi << 32) | mlo);
      }
    }
    if (lane == kWave - 1) {
      wc[w] = ic;
      wp[w] = ip;
      wm[w] = im;
    }
    __syncthreads();
    uint32_t c0 = carry_c + ic - nc, p0 = carry_p + ip - np;
    int64_t m0 = carry_m + im - nm;
    for (uint32_t q = 0; q < w; ++q) {
      c0 += wc[q];
      p0 += wp[q];
      m0 += wm[q];
    }
    if (i < cnt) {
      L.chunk_off[i] = c0;
      L.part_off[i] = p0;
      L.mat_off[i] = m0;
      if ((int64_t)c0 + nc <= L.map_cap && (int64_t)p0 + np <= L.map_cap) {
        for (uint32_t c = 0; c < nc; ++c) L.chunk_hub[c0 + c] = i;
        for (uint32_t p = 0; p < np; ++p) L.part_hub[p0 + p] = i;
      } else {
        *L.overflow = 1;
      }
    }
    __syncthreads();
    if (threadIdx.x == blockDim.x - 1) {
      // the last thread's exclusive offsets plus its own sizes: every hub so far
      carry_c = c0 + nc;
      carry_p = p0 + np;
      carry_m = m0 + nm;
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    L.totals[0] = carry_c;
    L.totals[1] = carry_p;
    L.totals_kept[0] = carry_c;
    L.totals_kept[1] = carry_p;
    if ((int64_t)carry_c * kHubChunk > L.stage_cap || carry_m > L.mat_cap || carry_p > L.parts_cap)
      *L.overflow = 1;
  }
}

// A clustering round whose bins are the previous round's keeps that round's
// hub layout (it depends on the hubs, their degrees and the label count
// only); the round's counters were zeroed, so the totals are restored.
__global__ void k_hub_reuse(HubLayout L) {
  L.totals[0] = L.totals_kept[0];
  L.totals[1] = L.totals_kept[1];
}

constexpr int kHubChunkThreads = 512;

template <bool ONE>
__global__ void __launch_bounds__(kHubChunkThreads) k_hub_chunk(const DevSlot* __restrict__ S, int ns,
                                                                const int32_t* __restrict__ list, HubLayout L) {
  constexpr int NT = kHubChunkThreads;
  __shared__ int32_t keys[kHubTable];
  __shared__ int32_t vals[kHubTable];
  __shared__ uint32_t ulist[kHubChunk];  // used table slots (low 16 bits) | rank in their part << 16
  // pairs per part, then (scanned in place) the part's first staged pair; one
  // array for both keeps the workgroup within a third of the CU's LDS
  __shared__ uint32_t loff[kHubMaxParts + 1];
  __shared__ int64_t redi[8];
  __shared__ int redo[8];
  __shared__ uint32_t s_wsum[8];
  __shared__ uint32_t s_used;
  if (*L.overflow) return;
  const uint32_t nchunks = L.totals[0];
  // the table is cleared once here, and after every chunk only where it was used
  for (int j = threadIdx.x; j < kHubTable; j += NT) {
    keys[j] = -1;
    vals[j] = 0;
  }
  for (uint32_t c = blockIdx.x; c < nchunks; c += gridDim.x) {
    const uint32_t i = L.chunk_hub[c];
    const uint32_t lc = c - L.chunk_off[i];
    const uint32_t P = L.hub_P[i];
    const int64_t u = list[i];
    const DevSlot& sl = S[SLOT(u)];
    const int64_t v = u - sl.nbase;
    const int64_t row0 = gld(sl.rp, v);
    const int64_t d = gld(sl.rp, v + 1) - row0;
    const int64_t e_begin = (int64_t)lc * kHubChunk;
    const int64_t e_end = e_begin + kHubChunk < d ? e_begin + kHubChunk : d;
    const int32_t own = gld(sl.lab, v);
    if (sl.ident) {
      // first clustering round: the chunk's best neighbour (a maximum, see
      // ident_best) goes straight to the hub's best; nothing is staged
      int32_t lo, hi;
      dir_interval(sl, own, lo, hi);
      const int64_t cv = gld(sl.nw, v);
      uint64_t best = 0;
      for (int64_t e = e_begin + threadIdx.x; e < e_end; e += NT) {
        const int32_t t = gld(sl.col, row0 + e);
        const int32_t w = sl.ew ? gld(sl.ew, row0 + e) : 1;
        if (t < lo || t > hi) continue;
        if (!sl.all_elig && gld(sl.W, t) + cv > sl.cap) continue;
        const uint64_t k = pack_key(w, t);
        best = best > k ? best : k;
      }
      best = block_reduce(best, reinterpret_cast<uint64_t*>(redi), OpMax64());
      uint32_t* mat_loff = L.mat + L.mat_off[i] + (int64_t)lc * (P + 1);
      for (uint32_t p = threadIdx.x; p <= P; p += NT) mat_loff[p] = 0u;
      if (threadIdx.x == 0 && best) atomicMax(&L.best[i], (unsigned long long)best);
      __syncthreads();
      continue;
    }
    for (uint32_t p = threadIdx.x; p < P; p += NT) loff[p] = 0;
    if (threadIdx.x == 0) s_used = 0;
    __syncthreads();
    // aggregate the chunk's entries by label, listing every slot taken
    int64_t my_own = 0;
    bool foreign = false;
    // a chunk is one pass: QC entries per thread, their loads in flight together
    constexpr int QC = kHubChunk / NT;
    for (int64_t e = e_begin + threadIdx.x; e < e_end; e += (int64_t)NT * QC) {
      int32_t nb[QC], wt[QC], tt[QC];
      bool ok[QC];
#pragma unroll
      for (int q = 0; q < QC; ++q) {
        const int64_t ee = e + (int64_t)q * NT;
        ok[q] = ee < e_end;
        const int64_t ec = row0 + (ok[q] ? ee : e_end - 1);
        nb[q] = gld(sl.col, ec);
        wt[q] = sl.ew ? gld(sl.ew, ec) : 1;
      }
#pragma unroll
      for (int q = 0; q < QC; ++q) tt[q] = gld(sl.lab, nb[q]);
#pragma unroll
      for (int q = 0; q < QC; ++q) {
        const int32_t tq = tt[q];
        if (!ok[q]) continue;
        if (tq == own) {
          my_own += wt[q];
          continue;
        }
        foreign = true;
        if (dir_blocked(sl, tq, own)) continue;
        // at most kHubChunk distinct labels in a table of 2 x kHubChunk slots
        uint32_t h = hash32((uint32_t)tq) & (kHubTable - 1);
        for (uint32_t probes = 0;; ++probes) {
          if (probes == (uint32_t)kHubTable) {
            *L.overflow = 1;
            break;
          }
          const int32_t prev = atomicCAS(&keys[h], -1, tq);
          if (prev == -1 || prev == tq) {
            if (prev == -1) ulist[atomicAdd(&s_used, 1u)] = h;
            atomicAdd(&vals[h], wt[q]);
            break;
          }
          h = (h + 1) & (kHubTable - 1);
        }
      }
    }
    const int64_t co = block_reduce(my_own, redi, OpAdd64());
    const int boundary = block_reduce(foreign ? 1 : 0, redo, OpOr());
    if (threadIdx.x == 0) {
      if (co) atomicAdd((unsigned long long*)&L.own[i], (unsigned long long)co);
      if (sl.mode == MODE_REFINE && boundary) gst(sl.flag_next, v, (uint8_t)1);
    }
    const uint32_t nu = s_used;
    // label part of every pair and its rank within the part
    for (uint32_t k = threadIdx.x; k < nu; k += NT) {
      const uint32_t h = ulist[k];
      const uint32_t r = atomicAdd(&loff[hub_part_of(keys[h], P)], 1u);
      ulist[k] = h | (r << 16);
    }
    __syncthreads();
    {
      // exclusive scan of the counts loff[0..P) in place, total in loff[P]
      // (every thread reads and writes only its own PT entries)
      constexpr int PT = kHubMaxParts / NT;
      uint32_t mine[PT], tot = 0;
#pragma unroll
      for (int q = 0; q < PT; ++q) {
        const uint32_t p = threadIdx.x * PT + q;
        mine[q] = p < P ? loff[p] : 0u;
        tot += mine[q];
      }
      uint32_t incl = tot;
      for (int off = 1; off < kWave; off <<= 1) {
        const uint32_t o = __shfl_up(incl, off);
        if ((int)lane_id() >= off) incl += o;
      }
      if (lane_id() == kWave - 1) s_wsum[threadIdx.x / kWave] = incl;
      __syncthreads();
      uint32_t run = incl - tot;
      for (int k = 0; k < (int)(threadIdx.x / kWave); ++k) run += s_wsum[k];
#pragma unroll
      for (int q = 0; q < PT; ++q) {
        const uint32_t p = threadIdx.x * PT + q;
        if (p < P) loff[p] = run;
        run += mine[q];
      }
      // the total: the last thread's running sum covers every part, also
      // when P = kHubMaxParts (its index is past the threads' entries)
      if (threadIdx.x == NT - 1) loff[P] = run;
    }
    __syncthreads();
    // chunk x part matrix: the part offsets of the staged pairs (a part's
    // pairs in this chunk are the difference of two of them)
    uint32_t* mat_loff = L.mat + L.mat_off[i] + (int64_t)lc * (P + 1);
    for (uint32_t p = threadIdx.x; p <= P; p += NT) mat_loff[p] = loff[p];
    // staged pairs grouped by part; the used slots are cleared
    int2* stage = L.stage + (int64_t)c * kHubChunk;
    for (uint32_t k = threadIdx.x; k < nu; k += NT) {
      const uint32_t x = ulist[k];
      const uint32_t h = x & 0xFFFFu;
      const int32_t t = keys[h];
      stage[loff[hub_part_of(t, P)] + (x >> 16)] = make_int2(t, vals[h]);
      keys[h] = -1;
      vals[h] = 0;
    }
    __syncthreads();
  }
}

// Best eligible label of every part.  The part's pairs are read where its
// hub's chunks staged them, and counted from the hub's chunk x part matrix: for hubs of up
// to kHubFlat chunks, the workgroup's threads stride over the part's pairs
// of all chunks in a row (each finds its chunk by binary search over the
// prefix of the chunks' pair counts in LDS); larger hubs take a thread per
// chunk.  A part whose distinct labels would overfill the LDS table is taken
// in Q passes, each over the labels of one residue of a further hash (Q
// doubles until the passes fit), so any label distribution is handled
// exactly.
constexpr uint32_t kHubMaxPasses = 64;
constexpr uint32_t kHubFlat = 512;

template <bool ONE>
__global__ void __launch_bounds__(256) k_hub_part(const DevSlot* __restrict__ S, int ns,
                                                  const int32_t* __restrict__ list, HubLayout L) {
  __shared__ int32_t keys[kHubPartTable];
  __shared__ int32_t vals[kHubPartTable];
  __shared__ uint32_t s_used;
  __shared__ uint64_t red64[8];
  __shared__ uint32_t s_beg[kHubFlat];      // first pair of the part in each chunk's stage
  __shared__ uint32_t s_pre[kHubFlat + 1];  // exclusive prefix of the chunks' pair counts
  __shared__ uint32_t s_wsum[4];
  __shared__ int64_t s_red[4];
  constexpr uint32_t NT = 256;
  if (*L.overflow) return;
  const uint32_t nparts = L.totals[1];
  const uint32_t lane = lane_id(), wave = threadIdx.x / kWave;
  for (uint32_t g = blockIdx.x; g < nparts; g += gridDim.x) {
    const uint32_t i = L.part_hub[g];
    const int64_t u = list[i];
    const DevSlot& sl = S[SLOT(u)];
    const int64_t v = u - sl.nbase;
    const int32_t own = gld(sl.lab, v);
    const int64_t cv = gld(sl.nw, v);
    const int64_t conn_own = L.own[i];
    const bool own_ok = own_allowed(sl, own);
    const uint32_t P = L.hub_P[i];
    const uint32_t pp = g - L.part_off[i];
    const int64_t d = gld(sl.rp, v + 1) - gld(sl.rp, v);
    const uint32_t nc = (uint32_t)((d + kHubChunk - 1) / kHubChunk);
    const uint32_t* mat = L.mat + L.mat_off[i];
    const int2* stage0 = L.stage + (int64_t)L.chunk_off[i] * kHubChunk;
    const bool flat = nc <= kHubFlat;
    if (flat) {
      // two chunks per thread: their pair counts, scanned across the workgroup
      uint32_t c2[2], tot = 0;
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        const uint32_t lc = 2 * threadIdx.x + q;
        c2[q] = 0;
        if (lc < nc) {
          const uint32_t* ml = mat + (int64_t)lc * (P + 1);
          const uint32_t b0 = ml[pp];
          s_beg[lc] = b0;
          c2[q] = ml[pp + 1] - b0;
        }
        tot += c2[q];
      }
      uint32_t incl = tot;
      for (int off = 1; off < kWave; off <<= 1) {
        const uint32_t o = __shfl_up(incl, off);
        if ((int)lane >= off) incl += o;
      }
      if (lane == kWave - 1) s_wsum[wave] = incl;
      __syncthreads();
      uint32_t run = incl - tot;
      for (uint32_t k = 0; k < wave; ++k) run += s_wsum[k];
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        const uint32_t lc = 2 * threadIdx.x + q;
        if (lc < nc) s_pre[lc] = run;
        run += c2[q];
      }
      if (threadIdx.x == NT - 1) s_pre[nc] = run;
      __syncthreads();
    }
    // the part's pairs over all chunks of its hub
    uint32_t len;
    if (flat) {
      len = s_pre[nc];
    } else {
      int64_t acc = 0;
      for (uint32_t lc = threadIdx.x; lc < nc; lc += NT) {
        const uint32_t* ml = mat + (int64_t)lc * (P + 1);
        acc += ml[pp + 1] - ml[pp];
      }
      len = (uint32_t)block_reduce(acc, s_red, OpAdd64());
    }
    uint64_t best = 0;
    for (uint32_t Q = 1;; Q <<= 1) {
      if (Q > kHubMaxPasses) {
        if (threadIdx.x == 0) *L.overflow = 1;
        return;
      }
      // one pass: a table of at least twice the pairs (then it never fills)
      uint32_t tsz = 256;
      while (tsz < 2 * len && tsz < (uint32_t)kHubPartTable) tsz <<= 1;
      const uint32_t mask = tsz - 1;
      bool fits = true;
      best = 0;
      for (uint32_t q = 0; q < Q && fits; ++q) {
        for (uint32_t j = threadIdx.x; j < tsz; j += NT) {
          keys[j] = -1;
          vals[j] = 0;
        }
        if (threadIdx.x == 0) s_used = 0;
        __syncthreads();
        // false once the table is too full for this pass (more passes follow)
        auto insert = [&](int2 pr) -> bool {
          const uint32_t hh = hash32((uint32_t)pr.x);
          if (((hh >> 12) & (Q - 1)) != q) return true;
          uint32_t h = hh & mask;
          for (uint32_t probes = 0;; ++probes) {
            if (probes > mask) {
              *L.overflow = 1;
              break;
            }
            const int32_t prev = atomicCAS(&keys[h], -1, pr.x);
            if (prev == -1 || prev == pr.x) {
              if (prev == -1) atomicAdd(&s_used, 1u);
              atomicAdd(&vals[h], pr.y);
              break;
            }
            h = (h + 1) & mask;
          }
          return s_used <= (uint32_t)kHubPartFill;
        };
        if (flat) {
          const uint32_t total = s_pre[nc];
          for (uint32_t x = threadIdx.x; x < total; x += NT) {
            uint32_t lo = 0, hi = nc - 1;  // the last chunk whose pairs start at or before x
            while (lo < hi) {
              const uint32_t mid = (lo + hi + 1) >> 1;
              if (s_pre[mid] <= x) lo = mid;
              else hi = mid - 1;
            }
            if (!insert(stage0[(int64_t)lo * kHubChunk + s_beg[lo] + (x - s_pre[lo])])) break;
          }
        } else {
          bool go = true;
          for (uint32_t lc = threadIdx.x; lc < nc && go; lc += NT) {
            const uint32_t* ml = mat + (int64_t)lc * (P + 1);
            const uint32_t s0 = ml[pp], s1 = ml[pp + 1];
            const int2* st = stage0 + (int64_t)lc * kHubChunk;
            for (uint32_t j = s0; j < s1 && go; ++j) go = insert(st[j]);
          }
        }
        __syncthreads();
        fits = s_used <= (uint32_t)kHubPartFill;
        if (fits) {
          uint64_t b = scan_table<8>(sl, keys, vals, tsz, threadIdx.x, NT, own_ok, conn_own, own, cv);
          b = block_reduce(b, red64, OpMax64());
          best = best > b ? best : b;
        }
        __syncthreads();
      }
      if (fits) break;
    }
    if (threadIdx.x == 0) {
      if (best) atomicMax(&L.best[i], (unsigned long long)best);
    }
    __syncthreads();
  }
}

template <bool ONE>
__global__ void __launch_bounds__(256) k_hub_final(const DevSlot* __restrict__ S, int ns,
                                                   const int32_t* __restrict__ list,
                                                   const uint32_t* __restrict__ cnt_ptr, HubLayout L) {
  if (*L.overflow) return;
  const uint32_t cnt = *cnt_ptr;
  const uint32_t stride = gridDim.x * blockDim.x;
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < cnt; i += stride) {
    const int64_t u = list[i];
    const DevSlot& sl = S[SLOT(u)];
    const int64_t v = u - sl.nbase;
    const int32_t own = gld(sl.lab, v);
    uint64_t best = L.best[i];
    if (own_allowed(sl, own)) {
      const uint64_t ok = pack_key(L.own[i], own);
      best = best > ok ? best : ok;
    }
    gst(sl.desire, v, best ? key_label(best) : own);
    L.own[i] = 0;
    L.best[i] = 0;
  }
}

// ---------------------------------------------------------------------------
// Admission.
// ---------------------------------------------------------------------------

// LDS table combining int64 additions to (slot, label) keys within a workgroup.
// Additions from many workgroups to one address are serialised by the
// memory system, and a few labels (the targets of hubs' neighbours, a block)
// receive most of them; so the admission kernels run a bounded grid, each
// workgroup walks one contiguous range of the rated list and keeps its table
// over the whole range, flushing it only when it fills or at the end.
constexpr unsigned long long kEmpty = ~0ull;
constexpr uint32_t kCountLabel = 0xFFFFFFFFu;  // key label used for per-slot counters

// Returns whether the key was new to the table; a key found there is marked
// hot (hot may be null).  The flush rule below keeps the table at most 3/4
// full; a probe over every slot sets *err (the round fails) instead of
// probing forever.
__device__ __forceinline__ bool agg_add(unsigned long long* hk, long long* hv, uint32_t mask, unsigned long long key,
                                        long long val, uint8_t* hot, uint32_t* err) {
  uint32_t h = hash32((uint32_t)key ^ (uint32_t)(key >> 32) * 0x9E3779B1u) & mask;
  for (uint32_t probes = 0; probes <= mask; ++probes) {
    // a slot that already holds the key needs no compare-and-swap
    unsigned long long prev = hk[h];
    if (prev == kEmpty) prev = atomicCAS(&hk[h], kEmpty, key);
    if (prev == kEmpty || prev == key) {
      atomicAdd((unsigned long long*)&hv[h], (unsigned long long)val);
      if (hot && prev == key) hot[h] = 1;
      return prev == kEmpty;
    }
    h = (h + 1) & mask;
  }
  atomicOr(err, 1u);
  return false;
}

constexpr int kAggNodes = 512;    // nodes per workgroup iteration
constexpr int kAggGrid = 1024;    // workgroups of the admission kernels at most
constexpr int kIncTable = 2048;   // new keys per iteration: at most kAggNodes
constexpr int kApplyTable = 2048; // new keys per iteration (departures): at most kAggNodes
constexpr int kDecideBuf = 2048;  // contended keys buffered per workgroup

// Range [b, e) of the N rated entries walked by this workgroup: whole
// iterations of `per_iter` entries, split evenly over the grid.
__device__ __forceinline__ void agg_range(int64_t N, int per_iter, int64_t& b, int64_t& e) {
  const int64_t iters = (N + per_iter - 1) / per_iter;
  const int64_t per = (iters + gridDim.x - 1) / gridDim.x;
  b = (int64_t)blockIdx.x * per * per_iter;
  e = b + per * per_iter < N ? b + per * per_iter : N;
  if (b > e) b = e;
}

// Counters of a carried table: keys inserted, keys removed by flushes, and
// hot keys counted at flushes (all only grow).
struct AggCtr {
  uint32_t ins, rem, hot;
};

template <int T>
__device__ __forceinline__ void agg_init(unsigned long long* hk, long long* hv, uint8_t* hot, AggCtr* c) {
  for (int j = threadIdx.x; j < T; j += blockDim.x) {
    hk[j] = kEmpty;
    hv[j] = 0;
    hot[j] = 0;
  }
  if (threadIdx.x == 0) c->ins = c->rem = c->hot = 0;
}

// Number of keys the workgroup's threads inserted (each passes its own
// count), added to *ctr by one lane per wave.
__device__ __forceinline__ void agg_count(uint32_t mine, uint32_t* ctr) {
  for (int off = 32; off > 0; off >>= 1) mine += __shfl_xor(mine, off);
  if (lane_id() == 0 && mine) atomicAdd(ctr, mine);
}

// End of an iteration of a 256-thread workgroup in which this thread
// inserted `ins` keys.  When the next iteration (at most `knew` new keys)
// could fill the table past 3/4, or at the end of the range (`last`), the
// table is flushed: every key is added to global memory by `emit` and
// removed, except, when not `last`, the keys added to more than once since
// the last flush if they are at most T/4 (they stay and keep summing: the
// labels most movers go to).  Then at most T/4 + knew <= 3T/4 slots are
// taken when the next flush is decided, so the table never fills.  A
// removed slot can cut the probe chain of a kept key; a later add of that
// key then takes a second slot, and both are emitted, so the sums stay
// exact.
template <int T, class Emit>
__device__ __forceinline__ void agg_step(unsigned long long* hk, long long* hv, uint8_t* hot, AggCtr* c,
                                         uint32_t ins, bool last, int knew, uint32_t& hot_seen, Emit emit) {
  constexpr int FQ = T / 256;
  static_assert(T % 256 == 0, "table size");
  agg_count(ins, &c->ins);
  __syncthreads();
  const uint32_t live = c->ins - c->rem;
  if (last || live + (uint32_t)knew > (uint32_t)T * 3 / 4) {
    bool keep = false;
    if (!last) {
      uint32_t nh = 0;
#pragma unroll
      for (int q = 0; q < FQ; ++q) {
        const int j = threadIdx.x + q * 256;
        nh += hk[j] != kEmpty && hot[j] ? 1u : 0u;
      }
      agg_count(nh, &c->hot);
      __syncthreads();
      const uint32_t now = c->hot;
      keep = now - hot_seen <= (uint32_t)T / 4;
      hot_seen = now;
    }
    unsigned long long fk[FQ];
    long long fv[FQ];
    uint32_t rem = 0;
#pragma unroll
    for (int q = 0; q < FQ; ++q) {
      const int j = threadIdx.x + q * 256;
      fk[q] = hk[j];
      fv[q] = hv[j];
      if (fk[q] == kEmpty) continue;
      if (keep && hot[j]) {
        hot[j] = 0;
        fk[q] = kEmpty;
      } else {
        hk[j] = kEmpty;
        hv[j] = 0;
        hot[j] = 0;
        ++rem;
      }
    }
    agg_count(rem, &c->rem);
    // the table is read first so that the atomics are issued back to back
#pragma unroll
    for (int q = 0; q < FQ; ++q)
      if (fk[q] != kEmpty && fv[q] != 0) emit(fk[q], fv[q]);
  }
  __syncthreads();
}

// inc(t) += c(v) for every mover v -> t (movers are rated nodes).
template <bool ONE>
__global__ void __launch_bounds__(256) k_incoming(const DevSlot* __restrict__ S, int ns,
                                                  const int32_t* __restrict__ rated, const uint32_t* __restrict__ rcnt) {
  __shared__ unsigned long long hk[kIncTable];
  __shared__ long long hv[kIncTable];
  __shared__ uint8_t hot[kIncTable];
  __shared__ AggCtr ctr;
  int64_t b, e;
  agg_range(*rcnt, kAggNodes, b, e);
  if (b == e) return;
  agg_init<kIncTable>(hk, hv, hot, &ctr);
  uint32_t hot_seen = 0;
  __syncthreads();
  for (int64_t base = b; base < e; base += kAggNodes) {
    constexpr int IT = kAggNodes / 256;
    int64_t u[IT], v[IT], cv[IT];
    int sv[IT];
    int32_t t[IT], own[IT];
    bool ok[IT];
#pragma unroll
    for (int it = 0; it < IT; ++it) {
      const int64_t i = base + it * 256 + threadIdx.x;
      ok[it] = i < e;
      u[it] = gld(rated, ok[it] ? i : e - 1);
    }
#pragma unroll
    for (int it = 0; it < IT; ++it) {
      sv[it] = SLOT(u[it]);
      const DevSlot& sl = S[sv[it]];
      v[it] = u[it] - sl.nbase;
      t[it] = gld(sl.desire, v[it]);
      own[it] = gld(sl.lab, v[it]);
      cv[it] = gld(sl.nw, v[it]);
    }
    uint32_t ins = 0;
#pragma unroll
    for (int it = 0; it < IT; ++it)
      if (ok[it] && t[it] != own[it] && !tile_admission(S[sv[it]]))
        ins += agg_add(hk, hv, kIncTable - 1, ((unsigned long long)sv[it] << 32) | (uint32_t)t[it], cv[it], hot,
                       S[0].err);
    agg_step<kIncTable>(hk, hv, hot, &ctr, ins, base + kAggNodes >= e, kAggNodes, hot_seen,
                        [&](unsigned long long k, long long x) { gadd64(S[ONE ? 0 : (k >> 32)].inc, (uint32_t)k, x); });
  }
}

// Movers into targets whose whole incoming weight fits are admitted; the
// others are appended as (target, node) keys for the exact path.  adm(v):
// bit 0 admitted by the exact path, bit 1 admitted at once, bit 2 alone.
constexpr uint8_t kAdmExact = 1, kAdmFast = 2, kAdmAlone = 4;
template <bool ONE>
__global__ void __launch_bounds__(256) k_decide(const DevSlot* __restrict__ S, int ns,
                                                const int32_t* __restrict__ rated, const uint32_t* __restrict__ rcnt,
                                                uint64_t* __restrict__ ckeys, uint32_t* __restrict__ ccnt,
                                                int node_bits) {
  __shared__ uint32_t s_w[4];
  __shared__ uint32_t s_n, s_base;
  __shared__ uint64_t buf[kDecideBuf];  // contended keys not yet reserved in ckeys
  const int w = threadIdx.x / kWave;
  const uint64_t lt = (1ull << lane_id()) - 1ull;
  int64_t b, e;
  agg_range(*rcnt, 256, b, e);
  if (b == e) return;
  if (threadIdx.x == 0) s_n = 0;
  __syncthreads();
  for (int64_t base = b; base < e; base += 256) {
    const int64_t i = base + threadIdx.x;
    bool contended = false;
    uint64_t key = 0;
    {
      const bool ok = i < e;
      const int64_t u = gld(rated, ok ? i : e - 1);
      const DevSlot& sl = S[SLOT(u)];
      const int64_t v = u - sl.nbase;
      const int32_t t = gld(sl.desire, v);
      const int32_t own = gld(sl.lab, v);
      if (ok && t != own && !tile_admission(sl)) {
        // kAdmAlone: W(own) = c(v), so every other member of the label has
        // weight 0 (node weights are >= 0) and v's departure is the only
        // change of W(own) in k_apply (departures of weight 0 are skipped)
        const uint8_t alone = gld(sl.W, own) == gld(sl.nw, v) ? kAdmAlone : 0;
        if (gld(sl.W, t) + gld(sl.inc, t) <= sl.cap) {
          gst(sl.adm, v, (uint8_t)(kAdmFast | alone));  // the target takes all its movers (k_fold adds them)
        } else {
          gst(sl.adm, v, alone);
          contended = true;
          key = ((uint64_t)(sl.lbase + t) << node_bits) | (uint64_t)u;
        }
      }
    }
    const uint64_t m = __ballot(contended);
    if (lane_id() == 0) s_w[w] = (uint32_t)__popcll(m);
    __syncthreads();
    const uint32_t n0 = s_n;
    uint32_t off = n0, tot = 0;
    for (int q = 0; q < 4; ++q) {
      if (q < w) off += s_w[q];
      tot += s_w[q];
    }
    if (contended) buf[off + (uint32_t)__popcll(m & lt)] = key;
    __syncthreads();
    // one reservation in ckeys per buffer load
    const uint32_t n1 = n0 + tot;
    if (n1 > 0 && (base + 256 >= e || n1 + 256 > kDecideBuf)) {
      if (threadIdx.x == 0) s_base = atomicAdd(ccnt, n1);
      __syncthreads();
      const uint32_t at = s_base;
      for (uint32_t j = threadIdx.x; j < n1; j += 256) ckeys[at + j] = buf[j];
      if (threadIdx.x == 0) s_n = 0;
    } else if (threadIdx.x == 0) {
      s_n = n1;
    }
    __syncthreads();
  }
}

// Targets whose whole incoming weight fits take it at once: W(t) += inc(t);
// inc is cleared for every label.  Runs after k_decide (which made the same
// test per mover) and before any other change of W in the round.
template <bool ONE>
__global__ void __launch_bounds__(256) k_fold(const DevSlot* __restrict__ S, int ns, int64_t Lt) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < Lt; g += stride) {
    int s = 0;
    if (!ONE) {
      int lo = 0, hi = ns - 1;
      while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (S[mid].lbase <= g) lo = mid;
        else hi = mid - 1;
      }
      s = lo;
    }
    const DevSlot& sl = S[s];
    const int64_t t = g - sl.lbase;
    if (t >= sl.nlabels || tile_admission(sl)) continue;
    const int64_t x = gld(sl.inc, t);
    if (x == 0) continue;
    const int64_t w = gld(sl.W, t);
    if (w + x <= sl.cap) gst(sl.W, t, w + x);
    gst(sl.inc, t, (int64_t)0);
  }
}

// For sorted contended keys: segment key (target) and weight of each entry.
template <bool ONE>
__global__ void __launch_bounds__(256) k_contended_split(const DevSlot* __restrict__ S, int ns,
                                                         const uint64_t* __restrict__ keys, uint32_t cnt,
                                                         int node_bits, uint32_t* __restrict__ tkey,
                                                         int64_t* __restrict__ wv) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= cnt) return;
  const uint64_t k = keys[i];
  const int64_t u = (int64_t)(k & ((1ull << node_bits) - 1ull));
  const DevSlot& sl = S[SLOT(u)];
  tkey[i] = (uint32_t)(k >> node_bits);
  wv[i] = sl.nw[u - sl.nbase];
}

// Admit contended movers whose inclusive prefix fits.
template <bool ONE>
__global__ void __launch_bounds__(256) k_contended_mark(const DevSlot* __restrict__ S, int ns,
                                                        const uint64_t* __restrict__ keys, uint32_t cnt,
                                                        int node_bits, const int64_t* __restrict__ prefix) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= cnt) return;
  const uint64_t k = keys[i];
  const int64_t u = (int64_t)(k & ((1ull << node_bits) - 1ull));
  const DevSlot& sl = S[SLOT(u)];
  const int64_t v = u - sl.nbase;
  const int32_t t = sl.desire[v];
  sl.adm[v] = (uint8_t)((sl.adm[v] & kAdmAlone) | (sl.W[t] + prefix[i] <= sl.cap ? kAdmExact : 0));
}

// Arrivals of the admitted contended movers (after k_contended_mark): the last
// admitted entry of each target's segment adds its inclusive prefix to W.
template <bool ONE>
__global__ void __launch_bounds__(256) k_contended_add(const DevSlot* __restrict__ S, int ns,
                                                       const uint64_t* __restrict__ keys, uint32_t cnt,
                                                       int node_bits, const int64_t* __restrict__ prefix) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= cnt) return;
  const uint64_t nmask = (1ull << node_bits) - 1ull;
  const uint64_t k = keys[i];
  const int64_t u = (int64_t)(k & nmask);
  const DevSlot& sl = S[SLOT(u)];
  const int64_t v = u - sl.nbase;
  if (!(sl.adm[v] & kAdmExact)) return;
  if (i + 1 < cnt && (keys[i + 1] >> node_bits) == (k >> node_bits)) {
    const int64_t u2 = (int64_t)(keys[i + 1] & nmask);
    const DevSlot& s2 = S[SLOT(u2)];
    if (s2.adm[u2 - s2.nbase] & kAdmExact) return;
  }
  const int32_t t = sl.desire[v];
  gst(sl.W, t, gld(sl.W, t) + prefix[i]);
}

// Contended movers, when at most kSmallContended: one workgroup sorts the
// (target, node) keys in LDS (bitonic), scans the weights per target and
// admits the inclusive prefixes that fit.  Larger sets are left to the
// device-wide path and flagged.
constexpr int kSmallContended = 2048;

template <bool ONE>
__global__ void __launch_bounds__(1024) k_contended_small(const DevSlot* __restrict__ S, int ns,
                                                          const uint64_t* __restrict__ keys,
                                                          const uint32_t* __restrict__ ccnt, int node_bits,
                                                          uint32_t* __restrict__ big_flag) {
  __shared__ uint64_t k[kSmallContended];
  __shared__ int64_t w[kSmallContended];
  __shared__ int8_t head[kSmallContended];
  __shared__ int8_t ad[kSmallContended];
  const uint32_t cnt = *ccnt;
  if (cnt == 0) return;
  if (cnt > kSmallContended) {
    if (threadIdx.x == 0) *big_flag = 1;
    return;
  }
  uint32_t P = 1;
  while (P < cnt) P <<= 1;
  for (uint32_t i = threadIdx.x; i < P; i += blockDim.x) k[i] = i < cnt ? keys[i] : ~0ull;
  __syncthreads();
  for (uint32_t size = 2; size <= P; size <<= 1) {
    for (uint32_t stride = size >> 1; stride > 0; stride >>= 1) {
      for (uint32_t i = threadIdx.x; i < P; i += blockDim.x) {
        const uint32_t j = i ^ stride;
        if (j > i) {
          const bool up = (i & size) == 0;
          const uint64_t a = k[i], b = k[j];
          if ((a > b) == up) {
            k[i] = b;
            k[j] = a;
          }
        }
      }
      __syncthreads();
    }
  }
  const uint64_t nmask = (1ull << node_bits) - 1ull;
  for (uint32_t i = threadIdx.x; i < cnt; i += blockDim.x) {
    const int64_t u = (int64_t)(k[i] & nmask);
    const DevSlot& sl = S[SLOT(u)];
    w[i] = sl.nw[u - sl.nbase];
    head[i] = (i == 0 || (k[i] >> node_bits) != (k[i - 1] >> node_bits)) ? 1 : 0;
  }
  __syncthreads();
  // inclusive segmented scan (Hillis-Steele on (value, head) pairs)
  for (uint32_t off = 1; off < cnt; off <<= 1) {
    int64_t nv[2];
    int8_t nh[2];
    int c = 0;
    for (uint32_t i = threadIdx.x; i < cnt; i += blockDim.x, ++c) {
      nv[c] = w[i];
      nh[c] = head[i];
      if (i >= off && !head[i]) {
        nv[c] += w[i - off];
        nh[c] = head[i - off];
      }
    }
    __syncthreads();
    c = 0;
    for (uint32_t i = threadIdx.x; i < cnt; i += blockDim.x, ++c) {
      w[i] = nv[c];
      head[i] = nh[c];
    }
    __syncthreads();
  }
  for (uint32_t i = threadIdx.x; i < cnt; i += blockDim.x) {
    const int64_t u = (int64_t)(k[i] & nmask);
    const DevSlot& sl = S[SLOT(u)];
    const int64_t v = u - sl.nbase;
    const int32_t t = sl.desire[v];
    ad[i] = sl.W[t] + w[i] <= sl.cap ? 1 : 0;
    sl.adm[v] = (uint8_t)((sl.adm[v] & kAdmAlone) | ad[i]);
  }
  __syncthreads();
  // the admitted movers of a target are a prefix of its segment (weights are
  // positive): the last of them adds the prefix sum to the target's weight
  for (uint32_t i = threadIdx.x; i < cnt; i += blockDim.x) {
    if (!ad[i]) continue;
    if (i + 1 < cnt && ad[i + 1] && (k[i + 1] >> node_bits) == (k[i] >> node_bits)) continue;
    const int64_t u = (int64_t)(k[i] & nmask);
    const DevSlot& sl = S[SLOT(u)];
    const int32_t t = sl.desire[u - sl.nbase];
    gst(sl.W, t, gld(sl.W, t) + w[i]);
  }
}

// Apply admitted moves; reset rejected desires and the incoming sums; in
// refinement add the neighbours of moved nodes to the next rated set.
template <bool ONE>
__global__ void __launch_bounds__(256) k_apply(const DevSlot* __restrict__ S, int ns,
                                               const int32_t* __restrict__ rated, const uint32_t* __restrict__ rcnt,
                                               int32_t* __restrict__ mold, const uint32_t* __restrict__ skip) {
  __shared__ unsigned long long hk[kApplyTable];
  __shared__ long long hv[kApplyTable];
  __shared__ uint8_t hot[kApplyTable];
  __shared__ AggCtr ctr;
  __shared__ int s_cs[4];      // per wave: slot of the moved count carried to the end
  __shared__ long long s_cv[4];
  if (skip && *skip) return;  // the admission is completed on the host-driven path first
  int64_t b, e;
  agg_range(*rcnt, kAggNodes, b, e);
  if (b == e) return;
  agg_init<kApplyTable>(hk, hv, hot, &ctr);
  uint32_t hot_seen = 0;
  // moved count of the wave's current slot run (lane 0)
  int cnt_slot = -1;
  long long cnt_val = 0;
  __syncthreads();
  for (int64_t base = b; base < e; base += kAggNodes) {
    constexpr int IT = kAggNodes / 256;
    int64_t uu[IT];
    bool ok[IT];
#pragma unroll
    for (int it = 0; it < IT; ++it) {
      const int64_t i = base + it * 256 + threadIdx.x;
      ok[it] = i < e;
      uu[it] = gld(rated, ok[it] ? i : e - 1);
    }
    // every load of the iteration is issued before its first store (memory
    // operations complete in order, so a load after a store waits for it)
    int32_t tt[IT], oo[IT];
    uint8_t aa[IT];
    int64_t ww[IT];
#pragma unroll
    for (int it = 0; it < IT; ++it) {
      const DevSlot& sl = S[SLOT(uu[it])];
      const int64_t v = uu[it] - sl.nbase;
      tt[it] = gld(sl.desire, v);
      oo[it] = gld(sl.lab, v);
      aa[it] = gld(sl.adm, v);
      ww[it] = gld(sl.nw, v);
    }
    uint32_t ins = 0;
    for (int it = 0; it < IT; ++it) {
      const int64_t u = uu[it];
      const int s = SLOT(u);
      const DevSlot& sl = S[s];
      const int64_t v = u - sl.nbase;
      const int32_t t = tt[it];
      const int32_t own = oo[it];
      bool admitted = false;
      int64_t cv = 0;
      const bool mine = ok[it] && !tile_admission(sl);
      bool alone = false;
      if (mine && t != own) {
        admitted = (aa[it] & (kAdmExact | kAdmFast)) != 0;
        alone = (aa[it] & kAdmAlone) != 0;
        if (admitted) {
          cv = ww[it];
          gst(sl.lab, v, t);
        } else {
          gst(sl.desire, v, own);
        }
      }
      // refinement: old block of every admitted mover by rated position (-1: stayed)
      if (mine && sl.mode == MODE_REFINE) gst(mold, base + it * 256 + threadIdx.x, admitted ? own : -1);
      // departures (-c(v) from the old label); the arrivals were added
      // before (k_fold for targets that take all their movers, the exact
      // path for the others)
      const unsigned long long ks = (unsigned long long)s << 32;
      if (admitted && cv != 0) {
        if (alone) gst(sl.W, own, gld(sl.W, own) - cv);  // no other change of W(own) here
        else ins += agg_add(hk, hv, kApplyTable - 1, ks | (uint32_t)own, -cv, hot, S[0].err);
      }
      // moved count: carried by the wave while its slot does not change
      const int s0 = __shfl(s, 0);
      if (__all(s == s0)) {
        const uint64_t m = __ballot(admitted);
        if (lane_id() == 0 && m) {
          if (s0 != cnt_slot) {
            if (cnt_val) gadd64(S[cnt_slot].ctr, CTR_MOVED, cnt_val);
            cnt_slot = s0;
            cnt_val = 0;
          }
          cnt_val += (long long)__popcll(m);
        }
      } else if (admitted) {
        gadd64(sl.ctr, CTR_MOVED, (int64_t)1);
      }
    }
    agg_step<kApplyTable>(hk, hv, hot, &ctr, ins, base + kAggNodes >= e, kAggNodes, hot_seen,
                          [&](unsigned long long k, long long x) { gadd64(S[ONE ? 0 : (k >> 32)].W, (uint32_t)k, x); });
  }
  // moved counts: the waves' carried counts combined per slot
  if (lane_id() == 0) {
    s_cs[threadIdx.x / kWave] = cnt_val ? cnt_slot : -1;
    s_cv[threadIdx.x / kWave] = cnt_val;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int q = 0; q < 4; ++q) {
      if (s_cs[q] < 0) continue;
      long long x = s_cv[q];
      for (int r = q + 1; r < 4; ++r)
        if (s_cs[r] == s_cs[q]) {
          x += s_cv[r];
          s_cs[r] = -1;
        }
      gadd64(S[s_cs[q]].ctr, CTR_MOVED, (int64_t)x);
    }
  }
}

// Refinement: the neighbours of moved nodes join the next rated set, and
// where block connections are kept, every entry (u, v, w) of a mover u from
// block a to block b moves w from conn(v, a) to conn(v, b).  Each wave takes
// 64 movers; rows of up to 64 entries are walked by their lane, rows of up
// to kMarkBig entries by the whole wave; longer rows are listed (by mover
// index) for k_mark_big: rows of up to kMarkHuge entries are walked by one
// workgroup each, longer ones by all workgroups together.
constexpr int64_t kMarkBig = 4096;
constexpr int64_t kMarkHuge = 65536;

__device__ __forceinline__ void conn_add(int32_t* conn, int64_t i, int32_t v) {
  __hip_atomic_fetch_add((SCLAP_GLOBAL int*)(conn + i), v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Entries first, first + step, ... below d of a mover's row starting at e0:
// mark every neighbour, and move the entry's weight from block a to block b in
// the neighbour's connections (a < 0: no connections).  The next B entries
// are loaded before the current ones are written, so that a thread does not
// wait for its stores and atomics (memory operations complete in order).
template <int B>
__device__ __forceinline__ void mark_row(const DevSlot& sl, int64_t e0, int64_t first, int64_t d, int step,
                                         int32_t a, int32_t b) {
  if (first >= d) return;
  const bool conn = a >= 0;
  int32_t nb[B], w[B];
#pragma unroll
  for (int q = 0; q < B; ++q) {
    const int64_t ee = first + (int64_t)q * step;
    const int64_t ec = e0 + (ee < d ? ee : d - 1);
    nb[q] = gld(sl.col, ec);
    w[q] = conn && sl.ew ? gld(sl.ew, ec) : 1;
  }
  for (int64_t base = first; base < d; base += (int64_t)step * B) {
    int32_t cn[B], cw[B];
#pragma unroll
    for (int q = 0; q < B; ++q) {
      cn[q] = nb[q];
      cw[q] = w[q];
    }
    const int64_t next = base + (int64_t)step * B;
    if (next < d) {
#pragma unroll
      for (int q = 0; q < B; ++q) {
        const int64_t ee = next + (int64_t)q * step;
        const int64_t ec = e0 + (ee < d ? ee : d - 1);
        nb[q] = gld(sl.col, ec);
        w[q] = conn && sl.ew ? gld(sl.ew, ec) : 1;
      }
    }
#pragma unroll
    for (int q = 0; q < B; ++q) {
      if (base + (int64_t)q * step >= d) continue;
      gst(sl.flag_next, cn[q], (uint8_t)1);
      if (conn) {
        const int64_t r = (int64_t)cn[q] * sl.conn_k;
        conn_add(sl.conn, r + a, -cw[q]);
        conn_add(sl.conn, r + b, cw[q]);
      }
    }
  }
}

// Whether the moves of the round are added to the slot's block connections
// (the same answer for every thread: it depends on the final moved count).
__device__ __forceinline__ bool conn_push(const DevSlot& sl) {
  return sl.conn && !sl.last_round && gld(sl.ctr, CTR_MOVED) * kConnPushDiv <= sl.n;
}

// Blocks (a, b) of a mover from block oa when its moves are added to block
// connections, else -1.
__device__ __forceinline__ void mover_blocks(const DevSlot& sl, int32_t oa, int64_t v, int32_t& a, int32_t& b) {
  a = b = -1;
  if (conn_push(sl)) {
    const int32_t nb = gld(sl.lab, v);
    if ((uint32_t)oa < (uint32_t)sl.conn_k && (uint32_t)nb < (uint32_t)sl.conn_k) {
      a = oa;
      b = nb;
    }
  }
}

// Entries x .. of the short rows listed in a wave's LDS arrays (ex: exclusive
// prefix of the row lengths, e0: first entry, ab: blocks a | b << 32 or a < 0,
// sl: slot): lane l takes entry x0 + l of the concatenated rows and loads its
// neighbour and weight.
struct ShortRows {
  int32_t* ex;
  int64_t* e0;
  int64_t* ab;
  int32_t* sl;
};

struct ShortEntry {
  int32_t nb, w, a, b, s;
};

template <bool ONE>
__device__ __forceinline__ ShortEntry short_entry(const DevSlot* __restrict__ S, const ShortRows& R, int32_t x,
                                                  int32_t tot) {
  ShortEntry r{-1, 0, -1, -1, 0};
  if (x >= tot) return r;
  int lo = 0, hi = kWave - 1;  // the last row starting at or before x
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (R.ex[mid] <= x) lo = mid;
    else hi = mid - 1;
  }
  r.s = ONE ? 0 : R.sl[lo];
  const DevSlot& q = S[r.s];
  const int64_t e = R.e0[lo] + (x - R.ex[lo]);
  const int64_t ab = R.ab[lo];
  r.nb = gld(q.col, e);
  r.a = (int32_t)ab;
  r.b = (int32_t)(ab >> 32);
  r.w = r.a >= 0 && q.ew ? gld(q.ew, e) : 1;
  return r;
}

template <bool ONE>
__device__ __forceinline__ void short_apply(const DevSlot* __restrict__ S, const ShortEntry& r) {
  if (r.nb < 0) return;
  const DevSlot& q = S[r.s];
  gst(q.flag_next, r.nb, (uint8_t)1);
  if (r.a >= 0) {
    const int64_t row = (int64_t)r.nb * q.conn_k;
    conn_add(q.conn, row + r.a, -r.w);
    conn_add(q.conn, row + r.b, r.w);
  }
}

// Movers: rated positions i of refinement slots with mold[i] >= 0 (the old
// block).  Rows of up to 64 entries are walked by the whole wave over their
// concatenated entries (a batch costs its total entries / 64 steps rather
// than its longest row), the next step's loads issued before the current
// step's stores.
template <bool ONE>
__global__ void __launch_bounds__(256) k_mark(const DevSlot* __restrict__ S, int ns,
                                              const int32_t* __restrict__ rated, const uint32_t* __restrict__ rcnt,
                                              const int32_t* __restrict__ mold,
                                              int32_t* __restrict__ big, uint32_t* __restrict__ big_cnt,
                                              uint32_t* __restrict__ huge_cnt, int64_t big_cap,
                                              const uint32_t* __restrict__ skip,
                                              unsigned long long* __restrict__ entries) {
  __shared__ int32_t s_ex[4][kWave];
  __shared__ int64_t s_e0[4][kWave];
  __shared__ int64_t s_ab[4][kWave];
  __shared__ int32_t s_sl[4][kWave];
  if (skip && *skip) return;
  if (blockIdx.x == 0)
    for (int s = threadIdx.x; s < ns; s += blockDim.x)
      if (S[s].conn && !S[s].last_round && !conn_push(S[s])) gst(S[s].ctr, CTR_STALE, (int64_t)1);
  const int wv = threadIdx.x / kWave;
  const ShortRows R{s_ex[wv], s_e0[wv], s_ab[wv], s_sl[wv]};
  const uint32_t cnt = *rcnt;
  const uint32_t waves = gridDim.x * (blockDim.x / kWave);
  const uint32_t wid = blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave;
  for (uint32_t base = wid * kWave; base < cnt; base += waves * kWave) {
    const uint32_t i = base + lane_id();
    const DevSlot* sl = nullptr;
    int64_t e0 = 0, d = 0;
    int32_t u = 0, a = -1, b = -1, si = 0;
    if (i < cnt) {
      u = gld(rated, i);
      si = SLOT(u);
      sl = &S[si];
      // the last round of a stage has no next rated set to mark
      const int32_t oa = sl->mode == MODE_REFINE && !sl->last_round ? gld(mold, i) : -1;
      if (oa >= 0) {
        const int64_t v = u - sl->nbase;
        e0 = gld(sl->rp, v);
        d = gld(sl->rp, v + 1) - e0;
        mover_blocks(*sl, oa, v, a, b);
      }
    }
    if (entries) {
      // measurement only: the entries of the movers' rows, one add per wave
      uint64_t wd = (uint64_t)d;
      for (int off = 32; off > 0; off >>= 1) wd += __shfl_xor(wd, off);
      if (lane_id() == 0 && wd) atomicAdd(entries, (unsigned long long)wd);
    }
    {
      const int32_t ds = d > 0 && d <= kWave ? (int32_t)d : 0;
      int32_t incl = ds;
      for (int off = 1; off < kWave; off <<= 1) {
        const int32_t o = __shfl_up(incl, off);
        if ((int)lane_id() >= off) incl += o;
      }
      const int32_t tot = __shfl(incl, kWave - 1);
      if (tot > 0) {
        R.ex[lane_id()] = incl - ds;
        R.e0[lane_id()] = e0;
        R.ab[lane_id()] = (int64_t)((uint64_t)(uint32_t)a | ((uint64_t)(uint32_t)b << 32));
        R.sl[lane_id()] = si;
        wave_sync();
        ShortEntry cur = short_entry<ONE>(S, R, (int32_t)lane_id(), tot);
        for (int32_t x0 = 0; x0 < tot; x0 += kWave) {
          const ShortEntry nxt = short_entry<ONE>(S, R, x0 + kWave + (int32_t)lane_id(), tot);
          short_apply<ONE>(S, cur);
          cur = nxt;
        }
        wave_sync();  // the rows are read before the next batch writes them
      }
    }
    // without a big list (no row above kMarkBig) the wave walks every row
    // rows above kMarkBig go to the big list from its front, rows above
    // kMarkHuge from its back (the two counts add up to at most big_cap)
    if (big && d > kMarkBig) {
      if (d > kMarkHuge) big[big_cap - 1 - (int64_t)atomicAdd(huge_cnt, 1u)] = (int32_t)i;
      else big[atomicAdd(big_cnt, 1u)] = (int32_t)i;
    }
    uint64_t mid = __ballot(d > kWave && (d <= kMarkBig || !big));
    while (mid) {
      const int l = __ffsll((unsigned long long)mid) - 1;
      mid &= mid - 1;
      const int64_t be0 = __shfl(e0, l), bd = __shfl(d, l);
      const int32_t bu = __shfl(u, l), ba = __shfl(a, l), bb = __shfl(b, l);
      const DevSlot& bs = S[SLOT(bu)];
      mark_row<4>(bs, be0, lane_id(), bd, kWave, ba, bb);
    }
  }
}

template <bool ONE>
__global__ void __launch_bounds__(256) k_mark_big(const DevSlot* __restrict__ S, int ns,
                                                  const int32_t* __restrict__ rated, const int32_t* __restrict__ mold,
                                                  const int32_t* __restrict__ big, const uint32_t* __restrict__ big_cnt,
                                                  const uint32_t* __restrict__ huge_cnt, int64_t big_cap,
                                                  const uint32_t* __restrict__ skip) {
  if (skip && *skip) return;
  // rows of up to kMarkHuge entries: one workgroup each
  const uint32_t cnt = *big_cnt;
  for (uint32_t k = blockIdx.x; k < cnt; k += gridDim.x) {
    const uint32_t mi = (uint32_t)big[k];
    const int64_t u = rated[mi];
    const DevSlot& sl = S[SLOT(u)];
    const int64_t v = u - sl.nbase;
    int32_t a, b;
    mover_blocks(sl, mold[mi], v, a, b);
    const int64_t e0 = sl.rp[v], e1 = sl.rp[v + 1];
    mark_row<4>(sl, e0, (int64_t)threadIdx.x, e1 - e0, (int)blockDim.x, a, b);
  }
  // longer rows: every workgroup takes a share of each
  const uint32_t hc = *huge_cnt;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (uint32_t k = 0; k < hc; ++k) {
    const uint32_t mi = (uint32_t)big[big_cap - 1 - (int64_t)k];
    const int64_t u = rated[mi];
    const DevSlot& sl = S[SLOT(u)];
    const int64_t v = u - sl.nbase;
    int32_t a, b;
    mover_blocks(sl, mold[mi], v, a, b);
    const int64_t e0 = sl.rp[v], e1 = sl.rp[v + 1];
    mark_row<4>(sl, e0, (int64_t)blockIdx.x * blockDim.x + threadIdx.x, e1 - e0, (int)stride, a, b);
  }
}

// ---------------------------------------------------------------------------
// Admission of tile-admitted refinement slots by binning tiles (the rated
// nodes of a tile form a node-ordered range of the rated list, and a tile
// belongs to one slot):
//   sums    per tile and target block: the weight of its movers
//   (scan)  per target and slot, an inclusive scan of the tile sums
//   admit   a mover's inclusive prefix among the movers to its target in node
//           order = earlier tiles + earlier waves of the tile + earlier lanes
//           + its own weight; admitted iff W(t) + prefix <= cap (Section 3:
//           the longest fitting prefix, as every weight is >= 0).  Moves are
//           applied at once; per tile the block weight changes and the moved
//           count are written out
//   reduce  per slot and block: W(b) += the tiles' changes, and the moved count.
// ---------------------------------------------------------------------------
template <bool ONE>
__global__ void __launch_bounds__(kBinTile) k_ta_sums(const DevSlot* __restrict__ S, int ns,
                                                      const int32_t* __restrict__ rated, TileAdm A) {
  __shared__ unsigned long long sums[kConnMaxK];
  for (int64_t t = blockIdx.x; t < A.T; t += gridDim.x) {
    const int s = ONE ? 0 : slot_of_tile(S, ns, t);
    const DevSlot& sl = S[s];
    const bool on = tile_admission(sl) && sl.round > 0;
    if (threadIdx.x < kConnMaxK) sums[threadIdx.x] = 0;
    __syncthreads();
    if (on) {
      const uint32_t i = A.roff[t] - A.roff[0] + threadIdx.x;
      if (i < A.roff[t + 1] - A.roff[0]) {
        const int64_t v = gld(rated, i) - sl.nbase;
        const int32_t tt = gld(sl.desire, v), own = gld(sl.lab, v);
        if (tt != own && (uint32_t)tt < (uint32_t)sl.nlabels)
          atomicAdd(&sums[tt], (unsigned long long)gld(sl.nw, v));
      }
    }
    __syncthreads();
    if ((int)threadIdx.x < A.kmax) {
      A.tsum[threadIdx.x * A.T + t] = on ? (int64_t)sums[threadIdx.x] : 0;
      A.keys[threadIdx.x * A.T + t] = threadIdx.x * (uint32_t)ns + (uint32_t)s;
    }
    __syncthreads();
  }
}

template <bool ONE>
__global__ void __launch_bounds__(kBinTile) k_ta_admit(const DevSlot* __restrict__ S, int ns,
                                                       const int32_t* __restrict__ rated, TileAdm A,
                                                       int32_t* __restrict__ mold) {
  __shared__ long long wtot[kBinTile / kWave][kConnMaxK];
  __shared__ unsigned long long dsum[kConnMaxK];
  __shared__ uint32_t s_moved;
  const int w = threadIdx.x / kWave;
  const int lane = (int)lane_id();
  for (int64_t t = blockIdx.x; t < A.T; t += gridDim.x) {
    const int s = ONE ? 0 : slot_of_tile(S, ns, t);
    const DevSlot& sl = S[s];
    if (!(tile_admission(sl) && sl.round > 0)) continue;  // the same for the whole workgroup
    for (int j = threadIdx.x; j < (kBinTile / kWave) * kConnMaxK; j += blockDim.x) (&wtot[0][0])[j] = 0;
    if (threadIdx.x < kConnMaxK) dsum[threadIdx.x] = 0;
    if (threadIdx.x == 0) s_moved = 0;
    __syncthreads();
    const uint32_t i = A.roff[t] - A.roff[0] + threadIdx.x;
    const bool valid = i < A.roff[t + 1] - A.roff[0];
    int64_t v = 0, c = 0;
    int32_t tt = -1, own = -1;
    if (valid) {
      v = gld(rated, i) - sl.nbase;
      tt = gld(sl.desire, v);
      own = gld(sl.lab, v);
      c = gld(sl.nw, v);
    }
    const bool mover =
        valid && tt != own && (uint32_t)tt < (uint32_t)sl.nlabels && (uint32_t)own < (uint32_t)sl.nlabels;
    // exclusive prefix among the wave's movers to the same target
    int64_t excl = 0;
    uint64_t rem = __ballot(mover);
    while (rem) {
      const int lead = __ffsll((unsigned long long)rem) - 1;
      const int32_t j0 = __shfl(tt, lead);
      const bool mine = mover && tt == j0;
      const uint64_t m = __ballot(mine);
      int64_t x = mine ? c : 0;
      for (int off = 1; off < kWave; off <<= 1) {
        const int64_t y = __shfl_up(x, off);
        if (lane >= off) x += y;
      }
      if (mine) excl = x - c;
      if (lane == kWave - 1) wtot[w][j0] = x;
      rem &= ~m;
    }
    __syncthreads();
    bool adm = false;
    if (mover) {
      int64_t before = 0;
      for (int q = 0; q < w; ++q) before += wtot[q][tt];
      const int64_t k = (int64_t)tt * A.T + t;
      const int64_t incl = (A.tpre[k] - A.tsum[k]) + before + excl + c;
      adm = gld(sl.W, tt) + incl <= sl.cap;
    }
    if (valid) {
      if (adm) {
        gst(sl.lab, v, tt);
        atomicAdd(&dsum[tt], (unsigned long long)c);
        atomicAdd(&dsum[own], (unsigned long long)(-c));
      } else if (mover) {
        gst(sl.desire, v, own);
      }
      gst(mold, i, adm ? own : -1);
    }
    const uint64_t am = __ballot(adm);
    if (lane == 0 && am) atomicAdd(&s_moved, (uint32_t)__popcll(am));
    __syncthreads();
    if ((int)threadIdx.x < A.kmax) A.dW[threadIdx.x * A.T + t] = (int64_t)dsum[threadIdx.x];
    if (threadIdx.x == 0) A.tmoved[t] = s_moved;
    __syncthreads();
  }
}

// Inclusive scan of the tile sums of workgroup (j, s): block j, slot s, for
// slots of at most kTaScanTiles tiles (one launch instead of the
// device-wide scan-by-key).
constexpr int kTaScanTiles = 4 * 1024;

__global__ void __launch_bounds__(1024) k_ta_scan_small(const DevSlot* __restrict__ S, int ns, TileAdm A) {
  __shared__ int64_t sh[1024 / kWave];
  const int j = (int)(blockIdx.x % (uint32_t)A.kmax), s = (int)(blockIdx.x / (uint32_t)A.kmax);
  const DevSlot& sl = S[s];
  if (!(tile_admission(sl) && sl.round > 0) || j >= sl.nlabels) return;
  const int64_t t0 = sl.tbase, t1 = s + 1 < ns ? S[s + 1].tbase : A.T;
  constexpr int Q = kTaScanTiles / 1024;
  const int64_t* in = A.tsum + (int64_t)j * A.T;
  int64_t* out = A.tpre + (int64_t)j * A.T;
  int64_t x[Q], sum = 0;
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    const int64_t t = t0 + (int64_t)threadIdx.x * Q + q;
    x[q] = t < t1 ? in[t] : 0;
    sum += x[q];
  }
  int64_t incl = sum;
  for (int o = 1; o < kWave; o <<= 1) {
    const int64_t y = __shfl_up(incl, o);
    if ((int)lane_id() >= o) incl += y;
  }
  const int w = threadIdx.x / kWave;
  if (lane_id() == kWave - 1) sh[w] = incl;
  __syncthreads();
  int64_t run = incl - sum;
  for (int q = 0; q < w; ++q) run += sh[q];
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    const int64_t t = t0 + (int64_t)threadIdx.x * Q + q;
    run += x[q];
    if (t < t1) out[t] = run;
  }
}

// Workgroup (s, j): slot s, block j < kmax (its weight) or j = kmax (moved).
__global__ void __launch_bounds__(256) k_ta_reduce(const DevSlot* __restrict__ S, int ns, TileAdm A) {
  __shared__ int64_t red[8];
  const int s = (int)(blockIdx.x / (uint32_t)(A.kmax + 1)), j = (int)(blockIdx.x % (uint32_t)(A.kmax + 1));
  const DevSlot& sl = S[s];
  if (!(tile_admission(sl) && sl.round > 0) || (j < A.kmax && j >= sl.nlabels)) return;
  const int64_t t0 = sl.tbase, t1 = s + 1 < ns ? S[s + 1].tbase : A.T;
  int64_t sum = 0;
  for (int64_t t = t0 + threadIdx.x; t < t1; t += blockDim.x) sum += j < A.kmax ? A.dW[(int64_t)j * A.T + t] : A.tmoved[t];
  for (int off = 32; off > 0; off >>= 1) sum += __shfl_xor(sum, off);
  if (lane_id() == 0) red[threadIdx.x / kWave] = sum;
  __syncthreads();
  if (threadIdx.x == 0) {
    int64_t tot = 0;
    for (int q = 0; q < (int)(blockDim.x / kWave); ++q) tot += red[q];
    if (j < A.kmax) gst(sl.W, j, gld(sl.W, j) + tot);
    else gst(sl.ctr, CTR_MOVED, tot);
  }
}

// ---------------------------------------------------------------------------
// Block connections, first round of a refined level: conn(v, b) for every
// binned node of a CONN_BUILD slot, by G lanes per node (degree bins 0-7)
// adding into a per-node LDS row, or one wave per hub chunk (bin 8) adding
// its LDS row to the (zeroed) global row.
// ---------------------------------------------------------------------------
template <int G, bool ONE>
__device__ __forceinline__ void conn_build_group(const DevSlot* __restrict__ S, int ns,
                                                 const int32_t* __restrict__ list, const uint64_t* __restrict__ info,
                                                 uint32_t cnt, uint32_t wid, uint32_t nwaves, int32_t* rows) {
  constexpr int NG = kWave / G;
  constexpr int B = 4;
  const int lane = (int)lane_id(), gl = lane & (G - 1), gi = lane / G;
  int32_t* my = rows + gi * kConnMaxK;
  for (uint32_t base = wid * NG; base < cnt; base += nwaves * NG) {
    const uint32_t i = base + gi;
    const bool valid = i < cnt;
    const uint32_t ic = valid ? i : cnt - 1;
    const int64_t u = gld(list, ic);
    const uint64_t x = gld(info, ic);
    const DevSlot& sl = S[SLOT(u)];
    const bool build = valid && sl.conn_mode == CONN_BUILD;
    const int K = sl.conn_k;
    for (int t = gl; t < kConnMaxK; t += G) my[t] = 0;
    wave_sync();
    if (build) {
      const int64_t e0 = info_e0(x);
      const int d = info_d(x);
      for (int e = gl; e < d; e += G * B) {
        int32_t nb[B], w[B], t[B];
#pragma unroll
        for (int q = 0; q < B; ++q) {
          const int ee = e + q * G;
          const int64_t ec = e0 + (ee < d ? ee : d - 1);
          nb[q] = gld(sl.col, ec);
          w[q] = sl.ew ? gld(sl.ew, ec) : 1;
        }
// the blocks of the neighbours, from the byte copy when there is one
        if (sl.lab8) {
#pragma unroll
          for (int q = 0; q < B; ++q) t[q] = (int32_t)gld(sl.lab8, nb[q]);
        } else {
#pragma unroll
          for (int q = 0; q < B; ++q) t[q] = gld(sl.lab, nb[q]);
        }
#pragma unroll
        for (int q = 0; q < B; ++q)
          if (e + q * G < d && (uint32_t)t[q] < (uint32_t)K) atomicAdd(&my[t[q]], w[q]);
      }
    }
    wave_sync();
    if (build) {
      const int64_t r = (u - sl.nbase) * K;
      for (int t = gl; t < K; t += G) gst(sl.conn, r + t, my[t]);
    }
    wave_sync();
  }
}

template <bool ONE>
__device__ __forceinline__ void conn_build_hubs(const DevSlot* __restrict__ S, int ns, const int32_t* __restrict__ list,
                                                const HubLayout& L, uint32_t wid, uint32_t nwaves, int32_t* row) {
  constexpr int B = 4;
  const int lane = (int)lane_id();
  const uint32_t nchunks = L.totals[0];
  for (uint32_t c = wid; c < nchunks; c += nwaves) {
    const uint32_t h = L.chunk_hub[c];
    const int64_t u = gld(list, h);
    const DevSlot& sl = S[SLOT(u)];
    if (sl.conn_mode != CONN_BUILD) continue;
    const int K = sl.conn_k;
    const int64_t v = u - sl.nbase;
    const int64_t e0 = gld(sl.rp, v), d = gld(sl.rp, v + 1) - e0;
    const int64_t c0 = (int64_t)(c - L.chunk_off[h]) * kHubChunk;
    const int64_t c1 = c0 + kHubChunk < d ? c0 + kHubChunk : d;
    row[lane] = 0;
    wave_sync();
    for (int64_t e = c0 + lane; e < c1; e += kWave * B) {
      int32_t nb[B], w[B], t[B];
#pragma unroll
      for (int q = 0; q < B; ++q) {
        const int64_t ee = e + q * kWave;
        const int64_t ec = e0 + (ee < c1 ? ee : c1 - 1);
        nb[q] = gld(sl.col, ec);
        w[q] = sl.ew ? gld(sl.ew, ec) : 1;
      }
      if (sl.lab8) {
#pragma unroll
        for (int q = 0; q < B; ++q) t[q] = (int32_t)gld(sl.lab8, nb[q]);
      } else {
#pragma unroll
        for (int q = 0; q < B; ++q) t[q] = gld(sl.lab, nb[q]);
      }
#pragma unroll
      for (int q = 0; q < B; ++q)
        if (e + q * kWave < c1 && (uint32_t)t[q] < (uint32_t)K) atomicAdd(&row[t[q]], w[q]);
    }
    wave_sync();
    if (lane < K && row[lane]) conn_add(sl.conn, v * K + lane, row[lane]);
    wave_sync();
  }
}

// Rows of the hubs of CONN_BUILD slots cleared (their chunks add into them).
template <bool ONE>
__global__ void __launch_bounds__(256) k_conn_zero_hubs(const DevSlot* __restrict__ S, int ns,
                                                        const int32_t* __restrict__ list,
                                                        const uint32_t* __restrict__ cnt_ptr) {
  const uint32_t cnt = *cnt_ptr;
  const int lane = (int)lane_id();
  const uint32_t waves = gridDim.x * (blockDim.x / kWave);
  for (uint32_t i = blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave; i < cnt; i += waves) {
    const int64_t u = gld(list, i);
    const DevSlot& sl = S[SLOT(u)];
    if (sl.conn_mode != CONN_BUILD || lane >= sl.conn_k) continue;
    gst(sl.conn, (u - sl.nbase) * sl.conn_k + lane, 0);
  }
}

// Blocks [0, hblk) serve the hub chunks (when `hubs`; dispatched first, as
// they hold the most entries), blocks hblk + [b * nblk, (b + 1) * nblk) bin b
// (0-7).
template <bool ONE>
__global__ void __launch_bounds__(256) k_conn_build(const DevSlot* __restrict__ S, int ns,
                                                    const int32_t* __restrict__ bins,
                                                    const uint64_t* __restrict__ binfo, int64_t bin_cap,
                                                    const uint32_t* __restrict__ bin_cnt, uint32_t nblk,
                                                    uint32_t hblk, HubLayout L) {
  __shared__ int32_t rows[4][8 * kConnMaxK];
  const int w = threadIdx.x / kWave;
  if (blockIdx.x < hblk) {
    if (!*L.overflow) conn_build_hubs<ONE>(S, ns, bins + 8 * bin_cap, L, blockIdx.x * 4 + w, hblk * 4, rows[w]);
    return;
  }
  const uint32_t b = (blockIdx.x - hblk) / nblk, bid = (blockIdx.x - hblk) % nblk;
  const uint32_t wid = bid * 4 + w, nw = nblk * 4;
  const int32_t* list = bins + b * bin_cap;
  const uint64_t* info = binfo + b * bin_cap;
  const uint32_t cnt = bin_cnt[b];
  if (b == 0) conn_build_group<8, ONE>(S, ns, list, info, cnt, wid, nw, rows[w]);
  else if (b == 1) conn_build_group<16, ONE>(S, ns, list, info, cnt, wid, nw, rows[w]);
  else if (b == 2) conn_build_group<32, ONE>(S, ns, list, info, cnt, wid, nw, rows[w]);
  else conn_build_group<64, ONE>(S, ns, list, info, cnt, wid, nw, rows[w]);
}

// ---------------------------------------------------------------------------
// Rating from block connections: one thread per rated node of a slot that
// keeps them (CONN_RATE, or CONN_BUILD once k_conn_build has written the
// rows; nodes of other slots are rated from the bins).  The candidates are
// the blocks with conn(v, b) > 0; the choice is the same as from the
// neighbour labels.
// ---------------------------------------------------------------------------
template <bool ONE>
__global__ void __launch_bounds__(256) k_rate_cached(const DevSlot* __restrict__ S, int ns,
                                                     const int32_t* __restrict__ rated,
                                                     const uint32_t* __restrict__ rcnt) {
  // a group of G lanes per rated node: lane g reads the 16-byte pieces g,
  // g + G, ... of the node's row, so the rows of consecutive rated nodes are
  // read as consecutive bytes; a row whose column count is not a multiple
  // of 4 is scanned by the group's first lane
  constexpr int G = 8;
  const uint32_t cnt = *rcnt;
  const uint32_t lane = lane_id();
  const int g = (int)(lane & (G - 1));
  const uint32_t ngroups = gridDim.x * blockDim.x / G;
  const uint32_t first = (blockIdx.x * blockDim.x + threadIdx.x - lane) / G;  // the wave's first group
  for (uint32_t i0 = first; i0 < cnt; i0 += ngroups) {
    const uint32_t i = i0 + lane / G;
    const bool valid = i < cnt;
    const int64_t u = gld(rated, valid ? i : cnt - 1);
    const DevSlot& sl = S[SLOT(u)];
    // CONN_NONE slots are rated from the bins; CONN_BUILD rows were just built
    const bool act = valid && sl.conn_mode != CONN_NONE;
    const int64_t v = u - sl.nbase;
    const int K = sl.conn_k;
    const int32_t own = gld(sl.lab, v);
    const int64_t cv = gld(sl.nw, v);
    const int32_t* row = sl.conn + v * K;
    int32_t lo, hi;
    dir_interval(sl, own, lo, hi);
    const bool own_ok = own_allowed(sl, own);
    const int64_t conn_own = act && (uint32_t)own < (uint32_t)K ? gld(row, own) : 0;
    bool foreign = false;
    uint64_t best = 0;
    auto consider = [&](int t, int64_t c) {
      if (c <= 0 || t == own) return;
      foreign = true;
      if (t < lo || t > hi) return;
      const bool beats = !own_ok || c > conn_own || (c == conn_own && t < own);
      if (beats && gld(sl.W, t) + cv <= sl.cap) {
        const uint64_t k = pack_key(c, t);
        best = best > k ? best : k;
      }
    };
    if (act) {
      if ((K & 3) == 0) {
        // rows of a multiple of 4 columns are 16-byte aligned
        const int4* row4 = (const int4*)row;
        for (int t = 4 * g; t < K; t += 4 * G) {
          const int4 q = row4[t >> 2];
          consider(t, q.x);
          consider(t + 1, q.y);
          consider(t + 2, q.z);
          consider(t + 3, q.w);
        }
      } else if (g == 0) {
        for (int t = 0; t < K; ++t) consider(t, gld(row, t));
      }
    }
    // the group's best candidate (a maximum) and whether any lane saw a
    // foreign block
    int any = foreign ? 1 : 0;
    for (int off = 1; off < G; off <<= 1) {
      const uint32_t lo32 = __shfl_xor((uint32_t)best, off);
      const uint32_t hi32 = __shfl_xor((uint32_t)(best >> 32), off);
      const uint64_t o = ((uint64_t)hi32 << 32) | lo32;
      best = best > o ? best : o;
      any |= __shfl_xor(any, off);
    }
    if (act && g == 0) {
      if (own_ok) {
        const uint64_t ok = pack_key(conn_own, own);
        best = best > ok ? best : ok;
      }
      gst(sl.desire, v, best ? key_label(best) : own);
      if (any) gst(sl.flag_next, v, (uint8_t)1);
    }
  }
}

// ---------------------------------------------------------------------------
// Host-side launchers.
// ---------------------------------------------------------------------------
static inline unsigned grid_for(int64_t items, int per_block, unsigned cap) {
  int64_t g = (items + per_block - 1) / per_block;
  if (g < 1) g = 1;
  return (unsigned)(g < cap ? g : cap);
}

// Launch the single-slot instantiation when one graph takes part.
#define LAUNCH(kern, grid, block, ...)                                                     \
  do {                                                                                     \
    if (ns == 1) hipLaunchKernelGGL(kern<true>, dim3(grid), dim3(block), 0, st, __VA_ARGS__); \
    else hipLaunchKernelGGL(kern<false>, dim3(grid), dim3(block), 0, st, __VA_ARGS__);       \
  } while (0)

int64_t bin_tiles(int64_t n) { return (n + kBinTile - 1) / kBinTile; }

// Start of a round with at most kArgSlots slots: the slot descriptors travel
// as kernel arguments and one launch stores them and zeroes the round's
// counters (instead of a host-to-device copy and a fill).
constexpr int kArgSlots = 8;
struct SlotArgs {
  DevSlot s[kArgSlots];
};

__global__ void __launch_bounds__(256) k_round_begin(const SlotArgs a, int ns, DevSlot* __restrict__ S,
                                                     uint32_t* __restrict__ zero, int nzero) {
  static_assert(sizeof(DevSlot) % 8 == 0, "slot descriptor size");
  constexpr int W = (int)(sizeof(DevSlot) / 8);
  uint64_t* dst = reinterpret_cast<uint64_t*>(S);
  for (int i = threadIdx.x; i < ns * W; i += blockDim.x) {
    uint64_t x;
    __builtin_memcpy(&x, reinterpret_cast<const char*>(&a.s[i / W]) + (i % W) * 8, 8);
    dst[i] = x;
  }
  for (int i = threadIdx.x; i < nzero; i += blockDim.x) zero[i] = 0;
}

int round_begin(const DevSlot* host_slots, int ns, DevSlot* S, uint32_t* zero, int64_t nzero, hipStream_t st) {
  if (ns <= kArgSlots && nzero <= (int64_t)1 << 20) {
    SlotArgs a;
    std::memcpy(a.s, host_slots, (size_t)ns * sizeof(DevSlot));
    hipLaunchKernelGGL(k_round_begin, dim3(1), dim3(256), 0, st, a, ns, S, zero, (int)nzero);
    SCLAP_HIP(hipGetLastError());
    return SCLAP_OK;
  }
  SCLAP_HIP(hipMemcpyAsync(S, host_slots, (size_t)ns * sizeof(DevSlot), hipMemcpyHostToDevice, st));
  return fill_u32(zero, nzero, 0, st);
}

size_t bin_scratch_bytes(int64_t T) {
  const size_t rows = (size_t)kBinRows * (size_t)T + 1;
  return rows * 4 * 2 + rows * 8 * 2 + 256 + std::max(prim_exscan_i32_bytes(rows), prim_exscan_i64_bytes(rows));
}

int launch_bin(const DevSlot* S, int ns, int64_t T, int32_t* bins, uint64_t* binfo, int64_t bin_cap,
               uint32_t* bin_cnt, unsigned long long* bin_visits, int32_t* rated, uint32_t* rated_cnt,
               void* scratch, size_t scratch_bytes, hipStream_t st) {
  const size_t rows = (size_t)kBinRows * (size_t)T + 1;
  char* p = (char*)scratch;
  uint32_t* cnt = (uint32_t*)p;
  uint32_t* off = cnt + rows;
  int64_t* vis = (int64_t*)(((uintptr_t)(off + rows) + 255) & ~(uintptr_t)255);
  int64_t* voff = vis + rows;
  void* tmp = voff + rows;
  const size_t tmp_bytes = scratch_bytes - (size_t)((char*)tmp - p);
  if (T > 0) {
    const unsigned G = (unsigned)std::min<int64_t>(T, 4096);
    // the entry after the last tile is the total of the scans
    LAUNCH(k_bin_count, G, kBinTile, S, ns, T, cnt, vis);
    if ((int64_t)rows <= kScan1Rows) {
      hipLaunchKernelGGL(k_bin_scan1, dim3(1), dim3(kScan1Threads), 0, st, cnt, vis, (int64_t)rows, off, voff, S, ns,
                         T, bin_cnt, bin_visits, rated_cnt);
    } else {
      SCLAP_TRY(prim_exscan_i32(tmp, tmp_bytes, (const int32_t*)cnt, (int32_t*)off, rows, st));
      SCLAP_TRY(prim_exscan_i64(tmp, tmp_bytes, vis, voff, rows, st));
      hipLaunchKernelGGL(k_bin_totals, dim3(1), dim3(256), 0, st, S, ns, T, off, voff, bin_cnt, bin_visits,
                         rated_cnt);
    }
    LAUNCH(k_bin_write, G, kBinTile, S, ns, T, off, bins, binfo, bin_cap, rated);
  } else {
    SCLAP_TRY(fill_u32(off, 1, 0, st));
    SCLAP_TRY(fill_i64(voff, 1, 0, st));
    hipLaunchKernelGGL(k_bin_totals, dim3(1), dim3(256), 0, st, S, ns, T, off, voff, bin_cnt, bin_visits, rated_cnt);
  }
  SCLAP_HIP(hipGetLastError());
  return SCLAP_OK;
}

int launch_rate(const DevSlot* S, int ns, const int32_t* bins, const uint64_t* binfo, int64_t bin_cap,
                const uint32_t* bin_cnt, const HubLayout& hub, int64_t n_hint, bool hubs, bool unit_weights,
                int64_t max_deg, int32_t lo5, int32_t lo7, bool hubs_ident, bool hub_layout_kept, hipStream_t st,
                hipEvent_t* evs, unsigned* groups) {
  const unsigned G = grid_for(n_hint, 64, 2048);
  // bins 5-6 hold degrees above lo5, bin 7 degrees above lo7 (the smallest
  // such bounds over the slots)
  if (groups) *groups = 1u | (max_deg > 32 ? 2u : 0u) | (max_deg > lo5 ? 4u : 0u) | (max_deg > lo7 ? 8u : 0u) |
                        (hubs ? 16u : 0u);
  auto rec = [&](int i) {
    if (evs) (void)hipEventRecord(evs[i], st);
  };
  rec(0);
  const int uw = unit_weights ? 1 : 0;
  LAUNCH(k_rate_tiny, 2 * G, 256, S, ns, bins, binfo, bin_cap, bin_cnt, G, uw);
  if (max_deg > 16) LAUNCH(k_rate_b32, G, 256, S, ns, bins + 2 * bin_cap, binfo + 2 * bin_cap, bin_cnt + 2, uw);
  rec(1);
  if (max_deg > 32) LAUNCH(k_rate_small, 2 * G, 256, S, ns, bins, binfo, bin_cap, bin_cnt, G);
  rec(2);
  if (max_deg > lo5) LAUNCH(k_rate_mid, 2 * G, 256, S, ns, bins, binfo, bin_cap, bin_cnt, G);
  rec(3);
  if (max_deg > lo7) LAUNCH(k_rate_large, G, 512, S, ns, bins + 7 * bin_cap, binfo + 7 * bin_cap, bin_cnt + 7);
  rec(4);
  if (hubs) {
    const int32_t* hb = bins + 8 * bin_cap;
    const uint32_t* hc = bin_cnt + 8;
    if (hub_layout_kept) hipLaunchKernelGGL(k_hub_reuse, dim3(1), dim3(1), 0, st, hub);
    else LAUNCH(k_hub_prep, 1, 1024, S, ns, hb, hc, hub);
    LAUNCH(k_hub_chunk, G, kHubChunkThreads, S, ns, hb, hub);
    if (!hubs_ident) {
      // (first clustering rounds stage no pairs: their chunks went to the hubs' best directly)
      LAUNCH(k_hub_part, G, 256, S, ns, hb, hub);
    }
    LAUNCH(k_hub_final, 64, 256, S, ns, hb, hc, hub);
  }
  rec(5);
  SCLAP_HIP(hipGetLastError());
  return SCLAP_OK;
}

size_t tile_adm_bytes(int64_t T, int kmax) {
  const size_t n = (size_t)kmax * (size_t)T;
  return n * 8 * 3 + n * 4 + (size_t)T * 8 + 1024 + prim_scan_by_key_bytes(std::max<size_t>(n, 1));
}

int launch_tile_admission(const DevSlot* S, int ns, const int32_t* rated, const uint32_t* roff, int64_t T, int kmax,
                          int64_t max_slot_tiles, void* scratch, size_t scratch_bytes, int32_t* mold,
                          hipStream_t st) {
  if (T == 0) return SCLAP_OK;
  const size_t n = (size_t)kmax * (size_t)T;
  TileAdm A{};
  A.roff = roff;
  A.T = T;
  A.kmax = kmax;
  char* p = (char*)scratch;
  A.tsum = (int64_t*)p;
  A.tpre = A.tsum + n;
  A.dW = A.tpre + n;
  A.tmoved = A.dW + n;
  A.keys = (uint32_t*)(A.tmoved + T);
  void* tmp = (void*)(((uintptr_t)(A.keys + n) + 255) & ~(uintptr_t)255);
  const size_t tmp_bytes = scratch_bytes - (size_t)((char*)tmp - p);
  const unsigned G = (unsigned)std::min<int64_t>(T, 4096);
  LAUNCH(k_ta_sums, G, kBinTile, S, ns, rated, A);
  if (max_slot_tiles <= kTaScanTiles) {
    hipLaunchKernelGGL(k_ta_scan_small, dim3((unsigned)(ns * kmax)), dim3(1024), 0, st, S, ns, A);
  } else {
    SCLAP_TRY(prim_scan_by_key(tmp, tmp_bytes, A.keys, A.tsum, A.tpre, n, st));
  }
  LAUNCH(k_ta_admit, G, kBinTile, S, ns, rated, A, mold);
  hipLaunchKernelGGL(k_ta_reduce, dim3((unsigned)(ns * (kmax + 1))), dim3(256), 0, st, S, ns, A);
  SCLAP_HIP(hipGetLastError());
  return SCLAP_OK;
}

const uint32_t* bin_rated_offsets(void* scratch, int64_t T) {
  return (const uint32_t*)scratch + (size_t)kBinRows * (size_t)T + 1 + (size_t)kBins * (size_t)T;
}

int launch_hub_prep(const DevSlot* S, int ns, const int32_t* bins, int64_t bin_cap, const uint32_t* bin_cnt,
                    const HubLayout& hub, hipStream_t st) {
  LAUNCH(k_hub_prep, 1, 1024, S, ns, bins + 8 * bin_cap, bin_cnt + 8, hub);
  SCLAP_HIP(hipGetLastError());
  return SCLAP_OK;
}

int launch_conn_build(const DevSlot* S, int ns, const int32_t* bins, const uint64_t* binfo, int64_t bin_cap,
                      const uint32_t* bin_cnt, const HubLayout& hub, int64_t n_hint, bool hubs, hipStream_t st) {
  const unsigned G = grid_for(n_hint, 256, 1024);
  // the hub chunks get a full grid of their own (2048 entries per wave)
  const unsigned H = hubs ? 2048u : 0u;
  if (hubs) LAUNCH(k_conn_zero_hubs, 64, 256, S, ns, bins + 8 * bin_cap, bin_cnt + 8);
  LAUNCH(k_conn_build, 8 * G + H, 256, S, ns, bins, binfo, bin_cap, bin_cnt, G, H, hub);
  SCLAP_HIP(hipGetLastError());
  return SCLAP_OK;
}

int launch_rate_cached(const DevSlot* S, int ns, int64_t N, const int32_t* rated, const uint32_t* rcnt,
                       hipStream_t st) {
  LAUNCH(k_rate_cached, grid_for(N, 32, 8192), 256, S, ns, rated, rcnt);
  SCLAP_HIP(hipGetLastError());
  return SCLAP_OK;
}

int launch_incoming_decide(const DevSlot* S, int ns, int64_t N, int64_t Lt, const int32_t* rated,
                           const uint32_t* rcnt, uint64_t* ckeys, uint32_t* ccnt, int node_bits, hipStream_t st) {
  LAUNCH(k_incoming, grid_for(N, kAggNodes, kAggGrid), 256, S, ns, rated, rcnt);
  LAUNCH(k_decide, grid_for(N, 256, kAggGrid), 256, S, ns, rated, rcnt, ckeys, ccnt, node_bits);
  LAUNCH(k_fold, grid_for(Lt, 256, 4096), 256, S, ns, Lt);
  SCLAP_HIP(hipGetLastError());
  return SCLAP_OK;
}

int launch_contended_split(const DevSlot* S, int ns, const uint64_t* keys, uint32_t cnt, int node_bits,
                           uint32_t* tkey, int64_t* wv, hipStream_t st) {
  if (cnt == 0) return SCLAP_OK;
  LAUNCH(k_contended_split, (cnt + 255) / 256, 256, S, ns, keys, cnt, node_bits, tkey, wv);
  SCLAP_HIP(hipGetLastError());
  return SCLAP_OK;
}

int launch_contended_mark(const DevSlot* S, int ns, const uint64_t* keys, uint32_t cnt, int node_bits,
                          const int64_t* prefix, hipStream_t st) {
  if (cnt == 0) return SCLAP_OK;
  LAUNCH(k_contended_mark, (cnt + 255) / 256, 256, S, ns, keys, cnt, node_bits, prefix);
  SCLAP_HIP(hipGetLastError());
  return SCLAP_OK;
}

int launch_contended_add(const DevSlot* S, int ns, const uint64_t* keys, uint32_t cnt, int node_bits,
                         const int64_t* prefix, hipStream_t st) {
  if (cnt == 0) return SCLAP_OK;
  LAUNCH(k_contended_add, (cnt + 255) / 256, 256, S, ns, keys, cnt, node_bits, prefix);
  SCLAP_HIP(hipGetLastError());
  return SCLAP_OK;
}

int launch_contended_small(const DevSlot* S, int ns, const uint64_t* keys, const uint32_t* ccnt, int node_bits,
                           uint32_t* big_flag, hipStream_t st) {
  LAUNCH(k_contended_small, 1, 1024, S, ns, keys, ccnt, node_bits, big_flag);
  SCLAP_HIP(hipGetLastError());
  return SCLAP_OK;
}

int launch_apply(const DevSlot* S, int ns, int64_t N, const int32_t* rated, const uint32_t* rcnt, int32_t* mold,
                 int32_t* big, uint32_t* big_cnt, uint32_t* huge_cnt, int64_t big_cap, bool run_apply,
                 bool any_refine, const uint32_t* skip, hipStream_t st, hipEvent_t* mark_ev,
                 unsigned long long* mark_entries) {
  if (run_apply) LAUNCH(k_apply, grid_for(N, kAggNodes, kAggGrid), 256, S, ns, rated, rcnt, mold, skip);
  if (any_refine) {
    if (mark_ev) SCLAP_HIP(hipEventRecord(mark_ev[0], st));
    LAUNCH(k_mark, grid_for(N, 256 * kWave / 4, 2048), 256, S, ns, rated, rcnt, mold, big, big_cnt, huge_cnt,
           big_cap, skip, mark_entries);
    if (big) LAUNCH(k_mark_big, 1024, 256, S, ns, rated, mold, big, big_cnt, huge_cnt, big_cap, skip);
    if (mark_ev) SCLAP_HIP(hipEventRecord(mark_ev[1], st));
  }
  SCLAP_HIP(hipGetLastError());
  return SCLAP_OK;
}

}  // namespace sclap
