// lp_kernels.hip -- one synchronous size-constrained label propagation round
// (Section 3.1) over a set of graphs ("slots"), as gfx950 kernels:
//
//   bin      nodes to rate -> four degree bins, edge visits per slot
//   rate     per-node neighbour-cluster rating: conn(v, t) = sum of w(v, u)
//            over neighbours u with label t; candidates = own label and
//            neighbour labels in the allowed direction; eligible if
//            W(t) + c(v) <= cap; argmax with ties to the smallest label.
//              8 lanes per node (deg <= 8), one wave per node (deg <= 64),
//              one workgroup with an LDS hash table (deg <= 4096), several
//              workgroups with a global hash table (hubs).
//   admit    movers into a target are admitted in increasing node id while
//            W(t) + inclusive prefix of their weights <= cap: targets whose
//            total incoming weight fits admit everyone; the others sort
//            their movers by (target, node) and scan.
//   apply    labels, label weights (integer atomics), moved counts, and in
//            refinement the rated set of the next round.
//
// Every result is a pure function of the previous round's state: integer
// atomics only ever sum or take maxima, so the order of execution does not
// change any value.
#include <hip/hip_runtime.h>

#include "common.h"
#include "lp.h"

namespace sclap {

__device__ __forceinline__ uint32_t lane_id() { return __lane_id(); }

// Wave-aggregated append: returns this lane's slot (valid if pred).
__device__ __forceinline__ uint32_t wave_append(uint32_t* counter, bool pred) {
  const uint64_t mask = __ballot(pred);
  if (mask == 0) return 0;
  const int leader = __ffsll((unsigned long long)mask) - 1;
  uint32_t base = 0;
  if ((int)lane_id() == leader) base = atomicAdd(counter, (uint32_t)__popcll(mask));
  base = __shfl(base, leader);
  return base + (uint32_t)__popcll(mask & ((1ull << lane_id()) - 1ull));
}

// Add `val` to S[s].ctr[which], aggregated over the wave when the slot is
// the same for all lanes.
__device__ __forceinline__ void wave_count(const DevSlot* __restrict__ S, int s, int which, int64_t val) {
  const int s0 = __shfl(s, 0);
  if (__all(s == s0)) {
    int64_t sum = val;
    for (int off = 32; off > 0; off >>= 1) sum += __shfl_xor(sum, off);
    if (lane_id() == 0 && sum != 0) atomicAdd((unsigned long long*)&S[s0].ctr[which], (unsigned long long)sum);
  } else if (val != 0) {
    atomicAdd((unsigned long long*)&S[s].ctr[which], (unsigned long long)val);
  }
}

__device__ __forceinline__ int bin_of(int64_t d) {
  return d <= kBinG8 ? 0 : d <= kBinG64 ? 1 : d <= kBinBlock ? 2 : 3;
}

// ---------------------------------------------------------------------------
// Binning: every node of an active slot with degree > 0 (and, in refinement
// after round 1, in the rated set) is appended to its degree bin.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_bin(const DevSlot* __restrict__ S, int ns, int64_t N,
                                             int32_t* __restrict__ bins, int64_t bin_cap,
                                             uint32_t* __restrict__ bin_cnt) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  // all lanes iterate the same number of times (convergent wave_append)
  for (int64_t base = (int64_t)blockIdx.x * blockDim.x; base < N; base += stride) {
    const int64_t u = base + threadIdx.x;
    bool take = false;
    int b = 0;
    int s = 0;
    int64_t d = 0;
    if (u < N) {
      s = slot_of(S, ns, u);
      const DevSlot& sl = S[s];
      const int64_t v = u - sl.nbase;
      if (sl.round > 0 && (!sl.use_flags || sl.flag_cur[v])) {
        d = sl.rp[v + 1] - sl.rp[v];
        take = d > 0;
        b = bin_of(d);
      }
    }
    wave_count(S, s, CTR_VISITS, take ? d : 0);
#pragma unroll
    for (int j = 0; j < kBins; ++j) {
      const uint32_t pos = wave_append(&bin_cnt[j], take && b == j);
      if (take && b == j) bins[j * bin_cap + pos] = (int32_t)u;
    }
  }
}

// ---------------------------------------------------------------------------
// Rating, G lanes per node (degree <= G).
// ---------------------------------------------------------------------------
template <int G>
__global__ void __launch_bounds__(256) k_rate_group(const DevSlot* __restrict__ S, int ns,
                                                    const int32_t* __restrict__ list,
                                                    const uint32_t* __restrict__ cnt_ptr) {
  const uint32_t cnt = *cnt_ptr;
  const int lane = (int)lane_id();
  const int gl = lane & (G - 1);
  const int gbase = lane & ~(G - 1);
  const uint32_t per_block = blockDim.x / G;
  for (uint32_t base = blockIdx.x * per_block; base < cnt; base += gridDim.x * per_block) {
    const uint32_t i = base + threadIdx.x / G;
    const bool valid = i < cnt;
    const int64_t u = valid ? list[i] : 0;
    const int s = slot_of(S, ns, u);
    const DevSlot& sl = S[s];
    const int64_t v = u - sl.nbase;
    int64_t e0 = 0;
    int d = 0;
    int32_t own = -1;
    if (valid) {
      e0 = sl.rp[v];
      d = (int)(sl.rp[v + 1] - e0);
      own = sl.lab[v];
    }
    int32_t t = -1, w = 0;
    if (gl < d) {
      t = sl.lab[sl.col[e0 + gl]];
      w = sl.ew ? sl.ew[e0 + gl] : 1;
    }
    const bool foreign = t >= 0 && t != own;
    const uint64_t fmask = __ballot(foreign);
    const bool boundary = ((fmask >> gbase) & (G == 64 ? ~0ull : ((1ull << G) - 1ull))) != 0;
    int32_t te = t;
    if (foreign && sl.dir_rule) {
      const bool odd = sl.round & 1;
      if (odd ? t > own : t < own) te = -1;
    }
    int64_t conn = 0, conn_own = 0;
    bool leader = te >= 0;
#pragma unroll
    for (int j = 0; j < G; ++j) {
      const int32_t tj = __shfl(te, gbase + j);
      const int32_t wj = __shfl(w, gbase + j);
      if (tj == te) {
        conn += wj;
        if (j < gl) leader = false;
      }
      if (tj == own) conn_own += wj;
    }
    uint64_t key = 0;
    if (valid) {
      const int64_t cv = sl.nw[v];
      const bool own_ok = !(sl.mode == MODE_REFINE && sl.W[own] > sl.cap);
      if (leader && te != own) {
        const bool beats = !own_ok || conn > conn_own || (conn == conn_own && te < own);
        if (beats && sl.W[te] + cv <= sl.cap) key = pack_key(conn, te);
      }
      if (own_ok) {
        const uint64_t ok = pack_key(conn_own, own);
        key = key > ok ? key : ok;
      }
    }
#pragma unroll
    for (int off = G / 2; off > 0; off >>= 1) {
      const uint64_t o = __shfl_xor(key, off);
      key = key > o ? key : o;
    }
    if (valid && gl == 0) {
      sl.desire[v] = key ? key_label(key) : own;
      if (sl.mode == MODE_REFINE && boundary) sl.flag_next[v] = 1;
    }
  }
}

// Block-wide reductions for 256 threads.
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

// Insert (t, w) into an open-addressing table (keys -1 = empty).
__device__ __forceinline__ void table_add(int32_t* keys, int32_t* vals, uint32_t mask, int32_t t, int32_t w) {
  uint32_t h = hash32((uint32_t)t) & mask;
  for (;;) {
    const int32_t prev = atomicCAS(&keys[h], -1, t);
    if (prev == -1 || prev == t) {
      atomicAdd(&vals[h], w);
      return;
    }
    h = (h + 1) & mask;
  }
}

// ---------------------------------------------------------------------------
// Rating, one workgroup per node (degree <= kBinBlock), LDS hash table.
// ---------------------------------------------------------------------------
constexpr int kBlockTable = 2 * kBinBlock;

__global__ void __launch_bounds__(256) k_rate_block(const DevSlot* __restrict__ S, int ns,
                                                    const int32_t* __restrict__ list,
                                                    const uint32_t* __restrict__ cnt_ptr) {
  __shared__ int32_t keys[kBlockTable];
  __shared__ int32_t vals[kBlockTable];
  __shared__ uint64_t red64[4];
  __shared__ int64_t redi[4];
  __shared__ int redo[4];
  const uint32_t cnt = *cnt_ptr;
  for (uint32_t i = blockIdx.x; i < cnt; i += gridDim.x) {
    const int64_t u = list[i];
    const int s = slot_of(S, ns, u);
    const DevSlot& sl = S[s];
    const int64_t v = u - sl.nbase;
    const int64_t e0 = sl.rp[v];
    const int d = (int)(sl.rp[v + 1] - e0);
    const int32_t own = sl.lab[v];
    int64_t distinct = d < sl.nlabels ? d : sl.nlabels;
    uint32_t tsz = 64;
    while (tsz < 2 * distinct) tsz <<= 1;
    const uint32_t mask = tsz - 1;
    for (uint32_t j = threadIdx.x; j < tsz; j += blockDim.x) {
      keys[j] = -1;
      vals[j] = 0;
    }
    __syncthreads();
    const bool odd = sl.round & 1;
    int64_t my_own = 0;
    int foreign = 0;
    for (int e = threadIdx.x; e < d; e += blockDim.x) {
      const int32_t t = sl.lab[sl.col[e0 + e]];
      const int32_t w = sl.ew ? sl.ew[e0 + e] : 1;
      if (t == own) {
        my_own += w;
        continue;
      }
      foreign = 1;
      if (sl.dir_rule && (odd ? t > own : t < own)) continue;
      table_add(keys, vals, mask, t, w);
    }
    const int64_t conn_own = block_reduce(my_own, redi, OpAdd64());
    const int boundary = block_reduce(foreign, redo, OpOr());
    const int64_t cv = sl.nw[v];
    const bool own_ok = !(sl.mode == MODE_REFINE && sl.W[own] > sl.cap);
    uint64_t best = 0;
    for (uint32_t j = threadIdx.x; j < tsz; j += blockDim.x) {
      const int32_t t = keys[j];
      if (t < 0) continue;
      const int64_t c = vals[j];
      const bool beats = !own_ok || c > conn_own || (c == conn_own && t < own);
      if (beats && sl.W[t] + cv <= sl.cap) {
        const uint64_t k = pack_key(c, t);
        best = best > k ? best : k;
      }
    }
    best = block_reduce(best, red64, OpMax64());
    if (threadIdx.x == 0) {
      if (own_ok) {
        const uint64_t ok = pack_key(conn_own, own);
        best = best > ok ? best : ok;
      }
      sl.desire[v] = best ? key_label(best) : own;
      if (sl.mode == MODE_REFINE && boundary) sl.flag_next[v] = 1;
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// Rating of hubs (degree > kBinBlock): chunks of kHubChunk entries per
// workgroup, aggregated in LDS and flushed into a per-hub global table.
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint32_t hub_table_size(int64_t d, int64_t nlabels) {
  const int64_t distinct = d < nlabels ? d : nlabels;
  uint32_t tsz = 64;
  while (tsz < 2 * distinct) tsz <<= 1;
  return tsz;
}

// One workgroup: exclusive offsets of chunk counts and table sizes.
__global__ void __launch_bounds__(1024) k_hub_prep(const DevSlot* __restrict__ S, int ns,
                                                   const int32_t* __restrict__ list,
                                                   const uint32_t* __restrict__ cnt_ptr,
                                                   uint32_t* __restrict__ chunk_off, int64_t* __restrict__ tab_off,
                                                   uint32_t* __restrict__ totals, int64_t tab_cap,
                                                   uint32_t* __restrict__ overflow) {
  __shared__ uint32_t sc[1024];
  __shared__ int64_t st[1024];
  __shared__ uint32_t carry_c;
  __shared__ int64_t carry_t;
  const uint32_t cnt = *cnt_ptr;
  if (threadIdx.x == 0) {
    carry_c = 0;
    carry_t = 0;
  }
  __syncthreads();
  for (uint32_t base = 0; base < cnt; base += blockDim.x) {
    const uint32_t i = base + threadIdx.x;
    uint32_t nc = 0;
    int64_t tz = 0;
    if (i < cnt) {
      const int64_t u = list[i];
      const DevSlot& sl = S[slot_of(S, ns, u)];
      const int64_t v = u - sl.nbase;
      const int64_t d = sl.rp[v + 1] - sl.rp[v];
      nc = (uint32_t)((d + kHubChunk - 1) / kHubChunk);
      tz = hub_table_size(d, sl.nlabels);
    }
    sc[threadIdx.x] = nc;
    st[threadIdx.x] = tz;
    __syncthreads();
    for (uint32_t off = 1; off < blockDim.x; off <<= 1) {  // inclusive Hillis-Steele
      uint32_t a = threadIdx.x >= off ? sc[threadIdx.x - off] : 0;
      int64_t b = threadIdx.x >= off ? st[threadIdx.x - off] : 0;
      __syncthreads();
      sc[threadIdx.x] += a;
      st[threadIdx.x] += b;
      __syncthreads();
    }
    if (i < cnt) {
      chunk_off[i] = carry_c + sc[threadIdx.x] - nc;
      tab_off[i] = carry_t + st[threadIdx.x] - tz;
    }
    __syncthreads();
    if (threadIdx.x == blockDim.x - 1) {
      carry_c += sc[threadIdx.x];
      carry_t += st[threadIdx.x];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    totals[0] = carry_c;
    chunk_off[cnt] = carry_c;
    if (carry_t > tab_cap) *overflow = 1;
  }
}

constexpr int kHubLds = 2 * kHubChunk;

__global__ void __launch_bounds__(256) k_hub_chunk(const DevSlot* __restrict__ S, int ns,
                                                   const int32_t* __restrict__ list,
                                                   const uint32_t* __restrict__ cnt_ptr,
                                                   const uint32_t* __restrict__ chunk_off,
                                                   const int64_t* __restrict__ tab_off,
                                                   const uint32_t* __restrict__ totals,
                                                   int32_t* __restrict__ gkeys, int32_t* __restrict__ gvals,
                                                   int64_t* __restrict__ hub_own,
                                                   const uint32_t* __restrict__ overflow) {
  __shared__ int32_t keys[kHubLds];
  __shared__ int32_t vals[kHubLds];
  __shared__ int64_t redi[4];
  __shared__ int redo[4];
  if (*overflow) return;
  const uint32_t cnt = *cnt_ptr;
  const uint32_t nchunks = totals[0];
  for (uint32_t c = blockIdx.x; c < nchunks; c += gridDim.x) {
    // hub i with chunk_off[i] <= c < chunk_off[i + 1]
    uint32_t lo = 0, hi = cnt - 1;
    while (lo < hi) {
      const uint32_t mid = (lo + hi + 1) >> 1;
      if (chunk_off[mid] <= c) lo = mid;
      else hi = mid - 1;
    }
    const uint32_t i = lo;
    const int64_t u = list[i];
    const DevSlot& sl = S[slot_of(S, ns, u)];
    const int64_t v = u - sl.nbase;
    const int64_t row0 = sl.rp[v];
    const int64_t d = sl.rp[v + 1] - row0;
    const int64_t e_begin = (int64_t)(c - chunk_off[i]) * kHubChunk;
    const int64_t e_end = e_begin + kHubChunk < d ? e_begin + kHubChunk : d;
    const int32_t own = sl.lab[v];
    for (int j = threadIdx.x; j < kHubLds; j += blockDim.x) {
      keys[j] = -1;
      vals[j] = 0;
    }
    __syncthreads();
    const bool odd = sl.round & 1;
    int64_t my_own = 0;
    int foreign = 0;
    for (int64_t e = e_begin + threadIdx.x; e < e_end; e += blockDim.x) {
      const int32_t t = sl.lab[sl.col[row0 + e]];
      const int32_t w = sl.ew ? sl.ew[row0 + e] : 1;
      if (t == own) {
        my_own += w;
        continue;
      }
      foreign = 1;
      if (sl.dir_rule && (odd ? t > own : t < own)) continue;
      table_add(keys, vals, kHubLds - 1, t, w);
    }
    const int64_t co = block_reduce(my_own, redi, OpAdd64());
    const int boundary = block_reduce(foreign, redo, OpOr());
    if (threadIdx.x == 0) {
      if (co) atomicAdd((unsigned long long*)&hub_own[i], (unsigned long long)co);
      if (sl.mode == MODE_REFINE && boundary) sl.flag_next[v] = 1;
    }
    const uint32_t gmask = hub_table_size(d, sl.nlabels) - 1;
    int32_t* gk = gkeys + tab_off[i];
    int32_t* gv = gvals + tab_off[i];
    for (int j = threadIdx.x; j < kHubLds; j += blockDim.x) {
      const int32_t t = keys[j];
      if (t >= 0) table_add(gk, gv, gmask, t, vals[j]);
    }
    __syncthreads();
  }
}

__global__ void __launch_bounds__(256) k_hub_final(const DevSlot* __restrict__ S, int ns,
                                                   const int32_t* __restrict__ list,
                                                   const uint32_t* __restrict__ cnt_ptr,
                                                   const int64_t* __restrict__ tab_off,
                                                   int32_t* __restrict__ gkeys, int32_t* __restrict__ gvals,
                                                   int64_t* __restrict__ hub_own,
                                                   const uint32_t* __restrict__ overflow) {
  __shared__ uint64_t red64[4];
  if (*overflow) return;
  const uint32_t cnt = *cnt_ptr;
  for (uint32_t i = blockIdx.x; i < cnt; i += gridDim.x) {
    const int64_t u = list[i];
    const DevSlot& sl = S[slot_of(S, ns, u)];
    const int64_t v = u - sl.nbase;
    const int64_t d = sl.rp[v + 1] - sl.rp[v];
    const int32_t own = sl.lab[v];
    const int64_t conn_own = hub_own[i];
    const int64_t cv = sl.nw[v];
    const bool own_ok = !(sl.mode == MODE_REFINE && sl.W[own] > sl.cap);
    const uint32_t tsz = hub_table_size(d, sl.nlabels);
    int32_t* gk = gkeys + tab_off[i];
    int32_t* gv = gvals + tab_off[i];
    uint64_t best = 0;
    for (uint32_t j = threadIdx.x; j < tsz; j += blockDim.x) {
      const int32_t t = gk[j];
      if (t < 0) continue;
      const int64_t c = gv[j];
      gk[j] = -1;
      gv[j] = 0;
      const bool beats = !own_ok || c > conn_own || (c == conn_own && t < own);
      if (beats && sl.W[t] + cv <= sl.cap) {
        const uint64_t k = pack_key(c, t);
        best = best > k ? best : k;
      }
    }
    best = block_reduce(best, red64, OpMax64());
    if (threadIdx.x == 0) {
      if (own_ok) {
        const uint64_t ok = pack_key(conn_own, own);
        best = best > ok ? best : ok;
      }
      sl.desire[v] = best ? key_label(best) : own;
      hub_own[i] = 0;
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// Admission.
// ---------------------------------------------------------------------------

// inc(t) += c(v) for every mover v -> t.
__global__ void __launch_bounds__(256) k_incoming(const DevSlot* __restrict__ S, int ns, int64_t N) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; u < N; u += stride) {
    const int s = slot_of(S, ns, u);
    const DevSlot& sl = S[s];
    if (sl.round == 0) continue;
    const int64_t v = u - sl.nbase;
    const int32_t t = sl.desire[v];
    if (t != sl.lab[v]) atomicAdd((unsigned long long*)&sl.inc[t], (unsigned long long)sl.nw[v]);
  }
}

// Movers into targets whose whole incoming weight fits are admitted; the
// others are appended as (target, node) keys for the exact path.
__global__ void __launch_bounds__(256) k_decide(const DevSlot* __restrict__ S, int ns, int64_t N,
                                                uint64_t* __restrict__ ckeys, uint32_t* __restrict__ ccnt,
                                                int node_bits) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t base = (int64_t)blockIdx.x * blockDim.x; base < N; base += stride) {
    const int64_t u = base + threadIdx.x;
    bool contended = false;
    uint64_t key = 0;
    int s = 0;
    bool mover = false;
    if (u < N) {
      s = slot_of(S, ns, u);
      const DevSlot& sl = S[s];
      if (sl.round > 0) {
        const int64_t v = u - sl.nbase;
        const int32_t t = sl.desire[v];
        if (t != sl.lab[v]) {
          mover = true;
          if (sl.W[t] + sl.inc[t] <= sl.cap) {
            sl.adm[v] = 1;
          } else {
            sl.adm[v] = 0;
            contended = true;
            key = ((uint64_t)(sl.lbase + t) << node_bits) | (uint64_t)u;
          }
        }
      }
    }
    wave_count(S, s, CTR_MOVERS, mover ? 1 : 0);
    const uint32_t pos = wave_append(ccnt, contended);
    if (contended) ckeys[pos] = key;
  }
}

// For sorted contended keys: segment key (target) and weight of each entry.
__global__ void __launch_bounds__(256) k_contended_split(const DevSlot* __restrict__ S, int ns,
                                                         const uint64_t* __restrict__ keys, uint32_t cnt,
                                                         int node_bits, uint32_t* __restrict__ tkey,
                                                         int64_t* __restrict__ wv) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= cnt) return;
  const uint64_t k = keys[i];
  const int64_t u = (int64_t)(k & ((1ull << node_bits) - 1ull));
  const DevSlot& sl = S[slot_of(S, ns, u)];
  tkey[i] = (uint32_t)(k >> node_bits);
  wv[i] = sl.nw[u - sl.nbase];
}

// Admit contended movers whose inclusive prefix fits.
__global__ void __launch_bounds__(256) k_contended_mark(const DevSlot* __restrict__ S, int ns,
                                                        const uint64_t* __restrict__ keys, uint32_t cnt,
                                                        int node_bits, const int64_t* __restrict__ prefix) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= cnt) return;
  const uint64_t k = keys[i];
  const int64_t u = (int64_t)(k & ((1ull << node_bits) - 1ull));
  const DevSlot& sl = S[slot_of(S, ns, u)];
  const int64_t v = u - sl.nbase;
  const int32_t t = sl.desire[v];
  sl.adm[v] = sl.W[t] + prefix[i] <= sl.cap ? 1 : 0;
}

// Apply admitted moves; reset rejected desires and the incoming sums; in
// refinement add the neighbours of moved nodes to the next rated set.
__global__ void __launch_bounds__(256) k_apply(const DevSlot* __restrict__ S, int ns, int64_t N) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t base = (int64_t)blockIdx.x * blockDim.x; base < N; base += stride) {
    const int64_t u = base + threadIdx.x;
    int s = 0;
    bool moved = false;
    if (u < N) {
      s = slot_of(S, ns, u);
      const DevSlot& sl = S[s];
      if (sl.round > 0) {
        const int64_t v = u - sl.nbase;
        const int32_t t = sl.desire[v];
        const int32_t own = sl.lab[v];
        if (t != own) {
          sl.inc[t] = 0;
          if (sl.adm[v]) {
            const int64_t cv = sl.nw[v];
            sl.lab[v] = t;
            atomicAdd((unsigned long long*)&sl.W[t], (unsigned long long)cv);
            atomicAdd((unsigned long long*)&sl.W[own], (unsigned long long)(-cv));
            moved = true;
            if (sl.mode == MODE_REFINE) {
              for (int64_t e = sl.rp[v]; e < sl.rp[v + 1]; ++e) sl.flag_next[sl.col[e]] = 1;
            }
          } else {
            sl.desire[v] = own;
          }
        }
      }
    }
    wave_count(S, s, CTR_MOVED, moved ? 1 : 0);
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

int launch_bin(const DevSlot* S, int ns, int64_t N, int32_t* bins, int64_t bin_cap, uint32_t* bin_cnt,
               hipStream_t st) {
  hipLaunchKernelGGL(k_bin, dim3(grid_for(N, 256, 8192)), dim3(256), 0, st, S, ns, N, bins, bin_cap, bin_cnt);
  SCLAP_HIP(hipGetLastError());
  return SCLAP_OK;
}

int launch_rate(const DevSlot* S, int ns, const int32_t* bins, int64_t bin_cap, const uint32_t* bin_cnt,
                const RateHubScratch& hub, hipStream_t st) {
  const unsigned G = 2048;
  hipLaunchKernelGGL(k_rate_group<8>, dim3(G), dim3(256), 0, st, S, ns, bins, bin_cnt);
  hipLaunchKernelGGL(k_rate_group<64>, dim3(G), dim3(256), 0, st, S, ns, bins + bin_cap, bin_cnt + 1);
  hipLaunchKernelGGL(k_rate_block, dim3(G), dim3(256), 0, st, S, ns, bins + 2 * bin_cap, bin_cnt + 2);
  hipLaunchKernelGGL(k_hub_prep, dim3(1), dim3(1024), 0, st, S, ns, bins + 3 * bin_cap, bin_cnt + 3,
                     hub.chunk_off, hub.tab_off, hub.totals, hub.tab_cap, hub.overflow);
  hipLaunchKernelGGL(k_hub_chunk, dim3(G), dim3(256), 0, st, S, ns, bins + 3 * bin_cap, bin_cnt + 3,
                     hub.chunk_off, hub.tab_off, hub.totals, hub.gkeys, hub.gvals, hub.own, hub.overflow);
  hipLaunchKernelGGL(k_hub_final, dim3(G), dim3(256), 0, st, S, ns, bins + 3 * bin_cap, bin_cnt + 3,
                     hub.tab_off, hub.gkeys, hub.gvals, hub.own, hub.overflow);
  SCLAP_HIP(hipGetLastError());
  return SCLAP_OK;
}

int launch_incoming_decide(const DevSlot* S, int ns, int64_t N, uint64_t* ckeys, uint32_t* ccnt, int node_bits,
                           hipStream_t st) {
  const unsigned g = grid_for(N, 256, 8192);
  hipLaunchKernelGGL(k_incoming, dim3(g), dim3(256), 0, st, S, ns, N);
  hipLaunchKernelGGL(k_decide, dim3(g), dim3(256), 0, st, S, ns, N, ckeys, ccnt, node_bits);
  SCLAP_HIP(hipGetLastError());
  return SCLAP_OK;
}

int launch_contended_split(const DevSlot* S, int ns, const uint64_t* keys, uint32_t cnt, int node_bits,
                           uint32_t* tkey, int64_t* wv, hipStream_t st) {
  if (cnt == 0) return SCLAP_OK;
  hipLaunchKernelGGL(k_contended_split, dim3((cnt + 255) / 256), dim3(256), 0, st, S, ns, keys, cnt, node_bits,
                     tkey, wv);
  SCLAP_HIP(hipGetLastError());
  return SCLAP_OK;
}

int launch_contended_mark(const DevSlot* S, int ns, const uint64_t* keys, uint32_t cnt, int node_bits,
                          const int64_t* prefix, hipStream_t st) {
  if (cnt == 0) return SCLAP_OK;
  hipLaunchKernelGGL(k_contended_mark, dim3((cnt + 255) / 256), dim3(256), 0, st, S, ns, keys, cnt, node_bits,
                     prefix);
  SCLAP_HIP(hipGetLastError());
  return SCLAP_OK;
}

int launch_apply(const DevSlot* S, int ns, int64_t N, hipStream_t st) {
  hipLaunchKernelGGL(k_apply, dim3(grid_for(N, 256, 8192)), dim3(256), 0, st, S, ns, N);
  SCLAP_HIP(hipGetLastError());
  return SCLAP_OK;
}

}  // namespace sclap
