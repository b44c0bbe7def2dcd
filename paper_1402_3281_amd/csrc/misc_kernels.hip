// misc_kernels.hip -- contraction (Section 3.1), initial partition, projection,
// cut and block weights (Section 2.1), placement of degree-0 nodes, input
// validation, and small initialisation / reduction kernels.
#include <hip/hip_runtime.h>

#include <climits>

#include "common.h"
#include "lp.h"
#include "misc.h"

namespace sclap {

__device__ __forceinline__ uint32_t lane() { return __lane_id(); }

template <class T>
__global__ void __launch_bounds__(256) k_fill(T* __restrict__ p, int64_t n, T v) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) p[i] = v;
}

static inline unsigned grid1(int64_t n, unsigned cap = 8192) {
  int64_t g = (n + 255) / 256;
  if (g < 1) g = 1;
  return (unsigned)(g < cap ? g : cap);
}

template <class T>
int fill_t(T* p, int64_t n, T v, hipStream_t st) {
  if (n <= 0) return SCLAP_OK;
  hipLaunchKernelGGL(k_fill<T>, dim3(grid1(n)), dim3(256), 0, st, p, n, v);
  SCLAP_HIP(hipGetLastError());
  return SCLAP_OK;
}
int fill_i32(int32_t* p, int64_t n, int32_t v, hipStream_t st) { return fill_t(p, n, v, st); }
int fill_i64(int64_t* p, int64_t n, int64_t v, hipStream_t st) { return fill_t(p, n, v, st); }
int fill_u8(uint8_t* p, int64_t n, uint8_t v, hipStream_t st) { return fill_t(p, n, v, st); }
int fill_u32(uint32_t* p, int64_t n, uint32_t v, hipStream_t st) { return fill_t(p, n, v, st); }

// ---------------------------------------------------------------------------
// Small reductions over a graph: totals[0] += sum c, totals[1] = max c,
// totals[2] += #degree>0 nodes, totals[3] += hub table entries for
// `nlabels` labels, totals[4] += #hubs.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_graph_totals(const int64_t* __restrict__ rp, const int64_t* __restrict__ nw,
                                                      int64_t n, int64_t nlabels, unsigned long long* __restrict__ out) {
  int64_t s = 0, mx = 0, nz = 0, hub = 0, hubs = 0;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += stride) {
    const int64_t c = nw[v];
    s += c;
    mx = c > mx ? c : mx;
    const int64_t d = rp[v + 1] - rp[v];
    nz += d > 0;
    if (d > kBinBlock) {
      const int64_t distinct = d < nlabels ? d : nlabels;
      int64_t t = 64;
      while (t < 2 * distinct) t <<= 1;
      hub += t;
      ++hubs;
    }
  }
  for (int off = 32; off > 0; off >>= 1) {
    s += __shfl_xor(s, off);
    const int64_t o = __shfl_xor(mx, off);
    mx = o > mx ? o : mx;
    nz += __shfl_xor(nz, off);
    hub += __shfl_xor(hub, off);
    hubs += __shfl_xor(hubs, off);
  }
  if (lane() == 0) {
    atomicAdd(&out[0], (unsigned long long)s);
    atomicMax(&out[1], (unsigned long long)mx);
    atomicAdd(&out[2], (unsigned long long)nz);
    atomicAdd(&out[3], (unsigned long long)hub);
    atomicAdd(&out[4], (unsigned long long)hubs);
  }
}

int graph_totals(const int64_t* rp, const int64_t* nw, int64_t n, int64_t nlabels, unsigned long long* out4,
                 hipStream_t st) {
  SCLAP_TRY(fill_t((uint64_t*)out4, 5, (uint64_t)0, st));
  if (n <= 0) return SCLAP_OK;
  hipLaunchKernelGGL(k_graph_totals, dim3(grid1(n, 2048)), dim3(256), 0, st, rp, nw, n, nlabels, out4);
  SCLAP_HIP(hipGetLastError());
  return SCLAP_OK;
}

__global__ void __launch_bounds__(256) k_widen_nw(const void* __restrict__ src, int bytes, int64_t n,
                                                  int64_t* __restrict__ dst) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += stride) {
    if (!src) dst[v] = 1;
    else if (bytes == 4) dst[v] = ((const int32_t*)src)[v];
    else dst[v] = ((const int64_t*)src)[v];
  }
}

int widen_nw(const void* src, int bytes, int64_t n, int64_t* dst, hipStream_t st) {
  if (n <= 0) return SCLAP_OK;
  hipLaunchKernelGGL(k_widen_nw, dim3(grid1(n)), dim3(256), 0, st, src, bytes, n, dst);
  SCLAP_HIP(hipGetLastError());
  return SCLAP_OK;
}

// Cluster init: lab(v) = v, desire(v) = v, W(v) = c(v) (each node its own
// cluster, Section 3.1).
__global__ void __launch_bounds__(256) k_init_cluster(int32_t* __restrict__ lab, int32_t* __restrict__ desire,
                                                      int64_t* __restrict__ W, const int64_t* __restrict__ nw,
                                                      int64_t n) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += stride) {
    lab[v] = (int32_t)v;
    desire[v] = (int32_t)v;
    W[v] = nw[v];
  }
}

int init_cluster(int32_t* lab, int32_t* desire, int64_t* W, const int64_t* nw, int64_t n, hipStream_t st) {
  if (n <= 0) return SCLAP_OK;
  hipLaunchKernelGGL(k_init_cluster, dim3(grid1(n)), dim3(256), 0, st, lab, desire, W, nw, n);
  SCLAP_HIP(hipGetLastError());
  return SCLAP_OK;
}

__global__ void __launch_bounds__(256) k_copy_i32(const int32_t* __restrict__ a, int32_t* __restrict__ b, int64_t n) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += stride) b[v] = a[v];
}

int copy_i32(const int32_t* a, int32_t* b, int64_t n, hipStream_t st) {
  if (n <= 0) return SCLAP_OK;
  hipLaunchKernelGGL(k_copy_i32, dim3(grid1(n)), dim3(256), 0, st, a, b, n);
  SCLAP_HIP(hipGetLastError());
  return SCLAP_OK;
}

// ---------------------------------------------------------------------------
// Block weights: W(b) = sum of c(v) over nodes with part(v) = b >= 0.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_block_weights(const int32_t* __restrict__ part, const int64_t* __restrict__ nw,
                                                       int64_t n, int32_t k, int64_t* __restrict__ W) {
  extern __shared__ unsigned long long hist[];
  const bool lds = k <= 4096;
  if (lds)
    for (int b = threadIdx.x; b < k; b += blockDim.x) hist[b] = 0;
  __syncthreads();
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += stride) {
    const int32_t b = part[v];
    if (b < 0) continue;
    if (lds) atomicAdd(&hist[b], (unsigned long long)nw[v]);
    else atomicAdd((unsigned long long*)&W[b], (unsigned long long)nw[v]);
  }
  __syncthreads();
  if (lds)
    for (int b = threadIdx.x; b < k; b += blockDim.x)
      if (hist[b]) atomicAdd((unsigned long long*)&W[b], hist[b]);
}

int block_weights(const int32_t* part, const int64_t* nw, int64_t n, int32_t k, int64_t* W, hipStream_t st) {
  SCLAP_TRY(fill_i64(W, k, 0, st));
  if (n <= 0) return SCLAP_OK;
  const size_t sh = k <= 4096 ? (size_t)k * 8 : 0;
  hipLaunchKernelGGL(k_block_weights, dim3(grid1(n, 1024)), dim3(256), sh, st, part, nw, n, k, W);
  SCLAP_HIP(hipGetLastError());
  return SCLAP_OK;
}

// ---------------------------------------------------------------------------
// Wave-cooperative row traversal: each wave takes 64 consecutive nodes; a
// lane walks its own row when it has at most kShort entries, longer rows are
// walked by the whole wave, one after the other.
// ---------------------------------------------------------------------------
constexpr int kShort = 32;

// Cut: sum of w(u, v) over stored entries with part(u) != part(v), halved on
// the host.  Nodes with part -1 have no entries.
__global__ void __launch_bounds__(256) k_cut(const int64_t* __restrict__ rp, const int32_t* __restrict__ col,
                                             const int32_t* __restrict__ ew, const int32_t* __restrict__ part,
                                             int64_t n, unsigned long long* __restrict__ out) {
  const int64_t waves = (int64_t)gridDim.x * (blockDim.x / kWave);
  const int64_t wid = (int64_t)blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave;
  int64_t acc = 0;
  for (int64_t base = wid * kWave; base < n; base += waves * kWave) {
    const int64_t v = base + lane();
    int64_t e0 = 0, d = 0;
    int32_t pv = 0;
    if (v < n) {
      e0 = rp[v];
      d = rp[v + 1] - e0;
      pv = part[v];
    }
    if (d <= kShort)
      for (int64_t e = e0; e < e0 + d; ++e)
        if (part[col[e]] != pv) acc += ew ? ew[e] : 1;
    uint64_t big = __ballot(d > kShort);
    while (big) {
      const int l = __ffsll((unsigned long long)big) - 1;
      big &= big - 1;
      const int64_t be0 = __shfl(e0, l), bd = __shfl(d, l);
      const int32_t bp = __shfl(pv, l);
      for (int64_t e = be0 + lane(); e < be0 + bd; e += kWave)
        if (part[col[e]] != bp) acc += ew ? ew[e] : 1;
    }
  }
  for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off);
  if (lane() == 0 && acc) atomicAdd(out, (unsigned long long)acc);
}

int cut_twice(const int64_t* rp, const int32_t* col, const int32_t* ew, const int32_t* part, int64_t n,
              unsigned long long* out, hipStream_t st) {
  SCLAP_TRY(fill_t((uint64_t*)out, 1, (uint64_t)0, st));
  if (n <= 0) return SCLAP_OK;
  hipLaunchKernelGGL(k_cut, dim3(grid1((n + 63) / 64 * 64 / 4, 4096)), dim3(256), 0, st, rp, col, ew, part, n, out);
  SCLAP_HIP(hipGetLastError());
  return SCLAP_OK;
}

// ---------------------------------------------------------------------------
// Contraction (Section 3.1): each cluster becomes one node.
// ---------------------------------------------------------------------------

// used(lab(v)) = 1 for every node that joins a coarse node.
__global__ void __launch_bounds__(256) k_flag_used(const int32_t* __restrict__ lab, const int64_t* __restrict__ rp,
                                                   int64_t n, int drop, int32_t* __restrict__ used) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += stride) {
    if (drop && rp[v + 1] == rp[v]) continue;
    used[lab[v]] = 1;
  }
}

// coarse_of(v) = rank of lab(v) among the used labels; coarse weights.
__global__ void __launch_bounds__(256) k_coarse_of(const int32_t* __restrict__ lab, const int64_t* __restrict__ rp,
                                                   const int64_t* __restrict__ nw, int64_t n, int drop,
                                                   const int32_t* __restrict__ cid, int32_t* __restrict__ cof,
                                                   int64_t* __restrict__ cnw) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += stride) {
    if (drop && rp[v + 1] == rp[v]) {
      cof[v] = -1;
      continue;
    }
    const int32_t x = cid[lab[v]];
    cof[v] = x;
    atomicAdd((unsigned long long*)&cnw[x], (unsigned long long)nw[v]);
  }
}

// Count (mode 0) or emit (mode 1) the entries that join different coarse
// nodes, as keys x * 2^b + y with their weights.
__global__ void __launch_bounds__(256) k_cross(const int64_t* __restrict__ rp, const int32_t* __restrict__ col,
                                               const int32_t* __restrict__ ew, const int32_t* __restrict__ cof,
                                               int64_t n, int bits, int mode, unsigned long long* __restrict__ cnt,
                                               uint64_t* __restrict__ keys, int32_t* __restrict__ vals) {
  const int64_t waves = (int64_t)gridDim.x * (blockDim.x / kWave);
  const int64_t wid = (int64_t)blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave;
  int64_t total = 0;
  for (int64_t base = wid * kWave; base < n; base += waves * kWave) {
    const int64_t v = base + lane();
    int64_t e0 = 0, d = 0;
    int32_t x = -1;
    if (v < n) {
      e0 = rp[v];
      d = rp[v + 1] - e0;
      x = cof[v];
    }
    // short rows: count own entries, then claim a range with one atomic
    int64_t mine = 0;
    if (d <= kShort)
      for (int64_t e = e0; e < e0 + d; ++e) mine += cof[col[e]] != x;
    if (mode == 0) {
      total += mine;
    } else {
      int64_t incl = mine;
      for (int off = 1; off < kWave; off <<= 1) {
        const int64_t o = __shfl_up(incl, off);
        if ((int)lane() >= off) incl += o;
      }
      const int64_t wsum = __shfl(incl, kWave - 1);
      unsigned long long base_pos = 0;
      if (lane() == kWave - 1 && wsum) base_pos = atomicAdd(cnt, (unsigned long long)wsum);
      base_pos = __shfl(base_pos, kWave - 1);
      int64_t p = (int64_t)base_pos + incl - mine;
      if (d <= kShort)
        for (int64_t e = e0; e < e0 + d; ++e) {
          const int32_t y = cof[col[e]];
          if (y != x) {
            keys[p] = ((uint64_t)(uint32_t)x << bits) | (uint64_t)(uint32_t)y;
            vals[p] = ew ? ew[e] : 1;
            ++p;
          }
        }
    }
    uint64_t big = __ballot(d > kShort);
    while (big) {
      const int l = __ffsll((unsigned long long)big) - 1;
      big &= big - 1;
      const int64_t be0 = __shfl(e0, l), bd = __shfl(d, l);
      const int32_t bx = __shfl(x, l);
      for (int64_t eb = be0; eb < be0 + bd; eb += kWave) {
        const int64_t e = eb + lane();
        bool c = false;
        int32_t y = 0;
        if (e < be0 + bd) {
          y = cof[col[e]];
          c = y != bx;
        }
        const uint64_t m = __ballot(c);
        if (mode == 0) {
          total += c ? 1 : 0;
        } else if (m) {
          unsigned long long bp = 0;
          if (lane() == 0) bp = atomicAdd(cnt, (unsigned long long)__popcll(m));
          bp = __shfl(bp, 0);
          if (c) {
            const int64_t p = (int64_t)bp + __popcll(m & ((1ull << lane()) - 1ull));
            keys[p] = ((uint64_t)(uint32_t)bx << bits) | (uint64_t)(uint32_t)y;
            vals[p] = ew ? ew[e] : 1;
          }
        }
      }
    }
  }
  if (mode == 0) {
    for (int off = 32; off > 0; off >>= 1) total += __shfl_xor(total, off);
    if (lane() == 0 && total) atomicAdd(cnt, (unsigned long long)total);
  }
}

// Coarse neighbour ids and weights from the reduced keys.
__global__ void __launch_bounds__(256) k_coarse_cols(const uint64_t* __restrict__ ukeys, const int64_t* __restrict__ aggs,
                                                     int64_t m, int bits, int32_t* __restrict__ col,
                                                     int32_t* __restrict__ ew, unsigned* __restrict__ overflow) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const uint64_t mask = (1ull << bits) - 1ull;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m; i += stride) {
    col[i] = (int32_t)(ukeys[i] & mask);
    const int64_t a = aggs[i];
    if (a > INT32_MAX) *overflow = 1;
    ew[i] = (int32_t)a;
  }
}

// row_ptr(x) = first entry with row >= x.
__global__ void __launch_bounds__(256) k_coarse_rowptr(const uint64_t* __restrict__ ukeys, int64_t m, int bits,
                                                       int64_t nc, int64_t* __restrict__ rp) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; x <= nc; x += stride) {
    const uint64_t key = (uint64_t)x << bits;
    int64_t lo = 0, hi = m;
    while (lo < hi) {
      const int64_t mid = (lo + hi) >> 1;
      if (ukeys[mid] < key) lo = mid + 1;
      else hi = mid;
    }
    rp[x] = lo;
  }
}

int contract_flag(const int32_t* lab, const int64_t* rp, int64_t n, int drop, int32_t* used, hipStream_t st) {
  SCLAP_TRY(fill_i32(used, n, 0, st));
  if (n <= 0) return SCLAP_OK;
  hipLaunchKernelGGL(k_flag_used, dim3(grid1(n)), dim3(256), 0, st, lab, rp, n, drop, used);
  SCLAP_HIP(hipGetLastError());
  return SCLAP_OK;
}

int contract_coarse_of(const int32_t* lab, const int64_t* rp, const int64_t* nw, int64_t n, int drop,
                       const int32_t* cid, int32_t* cof, int64_t* cnw, int64_t nc, hipStream_t st) {
  SCLAP_TRY(fill_i64(cnw, nc, 0, st));
  if (n <= 0) return SCLAP_OK;
  hipLaunchKernelGGL(k_coarse_of, dim3(grid1(n)), dim3(256), 0, st, lab, rp, nw, n, drop, cid, cof, cnw);
  SCLAP_HIP(hipGetLastError());
  return SCLAP_OK;
}

int contract_cross(const int64_t* rp, const int32_t* col, const int32_t* ew, const int32_t* cof, int64_t n,
                   int bits, int mode, unsigned long long* cnt, uint64_t* keys, int32_t* vals, hipStream_t st) {
  SCLAP_TRY(fill_t((uint64_t*)cnt, 1, (uint64_t)0, st));
  if (n <= 0) return SCLAP_OK;
  hipLaunchKernelGGL(k_cross, dim3(grid1((n + 3) / 4, 4096)), dim3(256), 0, st, rp, col, ew, cof, n, bits, mode,
                     cnt, keys, vals);
  SCLAP_HIP(hipGetLastError());
  return SCLAP_OK;
}

int contract_finish(const uint64_t* ukeys, const int64_t* aggs, int64_t m, int bits, int64_t nc, int64_t* rp,
                    int32_t* col, int32_t* ew, unsigned* overflow, hipStream_t st) {
  if (m > 0)
    hipLaunchKernelGGL(k_coarse_cols, dim3(grid1(m)), dim3(256), 0, st, ukeys, aggs, m, bits, col, ew, overflow);
  hipLaunchKernelGGL(k_coarse_rowptr, dim3(grid1(nc + 1)), dim3(256), 0, st, ukeys, m, bits, nc, rp);
  SCLAP_HIP(hipGetLastError());
  return SCLAP_OK;
}

// ---------------------------------------------------------------------------
// Projection (Section 3.1): a fine node takes its coarse node's block.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_project(const int32_t* __restrict__ cof, const int32_t* __restrict__ pc,
                                                 int64_t n, int32_t* __restrict__ pf) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += stride) {
    const int32_t x = cof[v];
    pf[v] = x >= 0 ? pc[x] : -1;
  }
}

int project(const int32_t* cof, const int32_t* pc, int64_t n, int32_t* pf, hipStream_t st) {
  if (n <= 0) return SCLAP_OK;
  hipLaunchKernelGGL(k_project, dim3(grid1(n)), dim3(256), 0, st, cof, pc, n, pf);
  SCLAP_HIP(hipGetLastError());
  return SCLAP_OK;
}

// ---------------------------------------------------------------------------
// Initial partition: breadth-first order cut into k chunks, one workgroup
// (1024 threads) per graph.  Frontiers expand level by level; a node joins
// the earliest frontier node adjacent to it (atomic minimum of frontier
// positions), and each frontier node appends its children in ascending id,
// which reproduces the order of a FIFO search that appends neighbours in
// ascending id.  Searches start at the smallest unvisited id; degree-0
// nodes are single-node searches and are appended in bulk.
// ---------------------------------------------------------------------------
constexpr int kIpThreads = 1024;
constexpr int kIpWaves = kIpThreads / kWave;

template <class T>
__device__ __forceinline__ T ld_acq(const T* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <class T>
__device__ __forceinline__ void st_rel(T* p, T v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Exclusive block scan of one int64 per thread; returns the block total.
__device__ int64_t block_exscan(int64_t x, int64_t* excl, int64_t* sh) {
  int64_t incl = x;
  for (int off = 1; off < kWave; off <<= 1) {
    const int64_t o = __shfl_up(incl, off);
    if ((int)lane() >= off) incl += o;
  }
  const int w = threadIdx.x / kWave;
  __syncthreads();
  if (lane() == kWave - 1) sh[w] = incl;
  __syncthreads();
  int64_t before = 0, total = 0;
  for (int i = 0; i < kIpWaves; ++i) {
    if (i < w) before += sh[i];
    total += sh[i];
  }
  *excl = before + incl - x;
  return total;
}

__device__ int64_t block_min64(int64_t x, int64_t* sh) {
  for (int off = 32; off > 0; off >>= 1) {
    const int64_t o = __shfl_xor(x, off);
    x = o < x ? o : x;
  }
  const int w = threadIdx.x / kWave;
  __syncthreads();
  if (lane() == 0) sh[w] = x;
  __syncthreads();
  int64_t r = sh[0];
  for (int i = 1; i < kIpWaves; ++i) r = sh[i] < r ? sh[i] : r;
  return r;
}

__global__ void __launch_bounds__(kIpThreads) k_ip_bfs(const IpSlot* __restrict__ slots) {
  const IpSlot sl = slots[blockIdx.x];
  __shared__ int64_t sh[kIpWaves];
  __shared__ int64_t s_head, s_tail, s_next;
  const int64_t n = sl.n;
  const int wv = threadIdx.x / kWave;
  if (threadIdx.x == 0) {
    s_head = 0;
    s_tail = 0;
    s_next = 0;
  }
  __syncthreads();
  for (;;) {
    __syncthreads();
    const int64_t head = s_head, tail = s_tail, next = s_next;
    __syncthreads();
    if (head == tail) {
      if (next >= n) break;
      // seeds: unvisited degree-0 nodes before the first unvisited node with
      // neighbours are whole searches of their own
      const int64_t id = next + threadIdx.x;
      const bool valid = id < n;
      int64_t d = 0;
      bool unv = false;
      if (valid) {
        d = sl.rp[id + 1] - sl.rp[id];
        unv = ld_acq(&sl.pos[id]) == -1;
      }
      const bool skip = valid && sl.skip_isolated && d == 0;
      const bool iso = unv && !skip && d == 0;
      const bool seed = unv && !skip && d > 0;
      const int64_t first = block_min64(seed ? id : INT64_MAX, sh);
      const bool take = (iso && id < first) || (seed && id == first);
      int64_t ex;
      const int64_t tot = block_exscan(take ? 1 : 0, &ex, sh);
      if (take) {
        st_rel(&sl.order[tail + ex], (int32_t)id);
        st_rel(&sl.pos[id], (int32_t)(tail + ex));
      }
      __syncthreads();
      if (threadIdx.x == 0) {
        s_tail = tail + tot;
        s_next = first != INT64_MAX ? first + 1 : next + kIpThreads;
        // degree-0 nodes have nothing to expand: the frontier is the seed
        s_head = first != INT64_MAX ? tail + tot - 1 : tail + tot;
      }
      continue;
    }
    const int64_t F = tail - head;
    // pass 1: claims
    for (int64_t fi = wv; fi < F; fi += kIpWaves) {
      const int32_t f = ld_acq(&sl.order[head + fi]);
      const int64_t e0 = sl.rp[f], e1 = sl.rp[f + 1];
      for (int64_t e = e0 + lane(); e < e1; e += kWave) {
        const int32_t u = sl.col[e];
        if (ld_acq(&sl.pos[u]) == -1) atomicMin(&sl.claim[u], (int32_t)fi);
      }
    }
    __syncthreads();
    // pass 2: children per frontier node
    for (int64_t fi = wv; fi < F; fi += kIpWaves) {
      const int32_t f = ld_acq(&sl.order[head + fi]);
      const int64_t e0 = sl.rp[f], e1 = sl.rp[f + 1];
      int64_t c = 0;
      for (int64_t e = e0 + lane(); e < e1; e += kWave) {
        const int32_t u = sl.col[e];
        c += (ld_acq(&sl.claim[u]) == (int32_t)fi && ld_acq(&sl.pos[u]) == -1) ? 1 : 0;
      }
      for (int off = 32; off > 0; off >>= 1) c += __shfl_xor(c, off);
      if (lane() == 0) st_rel(&sl.cnt[fi], (int32_t)c);
    }
    __syncthreads();
    // pass 3: exclusive offsets of the child counts
    int64_t carry = 0;
    for (int64_t b = 0; b < F; b += kIpThreads) {
      const int64_t fi = b + threadIdx.x;
      const int64_t c = fi < F ? ld_acq(&sl.cnt[fi]) : 0;
      int64_t ex;
      const int64_t tot = block_exscan(c, &ex, sh);
      if (fi < F) st_rel(&sl.cnt[fi], (int32_t)(carry + ex));
      carry += tot;
      __syncthreads();
    }
    const int64_t T = carry;
    __syncthreads();
    // pass 4: children in ascending id
    for (int64_t fi = wv; fi < F; fi += kIpWaves) {
      const int32_t f = ld_acq(&sl.order[head + fi]);
      const int64_t e0 = sl.rp[f], e1 = sl.rp[f + 1];
      const int64_t off = tail + ld_acq(&sl.cnt[fi]);
      if (sl.rows_sorted) {
        int64_t run = 0;
        for (int64_t eb = e0; eb < e1; eb += kWave) {
          const int64_t e = eb + lane();
          int32_t u = 0;
          bool ch = false;
          if (e < e1) {
            u = sl.col[e];
            ch = ld_acq(&sl.claim[u]) == (int32_t)fi && ld_acq(&sl.pos[u]) == -1;
          }
          const uint64_t m = __ballot(ch);
          if (ch) st_rel(&sl.order[off + run + __popcll(m & ((1ull << lane()) - 1ull))], u);
          run += __popcll(m);
        }
      } else {
        for (int64_t e = e0 + lane(); e < e1; e += kWave) {
          const int32_t u = sl.col[e];
          if (!(ld_acq(&sl.claim[u]) == (int32_t)fi && ld_acq(&sl.pos[u]) == -1)) continue;
          int64_t rank = 0;
          for (int64_t e2 = e0; e2 < e1; ++e2) {
            const int32_t w2 = sl.col[e2];
            if (w2 < u && ld_acq(&sl.claim[w2]) == (int32_t)fi && ld_acq(&sl.pos[w2]) == -1) ++rank;
          }
          st_rel(&sl.order[off + rank], u);
        }
      }
    }
    __syncthreads();
    // pass 5: positions of the new nodes
    for (int64_t i = threadIdx.x; i < T; i += kIpThreads) {
      const int32_t u = ld_acq(&sl.order[tail + i]);
      st_rel(&sl.pos[u], (int32_t)(tail + i));
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      s_head = tail;
      s_tail = tail + T;
    }
  }
  __syncthreads();
  // chunks of the BFS order: block(v) = min(k-1, floor(k P(v) / C))
  const int64_t placed = s_tail;
  int64_t C = 0;
  for (int64_t b = 0; b < placed; b += kIpThreads) {
    const int64_t i = b + threadIdx.x;
    const int64_t c = i < placed ? sl.nw[ld_acq(&sl.order[i])] : 0;
    int64_t ex;
    C += block_exscan(c, &ex, sh);
    __syncthreads();
  }
  int64_t carry = 0;
  for (int64_t b = 0; b < placed; b += kIpThreads) {
    const int64_t i = b + threadIdx.x;
    int32_t v = 0;
    int64_t c = 0;
    if (i < placed) {
      v = ld_acq(&sl.order[i]);
      c = sl.nw[v];
    }
    int64_t ex;
    const int64_t tot = block_exscan(c, &ex, sh);
    if (i < placed) {
      const int64_t P = carry + ex;
      int64_t blk = C > 0 ? ((int64_t)sl.k * P) / C : 0;
      if (blk > sl.k - 1) blk = sl.k - 1;
      sl.part[v] = (int32_t)blk;
    }
    carry += tot;
    __syncthreads();
  }
}

int initial_partition(const IpSlot* dev_slots, int count, hipStream_t st) {
  if (count <= 0) return SCLAP_OK;
  hipLaunchKernelGGL(k_ip_bfs, dim3(count), dim3(kIpThreads), 0, st, dev_slots);
  SCLAP_HIP(hipGetLastError());
  return SCLAP_OK;
}

// ---------------------------------------------------------------------------
// Degree-0 nodes of the input: fill the lightest blocks up to a common level
// lambda (smallest with sum_b max(0, lambda - B(b)) >= C_I), block intervals
// of the isolated weight in block order, node i (prefix P_i) to the first
// block whose interval end exceeds P_i, else the last block with room.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_iso_weights(const int64_t* __restrict__ rp, const int64_t* __restrict__ nw,
                                                     int64_t n, int64_t* __restrict__ w) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += stride)
    w[v] = rp[v + 1] == rp[v] ? nw[v] : 0;
}

__global__ void __launch_bounds__(256) k_iso_level(const int64_t* __restrict__ B, int32_t k,
                                                   const int64_t* __restrict__ pre, const int64_t* __restrict__ w,
                                                   int64_t n, int64_t* __restrict__ ends, int32_t* __restrict__ last) {
  __shared__ int64_t red[4], rlo[4], rhi[4];
  const int64_t CI = n > 0 ? pre[n - 1] + w[n - 1] : 0;
  int64_t lo = INT64_MAX, hi = INT64_MIN;
  for (int b = threadIdx.x; b < k; b += blockDim.x) {
    lo = B[b] < lo ? B[b] : lo;
    hi = B[b] > hi ? B[b] : hi;
  }
  for (int off = 32; off > 0; off >>= 1) {
    const int64_t a = __shfl_xor(lo, off), c = __shfl_xor(hi, off);
    lo = a < lo ? a : lo;
    hi = c > hi ? c : hi;
  }
  if (lane() == 0) {
    rlo[threadIdx.x / kWave] = lo;
    rhi[threadIdx.x / kWave] = hi;
  }
  __syncthreads();
  for (int i = 0; i < 4; ++i) {
    lo = rlo[i] < lo ? rlo[i] : lo;
    hi = rhi[i] > hi ? rhi[i] : hi;
  }
  int64_t a = lo, z = hi + CI;
  while (a < z) {  // uniform across the block
    const int64_t mid = a + (z - a) / 2;
    int64_t D = 0;
    for (int b = threadIdx.x; b < k; b += blockDim.x) D += mid > B[b] ? mid - B[b] : 0;
    for (int off = 32; off > 0; off >>= 1) D += __shfl_xor(D, off);
    __syncthreads();
    if (lane() == 0) red[threadIdx.x / kWave] = D;
    __syncthreads();
    D = red[0] + red[1] + red[2] + red[3];
    if (D >= CI) z = mid;
    else a = mid + 1;
  }
  if (threadIdx.x == 0) {
    const int64_t lambda = a;
    int64_t D = 0;
    int32_t lp = 0;
    for (int b = 0; b < k; ++b) {
      const int64_t d = lambda > B[b] ? lambda - B[b] : 0;
      D += d;
      ends[b] = D;
      if (d > 0) lp = b;
    }
    *last = lp;
  }
}

__global__ void __launch_bounds__(256) k_iso_assign(const int64_t* __restrict__ rp, int64_t n,
                                                    const int64_t* __restrict__ pre, const int64_t* __restrict__ ends,
                                                    const int32_t* __restrict__ last, int32_t k,
                                                    int32_t* __restrict__ part) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += stride) {
    if (rp[v + 1] != rp[v]) continue;
    const int64_t P = pre[v];
    int lo = 0, hi = k;  // first b with ends[b] > P
    while (lo < hi) {
      const int mid = (lo + hi) >> 1;
      if (ends[mid] > P) hi = mid;
      else lo = mid + 1;
    }
    part[v] = lo < k ? lo : *last;
  }
}

int place_isolated(const int64_t* rp, const int64_t* nw, int64_t n, const int64_t* B, int32_t k, int32_t* part,
                   int64_t* tmp_w, int64_t* tmp_pre, int64_t* ends, int32_t* last, void* scan_tmp, size_t scan_bytes,
                   hipStream_t st) {
  if (n <= 0) return SCLAP_OK;
  hipLaunchKernelGGL(k_iso_weights, dim3(grid1(n)), dim3(256), 0, st, rp, nw, n, tmp_w);
  SCLAP_HIP(hipGetLastError());
  SCLAP_TRY(prim_exscan_i64(scan_tmp, scan_bytes, tmp_w, tmp_pre, (size_t)n, st));
  hipLaunchKernelGGL(k_iso_level, dim3(1), dim3(256), 0, st, B, k, tmp_pre, tmp_w, n, ends, last);
  hipLaunchKernelGGL(k_iso_assign, dim3(grid1(n)), dim3(256), 0, st, rp, n, tmp_pre, ends, last, k, part);
  SCLAP_HIP(hipGetLastError());
  return SCLAP_OK;
}

// ---------------------------------------------------------------------------
// Validation: forward keys (u, v) and reverse keys (v, u) with weights,
// sorted; equal arrays <=> symmetric with equal weights.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_val_keys(const int64_t* __restrict__ rp, const int32_t* __restrict__ col,
                                                  const int32_t* __restrict__ ew, int64_t n, int64_t m, int bits,
                                                  uint64_t* __restrict__ fk, uint64_t* __restrict__ rk,
                                                  int32_t* __restrict__ fw, unsigned* __restrict__ bad) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; u < n; u += stride) {
    const int64_t e0 = rp[u], e1 = rp[u + 1];
    if (e0 > e1 || e0 < 0 || e1 > m) {
      atomicOr(bad, 2u);
      continue;
    }
    for (int64_t e = e0; e < e1; ++e) {
      const int32_t v = col[e];
      const int32_t w = ew ? ew[e] : 1;
      if (v < 0 || v >= n || w < 1) {
        atomicOr(bad, 2u);
        fk[e] = rk[e] = 0;
        fw[e] = 0;
        continue;
      }
      if (v == u) atomicOr(bad, 1u);
      fk[e] = ((uint64_t)u << bits) | (uint64_t)v;
      rk[e] = ((uint64_t)v << bits) | (uint64_t)u;
      fw[e] = w;
    }
  }
}

__global__ void __launch_bounds__(256) k_val_cmp(const uint64_t* __restrict__ fk, const uint64_t* __restrict__ rk,
                                                 const int32_t* __restrict__ fw, const int32_t* __restrict__ rw,
                                                 int64_t m, unsigned* __restrict__ bad) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m; i += stride) {
    if (fk[i] != rk[i] || fw[i] != rw[i]) atomicOr(bad, 1u);
    if (i > 0 && fk[i] == fk[i - 1]) atomicOr(bad, 1u);
  }
}

__global__ void __launch_bounds__(256) k_val_nw(const void* __restrict__ nw, int bytes, int64_t n,
                                                unsigned* __restrict__ bad) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += stride) {
    const int64_t c = bytes == 4 ? ((const int32_t*)nw)[v] : ((const int64_t*)nw)[v];
    if (c < 0) atomicOr(bad, 2u);
  }
}

int validate_keys(const int64_t* rp, const int32_t* col, const int32_t* ew, int64_t n, int64_t m, int bits,
                  uint64_t* fk, uint64_t* rk, int32_t* fw, unsigned* bad, hipStream_t st) {
  hipLaunchKernelGGL(k_val_keys, dim3(grid1(n)), dim3(256), 0, st, rp, col, ew, n, m, bits, fk, rk, fw, bad);
  SCLAP_HIP(hipGetLastError());
  return SCLAP_OK;
}

int validate_cmp(const uint64_t* fk, const uint64_t* rk, const int32_t* fw, const int32_t* rw, int64_t m,
                 unsigned* bad, hipStream_t st) {
  if (m > 0) hipLaunchKernelGGL(k_val_cmp, dim3(grid1(m)), dim3(256), 0, st, fk, rk, fw, rw, m, bad);
  SCLAP_HIP(hipGetLastError());
  return SCLAP_OK;
}

int validate_nw(const void* nw, int bytes, int64_t n, unsigned* bad, hipStream_t st) {
  if (nw && n > 0) hipLaunchKernelGGL(k_val_nw, dim3(grid1(n)), dim3(256), 0, st, nw, bytes, n, bad);
  SCLAP_HIP(hipGetLastError());
  return SCLAP_OK;
}

}  // namespace sclap
