// misc_kernels.hip -- contraction (Section 3.1), initial partition, projection,
// cut and block weights (Section 2.1), placement of degree-0 nodes, input
// validation, and small initialisation / reduction kernels.
#include <hip/hip_runtime.h>

#include <climits>

#include "common.h"
#include "edges.h"
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
// Level totals: [0] sum c, [1] max c, [2] nodes of degree > 0, and for the
// hub rating path [3] staged pair slots, [4] hubs, [5] label parts and
// [6] matrix entries when clustering (labels = nodes), [7], [8] the same
// when refining (labels = k blocks).
__global__ void __launch_bounds__(256) k_graph_totals(const int64_t* __restrict__ rp, const int64_t* __restrict__ nw,
                                                      int64_t n, int64_t k, unsigned long long* __restrict__ out) {
  int64_t acc[kGraphTotals] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += stride) {
    const int64_t c = nw[v];
    acc[0] += c;
    acc[1] = c > acc[1] ? c : acc[1];
    const int64_t d = rp[v + 1] - rp[v];
    acc[2] += d > 0;
    acc[9] = d > acc[9] ? d : acc[9];
    if (d > kBinBlock) {
      const int64_t nc = (d + kHubChunk - 1) / kHubChunk;
      const int64_t pc = hub_parts(d, n), pr = hub_parts(d, k);
      acc[3] += nc * kHubChunk;
      acc[4] += 1;
      acc[5] += pc;
      acc[6] += nc * (pc + 1);
      acc[7] += pr;
      acc[8] += nc * (pr + 1);
    }
  }
  // wave, then workgroup combination: one atomic per workgroup and counter
  // entries 1 and 9 are maxima, the others sums
  __shared__ int64_t red[4][kGraphTotals];
  for (int off = 32; off > 0; off >>= 1)
    for (int q = 0; q < kGraphTotals; ++q) {
      const int64_t o = __shfl_xor(acc[q], off);
      acc[q] = (q == 1 || q == 9) ? (o > acc[q] ? o : acc[q]) : acc[q] + o;
    }
  if (lane() == 0)
    for (int q = 0; q < kGraphTotals; ++q) red[threadIdx.x / kWave][q] = acc[q];
  __syncthreads();
  if (threadIdx.x < kGraphTotals) {
    const int q = threadIdx.x;
    const bool mx = q == 1 || q == 9;
    int64_t a = red[0][q];
    for (int w = 1; w < (int)(blockDim.x / kWave); ++w) a = mx ? (red[w][q] > a ? red[w][q] : a) : a + red[w][q];
    if (mx) atomicMax(&out[q], (unsigned long long)a);
    else if (a) atomicAdd(&out[q], (unsigned long long)a);
  }
}

int graph_totals(const int64_t* rp, const int64_t* nw, int64_t n, int64_t k, unsigned long long* out,
                 hipStream_t st) {
  SCLAP_TRY(fill_t((uint64_t*)out, kGraphTotals, (uint64_t)0, st));
  if (n <= 0) return SCLAP_OK;
  hipLaunchKernelGGL(k_graph_totals, dim3(grid1(n, 512)), dim3(256), 0, st, rp, nw, n, k, out);
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

// The input without its degree-0 nodes: node i of the compacted graph is
// input node act(i), ids kept in increasing order.  The rank of a node (the
// nodes of degree > 0 before it) is read from one 64-bit mask per 64 ids
// (ballot of degree > 0) and the exclusive count before each mask: 12 bytes
// per 64 nodes, small enough to stay in cache while the columns are
// renumbered.  Degree-0 nodes own no entries, so the entries keep their
// places and the row offsets are the input's at the kept nodes.
__device__ __forceinline__ int32_t rank_of(const uint64_t* __restrict__ words, const int32_t* __restrict__ wpre,
                                           int64_t v) {
  const int bit = (int)(v & 63);
  const uint64_t below = bit ? (words[v >> 6] & ((1ull << bit) - 1ull)) : 0ull;
  return wpre[v >> 6] + __popcll(below);
}

__global__ void __launch_bounds__(256) k_active_words(const int64_t* __restrict__ rp, int64_t n,
                                                      uint64_t* __restrict__ words, int32_t* __restrict__ wcnt) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  // whole waves walk whole 64-id words (the grid stride is a multiple of 64)
  for (int64_t v0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v0 - (int64_t)lane() < n; v0 += stride) {
    const bool act = v0 < n && rp[v0 + 1] > rp[v0];
    const uint64_t m = __ballot(act);
    if (lane() == 0) {
      words[v0 >> 6] = m;
      wcnt[v0 >> 6] = __popcll(m);
    }
  }
}

__global__ void __launch_bounds__(256) k_compact_rows(const int64_t* __restrict__ rp, const int64_t* __restrict__ nw,
                                                      const uint64_t* __restrict__ words,
                                                      const int32_t* __restrict__ wpre, int64_t n, int64_t m,
                                                      int64_t n0, int64_t* __restrict__ rp0,
                                                      int64_t* __restrict__ nw0, int32_t* __restrict__ act) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += stride) {
    const int64_t e0 = rp[v];
    if (rp[v + 1] == e0) continue;
    const int32_t i = rank_of(words, wpre, v);
    rp0[i] = e0;
    nw0[i] = nw[v];
    act[i] = (int32_t)v;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) rp0[n0] = m;
}

// A 64-id mask and the count before it in one 16-byte record, so renaming
// a column costs one gather.
struct alignas(16) RankRec {
  uint64_t mask;
  int32_t pre;
  int32_t pad;
};

__global__ void __launch_bounds__(256) k_pack_ranks(const uint64_t* __restrict__ words,
                                                    const int32_t* __restrict__ wpre, int64_t W,
                                                    RankRec* __restrict__ rec) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < W; i += stride) {
    RankRec r;
    r.mask = words[i];
    r.pre = wpre[i];
    r.pad = 0;
    rec[i] = r;
  }
}

// Tiles of 2048 entries, 8 per thread: the tile's column loads, then its
// record gathers, are in flight together.
__global__ void __launch_bounds__(256) k_compact_col(const int32_t* __restrict__ col,
                                                     const RankRec* __restrict__ rec, int64_t m,
                                                     int32_t* __restrict__ col0) {
  constexpr int kPer = 8;
  for (int64_t E0 = (int64_t)blockIdx.x * (256 * kPer); E0 < m; E0 += (int64_t)gridDim.x * (256 * kPer)) {
    int32_t c[kPer];
#pragma unroll
    for (int j = 0; j < kPer; ++j) {
      const int64_t e = E0 + j * 256 + threadIdx.x;
      c[j] = e < m ? col[e] : 0;
    }
    RankRec r[kPer];
#pragma unroll
    for (int j = 0; j < kPer; ++j) r[j] = rec[c[j] >> 6];
#pragma unroll
    for (int j = 0; j < kPer; ++j) {
      const int64_t e = E0 + j * 256 + threadIdx.x;
      const int bit = c[j] & 63;
      const uint64_t below = bit ? (r[j].mask & ((1ull << bit) - 1ull)) : 0ull;
      if (e < m) col0[e] = r[j].pre + __popcll(below);
    }
  }
}

int active_words(const int64_t* rp, int64_t n, uint64_t* words, int32_t* wcnt, hipStream_t st) {
  if (n <= 0) return SCLAP_OK;
  hipLaunchKernelGGL(k_active_words, dim3(grid1(n)), dim3(256), 0, st, rp, n, words, wcnt);
  SCLAP_HIP(hipGetLastError());
  return SCLAP_OK;
}

int64_t compact_rec_bytes(int64_t n) { return ((n + 63) / 64) * (int64_t)sizeof(RankRec); }

int compact_graph(const int64_t* rp, const int32_t* col, const int64_t* nw, const uint64_t* words,
                  const int32_t* wpre, int64_t n, int64_t m, int64_t n0, int64_t* rp0, int32_t* col0, int64_t* nw0,
                  int32_t* act, void* rec, hipStream_t st) {
  if (n <= 0) return SCLAP_OK;
  hipLaunchKernelGGL(k_compact_rows, dim3(grid1(n)), dim3(256), 0, st, rp, nw, words, wpre, n, m, n0, rp0, nw0, act);
  const int64_t W = (n + 63) / 64;
  if (m > 0) {
    hipLaunchKernelGGL(k_pack_ranks, dim3(grid1(W)), dim3(256), 0, st, words, wpre, W, (RankRec*)rec);
    const int64_t tiles = (m + 2047) / 2048;
    const unsigned G = (unsigned)(tiles < 16384 ? tiles : 16384);
    hipLaunchKernelGGL(k_compact_col, dim3(G), dim3(256), 0, st, col, (const RankRec*)rec, m, col0);
  }
  SCLAP_HIP(hipGetLastError());
  return SCLAP_OK;
}

__global__ void __launch_bounds__(256) k_gather_i32(const int32_t* __restrict__ idx, const int32_t* __restrict__ src,
                                                    int64_t n, int32_t* __restrict__ dst) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) dst[i] = src[idx[i]];
}

__global__ void __launch_bounds__(256) k_scatter_i32(const int32_t* __restrict__ idx, const int32_t* __restrict__ src,
                                                     int64_t n, int32_t* __restrict__ dst) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) dst[idx[i]] = src[i];
}

int gather_i32(const int32_t* idx, const int32_t* src, int64_t n, int32_t* dst, hipStream_t st) {
  if (n <= 0) return SCLAP_OK;
  hipLaunchKernelGGL(k_gather_i32, dim3(grid1(n)), dim3(256), 0, st, idx, src, n, dst);
  SCLAP_HIP(hipGetLastError());
  return SCLAP_OK;
}

int scatter_i32(const int32_t* idx, const int32_t* src, int64_t n, int32_t* dst, hipStream_t st) {
  if (n <= 0) return SCLAP_OK;
  hipLaunchKernelGGL(k_scatter_i32, dim3(grid1(n)), dim3(256), 0, st, idx, src, n, dst);
  SCLAP_HIP(hipGetLastError());
  return SCLAP_OK;
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

// The same from the caller's node weights as given (int32, int64 or NULL
// for unit weights), without a widened copy.
__global__ void __launch_bounds__(256) k_block_weights_raw(const int32_t* __restrict__ part,
                                                           const void* __restrict__ nw, int bytes, int64_t n,
                                                           int32_t k, int64_t* __restrict__ W) {
  extern __shared__ unsigned long long hist[];
  for (int b = threadIdx.x; b < k; b += blockDim.x) hist[b] = 0;
  __syncthreads();
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += stride) {
    const int32_t b = part[v];
    if (b < 0) continue;
    const int64_t c = !nw ? 1 : bytes == 4 ? (int64_t)((const int32_t*)nw)[v] : ((const int64_t*)nw)[v];
    atomicAdd(&hist[b], (unsigned long long)c);
  }
  __syncthreads();
  for (int b = threadIdx.x; b < k; b += blockDim.x)
    if (hist[b]) atomicAdd((unsigned long long*)&W[b], hist[b]);
}

int block_weights_raw(const int32_t* part, const void* nw, int nw_bytes, int64_t n, int32_t k, int64_t* W,
                      hipStream_t st) {
  if (k > kBlockWeightsLdsK) return fail(SCLAP_EINVAL, "block_weights_raw: k above the LDS histogram");
  SCLAP_TRY(fill_i64(W, k, 0, st));
  if (n <= 0) return SCLAP_OK;
  hipLaunchKernelGGL(k_block_weights_raw, dim3(grid1(n, 1024)), dim3(256), (size_t)k * 8, st, part, nw, nw_bytes, n,
                     k, W);
  SCLAP_HIP(hipGetLastError());
  return SCLAP_OK;
}

int block_weights(const int32_t* part, const int64_t* nw, int64_t n, int32_t k, int64_t* W, hipStream_t st) {
  SCLAP_TRY(fill_i64(W, k, 0, st));
  if (n <= 0) return SCLAP_OK;
  const size_t sh = k <= 4096 ? (size_t)k * 8 : 0;
  hipLaunchKernelGGL(k_block_weights, dim3(grid1(n, 1024)), dim3(256), sh, st, part, nw, n, k, W);
  SCLAP_HIP(hipGetLastError());
  return SCLAP_OK;
}

// Cut: sum of w(u, v) over the entries with u < v and part(u) != part(v) (one
// per undirected edge of the symmetric graph).  Nodes with part -1 have no
// entries.
template <typename P>
__global__ void __launch_bounds__(256) k_cut(const int64_t* __restrict__ rp, const int32_t* __restrict__ col,
                                             const int32_t* __restrict__ ew, const P* __restrict__ part,
                                             int64_t n, int64_t m, int64_t* __restrict__ partial,
                                             const int32_t* __restrict__ trow) {
  __shared__ int64_t s_rp[kRpLds];
  __shared__ int64_t s_bounds[3];
  int64_t acc = 0;
  for (int64_t E0 = (int64_t)blockIdx.x * kEpb; E0 < m; E0 += (int64_t)gridDim.x * kEpb) {
    const EdgeRange r = edge_range(rp, n, m, E0, s_rp, s_bounds, trow);
    // the tile's columns first, so their loads are in flight together
    int32_t v[kItems];
#pragma unroll
    for (int j = 0; j < kItems; ++j) {
      const int64_t e = E0 + j * 256 + threadIdx.x;
      v[j] = e < r.e1 ? col[e] : -1;
    }
#pragma unroll
    for (int j = 0; j < kItems; ++j) {
      const int64_t e = E0 + j * 256 + threadIdx.x;
      if (e >= r.e1) continue;
      const int64_t u = edge_row(rp, r, s_rp, e);
      // each undirected edge once: its entry with u < v (the graph is symmetric)
      if (u < v[j] && part[u] != part[v[j]]) acc += ew ? ew[e] : 1;
    }
  }
  __shared__ int64_t red[4];
  for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off);
  if (lane() == 0) red[threadIdx.x / kWave] = acc;
  __syncthreads();
  if (threadIdx.x == 0) partial[blockIdx.x] = red[0] + red[1] + red[2] + red[3];
}

// out = sum of the k partial results (one workgroup).
__global__ void __launch_bounds__(256) k_sum_partials(const int64_t* __restrict__ partial, int k,
                                                      unsigned long long* __restrict__ out) {
  __shared__ int64_t red[4];
  int64_t a = 0;
  for (int i = threadIdx.x; i < k; i += blockDim.x) a += partial[i];
  for (int off = 32; off > 0; off >>= 1) a += __shfl_xor(a, off);
  if (lane() == 0) red[threadIdx.x / kWave] = a;
  __syncthreads();
  if (threadIdx.x == 0) *out = (unsigned long long)(red[0] + red[1] + red[2] + red[3]);
}

static inline unsigned grid_edges(int64_t m) {
  int64_t g = (m + kEpb - 1) / kEpb;
  if (g < 1) g = 1;
  return (unsigned)(g < 8192 ? g : 8192);
}



// The tile-row table of edges.h: one thread per row writes the tile starts
// that fall in its row; each tile start lies in exactly one non-empty row.
__global__ void __launch_bounds__(256) k_tile_rows(const int64_t* __restrict__ rp, int64_t n, int64_t m,
                                                   int32_t* __restrict__ trow) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += stride) {
    const int64_t a = rp[v], b = rp[v + 1];
    for (int64_t t = (a + kEpb - 1) / kEpb; t * kEpb < b; ++t) trow[t] = (int32_t)v;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) trow[(m + kEpb - 1) / kEpb] = (int32_t)(n - 1);
}

int64_t tile_rows_len(int64_t m) { return (m + kEpb - 1) / kEpb + 1; }

int tile_rows(const int64_t* rp, int64_t n, int64_t m, int32_t* trow, hipStream_t st) {
  if (n <= 0 || m <= 0) return SCLAP_OK;
  hipLaunchKernelGGL(k_tile_rows, dim3(grid1(n)), dim3(256), 0, st, rp, n, m, trow);
  SCLAP_HIP(hipGetLastError());
  return SCLAP_OK;
}

int cut_partials(int64_t m) { return (int)grid_edges(m); }

__global__ void __launch_bounds__(256) k_narrow_u8(const int32_t* __restrict__ a, int64_t n,
                                                   uint8_t* __restrict__ b) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += stride) b[v] = (uint8_t)a[v];
}

int narrow_u8(const int32_t* a, int64_t n, uint8_t* b, hipStream_t st) {
  if (n <= 0) return SCLAP_OK;
  hipLaunchKernelGGL(k_narrow_u8, dim3(grid1(n)), dim3(256), 0, st, a, n, b);
  SCLAP_HIP(hipGetLastError());
  return SCLAP_OK;
}

int cut_edges(const int64_t* rp, const int32_t* col, const int32_t* ew, const int32_t* part, int64_t n, int64_t m,
              unsigned long long* out, int64_t* partial, hipStream_t st, const int32_t* trow,
              const uint8_t* part8) {
  SCLAP_TRY(fill_t((uint64_t*)out, 1, (uint64_t)0, st));
  if (n <= 0 || m <= 0) return SCLAP_OK;
  // per-workgroup partial sums, added by one workgroup
  const unsigned G = grid_edges(m);
  if (part8) hipLaunchKernelGGL(k_cut<uint8_t>, dim3(G), dim3(256), 0, st, rp, col, ew, part8, n, m, partial, trow);
  else hipLaunchKernelGGL(k_cut<int32_t>, dim3(G), dim3(256), 0, st, rp, col, ew, part, n, m, partial, trow);
  hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(256), 0, st, partial, (int)G, out);
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

// Emit the entries that join different coarse nodes, as keys
// min(x, y) * 2^b + max(x, y) with their weights, in one pass: each tile of
// kEpb entries reserves its range of the output with one atomic on *cursor
// and writes its keys there in entry order.  The tiles' ranges come in
// scheduling order, which the sort that follows makes irrelevant: the
// reduction sums the weights of equal keys.
__global__ void __launch_bounds__(256) k_cross(const int64_t* __restrict__ rp, const int32_t* __restrict__ col,
                                               const int32_t* __restrict__ ew, const int32_t* __restrict__ cof,
                                               int64_t n, int64_t m, int bits, unsigned long long* __restrict__ cursor,
                                               uint64_t* __restrict__ keys, int32_t* __restrict__ vals, int packed,
                                               const int32_t* __restrict__ trow) {
  __shared__ int64_t s_rp[kRpLds];
  __shared__ int64_t s_bounds[3];
  __shared__ uint32_t s_cnt[4][kItems];
  __shared__ unsigned long long s_base;
  constexpr uint64_t kSame = ~0ull;
  const int w = threadIdx.x / kWave;
  const uint64_t lt = (1ull << lane()) - 1ull;
  for (int64_t E0 = (int64_t)blockIdx.x * kEpb; E0 < m; E0 += (int64_t)gridDim.x * kEpb) {
    const EdgeRange r = edge_range(rp, n, m, E0, s_rp, s_bounds, trow);
    int32_t vv[kItems];
#pragma unroll
    for (int j = 0; j < kItems; ++j) {
      const int64_t e = E0 + j * 256 + threadIdx.x;
      vv[j] = e < r.e1 ? col[e] : -1;
    }
    uint64_t kk[kItems];
#pragma unroll
    for (int j = 0; j < kItems; ++j) {
      const int64_t e = E0 + j * 256 + threadIdx.x;
      kk[j] = kSame;
      if (e >= r.e1) continue;
      // the graph is symmetric with equal weights: the entry (u, v) with
      // u < v stands for its undirected edge (only its endpoints' coarse
      // ids are gathered), keyed by the coarse pair in ascending order;
      // the mirror is added after the reduction
      const int64_t u = edge_row(rp, r, s_rp, e);
      const int32_t v = vv[j];
      if (u < v) {
        const int32_t x = cof[u], y = cof[v];
        if (x != y) {
          const int32_t lo = x < y ? x : y, hi = x < y ? y : x;
          kk[j] = ((uint64_t)(uint32_t)lo << bits) | (uint64_t)(uint32_t)hi;
        }
      }
    }
    // ranks: entry-slot j of wave w takes the places after every earlier
    // slot of the tile and the same slot of earlier waves
    uint32_t rank[kItems];
#pragma unroll
    for (int j = 0; j < kItems; ++j) {
      const uint64_t bl = __ballot(kk[j] != kSame);
      rank[j] = (uint32_t)__popcll(bl & lt);
      if (lane() == 0) s_cnt[w][j] = (uint32_t)__popcll(bl);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      unsigned long long total = 0;
      for (int j = 0; j < kItems; ++j) total += s_cnt[0][j] + s_cnt[1][j] + s_cnt[2][j] + s_cnt[3][j];
      s_base = total ? atomicAdd(cursor, total) : 0ull;
    }
    __syncthreads();
    int64_t base = (int64_t)s_base;
#pragma unroll
    for (int j = 0; j < kItems; ++j) {
      int64_t before = 0;
      for (int q = 0; q < w; ++q) before += s_cnt[q][j];
      if (kk[j] != kSame) {
        const int64_t pos = base + before + rank[j];
        const int32_t wgt = ew ? ew[E0 + j * 256 + threadIdx.x] : 1;
        // packed: key << 32 | weight in one item (keys of at most 32 bits)
        keys[pos] = packed ? (kk[j] << 32) | (uint32_t)wgt : kk[j];
        if (vals) vals[pos] = wgt;
      }
      base += s_cnt[0][j] + s_cnt[1][j] + s_cnt[2][j] + s_cnt[3][j];
    }
  }
}

// Mirror of the reduced upper entries: (x, y, w) -> key y * 2^bits + x with
// weight w (packed: key << 32 | w), for the lower half of the coarse CSR.
__global__ void __launch_bounds__(256) k_coarse_mirror(const uint64_t* __restrict__ ukeys,
                                                       const int64_t* __restrict__ aggs, int64_t m, int bits,
                                                       int packed, uint64_t* __restrict__ mkeys,
                                                       int32_t* __restrict__ mw, unsigned* __restrict__ overflow) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const uint64_t mask = (1ull << bits) - 1ull;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m; i += stride) {
    const uint64_t k = ukeys[i];
    const uint64_t mk = ((k & mask) << bits) | (k >> bits);
    const int64_t a = aggs[i];
    if (a > INT32_MAX) *overflow = 1;
    if (packed) {
      mkeys[i] = (mk << 32) | (uint32_t)(int32_t)a;
    } else {
      mkeys[i] = mk;
      mw[i] = (int32_t)a;
    }
  }
}

// Row starts of the two sorted halves (upper: keys; lower: mirrored keys,
// compared above bit mshift) and of the coarse CSR: rp = ru + rl.
__global__ void __launch_bounds__(256) k_coarse_rowptr2(const uint64_t* __restrict__ ukeys, int64_t mu,
                                                        const uint64_t* __restrict__ lkeys, int64_t ml, int bits,
                                                        int lshift, int64_t nc, int64_t* __restrict__ ru,
                                                        int64_t* __restrict__ rl, int64_t* __restrict__ rp) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; x <= nc; x += stride) {
    const uint64_t key = (uint64_t)x << bits;
    int64_t lo = 0, hi = mu;
    while (lo < hi) {
      const int64_t mid = (lo + hi) >> 1;
      if (ukeys[mid] < key) lo = mid + 1;
      else hi = mid;
    }
    const int64_t a = lo;
    const uint64_t lkey = key << lshift;
    lo = 0;
    hi = ml;
    while (lo < hi) {
      const int64_t mid = (lo + hi) >> 1;
      if (lkeys[mid] < lkey) lo = mid + 1;
      else hi = mid;
    }
    ru[x] = a;
    rl[x] = lo;
    rp[x] = a + lo;
  }
}

// Row x of the coarse CSR: its lower entries (neighbours < x, from the sorted
// mirror) then its upper entries (neighbours > x), each ascending.  Upper
// entry i of row x lands at rp(x) + (rl(x+1) - rl(x)) + (i - ru(x)) =
// i + rl(x+1); lower entry j of row y at rp(y) + (j - rl(y)) = j + ru(y).
__global__ void __launch_bounds__(256) k_coarse_place(const uint64_t* __restrict__ ukeys,
                                                      const int64_t* __restrict__ aggs, int64_t mu,
                                                      const uint64_t* __restrict__ lkeys,
                                                      const int32_t* __restrict__ lw, int64_t ml, int bits,
                                                      int packed, const int64_t* __restrict__ ru,
                                                      const int64_t* __restrict__ rl, int32_t* __restrict__ col,
                                                      int32_t* __restrict__ ew) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const uint64_t mask = (1ull << bits) - 1ull;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < mu + ml; i += stride) {
    if (i < mu) {
      const uint64_t k = ukeys[i];
      const int64_t pos = i + rl[(k >> bits) + 1];
      col[pos] = (int32_t)(k & mask);
      ew[pos] = (int32_t)aggs[i];
    } else {
      const int64_t j = i - mu;
      const uint64_t item = lkeys[j];
      const uint64_t k = packed ? item >> 32 : item;
      const int64_t pos = j + ru[k >> bits];
      col[pos] = (int32_t)(k & mask);
      ew[pos] = packed ? (int32_t)(uint32_t)item : lw[j];
    }
  }
}

int contract_mirror(const uint64_t* ukeys, const int64_t* aggs, int64_t m, int bits, int packed, uint64_t* mkeys,
                    int32_t* mw, unsigned* overflow, hipStream_t st) {
  if (m <= 0) return SCLAP_OK;
  hipLaunchKernelGGL(k_coarse_mirror, dim3(grid1(m)), dim3(256), 0, st, ukeys, aggs, m, bits, packed, mkeys, mw,
                     overflow);
  SCLAP_HIP(hipGetLastError());
  return SCLAP_OK;
}

int contract_finish2(const uint64_t* ukeys, const int64_t* aggs, int64_t mu, const uint64_t* lkeys, const int32_t* lw,
                     int64_t ml, int bits, int packed, int64_t nc, int64_t* ru, int64_t* rl, int64_t* rp,
                     int32_t* col, int32_t* ew, hipStream_t st) {
  hipLaunchKernelGGL(k_coarse_rowptr2, dim3(grid1(nc + 1)), dim3(256), 0, st, ukeys, mu, lkeys, ml, bits,
                     packed ? 32 : 0, nc, ru, rl, rp);
  if (mu + ml > 0)
    hipLaunchKernelGGL(k_coarse_place, dim3(grid1(mu + ml)), dim3(256), 0, st, ukeys, aggs, mu, lkeys, lw, ml, bits,
                       packed, ru, rl, col, ew);
  SCLAP_HIP(hipGetLastError());
  return SCLAP_OK;
}

int contract_flag(const int32_t* lab, const int64_t* rp, int64_t n, int drop, int32_t* used, hipStream_t st) {
  SCLAP_TRY(fill_i32(used, n, 0, st));
  if (n <= 0) return SCLAP_OK;
  hipLaunchKernelGGL(k_flag_used, dim3(grid1(n)), dim3(256), 0, st, lab, rp, n, drop, used);
  SCLAP_HIP(hipGetLastError());
  return SCLAP_OK;
}

// coarse_of(v) = rank of lab(v) only (weights come from the label weights).
__global__ void __launch_bounds__(256) k_coarse_map(const int32_t* __restrict__ lab, const int64_t* __restrict__ rp,
                                                    int64_t n, int drop, const int32_t* __restrict__ cid,
                                                    int32_t* __restrict__ cof) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += stride)
    cof[v] = (drop && rp[v + 1] == rp[v]) ? -1 : cid[lab[v]];
}

// c'(cid(t)) = W(t) for every used label t: the weight of a cluster is the
// weight of its coarse node, written by the label's single owner thread.
__global__ void __launch_bounds__(256) k_coarse_w(const int32_t* __restrict__ used, const int32_t* __restrict__ cid,
                                                  const int64_t* __restrict__ W, int64_t nlabels,
                                                  int64_t* __restrict__ cnw) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < nlabels; t += stride)
    if (used[t]) cnw[cid[t]] = W[t];
}

int contract_coarse_of(const int32_t* lab, const int64_t* rp, const int64_t* nw, int64_t n, int drop,
                       const int32_t* cid, int32_t* cof, int64_t* cnw, int64_t nc, const int32_t* used,
                       const int64_t* W, hipStream_t st) {
  if (W) {
    if (n <= 0) return SCLAP_OK;
    hipLaunchKernelGGL(k_coarse_map, dim3(grid1(n)), dim3(256), 0, st, lab, rp, n, drop, cid, cof);
    hipLaunchKernelGGL(k_coarse_w, dim3(grid1(n)), dim3(256), 0, st, used, cid, W, n, cnw);
    SCLAP_HIP(hipGetLastError());
    return SCLAP_OK;
  }
  SCLAP_TRY(fill_i64(cnw, nc, 0, st));
  if (n <= 0) return SCLAP_OK;
  hipLaunchKernelGGL(k_coarse_of, dim3(grid1(n)), dim3(256), 0, st, lab, rp, nw, n, drop, cid, cof, cnw);
  SCLAP_HIP(hipGetLastError());
  return SCLAP_OK;
}

int contract_cross(const int64_t* rp, const int32_t* col, const int32_t* ew, const int32_t* cof, int64_t n,
                   int64_t m, int bits, unsigned long long* cursor, uint64_t* keys, int32_t* vals, int packed,
                   const int32_t* trow, hipStream_t st) {
  SCLAP_TRY(fill_t((uint64_t*)cursor, 1, (uint64_t)0, st));
  if (n <= 0 || m <= 0) return SCLAP_OK;
  hipLaunchKernelGGL(k_cross, dim3(grid_edges(m)), dim3(256), 0, st, rp, col, ew, cof, n, m, bits, cursor, keys, vals,
                     packed, trow);
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

// One workgroup owns a graph's search state; its waves share the CU's
// caches and order their accesses with workgroup barriers, and kernel
// boundaries order them with the grid-wide level kernels.  Plain accesses
// therefore suffice (no device-scope coherence is needed).
template <class T>
__device__ __forceinline__ T ld_acq(const T* p) {
  return gld(p, 0);
}
template <class T>
__device__ __forceinline__ void st_rel(T* p, T v) {
  gst(p, 0, v);
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

// The same without the leading barrier: the caller guarantees that no thread
// still reads sh from an earlier scan (a barrier since its last use).
__device__ int64_t block_exscan_nb(int64_t x, int64_t* excl, int64_t* sh) {
  int64_t incl = x;
  for (int off = 1; off < kWave; off <<= 1) {
    const int64_t o = __shfl_up(incl, off);
    if ((int)lane() >= off) incl += o;
  }
  const int w = threadIdx.x / kWave;
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

// largest l in [0, cnt) with pre[l] <= x (LDS)
__device__ __forceinline__ int lds_upper(const int64_t* pre, int cnt, int64_t x) {
  int lo = 0, hi = cnt - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (pre[mid] <= x) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

// LDS search state of graphs of at most kIpBitmapNodes nodes: a visited bit
// per node (kept equal to pos != -1) and a claim table for levels of at most
// kIpFastEntries entries (kIpClaimSlots keys, a neighbour id -> its first
// entry index).
constexpr int64_t kIpBitmapNodes = 1 << 18;
constexpr int kIpFastEntries = 4 * kIpThreads;
constexpr int kIpClaimSlots = 2 * kIpFastEntries;

size_t ip_dynamic_lds(int64_t max_n) {
  if (max_n > kIpBitmapNodes) return 0;
  return (size_t)((max_n + 31) / 32 + 2 * kIpClaimSlots) * 4;
}

__device__ __forceinline__ bool bm_test(const uint32_t* bm, int32_t u) { return (bm[u >> 5] >> (u & 31)) & 1u; }
__device__ __forceinline__ void bm_set(uint32_t* bm, int32_t u) { atomicOr(&bm[u >> 5], 1u << (u & 31)); }

// state[0..3] = head, tail, next seed, yielded flag.  With allow_yield the
// kernel stops before a level whose frontier has more than big_entries
// stored entries (rows ascending only); the host expands that level with
// grid-wide kernels and relaunches.  bm_words > 0: the dynamic LDS holds the
// visited bitmap (bm_words words, at least (n + 31) / 32) and the claim table.
__global__ void __launch_bounds__(kIpThreads) k_ip_bfs(const IpSlot* __restrict__ slots, int allow_yield,
                                                      int64_t big_entries, int bm_words) {
  const IpSlot sl = slots[blockIdx.x];
  __shared__ int64_t sh[kIpWaves];
  __shared__ int64_t sh2[kIpWaves];  // the claim-count scan of the LDS fast path
  __shared__ int64_t s_head, s_tail, s_next;
  __shared__ int s_frv;  // the frontier's rows are in LDS: start in s_e0, degree in s_pre
  __shared__ int64_t s_pre[kIpThreads];
  __shared__ int64_t s_e0[kIpThreads];
  extern __shared__ uint32_t s_dyn[];
  uint32_t* bm = bm_words > 0 ? s_dyn : nullptr;
  int32_t* ckey = (int32_t*)(s_dyn + bm_words);
  int32_t* cval = ckey + kIpClaimSlots;
  const int64_t n = sl.n;
  const int wv = threadIdx.x / kWave;
  if (threadIdx.x == 0) {
    s_head = sl.state[0];
    s_tail = sl.state[1];
    s_next = sl.state[2];
    s_frv = 0;
  }
  if (bm) {
    // the visited bits of the current state (the grid-wide level kernels
    // between launches update pos only)
    for (int j = threadIdx.x; j < bm_words; j += kIpThreads) bm[j] = 0;
    __syncthreads();
    for (int64_t v = threadIdx.x; v < n; v += kIpThreads)
      if (ld_acq(&sl.pos[v]) != -1) bm_set(bm, (int32_t)v);
  }
  __syncthreads();
  for (;;) {
    // thread 0 updates these at the end of an iteration, after a barrier
    // that follows every thread's read here
    __syncthreads();
    const int64_t head = s_head, tail = s_tail, next = s_next;
    const bool frv = s_frv != 0;
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
        unv = bm ? !bm_test(bm, (int32_t)id) : ld_acq(&sl.pos[id]) == -1;
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
        if (bm) bm_set(bm, (int32_t)id);
      }
      __syncthreads();
      if (threadIdx.x == 0) {
        s_frv = 0;
        s_tail = tail + tot;
        s_next = first != INT64_MAX ? first + 1 : next + kIpThreads;
        // degree-0 nodes have nothing to expand: the frontier is the seed
        s_head = first != INT64_MAX ? tail + tot - 1 : tail + tot;
      }
      continue;
    }
    const int64_t F = tail - head;
    bool E_known = false;
    if (sl.rows_sorted && F <= kIpThreads) {
      // a frontier of one chunk: its rows are read once; with at most one
      // entry per thread, each thread keeps its entry through the claim and
      // emit passes, and the new nodes' positions are written at once
      int64_t d = 0, e0 = 0;
      if ((int64_t)threadIdx.x < F) {
        if (frv) {
          e0 = s_e0[threadIdx.x];
          d = s_pre[threadIdx.x];
        } else {
          const int32_t f = ld_acq(&sl.order[head + threadIdx.x]);
          e0 = sl.rp[f];
          d = sl.rp[f + 1] - e0;
        }
      }
      int64_t ex;
      // sh was last read before the barrier above
      const int64_t Tc = block_exscan_nb(d, &ex, sh);
      if (allow_yield && Tc > big_entries) {
        if (threadIdx.x == 0) {
          sl.state[0] = head;
          sl.state[1] = tail;
          sl.state[2] = next;
          sl.state[3] = 1;
        }
        return;
      }
      E_known = true;
      if (bm && Tc <= kIpFastEntries) {
        // claims in LDS: a neighbour goes to its first entry in frontier
        // order (= the smallest frontier position), read from the claim table.
        // Thread t takes the consecutive entries tQ .. tQ+Q-1, so one scan of
        // the per-thread claim counts orders the new nodes; their rows are
        // loaded with the candidates and left in LDS for the next level.
        s_pre[threadIdx.x] = ex;
        s_e0[threadIdx.x] = e0;
        for (int j = threadIdx.x; j < kIpClaimSlots; j += kIpThreads) {
          ckey[j] = -1;
          cval[j] = INT32_MAX;
        }
        __syncthreads();
        constexpr int Q = kIpFastEntries / kIpThreads;
        const int64_t i0 = (int64_t)threadIdx.x * Q;
        int32_t uq[Q];
        bool hq[Q];
        int l = i0 < Tc ? lds_upper(s_pre, (int)F, i0) : 0;
#pragma unroll
        for (int q = 0; q < Q; ++q) {
          const int64_t idx = i0 + q;
          hq[q] = idx < Tc;
          uq[q] = 0;
          if (hq[q]) {
            while (l + 1 < (int)F && s_pre[l + 1] <= idx) ++l;
            uq[q] = sl.col[s_e0[l] + idx - s_pre[l]];
          }
        }
        int64_t re0[Q], re1[Q];
#pragma unroll
        for (int q = 0; q < Q; ++q) {
          hq[q] = hq[q] && !bm_test(bm, uq[q]);
          re0[q] = re1[q] = 0;
          if (hq[q]) {
            re0[q] = sl.rp[uq[q]];
            re1[q] = sl.rp[uq[q] + 1];
          }
        }
        // at most kIpFastEntries keys in 2 x kIpFastEntries slots: a probe
        // ends long before it has seen every slot (else the partition fails)
#pragma unroll
        for (int q = 0; q < Q; ++q) {
          if (!hq[q]) continue;
          uint32_t h = hash32((uint32_t)uq[q]) & (kIpClaimSlots - 1);
          for (int probes = 0;; ++probes) {
            if (probes == kIpClaimSlots) {
              atomicOr(sl.err, 1u);
              hq[q] = false;
              break;
            }
            const int32_t prev = atomicCAS(&ckey[h], -1, uq[q]);
            if (prev == -1 || prev == uq[q]) {
              atomicMin(&cval[h], (int32_t)(i0 + q));
              break;
            }
            h = (h + 1) & (kIpClaimSlots - 1);
          }
        }
        int32_t rd[Q];  // degrees of the candidates (at most n)
#pragma unroll
        for (int q = 0; q < Q; ++q) rd[q] = (int32_t)(re1[q] - re0[q]);
        __syncthreads();
        bool ch[Q];
        int64_t mine = 0;
#pragma unroll
        for (int q = 0; q < Q; ++q) {
          ch[q] = false;
          if (hq[q]) {
            uint32_t h = hash32((uint32_t)uq[q]) & (kIpClaimSlots - 1);
            for (int probes = 0; ckey[h] != uq[q] && probes < kIpClaimSlots; ++probes)
              h = (h + 1) & (kIpClaimSlots - 1);
            ch[q] = ckey[h] == uq[q] && cval[h] == (int32_t)(i0 + q);
          }
          mine += ch[q] ? 1 : 0;
        }
        int64_t p;
        // sh2 was last read in the previous level; the LDS rows read above
        // were read before the claim barrier
        const int64_t T = block_exscan_nb(mine, &p, sh2);
#pragma unroll
        for (int q = 0; q < Q; ++q) {
          if (!ch[q]) continue;
          st_rel(&sl.order[tail + p], uq[q]);
          st_rel(&sl.pos[uq[q]], (int32_t)(tail + p));
          bm_set(bm, uq[q]);
          if (p < kIpThreads) {
            s_e0[p] = re0[q];
            s_pre[p] = rd[q];
          }
          ++p;
        }
        __syncthreads();
        if (threadIdx.x == 0) {
          s_head = tail;
          s_tail = tail + T;
          s_frv = T <= kIpThreads ? 1 : 0;
        }
        continue;
      }
      if (Tc <= kIpThreads) {
        s_pre[threadIdx.x] = ex;
        s_e0[threadIdx.x] = e0;
        __syncthreads();
        const bool has = (int64_t)threadIdx.x < Tc;
        int32_t u = 0;
        int l = 0;
        if (has) {
          l = lds_upper(s_pre, (int)F, threadIdx.x);
          u = sl.col[s_e0[l] + threadIdx.x - s_pre[l]];
          if (ld_acq(&sl.pos[u]) == -1) atomicMin(&sl.claim[u], (int32_t)l);
        }
        __syncthreads();
        const bool ch = has && ld_acq(&sl.claim[u]) == (int32_t)l && ld_acq(&sl.pos[u]) == -1;
        int64_t cx;
        const int64_t T = block_exscan(ch ? 1 : 0, &cx, sh);  // all reads above precede the writes
        if (ch) {
          st_rel(&sl.order[tail + cx], u);
          st_rel(&sl.pos[u], (int32_t)(tail + cx));
        }
        __syncthreads();
        if (threadIdx.x == 0) {
          s_head = tail;
          s_tail = tail + T;
          s_frv = 0;
        }
        continue;
      }
    }
    if (allow_yield && sl.rows_sorted && !E_known) {
      int64_t E = 0;
      for (int64_t fc = 0; fc < F; fc += kIpThreads) {
        const int64_t fi = fc + threadIdx.x;
        int64_t d = 0;
        if (fi < F) {
          const int32_t f = ld_acq(&sl.order[head + fi]);
          d = sl.rp[f + 1] - sl.rp[f];
        }
        int64_t ex;
        E += block_exscan(d, &ex, sh);
        __syncthreads();
      }
      if (E > big_entries) {
        if (threadIdx.x == 0) {
          sl.state[0] = head;
          sl.state[1] = tail;
          sl.state[2] = next;
          sl.state[3] = 1;
        }
        return;
      }
    }
    // pass A: every unvisited neighbour takes the smallest frontier position
    for (int64_t fc = 0; fc < F; fc += kIpThreads) {
      const int64_t fi = fc + threadIdx.x;
      int64_t d = 0, e0 = 0;
      if (fi < F) {
        const int32_t f = ld_acq(&sl.order[head + fi]);
        e0 = sl.rp[f];
        d = sl.rp[f + 1] - e0;
      }
      int64_t ex;
      const int64_t Tc = block_exscan(d, &ex, sh);
      s_pre[threadIdx.x] = ex;
      s_e0[threadIdx.x] = e0;
      __syncthreads();
      const int nf = (int)(F - fc < kIpThreads ? F - fc : kIpThreads);
      for (int64_t idx = threadIdx.x; idx < Tc; idx += kIpThreads) {
        const int l = lds_upper(s_pre, nf, idx);
        const int32_t u = sl.col[s_e0[l] + idx - s_pre[l]];
        if (ld_acq(&sl.pos[u]) == -1) atomicMin(&sl.claim[u], (int32_t)(fc + l));
      }
      __syncthreads();
    }
    __syncthreads();
    int64_t T = 0;
    if (sl.rows_sorted) {
      // pass B: children in frontier order, each frontier node's children in
      // row order = ascending id
      for (int64_t fc = 0; fc < F; fc += kIpThreads) {
        const int64_t fi = fc + threadIdx.x;
        int64_t d = 0, e0 = 0;
        if (fi < F) {
          const int32_t f = ld_acq(&sl.order[head + fi]);
          e0 = sl.rp[f];
          d = sl.rp[f + 1] - e0;
        }
        int64_t ex;
        const int64_t Tc = block_exscan(d, &ex, sh);
        s_pre[threadIdx.x] = ex;
        s_e0[threadIdx.x] = e0;
        __syncthreads();
        const int nf = (int)(F - fc < kIpThreads ? F - fc : kIpThreads);
        for (int64_t ib = 0; ib < Tc; ib += kIpThreads) {
          const int64_t idx = ib + threadIdx.x;
          bool ch = false;
          int32_t u = 0;
          if (idx < Tc) {
            const int l = lds_upper(s_pre, nf, idx);
            u = sl.col[s_e0[l] + idx - s_pre[l]];
            ch = ld_acq(&sl.claim[u]) == (int32_t)(fc + l) && ld_acq(&sl.pos[u]) == -1;
          }
          int64_t cx;
          const int64_t ct = block_exscan(ch ? 1 : 0, &cx, sh);
          if (ch) st_rel(&sl.order[tail + T + cx], u);
          T += ct;
          __syncthreads();
        }
      }
    } else {
      // rows in any order: per frontier node, count children, offsets, and
      // place each child by its rank among the node's children
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
      for (int64_t b = 0; b < F; b += kIpThreads) {
        const int64_t fi = b + threadIdx.x;
        const int64_t c = fi < F ? ld_acq(&sl.cnt[fi]) : 0;
        int64_t ex;
        const int64_t tot = block_exscan(c, &ex, sh);
        if (fi < F) st_rel(&sl.cnt[fi], (int32_t)(T + ex));
        T += tot;
        __syncthreads();
      }
      __syncthreads();
      for (int64_t fi = wv; fi < F; fi += kIpWaves) {
        const int32_t f = ld_acq(&sl.order[head + fi]);
        const int64_t e0 = sl.rp[f], e1 = sl.rp[f + 1];
        const int64_t off = tail + ld_acq(&sl.cnt[fi]);
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
    // pass C: positions of the new nodes
    for (int64_t i = threadIdx.x; i < T; i += kIpThreads) {
      const int32_t u = ld_acq(&sl.order[tail + i]);
      st_rel(&sl.pos[u], (int32_t)(tail + i));
      if (bm) bm_set(bm, u);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      s_head = tail;
      s_tail = tail + T;
      s_frv = 0;
    }
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    sl.state[0] = s_head;
    sl.state[1] = s_tail;
    sl.state[2] = s_next;
    sl.state[3] = 0;
  }
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

// ---- grid-wide expansion of one large BFS level (rows ascending) ----------

// dpre[fi] = degree of frontier node fi (scanned on the host side)
__global__ void __launch_bounds__(256) k_lvl_deg(const IpSlot* __restrict__ slp, int64_t head, int64_t F,
                                                 int64_t* __restrict__ deg) {
  const IpSlot sl = *slp;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t fi = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; fi <= F; fi += stride) {
    if (fi == F) {
      deg[fi] = 0;
      continue;
    }
    const int32_t f = sl.order[head + fi];
    deg[fi] = sl.rp[f + 1] - sl.rp[f];
  }
}

// mode 0: claims; mode 1: child flags (1 = child) per flattened entry
__global__ void __launch_bounds__(256) k_lvl_entries(const IpSlot* __restrict__ slp, int64_t head, int64_t F,
                                                     const int64_t* __restrict__ dpre, int64_t E, int mode,
                                                     int32_t* __restrict__ flags) {
  const IpSlot sl = *slp;
  __shared__ int64_t s_rp[kRpLds];
  __shared__ int64_t s_bounds[3];
  for (int64_t E0 = (int64_t)blockIdx.x * kEpb; E0 < E; E0 += (int64_t)gridDim.x * kEpb) {
    const EdgeRange r = edge_range(dpre, F, E, E0, s_rp, s_bounds);
#pragma unroll
    for (int j = 0; j < kItems; ++j) {
      const int64_t idx = E0 + j * 256 + threadIdx.x;
      if (idx >= r.e1) continue;
      const int64_t fi = edge_row(dpre, r, s_rp, idx);
      const int32_t f = sl.order[head + fi];
      const int32_t u = sl.col[sl.rp[f] + idx - dpre[fi]];
      if (mode == 0) {
        if (sl.pos[u] == -1) atomicMin(&sl.claim[u], (int32_t)fi);
      } else {
        flags[idx] = (sl.claim[u] == (int32_t)fi && sl.pos[u] == -1) ? 1 : 0;
      }
    }
  }
}

__global__ void __launch_bounds__(256) k_lvl_emit(const IpSlot* __restrict__ slp, int64_t head, int64_t tail,
                                                  int64_t F, const int64_t* __restrict__ dpre, int64_t E,
                                                  const int32_t* __restrict__ flags, const int32_t* __restrict__ fpos) {
  const IpSlot sl = *slp;
  __shared__ int64_t s_rp[kRpLds];
  __shared__ int64_t s_bounds[3];
  for (int64_t E0 = (int64_t)blockIdx.x * kEpb; E0 < E; E0 += (int64_t)gridDim.x * kEpb) {
    const EdgeRange r = edge_range(dpre, F, E, E0, s_rp, s_bounds);
#pragma unroll
    for (int j = 0; j < kItems; ++j) {
      const int64_t idx = E0 + j * 256 + threadIdx.x;
      if (idx >= r.e1 || !flags[idx]) continue;
      const int64_t fi = edge_row(dpre, r, s_rp, idx);
      const int32_t f = sl.order[head + fi];
      sl.order[tail + fpos[idx]] = sl.col[sl.rp[f] + idx - dpre[fi]];
    }
  }
}

__global__ void __launch_bounds__(256) k_lvl_pos(const IpSlot* __restrict__ slp, int64_t tail, int64_t T) {
  const IpSlot sl = *slp;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < T; i += stride)
    sl.pos[sl.order[tail + i]] = (int32_t)(tail + i);
}

int initial_partition(const IpSlot* dev_slots, int count, int64_t max_n, int allow_yield, int64_t big_entries,
                      hipStream_t st) {
  if (count <= 0) return SCLAP_OK;
  const size_t lds = ip_dynamic_lds(max_n);
  static bool attr_set = false;
  if (!attr_set) {
    SCLAP_HIP(hipFuncSetAttribute((const void*)k_ip_bfs, hipFuncAttributeMaxDynamicSharedMemorySize,
                                  (int)ip_dynamic_lds(kIpBitmapNodes)));
    attr_set = true;
  }
  const int bm_words = lds ? (int)((max_n + 31) / 32) : 0;
  hipLaunchKernelGGL(k_ip_bfs, dim3(count), dim3(kIpThreads), lds, st, dev_slots, allow_yield, big_entries,
                     bm_words);
  SCLAP_HIP(hipGetLastError());
  return SCLAP_OK;
}

int ip_level_deg(const IpSlot* slot, int64_t head, int64_t F, int64_t* deg, hipStream_t st) {
  hipLaunchKernelGGL(k_lvl_deg, dim3(grid1(F + 1)), dim3(256), 0, st, slot, head, F, deg);
  SCLAP_HIP(hipGetLastError());
  return SCLAP_OK;
}

int ip_level_entries(const IpSlot* slot, int64_t head, int64_t F, const int64_t* dpre, int64_t E, int mode,
                     int32_t* flags, hipStream_t st) {
  if (E <= 0) return SCLAP_OK;
  hipLaunchKernelGGL(k_lvl_entries, dim3(grid_edges(E)), dim3(256), 0, st, slot, head, F, dpre, E, mode, flags);
  SCLAP_HIP(hipGetLastError());
  return SCLAP_OK;
}

int ip_level_emit(const IpSlot* slot, int64_t head, int64_t tail, int64_t F, const int64_t* dpre, int64_t E,
                  const int32_t* flags, const int32_t* fpos, int64_t T, hipStream_t st) {
  if (E > 0)
    hipLaunchKernelGGL(k_lvl_emit, dim3(grid_edges(E)), dim3(256), 0, st, slot, head, tail, F, dpre, E, flags, fpos);
  if (T > 0) hipLaunchKernelGGL(k_lvl_pos, dim3(grid1(T)), dim3(256), 0, st, slot, tail, T);
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
