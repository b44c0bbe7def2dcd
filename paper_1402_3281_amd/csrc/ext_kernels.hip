// ext_kernels.hip -- kernels of the extensions of Section 4 of the paper:
//   - the graph without the cut edges of a partition, which the clustering
//     that respects the partition rates (Appendix B.1: a node may only join a
//     cluster inside its own block; every member of such a cluster is in that
//     block, so the neighbours in other blocks never carry a candidate and the
//     choice is that of the plain rating on the filtered graph);
//   - the blocks of the coarse nodes (a coarse node's members share a block);
//   - the degree classes of the degree-ordered sub-rounds;
//   - the initial labels of an ensemble member (an affine permutation);
//   - the overlay of two clusterings, numbered by first occurrence.
#include <hip/hip_runtime.h>

#include "common.h"
#include "edges.h"
#include "ext.h"
#include "lp.h"

namespace sclap {

namespace {

__device__ __forceinline__ uint32_t ext_lane() { return __lane_id(); }

inline unsigned ext_grid(int64_t n, unsigned cap = 8192) {
  int64_t g = (n + 255) / 256;
  if (g < 1) g = 1;
  return (unsigned)(g < cap ? g : cap);
}

}  // namespace

// ---------------------------------------------------------------------------
// The graph without the cut edges of a partition.
// ---------------------------------------------------------------------------

int64_t filter_tiles(int64_t m) { return (m + kEpb - 1) / kEpb; }

// Per tile of kEpb entries: keep bit of every entry (both ends in one block)
// in 64-entry words, the kept entries of the tile before each word, and the
// tile's kept count.  A wave's ballot over 64 consecutive entries is one
// word (tiles start at multiples of kEpb, a multiple of 64).
__global__ void __launch_bounds__(256) k_filter_mark(const int64_t* __restrict__ rp, const int32_t* __restrict__ col,
                                                     const int32_t* __restrict__ blk, int64_t n, int64_t m,
                                                     uint64_t* __restrict__ kw, uint32_t* __restrict__ wpre,
                                                     int64_t* __restrict__ tcnt, const int32_t* __restrict__ trow) {
  __shared__ int64_t s_rp[kRpLds];
  __shared__ int64_t s_bounds[3];
  __shared__ uint32_t s_pc[kEpb / kWave];
  const int w = threadIdx.x / kWave;
  for (int64_t E0 = (int64_t)blockIdx.x * kEpb; E0 < m; E0 += (int64_t)gridDim.x * kEpb) {
    const EdgeRange r = edge_range(rp, n, m, E0, s_rp, s_bounds, trow);
#pragma unroll
    for (int j = 0; j < kItems; ++j) {
      const int64_t e = E0 + j * 256 + threadIdx.x;
      bool keep = false;
      if (e < r.e1) {
        const int64_t u = edge_row(rp, r, s_rp, e);
        keep = blk[u] == blk[col[e]];
      }
      const uint64_t mask = __ballot(keep);
      if (ext_lane() == 0) {
        kw[(E0 + j * 256 + w * kWave) / kWave] = mask;
        s_pc[j * 4 + w] = (uint32_t)__popcll(mask);
      }
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      uint32_t acc = 0;
      const int64_t w0 = E0 / kWave;
      for (int q = 0; q < kEpb / kWave; ++q) {
        wpre[w0 + q] = acc;
        acc += s_pc[q];
      }
      tcnt[E0 / kEpb] = acc;
    }
  }
}

// Kept entries before entry e (e < m): the tile's offset, the tile's kept
// entries before e's word, and those of e's word below e.
__device__ __forceinline__ int64_t kept_before(const uint64_t* __restrict__ kw, const uint32_t* __restrict__ wpre,
                                               const int64_t* __restrict__ toff, int64_t e) {
  const int64_t wd = e / kWave;
  const int bit = (int)(e % kWave);
  const uint64_t below = bit ? (kw[wd] & ((1ull << bit) - 1ull)) : 0ull;
  return toff[e / kEpb] + wpre[wd] + __popcll(below);
}

__global__ void __launch_bounds__(256) k_filter_place(const int32_t* __restrict__ col, const int32_t* __restrict__ ew,
                                                      int64_t m, const uint64_t* __restrict__ kw,
                                                      const uint32_t* __restrict__ wpre,
                                                      const int64_t* __restrict__ toff, int32_t* __restrict__ col2,
                                                      int32_t* __restrict__ ew2) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < m; e += stride) {
    if (!((kw[e / kWave] >> (e % kWave)) & 1ull)) continue;
    const int64_t pos = kept_before(kw, wpre, toff, e);
    col2[pos] = col[e];
    if (ew) ew2[pos] = ew[e];
  }
}

__global__ void __launch_bounds__(256) k_filter_rows(const int64_t* __restrict__ rp, int64_t n, int64_t m,
                                                     const uint64_t* __restrict__ kw,
                                                     const uint32_t* __restrict__ wpre,
                                                     const int64_t* __restrict__ toff, int64_t T,
                                                     int64_t* __restrict__ rp2) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v <= n; v += stride) {
    const int64_t e = rp[v];
    rp2[v] = e >= m ? toff[T] : kept_before(kw, wpre, toff, e);
  }
}

int filter_mark(const int64_t* rp, const int32_t* col, const int32_t* blk, int64_t n, int64_t m, uint64_t* kw,
                uint32_t* wpre, int64_t* tcnt, const int32_t* trow, hipStream_t st) {
  const int64_t T = filter_tiles(m);
  if (T == 0) return SCLAP_OK;
  const unsigned G = (unsigned)(T < 8192 ? T : 8192);
  hipLaunchKernelGGL(k_filter_mark, dim3(G), dim3(256), 0, st, rp, col, blk, n, m, kw, wpre, tcnt, trow);
  SCLAP_HIP(hipGetLastError());
  return SCLAP_OK;
}

int filter_place(const int32_t* col, const int32_t* ew, int64_t m, const uint64_t* kw, const uint32_t* wpre,
                 const int64_t* toff, int32_t* col2, int32_t* ew2, hipStream_t st) {
  if (m <= 0) return SCLAP_OK;
  hipLaunchKernelGGL(k_filter_place, dim3(ext_grid(m)), dim3(256), 0, st, col, ew, m, kw, wpre, toff, col2, ew2);
  SCLAP_HIP(hipGetLastError());
  return SCLAP_OK;
}

int filter_rows(const int64_t* rp, int64_t n, int64_t m, const uint64_t* kw, const uint32_t* wpre,
                const int64_t* toff, int64_t T, int64_t* rp2, hipStream_t st) {
  hipLaunchKernelGGL(k_filter_rows, dim3(ext_grid(n + 1)), dim3(256), 0, st, rp, n, m, kw, wpre, toff, T, rp2);
  SCLAP_HIP(hipGetLastError());
  return SCLAP_OK;
}

// ---------------------------------------------------------------------------
// Blocks of the coarse nodes, degree classes, member labels.
// ---------------------------------------------------------------------------

// Every member of a coarse node carries the same block, so the concurrent
// stores of one coarse node all write the same value.
__global__ void __launch_bounds__(256) k_blocks_up(const int32_t* __restrict__ cof, const int32_t* __restrict__ bf,
                                                   int64_t n, int32_t* __restrict__ bc) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += stride) {
    const int32_t c = cof[v];
    if (c >= 0) bc[c] = bf[v];
  }
}

int blocks_up(const int32_t* cof, const int32_t* bf, int64_t n, int32_t* bc, hipStream_t st) {
  if (n <= 0) return SCLAP_OK;
  hipLaunchKernelGGL(k_blocks_up, dim3(ext_grid(n)), dim3(256), 0, st, cof, bf, n, bc);
  SCLAP_HIP(hipGetLastError());
  return SCLAP_OK;
}

// Class 0 below degree 4, else floor(log4(degree)), at most S - 1.
__global__ void __launch_bounds__(256) k_deg_class(const int64_t* __restrict__ rp, int64_t n, int S,
                                                   uint8_t* __restrict__ cls) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += stride) {
    const int64_t d = rp[v + 1] - rp[v];
    // floor(log4 d) = floor(log2 d) / 2 for d >= 1
    const int c = d >= 4 ? (63 - __clzll((unsigned long long)d)) >> 1 : 0;
    cls[v] = (uint8_t)(c < S - 1 ? c : S - 1);
  }
}

int degree_classes(const int64_t* rp, int64_t n, int S, uint8_t* cls, hipStream_t st) {
  if (n <= 0) return SCLAP_OK;
  hipLaunchKernelGGL(k_deg_class, dim3(ext_grid(n)), dim3(256), 0, st, rp, n, S, cls);
  SCLAP_HIP(hipGetLastError());
  return SCLAP_OK;
}

__global__ void __launch_bounds__(256) k_init_member(int32_t* __restrict__ lab, int32_t* __restrict__ desire,
                                                     int64_t* __restrict__ W, const int64_t* __restrict__ nw,
                                                     int64_t n, uint64_t a, uint64_t b) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += stride) {
    // a, b < n < 2^31 and v < 2^31: the product fits 64 bits
    const int32_t p = (int32_t)((a * (uint64_t)v + b) % (uint64_t)n);
    lab[v] = p;
    desire[v] = p;
    W[p] = nw[v];  // p is a permutation: every label gets exactly one weight
  }
}

static int64_t gcd_i64(int64_t a, int64_t b) {
  while (b) {
    const int64_t t = a % b;
    a = b;
    b = t;
  }
  return a;
}

void member_affine(int64_t n, int32_t e, int64_t* a, int64_t* b) {
  *a = 1;
  *b = 0;
  if (e == 0 || n <= 1) return;
  int64_t x = (int64_t)((2654435761ull * (uint64_t)e) % (uint64_t)n);
  for (;;) {
    if (x == 0) x = 1;
    if (gcd_i64(x, n) == 1) break;
    x = (x + 1) % n;
  }
  *a = x;
  *b = (int64_t)((2246822519ull * (uint64_t)e) % (uint64_t)n);
}

int init_member(int32_t* lab, int32_t* desire, int64_t* W, const int64_t* nw, int64_t n, int32_t e,
                hipStream_t st) {
  if (n <= 0) return SCLAP_OK;
  int64_t a, b;
  member_affine(n, e, &a, &b);
  hipLaunchKernelGGL(k_init_member, dim3(ext_grid(n)), dim3(256), 0, st, lab, desire, W, nw, n, (uint64_t)a,
                     (uint64_t)b);
  SCLAP_HIP(hipGetLastError());
  return SCLAP_OK;
}

// ---------------------------------------------------------------------------
// Overlay (Section 4, ensemble clusterings): nodes sharing (O(v), C(v)) share
// a cluster; clusters are numbered in the order of their smallest node id,
// which is the order in which a pass over the nodes in increasing id first
// meets them.  Keys O << bits | C are sorted with the node ids as values
// (a stable sort of ids in increasing order keeps every key's smallest id
// first).
// ---------------------------------------------------------------------------

__global__ void __launch_bounds__(256) k_ovl_keys(const int32_t* __restrict__ O, const int32_t* __restrict__ C,
                                                  int64_t n, int bits, uint64_t* __restrict__ keys,
                                                  int32_t* __restrict__ vals) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += stride) {
    keys[v] = ((uint64_t)(uint32_t)O[v] << bits) | (uint64_t)(uint32_t)C[v];
    vals[v] = (int32_t)v;
  }
}

__global__ void __launch_bounds__(256) k_ovl_heads(const uint64_t* __restrict__ K, int64_t n,
                                                   int32_t* __restrict__ head) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
    head[i] = (i == 0 || K[i] != K[i - 1]) ? 1 : 0;
}

// segmin[s] = smallest id of key segment s; first[u] = 1 for those ids
// (first zeroed before).  hx: exclusive scan of head.
__global__ void __launch_bounds__(256) k_ovl_first(const int32_t* __restrict__ V, const int32_t* __restrict__ head,
                                                   const int32_t* __restrict__ hx, int64_t n,
                                                   int32_t* __restrict__ segmin, int32_t* __restrict__ first) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
    if (!head[i]) continue;
    const int32_t u = V[i];
    segmin[hx[i]] = u;
    first[u] = 1;
  }
}

// O(V[i]) = rank (by smallest id) of the segment of position i; rank:
// exclusive scan of first.
__global__ void __launch_bounds__(256) k_ovl_assign(const int32_t* __restrict__ V, const int32_t* __restrict__ head,
                                                    const int32_t* __restrict__ hx,
                                                    const int32_t* __restrict__ segmin,
                                                    const int32_t* __restrict__ rank, int64_t n,
                                                    int32_t* __restrict__ O) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
    const int32_t s = hx[i] + head[i] - 1;
    O[V[i]] = rank[segmin[s]];
  }
}

int overlay_keys(const int32_t* O, const int32_t* C, int64_t n, int bits, uint64_t* keys, int32_t* vals,
                 hipStream_t st) {
  if (n <= 0) return SCLAP_OK;
  hipLaunchKernelGGL(k_ovl_keys, dim3(ext_grid(n)), dim3(256), 0, st, O, C, n, bits, keys, vals);
  SCLAP_HIP(hipGetLastError());
  return SCLAP_OK;
}

int overlay_heads(const uint64_t* K, int64_t n, int32_t* head, hipStream_t st) {
  if (n <= 0) return SCLAP_OK;
  hipLaunchKernelGGL(k_ovl_heads, dim3(ext_grid(n)), dim3(256), 0, st, K, n, head);
  SCLAP_HIP(hipGetLastError());
  return SCLAP_OK;
}

int overlay_first(const int32_t* V, const int32_t* head, const int32_t* hx, int64_t n, int32_t* segmin,
                  int32_t* first, hipStream_t st) {
  if (n <= 0) return SCLAP_OK;
  hipLaunchKernelGGL(k_ovl_first, dim3(ext_grid(n)), dim3(256), 0, st, V, head, hx, n, segmin, first);
  SCLAP_HIP(hipGetLastError());
  return SCLAP_OK;
}

int overlay_assign(const int32_t* V, const int32_t* head, const int32_t* hx, const int32_t* segmin,
                   const int32_t* rank, int64_t n, int32_t* O, hipStream_t st) {
  if (n <= 0) return SCLAP_OK;
  hipLaunchKernelGGL(k_ovl_assign, dim3(ext_grid(n)), dim3(256), 0, st, V, head, hx, segmin, rank, n, O);
  SCLAP_HIP(hipGetLastError());
  return SCLAP_OK;
}

}  // namespace sclap
