// common.h -- internal declarations shared by the device library's sources.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>

#include "../../include/sclap.h"

namespace sclap {

constexpr int kWave = 64;

// ---------------------------------------------------------------------------
// Errors: every internal function returns an int status; the message of the
// last failure is kept per thread.
// ---------------------------------------------------------------------------
void set_error(const std::string& msg);
int fail(int code, const std::string& msg);

#define SCLAP_HIP(expr)                                                                        \
  do {                                                                                         \
    hipError_t _e = (expr);                                                                    \
    if (_e != hipSuccess)                                                                      \
      return ::sclap::fail(_e == hipErrorOutOfMemory ? SCLAP_ENOMEM : SCLAP_EHIP,              \
                           std::string(#expr) + ": " + hipGetErrorString(_e));                 \
  } while (0)

#define SCLAP_TRY(expr)      \
  do {                       \
    int _rc = (expr);        \
    if (_rc != SCLAP_OK) return _rc; \
  } while (0)

// ---------------------------------------------------------------------------
// One graph taking part in a fused label-propagation round.  Nodes of all
// slots of a round form one global id space: slot s owns [nbase, nbase + n).
// Labels of slot s live in [0, nlabels) and form the global target range
// [lbase, lbase + nlabels) used to key contended admissions.
// ---------------------------------------------------------------------------
enum : int32_t { MODE_CLUSTER = 0, MODE_REFINE = 1 };

struct DevSlot {
  const int64_t* rp;
  const int32_t* col;
  const int32_t* ew;      // nullptr: unit edge weights
  const int64_t* nw;      // never null
  int32_t* lab;           // n: cluster label / block id (-1: takes no part)
  int32_t* desire;        // n
  uint8_t* adm;           // n: admitted flag of the current round
  int64_t* W;             // nlabels: label weights before the round
  int64_t* inc;           // nlabels: incoming mover weight (kept zero between rounds)
  uint8_t* flag_cur;      // refine: rated set of this round (use_flags)
  uint8_t* flag_next;     // refine: rated set of the next round
  int64_t* ctr;           // device counters of this slot, see CTR_*
  int64_t n;
  int64_t m;              // stored entries of the graph
  int64_t nbase;
  int64_t tbase;          // first binning tile of the slot
  int64_t nlabels;
  int64_t lbase;
  int64_t cap;
  int32_t round;          // 1-based round number; 0: slot idle this step
  int32_t mode;           // MODE_CLUSTER / MODE_REFINE
  int32_t dir_rule;
  int32_t use_flags;      // rate only nodes with flag_cur set
  int32_t conn_k;         // refine: columns of conn (the block count k)
  int32_t conn_mode;      // CONN_NONE / CONN_BUILD / CONN_RATE
  int32_t* conn;          // refine: n x conn_k block connections conn(v, b), or nullptr
  int32_t last_round;     // no LP round of this stage follows (its moves need no bookkeeping)
  int32_t ident;          // first clustering round of a level: lab(v) = v, so a neighbour's label is its id
  int32_t all_elig;       // ident round on a level with 2 max c(v) <= cap: every candidate is eligible
  int32_t bin_hi[4];      // largest degree of bins 3..6 (see bin_of; tuned for clustering slots)
  int32_t sub;            // degree-ordered sub-rounds: the degree class rated in this step
  const uint8_t* cls;     // ... the degree class of every node, or nullptr (every node is rated)
  const uint8_t* lab8;    // CONN_BUILD slots: lab as one byte per node (blocks < 256), or nullptr
  uint32_t* err;          // set nonzero when an LDS hash table of the round fills up (the round fails)
};

// Refinement with block connections kept per node: the first round of a
// level builds them (CONN_BUILD); later rounds rate from them (CONN_RATE),
// and every move updates the rows of the mover's neighbours.  A round whose
// movers are more than 1 / kConnPushDiv of the nodes does not update them (two
// atomics per entry of every mover would cost more than rebuilding): the next
// round rebuilds the rows of its rated nodes, which include every node with a
// moved neighbour.
enum : int { CONN_NONE = 0, CONN_BUILD = 1, CONN_RATE = 2 };
constexpr int kConnMaxK = 64;  // at most one wave of columns
constexpr int64_t kConnPushDiv = 16;

// CTR_STALE: the moves of the round were not added to the block
// connections (the rows of the next rated set are rebuilt instead).
enum : int { CTR_MOVED = 0, CTR_VISITS = 1, CTR_MOVERS = 2, CTR_STALE = 3, CTR_N = 4 };

// Degree bins of the rating kernels:
//   0: 1..8       8 lanes per node        5: 129..512    one wave, 1024-entry LDS table
//   1: 9..16      16 lanes per node       6: 513..1024   one workgroup of 256, LDS table of up to 4096
//   2: 17..32     32 lanes per node       7: 1025..4096  one workgroup, 8192-entry LDS table
//   3: 33..64     one wave, 128-entry LDS 8: > 4096      several workgroups, global table
//   4: 65..128    one wave, 256-entry LDS table
constexpr int kBins = 9;
// Default upper degree bounds of bins 3..6, and the most each bin's kernel
// takes (its table holds twice the degree): bin 3 one wave with 128 slots,
// bin 4 one wave with 256, bin 5 one wave with 1024, bin 6 one workgroup of
// 256 threads with 4096 (bin 7 takes the rest up to 4096 with workgroups of
// 512 and 8192 slots).  The lower bound of bin 3 (33) and of the hub bin
// (4097) are fixed.
constexpr int32_t kBinHiDefault[4] = {64, 128, 512, 1024};
constexpr int32_t kBinHiCap[4] = {64, 128, 512, 2048};
constexpr int kPathCounters = 5;
constexpr int64_t kBinBlock = 4096;

constexpr int kHubChunk = 2048;      // entries per workgroup in the multi-workgroup path
constexpr int kHubPartLabels = 2048; // target distinct labels per label part of a hub
constexpr int kHubMaxParts = 2048;

// Label parts of a hub of degree d: a power of two, about kHubPartLabels
// distinct labels each.
__host__ __device__ __forceinline__ uint32_t hub_parts(int64_t d, int64_t nlabels) {
  const int64_t distinct = d < nlabels ? d : nlabels;
  uint32_t P = 1;
  while (P < (uint32_t)kHubMaxParts && (int64_t)P * kHubPartLabels < distinct) P <<= 1;
  return P;
}

// Loads and stores through the global address space: global_load /
// global_store with an SGPR base, instead of the flat instructions that
// pointers read from a descriptor would otherwise get (flat accesses also
// count against the LDS/scalar wait counter and serialise with them).
#define SCLAP_GLOBAL __attribute__((address_space(1)))
template <class T>
__device__ __forceinline__ T gld(const T* p, int64_t i) {
  return ((const SCLAP_GLOBAL T*)p)[i];
}
template <class T>
__device__ __forceinline__ void gst(T* p, int64_t i, T v) {
  ((SCLAP_GLOBAL T*)p)[i] = v;
}
// Relaxed device-scope atomic sum on a global int64 element.
__device__ __forceinline__ void gadd64(int64_t* p, int64_t i, int64_t v) {
  __hip_atomic_fetch_add((SCLAP_GLOBAL unsigned long long*)(p + i), (unsigned long long)v, __ATOMIC_RELAXED,
                         __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ int slot_of(const DevSlot* __restrict__ S, int ns, int64_t u) {
  int lo = 0, hi = ns - 1;
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if (S[mid].nbase <= u) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

// Candidate key: larger connection wins, then smaller label.  0 = none.
__device__ __forceinline__ uint64_t pack_key(int64_t conn, int32_t t) {
  return ((uint64_t)conn << 32) | (uint64_t)(0xFFFFFFFFu - (uint32_t)t);
}
__device__ __forceinline__ int32_t key_label(uint64_t key) {
  return (int32_t)(0xFFFFFFFFu - (uint32_t)(key & 0xFFFFFFFFu));
}

__device__ __forceinline__ uint32_t hash32(uint32_t x) {
  x ^= x >> 16;
  x *= 0x7feb352dU;
  x ^= x >> 15;
  x *= 0x846ca68bU;
  x ^= x >> 16;
  return x;
}

// ---------------------------------------------------------------------------
// Device memory: stream-ordered allocations from the device's default pool.
// ---------------------------------------------------------------------------
struct Ctx;

template <class T>
struct DBuf {
  T* p = nullptr;
  size_t n = 0;
};

int dalloc(void** p, size_t bytes, hipStream_t st);
void dfree(void* p, hipStream_t st);

template <class T>
int dalloc_t(T** p, size_t count, hipStream_t st) {
  return dalloc(reinterpret_cast<void**>(p), count * sizeof(T), st);
}

// Growable scratch buffer owned by the context.
struct Scratch {
  void* p = nullptr;
  size_t bytes = 0;
  int ensure(size_t need, hipStream_t st);
  void release(hipStream_t st);
};

}  // namespace sclap
