// prims.hip -- thin wrappers over rocPRIM device-wide primitives (radix sort,
// scans, reduce-by-key), kept in one translation unit.  All of them operate
// on integers, so their results do not depend on scheduling.
#include <hip/hip_runtime.h>

#include <cstring>
#include <string>

#include <rocprim/rocprim.hpp>

#include "lp.h"

namespace sclap {

#define PRIM_CALL(expr)                                                              \
  do {                                                                               \
    hipError_t _e = (expr);                                                          \
    if (_e != hipSuccess) return fail(SCLAP_EHIP, std::string("rocprim: ") + hipGetErrorString(_e)); \
  } while (0)

size_t prim_sort_keys_bytes(size_t n) {
  size_t b = 0;
  (void)rocprim::radix_sort_keys(nullptr, b, (const uint64_t*)nullptr, (uint64_t*)nullptr, n, 0, 64);
  return b;
}

int prim_sort_keys(void* tmp, size_t tmp_bytes, const uint64_t* in, uint64_t* out, size_t n, int end_bit,
                   hipStream_t st, int begin_bit) {
  if (n == 0) return SCLAP_OK;
  // the merge path's bit mask is wrong for ranges that end at bit 64 and
  // start above bit 0 (see lp.h)
  if (begin_bit > 0 && end_bit >= 64) return fail(SCLAP_EINVAL, "radix sort: bit range [b, 64) with b > 0");
  PRIM_CALL(rocprim::radix_sort_keys(tmp, tmp_bytes, in, out, n, (unsigned)begin_bit, (unsigned)end_bit, st));
  return SCLAP_OK;
}

size_t prim_sort_pairs_bytes(size_t n) {
  size_t b = 0;
  (void)rocprim::radix_sort_pairs(nullptr, b, (const uint64_t*)nullptr, (uint64_t*)nullptr, (const int32_t*)nullptr,
                            (int32_t*)nullptr, n, 0, 64);
  return b;
}

int prim_sort_pairs(void* tmp, size_t tmp_bytes, const uint64_t* kin, uint64_t* kout, const int32_t* vin,
                    int32_t* vout, size_t n, int end_bit, hipStream_t st, int begin_bit) {
  if (n == 0) return SCLAP_OK;
  if (begin_bit > 0 && end_bit >= 64) return fail(SCLAP_EINVAL, "radix sort: bit range [b, 64) with b > 0");
  PRIM_CALL(rocprim::radix_sort_pairs(tmp, tmp_bytes, kin, kout, vin, vout, n, (unsigned)begin_bit, (unsigned)end_bit,
                                      st));
  return SCLAP_OK;
}

size_t prim_scan_by_key_bytes(size_t n) {
  size_t b = 0;
  (void)rocprim::inclusive_scan_by_key(nullptr, b, (const uint32_t*)nullptr, (const int64_t*)nullptr, (int64_t*)nullptr,
                                 n, rocprim::plus<int64_t>());
  return b;
}

int prim_scan_by_key(void* tmp, size_t tmp_bytes, const uint32_t* keys, const int64_t* in, int64_t* out, size_t n,
                     hipStream_t st) {
  if (n == 0) return SCLAP_OK;
  PRIM_CALL(rocprim::inclusive_scan_by_key(tmp, tmp_bytes, keys, in, out, n, rocprim::plus<int64_t>(),
                                           rocprim::equal_to<uint32_t>(), st));
  return SCLAP_OK;
}

size_t prim_exscan_i32_bytes(size_t n) {
  size_t b = 0;
  (void)rocprim::exclusive_scan(nullptr, b, (const int32_t*)nullptr, (int32_t*)nullptr, (int32_t)0, n,
                          rocprim::plus<int32_t>());
  return b;
}

int prim_exscan_i32(void* tmp, size_t tmp_bytes, const int32_t* in, int32_t* out, size_t n, hipStream_t st) {
  if (n == 0) return SCLAP_OK;
  PRIM_CALL(rocprim::exclusive_scan(tmp, tmp_bytes, in, out, (int32_t)0, n, rocprim::plus<int32_t>(), st));
  return SCLAP_OK;
}

size_t prim_exscan_i64_bytes(size_t n) {
  size_t b = 0;
  (void)rocprim::exclusive_scan(nullptr, b, (const int64_t*)nullptr, (int64_t*)nullptr, (int64_t)0, n,
                          rocprim::plus<int64_t>());
  return b;
}

int prim_exscan_i64(void* tmp, size_t tmp_bytes, const int64_t* in, int64_t* out, size_t n, hipStream_t st) {
  if (n == 0) return SCLAP_OK;
  PRIM_CALL(rocprim::exclusive_scan(tmp, tmp_bytes, in, out, (int64_t)0, n, rocprim::plus<int64_t>(), st));
  return SCLAP_OK;
}

size_t prim_rle_bytes(size_t n) {
  size_t b = 0;
  (void)rocprim::run_length_encode(nullptr, b, (const uint64_t*)nullptr, (unsigned)n, (uint64_t*)nullptr,
                                   (int64_t*)nullptr, (uint32_t*)nullptr);
  return b;
}

int prim_rle(void* tmp, size_t tmp_bytes, const uint64_t* keys, uint64_t* ukeys, int64_t* counts, uint32_t* runs,
             size_t n, hipStream_t st) {
  PRIM_CALL(rocprim::run_length_encode(tmp, tmp_bytes, keys, (unsigned)n, ukeys, counts, runs, st));
  return SCLAP_OK;
}

// Packed items key << 32 | weight (sorted by key): the upper and lower halves.
struct PackedKey {
  __host__ __device__ uint32_t operator()(uint64_t v) const { return (uint32_t)(v >> 32); }
};
struct PackedWeight {
  __host__ __device__ int64_t operator()(uint64_t v) const { return (int64_t)(uint32_t)v; }
};

size_t prim_reduce_packed_bytes(size_t n) {
  size_t b = 0;
  const uint64_t* p = nullptr;
  (void)rocprim::reduce_by_key(nullptr, b, rocprim::make_transform_iterator(p, PackedKey()),
                               rocprim::make_transform_iterator(p, PackedWeight()), n, (uint64_t*)nullptr,
                               (int64_t*)nullptr, (uint32_t*)nullptr, rocprim::plus<int64_t>());
  return b;
}

int prim_reduce_packed(void* tmp, size_t tmp_bytes, const uint64_t* items, uint64_t* ukeys, int64_t* sums,
                       uint32_t* count, size_t n, hipStream_t st) {
  PRIM_CALL(rocprim::reduce_by_key(tmp, tmp_bytes, rocprim::make_transform_iterator(items, PackedKey()),
                                   rocprim::make_transform_iterator(items, PackedWeight()), n, ukeys, sums, count,
                                   rocprim::plus<int64_t>(), rocprim::equal_to<uint32_t>(), st));
  return SCLAP_OK;
}

size_t prim_reduce_by_key_bytes(size_t n) {
  size_t b = 0;
  (void)rocprim::reduce_by_key(nullptr, b, (const uint64_t*)nullptr, (const int32_t*)nullptr, n, (uint64_t*)nullptr,
                         (int64_t*)nullptr, (uint32_t*)nullptr, rocprim::plus<int64_t>());
  return b;
}

int prim_reduce_by_key(void* tmp, size_t tmp_bytes, const uint64_t* keys, const int32_t* vals, uint64_t* ukeys,
                       int64_t* aggs, uint32_t* count, size_t n, hipStream_t st) {
  PRIM_CALL(rocprim::reduce_by_key(tmp, tmp_bytes, keys, vals, n, ukeys, aggs, count, rocprim::plus<int64_t>(),
                                   rocprim::equal_to<uint64_t>(), st));
  return SCLAP_OK;
}

}  // namespace sclap
