// noalloc.hip -- the cut and block weights (Section 2.1) for callers that
// cannot allocate device memory (code under HIP graph capture, serving
// loops, harnesses that forbid allocation).  The per-workgroup partial sums
// of the cut live in a fixed device array of this file, one copy per GPU,
// instead of the context's growable scratch; the results go to device
// memory the caller passes.  Nothing here allocates.
#include <hip/hip_runtime.h>

#include <mutex>

#include "common.h"
#include "misc.h"

namespace sclap {

// Partial sums of the cut kernel: one per workgroup of its launch, whose grid
// is capped at kNoAllocPartials workgroups for any edge count.
constexpr int kNoAllocPartials = 8192;
static __device__ __align__(256) int64_t scratch[kNoAllocPartials];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_mu;
int64_t* g_scratch[kMaxDevices] = {};  // device address of `scratch` on each GPU
}  // namespace

// Looks up the device address of `scratch` on the current device once (the
// array's name is a host-side stand-in that kernels must not be given).
int noalloc_setup(int device) {
  if (device < 0 || device >= kMaxDevices) return fail(SCLAP_EINVAL, "device index out of range");
  std::lock_guard<std::mutex> lk(g_mu);
  if (g_scratch[device]) return SCLAP_OK;
  int cur = -1;
  SCLAP_HIP(hipGetDevice(&cur));
  if (cur != device) SCLAP_HIP(hipSetDevice(device));
  void* p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (cur != device) (void)hipSetDevice(cur);
  if (e != hipSuccess || !p)
    return fail(SCLAP_EHIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
  g_scratch[device] = (int64_t*)p;
  return SCLAP_OK;
}

}  // namespace sclap

using namespace sclap;

extern "C" int sclap_cut_noalloc(const sclap_csr* g, const int32_t* part, int32_t k, int64_t* cut_out,
                                 int64_t* block_w_out, void* stream) {
  if (!g || !cut_out) return fail(SCLAP_EINVAL, "NULL argument");
  if (g->n < 0 || g->m < 0 || (g->n > 0 && (!g->row_ptr || !part)) || (g->m > 0 && !g->col))
    return fail(SCLAP_EINVAL, "bad graph");
  if (k < 1) return fail(SCLAP_EINVAL, "k must be >= 1");
  if (block_w_out && k > kBlockWeightsLdsK)
    return fail(SCLAP_EINVAL, "block weights without allocation: k must be at most 4096");
  if (g->nw && g->nw_bytes != 4 && g->nw_bytes != 8) return fail(SCLAP_EINVAL, "nw_bytes must be 4 or 8");
  if (cut_partials(g->m) > kNoAllocPartials) return fail(SCLAP_EINVAL, "cut partial sums exceed the fixed scratch");
  int dev = 0;
  SCLAP_HIP(hipGetDevice(&dev));
  SCLAP_TRY(noalloc_setup(dev));
  hipStream_t st = (hipStream_t)stream;
  // cut_edges zeroes *cut_out with a kernel and writes one partial per
  // workgroup before summing them, so the scratch needs no clearing
  SCLAP_TRY(cut_edges(g->row_ptr, g->col, g->ew, part, g->n, g->m, (unsigned long long*)cut_out, g_scratch[dev], st));
  if (block_w_out) SCLAP_TRY(block_weights_raw(part, g->nw, g->nw_bytes, g->n, k, block_w_out, st));
  return SCLAP_OK;
}
