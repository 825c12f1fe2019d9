// Allocation-free partial evaluation: vl_mle_partial_eval with its scratch in
// a fixed device array of this library instead of a caller workspace, for
// callers that cannot allocate device memory (code under stream capture,
// tight serving loops, harnesses that forbid allocation).
//
// The array below is a file-scope __device__ variable: every GPU the library
// runs on holds its own copy, at its own address, for the life of the
// process.  In host code its name is only a host-side stand-in, so the
// device address is looked up once per device (hipGetSymbolAddress, with that
// device current, on the entry point's first call there) and that pointer is
// what the kernels get.  Calls on one device share the array: the pack table,
// the job blob and the chunk partials of a call are all written by that
// call's own kernels before they are read (the blob's range flag is written
// as zero by the upload), so nothing needs clearing between calls; calls that
// overlap on one device (two streams, or two host threads) race on it.
#include <hip/hip_runtime.h>

#include <map>
#include <mutex>

#include "plan.hpp"

namespace vl {

constexpr uint64_t kNoallocScratchBytes = VL_NOALLOC_SCRATCH_BYTES;
static_assert(kNoallocScratchBytes % 256 == 0, "the scratch size keeps 256-byte alignment");

static __device__ __align__(256) uint8_t scratch[kNoallocScratchBytes];

// device address of `scratch` on the current device (looked up once per device)
static vl_status scratch_address(void** out) {
  static std::mutex mu;
  static std::map<int, void*> addr;
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return fail(VL_ERR_HIP, "device: %s", hipGetErrorString(e));
  std::lock_guard<std::mutex> lock(mu);
  auto it = addr.find(dev);
  if (it != addr.end()) {
    *out = it->second;
    return VL_OK;
  }
  void* p = nullptr;
  e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !p) return fail(VL_ERR_HIP, "scratch address: %s", hipGetErrorString(e));
  if (reinterpret_cast<uintptr_t>(p) % 256) return fail(VL_ERR_HIP, "scratch is not 256-byte aligned");
  addr[dev] = p;
  *out = p;
  return VL_OK;
}

}  // namespace vl

using namespace vl;

extern "C" vl_status vl_mle_partial_eval_noalloc(const void* M, int32_t dtype, uint32_t rows, uint32_t cols,
                                                 uint64_t ld, int32_t contract, vl_fr_vec eq, vl_fr_vec out,
                                                 const vl_tuning* tuning, void* stream) {
  {
    const vl_status st = partial_eval_check(M, dtype, rows, cols, ld, contract, eq, out, tuning);
    if (st != VL_OK) return st;
  }
  const uint64_t need = vl_partial_eval_workspace_size(rows, cols, contract, dtype, tuning);
  if (need == 0) return fail(VL_ERR_INVALID_ARG, "no workspace size for these arguments");
  if (need > kNoallocScratchBytes)
    return fail(VL_ERR_WORKSPACE, "this partial evaluation needs %llu bytes of scratch; the fixed scratch "
                "holds %llu (use vl_mle_partial_eval with a workspace)",
                (unsigned long long)need, (unsigned long long)kNoallocScratchBytes);
  void* ws = nullptr;
  {
    const vl_status st = scratch_address(&ws);
    if (st != VL_OK) return st;
  }
  return partial_eval_launch(M, dtype, rows, cols, ld, contract, eq, out, ws, kNoallocScratchBytes, tuning,
                             stream);
}
