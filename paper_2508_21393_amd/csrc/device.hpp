// Device-side helpers shared by the kernel sources: address-space pointer
// types, vector types, structure-of-limbs element access and the signed
// digits of an eq value.
#pragma once
#include "internal.hpp"

namespace vl {

typedef const __attribute__((address_space(4))) uint32_t* cu32_ptr;
typedef const __attribute__((address_space(4))) int32_t* ci32_ptr;
template <typename T>
using gptr = const __attribute__((address_space(1))) T*;
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));

// e (canonical, < p < 2^255) as 8 signed 32-bit digits, e = sum_j d_j 2^(32 j),
// d_j in [-2^31, 2^31); the top limb of p is below 2^31 - 1, so d_7 never
// carries into a ninth digit
__device__ __forceinline__ void signed_digits(const Fr& e, uint32_t* out) {
  uint32_t c = 0;
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    const uint32_t v = e.w[j] + c;        // e.w[j] + c <= 2^32 - 1 + 1: v == 0 means wrap
    const bool wrap = c && v == 0;
    const bool up = j < 7 && (wrap || v >= 0x80000000u);
    out[j] = v;                           // as int32: v - 2^32 when up
    c = up ? 1u : 0u;
  }
}

__device__ __forceinline__ Fr load_sol(const uint32_t* base, uint64_t ld, uint64_t i) {
  Fr r;
#pragma unroll
  for (int j = 0; j < 8; ++j) r.w[j] = base[j * ld + i];
  return r;
}

__device__ __forceinline__ void store_sol(uint32_t* base, uint64_t ld, uint64_t i, const Fr& v) {
#pragma unroll
  for (int j = 0; j < 8; ++j) base[j * ld + i] = v.w[j];
}

static inline uint32_t blocks_for(uint64_t n, uint32_t b) { return (uint32_t)((n + b - 1) / b); }

}  // namespace vl
