// Device helpers of the sumcheck kernels (kernels.hip, bmm.hip): wave and
// workgroup sums of field elements, proof-byte stores, LDS element access.
#pragma once
#include "device.hpp"

namespace vl {

// sum of K field elements over the lanes of a wave (xor butterfly over
// lane distances < width, a power of two <= 64: every lane of each aligned
// group of `width` lanes ends with that group's sum)
template <int K>
__device__ __forceinline__ void wave_sum(Fr (&v)[K], uint32_t width) {
  for (uint32_t off = width >> 1; off >= 1; off >>= 1) {
#pragma unroll
    for (int k = 0; k < K; ++k) {
      Fr o;
#pragma unroll
      for (int j = 0; j < 8; ++j) o.w[j] = __shfl_xor(v[k].w[j], (int)off, kWave);
      v[k] = fr_add(v[k], o);
    }
  }
}

// rounds workgroup: 8 waves, two per SIMD, so that the global sweeps have a
// second wave to issue from while one waits on its loads or its multiply
// chains.  At up to 256 VGPRs per wave one such workgroup fills its CU's
// register file.
constexpr int kRoundsBlock = 512;

// sum over the workgroup; the total lands in lanes 0..7 of wave 0 (the
// transcript's lanes), the other lanes keep partial values
template <int K>
__device__ __forceinline__ void block_sum_w0(Fr (&v)[K], uint32_t* lds) {
  constexpr int NW = kRoundsBlock / kWave;
  wave_sum<K>(v, kWave);
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  if (lane == 0) {
#pragma unroll
    for (int k = 0; k < K; ++k)
#pragma unroll
      for (int j = 0; j < 8; ++j) lds[(k * 8 + j) * NW + wave] = v[k].w[j];
  }
  __syncthreads();
  if (wave == 0) {
#pragma unroll
    for (int k = 0; k < K; ++k)
#pragma unroll
      for (int j = 0; j < 8; ++j) v[k].w[j] = lane < NW ? lds[(k * 8 + j) * NW + lane] : 0u;
    wave_sum<K>(v, NW);
  }
}

// canonical element c to 32 proof bytes (little-endian words); word stores
// when the destination is 4-byte aligned
__device__ __forceinline__ void put_canon(uint8_t* dst, const Fr& c) {
  if ((reinterpret_cast<uintptr_t>(dst) & 3u) == 0) {
    uint32_t* d = reinterpret_cast<uint32_t*>(dst);
#pragma unroll
    for (int j = 0; j < 8; ++j) d[j] = c.w[j];
  } else {
    uint8_t b[32];
    fr_to_bytes(c, b);
    for (int i = 0; i < 32; ++i) dst[i] = b[i];
  }
}

__device__ __forceinline__ void lds_put(uint32_t* dst, const Fr& v) {
#pragma unroll
  for (int j = 0; j < 8; ++j) dst[j] = v.w[j];
}
__device__ __forceinline__ Fr lds_get(const uint32_t* src) {
  Fr v;
#pragma unroll
  for (int j = 0; j < 8; ++j) v.w[j] = src[j];
  return v;
}

__device__ __forceinline__ Fr lds_or_global_fr(const uint32_t* src) {
  Fr v;
#pragma unroll
  for (int j = 0; j < 8; ++j) v.w[j] = src[j];
  return v;
}

__device__ __forceinline__ Fr readlane_fr(const Fr& x, int l) {
  Fr r;
#pragma unroll
  for (int j = 0; j < 8; ++j) r.w[j] = __builtin_amdgcn_readlane(x.w[j], l);
  return r;
}

// (2 b - a) for the evaluation at X = 2 of the line through (0, a), (1, b)
__device__ __forceinline__ Fr at_two(const Fr& a, const Fr& b) { return fr_sub(fr_double(b), a); }

}  // namespace vl
