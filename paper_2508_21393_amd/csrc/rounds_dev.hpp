// Device helpers of the sumcheck kernels (kernels.hip, bmm.hip): wave and
// workgroup sums of field elements, proof-byte stores, LDS element access.
#pragma once
#include "device.hpp"
#include "sha256.hpp"

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


// absorb("round", g(0..K-1)) by the lanes of wave 0 (K = 3 or 4; the
// message of the state, the label and K canonical values fits three SHA-256
// blocks): lane b < 3 computes block b's message schedule, and every lane
// runs the 3 x 64 compression rounds on those words, read with v_readlane.
// The same digest as tr_absorb_frs; the state is taken from lane 0.
template <int K>
__device__ __forceinline__ void absorb_round_lanes_k(Transcript& tr, const Fr (&gc)[K], uint32_t lane) {
  constexpr int L = sizeof(VL_LBL_ROUND) - 1;
  constexpr int N = 32 + L + 32 * K;
  constexpr int NB = (N + 9 + 63) / 64;
  static_assert(NB == 3, "the round absorb is three blocks");
  uint32_t st[8];
#pragma unroll
  for (int i = 0; i < 8; ++i) st[i] = __builtin_amdgcn_readlane(tr.h[i], 0);
  auto byte_at = [&](int k) -> uint32_t {
    if (k < 32) return (st[k >> 2] >> (24 - 8 * (k & 3))) & 0xffu;
    if (k < 32 + L) return (uint8_t)VL_LBL_ROUND[k - 32];
    if (k < N) return fr_byte(gc[(k - 32 - L) >> 5], (k - 32 - L) & 31);
    if (k == N) return 0x80u;
    if (k >= NB * 64 - 8) return (uint32_t)(((uint64_t)N * 8) >> (8 * (NB * 64 - 1 - k))) & 0xffu;
    return 0u;
  };
  const uint32_t blk = min(lane, 2u);
  uint32_t w[64];
#pragma unroll
  for (int i = 0; i < 16; ++i) {
    uint32_t v[NB];
#pragma unroll
    for (int b = 0; b < NB; ++b) {
      uint32_t x = 0;
#pragma unroll
      for (int q = 0; q < 4; ++q) x |= byte_at(64 * b + 4 * i + q) << (24 - 8 * q);
      v[b] = x;
    }
    w[i] = blk == 0 ? v[0] : (blk == 1 ? v[1] : v[2]);
  }
#pragma unroll
  for (int i = 16; i < 64; ++i) {
    const uint32_t w15 = w[i - 15], w2 = w[i - 2];
    const uint32_t s0 = xor3_u32(rotr32(w15, 7), rotr32(w15, 18), w15 >> 3);
    const uint32_t s1 = xor3_u32(rotr32(w2, 17), rotr32(w2, 19), w2 >> 10);
    w[i] = add3_u32(w[i - 16], s0, w[i - 7]) + s1;
  }
  const uint32_t* KK = sha256_k();
#pragma unroll
  for (int i = 0; i < 64; ++i) w[i] += KK[i];
  uint32_t h[8] = {0x6a09e667u, 0xbb67ae85u, 0x3c6ef372u, 0xa54ff53au,
                   0x510e527fu, 0x9b05688cu, 0x1f83d9abu, 0x5be0cd19u};
#pragma unroll 1
  for (uint32_t b = 0; b < (uint32_t)NB; ++b) {
    uint32_t a = h[0], bb = h[1], c = h[2], dd = h[3], e = h[4], f = h[5], g = h[6], hh = h[7];
#pragma unroll
    for (int i = 0; i < 64; ++i) {
      const uint32_t wk = __builtin_amdgcn_readlane(w[i], b);
      const uint32_t S1 = xor3_u32(rotr32(e, 6), rotr32(e, 11), rotr32(e, 25));
      const uint32_t ch = bitsel(e, f, g);
      const uint32_t t1 = add3_u32(hh, S1, ch) + wk;
      const uint32_t S0 = xor3_u32(rotr32(a, 2), rotr32(a, 13), rotr32(a, 22));
      const uint32_t mj = maj_u32(a, bb, c);
      hh = g; g = f; f = e; e = dd + t1; dd = c; c = bb; bb = a; a = add3_u32(t1, S0, mj);
    }
    h[0] += a; h[1] += bb; h[2] += c; h[3] += dd; h[4] += e; h[5] += f; h[6] += g; h[7] += hh;
  }
#pragma unroll
  for (int i = 0; i < 8; ++i) tr.h[i] = h[i];
}

// One round's messages and challenge by wave 0 (all 64 lanes active; gc
// canonical and uniform): lane k < K writes g(k) to out, the wave absorbs,
// lane 0 squeezes r.  Returns r in Montgomery form in every lane; the
// transcript state afterwards is lane 0's.
template <int K>
__device__ __forceinline__ Fr round_challenge_k(Transcript& tr, const Fr (&gc)[K], uint8_t* out, uint32_t lane) {
  Fr mine = gc[0];
#pragma unroll
  for (int k = 1; k < K; ++k)
#pragma unroll
    for (int j = 0; j < 8; ++j) mine.w[j] = lane == (uint32_t)k ? gc[k].w[j] : mine.w[j];
  if (lane < (uint32_t)K) put_canon(out + 32 * lane, mine);
  Fr r = fr_zero();
  absorb_round_lanes_k<K>(tr, gc, lane);
  if (lane == 0) r = fr_to_mont(tr_squeeze_fixed(tr, VL_LBL_R));
  return readlane_fr(r, 0);
}

// sum of 4 elements over a 256-thread block; the total lands in lanes 0..3
// of wave 0 (red: 4 * 8 * 4 words of LDS)
__device__ __forceinline__ void block256_sum4(Fr (&g)[4], uint32_t* red) {
  wave_sum<4>(g, kWave);
  const uint32_t wave = threadIdx.x >> 6, lane = threadIdx.x & 63u;
  if (lane == 0)
#pragma unroll
    for (int k = 0; k < 4; ++k)
#pragma unroll
      for (int j = 0; j < 8; ++j) red[(k * 8 + j) * 4 + wave] = g[k].w[j];
  __syncthreads();
  if (wave == 0) {
#pragma unroll
    for (int k = 0; k < 4; ++k)
#pragma unroll
      for (int j = 0; j < 8; ++j) g[k].w[j] = lane < 4 ? red[(k * 8 + j) * 4 + lane] : 0u;
    wave_sum<4>(g, 4);
  }
}

}  // namespace vl
