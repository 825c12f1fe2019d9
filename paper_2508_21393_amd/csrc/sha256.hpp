// SHA-256 (FIPS 180-4) and the Fiat-Shamir transcript, host and device.
//
// The paper turns its interactive protocols non-interactive by hashing every
// earlier public message into each verifier challenge (Fiat-Shamir; Sec. IV-A
// footnote, Sec. V).  It names no hash or byte layout; this library fixes:
//   init:    st = H("VeriLoRA-zkMat-v1" || u64 seed || u32 group_id
//                   || u32 n_products || (u32 D0, D1, D2) per product)
//   absorb:  st = H(st || label || data)
//   squeeze: for ctr = 0, 1, ...: h = H(st || label || u32 ctr);
//            x = LE(h) mod 2^255; if x < p { st = h; return x }
// with little-endian integers and canonical 32-byte field elements.
#pragma once
#include <stdint.h>
#if !defined(__HIP_DEVICE_COMPILE__) && defined(__x86_64__)
#include <cpuid.h>
#include <immintrin.h>
#endif

#include "fr.hpp"

namespace vl {

VL_HD uint32_t rotr32(uint32_t x, int n) { return (x >> n) | (x << (32 - n)); }

// Three-input helpers.  On the device each is one VALU instruction
// (v_add3_u32, v_bfi_b32), which the compiler does not form by itself here;
// the SHA-256 rounds of the transcript run on a single lane and are latency
// bound, so instruction count is time.
VL_HD uint32_t add3_u32(uint32_t a, uint32_t b, uint32_t c) {
#if __HIP_DEVICE_COMPILE__
  uint32_t r;
  asm("v_add3_u32 %0, %1, %2, %3" : "=v"(r) : "v"(a), "v"(b), "v"(c));
  return r;
#else
  return a + b + c;
#endif
}

// bitwise select: bits of x where m is 1, bits of y where m is 0
VL_HD uint32_t bitsel(uint32_t m, uint32_t x, uint32_t y) {
#if __HIP_DEVICE_COMPILE__
  uint32_t r;
  asm("v_bfi_b32 %0, %1, %2, %3" : "=v"(r) : "v"(m), "v"(x), "v"(y));
  return r;
#else
  return (m & x) | (~m & y);
#endif
}

// three-input xor; on the device one v_bitop3_b32 (truth table 0x96)
VL_HD uint32_t xor3_u32(uint32_t a, uint32_t b, uint32_t c) {
#if __HIP_DEVICE_COMPILE__
  uint32_t r;
  asm("v_bitop3_b32 %0, %1, %2, %3 bitop3:0x96" : "=v"(r) : "v"(a), "v"(b), "v"(c));
  return r;
#else
  return a ^ b ^ c;
#endif
}

// bitwise majority Maj(a, b, c); on the device one v_bitop3_b32 (truth
// table 0xe8)
VL_HD uint32_t maj_u32(uint32_t a, uint32_t b, uint32_t c) {
#if __HIP_DEVICE_COMPILE__
  uint32_t r;
  asm("v_bitop3_b32 %0, %1, %2, %3 bitop3:0xe8" : "=v"(r) : "v"(a), "v"(b), "v"(c));
  return r;
#else
  return (a & b) | (a & c) | (b & c);
#endif
}

// FIPS 180-4 round constants
#define VL_SHA256_K                                                                                \
  0x428a2f98u, 0x71374491u, 0xb5c0fbcfu, 0xe9b5dba5u, 0x3956c25bu, 0x59f111f1u, 0x923f82a4u,     \
      0xab1c5ed5u, 0xd807aa98u, 0x12835b01u, 0x243185beu, 0x550c7dc3u, 0x72be5d74u, 0x80deb1feu, \
      0x9bdc06a7u, 0xc19bf174u, 0xe49b69c1u, 0xefbe4786u, 0x0fc19dc6u, 0x240ca1ccu, 0x2de92c6fu, \
      0x4a7484aau, 0x5cb0a9dcu, 0x76f988dau, 0x983e5152u, 0xa831c66du, 0xb00327c8u, 0xbf597fc7u, \
      0xc6e00bf3u, 0xd5a79147u, 0x06ca6351u, 0x14292967u, 0x27b70a85u, 0x2e1b2138u, 0x4d2c6dfcu, \
      0x53380d13u, 0x650a7354u, 0x766a0abbu, 0x81c2c92eu, 0x92722c85u, 0xa2bfe8a1u, 0xa81a664bu, \
      0xc24b8b70u, 0xc76c51a3u, 0xd192e819u, 0xd6990624u, 0xf40e3585u, 0x106aa070u, 0x19a4c116u, \
      0x1e376c08u, 0x2748774cu, 0x34b0bcb5u, 0x391c0cb3u, 0x4ed8aa4au, 0x5b9cca4fu, 0x682e6ff3u, \
      0x748f82eeu, 0x78a5636fu, 0x84c87814u, 0x8cc70208u, 0x90befffau, 0xa4506cebu, 0xbef9a3f7u, \
      0xc67178f2u

#if defined(__HIP__)
// device copy: the compression loop below reads 16 of them per iteration
// with scalar loads
static __constant__ uint32_t kSha256KDev[64] = {VL_SHA256_K};
#endif
static const uint32_t kSha256KHost[64] = {VL_SHA256_K};

VL_HD const uint32_t* sha256_k() {
#if __HIP_DEVICE_COMPILE__
  return kSha256KDev;
#else
  return kSha256KHost;
#endif
}

#if !defined(__HIP_DEVICE_COMPILE__) && defined(__x86_64__)
// Host: the x86 SHA extensions (SHA256RNDS2 does two rounds on the state
// held as {A, B, E, F} and {C, D, G, H}; SHA256MSG1/MSG2 extend the message
// schedule four words at a time), used when the CPU has them.
__attribute__((target("sha,sse4.1"))) inline void sha256_compress_ni(uint32_t h[8], const uint32_t (&w)[16]) {
  const uint32_t* K = kSha256KHost;
  __m128i abef = _mm_set_epi32((int)h[0], (int)h[1], (int)h[4], (int)h[5]);
  __m128i cdgh = _mm_set_epi32((int)h[2], (int)h[3], (int)h[6], (int)h[7]);
  const __m128i abef0 = abef, cdgh0 = cdgh;
  __m128i W[4];   // ring of the last 16 schedule words, 4 per register (lowest = first)
  for (int j = 0; j < 16; ++j) {
    __m128i m;
    if (j < 4) {
      m = _mm_set_epi32((int)w[4 * j + 3], (int)w[4 * j + 2], (int)w[4 * j + 1], (int)w[4 * j]);
    } else {
      // W[4j..4j+3] from W[4j-16..], W[4j-15..] (msg1), W[4j-7..] and W[4j-2..] (msg2)
      __m128i t = _mm_sha256msg1_epu32(W[j & 3], W[(j + 1) & 3]);
      t = _mm_add_epi32(t, _mm_alignr_epi8(W[(j + 3) & 3], W[(j + 2) & 3], 4));
      m = _mm_sha256msg2_epu32(t, W[(j + 3) & 3]);
    }
    W[j & 3] = m;
    __m128i wk = _mm_add_epi32(m, _mm_loadu_si128(reinterpret_cast<const __m128i*>(K + 4 * j)));
    cdgh = _mm_sha256rnds2_epu32(cdgh, abef, wk);   // rounds 4j, 4j+1: cdgh now holds ABEF
    wk = _mm_shuffle_epi32(wk, 0x0E);
    abef = _mm_sha256rnds2_epu32(abef, cdgh, wk);   // rounds 4j+2, 4j+3
  }
  abef = _mm_add_epi32(abef, abef0);
  cdgh = _mm_add_epi32(cdgh, cdgh0);
  alignas(16) uint32_t x[4], y[4];
  _mm_store_si128(reinterpret_cast<__m128i*>(x), abef);
  _mm_store_si128(reinterpret_cast<__m128i*>(y), cdgh);
  h[0] = x[3]; h[1] = x[2]; h[4] = x[1]; h[5] = x[0];
  h[2] = y[3]; h[3] = y[2]; h[6] = y[1]; h[7] = y[0];
}

inline bool sha256_ni_available() {
  static const bool ok = [] {
    unsigned a, b, c, d;
    if (!__get_cpuid_count(7, 0, &a, &b, &c, &d)) return false;
    const bool sha = (b >> 29) & 1u;
    if (!__get_cpuid(1, &a, &b, &c, &d)) return false;
    const bool sse41 = (c >> 19) & 1u, ssse3 = (c >> 9) & 1u;
    return sha && sse41 && ssse3;
  }();
  return ok;
}
#endif

// FIPS 180-4 compression of one block given as 16 big-endian message words.
// The 64 rounds run as 4 iterations of 16 (the message schedule's ring
// length): the device code stays small enough for the instruction cache,
// which matters more than the loop overhead on the single lane that hashes.
VL_HD void sha256_compress_w(uint32_t h[8], const uint32_t (&win)[16]) {
#if !defined(__HIP_DEVICE_COMPILE__) && defined(__x86_64__)
  if (sha256_ni_available()) {
    sha256_compress_ni(h, win);
    return;
  }
#endif
  const uint32_t* K = sha256_k();
  uint32_t w[16];
#pragma unroll
  for (int i = 0; i < 16; ++i) w[i] = win[i];
  uint32_t a = h[0], b = h[1], c = h[2], d = h[3], e = h[4], f = h[5], g = h[6], hh = h[7];
#pragma unroll 1
  for (int it = 0; it < 4; ++it) {
    if (it > 0) {
      // w[i] <- W[16 it + i] for i = 0..15, in order (each uses the new w[i-2])
#pragma unroll
      for (int i = 0; i < 16; ++i) {
        const uint32_t w15 = w[(i + 1) & 15], w2 = w[(i + 14) & 15];
        const uint32_t s0 = xor3_u32(rotr32(w15, 7), rotr32(w15, 18), w15 >> 3);
        const uint32_t s1 = xor3_u32(rotr32(w2, 17), rotr32(w2, 19), w2 >> 10);
        w[i] = add3_u32(w[i], s0, w[(i + 9) & 15]) + s1;
      }
    }
    const uint32_t* Kt = K + 16 * it;
#pragma unroll
    for (int i = 0; i < 16; ++i) {
      const uint32_t S1 = xor3_u32(rotr32(e, 6), rotr32(e, 11), rotr32(e, 25));
      const uint32_t ch = bitsel(e, f, g);                 // Ch(e, f, g)
      const uint32_t t1 = add3_u32(hh, S1, ch) + (w[i] + Kt[i]);
      const uint32_t S0 = xor3_u32(rotr32(a, 2), rotr32(a, 13), rotr32(a, 22));
      const uint32_t mj = maj_u32(a, b, c);
      hh = g; g = f; f = e; e = d + t1; d = c; c = b; b = a; a = add3_u32(t1, S0, mj);
    }
  }
  h[0] += a; h[1] += b; h[2] += c; h[3] += d; h[4] += e; h[5] += f; h[6] += g; h[7] += hh;
}

VL_HD void sha256_compress(uint32_t h[8], const uint8_t blk[64]) {
  uint32_t w[16];
  for (int i = 0; i < 16; ++i)
    w[i] = ((uint32_t)blk[4 * i] << 24) | ((uint32_t)blk[4 * i + 1] << 16) |
           ((uint32_t)blk[4 * i + 2] << 8) | (uint32_t)blk[4 * i + 3];
  sha256_compress_w(h, w);
}

// Streaming hasher for short messages.
struct Sha256 {
  uint32_t h[8];
  uint8_t buf[64];
  uint32_t fill;
  uint64_t total;
};

VL_HD void sha256_init(Sha256& s) {
  s.h[0] = 0x6a09e667u; s.h[1] = 0xbb67ae85u; s.h[2] = 0x3c6ef372u; s.h[3] = 0xa54ff53au;
  s.h[4] = 0x510e527fu; s.h[5] = 0x9b05688cu; s.h[6] = 0x1f83d9abu; s.h[7] = 0x5be0cd19u;
  s.fill = 0;
  s.total = 0;
}

VL_HD void sha256_update(Sha256& s, const uint8_t* p, uint32_t n) {
  for (uint32_t i = 0; i < n; ++i) {
    s.buf[s.fill++] = p[i];
    if (s.fill == 64) {
      sha256_compress(s.h, s.buf);
      s.fill = 0;
    }
  }
  s.total += n;
}

VL_HD void sha256_final(Sha256& s, uint8_t out[32]) {
  const uint64_t bits = s.total * 8;
  uint8_t one = 0x80;
  sha256_update(s, &one, 1);
  uint8_t z = 0;
  while (s.fill != 56) sha256_update(s, &z, 1);
  uint8_t len[8];
  for (int i = 0; i < 8; ++i) len[i] = (uint8_t)(bits >> (56 - 8 * i));
  sha256_update(s, len, 8);
  for (int i = 0; i < 8; ++i) {
    out[4 * i] = (uint8_t)(s.h[i] >> 24);
    out[4 * i + 1] = (uint8_t)(s.h[i] >> 16);
    out[4 * i + 2] = (uint8_t)(s.h[i] >> 8);
    out[4 * i + 3] = (uint8_t)(s.h[i]);
  }
}

VL_HD void put_u32le(uint8_t* o, uint32_t v) {
  o[0] = (uint8_t)v; o[1] = (uint8_t)(v >> 8); o[2] = (uint8_t)(v >> 16); o[3] = (uint8_t)(v >> 24);
}

// The transcript state is the last digest, kept as its 8 big-endian words
// (digest byte i is byte 3 - i % 4 of word i / 4).
struct Transcript {
  uint32_t h[8];
};

VL_HD void tr_to_bytes(const Transcript& t, uint8_t out[32]) {
  for (int i = 0; i < 8; ++i) {
    out[4 * i] = (uint8_t)(t.h[i] >> 24);
    out[4 * i + 1] = (uint8_t)(t.h[i] >> 16);
    out[4 * i + 2] = (uint8_t)(t.h[i] >> 8);
    out[4 * i + 3] = (uint8_t)(t.h[i]);
  }
}

VL_HD void tr_from_bytes(Transcript& t, const uint8_t in[32]) {
  for (int i = 0; i < 8; ++i)
    t.h[i] = ((uint32_t)in[4 * i] << 24) | ((uint32_t)in[4 * i + 1] << 16) |
             ((uint32_t)in[4 * i + 2] << 8) | (uint32_t)in[4 * i + 3];
}

// labels used by the protocol (string literals, so their lengths are known
// at compile time)
#define VL_LBL_U "u"
#define VL_LBL_V "v"
#define VL_LBL_CLAIM "claim"
#define VL_LBL_PART "part"
#define VL_LBL_ROUND "round"
#define VL_LBL_R "r"
#define VL_LBL_FINAL "final"
#define VL_LBL_RFINAL "rfinal"
#define VL_LBL_SIGMA "sigma"
#define VL_LBL_BIND "bind"

VL_HD void tr_init(Transcript& t, uint64_t seed, uint32_t group_id, uint32_t n_prods,
                   const uint32_t* dims /* 3 per product */) {
  Sha256 s;
  sha256_init(s);
  const char dom[] = "VeriLoRA-zkMat-v1";
  sha256_update(s, (const uint8_t*)dom, 17);
  uint8_t b[8];
  for (int i = 0; i < 8; ++i) b[i] = (uint8_t)(seed >> (8 * i));
  sha256_update(s, b, 8);
  put_u32le(b, group_id);
  sha256_update(s, b, 4);
  put_u32le(b, n_prods);
  sha256_update(s, b, 4);
  for (uint32_t k = 0; k < 3 * n_prods; ++k) {
    put_u32le(b, dims[k]);
    sha256_update(s, b, 4);
  }
  uint8_t st[32];
  sha256_final(s, st);
  tr_from_bytes(t, st);
}

// One-shot SHA-256 of an N-byte message, N a compile-time constant, whose
// byte k is byte_at(k).  Every loop is unrolled, so k is a constant at each
// call of byte_at and the message words are assembled in registers (no byte
// arrays, hence no scratch memory on the device).
template <int N, typename ByteAt>
VL_HD void sha256_gen(uint32_t (&h)[8], ByteAt byte_at) {
  constexpr int NB = (N + 9 + 63) / 64;
  constexpr uint64_t bits = (uint64_t)N * 8;
  h[0] = 0x6a09e667u; h[1] = 0xbb67ae85u; h[2] = 0x3c6ef372u; h[3] = 0xa54ff53au;
  h[4] = 0x510e527fu; h[5] = 0x9b05688cu; h[6] = 0x1f83d9abu; h[7] = 0x5be0cd19u;
#pragma unroll
  for (int b = 0; b < NB; ++b) {
    uint32_t w[16];
#pragma unroll
    for (int i = 0; i < 16; ++i) {
      uint32_t v = 0;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int k = b * 64 + 4 * i + q;
        uint32_t byte = 0;
        if (k < N) byte = byte_at(k);
        else if (k == N) byte = 0x80u;
        else if (k >= NB * 64 - 8) byte = (uint32_t)(bits >> (8 * (NB * 64 - 1 - k))) & 0xffu;
        v |= byte << (24 - 8 * q);
      }
      w[i] = v;
    }
    sha256_compress_w(h, w);
  }
}

VL_HD uint32_t state_byte(const Transcript& t, int k) { return (t.h[k >> 2] >> (24 - 8 * (k & 3))) & 0xffu; }
VL_HD uint32_t fr_byte(const Fr& x, int b) { return (x.w[b >> 2] >> (8 * (b & 3))) & 0xffu; }

// absorb(label, x_0 .. x_{K-1}): st = H(st || label || enc(x_0) || ...), xs canonical
template <int LN, int K>
VL_HD void tr_absorb_frs(Transcript& t, const char (&label)[LN], const Fr (&xs)[K]) {
  constexpr int L = LN - 1;
  const Transcript old = t;
  sha256_gen<32 + L + 32 * K>(t.h, [&](int k) -> uint32_t {
    if (k < 32) return state_byte(old, k);
    if (k < 32 + L) return (uint8_t)label[k - 32];
    const int e = (k - 32 - L) >> 5, b = (k - 32 - L) & 31;
    return fr_byte(xs[e], b);
  });
}

// absorb(label, d): st = H(st || label || d) for a 32-byte message d
template <int LN>
VL_HD void tr_absorb32(Transcript& t, const char (&label)[LN], const uint8_t* d) {
  constexpr int L = LN - 1;
  const Transcript old = t;
  sha256_gen<32 + L + 32>(t.h, [&](int k) -> uint32_t {
    if (k < 32) return state_byte(old, k);
    if (k < 32 + L) return (uint8_t)label[k - 32];
    return d[k - 32 - L];
  });
}

// squeeze(label): a canonical, uniformly distributed field element
template <int LN>
VL_HD Fr tr_squeeze_fixed(Transcript& t, const char (&label)[LN]) {
  constexpr int L = LN - 1;
  for (uint32_t ctr = 0;; ++ctr) {
    uint32_t h[8];
    sha256_gen<32 + L + 4>(h, [&](int k) -> uint32_t {
      if (k < 32) return state_byte(t, k);
      if (k < 32 + L) return (uint8_t)label[k - 32];
      return (ctr >> (8 * (k - 32 - L))) & 0xffu;
    });
    // the digest read as a little-endian integer: limb j is byte-swapped word j
    Fr x;
#pragma unroll
    for (int j = 0; j < 8; ++j)
      x.w[j] = ((h[j] & 0xffu) << 24) | ((h[j] & 0xff00u) << 8) | ((h[j] >> 8) & 0xff00u) | (h[j] >> 24);
    x.w[7] &= 0x7fffffffu;
    if (fr_lt_p(x)) {
#pragma unroll
      for (int i = 0; i < 8; ++i) t.h[i] = h[i];
      return x;
    }
  }
}

}  // namespace vl
