// Arithmetic in Fr, the BLS12-381 scalar field (host and device).
//
// The paper only asks for a field of about 2^254 elements "such as" the
// BLS12-381 one (Sec. V); this library fixes that field.
//   p = 0x73eda753299d7d483339d80809a1d80553bda402fffe5bfeffffffff00000001
// Elements are 8 little-endian 32-bit limbs.  Inside the library they are kept
// in Montgomery form x*R mod p with R = 2^256; on the wire (proof bytes, host
// API) they are canonical.  Multiplication is CIOS Montgomery multiplication
// (Koc, Acar, Kaliski, IEEE Micro 1996).  Because the top limb of p is below
// 2^31 - 1, the running value of each CIOS step fits in 8 limbs plus one carry
// word, so no ninth limb is kept.  -p^-1 mod 2^32 = 0xFFFFFFFF, so the
// Montgomery quotient digit of a step is simply -t0.
#pragma once
#include <stdint.h>

#if defined(__HIPCC__) || defined(__HIP__)
#include <hip/hip_runtime.h>
#define VL_HD __host__ __device__ __forceinline__
#else
#define VL_HD inline
#endif

namespace vl {

struct Fr {
  uint32_t w[8];
};

// p, R mod p and R^2 mod p as limbs.
#define VL_P_LIMBS 0x00000001u, 0xffffffffu, 0xfffe5bfeu, 0x53bda402u, \
                   0x09a1d805u, 0x3339d808u, 0x299d7d48u, 0x73eda753u
#define VL_R_LIMBS 0xfffffffeu, 0x00000001u, 0x00034802u, 0x5884b7fau, \
                   0xecbc4ff5u, 0x998c4fefu, 0xacc5056fu, 0x1824b159u
#define VL_R2_LIMBS 0xf3f29c6du, 0xc999e990u, 0x87925c23u, 0x2b6cedcbu, \
                    0x7254398fu, 0x05d31496u, 0x9f59ff11u, 0x0748d9d9u
VL_HD uint32_t p_limb(int i) {
  // switch keeps the constant in the instruction stream on the device
  switch (i) {
    case 0: return 0x00000001u; case 1: return 0xffffffffu;
    case 2: return 0xfffe5bfeu; case 3: return 0x53bda402u;
    case 4: return 0x09a1d805u; case 5: return 0x3339d808u;
    case 6: return 0x299d7d48u; default: return 0x73eda753u;
  }
}

VL_HD Fr fr_zero() { Fr r; for (int i = 0; i < 8; ++i) r.w[i] = 0; return r; }
VL_HD Fr fr_from_limbs(uint32_t a0, uint32_t a1, uint32_t a2, uint32_t a3, uint32_t a4,
                       uint32_t a5, uint32_t a6, uint32_t a7) {
  Fr r; r.w[0] = a0; r.w[1] = a1; r.w[2] = a2; r.w[3] = a3;
  r.w[4] = a4; r.w[5] = a5; r.w[6] = a6; r.w[7] = a7; return r;
}
VL_HD Fr fr_R() { return fr_from_limbs(VL_R_LIMBS); }     // Montgomery form of 1
VL_HD Fr fr_R2() { return fr_from_limbs(VL_R2_LIMBS); }
VL_HD Fr fr_one_raw() { return fr_from_limbs(1, 0, 0, 0, 0, 0, 0, 0); }

VL_HD bool fr_eq(const Fr& a, const Fr& b) {
  uint32_t d = 0;
#pragma unroll
  for (int i = 0; i < 8; ++i) d |= a.w[i] ^ b.w[i];
  return d == 0;
}

VL_HD bool fr_is_zero(const Fr& a) {
  uint32_t d = 0;
#pragma unroll
  for (int i = 0; i < 8; ++i) d |= a.w[i];
  return d == 0;
}

// 32-bit add/subtract with carry in and out (one v_add_co/v_addc_co or
// v_sub_co/v_subb_co on the device with clang's builtins)
VL_HD uint32_t adc32(uint32_t a, uint32_t b, uint32_t cin, uint32_t& cout) {
#if defined(__clang__)
  unsigned c;
  const uint32_t r = __builtin_addc(a, b, cin, &c);
  cout = c;
  return r;
#else
  const uint64_t t = (uint64_t)a + b + cin;
  cout = (uint32_t)(t >> 32);
  return (uint32_t)t;
#endif
}
VL_HD uint32_t sbb32(uint32_t a, uint32_t b, uint32_t bin, uint32_t& bout) {
#if defined(__clang__)
  unsigned c;
  const uint32_t r = __builtin_subc(a, b, bin, &c);
  bout = c;
  return r;
#else
  const uint64_t t = (uint64_t)a - b - bin;
  bout = (uint32_t)(t >> 63);
  return (uint32_t)t;
#endif
}

// a < p ?
VL_HD bool fr_lt_p(const Fr& a) {
  uint32_t borrow = 0;
#pragma unroll
  for (int i = 0; i < 8; ++i) (void)sbb32(a.w[i], p_limb(i), borrow, borrow);
  return borrow != 0;
}

// r = a - p if a >= p else a   (a < 2p)
VL_HD Fr fr_reduce_once(const Fr& a) {
  Fr t;
  uint32_t borrow = 0;
#pragma unroll
  for (int i = 0; i < 8; ++i) t.w[i] = sbb32(a.w[i], p_limb(i), borrow, borrow);
  Fr r;
#pragma unroll
  for (int i = 0; i < 8; ++i) r.w[i] = borrow ? a.w[i] : t.w[i];
  return r;
}

VL_HD Fr fr_add(const Fr& a, const Fr& b) {
  Fr s;
  uint32_t c = 0;
#pragma unroll
  for (int i = 0; i < 8; ++i) s.w[i] = adc32(a.w[i], b.w[i], c, c);
  return fr_reduce_once(s);   // a + b < 2p < 2^256: no carry out
}

VL_HD Fr fr_sub(const Fr& a, const Fr& b) {
  Fr d;
  uint32_t borrow = 0;
#pragma unroll
  for (int i = 0; i < 8; ++i) d.w[i] = sbb32(a.w[i], b.w[i], borrow, borrow);
  // if it went negative add p back
  const uint32_t mask = 0u - borrow;
  uint32_t c = 0;
#pragma unroll
  for (int i = 0; i < 8; ++i) d.w[i] = adc32(d.w[i], p_limb(i) & mask, c, c);
  return d;
}

VL_HD Fr fr_neg(const Fr& a) { return fr_sub(fr_zero(), a); }
VL_HD Fr fr_double(const Fr& a) { return fr_add(a, a); }

// a / 2: a (even) or a + p (odd) shifted right by one; a + p < 2^256
VL_HD Fr fr_half(const Fr& a) {
  const uint32_t mask = 0u - (a.w[0] & 1u);
  Fr t;
  uint32_t c = 0;
#pragma unroll
  for (int j = 0; j < 8; ++j) t.w[j] = adc32(a.w[j], p_limb(j) & mask, c, c);
  Fr r;
#pragma unroll
  for (int j = 0; j < 7; ++j) r.w[j] = (t.w[j] >> 1) | (t.w[j + 1] << 31);
  r.w[7] = t.w[7] >> 1;
  return r;
}

#if defined(__HIP_DEVICE_COMPILE__)
// Device Montgomery product by product scanning with the reduction folded in
// (Koc, Acar, Kaliski's finely integrated product scanning).  Column k sums
// a_i b_{k-i} and m_i p_{k-i} (i < k); for k < 8 the digit m_k = -t0 (as
// -p^-1 = 0xFFFFFFFF mod 2^32) clears the column's low word, for k >= 8 the
// low word is result word k - 8.  The column sum is kept as a 64-bit pair
// (low, middle word) that each partial product is multiply-added into with
// v_mad_u64_u32, plus a top word that takes its carry-out through
// v_addc_co_u32: two instructions per partial product.  Carries go through
// scalar registers the compiler picks, so independent products interleave.
__device__ __forceinline__ void fr_mac96(uint64_t& acc, uint32_t& top, uint32_t x, uint32_t y) {
  uint64_t c, dummy;
  asm("v_mad_u64_u32 %0, %1, %2, %3, %0" : "+v"(acc), "=s"(c) : "v"(x), "v"(y));
  asm("v_addc_co_u32 %0, %1, %0, 0, %2" : "+v"(top), "=s"(dummy) : "s"(c));
}

__device__ __forceinline__ void fr_mac96s(uint64_t& acc, uint32_t& top, uint32_t x, uint32_t ys) {
  uint64_t c, dummy;
  asm("v_mad_u64_u32 %0, %1, %2, %3, %0" : "+v"(acc), "=s"(c) : "v"(x), "s"(ys));
  asm("v_addc_co_u32 %0, %1, %0, 0, %2" : "+v"(top), "=s"(dummy) : "s"(c));
}

#endif

#if !defined(__HIP_DEVICE_COMPILE__)
// Host Montgomery product with 64-bit limbs (CIOS, 128-bit partial
// products): 32 multiplications instead of the 128 of 32-bit limbs.  R is
// 2^256 either way, so the result is the same field element.
inline Fr fr_mul_host64(const Fr& a, const Fr& b) {
  typedef unsigned __int128 u128;
  constexpr uint64_t P[4] = {0xffffffff00000001ull, 0x53bda402fffe5bfeull, 0x3339d80809a1d805ull,
                             0x73eda753299d7d48ull};
  constexpr uint64_t kPInv64 = 0xfffffffeffffffffull;   // -p^-1 mod 2^64
  uint64_t A[4], Bv[4], t[6] = {0, 0, 0, 0, 0, 0};
  for (int j = 0; j < 4; ++j) {
    A[j] = (uint64_t)a.w[2 * j] | ((uint64_t)a.w[2 * j + 1] << 32);
    Bv[j] = (uint64_t)b.w[2 * j] | ((uint64_t)b.w[2 * j + 1] << 32);
  }
  for (int i = 0; i < 4; ++i) {
    u128 C = 0;
    for (int j = 0; j < 4; ++j) {
      C = (u128)A[j] * Bv[i] + t[j] + (uint64_t)(C >> 64);
      t[j] = (uint64_t)C;
    }
    u128 s = (u128)t[4] + (uint64_t)(C >> 64);
    t[4] = (uint64_t)s;
    t[5] = (uint64_t)(s >> 64);
    const uint64_t m = t[0] * kPInv64;
    C = (u128)m * P[0] + t[0];
    for (int j = 1; j < 4; ++j) {
      C = (u128)m * P[j] + t[j] + (uint64_t)(C >> 64);
      t[j - 1] = (uint64_t)C;
    }
    s = (u128)t[4] + (uint64_t)(C >> 64);
    t[3] = (uint64_t)s;
    t[4] = t[5] + (uint64_t)(s >> 64);
  }
  Fr r;
  for (int j = 0; j < 4; ++j) {
    r.w[2 * j] = (uint32_t)t[j];
    r.w[2 * j + 1] = (uint32_t)(t[j] >> 32);
  }
  return fr_reduce_once(r);
}
#endif

// Montgomery product a*b*R^-1 mod p (inputs < p, output < p).  The device
// build uses the product-scanning form above; the host build the 64-bit
// CIOS form.
VL_HD Fr fr_mul(const Fr& a, const Fr& b) {
#if defined(__HIP_DEVICE_COMPILE__)
  uint32_t m[8], u[8];
  uint64_t acc = 0;
  uint32_t top = 0;
#pragma unroll
  for (int k = 0; k < 15; ++k) {
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      const int j = k - i;
      if (j >= 0 && j < 8) fr_mac96(acc, top, a.w[i], b.w[j]);
    }
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      const int j = k - i;
      if (i < k && j >= 1 && j < 8) fr_mac96s(acc, top, m[i], p_limb(j));
    }
    const uint32_t t0 = (uint32_t)acc;
    // a column sum stays below 2^69, so the shifted value is below 2^37 and
    // the +1 below cannot carry out of 64 bits
    acc = (acc >> 32) | ((uint64_t)top << 32);
    top = 0;
    if (k < 8) {
      m[k] = 0u - t0;
      acc += t0 != 0u ? 1u : 0u;            // t0 + m_k * p_0 = t0 + m_k = 0 or 2^32
    } else {
      u[k - 8] = t0;
    }
  }
  u[7] = (uint32_t)acc;                      // the result is below 2p < 2^256
  Fr r;
#pragma unroll
  for (int j = 0; j < 8; ++j) r.w[j] = u[j];
  return fr_reduce_once(r);
#else
  return fr_mul_host64(a, b);
#endif
}

#if defined(__HIP_DEVICE_COMPILE__)
// N independent Montgomery products (N = 2 or 3) with their partial products
// interleaved instruction by instruction: the same algorithm as fr_mul, but
// each asm block carries one multiply-add of every product, so the products'
// dependency chains overlap (the compiler keeps separate fr_mul calls' asm
// in order, one product after the other).  Within a block each carry is read
// at least one instruction after the multiply-add that wrote it.
template <int N>
__device__ __forceinline__ void fr_macn(uint64_t (&acc)[N], uint32_t (&top)[N], const uint32_t (&x)[N], const uint32_t (&y)[N]) {
  if constexpr (N == 2) {
    uint64_t c0, c1;
    asm("v_mad_u64_u32 %0, %4, %6, %7, %0\n\t"
        "v_mad_u64_u32 %1, %5, %8, %9, %1\n\t"
        "v_addc_co_u32 %2, %4, %2, 0, %4\n\t"
        "v_addc_co_u32 %3, %5, %3, 0, %5"
        : "+v"(acc[0]), "+v"(acc[1]), "+v"(top[0]), "+v"(top[1]), "=&s"(c0), "=&s"(c1)
        : "v"(x[0]), "v"(y[0]), "v"(x[1]), "v"(y[1]));
  } else {
    uint64_t c0, c1, c2;
    asm("v_mad_u64_u32 %0, %6, %9, %10, %0\n\t"
        "v_mad_u64_u32 %1, %7, %11, %12, %1\n\t"
        "v_mad_u64_u32 %2, %8, %13, %14, %2\n\t"
        "v_addc_co_u32 %3, %6, %3, 0, %6\n\t"
        "v_addc_co_u32 %4, %7, %4, 0, %7\n\t"
        "v_addc_co_u32 %5, %8, %5, 0, %8"
        : "+v"(acc[0]), "+v"(acc[1]), "+v"(acc[2]), "+v"(top[0]), "+v"(top[1]), "+v"(top[2]),
          "=&s"(c0), "=&s"(c1), "=&s"(c2)
        : "v"(x[0]), "v"(y[0]), "v"(x[1]), "v"(y[1]), "v"(x[2]), "v"(y[2]));
  }
}

template <int N>
__device__ __forceinline__ void fr_macns(uint64_t (&acc)[N], uint32_t (&top)[N], const uint32_t (&x)[N], uint32_t ys) {
  if constexpr (N == 2) {
    uint64_t c0, c1;
    asm("v_mad_u64_u32 %0, %4, %6, %8, %0\n\t"
        "v_mad_u64_u32 %1, %5, %7, %8, %1\n\t"
        "v_addc_co_u32 %2, %4, %2, 0, %4\n\t"
        "v_addc_co_u32 %3, %5, %3, 0, %5"
        : "+v"(acc[0]), "+v"(acc[1]), "+v"(top[0]), "+v"(top[1]), "=&s"(c0), "=&s"(c1)
        : "v"(x[0]), "v"(x[1]), "s"(ys));
  } else {
    uint64_t c0, c1, c2;
    asm("v_mad_u64_u32 %0, %6, %9, %12, %0\n\t"
        "v_mad_u64_u32 %1, %7, %10, %12, %1\n\t"
        "v_mad_u64_u32 %2, %8, %11, %12, %2\n\t"
        "v_addc_co_u32 %3, %6, %3, 0, %6\n\t"
        "v_addc_co_u32 %4, %7, %4, 0, %7\n\t"
        "v_addc_co_u32 %5, %8, %5, 0, %8"
        : "+v"(acc[0]), "+v"(acc[1]), "+v"(acc[2]), "+v"(top[0]), "+v"(top[1]), "+v"(top[2]),
          "=&s"(c0), "=&s"(c1), "=&s"(c2)
        : "v"(x[0]), "v"(x[1]), "v"(x[2]), "s"(ys));
  }
}

template <int N>
__device__ __forceinline__ void fr_mul_dev_n(const Fr (&a)[N], const Fr (&b)[N], Fr (&r)[N]) {
  uint32_t m[N][8], u[N][8];
  uint64_t acc[N];
  uint32_t top[N];
#pragma unroll
  for (int c = 0; c < N; ++c) { acc[c] = 0; top[c] = 0; }
#pragma unroll
  for (int k = 0; k < 15; ++k) {
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      const int j = k - i;
      if (j >= 0 && j < 8) {
        uint32_t x[N], y[N];
#pragma unroll
        for (int c = 0; c < N; ++c) { x[c] = a[c].w[i]; y[c] = b[c].w[j]; }
        fr_macn<N>(acc, top, x, y);
      }
    }
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      const int j = k - i;
      if (i < k && j >= 1 && j < 8) {
        uint32_t x[N];
#pragma unroll
        for (int c = 0; c < N; ++c) x[c] = m[c][i];
        fr_macns<N>(acc, top, x, p_limb(j));
      }
    }
#pragma unroll
    for (int c = 0; c < N; ++c) {
      const uint32_t t0 = (uint32_t)acc[c];
      acc[c] = (acc[c] >> 32) | ((uint64_t)top[c] << 32);
      top[c] = 0;
      if (k < 8) {
        m[c][k] = 0u - t0;
        acc[c] += t0 != 0u ? 1u : 0u;
      } else {
        u[c][k - 8] = t0;
      }
    }
  }
#pragma unroll
  for (int c = 0; c < N; ++c) {
    u[c][7] = (uint32_t)acc[c];
    Fr t;
#pragma unroll
    for (int j = 0; j < 8; ++j) t.w[j] = u[c][j];
    r[c] = fr_reduce_once(t);
  }
}

#endif

// r[c] = a[c] * b[c] * R^-1 for c < N (N = 2 or 3): the same values as N
// calls of fr_mul, faster on the device when the products are independent.
template <int N>
VL_HD void fr_mul_n(const Fr (&a)[N], const Fr (&b)[N], Fr (&r)[N]) {
  static_assert(N == 2 || N == 3, "two or three products");
#if defined(__HIP_DEVICE_COMPILE__)
  fr_mul_dev_n<N>(a, b, r);
#else
  for (int c = 0; c < N; ++c) r[c] = fr_mul(a[c], b[c]);
#endif
}

VL_HD Fr fr_to_mont(const Fr& a) { return fr_mul(a, fr_R2()); }
VL_HD Fr fr_from_mont(const Fr& a) { return fr_mul(a, fr_one_raw()); }

// canonical little-endian 32-byte encoding
VL_HD void fr_to_bytes(const Fr& a, uint8_t* out) {
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    out[4 * i + 0] = (uint8_t)(a.w[i]);
    out[4 * i + 1] = (uint8_t)(a.w[i] >> 8);
    out[4 * i + 2] = (uint8_t)(a.w[i] >> 16);
    out[4 * i + 3] = (uint8_t)(a.w[i] >> 24);
  }
}

VL_HD Fr fr_from_bytes(const uint8_t* in) {
  Fr a;
#pragma unroll
  for (int i = 0; i < 8; ++i)
    a.w[i] = (uint32_t)in[4 * i] | ((uint32_t)in[4 * i + 1] << 8) |
             ((uint32_t)in[4 * i + 2] << 16) | ((uint32_t)in[4 * i + 3] << 24);
  return a;
}

}  // namespace vl
