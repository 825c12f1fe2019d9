// Arithmetic in Fq, the base field of BLS12-381, and in its group G1
// (host and device), for the Hyrax commitments.
//
// G1 is the group of points of y^2 = x^3 + 4 over Fq of prime order p, the
// order of Fr, so a G1 point times an Fr element is well defined.
//   q = 0x1a0111ea397fe69a4b1ba7b6434bacd764774b84f38512bf6730d2a0f6b0f6241eab
//       fffeb153ffffb9feffffffffaaab   (381 bits, q = 3 mod 4)
// Elements are 12 little-endian 32-bit limbs, in Montgomery form x*R mod q
// with R = 2^384 inside the library and canonical on the wire.  On the device
// the Montgomery product is the finely integrated product scanning of fr.hpp
// with 12 limbs; -q^-1 mod 2^32 = 0xfffcfffd, so the quotient digit of a
// column is a 32-bit multiply.  The host uses 6 64-bit limbs (the same bytes:
// little-endian 32-bit limbs pair into 64-bit limbs) with CIOS.  The top limb
// of q is below 2^29, so every running value fits in the limbs plus one
// carry word and a product of two reduced values is below 2q.
//
// Points of G1 are kept in XYZZ coordinates (X, Y, ZZ, ZZZ) with
// x = X / ZZ, y = Y / ZZZ and ZZ^3 = ZZZ^2; ZZ = 0 is the point at infinity.
// The formulas are the a = 0 cases of the XYZZ formulas for short
// Weierstrass curves (Bernstein and Lange, Explicit-Formulas Database,
// madd-2008-s, mdbl-2008-s-1, add-2008-s, dbl-2008-s-1): a mixed addition
// costs 8 multiplications and 2 squarings.  Additions detect equal and
// opposite inputs and fall back to doubling or infinity, so every sum is
// exact.
#pragma once
#include <stdint.h>
#include <string.h>

#include <type_traits>

#include "fr.hpp"
#include "sha256.hpp"

namespace vl {

struct Fq {
  uint32_t w[12];
};

VL_HD uint32_t q_limb(int i) {
  switch (i) {
    case 0: return 0xffffaaabu; case 1: return 0xb9feffffu; case 2: return 0xb153ffffu;
    case 3: return 0x1eabfffeu; case 4: return 0xf6b0f624u; case 5: return 0x6730d2a0u;
    case 6: return 0xf38512bfu; case 7: return 0x64774b84u; case 8: return 0x434bacd7u;
    case 9: return 0x4b1ba7b6u; case 10: return 0x397fe69au; default: return 0x1a0111eau;
  }
}
constexpr uint32_t kQInv32 = 0xfffcfffdu;              // -q^-1 mod 2^32
constexpr uint64_t kQInv64 = 0x89f3fffcfffcfffdull;    // -q^-1 mod 2^64

#define VL_FQ_R_LIMBS 0x0002fffdu, 0x76090000u, 0xc40c0002u, 0xebf4000bu, 0x53c758bau, 0x5f489857u, \
                      0x70525745u, 0x77ce5853u, 0xa256ec6du, 0x5c071a97u, 0xfa80e493u, 0x15f65ec3u
#define VL_FQ_R2_LIMBS 0x1c341746u, 0xf4df1f34u, 0x09d104f1u, 0x0a76e6a6u, 0x4c95b6d5u, 0x8de5476cu, \
                       0x939d83c0u, 0x67eb88a9u, 0xb519952du, 0x9a793e85u, 0x92cae3aau, 0x11988fe5u
#define VL_FQ_R3_LIMBS 0xd94ca1e0u, 0xed48ac6bu, 0x03a7adf8u, 0x315f831eu, 0x615e29ddu, 0x9a53352au, \
                       0x921e1761u, 0x34c04e5eu, 0x65724728u, 0x2512d435u, 0x91755d4du, 0x0aa63460u
// 4 R mod q: the curve's b in Montgomery form
#define VL_FQ_B_LIMBS 0x000cfff3u, 0xaa270000u, 0xfc34000au, 0x53cc0032u, 0x6b0a807fu, 0x478fe97au, \
                      0xe6ba24d7u, 0xb1d37ebeu, 0xbf78ab2fu, 0x8ec9733bu, 0x3d83de7eu, 0x09d64551u
// exponents: (q - 1) / 2 (Euler's criterion) and (q + 1) / 4 (square root, q = 3 mod 4)
#define VL_FQ_QM1H_LIMBS 0xffffd555u, 0xdcff7fffu, 0x58a9ffffu, 0x0f55ffffu, 0x7b587b12u, 0xb3986950u, \
                         0x79c2895fu, 0xb23ba5c2u, 0x21a5d66bu, 0x258dd3dbu, 0x1cbff34du, 0x0d0088f5u
#define VL_FQ_QP1Q_LIMBS 0xffffeaabu, 0xee7fbfffu, 0xac54ffffu, 0x07aaffffu, 0x3dac3d89u, 0xd9cc34a8u, \
                         0x3ce144afu, 0xd91dd2e1u, 0x90d2eb35u, 0x92c6e9edu, 0x8e5ff9a6u, 0x0680447au

VL_HD Fq fq_from12(uint32_t a0, uint32_t a1, uint32_t a2, uint32_t a3, uint32_t a4, uint32_t a5,
                   uint32_t a6, uint32_t a7, uint32_t a8, uint32_t a9, uint32_t a10, uint32_t a11) {
  Fq r;
  r.w[0] = a0; r.w[1] = a1; r.w[2] = a2; r.w[3] = a3; r.w[4] = a4; r.w[5] = a5;
  r.w[6] = a6; r.w[7] = a7; r.w[8] = a8; r.w[9] = a9; r.w[10] = a10; r.w[11] = a11;
  return r;
}
VL_HD Fq fq_zero() { Fq r; for (int i = 0; i < 12; ++i) r.w[i] = 0; return r; }
VL_HD Fq fq_one() { return fq_from12(VL_FQ_R_LIMBS); }      // Montgomery form of 1
VL_HD Fq fq_R2() { return fq_from12(VL_FQ_R2_LIMBS); }
VL_HD Fq fq_R3() { return fq_from12(VL_FQ_R3_LIMBS); }
VL_HD Fq fq_b() { return fq_from12(VL_FQ_B_LIMBS); }
VL_HD Fq fq_raw_one() { Fq r = fq_zero(); r.w[0] = 1; return r; }
VL_HD Fq fq_q() { Fq r; for (int i = 0; i < 12; ++i) r.w[i] = q_limb(i); return r; }

VL_HD bool fq_is_zero(const Fq& a) {
  uint32_t d = 0;
#pragma unroll
  for (int i = 0; i < 12; ++i) d |= a.w[i];
  return d == 0;
}
VL_HD bool fq_eq(const Fq& a, const Fq& b) {
  uint32_t d = 0;
#pragma unroll
  for (int i = 0; i < 12; ++i) d |= a.w[i] ^ b.w[i];
  return d == 0;
}

// a - q if a >= q else a   (a < 2q)
VL_HD Fq fq_reduce_once(const Fq& a) {
  Fq t;
  uint32_t borrow = 0;
#pragma unroll
  for (int i = 0; i < 12; ++i) t.w[i] = sbb32(a.w[i], q_limb(i), borrow, borrow);
  Fq r;
#pragma unroll
  for (int i = 0; i < 12; ++i) r.w[i] = borrow ? a.w[i] : t.w[i];
  return r;
}
VL_HD bool fq_lt_q(const Fq& a) {
  uint32_t borrow = 0;
#pragma unroll
  for (int i = 0; i < 12; ++i) (void)sbb32(a.w[i], q_limb(i), borrow, borrow);
  return borrow != 0;
}

VL_HD Fq fq_add(const Fq& a, const Fq& b) {
  Fq s;
  uint32_t c = 0;
#pragma unroll
  for (int i = 0; i < 12; ++i) s.w[i] = adc32(a.w[i], b.w[i], c, c);
  return fq_reduce_once(s);   // a + b < 2q < 2^382
}
VL_HD Fq fq_sub(const Fq& a, const Fq& b) {
  Fq d;
  uint32_t borrow = 0;
#pragma unroll
  for (int i = 0; i < 12; ++i) d.w[i] = sbb32(a.w[i], b.w[i], borrow, borrow);
  const uint32_t mask = 0u - borrow;
  uint32_t c = 0;
#pragma unroll
  for (int i = 0; i < 12; ++i) d.w[i] = adc32(d.w[i], q_limb(i) & mask, c, c);
  return d;
}
VL_HD Fq fq_neg(const Fq& a) { return fq_is_zero(a) ? a : fq_sub(fq_zero(), a); }
VL_HD Fq fq_dbl(const Fq& a) { return fq_add(a, a); }

#if defined(__HIP_DEVICE_COMPILE__)
// Montgomery product a b R^-1 mod q by product scanning (see fr_mul): column
// k collects a_i b_{k-i} and m_i q_{k-i}; for k < 12 the digit m_k =
// t0 (-q^-1) mod 2^32 is chosen so that m_k q_0 clears the column's low word,
// for k >= 12 the low word is result word k - 12.  A column sum of at most
// 24 products stays below 2^69, held as a 64-bit pair plus a top word.
// compile-time loop: f(std::integral_constant<int, I>) for I = B .. E - 1
// (the product's 23 x 24 multiply-adds exceed the unroller's budget, and a
// partly rolled loop would index the limbs dynamically)
template <int B, int E, typename F>
__device__ __forceinline__ void static_for(F&& f) {
  if constexpr (B < E) {
    f(std::integral_constant<int, B>{});
    static_for<B + 1, E>(f);
  }
}

__device__ __forceinline__ Fq fq_mul_dev(const Fq& a, const Fq& b) {
  uint32_t m[12], u[12];
  uint64_t acc = 0;
  uint32_t top = 0;
  static_for<0, 23>([&](auto K) {
    constexpr int k = decltype(K)::value;
    static_for<0, 12>([&](auto I) {
      constexpr int i = decltype(I)::value;
      constexpr int j = k - i;
      if constexpr (j >= 0 && j < 12) fr_mac96(acc, top, a.w[i], b.w[j]);
    });
    static_for<0, 12>([&](auto I) {
      constexpr int i = decltype(I)::value;
      constexpr int j = k - i;
      if constexpr (i < k && j >= 1 && j < 12) fr_mac96s(acc, top, m[i], q_limb(j));
    });
    if constexpr (k < 12) {
      const uint32_t mk = (uint32_t)acc * kQInv32;
      m[k] = mk;
      fr_mac96s(acc, top, mk, q_limb(0));   // the column's low word becomes 0
    } else {
      u[k - 12] = (uint32_t)acc;
    }
    acc = (acc >> 32) | ((uint64_t)top << 32);
    top = 0;
  });
  u[11] = (uint32_t)acc;                      // the result is below 2q < 2^384
  Fq r;
#pragma unroll
  for (int j = 0; j < 12; ++j) r.w[j] = u[j];
  return fq_reduce_once(r);
}
// N (2 or 3) independent products with their partial products interleaved
// instruction by instruction (the multiply-adds of fr_macn / fr_macns carry
// one step of every product), so that the products' dependency chains and
// carry hazards overlap; the same results as N calls of fq_mul_dev.
template <int N>
__device__ __forceinline__ void fq_mul_dev_n(const Fq (&a)[N], const Fq (&b)[N], Fq (&r)[N]) {
  uint32_t m[N][12], u[N][12];
  uint64_t acc[N];
  uint32_t top[N];
#pragma unroll
  for (int c = 0; c < N; ++c) { acc[c] = 0; top[c] = 0; }
  static_for<0, 23>([&](auto K) {
    constexpr int k = decltype(K)::value;
    static_for<0, 12>([&](auto I) {
      constexpr int i = decltype(I)::value;
      constexpr int j = k - i;
      if constexpr (j >= 0 && j < 12) {
        uint32_t x[N], y[N];
#pragma unroll
        for (int c = 0; c < N; ++c) { x[c] = a[c].w[i]; y[c] = b[c].w[j]; }
        fr_macn<N>(acc, top, x, y);
      }
    });
    static_for<0, 12>([&](auto I) {
      constexpr int i = decltype(I)::value;
      constexpr int j = k - i;
      if constexpr (i < k && j >= 1 && j < 12) {
        uint32_t x[N];
#pragma unroll
        for (int c = 0; c < N; ++c) x[c] = m[c][i];
        fr_macns<N>(acc, top, x, q_limb(j));
      }
    });
    if constexpr (k < 12) {
      uint32_t x[N];
#pragma unroll
      for (int c = 0; c < N; ++c) {
        m[c][k] = (uint32_t)acc[c] * kQInv32;
        x[c] = m[c][k];
      }
      fr_macns<N>(acc, top, x, q_limb(0));
    } else {
#pragma unroll
      for (int c = 0; c < N; ++c) u[c][k - 12] = (uint32_t)acc[c];
    }
#pragma unroll
    for (int c = 0; c < N; ++c) {
      acc[c] = (acc[c] >> 32) | ((uint64_t)top[c] << 32);
      top[c] = 0;
    }
  });
#pragma unroll
  for (int c = 0; c < N; ++c) {
    u[c][11] = (uint32_t)acc[c];
    Fq t;
#pragma unroll
    for (int j = 0; j < 12; ++j) t.w[j] = u[c][j];
    r[c] = fq_reduce_once(t);
  }
}

// one out-of-line copy for the code outside the commitment loop (setup,
// reductions, normalisation): inlining every product there makes the kernels
// many times larger and slow to compile; the loop's mixed addition inlines
// its products (g1_add_affine_inl)
__device__ __noinline__ Fq fq_mul_call(const Fq& a, const Fq& b) { return fq_mul_dev(a, b); }
#else
// host: CIOS on 6 64-bit limbs
inline Fq fq_mul_host(const Fq& a, const Fq& b) {
  uint64_t A[6], Bv[6], Qv[6], t[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  memcpy(A, a.w, 48);
  memcpy(Bv, b.w, 48);
  for (int j = 0; j < 6; ++j) Qv[j] = (uint64_t)q_limb(2 * j) | ((uint64_t)q_limb(2 * j + 1) << 32);
  typedef unsigned __int128 u128;
  for (int i = 0; i < 6; ++i) {
    u128 C = 0;
    for (int j = 0; j < 6; ++j) {
      C = (u128)A[j] * Bv[i] + t[j] + (uint64_t)(C >> 64);
      t[j] = (uint64_t)C;
    }
    u128 s = (u128)t[6] + (uint64_t)(C >> 64);
    t[6] = (uint64_t)s;
    t[7] = (uint64_t)(s >> 64);
    const uint64_t m = t[0] * kQInv64;
    C = (u128)m * Qv[0] + t[0];
    for (int j = 1; j < 6; ++j) {
      C = (u128)m * Qv[j] + t[j] + (uint64_t)(C >> 64);
      t[j - 1] = (uint64_t)C;
    }
    s = (u128)t[6] + (uint64_t)(C >> 64);
    t[5] = (uint64_t)s;
    t[6] = t[7] + (uint64_t)(s >> 64);
  }
  Fq r;
  memcpy(r.w, t, 48);
  return fq_reduce_once(r);
}
#endif

VL_HD Fq fq_mul(const Fq& a, const Fq& b) {
#if defined(__HIP_DEVICE_COMPILE__)
  return fq_mul_call(a, b);
#else
  return fq_mul_host(a, b);
#endif
}
VL_HD Fq fq_sqr(const Fq& a) { return fq_mul(a, a); }
VL_HD Fq fq_to_mont(const Fq& a) { return fq_mul(a, fq_R2()); }    // a < 2^384 gives a R mod q
VL_HD Fq fq_from_mont(const Fq& a) { return fq_mul(a, fq_raw_one()); }

// a^e for an exponent given as 12 little-endian limbs (square and multiply
// from the top bit)
template <typename ExpLimb>
VL_HD Fq fq_pow(const Fq& a, ExpLimb e) {
  Fq r = fq_one();
  for (int i = 11; i >= 0; --i) {
    const uint32_t ei = e(i);
    for (int b = 31; b >= 0; --b) {
      r = fq_sqr(r);
      if ((ei >> b) & 1u) r = fq_mul(r, a);
    }
  }
  return r;
}
VL_HD uint32_t pick12(int i, uint32_t a0, uint32_t a1, uint32_t a2, uint32_t a3, uint32_t a4, uint32_t a5,
                      uint32_t a6, uint32_t a7, uint32_t a8, uint32_t a9, uint32_t a10, uint32_t a11) {
  switch (i) {
    case 0: return a0; case 1: return a1; case 2: return a2; case 3: return a3;
    case 4: return a4; case 5: return a5; case 6: return a6; case 7: return a7;
    case 8: return a8; case 9: return a9; case 10: return a10; default: return a11;
  }
}
struct ExpQm1Half {
  VL_HD uint32_t operator()(int i) const { return pick12(i, VL_FQ_QM1H_LIMBS); }
};
struct ExpQp1Quarter {
  VL_HD uint32_t operator()(int i) const { return pick12(i, VL_FQ_QP1Q_LIMBS); }
};

// --- inversion: binary extended Euclid on canonical integers (Hankerson,
// Menezes, Vanstone, Guide to Elliptic Curve Cryptography, Alg. 2.22) ------
VL_HD bool fq_raw_is_one(const Fq& a) {
  uint32_t d = a.w[0] ^ 1u;
#pragma unroll
  for (int i = 1; i < 12; ++i) d |= a.w[i];
  return d == 0;
}
VL_HD Fq fq_raw_shr1(const Fq& a) {
  Fq r;
#pragma unroll
  for (int j = 0; j < 11; ++j) r.w[j] = (a.w[j] >> 1) | (a.w[j + 1] << 31);
  r.w[11] = a.w[11] >> 1;
  return r;
}
// x / 2 mod q for x < q: x or x + q (< 2^382), shifted
VL_HD Fq fq_half(const Fq& x) {
  const uint32_t mask = 0u - (x.w[0] & 1u);
  Fq t;
  uint32_t c = 0;
#pragma unroll
  for (int j = 0; j < 12; ++j) t.w[j] = adc32(x.w[j], q_limb(j) & mask, c, c);
  return fq_raw_shr1(t);
}
// a >= b as integers
VL_HD bool fq_raw_geq(const Fq& a, const Fq& b) {
  uint32_t borrow = 0;
#pragma unroll
  for (int i = 0; i < 12; ++i) (void)sbb32(a.w[i], b.w[i], borrow, borrow);
  return borrow == 0;
}
VL_HD Fq fq_raw_sub(const Fq& a, const Fq& b) {
  Fq d;
  uint32_t borrow = 0;
#pragma unroll
  for (int i = 0; i < 12; ++i) d.w[i] = sbb32(a.w[i], b.w[i], borrow, borrow);
  return d;
}
// The inverse of the Montgomery-form a (0 < a < q), in Montgomery form; 0 for
// a = 0.  The loop keeps x1 a = u and x2 a = v (mod q) with u, v odd after
// their shifts; every step shifts or subtracts, the bit lengths of u and v
// (at most 2 x 381 together) drop by one per shift and a subtraction is
// always followed by a shift, so at most 1524 steps run.  The integer
// inverse of a R is a^-1 R^-1; one product with R^3 gives a^-1 R.
VL_HD Fq fq_inv(const Fq& a) {
  if (fq_is_zero(a)) return a;
  Fq u = a, v = fq_q(), x1 = fq_raw_one(), x2 = fq_zero();
  for (int step = 0; step < 1600; ++step) {
    if (fq_raw_is_one(u) || fq_raw_is_one(v)) break;
    if ((u.w[0] & 1u) == 0) {
      u = fq_raw_shr1(u);
      x1 = fq_half(x1);
    } else if ((v.w[0] & 1u) == 0) {
      v = fq_raw_shr1(v);
      x2 = fq_half(x2);
    } else if (fq_raw_geq(u, v)) {
      u = fq_raw_sub(u, v);
      x1 = fq_sub(x1, x2);
    } else {
      v = fq_raw_sub(v, u);
      x2 = fq_sub(x2, x1);
    }
  }
  return fq_mul(fq_raw_is_one(u) ? x1 : x2, fq_R3());
}

// canonical little-endian bytes <-> limbs
VL_HD void fq_to_bytes(const Fq& a, uint8_t* out) {
  for (int i = 0; i < 12; ++i)
    for (int b = 0; b < 4; ++b) out[4 * i + b] = (uint8_t)(a.w[i] >> (8 * b));
}
VL_HD Fq fq_from_bytes(const uint8_t* in) {
  Fq a;
  for (int i = 0; i < 12; ++i)
    a.w[i] = (uint32_t)in[4 * i] | ((uint32_t)in[4 * i + 1] << 8) | ((uint32_t)in[4 * i + 2] << 16) |
             ((uint32_t)in[4 * i + 3] << 24);
  return a;
}

// ---------------------------------------------------------------- G1 ------
struct G1a {       // affine point (Montgomery coordinates); never infinity
  Fq x, y;
};
struct G1z {       // XYZZ point; ZZ = 0 is infinity
  Fq X, Y, ZZ, ZZZ;
};

VL_HD G1z g1_infinity() {
  G1z r;
  r.X = fq_one(); r.Y = fq_one(); r.ZZ = fq_zero(); r.ZZZ = fq_zero();
  return r;
}
VL_HD bool g1_is_inf(const G1z& p) { return fq_is_zero(p.ZZ); }
VL_HD G1z g1_from_affine(const G1a& a) {
  G1z r;
  r.X = a.x; r.Y = a.y; r.ZZ = fq_one(); r.ZZZ = fq_one();
  return r;
}
VL_HD bool g1_on_curve(const G1a& a) {
  return fq_eq(fq_sqr(a.y), fq_add(fq_mul(fq_sqr(a.x), a.x), fq_b()));
}

// 2 A for an affine A (mdbl-2008-s-1 with a = 0)
VL_HD G1z g1_dbl_affine(const G1a& a) {
  const Fq U = fq_dbl(a.y);
  const Fq V = fq_sqr(U);
  const Fq W = fq_mul(U, V);
  const Fq S = fq_mul(a.x, V);
  const Fq x2 = fq_sqr(a.x);
  const Fq M = fq_add(fq_dbl(x2), x2);
  G1z r;
  r.X = fq_sub(fq_sub(fq_sqr(M), S), S);
  r.Y = fq_sub(fq_mul(M, fq_sub(S, r.X)), fq_mul(W, a.y));
  r.ZZ = V;
  r.ZZZ = W;
  return r;
}

// 2 P (dbl-2008-s-1 with a = 0); infinity stays infinity (ZZ' = V ZZ = 0)
VL_HD G1z g1_dbl(const G1z& p) {
  const Fq U = fq_dbl(p.Y);
  const Fq V = fq_sqr(U);
  const Fq W = fq_mul(U, V);
  const Fq S = fq_mul(p.X, V);
  const Fq x2 = fq_sqr(p.X);
  const Fq M = fq_add(fq_dbl(x2), x2);
  G1z r;
  r.X = fq_sub(fq_sub(fq_sqr(M), S), S);
  r.Y = fq_sub(fq_mul(M, fq_sub(S, r.X)), fq_mul(W, p.Y));
  r.ZZ = fq_mul(V, p.ZZ);
  r.ZZZ = fq_mul(W, p.ZZZ);
  return r;
}

// P + A for an affine A (madd-2008-s)
VL_HD G1z g1_add_affine(const G1z& p, const G1a& a) {
  if (g1_is_inf(p)) return g1_from_affine(a);
  const Fq U2 = fq_mul(a.x, p.ZZ);
  const Fq S2 = fq_mul(a.y, p.ZZZ);
  const Fq P = fq_sub(U2, p.X);
  const Fq R = fq_sub(S2, p.Y);
  if (fq_is_zero(P)) {
    if (fq_is_zero(R)) return g1_dbl_affine(a);
    return g1_infinity();
  }
  const Fq PP = fq_sqr(P);
  const Fq PPP = fq_mul(P, PP);
  const Fq Qv = fq_mul(p.X, PP);
  G1z r;
  r.X = fq_sub(fq_sub(fq_sub(fq_sqr(R), PPP), Qv), Qv);
  r.Y = fq_sub(fq_mul(R, fq_sub(Qv, r.X)), fq_mul(p.Y, PPP));
  r.ZZ = fq_mul(p.ZZ, PP);
  r.ZZZ = fq_mul(p.ZZZ, PPP);
  return r;
}

// P1 + P2 (add-2008-s)
VL_HD G1z g1_add(const G1z& p, const G1z& q2) {
  if (g1_is_inf(p)) return q2;
  if (g1_is_inf(q2)) return p;
  const Fq U1 = fq_mul(p.X, q2.ZZ);
  const Fq U2 = fq_mul(q2.X, p.ZZ);
  const Fq S1 = fq_mul(p.Y, q2.ZZZ);
  const Fq S2 = fq_mul(q2.Y, p.ZZZ);
  const Fq P = fq_sub(U2, U1);
  const Fq R = fq_sub(S2, S1);
  if (fq_is_zero(P)) {
    if (fq_is_zero(R)) return g1_dbl(p);
    return g1_infinity();
  }
  const Fq PP = fq_sqr(P);
  const Fq PPP = fq_mul(P, PP);
  const Fq Qv = fq_mul(U1, PP);
  G1z r;
  r.X = fq_sub(fq_sub(fq_sub(fq_sqr(R), PPP), Qv), Qv);
  r.Y = fq_sub(fq_mul(R, fq_sub(Qv, r.X)), fq_mul(S1, PPP));
  r.ZZ = fq_mul(fq_mul(p.ZZ, q2.ZZ), PP);
  r.ZZZ = fq_mul(fq_mul(p.ZZZ, q2.ZZZ), PPP);
  return r;
}

// affine coordinates of a finite P: x = X / ZZ, y = Y / ZZZ from the one
// inverse of ZZ ZZZ
VL_HD G1a g1_to_affine(const G1z& p) {
  const Fq t = fq_inv(fq_mul(p.ZZ, p.ZZZ));
  G1a a;
  a.x = fq_mul(p.X, fq_mul(t, p.ZZZ));
  a.y = fq_mul(p.Y, fq_mul(t, p.ZZ));
  return a;
}

// k A for an affine A and an unsigned scalar (double and add from the top bit)
VL_HD G1z g1_mul_u64(const G1a& a, uint64_t k) {
  if (k == 0) return g1_infinity();
  int b = 63;
  while (!((k >> b) & 1u)) --b;
  G1z r = g1_from_affine(a);
  for (--b; b >= 0; --b) {
    r = g1_dbl(r);
    if ((k >> b) & 1u) r = g1_add_affine(r, a);
  }
  return r;
}

// 96-byte encoding: x then y, each 48 bytes little-endian canonical; the
// point at infinity is 96 zero bytes
VL_HD void g1_encode(const G1z& p, uint8_t* out) {
  if (g1_is_inf(p)) {
    for (int i = 0; i < 96; ++i) out[i] = 0;
    return;
  }
  const G1a a = g1_to_affine(p);
  fq_to_bytes(fq_from_mont(a.x), out);
  fq_to_bytes(fq_from_mont(a.y), out + 48);
}

// ------------------------------------------------ hashing to the curve ----
// SHA-256 of tag || u32 j || u32 ctr || u8 b (26 bytes, one padded block),
// tag = "VeriLoRA-hyrax-v1"; h receives the digest's 8 big-endian words.
VL_HD void hyrax_hash(uint32_t j, uint32_t ctr, uint32_t b, uint32_t h[8]) {
  // the 17 tag bytes as big-endian words, then j, ctr, b, the 0x80 pad byte
  // and the bit length 208 in the last word
  uint32_t w[16];
  w[0] = 0x56657269u;   // "Veri"
  w[1] = 0x4c6f5241u;   // "LoRA"
  w[2] = 0x2d687972u;   // "-hyr"
  w[3] = 0x61782d76u;   // "ax-v"
  const uint32_t jb[4] = {j & 0xffu, (j >> 8) & 0xffu, (j >> 16) & 0xffu, j >> 24};
  const uint32_t cb[4] = {ctr & 0xffu, (ctr >> 8) & 0xffu, (ctr >> 16) & 0xffu, ctr >> 24};
  w[4] = (0x31u << 24) | (jb[0] << 16) | (jb[1] << 8) | jb[2];          // "1", j0..j2
  w[5] = (jb[3] << 24) | (cb[0] << 16) | (cb[1] << 8) | cb[2];          // j3, ctr0..ctr2
  w[6] = (cb[3] << 24) | ((b & 0xffu) << 16) | (0x80u << 8);            // ctr3, b, pad
  for (int i = 7; i < 15; ++i) w[i] = 0;
  w[15] = 26 * 8;
  h[0] = 0x6a09e667u; h[1] = 0xbb67ae85u; h[2] = 0x3c6ef372u; h[3] = 0xa54ff53au;
  h[4] = 0x510e527fu; h[5] = 0x9b05688cu; h[6] = 0x1f83d9abu; h[7] = 0x5be0cd19u;
  sha256_compress_w(h, w);
}

VL_HD uint32_t bswap32(uint32_t x) {
  return (x >> 24) | ((x >> 8) & 0xff00u) | ((x << 8) & 0xff0000u) | (x << 24);
}

// G_j, the j-th Hyrax generator: for ctr = 0, 1, ..:
// X = LE(H(.., ctr, 0) || H(.., ctr, 1)) mod q; when X^3 + 4 is a square
// (Euler's criterion) its even root y gives the point (X, y), and
// G_j = h_eff (X, y) lies in the order-p subgroup (h_eff = 1 - x for the
// curve's parameter x = -0xd201000000010000).  The 512-bit X is reduced as
// lo + hi 2^384 with Montgomery products by R^2 and R^3.  Returns false if
// no counter below max_ctr succeeds (each succeeds with probability 1/2).
constexpr uint64_t kHyraxHEff = 0xd201000000010001ull;
VL_HD bool hyrax_generator(uint32_t j, G1a& out, uint32_t max_ctr = 256) {
  for (uint32_t ctr = 0; ctr < max_ctr; ++ctr) {
    uint32_t h0[8], h1[8];
    hyrax_hash(j, ctr, 0, h0);
    hyrax_hash(j, ctr, 1, h1);
    Fq lo, hi = fq_zero();
    for (int k = 0; k < 8; ++k) lo.w[k] = bswap32(h0[k]);
    for (int k = 0; k < 4; ++k) lo.w[8 + k] = bswap32(h1[k]);
    for (int k = 0; k < 4; ++k) hi.w[k] = bswap32(h1[4 + k]);
    const Fq X = fq_add(fq_mul(lo, fq_R2()), fq_mul(hi, fq_R3()));
    const Fq s = fq_add(fq_mul(fq_sqr(X), X), fq_b());
    if (!fq_eq(fq_pow(s, ExpQm1Half{}), fq_one())) continue;
    Fq y = fq_pow(s, ExpQp1Quarter{});
    if (fq_from_mont(y).w[0] & 1u) y = fq_neg(y);
    G1a a;
    a.x = X;
    a.y = y;
    const G1z G = g1_mul_u64(a, kHyraxHEff);
    if (g1_is_inf(G)) continue;
    out = g1_to_affine(G);
    return true;
  }
  return false;
}

}  // namespace vl
