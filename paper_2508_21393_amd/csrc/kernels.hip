// Device kernels of the matmul-sumcheck prover (gfx950).
//
// Paths and the paper passages they compute:
//   eq_kernel        eq(x, i) tables, eq. (MLE) Lagrange basis
//   contract_kernel  A~(u, w) and B~(w, v) partial evaluations and the claim's
//                    first contraction, eq. (zk-mle-matmul)
//   finish_kernel    sums split contractions, zero pads to a power of two
//   rounds_kernel    claim c = C~(u, v), the sumcheck rounds (Sec. II-B.1)
//                    with Fiat-Shamir challenges, and the fold of each round
//   lift/export      integer -> Fr lifting (x < 0 -> p - |x|) and back to
//                    canonical form
//
// The integer contraction (the hot loop) never multiplies two field elements.
// Each eq entry e (stored as e * R^2 mod p < 2^255, so that one Montgomery
// reduction at the end lands in Montgomery form) is cut into 32 bytes e_k,
// each matrix entry x into signed 16-bit digits d_t.  The exact integer
//     sum_m e[m] * x[m] = sum_{k,t} 2^(8k + 16t) * sum_m e_k[m] * d_t[m]
// is accumulated with v_dot2_i32_i16, two consecutive m per instruction:
// the byte pair (e_k[m], e_k[m+1]) comes from a scalar register (the eq
// table is wave-uniform) and the digit pair from a vector register.  Each
// dot2 adds at most 2 * 255 * 2^15 < 2^24 in magnitude, so 128 of them fit an
// int32 accumulator; every 128 pairs the 32 accumulators are folded into
// 64-bit limb sums.  At the end of a chunk the signed ~300-bit sum is reduced
// with one Montgomery multiplication (see finalize).
#include <cstring>

#include "internal.hpp"
#include "sha256.hpp"

namespace vl {

typedef short v2i16 __attribute__((ext_vector_type(2)));
typedef const __attribute__((address_space(4))) uint32_t* cu32_ptr;
typedef const __attribute__((address_space(4))) int32_t* ci32_ptr;

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

__device__ __forceinline__ int32_t sdot2(uint32_t e, uint32_t x, int32_t acc) {
  return __builtin_amdgcn_sdot2(__builtin_bit_cast(v2i16, e), __builtin_bit_cast(v2i16, x), acc,
                                false);
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

// ---------------------------------------------------------------- eq -------
__global__ void __launch_bounds__(256) eq_kernel(const EqJob* __restrict__ jobs, uint32_t n_jobs,
                                                 uint32_t n_threads) {
  const uint32_t tid = blockIdx.x * blockDim.x + threadIdx.x;
  if (tid >= n_threads) return;
  uint32_t lo = 0, hi = n_jobs;
  while (hi - lo > 1) {
    const uint32_t mid = (lo + hi) >> 1;
    if (jobs[mid].thread_begin <= tid) lo = mid; else hi = mid;
  }
  const EqJob& J = jobs[lo];
  const uint32_t t = tid - J.thread_begin;   // pair index: entries 2t and 2t+1
  const uint32_t n = J.nvars;
  const uint64_t len = 1ull << n;
  Fr e0, e1;
  if (n == 0) {
    e0 = fr_R();
    e1 = fr_zero();
  } else {
    Fr base = fr_R();
    for (uint32_t j = 0; j + 1 < n; ++j) {
      const uint32_t bit = (t >> (n - 2 - j)) & 1u;
      const uint32_t* xp = J.point + (2 * j + (bit ? 0 : 1)) * 8;
      Fr x;
#pragma unroll
      for (int k = 0; k < 8; ++k) x.w[k] = xp[k];
      base = fr_mul(base, x);
    }
    Fr xl, oml;
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      xl.w[k] = J.point[(2 * (n - 1)) * 8 + k];
      oml.w[k] = J.point[(2 * (n - 1) + 1) * 8 + k];
    }
    e0 = fr_mul(base, oml);
    e1 = fr_mul(base, xl);
  }
  if (J.eq) {
    if (2ull * t < len) store_sol(J.eq, J.eq_ld, 2ull * t, e0);
    if (2ull * t + 1 < len) store_sol(J.eq, J.eq_ld, 2ull * t + 1, e1);
  }
  if (J.pack) {
    // pack: e * R^2 mod p as signed digits, 8 words per entry
    if (2 * t < J.pack_len) signed_digits(fr_to_mont(e0), J.pack + (uint64_t)(2 * t) * 8);
    if (2 * t + 1 < J.pack_len) signed_digits(fr_to_mont(e1), J.pack + (uint64_t)(2 * t + 1) * 8);
  }
}

// eq table for a point passed by value (vl_eq_table): no device staging
__global__ void __launch_bounds__(256) eq_point_kernel(EqPointArgs a) {
  const uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const uint32_t n = a.nvars;
  const uint64_t len = 1ull << n;
  if (2 * t >= len && !(n == 0 && t == 0)) return;
  Fr e0, e1;
  if (n == 0) {
    e0 = fr_R();
    e1 = fr_zero();
  } else {
    Fr base = fr_R();
    for (uint32_t j = 0; j + 1 < n; ++j) {
      const uint32_t bit = (uint32_t)(t >> (n - 2 - j)) & 1u;
      Fr x;
#pragma unroll
      for (int k = 0; k < 8; ++k) x.w[k] = a.pt[j][bit ? 0 : 1][k];
      base = fr_mul(base, x);
    }
    Fr xl, oml;
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      xl.w[k] = a.pt[n - 1][0][k];
      oml.w[k] = a.pt[n - 1][1][k];
    }
    e0 = fr_mul(base, oml);
    e1 = fr_mul(base, xl);
  }
  if (2 * t < len) store_sol(a.out, a.ld, 2 * t, e0);
  if (2 * t + 1 < len) store_sol(a.out, a.ld, 2 * t + 1, e1);
}

// pack form of a caller-provided eq vector (vl_mle_partial_eval)
__global__ void __launch_bounds__(256) pack_kernel(const uint32_t* __restrict__ eq, uint64_t ld,
                                                   uint64_t len, uint32_t* __restrict__ pack) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= len) return;
  signed_digits(fr_to_mont(load_sol(eq, ld, i)), pack + i * 8);
}

// ---------------------------------------------------------------- contract --
// Signed digits of an entry for v_mad_i64_i32: x = sum_t d_t 2^(DB t) with
// d_t in [-2^(DB-1), 2^(DB-1)).  int16 entries are their own single digit.
template <typename T, int ND, int DB>
__device__ __forceinline__ void entry_digits(T x, int32_t (&d)[ND], uint32_t& bad) {
  if constexpr (ND == 1 && sizeof(T) == 2) {
    d[0] = (int32_t)x;
  } else {
    int64_t r = (int64_t)x;
#pragma unroll
    for (int t = 0; t < ND; ++t) {
      d[t] = (int32_t)((uint32_t)r << (32 - DB)) >> (32 - DB);
      // r <- (r - d_t) / 2^DB, written so that it cannot overflow
      r = (r >> DB) + ((r >> (DB - 1)) & 1);
    }
    bad |= (uint32_t)(r != 0);
  }
}

// acc[o][t][j] += e_j * d[o][t] for the 8 signed eq digits e_j (wave-uniform,
// scalar registers); one v_mad_i64_i32 each
template <int OPL, int ND>
__device__ __forceinline__ void mac8(ci32_ptr e, const int32_t (&d)[OPL][ND],
                                     int64_t (&acc)[OPL][ND][8]) {
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    const int32_t ev = e[j];
#pragma unroll
    for (int o = 0; o < OPL; ++o)
#pragma unroll
      for (int t = 0; t < ND; ++t) acc[o][t][j] += (int64_t)ev * (int64_t)d[o][t];
  }
}

// wide digits (DB = 24): move the high words out before an int64 can overflow
template <int OPL, int ND>
__device__ __forceinline__ void spill_high(int64_t (&acc)[OPL][ND][8], int64_t (&hi)[OPL][ND][8]) {
#pragma unroll
  for (int o = 0; o < OPL; ++o)
#pragma unroll
    for (int t = 0; t < ND; ++t)
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const int64_t h = acc[o][t][j] >> 32;
        hi[o][t][j] += h;
        acc[o][t][j] -= (int64_t)((uint64_t)h << 32);
      }
}

// V = sum_{t,j} (acc + 2^32 hi) 2^(DB t + 32 j), congruent to R^2 * value
// (the eq digits hold e * R^2 mod p).  With V = lo + 2^256 hi (lo unsigned
// 256-bit, |hi| < 2^80): V * R^-1 = lo * R^-1 + hi (mod p), i.e. one
// Montgomery multiplication by 1 plus a small signed lift.  (A direct
// 12-limb REDC written with 64-bit adds lost a carry when compiled for gfx950
// at -O3, so the reduction goes through the field multiplier.)
template <int ND, int DB>
__device__ __forceinline__ Fr finalize_digits(const int64_t (&acc)[ND][8], const int64_t (&hi)[ND][8]) {
  int64_t S[12];
#pragma unroll
  for (int q = 0; q < 12; ++q) S[q] = 0;
#pragma unroll
  for (int t = 0; t < ND; ++t) {
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int bit = DB * t;
      const int b = j + bit / 32, sh = bit % 32;
      const int64_t a = acc[t][j];
      const int64_t H = (a >> 32) + hi[t][j];
      const uint64_t lo = (uint64_t)(uint32_t)a << sh;
      S[b] += (int64_t)(lo & 0xffffffffu);
      S[b + 1] += (int64_t)(lo >> 32);
      S[b + 1] += (int64_t)(uint32_t)((uint64_t)H << sh);
      S[b + 2] += sh == 0 ? (H >> 32) : (H >> (32 - sh));
    }
  }
  uint32_t L[12];
  int64_t carry = 0;
#pragma unroll
  for (int q = 0; q < 12; ++q) {
    const int64_t v = S[q] + carry;
    L[q] = (uint32_t)v;
    carry = v >> 32;
  }
  Fr lo;
#pragma unroll
  for (int j = 0; j < 8; ++j) lo.w[j] = L[j];
  lo = fr_reduce_once(fr_reduce_once(lo));   // 2^256 < 3p
  const Fr part = fr_mul(lo, fr_one_raw());
  const bool neg = (L[11] >> 31) != 0;
  Fr h = fr_zero();
  if (!neg) {
#pragma unroll
    for (int j = 0; j < 4; ++j) h.w[j] = L[8 + j];
  } else {
    uint32_t c = 1;   // |hi| = ~hi + 1
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const uint32_t w = ~L[8 + j];
      h.w[j] = w + c;
      c = (h.w[j] < w) ? 1u : 0u;
    }
    h = fr_neg(h);
  }
  return fr_add(part, h);
}

// One wave per task: OPL consecutive outputs per lane (rows kernel: columns
// of the stored matrix; cols kernel: its rows), one chunk of the contraction
// index.  DB = 16 (int16 entries): products < 2^46, so int64 accumulators
// hold 2^16 entries (chunks never exceed that).  DB = 24: products < 2^54,
// high words are moved out every 256 entries.
template <typename T, int ND, int DB, bool ROWS, bool VEC, int OPL>
__global__ void __launch_bounds__(kContractBlock)
contract_kernel(const ContractJob* __restrict__ jobs, uint32_t n_jobs, uint32_t n_tasks) {
  constexpr bool WIDE = DB > 16;
  constexpr uint32_t kSpill = 256;
  const uint32_t task = __builtin_amdgcn_readfirstlane(blockIdx.x * 4 + (threadIdx.x >> 6));
  if (task >= n_tasks) return;
  uint32_t lo = 0, hi_i = n_jobs;
  while (hi_i - lo > 1) {
    const uint32_t mid = (lo + hi_i) >> 1;
    if (jobs[mid].task_begin <= task) lo = mid; else hi_i = mid;
  }
  const ContractJob& J = jobs[lo];
  const uint32_t local = task - J.task_begin;
  const uint32_t chunk = local % J.n_chunks;
  const uint32_t owave = local / J.n_chunks;
  const uint32_t lane = threadIdx.x & 63u;
  const uint32_t n0 = (owave * 64u + lane) * OPL;
  const uint32_t m0 = chunk * J.chunk;
  const uint32_t m1 = min(m0 + J.chunk, J.len);
  const T* __restrict__ M = (const T*)J.M;
  const uint64_t ld = J.ld;
  const uint32_t n_out = J.n_out;
  cu32_ptr pk32 = (cu32_ptr)J.pack;
  ci32_ptr pack = (ci32_ptr)pk32;

  int64_t acc[OPL][ND][8];
  int64_t hi[OPL][ND][8];
#pragma unroll
  for (int o = 0; o < OPL; ++o)
#pragma unroll
    for (int t = 0; t < ND; ++t)
#pragma unroll
      for (int j = 0; j < 8; ++j) acc[o][t][j] = hi[o][t][j] = 0;
  uint32_t bad = 0;

  uint32_t m = m0;
  if constexpr (VEC && !ROWS) {
    // cols layout, 16-byte aligned rows: each lane streams its own row 16
    // bytes at a time, the next 16 bytes in flight while these are used
    static_assert(OPL == 1, "vector cols kernel has one row per lane");
    constexpr uint32_t BE = 16 / sizeof(T);
    const bool valid = n0 < n_out;
    const uint4* row = (const uint4*)(M + (uint64_t)(valid ? n0 : 0u) * ld);
    const uint32_t mv = m0 + ((m1 - m0) / BE) * BE;
    if (m < mv) {
      uint4 cur = valid ? row[m / BE] : make_uint4(0, 0, 0, 0);
      while (m < mv) {
        const uint32_t bend = WIDE ? min(m + kSpill, mv) : mv;
        for (; m < bend; m += BE) {
          uint4 nxt = make_uint4(0, 0, 0, 0);
          if (valid && m + BE < mv) nxt = row[m / BE + 1];
          const T* x = (const T*)&cur;
#pragma unroll
          for (uint32_t q = 0; q < BE; ++q) {
            int32_t d[1][ND];
            entry_digits<T, ND, DB>(x[q], d[0], bad);
            mac8<1, ND>(pack + (uint64_t)(m + q) * 8, d, acc);
          }
          cur = nxt;
        }
        if constexpr (WIDE) spill_high<OPL, ND>(acc, hi);
      }
    }
  }
  if constexpr (VEC && ROWS) {
    // rows layout, four int16 columns per lane read as one 8-byte load;
    // batches of four rows, the next batch in flight while this one is used
    static_assert(OPL == 4 && sizeof(T) == 2 && !WIDE, "vector rows kernel: int16, 4 columns");
    constexpr uint32_t BR = 4;
    const bool full = n0 + 3 < n_out;
    auto load4 = [&](uint32_t mm) -> uint2 {
      uint2 v = make_uint2(0, 0);
      if (mm < m1) {
        if (full) {
          v = *(const uint2*)(M + (uint64_t)mm * ld + n0);
        } else {
          uint16_t e[4] = {0, 0, 0, 0};
#pragma unroll
          for (int o = 0; o < 4; ++o)
            if (n0 + o < n_out) e[o] = (uint16_t)M[(uint64_t)mm * ld + n0 + o];
          v = make_uint2(e[0] | ((uint32_t)e[1] << 16), e[2] | ((uint32_t)e[3] << 16));
        }
      }
      return v;
    };
    uint2 cur[BR];
#pragma unroll
    for (uint32_t r = 0; r < BR; ++r) cur[r] = load4(m + r);
    for (; m < m1; m += BR) {
      uint2 nxt[BR];
#pragma unroll
      for (uint32_t r = 0; r < BR; ++r) nxt[r] = load4(m + BR + r);
#pragma unroll
      for (uint32_t r = 0; r < BR; ++r) {
        if (m + r < m1) {
          int32_t d[OPL][ND];
          d[0][0] = (int32_t)(int16_t)(cur[r].x & 0xffffu);
          d[1][0] = (int32_t)(int16_t)(cur[r].x >> 16);
          d[2][0] = (int32_t)(int16_t)(cur[r].y & 0xffffu);
          d[3][0] = (int32_t)(int16_t)(cur[r].y >> 16);
          mac8<OPL, ND>(pack + (uint64_t)(m + r) * 8, d, acc);
        }
      }
#pragma unroll
      for (uint32_t r = 0; r < BR; ++r) cur[r] = nxt[r];
    }
  }
  while (m < m1) {
    const uint32_t bend = WIDE ? min(m + kSpill, m1) : m1;
#pragma unroll 4
    for (; m < bend; ++m) {
      int32_t d[OPL][ND];
#pragma unroll
      for (int o = 0; o < OPL; ++o) {
        const uint32_t n = n0 + o;
        T x = 0;
        if (n < n_out) x = ROWS ? M[(uint64_t)m * ld + n] : M[(uint64_t)n * ld + m];
        entry_digits<T, ND, DB>(x, d[o], bad);
      }
      mac8<OPL, ND>(pack + (uint64_t)m * 8, d, acc);
    }
    if constexpr (WIDE) spill_high<OPL, ND>(acc, hi);
  }
  if constexpr (ND > 1 || sizeof(T) > 2) {
    if (bad && J.err) atomicOr(J.err, 1);
  }
#pragma unroll
  for (int o = 0; o < OPL; ++o) {
    const Fr r = finalize_digits<ND, DB>(acc[o], hi[o]);
    const uint32_t n = n0 + o;
    if (n < n_out) store_sol(J.dst + (uint64_t)chunk * J.chunk_stride, J.dst_ld, n, r);
  }
}

// ---------------------------------------------------------------- finish ----
__global__ void __launch_bounds__(256) finish_kernel(const FinishJob* __restrict__ jobs,
                                                     uint32_t n_jobs, uint32_t n_threads) {
  const uint32_t tid = blockIdx.x * blockDim.x + threadIdx.x;
  if (tid >= n_threads) return;
  uint32_t lo = 0, hi = n_jobs;
  while (hi - lo > 1) {
    const uint32_t mid = (lo + hi) >> 1;
    if (jobs[mid].thread_begin <= tid) lo = mid; else hi = mid;
  }
  const FinishJob& J = jobs[lo];
  const uint32_t i = tid - J.thread_begin;
  if (i < J.n_valid) {
    if (!J.part) return;
    Fr s = load_sol(J.part, J.part_ld, i);
    for (uint32_t c = 1; c < J.n_chunks; ++c)
      s = fr_add(s, load_sol(J.part + (uint64_t)c * J.chunk_stride, J.part_ld, i));
    store_sol(J.out, J.out_ld, i, s);
  } else if (i < J.n_total) {
    store_sol(J.out, J.out_ld, i, fr_zero());
  }
}

// ---------------------------------------------------------------- rounds ----
template <int K>
__device__ __forceinline__ void block_sum(Fr (&v)[K], uint32_t* lds) {
  constexpr int NW = kRoundsBlock / kWave;
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) {
#pragma unroll
    for (int k = 0; k < K; ++k) {
      Fr o;
#pragma unroll
      for (int j = 0; j < 8; ++j) o.w[j] = __shfl_xor(v[k].w[j], off, kWave);
      v[k] = fr_add(v[k], o);
    }
  }
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  if (lane == 0) {
#pragma unroll
    for (int k = 0; k < K; ++k)
#pragma unroll
      for (int j = 0; j < 8; ++j) lds[(k * 8 + j) * NW + wave] = v[k].w[j];
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < K; ++k) {
    Fr s = fr_zero();
    for (int w = 0; w < NW; ++w) {
      Fr o;
#pragma unroll
      for (int j = 0; j < 8; ++j) o.w[j] = lds[(k * 8 + j) * NW + w];
      s = fr_add(s, o);
    }
    v[k] = s;
  }
  __syncthreads();
}

__device__ __forceinline__ void put_fr(uint8_t* dst, const Fr& mont) {
  const Fr c = fr_from_mont(mont);
  uint8_t b[32];
  fr_to_bytes(c, b);
  for (int i = 0; i < 32; ++i) dst[i] = b[i];
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

// (2 b - a) for the evaluation at X = 2 of the line through (0, a), (1, b)
__device__ __forceinline__ Fr at_two(const Fr& a, const Fr& b) { return fr_sub(fr_double(b), a); }

// One workgroup per group.  Round 1 of every product is computed in a first
// pass (its g(0) + g(1) is the product's sum, so the prover guard needs no
// extra pass); later rounds compute g(0) and g(2) and take g(1) = claim - g(0),
// the claim moving to g(r) by interpolation on {0, 1, 2}.  All of it leaves
// the proof bytes unchanged.
__global__ void __launch_bounds__(kRoundsBlock) rounds_kernel(const RoundsJob* __restrict__ jobs) {
  const RoundsJob& J = jobs[blockIdx.x];
  __shared__ uint32_t red[3 * 8 * (kRoundsBlock / kWave)];
  __shared__ uint32_t first[VL_MAX_PRODS][3][8];   // round-1 values per product
  __shared__ uint32_t bcast[2][8];                 // r and the next claim
  const uint32_t tid = threadIdx.x, NT = blockDim.x;

  if (J.err && *(volatile const int32_t*)J.err) {
    if (tid == 0) *J.status = VL_ERR_RANGE;
    return;
  }
  // c = C~(u, v) = sum_i eq(u, i) t[i]
  Fr v1[1];
  v1[0] = fr_zero();
  const uint32_t len0 = 1u << J.n0;
  for (uint32_t i = tid; i < len0; i += NT)
    v1[0] = fr_add(v1[0], fr_mul(load_sol(J.eqU, J.eqU_ld, i), load_sol(J.t, J.t_ld, i)));
  block_sum<1>(v1, red);
  const Fr c = v1[0];

  // round 1 of every product; its g(0) + g(1) = sum_w a_p[w] b_p[w]
  Fr total = fr_zero();
  for (uint32_t p = 0; p < J.n_prods; ++p) {
    const RoundsProd& P = J.prods[p];
    Fr g[3];
    g[0] = g[1] = g[2] = fr_zero();
    if (P.n1 == 0) {
      if (tid == 0) g[0] = fr_mul(load_sol(P.a, P.ld, 0), load_sol(P.b, P.ld, 0));
    } else {
      const uint32_t h = 1u << (P.n1 - 1);
      for (uint32_t t = tid; t < h; t += NT) {
        const Fr a0 = load_sol(P.a, P.ld, t), a1 = load_sol(P.a, P.ld, t + h);
        const Fr b0 = load_sol(P.b, P.ld, t), b1 = load_sol(P.b, P.ld, t + h);
        g[0] = fr_add(g[0], fr_mul(a0, b0));
        g[1] = fr_add(g[1], fr_mul(a1, b1));
        g[2] = fr_add(g[2], fr_mul(at_two(a0, a1), at_two(b0, b1)));
      }
    }
    block_sum<3>(g, red);
    if (tid == 0)
#pragma unroll
      for (int k = 0; k < 3; ++k) lds_put(first[p][k], g[k]);
    total = fr_add(total, fr_add(g[0], g[1]));
  }
  if (!fr_eq(total, c)) {
    if (tid == 0) *J.status = VL_ERR_FALSE_STATEMENT;
    return;
  }
  __syncthreads();

  Transcript tr;
  uint8_t* out = J.proof;
  if (tid == 0) {
#pragma unroll
    for (int i = 0; i < 8; ++i) tr.h[i] = J.st[i];
    const Fr cc[1] = {fr_from_mont(c)};
    put_fr(out, c);
    out += 32;
    tr_absorb_frs(tr, VL_LBL_CLAIM, cc);
    for (uint32_t p = 0; p + 1 < J.n_prods; ++p) {
      const Fr sp = fr_add(lds_get(first[p][0]), lds_get(first[p][1]));
      const Fr sc[1] = {fr_from_mont(sp)};
      put_fr(out, sp);
      out += 32;
      tr_absorb_frs(tr, VL_LBL_PART, sc);
    }
  }
  const Fr one = fr_R(), two = fr_double(fr_R());
  const Fr inv2 = fr_from_limbs(0xffffffffu, 0x00000000u, 0x0001a401u, 0xac425bfdu, 0xf65e27fau,
                                0xccc627f7u, 0xd66282b7u, 0x0c1258acu);  // 2^-1 R mod p
  for (uint32_t p = 0; p < J.n_prods; ++p) {
    const RoundsProd& P = J.prods[p];
    uint32_t* a = P.a;
    uint32_t* b = P.b;
    const uint64_t ld = P.ld;
    Fr claim = fr_add(lds_get(first[p][0]), lds_get(first[p][1]));
    for (uint32_t rd = 0; rd < P.n1; ++rd) {
      const uint32_t h = 1u << (P.n1 - 1 - rd);
      Fr g[3];
      if (rd == 0) {
#pragma unroll
        for (int k = 0; k < 3; ++k) g[k] = lds_get(first[p][k]);
      } else {
        Fr q[2];
        q[0] = q[1] = fr_zero();
        for (uint32_t t = tid; t < h; t += NT) {
          const Fr a0 = load_sol(a, ld, t), a1 = load_sol(a, ld, t + h);
          const Fr b0 = load_sol(b, ld, t), b1 = load_sol(b, ld, t + h);
          q[0] = fr_add(q[0], fr_mul(a0, b0));
          q[1] = fr_add(q[1], fr_mul(at_two(a0, a1), at_two(b0, b1)));
        }
        block_sum<2>(q, red);
        g[0] = q[0];
        g[1] = fr_sub(claim, q[0]);
        g[2] = q[1];
      }
      if (tid == 0) {
        Fr gc[3];
        for (int k = 0; k < 3; ++k) {
          gc[k] = fr_from_mont(g[k]);
          put_fr(out, g[k]);
          out += 32;
        }
        tr_absorb_frs(tr, VL_LBL_ROUND, gc);
        const Fr r = fr_to_mont(tr_squeeze_fixed(tr, VL_LBL_R));
        // g(r) = g0 (r-1)(r-2)/2 - g1 r (r-2) + g2 r (r-1)/2
        const Fr rm1 = fr_sub(r, one), rm2 = fr_sub(r, two);
        const Fr l0 = fr_mul(fr_mul(rm1, rm2), inv2);
        const Fr l1 = fr_neg(fr_mul(r, rm2));
        const Fr l2 = fr_mul(fr_mul(r, rm1), inv2);
        const Fr next = fr_add(fr_add(fr_mul(g[0], l0), fr_mul(g[1], l1)), fr_mul(g[2], l2));
        lds_put(bcast[0], r);
        lds_put(bcast[1], next);
      }
      __syncthreads();
      const Fr r = lds_get(bcast[0]);
      claim = lds_get(bcast[1]);
      for (uint32_t t = tid; t < h; t += NT) {
        const Fr a0 = load_sol(a, ld, t), a1 = load_sol(a, ld, t + h);
        const Fr b0 = load_sol(b, ld, t), b1 = load_sol(b, ld, t + h);
        store_sol(a, ld, t, fr_add(a0, fr_mul(r, fr_sub(a1, a0))));
        store_sol(b, ld, t, fr_add(b0, fr_mul(r, fr_sub(b1, b0))));
      }
      __threadfence_block();
      __syncthreads();
    }
    if (tid == 0) {
      Fr fin[2];
      fin[0] = load_sol(a, ld, 0);
      fin[1] = load_sol(b, ld, 0);
      put_fr(out, fin[0]);
      out += 32;
      put_fr(out, fin[1]);
      out += 32;
      fin[0] = fr_from_mont(fin[0]);
      fin[1] = fr_from_mont(fin[1]);
      tr_absorb_frs(tr, VL_LBL_FINAL, fin);
    }
    __syncthreads();
  }
  if (tid == 0) {
    if (J.digest) {
      uint8_t d[32];
      tr_to_bytes(tr, d);
      for (int i = 0; i < 32; ++i) J.digest[i] = d[i];
    }
    *J.status = VL_OK;
  }
}

// ---------------------------------------------------------------- lift ------
template <typename T>
__global__ void __launch_bounds__(256) lift_kernel(const T* __restrict__ src, uint64_t n,
                                                   uint32_t* __restrict__ dst, uint64_t ld) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int64_t x = (int64_t)src[i];
  const uint64_t mag = x < 0 ? (uint64_t)0 - (uint64_t)x : (uint64_t)x;
  Fr v = fr_zero();
  v.w[0] = (uint32_t)mag;
  v.w[1] = (uint32_t)(mag >> 32);
  if (x < 0) v = fr_sub(fr_zero(), v);
  store_sol(dst, ld, i, fr_to_mont(v));
}

__global__ void __launch_bounds__(256) export_kernel(const uint32_t* __restrict__ src, uint64_t ld,
                                                     uint64_t n, uint32_t* __restrict__ dst) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const Fr c = fr_from_mont(load_sol(src, ld, i));
#pragma unroll
  for (int j = 0; j < 8; ++j) dst[8 * i + j] = c.w[j];
}

// descriptor upload through kernel arguments: the runtime copies the
// arguments at launch, so the host image can be reused at once and nothing
// waits on the stream (also valid inside a captured graph)
__global__ void __launch_bounds__(256) upload_kernel(UploadArgs a) {
  const uint32_t i = threadIdx.x;
  const uint32_t nw = (a.bytes + 3) / 4;
  uint32_t* d = reinterpret_cast<uint32_t*>(a.dst);
  for (uint32_t k = i; k < nw; k += blockDim.x) d[k] = a.words[k];
}

__global__ void __launch_bounds__(256) zero_kernel(uint32_t* __restrict__ p, uint64_t n) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0;
}

// ---------------------------------------------------------------- launchers -
static inline uint32_t blocks_for(uint64_t n, uint32_t b) { return (uint32_t)((n + b - 1) / b); }

hipError_t launch_eq(const EqJob* jobs, uint32_t n_jobs, uint32_t n_threads, hipStream_t s) {
  if (n_threads == 0) return hipSuccess;
  hipLaunchKernelGGL(eq_kernel, dim3(blocks_for(n_threads, 256)), dim3(256), 0, s, jobs, n_jobs,
                     n_threads);
  return hipGetLastError();
}

hipError_t launch_eq_point(const EqPointArgs& a, hipStream_t s) {
  const uint64_t pairs = a.nvars ? (1ull << a.nvars) / 2 : 1;
  hipLaunchKernelGGL(eq_point_kernel, dim3(blocks_for(pairs, 256)), dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_pack(const uint32_t* eq, uint64_t ld, uint64_t len, uint32_t* pack,
                       hipStream_t s) {
  if (len == 0) return hipSuccess;
  hipLaunchKernelGGL(pack_kernel, dim3(blocks_for(len, 256)), dim3(256), 0, s, eq, ld, len, pack);
  return hipGetLastError();
}

template <typename T, int ND, int DB, bool ROWS, bool VEC, int OPL>
static hipError_t launch_contract_t(const ContractJob* jobs, uint32_t n_jobs, uint32_t n_tasks,
                                    hipStream_t s) {
  hipLaunchKernelGGL((contract_kernel<T, ND, DB, ROWS, VEC, OPL>), dim3(blocks_for(n_tasks, 4)),
                     dim3(kContractBlock), 0, s, jobs, n_jobs, n_tasks);
  return hipGetLastError();
}

hipError_t launch_contract(int kind, const ContractJob* jobs, uint32_t n_jobs, uint32_t n_tasks,
                           hipStream_t s) {
  if (n_tasks == 0) return hipSuccess;
#define VL_CK(K, T, ND, DB, R, V, O) \
  case K: return launch_contract_t<T, ND, DB, R, V, O>(jobs, n_jobs, n_tasks, s);
  switch (kind) {
    VL_CK(CK_I16_ROWS, int16_t, 1, 16, true, false, 1)
    VL_CK(CK_I16_ROWS4, int16_t, 1, 16, true, false, 4)
    VL_CK(CK_I16_ROWS4_VEC, int16_t, 1, 16, true, true, 4)
    VL_CK(CK_I16_COLS, int16_t, 1, 16, false, false, 1)
    VL_CK(CK_I16_COLS_VEC, int16_t, 1, 16, false, true, 1)
    VL_CK(CK_I32_ROWS, int32_t, 2, 24, true, false, 1)
    VL_CK(CK_I32_COLS, int32_t, 2, 24, false, false, 1)
    VL_CK(CK_I32_COLS_VEC, int32_t, 2, 24, false, true, 1)
    VL_CK(CK_I64S_ROWS, int64_t, 2, 24, true, false, 1)
    VL_CK(CK_I64S_COLS, int64_t, 2, 24, false, false, 1)
    VL_CK(CK_I64S_COLS_VEC, int64_t, 2, 24, false, true, 1)
    VL_CK(CK_I64_ROWS, int64_t, 3, 24, true, false, 1)
    VL_CK(CK_I64_COLS, int64_t, 3, 24, false, false, 1)
    VL_CK(CK_I64_COLS_VEC, int64_t, 3, 24, false, true, 1)
    default: return hipErrorInvalidValue;
  }
#undef VL_CK
}

hipError_t launch_finish(const FinishJob* jobs, uint32_t n_jobs, uint32_t n_threads, hipStream_t s) {
  if (n_threads == 0) return hipSuccess;
  hipLaunchKernelGGL(finish_kernel, dim3(blocks_for(n_threads, 256)), dim3(256), 0, s, jobs, n_jobs,
                     n_threads);
  return hipGetLastError();
}

hipError_t launch_rounds(const RoundsJob* jobs, uint32_t n_jobs, hipStream_t s) {
  if (n_jobs == 0) return hipSuccess;
  hipLaunchKernelGGL(rounds_kernel, dim3(n_jobs), dim3(kRoundsBlock), 0, s, jobs);
  return hipGetLastError();
}

hipError_t launch_lift(const void* src, int dtype, uint64_t n, uint32_t* dst, uint64_t ld,
                       hipStream_t s) {
  if (n == 0) return hipSuccess;
  const dim3 g(blocks_for(n, 256)), b(256);
  switch (dtype) {
    case VL_I16: hipLaunchKernelGGL(lift_kernel<int16_t>, g, b, 0, s, (const int16_t*)src, n, dst, ld); break;
    case VL_I32: hipLaunchKernelGGL(lift_kernel<int32_t>, g, b, 0, s, (const int32_t*)src, n, dst, ld); break;
    case VL_I64: hipLaunchKernelGGL(lift_kernel<int64_t>, g, b, 0, s, (const int64_t*)src, n, dst, ld); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_export(const uint32_t* src, uint64_t ld, uint64_t n, uint32_t* dst, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(export_kernel, dim3(blocks_for(n, 256)), dim3(256), 0, s, src, ld, n, dst);
  return hipGetLastError();
}

hipError_t launch_upload(void* dst, const void* src, uint64_t bytes, hipStream_t s) {
  const uint8_t* p = reinterpret_cast<const uint8_t*>(src);
  uint8_t* d = reinterpret_cast<uint8_t*>(dst);
  for (uint64_t o = 0; o < bytes; o += kUploadBytes) {
    UploadArgs a;
    a.dst = d + o;
    a.bytes = (uint32_t)((bytes - o) < kUploadBytes ? (bytes - o) : kUploadBytes);
    memcpy(a.words, p + o, a.bytes);
    hipLaunchKernelGGL(upload_kernel, dim3(1), dim3(256), 0, s, a);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_zero_words(uint32_t* p, uint64_t n, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(zero_kernel, dim3(blocks_for(n, 256)), dim3(256), 0, s, p, n);
  return hipGetLastError();
}

}  // namespace vl
