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
  if (J.pack && t < J.pack_pairs) {
    const Fr p0 = fr_to_mont(e0);   // e * R^2 mod p
    const Fr p1 = fr_to_mont(e1);
    uint32_t* out = J.pack + (uint64_t)t * 32;
#pragma unroll
    for (int k = 0; k < 32; ++k) {
      const uint32_t b0 = (p0.w[k >> 2] >> (8 * (k & 3))) & 0xffu;
      const uint32_t b1 = (p1.w[k >> 2] >> (8 * (k & 3))) & 0xffu;
      out[k] = b0 | (b1 << 16);
    }
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
  const uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (2 * t >= len) return;
  const Fr p0 = fr_to_mont(load_sol(eq, ld, 2 * t));
  const Fr p1 = (2 * t + 1 < len) ? fr_to_mont(load_sol(eq, ld, 2 * t + 1)) : fr_zero();
  uint32_t* out = pack + t * 32;
#pragma unroll
  for (int k = 0; k < 32; ++k) {
    const uint32_t b0 = (p0.w[k >> 2] >> (8 * (k & 3))) & 0xffu;
    const uint32_t b1 = (p1.w[k >> 2] >> (8 * (k & 3))) & 0xffu;
    out[k] = b0 | (b1 << 16);
  }
}

// ---------------------------------------------------------------- contract --
constexpr int q_count(int nd) { return (8 * 31 + 16 * (nd - 1)) / 32 + 1; }

// signed 16-bit digits of a pair of entries, packed per digit as (x0 | x1 << 16)
template <int ND, typename T>
__device__ __forceinline__ void pair_digits(T x0, T x1, uint32_t (&w)[ND], uint32_t& bad) {
  if constexpr (ND == 1) {
    w[0] = (uint32_t)(uint16_t)x0 | ((uint32_t)(uint16_t)x1 << 16);
  } else {
    int64_t r0 = (int64_t)x0, r1 = (int64_t)x1;
#pragma unroll
    for (int t = 0; t < ND; ++t) {
      const uint32_t d0 = (uint32_t)r0 & 0xffffu, d1 = (uint32_t)r1 & 0xffffu;
      w[t] = d0 | (d1 << 16);
      // r <- (r - sext16(d)) / 2^16 without overflow
      r0 = (r0 >> 16) + ((r0 >> 15) & 1);
      r1 = (r1 >> 16) + ((r1 >> 15) & 1);
    }
    bad |= (uint32_t)((r0 | r1) != 0);
  }
}

template <int ND>
__device__ __forceinline__ void dot_pair(cu32_ptr e, const uint32_t (&w)[ND],
                                         int32_t (&acc)[ND][32]) {
#pragma unroll
  for (int k = 0; k < 32; ++k) {
    const uint32_t ev = e[k];
#pragma unroll
    for (int t = 0; t < ND; ++t) acc[t][k] = sdot2(ev, w[t], acc[t][k]);
  }
}

template <int ND, int QC>
__device__ __forceinline__ void flush(int32_t (&acc)[ND][32], int64_t (&T)[QC]) {
#pragma unroll
  for (int t = 0; t < ND; ++t) {
#pragma unroll
    for (int k = 0; k < 32; ++k) {
      const int bit = 8 * k + 16 * t;
      T[bit >> 5] += (int64_t)((uint64_t)(int64_t)acc[t][k] << (bit & 31));
      acc[t][k] = 0;
    }
  }
  // keep all but the top limb sum in [0, 2^32)
#pragma unroll
  for (int q = 0; q + 1 < QC; ++q) {
    const int64_t c = T[q] >> 32;
    T[q] -= (int64_t)((uint64_t)c << 32);
    T[q + 1] += c;
  }
}

// The signed sum V = sum_q T[q] 2^(32q) (two's complement over 12 limbs) is
// congruent to R^2 * value, so V * R^-1 mod p is the Montgomery form of the
// value.  With V = lo + 2^256 * hi (lo unsigned 256-bit, |hi| < 2^80):
//     V * R^-1 = lo * R^-1 + hi  (mod p),
// one Montgomery multiplication of lo by 1 plus a small signed lift.  (A
// direct 12-limb REDC was miscompiled for gfx950 at -O3 -- one carry was
// lost -- so the reduction goes through the field multiplier instead.)
template <int QC>
__device__ __forceinline__ Fr finalize(const int64_t (&T)[QC]) {
  uint32_t L[12];
  int64_t carry = 0;
#pragma unroll
  for (int q = 0; q < 12; ++q) {
    const int64_t v = (q < QC ? T[q] : 0) + carry;
    L[q] = (uint32_t)v;
    carry = v >> 32;
  }
  Fr lo;
#pragma unroll
  for (int j = 0; j < 8; ++j) lo.w[j] = L[j];
  lo = fr_reduce_once(fr_reduce_once(lo));   // 2^256 < 3p
  const Fr part = fr_mul(lo, fr_one_raw());
  // the signed top part as a field element (|hi| < 2^80)
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

template <typename T, int ND, bool ROWS, bool VEC>
__global__ void __launch_bounds__(kContractBlock)
contract_kernel(const ContractJob* __restrict__ jobs, uint32_t n_jobs, uint32_t n_tasks) {
  constexpr int QC = q_count(ND);
  const uint32_t task = __builtin_amdgcn_readfirstlane(blockIdx.x * 4 + (threadIdx.x >> 6));
  if (task >= n_tasks) return;
  uint32_t lo = 0, hi = n_jobs;
  while (hi - lo > 1) {
    const uint32_t mid = (lo + hi) >> 1;
    if (jobs[mid].task_begin <= task) lo = mid; else hi = mid;
  }
  const ContractJob& J = jobs[lo];
  const uint32_t local = task - J.task_begin;
  const uint32_t chunk = local % J.n_chunks;
  const uint32_t owave = local / J.n_chunks;
  const uint32_t lane = threadIdx.x & 63u;
  const uint32_t n = owave * 64u + lane;
  const bool valid = n < J.n_out;
  const uint32_t m0 = chunk * J.chunk;
  const uint32_t m1 = min(m0 + J.chunk, J.len);
  const T* __restrict__ M = (const T*)J.M;
  const uint64_t ld = J.ld;
  cu32_ptr pack = (cu32_ptr)J.pack;

  int32_t acc[ND][32];
#pragma unroll
  for (int t = 0; t < ND; ++t)
#pragma unroll
    for (int k = 0; k < 32; ++k) acc[t][k] = 0;
  int64_t Tq[QC];
#pragma unroll
  for (int q = 0; q < QC; ++q) Tq[q] = 0;
  uint32_t bad = 0;

  auto elem = [&](uint32_t m) -> T {
    return ROWS ? M[(uint64_t)m * ld + n] : M[(uint64_t)n * ld + m];
  };

  uint32_t m = m0;
  if constexpr (VEC) {
    // cols layout, 16-byte aligned rows: 64 bytes of the lane's row per step
    constexpr uint32_t BE = 64 / sizeof(T);
    const T* row = M + (uint64_t)(valid ? n : 0u) * ld;
    const uint32_t mv = m0 + ((m1 - m0) / BE) * BE;
    while (m < mv) {
      const uint32_t bend = min(m + 2 * kFlushPairs, mv);
      for (; m < bend; m += BE) {
        uint4 buf[4];
        if (valid) {
          const uint4* src = (const uint4*)(row + m);
#pragma unroll
          for (int i = 0; i < 4; ++i) buf[i] = src[i];
        } else {
#pragma unroll
          for (int i = 0; i < 4; ++i) buf[i] = make_uint4(0, 0, 0, 0);
        }
        const T* x = (const T*)buf;
#pragma unroll
        for (uint32_t q = 0; q < BE / 2; ++q) {
          uint32_t w[ND];
          pair_digits<ND, T>(x[2 * q], x[2 * q + 1], w, bad);
          dot_pair<ND>(pack + ((m >> 1) + q) * 32, w, acc);
        }
      }
      flush<ND, QC>(acc, Tq);
    }
  }
  {
    const uint32_t m1e = m + ((m1 - m) & ~1u);
    while (m < m1e) {
      const uint32_t bend = min(m + 2 * kFlushPairs, m1e);
#pragma unroll 2
      for (; m < bend; m += 2) {
        T x0 = 0, x1 = 0;
        if (valid) {
          x0 = elem(m);
          x1 = elem(m + 1);
        }
        uint32_t w[ND];
        pair_digits<ND, T>(x0, x1, w, bad);
        dot_pair<ND>(pack + (m >> 1) * 32, w, acc);
      }
      flush<ND, QC>(acc, Tq);
    }
    if (m < m1) {  // odd contraction length: last entry pairs with zero
      T x0 = valid ? elem(m) : (T)0;
      uint32_t w[ND];
      pair_digits<ND, T>(x0, (T)0, w, bad);
      dot_pair<ND>(pack + (m >> 1) * 32, w, acc);
      flush<ND, QC>(acc, Tq);
    }
  }
  if (ND > 1 && valid && bad && J.err) atomicOr(J.err, 1);
  const Fr r = finalize<QC>(Tq);
  if (valid) store_sol(J.dst + (uint64_t)chunk * J.chunk_stride, J.dst_ld, n, r);
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

__global__ void __launch_bounds__(kRoundsBlock) rounds_kernel(const RoundsJob* __restrict__ jobs) {
  const RoundsJob& J = jobs[blockIdx.x];
  __shared__ uint32_t red[3 * 8 * (kRoundsBlock / kWave)];
  __shared__ uint32_t bcast[8];
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
  // s_p = sum_w a_p[w] b_p[w]; the products must sum to c
  Fr s[VL_MAX_PRODS];
  Fr total = fr_zero();
  for (uint32_t p = 0; p < J.n_prods; ++p) {
    const RoundsProd& P = J.prods[p];
    v1[0] = fr_zero();
    const uint32_t len1 = 1u << P.n1;
    for (uint32_t k = tid; k < len1; k += NT)
      v1[0] = fr_add(v1[0], fr_mul(load_sol(P.a, P.ld, k), load_sol(P.b, P.ld, k)));
    block_sum<1>(v1, red);
    s[p] = v1[0];
    total = fr_add(total, s[p]);
  }
  if (!fr_eq(total, c)) {
    if (tid == 0) *J.status = VL_ERR_FALSE_STATEMENT;
    return;
  }

  Transcript tr;
  uint8_t* out = J.proof;
  if (tid == 0) {
#pragma unroll
    for (int i = 0; i < 32; ++i) tr.st[i] = J.st[i];
    const Fr cc[1] = {fr_from_mont(c)};
    put_fr(out, c);
    out += 32;
    tr_absorb_frs(tr, VL_LBL_CLAIM, cc);
    for (uint32_t p = 0; p + 1 < J.n_prods; ++p) {
      const Fr sc[1] = {fr_from_mont(s[p])};
      put_fr(out, s[p]);
      out += 32;
      tr_absorb_frs(tr, VL_LBL_PART, sc);
    }
  }
  for (uint32_t p = 0; p < J.n_prods; ++p) {
    const RoundsProd& P = J.prods[p];
    uint32_t* a = P.a;
    uint32_t* b = P.b;
    const uint64_t ld = P.ld;
    for (uint32_t rd = 0; rd < P.n1; ++rd) {
      const uint32_t h = 1u << (P.n1 - 1 - rd);
      Fr g[3];
      g[0] = g[1] = g[2] = fr_zero();
      for (uint32_t t = tid; t < h; t += NT) {
        const Fr a0 = load_sol(a, ld, t), a1 = load_sol(a, ld, t + h);
        const Fr b0 = load_sol(b, ld, t), b1 = load_sol(b, ld, t + h);
        g[0] = fr_add(g[0], fr_mul(a0, b0));
        g[1] = fr_add(g[1], fr_mul(a1, b1));
        const Fr da = fr_sub(fr_double(a1), a0), db = fr_sub(fr_double(b1), b0);
        g[2] = fr_add(g[2], fr_mul(da, db));
      }
      block_sum<3>(g, red);
      if (tid == 0) {
        Fr gc[3];
        for (int k = 0; k < 3; ++k) {
          gc[k] = fr_from_mont(g[k]);
          put_fr(out, g[k]);
          out += 32;
        }
        tr_absorb_frs(tr, VL_LBL_ROUND, gc);
        const Fr r = fr_to_mont(tr_squeeze_fixed(tr, VL_LBL_R));
        for (int j = 0; j < 8; ++j) bcast[j] = r.w[j];
      }
      __syncthreads();
      Fr r;
#pragma unroll
      for (int j = 0; j < 8; ++j) r.w[j] = bcast[j];
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
    if (J.digest)
      for (int i = 0; i < 32; ++i) J.digest[i] = tr.st[i];
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
  const uint64_t pairs = (len + 1) / 2;
  if (pairs == 0) return hipSuccess;
  hipLaunchKernelGGL(pack_kernel, dim3(blocks_for(pairs, 256)), dim3(256), 0, s, eq, ld, len, pack);
  return hipGetLastError();
}

template <typename T, int ND, bool ROWS, bool VEC>
static hipError_t launch_contract_t(const ContractJob* jobs, uint32_t n_jobs, uint32_t n_tasks,
                                    hipStream_t s) {
  hipLaunchKernelGGL((contract_kernel<T, ND, ROWS, VEC>), dim3(blocks_for(n_tasks, 4)),
                     dim3(kContractBlock), 0, s, jobs, n_jobs, n_tasks);
  return hipGetLastError();
}

hipError_t launch_contract(int kind, const ContractJob* jobs, uint32_t n_jobs, uint32_t n_tasks,
                           hipStream_t s) {
  if (n_tasks == 0) return hipSuccess;
  switch (kind) {
    case CK_I16_ROWS: return launch_contract_t<int16_t, 1, true, false>(jobs, n_jobs, n_tasks, s);
    case CK_I16_COLS: return launch_contract_t<int16_t, 1, false, false>(jobs, n_jobs, n_tasks, s);
    case CK_I16_COLS_VEC: return launch_contract_t<int16_t, 1, false, true>(jobs, n_jobs, n_tasks, s);
    case CK_I32_ROWS: return launch_contract_t<int32_t, 3, true, false>(jobs, n_jobs, n_tasks, s);
    case CK_I32_COLS: return launch_contract_t<int32_t, 3, false, false>(jobs, n_jobs, n_tasks, s);
    case CK_I32_COLS_VEC: return launch_contract_t<int32_t, 3, false, true>(jobs, n_jobs, n_tasks, s);
    case CK_I64N3_ROWS: return launch_contract_t<int64_t, 3, true, false>(jobs, n_jobs, n_tasks, s);
    case CK_I64N3_COLS: return launch_contract_t<int64_t, 3, false, false>(jobs, n_jobs, n_tasks, s);
    case CK_I64N3_COLS_VEC:
      return launch_contract_t<int64_t, 3, false, true>(jobs, n_jobs, n_tasks, s);
    case CK_I64N4_ROWS: return launch_contract_t<int64_t, 4, true, false>(jobs, n_jobs, n_tasks, s);
    case CK_I64N4_COLS: return launch_contract_t<int64_t, 4, false, false>(jobs, n_jobs, n_tasks, s);
    case CK_I64N4_COLS_VEC:
      return launch_contract_t<int64_t, 4, false, true>(jobs, n_jobs, n_tasks, s);
    default: return hipErrorInvalidValue;
  }
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
