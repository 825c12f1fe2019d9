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
// Each eq entry e is stored as e * R^2 mod p (so that one Montgomery
// reduction at the end lands in Montgomery form) cut into 8 signed 32-bit
// digits e_j; each matrix entry x is one signed 16-bit digit (int16) or two or
// three signed 24-bit digits d_t (wider types).  The exact integer
//     sum_m e[m] * x[m] = sum_{j,t} 2^(32 j + DB t) * sum_m e_j[m] * d_t[m]
// is accumulated with v_mad_i64_i32 into 64-bit accumulators, one
// instruction per (j, t) and entry: the eq digits are wave-uniform and come
// from scalar registers, the matrix digits from vector registers.  The
// signed ~300-bit sum is reduced with one Montgomery multiplication
// (limbs_to_fr) once per output: a contraction split into chunks stores each
// chunk's sum as raw limbs, which finish_kernel adds up before reducing.
#include <cstring>
#include <type_traits>

#include "internal.hpp"
#include "sha256.hpp"

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
    // factor j is x_j for bit 1 and 1 - x_j for bit 0 (point: x_j only)
    Fr base = fr_R();
    for (uint32_t j = 0; j + 1 < n; ++j) {
      const uint32_t bit = (t >> (n - 2 - j)) & 1u;
      Fr x;
#pragma unroll
      for (int k = 0; k < 8; ++k) x.w[k] = J.point[j * 8 + k];
      base = fr_mul(base, bit ? x : fr_sub(fr_R(), x));
    }
    Fr xl;
#pragma unroll
    for (int k = 0; k < 8; ++k) xl.w[k] = J.point[(n - 1) * 8 + k];
    e0 = fr_mul(base, fr_sub(fr_R(), xl));
    e1 = fr_mul(base, xl);
  }
  if (J.eq) {
    if (2ull * t < len) store_sol(J.eq, J.eq_ld, 2ull * t, J.eq_canon ? fr_from_mont(e0) : e0);
    if (2ull * t + 1 < len) store_sol(J.eq, J.eq_ld, 2ull * t + 1, J.eq_canon ? fr_from_mont(e1) : e1);
  }
  if (J.pack) {
    // pack: e * R^2 (or e * R) mod p as signed digits, 8 words per entry
    if (2 * t < J.pack_len) signed_digits(J.pack_r2 ? fr_to_mont(e0) : e0, J.pack + (uint64_t)(2 * t) * 8);
    if (2 * t + 1 < J.pack_len) signed_digits(J.pack_r2 ? fr_to_mont(e1) : e1, J.pack + (uint64_t)(2 * t + 1) * 8);
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
  } else if constexpr (ND == 2 && DB == 24) {
    // x = d0 + 2^24 d1: d0 the sign-extended low 24 bits, d1 = floor(x / 2^24)
    // plus bit 23 (the borrow of a negative d0).  For int64 the entry must
    // satisfy -2^47 <= x < 2^47, so d1 fits 32 bits (|d1| <= 2^23 keeps the
    // int64 accumulators safe between spills); otherwise it is flagged.
    const uint32_t lo = (uint32_t)(uint64_t)(int64_t)x;
    const uint32_t hw = sizeof(T) == 8 ? (uint32_t)((uint64_t)(int64_t)x >> 32) : (uint32_t)((int32_t)lo >> 31);
    d[0] = __builtin_amdgcn_sbfe((int32_t)lo, 0, 24);
    const uint32_t top = sizeof(T) == 8 ? __builtin_amdgcn_alignbit(hw, lo, 24) : (uint32_t)((int32_t)lo >> 24);
    d[1] = (int32_t)(top + __builtin_amdgcn_ubfe(lo, 23, 1));
    if constexpr (sizeof(T) == 8) bad |= (hw + 0x8000u) >> 16;
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

// the same with the eq digits already in registers
template <int OPL, int ND>
__device__ __forceinline__ void mac8v(const int32_t (&e)[8], const int32_t (&d)[OPL][ND],
                                      int64_t (&acc)[OPL][ND][8]) {
#pragma unroll
  for (int j = 0; j < 8; ++j)
#pragma unroll
    for (int o = 0; o < OPL; ++o)
#pragma unroll
      for (int t = 0; t < ND; ++t) acc[o][t][j] += (int64_t)e[j] * (int64_t)d[o][t];
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
// (the eq digits hold e * R^2 mod p), as kLimbs 32-bit two's-complement
// limbs (|V| < 2^340 for every entry type and length).
template <int ND, int DB>
__device__ __forceinline__ void digits_to_limbs(const int64_t (&acc)[ND][8], const int64_t (&hi)[ND][8],
                                                uint32_t (&L)[kLimbs]) {
  int64_t S[kLimbs];
#pragma unroll
  for (int q = 0; q < kLimbs; ++q) S[q] = 0;
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
  int64_t carry = 0;
#pragma unroll
  for (int q = 0; q < kLimbs; ++q) {
    const int64_t v = S[q] + carry;
    L[q] = (uint32_t)v;
    carry = v >> 32;
  }
}

// V * R^-1 mod p in Montgomery form for V given as limbs.  With V = lo +
// 2^256 hi (lo unsigned 256-bit, |hi| < 2^127): V * R^-1 = lo * R^-1 + hi
// (mod p), i.e. one Montgomery multiplication by 1 plus a small signed lift.
// (A direct 12-limb REDC written with 64-bit adds lost a carry when compiled
// for gfx950 at -O3, so the reduction goes through the field multiplier.)
__device__ __forceinline__ Fr limbs_to_fr(const uint32_t (&L)[kLimbs]) {
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
  constexpr uint32_t kSpill = kWideSpill;
  const uint32_t task = __builtin_amdgcn_readfirstlane(blockIdx.x * 4 + (threadIdx.x >> 6));
  if (task >= n_tasks) return;
  uint32_t lo = 0, hi_i = n_jobs;
  while (hi_i - lo > 1) {
    const uint32_t mid = (lo + hi_i) >> 1;
    if (jobs[mid].task_begin <= task) lo = mid; else hi_i = mid;
  }
  const ContractJob& J = jobs[lo];
  const uint32_t local = task - J.task_begin;
  // output groups vary fastest: the waves of a block (one CU) work on the
  // same chunk, so they share its eq digits in the scalar cache (and the
  // row kernels read adjacent segments of the same rows)
  const uint32_t owave = local % J.out_waves;
  const uint32_t chunk = local / J.out_waves;
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

  // All matrix reads go through global (not generic) pointers: generic loads
  // also count against the scalar-load counter, so every wait for the eq
  // digits would drain the vector loads in flight as well.
  const gptr<T> Mg = (gptr<T>)M;
  if constexpr (VEC && !ROWS) {
    // cols layout, 16-byte aligned rows (m0 is a multiple of the vector
    // width): OPL rows per lane.  Each lane reads its row 128 bytes at a
    // time (GV 16-byte loads issued together, so every cache line is fetched
    // once instead of being re-read after eviction), the next group in
    // flight while this one is used.  Lanes past the last row re-read the
    // last row (their results are not stored); load indices are clamped to
    // the chunk, and the aligned 16-byte block holding a row's last entry
    // never crosses a page, so every load stays inside the matrix's pages.
    constexpr uint32_t BE = 16 / sizeof(T);
    constexpr uint32_t GV = 8;
    const uint32_t span = m1 - m0, full = span / BE, nvec = (span + BE - 1) / BE;
    gptr<u32x4> rowp[OPL];
#pragma unroll
    for (int o = 0; o < OPL; ++o)
      rowp[o] = (gptr<u32x4>)(Mg + (uint64_t)min(n0 + o, n_out - 1) * ld + m0);
    auto ldg = [&](uint32_t g, u32x4 (&b)[GV][OPL]) {
#pragma unroll
      for (uint32_t v = 0; v < GV; ++v)
#pragma unroll
        for (int o = 0; o < OPL; ++o) b[v][o] = rowp[o][min(g * GV + v, nvec - 1)];
    };
    // one 16-byte vector: its eq digits in one batch of scalar loads (one
    // wait), then the multiply-adds
    auto vec16 = [&](const u32x4 (&x)[OPL], uint32_t v) {
      ci32_ptr pe = pack + (uint64_t)(m0 + v * BE) * 8;
      int32_t e[BE][8];
#pragma unroll
      for (uint32_t q = 0; q < BE; ++q)
#pragma unroll
        for (int j = 0; j < 8; ++j) e[q][j] = pe[q * 8 + j];
#pragma unroll
      for (uint32_t q = 0; q < BE; ++q) {
        int32_t d[OPL][ND];
#pragma unroll
        for (int o = 0; o < OPL; ++o) entry_digits<T, ND, DB>(((const T*)&x[o])[q], d[o], bad);
        mac8v<OPL, ND>(e[q], d, acc);
      }
    };
    // complete groups; wide entries spill their high words every kSpill
    // entries (GB groups)
    constexpr uint32_t GB = WIDE ? kSpill / (BE * GV) : 1;
    const uint32_t ng = full / GV;
    u32x4 cur[GV][OPL];
    ldg(0, cur);
    for (uint32_t gb = 0; gb < ng; gb += (WIDE ? GB : ng)) {
      const uint32_t ge = WIDE ? min(gb + GB, ng) : ng;
      for (uint32_t g = gb; g < ge; ++g) {
        u32x4 nxt[GV][OPL];
        ldg(g + 1, nxt);
#pragma unroll
        for (uint32_t v = 0; v < GV; ++v) vec16(cur[v], g * GV + v);
#pragma unroll
        for (uint32_t v = 0; v < GV; ++v)
#pragma unroll
          for (int o = 0; o < OPL; ++o) cur[v][o] = nxt[v][o];
      }
      if constexpr (WIDE) spill_high<OPL, ND>(acc, hi);
    }
    // the full vectors of the last, incomplete group (already loaded)
#pragma unroll
    for (uint32_t v = 0; v < GV; ++v)
      if (ng * GV + v < full) vec16(cur[v], ng * GV + v);
    if (full < nvec) {   // last, partial vector of the row
      u32x4 t[OPL];
#pragma unroll
      for (int o = 0; o < OPL; ++o) t[o] = rowp[o][full];
      const uint32_t rem = span - full * BE;
#pragma unroll
      for (uint32_t q = 0; q < BE; ++q) {
        if (q < rem) {
          int32_t d[OPL][ND];
#pragma unroll
          for (int o = 0; o < OPL; ++o) entry_digits<T, ND, DB>(((const T*)&t[o])[q], d[o], bad);
          mac8<OPL, ND>(pack + (uint64_t)(m0 + full * BE + q) * 8, d, acc);
        }
      }
    }
  } else if constexpr (VEC && ROWS) {
    // rows layout: OPL adjacent columns per lane read as one vector per row
    // (4 int16 = 8 bytes; 4 int32 or 2 int64 = 16 bytes), so a wave reads 512
    // or 1024 contiguous bytes of each row; a ring of PF rows in flight.
    // Lanes past the last column group re-read the last group, whose columns
    // past n_out (inside the aligned vector that holds column n_out - 1, so
    // inside the matrix's pages) are read but neither stored nor range
    // checked.  Wide entries: the chunk holds at most kWideSpill rows (the
    // planner caps it), so the accumulators need no high-word spill.
    constexpr uint32_t VB = OPL * sizeof(T);
    static_assert(VB == 8 || VB == 16, "vector rows kernel: 8- or 16-byte column groups");
    static_assert(WIDE == (sizeof(T) > 2), "int16 entries are single 16-bit digits");
    typedef typename std::conditional<VB == 8, u32x2, u32x4>::type LT;
    constexpr uint32_t PF = 8;
    static_assert((PF & (PF - 1)) == 0, "the ring length is a power of two");
    const uint32_t nc = min(n0, ((n_out - 1) / OPL) * OPL);
    const gptr<T> base = Mg + (uint64_t)m0 * ld + nc;
    const uint32_t rows = m1 - m0;
    auto row = [&](uint32_t r) -> LT { return *(gptr<LT>)(base + (uint64_t)min(r, rows - 1) * ld); };
    uint32_t bad_o[OPL];
#pragma unroll
    for (int o = 0; o < OPL; ++o) bad_o[o] = 0;
    auto digits = [&](const LT& x, int32_t (&d)[OPL][ND]) {
#pragma unroll
      for (int o = 0; o < OPL; ++o) entry_digits<T, ND, DB>(((const T*)&x)[o], d[o], bad_o[o]);
    };
    LT buf[PF];
#pragma unroll
    for (uint32_t s = 0; s < PF; ++s) buf[s] = row(s);
    const uint32_t fullr = rows & ~(PF - 1);
    for (uint32_t r = 0; r < fullr; r += PF) {
      // eq digits of the PF rows in one batch of scalar loads, one wait
      ci32_ptr pe = pack + (uint64_t)(m0 + r) * 8;
      int32_t e[PF][8];
#pragma unroll
      for (uint32_t s = 0; s < PF; ++s)
#pragma unroll
        for (int j = 0; j < 8; ++j) e[s][j] = pe[s * 8 + j];
#pragma unroll
      for (uint32_t s = 0; s < PF; ++s) {
        int32_t d[OPL][ND];
        digits(buf[s], d);
        mac8v<OPL, ND>(e[s], d, acc);
        buf[s] = row(r + s + PF);
      }
    }
#pragma unroll
    for (uint32_t s = 0; s < PF; ++s) {   // last rows (fewer than PF)
      if (fullr + s < rows) {
        int32_t d[OPL][ND];
        digits(buf[s], d);
        mac8<OPL, ND>(pack + (uint64_t)(m0 + fullr + s) * 8, d, acc);
      }
    }
#pragma unroll
    for (int o = 0; o < OPL; ++o)
      if (n0 + o < n_out) bad |= bad_o[o];
  } else {
    // element loads (unaligned or narrow matrices): UB entries per output
    // and their eq digits loaded together, then used (left to itself the
    // scheduler waits for each load in turn).  Outputs past n_out read the
    // last output's entries (in bounds) and use zero.
    constexpr uint32_t UB = 8;
    uint64_t eoff[OPL];
    bool valid[OPL];
#pragma unroll
    for (int o = 0; o < OPL; ++o) {
      const uint32_t n = min(n0 + o, n_out - 1);
      valid[o] = n0 + o < n_out;
      eoff[o] = ROWS ? n : (uint64_t)n * ld;
    }
    const uint64_t mstep = ROWS ? ld : 1;
    auto elem = [&](uint32_t m, int o) -> T {
      const T x = Mg[eoff[o] + (uint64_t)m * mstep];
      return valid[o] ? x : T(0);
    };
    uint32_t m = m0;
    while (m < m1) {
      const uint32_t bend = WIDE ? min(m + kSpill, m1) : m1;
      for (; m + UB <= bend; m += UB) {
        ci32_ptr pe = pack + (uint64_t)m * 8;
        int32_t e[UB][8];
#pragma unroll
        for (uint32_t u = 0; u < UB; ++u)
#pragma unroll
          for (int j = 0; j < 8; ++j) e[u][j] = pe[u * 8 + j];
        T x[UB][OPL];
#pragma unroll
        for (uint32_t u = 0; u < UB; ++u)
#pragma unroll
          for (int o = 0; o < OPL; ++o) x[u][o] = elem(m + u, o);
#pragma unroll
        for (uint32_t u = 0; u < UB; ++u) {
          int32_t d[OPL][ND];
#pragma unroll
          for (int o = 0; o < OPL; ++o) entry_digits<T, ND, DB>(x[u][o], d[o], bad);
          mac8v<OPL, ND>(e[u], d, acc);
        }
      }
      for (; m < bend; ++m) {
        int32_t d[OPL][ND];
#pragma unroll
        for (int o = 0; o < OPL; ++o) entry_digits<T, ND, DB>(elem(m, o), d[o], bad);
        mac8<OPL, ND>(pack + (uint64_t)m * 8, d, acc);
      }
      if constexpr (WIDE) spill_high<OPL, ND>(acc, hi);
    }
  }
  if constexpr (ND > 1 || sizeof(T) > 2) {
    if (bad && J.err) atomicOr(J.err, 1);
  }
#pragma unroll
  for (int o = 0; o < OPL; ++o) {
    uint32_t L[kLimbs];
    digits_to_limbs<ND, DB>(acc[o], hi[o], L);
    const uint32_t n = n0 + o;
    if (J.n_chunks == 1) {              // the whole contraction: final value
      const Fr r = limbs_to_fr(L);
      if (n < n_out) store_sol(J.dst, J.dst_ld, n, r);
    } else if (n < n_out) {             // one chunk: raw limbs, reduced by finish_kernel
      uint32_t* d = J.dst + partial_word(n, chunk, 0, J.n_chunks);
#pragma unroll
      for (int q = 0; q < kLimbs; ++q) d[q * 64] = L[q];
    }
  }
}

// ---------------------------------------------------------------- finish ----
// Sums each output's raw chunk limbs (64-bit sums per limb, exact),
// propagates the carries and reduces once.  Jobs with few chunks take one
// thread per output (256 per block); jobs with many chunks take 64 outputs
// per block, the four waves adding up every fourth chunk and wave 0
// combining them.  Outputs past n_valid up to n_total are the zero padding
// of the table.
__device__ __forceinline__ void finish_store(const FinishJob& J, uint32_t i, const int64_t (&T)[kLimbs]) {
  // each T[q] < n_chunks * 2^32 in magnitude: carries fit in 64 bits
  uint32_t L[kLimbs];
  int64_t carry = 0;
#pragma unroll
  for (int q = 0; q < kLimbs; ++q) {
    const int64_t v = T[q] + carry;
    L[q] = (uint32_t)v;
    carry = v >> 32;
  }
  store_sol(J.out, J.out_ld, i, limbs_to_fr(L));
}

// chunks [c0, c1) step dc of an output's limbs (p: chunk 0, limb 0 in the
// tiled layout), FC chunks' loads issued together before they are added
// (left to itself the scheduler waits for each load in turn)
template <int FC>
__device__ __forceinline__ void finish_add(int64_t (&T)[kLimbs], gptr<uint32_t> p, uint32_t c0, uint32_t c1,
                                           uint32_t dc) {
  uint32_t c = c0;
  for (; c + (FC - 1) * dc < c1; c += FC * dc) {
    uint32_t v[FC][kLimbs];
#pragma unroll
    for (int k = 0; k < FC; ++k)
#pragma unroll
      for (int q = 0; q < kLimbs; ++q) v[k][q] = __builtin_nontemporal_load(&p[(uint64_t)(c + k * dc) * (kLimbs * 64) + q * 64]);
#pragma unroll
    for (int k = 0; k < FC; ++k) {
#pragma unroll
      for (int q = 0; q < kLimbs - 1; ++q) T[q] += (int64_t)v[k][q];
      T[kLimbs - 1] += (int64_t)(int32_t)v[k][kLimbs - 1];
    }
  }
  for (; c < c1; c += dc) {
    uint32_t v[kLimbs];
#pragma unroll
    for (int q = 0; q < kLimbs; ++q) v[q] = __builtin_nontemporal_load(&p[(uint64_t)c * (kLimbs * 64) + q * 64]);
#pragma unroll
    for (int q = 0; q < kLimbs - 1; ++q) T[q] += (int64_t)v[q];
    T[kLimbs - 1] += (int64_t)(int32_t)v[kLimbs - 1];
  }
}

__global__ void __launch_bounds__(256) finish_kernel(const FinishJob* __restrict__ jobs,
                                                     uint32_t n_jobs, uint32_t n_blocks) {
  const uint32_t blk = blockIdx.x;
  if (blk >= n_blocks) return;
  uint32_t lo = 0, hi = n_jobs;
  while (hi - lo > 1) {
    const uint32_t mid = (lo + hi) >> 1;
    if (jobs[mid].block_begin <= blk) lo = mid; else hi = mid;
  }
  const FinishJob& J = jobs[lo];
  int64_t T[kLimbs];
#pragma unroll
  for (int q = 0; q < kLimbs; ++q) T[q] = 0;
  if (!J.split) {   // uniform over the block
    const uint32_t i = (blk - J.block_begin) * 256u + threadIdx.x;
    if (i >= J.n_total) return;
    if (i >= J.n_valid) {
      store_sol(J.out, J.out_ld, i, fr_zero());
      return;
    }
    if (!J.part) return;
    finish_add<4>(T, (gptr<uint32_t>)J.part + partial_word(i, 0, 0, J.n_chunks), 0, J.n_chunks, 1);
    finish_store(J, i, T);
    return;
  }
  const uint32_t wave = threadIdx.x >> 6, lane = threadIdx.x & 63u;
  const uint32_t i = (blk - J.block_begin) * 64u + lane;
  __shared__ int64_t red[3][kLimbs][64];
  if (i < J.n_valid) {
    finish_add<4>(T, (gptr<uint32_t>)J.part + partial_word(i, 0, 0, J.n_chunks), wave, J.n_chunks, 4);
  }
  if (wave > 0)
#pragma unroll
    for (int q = 0; q < kLimbs; ++q) red[wave - 1][q][lane] = T[q];
  __syncthreads();
  if (wave != 0 || i >= J.n_total) return;
  if (i >= J.n_valid) {
    store_sol(J.out, J.out_ld, i, fr_zero());
    return;
  }
#pragma unroll
  for (int w = 0; w < 3; ++w)
#pragma unroll
    for (int q = 0; q < kLimbs; ++q) T[q] += red[w][q][lane];
  finish_store(J, i, T);
}

// ---------------------------------------------------------------- rounds ----
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

// One sumcheck round's messages and challenge, run by wave 0 (all its
// lanes, g canonical and valid in lane 0): lane k < 3 writes g(k) to the
// proof; lane 0 absorbs the three values and squeezes r.  Returns r in
// Montgomery form in every lane of wave 0.
__device__ __forceinline__ Fr round_challenge(Transcript& tr, const Fr (&g)[3], uint8_t* out, uint32_t lane) {
  Fr gc[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) gc[k] = readlane_fr(g[k], 0);
  const Fr mine = lane == 0 ? gc[0] : (lane == 1 ? gc[1] : gc[2]);
  if (lane < 3) put_canon(out + 32 * lane, mine);
  Fr r = fr_zero();
  if (lane == 0) {
    tr_absorb_frs(tr, VL_LBL_ROUND, gc);
    r = fr_to_mont(tr_squeeze_fixed(tr, VL_LBL_R));
  }
  return readlane_fr(r, 0);
}

// Pass 1: the claim's dot product and round 1 of every product as partial
// sums, kPass1Pairs pairs per 256-thread block, spread over the whole GPU
// (the rounds kernel of a group runs on one CU and only adds the partials).
__global__ void __launch_bounds__(256) pass1_kernel(const Pass1Job* __restrict__ jobs, uint32_t n_jobs,
                                                    uint32_t n_blocks) {
  const uint32_t blk = blockIdx.x;
  if (blk >= n_blocks) return;
  uint32_t lo = 0, hi = n_jobs;
  while (hi - lo > 1) {
    const uint32_t mid = (lo + hi) >> 1;
    if (jobs[mid].block_begin <= blk) lo = mid; else hi = mid;
  }
  const Pass1Job& J = jobs[lo];
  const uint32_t base = (blk - J.block_begin) * kPass1Pairs;
  const uint32_t end = min(base + kPass1Pairs, J.h);
  Fr g[3];
  g[0] = g[1] = g[2] = fr_zero();
  for (uint32_t t = base + threadIdx.x; t < end; t += 256) {
    if (J.dot) {
      g[0] = fr_add(g[0], fr_mul(load_sol(J.a, J.a_ld, t), load_sol(J.b, J.b_ld, t)));
    } else {
      const Fr a0 = load_sol(J.a, J.a_ld, t), a1 = load_sol(J.a, J.a_ld, t + J.h);
      const Fr b0 = load_sol(J.b, J.b_ld, t), b1 = load_sol(J.b, J.b_ld, t + J.h);
      g[0] = fr_add(g[0], fr_mul(a0, b0));
      g[1] = fr_add(g[1], fr_mul(a1, b1));
      g[2] = fr_add(g[2], fr_mul(at_two(a0, a1), at_two(b0, b1)));
    }
  }
  __shared__ uint32_t red[3 * 8 * 4];
  wave_sum<3>(g, kWave);
  const uint32_t wave = threadIdx.x >> 6, lane = threadIdx.x & 63u;
  if (lane == 0)
#pragma unroll
    for (int k = 0; k < 3; ++k)
#pragma unroll
      for (int j = 0; j < 8; ++j) red[(k * 8 + j) * 4 + wave] = g[k].w[j];
  __syncthreads();
  if (wave == 0) {
#pragma unroll
    for (int k = 0; k < 3; ++k)
#pragma unroll
      for (int j = 0; j < 8; ++j) g[k].w[j] = lane < 4 ? red[(k * 8 + j) * 4 + lane] : 0u;
    wave_sum<3>(g, 4);
    if (lane == 0) {
      uint32_t* o = J.out + (uint64_t)(blk - J.block_begin) * 24;
#pragma unroll
      for (int k = 0; k < 3; ++k)
#pragma unroll
        for (int j = 0; j < 8; ++j) o[k * 8 + j] = g[k].w[j];
      // persistent mode: count this block for the group's resident rounds
      // workgroup (release: the partials, and everything the earlier
      // kernels of the stream wrote, are visible to whoever sees the count)
      if (J.ready) __hip_atomic_fetch_add(J.ready, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    }
  }
}

// One workgroup per group.  Round 1 of every product comes from the pass-1
// partials (its g(0) + g(1) is the product's sum, so the prover guard needs
// no extra pass).  Every later round computes g(0), g(1) and g(2) from the
// folded tables (g(0) + g(1) equals the previous round's g(r) by the folding
// identity, for any tables).  The a~ tables are in Montgomery form and the
// b~ tables in canonical form, so every product a * b, and with it every
// round value, is canonical; folding by r in Montgomery form keeps both
// forms.  While the half-table is
// larger than a wave the tables live in global memory and the whole group
// works; the last rounds (half-table <= 64) run in wave 0 alone with the
// pairs in registers: lane t holds entries t and t + h, and folding moves
// entry t + h/2 down by h/2 lanes.  The transcript lane's chain (hashing,
// two field conversions) is the serial part of every round.
__global__ void __launch_bounds__(kRoundsBlock) rounds_kernel(const RoundsJob* __restrict__ jobs) {
  const RoundsJob& J = jobs[blockIdx.x];
  // the rounds are one serial chain per group (transcript hashing on a
  // single lane); when they overlap contraction kernels on the same CUs,
  // their waves go first
  __builtin_amdgcn_s_setprio(3);
  __shared__ uint32_t red[3 * 8 * (kRoundsBlock / kWave)];
  __shared__ uint32_t first[VL_MAX_PRODS][3][8];   // round-1 values per product
  __shared__ uint32_t bcast[8];                    // the round's challenge
  __shared__ int32_t verdict;
  const uint32_t tid = threadIdx.x, NT = blockDim.x;
  const uint32_t wave = tid >> 6, lane = tid & 63u;

  if (J.ready) {
    // persistent mode: wait until every pass-1 block of this group has
    // counted itself (acquire), at most spin_limit polls
    if (tid == 0) {
      uint32_t polls = 0;
      int32_t ok = 1;
      while (__hip_atomic_load(J.ready, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) < J.ready_target) {
        if (++polls > J.spin_limit) {
          ok = 0;
          break;
        }
        __builtin_amdgcn_s_sleep(8);
      }
      verdict = ok;
    }
    __syncthreads();
    if (!verdict) {
      if (tid == 0) *J.status = VL_ERR_TIMEOUT;
      return;
    }
  }
  if (J.err && *(volatile const int32_t*)J.err) {
    if (tid == 0) *J.status = VL_ERR_RANGE;
    return;
  }
  // c = C~(u, v) from the pass-1 partials of its dot product (canonical:
  // one factor in Montgomery form, the other canonical)
  Fr v1[1];
  v1[0] = fr_zero();
  for (uint32_t i = tid; i < J.c_nparts; i += NT) v1[0] = fr_add(v1[0], lds_or_global_fr(J.c_part + 24ull * i));
  block_sum_w0<1>(v1, red);
  const Fr c = v1[0];   // valid in lane 0 of wave 0
  __syncthreads();      // red is reused by the next sum

  // round 1 of every product from its partials; its g(0) + g(1) is
  // sum_w a_p[w] b_p[w]
  Fr total = fr_zero();
  for (uint32_t p = 0; p < J.n_prods; ++p) {
    const RoundsProd& P = J.prods[p];
    Fr g[3];
    g[0] = g[1] = g[2] = fr_zero();
    for (uint32_t i = tid; i < P.g_nparts; i += NT)
#pragma unroll
      for (int k = 0; k < 3; ++k) g[k] = fr_add(g[k], lds_or_global_fr(P.g_part + 24ull * i + 8 * k));
    block_sum_w0<3>(g, red);
    if (tid == 0)
#pragma unroll
      for (int k = 0; k < 3; ++k) lds_put(first[p][k], g[k]);
    total = fr_add(total, fr_add(g[0], g[1]));
    __syncthreads();   // red is reused by the next sum
  }
  if (tid == 0) verdict = fr_eq(total, c) ? 1 : 0;
  __syncthreads();
  if (!verdict) {
    if (tid == 0) *J.status = VL_ERR_FALSE_STATEMENT;
    return;
  }

  // the transcript lives in thread 0; every thread keeps the same proof cursor
  Transcript tr;
  uint8_t* out = J.proof;
  if (tid == 0) {
#pragma unroll
    for (int i = 0; i < 8; ++i) tr.h[i] = J.st[i];
    const Fr cc[1] = {c};
    put_canon(out, cc[0]);
    tr_absorb_frs(tr, VL_LBL_CLAIM, cc);
    for (uint32_t p = 0; p + 1 < J.n_prods; ++p) {
      const Fr sc[1] = {fr_add(lds_get(first[p][0]), lds_get(first[p][1]))};
      put_canon(out + 32 * (1 + p), sc[0]);
      tr_absorb_frs(tr, VL_LBL_PART, sc);
    }
  }
  out += 32 * J.n_prods;
  for (uint32_t p = 0; p < J.n_prods; ++p) {
    const RoundsProd& P = J.prods[p];
    uint32_t* a = P.a;
    uint32_t* b = P.b;
    const uint64_t ld = P.ld;
    uint32_t rd = 0;
    // rounds over tables in global memory, the whole workgroup.  Round 0's
    // values come from pass 1; every later one folds the tables by the
    // previous challenge and sums the new pairs in the same sweep: for
    // t < h, entries t, t + h, t + 2h, t + 3h of the tables as they stand
    // (half-size 2h) fold into entries t and t + h (half-size h), which are
    // the round's pair.  Each thread reads and writes only its own entries.
    bool pending = false;   // tables still to be folded by r
    Fr r = fr_zero();
    for (; rd < P.n1; ++rd) {
      const uint32_t h = 1u << (P.n1 - 1 - rd);
      if (h <= kWave) break;
      Fr g[3];
      if (rd == 0) {
#pragma unroll
        for (int k = 0; k < 3; ++k) g[k] = lds_get(first[p][k]);
      } else {
        g[0] = g[1] = g[2] = fr_zero();
        for (uint32_t t = tid; t < h; t += NT) {
          const Fr a00 = load_sol(a, ld, t), a01 = load_sol(a, ld, t + 2 * h);
          const Fr a10 = load_sol(a, ld, t + h), a11 = load_sol(a, ld, t + 3 * h);
          const Fr b00 = load_sol(b, ld, t), b01 = load_sol(b, ld, t + 2 * h);
          const Fr b10 = load_sol(b, ld, t + h), b11 = load_sol(b, ld, t + 3 * h);
          const Fr a0 = fr_add(a00, fr_mul(r, fr_sub(a01, a00)));
          const Fr a1 = fr_add(a10, fr_mul(r, fr_sub(a11, a10)));
          const Fr b0 = fr_add(b00, fr_mul(r, fr_sub(b01, b00)));
          const Fr b1 = fr_add(b10, fr_mul(r, fr_sub(b11, b10)));
          store_sol(a, ld, t, a0);
          store_sol(a, ld, t + h, a1);
          store_sol(b, ld, t, b0);
          store_sol(b, ld, t + h, b1);
          g[0] = fr_add(g[0], fr_mul(a0, b0));
          g[1] = fr_add(g[1], fr_mul(a1, b1));
          g[2] = fr_add(g[2], fr_mul(at_two(a0, a1), at_two(b0, b1)));
        }
        __threadfence_block();   // the folded entries, for the next sweep
        block_sum_w0<3>(g, red);
      }
      if (wave == 0) {
        const Fr rr = round_challenge(tr, g, out, lane);
        if (lane == 0) lds_put(bcast, rr);
      }
      out += 96;
      __syncthreads();
      // every thread reads r before its next sweep's block sum, whose
      // barrier wave 0 passes before it writes bcast again
      r = lds_get(bcast);
      pending = true;
    }
    // the last rounds (half-table h <= 64): wave 0, pairs in registers (the
    // last global challenge, if any, folded in as they are loaded)
    if (wave == 0) {
      Fr fa, fb;   // the product's final a~ and b~ (lane 0)
      if (rd < P.n1) {
        uint32_t h = 1u << (P.n1 - 1 - rd);
        Fr A0 = fr_zero(), A1 = fr_zero(), B0 = fr_zero(), B1 = fr_zero();
        if (lane < h) {
          A0 = load_sol(a, ld, lane);
          A1 = load_sol(a, ld, lane + h);
          B0 = load_sol(b, ld, lane);
          B1 = load_sol(b, ld, lane + h);
          if (pending) {
            A0 = fr_add(A0, fr_mul(r, fr_sub(load_sol(a, ld, lane + 2 * h), A0)));
            A1 = fr_add(A1, fr_mul(r, fr_sub(load_sol(a, ld, lane + 3 * h), A1)));
            B0 = fr_add(B0, fr_mul(r, fr_sub(load_sol(b, ld, lane + 2 * h), B0)));
            B1 = fr_add(B1, fr_mul(r, fr_sub(load_sol(b, ld, lane + 3 * h), B1)));
          }
        }
        for (; rd < P.n1; ++rd, h >>= 1) {
          Fr g[3];
          g[0] = fr_mul(A0, B0);   // lanes >= h hold zeros
          g[1] = fr_mul(A1, B1);
          g[2] = fr_mul(at_two(A0, A1), at_two(B0, B1));
          wave_sum<3>(g, h);
          const Fr rr = round_challenge(tr, g, out, lane);
          out += 96;
          // fold; then entry t + h/2 of the folded table comes from lane t + h/2
          Fr na = fr_add(A0, fr_mul(rr, fr_sub(A1, A0)));
          Fr nb = fr_add(B0, fr_mul(rr, fr_sub(B1, B0)));
          if (lane >= h) na = nb = fr_zero();
          const uint32_t hh = h >> 1;
          Fr ua, ub;
#pragma unroll
          for (int j = 0; j < 8; ++j) {
            ua.w[j] = __shfl(na.w[j], (int)(lane + hh), kWave);
            ub.w[j] = __shfl(nb.w[j], (int)(lane + hh), kWave);
          }
          A0 = na;
          B0 = nb;
          A1 = lane < hh ? ua : fr_zero();
          B1 = lane < hh ? ub : fr_zero();
          if (lane >= hh) A0 = B0 = fr_zero();
          if (h == 1) {   // last round: the folded single entries
            fa = na;
            fb = nb;
          }
        }
      } else {   // no rounds (D1 = 1)
        fa = load_sol(a, ld, 0);
        fb = load_sol(b, ld, 0);
      }
      if (lane == 0) {
        Fr fin[2];
        fin[0] = fr_from_mont(fa);   // a~ tables are in Montgomery form,
        fin[1] = fb;                 // b~ tables in canonical form
        put_canon(out, fin[0]);
        put_canon(out + 32, fin[1]);
        tr_absorb_frs(tr, VL_LBL_FINAL, fin);
      }
    } else {
      out += 96 * (P.n1 - rd);
    }
    out += 64;
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

// device copy of a pinned host buffer (src is its device-side address): the
// GPU reads host memory directly, so the copy runs on the caller's stream
// with no copy-engine command, which other streams' copies could queue behind
__global__ void __launch_bounds__(256) copy_in_kernel(u32x4* __restrict__ dst, const u32x4* __restrict__ src,
                                                      uint64_t n16) {
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n16; i += (uint64_t)gridDim.x * blockDim.x)
    dst[i] = src[i];
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
    VL_CK(CK_I16_COLS2_VEC, int16_t, 1, 16, false, true, 2)
    VL_CK(CK_I32_ROWS, int32_t, 2, 24, true, false, 1)
    VL_CK(CK_I32_ROWS4_VEC, int32_t, 2, 24, true, true, 4)
    VL_CK(CK_I32_COLS, int32_t, 2, 24, false, false, 1)
    VL_CK(CK_I32_COLS_VEC, int32_t, 2, 24, false, true, 1)
    VL_CK(CK_I64S_ROWS, int64_t, 2, 24, true, false, 1)
    VL_CK(CK_I64S_ROWS2_VEC, int64_t, 2, 24, true, true, 2)
    VL_CK(CK_I64S_COLS, int64_t, 2, 24, false, false, 1)
    VL_CK(CK_I64S_COLS_VEC, int64_t, 2, 24, false, true, 1)
    VL_CK(CK_I64S_COLS2_VEC, int64_t, 2, 24, false, true, 2)
    VL_CK(CK_I64_ROWS, int64_t, 3, 24, true, false, 1)
    VL_CK(CK_I64_ROWS2_VEC, int64_t, 3, 24, true, true, 2)
    VL_CK(CK_I64_COLS, int64_t, 3, 24, false, false, 1)
    VL_CK(CK_I64_COLS_VEC, int64_t, 3, 24, false, true, 1)
    default: return hipErrorInvalidValue;
  }
#undef VL_CK
}

hipError_t launch_finish(const FinishJob* jobs, uint32_t n_jobs, uint32_t n_blocks, hipStream_t s) {
  if (n_blocks == 0) return hipSuccess;
  hipLaunchKernelGGL(finish_kernel, dim3(n_blocks), dim3(256), 0, s, jobs, n_jobs, n_blocks);
  return hipGetLastError();
}

hipError_t launch_pass1(const Pass1Job* jobs, uint32_t n_jobs, uint32_t n_blocks, hipStream_t s) {
  if (n_blocks == 0) return hipSuccess;
  hipLaunchKernelGGL(pass1_kernel, dim3(n_blocks), dim3(256), 0, s, jobs, n_jobs, n_blocks);
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

hipError_t launch_copy_in(void* dst, const void* src, uint64_t bytes, hipStream_t s) {
  if (bytes == 0) return hipSuccess;
  const uint64_t n16 = bytes / 16;
  hipLaunchKernelGGL(copy_in_kernel, dim3((uint32_t)std::min<uint64_t>(blocks_for(n16, 256), 64)), dim3(256), 0, s,
                     reinterpret_cast<u32x4*>(dst), reinterpret_cast<const u32x4*>(src), n16);
  return hipGetLastError();
}

hipError_t launch_zero_words(uint32_t* p, uint64_t n, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(zero_kernel, dim3(blocks_for(n, 256)), dim3(256), 0, s, p, n);
  return hipGetLastError();
}

}  // namespace vl
