// Integer contraction kernels of the matmul-sumcheck prover (gfx950): the
// partial evaluations A~(u, w) and B~(w, v) and the claim's contraction of C,
// eq. (zk-mle-matmul), and the finish pass that adds up split contractions.
//
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
#include <type_traits>

#include "device.hpp"

namespace vl {

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
  if constexpr (VEC && !ROWS && sizeof(T) == 2 && OPL == 1) {
    // cols layout, int16, 16-byte aligned rows: the wave's 64 rows (one per
    // lane) are read in stages of 64 entries (128 bytes) per row.  Each of a
    // stage's 8 load instructions fetches 8 rows whole (lanes 8k .. 8k + 7
    // one row, its eight 16-byte pieces rotated by the row index), so a load
    // touches 8 cache lines instead of 64, and the pieces go through LDS to
    // the lane of their row.  Lane r finds piece p of its row at slot
    // ((r & 7) << 3) | ((p + r) & 7) of load r >> 3: each group of 8 lanes
    // reads 8 different 16-byte bank groups, and at step p every lane holds
    // entries 8p .. 8p + 7 of the stage, so the eq digits stay wave-uniform.
    // One LDS buffer per wave (a wave's LDS accesses execute in order, so the
    // next stage is written only after this one was read) and one stage in
    // flight in registers keep the footprint at 8 KB of LDS and about 90
    // VGPRs, five waves per SIMD.  Lanes past the last row re-read the last
    // row; vector indexes are clamped to the row's last (partly) valid one,
    // and eq digits are read only for entries inside the chunk.
    constexpr uint32_t BE = 8, NP = 8, SE = BE * NP;
    __shared__ u32x4 stage_lds[kContractBlock / kWave][NP * kWave];
    u32x4* buf = stage_lds[threadIdx.x >> 6];
    const uint32_t span = m1 - m0, nvec = (span + BE - 1) / BE, nst = (span + SE - 1) / SE;
    const uint32_t lrow = lane >> 3, lpiece = ((lane & 7) - lrow) & 7;
    const gptr<u32x4> lbase = (gptr<u32x4>)(Mg + (uint64_t)min(owave * 64u + lrow, n_out - 1) * ld + m0);
    const uint64_t ldv = ld / BE;   // row stride in 16-byte vectors (ld * 2 is a multiple of 16)
    auto lrowp = [&](uint32_t i) -> gptr<u32x4> {
      // row owave*64 + 8i + lrow, clamped to the last row
      const uint32_t row = owave * 64u + 8 * i + lrow;
      return row < n_out ? lbase + (uint64_t)(8 * i) * ldv : (gptr<u32x4>)(Mg + (uint64_t)(n_out - 1) * ld + m0);
    };
    auto ldst = [&](uint32_t st, u32x4 (&b)[NP]) {   // nontemporal: read once
#pragma unroll
      for (uint32_t i = 0; i < NP; ++i) b[i] = __builtin_nontemporal_load(&lrowp(i)[min(st * NP + lpiece, nvec - 1)]);
    };
    u32x4 r[NP];
    ldst(0, r);
    for (uint32_t st = 0; st < nst; ++st) {
#pragma unroll
      for (uint32_t i = 0; i < NP; ++i) buf[i * kWave + lane] = r[i];
      ldst(st + 1, r);
      const uint32_t mst = m0 + st * SE;
#pragma unroll 1
      for (uint32_t pc = 0; pc < NP; ++pc) {
        const u32x4 x = buf[(lane >> 3) * kWave + (((lane & 7) << 3) | ((pc + lane) & 7))];
        const uint32_t mp = mst + pc * BE;
        if (mp >= m1) break;   // uniform: the rest of the stage is past the chunk
        if (mp + BE <= m1) {   // the piece's eq digits in one batch of scalar loads
          ci32_ptr pe = pack + (uint64_t)mp * 8;
          int32_t e[BE][8];
#pragma unroll
          for (uint32_t q = 0; q < BE; ++q)
#pragma unroll
            for (int j = 0; j < 8; ++j) e[q][j] = pe[q * 8 + j];
#pragma unroll
          for (uint32_t q = 0; q < BE; ++q) {
            int32_t d[1][ND];
            const uint32_t w = x[q >> 1];
            d[0][0] = (q & 1) ? ((int32_t)w >> 16) : ((int32_t)(w << 16) >> 16);
            mac8v<1, ND>(e[q], d, acc);
          }
        } else {               // the chunk's last, partial piece
#pragma unroll
          for (uint32_t q = 0; q < BE; ++q) {
            if (mp + q < m1) {
              int32_t d[1][ND];
              const uint32_t w = x[q >> 1];
              d[0][0] = (q & 1) ? ((int32_t)w >> 16) : ((int32_t)(w << 16) >> 16);
              mac8<1, ND>(pack + (uint64_t)(mp + q) * 8, d, acc);
            }
          }
        }
      }
    }
  } else if constexpr (VEC && !ROWS) {
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
    // nontemporal loads: each row segment is read once, so the caches may
    // treat it as streaming data
    auto row = [&](uint32_t r) -> LT {
      return __builtin_nontemporal_load((gptr<LT>)(base + (uint64_t)min(r, rows - 1) * ld));
    };
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

// ---------------------------------------------------------------- launchers -
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

}  // namespace vl
