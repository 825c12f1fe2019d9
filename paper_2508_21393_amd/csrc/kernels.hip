// Device kernels of the matmul-sumcheck prover (gfx950), apart from the
// integer contractions (contract.hip).
//
// Paths and the paper passages they compute:
//   eq_kernel        eq(x, i) tables, eq. (MLE) Lagrange basis, and their
//                    signed-digit pack form for the contractions
//   pass1_kernel     the claim's dot product and round 1 of every product
//                    as partial sums across the GPU
//   rounds_kernel    claim c = C~(u, v), the sumcheck rounds (Sec. II-B.1)
//                    with Fiat-Shamir challenges, and the fold of each round
//   lift/export      integer -> Fr lifting (x < 0 -> p - |x|) and back to
//                    canonical form
//   upload/copy_in   job descriptors to the workspace
#include <cstring>

#include "device.hpp"
#include "rounds_dev.hpp"
#include "sha256.hpp"

namespace vl {

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
  // thread t covers entries 4t .. 4t + 3 (the whole table when nvars < 2)
  const uint32_t t = tid - J.thread_begin;
  const uint32_t n = J.nvars;
  const uint64_t len = 1ull << n;
  auto point = [&](uint32_t j) {
    Fr x;
#pragma unroll
    for (int k = 0; k < 8; ++k) x.w[k] = J.point[j * 8 + k];
    return x;
  };
  Fr e[4];
  Fr sc = fr_R();
  if (J.scaled)
#pragma unroll
    for (int k = 0; k < 8; ++k) sc.w[k] = J.scale[k];
  if (n < 2) {
    e[0] = n == 0 ? sc : fr_mul(sc, fr_sub(fr_R(), point(0)));
    e[1] = n == 0 ? fr_zero() : fr_mul(sc, point(0));
    e[2] = e[3] = fr_zero();
  } else {
    // factor j is x_j for bit 1 and 1 - x_j for bit 0 (b_1 the most
    // significant bit): the first n - 2 come from t, shared by the four
    // entries; the last two split the product into a tree of 2 + 4 products
    Fr base = fr_R();
    for (uint32_t j = 0; j + 2 < n; ++j) {
      const Fr x = point(j);
      const Fr f = ((t >> (n - 3 - j)) & 1u) ? x : fr_sub(fr_R(), x);
      base = j == 0 ? f : fr_mul(base, f);
    }
    if (J.scaled) base = n > 2 ? fr_mul(base, sc) : sc;
    const Fr xa = point(n - 2), xb = point(n - 1);
    const Fr bb[2] = {base, base}, fa[2] = {fr_sub(fr_R(), xa), xa}, fb[2] = {fr_sub(fr_R(), xb), xb};
    Fr h[2], q0[2], q1[2];
    fr_mul_n<2>(bb, fa, h);
    const Fr h0[2] = {h[0], h[0]}, h1[2] = {h[1], h[1]};
    fr_mul_n<2>(h0, fb, q0);
    fr_mul_n<2>(h1, fb, q1);
    e[0] = q0[0];
    e[1] = q0[1];
    e[2] = q1[0];
    e[3] = q1[1];
  }
  const uint64_t i0 = 4ull * t;
#pragma unroll
  for (uint32_t q = 0; q < 4; ++q) {
    const uint64_t i = i0 + q;
    if (J.eq && i < len) store_sol(J.eq, J.eq_ld, i, J.eq_canon ? fr_from_mont(e[q]) : e[q]);
    // pack: e * R^2 (or e * R) mod p as signed digits, 8 words per entry
    if (J.pack && i < J.pack_len) signed_digits(J.pack_r2 ? fr_to_mont(e[q]) : e[q], J.pack + i * 8);
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

// ---------------------------------------------------------------- rounds ----
// absorb("round", g(0), g(1), g(2)) by the lanes of wave 0: the message
// (the state, the label and the three canonical values, 133 bytes in three
// SHA-256 blocks) has its three blocks' message schedules computed side by
// side, lane b < 3 holding block b's, and every lane then runs the 3 x 64
// compression rounds on those words (uniform values read with v_readlane).
// The same digest as tr_absorb_frs; the state is taken from lane 0.
__device__ __forceinline__ void absorb_round_lanes(Transcript& tr, const Fr (&gc)[3], uint32_t lane) {
  constexpr int L = sizeof(VL_LBL_ROUND) - 1;
  constexpr int N = 32 + L + 96;
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
  const uint32_t* K = sha256_k();
#pragma unroll
  for (int i = 0; i < 64; ++i) w[i] += K[i];
  // a fresh SHA-256 hash: the chaining value starts at the initial hash value
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

// One sumcheck round's messages and challenge, run by wave 0 (all its
// lanes, g canonical and valid in lane 0): lane k < 3 writes g(k) to the
// proof; the wave absorbs the three values (all 64 lanes must be active:
// lanes 1 and 2 hold message schedules) and lane 0 squeezes r.  Returns r in
// Montgomery form in every lane of wave 0.
__device__ __forceinline__ Fr round_challenge(Transcript& tr, const Fr (&g)[3], uint8_t* out, uint32_t lane,
                                              bool write = true) {
  Fr gc[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) gc[k] = readlane_fr(g[k], 0);
  Fr mine;   // word by word: a select of whole values goes through scratch memory
#pragma unroll
  for (int j = 0; j < 8; ++j) mine.w[j] = lane == 0 ? gc[0].w[j] : (lane == 1 ? gc[1].w[j] : gc[2].w[j]);
  if (write && lane < 3) put_canon(out + 32 * lane, mine);
  Fr r = fr_zero();
  absorb_round_lanes(tr, gc, lane);
  if (lane == 0) r = fr_to_mont(tr_squeeze_fixed(tr, VL_LBL_R));
  return readlane_fr(r, 0);
}

// ------------------------------------------------------- wide rounds ------
// The transcript step of wide round k of a group (its values from partial
// sums, absorbed; r_k squeezed), computed by a 256-thread block.  Every block
// of the launch that needs r_k computes the step itself from the same
// partials, so no block waits for another and no fence is needed; only the
// launch's first block of the group (write) stores the proof bytes and io.
// Round 0 (k = 0): the range flag, c = C~(u, v) and every product's round-1
// values from the pass-1 partials, the prover guard, the claim and the part
// claims, as the rounds kernel does without wide rounds; a failure is
// reported (by the writing block) and every block returns false.  Later
// rounds: the partials of sweep k (buffer k & 1), the state after round
// k - 1 (io slot (k - 1) & 1).  r_k is returned in every thread.
__device__ bool mat_step_block(const RoundsJob& J, uint32_t k, bool write, Fr& r_out) {
  __shared__ uint32_t red[4 * 8 * 4];
  __shared__ uint32_t first[VL_MAX_PRODS][3][8];
  __shared__ uint32_t bcast[8];
  __shared__ int32_t verdict;
  const uint32_t tid = threadIdx.x, wave = tid >> 6, lane = tid & 63u;
  uint8_t* out = J.proof + 32ull * J.n_prods + 96ull * k;
  Transcript tr;
  Fr g[4];
  g[0] = g[1] = g[2] = g[3] = fr_zero();
  if (k == 0) {
    const int32_t bad = J.err && *(volatile const int32_t*)J.err;
    if (bad) {
      if (write && tid == 0) {
        J.io[0] = (uint32_t)VL_ERR_RANGE;
        *J.status = VL_ERR_RANGE;
      }
      return false;
    }
    Fr v[4];
    v[0] = v[1] = v[2] = v[3] = fr_zero();
    for (uint32_t i = tid; i < J.c_nparts; i += 256) v[0] = fr_add(v[0], lds_or_global_fr(J.c_part + 24ull * i));
    block256_sum4(v, red);
    const Fr c = v[0];   // valid in thread 0
    __syncthreads();
    Fr total = fr_zero();
    for (uint32_t p = 0; p < J.n_prods; ++p) {
      const RoundsProd& P = J.prods[p];
      Fr gp[4];
      gp[0] = gp[1] = gp[2] = gp[3] = fr_zero();
      for (uint32_t i = tid; i < P.g_nparts; i += 256)
#pragma unroll
        for (int q = 0; q < 3; ++q) gp[q] = fr_add(gp[q], lds_or_global_fr(P.g_part + 24ull * i + 8 * q));
      block256_sum4(gp, red);
      if (tid == 0)
#pragma unroll
        for (int q = 0; q < 3; ++q) lds_put(first[p][q], gp[q]);
      total = fr_add(total, fr_add(gp[0], gp[1]));
      __syncthreads();
    }
    if (tid == 0) verdict = fr_eq(total, c) ? 1 : 0;
    __syncthreads();
    if (!verdict) {
      if (write && tid == 0) {
        J.io[0] = (uint32_t)VL_ERR_FALSE_STATEMENT;
        *J.status = VL_ERR_FALSE_STATEMENT;
      }
      return false;
    }
    if (tid == 0) {
#pragma unroll
      for (int i = 0; i < 8; ++i) tr.h[i] = J.st[i];
      const Fr cc[1] = {c};
      if (write) put_canon(J.proof, cc[0]);
      tr_absorb_frs(tr, VL_LBL_CLAIM, cc);
      for (uint32_t p = 0; p + 1 < J.n_prods; ++p) {
        const Fr sc[1] = {fr_add(lds_get(first[p][0]), lds_get(first[p][1]))};
        if (write) put_canon(J.proof + 32 * (1 + p), sc[0]);
        tr_absorb_frs(tr, VL_LBL_PART, sc);
      }
    }
#pragma unroll
    for (int q = 0; q < 3; ++q) g[q] = lds_get(first[0][q]);
  } else {
    const uint32_t h = 1u << (J.prods[0].n1 - 1 - k);
    const uint32_t nb = (h + kMatSweepPairs - 1) / kMatSweepPairs;
    const uint32_t* part = J.wpart + (uint64_t)(k & 1) * J.wpart_stride;
    for (uint32_t i = tid; i < nb; i += 256)
#pragma unroll
      for (int q = 0; q < 3; ++q) g[q] = fr_add(g[q], lds_or_global_fr(part + 24ull * i + 8 * q));
    block256_sum4(g, red);   // valid in thread 0
    if (tid == 0)
#pragma unroll
      for (int i = 0; i < 8; ++i) tr.h[i] = J.io[kMatIoState + 8 * ((k - 1) & 1) + i];
  }
  if (wave == 0) {
    const Fr g3[3] = {g[0], g[1], g[2]};
    const Fr r = round_challenge(tr, g3, out, lane, write);
    if (lane == 0) {
      if (write)
#pragma unroll
        for (int i = 0; i < 8; ++i) {
          J.io[kMatIoState + 8 * (k & 1) + i] = tr.h[i];
          J.io[kMatIoR + 8 * (k & 1) + i] = r.w[i];
        }
      lds_put(bcast, r);
    }
  }
  __syncthreads();
  r_out = lds_get(bcast);
  return true;
}

// Wide round rd >= 1 of product 0 across the GPU: every block first takes
// round rd - 1's transcript step (mat_step_block) for r_{rd-1}; then every
// thread takes one pair t < h of round rd, folds the entries t, t + h,
// t + 2h, t + 3h of the tables by r_{rd-1} into t and t + h (as the rounds
// kernel's sweeps do; each thread reads and writes only its own entries)
// and adds the pair's three products; a block writes its sums to the
// partials buffer rd & 1.
__global__ void __launch_bounds__(256) mat_sweep_kernel(const RoundsJob* __restrict__ jobs,
                                                        const MatSweep* __restrict__ list, uint32_t n_list,
                                                        uint32_t n_blocks, uint32_t rd) {
  const uint32_t blk = blockIdx.x;
  if (blk >= n_blocks) return;
  uint32_t lo = 0, hi = n_list;
  while (hi - lo > 1) {
    const uint32_t mid = (lo + hi) >> 1;
    if (list[mid].block_begin <= blk) lo = mid; else hi = mid;
  }
  const MatSweep& S = list[lo];
  const RoundsJob& J = jobs[S.job];
  if (*reinterpret_cast<volatile const int32_t*>(J.io) != VL_OK) return;
  Fr r;
  if (!mat_step_block(J, rd - 1, blk == S.block_begin, r)) return;
  const RoundsProd& P = J.prods[0];
  uint32_t* a = P.a;
  uint32_t* b = P.b;
  const uint64_t ld = P.ld;
  const uint32_t h = 1u << (P.n1 - 1 - rd);
  const uint32_t t = (blk - S.block_begin) * kMatSweepPairs + threadIdx.x;
  Fr g[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) g[k] = fr_zero();
  if (t < h) {
    const Fr a00 = load_sol(a, ld, t), a01 = load_sol(a, ld, t + 2 * h);
    const Fr a10 = load_sol(a, ld, t + h), a11 = load_sol(a, ld, t + 3 * h);
    const Fr b00 = load_sol(b, ld, t), b01 = load_sol(b, ld, t + 2 * h);
    const Fr b10 = load_sol(b, ld, t + h), b11 = load_sol(b, ld, t + 3 * h);
    const Fr rr2[2] = {r, r}, da[2] = {fr_sub(a01, a00), fr_sub(a11, a10)};
    const Fr db[2] = {fr_sub(b01, b00), fr_sub(b11, b10)};
    Fr fa[2], fb[2];
    fr_mul_n<2>(rr2, da, fa);
    fr_mul_n<2>(rr2, db, fb);
    const Fr a0 = fr_add(a00, fa[0]), a1 = fr_add(a10, fa[1]);
    const Fr b0 = fr_add(b00, fb[0]), b1 = fr_add(b10, fb[1]);
    store_sol(a, ld, t, a0);
    store_sol(a, ld, t + h, a1);
    store_sol(b, ld, t, b0);
    store_sol(b, ld, t + h, b1);
    const Fr x[3] = {a0, a1, at_two(a0, a1)}, y[3] = {b0, b1, at_two(b0, b1)};
    Fr pr[3];
    fr_mul_n<3>(x, y, pr);
#pragma unroll
    for (int k = 0; k < 3; ++k) g[k] = pr[k];
  }
  __shared__ uint32_t red[4 * 8 * 4];
  block256_sum4(g, red);
  if (threadIdx.x == 0) {
    uint32_t* o = J.wpart + (uint64_t)(rd & 1) * J.wpart_stride + (uint64_t)(blk - S.block_begin) * 24;
#pragma unroll
    for (int k = 0; k < 3; ++k)
#pragma unroll
      for (int j = 0; j < 8; ++j) o[k * 8 + j] = g[k].w[j];
  }
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
      const Fr x[3] = {a0, a1, at_two(a0, a1)}, y[3] = {b0, b1, at_two(b0, b1)};
      Fr pr[3];
      fr_mul_n<3>(x, y, pr);
#pragma unroll
      for (int k = 0; k < 3; ++k) g[k] = fr_add(g[k], pr[k]);
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
  __shared__ uint32_t coef[2][3][3][8];            // register rounds: value k as c0 + c1 r + c2 r^2
  __shared__ uint32_t rbuf[2][8];                  // register rounds: r_j by parity
  __shared__ uint32_t finv[2][8];                  // the product's final a~, b~
  __shared__ int32_t verdict;
  const uint32_t tid = threadIdx.x, NT = blockDim.x;
  const uint32_t wave = tid >> 6, lane = tid & 63u;

  if (J.ready) {
    // persistent mode: wait until every pass-1 block of this group has
    // counted itself, at most spin_limit polls.  The polls are relaxed loads
    // and one acquire fence follows the loop (an acquire load per poll would
    // invalidate this XCD's L2 on every poll, under the contraction kernels
    // that share it); the fence pairs with the pass-1 blocks' release
    // increments.
    if (tid == 0) {
      uint32_t polls = 0;
      int32_t ok = 1;
      while (__hip_atomic_load(J.ready, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < J.ready_target) {
        if (++polls > J.spin_limit) {
          ok = 0;
          break;
        }
        __builtin_amdgcn_s_sleep(8);
      }
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
      verdict = ok;
    }
    __syncthreads();
    if (!verdict) {
      if (tid == 0) *J.status = VL_ERR_TIMEOUT;
      return;
    }
  }
  if (J.wide) {
    // the range flag, the claim, the prover guard and product 0's first
    // J.wide rounds ran as wide launches, which left their status in io
    const int32_t st = *reinterpret_cast<volatile const int32_t*>(J.io);
    if (st != VL_OK) {
      if (tid == 0) *J.status = st;
      return;
    }
  } else if (J.err && *(volatile const int32_t*)J.err) {
    if (tid == 0) *J.status = VL_ERR_RANGE;
    return;
  }
  // c = C~(u, v) from the pass-1 partials of its dot product (canonical:
  // one factor in Montgomery form, the other canonical)
  Fr c = fr_zero();
  if (!J.wide) {
    Fr v1[1];
    v1[0] = fr_zero();
    for (uint32_t i = tid; i < J.c_nparts; i += NT) v1[0] = fr_add(v1[0], lds_or_global_fr(J.c_part + 24ull * i));
    block_sum_w0<1>(v1, red);
    c = v1[0];          // valid in lane 0 of wave 0
    __syncthreads();    // red is reused by the next sum
  }

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
  if (!J.wide) {
    if (tid == 0) verdict = fr_eq(total, c) ? 1 : 0;
    __syncthreads();
    if (!verdict) {
      if (tid == 0) *J.status = VL_ERR_FALSE_STATEMENT;
      return;
    }
  }

  // the transcript lives in thread 0; every thread keeps the same proof cursor
  Transcript tr;
  uint8_t* out = J.proof;
  if (J.wide) {
    // the state after round wide - 2, the last step a wide launch took
    if (tid == 0)
#pragma unroll
      for (int i = 0; i < 8; ++i) tr.h[i] = J.io[kMatIoState + 8 * ((J.wide - 2) & 1) + i];
  } else if (tid == 0) {
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
    if (p == 0 && J.wide) {
      // rounds 0 .. wide - 1 were summed by wide launches, which also took
      // the transcript steps of rounds 0 .. wide - 2; take round wide - 1's
      // step here (its values from the last sweep's partials), then resume
      // with the tables still to be folded by its challenge
      const uint32_t k = J.wide - 1;
      const uint32_t hk = 1u << (P.n1 - 1 - k);
      const uint32_t nb = (hk + kMatSweepPairs - 1) / kMatSweepPairs;
      const uint32_t* part = J.wpart + (uint64_t)(k & 1) * J.wpart_stride;
      Fr g[3];
      g[0] = g[1] = g[2] = fr_zero();
      for (uint32_t i = tid; i < nb; i += NT)
#pragma unroll
        for (int q = 0; q < 3; ++q) g[q] = fr_add(g[q], lds_or_global_fr(part + 24ull * i + 8 * q));
      block_sum_w0<3>(g, red);
      if (wave == 0) {
        const Fr rr = round_challenge(tr, g, out + 96ull * k, lane);
        if (lane == 0) lds_put(bcast, rr);
      }
      __syncthreads();
      r = lds_get(bcast);
      rd = J.wide;
      pending = true;
      out += 96ull * J.wide;
    }
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
          const Fr rr2[2] = {r, r}, da[2] = {fr_sub(a01, a00), fr_sub(a11, a10)};
          const Fr db[2] = {fr_sub(b01, b00), fr_sub(b11, b10)};
          Fr fa[2], fb[2];
          fr_mul_n<2>(rr2, da, fa);
          fr_mul_n<2>(rr2, db, fb);
          const Fr a0 = fr_add(a00, fa[0]), a1 = fr_add(a10, fa[1]);
          const Fr b0 = fr_add(b00, fb[0]), b1 = fr_add(b10, fb[1]);
          store_sol(a, ld, t, a0);
          store_sol(a, ld, t + h, a1);
          store_sol(b, ld, t, b0);
          store_sol(b, ld, t + h, b1);
          const Fr x[3] = {a0, a1, at_two(a0, a1)}, y[3] = {b0, b1, at_two(b0, b1)};
          Fr pr[3];
          fr_mul_n<3>(x, y, pr);
#pragma unroll
          for (int k = 0; k < 3; ++k) g[k] = fr_add(g[k], pr[k]);
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
    // The last rounds (half-table h <= 64), split over two waves so that the
    // table work of a round overlaps the hashing of the one before:
    //  - wave 1 holds the pairs in registers (lane t: entries t and t + h of
    //    a and b; the last global challenge, if any, folded in as they are
    //    loaded).  While wave 0 hashes round j it folds the tables by r_{j-1}
    //    and writes the next round's three values as quadratics in the
    //    challenge r_j it does not know yet: with the folded entries
    //    x + r y, each value sum (x + r y)(x' + r y') has the coefficients
    //    sum x x', sum (x y' + y x'), sum y y' (three products per pair);
    //  - wave 0 evaluates round j's values from those coefficients at r_{j-1}
    //    (exact: the same field elements as a direct sum), writes them to the
    //    proof, absorbs them and squeezes r_j.
    // One barrier per round hands r_j to wave 1 and the coefficients to wave
    // 0 (both double-buffered by round parity); the other waves only take part
    // in the barriers.
    if (rd < P.n1) {
      const uint32_t rd0 = rd;
      uint32_t h = 1u << (P.n1 - 1 - rd0);
      Fr A0 = fr_zero(), A1 = fr_zero(), B0 = fr_zero(), B1 = fr_zero();
      if (wave >= 1 && wave <= 3) {
        if (lane < h) {
          A0 = load_sol(a, ld, lane);
          A1 = load_sol(a, ld, lane + h);
          B0 = load_sol(b, ld, lane);
          B1 = load_sol(b, ld, lane + h);
          if (pending) {
            const Fr rr2[2] = {r, r};
            const Fr da[2] = {fr_sub(load_sol(a, ld, lane + 2 * h), A0), fr_sub(load_sol(a, ld, lane + 3 * h), A1)};
            const Fr db[2] = {fr_sub(load_sol(b, ld, lane + 2 * h), B0), fr_sub(load_sol(b, ld, lane + 3 * h), B1)};
            Fr fa[2], fb[2];
            fr_mul_n<2>(rr2, da, fa);
            fr_mul_n<2>(rr2, db, fb);
            A0 = fr_add(A0, fa[0]);
            A1 = fr_add(A1, fa[1]);
            B0 = fr_add(B0, fb[0]);
            B1 = fr_add(B1, fb[1]);
          }
        }
        // round rd0's values directly, as constant quadratics (wave 1)
        if (wave == 1) {
          Fr g[3];   // lanes >= h hold zeros
          {
            const Fr x[3] = {A0, A1, at_two(A0, A1)}, y[3] = {B0, B1, at_two(B0, B1)};
            fr_mul_n<3>(x, y, g);
          }
          wave_sum<3>(g, h);
          if (lane == 0)
#pragma unroll
            for (int k = 0; k < 3; ++k) {
              lds_put(coef[rd0 & 1][k][0], g[k]);
              lds_put(coef[rd0 & 1][k][1], g[k]);   // c1 = [1] - [0] - [2] = 0
              lds_put(coef[rd0 & 1][k][2], fr_zero());
            }
        }
      }
      __syncthreads();
      for (uint32_t j = rd0; j < P.n1; ++j, h >>= 1) {
        if (wave == 0) {
          const Fr rp = j > rd0 ? lds_get(rbuf[(j - 1) & 1]) : fr_zero();
          // g_k = c0 + r (c1 + r c2) with c1 = [1] - c0 - c2, lane k < 3
          // evaluating value k (the three side by side), then gathered
          const uint32_t kk = lane < 3 ? lane : 2u;
          const Fr c0 = lds_get(coef[j & 1][kk][0]), c2 = lds_get(coef[j & 1][kk][2]);
          const Fr c1 = fr_sub(fr_sub(lds_get(coef[j & 1][kk][1]), c0), c2);
          const Fr mine = fr_add(c0, fr_mul(rp, fr_add(c1, fr_mul(rp, c2))));
          Fr g[3];
#pragma unroll
          for (int k = 0; k < 3; ++k) g[k] = readlane_fr(mine, k);
          const Fr rj = round_challenge(tr, g, out, lane);
          if (lane == 0) lds_put(rbuf[j & 1], rj);
        } else if (wave >= 1 && wave <= 3) {
          if (j > rd0) {
            // fold by r_{j-1}; entry t + h of the folded table comes from lane t + h
            const Fr rp = lds_get(rbuf[(j - 1) & 1]);
            const uint32_t hp = 2 * h;   // the previous round's half-size
            const Fr rp2[2] = {rp, rp}, d[2] = {fr_sub(A1, A0), fr_sub(B1, B0)};
            Fr f[2];
            fr_mul_n<2>(rp2, d, f);
            Fr na = fr_add(A0, f[0]);
            Fr nb = fr_add(B0, f[1]);
            if (lane >= hp) na = nb = fr_zero();
            Fr ua, ub;
#pragma unroll
            for (int w = 0; w < 8; ++w) {
              ua.w[w] = __shfl(na.w[w], (int)(lane + h), kWave);
              ub.w[w] = __shfl(nb.w[w], (int)(lane + h), kWave);
            }
            const bool in = lane < h;
            A0 = in ? na : fr_zero();
            B0 = in ? nb : fr_zero();
            A1 = in ? ua : fr_zero();
            B1 = in ? ub : fr_zero();
          }
          if (j + 1 < P.n1) {
            // round j + 1 as quadratics in r_j: lane t < h/2 pairs its
            // folded entry x + r y (from entries t, t + h) with lane
            // t + h/2's (entries t + h/2, t + h/2 + h)
            const uint32_t hh = h >> 1;
            Fr qa0, qa1, qb0, qb1;   // lane t + hh's pair
#pragma unroll
            for (int w = 0; w < 8; ++w) {
              qa0.w[w] = __shfl(A0.w[w], (int)(lane + hh), kWave);
              qa1.w[w] = __shfl(A1.w[w], (int)(lane + hh), kWave);
              qb0.w[w] = __shfl(B0.w[w], (int)(lane + hh), kWave);
              qb1.w[w] = __shfl(B1.w[w], (int)(lane + hh), kWave);
            }
            Fr xa[3], ya[3], xb[3], yb[3];
            xa[0] = A0;  ya[0] = fr_sub(A1, A0);
            xb[0] = B0;  yb[0] = fr_sub(B1, B0);
            xa[1] = qa0; ya[1] = fr_sub(qa1, qa0);
            xb[1] = qb0; yb[1] = fr_sub(qb1, qb0);
            xa[2] = at_two(xa[0], xa[1]); ya[2] = at_two(ya[0], ya[1]);
            xb[2] = at_two(xb[0], xb[1]); yb[2] = at_two(yb[0], yb[1]);
            // Karatsuba's three products split over waves 1, 2, 3: the sums of
            // x x' (term 0), (x + y)(x' + y') (term 1) and y y' (term 2);
            // wave 0 forms c1 = [1] - [0] - [2]
            const uint32_t role = wave - 1;
            Fr ua[3], ub[3], pr[3];
#pragma unroll
            for (int k = 0; k < 3; ++k) {
              ua[k] = role == 0 ? xa[k] : (role == 2 ? ya[k] : fr_add(xa[k], ya[k]));
              ub[k] = role == 0 ? xb[k] : (role == 2 ? yb[k] : fr_add(xb[k], yb[k]));
            }
            fr_mul_n<3>(ua, ub, pr);
            if (lane >= hh)
#pragma unroll
              for (int k = 0; k < 3; ++k) pr[k] = fr_zero();
            wave_sum<3>(pr, hh);
            if (lane == 0)
#pragma unroll
              for (int k = 0; k < 3; ++k) lds_put(coef[(j + 1) & 1][k][role], pr[k]);
          }
        }
        out += 96;
        __syncthreads();
      }
      // the last challenge folds the single remaining pair into the finals
      if (wave == 1 && lane == 0) {
        const Fr rl = lds_get(rbuf[(P.n1 - 1) & 1]);
        const Fr rl2[2] = {rl, rl}, d[2] = {fr_sub(A1, A0), fr_sub(B1, B0)};
        Fr f[2];
        fr_mul_n<2>(rl2, d, f);
        lds_put(finv[0], fr_add(A0, f[0]));
        lds_put(finv[1], fr_add(B0, f[1]));
      }
      __syncthreads();
    }
    if (wave == 0) {
      Fr fa, fb;   // the product's final a~ and b~ (lane 0)
      if (P.n1 > 0) {
        fa = lds_get(finv[0]);
        fb = lds_get(finv[1]);
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

// ------------------------------------------------------- chained proofs ----
// M~(x, y) of a chained proof's evaluation step: the pass-1 partials of its
// dot product added (one block per value) and written canonical.
__global__ void __launch_bounds__(256) eval_kernel(const EvalJob* __restrict__ jobs) {
  const EvalJob& J = jobs[blockIdx.x];
  if (J.err && *(volatile const int32_t*)J.err) {
    if (threadIdx.x == 0) *J.status = VL_ERR_RANGE;
    return;
  }
  Fr v[1];
  v[0] = fr_zero();
  for (uint32_t i = threadIdx.x; i < J.nparts; i += 256) v[0] = fr_add(v[0], lds_or_global_fr(J.part + 24ull * i));
  __shared__ uint32_t red[8 * 4];
  wave_sum<1>(v, kWave);
  const uint32_t wave = threadIdx.x >> 6, lane = threadIdx.x & 63u;
  if (lane == 0)
#pragma unroll
    for (int j = 0; j < 8; ++j) red[j * 4 + wave] = v[0].w[j];
  __syncthreads();
  if (wave == 0) {
#pragma unroll
    for (int j = 0; j < 8; ++j) v[0].w[j] = lane < 4 ? red[j * 4 + lane] : 0u;
    wave_sum<1>(v, 4);
    if (lane == 0) {
      put_canon(J.out, v[0]);
      *J.status = VL_OK;
    }
  }
}

// absorb(label, x_0 .. x_{K-1}) for a run-time K <= kMaxClaims
template <int LN>
__device__ __forceinline__ void absorb_k(Transcript& tr, const char (&label)[LN], const Fr* xs, uint32_t K) {
  switch (K) {
    case 1: { const Fr a[1] = {xs[0]}; tr_absorb_frs(tr, label, a); break; }
    case 2: { const Fr a[2] = {xs[0], xs[1]}; tr_absorb_frs(tr, label, a); break; }
    case 3: { const Fr a[3] = {xs[0], xs[1], xs[2]}; tr_absorb_frs(tr, label, a); break; }
    default: { const Fr a[4] = {xs[0], xs[1], xs[2], xs[3]}; tr_absorb_frs(tr, label, a); break; }
  }
}

// One workgroup per reduction phase (ReduceJob).  Both phases are sumchecks
// of sum_t sum_k a_k[t] b_k[t] over tables in global memory: the a tables in
// Montgomery form, the b tables canonical, so every product and round value
// is canonical (as in the rounds kernel).  Round i > 0 folds the tables by
// the previous challenge in the same sweep that sums the round's pairs (each
// thread reads and writes only its own entries).  Wave 0 runs the
// transcript: it writes g(0), g(1), g(2), absorbs them and squeezes r.
__global__ void __launch_bounds__(kRoundsBlock) reduce_kernel(const ReduceJob* __restrict__ jobs) {
  const ReduceJob& J = jobs[blockIdx.x];
  __shared__ uint32_t red[3 * 8 * (kRoundsBlock / kWave)];
  __shared__ uint32_t bcast[8];
  const uint32_t tid = threadIdx.x, NT = blockDim.x;
  const uint32_t wave = tid >> 6, lane = tid & 63u;
  const uint32_t K = J.phase == 1 ? J.K : 1;
  const uint64_t ld = J.ld, len = 1ull << J.n;
  uint32_t* A[kMaxClaims];
  uint32_t* Bt[kMaxClaims];
  for (uint32_t k = 0; k < kMaxClaims; ++k) {
    A[k] = J.a[k];
    Bt[k] = J.b[k];
  }
  Transcript tr;
#pragma unroll
  for (int i = 0; i < 8; ++i) tr.h[i] = J.phase == 1 ? J.st[i] : J.io[i];
  if (J.phase == 1) {
    // scale the eq(x_k, .) tables by rho_k: the round sums then need no
    // per-claim coefficient, and folding keeps the scale
    for (uint32_t k = 0; k < K; ++k) {
      const Fr rho = lds_or_global_fr(J.coef[k]);
      for (uint64_t t = tid; t < len; t += NT) store_sol(A[k], ld, t, fr_mul(rho, load_sol(A[k], ld, t)));
    }
  } else {
    // b = sum_k sigma_k eq(y_k, .), canonical
    Fr sig[kMaxClaims];
    for (uint32_t k = 0; k < J.K; ++k) sig[k] = lds_or_global_fr(J.io + kReduceIoSigma + 8 * k);
    for (uint64_t t = tid; t < len; t += NT) {
      Fr acc = fr_zero();
      for (uint32_t k = 0; k < J.K; ++k) acc = fr_add(acc, fr_mul(sig[k], load_sol(J.b[k], ld, t)));
      store_sol(J.bsum, ld, t, acc);
    }
    Bt[0] = J.bsum;
  }
  __threadfence_block();
  __syncthreads();
  uint8_t* out = J.proof;
  bool pending = false;
  Fr r = fr_zero();
  for (uint32_t rd = 0; rd < J.n; ++rd) {
    const uint32_t h = 1u << (J.n - 1 - rd);
    Fr g[3];
    g[0] = g[1] = g[2] = fr_zero();
    for (uint32_t t = tid; t < h; t += NT) {
      for (uint32_t k = 0; k < K; ++k) {
        Fr a0 = load_sol(A[k], ld, t), a1 = load_sol(A[k], ld, t + h);
        Fr b0 = load_sol(Bt[k], ld, t), b1 = load_sol(Bt[k], ld, t + h);
        if (pending) {
          // entries t, t + h of the folded table come from t, t + 2h and
          // t + h, t + 3h of the table as it stands (half-size 2h)
          const Fr rr2[2] = {r, r};
          const Fr da[2] = {fr_sub(load_sol(A[k], ld, t + 2 * h), a0), fr_sub(load_sol(A[k], ld, t + 3 * h), a1)};
          const Fr db[2] = {fr_sub(load_sol(Bt[k], ld, t + 2 * h), b0), fr_sub(load_sol(Bt[k], ld, t + 3 * h), b1)};
          Fr fa[2], fb[2];
          fr_mul_n<2>(rr2, da, fa);
          fr_mul_n<2>(rr2, db, fb);
          a0 = fr_add(a0, fa[0]);
          a1 = fr_add(a1, fa[1]);
          b0 = fr_add(b0, fb[0]);
          b1 = fr_add(b1, fb[1]);
          store_sol(A[k], ld, t, a0);
          store_sol(A[k], ld, t + h, a1);
          store_sol(Bt[k], ld, t, b0);
          store_sol(Bt[k], ld, t + h, b1);
        }
        const Fr x[3] = {a0, a1, at_two(a0, a1)}, y[3] = {b0, b1, at_two(b0, b1)};
        Fr pr[3];
        fr_mul_n<3>(x, y, pr);
#pragma unroll
        for (int q = 0; q < 3; ++q) g[q] = fr_add(g[q], pr[q]);
      }
    }
    __threadfence_block();   // the folded entries, for the next sweep
    block_sum_w0<3>(g, red);
    if (wave == 0) {
      const Fr rr = round_challenge(tr, g, out, lane);
      if (lane == 0) {
        lds_put(bcast, rr);
        if (J.phase == 1)
#pragma unroll
          for (int j = 0; j < 8; ++j) J.io[kReduceIoR + 8 * rd + j] = rr.w[j];   // Montgomery, for eq(r, .)
      }
    }
    out += 96;
    __syncthreads();
    r = lds_get(bcast);
    pending = true;
  }
  // the last challenge folds the remaining pair of each table
  if (tid == 0) {
    Fr fin[kMaxClaims];
    for (uint32_t k = 0; k < K; ++k) {
      if (J.phase == 1) {
        const Fr b0 = load_sol(Bt[k], ld, 0);
        fin[k] = pending ? fr_add(b0, fr_mul(r, fr_sub(load_sol(Bt[k], ld, 1), b0))) : b0;
      } else {
        const Fr a0 = load_sol(A[k], ld, 0);
        fin[k] = fr_from_mont(pending ? fr_add(a0, fr_mul(r, fr_sub(load_sol(A[k], ld, 1), a0))) : a0);
      }
      put_canon(out + 32 * k, fin[k]);
    }
    if (J.phase == 1) {
      // t_k(r) sent and absorbed; sigma_1..sigma_K squeezed for phase 2
      absorb_k(tr, VL_LBL_RFINAL, fin, K);
      for (uint32_t k = 0; k < K; ++k) {
        const Fr sg = fr_to_mont(tr_squeeze_fixed(tr, VL_LBL_SIGMA));
#pragma unroll
        for (int j = 0; j < 8; ++j) J.io[kReduceIoSigma + 8 * k + j] = sg.w[j];
      }
#pragma unroll
      for (int i = 0; i < 8; ++i) J.io[i] = tr.h[i];
    } else {
      const Fr f1[1] = {fin[0]};
      tr_absorb_frs(tr, VL_LBL_FINAL, f1);
      if (J.digest) {
        uint8_t d[32];
        tr_to_bytes(tr, d);
        for (int i = 0; i < 32; ++i) J.digest[i] = d[i];
      }
      if (J.status) *J.status = VL_OK;
    }
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

hipError_t launch_pass1(const Pass1Job* jobs, uint32_t n_jobs, uint32_t n_blocks, hipStream_t s) {
  if (n_blocks == 0) return hipSuccess;
  hipLaunchKernelGGL(pass1_kernel, dim3(n_blocks), dim3(256), 0, s, jobs, n_jobs, n_blocks);
  return hipGetLastError();
}

hipError_t launch_mat_sweep(const RoundsJob* jobs, const MatSweep* list, uint32_t n_list, uint32_t n_blocks,
                            uint32_t round, hipStream_t s) {
  if (!n_blocks) return hipSuccess;
  hipLaunchKernelGGL(mat_sweep_kernel, dim3(n_blocks), dim3(256), 0, s, jobs, list, n_list, n_blocks, round);
  return hipGetLastError();
}

hipError_t launch_rounds(const RoundsJob* jobs, uint32_t n_jobs, hipStream_t s) {
  if (n_jobs == 0) return hipSuccess;
  hipLaunchKernelGGL(rounds_kernel, dim3(n_jobs), dim3(kRoundsBlock), 0, s, jobs);
  return hipGetLastError();
}

hipError_t launch_eval(const EvalJob* jobs, uint32_t n_jobs, hipStream_t s) {
  if (n_jobs == 0) return hipSuccess;
  hipLaunchKernelGGL(eval_kernel, dim3(n_jobs), dim3(256), 0, s, jobs);
  return hipGetLastError();
}

hipError_t launch_reduce(const ReduceJob* jobs, uint32_t n_jobs, hipStream_t s) {
  if (n_jobs == 0) return hipSuccess;
  hipLaunchKernelGGL(reduce_kernel, dim3(n_jobs), dim3(kRoundsBlock), 0, s, jobs);
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
