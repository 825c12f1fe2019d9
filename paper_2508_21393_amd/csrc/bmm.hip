// Device kernels of the per-head batched matmul sumcheck (vl_bmm_prove).
//
// Attention multiplies one pair of matrices per head (Sec. III-A, eq. (att));
// the H products C_h = A_h B_h are proved with one sumcheck over the head
// variables and the inner variables of
//     C~(rho, u, v) = sum_{h, w} eq(rho, h) A~(h, u, w) B~(h, w, v),
// the multilinear extension of eq. (MLE) over (head, row, column) indices of
// the 3-D tensors, head index most significant.  Head rounds come first:
// their summand is a product of three multilinear tables (E = eq(rho, .), a,
// b), so each round polynomial has degree 3 and is sent as g(0..3).  Once the
// head variables are bound E is one value e*, and the inner rounds are the
// plain degree-2 rounds of eq. (zk-mle-matmul) scaled by e*.
//
//   bmm_start_kernel   the claim c from its pass-1 partials, absorbed
//   bmm_sweep_kernel   one round over large tables across the GPU: fold by
//                      the previous challenge and the round's partial sums
//   bmm_chal_kernel    one block per job: the round values, the prover guard
//                      (round 1: g(0) + g(1) = c), transcript, challenge,
//                      and the fold of E in a head round
//   bmm_rounds_kernel  one workgroup per job: the remaining rounds and the
//                      final values a_final = A~(r_h, u, r_w),
//                      b_final = B~(r_h, r_w, v)
#include "device.hpp"
#include "rounds_dev.hpp"
#include "sha256.hpp"

namespace vl {

namespace {

// proof byte offset of round rd's values: c, then 4 values per head round
// and 3 per inner round
__device__ __forceinline__ uint64_t bmm_round_off(const BmmJob& J, uint32_t rd) {
  const uint32_t hr = rd < J.nh ? rd : J.nh;
  return 32ull * (1 + 4ull * hr + 3ull * (rd - hr));
}

__device__ __forceinline__ int32_t bmm_io_status(const BmmJob& J) {
  return *reinterpret_cast<volatile const int32_t*>(J.io);
}

// x0 + r (x2 - x0) and x1 + r (x3 - x1): one step of folding by r, the
// entries t, t + h of the folded table from t, t + 2h and t + h, t + 3h
__device__ __forceinline__ void fold_pair(const Fr& r, Fr& x0, Fr& x1, const Fr& x2, const Fr& x3) {
  const Fr rr[2] = {r, r};
  const Fr d[2] = {fr_sub(x2, x0), fr_sub(x3, x1)};
  Fr f[2];
  fr_mul_n<2>(rr, d, f);
  x0 = fr_add(x0, f[0]);
  x1 = fr_add(x1, f[1]);
}

// a head round's terms of one pair: E_X a_X b_X at X = 0, 1, 2, 3, where each
// table is the line x_X = x0 + X (x1 - x0) through the pair's entries.  E and
// a are in Montgomery form and b canonical, so each term is canonical.
__device__ __forceinline__ void head_terms(const Fr& e0, const Fr& e1, const Fr& a0, const Fr& a1, const Fr& b0,
                                           const Fr& b1, Fr (&g)[4]) {
  const Fr de = fr_sub(e1, e0), da = fr_sub(a1, a0), db = fr_sub(b1, b0);
  const Fr e2 = fr_add(e1, de), a2 = fr_add(a1, da), b2 = fr_add(b1, db);
  const Fr e3 = fr_add(e2, de), a3 = fr_add(a2, da), b3 = fr_add(b2, db);
  Fr ea[4], t[4];
  {
    const Fr x[2] = {e0, e1}, y[2] = {a0, a1};
    Fr r[2];
    fr_mul_n<2>(x, y, r);
    ea[0] = r[0];
    ea[1] = r[1];
  }
  {
    const Fr x[2] = {e2, e3}, y[2] = {a2, a3};
    Fr r[2];
    fr_mul_n<2>(x, y, r);
    ea[2] = r[0];
    ea[3] = r[1];
  }
  {
    const Fr x[2] = {ea[0], ea[1]}, y[2] = {b0, b1};
    Fr r[2];
    fr_mul_n<2>(x, y, r);
    t[0] = r[0];
    t[1] = r[1];
  }
  {
    const Fr x[2] = {ea[2], ea[3]}, y[2] = {b2, b3};
    Fr r[2];
    fr_mul_n<2>(x, y, r);
    t[2] = r[0];
    t[3] = r[1];
  }
#pragma unroll
  for (int k = 0; k < 4; ++k) g[k] = fr_add(g[k], t[k]);
}

// an inner round's terms of one pair: a_X b_X at X = 0, 1, 2
__device__ __forceinline__ void inner_terms(const Fr& a0, const Fr& a1, const Fr& b0, const Fr& b1, Fr (&g)[4]) {
  const Fr x[3] = {a0, a1, at_two(a0, a1)}, y[3] = {b0, b1, at_two(b0, b1)};
  Fr pr[3];
  fr_mul_n<3>(x, y, pr);
#pragma unroll
  for (int k = 0; k < 3; ++k) g[k] = fr_add(g[k], pr[k]);
}

// one pair t < h of round rd: the pending fold by r (tables of 4h entries),
// then the round's terms
__device__ __forceinline__ void bmm_pair(const BmmJob& J, uint64_t ld, uint64_t h, uint64_t t, bool head,
                                         bool pending, const Fr& r, Fr (&g)[4]) {
  Fr a0 = load_sol(J.a, ld, t), a1 = load_sol(J.a, ld, t + h);
  Fr b0 = load_sol(J.b, ld, t), b1 = load_sol(J.b, ld, t + h);
  if (pending) {
    fold_pair(r, a0, a1, load_sol(J.a, ld, t + 2 * h), load_sol(J.a, ld, t + 3 * h));
    fold_pair(r, b0, b1, load_sol(J.b, ld, t + 2 * h), load_sol(J.b, ld, t + 3 * h));
    store_sol(J.a, ld, t, a0);
    store_sol(J.a, ld, t + h, a1);
    store_sol(J.b, ld, t, b0);
    store_sol(J.b, ld, t + h, b1);
  }
  if (head) {
    const uint64_t eld = 1ull << J.nh;
    head_terms(load_sol(J.E, eld, t >> J.n1), load_sol(J.E, eld, (t + h) >> J.n1), a0, a1, b0, b1, g);
  } else {
    inner_terms(a0, a1, b0, b1, g);
  }
}

// an inner round's values times e* = E[0] (the folded eq(rho, .)), uniform
__device__ __forceinline__ void bmm_scale_inner(const BmmJob& J, bool head, Fr (&g)[4]) {
  if (head) return;
  const Fr es = load_sol(J.E, 1ull << J.nh, 0);
  const Fr x[3] = {es, es, es}, y[3] = {g[0], g[1], g[2]};
  Fr s[3];
  fr_mul_n<3>(x, y, s);
  g[0] = s[0];
  g[1] = s[1];
  g[2] = s[2];
}

// round rd's values written to the proof, absorbed ("round", four values in a
// head round, three in an inner round) and r squeezed, by wave 0
__device__ __forceinline__ Fr bmm_round_msg(const BmmJob& J, uint32_t rd, bool head, const Fr (&g)[4],
                                            Transcript& tr, uint32_t lane) {
  uint8_t* out = J.proof + bmm_round_off(J, rd);
  if (head) {
    const Fr m[4] = {g[0], g[1], g[2], g[3]};
    return round_challenge_k<4>(tr, m, out, lane);
  }
  const Fr m[3] = {g[0], g[1], g[2]};
  return round_challenge_k<3>(tr, m, out, lane);
}

}  // namespace

// The claim c = C~(rho, u, v) from its pass-1 partials; c is written as the
// first proof element and absorbed.  One wave per job.
__global__ void __launch_bounds__(64) bmm_start_kernel(const BmmJob* __restrict__ jobs) {
  const BmmJob& J = jobs[blockIdx.x];
  const uint32_t lane = threadIdx.x;
  if (J.err && *(volatile const int32_t*)J.err) {
    if (lane == 0) {
      J.io[0] = (uint32_t)VL_ERR_RANGE;
      *J.status = VL_ERR_RANGE;
    }
    return;
  }
  Fr c[1];
  c[0] = fr_zero();
  for (uint32_t i = lane; i < J.c_nparts; i += kWave) c[0] = fr_add(c[0], lds_or_global_fr(J.c_part + 24ull * i));
  wave_sum<1>(c, kWave);
  if (lane == 0) {
    put_canon(J.proof, c[0]);
    Transcript tr;
#pragma unroll
    for (int i = 0; i < 8; ++i) tr.h[i] = J.st[i];
    const Fr cc[1] = {c[0]};
    tr_absorb_frs(tr, VL_LBL_CLAIM, cc);
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      J.io[kBmmIoState + i] = tr.h[i];
      J.io[kBmmIoC + i] = c[0].w[i];
    }
    J.io[0] = (uint32_t)VL_OK;
  }
}

// One wide round: every job of the round's list, kBmmSweepPairs pairs per
// block (one per thread).  Round rd > 0 first folds the tables by the
// previous challenge (read from io), in place.  Each block writes the sums
// of its pairs' terms (4 elements) to the job's partials.
__global__ void __launch_bounds__(256) bmm_sweep_kernel(const BmmJob* __restrict__ jobs,
                                                        const BmmSweep* __restrict__ list, uint32_t n_list,
                                                        uint32_t n_blocks, uint32_t rd) {
  const uint32_t blk = blockIdx.x;
  if (blk >= n_blocks) return;
  uint32_t lo = 0, hi = n_list;
  while (hi - lo > 1) {
    const uint32_t mid = (lo + hi) >> 1;
    if (list[mid].block_begin <= blk) lo = mid; else hi = mid;
  }
  const BmmSweep& S = list[lo];
  const BmmJob& J = jobs[S.job];
  if (bmm_io_status(J) != VL_OK) return;
  const uint32_t nv = J.nh + J.n1;
  const uint64_t ld = 1ull << nv, h = 1ull << (nv - 1 - rd);
  const uint64_t base = (uint64_t)(blk - S.block_begin) * kBmmSweepPairs;
  const bool head = rd < J.nh;
  Fr g[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) g[k] = fr_zero();
  {
    Fr r = fr_zero();
    if (rd > 0) r = lds_or_global_fr(J.io + kBmmIoR);
#pragma unroll 1
    for (uint64_t t = base + threadIdx.x; t < h && t < base + kBmmSweepPairs; t += 256)
      bmm_pair(J, ld, h, t, head, rd > 0, r, g);
  }
  __shared__ uint32_t red[4 * 8 * 4];
  block256_sum4(g, red);
  const uint32_t lane = threadIdx.x & 63u;
  if (threadIdx.x < 64) {
    if (lane == 0) {
      uint32_t* o = J.part + (uint64_t)(blk - S.block_begin) * 32;
#pragma unroll
      for (int k = 0; k < 4; ++k)
#pragma unroll
        for (int j = 0; j < 8; ++j) o[k * 8 + j] = g[k].w[j];
    }
  }
}

// The transcript step after a wide round, one 256-thread block per job:
// the partials added, an inner round's values scaled by e* = E[0], the
// prover guard in round 1, the values written and absorbed by wave 0, r
// squeezed (kept in io in Montgomery form for the next fold), and in a head
// round E folded by r.
__global__ void __launch_bounds__(256) bmm_chal_kernel(const BmmJob* __restrict__ jobs,
                                                       const BmmSweep* __restrict__ list, uint32_t rd) {
  const BmmJob& J = jobs[list[blockIdx.x].job];
  const uint32_t tid = threadIdx.x, lane = tid & 63u;
  if (bmm_io_status(J) != VL_OK) return;
  const uint32_t nv = J.nh + J.n1;
  const uint64_t h = 1ull << (nv - 1 - rd);
  const uint32_t nblocks = (uint32_t)((h + kBmmSweepPairs - 1) / kBmmSweepPairs);
  const bool head = rd < J.nh;
  __shared__ uint32_t red[4 * 8 * 4];
  __shared__ uint32_t bcast[8];
  __shared__ uint32_t dead_s;
  Fr g[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) g[k] = fr_zero();
  for (uint32_t i = tid; i < nblocks; i += 256)
#pragma unroll
    for (int k = 0; k < 4; ++k) g[k] = fr_add(g[k], lds_or_global_fr(J.part + 32ull * i + 8 * k));
  block256_sum4(g, red);
  if (tid < 64) {
    Fr gt[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) gt[k] = readlane_fr(g[k], 0);
    bmm_scale_inner(J, head, gt);
    const bool dead = rd == 0 && !fr_eq(fr_add(gt[0], gt[1]), lds_or_global_fr(J.io + kBmmIoC));
    if (dead) {
      if (lane == 0) {
        J.io[0] = (uint32_t)VL_ERR_FALSE_STATEMENT;
        *J.status = VL_ERR_FALSE_STATEMENT;
        dead_s = 1;
      }
    } else {
      Transcript tr;
#pragma unroll
      for (int i = 0; i < 8; ++i) tr.h[i] = J.io[kBmmIoState + i];
      const Fr r = bmm_round_msg(J, rd, head, gt, tr, lane);
      if (lane == 0) {
#pragma unroll
        for (int i = 0; i < 8; ++i) {
          J.io[kBmmIoState + i] = tr.h[i];
          J.io[kBmmIoR + i] = r.w[i];
        }
        lds_put(bcast, r);
        dead_s = 0;
      }
    }
  }
  __syncthreads();
  if (dead_s || !head) return;
  const Fr r = lds_get(bcast);
  const uint64_t eld = 1ull << J.nh, hh = 1ull << (J.nh - 1 - rd);
  for (uint64_t t = tid; t < hh; t += 256) {
    const Fr e0 = load_sol(J.E, eld, t);
    store_sol(J.E, eld, t, fr_add(e0, fr_mul(r, fr_sub(load_sol(J.E, eld, t + hh), e0))));
  }
}

// The rounds left after the wide ones, one workgroup per job, the tables in
// global memory: every round folds by the previous challenge in the same
// sweep that sums its pairs (each thread reads and writes only its own
// entries); wave 0's lane 0 runs the transcript.  Then the final values.
__global__ void __launch_bounds__(kRoundsBlock) bmm_rounds_kernel(const BmmJob* __restrict__ jobs) {
  const BmmJob& J = jobs[blockIdx.x];
  __shared__ uint32_t red[4 * 8 * (kRoundsBlock / kWave)];
  __shared__ uint32_t bcast[8];
  __shared__ uint32_t dead_s;
  const uint32_t tid = threadIdx.x, NT = blockDim.x;
  const uint32_t wave = tid >> 6, lane = tid & 63u;
  const int32_t st0 = bmm_io_status(J);
  if (st0 != VL_OK) {
    if (tid == 0) *J.status = st0;
    return;
  }
  const uint32_t nv = J.nh + J.n1;
  const uint64_t ld = 1ull << nv, eld = 1ull << J.nh;
  Transcript tr;
#pragma unroll
  for (int i = 0; i < 8; ++i) tr.h[i] = J.io[kBmmIoState + i];
  bool pending = J.wide > 0;
  Fr r = pending ? lds_or_global_fr(J.io + kBmmIoR) : fr_zero();
  for (uint32_t rd = J.wide; rd < nv; ++rd) {
    const uint64_t h = 1ull << (nv - 1 - rd);
    const bool head = rd < J.nh;
    Fr g[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) g[k] = fr_zero();
#pragma unroll 1
    for (uint64_t t = tid; t < h; t += NT) bmm_pair(J, ld, h, t, head, pending, r, g);
    __threadfence_block();   // the folded entries, for the next sweep
    block_sum_w0<4>(g, red);
    if (wave == 0) {
      Fr gt[4];
#pragma unroll
      for (int k = 0; k < 4; ++k) gt[k] = readlane_fr(g[k], 0);
      bmm_scale_inner(J, head, gt);
      if (rd == 0 && !fr_eq(fr_add(gt[0], gt[1]), lds_or_global_fr(J.io + kBmmIoC))) {
        if (lane == 0) {
          dead_s = 1;
          *J.status = VL_ERR_FALSE_STATEMENT;
        }
      } else {
        const Fr rr = bmm_round_msg(J, rd, head, gt, tr, lane);
        if (lane == 0) {
          dead_s = 0;
          lds_put(bcast, rr);
        }
      }
    }
    __syncthreads();
    if (dead_s) return;
    r = lds_get(bcast);
    pending = true;
    if (head) {
      const uint64_t hh = 1ull << (J.nh - 1 - rd);
      for (uint64_t t = tid; t < hh; t += NT) {
        const Fr e0 = load_sol(J.E, eld, t);
        store_sol(J.E, eld, t, fr_add(e0, fr_mul(r, fr_sub(load_sol(J.E, eld, t + hh), e0))));
      }
      __threadfence_block();
      __syncthreads();
    }
  }
  if (tid != 0) return;
  // the last challenge folds the remaining pair of each table
  Fr af = load_sol(J.a, ld, 0), bf = load_sol(J.b, ld, 0);
  if (pending) {
    af = fr_add(af, fr_mul(r, fr_sub(load_sol(J.a, ld, 1), af)));
    bf = fr_add(bf, fr_mul(r, fr_sub(load_sol(J.b, ld, 1), bf)));
  } else if (!fr_eq(fr_mul(fr_mul(load_sol(J.E, eld, 0), af), bf), lds_or_global_fr(J.io + kBmmIoC))) {
    // no rounds at all (one head, inner dimension 1): the guard is e a b = c
    *J.status = VL_ERR_FALSE_STATEMENT;
    return;
  }
  const Fr fin[2] = {fr_from_mont(af), bf};
  uint8_t* out = J.proof + bmm_round_off(J, nv);
  put_canon(out, fin[0]);
  put_canon(out + 32, fin[1]);
  tr_absorb_frs(tr, VL_LBL_FINAL, fin);
  if (J.digest) {
    uint8_t d[32];
    tr_to_bytes(tr, d);
    for (int i = 0; i < 32; ++i) J.digest[i] = d[i];
  }
  *J.status = VL_OK;
}

hipError_t launch_bmm_start(const BmmJob* jobs, uint32_t n_jobs, hipStream_t s) {
  if (n_jobs == 0) return hipSuccess;
  hipLaunchKernelGGL(bmm_start_kernel, dim3(n_jobs), dim3(kWave), 0, s, jobs);
  return hipGetLastError();
}

hipError_t launch_bmm_sweep(const BmmJob* jobs, const BmmSweep* list, uint32_t n_list, uint32_t n_blocks,
                            uint32_t round, hipStream_t s) {
  if (n_blocks == 0) return hipSuccess;
  hipLaunchKernelGGL(bmm_sweep_kernel, dim3(n_blocks), dim3(256), 0, s, jobs, list, n_list, n_blocks, round);
  return hipGetLastError();
}

hipError_t launch_bmm_chal(const BmmJob* jobs, const BmmSweep* list, uint32_t n_list, uint32_t round,
                           hipStream_t s) {
  if (n_list == 0) return hipSuccess;
  hipLaunchKernelGGL(bmm_chal_kernel, dim3(n_list), dim3(256), 0, s, jobs, list, round);
  return hipGetLastError();
}

hipError_t launch_bmm_rounds(const BmmJob* jobs, uint32_t n_jobs, hipStream_t s) {
  if (n_jobs == 0) return hipSuccess;
  hipLaunchKernelGGL(bmm_rounds_kernel, dim3(n_jobs), dim3(kRoundsBlock), 0, s, jobs);
  return hipGetLastError();
}

}  // namespace vl
