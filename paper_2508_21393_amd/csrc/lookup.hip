// Device kernels of the lookup argument (vl_lookup_prove).
//
// Protocol 1 proves that every entry s_i of a secret tensor lies in a public
// table T through the identity of eq. (rational-function): at a random beta,
// sum_i 1/(beta + s_i) = sum_j m_j/(beta + t_j), with m_j the multiplicity of
// t_j.  Eq. (lookup-sumcheck) turns this and the two inverse relations into
// one sum over the entries x = (x_H, x_L) of
//     alpha A eq(u, .) (S + beta) + A + (N/D) alpha^2 B eq(u_L, .) (T + beta)
//     - (N/D) B m,
// whose value is alpha + alpha^2.  Because the table is small (N rows) and
// every entry is one of its rows, A_i = B_{j(i)}: the N inverses are the only
// ones computed (a batch inversion per chunk of rows), and A is gathered.
//
//   lookup_hist_kernel   multiplicities (atomic counts) and the membership
//                        check of every entry
//   lookup_inv_kernel    Tb = T + beta, B = 1/Tb (chunked batch inversion)
//   lookup_mult_kernel   m in the field, partial sums of B m
//   lookup_prep_kernel   Sb = S + beta and A = B[row of the entry]
//   lookup_start_kernel  the constant K of the high rounds, the status
//   lookup_sweep/chal    the first rounds across the GPU, then a one-block
//                        transcript step
//   lookup_rounds_kernel the remaining rounds in one workgroup, and the
//                        final values A(r), S(r), B(r_L), T(r_L), m(r_L)
// Every table is in Montgomery form; round values are converted to
// canonical form for the proof.  The constant factors of the sum are folded
// into tables that are never sent: E' = alpha eq(u, .), EL' = c1 eq(u_L, .)
// (both built scaled by the eq kernel) and M' = c2 m (m(r_L) is recovered
// as 2^nH M'(r_L)), so a round's terms add up without further products.
#include "device.hpp"
#include "rounds_dev.hpp"
#include "sha256.hpp"

namespace vl {

namespace {

__device__ __forceinline__ int64_t lk_entry(const void* p, int dt, uint64_t i) {
  return dt == VL_I16 ? (int64_t)reinterpret_cast<const int16_t*>(p)[i]
                      : (int64_t)reinterpret_cast<const int32_t*>(p)[i];
}

// canonical field element of a signed integer
__device__ __forceinline__ Fr fr_of_int(int64_t v) {
  const uint64_t mag = v < 0 ? (uint64_t)0 - (uint64_t)v : (uint64_t)v;
  Fr r = fr_zero();
  r.w[0] = (uint32_t)mag;
  r.w[1] = (uint32_t)(mag >> 32);
  return v < 0 ? fr_neg(r) : r;
}

// Montgomery form of x + gamma y + beta (gamma, beta Montgomery)
__device__ __forceinline__ Fr compress_mont(int64_t x, int64_t y, bool two, const Fr& gamma, const Fr& beta) {
  Fr v = fr_of_int(x);
  if (two) v = fr_add(v, fr_mul(gamma, fr_of_int(y)));   // Montgomery x canonical: canonical
  return fr_add(fr_mul(v, fr_R2()), beta);
}

// limb i of p - 2 (p's low limb is 1)
__device__ __forceinline__ uint32_t pm2_limb(int i) { return i == 0 ? 0xffffffffu : (i == 1 ? 0xfffffffeu : p_limb(i)); }

// x^-1 = x^(p - 2) (Fermat), Montgomery in and out
__device__ Fr fr_inv_mont(const Fr& x) {
  Fr r = fr_R();
  for (int i = 254; i >= 0; --i) {
    r = fr_mul(r, r);
    if ((pm2_limb(i >> 5) >> (i & 31)) & 1u) r = fr_mul(r, x);
  }
  return r;
}

__device__ __forceinline__ Fr lk_fr(const uint32_t (&w)[8]) {
  Fr r;
#pragma unroll
  for (int j = 0; j < 8; ++j) r.w[j] = w[j];
  return r;
}

__device__ __forceinline__ int32_t lk_io_status(const LookupJob& J) {
  return *reinterpret_cast<volatile const int32_t*>(J.io);
}

__device__ __forceinline__ void lk_fold(const Fr& r, Fr& x0, Fr& x1, const Fr& x2, const Fr& x3) {
  const Fr rr[2] = {r, r};
  const Fr d[2] = {fr_sub(x2, x0), fr_sub(x3, x1)};
  Fr f[2];
  fr_mul_n<2>(rr, d, f);
  x0 = fr_add(x0, f[0]);
  x1 = fr_add(x1, f[1]);
}

// entries t, t + h of a table of 2h entries (4h before a pending fold,
// which is done and stored): the table's line at X = 0 and X = 1
__device__ __forceinline__ void lk_load(uint32_t* tab, uint64_t ld, uint64_t h, uint64_t t, bool fold, const Fr& r,
                                        Fr& x0, Fr& x1) {
  x0 = load_sol(tab, ld, t);
  x1 = load_sol(tab, ld, t + h);
  if (fold) {
    lk_fold(r, x0, x1, load_sol(tab, ld, t + 2 * h), load_sol(tab, ld, t + 3 * h));
    store_sol(tab, ld, t, x0);
    store_sol(tab, ld, t + h, x1);
  }
}

// the line at X, X + 1 moved on to X + 2, X + 3
__device__ __forceinline__ void lk_adv(Fr& x0, Fr& x1) {
  const Fr d = fr_sub(x1, x0);
  x0 = fr_add(x1, d);
  x1 = fr_add(x0, d);
}

__device__ __forceinline__ void lk_mul2(const Fr& x0, const Fr& x1, const Fr& y0, const Fr& y1, Fr& z0, Fr& z1) {
  const Fr a[2] = {x0, x1}, b[2] = {y0, y1};
  Fr c[2];
  fr_mul_n<2>(a, b, c);
  z0 = c[0];
  z1 = c[1];
}

// One pair t < h of a round whose variable is a high index bit: only A, Sb
// and E' = alpha eq(u, .) depend on it.  Adds alpha E A Sb + A at X = 0..3
// to g, two points at a time.  pending: fold by r first.
__device__ __forceinline__ void lk_pair_high(const LookupJob& J, uint64_t h, uint64_t t, bool pending, const Fr& r,
                                             Fr (&g)[4]) {
  const uint64_t ldD = 1ull << (J.nH + J.nL);
  Fr e0, e1, a0, a1, s0, s1;
  lk_load(J.E, ldD, h, t, pending, r, e0, e1);
  lk_load(J.A, ldD, h, t, pending, r, a0, a1);
  lk_load(J.S, ldD, h, t, pending, r, s0, s1);
#pragma unroll
  for (int half = 0; half < 2; ++half) {
    if (half) {
      lk_adv(e0, e1);
      lk_adv(a0, a1);
      lk_adv(s0, s1);
    }
    Fr p0, p1, q0, q1;
    lk_mul2(e0, e1, a0, a1, p0, p1);
    lk_mul2(p0, p1, s0, s1, q0, q1);
    g[2 * half] = fr_add(g[2 * half], fr_add(q0, a0));
    g[2 * half + 1] = fr_add(g[2 * half + 1], fr_add(q1, a1));
  }
}

// One pair of a round whose variable is a low index bit: every table.  Adds
// alpha E A Sb + A + c1 B EL Tb - c2 B m (EL' = c1 eq(u_L, .), M' = c2 m).
// pend_hi: the pending challenge bound a high bit (only A, Sb, E fold).
__device__ __forceinline__ void lk_pair_low(const LookupJob& J, uint64_t h, uint64_t t, bool pending, bool pend_hi,
                                            const Fr& r, Fr (&g)[4]) {
  lk_pair_high(J, h, t, pending, r, g);
  const uint64_t ldN = 1ull << J.nL;
  const bool fold = pending && !pend_hi;
  Fr b0, b1, l0, l1, t0, t1, m0, m1;
  lk_load(J.B, ldN, h, t, fold, r, b0, b1);
  lk_load(J.EL, ldN, h, t, fold, r, l0, l1);
  lk_load(J.T, ldN, h, t, fold, r, t0, t1);
  lk_load(J.M, ldN, h, t, fold, r, m0, m1);
#pragma unroll
  for (int half = 0; half < 2; ++half) {
    if (half) {
      lk_adv(b0, b1);
      lk_adv(l0, l1);
      lk_adv(t0, t1);
      lk_adv(m0, m1);
    }
    Fr p0, p1, q0, q1, w0, w1;
    lk_mul2(b0, b1, l0, l1, p0, p1);
    lk_mul2(p0, p1, t0, t1, q0, q1);
    lk_mul2(b0, b1, m0, m1, w0, w1);
    g[2 * half] = fr_add(g[2 * half], fr_sub(q0, w0));
    g[2 * half + 1] = fr_add(g[2 * half + 1], fr_sub(q1, w1));
  }
}

// Round rd by wave 0 (all lanes; the block totals in lane 0): a high round
// adds the constant 2^(nH - rd - 1) K; round 1 checks the guard
// g(0) + g(1) = alpha + alpha^2; the values are written canonical, absorbed
// and r squeezed (Montgomery, every lane).  Returns false, in every lane, if
// the guard fails.
__device__ __forceinline__ bool lk_round_wave(const LookupJob& J, uint32_t rd, const Fr (&g)[4], Transcript& tr,
                                              Fr& r, uint32_t lane) {
  Fr gt[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) gt[q] = readlane_fr(g[q], 0);
  if (rd < J.nH) {
    Fr k = lds_or_global_fr(J.io + kLkIoK);
    for (uint32_t i = 0; i + 1 < J.nH - rd; ++i) k = fr_double(k);
#pragma unroll
    for (int q = 0; q < 4; ++q) gt[q] = fr_add(gt[q], k);
  }
  if (rd == 0 && !fr_eq(fr_add(gt[0], gt[1]), lk_fr(J.claim))) return false;
  Fr gc[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) gc[q] = fr_from_mont(gt[q]);
  r = round_challenge_k<4>(tr, gc, J.proof + 128ull * rd, lane);
  return true;
}

// block sum of 4 elements over 256 threads into out (32 words)
__device__ __forceinline__ void lk_block_out(Fr (&g)[4], uint32_t* out) {
  __shared__ uint32_t red[4 * 8 * 4];
  block256_sum4(g, red);
  if (threadIdx.x == 0)
#pragma unroll
    for (int k = 0; k < 4; ++k)
#pragma unroll
      for (int j = 0; j < 8; ++j) out[k * 8 + j] = g[k].w[j];
}

template <typename Get>
__device__ __forceinline__ uint32_t lk_find(Get begin_of, uint32_t n, uint32_t blk) {
  uint32_t lo = 0, hi = n;
  while (hi - lo > 1) {
    const uint32_t mid = (lo + hi) >> 1;
    if (begin_of(mid) <= blk) lo = mid; else hi = mid;
  }
  return lo;
}

}  // namespace

// Multiplicities and membership: one thread per entry.  An entry outside
// the table (or, with two columns, whose second value differs from the
// table's) sets the job's flag; the padding entries are counted on row 0.
__global__ void __launch_bounds__(256) lookup_hist_kernel(const LookupJob* __restrict__ jobs, uint32_t n_jobs,
                                                          uint32_t n_blocks) {
  const uint32_t blk = blockIdx.x;
  if (blk >= n_blocks) return;
  const LookupJob& J = jobs[lk_find([&](uint32_t k) { return jobs[k].hist_begin; }, n_jobs, blk)];
  const uint64_t i = (uint64_t)(blk - J.hist_begin) * 256 + threadIdx.x;
  const uint64_t N = 1ull << J.nL, Dp = 1ull << (J.nH + J.nL);
  if (i == 0 && Dp > J.D) atomicAdd(J.cnt, (uint32_t)(Dp - J.D));
  if (i >= J.D) return;
  const int64_t j = lk_entry(J.x, J.dtype, i) - J.t0;
  bool ok = j >= 0 && j < (int64_t)N;
  if (ok && J.y) ok = lk_entry(J.y, J.dtype_y, i) == (int64_t)J.tb[j];
  if (ok) atomicAdd(J.cnt + j, 1u);
  else *reinterpret_cast<volatile int32_t*>(J.flag) = 1;
}

// Table rows, in two kernels.  lookup_inv_kernel, kLookupInvChunk rows per
// thread: Tb_j = t0 + j + gamma tb_j + beta and
// B_j = 1/Tb_j by a batch inversion over the chunk (prefix products, one
// inversion, back-substitution); it reads no count, so it runs beside the
// count kernel.  A zero Tb_j (beta at a pole, probability N/p) sets the
// flag.  lookup_mult_kernel, after the counts, one row per thread:
// M'_j = c2 m_j and per block the sum of B_j M'_j.
__global__ void __launch_bounds__(256) lookup_inv_kernel(const LookupJob* __restrict__ jobs, uint32_t n_jobs,
                                                         uint32_t n_blocks) {
  const uint32_t blk = blockIdx.x;
  if (blk >= n_blocks) return;
  const LookupJob& J = jobs[lk_find([&](uint32_t k) { return jobs[k].tab_begin; }, n_jobs, blk)];
  const uint64_t N = 1ull << J.nL;
  const uint64_t ch = (uint64_t)(blk - J.tab_begin) * 256 + threadIdx.x;
  const uint64_t j0 = ch * kLookupInvChunk, j1 = min(j0 + kLookupInvChunk, N);
  if (j0 >= N) return;
  const Fr gamma = lk_fr(J.gamma), beta = lk_fr(J.beta);
  Fr acc = fr_R();
  for (uint64_t j = j0; j < j1; ++j) {
    const Fr tb = compress_mont(J.t0 + (int64_t)j, J.tb ? J.tb[j] : 0, J.tb != nullptr, gamma, beta);
    if (fr_is_zero(tb)) *reinterpret_cast<volatile int32_t*>(J.flag) = 1;
    store_sol(J.T, N, j, tb);
    store_sol(J.B, N, j, acc);      // prefix product, replaced below
    acc = fr_mul(acc, tb);
  }
  Fr inv = fr_inv_mont(acc);
  for (uint64_t jj = j1; jj > j0; --jj) {
    const uint64_t j = jj - 1;
    const Fr b = fr_mul(inv, load_sol(J.B, N, j));
    inv = fr_mul(inv, load_sol(J.T, N, j));
    store_sol(J.B, N, j, b);
  }
}

__global__ void __launch_bounds__(256) lookup_mult_kernel(const LookupJob* __restrict__ jobs, uint32_t n_jobs,
                                                          uint32_t n_blocks) {
  const uint32_t blk = blockIdx.x;
  if (blk >= n_blocks) return;
  const LookupJob& J = jobs[lk_find([&](uint32_t k) { return jobs[k].mult_begin; }, n_jobs, blk)];
  const uint64_t N = 1ull << J.nL;
  const uint64_t j = (uint64_t)(blk - J.mult_begin) * 256 + threadIdx.x;
  Fr g[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) g[k] = fr_zero();
  if (j < N) {
    Fr m = fr_zero();
    m.w[0] = J.cnt[j];
    m = fr_mul(fr_mul(lk_fr(J.c2), fr_R2()), m);   // c2 m in Montgomery form (c2 R^2 times the count)
    store_sol(J.M, N, j, m);
    g[0] = fr_mul(load_sol(J.B, N, j), m);
  }
  lk_block_out(g, J.kpart + (uint64_t)(blk - J.mult_begin) * 32);
}

// Entries: Sb_i = x_i + gamma y_i + beta and A_i = B_{x_i - t0} (padding
// entries are the table's first row).  One thread per padded entry.
__global__ void __launch_bounds__(256) lookup_prep_kernel(const LookupJob* __restrict__ jobs, uint32_t n_jobs,
                                                          uint32_t n_blocks) {
  const uint32_t blk = blockIdx.x;
  if (blk >= n_blocks) return;
  const LookupJob& J = jobs[lk_find([&](uint32_t k) { return jobs[k].prep_begin; }, n_jobs, blk)];
  const uint64_t i = (uint64_t)(blk - J.prep_begin) * 256 + threadIdx.x;
  const uint64_t N = 1ull << J.nL, Dp = 1ull << (J.nH + J.nL);
  if (i >= Dp) return;
  const bool two = J.y != nullptr;
  int64_t x = J.t0, y = two ? J.tb[0] : 0;
  if (i < J.D) {
    x = lk_entry(J.x, J.dtype, i);
    if (two) y = lk_entry(J.y, J.dtype_y, i);
  }
  int64_t j = x - J.t0;
  j = j < 0 ? 0 : (j >= (int64_t)N ? (int64_t)N - 1 : j);   // out-of-table entries have set the flag
  store_sol(J.S, Dp, i, compress_mont(x, y, two, lk_fr(J.gamma), lk_fr(J.beta)));
  store_sol(J.A, Dp, i, load_sol(J.B, N, (uint64_t)j));
}

// Status and the constant of the high rounds: K = c1 - sum_j B_j M'_j with
// M' = c2 m (the table rows' terms summed over x_L; sum_j eq(u_L, j) = 1 and
// B_j Tb_j = 1).
__global__ void __launch_bounds__(64) lookup_start_kernel(const LookupJob* __restrict__ jobs) {
  const LookupJob& J = jobs[blockIdx.x];
  const uint32_t lane = threadIdx.x;
  if (*reinterpret_cast<volatile const int32_t*>(J.flag)) {
    if (lane == 0) {
      J.io[0] = (uint32_t)VL_ERR_FALSE_STATEMENT;
      *J.status = VL_ERR_FALSE_STATEMENT;
    }
    return;
  }
  Fr s[1];
  s[0] = fr_zero();
  for (uint32_t i = lane; i < J.nkparts; i += kWave) s[0] = fr_add(s[0], lds_or_global_fr(J.kpart + 32ull * i));
  wave_sum<1>(s, kWave);
  if (lane == 0) {
    const Fr K = fr_sub(lk_fr(J.c1), s[0]);
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      J.io[kLkIoK + i] = K.w[i];
      J.io[kLkIoState + i] = J.st[i];
    }
    J.io[0] = (uint32_t)VL_OK;
  }
}

// One wide round over every job of its list (kLookupSweepPairs pairs per
// 256-thread block), high or low index bit (separate kernels: the high one
// keeps three tables live).
template <bool LOW>
__global__ void __launch_bounds__(256) lookup_sweep_kernel(const LookupJob* __restrict__ jobs,
                                                           const LookupSweep* __restrict__ list, uint32_t n_list,
                                                           uint32_t n_blocks, uint32_t rd) {
  const uint32_t blk = blockIdx.x;
  if (blk >= n_blocks) return;
  const LookupSweep& S = list[lk_find([&](uint32_t k) { return list[k].block_begin; }, n_list, blk)];
  const LookupJob& J = jobs[S.job];
  if (lk_io_status(J) != VL_OK) return;
  const uint32_t n = J.nH + J.nL;
  const uint64_t h = 1ull << (n - 1 - rd);
  const uint64_t base = (uint64_t)(blk - S.block_begin) * kLookupSweepPairs;
  Fr g[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) g[k] = fr_zero();
  const Fr r = rd > 0 ? lds_or_global_fr(J.io + kLkIoR) : fr_zero();
#pragma unroll 1
  for (uint64_t t = base + threadIdx.x; t < h && t < base + kLookupSweepPairs; t += 256) {
    if (LOW) lk_pair_low(J, h, t, rd > 0, rd > 0 && rd - 1 < J.nH, r, g);
    else lk_pair_high(J, h, t, rd > 0, r, g);
  }
  lk_block_out(g, J.part + (uint64_t)(blk - S.block_begin) * 32);
}

// The transcript step after a wide round, one 256-thread block per job.
__global__ void __launch_bounds__(256) lookup_chal_kernel(const LookupJob* __restrict__ jobs,
                                                          const LookupSweep* __restrict__ list, uint32_t rd) {
  const LookupJob& J = jobs[list[blockIdx.x].job];
  const uint32_t tid = threadIdx.x, lane = tid & 63u;
  if (lk_io_status(J) != VL_OK) return;
  const uint32_t n = J.nH + J.nL;
  const uint64_t h = 1ull << (n - 1 - rd);
  const uint32_t nblocks = (uint32_t)((h + kLookupSweepPairs - 1) / kLookupSweepPairs);
  __shared__ uint32_t red[4 * 8 * 4];
  Fr g[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) g[k] = fr_zero();
  for (uint32_t i = tid; i < nblocks; i += 256)
#pragma unroll
    for (int k = 0; k < 4; ++k) g[k] = fr_add(g[k], lds_or_global_fr(J.part + 32ull * i + 8 * k));
  block256_sum4(g, red);
  if (tid >= 64) return;
  Transcript tr;
#pragma unroll
  for (int i = 0; i < 8; ++i) tr.h[i] = J.io[kLkIoState + i];
  Fr r;
  if (!lk_round_wave(J, rd, g, tr, r, lane)) {
    if (lane == 0) {
      J.io[0] = (uint32_t)VL_ERR_FALSE_STATEMENT;
      *J.status = VL_ERR_FALSE_STATEMENT;
    }
    return;
  }
  if (lane == 0)
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      J.io[kLkIoState + i] = tr.h[i];
      J.io[kLkIoR + i] = r.w[i];
    }
}

// The remaining rounds in one workgroup of 256 threads (one wave per SIMD,
// so the pair arithmetic and the hashing lane keep their registers), then
// the final values.
__global__ void __launch_bounds__(256) lookup_rounds_kernel(const LookupJob* __restrict__ jobs) {
  const LookupJob& J = jobs[blockIdx.x];
  __shared__ uint32_t red[4 * 8 * 4];
  __shared__ uint32_t bcast[8];
  __shared__ uint32_t dead_s;
  const uint32_t tid = threadIdx.x, NT = blockDim.x;
  const int32_t st0 = lk_io_status(J);
  if (st0 != VL_OK) {
    if (tid == 0) *J.status = st0;
    return;
  }
  const uint32_t n = J.nH + J.nL;
  Transcript tr;
#pragma unroll
  for (int i = 0; i < 8; ++i) tr.h[i] = J.io[kLkIoState + i];
  bool pending = J.wide > 0;
  Fr r = pending ? lds_or_global_fr(J.io + kLkIoR) : fr_zero();
  for (uint32_t rd = J.wide; rd < n; ++rd) {
    const uint64_t h = 1ull << (n - 1 - rd);
    Fr g[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) g[k] = fr_zero();
    if (rd < J.nH) {
#pragma unroll 1
      for (uint64_t t = tid; t < h; t += NT) lk_pair_high(J, h, t, pending, r, g);
    } else {
      const bool pend_hi = pending && rd - 1 < J.nH;
#pragma unroll 1
      for (uint64_t t = tid; t < h; t += NT) lk_pair_low(J, h, t, pending, pend_hi, r, g);
    }
    __threadfence_block();   // the folded entries, for the next sweep
    block256_sum4(g, red);
    if (tid < 64) {
      Fr rr;
      const bool ok = lk_round_wave(J, rd, g, tr, rr, tid);
      if (tid == 0) {
        dead_s = ok ? 0 : 1;
        if (ok) lds_put(bcast, rr);
        else *J.status = VL_ERR_FALSE_STATEMENT;
      }
    }
    __syncthreads();
    if (dead_s) return;
    r = lds_get(bcast);
    pending = true;
  }
  if (tid != 0) return;
  const uint64_t ldD = 1ull << n, ldN = 1ull << J.nL;
  Fr v[7];
  uint32_t* const tabs[7] = {J.A, J.S, J.E, J.B, J.T, J.M, J.EL};
  for (int k = 0; k < 7; ++k) {
    const uint64_t ld = k < 3 ? ldD : ldN;
    v[k] = load_sol(tabs[k], ld, 0);
    // the last challenge bound a high bit (no low rounds) or a low bit
    const bool folds = pending && (k < 3 || n - 1 >= J.nH);
    if (folds) v[k] = fr_add(v[k], fr_mul(r, fr_sub(load_sol(tabs[k], ld, 1), v[k])));
  }
  if (n == 0) {
    // no rounds (one entry, one row): the guard is the summand itself
    const Fr f = fr_add(fr_add(fr_mul(fr_mul(v[2], v[0]), v[1]), v[0]),
                        fr_sub(fr_mul(fr_mul(v[3], v[6]), v[4]), fr_mul(v[3], v[5])));
    if (!fr_eq(f, lk_fr(J.claim))) {
      *J.status = VL_ERR_FALSE_STATEMENT;
      return;
    }
  }
  // m(r_L) = M'(r_L) / c2 = 2^nH M'(r_L)
  Fr mv = v[5];
  for (uint32_t i = 0; i < J.nH; ++i) mv = fr_double(mv);
  const Fr beta = lk_fr(J.beta);
  const Fr fin[5] = {fr_from_mont(v[0]), fr_from_mont(fr_sub(v[1], beta)), fr_from_mont(v[3]),
                     fr_from_mont(fr_sub(v[4], beta)), fr_from_mont(mv)};
  uint8_t* out = J.proof + 128ull * n;
  for (int k = 0; k < 5; ++k) put_canon(out + 32 * k, fin[k]);
  tr_absorb_frs(tr, VL_LBL_FINAL, fin);
  if (J.digest) {
    uint8_t d[32];
    tr_to_bytes(tr, d);
    for (int i = 0; i < 32; ++i) J.digest[i] = d[i];
  }
  *J.status = VL_OK;
}

hipError_t launch_lookup_hist(const LookupJob* jobs, uint32_t n_jobs, uint32_t n_blocks, hipStream_t s) {
  if (n_blocks == 0) return hipSuccess;
  hipLaunchKernelGGL(lookup_hist_kernel, dim3(n_blocks), dim3(256), 0, s, jobs, n_jobs, n_blocks);
  return hipGetLastError();
}

hipError_t launch_lookup_inv(const LookupJob* jobs, uint32_t n_jobs, uint32_t n_blocks, hipStream_t s) {
  if (n_blocks == 0) return hipSuccess;
  hipLaunchKernelGGL(lookup_inv_kernel, dim3(n_blocks), dim3(256), 0, s, jobs, n_jobs, n_blocks);
  return hipGetLastError();
}

hipError_t launch_lookup_mult(const LookupJob* jobs, uint32_t n_jobs, uint32_t n_blocks, hipStream_t s) {
  if (n_blocks == 0) return hipSuccess;
  hipLaunchKernelGGL(lookup_mult_kernel, dim3(n_blocks), dim3(256), 0, s, jobs, n_jobs, n_blocks);
  return hipGetLastError();
}

hipError_t launch_lookup_prep(const LookupJob* jobs, uint32_t n_jobs, uint32_t n_blocks, hipStream_t s) {
  if (n_blocks == 0) return hipSuccess;
  hipLaunchKernelGGL(lookup_prep_kernel, dim3(n_blocks), dim3(256), 0, s, jobs, n_jobs, n_blocks);
  return hipGetLastError();
}

hipError_t launch_lookup_start(const LookupJob* jobs, uint32_t n_jobs, hipStream_t s) {
  if (n_jobs == 0) return hipSuccess;
  hipLaunchKernelGGL(lookup_start_kernel, dim3(n_jobs), dim3(kWave), 0, s, jobs);
  return hipGetLastError();
}

hipError_t launch_lookup_sweep(const LookupJob* jobs, const LookupSweep* list, uint32_t n_list, uint32_t n_blocks,
                               uint32_t round, bool low, hipStream_t s) {
  if (n_blocks == 0) return hipSuccess;
  if (low)
    hipLaunchKernelGGL(lookup_sweep_kernel<true>, dim3(n_blocks), dim3(256), 0, s, jobs, list, n_list, n_blocks, round);
  else
    hipLaunchKernelGGL(lookup_sweep_kernel<false>, dim3(n_blocks), dim3(256), 0, s, jobs, list, n_list, n_blocks, round);
  return hipGetLastError();
}

hipError_t launch_lookup_chal(const LookupJob* jobs, const LookupSweep* list, uint32_t n_list, uint32_t round,
                              hipStream_t s) {
  if (n_list == 0) return hipSuccess;
  hipLaunchKernelGGL(lookup_chal_kernel, dim3(n_list), dim3(256), 0, s, jobs, list, round);
  return hipGetLastError();
}

hipError_t launch_lookup_rounds(const LookupJob* jobs, uint32_t n_jobs, hipStream_t s) {
  if (n_jobs == 0) return hipSuccess;
  hipLaunchKernelGGL(lookup_rounds_kernel, dim3(n_jobs), dim3(256), 0, s, jobs);
  return hipGetLastError();
}

}  // namespace vl
