// Lookup arguments: planning, proving and the host verifier
// (vl_lookup_prove, vl_lookup_verify).
//
// Protocol 1 (Sec. II-D): the secret entries S (D of them, padded to a power
// of two D' >= N with the table's first row) lie in the public table T (N
// rows) iff at random beta sum_i 1/(beta + s_i) = sum_j m_j/(beta + t_j)
// (eq. (rational-function)); with random alpha and u the sumcheck of
// eq. (lookup-sumcheck) proves it.  Every challenge is known before the
// first kernel runs (there are no commitments here), so the host squeezes
// gamma, beta, alpha and u, and the device computes the multiplicities, the
// inverses and the rounds (lookup.hip).
#include <hip/hip_runtime.h>

#include <cstring>
#include <vector>

#include "plan.hpp"
#include "sha256.hpp"

namespace vl {
namespace {

constexpr uint32_t kLookupMaxVars = 30;

uint64_t padded(uint64_t D, uint32_t N) {
  uint64_t n = N;
  while (n < D) n *= 2;
  return n;
}

vl_status check_lookup(const vl_lookup& L, bool need_ptrs) {
  if (!L.D || !L.N || L.N > (1u << 20) || (L.N & (L.N - 1)))
    return fail(VL_ERR_SHAPE, "lookup: D must be >= 1 and N a power of two in 1 .. 2^20");
  if (L.D > (1ull << kLookupMaxVars)) return fail(VL_ERR_SHAPE, "lookup: D must be <= 2^%u", kLookupMaxVars);
  if (L.dtype != VL_I16 && L.dtype != VL_I32) return fail(VL_ERR_DTYPE, "lookup: entries must be int16 or int32");
  if (L.two_col && L.dtype_y != VL_I16 && L.dtype_y != VL_I32)
    return fail(VL_ERR_DTYPE, "lookup: second-column entries must be int16 or int32");
  if (need_ptrs && (L.two_col ? (!L.y || !L.tb) : (L.y || L.tb)))
    return fail(VL_ERR_INVALID_ARG, "lookup: two_col needs both y and tb, one column neither");
  if ((int64_t)L.t0 + L.N - 1 > INT32_MAX) return fail(VL_ERR_SHAPE, "lookup: table rows exceed int32");
  if (need_ptrs && !L.x) return fail(VL_ERR_INVALID_ARG, "lookup: null entries");
  return VL_OK;
}

uint64_t lookup_elems(const vl_lookup& L) { return 4ull * nvars_of(padded(L.D, L.N)) + 5; }

bool two_col(const vl_lookup& L) { return L.two_col != 0; }

Transcript lookup_init(uint64_t seed, const vl_lookup& L, bool two) {
  Sha256 s;
  sha256_init(s);
  const char dom[] = "VeriLoRA-lookup-v1";
  sha256_update(s, reinterpret_cast<const uint8_t*>(dom), 18);
  uint8_t w[8];
  for (int i = 0; i < 8; ++i) w[i] = (uint8_t)(seed >> (8 * i));
  sha256_update(s, w, 8);
  put_u32le(w, L.id);
  sha256_update(s, w, 4);
  for (int i = 0; i < 8; ++i) w[i] = (uint8_t)(L.D >> (8 * i));
  sha256_update(s, w, 8);
  for (uint32_t x : {L.N, (uint32_t)L.t0, (uint32_t)(two ? 1 : 0)}) {
    put_u32le(w, x);
    sha256_update(s, w, 4);
  }
  uint8_t st[32];
  sha256_final(s, st);
  Transcript t;
  tr_from_bytes(t, st);
  return t;
}

struct LookupChallenges {
  Transcript tr;
  Fr gamma, beta, alpha;      // canonical
  std::vector<Fr> u;
};

LookupChallenges lookup_challenges(const vl_lookup& L, uint64_t seed, bool two) {
  LookupChallenges c;
  c.tr = lookup_init(seed, L, two);
  c.gamma = two ? tr_squeeze_fixed(c.tr, "gamma") : fr_zero();
  c.beta = tr_squeeze_fixed(c.tr, "beta");
  c.alpha = tr_squeeze_fixed(c.tr, "alpha");
  const uint32_t n = nvars_of(padded(L.D, L.N));
  for (uint32_t i = 0; i < n; ++i) c.u.push_back(tr_squeeze_fixed(c.tr, VL_LBL_U));
  return c;
}

// N / D' = 2^-nH and alpha^2 N / D' (Montgomery)
void lookup_consts(uint32_t nH, const Fr& alpha_m, Fr& c1, Fr& c2) {
  c2 = fr_R();
  const Fr inv2 = fr_inv2_mont();
  for (uint32_t i = 0; i < nH; ++i) c2 = fr_mul(c2, inv2);
  c1 = fr_mul(c2, fr_mul(alpha_m, alpha_m));
}

void plan_lookup(Builder& B, const vl_lookup& L, const LookupChallenges& ch, uint8_t* proof_dev,
                 int32_t* status_dev, uint8_t* digest_dev, int32_t* flag) {
  const uint64_t Dp = padded(L.D, L.N), N = L.N;
  const uint32_t n = nvars_of(Dp), nL = nvars_of(N), nH = n - nL;
  LookupJob j{};
  memcpy(j.st, ch.tr.h, 32);
  const Fr gm = fr_to_mont(ch.gamma), bm = fr_to_mont(ch.beta), am = fr_to_mont(ch.alpha);
  Fr c1, c2;
  lookup_consts(nH, am, c1, c2);
  const Fr claim = fr_add(am, fr_mul(am, am));
  memcpy(j.gamma, gm.w, 32);
  memcpy(j.beta, bm.w, 32);
  memcpy(j.alpha, am.w, 32);
  memcpy(j.c1, c1.w, 32);
  memcpy(j.c2, c2.w, 32);
  memcpy(j.claim, claim.w, 32);
  j.x = L.x;
  j.y = L.y;
  j.tb = L.tb;
  j.dtype = L.dtype;
  j.dtype_y = L.dtype_y;
  j.t0 = L.t0;
  j.D = L.D;
  j.nH = nH;
  j.nL = nL;
  j.cnt = B.dev<uint32_t>(B.take(4 * N));
  B.P.lookup_zero.push_back({j.cnt, N});
  j.A = B.dev<uint32_t>(B.take(32 * Dp));
  j.S = B.dev<uint32_t>(B.take(32 * Dp));
  j.E = B.dev<uint32_t>(B.take(32 * Dp));
  j.B = B.dev<uint32_t>(B.take(32 * N));
  j.T = B.dev<uint32_t>(B.take(32 * N));
  j.M = B.dev<uint32_t>(B.take(32 * N));
  j.EL = B.dev<uint32_t>(B.take(32 * N));
  // E' = alpha eq(u, .) and EL' = c1 eq(u_L, .): the constant factors of
  // their terms built into the tables (neither is sent)
  B.eq_job(ch.u, j.E, nullptr, 0, false, false, &am);
  B.eq_job(std::vector<Fr>(ch.u.begin() + nH, ch.u.end()), j.EL, nullptr, 0, false, false, &c1);
  const uint64_t chunks = (N + kLookupInvChunk - 1) / kLookupInvChunk;
  j.nkparts = (uint32_t)((N + 255) / 256);
  j.kpart = B.dev<uint32_t>(B.take(128ull * j.nkparts));
  j.io = B.dev<uint32_t>(B.take(4 * kLkIoWords));
  j.flag = flag;
  j.proof = proof_dev;
  j.digest = digest_dev;
  j.status = status_dev;
  j.hist_begin = B.P.lk_hist_blocks;
  B.P.lk_hist_blocks += (uint32_t)((L.D + 255) / 256);
  j.prep_begin = B.P.lk_prep_blocks;
  B.P.lk_prep_blocks += (uint32_t)((Dp + 255) / 256);
  j.tab_begin = B.P.lk_tab_blocks;
  B.P.lk_tab_blocks += (uint32_t)((chunks + 255) / 256);
  j.mult_begin = B.P.lk_mult_blocks;
  B.P.lk_mult_blocks += j.nkparts;
  uint32_t wide = 0;
  while (wide < n && wide < kLookupMaxWide && (Dp >> (wide + 1)) >= kLookupWidePairs) ++wide;
  j.wide = wide;
  if (wide) j.part = B.dev<uint32_t>(B.take(((Dp / 2 + kLookupSweepPairs - 1) / kLookupSweepPairs) * 128));
  const uint32_t idx = (uint32_t)B.P.lookups.size();
  B.P.lookups.push_back(j);
  for (int lo = 0; lo < 2; ++lo)
    if (B.P.lk_wide[lo].size() < wide) {
      B.P.lk_wide[lo].resize(wide);
      B.P.lk_wide_blocks[lo].resize(wide, 0);
    }
  for (uint32_t k = 0; k < wide; ++k) {
    const uint64_t h = Dp >> (k + 1);
    const int lo = k >= nH ? 1 : 0;
    B.P.lk_wide[lo][k].push_back(LookupSweep{idx, B.P.lk_wide_blocks[lo][k]});
    B.P.lk_wide_blocks[lo][k] += (uint32_t)((h + kLookupSweepPairs - 1) / kLookupSweepPairs);
  }
}

vl_status lookup_run(const vl_lookup* ls, uint64_t n, uint64_t seed, uint8_t* ws, uint64_t ws_bytes,
                     uint8_t* proofs, const uint64_t* offsets, uint8_t* digests, hipStream_t s, uint64_t* ws_need) {
  const bool sizing = ws == nullptr;
  const uint64_t plen = sizing ? 0 : offsets[n];
  const uint64_t st_off = align_up(plen, 256), dg_off = st_off + align_up(4 * n, 256);
  const uint64_t out_bytes = dg_off + 32 * n;
  PinnedOut* po = nullptr;
  uint8_t *oh = nullptr, *od = nullptr;
  if (!sizing) {
    const hipError_t e = pinned_out(out_bytes, &po);
    if (e != hipSuccess) return fail(VL_ERR_HIP, "pinned output buffer: %s", hipGetErrorString(e));
    oh = reinterpret_cast<uint8_t*>(po->host);
    od = reinterpret_cast<uint8_t*>(po->dev);
    memset(oh, 0, out_bytes);
    memset(oh + st_off, 0xff, 4 * n);
  }
  std::vector<LookupChallenges> ch(n);
  for (uint64_t k = 0; k < n; ++k) ch[k] = lookup_challenges(ls[k], seed, two_col(ls[k]));
  Tuning T;
  Plan P;
  uint64_t blob = 0;
  for (int pass = 0; pass < 2; ++pass) {
    P = Plan();
    Builder B(P, T, reinterpret_cast<uint64_t>(ws), blob);
    P.n_err = (uint32_t)n;
    for (uint64_t k = 0; k < n; ++k)
      plan_lookup(B, ls[k], ch[k], od ? od + offsets[k] : nullptr,
                  od ? reinterpret_cast<int32_t*>(od + st_off) + k : nullptr, od ? od + dg_off + 32 * k : nullptr,
                  reinterpret_cast<int32_t*>(B.base) + k);
    P.data_end = B.off;
    if (pass == 0) blob = align_up(blob_layout(P).total, 256);
  }
  if (sizing) {
    *ws_need = align_up(P.data_end, 256);
    return VL_OK;
  }
  if (P.data_end > ws_bytes)
    return fail(VL_ERR_WORKSPACE, "workspace of %llu bytes, %llu needed", (unsigned long long)ws_bytes,
                (unsigned long long)align_up(P.data_end, 256));
  const BlobLayout BL = blob_layout(P);
  fill_blob(P, BL, ws);
  // the eq tables on the internal side stream and the table inversions on
  // the internal rounds stream, beside the count kernel
  hipStream_t s2 = nullptr, s3 = nullptr;
  hipError_t e = rounds_stream_for(s, &s2);
  if (e == hipSuccess) e = side_stream_for(s, &s3);
  if (e != hipSuccess) return fail(VL_ERR_HIP, "internal streams: %s", hipGetErrorString(e));
  P.eq_fork = true;
  e = enqueue_plan(P, BL, ws, s, s2, nullptr, nullptr, s3);
  const hipError_t e2 = hipStreamSynchronize(s);
  // both are joined into s unless the enqueue failed
  const hipError_t e3 = hipStreamSynchronize(s2), e4 = hipStreamSynchronize(s3);
  if (e == hipSuccess) e = e2;
  if (e == hipSuccess) e = e3;
  if (e == hipSuccess) e = e4;
  if (e != hipSuccess) return fail(VL_ERR_HIP, "lookup prove: %s", hipGetErrorString(e));
  const int32_t* st = reinterpret_cast<const int32_t*>(oh + st_off);
  for (uint64_t k = 0; k < n; ++k) {
    if (st[k] == VL_ERR_FALSE_STATEMENT)
      return fail(VL_ERR_FALSE_STATEMENT, "lookup %llu: an entry is not in the table", (unsigned long long)k);
    if (st[k] != VL_OK) return fail(VL_ERR_HIP, "lookup %llu: status %d", (unsigned long long)k, st[k]);
  }
  memcpy(proofs, oh, plen);
  if (digests) memcpy(digests, oh + dg_off, 32 * n);
  return VL_OK;
}

int64_t entry_of(const void* p, int dt, uint64_t i) {
  return dt == VL_I16 ? (int64_t)reinterpret_cast<const int16_t*>(p)[i] : (int64_t)reinterpret_cast<const int32_t*>(p)[i];
}

// sum_i v_i eq(r, i) for Montgomery values and point
Fr mle_vals(const std::vector<Fr>& vals, const std::vector<Fr>& r) {
  const std::vector<Fr> e = eq_host(r);
  Fr t = fr_zero();
  for (size_t i = 0; i < vals.size(); ++i) t = fr_add(t, fr_mul(vals[i], e[i]));
  return t;
}

}  // namespace
}  // namespace vl

using namespace vl;

extern "C" {

uint64_t vl_lookup_proof_size(const vl_lookup* L) {
  if (!L || check_lookup(*L, false) != VL_OK) return 0;
  return 32 * lookup_elems(*L);
}

uint64_t vl_lookup_workspace_size(const vl_lookup* L, uint64_t n) {
  if (!L || !n) return 0;
  for (uint64_t k = 0; k < n; ++k)
    if (check_lookup(L[k], false) != VL_OK) return 0;
  uint64_t need = 0;
  if (lookup_run(L, n, 0, nullptr, 0, nullptr, nullptr, nullptr, nullptr, &need) != VL_OK) return 0;
  return need;
}

vl_status vl_lookup_prove(const vl_lookup* L, uint64_t n, uint64_t seed, void* workspace, uint64_t workspace_bytes,
                          uint8_t* proofs, uint64_t proofs_len, uint64_t* offsets, uint8_t* digests, void* stream) {
  if (!L || !n || !proofs || !offsets) return fail(VL_ERR_INVALID_ARG, "null argument");
  for (uint64_t k = 0; k < n; ++k) {
    const vl_status st = check_lookup(L[k], true);
    if (st != VL_OK) return st;
  }
  if (!workspace) return fail(VL_ERR_WORKSPACE, "no workspace");
  if (reinterpret_cast<uintptr_t>(workspace) % 256) return fail(VL_ERR_WORKSPACE, "workspace must be 256-byte aligned");
  offsets[0] = 0;
  for (uint64_t k = 0; k < n; ++k) offsets[k + 1] = offsets[k] + 32 * lookup_elems(L[k]);
  if (proofs_len < offsets[n])
    return fail(VL_ERR_BUFFER_TOO_SMALL, "proof buffer holds %llu bytes, %llu needed", (unsigned long long)proofs_len,
                (unsigned long long)offsets[n]);
  return lookup_run(L, n, seed, reinterpret_cast<uint8_t*>(workspace), workspace_bytes, proofs, offsets, digests,
                    reinterpret_cast<hipStream_t>(stream), nullptr);
}

vl_status vl_lookup_verify(const uint8_t* proof, uint64_t len, const vl_lookup* L, uint64_t seed, vl_fr* reduced,
                           uint64_t reduced_cap, uint64_t* reduced_len, int32_t* fail_round) {
  if (fail_round) *fail_round = 0;
  if (!L || (!proof && len)) return fail(VL_ERR_INVALID_ARG, "null argument");
  {
    const vl_status cs = check_lookup(*L, false);
    if (cs != VL_OK) return cs;
  }
  const bool two = two_col(*L);
  const uint64_t ne = lookup_elems(*L);
  if (len != 32 * ne)
    return fail(VL_ERR_REJECT, "proof has %llu bytes, expected %llu", (unsigned long long)len,
                (unsigned long long)(32 * ne));
  std::vector<Fr> el(ne);
  for (uint64_t i = 0; i < ne; ++i) {
    el[i] = fr_from_bytes(proof + 32 * i);
    if (!fr_lt_p(el[i])) return fail(VL_ERR_REJECT, "element %llu is not canonical", (unsigned long long)i);
  }
  LookupChallenges ch = lookup_challenges(*L, seed, two);
  Transcript& tr = ch.tr;
  const uint64_t Dp = padded(L->D, L->N);
  const uint32_t n = nvars_of(Dp), nL = nvars_of(L->N), nH = n - nL;
  const Fr am = fr_to_mont(ch.alpha), bm = fr_to_mont(ch.beta), gm = fr_to_mont(ch.gamma);
  Fr c1, c2;
  lookup_consts(nH, am, c1, c2);
  Fr claim = fr_add(am, fr_mul(am, am));
  std::vector<Fr> out;
  for (const Fr& x : {ch.gamma, ch.beta, ch.alpha}) out.push_back(x);
  for (const Fr& x : ch.u) out.push_back(x);
  std::vector<Fr> rs, um(ch.u.size());
  for (size_t i = 0; i < um.size(); ++i) um[i] = fr_to_mont(ch.u[i]);
  for (uint32_t rd = 0; rd < n; ++rd) {
    const Fr gc[4] = {el[4 * rd], el[4 * rd + 1], el[4 * rd + 2], el[4 * rd + 3]};
    Fr gmv[4];
    for (int k = 0; k < 4; ++k) gmv[k] = fr_to_mont(gc[k]);
    if (!fr_eq(fr_add(gmv[0], gmv[1]), claim)) {
      if (fail_round) *fail_round = (int32_t)rd + 1;
      return fail(VL_ERR_REJECT, "round %u: g(0) + g(1) differs from the claim", rd + 1);
    }
    tr_absorb_frs(tr, VL_LBL_ROUND, gc);
    const Fr rc = tr_squeeze_fixed(tr, VL_LBL_R);
    out.push_back(rc);
    rs.push_back(fr_to_mont(rc));
    claim = lagrange_host(gmv, 4, rs.back());
  }
  const Fr fin[5] = {el[4 * n], el[4 * n + 1], el[4 * n + 2], el[4 * n + 3], el[4 * n + 4]};
  Fr f[5];
  for (int k = 0; k < 5; ++k) f[k] = fr_to_mont(fin[k]);
  const std::vector<Fr> rL(rs.begin() + nH, rs.end()), uL(um.begin() + nH, um.end());
  // alpha A eq(u, r) (S + beta) + A + c1 B eq(u_L, r_L) (T + beta) - c2 B m
  const Fr expect =
      fr_sub(fr_add(fr_add(fr_mul(fr_mul(am, f[0]), fr_mul(eq_point(um, rs), fr_add(f[1], bm))), f[0]),
                    fr_mul(fr_mul(c1, f[2]), fr_mul(eq_point(uL, rL), fr_add(f[3], bm)))),
             fr_mul(c2, fr_mul(f[2], f[4])));
  if (!fr_eq(expect, claim)) return fail(VL_ERR_REJECT, "final claim differs from the summand at r");
  tr_absorb_frs(tr, VL_LBL_FINAL, fin);
  for (const Fr& x : fin) out.push_back(x);
  if (L->x && (!two || (L->y && L->tb))) {
    // the five values by direct evaluation (standing in for the openings)
    const uint64_t N = L->N;
    std::vector<Fr> S(Dp), T(N), Bv(N), A(Dp), M(N, fr_zero());
    std::vector<uint64_t> cnt(N, 0);
    auto row = [&](int64_t x, int64_t y) {
      Fr v = lift_int(x);
      if (two) v = fr_add(v, fr_mul(gm, lift_int(y)));
      return v;
    };
    for (uint64_t j = 0; j < N; ++j) {
      T[j] = row(L->t0 + (int64_t)j, two ? L->tb[j] : 0);
      Bv[j] = fr_inv_host(fr_add(T[j], bm));
    }
    for (uint64_t i = 0; i < Dp; ++i) {
      const int64_t x = i < L->D ? entry_of(L->x, L->dtype, i) : L->t0;
      const int64_t y = two ? (i < L->D ? entry_of(L->y, L->dtype_y, i) : L->tb[0]) : 0;
      const int64_t j = x - L->t0;
      if (j < 0 || j >= (int64_t)N || (two && y != L->tb[j])) return fail(VL_ERR_REJECT, "witness entry not in the table");
      S[i] = row(x, y);
      A[i] = Bv[j];
      ++cnt[j];
    }
    for (uint64_t j = 0; j < N; ++j) M[j] = lift_int((int64_t)cnt[j]);
    if (!fr_eq(mle_vals(A, rs), f[0]) || !fr_eq(mle_vals(S, rs), f[1]) || !fr_eq(mle_vals(Bv, rL), f[2]) ||
        !fr_eq(mle_vals(T, rL), f[3]) || !fr_eq(mle_vals(M, rL), f[4]))
      return fail(VL_ERR_REJECT, "final values differ from the witness's multilinear extensions");
  }
  if (reduced_len) *reduced_len = out.size();
  if (reduced) {
    if (reduced_cap < out.size()) return fail(VL_ERR_BUFFER_TOO_SMALL, "reduced buffer too small");
    for (size_t i = 0; i < out.size(); ++i) memcpy(reduced[i].w, out[i].w, 32);
  }
  if (fail_round) *fail_round = -1;
  return VL_OK;
}

}  // extern "C"
