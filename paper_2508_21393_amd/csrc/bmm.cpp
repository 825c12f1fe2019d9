// Per-head batched products: planning, proving and the host verifier
// (vl_bmm_prove, vl_bmm_verify).
//
// Multi-head attention (Sec. III-A, eq. (att)) multiplies one pair of
// matrices per head.  For H heads the statement C_h = A_h B_h (h < H) is
// proved by one sumcheck over the head and inner variables of
//     C~(rho, u, v) = sum_{h, w} eq(rho, h) A~(h, u, w) B~(h, w, v)
// (eq. (MLE) over the 3-D tensors, head index most significant).  The device
// work reuses the contraction machinery of the matmul prover: eq(u, .) and
// eq(v, .) in signed-digit form contract every head's A and B into the
// tables a[h, w] = A~(h, u, w), b[h, w] = B~(h, w, v); the claim contracts
// each head's C with one of them and takes the dot product with the eq table
// of the concatenated point (rho, v) or (rho, u), since
// eq(rho, h) eq(v, j) = eq((rho, v), (h, j)).  The rounds run in bmm.hip.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <vector>

#include "plan.hpp"
#include "sha256.hpp"

namespace vl {
namespace {

constexpr uint32_t kBmmMaxVars = 26;

vl_status check_bmm(const vl_bmm& b, bool need_ptrs) {
  if (!b.H || !b.D0 || !b.D1 || !b.D2 || b.H > VL_MAX_DIM || b.D0 > VL_MAX_DIM || b.D1 > VL_MAX_DIM ||
      b.D2 > VL_MAX_DIM)
    return fail(VL_ERR_SHAPE, "batched product: H, D0, D1, D2 must be 1..2^20");
  for (int32_t dt : {b.dtype_a, b.dtype_b, b.dtype_c})
    if (dt != VL_I16 && dt != VL_I32 && dt != VL_I64) return fail(VL_ERR_DTYPE, "batched product: bad dtype");
  if (nvars_of(b.H) + nvars_of(b.D1) > kBmmMaxVars)
    return fail(VL_ERR_SHAPE, "batched product: log2 H + log2 D1 must be <= %u", kBmmMaxVars);
  if (b.lda < (b.trans_a ? b.D0 : b.D1) || b.ldb < (b.trans_b ? b.D1 : b.D2) || b.ldc < b.D2)
    return fail(VL_ERR_SHAPE, "batched product: leading dimension smaller than the row length");
  if (need_ptrs && (!b.A || !b.B || !b.C)) return fail(VL_ERR_INVALID_ARG, "batched product: null tensor");
  return VL_OK;
}

uint64_t bmm_elems(const vl_bmm& b) { return 1 + 4ull * nvars_of(b.H) + 3ull * nvars_of(b.D1) + 2; }

Transcript bmm_init(uint64_t seed, const vl_bmm& b) {
  Sha256 s;
  sha256_init(s);
  const char dom[] = "VeriLoRA-zkBMat-v1";
  sha256_update(s, reinterpret_cast<const uint8_t*>(dom), 18);
  uint8_t w[8];
  for (int i = 0; i < 8; ++i) w[i] = (uint8_t)(seed >> (8 * i));
  sha256_update(s, w, 8);
  for (uint32_t x : {b.group_id, b.H, b.D0, b.D1, b.D2}) {
    put_u32le(w, x);
    sha256_update(s, w, 4);
  }
  uint8_t st[32];
  sha256_final(s, st);
  Transcript t;
  tr_from_bytes(t, st);
  return t;
}

struct BmmChallenges {
  Transcript tr;
  std::vector<Fr> rho, u, v;   // canonical
};

BmmChallenges bmm_challenges(const vl_bmm& b, uint64_t seed) {
  BmmChallenges c;
  c.tr = bmm_init(seed, b);
  for (uint32_t i = 0; i < nvars_of(b.H); ++i) c.rho.push_back(tr_squeeze_fixed(c.tr, "h"));
  for (uint32_t i = 0; i < nvars_of(b.D0); ++i) c.u.push_back(tr_squeeze_fixed(c.tr, VL_LBL_U));
  for (uint32_t i = 0; i < nvars_of(b.D2); ++i) c.v.push_back(tr_squeeze_fixed(c.tr, VL_LBL_V));
  return c;
}

std::vector<Fr> concat(const std::vector<Fr>& x, const std::vector<Fr>& y) {
  std::vector<Fr> z(x);
  z.insert(z.end(), y.begin(), y.end());
  return z;
}

// The jobs of one batched product (device addresses from the builder).
void plan_bmm(Builder& B, const vl_bmm& b, const BmmChallenges& ch, uint8_t* proof_dev, int32_t* status_dev,
              uint8_t* digest_dev, int32_t* err) {
  const uint32_t nh = nvars_of(b.H), n0 = nvars_of(b.D0), n1 = nvars_of(b.D1), n2 = nvars_of(b.D2);
  const uint64_t L0 = 1ull << n0, L1 = 1ull << n1, L2 = 1ull << n2, Hp = 1ull << nh, N = Hp * L1;
  const uint64_t esa = esize(b.dtype_a), esb = esize(b.dtype_b), esc = esize(b.dtype_c);
  uint32_t* packU = B.dev<uint32_t>(B.take((uint64_t)b.D0 * 32));
  uint32_t* packV = B.dev<uint32_t>(B.take((uint64_t)b.D2 * 32));
  uint32_t* E = B.dev<uint32_t>(B.take(8 * Hp * 4));
  B.eq_job(ch.rho, E, nullptr, 0, false, false);            // eq(rho, .), Montgomery
  B.eq_job(ch.u, nullptr, packU, b.D0, true, false);        // e R^2 digits: a lands in Montgomery form
  B.eq_job(ch.v, nullptr, packV, b.D2, false, false);       // e R digits: b and t land canonical

  // claim: per head, s_h[j] = sum_i eq(u, i) C_h[i][j] (Montgomery) dotted
  // with eq((rho, v), .) canonical, or t_h[i] = sum_j C_h[i][j] eq(v, j)
  // (canonical) dotted with eq((rho, u), .) in Montgomery form
  int ndc = digits_for(b.dtype_c);
  if (b.dtype_c == VL_I64 && b.dtype_a == VL_I16 && b.dtype_b == VL_I16 && b.D1 <= (1u << 16)) ndc = 2;
  const bool by_rows = b.D2 >= 256;
  const uint64_t Lc = by_rows ? L2 : L0;
  uint32_t* eqc = B.dev<uint32_t>(B.take(8 * Hp * Lc * 4));
  uint32_t* cv = B.dev<uint32_t>(B.take(8 * b.H * Lc * 4));
  const uint8_t* C = reinterpret_cast<const uint8_t*>(b.C);
  if (by_rows) {
    B.eq_job(concat(ch.rho, ch.v), eqc, nullptr, 0, false, true);
    for (uint32_t h = 0; h < b.H; ++h)
      B.contract(C + h * b.head_stride_c * esc, b.dtype_c, ndc, b.ldc, true, b.D2, b.D0, packU, cv + h * Lc,
                 b.H * Lc, Lc, err);
  } else {
    B.eq_job(concat(ch.rho, ch.u), eqc, nullptr, 0, false, false);
    for (uint32_t h = 0; h < b.H; ++h)
      B.contract(C + h * b.head_stride_c * esc, b.dtype_c, ndc, b.ldc, false, b.D0, b.D2, packV, cv + h * Lc,
                 b.H * Lc, Lc, err);
  }
  BmmJob j{};
  j.c_part = B.pass1(eqc, Hp * Lc, cv, b.H * Lc, (uint32_t)(b.H * Lc), true, j.c_nparts, nullptr);

  // tables over (h, w): a[h, w] = sum_i eq(u, i) op(A_h)[i][w], b[h, w] =
  // sum_j op(B_h)[w][j] eq(v, j); padding heads are zero
  uint32_t* ta = B.dev<uint32_t>(B.take(8 * N * 4));
  uint32_t* tb = B.dev<uint32_t>(B.take(8 * N * 4));
  const uint8_t* A = reinterpret_cast<const uint8_t*>(b.A);
  const uint8_t* Bm = reinterpret_cast<const uint8_t*>(b.B);
  for (uint32_t h = 0; h < b.H; ++h) {
    B.contract(A + h * b.head_stride_a * esa, b.dtype_a, digits_for(b.dtype_a), b.lda, !b.trans_a, b.D1, b.D0,
               packU, ta + h * L1, N, L1, err);
    B.contract(Bm + h * b.head_stride_b * esb, b.dtype_b, digits_for(b.dtype_b), b.ldb, b.trans_b != 0, b.D1,
               b.D2, packV, tb + h * L1, N, L1, err);
  }
  if (Hp > b.H) {
    B.zero_fill(ta + b.H * L1, N, (uint32_t)((Hp - b.H) * L1));
    B.zero_fill(tb + b.H * L1, N, (uint32_t)((Hp - b.H) * L1));
  }

  memcpy(j.st, ch.tr.h, 32);
  j.nh = nh;
  j.n1 = n1;
  j.E = E;
  j.a = ta;
  j.b = tb;
  j.io = B.dev<uint32_t>(B.take(4 * kBmmIoWords));
  j.proof = proof_dev;
  j.digest = digest_dev;
  j.status = status_dev;
  j.err = err;
  // wide rounds: while a round has at least kBmmWidePairs pairs
  const uint32_t nv = nh + n1;
  uint32_t wide = 0;
  while (wide < nv && wide < kBmmMaxWide && (N >> (wide + 1)) >= kBmmWidePairs) ++wide;
  j.wide = wide;
  if (wide) j.part = B.dev<uint32_t>(B.take(((N / 2 + kBmmSweepPairs - 1) / kBmmSweepPairs) * 32 * 4));
  const uint32_t idx = (uint32_t)B.P.bmms.size();
  B.P.bmms.push_back(j);
  if (B.P.bmm_wide.size() < wide) {
    B.P.bmm_wide.resize(wide);
    B.P.bmm_wide_blocks.resize(wide, 0);
  }
  for (uint32_t k = 0; k < wide; ++k) {
    const uint64_t h = N >> (k + 1);
    B.P.bmm_wide[k].push_back(BmmSweep{idx, B.P.bmm_wide_blocks[k]});
    B.P.bmm_wide_blocks[k] += (uint32_t)((h + kBmmSweepPairs - 1) / kBmmSweepPairs);
  }
}

// Sizes (ws == nullptr: *ws_need gets the bytes) or runs the proofs; the
// same planning code does both.
vl_status bmm_run(const vl_bmm* bs, uint64_t n, uint64_t seed, uint8_t* ws, uint64_t ws_bytes, uint8_t* proofs,
                  const uint64_t* offsets, uint8_t* digests, hipStream_t s, uint64_t* ws_need) {
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
  std::vector<BmmChallenges> ch(n);
  for (uint64_t k = 0; k < n; ++k) ch[k] = bmm_challenges(bs[k], seed);
  Tuning T;
  T.per_instance = false;
  T.min_tasks = 1;
  T.segments = 1;
  Plan P;
  uint64_t blob = 0;
  for (int pass = 0; pass < 2; ++pass) {
    P = Plan();
    Builder B(P, T, reinterpret_cast<uint64_t>(ws), blob);
    P.n_err = (uint32_t)n;
    for (uint64_t k = 0; k < n; ++k)
      plan_bmm(B, bs[k], ch[k], od ? od + offsets[k] : nullptr,
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
  hipError_t e = enqueue_plan(P, BL, ws, s, s, nullptr);
  const hipError_t e2 = hipStreamSynchronize(s);
  if (e == hipSuccess) e = e2;
  if (e != hipSuccess) return fail(VL_ERR_HIP, "batched prove: %s", hipGetErrorString(e));
  const int32_t* st = reinterpret_cast<const int32_t*>(oh + st_off);
  for (uint64_t k = 0; k < n; ++k) {
    if (st[k] == VL_ERR_FALSE_STATEMENT)
      return fail(VL_ERR_FALSE_STATEMENT, "batched product %llu: C is not the heads' products",
                  (unsigned long long)k);
    if (st[k] == VL_ERR_RANGE)
      return fail(VL_ERR_RANGE, "batched product %llu: an entry exceeds the digit range", (unsigned long long)k);
    if (st[k] != VL_OK) return fail(VL_ERR_HIP, "batched product %llu: status %d", (unsigned long long)k, st[k]);
  }
  memcpy(proofs, oh, plen);
  if (digests) memcpy(digests, oh + dg_off, 32 * n);
  return VL_OK;
}

// sum_h eq(hp, h) M_h~(x, y) of H stored head matrices (accessor per head)
template <typename G>
Fr tensor_mle_host(G get, uint32_t H, uint32_t rows, uint32_t cols, const std::vector<Fr>& hp,
                   const std::vector<Fr>& x, const std::vector<Fr>& y) {
  const std::vector<Fr> eh = eq_host(hp);
  Fr total = fr_zero();
  for (uint32_t h = 0; h < H; ++h) {
    const Fr m = mle2([&](uint32_t i, uint32_t j) { return get(h, i, j); }, rows, cols, x, y);
    total = fr_add(total, fr_mul(eh[h], m));
  }
  return total;
}

}  // namespace
}  // namespace vl

using namespace vl;

extern "C" {

uint64_t vl_bmm_proof_size(const vl_bmm* b) {
  if (!b || check_bmm(*b, false) != VL_OK) return 0;
  return 32 * bmm_elems(*b);
}

uint64_t vl_bmm_workspace_size(const vl_bmm* b, uint64_t n) {
  if (!b || !n) return 0;
  for (uint64_t k = 0; k < n; ++k)
    if (check_bmm(b[k], false) != VL_OK) return 0;
  uint64_t need = 0;
  if (bmm_run(b, n, 0, nullptr, 0, nullptr, nullptr, nullptr, nullptr, &need) != VL_OK) return 0;
  return need;
}

vl_status vl_bmm_prove(const vl_bmm* b, uint64_t n, uint64_t seed, void* workspace, uint64_t workspace_bytes,
                       uint8_t* proofs, uint64_t proofs_len, uint64_t* offsets, uint8_t* digests, void* stream) {
  if (!b || !n || !proofs || !offsets) return fail(VL_ERR_INVALID_ARG, "null argument");
  for (uint64_t k = 0; k < n; ++k) {
    const vl_status st = check_bmm(b[k], true);
    if (st != VL_OK) return st;
  }
  if (!workspace) return fail(VL_ERR_WORKSPACE, "no workspace");
  if (reinterpret_cast<uintptr_t>(workspace) % 256) return fail(VL_ERR_WORKSPACE, "workspace must be 256-byte aligned");
  offsets[0] = 0;
  for (uint64_t k = 0; k < n; ++k) offsets[k + 1] = offsets[k] + 32 * bmm_elems(b[k]);
  if (proofs_len < offsets[n])
    return fail(VL_ERR_BUFFER_TOO_SMALL, "proof buffer holds %llu bytes, %llu needed", (unsigned long long)proofs_len,
                (unsigned long long)offsets[n]);
  return bmm_run(b, n, seed, reinterpret_cast<uint8_t*>(workspace), workspace_bytes, proofs, offsets, digests,
                 reinterpret_cast<hipStream_t>(stream), nullptr);
}

vl_status vl_bmm_verify(const uint8_t* proof, uint64_t len, const vl_bmm* b, uint64_t seed, vl_fr* reduced,
                        uint64_t reduced_cap, uint64_t* reduced_len, int32_t* fail_round) {
  if (fail_round) *fail_round = 0;
  if (!b || (!proof && len)) return fail(VL_ERR_INVALID_ARG, "null argument");
  {
    const vl_status cs = check_bmm(*b, false);
    if (cs != VL_OK) return cs;
  }
  const uint64_t ne = bmm_elems(*b);
  if (len != 32 * ne)
    return fail(VL_ERR_REJECT, "proof has %llu bytes, expected %llu", (unsigned long long)len,
                (unsigned long long)(32 * ne));
  std::vector<Fr> el(ne);   // canonical
  for (uint64_t i = 0; i < ne; ++i) {
    el[i] = fr_from_bytes(proof + 32 * i);
    if (!fr_lt_p(el[i])) return fail(VL_ERR_REJECT, "element %llu is not canonical", (unsigned long long)i);
  }
  BmmChallenges ch = bmm_challenges(*b, seed);
  Transcript& tr = ch.tr;
  const uint32_t nh = nvars_of(b->H), n1 = nvars_of(b->D1);
  std::vector<Fr> out;
  size_t pos = 0;
  const Fr c = el[pos++];
  out.push_back(c);
  for (const auto* vec : {&ch.rho, &ch.u, &ch.v})
    for (const Fr& x : *vec) out.push_back(x);
  {
    const Fr cc[1] = {c};
    tr_absorb_frs(tr, VL_LBL_CLAIM, cc);
  }
  Fr claim = fr_to_mont(c);
  std::vector<Fr> rh, rw;   // Montgomery
  for (uint32_t rd = 0; rd < nh + n1; ++rd) {
    const bool head = rd < nh;
    const int m = head ? 4 : 3;
    Fr gm[4];
    for (int k = 0; k < m; ++k) gm[k] = fr_to_mont(el[pos + k]);
    if (!fr_eq(fr_add(gm[0], gm[1]), claim)) {
      if (fail_round) *fail_round = (int32_t)rd + 1;
      return fail(VL_ERR_REJECT, "round %u: g(0) + g(1) differs from the claim", rd + 1);
    }
    if (head) {
      const Fr gc[4] = {el[pos], el[pos + 1], el[pos + 2], el[pos + 3]};
      tr_absorb_frs(tr, VL_LBL_ROUND, gc);
    } else {
      const Fr gc[3] = {el[pos], el[pos + 1], el[pos + 2]};
      tr_absorb_frs(tr, VL_LBL_ROUND, gc);
    }
    pos += m;
    const Fr rc = tr_squeeze_fixed(tr, VL_LBL_R);
    out.push_back(rc);
    const Fr r = fr_to_mont(rc);
    (head ? rh : rw).push_back(r);
    claim = lagrange_host(gm, m, r);
  }
  const Fr fin[2] = {el[pos], el[pos + 1]};
  std::vector<Fr> rhom(ch.rho.size()), um(ch.u.size()), vm(ch.v.size());
  for (size_t i = 0; i < rhom.size(); ++i) rhom[i] = fr_to_mont(ch.rho[i]);
  for (size_t i = 0; i < um.size(); ++i) um[i] = fr_to_mont(ch.u[i]);
  for (size_t i = 0; i < vm.size(); ++i) vm[i] = fr_to_mont(ch.v[i]);
  const Fr af = fr_to_mont(fin[0]), bf = fr_to_mont(fin[1]);
  if (!fr_eq(fr_mul(fr_mul(eq_point(rhom, rh), af), bf), claim))
    return fail(VL_ERR_REJECT, "final claim differs from eq(rho, r_h) a_final b_final");
  tr_absorb_frs(tr, VL_LBL_FINAL, fin);
  out.push_back(fin[0]);
  out.push_back(fin[1]);
  if (b->A && b->B && b->C) {
    const vl_bmm& m = *b;
    const Fr cw = tensor_mle_host(
        [&](uint32_t h, uint32_t i, uint32_t j) {
          return get_int(m.C, m.dtype_c, h * m.head_stride_c + (uint64_t)i * m.ldc + j);
        },
        m.H, m.D0, m.D2, rhom, um, vm);
    if (!fr_eq(cw, fr_to_mont(c))) return fail(VL_ERR_REJECT, "c differs from C~(rho, u, v)");
    const Fr aw = tensor_mle_host(
        [&](uint32_t h, uint32_t i, uint32_t w) {
          const uint64_t o = h * m.head_stride_a;
          return m.trans_a ? get_int(m.A, m.dtype_a, o + (uint64_t)w * m.lda + i)
                           : get_int(m.A, m.dtype_a, o + (uint64_t)i * m.lda + w);
        },
        m.H, m.D0, m.D1, rh, um, rw);
    const Fr bw = tensor_mle_host(
        [&](uint32_t h, uint32_t w, uint32_t j) {
          const uint64_t o = h * m.head_stride_b;
          return m.trans_b ? get_int(m.B, m.dtype_b, o + (uint64_t)j * m.ldb + w)
                           : get_int(m.B, m.dtype_b, o + (uint64_t)w * m.ldb + j);
        },
        m.H, m.D1, m.D2, rh, rw, vm);
    if (!fr_eq(aw, af) || !fr_eq(bw, bf))
      return fail(VL_ERR_REJECT, "final values differ from A~(r_h, u, r_w), B~(r_h, r_w, v)");
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
