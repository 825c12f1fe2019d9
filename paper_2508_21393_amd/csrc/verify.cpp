// Host verifier of the matmul sumcheck (CPU only; vl_verify_transcript).
//
// Replays the Fiat-Shamir transcript (Sec. IV-A footnote, Sec. V) and checks
// the sumcheck rounds of Sec. II-B.1 for the claim of eq. (zk-mle-matmul):
// each round g(0) + g(1) must equal the running claim, which then moves to
// g(r) (interpolation on {0, 1, 2}); the last claim must be a_final * b_final.
// With a host witness it also evaluates the multilinear extensions of
// eq. (MLE) directly: c = C~(u, v), a_final = A~(u, r), b_final = B~(r, v).
#include <cstring>
#include <vector>

#include "plan.hpp"
#include "sha256.hpp"

namespace vl {

Fr fr_inv2_mont() {
  // (p + 1) / 2 in Montgomery form
  return fr_to_mont(fr_from_limbs(0x80000001u, 0x7fffffffu, 0x7fff2dffu, 0xa9ded201u, 0x04d0ec02u,
                                  0x199cec04u, 0x94cebea4u, 0x39f6d3a9u));
}

Fr lift_int(int64_t x) {
  const uint64_t mag = x < 0 ? (uint64_t)0 - (uint64_t)x : (uint64_t)x;
  Fr v = fr_zero();
  v.w[0] = (uint32_t)mag;
  v.w[1] = (uint32_t)(mag >> 32);
  if (x < 0) v = fr_sub(fr_zero(), v);
  return fr_to_mont(v);
}

int64_t get_int(const void* base, int dt, uint64_t idx) {
  switch (dt) {
    case VL_I16: return reinterpret_cast<const int16_t*>(base)[idx];
    case VL_I32: return reinterpret_cast<const int32_t*>(base)[idx];
    default: return reinterpret_cast<const int64_t*>(base)[idx];
  }
}

// eq table (Montgomery) of a Montgomery point, index bits most significant first
std::vector<Fr> eq_host(const std::vector<Fr>& x) {
  std::vector<Fr> t(1, fr_R());
  for (const Fr& xj : x) {
    std::vector<Fr> n(2 * t.size());
    const Fr om = fr_sub(fr_R(), xj);
    for (size_t i = 0; i < t.size(); ++i) {
      n[2 * i] = fr_mul(t[i], om);
      n[2 * i + 1] = fr_mul(t[i], xj);
    }
    t.swap(n);
  }
  return t;
}

// x^e mod p for a Montgomery x, e given as 8 little-endian limbs
static Fr fr_pow_mont(const Fr& x, const uint32_t (&e)[8]) {
  Fr r = fr_R();
  for (int i = 255; i >= 0; --i) {
    r = fr_mul(r, r);
    if ((e[i >> 5] >> (i & 31)) & 1u) r = fr_mul(r, x);
  }
  return r;
}

Fr fr_inv_host(const Fr& x) {
  uint32_t e[8] = {VL_P_LIMBS};
  e[0] -= 2;   // p - 2 (p's low limb is 1: the borrow propagates)
  if (e[0] == 0xffffffffu) {
    int i = 1;
    while (e[i] == 0) e[i++] = 0xffffffffu;
    --e[i];
  }
  return fr_pow_mont(x, e);
}

static Fr small_mont(int64_t v) { return lift_int(v); }

// the polynomial through (k, g[k]), k < m (m = 3 or 4), at r (Montgomery)
Fr lagrange_host(const Fr* g, int m, const Fr& r) {
  Fr total = fr_zero();
  for (int k = 0; k < m; ++k) {
    Fr num = fr_R(), den = fr_R();
    for (int q = 0; q < m; ++q) {
      if (q == k) continue;
      num = fr_mul(num, fr_sub(r, small_mont(q)));
      den = fr_mul(den, small_mont(k - q));
    }
    total = fr_add(total, fr_mul(g[k], fr_mul(num, fr_inv_host(den))));
  }
  return total;
}

// eq(x, y) for Montgomery points of one length
Fr eq_point(const std::vector<Fr>& x, const std::vector<Fr>& y) {
  Fr e = fr_R();
  for (size_t i = 0; i < x.size(); ++i) {
    const Fr xy = fr_mul(x[i], y[i]);
    const Fr t = fr_add(xy, fr_sub(fr_sub(fr_R(), x[i]), fr_sub(y[i], xy)));   // xy + (1 - x)(1 - y)
    e = fr_mul(e, t);
  }
  return e;
}

}  // namespace vl

using namespace vl;

extern "C" vl_status vl_verify_transcript(const uint8_t* proof, uint64_t len, const vl_group* g,
                                          uint64_t seed, vl_fr* reduced, uint64_t reduced_cap,
                                          uint64_t* reduced_len, int32_t* fail_round) {
  if (fail_round) *fail_round = 0;
  if (!g || (!proof && len)) return fail(VL_ERR_INVALID_ARG, "null argument");
  const vl_status cs = check_group(*g, false);
  if (cs != VL_OK) return cs;
  const uint64_t ne = proof_elems(*g);
  if (len != 32 * ne) return fail(VL_ERR_REJECT, "proof has %llu bytes, expected %llu",
                                  (unsigned long long)len, (unsigned long long)(32 * ne));
  std::vector<Fr> el(ne);  // canonical
  for (uint64_t i = 0; i < ne; ++i) {
    el[i] = fr_from_bytes(proof + 32 * i);
    if (!fr_lt_p(el[i])) return fail(VL_ERR_REJECT, "element %llu is not canonical", (unsigned long long)i);
  }
  Transcript tr;
  std::vector<Fr> u, v;
  group_challenges(*g, seed, tr, u, v);
  std::vector<Fr> out;  // canonical reduced claims
  size_t pos = 0;
  const Fr c = el[pos++];
  out.push_back(c);
  for (const Fr& x : u) out.push_back(x);
  for (const Fr& x : v) out.push_back(x);
  {
    const Fr cc[1] = {c};
    tr_absorb_frs(tr, VL_LBL_CLAIM, cc);
  }
  std::vector<Fr> claims;  // Montgomery
  Fr parts_sum = fr_zero();
  for (uint32_t k = 0; k + 1 < g->n_prods; ++k) {
    const Fr s = el[pos++];
    const Fr sa[1] = {s};
    tr_absorb_frs(tr, VL_LBL_PART, sa);
    const Fr sm = fr_to_mont(s);
    claims.push_back(sm);
    parts_sum = fr_add(parts_sum, sm);
  }
  claims.push_back(fr_sub(fr_to_mont(c), parts_sum));
  const Fr inv2 = fr_inv2_mont(), one = fr_R(), two = fr_add(one, one);
  int32_t round_no = 0;
  std::vector<std::vector<Fr>> rvecs(g->n_prods);
  std::vector<Fr> finals_a(g->n_prods), finals_b(g->n_prods);
  for (uint32_t k = 0; k < g->n_prods; ++k) {
    Fr claim = claims[k];
    const uint32_t n1 = nvars_of(g->prods[k].D1);
    for (uint32_t i = 0; i < n1; ++i) {
      ++round_no;
      const Fr gc[3] = {el[pos], el[pos + 1], el[pos + 2]};
      pos += 3;
      const Fr g0 = fr_to_mont(gc[0]), g1 = fr_to_mont(gc[1]), g2 = fr_to_mont(gc[2]);
      if (!fr_eq(fr_add(g0, g1), claim)) {
        if (fail_round) *fail_round = round_no;
        return fail(VL_ERR_REJECT, "round %d: g(0) + g(1) differs from the claim", round_no);
      }
      tr_absorb_frs(tr, VL_LBL_ROUND, gc);
      const Fr rc = tr_squeeze_fixed(tr, VL_LBL_R);
      const Fr r = fr_to_mont(rc);
      rvecs[k].push_back(r);
      out.push_back(rc);
      // g(r) = g0 (r-1)(r-2)/2 - g1 r (r-2) + g2 r (r-1)/2
      const Fr rm1 = fr_sub(r, one), rm2 = fr_sub(r, two);
      const Fr l0 = fr_mul(fr_mul(rm1, rm2), inv2);
      const Fr l1 = fr_neg(fr_mul(r, rm2));
      const Fr l2 = fr_mul(fr_mul(r, rm1), inv2);
      claim = fr_add(fr_add(fr_mul(g0, l0), fr_mul(g1, l1)), fr_mul(g2, l2));
    }
    const Fr fin[2] = {el[pos], el[pos + 1]};
    pos += 2;
    finals_a[k] = fr_to_mont(fin[0]);
    finals_b[k] = fr_to_mont(fin[1]);
    if (!fr_eq(fr_mul(finals_a[k], finals_b[k]), claim)) {
      if (fail_round) *fail_round = 0;
      return fail(VL_ERR_REJECT, "product %u: final claim differs from a_final * b_final", k);
    }
    tr_absorb_frs(tr, VL_LBL_FINAL, fin);
    out.push_back(fin[0]);
    out.push_back(fin[1]);
  }
  // witness check by direct evaluation when every matrix is given (host memory)
  bool have = g->C != nullptr;
  for (uint32_t k = 0; k < g->n_prods; ++k) have = have && g->prods[k].A && g->prods[k].B;
  if (have) {
    std::vector<Fr> um(u.size()), vm(v.size());
    for (size_t i = 0; i < u.size(); ++i) um[i] = fr_to_mont(u[i]);
    for (size_t i = 0; i < v.size(); ++i) vm[i] = fr_to_mont(v[i]);
    const vl_product& p0 = g->prods[0];
    const Fr cw = mle2([&](uint32_t i, uint32_t j) { return get_int(g->C, g->dtype_c, (uint64_t)i * g->ldc + j); },
                       p0.D0, p0.D2, um, vm);
    if (!fr_eq(cw, fr_to_mont(c))) return fail(VL_ERR_REJECT, "c differs from C~(u, v)");
    for (uint32_t k = 0; k < g->n_prods; ++k) {
      const vl_product& p = g->prods[k];
      const Fr aw = mle2(
          [&](uint32_t i, uint32_t w) {
            return p.trans_a ? get_int(p.A, p.dtype_a, (uint64_t)w * p.lda + i)
                             : get_int(p.A, p.dtype_a, (uint64_t)i * p.lda + w);
          },
          p.D0, p.D1, um, rvecs[k]);
      const Fr bw = mle2(
          [&](uint32_t w, uint32_t j) {
            return p.trans_b ? get_int(p.B, p.dtype_b, (uint64_t)j * p.ldb + w)
                             : get_int(p.B, p.dtype_b, (uint64_t)w * p.ldb + j);
          },
          p.D1, p.D2, rvecs[k], vm);
      if (!fr_eq(aw, finals_a[k]) || !fr_eq(bw, finals_b[k]))
        return fail(VL_ERR_REJECT, "product %u: final values differ from A~(u, r), B~(r, v)", k);
    }
  }
  if (reduced_len) *reduced_len = out.size();
  if (reduced) {
    if (reduced_cap < out.size()) return fail(VL_ERR_BUFFER_TOO_SMALL, "reduced buffer too small");
    for (size_t i = 0; i < out.size(); ++i) memcpy(reduced[i].w, out[i].w, 32);
  }
  if (fail_round) *fail_round = -1;
  return VL_OK;
}
