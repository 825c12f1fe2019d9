// Chained proof of one LoRA layer's training step (vl_lora_chain_prove).
//
// zkMat proves every product and addition of a LoRA step, and the steps are
// composed sequentially (Sec. IV-B): a sumcheck fixes point-value claims, the
// next step justifies exactly those points, and the last claims are left for
// the openings of committed tensors.  The update of eq. (grad_update_ab) is
// proved with zkMat too (the update phase of Protocol 2).  For one layer the
// chain runs in one transcript, in four stages:
//   1. update relation at random points zA, zB: the values UA~, A~, dA~ (and
//      for B) are evaluated on the GPU and UA~ = 2^F A~ - eta dA~ is checked;
//   2. the points of the outputs (zY, zX) and of the product claims that
//      re-quantisation cuts (z2, z4) are squeezed;
//   3. six group sumchecks at those points, in parallel on forked branches of
//      the transcript: {X^T G} = dA, {H^T dY} = dB, {X W + H B} = Y,
//      {dY W^T + G A^T} = dX, {X A} = C2, {dY B^T} = C4;
//   4. the claims left on each of X, W, A, B, dY, H, G reduced to one by a
//      random combination and two sumchecks (rows, then columns), one branch
//      per tensor, all seven in parallel.
// The host squeezes every point and replays each stage's messages (reading
// the proof bytes the kernels wrote) to learn the challenges the next stage
// needs; every contraction, evaluation and sumcheck round runs on the GPU.
// The byte layout and the transcript are those of the oracle's chain module.
#include <hip/hip_runtime.h>

#include <cstring>
#include <string>
#include <vector>

#include "plan.hpp"
#include "sha256.hpp"

namespace vl {
namespace {

constexpr int kGroups = 6, kTensors = 7;
const char* const kTensorNames[kTensors] = {"X", "W", "A", "B", "dY", "H", "G"};

// ------------------------------------------------------------ transcript --
void absorb_bytes(Transcript& t, const char* label, const uint8_t* data, size_t n) {
  Sha256 s;
  sha256_init(s);
  uint8_t st[32];
  tr_to_bytes(t, st);
  sha256_update(s, st, 32);
  sha256_update(s, reinterpret_cast<const uint8_t*>(label), (uint32_t)strlen(label));
  sha256_update(s, data, (uint32_t)n);
  uint8_t d[32];
  sha256_final(s, d);
  tr_from_bytes(t, d);
}

// H(st || label || u32 k), leaving t unchanged
Transcript fork(const Transcript& t, const char* label, uint32_t k) {
  Transcript c = t;
  uint8_t b[4];
  put_u32le(b, k);
  absorb_bytes(c, label, b, 4);
  return c;
}

Transcript chain_init(uint64_t seed, const vl_lora_layer& L) {
  Sha256 s;
  sha256_init(s);
  const char dom[] = "VeriLoRA-chain-v1";
  sha256_update(s, reinterpret_cast<const uint8_t*>(dom), 17);
  uint8_t b[8];
  for (int i = 0; i < 8; ++i) b[i] = (uint8_t)(seed >> (8 * i));
  sha256_update(s, b, 8);
  for (uint32_t v : {L.T, L.d_in, L.d_out, L.r, L.F, L.eta}) {
    put_u32le(b, v);
    sha256_update(s, b, 4);
  }
  uint8_t st[32];
  sha256_final(s, st);
  Transcript t;
  tr_from_bytes(t, st);
  return t;
}

template <int LN>
std::vector<Fr> squeeze_n(Transcript& t, const char (&label)[LN], uint32_t n) {
  std::vector<Fr> v(n);
  for (uint32_t i = 0; i < n; ++i) v[i] = tr_squeeze_fixed(t, label);
  return v;
}

Fr fr_small(uint64_t x) {
  Fr v = fr_zero();
  v.w[0] = (uint32_t)x;
  v.w[1] = (uint32_t)(x >> 32);
  return v;
}

// ---------------------------------------------------------------- shapes --
struct Mat {
  const void* p;
  int dtype;
  uint32_t rows, cols;
};

struct Shapes {
  uint32_t nT, nin, nout, nr;
};

Shapes shapes_of(const vl_lora_layer& L) {
  return {nvars_of(L.T), nvars_of(L.d_in), nvars_of(L.d_out), nvars_of(L.r)};
}

Mat tensor(const vl_lora_layer& L, int k) {
  switch (k) {
    case 0: return {L.X, VL_I16, L.T, L.d_in};
    case 1: return {L.W, VL_I16, L.d_in, L.d_out};
    case 2: return {L.A, VL_I16, L.d_in, L.r};
    case 3: return {L.B, VL_I16, L.r, L.d_out};
    case 4: return {L.dY, VL_I16, L.T, L.d_out};
    case 5: return {L.H, VL_I16, L.T, L.r};
    default: return {L.G, VL_I16, L.T, L.r};
  }
}

constexpr uint32_t kClaimsPerTensor[kTensors] = {3, 2, 3, 3, 3, 2, 2};

vl_product prod(const void* A, bool ta, uint32_t a_rows, uint32_t a_cols, const void* B, bool tb,
                uint32_t b_rows, uint32_t b_cols) {
  vl_product p{};
  p.A = A;
  p.B = B;
  p.dtype_a = p.dtype_b = VL_I16;
  p.D0 = ta ? a_cols : a_rows;
  p.D1 = ta ? a_rows : a_cols;
  p.D2 = tb ? b_rows : b_cols;
  p.lda = a_cols;
  p.ldb = b_cols;
  p.trans_a = ta;
  p.trans_b = tb;
  return p;
}

// The six groups of stage 3 (products with their stored operands) and the
// names of their points: {X^T G} = dA at zA, {H^T dY} = dB at zB,
// {X W, H B} = Y at zY, {dY W^T, G A^T} = dX at zX, {X A} = C2 at z2,
// {dY B^T} = C4 at z4.
struct Stage3 {
  vl_product prods[8];
  vl_group groups[kGroups];
};

void stage3_groups(const vl_lora_layer& L, Stage3& S) {
  const uint32_t T = L.T, di = L.d_in, dout = L.d_out, r = L.r;
  S.prods[0] = prod(L.X, true, T, di, L.G, false, T, r);          // P5 X^T G
  S.prods[1] = prod(L.H, true, T, r, L.dY, false, T, dout);       // P6 H^T dY
  S.prods[2] = prod(L.X, false, T, di, L.W, false, di, dout);     // P1 X W
  S.prods[3] = prod(L.H, false, T, r, L.B, false, r, dout);       // P3 H B
  S.prods[4] = prod(L.dY, false, T, dout, L.W, true, di, dout);   // P7 dY W^T
  S.prods[5] = prod(L.G, false, T, r, L.A, true, di, r);          // P8 G A^T
  S.prods[6] = prod(L.X, false, T, di, L.A, false, di, r);        // P2 X A
  S.prods[7] = prod(L.dY, false, T, dout, L.B, true, r, dout);    // P4 dY B^T
  const struct { int first, n; const void* C; uint32_t ldc; } g[kGroups] = {
      {0, 1, L.dA, r}, {1, 1, L.dB, dout}, {2, 2, L.Y, dout}, {4, 2, L.dX, di}, {6, 1, L.C2, r}, {7, 1, L.C4, r}};
  for (int k = 0; k < kGroups; ++k) {
    S.groups[k] = vl_group{};
    S.groups[k].prods = &S.prods[g[k].first];
    S.groups[k].n_prods = (uint32_t)g[k].n;
    S.groups[k].group_id = (uint32_t)k;
    S.groups[k].C = g[k].C;
    S.groups[k].dtype_c = VL_I64;
    S.groups[k].ldc = g[k].ldc;
  }
}

uint64_t reduce_bytes(uint32_t rows, uint32_t cols, uint32_t K) {
  return 32ull * (3ull * nvars_of(rows) + K + 3ull * nvars_of(cols) + 1);
}

uint64_t chain_len(const vl_lora_layer& L, uint64_t* group_off, uint64_t* reduce_off) {
  Stage3 S;
  stage3_groups(L, S);
  uint64_t o = 6 * 32;
  for (int k = 0; k < kGroups; ++k) {
    if (group_off) group_off[k] = o;
    o += 32 * proof_elems(S.groups[k]);
  }
  for (int j = 0; j < kTensors; ++j) {
    if (reduce_off) reduce_off[j] = o;
    const Mat m = tensor(L, j);
    o += reduce_bytes(m.rows, m.cols, kClaimsPerTensor[j]);
  }
  return o;
}

vl_status check_layer(const vl_lora_layer* L, bool need_ptrs) {
  if (!L) return fail(VL_ERR_INVALID_ARG, "null layer");
  if (!L->T || !L->d_in || !L->d_out || !L->r || L->T > VL_MAX_DIM || L->d_in > VL_MAX_DIM ||
      L->d_out > VL_MAX_DIM || L->r > VL_MAX_DIM)
    return fail(VL_ERR_SHAPE, "layer dims must be 1..2^20");
  if (L->F > 62) return fail(VL_ERR_INVALID_ARG, "F must be <= 62");
  if ((uint64_t)L->T + L->r > (1u << 16) || (uint64_t)L->d_in + L->r > (1u << 16) ||
      (uint64_t)L->d_out + L->r > (1u << 16))
    return fail(VL_ERR_SHAPE, "inner dimensions of the layer's sums must be <= 2^16");
  if (need_ptrs) {
    const void* ps[] = {L->X, L->W, L->A, L->B, L->dY, L->H, L->G, L->Y, L->C2, L->C4, L->dA, L->dB, L->dX,
                        L->UA, L->UB};
    for (const void* p : ps)
      if (!p) return fail(VL_ERR_INVALID_ARG, "null tensor");
  }
  return VL_OK;
}

// ----------------------------------------------------------------- plans --
Tuning chain_tuning() {
  Tuning t;
  t.per_instance = false;
  t.min_tasks = 1;
  t.segments = 1;
  return t;
}

// builds a plan whose blob sits at base and data after it: fill(B) adds the
// jobs; run twice, once to size the blob, once at the final offsets
template <typename Fill>
uint64_t build_plan(Plan& P, const Tuning& T, uint8_t* base, Fill&& fill) {
  uint64_t blob = 0;
  for (int pass = 0; pass < 2; ++pass) {
    P = Plan();
    Builder B(P, T, reinterpret_cast<uint64_t>(base), blob);
    fill(B);
    P.data_end = B.off;
    if (pass == 0) blob = align_up(blob_layout(P).total, 256);
  }
  return P.data_end;
}

// an evaluation job M~(x, y) (canonical, 32 bytes at out): contraction over
// the rows with eq(x, .) in e R^2 digits, then the dot with eq(y, .)
// canonical; the range flag is the plan's flag `flag`
void add_eval(Builder& B, const Mat& m, const std::vector<Fr>& x, const std::vector<Fr>& y, uint8_t* out,
              int32_t* status, uint32_t flag) {
  const uint64_t Lc = 1ull << y.size();
  uint32_t* packX = B.dev<uint32_t>(B.take((uint64_t)m.rows * 32));
  uint32_t* eqY = B.dev<uint32_t>(B.take(8 * Lc * 4));
  uint32_t* svec = B.dev<uint32_t>(B.take(8 * Lc * 4));
  int32_t* err = reinterpret_cast<int32_t*>(B.base) + flag;
  B.eq_job(x, nullptr, packX, m.rows, true, false);
  B.eq_job(y, eqY, nullptr, 0, false, true);
  B.contract(m.p, m.dtype, digits_for(m.dtype), m.cols, true, m.cols, m.rows, packX, svec, Lc, Lc, err);
  uint32_t nparts = 0;
  const uint32_t* part = B.pass1(eqY, Lc, svec, Lc, (uint32_t)Lc, true, nparts, nullptr);
  EvalJob e{};
  e.part = part;
  e.nparts = nparts;
  e.out = out;
  e.err = err;
  e.status = status;
  B.P.evals.push_back(e);
}

struct Claim {
  std::vector<Fr> x, y;   // row and column point (canonical)
  Fr v;                   // value (canonical)
};

struct GroupOut {
  Fr c;
  std::vector<std::vector<Fr>> r;                 // per product, canonical
  std::vector<std::pair<Fr, Fr>> finals;          // per product (a_final, b_final)
};

// replays a group's sumcheck messages (the bytes the rounds kernel wrote) on
// the transcript of its branch: the challenges and finals of every product
void replay_group(Transcript& tr, const vl_group& g, const uint8_t* proof, GroupOut& o) {
  const uint8_t* p = proof;
  o.c = fr_from_bytes(p);
  p += 32;
  {
    const Fr cc[1] = {o.c};
    tr_absorb_frs(tr, VL_LBL_CLAIM, cc);
  }
  for (uint32_t k = 0; k + 1 < g.n_prods; ++k) {
    const Fr sc[1] = {fr_from_bytes(p)};
    p += 32;
    tr_absorb_frs(tr, VL_LBL_PART, sc);
  }
  o.r.assign(g.n_prods, {});
  o.finals.assign(g.n_prods, {});
  for (uint32_t k = 0; k < g.n_prods; ++k) {
    const uint32_t n1 = nvars_of(g.prods[k].D1);
    for (uint32_t i = 0; i < n1; ++i) {
      const Fr gc[3] = {fr_from_bytes(p), fr_from_bytes(p + 32), fr_from_bytes(p + 64)};
      p += 96;
      tr_absorb_frs(tr, VL_LBL_ROUND, gc);
      o.r[k].push_back(tr_squeeze_fixed(tr, VL_LBL_R));
    }
    const Fr fin[2] = {fr_from_bytes(p), fr_from_bytes(p + 32)};
    p += 64;
    tr_absorb_frs(tr, VL_LBL_FINAL, fin);
    o.finals[k] = {fin[0], fin[1]};
  }
}

std::vector<Fr> head(const std::vector<Fr>& z, uint32_t n) { return std::vector<Fr>(z.begin(), z.begin() + n); }
std::vector<Fr> tail(const std::vector<Fr>& z, uint32_t n) { return std::vector<Fr>(z.begin() + n, z.end()); }

}  // namespace

// Sizes (ws == nullptr: *ws_need gets the workspace bytes) or proves the
// chain; the same planning code does both, so the two cannot disagree.
static vl_status chain_run(const vl_lora_layer& L, uint64_t seed, uint8_t* ws, uint64_t ws_bytes,
                           uint8_t* proof_out, uint8_t* digest_out, hipStream_t s, uint64_t* ws_need) {
  const Shapes N = shapes_of(L);
  const bool sizing = ws == nullptr;
  const Tuning T = chain_tuning();
  uint64_t goff[kGroups], roff[kTensors];
  const uint64_t plen = chain_len(L, goff, roff);
  // pinned output region: [proof][status words][digests]
  const uint64_t st_off = align_up(plen, 256), dg_off = st_off + 256;
  const uint64_t out_bytes = dg_off + 32 * (kGroups + kTensors);
  PinnedOut* po = nullptr;
  uint8_t* oh = nullptr;   // host view
  uint8_t* od = nullptr;   // device view
  if (!sizing) {
    const hipError_t e = pinned_out(out_bytes, &po);
    if (e != hipSuccess) return fail(VL_ERR_HIP, "pinned output buffer: %s", hipGetErrorString(e));
    oh = reinterpret_cast<uint8_t*>(po->host);
    od = reinterpret_cast<uint8_t*>(po->dev);
    memset(oh, 0, out_bytes);
    memset(oh + st_off, 0xff, 4 * (kGroups + kTensors + 8));
  }
  int32_t* status_d = sizing ? nullptr : reinterpret_cast<int32_t*>(od + st_off);
  const int32_t* status_h = sizing ? nullptr : reinterpret_cast<const int32_t*>(oh + st_off);
  auto run = [&](Plan& P) -> vl_status {
    if (P.data_end > ws_bytes)
      return fail(VL_ERR_WORKSPACE, "workspace of %llu bytes, %llu needed", (unsigned long long)ws_bytes,
                  (unsigned long long)align_up(P.data_end, 256));
    const BlobLayout BL = blob_layout(P);
    fill_blob(P, BL, ws);
    hipError_t e = enqueue_plan(P, BL, ws, s, s, nullptr);
    const hipError_t e2 = hipStreamSynchronize(s);
    if (e == hipSuccess) e = e2;
    if (e != hipSuccess) return fail(VL_ERR_HIP, "chain: %s", hipGetErrorString(e));
    return VL_OK;
  };
  auto bad_status = [&](int first, int n) -> vl_status {
    for (int i = first; i < first + n; ++i) {
      const int32_t st = status_h[i];
      if (st == VL_ERR_FALSE_STATEMENT) return fail(VL_ERR_FALSE_STATEMENT, "chain step %d: false statement", i);
      if (st == VL_ERR_RANGE) return fail(VL_ERR_RANGE, "chain step %d: an entry exceeds the digit range", i);
      if (st != VL_OK) return fail(VL_ERR_HIP, "chain step %d: status %d", i, st);
    }
    return VL_OK;
  };

  // ---- stage 1: the update relation at zA, zB
  Transcript tr = chain_init(seed, L);
  const std::vector<Fr> zA = squeeze_n(tr, "zA", N.nin + N.nr);
  const std::vector<Fr> zB = squeeze_n(tr, "zB", N.nr + N.nout);
  Plan P1;
  const Mat mUA{L.UA, VL_I64, L.d_in, L.r}, mA{L.A, VL_I16, L.d_in, L.r}, mdA{L.dA, VL_I64, L.d_in, L.r};
  const Mat mUB{L.UB, VL_I64, L.r, L.d_out}, mB{L.B, VL_I16, L.r, L.d_out}, mdB{L.dB, VL_I64, L.r, L.d_out};
  const uint64_t s1 = build_plan(P1, T, ws, [&](Builder& B) {
    B.P.n_err = 6;
    const Mat ms[6] = {mUA, mA, mdA, mUB, mB, mdB};
    for (uint32_t i = 0; i < 6; ++i) {
      const std::vector<Fr>& z = i < 3 ? zA : zB;
      const uint32_t nrow = i < 3 ? N.nin : N.nr;
      add_eval(B, ms[i], head(z, nrow), tail(z, nrow), od ? od + 32 * i : nullptr, status_d ? status_d + i : nullptr,
               i);
    }
  });
  Fr upd[6];
  if (!sizing) {
    vl_status st = run(P1);
    if (st == VL_OK) st = bad_status(0, 6);
    if (st != VL_OK) return st;
    for (int i = 0; i < 6; ++i) upd[i] = fr_from_bytes(oh + 32 * i);
    const Fr twoF = fr_to_mont(fr_small(1ull << L.F)), eta = fr_to_mont(fr_small(L.eta));
    for (int u = 0; u < 2; ++u) {
      const Fr U = fr_to_mont(upd[3 * u]), X0 = fr_to_mont(upd[3 * u + 1]), D = fr_to_mont(upd[3 * u + 2]);
      if (!fr_eq(U, fr_sub(fr_mul(twoF, X0), fr_mul(eta, D))))
        return fail(VL_ERR_FALSE_STATEMENT, "%s differs from 2^F %s - eta %s", u ? "UB" : "UA", u ? "B" : "A",
                    u ? "dB" : "dA");
    }
    absorb_bytes(tr, "upd", oh, 6 * 32);
  }

  // ---- stage 2: points of the outputs and cut products
  const std::vector<Fr> zY = squeeze_n(tr, "zY", N.nT + N.nout);
  const std::vector<Fr> zX = squeeze_n(tr, "zX", N.nT + N.nin);
  const std::vector<Fr> z2 = squeeze_n(tr, "z2", N.nT + N.nr);
  const std::vector<Fr> z4 = squeeze_n(tr, "z4", N.nT + N.nr);

  // ---- stage 3: group sumchecks at those points, one branch each
  Stage3 S;
  stage3_groups(L, S);
  const std::vector<Fr>* zs[kGroups] = {&zA, &zB, &zY, &zX, &z2, &z4};
  const uint32_t nrow[kGroups] = {N.nin, N.nr, N.nT, N.nT, N.nT, N.nT};
  std::vector<Challenges> ch(kGroups);
  for (int k = 0; k < kGroups; ++k) {
    ch[k].tr = fork(tr, "fork", (uint32_t)k);
    ch[k].u = head(*zs[k], nrow[k]);
    ch[k].v = tail(*zs[k], nrow[k]);
  }
  uint64_t offs[kGroups + 1];
  for (int k = 0; k < kGroups; ++k) offs[k] = goff[k] - goff[0];
  offs[kGroups] = plen;
  Plan P3;
  plan_groups(P3, T, S.groups, 0, kGroups, 0, sizing ? nullptr : ws, true, od ? od + goff[0] : nullptr, offs,
              status_d ? status_d + 6 : nullptr, od ? od + dg_off : nullptr, nullptr, ch.data());
  const uint64_t s3 = P3.data_end;
  GroupOut go[kGroups];
  if (!sizing) {
    vl_status st = run(P3);
    if (st == VL_OK) st = bad_status(6, kGroups);
    if (st != VL_OK) return st;
    uint8_t joined[32 * kGroups];
    for (int k = 0; k < kGroups; ++k) {
      Transcript br = ch[k].tr;
      replay_group(br, S.groups[k], oh + goff[k], go[k]);
      uint8_t d[32];
      tr_to_bytes(br, d);
      if (memcmp(d, oh + dg_off + 32 * k, 32) != 0)
        return fail(VL_ERR_HIP, "chain: group %d's transcript differs from its replay", k);
      memcpy(joined + 32 * k, d, 32);
    }
    if (!fr_eq(go[0].c, upd[2]) || !fr_eq(go[1].c, upd[5]))
      return fail(VL_ERR_HIP, "chain: a gradient's claim differs from its update evaluation");
    absorb_bytes(tr, "join", joined, sizeof joined);
  }

  // ---- stage 4: the claims left on each tensor, reduced to one
  // (the same collection as the oracle's: an operand used transposed leaves
  // (M^T)~(x, y) = M~(y, x))
  std::vector<Claim> claims[kTensors];
  if (!sizing) {
    auto cl = [](const std::vector<Fr>& x, const std::vector<Fr>& y, const Fr& v) { return Claim{x, y, v}; };
    const std::vector<Fr> zAu = head(zA, N.nin), zAv = tail(zA, N.nin), zBu = head(zB, N.nr), zBv = tail(zB, N.nr);
    const std::vector<Fr> zYu = head(zY, N.nT), zYv = tail(zY, N.nT), zXu = head(zX, N.nT), zXv = tail(zX, N.nT);
    const std::vector<Fr> z2u = head(z2, N.nT), z2v = tail(z2, N.nT), z4u = head(z4, N.nT), z4v = tail(z4, N.nT);
    const GroupOut &g5 = go[0], &g6 = go[1], &gY = go[2], &gX = go[3], &g2 = go[4], &g4 = go[5];
    claims[0] = {cl(zYu, gY.r[0], gY.finals[0].first), cl(z2u, g2.r[0], g2.finals[0].first),
                 cl(g5.r[0], zAu, g5.finals[0].first)};
    claims[1] = {cl(gY.r[0], zYv, gY.finals[0].second), cl(zXv, gX.r[0], gX.finals[0].second)};
    claims[2] = {cl(zAu, zAv, upd[1]), cl(g2.r[0], z2v, g2.finals[0].second), cl(zXv, gX.r[1], gX.finals[1].second)};
    claims[3] = {cl(zBu, zBv, upd[4]), cl(gY.r[1], zYv, gY.finals[1].second), cl(z4v, g4.r[0], g4.finals[0].second)};
    claims[4] = {cl(z4u, g4.r[0], g4.finals[0].first), cl(g6.r[0], zBv, g6.finals[0].second),
                 cl(zXu, gX.r[0], gX.finals[0].first)};
    claims[5] = {cl(zYu, gY.r[1], gY.finals[1].first), cl(g6.r[0], zBu, g6.finals[0].first)};
    claims[6] = {cl(g5.r[0], zAv, g5.finals[0].second), cl(zXu, gX.r[1], gX.finals[1].first)};
  } else {
    for (int j = 0; j < kTensors; ++j) {
      const Mat m = tensor(L, j);
      claims[j].assign(kClaimsPerTensor[j],
                       Claim{std::vector<Fr>(nvars_of(m.rows), fr_zero()), std::vector<Fr>(nvars_of(m.cols), fr_zero()),
                             fr_zero()});
    }
  }
  // branches, rho squeezes (host); tables and rounds (device)
  Transcript rb[kTensors];
  std::vector<Fr> rho[kTensors];
  for (int j = 0; j < kTensors; ++j) {
    rb[j] = fork(tr, "rfork", (uint32_t)j);
    std::vector<uint8_t> vals;
    for (const Claim& c : claims[j]) {
      uint8_t b[32];
      fr_to_bytes(c.v, b);
      vals.insert(vals.end(), b, b + 32);
    }
    absorb_bytes(rb[j], "rclaims", vals.data(), vals.size());
    rho[j] = squeeze_n(rb[j], "rho", (uint32_t)claims[j].size());
  }
  // plan A: eq tables, the column contractions t_k, phase 1; plan B (after
  // it, at data offsets beyond it): eq(r, .) from the row challenges phase 1
  // wrote, the row contraction M~(r, .), phase 2
  struct RedBufs {
    uint32_t* io;
    uint32_t* ey[kMaxClaims];
  } rbufs[kTensors];
  Plan PA;
  const uint64_t s4a = build_plan(PA, T, ws, [&](Builder& B) {
    B.P.n_err = kTensors;
    for (int j = 0; j < kTensors; ++j) {
      const Mat m = tensor(L, j);
      const uint32_t nR = nvars_of(m.rows), nC = nvars_of(m.cols), K = (uint32_t)claims[j].size();
      const uint64_t LR = 1ull << nR, LC = 1ull << nC;
      int32_t* err = reinterpret_cast<int32_t*>(B.base) + j;
      ReduceJob rj{};
      Transcript st = rb[j];
      memcpy(rj.st, st.h, 32);
      rj.phase = 1;
      rj.K = K;
      rj.n = nR;
      rj.ld = LR;
      rbufs[j].io = B.dev<uint32_t>(B.take(4ull * reduce_io_words(nR)));
      rj.io = rbufs[j].io;
      for (uint32_t k = 0; k < K; ++k) {
        const Claim& c = claims[j][k];
        const Fr rm = fr_to_mont(rho[j][k]);
        memcpy(rj.coef[k], rm.w, 32);
        rj.a[k] = B.dev<uint32_t>(B.take(8 * LR * 4));
        rj.b[k] = B.dev<uint32_t>(B.take(8 * LR * 4));
        uint32_t* packY = B.dev<uint32_t>(B.take((uint64_t)m.cols * 32));
        rbufs[j].ey[k] = B.dev<uint32_t>(B.take(8 * LC * 4));
        B.eq_job(c.x, rj.a[k], nullptr, 0, false, false);              // eq(x_k, .), Montgomery
        B.eq_job(c.y, rbufs[j].ey[k], packY, m.cols, false, true);     // eq(y_k, .): canonical + e R digits
        B.contract(m.p, m.dtype, digits_for(m.dtype), m.cols, false, m.rows, m.cols, packY, rj.b[k], LR, LR, err);
      }
      rj.proof = od ? od + roff[j] : nullptr;
      B.P.reduces.push_back(rj);
    }
  });
  Plan PB;
  const uint64_t s4b = build_plan(PB, T, ws + (sizing ? 0 : align_up(s4a, 256)), [&](Builder& B) {
    B.P.n_err = kTensors;
    for (int j = 0; j < kTensors; ++j) {
      const Mat m = tensor(L, j);
      const uint32_t nR = nvars_of(m.rows), nC = nvars_of(m.cols), K = (uint32_t)claims[j].size();
      const uint64_t LC = 1ull << nC;
      int32_t* err = reinterpret_cast<int32_t*>(B.base) + j;
      ReduceJob rj{};
      rj.phase = 2;
      rj.K = K;
      rj.n = nC;
      rj.ld = LC;
      rj.io = rbufs[j].io;
      uint32_t* packR = B.dev<uint32_t>(B.take((uint64_t)m.rows * 32));
      rj.a[0] = B.dev<uint32_t>(B.take(8 * LC * 4));
      rj.bsum = B.dev<uint32_t>(B.take(8 * LC * 4));
      for (uint32_t k = 0; k < K; ++k) rj.b[k] = rbufs[j].ey[k];
      B.eq_job_dev(nR, rbufs[j].io ? rbufs[j].io + kReduceIoR : nullptr, nullptr, packR, m.rows, true, false);
      B.contract(m.p, m.dtype, digits_for(m.dtype), m.cols, true, m.cols, m.rows, packR, rj.a[0], LC, LC, err);
      rj.proof = od ? od + roff[j] + 32ull * (3ull * nR + K) : nullptr;
      rj.digest = od ? od + dg_off + 32 * (kGroups + j) : nullptr;
      rj.status = status_d ? status_d + 12 + j : nullptr;
      B.P.reduces.push_back(rj);
    }
  });
  const uint64_t s4 = align_up(s4a, 256) + s4b;
  if (sizing) {
    *ws_need = align_up(std::max(std::max(s1, s3), s4), 256);
    return VL_OK;
  }
  {
    // the two plans run back to back on the stream: B's eq job reads the row
    // challenges A's reduce kernel wrote
    if (s4 > ws_bytes)
      return fail(VL_ERR_WORKSPACE, "workspace of %llu bytes, %llu needed", (unsigned long long)ws_bytes,
                  (unsigned long long)align_up(s4, 256));
    const BlobLayout LA = blob_layout(PA), LB = blob_layout(PB);
    fill_blob(PA, LA, ws);
    uint8_t* wsb = ws + align_up(s4a, 256);
    fill_blob(PB, LB, wsb);
    hipError_t e = enqueue_plan(PA, LA, ws, s, s, nullptr);
    if (e == hipSuccess) e = enqueue_plan(PB, LB, wsb, s, s, nullptr);
    const hipError_t e2 = hipStreamSynchronize(s);
    if (e == hipSuccess) e = e2;
    if (e != hipSuccess) return fail(VL_ERR_HIP, "chain: %s", hipGetErrorString(e));
    const vl_status st = bad_status(12, kTensors);
    if (st != VL_OK) return st;
  }
  uint8_t joined[32 * kTensors];
  memcpy(joined, oh + dg_off + 32 * kGroups, sizeof joined);
  absorb_bytes(tr, "join", joined, sizeof joined);
  memcpy(proof_out, oh, plen);
  if (digest_out) tr_to_bytes(tr, digest_out);
  return VL_OK;
}

}  // namespace vl

using namespace vl;

extern "C" {

uint64_t vl_lora_chain_proof_size(const vl_lora_layer* L) {
  if (check_layer(L, false) != VL_OK) return 0;
  return chain_len(*L, nullptr, nullptr);
}

uint64_t vl_lora_chain_workspace_size(const vl_lora_layer* L) {
  if (check_layer(L, false) != VL_OK) return 0;
  uint64_t need = 0;
  if (chain_run(*L, 0, nullptr, 0, nullptr, nullptr, nullptr, &need) != VL_OK) return 0;
  return need;
}

vl_status vl_lora_chain_prove(const vl_lora_layer* L, uint64_t seed, void* workspace, uint64_t workspace_bytes,
                              uint8_t* proof, uint64_t proof_len, uint8_t* digest, void* stream) {
  {
    const vl_status st = check_layer(L, true);
    if (st != VL_OK) return st;
  }
  if (!proof) return fail(VL_ERR_INVALID_ARG, "null proof buffer");
  if (!workspace) return fail(VL_ERR_WORKSPACE, "no workspace");
  if (reinterpret_cast<uintptr_t>(workspace) % 256) return fail(VL_ERR_WORKSPACE, "workspace must be 256-byte aligned");
  const uint64_t need = chain_len(*L, nullptr, nullptr);
  if (proof_len < need)
    return fail(VL_ERR_BUFFER_TOO_SMALL, "proof buffer holds %llu bytes, %llu needed", (unsigned long long)proof_len,
                (unsigned long long)need);
  return chain_run(*L, seed, reinterpret_cast<uint8_t*>(workspace), workspace_bytes, proof, digest,
                   reinterpret_cast<hipStream_t>(stream), nullptr);
}

}  // extern "C"
