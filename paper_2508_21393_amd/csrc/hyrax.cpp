// Hyrax commitments: parameter checks, launch planning and the host side
// (vl_hyrax_setup, vl_hyrax_commit, vl_hyrax_generators,
// vl_hyrax_verify_open).
//
// Sec. II-A's polynomial commitments, instantiated with Hyrax as the
// paper's implementation does: the MLE of an R x m matrix M is committed row
// by row, C_i = sum_j M[i][j] G_j, and opened at (x, y) with the vector
// w = sum_i eq(x, i) M[i][.] (the partial evaluation vl_mle_partial_eval
// computes), which the verifier checks against the commitments through
// sum_j w_j G_j = sum_i eq(x, i) C_i before it takes the value
// sum_j w_j eq(y, j).  The device work is in hyrax.hip; the verifier's two
// multi-scalar multiplications run on the host with Pippenger's bucket
// method.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <mutex>
#include <thread>
#include <vector>

#include "fq.hpp"
#include "plan.hpp"

namespace vl {
namespace {

constexpr uint64_t kPointBytes = 96;
constexpr uint64_t kTablePoints = 128;
constexpr uint32_t kMaxGens = 1u << 20;
constexpr uint32_t kMaxRows = 1u << 24;
constexpr uint64_t kTargetTasks = 4096;   // waves that fill the GPU a few times over
constexpr uint32_t kMinSlice = 256;       // columns per task (4 per lane) at the least

vl_status check_setup(uint32_t m, uint32_t W) {
  if (m == 0 || m > kMaxGens) return fail(VL_ERR_SHAPE, "hyrax: m must be in 1 .. 2^20");
  if (W == 0 || W > 8) return fail(VL_ERR_INVALID_ARG, "hyrax: windows must be in 1 .. 8");
  return VL_OK;
}

struct Split {
  uint32_t n_split, chunk;
};

Split plan_split(uint32_t R, uint32_t m, uint32_t split) {
  uint64_t n = split;
  if (n == 0) {
    n = (kTargetTasks + R - 1) / R;
    n = std::min<uint64_t>(n, (m + kMinSlice - 1) / kMinSlice);
  }
  n = std::max<uint64_t>(1, std::min<uint64_t>(n, (m + 63) / 64));
  const uint64_t chunk = align_up((m + n - 1) / n, 64);
  Split s;
  s.chunk = (uint32_t)chunk;
  s.n_split = (uint32_t)((m + chunk - 1) / chunk);
  return s;
}

// ---- host G1 helpers ------------------------------------------------------

bool decode_point(const uint8_t* b, bool& inf, G1a& a) {
  inf = true;
  for (int i = 0; i < 96; ++i)
    if (b[i]) inf = false;
  if (inf) return true;
  const Fq x = fq_from_bytes(b), y = fq_from_bytes(b + 48);
  if (!fq_lt_q(x) || !fq_lt_q(y)) return false;
  a.x = fq_to_mont(x);
  a.y = fq_to_mont(y);
  return g1_on_curve(a);
}

void encode_affine(const G1a& a, uint8_t* out) {
  fq_to_bytes(fq_from_mont(a.x), out);
  fq_to_bytes(fq_from_mont(a.y), out + 48);
}

bool g1_same(const G1z& a, const G1z& b) {
  if (g1_is_inf(a) || g1_is_inf(b)) return g1_is_inf(a) && g1_is_inf(b);
  // X1 ZZ2 = X2 ZZ1 and Y1 ZZZ2 = Y2 ZZZ1
  return fq_eq(fq_mul(a.X, b.ZZ), fq_mul(b.X, a.ZZ)) && fq_eq(fq_mul(a.Y, b.ZZZ), fq_mul(b.Y, a.ZZZ));
}

// scalar bits c*k .. c*k + c - 1 of a canonical element
uint32_t window_of(const Fr& s, uint32_t bit, uint32_t c) {
  uint32_t v = 0;
  for (uint32_t b = 0; b < c; ++b) {
    const uint32_t i = bit + b;
    if (i < 256 && ((s.w[i >> 5] >> (i & 31)) & 1u)) v |= 1u << b;
  }
  return v;
}

// sum_k s_k P_k by Pippenger's bucket method (canonical scalars, affine
// points; infinity points are left out by the caller)
G1z msm_host(const std::vector<Fr>& s, const std::vector<G1a>& P) {
  const size_t n = P.size();
  uint32_t c = 4;
  while (c < 16 && (1ull << (c + 2)) < n) ++c;
  const uint32_t nb = (1u << c) - 1;
  std::vector<G1z> bucket(nb);
  G1z acc = g1_infinity();
  const int nwin = (int)((255 + c - 1) / c);
  for (int win = nwin - 1; win >= 0; --win) {
    for (uint32_t k = 0; k < c; ++k) acc = g1_dbl(acc);
    std::fill(bucket.begin(), bucket.end(), g1_infinity());
    for (size_t i = 0; i < n; ++i) {
      const uint32_t d = window_of(s[i], (uint32_t)win * c, c);
      if (d) bucket[d - 1] = g1_add_affine(bucket[d - 1], P[i]);
    }
    G1z run = g1_infinity(), tot = g1_infinity();
    for (int b = (int)nb - 1; b >= 0; --b) {
      run = g1_add(run, bucket[b]);
      tot = g1_add(tot, run);
    }
    acc = g1_add(acc, tot);
  }
  return acc;
}

// p G for the group order p: the point at infinity iff G lies in the
// order-p subgroup
bool in_subgroup(const G1a& a) {
  const G1z P = g1_from_affine(a);
  G1z acc = g1_infinity();
  for (int i = 254; i >= 0; --i) {
    acc = g1_dbl(acc);
    if ((p_limb(i >> 5) >> (i & 31)) & 1u) acc = g1_add(acc, P);
  }
  return g1_is_inf(acc);
}

// generators, computed once per process and kept (the hash to the curve
// costs two exponentiations per try)
std::mutex g_gen_mu;
std::vector<G1a> g_gens;

vl_status host_generators(uint32_t m, std::vector<G1a>& out) {
  std::lock_guard<std::mutex> lk(g_gen_mu);
  if (g_gens.size() < m) {
    const uint32_t from = (uint32_t)g_gens.size();
    std::vector<G1a> add(m - from);
    std::vector<char> ok(m - from, 1);
    const uint32_t nt = std::max(1u, std::min<uint32_t>(16, std::thread::hardware_concurrency()));
    std::vector<std::thread> th;
    for (uint32_t t = 0; t < nt; ++t)
      th.emplace_back([&, t] {
        for (uint32_t j = from + t; j < m; j += nt) ok[j - from] = hyrax_generator(j, add[j - from]) ? 1 : 0;
      });
    for (auto& x : th) x.join();
    for (char o : ok)
      if (!o) return fail(VL_ERR_INVALID_ARG, "hyrax: a generator did not hash to the curve");
    g_gens.insert(g_gens.end(), add.begin(), add.end());
  }
  out.assign(g_gens.begin(), g_gens.begin() + m);
  return VL_OK;
}

}  // namespace
}  // namespace vl

using namespace vl;

extern "C" {

uint64_t vl_hyrax_table_size(uint32_t m, uint32_t windows) {
  if (check_setup(m, windows) != VL_OK) return 0;
  return (uint64_t)m * windows * kTablePoints * kPointBytes;
}

vl_status vl_hyrax_setup(uint32_t m, uint32_t windows, void* table, uint64_t table_bytes, void* stream) {
  vl_status st = check_setup(m, windows);
  if (st != VL_OK) return st;
  if (!table) return fail(VL_ERR_INVALID_ARG, "hyrax: null table");
  if ((uintptr_t)table % 16) return fail(VL_ERR_INVALID_ARG, "hyrax: the table must be 16-byte aligned");
  if (table_bytes < vl_hyrax_table_size(m, windows))
    return fail(VL_ERR_BUFFER_TOO_SMALL, "hyrax: table of %llu bytes, %llu needed", (unsigned long long)table_bytes,
                (unsigned long long)vl_hyrax_table_size(m, windows));
  hipError_t e = launch_hyrax_setup(m, windows, reinterpret_cast<uint32_t*>(table), reinterpret_cast<hipStream_t>(stream));
  if (e != hipSuccess) return fail(VL_ERR_HIP, "hyrax setup: %s", hipGetErrorString(e));
  return VL_OK;
}

uint64_t vl_hyrax_commit_workspace_size(uint32_t R, uint32_t m, uint32_t split) {
  if (R == 0 || m == 0 || R > kMaxRows || m > kMaxGens) return 0;
  const Split s = plan_split(R, m, split);
  return align_up((uint64_t)R * s.n_split * 48 * 4, 256);
}

vl_status vl_hyrax_commit(const void* M, int32_t dtype, uint32_t R, uint32_t m, uint64_t ld, const void* table,
                          uint32_t table_m, uint32_t windows, uint32_t split, void* commits, void* workspace,
                          uint64_t workspace_bytes, void* stream) {
  if (!M || !table || !commits) return fail(VL_ERR_INVALID_ARG, "hyrax commit: null pointer");
  if (dtype != VL_I16 && dtype != VL_I32 && dtype != VL_I64)
    return fail(VL_ERR_DTYPE, "hyrax commit: entries must be int16, int32 or int64");
  if (R == 0 || m == 0 || R > kMaxRows) return fail(VL_ERR_SHAPE, "hyrax commit: R must be in 1 .. 2^24, m >= 1");
  if (ld < m) return fail(VL_ERR_SHAPE, "hyrax commit: ld < m");
  vl_status st = check_setup(table_m, windows);
  if (st != VL_OK) return st;
  if (m > table_m) return fail(VL_ERR_SHAPE, "hyrax commit: m = %u exceeds the table's %u generators", m, table_m);
  if (windows < esize(dtype))
    return fail(VL_ERR_INVALID_ARG, "hyrax commit: %d-byte entries need a table of >= %d windows", (int)esize(dtype),
                (int)esize(dtype));
  if ((uintptr_t)table % 16 || (uintptr_t)commits % 4)
    return fail(VL_ERR_INVALID_ARG, "hyrax commit: table must be 16-byte, commits 4-byte aligned");
  if (split > (m + 63) / 64) return fail(VL_ERR_INVALID_ARG, "hyrax commit: split exceeds ceil(m / 64)");
  const uint64_t need = vl_hyrax_commit_workspace_size(R, m, split);
  if (!workspace || workspace_bytes < need)
    return fail(VL_ERR_WORKSPACE, "hyrax commit: workspace of %llu bytes, %llu needed",
                (unsigned long long)workspace_bytes, (unsigned long long)need);
  const Split s = plan_split(R, m, split);
  hipError_t e = launch_hyrax_commit(M, dtype, ld, R, m, windows, reinterpret_cast<const uint32_t*>(table), s.n_split,
                                     s.chunk, reinterpret_cast<uint32_t*>(workspace),
                                     reinterpret_cast<uint32_t*>(commits), reinterpret_cast<hipStream_t>(stream));
  if (e != hipSuccess) return fail(VL_ERR_HIP, "hyrax commit: %s", hipGetErrorString(e));
  return VL_OK;
}

vl_status vl_hyrax_generators(uint32_t m, uint8_t* out) {
  if (!out) return fail(VL_ERR_INVALID_ARG, "hyrax generators: null output");
  if (m == 0 || m > kMaxGens) return fail(VL_ERR_SHAPE, "hyrax generators: m must be in 1 .. 2^20");
  std::vector<G1a> g;
  vl_status st = host_generators(m, g);
  if (st != VL_OK) return st;
  for (uint32_t j = 0; j < m; ++j) encode_affine(g[j], out + kPointBytes * j);
  return VL_OK;
}

vl_status vl_hyrax_verify_open(const uint8_t* commits, uint32_t R, uint32_t m, const vl_fr* x, const vl_fr* y,
                               const vl_fr* w, vl_fr* value) {
  if (!commits || !w || (!x && nvars_of(R)) || (!y && nvars_of(m)))
    return fail(VL_ERR_INVALID_ARG, "hyrax verify: null pointer");
  if (R == 0 || m == 0 || R > kMaxRows || m > kMaxGens) return fail(VL_ERR_SHAPE, "hyrax verify: bad R or m");
  const uint32_t nx = nvars_of(R), ny = nvars_of(m);
  std::vector<Fr> xm(nx), ym(ny), wc(m);
  for (uint32_t k = 0; k < nx; ++k) {
    Fr v;
    memcpy(v.w, x[k].w, 32);
    if (!fr_lt_p(v)) return fail(VL_ERR_REJECT, "hyrax verify: x[%u] is not canonical", k);
    xm[k] = fr_to_mont(v);
  }
  for (uint32_t k = 0; k < ny; ++k) {
    Fr v;
    memcpy(v.w, y[k].w, 32);
    if (!fr_lt_p(v)) return fail(VL_ERR_REJECT, "hyrax verify: y[%u] is not canonical", k);
    ym[k] = fr_to_mont(v);
  }
  for (uint32_t j = 0; j < m; ++j) {
    memcpy(wc[j].w, w[j].w, 32);
    if (!fr_lt_p(wc[j])) return fail(VL_ERR_REJECT, "hyrax verify: w[%u] is not canonical", j);
  }
  // the commitments: canonical points of the curve in the order-p subgroup
  std::vector<Fr> ex = eq_host(xm);
  std::vector<Fr> cs;
  std::vector<G1a> cp;
  for (uint32_t i = 0; i < R; ++i) {
    bool inf;
    G1a a;
    if (!decode_point(commits + kPointBytes * i, inf, a))
      return fail(VL_ERR_REJECT, "hyrax verify: commitment %u is not a canonical curve point", i);
    if (inf) continue;
    if (!in_subgroup(a)) return fail(VL_ERR_REJECT, "hyrax verify: commitment %u is outside the group", i);
    cs.push_back(fr_from_mont(ex[i]));
    cp.push_back(a);
  }
  std::vector<G1a> gens;
  vl_status st = host_generators(m, gens);
  if (st != VL_OK) return st;
  const G1z lhs = msm_host(wc, gens);
  const G1z rhs = msm_host(cs, cp);
  if (!g1_same(lhs, rhs)) return fail(VL_ERR_REJECT, "hyrax verify: the opening does not match the commitments");
  const std::vector<Fr> ey = eq_host(ym);
  Fr acc = fr_zero();
  for (uint32_t j = 0; j < m; ++j) acc = fr_add(acc, fr_mul(fr_to_mont(wc[j]), ey[j]));
  if (value) {
    const Fr c = fr_from_mont(acc);
    memcpy(value->w, c.w, 32);
  }
  return VL_OK;
}

}  // extern "C"
