// Device kernels of the Hyrax commitments (vl_hyrax_setup, vl_hyrax_commit).
//
// A Hyrax commitment to the multilinear extension of an R x m matrix M (rows
// indexed by the first variables) is one Pedersen vector commitment per row,
// C_i = sum_j M[i][j] G_j, over generators G_j of G1 that nobody knows a
// relation between (Sec. II-A's polynomial commitments; the paper's
// implementation uses Hyrax, whose commitment time dominates its wall clock,
// Table t2).  The entries of the committed tensors are small signed integers,
// so each entry is recoded into signed base-256 digits d_w in [-128, 128],
// M[i][j] = sum_w d_w 256^w, and the commitment becomes a sum of table points:
//     C_i = sum_j sum_w sign(d_w) T_j,w[|d_w|],  T_j,w[k] = k 256^w G_j,
// one mixed addition per nonzero digit (fixed-base precomputation; the
// tables are public parameters computed once per generator count).
//
//   hyrax_gen_kernel     G_j by try-and-increment hashing to the curve and
//                        cofactor clearing (one thread per generator)
//   hyrax_table_kernel   T_j,w[k] for k = 1..128 (one thread per point)
//   hyrax_commit_kernel  one wave per (row, column slice): each lane sums the
//                        table points of its entries, the wave adds its lanes
//   hyrax_final_kernel   one thread per row: the slices' sum, in affine
//                        coordinates, encoded as 96 canonical bytes
#include "device.hpp"
#include "fq.hpp"

namespace vl {

namespace {

constexpr uint32_t kHyraxDigits = 128;       // table points per (generator, window)
constexpr uint32_t kPointWords = 24;         // affine point: x, y of 12 limbs
constexpr uint32_t kZWords = 48;             // XYZZ point

__device__ __forceinline__ void store_point(uint32_t* dst, const G1a& a) {
  u32x4* d = reinterpret_cast<u32x4*>(dst);
#pragma unroll
  for (int v = 0; v < 3; ++v) d[v] = u32x4{a.x.w[4 * v], a.x.w[4 * v + 1], a.x.w[4 * v + 2], a.x.w[4 * v + 3]};
#pragma unroll
  for (int v = 0; v < 3; ++v) d[3 + v] = u32x4{a.y.w[4 * v], a.y.w[4 * v + 1], a.y.w[4 * v + 2], a.y.w[4 * v + 3]};
}

__device__ __forceinline__ G1a load_point(const uint32_t* src) {
  const u32x4* s = reinterpret_cast<const u32x4*>(src);
  G1a a;
#pragma unroll
  for (int v = 0; v < 3; ++v) {
    const u32x4 t = s[v];
    a.x.w[4 * v] = t.x; a.x.w[4 * v + 1] = t.y; a.x.w[4 * v + 2] = t.z; a.x.w[4 * v + 3] = t.w;
  }
#pragma unroll
  for (int v = 0; v < 3; ++v) {
    const u32x4 t = s[3 + v];
    a.y.w[4 * v] = t.x; a.y.w[4 * v + 1] = t.y; a.y.w[4 * v + 2] = t.z; a.y.w[4 * v + 3] = t.w;
  }
  return a;
}

__device__ __forceinline__ uint64_t table_index(uint32_t j, uint32_t W, uint32_t w, uint32_t k) {
  return (((uint64_t)j * W + w) * kHyraxDigits + (k - 1)) * kPointWords;
}

// G_j (one thread per generator); a generator no counter below 256 yields
// (probability 2^-256) is left as zero words, which the table kernel and
// every later check treat as invalid
__global__ void __launch_bounds__(64) hyrax_gen_kernel(uint32_t m, uint32_t W, uint32_t* table) {
  const uint32_t j = blockIdx.x * 64 + threadIdx.x;
  if (j >= m) return;
  G1a G;
  if (!hyrax_generator(j, G)) {
    G.x = fq_zero();
    G.y = fq_zero();
  }
  store_point(table + table_index(j, W, 0, 1), G);
}

// T_j,w[k] = (k 256^w) G_j for k = 1..128; block (j, w), thread k - 1.  The
// entry (w = 0, k = 1) is G_j itself, written by the generator kernel.
__global__ void __launch_bounds__(128) hyrax_table_kernel(uint32_t m, uint32_t W, uint32_t* table) {
  const uint32_t jw = blockIdx.x;
  const uint32_t j = jw / W, w = jw % W, k = threadIdx.x + 1;
  if (j >= m || (w == 0 && k == 1)) return;
  const G1a G = load_point(table + table_index(j, W, 0, 1));
  const uint64_t s = (uint64_t)k << (8 * w);
  store_point(table + table_index(j, W, w, k), g1_to_affine(g1_mul_u64(G, s)));
}

__device__ __forceinline__ G1z shfl_xor_z(const G1z& p, int mask) {
  G1z r;
#pragma unroll
  for (int i = 0; i < 12; ++i) {
    r.X.w[i] = __shfl_xor(p.X.w[i], mask);
    r.Y.w[i] = __shfl_xor(p.Y.w[i], mask);
    r.ZZ.w[i] = __shfl_xor(p.ZZ.w[i], mask);
    r.ZZZ.w[i] = __shfl_xor(p.ZZZ.w[i], mask);
  }
  return r;
}

__device__ __forceinline__ void store_z(uint32_t* dst, const G1z& p) {
#pragma unroll
  for (int i = 0; i < 12; ++i) {
    dst[i] = p.X.w[i];
    dst[12 + i] = p.Y.w[i];
    dst[24 + i] = p.ZZ.w[i];
    dst[36 + i] = p.ZZZ.w[i];
  }
}
__device__ __forceinline__ G1z load_z(const uint32_t* src) {
  G1z p;
#pragma unroll
  for (int i = 0; i < 12; ++i) {
    p.X.w[i] = src[i];
    p.Y.w[i] = src[12 + i];
    p.ZZ.w[i] = src[24 + i];
    p.ZZZ.w[i] = src[36 + i];
  }
  return p;
}

// The group operations of the commitment loop and its wave reduction with
// their products inlined: the same formulas as g1_dbl_affine (mdbl-2008-s-1),
// g1_add_affine (madd-2008-s) and g1_add (add-2008-s), written out again
// because a call inside the loop would keep the accumulator in memory.
#if defined(__HIP_DEVICE_COMPILE__)
__device__ __forceinline__ G1z g1_dbl_affine_inl(const G1a& a) {
  const Fq U = fq_dbl(a.y);
  const Fq V = fq_mul_dev(U, U);
  const Fq W = fq_mul_dev(U, V);
  const Fq S = fq_mul_dev(a.x, V);
  const Fq x2 = fq_mul_dev(a.x, a.x);
  const Fq Mv = fq_add(fq_dbl(x2), x2);
  G1z r;
  r.X = fq_sub(fq_sub(fq_mul_dev(Mv, Mv), S), S);
  r.Y = fq_sub(fq_mul_dev(Mv, fq_sub(S, r.X)), fq_mul_dev(W, a.y));
  r.ZZ = V;
  r.ZZZ = W;
  return r;
}

__device__ __forceinline__ G1z g1_add_affine_inl(const G1z& p, const G1a& a) {
  if (g1_is_inf(p)) return g1_from_affine(a);
  // the ten products in four rounds of independent ones, each round's
  // products interleaved (fq_mul_dev_n)
  Fq t2[2];
  fq_mul_dev_n<2>({a.x, a.y}, {p.ZZ, p.ZZZ}, t2);                 // U2, S2
  const Fq P = fq_sub(t2[0], p.X);
  const Fq R = fq_sub(t2[1], p.Y);
  if (fq_is_zero(P)) {
    if (fq_is_zero(R)) return g1_dbl_affine_inl(a);
    return g1_infinity();
  }
  Fq sq[2];
  fq_mul_dev_n<2>({P, R}, {P, R}, sq);                              // PP, R^2
  Fq t3[3];
  fq_mul_dev_n<3>({P, p.X, p.ZZ}, {sq[0], sq[0], sq[0]}, t3);      // PPP, Q, ZZ PP
  const Fq& PPP = t3[0];
  const Fq& Qv = t3[1];
  G1z r;
  r.X = fq_sub(fq_sub(fq_sub(sq[1], PPP), Qv), Qv);
  Fq t4[3];
  fq_mul_dev_n<3>({R, p.Y, p.ZZZ}, {fq_sub(Qv, r.X), PPP, PPP}, t4);  // R (Q - X3), Y PPP, ZZZ PPP
  r.Y = fq_sub(t4[0], t4[1]);
  r.ZZ = t3[2];
  r.ZZZ = t4[2];
  return r;
}

__device__ __forceinline__ G1z g1_dbl_inl(const G1z& p) {
  const Fq U = fq_dbl(p.Y);
  const Fq V = fq_mul_dev(U, U);
  const Fq W = fq_mul_dev(U, V);
  const Fq S = fq_mul_dev(p.X, V);
  const Fq x2 = fq_mul_dev(p.X, p.X);
  const Fq Mv = fq_add(fq_dbl(x2), x2);
  G1z r;
  r.X = fq_sub(fq_sub(fq_mul_dev(Mv, Mv), S), S);
  r.Y = fq_sub(fq_mul_dev(Mv, fq_sub(S, r.X)), fq_mul_dev(W, p.Y));
  r.ZZ = fq_mul_dev(V, p.ZZ);
  r.ZZZ = fq_mul_dev(W, p.ZZZ);
  return r;
}

__device__ __forceinline__ G1z g1_add_inl(const G1z& p, const G1z& q2) {
  if (g1_is_inf(p)) return q2;
  if (g1_is_inf(q2)) return p;
  const Fq U1 = fq_mul_dev(p.X, q2.ZZ);
  const Fq U2 = fq_mul_dev(q2.X, p.ZZ);
  const Fq S1 = fq_mul_dev(p.Y, q2.ZZZ);
  const Fq S2 = fq_mul_dev(q2.Y, p.ZZZ);
  const Fq P = fq_sub(U2, U1);
  const Fq R = fq_sub(S2, S1);
  if (fq_is_zero(P)) {
    if (fq_is_zero(R)) return g1_dbl_inl(p);
    return g1_infinity();
  }
  const Fq PP = fq_mul_dev(P, P);
  const Fq PPP = fq_mul_dev(P, PP);
  const Fq Qv = fq_mul_dev(U1, PP);
  G1z r;
  r.X = fq_sub(fq_sub(fq_sub(fq_mul_dev(R, R), PPP), Qv), Qv);
  r.Y = fq_sub(fq_mul_dev(R, fq_sub(Qv, r.X)), fq_mul_dev(S1, PPP));
  r.ZZ = fq_mul_dev(fq_mul_dev(p.ZZ, q2.ZZ), PP);
  r.ZZZ = fq_mul_dev(fq_mul_dev(p.ZZZ, q2.ZZZ), PPP);
  return r;
}
#else
__device__ G1z g1_add_affine_inl(const G1z& p, const G1a& a);
__device__ G1z g1_add_inl(const G1z& p, const G1z& q2);
#endif

// digit w of v's signed base-256 recoding given the carry into window w:
// d in [-128, 127] below the top window (carry out when the byte plus carry
// is >= 128), the top digit in [-128, 128]; sum_w d_w 256^w = v
template <int WD>
__device__ __forceinline__ int digit_of(int64_t v, uint32_t w, int carry, int& cout) {
  if (w + 1 < (uint32_t)WD) {
    const int x = (int)(((uint64_t)v >> (8 * w)) & 0xffu) + carry;
    cout = x >= 128 ? 1 : 0;
    return x - (cout << 8);
  }
  cout = 0;
  return (int)(v >> (8 * (WD - 1))) + carry;
}

// A lane's nonzero terms (entry t, window w, digit d) in order.  Every
// madd of the commitment loop is executed by the whole wave, so a lane must
// not spend an iteration on a zero digit while the others add: each lane
// walks its own entries to its next nonzero digit (quantised weights mostly
// have a zero top digit), and the loop runs as many iterations as the lane
// with the most nonzero terms.  Entry t + 1 is loaded while entry t is in
// use.
template <typename T>
struct NonzeroTerms {
  static constexpr int WD = (int)sizeof(T);
  const T* row;
  uint32_t j0, je, cnt;   // the lane's entries j0 + 64 t, t < cnt, of a slice ending at je
  uint32_t t, w;          // the next term to examine
  int c;                  // carry into window w
  int64_t v;              // entry t
  T vn;                   // entry t + 1

  __device__ __forceinline__ T load(uint32_t k) const {
    return __builtin_nontemporal_load(row + min(j0 + 64 * k, je - 1));   // clamped: always in the slice
  }
  __device__ __forceinline__ void init(const T* r, uint32_t j0_, uint32_t je_, uint32_t cnt_) {
    row = r; j0 = j0_; je = je_; cnt = cnt_; t = 0; w = 0; c = 0;
    v = (int64_t)load(0);
    vn = load(1);
  }
  __device__ __forceinline__ bool next(int& d, uint32_t& j, uint32_t& win) {
    while (t < cnt) {
      int co;
      const int x = digit_of<WD>(v, w, c, co);
      const uint32_t jj = j0 + 64 * t, ww = w;
      if (w + 1 < (uint32_t)WD) {
        c = co;
        ++w;
      } else {
        w = 0;
        c = 0;
        ++t;
        v = (int64_t)vn;
        vn = load(t + 1);
      }
      if (x != 0) {
        d = x;
        j = jj;
        win = ww;
        return true;
      }
    }
    return false;
  }
};

// Task t = s R + i (slice-major, so the waves running together read the same
// generators' tables) sums M[i][j] G_j over the slice j in [s chunk, (s + 1)
// chunk) of columns; lane l takes j = s chunk + l + 64 t.  Each iteration
// finds every lane's next nonzero term and loads its table point (a lane
// without one loads the slice's first point and adds nothing), then adds the
// current points.
template <typename T>
__global__ void __launch_bounds__(256) hyrax_commit_kernel(const T* __restrict__ M, uint64_t ld, uint32_t R,
                                                           uint32_t m, uint32_t W, const uint32_t* __restrict__ table,
                                                           uint32_t n_split, uint32_t chunk, uint32_t* partials) {
  const uint32_t lane = threadIdx.x & 63;
  const uint64_t task = (uint64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (task >= (uint64_t)R * n_split) return;
  const uint32_t sl = (uint32_t)(task / R), i = (uint32_t)(task % R);
  const uint32_t jb = sl * chunk;
  const uint32_t je = min(m, jb + chunk);
  const uint32_t j0 = jb + lane;
  const uint32_t cnt = j0 < je ? (je - j0 + 63) / 64 : 0;
  const uint32_t* safe = table + table_index(jb, W, 0, 1);

  NonzeroTerms<T> ts;
  ts.init(M + (uint64_t)i * ld, j0, je, cnt);
  int dn = 0;
  uint32_t jn = 0, wn = 0;
  bool have = ts.next(dn, jn, wn);
  G1a nxt = load_point(have ? table + table_index(jn, W, wn, (uint32_t)abs(dn)) : safe);
  G1z acc = g1_infinity();
  while (__ballot(have) != 0) {
    const G1a cur = nxt;
    const int d = have ? dn : 0;
    have = ts.next(dn, jn, wn);
    nxt = load_point(have ? table + table_index(jn, W, wn, (uint32_t)abs(dn)) : safe);
    if (d != 0) {
      G1a p = cur;
      if (d < 0) p.y = fq_neg(p.y);
      acc = g1_add_affine_inl(acc, p);
    }
  }
#pragma unroll 1
  for (int mask = 32; mask >= 1; mask >>= 1) acc = g1_add_inl(acc, shfl_xor_z(acc, mask));
  if (lane == 0) store_z(partials + task * kZWords, acc);
}

__device__ __forceinline__ Fq fq_shfl_up(const Fq& a, int d) {
  Fq r;
#pragma unroll
  for (int k = 0; k < 12; ++k) r.w[k] = __shfl_up(a.w[k], d);
  return r;
}
__device__ __forceinline__ Fq fq_shfl_down(const Fq& a, int d) {
  Fq r;
#pragma unroll
  for (int k = 0; k < 12; ++k) r.w[k] = __shfl_down(a.w[k], d);
  return r;
}
__device__ __forceinline__ Fq fq_shfl(const Fq& a, int src) {
  Fq r;
#pragma unroll
  for (int k = 0; k < 12; ++k) r.w[k] = __shfl(a.w[k], src);
  return r;
}

// C_i = the sum of row i's slices, as 96 canonical bytes (24 words).  One
// wave per 64 rows: the affine conversions need 1 / (ZZ ZZZ) per row, which
// Montgomery's simultaneous inversion gets from one inversion per wave (the
// product of all 64 values, by prefix and suffix products across the lanes;
// every lane inverts the same value, so the inversion's branches do not
// diverge).
__global__ void __launch_bounds__(64) hyrax_final_kernel(uint32_t R, uint32_t n_split, const uint32_t* partials,
                                                         uint32_t* commits) {
  const int lane = (int)threadIdx.x;
  const uint32_t i = blockIdx.x * 64 + lane;
  const bool valid = i < R;
  G1z acc = g1_infinity();
  if (valid) {
    acc = load_z(partials + (uint64_t)i * kZWords);
    for (uint32_t s = 1; s < n_split; ++s) acc = g1_add(acc, load_z(partials + ((uint64_t)s * R + i) * kZWords));
  }
  const bool fin = valid && !g1_is_inf(acc);
  const Fq a = fin ? fq_mul(acc.ZZ, acc.ZZZ) : fq_one();
  Fq P = a, S = a;                       // inclusive prefix and suffix products
  for (int off = 1; off < 64; off <<= 1) {
    const Fq tp = fq_shfl_up(P, off);
    const Fq ts = fq_shfl_down(S, off);
    if (lane >= off) P = fq_mul(P, tp);
    if (lane + off < 64) S = fq_mul(S, ts);
  }
  const Fq inv = fq_inv(fq_shfl(P, 63));
  Fq pre = fq_shfl_up(P, 1), suf = fq_shfl_down(S, 1);
  if (lane == 0) pre = fq_one();
  if (lane == 63) suf = fq_one();
  const Fq ainv = fq_mul(fq_mul(pre, suf), inv);   // 1 / (ZZ ZZZ) of this row
  if (!valid) return;
  uint32_t* out = commits + (uint64_t)i * 24;
  if (!fin) {
#pragma unroll
    for (int k = 0; k < 24; ++k) out[k] = 0;
    return;
  }
  const Fq x = fq_from_mont(fq_mul(acc.X, fq_mul(ainv, acc.ZZZ)));
  const Fq y = fq_from_mont(fq_mul(acc.Y, fq_mul(ainv, acc.ZZ)));
#pragma unroll
  for (int k = 0; k < 12; ++k) {
    out[k] = x.w[k];
    out[12 + k] = y.w[k];
  }
}

}  // namespace

hipError_t launch_hyrax_setup(uint32_t m, uint32_t W, uint32_t* table, hipStream_t s) {
  hipLaunchKernelGGL(hyrax_gen_kernel, dim3(blocks_for(m, 64)), dim3(64), 0, s, m, W, table);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(hyrax_table_kernel, dim3((uint32_t)((uint64_t)m * W)), dim3(kHyraxDigits), 0, s, m, W, table);
  return hipGetLastError();
}

hipError_t launch_hyrax_commit(const void* M, int dtype, uint64_t ld, uint32_t R, uint32_t m, uint32_t W,
                               const uint32_t* table, uint32_t n_split, uint32_t chunk, uint32_t* partials,
                               uint32_t* commits, hipStream_t s) {
  const uint64_t tasks = (uint64_t)R * n_split;
  const uint32_t blocks = (uint32_t)((tasks + 3) / 4);
  switch (dtype) {
    case VL_I16:
      hipLaunchKernelGGL(hyrax_commit_kernel<int16_t>, dim3(blocks), dim3(256), 0, s,
                         reinterpret_cast<const int16_t*>(M), ld, R, m, W, table, n_split, chunk, partials);
      break;
    case VL_I32:
      hipLaunchKernelGGL(hyrax_commit_kernel<int32_t>, dim3(blocks), dim3(256), 0, s,
                         reinterpret_cast<const int32_t*>(M), ld, R, m, W, table, n_split, chunk, partials);
      break;
    default:
      hipLaunchKernelGGL(hyrax_commit_kernel<int64_t>, dim3(blocks), dim3(256), 0, s,
                         reinterpret_cast<const int64_t*>(M), ld, R, m, W, table, n_split, chunk, partials);
      break;
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(hyrax_final_kernel, dim3(blocks_for(R, 64)), dim3(64), 0, s, R, n_split, partials, commits);
  return hipGetLastError();
}

}  // namespace vl
