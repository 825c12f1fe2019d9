// Internal job descriptors shared by the kernels and the host orchestration.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/verilora.h"
#include "contract_job.hpp"
#include "fr.hpp"

namespace vl {


// An eq table to build: out[i] = prod_j (x_j or 1 - x_j), i < 2^nvars, plus
// its "pack" form used by the integer contractions (see contract kernel).
struct EqJob {
  uint32_t nvars;
  uint32_t pack_len;          // entries to emit into pack (8 signed digits each)
  uint32_t thread_begin;      // prefix sum of threads over jobs in a launch
  uint32_t pack_r2;           // 1: pack holds e * R^2 (contractions land in Montgomery
                              // form); 0: e * R (they land in canonical form)
  uint32_t eq_canon;          // 1: eq holds canonical values, 0: Montgomery form
  uint32_t scaled;            // 1: every entry multiplied by scale
  const uint32_t* point;      // device: nvars Montgomery elements x_j (8 words each)
  uint32_t* eq;               // SoL output, may be null
  uint64_t eq_ld;
  uint32_t* pack;             // pack_len * 8 words, may be null
  uint32_t scale[8];          // Montgomery
};

// eq table of a point passed by value (at most 20 variables)
struct EqPointArgs {
  uint32_t nvars;
  uint32_t pad_;
  uint32_t* out;
  uint64_t ld;
  uint32_t pt[20][2][8];      // Montgomery (x_j, 1 - x_j)
};

// A slice of a host image copied to device memory by a kernel launch.
constexpr uint32_t kUploadBytes = 3072;   // multiple of 4 (blob sizes are multiples of 256)
struct UploadArgs {
  void* dst;
  uint32_t bytes;
  uint32_t pad_;
  uint32_t words[kUploadBytes / 4];
};

// Round 1 of one product (or the claim's dot product: c = sum_i eqU[i] t[i]
// after a contraction of C by columns, c = sum_j eqV[j] s[j] after one by rows)
// as per-block partial sums, computed across the GPU before the rounds.
constexpr uint32_t kPass1Pairs = 512;   // pairs (entries for the dot) per 256-thread block
struct Pass1Job {
  const uint32_t* a;          // SoL table (eqU or eqV for the claim)
  const uint32_t* b;          // SoL table (t or s for the claim)
  uint64_t a_ld, b_ld;
  uint32_t h;                 // pairs (t, t + h), or entries of the dot product
  uint32_t dot;               // 1: sum_i a[i] b[i]; 0: the round-1 values g(0), g(1), g(2)
  uint32_t block_begin;       // prefix sum of blocks within a launch
  uint32_t pad_;
  uint32_t* out;              // 3 elements (24 words) per block
  uint32_t* ready;            // persistent mode: the group's readiness counter, else null
};

struct RoundsProd {
  uint32_t* a;
  uint32_t* b;
  uint64_t ld;
  uint32_t n1;
  uint32_t g_nparts;          // pass-1 partials of round 1 (3 elements each)
  const uint32_t* g_part;
};

// Wide rounds: a group whose first product's half-table has at least
// kMatWidePairs pairs in round 2 sums that product's first `wide` rounds
// across the GPU before its rounds workgroup starts: round 1 in pass 1 as
// always, each later one in a launch of mat_sweep_kernel (fold by the previous
// challenge, the round's partial sums, kMatSweepPairs pairs per block) whose
// every block first takes the previous round's transcript step from the
// previous launch's partials; the rounds workgroup takes the last wide
// round's step.  io (in the descriptor blob, so every call starts from
// zeros): [0] status, [8..23] transcript state after round k in slot k & 1,
// [24..39] r_k in slot k & 1 (Montgomery).  Sweep partials: two buffers of
// wpart_stride words, round k's in buffer k & 1.
constexpr uint32_t kMatSweepPairs = 256;
// a product goes wide when its round 2 has kMatWideStart pairs or more (at
// 1024 a sweep launch costs more than the round on one workgroup), and stays
// wide while a round has kMatWidePairs or more
constexpr uint32_t kMatWideStart = 2048;
constexpr uint32_t kMatWidePairs = 1024;
constexpr uint32_t kMatMaxWide = 16;          // n1 <= 20 needs at most 10
constexpr uint32_t kMatIoState = 8, kMatIoR = 24, kMatIoWords = 48;
struct MatSweep {
  uint32_t job;               // index in the launch's RoundsJob array
  uint32_t block_begin;       // prefix sum of sweep blocks within the launch
};
// int16 row contractions of large asynchronous calls: chunk factor, and the
// matrix bytes a call must stream to use it
constexpr uint32_t kRows16LongChunks = 16;
constexpr double kRows16LongMinBytes = 1e9;

// The sumcheck rounds of one group, run by one workgroup.
struct RoundsJob {
  uint32_t st[8];             // transcript state (digest words) after squeezing u and v
  uint32_t n_prods;
  uint32_t n0;
  uint8_t* proof;             // device proof bytes of this group
  int32_t* status;            // device status word of this group
  uint8_t* digest;            // device 32 bytes or null
  const int32_t* err;         // range flag of this group's contractions
  const uint32_t* c_part;     // pass-1 partials of c (element 0 of each)
  uint32_t c_nparts;
  uint32_t ready_target;      // persistent mode: pass-1 blocks of this group
  const uint32_t* ready;      // persistent mode: readiness counter, else null
  uint32_t spin_limit;        // polls of `ready` before giving up (VL_ERR_TIMEOUT)
  uint32_t wide;              // product 0's rounds summed by wide launches (0: none, else >= 2)
  uint32_t* io;               // wide rounds: status, transcript states, challenges
  uint32_t* wpart;            // wide rounds: sweep partials, 3 elements per block, two buffers
  uint64_t wpart_stride;      // words per partials buffer
  RoundsProd prods[VL_MAX_PRODS];
};

// A matrix MLE value M~(x, y) from the pass-1 partial sums of its dot
// product (a chained proof's evaluation at a random point): the partials are
// added and the canonical value written as 32 proof bytes.
struct EvalJob {
  const uint32_t* part;       // pass-1 partials (element 0 of each is used)
  uint32_t nparts;
  uint32_t pad_;
  uint8_t* out;               // 32 bytes, canonical little-endian
  const int32_t* err;         // range flag of the contraction
  int32_t* status;            // VL_OK, or VL_ERR_RANGE
};

// One phase of a claim reduction (several claims M~(x_k, y_k) = v_k on one
// matrix turned into one), run by one workgroup:
//  phase 1: a sumcheck over the row variables of
//           sum_k rho_k sum_i eq(x_k, i) t_k(i),  t_k(i) = sum_j M[i][j] eq(y_k, j),
//           tables a[k] = eq(x_k, .) (Montgomery) and b[k] = t_k (canonical);
//           then the values t_k(r) are sent and absorbed, sigma_1..sigma_K
//           squeezed; r (Montgomery), sigma and the state go to io
//  phase 2: a sumcheck over the column variables of
//           sum_j M~(r, j) sum_k sigma_k eq(y_k, j),
//           a[0] = M~(r, .) (Montgomery), b[k] = eq(y_k, .) (canonical), their
//           sigma-combination built into bsum; then M~(r, s) is sent
constexpr int kMaxClaims = 4;
struct ReduceJob {
  uint32_t st[8];             // phase 1: transcript state after the rho squeezes
  uint32_t coef[kMaxClaims][8];   // phase 1: rho_k, Montgomery
  uint32_t phase;             // 1 or 2
  uint32_t K;                 // claims
  uint32_t n;                 // rounds (row or column variables)
  uint32_t pad_;
  uint64_t ld;                // table stride, 2^n
  uint32_t* a[kMaxClaims];
  uint32_t* b[kMaxClaims];
  uint32_t* bsum;             // phase 2: sum_k sigma_k b[k] (2^n entries)
  uint32_t* io;               // [state: 8][sigma: kMaxClaims x 8][r: n_rows x 8] words
  uint8_t* proof;             // this phase's proof bytes
  uint8_t* digest;            // phase 2: final state of the reduction's branch
  int32_t* status;            // phase 2: VL_OK when done
};
constexpr uint32_t kReduceIoSigma = 8, kReduceIoR = 8 + 8 * kMaxClaims;
constexpr uint32_t reduce_io_words(uint32_t n_rows) { return kReduceIoR + 8 * n_rows; }

// One per-head batched product (vl_bmm_prove): C_h = A_h B_h for h < H as
// one sumcheck over (head, inner) variables of
//     sum_{h, w} eq(rho, h) a[h, w] b[h, w],  a[h, w] = A~(h, u, w),
//     b[h, w] = B~(h, w, v),
// head variables first (rounds of degree 3, eq(rho, .) folded along), then
// the inner ones (degree 2, scaled by the folded eq value).  Tables: E =
// eq(rho, .) (2^nh entries, Montgomery), a (Montgomery) and b (canonical)
// over 2^(nh + n1) entries, head index most significant, so every round
// value is canonical.  The first `wide` rounds run as GPU-wide sweeps
// (bmm_sweep_kernel, one launch per round) each followed by a one-wave
// transcript step (bmm_chal_kernel); the rest run in one workgroup
// (bmm_rounds_kernel).  io holds the state handed between the launches.
constexpr uint32_t kBmmSweepPairs = 256;     // pairs per sweep block (one per thread)
constexpr uint32_t kBmmWidePairs = 1024;     // rounds with at least this many pairs run wide
constexpr uint32_t kBmmMaxWide = 24;
// io words: [0] status (VL_OK while running), [8, 16) transcript state,
// [16, 24) pending challenge r (Montgomery), [24, 32) the claim c (canonical)
constexpr uint32_t kBmmIoState = 8, kBmmIoR = 16, kBmmIoC = 24, kBmmIoWords = 32;
struct BmmJob {
  uint32_t st[8];             // transcript state after squeezing rho, u, v
  uint32_t nh, n1;            // head and inner variables
  uint32_t wide;              // rounds done by the sweep/chal launches
  uint32_t c_nparts;
  const uint32_t* c_part;     // pass-1 partials of the claim's dot product
  uint32_t* E;                // ld 2^nh
  uint32_t* a;                // ld 2^(nh + n1)
  uint32_t* b;
  uint32_t* part;             // sweep partials: 4 elements (32 words) per block
  uint32_t* io;
  uint8_t* proof;             // device-writable proof bytes
  uint8_t* digest;            // 32 bytes or null
  int32_t* status;            // device-writable status word
  const int32_t* err;         // range flag of the job's contractions
};
// a job's part in one wide round: its blocks start at block_begin
struct BmmSweep {
  uint32_t job;
  uint32_t block_begin;
};

// One lookup argument (vl_lookup_prove, Protocol 1 with the sum of
// eq. (lookup-sumcheck)): every entry (x_i[, y_i]) of a secret tensor is a
// row (t0 + j[, tb_j]) of a table of N = 2^nL rows.  S is padded to
// 2^(nH + nL) entries with the table's first row.  Tables (SoL, Montgomery):
// over the padded entries A = 1/(beta + S), Sb = S + beta, E = eq(u, .);
// over the table rows B = 1/(beta + T), Tb = T + beta, M = multiplicities,
// EL = eq(u_L, .).  Rounds bind the high index bits first (only A, Sb, E
// depend on them; the table rows' terms add a constant K per round), then
// the low bits (all seven tables).  As for batched products, the first
// `wide` rounds run as GPU-wide sweeps and a one-wave transcript step.
constexpr uint32_t kLookupInvChunk = 16;       // table rows per thread in the batch inversion
constexpr uint32_t kLookupSweepPairs = 256;    // pairs per sweep block (one per thread)
constexpr uint32_t kLookupWidePairs = 512;
constexpr uint32_t kLookupMaxWide = 32;
constexpr uint32_t kLookupParts = 14;          // sweep partial elements per block
// io words: [0] status, [8, 16) state, [16, 24) pending r, [24, 32) K
constexpr uint32_t kLkIoState = 8, kLkIoR = 16, kLkIoK = 24, kLkIoWords = 32;
struct LookupJob {
  uint32_t st[8];             // transcript state after gamma, beta, alpha, u
  uint32_t gamma[8], beta[8], alpha[8], c1[8], c2[8];   // Montgomery (c1 = alpha^2 N / D', c2 = N / D')
  uint32_t claim[8];          // alpha + alpha^2, Montgomery
  const void* x;              // D entries, dtype
  const void* y;              // second column or null
  const int32_t* tb;          // table's second column or null
  int32_t dtype, dtype_y;
  int32_t t0;
  uint32_t pad_;
  uint64_t D;
  uint32_t nH, nL;
  uint32_t wide;
  uint32_t hist_begin;        // block prefixes: histogram launch (D entries),
  uint32_t prep_begin;        // preparation launch (padded entries),
  uint32_t tab_begin;         // inversion launch (chunks of table rows)
  uint32_t mult_begin;        // multiplicity launch (one table row per thread)
  uint32_t nkparts;           // multiplicity-launch blocks (partials of sum_j B_j m_j)
  uint32_t pad2_;
  uint32_t* cnt;              // N counts, zeroed by the plan
  uint32_t* A;                // ld 2^(nH + nL)
  uint32_t* S;
  uint32_t* E;
  uint32_t* B;                // ld 2^nL
  uint32_t* T;
  uint32_t* M;
  uint32_t* EL;
  uint32_t* kpart;
  uint32_t* part;             // sweep partials, kLookupParts elements per block
  uint32_t* io;
  int32_t* flag;              // set when an entry is not in the table
  uint8_t* proof;
  uint8_t* digest;
  int32_t* status;
};
struct LookupSweep {
  uint32_t job;
  uint32_t block_begin;
};

// host launchers (kernels.hip)
hipError_t launch_eval(const EvalJob* jobs_dev, uint32_t n_jobs, hipStream_t s);
hipError_t launch_reduce(const ReduceJob* jobs_dev, uint32_t n_jobs, hipStream_t s);
hipError_t launch_eq(const EqJob* jobs_dev, uint32_t n_jobs, uint32_t n_threads, hipStream_t s);
hipError_t launch_contract(int kind, const ContractJob* jobs_dev, uint32_t n_jobs, uint32_t n_tasks,
                           hipStream_t s);
hipError_t launch_finish(const FinishJob* jobs_dev, uint32_t n_jobs, uint32_t n_blocks, hipStream_t s);
hipError_t launch_pass1(const Pass1Job* jobs_dev, uint32_t n_jobs, uint32_t n_blocks, hipStream_t s);
hipError_t launch_rounds(const RoundsJob* jobs_dev, uint32_t n_jobs, hipStream_t s);
hipError_t launch_mat_sweep(const RoundsJob* jobs_dev, const MatSweep* list_dev, uint32_t n_list, uint32_t n_blocks,
                            uint32_t round, hipStream_t s);

hipError_t launch_lift(const void* src, int dtype, uint64_t n, uint32_t* dst, uint64_t ld, hipStream_t s);
hipError_t launch_export(const uint32_t* src, uint64_t ld, uint64_t n, uint32_t* dst, hipStream_t s);
hipError_t launch_eq_point(const EqPointArgs& a, hipStream_t s);
hipError_t launch_pack(const uint32_t* eq, uint64_t ld, uint64_t len, uint32_t* pack, hipStream_t s);
hipError_t launch_upload(void* dst, const void* src, uint64_t bytes, hipStream_t s);
hipError_t launch_zero_words(uint32_t* p, uint64_t n_words, hipStream_t s);
// batched products (bmm.hip)
hipError_t launch_bmm_start(const BmmJob* jobs_dev, uint32_t n_jobs, hipStream_t s);
hipError_t launch_bmm_sweep(const BmmJob* jobs_dev, const BmmSweep* list_dev, uint32_t n_list, uint32_t n_blocks,
                            uint32_t round, hipStream_t s);
hipError_t launch_bmm_chal(const BmmJob* jobs_dev, const BmmSweep* list_dev, uint32_t n_list, uint32_t round,
                           hipStream_t s);
hipError_t launch_bmm_rounds(const BmmJob* jobs_dev, uint32_t n_jobs, hipStream_t s);
// lookup arguments (lookup.hip)
hipError_t launch_lookup_hist(const LookupJob* jobs_dev, uint32_t n_jobs, uint32_t n_blocks, hipStream_t s);
hipError_t launch_lookup_inv(const LookupJob* jobs_dev, uint32_t n_jobs, uint32_t n_blocks, hipStream_t s);
hipError_t launch_lookup_mult(const LookupJob* jobs_dev, uint32_t n_jobs, uint32_t n_blocks, hipStream_t s);
hipError_t launch_lookup_prep(const LookupJob* jobs_dev, uint32_t n_jobs, uint32_t n_blocks, hipStream_t s);
hipError_t launch_lookup_start(const LookupJob* jobs_dev, uint32_t n_jobs, hipStream_t s);
hipError_t launch_lookup_sweep(const LookupJob* jobs_dev, const LookupSweep* list_dev, uint32_t n_list,
                               uint32_t n_blocks, uint32_t round, bool low, hipStream_t s);
hipError_t launch_lookup_chal(const LookupJob* jobs_dev, const LookupSweep* list_dev, uint32_t n_list,
                              uint32_t round, hipStream_t s);
hipError_t launch_lookup_rounds(const LookupJob* jobs_dev, uint32_t n_jobs, hipStream_t s);
// Hyrax: generators and fixed-base tables of windows W for m generators;
// commitments of R rows of an int16/int32/int64 matrix in n_split column
// slices of chunk columns (partials: R n_split XYZZ points)
hipError_t launch_hyrax_setup(uint32_t m, uint32_t W, uint32_t* table, hipStream_t s);
hipError_t launch_hyrax_commit(const void* M, int dtype, uint64_t ld, uint32_t R, uint32_t m, uint32_t W,
                               const uint32_t* table, uint32_t n_split, uint32_t chunk, uint32_t* partials,
                               uint32_t* commits, hipStream_t s);
// bytes (a multiple of 16, both pointers 16-byte aligned) from pinned host
// memory, given by its device-side address
hipError_t launch_copy_in(void* dst, const void* src_dev, uint64_t bytes, hipStream_t s);


}  // namespace vl
