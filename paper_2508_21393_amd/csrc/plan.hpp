// Host-side planning: turns groups into device job descriptors and a
// workspace layout.
#pragma once
#include <stdint.h>

#include <vector>

#include "internal.hpp"
#include "sha256.hpp"

namespace vl {

inline uint64_t align_up(uint64_t x, uint64_t a) { return (x + a - 1) / a * a; }

vl_status fail(vl_status s, const char* fmt, ...);
uint32_t nvars_of(uint64_t d);
uint64_t esize(int dt);
int digits_for(int dtype);
vl_status check_group(const vl_group& g, bool need_ptrs);
uint64_t proof_elems(const vl_group& g);
void group_challenges(const vl_group& g, uint64_t seed, Transcript& tr, std::vector<Fr>& u,
                      std::vector<Fr>& v);

// a group's transcript after squeezing u (n0 values) and v (n2 values)
struct Challenges {
  Transcript tr;
  std::vector<Fr> u, v;
  std::vector<uint32_t> um, vm;   // u and v in Montgomery form, 8 words each (empty: not computed)
};

constexpr uint32_t kMaxSegments = 8;
// persistent mode: the resident rounds workgroups (each fills a CU's register
// file) may hold at most half of the 256 CUs, the contractions they wait for
// run on the rest
constexpr uint64_t kMaxPersistentGroups = 128;
constexpr uint32_t kDefaultSegments = 1;
constexpr uint32_t kBlockingSegments = 2;   // blocking calls: latency over throughput
constexpr uint32_t kPersistentSegments = 4;

struct Tuning {
  bool per_instance = false;
  uint32_t lane_macs = 8192;      // multiply-adds per lane and contraction task
  uint32_t segments = 1;          // pipeline segments (batched mode)
  uint32_t min_tasks = 1;         // split a contraction until it has this many tasks
  uint32_t cols_rows = 1;         // rows per lane, vector cols kernels (1 or 2)
  uint32_t claim_order = 0;       // claim contraction: 0 auto, 1 by columns, 2 by rows
  bool persistent = false;        // rounds launched first, waiting on readiness counters
  uint32_t spin_limit = 1u << 24; // persistent mode: polls before VL_ERR_TIMEOUT
  uint32_t contract_streams = 1;  // 2: large contraction kinds split over two streams
  uint32_t rows16_scale = 1;      // chunk length factor of the int16 vector rows kernels
};

// Jobs of one pipeline segment: its groups' contractions, finish jobs and
// rounds.  Segments run their contractions in order on the caller's stream;
// a segment's rounds start on a second stream as soon as its contractions
// are done, overlapping the later segments' contractions.
struct Segment {
  std::vector<ContractJob> cj[CK_COUNT];
  uint32_t cj_tasks[CK_COUNT] = {};
  uint64_t cj_bytes[CK_COUNT] = {};   // matrix bytes each kind streams
  std::vector<FinishJob> fin;
  uint32_t fin_blocks = 0;
  std::vector<Pass1Job> pass1;
  uint32_t pass1_blocks = 0;
  std::vector<RoundsJob> rounds;
  // wide rounds, per round rd: the groups (indices into rounds) and, for
  // rd >= 1, the sweep blocks of the launch
  std::vector<std::vector<MatSweep>> wide;
  std::vector<uint32_t> wide_blocks;
};

struct Plan {
  std::vector<uint8_t> blob;      // host image of [err flags][eq jobs][points][segments]
  bool persistent = false;        // rounds launched before the contractions
  bool fork = false;              // contraction kinds may use a side stream
  bool eq_fork = false;           // eq tables on a side stream beside the lookups' table kernels
  uint64_t data_end = 0;          // workspace bytes used
  std::vector<EqJob> eq;
  uint32_t eq_threads = 0;
  std::vector<Segment> seg;
  std::vector<std::vector<uint32_t>> points;  // per eq job: (x_j, 1 - x_j) Montgomery
  std::vector<const uint32_t*> point_dev;     // per eq job: a point already in device memory, or null
  uint32_t n_err = 0;
  uint32_t n_wide = 0;            // groups with wide rounds (one io slot each in the blob)
  uint64_t out_proof_bytes = 0;
  // launched after every segment, in this order, on the caller's stream
  std::vector<EvalJob> evals;
  std::vector<ReduceJob> reduces;
  // per-head batched products: start, wide rounds (per round, the jobs and
  // their first blocks), the one-workgroup rounds
  std::vector<BmmJob> bmms;
  std::vector<std::vector<BmmSweep>> bmm_wide;
  std::vector<uint32_t> bmm_wide_blocks;
  // lookup arguments: count buffers to zero, the entry-wise and table
  // launches, wide rounds, the one-workgroup rounds
  std::vector<LookupJob> lookups;
  std::vector<std::pair<uint32_t*, uint64_t>> lookup_zero;
  uint32_t lk_hist_blocks = 0, lk_prep_blocks = 0, lk_tab_blocks = 0, lk_mult_blocks = 0;
  std::vector<std::vector<LookupSweep>> lk_wide[2];   // per round: jobs binding a high [0] / low [1] bit
  std::vector<uint32_t> lk_wide_blocks[2];
};

struct SegLayout {
  uint64_t cj[CK_COUNT], fin, pass1, rounds;
  std::vector<uint64_t> wide;
};

struct BlobLayout {
  uint64_t err, eq, points, mat_io, evals, reduces, bmms, lookups, total;
  std::vector<SegLayout> seg;
  std::vector<uint64_t> bmm_wide, lk_wide[2];
};

// Builds jobs; device addresses are base + workspace offset (base 0 = sizing).
struct Builder {
  Plan& P;
  const Tuning& T;
  uint64_t base;
  uint64_t off;
  size_t cur = 0;                 // segment receiving new jobs
  Builder(Plan& p, const Tuning& t, uint64_t b, uint64_t start) : P(p), T(t), base(b), off(start) {
    if (P.seg.empty()) P.seg.resize(1);
  }
  Segment& S() { return P.seg[cur]; }
  uint64_t take(uint64_t bytes) {
    off = align_up(off, 256);
    const uint64_t r = off;
    off += bytes < 4 ? 4 : bytes;
    return r;
  }
  template <typename X>
  X* dev(uint64_t o) const { return reinterpret_cast<X*>(base + o); }
  void contract(const void* M, int dtype, int nd, uint64_t ld, bool rows, uint32_t n_out, uint32_t len,
                const uint32_t* pack, uint32_t* dst, uint64_t dst_ld, uint64_t n_total, int32_t* err);
  void eq_job(const std::vector<Fr>& x, uint32_t* eq, uint32_t* pack, uint32_t pack_len, bool pack_r2,
              bool eq_canon, const Fr* scale = nullptr,
              const std::vector<uint32_t>* mont = nullptr);
  // eq job of a point that a kernel earlier on the stream writes to device
  // memory (nvars Montgomery elements at point_dev)
  void eq_job_dev(uint32_t nvars, const uint32_t* point_dev, uint32_t* eq, uint32_t* pack, uint32_t pack_len,
                  bool pack_r2, bool eq_canon);
  // pass-1 job over a, b; returns the partials buffer, sets its block count
  const uint32_t* pass1(const uint32_t* a, uint64_t a_ld, const uint32_t* b, uint64_t b_ld, uint32_t h,
                        bool dot, uint32_t& nparts, uint32_t* ready);
  void group(const vl_group& g, const Challenges& ch, uint8_t* proof_dev, int32_t* status_dev,
             uint8_t* digest_dev, int32_t* err, uint32_t* ready);
  // n zero elements of an SoL vector (plane stride ld), written by the
  // finish launch
  void zero_fill(uint32_t* dst, uint64_t ld, uint32_t n);
};

BlobLayout blob_layout(const Plan& P);
uint64_t blob_bound(const vl_group* groups, uint64_t n);
void fill_blob(Plan& P, const BlobLayout& L, uint8_t* dblob);
// HIP events around every launch (blocking mode timing); one pair per
// launch, summed per stage after the call's streams are synchronised.
struct StageEvents {
  std::vector<hipEvent_t> pool;
  std::vector<int> stage;     // stage of pair i (events 2i, 2i+1)
  hipError_t begin(int st, hipStream_t s);
  hipError_t end(int st, hipStream_t s);
  void accumulate(float* ms);
  void destroy();
};

// Enqueue a filled plan on stream s; rounds of segment k run on stream s2
// after segment k's contractions (s2 may equal s: then everything is serial).
// blob_src_dev: device-side address of a pinned host buffer the blob is
// copied from (graph capture), else the blob goes through the staging ring.
// s3: a side stream for the contraction kinds of a segment (forked after the
// eq tables, joined before the finish pass; see fork_contractions) and, with
// P.eq_fork, for the eq tables of a lookup plan (joined before the first
// kernel that reads them), or null; unused when ev is given, so that stage
// times are each kernel's own.
hipError_t enqueue_plan(const Plan& P, const BlobLayout& L, uint8_t* dblob, hipStream_t s,
                        hipStream_t s2, StageEvents* ev = nullptr, const void* blob_src_dev = nullptr,
                        hipStream_t s3 = nullptr);
// the calling stream's internal rounds and side streams (one each per
// device and caller stream, kept for the process)
hipError_t rounds_stream_for(hipStream_t s, hipStream_t* out);
hipError_t side_stream_for(hipStream_t s, hipStream_t* out);
// whether a segment's contraction kinds are split over two streams
bool fork_contractions(const Segment& G);
bool plan_forks(const Plan& P);
Tuning tuning_for(const vl_prove_opts* o);
// partial evaluation (vl_mle_partial_eval): argument checks, and the launch
// with the caller's (or the fixed) scratch
vl_status partial_eval_check(const void* M, int32_t dtype, uint32_t rows, uint32_t cols, uint64_t ld,
                             int32_t contract, vl_fr_vec eq, vl_fr_vec out, const vl_tuning* tuning);
vl_status partial_eval_launch(const void* M, int32_t dtype, uint32_t rows, uint32_t cols, uint64_t ld,
                              int32_t contract, vl_fr_vec eq, vl_fr_vec out, void* workspace,
                              uint64_t workspace_bytes, const vl_tuning* tuning, void* stream);
// given: optional per-group challenges (transcript state after u and v, and
// u, v themselves) for groups whose point comes from an earlier step of a
// chained proof; null squeezes them from (seed, group id, shapes)
void plan_groups(Plan& P, const Tuning& T, const vl_group* groups, uint64_t g0, uint64_t g1,
                 uint64_t seed, uint8_t* ws, bool async, uint8_t* proofs_dev, const uint64_t* offsets,
                 int32_t* status_dev, uint8_t* digests_dev, uint8_t* out, const Challenges* given = nullptr);
// host verifier helpers (verify.cpp): 2^-1 and lifted integers in Montgomery
// form, an integer entry of a matrix of dtype dt, the eq table of a
// Montgomery point (index bits most significant first)
Fr fr_inv2_mont();
Fr lift_int(int64_t x);
int64_t get_int(const void* base, int dt, uint64_t idx);
std::vector<Fr> eq_host(const std::vector<Fr>& x);
// x^-1 (Montgomery in and out; Fermat), the polynomial through (k, g[k]),
// k < m, at r (Montgomery), and eq(x, y) of two Montgomery points
Fr fr_inv_host(const Fr& x);
Fr lagrange_host(const Fr* g, int m, const Fr& r);
Fr eq_point(const std::vector<Fr>& x, const std::vector<Fr>& y);

// M~(x, y) for an integer matrix given by an accessor over rows x cols
template <typename F>
Fr mle2(F get, uint32_t rows, uint32_t cols, const std::vector<Fr>& x, const std::vector<Fr>& y) {
  const std::vector<Fr> ex = eq_host(x), ey = eq_host(y);
  Fr total = fr_zero();
  for (uint32_t i = 0; i < rows; ++i) {
    Fr row = fr_zero();
    for (uint32_t k = 0; k < cols; ++k) {
      const int64_t v = get(i, k);
      if (v) row = fr_add(row, fr_mul(lift_int(v), ey[k]));
    }
    total = fr_add(total, fr_mul(ex[i], row));
  }
  return total;
}

// pinned host memory of this host thread and device that kernels write
// outputs into (grown on demand, kept for the process)
struct PinnedOut {
  void* host = nullptr;
  void* dev = nullptr;
  uint64_t cap = 0;
};
hipError_t pinned_out(uint64_t bytes, PinnedOut** out);

}  // namespace vl
