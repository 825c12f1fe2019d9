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
};

struct Tuning {
  bool per_instance = false;
  uint32_t lane_macs = 16384;     // multiply-adds per lane and contraction task
  uint32_t min_tasks = 1;         // split a contraction until it has this many tasks
};

struct Plan {
  std::vector<uint8_t> blob;      // host image of [err flags][jobs...][points]
  uint64_t data_end = 0;          // workspace bytes used
  std::vector<EqJob> eq;
  uint32_t eq_threads = 0;
  std::vector<ContractJob> cj[CK_COUNT];
  uint32_t cj_tasks[CK_COUNT] = {};
  std::vector<FinishJob> fin;
  uint32_t fin_threads = 0;
  std::vector<RoundsJob> rounds;
  std::vector<std::vector<uint32_t>> points;  // per eq job: (x_j, 1 - x_j) Montgomery
  uint32_t n_err = 0;
  uint64_t out_off = 0;                       // blocking mode: gathered proofs|status|digests
  uint64_t out_proof_bytes = 0;
};

struct BlobLayout {
  uint64_t err, eq, cj[CK_COUNT], fin, rounds, points, total;
};

// Builds jobs; device addresses are base + workspace offset (base 0 = sizing).
struct Builder {
  Plan& P;
  const Tuning& T;
  uint64_t base;
  uint64_t off;
  Builder(Plan& p, const Tuning& t, uint64_t b, uint64_t start) : P(p), T(t), base(b), off(start) {}
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
  void eq_job(const std::vector<Fr>& x, uint32_t* eq, uint32_t* pack, uint32_t pack_len);
  void group(const vl_group& g, const Challenges& ch, uint8_t* proof_dev, int32_t* status_dev,
             uint8_t* digest_dev, int32_t* err);
};

BlobLayout blob_layout(const Plan& P);
uint64_t blob_bound(const vl_group* groups, uint64_t n);
void fill_blob(Plan& P, const BlobLayout& L, uint8_t* dblob);
// HIP events around each stage (blocking mode timing)
struct StageEvents {
  hipEvent_t ev[2 * VL_STAGE_COUNT] = {};
  bool used[VL_STAGE_COUNT] = {};
  hipError_t create();
  void destroy();
  hipError_t begin(int stage, hipStream_t s);
  hipError_t end(int stage, hipStream_t s);
  void accumulate(float* ms);  // after the stream has been synchronised
};

hipError_t enqueue_plan(const Plan& P, const BlobLayout& L, uint8_t* dblob, hipStream_t s,
                        StageEvents* ev = nullptr);
Tuning tuning_for(const vl_prove_opts* o);
void plan_groups(Plan& P, const Tuning& T, const vl_group* groups, uint64_t g0, uint64_t g1,
                 uint64_t seed, uint8_t* ws, bool async, uint8_t* proofs_dev, const uint64_t* offsets,
                 int32_t* status_dev, uint8_t* digests_dev);

}  // namespace vl
