// Host orchestration and the C ABI of the prover (see include/verilora.h).
//
// A prove call turns each group into device jobs:
//   1. host: transcript init, squeeze u (n0 values) and v (n2 values)
//   2. eq jobs: eq(u, .) as a table and in pack form; eq(v, .) in pack form
//   3. contraction jobs: a_p = A_p~(u, .), b_p = B_p~(., v) for every product,
//      t = C eq(v, .) for the claim (eq. (zk-mle-matmul), Sec. II-C)
//   4. finish jobs: add split contractions, zero pad to powers of two
//   5. one rounds job per group: c = eq(u, .) . t, prover guard, sumcheck
// Per-instance mode runs these launches group by group with a host wait per
// group; batched mode runs each stage once for all groups (one launch per
// stage and contraction kind); both write identical bytes.
#include <hip/hip_runtime.h>
#include <pthread.h>

#include <algorithm>
#include <atomic>
#include <condition_variable>
#include <functional>
#include <cstdarg>
#include <map>
#include <mutex>
#include <cstdio>
#include <cstring>
#include <string>
#include <thread>
#include <vector>

#include "internal.hpp"
#include "plan.hpp"
#include "sha256.hpp"

namespace vl {

thread_local std::string g_err;

vl_status fail(vl_status s, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return s;
}

uint32_t nvars_of(uint64_t d) {
  uint32_t n = 0;
  while ((1ull << n) < d) ++n;
  return n;
}

uint64_t esize(int dt) {
  switch (dt) {
    case VL_I16: return 2;
    case VL_I32: return 4;
    case VL_I64: return 8;
    default: return 0;
  }
}

// ---------------------------------------------------------------- checks ----
vl_status check_group(const vl_group& g, bool need_ptrs) {
  if (!g.prods || g.n_prods == 0 || g.n_prods > VL_MAX_PRODS)
    return fail(VL_ERR_INVALID_ARG, "group %u: n_prods must be 1..%d", g.group_id, VL_MAX_PRODS);
  const vl_product& p0 = g.prods[0];
  for (uint32_t k = 0; k < g.n_prods; ++k) {
    const vl_product& p = g.prods[k];
    if (p.D0 == 0 || p.D1 == 0 || p.D2 == 0 || p.D0 > VL_MAX_DIM || p.D1 > VL_MAX_DIM ||
        p.D2 > VL_MAX_DIM)
      return fail(VL_ERR_SHAPE, "group %u product %u: dims must be 1..2^20", g.group_id, k);
    if (p.D0 != p0.D0 || p.D2 != p0.D2)
      return fail(VL_ERR_SHAPE, "group %u: products must share D0 and D2", g.group_id);
    if (!esize(p.dtype_a) || !esize(p.dtype_b))
      return fail(VL_ERR_DTYPE, "group %u product %u: dtype must be VL_I16/I32/I64", g.group_id, k);
    const uint64_t acols = p.trans_a ? p.D0 : p.D1, bcols = p.trans_b ? p.D1 : p.D2;
    if (p.lda < acols || p.ldb < bcols)
      return fail(VL_ERR_SHAPE, "group %u product %u: leading dimension too small", g.group_id, k);
    if (need_ptrs && (!p.A || !p.B))
      return fail(VL_ERR_INVALID_ARG, "group %u product %u: null matrix", g.group_id, k);
  }
  if (!esize(g.dtype_c)) return fail(VL_ERR_DTYPE, "group %u: dtype_c must be VL_I16/I32/I64", g.group_id);
  if (g.ldc < p0.D2) return fail(VL_ERR_SHAPE, "group %u: ldc < D2", g.group_id);
  if (need_ptrs && !g.C) return fail(VL_ERR_INVALID_ARG, "group %u: null C", g.group_id);
  return VL_OK;
}

// Descriptor upload.  Small images go as kernel arguments (no host buffer
// to keep alive, nothing to wait for); larger ones through a ring of pinned
// host buffers per device, which a kernel on the caller's stream copies to
// the device (no copy-engine command: those are ordered across streams, so
// one behind a busy stream would hold up the uploads of every other).  A
// slot is reused only after the copy it last issued has completed (an event
// per slot), so the host waits only if kStagingSlots uploads are in flight.
constexpr int kStagingSlots = 4;
constexpr uint64_t kArgUploadMax = 4 * kUploadBytes;

struct StagingRing {
  struct Slot {
    void* host = nullptr;
    uint64_t cap = 0;
    hipEvent_t done = nullptr;
    bool issued = false;
  };
  std::mutex mu;
  Slot slot[kStagingSlots];
  int next = 0;
};

static hipError_t upload_blob(void* dst, const void* src, uint64_t bytes, hipStream_t s) {
  if (bytes <= kArgUploadMax) return launch_upload(dst, src, bytes, s);
  static std::mutex mu;
  static std::map<int, StagingRing*> rings;   // per device, live for the process
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  StagingRing* ring;
  {
    std::lock_guard<std::mutex> lock(mu);
    StagingRing*& r = rings[dev];
    if (!r) r = new StagingRing();
    ring = r;
  }
  std::lock_guard<std::mutex> lock(ring->mu);
  StagingRing::Slot& sl = ring->slot[ring->next];
  ring->next = (ring->next + 1) % kStagingSlots;
  if (sl.issued) {
    e = hipEventSynchronize(sl.done);
    if (e != hipSuccess) return e;
    sl.issued = false;
  }
  if (!sl.done) {
    e = hipEventCreateWithFlags(&sl.done, hipEventDisableTiming);
    if (e != hipSuccess) return e;
  }
  if (sl.cap < bytes) {
    if (sl.host) (void)hipHostFree(sl.host);
    sl.host = nullptr;
    sl.cap = 0;
    const uint64_t cap = align_up(bytes + bytes / 2, 1 << 16);
    e = hipHostMalloc(&sl.host, cap, hipHostMallocDefault);
    if (e != hipSuccess) return e;
    sl.cap = cap;
  }
  memcpy(sl.host, src, bytes);
  void* src_dev = nullptr;
  e = hipHostGetDevicePointer(&src_dev, sl.host, 0);
  if (e != hipSuccess) return e;
  e = launch_copy_in(dst, src_dev, align_up(bytes, 16), s);
  if (e != hipSuccess) return e;
  e = hipEventRecord(sl.done, s);
  if (e != hipSuccess) return e;
  sl.issued = true;
  return hipSuccess;
}

// Pinned host memory that the kernels of a blocking call write the gathered
// proofs, status words and digests into (one per host thread and device,
// grown on demand): no copy back after the call's kernels.
// (kept for the life of the process, like the staging ring)
hipError_t pinned_out(uint64_t bytes, PinnedOut** out) {
  thread_local std::map<int, PinnedOut> bufs;
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  PinnedOut& b = bufs[dev];
  if (b.cap < bytes) {
    if (b.host) (void)hipHostFree(b.host);
    b.host = b.dev = nullptr;
    b.cap = 0;
    const uint64_t cap = align_up(bytes + bytes / 2, 1 << 16);
    void* h = nullptr;
    e = hipHostMalloc(&h, cap, hipHostMallocDefault);
    if (e != hipSuccess) return e;
    b.host = h;
    e = hipHostGetDevicePointer(&b.dev, h, 0);
    if (e != hipSuccess) return e;
    b.cap = cap;
  }
  *out = &b;
  return hipSuccess;
}

// An asynchronous call's output buffer: device memory as is; pinned host
// memory (identity-mapped, as hipHostMalloc memory is with unified
// addressing) at its own address.  Anything else (pageable host memory)
// could not be written by the kernels and is refused.
static vl_status device_writable(void* p, const char* what) {
  hipPointerAttribute_t a{};
  if (hipPointerGetAttributes(&a, p) != hipSuccess) {
    (void)hipGetLastError();
    return fail(VL_ERR_INVALID_ARG, "%s: neither device memory nor pinned host memory", what);
  }
  if (a.type == hipMemoryTypeDevice || a.type == hipMemoryTypeManaged) return VL_OK;
  if (a.type == hipMemoryTypeHost && a.hostPointer && a.devicePointer == a.hostPointer) return VL_OK;
  return fail(VL_ERR_INVALID_ARG, "%s: neither device memory nor identity-mapped pinned host memory", what);
}

// The rounds stream paired with a caller's stream: one of a fixed pool of
// kRoundsStreams internal streams per device (default priority), created on
// first use and kept for the life of the process.  Caller streams are given
// pool streams round-robin in the order they are first seen, so a handful of
// concurrent callers get distinct rounds streams while the number of streams
// the library holds stays bounded however many caller streams come and go.
// Two callers that share a rounds stream stay correct (every call forks and
// joins through events); their rounds stages then run one after the other.
// The side streams of the contraction fork come from a second pool of the
// same kind.
constexpr int kRoundsStreams = 8;

static hipError_t pool_stream_for(int pool, hipStream_t s, hipStream_t* out) {
  struct Pool {
    hipStream_t st[kRoundsStreams] = {};
    std::map<hipStream_t, int> of;   // caller stream -> pool index
    int next = 0;
  };
  static std::mutex mu;
  static std::map<std::pair<int, int>, Pool> pools;
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  std::lock_guard<std::mutex> lock(mu);
  Pool& P = pools[{dev, pool}];
  auto it = P.of.find(s);
  int k;
  if (it != P.of.end()) {
    k = it->second;
  } else {
    if (P.of.size() >= 256) P.of.clear();   // forget old caller streams (indices only)
    k = P.next;
    P.next = (P.next + 1) % kRoundsStreams;
    P.of[s] = k;
  }
  if (!P.st[k]) {
    e = hipStreamCreateWithFlags(&P.st[k], hipStreamNonBlocking);
    if (e != hipSuccess) {
      P.st[k] = nullptr;
      return e;
    }
  }
  *out = P.st[k];
  return hipSuccess;
}

hipError_t rounds_stream_for(hipStream_t s, hipStream_t* out) { return pool_stream_for(0, s, out); }
hipError_t side_stream_for(hipStream_t s, hipStream_t* out) { return pool_stream_for(1, s, out); }

// Persistent mode's resident rounds workgroups spin until the contractions of
// their groups have run.  That needs the contractions to be dispatched while
// the rounds workgroups wait: on a free hardware queue (the rounds stream and
// the caller's stream must not share one) and on CUs the resident workgroups
// leave free.  A second persistent call in flight on the same device would
// put up to 2 x 128 spinning workgroups on the 256 CUs, so at most one
// persistent call runs per device at a time: a call that finds another one
// still running on its device (its completion event not yet reached, or its
// host thread still enqueueing) runs in batched mode instead, which yields
// the same bytes.
struct PersistentGate {
  std::mutex mu;
  hipEvent_t done = nullptr;
  bool issued = false;
};

static PersistentGate& persistent_gate(int dev) {
  static std::mutex mu;
  static std::map<int, PersistentGate*> gates;   // per device, live for the process
  std::lock_guard<std::mutex> lock(mu);
  PersistentGate*& g = gates[dev];
  if (!g) g = new PersistentGate();
  return *g;
}

uint64_t proof_elems(const vl_group& g) {
  uint64_t n = g.n_prods;  // c and the part claims
  for (uint32_t k = 0; k < g.n_prods; ++k) n += 3ull * nvars_of(g.prods[k].D1) + 2;
  return n;
}

void group_challenges(const vl_group& g, uint64_t seed, Transcript& tr, std::vector<Fr>& u,
                      std::vector<Fr>& v) {
  std::vector<uint32_t> dims;
  for (uint32_t k = 0; k < g.n_prods; ++k) {
    dims.push_back(g.prods[k].D0);
    dims.push_back(g.prods[k].D1);
    dims.push_back(g.prods[k].D2);
  }
  tr_init(tr, seed, g.group_id, g.n_prods, dims.data());
  // the caller's commitments before the challenges (Sec. II-C after II-A)
  if (g.bind) tr_absorb32(tr, VL_LBL_BIND, g.bind);
  const uint32_t n0 = nvars_of(g.prods[0].D0), n2 = nvars_of(g.prods[0].D2);
  u.resize(n0);
  v.resize(n2);
  for (uint32_t i = 0; i < n0; ++i) u[i] = tr_squeeze_fixed(tr, VL_LBL_U);
  for (uint32_t i = 0; i < n2; ++i) v[i] = tr_squeeze_fixed(tr, VL_LBL_V);
}

// A few host threads kept for the life of the process, for the per-group
// hashing of large calls: starting threads per call costs about as much as
// the hashing it would spread (tens of microseconds).  run(n, fn) calls
// fn(i) for every i < n on the workers and the calling thread and returns
// when all are done; a call that finds the pool busy (another host thread
// planning) does its work alone.
class HostPool {
 public:
  // never destroyed: the workers stay blocked on the condition variable
  // until the process ends (destroying it under waiters would block, also in
  // a forked child, whose copy still counts the parent's workers)
  static HostPool& get() {
    static HostPool* pool = new HostPool();
    return *pool;
  }
  void run(uint64_t n, const std::function<void(uint64_t)>& fn) {
    if (forked_) {   // a child process: the workers stayed in the parent
      for (uint64_t i = 0; i < n; ++i) fn(i);
      return;
    }
    std::unique_lock<std::mutex> busy(run_mu_, std::try_to_lock);
    if (!busy.owns_lock() || th_.empty()) {
      for (uint64_t i = 0; i < n; ++i) fn(i);
      return;
    }
    Job job;
    job.fn = &fn;
    job.n = n;
    {
      std::lock_guard<std::mutex> lk(mu_);
      job_ = &job;
      ++gen_;
    }
    cv_.notify_all();
    work(job);
    // every index is taken; wait for the workers still inside this job (no
    // worker joins it once job_ is cleared)
    std::unique_lock<std::mutex> lk(mu_);
    job_ = nullptr;
    idle_cv_.wait(lk, [&] { return active_ == 0; });
  }
  // fn(i) for every i < n on the workers and the calling thread, and
  // consume(i) on the calling thread in order of i, each as soon as fn(i) is
  // done (while it waits, the calling thread takes indices itself)
  void run_ordered(uint64_t n, const std::function<void(uint64_t)>& fn,
                   const std::function<void(uint64_t)>& consume) {
    std::unique_lock<std::mutex> busy(run_mu_, std::defer_lock);
    if (forked_ || th_.empty() || !busy.try_lock()) {
      for (uint64_t i = 0; i < n; ++i) {
        fn(i);
        consume(i);
      }
      return;
    }
    std::vector<std::atomic<uint8_t>> done(n);
    for (auto& d : done) d.store(0, std::memory_order_relaxed);
    Job job;
    job.fn = &fn;
    job.n = n;
    job.done = done.data();
    {
      std::lock_guard<std::mutex> lk(mu_);
      job_ = &job;
      ++gen_;
    }
    cv_.notify_all();
    for (uint64_t i = 0; i < n; ++i) {
      while (!done[i].load(std::memory_order_acquire)) {
        const uint64_t j = job.next.fetch_add(1);
        if (j < n) {
          fn(j);
          done[j].store(1, std::memory_order_release);
        } else {
          std::this_thread::yield();   // index i is on a worker
        }
      }
      consume(i);
    }
    std::unique_lock<std::mutex> lk(mu_);
    job_ = nullptr;
    idle_cv_.wait(lk, [&] { return active_ == 0; });
  }
 private:
  struct Job {
    const std::function<void(uint64_t)>* fn = nullptr;
    uint64_t n = 0;
    std::atomic<uint64_t> next{0};
    std::atomic<uint8_t>* done = nullptr;   // run_ordered: index i finished
  };
  HostPool() {
    const unsigned hw = std::thread::hardware_concurrency();
    const unsigned nw = hw > 1 ? std::min(7u, hw - 1) : 0u;
    for (unsigned k = 0; k < nw; ++k) th_.emplace_back([this] { loop(); });
    pthread_atfork(nullptr, nullptr, [] { HostPool::get().forked_ = true; });
  }
  static void work(Job& j) {
    for (uint64_t i = j.next.fetch_add(1); i < j.n; i = j.next.fetch_add(1)) {
      (*j.fn)(i);
      if (j.done) j.done[i].store(1, std::memory_order_release);
    }
  }
  void loop() {
    uint64_t seen = 0;
    for (;;) {
      Job* j;
      {
        std::unique_lock<std::mutex> lk(mu_);
        cv_.wait(lk, [&] { return job_ && gen_ != seen; });
        seen = gen_;
        j = job_;
        ++active_;
      }
      work(*j);
      std::lock_guard<std::mutex> lk(mu_);
      if (--active_ == 0) idle_cv_.notify_all();
    }
  }
  std::mutex run_mu_, mu_;
  std::condition_variable cv_, idle_cv_;
  Job* job_ = nullptr;
  uint64_t gen_ = 0;
  uint32_t active_ = 0;
  bool forked_ = false;
  std::vector<std::thread> th_;
};

// Challenges of groups [g0, g1): transcript state after u and v.  Each group
// is independent (its own transcript); a group costs a few microseconds of
// hashing (tens of blocks), so calls of a dozen groups or more spread them
// over the host pool.
// (with u and v in Montgomery form for the eq jobs, converted with the
// challenges, on the pool, rather than by the serial job builder)
static void challenges_of(const vl_group& g, uint64_t seed, Challenges& c) {
  group_challenges(g, seed, c.tr, c.u, c.v);
  c.um.resize(8 * c.u.size());
  c.vm.resize(8 * c.v.size());
  for (size_t k = 0; k < c.u.size(); ++k) memcpy(c.um.data() + 8 * k, fr_to_mont(c.u[k]).w, 32);
  for (size_t k = 0; k < c.v.size(); ++k) memcpy(c.vm.data() + 8 * k, fr_to_mont(c.v[k]).w, 32);
}

void all_challenges(const vl_group* groups, uint64_t g0, uint64_t g1, uint64_t seed,
                    std::vector<Challenges>& out) {
  const uint64_t n = g1 - g0;
  out.assign(n, Challenges());
  const std::function<void(uint64_t)> one = [&](uint64_t i) { challenges_of(groups[g0 + i], seed, out[i]); };
  if (n < 12) {
    for (uint64_t i = 0; i < n; ++i) one(i);
    return;
  }
  HostPool::get().run(n, one);
}

// ---------------------------------------------------------------- planning --
// Digit layout of an entry type: int16 entries are one 16-bit digit; int32
// and int64 use 24-bit digits (two cover |x| < 2^47, three any int64).
int digits_for(int dtype) { return dtype == VL_I16 ? 1 : (dtype == VL_I32 ? 2 : 3); }

static int contract_kind(int dtype, int nd, bool rows, bool vec, int opl) {
  if (dtype == VL_I16) {
    if (rows) return opl == 4 ? (vec ? CK_I16_ROWS4_VEC : CK_I16_ROWS4) : CK_I16_ROWS;
    return vec ? (opl == 2 ? CK_I16_COLS2_VEC : CK_I16_COLS_VEC) : CK_I16_COLS;
  }
  if (dtype == VL_I32) {
    if (rows) return (vec && opl == 4) ? CK_I32_ROWS4_VEC : CK_I32_ROWS;
    return vec ? CK_I32_COLS_VEC : CK_I32_COLS;
  }
  if (nd == 2) {
    if (rows) return (vec && opl == 2) ? CK_I64S_ROWS2_VEC : CK_I64S_ROWS;
    return vec ? (opl == 2 ? CK_I64S_COLS2_VEC : CK_I64S_COLS_VEC) : CK_I64S_COLS;
  }
  if (rows) return (vec && opl == 2) ? CK_I64_ROWS2_VEC : CK_I64_ROWS;
  return vec ? CK_I64_COLS_VEC : CK_I64_COLS;
}

void Builder::contract(const void* M, int dtype, int nd, uint64_t ld, bool rows, uint32_t n_out,
                       uint32_t len, const uint32_t* pack, uint32_t* dst, uint64_t dst_ld,
                       uint64_t n_total, int32_t* err) {
  ContractJob j{};
  const uint64_t es = esize(dtype);
  const bool wide = dtype != VL_I16;
  // outputs per lane.  Rows kernels: adjacent columns read as one vector per
  // row (4 int16 = 8 bytes; 4 int32 or 2 int64 = 16 bytes), so that one
  // scalar load of eq digits feeds 32 or more multiply-adds.  Vector cols
  // kernels: two rows per lane on request (tuning).
  int opl = 1;
  if (rows && n_out >= 256) opl = (int)((dtype == VL_I16 ? 8 : 16) / es);
  if (rows && wide && es == 8 && n_out >= 128) opl = 2;
  // vector loads: aligned groups of opl columns (rows kernels), 16-byte
  // aligned rows (cols kernels)
  const uint64_t vb = rows ? opl * es : 16;
  const bool vec = (!rows || opl > 1) && (reinterpret_cast<uintptr_t>(M) % vb == 0) && ((ld * es) % vb == 0);
  if (rows && wide && !vec) opl = 1;   // wide rows kernels with element loads: one column per lane
  if (!rows && vec && T.cols_rows == 2 && (dtype == VL_I16 || nd == 2) && n_out >= 128) opl = 2;
  const int kind = contract_kind(dtype, nd, rows, vec, opl);
  const uint32_t out_waves = (n_out + 64 * opl - 1) / (64 * opl);
  // chunk: about T.lane_macs multiply-adds per lane and task
  uint64_t chunk = std::max<uint64_t>(64, T.lane_macs / (8ull * nd * opl));
  if (rows && !wide && opl > 1) chunk *= T.rows16_scale;
  chunk = std::min<uint64_t>(chunk, kMaxChunk);
  // the vector rows kernels of wide entries keep no high-word accumulators:
  // a chunk holds at most kWideSpill rows
  const bool no_spill = rows && wide && vec;
  if (no_spill) chunk = std::min<uint64_t>(chunk, kWideSpill);
  // narrow contractions (one output wave): split the contraction index finely
  // so that the job spreads over the GPU instead of one long chain per wave
  if (out_waves <= 2) chunk = std::min<uint64_t>(chunk, std::max<uint64_t>(64, len / 64));
  chunk = std::min<uint64_t>(chunk, align_up(len, kChunkAlign));
  chunk = align_up(chunk, kChunkAlign);
  while (T.min_tasks > 1 && chunk > 256 &&
         (uint64_t)out_waves * ((len + chunk - 1) / chunk) < T.min_tasks)
    chunk = align_up(chunk / 2, kChunkAlign);
  const uint32_t n_chunks = (uint32_t)((len + chunk - 1) / chunk);
  j.M = M;
  j.ld = ld;
  j.n_out = n_out;
  j.len = len;
  j.chunk = (uint32_t)chunk;
  j.n_chunks = n_chunks;
  j.out_waves = out_waves;
  j.task_begin = S().cj_tasks[kind];
  j.pack = pack;
  j.err = err;
  FinishJob f{};
  f.n_valid = n_out;
  f.n_total = (uint32_t)n_total;
  f.out = dst;
  f.out_ld = dst_ld;
  f.n_chunks = n_chunks;
  if (n_chunks == 1) {
    j.dst = dst;
    j.dst_ld = dst_ld;
    f.part = nullptr;
  } else {
    // 64-output tiles of n_chunks * kLimbs words per output
    uint32_t* part = dev<uint32_t>(take(partial_word(align_up(n_out, 64), 0, 0, n_chunks) * 4));
    j.dst = part;
    j.dst_ld = 0;
    f.part = part;
  }
  S().cj_tasks[kind] += out_waves * n_chunks;
  S().cj_bytes[kind] += (uint64_t)n_out * len * es;
  S().cj[kind].push_back(j);
  if (f.part || f.n_total > f.n_valid) {
    f.split = (f.part && n_chunks >= kFinishSplitChunks) ? 1u : 0u;
    f.block_begin = S().fin_blocks;
    S().fin_blocks += f.split ? (f.n_total + 63) / 64 : (f.n_total + 255) / 256;
    S().fin.push_back(f);
  }
}

void Builder::eq_job(const std::vector<Fr>& x, uint32_t* eq, uint32_t* pack, uint32_t pack_len, bool pack_r2,
                     bool eq_canon, const Fr* scale, const std::vector<uint32_t>* mont) {
  EqJob e{};
  if (scale) {
    e.scaled = 1;
    memcpy(e.scale, scale->w, 32);
  }
  e.nvars = (uint32_t)x.size();
  e.pack_r2 = pack_r2 ? 1u : 0u;
  e.eq_canon = eq_canon ? 1u : 0u;
  e.pack_len = pack_len;
  e.thread_begin = P.eq_threads;
  e.eq = eq;
  e.eq_ld = 1ull << x.size();
  e.pack = pack;
  if (mont && mont->size() == 8 * x.size()) {
    P.points.push_back(*mont);
  } else {
    std::vector<uint32_t> pts;
    pts.reserve(8 * x.size());
    for (const Fr& xi : x) {
      const Fr xm = fr_to_mont(xi);
      pts.insert(pts.end(), xm.w, xm.w + 8);
    }
    P.points.push_back(std::move(pts));
  }
  P.point_dev.push_back(nullptr);
  // one thread per 4 entries (one for the whole table below 2 variables);
  // pack_len <= 2^nvars
  const uint32_t threads = std::max<uint32_t>(1, (uint32_t)((1ull << x.size()) / 4));
  P.eq_threads += std::max(threads, (pack_len + 3) / 4);
  P.eq.push_back(e);
}

void Builder::eq_job_dev(uint32_t nvars, const uint32_t* point_dev, uint32_t* eq, uint32_t* pack,
                         uint32_t pack_len, bool pack_r2, bool eq_canon) {
  EqJob e{};
  e.nvars = nvars;
  e.pack_r2 = pack_r2 ? 1u : 0u;
  e.eq_canon = eq_canon ? 1u : 0u;
  e.pack_len = pack_len;
  e.thread_begin = P.eq_threads;
  e.eq = eq;
  e.eq_ld = 1ull << nvars;
  e.pack = pack;
  P.points.push_back({});
  P.point_dev.push_back(point_dev);
  const uint32_t threads = std::max<uint32_t>(1, (uint32_t)((1ull << nvars) / 4));
  P.eq_threads += std::max(threads, (pack_len + 3) / 4);
  P.eq.push_back(e);
}

void Builder::group(const vl_group& g, const Challenges& ch, uint8_t* proof_dev, int32_t* status_dev,
                    uint8_t* digest_dev, int32_t* err, uint32_t* ready) {
  const Transcript& tr = ch.tr;
  const std::vector<Fr>& u = ch.u;
  const std::vector<Fr>& v = ch.v;
  const vl_product& p0 = g.prods[0];
  const uint32_t D0 = p0.D0, D2 = p0.D2, n0 = (uint32_t)u.size();
  const uint64_t L0 = 1ull << n0;
  const uint32_t n2 = (uint32_t)v.size();
  const uint64_t L2 = 1ull << n2;
  uint32_t* packU = dev<uint32_t>(take((uint64_t)D0 * 32));
  uint32_t* packV = dev<uint32_t>(take((uint64_t)D2 * 32));

  // The claim c = C~(u, v) = sum_{i,j} eq(u, i) C[i][j] eq(v, j) (eq.
  // (zk-mle-matmul)), contracted in either order:
  //   by columns: t[i] = sum_j C[i][j] eq(v, j) (canonical, pack of e R), then
  //               c = sum_i eq(u, i) t[i] with eq(u, .) in Montgomery form;
  //   by rows:    s[j] = sum_i eq(u, i) C[i][j] (Montgomery, pack of e R^2),
  //               then c = sum_j eq(v, j) s[j] with eq(v, .) stored canonical.
  // Both give c in canonical form.  By rows a wave reads adjacent columns of
  // each row of C (coalesced), by columns each lane streams its own row.
  // Two 24-bit digits cover |C| < 2^47 - 2^23, enough for sums of int16
  // products with a total inner dimension <= 2^16; wider C uses three (an
  // out-of-range entry makes the prover refuse with VL_ERR_RANGE rather than
  // prove a wrong claim).
  int ndc = digits_for(g.dtype_c);
  if (g.dtype_c == VL_I64) {
    uint64_t sum_d1 = 0;
    bool small = true;
    for (uint32_t k = 0; k < g.n_prods; ++k) {
      sum_d1 += g.prods[k].D1;
      small &= g.prods[k].dtype_a == VL_I16 && g.prods[k].dtype_b == VL_I16;
    }
    if (small && sum_d1 <= (1u << 16)) ndc = 2;
  }
  const bool by_rows = T.claim_order == 2 || (T.claim_order == 0 && D2 >= 256);
  RoundsJob rj{};
  if (by_rows) {
    uint32_t* eqV = dev<uint32_t>(take(8 * L2 * 4));
    uint32_t* svec = dev<uint32_t>(take(8 * L2 * 4));
    eq_job(u, nullptr, packU, D0, true, false, nullptr, &ch.um);
    eq_job(v, eqV, packV, D2, false, true, nullptr, &ch.vm);
    contract(g.C, g.dtype_c, ndc, g.ldc, true, D2, D0, packU, svec, L2, L2, err);
    rj.c_part = pass1(eqV, L2, svec, L2, (uint32_t)L2, true, rj.c_nparts, ready);
  } else {
    uint32_t* eqU = dev<uint32_t>(take(8 * L0 * 4));
    uint32_t* tvec = dev<uint32_t>(take(8 * L0 * 4));
    eq_job(u, eqU, packU, D0, true, false, nullptr, &ch.um);
    eq_job(v, nullptr, packV, D2, false, false, nullptr, &ch.vm);
    contract(g.C, g.dtype_c, ndc, g.ldc, false, D0, D2, packV, tvec, L0, L0, err);
    rj.c_part = pass1(eqU, L0, tvec, L0, (uint32_t)L0, true, rj.c_nparts, ready);
  }
  rj.ready = ready;
  rj.ready_target = rj.c_nparts;
  rj.spin_limit = T.spin_limit;
  memcpy(rj.st, tr.h, 32);
  rj.n_prods = g.n_prods;
  rj.n0 = n0;
  rj.proof = proof_dev;
  rj.status = status_dev;
  rj.digest = digest_dev;
  rj.err = err;
  for (uint32_t k = 0; k < g.n_prods; ++k) {
    const vl_product& p = g.prods[k];
    const uint32_t n1 = nvars_of(p.D1);
    const uint64_t L1 = 1ull << n1;
    uint32_t* a = dev<uint32_t>(take(8 * L1 * 4));
    uint32_t* b = dev<uint32_t>(take(8 * L1 * 4));
    // a[w] = sum_i eq(u, i) op(A)[i][w]: rows of stored A, or columns of stored A^T
    contract(p.A, p.dtype_a, digits_for(p.dtype_a), p.lda, !p.trans_a, p.D1, D0, packU, a, L1, L1, err);
    // b[w] = sum_j op(B)[w][j] eq(v, j): columns of stored B, or rows of stored B^T
    contract(p.B, p.dtype_b, digits_for(p.dtype_b), p.ldb, p.trans_b != 0, p.D1, D2, packV, b, L1, L1, err);
    rj.prods[k].a = a;
    rj.prods[k].b = b;
    rj.prods[k].ld = L1;
    rj.prods[k].n1 = n1;
    // round 1 (for D1 = 1 the single product a[0] b[0])
    rj.prods[k].g_part = n1 ? pass1(a, L1, b, L1, (uint32_t)(L1 / 2), false, rj.prods[k].g_nparts, ready)
                            : pass1(a, L1, b, L1, 1, true, rj.prods[k].g_nparts, ready);
    rj.ready_target += rj.prods[k].g_nparts;
  }
  // wide rounds for product 0 while its half-table has >= kMatWidePairs pairs
  // (from round 2, when that has >= kMatWideStart); not in persistent mode,
  // whose rounds workgroups are resident before the contractions run
  const uint32_t n1w = rj.prods[0].n1;
  if (!T.persistent && n1w >= 2 && (1ull << (n1w - 2)) >= kMatWideStart) {
    uint32_t W = 1;
    while (W < kMatMaxWide && W + 1 < n1w && (1ull << (n1w - 1 - W)) >= kMatWidePairs) ++W;
    const uint32_t nb1 = (uint32_t)(((1ull << (n1w - 2)) + kMatSweepPairs - 1) / kMatSweepPairs);
    rj.wide = W;
    rj.io = nullptr;   // a slot of the descriptor blob, set when the blob is filled
    rj.wpart_stride = (uint64_t)nb1 * 24;
    rj.wpart = dev<uint32_t>(take((uint64_t)nb1 * 96 * 2));
    Segment& G = S();
    const uint32_t idx = (uint32_t)G.rounds.size();
    P.n_wide += 1;
    if (G.wide.size() < W) {
      G.wide.resize(W);
      G.wide_blocks.resize(W, 0);
    }
    for (uint32_t rd = 0; rd < W; ++rd) {
      MatSweep m{};
      m.job = idx;
      m.block_begin = G.wide_blocks[rd];
      G.wide[rd].push_back(m);
      if (rd > 0)
        G.wide_blocks[rd] +=
            (uint32_t)(((1ull << (n1w - 1 - rd)) + kMatSweepPairs - 1) / kMatSweepPairs);
    }
  }
  // persistent mode: one resident launch for every group (segment 0's list)
  (T.persistent ? P.seg[0] : S()).rounds.push_back(rj);
}

void Builder::zero_fill(uint32_t* dst, uint64_t ld, uint32_t n) {
  if (!n) return;
  FinishJob f{};
  f.n_valid = 0;
  f.n_total = n;
  f.out = dst;
  f.out_ld = ld;
  f.split = 0;
  f.block_begin = S().fin_blocks;
  S().fin_blocks += (n + 255) / 256;
  S().fin.push_back(f);
}

const uint32_t* Builder::pass1(const uint32_t* a, uint64_t a_ld, const uint32_t* b, uint64_t b_ld, uint32_t h,
                               bool dot, uint32_t& nparts, uint32_t* ready) {
  Pass1Job j{};
  j.ready = ready;
  j.a = a;
  j.b = b;
  j.a_ld = a_ld;
  j.b_ld = b_ld;
  j.h = h;
  j.dot = dot ? 1u : 0u;
  nparts = std::max<uint32_t>(1, (h + kPass1Pairs - 1) / kPass1Pairs);
  j.block_begin = S().pass1_blocks;
  j.out = dev<uint32_t>(take((uint64_t)nparts * 96));
  S().pass1_blocks += nparts;
  S().pass1.push_back(j);
  return j.out;
}

BlobLayout blob_layout(const Plan& P) {
  BlobLayout L{};
  uint64_t o = 0;
  L.err = o;   // per group: a range flag, then (persistent mode) a readiness counter
  o = align_up(o + 8ull * std::max<uint32_t>(P.n_err, 1), 64);
  L.eq = o;
  o = align_up(o + P.eq.size() * sizeof(EqJob), 64);
  L.points = o;
  for (const auto& pt : P.points) o = align_up(o + pt.size() * 4, 64);
  L.seg.resize(P.seg.size());
  for (size_t k = 0; k < P.seg.size(); ++k) {
    const Segment& G = P.seg[k];
    for (int c = 0; c < CK_COUNT; ++c) {
      L.seg[k].cj[c] = o;
      o = align_up(o + G.cj[c].size() * sizeof(ContractJob), 64);
    }
    L.seg[k].fin = o;
    o = align_up(o + G.fin.size() * sizeof(FinishJob), 64);
    L.seg[k].pass1 = o;
    o = align_up(o + G.pass1.size() * sizeof(Pass1Job), 64);
    L.seg[k].rounds = o;
    o = align_up(o + G.rounds.size() * sizeof(RoundsJob), 64);
    L.seg[k].wide.resize(G.wide.size());
    for (size_t rd = 0; rd < G.wide.size(); ++rd) {
      L.seg[k].wide[rd] = o;
      o = align_up(o + G.wide[rd].size() * sizeof(MatSweep), 64);
    }
  }
  L.mat_io = o;
  o = align_up(o + 4ull * kMatIoWords * P.n_wide, 64);
  L.evals = o;
  o = align_up(o + P.evals.size() * sizeof(EvalJob), 64);
  L.reduces = o;
  o = align_up(o + P.reduces.size() * sizeof(ReduceJob), 64);
  L.bmms = o;
  o = align_up(o + P.bmms.size() * sizeof(BmmJob), 64);
  L.bmm_wide.resize(P.bmm_wide.size());
  for (size_t k = 0; k < P.bmm_wide.size(); ++k) {
    L.bmm_wide[k] = o;
    o = align_up(o + P.bmm_wide[k].size() * sizeof(BmmSweep), 64);
  }
  L.lookups = o;
  o = align_up(o + P.lookups.size() * sizeof(LookupJob), 64);
  for (int lo = 0; lo < 2; ++lo) {
    L.lk_wide[lo].resize(P.lk_wide[lo].size());
    for (size_t k = 0; k < P.lk_wide[lo].size(); ++k) {
      L.lk_wide[lo][k] = o;
      o = align_up(o + P.lk_wide[lo][k].size() * sizeof(LookupSweep), 64);
    }
  }
  L.total = align_up(o, 256);
  return L;
}

uint64_t blob_bound(const vl_group* groups, uint64_t n) {
  uint64_t cj = 0, pts = 0;
  for (uint64_t i = 0; i < n; ++i) {
    cj += 1 + 2ull * groups[i].n_prods;
    pts += 2ull * (nvars_of(groups[i].prods[0].D0) + nvars_of(groups[i].prods[0].D2)) * 32 + 128;
  }
  // pass-1 jobs: the claim and one per product; every segment may pad each
  // of its CK_COUNT + 3 arrays to 64 bytes
  return align_up(8 * n + 64 + 2 * n * (sizeof(EqJob) + 64) +
                      cj * (sizeof(ContractJob) + sizeof(FinishJob) + sizeof(Pass1Job) + 128) +
                      n * (sizeof(RoundsJob) + 64) + pts + 64 * (CK_COUNT + 3) * (n + 1) + 1024 +
                      kMatMaxWide * (n * sizeof(MatSweep) + 64ull * (kMaxSegments + 1)) +
                      n * 4ull * kMatIoWords + 64,
                  256);
}

// fills the blob (descriptor pointers patched to the workspace copy)
void fill_blob(Plan& P, const BlobLayout& L, uint8_t* dblob) {
  P.blob.assign(L.total, 0);
  uint64_t po = L.points;
  for (size_t i = 0; i < P.eq.size(); ++i) {
    if (P.point_dev[i]) {   // written on the device by an earlier kernel
      P.eq[i].point = P.point_dev[i];
      continue;
    }
    P.eq[i].point = reinterpret_cast<const uint32_t*>(dblob + po);
    memcpy(P.blob.data() + po, P.points[i].data(), P.points[i].size() * 4);
    po = align_up(po + P.points[i].size() * 4, 64);
  }
  if (!P.evals.empty()) memcpy(P.blob.data() + L.evals, P.evals.data(), P.evals.size() * sizeof(EvalJob));
  if (!P.reduces.empty())
    memcpy(P.blob.data() + L.reduces, P.reduces.data(), P.reduces.size() * sizeof(ReduceJob));
  if (!P.bmms.empty()) memcpy(P.blob.data() + L.bmms, P.bmms.data(), P.bmms.size() * sizeof(BmmJob));
  for (size_t k = 0; k < P.bmm_wide.size(); ++k)
    memcpy(P.blob.data() + L.bmm_wide[k], P.bmm_wide[k].data(), P.bmm_wide[k].size() * sizeof(BmmSweep));
  if (!P.lookups.empty())
    memcpy(P.blob.data() + L.lookups, P.lookups.data(), P.lookups.size() * sizeof(LookupJob));
  for (int lo = 0; lo < 2; ++lo)
    for (size_t k = 0; k < P.lk_wide[lo].size(); ++k)
      if (!P.lk_wide[lo][k].empty())
        memcpy(P.blob.data() + L.lk_wide[lo][k], P.lk_wide[lo][k].data(),
               P.lk_wide[lo][k].size() * sizeof(LookupSweep));
  memcpy(P.blob.data() + L.eq, P.eq.data(), P.eq.size() * sizeof(EqJob));
  // wide rounds' io slots: zeros in the blob, so every call starts its counts
  // and status afresh
  uint32_t slot = 0;
  for (auto& G : P.seg)
    for (auto& rj : G.rounds)
      if (rj.wide) rj.io = reinterpret_cast<uint32_t*>(dblob + L.mat_io + 4ull * kMatIoWords * slot++);
  for (size_t k = 0; k < P.seg.size(); ++k) {
    const Segment& G = P.seg[k];
    for (int c = 0; c < CK_COUNT; ++c)
      if (!G.cj[c].empty())
        memcpy(P.blob.data() + L.seg[k].cj[c], G.cj[c].data(), G.cj[c].size() * sizeof(ContractJob));
    if (!G.fin.empty()) memcpy(P.blob.data() + L.seg[k].fin, G.fin.data(), G.fin.size() * sizeof(FinishJob));
    if (!G.pass1.empty())
      memcpy(P.blob.data() + L.seg[k].pass1, G.pass1.data(), G.pass1.size() * sizeof(Pass1Job));
    if (!G.rounds.empty())
      memcpy(P.blob.data() + L.seg[k].rounds, G.rounds.data(), G.rounds.size() * sizeof(RoundsJob));
    for (size_t rd = 0; rd < G.wide.size(); ++rd)
      if (!G.wide[rd].empty())
        memcpy(P.blob.data() + L.seg[k].wide[rd], G.wide[rd].data(), G.wide[rd].size() * sizeof(MatSweep));
  }
}

hipError_t StageEvents::begin(int st, hipStream_t s) {
  const size_t i = stage.size();
  while (pool.size() < 2 * i + 2) {
    hipEvent_t e;
    const hipError_t r = hipEventCreate(&e);
    if (r != hipSuccess) return r;
    pool.push_back(e);
  }
  stage.push_back(st);
  return hipEventRecord(pool[2 * i], s);
}

hipError_t StageEvents::end(int, hipStream_t s) { return hipEventRecord(pool[2 * (stage.size() - 1) + 1], s); }

void StageEvents::accumulate(float* ms) {
  for (size_t i = 0; i < stage.size(); ++i) {
    float t = 0.f;
    if (hipEventElapsedTime(&t, pool[2 * i], pool[2 * i + 1]) == hipSuccess) ms[stage[i]] += t;
  }
  stage.clear();
}

void StageEvents::destroy() {
  for (auto e : pool) (void)hipEventDestroy(e);
  pool.clear();
}

#define VL_STAGE(ev, st, s, launch)                   \
  do {                                                 \
    if (ev) {                                          \
      const hipError_t e0_ = (ev)->begin((st), (s));  \
      if (e0_ != hipSuccess) return e0_;               \
    }                                                  \
    const hipError_t e1_ = (launch);                   \
    if (e1_ != hipSuccess) return e1_;                 \
    if (ev) {                                          \
      const hipError_t e2_ = (ev)->end((st), (s));    \
      if (e2_ != hipSuccess) return e2_;               \
    }                                                  \
  } while (0)

// Per-call fork/join events between the caller's stream and the rounds
// stream: cached per host thread, created on first use.
struct ForkEvents {
  std::vector<hipEvent_t> ev;
  hipError_t need(size_t n) {
    while (ev.size() < n) {
      hipEvent_t e;
      const hipError_t r = hipEventCreateWithFlags(&e, hipEventDisableTiming);
      if (r != hipSuccess) return r;
      ev.push_back(e);
    }
    return hipSuccess;
  }
  ~ForkEvents() {
    for (auto e : ev) (void)hipEventDestroy(e);
  }
};

// The contraction kinds of a segment write disjoint outputs, and the int16
// kinds are held by latency rather than by HBM: split over two streams they
// overlap, and the launch gaps between them close.  Worth it when at least
// two kinds each stream 8 MB or more.
constexpr uint64_t kForkMinBytes = 8ull << 20;

bool fork_contractions(const Segment& G) {
  int big = 0;
  for (int c = 0; c < CK_COUNT; ++c) big += !G.cj[c].empty() && G.cj_bytes[c] >= kForkMinBytes;
  return big >= 2;
}

bool plan_forks(const Plan& P) {
  if (!P.fork) return false;
  for (const Segment& G : P.seg)
    if (fork_contractions(G)) return true;
  return false;
}

// whether a plan holds lookups alone (then its eq tables are first read by
// the lookup sweeps, and the table kernels may use the internal streams)
static bool lookups_only(const Plan& P) {
  if (P.lookups.empty() || !P.bmms.empty() || !P.evals.empty() || !P.reduces.empty()) return false;
  for (const Segment& G : P.seg) {
    if (!G.fin.empty() || !G.pass1.empty() || !G.rounds.empty()) return false;
    for (int c = 0; c < CK_COUNT; ++c)
      if (!G.cj[c].empty()) return false;
  }
  return true;
}

hipError_t enqueue_plan(const Plan& P, const BlobLayout& L, uint8_t* dblob, hipStream_t s,
                        hipStream_t s2, StageEvents* ev, const void* blob_src_dev, hipStream_t s3) {
  thread_local std::map<int, ForkEvents> forks;   // per host thread and device
  const size_t nseg = P.seg.size();
  const bool two = s2 != s;
  const bool side = s3 && s3 != s && !ev && P.fork;
  const bool eq_side = s3 && s3 != s && !ev && P.eq_fork && lookups_only(P);
  const bool inv_side = two && !ev && lookups_only(P);
  int dev = 0;
  if (two || side || eq_side) {
    const hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
  }
  ForkEvents& fork = forks[dev];
  if (two || side || eq_side) {
    // [0, nseg): rounds forks; nseg, nseg + 1: rounds start and join;
    // nseg + 2 + 2k, nseg + 3 + 2k: segment k's contraction fork and join;
    // 3 nseg + 2 + k: the end of segment k's wide rounds; 4 nseg + 2,
    // 4 nseg + 3: the eq fork and join; 4 nseg + 4, 4 nseg + 5: the fork and
    // join of the lookups' table inversions
    const hipError_t e = fork.need(4 * nseg + 6);
    if (e != hipSuccess) return e;
  }
  VL_STAGE(ev, VL_STAGE_UPLOAD, s,
           blob_src_dev ? launch_copy_in(dblob, blob_src_dev, L.total, s)
                        : upload_blob(dblob, P.blob.data(), L.total, s));
  if (eq_side) {
    // lookups: the eq tables are first read by the sweeps, after the
    // multiplicities, the table inverses and the entries' terms; the eq
    // kernel (bound by its field products) runs beside those (bound by
    // atomics, one inversion chain per thread, and memory)
    hipError_t e = hipEventRecord(fork.ev[4 * nseg + 2], s);
    if (e == hipSuccess) e = hipStreamWaitEvent(s3, fork.ev[4 * nseg + 2], 0);
    if (e == hipSuccess)
      e = launch_eq(reinterpret_cast<const EqJob*>(dblob + L.eq), (uint32_t)P.eq.size(), P.eq_threads, s3);
    if (e == hipSuccess) e = hipEventRecord(fork.ev[4 * nseg + 3], s3);
    if (e != hipSuccess) return e;
  } else {
    VL_STAGE(ev, VL_STAGE_EQ, s,
             launch_eq(reinterpret_cast<const EqJob*>(dblob + L.eq), (uint32_t)P.eq.size(), P.eq_threads, s));
  }
  if (two) {
    // the rounds stream starts after everything queued before this call
    hipError_t e = hipEventRecord(fork.ev[nseg], s);
    if (e == hipSuccess) e = hipStreamWaitEvent(s2, fork.ev[nseg], 0);
    if (e != hipSuccess) return e;
  }
  if (P.persistent) {
    // resident rounds first: each workgroup waits for its group's pass 1
    for (size_t k = 0; k < nseg; ++k)
      if (!P.seg[k].rounds.empty())
        VL_STAGE(ev, VL_STAGE_ROUNDS, s2,
                 launch_rounds(reinterpret_cast<const RoundsJob*>(dblob + L.seg[k].rounds),
                               (uint32_t)P.seg[k].rounds.size(), s2));
  }
  bool wide_wait = false;   // the previous segment's wide rounds run on the rounds stream
  for (size_t k = 0; k < nseg; ++k) {
    const Segment& G = P.seg[k];
    if (wide_wait) {
      // this segment's contractions start after the previous segment's wide
      // rounds: those are on the path to its rounds kernel (the chain that
      // ends the call), and beside HBM-bound contractions a sweep took up to
      // 1.7 times as long; the contractions then overlap the rounds kernel,
      // which holds one CU per group
      const hipError_t e = hipStreamWaitEvent(s, fork.ev[3 * nseg + 2 + k - 1], 0);
      if (e != hipSuccess) return e;
      wide_wait = false;
    }
    const bool fk = side && fork_contractions(G);
    if (fk) {
      hipError_t e = hipEventRecord(fork.ev[nseg + 2 + 2 * k], s);
      if (e == hipSuccess) e = hipStreamWaitEvent(s3, fork.ev[nseg + 2 + 2 * k], 0);
      if (e != hipSuccess) return e;
    }
    // streams: kinds largest first, each to the stream with fewer bytes so
    // far; then each stream runs its kinds smallest first, so that the
    // narrower kinds (the int16 ones, held by latency) run beside the
    // largest one (the claim, which saturates HBM on its own)
    int order[CK_COUNT], which[CK_COUNT] = {};
    for (int c = 0; c < CK_COUNT; ++c) order[c] = c;
    std::stable_sort(order, order + CK_COUNT, [&](int a, int b) { return G.cj_bytes[a] > G.cj_bytes[b]; });
    uint64_t load[2] = {0, 0};
    for (int i = 0; i < CK_COUNT; ++i) {
      const int c = order[i];
      if (G.cj[c].empty()) continue;
      which[c] = (fk && load[1] < load[0]) ? 1 : 0;
      load[which[c]] += G.cj_bytes[c];
    }
    // (the caller's stream first: its kinds wait on nothing)
    for (int w = 0; w < 2; ++w)
      for (int i = CK_COUNT - 1; i >= 0; --i) {
        const int c = order[i];
        if (G.cj[c].empty() || which[c] != w) continue;
        hipStream_t sc = w ? s3 : s;
        VL_STAGE(ev, VL_STAGE_CONTRACT + c, sc,
                 launch_contract(c, reinterpret_cast<const ContractJob*>(dblob + L.seg[k].cj[c]),
                                 (uint32_t)G.cj[c].size(), G.cj_tasks[c], sc));
      }
    if (fk) {
      hipError_t e = hipEventRecord(fork.ev[nseg + 3 + 2 * k], s3);
      if (e == hipSuccess) e = hipStreamWaitEvent(s, fork.ev[nseg + 3 + 2 * k], 0);
      if (e != hipSuccess) return e;
    }
    if (!G.fin.empty())
      VL_STAGE(ev, VL_STAGE_FINISH, s,
               launch_finish(reinterpret_cast<const FinishJob*>(dblob + L.seg[k].fin), (uint32_t)G.fin.size(),
                             G.fin_blocks, s));
    if (!G.pass1.empty())
      VL_STAGE(ev, VL_STAGE_PASS1, s,
               launch_pass1(reinterpret_cast<const Pass1Job*>(dblob + L.seg[k].pass1), (uint32_t)G.pass1.size(),
                            G.pass1_blocks, s));
    if (G.rounds.empty() || P.persistent) continue;
    // the last segment's rounds on the caller's stream (nothing follows its
    // contractions there), beside the earlier segments' on the rounds stream
    hipStream_t sr = (two && k + 1 < nseg) ? s2 : s;
    if (sr != s) {
      hipError_t e = hipEventRecord(fork.ev[k], s);
      if (e == hipSuccess) e = hipStreamWaitEvent(s2, fork.ev[k], 0);
      if (e != hipSuccess) return e;
    }
    const RoundsJob* rjobs = reinterpret_cast<const RoundsJob*>(dblob + L.seg[k].rounds);
    // wide rounds 2, 3, ..: one sweep launch each (round 1 is in pass 1)
    for (size_t rd = 1; rd < G.wide.size(); ++rd) {
      if (G.wide[rd].empty()) continue;
      const MatSweep* lst = reinterpret_cast<const MatSweep*>(dblob + L.seg[k].wide[rd]);
      VL_STAGE(ev, VL_STAGE_ROUNDS, sr,
               launch_mat_sweep(rjobs, lst, (uint32_t)G.wide[rd].size(), G.wide_blocks[rd], (uint32_t)rd, sr));
    }
    if (sr != s && G.wide.size() > 1 && k + 1 < nseg) {
      const hipError_t e = hipEventRecord(fork.ev[3 * nseg + 2 + k], sr);
      if (e != hipSuccess) return e;
      wide_wait = true;
    }
    VL_STAGE(ev, VL_STAGE_ROUNDS, sr, launch_rounds(rjobs, (uint32_t)G.rounds.size(), sr));
  }
  if (two) {
    // join: the caller's stream sees every rounds launch
    hipError_t e = hipEventRecord(fork.ev[nseg + 1], s2);
    if (e == hipSuccess) e = hipStreamWaitEvent(s, fork.ev[nseg + 1], 0);
    if (e != hipSuccess) return e;
  }
  if (!P.evals.empty())
    VL_STAGE(ev, VL_STAGE_ROUNDS, s,
             launch_eval(reinterpret_cast<const EvalJob*>(dblob + L.evals), (uint32_t)P.evals.size(), s));
  if (!P.reduces.empty())
    VL_STAGE(ev, VL_STAGE_ROUNDS, s,
             launch_reduce(reinterpret_cast<const ReduceJob*>(dblob + L.reduces), (uint32_t)P.reduces.size(), s));
  if (!P.bmms.empty()) {
    const BmmJob* bj = reinterpret_cast<const BmmJob*>(dblob + L.bmms);
    const uint32_t nb = (uint32_t)P.bmms.size();
    VL_STAGE(ev, VL_STAGE_PASS1, s, launch_bmm_start(bj, nb, s));
    for (size_t k = 0; k < P.bmm_wide.size(); ++k) {
      const BmmSweep* lst = reinterpret_cast<const BmmSweep*>(dblob + L.bmm_wide[k]);
      const uint32_t nl = (uint32_t)P.bmm_wide[k].size();
      VL_STAGE(ev, VL_STAGE_PASS1, s, launch_bmm_sweep(bj, lst, nl, P.bmm_wide_blocks[k], (uint32_t)k, s));
      VL_STAGE(ev, VL_STAGE_ROUNDS, s, launch_bmm_chal(bj, lst, nl, (uint32_t)k, s));
    }
    VL_STAGE(ev, VL_STAGE_ROUNDS, s, launch_bmm_rounds(bj, nb, s));
  }
  if (!P.lookups.empty()) {
    const LookupJob* lj = reinterpret_cast<const LookupJob*>(dblob + L.lookups);
    const uint32_t nl = (uint32_t)P.lookups.size();
    for (const auto& z : P.lookup_zero) VL_STAGE(ev, VL_STAGE_FINISH, s, launch_zero_words(z.first, z.second, s));
    if (inv_side) {
      // the table inversions (one chain of field products per thread, a few
      // dozen blocks) read no count: they run on the rounds stream beside
      // the count kernel, joined before the multiplicities
      hipError_t e = hipEventRecord(fork.ev[4 * nseg + 4], s);
      if (e == hipSuccess) e = hipStreamWaitEvent(s2, fork.ev[4 * nseg + 4], 0);
      if (e == hipSuccess) e = launch_lookup_inv(lj, nl, P.lk_tab_blocks, s2);
      if (e == hipSuccess) e = hipEventRecord(fork.ev[4 * nseg + 5], s2);
      if (e == hipSuccess) e = launch_lookup_hist(lj, nl, P.lk_hist_blocks, s);
      if (e == hipSuccess) e = hipStreamWaitEvent(s, fork.ev[4 * nseg + 5], 0);
      if (e != hipSuccess) return e;
    } else {
      VL_STAGE(ev, VL_STAGE_FINISH, s, launch_lookup_hist(lj, nl, P.lk_hist_blocks, s));
      VL_STAGE(ev, VL_STAGE_FINISH, s, launch_lookup_inv(lj, nl, P.lk_tab_blocks, s));
    }
    VL_STAGE(ev, VL_STAGE_FINISH, s, launch_lookup_mult(lj, nl, P.lk_mult_blocks, s));
    VL_STAGE(ev, VL_STAGE_FINISH, s, launch_lookup_prep(lj, nl, P.lk_prep_blocks, s));
    if (eq_side) {
      const hipError_t e = hipStreamWaitEvent(s, fork.ev[4 * nseg + 3], 0);
      if (e != hipSuccess) return e;
    }
    VL_STAGE(ev, VL_STAGE_PASS1, s, launch_lookup_start(lj, nl, s));
    const size_t nk = std::max(P.lk_wide[0].size(), P.lk_wide[1].size());
    for (size_t k = 0; k < nk; ++k) {
      for (int lo = 0; lo < 2; ++lo) {
        if (k >= P.lk_wide[lo].size() || P.lk_wide[lo][k].empty()) continue;
        const LookupSweep* lst = reinterpret_cast<const LookupSweep*>(dblob + L.lk_wide[lo][k]);
        const uint32_t nw = (uint32_t)P.lk_wide[lo][k].size();
        VL_STAGE(ev, VL_STAGE_PASS1, s,
                 launch_lookup_sweep(lj, lst, nw, P.lk_wide_blocks[lo][k], (uint32_t)k, lo == 1, s));
        VL_STAGE(ev, VL_STAGE_ROUNDS, s, launch_lookup_chal(lj, lst, nw, (uint32_t)k, s));
      }
    }
    VL_STAGE(ev, VL_STAGE_ROUNDS, s, launch_lookup_rounds(lj, nl, s));
  }
  return hipSuccess;
}

// defaults, then the caller's non-zero knobs
static void apply_tuning(Tuning& t, const vl_tuning* k) {
  if (!k) return;
  if (k->lane_macs) t.lane_macs = k->lane_macs;
  if (k->min_tasks) t.min_tasks = k->min_tasks;
  if (k->segments && !t.per_instance) t.segments = k->segments;
  if (k->cols_rows) t.cols_rows = k->cols_rows;
  if (k->spin_limit) t.spin_limit = k->spin_limit;
  if (k->claim_order) t.claim_order = k->claim_order;
  if (k->contract_streams) t.contract_streams = k->contract_streams;
}

static vl_status check_tuning(const vl_tuning* k) {
  if (!k) return VL_OK;
  if (k->claim_order > 2) return fail(VL_ERR_INVALID_ARG, "vl_tuning.claim_order must be 0, 1 or 2");
  if (k->segments > kMaxSegments)
    return fail(VL_ERR_INVALID_ARG, "vl_tuning.segments must be <= %u", kMaxSegments);
  if (k->lane_macs && k->lane_macs < 64) return fail(VL_ERR_INVALID_ARG, "vl_tuning.lane_macs must be >= 64");
  if (k->cols_rows > 2) return fail(VL_ERR_INVALID_ARG, "vl_tuning.cols_rows must be 0, 1 or 2");
  if (k->contract_streams > 2)
    return fail(VL_ERR_INVALID_ARG, "vl_tuning.contract_streams must be 0, 1 or 2");
  return VL_OK;
}

Tuning tuning_for(const vl_prove_opts* o) {
  Tuning t;
  t.per_instance = !o || o->mode == VL_MODE_PER_INSTANCE;
  t.persistent = o && o->mode == VL_MODE_PERSISTENT;
  t.min_tasks = t.per_instance ? 1024 : 1;
  t.segments = t.per_instance ? 1 : (t.persistent ? kPersistentSegments : kDefaultSegments);
  // a blocking call proves one batch at a time: two segments let the longest
  // sumchecks start while the last groups' contractions run (1.55 -> 1.50 ms
  // on the 7B block); with several proofs in flight the other proofs fill the
  // GPU instead, and one segment gave 2-3% more throughput
  if (!t.per_instance && !t.persistent && o && !o->async) t.segments = kBlockingSegments;
  // the contraction fork by default only in blocking calls: asynchronous
  // calls and prove graphs are made to have several proofs in flight, which
  // then share the GPU's few hardware queues, and a second stream per proof
  // made their throughput depend on how the runtime happened to map streams
  // to queues (one proof's rounds kernel holding up another's contractions)
  t.contract_streams = (o && !o->async) ? 2 : 1;
  // the int16 contractions over rows write 48 bytes of chunk sums per output
  // and chunk (about a tenth of their matrix bytes at 256-row chunks), which
  // the finish pass reads back: with several proofs of a large batch in
  // flight the GPU is bound by HBM, and chunks kRows16LongChunks times longer
  // gave more throughput (plan_groups keeps short chunks for small calls); a
  // lone blocking call needs the tasks of short chunks more than the bytes
  if (!t.per_instance && o && o->async && !(o->tuning && o->tuning->lane_macs)) t.rows16_scale = kRows16LongChunks;
  if (o) apply_tuning(t, o->tuning);
  return t;
}

static Tuning pe_tuning(const vl_tuning* k) {
  Tuning t;
  t.min_tasks = 1024;
  apply_tuning(t, k);
  return t;
}

// Time model of a group for pipeline segments (µs, measured on MI355X): its
// rounds chain, a base of about 50 µs plus 13 µs per round held in
// registers (half-table of 64 pairs or fewer) and 24 µs per round swept in
// memory, per product in order; and its contraction bytes at about 4.5 TB/s.
static double rounds_us(const vl_group& g) {
  double t = 50.0;
  for (uint32_t k = 0; k < g.n_prods; ++k) {
    const double n1 = nvars_of(g.prods[k].D1);
    t += 13.0 * std::min(n1, 7.0) + 24.0 * std::max(0.0, n1 - 7.0) + (k ? 15.0 : 0.0);
  }
  return t;
}

// Segment boundaries over the groups in order (longest chains first):
// segment k holds positions [cut[k], cut[k + 1]).  Segment k's rounds start
// once its contractions (all earlier segments' too, on the caller's stream)
// and its finish pass are done; the rounds of segments 0 .. nseg - 2 run one
// after another on the rounds stream, the last segment's on the caller's
// stream beside them.  Two or three segments: the cuts that minimise the
// modelled end of the call (over all cuts; few groups per call); otherwise,
// and in persistent mode, equal numbers of groups.
static std::vector<uint64_t> segment_cuts(const std::vector<uint64_t>& order, const std::vector<double>& chain,
                                          const std::vector<double>& bytes, uint32_t nseg, bool persistent) {
  const uint64_t n = order.size();
  std::vector<uint64_t> cut(nseg + 1);
  for (uint32_t k = 0; k <= nseg; ++k) cut[k] = (uint64_t)k * n / nseg;
  if (persistent || nseg < 2 || nseg > 3 || n > 512) return cut;
  constexpr double kBytesPerUs = 4.5e6, kFinishUs = 60.0;
  std::vector<double> pre(n + 1, 0.0);   // contraction time of positions [0, i)
  for (uint64_t i = 0; i < n; ++i) pre[i + 1] = pre[i] + bytes[order[i]] / kBytesPerUs;
  auto end_of = [&](const std::vector<uint64_t>& c) {
    double rs = 0.0, end = 0.0;   // the rounds stream's free time; the call's end
    for (uint32_t k = 0; k < nseg; ++k) {
      const double ready = pre[c[k + 1]] + kFinishUs * (k + 1);
      const double r = chain[order[c[k]]];   // the segment's longest chain
      if (k + 1 < nseg) {
        rs = std::max(rs, ready) + r;
        end = std::max(end, rs);
      } else {
        end = std::max(end, ready + r);
      }
    }
    return end;
  };
  double best = end_of(cut);
  std::vector<uint64_t> c(nseg + 1);
  c[0] = 0;
  c[nseg] = n;
  if (nseg == 2) {
    for (uint64_t a = 1; a < n; ++a) {
      c[1] = a;
      const double e = end_of(c);
      if (e < best) best = e, cut = c;
    }
  } else {
    for (uint64_t a = 1; a + 1 < n; ++a)
      for (uint64_t b = a + 1; b < n; ++b) {
        c[1] = a;
        c[2] = b;
        const double e = end_of(c);
        if (e < best) best = e, cut = c;
      }
  }
  return cut;
}

// Plans groups [g0, g1) with the blob at workspace offset 0 and data after it.
// Blocking mode gathers every proof, status word and digest of the call in
// one region of pinned host memory (out: its device-side address; proofs at
// their final offsets, then statuses, then digests) that the kernels write
// directly.  ws == nullptr plans for sizing only.
// matrix bytes a group's contractions stream (C once, every A and B once)
static double group_bytes(const vl_group& g) {
  double b = (double)g.prods[0].D0 * g.prods[0].D2 * (double)esize(g.dtype_c);
  for (uint32_t k = 0; k < g.n_prods; ++k) {
    const vl_product& p = g.prods[k];
    b += (double)p.D1 * ((double)p.D0 * esize(p.dtype_a) + (double)p.D2 * esize(p.dtype_b));
  }
  return b;
}

void plan_groups(Plan& P, const Tuning& T, const vl_group* groups, uint64_t g0, uint64_t g1,
                 uint64_t seed, uint8_t* ws, bool async, uint8_t* proofs_dev, const uint64_t* offsets,
                 int32_t* status_dev, uint8_t* digests_dev, uint8_t* out, const Challenges* given) {
  P = Plan();
  P.persistent = T.persistent;
  P.fork = !T.persistent && T.contract_streams == 2;
  const uint64_t blob = blob_bound(groups + g0, g1 - g0);
  // long int16 row chunks only for calls that stream enough matrix bytes to
  // keep the GPU's tasks plentiful at that length (a 7B-class block streams
  // 3.8 GB; the per-layer requests of a proof server, well under 1 GB, lost
  // 12% of their throughput with them)
  Tuning TT = T;
  if (TT.rows16_scale > 1) {
    double call_bytes = 0;
    for (uint64_t i = g0; i < g1; ++i) call_bytes += group_bytes(groups[i]);
    if (call_bytes < kRows16LongMinBytes) TT.rows16_scale = 1;
  }
  Builder B(P, TT, reinterpret_cast<uint64_t>(ws), blob);
  P.n_err = (uint32_t)(g1 - g0);
  const uint64_t n = g1 - g0;
  // challenges: given, computed with the groups' jobs below (ws), or for
  // sizing zeros (they change no size, only their count matters)
  std::vector<Challenges> ch;
  const bool stream_ch = !given && ws;
  if (given) {
    ch.assign(given, given + n);
  } else if (ws) {
    ch.assign(n, Challenges());
  } else {
    ch.assign(n, Challenges());
    for (uint64_t i = 0; i < n; ++i) {
      ch[i].u.assign(nvars_of(groups[g0 + i].prods[0].D0), fr_zero());
      ch[i].v.assign(nvars_of(groups[g0 + i].prods[0].D2), fr_zero());
    }
  }
  uint64_t proof_total = 0;
  for (uint64_t i = g0; i < g1; ++i) proof_total += 32 * proof_elems(groups[i]);
  if (!async) P.out_proof_bytes = proof_total;
  // pipeline segments: groups with the longest sumchecks first, so that their
  // rounds overlap the contractions of the groups after them
  std::vector<uint64_t> order(n);
  for (uint64_t i = 0; i < n; ++i) order[i] = i;
  std::vector<double> chain(n), bytes(n);
  for (uint64_t i = 0; i < n; ++i) {
    chain[i] = rounds_us(groups[g0 + i]);
    bytes[i] = group_bytes(groups[g0 + i]);
  }
  std::stable_sort(order.begin(), order.end(), [&](uint64_t a, uint64_t b) { return chain[a] > chain[b]; });
  const uint32_t nseg = (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>(T.segments, n));
  P.seg.assign(nseg, Segment());
  std::vector<uint32_t> seg_of(n);
  const std::vector<uint64_t> cut = segment_cuts(order, chain, bytes, nseg, T.persistent);
  for (uint64_t r = 0, k = 0; r < n; ++r) {
    while (k + 1 < nseg && r >= cut[k + 1]) ++k;
    seg_of[order[r]] = (uint32_t)k;
  }
  uint64_t rel = 0;
  // group jobs in group order, each as soon as its challenges are known:
  // the host pool hashes the groups' transcripts while this thread builds
  const std::function<void(uint64_t)> build = [&](uint64_t li) {
    const uint64_t i = g0 + li;
    uint8_t* pd;
    int32_t* sd;
    uint8_t* dd;
    if (async) {
      pd = proofs_dev ? proofs_dev + offsets[i] : nullptr;
      sd = status_dev ? status_dev + i : nullptr;
      dd = digests_dev ? digests_dev + 32 * i : nullptr;
    } else {
      uint8_t* base = out;
      pd = base + rel;
      sd = reinterpret_cast<int32_t*>(base + align_up(proof_total, 256)) + li;
      dd = base + align_up(proof_total, 256) + align_up(4 * n, 256) + 32 * li;
    }
    rel += 32 * proof_elems(groups[i]);
    int32_t* err = reinterpret_cast<int32_t*>(ws + 4 * li);  // blob starts with the flags
    uint32_t* ready = T.persistent ? reinterpret_cast<uint32_t*>(ws + 4 * (n + li)) : nullptr;
    B.cur = seg_of[li];
    B.group(groups[i], ch[li], pd, sd, dd, err, ready);
  };
  if (stream_ch && n >= 12) {
    const std::function<void(uint64_t)> hash = [&](uint64_t li) { challenges_of(groups[g0 + li], seed, ch[li]); };
    HostPool::get().run_ordered(n, hash, build);
  } else {
    for (uint64_t li = 0; li < n; ++li) {
      if (stream_ch) challenges_of(groups[g0 + li], seed, ch[li]);
      build(li);
    }
  }
  P.data_end = B.off;
}

}  // namespace vl

using namespace vl;

extern "C" {

const char* vl_last_error(void) { return g_err.c_str(); }

uint64_t vl_proof_size(const vl_group* g) {
  if (!g || check_group(*g, false) != VL_OK) return 0;
  return 32 * proof_elems(*g);
}

uint64_t vl_workspace_size(const vl_group* groups, uint64_t n, const vl_prove_opts* o) {
  if (!groups || n == 0) return 0;
  for (uint64_t i = 0; i < n; ++i)
    if (check_group(groups[i], false) != VL_OK) return 0;
  const Tuning T = tuning_for(o);
  const bool async = o && o->async;
  std::vector<uint64_t> offs(n + 1, 0);
  Plan P;
  if (T.per_instance) {
    uint64_t mx = 0;
    for (uint64_t i = 0; i < n; ++i) {
      plan_groups(P, T, groups, i, i + 1, 0, nullptr, async, nullptr, offs.data(), nullptr, nullptr, nullptr);
      mx = std::max(mx, P.data_end);
    }
    return align_up(mx, 256);
  }
  plan_groups(P, T, groups, 0, n, 0, nullptr, async, nullptr, offs.data(), nullptr, nullptr, nullptr);
  return align_up(P.data_end, 256);
}

// Checks shared by the prove entry points; fills offsets.
static vl_status validate_prove(const vl_group* groups, uint64_t n, const vl_prove_opts* o, uint8_t* proofs,
                                uint64_t proofs_len, uint64_t* offsets, uint8_t* digests) {
  if (!groups || n == 0 || !o || !proofs || !offsets)
    return fail(VL_ERR_INVALID_ARG, "null argument");
  if (check_tuning(o->tuning) != VL_OK) return VL_ERR_INVALID_ARG;
  if (o->mode < VL_MODE_PER_INSTANCE || o->mode > VL_MODE_PERSISTENT)
    return fail(VL_ERR_INVALID_ARG, "unknown mode %d", o->mode);
  if (o->async && !o->status) return fail(VL_ERR_INVALID_ARG, "async mode needs a status array");
  if (o->async) {
    vl_status st = device_writable(proofs, "proofs");
    if (st == VL_OK) st = device_writable(o->status, "status");
    if (st == VL_OK && digests) st = device_writable(digests, "digests");
    if (st != VL_OK) return st;
  }
  if (o->mode == VL_MODE_PERSISTENT && n > kMaxPersistentGroups)
    return fail(VL_ERR_INVALID_ARG, "persistent mode takes at most %llu groups per call",
                (unsigned long long)kMaxPersistentGroups);
  for (uint64_t i = 0; i < n; ++i) {
    const vl_status st = check_group(groups[i], true);
    if (st != VL_OK) return st;
  }
  uint64_t tot = 0;
  for (uint64_t i = 0; i < n; ++i) {
    offsets[i] = tot;
    tot += 32 * proof_elems(groups[i]);
  }
  offsets[n] = tot;
  if (proofs_len < tot)
    return fail(VL_ERR_BUFFER_TOO_SMALL, "proof buffer holds %llu bytes, %llu needed",
                (unsigned long long)proofs_len, (unsigned long long)tot);
  if (!o->workspace) return fail(VL_ERR_WORKSPACE, "no workspace");
  if (reinterpret_cast<uintptr_t>(o->workspace) % 256)
    return fail(VL_ERR_WORKSPACE, "workspace must be 256-byte aligned");
  return VL_OK;
}

vl_status vl_sumcheck_matmul_prove(const vl_group* groups, uint64_t n, uint64_t seed,
                                   const vl_prove_opts* o, uint8_t* proofs, uint64_t proofs_len,
                                   uint64_t* offsets, uint8_t* digests, void* stream) {
  {
    const vl_status st = validate_prove(groups, n, o, proofs, proofs_len, offsets, digests);
    if (st != VL_OK) return st;
  }
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  uint8_t* ws = reinterpret_cast<uint8_t*>(o->workspace);
  Tuning T = tuning_for(o);
  const bool async = o->async != 0;
  // persistent mode: one call per device at a time (see PersistentGate); the
  // gate's lock is held until this call's work is enqueued and its
  // completion event recorded
  std::unique_lock<std::mutex> gate_lock;
  PersistentGate* gate = nullptr;
  if (T.persistent) {
    int dev = 0;
    const hipError_t de = hipGetDevice(&dev);
    if (de != hipSuccess) return fail(VL_ERR_HIP, "device: %s", hipGetErrorString(de));
    PersistentGate& pg = persistent_gate(dev);
    gate_lock = std::unique_lock<std::mutex>(pg.mu, std::try_to_lock);
    bool free = gate_lock.owns_lock();
    if (free && pg.issued) {
      const hipError_t q = hipEventQuery(pg.done);
      if (q == hipErrorNotReady) {
        free = false;
      } else if (q != hipSuccess) {
        return fail(VL_ERR_HIP, "persistent gate: %s", hipGetErrorString(q));
      }
    }
    if (free) {
      gate = &pg;
      if (!pg.done) {
        const hipError_t ce = hipEventCreateWithFlags(&pg.done, hipEventDisableTiming);
        if (ce != hipSuccess) return fail(VL_ERR_HIP, "persistent gate: %s", hipGetErrorString(ce));
      }
    } else {
      if (gate_lock.owns_lock()) gate_lock.unlock();
      T.persistent = false;   // batched, same bytes
    }
  }
  Plan P;
  // stage timing events: a pool per host thread and device, kept for the
  // process (events belong to the device they were created on)
  thread_local std::map<int, StageEvents> event_pools;
  StageEvents* ev = nullptr;
  if (o->stage_ms && !async) {
    int dev = 0;
    const hipError_t de = hipGetDevice(&dev);
    if (de != hipSuccess) return fail(VL_ERR_HIP, "device: %s", hipGetErrorString(de));
    StageEvents& events = event_pools[dev];
    for (int i = 0; i < VL_STAGE_COUNT; ++i) o->stage_ms[i] = 0.f;
    events.stage.clear();
    ev = &events;
  }

  // blocking mode: the kernels write the gathered proofs, statuses and
  // digests into pinned host memory; wait, then hand them out
  PinnedOut* po = nullptr;
  auto fetch = [&](uint64_t g0, uint64_t g1) -> vl_status {
    const uint64_t n = g1 - g0;
    const uint64_t pa = align_up(P.out_proof_bytes, 256), sa = align_up(4 * n, 256);
    const hipError_t e = hipStreamSynchronize(s);
    if (e != hipSuccess) return fail(VL_ERR_HIP, "prove: %s", hipGetErrorString(e));
    if (ev) ev->accumulate(o->stage_ms);
    const uint8_t* host = reinterpret_cast<const uint8_t*>(po->host);
    memcpy(proofs + offsets[g0], host, P.out_proof_bytes);
    if (digests) memcpy(digests + 32 * g0, host + pa + sa, 32 * n);
    for (uint64_t i = g0; i < g1; ++i) {
      int32_t st;
      memcpy(&st, host + pa + 4 * (i - g0), 4);
      if (st == VL_ERR_FALSE_STATEMENT)
        return fail(VL_ERR_FALSE_STATEMENT, "group %u: the products do not sum to C", groups[i].group_id);
      if (st == VL_ERR_RANGE)
        return fail(VL_ERR_RANGE, "group %u: an entry of C exceeds the contraction digit range",
                    groups[i].group_id);
      if (st == VL_ERR_TIMEOUT)
        return fail(VL_ERR_TIMEOUT, "group %u: the rounds gave up waiting for the contractions",
                    groups[i].group_id);
      if (st != VL_OK) return fail(VL_ERR_HIP, "group %u: prover status %d", groups[i].group_id, st);
    }
    return VL_OK;
  };
  auto run = [&](uint64_t g0, uint64_t g1) -> vl_status {
    uint8_t* out = nullptr;
    if (!async) {
      const uint64_t n = g1 - g0;
      const uint64_t bytes = align_up(offsets[g1] - offsets[g0], 256) + align_up(4 * n, 256) + 32 * n;
      const hipError_t e = pinned_out(bytes, &po);
      if (e != hipSuccess) return fail(VL_ERR_HIP, "pinned output buffer: %s", hipGetErrorString(e));
      out = reinterpret_cast<uint8_t*>(po->dev);
    }
    plan_groups(P, T, groups, g0, g1, seed, ws, async, proofs, offsets, o->status, digests, out);
    if (P.data_end > o->workspace_bytes)
      return fail(VL_ERR_WORKSPACE, "workspace of %llu bytes, %llu needed",
                  (unsigned long long)o->workspace_bytes, (unsigned long long)align_up(P.data_end, 256));
    const BlobLayout L = blob_layout(P);
    fill_blob(P, L, ws);
    hipStream_t s2 = s, s3 = nullptr;
    if (P.seg.size() > 1 || P.persistent) {
      const hipError_t e2 = rounds_stream_for(s, &s2);
      if (e2 != hipSuccess) return fail(VL_ERR_HIP, "rounds stream: %s", hipGetErrorString(e2));
    }
    if (!ev && plan_forks(P)) {
      const hipError_t e3 = side_stream_for(s, &s3);
      if (e3 != hipSuccess) return fail(VL_ERR_HIP, "side stream: %s", hipGetErrorString(e3));
    }
    hipError_t e = enqueue_plan(P, L, ws, s, s2, ev, nullptr, s3);
    if (e == hipSuccess && gate) {
      // the caller's stream has joined the rounds stream: its position now
      // marks the end of this persistent call
      e = hipEventRecord(gate->done, s);
      if (e == hipSuccess) gate->issued = true;
    }
    if (e != hipSuccess) {
      // what was enqueued before the failure may still write the outputs
      // (the pinned buffer the next blocking call reuses): let it finish
      (void)hipStreamSynchronize(s);
      if (s2 != s) (void)hipStreamSynchronize(s2);
      if (s3) (void)hipStreamSynchronize(s3);
      return fail(VL_ERR_HIP, "launch: %s", hipGetErrorString(e));
    }
    return async ? VL_OK : fetch(g0, g1);
  };
  if (T.per_instance) {
    for (uint64_t i = 0; i < n; ++i) {
      const vl_status st = run(i, i + 1);
      if (st != VL_OK) return st;
    }
    return VL_OK;
  }
  return run(0, n);
}

vl_status vl_fr_lift(const void* src, int32_t dtype, uint64_t n, vl_fr_vec dst, void* stream) {
  if (!src || !dst.base) return fail(VL_ERR_INVALID_ARG, "null pointer");
  if (!esize(dtype)) return fail(VL_ERR_DTYPE, "dtype must be VL_I16/I32/I64");
  if (dst.n < n || dst.ld < dst.n) return fail(VL_ERR_SHAPE, "destination too small");
  const hipError_t e = launch_lift(src, dtype, n, dst.base, dst.ld, reinterpret_cast<hipStream_t>(stream));
  if (e != hipSuccess) return fail(VL_ERR_HIP, "lift: %s", hipGetErrorString(e));
  return VL_OK;
}

vl_status vl_fr_export(vl_fr_vec src, uint64_t n, uint32_t* dst, void* stream) {
  if (!src.base || !dst) return fail(VL_ERR_INVALID_ARG, "null pointer");
  if (src.n < n || src.ld < src.n) return fail(VL_ERR_SHAPE, "source too small");
  const hipError_t e = launch_export(src.base, src.ld, n, dst, reinterpret_cast<hipStream_t>(stream));
  if (e != hipSuccess) return fail(VL_ERR_HIP, "export: %s", hipGetErrorString(e));
  return VL_OK;
}

vl_status vl_eq_table(const vl_fr* point, uint32_t nvars, vl_fr_vec out, void* stream) {
  if ((!point && nvars) || !out.base) return fail(VL_ERR_INVALID_ARG, "null pointer");
  if (nvars > 20) return fail(VL_ERR_SHAPE, "nvars must be <= 20");
  if (out.n < (1ull << nvars) || out.ld < out.n) return fail(VL_ERR_SHAPE, "out.n < 2^nvars");
  EqPointArgs a{};
  a.nvars = nvars;
  a.out = out.base;
  a.ld = out.ld;
  for (uint32_t i = 0; i < nvars; ++i) {
    Fr x;
    memcpy(x.w, point[i].w, 32);
    if (!fr_lt_p(x)) return fail(VL_ERR_INVALID_ARG, "point[%u] is not canonical", i);
    const Fr xm = fr_to_mont(x), om = fr_sub(fr_R(), xm);
    memcpy(a.pt[i][0], xm.w, 32);
    memcpy(a.pt[i][1], om.w, 32);
  }
  const hipError_t e = launch_eq_point(a, reinterpret_cast<hipStream_t>(stream));
  if (e != hipSuccess) return fail(VL_ERR_HIP, "eq_table: %s", hipGetErrorString(e));
  return VL_OK;
}

// ------------------------------------------------------------ graph mode --
// A prove call captured once into a HIP graph.  The graph holds every
// launch of the call with fixed workspace and output addresses; its first
// node copies the descriptor blob from a pinned host buffer of the handle.
// A launch rebuilds the blob for its seed (the challenges and transcript
// states change, the layout does not), writes it into that buffer and
// replays the graph.
}  // extern "C"

struct vl_prove_graph {
  int device = 0;
  std::vector<vl_group> groups;
  std::vector<vl_product> prods;   // the groups' products, owned by the handle
  std::vector<uint8_t> binds;      // 32 bytes per group: the bind digests, owned by the handle
  vl_prove_opts opts{};
  vl_tuning tuning{};
  bool has_tuning = false;
  uint8_t* proofs = nullptr;
  uint8_t* digests = nullptr;
  std::vector<uint64_t> offsets;
  uint64_t blob_total = 0;
  void* pinned = nullptr;
  void* pinned_dev = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  hipEvent_t done = nullptr;
  bool launched = false;
};

namespace vl {
// plans the handle's call for a seed and fills P's blob
static vl_status graph_plan(vl_prove_graph* g, uint64_t seed, Plan& P, BlobLayout& L) {
  const Tuning T = tuning_for(&g->opts);
  plan_groups(P, T, g->groups.data(), 0, g->groups.size(), seed, reinterpret_cast<uint8_t*>(g->opts.workspace),
              true, g->proofs, g->offsets.data(), g->opts.status, g->digests, nullptr);
  if (P.data_end > g->opts.workspace_bytes)
    return fail(VL_ERR_WORKSPACE, "workspace of %llu bytes, %llu needed",
                (unsigned long long)g->opts.workspace_bytes, (unsigned long long)align_up(P.data_end, 256));
  L = blob_layout(P);
  fill_blob(P, L, reinterpret_cast<uint8_t*>(g->opts.workspace));
  return VL_OK;
}

static void graph_free(vl_prove_graph* g) {
  if (!g) return;
  if (g->exec) (void)hipGraphExecDestroy(g->exec);
  if (g->graph) (void)hipGraphDestroy(g->graph);
  if (g->done) (void)hipEventDestroy(g->done);
  if (g->pinned) (void)hipHostFree(g->pinned);
  delete g;
}
}  // namespace vl

extern "C" {

vl_status vl_prove_graph_create(const vl_group* groups, uint64_t n, const vl_prove_opts* o, uint8_t* proofs,
                                uint64_t proofs_len, uint64_t* offsets, uint8_t* digests, vl_prove_graph** out) {
  if (!out) return fail(VL_ERR_INVALID_ARG, "null handle pointer");
  *out = nullptr;
  if (!o) return fail(VL_ERR_INVALID_ARG, "null options");
  if (!o->async) return fail(VL_ERR_INVALID_ARG, "a prove graph writes device-writable outputs: async must be 1");
  // batched mode only: persistent mode's rounds workgroups wait for kernels
  // that a graph executor may run after them
  if (o->mode != VL_MODE_BATCHED) return fail(VL_ERR_INVALID_ARG, "a prove graph runs the batched mode");
  if (o->stage_ms) return fail(VL_ERR_INVALID_ARG, "stage timing is not available in a prove graph");
  {
    const vl_status st = validate_prove(groups, n, o, proofs, proofs_len, offsets, digests);
    if (st != VL_OK) return st;
  }
  vl_prove_graph* g = new vl_prove_graph();
  hipError_t e = hipGetDevice(&g->device);
  // deep copy: every launch re-plans from these descriptors, so the caller
  // may free or reuse its own group and product arrays after create
  g->groups.assign(groups, groups + n);
  {
    uint64_t np = 0;
    for (uint64_t i = 0; i < n; ++i) np += groups[i].n_prods;
    g->prods.reserve(np);
    for (uint64_t i = 0; i < n; ++i) {
      const size_t at = g->prods.size();
      g->prods.insert(g->prods.end(), groups[i].prods, groups[i].prods + groups[i].n_prods);
      g->groups[i].prods = g->prods.data() + at;   // no reallocation: reserved above
    }
    g->binds.assign(32 * n, 0);
    for (uint64_t i = 0; i < n; ++i)
      if (groups[i].bind) {
        memcpy(g->binds.data() + 32 * i, groups[i].bind, 32);
        g->groups[i].bind = g->binds.data() + 32 * i;
      }
  }
  g->opts = *o;
  if (o->tuning) {
    g->tuning = *o->tuning;
    g->has_tuning = true;
    g->opts.tuning = &g->tuning;
  }
  g->proofs = proofs;
  g->digests = digests;
  g->offsets.assign(offsets, offsets + n + 1);
  Plan P;
  BlobLayout L;
  vl_status st = graph_plan(g, 0, P, L);
  if (st != VL_OK) {
    graph_free(g);
    return st;
  }
  g->blob_total = L.total;
  if (e == hipSuccess) e = hipHostMalloc(&g->pinned, L.total, hipHostMallocDefault);
  if (e == hipSuccess) e = hipHostGetDevicePointer(&g->pinned_dev, g->pinned, 0);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&g->done, hipEventDisableTiming);
  // capture on a stream of our own (and, for segmented plans, a second
  // private stream for the rounds, created before the capture starts: not one
  // of the shared rounds streams, which other threads may be using for eager
  // calls while this one captures)
  hipStream_t cs = nullptr, s2 = nullptr, own2 = nullptr, own3 = nullptr;
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking);
  s2 = cs;
  if (e == hipSuccess && (P.seg.size() > 1 || P.persistent)) {
    e = hipStreamCreateWithFlags(&own2, hipStreamNonBlocking);
    if (e == hipSuccess) s2 = own2;
  }
  if (e == hipSuccess && plan_forks(P)) e = hipStreamCreateWithFlags(&own3, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipStreamBeginCapture(cs, hipStreamCaptureModeRelaxed);
  if (e == hipSuccess) {
    const hipError_t e1 = enqueue_plan(P, L, reinterpret_cast<uint8_t*>(g->opts.workspace), cs, s2, nullptr,
                                       g->pinned_dev, own3);
    const hipError_t e2 = hipStreamEndCapture(cs, &g->graph);
    e = e1 != hipSuccess ? e1 : e2;
  }
  if (e == hipSuccess) e = hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0);
  if (cs) (void)hipStreamDestroy(cs);
  if (own2) (void)hipStreamDestroy(own2);
  if (own3) (void)hipStreamDestroy(own3);
  if (e != hipSuccess) {
    graph_free(g);
    return fail(VL_ERR_HIP, "prove graph: %s", hipGetErrorString(e));
  }
  *out = g;
  return VL_OK;
}

vl_status vl_prove_graph_launch(vl_prove_graph* g, uint64_t seed, void* stream) {
  if (!g) return fail(VL_ERR_INVALID_ARG, "null prove graph");
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return fail(VL_ERR_HIP, "device: %s", hipGetErrorString(e));
  if (dev != g->device) return fail(VL_ERR_INVALID_ARG, "the prove graph belongs to device %d", g->device);
  Plan P;
  BlobLayout L;
  const vl_status st = graph_plan(g, seed, P, L);
  if (st != VL_OK) return st;
  if (L.total != g->blob_total) return fail(VL_ERR_INVALID_ARG, "the plan changed since the graph was made");
  // the previous replay must have copied the blob before it is overwritten
  if (g->launched) {
    e = hipEventSynchronize(g->done);
    if (e != hipSuccess) return fail(VL_ERR_HIP, "prove graph: %s", hipGetErrorString(e));
  }
  memcpy(g->pinned, P.blob.data(), L.total);
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  e = hipGraphLaunch(g->exec, s);
  if (e == hipSuccess) e = hipEventRecord(g->done, s);
  if (e != hipSuccess) return fail(VL_ERR_HIP, "prove graph launch: %s", hipGetErrorString(e));
  g->launched = true;
  return VL_OK;
}

vl_status vl_prove_graph_bind(vl_prove_graph* g, const uint8_t* binds) {
  if (!g) return fail(VL_ERR_INVALID_ARG, "null prove graph");
  const uint64_t n = g->groups.size();
  if (binds) memcpy(g->binds.data(), binds, 32 * n);
  for (uint64_t i = 0; i < n; ++i) g->groups[i].bind = binds ? g->binds.data() + 32 * i : nullptr;
  return VL_OK;
}

void vl_prove_graph_destroy(vl_prove_graph* g) {
  if (g && g->launched) (void)hipEventSynchronize(g->done);
  graph_free(g);
}

// layout of the partial-eval workspace: [pack][job blob][split partials]
static uint64_t pe_pack_bytes(uint64_t len) { return align_up(len * 32, 256); }
static constexpr uint64_t kPeBlob = 1024;
}  // extern "C"

namespace vl {
// Argument checks of a partial evaluation (everything but the workspace).
vl_status partial_eval_check(const void* M, int32_t dtype, uint32_t rows, uint32_t cols, uint64_t ld,
                             int32_t contract, vl_fr_vec eq, vl_fr_vec out, const vl_tuning* tuning) {
  if (!M || !eq.base || !out.base) return fail(VL_ERR_INVALID_ARG, "null pointer");
  if (!esize(dtype)) return fail(VL_ERR_DTYPE, "dtype must be VL_I16/I32/I64");
  if (contract != VL_CONTRACT_ROWS && contract != VL_CONTRACT_COLS)
    return fail(VL_ERR_INVALID_ARG, "contract must be VL_CONTRACT_ROWS or VL_CONTRACT_COLS");
  if (rows == 0 || cols == 0 || rows > VL_MAX_DIM || cols > VL_MAX_DIM || ld < cols)
    return fail(VL_ERR_SHAPE, "bad matrix shape");
  const bool rws = contract == VL_CONTRACT_ROWS;
  const uint32_t len = rws ? rows : cols, n_out = rws ? cols : rows;
  if (eq.n < len || eq.ld < eq.n) return fail(VL_ERR_SHAPE, "eq vector shorter than the contraction");
  if (out.n < n_out || out.ld < out.n) return fail(VL_ERR_SHAPE, "out vector too short");
  if (check_tuning(tuning) != VL_OK) return VL_ERR_INVALID_ARG;
  return VL_OK;
}

// Enqueues a checked partial evaluation with its scratch at ws (256-byte
// aligned, at least the workspace size of this shape): the pack table of eq,
// the job blob (uploaded through kernel arguments) and, for a split
// contraction, the chunk partials.  Nothing is allocated.
vl_status partial_eval_launch(const void* M, int32_t dtype, uint32_t rows, uint32_t cols, uint64_t ld,
                              int32_t contract, vl_fr_vec eq, vl_fr_vec out, void* workspace,
                              uint64_t workspace_bytes, const vl_tuning* tuning, void* stream) {
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  const bool rws = contract == VL_CONTRACT_ROWS;
  const uint32_t len = rws ? rows : cols, n_out = rws ? cols : rows;
  uint8_t* ws = reinterpret_cast<uint8_t*>(workspace);
  uint32_t* pack = reinterpret_cast<uint32_t*>(ws);
  uint8_t* dblob = ws + pe_pack_bytes(len);
  Plan P;
  const Tuning T = pe_tuning(tuning);
  Builder B(P, T, reinterpret_cast<uint64_t>(ws), pe_pack_bytes(len) + kPeBlob);
  B.contract(M, dtype, digits_for(dtype), ld, rws, n_out, len, pack, out.base, out.ld, out.n,
             reinterpret_cast<int32_t*>(dblob));
  if (B.off > workspace_bytes)
    return fail(VL_ERR_WORKSPACE, "workspace too small for this matrix's layout");
  int kind = -1;
  const Segment& G = P.seg[0];
  for (int k = 0; k < CK_COUNT; ++k)
    if (!G.cj[k].empty()) kind = k;
  std::vector<uint8_t> blob(kPeBlob, 0);   // [err flag][contract job][finish job]
  const uint64_t jo = 64, fo = 64 + align_up(sizeof(ContractJob), 64);
  memcpy(blob.data() + jo, &G.cj[kind][0], sizeof(ContractJob));
  if (!G.fin.empty()) memcpy(blob.data() + fo, &G.fin[0], sizeof(FinishJob));
  hipError_t e = launch_upload(dblob, blob.data(), blob.size(), s);
  if (e == hipSuccess) e = launch_pack(eq.base, eq.ld, len, pack, s);
  if (e == hipSuccess)
    e = launch_contract(kind, reinterpret_cast<const ContractJob*>(dblob + jo), 1, G.cj_tasks[kind], s);
  if (e == hipSuccess && !G.fin.empty())
    e = launch_finish(reinterpret_cast<const FinishJob*>(dblob + fo), 1, G.fin_blocks, s);
  if (e != hipSuccess) return fail(VL_ERR_HIP, "partial_eval: %s", hipGetErrorString(e));
  return VL_OK;
}
}  // namespace vl

extern "C" {

uint64_t vl_partial_eval_workspace_size(uint32_t rows, uint32_t cols, int32_t contract, int32_t dtype,
                                        const vl_tuning* tuning) {
  if (rows == 0 || cols == 0 || !esize(dtype) ||
      (contract != VL_CONTRACT_ROWS && contract != VL_CONTRACT_COLS))
    return 0;
  const bool rws = contract == VL_CONTRACT_ROWS;
  const uint64_t len = rws ? rows : cols, n_out = rws ? cols : rows;
  if (check_tuning(tuning) != VL_OK) return 0;
  const Tuning T = pe_tuning(tuning);
  // the alignment of M and of its leading dimension (which pick vector or
  // element loads, and with them the chunking) are unknown here: the larger
  // of the two plans, one with M and ld aligned for every vector width, one
  // with M misaligned
  uint64_t need = 0;
  const uint64_t ld_vec = align_up(cols, 16);
  for (int k = 0; k < 2; ++k) {
    const uintptr_t m = k == 0 ? 0 : 2;
    const uint64_t ld = k == 0 ? ld_vec : cols;
    Plan P;
    Builder B(P, T, 0, pe_pack_bytes(len) + kPeBlob);
    B.contract(reinterpret_cast<const void*>(m), dtype, digits_for(dtype), ld, rws, (uint32_t)n_out,
               (uint32_t)len, nullptr, nullptr, 1, n_out, nullptr);
    need = std::max(need, B.off);
  }
  return align_up(need, 256);
}

vl_status vl_mle_partial_eval(const void* M, int32_t dtype, uint32_t rows, uint32_t cols, uint64_t ld,
                              int32_t contract, vl_fr_vec eq, vl_fr_vec out, void* workspace,
                              uint64_t workspace_bytes, const vl_tuning* tuning, void* stream) {
  {
    const vl_status st = vl::partial_eval_check(M, dtype, rows, cols, ld, contract, eq, out, tuning);
    if (st != VL_OK) return st;
  }
  if (!workspace) return fail(VL_ERR_INVALID_ARG, "null pointer");
  if (reinterpret_cast<uintptr_t>(workspace) % 256)
    return fail(VL_ERR_WORKSPACE, "workspace must be 256-byte aligned");
  if (workspace_bytes < vl_partial_eval_workspace_size(rows, cols, contract, dtype, tuning))
    return fail(VL_ERR_WORKSPACE, "workspace too small");
  return vl::partial_eval_launch(M, dtype, rows, cols, ld, contract, eq, out, workspace, workspace_bytes, tuning,
                                 stream);
}

}  // extern "C"
