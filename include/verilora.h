/*
 * verilora.h -- C ABI of the MI355X matmul-sumcheck prover.
 *
 * The library proves matrix-product claims C = A.B (and sums of products)
 * with the sumcheck protocol over the BLS12-381 scalar field Fr.  The field is
 * this library's choice; the paper asks only for |F| ~ 2^254 (Sec. V).  The
 * statement is Sec. II-C: with every dimension zero padded to a power of two,
 *     C~(u, v) = sum_{w in {0,1}^{n1}} A~(u, w) * B~(w, v)            (zk-mle-matmul)
 * for random u, v, where X~ is the multilinear extension of eq. (MLE).  zkMat
 * (Sec. IV-B) applies this to every matrix product of a LoRA step, given the
 * input matrices and the claimed output.
 *
 * Conventions shared by every entry point
 *   - Integer matrices are row-major with a leading dimension "ld" counted in
 *     elements (ld >= number of columns).  Signed integers enter the field as
 *     x mod p, so x < 0 becomes p - |x|.
 *   - A vl_fr_vec is a device vector of Fr elements in Montgomery form
 *     (x * 2^256 mod p) stored as structure-of-limbs: 32-bit limb j
 *     (little-endian, j = 0..7) of element k is at base[j * ld + k].
 *   - A vl_fr passed to or from the host is canonical (< p), little-endian.
 *   - Index bits are read most-significant first: index i of a length-2^n
 *     vector is the point (b_1, ..., b_n) with b_1 the top bit.
 *   - "stream" is a hipStream_t (NULL for the default stream).  Device
 *     calls are asynchronous on that stream unless stated otherwise.
 *   - The caller owns every buffer.  No entry point allocates device memory;
 *     scratch space comes from a caller-provided workspace.
 *   - Every call returns a vl_status; on failure vl_last_error() gives a
 *     message (thread-local, valid until the next call on that thread).
 */
#ifndef VERILORA_H
#define VERILORA_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  VL_OK = 0,
  VL_ERR_INVALID_ARG = 1,      /* null pointer, bad enum, inconsistent sizes   */
  VL_ERR_SHAPE = 2,            /* a dimension is 0, too large, or mismatched   */
  VL_ERR_DTYPE = 3,            /* unsupported element type                     */
  VL_ERR_WORKSPACE = 4,        /* workspace smaller than the size query says   */
  VL_ERR_HIP = 5,              /* a HIP runtime call failed                    */
  VL_ERR_FALSE_STATEMENT = 6,  /* the products do not sum to C: no proof       */
  VL_ERR_REJECT = 7,           /* verification failed                          */
  VL_ERR_BUFFER_TOO_SMALL = 8, /* an output buffer is too small                */
  VL_ERR_RANGE = 9,            /* a claimed C entry is outside the range the
                                  planned contraction digits represent (about
                                  |C| >= 2^47 for int64 C of int16 products)   */
  VL_ERR_TIMEOUT = 10          /* persistent mode: a group's rounds gave up
                                  waiting for its contractions (spin limit)    */
} vl_status;

typedef enum { VL_I16 = 1, VL_I32 = 2, VL_I64 = 3 } vl_dtype;

enum { VL_CONTRACT_ROWS = 0, VL_CONTRACT_COLS = 1 };
/* PER_INSTANCE: each group planned and launched on its own, one after the
 * other.  BATCHED: all groups in one launch per stage.  PERSISTENT
 * (experimental, slower than BATCHED on the 7B-class block): like BATCHED,
 * but the rounds workgroups (one per group) are launched first, on an
 * internal stream, and stay resident: each waits (bounded, see
 * vl_tuning.spin_limit) for its group's contractions, so the sumchecks of
 * early groups overlap the contractions of later ones.  This needs the
 * internal stream and the caller's stream on different hardware queues and
 * free CUs for the contractions; if they share a queue the rounds give up
 * after spin_limit polls with VL_ERR_TIMEOUT.  At most 128 groups per call,
 * and at most one persistent call per device at a time: a call made while
 * another persistent call is still running on the device runs in BATCHED
 * mode instead (same bytes). */
enum { VL_MODE_PER_INSTANCE = 0, VL_MODE_BATCHED = 1, VL_MODE_PERSISTENT = 2 };

typedef struct { uint32_t w[8]; } vl_fr;

typedef struct {
  uint32_t* base;
  uint64_t n;   /* number of elements                          */
  uint64_t ld;  /* plane stride in 32-bit words, ld >= n        */
} vl_fr_vec;

/* One product op(A) . op(B).  Without transposition A is D0 x D1 (lda >= D1)
 * and B is D1 x D2 (ldb >= D2).  With trans_a the stored A is D1 x D0
 * (lda >= D0) and op(A) is its transpose; likewise trans_b stores B as
 * D2 x D1 (ldb >= D1).  A and B are device pointers for proving and host
 * pointers (or NULL) for verification. */
typedef struct {
  const void* A;
  const void* B;
  int32_t dtype_a, dtype_b;
  uint32_t D0, D1, D2;
  uint64_t lda, ldb;
  int32_t trans_a, trans_b;
} vl_product;

/* A group: products sharing D0 and D2 whose sum is the claimed C (D0 x D2,
 * ldc >= D2).  A group of one product is a plain matmul; more products prove
 * a sum of products (zkMat covers additions, Sec. IV-B).  group_id and the
 * seed key the group's own Fiat-Shamir transcript.
 * bind: NULL, or 32 host bytes that the transcript absorbs (label "bind")
 * right after its initial state, before the challenges u and v: a digest of
 * the caller's commitments to the group's matrices (for instance SHA-256 of
 * their vl_hyrax_commit points).  Sec. II-C has the verifier draw its point
 * only after the commitments of Sec. II-A; with a bind the point depends on
 * them, so C cannot be chosen after u and v are known.  Read during the
 * call (vl_prove_graph_create copies it); the verifier is given the same
 * digest. */
typedef struct {
  const vl_product* prods;
  uint32_t n_prods;      /* 1 .. VL_MAX_PRODS */
  uint32_t group_id;
  const void* C;
  int32_t dtype_c;
  uint64_t ldc;
  const uint8_t* bind;   /* optional 32-byte commitment digest, see above */
} vl_group;

#define VL_MAX_PRODS 8
#define VL_MAX_DIM (1u << 20)

/* Launch-shape knobs, for autotuning.  A zero field takes the library's
 * default.  No value changes any result: they only decide how the
 * contractions are cut into wave tasks and how a batched call is pipelined. */
typedef struct {
  uint32_t lane_macs;      /* multiply-adds per lane and contraction task (default
                              8192; when left 0, asynchronous calls and graphs
                              whose groups stream 1 GB or more of matrices cut
                              int16 contractions over rows 16 times longer)      */
  uint32_t min_tasks;      /* halve a contraction's chunk until it has this many
                              wave tasks (chunks stay >= 256 entries)               */
  uint32_t segments;       /* batched mode: pipeline segments, 1..8; the rounds of
                              one segment overlap the contractions of the next
                              (default 2 in blocking calls, 1 otherwise)          */
  uint32_t cols_rows;      /* rows per lane in the vector cols kernels (int16 and
                              |x| < 2^47 int64): 1 or 2                            */
  uint32_t spin_limit;     /* persistent mode: polls (about 0.2 us each) of a
                              group's readiness before its rounds give up with
                              VL_ERR_TIMEOUT                                       */
  uint32_t claim_order;    /* the claim's contraction over C: 0 = by rows when C
                              has >= 256 columns, else by columns; 1 = always by
                              columns, t[i] = sum_j C[i][j] eq(v, j); 2 = always
                              by rows, s[j] = sum_i eq(u, i) C[i][j]              */
  uint32_t contract_streams; /* batched mode: 2 = the contraction kinds of a
                              pipeline segment with two or more large kinds run
                              on two streams (joined before the finish pass);
                              1 = one stream.  Default: 2 for blocking calls, 1
                              for asynchronous calls and prove graphs (several
                              proofs in flight share the hardware queues).
                              Calls that ask for stage times always use one      */
} vl_tuning;

typedef struct {
  int32_t mode;            /* VL_MODE_*; every mode yields identical bytes            */
  int32_t async;           /* 0: proofs/digests are host buffers and the call returns
                              after they are written (the kernels write them into
                              pinned host memory of the library, no copy-engine
                              transfer); 1: they are device-writable buffers, the
                              call only enqueues work, and per-group status codes
                              land in status[]                                       */
  void* workspace;         /* device memory, >= vl_workspace_size() bytes, 256-byte
                              aligned                                                 */
  uint64_t workspace_bytes;
  int32_t* status;         /* async only: device-writable int32[n_groups], VL_OK /
                              VL_ERR_*                                                */
  const vl_tuning* tuning; /* optional launch shape; NULL: defaults                    */
  float* stage_ms;         /* optional host float[VL_STAGE_COUNT] (blocking mode only):
                              device time of each stage, from HIP events recorded on
                              the call's stream around the stage's launches, summed over
                              the call; see VL_STAGE_*                                */
} vl_prove_opts;

/* stages of a prove call, in launch order */
#define VL_STAGE_UPLOAD 0      /* job descriptors to device memory                 */
#define VL_STAGE_EQ 1          /* eq tables and their byte-sliced "pack" form      */
#define VL_STAGE_CONTRACT 2    /* + kind: integer contraction kernels, 19 kinds:
                                  int16 rows (1 column per lane; 4 columns with
                                  element loads; 4 columns with 8-byte loads),
                                  int16 cols (element loads; 16-byte row loads,
                                  1 or 2 rows per lane); int32 rows (1 column;
                                  4 columns with 16-byte loads), cols, cols-vec;
                                  int64 with |x| < 2^47 rows (1 column; 2 columns
                                  with 16-byte loads), cols, cols-vec (1 or 2
                                  rows per lane); int64 rows (1 column; 2
                                  columns with 16-byte loads), cols, cols-vec     */
#define VL_STAGE_FINISH 21     /* split-contraction sums and zero padding          */
#define VL_STAGE_PASS1 22      /* claim c and round 1 of every product, as partial
                                  sums across the GPU                              */
#define VL_STAGE_ROUNDS 23     /* prover guard, sumcheck rounds, proof bytes       */
#define VL_STAGE_COUNT 24

/* Lift n signed integers (dtype) at device pointer src into Fr (Montgomery,
 * structure-of-limbs) at dst (dst.n >= n).  Negative x becomes p - |x|.
 * The quantised tensors of a LoRA step hold signed fixed-point values from a
 * bounded domain F_B = {-B/2, ..., B/2 - 1} of the field (Sec. IV-A,
 * zkSwiGLU, which quantises with a scale factor zeta); the field element of
 * such an x is x mod p, so that sums and products of lifted values are the
 * lifted integer sums and products (eq. (matmul) then holds in F exactly when
 * it holds over the integers without wrap-around).  The prove call performs
 * the same lift inside its contraction kernels; this entry point
 * materialises it for small tensors and tests.
 * Errors: VL_ERR_INVALID_ARG (null src or dst.base), VL_ERR_DTYPE,
 * VL_ERR_SHAPE (dst.n < n or dst.ld < dst.n), VL_ERR_HIP (launch). */
vl_status vl_fr_lift(const void* src, int32_t dtype, uint64_t n, vl_fr_vec dst, void* stream);

/* Convert n elements of a device vl_fr_vec to canonical form, written
 * element-major to the device array dst (8 words per element). */
vl_status vl_fr_export(vl_fr_vec src, uint64_t n, uint32_t* dst, void* stream);

/* eq table of eq. (MLE): out[i] = prod_j (x_j b_j(i) + (1 - x_j)(1 - b_j(i)))
 * for i < 2^nvars (b_1 = top bit).  point: host array of nvars canonical
 * elements; out.n must be >= 2^nvars.  nvars <= 20. */
vl_status vl_eq_table(const vl_fr* point, uint32_t nvars, vl_fr_vec out, void* stream);

/* Workspace bytes needed by vl_mle_partial_eval for this shape. */
uint64_t vl_partial_eval_workspace_size(uint32_t rows, uint32_t cols, int32_t contract, int32_t dtype,
                                        const vl_tuning* tuning);

/* Partial evaluation of a matrix MLE (the A~(u, .) and B~(., v) of
 * eq. (zk-mle-matmul)).  M: device rows x cols integers (dtype), row-major,
 * leading dimension ld.
 *   VL_CONTRACT_ROWS: out[c] = sum_r eq[r] M[r][c]   (needs eq.n >= rows)
 *   VL_CONTRACT_COLS: out[r] = sum_c M[r][c] eq[c]   (needs eq.n >= cols)
 * Entries of out beyond the result length (cols resp. rows) up to out.n are
 * set to zero, so out is the zero-padded table of a multilinear function.
 * tuning: optional (NULL: defaults); the workspace size depends on it.
 * workspace: device memory, 256-byte aligned. */
vl_status vl_mle_partial_eval(const void* M, int32_t dtype, uint32_t rows, uint32_t cols,
                              uint64_t ld, int32_t contract, vl_fr_vec eq, vl_fr_vec out,
                              void* workspace, uint64_t workspace_bytes, const vl_tuning* tuning,
                              void* stream);

/* vl_mle_partial_eval for callers that cannot allocate device memory (code
 * under stream capture, tight serving loops, harnesses that forbid
 * allocation): the same operation, arguments and results, with no workspace
 * argument.  Its scratch is a fixed device array of the library,
 * VL_NOALLOC_SCRATCH_BYTES per GPU, held by every GPU the library runs on
 * until the process ends; the call allocates nothing.  A shape whose
 * vl_partial_eval_workspace_size exceeds that size is refused with
 * VL_ERR_WORKSPACE before any device work.  Every call on one GPU uses that
 * GPU's one array: calls that overlap on a GPU (other streams, other host
 * threads) race and must be ordered by the caller. */
#define VL_NOALLOC_SCRATCH_BYTES (64ull << 20)
vl_status vl_mle_partial_eval_noalloc(const void* M, int32_t dtype, uint32_t rows, uint32_t cols,
                                      uint64_t ld, int32_t contract, vl_fr_vec eq, vl_fr_vec out,
                                      const vl_tuning* tuning, void* stream);

/* Bytes of one group's proof:
 * 32 * (1 + (n_prods - 1) + sum over products of (3 * n1 + 2)),
 * n1 = ceil(log2 D1).  Layout: c || part claims || per product the round
 * values g(0), g(1), g(2) per round || a_final || b_final, each a canonical
 * 32-byte little-endian field element. */
uint64_t vl_proof_size(const vl_group* group);

/* Device workspace needed to prove these groups with these options. */
uint64_t vl_workspace_size(const vl_group* groups, uint64_t n_groups, const vl_prove_opts* opts);

/* Prove every group (the matmul sumcheck of eq. (zk-mle-matmul), Sec. II-C,
 * run by zkMat for each product of a LoRA step, Sec. IV-B).
 *   proofs   : host (async = 0) or device-writable (async = 1) buffer of
 *              proofs_len bytes; group g's proof starts at offsets[g].
 *              Device-writable means device memory or pinned host memory
 *              (hipHostMalloc) given by its device-side address: the
 *              kernels then write the proof bytes straight into host memory,
 *              with no copy afterwards
 *   offsets  : host uint64[n_groups + 1], filled by the call
 *   digests  : optional (NULL) 32 bytes per group, the final transcript
 *              state; host or device-writable like proofs
 * The proof of a group depends only on (its matrices, seed, group_id); the
 * mode, the batching and other groups never change a byte.  Returns
 * VL_ERR_FALSE_STATEMENT (async = 0) if some group's products do not sum to
 * its C; in async mode that code lands in status[g] instead. */
vl_status vl_sumcheck_matmul_prove(const vl_group* groups, uint64_t n_groups, uint64_t seed,
                                   const vl_prove_opts* opts, uint8_t* proofs, uint64_t proofs_len,
                                   uint64_t* offsets, uint8_t* digests, void* stream);

/* The same batched prove captured once into a HIP graph (one graph launch per
 * call instead of the call's dozen kernel launches; Sec. IV-B's per-step
 * proofs of one block repeat with new data and seeds but the same shapes).
 * create: plans the groups with opts (async = 1, batched mode, no
 *   stage_ms), fills offsets, and captures every launch with
 *   the workspace, proofs, opts->status and digests addresses fixed; the
 *   caller keeps those buffers, and the matrices the groups point to, alive
 *   and unused by other work until destroy.  The group and product
 *   descriptors are copied (deep, bind digests included): the caller may
 *   free or reuse its vl_group and vl_product arrays and bind buffers after
 *   create; a launch reads the matrices at the same addresses.
 * launch: proves the groups' current matrix contents for seed on stream,
 *   asynchronously, with bytes identical to vl_sumcheck_matmul_prove.  The
 *   host rebuilds the descriptor blob (challenges depend on the seed and
 *   group ids) and writes it into a pinned buffer of the handle, which the
 *   graph's first kernel copies; a launch first waits for the previous
 *   launch of the same handle to finish.  Launches of one handle run one at
 *   a time; use one handle per workspace for overlap.
 * destroy: waits for the last launch and frees the handle (NULL is a no-op).
 * Errors: VL_ERR_INVALID_ARG (bad options, wrong device), VL_ERR_WORKSPACE,
 * VL_ERR_BUFFER_TOO_SMALL, VL_ERR_HIP; a failed create returns no handle. */
typedef struct vl_prove_graph vl_prove_graph;
vl_status vl_prove_graph_create(const vl_group* groups, uint64_t n_groups, const vl_prove_opts* opts,
                                uint8_t* proofs, uint64_t proofs_len, uint64_t* offsets, uint8_t* digests,
                                vl_prove_graph** graph);
vl_status vl_prove_graph_launch(vl_prove_graph* graph, uint64_t seed, void* stream);

/* Replaces the bind digests of a prove graph's groups for its next launches
 * (new data comes with new commitments, Sec. II-C): binds is NULL (no group
 * binds) or 32 host bytes per group in the order given to create, copied
 * here.  Not concurrent with a launch of the same handle.  Errors:
 * VL_ERR_INVALID_ARG. */
vl_status vl_prove_graph_bind(vl_prove_graph* graph, const uint8_t* binds);
void vl_prove_graph_destroy(vl_prove_graph* graph);

/* Host-side verifier (CPU only) of the sumcheck of eq. (zk-mle-matmul)
 * (Sec. II-C).  Replays the Fiat-Shamir transcript for (shape, seed,
 * group_id) -- every challenge is a hash of all earlier public messages (the
 * Fiat-Shamir footnote of Sec. IV-A, random-oracle model of Sec. V) -- and
 * runs the verifier's side of the sumcheck rounds (Sec. II-B.1): g(0) + g(1)
 * must equal the running claim in every round, the claim then moves to g(r)
 * by interpolation on {0, 1, 2}, and the last claim must equal
 * a_final * b_final, the product of the two evaluations at the random point
 * that ends eq. (zk-mle-matmul)'s protocol.  If the group's A, B (every
 * product) and C pointers are all non-NULL they are read as HOST matrices and
 * c = C~(u, v), a_final = A~(u, r), b_final = B~(r, v) are also checked by
 * direct evaluation of eq. (MLE), standing in for the commitment openings of
 * Sec. II-A, which are out of scope.
 * Commitments: the group's bind digest, if any, enters the transcript before
 * u and v, as in the prover.  In the paper the verifier draws u and v after
 * the prover has committed to the matrices (Sec. II-A, II-C).  Without a
 * bind, u and v follow from (seed, group_id, shapes) alone, nothing ties C
 * to them, and the witness check does not rule out a false C' = AB + D with
 * D~(u, v) = 0 chosen after seeing u and v.  With a bind of commitments to
 * A, B and C, the verifier checks the reduced claims below by openings
 * (vl_hyrax_verify_open: A at (u, r), B at (r, v), C at (u, v)) instead of
 * the witness.
 *   reduced : optional host output of the reduced claims, canonical:
 *             c, u[n0], v[n2], then per product r[n1], a_final, b_final
 *   reduced_len : elements written (or needed, on VL_ERR_BUFFER_TOO_SMALL)
 *   fail_round  : 1-based round of the group that failed, 0 for a length or
 *                 encoding error or a failed final or witness check, -1 on VL_OK
 * Returns VL_OK or VL_ERR_REJECT. */
vl_status vl_verify_transcript(const uint8_t* proof, uint64_t len, const vl_group* group,
                               uint64_t seed, vl_fr* reduced, uint64_t reduced_cap,
                               uint64_t* reduced_len, int32_t* fail_round);

/* One LoRA layer's training step (forward, backward and update of one LoRA
 * target) as a chain of claims in one Fiat-Shamir transcript: the sequential
 * composition of Sec. IV-B, where each step justifies exactly the
 * point-value claims the step before it fixed, applied to zkMat's products
 * and additions and to the update of eq. (grad_update_ab).
 * Tensors (device pointers, row-major, leading dimension = columns):
 *   int16: X (T x d_in), W (d_in x d_out), A (d_in x r), B (r x d_out),
 *          dY (T x d_out), H and G (T x r; the re-quantised X A and dY B^T)
 *   int64: Y = X W + H B (T x d_out), C2 = X A, C4 = dY B^T (T x r),
 *          dA = X^T G (d_in x r), dB = H^T dY (r x d_out),
 *          dX = dY W^T + G A^T (T x d_in),
 *          UA = 2^F A - eta dA, UB = 2^F B - eta dB (the update before its
 *          rounding to the next step's int16 parameters)
 * The proof has four stages: (1) UA~, A~, dA~ at a random point zA and UB~,
 * B~, dB~ at zB, with UA~ = 2^F A~ - eta dA~ and the same for B (the update
 * is linear, so it holds iff it holds at a random point); (2) points zY, zX,
 * z2, z4 for Y, dX, C2 and C4; (3) the sumchecks of eq. (zk-mle-matmul) of
 * the groups {X^T G} = dA at zA, {H^T dY} = dB at zB, {X W, H B} = Y at zY,
 * {dY W^T, G A^T} = dX at zX, {X A} = C2 at z2 and {dY B^T} = C4 at z4, each
 * on its own branch H(st || "fork" || k) of the transcript; (4) the claims
 * these leave on each of X, W, A, B, dY, H, G reduced to one: a random
 * combination sum_k rho_k M~(x_k, y_k), one sumcheck over the row variables,
 * then one over the column variables, ending at a single claim M~(r, s)
 * (branches H(st || "rfork" || j)).  The claims left at the end (one per
 * tensor, and those on UA, UB, Y, dX, C2 and C4) are for the openings of
 * committed tensors (Sec. II-A, out of scope).
 * Constraints: T + r, d_in + r and d_out + r are at most 2^16 (two 24-bit
 * digits then hold every int64 result of int16 products); F <= 62.
 * Blocking call: it synchronises the stream three times (the host squeezes
 * each stage's points from the proof bytes the kernels wrote) and returns
 * after the proof (vl_lora_chain_proof_size bytes) and the final transcript
 * state (digest, 32 bytes, optional) are in host memory.
 * Errors: VL_ERR_INVALID_ARG, VL_ERR_SHAPE, VL_ERR_WORKSPACE,
 * VL_ERR_BUFFER_TOO_SMALL, VL_ERR_FALSE_STATEMENT (the update relation or a
 * product group does not hold), VL_ERR_RANGE, VL_ERR_HIP. */
typedef struct {
  uint32_t T, d_in, d_out, r;
  uint32_t F, eta;
  const int16_t* X;
  const int16_t* W;
  const int16_t* A;
  const int16_t* B;
  const int16_t* dY;
  const int16_t* H;
  const int16_t* G;
  const int64_t* Y;
  const int64_t* C2;
  const int64_t* C4;
  const int64_t* dA;
  const int64_t* dB;
  const int64_t* dX;
  const int64_t* UA;
  const int64_t* UB;
} vl_lora_layer;

uint64_t vl_lora_chain_proof_size(const vl_lora_layer* layer);
uint64_t vl_lora_chain_workspace_size(const vl_lora_layer* layer);
vl_status vl_lora_chain_prove(const vl_lora_layer* layer, uint64_t seed, void* workspace, uint64_t workspace_bytes,
                              uint8_t* proof, uint64_t proof_len, uint8_t* digest, void* stream);

/* Per-head batched products (multi-head attention, Sec. III-A, eq. (att):
 * S_h = Q_h K_h^T and O_h = P_h V_h for every head h, and the backward
 * products dP = dO V^T, dV = P^T dO, dQ = dS K, dK = dS^T Q).  One vl_bmm
 * states C_h = op(A_h) op(B_h) for h < H; all H are proved by one sumcheck
 * over the head variables and the inner variables of
 *     C~(rho, u, v) = sum_h sum_w eq(rho, h) A~(h, u, w) B~(h, w, v),
 * the multilinear extension of eq. (MLE) over (head, row, column) with the
 * head index most significant and every dimension zero padded to a power of
 * two (Sec. II-C), for random rho, u, v (squeezed in that order).  Head
 * rounds come first and have degree 3; the inner rounds have degree 2 (the
 * matmul sumcheck of eq. (zk-mle-matmul) scaled by eq(rho, r_h)).
 * Head h's stored A is the matrix at A + h * head_stride_a elements: D0 x D1
 * row-major with leading dimension lda, or D1 x D0 if trans_a (op = its
 * transpose); likewise B (D1 x D2, or D2 x D1 if trans_b) and C (D0 x D2,
 * ldc).  Heads may sit side by side in the columns of one matrix (Q of
 * T x (H dh): head_stride = dh, ld = H dh) or stacked (an H x T x T array:
 * head_stride = T T, ld = T).  Pointers are device memory for proving and
 * host memory (or NULL) for verification.
 * Transcript: st = H("VeriLoRA-zkBMat-v1" || u64 seed || u32 group_id ||
 * u32 H || u32 D0 || u32 D1 || u32 D2), squeezes "h" (nh), "u" (n0), "v"
 * (n2), absorbs "claim" c, "round" (4 values per head round, 3 per inner
 * round, challenge "r"), "final" (a_final || b_final).
 * Proof: c || (g0..g3) per head round || (g0, g1, g2) per inner round ||
 * a_final || b_final, 32-byte canonical elements; vl_bmm_proof_size bytes.
 * Limits: H, D0, D1, D2 in 1 .. 2^20, nh + n1 <= 26. */
typedef struct {
  const void* A;
  const void* B;
  const void* C;
  int32_t dtype_a, dtype_b, dtype_c;
  uint32_t H, D0, D1, D2;
  uint64_t lda, ldb, ldc;
  uint64_t head_stride_a, head_stride_b, head_stride_c;
  int32_t trans_a, trans_b;
  uint32_t group_id;
} vl_bmm;

uint64_t vl_bmm_proof_size(const vl_bmm* b);
uint64_t vl_bmm_workspace_size(const vl_bmm* b, uint64_t n);
/* Prove n batched products with the sumcheck rounds of Sec. II-B.1 over the
 * statement above (blocking: returns after every proof is in the
 * host buffer proofs; group k's proof at offsets[k], offsets has n + 1
 * entries).  digests: optional host buffer of 32 bytes per product (the
 * final transcript state).  workspace: device memory of at least
 * vl_bmm_workspace_size bytes, 256-byte aligned.  The proof of a product
 * depends only on its matrices, seed and group_id.  Errors: VL_ERR_INVALID_ARG,
 * VL_ERR_SHAPE, VL_ERR_DTYPE, VL_ERR_WORKSPACE, VL_ERR_BUFFER_TOO_SMALL,
 * VL_ERR_FALSE_STATEMENT (some product's C is not the heads' products),
 * VL_ERR_RANGE, VL_ERR_HIP. */
vl_status vl_bmm_prove(const vl_bmm* b, uint64_t n, uint64_t seed, void* workspace, uint64_t workspace_bytes,
                       uint8_t* proofs, uint64_t proofs_len, uint64_t* offsets, uint8_t* digests, void* stream);
/* Host verifier (CPU only) of one batched proof: the rounds as above
 * (g(0) + g(1) equals the running claim; the claim moves to g(r) by
 * interpolation on {0, 1, 2, 3} or {0, 1, 2}), and the last claim must be
 * eq(rho, r_h) a_final b_final.  If b's A, B and C are all non-NULL they are
 * read as host tensors and c = C~(rho, u, v), a_final = A~(r_h, u, r_w),
 * b_final = B~(r_h, r_w, v) are checked by direct evaluation (standing in for
 * the commitment openings of Sec. II-A; the same caveat as
 * vl_verify_transcript: nothing binds C before the challenges).
 * reduced: optional, canonical: c, rho[nh], u[n0], v[n2], r[nh + n1],
 * a_final, b_final.  fail_round: 1-based failing round, 0 for a length,
 * encoding, final or witness failure, -1 on VL_OK. */
vl_status vl_bmm_verify(const uint8_t* proof, uint64_t len, const vl_bmm* b, uint64_t seed, vl_fr* reduced,
                        uint64_t reduced_cap, uint64_t* reduced_len, int32_t* fail_round);

/* Lookup arguments (Protocol 1, Sec. II-D): every entry of a secret tensor
 * S lies in a public table T.  With m_j the multiplicity of row j in S, the
 * identity of eq. (rational-function) at a random beta,
 *     sum_i 1/(beta + s_i) = sum_j m_j/(beta + t_j),
 * and the inverse relations are proved by the sumcheck of
 * eq. (lookup-sumcheck) over the D' entries x = (x_H, x_L):
 *     alpha + alpha^2 = sum_x alpha A(x) eq(u, x) (S(x) + beta) + A(x)
 *         + (N/D') alpha^2 B(x_L) eq(u_L, x_L) (T(x_L) + beta)
 *         - (N/D') B(x_L) m(x_L),
 * A = 1/(beta + S), B = 1/(beta + T), u_L the last log N coordinates of u;
 * rounds bind the most significant bit first and have degree 3.
 * Table rows are (t0 + j) for j < N (N a power of two), or with two_col the
 * pairs (t0 + j, tb[j]), compressed as (t0 + j) + gamma tb[j] and entries as
 * x_i + gamma y_i (a range check, or the input/output table of an
 * element-wise function: zkSwiGLU, zkSoftmax, zkElementProd and
 * zkTranspose of Sec. IV-A build on this).  S is padded to
 * D' = max(N, 2^ceil(log2 D)) entries with the table's first row.
 * Transcript: st = H("VeriLoRA-lookup-v1" || u64 seed || u32 id || u64 D ||
 * u32 N || i32 t0 || u32 two_col), squeezes "gamma" (two_col only),
 * "beta", "alpha", "u" (log2 D'), absorbs "round" (g(0..3), challenge "r")
 * and "final" (A(r), S(r), B(r_L), T(r_L), m(r_L)).  The claimed sum is not
 * sent.  Proof: (g0..g3) per round || the five final values, canonical
 * 32-byte elements, vl_lookup_proof_size bytes.
 * x, y: D int16 or int32 entries (dtype, dtype_y); tb: N int32; device pointers for
 * proving, host pointers (or NULL: shape only) for verification. */
typedef struct {
  const void* x;
  const void* y;
  const int32_t* tb;
  int32_t dtype;     /* of x */
  int32_t dtype_y;   /* of y (two_col) */
  int32_t t0;
  int32_t two_col;
  uint32_t N;
  uint64_t D;
  uint32_t id;
} vl_lookup;

uint64_t vl_lookup_proof_size(const vl_lookup* l);
uint64_t vl_lookup_workspace_size(const vl_lookup* l, uint64_t n);
/* Prove n lookups with the sumcheck rounds of Sec. II-B.1 over the sum
 * above (blocking; proofs, offsets (n + 1) and digests (optional, 32 bytes
 * each) in host memory; workspace of vl_lookup_workspace_size bytes,
 * 256-byte aligned).  The multiplicities, inverses, tables and rounds are
 * computed on the device.  Errors: VL_ERR_INVALID_ARG, VL_ERR_SHAPE,
 * VL_ERR_DTYPE, VL_ERR_WORKSPACE, VL_ERR_BUFFER_TOO_SMALL,
 * VL_ERR_FALSE_STATEMENT (an entry is not a row of the table, or beta hit a
 * pole), VL_ERR_HIP. */
vl_status vl_lookup_prove(const vl_lookup* l, uint64_t n, uint64_t seed, void* workspace, uint64_t workspace_bytes,
                          uint8_t* proofs, uint64_t proofs_len, uint64_t* offsets, uint8_t* digests, void* stream);
/* Host verifier of one lookup proof (Sec. II-B.1 rounds, cubic
 * interpolation, and the summand of eq. (lookup-sumcheck) at r from the five
 * final values).  If x (and y, tb with two_col) are host pointers, the
 * final values are also checked against the multilinear extensions of the
 * padded S, T, the multiplicities and the inverses (standing in for the
 * openings of Sec. II-A).  reduced: gamma, beta, alpha, u, r, the five final
 * values (canonical).  fail_round as for vl_bmm_verify. */
vl_status vl_lookup_verify(const uint8_t* proof, uint64_t len, const vl_lookup* l, uint64_t seed, vl_fr* reduced,
                           uint64_t reduced_cap, uint64_t* reduced_len, int32_t* fail_round);

/* Hyrax commitments to matrix MLEs: the polynomial commitments of Sec. II-A,
 * with the scheme the paper's implementation uses (Hyrax; its commitment
 * times and sizes are those of Table t2).  The multilinear extension of an
 * R x m integer matrix M (eq. (MLE), rows indexed by the first log2 R
 * variables, both dimensions zero padded to powers of two) is committed row
 * by row with Pedersen vector commitments in G1 of BLS12-381, the group of
 * order p (the order of Fr):
 *     C_i = sum_{j < m} M[i][j] G_j            (i < R; padded rows commit to 0)
 * and opened at a point (x, y) with w = sum_i eq(x, i) M[i][.] (m elements:
 * the partial evaluation vl_mle_partial_eval computes with
 * VL_CONTRACT_ROWS); the verifier checks
 *     sum_j w_j G_j = sum_i eq(x, i) C_i
 * and takes M~(x, y) = sum_j w_j eq(y, j).  Commitments are binding, not
 * hiding (no blinding term).
 * Generators: G_j by try-and-increment hashing to the curve y^2 = x^3 + 4:
 * for ctr = 0, 1, ..: X = LE(H(t || 0) || H(t || 1)) mod q with
 * t = "VeriLoRA-hyrax-v1" || u32 j || u32 ctr and H = SHA-256; the first
 * ctr for which X^3 + 4 is a square gives the point (X, y) with y its even
 * square root, and G_j = 0xd201000000010001 (X, y) (cofactor clearing into
 * the order-p subgroup).
 * Points are 96 bytes: x then y, each 48 bytes little-endian canonical; the
 * point at infinity is 96 zero bytes. */
#define VL_HYRAX_POINT_BYTES 96

/* Device bytes of the fixed-base table of m generators and W windows:
 * m * W * 128 * 96 (0 for m outside 1 .. 2^20 or W outside 1 .. 8). */
uint64_t vl_hyrax_table_size(uint32_t m, uint32_t windows);

/* Computes the public parameters on the device: for j < m, w < W and
 * k = 1..128 the affine point k 256^w G_j (Montgomery coordinates), point
 * ((j W + w) 128 + k - 1) of table.  A table of W windows commits entries of
 * up to W bytes (int16: 2, int32: 4, int64: 8) with one mixed addition per
 * nonzero signed base-256 digit.  table: device memory of
 * vl_hyrax_table_size bytes, 16-byte aligned, owned by the caller.
 * Asynchronous on stream.  Errors: VL_ERR_SHAPE, VL_ERR_INVALID_ARG,
 * VL_ERR_BUFFER_TOO_SMALL, VL_ERR_HIP. */
vl_status vl_hyrax_setup(uint32_t m, uint32_t windows, void* table, uint64_t table_bytes, void* stream);

/* Device workspace bytes of vl_hyrax_commit for R rows, m columns and the
 * given split (0 = the library's choice); 0 for a bad shape. */
uint64_t vl_hyrax_commit_workspace_size(uint32_t R, uint32_t m, uint32_t split);

/* Commits to the rows of M (device, R x m, row-major, leading dimension
 * ld >= m, dtype VL_I16/I32/I64; negative entries are x mod p) with a table
 * from vl_hyrax_setup of table_m >= m generators and windows >= the entry's
 * byte size.  commits: device memory of R * 96 bytes (4-byte aligned),
 * row i's commitment at 96 i.  split: column slices per row, 0 = the
 * library's choice, else 1 .. ceil(m / 64); it changes how the work is cut,
 * never the bytes.  workspace: vl_hyrax_commit_workspace_size bytes,
 * 256-byte aligned.  Asynchronous on stream.  Errors: VL_ERR_INVALID_ARG,
 * VL_ERR_SHAPE, VL_ERR_DTYPE, VL_ERR_WORKSPACE, VL_ERR_HIP. */
vl_status vl_hyrax_commit(const void* M, int32_t dtype, uint32_t R, uint32_t m, uint64_t ld, const void* table,
                          uint32_t table_m, uint32_t windows, uint32_t split, void* commits, void* workspace,
                          uint64_t workspace_bytes, void* stream);

/* Host: the generators G_0 .. G_{m-1} as 96-byte points into out (host,
 * 96 m bytes).  Computed on the host (and kept for later calls), so a
 * verifier does not trust the prover's table. */
vl_status vl_hyrax_generators(uint32_t m, uint8_t* out);

/* Host verifier of an opening.  commits: R points (host, 96 R bytes); x:
 * ceil(log2 R) and y: ceil(log2 m) canonical elements (NULL when there are
 * none); w: m canonical elements.  Checks that every commitment is a
 * canonical point of the curve in the order-p subgroup (or 96 zero bytes)
 * and that sum_j w_j G_j = sum_i eq(x, i) C_i (both multi-scalar products
 * by Pippenger's bucket method), then writes M~(x, y) = sum_j w_j eq(y, j)
 * to value (optional).  Returns VL_OK or VL_ERR_REJECT (message in
 * vl_last_error); VL_ERR_INVALID_ARG / VL_ERR_SHAPE for bad arguments. */
vl_status vl_hyrax_verify_open(const uint8_t* commits, uint32_t R, uint32_t m, const vl_fr* x, const vl_fr* y,
                               const vl_fr* w, vl_fr* value);

/* Message for the last non-OK status on this thread. */
const char* vl_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* VERILORA_H */
