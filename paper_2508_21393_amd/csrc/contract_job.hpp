// Descriptors of the integer contractions (the matrix partial evaluations of
// the hot path) and their finish pass, shared by contract.hip and the host
// planning.  Kept apart from the other job descriptors so that the
// contraction kernels' source fingerprint changes only with their own code.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/verilora.h"

namespace vl {

constexpr int kWave = 64;
constexpr int kContractBlock = 256;            // 4 waves, one task per wave
constexpr uint32_t kChunkAlign = 32;           // contraction chunks start at multiples of 32
constexpr uint32_t kMaxChunk = 1u << 16;       // int64 accumulators of int16 digits hold 2^16 entries
constexpr uint32_t kWideSpill = 256;           // ... and of 24-bit digits 256 entries (products < 2^54)

// One integer contraction: for each output n < n_out and each chunk of the
// contraction index m, sum_m eq[m] * M(m, n), where M(m, n) is the stored
// matrix at [m * ld + n] (rows kernel) or [n * ld + m] (cols kernel).
struct ContractJob {
  const void* M;
  uint64_t ld;
  uint32_t n_out;             // outputs (stored columns for rows, stored rows for cols)
  uint32_t len;               // contraction length
  uint32_t chunk;             // chunk length, multiple of kChunkAlign
  uint32_t n_chunks;
  uint32_t out_waves;         // ceil(n_out / 64)
  uint32_t task_begin;        // prefix sum of tasks (out_waves * n_chunks) within a launch
  const uint32_t* pack;       // eq pack table of the contraction index
  uint32_t* dst;              // n_chunks == 1: final SoL vector (8 planes, stride dst_ld);
                              // else raw chunk partials in 64-output tiles (partial_word)
  uint64_t dst_ld;
  int32_t* err;               // set to 1 if an entry cannot be represented (int32/int64)
};

// A split contraction's chunks leave their exact sums unreduced: kLimbs
// 32-bit two's-complement limbs per output and chunk.  The finish kernel
// adds them up and reduces once per output.  Layout: 64-output tiles, each
// holding every chunk's limbs of its outputs contiguously, so that the
// finish pass reads one contiguous region per 64 outputs.
constexpr int kLimbs = 12;
__host__ __device__ constexpr uint64_t partial_word(uint32_t n, uint32_t chunk, int q, uint32_t n_chunks) {
  return (uint64_t)(n >> 6) * n_chunks * (kLimbs * 64) + ((uint64_t)chunk * kLimbs + q) * 64 + (n & 63u);
}

// Sum the raw chunk partials into the final SoL vector and zero its padding.
struct FinishJob {
  const uint32_t* part;       // raw chunk partials (null if the contraction wrote out)
  uint32_t n_chunks;
  uint32_t n_valid;           // outputs written by the contraction
  uint32_t n_total;           // padded length (power of two)
  uint32_t block_begin;       // prefix sum of blocks within a launch
  uint32_t split;             // 0: 256 outputs per block, one thread each; 1: 64
                              // outputs per block, the 4 waves split the chunks
  uint32_t pad_;
  uint32_t* out;
  uint64_t out_ld;
};
constexpr uint32_t kFinishSplitChunks = 16;   // split jobs with at least this many chunks

// contraction kernel variants (index = kind)
// (entry type, digits x digit bits, orientation, outputs per lane)
enum ContractKind {
  CK_I16_ROWS = 0,       // int16, 1 x 16, rows, 1
  CK_I16_ROWS4 = 1,      // int16, 1 x 16, rows, 4 (element loads)
  CK_I16_ROWS4_VEC = 2,  // int16, 1 x 16, rows, 4 (8-byte loads)
  CK_I16_COLS = 3,       // int16, cols, element loads
  CK_I16_COLS_VEC = 4,   // int16, cols, 16-byte row loads, 1 row per lane
  CK_I16_COLS2_VEC = 5,  // int16, cols, 16-byte row loads, 2 rows per lane
  // wide entries (2 or 3 digits x 24 bits); the vector rows kinds read 16
  // bytes (4 int32 or 2 int64 columns) per lane and row
  CK_I32_ROWS = 6, CK_I32_ROWS4_VEC = 7, CK_I32_COLS = 8, CK_I32_COLS_VEC = 9,           // int32
  CK_I64S_ROWS = 10, CK_I64S_ROWS2_VEC = 11, CK_I64S_COLS = 12, CK_I64S_COLS_VEC = 13,   // int64, |x| < 2^47
  CK_I64S_COLS2_VEC = 14,                                                                // the same, 2 rows per lane
  CK_I64_ROWS = 15, CK_I64_ROWS2_VEC = 16, CK_I64_COLS = 17, CK_I64_COLS_VEC = 18,       // int64, 3 digits
  CK_COUNT = 19
};
static_assert(VL_STAGE_CONTRACT + CK_COUNT == VL_STAGE_FINISH, "one stage per contraction kind");

}  // namespace vl
