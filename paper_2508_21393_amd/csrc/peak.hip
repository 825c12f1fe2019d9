// Microbenchmarks (libvlpeak.so) used by bench.py to state the ceilings of
// the integer contraction:
//  - VALU issue rate: per-lane throughput of v_dot2c_i32_i16, v_mad_u64_u32,
//    v_mad_i64_i32, v_mul_lo_u32, v_mul_hi_u32 and v_add_u32, each as 8
//    independent dependency chains per lane so that issue rate, not latency,
//    is measured;
//  - HBM streaming read: 16-byte loads over a buffer much larger than the
//    caches, four loads in flight per lane, as plain and as nontemporal
//    loads (the better of the two is the ceiling).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

namespace {

constexpr int kChains = 8;

template <int OP>
__global__ void __launch_bounds__(256) rate_kernel(uint32_t* out, uint32_t iters, uint32_t seed) {
  uint32_t a = seed ^ threadIdx.x, b = seed + blockIdx.x * 7u;
  uint32_t acc[kChains];
  uint64_t acc64[kChains];
#pragma unroll
  for (int c = 0; c < kChains; ++c) {
    acc[c] = a + c;
    acc64[c] = (uint64_t)(b + c);
  }
  for (uint32_t i = 0; i < iters; ++i) {
#pragma unroll
    for (int c = 0; c < kChains; ++c) {
      if constexpr (OP == 0) {
        asm volatile("v_dot2c_i32_i16 %0, %1, %2" : "+v"(acc[c]) : "v"(a), "v"(b));
      } else if constexpr (OP == 1) {
        uint64_t sd;
        asm volatile("v_mad_u64_u32 %0, %1, %2, %3, %0" : "+v"(acc64[c]), "=s"(sd) : "v"(a), "v"(b));
      } else if constexpr (OP == 5) {
        uint64_t sd;
        asm volatile("v_mad_i64_i32 %0, %1, %2, %3, %0" : "+v"(acc64[c]), "=s"(sd) : "v"(a), "v"(b));
      } else if constexpr (OP == 2) {
        asm volatile("v_mul_lo_u32 %0, %0, %1" : "+v"(acc[c]) : "v"(b));
      } else if constexpr (OP == 3) {
        asm volatile("v_mul_hi_u32 %0, %0, %1" : "+v"(acc[c]) : "v"(b));
      } else {
        asm volatile("v_add_u32 %0, %0, %1" : "+v"(acc[c]) : "v"(b));
      }
    }
  }
  uint32_t s = 0;
#pragma unroll
  for (int c = 0; c < kChains; ++c) s ^= acc[c] ^ (uint32_t)acc64[c] ^ (uint32_t)(acc64[c] >> 32);
  out[blockIdx.x * blockDim.x + threadIdx.x] = s;
}

template <int OP>
double run(uint32_t blocks, uint32_t iters) {
  uint32_t* out = nullptr;
  if (hipMalloc(&out, (size_t)blocks * 256 * 4) != hipSuccess) return -1.0;
  hipEvent_t e0, e1;
  (void)hipEventCreate(&e0);
  (void)hipEventCreate(&e1);
  hipLaunchKernelGGL(rate_kernel<OP>, dim3(blocks), dim3(256), 0, 0, out, iters / 8, 1u);  // warm up
  (void)hipEventRecord(e0, 0);
  hipLaunchKernelGGL(rate_kernel<OP>, dim3(blocks), dim3(256), 0, 0, out, iters, 1u);
  (void)hipEventRecord(e1, 0);
  (void)hipEventSynchronize(e1);
  float ms = 0.f;
  (void)hipEventElapsedTime(&ms, e0, e1);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  (void)hipFree(out);
  const double ops = (double)blocks * 256.0 * iters * kChains;
  return ms > 0 ? ops / (ms * 1e-3) : -1.0;
}

typedef uint32_t v4u __attribute__((ext_vector_type(4)));

template <bool NT>
__device__ __forceinline__ v4u ld16(const v4u* p) {
  if constexpr (NT) return __builtin_nontemporal_load(p);
  else return *p;
}

template <bool NT>
__global__ void __launch_bounds__(256) read_kernel(const v4u* __restrict__ p, uint64_t n,
                                                   uint32_t* __restrict__ out) {
  const uint64_t tid = (uint64_t)blockIdx.x * 256u + threadIdx.x, stride = (uint64_t)gridDim.x * 256u;
  uint32_t x = 0;
  uint64_t i = tid;
  for (; i + 3 * stride < n; i += 4 * stride) {
    const v4u a = ld16<NT>(p + i), b = ld16<NT>(p + i + stride), c = ld16<NT>(p + i + 2 * stride),
              d = ld16<NT>(p + i + 3 * stride);
    const v4u e = a ^ b ^ c ^ d;
    x ^= e.x ^ e.y ^ e.z ^ e.w;
  }
  for (; i < n; i += stride) {
    const v4u a = ld16<NT>(p + i);
    x ^= a.x ^ a.y ^ a.z ^ a.w;
  }
  out[tid] = x;   // keeps the loads live
}

double read_rate(uint64_t bytes) {
  const uint64_t n = bytes / 16;
  const uint32_t blocks = 256 * 8;
  v4u* buf = nullptr;
  uint32_t* out = nullptr;
  if (n == 0 || hipMalloc(&buf, n * 16) != hipSuccess) return -1.0;
  if (hipMalloc(&out, (size_t)blocks * 256 * 4) != hipSuccess) {
    (void)hipFree(buf);
    return -1.0;
  }
  (void)hipMemset(buf, 1, n * 16);
  hipEvent_t e0, e1;
  (void)hipEventCreate(&e0);
  (void)hipEventCreate(&e1);
  double best = -1.0;
  for (int rep = 0; rep < 8; ++rep) {   // plain and nontemporal in turn; the first two warm up
    (void)hipEventRecord(e0, 0);
    if (rep & 1) hipLaunchKernelGGL(read_kernel<true>, dim3(blocks), dim3(256), 0, 0, buf, n, out);
    else hipLaunchKernelGGL(read_kernel<false>, dim3(blocks), dim3(256), 0, 0, buf, n, out);
    (void)hipEventRecord(e1, 0);
    (void)hipEventSynchronize(e1);
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, e0, e1);
    if (rep > 1 && ms > 0) best = std::max(best, (double)n * 16 / (ms * 1e-3) / 1e9);
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  (void)hipFree(out);
  (void)hipFree(buf);
  return best;
}

}  // namespace

// Streaming read of a fresh device buffer of `bytes` bytes (best of three
// timed runs each of plain and nontemporal loads): GB/s, or a negative value
// on error.
extern "C" double vlpeak_hbm_read_GBps(uint64_t bytes) { return read_rate(bytes); }

// which: 0 dot2_i32_i16, 1 mad_u64_u32, 2 mul_lo_u32, 3 mul_hi_u32, 4 add_u32,
// 5 mad_i64_i32.
// Returns lane-operations per second, or a negative value on error.
extern "C" double vlpeak_lane_ops_per_s(int which, uint32_t blocks, uint32_t iters) {
  switch (which) {
    case 0: return run<0>(blocks, iters);
    case 1: return run<1>(blocks, iters);
    case 2: return run<2>(blocks, iters);
    case 3: return run<3>(blocks, iters);
    case 4: return run<4>(blocks, iters);
    case 5: return run<5>(blocks, iters);
    default: return -1.0;
  }
}
