// Microbenchmark of the two ceilings the enumeration kernel can hit on one
// gfx950 CU: LDS atomic increments (ds_add_u32, non-returning) and 32-bit
// integer VALU operations.  Used to measure the roofline peaks that the
// benchmark reports against.
//
// LDS patterns (1024 threads per block, one 160 KB block per CU, every lane
// keeps 16 precomputed word addresses and increments them in turn):
//   lane-private   word = i * 64 + lane               (no bank conflict)
//   copies16-rand  word = bin * 16 + (lane mod 16)    (random bins)
//   copies32-rand  word = bin * 32 + (lane mod 32)    (random bins)
//   shared-rand    word = bin                         (one shared table, random bins)
//   same-word      every lane of a wave hits one word
// VALU: eight independent chains of v_add_u32 / v_xor_b32 / v_bcnt_u32_b32.
//
// Build: part of `python -m paper_1110_2561_amd.build`; run the produced
// executable paper_1110_2561_amd/microbench/lds_atomic.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>

#define CHECK(x)                                                                     \
  do {                                                                               \
    hipError_t e_ = (x);                                                             \
    if (e_ != hipSuccess) {                                                          \
      std::printf("HIP error %s at line %d\n", hipGetErrorString(e_), __LINE__);     \
      return 1;                                                                      \
    }                                                                                \
  } while (0)

constexpr int kWords = 40960;  // 160 KB
constexpr int kAddrs = 16;

__device__ __forceinline__ uint32_t mix(uint32_t x) {
  x ^= x >> 16; x *= 0x7feb352dU; x ^= x >> 15; x *= 0x846ca68bU; x ^= x >> 16;
  return x;
}

template <int PAT>
__global__ __launch_bounds__(1024) void k_lds(int iters, uint32_t *out) {
  __shared__ uint32_t h[kWords];
  for (int i = threadIdx.x; i < kWords; i += blockDim.x) h[i] = 0;
  __syncthreads();
  const int lane = threadIdx.x & 63;
  const uint32_t seed = mix(blockIdx.x * 1024 + threadIdx.x);
  uint32_t a[kAddrs];
#pragma unroll
  for (int i = 0; i < kAddrs; ++i) {
    const uint32_t r = mix(seed + i * 7919);
    if (PAT == 0) a[i] = uint32_t(i * 64 + lane);
    else if (PAT == 1) a[i] = (r % 1400) * 16 + (lane & 15);
    else if (PAT == 2) a[i] = (r % 1200) * 32 + (lane & 31);
    else if (PAT == 3) a[i] = r % 1400;
    else a[i] = 5;
  }
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int i = 0; i < kAddrs; ++i)
      __hip_atomic_fetch_add(&h[a[i]], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
  }
  __syncthreads();
  uint32_t s = 0;
  for (int i = threadIdx.x; i < kWords; i += blockDim.x) s += h[i];
  atomicAdd(out, s);
}

__global__ __launch_bounds__(1024) void k_valu(int iters, uint32_t *out) {
  uint32_t x[8];
#pragma unroll
  for (int i = 0; i < 8; ++i) x[i] = threadIdx.x * (i + 3) + blockIdx.x;
  const uint32_t k1 = iters * 3 + 1, k2 = iters ^ 0x55;
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      x[i] = x[i] + k1;
      x[i] = x[i] ^ k2;
      x[i] = __builtin_popcount(x[i]) + x[i];
    }
  }
  uint32_t s = 0;
#pragma unroll
  for (int i = 0; i < 8; ++i) s += x[i];
  if (s == 0x12345678u) out[0] = s;
}

template <int PAT>
static int run_lds(const char *name, int blocks, int iters, double clk_hz, int cus) {
  uint32_t *d;
  CHECK(hipMalloc(&d, 4));
  CHECK(hipMemset(d, 0, 4));
  hipEvent_t e0, e1;
  CHECK(hipEventCreate(&e0));
  CHECK(hipEventCreate(&e1));
  hipLaunchKernelGGL(k_lds<PAT>, dim3(blocks), dim3(1024), 0, 0, 4, d);
  CHECK(hipGetLastError());
  CHECK(hipDeviceSynchronize());
  CHECK(hipMemset(d, 0, 4));
  CHECK(hipEventRecord(e0));
  hipLaunchKernelGGL(k_lds<PAT>, dim3(blocks), dim3(1024), 0, 0, iters, d);
  CHECK(hipGetLastError());
  CHECK(hipEventRecord(e1));
  CHECK(hipEventSynchronize(e1));
  float ms;
  CHECK(hipEventElapsedTime(&ms, e0, e1));
  uint32_t total;
  CHECK(hipMemcpy(&total, d, 4, hipMemcpyDeviceToHost));
  const double ops = double(blocks) * 1024 * iters * kAddrs;
  const uint32_t expect = uint32_t(uint64_t(ops));
  std::printf("%-16s %8.3f ms  %7.3f T increments/s  %6.2f lanes/clk/CU  %s\n", name, ms, ops / ms / 1e9,
              ops / (ms * 1e-3) / cus / clk_hz, total == expect ? "count ok" : "COUNT MISMATCH");
  CHECK(hipFree(d));
  return total == expect ? 0 : 1;
}

int main() {
  hipDeviceProp_t p;
  CHECK(hipGetDeviceProperties(&p, 0));
  const double clk = 2.4e9;  // MI355X peak engine clock
  std::printf("device %s, %d CUs, LDS per block %zu bytes, rates at %.1f GHz\n", p.gcnArchName,
              p.multiProcessorCount, p.sharedMemPerBlock, clk / 1e9);
  const int B = p.multiProcessorCount * 4;
  int bad = 0;
  bad |= run_lds<0>("lane-private", B, 2048, clk, p.multiProcessorCount);
  bad |= run_lds<1>("copies16-rand", B, 2048, clk, p.multiProcessorCount);
  bad |= run_lds<2>("copies32-rand", B, 2048, clk, p.multiProcessorCount);
  bad |= run_lds<3>("shared-rand", B, 1024, clk, p.multiProcessorCount);
  bad |= run_lds<4>("same-word", B, 64, clk, p.multiProcessorCount);
  uint32_t *d;
  CHECK(hipMalloc(&d, 4));
  hipEvent_t e0, e1;
  CHECK(hipEventCreate(&e0));
  CHECK(hipEventCreate(&e1));
  const int blocks = p.multiProcessorCount * 8, iters = 1 << 14;
  hipLaunchKernelGGL(k_valu, dim3(blocks), dim3(1024), 0, 0, 16, d);
  CHECK(hipDeviceSynchronize());
  CHECK(hipEventRecord(e0));
  hipLaunchKernelGGL(k_valu, dim3(blocks), dim3(1024), 0, 0, iters, d);
  CHECK(hipEventRecord(e1));
  CHECK(hipEventSynchronize(e1));
  float ms;
  CHECK(hipEventElapsedTime(&ms, e0, e1));
  const double ops = double(blocks) * 1024 * iters * 8 * 3;
  std::printf("%-16s %8.3f ms  %7.3f T int32 lane-ops/s  %6.2f lanes/clk/CU\n", "valu-int32", ms, ops / ms / 1e9,
              ops / (ms * 1e-3) / p.multiProcessorCount / clk);
  return bad;
}
