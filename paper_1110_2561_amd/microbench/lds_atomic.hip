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
// and lane-private with part of the wave masked off (does the atomic unit
// spend its cycles per instruction or per active lane?):
//   even-lanes     only even lanes issue the atomic
//   low-half       only lanes 0-31
//   low-quarter    only lanes 0-15
//   rand-7/8       each (lane, address) pair active with probability 7/8
// Rates are reported per active lane and per wave instruction.  The
// measured rates include each block's set-up and final reduction, so they
// are lower bounds of the unit's steady-state rate.
// VALU: eight independent chains of add / xor / popcount-accumulate.  The
// compiler may fuse source operations (e.g. into v_bcnt_u32_b32 with an
// addend), so the printed "source ops" rate can exceed the issue rate; the
// issue rate is SQ_INSTS_VALU x 64 lanes over the same time (rocprofv3).
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
__global__ __launch_bounds__(1024) void k_lds(int iters, unsigned long long *out) {
  __shared__ uint32_t h[kWords];
  for (int i = threadIdx.x; i < kWords; i += blockDim.x) h[i] = 0;
  __syncthreads();
  const int lane = threadIdx.x & 63;
  const uint32_t seed = mix(blockIdx.x * 1024 + threadIdx.x);
  uint32_t a[kAddrs];
  uint32_t on = 0;   // bit i: this lane issues atomic i (masked patterns)
#pragma unroll
  for (int i = 0; i < kAddrs; ++i) {
    const uint32_t r = mix(seed + i * 7919);
    if (PAT == 0 || PAT >= 5) a[i] = uint32_t(i * 64 + lane);
    else if (PAT == 1) a[i] = (r % 1400) * 16 + (lane & 15);
    else if (PAT == 2) a[i] = (r % 1200) * 32 + (lane & 31);
    else if (PAT == 3) a[i] = r % 1400;
    else a[i] = 5;
    bool act = true;
    if (PAT == 5) act = (lane & 1) == 0;
    else if (PAT == 6) act = lane < 32;
    else if (PAT == 7) act = lane < 16;
    else if (PAT == 8) act = (r >> 29) != 0;
    on |= uint32_t(act) << i;
  }
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int i = 0; i < kAddrs; ++i) {
      if (PAT < 5 || ((on >> i) & 1u))
        __hip_atomic_fetch_add(&h[a[i]], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    }
  }
  __syncthreads();
  unsigned long long s = 0;
  for (int i = threadIdx.x; i < kWords; i += blockDim.x) s += h[i];
  atomicAdd(out, s);
}

// Integer VALU chains.  OP 0: add / xor / popcount-accumulate (one of each
// per step); OP 1: v_add_u32 only; OP 2: v_xor_b32 only; OP 3:
// v_bcnt_u32_b32 only.  CH independent chains per lane.
template <int OP, int CH>
__global__ __launch_bounds__(1024) void k_valu(int iters, uint32_t *out) {
  uint32_t x[CH];
#pragma unroll
  for (int i = 0; i < CH; ++i) x[i] = threadIdx.x * (i + 3) + blockIdx.x;
  const uint32_t k1 = iters * 3 + 1, k2 = iters ^ 0x55;
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int i = 0; i < CH; ++i) {
      if (OP == 0) {
        x[i] = x[i] + k1;
        x[i] = x[i] ^ k2;
        x[i] = __builtin_popcount(x[i]) + x[i];
      } else if (OP == 1) {
        x[i] = x[i] + k1;
      } else if (OP == 2) {
        x[i] = x[i] ^ k2;
      } else {
        x[i] = __builtin_popcount(x[i]) + x[i];
      }
    }
  }
  uint32_t s = 0;
#pragma unroll
  for (int i = 0; i < CH; ++i) s += x[i];
  if (s == 0x12345678u) out[0] = s;
}

template <int OP, int CH>
static int run_valu(const char *name, int blocks, int iters, int ops_per_step, double clk_hz, int cus) {
  uint32_t *d;
  CHECK(hipMalloc(&d, 4));
  hipEvent_t e0, e1;
  CHECK(hipEventCreate(&e0));
  CHECK(hipEventCreate(&e1));
  hipLaunchKernelGGL((k_valu<OP, CH>), dim3(blocks), dim3(1024), 0, 0, 16, d);
  CHECK(hipGetLastError());
  CHECK(hipDeviceSynchronize());
  CHECK(hipEventRecord(e0));
  hipLaunchKernelGGL((k_valu<OP, CH>), dim3(blocks), dim3(1024), 0, 0, iters, d);
  CHECK(hipGetLastError());
  CHECK(hipEventRecord(e1));
  CHECK(hipEventSynchronize(e1));
  float ms;
  CHECK(hipEventElapsedTime(&ms, e0, e1));
  const double ops = double(blocks) * 1024 * iters * CH * ops_per_step;
  std::printf("%-16s %8.3f ms  %7.3f T int32 source ops/s  %6.2f source ops/clk/CU (issue rate: SQ_INSTS_VALU)\n",
              name, ms, ops / ms / 1e9, ops / (ms * 1e-3) / cus / clk_hz);
  CHECK(hipFree(d));
  return 0;
}

// active_frac: the fraction of (lane, address) slots that issue an atomic
// (0 for rand-7/8, whose count only the kernel knows).
template <int PAT>
static int run_lds(const char *name, int blocks, int iters, double clk_hz, int cus, double active_frac) {
  unsigned long long *d;
  CHECK(hipMalloc(&d, 8));
  CHECK(hipMemset(d, 0, 8));
  hipEvent_t e0, e1;
  CHECK(hipEventCreate(&e0));
  CHECK(hipEventCreate(&e1));
  hipLaunchKernelGGL(k_lds<PAT>, dim3(blocks), dim3(1024), 0, 0, 4, d);
  CHECK(hipGetLastError());
  CHECK(hipDeviceSynchronize());
  CHECK(hipMemset(d, 0, 8));
  CHECK(hipEventRecord(e0));
  hipLaunchKernelGGL(k_lds<PAT>, dim3(blocks), dim3(1024), 0, 0, iters, d);
  CHECK(hipGetLastError());
  CHECK(hipEventRecord(e1));
  CHECK(hipEventSynchronize(e1));
  float ms;
  CHECK(hipEventElapsedTime(&ms, e0, e1));
  unsigned long long total;
  CHECK(hipMemcpy(&total, d, 8, hipMemcpyDeviceToHost));
  const double slots = double(blocks) * 1024 * iters * kAddrs;   // lane slots (64 per wave instruction)
  const unsigned long long expect = (unsigned long long)(slots * active_frac);
  const bool ok = active_frac > 0 ? total == expect : total > 0;
  const double ops = double(total);
  const double instr_rate = slots / 64 / (ms * 1e-3) / cus / clk_hz;   // wave instructions / clk / CU
  std::printf("%-16s %8.3f ms  %7.3f T increments/s  %6.2f active lanes/clk/CU  %6.3f wave instr/clk/CU  %s\n",
              name, ms, ops / ms / 1e9, ops / (ms * 1e-3) / cus / clk_hz, instr_rate,
              ok ? (active_frac > 0 ? "count ok" : "count from kernel") : "COUNT MISMATCH");
  CHECK(hipFree(d));
  return ok ? 0 : 1;
}

int main() {
  hipDeviceProp_t p;
  CHECK(hipGetDeviceProperties(&p, 0));
  const double clk = 2.4e9;  // MI355X peak engine clock
  std::printf("device %s, %d CUs, LDS per block %zu bytes, rates at %.1f GHz\n", p.gcnArchName,
              p.multiProcessorCount, p.sharedMemPerBlock, clk / 1e9);
  // one 160 KB block per CU at a time; 4 blocks per CU in sequence
  const int B = p.multiProcessorCount * 4;
  const int C = p.multiProcessorCount;
  int bad = 0;
  bad |= run_lds<0>("lane-private", B, 2048, clk, C, 1.0);
  bad |= run_lds<0>("lane-private-x8", C, 8 * 2048, clk, C, 1.0);
  bad |= run_lds<1>("copies16-rand", B, 2048, clk, C, 1.0);
  bad |= run_lds<2>("copies32-rand", B, 2048, clk, C, 1.0);
  bad |= run_lds<3>("shared-rand", B, 1024, clk, C, 1.0);
  bad |= run_lds<4>("same-word", B, 64, clk, C, 1.0);
  bad |= run_lds<5>("even-lanes", B, 2048, clk, C, 0.5);
  bad |= run_lds<6>("low-half", B, 2048, clk, C, 0.5);
  bad |= run_lds<7>("low-quarter", B, 2048, clk, C, 0.25);
  bad |= run_lds<8>("rand-7/8", B, 2048, clk, C, 0.0);
  const int vb = C * 8, vi = 1 << 14;
  bad |= run_valu<0, 8>("valu-mix-8", vb, vi, 3, clk, C);
  bad |= run_valu<1, 16>("valu-add-16", vb, vi, 1, clk, C);
  bad |= run_valu<2, 16>("valu-xor-16", vb, vi, 1, clk, C);
  bad |= run_valu<3, 16>("valu-bcnt-16", vb, vi, 1, clk, C);
  bad |= run_valu<1, 32>("valu-add-32", vb, vi / 2, 1, clk, C);
  return bad;
}
