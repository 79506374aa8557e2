// Exhaustive enumeration of the 2^N configurations of a finite Ising system
// into the integer degeneracy table g(E, M) on gfx950.
//
// What is computed follows Peretyatko et al., Section 2 (Eq. (1): each bond
// counted once, E = -sum_b J_b s_i s_j; M the spin excess; g counts the
// configurations per (E, M)) and Section 3 (configurations as bit vectors,
// enumerated exhaustively, the space split into independent ranges whose
// partial tables are summed at the end, Section 3d).
//
// How it runs on CDNA4:
//   * One lane owns one chunk: the 2^k configurations that share a prefix
//     (plan bits k..N-1).  The lane keeps the spin word in registers and walks
//     the k inner bits in reflected Gray-code order, so consecutive
//     configurations differ by one flipped spin and (E, n_up) is updated
//     incrementally.  The inner state is the same for every lane of a wave,
//     so the flipped bit, its direction and its neighbour masks are
//     wave-uniform (scalar registers).
//   * The low j inner bits ("tile") are spins with no coupling among them.
//     While only tile bits flip, the local field of each tile spin is fixed,
//     so the histogram-address change of every tile flip is a per-lane
//     constant D_i: one integer add per configuration.  When a higher inner
//     bit flips (once per 2^j configurations) its own delta comes from a
//     popcount of the spin word against its neighbour masks, and the D_i of
//     tile spins coupled to it move by a plan constant.
//   * Every configuration adds 1 to its (E, n_up) bin in an LDS histogram
//     with R copies per block (lane_copy in walk.h).  Copy-major words
//     (bin * R + copy), an even bin-row stride and the planner's placement of
//     the lane-distinguishing spins keep the 32 lanes one LDS cycle serves in
//     distinct banks.  Counters are u32; the
//     block flushes them (sum over copies, 64-bit global atomics into the
//     dense uint64 table) before any can reach 2^32, and at exit.
//   * No HBM traffic beyond the final flush: the kernel is bound by the LDS
//     atomic rate (one ds_add_u32 per configuration).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <string>

#include "internal.h"
#include "walk.h"

namespace ising {

#define HIP_TRY(expr)                                                                        \
  do {                                                                                       \
    hipError_t e_ = (expr);                                                                  \
    if (e_ != hipSuccess) return fail(ISING_EHIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

// Task t of this block covers chunks (task_lo + t) * blockDim.x + [0, blockDim.x),
// one per thread (thread -> offset by the plan's lane_chunk permutation);
// lanes whose chunk lies outside [chunk_lo, chunk_hi) idle.  With 16 copies
// (identity permutation) lanes l and l + 16 of a half-wave share LDS copy
// l mod 16; their chunks differ in one prefix spin, so their n_up differ by
// one, and with an even row stride W their words fall in different banks
// (bank = 16 * (bin mod 2) + copy on the 32-bank LDS).  With 8 copies the
// permutation gives the four lanes sharing a copy four n_up mod 4 and the
// stride is a multiple of 4 (bank = 8 * (bin mod 4) + copy).  All threads
// of a block run the same number of tasks, so the barriers around periodic
// flushes are uniform.
template <int TJ, int NC>
__global__ __launch_bounds__(1024) void k_enumerate(const DevPlan *__restrict__ P, uint64_t chunk_lo,
                                                    uint64_t chunk_hi, uint64_t task_lo, uint64_t n_tasks,
                                                    uint32_t flush_every, unsigned long long *__restrict__ g) {
  // Static (not dynamic) LDS: its base address is a compile-time constant, so
  // each histogram update is a single ds_add_u32 on the running address.
  __shared__ __align__(16) uint32_t h32[kHistBytes / 4];
  char *hist = reinterpret_cast<char *>(h32);
  const int words = P->n_ec * P->W * P->R;
  for (int w = threadIdx.x; w < words; w += blockDim.x) h32[w] = 0;
  __syncthreads();
  const uint32_t lane = threadIdx.x & (kWave - 1);
  const uint32_t rep = lane_copy(lane, P->R);
  SiteTable<NC> st;
  st.load(P, int(lane));
  const uint32_t offset = P->lane_chunk[threadIdx.x];
  uint32_t since = 0;
  for (uint64_t t = blockIdx.x; t < n_tasks; t += gridDim.x) {
    const uint64_t chunk = (task_lo + t) * blockDim.x + offset;
    if (chunk >= chunk_lo && chunk < chunk_hi) walk_chunk<TJ, NC>(st, chunk, rep, hist);
    if (++since == flush_every) {
      __syncthreads();
      flush_hist(P, h32, g);
      __syncthreads();
      since = 0;
    }
  }
  __syncthreads();
  flush_hist(P, h32, g);
}

// g(E, M) = g(E, -M) for every coupling set (H at h = 0 is even in the spins),
// and the configurations with the top plan bit down are the spin flips of
// those with it up.  So from h_up, the table of the upper half of the chunk
// range, g[e][nu] = h_up[e][nu] + h_up[e][N - nu]; done in place, one thread
// per (e, nu <= N - nu) pair.
__global__ void k_mirror_u64(unsigned long long *g, int n_e, int n_m) {
  const int half = (n_m + 1) / 2;   // nu in [0, half) pairs with n_m - 1 - nu
  const size_t cells = size_t(n_e) * half;
  for (size_t i = blockIdx.x * size_t(blockDim.x) + threadIdx.x; i < cells; i += size_t(gridDim.x) * blockDim.x) {
    const size_t e = i / half;
    const int nu = int(i - e * half), mu = n_m - 1 - nu;
    unsigned long long *row = g + e * n_m;
    const unsigned long long s = row[nu] + row[mu];
    row[nu] = s;
    row[mu] = s;
  }
}

__global__ void k_fill_u64(unsigned long long *p, size_t n) {
  for (size_t i = blockIdx.x * size_t(blockDim.x) + threadIdx.x; i < n; i += size_t(gridDim.x) * blockDim.x)
    p[i] = 0ull;
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------

const void *plan_device_constants(ising_plan *p, int device, ising_status *st) {
  *st = ISING_OK;
  if (device < 0 || device >= kMaxDevices) {
    *st = fail(ISING_EUNSUPPORTED, "device index out of range");
    return nullptr;
  }
  std::lock_guard<std::mutex> lk(p->mu);
  if (!p->dev_copy[device]) {
    void *ptr = nullptr;
    hipError_t e = hipMalloc(&ptr, sizeof(DevPlan));
    if (e != hipSuccess) {
      *st = fail(ISING_EHIP, std::string("hipMalloc(plan constants): ") + hipGetErrorString(e));
      return nullptr;
    }
    e = hipMemcpy(ptr, &p->dev, sizeof(DevPlan), hipMemcpyHostToDevice);
    if (e != hipSuccess) {
      (void)hipFree(ptr);
      *st = fail(ISING_EHIP, std::string("hipMemcpy(plan constants): ") + hipGetErrorString(e));
      return nullptr;
    }
    p->dev_copy[device] = ptr;
  }
  return p->dev_copy[device];
}

template <int TJ, int NC>
static ising_status launch_tj(const DevPlan *dP, uint64_t lo, uint64_t hi, uint64_t task_lo, uint64_t n_tasks,
                              int grid, int block, uint32_t flush_every, size_t smem,
                              unsigned long long *g, hipStream_t s) {
  (void)smem;
  hipLaunchKernelGGL((k_enumerate<TJ, NC>), dim3(grid), dim3(block), 0, s, dP, lo, hi, task_lo, n_tasks,
                     flush_every, g);
  HIP_TRY(hipGetLastError());
  return ISING_OK;
}

static ising_status enumerate_chunks(const ising_plan *pc, uint64_t first, uint64_t count, uint64_t *g_dev,
                                     hipStream_t stream) {
  ising_plan *p = const_cast<ising_plan *>(pc);  // only the lazy device copy is written
  if (count == 0) return ISING_OK;
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  ising_status st;
  const DevPlan *dP = static_cast<const DevPlan *>(plan_device_constants(p, dev, &st));
  if (!dP) return st;
  int cus = 0;
  HIP_TRY(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
  const DevPlan &d = p->dev;
  const int block = kWave * p->waves_per_block;
  const uint64_t lo = first, hi = first + count;
  const uint64_t task_lo = lo / uint64_t(block);
  const uint64_t task_hi = (hi + uint64_t(block) - 1) / uint64_t(block);
  const uint64_t n_tasks = task_hi - task_lo;
  uint64_t grid = uint64_t(cus) * uint64_t(p->blocks_per_cu);
  if (p->max_blocks > 0 && uint64_t(p->max_blocks) < grid) grid = uint64_t(p->max_blocks);
  if (n_tasks < grid) grid = n_tasks;
  const uint64_t per_task = (uint64_t(block) / uint64_t(d.R)) << d.inner;  // max adds per counter per task
  uint64_t fe = 0xFFFFFFFFull / per_task;
  if (fe < 1) return fail(ISING_EUNSUPPORTED, "chunk too large for 32-bit LDS counters");
  if (fe > 0x7FFFFFFFull) fe = 0x7FFFFFFFull;
  const size_t smem = size_t(d.n_ec) * d.W * d.R * 4;
  unsigned long long *g = reinterpret_cast<unsigned long long *>(g_dev);
#define ISING_NC(TJ)                                                                                  \
  switch (d.n_classes) {                                                                              \
    case 1: return launch_tj<TJ, 1>(dP, lo, hi, task_lo, n_tasks, int(grid), block, uint32_t(fe), smem, g, stream); \
    case 2: return launch_tj<TJ, 2>(dP, lo, hi, task_lo, n_tasks, int(grid), block, uint32_t(fe), smem, g, stream); \
    case 4: return launch_tj<TJ, 4>(dP, lo, hi, task_lo, n_tasks, int(grid), block, uint32_t(fe), smem, g, stream); \
    case 8: return launch_tj<TJ, 8>(dP, lo, hi, task_lo, n_tasks, int(grid), block, uint32_t(fe), smem, g, stream); \
  }                                                                                                   \
  break;
  switch (d.tile) {
    case 1: ISING_NC(1)
    case 2: ISING_NC(2)
    case 3: ISING_NC(3)
    case 4: ISING_NC(4)
    case 5: ISING_NC(5)
    case 6: ISING_NC(6)
    case 7: ISING_NC(7)
    case 8: ISING_NC(8)
  }
#undef ISING_NC
  return fail(ISING_EUNSUPPORTED, "tile bits or class count out of range");
}

}  // namespace ising

using namespace ising;

extern "C" ising_status ising_plan_destroy(ising_plan *p) {
  if (!p) return ISING_OK;
  for (int d = 0; d < kMaxDevices; ++d)
    if (p->dev_copy[d]) (void)hipFree(p->dev_copy[d]);
  bond_plan_free(p->bond);
  delete p;
  return ISING_OK;
}

extern "C" ising_status ising_enumerate(const ising_plan *p, uint64_t *g_dev, void *stream) {
  if (!p || !g_dev) return fail(ISING_EINVAL, "plan or g_dev is NULL");
  const size_t cells = size_t(2 * p->S + 1) * size_t(p->n_spins + 1);
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int threads = 256;
  const size_t blocks = std::min<size_t>((cells + threads - 1) / threads, 4096);
  hipLaunchKernelGGL(k_fill_u64, dim3(unsigned(blocks)), dim3(threads), 0, s,
                     reinterpret_cast<unsigned long long *>(g_dev), cells);
  HIP_TRY(hipGetLastError());
  return enumerate_chunks(p, 0, p->n_chunks, g_dev, s);
}

extern "C" ising_status ising_enumerate_range(const ising_plan *p, uint64_t first_chunk, uint64_t n_chunks,
                                              uint64_t *g_dev, void *stream) {
  if (!p || !g_dev) return fail(ISING_EINVAL, "plan or g_dev is NULL");
  if (first_chunk > p->n_chunks || n_chunks > p->n_chunks - first_chunk)
    return fail(ISING_EINVAL, "chunk range exceeds the plan's " + std::to_string(p->n_chunks) + " chunks");
  return enumerate_chunks(p, first_chunk, n_chunks, g_dev, static_cast<hipStream_t>(stream));
}

extern "C" ising_status ising_enumerate_symmetric(const ising_plan *p, uint64_t *g_dev, void *stream) {
  if (!p || !g_dev) return fail(ISING_EINVAL, "plan or g_dev is NULL");
  if (p->n_chunks < 2) return ising_enumerate(p, g_dev, stream);   // the top bit is not a prefix bit
  const size_t cells = size_t(2 * p->S + 1) * size_t(p->n_spins + 1);
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int threads = 256;
  hipLaunchKernelGGL(k_fill_u64, dim3(unsigned(std::min<size_t>((cells + threads - 1) / threads, 4096))),
                     dim3(threads), 0, s, reinterpret_cast<unsigned long long *>(g_dev), cells);
  HIP_TRY(hipGetLastError());
  const uint64_t half = p->n_chunks / 2;   // chunks [half, n_chunks): top plan bit up
  ising_status st = enumerate_chunks(p, half, half, g_dev, s);
  if (st != ISING_OK) return st;
  const int n_e = int(2 * p->S + 1), n_m = p->n_spins + 1;
  const size_t pairs = size_t(n_e) * size_t((n_m + 1) / 2);
  hipLaunchKernelGGL(k_mirror_u64, dim3(unsigned(std::min<size_t>((pairs + threads - 1) / threads, 4096))),
                     dim3(threads), 0, s, reinterpret_cast<unsigned long long *>(g_dev), n_e, n_m);
  HIP_TRY(hipGetLastError());
  return ISING_OK;
}
