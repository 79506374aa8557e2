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
//     with R copies per block; lane l writes copy l mod R.  Copy-major words
//     (bin * R + copy) and a bin-row stride that is a multiple of 4 keep the
//     32 lanes one LDS cycle serves in distinct banks.  Counters are u32; the
//     block flushes them (sum over copies, 64-bit global atomics into the
//     dense uint64 table) before any can reach 2^32, and at exit.
//   * No HBM traffic beyond the final flush: the kernel is bound by the LDS
//     atomic rate (one ds_add_u32 per configuration).
#include <hip/hip_runtime.h>

#include <string>

#include "internal.h"

namespace ising {

#define HIP_TRY(expr)                                                                        \
  do {                                                                                       \
    hipError_t e_ = (expr);                                                                  \
    if (e_ != hipSuccess) return fail(ISING_EHIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

// ---------------------------------------------------------------------------
// device helpers
// ---------------------------------------------------------------------------

__device__ __forceinline__ void lds_count(char *hist, uint32_t byte_addr) {
  __hip_atomic_fetch_add(reinterpret_cast<uint32_t *>(hist + byte_addr), 1u, __ATOMIC_RELAXED,
                         __HIP_MEMORY_SCOPE_WORKGROUP);
}

// One block of 2^TJ configurations: count the current one, then walk the
// tile bits in Gray order.  In odd blocks the tile starts with its top bit
// set (reflected code), so that bit's single flip goes down instead of up.
template <int TJ, bool ODD>
__device__ __forceinline__ void tile_walk(uint32_t &A, const int32_t (&D)[TJ], char *hist) {
  lds_count(hist, A);
#pragma unroll
  for (int t = 1; t < (1 << TJ); ++t) {
    const int b = __builtin_ctz(t);
    const int gray = t ^ (t >> 1);
    bool up = (gray >> b) & 1;
    if (ODD && b == TJ - 1) up = !up;
    A = up ? A + uint32_t(D[b]) : A - uint32_t(D[b]);
    lds_count(hist, A);
  }
}

// Plan constants held in registers for the whole launch.  Per-site data sit
// one site per lane (site b in lane b, N <= 64) and are fetched with
// v_readlane at a wave-uniform index, so neither the chunk set-up nor the
// walk issues a scalar memory load (whose wait would also drain the wave's
// outstanding LDS atomics).
template <int TJ, int NC>
struct SiteTable {
  uint32_t mlo[NC], mhi[NC];   // neighbour masks of the lane's site, per coupling class
  int32_t hdeg;                // sum_c J_c deg_c of the lane's site
  int32_t base;                // up_base of the lane's site
  int32_t kmid[TJ];            // lane m: tile-delta changes when middle bit TJ + m flips up
  int32_t jc[NC], step[NC];    // class couplings and byte steps (uniform)
  int32_t n, k, e_base, estep, row_bytes, col_bytes;   // uniform

  __device__ void load(const DevPlan *__restrict__ P, int lane) {
    n = P->n;
    k = P->inner;
    e_base = P->e_base;
    estep = P->estep;
    row_bytes = P->W * P->R * 4;
    col_bytes = P->R * 4;
    const bool site = lane < n;
    const int b = site ? lane : 0;
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      const uint64_t m = site ? P->mask[b][c] : 0ull;
      mlo[c] = uint32_t(m);
      mhi[c] = uint32_t(m >> 32);
      jc[c] = P->class_J[c];
      step[c] = P->cls_step[c];
    }
    hdeg = site ? P->hdeg[b] : 0;
    base = site ? P->up_base[b] : 0;
    const bool mid = lane < k - TJ;
#pragma unroll
    for (int i = 0; i < TJ; ++i) kmid[i] = mid ? P->kmid[mid ? lane : 0][i] : 0;
  }

  // popcount(x & mask of site b, class c) for a wave-uniform b
  __device__ __forceinline__ int32_t pop(int b, int c, uint32_t xlo, uint32_t xhi) const {
    return __popc(xlo & uint32_t(__builtin_amdgcn_readlane(int(mlo[c]), b))) +
           __popc(xhi & uint32_t(__builtin_amdgcn_readlane(int(mhi[c]), b)));
  }

  // local field h_b = sum_j J_bj s_j
  __device__ __forceinline__ int32_t field(int b, uint32_t xlo, uint32_t xhi) const {
    int32_t acc = 0;
#pragma unroll
    for (int c = 0; c < NC; ++c) acc += jc[c] * pop(b, c, xlo, xhi);
    return 2 * acc - __builtin_amdgcn_readlane(hdeg, b);
  }

  // histogram byte-offset change when bit b flips up
  __device__ __forceinline__ int32_t up_delta(int b, uint32_t xlo, uint32_t xhi) const {
    int32_t acc = __builtin_amdgcn_readlane(base, b);
#pragma unroll
    for (int c = 0; c < NC; ++c) acc -= step[c] * pop(b, c, xlo, xhi);
    return acc;
  }
};

// All 2^k configurations of one chunk (prefix bits fixed).
template <int TJ, int NC>
__device__ void walk_chunk(const SiteTable<TJ, NC> &st, uint64_t chunk, uint32_t rep, char *hist) {
  const int k = st.k;
  const uint64_t x0 = chunk << k;
  const uint32_t x0lo = uint32_t(x0), x0hi = uint32_t(x0 >> 32);

  // Full (E, n_up) of the first configuration: E = -(1/2) sum_i s_i h_i.
  int32_t hs = 0;
  for (int i = 0; i < st.n; ++i) {
    const int32_t h = st.field(i, x0lo, x0hi);
    hs += ((x0 >> i) & 1) ? h : -h;
  }
  const int32_t E0 = -(hs / 2);
  const int32_t nup = __popcll(x0);
  uint32_t A = uint32_t(((E0 - st.e_base) / st.estep) * st.row_bytes + nup * st.col_bytes) + rep * 4u;

  // Up-flip address change of each tile spin (its neighbours are all outside
  // the tile, so these stay fixed while only tile bits flip).
  int32_t D[TJ];
#pragma unroll
  for (int i = 0; i < TJ; ++i) D[i] = st.up_delta(i, x0lo, x0hi);

  const uint32_t nblk = 1u << (k - TJ);
  for (uint32_t q = 0; q < nblk; ++q) {
    if (q & 1)
      tile_walk<TJ, true>(A, D, hist);
    else
      tile_walk<TJ, false>(A, D, hist);
    if (q + 1 < nblk) {
      // Gray step q -> q+1 of the middle bits flips bit TJ + ctz(q+1).
      const uint32_t q1 = q + 1;
      const int mm = __builtin_ctz(q1);
      const bool up = (((q1 ^ (q1 >> 1)) >> mm) & 1u) != 0;
      // current inner bits: tile at its end state, middle bits = gray(q)
      const uint64_t inner = ((q & 1) ? 0ull : (1ull << (TJ - 1))) | (uint64_t(q ^ (q >> 1)) << TJ);
      const int32_t dm = st.up_delta(TJ + mm, x0lo | uint32_t(inner), x0hi | uint32_t(inner >> 32));
      A = up ? A + uint32_t(dm) : A - uint32_t(dm);
#pragma unroll
      for (int i = 0; i < TJ; ++i) {
        const int32_t kv = __builtin_amdgcn_readlane(st.kmid[i], mm);
        D[i] = up ? D[i] + kv : D[i] - kv;
      }
    }
  }
}

// Sum the R copies of every compact bin, clear them, add to the dense table.
__device__ void flush_hist(const DevPlan *__restrict__ P, uint32_t *h, unsigned long long *__restrict__ g) {
  const int W = P->W, R = P->R;
  const int bins = P->n_ec * W;
  for (int b = threadIdx.x; b < bins; b += blockDim.x) {
    unsigned long long s = 0;
    for (int r = 0; r < R; ++r) {
      s += h[b * R + r];
      h[b * R + r] = 0;
    }
    const int e_idx = b / W, nu = b - e_idx * W;
    if (s && nu < P->n_m) {
      const int E = P->e_base + e_idx * P->estep;
      atomicAdd(&g[size_t(E - P->e_min) * P->n_m + nu], s);
    }
  }
}

// Task t of this block covers chunks (task_lo + t) * blockDim.x + [0, blockDim.x),
// one per thread; lanes whose chunk lies outside [chunk_lo, chunk_hi) idle.
// Lanes l and l + 16 of a half-wave share LDS copy l mod 16; their chunks
// differ in one prefix spin, so their n_up differ by one, and with a row
// stride W = 0 (mod 4) their words fall in different banks (bank = 16 * (bin
// mod 4) + copy on the 64-bank LDS).  All threads of a block run the
// same number of tasks, so the barriers around periodic flushes are uniform.
template <int TJ, int NC>
__global__ __launch_bounds__(1024) void k_enumerate(const DevPlan *__restrict__ P, uint64_t chunk_lo,
                                                    uint64_t chunk_hi, uint64_t task_lo, uint64_t n_tasks,
                                                    uint32_t flush_every, unsigned long long *__restrict__ g) {
  // Static (not dynamic) LDS: its base address is a compile-time constant, so
  // each histogram update is a single ds_add_u32 on the running address.
  __shared__ __align__(16) uint32_t h32[kLdsBytes / 4];
  char *hist = reinterpret_cast<char *>(h32);
  const int words = P->n_ec * P->W * P->R;
  for (int w = threadIdx.x; w < words; w += blockDim.x) h32[w] = 0;
  __syncthreads();
  const uint32_t lane = threadIdx.x & (kWave - 1);
  const uint32_t rep = lane & uint32_t(P->R - 1);
  SiteTable<TJ, NC> st;
  st.load(P, int(lane));
  uint32_t since = 0;
  for (uint64_t t = blockIdx.x; t < n_tasks; t += gridDim.x) {
    const uint64_t chunk = (task_lo + t) * blockDim.x + threadIdx.x;
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
