// Batched enumeration: many finite Ising systems of uneven size in one
// persistent launch, and the batched FP64 moments; both can be captured in a
// HIP graph.
//
// Each member is planned exactly like a single lattice (same ordering, tile
// walk and LDS histogram; see enumerate.hip), with one coupling-class count
// shared by the batch so one kernel instantiation serves every member; each
// member keeps its own tile width, chunk width, LDS copy count and thread ->
// chunk table.  The work list holds (member, task) units - a task is one
// chunk per thread of a block - ordered largest member first; blocks take
// units from a device counter.  A block keeps one member's histogram in LDS
// and flushes it to that member's table whenever it moves to another member
// (or before its counters could overflow), so consecutive units of a large
// member cost no flush.  The smallest members, last in the list, take short
// chunks so that the launch ends on short units.  A second, halved work list
// covers only the chunks with each member's top spin up; k_batch_mirror then
// completes every table from the spin-flip symmetry.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <numeric>
#include <string>
#include <vector>

#include "internal.h"
#include "walk.h"

namespace ising {

ising_status batch_thermo_launch(const BatchMember *meta_dev, int n_members, const uint64_t *g_all,
                                 const double *T_dev, int32_t nT, const double *h_dev, int32_t nh, double *logz,
                                 double *mE, double *mM, double *C, double *chi, hipStream_t stream);

#define HIP_TRY(expr)                                                                                  \
  do {                                                                                                 \
    hipError_t e_ = (expr);                                                                            \
    if (e_ != hipSuccess) return fail(ISING_EHIP, std::string(#expr) + ": " + hipGetErrorString(e_));  \
  } while (0)

// Zero the concatenated tables and the work counter.
__global__ void k_batch_prepare(unsigned long long *g, size_t n, uint32_t *counter) {
  const size_t stride = size_t(gridDim.x) * blockDim.x;
  for (size_t i = blockIdx.x * size_t(blockDim.x) + threadIdx.x; i < n; i += stride) g[i] = 0ull;
  if (blockIdx.x == 0 && threadIdx.x == 0) *counter = 0u;
}

template <int NC>
__global__ __launch_bounds__(1024) void k_batch_enumerate(const DevPlan *__restrict__ plans,
                                                          const BatchMember *__restrict__ meta,
                                                          const BatchUnit *__restrict__ units, uint32_t n_units,
                                                          uint32_t *__restrict__ counter,
                                                          unsigned long long *__restrict__ g_all) {
  __shared__ __align__(16) uint32_t h32[kHistBytes / 4];
  __shared__ uint32_t s_unit[2];
  char *hist = reinterpret_cast<char *>(h32);
  for (int w = threadIdx.x; w < kHistBytes / 4; w += blockDim.x) h32[w] = 0;
  const uint32_t lane = threadIdx.x & (kWave - 1);
  SiteTable<NC> st;
  uint32_t offset = threadIdx.x;
  int cur = -1;
  uint32_t since = 0, it = 0;
  for (;; ++it) {
    // Thread 0 takes the next unit into slot it & 1; the barrier also ends
    // every thread's previous walk, so a flush may follow.  The other slot
    // cannot be overwritten before all threads pass the next barrier.
    if (threadIdx.x == 0) s_unit[it & 1] = atomicAdd(counter, 1u);
    __syncthreads();
    const uint32_t u = s_unit[it & 1];
    if (u >= n_units) break;
    const BatchUnit un = units[u];
    if (un.inst != cur || since == meta[cur].flush_every) {
      if (cur >= 0) {
        flush_hist(&plans[cur], h32, g_all + meta[cur].offset);
        __syncthreads();
      }
      if (un.inst != cur) {
        cur = un.inst;
        st.load(&plans[cur], int(lane));
        offset = plans[cur].lane_chunk[threadIdx.x];
      }
      since = 0;
    }
    const DevPlan *P = &plans[cur];
    const uint64_t chunk = un.task * blockDim.x + offset;
    if (chunk < meta[cur].n_chunks && offset >= uint32_t(un.first_offset)) {
      const uint32_t rep = lane_copy(lane, P->R);
      switch (P->tile) {  // uniform: each member keeps its own tile width
        case 1: walk_chunk<1, NC>(st, chunk, rep, hist); break;
        case 2: walk_chunk<2, NC>(st, chunk, rep, hist); break;
        case 3: walk_chunk<3, NC>(st, chunk, rep, hist); break;
        case 4: walk_chunk<4, NC>(st, chunk, rep, hist); break;
        case 5: walk_chunk<5, NC>(st, chunk, rep, hist); break;
        case 6: walk_chunk<6, NC>(st, chunk, rep, hist); break;
        case 7: walk_chunk<7, NC>(st, chunk, rep, hist); break;
        default: walk_chunk<8, NC>(st, chunk, rep, hist); break;
      }
    }
    ++since;
  }
  if (cur >= 0) flush_hist(&plans[cur], h32, g_all + meta[cur].offset);
}

static ising_status batch_device(ising_batch_plan *bp, int device, ising_batch_plan::Dev **out) {
  if (device < 0 || device >= kMaxDevices) return fail(ISING_EUNSUPPORTED, "device index out of range");
  std::lock_guard<std::mutex> lk(bp->mu);
  ising_batch_plan::Dev &d = bp->dev[device];
  if (!d.plans) {
    std::vector<DevPlan> plans(bp->n);
    for (int i = 0; i < bp->n; ++i) plans[i] = bp->members[i]->dev;
    HIP_TRY(hipMalloc(&d.plans, sizeof(DevPlan) * plans.size()));
    HIP_TRY(hipMalloc(&d.meta, sizeof(BatchMember) * bp->meta.size()));
    HIP_TRY(hipMalloc(&d.units, sizeof(BatchUnit) * std::max<size_t>(1, bp->units.size())));
    HIP_TRY(hipMalloc(&d.units_half, sizeof(BatchUnit) * std::max<size_t>(1, bp->units_half.size())));
    HIP_TRY(hipMalloc(&d.counter, sizeof(uint32_t)));
    HIP_TRY(hipMemcpy(d.plans, plans.data(), sizeof(DevPlan) * plans.size(), hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(d.meta, bp->meta.data(), sizeof(BatchMember) * bp->meta.size(), hipMemcpyHostToDevice));
    if (!bp->units.empty())
      HIP_TRY(hipMemcpy(d.units, bp->units.data(), sizeof(BatchUnit) * bp->units.size(), hipMemcpyHostToDevice));
    if (!bp->units_half.empty())
      HIP_TRY(hipMemcpy(d.units_half, bp->units_half.data(), sizeof(BatchUnit) * bp->units_half.size(),
                        hipMemcpyHostToDevice));
  }
  *out = &d;
  return ISING_OK;
}

template <int NC>
static void launch_batch_nc(const ising_batch_plan::Dev *d, const void *units, uint32_t n_units, int grid,
                            int block, unsigned long long *g, hipStream_t s) {
  hipLaunchKernelGGL((k_batch_enumerate<NC>), dim3(grid), dim3(block), 0, s,
                     static_cast<const DevPlan *>(d->plans), static_cast<const BatchMember *>(d->meta),
                     static_cast<const BatchUnit *>(units), n_units, static_cast<uint32_t *>(d->counter), g);
}

// Halved run: every member with at least two chunks was enumerated over the
// chunks with its top spin up; g(E, M) = h(E, M) + h(E, -M) restores it
// (a global flip keeps E and negates M).  One block row per member.
__global__ void k_batch_mirror(const BatchMember *__restrict__ meta, unsigned long long *__restrict__ g_all) {
  const BatchMember m = meta[blockIdx.y];
  if (m.n_chunks < 2) return;
  unsigned long long *g = g_all + m.offset;
  const int half = (m.n_m + 1) / 2;   // nu in [0, half) pairs with n_m - 1 - nu
  const size_t cells = size_t(m.n_e) * half;
  for (size_t i = blockIdx.x * size_t(blockDim.x) + threadIdx.x; i < cells; i += size_t(gridDim.x) * blockDim.x) {
    const size_t e = i / half;
    const int nu = int(i - e * half), mu = m.n_m - 1 - nu;
    unsigned long long *row = g + e * m.n_m;
    const unsigned long long v = row[nu] + row[mu];
    row[nu] = v;
    row[mu] = v;
  }
}

static ising_status batch_enumerate_launch(const ising_batch_plan *bpc, uint64_t *g_all, hipStream_t s,
                                           const ising_batch_plan::Dev *d, bool halve = false) {
  const ising_batch_plan *bp = bpc;
  int dev = 0, cus = 0;
  HIP_TRY(hipGetDevice(&dev));
  HIP_TRY(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
  unsigned long long *g = reinterpret_cast<unsigned long long *>(g_all);
  const size_t n_elems = size_t(bp->total_elems);
  const size_t fill_blocks = std::min<size_t>(std::max<size_t>(1, (n_elems + 255) / 256), 4096);
  hipLaunchKernelGGL(k_batch_prepare, dim3(unsigned(fill_blocks)), dim3(256), 0, s, g, n_elems,
                     static_cast<uint32_t *>(d->counter));
  HIP_TRY(hipGetLastError());
  const uint32_t n_units = uint32_t((halve ? bp->units_half : bp->units).size());
  const void *units = halve ? d->units_half : d->units;
  if (!n_units) return ISING_OK;
  int grid = cus;
  if (bp->max_blocks > 0 && bp->max_blocks < grid) grid = bp->max_blocks;
  if (uint32_t(grid) > n_units) grid = int(n_units);
  const int block = kWave * bp->waves_per_block;
  switch (bp->n_classes) {
    case 1: launch_batch_nc<1>(d, units, n_units, grid, block, g, s); break;
    case 2: launch_batch_nc<2>(d, units, n_units, grid, block, g, s); break;
    case 4: launch_batch_nc<4>(d, units, n_units, grid, block, g, s); break;
    case 8: launch_batch_nc<8>(d, units, n_units, grid, block, g, s); break;
    default: return fail(ISING_EUNSUPPORTED, "class count");
  }
  HIP_TRY(hipGetLastError());
  if (halve) {
    hipLaunchKernelGGL(k_batch_mirror, dim3(16, unsigned(bp->n)), dim3(256), 0, s,
                       static_cast<const BatchMember *>(d->meta), g);
    HIP_TRY(hipGetLastError());
  }
  return ISING_OK;
}

}  // namespace ising

using namespace ising;

struct ising_graph {
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

// Tail of the batch work list: a task is one chunk per thread of a
// 1024-thread block (2^10 chunks); kTailBlocks is the CU count of an MI355X.
constexpr int kTailTaskBits = 10;
constexpr int kTailBlocks = 256;
constexpr int kTailInner = 12;
// Per-member kernels index members by grid y (at most 65535).
constexpr int kMaxMembers = 65535;

extern "C" ising_status ising_batch_plan_create(const ising_lattice *lats, int32_t n, const ising_tune *tune,
                                                ising_batch_plan **out) {
  if (!out) return fail(ISING_EINVAL, "plan output pointer is NULL");
  *out = nullptr;
  if (n < 1 || !lats) return fail(ISING_EINVAL, "need at least one lattice");
  if (n > kMaxMembers) return fail(ISING_EINVAL, "at most " + std::to_string(kMaxMembers) + " lattices per batch");
  ising_tune tn{};
  if (tune) tn = *tune;
  // Members keep their own chunk width: inner_bits (default 14, at most N)
  // unless prefix_bits is given.  The batch, not one member, fills the GPU,
  // so chunks can be long enough to amortise their set-up.
  const int inner_default = tn.inner_bits ? tn.inner_bits : (tn.prefix_bits ? 0 : 14);
  // Pass 1: each member on its own, to find the largest class count (one
  // kernel instantiation serves the batch; members keep their own tile width,
  // capped by tune.tile_bits when given).
  // The smallest members, together about one round of units over the grid
  // (kTailBlocks tasks of the default width) and last in the longest-first
  // work list, take short chunks (at most 2^kTailInner configurations), so
  // the launch ends on short units and blocks finish closer together.
  std::vector<char> tail(size_t(n), 0);
  if (inner_default > 2) {
    std::vector<int> by_size(static_cast<size_t>(n));
    std::iota(by_size.begin(), by_size.end(), 0);
    std::stable_sort(by_size.begin(), by_size.end(),
                     [&](int a, int b) { return lats[a].n_spins < lats[b].n_spins; });
    const double budget = double(kTailBlocks) * std::ldexp(1.0, inner_default + kTailTaskBits);
    double cum = 0.0;
    for (int i : by_size) {
      cum += std::ldexp(1.0, std::max(0, std::min(lats[i].n_spins, 63)));
      if (cum > budget) break;
      tail[size_t(i)] = 1;
    }
  }
  auto member_tune = [&](int i) {
    ising_tune t = tn;
    int inner = inner_default;
    if (tail[size_t(i)]) inner = std::min(inner - 2, kTailInner);
    t.inner_bits = inner ? std::min(inner, lats[i].n_spins) : 0;
    if (t.inner_bits && !t.tile_bits) t.tile_bits = std::min(kMaxTile, t.inner_bits);
    return t;
  };
  int classes = 1;
  for (int i = 0; i < n; ++i) {
    if (!lats[i].n_spins || lats[i].n_spins < 0 || lats[i].n_spins > kMaxSpins)
      return fail(ISING_ETOO_MANY_SPINS, "member " + std::to_string(i) + ": n_spins must be 1..64");
    const ising_tune t1 = member_tune(i);
    ising_plan *p = nullptr;
    ising_status st = plan_create_internal(&lats[i], &t1, 1, &p, false);
    if (st != ISING_OK) return fail(st, "member " + std::to_string(i) + ": " + ising_last_error());
    classes = std::max(classes, p->dev.n_classes);
    ising_plan_destroy(p);
  }
  // Pass 2: final member plans with the shared class count.
  ising_batch_plan *bp = new (std::nothrow) ising_batch_plan();
  if (!bp) return fail(ISING_ENOMEM, "batch plan");
  bp->n = n;
  bp->n_classes = classes;
  bp->waves_per_block = tn.waves_per_block ? tn.waves_per_block : 16;
  bp->max_blocks = tn.max_blocks;
  int64_t off = 0;
  for (int i = 0; i < n; ++i) {
    const ising_tune t2 = member_tune(i);
    ising_plan *p = nullptr;
    ising_status st = plan_create_internal(&lats[i], &t2, classes, &p, false);
    if (st != ISING_OK) {
      ising_batch_plan_destroy(bp);
      return fail(st, "member " + std::to_string(i) + ": " + ising_last_error());
    }
    bp->members.push_back(p);
    const DevPlan &d = p->dev;
    BatchMember m{};
    m.n_chunks = p->n_chunks;
    m.offset = off;
    const int block = kWave * bp->waves_per_block;
    const uint64_t per_task = (uint64_t(block) / uint64_t(d.R)) << d.inner;
    uint64_t fe = 0xFFFFFFFFull / per_task;
    m.flush_every = uint32_t(std::max<uint64_t>(1, std::min<uint64_t>(fe, 0x7FFFFFFFull)));
    m.n_e = int32_t(2 * p->S + 1);
    m.n_m = p->n_spins + 1;
    m.e_min = int32_t(-p->S);
    m.n_spins = p->n_spins;
    off += int64_t(m.n_e) * m.n_m;
    bp->meta.push_back(m);
  }
  bp->total_elems = off;
  // Work list: members by decreasing 2^N (longest first), each member's tasks in order.
  std::vector<int> order(n);
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(),
                   [&](int a, int b) { return bp->members[a]->n_spins > bp->members[b]->n_spins; });
  const uint64_t block = uint64_t(kWave) * bp->waves_per_block;
  for (int i : order) {
    const uint64_t nc = bp->meta[i].n_chunks;
    const uint64_t tasks = (nc + block - 1) / block;
    for (uint64_t t = 0; t < tasks; ++t) bp->units.push_back(BatchUnit{i, 0, t});
    // Halved list: chunks [nc/2, nc), whose top chunk bit (the top spin) is
    // up (nc is a power of two); a one-chunk member runs whole.
    if (nc < 2) {
      bp->units_half.push_back(BatchUnit{i, 0, 0});
    } else {
      const uint64_t h0 = nc / 2, t0 = h0 / block;
      for (uint64_t t = t0; t < tasks; ++t)
        bp->units_half.push_back(BatchUnit{i, t == t0 ? int32_t(h0 - t0 * block) : 0, t});
    }
  }
  if (bp->units.size() >= (size_t(1) << 31)) {
    ising_batch_plan_destroy(bp);
    return fail(ISING_EUNSUPPORTED, "too many work units; use fewer, larger chunks (prefix_bits)");
  }
  *out = bp;
  set_error("");
  return ISING_OK;
}

extern "C" ising_status ising_batch_plan_destroy(ising_batch_plan *bp) {
  if (!bp) return ISING_OK;
  for (ising_plan *p : bp->members) ising_plan_destroy(p);
  for (int d = 0; d < kMaxDevices; ++d) {
    ising_batch_plan::Dev &x = bp->dev[d];
    if (x.plans) (void)hipFree(x.plans);
    if (x.meta) (void)hipFree(x.meta);
    if (x.units) (void)hipFree(x.units);
    if (x.units_half) (void)hipFree(x.units_half);
    if (x.counter) (void)hipFree(x.counter);
  }
  delete bp;
  return ISING_OK;
}

extern "C" ising_status ising_batch_layout(const ising_batch_plan *bp, int64_t *offsets, int32_t *n_e,
                                           int32_t *n_m, int32_t *e_min, int32_t *n_spins) {
  if (!bp) return fail(ISING_EINVAL, "batch plan is NULL");
  for (int i = 0; i < bp->n; ++i) {
    const BatchMember &m = bp->meta[i];
    if (offsets) offsets[i] = m.offset;
    if (n_e) n_e[i] = m.n_e;
    if (n_m) n_m[i] = m.n_m;
    if (e_min) e_min[i] = m.e_min;
    if (n_spins) n_spins[i] = m.n_spins;
  }
  if (offsets) offsets[bp->n] = bp->total_elems;
  return ISING_OK;
}

extern "C" ising_status ising_batch_enumerate(const ising_batch_plan *bp, uint64_t *g_all_dev, void *stream) {
  if (!bp || !g_all_dev) return fail(ISING_EINVAL, "batch plan or g_all_dev is NULL");
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  ising_batch_plan::Dev *d = nullptr;
  ising_status st = batch_device(const_cast<ising_batch_plan *>(bp), dev, &d);
  if (st != ISING_OK) return st;
  return batch_enumerate_launch(bp, g_all_dev, static_cast<hipStream_t>(stream), d);
}

extern "C" ising_status ising_batch_enumerate_symmetric(const ising_batch_plan *bp, uint64_t *g_all_dev,
                                                        void *stream) {
  if (!bp || !g_all_dev) return fail(ISING_EINVAL, "batch plan or g_all_dev is NULL");
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  ising_batch_plan::Dev *d = nullptr;
  ising_status st = batch_device(const_cast<ising_batch_plan *>(bp), dev, &d);
  if (st != ISING_OK) return st;
  return batch_enumerate_launch(bp, g_all_dev, static_cast<hipStream_t>(stream), d, true);
}

extern "C" ising_status ising_batch_moments(const ising_batch_plan *bp, const uint64_t *g_all_dev,
                                            const double *T_dev, int32_t nT, const double *h_dev, int32_t nh,
                                            double *logz, double *mean_E, double *mean_M, double *heat,
                                            double *susc, void *stream) {
  if (!bp || !g_all_dev) return fail(ISING_EINVAL, "batch plan or g_all_dev is NULL");
  if (nT < 0 || nh < 0 || int64_t(bp->n) * nT * nh >= (int64_t(1) << 31))
    return fail(ISING_EINVAL, "bad grid size");
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  ising_batch_plan::Dev *d = nullptr;
  ising_status st = batch_device(const_cast<ising_batch_plan *>(bp), dev, &d);
  if (st != ISING_OK) return st;
  return batch_thermo_launch(static_cast<const BatchMember *>(d->meta), bp->n, g_all_dev, T_dev, nT, h_dev, nh,
                             logz, mean_E, mean_M, heat, susc, static_cast<hipStream_t>(stream));
}

static ising_status batch_graph_create(const ising_batch_plan *bp, uint64_t *g_all_dev, const double *T_dev,
                                       int32_t nT, const double *h_dev, int32_t nh, double *logz, double *mean_E,
                                       double *mean_M, double *heat, double *susc, bool halve, ising_graph **out) {
  if (!out) return fail(ISING_EINVAL, "graph output pointer is NULL");
  *out = nullptr;
  if (!bp || !g_all_dev) return fail(ISING_EINVAL, "batch plan or g_all_dev is NULL");
  if (nT < 0 || nh < 0 || int64_t(bp->n) * nT * nh >= (int64_t(1) << 31))
    return fail(ISING_EINVAL, "bad grid size");
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  ising_batch_plan::Dev *d = nullptr;
  ising_status st = batch_device(const_cast<ising_batch_plan *>(bp), dev, &d);  // uploads outside capture
  if (st != ISING_OK) return st;
  hipStream_t s = nullptr;
  HIP_TRY(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
  ising_graph *gr = new (std::nothrow) ising_graph();
  if (!gr) {
    (void)hipStreamDestroy(s);
    return fail(ISING_ENOMEM, "graph");
  }
  hipError_t e = hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal);
  if (e == hipSuccess) {
    st = batch_enumerate_launch(bp, g_all_dev, s, d, halve);
    if (st == ISING_OK && nT > 0 && nh > 0 && (logz || mean_E || mean_M || heat || susc))
      st = batch_thermo_launch(static_cast<const BatchMember *>(d->meta), bp->n, g_all_dev, T_dev, nT, h_dev, nh,
                               logz, mean_E, mean_M, heat, susc, s);
    hipGraph_t graph = nullptr;
    hipError_t e2 = hipStreamEndCapture(s, &graph);
    if (st == ISING_OK && e2 != hipSuccess)
      st = fail(ISING_EHIP, std::string("hipStreamEndCapture: ") + hipGetErrorString(e2));
    gr->graph = graph;
    if (st == ISING_OK) {
      e2 = hipGraphInstantiate(&gr->exec, graph, nullptr, nullptr, 0);
      if (e2 != hipSuccess) st = fail(ISING_EHIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(e2));
    }
  } else {
    st = fail(ISING_EHIP, std::string("hipStreamBeginCapture: ") + hipGetErrorString(e));
  }
  (void)hipStreamDestroy(s);
  if (st != ISING_OK) {
    ising_graph_destroy(gr);
    return st;
  }
  *out = gr;
  return ISING_OK;
}

extern "C" ising_status ising_batch_graph_create(const ising_batch_plan *bp, uint64_t *g_all_dev,
                                                 const double *T_dev, int32_t nT, const double *h_dev, int32_t nh,
                                                 double *logz, double *mean_E, double *mean_M, double *heat,
                                                 double *susc, ising_graph **out) {
  return batch_graph_create(bp, g_all_dev, T_dev, nT, h_dev, nh, logz, mean_E, mean_M, heat, susc, false, out);
}

extern "C" ising_status ising_batch_graph_create_symmetric(const ising_batch_plan *bp, uint64_t *g_all_dev,
                                                           const double *T_dev, int32_t nT, const double *h_dev,
                                                           int32_t nh, double *logz, double *mean_E, double *mean_M,
                                                           double *heat, double *susc, ising_graph **out) {
  return batch_graph_create(bp, g_all_dev, T_dev, nT, h_dev, nh, logz, mean_E, mean_M, heat, susc, true, out);
}

extern "C" ising_status ising_graph_launch(const ising_graph *gr, void *stream) {
  if (!gr || !gr->exec) return fail(ISING_EINVAL, "graph is NULL");
  HIP_TRY(hipGraphLaunch(gr->exec, static_cast<hipStream_t>(stream)));
  return ISING_OK;
}

extern "C" ising_status ising_graph_destroy(ising_graph *gr) {
  if (!gr) return ISING_OK;
  if (gr->exec) (void)hipGraphExecDestroy(gr->exec);
  if (gr->graph) (void)hipGraphDestroy(gr->graph);
  delete gr;
  return ISING_OK;
}
