// Per-bond backward of log Z: dJ_b = sum over all 2^N configurations of
// W(E, M) s_i s_j, for a per-bin weight table W (k_bin_weights in
// thermo.hip makes W from a loss gradient).  Eq. (1) of Peretyatko et al.
// (Section 2) makes H depend on J_b only through -J_b s_i s_j, so
// d log Z / dJ_b = <s_i s_j> / T needs, besides g(E, M), the bond spin
// product of every configuration; the enumeration is recomputed here in the
// same Gray order as the forward walk, with FP64 sums in place of counts.
//
// Per lane and chunk (prefix fixed; k = tile + mj inner bits, mj <= 4; which
// chunk of a task a thread takes is a planner table chosen so that lanes
// sharing a weight-table copy read different LDS banks):
//   * the tile walk (2^TJ configurations, only tile bits flip, fully
//     unrolled) reads W of each configuration from an LDS copy of the table
//     (one ds_read_b64 on the same running address as the forward's
//     histogram add).  The sums of W over the configurations with tile spin
//     i up come from groups of 8 configurations: an add tree of the group
//     gives tile bits 0-2 (up on fixed positions of the group), and higher
//     tile bits, which flip only between groups, use a prefix-sum trick on
//     the running sum of group totals.  Which spin flips, and which way, is a
//     compile-time fact of the unrolled Gray sequence, so a configuration
//     costs one load, one integer add and about two FP64 adds.
//   * per tile block (walk) q the sums S_q = sum W and Y_q,i = sum W s_i are
//     folded into the lane's running totals: sum W, sum W s_t, sum W s_m,
//     sum W s_t s_m, sum W s_m1 s_m2 (s_m, the middle spins, are fixed within
//     a block).  They run over all of the lane's chunks, never reset.
//   * every coupled pair takes its sum from one of these (tile-middle,
//     middle-middle), from sum W s_a times the sign of a prefix spin b
//     (inner-prefix pairs), or from sum W times s_a s_b (both in the prefix).
//     A thread's chunks share their low 9 bits (the block has 512 threads),
//     so prefix spins there are fixed per thread; the rest ("task" bits) are
//     the same for the whole block within one task.  Pairs with no task bit
//     are summed over the wave once, at the end; the others after every task,
//     from the growth of the wave totals they need (about a dozen per task
//     rather than one per pair).  Wave sums use a DPP tree and go to per-wave
//     LDS accumulators; blocks write per-pair partial sums and a second
//     kernel adds them in a fixed order and scatters them to the input bonds.
//     Every sum runs in a fixed order, so results are reproducible.
// The tile is an independent set of the coupling graph, so there are no
// tile-tile pairs.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <string>

#include "bond.h"
#include "internal.h"
#include "walk.h"

namespace ising {

#define HIP_TRY(expr)                                                                        \
  do {                                                                                       \
    hipError_t e_ = (expr);                                                                  \
    if (e_ != hipSuccess) return fail(ISING_EHIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

__device__ __forceinline__ double lds_f64(const char *base, uint32_t byte_addr) {
  return *reinterpret_cast<const double *>(base + byte_addr);
}

// One tile block of 2^TJ configurations: sw = sum of W, U[i] = sum of W over
// the configurations with tile spin i up.  Odd blocks start with the top tile
// bit set (reflected Gray code), so the tile state at step t is
// gray(t) ^ (ODD ? top : 0).
template <int TJ, bool ODD>
__host__ __device__ constexpr uint32_t tile_state(int t) {
  return uint32_t(t ^ (t >> 1)) ^ (ODD ? (1u << (TJ - 1)) : 0u);
}

// Tile blocks of TJ >= 3 bits, in groups of 8 configurations (the low three
// tile bits): inside a group, tile bits 0-2 are up on fixed position sets
// ({1,2,5,6}, {2,3,4,5}, {4..7} or {0..3}, or their complements for the top
// bit of an odd block), so their sums come from a small add tree of the
// group (pairs, quads, total); higher tile bits flip only between groups and
// use the prefix-sum trick on the running sum of group totals (subtract it
// when the spin goes up, add it when it goes down, add the total at the end
// if still up).  About two FP64 adds per configuration, with a dependent
// chain of one add per group instead of one per configuration.
template <int TJ, bool ODD>
__device__ __forceinline__ double group_bit_sum(int g, int b, const double (&w)[8], double P23, double P45,
                                                double Q0, double Q1, double G) {
  uint32_t mask = 0;
#pragma unroll
  for (int u = 0; u < 8; ++u) mask |= ((tile_state<TJ, ODD>(8 * g + u) >> b) & 1u) << u;
  switch (mask) {
    case 0x66: return (w[1] + w[2]) + (w[5] + w[6]);
    case 0x99: return G - ((w[1] + w[2]) + (w[5] + w[6]));
    case 0x3c: return P23 + P45;
    case 0xc3: return G - (P23 + P45);
    case 0xf0: return Q1;
    case 0x0f: return Q0;
    default: {   // not reached for the reflected Gray code; kept general
      double acc = 0.0;
#pragma unroll
      for (int u = 0; u < 8; ++u)
        if ((mask >> u) & 1u) acc += w[u];
      return acc;
    }
  }
}

template <int TJ, bool ODD>
__device__ __forceinline__ void weight_walk(uint32_t &A, const int32_t (&D)[TJ], const char *wt, double &sw,
                                            double (&U)[TJ]) {
  constexpr int kN = 1 << TJ;
  constexpr uint32_t kEnd = tile_state<TJ, ODD>(kN - 1);
#pragma unroll
  for (int i = 0; i < TJ; ++i) U[i] = 0.0;
  sw = 0.0;
  if constexpr (TJ >= 3) {
    constexpr int kGroups = kN / 8;
    // W of a group is loaded one group ahead of its sums.
    double w[2][8];
#pragma unroll
    for (int g = 0; g <= kGroups; ++g) {
      if (g < kGroups) {
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          const int t = g * 8 + u;
          if (t > 0) {
            const int b = __builtin_ctz(t);
            A = ((tile_state<TJ, ODD>(t) >> b) & 1u) ? A + uint32_t(D[b]) : A - uint32_t(D[b]);
          }
          w[g & 1][u] = lds_f64(wt, A);
        }
      }
      if (g > 0) {
        const int gp = g - 1;
        const double(&v)[8] = w[gp & 1];
        if (gp > 0) {   // a tile bit >= 3 flipped on entering this group
          const int b = __builtin_ctz(gp * 8);
          if ((tile_state<TJ, ODD>(gp * 8) >> b) & 1u)
            U[b] -= sw;
          else
            U[b] += sw;
        }
        const double P01 = v[0] + v[1], P23 = v[2] + v[3], P45 = v[4] + v[5], P67 = v[6] + v[7];
        const double Q0 = P01 + P23, Q1 = P45 + P67, G = Q0 + Q1;
#pragma unroll
        for (int b = 0; b < 3; ++b) U[b] += group_bit_sum<TJ, ODD>(gp, b, v, P23, P45, Q0, Q1, G);
        sw += G;
      }
    }
#pragma unroll
    for (int i = 3; i < TJ; ++i)
      if ((kEnd >> i) & 1u) U[i] += sw;
  } else {
    // one or two tile bits: the prefix-sum trick per configuration
#pragma unroll
    for (int t = 0; t < kN; ++t) {
      if (t > 0) {
        const int b = __builtin_ctz(t);
        const bool up = ((tile_state<TJ, ODD>(t) >> b) & 1u) != 0;
        A = up ? A + uint32_t(D[b]) : A - uint32_t(D[b]);
        if (up)
          U[b] -= sw;
        else
          U[b] += sw;
      }
      sw += lds_f64(wt, A);
    }
#pragma unroll
    for (int i = 0; i < TJ; ++i)
      if ((kEnd >> i) & 1u) U[i] += sw;
  }
}

// Running totals of one lane over all the configurations it has walked.
template <int TJ>
struct LaneSums {
  double S;                 // W
  double Yt[TJ];            // W s_t, tile spins
  double Ym[kBwMid];        // W s_m, middle spins
  double Q[kBwMid][TJ];     // W s_m s_t
  double M2[6];             // W s_m1 s_m2, pairs (0,1) (0,2) (0,3) (1,2) (1,3) (2,3)

  __device__ __forceinline__ void clear() {
    S = 0.0;
#pragma unroll
    for (int i = 0; i < TJ; ++i) Yt[i] = 0.0;
#pragma unroll
    for (int m = 0; m < kBwMid; ++m) {
      Ym[m] = 0.0;
#pragma unroll
      for (int i = 0; i < TJ; ++i) Q[m][i] = 0.0;
    }
#pragma unroll
    for (int j = 0; j < 6; ++j) M2[j] = 0.0;
  }

  // W s_a for inner bit a (tile, then middle)
  __device__ __forceinline__ double inner(int a) const { return a < TJ ? Yt[a < TJ ? a : 0] : Ym[a < TJ ? 0 : a - TJ]; }
};

template <int TJ, int NC>
__device__ inline void bond_chunk(const SiteTable<NC> &st, uint64_t x0, uint32_t rep_bytes, const char *wt,
                                  LaneSums<TJ> &cs) {
  uint32_t A;
  int32_t D[TJ];
  chunk_start<TJ, NC>(st, x0, rep_bytes, A, D);
  const uint32_t nblk = 1u << (st.k - TJ);
  for (uint32_t q = 0; q < nblk; ++q) {
    double sw, U[TJ];
    if (q & 1)
      weight_walk<TJ, true>(A, D, wt, sw, U);
    else
      weight_walk<TJ, false>(A, D, wt, sw, U);
    // middle spins during block q: bits of gray(q) (unused slots read -1 and
    // are never consulted)
    const uint32_t mid = q ^ (q >> 1);
    double sg[kBwMid];
#pragma unroll
    for (int m = 0; m < kBwMid; ++m) sg[m] = ((mid >> m) & 1u) ? 1.0 : -1.0;
    cs.S += sw;
#pragma unroll
    for (int i = 0; i < TJ; ++i) {
      const double y = 2.0 * U[i] - sw;
      cs.Yt[i] += y;
#pragma unroll
      for (int m = 0; m < kBwMid; ++m) cs.Q[m][i] = fma(sg[m], y, cs.Q[m][i]);
    }
#pragma unroll
    for (int m = 0; m < kBwMid; ++m) cs.Ym[m] = fma(sg[m], sw, cs.Ym[m]);
    int j = 0;
#pragma unroll
    for (int m1 = 0; m1 < kBwMid; ++m1)
#pragma unroll
      for (int m2 = m1 + 1; m2 < kBwMid; ++m2, ++j) cs.M2[j] = fma(sg[m1] * sg[m2], sw, cs.M2[j]);
    if (q + 1 < nblk) middle_flip<TJ, NC>(st, x0, q, A, D);
  }
}

// One DPP move of a double (both 32-bit halves); lanes the pattern does not
// write read 0.
template <int CTRL, int ROW_MASK, bool BOUND_CTRL>
__device__ __forceinline__ double dpp_f64(double v) {
  const unsigned long long bits = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, int(uint32_t(bits)), CTRL, ROW_MASK, 0xf, BOUND_CTRL);
  const int hi = __builtin_amdgcn_update_dpp(0, int(uint32_t(bits >> 32)), CTRL, ROW_MASK, 0xf, BOUND_CTRL);
  return __longlong_as_double(static_cast<long long>((uint64_t(uint32_t(hi)) << 32) | uint32_t(lo)));
}

// Sum over the wave's 64 lanes, valid in lane 63, by a fixed DPP tree on the
// VALU (no LDS traffic): within each row of 16 lanes shifts by 1, 2, 4, 8 leave
// the row total in its lane 15; row_bcast:15 adds row 0 into row 1 and row 2
// into row 3, row_bcast:31 adds rows 0-1 into rows 2-3.
__device__ __forceinline__ double wave_total(double v) {
  v += dpp_f64<0x111, 0xf, true>(v);    // row_shr:1
  v += dpp_f64<0x112, 0xf, true>(v);    // row_shr:2
  v += dpp_f64<0x114, 0xf, true>(v);    // row_shr:4
  v += dpp_f64<0x118, 0xf, true>(v);    // row_shr:8
  v += dpp_f64<0x142, 0xa, false>(v);   // row_bcast:15
  v += dpp_f64<0x143, 0xc, false>(v);   // row_bcast:31
  return v;
}

// v s_b, and v s_a s_b, for the spins of bits a and b of state x
__device__ __forceinline__ double signed_by(uint64_t x, int b, double v) { return ((x >> b) & 1u) ? v : -v; }
__device__ __forceinline__ double signed_by2(uint64_t x, int a, int b, double v) {
  return (((x >> a) ^ (x >> b)) & 1u) ? -v : v;
}

// After a task: pairs with a task bit b, whose sign is the same for the whole
// block but changes from task to task.  The task's part of a lane sum is the
// growth of its wave total since the previous task (prev[], per wave, kept by
// lane 63, which holds the totals); it is added to the pair's accumulator with
// the task's sign of b.  One wave reduction per inner bit with task-bit
// partners, per lane-fixed bit with task-bit partners (of W s_a, s_a fixed per
// lane), and one of W for the task-task pairs.
template <int TJ>
__device__ inline void flush_task(const BondTables *__restrict__ T, const LaneSums<TJ> &cs, uint64_t x0,
                                  double *acc, double *prev, bool last_lane) {
#pragma unroll
  for (int a = 0; a < TJ + kBwMid; ++a) {
    const int e0 = T->it_start[a], e1 = T->it_start[a + 1];
    if (e0 < e1) {
      const double c = wave_total(cs.inner(a));
      if (last_lane) {
        const double r = c - prev[a];
        prev[a] = c;
        for (int e = e0; e < e1; ++e) acc[T->it_pair[e]] += signed_by(x0, T->it_bit[e], r);
      }
    }
  }
  const int n_ltg = T->n_ltg;
  for (int g = 0; g < n_ltg; ++g) {
    const double c = wave_total(signed_by(x0, T->ltg_a[g], cs.S));
    if (last_lane) {
      const double r = c - prev[kInner + g];
      prev[kInner + g] = c;
      const int e1 = T->ltg_start[g + 1];
      for (int e = T->ltg_start[g]; e < e1; ++e) acc[T->lt_pair[e]] += signed_by(x0, T->lt_bit[e], r);
    }
  }
  const int n_tt = T->n_tt;
  if (n_tt > 0) {
    const double c = wave_total(cs.S);
    if (last_lane) {
      const double r = c - prev[kInner + kLaneBits];
      prev[kInner + kLaneBits] = c;
      for (int e = 0; e < n_tt; ++e)
        acc[T->tt_pair[e]] += signed_by2(x0, T->tt_a[e], T->tt_b[e], r);
    }
  }
}

// At the end: pairs whose sign pattern is fixed per lane (x: the lane's
// lane-fixed bits in place, other prefix bits 0), one wave reduction each:
// tile-middle and middle-middle pairs from Q and M2, inner a - lane-fixed b
// from W s_a times s_b, lane-fixed pairs from W times s_a s_b.
template <int TJ>
__device__ inline void flush_end(const BondTables *__restrict__ T, const LaneSums<TJ> &cs, uint64_t x,
                                 double *acc, bool last_lane) {
#pragma unroll
  for (int m = 0; m < kBwMid; ++m)
#pragma unroll
    for (int i = 0; i < TJ; ++i) {
      const int p = T->qpair[m][i];
      if (p >= 0) {
        const double v = wave_total(cs.Q[m][i]);
        if (last_lane) acc[p] += v;
      }
    }
#pragma unroll
  for (int j = 0; j < 6; ++j) {
    const int p = T->m2pair[j];
    if (p >= 0) {
      const double v = wave_total(cs.M2[j]);
      if (last_lane) acc[p] += v;
    }
  }
#pragma unroll
  for (int a = 0; a < TJ + kBwMid; ++a) {
    const int e1 = T->il_start[a + 1];
    for (int e = T->il_start[a]; e < e1; ++e) {
      const double v = wave_total(signed_by(x, T->il_bit[e], cs.inner(a)));
      if (last_lane) acc[T->il_pair[e]] += v;
    }
  }
  const int n_ll = T->n_ll;
  for (int e = 0; e < n_ll; ++e) {
    const double v = wave_total(signed_by2(x, T->ll_a[e], T->ll_b[e], cs.S));
    if (last_lane) acc[T->ll_pair[e]] += v;
  }
}

template <int TJ, int NC>
__global__ __launch_bounds__(kBwWaves * kWave) void k_bond_backward(
    const DevPlan *__restrict__ P, const BondTables *__restrict__ T, const double *__restrict__ Wd,
    uint64_t n_chunks, uint64_t t_begin, uint64_t n_tasks, int mirror, double *__restrict__ partial) {
  // Tasks [t_begin, n_tasks).  With mirror set, the table holds
  // W(E, M) + W(E, -M) (column n_up plus column N - n_up), for a walk over the
  // half of the configurations whose top spin is up.
  // Static LDS (compile-time base): the weight table at offset 0, then the
  // per-wave pair accumulators.
  __shared__ __align__(16) double lds[kHistBytes / 8];
  const char *wt = reinterpret_cast<const char *>(lds);
  const int rw = T->rw, Wc = P->W, n_m = P->n_m;
  const int bins = P->n_ec * Wc;
  // Each bin's weight is read from global memory once (eight loads in flight
  // per thread) and written to its rw copies.
  constexpr int kFill = 8;
  for (int base = 0; base < bins; base += kFill * int(blockDim.x)) {
    double v[kFill];
#pragma unroll
    for (int j = 0; j < kFill; ++j) {
      const int bin = base + j * int(blockDim.x) + int(threadIdx.x);
      const int e_idx = bin / Wc, nu = bin - e_idx * Wc;
      const int E = P->e_base + e_idx * P->estep;
      const double *row = Wd + size_t(E - P->e_min) * n_m;
      v[j] = (bin < bins && nu < n_m) ? (mirror ? row[nu] + row[n_m - 1 - nu] : row[nu]) : 0.0;
    }
#pragma unroll
    for (int j = 0; j < kFill; ++j) {
      const int bin = base + j * int(blockDim.x) + int(threadIdx.x);
      if (bin < bins)
        for (int c = 0; c < rw; ++c) lds[bin * rw + c] = v[j];
    }
  }
  const int n_pairs = T->n_pairs;
  double *acc_all = lds + T->wt_bytes / 8;
  double *prev_all = acc_all + kBwWaves * n_pairs;
  for (int i = threadIdx.x; i < kBwWaves * (n_pairs + kPrevSlots); i += blockDim.x) acc_all[i] = 0.0;
  __syncthreads();
  const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
  const bool last_lane = lane == kWave - 1;
  double *acc = acc_all + wave * n_pairs;
  double *prev = prev_all + wave * kPrevSlots;
  SiteTable<NC> st;
  st.load(P, lane);
  const uint32_t rep_bytes = uint32_t(lane & (rw - 1)) * 8u;
  // A block has kBwWaves * kWave = 2^kLaneBits threads, so a thread's chunks
  // share their low kLaneBits bits (its offset).
  const uint32_t offset = T->lane_chunk[threadIdx.x];
  LaneSums<TJ> cs;
  cs.clear();
  for (uint64_t t = t_begin + blockIdx.x; t < n_tasks; t += gridDim.x) {
    const uint64_t chunk = (t << kLaneBits) + offset;
    const uint64_t x0 = chunk << st.k;
    if (chunk < n_chunks) bond_chunk<TJ, NC>(st, x0, rep_bytes, wt, cs);
    flush_task<TJ>(T, cs, x0, acc, prev, last_lane);
  }
  flush_end<TJ>(T, cs, uint64_t(offset) << st.k, acc, last_lane);
  __syncthreads();
  for (int p = threadIdx.x; p < n_pairs; p += blockDim.x) {
    double s = 0.0;
    for (int w = 0; w < kBwWaves; ++w) s += acc_all[w * n_pairs + p];
    partial[size_t(blockIdx.x) * n_pairs + p] = s;
  }
}

// dJ[b] = the sum over blocks of the partial sums of b's pair.  One block per
// pair: thread t adds the partials of blocks t, t + 256, ... in order, then a
// fixed tree over the threads, so the result does not depend on timing; the
// block then writes the total to every input bond of its pair.
constexpr int kFinishThreads = 256;

__global__ __launch_bounds__(kFinishThreads) void k_bond_finish(const BondTables *__restrict__ T,
                                                                const int32_t *__restrict__ pair_of_bond,
                                                                const double *__restrict__ partial, int blocks,
                                                                double *__restrict__ dJ) {
  __shared__ double sh[kFinishThreads];
  const int n_pairs = T->n_pairs, n_bonds = T->n_bonds;
  const int p = blockIdx.x;
  double s = 0.0;
  for (int k = threadIdx.x; k < blocks; k += kFinishThreads) s += partial[size_t(k) * n_pairs + p];
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int h = kFinishThreads / 2; h > 0; h >>= 1) {
    if (int(threadIdx.x) < h) sh[threadIdx.x] += sh[threadIdx.x + h];
    __syncthreads();
  }
  const double total = sh[0];
  for (int b = threadIdx.x; b < n_bonds; b += kFinishThreads)
    if (pair_of_bond[b] == p) dJ[b] = total;
}

// {DevPlan, BondTables, pair_of_bond} of the backward on `device`: uploaded
// on first use when `may_allocate`, else only looked up (null with
// ISING_EINVAL if not there yet).
static void *bond_device_tables(ising_plan *p, int device, bool may_allocate, ising_status *st) {
  *st = ISING_OK;
  if (device < 0 || device >= kMaxDevices) {
    *st = fail(ISING_EUNSUPPORTED, "device index out of range");
    return nullptr;
  }
  BondPlan *bp = p->bond;
  std::lock_guard<std::mutex> lk(p->mu);
  if (!bp->dev_copy[device] && !may_allocate) {
    *st = fail(ISING_EINVAL, "the plan's backward tables are not on device " + std::to_string(device) +
                                 " yet: one ising_bond_backward or ising_bond_backward_symmetric call there "
                                 "uploads them");
    return nullptr;
  }
  if (!bp->dev_copy[device]) {
    const size_t bytes = sizeof(DevPlan) + sizeof(BondTables) + bp->pair_of_bond.size() * sizeof(int32_t);
    std::vector<char> host(bytes);
    std::memcpy(host.data(), &bp->geo, sizeof(DevPlan));
    std::memcpy(host.data() + sizeof(DevPlan), &bp->tables, sizeof(BondTables));
    if (!bp->pair_of_bond.empty())
      std::memcpy(host.data() + sizeof(DevPlan) + sizeof(BondTables), bp->pair_of_bond.data(),
                  bp->pair_of_bond.size() * sizeof(int32_t));
    void *ptr = nullptr;
    hipError_t e = hipMalloc(&ptr, bytes);
    if (e != hipSuccess) {
      *st = fail(ISING_EHIP, std::string("hipMalloc(backward tables): ") + hipGetErrorString(e));
      return nullptr;
    }
    e = hipMemcpy(ptr, host.data(), bytes, hipMemcpyHostToDevice);
    if (e != hipSuccess) {
      (void)hipFree(ptr);
      *st = fail(ISING_EHIP, std::string("hipMemcpy(backward tables): ") + hipGetErrorString(e));
      return nullptr;
    }
    bp->dev_copy[device] = ptr;
  }
  return bp->dev_copy[device];
}

void bond_plan_free(BondPlan *b) {
  if (!b) return;
  for (int d = 0; d < kMaxDevices; ++d)
    if (b->dev_copy[d]) (void)hipFree(b->dev_copy[d]);
  delete b;
}

template <int TJ, int NC>
static ising_status launch_bond(const DevPlan *dP, const BondTables *dT, const double *W, uint64_t n_chunks,
                                uint64_t t_begin, uint64_t n_tasks, int mirror, int grid, double *partial,
                                hipStream_t s) {
  hipLaunchKernelGGL((k_bond_backward<TJ, NC>), dim3(grid), dim3(kBwWaves * kWave), 0, s, dP, dT, W, n_chunks,
                     t_begin, n_tasks, mirror, partial);
  HIP_TRY(hipGetLastError());
  return ISING_OK;
}

static ising_status bond_dispatch(int tile, int n_classes, const DevPlan *dP, const BondTables *dT, const double *W,
                                  uint64_t n_chunks, uint64_t t_begin, uint64_t n_tasks, int mirror, int grid,
                                  double *partial, hipStream_t s) {
#define ISING_BW_NC(TJ)                                                                                   \
  switch (n_classes) {                                                                                    \
    case 1: return launch_bond<TJ, 1>(dP, dT, W, n_chunks, t_begin, n_tasks, mirror, grid, partial, s);   \
    case 2: return launch_bond<TJ, 2>(dP, dT, W, n_chunks, t_begin, n_tasks, mirror, grid, partial, s);   \
    case 4: return launch_bond<TJ, 4>(dP, dT, W, n_chunks, t_begin, n_tasks, mirror, grid, partial, s);   \
    case 8: return launch_bond<TJ, 8>(dP, dT, W, n_chunks, t_begin, n_tasks, mirror, grid, partial, s);   \
  }                                                                                                       \
  break;
  switch (tile) {
    case 1: ISING_BW_NC(1)
    case 2: ISING_BW_NC(2)
    case 3: ISING_BW_NC(3)
    case 4: ISING_BW_NC(4)
    case 5: ISING_BW_NC(5)
    case 6: ISING_BW_NC(6)
    case 7: ISING_BW_NC(7)
    case 8: ISING_BW_NC(8)
  }
#undef ISING_BW_NC
  return fail(ISING_EUNSUPPORTED, "tile bits or class count out of range");
}

// One backward launch: device tables, work range and grid.
struct BondLaunch {
  const DevPlan *dP = nullptr;
  const BondTables *dT = nullptr;
  const int32_t *dmap = nullptr;
  uint64_t n_chunks = 0, t_begin = 0, n_tasks = 0;
  int grid = 0;
  bool mirror = false;
};

static ising_status bond_setup(const ising_plan *pc, bool halve, bool may_allocate, BondLaunch *L) {
  ising_plan *p = const_cast<ising_plan *>(pc);  // only the lazy device copy is written
  const BondPlan *bp = pc->bond;
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  ising_status st;
  char *tables = static_cast<char *>(bond_device_tables(p, dev, may_allocate, &st));
  if (!tables) return st;
  L->dP = reinterpret_cast<const DevPlan *>(tables);
  L->dT = reinterpret_cast<const BondTables *>(tables + sizeof(DevPlan));
  L->dmap = reinterpret_cast<const int32_t *>(tables + sizeof(DevPlan) + sizeof(BondTables));
  int cus = 0;
  HIP_TRY(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
  L->n_chunks = uint64_t(1) << (bp->geo.n - bp->geo.inner);
  static_assert(kBwWaves * kWave == 1 << kLaneBits, "a block walks 2^kLaneBits chunks per task");
  const uint64_t block = uint64_t(kBwWaves) * kWave;
  L->n_tasks = (L->n_chunks + block - 1) / block;
  // Halving needs the top spin to be a task bit (at least two tasks, both
  // powers of two): tasks [n_tasks/2, n_tasks) are the configurations with
  // it up.  Smaller lattices take the full walk, with the same result.
  L->mirror = halve && L->n_tasks >= 2;
  L->t_begin = L->mirror ? L->n_tasks / 2 : 0;
  L->grid = int(std::min<uint64_t>({L->n_tasks - L->t_begin, uint64_t(cus), uint64_t(kMaxBwBlocks)}));
  return ISING_OK;
}

static ising_status bond_launch(const ising_plan *pc, const BondLaunch &L, const double *W_dev, double *partial,
                                double *dJ_dev, hipStream_t s) {
  const BondPlan *bp = pc->bond;
  ising_status st = bond_dispatch(bp->geo.tile, bp->geo.n_classes, L.dP, L.dT, W_dev, L.n_chunks, L.t_begin,
                                  L.n_tasks, L.mirror ? 1 : 0, L.grid, partial, s);
  if (st != ISING_OK) return st;
  hipLaunchKernelGGL(k_bond_finish, dim3(unsigned(bp->tables.n_pairs)), dim3(kFinishThreads), 0, s, L.dT, L.dmap,
                     partial, L.grid, dJ_dev);
  HIP_TRY(hipGetLastError());
  return ISING_OK;
}

static ising_status bond_backward(const ising_plan *pc, const double *W_dev, double *dJ_dev, void *workspace,
                                  size_t workspace_bytes, bool halve, void *stream) {
  if (!pc) return fail(ISING_EINVAL, "plan is NULL");
  const BondPlan *bp = pc->bond;
  if (bp->status != ISING_OK) return fail(bp->status, bp->error);
  if (pc->n_bonds == 0) return ISING_OK;
  if (!W_dev || !dJ_dev || !workspace) return fail(ISING_EINVAL, "W_dev, dJ_dev or workspace is NULL");
  size_t need = 0;
  ising_status st = ising_bond_workspace(pc, &need);
  if (st != ISING_OK) return st;
  if (workspace_bytes < need)
    return fail(ISING_EINVAL, "workspace of " + std::to_string(workspace_bytes) + " bytes; " +
                                  std::to_string(need) + " needed");
  BondLaunch L;
  st = bond_setup(pc, halve, true, &L);
  if (st != ISING_OK) return st;
  return bond_launch(pc, L, W_dev, static_cast<double *>(workspace), dJ_dev, static_cast<hipStream_t>(stream));
}

// ---------------------------------------------------------------------------
// Allocation-free form: the per-block partial sums live in a static device
// array instead of a caller workspace.  Each device that runs it holds its
// own copy of the array until the process ends; calls on one device share
// it, so calls that overlap in time on one device race.  Every block writes
// all n_pairs entries of its row before the finishing kernel reads them, so
// nothing needs clearing between calls.
// ---------------------------------------------------------------------------

constexpr size_t kScratchDoubles = size_t(kMaxBwBlocks) * size_t(kMaxPairs);   // 4 MiB
static __device__ __align__(256) double scratch[kScratchDoubles];

static std::mutex g_scratch_mu;
static double *g_scratch[kMaxDevices];

// Device address of this device's copy of `scratch` (looked up once per
// device; the host-side name is only a stand-in for the symbol).
static ising_status scratch_on_device(int dev, double **out) {
  if (dev < 0 || dev >= kMaxDevices) return fail(ISING_EUNSUPPORTED, "device index out of range");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch[dev]) {
    void *ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
      return fail(ISING_EHIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    g_scratch[dev] = static_cast<double *>(ptr);
  }
  *out = g_scratch[dev];
  return ISING_OK;
}

static ising_status bond_backward_noalloc(const ising_plan *pc, const double *W_dev, double *dJ_dev, void *stream) {
  if (!pc) return fail(ISING_EINVAL, "plan is NULL");
  const BondPlan *bp = pc->bond;
  if (bp->status != ISING_OK) return fail(bp->status, bp->error);
  if (pc->n_bonds == 0) return ISING_OK;
  if (!W_dev || !dJ_dev) return fail(ISING_EINVAL, "W_dev or dJ_dev is NULL");
  BondLaunch L;
  ising_status st = bond_setup(pc, false, false, &L);
  if (st != ISING_OK) return st;
  const size_t need = size_t(L.grid) * size_t(bp->tables.n_pairs);
  if (need > kScratchDoubles)
    return fail(ISING_ERANGE, "partial sums of " + std::to_string(need) + " doubles exceed the " +
                                  std::to_string(kScratchDoubles) + " of the static scratch array");
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  double *partial = nullptr;
  st = scratch_on_device(dev, &partial);
  if (st != ISING_OK) return st;
  return bond_launch(pc, L, W_dev, partial, dJ_dev, static_cast<hipStream_t>(stream));
}

}  // namespace ising

using namespace ising;

extern "C" ising_status ising_bond_backward(const ising_plan *pc, const double *W_dev, double *dJ_dev,
                                            void *workspace, size_t workspace_bytes, void *stream) {
  return bond_backward(pc, W_dev, dJ_dev, workspace, workspace_bytes, false, stream);
}

extern "C" ising_status ising_bond_backward_symmetric(const ising_plan *pc, const double *W_dev, double *dJ_dev,
                                                      void *workspace, size_t workspace_bytes, void *stream) {
  return bond_backward(pc, W_dev, dJ_dev, workspace, workspace_bytes, true, stream);
}

extern "C" ising_status ising_bond_backward_noalloc(const ising_plan *pc, const double *W_dev, double *dJ_dev,
                                                    void *stream) {
  return bond_backward_noalloc(pc, W_dev, dJ_dev, stream);
}
