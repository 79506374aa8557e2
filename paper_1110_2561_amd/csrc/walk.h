// Device-side pieces of the enumeration shared by the single-lattice and the
// batched kernels: the register-resident plan table, the Gray walk of one
// chunk and the LDS histogram flush.  See enumerate.hip for the design.
#pragma once

#include <hip/hip_runtime.h>

#include "internal.h"

namespace ising {

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
template <int NC>
struct SiteTable {
  uint32_t mlo[NC], mhi[NC];   // neighbour masks of the lane's site, per coupling class
  int32_t hdeg;                // sum_c J_c deg_c of the lane's site
  int32_t base;                // up_base of the lane's site
  int32_t kmid[kMaxTile];      // lane m: tile-delta changes when middle bit tile + m flips up
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
    const bool mid = lane < k - P->tile;
#pragma unroll
    for (int i = 0; i < kMaxTile; ++i) kmid[i] = mid ? P->kmid[mid ? lane : 0][i] : 0;
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

// LDS copy of each lane: lane mod R.  The LDS has 32 banks of 4 bytes and
// serves one half-wave per cycle; word bin * R + copy sits in bank
// (bin * R + copy) mod 32.  With 16 copies the two lanes of a half-wave that
// share a copy are one prefix spin apart, so their n_up, and with an even row
// stride their bank groups bin mod 2, differ: no conflicts.  With 8 copies
// four lanes share a copy and need four distinct bin mod 4; their n_up and
// energy-index parities cannot supply that for every copy (the lane keys
// (n_up + 2 e) mod 4 over a half-wave are never equally frequent), so such
// histograms pay one extra cycle per half-wave.
__device__ __forceinline__ uint32_t lane_copy(uint32_t lane, int R) {
  return lane & uint32_t(R - 1);
}

// First configuration of a chunk (prefix bits fixed, inner bits zero): its
// histogram byte address A = e_idx * row + n_up * col + extra, and the
// up-flip address change D_i of every tile spin (their neighbours are all
// outside the tile, so these stay fixed while only tile bits flip).
template <int TJ, int NC>
__device__ __forceinline__ void chunk_start(const SiteTable<NC> &st, uint64_t x0, uint32_t extra, uint32_t &A,
                                            int32_t (&D)[TJ]) {
  const uint32_t x0lo = uint32_t(x0), x0hi = uint32_t(x0 >> 32);
  // Full (E, n_up) of the first configuration: E = -(1/2) sum_i s_i h_i.
  int32_t hs = 0;
  for (int i = 0; i < st.n; ++i) {
    const int32_t h = st.field(i, x0lo, x0hi);
    hs += ((x0 >> i) & 1) ? h : -h;
  }
  const int32_t E0 = -(hs / 2);
  const int32_t nup = __popcll(x0);
  A = uint32_t(((E0 - st.e_base) / st.estep) * st.row_bytes + nup * st.col_bytes) + extra;
#pragma unroll
  for (int i = 0; i < TJ; ++i) D[i] = st.up_delta(i, x0lo, x0hi);
}

// Gray step q -> q+1 of the middle bits (between tile blocks): it flips bit
// TJ + ctz(q+1); move A by that spin's delta and the D_i of the tile spins
// coupled to it by the plan constants kmid.
template <int TJ, int NC>
__device__ __forceinline__ void middle_flip(const SiteTable<NC> &st, uint64_t x0, uint32_t q, uint32_t &A,
                                            int32_t (&D)[TJ]) {
  const uint32_t q1 = q + 1;
  const int mm = __builtin_ctz(q1);
  const bool up = (((q1 ^ (q1 >> 1)) >> mm) & 1u) != 0;
  // current inner bits: tile at its end state, middle bits = gray(q)
  const uint64_t x = x0 | ((q & 1) ? 0ull : (1ull << (TJ - 1))) | (uint64_t(q ^ (q >> 1)) << TJ);
  const int32_t dm = st.up_delta(TJ + mm, uint32_t(x), uint32_t(x >> 32));
  A = up ? A + uint32_t(dm) : A - uint32_t(dm);
#pragma unroll
  for (int i = 0; i < TJ; ++i) {
    const int32_t kv = __builtin_amdgcn_readlane(st.kmid[i], mm);
    D[i] = up ? D[i] + kv : D[i] - kv;
  }
}

// All 2^k configurations of one chunk (prefix bits fixed).
template <int TJ, int NC>
__device__ inline void walk_chunk(const SiteTable<NC> &st, uint64_t chunk, uint32_t rep, char *hist) {
  const uint64_t x0 = chunk << st.k;
  uint32_t A;
  int32_t D[TJ];
  chunk_start<TJ, NC>(st, x0, rep * 4u, A, D);
  const uint32_t nblk = 1u << (st.k - TJ);
  for (uint32_t q = 0; q < nblk; ++q) {
    if (q & 1)
      tile_walk<TJ, true>(A, D, hist);
    else
      tile_walk<TJ, false>(A, D, hist);
    if (q + 1 < nblk) middle_flip<TJ, NC>(st, x0, q, A, D);
  }
}

// Sum the R copies of every compact bin, clear them, add to the dense table.
__device__ inline void flush_hist(const DevPlan *__restrict__ P, uint32_t *h, unsigned long long *__restrict__ g) {
  const int W = P->W, R = P->R;
  const int bins = P->n_ec * W;
  // Lane b of a half-wave visits the copies of bin b starting at copy
  // (b mod 32) / (32 / R): the 32 words it touches at each step then lie in
  // 32 different banks (in copy order they would share 32 / R banks).
  const int rot = (int(threadIdx.x) & 31) / (32 / R);
  for (int b = threadIdx.x; b < bins; b += blockDim.x) {
    unsigned long long s = 0;
    for (int r = 0; r < R; ++r) {
      const int w = b * R + ((r + rot) & (R - 1));
      s += h[w];
      h[w] = 0;
    }
    const int e_idx = b / W, nu = b - e_idx * W;
    if (s && nu < P->n_m) {
      const int E = P->e_base + e_idx * P->estep;
      atomicAdd(&g[size_t(E - P->e_min) * P->n_m + nu], s);
    }
  }
}

}  // namespace ising
