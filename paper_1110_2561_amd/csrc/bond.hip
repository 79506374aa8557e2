// Per-bond backward of log Z: dJ_b = sum over all 2^N configurations of
// W(E, M) s_i s_j, for a per-bin weight table W (k_bin_weights in
// thermo.hip makes W from a loss gradient).  Eq. (1) of Peretyatko et al.
// (Section 2) makes H depend on J_b only through -J_b s_i s_j, so
// d log Z / dJ_b = <s_i s_j> / T needs, besides g(E, M), the bond spin
// product of every configuration; the enumeration is recomputed here in the
// same Gray order as the forward walk, with FP64 sums in place of counts.
//
// Bit layout (bond.h): tile, middle, offset (fixed per thread), block (fixed
// per block) and hi bits.  A thread walks one chunk (tile + middle) per state
// of the hi bits, which every block visits in Gray order, so the next chunk's
// first configuration differs from the last one's in one middle or tile spin
// (back to the chunk's start) and one hi spin: two incremental flips instead
// of a fresh set-up.
//   * the tile walk (2^TJ configurations, only tile bits flip, fully
//     unrolled) reads W of each configuration from an LDS copy of the table
//     (one ds_read_b64 on the same running address as the forward's
//     histogram add).  The sums of W over the configurations with tile spin
//     i up come from groups of 4 configurations: tile bits 0-1 are up on
//     fixed positions of a group, so their sums are nodes of the group's add
//     tree; higher tile bits, which flip only between groups, use a
//     prefix-sum trick on the running sum of group totals.  Which spin
//     flips, and which way, is a compile-time fact of the unrolled Gray
//     sequence, so a configuration costs one load, one integer add and two
//     FP64 adds.
//   * after each tile block the block's sums are folded into the thread's
//     running sums of W over the configurations with given inner spins up
//     (none; tile spin t; middle spin m; m and t; both middle spins), from
//     which W s_a, W s_t s_m and W s_m1 s_m2 follow when they are read.
//   * pairs whose sign pattern is fixed for a thread are read from the
//     running sums at the end; a pair with a hi bit p also gets, at every
//     flip of p, -(change of s_p) times the running sums at that moment
//     (summation by parts over the walk), one wave reduction (DPP tree) per
//     partner of the flipped bit.  The final reduction goes through LDS in
//     rounds of 8 values per wave.  Per-wave accumulators in LDS, per-block
//     partial sums, and a second kernel that adds the blocks in a fixed order
//     and scatters the totals to the input bonds: every sum runs in a fixed
//     order, so results are reproducible.
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

// Tile state at step t of a block of 2^TJ configurations.  Odd blocks start
// with the top tile bit set (reflected Gray code), so the state is
// gray(t) ^ (ODD ? top : 0).
template <int TJ, bool ODD>
__host__ __device__ constexpr uint32_t tile_state(int t) {
  return uint32_t(t ^ (t >> 1)) ^ (ODD ? (1u << (TJ - 1)) : 0u);
}

// Sum of W over the configurations of group g (4 configurations) with tile
// bit b up, from the group's add tree (pairs P01, P23, total G).
template <int TJ, bool ODD>
__device__ __forceinline__ double group_bit_sum(int g, int b, const double (&w)[4], double P01, double P23,
                                                double G) {
  uint32_t mask = 0;
#pragma unroll
  for (int u = 0; u < 4; ++u) mask |= ((tile_state<TJ, ODD>(4 * g + u) >> b) & 1u) << u;
  switch (mask) {
    case 0x6: return w[1] + w[2];
    case 0x9: return w[0] + w[3];
    case 0xc: return P23;
    case 0x3: return P01;
    case 0xf: return G;
    case 0x0: return 0.0;
    default: {   // not reached for the reflected Gray code; kept general
      double acc = 0.0;
#pragma unroll
      for (int u = 0; u < 4; ++u)
        if ((mask >> u) & 1u) acc += w[u];
      return acc;
    }
  }
}

// One tile block of 2^TJ configurations: sw = sum of W, U[i] = sum of W over
// the configurations with tile spin i up.
template <int TJ, bool ODD>
__device__ __forceinline__ void weight_walk(uint32_t &A, const int32_t (&D)[TJ], const char *wt, double &sw,
                                            double (&U)[TJ]) {
  constexpr int kN = 1 << TJ;
  constexpr uint32_t kEnd = tile_state<TJ, ODD>(kN - 1);
  if constexpr (TJ >= 3) {
    // Each sum starts as its first term (no add of 0.0, which IEEE rules
    // keep as an instruction since -0.0 + 0.0 is +0.0): the group-0 sums, and
    // for a bit >= 2 the running total at its first flip.
    constexpr int kGroups = kN / 4;
#pragma unroll
    for (int g = 0; g < kGroups; ++g) {
      double v[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int t = g * 4 + u;
        if (t > 0) {
          const int b = __builtin_ctz(t);
          A = ((tile_state<TJ, ODD>(t) >> b) & 1u) ? A + uint32_t(D[b]) : A - uint32_t(D[b]);
        }
        v[u] = lds_f64(wt, A);
      }
      if (g > 0) {   // a tile bit >= 2 flipped on entering this group
        const int b = __builtin_ctz(g * 4);
        const bool up = ((tile_state<TJ, ODD>(g * 4) >> b) & 1u) != 0;
        if (g == (1 << (b - 2)))
          U[b] = up ? -sw : sw;
        else
          U[b] = up ? U[b] - sw : U[b] + sw;
      }
      const double P01 = v[0] + v[1], P23 = v[2] + v[3], G = P01 + P23;
#pragma unroll
      for (int b = 0; b < 2; ++b) {
        const double gs = group_bit_sum<TJ, ODD>(g, b, v, P01, P23, G);
        U[b] = g == 0 ? gs : U[b] + gs;
      }
      sw = g == 0 ? G : sw + G;
    }
#pragma unroll
    for (int i = 2; i < TJ; ++i)
      if ((kEnd >> i) & 1u) U[i] += sw;
  } else {
    // one or two tile bits: the prefix-sum trick per configuration
#pragma unroll
    for (int i = 0; i < TJ; ++i) U[i] = 0.0;
    sw = 0.0;
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

// Running sums of one thread over all the configurations it has walked,
// kept over the configurations with given spins up (what a tile block yields,
// and the middle spins are up for whole blocks), so folding a block costs one
// add per sum it touches.  With s = 2 [s up] - 1, the signed sums follow when
// they are read:
//   W s_a        = 2 W[a] - W,
//   W s_a s_b    = 4 W[a][b] - 2 W[a] - 2 W[b] + W,
// where W[a] is the sum over the configurations with spin a up.
template <int TJ>
struct LaneSums {
  double S;                 // W
  double Yu[TJ];            // W [t up], tile spins
  double Zm[kBwMid];        // W [m up], middle spins
  double Qb[kBwMid][TJ];    // W [m up][t up]
  double M2b;               // W [m0 up][m1 up]

  __device__ __forceinline__ void clear() {
    S = 0.0;
    M2b = 0.0;
#pragma unroll
    for (int i = 0; i < TJ; ++i) Yu[i] = 0.0;
#pragma unroll
    for (int m = 0; m < kBwMid; ++m) {
      Zm[m] = 0.0;
#pragma unroll
      for (int i = 0; i < TJ; ++i) Qb[m][i] = 0.0;
    }
  }

  // W s_a for inner bit a (tile, then middle); a is a compile-time index
  __device__ __forceinline__ double inner(int a) const {
    return fma(2.0, a < TJ ? Yu[a < TJ ? a : 0] : Zm[a < TJ ? 0 : a - TJ], -S);
  }
  // W s_m s_t for middle bit m and tile bit i
  __device__ __forceinline__ double tile_middle(int m, int i) const {
    return fma(4.0, Qb[m][i], fma(-2.0, Yu[i] + Zm[m], S));
  }
  // W s_m0 s_m1
  __device__ __forceinline__ double middle_pair() const { return fma(4.0, M2b, fma(-2.0, Zm[0] + Zm[1], S)); }
};

// Flip bit b (>= TJ) of state x (its own value in x does not matter: the
// masks exclude it): move A by the bit's delta and the tile deltas D_i by
// the plan constants kbit.  b is wave-uniform, so the plan constants come in
// by scalar loads (flips happen between tile blocks, where waiting for them
// costs nothing) and hold no vector registers during the walk.
template <int TJ, int NC>
__device__ __forceinline__ void flip_bit(const DevPlan *__restrict__ P, const BondTables *__restrict__ T,
                                         uint64_t x, int b, bool up, uint32_t &A, int32_t (&D)[TJ]) {
  int32_t dm = P->up_base[b];
#pragma unroll
  for (int c = 0; c < NC; ++c) dm -= P->cls_step[c] * int32_t(__popcll(x & P->mask[b][c]));
  A = up ? A + uint32_t(dm) : A - uint32_t(dm);
#pragma unroll
  for (int i = 0; i < TJ; ++i) {
    const int32_t kv = T->kbit[b][i];
    D[i] = up ? D[i] + kv : D[i] - kv;
  }
}

// All 2^k configurations of the chunk whose prefix is x0 (inner bits zero on
// entry, with A and D those of x0).  On return the inner state is bit k - 1
// alone (the reflected Gray code's last word), with A and D to match.
template <int TJ, int NC>
__device__ inline void bond_chunk(const DevPlan *__restrict__ P, const BondTables *__restrict__ T, uint64_t x0,
                                  int mj, const char *wt, uint32_t &A, int32_t (&D)[TJ], LaneSums<TJ> &cs) {
  const uint32_t nblk = 1u << mj;
  for (uint32_t q = 0; q < nblk; ++q) {
    double sw, U[TJ];
    if (q & 1)
      weight_walk<TJ, true>(A, D, wt, sw, U);
    else
      weight_walk<TJ, false>(A, D, wt, sw, U);
    // middle spins during block q: bits of gray(q) (slots beyond mj stay
    // down and are never consulted); the block's sums go into the sums of
    // the middle spins that are up
    const uint32_t mid = q ^ (q >> 1);
    cs.S += sw;
#pragma unroll
    for (int i = 0; i < TJ; ++i) cs.Yu[i] += U[i];
#pragma unroll
    for (int m = 0; m < kBwMid; ++m)
      if ((mid >> m) & 1u) {
        cs.Zm[m] += sw;
#pragma unroll
        for (int i = 0; i < TJ; ++i) cs.Qb[m][i] += U[i];
      }
    if (mid == 3u) cs.M2b += sw;
    if (q + 1 < nblk) {
      // Gray step q -> q + 1 of the middle bits: flips bit TJ + ctz(q + 1);
      // the tile is at its end state (top bit set after an even block)
      const uint32_t q1 = q + 1;
      const int mm = __builtin_ctz(q1);
      const bool up = (((q1 ^ (q1 >> 1)) >> mm) & 1u) != 0;
      const uint64_t x = x0 | ((q & 1) ? 0ull : (1ull << (TJ - 1))) | (uint64_t(mid) << TJ);
      flip_bit<TJ, NC>(P, T, x, TJ + mm, up, A, D);
    }
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

// At a flip of hi bit j (bit p, new sign s_p): every pair (a, p) gets
// -(s_p(new) - s_p(old)) = -2 s_p(new) times the wave's running sum of
// W s_a (inner a) or of W s_a over the state x before the flip (other a).
// Bits from `uniform` up (block and hi bits) are the same in every lane of
// the block, so for such a the wave sum is s_a times the wave's sum of W,
// taken once per flip.
template <int TJ>
__device__ inline void flush_flip(const BondTables *__restrict__ T, const LaneSums<TJ> &cs, uint64_t x, int j,
                                  bool up, int uniform, double *acc, bool last_lane) {
  const double c = up ? -2.0 : 2.0;
#pragma unroll
  for (int a = 0; a < TJ + kBwMid; ++a) {
    const int pr = T->hp_inner[j][a];
    if (pr >= 0) {
      const double v = wave_total(cs.inner(a));
      if (last_lane) acc[pr] += c * v;
    }
  }
  const int e1 = T->hp_start[j + 1];
  bool have_total = false;
  double total = 0.0;
  for (int e = T->hp_start[j]; e < e1; ++e) {
    const int a = T->hp_a[e];
    double v;
    if (a >= uniform) {
      if (!have_total) {
        total = wave_total(cs.S);
        have_total = true;
      }
      v = signed_by(x, a, total);
    } else {
      v = wave_total(signed_by(x, a, cs.S));
    }
    if (last_lane) acc[T->hp_pair[e]] += c * v;
  }
}

// Final reduction of per-lane values through LDS, one wave at a time: the
// wave stores up to kRound values of its 64 lanes (value c of lane s at slot
// 64 c + s), then lane 8 v + u adds value v of lanes 8 u .. 8 u + 7, reading
// them in the rotated order 8 u + ((r + u + v) mod 8), r = 0..7, so that the
// 32 lanes a cycle serves read 32 different banks; a DPP tree over the 8
// lanes of a group (row_shr 1, 2, 4: a group never straddles a row of 16)
// leaves value v's total in lane 8 v + 7, which adds it to the pair's
// accumulator.  Only the wave's own slots are used, so wave-scope fences
// order the writes and reads (no block barrier).
struct EndRounds {
  double *buf;     // this wave's kRound x 64 doubles
  int *ids;        // this wave's kRound pair ids
  double *acc;     // this wave's pair accumulators
  int lane;
  int cnt = 0;

  __device__ void push(double v, int pair) {
    buf[cnt * kWave + lane] = v;
    if (lane == 0) ids[cnt] = pair;
    if (++cnt == kRound) flush();
  }

  __device__ void flush() {
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
    const int v = lane >> 3, u = lane & 7;
    double s = 0.0;
    if (v < cnt)
#pragma unroll
      for (int r = 0; r < 8; ++r) s += buf[v * kWave + u * 8 + ((r + u + v) & 7)];
    s += dpp_f64<0x111, 0xf, true>(s);   // row_shr:1
    s += dpp_f64<0x112, 0xf, true>(s);   // row_shr:2
    s += dpp_f64<0x114, 0xf, true>(s);   // row_shr:4
    if (u == 7 && v < cnt) acc[ids[v]] += s;
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
    cnt = 0;
  }
};

// At the end: every pair with a non-inner bit (its sign pattern for the
// final state x of the thread) and the tile-middle and middle-middle pairs.
template <int TJ>
__device__ inline void flush_end(const BondTables *__restrict__ T, const LaneSums<TJ> &cs, uint64_t x,
                                 EndRounds &R) {
#pragma unroll
  for (int m = 0; m < kBwMid; ++m)
#pragma unroll
    for (int i = 0; i < TJ; ++i) {
      const int p = T->qpair[m][i];
      if (p >= 0) R.push(cs.tile_middle(m, i), p);
    }
  if (T->m2pair >= 0) R.push(cs.middle_pair(), T->m2pair);
#pragma unroll
  for (int a = 0; a < TJ + kBwMid; ++a) {
    const int e1 = T->end_start[a + 1];
    for (int e = T->end_start[a]; e < e1; ++e) R.push(signed_by(x, T->end_b[e], cs.inner(a)), T->end_pair[e]);
  }
  const int n_eo = T->n_end_outer;
  for (int e = 0; e < n_eo; ++e)
    R.push(signed_by(x, T->eo_b[e], signed_by(x, T->eo_a[e], cs.S)), T->eo_pair[e]);
  if (R.cnt > 0) R.flush();
}

template <int TJ, int NC>
__global__ __launch_bounds__(kBwWaves * kWave) void k_bond_backward(
    const DevPlan *__restrict__ P, const BondTables *__restrict__ T, const double *__restrict__ Wd,
    int n_walk, uint64_t hi_init, int mirror, double *__restrict__ partial) {
  // The hi bits walk 2^n_walk states in Gray order from hi_init (with mirror
  // set, the top hi bit stays up and the table holds W(E, M) + W(E, -M):
  // column n_up plus column N - n_up, for the half of the configurations
  // whose top spin is up).
  // Static LDS (compile-time base): the per-wave pair accumulators at offset
  // 0, then the weight table; the final reduction reuses the table's space.
  __shared__ __align__(16) double lds[kHistBytes / 8];
  const int n_pairs = T->n_pairs;
  const int acc_bytes = T->acc_bytes;
  const char *wt = reinterpret_cast<const char *>(lds);
  double *tbl = lds + acc_bytes / 8;
  const int rw = T->rw, Wc = P->W, n_m = P->n_m;
  const int bins = P->n_ec * Wc;
  // Each bin's weight is read from global memory once (four loads in flight
  // per thread) and written to its rw copies.
  constexpr int kFill = 4;
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
        for (int c = 0; c < rw; ++c) tbl[bin * rw + c] = v[j];
    }
  }
  for (int i = threadIdx.x; i < kBwWaves * n_pairs; i += blockDim.x) lds[i] = 0.0;
  __syncthreads();
  const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
  const bool last_lane = lane == kWave - 1;
  double *acc = lds + wave * n_pairs;
  const int k = P->inner, mj = T->mj;
  const int hi0 = k + kLaneBits + T->s_bits;
  const uint32_t offset = T->lane_chunk[threadIdx.x];
  const bool active = int(offset) < T->n_offsets;
  // first configuration: the thread's offset, the block's index, the hi start
  uint64_t x = (uint64_t(offset) << k) | (uint64_t(blockIdx.x) << (k + kLaneBits));
  if (T->n_hi > 0) x |= hi_init << hi0;
  const uint32_t extra = uint32_t(acc_bytes) + uint32_t(lane & (rw - 1)) * 8u;   // table base + copy
  uint32_t A = 0;
  int32_t D[TJ];
#pragma unroll
  for (int i = 0; i < TJ; ++i) D[i] = 0;
  {
    SiteTable<NC> st;   // only for the set-up: flips read the plan by scalar loads
    st.load(P, lane);
    if (active) chunk_start<TJ, NC>(st, x, extra, A, D);
  }
  LaneSums<TJ> cs;
  cs.clear();
  const uint64_t steps = uint64_t(1) << n_walk;
  for (uint64_t t = 0;; ++t) {
    if (active) bond_chunk<TJ, NC>(P, T, x, mj, wt, A, D, cs);
    if (t + 1 == steps) break;
    const int j = __builtin_ctzll(t + 1), p = hi0 + j;
    const bool up = ((x >> p) & 1u) == 0;
    flush_flip<TJ>(T, cs, x, j, up, k + kLaneBits, acc, last_lane);
    if (active) {
      // back to the chunk's start (bit k - 1 down), then flip hi bit p
      if (mj > 0)
        flip_bit<TJ, NC>(P, T, x | (uint64_t(1) << (k - 1)), k - 1, false, A, D);
      else
        A -= uint32_t(D[TJ - 1]);
      flip_bit<TJ, NC>(P, T, x, p, up, A, D);
    }
    x ^= uint64_t(1) << p;
  }
  // final pair terms through LDS rounds over the (now unused) weight table:
  // per wave kRound x 64 values, then kRound pair ids
  __syncthreads();
  int *round_ids = reinterpret_cast<int *>(tbl + kBwWaves * kRound * kWave);
  EndRounds R{tbl + size_t(wave) * kRound * kWave, round_ids + wave * kRound, acc, lane};
  flush_end<TJ>(T, cs, x, R);
  __syncthreads();
  for (int pr = threadIdx.x; pr < n_pairs; pr += blockDim.x) {
    double s = 0.0;
    for (int w = 0; w < kBwWaves; ++w) s += lds[w * n_pairs + pr];
    partial[size_t(blockIdx.x) * n_pairs + pr] = s;
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
static ising_status launch_bond(const DevPlan *dP, const BondTables *dT, const double *W, int n_walk,
                                uint64_t hi_init, int mirror, int grid, double *partial, hipStream_t s) {
  hipLaunchKernelGGL((k_bond_backward<TJ, NC>), dim3(grid), dim3(kBwWaves * kWave), 0, s, dP, dT, W, n_walk,
                     hi_init, mirror, partial);
  HIP_TRY(hipGetLastError());
  return ISING_OK;
}

static ising_status bond_dispatch(int tile, int n_classes, const DevPlan *dP, const BondTables *dT, const double *W,
                                  int n_walk, uint64_t hi_init, int mirror, int grid, double *partial,
                                  hipStream_t s) {
#define ISING_BW_NC(TJ)                                                                                   \
  switch (n_classes) {                                                                                    \
    case 1: return launch_bond<TJ, 1>(dP, dT, W, n_walk, hi_init, mirror, grid, partial, s);             \
    case 2: return launch_bond<TJ, 2>(dP, dT, W, n_walk, hi_init, mirror, grid, partial, s);             \
    case 4: return launch_bond<TJ, 4>(dP, dT, W, n_walk, hi_init, mirror, grid, partial, s);             \
    case 8: return launch_bond<TJ, 8>(dP, dT, W, n_walk, hi_init, mirror, grid, partial, s);             \
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

// One backward launch: device tables, the hi-bit walk and the grid.
struct BondLaunch {
  const DevPlan *dP = nullptr;
  const BondTables *dT = nullptr;
  const int32_t *dmap = nullptr;
  int n_walk = 0;          // hi bits walked in Gray order
  uint64_t hi_init = 0;    // their first state
  int grid = 0;            // 2^s_bits blocks
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
  static_assert(kBwWaves * kWave == 1 << kLaneBits, "a block has 2^kLaneBits threads, one chunk offset each");
  const int n_hi = bp->tables.n_hi;
  // Halving needs the top spin to be a hi bit: it stays up, the other hi
  // bits are walked.  Lattices without hi bits take the full walk, with the
  // same result.
  L->mirror = halve && n_hi >= 1;
  L->n_walk = L->mirror ? n_hi - 1 : n_hi;
  L->hi_init = L->mirror ? uint64_t(1) << (n_hi - 1) : 0;
  L->grid = 1 << bp->tables.s_bits;
  if (L->grid > kMaxBwBlocks) return fail(ISING_EUNSUPPORTED, "internal: backward grid too large");
  return ISING_OK;
}

static ising_status bond_launch(const ising_plan *pc, const BondLaunch &L, const double *W_dev, double *partial,
                                double *dJ_dev, hipStream_t s) {
  const BondPlan *bp = pc->bond;
  ising_status st = bond_dispatch(bp->geo.tile, bp->geo.n_classes, L.dP, L.dT, W_dev, L.n_walk, L.hi_init,
                                  L.mirror ? 1 : 0, L.grid, partial, s);
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

// thermo.hip
ising_status first_derivatives_launch(const uint64_t *g, int32_t n_e, int32_t n_m, int32_t e_min, int32_t n_spins,
                                      const double *T_dev, int32_t nT, const double *h_dev, int32_t nh,
                                      const double *logz, double *d_T, double *d_h, hipStream_t stream);
ising_status grid_contract_launch(const double *G, const double *d_T, const double *d_h, int nT, int nh,
                                  double *grad_T, double *grad_h, hipStream_t stream);
ising_status bin_weights_launch(const uint64_t *g, int32_t n_e, int32_t n_m, int32_t e_min, int32_t n_spins,
                                const double *T_dev, int32_t nT, const double *h_dev, int32_t nh,
                                const double *logz, const double *G, double *W, double *scratch,
                                hipStream_t stream);
size_t bin_weights_scratch_bytes(int32_t nT, int32_t n_m);

__global__ void k_zero_f64(double *p, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0.0;
}

static ising_status zero_f64(double *p, int n, hipStream_t s) {
  if (!p || n <= 0) return ISING_OK;
  hipLaunchKernelGGL(k_zero_f64, dim3(unsigned((n + 255) / 256)), dim3(256), 0, s, p, n);
  HIP_TRY(hipGetLastError());
  return ISING_OK;
}

// Workspace layout of ising_logz_backward: d_T and d_h on the grid, the bin
// weights, then the per-bond backward's partial sums, each 256-byte aligned.
struct BackwardLayout {
  size_t d_T = 0, d_h = 0, W = 0, wscratch = 0, bond = 0, total = 0;
};

static size_t align256(size_t b) { return (b + 255) & ~size_t(255); }

static ising_status backward_layout(const ising_plan *p, int32_t nT, int32_t nh, bool want_th, bool want_J,
                                    BackwardLayout *L) {
  if (nT < 0 || nh < 0 || int64_t(nT) * nh > (int64_t(1) << 30)) return fail(ISING_EINVAL, "bad grid size");
  const size_t pts = size_t(nT) * size_t(nh) * sizeof(double);
  const size_t tbl = size_t(2 * p->S + 1) * size_t(p->n_spins + 1) * sizeof(double);
  size_t at = 0;
  if (want_th) {
    L->d_T = at;
    at += align256(pts);
    L->d_h = at;
    at += align256(pts);
  }
  if (want_J) {
    size_t bw = 0;
    ising_status st = ising_bond_workspace(p, &bw);
    if (st != ISING_OK) return st;
    L->W = at;
    at += align256(tbl);
    L->wscratch = at;
    at += align256(bin_weights_scratch_bytes(nT, p->n_spins + 1));
    L->bond = at;
    at += align256(bw);
  }
  L->total = std::max<size_t>(at, 256);
  return ISING_OK;
}

}  // namespace ising

using namespace ising;

extern "C" ising_status ising_logz_backward_workspace(const ising_plan *p, int32_t nT, int32_t nh, size_t *bytes) {
  if (!p || !bytes) return fail(ISING_EINVAL, "plan or bytes is NULL");
  BackwardLayout L;
  ising_status st = backward_layout(p, nT, nh, true, p->n_bonds > 0, &L);
  if (st != ISING_OK) return st;
  *bytes = L.total;
  return ISING_OK;
}

extern "C" ising_status ising_logz_backward(const ising_plan *p, const uint64_t *g_dev, const double *T_dev,
                                            int32_t nT, const double *h_dev, int32_t nh, const double *logz_dev,
                                            const double *G_dev, double *grad_T, double *grad_h, double *grad_J,
                                            int32_t symmetric, void *workspace, size_t workspace_bytes,
                                            void *stream) {
  if (!p || !g_dev) return fail(ISING_EINVAL, "plan or g_dev is NULL");
  const bool want_th = grad_T || grad_h;
  const bool want_J = grad_J && p->n_bonds > 0;
  if (!want_th && !want_J) return ISING_OK;
  if (nT < 0 || nh < 0) return fail(ISING_EINVAL, "negative grid size");
  if (nT == 0 || nh == 0) {   // an empty grid: every gradient is zero (a fill kernel, no memset node)
    hipStream_t s = static_cast<hipStream_t>(stream);
    ising_status st = zero_f64(grad_T, nT, s);
    if (st == ISING_OK) st = zero_f64(grad_h, nh, s);
    if (st == ISING_OK && want_J) st = zero_f64(grad_J, p->n_bonds, s);
    return st;
  }
  if (!T_dev || !h_dev || !logz_dev || !G_dev || !workspace)
    return fail(ISING_EINVAL, "T_dev, h_dev, logz_dev, G_dev or workspace is NULL");
  BackwardLayout L;
  ising_status st = backward_layout(p, nT, nh, want_th, want_J, &L);
  if (st != ISING_OK) return st;
  if (workspace_bytes < L.total)
    return fail(ISING_EINVAL, "workspace of " + std::to_string(workspace_bytes) + " bytes; " +
                                  std::to_string(L.total) + " needed");
  char *ws = static_cast<char *>(workspace);
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int32_t n_e = int32_t(2 * p->S + 1), n_m = p->n_spins + 1, e_min = int32_t(-p->S);
  if (want_th) {
    double *dT = reinterpret_cast<double *>(ws + L.d_T), *dh = reinterpret_cast<double *>(ws + L.d_h);
    st = first_derivatives_launch(g_dev, n_e, n_m, e_min, p->n_spins, T_dev, nT, h_dev, nh, logz_dev, dT, dh, s);
    if (st != ISING_OK) return st;
    st = grid_contract_launch(G_dev, dT, dh, nT, nh, grad_T, grad_h, s);
    if (st != ISING_OK) return st;
  }
  if (want_J) {
    double *W = reinterpret_cast<double *>(ws + L.W);
    st = bin_weights_launch(g_dev, n_e, n_m, e_min, p->n_spins, T_dev, nT, h_dev, nh, logz_dev, G_dev, W,
                            reinterpret_cast<double *>(ws + L.wscratch), s);
    if (st != ISING_OK) return st;
    size_t bw = 0;
    st = ising_bond_workspace(p, &bw);
    if (st != ISING_OK) return st;
    st = bond_backward(p, W, grad_J, ws + L.bond, bw, symmetric != 0, stream);
    if (st != ISING_OK) return st;
  }
  return ISING_OK;
}

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
