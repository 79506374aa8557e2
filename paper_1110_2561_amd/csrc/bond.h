// Per-bond backward plan: geometry and tables of the recomputed walk that sums
// W(E, M) s_i s_j per bond (bond.hip, bond_plan.cpp).
#pragma once

#include <stdint.h>

#include <string>
#include <vector>

#include "internal.h"

namespace ising {

constexpr int kMaxPairs = 512;      // distinct bond pairs the per-bond backward handles
constexpr int kBwMid = 2;           // middle bits of the backward walk (at most)
constexpr int kBwWaves = 16;        // waves per block of the backward kernel
constexpr int kMaxBwBlocks = 1024;  // blocks whose partial sums the workspace holds
constexpr int kBlockBits = 8;       // block bits when the lattice has them: 256 blocks, one per CU

constexpr int kLaneBits = 10;       // log2(kBwWaves * kWave): chunk-offset bits fixed for a thread
constexpr int kInner = kMaxTile + kBwMid;   // inner bits (tile + middle) at most
constexpr int kRound = 8;           // values per wave in one LDS round of the final reduction

// Where the spins sit in the backward walk (bit positions of the plan's
// order):
//   [0, TJ)              tile: an independent set, walked per block of 2^TJ
//                        configurations with constant address deltas;
//   [TJ, k = TJ + mj)    middle bits, walked between tile blocks;
//   [k, k + L)           offset bits: the thread's chunk offset (fixed per thread);
//   [k + L, k + L + s)   block bits: the block index (fixed per block);
//   [k + L + s, N)       hi bits: every block walks all their states in Gray
//                        order, one chunk per thread per state, so the next
//                        chunk differs from the last in a single spin.
// Each thread keeps running sums over all it has walked, from which W, W s_a
// for every inner bit a, W s_t s_m (tile-middle) and W s_m1 s_m2
// (middle-middle) follow.  A
// pair whose sign pattern never changes for a thread (both bits inner,
// offset or block bits) is read from them at the end.  A pair (a, p) with a
// hi bit p takes, by summation by parts over the walk, s_p(end) times the
// final running sum minus, at every flip of p, the change of s_p times the
// running sum at that moment: one wave reduction per partner of the flipped
// bit per chunk.
struct BondTables {
  int32_t n_pairs;       // distinct bond pairs
  int32_t mj;            // middle bits
  int32_t rw;            // copies of the FP64 weight table in LDS
  int32_t wt_bytes;      // LDS bytes of the weight table (all copies)
  int32_t n_bonds;       // input bonds (pair_of_bond entries after this struct)
  int32_t s_bits;        // block bits: the grid has 2^s_bits blocks
  int32_t n_hi;          // hi bits
  int32_t n_offsets;     // chunk offsets that exist: min(2^L, 2^(N - k))
  int32_t acc_bytes;     // LDS bytes of the per-wave pair accumulators (the table follows)
  int32_t n_end_outer;   // end pairs with no inner bit
  int16_t qpair[kBwMid][kMaxTile];          // tile t - middle m pair, or -1
  int16_t m2pair;                           // middle pair (0, 1), or -1
  int16_t pad0;
  // end pairs with an inner bit a and a non-inner bit b, by a: [end_start[a], end_start[a+1])
  int16_t end_start[kInner + 1];
  int16_t end_pair[kMaxPairs];
  uint8_t end_b[kMaxPairs];
  // end pairs of two non-inner bits
  int16_t eo_pair[kMaxPairs];
  uint8_t eo_a[kMaxPairs], eo_b[kMaxPairs];
  // pairs with hi bit j: inner partners by partner bit, others in a list
  int16_t hp_inner[kMaxSpins][kInner];      // pair of (inner a, hi bit j), or -1
  int16_t hp_start[kMaxSpins + 1];          // non-inner partners of hi bit j
  int16_t hp_pair[2 * kMaxPairs];           // (a pair of two hi bits is listed under both)
  uint8_t hp_a[2 * kMaxPairs];
  // byte change of the tile delta i when bit b (>= TJ) flips up
  int32_t kbit[kMaxSpins][kMaxTile];
  uint16_t lane_chunk[kBwWaves * kWave];    // thread -> chunk offset (a permutation)
};

// Host-side backward plan, owned by its ising_plan.
struct BondPlan {
  ising_status status = ISING_OK;   // ISING_EUNSUPPORTED when the backward cannot run
  std::string error;
  DevPlan geo{};                    // walk geometry: same bit order, k = tile + middle,
                                    // byte constants for the FP64 weight table
  BondTables tables{};
  std::vector<int32_t> pair_of_bond;
  void *dev_copy[kMaxDevices] = {}; // per device: {DevPlan, BondTables, pair_of_bond}
};

}  // namespace ising
