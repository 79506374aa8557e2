// Per-bond backward plan: geometry and tables of the recomputed walk that sums
// W(E, M) s_i s_j per bond (bond.hip, bond_plan.cpp).
#pragma once

#include <stdint.h>

#include <string>
#include <vector>

#include "internal.h"

namespace ising {

constexpr int kMaxPairs = 512;      // distinct bond pairs the per-bond backward handles
constexpr int kBwMid = 4;           // middle bits of the backward walk (at most)
constexpr int kBwWaves = 8;         // waves per block of the backward kernel
constexpr int kMaxBwBlocks = 1024;  // blocks whose partial sums the workspace holds

constexpr int kLaneBits = 9;        // log2(kBwWaves * kWave): chunk bits fixed for a thread
constexpr int kInner = kMaxTile + kBwMid;   // inner bits (tile + middle) at most

// Where each distinct bond pair of the lattice sits in the backward walk, by
// the kind of its two bits (bit positions of the backward geometry: tile
// [0, TJ), middle [TJ, k = TJ + mj), then the prefix, whose first kLaneBits
// bits are fixed for a thread ("lane-fixed", the chunk's offset in its task)
// and the rest are the same for the whole block in one task ("task" bits)).
// Per-lane running sums accumulate over all of a thread's chunks.  Pairs whose
// sign pattern is fixed per thread are reduced once at the end; pairs with a
// task bit are reduced per task, as differences of the cumulative wave sums.
struct BondTables {
  int32_t n_pairs;       // distinct bond pairs
  int32_t mj;            // middle bits
  int32_t rw;            // copies of the FP64 weight table in LDS
  int32_t wt_bytes;      // LDS bytes of the weight table (all copies)
  int32_t n_bonds;       // input bonds (pair_of_bond entries after this struct)
  int32_t n_ltg;         // lane-fixed bits with task-bit partners
  int32_t n_ll, n_tt;    // lane-fixed / lane-fixed and task / task pairs
  int16_t qpair[kBwMid][kMaxTile];          // tile t - middle m pair, or -1
  int16_t m2pair[6];                        // middle pairs (0,1) (0,2) (0,3) (1,2) (1,3) (2,3), or -1
  int16_t it_start[kInner + 1];             // inner a - task b, by a: [it_start[a], it_start[a+1])
  int16_t it_pair[kMaxPairs];
  uint8_t it_bit[kMaxPairs];
  int16_t il_start[kInner + 1];             // inner a - lane-fixed b, by a
  int16_t il_pair[kMaxPairs];
  uint8_t il_bit[kMaxPairs];
  uint8_t ltg_a[kLaneBits];                 // lane-fixed a - task b, grouped by a
  int16_t ltg_start[kLaneBits + 1];
  int16_t lt_pair[kMaxPairs];
  uint8_t lt_bit[kMaxPairs];
  int16_t ll_pair[kMaxPairs];               // lane-fixed a - lane-fixed b
  uint8_t ll_a[kMaxPairs], ll_b[kMaxPairs];
  int16_t tt_pair[kMaxPairs];               // task a - task b
  uint8_t tt_a[kMaxPairs], tt_b[kMaxPairs];
  uint16_t lane_chunk[kBwWaves * kWave];    // thread -> chunk offset within a task (a permutation)
};

// LDS doubles per wave for the previous cumulative wave sums of the per-task
// reductions: one per inner bit, per lane-fixed group, and for the total.
constexpr int kPrevSlots = kInner + kLaneBits + 1;

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
