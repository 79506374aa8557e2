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

// Where each distinct bond pair of the lattice sits in the backward walk
// (bit positions of the backward geometry: tile [0, TJ), middle [TJ, TJ + mj),
// prefix above), and where its per-chunk sum comes from.
struct BondTables {
  int32_t n_pairs;       // distinct bond pairs
  int32_t mj;            // middle bits
  int32_t n_ip, n_pp;    // inner-prefix and prefix-prefix pairs
  int32_t rw;            // copies of the FP64 weight table in LDS
  int32_t wt_bytes;      // LDS bytes of the weight table (all copies)
  int32_t n_bonds;       // input bonds (pair_of_bond entries after this struct)
  int32_t pad;
  int16_t qpair[kBwMid][kMaxTile];          // tile t - middle m pair, or -1
  int16_t m2pair[6];                        // middle pairs (0,1) (0,2) (0,3) (1,2) (1,3) (2,3), or -1
  int16_t ip_start[kMaxTile + kBwMid + 1];  // inner bit a: entries [ip_start[a], ip_start[a+1])
  int16_t ip_pair[kMaxPairs];
  uint8_t ip_bit[kMaxPairs];                // prefix bit of the entry
  int16_t pp_pair[kMaxPairs];
  uint8_t pp_a[kMaxPairs], pp_b[kMaxPairs];
  uint16_t lane_chunk[kBwWaves * kWave];    // thread -> chunk offset within a task (a permutation)
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
