// Library-internal definitions shared by the host plan code and the kernels.
#pragma once

#include <stdint.h>

#include <mutex>
#include <string>
#include <vector>

#include "../../include/ising.h"

namespace ising {

struct BondPlan;   // per-bond backward plan (bond.h)

constexpr int kMaxSpins = 64;
constexpr int kMaxClasses = 8;      // distinct nonzero merged couplings
constexpr int kMaxTile = 8;         // tile bits j (independent-set spins)
constexpr int kMaxInner = 25;       // inner bits k (configurations per chunk 2^k)
constexpr int kMaxMiddle = kMaxInner - 1;
constexpr int kLdsBytes = 160 * 1024;
constexpr int kHistBytes = kLdsBytes - 64;   // LDS histogram; the rest holds block control words
constexpr int kWave = 64;
constexpr int kMaxBlockThreads = 1024;
constexpr int kMaxDevices = 64;

// Constants one enumeration launch reads (uploaded once per device).
// Spin indices are plan bit positions: bits [0, tile) are the tile (an
// independent set), [tile, inner) the middle bits, [inner, n) the chunk
// prefix.
struct DevPlan {
  int32_t n;             // spins
  int32_t inner;         // k
  int32_t tile;          // j
  int32_t n_classes;     // distinct merged couplings, padded to 1, 2, 4 or 8
  int32_t estep;         // every E lies on e_base + estep * Z
  int32_t e_base;        // lowest compact energy (>= -S_eff)
  int32_t n_ec;          // compact energy rows
  int32_t W;             // compact row stride: least even W >= n + 1
  int32_t R;             // LDS replicas (power of two)
  int32_t e_min;         // dense table: e_min = -S
  int32_t n_m;           // dense table columns = n + 1
  int32_t pad0;
  int32_t class_J[kMaxClasses];
  // Histogram byte offset change when bit b flips up, in the state x:
  //   up_base[b] - sum_c cls_step[c] * popcount(x & mask[b][c]),
  // i.e. (-2 h_b / estep) * row + col with h_b = 2 sum_c J_c popc - hdeg[b].
  int32_t cls_step[kMaxClasses];            // (4 J_c / estep) * row bytes
  int32_t up_base[kMaxSpins];               // (2 hdeg[b] / estep) * row bytes + column bytes
  int32_t hdeg[kMaxSpins];                  // sum_c J_c * deg_c(b)
  int32_t kmid[kMaxMiddle][kMaxTile];       // byte change of tile delta i when middle bit m goes up
  uint64_t mask[kMaxSpins][kMaxClasses];    // neighbours of bit i with coupling class c
  // Thread t of a block walks chunk task * blockDim + lane_chunk[t] (a
  // permutation of the block's chunk offsets; see balance_lane_chunks).
  uint16_t lane_chunk[kMaxBlockThreads];
};

}  // namespace ising

struct ising_plan {
  // input as given
  int32_t n_spins = 0;
  int32_t n_bonds = 0;
  int64_t S = 0;                 // sum |J_b| over the input bonds
  // ordering and decomposition
  int32_t bit_of_site[ising::kMaxSpins] = {};
  int32_t site_of_bit[ising::kMaxSpins] = {};
  uint64_t n_chunks = 0;
  int32_t waves_per_block = 16;
  int32_t max_blocks = 0;
  int32_t blocks_per_cu = 1;
  int64_t n_merged_pairs = 0;
  ising::DevPlan dev{};
  // per-device constant copies (lazy)
  std::mutex mu;
  void *dev_copy[ising::kMaxDevices] = {};
  // per-bond backward (bond.h), built with the plan; null if its set-up failed
  ising::BondPlan *bond = nullptr;
};

namespace ising {

// One unit of batched work: task `task` (chunks task*block .. +block) of member
// `inst`; chunks whose offset in the task is below first_offset are skipped
// (the lower half of a one-task member in a halved run).
struct BatchUnit {
  int32_t inst;
  int32_t first_offset;
  uint64_t task;
};

// Per-member launch data of a batch.
struct BatchMember {
  uint64_t n_chunks;
  int64_t offset;        // first element of the member's table in g_all
  uint32_t flush_every;  // tasks between LDS flushes
  int32_t n_e, n_m, e_min, n_spins;
  int32_t pad;
};

void set_error(const std::string &msg);
// plan_create with every member forced to `min_classes` or more coupling classes
// exact_tile: tune.tile_bits must be met exactly (else it is an upper bound)
ising_status plan_create_internal(const ising_lattice *lat, const ising_tune *tune, int min_classes,
                                  ising_plan **out, bool exact_tile = true);
ising_status fail(ising_status st, const std::string &msg);
const void *plan_device_constants(ising_plan *plan, int device, ising_status *st);
// Thread -> chunk-offset permutation of a block of `threads` (a multiple of
// 32) for histograms or tables kept in 8 interleaved LDS copies (copy = lane
// mod 8) with a row stride that is a multiple of 4 (plan.cpp).
void balance_lane_chunks(uint16_t *lane_chunk, int threads);
// per-bond backward plan of a finished forward plan (bond_plan.cpp); J is the
// merged n x n coupling matrix, classes the distinct merged couplings
BondPlan *bond_plan_create(const ising_plan *p, const ising_lattice *lat, const std::vector<int64_t> &J,
                           const std::vector<int64_t> &classes);
void bond_plan_free(BondPlan *b);   // frees its device copies too (bond.hip)
}  // namespace ising

struct ising_batch_plan {
  int32_t n = 0;
  int32_t n_classes = 0;
  int32_t waves_per_block = 16;
  int32_t max_blocks = 0;
  std::vector<ising_plan *> members;      // owned
  std::vector<ising::BatchMember> meta;
  std::vector<ising::BatchUnit> units;
  std::vector<ising::BatchUnit> units_half;   // halved run: chunks with the top spin up
  int64_t total_elems = 0;
  std::mutex mu;
  struct Dev {
    void *plans = nullptr;    // DevPlan[n]
    void *meta = nullptr;     // BatchMember[n]
    void *units = nullptr;    // BatchUnit[units]
    void *units_half = nullptr;  // BatchUnit[units_half]
    void *counter = nullptr;  // uint32 work counter
  } dev[ising::kMaxDevices];
};
