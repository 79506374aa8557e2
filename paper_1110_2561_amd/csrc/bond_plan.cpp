// Host-side planning of the per-bond backward (see bond.hip for the walk).
#include <algorithm>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "bond.h"

namespace ising {

// Geometry and pair tables of the per-bond backward walk (see bond.hip).  It
// keeps the forward bit order: tile bits [0, TJ), then mj <= 4 middle bits,
// the rest prefix.  Pairs are the distinct (i, j) of the input bonds, also
// those whose couplings cancel (their spin products still have averages).
// Byte constants address an FP64 weight table with rw interleaved copies:
// double (bin * rw + copy), bin = e_idx * W + n_up.
BondPlan *bond_plan_create(const ising_plan *p, const ising_lattice *lat, const std::vector<int64_t> &J,
                           const std::vector<int64_t> &classes) {
  BondPlan *bp = new (std::nothrow) BondPlan();
  if (!bp) return nullptr;
  const DevPlan &d = p->dev;
  const int n = d.n, TJ = d.tile;
  // Middle bits: up to kBwMid, fewer on small lattices so that the chunks
  // still make 2^kFillTaskBits tasks of 2^kLaneBits (one block per CU of a
  // 256-CU device) where the spins allow.
  constexpr int kFillTaskBits = 8;
  const int mj = std::max(0, std::min(kBwMid, n - TJ - kLaneBits - kFillTaskBits));
  const int kb = TJ + mj;
  auto bad = [&](const std::string &m) {
    bp->status = ISING_EUNSUPPORTED;
    bp->error = m;
    return bp;
  };
  // distinct pairs in order of first appearance among the input bonds
  std::vector<int32_t> pid(size_t(n) * n, -1);
  std::vector<std::pair<int, int>> pairs;
  bp->pair_of_bond.assign(size_t(lat->n_bonds), -1);
  for (int b = 0; b < lat->n_bonds; ++b) {
    const int i = std::min(lat->bond_i[b], lat->bond_j[b]), j = std::max(lat->bond_i[b], lat->bond_j[b]);
    int32_t &slot = pid[size_t(i) * n + j];
    if (slot < 0) {
      slot = int32_t(pairs.size());
      pairs.push_back({i, j});
    }
    bp->pair_of_bond[b] = slot;
  }
  if ((int)pairs.size() > kMaxPairs)
    return bad(std::to_string(pairs.size()) + " distinct bond pairs (the backward handles " +
               std::to_string(kMaxPairs) + ")");
  const int n_pairs = (int)pairs.size();
  // Weight-table row stride: a multiple of 4, so that bin mod 4 = n_up mod 4.
  // A 64-bit LDS read serves 32 lanes per cycle from 32 banks of 8 bytes;
  // double (bin * rw + copy) sits in bank (bin * rw + copy) mod 32.
  const int Wb = (n + 4) & ~3;
  // weight-table copies that fit next to the per-wave pair accumulators and
  // previous cumulative sums
  const int64_t acc_bytes = int64_t(kBwWaves) * (std::max(n_pairs, 1) + kPrevSlots) * 8;
  const int64_t copy_bytes = int64_t(d.n_ec) * Wb * 8;
  int rw = 8;
  while (rw > 1 && copy_bytes * rw + acc_bytes > kHistBytes) rw >>= 1;
  if (copy_bytes * rw + acc_bytes > kHistBytes)
    return bad("FP64 weight table of " + std::to_string(d.n_ec) + " x " + std::to_string(Wb) +
               " bins does not fit the LDS");
  DevPlan &w = bp->geo;
  w = d;
  w.W = Wb;
  w.inner = kb;
  w.R = 2 * rw;   // row bytes W * R * 4 = W * rw * 8
  const int64_t row_bytes = int64_t(w.W) * w.R * 4, col_bytes = int64_t(w.R) * 4;
  for (int c = 0; c < (int)classes.size(); ++c)
    w.cls_step[c] = (int32_t)((4 * classes[c] / w.estep) * row_bytes);
  for (int b = 0; b < n; ++b) w.up_base[b] = (int32_t)((2 * int64_t(w.hdeg[b]) / w.estep) * row_bytes + col_bytes);
  std::memset(w.kmid, 0, sizeof(w.kmid));
  for (int m = TJ; m < kb; ++m)
    for (int i = 0; i < TJ; ++i) {
      const int64_t v = J[size_t(p->site_of_bit[m]) * n + p->site_of_bit[i]];
      w.kmid[m - TJ][i] = (int32_t)((-4 * v / w.estep) * row_bytes);
    }

  BondTables &t = bp->tables;
  t = BondTables{};
  t.n_pairs = n_pairs;
  t.mj = mj;
  t.rw = rw;
  t.wt_bytes = (int32_t)(copy_bytes * rw);
  t.n_bonds = lat->n_bonds;
  for (auto &row : t.qpair)
    for (auto &v : row) v = -1;
  for (auto &v : t.m2pair) v = -1;
  const int lf_end = kb + kLaneBits;   // prefix bits [kb, lf_end) are lane-fixed
  std::vector<std::vector<std::pair<int, int>>> it(kInner), il(kInner), lt(kLaneBits);
  for (int q = 0; q < n_pairs; ++q) {
    int a = p->bit_of_site[pairs[q].first], b = p->bit_of_site[pairs[q].second];
    if (a > b) std::swap(a, b);
    if (b < TJ) return bad("internal: bond pair inside the tile");   // the tile holds no listed pair
    if (b < kb) {                      // both inner: from the lane running sums
      if (a < TJ) t.qpair[b - TJ][a] = (int16_t)q;
      else {
        const int m1 = a - TJ, m2 = b - TJ;
        t.m2pair[m1 * (7 - m1) / 2 + (m2 - m1 - 1)] = (int16_t)q;
      }
    } else if (a < kb) {               // inner - prefix
      (b < lf_end ? il : it)[size_t(a)].push_back({q, b});
    } else if (b < lf_end) {           // both lane-fixed
      t.ll_pair[t.n_ll] = (int16_t)q;
      t.ll_a[t.n_ll] = (uint8_t)a;
      t.ll_b[t.n_ll] = (uint8_t)b;
      ++t.n_ll;
    } else if (a < lf_end) {           // lane-fixed - task
      lt[size_t(a - kb)].push_back({q, b});
    } else {                           // both task bits
      t.tt_pair[t.n_tt] = (int16_t)q;
      t.tt_a[t.n_tt] = (uint8_t)a;
      t.tt_b[t.n_tt] = (uint8_t)b;
      ++t.n_tt;
    }
  }
  int e = 0, f = 0;
  for (int a = 0; a <= kInner; ++a) {
    t.it_start[a] = (int16_t)e;
    t.il_start[a] = (int16_t)f;
    if (a == kInner) break;
    for (auto &pr : it[size_t(a)]) {
      t.it_pair[e] = (int16_t)pr.first;
      t.it_bit[e++] = (uint8_t)pr.second;
    }
    for (auto &pr : il[size_t(a)]) {
      t.il_pair[f] = (int16_t)pr.first;
      t.il_bit[f++] = (uint8_t)pr.second;
    }
  }
  int g = 0;
  e = 0;
  for (int l = 0; l < kLaneBits; ++l) {
    if (lt[size_t(l)].empty()) continue;
    t.ltg_a[g] = (uint8_t)(kb + l);
    t.ltg_start[g] = (int16_t)e;
    for (auto &pr : lt[size_t(l)]) {
      t.lt_pair[e] = (int16_t)pr.first;
      t.lt_bit[e++] = (uint8_t)pr.second;
    }
    ++g;
  }
  t.ltg_start[g] = (int16_t)e;
  t.n_ltg = g;

  // Which chunk of a task each thread walks: with 8 copies, lanes sharing a
  // copy get chunks of four different n_up mod 4 (balance_lane_chunks).
  const int nthreads = kBwWaves * kWave;
  for (int i = 0; i < nthreads; ++i) t.lane_chunk[i] = (uint16_t)i;
  if (rw == 8) balance_lane_chunks(t.lane_chunk, nthreads);
  return bp;
}

}  // namespace ising

using namespace ising;

extern "C" ising_status ising_bond_workspace(const ising_plan *p, size_t *bytes) {
  if (!p || !bytes) return fail(ISING_EINVAL, "plan or bytes is NULL");
  if (p->bond->status != ISING_OK) return fail(p->bond->status, p->bond->error);
  *bytes = size_t(kMaxBwBlocks) * size_t(std::max(p->bond->tables.n_pairs, 1)) * sizeof(double);
  return ISING_OK;
}
