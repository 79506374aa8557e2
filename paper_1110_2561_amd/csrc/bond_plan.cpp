// Host-side planning of the per-bond backward (see bond.hip for the walk).
#include <algorithm>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "bond.h"

namespace ising {

// Geometry and pair tables of the per-bond backward walk (see bond.h for the
// bit layout and bond.hip for the walk).  It keeps the forward bit order.
// Pairs are the distinct (i, j) of the input bonds, also those whose
// couplings cancel (their spin products still have averages).  Byte
// constants address an FP64 weight table with rw interleaved copies:
// double (bin * rw + copy), bin = e_idx * W + n_up.
BondPlan *bond_plan_create(const ising_plan *p, const ising_lattice *lat, const std::vector<int64_t> &J,
                           const std::vector<int64_t> &classes) {
  BondPlan *bp = new (std::nothrow) BondPlan();
  if (!bp) return nullptr;
  const DevPlan &d = p->dev;
  const int n = d.n, TJ = d.tile;
  // Block bits first (256 blocks, one per CU of a 256-CU device, where the
  // spins allow), then up to kBwMid middle bits; the rest are hi bits.
  const int above = std::max(0, n - TJ - kLaneBits);
  const int s = std::min(kBlockBits, above);
  const int mj = std::min(kBwMid, above - s);
  const int kb = TJ + mj;
  const int n_hi = std::max(0, n - kb - kLaneBits - s);
  const int lf = kb + kLaneBits;      // offset bits [kb, lf)
  const int hi0 = lf + s;             // block bits [lf, hi0), hi bits [hi0, n)
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
  // per-wave pair accumulators first (16-byte aligned), then as many
  // weight-table copies as fit; the final reduction reuses the table's
  // space for kRound values per lane and wave
  const int64_t acc_bytes = (int64_t(kBwWaves) * std::max(n_pairs, 1) * 8 + 15) & ~int64_t(15);
  const int64_t round_bytes = int64_t(kBwWaves) * kRound * (kWave * 8 + 4);
  const int64_t copy_bytes = int64_t(d.n_ec) * Wb * 8;
  if (acc_bytes + round_bytes > kHistBytes) return bad("internal: pair accumulators exceed the LDS");
  int rw = 8;
  while (rw > 1 && acc_bytes + copy_bytes * rw > kHistBytes) rw >>= 1;
  if (acc_bytes + copy_bytes * rw > kHistBytes)
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
  std::memset(w.kmid, 0, sizeof(w.kmid));   // the backward uses kbit

  BondTables &t = bp->tables;
  t = BondTables{};
  t.n_pairs = n_pairs;
  t.mj = mj;
  t.rw = rw;
  t.wt_bytes = (int32_t)(copy_bytes * rw);
  t.n_bonds = lat->n_bonds;
  t.s_bits = s;
  t.n_hi = n_hi;
  t.n_offsets = n - kb >= kLaneBits ? (1 << kLaneBits) : (1 << (n - kb));
  t.acc_bytes = (int32_t)acc_bytes;
  for (auto &row : t.qpair)
    for (auto &v : row) v = -1;
  t.m2pair = -1;
  for (auto &row : t.hp_inner)
    for (auto &v : row) v = -1;
  for (int b = TJ; b < n; ++b)
    for (int i = 0; i < TJ; ++i) {
      const int64_t v = J[size_t(p->site_of_bit[b]) * n + p->site_of_bit[i]];
      t.kbit[b][i] = (int32_t)((-4 * v / w.estep) * row_bytes);
    }
  std::vector<std::vector<std::pair<int, int>>> end_in(kInner), hp(size_t(std::max(n_hi, 1)));
  for (int q = 0; q < n_pairs; ++q) {
    int a = p->bit_of_site[pairs[q].first], b = p->bit_of_site[pairs[q].second];
    if (a > b) std::swap(a, b);
    if (b < TJ) return bad("internal: bond pair inside the tile");   // the tile holds no listed pair
    if (b < kb) {                      // both inner: from the lane running sums
      if (a < TJ) t.qpair[b - TJ][a] = (int16_t)q;
      else t.m2pair = (int16_t)q;      // the two middle bits
      continue;
    }
    // an end term for every pair with a non-inner bit
    if (a < kb) {
      end_in[size_t(a)].push_back({q, b});
    } else {
      t.eo_pair[t.n_end_outer] = (int16_t)q;
      t.eo_a[t.n_end_outer] = (uint8_t)a;
      t.eo_b[t.n_end_outer] = (uint8_t)b;
      ++t.n_end_outer;
    }
    // flip terms at every flip of a hi bit of the pair
    for (const auto &ends : {std::pair<int, int>{a, b}, std::pair<int, int>{b, a}}) {
      const int hb = ends.second, other = ends.first;   // hb flips, `other` is its partner
      if (hb < hi0) continue;
      if (other < kb) t.hp_inner[hb - hi0][other] = (int16_t)q;
      else hp[size_t(hb - hi0)].push_back({q, other});
    }
  }
  int e = 0;
  for (int a = 0; a <= kInner; ++a) {
    t.end_start[a] = (int16_t)e;
    if (a == kInner) break;
    for (auto &pr : end_in[size_t(a)]) {
      t.end_pair[e] = (int16_t)pr.first;
      t.end_b[e++] = (uint8_t)pr.second;
    }
  }
  e = 0;
  for (int j = 0; j <= kMaxSpins; ++j) {
    t.hp_start[j] = (int16_t)e;
    if (j >= n_hi) continue;
    for (auto &pr : hp[size_t(j)]) {
      t.hp_pair[e] = (int16_t)pr.first;
      t.hp_a[e++] = (uint8_t)pr.second;
    }
  }

  // Which chunk offset each thread walks: with 8 copies, lanes sharing a
  // copy get offsets of four different n_up mod 4 (balance_lane_chunks).
  const int nthreads = kBwWaves * kWave;
  for (int i = 0; i < nthreads; ++i) t.lane_chunk[i] = (uint16_t)i;
  if (rw == 8 && t.n_offsets == nthreads) balance_lane_chunks(t.lane_chunk, nthreads);
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
