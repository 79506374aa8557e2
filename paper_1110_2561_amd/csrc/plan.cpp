// Host-side plan construction for libising: validation, coupling merge,
// spin ordering, chunk decomposition and histogram geometry.  No HIP calls:
// this file builds with any C++17 compiler (the library builds it with hipcc).
#include <algorithm>
#include <cstdlib>
#include <cstring>
#include <new>
#include <numeric>
#include <string>
#include <vector>

#include "internal.h"

namespace ising {

static thread_local std::string g_last_error;

void set_error(const std::string &msg) { g_last_error = msg; }

ising_status fail(ising_status st, const std::string &msg) {
  g_last_error = std::string(ising_status_str(st)) + ": " + msg;
  return st;
}

static int64_t floor_div(int64_t a, int64_t b) {
  int64_t q = a / b;
  if ((a % b != 0) && ((a < 0) != (b < 0))) --q;
  return q;
}

}  // namespace ising

using namespace ising;

extern "C" const char *ising_status_str(ising_status st) {
  switch (st) {
    case ISING_OK: return "ISING_OK";
    case ISING_EINVAL: return "ISING_EINVAL";
    case ISING_ETOO_MANY_SPINS: return "ISING_ETOO_MANY_SPINS";
    case ISING_EBOND: return "ISING_EBOND";
    case ISING_ERANGE: return "ISING_ERANGE";
    case ISING_EHIP: return "ISING_EHIP";
    case ISING_ENOMEM: return "ISING_ENOMEM";
    case ISING_EUNSUPPORTED: return "ISING_EUNSUPPORTED";
  }
  return "ISING_UNKNOWN";
}

extern "C" const char *ising_last_error(void) { return g_last_error.c_str(); }

extern "C" const char *ising_version(void) { return "libising 0.1 (gfx950)"; }

// Lanes l of a wave enumerate chunks base + l, so chunk bits 0..5 (plan bits
// k..k+5) tell a wave's lanes apart.  Lanes a, b that share an LDS copy
// (a = b mod R) hold configurations that differ by flipping the spin set F on
// the bits of a ^ b.  When their n_up agree (equal popcounts) they hit the
// same LDS word whenever their energies agree as well.  Flipping F changes
// the energy by 2 * sum_{bonds crossing F} J s_i s_j, which is 2 * (number of
// odd couplings crossing F) modulo 4, and that number has the parity of
// sum_{i in F} d_i, d_i being the count of odd couplings at spin i.  So when
// estep = 2 (mod 4) the two energy indices have different parity, and never
// agree, if the spins of F hold an odd number of odd d_i.  This picks the
// parity pattern of bits k..k+5 that does so for the most such lane pairs,
// among the patterns the prefix spins can supply, and moves matching prefix
// spins to those bits.  The order of prefix spins is otherwise free.
static void place_lane_spins(int n, int k, int R, const std::vector<int64_t> &J, int32_t *site_of_bit) {
  int want[64] = {0};  // flip patterns of same-copy lane pairs with equal n_up
  for (int a = 0; a < 64; ++a)
    for (int b = a + 1; b < 64; ++b)
      if ((a & (R - 1)) == (b & (R - 1)) && __builtin_popcount(a) == __builtin_popcount(b)) ++want[a ^ b];
  std::vector<int32_t> odd_sites, even_sites;  // prefix spins by parity of d_i
  for (int b = k; b < n; ++b) {
    const int i = site_of_bit[b];
    int d = 0;
    for (int j = 0; j < n; ++j) d += int(J[size_t(i) * n + j] & 1);
    (d & 1 ? odd_sites : even_sites).push_back(i);
  }
  int best = -1, best_p = 0;
  for (int p = 0; p < 64; ++p) {
    const int w = __builtin_popcount(p);
    if (w > int(odd_sites.size()) || 6 - w > int(even_sites.size())) continue;
    int sc = 0;
    for (int f = 1; f < 64; ++f)
      if (__builtin_popcount(f & p) & 1) sc += want[f];
    if (sc > best) { best = sc; best_p = p; }
  }
  size_t io = 0, ie = 0;
  int32_t *dst = site_of_bit + k;
  for (int b = 0; b < 6; ++b) *dst++ = (best_p >> b & 1) ? odd_sites[io++] : even_sites[ie++];
  while (io < odd_sites.size()) *dst++ = odd_sites[io++];
  while (ie < even_sites.size()) *dst++ = even_sites[ie++];
}

// Thread -> chunk offset for 8 interleaved LDS copies (copy = lane mod 8).
// The four lanes of a half-wave that share a copy hit four different banks
// when their chunks' n_up differ mod 4, i.e. when the popcounts of their
// chunk offsets (the prefix spins that tell a block's lanes apart) differ
// mod 4.  Offsets by popcount class are not equally many (for 2^m offsets
// the class sizes differ by about 2^(m/2)), so greedily give every copy group
// one offset of each class while the classes last; the few groups left over
// take repeats.
void ising::balance_lane_chunks(uint16_t *lane_chunk, int threads) {
  std::vector<int> cls[4];
  for (int o = 0; o < threads; ++o) cls[__builtin_popcount(unsigned(o)) & 3].push_back(o);
  size_t next[4] = {0, 0, 0, 0};
  auto left = [&](int c) { return cls[c].size() - next[c]; };
  for (int h = 0; h < threads / 32; ++h)
    for (int g = 0; g < 8; ++g) {
      bool used[4] = {false, false, false, false};
      for (int j = 0; j < 4; ++j) {
        int best = -1;
        for (int pass = 0; pass < 2 && best < 0; ++pass)
          for (int c = 0; c < 4; ++c)
            if (left(c) > 0 && (pass == 1 || !used[c]) && (best < 0 || left(c) > left(best))) best = c;
        used[best] = true;
        lane_chunk[h * 32 + g + 8 * j] = (uint16_t)cls[best][next[best]++];
      }
    }
}

extern "C" ising_status ising_plan_create(const ising_lattice *lat, const ising_tune *tune,
                                          ising_plan **out) {
  return ising::plan_create_internal(lat, tune, 1, out);
}

ising_status ising::plan_create_internal(const ising_lattice *lat, const ising_tune *tune, int min_classes,
                                         ising_plan **out, bool exact_tile) {
  if (!out) return fail(ISING_EINVAL, "plan output pointer is NULL");
  *out = nullptr;
  if (!lat) return fail(ISING_EINVAL, "lattice is NULL");
  const int n = lat->n_spins;
  if (n < 1 || n > kMaxSpins)
    return fail(ISING_ETOO_MANY_SPINS, "n_spins = " + std::to_string(n) + " (must be 1..64)");
  if (lat->n_bonds < 0) return fail(ISING_EINVAL, "n_bonds < 0");
  if (lat->n_bonds > 0 && (!lat->bond_i || !lat->bond_j || !lat->bond_J))
    return fail(ISING_EINVAL, "bond arrays are NULL");
  ising_tune tn{};
  if (tune) tn = *tune;
  if (tn.inner_bits < 0 || tn.inner_bits > kMaxInner || tn.tile_bits < 0 || tn.tile_bits > kMaxTile ||
      tn.waves_per_block < 0 || tn.waves_per_block > 16 || tn.max_blocks < 0 || tn.prefix_bits < 0 ||
      tn.prefix_bits > kMaxSpins ||
      (tn.replicas != 0 && (tn.replicas > 16 || (tn.replicas & (tn.replicas - 1)))))
    return fail(ISING_EINVAL, "tune values out of range");

  // ---- validate bonds and merge repeated pairs (E is linear in J per pair) ----
  const int64_t kJmax = int64_t(1) << 20;
  int64_t S = 0;
  std::vector<int64_t> J(size_t(n) * n, 0);
  std::vector<char> listed(size_t(n) * n, 0);   // pair appears among the bonds (even if its couplings cancel)
  for (int b = 0; b < lat->n_bonds; ++b) {
    const int i = lat->bond_i[b], j = lat->bond_j[b];
    const int64_t v = lat->bond_J[b];
    if (i < 0 || i >= n || j < 0 || j >= n)
      return fail(ISING_EBOND, "bond " + std::to_string(b) + " has an endpoint outside 0..n_spins-1");
    if (i == j) return fail(ISING_EBOND, "bond " + std::to_string(b) + " is a self-bond");
    if (v > kJmax || v < -kJmax) return fail(ISING_ERANGE, "|J| > 2^20 in bond " + std::to_string(b));
    S += v < 0 ? -v : v;
    if (S > kJmax) return fail(ISING_ERANGE, "sum |J| exceeds 2^20");
    J[size_t(std::min(i, j)) * n + std::max(i, j)] += v;
    J[size_t(std::max(i, j)) * n + std::min(i, j)] += v;
    listed[size_t(i) * n + j] = listed[size_t(j) * n + i] = 1;
  }

  // ---- coupling classes and the compact energy lattice ----
  std::vector<int64_t> classes;
  int64_t S_eff = 0, E_ref = 0, n_pairs = 0;
  for (int i = 0; i < n; ++i)
    for (int j = i + 1; j < n; ++j) {
      const int64_t v = J[size_t(i) * n + j];
      if (!v) continue;
      ++n_pairs;
      S_eff += v < 0 ? -v : v;
      E_ref -= v;  // all spins up: every pair contributes -J
      if (std::find(classes.begin(), classes.end(), v) == classes.end()) classes.push_back(v);
    }
  if ((int)classes.size() > kMaxClasses || min_classes > kMaxClasses)
    return fail(ISING_EUNSUPPORTED, std::to_string(classes.size()) +
                                        " distinct merged couplings (at most 8 supported)");
  std::sort(classes.begin(), classes.end());
  // Flipping spin i changes E by -2 s_new h_i, h_i = sum_j J_ij s_j, and
  // h_i = sum_j J_ij (mod 2 g_i) with g_i = gcd_j |J_ij|; so every energy lies
  // on E_ref + estep Z with estep = gcd_i gcd(2 |sum_j J_ij|, 4 g_i).
  int64_t estep = 0;
  std::vector<int> degree(n, 0);
  for (int i = 0; i < n; ++i) {
    int64_t gi = 0, sum = 0;
    for (int j = 0; j < n; ++j) {
      const int64_t v = J[size_t(i) * n + j];
      if (!v) continue;
      ++degree[i];
      gi = std::gcd(gi, v < 0 ? -v : v);
      sum += v;
    }
    if (!gi) continue;
    estep = std::gcd(estep, std::gcd(2 * (sum < 0 ? -sum : sum), 4 * gi));
  }
  if (!estep) estep = 1;
  const int64_t e_base = E_ref - estep * floor_div(E_ref + S_eff, estep);
  const int64_t n_ec = (S_eff - e_base) / estep + 1;
  // Row stride: the least even W >= n + 1.  With 16 copies a bin's bank on
  // the 32-bank LDS is 16 * (bin mod 2) + copy, and bin mod 2 = n_up mod 2
  // for even W, so lanes l and l + 16 (n_up one apart) never collide.
  int W = (n + 2) & ~1;

  // ---- histogram replicas that fit the LDS ----
  int R = tn.replicas ? tn.replicas : 16;
  while (R > 1 && n_ec * W * R * 4 > kHistBytes) R >>= 1;
  // With 8 copies a bin's bank is 8 * (bin mod 4) + copy: a stride that is a
  // multiple of 4 makes bin mod 4 = n_up mod 4, and the thread -> chunk
  // permutation (balance_lane_chunks) gives the four lanes of a half-wave
  // that share a copy four different n_up mod 4.
  if (R == 8 && n_ec * ((n + 4) & ~3) * R * 4 <= kHistBytes) W = (n + 4) & ~3;
  if (n_ec * W * R * 4 > kHistBytes)
    return fail(ISING_ERANGE, "compact histogram of " + std::to_string(n_ec) + " x " + std::to_string(W) +
                                  " bins exceeds the 160 KB LDS");
  const int wpb = tn.waves_per_block ? tn.waves_per_block : 16;
  // The enumeration kernel reserves the whole 160 KB LDS of a CU (a static
  // array, so histogram addresses need no base add): one block per CU.
  const int bpc = 1;

  // ---- tile: an independent set (no listed pair between members, so no
  // merged coupling either, and the per-bond backward never sees a pair
  // inside the tile), by the minimum-degree greedy rule: take a site of least
  // remaining degree, drop it and its neighbours, repeat ----
  std::vector<int> order(n);
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return degree[a] > degree[b]; });
  std::vector<int> tile;
  const int tile_want = tn.tile_bits ? tn.tile_bits : kMaxTile;
  {
    std::vector<char> alive(n, 1);
    std::vector<int> rem(n, 0);
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j) rem[i] += listed[size_t(i) * n + j];
    while ((int)tile.size() < tile_want) {
      int best = -1;
      for (int s2 = 0; s2 < n; ++s2)
        if (alive[s2] && (best < 0 || rem[s2] < rem[best])) best = s2;
      if (best < 0) break;
      tile.push_back(best);
      std::vector<int> gone{best};
      for (int j = 0; j < n; ++j)
        if (alive[j] && j != best && listed[size_t(best) * n + j]) gone.push_back(j);
      for (int g2 : gone) {
        alive[g2] = 0;
        for (int j = 0; j < n; ++j)
          if (alive[j] && listed[size_t(g2) * n + j]) --rem[j];
      }
    }
  }
  const int TJ = std::max(1, std::min<int>((int)tile.size(), n));
  if (exact_tile && tn.tile_bits && TJ != tn.tile_bits)
    return fail(ISING_EINVAL, "no independent set of " + std::to_string(tn.tile_bits) + " spins");

  // ---- inner bits k: enough chunks for several tasks per block ----
  int k;
  if (tn.inner_bits) {
    k = tn.inner_bits;
    if (k < TJ || k > n) return fail(ISING_EINVAL, "inner_bits must lie in [tile_bits, n_spins]");
  } else if (tn.prefix_bits) {
    k = std::max(TJ, std::min(std::min(n - tn.prefix_bits, n), kMaxInner));
  } else {
    // ~4 tasks per block on 256 CUs: enough to even out the blocks'
    // finishing times, with chunks large enough to amortise their set-up.
    const int lanes_log2 = 8 /* 256 CUs */ + (bpc > 1 ? 1 : 0) + 6 + (31 - __builtin_clz(unsigned(wpb)));
    k = n - (lanes_log2 + 2);
    k = std::max(TJ, std::min(std::min(k, n), kMaxInner));
  }
  // every u32 LDS counter must stay below 2^32 between flushes:
  // one task adds at most (lanes sharing a replica) * 2^k to a counter.
  const uint64_t lanes_per_replica = uint64_t(kWave) * wpb / R;
  if (lanes_per_replica << k >= (uint64_t(1) << 32)) {
    if (tn.inner_bits) return fail(ISING_EINVAL, "inner_bits too large for the counter width");
    while (k > TJ && (lanes_per_replica << k) >= (uint64_t(1) << 32)) --k;
    if ((lanes_per_replica << k) >= (uint64_t(1) << 32))
      return fail(ISING_EUNSUPPORTED, "no chunk size keeps LDS counters below 2^32");
  }

  // ---- bit order: tile, then middle, then prefix ----
  ising_plan *p = new (std::nothrow) ising_plan();
  if (!p) return fail(ISING_ENOMEM, "plan allocation");
  std::vector<char> used(n, 0);
  int bit = 0;
  for (int t = 0; t < TJ; ++t) { p->site_of_bit[bit++] = tile[t]; used[tile[t]] = 1; }
  for (int s : order)
    if (!used[s]) { p->site_of_bit[bit++] = s; used[s] = 1; }
  const bool balanced = R == 8 && W % 4 == 0;   // lanes sharing a copy never share a bin
  if (estep % 4 == 2 && n - k >= 6 && R >= 2 && !balanced) place_lane_spins(n, k, R, J, p->site_of_bit);
  for (int b = 0; b < n; ++b) p->bit_of_site[p->site_of_bit[b]] = b;

  p->n_spins = n;
  p->n_bonds = lat->n_bonds;
  p->S = S;
  p->n_chunks = uint64_t(1) << (n - k);
  p->waves_per_block = wpb;
  p->max_blocks = tn.max_blocks;
  p->blocks_per_cu = bpc;
  p->n_merged_pairs = n_pairs;

  DevPlan &d = p->dev;
  d.n = n;
  d.inner = k;
  d.tile = TJ;
  d.n_classes = 1;
  while (d.n_classes < (int)classes.size() || d.n_classes < min_classes) d.n_classes *= 2;  // kernels: 1, 2, 4, 8
  d.estep = (int32_t)estep;
  d.e_base = (int32_t)e_base;
  d.n_ec = (int32_t)n_ec;
  d.W = W;
  d.R = R;
  d.e_min = (int32_t)-S;
  d.n_m = n + 1;
  const int64_t row_bytes = int64_t(W) * R * 4, col_bytes = int64_t(R) * 4;
  for (int c = 0; c < (int)classes.size(); ++c) {
    d.class_J[c] = (int32_t)classes[c];
    d.cls_step[c] = (int32_t)((4 * classes[c] / estep) * row_bytes);   // estep divides 4 J_c
  }
  for (int b = 0; b < n; ++b) {
    const int s = p->site_of_bit[b];
    int64_t hd = 0;
    for (int b2 = 0; b2 < n; ++b2) {
      const int64_t v = J[size_t(s) * n + p->site_of_bit[b2]];
      if (!v) continue;
      const int c = int(std::find(classes.begin(), classes.end(), v) - classes.begin());
      d.mask[b][c] |= uint64_t(1) << b2;
      hd += v;
    }
    d.hdeg[b] = (int32_t)hd;
    d.up_base[b] = (int32_t)((2 * hd / estep) * row_bytes + col_bytes);  // estep divides 2 hdeg
  }
  for (int m = TJ; m < k; ++m)
    for (int i = 0; i < TJ; ++i) {
      const int64_t v = J[size_t(p->site_of_bit[m]) * n + p->site_of_bit[i]];
      // tile spin i's up-flip delta, in bytes, changes by this when bit m goes up
      d.kmid[m - TJ][i] = (int32_t)((-4 * v / estep) * row_bytes);
    }
  for (int i = 0; i < kMaxBlockThreads; ++i) d.lane_chunk[i] = (uint16_t)i;
  if (balanced) balance_lane_chunks(d.lane_chunk, kWave * wpb);
  p->bond = bond_plan_create(p, lat, J, classes);
  if (!p->bond) {
    delete p;
    return fail(ISING_ENOMEM, "plan allocation");
  }
  *out = p;
  set_error("");
  return ISING_OK;
}

extern "C" ising_status ising_hist_shape(const ising_plan *p, int32_t *n_e, int32_t *n_m, int32_t *e_min) {
  if (!p) return fail(ISING_EINVAL, "plan is NULL");
  if (n_e) *n_e = (int32_t)(2 * p->S + 1);
  if (n_m) *n_m = p->n_spins + 1;
  if (e_min) *e_min = (int32_t)-p->S;
  return ISING_OK;
}

extern "C" ising_status ising_plan_layout(const ising_plan *p, int32_t *bit_of_site, int32_t *inner_bits,
                                          int32_t *tile_bits, uint64_t *n_chunks) {
  if (!p) return fail(ISING_EINVAL, "plan is NULL");
  if (bit_of_site) std::memcpy(bit_of_site, p->bit_of_site, sizeof(int32_t) * p->n_spins);
  if (inner_bits) *inner_bits = p->dev.inner;
  if (tile_bits) *tile_bits = p->dev.tile;
  if (n_chunks) *n_chunks = p->n_chunks;
  return ISING_OK;
}
