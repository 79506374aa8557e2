// FP64 evaluation of the partition function (Peretyatko et al., Section 2,
// Eq. (2)) and its moments and derivatives from a dense degeneracy table on
// the device.
//
// Grouping the configurations of Eq. (2) by (E, M):
//   Z(T, h) = sum_{E,M} g(E, M) exp(-(E - h M)/T),  H = E - h M (Eq. (1)).
// One block per few temperatures (and, for one table, a group of up to 4
// fields): the table's nonzero bins are staged in LDS as (ln g, E, M), then
// for each temperature and group of up to 4 fields, per point:
//   pass 1  m = max over nonzero bins of a = ln g - (E - h M)/T;
//   pass 2  Z' = sum exp(a - m), and the weighted sums of E and M;
//   pass 3  centred sums of (H - <H>)^2, (M - <M>)^2 and (H - <H>)(M - <M>);
//   log Z = m + ln Z', <E>, <M>, C = Var(H)/T^2, chi = Var(M)/T, and the
//   derivatives of log Z that follow from differentiating Eq. (2):
//     d/dT = <H>/T^2, d/dh = <M>/T, d2/dT2 = Var(H)/T^4 - 2<H>/T^3,
//     d2/dTdh = (Cov(H, M)/T - <M>)/T^2, d2/dh2 = Var(M)/T^2.
// Reductions run in a fixed order (wave shuffles, then waves), so results are
// reproducible run to run.  The table is small (<= ~10^5 bins) and read from
// L2 by every block; this kernel is negligible next to the enumeration.
//
// k_bin_weights turns a loss gradient G[T][h] into the weight every
// configuration of bin (E, M) carries in d(sum G log Z)/dJ_b (the per-bond
// backward sums these weights times s_i s_j over all configurations):
//   w(E, M) = sum_{a,c} G[a][c] exp(-(E - h_c M)/T_a - log Z(T_a, h_c)) / T_a.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <string>

#include "internal.h"

namespace ising {

constexpr int kThermoThreads = 256;

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
  return v;
}

// Block-wide sums of N values; every thread gets the totals.  sh holds N
// doubles per wave.  Fixed order: wave shuffles, then waves in order.
template <int N>
__device__ __forceinline__ void block_sums(double (&v)[N], double *sh) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, nw = blockDim.x >> 6;
#pragma unroll
  for (int j = 0; j < N; ++j) v[j] = wave_sum(v[j]);
  __syncthreads();
  if (lane == 0) {
#pragma unroll
    for (int j = 0; j < N; ++j) sh[wv * N + j] = v[j];
  }
  __syncthreads();
#pragma unroll
  for (int j = 0; j < N; ++j) {
    double t = 0.0;
    for (int w = 0; w < nw; ++w) t += sh[w * N + j];
    v[j] = t;
  }
  __syncthreads();
}

// Output arrays of the FP64 evaluation; any may be NULL.
struct ThermoOut {
  double *logz, *mean_E, *mean_M, *heat, *susc;   // value and moments
  double *d_T, *d_h, *d_TT, *d_Th, *d_hh;         // derivatives of log Z
};

constexpr int kStageBins = 4096;  // nonzero bins a block keeps in LDS as (ln g, E, M)

// Bins of a dense table, read in place: zero bins are skipped, ln g computed.
struct DenseBins {
  static constexpr bool kStaged = false;
  const unsigned long long *g;
  int n_m, e_min, n_spins, bins;
  __device__ int count() const { return bins; }
  __device__ bool get(int i, double &lg, double &E, double &M) const {
    const unsigned long long v = g[i];
    if (!v) return false;
    const int e = i / n_m, nu = i - e * n_m;
    E = double(e + e_min);
    M = double(2 * nu - n_spins);
    lg = log(double(v));
    return true;
  }
};

// Nonzero bins staged in LDS (stage_bins): every entry is a real bin.
struct StagedBins {
  static constexpr bool kStaged = true;
  const double *lg;
  const int *E, *M;
  int n;
  __device__ int count() const { return n; }
  __device__ bool get(int i, double &l, double &e, double &m) const {
    l = lg[i];
    e = double(E[i]);
    m = double(M[i]);
    return true;
  }
};

// Copy the nonzero bins of a dense table into LDS as (ln g, E, M), thread by
// thread in a fixed order (thread t takes the bins t, t + blockDim, ...; its
// entries follow those of threads 0 .. t-1).  Returns their number, or -1
// (every thread) when more than kStageBins.  scan: blockDim.x / 64 + 1 ints
// of LDS for the per-wave totals.
__device__ int stage_bins(const unsigned long long *__restrict__ g, int n_e, int n_m, int e_min, int n_spins,
                          double *lg, int *E, int *M, int *scan) {
  const int bins = n_e * n_m;
  int mine = 0;
  for (int i = threadIdx.x; i < bins; i += blockDim.x) mine += g[i] != 0ull;
  // exclusive prefix over the block: inclusive scan within the wave by
  // shuffles, then the wave totals in order
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, nw = blockDim.x >> 6;
  int incl = mine;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const int v = __shfl_up(incl, off, 64);
    if (lane >= off) incl += v;
  }
  if (lane == 63) scan[wv] = incl;
  __syncthreads();
  int before = 0, total = 0;
  for (int w = 0; w < nw; ++w) {
    const int t = scan[w];
    if (w < wv) before += t;
    total += t;
  }
  __syncthreads();
  if (total > kStageBins) return -1;
  int at = before + incl - mine;
  for (int i = threadIdx.x; i < bins; i += blockDim.x) {
    const unsigned long long v = g[i];
    if (!v) continue;
    const int e = i / n_m, nu = i - e * n_m;
    lg[at] = log(double(v));
    E[at] = e + e_min;
    M[at] = 2 * nu - n_spins;
    ++at;
  }
  __syncthreads();
  return total;
}

// All outputs at temperature T and the fields h[0 .. cnt) (cnt <= kWaveFields)
// of one table, written at indices pt0 + j, by one wave: its lanes take the
// bins lane, lane + 64, ... and every sum or maximum over them is a fixed
// shuffle tree (the same value in every lane, independent of timing).  Each
// pass reads every bin once for all cnt points.  When the bins are staged
// and a lane holds at most kCacheBins of them, the lane keeps the weights of
// the second pass in registers for the third.
constexpr int kWaveFields = 2;
constexpr int kCacheBins = 32;

template <class Bins>
__device__ void wave_points(const Bins &B, double T, const double *__restrict__ h, int cnt, int pt0,
                            const ThermoOut &o) {
  constexpr int P = kWaveFields;
  const int lane = threadIdx.x & 63;
  const int bins = B.count();
  const bool want_second = o.heat || o.susc || o.d_TT || o.d_Th || o.d_hh;
  double *const all[10] = {o.logz, o.mean_E, o.mean_M, o.heat, o.susc, o.d_T, o.d_h, o.d_TT, o.d_Th, o.d_hh};
  double hv[P];
  bool ok[P];
#pragma unroll
  for (int j = 0; j < P; ++j) {
    hv[j] = j < cnt ? h[j] : 0.0;
    ok[j] = j < cnt && (T > 0.0) && isfinite(T) && isfinite(hv[j]);
    if (!ok[j]) hv[j] = 0.0;
  }
  const double inv_T = (T > 0.0 && isfinite(T)) ? 1.0 / T : 0.0;

  // pass 1: the largest exponent per point
  double m[P];
#pragma unroll
  for (int j = 0; j < P; ++j) m[j] = -INFINITY;
  for (int i = lane; i < bins; i += 64) {
    double lg, E, M;
    if (!B.get(i, lg, E, M)) continue;
#pragma unroll
    for (int j = 0; j < P; ++j)
      if (j < cnt) m[j] = fmax(m[j], lg - (E - hv[j] * M) * inv_T);
  }
#pragma unroll
  for (int j = 0; j < P; ++j) m[j] = wave_max(m[j]);
#pragma unroll
  for (int j = cnt; j < P; ++j) m[j] = m[0];

  // pass 2: Z' and first moments
  constexpr int KC = Bins::kStaged ? kCacheBins : 1;
  const bool cached = Bins::kStaged && bins <= KC * 64;
  double wc[KC][P];
  double acc[3 * P];
#pragma unroll
  for (int j = 0; j < 3 * P; ++j) acc[j] = 0.0;
  if (m[0] != -INFINITY) {   // all points see the same nonzero bins
    if (cached) {
#pragma unroll
      for (int k = 0; k < KC; ++k) {
        const int i = lane + 64 * k;
        double lg, E, M;
        if (i >= bins || !B.get(i, lg, E, M)) continue;
#pragma unroll
        for (int j = 0; j < P; ++j) {
          if (j >= cnt) break;
          const double w = exp(lg - (E - hv[j] * M) * inv_T - m[j]);
          wc[k][j] = w;
          acc[3 * j] += w;
          acc[3 * j + 1] += w * E;
          acc[3 * j + 2] += w * M;
        }
      }
    } else {
      for (int i = lane; i < bins; i += 64) {
        double lg, E, M;
        if (!B.get(i, lg, E, M)) continue;
#pragma unroll
        for (int j = 0; j < P; ++j) {
          if (j >= cnt) break;
          const double w = exp(lg - (E - hv[j] * M) * inv_T - m[j]);
          acc[3 * j] += w;
          acc[3 * j + 1] += w * E;
          acc[3 * j + 2] += w * M;
        }
      }
    }
  }
#pragma unroll
  for (int j = 0; j < 3 * P; ++j) acc[j] = wave_sum(acc[j]);
  double mE[P], mM[P], z[P];
#pragma unroll
  for (int j = 0; j < P; ++j) {
    z[j] = acc[3 * j];
    mE[j] = acc[3 * j + 1] / z[j];
    mM[j] = acc[3 * j + 2] / z[j];
  }

  // pass 3: centred second moments of H = E - hM and M
  if (want_second && m[0] != -INFINITY) {
#pragma unroll
    for (int j = 0; j < 3 * P; ++j) acc[j] = 0.0;
    if (cached) {
#pragma unroll
      for (int k = 0; k < KC; ++k) {
        const int i = lane + 64 * k;
        double lg, E, M;
        if (i >= bins || !B.get(i, lg, E, M)) continue;
#pragma unroll
        for (int j = 0; j < P; ++j) {
          if (j >= cnt) break;
          const double w = wc[k][j];
          const double dH = (E - hv[j] * M) - (mE[j] - hv[j] * mM[j]), dM = M - mM[j];
          acc[3 * j] += w * dH * dH;
          acc[3 * j + 1] += w * dM * dM;
          acc[3 * j + 2] += w * dH * dM;
        }
      }
    } else {
      for (int i = lane; i < bins; i += 64) {
        double lg, E, M;
        if (!B.get(i, lg, E, M)) continue;
#pragma unroll
        for (int j = 0; j < P; ++j) {
          if (j >= cnt) break;
          const double w = exp(lg - (E - hv[j] * M) * inv_T - m[j]);
          const double dH = (E - hv[j] * M) - (mE[j] - hv[j] * mM[j]), dM = M - mM[j];
          acc[3 * j] += w * dH * dH;
          acc[3 * j + 1] += w * dM * dM;
          acc[3 * j + 2] += w * dH * dM;
        }
      }
    }
#pragma unroll
    for (int j = 0; j < 3 * P; ++j) acc[j] = wave_sum(acc[j]);
  }

  if (lane != 0) return;
#pragma unroll
  for (int j = 0; j < P; ++j) {
    if (j >= cnt) break;
    const int pt = pt0 + j;
    if (!ok[j]) {
#pragma unroll
      for (int i = 0; i < 10; ++i)
        if (all[i]) all[i][pt] = NAN;
      continue;
    }
    if (m[j] == -INFINITY) {   // empty table: Z = 0
#pragma unroll
      for (int i = 1; i < 10; ++i)
        if (all[i]) all[i][pt] = NAN;
      if (o.logz) o.logz[pt] = -INFINITY;
      continue;
    }
    const double mH = mE[j] - hv[j] * mM[j], T2 = inv_T * inv_T;
    if (o.logz) o.logz[pt] = m[j] + log(z[j]);
    if (o.mean_E) o.mean_E[pt] = mE[j];
    if (o.mean_M) o.mean_M[pt] = mM[j];
    if (o.d_T) o.d_T[pt] = mH * T2;
    if (o.d_h) o.d_h[pt] = mM[j] * inv_T;
    if (want_second) {
      const double varH = acc[3 * j] / z[j], varM = acc[3 * j + 1] / z[j], cov = acc[3 * j + 2] / z[j];
      if (o.heat) o.heat[pt] = varH * T2;
      if (o.susc) o.susc[pt] = varM * inv_T;
      if (o.d_TT) o.d_TT[pt] = varH * T2 * T2 - 2.0 * mH * T2 * inv_T;
      if (o.d_Th) o.d_Th[pt] = (cov * inv_T - mM[j]) * T2;
      if (o.d_hh) o.d_hh[pt] = varM * T2;
    }
  }
}

// A block's table: its nonzero bins are staged in LDS once (ln g taken once
// per bin) for the block's waves, so every lane of every pass works on a real
// bin; tables with more nonzero bins than fit are read in place.
struct StageLds {
  double lg[kStageBins];
  int E[kStageBins], M[kStageBins];
  int scan[kThermoThreads / 64 + 1];
};

constexpr int kWavesPerBlock = kThermoThreads / 64;

// One table: wave u of the grid (4 per block) takes temperature u / n_fg and
// the field group u % n_fg (kWaveFields fields each); outputs [nT][nh].
__global__ __launch_bounds__(kThermoThreads) void k_thermo(
    const unsigned long long *__restrict__ g, int n_e, int n_m, int e_min, int n_spins,
    const double *__restrict__ Tg, int nT, const double *__restrict__ hg, int nh, ThermoOut o) {
  __shared__ StageLds L;
  const int staged = stage_bins(g, n_e, n_m, e_min, n_spins, L.lg, L.E, L.M, L.scan);
  const int n_fg = (nh + kWaveFields - 1) / kWaveFields;
  const int64_t u = int64_t(blockIdx.x) * kWavesPerBlock + threadIdx.x / 64;
  if (u >= int64_t(nT) * n_fg) return;
  const int a = int(u / n_fg), c0 = int(u % n_fg) * kWaveFields;
  const int cnt = min(kWaveFields, nh - c0), pt0 = a * nh + c0;
  if (staged >= 0)
    wave_points(StagedBins{L.lg, L.E, L.M, staged}, Tg[a], hg + c0, cnt, pt0, o);
  else
    wave_points(DenseBins{g, n_m, e_min, n_spins, n_e * n_m}, Tg[a], hg + c0, cnt, pt0, o);
}

// One thread block per dense bin; its threads split the (T, h) points and the
// partial sums meet in a fixed-order block reduction.
__global__ __launch_bounds__(256) void k_bin_weights(
    const unsigned long long *__restrict__ g, int n_e, int n_m, int e_min, int n_spins,
    const double *__restrict__ Tg, int nT, const double *__restrict__ hg, int nh,
    const double *__restrict__ logz, const double *__restrict__ G, double *__restrict__ W) {
  __shared__ double sh[256 / 64];
  const int bins = n_e * n_m;
  for (int i = blockIdx.x; i < bins; i += gridDim.x) {
    if (!g[i]) {   // uniform over the block
      if (threadIdx.x == 0) W[i] = 0.0;
      continue;
    }
    const int e = i / n_m, nu = i - e * n_m;
    const double E = double(e + e_min), M = double(2 * nu - n_spins);
    double acc = 0.0;
    for (int pt = threadIdx.x; pt < nT * nh; pt += blockDim.x) {
      const double gc = G[pt];
      if (gc == 0.0) continue;
      const int a = pt / nh, c = pt - a * nh;
      const double inv_T = 1.0 / Tg[a];
      acc += gc * exp(-(E - hg[c] * M) * inv_T - logz[pt]) * inv_T;
    }
    double one[1] = {acc};
    block_sums(one, sh);
    if (threadIdx.x == 0) W[i] = one[0];
  }
}

// The bin weights of the backward, from the factorisation of each term of
//   W(E, M) = sum_a (1/T_a) sum_c G[a][c] exp(-(E - h_c M)/T_a - logz[a][c])
// as exp(-(E - E0)/T_a) * exp((h_c M - E0)/T_a - logz[a][c]) with E0 = e_min
// (the table's lowest energy, so the first factor is at most 1):
// k_weight_factors forms, per temperature a and column n_up,
// R[a][n_up] = sum_c G[a][c] exp((h_c M - E0)/T_a - logz[a][c]) and the largest
// of those exponents X[a][n_up]; k_weight_combine adds, per nonzero bin,
// exp(-(E - E0)/T_a) R[a][n_up] / T_a over a.  Each term is the same number as
// in the direct sum; where splitting its exponent could leave the double
// range (X > 600, or the energy factor below e^-600 while the product may not
// be), that (bin, a) is summed directly over c.  One wave per output, lanes
// over the summed index, fixed shuffle trees: every sum has a fixed order.
__global__ __launch_bounds__(256) void k_weight_factors(
    int n_m, int e_min, int n_spins, const double *__restrict__ Tg, int nT, const double *__restrict__ hg, int nh,
    const double *__restrict__ logz, const double *__restrict__ G, double *__restrict__ R,
    double *__restrict__ X) {
  const int lane = threadIdx.x & 63;
  const int w = int(blockIdx.x * (blockDim.x / 64) + threadIdx.x / 64);
  if (w >= nT * n_m) return;
  const int a = w / n_m, nu = w - a * n_m;
  const double E0 = double(e_min);
  const double inv_T = 1.0 / Tg[a], M = double(2 * nu - n_spins);
  double r = 0.0, xm = -INFINITY;
  for (int c = lane; c < nh; c += 64) {
    const double x = (hg[c] * M - E0) * inv_T - logz[a * nh + c];
    xm = fmax(xm, x);
    const double gc = G[a * nh + c];
    if (gc != 0.0) r = fma(gc, exp(x), r);
  }
  r = wave_sum(r);
  xm = wave_max(xm);
  if (lane == 0) {
    R[w] = r;
    X[w] = xm;
  }
}

__global__ __launch_bounds__(256) void k_weight_combine(
    const unsigned long long *__restrict__ g, int n_e, int n_m, int e_min, int n_spins,
    const double *__restrict__ Tg, int nT, const double *__restrict__ hg, int nh,
    const double *__restrict__ logz, const double *__restrict__ G, const double *__restrict__ R,
    const double *__restrict__ X, double *__restrict__ W) {
  const int lane = threadIdx.x & 63;
  const int waves = int(gridDim.x * (blockDim.x / 64));
  for (int i = int(blockIdx.x * (blockDim.x / 64) + threadIdx.x / 64); i < n_e * n_m; i += waves) {
    if (!g[i]) {   // uniform over the wave
      if (lane == 0) W[i] = 0.0;
      continue;
    }
    const int e = i / n_m, nu = i - e * n_m;
    const double E = double(e + e_min), M = double(2 * nu - n_spins);
    const double E0 = double(e_min);
    double acc = 0.0;
    for (int a = lane; a < nT; a += 64) {
      const double inv_T = 1.0 / Tg[a];
      const double x1 = -(E - E0) * inv_T;        // <= 0
      const double xm = X[a * n_m + nu];           // largest second exponent of (a, n_up)
      double term;
      if (xm <= 600.0 && (x1 >= -600.0 || x1 + xm < -700.0)) {
        term = exp(x1) * R[a * n_m + nu];
      } else {   // direct: the exponent in one piece
        term = 0.0;
        for (int c = 0; c < nh; ++c) {
          const double gc = G[a * nh + c];
          if (gc != 0.0) term = fma(gc, exp(-(E - hg[c] * M) * inv_T - logz[a * nh + c]), term);
        }
      }
      acc = fma(term, inv_T, acc);
    }
    acc = wave_sum(acc);
    if (lane == 0) W[i] = acc;
  }
}

ising_status bin_weights_launch(const uint64_t *g, int32_t n_e, int32_t n_m, int32_t e_min, int32_t n_spins,
                                const double *T_dev, int32_t nT, const double *h_dev, int32_t nh,
                                const double *logz, const double *G, double *W, double *scratch,
                                hipStream_t stream) {
  // scratch: nT * n_m doubles (R), then nT * n_m doubles (X)
  double *R = scratch, *X = scratch + size_t(nT) * n_m;
  const int waves = nT * n_m;
  hipLaunchKernelGGL(k_weight_factors, dim3(unsigned((waves + 3) / 4)), dim3(256), 0, stream, n_m, e_min, n_spins,
                     T_dev, nT, h_dev, nh, logz, G, R, X);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(ISING_EHIP, std::string("k_weight_factors launch: ") + hipGetErrorString(e));
  const int bins = n_e * n_m;
  const int blocks = std::min((bins + 3) / 4, 65536);   // four waves per block, one bin each
  hipLaunchKernelGGL(k_weight_combine, dim3(unsigned(blocks)), dim3(256), 0, stream,
                     reinterpret_cast<const unsigned long long *>(g), n_e, n_m, e_min, n_spins, T_dev, nT, h_dev,
                     nh, logz, G, R, X, W);
  e = hipGetLastError();
  if (e != hipSuccess) return fail(ISING_EHIP, std::string("k_weight_combine launch: ") + hipGetErrorString(e));
  return ISING_OK;
}

size_t bin_weights_scratch_bytes(int32_t nT, int32_t n_m) { return size_t(2) * nT * n_m * sizeof(double); }

// First derivatives of log Z for the backward, with the log Z of the
// forward as normaliser (one pass, no max pass): block (a, f) covers the
// temperature T_a and fields 8 f .. 8 f + 7, two per wave; the table's
// nonzero bins are staged in LDS; per field, with p = g exp(-(E - hM)/T -
// log Z) over the bins: d_T = (sum p H / sum p) / T^2, d_h = (sum p M / sum p)
// / T, the sums over a wave's lanes in a fixed shuffle tree.  Tables with
// more nonzero bins than the stage holds are read in place.
constexpr int kFirstFields = 8;

template <class Bins>
__device__ void first_points(const Bins &B, double T, const double *__restrict__ hg, const double *__restrict__ lz,
                             int c0, int cnt, double *__restrict__ d_T, double *__restrict__ d_h, int pt0) {
  const int lane = threadIdx.x & 63;
  const int bins = B.count();
  const double inv_T = (T > 0.0 && isfinite(T)) ? 1.0 / T : 0.0;
  double hv[2], lzv[2], s0[2] = {0.0, 0.0}, sH[2] = {0.0, 0.0}, sM[2] = {0.0, 0.0};
#pragma unroll
  for (int j = 0; j < 2; ++j) {
    hv[j] = j < cnt ? hg[c0 + j] : 0.0;
    lzv[j] = j < cnt ? lz[pt0 + j] : 0.0;
  }
  for (int i = lane; i < bins; i += 64) {
    double lg, E, M;
    if (!B.get(i, lg, E, M)) continue;
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const double H = E - hv[j] * M;
      const double p = exp(lg - H * inv_T - lzv[j]);
      s0[j] += p;
      sH[j] += p * H;
      sM[j] += p * M;
    }
  }
#pragma unroll
  for (int j = 0; j < 2; ++j) {
    s0[j] = wave_sum(s0[j]);
    sH[j] = wave_sum(sH[j]);
    sM[j] = wave_sum(sM[j]);
  }
  if (lane != 0) return;
#pragma unroll
  for (int j = 0; j < 2; ++j) {
    if (j >= cnt) break;
    const bool ok = (T > 0.0) && isfinite(T) && isfinite(hv[j]) && isfinite(lzv[j]);
    d_T[pt0 + j] = ok ? (sH[j] / s0[j]) * inv_T * inv_T : NAN;
    d_h[pt0 + j] = ok ? (sM[j] / s0[j]) * inv_T : NAN;
  }
}

__global__ __launch_bounds__(kThermoThreads) void k_first_derivatives(
    const unsigned long long *__restrict__ g, int n_e, int n_m, int e_min, int n_spins,
    const double *__restrict__ Tg, int nT, const double *__restrict__ hg, int nh, const double *__restrict__ logz,
    double *__restrict__ d_T, double *__restrict__ d_h) {
  __shared__ StageLds L;
  const int a = blockIdx.x;
  const int staged = stage_bins(g, n_e, n_m, e_min, n_spins, L.lg, L.E, L.M, L.scan);
  const int c0 = blockIdx.y * kFirstFields + 2 * int(threadIdx.x / 64);
  if (c0 >= nh) return;
  const int cnt = min(2, nh - c0), pt0 = a * nh + c0;
  if (staged >= 0)
    first_points(StagedBins{L.lg, L.E, L.M, staged}, Tg[a], hg, logz, c0, cnt, d_T, d_h, pt0);
  else
    first_points(DenseBins{g, n_m, e_min, n_spins, n_e * n_m}, Tg[a], hg, logz, c0, cnt, d_T, d_h, pt0);
}

ising_status first_derivatives_launch(const uint64_t *g, int32_t n_e, int32_t n_m, int32_t e_min, int32_t n_spins,
                                      const double *T_dev, int32_t nT, const double *h_dev, int32_t nh,
                                      const double *logz, double *d_T, double *d_h, hipStream_t stream) {
  if (nT == 0 || nh == 0) return ISING_OK;
  const dim3 grid(unsigned(nT), unsigned((nh + kFirstFields - 1) / kFirstFields));
  if (grid.y > 65535) return fail(ISING_EINVAL, "too many field values");
  hipLaunchKernelGGL(k_first_derivatives, grid, dim3(kThermoThreads), 0, stream,
                     reinterpret_cast<const unsigned long long *>(g), n_e, n_m, e_min, n_spins, T_dev, nT, h_dev,
                     nh, logz, d_T, d_h);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(ISING_EHIP, std::string("k_first_derivatives launch: ") + hipGetErrorString(e));
  return ISING_OK;
}

// Batched: grid (ceil(nT / 4), members); wave w of block (x, member) takes
// temperature 4 x + w and every field group in turn; outputs
// [member][nT][nh].
__global__ __launch_bounds__(kThermoThreads) void k_batch_thermo(
    const unsigned long long *__restrict__ g_all, const BatchMember *__restrict__ meta,
    const double *__restrict__ Tg, int nT, const double *__restrict__ hg, int nh,
    double *__restrict__ logz, double *__restrict__ mean_E, double *__restrict__ mean_M,
    double *__restrict__ heat, double *__restrict__ susc) {
  __shared__ StageLds L;
  const int member = blockIdx.y;
  const BatchMember mb = meta[member];
  const ThermoOut o{logz, mean_E, mean_M, heat, susc, nullptr, nullptr, nullptr, nullptr, nullptr};
  const unsigned long long *g = g_all + mb.offset;
  const int staged = stage_bins(g, mb.n_e, mb.n_m, mb.e_min, mb.n_spins, L.lg, L.E, L.M, L.scan);
  const int a = int(blockIdx.x) * kWavesPerBlock + int(threadIdx.x / 64);
  if (a >= nT) return;
  for (int c0 = 0; c0 < nh; c0 += kWaveFields) {
    const int cnt = min(kWaveFields, nh - c0), pt0 = (member * nT + a) * nh + c0;
    if (staged >= 0)
      wave_points(StagedBins{L.lg, L.E, L.M, staged}, Tg[a], hg + c0, cnt, pt0, o);
    else
      wave_points(DenseBins{g, mb.n_m, mb.e_min, mb.n_spins, mb.n_e * mb.n_m}, Tg[a], hg + c0, cnt, pt0, o);
  }
}

ising_status batch_thermo_launch(const BatchMember *meta_dev, int n_members, const uint64_t *g_all,
                                 const double *T_dev, int32_t nT, const double *h_dev, int32_t nh, double *logz,
                                 double *mE, double *mM, double *C, double *chi, hipStream_t stream) {
  if (nT == 0 || nh == 0 || n_members == 0) return ISING_OK;
  if (!T_dev || !h_dev) return fail(ISING_EINVAL, "T_dev or h_dev is NULL");
  if (int64_t(nT) * nh > (int64_t(1) << 30) || n_members > 65535) return fail(ISING_EINVAL, "grid too large");
  hipLaunchKernelGGL(k_batch_thermo, dim3(unsigned((nT + kWavesPerBlock - 1) / kWavesPerBlock), unsigned(n_members)),
                     dim3(kThermoThreads), 0,
                     stream, reinterpret_cast<const unsigned long long *>(g_all), meta_dev, T_dev, nT, h_dev, nh,
                     logz, mE, mM, C, chi);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(ISING_EHIP, std::string("k_batch_thermo launch: ") + hipGetErrorString(e));
  return ISING_OK;
}

// Contraction of per-point first derivatives with a loss gradient G over the
// grid, for the backward of L = sum G log Z: wave a < nT writes
// grad_T[a] = sum_c G[a][c] d_T[a][c], wave nT + c writes
// grad_h[c] = sum_a G[a][c] d_h[a][c]; lane l adds the terms l, l + 64, ...
// in order, then a fixed shuffle tree adds the lanes.
__global__ __launch_bounds__(256) void k_grid_contract(const double *__restrict__ G, const double *__restrict__ d_T,
                                                       const double *__restrict__ d_h, int nT, int nh,
                                                       double *__restrict__ grad_T, double *__restrict__ grad_h) {
  const int w = int(blockIdx.x * blockDim.x + threadIdx.x) / 64, lane = threadIdx.x & 63;
  double s = 0.0;
  if (w < nT) {
    if (!grad_T) return;
    for (int c = lane; c < nh; c += 64) s = fma(G[w * nh + c], d_T[w * nh + c], s);
  } else if (w < nT + nh) {
    if (!grad_h) return;
    const int c = w - nT;
    for (int a = lane; a < nT; a += 64) s = fma(G[a * nh + c], d_h[a * nh + c], s);
  } else {
    return;
  }
  s = wave_sum(s);
  if (lane == 0) (w < nT ? grad_T[w] : grad_h[w - nT]) = s;
}

ising_status grid_contract_launch(const double *G, const double *d_T, const double *d_h, int nT, int nh,
                                  double *grad_T, double *grad_h, hipStream_t stream) {
  if (nT + nh == 0) return ISING_OK;
  const int waves = nT + nh, blocks = (waves + 3) / 4;   // 4 waves per block
  hipLaunchKernelGGL(k_grid_contract, dim3(unsigned(blocks)), dim3(256), 0, stream, G, d_T, d_h, nT, nh, grad_T,
                     grad_h);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(ISING_EHIP, std::string("k_grid_contract launch: ") + hipGetErrorString(e));
  return ISING_OK;
}

static ising_status check_table(const uint64_t *g_dev, int32_t n_e, int32_t n_m, int32_t n_spins, int32_t nT,
                                int32_t nh) {
  if (!g_dev) return fail(ISING_EINVAL, "g_dev is NULL");
  if (n_spins < 1 || n_spins > kMaxSpins) return fail(ISING_ETOO_MANY_SPINS, "n_spins must be 1..64");
  if (n_m != n_spins + 1) return fail(ISING_EINVAL, "n_m must equal n_spins + 1");
  if (n_e < 1 || int64_t(n_e) * n_m > (int64_t(1) << 30)) return fail(ISING_EINVAL, "bad n_e");
  if (nT < 0 || nh < 0) return fail(ISING_EINVAL, "negative grid size");
  if (int64_t(nT) * nh > (int64_t(1) << 30)) return fail(ISING_EINVAL, "grid too large");
  return ISING_OK;
}

static ising_status thermo_launch(const uint64_t *g_dev, int32_t n_e, int32_t n_m, int32_t e_min, int32_t n_spins,
                                  const double *T_dev, int32_t nT, const double *h_dev, int32_t nh,
                                  const ThermoOut &o, void *stream) {
  ising_status st = check_table(g_dev, n_e, n_m, n_spins, nT, nh);
  if (st != ISING_OK) return st;
  if (nT == 0 || nh == 0) return ISING_OK;
  if (!T_dev || !h_dev) return fail(ISING_EINVAL, "T_dev or h_dev is NULL");
  const int64_t waves = int64_t(nT) * ((nh + kWaveFields - 1) / kWaveFields);
  const dim3 grid(unsigned((waves + kWavesPerBlock - 1) / kWavesPerBlock));
  hipLaunchKernelGGL(k_thermo, grid, dim3(kThermoThreads), 0, static_cast<hipStream_t>(stream),
                     reinterpret_cast<const unsigned long long *>(g_dev), n_e, n_m, e_min, n_spins, T_dev, nT,
                     h_dev, nh, o);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(ISING_EHIP, std::string("k_thermo launch: ") + hipGetErrorString(e));
  return ISING_OK;
}

}  // namespace ising

using namespace ising;

extern "C" ising_status ising_logz(const uint64_t *g_dev, int32_t n_e, int32_t n_m, int32_t e_min, int32_t n_spins,
                                   const double *T_dev, int32_t nT, const double *h_dev, int32_t nh,
                                   double *logz_dev, void *stream) {
  if (!logz_dev && nT > 0 && nh > 0) return fail(ISING_EINVAL, "logz_dev is NULL");
  const ThermoOut o{logz_dev, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr};
  return thermo_launch(g_dev, n_e, n_m, e_min, n_spins, T_dev, nT, h_dev, nh, o, stream);
}

extern "C" ising_status ising_moments(const uint64_t *g_dev, int32_t n_e, int32_t n_m, int32_t e_min,
                                      int32_t n_spins, const double *T_dev, int32_t nT, const double *h_dev,
                                      int32_t nh, double *logz_dev, double *mean_E, double *mean_M,
                                      double *heat_capacity, double *susceptibility, void *stream) {
  const ThermoOut o{logz_dev, mean_E, mean_M, heat_capacity, susceptibility,
                    nullptr, nullptr, nullptr, nullptr, nullptr};
  return thermo_launch(g_dev, n_e, n_m, e_min, n_spins, T_dev, nT, h_dev, nh, o, stream);
}

extern "C" ising_status ising_logz_derivatives(const uint64_t *g_dev, int32_t n_e, int32_t n_m, int32_t e_min,
                                               int32_t n_spins, const double *T_dev, int32_t nT,
                                               const double *h_dev, int32_t nh, double *logz_dev, double *d_T,
                                               double *d_h, double *d_TT, double *d_Th, double *d_hh,
                                               void *stream) {
  const ThermoOut o{logz_dev, nullptr, nullptr, nullptr, nullptr, d_T, d_h, d_TT, d_Th, d_hh};
  return thermo_launch(g_dev, n_e, n_m, e_min, n_spins, T_dev, nT, h_dev, nh, o, stream);
}

extern "C" ising_status ising_bin_weights(const uint64_t *g_dev, int32_t n_e, int32_t n_m, int32_t e_min,
                                          int32_t n_spins, const double *T_dev, int32_t nT, const double *h_dev,
                                          int32_t nh, const double *logz_dev, const double *grad_dev,
                                          double *W_dev, void *stream) {
  ising_status st = check_table(g_dev, n_e, n_m, n_spins, nT, nh);
  if (st != ISING_OK) return st;
  if (!W_dev) return fail(ISING_EINVAL, "W_dev is NULL");
  if (nT > 0 && nh > 0 && (!T_dev || !h_dev || !logz_dev || !grad_dev))
    return fail(ISING_EINVAL, "T_dev, h_dev, logz_dev or grad_dev is NULL");
  const int bins = n_e * n_m;
  const int blocks = std::min(bins, 65536);
  hipLaunchKernelGGL(k_bin_weights, dim3(unsigned(blocks)), dim3(256), 0, static_cast<hipStream_t>(stream),
                     reinterpret_cast<const unsigned long long *>(g_dev), n_e, n_m, e_min, n_spins, T_dev,
                     nT > 0 && nh > 0 ? nT : 0, h_dev, nT > 0 && nh > 0 ? nh : 0, logz_dev, grad_dev, W_dev);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(ISING_EHIP, std::string("k_bin_weights launch: ") + hipGetErrorString(e));
  return ISING_OK;
}
