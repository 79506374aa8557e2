// FP64 evaluation of the partition function (Peretyatko et al., Section 2,
// Eq. (2)) and its moments and derivatives from a dense degeneracy table on
// the device.
//
// Grouping the configurations of Eq. (2) by (E, M):
//   Z(T, h) = sum_{E,M} g(E, M) exp(-(E - h M)/T),  H = E - h M (Eq. (1)).
// One block per (T, h) point:
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

// Block-wide sums of up to 3 values; every thread gets the totals.
__device__ __forceinline__ void block_sum3(double &a, double &b, double &c, double *sh) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, nw = blockDim.x >> 6;
  a = wave_sum(a); b = wave_sum(b); c = wave_sum(c);
  __syncthreads();
  if (lane == 0) { sh[wv] = a; sh[8 + wv] = b; sh[16 + wv] = c; }
  __syncthreads();
  a = b = c = 0.0;
  for (int w = 0; w < nw; ++w) { a += sh[w]; b += sh[8 + w]; c += sh[16 + w]; }
}

__device__ __forceinline__ double block_max(double v, double *sh) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, nw = blockDim.x >> 6;
  v = wave_max(v);
  __syncthreads();
  if (lane == 0) sh[wv] = v;
  __syncthreads();
  v = -INFINITY;
  for (int w = 0; w < nw; ++w) v = fmax(v, sh[w]);
  return v;
}

// Output arrays of the FP64 evaluation; any may be NULL.
struct ThermoOut {
  double *logz, *mean_E, *mean_M, *heat, *susc;   // value and moments
  double *d_T, *d_h, *d_TT, *d_Th, *d_hh;         // derivatives of log Z
};

// All outputs of one (T, h) point of one table, written at index pt.
__device__ void thermo_point(const unsigned long long *__restrict__ g, int n_e, int n_m, int e_min, int n_spins,
                             double T, double h, int pt, const ThermoOut &o, double *sh) {
  const int bins = n_e * n_m;
  const bool want_second = o.heat || o.susc || o.d_TT || o.d_Th || o.d_hh;
  double *const all[10] = {o.logz, o.mean_E, o.mean_M, o.heat, o.susc, o.d_T, o.d_h, o.d_TT, o.d_Th, o.d_hh};
  if (!(T > 0.0) || !isfinite(T) || !isfinite(h)) {
    if (threadIdx.x == 0)
      for (int i = 0; i < 10; ++i)
        if (all[i]) all[i][pt] = NAN;
    return;
  }
  const double inv_T = 1.0 / T;

  // pass 1: the largest exponent
  double m = -INFINITY;
  for (int i = threadIdx.x; i < bins; i += blockDim.x) {
    const unsigned long long v = g[i];
    if (!v) continue;
    const int e = i / n_m, nu = i - e * n_m;
    const double E = double(e + e_min), M = double(2 * nu - n_spins);
    m = fmax(m, log(double(v)) - (E - h * M) * inv_T);
  }
  m = block_max(m, sh);
  if (m == -INFINITY) {   // empty table: Z = 0
    if (threadIdx.x == 0) {
      for (int i = 1; i < 10; ++i)
        if (all[i]) all[i][pt] = NAN;
      if (o.logz) o.logz[pt] = -INFINITY;
    }
    return;
  }

  // pass 2: Z' and first moments
  double z = 0.0, se = 0.0, sm = 0.0;
  for (int i = threadIdx.x; i < bins; i += blockDim.x) {
    const unsigned long long v = g[i];
    if (!v) continue;
    const int e = i / n_m, nu = i - e * n_m;
    const double E = double(e + e_min), M = double(2 * nu - n_spins);
    const double w = exp(log(double(v)) - (E - h * M) * inv_T - m);
    z += w;
    se += w * E;
    sm += w * M;
  }
  block_sum3(z, se, sm, sh);
  const double mE = se / z, mM = sm / z;
  const double mH = mE - h * mM;
  if (threadIdx.x == 0) {
    if (o.logz) o.logz[pt] = m + log(z);
    if (o.mean_E) o.mean_E[pt] = mE;
    if (o.mean_M) o.mean_M[pt] = mM;
    if (o.d_T) o.d_T[pt] = mH * inv_T * inv_T;
    if (o.d_h) o.d_h[pt] = mM * inv_T;
  }
  if (!want_second) return;

  // pass 3: centred second moments of H = E - hM and M
  double vh = 0.0, vm = 0.0, chm = 0.0;
  for (int i = threadIdx.x; i < bins; i += blockDim.x) {
    const unsigned long long v = g[i];
    if (!v) continue;
    const int e = i / n_m, nu = i - e * n_m;
    const double E = double(e + e_min), M = double(2 * nu - n_spins);
    const double w = exp(log(double(v)) - (E - h * M) * inv_T - m);
    const double dH = (E - h * M) - mH, dM = M - mM;
    vh += w * dH * dH;
    vm += w * dM * dM;
    chm += w * dH * dM;
  }
  block_sum3(vh, vm, chm, sh);
  if (threadIdx.x == 0) {
    const double varH = vh / z, varM = vm / z, cov = chm / z;
    const double T2 = inv_T * inv_T;
    if (o.heat) o.heat[pt] = varH * T2;
    if (o.susc) o.susc[pt] = varM * inv_T;
    if (o.d_TT) o.d_TT[pt] = varH * T2 * T2 - 2.0 * mH * T2 * inv_T;
    if (o.d_Th) o.d_Th[pt] = (cov * inv_T - mM) * T2;
    if (o.d_hh) o.d_hh[pt] = varM * T2;
  }
}

__global__ __launch_bounds__(kThermoThreads) void k_thermo(
    const unsigned long long *__restrict__ g, int n_e, int n_m, int e_min, int n_spins,
    const double *__restrict__ Tg, int nT, const double *__restrict__ hg, int nh, ThermoOut o) {
  __shared__ double sh[24];
  const int pt = blockIdx.x;
  const int ia = pt / nh, ib = pt - ia * nh;
  thermo_point(g, n_e, n_m, e_min, n_spins, Tg[ia], hg[ib], pt, o, sh);
}

// One thread per dense bin; the (T, h) points are summed in a fixed order.
__global__ __launch_bounds__(256) void k_bin_weights(
    const unsigned long long *__restrict__ g, int n_e, int n_m, int e_min, int n_spins,
    const double *__restrict__ Tg, int nT, const double *__restrict__ hg, int nh,
    const double *__restrict__ logz, const double *__restrict__ G, double *__restrict__ W) {
  const int bins = n_e * n_m;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < bins; i += gridDim.x * blockDim.x) {
    double acc = 0.0;
    if (g[i]) {
      const int e = i / n_m, nu = i - e * n_m;
      const double E = double(e + e_min), M = double(2 * nu - n_spins);
      for (int a = 0; a < nT; ++a) {
        const double inv_T = 1.0 / Tg[a];
        for (int c = 0; c < nh; ++c) {
          const double gc = G[a * nh + c];
          if (gc != 0.0) acc += gc * exp(-(E - hg[c] * M) * inv_T - logz[a * nh + c]) * inv_T;
        }
      }
    }
    W[i] = acc;
  }
}

// Batched: block (pt, member) evaluates point pt of member `member`; outputs
// are [member][nT][nh].
__global__ __launch_bounds__(kThermoThreads) void k_batch_thermo(
    const unsigned long long *__restrict__ g_all, const BatchMember *__restrict__ meta,
    const double *__restrict__ Tg, int nT, const double *__restrict__ hg, int nh,
    double *__restrict__ logz, double *__restrict__ mean_E, double *__restrict__ mean_M,
    double *__restrict__ heat, double *__restrict__ susc) {
  __shared__ double sh[24];
  const int pt = blockIdx.x, member = blockIdx.y;
  const int ia = pt / nh, ib = pt - ia * nh;
  const BatchMember mb = meta[member];
  const int out = member * nT * nh + pt;
  const ThermoOut o{logz, mean_E, mean_M, heat, susc, nullptr, nullptr, nullptr, nullptr, nullptr};
  thermo_point(g_all + mb.offset, mb.n_e, mb.n_m, mb.e_min, mb.n_spins, Tg[ia], hg[ib], out, o, sh);
}

ising_status batch_thermo_launch(const BatchMember *meta_dev, int n_members, const uint64_t *g_all,
                                 const double *T_dev, int32_t nT, const double *h_dev, int32_t nh, double *logz,
                                 double *mE, double *mM, double *C, double *chi, hipStream_t stream) {
  if (nT == 0 || nh == 0 || n_members == 0) return ISING_OK;
  if (!T_dev || !h_dev) return fail(ISING_EINVAL, "T_dev or h_dev is NULL");
  if (int64_t(nT) * nh > 65535 * 64) return fail(ISING_EINVAL, "grid too large");
  hipLaunchKernelGGL(k_batch_thermo, dim3(unsigned(nT * nh), unsigned(n_members)), dim3(kThermoThreads), 0, stream,
                     reinterpret_cast<const unsigned long long *>(g_all), meta_dev, T_dev, nT, h_dev, nh, logz, mE,
                     mM, C, chi);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(ISING_EHIP, std::string("k_batch_thermo launch: ") + hipGetErrorString(e));
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
  hipLaunchKernelGGL(k_thermo, dim3(unsigned(nT * nh)), dim3(kThermoThreads), 0, static_cast<hipStream_t>(stream),
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
  const int blocks = std::min((bins + 255) / 256, 4096);
  hipLaunchKernelGGL(k_bin_weights, dim3(unsigned(blocks)), dim3(256), 0, static_cast<hipStream_t>(stream),
                     reinterpret_cast<const unsigned long long *>(g_dev), n_e, n_m, e_min, n_spins, T_dev,
                     nT > 0 && nh > 0 ? nT : 0, h_dev, nT > 0 && nh > 0 ? nh : 0, logz_dev, grad_dev, W_dev);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(ISING_EHIP, std::string("k_bin_weights launch: ") + hipGetErrorString(e));
  return ISING_OK;
}
