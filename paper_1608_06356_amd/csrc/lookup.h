// Rate and inverse-CDF lookups shared by the step kernels.  R = float for the
// mixed-precision path (float32 ln h, 16-bit quantile codes staged in LDS),
// R = double for the float64 path (float64 master tables in global memory).
#pragma once
#include "qed_device.h"

namespace qed {

// Node grids of the tables, computed once on the host when the tables are
// built: chi nodes log-spaced from 1e-3 (photon) or 1e-2 (pair) to an upper end
// chosen by the caller, quantile nodes uniform in t = logit(u).  A position on a
// grid is (coordinate - origin) * inverse spacing.
struct TabRange {
  double rad_hi, pair_hi;
  double rad_lnlo, rad_inv;                      // 256 photon chi nodes
  double pair_lnlo, pair_rate_inv, pair_cdf_inv;   // 512 pair-rate and 256 pair-CDF nodes
  double rad_tlo, rad_tinv, pair_tlo, pair_tinv;   // 256 quantile nodes each
};

__host__ __device__ inline TabRange make_range(double rad_hi, double pair_hi) {
  TabRange r;
  r.rad_hi = rad_hi;
  r.pair_hi = pair_hi;
  r.rad_lnlo = log(kRadChiMin);
  r.rad_inv = (kRadNChi - 1) / (log(rad_hi) - log(kRadChiMin));
  r.pair_lnlo = log(kPairChiMin);
  r.pair_rate_inv = (kPairNRate - 1) / (log(pair_hi) - log(kPairChiMin));
  r.pair_cdf_inv = (kPairNCdf - 1) / (log(pair_hi) - log(kPairChiMin));
  r.rad_tlo = log(kRadULo) - log1p(-kRadULo);
  r.rad_tinv = (kNU - 1) / ((log(kRadUHi) - log1p(-kRadUHi)) - r.rad_tlo);
  r.pair_tlo = log(kPairULo) - log1p(-kPairULo);
  r.pair_tinv = (kNU - 1) / ((log(kPairUHi) - log1p(-kPairUHi)) - r.pair_tlo);
  return r;
}

// ln and exp: Fast selects the hardware log2/exp2 instructions in float32
// (relative error ~1e-6 after the change of base), for the rate of the push.
template <typename R, bool Fast> struct Math {
  static __device__ __forceinline__ R ln(R v) { return log(v); }
  static __device__ __forceinline__ R ex(R v) { return exp(v); }
};
template <> struct Math<float, true> {
  static __device__ __forceinline__ float ln(float v) { return __logf(v); }
  static __device__ __forceinline__ float ex(float v) { return __expf(v); }
};

// Photon rate h(chi): linear in (ln chi, ln h) between nodes; small-chi expansion
// c1 chi (1 - c2 chi) below, chi^(2/3) growth above; 0 for chi <= 0.
template <typename R, bool Fast = false>
__device__ __forceinline__ R h_rad(R chi, const R *lnh, const TabRange &rg) {
  using M = Math<R, Fast>;
  if (!(chi > (R)0)) return (R)0;
  if (chi < (R)kRadChiMin) return (R)kHc1 * chi * ((R)1 - (R)kHc2 * chi);
  if (chi > (R)rg.rad_hi)
    return M::ex(lnh[kRadNChi - 1] + (R)(2.0 / 3.0) * M::ln(chi / (R)rg.rad_hi));
  const R x = (M::ln(chi) - (R)rg.rad_lnlo) * (R)rg.rad_inv;
  int i = (int)floor(x);
  i = i < 0 ? 0 : (i > kRadNChi - 2 ? kRadNChi - 2 : i);
  const R f = x - (R)i;
  return M::ex(((R)1 - f) * lnh[i] + f * lnh[i + 1]);
}

// Pair rate h_pair(chi) from L = ln h_pair + 8/(3 chi); 0 below chi = 1e-2.
// Fast (float32): hardware log/exp and reciprocal.
template <typename R, bool Fast = false>
__device__ __forceinline__ R h_pair(R chi, const R *L, const TabRange &rg) {
  using M = Math<R, Fast>;
  if (!(chi >= (R)kPairChiMin)) return (R)0;
  if (chi > (R)rg.pair_hi)
    return M::ex(L[kPairNRate - 1] - (R)(8.0 / (3.0 * rg.pair_hi)) + (R)(2.0 / 3.0) * M::ln(chi / (R)rg.pair_hi));
  const R x = (M::ln(chi) - (R)rg.pair_lnlo) * (R)rg.pair_rate_inv;
  int i = (int)floor(x);
  i = i < 0 ? 0 : (i > kPairNRate - 2 ? kPairNRate - 2 : i);
  const R f = x - (R)i;
  R inv3chi;
  if constexpr (Fast) inv3chi = __builtin_amdgcn_rcpf((R)3 * chi);
  else inv3chi = (R)1 / ((R)3 * chi);
  return M::ex(((R)1 - f) * L[i] + f * L[i + 1] - (R)8 * inv3chi);
}

// Envelopes of the total rates for Poisson thinning (the surrogate path):
// closed forms that lie above the rates everywhere, so that candidate events
// drawn at the envelope rate and kept with probability h / h_env are exactly
// events of the true rate.  Photons: h_rad <= (5 / (2 sqrt3)) chi
// (1 + chi)^(-1/3) (the small-chi law c1 chi times a factor that turns it into
// the chi^(2/3) growth); pairs: h_pair <= C chi exp(-8 / (3 chi)) (1 + chi/4)^(-1/3)
// with Erber's C = 3 sqrt3 / (16 sqrt2), zero below chi = 1e-2 like the table.
// Both carry a factor 1.002 above the tabulated rates, whose ratio to the
// bare forms stays within [0.90, 0.99999] (photons) and [0.93, 0.9992] (pairs)
// over chi in [1e-5, 1e4].
constexpr double kEnvMargin = 1.002;
// Lower bound of rate / envelope (both envelopes, over the same chi range):
// a candidate whose keep draw u is below it is kept without evaluating the rate
// (the squeeze of rejection sampling), which is exact as long as the rate used
// also stays above it (the surrogate's rates are within 1e-3 of the table's).
constexpr double kEnvSqueeze = 0.89;
constexpr double kErberC = 0.22963966338592295;   // 3 sqrt3 / (16 sqrt2)
__device__ __forceinline__ float h_rad_env(float chi) {
  if (!(chi > 0.f)) return 0.f;
  return (float)(kEnvMargin * kHc1) * chi * __builtin_amdgcn_exp2f(-(1.0f / 3.0f) * __builtin_amdgcn_logf(1.f + chi));
}
__device__ __forceinline__ float h_pair_env(float chi) {
  if (!(chi >= (float)kPairChiMin)) return 0.f;
  const float e = -(8.0f / 3.0f) * __builtin_amdgcn_rcpf(chi) * 1.4426950408889634f
                  - (1.0f / 3.0f) * __builtin_amdgcn_logf(1.f + 0.25f * chi);
  return (float)(kEnvMargin * kErberC) * chi * __builtin_amdgcn_exp2f(e);
}

// Row of a 256-row table: linear interpolation of the CDF in ln chi realised by
// taking row i+1 with probability equal to the fractional position.
template <typename R>
__device__ __forceinline__ int pick_row(R lnchi, R u_row, double lnlo, double inv) {
  const R x = (lnchi - (R)lnlo) * (R)inv;
  int i = (int)floor(x);
  i = i < 0 ? 0 : (i > 254 ? 254 : i);
  const R f = x - (R)i;
  int row = i + (u_row < f ? 1 : 0);
  if (x < (R)0) row = 0;
  if (x >= (R)255) row = 255;
  return row;
}

// Table row accessor: float64 master or 16-bit codes s = s0 + q * scale.
struct RowF64 {
  const double *S;
  __device__ __forceinline__ double at(int row, int j) const { return S[row * kNU + j]; }
};
struct RowQ16 {
  const uint16_t *q;
  const float *s0sc;
  __device__ __forceinline__ float at(int row, int j) const {
    return s0sc[2 * row] + (float)q[row * kNU + j] * s0sc[2 * row + 1];
  }
};

// logit(xi) at quantile u: linear in t = logit(u) between the 256 nodes.
// Returns false in the low tail (t < t_lo), where the caller applies its tail law.
template <typename R, typename Tab>
__device__ __forceinline__ bool interp_s(const Tab &tab, int row, R u, double tlo, double tinv, R &s) {
  const R t = log(u) - log1p(-u);
  const R y = (t - (R)tlo) * (R)tinv;
  if (y < (R)0) return false;
  if (y >= (R)(kNU - 1)) { s = (R)tab.at(row, kNU - 1); return true; }
  int j = (int)floor(y);
  j = j > kNU - 2 ? kNU - 2 : j;
  const R f = y - (R)j;
  s = ((R)1 - f) * (R)tab.at(row, j) + f * (R)tab.at(row, j + 1);
  return true;
}

// Photon energy fraction xi (and 1 - xi) from the emission inverse CDF (Eq. 7).
// Below the table's chi range the row-0 sample is scaled by chi / chi_min (the
// classical spectrum depends on xi/chi); above it the last row is used; below
// u = 1e-4 the infrared law xi ~ u^3 continues the first node.
template <typename R, typename Tab>
__device__ __forceinline__ void sample_rad(const Tab &tab, R chi, R u, R u_row, R &xi, R &om, const TabRange &rg) {
  const R lnchi = log(chi);
  const int row = pick_row<R>(lnchi, u_row, rg.rad_lnlo, rg.rad_inv);
  R s;
  if (interp_s<R>(tab, row, u, rg.rad_tlo, rg.rad_tinv, s)) {
    xi = (R)1 / ((R)1 + exp(-s));
    om = (R)1 / ((R)1 + exp(s));
  } else {
    const R xi0 = (R)1 / ((R)1 + exp(-(R)tab.at(row, 0)));
    const R r = u / (R)kRadULo;
    xi = xi0 * r * r * r;
    om = (R)1 - xi;
  }
  if (chi < (R)kRadChiMin) {
    xi = xi * (chi / (R)kRadChiMin);
    om = (R)1 - xi;
  }
}

// Half-spectrum sample xi in (0, 1/2] of the pair spectrum (Eq. 6), chi >= 1e-2.
template <typename R, typename Tab>
__device__ __forceinline__ void sample_pair_half(const Tab &tab, R chi, R u, R u_row, R &xi, R &om,
                                                 const TabRange &rg) {
  const int row = pick_row<R>(log(chi), u_row, rg.pair_lnlo, rg.pair_cdf_inv);
  R s;
  if (!interp_s<R>(tab, row, u, rg.pair_tlo, rg.pair_tinv, s)) s = (R)tab.at(row, 0);
  xi = (R)1 / ((R)1 + exp(-s));
  om = (R)1 / ((R)1 + exp(s));
}

}  // namespace qed
