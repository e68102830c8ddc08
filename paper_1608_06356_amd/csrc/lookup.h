// Rate and inverse-CDF lookups shared by the step kernels.  R = float for the
// mixed-precision path (float32 ln h, 16-bit quantile codes staged in LDS),
// R = double for the float64 path (float64 master tables in global memory).
#pragma once
#include "qed_device.h"

namespace qed {

// Upper ends of the chi ranges of the tables (the lower ends are fixed at 1e-3
// for photon emission and 1e-2 for pairs); chosen when the tables are built.
struct TabRange {
  double rad_hi = kRadChiMax, pair_hi = kPairChiMax;
};

// ln chi grid positions: x = (ln chi - ln chi_min) / step
template <typename R> struct Grid {
  static __device__ __forceinline__ R pos(R lnchi, double lo, double hi, int n) {
    const double step = (log(hi) - log(lo)) / (n - 1);
    return (lnchi - (R)log(lo)) / (R)step;
  }
};

// Photon rate h(chi): linear in (ln chi, ln h) between nodes; small-chi expansion
// c1 chi (1 - c2 chi) below, chi^(2/3) growth above; 0 for chi <= 0.
template <typename R>
__device__ __forceinline__ R h_rad(R chi, const R *lnh, const TabRange &rg) {
  if (!(chi > (R)0)) return (R)0;
  if (chi < (R)kRadChiMin) return (R)kHc1 * chi * ((R)1 - (R)kHc2 * chi);
  if (chi > (R)rg.rad_hi)
    return exp(lnh[kRadNChi - 1] + (R)(2.0 / 3.0) * log(chi / (R)rg.rad_hi));
  const R x = Grid<R>::pos(log(chi), kRadChiMin, rg.rad_hi, kRadNChi);
  int i = (int)floor(x);
  i = i < 0 ? 0 : (i > kRadNChi - 2 ? kRadNChi - 2 : i);
  const R f = x - (R)i;
  return exp(((R)1 - f) * lnh[i] + f * lnh[i + 1]);
}

// Pair rate h_pair(chi) from L = ln h_pair + 8/(3 chi); 0 below chi = 1e-2.
template <typename R>
__device__ __forceinline__ R h_pair(R chi, const R *L, const TabRange &rg) {
  if (!(chi >= (R)kPairChiMin)) return (R)0;
  if (chi > (R)rg.pair_hi)
    return exp(L[kPairNRate - 1] - (R)(8.0 / (3.0 * rg.pair_hi)) + (R)(2.0 / 3.0) * log(chi / (R)rg.pair_hi));
  const R x = Grid<R>::pos(log(chi), kPairChiMin, rg.pair_hi, kPairNRate);
  int i = (int)floor(x);
  i = i < 0 ? 0 : (i > kPairNRate - 2 ? kPairNRate - 2 : i);
  const R f = x - (R)i;
  return exp(((R)1 - f) * L[i] + f * L[i + 1] - (R)8 / ((R)3 * chi));
}

// Row of a 256-row table: linear interpolation of the CDF in ln chi realised by
// taking row i+1 with probability equal to the fractional position.
template <typename R>
__device__ __forceinline__ int pick_row(R lnchi, R u_row, double lo, double hi) {
  const R x = Grid<R>::pos(lnchi, lo, hi, 256);
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
__device__ __forceinline__ bool interp_s(const Tab &tab, int row, R u, double ulo, double uhi, R &s) {
  const double tlo = log(ulo) - log1p(-ulo), thi = log(uhi) - log1p(-uhi);
  const double dt = (thi - tlo) / (kNU - 1);
  const R t = log(u) - log1p(-u);
  const R y = (t - (R)tlo) / (R)dt;
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
  const int row = pick_row<R>(lnchi, u_row, kRadChiMin, rg.rad_hi);
  R s;
  if (interp_s<R>(tab, row, u, kRadULo, kRadUHi, s)) {
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
  const int row = pick_row<R>(log(chi), u_row, kPairChiMin, rg.pair_hi);
  R s;
  if (!interp_s<R>(tab, row, u, kPairULo, kPairUHi, s)) s = (R)tab.at(row, 0);
  xi = (R)1 / ((R)1 + exp(-s));
  om = (R)1 / ((R)1 + exp(s));
}

}  // namespace qed
