// Table builder: total rates and inverse CDFs of the photon spectrum (Eq. 1 or
// Eq. 4) and of the pair spectrum (Eq. 6), by float64 quadrature on the GPU.
//
// K_nu(x) = int_0^inf exp(-x cosh t) cosh(nu t) dt and its tail integral
// int_x^inf K_nu = int_0^inf exp(-x cosh t) cosh(nu t) / cosh t dt (DLMF 10.32.9)
// by the trapezoid rule with step min(0.1, 0.35/sqrt(x)) up to cosh t = 1 + 40/x.
// Per chi row: density in s = logit(xi) on 1024 uniform intervals, 3-point
// Gauss-Legendre per interval, cumulative sum, infrared tail below the grid
// (photons), quantiles at 256 nodes uniform in logit(u) from the cubic Hermite
// interpolant of the cumulative spectrum (52 bisections per node).
#include <hip/hip_runtime.h>
#include <math.h>

#include "internal.h"
#include "qed_device.h"

namespace qed {
namespace {

constexpr double kInvSqrt3Pi = 0.18377629847393068;   // 1 / (sqrt3 pi)
constexpr double kGamma23 = 1.3541179394264004;        // Gamma(2/3)
enum Kind { kFormulaI = 1, kFormulaII = 2, kPair = 3, kClassical = 4 };
constexpr int kPts = 4 * 1024 + 1;                     // 3M Gauss points + M+1 nodes

struct Job {
  int kind;
  int out;        // 0: rad row, 1: pair rate node, 2: pair CDF row
  int row;
  double chi, s_lo, s_hi, tail;
};

// (K_{2/3}(x), int_x^inf K_{1/3}) sharing exp(-x cosh t).
__device__ void bessel_k23_i13(double x, double &k23, double &i13) {
  const double h = fmin(0.1, 0.35 / sqrt(x));
  const int n = (int)ceil(acosh(1.0 + 40.0 / x) / h);
  double a = 0.5 * exp(-x), b = a;
  for (int j = 1; j <= n; ++j) {
    const double t = j * h, ch = cosh(t), e = exp(-x * ch);
    a += e * cosh((2.0 / 3.0) * t);
    b += e * cosh((1.0 / 3.0) * t) / ch;
  }
  k23 = h * a;
  i13 = h * b;
}

// (K_{1/3}(x), K_{2/3}(x)).
__device__ void bessel_k13_k23(double x, double &k13, double &k23) {
  const double h = fmin(0.1, 0.35 / sqrt(x));
  const int n = (int)ceil(acosh(1.0 + 40.0 / x) / h);
  double a = 0.5 * exp(-x), b = a;
  for (int j = 1; j <= n; ++j) {
    const double t = j * h, e = exp(-x * cosh(t));
    a += e * cosh((1.0 / 3.0) * t);
    b += e * cosh((2.0 / 3.0) * t);
  }
  k13 = h * a;
  k23 = h * b;
}

// int_x^inf K_{5/3}.
__device__ double bessel_i53(double x) {
  const double h = fmin(0.1, 0.35 / sqrt(x));
  const int n = (int)ceil(acosh(1.0 + 40.0 / x) / h);
  double a = 0.5 * exp(-x);
  for (int j = 1; j <= n; ++j) {
    const double t = j * h, ch = cosh(t);
    a += exp(-x * ch) * cosh((5.0 / 3.0) * t) / ch;
  }
  return h * a;
}

// J_1..J_3 of Eq. (4) after u = sigma cosh^3(theta): trapezoid in theta with step
// min(0.08, 0.3/sqrt(sigma)) up to sigma cosh^3 = sigma + 22.5.
__device__ void j_integrals(double sigma, double &j1, double &j2, double &j3) {
  const double h = fmin(0.08, 0.3 / sqrt(sigma));
  const double thmax = acosh(pow(1.0 + 22.5 / sigma, 1.0 / 3.0));
  const int n = (int)ceil(thmax / h);
  double a = 0, b = 0, c = 0;
  for (int j = 0; j <= n; ++j) {
    const double th = j * h, ch = cosh(th), sh = sinh(th);
    double k13, k23;
    bessel_k13_k23(sigma * ch * ch * ch, k13, k23);
    const double w = j ? 1.0 : 0.5;
    const double c3 = ch * ch * ch, c5 = c3 * ch * ch;
    a += w * c5 * k23 * k23;
    b += w * c3 * sh * sh * k13 * k13;
    c += w * c5 * k13 * k13;
  }
  j1 = h * a; j2 = h * b; j3 = h * c;
}

// Density in s: S(xi, chi) xi (1 - xi), S normalised so dW/dxi = alpha E_S S / gamma.
__device__ double density(int kind, double s, double chi) {
  const double xi = 1.0 / (1.0 + exp(-s));
  const double om = 1.0 / (1.0 + exp(s));
  double S;
  if (kind == kFormulaI) {                                      // Eq. (1)
    const double d = (2.0 / 3.0) * exp(s) / chi;
    double k23, i13;
    bessel_k23_i13(d, k23, i13);
    S = kInvSqrt3Pi * ((om + 1.0 / om) * k23 - i13);
  } else if (kind == kFormulaII) {                              // Eq. (4)
    const double sigma = exp(s) / (3.0 * chi);
    double j1, j2, j3;
    j_integrals(sigma, j1, j2, j3);
    const double f1 = 1.0 + 1.0 / (om * om), f2 = 2.0 / om, f3 = (xi / om) * (xi / om);
    S = xi / (3.0 * kPi * kPi * chi) * (f1 * j1 + f2 * j2 + f3 * j3);
  } else if (kind == kClassical) {                              // Eq. (5), z = 2 xi / (3 chi)
    const double z = (2.0 / 3.0) * xi / chi;
    S = 1.7320508075688772 * chi / (2.0 * kPi * xi) * z * bessel_i53(z);
  } else {                                                      // Eq. (6), "+" sign
    const double d = 2.0 / (3.0 * xi * om * chi);
    double k23, i13;
    bessel_k23_i13(d, k23, i13);
    S = kInvSqrt3Pi * ((1.0 / xi + 1.0 / om - 2.0) * k23 + i13);
  }
  return S * xi * om;
}

__device__ __forceinline__ double point_s(const Job &jb, int p, double ds) {
  const int M = 1024;
  if (p < 3 * M) {
    const int m = p / 3, g = p - 3 * m;
    const double x = g == 0 ? 0.5 - 0.5 * sqrt(0.6) : (g == 1 ? 0.5 : 0.5 + 0.5 * sqrt(0.6));
    return (jb.s_lo + m * ds) + ds * x;
  }
  return jb.s_lo + (p - 3 * M) * ds;
}

__global__ void k_density(const Job *jobs, int njobs, double *dens) {
  const int64_t total = (int64_t)njobs * kPts;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int j = (int)(i / kPts), p = (int)(i - (int64_t)j * kPts);
    const Job jb = jobs[j];
    if (jb.out == 1 && p >= 3 * 1024) { dens[i] = 0.0; continue; }   // rate-only row
    const double ds = (jb.s_hi - jb.s_lo) / 1024;
    dens[i] = density(jb.kind, point_s(jb, p, ds), jb.chi);
  }
}

__device__ __forceinline__ double hermite(double tau, double p0, double p1, double d0, double d1,
                                          double ds) {
  const double t2 = tau * tau, t3 = t2 * tau;
  return (2 * t3 - 3 * t2 + 1) * p0 + (t3 - 2 * t2 + tau) * ds * d0 + (-2 * t3 + 3 * t2) * p1 +
         (t3 - t2) * ds * d1;
}

struct TabOut {
  double *rad_lnh, *rad_S, *pair_L, *pair_S;
  float *chk;
  double rad_tlo, rad_dt, pair_tlo, pair_dt;
};

// One workgroup of 256 threads per job.
__global__ __launch_bounds__(256) void k_rows(const Job *jobs, const double *dens, TabOut o) {
  constexpr int M = 1024;
  __shared__ double F[M + 1];
  const Job jb = jobs[blockIdx.x];
  const double *d = dens + (int64_t)blockIdx.x * kPts;
  const double ds = (jb.s_hi - jb.s_lo) / M;
  if (threadIdx.x == 0) {
    const double w0 = 5.0 / 18.0, w1 = 8.0 / 18.0;
    double acc = jb.tail;
    F[0] = acc;
    for (int m = 0; m < M; ++m) {
      const double I = ds * (w0 * d[3 * m] + w1 * d[3 * m + 1] + w0 * d[3 * m + 2]);
      acc = acc + I;
      F[m + 1] = acc;
    }
  }
  __syncthreads();
  const double total = F[M];
  if (jb.out == 1) {
    if (threadIdx.x == 0) o.pair_L[jb.row] = log(2.0 * total) + 8.0 / (3.0 * jb.chi);
    return;
  }
  if (jb.out == 0 && threadIdx.x == 0) o.rad_lnh[jb.row] = log(total);
  const bool rad = jb.out == 0;
  if (rad && threadIdx.x < 40) {
    // residual-check row of the surrogate: P and dP/ds at 40 nodes uniform in s
    // over the fine grid, from the fine cubic Hermite interpolant
    constexpr int NC = 40;
    const double dsc = (jb.s_hi - jb.s_lo) / (NC - 1);
    const double sc = jb.s_lo + threadIdx.x * dsc;
    int m = (int)floor((sc - jb.s_lo) / ds);
    m = m < 0 ? 0 : (m > M - 1 ? M - 1 : m);
    const double tau = (sc - (jb.s_lo + m * ds)) / ds;
    const double p0 = F[m] / total, p1 = F[m + 1] / total;
    const double r0 = d[3 * M + m] / total, r1 = d[3 * M + m + 1] / total;
    const double t2 = tau * tau, t3 = t2 * tau;
    const double P = (2 * t3 - 3 * t2 + 1) * p0 + (t3 - 2 * t2 + tau) * ds * r0 + (-2 * t3 + 3 * t2) * p1 + (t3 - t2) * ds * r1;
    const double dP = ((6 * t2 - 6 * tau) * p0 + (3 * t2 - 4 * tau + 1) * ds * r0 + (-6 * t2 + 6 * tau) * p1 +
                       (3 * t2 - 2 * tau) * ds * r1) / ds;
    float *row = o.chk + jb.row * (2 + 2 * NC);
    if (threadIdx.x == 0) { row[0] = (float)jb.s_lo; row[1] = (float)dsc; }
    row[2 + 2 * threadIdx.x] = (float)P;
    row[3 + 2 * threadIdx.x] = (float)dP;
  }
  const int k = threadIdx.x;
  const double t = rad ? o.rad_tlo + k * o.rad_dt : o.pair_tlo + k * o.pair_dt;
  const double u = 1.0 / (1.0 + exp(-t));
  const double *rho = d + 3 * M;
  double s;
  if (u <= F[0] / total) {
    if (rad) {
      const double xi_lo = 1.0 / (1.0 + exp(-jb.s_lo));
      const double xi = xi_lo * pow(u / (F[0] / total), 3.0);
      s = log(xi) - log1p(-xi);
    } else {
      s = jb.s_lo;
    }
  } else if (u >= F[M] / total) {
    s = jb.s_hi;
  } else {
    // largest m with P[m] <= u
    int lo = 0, hi = M;           // P[lo] <= u < P[hi]
    while (hi - lo > 1) {
      const int mid = (lo + hi) >> 1;
      if (F[mid] / total <= u) lo = mid; else hi = mid;
    }
    const int m = lo;
    const double p0 = F[m] / total, p1 = F[m + 1] / total;
    const double d0 = rho[m] / total, d1 = rho[m + 1] / total;
    double a = 0.0, b = 1.0;
    for (int it = 0; it < 52; ++it) {
      const double mid = 0.5 * (a + b);
      if (hermite(mid, p0, p1, d0, d1, ds) < u) a = mid; else b = mid;
    }
    s = (jb.s_lo + m * ds) + 0.5 * (a + b) * ds;
  }
  (rad ? o.rad_S : o.pair_S)[jb.row * kNU + k] = s;
}

// 16-bit per-row copies and float32 rates.
__global__ void k_quantize(const double *S, uint16_t *q, float *s0sc, int rows) {
  const int r = blockIdx.x, k = threadIdx.x;
  if (r >= rows) return;
  const double a = S[r * kNU], b = S[r * kNU + kNU - 1];
  const double step = (b - a) / 65535.0;
  double v = rint((S[r * kNU + k] - a) / step);
  v = fmin(fmax(v, 0.0), 65535.0);
  q[r * kNU + k] = (uint16_t)v;
  if (k == 0) { s0sc[2 * r] = (float)a; s0sc[2 * r + 1] = (float)step; }
}

__global__ void k_to_f32(const double *a, float *b, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) b[i] = (float)a[i];
}

double chi_node(int i, int n, double lo, double hi) {
  return exp(log(lo) + i * ((log(hi) - log(lo)) / (n - 1)));
}

}  // namespace

hipError_t launch_build_tables(qed_ctx *c, int formula, TabRange rg, hipStream_t st) {
  const int kind_rad = formula == QED_FORMULA_II ? kFormulaII : (formula == QED_FORMULA_CLASSICAL ? kClassical : kFormulaI);
  const int njobs = kRadNChi + kPairNRate + kPairNCdf;
  Job *h = new Job[njobs];
  int n = 0;
  for (int i = 0; i < kRadNChi; ++i) {
    const double chi = chi_node(i, kRadNChi, kRadChiMin, rg.rad_hi);
    const double xi_lo = kRadXiLoOverChi * chi;
    const double tail = kInvSqrt3Pi * 3.0 * kGamma23 * pow(3.0 * chi, 2.0 / 3.0) * pow(xi_lo, 1.0 / 3.0);
    h[n++] = Job{kind_rad, 0, i, chi, log(xi_lo) - log1p(-xi_lo), log(1.5 * kRadDHi * chi), tail};
  }
  auto pair_lo = [](double chi) {
    const double q = 2.0 / (8.0 + 3.0 * chi * kPairDD);
    const double xi_lo = 2.0 * q / (1.0 + sqrt(1.0 - 4.0 * q));
    return log(xi_lo) - log1p(-xi_lo);
  };
  for (int i = 0; i < kPairNRate; ++i) {
    const double chi = chi_node(i, kPairNRate, kPairChiMin, rg.pair_hi);
    h[n++] = Job{kPair, 1, i, chi, pair_lo(chi), 0.0, 0.0};
  }
  for (int i = 0; i < kPairNCdf; ++i) {
    const double chi = chi_node(i, kPairNCdf, kPairChiMin, rg.pair_hi);
    h[n++] = Job{kPair, 2, i, chi, pair_lo(chi), 0.0, 0.0};
  }
  hipError_t e;
  Job *dj = nullptr;
  if ((e = hipMallocAsync((void **)&dj, sizeof(Job) * njobs, st)) != hipSuccess) { delete[] h; return e; }
  e = hipMemcpyAsync(dj, h, sizeof(Job) * njobs, hipMemcpyHostToDevice, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);   // h is freed below
  delete[] h;
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_density, dim3(4096), dim3(256), 0, st, dj, njobs, c->tab_work);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  TabOut o;
  o.rad_lnh = c->rad_lnh64; o.rad_S = c->rad_S64; o.pair_L = c->pair_L64; o.pair_S = c->pair_S64;
  o.chk = c->rad_chk;
  const double rtlo = log(kRadULo) - log1p(-kRadULo), rthi = log(kRadUHi) - log1p(-kRadUHi);
  const double ptlo = log(kPairULo) - log1p(-kPairULo), pthi = log(kPairUHi) - log1p(-kPairUHi);
  o.rad_tlo = rtlo; o.rad_dt = (rthi - rtlo) / (kNU - 1);
  o.pair_tlo = ptlo; o.pair_dt = (pthi - ptlo) / (kNU - 1);
  hipLaunchKernelGGL(k_rows, dim3(njobs), dim3(256), 0, st, dj, c->tab_work, o);
  hipLaunchKernelGGL(k_quantize, dim3(kRadNChi), dim3(kNU), 0, st, c->rad_S64, c->rad_q16, c->rad_s0sc, kRadNChi);
  hipLaunchKernelGGL(k_quantize, dim3(kPairNCdf), dim3(kNU), 0, st, c->pair_S64, c->pair_q16, c->pair_s0sc, kPairNCdf);
  hipLaunchKernelGGL(k_to_f32, dim3(1), dim3(256), 0, st, c->rad_lnh64, c->rad_lnh32, kRadNChi);
  hipLaunchKernelGGL(k_to_f32, dim3(2), dim3(256), 0, st, c->pair_L64, c->pair_L32, kPairNRate);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  return hipFreeAsync(dj, st);
}

}  // namespace qed
