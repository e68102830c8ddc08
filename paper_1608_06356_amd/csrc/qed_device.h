// Device helpers of the QED Monte Carlo step on gfx950: constants, Philox4x32-10,
// quantum parameters (Eqs. 2-3), Boris push, quadratic-spline gather, table
// lookups, and the single-pass decoupled look-back prefix scan used by every
// append.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace qed {

// ---------------------------------------------------------------- constants
// E_S = m_e c^2 / (hbar omega_0) at lambda_0 = 1 um (the value the paper's Fig. 1
// triples imply); alpha from CODATA 2018.  Units: m_e c omega_0 / e, 1/omega_0.
constexpr double kMeC2eV = 510998.95;
constexpr double kHcEvUm = 1.239841984;
constexpr double kES = kMeC2eV / kHcEvUm;
constexpr double kAlpha = 1.0 / 137.035999084;
constexpr double kInvES = 1.0 / kES;
constexpr double kRateUnit = kAlpha * kES;          // alpha m c^2 / hbar in omega_0
constexpr double kPi = 3.14159265358979323846;

// Table layout (identical on every path; see qed.h, qed_build_tables).
constexpr int kRadNChi = 256;
constexpr double kRadChiMin = 1e-3, kRadChiMax = 1e2;   // default range
constexpr double kMlpChiMax = 1e2;                       // surrogate domain [1e-3, 1e2]
constexpr int kRadM = 1024;
constexpr double kRadXiLoOverChi = 1e-15;
constexpr double kRadDHi = 40.0;
constexpr int kNU = 256;                       // quantile nodes per row (both tables)
constexpr double kRadULo = 1e-4, kRadUHi = 1.0 - 1e-7;
constexpr int kPairNRate = 512, kPairNCdf = 256;
constexpr double kPairChiMin = 1e-2, kPairChiMax = 1e2;  // default range
constexpr double kRadChiMaxLo = 1.0, kPairChiMaxLo = 10.0, kChiMaxHi = 1e6;  // allowed upper ends
constexpr int kPairM = 1024;
constexpr double kPairDD = 45.0;
constexpr double kPairULo = 1e-6, kPairUHi = 1.0 - 1e-6;
// small-chi expansion of the photon rate below the table: h = c1 chi (1 - c2 chi)
constexpr double kHc1 = 1.4433756729740644;    // 5 / (2 sqrt 3)
constexpr double kHc2 = 0.9237604307034013;    // 8 sqrt 3 / 15

constexpr uint64_t kDeadId = ~0ull;
enum Purpose : uint32_t { kInitTau = 0, kLeptonEvent = 1, kPhotonEvent = 2, kLeptonThin = 5, kPhotonThin = 6 };

// counters (layout of qed_counters_t)
enum Counter { cEvents = 0, cPhotons, cRejected, cCapped, cPairs, cDropped, cChiRange,
               cNanChi, cScanTimeout, cCompacted, cMlpFallbackXi, cMlpFallbackRate, cThinned,
               cEnvelopeExceeded, cRetired, cBoxFallback, cNumCounters };

// ------------------------------------------------------------------ Philox
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): 10 rounds of two 32x32->64
// multiplications with the round keys advanced by the Weyl constants.
__device__ __forceinline__ uint4 philox4x32_10(uint4 c, uint2 k) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r) { k.x += 0x9E3779B9u; k.y += 0xBB67AE85u; }
    const uint32_t lo0 = 0xD2511F53u * c.x, hi0 = __umulhi(0xD2511F53u, c.x);
    const uint32_t lo1 = 0xCD9E8D57u * c.z, hi1 = __umulhi(0xCD9E8D57u, c.z);
    c = make_uint4(hi1 ^ c.y ^ k.x, lo1, hi0 ^ c.w ^ k.y, lo0);
  }
  return c;
}

__device__ __forceinline__ uint4 stream4(uint64_t id, uint32_t seed, uint64_t step,
                                         uint32_t purpose, uint32_t k) {
  const uint2 key = make_uint2((uint32_t)id, (uint32_t)(id >> 32) ^ seed);
  const uint4 ctr = make_uint4((uint32_t)step,
                               ((uint32_t)(step >> 32) & 0x00FFFFFFu) | (purpose << 24), k, 0u);
  return philox4x32_10(ctr, key);
}

// u = ((x >> 9) + 0.5) 2^-23: exact in float and double, never 0 or 1.
template <typename R> __device__ __forceinline__ R unit(uint32_t x) {
  return ((R)(x >> 9) + (R)0.5) * (R)1.1920928955078125e-07;
}

// ---------------------------------------------------------------- chi
// Eq. (2) rearranged without subtraction of nearly equal squares: with n = p/|p|,
// beta = |p|/gamma and 1 - beta = 1 / (gamma^2 (1 + beta)),
//   (E + v x B)^2 - (v.E)^2 = (n.E)^2 / gamma^2 + |n x (E + beta n x B)|^2,
//   E + beta n x B = (E + n x B) - (n x B) / (gamma^2 (1 + beta)).
__device__ __forceinline__ double chi_lepton(double px, double py, double pz,
                                             double ex, double ey, double ez,
                                             double bx, double by, double bz) {
  const double p2 = px * px + py * py + pz * pz;
  if (p2 == 0.0) return sqrt(ex * ex + ey * ey + ez * ez) * kInvES;   // at rest: chi = |E| / E_S
  const double pa = sqrt(p2), g2 = 1.0 + p2, g = sqrt(g2);
  const double ipa = 1.0 / pa;
  const double nx = px * ipa, ny = py * ipa, nz = pz * ipa;
  const double cx = ny * bz - nz * by, cy = nz * bx - nx * bz, cz = nx * by - ny * bx;  // n x B
  const double f = 1.0 / (g * (g + pa));          // 1 / (gamma^2 (1 + beta))
  const double wx = (ex + cx) - cx * f, wy = (ey + cy) - cy * f, wz = (ez + cz) - cz * f;
  const double ux = ny * wz - nz * wy, uy = nz * wx - nx * wz, uz = nx * wy - ny * wx;  // n x w
  const double ne = nx * ex + ny * ey + nz * ez;
  return sqrt(g2 * (ux * ux + uy * uy + uz * uz) + ne * ne) * kInvES;
}

// Float64 square root and reciprocal from the float32 hardware estimates
// (relative error below 2^-22) refined by two float64 Newton steps, which
// square the error each time: below 1e-15 relative, for a fraction of the
// instructions of the correctly rounded float64 sequences.  Arguments outside
// [1e-30, 1e30] (float32 range of the estimate) take those sequences.
__device__ __forceinline__ double sqrt_nr(double s) {
  if (!(s >= 1e-30 && s <= 1e30)) return sqrt(s);
  double y = (double)__builtin_amdgcn_rsqf((float)s);      // 1 / sqrt(s)
  y = fma(0.5 * y, fma(-s * y, y, 1.0), y);
  y = fma(0.5 * y, fma(-s * y, y, 1.0), y);
  return s * y;
}
__device__ __forceinline__ double rcp_nr(double d) {
  if (!(d >= 1e-30 && d <= 1e30)) return 1.0 / d;
  double y = (double)__builtin_amdgcn_rcpf((float)d);
  y = fma(y, fma(-d, y, 1.0), y);
  y = fma(y, fma(-d, y, 1.0), y);
  return y;
}

// The same expression for the float32 step, whose inputs (p, E, B) are float32
// and therefore exact in float64: every operation is float64.  Only 1/|p|
// starts from the float32 reciprocal square root, refined by two float64 Newton
// steps (relative error below 1e-15), which saves the float64 division there;
// gamma, 1/(gamma^2 (1 + beta)) and the final root likewise (sqrt_nr, rcp_nr).
// Where E and -n x B nearly cancel, n must be exact to float64 rounding: it is.
// |p|^2 below 1e-30 (float32 underflow of the estimate) takes the form above.
__device__ __forceinline__ double chi_lepton_f32(float px, float py, float pz, const float F[6]) {
  const double dx = px, dy = py, dz = pz;
  const double p2 = dx * dx + dy * dy + dz * dz;
  if (!(p2 >= 1e-30)) return chi_lepton(dx, dy, dz, F[0], F[1], F[2], F[3], F[4], F[5]);
  double y = (double)__builtin_amdgcn_rsqf((float)p2);
  y = fma(0.5 * y, fma(-p2 * y, y, 1.0), y);
  y = fma(0.5 * y, fma(-p2 * y, y, 1.0), y);
  const double nx = dx * y, ny = dy * y, nz = dz * y;
  const double ex = F[0], ey = F[1], ez = F[2], bx = F[3], by = F[4], bz = F[5];
  const double cx = ny * bz - nz * by, cy = nz * bx - nx * bz, cz = nx * by - ny * bx;  // n x B
  const double g2 = 1.0 + p2, g = sqrt_nr(g2);
  const double f = rcp_nr(g * (g + p2 * y));      // 1 / (gamma^2 (1 + beta))
  const double wx = (ex + cx) - cx * f, wy = (ey + cy) - cy * f, wz = (ez + cz) - cz * f;
  const double ux = ny * wz - nz * wy, uy = nz * wx - nx * wz, uz = nx * wy - ny * wx;  // n x w
  const double ne = nx * ex + ny * ey + nz * ez;
  return sqrt_nr(g2 * (ux * ux + uy * uy + uz * uz) + ne * ne) * kInvES;
}

// Upper bound of chi_e (Eq. 2) in float32 arithmetic, for the envelope of the
// thinned lepton pass, which needs a bound and not the value (the candidates'
// chi is evaluated in float64 where they are finished).  With a = gamma E + p x B
// and s = p.E, chi E_S = sqrt(|a|^2 - s^2) for the same inputs.  With u = 2^-24,
// each component of a is off by at most 6u times the sum A of the magnitudes of
// its three terms (gamma = sqrt(1 + p^2) itself within 3u), s by at most 3u
// times its own such sum S, so |a|^2 - s^2 is within 17u (A_x^2 + A_y^2 + A_z^2
// + S^2) of the exact value (|a_x| <= A_x, |s| <= S); 32u times that sum is
// added before the root, whose rounding and the scaling are covered by a factor
// 1 + 2^-20.  Where E and -v x B nearly cancel
// the bound exceeds chi by up to ~1e-3 gamma |E| / E_S, elsewhere by ~1e-6
// relative.
__device__ __forceinline__ float chi_lepton_upper_f32(float px, float py, float pz, float g, const float F[6]) {
  const float ex = F[0], ey = F[1], ez = F[2], bx = F[3], by = F[4], bz = F[5];
  const float ax = g * ex + (py * bz - pz * by), ay = g * ey + (pz * bx - px * bz),
              az = g * ez + (px * by - py * bx);
  const float s = px * ex + py * ey + pz * ez;
  const float Ax = fabsf(g * ex) + fabsf(py * bz) + fabsf(pz * by);
  const float Ay = fabsf(g * ey) + fabsf(pz * bx) + fabsf(px * bz);
  const float Az = fabsf(g * ez) + fabsf(px * by) + fabsf(py * bx);
  const float S = fabsf(px * ex) + fabsf(py * ey) + fabsf(pz * ez);
  const float T = ax * ax + ay * ay + az * az - s * s;
  const float D = 0x1p-19f * (Ax * Ax + Ay * Ay + Az * Az + S * S);
  return __builtin_amdgcn_sqrtf(fmaxf(T + D, 0.f)) * (float)(kInvES * (1.0 + 0x1p-20));
}

// Eq. (3) for the float32 step (inputs k, E, B float32, exact in float64), all
// in float64 like chi_lepton_f32: k^ from the refined reciprocal square root,
// gamma_ph = |k| = k^2 / |k|, E + k^ x B and the (refined) root in float64.
__device__ __forceinline__ double chi_photon_f32(float kx, float ky, float kz, const float F[6]) {
  const double dx = kx, dy = ky, dz = kz;
  const double k2 = dx * dx + dy * dy + dz * dz;
  if (!(k2 >= 1e-30)) return 0.0;
  double y = (double)__builtin_amdgcn_rsqf((float)k2);
  y = fma(0.5 * y, fma(-k2 * y, y, 1.0), y);
  y = fma(0.5 * y, fma(-k2 * y, y, 1.0), y);
  const double nx = dx * y, ny = dy * y, nz = dz * y;
  const double bx = F[3], by = F[4], bz = F[5];
  const double wx = (double)F[0] + (ny * bz - nz * by), wy = (double)F[1] + (nz * bx - nx * bz),
               wz = (double)F[2] + (nx * by - ny * bx);
  const double ux = ny * wz - nz * wy, uy = nz * wx - nx * wz, uz = nx * wy - ny * wx;
  return k2 * y * sqrt_nr(ux * ux + uy * uy + uz * uz) * kInvES;
}

// Eq. (3) with |v| = 1: chi_ph = gamma_ph / E_S |k^ x (E + k^ x B)|.
__device__ __forceinline__ double chi_photon(double kx, double ky, double kz,
                                             double ex, double ey, double ez,
                                             double bx, double by, double bz) {
  const double g = sqrt(kx * kx + ky * ky + kz * kz);
  if (!(g > 0.0)) return 0.0;
  const double ig = 1.0 / g;
  const double nx = kx * ig, ny = ky * ig, nz = kz * ig;
  const double wx = ex + (ny * bz - nz * by), wy = ey + (nz * bx - nx * bz), wz = ez + (nx * by - ny * bx);
  const double ux = ny * wz - nz * wy, uy = nz * wx - nx * wz, uz = nx * wy - ny * wx;
  return g * sqrt(ux * ux + uy * uy + uz * uz) * kInvES;
}

// Square root: the hardware instruction (1 ulp) in float32, correctly rounded in float64.
template <typename R> __device__ __forceinline__ R root(R x);
template <> __device__ __forceinline__ float root<float>(float x) { return __builtin_amdgcn_sqrtf(x); }
template <> __device__ __forceinline__ double root<double>(double x) { return sqrt(x); }

// Reciprocal: the hardware estimate (1 ulp) in float32, exact division in float64.
template <typename R> __device__ __forceinline__ R rcp(R x);
template <> __device__ __forceinline__ float rcp<float>(float x) { return __builtin_amdgcn_rcpf(x); }
template <> __device__ __forceinline__ double rcp<double>(double x) { return 1.0 / x; }

// ---------------------------------------------------------------- push
// Relativistic Boris rotation (p in m_e c, q in units of e).
template <typename R>
__device__ __forceinline__ void boris(R &px, R &py, R &pz, R ex, R ey, R ez, R bx, R by, R bz,
                                      R q, R dt) {
  const R h = (R)0.5 * q * dt;
  R mx = px + h * ex, my = py + h * ey, mz = pz + h * ez;
  const R hg = h * rcp<R>(root<R>((R)1 + mx * mx + my * my + mz * mz));
  const R tx = hg * bx, ty = hg * by, tz = hg * bz;
  const R ax = mx + (my * tz - mz * ty), ay = my + (mz * tx - mx * tz), az = mz + (mx * ty - my * tx);
  const R s = (R)2 * rcp<R>((R)1 + tx * tx + ty * ty + tz * tz);
  const R sx = s * tx, sy = s * ty, sz = s * tz;
  mx += ay * sz - az * sy;
  my += az * sx - ax * sz;
  mz += ax * sy - ay * sx;
  px = mx + h * ex; py = my + h * ey; pz = mz + h * ez;
}

// ------------------------------------------------------- device-wide scan
// Single-pass prefix scan with decoupled look-back (Merrill & Garland 2016).
// Tiles take increasing ids from an atomic ticket, so every tile a later tile
// waits on is held by a workgroup that is already running.  Status word:
// bits 62-63 flag (1 = tile aggregate, 2 = inclusive prefix), bits 0-61 value.
// Flag and value travel in one 64-bit word, so the status accesses are relaxed
// device-scope atomics: acquire/release at device scope would write back or
// invalidate the whole (per-XCD, non-coherent) L2 on every spin.  Callers that
// need their own loads finished before publishing wait for them explicitly.
constexpr uint64_t kFlagAgg = 1ull << 62, kFlagPre = 2ull << 62, kValMask = (1ull << 62) - 1;
constexpr uint32_t kSpinLimit = 1u << 24;

__device__ __forceinline__ uint64_t ld_status(const uint64_t *p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_status(uint64_t *p, uint64_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ uint64_t wave_sum_u64(uint64_t v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Called by all 64 lanes of one wave; returns the exclusive prefix of `tile`
// (same value in every lane) and publishes the tile's inclusive prefix.
__device__ uint64_t lookback_scan(uint64_t *status, uint32_t tile, uint64_t agg,
                                  unsigned long long *timeouts) {
  const int lane = threadIdx.x & 63;
  if (tile == 0) {
    if (lane == 0) st_status(&status[0], kFlagPre | agg);
    return 0;
  }
  if (lane == 0) st_status(&status[tile], kFlagAgg | agg);
  uint64_t excl = 0;
  int64_t j = (int64_t)tile - 1;
  while (true) {
    const int64_t idx = j - lane;
    uint64_t s = idx >= 0 ? ld_status(&status[idx]) : kFlagPre;
    uint32_t spins = 0;
    while (__any((s >> 62) == 0)) {
      if ((s >> 62) == 0) {
        __builtin_amdgcn_s_sleep(1);
        s = ld_status(&status[idx]);
        if (++spins > kSpinLimit && (s >> 62) == 0) {
          atomicAdd(timeouts, 1ull);
          s = kFlagPre;              // give up: treat as zero so the wave exits
        }
      }
    }
    const uint64_t pre = __ballot((s >> 62) == 2);
    if (pre) {
      const int first = __ffsll((long long)pre) - 1;
      excl += wave_sum_u64(lane <= first ? (s & kValMask) : 0);
      break;
    }
    excl += wave_sum_u64(s & kValMask);
    j -= 64;
  }
  if (lane == 0) st_status(&status[tile], kFlagPre | (excl + agg));
  return excl;
}

// Workgroup-level exclusive scan of per-thread counts (blockDim multiple of 64,
// at most 1024 threads); `lds` holds >= 16 uint32.  Returns the thread's
// exclusive prefix within the workgroup; *total gets the workgroup sum.
__device__ __forceinline__ uint32_t block_exclusive(uint32_t v, uint32_t *lds, uint32_t *total) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
  uint32_t incl = v;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const uint32_t t = __shfl_up(incl, o, 64);
    if (lane >= o) incl += t;
  }
  if (lane == 63) lds[wave] = incl;
  __syncthreads();
  uint32_t base = 0, tot = 0;
  for (int w = 0; w < nw; ++w) {
    const uint32_t x = lds[w];
    if (w < wave) base += x;
    tot += x;
  }
  __syncthreads();
  *total = tot;
  return base + incl - v;
}

// The same scan for 64-bit values (blockDim multiple of 64, at most 1024
// threads); `lds` holds >= 16 uint64.
__device__ __forceinline__ uint64_t block_exclusive64(uint64_t v, uint64_t *lds, uint64_t *total) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
  uint64_t incl = v;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const uint64_t t = __shfl_up(incl, o, 64);
    if (lane >= o) incl += t;
  }
  if (lane == 63) lds[wave] = incl;
  __syncthreads();
  uint64_t base = 0, tot = 0;
  for (int w = 0; w < nw; ++w) {
    const uint64_t x = lds[w];
    if (w < wave) base += x;
    tot += x;
  }
  __syncthreads();
  *total = tot;
  return base + incl - v;
}

}  // namespace qed
