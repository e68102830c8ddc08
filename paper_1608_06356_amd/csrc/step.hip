// Kernels of the QED Monte Carlo step on gfx950.
//
//   k_gather_push  every lepton: field, Boris push, x advance, chi (Eq. 2, float64),
//                  rate, optical depth; emitters appended (index order) to a list
//   k_emit         every emitter: inverse-CDF xi (Eq. 7), infrared cut, recoil,
//                  further events within the step, photons appended in order
//   k_pairs        every photon: chi_ph (Eq. 3), pair rate (Eq. 6), optical depth,
//                  electron/positron appended at the same rank, photon killed
//   k_compact      stable in-place removal of dead particles
// Every append is a wave ballot / workgroup scan plus a single-pass decoupled
// look-back across workgroups, so output order never depends on scheduling.
#include <hip/hip_runtime.h>
#include <limits.h>
#include <math.h>

#include "internal.h"
#include "lookup.h"
#include "mlp_device.h"
#include "qed_device.h"

namespace qed {

constexpr int kKmaxMax = 4;

struct SpeciesDev {
  void *x, *y, *z, *px, *py, *pz;
  double *tau;
  uint64_t *id;
  int64_t cap;
  int64_t *count;
};

struct FieldDev {
  int kind, nx, ny, nz;
  const float *grid;
  double dx, dy, dz;
  double idx, idy, idz;      // inverse cell sizes
  float fid[3];              // the same in float32
  double L[3];               // box lengths n * d
  float fL[3];
  double E[3], B[3];
  const float *pE[3], *pB[3];
};

constexpr int kGPThreads = 256;   // gather/push workgroup

struct ScanDev {
  uint32_t *ticket;
  uint64_t *status;
};

// --------------------------------------------------------------- fields
// x in [-L, 2L) -> [0, L) (one period at most per step); selects, no branches
template <typename R>
__device__ __forceinline__ void wrap_coord(R &x, R L) {
  const R lo = x + L, hi = x - L;
  x = x < (R)0 ? lo : (x >= L ? hi : x);
}

// Inverse cell size and box length of axis d in the arithmetic type R.
template <typename R> __device__ __forceinline__ R inv_cell(const FieldDev &f, int d);
template <> __device__ __forceinline__ float inv_cell<float>(const FieldDev &f, int d) { return f.fid[d]; }
template <> __device__ __forceinline__ double inv_cell<double>(const FieldDev &f, int d) {
  return d == 0 ? f.idx : (d == 1 ? f.idy : f.idz);
}
template <typename R> __device__ __forceinline__ R box_len(const FieldDev &f, int d);
template <> __device__ __forceinline__ float box_len<float>(const FieldDev &f, int d) { return f.fL[d]; }
template <> __device__ __forceinline__ double box_len<double>(const FieldDev &f, int d) { return f.L[d]; }

template <typename R>
__device__ __forceinline__ void weights_tsc(R x, R inv_d, int n, int &j, R w[3]) {
  const R g = x * inv_d;
  const R jf = floor(g + (R)0.5);
  const R t = g - jf, tt = t * t;
  const R h = (R)0.5 * tt + (R)0.125;     // (1/2)(1/2 -+ t)^2 = 1/8 -+ t/2 + t^2/2
  w[0] = h - (R)0.5 * t;
  w[1] = (R)0.75 - tt;
  w[2] = h + (R)0.5 * t;
  int jj = (int)jf;
  j = jj < 0 ? 0 : (jj > n ? n : jj);
}

// j in [-1, n+1] -> [0, n)
__device__ __forceinline__ int wrap_index(int j, int n) {
  j = j < 0 ? j + n : j;
  return j >= n ? j - n : j;
}

// Quadratic-spline (TSC) stencil of a position: centre node j per axis (in
// [0, n]; n stands for node 0) and the three weights of nodes j-1, j, j+1.
template <typename R>
__device__ __forceinline__ void tsc_setup(const FieldDev &f, R x, R y, R z, int j[3], R w[3][3]) {
  weights_tsc<R>(x, inv_cell<R>(f, 0), f.nx, j[0], w[0]);
  weights_tsc<R>(y, inv_cell<R>(f, 1), f.ny, j[1], w[1]);
  weights_tsc<R>(z, inv_cell<R>(f, 2), f.nz, j[2], w[2]);
}

// TSC gather from the grid in global memory.  Offsets are 32-bit float
// indices (the API limits a grid to 2^32 floats).
template <typename R>
__device__ __forceinline__ void gather_global(const FieldDev &f, const int j[3], const R w[3][3], R F[6]) {
  uint32_t ox[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) ox[a] = (uint32_t)wrap_index(j[0] + a - 1, f.nx) * 6u;
#pragma unroll
  for (int c = 0; c < 6; ++c) F[c] = (R)0;
  const uint32_t sy6 = (uint32_t)f.nx * 6u, sz6 = sy6 * (uint32_t)f.ny;
  uint32_t oy[3];
#pragma unroll
  for (int b = 0; b < 3; ++b) oy[b] = (uint32_t)wrap_index(j[1] + b - 1, f.ny) * sy6;
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const uint32_t oz = (uint32_t)wrap_index(j[2] + c - 1, f.nz) * sz6;
#pragma unroll
    for (int b = 0; b < 3; ++b) {
      const R wyz = w[1][b] * w[2][c];
      const uint32_t row = oz + oy[b];
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        const float2 *p2 = reinterpret_cast<const float2 *>(f.grid + (row + ox[a]));
        const float2 v0 = p2[0], v1 = p2[1], v2 = p2[2];
        const R wt = w[0][a] * wyz;
        F[0] += wt * (R)v0.x; F[1] += wt * (R)v0.y; F[2] += wt * (R)v1.x;
        F[3] += wt * (R)v1.y; F[4] += wt * (R)v2.x; F[5] += wt * (R)v2.y;
      }
    }
  }
}

template <typename R>
__device__ __forceinline__ void gather_grid(const FieldDev &f, R x, R y, R z, R F[6]) {
  int j[3];
  R w[3][3];
  tsc_setup<R>(f, x, y, z, j, w);
  gather_global<R>(f, j, w, F);
}

// ----------------------------------------------- gather staged through LDS
// The particles of a workgroup, ordered by cell, usually occupy a compact set
// of cells.  The workgroup copies the box of grid nodes their stencils touch
// (the span of their centre nodes, one node wider on each side) into LDS once
// and every particle reads its 27 nodes from there, which cuts the bytes the
// vector L1 returns per particle from 27 x 24 to about the box's share.  A
// workgroup whose box exceeds kBoxCap nodes gathers from global memory.
constexpr int kBoxCap = 1024;
constexpr int kGPWaves = 6;     // LDS allows 6 workgroups of 256 threads per CU

struct BoxLds {
  float2 node[kBoxCap * 3];     // 6 floats per node; node (x, y, z) at z * pxy + y * px + x
  int ref[3];                   // centre node of the workgroup's first particle
  int lo[3], hi[3];             // extremes of the centre nodes relative to ref
  int bad;                      // a particle's stencil left the box (then: global gather)
};

// j - ref wrapped into [-n/2, n - n/2) (j, ref in [0, n))
__device__ __forceinline__ int centred(int j, int ref, int n) {
  int r = j - ref;
  const int h = n >> 1;
  r -= r >= n - h ? n : 0;
  r += r < -h ? n : 0;
  return r;
}

// Minimum or maximum over each row of 16 lanes with DPP moves (quad
// permutations, half-row and row mirrors); every lane of a row gets its row's
// result.
template <bool Max>
__device__ __forceinline__ int row_extreme(int v) {
  const int id = Max ? INT_MIN : INT_MAX;
#define QED_DPP_STEP(ctrl)                                                        \
  {                                                                               \
    const int t = __builtin_amdgcn_update_dpp(id, v, ctrl, 0xF, 0xF, false);      \
    v = Max ? max(v, t) : min(v, t);                                              \
  }
  QED_DPP_STEP(0xB1)    // quad_perm [1,0,3,2]
  QED_DPP_STEP(0x4E)    // quad_perm [2,3,0,1]
  QED_DPP_STEP(0x141)   // row_half_mirror
  QED_DPP_STEP(0x140)   // row_mirror
#undef QED_DPP_STEP
  return v;
}

// Box of the workgroup.  Every thread calls it; live[it]: the thread holds
// particle it, with stencil centre j[it].  On success the box is in LDS, rel holds the
// thread's stencil corner (node j-1) in box coordinates and pit the row and
// plane pitches (odd, which spreads neighbouring rows and planes over the LDS
// banks).  Returns false (uniformly) when the box exceeds kBoxCap nodes.  Its
// first barrier also publishes whatever the caller wrote to LDS before.
template <int IT>
__device__ __forceinline__ bool stage_box(BoxLds &S, const FieldDev &f, const bool live[IT], const int j[IT][3],
                                          int rel[IT][3], int pit[2]) {
  const int n3[3] = {f.nx, f.ny, f.nz};
  int jj[IT][3];
#pragma unroll
  for (int it = 0; it < IT; ++it)
#pragma unroll
    for (int d = 0; d < 3; ++d) jj[it][d] = j[it][d] == n3[d] ? 0 : j[it][d];
  if (threadIdx.x == 0) {
#pragma unroll
    for (int d = 0; d < 3; ++d) { S.ref[d] = jj[0][d]; S.lo[d] = INT_MAX; S.hi[d] = INT_MIN; }
    S.bad = 0;
  }
  __syncthreads();
  // extremes over the thread's particles, then over each row of 16 lanes, then
  // one LDS atomic per row
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    int lo = INT_MAX, hi = INT_MIN;
#pragma unroll
    for (int it = 0; it < IT; ++it) {
      rel[it][d] = centred(jj[it][d], S.ref[d], n3[d]);
      if (live[it]) { lo = min(lo, rel[it][d]); hi = max(hi, rel[it][d]); }
    }
    lo = row_extreme<false>(lo);
    hi = row_extreme<true>(hi);
    if ((threadIdx.x & 15) == 0) { atomicMin(&S.lo[d], lo); atomicMax(&S.hi[d], hi); }
  }
  __syncthreads();
  int bmin[3], bdim[3], ref[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const int l = __builtin_amdgcn_readfirstlane(S.lo[d]);
    const int h = __builtin_amdgcn_readfirstlane(S.hi[d]);
    ref[d] = __builtin_amdgcn_readfirstlane(S.ref[d]);
    bmin[d] = l - 1;
    bdim[d] = h - l + 3;
  }
  const int px = bdim[0] | 1, pxy = (px * bdim[1]) | 1;
  if ((int64_t)pxy * bdim[2] > kBoxCap) return false;
  // copy the box: node p of the dense enumeration (x fastest) -> (x, y, z).
  // The quotients use the hardware reciprocal (relative error below 2^-22):
  // (p + 0.5) / d is at least 0.5 / d <= 2^-11 away from an integer and below
  // 2^11, so the truncation is exact.
  const int bxy = bdim[0] * bdim[1], cnt = bxy * bdim[2];
  const float inv_bx = __builtin_amdgcn_rcpf((float)bdim[0]), inv_bxy = __builtin_amdgcn_rcpf((float)bxy);
  int g0[3];
  bool inside = true;      // the box does not cross the periodic boundary
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    g0[d] = ref[d] + bmin[d];
    inside = inside && g0[d] >= 0 && g0[d] + bdim[d] <= n3[d];
  }
  // box coordinates are below 2^11 and pitches below 2^11 (24-bit products);
  // the grid plane stride in floats may exceed 2^24 (full 32-bit product)
  unsigned char *lds = reinterpret_cast<unsigned char *>(S.node);
  if (inside) {
    const uint32_t sy6 = (uint32_t)f.nx * 6u, sz6 = (uint32_t)f.nx * (uint32_t)f.ny * 6u;
    const float *gb = f.grid + (uint32_t)g0[2] * sz6 + (uint32_t)g0[1] * sy6 + (uint32_t)g0[0] * 6u;
    for (int p = threadIdx.x; p < cnt; p += kGPThreads) {
      const uint32_t z = (uint32_t)(((float)p + 0.5f) * inv_bxy);
      const uint32_t q = (uint32_t)p - __umul24(z, (uint32_t)bxy);
      const uint32_t y = (uint32_t)(((float)q + 0.5f) * inv_bx);
      const uint32_t x = q - __umul24(y, (uint32_t)bdim[0]);
      const uint32_t go = z * sz6 + (y * sy6 + __umul24(x, 6u));
      const float2 *g2 = reinterpret_cast<const float2 *>(gb + go);
      const float2 v0 = g2[0], v1 = g2[1], v2 = g2[2];
      const uint32_t a = __umul24(z, (uint32_t)pxy) + __umul24(y, (uint32_t)px) + x;
      float2 *d = reinterpret_cast<float2 *>(lds + __umul24(a, 24u));
      d[0] = v0; d[1] = v1; d[2] = v2;
    }
  } else {
    for (int p = threadIdx.x; p < cnt; p += kGPThreads) {
      const int z = (int)(((float)p + 0.5f) * inv_bxy);
      const int q = p - (int)__umul24((uint32_t)z, (uint32_t)bxy);
      const int y = (int)(((float)q + 0.5f) * inv_bx);
      const int x = q - (int)__umul24((uint32_t)y, (uint32_t)bdim[0]);
      const uint32_t gx = (uint32_t)wrap_index(g0[0] + x, f.nx);
      const uint32_t gy = (uint32_t)wrap_index(g0[1] + y, f.ny);
      const uint32_t gz = (uint32_t)wrap_index(g0[2] + z, f.nz);
      const float2 *g2 = reinterpret_cast<const float2 *>(f.grid + ((gz * (uint32_t)f.ny + gy) * (uint32_t)f.nx + gx) * 6u);
      const float2 v0 = g2[0], v1 = g2[1], v2 = g2[2];
      const uint32_t a = __umul24((uint32_t)z, (uint32_t)pxy) + __umul24((uint32_t)y, (uint32_t)px) + (uint32_t)x;
      float2 *d = reinterpret_cast<float2 *>(lds + __umul24(a, 24u));
      d[0] = v0; d[1] = v1; d[2] = v2;
    }
  }
  // the stencil of every live particle lies inside the box by construction;
  // checked anyway, so that the LDS reads below can never leave it
  bool bad = false;
#pragma unroll
  for (int it = 0; it < IT; ++it) {
    bool fits = true;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      rel[it][d] -= bmin[d] + 1;
      fits = fits && rel[it][d] >= 0 && rel[it][d] + 2 < bdim[d];
    }
    bad = bad || (live[it] && !fits);
  }
  if (bad) S.bad = 1;
  pit[0] = px;
  pit[1] = pxy;
  __syncthreads();
  return S.bad == 0;
}

// Gather from the staged box.  A row of the stencil (three nodes along x) is
// 72 contiguous bytes of LDS; row offsets are byte offsets built from the
// pitches with adds only.  DB: the next row's reads are issued before the
// current row's products, so that LDS latency overlaps the arithmetic (18 more
// registers); without it the other waves of the SIMD hide that latency.
template <typename R, bool DB = true>
__device__ __forceinline__ void gather_box(const BoxLds &S, const int c0[3], const int pit[2], const R w[3][3],
                                           R F[6]) {
#pragma unroll
  for (int c = 0; c < 6; ++c) F[c] = (R)0;
  const uint32_t pb0 = (uint32_t)pit[0] * 24u, pb1 = (uint32_t)pit[1] * 24u;   // uniform
  const uint32_t b0 = (uint32_t)__umul24((uint32_t)c0[2], pb1) + (uint32_t)__umul24((uint32_t)c0[1], pb0) +
                      (uint32_t)c0[0] * 24u;
  const unsigned char *lds = reinterpret_cast<const unsigned char *>(S.node);
  float2 v[2][9];
  auto load_row = [&](float2 *dst, int r) {
    const float2 *q = reinterpret_cast<const float2 *>(lds + b0 + (uint32_t)(r / 3) * pb1 + (uint32_t)(r % 3) * pb0);
#pragma unroll
    for (int k = 0; k < 9; ++k) dst[k] = q[k];
  };
  if constexpr (DB) load_row(v[0], 0);
#pragma unroll
  for (int r = 0; r < 9; ++r) {
    if constexpr (DB) {
      if (r + 1 < 9) load_row(v[(r + 1) & 1], r + 1);
    } else {
      load_row(v[r & 1], r);
    }
    const float2 *u = v[r & 1];
    const R wyz = w[1][r % 3] * w[2][r / 3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const R wt = w[0][a] * wyz;
      F[0] += wt * (R)u[3 * a].x; F[1] += wt * (R)u[3 * a].y; F[2] += wt * (R)u[3 * a + 1].x;
      F[3] += wt * (R)u[3 * a + 1].y; F[4] += wt * (R)u[3 * a + 2].x; F[5] += wt * (R)u[3 * a + 2].y;
    }
  }
}

template <typename R>
__device__ __forceinline__ void field_at(const FieldDev &f, int64_t i, R x, R y, R z, R F[6]) {
  if (f.kind == QED_FIELD_UNIFORM) {
    F[0] = (R)f.E[0]; F[1] = (R)f.E[1]; F[2] = (R)f.E[2];
    F[3] = (R)f.B[0]; F[4] = (R)f.B[1]; F[5] = (R)f.B[2];
  } else if (f.kind == QED_FIELD_GRID) {
    gather_grid<R>(f, x, y, z, F);
  } else {
    F[0] = (R)f.pE[0][i]; F[1] = (R)f.pE[1][i]; F[2] = (R)f.pE[2][i];
    F[3] = (R)f.pB[0][i]; F[4] = (R)f.pB[1][i]; F[5] = (R)f.pB[2][i];
  }
}

template <typename R>
__device__ __forceinline__ bool fields_finite(const R F[6]) {
  return isfinite(F[0]) && isfinite(F[1]) && isfinite(F[2]) && isfinite(F[3]) && isfinite(F[4]) && isfinite(F[5]);
}

__device__ __forceinline__ void count_add(unsigned long long *c, int which, uint32_t v) {
  // one atomic per wave
  const uint32_t lane = threadIdx.x & 63;
  uint32_t s = v;
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
  if (lane == 0 && s) atomicAdd(&c[which], (unsigned long long)s);
}

// Sum over the 64 lanes of a wave with DPP moves: the row steps of
// row_extreme, then row broadcasts 15 and 31; the total collects in lane 63 and
// is returned to every lane.
__device__ __forceinline__ uint32_t wave_sum(uint32_t v) {
#define QED_DPP_ADD(ctrl, rows) v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, ctrl, rows, 0xF, false);
  QED_DPP_ADD(0xB1, 0xF)    // quad_perm [1,0,3,2]
  QED_DPP_ADD(0x4E, 0xF)    // quad_perm [2,3,0,1]
  QED_DPP_ADD(0x141, 0xF)   // row_half_mirror
  QED_DPP_ADD(0x140, 0xF)   // row_mirror
  QED_DPP_ADD(0x142, 0xA)   // row_bcast:15 into rows 1 and 3
  QED_DPP_ADD(0x143, 0xC)   // row_bcast:31 into rows 2 and 3
#undef QED_DPP_ADD
  return (uint32_t)__builtin_amdgcn_readlane((int)v, 63);
}

// Event counts of a workgroup gather in LDS (one LDS atomic per wave) and reach
// the device counters once, when the workgroup ends: a device atomic per wave on
// the same few counter words serialises at the L2 when thousands of waves add
// at once.  Zero the LDS words before the workgroup's first barrier.
__device__ __forceinline__ void count_lds(uint32_t *c, int which, uint32_t v) {
  const uint32_t s = wave_sum(v);
  if ((threadIdx.x & 63) == 0 && s) atomicAdd(&c[which], s);
}
__device__ __forceinline__ void count_zero(uint32_t *c) {
  if (threadIdx.x < cNumCounters) c[threadIdx.x] = 0;
}
__device__ __forceinline__ void count_flush(const uint32_t *c, unsigned long long *g) {
  __syncthreads();
  if (threadIdx.x < cNumCounters && c[threadIdx.x]) atomicAdd(&g[threadIdx.x], (unsigned long long)c[threadIdx.x]);
}

// Emitter records are packed per wave: the emitter of particle i keeps its record
// at (i & ~63) + (number of emitters before it in its wave), so that a wave's
// records are contiguous.  `bits` is the wave's emitter mask word.
__device__ __forceinline__ int64_t rec_slot(int64_t i, uint64_t bits) {
  const uint64_t below = (i & 63) ? bits & ((1ull << (i & 63)) - 1ull) : 0ull;
  return (i & ~(int64_t)63) + (int64_t)__popcll(below);
}

// Adds the number of lanes of the wave with `set` (one atomic per wave).
__device__ __forceinline__ void count_flags(unsigned long long *c, int which, bool set) {
  const uint32_t s = (uint32_t)__popcll(__ballot(set));
  if ((threadIdx.x & 63) == 0 && s) atomicAdd(&c[which], (unsigned long long)s);
}

// Workgroup: obtain a tile id from the ticket (thread 0) and broadcast.
__device__ __forceinline__ uint32_t next_tile(uint32_t *ticket, uint32_t *lds) {
  __syncthreads();
  if (threadIdx.x == 0) *lds = atomicAdd(ticket, 1u);
  __syncthreads();
  return *lds;
}

// Exclusive device-wide offset of this workgroup's tile given its per-thread count.
__device__ __forceinline__ uint64_t tile_offset(uint32_t tile, uint64_t agg, uint64_t *status,
                                                unsigned long long *counters, uint64_t *lds64) {
  if (threadIdx.x < 64) {
    const uint64_t e = lookback_scan(status, tile, agg, &counters[cScanTimeout]);
    if (threadIdx.x == 0) *lds64 = e;
  }
  __syncthreads();
  return *lds64;
}

// ============================================ photon retirement and tally
// A photon whose optical depth tau exceeds the largest optical depth it could
// still accumulate before the end of the run, W_max (t_end - t), cannot convert
// within the run: W_max = alpha E_S h_pair_env(chi_max) / gamma_ph bounds its
// pair rate, with chi_max = gamma_ph F / E_S and F a bound of |E| + |B| over the
// rest of the run given by the caller (|k x (E + k x B)| <= |E| + |B|), since
// h_pair and the surrogate's pair rate lie below the envelope and the envelope
// grows with chi.  Such a photon is counted into a histogram of ln gamma_ph (the
// tally) instead of being stored (at emission) or kept (in pair creation).
constexpr int kTallyBins = QED_TALLY_BINS;
constexpr double kTallyLnLo = 0.69314718055994531;   // ln 2
constexpr double kTallyLnHi = 16.118095650958319;    // ln 1e7

struct RetireDev {
  int on;
  double t_end;              // end of the run, t = step * dt
  float f_over_es;           // F / E_S
  unsigned long long *tally; // kTallyBins counts
};

__device__ __forceinline__ double pair_rate_max(float gph, const RetireDev &r) {
  if (!(gph >= 2.f)) return 0.0;                      // below the pair threshold W = 0
  return kRateUnit * (double)(h_pair_env(gph * r.f_over_es) * rcp<float>(gph));
}

// Time left in the run after step `step` (the photon's optical depth is final
// for t = (step + 1) dt).
__device__ __forceinline__ double time_left(const RetireDev &r, uint64_t step, double dt) {
  return r.t_end - (double)(step + 1) * dt;
}

__device__ __forceinline__ bool retirable(const RetireDev &r, double tau, float gph, double t_left) {
  return r.on && tau >= pair_rate_max(gph, r) * t_left;
}

// bin = floor((ln gamma - ln 2) / d) with d = (ln 1e7 - ln 2) / kTallyBins, clamped
__device__ __forceinline__ void tally_photon(const RetireDev &r, double gph) {
  const double b = floor((log(gph) - kTallyLnLo) * (kTallyBins / (kTallyLnHi - kTallyLnLo)));
  const int k = b < 0.0 ? 0 : (b >= (double)kTallyBins ? kTallyBins - 1 : (int)b);
  atomicAdd(&r.tally[k], 1ull);
}

// Photons of the emitters of one tile appended in (emitter, event) order: each
// thread holds nacc accepted photons (gph, tph); ids count every accepted photon
// (stored or retired, so the stored photons' ids and random streams do not
// depend on the retirement), storage slots count the stored ones.  Both prefix
// sums travel in one 64-bit scan value: total | stored << 31.
template <typename R>
__device__ void append_photons(const SpeciesDev &ph, const RetireDev &ret, uint64_t step, double dt, uint32_t tile,
                               int64_t n_em, int tile_size, uint32_t nacc, const R *gph, const double *tph, R x,
                               R y, R z, R nx, R ny, R nz, int64_t ph0, uint64_t id0, uint64_t *next_id,
                               const ScanDev &sc, unsigned long long *counters, uint64_t *scan_s, uint64_t *off_s,
                               uint32_t *cnt) {
  uint32_t keep = (1u << nacc) - 1u, nret = 0;
  if (ret.on && nacc) {
    const double tl = time_left(ret, step, dt);
#pragma unroll
    for (int s = 0; s < kKmaxMax; ++s)
      if (s < (int)nacc && retirable(ret, tph[s], (float)gph[s], tl)) {
        keep &= ~(1u << s);
        tally_photon(ret, (double)gph[s]);
        ++nret;
      }
  }
  const uint32_t nkeep = (uint32_t)__popc(keep);
  count_lds(cnt, cRetired, nret);
  uint64_t tot;
  const uint64_t off = block_exclusive64((uint64_t)nacc | ((uint64_t)nkeep << 31), scan_s, &tot);
  const uint64_t toff = tile_offset(tile, tot, sc.status, counters, off_s);
  const uint64_t base = toff + off;
  const uint64_t rank0 = base & 0x7FFFFFFFull, slot0 = base >> 31;
  R *X = (R *)ph.x, *Y = (R *)ph.y, *Z = (R *)ph.z;
  R *KX = (R *)ph.px, *KY = (R *)ph.py, *KZ = (R *)ph.pz;
  uint32_t ndrop = 0, k = 0;
#pragma unroll
  for (int s = 0; s < kKmaxMax; ++s) {
    if (s < (int)nacc && ((keep >> s) & 1u)) {
      const int64_t j = ph0 + (int64_t)(slot0 + k);
      ++k;
      if (j < ph.cap) {
        X[j] = x; Y[j] = y; Z[j] = z;
        KX[j] = nx * gph[s]; KY[j] = ny * gph[s]; KZ[j] = nz * gph[s];
        ph.tau[j] = tph[s];
        ph.id[j] = id0 + rank0 + (uint64_t)s;
      } else {
        ++ndrop;
      }
    }
  }
  count_lds(cnt, cDropped, ndrop);
  const int64_t last = (n_em - 1) / tile_size;
  if ((int64_t)tile == last && threadIdx.x == 0) {
    const uint64_t t = toff + tot;
    const int64_t stored = (int64_t)(t >> 31);
    *ph.count = ph0 + stored < ph.cap ? ph0 + stored : ph.cap;
    *next_id = id0 + (t & 0x7FFFFFFFull);
  }
}

// ========================================================= gather / push
// A pure streaming pass with no dependency between workgroups.  Workgroups are
// dispatched round-robin over the 8 XCDs; the tiles are dealt to the XCDs in
// chunks of kGPChunk consecutive tiles, chunk c to XCD c % 8, so that an XCD's
// L2 holds the grid around the particles of the chunk it works on (consecutive
// particles are close after a cell sort) while every part of the array, such
// as the unsorted particles appended since the last sort, is spread over all
// eight XCDs.  Block b = 8 k + x works on tile
// ((k / kGPChunk) * 8 + x) * kGPChunk + k % kGPChunk.  A
// particle whose optical depth runs out within the step sets its bit in a
// ballot mask and writes the fields, chi, rate and remaining time of its first
// event to its own slot; k_emit_index turns the mask into the ordered list.
constexpr int kXcds = 8;
constexpr int64_t kGPChunk = 32;

// Emitter record, written by the emitter to its own slot and read once by
// k_emit: what the event loop needs beyond the particle's id.
template <typename R>
struct alignas(16) EmRec {
  R x[3], p[3], F[6];       // position after the push, momentum p^{n+1/2}, E and B at x^n
  double tau, chi, W;       // optical depth at the start of the step, chi (thinned pass: its bound) and rate
  int32_t j0, nsub;         // method I: sub-step of the first event, number of sub-steps
};

template <typename R>
struct GPArgs {
  SpeciesDev sp;
  FieldDev f;
  const R *lnh;          // rad ln h table (float32 or float64 copy)
  R q, dt;
  double dtd;
  uint64_t *mask;        // one bit per particle
  EmRec<R> *rec;         // slot = particle index
  unsigned long long *counters;
  int gen;               // 0: optical depth; 1: method I with sub-steps; 2: method I, one step
  uint32_t seed;
  uint64_t step;
  const int64_t *d_step;
  TabRange rg;
};

constexpr double kSubstepW = 0.2;     // method I: W Dt / N <= 0.2
constexpr int kMaxSubsteps = 1024;

__device__ __forceinline__ uint64_t step_of(uint64_t v, const int64_t *p) { return p ? (uint64_t)*p : v; }

// Method I: number of sub-steps of the step and the first sub-step j in
// [j, N) whose draw r_1 (second Philox output of counter j) is below W Dt / N.
__device__ __forceinline__ int method1_nsub(double W, double dt, int gen) {
  if (gen != 1 || !(W > 0.0)) return 1;
  double N = ceil(W * dt / kSubstepW);
  N = N < 1.0 ? 1.0 : (N > kMaxSubsteps ? kMaxSubsteps : N);
  return (int)N;
}
__device__ __forceinline__ int method1_next(uint64_t id, uint32_t seed, uint64_t step, int j, int N, double W,
                                            double dt) {
  for (; j < N; ++j) {
    const uint4 u = stream4(id, seed, step, kLeptonEvent, (uint32_t)j);
    if (W * dt / N > unit<double>(u.y)) return j;
  }
  return N;
}

// Waves per SIMD the compiler must allow for (bounds the registers): the
// single-precision grid kernel without method I is the hot one.
template <typename R, int FK, bool M1> constexpr int gp_waves() {
  return (sizeof(R) == 4 && FK == QED_FIELD_GRID && !M1) ? kGPWaves : 1;
}

// First particle of this workgroup's tile, for tiles of `tile_size` particles
// dealt to the XCDs in chunks of kGPChunk tiles.
__device__ __forceinline__ int64_t gp_tile_base(int64_t tile_size) {
  const int64_t k = blockIdx.x / kXcds;
  return (((k / kGPChunk) * kXcds + blockIdx.x % kXcds) * kGPChunk + k % kGPChunk) * tile_size;
}

template <typename R>
struct GPTile {   // the tile's slices of the particle arrays (uniform bases, 32-bit offsets)
  R *x, *y, *z, *px, *py, *pz;
  double *tau;
  __device__ GPTile(const SpeciesDev &sp, int64_t base)
      : x((R *)sp.x + base), y((R *)sp.y + base), z((R *)sp.z + base), px((R *)sp.px + base),
        py((R *)sp.py + base), pz((R *)sp.pz + base), tau(sp.tau + base) {}
};

// Push, chi, rate and event decision of particle o of the tile (offset from
// base; ok: present, with fields F): a particle with non-finite fields is
// skipped and counted; the others are written back, with either the record of
// their first event within the step or their reduced optical depth.  Then the
// wave's mask word and counters.  Every lane of the wave calls it (the record
// slot is ranked among the wave's emitters).
template <typename R, int FK, bool M1, bool Thin>
__device__ __forceinline__ void gp_finish(const GPArgs<R> &a, const GPTile<R> &P, const FieldDev &f,
                                          const R *lnh_s, int64_t base, int o, int64_t n, bool ok, R x, R y, R z,
                                          R px, R py, R pz, double tau, const R F[6]) {
  const int64_t i = base + o;
  bool flag = false, nan = false, range = false;
  if (ok && !fields_finite<R>(F)) { ok = false; nan = true; }
  if (ok) {
    boris<R>(px, py, pz, F[0], F[1], F[2], F[3], F[4], F[5], a.q, a.dt);
    const R g = root<R>((R)1 + px * px + py * py + pz * pz);
    const R ig = rcp<R>(g), vdt = ig * a.dt;
    x += px * vdt; y += py * vdt; z += pz * vdt;
    if (FK == QED_FIELD_GRID) {
      wrap_coord<R>(x, box_len<R>(f, 0)); wrap_coord<R>(y, box_len<R>(f, 1));
      wrap_coord<R>(z, box_len<R>(f, 2));
    }
    P.x[o] = x; P.y[o] = y; P.z[o] = z; P.px[o] = px; P.py[o] = py; P.pz[o] = pz;
    // Thin: the envelope needs only an upper bound of chi (float32 with its
    // rounding bound); the emission pass evaluates chi itself for the candidates
    double chi;
    if constexpr (Thin) chi = (double)chi_lepton_upper_f32(px, py, pz, g, F);
    else if constexpr (sizeof(R) == 4) chi = chi_lepton_f32(px, py, pz, F);
    else chi = chi_lepton(px, py, pz, F[0], F[1], F[2], F[3], F[4], F[5]);
    double W = 0.0;
    if (isfinite(chi)) {
      range = chi > a.rg.rad_hi;
      R h;
      if constexpr (Thin) h = (R)h_rad_env((float)chi);
      else h = h_rad<R, true>((R)chi, lnh_s, a.rg);
      W = kRateUnit * (double)(h * ig);
    } else {
      nan = true;
    }
    int j0 = 0, nsub = 1;
    if (M1 && a.gen) {
      // method I: first sub-step with an event, if any
      const uint64_t id = a.sp.id[i];
      nsub = method1_nsub(W, a.dtd, a.gen);
      j0 = W > 0.0 ? method1_next(id, a.seed, step_of(a.step, a.d_step), 0, nsub, W, a.dtd) : nsub;
      flag = j0 < nsub;
    } else {
      flag = W > 0.0 && tau <= W * a.dtd;
    }
    const uint64_t fbits = __ballot(flag);   // the live lanes' flags (others are not emitters)
    if (flag) {
      EmRec<R> r;
      r.x[0] = x; r.x[1] = y; r.x[2] = z; r.p[0] = px; r.p[1] = py; r.p[2] = pz;
#pragma unroll
      for (int c = 0; c < 6; ++c) r.F[c] = F[c];
      r.tau = tau;
      r.chi = chi;
      r.W = W;
      r.j0 = j0;
      r.nsub = nsub;
      a.rec[rec_slot(i, fbits)] = r;
    } else if (!(M1 && a.gen)) {
      P.tau[o] = tau - W * a.dtd;
    }
  }
  const uint64_t bits = __ballot(flag);
  if ((threadIdx.x & 63) == 0 && base + (o & ~63) < n) a.mask[(base + o) >> 6] = bits;
  count_flags(a.counters, cNanChi, nan);
  count_flags(a.counters, cChiRange, range);
}

// One particle per thread.  M1: compiled with the method I generator
// (a.gen != 0), else optical depth only.  Thin (float32, surrogate path): the
// optical depth runs down at the envelope rate h_rad_env (Poisson thinning);
// the emission pass evaluates the rate net only at the candidate events this
// finds and keeps each with probability W / W_env.
template <typename R, int FK, bool M1, bool Thin = false>
__global__ __launch_bounds__(kGPThreads, (gp_waves<R, FK, M1>())) void k_gather_push(GPArgs<R> a) {
  __shared__ R lnh_s[kRadNChi];
  // (the grid is sized by the capacity: blocks beyond the particles present
  // return, and they are the last ones dispatched)
  const int64_t n = *a.sp.count;
  const int64_t base = gp_tile_base(kGPThreads);
  if (base >= n) return;
  const int t = threadIdx.x;
  const int64_t i = base + t;
  FieldDev f = a.f;
  f.kind = FK;
  const bool live = i < n;
  // every load of the particle is issued up front, to overlap with the staging
  R x = 0, y = 0, z = 0, px = 0, py = 0, pz = 0;
  double tau = 0.0;
  const GPTile<R> P(a.sp, base);
  if (live) {
    x = P.x[t]; y = P.y[t]; z = P.z[t];
    px = P.px[t]; py = P.py[t]; pz = P.pz[t];
    tau = P.tau[t];
  }
  for (int q = threadIdx.x; q < kRadNChi; q += blockDim.x) lnh_s[q] = a.lnh[q];
  R F[6];
  if (FK == QED_FIELD_GRID) {
    __shared__ BoxLds box_s;
    int j[1][3], rel[1][3], pit[2];
    R w[3][3];
    tsc_setup<R>(f, x, y, z, j[0], w);      // dead lanes hold x = 0: harmless, unused
    if (stage_box<1>(box_s, f, &live, j, rel, pit)) {   // its barriers also publish lnh_s
      if (live) gather_box<R>(box_s, rel[0], pit, w, F);
    } else {
      if (live) gather_global<R>(f, j[0], w, F);
      if (threadIdx.x == 0) atomicAdd(&a.counters[cBoxFallback], 1ull);
    }
  } else {
    __syncthreads();
    if (live) field_at<R>(f, i, x, y, z, F);
  }
  gp_finish<R, FK, M1, Thin>(a, P, f, lnh_s, base, t, n, live, x, y, z, px, py, pz, tau, F);
}

// Dense float32 species on a grid, optical depth only (the launcher takes it
// for species sized for at least kDenseGP particles per cell): two particles
// per thread, particle it of thread t at base + it * kGPThreads + t, so that
// the workgroup's fixed work (the box's extent, its staging and the barriers)
// is shared by 512 particles.  A sparse species' 512 particles span too many
// cells for one box, so it keeps the kernel above.
constexpr int64_t kDenseGP = 64;
template <bool Thin>
__global__ __launch_bounds__(kGPThreads, kGPWaves) void k_gather_push2(GPArgs<float> a) {
  using R = float;
  constexpr int IT = 2;
  __shared__ R lnh_s[kRadNChi];
  __shared__ BoxLds box_s;
  const int64_t n = *a.sp.count;
  const int64_t base = gp_tile_base((int64_t)kGPThreads * IT);
  if (base >= n) return;
  const int t = threadIdx.x;
  FieldDev f = a.f;
  f.kind = QED_FIELD_GRID;
  bool live[IT];
  // positions up front (the box needs them); momenta and optical depths after the staging
  R xs[IT][3];
  const GPTile<R> P(a.sp, base);
#pragma unroll
  for (int it = 0; it < IT; ++it) {
    const int o = it * kGPThreads + t;
    live[it] = base + o < n;
    xs[it][0] = live[it] ? P.x[o] : (R)0; xs[it][1] = live[it] ? P.y[o] : (R)0; xs[it][2] = live[it] ? P.z[o] : (R)0;
  }
  for (int q = threadIdx.x; q < kRadNChi; q += blockDim.x) lnh_s[q] = a.lnh[q];

  int j[IT][3], rel[IT][3], pit[2];
#pragma unroll
  for (int it = 0; it < IT; ++it) {
    R w[3][3];
    tsc_setup<R>(f, xs[it][0], xs[it][1], xs[it][2], j[it], w);   // dead particles hold x = 0: unused
  }
  const bool boxed = stage_box<IT>(box_s, f, live, j, rel, pit);   // its barriers also publish lnh_s
  if (!boxed && threadIdx.x == 0) atomicAdd(&a.counters[cBoxFallback], 1ull);
#pragma unroll
  for (int it = 0; it < IT; ++it) {
    // one particle after the other, its momentum and optical depth loaded
    // here, the weights recomputed from the position (held opaque, so that they
    // are not kept live across the staging) and the rows read one at a time:
    // 72 registers, which six waves per SIMD allow (the LDS allows six
    // workgroups per CU); holding any of these through the staging or a second
    // row in flight needs more and measured slower
    const int o = it * kGPThreads + t;
    R px = 0, py = 0, pz = 0;
    double tau = 0.0;
    if (live[it]) { px = P.px[o]; py = P.py[o]; pz = P.pz[o]; tau = P.tau[o]; }
    R x = xs[it][0], y = xs[it][1], z = xs[it][2];
    asm volatile("" : "+v"(x), "+v"(y), "+v"(z));
    int jc[3];
    R w[3][3];
    tsc_setup<R>(f, x, y, z, jc, w);
    R F[6];
    if (live[it]) {
      if (boxed) gather_box<R, false>(box_s, rel[it], pit, w, F);
      else gather_global<R>(f, jc, w, F);
    }
    gp_finish<R, QED_FIELD_GRID, false, Thin>(a, P, f, lnh_s, base, o, n, live[it], xs[it][0], xs[it][1],
                                              xs[it][2], px, py, pz, tau, F);
  }
}

// Ordered emitter list from the ballot mask: each thread owns W consecutive
// 64-bit words; popcounts are scanned across the workgroup and across tiles
// (decoupled look-back), and every set bit writes its particle index at its
// rank.  Large species take W = 8 (tiles of 131072 particles, a short look-back
// chain), small ones W = 1 (more workgroups).  Persistent workgroups take the
// tiles of the particles present from the ticket, so that a launch sized for a
// large capacity costs little when the species holds few particles.
constexpr int kEIThreads = 256;
template <int W> constexpr int64_t ei_tile() { return (int64_t)kEIThreads * W * 64; }
constexpr int64_t kEIWideFrom = (int64_t)1 << 22;   // capacity from which W = 8

// Idx = EmIdx: (particle index, record slot); Idx = int32_t: the particle index alone.
template <int W, typename Idx>
__global__ __launch_bounds__(kEIThreads) void k_emit_index(const uint64_t *mask, const int64_t *count,
                                                           Idx *em_idx, int64_t *n_emit, ScanDev sc,
                                                           unsigned long long *counters) {
  __shared__ uint32_t scan_s[16];
  __shared__ uint32_t tile_s;
  __shared__ uint64_t off_s;
  const int64_t n = *count;
  while (true) {
    const uint32_t tile = next_tile(sc.ticket, &tile_s);
    const int64_t base = (int64_t)tile * ei_tile<W>();
    if (base >= n) {
      if (tile == 0 && threadIdx.x == 0) *n_emit = 0;
      return;
    }
    const int64_t w0 = (base >> 6) + (int64_t)threadIdx.x * W;
    uint64_t m[W];
    uint32_t c = 0;
#pragma unroll
    for (int k = 0; k < W; ++k) {
      const int64_t w = w0 + k;
      m[k] = (w << 6) < n ? mask[w] : 0ull;
      const int64_t valid = n - (w << 6);
      if (valid < 64 && valid > 0) m[k] &= (1ull << valid) - 1ull;
      c += (uint32_t)__popcll(m[k]);
    }
    uint32_t total;
    const uint32_t off = block_exclusive(c, scan_s, &total);
    const uint64_t toff = tile_offset(tile, total, sc.status, counters, &off_s);
    uint64_t r = toff + off;
#pragma unroll
    for (int k = 0; k < W; ++k) {
      uint64_t b = m[k];
      const int32_t wb = (int32_t)((w0 + k) << 6);
      int32_t slot = wb;   // records of a mask word are packed from its base (rec_slot)
      while (b) {
        const int32_t p = wb + (__ffsll((long long)b) - 1);
        if constexpr (sizeof(Idx) == sizeof(EmIdx)) em_idx[r++] = EmIdx{p, slot++};
        else em_idx[r++] = p;
        b &= b - 1ull;
      }
    }
    const int64_t last = (n - 1) / ei_tile<W>();
    if ((int64_t)tile == last && threadIdx.x == 0) *n_emit = (int64_t)(toff + total);
  }
}

// ================================================================ emit
template <typename R>
struct EmitArgs {
  SpeciesDev lep, ph;
  const R *lnh;
  const double *S64;           // float64 quantiles (R = double)
  const uint16_t *q16;         // 16-bit quantiles (R = float)
  const float *s0sc;
  const EmIdx *em_idx;
  const EmRec<R> *rec;
  const int64_t *n_emit;
  uint64_t *next_id;
  uint32_t seed;
  int kmax;
  int recoil;
  uint64_t step;
  const int64_t *d_step;       // if set, the step index is read from the device
  ScanDev sc;
  unsigned long long *counters;
  int gen;                     // event generator (see GPArgs)
  double dtd;
  TabRange rg;
  RetireDev ret;
};

// Emitters per tile (= threads per workgroup): 1024 for the float32 optical-depth
// kernel (fewer tiles, a shorter look-back chain, 127 registers), 512 for the
// float64 and method I kernels, which need more than 128 registers.
template <typename R, bool M1> constexpr int emit_threads() { return (sizeof(R) == 4 && !M1) ? 1024 : 512; }

template <typename R, bool M1, typename Tab>
__device__ void emit_tile(const EmitArgs<R> &a, const Tab &tab, const R *lnh, uint32_t tile,
                          uint64_t *scan_s, uint64_t *off_s, int64_t n_em, int64_t ph_count0,
                          uint64_t id0, uint32_t *cnt) {
  constexpr int T = emit_threads<R, M1>();
  const int64_t r = (int64_t)tile * T + threadIdx.x;
  const bool valid = r < n_em;
  R gph[kKmaxMax];
  double tph[kKmaxMax];
  uint32_t nacc = 0, nev = 0, nrej = 0, ncap = 0;
  R nx = 0, ny = 0, nz = 0, x = 0, y = 0, z = 0;
  if (valid) {
    const EmIdx e = a.em_idx[r];
    const int64_t i = e.i;
    const EmRec<R> rc = a.rec[e.slot];
    R F[6];
#pragma unroll
    for (int c = 0; c < 6; ++c) F[c] = rc.F[c];
    const uint64_t id = a.lep.id[i];
    double chi = rc.chi, W = rc.W, rem = a.dtd - rc.tau / rc.W;   // time left after the first event
    R *PX = (R *)a.lep.px, *PY = (R *)a.lep.py, *PZ = (R *)a.lep.pz;
    R px = rc.p[0], py = rc.p[1], pz = rc.p[2];
    x = rc.x[0]; y = rc.x[1]; z = rc.x[2];
    const R pa = sqrt(px * px + py * py + pz * pz);
    if (pa > (R)0) { nx = px / pa; ny = py / pa; nz = pz / pa; }
    R g = sqrt((R)1 + px * px + py * py + pz * pz);
    double tau = 0.0;
    bool recoiled = false;
    const uint64_t step = step_of(a.step, a.d_step);
    // one event: sample xi, infrared cut, photon, recoil (counter k of the stream)
    auto event = [&](uint32_t k) {
      const uint4 u = stream4(id, a.seed, step, kLeptonEvent, k);
      R xi, om;
      sample_rad<R>(tab, (R)chi, unit<R>(u.x), unit<R>(u.z), xi, om, a.rg);
      const R gp = xi * g;
      ++nev;
      if (gp >= (R)2) {
#pragma unroll
        for (int s = 0; s < kKmaxMax; ++s)
          if (s == (int)nacc) { gph[s] = gp; tph[s] = -log(unit<double>(u.w)); }
        ++nacc;
        if (a.recoil) {
          const R gn = fmax(om * g, (R)1);
          const R pm = sqrt(fmax(gn * gn - (R)1, (R)0));
          px = nx * pm; py = ny * pm; pz = nz * pm;
          g = gn;
          recoiled = true;
          chi = chi_lepton(px, py, pz, F[0], F[1], F[2], F[3], F[4], F[5]);
          W = isfinite(chi) ? kRateUnit * (double)(h_rad<R>((R)chi, lnh, a.rg) / g) : 0.0;
        }
      } else {
        ++nrej;
      }
      return u;
    };
    if (M1 && a.gen) {
      // method I: at most one event per sub-step, W Dt / N > r_1
      const int N = rc.nsub;
      int j = rc.j0, done = 0;
      while (true) {
        event((uint32_t)j);
        ++done;
        ++j;
        if (done >= a.kmax) { if (j < N) ++ncap; break; }
        if (!(W > 0.0)) break;
        j = method1_next(id, a.seed, step, j, N, W, a.dtd);
        if (j >= N) break;
      }
    } else {
      int k = 0;
      while (true) {
        const uint4 u = event((uint32_t)k);
        tau = -log(unit<double>(u.y));
        ++k;
        const bool again = W > 0.0 && tau <= W * rem;
        if (!again) break;
        if (k >= a.kmax) { ++ncap; break; }
        rem -= tau / W;
      }
    }
    if (!(M1 && a.gen)) a.lep.tau[i] = tau - W * rem;
    if (recoiled) { PX[i] = px; PY[i] = py; PZ[i] = pz; }
  }
  count_lds(cnt, cEvents, nev);
  count_lds(cnt, cRejected, nrej);
  count_lds(cnt, cCapped, ncap);
  count_lds(cnt, cPhotons, nacc);
  append_photons<R>(a.ph, a.ret, step_of(a.step, a.d_step), a.dtd, tile, n_em, T, nacc, gph, tph, x, y, z, nx, ny,
                    nz, ph_count0, id0, a.next_id, a.sc, a.counters, scan_s, off_s, cnt);
}

// float path: 16-bit quantile table read through the caches (an emission step
// touches few rows), float32 ln h staged in LDS
template <bool M1>
__global__ __launch_bounds__((emit_threads<float, M1>())) void k_emit_f32(EmitArgs<float> a) {
  __shared__ float lnh_s[kRadNChi];
  __shared__ uint64_t scan_s[16];
  __shared__ uint32_t tile_s;
  __shared__ uint64_t off_s;
  __shared__ int64_t hdr_s[3];
  __shared__ uint32_t cnt_s[cNumCounters];
  count_zero(cnt_s);
  if (threadIdx.x == 0) { hdr_s[0] = *a.n_emit; hdr_s[1] = *a.ph.count; hdr_s[2] = (int64_t)*a.next_id; }
  __syncthreads();
  const int64_t n_em = hdr_s[0], ph0 = hdr_s[1];
  const uint64_t id0 = (uint64_t)hdr_s[2];
  if (n_em == 0) return;
  for (int k = threadIdx.x; k < kRadNChi; k += blockDim.x) lnh_s[k] = a.lnh[k];
  const RowQ16 tab{a.q16, a.s0sc};     // 16-bit quantile table through the caches
  while (true) {
    const uint32_t tile = next_tile(a.sc.ticket, &tile_s);
    if ((int64_t)tile * emit_threads<float, M1>() >= n_em) break;
    emit_tile<float, M1>(a, tab, lnh_s, tile, scan_s, &off_s, n_em, ph0, id0, cnt_s);
  }
  count_flush(cnt_s, a.counters);
}

// double path: float64 master tables read through the caches
template <bool M1>
__global__ __launch_bounds__((emit_threads<double, M1>())) void k_emit_f64(EmitArgs<double> a) {
  __shared__ double lnh_s[kRadNChi];
  __shared__ uint64_t scan_s[16];
  __shared__ uint32_t tile_s;
  __shared__ uint64_t off_s;
  __shared__ int64_t hdr_s[3];
  __shared__ uint32_t cnt_s[cNumCounters];
  count_zero(cnt_s);
  if (threadIdx.x == 0) { hdr_s[0] = *a.n_emit; hdr_s[1] = *a.ph.count; hdr_s[2] = (int64_t)*a.next_id; }
  __syncthreads();
  const int64_t n_em = hdr_s[0], ph0 = hdr_s[1];
  const uint64_t id0 = (uint64_t)hdr_s[2];
  if (n_em == 0) return;
  for (int k = threadIdx.x; k < kRadNChi; k += blockDim.x) lnh_s[k] = a.lnh[k];
  const RowF64 tab{a.S64};
  while (true) {
    const uint32_t tile = next_tile(a.sc.ticket, &tile_s);
    if ((int64_t)tile * emit_threads<double, M1>() >= n_em) break;
    emit_tile<double, M1>(a, tab, lnh_s, tile, scan_s, &off_s, n_em, ph0, id0, cnt_s);
  }
  count_flush(cnt_s, a.counters);
}

// ============================================== surrogate variants (float32)
// The learned part of the step: the rate net replaces the ln h lookup in the
// lepton pass, and the xi net (with the residual check against the Hermite CDF
// rows and the table as fallback) replaces the inverse-CDF lookup in the
// emission pass.  Both evaluate 16 particles per forward call per wave, so a
// wave of 64 particles makes four calls with inputs broadcast by shuffles.
struct MlpDev {
  TabRange rg;
  const float *thA, *thB;    // float32 parameters (split into bf16 hi/lo in LDS)
  const float *chk;          // residual-check CDF rows
  const float *lnh32;        // rad table (fallback)
  const uint16_t *q16;
  const float *s0sc;
  float tol;
};

// Output O of a net for the lanes of a wave with `need` (others get 0).
// The needing lanes are packed by ballot rank into the first ceil(m/16)
// 16-sample tiles (inputs pushed with ds_permute, outputs pulled back with a
// shuffle), so a wave makes one forward call per 16 needing lanes.  Samples are
// columns of the matrix products and do not interact, so every needing lane
// gets exactly what an unpacked evaluation would give it.  Every lane of the
// wave must call it (it returns at once when no lane needs it).
template <int O = 0, bool Lean = false>
__device__ __forceinline__ float mlp_packed(const mlp::NetLdsI &N, int nin, int nout, bool need, float in0,
                                            float in1) {
  const int lane = threadIdx.x & 63;
  const uint64_t bal = __ballot(need);
  const int m = __popcll(bal);
  if (m == 0) return 0.f;                                      // uniform
  const int rank = __popcll(bal & ((1ull << lane) - 1ull));     // needing lanes before this one
  const int dst = need ? rank : m + (lane - rank);              // a permutation of 0..63
  const float p0 = __int_as_float(__builtin_amdgcn_ds_permute(dst << 2, __float_as_int(in0)));
  const float p1 = __int_as_float(__builtin_amdgcn_ds_permute(dst << 2, __float_as_int(in1)));
  float yp = 0.f;
  const int nt = (m + 15) >> 4;
#pragma unroll 1
  for (int q = 0; q < nt; ++q) {
    mlp::reload_barrier();
    const float i0 = __shfl(p0, q * 16 + (lane & 15), 64), i1 = __shfl(p1, q * 16 + (lane & 15), 64);
    float y[2];
    mlp::forward_inf<Lean>(N, nin, nout, i0, i1, y);
    if ((lane >> 4) == q) yp = y[O];                           // slot q*16 + (lane & 15) = lane
  }
  const float y = __shfl(yp, rank, 64);
  return need ? y : 0.f;
}

// ln h_rad(chi) from net B for the lanes of a wave with `need`; ok = inside the
// trained chi range, finite and below the thinning envelope (else the caller
// takes the table).
__device__ __forceinline__ float mlp_lnh(const mlp::NetLdsI &B, double chi, bool need, bool &ok) {
  const bool in = chi >= kRadChiMin && chi <= kMlpChiMax;
  const float mine = mlp_packed<0>(B, 1, 1, need, mlp::xin(in ? chi : 1.0), 0.f);   // the photon rate head only
  const float lchi = logf((float)chi);
  const float lh = mlp::kBShift0 + mlp::kBScale0 * mine + lchi;
  ok = need && in && isfinite(lh) && expf(lh) <= h_rad_env((float)chi);
  return lh;
}

// ln h_pair(chi) from the pair head of net B, likewise (trained for chi in
// [1e-2, 1e2]).
__device__ __forceinline__ float mlp_lnh_pair(const mlp::NetLdsI &B, double chi, bool need, bool &ok) {
  const bool in = chi >= kPairChiMin && chi <= kMlpChiMax;
  const float y = mlp_packed<1, true>(B, 1, 2, need, mlp::xin(in ? chi : 1.0), 0.f);
  const float lchi = logf((float)chi);
  const float lh = mlp::kBShift1 + mlp::kBScale1 * y + lchi - 8.0f / (3.0f * (float)chi);
  ok = need && in && isfinite(lh) && expf(lh) <= h_pair_env((float)chi);
  return lh;
}

constexpr int kEmitMlpThreads = 512;

struct EmitMlpLds {
  mlp::NetLdsI A, B;
  float chk[kRadNChi * (2 + 2 * mlp::kChkN)];
  float lnh[kRadNChi];
};

// Surrogate emission: the candidate events of the thinned lepton pass.  A
// candidate at rate W_env = alpha E_S h_rad_env / gamma is kept with probability
// W / W_env, W from net B (table if the net's output fails its check); a kept
// event draws xi from net A with the residual check against the tabulated CDF
// (table sample if it fails), applies the infrared cut and the recoil (W_env
// follows the new chi and gamma); then the next candidate comes after a new
// optical depth at W_env, up to kmax candidates per step (the cap is counted).
// Counter k of the particle's stream serves candidate k: LEPTON_EVENT gives
// (u_xi, u_tau, u_row, u_ph) as on the table path, LEPTON_THIN the keep draw.
//
// Two passes.  Cont = false takes every emitter's first candidate; with
// kmax > 1 an emitter with a further candidate within the step sets its bit in
// cont_mask (at its position in the emitter list) and is left to the second
// pass.  Cont = true takes the emitters of that list (cont_idx, n_cont, in
// emitter order), re-runs their first candidate (identical: the same streams
// and per-lane arithmetic; neither counted nor appended again) and goes on with
// candidates 1 .. kmax - 1.  Packed densely, the few emitters with a second
// candidate fill whole net calls instead of a few lanes of every wave.  The
// photons of the second pass follow all those of the first, in (emitter, event)
// order.
template <bool Cont>
__global__ __launch_bounds__(kEmitMlpThreads) void k_emit_mlp(EmitArgs<float> a, MlpDev m, uint64_t *cont_mask,
                                                              const int32_t *cont_idx, const int64_t *n_cont) {
  extern __shared__ __align__(16) unsigned char lds_raw[];
  EmitMlpLds &S = *reinterpret_cast<EmitMlpLds *>(lds_raw);
  __shared__ uint64_t scan_s[16];
  __shared__ uint32_t tile_s;
  __shared__ uint64_t off_s;
  __shared__ int64_t hdr_s[3];
  __shared__ uint32_t cnt_s[cNumCounters];
  count_zero(cnt_s);
  if (threadIdx.x == 0) {
    hdr_s[0] = Cont ? *n_cont : *a.n_emit;
    hdr_s[1] = *a.ph.count;
    hdr_s[2] = (int64_t)*a.next_id;
  }
  __syncthreads();
  const int64_t n_em = hdr_s[0], ph0 = hdr_s[1];
  const uint64_t id0 = (uint64_t)hdr_s[2];
  if (n_em == 0) return;
  const int klim = Cont ? a.kmax : 1;
  mlp::stage_net_infer(m.thA, mlp::kA, &S.A);
  mlp::stage_net_infer(m.thB, mlp::kB, &S.B);
  for (int k = threadIdx.x; k < kRadNChi * (2 + 2 * mlp::kChkN); k += blockDim.x) S.chk[k] = m.chk[k];
  for (int k = threadIdx.x; k < kRadNChi; k += blockDim.x) S.lnh[k] = m.lnh32[k];
  const RowQ16 tab{m.q16, m.s0sc};     // fallback: 16-bit table through the caches
  const uint64_t step = step_of(a.step, a.d_step);
  while (true) {
    const uint32_t tile = next_tile(a.sc.ticket, &tile_s);
    if ((int64_t)tile * kEmitMlpThreads >= n_em) break;
    const int64_t r = (int64_t)tile * kEmitMlpThreads + threadIdx.x;
    const bool valid = r < n_em;
    float gph[kKmaxMax];
    double tph[kKmaxMax];
    uint32_t nacc = 0, nev = 0, nrej = 0, ncap = 0, nfx = 0, nfr = 0, nnull = 0, nexc = 0;
    float nx = 0, ny = 0, nz = 0, x = 0, y = 0, z = 0, px = 0, py = 0, pz = 0, g = 1;
    float F[6] = {0, 0, 0, 0, 0, 0};
    double chi = 1.0, Wenv = 0.0, rem = 0.0, tau = 0.0, sq = kEnvSqueeze;
    uint64_t id = 0;
    int64_t i = 0;
    bool recoiled = false;
    if (valid) {
      const EmIdx e = a.em_idx[Cont ? (int64_t)cont_idx[r] : r];
      i = e.i;
      id = a.lep.id[i];
      const EmRec<float> rc = a.rec[e.slot];
#pragma unroll
      for (int c = 0; c < 6; ++c) F[c] = rc.F[c];
      // chi itself, in float64; the lepton pass ran the envelope at its bound
      // rc.chi >= chi, so the squeeze (a lower bound of W / W_env) scales by
      // h_env(chi) / h_env(rc.chi) <= 1
      chi = chi_lepton_f32(rc.p[0], rc.p[1], rc.p[2], rc.F);
      const float he = h_rad_env((float)rc.chi);
      sq = he > 0.f ? kEnvSqueeze * (double)(h_rad_env((float)chi) / he) : 0.0;
      Wenv = rc.W; rem = a.dtd - rc.tau / rc.W;   // time left after the first candidate
      px = rc.p[0]; py = rc.p[1]; pz = rc.p[2];
      x = rc.x[0]; y = rc.x[1]; z = rc.x[2];
      const float pa = sqrtf(px * px + py * py + pz * pz);
      if (pa > 0.f) { nx = px / pa; ny = py / pa; nz = pz / pa; }
      g = sqrtf(1.f + px * px + py * py + pz * pz);
    }
    bool active = valid;       // a candidate is pending at time dt - rem
    for (int k = 0; k < klim; ++k) {
      if (!__any(active)) break;
      mlp::reload_barrier();
      const bool counted = !Cont || k > 0;   // the second pass re-runs candidate 0 silently
      // keep the candidate with probability W / W_env: below the squeeze the
      // draw keeps it at once, above it W comes from net B (packed over the
      // lanes that need it)
      const double ukeep = unit<double>(stream4(id, a.seed, step, kLeptonThin, (uint32_t)k).x);
      const bool need_w = active && !(ukeep < sq);
      bool ok;
      const float lh = mlp_lnh(S.B, chi, need_w, ok);
      bool keep = active && ukeep < sq;
      if (need_w) {
        float h = 0.f;
        if (isfinite(chi) && chi > 0.0) {
          h = ok ? expf(lh) : h_rad<float>((float)chi, S.lnh, m.rg);
          nfr += counted && !ok;
        }
        const double W = kRateUnit * (double)(h / g);
        nexc += counted && (W > Wenv || W < sq * Wenv);
        keep = ukeep * Wenv < W;
      }
      nnull += counted && active && !keep;
      const uint4 u = stream4(id, a.seed, step, kLeptonEvent, (uint32_t)k);
      const float uxi = unit<float>(u.x), urow = unit<float>(u.z);
      const float t = logf(uxi) - log1pf(-uxi);
      const bool in_chi = chi >= kRadChiMin && chi <= kMlpChiMax;
      const float xa0 = mlp::xin(in_chi ? chi : 1.0), xa1 = t / (float)mlp::kTmax;
      const float yA = mlp_packed<0>(S.A, 2, 1, keep, xa0, xa1);   // only the kept candidates
      if (keep) {
        const float lchi = logf((float)chi);
        const float s_hat = mlp::kAShift + mlp::kAScale * yA + lchi + 3.0f * (-log1pf(__expf(-t)));
        bool xi_ok = in_chi && fabsf(t) <= (float)mlp::kTmax && isfinite(s_hat);
        if (xi_ok) {
          const float xp = (lchi - (float)m.rg.rad_lnlo) * (float)m.rg.rad_inv;
          int ii = (int)floorf(xp);
          ii = ii < 0 ? 0 : (ii > kRadNChi - 2 ? kRadNChi - 2 : ii);
          const float w = xp - ii;
          const float P = (1.f - w) * mlp::check_cdf(S.chk, ii, s_hat) + w * mlp::check_cdf(S.chk, ii + 1, s_hat);
          xi_ok = fabsf(P - uxi) <= m.tol;
        }
        float xi, om;
        if (xi_ok) {
          xi = 1.f / (1.f + __expf(-s_hat));
          om = 1.f / (1.f + __expf(s_hat));
        } else {
          sample_rad<float>(tab, (float)chi, uxi, urow, xi, om, m.rg);
        }
        nev += counted;
        nfx += counted && !xi_ok;
        const float gp = xi * g;
        if (gp >= 2.f) {
          if (counted) {
#pragma unroll
            for (int sl = 0; sl < kKmaxMax; ++sl)
              if (sl == (int)nacc) { gph[sl] = gp; tph[sl] = -log(unit<double>(u.w)); }
            ++nacc;
          }
          if (a.recoil) {
            const float gn = fmaxf(om * g, 1.f);
            const float pm = sqrtf(fmaxf(gn * gn - 1.f, 0.f));
            px = nx * pm; py = ny * pm; pz = nz * pm;
            g = gn;
            recoiled = true;
            chi = chi_lepton(px, py, pz, F[0], F[1], F[2], F[3], F[4], F[5]);
            Wenv = isfinite(chi) ? kRateUnit * (double)(h_rad_env((float)chi) / g) : 0.0;
            sq = kEnvSqueeze;
          }
        } else {
          nrej += counted;
        }
      }
      if (active) {
        tau = -log(unit<double>(u.y));
        const bool again = Wenv > 0.0 && tau <= Wenv * rem;
        if (!again) {
          active = false;
        } else if (k + 1 >= a.kmax) {
          ++ncap;
          active = false;
        } else {
          rem -= tau / Wenv;
        }
      }
    }
    // first pass: a lane still active has a further candidate within the step
    const bool cont = !Cont && active;
    if (!Cont) {
      const uint64_t cb = __ballot(cont);
      const int64_t r0 = (int64_t)tile * kEmitMlpThreads + (threadIdx.x & ~63);
      if ((threadIdx.x & 63) == 0 && r0 < n_em) cont_mask[r0 >> 6] = cb;
    }
    if (valid && !cont) {
      a.lep.tau[i] = tau - Wenv * rem;
      if (recoiled) { ((float *)a.lep.px)[i] = px; ((float *)a.lep.py)[i] = py; ((float *)a.lep.pz)[i] = pz; }
    }
    count_lds(cnt_s, cEvents, nev);
    count_lds(cnt_s, cRejected, nrej);
    count_lds(cnt_s, cCapped, ncap);
    count_lds(cnt_s, cPhotons, nacc);
    count_lds(cnt_s, cMlpFallbackXi, nfx);
    count_lds(cnt_s, cMlpFallbackRate, nfr);
    count_lds(cnt_s, cThinned, nnull);
    count_lds(cnt_s, cEnvelopeExceeded, nexc);
    append_photons<float>(a.ph, a.ret, step, a.dtd, tile, n_em, kEmitMlpThreads, nacc, gph, tph, x, y, z, nx, ny, nz,
                          ph0, id0, a.next_id, a.sc, a.counters, scan_s, &off_s, cnt_s);
  }
  count_flush(cnt_s, a.counters);
}

// ================================================================ pairs
template <typename R>
struct PairArgs {
  SpeciesDev ph, el, po;
  FieldDev f;
  const R *L;
  const double *S64;
  const uint16_t *q16;
  const float *s0sc;
  R dt;
  double dtd;
  int move;
  uint64_t *next_id;
  uint32_t seed;
  uint64_t step;
  const int64_t *d_step;
  ScanDev sc;
  unsigned long long *counters;
  int64_t *killed;
  TabRange rg;
  RetireDev ret;
};

constexpr int kPairThreads = 256, kPairItems = 4, kPairTile = kPairThreads * kPairItems;

// Field, chi_ph and pair rate of photon i after its move; false if the fields
// are not finite (then chi is NaN and W = 0).
template <typename R>
__device__ __forceinline__ bool photon_rate_at(const PairArgs<R> &a, const R *L, const R F[6], R kx, R ky, R kz,
                                               R gph, double &chi, double &W) {
  W = 0.0;
  if (!fields_finite<R>(F)) { chi = NAN; return false; }
  if constexpr (sizeof(R) == 4) chi = chi_photon_f32(kx, ky, kz, F);
  else chi = chi_photon(kx, ky, kz, F[0], F[1], F[2], F[3], F[4], F[5]);
  if (!isfinite(chi)) return false;
  if (gph >= (R)2) {
    if constexpr (sizeof(R) == 4) W = kRateUnit * (double)(h_pair<R, true>((R)chi, L, a.rg) * rcp<R>(gph));
    else W = kRateUnit * (double)(h_pair<R>((R)chi, L, a.rg) / gph);
  }
  return true;
}

template <typename R>
__device__ __forceinline__ bool photon_rate(const PairArgs<R> &a, const R *L, int64_t i, R x, R y, R z, R kx,
                                            R ky, R kz, R gph, double &chi, double &W) {
  R F[6];
  field_at<R>(a.f, i, x, y, z, F);
  return photon_rate_at<R>(a, L, F, kx, ky, kz, gph, chi, W);
}

// Float64 pair pass.  One tile of kPairTile photons, kPairItems per thread (photon base + it *
// kPairThreads + thread, so that a pass over `it` is coalesced).  Pass 1 moves
// every photon and decides its event; the offsets of the pairs follow the photon
// index through one scan of per-level counts packed 16 bits per level; pass 2
// recomputes the (rare) events from the photon's stream and writes the pairs.
template <typename R, typename Tab>
__device__ void pair_tile(const PairArgs<R> &a, const Tab &tab, const R *L, uint32_t tile,
                          uint64_t *scan_s, uint64_t *off_s, int64_t n, int64_t e0, int64_t p0,
                          uint64_t id0, uint32_t *cnt) {
  static_assert(kPairThreads <= 0xFFFF, "per-level counts are packed in 16 bits");
  const int64_t base = (int64_t)tile * kPairTile;
  R *X = (R *)a.ph.x, *Y = (R *)a.ph.y, *Z = (R *)a.ph.z;
  const R *KX = (const R *)a.ph.px, *KY = (const R *)a.ph.py, *KZ = (const R *)a.ph.pz;
  uint32_t evbits = 0, nrange = 0, nnan = 0, nret = 0;
  const double t_left = time_left(a.ret, step_of(a.step, a.d_step), a.dtd);
  // loads per photon (all of a thread's photons at once would halve the
  // occupancy in float64); positions are needed to move the photon or to
  // gather from a grid
  const bool need_x = a.move || a.f.kind == QED_FIELD_GRID;
  uint64_t pids[kPairItems];
  R kk[kPairItems][3], xx[kPairItems][3];
  double taus[kPairItems];
#pragma unroll
  for (int it = 0; it < kPairItems; ++it) {
    const int64_t i = base + (int64_t)it * kPairThreads + threadIdx.x;
    const bool v = i < n;
    pids[it] = v ? a.ph.id[i] : kDeadId;
    if (pids[it] != kDeadId) {
      kk[it][0] = KX[i]; kk[it][1] = KY[i]; kk[it][2] = KZ[i];
      taus[it] = a.ph.tau[i];
      xx[it][0] = need_x ? X[i] : (R)0; xx[it][1] = need_x ? Y[i] : (R)0; xx[it][2] = need_x ? Z[i] : (R)0;
    }
    // photons converted earlier and not yet compacted away are skipped
    if (pids[it] == kDeadId) continue;
    const R kx = kk[it][0], ky = kk[it][1], kz = kk[it][2];
    R x = xx[it][0], y = xx[it][1], z = xx[it][2];
    const R gph = root<R>(kx * kx + ky * ky + kz * kz);
    if (a.move && gph > (R)0) {
      if constexpr (sizeof(R) == 4) {
        const R vdt = rcp<R>(gph) * a.dt;
        x += kx * vdt; y += ky * vdt; z += kz * vdt;
      } else {
        x += kx / gph * a.dt; y += ky / gph * a.dt; z += kz / gph * a.dt;
      }
      if (a.f.kind == QED_FIELD_GRID) {
        wrap_coord<R>(x, box_len<R>(a.f, 0)); wrap_coord<R>(y, box_len<R>(a.f, 1));
        wrap_coord<R>(z, box_len<R>(a.f, 2));
      }
      X[i] = x; Y[i] = y; Z[i] = z;
    }
    double chi, W;
    R F[6];
    field_at<R>(a.f, i, x, y, z, F);
    if (photon_rate_at<R>(a, L, F, kx, ky, kz, gph, chi, W)) {
      nrange += chi > a.rg.pair_hi;
    } else {
      ++nnan;
    }
    const double tau = taus[it];
    if (W > 0.0 && tau <= W * a.dtd) {
      evbits |= 1u << it;
    } else {
      const double tn = tau - W * a.dtd;
      a.ph.tau[i] = tn;
      if (retirable(a.ret, tn, (float)gph, t_left)) {
        a.ph.id[i] = kDeadId;
        tally_photon(a.ret, (double)gph);
        ++nret;
      }
    }
  }
  const uint32_t ev = (uint32_t)__popc(evbits);
  count_lds(cnt, cChiRange, nrange);
  count_lds(cnt, cNanChi, nnan);
  count_lds(cnt, cPairs, ev);
  count_lds(cnt, cRetired, nret);
  uint64_t packed = 0;
#pragma unroll
  for (int it = 0; it < kPairItems; ++it) packed |= (uint64_t)((evbits >> it) & 1u) << (16 * it);
  uint64_t tot;
  const uint64_t excl = block_exclusive64(packed, scan_s, &tot);
  uint32_t level0[kPairItems], total = 0;
#pragma unroll
  for (int it = 0; it < kPairItems; ++it) {
    level0[it] = total;
    total += (uint32_t)((tot >> (16 * it)) & 0xFFFFu);
  }
  const uint64_t toff = tile_offset(tile, total, a.sc.status, a.counters, off_s);
  uint32_t ndrop = 0;
  for (int it = 0; it < kPairItems; ++it) {
    if (!((evbits >> it) & 1u)) continue;
    const int64_t i = base + (int64_t)it * kPairThreads + threadIdx.x;
    const uint64_t pid = a.ph.id[i];
    const R kx = KX[i], ky = KY[i], kz = KZ[i];
    const R x = X[i], y = Y[i], z = Z[i];
    const R gph = root<R>(kx * kx + ky * ky + kz * kz);
    double chi, W;
    photon_rate<R>(a, L, i, x, y, z, kx, ky, kz, gph, chi, W);
    const uint4 u = stream4(pid, a.seed, step_of(a.step, a.d_step), kPhotonEvent, 0u);
    R xh, omh;
    sample_pair_half<R>(tab, (R)chi, unit<R>(u.x), unit<R>(u.y), xh, omh, a.rg);
    const bool flip = u.y & 1u;
    const R xe = flip ? omh : xh, xp = flip ? xh : omh;
    const R ge = xe * gph, gpos = xp * gph;
    const double te = -log(unit<double>(u.z)), tp = -log(unit<double>(u.w));
    a.ph.id[i] = kDeadId;
    const uint64_t rank = toff + level0[it] + (uint32_t)((excl >> (16 * it)) & 0xFFFFu);
    const int64_t je = e0 + (int64_t)rank, jp = p0 + (int64_t)rank;
    if (je < a.el.cap && jp < a.po.cap) {
      const R kxh = kx / gph, kyh = ky / gph, kzh = kz / gph;
      const R pe = sqrt(fmax(ge * ge - (R)1, (R)0)), pp = sqrt(fmax(gpos * gpos - (R)1, (R)0));
      ((R *)a.el.x)[je] = x; ((R *)a.el.y)[je] = y; ((R *)a.el.z)[je] = z;
      ((R *)a.el.px)[je] = kxh * pe; ((R *)a.el.py)[je] = kyh * pe; ((R *)a.el.pz)[je] = kzh * pe;
      a.el.tau[je] = te; a.el.id[je] = id0 + 2 * rank;
      ((R *)a.po.x)[jp] = x; ((R *)a.po.y)[jp] = y; ((R *)a.po.z)[jp] = z;
      ((R *)a.po.px)[jp] = kxh * pp; ((R *)a.po.py)[jp] = kyh * pp; ((R *)a.po.pz)[jp] = kzh * pp;
      a.po.tau[jp] = tp; a.po.id[jp] = id0 + 2 * rank + 1;
    } else {
      ndrop += 2;
    }
  }
  count_lds(cnt, cDropped, ndrop);
  const int64_t last = (n - 1) / kPairTile;
  if ((int64_t)tile == last && threadIdx.x == 0) {
    const int64_t tt = (int64_t)(toff + total);
    *a.el.count = e0 + tt < a.el.cap ? e0 + tt : a.el.cap;
    *a.po.count = p0 + tt < a.po.cap ? p0 + tt : a.po.cap;
    *a.next_id = id0 + 2 * (uint64_t)tt;
    if (a.killed) atomicAdd((unsigned long long *)a.killed, (unsigned long long)tt);
  }
}

// Surrogate pair pass (float32): Poisson thinning.  A photon's optical depth
// runs down at the envelope rate W_env (alpha E_S h_pair_env(chi) / gamma_ph at
// the photon's chi, or, with the retirement's field bound, the largest pair
// rate W_max(gamma_ph) it can reach, which needs no field); a photon whose
// optical depth runs out within the step is a candidate: it gets the pair head
// of net B (the table if the output fails its check) and its candidate is kept
// with probability W / W_env; an unkept candidate draws a new optical depth and
// the next candidate of the step follows at the same chi (the photon's chi does
// not change within the step), up to kmax candidates.  Counter k of the photon's
// PHOTON_THIN stream gives (keep draw, new optical depth) of candidate k; a kept
// candidate makes the pair exactly as pair_tile does (PHOTON_EVENT, counter 0).
// Three launches: k_photon_thin moves every photon, runs its optical depth down
// at W_env and marks the candidates in a ballot mask (the other photons'
// optical depths are final there); k_emit_index lists the candidates in photon
// order; k_pair_cand takes them one per lane, so that the net runs on full
// waves of candidates, and appends the pairs at their rank in candidate order,
// i.e. in photon order as pair_tile does.
constexpr int kPTThreads = 256, kPTItems = 4, kPTTile = kPTThreads * kPTItems;

// optical depth of a photon at the end of the step; retired if it can no longer
// convert before the end of the run
__device__ __forceinline__ void photon_settle(const PairArgs<float> &a, int64_t i, double tn, float gph,
                                              double t_left, uint32_t &nret) {
  a.ph.tau[i] = tn;
  if (retirable(a.ret, tn, gph, t_left)) {
    a.ph.id[i] = kDeadId;
    tally_photon(a.ret, (double)gph);
    ++nret;
  }
}

// Envelope rate of a photon with energy gph at chi (chi unused with the field
// bound); 0 below the pair threshold.
__device__ __forceinline__ double photon_envelope(const PairArgs<float> &a, double chi, float gph) {
  if (a.ret.on) return pair_rate_max(gph, a.ret);
  return gph >= 2.f ? kRateUnit * (double)(h_pair_env((float)chi) * rcp<float>(gph)) : 0.0;
}

// FieldFree: the envelope of the retirement's field bound (no field gathered).
template <bool FieldFree>
__global__ __launch_bounds__(kPTThreads) void k_photon_thin(PairArgs<float> a, uint64_t *cmask) {
  __shared__ uint32_t cnt_s[cNumCounters];
  count_zero(cnt_s);
  __syncthreads();
  const int64_t n = *a.ph.count;
  float *X = (float *)a.ph.x, *Y = (float *)a.ph.y, *Z = (float *)a.ph.z;
  const float *KX = (const float *)a.ph.px, *KY = (const float *)a.ph.py, *KZ = (const float *)a.ph.pz;
  const bool need_x = a.move || a.f.kind == QED_FIELD_GRID;
  const uint64_t step = step_of(a.step, a.d_step);
  const double t_left = time_left(a.ret, step, a.dtd);
  uint32_t nrange = 0, nnan = 0, nret = 0;
  for (int64_t tile = blockIdx.x; tile * kPTTile < n; tile += gridDim.x) {
    // every load of the tile first (photon tile * kPTTile + it * kPTThreads + thread)
    uint64_t pids[kPTItems];
    float kk[kPTItems][3], xx[kPTItems][3];
    double taus[kPTItems];
#pragma unroll
    for (int it = 0; it < kPTItems; ++it) {
      const int64_t i = tile * kPTTile + (int64_t)it * kPTThreads + threadIdx.x;
      const bool v = i < n, vx = v && need_x;
      pids[it] = v ? a.ph.id[i] : kDeadId;
      kk[it][0] = v ? KX[i] : 0.f; kk[it][1] = v ? KY[i] : 0.f; kk[it][2] = v ? KZ[i] : 0.f;
      taus[it] = v ? a.ph.tau[i] : 0.0;
      xx[it][0] = vx ? X[i] : 0.f; xx[it][1] = vx ? Y[i] : 0.f; xx[it][2] = vx ? Z[i] : 0.f;
    }
#pragma unroll
    for (int it = 0; it < kPTItems; ++it) {
      const int64_t i = tile * kPTTile + (int64_t)it * kPTThreads + threadIdx.x;
      bool cand = false;
      if (pids[it] != kDeadId) {             // converted photons not yet compacted are skipped
        const float kx = kk[it][0], ky = kk[it][1], kz = kk[it][2];
        const float gph = root<float>(kx * kx + ky * ky + kz * kz);
        float x = xx[it][0], y = xx[it][1], z = xx[it][2];
        if (a.move && gph > 0.f) {
          const float vdt = rcp<float>(gph) * a.dt;
          x += kx * vdt; y += ky * vdt; z += kz * vdt;
          if (a.f.kind == QED_FIELD_GRID) {
            wrap_coord<float>(x, box_len<float>(a.f, 0)); wrap_coord<float>(y, box_len<float>(a.f, 1));
            wrap_coord<float>(z, box_len<float>(a.f, 2));
          }
          X[i] = x; Y[i] = y; Z[i] = z;
        }
        double We = 0.0;
        if constexpr (FieldFree) {
          We = photon_envelope(a, 0.0, gph);
        } else {
          // the local envelope needs chi: the field at the moved position
          float F[6];
          field_at<float>(a.f, i, x, y, z, F);
          if (fields_finite<float>(F)) {
            const double chi = chi_photon_f32(kx, ky, kz, F);
            if (isfinite(chi)) {
              nrange += chi > a.rg.pair_hi;
              We = photon_envelope(a, chi, gph);
            } else {
              ++nnan;
            }
          } else {
            ++nnan;
          }
        }
        cand = We > 0.0 && taus[it] <= We * a.dtd;
        if (!cand) photon_settle(a, i, taus[it] - We * a.dtd, gph, t_left, nret);
      }
      const uint64_t bal = __ballot(cand);
      if ((threadIdx.x & 63) == 0 && i < n) cmask[i >> 6] = bal;   // lane 0 holds a multiple of 64
    }
  }
  count_lds(cnt_s, cChiRange, nrange);
  count_lds(cnt_s, cNanChi, nnan);
  count_lds(cnt_s, cRetired, nret);
  count_flush(cnt_s, a.counters);
  // retired photons are dead too: the compaction of this species must not skip
  if (threadIdx.x == 0 && a.killed && cnt_s[cRetired])
    atomicAdd((unsigned long long *)a.killed, (unsigned long long)cnt_s[cRetired]);
}

constexpr int kPCThreads = 256;   // candidates per tile, one per thread

__global__ __launch_bounds__(kPCThreads) void k_pair_cand(PairArgs<float> a, const int32_t *cidx,
                                                          const int64_t *n_cand, const float *thB, int kmax) {
  __shared__ mlp::NetLdsI B_s;
  __shared__ float L_s[kPairNRate];
  __shared__ uint32_t scan_s[16];
  __shared__ uint32_t tile_s;
  __shared__ uint64_t off_s;
  __shared__ int64_t hdr_s[4];
  __shared__ uint32_t cnt_s[cNumCounters];
  count_zero(cnt_s);
  if (threadIdx.x == 0) {
    hdr_s[0] = *n_cand; hdr_s[1] = *a.el.count; hdr_s[2] = *a.po.count;
    hdr_s[3] = (int64_t)*a.next_id;
  }
  __syncthreads();
  const int64_t nc = hdr_s[0], e0 = hdr_s[1], p0 = hdr_s[2];
  const uint64_t id0 = (uint64_t)hdr_s[3];
  if (nc == 0) return;
  mlp::stage_net_infer(thB, mlp::kB, &B_s);
  for (int k = threadIdx.x; k < kPairNRate; k += blockDim.x) L_s[k] = a.L[k];
  const RowQ16 tab{a.q16, a.s0sc};
  const float *X = (const float *)a.ph.x, *Y = (const float *)a.ph.y, *Z = (const float *)a.ph.z;
  const float *KX = (const float *)a.ph.px, *KY = (const float *)a.ph.py, *KZ = (const float *)a.ph.pz;
  const uint64_t step = step_of(a.step, a.d_step);
  const double t_left = time_left(a.ret, step, a.dtd);
  uint32_t nrange = 0, nnan = 0, nev = 0, nnull = 0, nfr = 0, ncap = 0, nexc = 0, nret = 0, ndrop = 0;
  while (true) {
    const uint32_t tile = next_tile(a.sc.ticket, &tile_s);   // its barriers also publish the staged net
    if ((int64_t)tile * kPCThreads >= nc) break;
    const int64_t r = (int64_t)tile * kPCThreads + threadIdx.x;
    const bool valid = r < nc;
    const int64_t i = valid ? (int64_t)cidx[r] : 0;
    uint64_t pid = kDeadId;
    float kx = 0.f, ky = 0.f, kz = 0.f, x = 0.f, y = 0.f, z = 0.f, gph = 0.f;
    float F[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    double tau = 0.0, chi = 0.0, We = 0.0;
    if (valid) {
      pid = a.ph.id[i];
      kx = KX[i]; ky = KY[i]; kz = KZ[i];
      x = X[i]; y = Y[i]; z = Z[i];                 // moved by k_photon_thin
      tau = a.ph.tau[i];                            // the optical depth before the step
      gph = root<float>(kx * kx + ky * ky + kz * kz);
      field_at<float>(a.f, i, x, y, z, F);
      // (without the field bound k_photon_thin counted these already)
      if (fields_finite<float>(F)) {
        chi = chi_photon_f32(kx, ky, kz, F);
        if (isfinite(chi)) {
          nrange += a.ret.on && chi > a.rg.pair_hi;
        } else {
          nnan += a.ret.on;
          chi = 0.0;
        }
      } else {
        nnan += a.ret.on;
      }
      We = photon_envelope(a, chi, gph);           // the envelope k_photon_thin used
    }
    // with the local envelope the first keep draw below the squeeze keeps the
    // candidate without the net; otherwise the pair head gives W
    const uint4 u0 = stream4(pid, a.seed, step, kPhotonThin, 0u);
    const bool squeeze = !a.ret.on && unit<double>(u0.x) < kEnvSqueeze;
    const bool need_w = valid && !squeeze;
    bool ok;
    const float lh = mlp_lnh_pair(B_s, chi, need_w, ok);
    bool ev = false;
    if (valid) {
      if (squeeze) {
        ev = true;
      } else {
        const float h = !(chi >= kPairChiMin) ? 0.f : (ok ? expf(lh) : h_pair<float, true>((float)chi, L_s, a.rg));
        nfr += !ok;
        const double W = kRateUnit * (double)(h * rcp<float>(gph));
        nexc += W > We || (!a.ret.on && W < kEnvSqueeze * We);
        double rem = a.dtd - tau / We;
        for (int k = 0;; ++k) {
          const uint4 u = k == 0 ? u0 : stream4(pid, a.seed, step, kPhotonThin, (uint32_t)k);
          if (unit<double>(u.x) * We < W) { ev = true; break; }
          ++nnull;
          tau = -log(unit<double>(u.y));
          if (!(tau <= We * rem)) { photon_settle(a, i, tau - We * rem, gph, t_left, nret); break; }
          if (k + 1 >= kmax) { ++ncap; photon_settle(a, i, tau - We * rem, gph, t_left, nret); break; }
          rem -= tau / We;
        }
      }
    }
    nev += ev;
    uint32_t total;
    const uint32_t excl = block_exclusive(ev ? 1u : 0u, scan_s, &total);
    const uint64_t toff = tile_offset(tile, total, a.sc.status, a.counters, &off_s);
    if (ev) {
      const uint4 u = stream4(pid, a.seed, step, kPhotonEvent, 0u);
      float xh, omh;
      sample_pair_half<float>(tab, (float)chi, unit<float>(u.x), unit<float>(u.y), xh, omh, a.rg);
      const bool flip = u.y & 1u;
      const float xe = flip ? omh : xh, xp = flip ? xh : omh;
      const float ge = xe * gph, gpos = xp * gph;
      const double te = -log(unit<double>(u.z)), tp = -log(unit<double>(u.w));
      a.ph.id[i] = kDeadId;
      const uint64_t rank = toff + excl;
      const int64_t je = e0 + (int64_t)rank, jp = p0 + (int64_t)rank;
      if (je < a.el.cap && jp < a.po.cap) {
        const float kxh = kx / gph, kyh = ky / gph, kzh = kz / gph;
        const float pe = sqrtf(fmaxf(ge * ge - 1.f, 0.f)), ppo = sqrtf(fmaxf(gpos * gpos - 1.f, 0.f));
        ((float *)a.el.x)[je] = x; ((float *)a.el.y)[je] = y; ((float *)a.el.z)[je] = z;
        ((float *)a.el.px)[je] = kxh * pe; ((float *)a.el.py)[je] = kyh * pe; ((float *)a.el.pz)[je] = kzh * pe;
        a.el.tau[je] = te; a.el.id[je] = id0 + 2 * rank;
        ((float *)a.po.x)[jp] = x; ((float *)a.po.y)[jp] = y; ((float *)a.po.z)[jp] = z;
        ((float *)a.po.px)[jp] = kxh * ppo; ((float *)a.po.py)[jp] = kyh * ppo; ((float *)a.po.pz)[jp] = kzh * ppo;
        a.po.tau[jp] = tp; a.po.id[jp] = id0 + 2 * rank + 1;
      } else {
        ndrop += 2;
      }
    }
    if ((int64_t)tile == (nc - 1) / kPCThreads && threadIdx.x == 0) {
      const int64_t tt = (int64_t)(toff + total);
      *a.el.count = e0 + tt < a.el.cap ? e0 + tt : a.el.cap;
      *a.po.count = p0 + tt < a.po.cap ? p0 + tt : a.po.cap;
      *a.next_id = id0 + 2 * (uint64_t)tt;
      if (a.killed) atomicAdd((unsigned long long *)a.killed, (unsigned long long)tt);
    }
  }
  count_lds(cnt_s, cChiRange, nrange);
  count_lds(cnt_s, cNanChi, nnan);
  count_lds(cnt_s, cPairs, nev);
  count_lds(cnt_s, cThinned, nnull);
  count_lds(cnt_s, cMlpFallbackRate, nfr);
  count_lds(cnt_s, cCapped, ncap);
  count_lds(cnt_s, cEnvelopeExceeded, nexc);
  count_lds(cnt_s, cRetired, nret);
  count_lds(cnt_s, cDropped, ndrop);
  count_flush(cnt_s, a.counters);
  if (threadIdx.x == 0 && a.killed && cnt_s[cRetired])
    atomicAdd((unsigned long long *)a.killed, (unsigned long long)cnt_s[cRetired]);
}

// Table pair pass (float32) in three launches like the surrogate pass:
// k_photon_table runs every photon's step (move, field, chi_ph, W_pair from
// the table, optical depth) and marks the photons whose optical depth runs out
// within the step in a ballot mask; k_emit_index lists them in photon order;
// k_pair_events makes the pair of each listed photon at its position in the
// list, which is its rank in photon order as pair_tile ranks them, and
// k_pair_commit advances the counts.  The streaming kernel has no scan, so its
// workgroups do not wait on each other; the events (a few per thousand photons)
// are handled one per thread.
// FK: the field kind (a.f.kind), a template parameter so that each kind keeps
// only its own field code and registers: at most 128 (four waves per SIMD),
// 168 on a grid (three waves: its four 27-node gathers in flight).
template <int FK> constexpr int pt_waves() { return FK == QED_FIELD_GRID ? 3 : 4; }
template <int FK>
__global__ __launch_bounds__(kPTThreads, (pt_waves<FK>())) void k_photon_table(PairArgs<float> a, uint64_t *emask) {
  __shared__ float L_s[kPairNRate];
  __shared__ uint32_t cnt_s[cNumCounters];
  count_zero(cnt_s);
  for (int k = threadIdx.x; k < kPairNRate; k += blockDim.x) L_s[k] = a.L[k];
  __syncthreads();
  a.f.kind = FK;
  const int64_t n = *a.ph.count;
  float *X = (float *)a.ph.x, *Y = (float *)a.ph.y, *Z = (float *)a.ph.z;
  const float *KX = (const float *)a.ph.px, *KY = (const float *)a.ph.py, *KZ = (const float *)a.ph.pz;
  const bool need_x = a.move || FK == QED_FIELD_GRID;
  constexpr bool pp = FK == QED_FIELD_PER_PARTICLE;
  const double t_left = time_left(a.ret, step_of(a.step, a.d_step), a.dtd);
  uint32_t nrange = 0, nnan = 0, nret = 0;
  for (int64_t tile = blockIdx.x; tile * kPTTile < n; tile += gridDim.x) {
    // every load of the thread's photons first, so that their latencies overlap
    uint64_t pids[kPTItems];
    float kk[kPTItems][3], xx[kPTItems][3], Fp[kPTItems][pp ? 6 : 1];
    double taus[kPTItems];
#pragma unroll
    for (int it = 0; it < kPTItems; ++it) {
      const int64_t i = tile * kPTTile + (int64_t)it * kPTThreads + threadIdx.x;
      const bool v = i < n, vx = v && need_x;
      pids[it] = v ? a.ph.id[i] : kDeadId;
      kk[it][0] = v ? KX[i] : 0.f; kk[it][1] = v ? KY[i] : 0.f; kk[it][2] = v ? KZ[i] : 0.f;
      taus[it] = v ? a.ph.tau[i] : 0.0;
      xx[it][0] = vx ? X[i] : 0.f; xx[it][1] = vx ? Y[i] : 0.f; xx[it][2] = vx ? Z[i] : 0.f;
      if constexpr (pp) {
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          Fp[it][c] = v ? a.f.pE[c][i] : 0.f;
          Fp[it][3 + c] = v ? a.f.pB[c][i] : 0.f;
        }
      }
    }
#pragma unroll
    for (int it = 0; it < kPTItems; ++it) {
      const int64_t i = tile * kPTTile + (int64_t)it * kPTThreads + threadIdx.x;
      bool ev = false;
      if (pids[it] != kDeadId) {             // converted photons not yet compacted are skipped
        const float kx = kk[it][0], ky = kk[it][1], kz = kk[it][2];
        float x = xx[it][0], y = xx[it][1], z = xx[it][2];
        const float gph = root<float>(kx * kx + ky * ky + kz * kz);
        if (a.move && gph > 0.f) {
          const float vdt = rcp<float>(gph) * a.dt;
          x += kx * vdt; y += ky * vdt; z += kz * vdt;
          if (a.f.kind == QED_FIELD_GRID) {
            wrap_coord<float>(x, box_len<float>(a.f, 0)); wrap_coord<float>(y, box_len<float>(a.f, 1));
            wrap_coord<float>(z, box_len<float>(a.f, 2));
          }
          X[i] = x; Y[i] = y; Z[i] = z;
        }
        double chi, W;
        float F[6];
        if constexpr (pp) {
#pragma unroll
          for (int c = 0; c < 6; ++c) F[c] = Fp[it][c];
        } else {
          field_at<float>(a.f, i, x, y, z, F);
        }
        if (photon_rate_at<float>(a, L_s, F, kx, ky, kz, gph, chi, W)) nrange += chi > a.rg.pair_hi;
        else ++nnan;
        ev = W > 0.0 && taus[it] <= W * a.dtd;
        if (!ev) photon_settle(a, i, taus[it] - W * a.dtd, gph, t_left, nret);
      }
      const uint64_t bal = __ballot(ev);
      if ((threadIdx.x & 63) == 0 && i < n) emask[i >> 6] = bal;   // lane 0 holds a multiple of 64
    }
  }
  count_lds(cnt_s, cChiRange, nrange);
  count_lds(cnt_s, cNanChi, nnan);
  count_lds(cnt_s, cRetired, nret);
  count_flush(cnt_s, a.counters);
  // retired photons are dead too: the compaction of this species must not skip
  if (threadIdx.x == 0 && a.killed && cnt_s[cRetired])
    atomicAdd((unsigned long long *)a.killed, (unsigned long long)cnt_s[cRetired]);
}

__global__ __launch_bounds__(256) void k_pair_events(PairArgs<float> a, const int32_t *eidx, const int64_t *n_ev) {
  __shared__ float L_s[kPairNRate];
  __shared__ int64_t hdr_s[4];
  __shared__ uint32_t cnt_s[cNumCounters];
  count_zero(cnt_s);
  if (threadIdx.x == 0) {
    hdr_s[0] = *n_ev; hdr_s[1] = *a.el.count; hdr_s[2] = *a.po.count; hdr_s[3] = (int64_t)*a.next_id;
  }
  __syncthreads();
  const int64_t nev = hdr_s[0], e0 = hdr_s[1], p0 = hdr_s[2];
  const uint64_t id0 = (uint64_t)hdr_s[3];
  if (nev == 0 || (int64_t)blockIdx.x * blockDim.x >= nev) return;
  for (int k = threadIdx.x; k < kPairNRate; k += blockDim.x) L_s[k] = a.L[k];
  __syncthreads();
  const RowQ16 tab{a.q16, a.s0sc};
  const float *X = (const float *)a.ph.x, *Y = (const float *)a.ph.y, *Z = (const float *)a.ph.z;
  const float *KX = (const float *)a.ph.px, *KY = (const float *)a.ph.py, *KZ = (const float *)a.ph.pz;
  const uint64_t step = step_of(a.step, a.d_step);
  uint32_t ndrop = 0;
  for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < nev; r += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = eidx[r];
    const uint64_t pid = a.ph.id[i];
    const float kx = KX[i], ky = KY[i], kz = KZ[i];
    const float x = X[i], y = Y[i], z = Z[i];      // moved by k_photon_table
    const float gph = root<float>(kx * kx + ky * ky + kz * kz);
    double chi, W;
    photon_rate<float>(a, L_s, i, x, y, z, kx, ky, kz, gph, chi, W);
    const uint4 u = stream4(pid, a.seed, step, kPhotonEvent, 0u);
    float xh, omh;
    sample_pair_half<float>(tab, (float)chi, unit<float>(u.x), unit<float>(u.y), xh, omh, a.rg);
    const bool flip = u.y & 1u;
    const float xe = flip ? omh : xh, xp = flip ? xh : omh;
    const float ge = xe * gph, gpos = xp * gph;
    const double te = -log(unit<double>(u.z)), tp = -log(unit<double>(u.w));
    a.ph.id[i] = kDeadId;
    const int64_t je = e0 + r, jp = p0 + r;
    if (je < a.el.cap && jp < a.po.cap) {
      const float kxh = kx / gph, kyh = ky / gph, kzh = kz / gph;
      const float pe = sqrtf(fmaxf(ge * ge - 1.f, 0.f)), ppo = sqrtf(fmaxf(gpos * gpos - 1.f, 0.f));
      ((float *)a.el.x)[je] = x; ((float *)a.el.y)[je] = y; ((float *)a.el.z)[je] = z;
      ((float *)a.el.px)[je] = kxh * pe; ((float *)a.el.py)[je] = kyh * pe; ((float *)a.el.pz)[je] = kzh * pe;
      a.el.tau[je] = te; a.el.id[je] = id0 + 2 * (uint64_t)r;
      ((float *)a.po.x)[jp] = x; ((float *)a.po.y)[jp] = y; ((float *)a.po.z)[jp] = z;
      ((float *)a.po.px)[jp] = kxh * ppo; ((float *)a.po.py)[jp] = kyh * ppo; ((float *)a.po.pz)[jp] = kzh * ppo;
      a.po.tau[jp] = tp; a.po.id[jp] = id0 + 2 * (uint64_t)r + 1;
    } else {
      ndrop += 2;
    }
  }
  count_lds(cnt_s, cDropped, ndrop);
  count_flush(cnt_s, a.counters);
}

// After the events: pairs appended (up to the capacities), ids used, photons killed.
__global__ void k_pair_commit(PairArgs<float> a, const int64_t *n_ev) {
  const int64_t tt = *n_ev, e0 = *a.el.count, p0 = *a.po.count;
  *a.el.count = e0 + tt < a.el.cap ? e0 + tt : a.el.cap;
  *a.po.count = p0 + tt < a.po.cap ? p0 + tt : a.po.cap;
  *a.next_id += 2 * (uint64_t)tt;
  if (tt) atomicAdd(&a.counters[cPairs], (unsigned long long)tt);
  if (a.killed && tt) atomicAdd((unsigned long long *)a.killed, (unsigned long long)tt);
}

__global__ __launch_bounds__(kPairThreads) void k_pairs_f64(PairArgs<double> a) {
  __shared__ double L_s[kPairNRate];
  __shared__ uint64_t scan_s[16];
  __shared__ uint32_t tile_s;
  __shared__ uint64_t off_s;
  __shared__ int64_t hdr_s[4];
  __shared__ uint32_t cnt_s[cNumCounters];
  count_zero(cnt_s);
  if (threadIdx.x == 0) {
    hdr_s[0] = *a.ph.count; hdr_s[1] = *a.el.count; hdr_s[2] = *a.po.count;
    hdr_s[3] = (int64_t)*a.next_id;
  }
  __syncthreads();
  const int64_t n = hdr_s[0], e0 = hdr_s[1], p0 = hdr_s[2];
  const uint64_t id0 = (uint64_t)hdr_s[3];
  if (n == 0) return;
  for (int k = threadIdx.x; k < kPairNRate; k += blockDim.x) L_s[k] = a.L[k];
  const RowF64 tab{a.S64};
  while (true) {
    const uint32_t tile = next_tile(a.sc.ticket, &tile_s);
    if ((int64_t)tile * kPairTile >= n) break;
    pair_tile<double>(a, tab, L_s, tile, scan_s, &off_s, n, e0, p0, id0, cnt_s);
  }
  count_flush(cnt_s, a.counters);
  // retired photons are dead too: the compaction of this species must not skip
  if (threadIdx.x == 0 && a.killed && cnt_s[cRetired])
    atomicAdd((unsigned long long *)a.killed, (unsigned long long)cnt_s[cRetired]);
}

// ============================================================== compact
constexpr int kCThreads = 256, kCItems = 4, kCTile = kCThreads * kCItems;

template <typename R>
__global__ __launch_bounds__(kCThreads) void k_compact(SpeciesDev sp, ScanDev sc,
                                                       unsigned long long *counters, int64_t *killed) {
  __shared__ uint32_t scan_s[16];
  __shared__ uint32_t tile_s;
  __shared__ uint64_t off_s;
  // killed: particles marked dead since the last compaction of this species, when
  // known (pair creation keeps it); nothing to do if none
  if (killed && *killed == 0) return;
  const int64_t n = *sp.count;
  R *A[6] = {(R *)sp.x, (R *)sp.y, (R *)sp.z, (R *)sp.px, (R *)sp.py, (R *)sp.pz};
  while (true) {
    const uint32_t tile = next_tile(sc.ticket, &tile_s);
    const int64_t base = (int64_t)tile * kCTile;
    if (base >= n) {
      if (tile == 0 && killed && threadIdx.x == 0) *killed = 0;
      break;
    }
    R v[kCItems][6];
    double tau[kCItems];
    uint64_t id[kCItems];
    uint32_t alive = 0, na = 0;
    const int64_t i0 = base + (int64_t)threadIdx.x * kCItems;
#pragma unroll
    for (int it = 0; it < kCItems; ++it) {
      const int64_t i = i0 + it;
      id[it] = kDeadId;
      if (i < n) {
#pragma unroll
        for (int c = 0; c < 6; ++c) v[it][c] = A[c][i];
        tau[it] = sp.tau[i];
        id[it] = sp.id[i];
      }
      if (id[it] != kDeadId) { alive |= 1u << it; ++na; }
    }
    // every load of the tile has returned before its count is published: later
    // tiles may overwrite these elements as soon as they see the count
    __builtin_amdgcn_s_waitcnt(0);
    uint32_t total;
    const uint32_t off = block_exclusive(na, scan_s, &total);
    const uint64_t toff = tile_offset(tile, total, sc.status, counters, &off_s);
    uint64_t r = toff + off;
#pragma unroll
    for (int it = 0; it < kCItems; ++it) {
      if (alive & (1u << it)) {
#pragma unroll
        for (int c = 0; c < 6; ++c) A[c][r] = v[it][c];
        sp.tau[r] = tau[it];
        sp.id[r] = id[it];
        ++r;
      }
    }
    const int64_t last = (n - 1) / kCTile;
    if ((int64_t)tile == last && threadIdx.x == 0) {
      // every tile has been claimed: workgroups that start later find no tile
      const int64_t nn = (int64_t)(toff + total);
      atomicAdd(&counters[cCompacted], (unsigned long long)(n - nn));
      *sp.count = nn;
      if (killed) *killed = 0;
    }
  }
}

// ================================================================ misc
__global__ void k_set_i64(int64_t *p, int64_t v) { *p = v; }

__global__ void k_zero_scan(uint32_t *ticket, uint64_t *status, int64_t n) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i == 0) *ticket = 0;
  if (i < n) status[i] = 0;
}

// Both scan regions at once: words [0, n0) of region 0, [0, n1) of region 1.
__global__ void k_zero_scan2(uint32_t *ticket, uint64_t *status, int64_t len, int64_t n0, int64_t n1) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i == 0) { ticket[0] = 0; ticket[1] = 0; }
  if (i < n0) status[i] = 0;
  if (i < n1) status[len + i] = 0;
}

__global__ void k_init_tau(const uint64_t *id, double *tau, const int64_t *count, uint32_t seed,
                           uint64_t step_v, const int64_t *d_step, int64_t cap) {
  const int64_t n = *count;
  const uint64_t step = step_of(step_v, d_step);
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n && i < cap;
       i += (int64_t)gridDim.x * blockDim.x) {
    const uint4 u = stream4(id[i], seed, step, kInitTau, 0u);
    tau[i] = -log(unit<double>(u.x));
  }
}

// The fields depend on x only, so every row (iy, iz) of the grid holds the same
// 6 n floats: each workgroup builds that row in LDS once (cos x, sin x per
// column) and streams it to its share of the rows with V-wide coalesced stores
// (float4 when rows and grid are 16-byte aligned, else float2).
template <typename V>
__global__ void k_standing_wave(float *grid, int n, double dx, double a0, double t0, double dt_step,
                                const int64_t *d_step) {
  extern __shared__ __align__(16) float row_s[];
  const double t = d_step ? t0 + dt_step * (double)*d_step : t0;
  const double ct = cos(t), st = sin(t);
  for (int ix = threadIdx.x; ix < n; ix += blockDim.x) {
    const double x = ix * dx;
    const double ca = a0 * cos(x), sa = a0 * sin(x);
    float *o = row_s + 6 * ix;
    o[0] = 0.0f; o[1] = (float)(ca * ct); o[2] = (float)(ca * st);
    o[3] = 0.0f; o[4] = (float)(sa * ct); o[5] = (float)(sa * st);
  }
  __syncthreads();
  constexpr int W = (int)(sizeof(V) / sizeof(float));
  const int per_row = 6 * n / W;
  const int64_t rows = (int64_t)n * n;
  const V *src = reinterpret_cast<const V *>(row_s);
  for (int k = threadIdx.x; k < per_row; k += blockDim.x) {
    const V v = src[k];
    for (int64_t r = blockIdx.x; r < rows; r += gridDim.x) reinterpret_cast<V *>(grid + r * 6 * n)[k] = v;
  }
}

// chi of every particle [0, *count) with the fields at its position: Eq. (2)
// for leptons (photon == 0) or Eq. (3) for photons, with the device functions
// the step uses (float32 species: chi_*_f32, float64: chi_lepton / chi_photon).
template <typename R>
__global__ void k_eval_chi(SpeciesDev sp, FieldDev f, int photon, double *out) {
  const int64_t n = *sp.count;
  const R *X = (const R *)sp.x, *Y = (const R *)sp.y, *Z = (const R *)sp.z;
  const R *PX = (const R *)sp.px, *PY = (const R *)sp.py, *PZ = (const R *)sp.pz;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    R F[6];
    field_at<R>(f, i, X[i], Y[i], Z[i], F);
    double chi;
    if constexpr (sizeof(R) == 4)
      chi = photon ? chi_photon_f32(PX[i], PY[i], PZ[i], F) : chi_lepton_f32(PX[i], PY[i], PZ[i], F);
    else
      chi = photon ? chi_photon(PX[i], PY[i], PZ[i], F[0], F[1], F[2], F[3], F[4], F[5])
                   : chi_lepton(PX[i], PY[i], PZ[i], F[0], F[1], F[2], F[3], F[4], F[5]);
    out[i] = chi;
  }
}

template <typename R, typename Tab>
__device__ void sample_one(const Tab &tab, const R *lnh, const R *L, double chi, double gamma,
                           uint64_t id, uint32_t seed, uint64_t step, float *lnw, float *xi_out,
                           float *lnwp, int64_t i, const TabRange &rg) {
  const R h = h_rad<R>((R)chi, lnh, rg);
  lnw[i] = (float)log(kRateUnit * (double)h / gamma);
  const uint4 u = stream4(id, seed, step, kLeptonEvent, 0u);
  R xi, om;
  sample_rad<R>(tab, (R)chi, unit<R>(u.x), unit<R>(u.z), xi, om, rg);
  xi_out[i] = (float)xi;
  if (lnwp) {
    const R hp = gamma >= 2.0 ? h_pair<R>((R)chi, L, rg) : (R)0;
    lnwp[i] = (float)log(kRateUnit * (double)hp / gamma);
  }
}

__global__ void k_sample_f64(const double *chi, const double *gamma, const uint64_t *id, int64_t n,
                             const double *lnh, const double *L, const double *S64, uint32_t seed,
                             uint64_t step_v, const int64_t *d_step, float *lnw, float *xi, float *lnwp,
                             TabRange rg) {
  const uint64_t step = step_of(step_v, d_step);
  const RowF64 tab{S64};
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    sample_one<double>(tab, lnh, L, chi[i], gamma[i], id[i], seed, step, lnw, xi, lnwp, i, rg);
}

__global__ void k_sample_f32(const double *chi, const double *gamma, const uint64_t *id, int64_t n,
                             const float *lnh, const float *L, const uint16_t *q16, const float *s0sc,
                             uint32_t seed, uint64_t step_v, const int64_t *d_step, float *lnw, float *xi,
                             float *lnwp, TabRange rg) {
  const uint64_t step = step_of(step_v, d_step);
  const RowQ16 tab{q16, s0sc};
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    sample_one<float>(tab, lnh, L, chi[i], gamma[i], id[i], seed, step, lnw, xi, lnwp, i, rg);
}

}  // namespace qed

// =============================================================== launchers
namespace qed {

static_assert(sizeof(EmRec<float>) == 80 && sizeof(EmRec<double>) == kEmRecMaxBytes, "emitter record size");

static SpeciesDev dev_species(const qed_species_t *s) {
  return SpeciesDev{s->x, s->y, s->z, s->px, s->py, s->pz, s->tau, s->id, s->capacity, s->count};
}

static FieldDev dev_fields(const qed_fields_t *f) {
  FieldDev d{};
  if (!f) { d.kind = QED_FIELD_UNIFORM; return d; }
  d.kind = f->kind; d.nx = f->nx; d.ny = f->ny; d.nz = f->nz; d.grid = f->grid;
  d.dx = f->dx; d.dy = f->dy; d.dz = f->dz;
  if (f->kind == QED_FIELD_GRID) {
    d.idx = 1.0 / f->dx; d.idy = 1.0 / f->dy; d.idz = 1.0 / f->dz;
    d.fid[0] = (float)d.idx; d.fid[1] = (float)d.idy; d.fid[2] = (float)d.idz;
    d.L[0] = f->dx * f->nx; d.L[1] = f->dy * f->ny; d.L[2] = f->dz * f->nz;
    for (int c = 0; c < 3; ++c) d.fL[c] = (float)d.L[c];
  }
  for (int c = 0; c < 3; ++c) { d.E[c] = f->E[c]; d.B[c] = f->B[c]; d.pE[c] = f->pE[c]; d.pB[c] = f->pB[c]; }
  return d;
}

// Clears the ticket and the first ntiles + 1 status words of a scan state
// (a kernel, not a memset, so that the clear can be captured in a graph).
static hipError_t zero_scan_at(uint32_t *ticket, uint64_t *status, int64_t status_len, int64_t ntiles,
                               hipStream_t st) {
  const int64_t n = ntiles + 1;
  if (n > status_len) return hipErrorInvalidValue;   // the caller sized the status array
  hipLaunchKernelGGL(k_zero_scan, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, ticket, status, n);
  return hipGetLastError();
}

static hipError_t zero_scan(qed_ctx *c, int64_t ntiles, hipStream_t st) {
  return zero_scan_at(c->d_ticket, c->d_status, c->status_len, ntiles, st);   // reserve() sizes it
}

// Blocks of a gather/push launch for a species of this capacity, IT particles
// per thread: every tile has its block (chunks per XCD, times the chunk, times
// the 8 XCDs).
static unsigned gp_grid(int64_t capacity, int it) {
  const int64_t tile = (int64_t)kGPThreads * it;
  const int64_t ntiles = (capacity + tile - 1) / tile;
  const int64_t cpx = ((ntiles + kGPChunk - 1) / kGPChunk + kXcds - 1) / kXcds;
  return (unsigned)(cpx * kGPChunk * kXcds);
}

// Two particles per thread (k_gather_push2) for a dense float32 species on a grid.
static bool gp_dense(const qed_fields_t *f, const qed_species_t *sp) {
  return sp->dtype == QED_F32 && f->kind == QED_FIELD_GRID &&
         sp->capacity >= kDenseGP * (int64_t)f->nx * f->ny * f->nz;
}

template <typename R, bool M1, bool Thin>
static void launch_gp_kind_m(const GPArgs<R> &a, int kind, int64_t cap, bool dense, hipStream_t st) {
  if (kind == QED_FIELD_GRID) {
    if constexpr (sizeof(R) == 4 && !M1) {
      if (dense) {
        hipLaunchKernelGGL((k_gather_push2<Thin>), dim3(gp_grid(cap, 2)), dim3(kGPThreads), 0, st, a);
        return;
      }
    }
    hipLaunchKernelGGL((k_gather_push<R, QED_FIELD_GRID, M1, Thin>), dim3(gp_grid(cap, 1)), dim3(kGPThreads), 0, st,
                       a);
  } else if (kind == QED_FIELD_UNIFORM) {
    hipLaunchKernelGGL((k_gather_push<R, QED_FIELD_UNIFORM, M1, Thin>), dim3(gp_grid(cap, 1)), dim3(kGPThreads), 0,
                       st, a);
  } else {
    hipLaunchKernelGGL((k_gather_push<R, QED_FIELD_PER_PARTICLE, M1, Thin>), dim3(gp_grid(cap, 1)),
                       dim3(kGPThreads), 0, st, a);
  }
}

template <typename R>
static void launch_gp_kind(const GPArgs<R> &a, int kind, int64_t cap, bool dense, hipStream_t st) {
  if (a.gen) launch_gp_kind_m<R, true, false>(a, kind, cap, dense, st);
  else launch_gp_kind_m<R, false, false>(a, kind, cap, dense, st);
}

static RetireDev retire_dev(const qed_ctx *c) {
  return RetireDev{c->ret_on, c->ret_t_end, (float)(c->ret_field * kInvES), c->d_tally};
}

static MlpDev mlp_dev(qed_ctx *c) {
  return MlpDev{c->range, c->mlp_theta[0], c->mlp_theta[1], c->rad_chk, c->rad_lnh32, c->rad_q16, c->rad_s0sc, 2e-3f};
}

// Dynamic LDS above the default limit (surrogate emission); called once per
// context, with the context's device current.
hipError_t step_set_attributes() {
  // the standing-wave row: 6 n floats for n up to kMaxWaveGrid
  const int row_bytes = 6 * kMaxWaveGrid * (int)sizeof(float);
  hipError_t e = hipFuncSetAttribute((const void *)k_emit_mlp<false>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                     (int)sizeof(EmitMlpLds));
  if (e == hipSuccess)
    e = hipFuncSetAttribute((const void *)k_emit_mlp<true>, hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)sizeof(EmitMlpLds));
  if (e == hipSuccess)
    e = hipFuncSetAttribute((const void *)k_standing_wave<float4>, hipFuncAttributeMaxDynamicSharedMemorySize,
                            row_bytes);
  if (e == hipSuccess)
    e = hipFuncSetAttribute((const void *)k_standing_wave<float2>, hipFuncAttributeMaxDynamicSharedMemorySize,
                            row_bytes);
  return e;
}

static int gen_mode(const qed_ctx *c) {
  if (!(c->params.flags & QED_FLAG_METHOD_I)) return 0;
  return (c->params.flags & QED_FLAG_NO_SUBSTEP) ? 2 : 1;
}

hipError_t launch_gather_push(qed_ctx *c, const qed_fields_t *f, const qed_species_t *sp, int charge,
                              double dt, int64_t step, hipStream_t st) {
  const int gen = gen_mode(c);
  const int64_t *dstep = step < 0 ? c->d_step : nullptr;
  const int64_t cap = sp->capacity;
  const bool use_mlp = (c->params.flags & QED_FLAG_SURROGATE) && sp->dtype == QED_F32;
  if (use_mlp) {
    // surrogate path: the same pass with the rate envelope (thinning); the
    // emission pass evaluates the nets at the candidates
    GPArgs<float> a{dev_species(sp), dev_fields(f), c->rad_lnh32, (float)charge, (float)dt, dt, c->em_mask,
                    (EmRec<float> *)c->em_rec, c->d_counters, 0, c->params.seed, (uint64_t)step, dstep, c->range};
    launch_gp_kind_m<float, false, true>(a, f->kind, cap, gp_dense(f, sp), st);
  } else if (sp->dtype == QED_F32) {
    GPArgs<float> a{dev_species(sp), dev_fields(f), c->rad_lnh32, (float)charge, (float)dt, dt, c->em_mask,
                    (EmRec<float> *)c->em_rec, c->d_counters, gen, c->params.seed, (uint64_t)step, dstep, c->range};
    launch_gp_kind<float>(a, f->kind, cap, gp_dense(f, sp), st);
  } else {
    GPArgs<double> a{dev_species(sp), dev_fields(f), c->rad_lnh64, (double)charge, dt, dt, c->em_mask,
                     (EmRec<double> *)c->em_rec, c->d_counters, gen, c->params.seed, (uint64_t)step, dstep, c->range};
    launch_gp_kind<double>(a, f->kind, cap, false, st);
  }
  return hipGetLastError();
}

hipError_t launch_emit(qed_ctx *c, const qed_species_t *lep, const qed_species_t *ph, int64_t step,
                       hipStream_t st) {
  const bool use_mlp = lep->dtype == QED_F32 && (c->params.flags & QED_FLAG_SURROGATE);
  // ordered emitter list from the mask of the last gather/push
  const bool wide = lep->capacity >= kEIWideFrom;
  const int64_t eit = wide ? ei_tile<8>() : ei_tile<1>();
  const int64_t etiles = (lep->capacity + eit - 1) / eit;
  const unsigned eig = (unsigned)(etiles < 2 * (int64_t)c->n_cu ? etiles : 2 * (int64_t)c->n_cu);   // persistent
  // one launch clears both scans: region 1 for the index, region 0 for the events
  const bool m1 = gen_mode(c) != 0;
  const int tile = use_mlp ? kEmitMlpThreads
                           : (lep->dtype == QED_F32 ? (m1 ? emit_threads<float, true>() : emit_threads<float, false>())
                                                    : (m1 ? emit_threads<double, true>() : emit_threads<double, false>()));
  const int64_t ntiles = (lep->capacity + tile - 1) / tile;
  const int64_t n0 = ntiles + 1, n1 = etiles + 1, nz = n0 > n1 ? n0 : n1;
  if (nz > c->status_len) return hipErrorInvalidValue;   // reserve() sizes the status regions
  hipLaunchKernelGGL(k_zero_scan2, dim3((unsigned)((nz + 255) / 256)), dim3(256), 0, st, c->d_ticket, c->d_status,
                     c->status_len, n0, n1);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const ScanDev isc{c->d_ticket + 1, c->d_status + c->status_len};
  if (wide)
    hipLaunchKernelGGL((k_emit_index<8, EmIdx>), dim3(eig), dim3(kEIThreads), 0, st, c->em_mask, lep->count,
                     c->em_idx, c->d_n_emit, isc, c->d_counters);
  else
    hipLaunchKernelGGL((k_emit_index<1, EmIdx>), dim3(eig), dim3(kEIThreads), 0, st, c->em_mask, lep->count,
                     c->em_idx, c->d_n_emit, isc, c->d_counters);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  const ScanDev sc{c->d_ticket, c->d_status};
  const int recoil = (c->params.flags & QED_FLAG_NO_RECOIL) ? 0 : 1;
  // persistent workgroups: one per CU for the surrogate (its nets fill the LDS),
  // up to four per CU otherwise
  const int64_t wgs = use_mlp ? (int64_t)c->n_cu : 4 * (int64_t)c->n_cu;
  const unsigned grid = (unsigned)(ntiles < wgs ? ntiles : wgs);
  const int64_t *dstep = step < 0 ? c->d_step : nullptr;
  if (use_mlp) {
    EmitArgs<float> a{dev_species(lep), dev_species(ph), c->rad_lnh32, c->rad_S64, c->rad_q16,
                      c->rad_s0sc, c->em_idx, (const EmRec<float> *)c->em_rec, c->d_n_emit,
                      c->d_next_id, c->params.seed, c->params.kmax, recoil, (uint64_t)step, dstep, sc,
                      c->d_counters, gen_mode(c), c->em_dt, c->range, retire_dev(c)};
    hipLaunchKernelGGL(k_emit_mlp<false>, dim3(grid), dim3(kEmitMlpThreads), sizeof(EmitMlpLds), st, a, mlp_dev(c),
                       c->em_mask, (const int32_t *)nullptr, (const int64_t *)nullptr);
    if (c->params.kmax > 1) {
      // the emitters with a further candidate (bits in the emitter mask, which
      // the list above no longer needs), listed in emitter order and finished
      // in a second pass; both scan regions cleared again
      hipLaunchKernelGGL(k_zero_scan2, dim3((unsigned)((nz + 255) / 256)), dim3(256), 0, st, c->d_ticket,
                         c->d_status, c->status_len, n0, n1);
      if (wide)
        hipLaunchKernelGGL((k_emit_index<8, int32_t>), dim3(eig), dim3(kEIThreads), 0, st, c->em_mask, c->d_n_emit,
                           c->cont_idx, c->d_n_cont, isc, c->d_counters);
      else
        hipLaunchKernelGGL((k_emit_index<1, int32_t>), dim3(eig), dim3(kEIThreads), 0, st, c->em_mask, c->d_n_emit,
                           c->cont_idx, c->d_n_cont, isc, c->d_counters);
      hipLaunchKernelGGL(k_emit_mlp<true>, dim3(grid), dim3(kEmitMlpThreads), sizeof(EmitMlpLds), st, a,
                         mlp_dev(c), (uint64_t *)nullptr, c->cont_idx, c->d_n_cont);
    }
  } else if (lep->dtype == QED_F32) {
    EmitArgs<float> a{dev_species(lep), dev_species(ph), c->rad_lnh32, c->rad_S64, c->rad_q16,
                      c->rad_s0sc, c->em_idx, (const EmRec<float> *)c->em_rec, c->d_n_emit,
                      c->d_next_id, c->params.seed, c->params.kmax, recoil, (uint64_t)step, dstep, sc,
                      c->d_counters, gen_mode(c), c->em_dt, c->range, retire_dev(c)};
    if (a.gen) hipLaunchKernelGGL(k_emit_f32<true>, dim3(grid), dim3(emit_threads<float, true>()), 0, st, a);
    else hipLaunchKernelGGL(k_emit_f32<false>, dim3(grid), dim3(emit_threads<float, false>()), 0, st, a);
  } else {
    EmitArgs<double> a{dev_species(lep), dev_species(ph), c->rad_lnh64, c->rad_S64, c->rad_q16,
                       c->rad_s0sc, c->em_idx, (const EmRec<double> *)c->em_rec, c->d_n_emit,
                       c->d_next_id, c->params.seed, c->params.kmax, recoil, (uint64_t)step, dstep, sc,
                       c->d_counters, gen_mode(c), c->em_dt, c->range, retire_dev(c)};
    if (a.gen) hipLaunchKernelGGL(k_emit_f64<true>, dim3(grid), dim3(emit_threads<double, true>()), 0, st, a);
    else hipLaunchKernelGGL(k_emit_f64<false>, dim3(grid), dim3(emit_threads<double, false>()), 0, st, a);
  }
  return hipGetLastError();
}

hipError_t launch_pairs(qed_ctx *c, const qed_fields_t *f, const qed_species_t *ph,
                        const qed_species_t *el, const qed_species_t *po, double dt, int64_t step,
                        hipStream_t st) {
  const int64_t ntiles = (ph->capacity + kPairTile - 1) / kPairTile;
  const bool thin = (c->params.flags & QED_FLAG_SURROGATE) && ph->dtype == QED_F32;
  if (ph->dtype != QED_F32) {   // (the float32 passes clear their scans themselves)
    hipError_t e = zero_scan(c, ntiles, st);
    if (e != hipSuccess) return e;
  }
  const ScanDev sc{c->d_ticket, c->d_status};
  const int move = (c->params.flags & QED_FLAG_STATIC_PHOTONS) ? 0 : 1;
  const int64_t wgs = (int64_t)c->n_cu * 4;   // persistent, tiles from the ticket
  const unsigned grid = (unsigned)(ntiles < wgs ? ntiles : wgs);
  // killed-photon count: known only if this species was compacted before
  int64_t *killed = ((c->params.flags & QED_FLAG_TRACK_DEAD) && c->killed_owner == ph->x) ? c->d_killed : nullptr;
  if (ph->dtype == QED_F32) {
    PairArgs<float> a{dev_species(ph), dev_species(el), dev_species(po), dev_fields(f), c->pair_L32,
                      c->pair_S64, c->pair_q16, c->pair_s0sc, (float)dt, dt, move, c->d_next_id,
                      c->params.seed, (uint64_t)step, step < 0 ? c->d_step : nullptr, sc, c->d_counters, killed, c->range,
                      retire_dev(c)};
    if (thin) {
      // thinning pass, candidate list, candidates (region 0 of the scan state
      // for the candidates' appends, region 1 for the list)
      const bool wide = ph->capacity >= kEIWideFrom;
      const int64_t eit = wide ? ei_tile<8>() : ei_tile<1>();
      const int64_t etiles = (ph->capacity + eit - 1) / eit;
      const unsigned eig = (unsigned)(etiles < 2 * (int64_t)c->n_cu ? etiles : 2 * (int64_t)c->n_cu);
      const int64_t ctiles = (ph->capacity + kPCThreads - 1) / kPCThreads;
      const int64_t n0 = ctiles + 1, n1 = etiles + 1, nz = n0 > n1 ? n0 : n1;
      if (nz > c->status_len || ph->capacity > c->cand_cap) return hipErrorInvalidValue;
      hipLaunchKernelGGL(k_zero_scan2, dim3((unsigned)((nz + 255) / 256)), dim3(256), 0, st, c->d_ticket,
                         c->d_status, c->status_len, n0, n1);
      const int64_t ttiles = (ph->capacity + kPTTile - 1) / kPTTile, twgs = (int64_t)c->n_cu * 8;
      const unsigned tgrid = (unsigned)(ttiles < twgs ? ttiles : twgs);
      if (a.ret.on)
        hipLaunchKernelGGL(k_photon_thin<true>, dim3(tgrid), dim3(kPTThreads), 0, st, a, c->cand_mask);
      else
        hipLaunchKernelGGL(k_photon_thin<false>, dim3(tgrid), dim3(kPTThreads), 0, st, a, c->cand_mask);
      const ScanDev isc{c->d_ticket + 1, c->d_status + c->status_len};
      if (wide)
        hipLaunchKernelGGL((k_emit_index<8, int32_t>), dim3(eig), dim3(kEIThreads), 0, st, c->cand_mask,
                           ph->count, c->cand_idx, c->d_n_cand, isc, c->d_counters);
      else
        hipLaunchKernelGGL((k_emit_index<1, int32_t>), dim3(eig), dim3(kEIThreads), 0, st, c->cand_mask,
                           ph->count, c->cand_idx, c->d_n_cand, isc, c->d_counters);
      const int64_t cwgs = (int64_t)c->n_cu * 4;
      hipLaunchKernelGGL(k_pair_cand, dim3((unsigned)(ctiles < cwgs ? ctiles : cwgs)), dim3(kPCThreads), 0, st, a,
                         c->cand_idx, c->d_n_cand, c->mlp_theta[1], c->params.kmax);
    } else {
      // streaming pass, event list (region 1 of the scan state), events, counts
      const bool wide = ph->capacity >= kEIWideFrom;
      const int64_t eit = wide ? ei_tile<8>() : ei_tile<1>();
      const int64_t etiles = (ph->capacity + eit - 1) / eit;
      const unsigned eig = (unsigned)(etiles < 2 * (int64_t)c->n_cu ? etiles : 2 * (int64_t)c->n_cu);
      if (etiles + 1 > c->status_len || ph->capacity > c->cand_cap) return hipErrorInvalidValue;
      hipLaunchKernelGGL(k_zero_scan2, dim3((unsigned)((etiles + 1 + 255) / 256)), dim3(256), 0, st, c->d_ticket,
                         c->d_status, c->status_len, (int64_t)1, etiles + 1);
      const int64_t ttiles = (ph->capacity + kPTTile - 1) / kPTTile, twgs = (int64_t)c->n_cu * 8;
      const unsigned tgrid = (unsigned)(ttiles < twgs ? ttiles : twgs);
      if (f->kind == QED_FIELD_GRID)
        hipLaunchKernelGGL(k_photon_table<QED_FIELD_GRID>, dim3(tgrid), dim3(kPTThreads), 0, st, a, c->cand_mask);
      else if (f->kind == QED_FIELD_UNIFORM)
        hipLaunchKernelGGL(k_photon_table<QED_FIELD_UNIFORM>, dim3(tgrid), dim3(kPTThreads), 0, st, a, c->cand_mask);
      else
        hipLaunchKernelGGL(k_photon_table<QED_FIELD_PER_PARTICLE>, dim3(tgrid), dim3(kPTThreads), 0, st, a,
                           c->cand_mask);
      const ScanDev isc{c->d_ticket + 1, c->d_status + c->status_len};
      if (wide)
        hipLaunchKernelGGL((k_emit_index<8, int32_t>), dim3(eig), dim3(kEIThreads), 0, st, c->cand_mask,
                           ph->count, c->cand_idx, c->d_n_cand, isc, c->d_counters);
      else
        hipLaunchKernelGGL((k_emit_index<1, int32_t>), dim3(eig), dim3(kEIThreads), 0, st, c->cand_mask,
                           ph->count, c->cand_idx, c->d_n_cand, isc, c->d_counters);
      const int64_t ewgs = (int64_t)c->n_cu * 4, eblocks = (ph->capacity + 255) / 256;
      hipLaunchKernelGGL(k_pair_events, dim3((unsigned)(eblocks < ewgs ? eblocks : ewgs)), dim3(256), 0, st, a,
                         c->cand_idx, c->d_n_cand);
      hipLaunchKernelGGL(k_pair_commit, dim3(1), dim3(1), 0, st, a, c->d_n_cand);
    }
  } else {
    PairArgs<double> a{dev_species(ph), dev_species(el), dev_species(po), dev_fields(f), c->pair_L64,
                       c->pair_S64, c->pair_q16, c->pair_s0sc, dt, dt, move, c->d_next_id,
                       c->params.seed, (uint64_t)step, step < 0 ? c->d_step : nullptr, sc, c->d_counters, killed, c->range,
                      retire_dev(c)};
    hipLaunchKernelGGL(k_pairs_f64, dim3(grid), dim3(kPairThreads), 0, st, a);
  }
  return hipGetLastError();
}

hipError_t launch_compact(qed_ctx *c, const qed_species_t *sp, hipStream_t st) {
  return launch_compact_scan(c, sp, c->d_ticket, c->d_status, c->status_len, st);
}

static_assert(kCTile == kCompactTile, "compaction tile size of the scan-state bound");

hipError_t launch_compact_scan(qed_ctx *c, const qed_species_t *sp, uint32_t *ticket, uint64_t *status,
                               int64_t status_len, hipStream_t st) {
  const int64_t ntiles = (sp->capacity + kCTile - 1) / kCTile;
  hipError_t e = zero_scan_at(ticket, status, status_len, ntiles, st);
  if (e != hipSuccess) return e;
  const ScanDev sc{ticket, status};
  const bool track = (c->params.flags & QED_FLAG_TRACK_DEAD) != 0;
  const bool owner = track && c->killed_owner == sp->x;
  int64_t *killed = owner ? c->d_killed : nullptr;
  // persistent workgroups take tiles from the ticket; with nothing killed they
  // all return at once
  const int64_t wgs = (int64_t)c->n_cu * 8;
  const unsigned grid = (unsigned)(ntiles < wgs ? ntiles : wgs);
  if (sp->dtype == QED_F32)
    hipLaunchKernelGGL(k_compact<float>, dim3(grid), dim3(kCThreads), 0, st, dev_species(sp), sc, c->d_counters,
                       killed);
  else
    hipLaunchKernelGGL(k_compact<double>, dim3(grid), dim3(kCThreads), 0, st, dev_species(sp), sc,
                       c->d_counters, killed);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  // the species now has no dead particles (the kernel clears the count of the
  // species it tracks already)
  if (!owner) hipLaunchKernelGGL(k_set_i64, dim3(1), dim3(1), 0, st, c->d_killed, (int64_t)0);
  c->killed_owner = sp->x;
  return hipGetLastError();
}

hipError_t launch_init_tau(qed_ctx *c, const qed_species_t *sp, int64_t step, hipStream_t st) {
  int64_t blocks = (sp->capacity + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  hipLaunchKernelGGL(k_init_tau, dim3((unsigned)blocks), dim3(256), 0, st, sp->id, sp->tau,
                     sp->count, c->params.seed, (uint64_t)step, step < 0 ? c->d_step : nullptr, sp->capacity);
  return hipGetLastError();
}

hipError_t launch_standing_wave(float *grid, int n, double L, double a0, double t0, double dt_step,
                                const int64_t *d_step, hipStream_t st) {
  const int64_t rows = (int64_t)n * n;
  const bool wide = n % 2 == 0 && ((uintptr_t)grid % 16) == 0;
  const int per_row = wide ? 6 * n / 4 : 3 * n;
  const int threads = per_row >= 256 ? 256 : (per_row + 63) / 64 * 64;
  const int64_t blocks = rows < 2048 ? rows : 2048;
  const size_t lds = (size_t)6 * n * sizeof(float);
  if (wide)
    hipLaunchKernelGGL(k_standing_wave<float4>, dim3((unsigned)blocks), dim3(threads), lds, st, grid, n, L / n, a0,
                       t0, dt_step, d_step);
  else
    hipLaunchKernelGGL(k_standing_wave<float2>, dim3((unsigned)blocks), dim3(threads), lds, st, grid, n, L / n, a0,
                       t0, dt_step, d_step);
  return hipGetLastError();
}

__global__ void k_add_i64(int64_t *p, int64_t v) { *p += v; }

hipError_t launch_set_step(qed_ctx *c, int64_t v, int add, hipStream_t st) {
  if (add) hipLaunchKernelGGL(k_add_i64, dim3(1), dim3(1), 0, st, c->d_step, v);
  else hipLaunchKernelGGL(k_set_i64, dim3(1), dim3(1), 0, st, c->d_step, v);
  return hipGetLastError();
}

template <typename R>
__global__ void k_tally_species(SpeciesDev sp, RetireDev r) {
  const int64_t n = *sp.count;
  const R *PX = (const R *)sp.px, *PY = (const R *)sp.py, *PZ = (const R *)sp.pz;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    if (sp.id[i] != kDeadId) {
      const double kx = PX[i], ky = PY[i], kz = PZ[i];
      tally_photon(r, sqrt(kx * kx + ky * ky + kz * kz));
    }
}

hipError_t launch_tally_species(qed_ctx *c, const qed_species_t *sp, hipStream_t st) {
  int64_t blocks = (sp->capacity + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  if (sp->dtype == QED_F32)
    hipLaunchKernelGGL(k_tally_species<float>, dim3((unsigned)blocks), dim3(256), 0, st, dev_species(sp), retire_dev(c));
  else
    hipLaunchKernelGGL(k_tally_species<double>, dim3((unsigned)blocks), dim3(256), 0, st, dev_species(sp), retire_dev(c));
  return hipGetLastError();
}

hipError_t launch_eval_chi(qed_ctx *c, const qed_fields_t *f, const qed_species_t *sp, int photon, double *out,
                           hipStream_t st) {
  int64_t blocks = (sp->capacity + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  if (sp->dtype == QED_F32)
    hipLaunchKernelGGL(k_eval_chi<float>, dim3((unsigned)blocks), dim3(256), 0, st, dev_species(sp), dev_fields(f),
                       photon, out);
  else
    hipLaunchKernelGGL(k_eval_chi<double>, dim3((unsigned)blocks), dim3(256), 0, st, dev_species(sp), dev_fields(f),
                       photon, out);
  (void)c;
  return hipGetLastError();
}

hipError_t launch_sample(qed_ctx *c, const double *chi, const double *gamma, const uint64_t *id,
                         int64_t n, int precision, int64_t step, float *lnw, float *xi, float *lnwp,
                         hipStream_t st) {
  int64_t blocks = (n + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  if (blocks < 1) blocks = 1;
  if (precision == QED_F64)
    hipLaunchKernelGGL(k_sample_f64, dim3((unsigned)blocks), dim3(256), 0, st, chi, gamma, id, n,
                       c->rad_lnh64, c->pair_L64, c->rad_S64, c->params.seed, (uint64_t)step,
                       step < 0 ? c->d_step : nullptr, lnw,
                       xi, lnwp, c->range);
  else
    hipLaunchKernelGGL(k_sample_f32, dim3((unsigned)blocks), dim3(256), 0, st, chi, gamma, id, n,
                       c->rad_lnh32, c->pair_L32, c->rad_q16, c->rad_s0sc, c->params.seed,
                       (uint64_t)step, step < 0 ? c->d_step : nullptr, lnw, xi, lnwp, c->range);
  return hipGetLastError();
}

}  // namespace qed
