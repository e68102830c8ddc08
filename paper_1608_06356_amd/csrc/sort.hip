// Stable reordering of a species by grid cell (nearest node of the quadratic
// stencil, cells grouped in 4x4x4 blocks), so that the field gather of
// neighbouring threads touches neighbouring nodes.  Keys are radix-sorted with rocPRIM (stable), then every
// array is gathered into the destination species, one array per launch.  Particle ids, and therefore
// every random stream, travel with the particles, so the physics is unchanged;
// only the storage order (and with it the append order) changes.
#include <hip/hip_runtime.h>
#include <algorithm>
#include <rocprim/device/device_radix_sort.hpp>

#include "internal.h"
#include "qed_device.h"

namespace qed {
namespace {

// Cells are grouped in cubes of kBlk^3: the particles of one gather/push
// workgroup then fill a compact 3-D region, whose stencil box the workgroup
// stages in LDS.
constexpr int kBlk = 4;

// Bits of v (below 2^10) spread to every third position (bit k to bit 3k).
__device__ __forceinline__ uint32_t spread3(uint32_t v) {
  v &= 0x3FFu;
  v = (v | (v << 16)) & 0x030000FFu;
  v = (v | (v << 8)) & 0x0300F00Fu;
  v = (v | (v << 4)) & 0x030C30C3u;
  v = (v | (v << 2)) & 0x09249249u;
  return v;
}

// Key of a particle: block of kBlk^3 cells, then the cell inside the block
// (z-major).  Blocks follow the Morton (Z-order) curve of their coordinates
// when morton != 0 (x in the lowest bit of each triple), so that neighbouring
// blocks lie close in the sorted order in every direction; otherwise z-major.
template <typename R>
__global__ void k_cell_keys(const R *x, const R *y, const R *z, const int64_t *count, int64_t cap, int nx,
                            int ny, int nz, double dx, double dy, double dz, int morton, uint32_t *keys,
                            uint32_t *vals) {
  const int64_t n = *count;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < cap; i += (int64_t)gridDim.x * blockDim.x) {
    uint32_t key = 0xFFFFFFFFu;
    if (i < n) {
      int jx = (int)floor((double)x[i] / dx + 0.5), jy = (int)floor((double)y[i] / dy + 0.5),
          jz = (int)floor((double)z[i] / dz + 0.5);
      jx = jx < 0 ? 0 : (jx >= nx ? jx - nx : jx);
      jy = jy < 0 ? 0 : (jy >= ny ? jy - ny : jy);
      jz = jz < 0 ? 0 : (jz >= nz ? jz - nz : jz);
      jx = jx >= nx ? nx - 1 : jx; jy = jy >= ny ? ny - 1 : jy; jz = jz >= nz ? nz - 1 : jz;
      const int nbx = (nx + kBlk - 1) / kBlk, nby = (ny + kBlk - 1) / kBlk;
      const uint32_t bx = (uint32_t)(jx / kBlk), by = (uint32_t)(jy / kBlk), bz = (uint32_t)(jz / kBlk);
      const uint32_t blk = morton ? spread3(bx) | (spread3(by) << 1) | (spread3(bz) << 2)
                                  : (bz * (uint32_t)nby + by) * (uint32_t)nbx + bx;
      key = blk * (uint32_t)(kBlk * kBlk * kBlk) + (uint32_t)(((jz % kBlk) * kBlk + jy % kBlk) * kBlk + jx % kBlk);
    }
    keys[i] = key;
    vals[i] = (uint32_t)i;
  }
}

// One array at a time, so that its source lines alone compete for the L2
// (the gathers follow a permutation that is nearly the identity once the
// particles have been sorted before), four consecutive destinations per
// thread.  The grid covers the array; block b takes chunk (b % 8) *
// (gridDim.x / 8) + b / 8, so that each XCD (blocks are dealt round-robin over
// the 8) sweeps its own eighth of the sorted order and its L2 keeps that
// stretch's source lines.
template <typename T>
__global__ void k_permute4(const T *src, T *dst, const uint32_t *perm, const int64_t *count) {
  const int64_t n = *count;
  const int64_t lb = (int64_t)(blockIdx.x % 8u) * (gridDim.x / 8u) + blockIdx.x / 8u;
  const int64_t j = 4 * (lb * blockDim.x + threadIdx.x);
  if (j + 4 <= n) {
    const uint32_t i0 = perm[j], i1 = perm[j + 1], i2 = perm[j + 2], i3 = perm[j + 3];
    const T a = src[i0], b = src[i1], c = src[i2], d = src[i3];
    dst[j] = a; dst[j + 1] = b; dst[j + 2] = c; dst[j + 3] = d;
  } else {
    for (int64_t k = j; k < n; ++k) dst[k] = src[perm[k]];
  }
}

__global__ void k_set_count(const int64_t *src, int64_t *dst) { *dst = *src; }

// Onesweep radix sort with 11-bit digits: the keys (at most 22 bits) take two
// passes instead of three.
using SortCfg = rocprim::radix_sort_config<
    rocprim::default_config, rocprim::default_config,
    rocprim::radix_sort_onesweep_config<rocprim::kernel_config<1024, 16>, rocprim::kernel_config<1024, 16>, 11,
                                        rocprim::block_radix_rank_algorithm::match>>;

// Sorts the n particles the species holds (n read from the device by the caller).
template <typename R>
hipError_t sort_impl(qed_ctx *c, const qed_fields_t *f, const qed_species_t *s, qed_species_t *d, int64_t n,
                     hipStream_t st) {
  const int64_t cap = n > 0 ? n : 1;
  int64_t blocks = (cap + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  uint32_t *k0 = c->sort_keys, *k1 = c->sort_keys + cap, *v0 = c->sort_vals, *v1 = c->sort_vals + cap;
  // Morton order of the blocks when its codes (3 bits per bit of the largest
  // block coordinate) and the 6 cell bits fit the 32-bit key
  const int nbmax = std::max((f->nx + kBlk - 1) / kBlk, std::max((f->ny + kBlk - 1) / kBlk, (f->nz + kBlk - 1) / kBlk));
  unsigned mb = 0;
  while ((1 << mb) < nbmax) ++mb;
  const int morton = 3 * mb + 6 <= 31 ? 1 : 0;
  hipLaunchKernelGGL(k_cell_keys<R>, dim3((unsigned)blocks), dim3(256), 0, st, (const R *)s->x, (const R *)s->y,
                     (const R *)s->z, s->count, cap, f->nx, f->ny, f->nz, f->dx, f->dy, f->dz, morton, k0, v0);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const uint64_t cells = (uint64_t)((f->nx + kBlk - 1) / kBlk) * ((f->ny + kBlk - 1) / kBlk) *
                        ((f->nz + kBlk - 1) / kBlk) * (kBlk * kBlk * kBlk);
  unsigned bits = 1;
  if (morton) {
    bits = 3 * mb + 6;                          // keys below 2^bits
  } else {
    while ((1ull << bits) <= cells) ++bits;
  }
  ++bits;   // the all-ones sentinel of unused slots sorts last
  if (bits > 32) bits = 32;
  size_t need = 0;
  // scratch sized for the capacity, so that it is allocated once per species size
  if ((e = rocprim::radix_sort_pairs<SortCfg>(nullptr, need, k0, k1, v0, v1, (size_t)s->capacity, 0u, bits, st)) != hipSuccess)
    return e;
  if (need > c->sort_tmp_bytes) {
    if ((e = hipStreamSynchronize(st)) != hipSuccess) return e;
    (void)hipFree(c->sort_tmp);
    c->sort_tmp = nullptr;
    c->sort_tmp_bytes = 0;
    if ((e = hipMalloc(&c->sort_tmp, need)) != hipSuccess) return e;
    c->sort_tmp_bytes = need;
  }
  size_t need_n = 0;
  if ((e = rocprim::radix_sort_pairs<SortCfg>(nullptr, need_n, k0, k1, v0, v1, (size_t)cap, 0u, bits, st)) != hipSuccess)
    return e;
  if ((e = rocprim::radix_sort_pairs<SortCfg>(c->sort_tmp, need_n, k0, k1, v0, v1, (size_t)cap, 0u, bits, st)) != hipSuccess)
    return e;
  const int64_t qblocks = ((cap + 1023) / 1024 + 7) / 8 * 8;   // 256 threads x 4 destinations, 8 | blocks
  const void *sa[6] = {s->x, s->y, s->z, s->px, s->py, s->pz};
  void *da[6] = {d->x, d->y, d->z, d->px, d->py, d->pz};
  for (int k = 0; k < 6; ++k)
    hipLaunchKernelGGL(k_permute4<R>, dim3((unsigned)qblocks), dim3(256), 0, st, (const R *)sa[k], (R *)da[k], v1,
                       s->count);
  hipLaunchKernelGGL(k_permute4<double>, dim3((unsigned)qblocks), dim3(256), 0, st, s->tau, d->tau, v1, s->count);
  hipLaunchKernelGGL(k_permute4<uint64_t>, dim3((unsigned)qblocks), dim3(256), 0, st, s->id, d->id, v1, s->count);
  hipLaunchKernelGGL(k_set_count, dim3(1), dim3(1), 0, st, s->count, d->count);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_sort_by_cell(qed_ctx *c, const qed_fields_t *f, const qed_species_t *s, qed_species_t *d,
                               hipStream_t st) {
  if (s->capacity > c->sort_cap) {
    hipError_t e = hipStreamSynchronize(st);
    if (e != hipSuccess) return e;
    (void)hipFree(c->sort_keys);
    (void)hipFree(c->sort_vals);
    c->sort_keys = c->sort_vals = nullptr;
    c->sort_cap = 0;
    if ((e = hipMalloc(&c->sort_keys, 2 * s->capacity * sizeof(uint32_t))) != hipSuccess) return e;
    if ((e = hipMalloc(&c->sort_vals, 2 * s->capacity * sizeof(uint32_t))) != hipSuccess) return e;
    c->sort_cap = s->capacity;
  }
  // sort only the particles present: the count is read from the device (this
  // synchronises the stream; the sort is not for graph capture anyway)
  int64_t n = 0;
  hipError_t e = hipMemcpyAsync(&n, s->count, sizeof(n), hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) return e;
  if (n > s->capacity) n = s->capacity;
  return s->dtype == QED_F32 ? sort_impl<float>(c, f, s, d, n, st) : sort_impl<double>(c, f, s, d, n, st);
}

}  // namespace qed
