// Device building blocks of the surrogate networks (shared by the training and
// sampling kernels in mlp.hip and the surrogate variants of the step kernels):
// split-BF16 64x64 layers on the K = 16 (training) and K = 32 (inference) bf16
// matrix instructions, the 16-sample forward passes, the input normalisation and
// the residual-check CDF rows.
#pragma once
#include <hip/hip_runtime.h>
#include <math.h>

#include "qed_device.h"

namespace qed {
namespace mlp {

typedef short s4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

constexpr int H = 64;
constexpr double kTmax = 9.2102403669758;   // logit(1 - 1e-4)
constexpr float kXShift = 0.5f, kXScale = 2.5f;
constexpr float kAShift = -1.0f, kAScale = 2.0f;
constexpr float kBShift0 = -0.4f, kBScale0 = 0.5f, kBShift1 = -2.0f, kBScale1 = 0.5f;
constexpr uint32_t kTrainPurpose = 3, kInitPurpose = 4;

struct Layout {
  int nin, nout, W1, b1, W2, b2, W3, b3, W4, b4, n;
};
__host__ __device__ constexpr Layout make_layout(int nin, int nout) {
  return Layout{nin, nout, 0, H * nin, H * nin + H, H * nin + H + H * H, H * nin + 2 * H + H * H,
                H * nin + 2 * H + 2 * H * H, H * nin + 3 * H + 2 * H * H,
                H * nin + 3 * H + 2 * H * H + nout * H, H * nin + 3 * H + 2 * H * H + nout * H + nout};
}
constexpr Layout kA = make_layout(2, 1), kB = make_layout(1, 2);

__device__ __forceinline__ uint16_t bf16_rne(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf16_f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }
// x = hi + lo with hi = bf16(x), lo = bf16(x - hi) (round to nearest even, the
// hardware conversion), packed four at a time
__device__ __forceinline__ void split4(const float x[4], s4 &hi, s4 &lo) {
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const __bf16 h = (__bf16)x[v];
    const __bf16 l = (__bf16)(x[v] - (float)h);
    hi[v] = __builtin_bit_cast(short, h);
    lo[v] = __builtin_bit_cast(short, l);
  }
}
__device__ __forceinline__ void split1(float x, uint16_t &hi, uint16_t &lo) {
  hi = bf16_rne(x);
  lo = bf16_rne(x - bf16_f(hi));
}
__device__ __forceinline__ float sigm(float z) { return __builtin_amdgcn_rcpf(1.0f + __expf(-z)); }
__device__ __forceinline__ float silu(float z) { return z * sigm(z); }
__device__ __forceinline__ float dsilu(float z) {
  const float s = sigm(z);
  return s * (1.0f + z * (1.0f - s));
}

// Weights of one net staged in LDS: split 64x64 layers, optionally their
// transposes, and the float32 small layers.  A 64x64 layer is stored in the
// order the matrix-core A operand is read: the 16x16 block (mt, ks) holds, for
// lane L, the four elements (row mt*16 + L%16, columns ks*16 + 4*(L/16) .. +3)
// at ((mt*4 + ks)*64 + L)*4, so that a wave reads 512 contiguous bytes per
// block (row-major rows of 128 B put 16 lanes on the same LDS banks).
__host__ __device__ constexpr int swz(int r, int c) {
  return (((r >> 4) * 4 + (c >> 4)) * 64 + (r & 15) + 16 * ((c & 15) >> 2)) * 4 + (c & 3);
}

struct NetLds {
  uint16_t W2h[H * H], W2l[H * H], W3h[H * H], W3l[H * H];
  float W1[H * 2], b1[H], b2[H], b3[H], W4[2 * H], b4[2];
};
struct NetLdsT {
  uint16_t W2h[H * H], W2l[H * H], W3h[H * H], W3l[H * H];   // transposed
};

__device__ void stage_net(const float *th, const Layout &L, NetLds *s, NetLdsT *t) {
  for (int k = threadIdx.x; k < H * H; k += blockDim.x) {
    const int r = k / H, c = k % H, sk = swz(r, c), tk = swz(c, r);
    uint16_t h, l;
    split1(th[L.W2 + k], h, l);
    s->W2h[sk] = h; s->W2l[sk] = l;
    if (t) { t->W2h[tk] = h; t->W2l[tk] = l; }
    split1(th[L.W3 + k], h, l);
    s->W3h[sk] = h; s->W3l[sk] = l;
    if (t) { t->W3h[tk] = h; t->W3l[tk] = l; }
  }
  for (int k = threadIdx.x; k < H; k += blockDim.x) {
    s->b1[k] = th[L.b1 + k]; s->b2[k] = th[L.b2 + k]; s->b3[k] = th[L.b3 + k];
    for (int c = 0; c < L.nin; ++c) s->W1[k * L.nin + c] = th[L.W1 + k * L.nin + c];
    for (int o = 0; o < L.nout; ++o) s->W4[o * H + k] = th[L.W4 + o * H + k];
  }
  if (threadIdx.x < L.nout) s->b4[threadIdx.x] = th[L.b4 + threadIdx.x];
}

// out = W a (64x64 layer, split products); a and out in the lane layout.
__device__ __forceinline__ void mm64(const uint16_t *Wh, const uint16_t *Wl, const float a[4][4],
                                     float out[4][4]) {
  const int lane = threadIdx.x & 63;
  s4 bh[4], bl[4];
#pragma unroll
  for (int ks = 0; ks < 4; ++ks) split4(a[ks], bh[ks], bl[ks]);
#pragma unroll
  for (int mt = 0; mt < 4; ++mt) {
    f4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int ks = 0; ks < 4; ++ks) {
      const int off = ((mt * 4 + ks) * 64 + lane) * 4;   // = swz(mt*16 + lane%16, ks*16 + 4*(lane/16))
      const s4 ah = *reinterpret_cast<const s4 *>(Wh + off);
      const s4 al = *reinterpret_cast<const s4 *>(Wl + off);
      acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ah, bh[ks], acc, 0, 0, 0);
      acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ah, bl[ks], acc, 0, 0, 0);
      acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(al, bh[ks], acc, 0, 0, 0);
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) out[mt][v] = acc[v];
  }
}

// Keeps LDS-resident weights from being hoisted into registers across tiles
// (the loop-invariant loads of two nets would exceed the register file).
__device__ __forceinline__ void reload_barrier() { asm volatile("" ::: "memory"); }

__device__ __forceinline__ int feat(int mt, int v) { return mt * 16 + 4 * ((threadIdx.x & 63) >> 4) + v; }

struct Cache {
  float z1[4][4], z2[4][4], z3[4][4], a3[4][4];
};

// Forward pass of one 16-sample tile; x0, x1 are the inputs of this lane's sample.
__device__ __forceinline__ void forward(const NetLds &s, int nin, int nout, float x0, float x1,
                                        float y[2], Cache &c) {
  float a[4][4], z[4][4];
#pragma unroll
  for (int mt = 0; mt < 4; ++mt)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int f = feat(mt, v);
      float t = s.b1[f] + s.W1[f * nin] * x0;
      if (nin > 1) t += s.W1[f * nin + 1] * x1;
      c.z1[mt][v] = t;
      a[mt][v] = silu(t);
    }
  mm64(s.W2h, s.W2l, a, z);
#pragma unroll
  for (int mt = 0; mt < 4; ++mt)
#pragma unroll
    for (int v = 0; v < 4; ++v) { z[mt][v] += s.b2[feat(mt, v)]; c.z2[mt][v] = z[mt][v]; a[mt][v] = silu(z[mt][v]); }
  mm64(s.W3h, s.W3l, a, z);
#pragma unroll
  for (int mt = 0; mt < 4; ++mt)
#pragma unroll
    for (int v = 0; v < 4; ++v) { z[mt][v] += s.b3[feat(mt, v)]; c.z3[mt][v] = z[mt][v]; c.a3[mt][v] = silu(z[mt][v]); }
  for (int o = 0; o < nout; ++o) {
    float p = 0.f;
#pragma unroll
    for (int mt = 0; mt < 4; ++mt)
#pragma unroll
      for (int v = 0; v < 4; ++v) p += s.W4[o * H + feat(mt, v)] * c.a3[mt][v];
    p += __shfl_xor(p, 16, 64);
    p += __shfl_xor(p, 32, 64);
    y[o] = p + s.b4[o];
  }
}

// ------------------------------------------------------------- inference
// Every inference kernel uses forward_inf: it evaluates the same function as
// `forward` (the same split products of the same activations) with fewer
// instructions: the biases are the initial accumulators of the matrix products,
// the small layers are read 16 bytes at a time, and the 64x64 products use the
// K = 32 matrix-core instruction (half the instructions of K = 16).  Measured on
// the lepton pass of the surrogate step: 1.21 -> 1.03 ms for 1e7 electrons.
typedef __bf16 b8 __attribute__((ext_vector_type(8)));

// K = 32 layout of a 64x64 layer.  The order of k inside a 32-wide block is
// chosen so that the B operand of a lane is made of the activations the lane
// already holds (units feat(2 ks, 0..3) and feat(2 ks + 1, 0..3)): block
// (mt, ks), lane L = 16 g + i, slot s holds row mt*16 + i and column
// 32 ks + 16 (s / 4) + 4 g + s % 4, at ((mt*2 + ks)*64 + L)*8 + s, so that a
// wave reads 1 KB of contiguous LDS per block.  The A and B operands of the
// instruction index k the same way, so any such order gives the same product.
__host__ __device__ constexpr int swz32(int r, int c) {
  return (((r >> 4) * 2 + (c >> 5)) * 64 + ((c & 15) >> 2) * 16 + (r & 15)) * 8 + ((c >> 4) & 1) * 4 + (c & 3);
}

// Inference copy of one net in LDS (distinct type: the 64x64 layers are in
// the swz32 order, not the swz order of NetLds).
struct alignas(16) NetLdsI {
  uint16_t W2h[H * H], W2l[H * H], W3h[H * H], W3l[H * H];
  float W1[H * 2], b1[H], b2[H], b3[H], W4[2 * H], b4[2];
};

__device__ void stage_net_infer(const float *th, const Layout &L, NetLdsI *s) {
  for (int k = threadIdx.x; k < H * H; k += blockDim.x) {
    const int sk = swz32(k / H, k % H);
    uint16_t h, l;
    split1(th[L.W2 + k], h, l);
    s->W2h[sk] = h; s->W2l[sk] = l;
    split1(th[L.W3 + k], h, l);
    s->W3h[sk] = h; s->W3l[sk] = l;
  }
  for (int k = threadIdx.x; k < H; k += blockDim.x) {
    s->b1[k] = th[L.b1 + k]; s->b2[k] = th[L.b2 + k]; s->b3[k] = th[L.b3 + k];
    for (int c = 0; c < L.nin; ++c) s->W1[k * L.nin + c] = th[L.W1 + k * L.nin + c];
    for (int o = 0; o < L.nout; ++o) s->W4[o * H + k] = th[L.W4 + o * H + k];
  }
  if (threadIdx.x < L.nout) s->b4[threadIdx.x] = th[L.b4 + threadIdx.x];
}

// acc += W a for a 64x64 layer in the swz32 layout, split products
// (hi*hi + hi*lo + lo*hi); a and acc in the lane layout.
// Lean: the weights of each 16-row block are read only when that block is
// multiplied (a compiler barrier per block), which keeps the register footprint
// small where the net is evaluated rarely (candidate events).
template <bool Lean = false>
__device__ __forceinline__ void mm64k32(const uint16_t *Wh, const uint16_t *Wl, const float a[4][4],
                                        float acc[4][4]) {
  const int lane = threadIdx.x & 63;
  b8 bh[2], bl[2];
#pragma unroll
  for (int ks = 0; ks < 2; ++ks)
#pragma unroll
    for (int s = 0; s < 8; ++s) {
      const float x = a[2 * ks + (s >> 2)][s & 3];
      const __bf16 h = (__bf16)x;
      bh[ks][s] = h;
      bl[ks][s] = (__bf16)(x - (float)h);
    }
#pragma unroll
  for (int mt = 0; mt < 4; ++mt) {
    if constexpr (Lean) reload_barrier();
    f4 c = {acc[mt][0], acc[mt][1], acc[mt][2], acc[mt][3]};
#pragma unroll
    for (int ks = 0; ks < 2; ++ks) {
      const int off = ((mt * 2 + ks) * 64 + lane) * 8;
      const b8 ah = *reinterpret_cast<const b8 *>(Wh + off);
      const b8 al = *reinterpret_cast<const b8 *>(Wl + off);
      c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bh[ks], c, 0, 0, 0);
      c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bl[ks], c, 0, 0, 0);
      c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, bh[ks], c, 0, 0, 0);
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) acc[mt][v] = c[v];
  }
}

// Four consecutive floats of a staged vector from feature feat(mt, 0) on: one
// 16-byte LDS read at a uniform base plus the lane's offset.
__device__ __forceinline__ float4 feat4(const float *v, int mt) {
  return *reinterpret_cast<const float4 *>(v + feat(mt, 0));
}

// Forward pass of one 16-sample tile for inference (no training cache).
template <bool Lean = false>
__device__ __forceinline__ void forward_inf(const NetLdsI &s, int nin, int nout, float x0, float x1, float y[2]) {
  float a[4][4], z[4][4];
#pragma unroll
  for (int mt = 0; mt < 4; ++mt) {
    const float4 b1 = feat4(s.b1, mt), b2 = feat4(s.b2, mt);
    float t[4] = {b1.x, b1.y, b1.z, b1.w};
    if (nin == 1) {
      const float4 w = feat4(s.W1, mt);
      t[0] += w.x * x0; t[1] += w.y * x0; t[2] += w.z * x0; t[3] += w.w * x0;
    } else {
      const float4 w0 = *reinterpret_cast<const float4 *>(s.W1 + 2 * feat(mt, 0));
      const float4 w1 = *reinterpret_cast<const float4 *>(s.W1 + 2 * feat(mt, 0) + 4);
      t[0] += w0.x * x0 + w0.y * x1; t[1] += w0.z * x0 + w0.w * x1;
      t[2] += w1.x * x0 + w1.y * x1; t[3] += w1.z * x0 + w1.w * x1;
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) a[mt][v] = silu(t[v]);
    z[mt][0] = b2.x; z[mt][1] = b2.y; z[mt][2] = b2.z; z[mt][3] = b2.w;
  }
  mm64k32<Lean>(s.W2h, s.W2l, a, z);
#pragma unroll
  for (int mt = 0; mt < 4; ++mt) {
    const float4 b3 = feat4(s.b3, mt);
#pragma unroll
    for (int v = 0; v < 4; ++v) a[mt][v] = silu(z[mt][v]);
    z[mt][0] = b3.x; z[mt][1] = b3.y; z[mt][2] = b3.z; z[mt][3] = b3.w;
  }
  mm64k32<Lean>(s.W3h, s.W3l, a, z);
  float p[2] = {0.f, 0.f};
#pragma unroll
  for (int mt = 0; mt < 4; ++mt) {
#pragma unroll
    for (int v = 0; v < 4; ++v) a[mt][v] = silu(z[mt][v]);
    for (int o = 0; o < nout; ++o) {
      const float4 w = feat4(s.W4 + o * H, mt);
      p[o] += w.x * a[mt][0] + w.y * a[mt][1] + w.z * a[mt][2] + w.w * a[mt][3];
    }
  }
  for (int o = 0; o < nout; ++o) {
    float q = p[o];
    q += __shfl_xor(q, 16, 64);
    q += __shfl_xor(q, 32, 64);
    y[o] = q + s.b4[o];
  }
}

__device__ __forceinline__ float xin(double chi) { return (float)((log10(chi) + kXShift) / kXScale); }

// ------------------------------------------------------------ residual check
// Photon CDF of the table row r on 40 nodes uniform in s over the row's fine
// grid bounds, with slopes: P(s) by cubic Hermite, linear mixing between rows.
constexpr int kChkN = 40;
__device__ float check_cdf(const float *chk, int r, float s) {
  const float *row = chk + r * (2 + 2 * kChkN);
  const float s0 = row[0], ds = row[1];
  const float y = (s - s0) / ds;
  if (y <= 0.f) return row[2] * __expf((s - s0) * (1.0f / 3.0f));
  if (y >= (float)(kChkN - 1)) return 1.0f;
  const int j = (int)y;
  const float t = y - j, t2 = t * t, t3 = t2 * t;
  const float p0 = row[2 + 2 * j], d0 = row[3 + 2 * j], p1 = row[4 + 2 * j], d1 = row[5 + 2 * j];
  return (2 * t3 - 3 * t2 + 1) * p0 + (t3 - 2 * t2 + t) * ds * d0 + (-2 * t3 + 3 * t2) * p1 + (t3 - t2) * ds * d1;
}


}  // namespace mlp
}  // namespace qed
