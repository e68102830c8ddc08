// Surrogate networks of the QED step and their training, on gfx950 matrix cores.
//
//   net A  (log10 chi, logit u) -> r,  logit(xi) = r + ln chi + 3 ln u
//   net B  log10 chi -> (ln h_rad - ln chi, ln h_pair + 8/(3 chi) - ln chi)
//
// Three hidden layers of width 64 with SiLU.  The two 64x64 layers run on
// bf16 matrix cores (v_mfma_f32_16x16x16_bf16 for training,
// v_mfma_f32_16x16x32_bf16 for inference) with every
// operand split into bf16 hi + lo parts and
// the three products hi*hi + hi*lo + lo*hi accumulated in float32 (about 16
// significant bits; one bf16 product alone would leave ~3e-3 relative error,
// too coarse for the 1e-3 rate target).  Input and output layers (1-2 inputs,
// 1-2 outputs) are float32 vector code.
//
// A forward call evaluates a tile of 16 samples.  Lane l holds features
// mt*16 + 4*(l/16) + v (mt, v = 0..3) of sample l%16 both as the D result and as
// the B operand of the next layer, so activations stay in registers between
// layers; waves that own 64 samples make four calls.  Training (forward, backward, weight gradients, Adam) uses the same
// products; training data are drawn from the float64 master tables.
#include <hip/hip_runtime.h>
#include <math.h>

#include "internal.h"
#include "lookup.h"
#include "qed_device.h"
#include "mlp_device.h"

namespace qed {
namespace {
using namespace mlp;

// ------------------------------------------------------------- inputs/targets

// Training sample g of net A: chi at a table row, logit u uniform in
// [-Tmax, Tmax]; target from the float64 master inverse CDF of that row.
__device__ void sample_A(uint64_t g, uint32_t seed, const double *S64, float &x0, float &x1, float &yt) {
  const uint4 r = philox4x32_10(make_uint4((uint32_t)g, (uint32_t)(g >> 32), kTrainPurpose << 24, 0u),
                                make_uint2(seed, 0xA5A5A5A5u));
  const int row = (int)(r.x >> 24);                                     // 0..255
  const double t = -kTmax + 2.0 * kTmax * unit<double>(r.y);
  const double chi = exp(log(kRadChiMin) + row * ((log(kRadChiMax) - log(kRadChiMin)) / (kRadNChi - 1)));
  const double tlo = log(kRadULo) - log1p(-kRadULo), thi = log(kRadUHi) - log1p(-kRadUHi);
  const double dtn = (thi - tlo) / (kNU - 1);
  const double y = (t - tlo) / dtn;
  int j = (int)floor(y);
  j = j < 0 ? 0 : (j > kNU - 2 ? kNU - 2 : j);
  const double f = y - j;
  const double s = (1.0 - f) * S64[row * kNU + j] + f * S64[row * kNU + j + 1];
  const double lnu = -log1p(exp(-t));
  x0 = xin(chi);
  x1 = (float)(t / kTmax);
  yt = (float)((s - log(chi) - 3.0 * lnu - kAShift) / kAScale);
}

// Training sample g of net B: log10 chi uniform in [-3, 2]; targets from the
// float64 master rate tables (pair output masked below chi = 1e-2).
__device__ void sample_B(uint64_t g, uint32_t seed, const double *lnh, const double *L, const TabRange &rg,
                         float &x0, float yt[2], float m[2]) {
  const uint4 r = philox4x32_10(make_uint4((uint32_t)g, (uint32_t)(g >> 32), (kTrainPurpose << 24) | 1u, 0u),
                                make_uint2(seed, 0x5A5A5A5Au));
  const double lx = -3.0 + 5.0 * unit<double>(r.x);
  const double chi = pow(10.0, lx);
  x0 = xin(chi);
  yt[0] = (float)((log(h_rad<double>(chi, lnh, rg)) - log(chi) - kBShift0) / kBScale0);
  if (chi >= kPairChiMin) {
    const double x = (log(chi) - rg.pair_lnlo) * rg.pair_rate_inv;
    int i = (int)floor(x);
    i = i < 0 ? 0 : (i > kPairNRate - 2 ? kPairNRate - 2 : i);
    const double f = x - i;
    yt[1] = (float)(((1.0 - f) * L[i] + f * L[i + 1] - log(chi) - kBShift1) / kBScale1);
    m[1] = 1.f;
  } else {
    yt[1] = 0.f;
    m[1] = 0.f;
  }
  m[0] = 1.f;
}

// ------------------------------------------------------------------ training
struct TrainArgs {
  int net;                 // 0 = A, 1 = B
  const float *theta;
  float *grad;
  const double *S64, *lnh, *L;
  const float *ext_x, *ext_t, *ext_m;   // optional external batch (gradient checks)
  int64_t nbatch;
  uint64_t sample0;
  uint32_t seed;
  TabRange rg;             // the default table range (the nets' domain)
};

constexpr int kTrainThreads = 256;

struct TrainLds {
  NetLds s;
  NetLdsT t;
  float g[kA.n > kB.n ? kA.n : kB.n];
  float stage[4][2][H * 16];          // per wave: delta and activation [feature][sample]
};

// dW += delta a^T for one wave tile, split products, accumulated into LDS.
__device__ void weight_grad(const float *D, const float *A, float *gW) {
  const int lane = threadIdx.x & 63;
  for (int it = 0; it < 4; ++it) {
    const float *dr = D + (it * 16 + (lane & 15)) * 16 + 4 * (lane >> 4);
    s4 dh, dl;
    split4(dr, dh, dl);
    for (int kt = 0; kt < 4; ++kt) {
      const float *ar = A + (kt * 16 + (lane & 15)) * 16 + 4 * (lane >> 4);
      s4 ah, al;
      split4(ar, ah, al);
      f4 acc = {0.f, 0.f, 0.f, 0.f};
      acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(dh, ah, acc, 0, 0, 0);
      acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(dh, al, acc, 0, 0, 0);
      acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(dl, ah, acc, 0, 0, 0);
#pragma unroll
      for (int v = 0; v < 4; ++v)
        atomicAdd(&gW[(it * 16 + 4 * (lane >> 4) + v) * H + kt * 16 + (lane & 15)], acc[v]);
    }
  }
}

// Orders this wave's LDS writes before its later LDS reads (and vice versa).
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

__device__ void stage_tile(float *dst, const float val[4][4]) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int mt = 0; mt < 4; ++mt)
#pragma unroll
    for (int v = 0; v < 4; ++v) dst[feat(mt, v) * 16 + (lane & 15)] = val[mt][v];
}

__global__ __launch_bounds__(kTrainThreads) void k_train(TrainArgs a) {
  extern __shared__ __align__(16) unsigned char lds_raw[];
  TrainLds &S = *reinterpret_cast<TrainLds *>(lds_raw);
  const Layout L = a.net == 0 ? kA : kB;
  stage_net(a.theta, L, &S.s, &S.t);
  for (int k = threadIdx.x; k < L.n; k += blockDim.x) S.g[k] = 0.f;
  __syncthreads();
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, j = lane & 15;
  const int64_t ntile = (a.nbatch + 15) / 16;
  const float inv_n = 1.0f / (float)a.nbatch;
  for (int64_t tile = (int64_t)blockIdx.x * 4 + wave; tile < ntile; tile += (int64_t)gridDim.x * 4) {
    reload_barrier();
    const int64_t smp = tile * 16 + j;
    const bool valid = smp < a.nbatch;
    float x0 = 0.f, x1 = 0.f, yt[2] = {0.f, 0.f}, m[2] = {0.f, 0.f};
    if (valid) {
      if (a.ext_x) {
        x0 = a.ext_x[smp * L.nin];
        if (L.nin > 1) x1 = a.ext_x[smp * L.nin + 1];
        for (int o = 0; o < L.nout; ++o) { yt[o] = a.ext_t[smp * L.nout + o]; m[o] = a.ext_m ? a.ext_m[smp * L.nout + o] : 1.f; }
      } else if (a.net == 0) {
        sample_A(a.sample0 + smp, a.seed, a.S64, x0, x1, yt[0]);
        m[0] = 1.f;
      } else {
        sample_B(a.sample0 + smp, a.seed, a.lnh, a.L, a.rg, x0, yt, m);
      }
    }
    Cache c;
    float y[2];
    forward(S.s, L.nin, L.nout, x0, x1, y, c);
    float dy[2];
    for (int o = 0; o < L.nout; ++o) dy[o] = 2.f * (y[o] - yt[o]) * m[o] * inv_n;
    // output layer
    float d[4][4];
#pragma unroll
    for (int mt = 0; mt < 4; ++mt)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int f = feat(mt, v);
        float t = 0.f;
        for (int o = 0; o < L.nout; ++o) {
          t += S.s.W4[o * H + f] * dy[o];
          atomicAdd(&S.g[L.W4 + o * H + f], dy[o] * c.a3[mt][v]);
        }
        d[mt][v] = t * dsilu(c.z3[mt][v]);
        atomicAdd(&S.g[L.b3 + f], d[mt][v]);
      }
    if ((lane >> 4) == 0)
      for (int o = 0; o < L.nout; ++o) atomicAdd(&S.g[L.b4 + o], dy[o]);
    // layer 3 weights: d3 a2^T
    float a2[4][4];
#pragma unroll
    for (int mt = 0; mt < 4; ++mt)
#pragma unroll
      for (int v = 0; v < 4; ++v) a2[mt][v] = silu(c.z2[mt][v]);
    stage_tile(S.stage[wave][0], d);
    stage_tile(S.stage[wave][1], a2);
    wave_lds_sync();
    weight_grad(S.stage[wave][0], S.stage[wave][1], &S.g[L.W3]);
    wave_lds_sync();
    float d2[4][4];
    mm64(S.t.W3h, S.t.W3l, d, d2);
#pragma unroll
    for (int mt = 0; mt < 4; ++mt)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        d2[mt][v] *= dsilu(c.z2[mt][v]);
        atomicAdd(&S.g[L.b2 + feat(mt, v)], d2[mt][v]);
      }
    float a1[4][4];
#pragma unroll
    for (int mt = 0; mt < 4; ++mt)
#pragma unroll
      for (int v = 0; v < 4; ++v) a1[mt][v] = silu(c.z1[mt][v]);
    stage_tile(S.stage[wave][0], d2);
    stage_tile(S.stage[wave][1], a1);
    wave_lds_sync();
    weight_grad(S.stage[wave][0], S.stage[wave][1], &S.g[L.W2]);
    wave_lds_sync();
    float d1[4][4];
    mm64(S.t.W2h, S.t.W2l, d2, d1);
#pragma unroll
    for (int mt = 0; mt < 4; ++mt)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int f = feat(mt, v);
        const float dd = d1[mt][v] * dsilu(c.z1[mt][v]);
        atomicAdd(&S.g[L.b1 + f], dd);
        atomicAdd(&S.g[L.W1 + f * L.nin], dd * x0);
        if (L.nin > 1) atomicAdd(&S.g[L.W1 + f * L.nin + 1], dd * x1);
      }
  }
  __syncthreads();
  for (int k = threadIdx.x; k < L.n; k += blockDim.x) atomicAdd(&a.grad[k], S.g[k]);
}

__global__ void k_adam(float *theta, float *grad, float *m, float *v, int n, float lr, float b1t, float b2t) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float g = grad[i];
  const float mm = 0.9f * m[i] + 0.1f * g;
  const float vv = 0.999f * v[i] + 0.001f * g * g;
  m[i] = mm;
  v[i] = vv;
  theta[i] -= lr * (mm / (1.f - b1t)) / (sqrtf(vv / (1.f - b2t)) + 1e-8f);
  grad[i] = 0.f;
}

// PyTorch-style initial weights: U(-1/sqrt(fan_in), 1/sqrt(fan_in)).
__global__ void k_init(float *theta, int net, uint32_t seed) {
  const Layout L = net == 0 ? kA : kB;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= L.n) return;
  const int fan = (i < L.W2) ? L.nin : H;
  const uint4 r = philox4x32_10(make_uint4((uint32_t)i, (uint32_t)net, kInitPurpose << 24, 0u), make_uint2(seed, 0u));
  theta[i] = (float)((2.0 * unit<double>(r.x) - 1.0) / sqrt((double)fan));
}

// --------------------------------------------------------------- inference
struct InferArgs {
  const float *thA, *thB;
  const double *chi, *gamma;
  const uint64_t *id;
  int64_t n;
  uint32_t seed;
  uint64_t step;
  const int64_t *d_step;
  const float *lnh32, *L32, *s0sc, *chk;
  const uint16_t *q16;
  float *lnw, *xi, *lnwp;
  float tol;
  unsigned long long *fallback;     // [0] xi fallbacks, [1] rate fallbacks
  TabRange rg;                      // the default table range (the nets' domain)
};

struct InferLds {
  NetLdsI A, B;
  float chk[kRadNChi * (2 + 2 * kChkN)];
};

constexpr int kInferThreads = 512;

__global__ __launch_bounds__(kInferThreads) void k_infer(InferArgs a) {
  extern __shared__ __align__(16) unsigned char lds_raw[];
  InferLds &S = *reinterpret_cast<InferLds *>(lds_raw);
  stage_net_infer(a.thA, kA, &S.A);
  stage_net_infer(a.thB, kB, &S.B);
  for (int k = threadIdx.x; k < kRadNChi * (2 + 2 * kChkN); k += blockDim.x) S.chk[k] = a.chk[k];
  __syncthreads();
  const RowQ16 tab{a.q16, a.s0sc};
  const int lane = threadIdx.x & 63;
  const int64_t ntile = (a.n + 63) / 64;     // 64 samples per wave, one per lane
  const int wpb = blockDim.x >> 6;
  uint32_t nfx = 0, nfr = 0;
  for (int64_t tile = (int64_t)blockIdx.x * wpb + (threadIdx.x >> 6); tile < ntile;
       tile += (int64_t)gridDim.x * wpb) {
    reload_barrier();
    const int64_t i = tile * 64 + lane;
    const bool valid = i < a.n;
    const double chi = valid ? a.chi[i] : 1.0;
    const double gam = valid ? a.gamma[i] : 1.0;
    const uint64_t id = valid ? a.id[i] : 0;
    const uint4 r = stream4(id, a.seed, a.d_step ? (uint64_t)*a.d_step : a.step, kLeptonEvent, 0u);
    const float u = unit<float>(r.x), urow = unit<float>(r.z);
    const float t = logf(u) - log1pf(-u);
    const bool in_chi = chi >= kRadChiMin && chi <= kRadChiMax;
    const float x0 = xin(in_chi ? chi : 1.0), x1 = (float)(t / kTmax);
    // the wave's 64 samples go through each net as four 16-sample tiles; lane
    // q*16 + j keeps the outputs of sample j of tile q, its own
    float yB0 = 0.f, yB1 = 0.f, yA = 0.f;
#pragma unroll 1
    for (int q = 0; q < 4; ++q) {
      reload_barrier();
      float y[2];
      forward_inf(S.B, 1, 2, __shfl(x0, q * 16 + (lane & 15), 64), 0.f, y);    // rates (net B)
      if ((lane >> 4) == q) { yB0 = y[0]; yB1 = y[1]; }
    }
#pragma unroll 1
    for (int q = 0; q < 4; ++q) {
      reload_barrier();
      float y[2];
      forward_inf(S.A, 2, 1, __shfl(x0, q * 16 + (lane & 15), 64), __shfl(x1, q * 16 + (lane & 15), 64), y);
      if ((lane >> 4) == q) yA = y[0];                                          // xi (net A)
    }
    const float lchi = logf((float)chi);
    float lh = kBShift0 + kBScale0 * yB0 + lchi;
    const float env = logf(1.001f * (float)kHc1 * (float)chi);
    bool rate_ok = in_chi && isfinite(lh) && lh <= env;
    if (!rate_ok) lh = logf(h_rad<float>((float)chi, a.lnh32, a.rg));
    float lhp;
    if (chi < kPairChiMin || gam < 2.0) lhp = -INFINITY;
    else if (chi <= kPairChiMax && isfinite(yB1)) lhp = kBShift1 + kBScale1 * yB1 + lchi - 8.0f / (3.0f * (float)chi);
    else lhp = logf(h_pair<float>((float)chi, a.L32, a.rg));
    // xi with residual check against the Hermite CDF table
    const bool in_u = fabsf(t) <= (float)kTmax;
    float s_hat = kAShift + kAScale * yA + lchi + 3.0f * (-log1pf(__expf(-t)));
    bool xi_ok = in_chi && in_u && isfinite(s_hat);
    float xi, om;
    if (xi_ok) {
      const float x = (lchi - (float)a.rg.rad_lnlo) * (float)a.rg.rad_inv;
      int ii = (int)floorf(x);
      ii = ii < 0 ? 0 : (ii > kRadNChi - 2 ? kRadNChi - 2 : ii);
      const float w = x - ii;
      const float P = (1.f - w) * check_cdf(S.chk, ii, s_hat) + w * check_cdf(S.chk, ii + 1, s_hat);
      xi_ok = fabsf(P - u) <= a.tol;
    }
    if (xi_ok) {
      xi = 1.f / (1.f + __expf(-s_hat));
      om = 1.f / (1.f + __expf(s_hat));
    } else {
      sample_rad<float>(tab, (float)chi, u, urow, xi, om, a.rg);
    }
    if (valid) {
      a.lnw[i] = (float)((double)lh + log(kRateUnit / gam));
      a.xi[i] = xi;
      if (a.lnwp) a.lnwp[i] = isfinite(lhp) ? (float)((double)lhp + log(kRateUnit / gam)) : -INFINITY;
      nfx += !xi_ok;
      nfr += !rate_ok;
    }
  }
  // per-wave totals of fallbacks
  for (int o = 32; o > 0; o >>= 1) { nfx += __shfl_xor(nfx, o, 64); nfr += __shfl_xor(nfr, o, 64); }
  if (lane == 0) {
    if (nfx) atomicAdd(&a.fallback[0], (unsigned long long)nfx);
    if (nfr) atomicAdd(&a.fallback[1], (unsigned long long)nfr);
  }
}

// raw forward for tests: y = net(x) for n samples (normalised inputs/outputs)
__global__ __launch_bounds__(256) void k_forward_raw(const float *theta, int net, const float *x, int64_t n, float *y) {
  extern __shared__ __align__(16) unsigned char lds_raw[];
  NetLdsI &S = *reinterpret_cast<NetLdsI *>(lds_raw);
  const Layout L = net == 0 ? kA : kB;
  stage_net_infer(theta, L, &S);
  __syncthreads();
  const int lane = threadIdx.x & 63, j = lane & 15;
  const int64_t ntile = (n + 15) / 16;
  for (int64_t tile = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6); tile < ntile; tile += (int64_t)gridDim.x * 4) {
    reload_barrier();
    const int64_t i = tile * 16 + j;
    const bool valid = i < n;
    const float x0 = valid ? x[i * L.nin] : 0.f;
    const float x1 = (valid && L.nin > 1) ? x[i * L.nin + 1] : 0.f;
    float yy[2];
    forward_inf(S, L.nin, L.nout, x0, x1, yy);
    if (valid && (lane >> 4) == 0)
      for (int o = 0; o < L.nout; ++o) y[i * L.nout + o] = yy[o];
  }
}

}  // namespace

int mlp_params(int net) { return net == 0 ? kA.n : kB.n; }

hipError_t launch_mlp_init(float *theta, int net, uint32_t seed, hipStream_t st) {
  const int n = mlp_params(net);
  hipLaunchKernelGGL(k_init, dim3((n + 255) / 256), dim3(256), 0, st, theta, net, seed);
  return hipGetLastError();
}

hipError_t launch_mlp_grad(int net, const float *theta, float *grad, const double *S64, const double *lnh,
                           const double *L, const float *ext_x, const float *ext_t, const float *ext_m,
                           int64_t nbatch, uint64_t sample0, uint32_t seed, hipStream_t st) {
  TrainArgs a{net, theta, grad, S64, lnh, L, ext_x, ext_t, ext_m, nbatch, sample0, seed,
              make_range(kRadChiMax, kPairChiMax)};
  const int64_t tiles = (nbatch + 15) / 16;
  int64_t blocks = (tiles + 3) / 4;
  if (blocks > 256) blocks = 256;
  hipLaunchKernelGGL(k_train, dim3((unsigned)blocks), dim3(kTrainThreads), sizeof(TrainLds), st, a);
  return hipGetLastError();
}

// Dynamic LDS above the default limit, for the kernels of this file; called
// once per context, with the context's device current.
hipError_t mlp_set_attributes() {
  hipError_t e = hipFuncSetAttribute((const void *)k_train, hipFuncAttributeMaxDynamicSharedMemorySize,
                                     (int)sizeof(TrainLds));
  if (e == hipSuccess)
    e = hipFuncSetAttribute((const void *)k_forward_raw, hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)sizeof(NetLdsI));
  if (e == hipSuccess)
    e = hipFuncSetAttribute((const void *)k_infer, hipFuncAttributeMaxDynamicSharedMemorySize, (int)sizeof(InferLds));
  return e;
}

hipError_t launch_adam(float *theta, float *grad, float *m, float *v, int net, float lr, float b1t, float b2t,
                       hipStream_t st) {
  const int n = mlp_params(net);
  hipLaunchKernelGGL(k_adam, dim3((n + 255) / 256), dim3(256), 0, st, theta, grad, m, v, n, lr, b1t, b2t);
  return hipGetLastError();
}

hipError_t launch_mlp_forward(const float *theta, int net, const float *x, int64_t n, float *y, hipStream_t st) {
  int64_t blocks = ((n + 15) / 16 + 3) / 4;
  if (blocks > 4096) blocks = 4096;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(k_forward_raw, dim3((unsigned)blocks), dim3(256), sizeof(NetLdsI), st, theta, net, x, n, y);
  return hipGetLastError();
}

hipError_t launch_mlp_sample(qed_ctx *c, const double *chi, const double *gamma, const uint64_t *id, int64_t n,
                             int64_t step, float *lnw, float *xi, float *lnwp, float tol, hipStream_t st) {
  InferArgs a{c->mlp_theta[0], c->mlp_theta[1], chi, gamma, id, n, c->params.seed, (uint64_t)step,
              step < 0 ? c->d_step : nullptr,
              c->rad_lnh32, c->pair_L32, c->rad_s0sc, c->rad_chk, c->rad_q16, lnw, xi, lnwp, tol,
              c->d_counters + cMlpFallbackXi, make_range(kRadChiMax, kPairChiMax)};
  int64_t blocks = ((n + 63) / 64 + 7) / 8;
  if (blocks > c->n_cu) blocks = c->n_cu;      // one workgroup per CU (LDS-bound)
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(k_infer, dim3((unsigned)blocks), dim3(kInferThreads), sizeof(InferLds), st, a);
  return hipGetLastError();
}

size_t mlp_infer_lds() { return sizeof(InferLds); }
size_t mlp_train_lds() { return sizeof(TrainLds); }

}  // namespace qed
