// Inference and training kernels of the candidate-proposal network on
// gfx950 matrix cores (see mlp_core.h for the operand layout).
//
// Training minimises the mean squared error over a batch. The backward pass
// keeps the forward orientation: the output-layer signal g2 = W3^T g3 masked
// by the ReLU gate is already in B layout, so dL/dh1 = W2^T g2 is one more
// set of MFMAs with W2^T as the A operand. The weight gradients contract over
// the samples of a tile, which need the samples along k: the tile's g2, h1,
// g1 and inputs are transposed through LDS for those products. Every sum is
// taken in a fixed order (lanes, waves, workgroups), so a gradient is
// reproducible bit for bit.

#include <algorithm>

#include "chap_internal.h"
#include "mlp_core.h"

namespace chap {
namespace {

using namespace mlp;

constexpr int kWaves = 4;

// Loads the inputs of sample `row` in B layout (inputs 4g..4g+3), zero when
// the sample does not exist.
__device__ __forceinline__ bf16x4 load_inputs(const uint16_t* __restrict__ feat, int64_t row, bool valid) {
  const int g = (threadIdx.x & 63) >> 4;
  const bf16x4 zero = {0, 0, 0, 0};
  return valid ? *(const bf16x4*)(feat + row * kIn + 4 * g) : zero;
}

__global__ __launch_bounds__(256) void k_mlp_forward(const float* __restrict__ w, const uint16_t* __restrict__ wb,
                                                     const uint16_t* __restrict__ feat, int64_t n,
                                                     float* __restrict__ out) {
  Weights W;
  load_weights(wb, w, W);
  const int l = threadIdx.x & 63, r = l & 15;
  const int64_t ntiles = (n + 15) / 16;
  const int64_t stride = (int64_t)gridDim.x * kWaves;
  for (int64_t tile = (int64_t)blockIdx.x * kWaves + (threadIdx.x >> 6); tile < ntiles; tile += stride) {
    const int64_t row = tile * 16 + r;
    Acts A;
    forward(W, load_inputs(feat, row, row < n), A);
    if (l < 16 && row < n) out[row] = A.y;
  }
}

// Sum over the 16 lanes of a lane group (same g), fixed butterfly order.
__device__ __forceinline__ float group16_sum(float v) {
#pragma unroll
  for (int o = 1; o < 16; o <<= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Per-workgroup gradient partials of the mean squared error over `nb`
// samples. Sample i is row i of (feat, target), or row
// splitmix64(seed, base + i) mod rows when `sample` is set. inv_nb = 1/nb.
// Writes partials[blockIdx.x][p] for every parameter p.
__global__ __launch_bounds__(256) void k_mlp_grad(const float* __restrict__ w, const uint16_t* __restrict__ wb,
                                                  const uint16_t* __restrict__ feat,
                                                  const float* __restrict__ target, int64_t rows, int64_t nb,
                                                  int32_t sample, uint64_t seed, uint64_t base, float inv_nb,
                                                  float* __restrict__ partials, const int32_t* active) {
  if (active && !*active) return;
  __shared__ uint16_t sG2[kWaves][kHid * 16];
  __shared__ uint16_t sH1[kWaves][kHid * 16];
  __shared__ uint16_t sG1[kWaves][kHid * 16];
  __shared__ uint16_t sX[kWaves][kIn * 16];
  __shared__ float sred[kNParam];
  const int l = threadIdx.x & 63, g = l >> 4, r = l & 15;
  const int wv = threadIdx.x >> 6;
  Weights W;
  load_weights(wb, w, W);
  // W2^T in A layout: element (i = r, k = 4g + t) of block (ib, ob) is W2[16ob + 4g + t][16ib + r]
  bf16x4 a2t[4][4];
  float w3r[4][4];  // W3[16o + 4g + t] as FP32 (bfloat16 values)
#pragma unroll
  for (int ib = 0; ib < 4; ++ib)
#pragma unroll
    for (int ob = 0; ob < 4; ++ob)
#pragma unroll
      for (int t = 0; t < 4; ++t) a2t[ib][ob][t] = (short)wb[kOffW2 + (16 * ob + 4 * g + t) * kHid + 16 * ib + r];
#pragma unroll
  for (int o = 0; o < 4; ++o)
#pragma unroll
    for (int t = 0; t < 4; ++t) w3r[o][t] = bf2f(wb[kOffW3 + 16 * o + 4 * g + t]);

  const f32x4 zero4 = {0.0f, 0.0f, 0.0f, 0.0f};
  f32x4 accW2[4][4], accW1[4];
  float accW3[4][4], accB2[4][4], accB1[4][4], accB3 = 0.0f;
#pragma unroll
  for (int a = 0; a < 4; ++a) {
    accW1[a] = zero4;
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      accW2[a][b] = zero4;
      accW3[a][b] = 0.0f;
      accB2[a][b] = 0.0f;
      accB1[a][b] = 0.0f;
    }
  }

  const int64_t ntiles = (nb + 15) / 16;
  const int64_t stride = (int64_t)gridDim.x * kWaves;
  // every wave runs the same number of rounds (barriers below); tiles past
  // the end are all-zero samples with a zero output signal
  for (int64_t base_tile = (int64_t)blockIdx.x * kWaves; base_tile < ntiles; base_tile += stride) {
    const int64_t tile = base_tile + wv;
    const int64_t i = tile * 16 + r;
    const bool valid = i < nb;
    int64_t row = i;
    if (valid && sample) row = (int64_t)(splitmix64(seed, base + (uint64_t)i) % (uint64_t)rows);
    const bf16x4 x = load_inputs(feat, row, valid);
    Acts A;
    forward(W, x, A);
    // output signal g3 = 2 (y - t) / nb of sample r, broadcast to its column
    float g3 = 0.0f;
    if (l < 16 && valid) g3 = 2.0f * (A.y - target[row]) * inv_nb;
    g3 = __shfl(g3, r, 64);
    if (l < 16) accB3 += g3;
    // output layer and g2 = W3 g3 gated by z2 > 0
    bf16x4 g2b[4];
#pragma unroll
    for (int o = 0; o < 4; ++o) {
      float v[4];
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        accW3[o][t] += g3 * bf2f((uint16_t)A.h2[o][t]);
        v[t] = (A.z2[o][t] > 0.0f) ? g3 * w3r[o][t] : 0.0f;
        accB2[o][t] += v[t];
      }
      g2b[o] = to_bf16x4(v[0], v[1], v[2], v[3]);
    }
    // dL/dh1 = W2^T g2, gated by z1 > 0
    bf16x4 g1b[4];
#pragma unroll
    for (int ib = 0; ib < 4; ++ib) {
      f32x4 acc = zero4;
#pragma unroll
      for (int ob = 0; ob < 4; ++ob) acc = mma(a2t[ib][ob], g2b[ob], acc);
      float v[4];
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        v[t] = (A.z1[ib][t] > 0.0f) ? acc[t] : 0.0f;
        accB1[ib][t] += v[t];
      }
      g1b[ib] = to_bf16x4(v[0], v[1], v[2], v[3]);
    }
    // transpose the tile through LDS: unit-major rows of 16 samples
#pragma unroll
    for (int b = 0; b < 4; ++b)
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const int u = 16 * b + 4 * g + t;
        sG2[wv][u * 16 + r] = (uint16_t)g2b[b][t];
        sH1[wv][u * 16 + r] = (uint16_t)A.h1[b][t];
        sG1[wv][u * 16 + r] = (uint16_t)g1b[b][t];
      }
#pragma unroll
    for (int t = 0; t < 4; ++t) sX[wv][(4 * g + t) * 16 + r] = (uint16_t)x[t];
    __syncthreads();
    // dW2[o][i] += sum_s g2[o][s] h1[i][s];  dW1[h][f] += sum_s g1[h][s] x[f][s]
    bf16x4 h1t[4];
#pragma unroll
    for (int ib = 0; ib < 4; ++ib) h1t[ib] = *(const bf16x4*)&sH1[wv][(16 * ib + r) * 16 + 4 * g];
#pragma unroll
    for (int ob = 0; ob < 4; ++ob) {
      const bf16x4 g2t = *(const bf16x4*)&sG2[wv][(16 * ob + r) * 16 + 4 * g];
#pragma unroll
      for (int ib = 0; ib < 4; ++ib) accW2[ob][ib] = mma(g2t, h1t[ib], accW2[ob][ib]);
    }
    const bf16x4 xt = *(const bf16x4*)&sX[wv][r * 16 + 4 * g];
#pragma unroll
    for (int hb = 0; hb < 4; ++hb) {
      const bf16x4 g1t = *(const bf16x4*)&sG1[wv][(16 * hb + r) * 16 + 4 * g];
      accW1[hb] = mma(g1t, xt, accW1[hb]);
    }
    __syncthreads();
  }
  // lane-group sums of the per-lane accumulators
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      accW3[a][t] = group16_sum(accW3[a][t]);
      accB2[a][t] = group16_sum(accB2[a][t]);
      accB1[a][t] = group16_sum(accB1[a][t]);
    }
  accB3 = group16_sum(accB3);
  // workgroup sum in wave order
  for (int p = threadIdx.x; p < kNParam; p += blockDim.x) sred[p] = 0.0f;
  for (int w2 = 0; w2 < kWaves; ++w2) {
    __syncthreads();
    if (wv != w2) continue;
#pragma unroll
    for (int ob = 0; ob < 4; ++ob)
#pragma unroll
      for (int ib = 0; ib < 4; ++ib)
#pragma unroll
        for (int t = 0; t < 4; ++t) sred[kOffW2 + (16 * ob + 4 * g + t) * kHid + 16 * ib + r] += accW2[ob][ib][t];
#pragma unroll
    for (int hb = 0; hb < 4; ++hb)
#pragma unroll
      for (int t = 0; t < 4; ++t) sred[kOffW1 + (16 * hb + 4 * g + t) * kIn + r] += accW1[hb][t];
    if (r == 0) {
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int t = 0; t < 4; ++t) {
          sred[kOffW3 + 16 * a + 4 * g + t] += accW3[a][t];
          sred[kOffB2 + 16 * a + 4 * g + t] += accB2[a][t];
          sred[kOffB1 + 16 * a + 4 * g + t] += accB1[a][t];
        }
    }
    if (l == 0) sred[kOffB3] += accB3;
  }
  __syncthreads();
  float* mine = partials + (int64_t)blockIdx.x * kNParamPad;
  for (int p = threadIdx.x; p < kNParam; p += blockDim.x) mine[p] = sred[p];
}

// Advances Adam's step counter and the powers beta1^t, beta2^t (FP64).
__global__ void k_adam_begin(double* adam, double beta1, double beta2, const int32_t* active) {
  if (threadIdx.x != 0 || blockIdx.x != 0 || (active && !*active)) return;
  adam[0] *= beta1;
  adam[1] *= beta2;
  adam[2] += 1.0;
}

// Sums the partials in workgroup order into grad; with `update`, one Adam
// step on the FP32 parameters and a fresh bfloat16 copy. omb1 and omb2 are
// 1 - beta1 and 1 - beta2 rounded once from FP64.
__global__ __launch_bounds__(256) void k_mlp_reduce(float* __restrict__ w, uint16_t* __restrict__ wb,
                                                    float* __restrict__ m, float* __restrict__ v,
                                                    const double* __restrict__ adam, float* __restrict__ grad,
                                                    const float* __restrict__ partials, int32_t nparts,
                                                    int32_t update, float lr, float beta1, float omb1, float beta2,
                                                    float omb2, float eps, const int32_t* active) {
  if (active && !*active) return;
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= kNParam) return;
  float gsum = 0.0f;
  for (int b = 0; b < nparts; ++b) gsum += partials[(int64_t)b * kNParamPad + p];
  grad[p] = gsum;
  if (!update) return;
  const float mo = beta1 * m[p] + omb1 * gsum;
  const float vo = beta2 * v[p] + omb2 * gsum * gsum;
  m[p] = mo;
  v[p] = vo;
  const float c1 = (float)(1.0 - adam[0]);
  const float c2 = (float)(1.0 - adam[1]);
  const float mh = mo / c1;
  const float vh = vo / c2;
  const float nw = w[p] - lr * mh / (sqrtf(vh) + eps);
  w[p] = nw;
  wb[p] = f2bf(nw);
}

__global__ __launch_bounds__(256) void k_mlp_bf16_copy(const float* __restrict__ w, uint16_t* __restrict__ wb) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p < kNParam) wb[p] = f2bf(w[p]);
}

}  // namespace

hipError_t launch_mlp_forward(const ModelDev& M, const uint16_t* feat, int64_t n, float* out, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const int64_t tiles = (n + 15) / 16;
  const int64_t blocks = std::min<int64_t>((tiles + kWaves - 1) / kWaves, 4096);
  hipLaunchKernelGGL(k_mlp_forward, dim3((unsigned)blocks), dim3(256), 0, s, M.w, M.wb, feat, n, out);
  return hipGetLastError();
}

int32_t mlp_grad_blocks(int64_t nb) {
  const int64_t tiles = (nb + 15) / 16;
  return (int32_t)std::max<int64_t>(1, std::min<int64_t>((tiles + kWaves - 1) / kWaves, kGradBlocks));
}

hipError_t grad_impl(const ModelDev& M, const int32_t* active, const uint16_t* feat, const float* target,
                     int64_t rows, int64_t nb, int sample, uint64_t seed, uint64_t base, hipStream_t s) {
  const int32_t blocks = mlp_grad_blocks(nb);
  hipLaunchKernelGGL(k_mlp_grad, dim3((unsigned)blocks), dim3(256), 0, s, M.w, M.wb, feat, target, rows, nb,
                     (int32_t)sample, seed, base, (float)(1.0 / (double)nb), M.partials, active);
  return hipGetLastError();
}

hipError_t reduce_impl(const ModelDev& M, const int32_t* active, int64_t nb, int update, float lr, hipStream_t s) {
  if (update) hipLaunchKernelGGL(k_adam_begin, dim3(1), dim3(64), 0, s, M.adam, kAdamBeta1, kAdamBeta2, active);
  hipLaunchKernelGGL(k_mlp_reduce, dim3((kNParam + 255) / 256), dim3(256), 0, s, M.w, M.wb, M.m, M.v, M.adam, M.grad,
                     M.partials, mlp_grad_blocks(nb), (int32_t)update, lr, (float)kAdamBeta1,
                     (float)(1.0 - kAdamBeta1), (float)kAdamBeta2, (float)(1.0 - kAdamBeta2), kAdamEps, active);
  return hipGetLastError();
}

hipError_t launch_mlp_grad(const ModelDev& M, const uint16_t* feat, const float* target, int64_t rows, int64_t nb,
                           int sample, uint64_t seed, uint64_t base, hipStream_t s) {
  return grad_impl(M, nullptr, feat, target, rows, nb, sample, seed, base, s);
}

hipError_t launch_mlp_reduce(const ModelDev& M, int64_t nb, int update, float lr, hipStream_t s) {
  return reduce_impl(M, nullptr, nb, update, lr, s);
}

hipError_t launch_mlp_grad_guarded(const ModelDev& M, const int32_t* active, const uint16_t* feat,
                                   const float* target, int64_t nb, hipStream_t s) {
  return grad_impl(M, active, feat, target, nb, nb, 0, 0, 0, s);
}

hipError_t launch_mlp_reduce_guarded(const ModelDev& M, const int32_t* active, int64_t nb, float lr, hipStream_t s) {
  return reduce_impl(M, active, nb, 1, lr, s);
}

hipError_t launch_mlp_bf16_copy(const ModelDev& M, hipStream_t s) {
  hipLaunchKernelGGL(k_mlp_bf16_copy, dim3((kNParam + 255) / 256), dim3(256), 0, s, M.w, M.wb);
  return hipGetLastError();
}

}  // namespace chap
