// Device core of the candidate-proposal network (16 inputs, two hidden
// layers of 64 ReLU units, one output) on gfx950 matrix cores.
//
// Every product runs on the matrix cores with bfloat16 operands and FP32
// accumulation. One wavefront handles a tile of 16 samples in the
// "feature-major" orientation: the weights are the A operand (16 output
// units x K inputs per instruction) and the activations the B operand
// (K inputs x 16 samples). v_mfma_f32_16x16x16_bf16, operand layout for
// lane l, g = l / 16, r = l % 16, t = 0..3:
//   A[i][k]: i = r, k = 4g + t        B[k][j]: j = r, k = 4g + t
//   D[i][j]: j = r, i = 4g + t
// The D layout of one layer equals the B layout of the next, so hidden
// activations pass between layers in registers: bias, ReLU and the rounding
// to bfloat16 (the native packed conversion, round to nearest even) are
// applied in place. The first layer (16 inputs) uses that instruction; the
// 64-input layers use v_mfma_f32_16x16x32_bf16, whose lanes bring 8 values
// of K each for A and for B under the same lane-and-element to k mapping:
// each lane passes two of its 4-unit pieces side by side (hidden units
// 32s + 4g + t and 32s + 16 + 4g + t for half s), and the weights in the
// same arrangement, so every instruction sums the 32 products of one half of
// the hidden layer (the order of those sums is the hardware's; the error
// bound of the reference allows any FP32 order).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace chap {
namespace mlp {

constexpr int kIn = 16;
constexpr int kHid = 64;
constexpr int kOffW1 = 0;      // W1[64][16], row = output unit
constexpr int kOffB1 = 1024;   // b1[64]
constexpr int kOffW2 = 1088;   // W2[64][64]
constexpr int kOffB2 = 5184;   // b2[64]
constexpr int kOffW3 = 5248;   // W3[64]
constexpr int kOffB3 = 5312;   // b3
constexpr int kNParam = 5313;

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// FP32 -> bfloat16, round to nearest, ties to even (finite inputs).
__device__ __forceinline__ uint16_t f2bf(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

__device__ __forceinline__ f32x4 mma(bf16x4 a, bf16x4 b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
}

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef short s16x8 __attribute__((ext_vector_type(8)));

// Two 4-value pieces as the 8 K values of one lane.
__device__ __forceinline__ bf16x8 pair(bf16x4 lo, bf16x4 hi) {
  const s16x8 v = __builtin_shufflevector(lo, hi, 0, 1, 2, 3, 4, 5, 6, 7);
  return __builtin_bit_cast(bf16x8, v);
}

__device__ __forceinline__ f32x4 mma32(bf16x8 a, bf16x8 b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

// Parameters of one wavefront in operand layout.
struct Weights {
  bf16x4 a1[4];     // W1[16h + r][4g + t]
  bf16x4 a2[4][4];  // W2[16o + r][16k + 4g + t]
  bf16x4 a3[4];     // output row: W3[16k + 4g + t] on lanes with r == 0, zero elsewhere
  f32x4 b1[4];      // b1[16h + 4g + t]
  f32x4 b2[4];
  float b3;
};

// wb: bfloat16 copy of the parameters, w: FP32 parameters (biases).
__device__ __forceinline__ void load_weights(const uint16_t* __restrict__ wb, const float* __restrict__ w,
                                             Weights& W) {
  const int l = threadIdx.x & 63, g = l >> 4, r = l & 15;
#pragma unroll
  for (int h = 0; h < 4; ++h) {
    W.a1[h] = *(const bf16x4*)(wb + kOffW1 + (16 * h + r) * kIn + 4 * g);
    W.b1[h] = *(const f32x4*)(w + kOffB1 + 16 * h + 4 * g);
    W.b2[h] = *(const f32x4*)(w + kOffB2 + 16 * h + 4 * g);
#pragma unroll
    for (int k = 0; k < 4; ++k) W.a2[h][k] = *(const bf16x4*)(wb + kOffW2 + (16 * h + r) * kHid + 16 * k + 4 * g);
    const bf16x4 w3 = *(const bf16x4*)(wb + kOffW3 + 16 * h + 4 * g);
    const bf16x4 zero = {0, 0, 0, 0};
    W.a3[h] = (r == 0) ? w3 : zero;
  }
  W.b3 = w[kOffB3];
}

// Activations of one tile, kept for the backward pass.
struct Acts {
  f32x4 z1[4];   // pre-activations of layer 1 (FP32)
  bf16x4 h1[4];  // bfloat16 ReLU outputs of layer 1
  f32x4 z2[4];
  bf16x4 h2[4];
  float y;  // network output of sample r, valid on lanes with g == 0
};

typedef __bf16 bf16x2n __attribute__((ext_vector_type(2)));

// Four FP32 values to bfloat16 (round to nearest even) with the native
// packed conversion.
__device__ __forceinline__ bf16x4 to_bf16x4(float a, float b, float c, float d) {
  bf16x2n lo, hi;
  lo[0] = (__bf16)a;
  lo[1] = (__bf16)b;
  hi[0] = (__bf16)c;
  hi[1] = (__bf16)d;
  const uint32_t ul = __builtin_bit_cast(uint32_t, lo), uh = __builtin_bit_cast(uint32_t, hi);
  bf16x4 h;
  h[0] = (short)(ul & 0xFFFFu);
  h[1] = (short)(ul >> 16);
  h[2] = (short)(uh & 0xFFFFu);
  h[3] = (short)(uh >> 16);
  return h;
}

__device__ __forceinline__ bf16x4 relu_bf16(f32x4 z) {
  return to_bf16x4(fmaxf(z[0], 0.0f), fmaxf(z[1], 0.0f), fmaxf(z[2], 0.0f), fmaxf(z[3], 0.0f));
}

// x: the tile's inputs in B layout (sample r, inputs 4g..4g+3) as bfloat16.
__device__ __forceinline__ void forward(const Weights& W, bf16x4 x, Acts& A) {
  const int g = (threadIdx.x & 63) >> 4;
#pragma unroll
  for (int h = 0; h < 4; ++h) A.z1[h] = mma(W.a1[h], x, W.b1[h]);
#pragma unroll
  for (int h = 0; h < 4; ++h) A.h1[h] = relu_bf16(A.z1[h]);
  const bf16x8 h1a = pair(A.h1[0], A.h1[1]), h1b = pair(A.h1[2], A.h1[3]);
#pragma unroll
  for (int o = 0; o < 4; ++o) {
    f32x4 acc = W.b2[o];
    acc = mma32(pair(W.a2[o][0], W.a2[o][1]), h1a, acc);
    acc = mma32(pair(W.a2[o][2], W.a2[o][3]), h1b, acc);
    A.z2[o] = acc;
  }
#pragma unroll
  for (int o = 0; o < 4; ++o) A.h2[o] = relu_bf16(A.z2[o]);
  f32x4 acc = {g == 0 ? W.b3 : 0.0f, 0.0f, 0.0f, 0.0f};
  acc = mma32(pair(W.a3[0], W.a3[1]), pair(A.h2[0], A.h2[1]), acc);
  acc = mma32(pair(W.a3[2], W.a3[3]), pair(A.h2[2], A.h2[3]), acc);
  A.y = acc[0];
}

}  // namespace mlp
}  // namespace chap
