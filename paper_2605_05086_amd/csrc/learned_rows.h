// Device helpers for the stored input rows of the learned proposal (shared
// by the proposal kernels and the move-selection kernels).
#pragma once

#include <cmath>

#include "chap_internal.h"
#include "mlp_core.h"

namespace chap {
namespace learned {

constexpr int64_t kAgeCap = 1024;
constexpr int32_t kNeverMoved = -1024;

// FP64 -> bfloat16 bits, round to nearest even, for magnitudes in FP32's
// normal range (or zero): round to 8 significant bits in FP64, then the FP32
// conversion and truncation to 16 bits are exact.
__device__ __forceinline__ uint16_t d2bf(double d) {
  unsigned long long b = (unsigned long long)__double_as_longlong(d);
  b += 0xFFFFFFFFFFFull + ((b >> 45) & 1ull);
  b &= ~((1ull << 45) - 1ull);
  return mlp::f2bf((float)__longlong_as_double((long long)b));
}

__device__ __forceinline__ double position(double x, double l, double u) {
  if (!isfinite(l) || !isfinite(u)) return 0.5;
  if (u > l) return (x - l) / (u - l);
  return 0.0;
}

__device__ __forceinline__ double sign_of(double v) { return v > 0.0 ? 1.0 : (v < 0.0 ? -1.0 : 0.0); }

__device__ __forceinline__ void set_last_move(uint16_t* row, int32_t k) {
  row[12] = (uint16_t)((uint32_t)k & 0xFFFFu);
  row[13] = (uint16_t)((uint32_t)k >> 16);
}

// Stored-row update after the walk moved column st->mv_j at iteration st->k
// (one thread, before the iteration ends).
__device__ __forceinline__ void after_move(const WalkCtx& C, const LearnCtx& L) {
  const WalkState* st = C.st;
  const int q = st->mv_j;
  if (q < 0) return;
  uint16_t* row = L.feat + (int64_t)q * 16;
  const int32_t mv = L.moves[q] + 1;
  L.moves[q] = mv;
  const double xn = st->mv_new;
  row[7] = d2bf(position(xn, C.P.lb[q], C.P.ub[q]));
  row[11] = d2bf(sign_of(L.xhat_last[q] - xn));
  row[15] = d2bf(log2(1.0 + (double)mv));
  set_last_move(row, (int32_t)st->k);
}

}  // namespace learned
}  // namespace chap
