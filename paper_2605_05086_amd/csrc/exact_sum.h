// Exact sums of FP64 values on the device, rounded once to nearest.
//
// The objective row c^T x is a sum over every variable: its FP64 value
// depends on the order of summation unless the exact value is rounded once.
// Walks whose objective products or partial sums may be inexact keep
// sum_j c_j x_j exactly, as a fixed-point integer of kExactLimbs limbs of 32
// bits (limb i weighs 2^(32 i - kExactBias)); the lowest limb lies below
// 2^-1074 and the highest above 2^1024 times 2^31 terms, so every finite
// double, and every sum of fewer than 2^31 of them, is represented exactly.
// A product c x enters as the pair (p, e) with p = c x rounded and
// e = fma(c, x, -p), whose sum is c x exactly (unless the product
// underflows). A move of x_j from a to b adds c b and subtracts c a, so the
// sum is kept incrementally with no drift, and f = c^T x and the cutoff
// residual c^T x - b_c are rounded from it (section 3.2).
//
// The wavefront form keeps limb i in lane i (register `a`) and limb 64 + i in
// lane i < 4 (register `b`); limbs 0..66 are kept in [0, 2^32) by carry
// propagation and the top limb holds the signed rest.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace chap {

constexpr int kExactLimbs = 68;
constexpr int kExactBias = 1088;

// Splits v into three signed 32-bit digits placed at limbs L, L+1, L+2:
// v = sum_t d[t] 2^(32 (L + t) - kExactBias). Returns L, or -1 for zero.
__device__ __forceinline__ int exact_split(double v, long long d[3]) {
  const unsigned long long bits = (unsigned long long)__double_as_longlong(v);
  const int ex = (int)((bits >> 52) & 0x7FF);
  unsigned long long m = bits & 0xFFFFFFFFFFFFFull;
  int e = -1074;
  if (ex != 0) {
    m |= 1ull << 52;
    e = ex - 1075;
  }
  if (m == 0) return -1;
  const int pos = e + kExactBias;  // >= 14
  const unsigned __int128 t = (unsigned __int128)m << (pos & 31);
  d[0] = (long long)(uint32_t)t;
  d[1] = (long long)(uint32_t)(t >> 32);
  d[2] = (long long)(uint32_t)(t >> 64);
  if (bits >> 63) {
    d[0] = -d[0];
    d[1] = -d[1];
    d[2] = -d[2];
  }
  return pos >> 5;
}

// The exact value of c x as p + e (TwoProduct with one fused multiply-add).
__device__ __forceinline__ void exact_product(double c, double x, double& p, double& e) {
  p = c * x;
  e = fma(c, x, -p);
}

// Adds v into an accumulator of kExactLimbs limbs in shared memory with
// 64-bit atomics (digits of many values may be added before a carry pass).
__device__ __forceinline__ void exact_atomic_add(long long* acc, double v) {
  long long d[3];
  const int L = exact_split(v, d);
  if (L < 0) return;
#pragma unroll
  for (int t = 0; t < 3; ++t)
    if (d[t] != 0) atomicAdd((unsigned long long*)&acc[L + t], (unsigned long long)d[t]);
}

// One wavefront's accumulator (every lane of the wavefront takes part in
// every call; results are uniform across the lanes).
struct WaveExact {
  long long a = 0;  // limb lane
  long long b = 0;  // limb 64 + lane (lanes 0..3)

  __device__ __forceinline__ static int lane() { return (int)(threadIdx.x & 63); }

  __device__ __forceinline__ void load(const long long* g) {
    const int l = lane();
    a = g[l];
    b = l < kExactLimbs - 64 ? g[64 + l] : 0;
  }
  __device__ __forceinline__ void store(long long* g) const {
    const int l = lane();
    g[l] = a;
    if (l < kExactLimbs - 64) g[64 + l] = b;
  }
  __device__ __forceinline__ void add(double v) {
    long long d[3];
    const int L = exact_split(v, d);
    if (L < 0) return;
    const int l = lane();
#pragma unroll
    for (int t = 0; t < 3; ++t) {
      if (l == L + t) a += d[t];
      if (l + 64 == L + t) b += d[t];
    }
  }
  // Carries of limbs 0..66 into the next limb until every one of them is in
  // [0, 2^32); one limb per round, so a round with no carry ends it.
  __device__ void normalize() {
    const int l = lane();
    for (;;) {
      const long long ca = a >> 32;
      const long long cb = (l < kExactLimbs - 64 - 1) ? (b >> 32) : 0;
      if (__ballot(ca != 0 || cb != 0) == 0ull) break;
      a -= ca * 4294967296LL;
      b -= cb * 4294967296LL;
      const long long up_a = __shfl_up(ca, 1, 64);
      const long long out_a = __shfl(ca, 63, 64);
      const long long up_b = __shfl_up(cb, 1, 64);
      if (l > 0) a += up_a;
      if (l == 0) b += out_a;
      if (l > 0 && l < kExactLimbs - 64) b += up_b;
    }
  }
  // The value rounded to the nearest double (ties to even); an exact zero
  // gives +0. Needs a normalised accumulator.
  __device__ double round_nearest() const {
    const int l = lane();
    long long A = a, B = b;
    const bool neg = __shfl(b, kExactLimbs - 64 - 1, 64) < 0;
    if (neg) {
      WaveExact t;
      t.a = -a;
      t.b = -b;
      t.normalize();
      A = t.a;
      B = t.b;
    }
    const unsigned long long mb = __ballot(B != 0 && l < kExactLimbs - 64);
    const unsigned long long ma = __ballot(A != 0);
    if (mb == 0ull && ma == 0ull) return 0.0;
    const int H = mb ? 64 + 63 - __builtin_clzll(mb) : 63 - __builtin_clzll(ma);
    auto limb = [&](int i) -> unsigned long long {
      if (i < 0) return 0ull;
      const long long v = i < 64 ? __shfl(A, i, 64) : __shfl(B, i - 64, 64);
      return (unsigned long long)v;
    };
    unsigned long long bits;
    const int nb = 64 - __builtin_clzll(limb(H));
    const int P = 32 * H + nb - 1 - kExactBias;  // exponent of the leading bit
    if (P >= -1022) {
      // H >= 2 here: 96 bits from the three top limbs, a sticky bit below
      const unsigned __int128 X = ((unsigned __int128)limb(H) << 64) | ((unsigned __int128)limb(H - 1) << 32) |
                                  (unsigned __int128)limb(H - 2);
      const bool sticky = __ballot(A != 0 && l < H - 2) != 0ull || __ballot(B != 0 && l + 64 < H - 2) != 0ull;
      const int sh = nb + 64 - 53;
      unsigned long long M = (unsigned long long)(X >> sh);
      const unsigned __int128 R = X & (((unsigned __int128)1 << sh) - 1);
      const unsigned __int128 half = (unsigned __int128)1 << (sh - 1);
      int E = P;
      if (R > half || (R == half && (sticky || (M & 1ull)))) M += 1;
      if (M >> 53) {
        M >>= 1;
        E += 1;
      }
      if (E > 1023)
        bits = 0x7FF0000000000000ull;
      else
        bits = ((unsigned long long)(E + 1023) << 52) | (M & 0xFFFFFFFFFFFFFull);
    } else {
      // below 2^-1022: the whole value sits in limbs 0..2, in units of 2^-1088
      const unsigned __int128 N = ((unsigned __int128)limb(2) << 64) | ((unsigned __int128)limb(1) << 32) |
                                  (unsigned __int128)limb(0);
      const int sh = kExactBias - 1074;
      unsigned long long q = (unsigned long long)(N >> sh);
      const unsigned long long r = (unsigned long long)(N & ((1u << sh) - 1));
      const unsigned long long half = 1ull << (sh - 1);
      if (r > half || (r == half && (q & 1ull))) q += 1;
      bits = q;
    }
    const double v = __longlong_as_double((long long)bits);
    return neg ? -v : v;
  }
  // (value + v) rounded to nearest, the accumulator unchanged.
  __device__ double round_plus(double v) const {
    WaveExact t = *this;
    t.add(v);
    t.normalize();
    return t.round_nearest();
  }
};

}  // namespace chap
