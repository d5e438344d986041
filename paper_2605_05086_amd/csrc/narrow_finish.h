// Last steps of Algorithm 1 (section 3.1) for a narrow integer column whose
// breakpoint terms are binned by value: the prefix scan over the bins, the
// argmax over candidate positions (Eq. 1, ties to the smallest shift) and
// the write of the column's best shift. The pass kernels use them, and so
// does the move selection, which combines the partial bins of long columns
// itself when the pass that produced them leaves that step to it.
#pragma once

#include <hip/hip_runtime.h>

#include <cfloat>
#include <climits>

#include "chap_internal.h"

namespace chap {

// (value desc, key asc) argmax across the wavefront; invalid lanes carry
// value = -inf and key = INT_MAX.
__device__ __forceinline__ void wave_argmax(double& v, int& key) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    const double ov = __shfl_xor(v, o, kWave);
    const int ok = __shfl_xor(key, o, kWave);
    if (ov > v || (ov == v && ok < key)) {
      v = ov;
      key = ok;
    }
  }
}

// The score a column keeps: the best positive score and its position, else
// score 0 at the current value.
template <typename Ptr>
__device__ __forceinline__ void write_result(Ptr xhat, Ptr sc, int j, bool found, double best, double bestp,
                                             double xb) {
  if (found && best > 0.0) {
    xhat[j] = bestp + 0.0;  // canonical +0.0
    sc[j] = best;
  } else {
    xhat[j] = xb;
    sc[j] = 0.0;
  }
}

// Scan + argmax over the 64 bins of one column by one wavefront; lane b holds
// bin b. The result is valid on every lane.
__device__ __forceinline__ void narrow_finish(double binv, double beta, double alpha, unsigned long long cand,
                                              double xb, double l, int W, int lane, bool& found, double& best,
                                              double& bestp) {
  double v = (lane < W) ? binv : 0.0;
#pragma unroll
  for (int o = 1; o < kWave; o <<= 1) {
    const double y = __shfl_up(v, o, kWave);
    if (lane >= o) v += y;
  }
  const double pos = l + (double)lane;
  double val = beta + v + ((pos > xb) ? alpha : 0.0);
  const bool ok = lane < W && ((((cand >> lane) & 1ull) != 0) || lane == 0 || lane == W - 1) && pos != xb;
  int key = ok ? lane : INT_MAX;
  if (!ok) val = -DBL_MAX;
  wave_argmax(val, key);
  found = key != INT_MAX;
  best = val;
  bestp = found ? l + (double)key : xb;
}

// Long narrow column idx (a ChunkCol record) from its chunks' partial bins,
// added in slot order (a fixed summation order); one wavefront. Writes the
// column's best shift and returns, on every lane, the score it kept; *q gets
// the column's internal index. Up to 64 partials at a time: lane t loads the
// scalars of partial t (added in slot order from its neighbours' registers)
// and every lane its bin of kCombineInFlight partials per load round.
constexpr int kCombineInFlight = 8;
__device__ __forceinline__ double combine_col(const WalkCtx& W0, int idx, int lane, int* q) {
  const DevProblem& P = W0.P;
  const ChunkCol C = W0.plan.chunk_cols[idx];
  *q = C.col;
  const double xb = gmem((const double*)W0.x)[C.col];
  const double l = gmem(P.lb)[C.col], u = gmem(P.ub)[C.col];
  const int W = (int)(u - l) + 1;
  double bv = 0.0, b = 0.0, a = 0.0;
  unsigned long long c = 0;
  const gptr<const ChunkPartial> pp = gmem((const ChunkPartial*)W0.partials) + C.first;
  for (int k0 = 0; k0 < C.nparts; k0 += kWave) {
    const int cnt = min(kWave, C.nparts - k0);
    double sb = 0.0, sa = 0.0;
    unsigned long long sc = 0;
    if (lane < cnt) {
      sb = pp[k0 + lane].beta;
      sa = pp[k0 + lane].alpha;
      sc = pp[k0 + lane].cand;
    }
    for (int k1 = 0; k1 < cnt; k1 += kCombineInFlight) {
      double pv[kCombineInFlight];
#pragma unroll
      for (int t = 0; t < kCombineInFlight; ++t)
        if (k1 + t < cnt) pv[t] = pp[k0 + k1 + t].bins[lane];
#pragma unroll
      for (int t = 0; t < kCombineInFlight; ++t)
        if (k1 + t < cnt) bv += pv[t];
    }
    for (int t = 0; t < cnt; ++t) {
      b += __shfl(sb, t, kWave);
      a += __shfl(sa, t, kWave);
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) sc |= __shfl_xor(sc, o, kWave);
    c |= sc;
  }
  bool found;
  double best, bestp;
  narrow_finish(bv, b, a, c, xb, l, W, lane, found, best, bestp);
  if (lane == 0) write_result(gmem(W0.xhat), gmem(W0.s), C.col, found, best, bestp, xb);
  return (found && best > 0.0) ? best : 0.0;
}

}  // namespace chap
