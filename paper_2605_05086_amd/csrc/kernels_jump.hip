// Jump values: for every variable the value that minimises the weighted
// violation of its constraints with the other variables held (the jump
// value of Feasibility Jump, which section 3.1 "Best Shift Moves" recalls
// as the move the paper's line sweep generalises).
//
// For column q at the point xbar,
//   V_q(t) = sum over q's stored rows i, in ascending order, of
//            w0_i max(0, y) and, for an equality row, then w1_i max(0, -y),
//            with y = r_i + a_iq (t - xbar_q);
//            then, with the cutoff row active and c_q != 0,
//            w_c max(0, r_c + c_q (t - xbar_q)).
// The jump value minimises V_q over the domain without xbar_q (ties: the
// value closest to xbar_q, then the smaller); the score is V_q(xbar_q) -
// V_q(t*); no value to try gives (xbar_q, 0). An integer variable with at
// most 64 values tries every value; any other variable the kinks of V_q
// (xbar - r_i / a_iq; an integer variable: the integers on either side),
// its finite bounds and, for an integer variable, xbar +- 1 (V_q is convex
// and piecewise linear, so its minimum over the domain is among them).
//
// Every V_q(t) is one sum in the order above, evaluated directly at t:
//   k_jump_lane    columns with at most kJumpLane stored entries, one lane
//                  each, entries in registers, candidates one after another;
//   k_jump_tasks   longer columns: one wavefront per (column, tile of 64
//                  candidates, chunk of kJumpChunk entries), a lane per
//                  candidate; the wavefront loads 64 entries at a time and
//                  every lane adds each entry's terms in order (entry values
//                  broadcast from the loading lane);
//   k_jump_combine one wavefront per longer column: the chunks' partial sums
//                  in chunk order, the cutoff term, the argmin over tiles.
// A column of one chunk is summed exactly in the stored order; longer
// columns add per-chunk partial sums, exact on integer data.

#include "chap_internal.h"

namespace chap {
namespace {

__device__ __forceinline__ double relu(double y) { return y > 0.0 ? y : 0.0; }

__device__ __forceinline__ bool jump_narrow(bool isint, double l, double u) {
  return isint && isfinite(l) && isfinite(u) && u - l + 1.0 <= (double)kJumpNarrow;
}

// (v, |t - xb|, t) lexicographically smaller than (bv, |bt - xb|, bt).
__device__ __forceinline__ bool jump_better(double v, double t, double bv, double bt, double xb) {
  if (v != bv) return v < bv;
  const double dt = fabs(t - xb), db = fabs(bt - xb);
  if (dt != db) return dt < db;
  return t < bt;
}

__device__ __forceinline__ double bcast(double v, int k) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffll), k);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), k);
  return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}
__device__ __forceinline__ float bcastf(float v, int k) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), k));
}

// Candidate c of a longer column (its tile-major numbering): for a narrow
// column the value l + c; otherwise entry c / 2's kink (integer: floor for
// even c, ceil for odd; continuous: even c only), then the cutoff row's
// kink(s), l, u, xb - 1, xb + 1 (integers) and last xb itself, the point
// whose V the score needs. `valid`: a value to try; `current`: t = xb.
struct JumpCand {
  double t;
  bool valid;
  bool current;
};

__device__ __forceinline__ JumpCand jump_candidate(const DevProblem& P, const RowState* rs, const WalkState* st,
                                                   int q, int beg, int deg, double xb, double l, double u, bool isint,
                                                   bool narrow, int c) {
  JumpCand o{xb, false, false};
  if (narrow) {
    const int W = (int)(u - l) + 1;
    if (c < W) {
      o.t = l + (double)c;
      o.current = o.t == xb;
      o.valid = !o.current;
    }
    return o;
  }
  double t = xb;
  bool ok = false;
  if (c < 2 * deg) {
    const int e = beg + (c >> 1);
    const double kink = xb - rs[P.col_row[e]].r / P.col_val[e];
    if (isint) {
      t = (c & 1) ? ceil(kink) : floor(kink);
      ok = true;
    } else {
      t = kink;
      ok = (c & 1) == 0;
    }
  } else {
    const int s = c - 2 * deg;
    const double cq = P.obj[q];
    const bool cact = st->cut_active && cq != 0.0;
    if (s < 2) {
      if (cact) {
        const double kink = xb - st->rc / cq;
        if (isint) {
          t = s ? ceil(kink) : floor(kink);
          ok = true;
        } else {
          t = kink;
          ok = s == 0;
        }
      }
    } else if (s == 2) {
      t = l;
      ok = true;
    } else if (s == 3) {
      t = u;
      ok = true;
    } else if (s == 4 || s == 5) {
      t = (s == 4) ? xb - 1.0 : xb + 1.0;
      ok = isint;
    } else if (s == 6) {
      o.current = true;
      return o;
    }
  }
  if (ok && isfinite(t) && t >= l && t <= u && t != xb) {
    o.t = t;
    o.valid = true;
  }
  return o;
}

// Candidates of a longer column: tiles of kWave.
__device__ __forceinline__ int jump_tiles(bool narrow, int deg) {
  return narrow ? 1 : (2 * deg + kJumpSpecials + kWave - 1) / kWave;
}

__global__ __launch_bounds__(256) void k_jump_lane(DevProblem P, const double* __restrict__ x,
                                                   const RowState* __restrict__ rs, const WalkState* __restrict__ st,
                                                   double* __restrict__ jv, double* __restrict__ js) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= P.n) return;
  const int beg = P.col_ptr[q], deg = P.col_ptr[q + 1] - beg;
  if (deg > kJumpLane) return;
  const double xb = x[q], l = P.lb[q], u = P.ub[q];
  const bool isint = P.is_int[q] != 0;
  double r[kJumpLane], a[kJumpLane];
  float w0[kJumpLane], w1[kJumpLane];
#pragma unroll
  for (int k = 0; k < kJumpLane; ++k) {
    r[k] = 0.0;
    a[k] = 1.0;
    w0[k] = 0.0f;
    w1[k] = -1.0f;
    if (k < deg) {
      const RowState s = rs[P.col_row[beg + k]];
      r[k] = s.r;
      w0[k] = s.w0;
      w1[k] = s.w1;
      a[k] = P.col_val[beg + k];
    }
  }
  const double cq = P.obj[q];
  const bool cact = st->cut_active && cq != 0.0;
  const double rc = st->rc, wc = (double)st->wc;
  auto V = [&](double t) {
    const double d = t - xb;
    double v = 0.0;
#pragma unroll
    for (int k = 0; k < kJumpLane; ++k) {
      if (k < deg) {
        const double y = r[k] + a[k] * d;
        v = v + (double)w0[k] * relu(y);
        if (w1[k] >= 0.0f) v = v + (double)w1[k] * relu(-y);
      }
    }
    if (cact) v = v + wc * relu(rc + cq * d);
    return v;
  };
  bool found = false;
  double bt = xb, bv = 0.0;
  auto consider = [&](double t) {
    if (!(isfinite(t) && t >= l && t <= u && t != xb)) return;
    const double v = V(t);
    if (!found || jump_better(v, t, bv, bt, xb)) {
      found = true;
      bt = t;
      bv = v;
    }
  };
  if (jump_narrow(isint, l, u)) {
    const int W = (int)(u - l) + 1;
    for (int p = 0; p < W; ++p) consider(l + (double)p);
  } else {
#pragma unroll
    for (int k = 0; k < kJumpLane; ++k) {
      if (k < deg) {
        const double kink = xb - r[k] / a[k];
        if (isint) {
          consider(floor(kink));
          consider(ceil(kink));
        } else {
          consider(kink);
        }
      }
    }
    if (cact) {
      const double kink = xb - rc / cq;
      if (isint) {
        consider(floor(kink));
        consider(ceil(kink));
      } else {
        consider(kink);
      }
    }
    consider(l);
    consider(u);
    if (isint) {
      consider(xb - 1.0);
      consider(xb + 1.0);
    }
  }
  jv[q] = found ? bt : xb;
  js[q] = found ? V(xb) - bv : 0.0;
}

__global__ __launch_bounds__(256) void k_jump_tasks(DevProblem P, const double* __restrict__ x,
                                                    const RowState* __restrict__ rs, const WalkState* __restrict__ st,
                                                    const JumpTask* __restrict__ tasks, int32_t ntasks,
                                                    double* __restrict__ part) {
  const int id = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (id >= ntasks) return;  // whole wavefronts leave together
  const int lane = threadIdx.x & (kWave - 1);
  const JumpTask T = tasks[id];
  const int q = T.q;
  const int beg = P.col_ptr[q], deg = P.col_ptr[q + 1] - beg;
  const double xb = x[q], l = P.lb[q], u = P.ub[q];
  const bool isint = P.is_int[q] != 0;
  const bool narrow = jump_narrow(isint, l, u);
  const JumpCand cd = jump_candidate(P, rs, st, q, beg, deg, xb, l, u, isint, narrow, T.tile * kWave + lane);
  const double d = cd.t - xb;
  const int e0 = beg + T.chunk * kJumpChunk;
  const int e1 = min(beg + deg, e0 + kJumpChunk);
  double v = 0.0;
  for (int base = e0; base < e1; base += kWave) {
    const int e = base + lane;
    double rr = 0.0, aa = 0.0;
    float ww0 = 0.0f, ww1 = -1.0f;
    if (e < e1) {
      const RowState s = rs[P.col_row[e]];
      rr = s.r;
      ww0 = s.w0;
      ww1 = s.w1;
      aa = P.col_val[e];
    }
    const int cnt = min(kWave, e1 - base);
    for (int k = 0; k < cnt; ++k) {
      const double rk = bcast(rr, k), ak = bcast(aa, k);
      const float w0k = bcastf(ww0, k), w1k = bcastf(ww1, k);
      const double y = rk + ak * d;
      v = v + (double)w0k * relu(y);
      if (w1k >= 0.0f) v = v + (double)w1k * relu(-y);
    }
  }
  part[(size_t)T.slot * kWave + lane] = v;
}

__global__ __launch_bounds__(256) void k_jump_combine(DevProblem P, const double* __restrict__ x,
                                                      const RowState* __restrict__ rs,
                                                      const WalkState* __restrict__ st,
                                                      const JumpCol* __restrict__ cols, int32_t ncols,
                                                      const double* __restrict__ part, double* __restrict__ jv,
                                                      double* __restrict__ js) {
  const int id = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (id >= ncols) return;  // whole wavefronts leave together
  const int lane = threadIdx.x & (kWave - 1);
  const JumpCol J = cols[id];
  const int q = J.q;
  const int beg = P.col_ptr[q], deg = P.col_ptr[q + 1] - beg;
  const double xb = x[q], l = P.lb[q], u = P.ub[q];
  const bool isint = P.is_int[q] != 0;
  const bool narrow = jump_narrow(isint, l, u);
  const double cq = P.obj[q];
  const bool cact = st->cut_active && cq != 0.0;
  const double rc = st->rc, wc = (double)st->wc;
  bool found = false;
  double bt = xb, bv = 0.0, v0 = 0.0;
  bool have0 = false;
  for (int tile = 0; tile < J.ntiles; ++tile) {
    const JumpCand cd = jump_candidate(P, rs, st, q, beg, deg, xb, l, u, isint, narrow, tile * kWave + lane);
    const int s0 = J.first_slot + tile * J.nchunks;
    double v = part[(size_t)s0 * kWave + lane];
    for (int ch = 1; ch < J.nchunks; ++ch) v = v + part[(size_t)(s0 + ch) * kWave + lane];
    if (cact) v = v + wc * relu(rc + cq * (cd.t - xb));
    if (cd.current) {
      v0 = v;
      have0 = true;
    }
    if (cd.valid && (!found || jump_better(v, cd.t, bv, bt, xb))) {
      found = true;
      bt = cd.t;
      bv = v;
    }
  }
  // argmin across the lanes; V(xb) from the lane that evaluated it
#pragma unroll
  for (int o = 1; o < kWave; o <<= 1) {
    const double ov = __shfl_xor(bv, o, kWave), ot = __shfl_xor(bt, o, kWave);
    const bool of = __shfl_xor((int)found, o, kWave) != 0;
    if (of && (!found || jump_better(ov, ot, bv, bt, xb))) {
      found = true;
      bt = ot;
      bv = ov;
    }
  }
  const unsigned long long m0 = __ballot(have0);
  const int l0 = m0 ? __builtin_ctzll(m0) : 0;
  v0 = __shfl(v0, l0, kWave);
  if (lane == 0) {
    jv[q] = found ? bt : xb;
    js[q] = found ? v0 - bv : 0.0;
  }
}

}  // namespace

hipError_t launch_jump(const DevProblem& P, const double* x, const RowState* rs, const WalkState* st,
                       const JumpTask* tasks, int32_t ntasks, const JumpCol* cols, int32_t ncols, double* part,
                       double* jv, double* js, hipStream_t s) {
  if (P.n > 0) hipLaunchKernelGGL(k_jump_lane, dim3((P.n + 255) / 256), dim3(256), 0, s, P, x, rs, st, jv, js);
  if (ntasks > 0)
    hipLaunchKernelGGL(k_jump_tasks, dim3((ntasks + 3) / 4), dim3(256), 0, s, P, x, rs, st, tasks, ntasks, part);
  if (ncols > 0)
    hipLaunchKernelGGL(k_jump_combine, dim3((ncols + 3) / 4), dim3(256), 0, s, P, x, rs, st, cols, ncols, part, jv,
                       js);
  return hipGetLastError();
}

}  // namespace chap
