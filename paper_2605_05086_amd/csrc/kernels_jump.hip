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
//                  each, entries in registers, candidates one after another
//                  (on exact integer data narrow columns too try only the
//                  kinks' neighbours, bounds and xbar +- 1);
//   k_jump_tasks   longer columns: one wavefront per (column, tile of 64
//                  candidates, chunk of kJumpChunk entries), a lane per
//                  candidate; the wavefront loads 64 entries at a time into
//                  its LDS slice and every lane adds each entry's terms in
//                  order (one broadcast read per entry);
//   k_jump_combine one wavefront per longer column: the chunks' partial sums
//                  in chunk order, the cutoff term, the argmin over tiles;
//   k_jump_bins_combine one workgroup per chunked column with a bins form on
//                  exact data: the chunks' bins, the scan and the argmin.
// A column of one chunk is summed exactly in the stored order; longer
// columns add per-chunk partial sums, exact on integer data.

#include <algorithm>

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

// Exact data for this call: the instance's data are integers with every
// residual within the bounds in int32 (exact_data), the weights are integers
// below 2^16 (st->compact_rows), and the cutoff row, when active, has small
// integer terms.
__device__ __forceinline__ bool jump_exact(const WalkState* st, int32_t exact_data, int32_t obj_small) {
  return exact_data && st->compact_rows &&
         (!st->cut_active || (obj_small && st->rc == floor(st->rc) && fabs(st->rc) < 2147483648.0));
}

// One entry of a column as the wavefront tasks read it from LDS.
struct JumpEntry {
  double r;
  double a;
  float w0;
  float w1;
};

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

// exact_data: every residual within the bounds fits int32 and the data are
// integers; with integer weights below 2^16 (st->compact_rows) and a cutoff
// term of small integers, every V the lane forms is an exact integer below
// 2^53, and then the kinks' neighbours, the bounds and xbar +- 1 hold the
// chosen value of a narrow column too (a value strictly between them has
// neighbours on one line through it; a zero slope makes the neighbour
// towards xbar tie and win, any other slope makes a neighbour smaller), so
// narrow columns try those (and the integers next to them) instead of
// every value.
__global__ __launch_bounds__(256) void k_jump_lane(DevProblem P, const double* __restrict__ x,
                                                   const RowState* __restrict__ rs,
                                                   const GatherRow* __restrict__ grow, const WalkState* __restrict__ st,
                                                   int32_t exact_data, int32_t obj_small, double* __restrict__ jv,
                                                   double* __restrict__ js) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= P.n) return;
  const int beg = P.col_ptr[q], deg = P.col_ptr[q + 1] - beg;
  if (deg > kJumpLane) return;
  const double xb = x[q], l = P.lb[q], u = P.ub[q];
  const bool isint = P.is_int[q] != 0;
  const bool exact = jump_exact(st, exact_data, obj_small);
  double r[kJumpLane], a[kJumpLane];
  float w0[kJumpLane], w1[kJumpLane];
  // rows from the 8-byte compact copy on exact data (the same values), else
  // the 16-byte row states
#pragma unroll
  for (int k = 0; k < kJumpLane; ++k) {
    r[k] = 0.0;
    a[k] = 1.0;
    w0[k] = 0.0f;
    w1[k] = -1.0f;
    if (k < deg) {
      const int i = P.col_row[beg + k];
      if (exact) {
        const GatherRow g = grow[i];
        r[k] = (double)g.r;
        w0[k] = (float)g.w0;
        w1[k] = g.w1 == kNoTwin ? -1.0f : (float)g.w1;
      } else {
        const RowState s = rs[i];
        r[k] = s.r;
        w0[k] = s.w0;
        w1[k] = s.w1;
      }
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
  const bool narrow = jump_narrow(isint, l, u);
  // a narrow column on exact data: each kink's neighbours, widened by one
  // on either side so that a rounding of the FP64 kink across an integer
  // cannot hide one
  const int pad = narrow ? 1 : 0;
  auto kink_values = [&](double kink) {
    if (isint) {
      for (int o = -pad; o <= 0; ++o) consider(floor(kink) + (double)o);
      for (int o = 0; o <= pad; ++o) consider(ceil(kink) + (double)o);
    } else {
      consider(kink);
    }
  };
  if (narrow && !exact) {
    const int W = (int)(u - l) + 1;
    for (int p = 0; p < W; ++p) consider(l + (double)p);
  } else {
#pragma unroll
    for (int k = 0; k < kJumpLane; ++k)
      if (k < deg) kink_values(xb - r[k] / a[k]);
    if (cact) kink_values(xb - rc / cq);
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

__device__ void jump_task(const DevProblem& P, const double* __restrict__ x, const RowState* __restrict__ rs,
                          const WalkState* __restrict__ st, const JumpTask T, double* __restrict__ part) {
  const int lane = threadIdx.x & (kWave - 1);
  const int q = T.q;
  const int beg = P.col_ptr[q], deg = P.col_ptr[q + 1] - beg;
  const double xb = x[q], l = P.lb[q], u = P.ub[q];
  const bool isint = P.is_int[q] != 0;
  const bool narrow = jump_narrow(isint, l, u);
  const JumpCand cd = jump_candidate(P, rs, st, q, beg, deg, xb, l, u, isint, narrow, T.tile * kWave + lane);
  const double d = cd.t - xb;
  const int e0 = beg + T.chunk * kJumpChunk;
  const int e1 = min(beg + deg, e0 + kJumpChunk);
  // each batch of 64 entries goes through this wavefront's LDS slice; every
  // lane then reads entry k at one address (a broadcast)
  __shared__ JumpEntry S[4][kWave];
  JumpEntry* E = S[threadIdx.x >> 6];
  double v = 0.0;
  for (int base = e0; base < e1; base += kWave) {
    const int e = base + lane;
    JumpEntry me{0.0, 0.0, 0.0f, -1.0f};
    if (e < e1) {
      const RowState s = rs[P.col_row[e]];
      me.r = s.r;
      me.w0 = s.w0;
      me.w1 = s.w1;
      me.a = P.col_val[e];
    }
    // the previous batch's reads are done before the slice is overwritten
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    E[lane] = me;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    const int cnt = min(kWave, e1 - base);
#pragma unroll 4
    for (int k = 0; k < cnt; ++k) {
      const JumpEntry q = E[k];
      const double y = q.r + q.a * d;
      v = v + (double)q.w0 * relu(y);
      if (q.w1 >= 0.0f) v = v + (double)q.w1 * relu(-y);
    }
  }
  part[(size_t)T.slot * kWave + lane] = v;
}

// Grid-stride over the tasks, one wavefront per task: every task, or on
// exact data only the first n_plain (the tasks of columns without a bins
// form; the others are scored from bins).
__global__ __launch_bounds__(256) void k_jump_tasks(DevProblem P, const double* __restrict__ x,
                                                    const RowState* __restrict__ rs, const WalkState* __restrict__ st,
                                                    int32_t exact_data, int32_t obj_small,
                                                    const JumpTask* __restrict__ tasks, int32_t ntasks,
                                                    int32_t n_plain, double* __restrict__ part) {
  const int nt = jump_exact(st, exact_data, obj_small) ? n_plain : ntasks;
  for (int id = blockIdx.x * 4 + (threadIdx.x >> 6); id < nt; id += gridDim.x * 4)  // whole wavefronts
    jump_task(P, x, rs, st, tasks[id], part);
}

// floor(n / d) and ceil(n / d) for d > 0 and |n|, |d| < 2^31, through one
// FP64 division: an integer quotient is exact, and any other lies at least
// 1/d from an integer while the rounding moves it by at most |n/d| 2^-53 <
// 2^-22 / d, so floor and ceil are unchanged (64-bit integer division is a
// long software sequence on the GPU).
__device__ __forceinline__ long long floor_div(long long n, long long d) {
  return (long long)floor((double)n / (double)d);
}
__device__ __forceinline__ long long ceil_div(long long n, long long d) {
  return (long long)ceil((double)n / (double)d);
}

// One term w max(0, c + a p) over positions p = 0 .. W-1 as bin updates:
// from the first positive position on (a > 0), or up to the last one
// (a < 0), the term is w c + w a p. Updates of bin 0 (every term with a < 0
// that is positive at p = 0, and every term with a > 0 positive from p = 0)
// go to the lane's own k0 and s0, added into the bin once per wavefront:
// as LDS atomics they would all hit one address.
__device__ __forceinline__ void add_ramp(unsigned long long* K, unsigned long long* S, long long& k0, long long& s0,
                                         long long c, long long a, long long w, int W) {
  if (w == 0) return;
  if (a > 0) {
    const long long p0 = floor_div(-c, a) + 1;  // first p with c + a p > 0
    if (p0 < W) {
      if (p0 > 0) {
        atomicAdd(&K[p0], (unsigned long long)(w * c));
        atomicAdd(&S[p0], (unsigned long long)(w * a));
      } else {
        k0 += w * c;
        s0 += w * a;
      }
    }
  } else {
    const long long p1 = ceil_div(c, -a);  // first p with c + a p <= 0
    const int k = (int)(p1 < 0 ? 0 : (p1 > W ? W : p1));
    if (k > 0) {
      k0 += w * c;
      s0 += w * a;
      if (k < W) {
        atomicAdd(&K[k], (unsigned long long)(-w * c));
        atomicAdd(&S[k], (unsigned long long)(-w * a));
      }
    }
  }
}

// The argmin of a narrow column from its bins (lane p holds bin p of the
// offsets k and slopes sl, summed over the column's chunks): prefix sums
// across the lanes give V(l + p) exactly, the cutoff term is added in
// integers; lane 0 writes the jump value and score.
__device__ __forceinline__ void bins_finish(const DevProblem& P, const WalkState* st, int q, double xb, long long k,
                                            long long sl, double* jv, double* js) {
  const int lane = threadIdx.x & (kWave - 1);
  const double l = P.lb[q];
  const int W = (int)(P.ub[q] - l) + 1;
  const double cq = P.obj[q];
  const bool cact = st->cut_active && cq != 0.0;
#pragma unroll
  for (int o = 1; o < kWave; o <<= 1) {
    const long long yk = __shfl_up(k, o, kWave), ys = __shfl_up(sl, o, kWave);
    if (lane >= o) {
      k += yk;
      sl += ys;
    }
  }
  long long vi = k + (long long)lane * sl;
  const double t = l + (double)lane;
  if (cact) {
    const long long y = (long long)st->rc + (long long)cq * (long long)(t - xb);
    vi += (long long)st->wc * (y > 0 ? y : 0);
  }
  const double v = (double)vi;
  bool found = false, have0 = false;
  double bt = xb, bv = 0.0, v0 = 0.0;
  if (lane < W) {
    if (t == xb) {
      v0 = v;
      have0 = true;
    } else {
      found = true;
      bt = t;
      bv = v;
    }
  }
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
  v0 = __shfl(v0, m0 ? __builtin_ctzll(m0) : 0, kWave);
  if (lane == 0) {
    jv[q] = found ? bt : xb;
    js[q] = found ? v0 - bv : 0.0;
  }
}

// One wavefront per bins task: the chunk's entries (and the twins of
// equality rows), one per lane, as slope and offset bins of the column's
// positions in the wavefront's own LDS slice. A task's entries lie in one
// eighth of the rows, and the four tasks of a workgroup in the same eighth,
// which the task order places on one XCD, so the row gathers stay in that
// XCD's L2.
__global__ __launch_bounds__(256) void k_jump_bins(DevProblem P, const double* __restrict__ x,
                                                   const GatherRow* __restrict__ grow, const WalkState* __restrict__ st,
                                                   int32_t exact_data, int32_t obj_small,
                                                   const JumpBinTask* __restrict__ tasks, int32_t ntasks,
                                                   long long* __restrict__ bpart, double* __restrict__ jv,
                                                   double* __restrict__ js) {
  if (!jump_exact(st, exact_data, obj_small)) return;
  const int id = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (id >= ntasks) return;  // whole wavefronts leave together
  const int lane = threadIdx.x & (kWave - 1);
  __shared__ unsigned long long KB[4][kWave], SB[4][kWave];
  unsigned long long* K = KB[threadIdx.x >> 6];
  unsigned long long* S = SB[threadIdx.x >> 6];
  K[lane] = 0ull;
  S[lane] = 0ull;
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  const JumpBinTask T = tasks[id];
  if (T.q < 0) return;  // padding of the row-range interleave
  const int q = T.q;
  const double xb = x[q], l = P.lb[q];
  const int W = (int)(P.ub[q] - l) + 1;
  long long k0 = 0, s0 = 0;
  // one entry per lane and step (two or four in flight measured slower:
  // 363 and 375 against 348 us for the call's kernels on the 20M
  // instance); rows from the compact copy (exact on this path: integer
  // residuals and weights)
  constexpr int kU = 1;
  for (int e0 = T.e_beg + lane; e0 < T.e_end; e0 += kU * kWave) {
    GatherRow r[kU];
    double a[kU];
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      const int e = e0 + u * kWave;
      if (e < T.e_end) {
        r[u] = grow[P.col_row[e]];
        a[u] = P.col_val[e];
      }
    }
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      if (e0 + u * kWave >= T.e_end) break;
      const long long c = (long long)((double)r[u].r + a[u] * (l - xb));  // residual at x_q = l: an integer
      const long long ai = (long long)a[u];
      add_ramp(K, S, k0, s0, c, ai, (long long)r[u].w0, W);
      if (r[u].w1 != kNoTwin) add_ramp(K, S, k0, s0, -c, -ai, (long long)r[u].w1, W);
    }
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    k0 += __shfl_xor(k0, o, kWave);
    s0 += __shfl_xor(s0, o, kWave);
  }
  if (lane == 0) {
    atomicAdd(&K[0], (unsigned long long)k0);
    atomicAdd(&S[0], (unsigned long long)s0);
  }
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  if (T.slot < 0) {
    bins_finish(P, st, q, xb, (long long)K[lane], (long long)S[lane], jv, js);  // the whole column
    return;
  }
  bpart[(size_t)T.slot * 2 * kWave + lane] = (long long)K[lane];
  bpart[(size_t)T.slot * 2 * kWave + kWave + lane] = (long long)S[lane];
}

constexpr int kJumpInFlight = 16;  // chunk partials per load round of the combines

// A chunked column with a bins form on exact data (one workgroup per such
// column record): each wavefront adds every fourth chunk's bins,
// kJumpInFlight chunks per load round (integer sums, so any order gives the
// same bins), wavefront 0 adds the four partial sums and finishes.
__global__ __launch_bounds__(256) void k_jump_bins_combine(DevProblem P, const double* __restrict__ x,
                                                           const WalkState* __restrict__ st, int32_t exact_data,
                                                           int32_t obj_small, const JumpCol* __restrict__ cols,
                                                           const long long* __restrict__ bpart,
                                                           double* __restrict__ jv, double* __restrict__ js) {
  const JumpCol J = cols[blockIdx.x];  // the records of chunked columns with a bins form
  if (J.bn <= 0 || !jump_exact(st, exact_data, obj_small)) return;  // whole workgroup
  __shared__ long long red[2][3][kWave];
  const int lane = threadIdx.x & (kWave - 1), wv = threadIdx.x >> 6;
  long long k = 0, sl = 0;
  for (int ch0 = wv * kJumpInFlight; ch0 < J.bn; ch0 += 4 * kJumpInFlight) {
    long long kk[kJumpInFlight], ss[kJumpInFlight];
#pragma unroll
    for (int t = 0; t < kJumpInFlight; ++t) {
      const size_t b = (size_t)(J.bfirst + ch0 + t) * 2 * kWave + lane;
      kk[t] = ch0 + t < J.bn ? bpart[b] : 0ll;
      ss[t] = ch0 + t < J.bn ? bpart[b + kWave] : 0ll;
    }
#pragma unroll
    for (int t = 0; t < kJumpInFlight; ++t) {
      k += kk[t];
      sl += ss[t];
    }
  }
  if (wv > 0) {
    red[0][wv - 1][lane] = k;
    red[1][wv - 1][lane] = sl;
  }
  __syncthreads();
  if (wv != 0) return;
  for (int w = 0; w < 3; ++w) {
    k += red[0][w][lane];
    sl += red[1][w][lane];
  }
  bins_finish(P, st, J.q, x[J.q], k, sl, jv, js);
}

__device__ void jump_combine(const DevProblem& P, const double* __restrict__ x, const RowState* __restrict__ rs,
                             const WalkState* __restrict__ st, int32_t exact_data, int32_t obj_small, const JumpCol J,
                             const double* __restrict__ part, double* __restrict__ jv, double* __restrict__ js) {
  const int lane = threadIdx.x & (kWave - 1);
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
  // bins form on exact data: finished by its bins task or by k_jump_bins_combine
  if (J.bn != 0 && jump_exact(st, exact_data, obj_small)) return;
  for (int tile = 0; tile < J.ntiles; ++tile) {
    const JumpCand cd = jump_candidate(P, rs, st, q, beg, deg, xb, l, u, isint, narrow, tile * kWave + lane);
    const int s0 = J.first_slot + tile * J.nchunks;
    // the chunks' partial sums added in chunk order, kJumpInFlight loaded
    // at a time
    double v = part[(size_t)s0 * kWave + lane];
    for (int ch0 = 1; ch0 < J.nchunks; ch0 += kJumpInFlight) {
      double pv[kJumpInFlight];
#pragma unroll
      for (int t = 0; t < kJumpInFlight; ++t)
        if (ch0 + t < J.nchunks) pv[t] = part[(size_t)(s0 + ch0 + t) * kWave + lane];
#pragma unroll
      for (int t = 0; t < kJumpInFlight; ++t)
        if (ch0 + t < J.nchunks) v = v + pv[t];
    }
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

// Grid-stride over the column records, one wavefront per record: every
// record, or on exact data only the first n_plain (the columns without a
// bins form).
__global__ __launch_bounds__(256) void k_jump_combine(DevProblem P, const double* __restrict__ x,
                                                      const RowState* __restrict__ rs,
                                                      const WalkState* __restrict__ st,
                                                      int32_t exact_data, int32_t obj_small,
                                                      const JumpCol* __restrict__ cols, int32_t ncols,
                                                      int32_t n_plain, const double* __restrict__ part,
                                                      double* __restrict__ jv, double* __restrict__ js) {
  const int nc = jump_exact(st, exact_data, obj_small) ? n_plain : ncols;
  for (int id = blockIdx.x * 4 + (threadIdx.x >> 6); id < nc; id += gridDim.x * 4)  // whole wavefronts
    jump_combine(P, x, rs, st, exact_data, obj_small, cols[id], part, jv, js);
}

}  // namespace

hipError_t launch_jump(const DevProblem& P, const double* x, const RowState* rs, const WalkState* st,
                       const GatherRow* grow, int32_t obj_small, const JumpTask* tasks, int32_t ntasks,
                       int32_t n_plain_tasks, const JumpBinTask* btasks, int32_t nbtasks, const JumpCol* cols,
                       int32_t ncols, int32_t n_plain_cols, int32_t n_chunk_cols, double* part, long long* bpart,
                       double* jv, double* js, hipStream_t s) {
  const int32_t exact_data = grow != nullptr ? 1 : 0;
  constexpr int kStrideGrid = 2048;  // workgroups of the grid-stride kernels
  if (P.n > 0)
    hipLaunchKernelGGL(k_jump_lane, dim3((P.n + 255) / 256), dim3(256), 0, s, P, x, rs, grow, st, exact_data,
                       obj_small, jv, js);
  if (nbtasks > 0)
    hipLaunchKernelGGL(k_jump_bins, dim3((unsigned)((nbtasks + 3) / 4)), dim3(256), 0, s, P, x, grow, st, exact_data,
                       obj_small, btasks, nbtasks, bpart, jv, js);
  if (ntasks > 0)
    hipLaunchKernelGGL(k_jump_tasks, dim3((unsigned)std::min((ntasks + 3) / 4, kStrideGrid)), dim3(256), 0, s, P, x,
                       rs, st, exact_data, obj_small, tasks, ntasks, n_plain_tasks, part);
  if (ncols > 0)
    hipLaunchKernelGGL(k_jump_combine, dim3((unsigned)std::min((ncols + 3) / 4, kStrideGrid)), dim3(256), 0, s, P, x,
                       rs, st, exact_data, obj_small, cols, ncols, n_plain_cols, part, jv, js);
  if (n_chunk_cols > 0)
    hipLaunchKernelGGL(k_jump_bins_combine, dim3((unsigned)n_chunk_cols), dim3(256), 0, s, P, x, st, exact_data,
                       obj_small, cols + n_plain_cols, bpart, jv, js);
  return hipGetLastError();
}

}  // namespace chap
