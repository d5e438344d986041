// Learned candidate proposal for one tabu walk on gfx950.
//
// The paper scores every column exactly in every iteration (section 3.1,
// "Scoring Functions"). Here a network ranks the columns and only its top K
// get the exact best shift; a full pass every few iterations (or after a
// proposal iteration without an admissible move) is the fallback, the judge
// of the network and the source of its training pairs. Every move taken is
// still an exact best shift under the tabu and aspiration rules.
//
// Stored feature rows (16 bfloat16 per column, internal order):
//   0 weighted violated share   sum_{viol} w / sum w over the column's rows
//   1 log2(1 + stored entries)
//   2 c_j / max |c|
//   3 s_last / sum w, clamped to [-4, 4] (score at the last full pass)
//   4 binary  5 general integer  6 continuous
//   7 position (x - l) / (u - l) (0.5 for an infinite bound, 0 for l = u)
//   8 log2(1 + min(u - l, 2^20)) (20 for an infinite bound)
//   9 unweighted violated share
//  10 violated mass: sum_{viol} |a| min(r, 1000) / (1000 sum |a|)
//  11 sign(xhat_last - x)
//  12..13 (storage) int32 iteration of the column's last move
//  15 log2(1 + moves of the column)
// Inputs 12..14 of the network are formed when a row is read: the tabu age
// min(k - last move, 1024) / 1024, min(k - last full pass, 64) / 64, and the
// violated fraction V / m'. Inputs 0, 3, 9, 10 are refreshed at full passes
// only; 7, 11, 12, 15 change with the column's own moves. Every value is
// computed in FP64 and rounded once to bfloat16.
//
// Top-K: scores become order-preserving 32-bit keys (0 = never proposed); a
// three-digit radix select (11, 11, 10 bits) finds the K-th key, and an
// order-preserving compaction lists the selected columns in ascending
// internal index (equal keys: lowest index first).

#include <climits>
#include <cmath>

#include "chap_internal.h"
#include "mlp_core.h"

namespace chap {
namespace {

using namespace mlp;

constexpr int kWave = 64;
constexpr int64_t kAgeCap = 1024;
constexpr int64_t kNeverMoved = -1024;

// FP64 -> bfloat16 bits, round to nearest even, for magnitudes in FP32's
// normal range (or zero).
__device__ __forceinline__ uint16_t d2bf(double d) {
  unsigned long long b = (unsigned long long)__double_as_longlong(d);
  b += 0xFFFFFFFFFFFull + ((b >> 45) & 1ull);
  b &= ~((1ull << 45) - 1ull);
  return f2bf((float)__longlong_as_double((long long)b));
}

// Order-preserving key of a finite score; never 0.
__device__ __forceinline__ uint32_t order_key(float y) {
  const uint32_t u = __float_as_uint(y);
  return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}

__device__ __forceinline__ double wsum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
  return v;
}

__device__ __forceinline__ bool active(const WalkState* st, const LearnState* ls) {
  return st->k < st->iters && !ls->idle;
}

__device__ __forceinline__ double position(double x, double l, double u) {
  if (!isfinite(l) || !isfinite(u)) return 0.5;
  if (u > l) return (x - l) / (u - l);
  return 0.0;
}

__device__ __forceinline__ double sign_of(double v) { return v > 0.0 ? 1.0 : (v < 0.0 ? -1.0 : 0.0); }

// The network inputs of column q in B layout (inputs 4g..4g+3 of this lane's
// group) at iteration k.
__device__ __forceinline__ bf16x4 assemble(const uint16_t* __restrict__ feat, int q, int g, int64_t k,
                                           int64_t k_last_full, int64_t V, int32_t mp) {
  const bf16x4 raw = *(const bf16x4*)(feat + (int64_t)q * 16 + 4 * g);
  if (g != 3) return raw;
  const int32_t last = (int32_t)(((uint32_t)(uint16_t)raw[1] << 16) | (uint32_t)(uint16_t)raw[0]);
  const int64_t age = min(k - (int64_t)last, kAgeCap);
  const int64_t since = min(k - k_last_full, (int64_t)64);
  bf16x4 x;
  x[0] = (short)d2bf((double)age / (double)kAgeCap);
  x[1] = (short)d2bf((double)since / 64.0);
  x[2] = (short)d2bf((double)V / (double)max(mp, 1));
  x[3] = raw[3];
  return x;
}

__device__ __forceinline__ void set_last_move(uint16_t* row, int32_t k) {
  row[12] = (uint16_t)((uint32_t)k & 0xFFFFu);
  row[13] = (uint16_t)((uint32_t)k >> 16);
}

// Static inputs and initial dynamic state of every column: never moved, or
// the given last-move iterations and move counts (original order).
__global__ __launch_bounds__(256) void k_learn_init(const WalkCtx* __restrict__ walks,
                                                    const LearnCtx* __restrict__ lc, int32_t n,
                                                    const int32_t* __restrict__ last_move,
                                                    const int32_t* __restrict__ moves) {
  const WalkCtx& C = walks[0];
  const LearnCtx& L = *lc;
  const DevProblem& P = C.P;
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= n) return;
  uint16_t* row = L.feat + (int64_t)q * 16;
  const double l = P.lb[q], u = P.ub[q];
  const bool isint = P.is_int[q] != 0;
  const bool isbin = isint && l == 0.0 && u == 1.0;
  const int deg = P.col_ptr[q + 1] - P.col_ptr[q];
  for (int t = 0; t < 16; ++t) row[t] = 0;
  row[1] = d2bf(log2(1.0 + (double)deg));
  row[2] = d2bf(L.c_max > 0.0 ? P.obj[q] / L.c_max : 0.0);
  row[4] = d2bf(isbin ? 1.0 : 0.0);
  row[5] = d2bf(isint && !isbin ? 1.0 : 0.0);
  row[6] = d2bf(isint ? 0.0 : 1.0);
  row[7] = d2bf(position(C.x[q], l, u));
  row[8] = d2bf((isfinite(l) && isfinite(u)) ? log2(1.0 + fmin(u - l, 1048576.0)) : 20.0);
  const int j = P.perm[q];
  const int32_t mv = moves ? moves[j] : 0;
  set_last_move(row, last_move ? last_move[j] : (int32_t)kNeverMoved);
  row[15] = d2bf(log2(1.0 + (double)mv));
  L.moves[q] = mv;
  L.xhat_last[q] = C.x[q];
}

// Row-aggregate inputs of every proposable column at the current point, one
// wavefront per column (fixed-order sums); also inputs 3, 7, 11 from the
// last full pass (s, xhat).
__global__ __launch_bounds__(256) void k_learn_refresh(const WalkCtx* __restrict__ walks,
                                                       const LearnCtx* __restrict__ lc) {
  const WalkCtx& C = walks[0];
  const LearnCtx& L = *lc;
  const DevProblem& P = C.P;
  if (!L.ls->train_active) return;
  const int lane = threadIdx.x & 63;
  const int64_t wstride = (int64_t)gridDim.x * (blockDim.x >> 6);
  const double eps = P.eps;
  for (int64_t idx = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6); idx < L.n_elig; idx += wstride) {
    const int q = L.elig_list[idx];
    double sw = 0.0, swv = 0.0, nv = 0.0, ne = 0.0, sa = 0.0, sav = 0.0;
    const int beg = P.col_ptr[q], end = P.col_ptr[q + 1];
    for (int e = beg + lane; e < end; e += kWave) {
      const RowState rs = C.rs[P.col_row[e]];
      const double a = fabs(P.col_val[e]);
      {
        const bool v = rs.r > eps;
        sw += (double)rs.w0;
        ne += 1.0;
        sa += a;
        if (v) {
          swv += (double)rs.w0;
          nv += 1.0;
          sav += a * fmin(rs.r, 1000.0);
        }
      }
      if (rs.w1 >= 0.0f) {
        const double r1 = -rs.r;
        const bool v = r1 > eps;
        sw += (double)rs.w1;
        ne += 1.0;
        sa += a;
        if (v) {
          swv += (double)rs.w1;
          nv += 1.0;
          sav += a * fmin(r1, 1000.0);
        }
      }
    }
    sw = wsum(sw);
    swv = wsum(swv);
    nv = wsum(nv);
    ne = wsum(ne);
    sa = wsum(sa);
    sav = wsum(sav);
    if (lane == 0) {
      uint16_t* row = L.feat + (int64_t)q * 16;
      const double x = C.x[q], xh = C.xhat[q];
      row[0] = d2bf(sw > 0.0 ? swv / sw : 0.0);
      row[3] = d2bf(sw > 0.0 ? fmin(fmax(C.s[q] / sw, -4.0), 4.0) : 0.0);
      row[7] = d2bf(position(x, P.lb[q], P.ub[q]));
      row[9] = d2bf(ne > 0.0 ? nv / ne : 0.0);
      row[10] = d2bf(sa > 0.0 ? sav / (1000.0 * sa) : 0.0);
      row[11] = d2bf(sign_of(xh - x));
      L.xhat_last[q] = xh;
    }
  }
}

// Start of a block of iterations (full evaluation first).
__global__ void k_learn_begin(const WalkCtx* __restrict__ walks, const LearnCtx* __restrict__ lc) {
  const WalkCtx& C = walks[0];
  LearnState* ls = lc->ls;
  if (threadIdx.x != 0) return;
  WalkState* st = C.st;
  st->skip = 0;
  if (st->k < st->iters) {
    ls->idle = 0;
    ls->train_active = 1;
    ls->k_last_full = st->k;
  } else {
    ls->idle = 1;
    ls->train_active = 0;
  }
}

__device__ __forceinline__ void flush_hist(uint32_t* lds, uint32_t* global) {
  __syncthreads();
  for (int b = threadIdx.x; b < kRadixBins; b += blockDim.x) {
    const uint32_t c = lds[b];
    if (c) atomicAdd(&global[b], c);
  }
}

// Network score key of every column plus the first-digit histogram.
__global__ __launch_bounds__(256) void k_learn_score(const WalkCtx* __restrict__ walks,
                                                     const LearnCtx* __restrict__ lc, const float* __restrict__ w,
                                                     const uint16_t* __restrict__ wb, int32_t n) {
  const WalkCtx& C = walks[0];
  const LearnCtx& L = *lc;
  const WalkState* st = C.st;
  if (!active(st, L.ls)) return;
  __shared__ uint32_t hist[kRadixBins];
  for (int b = threadIdx.x; b < kRadixBins; b += blockDim.x) hist[b] = 0;
  __syncthreads();
  Weights W;
  load_weights(wb, w, W);
  const int l = threadIdx.x & 63, g = l >> 4, r = l & 15;
  const int64_t k = st->k, klf = L.ls->k_last_full, V = st->V;
  const int ntiles = (n + 15) / 16;
  for (int tile = blockIdx.x * 4 + (threadIdx.x >> 6); tile < ntiles; tile += gridDim.x * 4) {
    const int q = tile * 16 + r;
    const bool valid = q < n;
    const bf16x4 zero = {0, 0, 0, 0};
    const bf16x4 x = valid ? assemble(L.feat, q, g, k, klf, V, L.mp) : zero;
    Acts A;
    forward(W, x, A);
    if (l < 16 && valid) {
      const uint32_t key = L.cls[q] != SUB_NONE ? order_key(A.y) : 0u;
      L.keys[0][q] = key;
      if (key) atomicAdd(&hist[key >> 21], 1u);
    }
  }
  flush_hist(hist, L.hist);
}

// Label keys (exact scores of the full pass) plus their first-digit histogram.
__global__ __launch_bounds__(256) void k_label_keys(const WalkCtx* __restrict__ walks,
                                                    const LearnCtx* __restrict__ lc, int32_t n) {
  const WalkCtx& C = walks[0];
  const LearnCtx& L = *lc;
  if (!active(C.st, L.ls)) return;
  __shared__ uint32_t hist[kRadixBins];
  for (int b = threadIdx.x; b < kRadixBins; b += blockDim.x) hist[b] = 0;
  __syncthreads();
  for (int q = blockIdx.x * blockDim.x + threadIdx.x; q < n; q += gridDim.x * blockDim.x) {
    const uint32_t key = L.cls[q] != SUB_NONE ? order_key((float)C.s[q]) : 0u;
    L.keys[1][q] = key;
    if (key) atomicAdd(&hist[key >> 21], 1u);
  }
  flush_hist(hist, L.hist + 3 * kRadixBins);
}

__device__ __forceinline__ uint32_t digit_of(uint32_t key, int level) {
  return level == 0 ? (key >> 21) : (level == 1 ? ((key >> 10) & 0x7FFu) : (key & 0x3FFu));
}

__device__ __forceinline__ uint32_t prefix_of(uint32_t key, int level) {
  return level == 1 ? (key >> 21) : (key >> 10);
}

// One digit of the radix select, one wavefront: the digit whose bin holds
// the remaining K-th largest key. Clears the histogram it read.
__global__ void k_topk_digit(const WalkCtx* __restrict__ walks, const LearnCtx* __restrict__ lc, int32_t which,
                             int32_t level) {
  const WalkCtx& C = walks[0];
  const LearnCtx& L = *lc;
  if (!active(C.st, L.ls)) return;
  TopkState& T = L.ls->tk[which];
  uint32_t* hist = L.hist + (which * 3 + level) * kRadixBins;
  const int lane = threadIdx.x;
  const int per = kRadixBins / kWave;  // 32 bins per lane, lane 0 the highest
  if (level == 0) {
    // first digit: the state starts here
    if (lane == 0) {
      T.prefix = 0;
      T.remaining = L.K[which];
      T.done = 0;
      T.thresh = 0;
      T.need_eq = 0;
    }
  }
  __syncthreads();
  const int rem = T.remaining;
  const bool done = T.done != 0;
  uint32_t c[32];
  uint32_t part = 0;
  for (int t = 0; t < per; ++t) {
    c[t] = hist[kRadixBins - 1 - (lane * per + t)];
    part += c[t];
  }
  // inclusive prefix over lanes (highest bins first)
  uint32_t inc = part;
#pragma unroll
  for (int o = 1; o < kWave; o <<= 1) {
    const uint32_t y = __shfl_up(inc, o, kWave);
    if (lane >= o) inc += y;
  }
  const uint32_t total = __shfl(inc, kWave - 1, kWave);
  __syncthreads();
  for (int t = 0; t < per; ++t) hist[kRadixBins - 1 - (lane * per + t)] = 0;
  if (done) return;
  if (level == 0 && total < (uint32_t)rem) {
    // fewer proposable columns than K: take every nonzero key
    if (lane == 0) {
      T.thresh = 0;
      T.need_eq = 0;
      T.done = 1;
    }
    return;
  }
  const uint32_t before = inc - part;
  const bool mine = before < (uint32_t)rem && inc >= (uint32_t)rem;
  if (mine) {
    uint32_t cum = before;
    int d = 0;
    for (int t = 0; t < per; ++t) {
      if (cum + c[t] >= (uint32_t)rem) {
        d = kRadixBins - 1 - (lane * per + t);
        break;
      }
      cum += c[t];
    }
    const int left = rem - (int)cum;
    const int bits = (level == 2) ? 10 : 11;
    const uint32_t pre = (level == 0) ? (uint32_t)d : ((T.prefix << bits) | (uint32_t)d);
    T.prefix = pre;
    T.remaining = left;
    if (level == 2) {
      T.thresh = pre;
      T.need_eq = left;
      T.done = 1;
    }
  }
}

// Histogram of the next digit over keys that match the chosen prefix.
__global__ __launch_bounds__(256) void k_topk_hist(const WalkCtx* __restrict__ walks, const LearnCtx* __restrict__ lc,
                                                   int32_t which, int32_t level, int32_t n) {
  const WalkCtx& C = walks[0];
  const LearnCtx& L = *lc;
  if (!active(C.st, L.ls)) return;
  const TopkState& T = L.ls->tk[which];
  if (T.done) return;
  __shared__ uint32_t hist[kRadixBins];
  for (int b = threadIdx.x; b < kRadixBins; b += blockDim.x) hist[b] = 0;
  __syncthreads();
  const uint32_t pre = T.prefix;
  const uint32_t* keys = L.keys[which];
  for (int q = blockIdx.x * blockDim.x + threadIdx.x; q < n; q += gridDim.x * blockDim.x) {
    const uint32_t key = keys[q];
    if (key && prefix_of(key, level) == pre) atomicAdd(&hist[digit_of(key, level)], 1u);
  }
  flush_hist(hist, L.hist + (which * 3 + level) * kRadixBins);
}

__device__ __forceinline__ bool above(uint32_t key, uint32_t thresh) { return key != 0u && key > thresh; }

// Per-workgroup counts of keys above and equal to the threshold.
__global__ __launch_bounds__(256) void k_topk_count(const WalkCtx* __restrict__ walks,
                                                    const LearnCtx* __restrict__ lc, int32_t which, int32_t n) {
  const WalkCtx& C = walks[0];
  const LearnCtx& L = *lc;
  if (!active(C.st, L.ls)) return;
  __shared__ int red[8];
  const TopkState& T = L.ls->tk[which];
  const uint32_t th = T.thresh;
  const uint32_t* keys = L.keys[which];
  int gt = 0, eq = 0;
  const int beg = blockIdx.x * kTopkChunk;
  const int end = min(n, beg + kTopkChunk);
  for (int q = beg + threadIdx.x; q < end; q += blockDim.x) {
    const uint32_t key = keys[q];
    gt += above(key, th) ? 1 : 0;
    eq += (th != 0u && key == th) ? 1 : 0;
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    gt += __shfl_xor(gt, o, kWave);
    eq += __shfl_xor(eq, o, kWave);
  }
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  if (lane == 0) {
    red[2 * wv] = gt;
    red[2 * wv + 1] = eq;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    int a = 0, b = 0;
    for (int k = 0; k < 4; ++k) {
      a += red[2 * k];
      b += red[2 * k + 1];
    }
    int32_t* cnt = L.wg_cnt + (int64_t)which * L.nwg * 2;
    cnt[2 * blockIdx.x] = a;
    cnt[2 * blockIdx.x + 1] = b;
  }
}

// Exclusive prefix of the per-workgroup counts (one workgroup).
__global__ __launch_bounds__(256) void k_topk_scan(const WalkCtx* __restrict__ walks, const LearnCtx* __restrict__ lc,
                                                   int32_t which) {
  const WalkCtx& C = walks[0];
  const LearnCtx& L = *lc;
  if (!active(C.st, L.ls)) return;
  if (threadIdx.x != 0) return;
  TopkState& T = L.ls->tk[which];
  const int32_t* cnt = L.wg_cnt + (int64_t)which * L.nwg * 2;
  int32_t* base = L.wg_base + (int64_t)which * L.nwg * 2;
  int gt = 0, eq = 0;
  for (int b = 0; b < L.nwg; ++b) {
    base[2 * b] = gt;
    base[2 * b + 1] = eq;
    gt += cnt[2 * b];
    eq += cnt[2 * b + 1];
  }
  T.count = gt + min(eq, T.need_eq);
}

// Order-preserving compaction of the selected columns.
__global__ __launch_bounds__(256) void k_topk_write(const WalkCtx* __restrict__ walks,
                                                    const LearnCtx* __restrict__ lc, int32_t which, int32_t n) {
  const WalkCtx& C = walks[0];
  const LearnCtx& L = *lc;
  if (!active(C.st, L.ls)) return;
  __shared__ int sg[4], se[4];
  const TopkState& T = L.ls->tk[which];
  const uint32_t th = T.thresh;
  const int need = T.need_eq;
  const uint32_t* keys = L.keys[which];
  const int32_t* base = L.wg_base + (int64_t)which * L.nwg * 2;
  const int gt_base = base[2 * blockIdx.x], eq_base = base[2 * blockIdx.x + 1];
  constexpr int per = kTopkChunk / 256;
  const int beg = blockIdx.x * kTopkChunk + threadIdx.x * per;
  int gt = 0, eq = 0;
  for (int t = 0; t < per; ++t) {
    const int q = beg + t;
    if (q >= n) break;
    const uint32_t key = keys[q];
    gt += above(key, th) ? 1 : 0;
    eq += (th != 0u && key == th) ? 1 : 0;
  }
  // exclusive scans over the workgroup's threads
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  int ig = gt, ie = eq;
#pragma unroll
  for (int o = 1; o < kWave; o <<= 1) {
    const int yg = __shfl_up(ig, o, kWave), ye = __shfl_up(ie, o, kWave);
    if (lane >= o) {
      ig += yg;
      ie += ye;
    }
  }
  if (lane == 63) {
    sg[wv] = ig;
    se[wv] = ie;
  }
  __syncthreads();
  int og = ig - gt, oe = ie - eq;
  for (int k = 0; k < wv; ++k) {
    og += sg[k];
    oe += se[k];
  }
  int eq_rank = eq_base + oe;  // equal keys before this thread's run
  int pos = gt_base + og + min(eq_rank, need);
  int32_t* out = L.sel[which];
  for (int t = 0; t < per; ++t) {
    const int q = beg + t;
    if (q >= n) break;
    const uint32_t key = keys[q];
    bool take = above(key, th);
    if (th != 0u && key == th) {
      take = eq_rank < need;
      ++eq_rank;
    }
    if (take) out[pos++] = q;
  }
}

// Materialised training inputs and targets of a full evaluation: the top T
// columns by exact score and T random proposable columns; target =
// max(s, 0) / max_j s_j (0 when no score is positive). Also appends them to
// the pair log. One workgroup.
__global__ __launch_bounds__(256) void k_learn_pairs(const WalkCtx* __restrict__ walks,
                                                     const LearnCtx* __restrict__ lc) {
  const WalkCtx& C = walks[0];
  const LearnCtx& L = *lc;
  const WalkState* st = C.st;
  if (!active(st, L.ls)) return;
  __shared__ double red[4];
  const int T2 = 2 * L.T;
  const int cnt = L.ls->tk[1].count;
  const int64_t ev = L.ls->evals;
  double smax = 0.0;
  for (int i = threadIdx.x; i < cnt; i += blockDim.x) smax = fmax(smax, C.s[L.sel[1][i]]);
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) smax = fmax(smax, __shfl_xor(smax, o, kWave));
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  if (lane == 0) red[wv] = smax;
  __syncthreads();
  smax = fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
  const int64_t k = st->k, klf = L.ls->k_last_full, V = st->V;
  const int64_t logged = L.ls->logged;
  const bool log = L.log_feat != nullptr && logged + T2 <= L.log_cap;
  for (int i = threadIdx.x; i < T2; i += blockDim.x) {
    int q;
    if (i < L.T && i < cnt)
      q = L.sel[1][i];
    else
      q = L.elig_list[splitmix64(L.seed, (uint64_t)(ev * T2 + i)) % (uint64_t)L.n_elig];
    const double tgt = smax > 0.0 ? fmax(C.s[q], 0.0) / smax : 0.0;
    L.pair_tgt[i] = (float)tgt;
    if (log) L.log_tgt[logged + i] = (float)tgt;
    for (int gg = 0; gg < 4; ++gg) {
      const bf16x4 x = assemble(L.feat, q, gg, k, klf, V, L.mp);
      for (int t = 0; t < 4; ++t) {
        L.pair_feat[(int64_t)i * 16 + 4 * gg + t] = (uint16_t)x[t];
        if (log) L.log_feat[(logged + i) * 16 + 4 * gg + t] = (uint16_t)x[t];
      }
    }
  }
  __syncthreads();
  if (threadIdx.x == 0 && log) L.ls->logged = logged + T2;
}

// Judge of a full evaluation: was its move in the network's proposal set?
__global__ void k_learn_judge(const WalkCtx* __restrict__ walks, const LearnCtx* __restrict__ lc) {
  const WalkCtx& C = walks[0];
  const LearnCtx& L = *lc;
  const WalkState* st = C.st;
  if (threadIdx.x != 0 || st->k >= st->iters) return;
  LearnState* ls = L.ls;
  ls->evals += 1;
  const int q = st->mv_j;
  if (q < 0) return;
  const int32_t* set = L.sel[0];
  int lo = 0, hi = ls->tk[0].count - 1;
  while (lo <= hi) {
    const int mid = (lo + hi) >> 1;
    if (set[mid] == q) {
      ls->hits += 1;
      return;
    }
    if (set[mid] < q)
      lo = mid + 1;
    else
      hi = mid - 1;
  }
}

// Pending incumbent copy of a proposal iteration (the full pass does it in
// its argmax kernel).
__global__ __launch_bounds__(256) void k_learn_copy_best(const WalkCtx* __restrict__ walks,
                                                         const LearnCtx* __restrict__ lc, int32_t n) {
  const WalkCtx& C = walks[0];
  if (!active(C.st, lc->ls) || !C.st->copy_best) return;
  for (int q = blockIdx.x * blockDim.x + threadIdx.x; q < n; q += gridDim.x * blockDim.x) C.best_x[q] = C.x[q];
}

// Appends the proposal set (original indices) to the set log; a full
// evaluation records an empty range.
__global__ __launch_bounds__(256) void k_learn_log_set(const WalkCtx* __restrict__ walks,
                                                       const LearnCtx* __restrict__ lc, int32_t full) {
  const WalkCtx& C = walks[0];
  const LearnCtx& L = *lc;
  const WalkState* st = C.st;
  if (!active(st, L.ls) || L.set_off == nullptr) return;
  const int64_t k = st->k;
  const int64_t pos = L.ls->set_pos;
  const int cnt = full ? 0 : L.ls->tk[0].count;
  const bool fits = pos + cnt <= L.set_log_cap;
  if (fits)
    for (int i = threadIdx.x; i < cnt; i += blockDim.x) L.set_log[pos + i] = C.P.perm[L.sel[0][i]];
  __syncthreads();
  if (threadIdx.x == 0) {
    const int64_t end = fits ? pos + cnt : pos;
    L.set_off[k] = pos;
    L.set_off[k + 1] = end;
    L.ls->set_pos = end;
  }
}

// Stored-row updates for the moved column (before k_finish advances k).
__global__ void k_learn_move(const WalkCtx* __restrict__ walks, const LearnCtx* __restrict__ lc) {
  const WalkCtx& C = walks[0];
  const LearnCtx& L = *lc;
  const WalkState* st = C.st;
  if (threadIdx.x != 0 || st->k >= st->iters || st->skip) return;
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

// All 16 inputs of every column in original order (zeros for columns that
// are never proposed).
__global__ __launch_bounds__(256) void k_learn_features_out(const WalkCtx* __restrict__ walks,
                                                            const LearnCtx* __restrict__ lc, int32_t n, int64_t k,
                                                            int64_t k_last_full, uint16_t* __restrict__ out) {
  const WalkCtx& C = walks[0];
  const LearnCtx& L = *lc;
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= n) return;
  uint16_t* o = out + (int64_t)C.P.perm[q] * 16;
  const bool ok = L.cls[q] != SUB_NONE;
  for (int gg = 0; gg < 4; ++gg) {
    const bf16x4 x = assemble(L.feat, q, gg, k, k_last_full, C.st->V, L.mp);
    for (int t = 0; t < 4; ++t) o[4 * gg + t] = ok ? (uint16_t)x[t] : 0;
  }
}

inline int grid_for(int64_t work, int per_block, int cap) {
  int64_t b = (work + per_block - 1) / per_block;
  return (int)std::max<int64_t>(1, std::min<int64_t>(b, cap));
}

hipError_t topk(const WalkCtx* C, const LearnCtx* L, const LearnCtx& Lh, int which, int32_t n, hipStream_t s) {
  const int hb = grid_for(n, 256 * 16, 1024);
  hipLaunchKernelGGL(k_topk_digit, dim3(1), dim3(64), 0, s, C, L, which, 0);
  hipLaunchKernelGGL(k_topk_hist, dim3(hb), dim3(256), 0, s, C, L, which, 1, n);
  hipLaunchKernelGGL(k_topk_digit, dim3(1), dim3(64), 0, s, C, L, which, 1);
  hipLaunchKernelGGL(k_topk_hist, dim3(hb), dim3(256), 0, s, C, L, which, 2, n);
  hipLaunchKernelGGL(k_topk_digit, dim3(1), dim3(64), 0, s, C, L, which, 2);
  hipLaunchKernelGGL(k_topk_count, dim3(Lh.nwg), dim3(256), 0, s, C, L, which, n);
  hipLaunchKernelGGL(k_topk_scan, dim3(1), dim3(64), 0, s, C, L, which);
  hipLaunchKernelGGL(k_topk_write, dim3(Lh.nwg), dim3(256), 0, s, C, L, which, n);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_learn_init(const WalkCtx* C, const LearnCtx* L, const LearnCtx& Lh, int32_t n,
                             const int32_t* last_move, const int32_t* moves, hipStream_t s) {
  if (n > 0) hipLaunchKernelGGL(k_learn_init, dim3((n + 255) / 256), dim3(256), 0, s, C, L, n, last_move, moves);
  return hipGetLastError();
}

hipError_t launch_learn_refresh(const WalkCtx* C, const LearnCtx* L, const LearnCtx& Lh, hipStream_t s) {
  if (Lh.n_elig > 0)
    hipLaunchKernelGGL(k_learn_refresh, dim3(grid_for(Lh.n_elig, 4, 8192)), dim3(256), 0, s, C, L);
  return hipGetLastError();
}

hipError_t launch_learn_begin(const WalkCtx* C, const LearnCtx* L, hipStream_t s) {
  hipLaunchKernelGGL(k_learn_begin, dim3(1), dim3(64), 0, s, C, L);
  return hipGetLastError();
}

hipError_t launch_learn_propose(const WalkCtx* C, const LearnCtx* L, const LearnCtx& Lh, const ModelDev& M,
                                int32_t n, int full_iteration, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_learn_score, dim3(grid_for(n, 64, 2048)), dim3(256), 0, s, C, L, M.w, M.wb, n);
  hipError_t e = topk(C, L, Lh, 0, n, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_learn_log_set, dim3(1), dim3(256), 0, s, C, L, (int32_t)full_iteration);
  return hipGetLastError();
}

hipError_t launch_learn_train(const WalkCtx* C, const LearnCtx* L, const LearnCtx& Lh, const ModelDev& M,
                              int32_t n, int32_t steps, float lr, hipStream_t s) {
  if (n <= 0 || (steps <= 0 && Lh.log_feat == nullptr)) return hipSuccess;
  hipLaunchKernelGGL(k_label_keys, dim3(grid_for(n, 256 * 16, 1024)), dim3(256), 0, s, C, L, n);
  hipError_t e = topk(C, L, Lh, 1, n, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_learn_pairs, dim3(1), dim3(256), 0, s, C, L);
  for (int32_t t = 0; t < steps; ++t) {
    e = launch_mlp_grad_guarded(M, &Lh.ls->train_active, Lh.pair_feat, Lh.pair_tgt, 2 * (int64_t)Lh.T, s);
    if (e != hipSuccess) return e;
    e = launch_mlp_reduce_guarded(M, &Lh.ls->train_active, 2 * (int64_t)Lh.T, lr, s);
    if (e != hipSuccess) return e;
  }
  return hipGetLastError();
}

hipError_t launch_learn_judge(const WalkCtx* C, const LearnCtx* L, hipStream_t s) {
  hipLaunchKernelGGL(k_learn_judge, dim3(1), dim3(64), 0, s, C, L);
  return hipGetLastError();
}

hipError_t launch_learn_copy_best(const WalkCtx* C, const LearnCtx* L, int32_t n, hipStream_t s) {
  hipLaunchKernelGGL(k_learn_copy_best, dim3(grid_for(n, 256, 256)), dim3(256), 0, s, C, L, n);
  return hipGetLastError();
}

hipError_t launch_learn_move(const WalkCtx* C, const LearnCtx* L, hipStream_t s) {
  hipLaunchKernelGGL(k_learn_move, dim3(1), dim3(64), 0, s, C, L);
  return hipGetLastError();
}

hipError_t launch_learn_features_out(const WalkCtx* C, const LearnCtx* L, int32_t n, int64_t k, int64_t k_last_full,
                                     uint16_t* out, hipStream_t s) {
  if (n > 0)
    hipLaunchKernelGGL(k_learn_features_out, dim3((n + 255) / 256), dim3(256), 0, s, C, L, n, k, k_last_full, out);
  return hipGetLastError();
}

}  // namespace chap
