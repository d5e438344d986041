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
// internal index (equal keys: lowest index first). Each kernel of the select
// re-derives the digits chosen so far from the histograms of the earlier
// kernels (a few kilobytes from L2), so no single-workgroup kernel sits
// between them.

#include <climits>
#include <cmath>

#include "chap_internal.h"
#include "learned_rows.h"
#include "mlp_core.h"

namespace chap {
namespace {

using namespace mlp;
using namespace learned;

constexpr int kBlock = 256;

// Order-preserving key of a finite score; never 0.
__device__ __forceinline__ uint32_t order_key(float y) {
  const uint32_t u = __float_as_uint(y);
  return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}

__device__ __forceinline__ bool active(const WalkState* st, const LearnState* ls) {
  return st->k < st->iters && !ls->idle;
}

// Inputs 13 and 14, the same for every column at one iteration.
struct Globals {
  short since;  // bfloat16 bits of min(k - k_last_full, 64) / 64
  short vfrac;  // bfloat16 bits of V / m'
};

__device__ __forceinline__ Globals globals(int64_t k, int64_t k_last_full, int64_t V, int32_t mp) {
  Globals G;
  G.since = (short)d2bf((double)min(k - k_last_full, (int64_t)64) / 64.0);
  G.vfrac = (short)d2bf((double)V / (double)max(mp, 1));
  return G;
}

// The network inputs of column q in B layout (inputs 4g..4g+3 of this lane's
// group) at iteration k. The tabu age min(k - last, 1024) / 1024 is a
// multiple of 2^-10 in [0, 1], exact in FP64 before its single rounding.
__device__ __forceinline__ bf16x4 assemble(const uint16_t* __restrict__ feat, int q, int g, int64_t k,
                                           const Globals& G) {
  const bf16x4 raw = *(const bf16x4*)(feat + (int64_t)q * 16 + 4 * g);
  if (g != 3) return raw;
  const int32_t last = (int32_t)(((uint32_t)(uint16_t)raw[1] << 16) | (uint32_t)(uint16_t)raw[0]);
  const int64_t age = min(k - (int64_t)last, kAgeCap);
  bf16x4 x;
  x[0] = (short)d2bf((double)age * (1.0 / (double)kAgeCap));
  x[1] = G.since;
  x[2] = G.vfrac;
  x[3] = raw[3];
  return x;
}

// ---------------------------------------------------------------------------
// Stored rows
// ---------------------------------------------------------------------------

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
  set_last_move(row, last_move ? last_move[j] : kNeverMoved);
  row[15] = d2bf(log2(1.0 + (double)mv));
  L.moves[q] = mv;
  L.xhat_last[q] = C.x[q];
}

// Contributions of stored entry e to the six refresh sums.
__device__ __forceinline__ void refresh_entry(const DevProblem& P, const RowState* rs, int e, double* v) {
  const RowState r = rs[P.col_row[e]];
  const double a = fabs(P.col_val[e]);
  const double eps = P.eps;
  v[0] += (double)r.w0;
  v[3] += 1.0;
  v[4] += a;
  if (r.r > eps) {
    v[1] += (double)r.w0;
    v[2] += 1.0;
    v[5] += a * fmin(r.r, 1000.0);
  }
  if (r.w1 >= 0.0f) {
    const double r1 = -r.r;
    v[0] += (double)r.w1;
    v[3] += 1.0;
    v[4] += a;
    if (r1 > eps) {
      v[1] += (double)r.w1;
      v[2] += 1.0;
      v[5] += a * fmin(r1, 1000.0);
    }
  }
}

// Inputs 0, 3, 7, 9, 10, 11 of column q from its six sums; xhat_last := xhat.
__device__ __forceinline__ void refresh_write(const WalkCtx& C, const LearnCtx& L, int q, const double* v) {
  uint16_t* row = L.feat + (int64_t)q * 16;
  const double sw = v[0], swv = v[1], nv = v[2], ne = v[3], sa = v[4], sav = v[5];
  const double x = C.x[q], xh = C.xhat[q];
  row[0] = d2bf(sw > 0.0 ? swv / sw : 0.0);
  row[3] = d2bf(sw > 0.0 ? fmin(fmax(C.s[q] / sw, -4.0), 4.0) : 0.0);
  row[7] = d2bf(position(x, C.P.lb[q], C.P.ub[q]));
  row[9] = d2bf(ne > 0.0 ? nv / ne : 0.0);
  row[10] = d2bf(sa > 0.0 ? sav / (1000.0 * sa) : 0.0);
  row[11] = d2bf(sign_of(xh - x));
  L.xhat_last[q] = xh;
}

// Short proposable columns: eight lanes per column, fixed-order sums.
__global__ __launch_bounds__(256) void k_refresh_short(const WalkCtx* __restrict__ walks,
                                                       const LearnCtx* __restrict__ lc) {
  const WalkCtx& C = walks[0];
  const LearnCtx& L = *lc;
  if (!L.ls->train_active) return;
  const int sub = threadIdx.x & 7;
  const int64_t groups = (int64_t)gridDim.x * (blockDim.x >> 3);
  for (int64_t idx = (int64_t)blockIdx.x * (blockDim.x >> 3) + (threadIdx.x >> 3); idx < L.n_ref_short;
       idx += groups) {
    const int q = L.ref_short[idx];
    double v[6] = {0, 0, 0, 0, 0, 0};
    for (int e = C.P.col_ptr[q] + sub; e < C.P.col_ptr[q + 1]; e += 8) refresh_entry(C.P, C.rs, e, v);
#pragma unroll
    for (int t = 0; t < 6; ++t)
#pragma unroll
      for (int o = 1; o < 8; o <<= 1) v[t] += __shfl_xor(v[t], o, kWave);
    if (sub == 0) refresh_write(C, L, q, v);
  }
}

__device__ __forceinline__ double block_sum(double v, double* red) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  double t = 0.0;
  for (int w = 0; w < (int)(blockDim.x >> 6); ++w) t += red[w];
  return t;
}

// Chunks of long proposable columns: one workgroup per chunk (grid-stride),
// partial sums per chunk.
__global__ __launch_bounds__(256) void k_refresh_chunks(const WalkCtx* __restrict__ walks,
                                                        const LearnCtx* __restrict__ lc) {
  const WalkCtx& C = walks[0];
  const LearnCtx& L = *lc;
  if (!L.ls->train_active) return;
  __shared__ double red[4];
  for (int t = blockIdx.x; t < L.n_ref_chunks; t += gridDim.x) {
    const ChunkTask T = L.ref_chunks[t];
    double v[6] = {0, 0, 0, 0, 0, 0};
    for (int e = T.e_beg + threadIdx.x; e < T.e_end; e += blockDim.x) refresh_entry(C.P, C.rs, e, v);
    double out[6];
    for (int k = 0; k < 6; ++k) out[k] = block_sum(v[k], red);
    if (threadIdx.x == 0)
      for (int k = 0; k < 6; ++k) L.ref_parts[T.slot].v[k] = out[k];
  }
}

// Long proposable columns: sums of their chunks in order.
__global__ __launch_bounds__(256) void k_refresh_combine(const WalkCtx* __restrict__ walks,
                                                         const LearnCtx* __restrict__ lc) {
  const WalkCtx& C = walks[0];
  const LearnCtx& L = *lc;
  if (!L.ls->train_active) return;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= L.n_ref_cols) return;
  const ChunkCol cc = L.ref_cols[i];
  double v[6] = {0, 0, 0, 0, 0, 0};
  for (int k = 0; k < cc.nparts; ++k)
    for (int t = 0; t < 6; ++t) v[t] += L.ref_parts[cc.first + k].v[t];
  refresh_write(C, L, cc.col, v);
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

// ---------------------------------------------------------------------------
// Radix top-K
// ---------------------------------------------------------------------------

struct Select {
  bool all;          // at most K nonzero keys: take every nonzero key
  uint32_t prefix;   // digits chosen so far (levels below `upto`)
  int rem;           // keys still to take under the prefix
  uint32_t thresh;   // final key T (upto == 3)
  int need_eq;       // keys == T to take (upto == 3)
  int count;         // keys selected (upto == 3 or all)
};

// Whole workgroup (256 threads): the bin of histogram h (bins from the top)
// that holds the rem-th largest key; *left = rank of that key inside the bin.
__device__ void find_digit(const uint32_t* __restrict__ h, int rem, int* digit, int* left, uint32_t* total) {
  __shared__ uint32_t part[kBlock / kWave];
  __shared__ int res[2];
  constexpr int per = kRadixBins / kBlock;  // 8 bins per thread, thread 0 the highest
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  uint32_t c[per];
  uint32_t sum = 0;
#pragma unroll
  for (int t = 0; t < per; ++t) {
    c[t] = h[kRadixBins - 1 - (tid * per + t)];
    sum += c[t];
  }
  uint32_t inc = sum;
#pragma unroll
  for (int o = 1; o < kWave; o <<= 1) {
    const uint32_t y = __shfl_up(inc, o, kWave);
    if (lane >= o) inc += y;
  }
  __syncthreads();
  if (lane == kWave - 1) part[wv] = inc;
  if (tid == 0) {
    res[0] = 0;
    res[1] = 0;
  }
  __syncthreads();
  uint32_t before_w = 0, all = 0;
  for (int w = 0; w < kBlock / kWave; ++w) {
    if (w < wv) before_w += part[w];
    all += part[w];
  }
  const uint32_t hi = before_w + inc, lo = hi - sum;
  if (lo < (uint32_t)rem && hi >= (uint32_t)rem) {
    uint32_t cum = lo;
#pragma unroll
    for (int t = 0; t < per; ++t) {
      if (cum < (uint32_t)rem && cum + c[t] >= (uint32_t)rem) {
        res[0] = kRadixBins - 1 - (tid * per + t);
        res[1] = rem - (int)cum;
      }
      cum += c[t];
    }
  }
  __syncthreads();
  *digit = res[0];
  *left = res[1];
  *total = all;
  __syncthreads();
}

// Digits of levels < upto (upto = 3: the final threshold) from the
// histograms of the earlier kernels. Whole workgroup.
__device__ Select derive(const LearnCtx& L, int which, int upto) {
  const uint32_t* H = L.hist + which * 3 * kRadixBins;
  const int K = L.K[which];
  Select S{false, 0u, K, 0u, 0, 0};
  int d, left;
  uint32_t total;
  find_digit(H, K, &d, &left, &total);
  if (total <= (uint32_t)K) {
    S.all = true;
    S.count = (int)total;
    return S;
  }
  S.prefix = (uint32_t)d;
  S.rem = left;
  if (upto >= 2) {
    find_digit(H + kRadixBins, S.rem, &d, &left, &total);
    S.prefix = (S.prefix << 11) | (uint32_t)d;
    S.rem = left;
  }
  if (upto >= 3) {
    find_digit(H + 2 * kRadixBins, S.rem, &d, &left, &total);
    S.thresh = (S.prefix << 10) | (uint32_t)d;
    S.need_eq = left;
    S.count = K;
  }
  return S;
}

__device__ __forceinline__ void flush_hist(uint32_t* lds, uint32_t* global) {
  __syncthreads();
  for (int b = threadIdx.x; b < kRadixBins; b += blockDim.x) {
    const uint32_t c = lds[b];
    if (c) atomicAdd(&global[b], c);
  }
}

// Network score key of every column plus the first-digit histogram; also the
// pending incumbent copy (before this iteration's move changes x).
__global__ __launch_bounds__(256) void k_learn_score(const WalkCtx* __restrict__ walks,
                                                     const LearnCtx* __restrict__ lc, const float* __restrict__ w,
                                                     const uint16_t* __restrict__ wb, int32_t n) {
  const WalkCtx& C = walks[0];
  const LearnCtx& L = *lc;
  const WalkState* st = C.st;
  if (!active(st, L.ls)) return;
  __shared__ uint32_t hist[kRadixBins];
  for (int b = threadIdx.x; b < kRadixBins; b += blockDim.x) hist[b] = 0;
  if (st->copy_best)
    for (int q = blockIdx.x * blockDim.x + threadIdx.x; q < n; q += gridDim.x * blockDim.x) C.best_x[q] = C.x[q];
  __syncthreads();
  Weights W;
  load_weights(wb, w, W);
  const int l = threadIdx.x & 63, g = l >> 4, r = l & 15;
  const int64_t k = st->k;
  const Globals Gl = globals(k, L.ls->k_last_full, st->V, L.mp);
  const int ntiles = (n + 15) / 16;
  const int stride = gridDim.x * 4;
  const bf16x4 zero = {0, 0, 0, 0};
  // a ring of kScoreDepth tiles per wavefront: the inputs of the tile
  // kScoreDepth steps ahead are loaded while the current one is computed
  constexpr int kScoreDepth = 8;
  const int tile0 = blockIdx.x * 4 + (threadIdx.x >> 6);
  bf16x4 ring[kScoreDepth];
#pragma unroll
  for (int d = 0; d < kScoreDepth; ++d) {
    const int t = tile0 + d * stride;
    ring[d] = (t < ntiles && t * 16 + r < n) ? assemble(L.feat, t * 16 + r, g, k, Gl) : zero;
  }
  for (int base = tile0; base < ntiles; base += kScoreDepth * stride) {
#pragma unroll
    for (int d = 0; d < kScoreDepth; ++d) {
      const int t = base + d * stride;
      if (t >= ntiles) break;
      const bf16x4 x = ring[d];
      const int tn = t + kScoreDepth * stride;
      ring[d] = (tn < ntiles && tn * 16 + r < n) ? assemble(L.feat, tn * 16 + r, g, k, Gl) : zero;
      Acts A;
      forward(W, x, A);
      const int q = t * 16 + r;
      if (l < 16 && q < n) {
        const uint32_t key = L.cls[q] != SUB_NONE ? order_key(A.y) : 0u;
        L.keys[0][q] = key;
        if (key) atomicAdd(&hist[key >> 21], 1u);
      }
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
  return level == 1 ? ((key >> 10) & 0x7FFu) : (key & 0x3FFu);
}

__device__ __forceinline__ uint32_t prefix_of(uint32_t key, int level) {
  return level == 1 ? (key >> 21) : (key >> 10);
}

// Histogram of digit `level` (1 or 2) over keys that match the digits above.
__global__ __launch_bounds__(256) void k_topk_hist(const WalkCtx* __restrict__ walks, const LearnCtx* __restrict__ lc,
                                                   int32_t which, int32_t level, int32_t n) {
  const WalkCtx& C = walks[0];
  const LearnCtx& L = *lc;
  if (!active(C.st, L.ls)) return;
  const Select S = derive(L, which, level);
  if (S.all) return;
  __shared__ uint32_t hist[kRadixBins];
  for (int b = threadIdx.x; b < kRadixBins; b += blockDim.x) hist[b] = 0;
  __syncthreads();
  const uint32_t* keys = L.keys[which];
  for (int q = blockIdx.x * blockDim.x + threadIdx.x; q < n; q += gridDim.x * blockDim.x) {
    const uint32_t key = keys[q];
    if (key && prefix_of(key, level) == S.prefix) atomicAdd(&hist[digit_of(key, level)], 1u);
  }
  flush_hist(hist, L.hist + (which * 3 + level) * kRadixBins);
}

__device__ __forceinline__ bool take_above(uint32_t key, const Select& S) {
  return key != 0u && (S.all || key > S.thresh);
}

__device__ __forceinline__ bool take_equal(uint32_t key, const Select& S) {
  return !S.all && key == S.thresh;
}

// Per-workgroup counts of keys above and equal to the threshold.
__global__ __launch_bounds__(256) void k_topk_count(const WalkCtx* __restrict__ walks,
                                                    const LearnCtx* __restrict__ lc, int32_t which, int32_t n) {
  const WalkCtx& C = walks[0];
  const LearnCtx& L = *lc;
  if (!active(C.st, L.ls)) return;
  const Select S = derive(L, which, 3);
  __shared__ int red[8];
  const uint32_t* keys = L.keys[which];
  int gt = 0, eq = 0;
  const int beg = blockIdx.x * kTopkChunk;
  const int end = min(n, beg + kTopkChunk);
  for (int q = beg + threadIdx.x; q < end; q += blockDim.x) {
    const uint32_t key = keys[q];
    gt += take_above(key, S) ? 1 : 0;
    eq += take_equal(key, S) ? 1 : 0;
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

// Order-preserving compaction of the selected columns; each workgroup sums
// the counts of the workgroups before it.
__global__ __launch_bounds__(256) void k_topk_write(const WalkCtx* __restrict__ walks,
                                                    const LearnCtx* __restrict__ lc, int32_t which, int32_t n) {
  const WalkCtx& C = walks[0];
  const LearnCtx& L = *lc;
  if (!active(C.st, L.ls)) return;
  const Select S = derive(L, which, 3);
  __shared__ int sg[4], se[4];
  const uint32_t* keys = L.keys[which];
  const int32_t* cnt = L.wg_cnt + (int64_t)which * L.nwg * 2;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  int bg = 0, be = 0;
  for (int b = threadIdx.x; b < (int)blockIdx.x; b += blockDim.x) {
    bg += cnt[2 * b];
    be += cnt[2 * b + 1];
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    bg += __shfl_xor(bg, o, kWave);
    be += __shfl_xor(be, o, kWave);
  }
  if (lane == 0) {
    sg[wv] = bg;
    se[wv] = be;
  }
  __syncthreads();
  const int gt_base = sg[0] + sg[1] + sg[2] + sg[3];
  const int eq_base = se[0] + se[1] + se[2] + se[3];
  __syncthreads();
  constexpr int per = kTopkChunk / kBlock;
  const int beg = blockIdx.x * kTopkChunk + threadIdx.x * per;
  int gt = 0, eq = 0;
  for (int t = 0; t < per; ++t) {
    const int q = beg + t;
    if (q >= n) break;
    const uint32_t key = keys[q];
    gt += take_above(key, S) ? 1 : 0;
    eq += take_equal(key, S) ? 1 : 0;
  }
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
  int pos = gt_base + og + min(eq_rank, S.need_eq);
  int32_t* out = L.sel[which];
  for (int t = 0; t < per; ++t) {
    const int q = beg + t;
    if (q >= n) break;
    const uint32_t key = keys[q];
    bool take = take_above(key, S);
    if (take_equal(key, S)) {
      take = eq_rank < S.need_eq;
      ++eq_rank;
    }
    if (take) out[pos++] = q;
  }
}

// Appends the c2 first columns of the proposal set to the set log as the set
// of the current iteration (one workgroup; no-op without the log).
__device__ void log_set(const WalkCtx& C, const LearnCtx& L, int c2) {
  if (L.set_off == nullptr) return;
  const int64_t k = C.st->k;
  const int64_t pos = L.ls->set_pos;
  const bool fits = pos + c2 <= L.set_log_cap;
  if (fits)
    for (int i = threadIdx.x; i < c2; i += blockDim.x) L.set_log[pos + i] = C.P.perm[L.sel[0][i]];
  __syncthreads();
  if (threadIdx.x == 0) {
    const int64_t end = fits ? pos + c2 : pos;
    L.set_off[k] = pos;
    L.set_off[k + 1] = end;
    L.ls->set_pos = end;
  }
}

// A proposal iteration that keeps the last proposal set: logs it again.
__global__ __launch_bounds__(256) void k_keep_set(const WalkCtx* __restrict__ walks,
                                                  const LearnCtx* __restrict__ lc) {
  const WalkCtx& C = walks[0];
  const LearnCtx& L = *lc;
  if (!active(C.st, L.ls)) return;
  log_set(C, L, L.ls->tk[0].count);
}

// End of a selection (one workgroup): the selected count; for the proposal
// set also the subset-pass chunk offsets and the set log; then clears the
// histograms for the next selection.
__global__ __launch_bounds__(256) void k_topk_finish(const WalkCtx* __restrict__ walks,
                                                     const LearnCtx* __restrict__ lc, int32_t which, int32_t full) {
  const WalkCtx& C = walks[0];
  const LearnCtx& L = *lc;
  const WalkState* st = C.st;
  if (!active(st, L.ls)) return;
  const Select S = derive(L, which, 3);
  const int cnt = S.count;
  __shared__ int wsum[4];
  __shared__ int carry;
  if (which == 0) {
    // exclusive prefix of per-column chunk counts, in tiles of 256 columns
    if (threadIdx.x == 0) carry = 0;
    __syncthreads();
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    for (int base = 0; base < cnt; base += kBlock) {
      const int i = base + threadIdx.x;
      int c = 0;
      if (i < cnt) {
        const int q = L.sel[0][i];
        const uint8_t cl = L.cls[q];
        const int e = C.P.col_ptr[q + 1] - C.P.col_ptr[q];
        c = (cl == SUB_GENERAL) ? 0 : max(1, (e + kSubsetChunk - 1) / kSubsetChunk);
      }
      int inc = c;
#pragma unroll
      for (int o = 1; o < kWave; o <<= 1) {
        const int y = __shfl_up(inc, o, kWave);
        if (lane >= o) inc += y;
      }
      if (lane == 63) wsum[wv] = inc;
      __syncthreads();
      int off = carry + inc - c;
      for (int k = 0; k < wv; ++k) off += wsum[k];
      if (i < cnt) L.sub_off[i] = off;
      __syncthreads();
      if (threadIdx.x == kBlock - 1) carry = off + c;
      __syncthreads();
    }
    if (threadIdx.x == 0) {
      L.sub_off[cnt] = carry;
      L.ls->tk[0].chunks = carry;
    }
    // proposal-set log (original indices); a full evaluation records an empty range
    log_set(C, L, full ? 0 : cnt);
  }
  if (threadIdx.x == 0) L.ls->tk[which].count = cnt;
  // every reader of the histograms has finished (earlier kernels, derive above)
  __syncthreads();
  uint32_t* H = L.hist + which * 3 * kRadixBins;
  for (int b = threadIdx.x; b < 3 * kRadixBins; b += blockDim.x) H[b] = 0;
}

// ---------------------------------------------------------------------------
// Training pairs, judge, features
// ---------------------------------------------------------------------------

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
  const int64_t k = st->k;
  const Globals Gl = globals(k, L.ls->k_last_full, st->V, L.mp);
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
      const bf16x4 x = assemble(L.feat, q, gg, k, Gl);
      for (int t = 0; t < 4; ++t) {
        L.pair_feat[(int64_t)i * 16 + 4 * gg + t] = (uint16_t)x[t];
        if (log) L.log_feat[(logged + i) * 16 + 4 * gg + t] = (uint16_t)x[t];
      }
    }
  }
  __syncthreads();
  if (threadIdx.x == 0 && log) L.ls->logged = logged + T2;
}

// Judge of a full evaluation (was its move in the network's proposal set?)
// and the stored-row update of the move.
__global__ void k_learn_judge(const WalkCtx* __restrict__ walks, const LearnCtx* __restrict__ lc) {
  const WalkCtx& C = walks[0];
  const LearnCtx& L = *lc;
  const WalkState* st = C.st;
  if (threadIdx.x != 0 || st->k >= st->iters) return;
  LearnState* ls = L.ls;
  ls->evals += 1;
  const int q = st->mv_j;
  if (q < 0) return;
  after_move(C, L);
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
  const Globals Gl = globals(k, k_last_full, C.st->V, L.mp);
  for (int gg = 0; gg < 4; ++gg) {
    const bf16x4 x = assemble(L.feat, q, gg, k, Gl);
    for (int t = 0; t < 4; ++t) o[4 * gg + t] = ok ? (uint16_t)x[t] : 0;
  }
}

inline int grid_for(int64_t work, int per_block, int cap) {
  int64_t b = (work + per_block - 1) / per_block;
  return (int)std::max<int64_t>(1, std::min<int64_t>(b, cap));
}

hipError_t topk(const WalkCtx* C, const LearnCtx* L, const LearnCtx& Lh, int which, int full, int32_t n,
                hipStream_t s) {
  const int hb = grid_for(n, 256 * 16, 1024);
  hipLaunchKernelGGL(k_topk_hist, dim3(hb), dim3(kBlock), 0, s, C, L, which, 1, n);
  hipLaunchKernelGGL(k_topk_hist, dim3(hb), dim3(kBlock), 0, s, C, L, which, 2, n);
  hipLaunchKernelGGL(k_topk_count, dim3(Lh.nwg), dim3(kBlock), 0, s, C, L, which, n);
  hipLaunchKernelGGL(k_topk_write, dim3(Lh.nwg), dim3(kBlock), 0, s, C, L, which, n);
  hipLaunchKernelGGL(k_topk_finish, dim3(1), dim3(kBlock), 0, s, C, L, which, (int32_t)full);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_learn_init(const WalkCtx* C, const LearnCtx* L, const LearnCtx& Lh, int32_t n,
                             const int32_t* last_move, const int32_t* moves, hipStream_t s) {
  if (n > 0) hipLaunchKernelGGL(k_learn_init, dim3((n + 255) / 256), dim3(256), 0, s, C, L, n, last_move, moves);
  return hipGetLastError();
}

hipError_t launch_learn_refresh(const WalkCtx* C, const LearnCtx* L, const LearnCtx& Lh, hipStream_t s) {
  if (Lh.n_ref_short > 0)
    hipLaunchKernelGGL(k_refresh_short, dim3(grid_for(Lh.n_ref_short, 32, 8192)), dim3(256), 0, s, C, L);
  if (Lh.n_ref_chunks > 0) {
    hipLaunchKernelGGL(k_refresh_chunks, dim3(std::min(Lh.n_ref_chunks, 4096)), dim3(256), 0, s, C, L);
    hipLaunchKernelGGL(k_refresh_combine, dim3((Lh.n_ref_cols + 255) / 256), dim3(256), 0, s, C, L);
  }
  return hipGetLastError();
}

hipError_t launch_learn_begin(const WalkCtx* C, const LearnCtx* L, hipStream_t s) {
  hipLaunchKernelGGL(k_learn_begin, dim3(1), dim3(64), 0, s, C, L);
  return hipGetLastError();
}

hipError_t launch_learn_propose(const WalkCtx* C, const LearnCtx* L, const LearnCtx& Lh, const ModelDev& M,
                                int32_t n, int full_iteration, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_learn_score, dim3(grid_for(n, 64, 768)), dim3(256), 0, s, C, L, M.w, M.wb, n);
  return topk(C, L, Lh, 0, full_iteration, n, s);
}

hipError_t launch_learn_train(const WalkCtx* C, const LearnCtx* L, const LearnCtx& Lh, const ModelDev& M,
                              int32_t n, int32_t steps, float lr, hipStream_t s) {
  if (n <= 0 || (steps <= 0 && Lh.log_feat == nullptr)) return hipSuccess;
  hipLaunchKernelGGL(k_label_keys, dim3(grid_for(n, 256 * 16, 1024)), dim3(256), 0, s, C, L, n);
  hipError_t e = topk(C, L, Lh, 1, 1, n, s);
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

hipError_t launch_learn_keep_set(const WalkCtx* C, const LearnCtx* L, hipStream_t s) {
  hipLaunchKernelGGL(k_keep_set, dim3(1), dim3(256), 0, s, C, L);
  return hipGetLastError();
}

hipError_t launch_learn_judge(const WalkCtx* C, const LearnCtx* L, hipStream_t s) {
  hipLaunchKernelGGL(k_learn_judge, dim3(1), dim3(64), 0, s, C, L);
  return hipGetLastError();
}

hipError_t launch_learn_features_out(const WalkCtx* C, const LearnCtx* L, int32_t n, int64_t k, int64_t k_last_full,
                                     uint16_t* out, hipStream_t s) {
  if (n > 0)
    hipLaunchKernelGGL(k_learn_features_out, dim3((n + 255) / 256), dim3(256), 0, s, C, L, n, k, k_last_full, out);
  return hipGetLastError();
}

}  // namespace chap
