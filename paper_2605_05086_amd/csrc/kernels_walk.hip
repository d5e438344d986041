// Tabu-walk kernels for gfx950: residual from scratch, state initialisation,
// global move selection under tabu/aspiration, sparse move application and
// weight update.
//
// Residuals r_i = sum_k a_ik x_k - b_i are stored per row (section 3.1
// "Memory Considerations", first remark) in the row's '<=' orientation; the
// negated twin of an equality row has residual -r_i. A move of variable j by
// d updates only the rows of column j: r_i += a_ij d. The objective cutoff
// row c^T x <= bc (section 3.2) is kept in the walk state.

#include <climits>
#include <cmath>

#include "chap_internal.h"
#include "exact_sum.h"
#include "learned_rows.h"
#include "narrow_finish.h"

namespace chap {
namespace {


__device__ __forceinline__ double wave_sum_d(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
  return v;
}

__device__ __forceinline__ long long wave_sum_ll(long long v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
  return v;
}

// Sum across a workgroup of 256 threads; every thread gets the total.
__device__ __forceinline__ long long block_sum_ll(long long v, long long* red) {
  v = wave_sum_ll(v);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) red[wv] = v;
  __syncthreads();
  long long t = 0;
  for (int q = 0; q < (int)(blockDim.x >> 6); ++q) t += red[q];
  return t;
}

__device__ __forceinline__ double block_sum_d(double v, double* red) {
  v = wave_sum_d(v);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) red[wv] = v;
  __syncthreads();
  double t = 0.0;
  for (int q = 0; q < (int)(blockDim.x >> 6); ++q) t += red[q];
  return t;
}

__device__ __forceinline__ int viol_change(double r, double r2, double eps) {
  return (r2 > eps ? 1 : 0) - (r > eps ? 1 : 0);
}


// The objective-related part of a walk state, held in registers by every
// lane of one wavefront (uniform values; lane 0 writes them back).
struct ObjState {
  double f, fbest, bc, rc;
  long long V;
  float wc;
  int has_best, copy_best, cut_active, obj_integral;
  __device__ void load(const WalkState* st) {
    f = st->f;
    fbest = st->fbest;
    bc = st->bc;
    rc = st->rc;
    V = st->V;
    wc = st->wc;
    has_best = st->has_best;
    copy_best = st->copy_best;
    cut_active = st->cut_active;
    obj_integral = st->obj_integral;
  }
  __device__ void store(WalkState* st) const {
    st->f = f;
    st->fbest = fbest;
    st->bc = bc;
    st->rc = rc;
    st->V = V;
    st->wc = wc;
    st->has_best = has_best;
    st->copy_best = copy_best;
    st->cut_active = cut_active;
    st->obj_integral = obj_integral;
  }
  // Cutoff residual c^T x - bc: rounded once from the exact sum acc, or (acc
  // null: FP64 sums of the objective are exact) f - bc.
  __device__ double cutoff_residual(const WaveExact* acc) const { return acc ? acc->round_plus(-bc) : f - bc; }
  // Incumbent rule when no normalised row is violated: the point is
  // feasible; record it if it improves the best objective and (re)set the
  // cutoff row c^T x <= f_best - delta (section 3.2).
  __device__ void incumbent_check(double eps, const WaveExact* acc) {
    if (V != 0) return;
    if (!has_best || f < fbest) {
      fbest = f;
      has_best = 1;
      copy_best = 1;
    }
    const double delta = obj_integral ? 1.0 : 1e-4 * fmax(1.0, fabs(fbest));
    bc = fbest - delta;
    cut_active = 1;
    rc = cutoff_residual(acc);
    V = (rc > eps) ? 1 : 0;
  }
};

// Residual from scratch of every stored row, r_i = sum_k a_ik x_k - b_i
// (coefficients from the int8 row copy when the instance has one), with the
// row's products summed one after another in the row's stored
// order (the order of the caller's CSR, as the definition is written). A
// group of kResidualLanes lanes owns kResidualRows consecutive rows, read
// side by side so that more loads are in flight: for each row the lanes
// load consecutive entries and form their products (coalesced row reads),
// and every lane of the group then adds the products in entry order from
// its neighbours' registers, so the sum is the sequential one bit for bit. On
// instances whose row activities are exact integers (P.sums_exact) the
// order cannot change the sum: each lane adds its own products and the
// group combines the lanes' sums in three exchanges.
// Weights: kWeightsKeep leaves them, kWeightsUnit sets every weight to 1,
// kWeightsScatter copies the caller's normalised weights. With grow, the
// compact row copy is written too (all-integer instances); with the
// caller's weights it is checked as well: st->compact_rows, set by the
// state initialisation that runs first, is cleared when a residual or a
// weight (the cutoff's included) does not fit.
constexpr int kResidualLanes = 8;
constexpr int kResidualSteps = 4;
constexpr int kResidualRows = 1;  // consecutive rows per group (4 measured no faster: 98 against 94 us)
static_assert(kResidualRows <= kResidualLanes, "a lane of the group writes each row");
enum { kWeightsKeep = 0, kWeightsUnit = 1, kWeightsScatter = 2 };

constexpr int kResidualRound = kResidualLanes * kResidualSteps;

// Sums of the products of one group's kResidualRows rows: where the row
// activities are exact (P.sums_exact) each lane's share, added up by the
// caller; otherwise the whole sequential sum on every lane of the group.
// kResidualSteps entries of each row per lane in flight, every load of a
// round issued before its products are summed. kSmall: int8 coefficients
// and the byte copy of x, whose products are exact integers, summed in any
// order (instances with exact row activities); otherwise the FP64 values
// (the byte copy of x when xc is given) and, unless P.sums_exact, the
// sequential order within each row.
template <bool kSmall>
__device__ __forceinline__ void residual_rounds(const DevProblem& P, const double* x, const int8_t* xc, int g,
                                                const int* beg, const int* end, int rounds, double* acc) {
  constexpr int R = kResidualRows, S = kResidualSteps;
  const gptr<const double> val = gmem(P.row_val);
  const gptr<const int8_t> c8 = gmem(P.row_c8);
  const gptr<const int32_t> col = gmem(P.row_col);
  const gptr<const double> xg = gmem(x);
  const gptr<const int8_t> xcg = gmem(xc);
#pragma unroll
  for (int rr = 0; rr < R; ++rr) acc[rr] = 0.0;
  for (int t0 = 0; t0 < rounds; ++t0) {
    int c[R][S];
    if constexpr (kSmall) {
      int a[R][S];
#pragma unroll
      for (int rr = 0; rr < R; ++rr)
#pragma unroll
        for (int u = 0; u < S; ++u) {
          const int e = beg[rr] + t0 * kResidualRound + u * kResidualLanes + g;
          const bool in = e < end[rr];
          c[rr][u] = in ? col[e] : 0;
          a[rr][u] = in ? (int)c8[e] : 0;
        }
#pragma unroll
      for (int rr = 0; rr < R; ++rr)
#pragma unroll
        for (int u = 0; u < S; ++u) acc[rr] = acc[rr] + (double)(a[rr][u] * (int)xcg[c[rr][u]]);
    }
  }
  if constexpr (!kSmall) {
    // one row after another: the FP64 path keeps the register count of a
    // single row in flight
#pragma unroll 1
    for (int rr = 0; rr < R; ++rr) {
      // register arrays indexed by a loop variable would go to scratch:
      // this row's range by selection
      int rb = 0, re = 0;
#pragma unroll
      for (int t = 0; t < R; ++t)
        if (t == rr) {
          rb = beg[t];
          re = end[t];
        }
      double sum = 0.0;
      for (int e0 = rb; e0 < re; e0 += kResidualRound) {
        int c[S];
        double a[S], prod[S];
#pragma unroll
        for (int u = 0; u < S; ++u) {
          const int e = e0 + u * kResidualLanes + g;
          const bool in = e < re;
          c[u] = in ? col[e] : 0;
          a[u] = in ? val[e] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < S; ++u) prod[u] = a[u] * (xc ? (double)xcg[c[u]] : xg[c[u]]);
        if (P.sums_exact) {
#pragma unroll
          for (int u = 0; u < S; ++u) sum = sum + prod[u];
        } else {
#pragma unroll
          for (int u = 0; u < S; ++u) {
            const int cnt = min(kResidualLanes, re - (e0 + u * kResidualLanes));
            for (int t = 0; t < cnt; ++t) sum = sum + __shfl(prod[u], t, kResidualLanes);
          }
        }
      }
#pragma unroll
      for (int t = 0; t < R; ++t)
        if (t == rr) acc[t] = sum;
    }
  }
}

// Writes row i's residual r and weights (kWeightsKeep: r only; Unit: 1 and
// the twin's 1; Scatter: the caller's w0 and w1) and, with grow, its compact
// copy; with the caller's weights the copy is checked as well: the state
// initialisation has run and checked the cutoff weight, and a residual or
// weight that does not fit clears st->compact_rows.
template <int kWeights>
__device__ __forceinline__ void write_residual(int64_t i, double r, float w0, float w1, bool twin,
                                               RowState* __restrict__ rs, GatherRow* __restrict__ grow,
                                               WalkState* st_w) {
  if constexpr (kWeights == kWeightsKeep) {
    rs[i].r = r;
  } else {
    RowState q;
    q.r = r;
    q.w0 = w0;
    q.w1 = twin ? w1 : -1.0f;
    if constexpr (kWeights == kWeightsUnit) {
      q.w0 = 1.0f;
      q.w1 = twin ? 1.0f : -1.0f;
      if (grow) {
        GatherRow cr;
        cr.r = (int32_t)r;
        cr.w0 = 1;
        cr.w1 = twin ? (uint16_t)1 : kNoTwin;
        grow[i] = cr;
      }
    } else if (grow) {
      const bool ok = r == floor(r) && fabs(r) <= 2147483647.0 && q.w0 == floorf(q.w0) && q.w0 >= 0.0f &&
                      q.w0 < 65535.0f && (q.w1 < 0.0f || (q.w1 == floorf(q.w1) && q.w1 < 65535.0f));
      if (!ok) st_w->compact_rows = 0;  // every writer stores the same value
      GatherRow cr;
      cr.r = ok ? (int32_t)r : 0;
      cr.w0 = ok ? (uint16_t)q.w0 : 0;
      cr.w1 = (ok && q.w1 >= 0.0f) ? (uint16_t)q.w1 : kNoTwin;
      grow[i] = cr;
    }
    rs[i] = q;
  }
}

template <int kWeights>
__global__ __launch_bounds__(256) void k_residual(DevProblem P, const double* __restrict__ x,
                                                  const int8_t* __restrict__ xc, const WalkState* st,
                                                  uint32_t epoch, RowState* __restrict__ rs,
                                                  const int32_t* __restrict__ nidx, const uint8_t* __restrict__ pair,
                                                  const float* __restrict__ w, GatherRow* __restrict__ grow) {
  constexpr int R = kResidualRows;
  WalkState* st_w = const_cast<WalkState*>(st);
  const int g = threadIdx.x & (kResidualLanes - 1);
  const int64_t i0 = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kResidualLanes * R;
  if (i0 >= P.ms) return;  // whole groups leave together
  const bool small = xc != nullptr && st->x_misfit != epoch;
  // lane g < R owns row i0 + g's right-hand side and weights: loaded first,
  // they arrive while the entries are read
  const int64_t mine = i0 + g;
  const bool owner = g < R && mine < P.ms;
  double rhs = 0.0;
  float w0 = 1.0f, w1 = -1.0f;
  bool twin = false;
  if (owner) {
    rhs = P.row_rhs[mine];
    if constexpr (kWeights != kWeightsKeep) twin = pair[mine] != 0;
    if constexpr (kWeights == kWeightsScatter) {
      const int k = nidx[mine];
      w0 = w[k];
      if (twin) w1 = w[k + 1];
    }
  }
  int beg[R], end[R], rounds = 0;
#pragma unroll
  for (int rr = 0; rr < R; ++rr) {
    const int64_t i = i0 + rr;
    beg[rr] = i < P.ms ? P.row_ptr[i] : 0;
    end[rr] = i < P.ms ? P.row_ptr[i + 1] : 0;
  }
#pragma unroll
  for (int rr = 0; rr < R; ++rr) rounds = max(rounds, (end[rr] - beg[rr] + kResidualRound - 1) / kResidualRound);
  double acc[R];
  if (P.row_c8 && small && P.sums_exact)
    residual_rounds<true>(P, x, xc, g, beg, end, rounds, acc);
  else
    residual_rounds<false>(P, x, small ? xc : nullptr, g, beg, end, rounds, acc);
  if (P.sums_exact) {
#pragma unroll
    for (int rr = 0; rr < R; ++rr)
#pragma unroll
      for (int o = 1; o < kResidualLanes; o <<= 1) acc[rr] = acc[rr] + __shfl_xor(acc[rr], o, kResidualLanes);
  }
  // every lane of the group holds every row's sum; lane g writes row i0 + g
  double sum = 0.0;
#pragma unroll
  for (int rr = 0; rr < R; ++rr)
    if (g == rr) sum = acc[rr];
  if (!owner) return;
  write_residual<kWeights>(mine, sum - rhs, w0, w1, twin, rs, grow, st_w);
}

// Row sums of one workgroup's kResGroupRows rows with x held in LDS: the
// byte copy of x is swept in kResXBlock-column blocks (the next block's
// bytes loaded into registers while the current one is used), and the
// group's entries of each block (int8 coefficient, word = row in group and
// column in block) add their products into int32 LDS sums (exact: the
// layout exists only where every row's byte-range activity fits). This
// trades the one random L2 request per nonzero of k_residual for whole-line
// reads of x. A call whose point does not fit the byte copy sums the rows
// from x as k_residual does.
constexpr int kResBlockedThreads = 1024;
static_assert(kResXBlock == (1 << 17) && kResGroupRows <= (1 << 15), "entry word: row << 17 | column");
template <int kWeights>
__global__ __launch_bounds__(kResBlockedThreads) void k_residual_blocked(
    DevProblem P, const double* __restrict__ x, const int8_t* __restrict__ xc, const WalkState* st, uint32_t epoch,
    RowState* __restrict__ rs, const int32_t* __restrict__ nidx, const uint8_t* __restrict__ pair,
    const float* __restrict__ w, GatherRow* __restrict__ grow) {
  __shared__ int32_t acc[kResGroupRows];
  __shared__ __align__(16) int8_t xs[kResXBlock];
  WalkState* st_w = const_cast<WalkState*>(st);
  const int64_t i0 = (int64_t)blockIdx.x * kResGroupRows;
  const int rows = (int)min((int64_t)kResGroupRows, (int64_t)P.ms - i0);
  const bool small = st->x_misfit != epoch;
  if (small) {
    constexpr int kV = kResXBlock / 16 / kResBlockedThreads;  // 16-byte words of a block per thread
    constexpr int kE = 4;                                      // entries per thread in flight
    const int4* __restrict__ xv = (const int4*)xc;
    const gptr<const int8_t> xb = gmem(xc);
    const gptr<const uint32_t> ent = gmem(P.rb_ent);
    const gptr<const int8_t> c8 = gmem(P.rb_c8);
    const int nxb = P.rb_nxb;
    const int32_t* seg = P.rb_seg + (int64_t)blockIdx.x * nxb;
    for (int t = threadIdx.x; t < kResGroupRows; t += kResBlockedThreads) acc[t] = 0;
    // block b's bytes: whole 16-byte words below n, single bytes past the
    // last whole word
    int4 pre[kV];
    auto load_block = [&](int b) {
      const int64_t c0 = (int64_t)b * kResXBlock;
      const int64_t words = ((int64_t)P.n - c0) / 16;
#pragma unroll
      for (int v = 0; v < kV; ++v) {
        const int t = threadIdx.x + v * kResBlockedThreads;
        if (t < words) {
          pre[v] = xv[c0 / 16 + t];
        } else {
          int32_t part[4] = {0, 0, 0, 0};
          for (int k = 0; k < 16; ++k) {
            const int64_t c = c0 + 16 * (int64_t)t + k;
            if (c < P.n) part[k >> 2] |= (int32_t)(uint8_t)xb[c] << (8 * (k & 3));
          }
          pre[v] = make_int4(part[0], part[1], part[2], part[3]);
        }
      }
    };
    int b = 0;
    while (b < nxb && seg[b] == seg[b + 1]) ++b;  // blocks without entries are skipped
    if (b < nxb) load_block(b);
    while (b < nxb) {
      int nb = b + 1;
      while (nb < nxb && seg[nb] == seg[nb + 1]) ++nb;
      __syncthreads();  // the previous block's readers are done
#pragma unroll
      for (int v = 0; v < kV; ++v) ((int4*)xs)[threadIdx.x + v * kResBlockedThreads] = pre[v];
      if (nb < nxb) load_block(nb);  // in flight while this block is used
      __syncthreads();
      const int e_end = seg[b + 1];
      for (int e0 = seg[b] + threadIdx.x; e0 < e_end; e0 += kE * kResBlockedThreads) {
        uint32_t wd[kE];
        int a[kE];
#pragma unroll
        for (int u = 0; u < kE; ++u) {
          const int e = e0 + u * kResBlockedThreads;
          wd[u] = e < e_end ? ent[e] : 0u;
          a[u] = e < e_end ? (int)c8[e] : 0;
        }
#pragma unroll
        for (int u = 0; u < kE; ++u)
          if (a[u] != 0) atomicAdd(&acc[wd[u] >> 17], a[u] * (int)xs[wd[u] & (kResXBlock - 1)]);
      }
      b = nb;
    }
    __syncthreads();
    for (int t = threadIdx.x; t < rows; t += kResBlockedThreads) {
      const int64_t i = i0 + t;
      float w0 = 1.0f, w1 = -1.0f;
      bool twin = false;
      if constexpr (kWeights != kWeightsKeep) twin = pair[i] != 0;
      if constexpr (kWeights == kWeightsScatter) {
        const int k = nidx[i];
        w0 = w[k];
        if (twin) w1 = w[k + 1];
      }
      write_residual<kWeights>(i, (double)acc[t] - P.row_rhs[i], w0, w1, twin, rs, grow, st_w);
    }
  } else {
    // kResidualLanes lanes per row, rows of the group one group of lanes
    // after another (the FP64 path of k_residual)
    const int g = threadIdx.x & (kResidualLanes - 1);
    for (int t = threadIdx.x / kResidualLanes; t < rows; t += kResBlockedThreads / kResidualLanes) {
      const int64_t i = i0 + t;
      const int beg[1] = {P.row_ptr[i]}, end[1] = {P.row_ptr[i + 1]};
      const int rounds = (end[0] - beg[0] + kResidualRound - 1) / kResidualRound;
      double sum[1];
      residual_rounds<false>(P, x, nullptr, g, beg, end, rounds, sum);
#pragma unroll
      for (int o = 1; o < kResidualLanes; o <<= 1) sum[0] = sum[0] + __shfl_xor(sum[0], o, kResidualLanes);
      if (g != 0) continue;
      float w0 = 1.0f, w1 = -1.0f;
      bool twin = false;
      if constexpr (kWeights != kWeightsKeep) twin = pair[i] != 0;
      if constexpr (kWeights == kWeightsScatter) {
        const int k = nidx[i];
        w0 = w[k];
        if (twin) w1 = w[k + 1];
      }
      write_residual<kWeights>(i, sum[0] - P.row_rhs[i], w0, w1, twin, rs, grow, st_w);
    }
  }
}

// Start point of a seeded walk (internal order): with seed > 0 an integer
// variable with finite bounds starts at l + (h mod (u - l + 1)), h the
// (j+1)-th SplitMix64 output of the seed for original index j; every other
// variable starts at 0 clamped into its bounds.
__global__ __launch_bounds__(256) void k_start_point(DevProblem P, uint64_t seed, double* __restrict__ x,
                                                     int8_t* __restrict__ xc) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= P.n) return;
  const double l = P.lb[q], u = P.ub[q];
  double v;
  if (seed != 0 && P.is_int[q] && isfinite(l) && isfinite(u)) {
    const uint64_t h = splitmix64(seed, (uint64_t)P.perm[q]);
    const uint64_t width = (uint64_t)(u - l) + 1;
    v = l + (double)(h % width);
  } else {
    v = 0.0;
    if (v < l) v = l;
    if (v > u) v = u;
  }
  x[q] = v;
  if (xc) xc[q] = (int8_t)v;  // an integer within [l, u] (byte copies are kept only then)
}

__global__ __launch_bounds__(256) void k_stage_x(const int32_t* __restrict__ perm, const double* __restrict__ src,
                                                 double* __restrict__ dst, int8_t* __restrict__ xc, WalkState* st,
                                                 uint32_t epoch, int32_t n) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= n) return;
  const double v = src[perm ? perm[q] : q];
  if (dst && dst != src) dst[q] = v;
  if (xc) {
    const bool fits = v == floor(v) && v >= -128.0 && v <= 127.0;
    xc[q] = fits ? (int8_t)v : (int8_t)0;
    if (!fits) st->x_misfit = epoch;  // every writer stores the same value
  }
}

// f = c^T x and V = violated rows as grid reductions; the last workgroup
// writes the walk state. With objacc (objectives whose FP64 sums may be
// inexact) every workgroup adds its products exactly into a fixed-point sum
// in LDS, the last one adds the workgroups' sums, keeps the result in objacc
// and rounds f and the cutoff residual from it; otherwise the FP64 sum is
// exact and its order does not matter.
__global__ __launch_bounds__(256) void k_state_init(DevProblem P, const double* __restrict__ x,
                                                    const RowState* __restrict__ rs, WalkState* st,
                                                    double* partial, uint32_t* ticket, long long* objacc,
                                                    int64_t iters, int32_t tenure, int32_t obj_integral,
                                                    double cutoff_rhs, const float* cutoff_w,
                                                    int32_t check_incumbent, int32_t need_obj, int32_t need_v) {
  __shared__ double redd[4];
  __shared__ long long redl[4];
  __shared__ long long lacc[kExactLimbs];
  __shared__ uint32_t last;
  long long* plimb = (long long*)(partial + 2 * kInitBlocks);
  const double eps = P.eps;
  const int gt = blockIdx.x * blockDim.x + threadIdx.x;
  const int gs = gridDim.x * blockDim.x;
  if (objacc) {
    for (int t = threadIdx.x; t < kExactLimbs; t += blockDim.x) lacc[t] = 0;
    __syncthreads();
  }
  // kU items per thread and step, every load issued before any is used
  constexpr int kU = 4;
  double f = 0.0;
  const int n_obj = need_obj ? P.n : 0;
  for (int j0 = gt; j0 < n_obj; j0 += kU * gs) {
    double c[kU], xv[kU];
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      const int j = j0 + u * gs;
      c[u] = j < n_obj ? P.obj[j] : 0.0;
      xv[u] = j < n_obj ? x[j] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      if (c[u] == 0.0) continue;
      if (objacc) {
        double p, e;
        exact_product(c[u], xv[u], p, e);
        exact_atomic_add(lacc, p);
        exact_atomic_add(lacc, e);
      } else {
        f += c[u] * xv[u];
      }
    }
  }
  long long v = 0;
  const int m_v = need_v ? P.ms : 0;
  for (int i0 = gt; i0 < m_v; i0 += kU * gs) {
    RowState q[kU];
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      const int i = i0 + u * gs;
      q[u] = i < m_v ? rs[i] : RowState{0.0, 0.0f, -1.0f};
    }
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      v += (q[u].r > eps) ? 1 : 0;
      if (q[u].w1 >= 0.0f && -q[u].r > eps) v += 1;
    }
  }
  f = block_sum_d(f, redd);
  v = block_sum_ll(v, redl);
  if (threadIdx.x == 0) {
    partial[2 * blockIdx.x] = f;
    partial[2 * blockIdx.x + 1] = (double)v;
  }
  if (objacc)
    for (int t = threadIdx.x; t < kExactLimbs; t += blockDim.x) plimb[blockIdx.x * kExactLimbs + t] = lacc[t];
  __threadfence();
  __syncthreads();
  if (threadIdx.x == 0) last = atomicAdd(ticket, 1u);
  __syncthreads();
  if (last != gridDim.x - 1) return;
  __threadfence();
  if (objacc) {
    for (int t = threadIdx.x; t < kExactLimbs; t += blockDim.x) {
      long long sum = 0;
      for (unsigned b = 0; b < gridDim.x; ++b) sum += plimb[b * kExactLimbs + t];
      lacc[t] = sum;
    }
    __syncthreads();
  }
  if (threadIdx.x >= 64) return;
  // one wavefront finishes; every lane computes the same values
  double ft = 0.0, vt = 0.0;
  for (unsigned b = 0; b < gridDim.x; ++b) {
    ft += partial[2 * b];
    vt += partial[2 * b + 1];
  }
  WaveExact acc;
  if (objacc) {
    acc.a = lacc[threadIdx.x];
    acc.b = threadIdx.x < kExactLimbs - 64 ? lacc[64 + threadIdx.x] : 0;
    acc.normalize();
    acc.store(objacc);
    ft = acc.round_nearest();
  }
  ObjState o;
  o.f = ft;
  o.fbest = HUGE_VAL;
  o.has_best = 0;
  o.copy_best = 0;
  o.obj_integral = obj_integral;
  o.V = (long long)vt;
  o.wc = cutoff_w ? *cutoff_w : 1.0f;
  o.bc = 0.0;
  o.rc = 0.0;
  o.cut_active = 0;
  if (isfinite(cutoff_rhs)) {
    o.cut_active = 1;
    o.bc = cutoff_rhs;
    o.rc = o.cutoff_residual(objacc ? &acc : nullptr);
    if (o.rc > eps) o.V += 1;
  }
  // the start point is the first candidate for the best infeasible point
  const long long v_orig = (long long)vt;
  if (check_incumbent) o.incumbent_check(eps, objacc ? &acc : nullptr);
  if (threadIdx.x != 0) return;
  st->inf_V = v_orig > 0 ? v_orig : LLONG_MAX;
  st->inf_k = v_orig > 0 ? -1 : -2;
  *ticket = 0u;
  st->k = 0;
  st->iters = iters;
  st->tenure = tenure;
  o.store(st);
  st->j_all = -1;
  st->j_nt = -1;
  st->mv_j = -1;
  st->mv_kind = 2;
  st->dV = 0ull;
  // single passes: the compact copy holds the cutoff weight as a count of
  // half weights only when it is an integer below 2^16 (the rows are
  // checked where the copy is written)
  st->compact_rows = (o.wc == floorf(o.wc) && o.wc >= 0.0f && o.wc < 65535.0f) ? 1 : 0;
  st->skip = 0;
  st->aff_ok = 0;
  st->pass_skip = 0;
  st->aff_iters = 0;
}

__device__ __forceinline__ bool better(double sa, int ja, double sb, int jb) {
  return sa > sb || (sa == sb && ja < jb);
}

// Running best (score desc, original index asc) with the internal index.
struct Best {
  double s = 0.0;
  int j = INT_MAX;  // original index
  int q = -1;       // internal index
  __device__ __forceinline__ void offer(double s2, int j2, int q2) {
    if (better(s2, j2, s, j)) {
      s = s2;
      j = j2;
      q = q2;
    }
  }
  __device__ __forceinline__ void wave_reduce() {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) offer(__shfl_xor(s, o, kWave), __shfl_xor(j, o, kWave), __shfl_xor(q, o, kWave));
  }
};

constexpr int kPartialStride = kArgmaxRecord;

// Best positive score overall and among non-tabu variables, ties to the
// lowest original index; one partial record per workgroup. The pending copy
// of a new incumbent (flagged by the previous iteration, before this
// iteration's move changes x) is done here too.
//
// With `combine` the long narrow columns' scores are not in s yet: the
// workgroups past argmax_blocks combine their partial bins, one wavefront
// per column (which writes the column's score), beside the scan, which
// skips their index range.
__global__ __launch_bounds__(256) void k_argmax(const WalkCtx* __restrict__ walks, const int32_t* __restrict__ off,
                                                int32_t nw, int32_t combine) {
  int lb;
  const int w_ = block_walk(off, nw, lb);
  if (w_ < 0) return;
  const WalkCtx& C = walks[w_];
  const gptr<const double> s = gmem((const double*)C.s);
  const gptr<const int32_t> tabu = gmem((const int32_t*)C.tabu);
  const gptr<const int32_t> perm = gmem(C.P.perm);
  const WalkState* st = C.st;
  const gptr<const double> x = gmem((const double*)C.x);
  const gptr<double> best_x = gmem(C.best_x);
  const int32_t n = C.P.n;
  if (st->k >= st->iters) return;
  __shared__ double sa_s[4], sn_s[4];
  __shared__ int ja_s[4], jn_s[4], qa_s[4], qn_s[4];
  const int64_t k = st->k;
  const bool copy = st->copy_best != 0;
  Best ba, bn;
  const int gt = lb * blockDim.x + threadIdx.x;
  const int gs = C.argmax_blocks * blockDim.x;
  const int ncc = combine ? C.plan.n_chunk_cols : 0;
  const int cq0 = ncc > 0 ? C.plan.chunk_cols[0].col : 0;
  if (lb >= C.argmax_blocks) {
    const int idx = (lb - C.argmax_blocks) * 4 + (int)(threadIdx.x >> 6);
    if (idx < ncc) {
      int q;
      const double v = combine_col(C, idx, threadIdx.x & 63, &q);
      if ((threadIdx.x & 63) == 0 && v > 0.0) {
        const int j = perm[q];
        ba.offer(v, j, q);
        if (k > (int64_t)tabu[q]) bn.offer(v, j, q);
      }
    }
  } else {
    if (copy)
      for (int q = gt; q < n; q += gs) best_x[q] = x[q];
    // kU columns per thread and step, every load issued before any is used
    constexpr int kU = 8;
    for (int q0 = gt; q0 < n; q0 += kU * gs) {
      double v[kU];
      int j[kU], tb[kU];
#pragma unroll
      for (int u = 0; u < kU; ++u) {
        const int q = q0 + u * gs;
        v[u] = 0.0;
        if (q < n) {
          v[u] = s[q];
          j[u] = perm[q];
          tb[u] = tabu[q];
        }
      }
#pragma unroll
      for (int u = 0; u < kU; ++u) {
        const int q = q0 + u * gs;
        if (q < n && v[u] > 0.0 && (unsigned)(q - cq0) >= (unsigned)ncc) {
          ba.offer(v[u], j[u], q);
          if (k > (int64_t)tb[u]) bn.offer(v[u], j[u], q);
        }
      }
    }
  }
  ba.wave_reduce();
  bn.wave_reduce();
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  if (lane == 0) {
    sa_s[wv] = ba.s;
    ja_s[wv] = ba.j;
    qa_s[wv] = ba.q;
    sn_s[wv] = bn.s;
    jn_s[wv] = bn.j;
    qn_s[wv] = bn.q;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < 4; ++w) {
      ba.offer(sa_s[w], ja_s[w], qa_s[w]);
      bn.offer(sn_s[w], jn_s[w], qn_s[w]);
    }
    double* rec = C.argmax_partial + kPartialStride * lb;
    rec[0] = ba.s;
    rec[1] = (double)ba.j;
    rec[2] = (double)ba.q;
    rec[3] = bn.s;
    rec[4] = (double)bn.j;
    rec[5] = (double)bn.q;
  }
}

// Reduces the per-thread bests of a workgroup (every thread gets the result).
__device__ __forceinline__ void block_best(Best& ba, Best& bn) {
  __shared__ double sa_s[4], sn_s[4];
  __shared__ int ja_s[4], jn_s[4], qa_s[4], qn_s[4];
  ba.wave_reduce();
  bn.wave_reduce();
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) {
    sa_s[wv] = ba.s;
    ja_s[wv] = ba.j;
    qa_s[wv] = ba.q;
    sn_s[wv] = bn.s;
    jn_s[wv] = bn.j;
    qn_s[wv] = bn.q;
  }
  __syncthreads();
  for (int w = 0; w < 4; ++w) {
    ba.offer(sa_s[w], ja_s[w], qa_s[w]);
    bn.offer(sn_s[w], jn_s[w], qn_s[w]);
  }
}

// Tabu/aspiration decision of one workgroup from the best positive score
// overall (ba) and among non-tabu columns (bn). A tabu overall best is taken
// only if its move leaves no violated row; since a move changes at most one
// violation per normalised entry of its column, that is impossible while V
// exceeds the column's entry count, and the column is only scanned
// otherwise. Without a move the kind is `none_kind` (a reweight for the full
// pass); moves get `kind_offset` added. Writes the chosen step and trace
// record; returns the kind.
__device__ int decide(const WalkCtx& C, const Best& ba, const Best& bn, int none_kind, int kind_offset) {
  __shared__ long long red[4];
  const DevProblem& P = C.P;
  const double* x = C.x;
  const double* xhat = C.xhat;
  const double* s = C.s;
  const RowState* rs = C.rs;
  WalkState* st = C.st;
  const double eps = P.eps;
  const int64_t k = st->k;
  const int qa = (ba.j == INT_MAX) ? -1 : ba.q;
  const int qn = (bn.j == INT_MAX) ? -1 : bn.q;
  int qstar = -1, jstar = -1, kind = none_kind;
  if (qa >= 0 && k > (int64_t)C.tabu[qa]) {
    qstar = qa;
    jstar = ba.j;
    kind = 0;
  } else if (qa >= 0) {
    const int beg = P.col_ptr[qa], end = P.col_ptr[qa + 1];
    const int64_t bound = 2 * (int64_t)(end - beg) + 1;
    long long dv = 0;
    if (st->V <= bound) {
      const double d = xhat[qa] - x[qa];
      for (int e = beg + threadIdx.x; e < end; e += blockDim.x) {
        const RowState r = rs[P.col_row[e]];
        const double r2 = r.r + P.col_val[e] * d;
        dv += viol_change(r.r, r2, eps);
        if (r.w1 >= 0.0f) dv += viol_change(-r.r, -r2, eps);
      }
      dv = block_sum_ll(dv, red);
      if (st->cut_active) {
        const double c = P.obj[qa];
        if (c != 0.0) dv += viol_change(st->rc, st->rc + c * d, eps);
      }
    }
    if (st->V <= bound && st->V + dv == 0) {
      qstar = qa;
      jstar = ba.j;
      kind = 1;
    } else if (qn >= 0) {
      qstar = qn;
      jstar = bn.j;
      kind = 0;
    }
  }
  if (qstar >= 0) kind += kind_offset;
  if (threadIdx.x != 0) return kind;
  st->j_all = (qa >= 0) ? ba.j : -1;
  st->s_all = ba.s;
  st->j_nt = (qn >= 0) ? bn.j : -1;
  st->s_nt = bn.s;
  st->copy_best = 0;
  st->mv_j = qstar;
  st->mv_kind = kind;
  chap_trace_record* t = C.trace + k;
  t->iter = k;
  t->var = jstar;
  t->kind = kind;
  if (qstar >= 0) {
    const double xo = x[qstar], xn = xhat[qstar];
    st->mv_old = xo;
    st->mv_new = xn;
    st->mv_delta = xn - xo;
    st->mv_score = s[qstar];
    t->x_old = xo;
    t->x_new = xn;
    t->score = s[qstar];
  } else {
    st->mv_delta = 0.0;
    t->x_old = 0.0;
    t->x_new = 0.0;
    t->score = 0.0;
  }
  return kind;
}

// One workgroup per walk: finishes the argmax over the partial records, then
// the tabu/aspiration decision.
__global__ __launch_bounds__(256) void k_select(const WalkCtx* __restrict__ walks) {
  const WalkCtx& C = walks[blockIdx.x];
  const double* partial = C.argmax_partial;
  const int32_t nparts = C.argmax_blocks + C.argmax_comb;
  if (C.st->k >= C.st->iters) return;
  Best ba, bn;
  const gptr<const double> pg = gmem(partial);
  // all of a thread's records are loaded before any is compared
  constexpr int kU = 4;
  for (int b0 = threadIdx.x; b0 < nparts; b0 += kU * blockDim.x) {
    double r[kU][6];
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      const int b = b0 + u * blockDim.x;
      if (b < nparts)
#pragma unroll
        for (int f = 0; f < 6; ++f) r[u][f] = pg[kPartialStride * b + f];
    }
#pragma unroll
    for (int u = 0; u < kU; ++u)
      if (b0 + u * (int)blockDim.x < nparts) {
        ba.offer(r[u][0], (int)r[u][1], (int)r[u][2]);
        bn.offer(r[u][3], (int)r[u][4], (int)r[u][5]);
      }
  }
  block_best(ba, bn);
  decide(C, ba, bn, 2, 0);
}

// Move choice of a proposal iteration over the proposal set, same rules as
// k_select. Without an admissible move the iteration is a stall (no
// reweight) and the block's remaining proposal iterations do nothing.
__global__ __launch_bounds__(256) void k_subset_select(const WalkCtx* __restrict__ walks,
                                                       const LearnCtx* __restrict__ lc) {
  const WalkCtx& C = walks[0];
  const LearnCtx& L = *lc;
  WalkState* st = C.st;
  if (st->k >= st->iters) return;
  if (L.ls->idle) {
    if (threadIdx.x == 0) st->skip = 1;
    return;
  }
  const int64_t k = st->k;
  const int cnt = L.ls->tk[0].count;
  Best ba, bn;
  for (int i = threadIdx.x; i < cnt; i += blockDim.x) {
    const int q = L.sel[0][i];
    const double v = C.s[q];
    if (!(v > 0.0)) continue;
    const int j = C.P.perm[q];
    ba.offer(v, j, q);
    if (k > (int64_t)C.tabu[q]) bn.offer(v, j, q);
  }
  block_best(ba, bn);
  const int kind = decide(C, ba, bn, kStallKind, kProposalKind);
  if (threadIdx.x == 0) {
    st->skip = 0;
    if (kind == kStallKind) {
      L.ls->stalls += 1;
      L.ls->idle = 1;
    } else {
      learned::after_move(C, L);
    }
  }
}


// Applies the chosen move to the rows of one column, or the weight update to
// every violated row; violation changes are summed into st->dV (read by
// k_finish after this kernel). With recompute = 0 the rows are updated as
// r += a_ij d, exact on all-integer data; otherwise each touched row is
// summed again from scratch so the kept residual equals its definition bit
// for bit.
__global__ __launch_bounds__(256) void k_apply(const WalkCtx* __restrict__ walks, const int32_t* __restrict__ off,
                                               int32_t nw) {
  int lb;
  const int w_ = block_walk(off, nw, lb);
  if (w_ < 0) return;
  const WalkCtx& C = walks[w_];
  const DevProblem& P = C.P;
  const double* x = C.x;
  RowState* rs = C.rs;
  WalkState* st = C.st;
  const int32_t recompute = C.recompute;
  if (st->k >= st->iters || st->skip || st->mv_kind == kStallKind) return;
  __shared__ long long red[4];
  const double eps = P.eps;
  const int jstar = st->mv_j;
  const int gt = lb * blockDim.x + threadIdx.x;
  const int gs = C.apply_blocks * blockDim.x;
  long long dv = 0;
  if (jstar >= 0 && recompute) {
    // kResidualLanes lanes per touched row: the row is summed again in its
    // stored order (products side by side, added in entry order)
    const double xn = st->mv_new;
    const int beg = P.col_ptr[jstar], end = P.col_ptr[jstar + 1];
    const int g = gt & (kResidualLanes - 1);
    for (int e = beg + gt / kResidualLanes; e < end; e += gs / kResidualLanes) {
      const int i = P.col_row[e];
      double acc = 0.0;
      const int rb = P.row_ptr[i], re = P.row_ptr[i + 1];
      for (int e0 = rb; e0 < re; e0 += kResidualLanes) {
        const int f = e0 + g;
        double prod = 0.0;
        if (f < re) {
          const int c = P.row_col[f];
          prod = P.row_val[f] * ((c == jstar) ? xn : x[c]);
        }
        const int cnt = min(kResidualLanes, re - e0);
        for (int t = 0; t < cnt; ++t) acc = acc + __shfl(prod, t, kResidualLanes);
      }
      if (g == 0) {
        const RowState q = rs[i];
        const double r2 = acc - P.row_rhs[i];
        rs[i].r = r2;
        if (C.grow) C.grow[i].r = (int32_t)r2;
        dv += viol_change(q.r, r2, eps);
        if (q.w1 >= 0.0f) dv += viol_change(-q.r, -r2, eps);
      }
    }
    dv = block_sum_ll(dv, red);
    if (threadIdx.x == 0 && dv != 0) atomicAdd(&st->dV, (unsigned long long)dv);
  } else if (jstar >= 0) {
    const double d = st->mv_delta;
    const int beg = P.col_ptr[jstar], end = P.col_ptr[jstar + 1];
    for (int e = beg + gt; e < end; e += gs) {
      const int i = P.col_row[e];
      const RowState q = rs[i];
      const double r2 = q.r + P.col_val[e] * d;
      rs[i].r = r2;
      if (C.grow) C.grow[i].r = (int32_t)r2;
      dv += viol_change(q.r, r2, eps);
      if (q.w1 >= 0.0f) dv += viol_change(-q.r, -r2, eps);
    }
    dv = block_sum_ll(dv, red);
    if (threadIdx.x == 0 && dv != 0) atomicAdd(&st->dV, (unsigned long long)dv);
  } else {
    for (int i = gt; i < P.ms; i += gs) {
      const RowState q = rs[i];
      if (q.r > eps) {
        rs[i].w0 = q.w0 + 1.0f;
        if (C.grow) C.grow[i].w0 = (uint16_t)(q.w0 + 1.0f);
      }
      if (q.w1 >= 0.0f && -q.r > eps) {
        rs[i].w1 = q.w1 + 1.0f;
        if (C.grow) C.grow[i].w1 = (uint16_t)(q.w1 + 1.0f);
      }
    }
  }
}

// Ends the iteration: objective, cutoff row, incumbent rule, trace, k + 1.
// One wavefront per walk (the exact objective sum is spread over its lanes);
// lane 0 writes.
__global__ __launch_bounds__(64) void k_finish(const WalkCtx* __restrict__ walks) {
  const WalkCtx& C = walks[blockIdx.x];
  const DevProblem& P = C.P;
  WalkState* st = C.st;
  if (st->k >= st->iters || st->skip) return;
  const int lane = threadIdx.x;
  const double eps = P.eps;
  const int64_t k = st->k;
  const int jstar = st->mv_j;
  ObjState o;
  o.load(st);
  o.V += (long long)st->dV;
  const bool exact = C.objacc != nullptr;
  WaveExact acc;
  if (exact) acc.load(C.objacc);
  if (jstar >= 0) {
    const double c = P.obj[jstar];
    const double xo = st->mv_old, xn = st->mv_new;
    if (c != 0.0) {
      double r2 = 0.0;
      if (exact) {
        double p, e;
        exact_product(c, xn, p, e);
        acc.add(p);
        acc.add(e);
        exact_product(c, xo, p, e);
        acc.add(-p);
        acc.add(-e);
        acc.normalize();
        acc.store(C.objacc);
        o.f = acc.round_nearest();
        if (o.cut_active) r2 = o.cutoff_residual(&acc);
      } else {
        const double d = st->mv_delta;
        r2 = o.rc + c * d;
        o.f = o.f + c * d;
      }
      if (o.cut_active) {
        o.V += viol_change(o.rc, r2, eps);
        o.rc = r2;
      }
    }
    if (lane == 0) {
      C.x[jstar] = xn;
      C.tabu[jstar] = (int32_t)(k + st->tenure);
    }
  } else if (st->mv_kind != kStallKind && o.cut_active && o.rc > eps) {
    o.wc = o.wc + 1.0f;
  }
  if (lane == 0) {
    C.trace[k].viol = o.V;
    C.trace[k].obj = o.f;
    if (jstar >= 0) {
      const long long v_orig = o.V - ((o.cut_active && o.rc > eps) ? 1 : 0);
      if (v_orig > 0 && v_orig < st->inf_V) {
        st->inf_V = v_orig;
        st->inf_k = k;
      }
    }
  }
  // the next iteration may rescore only the columns of the moved column's
  // rows when this step changed nothing else the scores depend on: no
  // reweight, no cutoff residual change, no incumbent (which moves the
  // cutoff row)
  int aff = (jstar >= 0 && !(o.cut_active && P.obj[jstar] != 0.0)) ? 1 : 0;
  if (o.V == 0) aff = 0;
  o.incumbent_check(eps, exact ? &acc : nullptr);
  if (lane != 0) return;
  o.store(st);
  st->aff_ok = aff;
  st->dV = 0ull;
  st->k = k + 1;
}

__global__ __launch_bounds__(256) void k_copy_best(const double* __restrict__ x, double* __restrict__ best_x,
                                                   const WalkState* st, int32_t n) {
  if (!st->copy_best) return;
  const int gs = gridDim.x * blockDim.x;
  for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < n; j += gs) best_x[j] = x[j];
}

__global__ __launch_bounds__(256) void k_copy_best_batch(const WalkCtx* __restrict__ walks,
                                                         const int32_t* __restrict__ off, int32_t nw) {
  int lb;
  const int w_ = block_walk(off, nw, lb);
  if (w_ < 0) return;
  const WalkCtx& C = walks[w_];
  if (!C.st->copy_best || lb >= C.argmax_blocks) return;
  const int gs = C.argmax_blocks * blockDim.x;
  for (int q = lb * blockDim.x + threadIdx.x; q < C.P.n; q += gs) C.best_x[q] = C.x[q];
}

__global__ __launch_bounds__(256) void k_gather(const int32_t* __restrict__ perm, const double* __restrict__ src,
                                                double* __restrict__ dst, int32_t n) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q < n) dst[q] = src[perm[q]];
}

// da[j] = a[inv[j]], db[j] = b[inv[j]] (internal order -> caller's order),
// written in the caller's order so that the stores are coalesced.
__global__ __launch_bounds__(256) void k_gather2(const int32_t* __restrict__ inv, const double* __restrict__ a,
                                                 const double* __restrict__ b, double* __restrict__ da,
                                                 double* __restrict__ db, int32_t n) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  const int q = inv[j];
  da[j] = a[q];
  db[j] = b[q];
}

// Planned permutation, first pass: workgroup c sorts input chunk c by output
// block in LDS, then writes the sorted chunk to its runs' staging slots
// (consecutive slots within a run). kArrays (1 or 2) arrays side by side,
// sharing the plan's index loads.
constexpr int kPermRunsThreads = 1024;
constexpr int kPermPlaceThreads = 512;
template <int kArrays>
__global__ __launch_bounds__(kPermRunsThreads) void k_perm_runs(PermPlan pl, const double* __restrict__ in0,
                                                                const double* __restrict__ in1,
                                                                double* __restrict__ st0, double* __restrict__ st1) {
  __shared__ double lds[kArrays][kPermChunk];
  constexpr int kU = kPermChunk / kPermRunsThreads;
  const double* in[2] = {in0, in1};
  double* st[2] = {st0, st1};
  const int64_t base = (int64_t)blockIdx.x * kPermChunk;
  const int cnt = (int)min((int64_t)kPermChunk, (int64_t)pl.n - base);
  double v[kArrays][kU];
  int pos[kU];
#pragma unroll
  for (int u = 0; u < kU; ++u) {
    const int t = threadIdx.x + u * kPermRunsThreads;
    if (t < cnt) {
      pos[u] = pl.lpos[base + t];
#pragma unroll
      for (int a = 0; a < kArrays; ++a) v[a][u] = in[a][base + t];
    }
  }
#pragma unroll
  for (int u = 0; u < kU; ++u)
    if (threadIdx.x + u * kPermRunsThreads < cnt)
#pragma unroll
      for (int a = 0; a < kArrays; ++a) lds[a][pos[u]] = v[a][u];
  __syncthreads();
#pragma unroll
  for (int u = 0; u < kU; ++u) {
    const int t = threadIdx.x + u * kPermRunsThreads;
    if (t < cnt) pos[u] = pl.sdst[base + t];
  }
#pragma unroll
  for (int u = 0; u < kU; ++u) {
    const int t = threadIdx.x + u * kPermRunsThreads;
    if (t < cnt)
#pragma unroll
      for (int a = 0; a < kArrays; ++a) st[a][pos[u]] = lds[a][t];
  }
}

// Second pass: workgroup b places output block b's values (contiguous in
// staging) at their offsets in LDS and writes the block, kArrays arrays side
// by side. With xc, the byte copy of array 0 as in k_stage_x.
template <int kArrays>
__global__ __launch_bounds__(kPermPlaceThreads) void k_perm_place(PermPlan pl, const double* __restrict__ st0,
                                                                  const double* __restrict__ st1,
                                                                  double* __restrict__ out0, double* __restrict__ out1,
                                                                  int8_t* __restrict__ xc, WalkState* ws,
                                                                  uint32_t epoch) {
  __shared__ double lds[kArrays][kPermBlock];
  constexpr int kU = kPermBlock / kPermPlaceThreads;
  const double* st[2] = {st0, st1};
  double* out[2] = {out0, out1};
  const int64_t base = (int64_t)blockIdx.x * kPermBlock;
  const int cnt = (int)min((int64_t)kPermBlock, (int64_t)pl.n - base);
  double v[kArrays][kU];
  int pos[kU];
#pragma unroll
  for (int u = 0; u < kU; ++u) {
    const int t = threadIdx.x + u * kPermPlaceThreads;
    if (t < cnt) {
      pos[u] = pl.dl[base + t];
#pragma unroll
      for (int a = 0; a < kArrays; ++a) v[a][u] = st[a][base + t];
    }
  }
#pragma unroll
  for (int u = 0; u < kU; ++u)
    if (threadIdx.x + u * kPermPlaceThreads < cnt)
#pragma unroll
      for (int a = 0; a < kArrays; ++a) lds[a][pos[u]] = v[a][u];
  __syncthreads();
  bool misfit = false;
#pragma unroll
  for (int u = 0; u < kU; ++u) {
    const int t = threadIdx.x + u * kPermPlaceThreads;
    if (t < cnt) {
#pragma unroll
      for (int a = 0; a < kArrays; ++a) out[a][base + t] = lds[a][t];
      if (xc) {
        const double x = lds[0][t];
        const bool fits = x == floor(x) && x >= -128.0 && x <= 127.0;
        xc[base + t] = fits ? (int8_t)x : (int8_t)0;
        misfit = misfit || !fits;
      }
    }
  }
  if (misfit) ws->x_misfit = epoch;  // every writer stores the same value
}

__global__ __launch_bounds__(256) void k_fill_compact(const RowState* __restrict__ rs, GatherRow* __restrict__ grow,
                                                      int32_t ms) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= ms) return;
  const RowState q = rs[i];
  GatherRow g;
  g.r = (int32_t)q.r;
  g.w0 = (uint16_t)q.w0;
  g.w1 = q.w1 >= 0.0f ? (uint16_t)q.w1 : kNoTwin;
  grow[i] = g;
}

__global__ __launch_bounds__(256) void k_fill_compact_checked(const RowState* __restrict__ rs,
                                                              GatherRow* __restrict__ grow, WalkState* st,
                                                              int32_t ms) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i == 0) {
    // the cutoff weight enters the staged scores as a count of half weights
    const float wc = st->wc;
    if (!(wc == floorf(wc) && wc >= 0.0f && wc < 65535.0f)) st->compact_rows = 0;
  }
  if (i >= ms) return;
  const RowState q = rs[i];
  const bool ok = q.r == floor(q.r) && fabs(q.r) <= 2147483647.0 && q.w0 == floorf(q.w0) && q.w0 >= 0.0f &&
                  q.w0 < 65535.0f && (q.w1 < 0.0f || (q.w1 == floorf(q.w1) && q.w1 < 65535.0f));
  if (!ok) st->compact_rows = 0;  // every writer stores the same value
  GatherRow g;
  g.r = ok ? (int32_t)q.r : 0;
  g.w0 = ok ? (uint16_t)q.w0 : 0;
  g.w1 = (ok && q.w1 >= 0.0f) ? (uint16_t)q.w1 : kNoTwin;
  grow[i] = g;
}

inline int blocks_for(int64_t work, int cap) {
  int64_t b = (work + 255) / 256;
  if (b < 1) b = 1;
  if (b > cap) b = cap;
  return (int)b;
}


// ---------------------------------------------------------------------------
// Affected rescoring. The best shift of column q depends on x_q, its bounds,
// the residuals and weights of its rows and, when the cutoff row is active,
// that row's residual and weight. A move of column j* with no reweight and
// no change of the cutoff row changes only the residuals of j*'s rows, so
// only x_j* and the columns sharing one of those rows need a new score.
// ---------------------------------------------------------------------------

// Short class of internal column q: 0 for a short binary, 1 + D for a short
// non-binary column with D stored entries, -1 for a column outside the
// short range.
__device__ __forceinline__ int aff_class(const int32_t* seg, int q) {
  if (q < seg[0] || q >= seg[kShortMax + 2]) return -1;
  if (q < seg[1]) return 0;
  int c = 1;
#pragma unroll
  for (int k = 1; k <= kShortMax; ++k)
    if (q >= seg[1 + k]) c = 1 + k;
  return c;
}

// One workgroup: lists the affected columns, splits the list into its short columns (grouped by
// class, each class padded to whole wavefronts) and the rest, with the rest's
// subset chunk offsets (ceil(entries / kSubsetChunk) chunks per binary or
// narrow column, none for a general one), and skips the full pass. When the
// step was not a plain move, the list is longer than cap, a listed column
// has no subset form, or the chunks exceed sub_cap, the iteration scores
// every column: through the split of all columns when there is one, else
// through the full pass. Points the subset record and the lane list at the
// lists it takes and clears the count.
__global__ __launch_bounds__(256) void k_aff_plan(const WalkCtx* __restrict__ walks, LearnCtx* __restrict__ lc,
                                                  AffLists A) {
  const WalkCtx& C = walks[0];
  WalkState* st = C.st;
  LearnCtx& L = *lc;
  if (st->k >= st->iters) return;
  __shared__ int ccount[kAffClasses], cfill[kAffClasses], cbase[kAffClasses];
  __shared__ int wsum[4];
  __shared__ int carry, bad, n_other, n_s, n_mark;
  const int tid = threadIdx.x;
  // the affected columns: the moved column and the columns of its rows
  // (stamp[q] = iteration + 1 marks a column already listed; stamps are
  // cleared when the walk starts); at most cap are listed, all are counted.
  // The rows' entries are taken as one flat range (prefix of the row
  // lengths in LDS), so every thread's stamps are in flight at once; a
  // column of more than kAffRows rows is left to the full scoring.
  __shared__ int rpre[kAffRows + 1];
  __shared__ int rrow[kAffRows];
  __shared__ int lst[kRescoreCapMax];  // the affected list
  __shared__ int olst[kRescoreCapMax];  // its columns outside the short range
  if (tid == 0) n_mark = 0;
  __syncthreads();
  if (st->aff_ok) {
    const DevProblem& P = C.P;
    const int32_t tag = (int32_t)st->k + 1;
    const int q0 = st->mv_j;
    const int beg = P.col_ptr[q0], deg = P.col_ptr[q0 + 1] - beg;
    if (deg > kAffRows) {
      if (tid == 0) n_mark = A.cap + 1;
    } else {
      const int lane = tid & 63, wv = tid >> 6;
      int len = 0;
      if (tid < deg) {
        const int i = P.col_row[beg + tid];
        rrow[tid] = i;
        len = P.row_ptr[i + 1] - P.row_ptr[i];
      }
      int inc = len;
#pragma unroll
      for (int o = 1; o < kWave; o <<= 1) {
        const int y = __shfl_up(inc, o, kWave);
        if (lane >= o) inc += y;
      }
      if (lane == 63) wsum[wv] = inc;
      __syncthreads();
      int off = inc - len;
      for (int k = 0; k < wv; ++k) off += wsum[k];
      if (tid < deg) rpre[tid] = off;
      if (tid == deg - 1) rpre[deg] = off + len;
      if (deg == 0 && tid == 0) rpre[0] = 0;
      __syncthreads();
      const int total = rpre[deg];
      auto push = [&](int q) {
        if (atomicExch(&A.stamp[q], tag) != tag) {
          const int k = atomicAdd(&n_mark, 1);
          if (k < A.cap) lst[k] = q;
        }
      };
      if (tid == 0) push(q0);
      for (int f = tid; f < total; f += 256) {
        int lo = 0, hi = deg - 1;
        while (lo < hi) {
          const int mid = (lo + hi + 1) >> 1;
          if (rpre[mid] <= f)
            lo = mid;
          else
            hi = mid - 1;
        }
        push(P.row_col[P.row_ptr[rrow[lo]] + (f - rpre[lo])]);
      }
    }
  }
  __syncthreads();
  const int n_list = st->aff_ok ? n_mark : 0;
  const bool listed = st->aff_ok && n_list <= A.cap;
  const int32_t* seg = C.plan.short_seg;
  if (tid < kAffClasses) {
    ccount[tid] = 0;
    cfill[tid] = 0;
  }
  if (tid == 0) {
    carry = 0;
    bad = 0;
    n_other = 0;
    n_s = 0;
  }
  __syncthreads();
  if (listed) {
    for (int i = tid; i < n_list; i += 256) {
      const int q = lst[i];
      const int c = aff_class(seg, q);
      if (c >= 0) {
        atomicAdd(&ccount[c], 1);
      } else {
        if (L.cls[q] == SUB_NONE) bad = 1;
        const int k = atomicAdd(&n_other, 1);
        olst[k] = q;
        A.olist[k] = q;
      }
    }
    __syncthreads();
    if (tid == 0) {
      int base = 0;
      for (int c = 0; c < kAffClasses; ++c) {
        cbase[c] = base;
        base += (ccount[c] + kWave - 1) / kWave * kWave;
      }
      n_s = base;
    }
    __syncthreads();
    for (int i = tid; i < n_list; i += 256) {
      const int q = lst[i];
      const int c = aff_class(seg, q);
      if (c >= 0) A.slist[cbase[c] + atomicAdd(&cfill[c], 1)] = q;
    }
    for (int c = 0; c < kAffClasses; ++c) {
      const int end = (ccount[c] + kWave - 1) / kWave * kWave;
      for (int t = ccount[c] + tid; t < end; t += 256) A.slist[cbase[c] + t] = -1;
    }
    const int n_o = n_other;
    const int lane = tid & 63, wv = tid >> 6;
    for (int base = 0; base < n_o; base += 256) {
      const int i = base + tid;
      int c = 0;
      if (i < n_o) {
        const int q = olst[i];
        const uint8_t cl = L.cls[q];
        const int e = C.P.col_ptr[q + 1] - C.P.col_ptr[q];
        c = (cl == SUB_GENERAL || cl == SUB_NONE) ? 0 : max(1, (e + kSubsetChunk - 1) / kSubsetChunk);
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
      if (i < n_o) A.ooff[i] = off;
      __syncthreads();
      if (tid == 255) carry = off + c;
      __syncthreads();
    }
  }
  if (tid != 0) return;
  const bool subset = listed && !bad && carry <= A.sub_cap;
  if (subset) {
    A.ooff[n_other] = carry;
    L.sel[0] = A.olist;
    L.sub_off = A.ooff;
    L.ls->tk[0].count = n_other;
    L.ls->tk[0].chunks = carry;
    L.ls->idle = 0;
    A.run->slist = A.slist;
    A.run->n_s = n_s;
    st->pass_skip = 1;
    st->aff_iters += 1;
  } else if (A.full_slist) {
    L.sel[0] = const_cast<int32_t*>(A.full_olist);
    L.sub_off = const_cast<int32_t*>(A.full_ooff);
    L.ls->tk[0].count = A.n_full_o;
    L.ls->tk[0].chunks = A.full_chunks;
    L.ls->idle = 0;
    A.run->slist = A.full_slist;
    A.run->n_s = A.n_full_s;
    st->pass_skip = 1;
  } else {
    L.ls->tk[0].count = 0;
    L.ls->tk[0].chunks = 0;
    L.ls->idle = 1;
    A.run->n_s = 0;
    st->pass_skip = 0;
  }
}


// ---------------------------------------------------------------------------
// Diversity restarts of batched walks (section 3.1 "Parallel Tabu Search
// Instances": walks whose points come too close to another walk's restart).
// ---------------------------------------------------------------------------

__global__ __launch_bounds__(64) void k_set_iters(const WalkCtx* __restrict__ walks, int32_t nw, int64_t iters_end) {
  const int w = blockIdx.x * blockDim.x + threadIdx.x;
  if (w < nw) walks[w].st->iters = iters_end;
}

// One workgroup per task: discrete variables of the task's column range at
// which the two points differ, added into dist[pair].
__global__ __launch_bounds__(256) void k_hamming(const HamTask* __restrict__ tasks, int32_t* __restrict__ dist) {
  const HamTask T = tasks[blockIdx.x];
  __shared__ long long red[4];
  long long c = 0;
  for (int q = T.begin + (int)threadIdx.x; q < T.end; q += (int)blockDim.x)
    c += (T.is_int[q] != 0 && T.xa[q] != T.xb[q]) ? 1 : 0;
  c = block_sum_ll(c, red);
  if (threadIdx.x == 0 && c != 0) atomicAdd(&dist[T.pair], (int32_t)c);
}

__global__ void k_restart_fix(WalkState* st, RestartKeep keep) {
  if (threadIdx.x != 0) return;
  const bool improved = st->has_best && st->copy_best;  // the restart point is a new incumbent
  if (!improved) {
    st->has_best = keep.has_best;
    st->fbest = keep.fbest;
    st->copy_best = 0;
  }
  st->k = keep.k;
  const bool fresh = st->inf_k != -2;  // the restart point is infeasible
  if (keep.inf_k != -2 && (!fresh || keep.inf_V <= st->inf_V)) {
    st->inf_V = keep.inf_V;
    st->inf_k = keep.inf_k;
  } else if (fresh) {
    st->inf_k = keep.k - 1;
  }
}

}  // namespace

namespace {

inline dim3 residual_grid(int32_t ms) {
  const int64_t groups = ((int64_t)ms + kResidualRows - 1) / kResidualRows;
  return dim3((unsigned)((groups * kResidualLanes + 255) / 256));
}

}  // namespace

hipError_t launch_residual(const DevProblem& P, const double* x, RowState* rs, hipStream_t stream) {
  if (P.ms > 0)
    hipLaunchKernelGGL(k_residual<kWeightsKeep>, residual_grid(P.ms), dim3(256), 0, stream, P, x, nullptr, nullptr,
                       0u, rs, nullptr, nullptr, nullptr, nullptr);
  return hipGetLastError();
}

// The x-block kernel where the problem has its row layout and the call has
// a byte copy of x (its own fallback covers a point that does not fit).
inline bool residual_blocked(const DevProblem& P, const int8_t* xc) { return P.rb_ent != nullptr && xc != nullptr; }

inline dim3 residual_blocked_grid(int32_t ms) { return dim3((unsigned)((ms + kResGroupRows - 1) / kResGroupRows)); }

hipError_t launch_residual_unit(const DevProblem& P, const uint8_t* pair, const double* x, const int8_t* xc,
                                const WalkState* st, uint32_t epoch, RowState* rs, GatherRow* grow,
                                hipStream_t stream) {
  if (P.ms > 0 && residual_blocked(P, xc))
    hipLaunchKernelGGL(k_residual_blocked<kWeightsUnit>, residual_blocked_grid(P.ms), dim3(kResBlockedThreads), 0,
                       stream, P, x, xc, st, epoch, rs, nullptr, pair, nullptr, grow);
  else if (P.ms > 0)
    hipLaunchKernelGGL(k_residual<kWeightsUnit>, residual_grid(P.ms), dim3(256), 0, stream, P, x, xc, st, epoch, rs,
                       nullptr, pair, nullptr, grow);
  return hipGetLastError();
}

hipError_t launch_residual_scatter(const DevProblem& P, const int32_t* nidx, const uint8_t* pair, const float* w,
                                   const double* x, const int8_t* xc, const WalkState* st, uint32_t epoch,
                                   RowState* rs, hipStream_t stream, GatherRow* grow) {
  if (P.ms > 0 && residual_blocked(P, xc))
    hipLaunchKernelGGL(k_residual_blocked<kWeightsScatter>, residual_blocked_grid(P.ms), dim3(kResBlockedThreads), 0,
                       stream, P, x, xc, st, epoch, rs, nidx, pair, w, grow);
  else if (P.ms > 0)
    hipLaunchKernelGGL(k_residual<kWeightsScatter>, residual_grid(P.ms), dim3(256), 0, stream, P, x, xc, st, epoch,
                       rs, nidx, pair, w, grow);
  return hipGetLastError();
}

hipError_t launch_start_point(const DevProblem& P, uint64_t seed, double* x, int8_t* xc, hipStream_t stream) {
  if (P.n > 0) hipLaunchKernelGGL(k_start_point, dim3((P.n + 255) / 256), dim3(256), 0, stream, P, seed, x, xc);
  return hipGetLastError();
}

hipError_t launch_stage_x(const int32_t* perm, const double* src, double* dst, int8_t* xc, WalkState* st,
                          uint32_t epoch, int32_t n, hipStream_t stream) {
  if (n > 0)
    hipLaunchKernelGGL(k_stage_x, dim3((n + 255) / 256), dim3(256), 0, stream, perm, src, dst, xc, st, epoch, n);
  return hipGetLastError();
}

hipError_t launch_state_init(const DevProblem& P, const double* x, const RowState* rs, WalkState* st,
                             double* partial, uint32_t* ticket, long long* objacc, int64_t iters, int32_t tenure,
                             int32_t obj_integral, double cutoff_rhs, const float* cutoff_w, int check_incumbent,
                             int count_violated, hipStream_t stream) {
  // a single pass needs neither V nor, without a cutoff row, f
  const int32_t need_v = (check_incumbent || count_violated) ? 1 : 0;
  const int32_t need_obj = (check_incumbent || std::isfinite(cutoff_rhs)) ? 1 : 0;
  const int64_t work = std::max<int64_t>(need_obj ? P.n : 0, need_v ? P.ms : 0);
  const int blocks = work > 0 ? blocks_for((work + 3) / 4, kInitBlocks) : 1;
  hipLaunchKernelGGL(k_state_init, dim3(blocks), dim3(256), 0, stream, P, x, rs, st, partial, ticket, objacc, iters,
                     tenure, obj_integral, cutoff_rhs, cutoff_w, check_incumbent, need_obj, need_v);
  return hipGetLastError();
}

hipError_t launch_walk_choose(const BatchLaunch& L, hipStream_t stream, bool combine) {
  const int nw = L.nw;
  const int32_t comb = (combine && pass_defers_combine(L)) ? 1 : 0;
  hipLaunchKernelGGL(k_argmax, dim3((unsigned)L.grid[KS_ARGMAX]), dim3(256), 0, stream, L.walks, L.off[KS_ARGMAX], nw,
                     comb);
  hipLaunchKernelGGL(k_select, dim3((unsigned)nw), dim3(256), 0, stream, L.walks);
  return hipGetLastError();
}

hipError_t launch_walk_apply(const BatchLaunch& L, hipStream_t stream) {
  hipLaunchKernelGGL(k_apply, dim3((unsigned)L.grid[KS_APPLY]), dim3(256), 0, stream, L.walks, L.off[KS_APPLY], L.nw);
  return hipGetLastError();
}

hipError_t launch_walk_finish(const BatchLaunch& L, hipStream_t stream) {
  hipLaunchKernelGGL(k_finish, dim3((unsigned)L.nw), dim3(64), 0, stream, L.walks);
  return hipGetLastError();
}

hipError_t launch_walk_step(const BatchLaunch& L, hipStream_t stream, bool combine) {
  hipError_t e = launch_walk_choose(L, stream, combine);
  if (e == hipSuccess) e = launch_walk_apply(L, stream);
  if (e == hipSuccess) e = launch_walk_finish(L, stream);
  return e;
}

hipError_t launch_affected(const WalkCtx* C, LearnCtx* L, const AffLists& A, hipStream_t s) {
  hipLaunchKernelGGL(k_aff_plan, dim3(1), dim3(256), 0, s, C, L, A);
  return hipGetLastError();
}

hipError_t launch_set_iters(const BatchLaunch& L, int64_t iters_end, hipStream_t s) {
  hipLaunchKernelGGL(k_set_iters, dim3((unsigned)((L.nw + 63) / 64)), dim3(64), 0, s, L.walks, L.nw, iters_end);
  return hipGetLastError();
}

hipError_t launch_hamming(const HamTask* tasks, int32_t ntasks, int32_t* dist, hipStream_t s) {
  if (ntasks > 0) hipLaunchKernelGGL(k_hamming, dim3((unsigned)ntasks), dim3(256), 0, s, tasks, dist);
  return hipGetLastError();
}

hipError_t launch_restart_fix(WalkState* st, const RestartKeep& keep, hipStream_t s) {
  hipLaunchKernelGGL(k_restart_fix, dim3(1), dim3(64), 0, s, st, keep);
  return hipGetLastError();
}

hipError_t launch_subset_select(const WalkCtx* C, const LearnCtx* L, hipStream_t s) {
  hipLaunchKernelGGL(k_subset_select, dim3(1), dim3(256), 0, s, C, L);
  return hipGetLastError();
}

hipError_t launch_copy_best_batch(const BatchLaunch& L, hipStream_t stream) {
  hipLaunchKernelGGL(k_copy_best_batch, dim3((unsigned)L.grid[KS_ARGMAX]), dim3(256), 0, stream, L.walks,
                     L.off[KS_ARGMAX], L.nw);
  return hipGetLastError();
}

hipError_t launch_gather(const int32_t* perm, const double* src, double* dst, int32_t n, hipStream_t stream) {
  if (n > 0) hipLaunchKernelGGL(k_gather, dim3((n + 255) / 256), dim3(256), 0, stream, perm, src, dst, n);
  return hipGetLastError();
}

hipError_t launch_stage_x_plan(const PermPlan& plan, const double* src, double* dst, int8_t* xc, WalkState* st,
                               uint32_t epoch, double* stage, hipStream_t stream) {
  if (plan.n > 0) {
    const unsigned nc = (unsigned)((plan.n + kPermChunk - 1) / kPermChunk);
    const unsigned nb = (unsigned)((plan.n + kPermBlock - 1) / kPermBlock);
    hipLaunchKernelGGL(k_perm_runs<1>, dim3(nc), dim3(kPermRunsThreads), 0, stream, plan, src, nullptr, stage,
                       nullptr);
    hipLaunchKernelGGL(k_perm_place<1>, dim3(nb), dim3(kPermPlaceThreads), 0, stream, plan, stage, nullptr, dst,
                       nullptr, xc, st, epoch);
  }
  return hipGetLastError();
}

hipError_t launch_gather2_plan(const PermPlan& plan, const double* a, const double* b, double* da, double* db,
                               double* stage, hipStream_t stream) {
  if (plan.n > 0) {
    const unsigned nc = (unsigned)((plan.n + kPermChunk - 1) / kPermChunk);
    const unsigned nb = (unsigned)((plan.n + kPermBlock - 1) / kPermBlock);
    double* stage_b = stage + plan.n;
    hipLaunchKernelGGL(k_perm_runs<2>, dim3(nc), dim3(kPermRunsThreads), 0, stream, plan, a, b, stage, stage_b);
    hipLaunchKernelGGL(k_perm_place<2>, dim3(nb), dim3(kPermPlaceThreads), 0, stream, plan, stage, stage_b, da, db,
                       nullptr, nullptr, 0u);
  }
  return hipGetLastError();
}

hipError_t launch_gather2(const int32_t* inv, const double* a, const double* b, double* da, double* db, int32_t n,
                          hipStream_t stream) {
  if (n > 0) hipLaunchKernelGGL(k_gather2, dim3((n + 255) / 256), dim3(256), 0, stream, inv, a, b, da, db, n);
  return hipGetLastError();
}

hipError_t launch_fill_compact_checked(const RowState* rs, GatherRow* grow, WalkState* st, int32_t ms,
                                       hipStream_t stream) {
  hipLaunchKernelGGL(k_fill_compact_checked, dim3(std::max(1, (ms + 255) / 256)), dim3(256), 0, stream, rs, grow, st,
                     ms);
  return hipGetLastError();
}

hipError_t launch_fill_compact(const RowState* rs, GatherRow* grow, int32_t ms, hipStream_t stream) {
  if (ms > 0) hipLaunchKernelGGL(k_fill_compact, dim3((ms + 255) / 256), dim3(256), 0, stream, rs, grow, ms);
  return hipGetLastError();
}

hipError_t launch_copy_best(const double* x, double* best_x, WalkState* st, int32_t n, hipStream_t stream) {
  hipLaunchKernelGGL(k_copy_best, dim3(blocks_for(n, 1024)), dim3(256), 0, stream, x, best_x, st, n);
  return hipGetLastError();
}

}  // namespace chap
