// Best-shift pass kernels for gfx950 (wave64).
//
// One pass computes, for every variable j, the best shift (Eq. 1 of section
// 3.1 "Best Shift Moves") at the current point: the flip for a binary
// variable, and for every other variable the result of Algorithm 1 ("Best
// Shift via Sort-Scan-Argmax"). Columns are routed by class and length:
//
//   k_short        one lane per column with at most 8 normalised entries;
//                  scores every candidate position directly (bounds and
//                  breakpoints, incumbent excluded) from the penalty
//                  definition written in breakpoint form.
//   k_flip_wave    one wavefront per longer binary column (flip score).
//   k_narrow_pack  integer columns with <= 64 values, packed whole into
//                  workgroups: the sort of Algorithm 1 becomes a counting sort
//                  into 64 LDS bins per column, the scan a wavefront prefix
//                  sum, the argmax a wavefront reduction over candidate bins.
//   k_narrow_chunk the same for long columns split over many workgroups by
//                  row range; k_narrow_combine adds the partial bins.
//   k_sort_block   one workgroup per general column: LDS bitonic sort of the
//                  breakpoints, block scan, block argmax.
//   k_sort_long    general columns beyond the LDS capacity: the same steps in
//                  global scratch memory.
//
// On all-integer instances with 0 < eps <= 1/2 the narrow columns are
// row-block staged instead:
//   k_stage_rows   one workgroup per slice of an 8192-row block held in LDS:
//                  each staged entry becomes an 8-byte breakpoint record, and
//                  single-entry columns are scored on the spot.
//   k_stage_score  one launch for the rest: packs of columns (counting sort
//                  of their records into LDS bins), groups of short columns
//                  of one degree (one lane per column) and the chunks of long
//                  columns, as interleaved units of the grid.
//
// Phase 1 of Algorithm 1 emits, per row, the accumulators beta/alpha and up to
// two triplets. Here the two triplets of an a_ij > 0 row, (t,-1,0) and
// (t,+1,d), are merged into one entry "d applies strictly after t, and t is a
// candidate"; an a_ij < 0 row gives "d applies from t on". The score at a
// candidate position p is beta + (sum of entries applying at p) +
// alpha [p > xbar], the value Algorithm 1's scan produces at that position.
// Only finite positions inside [l, u] other than xbar are candidates, ties go
// to the smallest position, and (xbar, 0) is returned when no candidate scores
// above zero.

#include <algorithm>
#include <cfloat>
#include <cmath>
#include <type_traits>

#include "chap_internal.h"
#include "narrow_finish.h"

namespace chap {
namespace {


// Row accessors: the walk's RowState array, or its compact GatherRow copy.
struct FullRows {
  gptr<const RowState> p;
  __device__ __forceinline__ RowState operator[](int i) const { return gload(p, i); }
};

struct CompactRows {
  gptr<const GatherRow> p;
  __device__ __forceinline__ RowState operator[](int i) const {
    const GatherRow g = gload(p, i);
    RowState o;
    o.r = (double)g.r;
    o.w0 = (float)g.w0;
    o.w1 = (g.w1 == kNoTwin) ? -1.0f : (float)g.w1;
    return o;
  }
};

// Either of the two, as the walk state says (single passes with caller weights).
struct DualRows {
  gptr<const RowState> p;
  gptr<const GatherRow> g;
  int32_t use_g;
  __device__ __forceinline__ RowState operator[](int i) const {
    if (use_g) return CompactRows{g}[i];
    return gload(p, i);
  }
};

template <typename Rows>
__device__ __forceinline__ Rows rows_of(const WalkCtx& C);
template <>
__device__ __forceinline__ DualRows rows_of<DualRows>(const WalkCtx& C) {
  return DualRows{gmem((const RowState*)C.rs), gmem((const GatherRow*)C.grow), C.st->compact_rows};
}
template <>
__device__ __forceinline__ FullRows rows_of<FullRows>(const WalkCtx& C) {
  return FullRows{gmem((const RowState*)C.rs)};
}
template <>
__device__ __forceinline__ CompactRows rows_of<CompactRows>(const WalkCtx& C) {
  return CompactRows{gmem((const GatherRow*)C.grow)};
}

// Whether staged records carry the weights (exact in 16 bits): always with
// the compact row copy, as the walk state says for single passes, never with
// full rows (the scoring kernel then reads them from the row states).
template <typename Rows>
__device__ __forceinline__ bool stage_weights(const WalkCtx& C);
template <>
__device__ __forceinline__ bool stage_weights<CompactRows>(const WalkCtx&) {
  return true;
}
template <>
__device__ __forceinline__ bool stage_weights<DualRows>(const WalkCtx& C) {
  return C.st->compact_rows != 0;
}
template <>
__device__ __forceinline__ bool stage_weights<FullRows>(const WalkCtx&) {
  return false;
}

// Whether the rows are read from the walk's compact copy (whose words then
// have the staged LDS row format, weights included).
__device__ __forceinline__ bool compact_source(const CompactRows&) { return true; }
__device__ __forceinline__ bool compact_source(const DualRows& r) { return r.use_g != 0; }
__device__ __forceinline__ bool compact_source(const FullRows&) { return false; }

__device__ __forceinline__ double breakpoint(double xb, double r, double a, double eps, bool is_int) {
  double t = xb + (eps - r) / a;
  if (is_int) t = (a > 0.0) ? floor(t) : ceil(t);
  return t;
}

// Penalty p_ij of section 3.1 "Scoring Functions" for a residual r -> r2.
__device__ __forceinline__ double penalty(double r, double r2, double w, double eps) {
  const bool v = r > eps, v2 = r2 > eps;
  if (!v && v2) return -w;
  if (v && !v2) return w;
  if (v && v2) {
    if (r2 < r) return 0.5 * w;
    if (r2 > r) return -0.5 * w;
  }
  return 0.0;
}

// Phase 1 of Algorithm 1 for one normalised row entry (a, r, w) of a
// non-binary column at xbar. Updates beta/alpha, returns the merged entry.
struct BkEntry {
  double t;
  double delta;
  int marker;  // -1: applies from t on, +1: applies after t
  bool has;
};

__device__ __forceinline__ BkEntry phase1(double xb, double r, double a, double w, double eps, bool is_int,
                                          double& beta, double& alpha) {
  BkEntry e;
  e.t = breakpoint(xb, r, a, eps, is_int);
  e.has = true;
  if (a < 0.0) {
    e.marker = -1;
    if (xb < e.t) {
      beta -= 0.5 * w;
      alpha += w;
      e.delta = 0.5 * w;
    } else if (xb > e.t) {
      beta -= w;
      e.delta = w;
    } else {
      beta -= w;
      alpha += w;
      e.delta = 0.0;
      e.has = false;
    }
  } else {
    e.marker = 1;
    if (xb > e.t) {
      beta += w;
      alpha -= w;
      e.delta = -0.5 * w;
    } else if (xb < e.t) {
      e.delta = -w;
    } else {
      alpha -= w;
      e.delta = 0.0;
      e.has = false;
    }
  }
  return e;
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
  return v;
}

__device__ __forceinline__ unsigned long long wave_or(unsigned long long v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v |= __shfl_xor(v, o, kWave);
  return v;
}


// ---------------------------------------------------------------------------
// k_short: one lane per column (at most 8 normalised entries).
// ---------------------------------------------------------------------------

template <typename Rows>
__device__ __forceinline__ void flip_column(const DevProblem& P, const double* x, const Rows& rs,
                                            const WalkState* st, double* xhat, double* sc, int q) {
  const double eps = P.eps;
  const double xb = x[q];
  const double xn = 1.0 - xb;
  const double d = xn - xb;
  double s = 0.0;
  const int beg = P.col_ptr[q], end = P.col_ptr[q + 1];
  // at most kShortMax entries here: every gather is issued before any is used
  RowState rr[kShortMax];
  double av[kShortMax];
#pragma unroll
  for (int k = 0; k < kShortMax; ++k) {
    if (beg + k < end) {
      av[k] = P.col_val[beg + k];
      rr[k] = rs[P.col_row[beg + k]];
    }
  }
#pragma unroll
  for (int k = 0; k < kShortMax; ++k) {
    if (beg + k < end) {
      const RowState& r = rr[k];
      const double r2 = r.r + av[k] * d;
      s += penalty(r.r, r2, (double)r.w0, eps);
      if (r.w1 >= 0.0f) s += penalty(-r.r, -r2, (double)r.w1, eps);
    }
  }
  if (st->cut_active) {
    const double c = P.obj[q];
    if (c != 0.0) {
      const double r2 = st->rc + c * d;
      s += penalty(st->rc, r2, (double)st->wc, eps);
    }
  }
  write_result(xhat, sc, q, true, s, xn, xb);
}

// Normalised entries of a short column held in compile-time indexed slots.
struct ShortSlots {
  double tau[kShortMax];
  double w[kShortMax];
  uint32_t apos = 0, sat0 = 0;
  int ns = 0;
  __device__ __forceinline__ void push(double t, double wt, bool ap, double xb) {
#pragma unroll
    for (int k = 0; k < kShortMax; ++k)
      if (k == ns) {
        tau[k] = t;
        w[k] = wt;
      }
    const bool s0 = ap ? (xb <= t) : (xb >= t);
    apos |= (ap ? 1u : 0u) << ns;
    sat0 |= (s0 ? 1u : 0u) << ns;
    ns += 1;
  }
};

// Scores every candidate position of a short column (both bounds and the
// breakpoints inside [l, u], xbar excluded) from the penalty definition: the
// largest score, the smallest position on ties.
__device__ __forceinline__ void short_best(const ShortSlots& S, double l, double u, double xb, bool& found,
                                           double& best, double& bestp) {
  found = false;
  best = 0.0;
  bestp = xb;
  auto consider = [&](double p) {
    if (!(p >= l && p <= u) || p == xb || !isfinite(p)) return;
    double v = 0.0;
#pragma unroll
    for (int k = 0; k < kShortMax; ++k) {
      if (k < S.ns) {
        const bool ap = (S.apos >> k) & 1u;
        const bool s0 = (S.sat0 >> k) & 1u;
        const bool s1 = ap ? (p <= S.tau[k]) : (p >= S.tau[k]);
        double c;
        if (s0)
          c = s1 ? 0.0 : -S.w[k];
        else if (s1)
          c = S.w[k];
        else
          c = (ap ? (p < xb) : (p > xb)) ? 0.5 * S.w[k] : -0.5 * S.w[k];
        v += c;
      }
    }
    if (!found || v > best || (v == best && p < bestp)) {
      found = true;
      best = v;
      bestp = p;
    }
  };
  consider(l);
  consider(u);
#pragma unroll
  for (int k = 0; k < kShortMax; ++k)
    if (k < S.ns) consider(S.tau[k]);
}

template <int D, typename Rows>
__device__ __forceinline__ void short_general(const DevProblem& P, const double* x, const Rows& rs,
                                              const WalkState* st, double* xhat, double* sc, int q) {
  const double eps = P.eps;
  const double xb = x[q];
  const bool isint = P.is_int[q] != 0;
  const double l = P.lb[q], u = P.ub[q];
  const int beg = P.col_ptr[q];
  ShortSlots S;
#pragma unroll
  for (int k = 0; k < kShortMax; ++k) {
    S.tau[k] = 0.0;
    S.w[k] = 0.0;
  }
  // loads of all D entries first (independent), then the breakpoints
  RowState rr[D > 0 ? D : 1];
  double av[D > 0 ? D : 1];
#pragma unroll
  for (int k = 0; k < D; ++k) {
    av[k] = P.col_val[beg + k];
    rr[k] = rs[P.col_row[beg + k]];
  }
#pragma unroll
  for (int k = 0; k < D; ++k) {
    const double a = av[k];
    S.push(breakpoint(xb, rr[k].r, a, eps, isint), (double)rr[k].w0, a > 0.0, xb);
    if (rr[k].w1 >= 0.0f) S.push(breakpoint(xb, -rr[k].r, -a, eps, isint), (double)rr[k].w1, -a > 0.0, xb);
  }
  if (st->cut_active) {
    const double c = P.obj[q];
    if (c != 0.0) S.push(breakpoint(xb, st->rc, c, eps, isint), (double)st->wc, c > 0.0, xb);
  }
  bool found;
  double best, bestp;
  short_best(S, l, u, xb, found, best, bestp);
  write_result(xhat, sc, q, found, best, bestp, xb);
}

// Short columns occupy the internal range [seg[0], seg[10]): binaries in
// [seg[0], seg[1]), then non-binary columns with D stored entries in
// [seg[1 + D], seg[2 + D]) for D = 0..8.
template <typename Rows>
__global__ __launch_bounds__(256) void k_short(const WalkCtx* __restrict__ walks, const int32_t* __restrict__ off,
                                               int32_t nw) {
  int lb;
  const int w_ = block_walk(off, nw, lb);
  if (w_ < 0) return;
  const WalkCtx& C = walks[w_];
  const Rows rs = rows_of<Rows>(C);
  if (C.st->k >= C.st->iters || C.st->pass_skip) return;
  const int32_t* seg = C.plan.short_seg;
  const int q = seg[0] + lb * 256 + threadIdx.x;
  if (q >= seg[kShortMax + 2]) return;
  if (q < seg[1]) {
    flip_column(C.P, C.x, rs, C.st, C.xhat, C.s, q);
    return;
  }
  int D = 0;
#pragma unroll
  for (int k = 1; k <= kShortMax; ++k)
    if (q >= seg[1 + k]) D = k;
  switch (D) {
    case 0: short_general<0>(C.P, C.x, rs, C.st, C.xhat, C.s, q); break;
    case 1: short_general<1>(C.P, C.x, rs, C.st, C.xhat, C.s, q); break;
    case 2: short_general<2>(C.P, C.x, rs, C.st, C.xhat, C.s, q); break;
    case 3: short_general<3>(C.P, C.x, rs, C.st, C.xhat, C.s, q); break;
    case 4: short_general<4>(C.P, C.x, rs, C.st, C.xhat, C.s, q); break;
    case 5: short_general<5>(C.P, C.x, rs, C.st, C.xhat, C.s, q); break;
    case 6: short_general<6>(C.P, C.x, rs, C.st, C.xhat, C.s, q); break;
    case 7: short_general<7>(C.P, C.x, rs, C.st, C.xhat, C.s, q); break;
    default: short_general<8>(C.P, C.x, rs, C.st, C.xhat, C.s, q); break;
  }
}

// The short columns of an affected-rescoring iteration, one lane each
// (grid-stride over the list; classes padded to whole wavefronts, -1 marks
// padding), with the full pass's per-column code.
// b, nb: this workgroup's index among the nb workgroups of the role.
template <typename Rows>
__device__ __forceinline__ void aff_short_body(const WalkCtx& C, const AffRun* run, int b, int nb) {
  if (C.st->k >= C.st->iters) return;
  const Rows rs = rows_of<Rows>(C);
  const int32_t* seg = C.plan.short_seg;
  const int count = run->n_s;
  const int32_t* list = run->slist;
  for (int i = b * (int)blockDim.x + (int)threadIdx.x; i < count; i += nb * (int)blockDim.x) {
    const int q = list[i];
    if (q < 0) continue;
    if (q < seg[1]) {
      flip_column(C.P, C.x, rs, C.st, C.xhat, C.s, q);
      continue;
    }
    int D = 0;
#pragma unroll
    for (int k = 1; k <= kShortMax; ++k)
      if (q >= seg[1 + k]) D = k;
    switch (D) {
      case 0: short_general<0>(C.P, C.x, rs, C.st, C.xhat, C.s, q); break;
      case 1: short_general<1>(C.P, C.x, rs, C.st, C.xhat, C.s, q); break;
      case 2: short_general<2>(C.P, C.x, rs, C.st, C.xhat, C.s, q); break;
      case 3: short_general<3>(C.P, C.x, rs, C.st, C.xhat, C.s, q); break;
      case 4: short_general<4>(C.P, C.x, rs, C.st, C.xhat, C.s, q); break;
      case 5: short_general<5>(C.P, C.x, rs, C.st, C.xhat, C.s, q); break;
      case 6: short_general<6>(C.P, C.x, rs, C.st, C.xhat, C.s, q); break;
      case 7: short_general<7>(C.P, C.x, rs, C.st, C.xhat, C.s, q); break;
      default: short_general<8>(C.P, C.x, rs, C.st, C.xhat, C.s, q); break;
    }
  }
}

// ---------------------------------------------------------------------------
// k_flip_wave: one wavefront per longer binary column.
// ---------------------------------------------------------------------------

template <typename Rows>
__global__ __launch_bounds__(256) void k_flip_wave(const WalkCtx* __restrict__ walks, const int32_t* __restrict__ off,
                                                   int32_t nw) {
  int lb;
  const int w_ = block_walk(off, nw, lb);
  if (w_ < 0) return;
  const WalkCtx& C = walks[w_];
  const DevProblem& P = C.P;
  const double* x = C.x;
  const Rows rs = rows_of<Rows>(C);
  const WalkState* st = C.st;
  double* xhat = C.xhat;
  double* sc = C.s;
  if (st->k >= st->iters || st->pass_skip) return;
  const int lane = threadIdx.x & (kWave - 1);
  const int q = C.plan.flip_begin + lb * 4 + (threadIdx.x >> 6);
  if (q >= C.plan.flip_end) return;
  const double eps = P.eps;
  const double xb = x[q];
  const double xn = 1.0 - xb;
  const double d = xn - xb;
  double s = 0.0;
  const int beg = P.col_ptr[q], end = P.col_ptr[q + 1];
  for (int e = beg + lane; e < end; e += kWave) {
    const RowState r = rs[P.col_row[e]];
    const double r2 = r.r + P.col_val[e] * d;
    s += penalty(r.r, r2, (double)r.w0, eps);
    if (r.w1 >= 0.0f) s += penalty(-r.r, -r2, (double)r.w1, eps);
  }
  if (lane == 0 && st->cut_active) {
    const double c = P.obj[q];
    if (c != 0.0) {
      const double r2 = st->rc + c * d;
      s += penalty(st->rc, r2, (double)st->wc, eps);
    }
  }
  s = wave_sum(s);
  if (lane == 0) write_result(xhat, sc, q, true, s, xn, xb);
}

// ---------------------------------------------------------------------------
// Narrow integer columns: counting sort into LDS bins.
// ---------------------------------------------------------------------------

// Adds one normalised entry of column (l, u, W) at xbar into the bins.
__device__ __forceinline__ void narrow_entry(double xb, double r, double a, double w, double eps, double l,
                                             double u, int W, double* bins, double& beta, double& alpha,
                                             unsigned long long& cand) {
  const BkEntry e = phase1(xb, r, a, w, eps, true, beta, alpha);
  if (!e.has) return;
  if (e.t < l) {
    beta += e.delta;
    return;
  }
  if (e.t > u) return;
  const int k = (int)(e.t - l);
  cand |= 1ull << k;
  if (e.marker < 0)
    atomicAdd(&bins[k], e.delta);
  else if (k + 1 < W)
    atomicAdd(&bins[k + 1], e.delta);
}


// One workgroup per pack of whole narrow columns (consecutive internal
// columns, at most kPackCols of them, about kPackEntries entries). The 256
// threads stream the pack's concatenated CSC entries as one flat range; each
// entry finds its column by binary search over the column starts and adds
// into that column's 64 LDS bins, beta, alpha and candidate mask. Each
// wavefront then scans and reduces a quarter of the pack's columns.
template <typename Rows>
__global__ __launch_bounds__(256) void k_narrow_pack(const WalkCtx* __restrict__ walks,
                                                     const int32_t* __restrict__ off, int32_t nw) {
  int lb;
  const int w_ = block_walk(off, nw, lb);
  if (w_ < 0) return;
  const WalkCtx& C = walks[w_];
  const DevProblem& P = C.P;
  const double* x = C.x;
  const Rows rs = rows_of<Rows>(C);
  const WalkState* st = C.st;
  double* xhat = C.xhat;
  double* sc = C.s;
  if (st->k >= st->iters || st->pass_skip) return;
  __shared__ double bins[kPackCols][kNarrowBins];
  __shared__ double sbeta[kPackCols], salpha[kPackCols], sxb[kPackCols], sl[kPackCols], su[kPackCols];
  __shared__ unsigned long long scand[kPackCols];
  __shared__ int sstart[kPackCols + 1];
  const int tid = threadIdx.x;
  const PackTask T = C.plan.packs[lb];
  const int nc = T.q_end - T.q_begin;
  if (tid < nc) {
    const int q = T.q_begin + tid;
    sxb[tid] = x[q];
    sl[tid] = P.lb[q];
    su[tid] = P.ub[q];
    sstart[tid] = P.col_ptr[q];
    sbeta[tid] = 0.0;
    salpha[tid] = 0.0;
    scand[tid] = 0ull;
  }
  if (tid == 0) sstart[nc] = P.col_ptr[T.q_end];
  for (int i = tid; i < nc * kNarrowBins; i += blockDim.x) bins[i / kNarrowBins][i % kNarrowBins] = 0.0;
  __syncthreads();
  const double eps = P.eps;
  const int e0 = sstart[0], e1 = sstart[nc];
  // Each thread takes kPackRun consecutive entries per step (the loads of a
  // run are issued together); runs mostly stay inside one column, so beta,
  // alpha and the candidate mask are summed in registers and added to LDS
  // once per column change instead of once per entry.
  constexpr int kPackRun = 4;
  const int step = blockDim.x * kPackRun;
  for (int base = e0 + tid * kPackRun; base < e1; base += step) {
    const int cnt = min(kPackRun, e1 - base);
    int row[kPackRun];
    double a[kPackRun];
    RowState r[kPackRun];
#pragma unroll
    for (int u = 0; u < kPackRun; ++u)
      if (u < cnt) {
        row[u] = P.col_row[base + u];
        a[u] = P.col_val[base + u];
      }
#pragma unroll
    for (int u = 0; u < kPackRun; ++u)
      if (u < cnt) r[u] = rs[row[u]];
    int lo = 0, hi = nc - 1;  // largest slot with sstart[slot] <= base
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (sstart[mid] <= base)
        lo = mid;
      else
        hi = mid - 1;
    }
    int slot = lo;
    double db = 0.0, da = 0.0;
    unsigned long long dc = 0ull;
#pragma unroll
    for (int u = 0; u < kPackRun; ++u) {
      if (u >= cnt) break;
      while (base + u >= sstart[slot + 1]) {
        if (db != 0.0) atomicAdd(&sbeta[slot], db);
        if (da != 0.0) atomicAdd(&salpha[slot], da);
        if (dc) atomicOr(&scand[slot], dc);
        db = 0.0;
        da = 0.0;
        dc = 0ull;
        ++slot;
      }
      const double xb = sxb[slot], l = sl[slot], u2 = su[slot];
      const int W = (int)(u2 - l) + 1;
      narrow_entry(xb, r[u].r, a[u], (double)r[u].w0, eps, l, u2, W, bins[slot], db, da, dc);
      if (r[u].w1 >= 0.0f) narrow_entry(xb, -r[u].r, -a[u], (double)r[u].w1, eps, l, u2, W, bins[slot], db, da, dc);
    }
    if (db != 0.0) atomicAdd(&sbeta[slot], db);
    if (da != 0.0) atomicAdd(&salpha[slot], da);
    if (dc) atomicOr(&scand[slot], dc);
  }
  if (tid < nc && st->cut_active) {
    const double c = P.obj[T.q_begin + tid];
    if (c != 0.0) {
      const double xb = sxb[tid], l = sl[tid], u = su[tid];
      double db = 0.0, da = 0.0;
      unsigned long long dc = 0ull;
      narrow_entry(xb, st->rc, c, (double)st->wc, eps, l, u, (int)(u - l) + 1, bins[tid], db, da, dc);
      if (db != 0.0) atomicAdd(&sbeta[tid], db);
      if (da != 0.0) atomicAdd(&salpha[tid], da);
      if (dc) atomicOr(&scand[tid], dc);
    }
  }
  __syncthreads();
  const int lane = tid & (kWave - 1);
  for (int slot = tid >> 6; slot < nc; slot += (int)(blockDim.x >> 6)) {
    const double l = sl[slot], xb = sxb[slot];
    const int W = (int)(su[slot] - l) + 1;
    bool found;
    double best, bestp;
    narrow_finish(bins[slot][lane], sbeta[slot], salpha[slot], scand[slot], xb, l, W, lane, found, best, bestp);
    if (lane == 0) write_result(xhat, sc, T.q_begin + slot, found, best, bestp, xb);
  }
}

// Offset of the cutoff row's breakpoint from xbar, clamped like the records.
__device__ __forceinline__ int cutoff_offset(double xb, const WalkState* st, double c, double eps) {
  const double t = breakpoint(xb, st->rc, c, eps, true);
  return (int)fmin(fmax(t - xb, -(double)kStageClamp), (double)kStageClamp);
}

// Coefficients, in half weights, of beta, alpha and delta of a row for the
// six cases of phase1() (index 3 [a > 0] + sign(d) + 1): 4-bit fields.
constexpr uint32_t pack6(int c0, int c1, int c2, int c3, int c4, int c5) {
  return (uint32_t)(c0 & 15) | (uint32_t)(c1 & 15) << 4 | (uint32_t)(c2 & 15) << 8 | (uint32_t)(c3 & 15) << 12 |
         (uint32_t)(c4 & 15) << 16 | (uint32_t)(c5 & 15) << 20;
}
constexpr uint32_t kCoefBeta = pack6(-2, -2, -1, 2, 0, 0);
constexpr uint32_t kCoefAlpha = pack6(0, 2, 2, -2, -2, 0);
constexpr uint32_t kCoefDelta = pack6(2, 0, 1, -1, 0, -2);
__device__ __forceinline__ int row_coef(uint32_t packed, int cs) { return ((int)(packed << (28 - 4 * cs))) >> 28; }

// One row of a long column (one column per workgroup) in half weights:
// beta, alpha and the candidate mask summed by the caller, delta into the
// bins (the cases of phase1() in offset form, as add_row).
__device__ __forceinline__ void add_row_reg(bool ap, int d, int32_t half, int k0, int W, int32_t* bins,
                                            int32_t& beta, int32_t& alpha, unsigned long long& cand) {
  const int cs = (ap ? 4 : 1) + (d > 0 ? 1 : 0) - (d < 0 ? 1 : 0);
  beta += row_coef(kCoefBeta, cs) * half;
  alpha += row_coef(kCoefAlpha, cs) * half;
  if (d == 0) return;
  const int32_t dl = row_coef(kCoefDelta, cs) * half;
  const int k = k0 + d;
  if (k < 0) {
    beta += dl;
    return;
  }
  if (k >= W) return;
  cand |= 1ull << k;
  const int kb = k + (ap ? 1 : 0);
  if (kb < W) atomicAdd(&bins[kb], dl);
}

// One workgroup per chunk of a long narrow column: bins, beta, alpha and the
// candidate mask of the chunk go to the chunk's partial record. Chunks are
// cut along row ranges and ordered so that consecutive workgroups (placed on
// consecutive XCDs) gather rows from one range each.
struct ChunkSmem {
  double bins[kNarrowBins];
  int32_t ibins[kNarrowBins];
  double red_b[4], red_a[4];
  unsigned long long red_c[4];
};

template <typename Rows>
__device__ __forceinline__ void chunk_task(const WalkCtx& C, int lb, ChunkSmem& S) {
  const DevProblem& P = C.P;
  const double* x = C.x;
  const Rows rs = rows_of<Rows>(C);
  const WalkState* st = C.st;
  ChunkPartial* partials = C.partials;
  if (st->k >= st->iters || st->pass_skip) return;
  double* bins = S.bins;
  int32_t* ibins = S.ibins;
  double* red_b = S.red_b;
  double* red_a = S.red_a;
  unsigned long long* red_c = S.red_c;
  const int tid = threadIdx.x;
  const int lane = tid & (kWave - 1);
  const int wv = tid >> 6;
  const ChunkTask T = C.plan.chunks[lb];
  // integer data with integral weights: breakpoint offsets from one quotient
  // and half-weight integer bins (the identity of row-block staging)
  const bool exact = C.plan.stage_exact != 0 && stage_weights<Rows>(C);
  if (tid < kNarrowBins) {
    bins[tid] = 0.0;
    ibins[tid] = 0;
  }
  __syncthreads();
  double beta = 0.0, alpha = 0.0;
  unsigned long long cand = 0;
  if (T.col >= 0 && exact) {
    const int q = T.col;
    const double xb = gmem(x)[q];
    const double l = gmem(P.lb)[q];
    const int W = (int)(gmem(P.ub)[q] - l) + 1, k0 = (int)(xb - l);
    const gptr<const int32_t> crow = gmem(P.col_row);
    const gptr<const double> cval = gmem(P.col_val);
    int32_t ib = 0, ia = 0;
    int e = T.e_beg + tid;
    // software pipeline: the next step's row indices and coefficients are in
    // flight while this step's rows are gathered and binned
    int ni0 = 0, ni1 = 0;
    double na0 = 0.0, na1 = 0.0;
    if (e < T.e_end) {
      ni0 = __builtin_nontemporal_load(&crow[e]);
      na0 = __builtin_nontemporal_load(&cval[e]);
      if (e + 256 < T.e_end) {
        ni1 = __builtin_nontemporal_load(&crow[e + 256]);
        na1 = __builtin_nontemporal_load(&cval[e + 256]);
      }
    }
    for (; e < T.e_end; e += 512) {
      const bool two = e + 256 < T.e_end;
      const int i0 = ni0;
      const double a0 = na0;
      const int i1 = two ? ni1 : i0;
      const double a1 = two ? na1 : a0;
      const RowState r0 = rs[i0];
      const RowState r1 = rs[i1];
      const int en = e + 512;
      if (en < T.e_end) {
        ni0 = __builtin_nontemporal_load(&crow[en]);
        na0 = __builtin_nontemporal_load(&cval[en]);
        if (en + 256 < T.e_end) {
          ni1 = __builtin_nontemporal_load(&crow[en + 256]);
          na1 = __builtin_nontemporal_load(&cval[en + 256]);
        }
      }
#pragma unroll
      for (int u = 0; u < 2; ++u) {
        if (u == 1 && !two) break;
        const RowState& r = u ? r1 : r0;
        const double a = u ? a1 : a0;
        const bool ap = a > 0.0;
        const double qv = -r.r / a;
        const double fl = fmin(fmax(floor(qv), -(double)kStageClamp), (double)kStageClamp);
        const double ce = fmin(fmax(ceil(qv), -(double)kStageClamp), (double)kStageClamp);
        add_row_reg(ap, (int)(ap ? fl : ce), (int32_t)r.w0, k0, W, ibins, ib, ia, cand);
        if (r.w1 >= 0.0f) add_row_reg(!ap, (int)(ap ? ce : fl), (int32_t)r.w1, k0, W, ibins, ib, ia, cand);
      }
    }
    if (tid == 0 && T.first && st->cut_active) {
      const double c = P.obj[q];
      if (c != 0.0)
        add_row_reg(c > 0.0, cutoff_offset(xb, st, c, P.eps), (int32_t)st->wc, k0, W, ibins, ib, ia, cand);
    }
    beta = 0.5 * (double)ib;
    alpha = 0.5 * (double)ia;
  } else if (T.col >= 0) {
    const int q = T.col;
    const double eps = P.eps;
    const double xb = gmem(x)[q];
    const double l = gmem(P.lb)[q], u2 = gmem(P.ub)[q];
    const gptr<const int32_t> crow = gmem(P.col_row);
    const gptr<const double> cval = gmem(P.col_val);
    const int W = (int)(u2 - l) + 1;
    int e = T.e_beg + tid;
    // two entries per step: both gathers are issued before either is used
    for (; e + 256 < T.e_end; e += 512) {
      const int i0 = __builtin_nontemporal_load(&crow[e]);
      const int i1 = __builtin_nontemporal_load(&crow[e + 256]);
      const double a0 = __builtin_nontemporal_load(&cval[e]);
      const double a1 = __builtin_nontemporal_load(&cval[e + 256]);
      const RowState r0 = rs[i0];
      const RowState r1 = rs[i1];
      narrow_entry(xb, r0.r, a0, (double)r0.w0, eps, l, u2, W, bins, beta, alpha, cand);
      if (r0.w1 >= 0.0f) narrow_entry(xb, -r0.r, -a0, (double)r0.w1, eps, l, u2, W, bins, beta, alpha, cand);
      narrow_entry(xb, r1.r, a1, (double)r1.w0, eps, l, u2, W, bins, beta, alpha, cand);
      if (r1.w1 >= 0.0f) narrow_entry(xb, -r1.r, -a1, (double)r1.w1, eps, l, u2, W, bins, beta, alpha, cand);
    }
    if (e < T.e_end) {
      const int i0 = __builtin_nontemporal_load(&crow[e]);
      const double a0 = __builtin_nontemporal_load(&cval[e]);
      const RowState r0 = rs[i0];
      narrow_entry(xb, r0.r, a0, (double)r0.w0, eps, l, u2, W, bins, beta, alpha, cand);
      if (r0.w1 >= 0.0f) narrow_entry(xb, -r0.r, -a0, (double)r0.w1, eps, l, u2, W, bins, beta, alpha, cand);
    }
    if (tid == 0 && T.first && st->cut_active) {
      const double c = P.obj[q];
      if (c != 0.0) narrow_entry(xb, st->rc, c, (double)st->wc, eps, l, u2, W, bins, beta, alpha, cand);
    }
  }
  beta = wave_sum(beta);
  alpha = wave_sum(alpha);
  cand = wave_or(cand);
  if (lane == 0) {
    red_b[wv] = beta;
    red_a[wv] = alpha;
    red_c[wv] = cand;
  }
  __syncthreads();
  if (T.col < 0) return;
  const gptr<ChunkPartial> mine = gmem(partials) + T.slot;
  if (tid < kNarrowBins) mine->bins[tid] = exact ? 0.5 * (double)ibins[tid] : bins[tid];
  if (tid == 0) {
    mine->beta = red_b[0] + red_b[1] + red_b[2] + red_b[3];
    mine->alpha = red_a[0] + red_a[1] + red_a[2] + red_a[3];
    mine->cand = red_c[0] | red_c[1] | red_c[2] | red_c[3];
  }
}

template <typename Rows>
__global__ __launch_bounds__(256) void k_narrow_chunk(const WalkCtx* __restrict__ walks,
                                                      const int32_t* __restrict__ off, int32_t nw) {
  int lb;
  const int w_ = block_walk(off, nw, lb);
  if (w_ < 0) return;
  const WalkCtx& C = walks[w_];
  __shared__ ChunkSmem S;
  chunk_task<Rows>(C, lb, S);
}

// One wavefront per long narrow column.
__global__ __launch_bounds__(256) void k_narrow_combine(const WalkCtx* __restrict__ walks,
                                                        const int32_t* __restrict__ off, int32_t nw) {
  int lb;
  const int w_ = block_walk(off, nw, lb);
  if (w_ < 0) return;
  const WalkCtx& W0 = walks[w_];
  if (W0.st->k >= W0.st->iters || W0.st->pass_skip) return;
  const int idx = lb * 4 + (threadIdx.x >> 6);
  if (idx >= W0.plan.n_chunk_cols) return;
  int q;
  (void)combine_col(W0, idx, threadIdx.x & (kWave - 1), &q);
}

// ---------------------------------------------------------------------------
// Row-range staging (all-integer instances).
// ---------------------------------------------------------------------------

// Staged scoring keeps values as int32 counts of half weights when the
// weights are integers (every term is a multiple of w/2: exact), else FP64.
__device__ __forceinline__ int32_t stage_one(double w, int32_t) { return 2 * (int32_t)w; }
__device__ __forceinline__ int32_t stage_half(double w, int32_t) { return (int32_t)w; }
__device__ __forceinline__ double stage_one(double w, double) { return w; }
__device__ __forceinline__ double stage_half(double w, double) { return 0.5 * w; }
__device__ __forceinline__ double stage_score_of(int32_t v) { return 0.5 * (double)v; }
__device__ __forceinline__ double stage_score_of(double v) { return v; }

// One normalised row of a narrow column in offset form (coefficient sign ap,
// breakpoint t = xbar + d, one = w and half = w/2 in value units): the cases
// of Algorithm 1 phase 1, as phase1() takes them, decided by the sign of d.
// The row adds beta at every position, alpha above xbar and delta from
// offset thr on (thr = d, or d + 1 when the row holds after t).
template <typename V>
__device__ __forceinline__ void row_terms(bool ap, int d, V one, V half, V& beta, V& alpha, V& delta, int& thr) {
  if (ap) {
    thr = d + 1;
    if (d < 0) {
      beta += one;
      alpha -= one;
      delta = -half;
    } else if (d > 0) {
      delta = -one;
    } else {
      alpha -= one;
      delta = 0;
    }
  } else {
    thr = d;
    if (d > 0) {
      beta -= half;
      alpha += one;
      delta = half;
    } else if (d < 0) {
      beta -= one;
      delta = one;
    } else {
      beta -= one;
      alpha += one;
      delta = 0;
    }
  }
}

// The same row added to a column's bins (k0 = xbar - l, W values; half =
// w/2 in value units): beta goes to bin 0, alpha to bin k0 + 1 (the first
// position above xbar), delta to the bin where it starts to apply (bin 0 when
// that is below l, the sink bin kNarrowBins when above u). The breakpoint is
// a candidate when inside [l, u].
template <typename V>
__device__ __forceinline__ void add_row(bool ap, int d, V half, int k0, int W, V* bins, unsigned long long* cand) {
  const int cs = (ap ? 4 : 1) + (d > 0 ? 1 : 0) - (d < 0 ? 1 : 0);
  const V b = (V)row_coef(kCoefBeta, cs) * half;
  const V al = (V)row_coef(kCoefAlpha, cs) * half;
  const V dl = (V)row_coef(kCoefDelta, cs) * half;
  const int k = k0 + d;
  const int kb = k + (ap ? 1 : 0);
  const int idx = k < 0 ? 0 : ((k >= W || kb >= W) ? kNarrowBins : kb);
  const int ia = k0 + 1 < W ? k0 + 1 : kNarrowBins;
  const V zero = 0;
  if (b != zero) atomicAdd(&bins[0], b);
  if (al != zero) atomicAdd(&bins[ia], al);
  if (dl != zero) atomicAdd(&bins[idx], dl);
  if (d != 0 && k >= 0 && k < W) atomicOr(cand, 1ull << k);
}

// add_row for a run of rows of one column: beta, alpha and the candidate
// mask go to the caller's registers (flushed once per run), the delta to its
// bin; deltas for bin 0 join beta, those beyond u (the sink bin, never read)
// are dropped.
template <typename V>
__device__ __forceinline__ void add_row_run(bool ap, int d, V half, int k0, int W, V* bins, V& beta, V& alpha,
                                            unsigned long long& cand) {
  const int cs = (ap ? 4 : 1) + (d > 0 ? 1 : 0) - (d < 0 ? 1 : 0);
  beta += (V)row_coef(kCoefBeta, cs) * half;
  alpha += (V)row_coef(kCoefAlpha, cs) * half;
  const V dl = (V)row_coef(kCoefDelta, cs) * half;
  const int k = k0 + d;
  const int kb = k + (ap ? 1 : 0);
  if (dl != (V)0) {
    if (k < 0)
      beta += dl;
    else if (k < W && kb < W)
      atomicAdd(&bins[kb], dl);
  }
  if (d != 0 && k >= 0 && k < W) cand |= 1ull << k;
}

struct StageRec {
  bool ap, twin;
  int d0, d1, lc;
  double w0, w1;
};

template <typename Rows>
__device__ __forceinline__ StageRec decode_rec(uint64_t r, bool wts, const Rows& rs) {
  StageRec o;
  o.lc = (int)(r & 0xFFu);
  o.ap = (r >> 8) & 1u;
  o.twin = (r >> 9) & 1u;
  o.d0 = (int)((r >> 10) & 0xFFu) - kStageClamp;
  o.d1 = (int)((r >> 18) & 0xFFu) - kStageClamp;
  if (wts) {
    o.w0 = (double)((r >> 32) & 0xFFFFu);
    o.w1 = (double)(r >> 48);
  } else {
    const RowState g = rs[(int)(r >> 32)];
    o.w0 = (double)g.w0;
    o.w1 = (double)g.w1;
  }
  return o;
}


template <typename V>
struct StagePackSmem {
  // columns binned at once: a whole pack with int32 values, half of one with
  // FP64 values (which then takes two passes over the records)
  static constexpr int kCols = sizeof(V) == 4 ? kStagePackCols : kStagePackCols / 2;
  V bins[kCols][kNarrowBins + 1];  // padded: lane c reads row c without bank conflicts
  unsigned long long cand[kCols];
  double xb[kCols];
  int32_t W[kCols], k0[kCols];
};

struct StageShortSmem {
  uint64_t rec[kShortMax][kStageShort];  // slot-major: thread c reads rec[*][c]
  int32_t cnt[kStageShort];
};

// Segment table of scoring task t in LDS: beg[rb] = first record of the
// task in row block rb, pre[rb] = the task's records in blocks before rb
// (pre[nrb] = all of them). Ends with a barrier.
struct StageSegs {
  int32_t beg[kStageMaxRb];
  int32_t pre[kStageMaxRb + 1];
};

__device__ __forceinline__ int stage_segments(const WalkCtx& C, int t, StageSegs& G) {
  const int nrb = C.plan.n_stage_rb;
  const int per = 2 * nrb + 1;
  const gptr<const int32_t> tab = gmem(C.plan.stage_seg + (size_t)t * per);
  for (int k = threadIdx.x; k < per; k += blockDim.x) {
    const int32_t v = tab[k];
    if (k < nrb)
      G.beg[k] = v;
    else
      G.pre[k - nrb] = v;
  }
  __syncthreads();
  return G.pre[nrb];
}

// A pack of narrow columns from its records: counting sort into LDS bins
// that also hold beta (bin 0) and alpha (bin xbar - l + 1), so the score of
// position l + k is the prefix sum of bins 0..k; one lane per column then
// scans its bins and keeps the best candidate (smallest position on ties).
template <typename Rows, typename V>
__device__ __forceinline__ void stage_pack(const WalkCtx& C, const Rows& rs, bool wts, int tix, StagePackSmem<V>& S,
                                           StageSegs& G) {
  constexpr int kCols = StagePackSmem<V>::kCols;
  const StageTask T = C.plan.stage_tasks[tix];
  const DevProblem& P = C.P;
  const WalkState* st = C.st;
  const int tid = threadIdx.x;
  const int nc = T.q_end - T.q_begin;
  const V zero = 0;
  const int nrb = C.plan.n_stage_rb;
  stage_segments(C, tix, G);
  const gptr<const uint64_t> recs = gmem((const uint64_t*)C.stage_rec);
  for (int c0 = 0; c0 < nc; c0 += kCols) {
    const int ncw = min(kCols, nc - c0);
    if (tid < ncw) {
      const int q = T.q_begin + c0 + tid;
      const double xb = gmem((const double*)C.x)[q], l = gmem(P.lb)[q];
      S.xb[tid] = xb;
      S.W[tid] = (int)(gmem(P.ub)[q] - l) + 1;
      S.k0[tid] = (int)(xb - l);
      S.cand[tid] = 0ull;
    }
    for (int i = tid; i < ncw * (kNarrowBins + 1); i += blockDim.x)
      S.bins[i / (kNarrowBins + 1)][i % (kNarrowBins + 1)] = 0;
    __syncthreads();
    // every thread takes an equal contiguous share of the task's records (in
    // segment order, crossing row-block segments), kRun records per step;
    // records of columns outside this window are skipped
    constexpr int kRun = 4;
    {
      const int total = G.pre[nrb];
      const int per = (total + (int)blockDim.x - 1) / (int)blockDim.x;
      const int f0 = min(total, tid * per), f1 = min(total, f0 + per);
      // segment of f0: the last one starting at or before it
      int lo = 0, hi = nrb - 1;
      while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (G.pre[mid] <= f0)
          lo = mid;
        else
          hi = mid - 1;
      }
      int sg = lo;
      int base = G.beg[sg] - G.pre[sg];  // record index of flat position f: base + f
      int send = G.pre[sg + 1];
      // a thread's run is sorted by column within a segment: beta, alpha and
      // the candidate mask of the current column stay in registers until the
      // column changes
      int cur = -1, k0 = 0, W = 0;
      V rb_ = 0, ra_ = 0;
      unsigned long long rc_ = 0ull;
      auto flush = [&]() {
        if (cur < 0) return;
        if (rb_ != zero) atomicAdd(&S.bins[cur][0], rb_);
        if (ra_ != zero && k0 + 1 < W) atomicAdd(&S.bins[cur][k0 + 1], ra_);
        if (rc_) atomicOr(&S.cand[cur], rc_);
        rb_ = zero;
        ra_ = zero;
        rc_ = 0ull;
      };
      for (int f = f0; f < f1; f += kRun) {
        uint64_t r[kRun];
#pragma unroll
        for (int u = 0; u < kRun; ++u) {
          const int fu = f + u;
          if (fu < f1) {
            while (fu >= send) {
              ++sg;
              base = G.beg[sg] - G.pre[sg];
              send = G.pre[sg + 1];
            }
            r[u] = recs[base + fu];
          }
        }
#pragma unroll
        for (int u = 0; u < kRun; ++u) {
          if (f + u < f1) {
            const int lc = (int)(r[u] & 0xFFu) - c0;
            if (lc < 0 || lc >= ncw) continue;
            if (lc != cur) {
              flush();
              cur = lc;
              k0 = S.k0[lc];
              W = S.W[lc];
            }
            const StageRec e = decode_rec(r[u], wts, rs);
            add_row_run(e.ap, e.d0, stage_half(e.w0, zero), k0, W, S.bins[lc], rb_, ra_, rc_);
            if (e.twin) add_row_run(!e.ap, e.d1, stage_half(e.w1, zero), k0, W, S.bins[lc], rb_, ra_, rc_);
          }
        }
      }
      flush();
    }
    if (tid < ncw && st->cut_active) {
      const double c = gmem(P.obj)[T.q_begin + c0 + tid];
      if (c != 0.0) {
        const double wc = (double)st->wc;
        add_row(c > 0.0, cutoff_offset(S.xb[tid], st, c, P.eps), stage_half(wc, zero), S.k0[tid], S.W[tid],
                S.bins[tid], &S.cand[tid]);
      }
    }
    __syncthreads();
    if (tid < ncw) {
      const int W = S.W[tid], k0 = S.k0[tid];
      const unsigned long long cand = S.cand[tid];
      const uint32_t clo = (uint32_t)cand, chi = (uint32_t)(cand >> 32);
      V acc = 0, best = 0;
      int bk = -1;
#pragma unroll
      for (int k = 0; k < kNarrowBins; ++k) {
        if (k < W) {
          acc += S.bins[tid][k];
          const bool bit = k < 32 ? ((clo >> k) & 1u) != 0 : ((chi >> (k - 32)) & 1u) != 0;
          const bool ok = (bit || k == 0 || k == W - 1) && k != k0;
          if (ok && (bk < 0 || acc > best)) {
            best = acc;
            bk = k;
          }
        }
      }
      const double xb = S.xb[tid];
      write_result(gmem(C.xhat), gmem(C.s), T.q_begin + c0 + tid, bk >= 0, stage_score_of(best),
                   xb + (double)(bk - k0), xb);
    }
    __syncthreads();  // the next window reuses the LDS
  }
}

__device__ __forceinline__ void cswap_u64(uint64_t& a, uint64_t& b) {
  const uint64_t lo = a < b ? a : b, hi = a < b ? b : a;
  a = lo;
  b = hi;
}

// One short narrow column with D stored entries (decoded records e[0..D-1])
// scored directly: value(c) = beta + alpha [c >= 1] + sum of delta [c >= thr]
// at the candidate offsets c (both bounds, breakpoints inside [l, u]; c = 0
// is xbar and excluded), the largest value, the smallest position on ties.
template <int D, typename V>
__device__ __forceinline__ void stage_short_col(const StageRec* e, double xb, int k0, int W, bool cut, bool cpos,
                                                int dcut, double wc, bool& found, double& best, double& bestp) {
  constexpr int NR = 2 * D + 1;
  const V zero = 0;
  V beta = 0, alpha = 0;
  V dl[NR];
  int th[NR], cd[NR];
  bool cv[NR];
#pragma unroll
  for (int k = 0; k < D; ++k) {
    row_terms(e[k].ap, e[k].d0, stage_one(e[k].w0, zero), stage_half(e[k].w0, zero), beta, alpha, dl[2 * k],
              th[2 * k]);
    cd[2 * k] = e[k].d0;
    cv[2 * k] = true;
    if (e[k].twin) {
      row_terms(!e[k].ap, e[k].d1, stage_one(e[k].w1, zero), stage_half(e[k].w1, zero), beta, alpha,
                dl[2 * k + 1], th[2 * k + 1]);
      cd[2 * k + 1] = e[k].d1;
      cv[2 * k + 1] = true;
    } else {
      dl[2 * k + 1] = 0;
      th[2 * k + 1] = 0;
      cd[2 * k + 1] = 0;
      cv[2 * k + 1] = false;
    }
  }
  if (cut) {
    row_terms(cpos, dcut, stage_one(wc, zero), stage_half(wc, zero), beta, alpha, dl[NR - 1], th[NR - 1]);
    cd[NR - 1] = dcut;
    cv[NR - 1] = true;
  } else {
    dl[NR - 1] = 0;
    th[NR - 1] = 0;
    cd[NR - 1] = 0;
    cv[NR - 1] = false;
  }
  const int lo = -k0, hi = W - 1 - k0;
  V bv = 0;
  int bc = 0;
  found = false;
  auto consider = [&](int c) {
    if (c < lo || c > hi || c == 0) return;
    V val = beta + (c >= 1 ? alpha : zero);
#pragma unroll
    for (int j = 0; j < NR; ++j) val += (c >= th[j]) ? dl[j] : zero;
    if (!found || val > bv || (val == bv && c < bc)) {
      found = true;
      bv = val;
      bc = c;
    }
  };
  consider(lo);
  consider(hi);
#pragma unroll
  for (int j = 0; j < NR; ++j)
    if (cv[j]) consider(cd[j]);
  best = stage_score_of(bv);
  bestp = xb + (double)bc;
}

// The integer case of stage_short_col for a column whose records sit in LDS
// slots rec[k][lane]: the records are decoded one at a time into thresholds
// and half-weight deltas, and the breakpoint of each term is its threshold,
// or one less where bit j of `below` is set (a row that holds after its
// breakpoint). Two registers per term, so a short group's workgroup keeps
// the occupancy of the other scoring kernels.
template <int D>
__device__ __forceinline__ void stage_short_int(const StageShortSmem& S, int lane, double xb, int k0, int W, bool cut,
                                                bool cpos, int dcut, int32_t wc, bool& found, double& best,
                                                double& bestp) {
  constexpr int NR = 2 * D + 1;
  constexpr int kNone = 127;  // threshold of an absent term: above every offset
  int32_t beta = 0, alpha = 0;
  int32_t dl[NR];
  int th[NR];
  uint32_t below = 0;
#pragma unroll
  for (int k = 0; k < D; ++k) {
    const uint64_t r = S.rec[k][lane];
    const bool ap = (r >> 8) & 1u;
    const int d0 = (int)((r >> 10) & 0xFFu) - kStageClamp;
    const int32_t w0 = (int32_t)((r >> 32) & 0xFFFFu);
    row_terms(ap, d0, 2 * w0, w0, beta, alpha, dl[2 * k], th[2 * k]);
    below |= (uint32_t)ap << (2 * k);
    if ((r >> 9) & 1u) {
      const int d1 = (int)((r >> 18) & 0xFFu) - kStageClamp;
      const int32_t w1 = (int32_t)(r >> 48);
      row_terms(!ap, d1, 2 * w1, w1, beta, alpha, dl[2 * k + 1], th[2 * k + 1]);
      below |= (uint32_t)(!ap) << (2 * k + 1);
    } else {
      dl[2 * k + 1] = 0;
      th[2 * k + 1] = kNone;
    }
  }
  if (cut) {
    row_terms(cpos, dcut, 2 * wc, wc, beta, alpha, dl[NR - 1], th[NR - 1]);
    below |= (uint32_t)cpos << (NR - 1);
  } else {
    dl[NR - 1] = 0;
    th[NR - 1] = kNone;
  }
  const int lo = -k0, hi = W - 1 - k0;
  int32_t bv = 0;
  int bc = 0;
  found = false;
  auto consider = [&](int c) {
    if (c < lo || c > hi || c == 0) return;
    int32_t val = beta + (c >= 1 ? alpha : 0);
#pragma unroll
    for (int j = 0; j < NR; ++j) val += (c >= th[j]) ? dl[j] : 0;
    if (!found || val > bv || (val == bv && c < bc)) {
      found = true;
      bv = val;
      bc = c;
    }
  };
  consider(lo);
  consider(hi);
#pragma unroll
  for (int j = 0; j < NR; ++j) consider(th[j] - (int)((below >> j) & 1u));
  best = stage_score_of(bv);
  bestp = xb + (double)bc;
}

// The FP64 case (weights gathered from the row states) in the same form:
// the records are decoded one at a time from the LDS slots, which the
// caller has sorted, so a lane holds three registers per term.
template <int D, typename Rows>
__device__ __forceinline__ void stage_short_dbl(const StageShortSmem& S, int lane, const Rows& rs, double xb, int k0,
                                                int W, bool cut, bool cpos, int dcut, double wc, bool& found,
                                                double& best, double& bestp) {
  constexpr int NR = 2 * D + 1;
  constexpr int kNone = 127;
  const double zero = 0.0;
  double beta = 0.0, alpha = 0.0;
  double dl[NR];
  int th[NR];
  uint32_t below = 0;
#pragma unroll
  for (int k = 0; k < D; ++k) {
    const StageRec e = decode_rec<Rows>(S.rec[k][lane], false, rs);
    row_terms(e.ap != 0, e.d0, stage_one(e.w0, zero), stage_half(e.w0, zero), beta, alpha, dl[2 * k], th[2 * k]);
    below |= (uint32_t)(e.ap != 0) << (2 * k);
    if (e.twin) {
      row_terms(e.ap == 0, e.d1, stage_one(e.w1, zero), stage_half(e.w1, zero), beta, alpha, dl[2 * k + 1],
                th[2 * k + 1]);
      below |= (uint32_t)(e.ap == 0) << (2 * k + 1);
    } else {
      dl[2 * k + 1] = 0.0;
      th[2 * k + 1] = kNone;
    }
  }
  if (cut) {
    row_terms(cpos, dcut, stage_one(wc, zero), stage_half(wc, zero), beta, alpha, dl[NR - 1], th[NR - 1]);
    below |= (uint32_t)cpos << (NR - 1);
  } else {
    dl[NR - 1] = 0.0;
    th[NR - 1] = kNone;
  }
  const int lo = -k0, hi = W - 1 - k0;
  double bv = 0.0;
  int bc = 0;
  found = false;
  auto consider = [&](int c) {
    if (c < lo || c > hi || c == 0) return;
    double val = beta + (c >= 1 ? alpha : zero);
#pragma unroll
    for (int j = 0; j < NR; ++j) val += (c >= th[j]) ? dl[j] : zero;
    if (!found || val > bv || (val == bv && c < bc)) {
      found = true;
      bv = val;
      bc = c;
    }
  };
  consider(lo);
  consider(hi);
#pragma unroll
  for (int j = 0; j < NR; ++j) consider(th[j] - (int)((below >> j) & 1u));
  best = bv;
  bestp = xb + (double)bc;
}

template <typename Rows>
__device__ __forceinline__ void stage_short(const WalkCtx& C, const Rows& rs, bool wts, int tix, StageShortSmem& S,
                                            StageSegs& G) {
  const StageTask T = C.plan.stage_tasks[tix];
  const DevProblem& P = C.P;
  const WalkState* st = C.st;
  const int tid = threadIdx.x;
  const int nc = T.q_end - T.q_begin;
  const int D = T.deg;
  // the column's own data is loaded while the records arrive
  const int q = T.q_begin + min(tid, max(nc - 1, 0));
  const double xb = gmem((const double*)C.x)[q], l = gmem(P.lb)[q], ub = gmem(P.ub)[q], c = gmem(P.obj)[q];
  S.cnt[tid] = 0;  // stage_segments ends with a barrier
  const int nrb = C.plan.n_stage_rb;
  stage_segments(C, tix, G);
  const gptr<const uint64_t> recs = gmem((const uint64_t*)C.stage_rec);
  constexpr int kRun = 4;
  const int tps = max(1, (int)blockDim.x / nrb);
  for (int sg = tid / tps; sg < nrb; sg += (int)blockDim.x / tps) {
    const int len = G.pre[sg + 1] - G.pre[sg];
    const int per = (len + tps - 1) / tps;
    const int i1 = G.beg[sg] + min(len, (tid % tps + 1) * per);
    for (int i0 = G.beg[sg] + min(len, (tid % tps) * per); i0 < i1; i0 += kRun) {
      uint64_t r[kRun];
#pragma unroll
      for (int u = 0; u < kRun; ++u)
        if (i0 + u < i1) r[u] = recs[i0 + u];
#pragma unroll
      for (int u = 0; u < kRun; ++u)
        if (i0 + u < i1) {
          const int lc = (int)(r[u] & 0xFFu);
          const int k = atomicAdd(&S.cnt[lc], 1);
          S.rec[k][lc] = r[u];
        }
    }
  }
  __syncthreads();
  if (tid >= nc) return;
  const int W = (int)(ub - l) + 1, k0 = (int)(xb - l);
  const bool cut = st->cut_active && c != 0.0;
  const int dcut = cut ? cutoff_offset(xb, st, c, P.eps) : 0;
  bool found = false;
  double best = 0.0, bestp = xb;
  if (wts) {
    const int32_t wc = (int32_t)st->wc;
#define CHAP_SHORT_CASE(DD)                                                                   \
  case DD:                                                                                    \
    stage_short_int<DD>(S, tid, xb, k0, W, cut, c > 0.0, dcut, wc, found, best, bestp);      \
    break;
    switch (D) {
      CHAP_SHORT_CASE(0)
      CHAP_SHORT_CASE(1)
      CHAP_SHORT_CASE(2)
      CHAP_SHORT_CASE(3)
      CHAP_SHORT_CASE(4)
      CHAP_SHORT_CASE(5)
      CHAP_SHORT_CASE(6)
      CHAP_SHORT_CASE(7)
      default:
        CHAP_SHORT_CASE(8)
    }
#undef CHAP_SHORT_CASE
  } else {
    // records arrive in varying order; sort each lane's slots (in LDS) so
    // that sums of non-integral weights are formed in one order
    for (int i = 0; i + 1 < D; ++i)
      for (int k = 0; k + 1 < D - i; ++k) {
        const uint64_t a = S.rec[k][tid], b = S.rec[k + 1][tid];
        if (b < a) {
          S.rec[k][tid] = b;
          S.rec[k + 1][tid] = a;
        }
      }
    const double wc = (double)st->wc;
#define CHAP_SHORT_CASE(DD)                                                                                \
  case DD:                                                                                                 \
    stage_short_dbl<DD, Rows>(S, tid, rs, xb, k0, W, cut, c > 0.0, dcut, wc, found, best, bestp);          \
    break;
    switch (D) {
      CHAP_SHORT_CASE(0)
      CHAP_SHORT_CASE(1)
      CHAP_SHORT_CASE(2)
      CHAP_SHORT_CASE(3)
      CHAP_SHORT_CASE(4)
      CHAP_SHORT_CASE(5)
      CHAP_SHORT_CASE(6)
      CHAP_SHORT_CASE(7)
      default:
        CHAP_SHORT_CASE(8)
    }
#undef CHAP_SHORT_CASE
  }
  write_result(gmem(C.xhat), gmem(C.s), q, found, best, bestp, xb);
}

// One workgroup per slice of a row block's staged entries: the block's rows
// go to LDS (as GatherRow; weights only when the records carry them), then
// every entry of the slice becomes the record of the same index, and the
// slice's single-entry columns (their entry lies in this block) are scored.
template <typename Rows>
__device__ __forceinline__ void stage_rows_body(const WalkCtx& C, const StageRowTask& T, GatherRow* rows) {
  const Rows rs = rows_of<Rows>(C);
  const bool wts = stage_weights<Rows>(C);
  const int r0 = T.rb * kStageRowBlock;
  const int nr = min(kStageRowBlock, C.P.ms - r0);
  const gptr<const uint64_t> ent = gmem(C.plan.stage_ent);
  const gptr<uint64_t> rec = gmem(C.stage_rec);
  constexpr int kThreads = 512;
  constexpr int kU = 8;  // entries per thread and step, loaded before any is used
  const int tid = threadIdx.x;
  uint64_t wd[kU];
  auto load_step = [&](int base) {
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      const int i = base + u * kThreads;
      if (i < T.e_end) wd[u] = __builtin_nontemporal_load(&ent[i]);
    }
  };
  // the first step's entries are in flight while the row block is loaded
  load_step(T.e_beg + tid);
  {
    constexpr int kPer = kStageRowBlock / kThreads;
    if (compact_source(rs)) {
      // the compact copy already has the LDS format (weights included)
      const gptr<const GatherRow> src = gmem((const GatherRow*)C.grow);
      GatherRow g[kPer];
#pragma unroll
      for (int k = 0; k < kPer; ++k)
        if (tid + k * kThreads < nr) g[k] = gload(src, r0 + tid + k * kThreads);
#pragma unroll
      for (int k = 0; k < kPer; ++k)
        if (tid + k * kThreads < nr) rows[tid + k * kThreads] = g[k];
    } else {
      RowState g[kPer];
#pragma unroll
      for (int k = 0; k < kPer; ++k)
        if (tid + k * kThreads < nr) g[k] = rs[r0 + tid + k * kThreads];
#pragma unroll
      for (int k = 0; k < kPer; ++k)
        if (tid + k * kThreads < nr) {
          GatherRow o;
          o.r = (int32_t)g[k].r;
          o.w0 = wts ? (uint16_t)g[k].w0 : (uint16_t)0;
          o.w1 = g[k].w1 >= 0.0f ? (wts ? (uint16_t)g[k].w1 : (uint16_t)0) : kNoTwin;
          rows[tid + k * kThreads] = o;
        }
    }
  }
  __syncthreads();
  for (int base = T.e_beg + tid; base < T.e_end; base += kU * kThreads) {
    if (base != T.e_beg + tid) load_step(base);
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      const int i = base + u * kThreads;
      if (i < T.e_end) {
        const int local = (int)(wd[u] & 0xFFFFu);
        const GatherRow g = rows[local];
        const int a = ((int32_t)((uint32_t)(wd[u] >> 24) << 8)) >> 8;
        const double qv = -(double)g.r / (double)a;
        const double fl = fmin(fmax(floor(qv), -(double)kStageClamp), (double)kStageClamp);
        const double ce = fmin(fmax(ceil(qv), -(double)kStageClamp), (double)kStageClamp);
        const int d0 = (int)(a > 0 ? fl : ce);
        const int d1 = (int)(a > 0 ? ce : fl);
        const bool twin = g.w1 != kNoTwin;
        const uint32_t lo = (uint32_t)((wd[u] >> 16) & 0xFFu) | ((a > 0 ? 1u : 0u) << 8) | ((twin ? 1u : 0u) << 9) |
                            ((uint32_t)(d0 + kStageClamp) << 10) | ((uint32_t)(d1 + kStageClamp) << 18);
        const uint32_t top = wts ? ((uint32_t)g.w0 | ((uint32_t)g.w1 << 16)) : (uint32_t)(r0 + local);
        rec[i] = (uint64_t)lo | ((uint64_t)top << 32);
      }
    }
  }
  // single-entry columns of this block: scored here from the LDS rows
  const DevProblem& P = C.P;
  const WalkState* st = C.st;
  const bool cut_on = st->cut_active != 0;
  const double wc = (double)st->wc;
  const gptr<const int32_t> cptr = gmem(P.col_ptr), crow = gmem(P.col_row);
  const gptr<const double> cval = gmem(P.col_val), xg = gmem((const double*)C.x), lbg = gmem(P.lb),
                           ubg = gmem(P.ub), objg = gmem(P.obj);
  const gptr<double> xhat = gmem(C.xhat), sco = gmem(C.s);
  for (int q = T.c_beg + tid; q < T.c_end; q += kThreads) {
    const int e = cptr[q];
    const int row = crow[e];
    const double a = cval[e];
    const double xb = xg[q], l = lbg[q], u = ubg[q];
    const double c = cut_on ? objg[q] : 0.0;
    const GatherRow g = rows[row - r0];
    StageRec re;
    re.lc = 0;
    re.ap = a > 0.0;
    const double qv = -(double)g.r / a;
    const double fl = fmin(fmax(floor(qv), -(double)kStageClamp), (double)kStageClamp);
    const double ce = fmin(fmax(ceil(qv), -(double)kStageClamp), (double)kStageClamp);
    re.d0 = (int)(re.ap ? fl : ce);
    re.d1 = (int)(re.ap ? ce : fl);
    re.twin = g.w1 != kNoTwin;
    if (wts) {
      re.w0 = (double)g.w0;
      re.w1 = (double)g.w1;
    } else {
      const RowState full = rs[row];
      re.w0 = (double)full.w0;
      re.w1 = (double)full.w1;
    }
    const int W = (int)(u - l) + 1, k0 = (int)(xb - l);
    const bool cut = c != 0.0;
    const int dcut = cut ? cutoff_offset(xb, st, c, P.eps) : 0;
    bool found;
    double best, bestp;
    if (wts)
      stage_short_col<1, int32_t>(&re, xb, k0, W, cut, c > 0.0, dcut, wc, found, best, bestp);
    else
      stage_short_col<1, double>(&re, xb, k0, W, cut, c > 0.0, dcut, wc, found, best, bestp);
    write_result(xhat, sco, q, found, best, bestp, xb);
  }
}

// Single passes with caller weights (DualRows) choose the row source once
// per workgroup from the walk state and run the specialised body, so the
// kernel holds the registers of one row accessor, not of both.
template <typename Rows>
__global__ __launch_bounds__(512) void k_stage_rows(const WalkCtx* __restrict__ walks,
                                                    const int32_t* __restrict__ off, int32_t nw) {
  int lb;
  const int w_ = block_walk(off, nw, lb);
  if (w_ < 0) return;
  const WalkCtx& C = walks[w_];
  if (C.st->k >= C.st->iters || C.st->pass_skip) return;
  const StageRowTask T = C.plan.stage_rtasks[lb];
  if (T.rb < 0) return;
  __shared__ GatherRow rows[kStageRowBlock];
  if constexpr (std::is_same<Rows, DualRows>::value) {
    if (C.st->compact_rows)
      stage_rows_body<CompactRows>(C, T, rows);
    else
      stage_rows_body<FullRows>(C, T, rows);
  } else {
    stage_rows_body<Rows>(C, T, rows);
  }
}

// Workgroups of a walk over ntask scoring tasks: kXcds * ceil(ntask / kXcds)
// of them, workgroup lb taking task (lb mod kXcds) * ceil(ntask / kXcds) +
// lb / kXcds, so that each XCD scores a contiguous run of tasks (whose
// segments share cache lines); -1 for the padding.
__device__ __forceinline__ int stage_task_of(int lb, int ntask) {
  const int per = (ntask + kXcds - 1) / kXcds;
  const int t = (lb % kXcds) * per + lb / kXcds;
  return t < ntask ? t : -1;
}

__host__ __device__ inline int32_t stage_blocks(int32_t ntask) { return kXcds * ((ntask + kXcds - 1) / kXcds); }

// The scoring of a staged pass in one launch: the long-column chunks, the packs and the short groups are units of kXcds
// workgroups of one grid, interleaved so that every CU runs latency-bound
// gathers beside VALU-bound scoring; a role's workgroups keep their
// XCD-aware task order. One launch on one stream, instead of three on three,
// keeps the iteration a chain of kernels without event hops between them.
union StageScoreSmem {
  ChunkSmem chunk;
  StagePackSmem<int32_t> pack_i;
  StagePackSmem<double> pack_d;
  StageShortSmem sh;
};

template <typename Rows>
__device__ __forceinline__ void stage_score_body(const WalkCtx& C, int lb, StageScoreSmem& sm, StageSegs& G) {
  const int32_t unit = gmem(C.plan.stage_units)[lb / kXcds];
  const int role = unit >> 28;
  const int rb = (unit & kStageUnitMask) * kXcds + lb % kXcds;
  if (role == 0) {
    chunk_task<Rows>(C, rb, sm.chunk);
    return;
  }
  const int npk = C.plan.n_stage_packs;
  const Rows rs = rows_of<Rows>(C);
  const bool wts = stage_weights<Rows>(C);
  if (role == 1) {
    const int t = stage_task_of(rb, npk);
    if (t < 0) return;
    if (wts)
      stage_pack<Rows, int32_t>(C, rs, true, t, sm.pack_i, G);
    else
      stage_pack<Rows, double>(C, rs, false, t, sm.pack_d, G);
    return;
  }
  const int t = stage_task_of(rb, C.plan.n_stage_tasks - npk);
  if (t >= 0) stage_short<Rows>(C, rs, wts, npk + t, sm.sh, G);
}

template <typename Rows>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(8))) void k_stage_score(
    const WalkCtx* __restrict__ walks, const int32_t* __restrict__ off, int32_t nw) {
  int lb;
  const int w_ = block_walk(off, nw, lb);
  if (w_ < 0) return;
  const WalkCtx& C = walks[w_];
  if (C.st->k >= C.st->iters || C.st->pass_skip) return;
  __shared__ StageScoreSmem sm;
  __shared__ StageSegs G;
  if constexpr (std::is_same<Rows, DualRows>::value) {
    if (C.st->compact_rows)
      stage_score_body<CompactRows>(C, lb, sm, G);
    else
      stage_score_body<FullRows>(C, lb, sm, G);
  } else {
    stage_score_body<Rows>(C, lb, sm, G);
  }
}

// ---------------------------------------------------------------------------
// General columns: Algorithm 1 with a bitonic sort.
// ---------------------------------------------------------------------------

// Sort key: position (canonical +0.0), then marker (-1 < +1 < pad).
__device__ __forceinline__ bool key_greater(double pa, int ma, double pb, int mb) {
  return pa > pb || (pa == pb && ma > mb);
}

constexpr int kPadMarker = 3;

// Emits the entries of column j into (pos, marker, delta) arrays through an
// atomic slot counter; beta/alpha are accumulated per thread.
template <typename Rows, typename Emit>
__device__ __forceinline__ void general_phase1(const DevProblem& P, const Rows& rs, const WalkState* st,
                                               int j, double xb, int tid, int nthreads, double& beta,
                                               double& alpha, Emit emit) {
  const double eps = P.eps;
  const bool isint = P.is_int[j] != 0;
  const int beg = P.col_ptr[j], end = P.col_ptr[j + 1];
  for (int e = beg + tid; e < end; e += nthreads) {
    const RowState q = rs[P.col_row[e]];
    const double a = P.col_val[e];
    BkEntry b0 = phase1(xb, q.r, a, (double)q.w0, eps, isint, beta, alpha);
    if (b0.has) emit(b0.t + 0.0, b0.marker, b0.delta);
    if (q.w1 >= 0.0f) {
      BkEntry b1 = phase1(xb, -q.r, -a, (double)q.w1, eps, isint, beta, alpha);
      if (b1.has) emit(b1.t + 0.0, b1.marker, b1.delta);
    }
  }
  if (tid == 0) {
    const double l = P.lb[j], u = P.ub[j];
    if (isfinite(l)) emit(l + 0.0, -1, 0.0);
    if (isfinite(u)) emit(u + 0.0, -1, 0.0);
    if (st->cut_active) {
      const double c = P.obj[j];
      if (c != 0.0) {
        BkEntry b2 = phase1(xb, st->rc, c, (double)st->wc, eps, isint, beta, alpha);
        if (b2.has) emit(b2.t + 0.0, b2.marker, b2.delta);
      }
    }
  }
}

__device__ __forceinline__ double block_sum256(double v, double* red) {
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) red[wv] = v;
  __syncthreads();
  double t = 0.0;
  for (int q = 0; q < (int)(blockDim.x >> 6); ++q) t += red[q];
  return t;
}

// In-place ascending bitonic sort of cap (power of two) keyed entries.
template <typename PosT, typename MarkT, typename DelT>
__device__ __forceinline__ void bitonic_sort(PosT pos, MarkT mk, DelT dl, int cap) {
  for (int size = 2; size <= cap; size <<= 1) {
    for (int stride = size >> 1; stride > 0; stride >>= 1) {
      for (int p = threadIdx.x; p < (cap >> 1); p += blockDim.x) {
        const int i = 2 * p - (p & (stride - 1));
        const int k = i + stride;
        const bool up = (i & size) == 0;
        const double pi = pos[i], pk = pos[k];
        const int mi = mk[i], mk2 = mk[k];
        if (key_greater(pi, mi, pk, mk2) == up) {
          const double di = dl[i];
          pos[i] = pk;
          pos[k] = pi;
          mk[i] = mk2;
          mk[k] = mi;
          dl[i] = dl[k];
          dl[k] = di;
        }
      }
      __syncthreads();
    }
  }
}

// Scan (phase 3) and argmax (phase 4) over sorted entries; one workgroup.
// Elements [0, cap) are split into contiguous per-thread runs.
template <typename PosT, typename MarkT, typename DelT>
__device__ __forceinline__ void scan_argmax(PosT pos, MarkT mk, DelT dl, int cap, double beta, double alpha,
                                            double xb, double l, double u, double* red, int* redk, bool& found,
                                            double& best, double& bestp) {
  const int tid = threadIdx.x, nt = blockDim.x;
  const int per = (cap + nt - 1) / nt;
  const int lo = min(cap, tid * per), hi = min(cap, lo + per);
  double run = 0.0;
  for (int i = lo; i < hi; ++i) run += dl[i];
  // exclusive scan of run totals across the workgroup
  const int lane = tid & 63, wv = tid >> 6;
  double inc = run;
#pragma unroll
  for (int o = 1; o < kWave; o <<= 1) {
    const double y = __shfl_up(inc, o, kWave);
    if (lane >= o) inc += y;
  }
  __syncthreads();
  if (lane == 63) red[wv] = inc;
  __syncthreads();
  double off = inc - run;
  for (int q = 0; q < wv; ++q) off += red[q];
  // per-entry score, best per thread (value desc, index asc)
  double bv = -DBL_MAX;
  int bk = INT_MAX;
  double prefix = off;
  for (int i = lo; i < hi; ++i) {
    const double d = dl[i];
    const double incl = prefix + d;
    const double p = pos[i];
    const int m = mk[i];
    if (m != kPadMarker && isfinite(p) && p >= l && p <= u && p != xb) {
      const double sigma = beta + ((m < 0) ? incl : prefix) + ((p > xb) ? alpha : 0.0);
      if (sigma > bv) {
        bv = sigma;
        bk = i;
      }
    }
    prefix = incl;
  }
  wave_argmax(bv, bk);
  __syncthreads();
  if (lane == 0) {
    red[wv] = bv;
    redk[wv] = bk;
  }
  __syncthreads();
  bv = red[0];
  bk = redk[0];
  for (int q = 1; q < (nt >> 6); ++q) {
    if (red[q] > bv || (red[q] == bv && redk[q] < bk)) {
      bv = red[q];
      bk = redk[q];
    }
  }
  found = bk != INT_MAX;
  best = bv;
  bestp = found ? pos[bk] : xb;
}

// General columns with at most 64 breakpoint slots: one wavefront per column
// (four per workgroup), one slot per lane. Phase 1 emits the entries into
// the wavefront's LDS slots by a ballot prefix count, the bitonic sort runs
// across lanes with exchanges between partner lanes (no barriers), then a
// wavefront scan and argmax.
struct WaveSortSmem {
  double pos[4][kWave];
  double del[4][kWave];
  int32_t mk[4][kWave];
};

// Inclusive prefix sum across the wavefront.
__device__ __forceinline__ double wave_inclusive(double v, int lane) {
#pragma unroll
  for (int o = 1; o < kWave; o <<= 1) {
    const double y = __shfl_up(v, o, kWave);
    if (lane >= o) v += y;
  }
  return v;
}

// Algorithm 1 for general column j with at most 64 breakpoints (bounds and
// cutoff included), by one wavefront: entries and breakpoints in registers,
// a bitonic sort across the lanes, wavefront scan and argmax. Every lane of
// the wavefront calls it with the same j; wv is the wavefront's slot in S.
template <typename Rows>
__device__ __forceinline__ void sort_wave_column(const WalkCtx& C, const Rows& rs, int j, WaveSortSmem& S, int wv) {
  const DevProblem& P = C.P;
  const WalkState* st = C.st;
  const int lane = threadIdx.x & (kWave - 1);
  const double eps = P.eps;
  const double xb = gmem((const double*)C.x)[j];
  const bool isint = P.is_int[j] != 0;
  const int beg = P.col_ptr[j], end = P.col_ptr[j + 1];
  double beta = 0.0, alpha = 0.0;
  // up to two entries per lane (a row and its twin), lane 0 adds the bounds
  // and the cutoff row; the class guarantees at most 64 in all
  BkEntry en[2];
  int ne = 0;
  const int e = beg + lane;
  if (e < end) {
    const RowState q = rs[P.col_row[e]];
    const double a = P.col_val[e];
    en[0] = phase1(xb, q.r, a, (double)q.w0, eps, isint, beta, alpha);
    if (en[0].has) ne = 1;
    if (q.w1 >= 0.0f) {
      const BkEntry b1 = phase1(xb, -q.r, -a, (double)q.w1, eps, isint, beta, alpha);
      if (b1.has) en[ne++] = b1;
    }
  }
  BkEntry ex[3];
  int nx = 0;
  if (lane == 0) {
    const double l = P.lb[j], u = P.ub[j];
    if (isfinite(l)) ex[nx++] = BkEntry{l, 0.0, -1, true};
    if (isfinite(u)) ex[nx++] = BkEntry{u, 0.0, -1, true};
    if (st->cut_active) {
      const double c = P.obj[j];
      if (c != 0.0) {
        const BkEntry b2 = phase1(xb, st->rc, c, (double)st->wc, eps, isint, beta, alpha);
        if (b2.has) ex[nx++] = b2;
      }
    }
  }
  // slot of each lane's first entry: exclusive prefix count of entries
  const int cnt_lane = ne + nx;
  int incl = cnt_lane;
#pragma unroll
  for (int o = 1; o < kWave; o <<= 1) {
    const int y = __shfl_up(incl, o, kWave);
    if (lane >= o) incl += y;
  }
  const int total = __shfl(incl, kWave - 1, kWave);
  int slot = incl - cnt_lane;
  for (int k = 0; k < ne; ++k, ++slot) {
    S.pos[wv][slot] = en[k].t + 0.0;
    S.mk[wv][slot] = en[k].marker;
    S.del[wv][slot] = en[k].delta;
  }
  for (int k = 0; k < nx; ++k, ++slot) {
    S.pos[wv][slot] = ex[k].t + 0.0;
    S.mk[wv][slot] = ex[k].marker;
    S.del[wv][slot] = ex[k].delta;
  }
  // the slots written by other lanes of this wavefront become visible
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  double p = HUGE_VAL, d = 0.0;
  int m = kPadMarker;
  if (lane < total) {
    p = S.pos[wv][lane];
    m = S.mk[wv][lane];
    d = S.del[wv][lane];
  }
  // bitonic sort of (position, marker) across the lanes; both lanes of a
  // pair take the same decision from the lower lane's point of view
#pragma unroll
  for (int size = 2; size <= kWave; size <<= 1) {
#pragma unroll
    for (int stride = size >> 1; stride > 0; stride >>= 1) {
      const double po = __shfl_xor(p, stride, kWave);
      const int mo = __shfl_xor(m, stride, kWave);
      const double dlo = __shfl_xor(d, stride, kWave);
      const bool lower = (lane & stride) == 0;
      const bool up = (lane & size) == 0;
      const double pl = lower ? p : po, ph = lower ? po : p;
      const int ml = lower ? m : mo, mh = lower ? mo : m;
      const bool swap = up ? key_greater(pl, ml, ph, mh) : key_greater(ph, mh, pl, ml);
      if (swap) {
        p = po;
        m = mo;
        d = dlo;
      }
    }
  }
  beta = wave_sum(beta);
  alpha = wave_sum(alpha);
  const double inc = wave_inclusive(d, lane);
  const double prefix = inc - d;
  double bv = -DBL_MAX;
  int bk = INT_MAX;
  const double l = P.lb[j], u = P.ub[j];
  if (m != kPadMarker && isfinite(p) && p >= l && p <= u && p != xb) {
    bv = beta + ((m < 0) ? inc : prefix) + ((p > xb) ? alpha : 0.0);
    bk = lane;
  }
  wave_argmax(bv, bk);
  const bool found = bk != INT_MAX;
  const double bestp = __shfl(p, found ? bk : 0, kWave);
  if (lane == 0) write_result(C.xhat, C.s, j, found, bv, found ? bestp : xb, xb);
}

template <typename Rows>
__global__ __launch_bounds__(256) void k_sort_wave(const WalkCtx* __restrict__ walks, const int32_t* __restrict__ off,
                                                   int32_t nw) {
  int lb;
  const int w_ = block_walk(off, nw, lb);
  if (w_ < 0) return;
  const WalkCtx& C = walks[w_];
  const WalkState* st = C.st;
  if (st->k >= st->iters || st->pass_skip) return;
  __shared__ WaveSortSmem S;
  const int wv = threadIdx.x >> 6;
  const int j = C.plan.sort_begin[0] + lb * 4 + wv;
  if (j >= C.plan.sort_begin[1]) return;  // whole wavefronts leave together
  const Rows rs = rows_of<Rows>(C);
  sort_wave_column<Rows>(C, rs, j, S, wv);
}

// The listed general columns of the wave-sort class (at most 64
// breakpoints) in an affected-rescoring iteration: one wavefront each
// (grid-stride over the subset list).
template <typename Rows>
__device__ __forceinline__ void aff_wave_body(const WalkCtx& C, const LearnCtx& L, int b, int nb, WaveSortSmem& S) {
  if (C.st->k >= C.st->iters || L.ls->idle) return;
  const int wv = threadIdx.x >> 6;
  const Rows rs = rows_of<Rows>(C);
  const int count = L.ls->tk[0].count;
  const int q0 = C.plan.sort_begin[0], q1 = C.plan.sort_begin[1];
  for (int i = b * 4 + wv; i < count; i += nb * 4) {
    const int q = L.sel[0][i];
    if (q < q0 || q >= q1) continue;  // uniform across the wavefront
    sort_wave_column<Rows>(C, rs, q, S, wv);
  }
}

template <int CAP, typename Rows>
__global__ __launch_bounds__(256) void k_sort_block(const WalkCtx* __restrict__ walks, const int32_t* __restrict__ off,
                                                    int32_t nw) {
  int lb;
  const int w_ = block_walk(off, nw, lb);
  if (w_ < 0) return;
  const WalkCtx& C = walks[w_];
  const DevProblem& P = C.P;
  const double* x = C.x;
  const Rows rs = rows_of<Rows>(C);
  const WalkState* st = C.st;
  double* xhat = C.xhat;
  double* sc = C.s;
  int c = 0;
  while (c < kSortCaps - 1 && kSortCap[c] != CAP) ++c;
  const int32_t q0 = C.plan.sort_begin[c];
  if (st->k >= st->iters || st->pass_skip) return;
  __shared__ double spos[CAP];
  __shared__ double sdel[CAP];
  __shared__ int smk[CAP];
  __shared__ int scount;
  __shared__ double red[8];
  __shared__ int redk[8];
  const int j = q0 + lb;
  const double xb = x[j];
  if (threadIdx.x == 0) scount = 0;
  __syncthreads();
  double beta = 0.0, alpha = 0.0;
  general_phase1(P, rs, st, j, xb, threadIdx.x, blockDim.x, beta, alpha, [&](double p, int m, double d) {
    const int s = atomicAdd(&scount, 1);
    spos[s] = p;
    smk[s] = m;
    sdel[s] = d;
  });
  beta = block_sum256(beta, red);
  alpha = block_sum256(alpha, red);
  __syncthreads();
  const int cnt = scount;
  for (int i = cnt + threadIdx.x; i < CAP; i += blockDim.x) {
    spos[i] = HUGE_VAL;
    smk[i] = kPadMarker;
    sdel[i] = 0.0;
  }
  __syncthreads();
  int cap = 64;
  while (cap < cnt) cap <<= 1;
  bitonic_sort(spos, smk, sdel, cap);
  bool found;
  double best, bestp;
  scan_argmax(spos, smk, sdel, cap, beta, alpha, xb, P.lb[j], P.ub[j], red, redk, found, best, bestp);
  if (threadIdx.x == 0) write_result(xhat, sc, j, found, best, bestp, xb);
}

template <typename Rows>
__global__ __launch_bounds__(1024) void k_sort_long(const WalkCtx* __restrict__ walks,
                                                    const int32_t* __restrict__ off, int32_t nw) {
  int lb;
  const int w_ = block_walk(off, nw, lb);
  if (w_ < 0) return;
  const WalkCtx& C = walks[w_];
  const DevProblem& P = C.P;
  const double* x = C.x;
  const Rows rs = rows_of<Rows>(C);
  const WalkState* st = C.st;
  double* xhat = C.xhat;
  double* sc = C.s;
  double* gpos = C.long_pos;
  int32_t* gmk = C.long_marker;
  double* gdel = C.long_delta;
  if (st->k >= st->iters || st->pass_skip) return;
  __shared__ int scount;
  __shared__ double red[16];
  __shared__ int redk[16];
  const LongTask T = C.plan.long_tasks[lb];
  const int j = T.col;
  double* pos = gpos + T.offset;
  int32_t* mk = gmk + T.offset;
  double* dl = gdel + T.offset;
  const double xb = x[j];
  if (threadIdx.x == 0) scount = 0;
  __syncthreads();
  double beta = 0.0, alpha = 0.0;
  general_phase1(P, rs, st, j, xb, threadIdx.x, blockDim.x, beta, alpha, [&](double p, int m, double d) {
    const int s = atomicAdd(&scount, 1);
    pos[s] = p;
    mk[s] = m;
    dl[s] = d;
  });
  {
    double b = wave_sum(beta), a = wave_sum(alpha);
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) {
      red[wv] = b;
      redk[wv] = 0;
    }
    __syncthreads();
    b = 0.0;
    for (int q = 0; q < 16; ++q) b += red[q];
    __syncthreads();
    if (lane == 0) red[wv] = a;
    __syncthreads();
    a = 0.0;
    for (int q = 0; q < 16; ++q) a += red[q];
    beta = b;
    alpha = a;
  }
  __syncthreads();
  const int cnt = scount;
  for (int i = cnt + threadIdx.x; i < T.cap; i += blockDim.x) {
    pos[i] = HUGE_VAL;
    mk[i] = kPadMarker;
    dl[i] = 0.0;
  }
  __threadfence_block();
  __syncthreads();
  bitonic_sort(pos, mk, dl, T.cap);
  bool found;
  double best, bestp;
  scan_argmax(pos, mk, dl, T.cap, beta, alpha, xb, P.lb[j], P.ub[j], red, redk, found, best, bestp);
  if (threadIdx.x == 0) write_result(xhat, sc, j, found, best, bestp, xb);
}

// ---------------------------------------------------------------------------
// Subset pass: exact best shift of the columns of a proposal set, with the
// same per-entry arithmetic as the full pass. Binary and narrow columns of
// any length are cut into chunks of kSubsetChunk stored entries
// (k_subset_chunks, partial flip sum or bins per chunk) and combined in chunk
// order (k_subset_combine); general columns use one workgroup's LDS sort
// (k_subset_general).
// ---------------------------------------------------------------------------

struct SubsetChunkSmem {
  double bins[kNarrowBins];
  double red[4];
  unsigned long long scand;
};

template <typename Rows>
__device__ __forceinline__ void subset_chunks_body(const WalkCtx& C, const LearnCtx& L, int b, int nb,
                                                   SubsetChunkSmem& SM) {
  const Rows rs = rows_of<Rows>(C);
  const DevProblem& P = C.P;
  const WalkState* st = C.st;
  if (st->k >= st->iters || L.ls->idle) return;
  double* bins = SM.bins;
  double* red = SM.red;
  unsigned long long& scand = SM.scand;
  const int cnt = L.ls->tk[0].count;
  const int chunks = L.ls->tk[0].chunks;
  const int tid = threadIdx.x;
  const double eps = P.eps;
  for (int c = b; c < chunks; c += nb) {
    // selected column of chunk c: the largest i with sub_off[i] <= c
    int lo = 0, hi = cnt - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (L.sub_off[mid] <= c)
        lo = mid;
      else
        hi = mid - 1;
    }
    const int q = L.sel[0][lo];
    const int first = (c == L.sub_off[lo]);
    const int e_beg = P.col_ptr[q] + (c - L.sub_off[lo]) * kSubsetChunk;
    const int e_end = min(P.col_ptr[q + 1], e_beg + kSubsetChunk);
    const double xb = C.x[q];
    ChunkPartial* out = L.sub_parts + c;
    if (L.cls[q] == SUB_FLIP) {
      const double d = (1.0 - xb) - xb;
      double v = 0.0;
      for (int e = e_beg + tid; e < e_end; e += blockDim.x) {
        const RowState r = rs[P.col_row[e]];
        const double r2 = r.r + P.col_val[e] * d;
        v += penalty(r.r, r2, (double)r.w0, eps);
        if (r.w1 >= 0.0f) v += penalty(-r.r, -r2, (double)r.w1, eps);
      }
      if (tid == 0 && first && st->cut_active && P.obj[q] != 0.0)
        v += penalty(st->rc, st->rc + P.obj[q] * d, (double)st->wc, eps);
      v = block_sum256(v, red);
      if (tid == 0) out->beta = v;
      __syncthreads();
      continue;
    }
    const double l = P.lb[q], u = P.ub[q];
    const int W = (int)(u - l) + 1;
    if (tid < kNarrowBins) bins[tid] = 0.0;
    if (tid == 0) scand = 0ull;
    __syncthreads();
    double beta = 0.0, alpha = 0.0;
    unsigned long long cand = 0ull;
    for (int e = e_beg + tid; e < e_end; e += blockDim.x) {
      const RowState r = rs[P.col_row[e]];
      const double a = P.col_val[e];
      narrow_entry(xb, r.r, a, (double)r.w0, eps, l, u, W, bins, beta, alpha, cand);
      if (r.w1 >= 0.0f) narrow_entry(xb, -r.r, -a, (double)r.w1, eps, l, u, W, bins, beta, alpha, cand);
    }
    if (tid == 0 && first && st->cut_active && P.obj[q] != 0.0)
      narrow_entry(xb, st->rc, P.obj[q], (double)st->wc, eps, l, u, W, bins, beta, alpha, cand);
    cand = wave_or(cand);
    if ((tid & 63) == 0 && cand) atomicOr(&scand, cand);
    beta = block_sum256(beta, red);
    alpha = block_sum256(alpha, red);
    __syncthreads();
    if (tid < kNarrowBins) out->bins[tid] = bins[tid];
    if (tid == 0) {
      out->beta = beta;
      out->alpha = alpha;
      out->cand = scand;
    }
    __syncthreads();
  }
}

template <typename Rows>
__global__ __launch_bounds__(256) void k_subset_chunks(const WalkCtx* __restrict__ walks,
                                                       const LearnCtx* __restrict__ lc) {
  __shared__ SubsetChunkSmem SM;
  subset_chunks_body<Rows>(walks[0], *lc, (int)blockIdx.x, (int)gridDim.x, SM);
}


// One wavefront per selected binary or narrow column (grid-stride): its
// chunks in order, then the flip score or the bins' scan and argmax.
__global__ __launch_bounds__(256) void k_subset_combine(const WalkCtx* __restrict__ walks,
                                                        const LearnCtx* __restrict__ lc) {
  const WalkCtx& C = walks[0];
  const LearnCtx& L = *lc;
  const DevProblem& P = C.P;
  const WalkState* st = C.st;
  if (st->k >= st->iters || L.ls->idle) return;
  const int count = L.ls->tk[0].count;
  const int lane = threadIdx.x & 63;
  for (int i = blockIdx.x * 4 + (threadIdx.x >> 6); i < count; i += gridDim.x * 4) {
    const int q = L.sel[0][i];
    const uint8_t cl = L.cls[q];
    if (cl == SUB_GENERAL) continue;
    if (L.short_lane && q >= C.plan.short_seg[0] && q < C.plan.short_seg[kShortMax + 2]) continue;
    const int c0 = L.sub_off[i], c1 = L.sub_off[i + 1];
    const double xb = C.x[q];
    if (cl == SUB_FLIP) {
      double v = 0.0;
      for (int c = c0; c < c1; ++c) v += L.sub_parts[c].beta;
      if (lane == 0) write_result(C.xhat, C.s, q, true, v, 1.0 - xb, xb);
      continue;
    }
    double bv = 0.0, b = 0.0, a = 0.0;
    unsigned long long cand = 0ull;
    for (int c = c0; c < c1; ++c) {
      const ChunkPartial* pp = L.sub_parts + c;
      bv += pp->bins[lane];
      b += pp->beta;
      a += pp->alpha;
      cand |= pp->cand;
    }
    const double l = P.lb[q];
    const int W = (int)(P.ub[q] - l) + 1;
    bool found;
    double best, bestp;
    narrow_finish(bv, b, a, cand, xb, l, W, lane, found, best, bestp);
    if (lane == 0) write_result(C.xhat, C.s, q, found, best, bestp, xb);
  }
}

// One workgroup per selected general column (grid-stride; Algorithm 1 with
// the LDS sort).
struct SubsetGeneralSmem {
  double spos[kSubsetCap];
  double sdel[kSubsetCap];
  int smk[kSubsetCap];
  int scount;
  double red[8];
  int redk[8];
};

__device__ __forceinline__ void subset_general_body(const WalkCtx& C, const LearnCtx& L, int b, int nb,
                                                    SubsetGeneralSmem& SM) {
  const DevProblem& P = C.P;
  const WalkState* st = C.st;
  if (st->k >= st->iters || L.ls->idle) return;
  double* spos = SM.spos;
  double* sdel = SM.sdel;
  int* smk = SM.smk;
  int& scount = SM.scount;
  double* red = SM.red;
  int* redk = SM.redk;
  const int tid = threadIdx.x;
  const int count = L.ls->tk[0].count;
  for (int i = b; i < count; i += nb) {
    const int q = L.sel[0][i];
    if (L.cls[q] != SUB_GENERAL) continue;
    // affected rescoring: short columns go to lanes, the wave-sort class to wavefronts (k_aff_score)
    if (L.short_lane && ((q >= C.plan.short_seg[0] && q < C.plan.short_seg[kShortMax + 2]) ||
                         (q >= C.plan.sort_begin[0] && q < C.plan.sort_begin[1])))
      continue;
    const double xb = C.x[q];
    if (tid == 0) scount = 0;
    __syncthreads();
    double beta = 0.0, alpha = 0.0;
    general_phase1(P, FullRows{gmem((const RowState*)C.rs)}, st, q, xb, tid, blockDim.x, beta, alpha,
                   [&](double p, int m, double d) {
                     const int k = atomicAdd(&scount, 1);
                     spos[k] = p;
                     smk[k] = m;
                     sdel[k] = d;
                   });
    beta = block_sum256(beta, red);
    alpha = block_sum256(alpha, red);
    __syncthreads();
    const int cnt = scount;
    int cap = 64;
    while (cap < cnt) cap <<= 1;
    for (int t = cnt + tid; t < cap; t += blockDim.x) {
      spos[t] = HUGE_VAL;
      smk[t] = kPadMarker;
      sdel[t] = 0.0;
    }
    __syncthreads();
    bitonic_sort(spos, smk, sdel, cap);
    bool found;
    double best, bestp;
    scan_argmax(spos, smk, sdel, cap, beta, alpha, xb, P.lb[q], P.ub[q], red, redk, found, best, bestp);
    if (tid == 0) write_result(C.xhat, C.s, q, found, best, bestp, xb);
    // every reader of this column's LDS arrays is done before the next one
    __syncthreads();
  }
}

__global__ __launch_bounds__(256) void k_subset_general(const WalkCtx* __restrict__ walks,
                                                        const LearnCtx* __restrict__ lc) {
  __shared__ SubsetGeneralSmem SM;
  subset_general_body(walks[0], *lc, (int)blockIdx.x, (int)gridDim.x, SM);
}

// The scoring of an affected-rescoring iteration in one launch: workgroups
// [0, g[0]) score the short columns by lanes, the next g[1] the wave-sort
// class, the next g[2] the subset chunks and the last g[3] the other general
// columns (each role strides over its own work).
template <typename Rows>
__global__ __launch_bounds__(256) void k_aff_score(const WalkCtx* __restrict__ walks,
                                                   const LearnCtx* __restrict__ lc, const AffRun* __restrict__ run,
                                                   int g0, int g1, int g2, int g3) {
  __shared__ union {
    WaveSortSmem w;
    SubsetChunkSmem c;
    SubsetGeneralSmem g;
  } U;
  const WalkCtx& C = walks[0];
  const int b = (int)blockIdx.x;
  if (b < g0) {
    aff_short_body<Rows>(C, run, b, g0);
  } else if (b < g0 + g1) {
    aff_wave_body<Rows>(C, *lc, b - g0, g1, U.w);
  } else if (b < g0 + g1 + g2) {
    subset_chunks_body<Rows>(C, *lc, b - g0 - g1, g2, U.c);
  } else if (b < g0 + g1 + g2 + g3) {
    subset_general_body(C, *lc, b - g0 - g1 - g2, g3, U.g);
  }
}

}  // namespace

hipError_t launch_subset_grids(const WalkCtx* C, const LearnCtx* L, int chunk_grid, int combine_grid, int general_grid,
                               int has_general, int compact, hipStream_t s) {
  const dim3 grid((unsigned)std::max(chunk_grid, 1));
  if (compact)
    hipLaunchKernelGGL(k_subset_chunks<CompactRows>, grid, dim3(256), 0, s, C, L);
  else
    hipLaunchKernelGGL(k_subset_chunks<FullRows>, grid, dim3(256), 0, s, C, L);
  hipLaunchKernelGGL(k_subset_combine, dim3((unsigned)std::max(combine_grid, 1)), dim3(256), 0, s, C, L);
  if (has_general) hipLaunchKernelGGL(k_subset_general, dim3((unsigned)std::max(general_grid, 1)), dim3(256), 0, s, C, L);
  return hipGetLastError();
}

hipError_t launch_aff_score(const WalkCtx* C, const LearnCtx* L, const AffRun* run, const int g[4], int combine_grid,
                            int compact, hipStream_t s) {
  const unsigned total = (unsigned)(g[0] + g[1] + g[2] + g[3]);
  if (compact)
    hipLaunchKernelGGL(k_aff_score<CompactRows>, dim3(total), dim3(256), 0, s, C, L, run, g[0], g[1], g[2], g[3]);
  else
    hipLaunchKernelGGL(k_aff_score<FullRows>, dim3(total), dim3(256), 0, s, C, L, run, g[0], g[1], g[2], g[3]);
  hipLaunchKernelGGL(k_subset_combine, dim3((unsigned)std::max(combine_grid, 1)), dim3(256), 0, s, C, L);
  return hipGetLastError();
}

hipError_t launch_subset_pass(const WalkCtx* C, const LearnCtx* L, const LearnCtx& Lh, int has_general, int compact,
                              hipStream_t s) {
  const int K = Lh.K[0];
  return launch_subset_grids(C, L, std::min(kSubsetGrid, std::max(Lh.sub_cap, 1)), (K + 3) / 4, K, has_general,
                             compact, s);
}

int32_t kernel_blocks(const WalkCtx& c, int slot) {
  const PassPlan& p = c.plan;
  switch (slot) {
    case KS_SHORT: return (p.short_seg[kShortMax + 2] - p.short_seg[0] + 255) / 256;
    case KS_FLIP: return (p.flip_end - p.flip_begin + 3) / 4;
    case KS_PACK: return p.n_packs;
    case KS_CHUNK: return p.stage ? 0 : p.n_chunks;  // a staged pass scores its chunks in k_stage_score
    case KS_COMBINE: return (p.n_chunk_cols + 3) / 4;
    case KS_LONG: return p.n_long;
    case KS_STAGE: return p.n_stage_rtasks;
    case KS_STAGE_SCORE: return p.n_stage_units * kXcds;
    case KS_ARGMAX: return c.argmax_blocks + c.argmax_comb;
    case KS_SELECT: return 1;
    case KS_APPLY: return c.apply_blocks;
    case KS_FINISH: return 1;
    default:
      if (slot == KS_SORT0) return (p.sort_begin[1] - p.sort_begin[0] + 3) / 4;  // a wavefront per column
      if (slot > KS_SORT0 && slot < KS_SORT0 + kSortCaps)
        return p.sort_begin[slot - KS_SORT0 + 1] - p.sort_begin[slot - KS_SORT0];
      return 0;
  }
}

hipError_t PassStreams::create() {
  for (int k = 0; k < 2; ++k) {
    hipError_t e = hipStreamCreateWithFlags(&side[k], hipStreamNonBlocking);
    if (e != hipSuccess) return e;
    e = hipEventCreateWithFlags(&join[k], hipEventDisableTiming);
    if (e != hipSuccess) return e;
  }
  return hipEventCreateWithFlags(&fork, hipEventDisableTiming);
}

void PassStreams::destroy() {
  for (int k = 0; k < 2; ++k) {
    if (side[k]) (void)hipStreamDestroy(side[k]);
    if (join[k]) (void)hipEventDestroy(join[k]);
    side[k] = nullptr;
    join[k] = nullptr;
  }
  if (fork) (void)hipEventDestroy(fork);
  fork = nullptr;
}

template <typename Rows>
#define CHAP_LAUNCH(...)      \
  do {                        \
    hipLaunchKernelGGL(__VA_ARGS__); \
    check();                  \
  } while (0)

hipError_t launch_pass_rows(const BatchLaunch& L, hipStream_t stream, const PassStreams* ps, bool defer_combine) {
  const int nw = L.nw;
  auto grid = [&](int slot) { return dim3((unsigned)L.grid[slot]); };
  // a launch error (say, an LDS size the device refuses) is kept by the first
  // check after it; later successful calls would otherwise clear it
  hipError_t first = hipSuccess;
  auto check = [&]() {
    const hipError_t le = hipGetLastError();
    if (first == hipSuccess) first = le;
  };
  // the staged scoring is one launch on the main stream; the side streams
  // carry the short, flip, chunk and long-sort kernels of unstaged columns
  const bool fork = ps && (L.total[KS_SHORT] > 0 || L.total[KS_FLIP] > 0 || L.total[KS_LONG] > 0 ||
                           L.total[KS_CHUNK] > 0);
  hipStream_t s_short = stream, s_long = stream;
  hipError_t e = hipSuccess;
  if (fork) {
    e = hipEventRecord(ps->fork, stream);
    for (int k = 0; k < 2 && e == hipSuccess; ++k) e = hipStreamWaitEvent(ps->side[k], ps->fork, 0);
    if (e != hipSuccess) return e;
    s_short = ps->side[0];
    s_long = ps->side[1];
  }
  if (L.total[KS_SHORT] > 0)
    CHAP_LAUNCH(k_short<Rows>, grid(KS_SHORT), dim3(256), 0, s_short, L.walks, L.off[KS_SHORT], nw);
  if (L.total[KS_FLIP] > 0)
    CHAP_LAUNCH(k_flip_wave<Rows>, grid(KS_FLIP), dim3(256), 0, s_short, L.walks, L.off[KS_FLIP], nw);
  // staged columns: the records (alone: they are bound by HBM), then the
  // scoring of every staged task and long-column chunk
  if (L.total[KS_STAGE] > 0)
    CHAP_LAUNCH(k_stage_rows<Rows>, grid(KS_STAGE), dim3(512), 0, stream, L.walks, L.off[KS_STAGE], nw);
  // long narrow columns: the chunks of staged walks are roles of
  // k_stage_score, those of unstaged walks k_narrow_chunk workgroups; a batch
  // may hold both, and k_narrow_combine then waits for both (after the join)
  bool combine_after_join = false;
  const bool combine = L.total[KS_COMBINE] > 0 && !(defer_combine && pass_defers_combine(L));
  if (L.total[KS_STAGE_SCORE] > 0)
    CHAP_LAUNCH(k_stage_score<Rows>, grid(KS_STAGE_SCORE), dim3(256), 0, stream, L.walks, L.off[KS_STAGE_SCORE],
                nw);
  if (L.total[KS_CHUNK] > 0)
    CHAP_LAUNCH(k_narrow_chunk<Rows>, grid(KS_CHUNK), dim3(256), 0, s_long, L.walks, L.off[KS_CHUNK], nw);
  if (combine) {
    if (L.total[KS_CHUNK] == 0)
      CHAP_LAUNCH(k_narrow_combine, grid(KS_COMBINE), dim3(256), 0, stream, L.walks, L.off[KS_COMBINE], nw);
    else if (L.total[KS_STAGE_SCORE] == 0)
      CHAP_LAUNCH(k_narrow_combine, grid(KS_COMBINE), dim3(256), 0, s_long, L.walks, L.off[KS_COMBINE], nw);
    else
      combine_after_join = true;
  }
  if (L.total[KS_LONG] > 0)
    CHAP_LAUNCH(k_sort_long<Rows>, grid(KS_LONG), dim3(1024), 0, s_long, L.walks, L.off[KS_LONG], nw);
  if (L.total[KS_PACK] > 0)
    CHAP_LAUNCH(k_narrow_pack<Rows>, grid(KS_PACK), dim3(256), 0, stream, L.walks, L.off[KS_PACK], nw);
  if (L.total[KS_SORT0] > 0)
    CHAP_LAUNCH(k_sort_wave<Rows>, grid(KS_SORT0), dim3(256), 0, stream, L.walks, L.off[KS_SORT0], nw);
  if (L.total[KS_SORT0 + 1] > 0)
    CHAP_LAUNCH((k_sort_block<256, Rows>), grid(KS_SORT0 + 1), dim3(256), 0, stream, L.walks,
                       L.off[KS_SORT0 + 1], nw);
  if (L.total[KS_SORT0 + 2] > 0)
    CHAP_LAUNCH((k_sort_block<1024, Rows>), grid(KS_SORT0 + 2), dim3(256), 0, stream, L.walks,
                       L.off[KS_SORT0 + 2], nw);
  if (L.total[KS_SORT0 + 3] > 0)
    CHAP_LAUNCH((k_sort_block<4096, Rows>), grid(KS_SORT0 + 3), dim3(256), 0, stream, L.walks,
                       L.off[KS_SORT0 + 3], nw);
  check();
  e = first;
  if (fork) {
    for (int k = 0; k < 2 && e == hipSuccess; ++k) {
      e = hipEventRecord(ps->join[k], ps->side[k]);
      if (e == hipSuccess) e = hipStreamWaitEvent(stream, ps->join[k], 0);
    }
  }
  if (e == hipSuccess && combine_after_join) {
    hipLaunchKernelGGL(k_narrow_combine, grid(KS_COMBINE), dim3(256), 0, stream, L.walks, L.off[KS_COMBINE], nw);
    e = hipGetLastError();
  }
  return e;
}

#undef CHAP_LAUNCH

hipError_t launch_pass(const BatchLaunch& L, hipStream_t stream, const PassStreams* ps, bool defer_combine) {
  if (L.compact == 1) return launch_pass_rows<CompactRows>(L, stream, ps, defer_combine);
  if (L.compact == 2) return launch_pass_rows<DualRows>(L, stream, ps, false);
  return launch_pass_rows<FullRows>(L, stream, ps, false);
}

}  // namespace chap
