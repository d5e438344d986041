// C ABI of the gfx950 tabu-search library: problem creation (validation,
// normalisation to '<=' rows, column routing, upload), the single best-shift
// pass and the graph-captured tabu walk.

#include <algorithm>
#include <cmath>
#include <cstring>
#include <limits>
#include <memory>
#include <numeric>
#include <string>
#include <vector>

#include "chap_internal.h"

using namespace chap;

namespace chap {

thread_local std::string g_error;

int fail(int code, const std::string& msg) {
  g_error = msg;
  return code;
}

}  // namespace chap

namespace {

__global__ void k_fill_i32(int32_t* a, int32_t v, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) a[i] = v;
}

}  // namespace

namespace chap {

// Uploads per-walk contexts and the per-kernel block prefix tables. A batch
// (more than one walk) is placed by XCD: every walk goes to one XCD, chosen
// greedily by its pass work (largest walks first, to the least loaded XCD),
// ctx is reordered XCD by XCD (order[i] = caller's index of ctx[i]) and each
// table gets the first virtual block and block count of every XCD appended
// (see block_walk); a kernel then launches kXcds x its largest XCD share.
hipError_t build_launch(DeviceArena& A, std::vector<WalkCtx>& ctx, BatchLaunch* L, std::vector<int32_t>* order) {
  const size_t nw = ctx.size();
  L->nw = (int32_t)nw;
  std::vector<int32_t> xcd(nw, 0), perm(nw);
  std::iota(perm.begin(), perm.end(), 0);
  if (nw > 1) {
    std::vector<int64_t> work(nw, 0);
    for (size_t w = 0; w < nw; ++w)
      for (int k = KS_SHORT; k <= KS_STAGE_SCORE; ++k) work[w] += kernel_blocks(ctx[w], k);
    std::vector<int32_t> by(nw);
    std::iota(by.begin(), by.end(), 0);
    std::stable_sort(by.begin(), by.end(), [&](int32_t a, int32_t b) { return work[a] > work[b]; });
    int64_t load[kXcds] = {0};
    for (int32_t w : by) {
      int x = 0;
      for (int y = 1; y < kXcds; ++y)
        if (load[y] < load[x]) x = y;
      xcd[w] = x;
      load[x] += std::max<int64_t>(work[w], 1);
    }
    std::stable_sort(perm.begin(), perm.end(), [&](int32_t a, int32_t b) { return xcd[a] < xcd[b]; });
    std::vector<WalkCtx> sorted(nw);
    std::vector<int32_t> xs(nw);
    for (size_t i = 0; i < nw; ++i) {
      sorted[i] = ctx[perm[i]];
      xs[i] = xcd[perm[i]];
    }
    ctx.swap(sorted);
    xcd.swap(xs);
  }
  if (order) *order = perm;
  WalkCtx* d;
  hipError_t e = A.upload(&d, ctx);
  if (e != hipSuccess) return e;
  L->walks = d;
  for (int k = 0; k < KS_COUNT; ++k) {
    std::vector<int32_t> off(nw + 1, 0);
    for (size_t w = 0; w < nw; ++w) off[w + 1] = off[w] + kernel_blocks(ctx[w], k);
    L->total[k] = off.back();
    L->grid[k] = off.back();
    if (nw > 1) {
      int32_t first[kXcds], count[kXcds] = {0};
      for (int x = 0; x < kXcds; ++x) first[x] = off.back();
      for (size_t w = 0; w < nw; ++w) {
        first[xcd[w]] = std::min(first[xcd[w]], off[w]);
        count[xcd[w]] += off[w + 1] - off[w];
      }
      int32_t most = 0;
      for (int x = 0; x < kXcds; ++x) {
        off.push_back(first[x]);
        most = std::max(most, count[x]);
      }
      for (int x = 0; x < kXcds; ++x) off.push_back(count[x]);
      L->grid[k] = kXcds * most;
    }
    int32_t* doff;
    e = A.upload(&doff, off);
    if (e != hipSuccess) return e;
    L->off[k] = doff;
  }
  return hipSuccess;
}

int blocks_for_host(int64_t work, int cap) {
  int64_t b = (work + 255) / 256;
  return (int)std::max<int64_t>(1, std::min<int64_t>(b, cap));
}

}  // namespace chap

extern "C" {

void chap_options_default(chap_options* opt) {
  if (!opt) return;
  opt->feas_tol = 1e-6;
  opt->graph_iters = 64;
  opt->short_max = kShortMax;
  opt->chunk_min = 4096;
  opt->chunk_len = 4096;
  opt->row_stage = 1;
  opt->rescore_cap = 0;
}

const char* chap_last_error(void) { return g_error.c_str(); }

int32_t chap_problem_num_norm_rows(const chap_problem* p) { return p ? p->mp : -1; }

int chap_problem_norm_row_map(const chap_problem* p, int32_t* orig_row, int8_t* sign) {
  if (!p || (p->mp > 0 && (!orig_row || !sign))) return fail(CHAP_EINVAL, "chap_problem_norm_row_map: null argument");
  std::copy(p->norm_orig.begin(), p->norm_orig.end(), orig_row);
  std::copy(p->norm_sign.begin(), p->norm_sign.end(), sign);
  return CHAP_OK;
}

void chap_problem_destroy(chap_problem* p) { delete p; }

int chap_problem_create(chap_problem** out, int32_t n, int32_t m, const int64_t* csr_row_ptr, const int32_t* csr_col,
                        const double* csr_val, const int64_t* csc_col_ptr, const int32_t* csc_row,
                        const double* csc_val, const char* sense, const double* rhs, const double* lb,
                        const double* ub, const uint8_t* is_int, const double* obj, const chap_options* opt) {
  if (!out) return fail(CHAP_EINVAL, "chap_problem_create: out is null");
  if (n < 0 || m < 0) return fail(CHAP_EINVAL, "chap_problem_create: negative size");
  if (!csr_row_ptr || !csc_col_ptr) return fail(CHAP_EINVAL, "chap_problem_create: null row/column pointers");
  if (n > 0 && (!lb || !ub || !is_int || !obj)) return fail(CHAP_EINVAL, "chap_problem_create: null variable array");
  if (m > 0 && (!sense || !rhs)) return fail(CHAP_EINVAL, "chap_problem_create: null row array");
  chap_options o;
  chap_options_default(&o);
  if (opt) {
    if (!(opt->feas_tol >= 0.0) || !std::isfinite(opt->feas_tol))
      return fail(CHAP_EINVAL, "chap_problem_create: feas_tol must be finite and >= 0");
    o.feas_tol = opt->feas_tol;
    if (opt->graph_iters < 0 || opt->short_max < 0 || opt->short_max > kShortMax || opt->chunk_min < 0 ||
        opt->chunk_len < 0 || opt->row_stage < -1 || opt->row_stage > 1 || opt->rescore_cap < 0 ||
        opt->rescore_cap > kRescoreCapMax)
      return fail(CHAP_EINVAL, "chap_problem_create: option out of range");
    o.rescore_cap = opt->rescore_cap;
    if (opt->row_stage) o.row_stage = opt->row_stage;
    if (opt->graph_iters) o.graph_iters = opt->graph_iters;
    if (opt->short_max) o.short_max = opt->short_max;
    if (opt->chunk_min) o.chunk_min = opt->chunk_min;
    if (opt->chunk_len) o.chunk_len = opt->chunk_len;
  }
  // ---- structural checks -------------------------------------------------
  if (csr_row_ptr[0] != 0) return fail(CHAP_EINVAL, "csr_row_ptr[0] must be 0");
  for (int32_t i = 0; i < m; ++i)
    if (csr_row_ptr[i + 1] < csr_row_ptr[i]) return fail(CHAP_EINVAL, "csr_row_ptr decreases at row " + std::to_string(i));
  const int64_t nnz_in = csr_row_ptr[m];
  if (csc_col_ptr[0] != 0) return fail(CHAP_EINVAL, "csc_col_ptr[0] must be 0");
  for (int32_t j = 0; j < n; ++j)
    if (csc_col_ptr[j + 1] < csc_col_ptr[j]) return fail(CHAP_EINVAL, "csc_col_ptr decreases at column " + std::to_string(j));
  if (csc_col_ptr[n] != nnz_in) return fail(CHAP_EINVAL, "CSR and CSC hold different numbers of entries");
  if (nnz_in > 0 && (!csr_col || !csr_val || !csc_row || !csc_val))
    return fail(CHAP_EINVAL, "chap_problem_create: null nonzero arrays");
  for (int64_t k = 0; k < nnz_in; ++k) {
    if (csr_col[k] < 0 || csr_col[k] >= n) return fail(CHAP_EINVAL, "csr_col out of range at entry " + std::to_string(k));
    if (!std::isfinite(csr_val[k])) return fail(CHAP_EINVAL, "non-finite csr_val at entry " + std::to_string(k));
    if (csc_row[k] < 0 || csc_row[k] >= m) return fail(CHAP_EINVAL, "csc_row out of range at entry " + std::to_string(k));
    if (!std::isfinite(csc_val[k])) return fail(CHAP_EINVAL, "non-finite csc_val at entry " + std::to_string(k));
  }
  for (int32_t i = 0; i < m; ++i) {
    if (sense[i] != 'L' && sense[i] != 'G' && sense[i] != 'E')
      return fail(CHAP_EINVAL, "row " + std::to_string(i) + ": sense must be 'L', 'G' or 'E'");
    if (!std::isfinite(rhs[i])) return fail(CHAP_EINVAL, "row " + std::to_string(i) + ": rhs must be finite");
  }
  std::unique_ptr<chap_problem> P(new chap_problem());
  {
    chap_problem::Raw& R = P->raw;
    R.csr_row_ptr.assign(csr_row_ptr, csr_row_ptr + (size_t)m + 1);
    R.csc_col_ptr.assign(csc_col_ptr, csc_col_ptr + (size_t)n + 1);
    R.csr_col.assign(csr_col, csr_col + nnz_in);
    R.csr_val.assign(csr_val, csr_val + nnz_in);
    R.csc_row.assign(csc_row, csc_row + nnz_in);
    R.csc_val.assign(csc_val, csc_val + nnz_in);
    R.sense.assign(sense, sense + m);
    R.rhs.assign(rhs, rhs + m);
    R.lb.assign(lb, lb + n);
    R.ub.assign(ub, ub + n);
    R.is_int.assign(is_int, is_int + n);
    R.obj.assign(obj, obj + n);
  }
  P->n = n;
  P->m = m;
  P->opt = o;
  P->eps = o.feas_tol;
  P->lb.resize(n);
  P->ub.resize(n);
  P->obj.assign(obj, obj + n);
  P->is_int.resize(n);
  for (int32_t j = 0; j < n; ++j) {
    if (is_int[j] > 1) return fail(CHAP_EINVAL, "variable " + std::to_string(j) + ": is_int must be 0 or 1");
    double l = lb[j], u = ub[j];
    if (std::isnan(l) || std::isnan(u)) return fail(CHAP_EINVAL, "variable " + std::to_string(j) + ": NaN bound");
    if (is_int[j]) {
      l = std::ceil(l);
      u = std::floor(u);
    }
    if (l > u || l == HUGE_VAL || u == -HUGE_VAL)
      return fail(CHAP_EINVAL, "variable " + std::to_string(j) + ": empty domain");
    if (!std::isfinite(obj[j])) return fail(CHAP_EINVAL, "variable " + std::to_string(j) + ": objective must be finite");
    P->lb[j] = l;
    P->ub[j] = u;
    P->is_int[j] = is_int[j];
    if (obj[j] != 0.0 && (!is_int[j] || std::floor(obj[j]) != obj[j])) P->obj_integral = 0;
  }
  {
    double mag = 0.0;
    bool fast = P->obj_integral != 0;
    for (int32_t j = 0; j < n && fast; ++j) {
      if (obj[j] == 0.0) continue;
      fast = std::isfinite(P->lb[j]) && std::isfinite(P->ub[j]);
      mag += std::fabs(obj[j]) * std::max(std::fabs(P->lb[j]), std::fabs(P->ub[j]));
    }
    P->obj_fast = (fast && mag < 4503599627370496.0) ? 1 : 0;  // 2^52
  }
  P->x_small = 1;
  for (int32_t j = 0; j < n && P->x_small; ++j)
    P->x_small = P->is_int[j] && P->lb[j] >= -128.0 && P->ub[j] <= 127.0;
  // ---- CSR and CSC must be the same matrix (stored zeros dropped) --------
  // transpose of the CSR, rows ascending within each column
  std::vector<int64_t> tptr((size_t)n + 1, 0);
  for (int64_t k = 0; k < nnz_in; ++k)
    if (csr_val[k] != 0.0) tptr[csr_col[k] + 1] += 1;
  for (int32_t j = 0; j < n; ++j) tptr[j + 1] += tptr[j];
  const int64_t nnz = tptr[n];
  if (nnz >= (int64_t)INT32_MAX) return fail(CHAP_EINVAL, "more than 2^31-1 nonzeros");
  std::vector<int32_t> trow(nnz);
  std::vector<double> tval(nnz);
  {
    std::vector<int64_t> fill(tptr.begin(), tptr.end() - 1);
    for (int32_t i = 0; i < m; ++i)
      for (int64_t k = csr_row_ptr[i]; k < csr_row_ptr[i + 1]; ++k) {
        if (csr_val[k] == 0.0) continue;
        const int32_t c = csr_col[k];
        trow[fill[c]] = i;
        tval[fill[c]] = csr_val[k];
        fill[c] += 1;
      }
  }
  {
    std::vector<std::pair<int32_t, double>> colbuf;
    for (int32_t j = 0; j < n; ++j) {
      colbuf.clear();
      for (int64_t k = csc_col_ptr[j]; k < csc_col_ptr[j + 1]; ++k)
        if (csc_val[k] != 0.0) colbuf.emplace_back(csc_row[k], csc_val[k]);
      if ((int64_t)colbuf.size() != tptr[j + 1] - tptr[j])
        return fail(CHAP_EINVAL, "column " + std::to_string(j) + ": CSR and CSC differ");
      std::sort(colbuf.begin(), colbuf.end(),
                [](const std::pair<int32_t, double>& a, const std::pair<int32_t, double>& b) { return a.first < b.first; });
      for (size_t q = 0; q < colbuf.size(); ++q) {
        const int64_t t = tptr[j] + (int64_t)q;
        if (q > 0 && (colbuf[q].first == colbuf[q - 1].first || trow[t] == trow[t - 1]))
          return fail(CHAP_EINVAL, "column " + std::to_string(j) + ": repeated row " + std::to_string(colbuf[q].first));
        if (colbuf[q].first != trow[t] || colbuf[q].second != tval[t])
          return fail(CHAP_EINVAL, "column " + std::to_string(j) + ": CSR and CSC differ at row " +
                                       std::to_string(colbuf[q].first));
      }
    }
  }
  // ---- normalisation: one stored row per original row --------------------
  std::vector<double> sgn(m);
  std::vector<int32_t> rptr((size_t)m + 1, 0);
  std::vector<int32_t> rcol;
  std::vector<double> rval, rrhs(m);
  rcol.reserve(nnz);
  rval.reserve(nnz);
  P->nidx.resize(m);
  P->pair.resize(m);
  int32_t mp = 0;
  for (int32_t i = 0; i < m; ++i) {
    const double s = (sense[i] == 'G') ? -1.0 : 1.0;
    sgn[i] = s;
    for (int64_t k = csr_row_ptr[i]; k < csr_row_ptr[i + 1]; ++k) {
      if (csr_val[k] == 0.0) continue;
      rcol.push_back(csr_col[k]);
      rval.push_back(s * csr_val[k]);
    }
    rptr[i + 1] = (int32_t)rcol.size();
    rrhs[i] = s * rhs[i];
    P->nidx[i] = mp;
    P->pair[i] = sense[i] == 'E';
    P->norm_orig.push_back(i);
    P->norm_sign.push_back((int8_t)s);
    mp += 1;
    if (sense[i] == 'E') {
      P->norm_orig.push_back(i);
      P->norm_sign.push_back(-1);
      mp += 1;
    }
  }
  P->mp = mp;
  {
    bool exact = true;
    double max_mag = 0.0;
    for (int32_t j = 0; j < n && exact; ++j)
      exact = P->is_int[j] && std::isfinite(P->lb[j]) && std::isfinite(P->ub[j]);
    for (int32_t i = 0; i < m && exact; ++i) {
      double mag = std::fabs(rrhs[i]);
      exact = std::floor(rrhs[i]) == rrhs[i];
      for (int32_t e = rptr[i]; e < rptr[i + 1] && exact; ++e) {
        const double a = rval[e];
        const int32_t c = rcol[e];
        exact = std::floor(a) == a;
        mag += std::fabs(a) * std::max(std::fabs(P->lb[c]), std::fabs(P->ub[c]));
      }
      exact = exact && mag < 4503599627370496.0;  // 2^52
      max_mag = std::max(max_mag, mag);
    }
    P->exact_incremental = exact ? 1 : 0;
    // every residual a^T x - b with l <= x <= u is bounded by mag
    P->compact_ok = (exact && max_mag < 2147483647.0) ? 1 : 0;
  }
  // per original column: stored entries (rows ascending), degree, entries
  std::vector<int32_t> deg(n), ne(n);
  for (int32_t j = 0; j < n; ++j) {
    int32_t d = 0, e = 0;
    for (int64_t k = csc_col_ptr[j]; k < csc_col_ptr[j + 1]; ++k) {
      if (csc_val[k] == 0.0) continue;
      d += 1;
      e += P->pair[csc_row[k]] ? 2 : 1;
    }
    deg[j] = d;
    ne[j] = e + (obj[j] != 0.0 ? 1 : 0);
    P->max_col_deg = std::max(P->max_col_deg, d);
  }
  // ---- column classes and the internal column order ----------------------
  // Every kernel of the pass scores one contiguous range of internal
  // columns: short binaries (by degree), short non-binary columns by stored
  // degree D = 0..8, long binaries, narrow columns, chunked narrow columns,
  // general columns by LDS sort capacity, very long general columns.
  enum Cls { BIN, NARROW, GENERAL };
  std::vector<uint8_t> cls(n);
  for (int32_t j = 0; j < n; ++j) {
    const double l = P->lb[j], u = P->ub[j];
    if (P->is_int[j] && l == 0.0 && u == 1.0)
      cls[j] = BIN;
    else if (P->is_int[j] && std::isfinite(l) && std::isfinite(u) && u - l + 1.0 <= (double)kNarrowBins)
      cls[j] = NARROW;
    else
      cls[j] = GENERAL;
  }
  // Row-range staging needs integer residuals and coefficients (compact_ok)
  // and 0 < eps <= 1/2, under which the integer breakpoint is xbar plus the
  // floor or ceiling of -r/a. The bound below keeps FP64 rounding of
  // xbar + (eps - r)/a near [l, u] (error below 6 * 2^-53 * max(|l|,|u|) + 1
  // relative units) under eps / max|a|, the least distance of that quotient
  // from an integer, so the FP64 breakpoint equals the integer one.
  bool stage = P->compact_ok && o.row_stage == 1 && o.rescore_cap == 0 && P->eps > 0.0 && P->eps <= 0.5;
  if (stage) {
    double amax = 0.0, lmax = 0.0;
    for (double a : rval) amax = std::max(amax, std::fabs(a));
    for (int32_t j = 0; j < n; ++j)
      if (cls[j] == NARROW) lmax = std::max(lmax, std::max(std::fabs(P->lb[j]), std::fabs(P->ub[j])) + 1.0);
    stage = amax < 4194304.0 && lmax * amax <= P->eps * 17592186044416.0 &&  // 2^22, 2^44
            (int64_t)m <= (int64_t)kStageMaxRb * kStageRowBlock;
  }
  std::vector<std::vector<int32_t>> short_seg(kShortMax + 2), sortl(kSortCaps);
  std::vector<int32_t> flip, narrow, chunked, longg, sshort, sone;
  for (int32_t j = 0; j < n; ++j) {
    if (ne[j] <= o.short_max) {
      if (stage && cls[j] == NARROW && deg[j] == 1)
        sone.push_back(j);
      else if (stage && cls[j] == NARROW)
        sshort.push_back(j);
      else
        short_seg[cls[j] == BIN ? 0 : 1 + deg[j]].push_back(j);
    } else if (cls[j] == BIN) {
      flip.push_back(j);
    } else if (cls[j] == NARROW) {
      if (ne[j] <= o.chunk_min) {
        narrow.push_back(j);
      } else {
        chunked.push_back(j);
      }
    } else {
      const int32_t entries = ne[j] + 2;
      int c = 0;
      while (c < kSortCaps && kSortCap[c] < entries) ++c;
      if (c < kSortCaps)
        sortl[c].push_back(j);
      else
        longg.push_back(j);
    }
  }
  std::stable_sort(short_seg[0].begin(), short_seg[0].end(), [&](int32_t a, int32_t b) { return deg[a] < deg[b]; });
  std::stable_sort(flip.begin(), flip.end(), [&](int32_t a, int32_t b) { return deg[a] < deg[b]; });
  PassPlan& L = P->plan;
  std::vector<int32_t> perm;
  perm.reserve(n);
  auto append = [&](const std::vector<int32_t>& v) { perm.insert(perm.end(), v.begin(), v.end()); };
  L.short_seg[0] = 0;
  for (int g = 0; g < kShortMax + 2; ++g) {
    append(short_seg[g]);
    L.short_seg[g + 1] = (int32_t)perm.size();
  }
  L.flip_begin = (int32_t)perm.size();
  append(flip);
  L.flip_end = (int32_t)perm.size();
  std::vector<PackTask> packs;
  {
    int32_t q = (int32_t)perm.size();
    PackTask t{q, q};
    int64_t entries = 0;
    const int32_t pcols = stage ? kStagePackCols : kPackCols;
    const int64_t pent = stage ? kStagePackEntries : kPackEntries;
    for (int32_t j : narrow) {
      if (t.q_end > t.q_begin && (t.q_end - t.q_begin == pcols || entries + deg[j] > pent)) {
        packs.push_back(t);
        t.q_begin = t.q_end;
        entries = 0;
      }
      t.q_end += 1;
      entries += deg[j];
    }
    if (t.q_end > t.q_begin) packs.push_back(t);
  }
  append(narrow);
  // single-entry columns ordered by the row of their entry: the columns of
  // one row block form one range
  std::vector<int32_t> one_row(n, 0);
  for (int32_t j : sone)
    for (int64_t k = csc_col_ptr[j]; k < csc_col_ptr[j + 1]; ++k)
      if (csc_val[k] != 0.0) one_row[j] = csc_row[k];
  std::stable_sort(sone.begin(), sone.end(), [&](int32_t a, int32_t b) { return one_row[a] < one_row[b]; });
  L.stage_one_begin = (int32_t)perm.size();
  append(sone);
  L.stage_one_end = (int32_t)perm.size();
  L.stage_short_begin = (int32_t)perm.size();
  std::stable_sort(sshort.begin(), sshort.end(), [&](int32_t a, int32_t b) { return deg[a] < deg[b]; });
  append(sshort);
  L.stage_short_end = (int32_t)perm.size();
  const int32_t chunk_begin = (int32_t)perm.size();
  append(chunked);
  for (int c = 0; c < kSortCaps; ++c) {
    L.sort_begin[c] = (int32_t)perm.size();
    append(sortl[c]);
  }
  L.sort_begin[kSortCaps] = (int32_t)perm.size();
  const int32_t long_begin = (int32_t)perm.size();
  append(longg);
  std::vector<int32_t> inv(n);
  for (int32_t q = 0; q < n; ++q) inv[perm[q]] = q;
  // internal CSC (stored orientation, rows ascending) and per-column data
  std::vector<int32_t> cptr((size_t)n + 1, 0), crow;
  std::vector<double> cval, lbq(n), ubq(n), objq(n);
  std::vector<uint8_t> isintq(n);
  crow.reserve(nnz);
  cval.reserve(nnz);
  {
    std::vector<std::pair<int32_t, double>> buf;
    for (int32_t q = 0; q < n; ++q) {
      const int32_t j = perm[q];
      buf.clear();
      for (int64_t k = csc_col_ptr[j]; k < csc_col_ptr[j + 1]; ++k) {
        if (csc_val[k] == 0.0) continue;
        const int32_t i = csc_row[k];
        buf.emplace_back(i, sgn[i] * csc_val[k]);
      }
      std::sort(buf.begin(), buf.end(),
                [](const std::pair<int32_t, double>& a, const std::pair<int32_t, double>& b) { return a.first < b.first; });
      for (const auto& e : buf) {
        crow.push_back(e.first);
        cval.push_back(e.second);
      }
      cptr[q + 1] = (int32_t)crow.size();
      lbq[q] = P->lb[j];
      ubq[q] = P->ub[j];
      objq[q] = P->obj[j];
      isintq[q] = P->is_int[j];
    }
  }
  for (int32_t& c : rcol) c = inv[c];
  // chunk tasks of long narrow columns: each column's entries are cut at the
  // kXcds row-range boundaries and into pieces of chunk_len; the task list
  // interleaves the ranges so that task t gathers from range t mod kXcds
  std::vector<ChunkTask> tasks;
  std::vector<ChunkCol> ccols;
  {
    std::vector<std::vector<ChunkTask>> per_range(kXcds);
    int32_t slot = 0;
    for (int32_t q = chunk_begin; q < chunk_begin + (int32_t)chunked.size(); ++q) {
      ChunkCol C;
      C.col = q;
      C.first = slot;
      bool first = true;
      int32_t e = cptr[q];
      for (int r = 0; r < kXcds; ++r) {
        const int64_t row_end = ((int64_t)m * (r + 1)) / kXcds;
        int32_t e_end = e;
        while (e_end < cptr[q + 1] && crow[e_end] < row_end) ++e_end;
        for (int32_t b = e; b < e_end; b += o.chunk_len) {
          ChunkTask t;
          t.col = q;
          t.e_beg = b;
          t.e_end = std::min(e_end, b + o.chunk_len);
          t.slot = slot++;
          t.first = first ? 1 : 0;
          first = false;
          per_range[r].push_back(t);
        }
        e = e_end;
      }
      C.nparts = slot - C.first;
      ccols.push_back(C);
    }
    size_t rounds = 0;
    for (const auto& v : per_range) rounds = std::max(rounds, v.size());
    for (size_t k = 0; k < rounds; ++k)
      for (int r = 0; r < kXcds; ++r) {
        if (k < per_range[r].size()) {
          tasks.push_back(per_range[r][k]);
        } else {
          ChunkTask t{-1, 0, 0, 0, 0};
          tasks.push_back(t);
        }
      }
  }
  // staged tasks (narrow packs, then groups of short narrow columns of one
  // degree); the staged entries in (row block, task, column, row) order; the
  // segment table of every task and row block; workgroup slices of each row
  // block, XCD-interleaved so that the slices of one block share an L2
  std::vector<StageTask> stasks;
  std::vector<int32_t> sseg;
  std::vector<uint64_t> sent;
  std::vector<StageRowTask> srtasks;
  std::vector<int32_t> sunits;
  L.stage_exact = stage ? 1 : 0;
  if (stage) {
    for (const PackTask& t : packs) stasks.push_back(StageTask{t.q_begin, t.q_end, -1, 0});
    packs.clear();
    const int32_t npk = (int32_t)stasks.size();
    for (int32_t q = L.stage_short_begin; q < L.stage_short_end;) {
      const int32_t d = deg[perm[q]];
      int32_t e = q + 1;
      while (e < L.stage_short_end && e - q < kStageShort && deg[perm[e]] == d) ++e;
      stasks.push_back(StageTask{q, e, d, 0});
      q = e;
    }
    const size_t T = stasks.size();
    const int32_t nrb = (int32_t)(((int64_t)m + kStageRowBlock - 1) / kStageRowBlock);
    std::vector<std::vector<uint64_t>> ent_rb(nrb);
    sseg.assign((T + 1) * (size_t)nrb, 0);
    for (size_t t = 0; t < T; ++t) {
      for (int32_t rb = 0; rb < nrb; ++rb) sseg[t * nrb + rb] = (int32_t)ent_rb[rb].size();
      for (int32_t q = stasks[t].q_begin; q < stasks[t].q_end; ++q) {
        const uint64_t lc = (uint64_t)(q - stasks[t].q_begin);
        for (int32_t e = cptr[q]; e < cptr[q + 1]; ++e) {
          const int32_t i = crow[e], rb = i / kStageRowBlock;
          const uint64_t a24 = (uint64_t)((uint32_t)(int32_t)cval[e] & 0xFFFFFFu);
          ent_rb[rb].push_back((uint64_t)(i - rb * kStageRowBlock) | (lc << 16) | (a24 << 24));
        }
      }
    }
    for (int32_t rb = 0; rb < nrb; ++rb) sseg[T * nrb + rb] = (int32_t)ent_rb[rb].size();
    std::vector<std::vector<StageRowTask>> per_xcd(kXcds);
    // slices per row block: at most one per kStageSlice entries, and at most
    // the block's share of the workgroups the device holds at once, so that
    // the record kernel runs in one round instead of a full round and a thin
    // second one
    int64_t staged = 0, resident = 0;
    {
      int dev = 0, cus = 0;
      if (hipGetDevice(&dev) != hipSuccess ||
          hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0)
        cus = 256;
      for (const auto& v : ent_rb) staged += (int64_t)v.size();
      resident = (int64_t)kStageRowsPerCu * cus;
    }
    int32_t qone = L.stage_one_begin;
    for (int32_t rb = 0; rb < nrb; ++rb) {
      const int32_t e0 = (int32_t)sent.size();
      for (size_t t = 0; t <= T; ++t) sseg[t * nrb + rb] += e0;
      sent.insert(sent.end(), ent_rb[rb].begin(), ent_rb[rb].end());
      const int32_t e1 = (int32_t)sent.size();
      const int32_t c0 = qone;
      while (qone < L.stage_one_end && crow[cptr[qone]] < (rb + 1) * kStageRowBlock) ++qone;
      const int32_t c1 = qone;
      const int32_t by_e = (e1 - e0 + kStageSlice - 1) / kStageSlice;
      const int32_t share = (int32_t)std::max<int64_t>(1, resident * (e1 - e0) / std::max<int64_t>(staged, 1));
      const int32_t ns = std::max(std::min(by_e, share), (c1 - c0 + kStageSliceCols - 1) / kStageSliceCols);
      if (ns == 0) continue;
      const int32_t se = (e1 - e0 + ns - 1) / ns, sc = (c1 - c0 + ns - 1) / ns;
      for (int32_t k = 0; k < ns; ++k) {
        StageRowTask rt{};
        rt.rb = rb;
        rt.e_beg = std::min(e1, e0 + k * se);
        rt.e_end = std::min(e1, e0 + (k + 1) * se);
        rt.c_beg = std::min(c1, c0 + k * sc);
        rt.c_end = std::min(c1, c0 + (k + 1) * sc);
        per_xcd[rb % kXcds].push_back(rt);
      }
    }
    // per task: segment starts, then prefix counts of its records
    {
      const size_t per = 2 * (size_t)nrb + 1;
      std::vector<int32_t> tab(T * per);
      for (size_t t = 0; t < T; ++t) {
        int32_t run = 0;
        for (int32_t rb = 0; rb < nrb; ++rb) {
          tab[t * per + rb] = sseg[t * nrb + rb];
          tab[t * per + nrb + rb] = run;
          run += sseg[(t + 1) * nrb + rb] - sseg[t * nrb + rb];
        }
        tab[t * per + 2 * nrb] = run;
      }
      sseg.swap(tab);
    }
    size_t rounds = 0;
    for (const auto& v : per_xcd) rounds = std::max(rounds, v.size());
    for (size_t k = 0; k < rounds; ++k)
      for (int x = 0; x < kXcds; ++x)
        srtasks.push_back(k < per_xcd[x].size() ? per_xcd[x][k] : StageRowTask{-1, 0, 0, 0, 0, {0, 0, 0}});
    // units of the single scoring launch: chunk and pack units interleaved
    // in proportion to their counts, so that the latency-bound chunk gathers
    // and the VALU-bound pack scoring share every CU, then the short-group
    // units, the shortest workgroups, which fill the grid's last round
    {
      const int32_t cnt[3] = {(int32_t)tasks.size() / kXcds, (npk + kXcds - 1) / kXcds,
                              ((int32_t)T - npk + kXcds - 1) / kXcds};
      int32_t done[2] = {0, 0};
      for (int32_t u = 0; u < cnt[0] + cnt[1]; ++u) {
        const int r = (done[0] < cnt[0] && (done[1] >= cnt[1] || (2.0 * done[0] + 1.0) * cnt[1] <=
                                                                     (2.0 * done[1] + 1.0) * cnt[0]))
                          ? 0
                          : 1;
        sunits.push_back((r << 28) | done[r]++);
      }
      for (int32_t u = 0; u < cnt[2]; ++u) sunits.push_back((2 << 28) | u);
    }
    L.n_stage_ent = (int32_t)sent.size();
    L.n_stage_tasks = (int32_t)T;
    L.n_stage_packs = npk;
    L.n_stage_rtasks = (int32_t)srtasks.size();
    L.n_stage_rb = nrb;
    L.stage = (T > 0 || L.stage_one_end > L.stage_one_begin) ? 1 : 0;
    L.n_stage_units = L.stage ? (int32_t)sunits.size() : 0;
  }
  std::vector<LongTask> longs;
  int64_t long_total = 0;
  for (int32_t q = long_begin; q < n; ++q) {
    const int32_t entries = ne[perm[q]] + 2;
    int32_t cap = kSortCap[kSortCaps - 1];
    while (cap < entries) cap <<= 1;
    LongTask t;
    t.col = q;
    t.cap = cap;
    t.offset = long_total;
    long_total += cap;
    longs.push_back(t);
  }
  P->perm = perm;
  // learned proposal: binaries and narrow columns of any length; general
  // columns whose breakpoints fit one workgroup's LDS sort
  P->sub_cls.assign(n, SUB_NONE);
  P->col_entries.assign(n, 0);
  P->nnz = (int64_t)crow.size();
  for (int32_t q = 0; q < n; ++q) {
    const int32_t j = perm[q];
    P->col_entries[q] = cptr[q + 1] - cptr[q];
    if (cls[j] == BIN)
      P->sub_cls[q] = SUB_FLIP;
    else if (cls[j] == NARROW)
      P->sub_cls[q] = SUB_NARROW;
    else if (ne[j] + 2 <= kSubsetCap)
      P->sub_cls[q] = SUB_GENERAL;
  }
  P->c_max = 0.0;
  for (int32_t j = 0; j < n; ++j) P->c_max = std::max(P->c_max, std::fabs(P->obj[j]));
  // ---- upload --------------------------------------------------------------
  {
    int dev = 0;
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || count == 0) return fail(CHAP_ENOTBUILT, "no HIP device visible");
    CHAP_HIP(hipGetDevice(&dev));
    P->device = dev;
  }
  DeviceArena& A = P->arena;
  DevProblem& D = P->dev;
  D.n = n;
  D.ms = m;
  D.sums_exact = P->exact_incremental;
  D.eps = P->eps;
  int32_t *d_cptr, *d_crow, *d_rptr, *d_rcol, *d_perm;
  double *d_cval, *d_rval, *d_rrhs, *d_lb, *d_ub, *d_obj;
  uint8_t *d_isint, *d_pair;
  int32_t* d_nidx;
  CHAP_HIP(A.upload(&d_cptr, cptr));
  CHAP_HIP(A.upload(&d_crow, crow));
  CHAP_HIP(A.upload(&d_cval, cval));
  CHAP_HIP(A.upload(&d_rptr, rptr));
  CHAP_HIP(A.upload(&d_rcol, rcol));
  CHAP_HIP(A.upload(&d_rval, rval));
  CHAP_HIP(A.upload(&d_rrhs, rrhs));
  CHAP_HIP(A.upload(&d_lb, lbq));
  CHAP_HIP(A.upload(&d_ub, ubq));
  CHAP_HIP(A.upload(&d_obj, objq));
  CHAP_HIP(A.upload(&d_isint, isintq));
  CHAP_HIP(A.upload(&d_perm, perm));
  {
    int32_t* d_inv;
    CHAP_HIP(A.upload(&d_inv, inv));
    P->d_inv = d_inv;
  }
  // caller's order -> internal order sends j to inv[j]; back, q to perm[q]
  CHAP_HIP(build_perm_plan(inv, A, &P->to_internal));
  CHAP_HIP(build_perm_plan(perm, A, &P->to_caller));
  CHAP_HIP(A.alloc(&P->bs_stage, 2 * (size_t)n));
  CHAP_HIP(A.upload(&d_pair, P->pair));
  CHAP_HIP(A.upload(&d_nidx, P->nidx));
  D.col_ptr = d_cptr;
  D.col_row = d_crow;
  D.col_val = d_cval;
  D.row_ptr = d_rptr;
  D.row_col = d_rcol;
  D.row_val = d_rval;
  D.row_rhs = d_rrhs;
  D.lb = d_lb;
  D.ub = d_ub;
  D.obj = d_obj;
  D.is_int = d_isint;
  D.perm = d_perm;
  P->d_pair = d_pair;
  P->d_nidx = d_nidx;
  D.row_c8 = nullptr;
  {
    bool fits = true;
    for (double a : rval) fits = fits && a == std::nearbyint(a) && std::fabs(a) <= 127.0;
    if (fits && !rval.empty()) {
      std::vector<int8_t> c8(rval.size());
      for (size_t e = 0; e < rval.size(); ++e) c8[e] = (int8_t)rval[e];
      int8_t* d_c8;
      CHAP_HIP(A.upload(&d_c8, c8));
      D.row_c8 = d_c8;
    }
  }
  D.rb_ent = nullptr;
  D.rb_c8 = nullptr;
  D.rb_seg = nullptr;
  D.rb_nxb = 0;
  if (D.row_c8 && P->x_small && P->exact_incremental && m > 0 && n > 0) {
    // int32 row sums: |a| <= 127 and |x| <= 128, so sum |a| < 2^24 bounds them
    bool fits = true;
    for (int32_t i = 0; i < m && fits; ++i) {
      double mag = 0.0;
      for (int32_t e = rptr[i]; e < rptr[i + 1]; ++e) mag += std::fabs(rval[e]);
      fits = mag < 16777216.0;
    }
    if (fits) {
      const int32_t ng = (m + kResGroupRows - 1) / kResGroupRows;
      const int32_t nxb = (int32_t)(((int64_t)n + kResXBlock - 1) / kResXBlock);
      std::vector<int32_t> seg((size_t)ng * nxb + 1, 0);
      for (int32_t i = 0; i < m; ++i)
        for (int32_t e = rptr[i]; e < rptr[i + 1]; ++e)
          ++seg[(size_t)(i / kResGroupRows) * nxb + rcol[e] / kResXBlock + 1];
      for (size_t k = 1; k < seg.size(); ++k) seg[k] += seg[k - 1];
      std::vector<int32_t> fill(seg.begin(), seg.end() - 1);
      std::vector<uint32_t> ent(rcol.size());
      std::vector<int8_t> c8(rcol.size());
      for (int32_t i = 0; i < m; ++i) {
        const int32_t g = i / kResGroupRows;
        for (int32_t e = rptr[i]; e < rptr[i + 1]; ++e) {
          const int32_t b = rcol[e] / kResXBlock;
          const int32_t at = fill[(size_t)g * nxb + b]++;
          ent[at] = ((uint32_t)(i - g * kResGroupRows) << 17) | (uint32_t)(rcol[e] - b * kResXBlock);
          c8[at] = (int8_t)rval[e];
        }
      }
      uint32_t* d_ent;
      int8_t* d_c8b;
      int32_t* d_seg;
      CHAP_HIP(A.upload(&d_ent, ent));
      CHAP_HIP(A.upload(&d_c8b, c8));
      CHAP_HIP(A.upload(&d_seg, seg));
      D.rb_ent = d_ent;
      D.rb_c8 = d_c8b;
      D.rb_seg = d_seg;
      D.rb_nxb = nxb;
    }
  }
  if (!packs.empty()) {
    PackTask* dp;
    CHAP_HIP(A.upload(&dp, packs));
    L.packs = dp;
    L.n_packs = (int32_t)packs.size();
  }
  if (L.stage) {
    StageTask* dt;
    int32_t* dseg;
    uint64_t* dent;
    StageRowTask* drt;
    CHAP_HIP(A.upload(&dt, stasks));
    CHAP_HIP(A.upload(&dseg, sseg));
    CHAP_HIP(A.upload(&dent, sent));
    CHAP_HIP(A.upload(&drt, srtasks));
    L.stage_tasks = dt;
    L.stage_seg = dseg;
    L.stage_ent = dent;
    L.stage_rtasks = drt;
    if (!sunits.empty()) {
      int32_t* du;
      CHAP_HIP(A.upload(&du, sunits));
      L.stage_units = du;
    }
  }
  if (!tasks.empty()) {
    ChunkTask* dt;
    CHAP_HIP(A.upload(&dt, tasks));
    L.chunks = dt;
    L.n_chunks = (int32_t)tasks.size();
    L.n_partials = ccols.back().first + ccols.back().nparts;
    ChunkCol* dc;
    CHAP_HIP(A.upload(&dc, ccols));
    L.chunk_cols = dc;
    L.n_chunk_cols = (int32_t)ccols.size();
  }
  if (!longs.empty()) {
    LongTask* d;
    CHAP_HIP(A.upload(&d, longs));
    L.long_tasks = d;
    L.n_long = (int32_t)longs.size();
    L.long_scratch = long_total;
  }
  CHAP_HIP(A.alloc(&P->bs_x, (size_t)n));
  CHAP_HIP(A.alloc(&P->bs_xhat, (size_t)n));
  CHAP_HIP(A.alloc(&P->bs_s, (size_t)n));
  CHAP_HIP(A.alloc(&P->bs_rs, (size_t)m));
  CHAP_HIP(A.alloc(&P->bs_state, 1));
  CHAP_HIP(A.alloc(&P->bs_partial, kInitPartial));
  if (!P->obj_fast) CHAP_HIP(A.alloc(&P->bs_objacc, kExactLimbs));
  if (P->x_small) CHAP_HIP(A.alloc(&P->bs_xc, (size_t)n));
  CHAP_HIP(A.alloc(&P->bs_ticket, 1));
  CHAP_HIP(hipMemset(P->bs_ticket, 0, sizeof(uint32_t)));
  {
    // one-walk launch table of chap_best_shift over the problem's scratch
    WalkCtx c{};
    c.P = P->dev;
    c.plan = P->plan;
    c.x = P->bs_x;
    c.xhat = P->bs_xhat;
    c.s = P->bs_s;
    c.rs = P->bs_rs;
    c.st = P->bs_state;
    if (P->compact_ok) {
      CHAP_HIP(A.alloc(&P->bs_grow, (size_t)m));
      c.grow = P->bs_grow;
    }
    CHAP_HIP(A.alloc(&c.partials, (size_t)P->plan.n_partials));
    CHAP_HIP(A.alloc(&c.long_pos, (size_t)P->plan.long_scratch));
    CHAP_HIP(A.alloc(&c.long_delta, (size_t)P->plan.long_scratch));
    CHAP_HIP(A.alloc(&c.long_marker, (size_t)P->plan.long_scratch));
    CHAP_HIP(A.alloc(&c.stage_rec, (size_t)P->plan.n_stage_ent));
    std::vector<WalkCtx> one{c};
    CHAP_HIP(build_launch(A, one, &P->bs_launch, nullptr));
    P->bs_launch.compact = P->compact_ok ? 2 : 0;
  }
  CHAP_HIP(P->bs_streams.create());
  CHAP_HIP(hipEventCreate(&P->pass_ev[0]));
  CHAP_HIP(hipEventCreate(&P->pass_ev[1]));
  P->pool = std::make_shared<WalkPool>();
  P->pool->n = n;
  P->pool->m = m;
  P->pool->mp = P->mp;
  P->pool->perm = P->perm;
  P->pool->nidx = P->nidx;
  P->pool->pair = P->pair;
  CHAP_HIP(hipDeviceSynchronize());
  *out = P.release();
  return CHAP_OK;
}

int chap_best_shift(chap_problem* p, const double* d_x, const float* d_w, double cutoff_rhs, double* d_shift,
                    double* d_score, void* hip_stream) {
  if (!p) return fail(CHAP_EINVAL, "chap_best_shift: null problem");
  if (p->n > 0 && (!d_x || !d_shift || !d_score)) return fail(CHAP_EINVAL, "chap_best_shift: null device array");
  if (!d_w) return fail(CHAP_EINVAL, "chap_best_shift: null weights");
  if (std::isnan(cutoff_rhs)) return fail(CHAP_EINVAL, "chap_best_shift: cutoff_rhs is NaN");
  hipStream_t s = (hipStream_t)hip_stream;
  const uint32_t epoch = ++p->bs_epoch == 0 ? ++p->bs_epoch : p->bs_epoch;  // never 0
  CHAP_HIP(launch_stage_x_plan(p->to_internal, d_x, p->bs_x, p->bs_xc, p->bs_state, epoch, p->bs_stage, s));
  // the state first (a single pass counts no violated rows, so it reads no
  // residual), then the residuals with the compact copy and its check
  const double cut = (cutoff_rhs == HUGE_VAL) ? HUGE_VAL : cutoff_rhs;
  CHAP_HIP(launch_state_init(p->dev, p->bs_x, p->bs_rs, p->bs_state, p->bs_partial, p->bs_ticket, p->bs_objacc, 1,
                             0, p->obj_integral, cut, d_w + p->mp, 0, 0, s));
  CHAP_HIP(launch_residual_scatter(p->dev, p->d_nidx, p->d_pair, d_w, p->bs_x, p->bs_xc, p->bs_state, epoch,
                                   p->bs_rs, s, p->bs_grow));
  if (p->n > 0 && !p->bs_exec) {
    // capture the pass once (its arguments are the problem's own buffers)
    if (!p->bs_cap) CHAP_HIP(hipStreamCreateWithFlags(&p->bs_cap, hipStreamNonBlocking));
    CHAP_HIP(hipStreamBeginCapture(p->bs_cap, hipStreamCaptureModeThreadLocal));
    const hipError_t cap_err = launch_pass(p->bs_launch, p->bs_cap, &p->bs_streams);
    hipGraph_t graph = nullptr;
    const hipError_t end_err = hipStreamEndCapture(p->bs_cap, &graph);
    if (cap_err != hipSuccess || end_err != hipSuccess) {
      if (graph) (void)hipGraphDestroy(graph);
      return fail(CHAP_EHIP, std::string("pass capture: ") +
                                 hipGetErrorString(cap_err != hipSuccess ? cap_err : end_err));
    }
    hipGraphExec_t exec = nullptr;
    const hipError_t ie = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    if (ie != hipSuccess) {
      (void)hipGraphDestroy(graph);
      return fail(CHAP_EHIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(ie));
    }
    p->bs_graph = graph;
    p->bs_exec = exec;
  }
  CHAP_HIP(hipEventRecord(p->pass_ev[0], s));
  if (p->n > 0) CHAP_HIP(hipGraphLaunch(p->bs_exec, s));
  CHAP_HIP(hipEventRecord(p->pass_ev[1], s));
  CHAP_HIP(launch_gather2_plan(p->to_caller, p->bs_xhat, p->bs_s, d_shift, d_score, p->bs_stage, s));
  p->pass_timed = true;
  return CHAP_OK;
}

int chap_best_shift_pass_ms(chap_problem* p, double* ms) {
  if (!p || !ms) return fail(CHAP_EINVAL, "chap_best_shift_pass_ms: null argument");
  *ms = 0.0;
  if (!p->pass_timed) return CHAP_OK;
  CHAP_HIP(hipEventSynchronize(p->pass_ev[1]));
  float t = 0.0f;
  CHAP_HIP(hipEventElapsedTime(&t, p->pass_ev[0], p->pass_ev[1]));
  *ms = t;
  return CHAP_OK;
}

}  // extern "C"

namespace chap {

hipError_t build_perm_plan(const std::vector<int32_t>& dest, DeviceArena& A, PermPlan* plan) {
  const int32_t n = (int32_t)dest.size();
  plan->n = n;
  if (n == 0) return hipSuccess;
  const int32_t nb = (int32_t)(((int64_t)n + kPermBlock - 1) / kPermBlock);
  std::vector<uint16_t> lpos((size_t)n), dl((size_t)n);
  std::vector<int32_t> sdst((size_t)n);
  std::vector<int32_t> filled((size_t)nb, 0);  // slots of each output block taken by earlier chunks
  std::vector<std::pair<int32_t, int32_t>> items;
  items.reserve(kPermChunk);
  for (int64_t base = 0; base < n; base += kPermChunk) {
    const int64_t end = std::min<int64_t>(n, base + kPermChunk);
    items.clear();
    for (int64_t e = base; e < end; ++e) items.emplace_back(dest[(size_t)e] / kPermBlock, (int32_t)e);
    std::sort(items.begin(), items.end());  // by output block, then input index
    for (size_t r = 0; r < items.size(); ++r) {
      const int32_t b = items[r].first, e = items[r].second;
      const int32_t slot = b * kPermBlock + filled[(size_t)b]++;
      lpos[(size_t)e] = (uint16_t)r;
      sdst[(size_t)(base + (int64_t)r)] = slot;
      dl[(size_t)slot] = (uint16_t)(dest[(size_t)e] - b * kPermBlock);
    }
  }
  uint16_t *d_lpos, *d_dl;
  int32_t* d_sdst;
  hipError_t e;
  if ((e = A.upload(&d_lpos, lpos)) != hipSuccess) return e;
  if ((e = A.upload(&d_sdst, sdst)) != hipSuccess) return e;
  if ((e = A.upload(&d_dl, dl)) != hipSuccess) return e;
  plan->lpos = d_lpos;
  plan->sdst = d_sdst;
  plan->dl = d_dl;
  return hipSuccess;
}

int alloc_walk(const chap_problem* p, int64_t trace_cap, DeviceArena& A, WalkCtx& c) {
  const int32_t n = p->n;
  c = WalkCtx{};
  c.P = p->dev;
  c.plan = p->plan;
  c.argmax_blocks = blocks_for_host(n, kArgmaxBlocks);
  c.argmax_comb = p->plan.stage ? (p->plan.n_chunk_cols + 3) / 4 : 0;
  c.apply_blocks = blocks_for_host(std::max(p->m, p->max_col_deg), 256);
  c.recompute = p->exact_incremental ? 0 : 1;
  CHAP_HIP(A.alloc(&c.x, (size_t)n));
  CHAP_HIP(A.alloc(&c.xhat, (size_t)n));
  CHAP_HIP(A.alloc(&c.s, (size_t)n));
  CHAP_HIP(A.alloc(&c.best_x, (size_t)n));
  CHAP_HIP(A.alloc(&c.tabu, (size_t)n));
  CHAP_HIP(A.alloc(&c.rs, (size_t)p->m));
  CHAP_HIP(A.alloc(&c.st, 1));
  if (trace_cap > 0) CHAP_HIP(A.alloc(&c.trace, (size_t)trace_cap));
  CHAP_HIP(A.alloc(&c.argmax_partial, (size_t)kArgmaxRecord * (c.argmax_blocks + c.argmax_comb)));
  CHAP_HIP(A.alloc(&c.partials, (size_t)p->plan.n_partials));
  CHAP_HIP(A.alloc(&c.long_pos, (size_t)p->plan.long_scratch));
  CHAP_HIP(A.alloc(&c.long_delta, (size_t)p->plan.long_scratch));
  CHAP_HIP(A.alloc(&c.long_marker, (size_t)p->plan.long_scratch));
  CHAP_HIP(A.alloc(&c.stage_rec, (size_t)p->plan.n_stage_ent));
  if (p->compact_ok) CHAP_HIP(A.alloc(&c.grow, (size_t)p->m));
  if (!p->obj_fast) CHAP_HIP(A.alloc(&c.objacc, (size_t)kExactLimbs));
  if (p->x_small) CHAP_HIP(A.alloc(&c.xc, (size_t)n));
  return CHAP_OK;
}

int init_walk(const WalkSpec& spec, int64_t iters, int32_t tenure, const WalkCtx& c, double* partial,
              uint32_t* ticket, hipStream_t s) {
  const chap_problem* p = spec.p;
  const int32_t n = p->n;
  if (spec.x0) {
    for (int32_t j = 0; j < n; ++j) {
      const double v = spec.x0[j];
      if (!std::isfinite(v)) return fail(CHAP_EINVAL, "non-finite start value at " + std::to_string(j));
      if (v < p->lb[j] || v > p->ub[j] || (p->is_int[j] && std::floor(v) != v))
        return fail(CHAP_EINVAL, "start value at " + std::to_string(j) +
                                     " outside the bounds or fractional on an integer variable");
    }
  }
  // the cleared state has x_misfit = 0; this call's epoch is 1
  CHAP_HIP(hipMemsetAsync(c.st, 0, sizeof(WalkState), s));
  if (spec.x0) {
    // caller's order into xhat (free until the first pass), then internal order
    if (n > 0) {
      CHAP_HIP(hipStreamSynchronize(s));
      CHAP_HIP(hipMemcpy(c.xhat, spec.x0, sizeof(double) * (size_t)n, hipMemcpyHostToDevice));
      CHAP_HIP(launch_stage_x(p->dev.perm, c.xhat, c.x, c.xc, c.st, 1u, n, s));
    }
  } else {
    CHAP_HIP(launch_start_point(p->dev, spec.seed, c.x, c.xc, s));
  }
  if (n > 0) {
    hipLaunchKernelGGL(k_fill_i32, dim3((n + 255) / 256), dim3(256), 0, s, c.tabu, -1, (int64_t)n);
    CHAP_HIP(hipGetLastError());
  }
  CHAP_HIP(launch_residual_unit(p->dev, p->d_pair, c.x, c.xc, c.st, 1u, c.rs, c.grow, s));
  CHAP_HIP(launch_state_init(p->dev, c.x, c.rs, c.st, partial, ticket, c.objacc, iters, tenure, p->obj_integral,
                             HUGE_VAL, nullptr, 1, 1, s));
  CHAP_HIP(launch_copy_best(c.x, c.best_x, c.st, n, s));
  return CHAP_OK;
}

int prepare_walk(const WalkSpec& spec, int64_t iters, int32_t tenure, DeviceArena& A, WalkCtx& c, double* partial,
                 uint32_t* ticket, hipStream_t s, int compact) {
  int rc = alloc_walk(spec.p, std::max<int64_t>(iters, 1), A, c);
  if (rc != CHAP_OK) return rc;
  if (!compact) c.grow = nullptr;
  rc = init_walk(spec, iters, tenure, c, partial, ticket, s);
  if (rc != CHAP_OK) return rc;
  CHAP_HIP(hipStreamSynchronize(s));
  return CHAP_OK;
}

namespace {

// Final state in the caller's order: x and best_x from internal order,
// residuals and weights of the normalised rows (an equality row's twin has
// residual -r and the second weight), the cutoff row last.
void fill_state(int32_t n, int32_t m, int32_t mp, const int32_t* perm, const int32_t* nidx, const uint8_t* pair,
                const double* xin, const double* bxin, const RowState* rs, const WalkState& st, chap_run* R) {
  R->x.resize(n);
  std::vector<double> bx(n);
  for (int32_t q = 0; q < n; ++q) {
    R->x[perm[q]] = xin[q];
    bx[perm[q]] = bxin[q];
  }
  R->resid.assign((size_t)mp + 1, 0.0);
  R->w.assign((size_t)mp + 1, 0.0f);
  for (int32_t i = 0; i < m; ++i) {
    const int32_t k = nidx[i];
    R->resid[k] = rs[i].r;
    R->w[k] = rs[i].w0;
    if (pair[i]) {
      R->resid[k + 1] = -rs[i].r;
      R->w[k + 1] = rs[i].w1;
    }
  }
  R->resid[mp] = st.cut_active ? st.rc : 0.0;
  R->w[mp] = st.wc;
  if (R->has_best) R->best_x.swap(bx);
}

void fill_summary(const WalkState& st, chap_run* R) {
  R->st_end = st;
  R->has_best = st.has_best != 0;
  R->best_obj = st.has_best ? st.fbest : HUGE_VAL;
  R->cutoff_rhs = st.cut_active ? st.bc : HUGE_VAL;
  R->inf_iter = st.inf_k;
  R->inf_viol = st.inf_k == -2 ? 0 : st.inf_V;
}

// The best infeasible point from the final point: the moves after the
// iteration that reached it are undone in reverse order.
void rebuild_infeasible(chap_run* R) {
  R->inf_x.clear();
  if (R->inf_iter == -2) return;
  R->inf_x = R->x;
  for (int64_t k = (int64_t)R->trace.size() - 1; k > R->inf_iter; --k) {
    const chap_trace_record& t = R->trace[(size_t)k];
    if (t.var >= 0) R->inf_x[t.var] = t.x_old;
  }
}

}  // namespace

int collect_walk(const chap_problem* p, const WalkCtx& c, int64_t iters, double ms, chap_run* R) {
  const int32_t n = p->n, m = p->m;
  R->elapsed_ms = ms;
  R->trace.resize((size_t)iters);
  if (iters > 0)
    CHAP_HIP(hipMemcpy(R->trace.data(), c.trace, sizeof(chap_trace_record) * (size_t)iters, hipMemcpyDeviceToHost));
  std::vector<double> xin(n), bxin(n);
  if (n > 0) {
    CHAP_HIP(hipMemcpy(xin.data(), c.x, sizeof(double) * (size_t)n, hipMemcpyDeviceToHost));
    CHAP_HIP(hipMemcpy(bxin.data(), c.best_x, sizeof(double) * (size_t)n, hipMemcpyDeviceToHost));
  }
  std::vector<RowState> rs(m);
  if (m > 0) CHAP_HIP(hipMemcpy(rs.data(), c.rs, sizeof(RowState) * (size_t)m, hipMemcpyDeviceToHost));
  WalkState st;
  CHAP_HIP(hipMemcpy(&st, c.st, sizeof(WalkState), hipMemcpyDeviceToHost));
  fill_summary(st, R);
  fill_state(n, m, p->mp, p->perm.data(), p->nidx.data(), p->pair.data(), xin.data(), bxin.data(), rs.data(), st, R);
  rebuild_infeasible(R);
  return CHAP_OK;
}

// Reads a single walk's final state from its slot (first chap_run_state
// that asks for it), then returns the slot to the problem.
int materialize(const chap_run* R) {
  if (R->state_ready) return CHAP_OK;
  const WalkPool& M = *R->pool;
  const WalkCtx& c = R->slot->ctx;
  std::vector<double> xin(M.n), bxin(M.n);
  std::vector<RowState> rs(M.m);
  if (M.n > 0) {
    CHAP_HIP(hipMemcpy(xin.data(), c.x, sizeof(double) * (size_t)M.n, hipMemcpyDeviceToHost));
    CHAP_HIP(hipMemcpy(bxin.data(), c.best_x, sizeof(double) * (size_t)M.n, hipMemcpyDeviceToHost));
  }
  if (M.m > 0) CHAP_HIP(hipMemcpy(rs.data(), c.rs, sizeof(RowState) * (size_t)M.m, hipMemcpyDeviceToHost));
  chap_run* W = const_cast<chap_run*>(R);
  fill_state(M.n, M.m, M.mp, M.perm.data(), M.nidx.data(), M.pair.data(), xin.data(), bxin.data(), rs.data(),
             R->st_end, W);
  rebuild_infeasible(W);
  R->state_ready = true;
  R->pool->give_back(R->slot);
  return CHAP_OK;
}

}  // namespace chap

namespace chap {

int compact_walks(const std::vector<WalkSpec>& specs, int64_t iters) {
  // weights start at 1 and grow by at most 1 per iteration
  if (iters + 1 >= (int64_t)kNoTwin) return 0;
  for (const WalkSpec& w : specs)
    if (!w.p->compact_ok) return 0;
  return 1;
}

}  // namespace chap

namespace {

// Diversity restarts of a batch: segments of `every` iterations; at the end
// of each segment but the last, walk w restarts when a walk w' < w on the
// same problem lies at Hamming distance < min_distance over the discrete
// variables (distances of the points before any restart of that boundary).
struct RestartSpec {
  int64_t every = 0;
  int64_t min_distance = 0;
};

constexpr uint64_t kRestartSeedStep = 0x9E3779B97F4A7C15ull;

// Hamming tasks of every pair (w' < w) of walks on one problem, in chunks of
// 65536 columns; pair index = position in `pairs`.
void hamming_tasks(const std::vector<WalkSpec>& specs, const std::vector<WalkCtx>& ctx,
                   const std::vector<int32_t>& slot_of, std::vector<std::pair<int32_t, int32_t>>& pairs,
                   std::vector<HamTask>& tasks) {
  const int32_t nw = (int32_t)specs.size();
  for (int32_t w = 0; w < nw; ++w)
    for (int32_t v = 0; v < w; ++v) {
      if (specs[v].p != specs[w].p) continue;
      const int32_t pair = (int32_t)pairs.size();
      pairs.emplace_back(w, v);
      const WalkCtx& a = ctx[slot_of[w]];
      const WalkCtx& b = ctx[slot_of[v]];
      const int32_t n = specs[w].p->n;
      for (int32_t q = 0; q < n; q += 65536)
        tasks.push_back(HamTask{a.x, b.x, a.P.is_int, q, std::min(n, q + 65536), pair, 0});
    }
}

// Runs every walk for `iters` iterations: per-walk buffers, set-up kernels,
// then a HIP graph of `graph_iters` iterations in which each kernel is one
// launch over all walks. Results are copied back into chap_run objects.
// With rsp, the walks run in segments with diversity restarts between them.
int run_walks(const std::vector<WalkSpec>& specs, int64_t iters, int32_t tenure, hipStream_t user,
              std::vector<std::unique_ptr<chap_run>>& out, const RestartSpec* rsp = nullptr) {
  if (iters < 0 || tenure < 0 || iters + (int64_t)tenure >= (int64_t)INT32_MAX)
    return fail(CHAP_EINVAL, "iters and tenure must be >= 0 with iters + tenure < 2^31");
  const size_t nw = specs.size();
  DeviceArena A;
  std::vector<WalkCtx> ctx(nw);
  double* partial;
  uint32_t* ticket;
  CHAP_HIP(A.alloc(&partial, kInitPartial));
  CHAP_HIP(A.alloc(&ticket, 1));
  hipStream_t s;
  CHAP_HIP(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
  struct StreamGuard {
    hipStream_t s;
    PassStreams ps;
    ~StreamGuard() {
      ps.destroy();
      (void)hipStreamDestroy(s);
    }
  } sg{s, {}};
  CHAP_HIP(sg.ps.create());
  hipEvent_t e_user, e0, e1;
  CHAP_HIP(hipEventCreate(&e_user));
  CHAP_HIP(hipEventCreate(&e0));
  CHAP_HIP(hipEventCreate(&e1));
  struct EventGuard {
    hipEvent_t a, b, c;
    ~EventGuard() {
      (void)hipEventDestroy(a);
      (void)hipEventDestroy(b);
      (void)hipEventDestroy(c);
    }
  } eg{e_user, e0, e1};
  CHAP_HIP(hipEventRecord(e_user, user));
  CHAP_HIP(hipStreamWaitEvent(s, e_user, 0));
  CHAP_HIP(hipMemsetAsync(ticket, 0, sizeof(uint32_t), s));
  const int compact = compact_walks(specs, iters);
  for (size_t w = 0; w < nw; ++w) {
    const int rc = prepare_walk(specs[w], iters, tenure, A, ctx[w], partial, ticket, s, compact);
    if (rc != CHAP_OK) return rc;
  }
  BatchLaunch L;
  std::vector<int32_t> order;
  CHAP_HIP(build_launch(A, ctx, &L, &order));
  L.compact = compact;
  double ms_total = 0.0;
  std::vector<std::vector<int64_t>> restarts;
  if (iters > 0) {
    int64_t K = std::min<int64_t>(iters, specs[0].p->opt.graph_iters);
    if (rsp && rsp->every > 0) K = std::min<int64_t>(K, rsp->every);
    hipGraph_t graph;
    CHAP_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
    hipError_t cap_err = hipSuccess;
    for (int64_t q = 0; q < K && cap_err == hipSuccess; ++q) {
      cap_err = launch_pass(L, s, &sg.ps, true);
      if (cap_err == hipSuccess) cap_err = launch_walk_step(L, s, true);
    }
    hipError_t end_err = hipStreamEndCapture(s, &graph);
    if (cap_err != hipSuccess) return fail(CHAP_EHIP, std::string("graph capture: ") + hipGetErrorString(cap_err));
    if (end_err != hipSuccess) return fail(CHAP_EHIP, std::string("hipStreamEndCapture: ") + hipGetErrorString(end_err));
    hipGraphExec_t exec;
    hipError_t ie = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    if (ie != hipSuccess) {
      (void)hipGraphDestroy(graph);
      return fail(CHAP_EHIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(ie));
    }
    struct GraphGuard {
      hipGraph_t g;
      hipGraphExec_t x;
      ~GraphGuard() {
        (void)hipGraphExecDestroy(x);
        (void)hipGraphDestroy(g);
      }
    } gg{graph, exec};
    const int64_t every = (rsp && rsp->every > 0) ? rsp->every : iters;
    std::vector<int32_t> slot_of(nw);
    for (size_t i = 0; i < nw; ++i) slot_of[order[i]] = (int32_t)i;
    std::vector<std::pair<int32_t, int32_t>> pairs;
    std::vector<HamTask> htasks;
    HamTask* d_htasks = nullptr;
    int32_t* d_dist = nullptr;
    std::vector<WalkState> hst;
    if (every < iters) {
      hamming_tasks(specs, ctx, slot_of, pairs, htasks);
      if (!htasks.empty()) CHAP_HIP(A.upload(&d_htasks, htasks));
      CHAP_HIP(A.alloc(&d_dist, std::max<size_t>(pairs.size(), 1)));
      hst.resize(nw);
    }
    restarts.assign(nw, {});
    std::vector<int64_t> count(nw, 0);
    for (int64_t k0 = 0; k0 < iters;) {
      const int64_t k1 = std::min(iters, k0 + every);
      // the segment: every walk stops at k1; surplus iterations of the last
      // graph launch do nothing
      if (every < iters) CHAP_HIP(launch_set_iters(L, k1, s));
      const int64_t launches = (k1 - k0 + K - 1) / K;
      hipError_t le = hipEventRecord(e0, s);
      for (int64_t q = 0; q < launches && le == hipSuccess; ++q) le = hipGraphLaunch(exec, s);
      if (le == hipSuccess) le = hipEventRecord(e1, s);
      // an incumbent found by a walk's last iteration is copied here
      if (le == hipSuccess) le = launch_copy_best_batch(L, s);
      if (le == hipSuccess) le = hipStreamSynchronize(s);
      float ms = 0.0f;
      if (le == hipSuccess) le = hipEventElapsedTime(&ms, e0, e1);
      if (le != hipSuccess) return fail(CHAP_EHIP, std::string("graph launch: ") + hipGetErrorString(le));
      ms_total += ms;
      k0 = k1;
      if (k1 >= iters || pairs.empty()) continue;
      // distances at the boundary, then the restarts
      CHAP_HIP(hipMemsetAsync(d_dist, 0, sizeof(int32_t) * pairs.size(), s));
      CHAP_HIP(launch_hamming(d_htasks, (int32_t)htasks.size(), d_dist, s));
      std::vector<int32_t> dist(pairs.size());
      CHAP_HIP(hipMemcpyAsync(dist.data(), d_dist, sizeof(int32_t) * pairs.size(), hipMemcpyDeviceToHost, s));
      for (size_t i = 0; i < nw; ++i)
        CHAP_HIP(hipMemcpyAsync(&hst[i], ctx[i].st, sizeof(WalkState), hipMemcpyDeviceToHost, s));
      CHAP_HIP(hipStreamSynchronize(s));
      std::vector<char> restart(nw, 0);
      for (size_t pi = 0; pi < pairs.size(); ++pi)
        if (dist[pi] < rsp->min_distance) restart[pairs[pi].first] = 1;
      for (size_t w = 0; w < nw; ++w) {
        if (!restart[w]) continue;
        const int32_t i = slot_of[w];
        const WalkCtx& c = ctx[i];
        const chap_problem* p = specs[w].p;
        const WalkState& old = hst[i];
        count[w] += 1;
        restarts[w].push_back(k1);
        const uint64_t seed = specs[w].seed + (uint64_t)count[w] * kRestartSeedStep;
        CHAP_HIP(launch_start_point(p->dev, seed, c.x, c.xc, s));
        if (p->n > 0) {
          hipLaunchKernelGGL(k_fill_i32, dim3((p->n + 255) / 256), dim3(256), 0, s, c.tabu, -1, (int64_t)p->n);
          CHAP_HIP(hipGetLastError());
        }
        CHAP_HIP(launch_residual_unit(p->dev, p->d_pair, c.x, c.xc, c.st, 1u, c.rs, c.grow, s));
        CHAP_HIP(launch_state_init(p->dev, c.x, c.rs, c.st, partial, ticket, c.objacc, k1, tenure, p->obj_integral,
                                   old.cut_active ? old.bc : HUGE_VAL, nullptr, 1, 1, s));
        RestartKeep keep{old.k, old.fbest, old.inf_V, old.inf_k, old.has_best, 0};
        CHAP_HIP(launch_restart_fix(c.st, keep, s));
      }
    }
  }
  CHAP_HIP(hipStreamSynchronize(s));
  out.clear();
  out.resize(nw);
  for (size_t i = 0; i < nw; ++i) {
    const int32_t w = order[i];  // ctx is in XCD order
    std::unique_ptr<chap_run> R(new chap_run());
    const int rc = collect_walk(specs[w].p, ctx[i], iters, ms_total, R.get());
    if (rc != CHAP_OK) return rc;
    if (rsp) {
      R->restarts = restarts.empty() ? std::vector<int64_t>() : restarts[w];
      R->restart_run = true;
    }
    out[w] = std::move(R);
  }
  return CHAP_OK;
}

// Buffers, launch table and streams of a new walk slot for problem p.
int slot_setup(const chap_problem* p, WalkSlot& S) {
  int rc = alloc_walk(p, 0, S.A, S.ctx);
  if (rc != CHAP_OK) return rc;
  S.grow_buf = S.ctx.grow;
  S.ctx.grow = nullptr;
  CHAP_HIP(S.A.alloc(&S.partial, kInitPartial));
  CHAP_HIP(S.A.alloc(&S.ticket, 1));
  CHAP_HIP(hipMemset(S.ticket, 0, sizeof(uint32_t)));
  CHAP_HIP(hipStreamCreateWithFlags(&S.s, hipStreamNonBlocking));
  CHAP_HIP(S.ps.create());
  for (hipEvent_t& e : S.ev) CHAP_HIP(hipEventCreate(&e));
  std::vector<WalkCtx> one{S.ctx};
  CHAP_HIP(build_launch(S.A, one, &S.L, nullptr));
  if (p->opt.rescore_cap > 0) {
    // affected rescoring: the subset pass's record and the lane list, fed
    // with the affected columns of each iteration (or with all columns)
    const int32_t n = p->n;
    const int32_t cap = p->opt.rescore_cap;
    const int32_t* seg = p->plan.short_seg;
    AffLists& F = S.aff;
    CHAP_HIP(S.A.alloc(&F.stamp, (size_t)std::max<int32_t>(n, 1)));
    CHAP_HIP(S.A.alloc(&F.slist, (size_t)cap + (size_t)kWave * kAffClasses));
    CHAP_HIP(S.A.alloc(&F.olist, (size_t)cap));
    CHAP_HIP(S.A.alloc(&F.ooff, (size_t)cap + 1));
    CHAP_HIP(S.A.alloc(&F.run, 1));
    CHAP_HIP(hipMemset(F.run, 0, sizeof(AffRun)));
    F.cap = cap;
    // all columns, split as an iteration's list is, when every column outside
    // the short range has a subset form
    bool all = n > 0;
    std::vector<int32_t> sl, ol, oo(1, 0);
    for (int c = 0; c < kAffClasses; ++c) {
      const int32_t lo = seg[c], hi = seg[c + 1];
      for (int32_t q = lo; q < hi; ++q) sl.push_back(q);
      while (sl.size() % kWave) sl.push_back(-1);
    }
    for (int32_t q = 0; q < n; ++q) {
      if (q >= seg[0] && q < seg[kShortMax + 2]) continue;
      const uint8_t cl = p->sub_cls[q];
      if (cl == SUB_NONE) all = false;
      ol.push_back(q);
      const int32_t c = (cl == SUB_GENERAL || cl == SUB_NONE)
                            ? 0
                            : std::max<int32_t>(1, (p->col_entries[q] + kSubsetChunk - 1) / kSubsetChunk);
      oo.push_back(oo.back() + c);
    }
    int64_t sub_cap = p->nnz / kSubsetChunk + cap + 1;
    if (all) {
      int32_t *d_sl = nullptr, *d_ol = nullptr, *d_oo = nullptr;
      CHAP_HIP(S.A.upload(&d_sl, sl.empty() ? std::vector<int32_t>(1, -1) : sl));
      CHAP_HIP(S.A.upload(&d_ol, ol.empty() ? std::vector<int32_t>(1, 0) : ol));
      CHAP_HIP(S.A.upload(&d_oo, oo));
      F.full_slist = d_sl;
      F.full_olist = d_ol;
      F.full_ooff = d_oo;
      F.n_full_s = (int32_t)sl.size();
      F.n_full_o = (int32_t)ol.size();
      F.full_chunks = oo.back();
      sub_cap = std::max<int64_t>(sub_cap, oo.back());
    }
    F.sub_cap = (int32_t)std::min<int64_t>(INT32_MAX, sub_cap);
    LearnCtx& L = S.aff_Lh;
    L = LearnCtx{};
    uint8_t* d_cls;
    CHAP_HIP(S.A.upload(&d_cls, p->sub_cls));
    L.cls = d_cls;
    L.short_lane = 1;
    L.K[0] = cap;
    L.sel[0] = F.olist;
    L.sub_off = F.ooff;
    L.sub_cap = F.sub_cap;
    CHAP_HIP(S.A.alloc(&L.sub_parts, (size_t)L.sub_cap));
    CHAP_HIP(S.A.alloc(&L.ls, 1));
    CHAP_HIP(hipMemset(L.ls, 0, sizeof(LearnState)));
    CHAP_HIP(S.A.alloc(&S.aff_L, 1));
    CHAP_HIP(hipMemcpy(S.aff_L, &L, sizeof(LearnCtx), hipMemcpyHostToDevice));
    S.aff_general = 0;
    for (uint8_t c : p->sub_cls) S.aff_general |= (c == SUB_GENERAL) ? 1 : 0;
  }
  return CHAP_OK;
}

// The graph of K iterations for the slot's walk (captured on first use).
int slot_graph(WalkSlot& S, int64_t K, int compact, hipGraphExec_t* out) {
  for (const WalkSlot::Graph& g : S.graphs)
    if (g.K == K && g.compact == compact) {
      *out = g.x;
      return CHAP_OK;
    }
  hipGraph_t graph = nullptr;
  CHAP_HIP(hipStreamBeginCapture(S.s, hipStreamCaptureModeThreadLocal));
  hipError_t cap_err = hipSuccess;
  const AffLists& F = S.aff;
  const int32_t n = S.ctx.P.n;
  for (int64_t q = 0; q < K && cap_err == hipSuccess; ++q) {
    if (S.aff_L) {
      // affected rescoring: the lists, the full pass only where no split of
      // all columns exists, the short columns by lanes, the rest by the
      // subset kernels
      cap_err = launch_affected(S.L.walks, S.aff_L, F, S.s);
      if (cap_err == hipSuccess && !F.full_slist) cap_err = launch_pass(S.L, S.s, &S.ps, true);
      if (cap_err == hipSuccess) {
        const int g[4] = {std::min(1024, (n + 255) / 256), S.aff_general ? std::min(256, (n + 3) / 4) : 0,
                          std::min(256, F.sub_cap), S.aff_general ? 32 : 0};
        cap_err = launch_aff_score(S.L.walks, S.aff_L, F.run, g, 64, compact, S.s);
      }
    } else {
      cap_err = launch_pass(S.L, S.s, &S.ps, true);
    }
    if (cap_err == hipSuccess) cap_err = launch_walk_step(S.L, S.s, true);
  }
  const hipError_t end_err = hipStreamEndCapture(S.s, &graph);
  if (cap_err != hipSuccess || end_err != hipSuccess) {
    if (graph) (void)hipGraphDestroy(graph);
    return fail(CHAP_EHIP, std::string("graph capture: ") + hipGetErrorString(cap_err != hipSuccess ? cap_err : end_err));
  }
  hipGraphExec_t exec = nullptr;
  const hipError_t ie = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
  if (ie != hipSuccess) {
    (void)hipGraphDestroy(graph);
    return fail(CHAP_EHIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(ie));
  }
  S.graphs.push_back(WalkSlot::Graph{K, compact, graph, exec});
  *out = exec;
  return CHAP_OK;
}

// One walk on the problem's cached slot. The iterations run as graphs of
// graph_iters iterations and, for the rest, of decreasing powers of two, so
// a slot holds a handful of graphs whatever `iters` is and no iteration is
// launched beyond `iters`. The final point, residuals and weights stay on the
// device until the caller asks for them.
int run_single(chap_problem* p, uint64_t seed, const double* x0, int64_t iters, int32_t tenure, hipStream_t user,
               std::unique_ptr<chap_run>& out) {
  if (iters < 0 || tenure < 0 || iters + (int64_t)tenure >= (int64_t)INT32_MAX)
    return fail(CHAP_EINVAL, "iters and tenure must be >= 0 with iters + tenure < 2^31");
  const WalkSpec spec{p, seed, x0};
  const int compact = compact_walks({spec}, iters);
  std::unique_ptr<WalkSlot> slot;
  if (!p->pool->idle.empty()) {
    slot = std::move(p->pool->idle.back());
    p->pool->idle.pop_back();
  } else {
    slot.reset(new WalkSlot());
    const int rc = slot_setup(p, *slot);
    if (rc != CHAP_OK) return rc;
  }
  WalkSlot& S = *slot;
  // trace capacity and compact rows of this run, in the device record
  bool dirty = false;
  if (iters > S.trace_cap) {
    if (S.trace_buf) CHAP_HIP(hipFree(S.trace_buf));
    S.trace_buf = nullptr;
    S.trace_cap = 0;
    CHAP_HIP(hipMalloc(&S.trace_buf, sizeof(chap_trace_record) * (size_t)iters));
    S.trace_cap = iters;
    S.ctx.trace = S.trace_buf;
    dirty = true;
  }
  GatherRow* g = compact ? S.grow_buf : nullptr;
  if (g != S.ctx.grow) {
    S.ctx.grow = g;
    dirty = true;
  }
  if (dirty) CHAP_HIP(hipMemcpy((void*)S.L.walks, &S.ctx, sizeof(WalkCtx), hipMemcpyHostToDevice));
  S.L.compact = compact;
  std::vector<hipGraphExec_t> launches;
  {
    const int64_t G = std::max<int32_t>(1, p->opt.graph_iters);
    for (int64_t left = iters; left > 0;) {
      int64_t K = G;
      if (left < G) {
        K = 1;
        while (2 * K <= left) K *= 2;
      }
      hipGraphExec_t x;
      const int rc = slot_graph(S, K, compact, &x);
      if (rc != CHAP_OK) return rc;
      launches.push_back(x);
      left -= K;
    }
  }
  CHAP_HIP(hipEventRecord(S.ev[0], user));
  CHAP_HIP(hipStreamWaitEvent(S.s, S.ev[0], 0));
  int rc = init_walk(spec, iters, tenure, S.ctx, S.partial, S.ticket, S.s);
  if (rc != CHAP_OK) return rc;
  if (S.aff_L) {
    // stamps of earlier runs on this slot could equal this run's iteration tags
    if (p->n > 0) {
      hipLaunchKernelGGL(k_fill_i32, dim3((p->n + 255) / 256), dim3(256), 0, S.s, S.aff.stamp, 0, (int64_t)p->n);
      CHAP_HIP(hipGetLastError());
    }
  }
  std::unique_ptr<chap_run> R(new chap_run());
  R->trace.resize((size_t)iters);
  WalkState st;
  CHAP_HIP(hipEventRecord(S.ev[1], S.s));
  for (hipGraphExec_t x : launches) CHAP_HIP(hipGraphLaunch(x, S.s));
  CHAP_HIP(hipEventRecord(S.ev[2], S.s));
  // an incumbent found by the last iteration is copied here
  CHAP_HIP(launch_copy_best_batch(S.L, S.s));
  if (iters > 0)
    CHAP_HIP(hipMemcpyAsync(R->trace.data(), S.trace_buf, sizeof(chap_trace_record) * (size_t)iters,
                            hipMemcpyDeviceToHost, S.s));
  CHAP_HIP(hipMemcpyAsync(&st, S.ctx.st, sizeof(WalkState), hipMemcpyDeviceToHost, S.s));
  CHAP_HIP(hipStreamSynchronize(S.s));
  float ms = 0.0f;
  CHAP_HIP(hipEventElapsedTime(&ms, S.ev[1], S.ev[2]));
  R->elapsed_ms = ms;
  fill_summary(st, R.get());
  R->state_ready = false;
  R->pool = p->pool;
  R->slot = std::move(slot);
  out = std::move(R);
  return CHAP_OK;
}

}  // namespace

extern "C" {

int chap_tabu_run(chap_problem* p, int64_t iters, int32_t tenure, uint64_t seed, const double* x0, chap_run** out,
                  void* hip_stream) {
  if (!p || !out) return fail(CHAP_EINVAL, "chap_tabu_run: null argument");
  std::unique_ptr<chap_run> run;
  const int rc = run_single(p, seed, x0, iters, tenure, (hipStream_t)hip_stream, run);
  if (rc != CHAP_OK) return rc;
  *out = run.release();
  return CHAP_OK;
}

int chap_batch_run(chap_problem* const* probs, int32_t nprob, const int32_t* walk_prob, const uint64_t* walk_seed,
                   const double* const* walk_x0, int32_t nwalks, int64_t iters, int32_t tenure, chap_run** out,
                   void* hip_stream) {
  if (!probs || !walk_prob || !walk_seed || !out || nprob <= 0 || nwalks <= 0)
    return fail(CHAP_EINVAL, "chap_batch_run: null argument or empty batch");
  std::vector<WalkSpec> specs;
  for (int32_t w = 0; w < nwalks; ++w) {
    if (walk_prob[w] < 0 || walk_prob[w] >= nprob || !probs[walk_prob[w]])
      return fail(CHAP_EINVAL, "chap_batch_run: walk " + std::to_string(w) + " names no problem");
    specs.push_back(WalkSpec{probs[walk_prob[w]], walk_seed[w], walk_x0 ? walk_x0[w] : nullptr});
  }
  const int dev = specs[0].p->device;
  for (const WalkSpec& ws : specs)
    if (ws.p->device != dev) return fail(CHAP_EINVAL, "chap_batch_run: problems on different devices");
  std::vector<std::unique_ptr<chap_run>> runs;
  const int rc = run_walks(specs, iters, tenure, (hipStream_t)hip_stream, runs);
  if (rc != CHAP_OK) return rc;
  for (int32_t w = 0; w < nwalks; ++w) out[w] = runs[w].release();
  return CHAP_OK;
}

int chap_batch_restarts(chap_problem* const* probs, int32_t nprob, const int32_t* walk_prob, const uint64_t* walk_seed,
                        int32_t nwalks, int64_t iters, int32_t tenure, int64_t restart_every, int64_t min_distance,
                        chap_run** out, void* hip_stream) {
  if (!probs || !walk_prob || !walk_seed || !out || nprob <= 0 || nwalks <= 0)
    return fail(CHAP_EINVAL, "chap_batch_restarts: null argument or empty batch");
  if (restart_every <= 0 || min_distance < 0)
    return fail(CHAP_EINVAL, "chap_batch_restarts: restart_every must be > 0 and min_distance >= 0");
  std::vector<WalkSpec> specs;
  for (int32_t w = 0; w < nwalks; ++w) {
    if (walk_prob[w] < 0 || walk_prob[w] >= nprob || !probs[walk_prob[w]])
      return fail(CHAP_EINVAL, "chap_batch_restarts: walk " + std::to_string(w) + " names no problem");
    specs.push_back(WalkSpec{probs[walk_prob[w]], walk_seed[w], nullptr});
  }
  const int dev = specs[0].p->device;
  for (const WalkSpec& ws : specs)
    if (ws.p->device != dev) return fail(CHAP_EINVAL, "chap_batch_restarts: problems on different devices");
  RestartSpec rs;
  rs.every = restart_every;
  rs.min_distance = min_distance;
  std::vector<std::unique_ptr<chap_run>> runs;
  const int rc = run_walks(specs, iters, tenure, (hipStream_t)hip_stream, runs, &rs);
  if (rc != CHAP_OK) return rc;
  for (int32_t w = 0; w < nwalks; ++w) out[w] = runs[w].release();
  return CHAP_OK;
}

int chap_run_restarts(const chap_run* r, const int64_t** iters, int64_t* count) {
  if (!r || !iters || !count) return fail(CHAP_EINVAL, "chap_run_restarts: null argument");
  *iters = r->restarts.data();
  *count = (int64_t)r->restarts.size();
  return CHAP_OK;
}

int chap_autotune(const chap_problem* p, const chap_options* cands, int32_t ncand, int64_t walk_iters,
                  chap_options* best, double* ms_per_iter) {
  if (!p || !best || ncand < 0 || (ncand > 0 && !cands) || walk_iters <= 0 || walk_iters > (1 << 20))
    return fail(CHAP_EINVAL, "chap_autotune: bad argument");
  std::vector<chap_options> grid;
  if (ncand > 0) {
    grid.assign(cands, cands + ncand);
  } else {
    for (int32_t sm : {4, 8})
      for (int32_t cl : {2048, 4096})
        for (int32_t gi : {32, 64}) {
          chap_options o = p->opt;
          o.short_max = sm;
          o.chunk_min = cl;
          o.chunk_len = cl;
          o.graph_iters = gi;
          grid.push_back(o);
        }
  }
  const chap_problem::Raw& R = p->raw;
  double best_ms = HUGE_VAL;
  int32_t best_i = -1;
  for (size_t c = 0; c < grid.size(); ++c) {
    chap_options o = grid[c];
    o.feas_tol = p->opt.feas_tol;  // the tolerance is part of the problem, not a tuning knob
    chap_problem* t = nullptr;
    int rc = chap_problem_create(&t, p->n, p->m, R.csr_row_ptr.data(), R.csr_col.data(), R.csr_val.data(),
                                 R.csc_col_ptr.data(), R.csc_row.data(), R.csc_val.data(), R.sense.data(),
                                 R.rhs.data(), R.lb.data(), R.ub.data(), R.is_int.data(), R.obj.data(), &o);
    if (rc != CHAP_OK) return rc;
    std::unique_ptr<chap_problem> guard(t);
    std::vector<std::unique_ptr<chap_run>> runs;
    rc = run_walks({WalkSpec{t, 0, nullptr}}, std::min<int64_t>(walk_iters, 8), 10, nullptr, runs);  // warm-up
    if (rc == CHAP_OK) rc = run_walks({WalkSpec{t, 0, nullptr}}, walk_iters, 10, nullptr, runs);
    if (rc != CHAP_OK) return rc;
    const double ms = runs[0]->elapsed_ms / (double)walk_iters;
    if (ms_per_iter) ms_per_iter[c] = ms;
    if (ms < best_ms) {
      best_ms = ms;
      best_i = (int32_t)c;
    }
  }
  *best = grid[best_i];
  best->feas_tol = p->opt.feas_tol;
  return CHAP_OK;
}

int chap_run_trace(const chap_run* r, const chap_trace_record** records, int64_t* count) {
  if (!r || !records || !count) return fail(CHAP_EINVAL, "chap_run_trace: null argument");
  *records = r->trace.data();
  *count = (int64_t)r->trace.size();
  return CHAP_OK;
}

int chap_run_state(const chap_run* r, double* x, double* resid, float* w, double* best_obj, double* best_x,
                   double* cutoff_rhs) {
  if (!r) return fail(CHAP_EINVAL, "chap_run_state: null run");
  if (x || resid || w || best_x) {
    const int rc = materialize(r);
    if (rc != CHAP_OK) return rc;
  }
  if (x) std::copy(r->x.begin(), r->x.end(), x);
  if (resid) std::copy(r->resid.begin(), r->resid.end(), resid);
  if (w) std::copy(r->w.begin(), r->w.end(), w);
  if (best_obj) *best_obj = r->best_obj;
  if (best_x && r->has_best) std::copy(r->best_x.begin(), r->best_x.end(), best_x);
  if (cutoff_rhs) *cutoff_rhs = r->cutoff_rhs;
  return CHAP_OK;
}

int chap_run_best_infeasible(const chap_run* r, double* x, int64_t* violated, int64_t* iter) {
  if (!r) return fail(CHAP_EINVAL, "chap_run_best_infeasible: null run");
  if (!r->restarts.empty())
    return fail(CHAP_EINVAL, "chap_run_best_infeasible: not recorded for a walk that restarted");
  if (x && r->inf_iter != -2) {
    const int rc = materialize(r);
    if (rc != CHAP_OK) return rc;
    std::copy(r->inf_x.begin(), r->inf_x.end(), x);
  }
  if (violated) *violated = r->inf_viol;
  if (iter) *iter = r->inf_iter;
  return CHAP_OK;
}

double chap_run_elapsed_ms(const chap_run* r) { return r ? r->elapsed_ms : 0.0; }

void chap_run_destroy(chap_run* r) { delete r; }

}  // extern "C"
