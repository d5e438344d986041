// CPU oracle for the GPU tabu-search best-shift path.
//
// TEST INFRASTRUCTURE ONLY. Nothing in the product library links, loads or
// calls this file; only the tests, the smoke check and the benchmark's CPU
// baseline use it. It shares no code, header or constant table with the HIP
// library. It is deliberately plain and slow: every quantity is recomputed
// from its definition, in FP64, in the order the paper states it.
//
// What it follows (CHAP, section 3.1 "GPU Tabu Search"):
//   * problem form min c^T x, Ax <= b, l <= x <= u, x_I integer (3.1, problem
//     statement); every row normalised to '<=' (3.1 "Memory Considerations",
//     second remark): 'G' rows negated, 'E' rows as a (row, negated row) pair;
//   * residual r_i = sum_k a_ik x_k - b_i (3.1 "Memory Considerations", first
//     remark), recomputed from scratch in CSR order every iteration;
//   * penalty p_ij and score s_j (3.1 "Scoring Functions");
//   * best shift (Eq. 1), flip for binaries, Algorithm 1 (sort, scan, argmax)
//     for every other variable, with integer breakpoints rounded down for
//     a_ij > 0 and up for a_ij < 0;
//   * objective cutoff row from the best objective found (3.2);
//   * tabu list, aspiration and weight update follow the readings listed in
//     the design notes (the paper defers them to LocalMIP): variable-level
//     tabu for `tenure` iterations, aspiration only for the overall best
//     improving variable when its move makes the point feasible, and +1 on
//     every violated row when no admissible improving move exists.
// Feasibility tolerance eps: a normalised row is violated iff r_i > eps, and
// the breakpoint of row i on variable j is tau = xbar_j + (eps - r_i)/a_ij.
//
// Build: g++ -O2 -std=c++17 -ffp-contract=off -fopenmp -fPIC -shared (no
// fast-math). Threads (orc_set_threads, default 1) only split the
// independent per-column best shifts and per-row residuals of a full
// evaluation across cores; every value is computed exactly as with one.

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <limits>
#include <vector>

#include <omp.h>

namespace {

const double kInf = std::numeric_limits<double>::infinity();

struct OracleProblem {
  int32_t n = 0;
  int32_t m = 0;   // original rows
  int32_t mp = 0;  // normalised rows (the cutoff row has index mp)
  double eps = 1e-6;
  // normalised rows, CSR
  std::vector<int64_t> rptr;
  std::vector<int32_t> rcol;
  std::vector<double> rval;
  std::vector<double> rb;
  std::vector<int32_t> orig_row;
  std::vector<int8_t> sign;
  // normalised rows, column view (row indices ascending within a column)
  std::vector<int64_t> cptr;
  std::vector<int32_t> crow;
  std::vector<double> cval;
  // variables
  std::vector<double> lb, ub, obj;
  std::vector<uint8_t> is_int, is_bin;
  bool obj_integral = true;
};

// One normalised row restricted to one column: coefficient and row index.
struct ColEntry {
  int32_t row;
  double a;
};

// Algorithm 1 triplet (position, marker, score change).
struct Triplet {
  double pos;
  int marker;
  double delta;
};

bool triplet_less(const Triplet& p, const Triplet& q) {
  if (p.pos != q.pos) return p.pos < q.pos;
  if (p.marker != q.marker) return p.marker < q.marker;
  return p.delta < q.delta;
}

// Penalty of one row for a move taking its residual from r to r2
// (3.1 "Scoring Functions"; "y > b" read as residual > eps).
double penalty(double r, double r2, double w, double eps) {
  bool viol = r > eps;
  bool viol2 = r2 > eps;
  if (!viol && viol2) return -w;
  if (viol && !viol2) return w;
  if (viol && viol2 && r2 < r) return 0.5 * w;
  if (viol && viol2 && r2 > r) return -0.5 * w;
  return 0.0;
}

// Column j's rows in the normalised system, plus the cutoff row when active.
std::vector<ColEntry> column_rows(const OracleProblem& P, int32_t j, bool cutoff_active) {
  std::vector<ColEntry> out;
  for (int64_t k = P.cptr[j]; k < P.cptr[j + 1]; ++k) out.push_back({P.crow[k], P.cval[k]});
  if (cutoff_active && P.obj[j] != 0.0) out.push_back({P.mp, P.obj[j]});
  return out;
}

// Flip score of a binary variable: the only move is xbar -> 1 - xbar (3.1
// "Best Shift Moves").
void flip_score(const OracleProblem& P, int32_t j, double xbar, const std::vector<double>& r,
                const float* w, bool cutoff_active, double* xhat, double* s) {
  double xnew = 1.0 - xbar;
  double delta = xnew - xbar;
  double total = 0.0;
  for (const ColEntry& e : column_rows(P, j, cutoff_active)) {
    double r2 = r[e.row] + e.a * delta;
    total += penalty(r[e.row], r2, (double)w[e.row], P.eps);
  }
  if (total > 0.0) {
    *xhat = xnew;
    *s = total;
  } else {
    *xhat = xbar;
    *s = 0.0;
  }
}

// Algorithm 1, "Best Shift via Sort-Scan-Argmax", for one non-binary column.
void alg1_best_shift(const OracleProblem& P, int32_t j, double xbar, const std::vector<double>& r,
                     const float* w, bool cutoff_active, double* xhat, double* s) {
  const double l = P.lb[j], u = P.ub[j];
  // phase 1: breakpoints and the two accumulators
  double beta = 0.0, alpha = 0.0;
  std::vector<Triplet> B;
  if (std::isfinite(l)) B.push_back({l, -1, 0.0});
  if (std::isfinite(u)) B.push_back({u, -1, 0.0});
  for (const ColEntry& e : column_rows(P, j, cutoff_active)) {
    double a = e.a;
    double wi = (double)w[e.row];
    double t = xbar + (P.eps - r[e.row]) / a;
    if (P.is_int[j]) t = (a > 0.0) ? std::floor(t) : std::ceil(t);
    if (a < 0.0) {  // the row asks for x_j >= t
      if (xbar < t) {
        beta -= 0.5 * wi;
        alpha += wi;
        B.push_back({t, -1, 0.5 * wi});
      } else if (xbar > t) {
        beta -= wi;
        B.push_back({t, -1, wi});
      } else {
        beta -= wi;
        alpha += wi;
      }
    } else {  // the row asks for x_j <= t
      if (xbar > t) {
        beta += wi;
        alpha -= wi;
        B.push_back({t, -1, 0.0});
        B.push_back({t, +1, -0.5 * wi});
      } else if (xbar < t) {
        B.push_back({t, -1, 0.0});
        B.push_back({t, +1, -wi});
      } else {
        alpha -= wi;
      }
    }
  }
  // phase 2: lexicographic sort
  std::sort(B.begin(), B.end(), triplet_less);
  // phase 3: inclusive scan, sigma = beta + P + alpha [pos > xbar]
  // phase 4: argmax over entries inside the bounds, excluding the incumbent
  double prefix = 0.0;
  bool found = false;
  double best = 0.0, best_pos = xbar;
  for (const Triplet& t : B) {
    prefix += t.delta;
    double sigma = beta + prefix + ((t.pos > xbar) ? alpha : 0.0);
    bool inside = std::isfinite(t.pos) && t.pos >= l && t.pos <= u && t.pos != xbar;
    if (!inside) continue;
    if (!found || sigma > best) {
      found = true;
      best = sigma;
      best_pos = t.pos;
    }
  }
  if (found && best > 0.0) {
    *xhat = best_pos;
    *s = best;
  } else {
    *xhat = xbar;
    *s = 0.0;
  }
}

void best_shift_one(const OracleProblem& P, int32_t j, const double* x, const std::vector<double>& r,
                    const float* w, bool cutoff_active, double* xhat, double* s) {
  if (P.is_bin[j])
    flip_score(P, j, x[j], r, w, cutoff_active, xhat, s);
  else
    alg1_best_shift(P, j, x[j], r, w, cutoff_active, xhat, s);
}

// ---- jump values (weighted violation, after Feasibility Jump) ------------
// Section 3.1 "Best Shift Moves" recalls the jump value of Feasibility Jump
// (its line sweep motivates Algorithm 1): the value of x_j that minimises the
// weighted violation of x_j's constraints with the other variables held.
// Readings (design notes): the violation of normalised row i at x_j = t is
// max(0, r_i + a_ij (t - xbar_j)), its amount beyond the right-hand side,
// weighted by w_i, and the cutoff row takes part when active, as in the
// score; the jump leaves xbar_j (t != xbar_j); ties go to the value closest
// to xbar_j, then to the smaller one; the jump score is V(xbar_j) - V(t*).

// V_j(t): the weighted violation of j's normalised rows (ascending) and then
// the cutoff row, with x_j = t and every other variable at the point.
double weighted_violation(const OracleProblem& P, int32_t j, double xbar, const std::vector<double>& r,
                          const float* w, bool cutoff_active, double t) {
  const double d = t - xbar;
  double v = 0.0;
  for (const ColEntry& e : column_rows(P, j, cutoff_active)) {
    const double y = r[e.row] + e.a * d;
    v += (double)w[e.row] * (y > 0.0 ? y : 0.0);
  }
  return v;
}

// The jump value of column j and its score. An integer variable with at most
// 64 values is tried at every value of its domain. Otherwise V_j is convex
// and piecewise linear with kinks where a row's violation reaches zero,
// t = xbar - r_i / a_ij, so its minimum over the domain lies at a kink (an
// integer variable: the integers on either side of one), a finite bound, or,
// for an integer variable whose minimum is at xbar itself, xbar - 1 or
// xbar + 1; those are the values tried. No value to try: (xbar, 0).
void jump_value_one(const OracleProblem& P, int32_t j, const double* x, const std::vector<double>& r,
                    const float* w, bool cutoff_active, double* jv, double* js) {
  const double xbar = x[j];
  const double l = P.lb[j], u = P.ub[j];
  const bool integer = P.is_int[j] != 0;
  std::vector<double> cand;
  if (integer && std::isfinite(l) && std::isfinite(u) && u - l + 1.0 <= 64.0) {
    for (double t = l; t <= u; t += 1.0) cand.push_back(t);
  } else {
    for (const ColEntry& e : column_rows(P, j, cutoff_active)) {
      const double kink = xbar - r[e.row] / e.a;
      if (integer) {
        cand.push_back(std::floor(kink));
        cand.push_back(std::ceil(kink));
      } else {
        cand.push_back(kink);
      }
    }
    cand.push_back(l);
    cand.push_back(u);
    if (integer) {
      cand.push_back(xbar - 1.0);
      cand.push_back(xbar + 1.0);
    }
  }
  bool found = false;
  double bt = xbar, bv = 0.0;
  for (double t : cand) {
    if (!std::isfinite(t) || t < l || t > u || t == xbar) continue;
    const double v = weighted_violation(P, j, xbar, r, w, cutoff_active, t);
    const bool better = !found || v < bv ||
                        (v == bv && (std::fabs(t - xbar) < std::fabs(bt - xbar) ||
                                     (std::fabs(t - xbar) == std::fabs(bt - xbar) && t < bt)));
    if (better) {
      found = true;
      bt = t;
      bv = v;
    }
  }
  if (!found) {
    *jv = xbar;
    *js = 0.0;
    return;
  }
  *jv = bt;
  *js = weighted_violation(P, j, xbar, r, w, cutoff_active, xbar) - bv;
}

// r = A'x - b' over the normalised rows, in CSR order; cutoff row c^T x - bc.
// Exactly rounded sum of a list of doubles. Each term is merged into a list
// of nonoverlapping partials with error-free additions (Shewchuk, "Adaptive
// Precision Floating-Point Arithmetic and Fast Robust Geometric Predicates",
// 1997); the partials are then added from the largest down until an addition
// is inexact, and a tie at half an ulp is settled by the sign of the next
// partial (the method of Python's math.fsum). The result is the exact sum
// rounded once to nearest, ties to even; an exact zero gives +0.
double exact_sum(const std::vector<double>& terms) {
  std::vector<double> part;  // nonoverlapping, increasing magnitude
  for (double v : terms) {
    double x = v;
    size_t keep = 0;
    for (size_t q = 0; q < part.size(); ++q) {
      double y = part[q];
      if (std::fabs(x) < std::fabs(y)) std::swap(x, y);
      const double hi = x + y;
      const double lo = y - (hi - x);
      if (lo != 0.0) part[keep++] = lo;
      x = hi;
    }
    part.resize(keep);
    part.push_back(x);
  }
  if (part.empty()) return 0.0;
  size_t k = part.size() - 1;
  double hi = part[k];
  double lo = 0.0;
  while (k > 0) {
    const double x = hi;
    const double y = part[--k];
    hi = x + y;
    lo = y - (hi - x);
    if (lo != 0.0) break;
  }
  if (k > 0 && ((lo < 0.0 && part[k - 1] < 0.0) || (lo > 0.0 && part[k - 1] > 0.0))) {
    const double y = lo * 2.0;
    const double x = hi + y;
    if (y == x - hi) hi = x;
  }
  return hi == 0.0 ? 0.0 : hi;
}

// The terms of c^T x: for every nonzero c_j the product c_j x_j as the pair
// (p, e) with p the rounded product and e = fma(c_j, x_j, -p) its rounding
// error, so that p + e equals c_j x_j exactly (unless the product underflows).
std::vector<double> objective_terms(const OracleProblem& P, const double* x) {
  std::vector<double> t;
  for (int32_t j = 0; j < P.n; ++j) {
    if (P.obj[j] == 0.0) continue;
    const double p = P.obj[j] * x[j];
    t.push_back(p);
    t.push_back(std::fma(P.obj[j], x[j], -p));
  }
  return t;
}

// The objective row is one sum over every variable; its FP64 value depends
// on the summation order unless it is rounded once. Reading: the objective
// f = c^T x and the cutoff residual c^T x - b_c are the exact values rounded
// once to nearest (section 3.2 does not fix an order).
void residual_from_scratch(const OracleProblem& P, const double* x, bool cutoff_active, double bc,
                           std::vector<double>& r) {
  r.assign((size_t)P.mp + 1, 0.0);
#pragma omp parallel for schedule(static)
  for (int32_t i = 0; i < P.mp; ++i) {
    double acc = 0.0;
    for (int64_t k = P.rptr[i]; k < P.rptr[i + 1]; ++k) {
      double prod = P.rval[k] * x[P.rcol[k]];
      acc = acc + prod;
    }
    r[i] = acc - P.rb[i];
  }
  if (cutoff_active) {
    std::vector<double> t = objective_terms(P, x);
    t.push_back(-bc);
    r[P.mp] = exact_sum(t);
  }
}

int64_t count_violated(const OracleProblem& P, const std::vector<double>& r, bool cutoff_active) {
  int64_t v = 0;
  for (int32_t i = 0; i < P.mp; ++i) v += (r[i] > P.eps) ? 1 : 0;
  if (cutoff_active && r[P.mp] > P.eps) v += 1;
  return v;
}

double objective(const OracleProblem& P, const double* x) { return exact_sum(objective_terms(P, x)); }

uint64_t splitmix64_output(uint64_t seed, uint64_t index) {
  // The (index+1)-th output of SplitMix64 (Steele, Lea & Flood 2014) started
  // from state `seed`.
  uint64_t z = seed + (index + 1) * 0x9E3779B97F4A7C15ULL;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}

double clamp0(double l, double u) {
  double v = 0.0;
  if (v < l) v = l;
  if (v > u) v = u;
  return v;
}

void start_point(const OracleProblem& P, uint64_t seed, double* x) {
  for (int32_t j = 0; j < P.n; ++j) {
    double l = P.lb[j], u = P.ub[j];
    if (seed != 0 && P.is_int[j] && std::isfinite(l) && std::isfinite(u)) {
      uint64_t h = splitmix64_output(seed, (uint64_t)j);
      uint64_t width = (uint64_t)(u - l) + 1;
      x[j] = l + (double)(h % width);
    } else {
      x[j] = clamp0(l, u);
    }
  }
}

struct TraceRec {
  int64_t iter;
  int32_t var;   // -1 for a reweight step
  int32_t kind;  // 0 move, 1 move by aspiration, 2 reweight
  double x_old;
  double x_new;
  double score;
  int64_t viol;  // violated normalised rows after the step
  double obj;    // c^T x after the step
};

}  // namespace

extern "C" {

void* orc_create(int32_t n, int32_t m, const int64_t* csr_row_ptr, const int32_t* csr_col,
                 const double* csr_val, const uint8_t* sense, const double* rhs, const double* lb,
                 const double* ub, const uint8_t* is_int, const double* obj, double eps,
                 int32_t binary_as_general) {
  // binary_as_general = 1 sends [0,1] integer variables through Algorithm 1
  // instead of the flip score (used to check that both give the same move).
  OracleProblem* P = new OracleProblem();
  P->n = n;
  P->m = m;
  P->eps = eps;
  P->rptr.push_back(0);
  auto push_row = [&](int32_t i, double sgn) {
    for (int64_t k = csr_row_ptr[i]; k < csr_row_ptr[i + 1]; ++k) {
      if (csr_val[k] == 0.0) continue;  // stored zeros are dropped
      P->rcol.push_back(csr_col[k]);
      P->rval.push_back(sgn * csr_val[k]);
    }
    P->rptr.push_back((int64_t)P->rcol.size());
    P->rb.push_back(sgn * rhs[i]);
    P->orig_row.push_back(i);
    P->sign.push_back((int8_t)sgn);
  };
  for (int32_t i = 0; i < m; ++i) {
    char s = (char)sense[i];
    if (s == 'L') {
      push_row(i, 1.0);
    } else if (s == 'G') {
      push_row(i, -1.0);
    } else {
      push_row(i, 1.0);
      push_row(i, -1.0);
    }
  }
  P->mp = (int32_t)P->rb.size();
  // column view by counting sort of the normalised rows
  P->cptr.assign((size_t)n + 1, 0);
  for (int32_t c : P->rcol) P->cptr[c + 1] += 1;
  for (int32_t j = 0; j < n; ++j) P->cptr[j + 1] += P->cptr[j];
  P->crow.resize(P->rcol.size());
  P->cval.resize(P->rcol.size());
  std::vector<int64_t> fill(P->cptr.begin(), P->cptr.end() - 1);
  for (int32_t i = 0; i < P->mp; ++i) {
    for (int64_t k = P->rptr[i]; k < P->rptr[i + 1]; ++k) {
      int32_t c = P->rcol[k];
      P->crow[fill[c]] = i;
      P->cval[fill[c]] = P->rval[k];
      fill[c] += 1;
    }
  }
  P->lb.resize(n);
  P->ub.resize(n);
  P->obj.assign(obj, obj + n);
  P->is_int.assign(is_int, is_int + n);
  P->is_bin.resize(n);
  for (int32_t j = 0; j < n; ++j) {
    double l = lb[j], u = ub[j];
    if (is_int[j]) {
      l = std::ceil(l);
      u = std::floor(u);
    }
    P->lb[j] = l;
    P->ub[j] = u;
    P->is_bin[j] = (!binary_as_general && is_int[j] && l == 0.0 && u == 1.0) ? 1 : 0;
    if (obj[j] != 0.0 && (!is_int[j] || std::floor(obj[j]) != obj[j])) P->obj_integral = false;
  }
  return P;
}

void orc_destroy(void* h) { delete (OracleProblem*)h; }

int32_t orc_num_norm_rows(void* h) { return ((OracleProblem*)h)->mp; }

void orc_norm_rows(void* h, int32_t* orig_row, int8_t* sign) {
  OracleProblem* P = (OracleProblem*)h;
  for (int32_t i = 0; i < P->mp; ++i) {
    orig_row[i] = P->orig_row[i];
    sign[i] = P->sign[i];
  }
}

void orc_bounds(void* h, double* lb, double* ub, uint8_t* is_bin) {
  OracleProblem* P = (OracleProblem*)h;
  for (int32_t j = 0; j < P->n; ++j) {
    lb[j] = P->lb[j];
    ub[j] = P->ub[j];
    is_bin[j] = P->is_bin[j];
  }
}

// r (mp+1 entries; the last is the cutoff row, 0 when cutoff_rhs is +inf).
int64_t orc_residual(void* h, const double* x, double cutoff_rhs, double* r_out) {
  OracleProblem* P = (OracleProblem*)h;
  bool active = !std::isinf(cutoff_rhs);
  std::vector<double> r;
  residual_from_scratch(*P, x, active, cutoff_rhs, r);
  std::memcpy(r_out, r.data(), sizeof(double) * (size_t)(P->mp + 1));
  return count_violated(*P, r, active);
}

// Best shift of the listed columns (all columns when cols is null) at point x
// with weights w (mp+1 entries), cutoff row active iff cutoff_rhs is finite.
void orc_best_shift(void* h, const double* x, const float* w, double cutoff_rhs, const int32_t* cols,
                    int64_t ncols, double* xhat, double* s) {
  OracleProblem* P = (OracleProblem*)h;
  bool active = !std::isinf(cutoff_rhs);
  std::vector<double> r;
  residual_from_scratch(*P, x, active, cutoff_rhs, r);
  if (cols == nullptr) {
#pragma omp parallel for schedule(dynamic, 1024)
    for (int32_t j = 0; j < P->n; ++j) best_shift_one(*P, j, x, r, w, active, &xhat[j], &s[j]);
  } else {
#pragma omp parallel for schedule(dynamic, 1024)
    for (int64_t q = 0; q < ncols; ++q)
      best_shift_one(*P, cols[q], x, r, w, active, &xhat[q], &s[q]);
  }
}

// Jump value and jump score of every column at point x with weights w
// (mp+1 entries), cutoff row active iff cutoff_rhs is finite.
void orc_jump_values(void* h, const double* x, const float* w, double cutoff_rhs, double* jv, double* js) {
  OracleProblem* P = (OracleProblem*)h;
  bool active = !std::isinf(cutoff_rhs);
  std::vector<double> r;
  residual_from_scratch(*P, x, active, cutoff_rhs, r);
#pragma omp parallel for schedule(dynamic, 1024)
  for (int32_t j = 0; j < P->n; ++j) jump_value_one(*P, j, x, r, w, active, &jv[j], &js[j]);
}

// V_j(t) at point x (the weighted violation the jump value minimises).
double orc_weighted_violation(void* h, const double* x, const float* w, double cutoff_rhs, int32_t j, double t) {
  OracleProblem* P = (OracleProblem*)h;
  bool active = !std::isinf(cutoff_rhs);
  std::vector<double> r;
  residual_from_scratch(*P, x, active, cutoff_rhs, r);
  return weighted_violation(*P, j, x[j], r, w, active, t);
}

// Threads of the per-column and per-row loops (1 = sequential).
void orc_set_threads(int32_t k) { omp_set_num_threads(k > 0 ? k : 1); }
int32_t orc_threads(void) { return (int32_t)omp_get_max_threads(); }

// Exactly rounded sum of n doubles (the summation used for the objective).
double orc_exact_sum(const double* v, int64_t n) { return exact_sum(std::vector<double>(v, v + n)); }

// c^T x rounded once.
double orc_objective(void* h, const double* x) { return objective(*(OracleProblem*)h, x); }

void orc_start_point(void* h, uint64_t seed, double* x) { start_point(*(OracleProblem*)h, seed, x); }

uint64_t orc_splitmix64(uint64_t seed, uint64_t index) { return splitmix64_output(seed, index); }

// One tabu walk. With full_every = 1 every iteration evaluates every column
// (the method of section 3.1). With full_every > 1 the walk is the learned
// proposal form: an iteration is a full evaluation when it is the first,
// follows a stall, or comes full_every iterations after the last full
// evaluation; any other iteration evaluates only the columns listed for it in
// sets[set_off[k] .. set_off[k+1]) (original indices) and chooses among them
// with the same rules; without an admissible move there it is a stall (kind
// 3: no move, no reweight). Moves chosen from a list get kind + 8.
// The state of a walk at the start of iteration k0, to continue it from
// there: weights (mp+1), the last tabu iteration of every variable, the best
// feasible point and objective, the cutoff right-hand side (+inf: inactive).
struct WalkResume {
  const float* w;
  const int64_t* tabu_until;
  int64_t k0;
  int32_t has_best;
  double fbest;
  const double* best_x;
  double cutoff_rhs;
};

// The best infeasible point of a walk (reading of the pool's partial
// solutions, section 3.2): among the points the walk visits (its start and
// the point after each iteration) that violate at least one normalised row
// of the problem (the cutoff row not counted), the first with the fewest
// such rows. iter = -1 for the start point, -2 when every point was
// feasible.
struct WalkInfeasible {
  int64_t* viol;
  int64_t* iter;
  double* x;
};

int64_t learned_walk(OracleProblem& P, int64_t iters, int32_t tenure, uint64_t seed, const double* x0,
                     int32_t full_every, const int32_t* sets, const int64_t* set_off, void* trace_out,
                     double* x_out, double* r_out, float* w_out, double* best_obj, double* best_x, int32_t* has_best,
                     double* cutoff_rhs_out, const WalkResume* resume = nullptr,
                     const WalkInfeasible* inf_out = nullptr) {
  const int32_t n = P.n;
  std::vector<double> x(n);
  if (x0)
    std::memcpy(x.data(), x0, sizeof(double) * (size_t)n);
  else
    start_point(P, seed, x.data());
  std::vector<float> w((size_t)P.mp + 1, 1.0f);
  std::vector<int64_t> tabu_until(n, -1);
  std::vector<double> xbest(n, 0.0);
  double fbest = kInf;
  bool found = false;
  bool cutoff = false;
  double bc = 0.0;
  int64_t k0 = 0;
  if (resume) {
    w.assign(resume->w, resume->w + P.mp + 1);
    tabu_until.assign(resume->tabu_until, resume->tabu_until + n);
    k0 = resume->k0;
    found = resume->has_best != 0;
    if (found) {
      fbest = resume->fbest;
      xbest.assign(resume->best_x, resume->best_x + n);
    }
    cutoff = !std::isinf(resume->cutoff_rhs);
    bc = cutoff ? resume->cutoff_rhs : 0.0;
  }
  std::vector<double> r;
  std::vector<double> xhat(n), s(n);
  std::vector<int32_t> cands;
  TraceRec* trace = (TraceRec*)trace_out;

  residual_from_scratch(P, x.data(), cutoff, bc, r);
  int64_t V = count_violated(P, r, cutoff);
  int64_t inf_v = std::numeric_limits<int64_t>::max(), inf_k = -2;
  std::vector<double> inf_x(n, 0.0);
  auto track_infeasible = [&](int64_t k) {
    const int64_t v = count_violated(P, r, false);
    if (v > 0 && v < inf_v) {
      inf_v = v;
      inf_k = k;
      inf_x = x;
    }
  };
  track_infeasible(k0 - 1);

  auto incumbent_check = [&]() {
    if (V != 0) return;
    double f = objective(P, x.data());
    if (f < fbest) {
      fbest = f;
      xbest = x;
      found = true;
    }
    double delta = P.obj_integral ? 1.0 : 1e-4 * std::max(1.0, std::fabs(fbest));
    bc = fbest - delta;
    cutoff = true;
    residual_from_scratch(P, x.data(), cutoff, bc, r);
    V = count_violated(P, r, cutoff);
  };
  incumbent_check();

  int64_t k_last_full = k0;
  bool stalled = false;
  for (int64_t k = k0; k < k0 + iters; ++k) {
    const bool full = full_every <= 1 || k == k0 || stalled || k - k_last_full >= full_every;
    if (full) k_last_full = k;
    residual_from_scratch(P, x.data(), cutoff, bc, r);
    V = count_violated(P, r, cutoff);
    cands.clear();
    if (full) {
      for (int32_t j = 0; j < n; ++j) cands.push_back(j);
    } else {
      for (int64_t t = set_off[k]; t < set_off[k + 1]; ++t) cands.push_back(sets[t]);
    }
    const int64_t nc = (int64_t)cands.size();
#pragma omp parallel for schedule(dynamic, 1024)
    for (int64_t t = 0; t < nc; ++t) {
      const int32_t j = cands[t];
      best_shift_one(P, j, x.data(), r, w.data(), cutoff, &xhat[j], &s[j]);
    }
    int32_t j_all = -1, j_nt = -1;
    for (int32_t j : cands) {
      if (!(s[j] > 0.0)) continue;
      if (j_all < 0 || s[j] > s[j_all] || (s[j] == s[j_all] && j < j_all)) j_all = j;
      if (k > tabu_until[j] && (j_nt < 0 || s[j] > s[j_nt] || (s[j] == s[j_nt] && j < j_nt))) j_nt = j;
    }
    int32_t jstar = -1;
    int32_t kind = full ? 2 : 3;
    if (j_all >= 0 && k > tabu_until[j_all]) {
      jstar = j_all;
      kind = 0;
    } else if (j_all >= 0) {
      double dx = xhat[j_all] - x[j_all];
      int64_t V2 = V;
      for (const ColEntry& e : column_rows(P, j_all, cutoff)) {
        bool viol = r[e.row] > P.eps;
        bool viol2 = (r[e.row] + e.a * dx) > P.eps;
        if (viol && !viol2) V2 -= 1;
        if (!viol && viol2) V2 += 1;
      }
      if (V2 == 0) {
        jstar = j_all;
        kind = 1;
      } else if (j_nt >= 0) {
        jstar = j_nt;
        kind = 0;
      }
    }
    if (jstar >= 0 && !full) kind += 8;
    stalled = (jstar < 0 && !full);
    TraceRec& t = trace[k - k0];
    t.iter = k;
    t.kind = kind;
    if (jstar < 0) {
      if (full) {
        for (int32_t i = 0; i < P.mp; ++i)
          if (r[i] > P.eps) w[i] += 1.0f;
        if (cutoff && r[P.mp] > P.eps) w[P.mp] += 1.0f;
      }
      t.var = -1;
      t.x_old = 0.0;
      t.x_new = 0.0;
      t.score = 0.0;
      t.viol = V;
      t.obj = objective(P, x.data());
    } else {
      t.var = jstar;
      t.x_old = x[jstar];
      t.x_new = xhat[jstar];
      t.score = s[jstar];
      x[jstar] = xhat[jstar];
      tabu_until[jstar] = k + tenure;
      residual_from_scratch(P, x.data(), cutoff, bc, r);
      V = count_violated(P, r, cutoff);
      t.viol = V;
      t.obj = objective(P, x.data());
      track_infeasible(k);
    }
    incumbent_check();
  }
  residual_from_scratch(P, x.data(), cutoff, bc, r);
  std::memcpy(x_out, x.data(), sizeof(double) * (size_t)n);
  std::memcpy(r_out, r.data(), sizeof(double) * (size_t)(P.mp + 1));
  std::memcpy(w_out, w.data(), sizeof(float) * (size_t)(P.mp + 1));
  *best_obj = fbest;
  std::memcpy(best_x, xbest.data(), sizeof(double) * (size_t)n);
  *has_best = found ? 1 : 0;
  *cutoff_rhs_out = cutoff ? bc : kInf;
  if (inf_out) {
    *inf_out->viol = inf_k == -2 ? 0 : inf_v;
    *inf_out->iter = inf_k;
    std::memcpy(inf_out->x, inf_x.data(), sizeof(double) * (size_t)n);
  }
  return iters;
}

// One tabu walk. trace must hold `iters` records. Returns the number of
// records written (== iters).
int64_t orc_tabu_run(void* h, int64_t iters, int32_t tenure, uint64_t seed, const double* x0,
                     void* trace_out, double* x_out, double* r_out, float* w_out, double* best_obj,
                     double* best_x, int32_t* has_best, double* cutoff_rhs_out, int64_t* inf_viol,
                     int64_t* inf_iter, double* inf_x) {
  const WalkInfeasible I{inf_viol, inf_iter, inf_x};
  return learned_walk(*(OracleProblem*)h, iters, tenure, seed, x0, 1, nullptr, nullptr, trace_out, x_out, r_out,
                      w_out, best_obj, best_x, has_best, cutoff_rhs_out, nullptr, &I);
}

// The plain walk continued for `iters` iterations from a given state at the
// start of iteration k0 (trace records k0 .. k0 + iters - 1).
int64_t orc_tabu_resume(void* h, int64_t iters, int32_t tenure, const double* x, const float* w,
                        const int64_t* tabu_until, int64_t k0, int32_t has_best_in, double fbest_in,
                        const double* best_x_in, double cutoff_rhs_in, void* trace_out, double* x_out, double* r_out,
                        float* w_out, double* best_obj, double* best_x, int32_t* has_best, double* cutoff_rhs_out,
                        int64_t* inf_viol, int64_t* inf_iter, double* inf_x) {
  const WalkResume R{w, tabu_until, k0, has_best_in, fbest_in, best_x_in, cutoff_rhs_in};
  const WalkInfeasible I{inf_viol, inf_iter, inf_x};
  return learned_walk(*(OracleProblem*)h, iters, tenure, 0, x, 1, nullptr, nullptr, trace_out, x_out, r_out, w_out,
                      best_obj, best_x, has_best, cutoff_rhs_out, &R, &I);
}

// The learned proposal form of the walk, replaying the listed sets.
int64_t orc_learned_replay(void* h, int64_t iters, int32_t tenure, uint64_t seed, const double* x0,
                           int32_t full_every, const int32_t* sets, const int64_t* set_off, void* trace_out,
                           double* x_out, double* r_out, float* w_out, double* best_obj, double* best_x,
                           int32_t* has_best, double* cutoff_rhs_out, int64_t* inf_viol, int64_t* inf_iter,
                           double* inf_x) {
  const WalkInfeasible I{inf_viol, inf_iter, inf_x};
  return learned_walk(*(OracleProblem*)h, iters, tenure, seed, x0, full_every, sets, set_off, trace_out, x_out,
                      r_out, w_out, best_obj, best_x, has_best, cutoff_rhs_out, nullptr, &I);
}

}  // extern "C"
