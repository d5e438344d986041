// Internal types of the gfx950 tabu-search library (not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "chap.h"

namespace chap {

// Column classes, decided once at problem creation.
enum : uint8_t {
  COL_GENERAL = 0,  // continuous, or integer with more than 64 values / infinite bounds
  COL_BINARY = 1,   // integer with bounds [0, 1]: the flip is the only move
  COL_NARROW = 2,   // integer with finite bounds and at most 64 values
};

constexpr int kShortMax = 8;       // normalised entries a single lane can score
constexpr int kNarrowBins = 64;    // values of a narrow integer column
constexpr int kSortCaps = 4;       // LDS sort capacities: 64, 256, 1024, 4096
constexpr int kSortCap[kSortCaps] = {64, 256, 1024, 4096};
constexpr int kArgmaxBlocks = 1024;  // workgroups of the move-selection reduction

// Residual and weights of one stored row. A stored row is a normalised row;
// an equality row is stored once in its '<=' orientation and carries a second
// weight for its negated twin (whose residual is -r). w1 < 0 marks a row
// without a twin.
struct __align__(16) RowState {
  double r;
  float w0;
  float w1;
};

// Read-only problem data on the device, passed to kernels by value.
struct DevProblem {
  int32_t n;
  int32_t ms;  // stored rows
  double eps;
  const int32_t* col_ptr;  // n+1
  const int32_t* col_row;  // stored row of each CSC entry
  const double* col_val;   // coefficient in the stored orientation
  const int32_t* row_ptr;  // ms+1
  const int32_t* row_col;
  const double* row_val;
  const double* row_rhs;
  const double* lb;
  const double* ub;
  const double* obj;
  const uint8_t* cls;
  const uint8_t* is_int;
};

// Mutable state of one walk (also used, with k = 0 and iters = 1, by a single
// best-shift pass). Lives in device memory.
struct __align__(16) WalkState {
  int64_t k;      // current iteration
  int64_t iters;  // iterations requested
  int32_t tenure;
  int32_t cut_active;
  double bc;  // cutoff right-hand side
  double rc;  // cutoff residual
  float wc;   // cutoff weight
  int32_t obj_integral;
  double f;      // objective at the current point
  double fbest;  // best feasible objective
  int64_t V;     // violated normalised rows (cutoff included when active)
  int32_t has_best;
  int32_t copy_best;
  // selection
  int32_t j_all;
  int32_t j_nt;
  double s_all;
  double s_nt;
  // chosen step
  int32_t mv_j;
  int32_t mv_kind;
  double mv_old;
  double mv_new;
  double mv_delta;
  double mv_score;
  unsigned long long dV;  // two's complement accumulator of violation changes
};

// A slice of a long narrow-integer column handled by one workgroup.
struct ChunkTask {
  int32_t col;
  int32_t e_beg;
  int32_t e_end;
  int32_t first;     // task index of the column's first chunk
  int32_t nchunks;
};

// Per-chunk partial result: bins, beta, alpha, candidate mask.
struct __align__(16) ChunkPartial {
  double bins[kNarrowBins];
  double beta;
  double alpha;
  unsigned long long cand;
  double pad;
};

// A general column whose entries exceed the largest LDS sort.
struct LongTask {
  int32_t col;
  int32_t cap;       // power of two >= entries
  int64_t offset;    // into the long-sort scratch arrays
};

// Device work lists of one best-shift pass.
struct PassPlan {
  const int32_t* short_cols = nullptr;  // padded to whole workgroups with -1
  int32_t n_short = 0;
  // workgroup ranges of the short-column segments: 0 binary, 1 + D non-binary
  // with D stored entries (D = 0..8); the last entry is the total
  int32_t short_segs[kShortMax + 3] = {0};
  const int32_t* flip_cols = nullptr;
  int32_t n_flip = 0;
  const int32_t* narrow_cols = nullptr;
  int32_t n_narrow = 0;
  const ChunkTask* chunks = nullptr;
  int32_t n_chunks = 0;
  ChunkPartial* partials = nullptr;
  const ChunkTask* chunk_heads = nullptr;  // first chunk of each long narrow column
  int32_t n_chunk_cols = 0;
  const int32_t* sort_cols[kSortCaps] = {nullptr, nullptr, nullptr, nullptr};
  int32_t n_sort[kSortCaps] = {0, 0, 0, 0};
  const LongTask* long_tasks = nullptr;
  int32_t n_long = 0;
  double* long_pos = nullptr;
  double* long_delta = nullptr;
  int32_t* long_marker = nullptr;
  int32_t short_max = kShortMax;
};

// ---- launchers (kernels_pass.hip) -----------------------------------------
// One exact best-shift pass over all columns: xhat, s per variable.
hipError_t launch_best_shift_pass(const DevProblem& P, const PassPlan& plan, const double* x,
                                  const RowState* rs, const WalkState* st, double* xhat, double* s,
                                  hipStream_t stream);

// ---- launchers (kernels_walk.hip) -----------------------------------------
hipError_t launch_residual(const DevProblem& P, const double* x, RowState* rs, hipStream_t stream);
hipError_t launch_set_weights_unit(const uint8_t* pair, RowState* rs, int32_t ms, hipStream_t stream);
hipError_t launch_scatter_weights(const int32_t* nidx, const uint8_t* pair, const float* w_norm, RowState* rs,
                                  int32_t ms, hipStream_t stream);
// Initialise a walk state; computes f = c^T x, V, and the cutoff from
// cutoff_rhs (active iff finite) or the incumbent rule when check_incumbent.
hipError_t launch_state_init(const DevProblem& P, const double* x, const RowState* rs, WalkState* st,
                             double* partial, uint32_t* ticket, int64_t iters, int32_t tenure,
                             int32_t obj_integral, double cutoff_rhs, const float* cutoff_w,
                             int check_incumbent, hipStream_t stream);
hipError_t launch_walk_step(const DevProblem& P, double* x, const double* xhat, const double* s, RowState* rs,
                            int32_t* tabu_until, WalkState* st, chap_trace_record* trace, double* best_x,
                            double* argmax_partial, int32_t apply_blocks, int32_t recompute,
                            hipStream_t stream);
hipError_t launch_copy_best(const double* x, double* best_x, WalkState* st, int32_t n, hipStream_t stream);

}  // namespace chap
