// Internal types of the gfx950 tabu-search library (not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <memory>
#include <string>
#include <vector>

#include "chap.h"
#include "exact_sum.h"

namespace chap {

// (index+1)-th output of SplitMix64 started at state `seed` (Steele, Lea and
// Flood, "Fast splittable pseudorandom number generators", 2014).
__host__ __device__ inline uint64_t splitmix64(uint64_t seed, uint64_t index) {
  uint64_t z = seed + (index + 1) * 0x9E3779B97F4A7C15ULL;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}

// Pointers kept in structures are generic to the compiler, which then emits
// flat memory instructions and orders them behind pending LDS operations.
// Device allocations are global memory: casting such pointers to the global
// address space lets loads and stores issue without those waits.
template <typename T>
using gptr = __attribute__((address_space(1))) T*;
template <typename T>
__device__ __forceinline__ gptr<T> gmem(T* p) {
  return (gptr<T>)p;
}

// Loads element i of an 8- or 16-byte record array through a global pointer
// (a plain vector load: records have no copy from the global address space).
template <typename T>
__device__ __forceinline__ T gload(gptr<const T> p, int64_t i) {
  static_assert(sizeof(T) == 8 || sizeof(T) == 16, "8- or 16-byte records");
  if constexpr (sizeof(T) == 16) {
    typedef unsigned int v4 __attribute__((ext_vector_type(4)));
    const v4 v = ((gptr<const v4>)p)[i];
    return __builtin_bit_cast(T, v);
  } else {
    const unsigned long long v = ((gptr<const unsigned long long>)p)[i];
    return __builtin_bit_cast(T, v);
  }
}

// Records msg as the calling thread's last error and returns code.
int fail(int code, const std::string& msg);

#define CHAP_HIP(call)                                                                               \
  do {                                                                                              \
    hipError_t e_ = (call);                                                                         \
    if (e_ != hipSuccess) return fail(CHAP_EHIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
  } while (0)

// Device allocations owned by one object, freed together.
struct DeviceArena {
  std::vector<void*> ptrs;
  DeviceArena() = default;
  DeviceArena(const DeviceArena&) = delete;
  DeviceArena& operator=(const DeviceArena&) = delete;
  ~DeviceArena() {
    for (void* p : ptrs) (void)hipFree(p);
  }
  template <typename T>
  hipError_t alloc(T** out, size_t count) {
    void* p = nullptr;
    hipError_t e = hipMalloc(&p, std::max<size_t>(count, 1) * sizeof(T));
    if (e != hipSuccess) return e;
    ptrs.push_back(p);
    *out = (T*)p;
    return hipSuccess;
  }
  template <typename T>
  hipError_t upload(T** out, const std::vector<T>& v) {
    hipError_t e = alloc(out, v.size());
    if (e != hipSuccess) return e;
    if (!v.empty()) e = hipMemcpy(*out, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice);
    return e;
  }
};

// Column classes, decided once at problem creation.
enum : uint8_t {
  COL_GENERAL = 0,  // continuous, or integer with more than 64 values / infinite bounds
  COL_BINARY = 1,   // integer with bounds [0, 1]: the flip is the only move
  COL_NARROW = 2,   // integer with finite bounds and at most 64 values
};

constexpr int kShortMax = 8;       // normalised entries a single lane can score
constexpr int kXcds = 8;           // L2 domains (XCDs) of an MI355X; chunks are cut into as many row ranges
constexpr int kWave = 64;          // lanes of a gfx950 wavefront
constexpr int kNarrowBins = 64;
constexpr int32_t kStageUnitMask = 0x0FFFFFFF;    // values of a narrow integer column
constexpr int kSortCaps = 4;       // LDS sort capacities: 64, 256, 1024, 4096
constexpr int kSortCap[kSortCaps] = {64, 256, 1024, 4096};
constexpr int kResGroupRows = 4096;  // rows per workgroup of the x-block residual kernel
constexpr int kResXBlock = 131072;   // columns of x (bytes) per LDS block of that kernel
constexpr int kArgmaxBlocks = 256;  // workgroups of the move-selection reduction
constexpr int kArgmaxRecord = 8;     // doubles per workgroup record of that reduction
constexpr int kInitBlocks = 256;     // workgroups of the walk state initialisation
// its scratch in doubles: (f, V) per workgroup, then the workgroups' exact
// objective sums (kExactLimbs 64-bit limbs each)
constexpr int kInitPartial = kInitBlocks * (2 + kExactLimbs);

// Residual and weights of one stored row. A stored row is a normalised row;
// an equality row is stored once in its '<=' orientation and carries a second
// weight for its negated twin (whose residual is -r). w1 < 0 marks a row
// without a twin.
struct __align__(16) RowState {
  double r;
  float w0;
  float w1;
};

// Exact 8-byte copy of a RowState for all-integer walks whose residuals fit
// int32 and whose weights stay below 65535 (w1 = 0xFFFF: no twin row). The
// pass gathers it instead of the 16-byte RowState: half the footprint, the
// same FP64 values after conversion.
struct __align__(8) GatherRow {
  int32_t r;
  uint16_t w0;
  uint16_t w1;
};
constexpr uint16_t kNoTwin = 0xFFFF;

// Read-only problem data on the device, passed to kernels by value.
struct DevProblem {
  int32_t n;
  int32_t ms;  // stored rows
  double eps;
  const int32_t* col_ptr;  // n+1, internal column order
  const int32_t* col_row;  // stored row of each CSC entry (ascending within a column)
  const double* col_val;   // coefficient in the stored orientation
  const int32_t* row_ptr;  // ms+1
  const int32_t* row_col;  // internal column index, caller's order within the row
  const double* row_val;
  const double* row_rhs;
  const double* lb;  // per internal column
  const double* ub;
  const double* obj;
  const uint8_t* is_int;
  const int32_t* perm;  // original index of each internal column
  // row_val as int8 when every stored coefficient is an integer in
  // [-127, 127] (the same values, a fifth of the bytes); null otherwise
  const int8_t* row_c8;
  // Row-group x-block copy of the rows for residuals from the byte copy of
  // x (all-integer instances with row_c8, bytes for x and exact activities
  // whose byte-range bound fits int32), else null: the entries of rows
  // [g kResGroupRows, (g + 1) kResGroupRows) whose column lies in
  // [b kResXBlock, (b + 1) kResXBlock) are rb_ent/rb_c8[rb_seg[g rb_nxb + b]
  // .. rb_seg[g rb_nxb + b + 1]), each word (row in group << 17) | (column
  // in block)
  const uint32_t* rb_ent;
  const int8_t* rb_c8;
  const int32_t* rb_seg;
  int32_t rb_nxb;
  int32_t rb_pad_;
  // 1: every row activity within the bounds is an exact integer below 2^52,
  // so the residual sums of a point inside the bounds may be added in any
  // order
  int32_t sums_exact;
  int32_t pad_;
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
  // selection (original indices)
  int32_t j_all;
  int32_t j_nt;
  double s_all;
  double s_nt;
  // chosen step (internal column index)
  int32_t mv_j;
  int32_t mv_kind;
  double mv_old;
  double mv_new;
  double mv_delta;
  double mv_score;
  unsigned long long dV;  // two's complement accumulator of violation changes
  int32_t skip;           // learned walks: this iteration does nothing (block idle)
  int32_t compact_rows;   // single passes: the compact row copy is exact for these weights
  // the call (epoch) whose point did not fit the byte copy of x (see
  // launch_stage_x); 0 after the state is cleared
  uint32_t x_misfit;
  // 1 when the last step was a move whose only effect on the scores is
  // through the rows of the moved column: no reweight, no incumbent update,
  // and no cutoff row change (inactive, or c = 0 on the moved column)
  int32_t aff_ok;
  // best infeasible point so far: the fewest violated normalised rows (the
  // cutoff row not counted) among the infeasible points visited, and the
  // iteration after which it was reached (-1: the start, -2: none yet)
  int64_t inf_V;
  int64_t inf_k;
  // affected rescoring: this iteration's full pass does nothing (the
  // affected columns are scored by the subset pass instead)
  int32_t pass_skip;
  int32_t pad2_;
  int64_t aff_iters;  // iterations scored by the subset pass (affected rescoring)
};

// A slice of a long narrow-integer column handled by one workgroup; col < 0
// marks an empty task that only keeps the row-range interleave.
struct ChunkTask {
  int32_t col;    // internal column index
  int32_t e_beg;  // CSC entry range
  int32_t e_end;
  int32_t slot;   // partial record written by this task
  int32_t first;  // 1 for exactly one task per column (adds the cutoff entry)
};

// Whole narrow columns [q_begin, q_end) scored by one workgroup.
constexpr int kPackCols = 32;       // columns per pack (LDS: 32 x 64 bins)
constexpr int kPackEntries = 1024;  // target stored entries per pack
struct PackTask {
  int32_t q_begin;
  int32_t q_end;
};

// A long narrow column and its partial records [first, first + nparts).
struct ChunkCol {
  int32_t col;
  int32_t first;
  int32_t nparts;
};

// Per-chunk partial result: bins, beta, alpha, candidate mask.
struct __align__(16) ChunkPartial {
  double bins[kNarrowBins];
  double beta;
  double alpha;
  unsigned long long cand;
  double pad;
};

// Row-block staging (all-integer instances). The stored entries of narrow
// packs and of short narrow columns are kept a second time, grouped by the
// block of kStageRowBlock stored rows they touch. A workgroup of k_stage_rows
// copies one row block into LDS and turns a slice of that block's entries
// into per-entry records (in entry order), so no gather leaves the
// workgroup's LDS. A scoring task finds its records in one segment per row
// block. For integer r and a and 0 < eps < 1 the integer
// breakpoint of Algorithm 1 phase 1 is xbar + floor(-r/a) for a > 0 and
// xbar + ceil(-r/a) for a < 0, so a record holds the offset from xbar and
// needs no column data.
//
// Staged entry (uint64): bits 0..15 row inside its block, 16..23 column
// slot inside its task, 24..47 coefficient (24-bit two's complement).
// Record (uint64): bits 0..7 column slot, bit 8 coefficient > 0, bit 9 twin
// row present, bits 10..17 and 18..25 the offsets of the row and of its twin
// plus 64 (clamped to [-64, 64]); bits 32..63 the weights w0 | w1 << 16 when
// the walk keeps compact rows, else the stored row.
constexpr int kStageRowBlock = 8192;  // stored rows per block (64 KB of LDS)
constexpr int kStageSlice = 16384;    // staged entries per workgroup of k_stage_rows (fewest)
constexpr int kStageRowsPerCu = 2;    // k_stage_rows workgroups resident per CU (64 KB of LDS each)
constexpr int kStageShort = 256;      // short narrow columns per scoring task
constexpr int kStageClamp = 64;       // offsets beyond +-64 leave every narrow column
constexpr int kStageMaxRb = 256;      // row blocks a scoring workgroup can index in LDS
constexpr int kStageSliceCols = 4096; // single-entry columns per workgroup of k_stage_rows
constexpr int kStagePackCols = 64;    // columns per staged pack (one lane each in the final scan)
constexpr int kStagePackEntries = 3072;  // target stored entries per staged pack

// A slice [e_beg, e_end) of the staged entries of row block rb, and a range
// [c_beg, c_end) of the short narrow columns whose one stored entry lies in
// that block (scored there directly); rb < 0: an empty task that only keeps
// the XCD interleave.
struct StageRowTask {
  int32_t rb;
  int32_t e_beg;
  int32_t e_end;
  int32_t c_beg;
  int32_t c_end;
  int32_t pad[3];
};

// Columns [q_begin, q_end) scored by one workgroup of the staged kernels;
// deg >= 0 marks a group of short columns that all hold deg stored entries.
struct StageTask {
  int32_t q_begin;
  int32_t q_end;
  int32_t deg;
  int32_t pad;
};

// A general column whose entries exceed the largest LDS sort.
struct LongTask {
  int32_t col;
  int32_t cap;       // power of two >= entries
  int64_t offset;    // into the long-sort scratch arrays
};

// Work of one best-shift pass over one instance. Columns live in an internal
// order in which each kernel's columns form one contiguous range of internal
// indices.
struct PassPlan {
  // short columns: binaries [short_seg[0], short_seg[1]), then non-binary
  // columns with D stored entries [short_seg[1+D], short_seg[2+D])
  int32_t short_seg[kShortMax + 3] = {0};
  int32_t flip_begin = 0, flip_end = 0;
  // packs of whole narrow columns
  const PackTask* packs = nullptr;
  int32_t n_packs = 0;
  // long narrow columns cut into chunks, and their partial records
  const ChunkTask* chunks = nullptr;
  int32_t n_chunks = 0;
  const ChunkCol* chunk_cols = nullptr;
  int32_t n_chunk_cols = 0;
  int32_t n_partials = 0;
  int32_t sort_begin[kSortCaps + 1] = {0};
  const LongTask* long_tasks = nullptr;
  int32_t n_long = 0;
  int64_t long_scratch = 0;  // entries of the long-sort scratch arrays
  // row-block staging: scoring tasks [0, n_stage_packs) are packs of narrow
  // columns, the rest groups of at most kStageShort short narrow columns of
  // one degree; stage_seg holds 2 n_stage_rb + 1 values per task: the first
  // record of the task in each row block, then the task's records in the
  // blocks before each block (the last value: all of them)
  int32_t stage = 0;
  int32_t stage_exact = 0;  // the integer breakpoint identity holds (staging eligible)
  int32_t n_stage_tasks = 0;
  int32_t n_stage_packs = 0;
  int32_t n_stage_rtasks = 0;
  int32_t n_stage_rb = 0;
  const StageTask* stage_tasks = nullptr;
  const int32_t* stage_seg = nullptr;
  const StageRowTask* stage_rtasks = nullptr;
  const uint64_t* stage_ent = nullptr;
  int32_t n_stage_ent = 0;
  int32_t stage_short_begin = 0, stage_short_end = 0;
  int32_t stage_one_begin = 0, stage_one_end = 0;  // single-entry short narrow columns
  // the scoring launch of a staged pass, in units of kXcds workgroups: unit
  // u runs role (stage_units[u] >> 28) (0 chunks, 1 packs, 2 short groups)
  // on that role's unit (stage_units[u] & kStageUnitMask)
  const int32_t* stage_units = nullptr;
  int32_t n_stage_units = 0;
};

// Everything the kernels of one walk need: its instance, the instance's pass
// plan, and the walk's own buffers. One record per walk in device memory;
// a single best-shift pass or a single walk is a batch of one.
struct WalkCtx {
  DevProblem P;
  PassPlan plan;
  double* x;
  double* xhat;
  double* s;
  double* best_x;
  int32_t* tabu;
  RowState* rs;
  GatherRow* grow;  // compact copy of rs kept by the walk kernels, or null
  WalkState* st;
  chap_trace_record* trace;
  double* argmax_partial;
  ChunkPartial* partials;
  double* long_pos;
  double* long_delta;
  int32_t* long_marker;
  uint64_t* stage_rec;  // records of the staged entries (row-block staging)
  // exact fixed-point sum of c^T x (kExactLimbs limbs) when FP64 sums of the
  // objective may be inexact; null otherwise
  long long* objacc;
  // byte copy of x for residuals from scratch (problems whose variables are
  // all integers with bounds in [-128, 127]), or null
  int8_t* xc;
  int32_t argmax_blocks;
  // further move-selection workgroups, one wavefront per long narrow column:
  // they combine those columns' partial bins when the pass leaves that to
  // the move selection, else they only write empty records
  int32_t argmax_comb;
  int32_t apply_blocks;
  int32_t recompute;
};

// Kernels of one iteration; each has its own per-walk block counts.
enum KernelSlot {
  KS_SHORT = 0,
  KS_FLIP,
  KS_PACK,
  KS_CHUNK,
  KS_COMBINE,
  KS_SORT0,
  KS_LONG = KS_SORT0 + kSortCaps,
  KS_STAGE,
  KS_STAGE_SCORE,
  KS_ARGMAX,
  KS_SELECT,
  KS_APPLY,
  KS_FINISH,
  KS_COUNT
};

// Launch table of a batch of walks: for every kernel the prefix sums of the
// per-walk block counts (device arrays of nw + 1 entries) and their total.
// Block b of a launch belongs to the walk w with off[w] <= b < off[w + 1].
struct BatchLaunch {
  int32_t nw = 0;
  // 0: the pass gathers RowState; 1: every walk keeps a GatherRow copy and the
  // pass gathers it; 2: the copy is used where WalkState::compact_rows says so
  int32_t compact = 0;
  const WalkCtx* walks = nullptr;
  const int32_t* off[KS_COUNT] = {};
  int32_t total[KS_COUNT] = {};
  int32_t grid[KS_COUNT] = {};  // workgroups to launch (total, or kXcds x the largest XCD share)
};

// Blocks kernel `slot` needs for one walk.
int32_t kernel_blocks(const WalkCtx& c, int slot);

// Walk of this workgroup and its index inside that walk, or -1 for a
// padding workgroup. off holds the prefix of per-walk block counts (nw + 1
// values). A batch (nw > 1) places every walk on one XCD: its walks are
// ordered by XCD and off is followed by the first virtual block of each XCD
// and the XCD's block count; workgroup b runs on XCD b mod kXcds (the
// dispatch order) and takes the (b / kXcds)-th block of that XCD, so a
// walk's row states stay in one L2.
__device__ __forceinline__ int block_walk(const int32_t* __restrict__ off, int nw, int& local) {
  int b = blockIdx.x;
  if (nw > 1) {
    const int x = b % kXcds, s = b / kXcds;
    if (s >= off[nw + 1 + kXcds + x]) return -1;
    b = off[nw + 1 + x] + s;
  }
  int lo = 0, hi = nw - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (off[mid] <= b)
      lo = mid;
    else
      hi = mid - 1;
  }
  local = b - off[lo];
  return lo;
}

// Side streams on which the pass kernels run beside the main stream (they
// write disjoint columns): fork and join events order them with the main
// stream, also under graph capture.
struct PassStreams {
  hipStream_t side[2] = {nullptr, nullptr};
  hipEvent_t fork = nullptr;
  hipEvent_t join[2] = {nullptr, nullptr};
  hipError_t create();
  void destroy();
};

// ---- launchers (kernels_pass.hip) -----------------------------------------
// One exact best-shift pass over all columns of every walk of the batch;
// with `ps`, the short-column and long-column kernels run on side streams
// beside the pack kernel. With defer_combine, a pass for which
// pass_defers_combine(L) holds leaves the long narrow columns' partial bins
// uncombined: the move selection that follows (launch_walk_choose with
// combine) scores them while it scans.
hipError_t launch_pass(const BatchLaunch& L, hipStream_t stream, const PassStreams* ps = nullptr,
                       bool defer_combine = false);
// Only when every walk with long narrow columns is staged (no k_narrow_chunk
// blocks): the move selection's extra workgroups exist for staged walks only.
inline bool pass_defers_combine(const BatchLaunch& L) {
  return L.compact == 1 && L.total[KS_STAGE_SCORE] > 0 && L.total[KS_COMBINE] > 0 && L.total[KS_CHUNK] == 0;
}

// A fixed permutation out[i] = in[src[i]] of n FP64 values applied in two
// coalesced passes through LDS instead of one gather of random 8-byte
// words: the first pass sorts each input chunk of kPermChunk values by
// output block in LDS and writes it to a staging array in which each
// output block's values are contiguous (one run per chunk); the second
// places each block's values at their offsets in LDS and writes the block.
constexpr int kPermChunk = 8192;  // input values per workgroup of the first pass
constexpr int kPermBlock = 4096;  // output values per workgroup of the second pass
struct PermPlan {
  int32_t n = 0;
  const uint16_t* lpos = nullptr;  // input e: rank in its chunk's (output block, e) order
  const int32_t* sdst = nullptr;   // chunk base + rank: its staging slot
  const uint16_t* dl = nullptr;    // staging slot s: offset of its value in its output block
};
// Plan of the permutation that sends input e to output dest[e] (dest a
// bijection of [0, n)), uploaded into A.
hipError_t build_perm_plan(const std::vector<int32_t>& dest, DeviceArena& A, PermPlan* plan);

// ---- launchers (kernels_walk.hip) -----------------------------------------
// Single-walk set-up kernels.
// The point of a call in internal order: dst[q] = src[perm[q]] (src already
// in internal order when perm is null, dst then equal to src or null). With
// xc, also its byte copy: a value that is not an integer in [-128, 127]
// stores `epoch` in st->x_misfit, and residuals of this call then read dst.
hipError_t launch_stage_x(const int32_t* perm, const double* src, double* dst, int8_t* xc, WalkState* st,
                          uint32_t epoch, int32_t n, hipStream_t stream);
// Residuals from scratch (weights left as they are). With xc (and
// st->x_misfit != epoch) the products read the byte copy of x.
hipError_t launch_residual(const DevProblem& P, const double* x, RowState* rs, hipStream_t stream);
// Residuals from scratch with unit weights, and the compact copy when grow
// is not null.
hipError_t launch_residual_unit(const DevProblem& P, const uint8_t* pair, const double* x, const int8_t* xc,
                                const WalkState* st, uint32_t epoch, RowState* rs, GatherRow* grow,
                                hipStream_t stream);
// Residuals from scratch with the caller's normalised weights w_norm. With
// grow, also the checked compact copy (launch_fill_compact_checked's work):
// the state initialisation must have run, and st is then written.
hipError_t launch_residual_scatter(const DevProblem& P, const int32_t* nidx, const uint8_t* pair,
                                   const float* w_norm, const double* x, const int8_t* xc, const WalkState* st,
                                   uint32_t epoch, RowState* rs, hipStream_t stream, GatherRow* grow = nullptr);
// Seeded start point (internal order), and its byte copy when xc is set.
hipError_t launch_start_point(const DevProblem& P, uint64_t seed, double* x, int8_t* xc, hipStream_t stream);
// Initialise a walk state; computes f = c^T x, V, and the cutoff from
// cutoff_rhs (active iff finite) or the incumbent rule when check_incumbent.
// partial: kInitPartial doubles; ticket: zero on entry (left zero); objacc:
// the exact objective sum to initialise (kExactLimbs), or null when FP64
// sums of the objective are exact. V is counted with check_incumbent or
// count_violated; f with check_incumbent or a finite cutoff_rhs (a single
// pass needs neither V nor, without a cutoff row, f).
hipError_t launch_state_init(const DevProblem& P, const double* x, const RowState* rs, WalkState* st,
                             double* partial, uint32_t* ticket, long long* objacc, int64_t iters, int32_t tenure,
                             int32_t obj_integral, double cutoff_rhs, const float* cutoff_w,
                             int check_incumbent, int count_violated, hipStream_t stream);
hipError_t launch_copy_best(const double* x, double* best_x, WalkState* st, int32_t n, hipStream_t stream);
// grow[i] = compact copy of rs[i]
hipError_t launch_fill_compact(const RowState* rs, GatherRow* grow, int32_t ms, hipStream_t stream);
// The same for a single pass with caller weights: clears st->compact_rows
// (set by the state initialisation) when a residual or weight does not fit.
hipError_t launch_fill_compact_checked(const RowState* rs, GatherRow* grow, WalkState* st, int32_t ms,
                                       hipStream_t stream);
// dst[q] = src[perm[q]] (original order -> internal order)
hipError_t launch_gather(const int32_t* perm, const double* src, double* dst, int32_t n, hipStream_t stream);
// launch_stage_x (dst not null, not src) through a plan of the same
// permutation; stage: n doubles.
hipError_t launch_stage_x_plan(const PermPlan& plan, const double* src, double* dst, int8_t* xc, WalkState* st,
                               uint32_t epoch, double* stage, hipStream_t stream);
// launch_gather2 through a plan of the same permutation; stage: 2n doubles.
hipError_t launch_gather2_plan(const PermPlan& plan, const double* a, const double* b, double* da, double* db,
                               double* stage, hipStream_t stream);
// da[j] = a[inv[j]], db[j] = b[inv[j]] (internal order -> original order)
hipError_t launch_gather2(const int32_t* inv, const double* a, const double* b, double* da, double* db, int32_t n,
                          hipStream_t stream);
// Move selection, application and iteration end for every walk of the batch
// (combine: after a pass launched with defer_combine).
hipError_t launch_walk_step(const BatchLaunch& L, hipStream_t stream, bool combine = false);
// Final copy of an incumbent found by a walk's last iteration.
hipError_t launch_copy_best_batch(const BatchLaunch& L, hipStream_t stream);

// ---- proposal network (kernels_mlp.hip) -----------------------------------
constexpr int kNParamPad = 5376;   // row stride of gradient partials (>= 5313 parameters)
constexpr int kGradBlocks = 64;    // most workgroups of one gradient launch
constexpr double kAdamBeta1 = 0.9;
constexpr double kAdamBeta2 = 0.999;
constexpr float kAdamEps = 1e-8f;

// Device state of one network: FP32 parameters (flat order W1, b1, W2, b2,
// W3, b3), their bfloat16 copy, Adam moments and step, gradient buffers.
struct ModelDev {
  float* w = nullptr;
  uint16_t* wb = nullptr;
  float* m = nullptr;
  float* v = nullptr;
  double* adam = nullptr;  // beta1^t, beta2^t, t
  float* grad = nullptr;
  float* partials = nullptr;  // kGradBlocks x kNParamPad
};

hipError_t launch_mlp_forward(const ModelDev& M, const uint16_t* feat, int64_t n, float* out, hipStream_t s);
// Gradient partials of the mean squared error over nb samples of (feat,
// target) with `rows` rows: sample i is row i, or with `sample` row
// splitmix64(seed, base + i) mod rows.
hipError_t launch_mlp_grad(const ModelDev& M, const uint16_t* feat, const float* target, int64_t rows, int64_t nb,
                           int sample, uint64_t seed, uint64_t base, hipStream_t s);
// Reduces the partials of the last gradient launch over nb samples into
// M.grad; with `update`, one Adam step with learning rate lr.
hipError_t launch_mlp_reduce(const ModelDev& M, int64_t nb, int update, float lr, hipStream_t s);
hipError_t launch_mlp_bf16_copy(const ModelDev& M, hipStream_t s);
// Guarded variants used inside a learned walk's graph: they do nothing while
// *active == 0.
hipError_t launch_mlp_grad_guarded(const ModelDev& M, const int32_t* active, const uint16_t* feat,
                                   const float* target, int64_t nb, hipStream_t s);
hipError_t launch_mlp_reduce_guarded(const ModelDev& M, const int32_t* active, int64_t nb, float lr, hipStream_t s);

// ---- learned candidate proposal (kernels_learned.hip) ---------------------
constexpr int kRadixBins = 2048;    // radix-select digit bins (11, 11, 10 bits)
constexpr int kTopkChunk = 4096;    // columns per workgroup of the top-K compaction
constexpr int kTopkMax = 8192;      // largest proposal set
constexpr int kSubsetCap = 4096;    // breakpoint capacity of the subset sort workgroup
constexpr int kSubsetChunk = 2048;  // stored entries per workgroup chunk of the subset pass
constexpr int kSubsetGrid = 2048;   // workgroups of the subset chunk kernel (grid-stride)
constexpr int kJumpLane = 8;       // stored entries up to which one lane finds a column's jump value
constexpr int kJumpChunk = 4096;   // entries per wavefront task of a longer column
constexpr int kJumpBinChunk = 1024;  // entries per wavefront of a column scored from bins
constexpr int kJumpNarrow = 64;    // integer domains up to this size try every value
constexpr int kJumpSpecials = 7;   // cutoff kinks (2), l, u, xbar - 1, xbar + 1, xbar
constexpr int kRescoreCapMax = 4096;  // largest rescore_cap (columns of an affected set, listed in LDS)
constexpr int kRefreshShort = 64;   // stored entries up to which 8 lanes refresh a column
constexpr int kRefreshChunk = 4096; // stored entries per workgroup chunk of the long-column refresh
constexpr int kStallKind = 3;       // trace kind of a proposal iteration without a move
constexpr int kProposalKind = 8;    // added to the kind of a move chosen from a proposal set

// Per-column proposal class (internal order): binaries and narrow integer
// columns of any length (chunked subset pass), general columns whose
// breakpoints fit one workgroup's LDS sort.
enum : uint8_t { SUB_NONE = 0, SUB_FLIP = 1, SUB_NARROW = 2, SUB_GENERAL = 3 };

struct TopkState {
  int32_t count;   // entries selected
  int32_t chunks;  // subset-pass chunks of the selected columns (proposal set only)
};

struct LearnState {
  int32_t idle;          // the rest of this block's proposal iterations do nothing
  int32_t train_active;  // the block's full evaluation ran: train, refresh the rows
  int64_t k_last_full;   // iteration of the last full evaluation
  int64_t evals;         // full evaluations
  int64_t hits;          // full evaluations whose move was in the network's proposal set
  int64_t stalls;        // proposal iterations without an admissible move
  int64_t logged;        // pairs written to the pair log
  int64_t set_pos;       // entries written to the proposal-set log
  TopkState tk[2];       // 0: proposal set, 1: training labels
};

// Partial sums of one refresh chunk: sum w, sum w (violated), violated rows,
// rows, sum |a|, sum |a| min(r, 1000) (violated).
struct __align__(16) RefreshPart {
  double v[6];
};

// Stored feature rows (16 bfloat16 per column): slots 0..11 hold network
// inputs 0..11, slots 12..13 the int32 iteration of the column's last move,
// slot 14 is unused and slot 15 holds input 15. Inputs 12..14 are computed
// when a row is read.
struct LearnCtx {
  const uint8_t* cls;        // SUB_* per internal column
  const int32_t* elig_list;  // internal indices of proposable columns
  int32_t n_elig;
  // 1: listed short columns (the plan's short range) are scored one per lane
  // by k_aff_score's lane role, and the subset kernels leave them alone
  int32_t short_lane;
  int32_t mp;                // normalised rows (for the violated fraction)
  double c_max;              // max |c_j| (0 when c = 0)
  // row refresh work: short proposable columns, chunks of long ones
  const int32_t* ref_short;
  int32_t n_ref_short;
  int32_t n_ref_chunks;
  const ChunkTask* ref_chunks;
  const ChunkCol* ref_cols;
  int32_t n_ref_cols;
  int32_t pad0;
  RefreshPart* ref_parts;
  uint16_t* feat;            // n x 16 stored rows
  int32_t* moves;            // moves per column
  double* xhat_last;         // best shift at the last full evaluation
  uint32_t* keys[2];         // 0: network scores, 1: labels
  uint32_t* hist;            // 2 x 3 x kRadixBins
  int32_t* wg_cnt;           // 2 x nwg x 2 (greater, equal)
  int32_t* sel[2];           // selected columns, ascending internal index
  int32_t K[2];
  int32_t nwg;               // workgroups of the compaction
  int32_t sub_cap;           // capacity of sub_parts
  int32_t* sub_off;          // K[0] + 1 chunk offsets of the selected columns
  ChunkPartial* sub_parts;   // per-chunk partial bins of the subset pass
  uint16_t* pair_feat;       // 2T x 16 training inputs
  float* pair_tgt;           // 2T targets
  uint16_t* log_feat;        // pair log (nullable)
  float* log_tgt;
  int64_t log_cap;
  int32_t* set_log;          // proposal-set log (nullable), original indices
  int64_t* set_off;          // iters + 1 offsets into set_log (nullable)
  int64_t set_log_cap;
  int32_t T;
  int32_t full_every;
  uint64_t seed;
  LearnState* ls;
};

// One learned walk (C: one walk context on the device, L: its learned
// context on the device, Lh: host copy of L).
// Stored rows of every column; last_move and moves (original order) may be
// null for a walk's start (never moved).
hipError_t launch_learn_init(const WalkCtx* C, const LearnCtx* L, const LearnCtx& Lh, int32_t n,
                             const int32_t* last_move, const int32_t* moves, hipStream_t s);
hipError_t launch_learn_refresh(const WalkCtx* C, const LearnCtx* L, const LearnCtx& Lh, hipStream_t s);
hipError_t launch_learn_begin(const WalkCtx* C, const LearnCtx* L, hipStream_t s);
// Network scores of every column and the proposal set (top K[0]); also the
// pending incumbent copy of the iteration.
hipError_t launch_learn_propose(const WalkCtx* C, const LearnCtx* L, const LearnCtx& Lh, const ModelDev& M,
                                int32_t n, int full_iteration, hipStream_t s);
// Training pairs of a full evaluation (top T by score + T random) and the
// network update.
hipError_t launch_learn_train(const WalkCtx* C, const LearnCtx* L, const LearnCtx& Lh, const ModelDev& M,
                              int32_t n, int32_t steps, float lr, hipStream_t s);
// A proposal iteration that keeps the last proposal set (logs it again).
hipError_t launch_learn_keep_set(const WalkCtx* C, const LearnCtx* L, hipStream_t s);
// Judge of a full evaluation and the stored-row update of its move.
hipError_t launch_learn_judge(const WalkCtx* C, const LearnCtx* L, hipStream_t s);
// Materialised inputs of every column at the walk's state (original order).
hipError_t launch_learn_features_out(const WalkCtx* C, const LearnCtx* L, int32_t n, int64_t k, int64_t k_last_full,
                                     uint16_t* out, hipStream_t s);
// Exact best shift of the proposal set (kernels_pass.hip).
hipError_t launch_subset_pass(const WalkCtx* C, const LearnCtx* L, const LearnCtx& Lh, int has_general, int compact,
                              hipStream_t s);
// Jump values (kernels_jump.hip): one wavefront task of a longer column (its
// candidate tile and entry chunk; slot = the column's first slot + tile x
// chunks + chunk), and the column's record for the combine.
struct JumpTask {
  int32_t q, tile, chunk, slot;
  int32_t bins;  // the column also has a bins form (see JumpBinTask)
};
struct JumpCol {
  int32_t q, first_slot, ntiles, nchunks;
  int32_t bfirst, bn;  // its bins slots (bn = 0: no bins form; -1: one bins task finishes it)
};
// A chunk of a narrow column's entries scored into slope and offset bins
// (exact integer data): V(l + p) = sum_{k <= p} K[k] + p sum_{k <= p} S[k].
struct JumpBinTask {
  int32_t q, e_beg, e_end, slot;  // q < 0: padding; slot < 0: the whole column, finished by the task
};
// Jump value and score of every column (internal order) into jv, js; part
// holds kWave doubles per task slot.
// grow: the instance's compact row copy as this call wrote it, when that
// copy can be exact (all-integer data, residuals within int32), else null
// (exact_data below is grow != null); obj_small: objective sums are exact
// small integers. With integer weights (checked on the device) the lane kernel
// then tries fewer values of narrow columns, with the same results.
// Columns with a bins form are scored from int64 slope and offset bins
// when the call's data are exact (integer weights; then every V is an
// integer below 2^53 and any order of summation gives the oracle's value),
// else by the wavefront tasks like every other long column.
// Tasks come as [tasks of columns without a bins form (n_plain_tasks)]
// [the others]; column records as [no bins form (n_plain_cols)] [chunked
// bins form (n_chunk_cols)] [bins form finished by one bins task], so that
// exact calls visit only what they need.
hipError_t launch_jump(const DevProblem& P, const double* x, const RowState* rs, const WalkState* st,
                       const GatherRow* grow, int32_t obj_small, const JumpTask* tasks, int32_t ntasks,
                       int32_t n_plain_tasks, const JumpBinTask* btasks, int32_t nbtasks, const JumpCol* cols,
                       int32_t ncols, int32_t n_plain_cols, int32_t n_chunk_cols, double* part, long long* bpart,
                       double* jv, double* js, hipStream_t s);
// The same kernels with explicit grids (each kernel strides over its work).
hipError_t launch_subset_grids(const WalkCtx* C, const LearnCtx* L, int chunk_grid, int combine_grid, int general_grid,
                               int has_general, int compact, hipStream_t s);

// The lists of affected rescoring. The affected columns of an iteration are
// split into its short columns (slist: grouped by short class, binaries then
// D = 0..8 stored entries, each class padded with -1 to a multiple of 64 so
// that a wavefront holds one class) and the rest (olist, with the subset
// chunk offsets ooff). When every column has a subset form, the same split
// of all columns (full_*) serves iterations that must score every column.
struct AffRun {
  const int32_t* slist;  // short columns of this iteration (-1: padding)
  int32_t n_s;           // entries of slist, padding included
  int32_t pad_;
};
constexpr int kAffClasses = kShortMax + 2;  // binaries, then D = 0..kShortMax
constexpr int kAffRows = 256;  // rows of a moved column up to which its affected columns are listed

struct AffLists {
  int32_t* stamp = nullptr;  // n
  int32_t* slist = nullptr;  // cap + 64 kAffClasses
  int32_t* olist = nullptr;  // cap
  int32_t* ooff = nullptr;   // cap + 1
  AffRun* run = nullptr;     // 1
  int32_t cap = 0;
  int32_t sub_cap = 0;
  const int32_t* full_slist = nullptr;  // null: those iterations run the full pass
  const int32_t* full_olist = nullptr;
  const int32_t* full_ooff = nullptr;
  int32_t n_full_s = 0;
  int32_t n_full_o = 0;
  int32_t full_chunks = 0;
};

// Affected rescoring of one walk (kernels_walk.hip). After a move whose
// effect on the scores goes only through the rows of the moved column,
// those rows' columns (and the moved column) are the only ones whose best
// shift can change: k_aff_plan lists them and hands the list to the lane
// kernel and the subset pass or, when it holds more than `cap` columns, a
// column the subset pass cannot score, or more than `sub_cap` chunks, makes
// the iteration score every column.
hipError_t launch_affected(const WalkCtx* C, LearnCtx* L, const AffLists& A, hipStream_t s);
// Diversity restarts of batched walks (kernels_walk.hip). A Hamming task
// counts, over internal columns [begin, end) of one problem, the discrete
// variables at which two walks' points differ, into dist[pair].
struct HamTask {
  const double* xa;
  const double* xb;
  const uint8_t* is_int;
  int32_t begin, end;
  int32_t pair;
  int32_t pad_;
};
// What a restarted walk keeps: its iteration count, best feasible objective
// and its best infeasible point's record.
struct RestartKeep {
  int64_t k;
  double fbest;
  int64_t inf_V;
  int64_t inf_k;
  int32_t has_best;
  int32_t pad_;
};
// st->iters = iters_end for every walk of the launch table.
hipError_t launch_set_iters(const BatchLaunch& L, int64_t iters_end, hipStream_t s);
hipError_t launch_hamming(const HamTask* tasks, int32_t ntasks, int32_t* dist, hipStream_t s);
// After the set-up kernels of a restart (start point, residuals, state at
// the kept cutoff): the kept iteration count and, unless the restart point
// is a new incumbent, the kept best objective; the better best infeasible
// record.
hipError_t launch_restart_fix(WalkState* st, const RestartKeep& keep, hipStream_t s);
// The whole scoring of an affected-rescoring iteration: one launch whose
// workgroups take four roles: the short columns by lanes (g[0]), general
// columns of at most 64 breakpoints by wavefronts (g[1]), the subset chunks
// (g[2]) and the subset general columns (g[3]); then the subset combine.
hipError_t launch_aff_score(const WalkCtx* C, const LearnCtx* L, const AffRun* run, const int g[4], int combine_grid,
                            int compact, hipStream_t s);
// Move choice over the proposal set and the stored-row update of its move
// (kernels_walk.hip).
hipError_t launch_subset_select(const WalkCtx* C, const LearnCtx* L, hipStream_t s);

}  // namespace chap

namespace chap {
struct WalkPool;
}  // namespace chap

// Handles of the C ABI (defined here so every source file of the library
// sees them).
struct chap_problem {
  int32_t n = 0, m = 0, mp = 0;
  double eps = 1e-6;
  chap_options opt{};
  int32_t obj_integral = 1;
  int32_t max_col_deg = 0;
  // 1 when every variable is integer with finite bounds and every
  // coefficient and right-hand side is an integer small enough that all row
  // activities are exact in FP64: incremental residual updates are then exact
  int32_t exact_incremental = 0;
  // 1 when additionally every row activity fits int32 (walks may then gather
  // residuals from the compact GatherRow copy)
  int32_t compact_ok = 0;
  // 1 when every variable with c_j != 0 is integer with finite bounds, every
  // such c_j is an integer and sum |c_j| max(|l_j|, |u_j|) < 2^52: every FP64
  // sum of the objective (and the cutoff residual) is then exact, in any order;
  // otherwise walks keep the exact fixed-point sum of c^T x
  int32_t obj_fast = 1;
  // 1 when every variable is an integer with bounds in [-128, 127]: points
  // within the bounds have an exact byte copy, which residuals from scratch
  // gather instead of FP64 values (a 1-byte gather per nonzero)
  int32_t x_small = 0;
  // host copies used by runs
  std::vector<double> lb, ub, obj;
  std::vector<uint8_t> is_int;
  std::vector<int32_t> nidx;  // normalised index of each stored row
  std::vector<uint8_t> pair;  // stored row is an equality (two normalised rows)
  std::vector<int32_t> norm_orig;
  std::vector<int8_t> norm_sign;
  // device
  chap::DeviceArena arena;
  chap::DevProblem dev{};
  chap::PassPlan plan{};
  const int32_t* d_nidx = nullptr;
  const uint8_t* d_pair = nullptr;
  const int32_t* d_inv = nullptr;  // internal index of each original column
  int32_t device = 0;
  // scratch of chap_best_shift
  chap::RowState* bs_rs = nullptr;
  chap::WalkState* bs_state = nullptr;
  double* bs_partial = nullptr;
  uint32_t* bs_ticket = nullptr;
  double* bs_x = nullptr;
  double* bs_xhat = nullptr;
  double* bs_s = nullptr;
  chap::GatherRow* bs_grow = nullptr;
  long long* bs_objacc = nullptr;
  int8_t* bs_xc = nullptr;
  uint32_t bs_epoch = 0;
  // chap_best_shift and chap_jump_values: the caller's point into internal
  // order and the results back, as two-pass permutations over bs_stage
  // (2n doubles)
  chap::PermPlan to_internal, to_caller;
  double* bs_stage = nullptr;
  std::vector<int32_t> perm;  // original index of each internal column
  // host copy of the caller's arrays (the autotuner re-plans from them)
  struct Raw {
    std::vector<int64_t> csr_row_ptr, csc_col_ptr;
    std::vector<int32_t> csr_col, csc_row;
    std::vector<double> csr_val, csc_val, rhs, lb, ub, obj;
    std::vector<char> sense;
    std::vector<uint8_t> is_int;
  } raw;
  // learned proposal: SUB_* class and stored entries per internal column,
  // max |c_j|
  std::vector<uint8_t> sub_cls;
  std::vector<int32_t> col_entries;
  int64_t nnz = 0;
  double c_max = 0.0;
  chap::BatchLaunch bs_launch;
  hipEvent_t pass_ev[2] = {nullptr, nullptr};
  chap::PassStreams bs_streams;
  bool pass_timed = false;
  // the pass kernels of chap_best_shift as one HIP graph, captured on the
  // first call and replayed on the caller's stream
  hipStream_t bs_cap = nullptr;
  hipGraph_t bs_graph = nullptr;
  hipGraphExec_t bs_exec = nullptr;
  // buffers of single walks kept between chap_tabu_run calls
  std::shared_ptr<chap::WalkPool> pool;
  // jump values: wavefront tasks of the longer columns (built on the first
  // chap_jump_values call), their partial sums, timing events
  bool jump_ready = false;
  const chap::JumpTask* jump_tasks = nullptr;
  const chap::JumpCol* jump_cols = nullptr;
  const chap::JumpBinTask* jump_btasks = nullptr;
  int32_t n_jump_tasks = 0, n_jump_cols = 0, n_jump_btasks = 0;
  int32_t n_jump_plain_tasks = 0, n_jump_plain_cols = 0, n_jump_chunk_cols = 0;
  double* jump_part = nullptr;
  long long* jump_bpart = nullptr;
  hipEvent_t jump_ev[2] = {nullptr, nullptr};
  bool jump_timed = false;
  ~chap_problem() {
    for (hipEvent_t e : pass_ev)
      if (e) (void)hipEventDestroy(e);
    for (hipEvent_t e : jump_ev)
      if (e) (void)hipEventDestroy(e);
    if (bs_exec) (void)hipGraphExecDestroy(bs_exec);
    if (bs_graph) (void)hipGraphDestroy(bs_graph);
    if (bs_cap) (void)hipStreamDestroy(bs_cap);
    bs_streams.destroy();
  }
};

namespace chap {

// Device buffers, launch table, streams and captured iteration graphs of one
// single walk. A problem keeps one idle slot between runs, so repeated
// chap_tabu_run calls allocate, upload and capture nothing: a call is the
// set-up kernels, the graph launches and the trace copy.
struct WalkSlot {
  DeviceArena A;
  WalkCtx ctx{};  // host copy of the device record L.walks[0]
  BatchLaunch L{};
  GatherRow* grow_buf = nullptr;  // compact rows (all-integer instances), used when a run allows them
  chap_trace_record* trace_buf = nullptr;
  int64_t trace_cap = 0;
  double* partial = nullptr;
  uint32_t* ticket = nullptr;
  hipStream_t s = nullptr;
  PassStreams ps;
  hipEvent_t ev[3] = {nullptr, nullptr, nullptr};  // caller's stream, graph start, graph end
  struct Graph {
    int64_t K;
    int compact;
    hipGraph_t g;
    hipGraphExec_t x;
  };
  std::vector<Graph> graphs;  // K iterations each (K a power of two or graph_iters)
  // affected rescoring (problems created with rescore_cap > 0)
  AffLists aff{};
  LearnCtx* aff_L = nullptr;     // device record for the subset pass
  LearnCtx aff_Lh{};             // its host copy
  int aff_general = 0;           // the problem has general columns
  WalkSlot() = default;
  WalkSlot(const WalkSlot&) = delete;
  WalkSlot& operator=(const WalkSlot&) = delete;
  ~WalkSlot() {
    for (Graph& g : graphs) {
      (void)hipGraphExecDestroy(g.x);
      (void)hipGraphDestroy(g.g);
    }
    if (trace_buf) (void)hipFree(trace_buf);
    for (hipEvent_t e : ev)
      if (e) (void)hipEventDestroy(e);
    ps.destroy();
    if (s) (void)hipStreamDestroy(s);
  }
};

// Host maps a run needs to return its state in the caller's order, and the
// problem's idle walk slot. Shared by the problem and its runs, so a run may
// outlive its problem.
struct WalkPool {
  int32_t n = 0, m = 0, mp = 0;
  std::vector<int32_t> perm, nidx;
  std::vector<uint8_t> pair;
  std::vector<std::unique_ptr<WalkSlot>> idle;
  void give_back(std::unique_ptr<WalkSlot>& slot) {
    if (slot && idle.empty()) idle.push_back(std::move(slot));
    slot.reset();
  }
};

}  // namespace chap

struct chap_run {
  std::vector<chap_trace_record> trace;
  std::vector<double> x, resid, best_x;
  std::vector<float> w;
  double best_obj = HUGE_VAL;
  double cutoff_rhs = HUGE_VAL;
  bool has_best = false;
  double elapsed_ms = 0.0;
  // single walks: x, resid, w and best_x are read from the walk's device
  // buffers on the first chap_run_state that asks for them; the buffers then
  // go back to the problem
  mutable std::shared_ptr<chap::WalkPool> pool;
  mutable std::unique_ptr<chap::WalkSlot> slot;
  chap::WalkState st_end{};
  mutable bool state_ready = true;
  // best infeasible point (see WalkState::inf_V): its violated rows, the
  // iteration after which it was reached, and the point (caller's order,
  // rebuilt from the final point and the trace when the state is read)
  int64_t inf_viol = 0;
  int64_t inf_iter = -2;
  std::vector<double> inf_x;
  // walks of chap_batch_restarts: the iterations at which the walk restarted
  std::vector<int64_t> restarts;
  bool restart_run = false;
  ~chap_run() {
    if (pool) pool->give_back(slot);
  }
  // learned walks
  int64_t evals = 0, hits = 0, stalls = 0;
  std::vector<int32_t> sets;     // proposal sets (original indices)
  std::vector<int64_t> set_off;  // iters + 1 offsets into sets
  std::vector<uint16_t> pair_feat;
  std::vector<float> pair_tgt;
};


struct chap_model {
  int32_t device = 0;
  chap::DeviceArena arena;
  chap::ModelDev dev;
};

namespace chap {

// One walk of a run: its problem, start point (original order, or null for
// the seeded start point) and seed.
struct WalkSpec {
  chap_problem* p;
  uint64_t seed;
  const double* x0;
};

// Allocates one walk's buffers in A (a trace of trace_cap records when
// trace_cap > 0; the compact row copy when the problem allows it).
int alloc_walk(const chap_problem* p, int64_t trace_cap, DeviceArena& A, WalkCtx& c);
// Start point (seeded on the device, or the caller's x0) and the set-up
// kernels of a walk on stream s: tabu list, residuals with unit weights (and
// c.grow when set), state, incumbent check.
int init_walk(const WalkSpec& spec, int64_t iters, int32_t tenure, const WalkCtx& c, double* partial,
              uint32_t* ticket, hipStream_t s);
// alloc_walk + init_walk (the compact copy only when `compact`).
int prepare_walk(const WalkSpec& spec, int64_t iters, int32_t tenure, DeviceArena& A, WalkCtx& c, double* partial,
                 uint32_t* ticket, hipStream_t s, int compact);
// 1 when every walk of a run may keep the compact GatherRow copy.
int compact_walks(const std::vector<WalkSpec>& specs, int64_t iters);
// Copies a finished walk back into R (host order).
int collect_walk(const chap_problem* p, const WalkCtx& c, int64_t iters, double ms, chap_run* R);
// Device copy of the walk contexts and the per-kernel launch tables; a batch
// is reordered by XCD (order[i]: caller's index of ctx[i]; may be null).
hipError_t build_launch(DeviceArena& A, std::vector<WalkCtx>& ctx, BatchLaunch* L, std::vector<int32_t>* order);
int blocks_for_host(int64_t work, int cap);
// The parts of launch_walk_step: argmax + selection, application, end of
// iteration.
hipError_t launch_walk_choose(const BatchLaunch& L, hipStream_t stream, bool combine = false);
hipError_t launch_walk_apply(const BatchLaunch& L, hipStream_t stream);
hipError_t launch_walk_finish(const BatchLaunch& L, hipStream_t stream);

}  // namespace chap
