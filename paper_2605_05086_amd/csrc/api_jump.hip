// chap_jump_values: the jump value (weighted-violation minimiser) of every
// variable at a caller's point, with the set-up of chap_best_shift
// (residuals from scratch, weights, cutoff row) and the kernels of
// kernels_jump.hip.

#include <algorithm>
#include <string>
#include <vector>

#include "chap_internal.h"

using namespace chap;

namespace {

// Wavefront tasks of the columns longer than kJumpLane entries: per column
// its candidate tiles times its entry chunks, the longest chunks first.
int build_jump_plan(chap_problem* p) {
  const int32_t n = p->n;
  std::vector<JumpCol> cols;
  std::vector<JumpTask> tasks;
  std::vector<int32_t> len;  // entries of each task's chunk
  int32_t slot = 0;
  for (int32_t q = 0; q < n; ++q) {
    const int32_t deg = p->col_entries[q];
    if (deg <= kJumpLane) continue;
    const int32_t j = p->perm[q];
    const double l = p->lb[j], u = p->ub[j];
    const bool narrow = p->is_int[j] && std::isfinite(l) && std::isfinite(u) && u - l + 1.0 <= (double)kJumpNarrow;
    const int32_t tiles = narrow ? 1 : (2 * deg + kJumpSpecials + kWave - 1) / kWave;
    const int32_t chunks = (deg + kJumpChunk - 1) / kJumpChunk;
    if ((int64_t)slot + (int64_t)tiles * chunks >= INT32_MAX / kWave)
      return fail(CHAP_ENOMEM, "chap_jump_values: too many candidate tiles");
    cols.push_back(JumpCol{q, slot, tiles, chunks});
    for (int32_t t = 0; t < tiles; ++t)
      for (int32_t c = 0; c < chunks; ++c) {
        tasks.push_back(JumpTask{q, t, c, slot + t * chunks + c});
        len.push_back(std::min(kJumpChunk, deg - c * kJumpChunk));
      }
    slot += tiles * chunks;
  }
  std::vector<int32_t> order(tasks.size());
  for (size_t i = 0; i < order.size(); ++i) order[i] = (int32_t)i;
  std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t b) { return len[a] > len[b]; });
  std::vector<JumpTask> sorted(tasks.size());
  for (size_t i = 0; i < order.size(); ++i) sorted[i] = tasks[order[i]];
  DeviceArena& A = p->arena;
  if (!sorted.empty()) {
    JumpTask* dt;
    JumpCol* dc;
    CHAP_HIP(A.upload(&dt, sorted));
    CHAP_HIP(A.upload(&dc, cols));
    CHAP_HIP(A.alloc(&p->jump_part, (size_t)slot * kWave));
    p->jump_tasks = dt;
    p->jump_cols = dc;
  }
  p->n_jump_tasks = (int32_t)sorted.size();
  p->n_jump_cols = (int32_t)cols.size();
  CHAP_HIP(hipEventCreate(&p->jump_ev[0]));
  CHAP_HIP(hipEventCreate(&p->jump_ev[1]));
  p->jump_ready = true;
  return CHAP_OK;
}

}  // namespace

extern "C" {

int chap_jump_values(chap_problem* p, const double* d_x, const float* d_w, double cutoff_rhs, double* d_jump,
                     double* d_score, void* hip_stream) {
  if (!p) return fail(CHAP_EINVAL, "chap_jump_values: null problem");
  if (p->n > 0 && (!d_x || !d_jump || !d_score)) return fail(CHAP_EINVAL, "chap_jump_values: null device array");
  if (!d_w) return fail(CHAP_EINVAL, "chap_jump_values: null weights");
  if (std::isnan(cutoff_rhs)) return fail(CHAP_EINVAL, "chap_jump_values: cutoff_rhs is NaN");
  if (!p->jump_ready) {
    const int rc = build_jump_plan(p);
    if (rc != CHAP_OK) return rc;
  }
  hipStream_t s = (hipStream_t)hip_stream;
  const uint32_t epoch = ++p->bs_epoch == 0 ? ++p->bs_epoch : p->bs_epoch;  // never 0
  CHAP_HIP(launch_stage_x(p->dev.perm, d_x, p->bs_x, p->bs_xc, p->bs_state, epoch, p->n, s));
  CHAP_HIP(launch_residual_scatter(p->dev, p->d_nidx, p->d_pair, d_w, p->bs_x, p->bs_xc, p->bs_state, epoch,
                                   p->bs_rs, s));
  CHAP_HIP(launch_state_init(p->dev, p->bs_x, p->bs_rs, p->bs_state, p->bs_partial, p->bs_ticket, p->bs_objacc, 1,
                             0, p->obj_integral, cutoff_rhs, d_w + p->mp, 0, 0, s));
  CHAP_HIP(hipEventRecord(p->jump_ev[0], s));
  CHAP_HIP(launch_jump(p->dev, p->bs_x, p->bs_rs, p->bs_state, p->jump_tasks, p->n_jump_tasks, p->jump_cols,
                       p->n_jump_cols, p->jump_part, p->bs_xhat, p->bs_s, s));
  CHAP_HIP(hipEventRecord(p->jump_ev[1], s));
  CHAP_HIP(launch_gather2(p->d_inv, p->bs_xhat, p->bs_s, d_jump, d_score, p->n, s));
  p->jump_timed = true;
  return CHAP_OK;
}

int chap_jump_values_ms(chap_problem* p, double* ms) {
  if (!p || !ms) return fail(CHAP_EINVAL, "chap_jump_values_ms: null argument");
  *ms = 0.0;
  if (!p->jump_timed) return CHAP_OK;
  CHAP_HIP(hipEventSynchronize(p->jump_ev[1]));
  float t = 0.0f;
  CHAP_HIP(hipEventElapsedTime(&t, p->jump_ev[0], p->jump_ev[1]));
  *ms = t;
  return CHAP_OK;
}

}  // extern "C"
