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
// its candidate tiles times its entry chunks, the longest chunks first. On
// instances whose data give exact integer sums, a narrow column whose terms
// are bounded well below 2^53 also gets bins tasks (chunks of its entries):
// the bound takes the largest weight the exactness check admits (2^16) on
// every term, each term's residual bound over the box (a row and its
// negation), and the cutoff term.
int build_jump_plan(chap_problem* p) {
  const int32_t n = p->n;
  const auto& raw = p->raw;
  // bound of |residual| of each original row over the box
  std::vector<double> mag;
  if (p->compact_ok) {
    mag.assign((size_t)p->m, 0.0);
    for (int32_t i = 0; i < p->m; ++i) {
      double v = std::fabs(raw.rhs[i]);
      for (int64_t e = raw.csr_row_ptr[i]; e < raw.csr_row_ptr[i + 1]; ++e) {
        const int32_t c = raw.csr_col[e];
        v += std::fabs(raw.csr_val[e]) * std::max(std::fabs(p->lb[c]), std::fabs(p->ub[c]));
      }
      mag[i] = v;
    }
  }
  const double wmax = 65536.0, limit = 4503599627370496.0;  // 2^52
  std::vector<JumpCol> cols;
  std::vector<JumpTask> tasks;
  std::vector<JumpBinTask> btasks;
  std::vector<std::vector<JumpBinTask>> range_tasks(kXcds);  // bins tasks by row range
  std::vector<int32_t> len;  // entries of each task's chunk
  std::vector<int32_t> cptr((size_t)n + 1, 0);  // internal CSC offsets
  for (int32_t q = 0; q < n; ++q) cptr[q + 1] = cptr[q] + p->col_entries[q];
  int32_t slot = 0, bslot = 0;
  int64_t nsingle = 0;
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
    bool bins = false;
    if (narrow && p->compact_ok) {
      double B = 0.0;
      for (int64_t e = raw.csc_col_ptr[j]; e < raw.csc_col_ptr[j + 1]; ++e) {
        const int32_t i = raw.csc_row[e];
        B += (raw.sense[i] == 'E' ? 2.0 : 1.0) * wmax * mag[i];
      }
      B += wmax * (2147483648.0 + std::fabs(p->obj[j]) * (double)kJumpNarrow);
      bins = B < limit;
    }
    JumpCol col{q, slot, tiles, chunks, 0, 0};
    if (bins && deg <= kJumpBinChunk) {
      // one wavefront scores the whole column and finishes it (slot -1)
      range_tasks[(size_t)(nsingle++ % kXcds)].push_back(JumpBinTask{q, cptr[q], cptr[q + 1], -1});
      col.bn = -1;
    } else if (bins) {
      // long columns: the entries of each eighth of the rows (one stretch of
      // the ascending internal CSC order) in chunks of kJumpBinChunk, so that
      // the row gathers of a range stay in one XCD's L2
      std::vector<int32_t> rows;
      for (int64_t k = raw.csc_col_ptr[j]; k < raw.csc_col_ptr[j + 1]; ++k)
        if (raw.csc_val[k] != 0.0) rows.push_back(raw.csc_row[k]);  // stored zeros are dropped
      std::sort(rows.begin(), rows.end());
      if ((int32_t)rows.size() != deg) return fail(CHAP_EINVAL, "chap_jump_values: column entries disagree");
      col.bfirst = bslot;
      int32_t e = 0;
      for (int r = 0; r < kXcds; ++r) {
        const int32_t hi = (int32_t)(((int64_t)p->m * (r + 1)) / kXcds);
        const int32_t e_end = (int32_t)(std::lower_bound(rows.begin(), rows.end(), hi) - rows.begin());
        for (int32_t b = e; b < e_end; b += kJumpBinChunk) {
          range_tasks[r].push_back(JumpBinTask{q, cptr[q] + b, cptr[q] + std::min(e_end, b + kJumpBinChunk), bslot});
          bslot += 1;
        }
        e = e_end;
      }
      col.bn = bslot - col.bfirst;
    }
    cols.push_back(col);
    for (int32_t t = 0; t < tiles; ++t)
      for (int32_t c = 0; c < chunks; ++c) {
        tasks.push_back(JumpTask{q, t, c, slot + t * chunks + c, bins ? 1 : 0});
        len.push_back(std::min(kJumpChunk, deg - c * kJumpChunk));
      }
    slot += tiles * chunks;
  }
  // bins tasks in workgroups of four from one row range, the workgroups
  // cycling through the ranges so that workgroup w (on XCD w mod 8) takes
  // range w mod 8; ranges that run out are padded with empty tasks
  {
    std::vector<size_t> pos(kXcds, 0);
    bool left = true;
    while (left) {
      left = false;
      for (int r = 0; r < kXcds; ++r) {
        for (int t = 0; t < 4; ++t) {
          if (pos[r] < range_tasks[r].size())
            btasks.push_back(range_tasks[r][pos[r]++]);
          else
            btasks.push_back(JumpBinTask{-1, 0, 0, 0});
        }
      }
      for (int r = 0; r < kXcds; ++r) left = left || pos[r] < range_tasks[r].size();
    }
    bool any = false;
    for (const JumpBinTask& t : btasks) any = any || t.q >= 0;
    if (!any) btasks.clear();
  }
  // tasks of columns without a bins form first (the only ones an exact call
  // runs), each part by chunk length; column records as [no bins form]
  // [chunked bins form] [finished by one bins task]
  std::vector<int32_t> order(tasks.size());
  for (size_t i = 0; i < order.size(); ++i) order[i] = (int32_t)i;
  std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t b) {
    if (tasks[a].bins != tasks[b].bins) return tasks[a].bins < tasks[b].bins;
    return len[a] > len[b];
  });
  int32_t n_plain_tasks = 0;
  for (const JumpTask& t : tasks) n_plain_tasks += t.bins ? 0 : 1;
  auto col_group = [](const JumpCol& c) { return c.bn == 0 ? 0 : (c.bn > 0 ? 1 : 2); };
  std::stable_sort(cols.begin(), cols.end(),
                   [&](const JumpCol& a, const JumpCol& b) { return col_group(a) < col_group(b); });
  int32_t n_plain_cols = 0, n_chunk_cols = 0;
  for (const JumpCol& c : cols) {
    n_plain_cols += col_group(c) == 0 ? 1 : 0;
    n_chunk_cols += col_group(c) == 1 ? 1 : 0;
  }
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
  if (!btasks.empty()) {
    JumpBinTask* db;
    CHAP_HIP(A.upload(&db, btasks));
    CHAP_HIP(A.alloc(&p->jump_bpart, (size_t)bslot * 2 * kWave));
    p->jump_btasks = db;
  }
  p->n_jump_tasks = (int32_t)sorted.size();
  p->n_jump_cols = (int32_t)cols.size();
  p->n_jump_plain_tasks = n_plain_tasks;
  p->n_jump_plain_cols = n_plain_cols;
  p->n_jump_chunk_cols = n_chunk_cols;
  p->n_jump_btasks = (int32_t)btasks.size();
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
  CHAP_HIP(launch_stage_x_plan(p->to_internal, d_x, p->bs_x, p->bs_xc, p->bs_state, epoch, p->bs_stage, s));
  // the state first (no violated rows are counted, so it reads no
  // residual), then the residuals with the compact copy and its check
  // (integer weights below 2^16)
  CHAP_HIP(launch_state_init(p->dev, p->bs_x, p->bs_rs, p->bs_state, p->bs_partial, p->bs_ticket, p->bs_objacc, 1,
                             0, p->obj_integral, cutoff_rhs, d_w + p->mp, 0, 0, s));
  CHAP_HIP(launch_residual_scatter(p->dev, p->d_nidx, p->d_pair, d_w, p->bs_x, p->bs_xc, p->bs_state, epoch,
                                   p->bs_rs, s, p->bs_grow));
  CHAP_HIP(hipEventRecord(p->jump_ev[0], s));
  CHAP_HIP(launch_jump(p->dev, p->bs_x, p->bs_rs, p->bs_state, p->bs_grow, p->obj_fast, p->jump_tasks,
                       p->n_jump_tasks, p->n_jump_plain_tasks, p->jump_btasks, p->n_jump_btasks, p->jump_cols,
                       p->n_jump_cols, p->n_jump_plain_cols, p->n_jump_chunk_cols, p->jump_part,
                       p->jump_bpart, p->bs_xhat, p->bs_s, s));
  CHAP_HIP(hipEventRecord(p->jump_ev[1], s));
  CHAP_HIP(launch_gather2_plan(p->to_caller, p->bs_xhat, p->bs_s, d_jump, d_score, p->bs_stage, s));
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
