// C ABI of the learned candidate proposal: the learned tabu walk and the
// materialised network inputs of a point.

#include <cmath>
#include <cstring>
#include <memory>
#include <string>
#include <vector>

#include "chap_internal.h"

using namespace chap;

namespace {

int check_options(const chap_learned_options& o) {
  if (o.topk <= 0 || o.full_every <= 0 || o.train_steps < 0 || o.train_pairs <= 0 || !(o.lr > 0.0f) ||
      !std::isfinite(o.lr) || o.log_pairs < 0 || o.refresh_every <= 0)
    return fail(CHAP_EINVAL, "chap_learned_run: invalid options");
  if (o.topk > kTopkMax || o.train_pairs > kTopkMax)
    return fail(CHAP_EINVAL, "chap_learned_run: topk and train_pairs must be at most " + std::to_string(kTopkMax));
  return CHAP_OK;
}

// Device buffers of one learned walk.
int build_learn_ctx(const chap_problem* p, const chap_learned_options& o, int64_t iters, DeviceArena& A,
                    LearnCtx& L) {
  const int32_t n = p->n;
  L = LearnCtx{};
  std::vector<int32_t> elig;
  for (int32_t q = 0; q < n; ++q)
    if (p->sub_cls[q] != SUB_NONE) elig.push_back(q);
  uint8_t* d_cls;
  int32_t* d_elig;
  CHAP_HIP(A.upload(&d_cls, p->sub_cls));
  CHAP_HIP(A.upload(&d_elig, elig));
  L.cls = d_cls;
  L.elig_list = d_elig;
  L.n_elig = (int32_t)elig.size();
  L.mp = p->mp;
  L.c_max = p->c_max;
  // refresh work: short columns by lane groups, long ones in chunks
  {
    std::vector<int32_t> shorts;
    std::vector<ChunkTask> chunks;
    std::vector<ChunkCol> cols;
    std::vector<int32_t> cptr((size_t)n + 1, 0);  // internal CSC offsets
    for (int32_t q = 0; q < n; ++q) cptr[q + 1] = cptr[q] + p->col_entries[q];
    for (int32_t q = 0; q < n; ++q) {
      if (p->sub_cls[q] == SUB_NONE) continue;
      const int32_t e = p->col_entries[q];
      if (e <= kRefreshShort) {
        shorts.push_back(q);
        continue;
      }
      ChunkCol cc{q, (int32_t)chunks.size(), 0};
      for (int32_t b = cptr[q]; b < cptr[q + 1]; b += kRefreshChunk) {
        ChunkTask t{q, b, std::min(cptr[q + 1], b + kRefreshChunk), (int32_t)chunks.size(), 0};
        chunks.push_back(t);
      }
      cc.nparts = (int32_t)chunks.size() - cc.first;
      cols.push_back(cc);
    }
    int32_t* d_short;
    ChunkTask* d_chunks;
    ChunkCol* d_cols;
    CHAP_HIP(A.upload(&d_short, shorts));
    CHAP_HIP(A.upload(&d_chunks, chunks));
    CHAP_HIP(A.upload(&d_cols, cols));
    L.ref_short = d_short;
    L.n_ref_short = (int32_t)shorts.size();
    L.ref_chunks = d_chunks;
    L.n_ref_chunks = (int32_t)chunks.size();
    L.ref_cols = d_cols;
    L.n_ref_cols = (int32_t)cols.size();
    CHAP_HIP(A.alloc(&L.ref_parts, std::max<size_t>(chunks.size(), 1)));
  }
  CHAP_HIP(A.alloc(&L.feat, (size_t)n * 16));
  CHAP_HIP(A.alloc(&L.moves, (size_t)n));
  CHAP_HIP(A.alloc(&L.xhat_last, (size_t)n));
  CHAP_HIP(A.alloc(&L.keys[0], (size_t)n));
  CHAP_HIP(A.alloc(&L.keys[1], (size_t)n));
  CHAP_HIP(A.alloc(&L.hist, (size_t)2 * 3 * kRadixBins));
  CHAP_HIP(hipMemset(L.hist, 0, sizeof(uint32_t) * 2 * 3 * kRadixBins));
  L.nwg = std::max<int32_t>(1, (n + kTopkChunk - 1) / kTopkChunk);
  CHAP_HIP(A.alloc(&L.wg_cnt, (size_t)2 * L.nwg * 2));
  L.K[0] = o.topk;
  L.K[1] = o.train_pairs;
  CHAP_HIP(A.alloc(&L.sel[0], (size_t)L.K[0]));
  CHAP_HIP(A.alloc(&L.sel[1], (size_t)L.K[1]));
  // subset-pass chunks: at most sum over the selected columns of
  // ceil(entries / kSubsetChunk) <= nnz / kSubsetChunk + K
  L.sub_cap = (int32_t)std::min<int64_t>(INT32_MAX, p->nnz / kSubsetChunk + L.K[0] + 1);
  CHAP_HIP(A.alloc(&L.sub_off, (size_t)L.K[0] + 1));
  CHAP_HIP(A.alloc(&L.sub_parts, (size_t)L.sub_cap));
  L.T = o.train_pairs;
  CHAP_HIP(A.alloc(&L.pair_feat, (size_t)2 * L.T * 16));
  CHAP_HIP(A.alloc(&L.pair_tgt, (size_t)2 * L.T));
  if (o.log_pairs > 0) {
    CHAP_HIP(A.alloc(&L.log_feat, (size_t)o.log_pairs * 16));
    CHAP_HIP(A.alloc(&L.log_tgt, (size_t)o.log_pairs));
    L.log_cap = o.log_pairs;
  }
  if (o.log_sets) {
    L.set_log_cap = std::max<int64_t>(1, iters * (int64_t)std::min<int32_t>(o.topk, std::max(L.n_elig, 1)));
    CHAP_HIP(A.alloc(&L.set_log, (size_t)L.set_log_cap));
    CHAP_HIP(A.alloc(&L.set_off, (size_t)iters + 1));
    CHAP_HIP(hipMemset(L.set_off, 0, sizeof(int64_t) * ((size_t)iters + 1)));
  }
  L.full_every = o.full_every;
  L.seed = o.train_seed;
  CHAP_HIP(A.alloc(&L.ls, 1));
  LearnState ls{};
  ls.train_active = 1;
  CHAP_HIP(hipMemcpy(L.ls, &ls, sizeof(LearnState), hipMemcpyHostToDevice));
  return CHAP_OK;
}

hipError_t capture_block(const BatchLaunch& BL, const WalkCtx* C, const LearnCtx* L, const LearnCtx& Lh,
                         const ModelDev& M, const chap_learned_options& o, int32_t n, int has_general,
                         hipStream_t s, const PassStreams* ps) {
  hipError_t e = launch_learn_begin(C, L, s);
  // full evaluation: exact pass, judge set, training, move, row refresh
  if (e == hipSuccess) e = launch_pass(BL, s, ps);
  if (e == hipSuccess && Lh.n_elig > 0) e = launch_learn_propose(C, L, Lh, M, n, 1, s);
  if (e == hipSuccess && Lh.n_elig > 0) e = launch_learn_train(C, L, Lh, M, n, o.train_steps, o.lr, s);
  if (e == hipSuccess) e = launch_walk_choose(BL, s);
  if (e == hipSuccess) e = launch_learn_judge(C, L, s);
  if (e == hipSuccess) e = launch_walk_apply(BL, s);
  if (e == hipSuccess) e = launch_walk_finish(BL, s);
  if (e == hipSuccess) e = launch_learn_refresh(C, L, Lh, s);
  // proposal iterations: a new set from the network every refresh_every of
  // them (the scoring kernel also copies a pending incumbent); otherwise the
  // last set is logged again and the pending copy runs on its own
  for (int32_t t = 1; t < o.full_every && e == hipSuccess; ++t) {
    const bool fresh = (t - 1) % o.refresh_every == 0;
    if (Lh.n_elig > 0 && fresh) {
      e = launch_learn_propose(C, L, Lh, M, n, 0, s);
    } else {
      e = launch_copy_best_batch(BL, s);
      if (e == hipSuccess && Lh.n_elig > 0) e = launch_learn_keep_set(C, L, s);
    }
    if (e == hipSuccess && Lh.n_elig > 0) e = launch_subset_pass(C, L, Lh, has_general, BL.compact, s);
    if (e == hipSuccess) e = launch_subset_select(C, L, s);
    if (e == hipSuccess) e = launch_walk_apply(BL, s);
    if (e == hipSuccess) e = launch_walk_finish(BL, s);
  }
  return e;
}

}  // namespace

extern "C" {

void chap_learned_options_default(chap_learned_options* o) {
  if (!o) return;
  o->topk = 1024;
  o->full_every = 64;
  o->train_steps = 0;
  o->train_pairs = 1024;
  o->lr = 1e-3f;
  o->log_sets = 0;
  o->log_pairs = 0;
  o->train_seed = 0;
  o->refresh_every = 1;
}

int chap_learned_run(chap_problem* p, chap_model* m, const chap_learned_options* opt, int64_t iters, int32_t tenure,
                     uint64_t seed, const double* x0, chap_run** out, void* hip_stream) {
  if (!p || !m || !out) return fail(CHAP_EINVAL, "chap_learned_run: null argument");
  chap_learned_options o;
  chap_learned_options_default(&o);
  if (opt) o = *opt;
  int rc = check_options(o);
  if (rc != CHAP_OK) return rc;
  if (iters < 0 || tenure < 0 || iters + (int64_t)tenure >= (int64_t)INT32_MAX)
    return fail(CHAP_EINVAL, "iters and tenure must be >= 0 with iters + tenure < 2^31");
  if (p->device != m->device) return fail(CHAP_EINVAL, "chap_learned_run: problem and model on different devices");
  const int32_t n = p->n;
  DeviceArena A;
  double* partial;
  uint32_t* ticket;
  CHAP_HIP(A.alloc(&partial, kInitPartial));
  CHAP_HIP(A.alloc(&ticket, 1));
  CHAP_HIP(hipMemset(ticket, 0, sizeof(uint32_t)));
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
  CHAP_HIP(hipEventRecord(e_user, (hipStream_t)hip_stream));
  CHAP_HIP(hipStreamWaitEvent(s, e_user, 0));
  WalkCtx c;
  const int compact = compact_walks({WalkSpec{p, seed, x0}}, iters);
  rc = prepare_walk(WalkSpec{p, seed, x0}, iters, tenure, A, c, partial, ticket, s, compact);
  if (rc != CHAP_OK) return rc;
  BatchLaunch BL;
  std::vector<WalkCtx> one{c};
  CHAP_HIP(build_launch(A, one, &BL, nullptr));
  BL.compact = compact;
  LearnCtx Lh;
  rc = build_learn_ctx(p, o, iters, A, Lh);
  if (rc != CHAP_OK) return rc;
  LearnCtx* dL;
  CHAP_HIP(A.upload(&dL, std::vector<LearnCtx>{Lh}));
  const WalkCtx* dC = BL.walks;
  // initial rows: s_last = 0, xhat_last = x
  if (n > 0) {
    CHAP_HIP(hipMemsetAsync(c.s, 0, sizeof(double) * (size_t)n, s));
    CHAP_HIP(hipMemcpyAsync(c.xhat, c.x, sizeof(double) * (size_t)n, hipMemcpyDeviceToDevice, s));
    CHAP_HIP(launch_learn_init(dC, dL, Lh, n, nullptr, nullptr, s));
    CHAP_HIP(launch_learn_refresh(dC, dL, Lh, s));
  }
  double ms_total = 0.0;
  if (iters > 0) {
    hipGraph_t graph;
    CHAP_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
    int has_general = 0;
    for (uint8_t c : p->sub_cls) has_general |= (c == SUB_GENERAL) ? 1 : 0;
    const hipError_t cap_err = capture_block(BL, dC, dL, Lh, m->dev, o, n, has_general, s, &sg.ps);
    const hipError_t end_err = hipStreamEndCapture(s, &graph);
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
    // every block of iterations advances the walk by at least one iteration
    int64_t k = 0;
    while (k < iters) {
      const int64_t k_before = k;
      const int64_t launches = (iters - k + o.full_every - 1) / o.full_every;
      CHAP_HIP(hipEventRecord(e0, s));
      for (int64_t q = 0; q < launches; ++q) CHAP_HIP(hipGraphLaunch(exec, s));
      CHAP_HIP(hipEventRecord(e1, s));
      CHAP_HIP(hipStreamSynchronize(s));
      float ms = 0.0f;
      CHAP_HIP(hipEventElapsedTime(&ms, e0, e1));
      ms_total += ms;
      CHAP_HIP(hipMemcpy(&k, &c.st->k, sizeof(int64_t), hipMemcpyDeviceToHost));
      if (k <= k_before) return fail(CHAP_ESTATE, "chap_learned_run: a block of iterations made no progress");
    }
  }
  CHAP_HIP(launch_copy_best_batch(BL, s));
  CHAP_HIP(hipStreamSynchronize(s));
  std::unique_ptr<chap_run> R(new chap_run());
  rc = collect_walk(p, c, iters, ms_total, R.get());
  if (rc != CHAP_OK) return rc;
  LearnState ls;
  CHAP_HIP(hipMemcpy(&ls, Lh.ls, sizeof(LearnState), hipMemcpyDeviceToHost));
  R->evals = ls.evals;
  R->hits = ls.hits;
  R->stalls = ls.stalls;
  if (Lh.set_off) {
    R->set_off.resize((size_t)iters + 1);
    CHAP_HIP(hipMemcpy(R->set_off.data(), Lh.set_off, sizeof(int64_t) * ((size_t)iters + 1), hipMemcpyDeviceToHost));
    R->sets.resize((size_t)ls.set_pos);
    if (ls.set_pos > 0)
      CHAP_HIP(hipMemcpy(R->sets.data(), Lh.set_log, sizeof(int32_t) * (size_t)ls.set_pos, hipMemcpyDeviceToHost));
  }
  if (Lh.log_feat && ls.logged > 0) {
    R->pair_feat.resize((size_t)ls.logged * 16);
    R->pair_tgt.resize((size_t)ls.logged);
    CHAP_HIP(hipMemcpy(R->pair_feat.data(), Lh.log_feat, sizeof(uint16_t) * (size_t)ls.logged * 16,
                       hipMemcpyDeviceToHost));
    CHAP_HIP(hipMemcpy(R->pair_tgt.data(), Lh.log_tgt, sizeof(float) * (size_t)ls.logged, hipMemcpyDeviceToHost));
  }
  *out = R.release();
  return CHAP_OK;
}

int chap_run_learned_stats(const chap_run* r, int64_t* evals, int64_t* hits, int64_t* stalls) {
  if (!r) return fail(CHAP_EINVAL, "chap_run_learned_stats: null run");
  if (evals) *evals = r->evals;
  if (hits) *hits = r->hits;
  if (stalls) *stalls = r->stalls;
  return CHAP_OK;
}

int chap_run_rescored(const chap_run* r, int64_t* iters) {
  if (!r || !iters) return fail(CHAP_EINVAL, "chap_run_rescored: null argument");
  *iters = r->st_end.aff_iters;
  return CHAP_OK;
}

int chap_run_proposals(const chap_run* r, const int32_t** sets, const int64_t** offsets, int64_t* iters) {
  if (!r || !sets || !offsets || !iters) return fail(CHAP_EINVAL, "chap_run_proposals: null argument");
  *sets = r->sets.data();
  *offsets = r->set_off.data();
  *iters = r->set_off.empty() ? 0 : (int64_t)r->set_off.size() - 1;
  return CHAP_OK;
}

int chap_run_pairs(const chap_run* r, const uint16_t** feat, const float** target, int64_t* count) {
  if (!r || !feat || !target || !count) return fail(CHAP_EINVAL, "chap_run_pairs: null argument");
  *feat = r->pair_feat.data();
  *target = r->pair_tgt.data();
  *count = (int64_t)r->pair_tgt.size();
  return CHAP_OK;
}

int chap_features(chap_problem* p, const double* d_x, const float* d_w, double cutoff_rhs, const double* d_s_last,
                  const double* d_xhat_last, const int32_t* d_last_move, const int32_t* d_moves, int64_t k,
                  int64_t k_last_full, uint16_t* d_out, void* hip_stream) {
  if (!p || (p->n > 0 && (!d_x || !d_s_last || !d_xhat_last || !d_last_move || !d_moves || !d_out)) || !d_w)
    return fail(CHAP_EINVAL, "chap_features: null argument");
  if (std::isnan(cutoff_rhs) || k < 0 || k_last_full > k || k > INT32_MAX)
    return fail(CHAP_EINVAL, "chap_features: bad iteration or cutoff");
  const int32_t n = p->n;
  if (n == 0) return CHAP_OK;
  hipStream_t s = (hipStream_t)hip_stream;
  DeviceArena A;
  WalkCtx c{};
  c.P = p->dev;
  c.plan = p->plan;
  CHAP_HIP(A.alloc(&c.x, (size_t)n));
  CHAP_HIP(A.alloc(&c.s, (size_t)n));
  CHAP_HIP(A.alloc(&c.xhat, (size_t)n));
  CHAP_HIP(A.alloc(&c.rs, (size_t)p->m));
  CHAP_HIP(A.alloc(&c.st, 1));
  double* partial;
  uint32_t* ticket;
  CHAP_HIP(A.alloc(&partial, kInitPartial));
  CHAP_HIP(A.alloc(&ticket, 1));
  CHAP_HIP(hipMemsetAsync(ticket, 0, sizeof(uint32_t), s));
  CHAP_HIP(launch_gather(p->dev.perm, d_x, c.x, n, s));
  CHAP_HIP(launch_gather(p->dev.perm, d_s_last, c.s, n, s));
  CHAP_HIP(launch_gather(p->dev.perm, d_xhat_last, c.xhat, n, s));
  CHAP_HIP(launch_residual_scatter(p->dev, p->d_nidx, p->d_pair, d_w, c.x, nullptr, nullptr, 0u, c.rs, s));
  if (!p->obj_fast) CHAP_HIP(A.alloc(&c.objacc, (size_t)kExactLimbs));
  CHAP_HIP(launch_state_init(p->dev, c.x, c.rs, c.st, partial, ticket, c.objacc, 1, 0, p->obj_integral, cutoff_rhs,
                             d_w + p->mp, 0, 1, s));
  chap_learned_options o;
  chap_learned_options_default(&o);
  o.log_pairs = 0;
  o.log_sets = 0;
  LearnCtx Lh;
  int rc = build_learn_ctx(p, o, 1, A, Lh);
  if (rc != CHAP_OK) return rc;
  WalkCtx* dC;
  LearnCtx* dL;
  CHAP_HIP(A.upload(&dC, std::vector<WalkCtx>{c}));
  CHAP_HIP(A.upload(&dL, std::vector<LearnCtx>{Lh}));
  CHAP_HIP(launch_learn_init(dC, dL, Lh, n, d_last_move, d_moves, s));
  CHAP_HIP(launch_learn_refresh(dC, dL, Lh, s));
  CHAP_HIP(launch_learn_features_out(dC, dL, n, k, k_last_full, d_out, s));
  CHAP_HIP(hipStreamSynchronize(s));
  return CHAP_OK;
}

}  // extern "C"
