// chap_best_shift_noalloc: the single best-shift pass for callers that cannot
// allocate device memory (code under HIP graph capture, serving loops,
// harnesses that forbid hipMalloc). Every per-call buffer of the pass (the
// point in internal order and its byte copy, row states and their compact
// copy, walk state, set-up partials, the exact objective sum, staged records,
// long-column partials and sort scratch, the launch record) is carved from
// one file-scope device array, `scratch`, of kNoAllocBytes per GPU; the
// kernels are the ones chap_best_shift runs, launched one by one on the
// caller's stream (no graph, no side streams, no events).

#include <mutex>
#include <string>

#include "chap_internal.h"

using namespace chap;

namespace {

constexpr size_t kNoAllocBytes = (size_t)64 << 20;
constexpr int kMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];

std::mutex g_mu;
void* g_scratch[kMaxDevices] = {};   // device address of `scratch` on each device
uint32_t g_epoch[kMaxDevices] = {};  // call counter per device (byte copies of x)

// The launch record of one pass: the walk context and the block prefix
// table of every kernel slot (one walk: 0 and its block count).
struct LaunchRecord {
  WalkCtx c;
  int32_t off[KS_COUNT][2];
};

// Writes the launch record into scratch and clears the set-up ticket.
__global__ __launch_bounds__(256) void k_put_record(LaunchRecord r, LaunchRecord* dst, uint32_t* ticket) {
  static_assert(sizeof(LaunchRecord) % 4 == 0, "copied as 32-bit words");
  const uint32_t* src = reinterpret_cast<const uint32_t*>(&r);
  uint32_t* out = reinterpret_cast<uint32_t*>(dst);
  for (int i = threadIdx.x; i < (int)(sizeof(LaunchRecord) / 4); i += blockDim.x) out[i] = src[i];
  if (threadIdx.x == 0) *ticket = 0u;
}

// Hands out 256-byte aligned pieces of [base, base + cap); used + size
// report what a call needs, whether or not it fits.
struct Carve {
  unsigned char* base;
  size_t cap;
  size_t used = 0;
  template <typename T>
  T* take(size_t count) {
    const size_t at = (used + 255) & ~(size_t)255;
    used = at + std::max<size_t>(count, 1) * sizeof(T);
    return used <= cap ? reinterpret_cast<T*>(base + at) : nullptr;
  }
};

int scratch_of_device(int dev, void** out) {
  if (dev < 0 || dev >= kMaxDevices) return fail(CHAP_EINVAL, "chap_best_shift_noalloc: device index out of range");
  std::lock_guard<std::mutex> lock(g_mu);
  if (!g_scratch[dev]) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
      return fail(CHAP_EHIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    g_scratch[dev] = ptr;
  }
  *out = g_scratch[dev];
  return CHAP_OK;
}

}  // namespace

extern "C" {

int chap_best_shift_noalloc(chap_problem* p, const double* d_x, const float* d_w, double cutoff_rhs,
                            double* d_shift, double* d_score, void* hip_stream) {
  if (!p) return fail(CHAP_EINVAL, "chap_best_shift_noalloc: null problem");
  if (p->n > 0 && (!d_x || !d_shift || !d_score))
    return fail(CHAP_EINVAL, "chap_best_shift_noalloc: null device array");
  if (!d_w) return fail(CHAP_EINVAL, "chap_best_shift_noalloc: null weights");
  if (std::isnan(cutoff_rhs)) return fail(CHAP_EINVAL, "chap_best_shift_noalloc: cutoff_rhs is NaN");
  int dev = 0;
  CHAP_HIP(hipGetDevice(&dev));
  if (dev != p->device)
    return fail(CHAP_EINVAL, "chap_best_shift_noalloc: the problem lives on device " + std::to_string(p->device) +
                                 ", device " + std::to_string(dev) + " is current");
  void* base = nullptr;
  int rc = scratch_of_device(dev, &base);
  if (rc != CHAP_OK) return rc;
  const int32_t n = p->n, m = p->m;
  const PassPlan& plan = p->plan;
  Carve cv{(unsigned char*)base, kNoAllocBytes};
  WalkCtx c{};
  c.P = p->dev;
  c.plan = plan;
  c.x = cv.take<double>((size_t)n);
  c.xhat = cv.take<double>((size_t)n);
  c.s = cv.take<double>((size_t)n);
  c.rs = cv.take<RowState>((size_t)m);
  c.grow = p->compact_ok ? cv.take<GatherRow>((size_t)m) : nullptr;
  c.st = cv.take<WalkState>(1);
  c.partials = cv.take<ChunkPartial>((size_t)plan.n_partials);
  c.long_pos = cv.take<double>((size_t)plan.long_scratch);
  c.long_delta = cv.take<double>((size_t)plan.long_scratch);
  c.long_marker = cv.take<int32_t>((size_t)plan.long_scratch);
  c.stage_rec = cv.take<uint64_t>((size_t)plan.n_stage_ent);
  int8_t* xc = p->x_small ? cv.take<int8_t>((size_t)n) : nullptr;
  double* partial = cv.take<double>(kInitPartial);
  uint32_t* ticket = cv.take<uint32_t>(1);
  long long* objacc = p->obj_fast ? nullptr : cv.take<long long>(kExactLimbs);
  LaunchRecord* rec = cv.take<LaunchRecord>(1);
  if (cv.used > cv.cap)
    return fail(CHAP_EINVAL, "chap_best_shift_noalloc: this problem needs " + std::to_string(cv.used) +
                                 " bytes of scratch, more than the " + std::to_string(kNoAllocBytes) +
                                 " the entry point holds per device (use chap_best_shift)");
  LaunchRecord r{};
  r.c = c;
  BatchLaunch L;
  L.nw = 1;
  L.walks = &rec->c;
  for (int k = 0; k < KS_COUNT; ++k) {
    r.off[k][0] = 0;
    r.off[k][1] = kernel_blocks(c, k);
    L.off[k] = rec->off[k];
    L.total[k] = r.off[k][1];
    L.grid[k] = r.off[k][1];
  }
  L.compact = p->compact_ok ? 2 : 0;
  hipStream_t s = (hipStream_t)hip_stream;
  uint32_t epoch;
  {
    std::lock_guard<std::mutex> lock(g_mu);
    epoch = ++g_epoch[dev] == 0 ? ++g_epoch[dev] : g_epoch[dev];  // never 0
  }
  hipLaunchKernelGGL(k_put_record, dim3(1), dim3(256), 0, s, r, rec, ticket);
  CHAP_HIP(hipGetLastError());
  CHAP_HIP(launch_stage_x(p->dev.perm, d_x, c.x, xc, c.st, epoch, n, s));
  CHAP_HIP(launch_residual_scatter(p->dev, p->d_nidx, p->d_pair, d_w, c.x, xc, c.st, epoch, c.rs, s));
  CHAP_HIP(launch_state_init(p->dev, c.x, c.rs, c.st, partial, ticket, objacc, 1, 0, p->obj_integral, cutoff_rhs,
                             d_w + p->mp, 0, 0, s));
  if (c.grow) CHAP_HIP(launch_fill_compact_checked(c.rs, c.grow, c.st, m, s));
  if (n > 0) CHAP_HIP(launch_pass(L, s, nullptr, false));
  CHAP_HIP(launch_gather2(p->d_inv, c.xhat, c.s, d_shift, d_score, n, s));
  return CHAP_OK;
}

size_t chap_best_shift_noalloc_max_bytes(void) { return kNoAllocBytes; }

}  // extern "C"
