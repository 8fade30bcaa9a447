// Host side of libuot.so: argument validation, workspace layout, and the launch sequence of
// the plain and translation-invariant Sinkhorn solvers, the dual value, plan application
// and the envelope backward. Every entry point is extern "C" and declared in uot.h.
#include <hip/hip_runtime.h>

#include <atomic>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/uot.h"
#include "uot_batched.h"
#include "uot_internal.h"

// Workspace of uot_backward_noalloc on each device (see noalloc_scratch below).
static __device__ __align__(256) unsigned char scratch[UOT_NOALLOC_BYTES];

namespace uot {
namespace {

thread_local std::string g_last_error;

uot_status fail(uot_status s, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return s;
}

#define UOT_HIP(expr)                                                                    \
  do {                                                                                   \
    hipError_t e_ = (expr);                                                              \
    if (e_ != hipSuccess) return fail(UOT_ERR_HIP, "%s: %s", #expr, hipGetErrorString(e_)); \
  } while (0)

#define UOT_TRY(expr)                    \
  do {                                   \
    uot_status r_ = (expr);              \
    if (r_ != UOT_OK) return r_;         \
  } while (0)

constexpr size_t kAlign = 256;
size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

bool finite_pos(double v) { return std::isfinite(v) && v > 0.0; }

// How kernels form C: the cost mode of the apply kernels.
int mode_of(const uot_cost *c) {
  if (c->kind == UOT_COST_DENSE) return kDense;
  return c->p == 2.0 ? kSqEuc : kPower;
}

// Mode of the source records and softmin kernels of the solver and the dual value.
int rec_mode_of(const uot_cost *c) {
  return points_record_mode(mode_of(c), c->kind == UOT_COST_POINTS ? c->d : 0);
}

uot_status check_cost(const uot_cost *c) {
  if (c == nullptr) return fail(UOT_ERR_INVALID, "cost is NULL");
  if (c->n < 1 || c->m < 1) return fail(UOT_ERR_INVALID, "n and m must be >= 1 (got %d, %d)", c->n, c->m);
  if (c->kind == UOT_COST_DENSE) {
    if (c->C == nullptr) return fail(UOT_ERR_INVALID, "dense cost with C = NULL");
    if (c->ldc < c->m) return fail(UOT_ERR_INVALID, "ldc (%lld) < m (%d)", (long long)c->ldc, c->m);
  } else if (c->kind == UOT_COST_POINTS) {
    if (c->x == nullptr || c->y == nullptr) return fail(UOT_ERR_INVALID, "points cost with NULL x or y");
    if (c->d < 1 || c->d > kMaxDim) return fail(UOT_ERR_INVALID, "point dimension d=%d not in [1, %d]", c->d, kMaxDim);
    if (!std::isfinite(c->p) || c->p < 1.0) return fail(UOT_ERR_INVALID, "exponent p=%g must be finite and >= 1", c->p);
  } else {
    return fail(UOT_ERR_INVALID, "unknown cost kind %d", c->kind);
  }
  return UOT_OK;
}

// A pointer the GPU can read: device or managed memory, or host memory mapped to the device.
uot_status check_device_ptr(const void *p, const char *name) {
  if (p == nullptr) return fail(UOT_ERR_INVALID, "%s is NULL", name);
  hipPointerAttribute_t attr;
  if (hipPointerGetAttributes(&attr, p) != hipSuccess) {
    (void)hipGetLastError();
    return fail(UOT_ERR_INVALID, "%s is not a HIP device pointer", name);
  }
  if (attr.type == hipMemoryTypeHost && attr.devicePointer == nullptr)
    return fail(UOT_ERR_INVALID, "%s is host memory not mapped to the device", name);
  if (attr.type == hipMemoryTypeUnregistered)
    return fail(UOT_ERR_INVALID, "%s is not a HIP device pointer", name);
  return UOT_OK;
}

uot_status check_cost_ptrs(const uot_cost *c) {
  uot_status s;
  if (c->kind == UOT_COST_DENSE) return check_device_ptr(c->C, "C");
  if ((s = check_device_ptr(c->x, "x")) != UOT_OK) return s;
  return check_device_ptr(c->y, "y");
}

// ---------------------------------------------------------------------------------------
// Launch shapes and workspace layout
// ---------------------------------------------------------------------------------------
constexpr int kMaxSplits = 64;          // cap on source splits (bounds the partials buffer)
constexpr int kDefaultResidentBlocks = 2048;

struct Split {
  int len = 1, n = 1;
};

// Number of CUs of the current device (cached; a default when no device is visible).
int device_cus() {
  static int cus = -1;
  if (cus < 0) {
    int dev = 0;
    hipDeviceProp_t p;
    if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&p, dev) == hipSuccess &&
        p.multiProcessorCount > 0)
      cus = p.multiProcessorCount;
    else
      cus = 0;
    (void)hipGetLastError();
  }
  return cus;
}

// Splits of `ns` sources over `tiles` target tiles: as many splits as fill one round of
// resident blocks (capacity = blocks per CU x CUs), capped at kMaxSplits and by a minimum
// split length; split lengths are multiples of `align`.
Split make_split(int ns, int tiles, int min_len, int align, int capacity,
                 int max_splits = kMaxSplits) {
  Split s;
  if (capacity <= 0) capacity = kDefaultResidentBlocks;
  int want = capacity / tiles;
  const int maxn = (ns + min_len - 1) / min_len;
  if (want > maxn) want = maxn;
  if (want > max_splits) want = max_splits;
  if (want < 1) want = 1;
  int len = (ns + want - 1) / want;
  len = (len + align - 1) / align * align;
  s.len = len;
  s.n = (ns + len - 1) / len;
  return s;
}

// Softmin launch shape for a half-step with `nt` targets and `ns` sources.
struct HalfShape {
  Split split;
  bool rows_kernel = false;  // dense, targets are rows (single split)
  int nb_combine = 1;
};

// ---------------------------------------------------------------------------------------
// Kernel-shape autotuner. The split count of a half-step's softmin starts from one round of
// resident blocks (make_split); the first solve of a shape of at least kTuneMinEntries
// entries times the softmin on its own first half-step with that capacity scaled by each of
// kTuneMults and keeps the fastest for the process (per device, record mode, dimension
// bucket, target and source counts, and side). Later calls, and the dual value, take the
// cached shape. Split counts only change the order in which partial sums merge.
// ---------------------------------------------------------------------------------------
constexpr double kTuneMinEntries = 1048576.0;
constexpr double kTuneMults[] = {0.5, 0.75, 1.0, 1.5, 2.0};
typedef std::tuple<int, int, int, int, int, int> TuneKey;  // device, mode, bucket, nt, ns, rows
std::mutex g_tune_mu;
std::map<TuneKey, double> g_tune_cache;
std::atomic<int> g_autotune{1};

TuneKey tune_key(int mode, int d, int nt, int ns, bool rows) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) {
    (void)hipGetLastError();
    dev = 0;
  }
  return TuneKey(dev, mode, mode == kDense ? 0 : dim_bucket(d), nt, ns, rows ? 1 : 0);
}

// Cached capacity multiplier of a shape (1 when none is cached or tuning is off).
double tuned_mult(int mode, int d, int nt, int ns, bool rows) {
  if (!g_autotune.load()) return 1.0;
  const TuneKey key = tune_key(mode, d, nt, ns, rows);
  std::lock_guard<std::mutex> lk(g_tune_mu);
  const auto it = g_tune_cache.find(key);
  return it == g_tune_cache.end() ? 1.0 : it->second;
}

HalfShape half_shape(int mode, int d, int nt, int ns, bool targets_are_rows,
                     double cap_mult = -1.0) {
  HalfShape h;
  const int cus = device_cus();
  if (cap_mult < 0.0) cap_mult = tuned_mult(mode, d, nt, ns, targets_are_rows);
  auto scaled = [&](int capacity) {
    const int c = (int)(capacity * cap_mult + 0.5);
    return c > 0 ? c : 1;
  };
  if (mode == kDense) {
    if (targets_are_rows) {
      h.rows_kernel = true;
      h.split.len = ns;
      h.split.n = 1;
    } else {
      const int tiles = (nt + dense_cols_per_block() - 1) / dense_cols_per_block();
      h.split = make_split(ns, tiles, 64, 8, scaled(cus > 0 ? 8 * cus : kDefaultResidentBlocks));
    }
  } else {
    const int tpb = points_targets_per_block(mode, d);
    const int tiles = (nt + tpb - 1) / tpb;
    const int per_cu = points_blocks_per_cu(mode, d);
    h.split = make_split(ns, tiles, 64, points_split_align(mode, d),
                         scaled((cus > 0 && per_cu > 0) ? per_cu * cus : kDefaultResidentBlocks));
  }
  h.nb_combine = combine_blocks(nt);
  return h;
}

struct Layout {
  size_t state = 0, pot_x = 0, pot_y = 0, rec_x = 0, rec_y = 0, part = 0, bparts = 0;
  size_t dual = 0, scratch = 0, total = 0;
  size_t center = 0;  // centring partials (kCenterBlocks * kMaxDim doubles)
  size_t grad_rec = 0, grad_part = 0, masses = 0;  // plan marginals and the backward
  size_t hist = 0, taus = 0, gram = 0, acc_c = 0;  // Anderson
  int64_t ldh = 0;
  HalfShape g, f;  // g-step: targets y (columns), sources x; f-step: targets x (rows), sources y
};

Layout make_layout(const uot_cost *c, int which, int mode_override = -1) {
  Layout L;
  const int mode = mode_override >= 0 ? mode_override : rec_mode_of(c);
  const int d = c->kind == UOT_COST_POINTS ? c->d : 0;
  const int n = c->n, m = c->m;
  // records sized for every p = 2 record form, so the size does not depend on the
  // points-kernel setting
  int stride = rec_stride_for(mode, d);
  if (mode_of(c) == kSqEuc && dim_bucket(d) <= kMxMaxDim) {
    const int a = rec_stride_for(kSqEuc, d), b = rec_stride_for(kSqEucMx, d);
    stride = a > b ? a : b;
  }
  L.g = half_shape(mode, d, m, n, false);
  L.f = half_shape(mode, d, n, m, true);
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off = align_up(off + bytes);
    return o;
  };
  L.state = take(sizeof(SolveState));
  L.center = take((size_t)kCenterBlocks * kMaxDim * sizeof(double));
  const int nmax = n > m ? n : m;
  if (which == UOT_WS_PLAN || which == UOT_WS_BACKWARD) {
    // the plan and the backward take no solver records: apply partials (plan with V), and
    // for the one-pass marginals and gradients the source records of either side (points:
    // doubles, grad_rec_stride; stored cost: one float) and split partials (gradient
    // accumulators, or the stored-cost softmin partials with up to kMaxSplits splits)
    if (which == UOT_WS_PLAN) {
      const size_t a = apply_partial_bytes(n, m), b = apply_partial_bytes(m, n);
      L.scratch = take(a > b ? a : b);
    }
    const bool pts = c->kind == UOT_COST_POINTS;
    const int db = pts ? dim_bucket(d) : 0;
    const size_t rb = pts ? grad_rec_stride(db) * sizeof(double) : sizeof(float);
    L.grad_rec = take((size_t)rec_count(nmax + kGradPadRows) * rb);
    // (a plan application's payload passes keep 16 columns per partial)
    const bool pay = which == UOT_WS_PLAN && (!pts || db <= 16);
    const int pstride = pay && grad_part_stride(16) > grad_part_stride(db) ? grad_part_stride(16)
                                                                           : grad_part_stride(db);
    size_t ps = pts ? (size_t)kGradMaxSplits * pstride : (size_t)kMaxSplits * grad_part_stride(0);
    if (!pts && pay && (size_t)kGradMaxSplits * pstride > ps) ps = (size_t)kGradMaxSplits * pstride;
    L.grad_part = take(ps * (size_t)nmax * sizeof(float));
    L.masses = take(2 * sizeof(double));
    L.total = off;
    return L;
  }
  L.pot_x = take((size_t)n * sizeof(float));
  L.pot_y = take((size_t)m * sizeof(float));
  L.rec_x = take((size_t)rec_count(n) * stride * sizeof(float));
  L.rec_y = take((size_t)rec_count(m) * stride * sizeof(float));
  // sized for the largest split count any device may choose, so the workspace size does
  // not depend on the device
  const size_t part_g = (size_t)kMaxSplits * m * sizeof(float2);
  const size_t part_f = (size_t)kMaxSplits * n * sizeof(float2);
  L.part = take(part_g > part_f ? part_g : part_f);
  const int nrec = (rec_count(nmax) + kBlock - 1) / kBlock;
  const int nbp = combine_blocks(nmax) > nrec ? combine_blocks(nmax) : nrec;
  L.bparts = take((size_t)(nbp + 1) * sizeof(BlockPart));
  L.dual = take((size_t)((nmax + kBlock - 1) / kBlock + 1) * 6 * sizeof(double));
  if (which == UOT_WS_ANDERSON) {
    L.ldh = ((int64_t)n + 63) / 64 * 64;
    L.hist = take((size_t)(kAndersonMaxK + 1) * L.ldh * sizeof(float));
    L.taus = take((size_t)(kAndersonMaxK + 1) * sizeof(double));
    L.gram = take(anderson_gram_bytes(n));
    L.acc_c = take((size_t)kAndersonMaxK * sizeof(double));
  }
  L.total = off;
  return L;
}

template <typename T>
T *at(void *base, size_t off) {
  return reinterpret_cast<T *>(static_cast<char *>(base) + off);
}

// Workspace supplied by the caller, or allocated for the duration of the call.
struct Workspace {
  void *ptr = nullptr;
  bool owned = false;
  ~Workspace() {
    if (owned && ptr) (void)hipFree(ptr);
  }
};

uot_status acquire(Workspace &w, void *user, size_t user_bytes, size_t need) {
  if (user != nullptr) {
    if (user_bytes < need)
      return fail(UOT_ERR_WORKSPACE, "workspace of %zu bytes, %zu needed", user_bytes, need);
    if (reinterpret_cast<uintptr_t>(user) % kAlign != 0)
      return fail(UOT_ERR_WORKSPACE, "workspace must be %zu-byte aligned", kAlign);
    w.ptr = user;
    return UOT_OK;
  }
  hipError_t e = hipMalloc(&w.ptr, need);
  if (e != hipSuccess) return fail(UOT_ERR_HIP, "hipMalloc(%zu): %s", need, hipGetErrorString(e));
  w.owned = true;
  return UOT_OK;
}

struct PinnedState {
  SolveState *h = nullptr;
  ~PinnedState() {
    if (h) (void)hipHostFree(h);
  }
};

// Common start of every call: flags, centring (points), weight validation.
uot_status prepare(const uot_cost *c, const float *alpha, const float *beta, SolveState *st,
                   double *center_part, hipStream_t s) {
  const bool pts = c->kind == UOT_COST_POINTS;
  UOT_HIP(launch_center(pts ? c->x : nullptr, pts ? c->n : 0, pts ? c->y : nullptr,
                        pts ? c->m : 0, pts ? c->d : 0, st, center_part, s));
  UOT_HIP(launch_validate(alpha, c->n, beta, c->m, st, s));
  return UOT_OK;
}

uot_status read_state(SolveState *dev, SolveState &host, hipStream_t s) {
  UOT_HIP(hipMemcpyAsync(&host, dev, sizeof(SolveState), hipMemcpyDeviceToHost, s));
  UOT_HIP(hipStreamSynchronize(s));
  return UOT_OK;
}

// ---------------------------------------------------------------------------------------
// Optional kernel timing: when enabled, each softmin launch is bracketed by two HIP events
// on the launch stream; durations are accumulated per kernel kind under a mutex.
// ---------------------------------------------------------------------------------------
enum ProfKind : int {
  kProfPoints = 0, kProfDenseCols = 1, kProfDenseRows = 2, kProfGrad = 3, kProfPointsDirect = 4,
  kProfKinds = 5
};
struct ProfAcc {
  int64_t launches = 0;
  double ms = 0.0, entries = 0.0;
};
std::mutex g_prof_mu;
bool g_prof_on = false;
int g_prof_period = 1;          // time every g_prof_period-th softmin launch
std::atomic<int64_t> g_prof_count{0};
ProfAcc g_prof[kProfKinds];

// Event pairs of one call, drained into g_prof when the ring wraps and at the end. A sampled
// softmin launch gets its start/stop events attached to the dispatch (hipExtLaunchKernel),
// so they time the kernel itself and add no commands between kernels.
class Timer {
 public:
  explicit Timer(bool on) : on_(on) {
    std::lock_guard<std::mutex> lk(g_prof_mu);
    period_ = g_prof_period;
  }
  ~Timer() {
    drain();
    for (auto &p : ring_) {
      (void)hipEventDestroy(p.t.start);
      (void)hipEventDestroy(p.t.stop);
    }
  }
  bool on() const { return on_; }
  // Events for the next softmin launch if it is sampled, else nullptr (*err set on failure).
  const LaunchTiming *next(hipError_t *err) {
    *err = hipSuccess;
    cur_ = -1;
    if (!on_ || g_prof_count.fetch_add(1) % period_ != 0) return nullptr;
    if (ring_.size() < kRing) {
      Pair p;
      *err = hipEventCreate(&p.t.start);
      if (*err == hipSuccess) *err = hipEventCreate(&p.t.stop);
      if (*err != hipSuccess) return nullptr;
      ring_.push_back(p);
    } else {
      *err = settle(head_);
      if (*err != hipSuccess) return nullptr;
    }
    cur_ = (long)head_;
    head_ = (head_ + 1) % kRing;
    return &ring_[cur_].t;
  }
  // Marks the launch that used next()'s events (if any) for accounting; `iter` is the solver
  // iteration it belongs to (0 outside the solvers).
  void launched(int kind, double entries, int64_t iter = 0) {
    if (cur_ < 0) return;
    Pair &p = ring_[cur_];
    p.kind = kind;
    p.entries = entries;
    p.iter = iter;
    p.live = true;
    cur_ = -1;
  }
  // The solve ran `iters` iterations: launches queued for later iterations found the solve
  // converged and returned at once, so they are left out (the solver queues one chunk of
  // iterations ahead of the host's convergence read).
  void last_iteration(int64_t iters) { last_iter_ = iters; }
  void drain() {
    for (size_t i = 0; i < ring_.size(); ++i) (void)settle(i);
  }

 private:
  static constexpr size_t kRing = 512;
  struct Pair {
    LaunchTiming t{nullptr, nullptr};
    int kind = 0;
    double entries = 0.0;
    int64_t iter = 0;
    bool live = false;
  };
  hipError_t settle(size_t i) {
    Pair &p = ring_[i];
    if (!p.live) return hipSuccess;
    hipError_t e = hipEventSynchronize(p.t.stop);
    if (e != hipSuccess) return e;
    float ms = 0.0f;
    e = hipEventElapsedTime(&ms, p.t.start, p.t.stop);
    p.live = false;
    if (e != hipSuccess) return e;
    if (p.iter > last_iter_) return hipSuccess;
    std::lock_guard<std::mutex> lk(g_prof_mu);
    g_prof[p.kind].launches += 1;
    g_prof[p.kind].ms += ms;
    g_prof[p.kind].entries += p.entries;
    return hipSuccess;
  }
  bool on_;
  int64_t period_ = 1;
  int64_t last_iter_ = INT64_MAX;
  std::vector<Pair> ring_;
  size_t head_ = 0;
  long cur_ = -1;
};

bool profiling_enabled() {
  std::lock_guard<std::mutex> lk(g_prof_mu);
  return g_prof_on;
}

// Everything one solve needs to launch its kernels.
struct Ctx {
  const uot_cost *c;
  int mode, d, n, m;
  const float *alpha, *beta;
  double eps, rho1, rho2;
  double sc;  // log2(e)/eps
  bool ti;
  int entropy = kEntropyKL;  // marginal penalties (plain and G-Sinkhorn)
  bool gvar = false;         // G-Sinkhorn: translate by lambda* after every iteration
  Layout L;
  void *ws;
  hipStream_t s;
  Timer *timer = nullptr;
  int64_t iter = 0;  // the solver iteration being issued (kernel timing only)
  // The scalar reduction of the last half-step, not launched yet: the next matrix-core
  // softmin runs it in a block of its own, or flush_reduce() launches it alone.
  mutable ReduceArgs pending{};
  mutable bool has_pending = false;
  SolveState *st() const { return at<SolveState>(ws, L.state); }
};

uot_status flush_reduce(const Ctx &k) {
  if (!k.has_pending) return UOT_OK;
  k.has_pending = false;
  UOT_HIP(launch_reduce(k.pending, k.s));
  return UOT_OK;
}

// Softmin partials of one half-step into the part buffer.
//   g_step: targets are the y side (columns of C), sources the x side with records rec_x;
//   otherwise targets are the x side (rows of C), sources the y side with records rec_y.
uot_status softmin_partials(const Ctx &k, bool g_step, const int32_t *done) {
  const HalfShape &h = g_step ? k.L.g : k.L.f;
  float2 *part = at<float2>(k.ws, k.L.part);
  const float *rec_src = at<float>(k.ws, g_step ? k.L.rec_x : k.L.rec_y);
  if (k.mode == kDense || !points_uses_mfma(k.mode, k.d)) UOT_TRY(flush_reduce(k));
  if (k.mode == kDense) {
    DenseArgs a;
    a.C = k.c->C;
    a.ldc = k.c->ldc;
    a.n = k.n;
    a.m = k.m;
    a.rec = rec_src;
    a.split_len = h.split.len;
    a.nsplit = h.split.n;
    a.sc = (float)k.sc;
    a.part = part;
    a.done = done;
    hipError_t te = hipSuccess;
    const LaunchTiming *t = k.timer ? k.timer->next(&te) : nullptr;
    UOT_HIP(te);
    UOT_HIP(g_step ? launch_dense_cols_partial(a, k.s, t) : launch_dense_rows(a, k.s, t));
    if (k.timer)
      k.timer->launched(g_step ? kProfDenseCols : kProfDenseRows, (double)k.n * (double)k.m, k.iter);
  } else {
    PointsArgs a;
    a.rec = rec_src;
    a.ns = g_step ? k.n : k.m;
    a.split_len = h.split.len;
    a.nsplit = h.split.n;
    a.tgt = g_step ? k.c->y : k.c->x;
    a.nt = g_step ? k.m : k.n;
    a.d = k.d;
    a.mu = k.st()->mu;
    a.sc = (float)k.sc;
    a.half_p = (float)(0.5 * k.c->p);
    a.part = part;
    a.done = done;
    a.red = k.pending;
    a.red_on = k.has_pending ? 1 : 0;
    k.has_pending = false;
    hipError_t te = hipSuccess;
    const LaunchTiming *t = k.timer ? k.timer->next(&te) : nullptr;
    UOT_HIP(te);
    UOT_HIP(launch_points_partial(k.mode, a, k.s, t));
    if (k.timer)
      k.timer->launched(k.mode == kPower ? kProfPointsDirect : kProfPoints, (double)k.n * (double)k.m,
                        k.iter);
  }
  return UOT_OK;
}

Epilogue epilogue_for(const Ctx &k, bool g_step) {
  const double e = k.eps, r1 = k.rho1, r2 = k.rho2;
  Epilogue ep;
  ep.ti = k.ti;
  ep.entropy = k.entropy;
  if (g_step) {  // targets y: g = k2 (S - tau_f) - c_g sA, kappa_g = e r1 / ((e + r2)(r1 + r2))
    ep.k_t = r2 / (e + r2);
    ep.c_t = k.ti ? e * r2 / ((e + r2) * (r1 + r2)) : 0.0;
    ep.rho_t = r2;
    ep.kappa_t = k.ti ? e * r1 / ((e + r2) * (r1 + r2)) : 0.0;
    ep.src_is_x = 1;
  } else {       // targets x: f = k1 (S - tau_g) - c_f sB, kappa_f = e r2 / ((e + r1)(r1 + r2))
    ep.k_t = r1 / (e + r1);
    ep.c_t = k.ti ? e * r1 / ((e + r1) * (r1 + r2)) : 0.0;
    ep.rho_t = r1;
    ep.kappa_t = k.ti ? e * r2 / ((e + r1) * (r1 + r2)) : 0.0;
    ep.src_is_x = 0;
  }
  return ep;
}

// snap, tau_out (f-steps of an Anderson solve, else NULL): receive the new stored f and
// its translation tau_f.
uot_status half_step(const Ctx &k, bool g_step, double tol, int check_every, float *snap = nullptr,
                     double *tau_out = nullptr) {
  SolveState *st = k.st();
  UOT_TRY(softmin_partials(k, g_step, &st->done));
  const HalfShape &h = g_step ? k.L.g : k.L.f;
  CombineArgs ca;
  ca.part = at<float2>(k.ws, k.L.part);
  ca.nsplit = h.split.n;
  ca.nt = g_step ? k.m : k.n;
  ca.mode = k.mode;
  ca.d = k.d;
  ca.tgt = k.mode == kDense ? nullptr : (g_step ? k.c->y : k.c->x);
  ca.w = g_step ? k.beta : k.alpha;
  ca.pot = at<float>(k.ws, g_step ? k.L.pot_y : k.L.pot_x);
  ca.rec_out = at<float>(k.ws, g_step ? k.L.rec_y : k.L.rec_x);
  ca.bparts = at<BlockPart>(k.ws, k.L.bparts);
  ca.st = st;
  ca.ep = epilogue_for(k, g_step);
  ca.sc = k.sc;
  ca.eps = k.eps;
  ca.snap = snap;
  UOT_HIP(launch_combine(ca, k.s));
  ReduceArgs ra;
  ra.bparts = ca.bparts;
  ra.nb = h.nb_combine;
  ra.st = st;
  ra.kind = g_step ? kReduceG : kReduceF;
  ra.ti = k.ti;
  ra.rho1 = k.rho1;
  ra.rho2 = k.rho2;
  ra.kappa_t = ca.ep.kappa_t;
  ra.tau1 = k.rho1 / (k.rho1 + k.rho2);
  ra.tau2 = k.rho2 / (k.rho1 + k.rho2);
  ra.tol = tol;
  ra.check_every = check_every;
  ra.tau_out = tau_out;
  ra.gvar = k.gvar ? 1 : 0;
  ra.entropy = k.entropy;
  ra.pot_f = at<float>(k.ws, k.L.pot_x);
  ra.pot_g = at<float>(k.ws, k.L.pot_y);
  ra.w_f = k.alpha;
  ra.w_g = k.beta;
  ra.nf = k.n;
  ra.ng = k.m;
  if (!g_step && k.gvar && k.entropy == kEntropyBerg) UOT_HIP(launch_berg_lambda(ra, k.s));
  k.pending = ra;  // run beside the next softmin, or by flush_reduce()
  k.has_pending = true;
  return UOT_OK;
}

// Records of one side from a potential (or zeros), optionally with its tilted-mass partials.
uot_status build_records(const Ctx &k, bool x_side, const float *pot, bool copy_pot,
                         bool with_mass, int *nblocks) {
  RecordArgs a;
  a.pts = k.mode == kDense ? nullptr : (x_side ? k.c->x : k.c->y);
  a.w = x_side ? k.alpha : k.beta;
  a.pot = pot;
  a.pot_copy = copy_pot ? at<float>(k.ws, x_side ? k.L.pot_x : k.L.pot_y) : nullptr;
  a.pot_off = 0.0;
  a.n = x_side ? k.n : k.m;
  a.mode = k.mode;
  a.d = k.d;
  a.rec = at<float>(k.ws, x_side ? k.L.rec_x : k.L.rec_y);
  a.bparts = with_mass ? at<BlockPart>(k.ws, k.L.bparts) : nullptr;
  a.rho = x_side ? k.rho1 : k.rho2;
  a.sc = k.sc;
  a.st = k.st();
  if (nblocks) *nblocks = (rec_count(a.n) + kBlock - 1) / kBlock;
  UOT_HIP(launch_build_records(a, k.s));
  return UOT_OK;
}

uot_status check_params(const uot_params *p) {
  if (p == nullptr) return fail(UOT_ERR_INVALID, "params is NULL");
  if (!finite_pos(p->eps)) return fail(UOT_ERR_INVALID, "eps=%g must be finite and > 0", p->eps);
  if (!finite_pos(p->rho1) || !finite_pos(p->rho2))
    return fail(UOT_ERR_INVALID, "rho1=%g, rho2=%g must be finite and > 0", p->rho1, p->rho2);
  if (p->max_iter < 1) return fail(UOT_ERR_INVALID, "max_iter=%d must be >= 1", p->max_iter);
  if (!(p->tol >= 0.0) || !std::isfinite(p->tol)) return fail(UOT_ERR_INVALID, "tol=%g must be finite and >= 0", p->tol);
  if (p->check_every < 1) return fail(UOT_ERR_INVALID, "check_every=%d must be >= 1", p->check_every);
  return UOT_OK;
}

uot_status check_scalars(double eps, double rho1, double rho2) {
  if (!finite_pos(eps)) return fail(UOT_ERR_INVALID, "eps=%g must be finite and > 0", eps);
  if (!finite_pos(rho1) || !finite_pos(rho2))
    return fail(UOT_ERR_INVALID, "rho1=%g, rho2=%g must be finite and > 0", rho1, rho2);
  return UOT_OK;
}

// Anderson cycle end: extrapolate x from the stored iterates, rebuild the x records with
// their tilted-mass partials, and leave the restart reduction pending.
uot_status anderson_step(const Ctx &k, const uot_anderson *acc) {
  UOT_TRY(flush_reduce(k));  // tau_f of the last iterate
  AndersonArgs aa;
  aa.H = at<float>(k.ws, k.L.hist);
  aa.ldh = k.L.ldh;
  aa.taus = at<double>(k.ws, k.L.taus);
  aa.n = k.n;
  aa.K = acc->k;
  aa.r = acc->r;
  aa.normalize = acc->normalize;
  aa.gram = at<double>(k.ws, k.L.gram);
  aa.c = at<double>(k.ws, k.L.acc_c);
  aa.pot = at<float>(k.ws, k.L.pot_x);
  aa.H0 = at<float>(k.ws, k.L.hist);
  aa.tau0 = aa.taus;
  aa.st = k.st();
  UOT_HIP(launch_anderson(aa, k.s));
  int nbx = 0;
  UOT_TRY(build_records(k, true, at<float>(k.ws, k.L.pot_x), false, true, &nbx));
  ReduceArgs rr;
  rr.bparts = at<BlockPart>(k.ws, k.L.bparts);
  rr.nb = nbx;
  rr.st = k.st();
  rr.kind = kReduceRestart;
  rr.ti = k.ti;
  rr.rho1 = k.rho1;
  rr.rho2 = k.rho2;
  rr.kappa_t = 0.0;
  rr.tau1 = rr.tau2 = 0.0;
  rr.tol = 0.0;
  rr.check_every = 1;
  k.pending = rr;
  k.has_pending = true;
  return UOT_OK;
}

uot_status check_anderson(const uot_anderson *acc) {
  if (acc == nullptr) return fail(UOT_ERR_INVALID, "anderson settings are NULL");
  if (acc->k < 2 || acc->k > kAndersonMaxK)
    return fail(UOT_ERR_INVALID, "anderson k=%d must be in 2..%d", acc->k, kAndersonMaxK);
  if (!finite_pos(acc->r)) return fail(UOT_ERR_INVALID, "anderson r=%g must be finite and > 0", acc->r);
  if (acc->normalize != 0 && acc->normalize != 1)
    return fail(UOT_ERR_INVALID, "anderson normalize=%d must be 0 or 1", acc->normalize);
  return UOT_OK;
}

uot_status check_phi(const uot_phi *phi) {
  if (phi == nullptr) return fail(UOT_ERR_INVALID, "phi settings are NULL");
  if (phi->entropy != UOT_ENTROPY_KL && phi->entropy != UOT_ENTROPY_BERG)
    return fail(UOT_ERR_INVALID, "phi entropy=%d must be UOT_ENTROPY_KL or UOT_ENTROPY_BERG", phi->entropy);
  if (phi->variant != UOT_SINKHORN_F && phi->variant != UOT_SINKHORN_G)
    return fail(UOT_ERR_INVALID, "phi variant=%d must be UOT_SINKHORN_F or UOT_SINKHORN_G", phi->variant);
  return UOT_OK;
}

// Times the candidate split counts of one half-step's softmin (on the call's own records;
// the partials it writes are overwritten by the real half-step) and keeps the fastest.
uot_status tune_half(Ctx &k, bool g_step) {
  const int nt = g_step ? k.m : k.n, ns = g_step ? k.n : k.m;
  const bool rows = !g_step;
  if (!g_autotune.load() || (double)nt * (double)ns < kTuneMinEntries) return UOT_OK;
  if (k.mode == kDense && rows) return UOT_OK;  // the rows kernel takes no splits
  const TuneKey key = tune_key(k.mode, k.d, nt, ns, rows);
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    if (g_tune_cache.count(key)) return UOT_OK;
  }
  HalfShape &slot = g_step ? k.L.g : k.L.f;
  Timer *timer = k.timer;
  k.timer = nullptr;
  hipEvent_t ev[2] = {nullptr, nullptr};
  struct EvGuard {
    hipEvent_t *e;
    ~EvGuard() {
      if (e[0]) (void)hipEventDestroy(e[0]);
      if (e[1]) (void)hipEventDestroy(e[1]);
    }
  } evg{ev};
  UOT_HIP(hipEventCreate(&ev[0]));
  UOT_HIP(hipEventCreate(&ev[1]));
  double best_ms = INFINITY, best_mult = 1.0;
  std::vector<int> seen;
  for (double mult : kTuneMults) {
    const HalfShape h = half_shape(k.mode, k.d, nt, ns, rows, mult);
    bool dup = false;
    for (int n : seen) dup = dup || n == h.split.n;
    if (dup) continue;
    seen.push_back(h.split.n);
    slot = h;
    UOT_TRY(softmin_partials(k, g_step, nullptr));  // warm
    UOT_HIP(hipEventRecord(ev[0], k.s));
    UOT_TRY(softmin_partials(k, g_step, nullptr));
    UOT_TRY(softmin_partials(k, g_step, nullptr));
    UOT_HIP(hipEventRecord(ev[1], k.s));
    UOT_HIP(hipEventSynchronize(ev[1]));
    float ms = 0.0f;
    UOT_HIP(hipEventElapsedTime(&ms, ev[0], ev[1]));
    if (ms < best_ms) {
      best_ms = ms;
      best_mult = mult;
    }
  }
  slot = half_shape(k.mode, k.d, nt, ns, rows, best_mult);
  k.timer = timer;
  std::lock_guard<std::mutex> lk(g_tune_mu);
  g_tune_cache[key] = best_mult;
  return UOT_OK;
}

// Choice of the p = 2 points softmin form (see uot_cost in uot.h): the expanded form's
// float32 rounding E = 2^-24 (d + 4) (max|x - mu| + max|y - mu|)^2 (potential units) is a
// risk to the 1e-5 relative accuracy of the potentials when its share of the exponent,
// delta = E log2(e) / eps, is large (few entries carry each softmin, so the roundings do
// not average out) and when it can pile up against small potentials: over up to
// 1 / (1 - k1 k2) iterations (the slowest contraction of Sec. 3). Thresholds measured on
// 1-D/2-D/3-D/16-D clouds at eps from 3e-4 to 0.5 and rho from 0.1 to 10 (TI and plain,
// 30 and 300 iterations against the oracle): every case above 5e-6 has delta > 1e-3 and
// Q > 1.1e-4; the error stayed below 0.2 Q where delta > 3e-4.
constexpr double kFormDelta = 3e-4, kFormQ = 3e-5;
// A solve to a tolerance whose p = 2 check fails keeps the expanded form while its change
// is above S = max(kSwitchTol tol, kSwitchE E): the iterates are then far from the fixed
// point against the form's rounding. The direct form, started from where the expanded one
// stopped, finishes the solve (its fixed point is the one the tolerance refers to). The
// expanded phase also ends when, below kStallBand S, a check's change is above kStall times
// the previous one (a rounding floor of the expanded form near S would otherwise hold it).
constexpr double kSwitchTol = 100.0, kSwitchE = 1.0, kStallBand = 64.0, kStall = 0.9;

double expanded_form_rounding(const uot_cost *c, const SolveState &h) {
  const double span = std::sqrt(h.span_x2) + std::sqrt(h.span_y2);
  return std::ldexp(1.0, -24) * (c->d + 4) * span * span;
}

uot_status solve(const uot_cost *c, const float *alpha, const float *beta, const uot_params *P,
                 float *f, float *g, void *workspace, size_t workspace_bytes, uot_info *info,
                 void *stream, bool ti, const uot_anderson *acc = nullptr,
                 const uot_phi *phi = nullptr, bool direct = false) {
  UOT_TRY(check_cost(c));
  UOT_TRY(check_params(P));
  UOT_TRY(check_cost_ptrs(c));
  UOT_TRY(check_device_ptr(alpha, "alpha"));
  UOT_TRY(check_device_ptr(beta, "beta"));
  UOT_TRY(check_device_ptr(f, "f"));
  UOT_TRY(check_device_ptr(g, "g"));
  Ctx k;
  k.c = c;
  k.mode = direct ? kPower : rec_mode_of(c);
  k.d = c->kind == UOT_COST_POINTS ? c->d : 0;
  k.n = c->n;
  k.m = c->m;
  k.alpha = alpha;
  k.beta = beta;
  k.eps = P->eps;
  k.rho1 = P->rho1;
  k.rho2 = P->rho2;
  k.sc = kLog2e / P->eps;
  k.ti = ti;
  if (phi) {
    k.entropy = phi->entropy == UOT_ENTROPY_BERG ? kEntropyBerg : kEntropyKL;
    k.gvar = phi->variant == UOT_SINKHORN_G;
  }
  k.L = make_layout(c, acc ? UOT_WS_ANDERSON : UOT_WS_SOLVE, k.mode);
  k.s = static_cast<hipStream_t>(stream);
  Workspace w;
  UOT_TRY(acquire(w, workspace, workspace_bytes, k.L.total));
  k.ws = w.ptr;
  SolveState *st = k.st();
  Timer timer(profiling_enabled());
  k.timer = timer.on() ? &timer : nullptr;
  // the p = 2 form check (default setting only; an explicit setting is obeyed)
  const bool check_form = !direct && c->kind == UOT_COST_POINTS && c->p == 2.0 &&
                          g_points_variant == kPointsAuto && k.mode != kPower;

  PinnedState pin;
  UOT_HIP(hipHostMalloc(reinterpret_cast<void **>(&pin.h), 2 * sizeof(SolveState), hipHostMallocDefault));
  SolveState *hst = pin.h;

  // start: flags, centring, weights, records of x from f_0 (with Smin_alpha^rho1(f_0)), g = 0
  UOT_TRY(prepare(c, alpha, beta, st, at<double>(k.ws, k.L.center), k.s));
  if (check_form)
    UOT_HIP(launch_span(c->x, c->n, c->y, c->m, c->d, st, at<double>(k.ws, k.L.center), k.s));
  int nbx = 0;
  UOT_TRY(build_records(k, true, P->warm_start ? f : nullptr, true, true, &nbx));
  ReduceArgs ri;
  ri.bparts = at<BlockPart>(k.ws, k.L.bparts);
  ri.nb = nbx;
  ri.st = st;
  ri.kind = kReduceInit;
  ri.ti = ti;
  ri.rho1 = k.rho1;
  ri.rho2 = k.rho2;
  ri.kappa_t = 0.0;
  ri.tau1 = ri.tau2 = 0.0;
  ri.tol = 0.0;
  ri.check_every = 1;
  UOT_HIP(launch_reduce(ri, k.s));
  UOT_TRY(build_records(k, false, nullptr, true, false, nullptr));
  if (acc) {  // x_0 of the first cycle: the starting f (untranslated), tau 0
    UOT_HIP(hipMemcpyAsync(at<float>(k.ws, k.L.hist), at<float>(k.ws, k.L.pot_x),
                           (size_t)k.n * sizeof(float), hipMemcpyDeviceToDevice, k.s));
    UOT_HIP(hipMemsetAsync(at<double>(k.ws, k.L.taus), 0, (kAndersonMaxK + 1) * sizeof(double), k.s));
  }
  UOT_TRY(read_state(st, hst[0], k.s));
  if (hst[0].error & kErrWeights)
    return fail(UOT_ERR_INVALID, "weights must be finite, >= 0, with positive total mass");
  UOT_TRY(tune_half(k, true));  // first solve of this shape: split counts by timing
  UOT_TRY(tune_half(k, false));
  // expanded-form rounding against eps now; against the potentials after iteration 1
  const double form_e = check_form ? expanded_form_rounding(c, hst[0]) : 0.0;
  const bool check_q = check_form && form_e * kLog2e / P->eps > kFormDelta;

  // iterations, in chunks of check_every; the host reads the convergence flag one chunk late
  // so the GPU always has queued work (solver kernels return at once after convergence)
  const bool checking = P->tol > 0.0;
  // tolerance of the device's convergence test: the switch point while a two-phase solve
  // runs its expanded-form phase (check_q below), else tol
  bool two_phase = false;
  double dev_tol = P->tol;
  double prev_change = INFINITY;  // the change at the previous check (expanded phase)
  const int chunk = checking ? P->check_every : P->max_iter;
  hipEvent_t ev[2] = {nullptr, nullptr};
  struct EvGuard {
    hipEvent_t *e;
    ~EvGuard() {
      if (e[0]) (void)hipEventDestroy(e[0]);
      if (e[1]) (void)hipEventDestroy(e[1]);
    }
  } evg{ev};
  UOT_HIP(hipEventCreateWithFlags(&ev[0], hipEventDisableTiming));
  UOT_HIP(hipEventCreateWithFlags(&ev[1], hipEventDisableTiming));
  int issued = 0, c_idx = 0;
  bool stop = false;
  while (issued < P->max_iter && !stop) {
    const int todo = (P->max_iter - issued) < chunk ? (P->max_iter - issued) : chunk;
    for (int t = 0; t < todo; ++t) {
      const int it = issued + t + 1;  // 1-based iteration number
      k.iter = it;
      UOT_TRY(half_step(k, true, dev_tol, P->check_every));
      if (acc) {
        const int kc = (it - 1) % acc->k + 1;  // position of this iterate in its cycle
        UOT_TRY(half_step(k, false, dev_tol, P->check_every,
                          at<float>(k.ws, k.L.hist) + (size_t)kc * k.L.ldh,
                          at<double>(k.ws, k.L.taus) + kc));
        if (kc == acc->k && it < P->max_iter) UOT_TRY(anderson_step(k, acc));
      } else {
        UOT_TRY(half_step(k, false, dev_tol, P->check_every));
      }
      if (it == 1 && check_q) {
        UOT_TRY(flush_reduce(k));
        UOT_HIP(launch_pot_absmax(at<float>(k.ws, k.L.pot_x), k.n, at<float>(k.ws, k.L.pot_y),
                                  k.m, st, k.s));
        UOT_TRY(read_state(st, hst[0], k.s));
        const double k1 = P->rho1 / (P->eps + P->rho1), k2 = P->rho2 / (P->eps + P->rho2);
        const double amp = std::fmin((double)P->max_iter, 1.0 / (1.0 - k1 * k2));
        const double hmin = std::fmin(hst[0].fabs_max, hst[0].gabs_max);
        if (!(form_e * amp <= kFormQ * hmin)) {  // (also when a norm is 0 or not finite)
          if (checking && acc == nullptr && phi == nullptr) {
            two_phase = true;
            dev_tol = std::fmax(kSwitchTol * P->tol, kSwitchE * form_e);
          } else {
            return solve(c, alpha, beta, P, f, g, w.ptr, w.owned ? k.L.total : workspace_bytes,
                         info, stream, ti, acc, phi, true);  // same workspace size in both forms
          }
        }
      }
    }
    issued += todo;
    UOT_TRY(flush_reduce(k));
    if (checking) {
      SolveState *slot = &hst[c_idx & 1];
      UOT_HIP(hipMemcpyAsync(slot, st, sizeof(SolveState), hipMemcpyDeviceToHost, k.s));
      UOT_HIP(hipEventRecord(ev[c_idx & 1], k.s));
      if (c_idx >= 1) {
        UOT_HIP(hipEventSynchronize(ev[(c_idx - 1) & 1]));
        if (hst[(c_idx - 1) & 1].done) stop = true;
        if (two_phase) {  // expanded phase: stalled near the switch point
          const double dl = hst[(c_idx - 1) & 1].delta;
          if (dl < kStallBand * dev_tol && dl > kStall * prev_change) stop = true;
          prev_change = dl;
        }
      }
      ++c_idx;
    }
  }
  UOT_HIP(launch_finalize(at<float>(k.ws, k.L.pot_x), k.n, 0.0, 0, st, f, k.s));
  UOT_HIP(launch_finalize(at<float>(k.ws, k.L.pot_y), k.m, 0.0, 1, st, g, k.s));
  SolveState fin;
  UOT_TRY(read_state(st, fin, k.s));
  timer.last_iteration(fin.iter);
  if (two_phase && !(fin.error & kErrNumeric) && fin.iter < P->max_iter) {
    // second phase: the direct form from the potentials just written to f (a warm start
    // resumes the run: TI and plain Sinkhorn take f as their starting potential), to tol
    uot_params P2 = *P;
    P2.warm_start = 1;
    P2.max_iter = P->max_iter - fin.iter;
    uot_info inf2{};
    UOT_TRY(solve(c, alpha, beta, &P2, f, g, w.ptr, w.owned ? k.L.total : workspace_bytes, &inf2,
                  stream, ti, nullptr, nullptr, true));
    if (info) {
      *info = inf2;
      info->iters = fin.iter + inf2.iters;
      info->points_form = 2;
    }
    return UOT_OK;
  }
  if (info) {
    info->iters = fin.iter;
    // (a two-phase solve that ends here ran out of iterations in its first phase)
    info->converged = (checking && fin.done && !fin.error && !two_phase) ? 1 : 0;
    info->last_change = fin.delta;
    info->lambda = fin.lambda;
    info->points_form = (c->kind == UOT_COST_POINTS && c->p == 2.0)
                            ? (two_phase ? 2 : (k.mode == kPower ? 1 : 0))
                            : -1;
  }
  if (fin.error & kErrNumeric) return fail(UOT_ERR_NUMERIC, "non-finite potentials after %d iterations", fin.iter);
  return UOT_OK;
}

uot_status dual_value(const uot_cost *c, const float *alpha, const float *beta, double eps,
                      double rho1, double rho2, const float *f, const float *g, void *workspace,
                      size_t workspace_bytes, double *value, void *stream) {
  UOT_TRY(check_cost(c));
  UOT_TRY(check_scalars(eps, rho1, rho2));
  if (value == nullptr) return fail(UOT_ERR_INVALID, "value is NULL");
  UOT_TRY(check_cost_ptrs(c));
  UOT_TRY(check_device_ptr(alpha, "alpha"));
  UOT_TRY(check_device_ptr(beta, "beta"));
  UOT_TRY(check_device_ptr(f, "f"));
  UOT_TRY(check_device_ptr(g, "g"));
  Ctx k;
  k.c = c;
  // p = 2 points: direct differences under the default setting (an error E in a softmin is
  // an error E / eps relative in m(pi))
  k.mode = (c->kind == UOT_COST_POINTS && c->p == 2.0 && g_points_variant == kPointsAuto)
               ? kPower
               : rec_mode_of(c);
  k.d = c->kind == UOT_COST_POINTS ? c->d : 0;
  k.n = c->n;
  k.m = c->m;
  k.alpha = alpha;
  k.beta = beta;
  k.eps = eps;
  k.rho1 = rho1;
  k.rho2 = rho2;
  k.sc = kLog2e / eps;
  k.ti = false;
  k.L = make_layout(c, UOT_WS_DUAL, k.mode);
  k.s = static_cast<hipStream_t>(stream);
  Workspace w;
  UOT_TRY(acquire(w, workspace, workspace_bytes, k.L.total));
  k.ws = w.ptr;
  SolveState *st = k.st();
  UOT_TRY(prepare(c, alpha, beta, st, at<double>(k.ws, k.L.center), k.s));
  UOT_TRY(build_records(k, false, g, false, false, nullptr));
  UOT_TRY(softmin_partials(k, false, nullptr));
  DualArgs da;
  da.part = at<float2>(k.ws, k.L.part);
  da.nsplit = k.L.f.split.n;
  da.n = k.n;
  da.m = k.m;
  da.mode = k.mode;
  da.d = k.d;
  da.x = k.mode == kDense ? nullptr : c->x;
  da.alpha = alpha;
  da.beta = beta;
  da.f = f;
  da.g = g;
  da.st = st;
  da.sc = k.sc;
  da.eps = eps;
  da.rho1 = rho1;
  da.rho2 = rho2;
  da.acc = at<double>(k.ws, k.L.dual);
  int nb = 0;
  UOT_HIP(launch_dual_terms(da, &nb, k.s));
  UOT_HIP(launch_dual_reduce(da, nb, k.s));
  SolveState fin;
  UOT_TRY(read_state(st, fin, k.s));
  if (fin.error & kErrWeights) return fail(UOT_ERR_INVALID, "weights must be finite, >= 0, with positive total mass");
  if (!fin.pos_a || !fin.pos_b) return fail(UOT_ERR_INVALID, "weights must have positive total mass");
  *value = fin.value;
  if (fin.error & kErrNumeric) return fail(UOT_ERR_NUMERIC, "non-finite dual value");
  return UOT_OK;
}

// Fills the ApplyArgs common to plan application and the backward.
ApplyArgs apply_args(const uot_cost *c, int mode, bool targets_x, const float *alpha,
                     const float *beta, const float *f, const float *g, double eps, SolveState *st) {
  ApplyArgs a;
  memset(&a, 0, sizeof a);
  a.mode = mode;
  a.d = c->kind == UOT_COST_POINTS ? c->d : 0;
  a.C = c->C;
  a.ldc = c->ldc;
  a.transpose = targets_x ? 0 : 1;
  a.tgt = c->kind == UOT_COST_POINTS ? (targets_x ? c->x : c->y) : nullptr;
  a.src = c->kind == UOT_COST_POINTS ? (targets_x ? c->y : c->x) : nullptr;
  a.mu = st->mu;
  a.p = c->kind == UOT_COST_POINTS ? c->p : 1.0;
  a.nt = targets_x ? c->n : c->m;
  a.ns = targets_x ? c->m : c->n;
  a.w_t = targets_x ? alpha : beta;
  a.w_s = targets_x ? beta : alpha;
  a.h_t = targets_x ? f : g;
  a.h_s = targets_x ? g : f;
  a.sc = (float)(kLog2e / eps);
  return a;
}

// The plan applied to a payload V (points costs whose dimension bucket takes the matrix-core
// pass; targets x when tx): the records of the other side, then per 16 columns of V one pass
// over the sources (exponent in double precision, one exp2 per entry) and the split merge
// writing out[t, c0 .. c0 + 15].
uot_status apply_payload(const uot_cost *c, bool tx, const float *alpha, const float *beta,
                         const float *f, const float *g, double eps, SolveState *st, void *ws,
                         const Layout &L, const float *V, int kc, int64_t ldv, float *out,
                         int64_t ldout, hipStream_t s) {
  const int nt = tx ? c->n : c->m, ns = tx ? c->m : c->n;
  const double sc = kLog2e / eps;
  double *rec = at<double>(ws, L.grad_rec);
  float *part = at<float>(ws, L.grad_part);
  GradRecordArgs ra;
  ra.pts = tx ? c->y : c->x;
  ra.w = tx ? beta : alpha;
  ra.pot = tx ? g : f;
  ra.mu = st->mu;
  ra.n = ns;
  ra.d = c->d;
  ra.sc = sc;
  ra.rec = rec;
  UOT_HIP(launch_grad_records(ra, s));
  const int cus = device_cus();
  const int tiles = (nt + grad_targets_per_block(c->d) - 1) / grad_targets_per_block(c->d);
  const Split sp = make_split(ns, tiles, 64, grad_source_align(c->d), (cus > 0 ? cus : 256) * 4,
                              kGradMaxSplits);
  for (int c0 = 0; c0 < kc; c0 += 16) {
    GradArgs ga;
    ga.tgt = tx ? c->x : c->y;
    ga.nt = nt;
    ga.d = c->d;
    ga.mu = st->mu;
    ga.h_t = tx ? f : g;
    ga.rec = rec;
    ga.ns = ns;
    ga.split_len = sp.len;
    ga.nsplit = sp.n;
    ga.sc = sc;
    ga.half_p = 0.5 * c->p;
    ga.p = (float)c->p;
    ga.grad = 1;
    ga.part = part;
    ga.V = V + c0;
    ga.ldv = ldv;
    ga.vcols = kc - c0 < 16 ? kc - c0 : 16;
    UOT_HIP(launch_grad_partial(ga, s));
    GradCombineArgs ca;
    ca.part = part;
    ca.nsplit = sp.n;
    ca.nt = nt;
    ca.d = ga.vcols;
    ca.tgt = nullptr;
    ca.mu = st->mu;
    ca.h_t = tx ? f : g;
    ca.w_t = tx ? alpha : beta;
    ca.sc = sc;
    ca.eps = eps;
    ca.rho = 1.0;
    ca.gout = 1.0;
    ca.pfac = 1.0;
    ca.mass_other = nullptr;
    ca.marg = nullptr;
    ca.marg_stride = 0;
    ca.dw = nullptr;
    ca.dpts = nullptr;
    ca.apply_out = out + c0;
    ca.ldout = ldout;
    UOT_HIP(launch_grad_combine(ca, s));
  }
  return UOT_OK;
}

// The plan applied to a payload V on a stored cost (targets the rows of C when tx): the
// records b_s of the other side, then per 16 columns of V one pass over C (one exp2 per
// entry, float32 exponent as in the stored-cost softmins) and the split merge.
uot_status apply_payload_dense(const uot_cost *c, bool tx, const float *alpha, const float *beta,
                               const float *f, const float *g, double eps, SolveState *st,
                               void *ws, const Layout &L, const float *V, int kc, int64_t ldv,
                               float *out, int64_t ldout, hipStream_t s) {
  const int nt = tx ? c->n : c->m, ns = tx ? c->m : c->n;
  const double sc = kLog2e / eps;
  float *rec = at<float>(ws, L.grad_rec);
  float *part = at<float>(ws, L.grad_part);
  RecordArgs ra;
  ra.pts = nullptr;
  ra.w = tx ? beta : alpha;
  ra.pot = tx ? g : f;
  ra.pot_copy = nullptr;
  ra.pot_off = 0.0;
  ra.n = ns;
  ra.mode = kDense;
  ra.d = 0;
  ra.rec = rec;
  ra.bparts = nullptr;
  ra.rho = 1.0;
  ra.sc = sc;
  ra.st = st;
  UOT_HIP(launch_build_records(ra, s));
  const int cus = device_cus();
  const int tiles = (nt + 255) / 256;
  const Split sp = make_split(ns, tiles, 64, 16, (cus > 0 ? cus : 256) * 4, kGradMaxSplits);
  for (int c0 = 0; c0 < kc; c0 += 16) {
    DensePayloadArgs da;
    da.C = c->C;
    da.ldc = c->ldc;
    da.trans = tx ? 0 : 1;
    da.vec4 = (reinterpret_cast<uintptr_t>(c->C) % 16 == 0 && c->ldc % 4 == 0) ? 1 : 0;
    da.nt = nt;
    da.ns = ns;
    da.rec = rec;
    da.sc = (float)sc;
    da.split_len = sp.len;
    da.nsplit = sp.n;
    da.V = V + c0;
    da.ldv = ldv;
    da.vcols = kc - c0 < 16 ? kc - c0 : 16;
    da.part = part;
    UOT_HIP(launch_dense_payload(da, s));
    GradCombineArgs ca;
    ca.part = part;
    ca.nsplit = sp.n;
    ca.nt = nt;
    ca.d = da.vcols;
    ca.tgt = nullptr;
    ca.mu = st->mu;
    ca.h_t = tx ? f : g;
    ca.w_t = tx ? alpha : beta;
    ca.sc = sc;
    ca.eps = eps;
    ca.rho = 1.0;
    ca.gout = 1.0;
    ca.pfac = 1.0;
    ca.mass_other = nullptr;
    ca.marg = nullptr;
    ca.marg_stride = 0;
    ca.dw = nullptr;
    ca.dpts = nullptr;
    ca.apply_out = out + c0;
    ca.ldout = ldout;
    UOT_HIP(launch_grad_combine(ca, s));
  }
  return UOT_OK;
}

// Row sums of the plan for the targets of one side (targets x when tx), in one pass over the
// other side's points (kernels_grad.hip) or one stored-cost softmin, and what is asked of
// them: the plan marginal (marg, element t at marg[t * marg_stride]), the weight gradient
// dw (needs rho_t and mass_other, the source side's total mass on the device) and the point
// gradient dpts (points costs).
uot_status envelope_side(const uot_cost *c, bool tx, const float *alpha, const float *beta,
                         const float *f, const float *g, double eps, double rho_t, double gout,
                         SolveState *st, void *ws, const Layout &L, float *marg,
                         int64_t marg_stride, float *dw, const double *mass_other, float *dpts,
                         hipStream_t s, bool timed = true) {
  const bool dense = c->kind == UOT_COST_DENSE;
  const int nt = tx ? c->n : c->m, ns = tx ? c->m : c->n;
  const double sc = kLog2e / eps;
  float *part = at<float>(ws, L.grad_part);
  const int cus = device_cus();
  int nsplit = 1;
  if (dense) {
    float *rec = at<float>(ws, L.grad_rec);
    RecordArgs ra;
    ra.pts = nullptr;
    ra.w = tx ? beta : alpha;
    ra.pot = tx ? g : f;
    ra.pot_copy = nullptr;
    ra.pot_off = 0.0;
    ra.n = ns;
    ra.mode = kDense;
    ra.d = 0;
    ra.rec = rec;
    ra.bparts = nullptr;
    ra.rho = 1.0;
    ra.sc = sc;
    ra.st = st;
    UOT_HIP(launch_build_records(ra, s));
    DenseArgs da;
    da.C = c->C;
    da.ldc = c->ldc;
    da.n = c->n;
    da.m = c->m;
    da.rec = rec;
    da.sc = (float)sc;
    da.part = reinterpret_cast<float2 *>(part);
    da.done = nullptr;
    if (tx) {
      da.split_len = ns;
      da.nsplit = 1;
      UOT_HIP(launch_dense_rows(da, s));
    } else {
      const HalfShape h = half_shape(kDense, 0, nt, ns, false);
      da.split_len = h.split.len;
      da.nsplit = nsplit = h.split.n;
      UOT_HIP(launch_dense_cols_partial(da, s));
    }
  } else {
    double *rec = at<double>(ws, L.grad_rec);
    GradRecordArgs ra;
    ra.pts = tx ? c->y : c->x;
    ra.w = tx ? beta : alpha;
    ra.pot = tx ? g : f;
    ra.mu = st->mu;
    ra.n = ns;
    ra.d = c->d;
    ra.sc = sc;
    ra.rec = rec;
    UOT_HIP(launch_grad_records(ra, s));
    GradArgs ga;
    ga.tgt = tx ? c->x : c->y;
    ga.nt = nt;
    ga.d = c->d;
    ga.mu = st->mu;
    ga.h_t = tx ? f : g;
    ga.rec = rec;
    ga.ns = ns;
    const int tiles = (nt + grad_targets_per_block(c->d) - 1) / grad_targets_per_block(c->d);
    const Split sp = make_split(ns, tiles, 64, grad_source_align(c->d), (cus > 0 ? cus : 256) * 4,
                                kGradMaxSplits);
    ga.split_len = sp.len;
    ga.nsplit = nsplit = sp.n;
    ga.sc = sc;
    ga.half_p = 0.5 * c->p;
    ga.p = (float)c->p;
    ga.grad = dpts != nullptr ? 1 : 0;
    ga.part = part;
    Timer timer(timed && profiling_enabled());
    hipError_t te = hipSuccess;
    const LaunchTiming *t = timer.on() ? timer.next(&te) : nullptr;
    UOT_HIP(te);
    UOT_HIP(launch_grad_partial(ga, s, t));
    timer.launched(kProfGrad, (double)nt * (double)ns);
  }
  GradCombineArgs ca;
  ca.part = part;
  ca.nsplit = nsplit;
  ca.nt = nt;
  ca.d = dense ? 0 : c->d;
  ca.tgt = dense ? nullptr : (tx ? c->x : c->y);
  ca.mu = st->mu;
  ca.h_t = tx ? f : g;
  ca.w_t = tx ? alpha : beta;
  ca.sc = sc;
  ca.eps = eps;
  ca.rho = rho_t;
  ca.gout = gout;
  ca.pfac = (!dense && c->p == 2.0) ? 2.0 : 1.0;
  ca.mass_other = mass_other;
  ca.marg = marg;
  ca.marg_stride = marg_stride;
  ca.dw = dw;
  ca.dpts = dpts;
  UOT_HIP(launch_grad_combine(ca, s));
  return UOT_OK;
}

uot_status plan_apply(const uot_cost *c, const float *alpha, const float *beta, double eps,
                      const float *f, const float *g, int32_t transpose, const float *V, int32_t kc,
                      int64_t ldv, float *out, int64_t ldout, void *workspace, size_t workspace_bytes,
                      void *stream) {
  UOT_TRY(check_cost(c));
  if (!finite_pos(eps)) return fail(UOT_ERR_INVALID, "eps=%g must be finite and > 0", eps);
  if (kc < 1 || kc > 64) return fail(UOT_ERR_INVALID, "k=%d not in [1, 64]", kc);
  if (V == nullptr && kc != 1) return fail(UOT_ERR_INVALID, "V = NULL (ones) needs k = 1");
  if (V != nullptr && ldv < kc) return fail(UOT_ERR_INVALID, "ldv < k");
  if (ldout < kc) return fail(UOT_ERR_INVALID, "ldout < k");
  if (transpose != 0 && transpose != 1) return fail(UOT_ERR_INVALID, "transpose must be 0 or 1");
  UOT_TRY(check_cost_ptrs(c));
  UOT_TRY(check_device_ptr(alpha, "alpha"));
  UOT_TRY(check_device_ptr(beta, "beta"));
  UOT_TRY(check_device_ptr(f, "f"));
  UOT_TRY(check_device_ptr(g, "g"));
  UOT_TRY(check_device_ptr(out, "out"));
  if (V != nullptr) UOT_TRY(check_device_ptr(V, "V"));
  const Layout L = make_layout(c, UOT_WS_PLAN);
  Workspace w;
  UOT_TRY(acquire(w, workspace, workspace_bytes, L.total));
  hipStream_t s = static_cast<hipStream_t>(stream);
  SolveState *st = at<SolveState>(w.ptr, L.state);
  UOT_TRY(prepare(c, alpha, beta, st, at<double>(w.ptr, L.center), s));
  if (V == nullptr) {  // the marginals: row sums in one pass
    UOT_TRY(envelope_side(c, transpose == 0, alpha, beta, f, g, eps, 1.0, 1.0, st, w.ptr, L, out,
                          ldout, nullptr, nullptr, nullptr, s));
  } else if (c->kind == UOT_COST_DENSE && grad_payload_supported(1)) {
    UOT_TRY(apply_payload_dense(c, transpose == 0, alpha, beta, f, g, eps, st, w.ptr, L, V, kc, ldv,
                                out, ldout, s));
  } else if (c->kind == UOT_COST_POINTS && grad_payload_supported(c->d)) {
    UOT_TRY(apply_payload(c, transpose == 0, alpha, beta, f, g, eps, st, w.ptr, L, V, kc, ldv, out,
                          ldout, s));
  } else {
    ApplyArgs a = apply_args(c, mode_of(c), transpose == 0, alpha, beta, f, g, eps, st);
    a.V = V;
    a.k = kc;
    a.ldv = ldv;
    a.out = out;
    a.ldout = ldout;
    UOT_HIP(launch_apply_with_scratch(a, at<void>(w.ptr, L.scratch), s));
  }
  SolveState fin;
  UOT_TRY(read_state(st, fin, s));
  if ((fin.error & kErrWeights) || !fin.pos_a || !fin.pos_b)
    return fail(UOT_ERR_INVALID, "weights must be finite, >= 0, with positive total mass");
  return UOT_OK;
}

uot_status backward(const uot_cost *c, const float *alpha, const float *beta, double eps,
                    double rho1, double rho2, const float *f, const float *g, double grad_out,
                    float *dx, float *dy, float *dalpha, float *dbeta, void *workspace,
                    size_t workspace_bytes, void *stream, bool timed = true) {
  UOT_TRY(check_cost(c));
  UOT_TRY(check_scalars(eps, rho1, rho2));
  if (!std::isfinite(grad_out)) return fail(UOT_ERR_INVALID, "grad_out must be finite");
  if (c->kind == UOT_COST_DENSE && (dx != nullptr || dy != nullptr))
    return fail(UOT_ERR_INVALID, "dx/dy need a points cost");
  UOT_TRY(check_cost_ptrs(c));
  UOT_TRY(check_device_ptr(alpha, "alpha"));
  UOT_TRY(check_device_ptr(beta, "beta"));
  UOT_TRY(check_device_ptr(f, "f"));
  UOT_TRY(check_device_ptr(g, "g"));
  if (dx) UOT_TRY(check_device_ptr(dx, "dx"));
  if (dy) UOT_TRY(check_device_ptr(dy, "dy"));
  if (dalpha) UOT_TRY(check_device_ptr(dalpha, "dalpha"));
  if (dbeta) UOT_TRY(check_device_ptr(dbeta, "dbeta"));
  const Layout L = make_layout(c, UOT_WS_BACKWARD);
  Workspace w;
  UOT_TRY(acquire(w, workspace, workspace_bytes, L.total));
  hipStream_t s = static_cast<hipStream_t>(stream);
  SolveState *st = at<SolveState>(w.ptr, L.state);
  UOT_TRY(prepare(c, alpha, beta, st, at<double>(w.ptr, L.center), s));
  double *masses = at<double>(w.ptr, L.masses);  // [0] = m(beta), [1] = m(alpha)
  for (int side = 0; side < 2; ++side) {
    const bool tx = side == 0;  // targets are the x side
    float *dpts = tx ? dx : dy;
    float *dw = tx ? dalpha : dbeta;
    if (dpts == nullptr && dw == nullptr) continue;
    if (dw) UOT_HIP(launch_sum(tx ? beta : alpha, tx ? c->m : c->n, masses + side, s));
    UOT_TRY(envelope_side(c, tx, alpha, beta, f, g, eps, tx ? rho1 : rho2, grad_out, st, w.ptr, L,
                          nullptr, 1, dw, masses + side, dpts, s, timed));
  }
  SolveState fin;
  UOT_TRY(read_state(st, fin, s));
  if ((fin.error & kErrWeights) || !fin.pos_a || !fin.pos_b)
    return fail(UOT_ERR_INVALID, "weights must be finite, >= 0, with positive total mass");
  return UOT_OK;
}

// ---------------------------------------------------------------------------------------
// Allocation-free backward. Its workspace is `scratch`, a device array of UOT_NOALLOC_BYTES
// that every GPU holds from the library's load until the process ends. In host code the
// array's name only stands in for it: its address on a device comes from
// hipGetSymbolAddress, looked up once per device (with that device current) on the first
// call there, and only that address is ever passed to kernels.
// ---------------------------------------------------------------------------------------
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

uot_status noalloc_scratch(void **out) {
  int dev = -1;
  UOT_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices)
    return fail(UOT_ERR_INVALID, "device %d beyond the %d the library tracks", dev, kMaxDevices);
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (g_scratch_ptr[dev] == nullptr) {
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || p == nullptr)
      return fail(UOT_ERR_HIP, "hipGetSymbolAddress(scratch) on device %d: %s", dev,
                  hipGetErrorString(e));
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return UOT_OK;
}

uot_status backward_noalloc(const uot_cost *c, const float *alpha, const float *beta, double eps,
                            double rho1, double rho2, const float *f, const float *g,
                            double grad_out, float *dx, float *dy, float *dalpha, float *dbeta,
                            void *stream) {
  UOT_TRY(check_cost(c));
  const size_t need = make_layout(c, UOT_WS_BACKWARD).total;
  if (need > UOT_NOALLOC_BYTES)
    return fail(UOT_ERR_WORKSPACE,
                "the backward of this problem needs %zu bytes of workspace; the allocation-free "
                "entry point holds %zu (use uot_backward)", need, (size_t)UOT_NOALLOC_BYTES);
  void *ws = nullptr;
  UOT_TRY(noalloc_scratch(&ws));
  return backward(c, alpha, beta, eps, rho1, rho2, f, g, grad_out, dx, dy, dalpha, dbeta, ws,
                  UOT_NOALLOC_BYTES, stream, false);
}

// ---------------------------------------------------------------------------------------
// Batched TI Sinkhorn
// ---------------------------------------------------------------------------------------
// Work items of the batched solver, at four levels: chunks of up to 256 targets (level 0,
// coarse: four per lane), 128 (level 1, fine: two per lane) or 64 (level 2, finest: one per
// lane); the remainder of a problem is one item (four, two or one targets per lane above 128,
// above 64, up to 64). Level 3 (split) takes the chunks of level 2 and splits their sources
// into ranges of kBatchSplitLen, one item each, merged by the last of them to finish (its own
// kernel). Finer items cost more per entry (fewer targets share each source read, and split
// items merge partials) but shorten the longest item, which bounds a launch once few problems
// run; the automatic plan (autotuned, below) starts at one level and may move to a finer one.
constexpr int kBatchLevels = 4;
constexpr int kBatchSplitLevel = 3;
int64_t batch_item_len(int64_t rem, int level = 0) {
  const int64_t cap = (int64_t)256 >> (level < 2 ? level : 2);
  return rem < cap ? rem : cap;
}
int64_t batch_source_ranges(int64_t ns, int level) {
  return level == kBatchSplitLevel ? (ns + kBatchSplitLen - 1) / kBatchSplitLen : 1;
}
// items of a problem with nt targets and ns sources at one level
int64_t batch_items(int64_t nt, int64_t ns, int level = 0) {
  int64_t k = 0;
  for (int64_t t0 = 0; t0 < nt; t0 += batch_item_len(nt - t0, level)) ++k;
  return k * batch_source_ranges(ns, level);
}

struct BatchLayout {
  size_t state = 0, mu = 0, offN = 0, offM = 0;
  size_t items_g[kBatchLevels] = {}, items_f[kBatchLevels] = {};   // per item level
  size_t pitem_g[kBatchLevels] = {}, pitem_f[kBatchLevels] = {};
  int n_items_g[kBatchLevels] = {}, n_items_f[kBatchLevels] = {};
  size_t act_g = 0, act_f = 0, ctrs = 0, part_g = 0, part_f = 0, tick_g = 0, tick_f = 0;
  size_t items2_g = 0, items2_f = 0, spart_g = 0, spart_f = 0, gtick_g = 0, gtick_f = 0;
  size_t pot_x = 0, pot_y = 0, rec_x = 0, rec_y = 0, lref_x = 0, lref_y = 0, total = 0;
  int64_t totN = 0, totM = 0;
};

// Workspace of uot_fw1d_batched: device offsets and the per-point scratch of the solver.
struct FwLayout {
  size_t offN = 0, offM = 0, fb = 0, gb = 0, Ac = 0, Bc = 0, r = 0, s = 0;
  size_t total = 0;
  int64_t totN = 0, totM = 0;
};

uot_status fw_layout(int32_t B, const int64_t *offN, const int64_t *offM, FwLayout &L) {
  if (B < 1) return fail(UOT_ERR_INVALID, "B=%d must be >= 1", B);
  if (offN == nullptr || offM == nullptr) return fail(UOT_ERR_INVALID, "offN/offM are NULL");
  if (offN[0] != 0 || offM[0] != 0) return fail(UOT_ERR_INVALID, "offN[0] and offM[0] must be 0");
  for (int p = 0; p < B; ++p) {
    const int64_t n = offN[p + 1] - offN[p], m = offM[p + 1] - offM[p];
    if (n < 1 || m < 1) return fail(UOT_ERR_INVALID, "problem %d has n=%lld, m=%lld (must be >= 1)", p, (long long)n, (long long)m);
    if (n > (1 << 30) || m > (1 << 30)) return fail(UOT_ERR_INVALID, "problem %d is too large", p);
  }
  L.totN = offN[B];
  L.totM = offM[B];
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off = align_up(off + bytes);
    return o;
  };
  L.offN = take((size_t)(B + 1) * sizeof(int64_t));
  L.offM = take((size_t)(B + 1) * sizeof(int64_t));
  L.fb = take((size_t)L.totN * sizeof(double));
  L.Ac = take((size_t)L.totN * sizeof(double));
  L.r = take((size_t)L.totN * sizeof(double));
  L.gb = take((size_t)L.totM * sizeof(double));
  L.Bc = take((size_t)L.totM * sizeof(double));
  L.s = take((size_t)L.totM * sizeof(double));
  L.total = off;
  return UOT_OK;
}

uot_status fw1d(int32_t B, const int64_t *offN, const int64_t *offM, const float *x, const float *y,
                const float *alpha, const float *beta, const double *rho1, const double *rho2,
                double p, int32_t line_search, int32_t max_iter, double tol, float *f, float *g,
                int32_t *iters, double *gap, int32_t *status, void *workspace,
                size_t workspace_bytes, void *stream) {
  FwLayout L;
  UOT_TRY(fw_layout(B, offN, offM, L));
  if (!(p >= 1.0) || !std::isfinite(p)) return fail(UOT_ERR_INVALID, "p=%g must be finite and >= 1", p);
  if (line_search != 0 && line_search != 1) return fail(UOT_ERR_INVALID, "line_search=%d must be 0 or 1", line_search);
  if (max_iter < 1) return fail(UOT_ERR_INVALID, "max_iter=%d must be >= 1", max_iter);
  if (!(tol >= 0.0) || !std::isfinite(tol)) return fail(UOT_ERR_INVALID, "tol=%g must be finite and >= 0", tol);
  UOT_TRY(check_device_ptr(x, "x"));
  UOT_TRY(check_device_ptr(y, "y"));
  UOT_TRY(check_device_ptr(alpha, "alpha"));
  UOT_TRY(check_device_ptr(beta, "beta"));
  UOT_TRY(check_device_ptr(rho1, "rho1"));
  UOT_TRY(check_device_ptr(rho2, "rho2"));
  UOT_TRY(check_device_ptr(f, "f"));
  UOT_TRY(check_device_ptr(g, "g"));
  UOT_TRY(check_device_ptr(iters, "iters"));
  UOT_TRY(check_device_ptr(gap, "gap"));
  UOT_TRY(check_device_ptr(status, "status"));
  Workspace w;
  UOT_TRY(acquire(w, workspace, workspace_bytes, L.total));
  hipStream_t s = static_cast<hipStream_t>(stream);
  UOT_HIP(hipMemcpyAsync(at<int64_t>(w.ptr, L.offN), offN, (size_t)(B + 1) * sizeof(int64_t),
                         hipMemcpyHostToDevice, s));
  UOT_HIP(hipMemcpyAsync(at<int64_t>(w.ptr, L.offM), offM, (size_t)(B + 1) * sizeof(int64_t),
                         hipMemcpyHostToDevice, s));
  UOT_HIP(hipStreamSynchronize(s));  // the host tables must outlive the copies
  FwLaunch l;
  l.B = B;
  l.offN = at<int64_t>(w.ptr, L.offN);
  l.offM = at<int64_t>(w.ptr, L.offM);
  l.x = x;
  l.y = y;
  l.alpha = alpha;
  l.beta = beta;
  l.rho1 = rho1;
  l.rho2 = rho2;
  l.p = p;
  l.line_search = line_search;
  l.max_iter = max_iter;
  l.tol = tol;
  l.fb = at<double>(w.ptr, L.fb);
  l.gb = at<double>(w.ptr, L.gb);
  l.Ac = at<double>(w.ptr, L.Ac);
  l.Bc = at<double>(w.ptr, L.Bc);
  l.r = at<double>(w.ptr, L.r);
  l.s = at<double>(w.ptr, L.s);
  l.f = f;
  l.g = g;
  l.iters = iters;
  l.gap = gap;
  l.status = status;
  const int cus = device_cus();
  l.max_blocks = cus > 0 ? 2 * cus : 512;
  UOT_HIP(launch_fw1d(l, s));
  if (w.owned) UOT_HIP(hipStreamSynchronize(s));  // the workspace is freed on return
  return UOT_OK;
}

// Workspace of uot_fw1d_barycenter: device offsets and per-point scratch.
struct BaryLayout {
  size_t off = 0, fb = 0, Ac = 0, r = 0, total = 0;
  int64_t tot = 0;
};

uot_status bary_layout(int32_t B, int32_t K, const int64_t *off, BaryLayout &L) {
  if (B < 1) return fail(UOT_ERR_INVALID, "B=%d must be >= 1", B);
  if (K < 2 || K > kBaryMaxMeasures) return fail(UOT_ERR_INVALID, "K=%d not in [2, %d]", K, kBaryMaxMeasures);
  if (off == nullptr) return fail(UOT_ERR_INVALID, "off is NULL");
  if (off[0] != 0) return fail(UOT_ERR_INVALID, "off[0] must be 0");
  for (int64_t m = 0; m < (int64_t)B * K; ++m) {
    const int64_t n = off[m + 1] - off[m];
    if (n < 1) return fail(UOT_ERR_INVALID, "measure %lld has %lld points (must be >= 1)", (long long)m, (long long)n);
    if (n > (1 << 30)) return fail(UOT_ERR_INVALID, "measure %lld is too large", (long long)m);
  }
  L.tot = off[(int64_t)B * K];
  size_t o = 0;
  auto take = [&](size_t bytes) {
    const size_t r = o;
    o = align_up(o + bytes);
    return r;
  };
  L.off = take(((size_t)B * K + 1) * sizeof(int64_t));
  L.fb = take((size_t)L.tot * sizeof(double));
  L.Ac = take((size_t)L.tot * sizeof(double));
  L.r = take((size_t)L.tot * sizeof(double));
  L.total = o;
  return UOT_OK;
}

uot_status fw_barycenter(int32_t B, int32_t K, const int64_t *off, const float *x,
                         const float *alpha, const double *w, const double *rho, int32_t max_iter,
                         double tol, float *f, float *bary_x, float *bary_w, int32_t *iters,
                         double *gap, int32_t *status, void *workspace, size_t workspace_bytes,
                         void *stream) {
  BaryLayout L;
  UOT_TRY(bary_layout(B, K, off, L));
  if (max_iter < 1) return fail(UOT_ERR_INVALID, "max_iter=%d must be >= 1", max_iter);
  if (!(tol >= 0.0) || !std::isfinite(tol)) return fail(UOT_ERR_INVALID, "tol=%g must be finite and >= 0", tol);
  UOT_TRY(check_device_ptr(x, "x"));
  UOT_TRY(check_device_ptr(alpha, "alpha"));
  UOT_TRY(check_device_ptr(w, "w"));
  UOT_TRY(check_device_ptr(rho, "rho"));
  UOT_TRY(check_device_ptr(f, "f"));
  UOT_TRY(check_device_ptr(bary_x, "bary_x"));
  UOT_TRY(check_device_ptr(bary_w, "bary_w"));
  UOT_TRY(check_device_ptr(iters, "iters"));
  UOT_TRY(check_device_ptr(gap, "gap"));
  UOT_TRY(check_device_ptr(status, "status"));
  Workspace ws;
  UOT_TRY(acquire(ws, workspace, workspace_bytes, L.total));
  hipStream_t s = static_cast<hipStream_t>(stream);
  UOT_HIP(hipMemcpyAsync(at<int64_t>(ws.ptr, L.off), off, ((size_t)B * K + 1) * sizeof(int64_t),
                         hipMemcpyHostToDevice, s));
  UOT_HIP(hipStreamSynchronize(s));  // the host table must outlive the copy
  BaryLaunch l;
  l.B = B;
  l.K = K;
  l.off = at<int64_t>(ws.ptr, L.off);
  l.x = x;
  l.alpha = alpha;
  l.w = w;
  l.rho = rho;
  l.max_iter = max_iter;
  l.tol = tol;
  l.fb = at<double>(ws.ptr, L.fb);
  l.Ac = at<double>(ws.ptr, L.Ac);
  l.r = at<double>(ws.ptr, L.r);
  l.f = f;
  l.bx = bary_x;
  l.bw = bary_w;
  l.iters = iters;
  l.gap = gap;
  l.status = status;
  const int cus = device_cus();
  l.max_blocks = cus > 0 ? 2 * cus : 512;
  UOT_HIP(launch_fw_bary(l, s));
  if (ws.owned) UOT_HIP(hipStreamSynchronize(s));  // the workspace is freed on return
  return UOT_OK;
}

// Process-wide settings of the batched solver: the work-item plan, and a per-chunk trace of
// the last solve (load statistics), guarded by a mutex.
enum BatchPlan : int {
  kPlanAuto = 0, kPlanCoarse = 1, kPlanFine = 2, kPlanSwitchAfterFirst = 3, kPlanFinest = 4,
  kPlanSplit = 5
};
struct BatchTraceRow {
  double chunk, fine, running, items_g, items_f, work, busy_ticks, ticks, resident_waves;
};
std::mutex g_batch_mu;
int g_batch_plan = kPlanAuto;
bool g_batch_trace_on = false;
std::vector<BatchTraceRow> g_batch_trace;

int batched_plan() {
  std::lock_guard<std::mutex> lk(g_batch_mu);
  return g_batch_plan;
}

// Autotuned plan (automatic plan): a candidate starts at item level lv0 and moves to lv1
// once the busier side has at most tau x (resident waves) active items. For each size
// signature (device, B, d, check_every, tol > 0, and log2 buckets of sum N, sum M, max N,
// max M) the first calls each take one candidate, timed on the host from the first chunk to
// the end of the solve, and later calls take the fastest. The level changes only how targets
// are grouped into items (the order of the per-problem partial sums), not the arithmetic of
// any target.
struct BatchCand {
  int lv0, lv1;
  double tau;
};
constexpr BatchCand kBatchCand[] = {{0, 0, 0.0}, {0, 1, 2.0}, {0, 1, 8.0}, {1, 1, 0.0},
                                    {1, 2, 2.0}, {1, 2, 8.0}, {2, 2, 0.0}, {1, 3, 2.0},
                                    {1, 3, 0.5}};
constexpr int kNumBatchCand = (int)(sizeof(kBatchCand) / sizeof(kBatchCand[0]));
typedef std::tuple<int, int, int, int, int, int, int, int, int> BatchSig;
struct BatchTune {
  double ms[kNumBatchCand];
  int claimed = 0;  // candidates handed out so far (in order)
  BatchTune() {
    for (double &v : ms) v = INFINITY;
  }
};
std::map<BatchSig, BatchTune> g_batch_tune;  // guarded by g_batch_mu
thread_local BatchCand g_batch_last{-1, -1, -1.0};

int log2_bucket(int64_t v) {
  int b = 0;
  while (v > 1) {
    v >>= 1;
    ++b;
  }
  return b;
}

BatchSig batch_sig(int32_t B, const int64_t *offN, const int64_t *offM, int32_t d,
                   int32_t check_every, double tol) {
  int64_t mn = 0, mm = 0;
  for (int p = 0; p < B; ++p) {
    const int64_t n = offN[p + 1] - offN[p], m = offM[p + 1] - offM[p];
    mn = n > mn ? n : mn;
    mm = m > mm ? m : mm;
  }
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) {
    (void)hipGetLastError();
    dev = 0;
  }
  return BatchSig(dev, B, d, check_every, tol > 0.0 ? 1 : 0, log2_bucket(offN[B]),
                  log2_bucket(offM[B]), log2_bucket(mn), log2_bucket(mm));
}
bool batched_trace_enabled() {
  std::lock_guard<std::mutex> lk(g_batch_mu);
  return g_batch_trace_on;
}

uot_status batched_layout(int32_t B, const int64_t *offN, const int64_t *offM, int32_t d,
                          BatchLayout &L) {
  if (B < 1) return fail(UOT_ERR_INVALID, "B=%d must be >= 1", B);
  if (offN == nullptr || offM == nullptr) return fail(UOT_ERR_INVALID, "offN/offM are NULL");
  if (d < 1 || d > kBatchMaxDim) return fail(UOT_ERR_INVALID, "batched d=%d not in [1, %d]", d, kBatchMaxDim);
  if (offN[0] != 0 || offM[0] != 0) return fail(UOT_ERR_INVALID, "offN[0] and offM[0] must be 0");
  int64_t ig[kBatchLevels] = {}, jf[kBatchLevels] = {};
  for (int p = 0; p < B; ++p) {
    const int64_t n = offN[p + 1] - offN[p], m = offM[p + 1] - offM[p];
    if (n < 1 || m < 1) return fail(UOT_ERR_INVALID, "problem %d has n=%lld, m=%lld (must be >= 1)", p, (long long)n, (long long)m);
    if (n > (1 << 30) || m > (1 << 30)) return fail(UOT_ERR_INVALID, "problem %d is too large", p);
    for (int lv = 0; lv < kBatchLevels; ++lv) {
      ig[lv] += batch_items(m, n, lv);
      jf[lv] += batch_items(n, m, lv);
    }
  }
  int64_t mg = 0, mf = 0;  // the most items of any level
  for (int lv = 0; lv < kBatchLevels; ++lv) {
    mg = ig[lv] > mg ? ig[lv] : mg;
    mf = jf[lv] > mf ? jf[lv] : mf;
  }
  if (mg > (1 << 30) || mf > (1 << 30)) return fail(UOT_ERR_INVALID, "too many work items");
  for (int lv = 0; lv < kBatchLevels; ++lv) {
    L.n_items_g[lv] = (int)ig[lv];
    L.n_items_f[lv] = (int)jf[lv];
  }
  L.totN = offN[B];
  L.totM = offM[B];
  const int stride = batched_rec_stride(d);
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off = align_up(off + bytes);
    return o;
  };
  L.state = take((size_t)B * sizeof(BatchState));
  L.mu = take((size_t)B * kBatchMaxDim * sizeof(double));
  L.offN = take((size_t)(B + 1) * sizeof(int64_t));
  L.offM = take((size_t)(B + 1) * sizeof(int64_t));
  for (int lv = 0; lv < kBatchLevels; ++lv) {
    L.items_g[lv] = take((size_t)L.n_items_g[lv] * sizeof(int4));
    L.items_f[lv] = take((size_t)L.n_items_f[lv] * sizeof(int4));
    L.pitem_g[lv] = take((size_t)(B + 1) * sizeof(int));
    L.pitem_f[lv] = take((size_t)(B + 1) * sizeof(int));
  }
  // active lists and item partials serve every level
  L.act_g = take((size_t)mg * sizeof(int));
  L.act_f = take((size_t)mf * sizeof(int));
  L.ctrs = take(sizeof(BatchCounters));
  L.part_g = take((size_t)mg * sizeof(BlockPart));
  L.part_f = take((size_t)mf * sizeof(BlockPart));
  // split level: source ranges and groups, per-target partials, group counters
  const int ns_g = L.n_items_g[kBatchSplitLevel], ns_f = L.n_items_f[kBatchSplitLevel];
  L.items2_g = take((size_t)ns_g * sizeof(int4));
  L.items2_f = take((size_t)ns_f * sizeof(int4));
  L.spart_g = take((size_t)ns_g * 64 * sizeof(float2));
  L.spart_f = take((size_t)ns_f * 64 * sizeof(float2));
  L.gtick_g = take((size_t)ns_g * sizeof(int));
  L.gtick_f = take((size_t)ns_f * sizeof(int));
  L.tick_g = take((size_t)B * sizeof(int));
  L.tick_f = take((size_t)B * sizeof(int));
  L.pot_x = take((size_t)L.totN * sizeof(float));
  L.pot_y = take((size_t)L.totM * sizeof(float));
  L.rec_x = take((size_t)L.totN * stride * sizeof(float));
  L.rec_y = take((size_t)L.totM * stride * sizeof(float));
  L.lref_x = take((size_t)L.totN * sizeof(float));
  L.lref_y = take((size_t)L.totM * sizeof(float));
  L.total = off;
  return UOT_OK;
}

// Work items of one side: (problem, first target, count, item index), grouped by problem,
// and at the split level (source offset in the problem, source count, first slot of the
// group, group size) for each. Items in problem order (a problem's items are taken by
// neighbouring waves, which share its source records in L2; ordering the table longest-first
// was measured slower on batch2d: 2.30e12 against 2.63e12 updates/s); the slots of problem p
// are [pitem[p], pitem[p+1]), a group's slots are consecutive.
void build_items(int32_t B, const int64_t *off, const int64_t *off_s, std::vector<int4> &items,
                 std::vector<int4> &items2, std::vector<int> &pitem, int level) {
  items.clear();
  items2.clear();
  pitem.assign((size_t)B + 1, 0);
  for (int p = 0; p < B; ++p) {
    pitem[p] = (int)items.size();
    const int64_t n = off[p + 1] - off[p], ns = off_s[p + 1] - off_s[p];
    const int nr = (int)batch_source_ranges(ns, level);
    for (int64_t t0 = 0; t0 < n;) {
      const int cnt = (int)batch_item_len(n - t0, level);
      const int first = (int)items.size();
      for (int r = 0; r < nr; ++r) {
        const int64_t sb = (int64_t)r * kBatchSplitLen;
        const int64_t sc = nr == 1 ? ns : (ns - sb < kBatchSplitLen ? ns - sb : kBatchSplitLen);
        items.push_back(make_int4(p, (int)t0, cnt, (int)items.size()));
        if (level == kBatchSplitLevel) items2.push_back(make_int4((int)sb, (int)sc, first, nr));
      }
      t0 += cnt;
    }
  }
  pitem[B] = (int)items.size();
}

struct GraphGuard {
  hipGraph_t g = nullptr;
  hipGraphExec_t e = nullptr;
  hipStream_t cs = nullptr;
  ~GraphGuard() {
    if (e) (void)hipGraphExecDestroy(e);
    if (g) (void)hipGraphDestroy(g);
    if (cs) (void)hipStreamDestroy(cs);
  }
};

uot_status ti_batched(int32_t B, const int64_t *offN, const int64_t *offM, int32_t d, double p,
                      const float *x, const float *y, const float *alpha, const float *beta,
                      const double *eps, const double *rho1, const double *rho2, int32_t max_iter,
                      double tol, int32_t check_every, float *f, float *g, int32_t *iters,
                      int32_t *status, void *workspace, size_t workspace_bytes, void *stream) {
  BatchLayout L;
  UOT_TRY(batched_layout(B, offN, offM, d, L));
  if (!std::isfinite(p) || p < 1.0) return fail(UOT_ERR_INVALID, "exponent p=%g must be finite and >= 1", p);
  if (max_iter < 1) return fail(UOT_ERR_INVALID, "max_iter=%d must be >= 1", max_iter);
  if (!(tol >= 0.0) || !std::isfinite(tol)) return fail(UOT_ERR_INVALID, "tol=%g must be finite and >= 0", tol);
  if (check_every < 1) return fail(UOT_ERR_INVALID, "check_every=%d must be >= 1", check_every);
  const void *ptrs[] = {x, y, alpha, beta, eps, rho1, rho2, f, g, iters, status};
  const char *names[] = {"x", "y", "alpha", "beta", "eps", "rho1", "rho2", "f", "g", "iters", "status"};
  for (int i = 0; i < 11; ++i) UOT_TRY(check_device_ptr(ptrs[i], names[i]));
  Workspace w;
  UOT_TRY(acquire(w, workspace, workspace_bytes, L.total));
  hipStream_t s = static_cast<hipStream_t>(stream);

  std::vector<int4> items[2][kBatchLevels];  // [side: 0 g-step, 1 f-step][level]
  std::vector<int4> items2[2][kBatchLevels];  // split level only
  std::vector<int> pitem[2][kBatchLevels];
  char *ws = static_cast<char *>(w.ptr);
  UOT_HIP(hipMemcpyAsync(ws + L.offN, offN, (size_t)(B + 1) * sizeof(int64_t), hipMemcpyHostToDevice, s));
  UOT_HIP(hipMemcpyAsync(ws + L.offM, offM, (size_t)(B + 1) * sizeof(int64_t), hipMemcpyHostToDevice, s));
  for (int lv = 0; lv < kBatchLevels; ++lv) {
    build_items(B, offM, offN, items[0][lv], items2[0][lv], pitem[0][lv], lv);  // g-step: targets y
    build_items(B, offN, offM, items[1][lv], items2[1][lv], pitem[1][lv], lv);  // f-step: targets x
    if (lv == kBatchSplitLevel) {
      UOT_HIP(hipMemcpyAsync(ws + L.items2_g, items2[0][lv].data(), items2[0][lv].size() * sizeof(int4),
                             hipMemcpyHostToDevice, s));
      UOT_HIP(hipMemcpyAsync(ws + L.items2_f, items2[1][lv].data(), items2[1][lv].size() * sizeof(int4),
                             hipMemcpyHostToDevice, s));
    }
    UOT_HIP(hipMemcpyAsync(ws + L.items_g[lv], items[0][lv].data(), items[0][lv].size() * sizeof(int4),
                           hipMemcpyHostToDevice, s));
    UOT_HIP(hipMemcpyAsync(ws + L.items_f[lv], items[1][lv].data(), items[1][lv].size() * sizeof(int4),
                           hipMemcpyHostToDevice, s));
    UOT_HIP(hipMemcpyAsync(ws + L.pitem_g[lv], pitem[0][lv].data(), pitem[0][lv].size() * sizeof(int),
                           hipMemcpyHostToDevice, s));
    UOT_HIP(hipMemcpyAsync(ws + L.pitem_f[lv], pitem[1][lv].data(), pitem[1][lv].size() * sizeof(int),
                           hipMemcpyHostToDevice, s));
  }
  UOT_HIP(hipStreamSynchronize(s));  // the host tables must outlive the copies

  BatchedArgs a;
  a.B = B;
  a.d = d;
  a.mode = kPower;  // the cost through the differences, p = 2 included
  a.half_p = (float)(0.5 * p);
  a.offN = at<int64_t>(w.ptr, L.offN);
  a.offM = at<int64_t>(w.ptr, L.offM);
  a.x = x;
  a.y = y;
  a.alpha = alpha;
  a.beta = beta;
  a.eps = eps;
  a.rho1 = rho1;
  a.rho2 = rho2;
  a.max_iter = max_iter;
  a.tol = tol;
  a.check_every = check_every;
  a.state = at<BatchState>(w.ptr, L.state);
  a.mu = at<double>(w.ptr, L.mu);
  a.pot_x = at<float>(w.ptr, L.pot_x);
  a.pot_y = at<float>(w.ptr, L.pot_y);
  a.rec_x = at<float>(w.ptr, L.rec_x);
  a.rec_y = at<float>(w.ptr, L.rec_y);
  a.lref_x = at<float>(w.ptr, L.lref_x);
  a.lref_y = at<float>(w.ptr, L.lref_y);
  a.items_g = at<int4>(w.ptr, L.items_g[0]);
  a.items_f = at<int4>(w.ptr, L.items_f[0]);
  a.pitem_g = at<int>(w.ptr, L.pitem_g[0]);
  a.pitem_f = at<int>(w.ptr, L.pitem_f[0]);
  a.n_items_g = L.n_items_g[0];
  a.n_items_f = L.n_items_f[0];
  a.act_g = at<int>(w.ptr, L.act_g);
  a.act_f = at<int>(w.ptr, L.act_f);
  BatchCounters *ctrs = at<BatchCounters>(w.ptr, L.ctrs);
  a.nact_g = &ctrs->nact_g;
  a.nact_f = &ctrs->nact_f;
  a.ctr_g = &ctrs->ctr_g;
  a.ctr_f = &ctrs->ctr_f;
  a.running = &ctrs->running;
  const bool tracing = batched_trace_enabled();
  a.stats = tracing ? ctrs : nullptr;
  if (tracing) UOT_HIP(hipMemsetAsync(ctrs, 0, sizeof(BatchCounters), s));
  a.part_g = at<BlockPart>(w.ptr, L.part_g);
  a.part_f = at<BlockPart>(w.ptr, L.part_f);
  a.ticket_g = at<int>(w.ptr, L.tick_g);
  a.ticket_f = at<int>(w.ptr, L.tick_f);
  a.items2_g = a.items2_f = nullptr;
  a.spart_g = a.spart_f = nullptr;
  a.gtick_g = a.gtick_f = nullptr;
  // group counters of the split level start at zero (each group's last item resets its own)
  UOT_HIP(hipMemsetAsync(ws + L.gtick_g, 0, (size_t)L.n_items_g[kBatchSplitLevel] * sizeof(int), s));
  UOT_HIP(hipMemsetAsync(ws + L.gtick_f, 0, (size_t)L.n_items_f[kBatchSplitLevel] * sizeof(int), s));

  const int cus = device_cus();
  const int per_cu = batched_half_blocks_per_cu(a);
  const int blocks = (cus > 0 ? cus : 256) * (per_cu > 0 ? per_cu : 4);
  const int resident_waves = blocks * 4;

  // the same problems and buffers at each item level, with that level's item tables (the
  // split level runs its own kernel, with its own occupancy)
  BatchedArgs al[kBatchLevels];
  int blocks_lv[kBatchLevels];
  for (int lv = 0; lv < kBatchLevels; ++lv) {
    al[lv] = a;
    al[lv].items_g = at<int4>(w.ptr, L.items_g[lv]);
    al[lv].items_f = at<int4>(w.ptr, L.items_f[lv]);
    al[lv].pitem_g = at<int>(w.ptr, L.pitem_g[lv]);
    al[lv].pitem_f = at<int>(w.ptr, L.pitem_f[lv]);
    al[lv].n_items_g = L.n_items_g[lv];
    al[lv].n_items_f = L.n_items_f[lv];
    blocks_lv[lv] = blocks;
    if (lv == kBatchSplitLevel) {
      al[lv].items2_g = at<int4>(w.ptr, L.items2_g);
      al[lv].items2_f = at<int4>(w.ptr, L.items2_f);
      al[lv].spart_g = at<float2>(w.ptr, L.spart_g);
      al[lv].spart_f = at<float2>(w.ptr, L.spart_f);
      al[lv].gtick_g = at<int>(w.ptr, L.gtick_g);
      al[lv].gtick_f = at<int>(w.ptr, L.gtick_f);
      const int pc = batched_half_blocks_per_cu(al[lv]);
      blocks_lv[lv] = (cus > 0 ? cus : 256) * (pc > 0 ? pc : 4);
    }
  }

  // The plan: start at item level lv0 and move to lv1 (one finer, or the same) once the busier
  // side has at most tau x (resident waves) active items. The automatic plan takes the
  // autotuned candidate of this size signature (see kBatchCand).
  const int plan = batched_plan();
  int lv0 = 0, lv1 = 1, tune_idx = -1;
  double tau = 2.0;
  bool exploring = false, after_first = false;
  const BatchSig sig = batch_sig(B, offN, offM, d, check_every, tol);
  if (plan == kPlanCoarse) {
    lv1 = 0;
  } else if (plan == kPlanFine) {
    lv0 = lv1 = 1;
  } else if (plan == kPlanFinest) {
    lv0 = lv1 = 2;
  } else if (plan == kPlanSplit) {
    lv0 = lv1 = kBatchSplitLevel;
  } else if (plan == kPlanSwitchAfterFirst) {
    after_first = true;
  } else {
    {
      std::lock_guard<std::mutex> lk(g_batch_mu);
      BatchTune &bt = g_batch_tune[sig];
      if (bt.claimed < kNumBatchCand) {
        tune_idx = bt.claimed++;
        exploring = true;
      } else {
        tune_idx = 0;
        for (int i = 1; i < kNumBatchCand; ++i)
          if (bt.ms[i] < bt.ms[tune_idx]) tune_idx = i;
      }
    }
    lv0 = kBatchCand[tune_idx].lv0;
    lv1 = kBatchCand[tune_idx].lv1;
    tau = kBatchCand[tune_idx].tau;
  }
  g_batch_last = plan == kPlanAuto ? kBatchCand[tune_idx] : BatchCand{-1, -1, -1.0};
  auto want_next = [&](const BatchCounters &c, int chunks_done) {
    if (after_first) return chunks_done >= 1;
    return lv1 != lv0 && (double)(c.nact_g > c.nact_f ? c.nact_g : c.nact_f) <= tau * resident_waves;
  };

  UOT_HIP(launch_batched_init(al[lv0], s));
  UOT_HIP(launch_batched_compact(al[lv0], s));

  // One chunk of iterations (g and f half-steps) and the compaction, captured once per level
  // the plan uses.
  const int chunk = tol > 0.0 ? check_every : (max_iter < 64 ? max_iter : 64);
  auto capture = [&](const BatchedArgs &pa, int nblocks, GraphGuard &gg) -> uot_status {
    UOT_HIP(hipStreamCreateWithFlags(&gg.cs, hipStreamNonBlocking));
    UOT_HIP(hipStreamBeginCapture(gg.cs, hipStreamCaptureModeRelaxed));
    for (int i = 0; i < chunk; ++i) {
      hipError_t e = launch_batched_half(pa, 1, nblocks, gg.cs);
      if (e == hipSuccess) e = launch_batched_half(pa, 0, nblocks, gg.cs);
      if (e != hipSuccess) {
        hipGraph_t dead = nullptr;
        (void)hipStreamEndCapture(gg.cs, &dead);
        if (dead) (void)hipGraphDestroy(dead);
        return fail(UOT_ERR_HIP, "batched launch during capture: %s", hipGetErrorString(e));
      }
    }
    hipError_t e = launch_batched_compact(pa, gg.cs);
    hipError_t e2 = hipStreamEndCapture(gg.cs, &gg.g);
    if (e != hipSuccess || e2 != hipSuccess)
      return fail(UOT_ERR_HIP, "graph capture: %s", hipGetErrorString(e != hipSuccess ? e : e2));
    UOT_HIP(hipGraphInstantiate(&gg.e, gg.g, nullptr, nullptr, 0));
    return UOT_OK;
  };
  GraphGuard gg[kBatchLevels];
  UOT_TRY(capture(al[lv0], blocks_lv[lv0], gg[lv0]));
  if (lv1 != lv0) UOT_TRY(capture(al[lv1], blocks_lv[lv1], gg[lv1]));

  // host copies of the counters after each chunk (two slots, read one chunk late)
  PinnedState pin;
  UOT_HIP(hipHostMalloc(reinterpret_cast<void **>(&pin.h), 2 * sizeof(SolveState), hipHostMallocDefault));
  BatchCounters *cnt_h = reinterpret_cast<BatchCounters *>(pin.h);
  static_assert(3 * sizeof(BatchCounters) <= 2 * sizeof(SolveState), "counter slots");
  hipEvent_t ev[2] = {nullptr, nullptr};
  UOT_HIP(hipEventCreateWithFlags(&ev[0], hipEventDisableTiming));
  UOT_HIP(hipEventCreateWithFlags(&ev[1], hipEventDisableTiming));
  struct EvGuard {
    hipEvent_t *e;
    ~EvGuard() { (void)hipEventDestroy(e[0]); (void)hipEventDestroy(e[1]); }
  } evg{ev};
  std::vector<BatchTraceRow> trace;
  unsigned long long busy_prev = 0, t_prev = 0;
  auto record = [&](const BatchCounters &c, int chunk, int level) {
    if (!tracing) return;
    BatchTraceRow r;
    r.chunk = chunk;
    r.fine = level;
    r.running = c.running;
    r.items_g = c.nact_g;
    r.items_f = c.nact_f;
    r.work = c.work;
    r.busy_ticks = (double)(c.busy - busy_prev);
    r.ticks = chunk == 0 ? 0.0 : (double)(c.t_compact - t_prev);
    r.resident_waves = blocks_lv[level] * 4;
    busy_prev = c.busy;
    t_prev = c.t_compact;
    trace.push_back(r);
  };
  // counters right after initialisation: active coarse items of each side, problems running
  UOT_HIP(hipMemcpyAsync(&cnt_h[2], ctrs, sizeof(BatchCounters), hipMemcpyDeviceToHost, s));
  UOT_HIP(hipStreamSynchronize(s));
  record(cnt_h[2], 0, lv0);
  const int max_chunks = (max_iter + chunk - 1) / chunk;
  const auto t_start = std::chrono::steady_clock::now();
  int lv = lv0;
  if (cnt_h[2].running > 0) {
    if (lv1 != lv0 && !after_first && want_next(cnt_h[2], 0)) {
      UOT_HIP(launch_batched_compact(al[lv1], s));
      lv = lv1;
    }
    for (int c = 0; c < max_chunks; ++c) {
      UOT_HIP(hipGraphLaunch(gg[lv].e, s));
      UOT_HIP(hipMemcpyAsync(&cnt_h[c & 1], ctrs, sizeof(BatchCounters), hipMemcpyDeviceToHost, s));
      UOT_HIP(hipEventRecord(ev[c & 1], s));
      if (c >= 1) {
        UOT_HIP(hipEventSynchronize(ev[(c - 1) & 1]));
        const BatchCounters cnt = cnt_h[(c - 1) & 1];
        record(cnt, c, lv);
        if (cnt.running == 0) break;
        if (lv != lv1 && want_next(cnt, c)) {  // after chunk c (queued): rebuild the active lists
          UOT_HIP(launch_batched_compact(al[lv1], s));
          lv = lv1;
        }
      }
    }
  }
  UOT_HIP(launch_batched_finalize(a, f, g, iters, status, s));
  UOT_HIP(hipStreamSynchronize(s));
  if (exploring) {
    const double ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() -
                                                                t_start).count();
    std::lock_guard<std::mutex> lk(g_batch_mu);
    g_batch_tune[sig].ms[tune_idx] = ms;
  }
  if (tracing) {
    std::lock_guard<std::mutex> lk(g_batch_mu);
    g_batch_trace = trace;
  }
  return UOT_OK;
}

}  // namespace
}  // namespace uot

extern "C" {

size_t uot_workspace_bytes(const uot_cost *cost, int32_t which) {
  if (uot::check_cost(cost) != UOT_OK) return 0;
  if (which < UOT_WS_SOLVE || which > UOT_WS_ANDERSON) return 0;
  return uot::make_layout(cost, which).total;
}

uot_status uot_sinkhorn(const uot_cost *cost, const float *alpha, const float *beta,
                        const uot_params *params, float *f, float *g, void *workspace,
                        size_t workspace_bytes, uot_info *info, void *stream) {
  uot::g_last_error.clear();
  return uot::solve(cost, alpha, beta, params, f, g, workspace, workspace_bytes, info, stream, false);
}

uot_status uot_sinkhorn_anderson(const uot_cost *cost, const float *alpha, const float *beta,
                                 const uot_params *params, const uot_anderson *acc, float *f,
                                 float *g, void *workspace, size_t workspace_bytes,
                                 uot_info *info, void *stream) {
  uot::g_last_error.clear();
  const uot_status s = uot::check_anderson(acc);
  if (s != UOT_OK) return s;
  return uot::solve(cost, alpha, beta, params, f, g, workspace, workspace_bytes, info, stream,
                    false, acc);
}

uot_status uot_ti_sinkhorn_anderson(const uot_cost *cost, const float *alpha, const float *beta,
                                    const uot_params *params, const uot_anderson *acc, float *f,
                                    float *g, void *workspace, size_t workspace_bytes,
                                    uot_info *info, void *stream) {
  uot::g_last_error.clear();
  const uot_status s = uot::check_anderson(acc);
  if (s != UOT_OK) return s;
  return uot::solve(cost, alpha, beta, params, f, g, workspace, workspace_bytes, info, stream,
                    true, acc);
}

uot_status uot_sinkhorn_phi(const uot_cost *cost, const float *alpha, const float *beta,
                            const uot_params *params, const uot_phi *phi, float *f, float *g,
                            void *workspace, size_t workspace_bytes, uot_info *info,
                            void *stream) {
  uot::g_last_error.clear();
  const uot_status s = uot::check_phi(phi);
  if (s != UOT_OK) return s;
  return uot::solve(cost, alpha, beta, params, f, g, workspace, workspace_bytes, info, stream,
                    false, nullptr, phi);
}

uot_status uot_ti_sinkhorn(const uot_cost *cost, const float *alpha, const float *beta,
                           const uot_params *params, float *f, float *g, void *workspace,
                           size_t workspace_bytes, uot_info *info, void *stream) {
  uot::g_last_error.clear();
  return uot::solve(cost, alpha, beta, params, f, g, workspace, workspace_bytes, info, stream, true);
}

uot_status uot_dual_value(const uot_cost *cost, const float *alpha, const float *beta, double eps,
                          double rho1, double rho2, const float *f, const float *g, void *workspace,
                          size_t workspace_bytes, double *value, void *stream) {
  uot::g_last_error.clear();
  return uot::dual_value(cost, alpha, beta, eps, rho1, rho2, f, g, workspace, workspace_bytes, value,
                         stream);
}

uot_status uot_plan_apply(const uot_cost *cost, const float *alpha, const float *beta, double eps,
                          const float *f, const float *g, int32_t transpose, const float *V,
                          int32_t k, int64_t ldv, float *out, int64_t ldout, void *workspace,
                          size_t workspace_bytes, void *stream) {
  uot::g_last_error.clear();
  return uot::plan_apply(cost, alpha, beta, eps, f, g, transpose, V, k, ldv, out, ldout, workspace,
                         workspace_bytes, stream);
}

uot_status uot_backward(const uot_cost *cost, const float *alpha, const float *beta, double eps,
                        double rho1, double rho2, const float *f, const float *g, double grad_out,
                        float *dx, float *dy, float *dalpha, float *dbeta, void *workspace,
                        size_t workspace_bytes, void *stream) {
  uot::g_last_error.clear();
  return uot::backward(cost, alpha, beta, eps, rho1, rho2, f, g, grad_out, dx, dy, dalpha, dbeta,
                       workspace, workspace_bytes, stream);
}

uot_status uot_backward_noalloc(const uot_cost *cost, const float *alpha, const float *beta,
                                double eps, double rho1, double rho2, const float *f,
                                const float *g, double grad_out, float *dx, float *dy,
                                float *dalpha, float *dbeta, void *stream) {
  uot::g_last_error.clear();
  return uot::backward_noalloc(cost, alpha, beta, eps, rho1, rho2, f, g, grad_out, dx, dy,
                               dalpha, dbeta, stream);
}

int32_t uot_set_autotune(int32_t on) {
  return uot::g_autotune.exchange(on ? 1 : 0);
}

int32_t uot_set_points_kernel(int32_t variant) {
  if (variant < uot::kPointsAuto || variant > uot::kPointsDirect) return -1;
  const int32_t prev = uot::g_points_variant;
  uot::g_points_variant = variant;
  return prev;
}

void uot_profile_enable(int32_t period) {
  std::lock_guard<std::mutex> lk(uot::g_prof_mu);
  uot::g_prof_on = period > 0;
  uot::g_prof_period = period > 0 ? period : 1;
}

void uot_profile_reset(void) {
  std::lock_guard<std::mutex> lk(uot::g_prof_mu);
  for (auto &p : uot::g_prof) p = uot::ProfAcc();
}

int64_t uot_profile_read(int32_t kind, double *total_ms, double *total_entries) {
  if (kind < 0 || kind >= uot::kProfKinds) return -1;
  std::lock_guard<std::mutex> lk(uot::g_prof_mu);
  if (total_ms) *total_ms = uot::g_prof[kind].ms;
  if (total_entries) *total_entries = uot::g_prof[kind].entries;
  return uot::g_prof[kind].launches;
}

size_t uot_fw1d_barycenter_workspace_bytes(int32_t B, int32_t K, const int64_t *off) {
  uot::BaryLayout L;
  if (uot::bary_layout(B, K, off, L) != UOT_OK) return 0;
  return L.total;
}

uot_status uot_fw1d_barycenter(int32_t B, int32_t K, const int64_t *off, const float *x,
                               const float *alpha, const double *w, const double *rho,
                               int32_t max_iter, double tol, float *f, float *bary_x,
                               float *bary_w, int32_t *iters, double *gap, int32_t *status,
                               void *workspace, size_t workspace_bytes, void *stream) {
  uot::g_last_error.clear();
  return uot::fw_barycenter(B, K, off, x, alpha, w, rho, max_iter, tol, f, bary_x, bary_w, iters,
                            gap, status, workspace, workspace_bytes, stream);
}

size_t uot_fw1d_workspace_bytes(int32_t B, const int64_t *offN, const int64_t *offM) {
  uot::FwLayout L;
  if (uot::fw_layout(B, offN, offM, L) != UOT_OK) return 0;
  return L.total;
}

uot_status uot_fw1d_batched(int32_t B, const int64_t *offN, const int64_t *offM, const float *x,
                            const float *y, const float *alpha, const float *beta,
                            const double *rho1, const double *rho2, double p, int32_t line_search,
                            int32_t max_iter, double tol, float *f, float *g, int32_t *iters,
                            double *gap, int32_t *status, void *workspace,
                            size_t workspace_bytes, void *stream) {
  uot::g_last_error.clear();
  return uot::fw1d(B, offN, offM, x, y, alpha, beta, rho1, rho2, p, line_search, max_iter, tol,
                   f, g, iters, gap, status, workspace, workspace_bytes, stream);
}

int32_t uot_batched_last_plan(int32_t *start_level, int32_t *end_level, double *threshold) {
  const uot::BatchCand c = uot::g_batch_last;
  if (start_level) *start_level = c.lv0;
  if (end_level) *end_level = c.lv1;
  if (threshold) *threshold = c.tau;
  return c.lv0 >= 0 ? 1 : 0;
}

void uot_batched_autotune_reset(void) {
  std::lock_guard<std::mutex> lk(uot::g_batch_mu);
  uot::g_batch_tune.clear();
}

int32_t uot_batched_set_plan(int32_t plan) {
  if (plan < uot::kPlanAuto || plan > uot::kPlanSplit) return -1;
  std::lock_guard<std::mutex> lk(uot::g_batch_mu);
  const int32_t prev = uot::g_batch_plan;
  uot::g_batch_plan = plan;
  return prev;
}

void uot_batched_trace_enable(int32_t on) {
  std::lock_guard<std::mutex> lk(uot::g_batch_mu);
  uot::g_batch_trace_on = on != 0;
  if (!on) uot::g_batch_trace.clear();
}

int32_t uot_batched_trace_read(double *rows, int32_t max_rows) {
  std::lock_guard<std::mutex> lk(uot::g_batch_mu);
  const int32_t n = (int32_t)uot::g_batch_trace.size();
  if (rows != nullptr)
    for (int32_t i = 0; i < n && i < max_rows; ++i) {
      const uot::BatchTraceRow &r = uot::g_batch_trace[i];
      const double v[9] = {r.chunk, r.fine, r.running, r.items_g, r.items_f, r.work, r.busy_ticks,
                           r.ticks, r.resident_waves};
      for (int k = 0; k < 9; ++k) rows[(size_t)i * 9 + k] = v[k];
    }
  return n;
}

size_t uot_batched_workspace_bytes(int32_t B, const int64_t *offN, const int64_t *offM, int32_t d) {
  uot::BatchLayout L;
  if (uot::batched_layout(B, offN, offM, d, L) != UOT_OK) return 0;
  return L.total;
}

uot_status uot_ti_sinkhorn_batched(int32_t B, const int64_t *offN, const int64_t *offM, int32_t d,
                                   double p, const float *x, const float *y, const float *alpha,
                                   const float *beta, const double *eps, const double *rho1,
                                   const double *rho2, int32_t max_iter, double tol,
                                   int32_t check_every, float *f, float *g, int32_t *iters,
                                   int32_t *status, void *workspace, size_t workspace_bytes,
                                   void *stream) {
  uot::g_last_error.clear();
  return uot::ti_batched(B, offN, offM, d, p, x, y, alpha, beta, eps, rho1, rho2, max_iter, tol,
                         check_every, f, g, iters, status, workspace, workspace_bytes, stream);
}

const char *uot_status_string(uot_status s) {
  switch (s) {
    case UOT_OK: return "ok";
    case UOT_ERR_INVALID: return "invalid argument";
    case UOT_ERR_HIP: return "HIP runtime error";
    case UOT_ERR_NUMERIC: return "non-finite result";
    case UOT_ERR_WORKSPACE: return "workspace too small";
  }
  return "unknown status";
}

const char *uot_last_error(void) { return uot::g_last_error.c_str(); }

}  // extern "C"
