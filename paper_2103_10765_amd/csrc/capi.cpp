// C ABI of the G-BM3D library: argument validation, device workspace, the
// stage pipelines for one image and for batches (work lists, launches over
// all of a batch's items, hipGraph capture).  Every compute step runs in the library's HIP
// kernels.
#include <hip/hip_runtime.h>
#include <rocprofiler-sdk-roctx/roctx.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/gbm3d.h"
#include "kernels.h"
#include "pilot.h"

namespace {

// A named range on the host timeline (roctx) around each entry point and
// pipeline stage, so that a profiler's marker trace groups the launches of
// each (rocprofv3 --marker-trace); without a profiler attached it costs a
// call into an empty dispatch table.
struct TraceRange {
  explicit TraceRange(const char* name) { roctxRangePushA(name); }
  ~TraceRange() { roctxRangePop(); }
  TraceRange(const TraceRange&) = delete;
  TraceRange& operator=(const TraceRange&) = delete;
};

}  // namespace

using gbm3d::ImgRec;
using gbm3d::WorkList;

// Workspace of gbm3d_denoise_noalloc: one fixed array per device, reserved
// when the library's code object is loaded there and held until the process
// ends.  Its host-side name is only a stand-in for the symbol: host code
// reaches the memory through the address hipGetSymbolAddress returns for
// the current device (scratch_addr below), never through the name itself.
static __device__ __align__(256) unsigned char scratch[GBM3D_NOALLOC_SCRATCH_BYTES];

namespace {

struct Buffer {
  void* p = nullptr;
  size_t bytes = 0;
};

struct TimingRecord {
  const char* name;
  hipEvent_t start, stop;
};

thread_local std::string g_thread_error;

// Device address of `scratch` on each device, looked up once per device by
// gbm3d_create with that device current.
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_addr[kMaxDevices] = {};

hipError_t resolve_scratch(int dev) {
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch_addr[dev]) return hipSuccess;
  void* ptr = nullptr;
  const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess) return e;
  if (!ptr) return hipErrorInvalidSymbol;
  g_scratch_addr[dev] = ptr;
  return hipSuccess;
}

void* scratch_addr(int dev) {
  if (dev < 0 || dev >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  return g_scratch_addr[dev];
}

// Work lists of the batch phases: per-image prefix offsets of the items.
enum Phase { kNorm1, kBm1, kStack1, kGroup1, kReduce1, kNorm2, kBm2, kStack2, kGroup2, kReduce2, kPhases };

struct BatchPlan {
  std::vector<ImgRec> recs;
  std::vector<int> begin[kPhases];  // n + 1 each
  std::vector<int> start[kPhases];  // total / kItemBlock + 1 each: the image owning item kItemBlock * b
  int bm_method1 = GBM3D_BM_SHIFT, bm_method2 = GBM3D_BM_SHIFT;
  int bm_split1 = 1, bm_split2 = 1;
  int ht_shape = 0;  // stage-1 group kernel shape
  bool any_stage1 = false, any_stage2 = false;
};

// A block-matching launch choice recorded by the autotuner.
struct TuneEntry {
  int method = GBM3D_BM_SHIFT, split = 1;
  float ms = 0.0f;
};

// A stage-1 group-kernel shape recorded by the autotuner.
struct ShapeEntry {
  int shape = 0;
  float ms = 0.0f;
};

// Tuning key: group size, search window, shape class of the image(s).
struct TuneKey {
  int K, search, cls;
  bool operator<(const TuneKey& o) const {
    return K != o.K ? K < o.K : (search != o.search ? search < o.search : cls < o.cls);
  }
};

struct GraphEntry {
  std::string key;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

}  // namespace

struct gbm3d_ctx {
  int device = 0;
  int n_cu = 256;
  std::string err;
  Buffer stack_a, stack_b, idx, partials, basic, q, norm;
  // global stage 1
  Buffer gl_a, gl_b, gl_num, gl_idx, gl_shift, gl_pad, gl_out;
  // block-matching choices per (K, shape class)
  std::map<TuneKey, TuneEntry> tuned;
  std::map<TuneKey, ShapeEntry> tuned_shape;  // stage-1 group kernel, keyed by k_ht
  // batches
  Buffer batch_ws, batch_table;
  void* host_stage = nullptr;  // pinned staging of the batch table
  size_t host_stage_bytes = 0;
  hipEvent_t table_copied = nullptr;
  hipStream_t capture_stream = nullptr;
  GraphEntry graph;
  // learned pilot
  Buffer pilot_w, pilot_act, pilot_part;
  bool pilot_loaded = false;
  // per-kernel timing (off by default)
  bool timing = false;
  std::vector<TimingRecord> pending;
  std::vector<hipEvent_t> event_pool;
  std::map<std::string, std::pair<double, int64_t>> totals;
};

namespace {

int fail(gbm3d_ctx* ctx, int status, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  if (ctx)
    ctx->err = buf;
  else
    g_thread_error = buf;
  return status;
}

int hip_fail(gbm3d_ctx* ctx, hipError_t e, const char* what) {
  return fail(ctx, e == hipErrorOutOfMemory ? GBM3D_ENOMEM : GBM3D_EHIP, "%s: %s", what, hipGetErrorString(e));
}

#define HIP_TRY(ctx, expr, what)                          \
  do {                                                    \
    hipError_t e_ = (expr);                               \
    if (e_ != hipSuccess) return hip_fail(ctx, e_, what); \
  } while (0)

#define CHECK(expr)                \
  do {                             \
    int s_ = (expr);               \
    if (s_ != GBM3D_OK) return s_; \
  } while (0)

hipEvent_t take_event(gbm3d_ctx* ctx) {
  if (!ctx->event_pool.empty()) {
    hipEvent_t e = ctx->event_pool.back();
    ctx->event_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

// Runs one launch; with timing on, brackets it with events on its stream.
template <typename F>
hipError_t timed(gbm3d_ctx* ctx, const char* name, hipStream_t st, F&& launch) {
  if (!ctx->timing) return launch();
  hipEvent_t a = take_event(ctx), b = take_event(ctx);
  if (!a || !b) return hipErrorOutOfMemory;
  hipError_t e = hipEventRecord(a, st);
  if (e != hipSuccess) return e;
  e = launch();
  if (e != hipSuccess) return e;
  e = hipEventRecord(b, st);
  if (e != hipSuccess) return e;
  ctx->pending.push_back({name, a, b});
  return hipSuccess;
}

bool is_pow2_group(int k) { return k == 2 || k == 4 || k == 8 || k == 16 || k == 32; }

// Host-side validation; no side effects beyond the error text.
int check_params(gbm3d_ctx* ctx, const gbm3d_params& p) {
  if (p.struct_size != sizeof(gbm3d_params))
    return fail(ctx, GBM3D_EINVAL, "params.struct_size %u != %zu", p.struct_size, sizeof(gbm3d_params));
  if (p.patch != 8) return fail(ctx, GBM3D_EUNSUPPORTED, "patch %d unsupported (only 8)", p.patch);
  if (p.step != 3) return fail(ctx, GBM3D_EUNSUPPORTED, "step %d unsupported (only 3)", p.step);
  if (p.search < 1 || p.search > 39 || p.search % 2 == 0)
    return fail(ctx, GBM3D_EINVAL, "search %d must be odd and in [1, 39]", p.search);
  if (p.bm_split != 0 && p.bm_split != 1 && p.bm_split != 2 && p.bm_split != 4)
    return fail(ctx, GBM3D_EINVAL, "bm_split %d must be 0, 1, 2 or 4", p.bm_split);
  if (p.bm_method != GBM3D_BM_AUTO && p.bm_method != GBM3D_BM_SHIFT && p.bm_method != GBM3D_BM_CORR)
    return fail(ctx, GBM3D_EINVAL, "bm_method %d unknown", p.bm_method);
  return GBM3D_OK;
}

int check_shape(gbm3d_ctx* ctx, int H, int W, const gbm3d_params& p) {
  CHECK(check_params(ctx, p));
  const int lo = p.search > 8 ? p.search : 8;
  if (H < lo || W < lo || H > 32768 || W > 32768)
    return fail(ctx, GBM3D_EINVAL, "image %dx%d outside [%d, 32768]", H, W, lo);
  return GBM3D_OK;
}

int check_k(gbm3d_ctx* ctx, int K, const gbm3d_params& p, const char* name) {
  if (!is_pow2_group(K)) return fail(ctx, GBM3D_EINVAL, "%s %d must be one of 2, 4, 8, 16, 32", name, K);
  if (K > p.search * p.search) return fail(ctx, GBM3D_EINVAL, "%s %d exceeds search^2", name, K);
  return GBM3D_OK;
}

int check_sigma(gbm3d_ctx* ctx, float sigma) {
  if (!(sigma > 0.0f) || !std::isfinite(sigma))
    return fail(ctx, GBM3D_EINVAL, "sigma %g must be > 0 and finite", sigma);
  return GBM3D_OK;
}

int check_ht(gbm3d_ctx* ctx, const gbm3d_params& p) {
  if (!std::isfinite(p.ht_a) || !std::isfinite(p.ht_b)) return fail(ctx, GBM3D_EINVAL, "ht_a/ht_b must be finite");
  if (p.ht_weight < GBM3D_W_TV || p.ht_weight > GBM3D_W_UNIT)
    return fail(ctx, GBM3D_EINVAL, "ht_weight %d unknown", p.ht_weight);
  if (!(p.tv_eps_rel > 0.0f) || !std::isfinite(p.tv_eps_rel))
    return fail(ctx, GBM3D_EINVAL, "tv_eps_rel must be > 0 and finite");
  if (p.ht_source != GBM3D_HT_STACK && p.ht_source != GBM3D_HT_RECOMPUTE)
    return fail(ctx, GBM3D_EINVAL, "ht_source %d unknown", p.ht_source);
  return GBM3D_OK;
}

gbm3d_params resolve(const gbm3d_params* p) {
  gbm3d_params d;
  gbm3d_default_params(&d);
  return p ? *p : d;
}

int ensure(gbm3d_ctx* ctx, Buffer& b, size_t bytes, const char* name) {
  if (bytes <= b.bytes) return GBM3D_OK;
  if (std::getenv("GBM3D_FAULT_ALLOC"))
    return fail(ctx, GBM3D_ENOMEM, "workspace %s (%zu bytes): allocation failure injected", name, bytes);
  if (b.p) {
    // queued work may still read the old buffer
    HIP_TRY(ctx, hipDeviceSynchronize(), "hipDeviceSynchronize");
    HIP_TRY(ctx, hipFree(b.p), "hipFree");
    b.p = nullptr;
    b.bytes = 0;
  }
  const size_t rounded = (bytes + 4095) & ~static_cast<size_t>(4095);
  hipError_t e = hipMalloc(&b.p, rounded);
  if (e != hipSuccess) {
    b.p = nullptr;
    return fail(ctx, GBM3D_ENOMEM, "workspace %s (%zu bytes): %s", name, rounded, hipGetErrorString(e));
  }
  b.bytes = rounded;
  return GBM3D_OK;
}

struct DeviceGuard {
  int prev = -1;
  bool ok = false;
  explicit DeviceGuard(int dev) {
    if (hipGetDevice(&prev) != hipSuccess) prev = -1;
    ok = hipSetDevice(dev) == hipSuccess;
  }
  ~DeviceGuard() {
    if (prev >= 0) (void)hipSetDevice(prev);
  }
};

size_t align256(size_t x) { return (x + 255) & ~static_cast<size_t>(255); }
size_t stack_bytes(int H, int W) { return static_cast<size_t>(H) * W * 64 * sizeof(float); }
size_t n_refs(int H, int W) { return static_cast<size_t>((H + 2) / 3) * ((W + 2) / 3); }

ImgRec blank_rec(int H, int W, float sigma) {
  ImgRec r;
  std::memset(&r, 0, sizeof(r));
  r.H = H;
  r.W = W;
  r.sigma = sigma;
  return r;
}

// Shape class of a block-matching launch: floor(log2) of its 4x4 reference tiles.
int tile_class(long tiles) {
  int c = 0;
  while (tiles >= (2L << c)) ++c;
  return c;
}

struct BmChoice {
  int method, split;  // split 0: by size inside the launcher
};

// Explicit params win.  Zeros take the tuned choice of the class (same K and
// search); without one, the method of the nearest tuned class of the same K
// and search (split then by size), else the default.
BmChoice choose_bm(const gbm3d_ctx* ctx, const gbm3d_params& p, long tiles, int K) {
  BmChoice c{p.bm_method, p.bm_split};
  const int cls = tile_class(tiles);
  const auto it = ctx->tuned.find({K, p.search, cls});
  if (it != ctx->tuned.end()) {
    if (c.method == GBM3D_BM_AUTO) c.method = it->second.method;
    if (c.split == 0 && c.method == it->second.method) c.split = it->second.split;
  } else if (c.method == GBM3D_BM_AUTO) {
    int best = 1 << 30;
    for (const auto& kv : ctx->tuned) {
      const int d = std::abs(kv.first.cls - cls);
      if (kv.first.K == K && kv.first.search == p.search && d < best) {
        best = d;
        c.method = kv.second.method;
      }
    }
  }
  if (c.method == GBM3D_BM_AUTO) c.method = GBM3D_BM_CORR;  // the faster kernel on every measured shape
  return c;
}

// The stage-1 group-kernel shape: the tuned one of the class, else that of
// the nearest tuned class of the same k_ht and search, else two tiles per CU.
int choose_shape(const gbm3d_ctx* ctx, const gbm3d_params& p, long tiles) {
  const int cls = tile_class(tiles);
  const auto it = ctx->tuned_shape.find({p.k_ht, p.search, cls});
  if (it != ctx->tuned_shape.end()) return it->second.shape;
  int best = 1 << 30, shape = 0;
  for (const auto& kv : ctx->tuned_shape) {
    const int d = std::abs(kv.first.cls - cls);
    if (kv.first.K == p.k_ht && kv.first.search == p.search && d < best) {
      best = d;
      shape = kv.second.shape;
    }
  }
  return shape;
}

// The correlation kernel's norm table: r.norm when set, else the context's.
int bind_norm(gbm3d_ctx* ctx, ImgRec& r) {
  if (!r.norm) {
    CHECK(ensure(ctx, ctx->norm, gbm3d::norm_bytes(r.H, r.W), "norm table"));
    r.norm = static_cast<double*>(ctx->norm.p);
  }
  return GBM3D_OK;
}

// Block matching of one image (r.noisy, or r.pilot with use_pilot) into r.idx.
// norm_ready: the correlation kernel's norm table is already in r.norm (formed
// by the stack launch before it).
int run_match(gbm3d_ctx* ctx, ImgRec& r, int R, int K, const BmChoice& c, int use_pilot, hipStream_t st,
              bool norm_ready = false) {
  if (c.method == GBM3D_BM_CORR) {
    CHECK(bind_norm(ctx, r));
    if (!norm_ready)
      HIP_TRY(ctx, timed(ctx, "bm_norm", st, [&] { return gbm3d::launch_bm_norm(r, nullptr, R, use_pilot, 0, st); }),
              "norm table launch");
    HIP_TRY(ctx, timed(ctx, "bm", st, [&] {
              return gbm3d::launch_bm_corr(r, nullptr, R, K, c.split, use_pilot, 0, st);
            }),
            "block matching launch");
  } else {
    HIP_TRY(ctx, timed(ctx, "bm", st, [&] { return gbm3d::launch_bm(r, nullptr, R, K, c.split, use_pilot, 0, st); }),
            "block matching launch");
  }
  return GBM3D_OK;
}

int run_match(gbm3d_ctx* ctx, ImgRec& r, int R, int K, const gbm3d_params& p, int use_pilot, hipStream_t st) {
  return run_match(ctx, r, R, K, choose_bm(ctx, p, gbm3d::corr_tiles(r.H, r.W), K), use_pilot, st);
}

float tv_eps(const gbm3d_params& p, float sigma) { return p.tv_eps_rel * sigma * 64.0f * static_cast<float>(p.k_ht); }

// Device buffers of one image's stages: the context's workspace (grown on
// demand), or slices of the static scratch (gbm3d_denoise_noalloc).
struct Workspace {
  float* stack_a = nullptr;
  float* stack_b = nullptr;
  int16_t* idx = nullptr;
  unsigned long long* partials = nullptr;
  double* norm = nullptr;
};

// Stage 1 of one image into `basic` (and optionally its quantisation into q).
// ws: preassigned buffers, or NULL for the context's workspace.
int run_basic(gbm3d_ctx* ctx, const uint16_t* noisy, int H, int W, float sigma, const gbm3d_params& p,
              float* basic, uint16_t* q, hipStream_t st, const Workspace* ws = nullptr) {
  TraceRange trace("stage1");
  const int R = p.search / 2;
  const int recompute = p.ht_source == GBM3D_HT_RECOMPUTE ? 1 : 0;
  Workspace w;
  if (ws) {
    w = *ws;
  } else {
    // the recompute form transforms each matched block from its pixels: no stack
    if (!recompute) CHECK(ensure(ctx, ctx->stack_a, stack_bytes(H, W), "stack"));
    CHECK(ensure(ctx, ctx->idx, n_refs(H, W) * p.k_ht * sizeof(int16_t), "idx"));
    CHECK(ensure(ctx, ctx->partials, gbm3d::partials_bytes(H, W), "partials"));
    w.stack_a = static_cast<float*>(ctx->stack_a.p);
    w.idx = static_cast<int16_t*>(ctx->idx.p);
    w.partials = static_cast<unsigned long long*>(ctx->partials.p);
  }
  ImgRec r = blank_rec(H, W, sigma);
  r.noisy = noisy;
  r.basic = basic;
  r.q = q;
  r.stack_a = recompute ? nullptr : w.stack_a;
  r.idx = w.idx;
  r.partials = w.partials;
  r.norm = w.norm;
  r.eps = tv_eps(p, sigma);
  const BmChoice c = choose_bm(ctx, p, gbm3d::corr_tiles(H, W), p.k_ht);
  if (recompute) {
    CHECK(run_match(ctx, r, R, p.k_ht, c, 0, st));
    HIP_TRY(ctx, gbm3d::launch_clear_weights(r, st), "weight clearing launch");
  } else if (c.method == GBM3D_BM_CORR) {
    // the stack and the matcher's norm table in one launch, then the matching
    CHECK(bind_norm(ctx, r));
    HIP_TRY(ctx, timed(ctx, "stack_bior", st, [&] {
              return gbm3d::launch_stack_norm(r, 0, 0, 0, R, 0, st);
            }),
            "stack launch");
    CHECK(run_match(ctx, r, R, p.k_ht, c, 0, st, true));
  } else {
    CHECK(run_match(ctx, r, R, p.k_ht, c, 0, st));
    HIP_TRY(ctx, timed(ctx, "stack_bior", st, [&] { return gbm3d::launch_stack(r, nullptr, 0, 0, 0, 0, st); }),
            "stack launch");
  }
  HIP_TRY(ctx, timed(ctx, "group_ht", st, [&] {
            return gbm3d::launch_group_ht(r, nullptr, R, p.k_ht, p.ht_a, p.ht_b, p.ht_weight, p.keep_dc, recompute,
                                          choose_shape(ctx, p, gbm3d::corr_tiles(H, W)), 0, st);
          }),
          "hard-threshold group launch");
  HIP_TRY(ctx, timed(ctx, "reduce", st, [&] { return gbm3d::launch_reduce(r, nullptr, 0, 0, st); }),
          "aggregation launch");
  return GBM3D_OK;
}

int run_wiener(gbm3d_ctx* ctx, const uint16_t* noisy, const uint16_t* pilot, int H, int W, float sigma,
               const gbm3d_params& p, float* out, hipStream_t st, const Workspace* ws = nullptr) {
  TraceRange trace("stage2");
  const int R = p.search / 2;
  Workspace w;
  if (ws) {
    w = *ws;
  } else {
    CHECK(ensure(ctx, ctx->stack_a, stack_bytes(H, W), "stack"));
    CHECK(ensure(ctx, ctx->stack_b, stack_bytes(H, W), "pilot stack"));
    CHECK(ensure(ctx, ctx->idx, n_refs(H, W) * p.k_wiener * sizeof(int16_t), "idx"));
    CHECK(ensure(ctx, ctx->partials, gbm3d::partials_bytes(H, W), "partials"));
    w.stack_a = static_cast<float*>(ctx->stack_a.p);
    w.stack_b = static_cast<float*>(ctx->stack_b.p);
    w.idx = static_cast<int16_t*>(ctx->idx.p);
    w.partials = static_cast<unsigned long long*>(ctx->partials.p);
  }
  ImgRec r = blank_rec(H, W, sigma);
  r.noisy = noisy;
  r.pilot = pilot;
  r.out = out;
  r.stack_a = w.stack_a;
  r.stack_b = w.stack_b;
  r.idx = w.idx;
  r.partials = w.partials;
  r.norm = w.norm;
  // the noisy and the pilot's DCT stacks in one launch, with the matcher's
  // norm table of the pilot when the correlation kernel matches
  const BmChoice c = choose_bm(ctx, p, gbm3d::corr_tiles(H, W), p.k_wiener);
  if (c.method == GBM3D_BM_CORR) {
    CHECK(bind_norm(ctx, r));
    HIP_TRY(ctx, timed(ctx, "stack_dct", st, [&] {
              return gbm3d::launch_stack_norm(r, 1, -1, -1, R, 1, st);
            }),
            "stack launch");
    CHECK(run_match(ctx, r, R, p.k_wiener, c, 1, st, true));
  } else {
    CHECK(run_match(ctx, r, R, p.k_wiener, c, 1, st));
    HIP_TRY(ctx, timed(ctx, "stack_dct", st, [&] { return gbm3d::launch_stack(r, nullptr, 1, -1, -1, 0, st); }),
            "stack launch");
  }
  HIP_TRY(ctx, timed(ctx, "group_wiener", st, [&] {
            return gbm3d::launch_group_wiener(r, nullptr, R, p.k_wiener, 0, st);
          }),
          "Wiener group launch");
  HIP_TRY(ctx, timed(ctx, "reduce", st, [&] { return gbm3d::launch_reduce(r, nullptr, 1, 0, st); }),
          "aggregation launch");
  return GBM3D_OK;
}

// ---------------------------------------------------------------------------
// batches
// ---------------------------------------------------------------------------

// Device table layout: recs[n], then kPhases prefix arrays of n + 1 ints,
// then each phase's item-block start table.
size_t start_offset(const BatchPlan& plan, int n, int phase) {
  size_t o = kPhases * (n + 1);
  for (int ph = 0; ph < phase; ++ph) o += plan.start[ph].size();
  return o;
}
size_t table_bytes(const BatchPlan& plan, int n) {
  return align256(sizeof(ImgRec) * n) + sizeof(int) * start_offset(plan, n, kPhases);
}

int plan_batch(gbm3d_ctx* ctx, const gbm3d_image* imgs, int n, const gbm3d_params& p, int flags, BatchPlan& plan) {
  const int R = p.search / 2;
  const bool basic_only = (flags & GBM3D_BATCH_BASIC_ONLY) != 0;
  const int kmax = std::max(p.k_ht, p.k_wiener);
  // matching kernels of the two stages, from the tiles of all their images
  long tiles1 = 0, tiles2 = 0, waves1 = 0, waves2 = 0;
  for (int i = 0; i < n; ++i) {
    const int H = imgs[i].H, W = imgs[i].W;
    if (imgs[i].pilot == nullptr) {
      tiles1 += gbm3d::corr_tiles(H, W);
      waves1 += gbm3d::bm_waves_unsplit(H, W);
    }
    if (!basic_only) {
      tiles2 += gbm3d::corr_tiles(H, W);
      waves2 += gbm3d::bm_waves_unsplit(H, W);
    }
  }
  const BmChoice c1 = choose_bm(ctx, p, tiles1, p.k_ht), c2 = choose_bm(ctx, p, tiles2, p.k_wiener);
  plan.bm_method1 = c1.method;
  plan.bm_method2 = c2.method;
  auto split_of = [](const BmChoice& c, long tiles, long waves) {
    if (c.split > 0) return c.split;
    return c.method == GBM3D_BM_CORR ? gbm3d::corr_auto_split(tiles) : gbm3d::bm_auto_split(waves);
  };
  plan.bm_split1 = split_of(c1, tiles1, waves1);
  plan.bm_split2 = split_of(c2, tiles2, waves2);
  plan.ht_shape = choose_shape(ctx, p, tiles1);
  const bool need_norm = (tiles1 > 0 && c1.method == GBM3D_BM_CORR) || (tiles2 > 0 && c2.method == GBM3D_BM_CORR);
  // workspace slices
  size_t total = 0;
  std::vector<size_t> off(n);
  for (int i = 0; i < n; ++i) {
    const int H = imgs[i].H, W = imgs[i].W;
    const bool s1 = imgs[i].pilot == nullptr;
    off[i] = total;
    if (need_norm) total += align256(gbm3d::norm_bytes(H, W));              // norm table
    total += align256(stack_bytes(H, W));                                   // stack_a
    if (!basic_only) total += align256(stack_bytes(H, W));                  // stack_b
    total += align256(n_refs(H, W) * kmax * sizeof(int16_t));               // idx
    total += align256(gbm3d::partials_bytes(H, W));                      // partials
    if (s1 && !basic_only) total += align256(static_cast<size_t>(H) * W * (sizeof(float) + sizeof(uint16_t)));
  }
  CHECK(ensure(ctx, ctx->batch_ws, total, "batch workspace"));
  char* base = static_cast<char*>(ctx->batch_ws.p);
  plan.recs.resize(n);
  for (int i = 0; i < n; ++i) {
    const gbm3d_image& im = imgs[i];
    const int H = im.H, W = im.W;
    const bool s1 = im.pilot == nullptr;
    ImgRec r = blank_rec(H, W, im.sigma);
    char* c = base + off[i];
    if (need_norm) {
      r.norm = reinterpret_cast<double*>(c);
      c += align256(gbm3d::norm_bytes(H, W));
    }
    r.stack_a = reinterpret_cast<float*>(c);
    c += align256(stack_bytes(H, W));
    if (!basic_only) {
      r.stack_b = reinterpret_cast<float*>(c);
      c += align256(stack_bytes(H, W));
    }
    r.idx = reinterpret_cast<int16_t*>(c);
    c += align256(n_refs(H, W) * kmax * sizeof(int16_t));
    r.partials = reinterpret_cast<unsigned long long*>(c);
    c += align256(gbm3d::partials_bytes(H, W));
    r.noisy = im.noisy;
    r.eps = tv_eps(p, im.sigma);
    if (basic_only) {
      r.basic = im.out;
    } else if (s1) {
      r.basic = reinterpret_cast<float*>(c);
      c += static_cast<size_t>(H) * W * sizeof(float);
      r.q = reinterpret_cast<uint16_t*>(c);
      r.pilot = r.q;
      r.out = im.out;
    } else {
      r.pilot = im.pilot;
      r.out = im.out;
    }
    plan.recs[i] = r;
    plan.any_stage1 = plan.any_stage1 || s1;
  }
  plan.any_stage2 = !basic_only;
  for (int ph = 0; ph < kPhases; ++ph) plan.begin[ph].assign(n + 1, 0);
  for (int i = 0; i < n; ++i) {
    const int H = imgs[i].H, W = imgs[i].W;
    const bool s1 = imgs[i].pilot == nullptr;
    const bool s2 = !basic_only;
    const bool corr1 = plan.bm_method1 == GBM3D_BM_CORR, corr2 = plan.bm_method2 == GBM3D_BM_CORR;
    const int items[kPhases] = {
        s1 && corr1 ? gbm3d::norm_items_for(H, W) : 0,
        s1 ? (corr1 ? gbm3d::corr_items_for(H, W, plan.bm_split1) : gbm3d::bm_items_for(H, W, plan.bm_split1)) : 0,
        s1 ? gbm3d::stack_items_for(H, W) : 0,
        s1 ? gbm3d::group_items_for(H, W, R) : 0,
        s1 ? gbm3d::reduce_items_for(H, W) : 0,
        s2 && corr2 ? gbm3d::norm_items_for(H, W) : 0,
        s2 ? (corr2 ? gbm3d::corr_items_for(H, W, plan.bm_split2) : gbm3d::bm_items_for(H, W, plan.bm_split2)) : 0,
        s2 ? gbm3d::stack_items_for(H, W) : 0,
        s2 ? gbm3d::group_items_for(H, W, R) : 0,
        s2 ? gbm3d::reduce_items_for(H, W) : 0,
    };
    for (int ph = 0; ph < kPhases; ++ph) plan.begin[ph][i + 1] = plan.begin[ph][i] + items[ph];
  }
  // the image owning the first item of each block of kItemBlock items
  for (int ph = 0; ph < kPhases; ++ph) {
    const std::vector<int>& b = plan.begin[ph];
    plan.start[ph].assign(b[n] / gbm3d::kItemBlock + 1, 0);
    int i = 0;
    for (size_t blk = 0; blk < plan.start[ph].size(); ++blk) {
      const int item = static_cast<int>(blk) * gbm3d::kItemBlock;
      while (i < n - 1 && b[i + 1] <= item) ++i;
      plan.start[ph][blk] = i;
    }
  }
  return GBM3D_OK;
}

WorkList worklist(const gbm3d_ctx* ctx, const BatchPlan& plan, int n, int phase) {
  const char* t = static_cast<const char*>(ctx->batch_table.p);
  WorkList w;
  w.recs = reinterpret_cast<const ImgRec*>(t);
  w.begin = reinterpret_cast<const int*>(t + align256(sizeof(ImgRec) * n)) + phase * (n + 1);
  w.start = reinterpret_cast<const int*>(t + align256(sizeof(ImgRec) * n)) + start_offset(plan, n, phase);
  w.n = n;
  w.total = plan.begin[phase][n];
  return w;
}

// Grid cap of the batch launches: none (one workgroup per item).
constexpr int kFullGrid = 1 << 30;

// Batch matching of a stage, norm tables first when the correlation kernel
// matches, then its stacks (kind 0: the bior1.5 stack of the noisy images;
// 1: the DCT stacks of the noisy images and of the pilots).  Unlike a single
// image, a batch keeps the norm tables in a launch of their own: carried by
// the stack launch they made the 64-image batch slower (913 vs 940
// Mpixel/s).
int launch_batch_prep(gbm3d_ctx* ctx, const WorkList& sk, const WorkList& nm, const WorkList& bm, int R, int K,
                      int method, int split, int kind, hipStream_t st) {
  const ImgRec none = blank_rec(0, 0, 0.0f);
  const int use_pilot = kind;
  const int sel = kind == 0 ? 0 : -1;
  if (method == GBM3D_BM_CORR) {
    HIP_TRY(ctx, timed(ctx, "bm_norm", st, [&] { return gbm3d::launch_bm_norm(none, &nm, R, use_pilot, kFullGrid, st); }),
            "batch norm tables");
    HIP_TRY(ctx, timed(ctx, "bm", st, [&] {
              return gbm3d::launch_bm_corr(none, &bm, R, K, split, use_pilot, kFullGrid, st);
            }),
            "batch block matching");
  } else {
    HIP_TRY(ctx, timed(ctx, "bm", st, [&] { return gbm3d::launch_bm(none, &bm, R, K, split, use_pilot, kFullGrid, st); }),
            "batch block matching");
  }
  HIP_TRY(ctx, timed(ctx, kind == 0 ? "stack_bior" : "stack_dct", st, [&] {
            return gbm3d::launch_stack(none, &sk, kind, sel, sel, kFullGrid, st);
          }),
          "batch stacks");
  return GBM3D_OK;
}

// The batch launch sequence (also what a graph captures).  Every launch has
// one workgroup per work item of the whole batch (not a persistent grid
// walking several items): a workgroup's global stores then never hold up
// the loads of its next item (both count against the one vector-memory
// counter), and a finished workgroup's slot is refilled at once.
int launch_batch(gbm3d_ctx* ctx, const BatchPlan& plan, int n, const gbm3d_params& p, hipStream_t st) {
  const int R = p.search / 2;
  const ImgRec none = blank_rec(0, 0, 0.0f);
  if (plan.any_stage1) {
    TraceRange trace("batch stage1");
    const WorkList nm = worklist(ctx, plan, n, kNorm1), bm = worklist(ctx, plan, n, kBm1);
    const WorkList sk = worklist(ctx, plan, n, kStack1);
    const WorkList gr = worklist(ctx, plan, n, kGroup1), rd = worklist(ctx, plan, n, kReduce1);
    CHECK(launch_batch_prep(ctx, sk, nm, bm, R, p.k_ht, plan.bm_method1, plan.bm_split1, 0, st));
    HIP_TRY(ctx, timed(ctx, "group_ht", st, [&] {
              return gbm3d::launch_group_ht(none, &gr, R, p.k_ht, p.ht_a, p.ht_b, p.ht_weight, p.keep_dc, 0,
                                            plan.ht_shape, kFullGrid,
                                            st);
            }),
            "batch hard-threshold groups");
    HIP_TRY(ctx, timed(ctx, "reduce", st, [&] { return gbm3d::launch_reduce(none, &rd, 0, kFullGrid, st); }),
            "batch aggregation");
  }
  if (plan.any_stage2) {
    TraceRange trace("batch stage2");
    const WorkList nm = worklist(ctx, plan, n, kNorm2), bm = worklist(ctx, plan, n, kBm2);
    const WorkList sk = worklist(ctx, plan, n, kStack2);
    const WorkList gr = worklist(ctx, plan, n, kGroup2), rd = worklist(ctx, plan, n, kReduce2);
    CHECK(launch_batch_prep(ctx, sk, nm, bm, R, p.k_wiener, plan.bm_method2, plan.bm_split2, 1, st));
    HIP_TRY(ctx, timed(ctx, "group_wiener", st, [&] {
              return gbm3d::launch_group_wiener(none, &gr, R, p.k_wiener, kFullGrid, st);
            }),
            "batch Wiener groups");
    HIP_TRY(ctx, timed(ctx, "reduce", st, [&] { return gbm3d::launch_reduce(none, &rd, 1, kFullGrid, st); }),
            "batch aggregation");
  }
  return GBM3D_OK;
}

// Copies the plan's table to the device (stream-ordered, from pinned memory).
int upload_table(gbm3d_ctx* ctx, const BatchPlan& plan, int n, hipStream_t st) {
  const size_t bytes = table_bytes(plan, n);
  CHECK(ensure(ctx, ctx->batch_table, bytes, "batch table"));
  if (ctx->host_stage_bytes < bytes) {
    if (ctx->host_stage) {
      HIP_TRY(ctx, hipDeviceSynchronize(), "hipDeviceSynchronize");
      HIP_TRY(ctx, hipHostFree(ctx->host_stage), "hipHostFree");
      ctx->host_stage = nullptr;
      ctx->host_stage_bytes = 0;
    }
    HIP_TRY(ctx, hipHostMalloc(&ctx->host_stage, bytes, hipHostMallocDefault), "hipHostMalloc");
    ctx->host_stage_bytes = bytes;
  }
  if (!ctx->table_copied) HIP_TRY(ctx, hipEventCreateWithFlags(&ctx->table_copied, hipEventDisableTiming), "event");
  // the previous copy out of the staging buffer must have finished
  HIP_TRY(ctx, hipEventSynchronize(ctx->table_copied), "hipEventSynchronize");
  char* h = static_cast<char*>(ctx->host_stage);
  std::memcpy(h, plan.recs.data(), sizeof(ImgRec) * n);
  int* b = reinterpret_cast<int*>(h + align256(sizeof(ImgRec) * n));
  for (int ph = 0; ph < kPhases; ++ph) {
    std::memcpy(b + ph * (n + 1), plan.begin[ph].data(), sizeof(int) * (n + 1));
    std::memcpy(b + start_offset(plan, n, ph), plan.start[ph].data(), sizeof(int) * plan.start[ph].size());
  }
  HIP_TRY(ctx, hipMemcpyAsync(ctx->batch_table.p, h, bytes, hipMemcpyHostToDevice, st), "table copy");
  HIP_TRY(ctx, hipEventRecord(ctx->table_copied, st), "hipEventRecord");
  return GBM3D_OK;
}

void drop_graph(gbm3d_ctx* ctx) {
  if (ctx->graph.exec) (void)hipGraphExecDestroy(ctx->graph.exec);
  if (ctx->graph.graph) (void)hipGraphDestroy(ctx->graph.graph);
  ctx->graph = GraphEntry{};
}

// Everything that fixes the launch sequence: grids, work lists and kernel
// arguments other than the table contents.
std::string graph_key(const BatchPlan& plan, int n, const gbm3d_params& p, int flags, const gbm3d_ctx* ctx) {
  std::string k;
  auto add = [&](const void* d, size_t s) { k.append(static_cast<const char*>(d), s); };
  add(&n, sizeof(n));
  add(&p, sizeof(p));
  add(&flags, sizeof(flags));
  add(&ctx->batch_table.p, sizeof(void*));
  add(&plan.bm_split1, sizeof(int));
  add(&plan.bm_split2, sizeof(int));
  add(&plan.bm_method1, sizeof(int));
  add(&plan.bm_method2, sizeof(int));
  add(&plan.ht_shape, sizeof(int));
  for (int ph = 0; ph < kPhases; ++ph) add(plan.begin[ph].data(), sizeof(int) * (n + 1));
  return k;
}

}  // namespace

extern "C" {

void gbm3d_default_params(gbm3d_params* p) {
  if (!p) return;
  std::memset(p, 0, sizeof(*p));
  p->struct_size = sizeof(gbm3d_params);
  p->patch = 8;
  p->step = 3;
  p->search = 39;
  p->k_ht = 16;
  p->k_wiener = 32;
  p->ht_a = 3.6f;
  p->ht_b = 0.3f;
  p->ht_weight = GBM3D_W_TV;
  p->tv_eps_rel = 1e-3f;
  p->keep_dc = 1;
  p->bm_split = 0;
  p->bm_method = GBM3D_BM_AUTO;
  p->ht_source = GBM3D_HT_STACK;
}

int gbm3d_create(gbm3d_ctx** out, int hip_device) {
  if (!out) return fail(nullptr, GBM3D_EINVAL, "ctx output pointer is NULL");
  *out = nullptr;
  int n = 0;
  hipError_t e = hipGetDeviceCount(&n);
  if (e != hipSuccess || n == 0) return fail(nullptr, GBM3D_EHIP, "no HIP device: %s", hipGetErrorString(e));
  int dev = hip_device;
  if (dev < 0 && hipGetDevice(&dev) != hipSuccess) dev = 0;
  if (dev >= n) return fail(nullptr, GBM3D_EINVAL, "device %d out of range (%d devices)", dev, n);
  hipDeviceProp_t prop;
  e = hipGetDeviceProperties(&prop, dev);
  if (e != hipSuccess) return fail(nullptr, GBM3D_EHIP, "hipGetDeviceProperties: %s", hipGetErrorString(e));
  if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
    return fail(nullptr, GBM3D_EUNSUPPORTED, "device %d is %s; this library is built for gfx950", dev,
                prop.gcnArchName);
  {
    // the no-allocation entry point's scratch on this device
    DeviceGuard g(dev);
    if (!g.ok) return fail(nullptr, GBM3D_EHIP, "hipSetDevice(%d) failed", dev);
    e = resolve_scratch(dev);
    if (e != hipSuccess)
      return fail(nullptr, GBM3D_EHIP, "device scratch of device %d: %s", dev, hipGetErrorString(e));
  }
  gbm3d_ctx* ctx = new gbm3d_ctx();
  ctx->device = dev;
  ctx->n_cu = prop.multiProcessorCount > 0 ? prop.multiProcessorCount : 256;
  *out = ctx;
  return GBM3D_OK;
}

void gbm3d_destroy(gbm3d_ctx* ctx) {
  if (!ctx) return;
  {
    DeviceGuard g(ctx->device);
    (void)hipDeviceSynchronize();
    drop_graph(ctx);
    for (Buffer* b : {&ctx->stack_a, &ctx->stack_b, &ctx->idx, &ctx->partials, &ctx->basic, &ctx->q, &ctx->norm, &ctx->batch_ws,
                      &ctx->batch_table, &ctx->pilot_w, &ctx->pilot_act, &ctx->pilot_part, &ctx->gl_a, &ctx->gl_b,
                      &ctx->gl_num, &ctx->gl_idx, &ctx->gl_shift, &ctx->gl_pad, &ctx->gl_out})
      if (b->p) (void)hipFree(b->p);
    if (ctx->host_stage) (void)hipHostFree(ctx->host_stage);
    if (ctx->table_copied) (void)hipEventDestroy(ctx->table_copied);
    if (ctx->capture_stream) (void)hipStreamDestroy(ctx->capture_stream);
    for (auto& r : ctx->pending) {
      (void)hipEventDestroy(r.start);
      (void)hipEventDestroy(r.stop);
    }
    for (hipEvent_t e : ctx->event_pool) (void)hipEventDestroy(e);
  }
  delete ctx;
}

const char* gbm3d_status_str(int s) {
  switch (s) {
    case GBM3D_OK: return "ok";
    case GBM3D_EINVAL: return "invalid argument";
    case GBM3D_EUNSUPPORTED: return "unsupported";
    case GBM3D_ENOMEM: return "out of device memory";
    case GBM3D_EHIP: return "HIP runtime error";
    default: return "unknown status";
  }
}

const char* gbm3d_last_error(const gbm3d_ctx* ctx) { return ctx ? ctx->err.c_str() : g_thread_error.c_str(); }

int64_t gbm3d_n_refs(int H, int W, int step) {
  if (H <= 0 || W <= 0 || step <= 0) return 0;
  return static_cast<int64_t>((H + step - 1) / step) * ((W + step - 1) / step);
}

const char* gbm3d_version(void) { return "gbm3d-mi355x 0.2 (gfx950)"; }

int gbm3d_match(gbm3d_ctx* ctx, const uint16_t* img, int H, int W, int K, const gbm3d_params* params, int16_t* idx,
                void* stream) {
  TraceRange trace("gbm3d_match");
  const gbm3d_params p = resolve(params);
  if (!ctx) return fail(nullptr, GBM3D_EINVAL, "ctx is NULL");
  if (!img || !idx) return fail(ctx, GBM3D_EINVAL, "NULL image or idx pointer");
  CHECK(check_shape(ctx, H, W, p));
  CHECK(check_k(ctx, K, p, "K"));
  DeviceGuard g(ctx->device);
  if (!g.ok) return fail(ctx, GBM3D_EHIP, "hipSetDevice(%d) failed", ctx->device);
  ImgRec r = blank_rec(H, W, 1.0f);
  r.noisy = img;
  r.idx = idx;
  hipStream_t st = static_cast<hipStream_t>(stream);
  return run_match(ctx, r, p.search / 2, K, p, 0, st);
}

int gbm3d_autotune(gbm3d_ctx* ctx, const uint16_t* img, int H, int W, int K, const gbm3d_params* params, int reps,
                   int* best_method, int* best_split, float* best_ms, void* stream) {
  TraceRange trace("gbm3d_autotune");
  gbm3d_params p = resolve(params);
  if (!ctx) return fail(nullptr, GBM3D_EINVAL, "ctx is NULL");
  if (!img) return fail(ctx, GBM3D_EINVAL, "NULL image pointer");
  if (reps < 1) return fail(ctx, GBM3D_EINVAL, "reps %d must be >= 1", reps);
  CHECK(check_shape(ctx, H, W, p));
  CHECK(check_k(ctx, K, p, "K"));
  const bool tune_shape = K == p.k_ht && K <= 16;
  if (tune_shape) CHECK(check_ht(ctx, p));
  DeviceGuard g(ctx->device);
  if (!g.ok) return fail(ctx, GBM3D_EHIP, "hipSetDevice(%d) failed", ctx->device);
  hipStream_t st = static_cast<hipStream_t>(stream);
  CHECK(ensure(ctx, ctx->idx, n_refs(H, W) * K * sizeof(int16_t), "idx"));
  ImgRec r = blank_rec(H, W, 1.0f);
  r.noisy = img;
  r.idx = static_cast<int16_t*>(ctx->idx.p);
  struct Events {
    hipEvent_t a = nullptr, b = nullptr;
    ~Events() {
      if (a) (void)hipEventDestroy(a);
      if (b) (void)hipEventDestroy(b);
    }
  } ev;
  HIP_TRY(ctx, hipEventCreate(&ev.a), "hipEventCreate");
  HIP_TRY(ctx, hipEventCreate(&ev.b), "hipEventCreate");
  struct TimingOff {
    gbm3d_ctx* c;
    bool was;
    ~TimingOff() { c->timing = was; }
  } off{ctx, ctx->timing};
  ctx->timing = false;
  // milliseconds per run of f, after one warm-up run (which also sizes the workspace)
  auto time_runs = [&](auto&& f, float& ms) -> int {
    CHECK(f());
    HIP_TRY(ctx, hipEventRecord(ev.a, st), "hipEventRecord");
    for (int i = 0; i < reps; ++i) CHECK(f());
    HIP_TRY(ctx, hipEventRecord(ev.b, st), "hipEventRecord");
    HIP_TRY(ctx, hipEventSynchronize(ev.b), "hipEventSynchronize");
    HIP_TRY(ctx, hipEventElapsedTime(&ms, ev.a, ev.b), "hipEventElapsedTime");
    ms /= static_cast<float>(reps);
    return GBM3D_OK;
  };
  TuneEntry best;
  best.ms = INFINITY;
  const int R = p.search / 2;
  for (int method : {GBM3D_BM_SHIFT, GBM3D_BM_CORR}) {
    for (int split : {1, 2, 4}) {
      const BmChoice c{method, split};
      float ms = 0.0f;
      CHECK(time_runs([&] { return run_match(ctx, r, R, K, c, 0, st); }, ms));
      if (ms < best.ms) best = TuneEntry{method, split, ms};
    }
  }
  const int cls = tile_class(gbm3d::corr_tiles(H, W));
  ctx->tuned[{K, p.search, cls}] = best;
  if (tune_shape) {
    // the stage-1 group kernel's shape: whole stage-1 runs (matching as just
    // tuned) at a nominal noise level, one per shape
    CHECK(ensure(ctx, ctx->basic, static_cast<size_t>(H) * W * sizeof(float), "basic"));
    gbm3d_params q = p;
    q.bm_method = best.method;
    q.bm_split = best.split;
    ShapeEntry sbest;
    sbest.ms = INFINITY;
    for (int shape : {0, 1}) {
      ctx->tuned_shape[{K, p.search, cls}] = ShapeEntry{shape, 0.0f};
      float ms = 0.0f;
      CHECK(time_runs(
          [&] {
            return run_basic(ctx, img, H, W, 25.0f / 255.0f, q, static_cast<float*>(ctx->basic.p), nullptr, st);
          },
          ms));
      if (ms < sbest.ms) sbest = ShapeEntry{shape, ms};
    }
    ctx->tuned_shape[{K, p.search, cls}] = sbest;
  }
  if (best_method) *best_method = best.method;
  if (best_split) *best_split = best.split;
  if (best_ms) *best_ms = best.ms;
  return GBM3D_OK;
}

int gbm3d_tune_save(const gbm3d_ctx* ctx, const char* path) {
  if (!ctx) return fail(nullptr, GBM3D_EINVAL, "ctx is NULL");
  gbm3d_ctx* c = const_cast<gbm3d_ctx*>(ctx);
  if (!path) return fail(c, GBM3D_EINVAL, "NULL path");
  FILE* f = std::fopen(path, "w");
  if (!f) return fail(c, GBM3D_EINVAL, "cannot write %s", path);
  for (const auto& kv : ctx->tuned)
    std::fprintf(f, "bm %d %d %d %d %d %.6f\n", kv.first.K, kv.first.search, kv.first.cls, kv.second.method,
                 kv.second.split, static_cast<double>(kv.second.ms));
  for (const auto& kv : ctx->tuned_shape)
    std::fprintf(f, "ht %d %d %d %d %.6f\n", kv.first.K, kv.first.search, kv.first.cls, kv.second.shape,
                 static_cast<double>(kv.second.ms));
  const bool ok = std::fclose(f) == 0;
  return ok ? GBM3D_OK : fail(c, GBM3D_EINVAL, "cannot write %s", path);
}

int gbm3d_tune_load(gbm3d_ctx* ctx, const char* path) {
  if (!ctx) return fail(nullptr, GBM3D_EINVAL, "ctx is NULL");
  if (!path) return fail(ctx, GBM3D_EINVAL, "NULL path");
  FILE* f = std::fopen(path, "r");
  if (!f) return fail(ctx, GBM3D_EINVAL, "cannot read %s", path);
  std::vector<std::pair<TuneKey, TuneEntry>> rows;
  std::vector<std::pair<TuneKey, ShapeEntry>> shapes;
  char line[256];
  int n = 0;
  bool bad = false;
  while (std::fgets(line, sizeof(line), f)) {
    ++n;
    char tag[8] = {0};
    int K = 0, search = 0, cls = 0, a = 0, b = 0;
    double ms = 0.0;
    if (std::sscanf(line, " %7s", tag) != 1) continue;  // blank line
    if (std::strcmp(tag, "bm") == 0 &&
        std::sscanf(line, " bm %d %d %d %d %d %lf", &K, &search, &cls, &a, &b, &ms) == 6 && is_pow2_group(K) &&
        search >= 1 && search <= 39 && (search & 1) && cls >= 0 && cls <= 62 &&
        (a == GBM3D_BM_SHIFT || a == GBM3D_BM_CORR) && (b == 1 || b == 2 || b == 4) && ms >= 0.0) {
      rows.push_back({{K, search, cls}, TuneEntry{a, b, static_cast<float>(ms)}});
    } else if (std::strcmp(tag, "ht") == 0 &&
               std::sscanf(line, " ht %d %d %d %d %lf", &K, &search, &cls, &a, &ms) == 5 && is_pow2_group(K) &&
               search >= 1 && search <= 39 && (search & 1) && cls >= 0 && cls <= 62 && (a == 0 || a == 1) &&
               ms >= 0.0) {
      shapes.push_back({{K, search, cls}, ShapeEntry{a, static_cast<float>(ms)}});
    } else {
      bad = true;
      break;
    }
  }
  std::fclose(f);
  if (bad) return fail(ctx, GBM3D_EINVAL, "%s: cannot parse entry %d", path, n);
  for (const auto& r : rows) ctx->tuned[r.first] = r.second;
  for (const auto& r : shapes) ctx->tuned_shape[r.first] = r.second;
  return GBM3D_OK;
}

int gbm3d_stack(gbm3d_ctx* ctx, const uint16_t* img, int H, int W, int kind, float* out, void* stream) {
  TraceRange trace("gbm3d_stack");
  gbm3d_params p;
  gbm3d_default_params(&p);
  p.search = 1;
  if (!ctx) return fail(nullptr, GBM3D_EINVAL, "ctx is NULL");
  if (!img || !out) return fail(ctx, GBM3D_EINVAL, "NULL image or output pointer");
  if (kind != GBM3D_STACK_BIOR15 && kind != GBM3D_STACK_DCT) return fail(ctx, GBM3D_EINVAL, "stack kind %d", kind);
  CHECK(check_shape(ctx, H, W, p));
  DeviceGuard g(ctx->device);
  if (!g.ok) return fail(ctx, GBM3D_EHIP, "hipSetDevice(%d) failed", ctx->device);
  ImgRec r = blank_rec(H, W, 1.0f);
  r.noisy = img;
  r.stack_a = out;
  HIP_TRY(ctx, gbm3d::launch_stack(r, nullptr, kind, 0, 0, 0, static_cast<hipStream_t>(stream)), "stack launch");
  return GBM3D_OK;
}

int gbm3d_basic(gbm3d_ctx* ctx, const uint16_t* noisy, int H, int W, float sigma, const gbm3d_params* params,
                float* basic, void* stream) {
  TraceRange trace("gbm3d_basic");
  const gbm3d_params p = resolve(params);
  if (!ctx) return fail(nullptr, GBM3D_EINVAL, "ctx is NULL");
  if (!noisy || !basic) return fail(ctx, GBM3D_EINVAL, "NULL image or output pointer");
  CHECK(check_shape(ctx, H, W, p));
  CHECK(check_k(ctx, p.k_ht, p, "k_ht"));
  CHECK(check_sigma(ctx, sigma));
  CHECK(check_ht(ctx, p));
  DeviceGuard g(ctx->device);
  if (!g.ok) return fail(ctx, GBM3D_EHIP, "hipSetDevice(%d) failed", ctx->device);
  return run_basic(ctx, noisy, H, W, sigma, p, basic, nullptr, static_cast<hipStream_t>(stream));
}

void gbm3d_global_default_params(gbm3d_global_params* p) {
  if (!p) return;
  std::memset(p, 0, sizeof(*p));
  p->struct_size = sizeof(gbm3d_global_params);
  p->patch = 16;
  p->search = 33;
  p->k = 16;
  p->levels = 3;
  p->cycles = 2;
  p->n_shifts = 2;
  p->shifts[0] = 0;
  p->shifts[1] = 4;
  p->ht_a = 3.6f;
  p->ht_b = 0.3f;
  p->tv_eps_rel = 1e-3f;
}

namespace {

int resolve_global(gbm3d_ctx* ctx, const gbm3d_global_params* params, int H, int W, gbm3d_global_params& p,
                   bool any_size) {
  gbm3d_global_default_params(&p);
  if (params) {
    if (params->struct_size != sizeof(gbm3d_global_params))
      return fail(ctx, GBM3D_EINVAL, "gbm3d_global_params.struct_size %u != %zu", params->struct_size,
                  sizeof(gbm3d_global_params));
    p = *params;
  }
  if (p.patch != 8 && p.patch != 16) return fail(ctx, GBM3D_EINVAL, "global patch %d must be 8 or 16", p.patch);
  if (p.search < 3 || p.search > 39 || !(p.search & 1))
    return fail(ctx, GBM3D_EINVAL, "global search %d must be odd in [3, 39]", p.search);
  if (p.k != 8 && p.k != 16 && p.k != 32) return fail(ctx, GBM3D_EINVAL, "global k %d must be 8, 16 or 32", p.k);
  if (p.k > p.search * p.search) return fail(ctx, GBM3D_EINVAL, "global k %d exceeds search^2", p.k);
  if (p.levels < 1 || p.levels > 3 || (p.k >> p.levels) < 1)
    return fail(ctx, GBM3D_EINVAL, "global levels %d must be in [1, 3] with k >= 2^levels", p.levels);
  if (p.cycles < 1 || p.cycles > 4) return fail(ctx, GBM3D_EINVAL, "global cycles %d must be in [1, 4]", p.cycles);
  if (p.n_shifts < 1 || p.n_shifts > 4)
    return fail(ctx, GBM3D_EINVAL, "global n_shifts %d must be in [1, 4]", p.n_shifts);
  for (int i = 0; i < p.n_shifts; ++i)
    if (p.shifts[i] < 0 || p.shifts[i] >= p.patch)
      return fail(ctx, GBM3D_EINVAL, "global shift %d must be in [0, patch)", p.shifts[i]);
  if (!(p.ht_a >= 0.0f) || !(p.ht_b >= 0.0f) || !(p.tv_eps_rel > 0.0f))
    return fail(ctx, GBM3D_EINVAL, "global thresholds and eps must be non-negative (eps > 0)");
  const int lo = p.search > p.patch ? p.search : p.patch;
  if (H < lo || W < lo || H > 32768 || W > 32768)
    return fail(ctx, GBM3D_EINVAL, "image %dx%d: sides must be in [%d, 32768]", H, W, lo);
  if (!any_size && (H % p.patch || W % p.patch))
    return fail(ctx, GBM3D_EINVAL, "image %dx%d: sides must be multiples of %d", H, W, p.patch);
  return GBM3D_OK;
}

}  // namespace

int gbm3d_global_match(gbm3d_ctx* ctx, const uint16_t* img, int H, int W, const gbm3d_global_params* params,
                       int16_t* idx, void* stream) {
  if (!ctx) return fail(nullptr, GBM3D_EINVAL, "ctx is NULL");
  if (!img || !idx) return fail(ctx, GBM3D_EINVAL, "NULL image or index pointer");
  gbm3d_global_params p;
  CHECK(resolve_global(ctx, params, H, W, p, false));
  DeviceGuard g(ctx->device);
  if (!g.ok) return fail(ctx, GBM3D_EHIP, "hipSetDevice(%d) failed", ctx->device);
  HIP_TRY(ctx, gbm3d::launch_global_match(img, H, W, p.patch, p.search, p.k, idx, static_cast<hipStream_t>(stream)),
          "global matching launch");
  return GBM3D_OK;
}

int gbm3d_global_basic(gbm3d_ctx* ctx, const uint16_t* noisy, int H, int W, float sigma,
                       const gbm3d_global_params* params, float* out, void* stream) {
  TraceRange trace("gbm3d_global_basic");
  if (!ctx) return fail(nullptr, GBM3D_EINVAL, "ctx is NULL");
  if (!noisy || !out) return fail(ctx, GBM3D_EINVAL, "NULL image or output pointer");
  CHECK(check_sigma(ctx, sigma));
  gbm3d_global_params p;
  CHECK(resolve_global(ctx, params, H, W, p, true));
  DeviceGuard g(ctx->device);
  if (!g.ok) return fail(ctx, GBM3D_EHIP, "hipSetDevice(%d) failed", ctx->device);
  hipStream_t st = static_cast<hipStream_t>(stream);
  // sides that are not multiples of the tile side: filter the image
  // mirror-padded at the bottom and right, then crop (Sec. 3.1)
  const int Hp = (H + p.patch - 1) / p.patch * p.patch, Wp = (W + p.patch - 1) / p.patch * p.patch;
  const bool padded = Hp != H || Wp != W;
  const size_t hw = static_cast<size_t>(Hp) * Wp;
  const size_t vb = gbm3d::global_volume_bytes(Hp, Wp, p.k);
  if (padded) {
    CHECK(ensure(ctx, ctx->gl_pad, hw * sizeof(uint16_t), "padded image"));
    CHECK(ensure(ctx, ctx->gl_out, hw * sizeof(float), "padded estimate"));
    HIP_TRY(ctx,
            gbm3d::launch_global_pad(noisy, H, W, static_cast<uint16_t*>(ctx->gl_pad.p), Hp, Wp, st),
            "mirror padding launch");
  }
  // per translation: cycles volume pairs, its sums, matches and translated image
  const size_t T = static_cast<size_t>(p.n_shifts);
  CHECK(ensure(ctx, ctx->gl_a, T * p.cycles * vb, "global volumes"));
  CHECK(ensure(ctx, ctx->gl_b, T * p.cycles * vb, "global volumes"));
  CHECK(ensure(ctx, ctx->gl_num, T * 2 * hw * sizeof(unsigned long long), "global sums"));
  CHECK(ensure(ctx, ctx->gl_idx, T * (hw / (p.patch * p.patch)) * p.k * sizeof(int16_t), "global matches"));
  CHECK(ensure(ctx, ctx->gl_shift, T * hw * sizeof(uint16_t), "translated images"));
  gbm3d::GlobalJob j{};
  j.noisy = padded ? static_cast<const uint16_t*>(ctx->gl_pad.p) : noisy;
  j.out = padded ? static_cast<float*>(ctx->gl_out.p) : out;
  j.H = Hp;
  j.W = Wp;
  j.sigma = sigma;
  j.patch = p.patch;
  j.search = p.search;
  j.k = p.k;
  j.levels = p.levels;
  j.cycles = p.cycles;
  j.n_shifts = p.n_shifts;
  for (int i = 0; i < 4; ++i) j.shifts[i] = p.shifts[i];
  j.ht_a = p.ht_a;
  j.ht_b = p.ht_b;
  j.tv_eps_rel = p.tv_eps_rel;
  j.vol_a = static_cast<float*>(ctx->gl_a.p);
  j.vol_b = static_cast<float*>(ctx->gl_b.p);
  j.num = static_cast<unsigned long long*>(ctx->gl_num.p);
  j.idx = static_cast<int16_t*>(ctx->gl_idx.p);
  j.shifted = static_cast<uint16_t*>(ctx->gl_shift.p);
  HIP_TRY(ctx, timed(ctx, "global_basic", st, [&] { return gbm3d::launch_global_basic(j, st); }),
          "global stage 1 launch");
  if (padded)
    HIP_TRY(ctx,
            hipMemcpy2DAsync(out, static_cast<size_t>(W) * sizeof(float), ctx->gl_out.p,
                             static_cast<size_t>(Wp) * sizeof(float), static_cast<size_t>(W) * sizeof(float), H,
                             hipMemcpyDeviceToDevice, st),
            "crop copy");
  return GBM3D_OK;
}

int gbm3d_wiener(gbm3d_ctx* ctx, const uint16_t* noisy, const uint16_t* pilot, int H, int W, float sigma,
                 const gbm3d_params* params, float* out, void* stream) {
  TraceRange trace("gbm3d_wiener");
  const gbm3d_params p = resolve(params);
  if (!ctx) return fail(nullptr, GBM3D_EINVAL, "ctx is NULL");
  if (!noisy || !pilot || !out) return fail(ctx, GBM3D_EINVAL, "NULL image, pilot or output pointer");
  CHECK(check_shape(ctx, H, W, p));
  CHECK(check_k(ctx, p.k_wiener, p, "k_wiener"));
  CHECK(check_sigma(ctx, sigma));
  DeviceGuard g(ctx->device);
  if (!g.ok) return fail(ctx, GBM3D_EHIP, "hipSetDevice(%d) failed", ctx->device);
  return run_wiener(ctx, noisy, pilot, H, W, sigma, p, out, static_cast<hipStream_t>(stream));
}

int gbm3d_denoise(gbm3d_ctx* ctx, const uint16_t* noisy, int H, int W, float sigma, const gbm3d_params* params,
                  float* out, float* basic_out, uint16_t* q_out, void* stream) {
  TraceRange trace("gbm3d_denoise");
  const gbm3d_params p = resolve(params);
  if (!ctx) return fail(nullptr, GBM3D_EINVAL, "ctx is NULL");
  if (!noisy || !out) return fail(ctx, GBM3D_EINVAL, "NULL image or output pointer");
  CHECK(check_shape(ctx, H, W, p));
  CHECK(check_k(ctx, p.k_ht, p, "k_ht"));
  CHECK(check_k(ctx, p.k_wiener, p, "k_wiener"));
  CHECK(check_sigma(ctx, sigma));
  CHECK(check_ht(ctx, p));
  DeviceGuard g(ctx->device);
  if (!g.ok) return fail(ctx, GBM3D_EHIP, "hipSetDevice(%d) failed", ctx->device);
  hipStream_t st = static_cast<hipStream_t>(stream);
  float* basic = basic_out;
  uint16_t* q = q_out;
  if (!basic) {
    CHECK(ensure(ctx, ctx->basic, static_cast<size_t>(H) * W * sizeof(float), "basic"));
    basic = static_cast<float*>(ctx->basic.p);
  }
  if (!q) {
    CHECK(ensure(ctx, ctx->q, static_cast<size_t>(H) * W * sizeof(uint16_t), "pilot"));
    q = static_cast<uint16_t*>(ctx->q.p);
  }
  CHECK(run_basic(ctx, noisy, H, W, sigma, p, basic, q, st));
  return run_wiener(ctx, noisy, q, H, W, sigma, p, out, st);
}

int gbm3d_denoise_noalloc(gbm3d_ctx* ctx, const uint16_t* noisy, int H, int W, float sigma,
                          const gbm3d_params* params, float* out, float* basic_out, uint16_t* q_out, void* stream) {
  TraceRange trace("gbm3d_denoise_noalloc");
  const gbm3d_params p = resolve(params);
  if (!ctx) return fail(nullptr, GBM3D_EINVAL, "ctx is NULL");
  if (!noisy || !out) return fail(ctx, GBM3D_EINVAL, "NULL image or output pointer");
  CHECK(check_shape(ctx, H, W, p));
  CHECK(check_k(ctx, p.k_ht, p, "k_ht"));
  CHECK(check_k(ctx, p.k_wiener, p, "k_wiener"));
  CHECK(check_sigma(ctx, sigma));
  CHECK(check_ht(ctx, p));
  // slices of the scratch: the same buffers gbm3d_denoise takes from the
  // context's workspace
  const size_t hw = static_cast<size_t>(H) * W;
  size_t off = 0;
  auto take = [&off](size_t bytes) {
    const size_t o = off;
    off += align256(bytes);
    return o;
  };
  const size_t o_norm = take(gbm3d::norm_bytes(H, W));
  const size_t o_sa = take(stack_bytes(H, W));
  const size_t o_sb = take(stack_bytes(H, W));
  const size_t o_idx = take(n_refs(H, W) * std::max(p.k_ht, p.k_wiener) * sizeof(int16_t));
  const size_t o_part = take(gbm3d::partials_bytes(H, W));
  const size_t o_basic = basic_out ? 0 : take(hw * sizeof(float));
  const size_t o_q = q_out ? 0 : take(hw * sizeof(uint16_t));
  if (off > static_cast<size_t>(GBM3D_NOALLOC_SCRATCH_BYTES))
    return fail(ctx, GBM3D_EINVAL, "image %dx%d needs %zu bytes of scratch; the static scratch holds %zu", H, W, off,
                static_cast<size_t>(GBM3D_NOALLOC_SCRATCH_BYTES));
  DeviceGuard g(ctx->device);
  if (!g.ok) return fail(ctx, GBM3D_EHIP, "hipSetDevice(%d) failed", ctx->device);
  char* base = static_cast<char*>(scratch_addr(ctx->device));
  if (!base) return fail(ctx, GBM3D_EHIP, "device scratch of device %d not resolved", ctx->device);
  Workspace ws;
  ws.norm = reinterpret_cast<double*>(base + o_norm);
  ws.stack_a = reinterpret_cast<float*>(base + o_sa);
  ws.stack_b = reinterpret_cast<float*>(base + o_sb);
  ws.idx = reinterpret_cast<int16_t*>(base + o_idx);
  ws.partials = reinterpret_cast<unsigned long long*>(base + o_part);
  float* basic = basic_out ? basic_out : reinterpret_cast<float*>(base + o_basic);
  uint16_t* q = q_out ? q_out : reinterpret_cast<uint16_t*>(base + o_q);
  // per-kernel timing would create events: none for this call
  struct TimingOff {
    gbm3d_ctx* c;
    bool was;
    ~TimingOff() { c->timing = was; }
  } off_timing{ctx, ctx->timing};
  ctx->timing = false;
  hipStream_t st = static_cast<hipStream_t>(stream);
  CHECK(run_basic(ctx, noisy, H, W, sigma, p, basic, q, st, &ws));
  return run_wiener(ctx, noisy, q, H, W, sigma, p, out, st, &ws);
}

int gbm3d_denoise_batch(gbm3d_ctx* ctx, const gbm3d_image* imgs, int n, const gbm3d_params* params, int flags,
                        void* stream) {
  TraceRange trace("gbm3d_denoise_batch");
  const gbm3d_params p = resolve(params);
  if (!ctx) return fail(nullptr, GBM3D_EINVAL, "ctx is NULL");
  if (n < 0 || (n > 0 && !imgs)) return fail(ctx, GBM3D_EINVAL, "bad image array");
  if (flags & ~(GBM3D_BATCH_GRAPH | GBM3D_BATCH_BASIC_ONLY)) return fail(ctx, GBM3D_EINVAL, "unknown flags %d", flags);
  if (n == 0) return GBM3D_OK;
  CHECK(check_params(ctx, p));
  CHECK(check_k(ctx, p.k_ht, p, "k_ht"));
  CHECK(check_k(ctx, p.k_wiener, p, "k_wiener"));
  CHECK(check_ht(ctx, p));
  if (p.ht_source != GBM3D_HT_STACK)
    return fail(ctx, GBM3D_EUNSUPPORTED, "batches take stage-1 spectra from the stack (ht_source %d)", p.ht_source);
  const bool basic_only = (flags & GBM3D_BATCH_BASIC_ONLY) != 0;
  for (int i = 0; i < n; ++i) {
    const gbm3d_image& im = imgs[i];
    if (!im.noisy || !im.out) return fail(ctx, GBM3D_EINVAL, "image %d: NULL noisy or out pointer", i);
    if (basic_only && im.pilot) return fail(ctx, GBM3D_EINVAL, "image %d: stage 1 only takes no pilot", i);
    CHECK(check_shape(ctx, im.H, im.W, p));
    CHECK(check_sigma(ctx, im.sigma));
  }
  DeviceGuard g(ctx->device);
  if (!g.ok) return fail(ctx, GBM3D_EHIP, "hipSetDevice(%d) failed", ctx->device);
  hipStream_t st = static_cast<hipStream_t>(stream);
  BatchPlan plan;
  CHECK(plan_batch(ctx, imgs, n, p, flags, plan));
  CHECK(upload_table(ctx, plan, n, st));
  if (!(flags & GBM3D_BATCH_GRAPH) || ctx->timing) return launch_batch(ctx, plan, n, p, st);

  const std::string key = graph_key(plan, n, p, flags, ctx);
  if (!ctx->graph.exec || ctx->graph.key != key) {
    drop_graph(ctx);
    if (!ctx->capture_stream)
      HIP_TRY(ctx, hipStreamCreateWithFlags(&ctx->capture_stream, hipStreamNonBlocking), "stream");
    HIP_TRY(ctx, hipStreamBeginCapture(ctx->capture_stream, hipStreamCaptureModeThreadLocal), "begin capture");
    const int s = launch_batch(ctx, plan, n, p, ctx->capture_stream);
    hipGraph_t graph = nullptr;
    const hipError_t e = hipStreamEndCapture(ctx->capture_stream, &graph);
    if (s != GBM3D_OK) {
      if (graph) (void)hipGraphDestroy(graph);
      return s;
    }
    HIP_TRY(ctx, e, "end capture");
    hipGraphExec_t exec = nullptr;
    const hipError_t ei = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    if (ei != hipSuccess) {
      (void)hipGraphDestroy(graph);
      return hip_fail(ctx, ei, "graph instantiate");
    }
    ctx->graph.key = key;
    ctx->graph.graph = graph;
    ctx->graph.exec = exec;
  }
  HIP_TRY(ctx, hipGraphLaunch(ctx->graph.exec, st), "graph launch");
  return GBM3D_OK;
}

int gbm3d_quantize(gbm3d_ctx* ctx, const float* in, uint16_t* out, size_t n, void* stream) {
  if (!ctx) return fail(nullptr, GBM3D_EINVAL, "ctx is NULL");
  if (n == 0) return GBM3D_OK;
  if (!in || !out) return fail(ctx, GBM3D_EINVAL, "NULL input or output pointer");
  DeviceGuard g(ctx->device);
  if (!g.ok) return fail(ctx, GBM3D_EHIP, "hipSetDevice(%d) failed", ctx->device);
  HIP_TRY(ctx, gbm3d::launch_quantize(in, out, n, static_cast<hipStream_t>(stream)), "quantize launch");
  return GBM3D_OK;
}

int gbm3d_probe(gbm3d_ctx* ctx, int kind, int blocks, int iters, float* sink, void* stream) {
  if (!ctx) return fail(nullptr, GBM3D_EINVAL, "ctx is NULL");
  if (kind < GBM3D_PROBE_FP64 || kind > GBM3D_PROBE_MFMA_BF16) return fail(ctx, GBM3D_EINVAL, "probe kind %d", kind);
  if (blocks < 1 || blocks > (1 << 20) || iters < 1 || iters > (1 << 20))
    return fail(ctx, GBM3D_EINVAL, "probe blocks %d / iters %d out of [1, 2^20]", blocks, iters);
  if (!sink) return fail(ctx, GBM3D_EINVAL, "NULL sink");
  DeviceGuard g(ctx->device);
  if (!g.ok) return fail(ctx, GBM3D_EHIP, "hipSetDevice(%d) failed", ctx->device);
  HIP_TRY(ctx, gbm3d::launch_microbench(kind, blocks, iters, sink, static_cast<hipStream_t>(stream)), "probe launch");
  return GBM3D_OK;
}

double gbm3d_probe_ops(int kind, int blocks, int iters) { return gbm3d::microbench_ops(kind, blocks, iters); }

// ---------------------------------------------------------------------------
// learned pilot
// ---------------------------------------------------------------------------

int gbm3d_pilot_param_count(void) { return gbm3d::kPilotParams; }

}  // extern "C"

namespace {

constexpr int kPilotC = 32;

struct PilotWeights {
  uint16_t* wf;   // [layer][9][32][32] forward
  uint16_t* wb;   // [layer][9][32][32] input gradient
  float* bias;    // [layer][32]
};

PilotWeights pilot_weights(gbm3d_ctx* ctx) {
  char* base = static_cast<char*>(ctx->pilot_w.p);
  const size_t half = gbm3d::pilot_packed_bytes() / 2;
  return {reinterpret_cast<uint16_t*>(base), reinterpret_cast<uint16_t*>(base + half),
          reinterpret_cast<float*>(base + 2 * half)};
}

size_t act_bytes(int B, int H, int W) { return static_cast<size_t>(B) * H * W * kPilotC * sizeof(uint16_t); }

int check_pilot_shape(gbm3d_ctx* ctx, int B, int H, int W) {
  if (B < 1 || H < 1 || W < 1 || H > 32768 || W > 32768)
    return fail(ctx, GBM3D_EINVAL, "pilot batch %dx%dx%d invalid", B, H, W);
  if (static_cast<double>(B) * H * W > 2.0e9) return fail(ctx, GBM3D_EINVAL, "pilot batch too large");
  if (!ctx->pilot_loaded) return fail(ctx, GBM3D_EINVAL, "no pilot weights loaded (gbm3d_pilot_load)");
  return GBM3D_OK;
}

// training forward pass, one launch per layer: the input of every layer is
// kept in HBM for the backward pass
int pilot_forward(gbm3d_ctx* ctx, const uint16_t* noisy, int B, int H, int W, const float* sigma,
                  uint16_t* pilot_u16, float* pilot_f32, hipStream_t st) {
  const size_t ab = act_bytes(B, H, W);
  const PilotWeights pw = pilot_weights(ctx);
  char* act = static_cast<char*>(ctx->pilot_act.p);
  auto buf = [&](int l) { return reinterpret_cast<uint16_t*>(act + l * ab); };
  const int cap = 4 * ctx->n_cu;
  HIP_TRY(ctx, timed(ctx, "pilot_prep", st, [&] { return gbm3d::launch_pilot_prep(noisy, sigma, B, H, W, buf(0), st); }),
          "pilot input");
  for (int l = 0; l < gbm3d::kPilotLayers; ++l) {
    const bool last = l == gbm3d::kPilotLayers - 1;
    const uint16_t* w = pw.wf + static_cast<size_t>(l) * 9 * kPilotC * kPilotC;
    HIP_TRY(ctx, timed(ctx, "pilot_conv", st, [&] {
              return gbm3d::launch_pilot_conv(last ? 1 : 0, buf(l), w, pw.bias + l * kPilotC, nullptr,
                                              last ? nullptr : buf(l + 1), noisy, pilot_f32, pilot_u16, B, H, W, cap,
                                              st);
            }),
            "pilot conv");
  }
  return GBM3D_OK;
}

}  // namespace

extern "C" {

int gbm3d_pilot_load(gbm3d_ctx* ctx, const float* master, void* stream) {
  if (!ctx) return fail(nullptr, GBM3D_EINVAL, "ctx is NULL");
  if (!master) return fail(ctx, GBM3D_EINVAL, "NULL master vector");
  DeviceGuard g(ctx->device);
  if (!g.ok) return fail(ctx, GBM3D_EHIP, "hipSetDevice(%d) failed", ctx->device);
  CHECK(ensure(ctx, ctx->pilot_w, gbm3d::pilot_packed_bytes() + gbm3d::kPilotLayers * kPilotC * sizeof(float),
               "pilot weights"));
  const PilotWeights pw = pilot_weights(ctx);
  HIP_TRY(ctx, gbm3d::launch_pilot_pack(master, pw.wf, pw.wb, pw.bias, static_cast<hipStream_t>(stream)),
          "pilot pack");
  ctx->pilot_loaded = true;
  return GBM3D_OK;
}

int gbm3d_pilot_infer(gbm3d_ctx* ctx, const uint16_t* noisy, int B, int H, int W, const float* sigma,
                      uint16_t* pilot_u16, float* pilot_f32, void* stream) {
  TraceRange trace("gbm3d_pilot_infer");
  if (!ctx) return fail(nullptr, GBM3D_EINVAL, "ctx is NULL");
  if (!noisy || !sigma || (!pilot_u16 && !pilot_f32)) return fail(ctx, GBM3D_EINVAL, "NULL input or no output");
  CHECK(check_pilot_shape(ctx, B, H, W));
  DeviceGuard g(ctx->device);
  if (!g.ok) return fail(ctx, GBM3D_EHIP, "hipSetDevice(%d) failed", ctx->device);
  const PilotWeights pw = pilot_weights(ctx);
  hipStream_t st = static_cast<hipStream_t>(stream);
  HIP_TRY(ctx, timed(ctx, "pilot_fused", st, [&] {
            return gbm3d::launch_pilot_infer_fused(noisy, sigma, pw.wf, pw.bias, B, H, W, pilot_f32, pilot_u16,
                                                   ctx->n_cu, st);
          }),
          "pilot inference");
  return GBM3D_OK;
}

int gbm3d_pilot_grad(gbm3d_ctx* ctx, const uint16_t* noisy, const float* target, int B, int H, int W,
                     const float* sigma, const float* weight, float* grad, float* loss, void* stream) {
  TraceRange trace("gbm3d_pilot_grad");
  if (!ctx) return fail(nullptr, GBM3D_EINVAL, "ctx is NULL");
  if (!noisy || !target || !sigma || !grad || !loss) return fail(ctx, GBM3D_EINVAL, "NULL argument");
  CHECK(check_pilot_shape(ctx, B, H, W));
  DeviceGuard g(ctx->device);
  if (!g.ok) return fail(ctx, GBM3D_EHIP, "hipSetDevice(%d) failed", ctx->device);
  hipStream_t st = static_cast<hipStream_t>(stream);
  const size_t ab = act_bytes(B, H, W);
  const size_t npix = static_cast<size_t>(B) * H * W;
  // layout: layer inputs x0 .. x(L-1) | grad ping-pong g0, g1 | pilot f32
  constexpr int L = gbm3d::kPilotLayers;
  CHECK(ensure(ctx, ctx->pilot_act, (L + 2) * ab + align256(npix * sizeof(float)), "pilot training activations"));
  const int wg_grid = 2 * ctx->n_cu;
  const int loss_blocks = 1024;
  CHECK(ensure(ctx, ctx->pilot_part,
               gbm3d::pilot_wgrad_partial_floats(wg_grid) * sizeof(float) + loss_blocks * sizeof(double),
               "pilot partial sums"));
  char* act = static_cast<char*>(ctx->pilot_act.p);
  auto x = [&](int l) { return reinterpret_cast<uint16_t*>(act + l * ab); };
  uint16_t* gbuf[2] = {reinterpret_cast<uint16_t*>(act + L * ab), reinterpret_cast<uint16_t*>(act + (L + 1) * ab)};
  float* pil = reinterpret_cast<float*>(act + (L + 2) * ab);
  float* wpart = static_cast<float*>(ctx->pilot_part.p);
  double* lpart = reinterpret_cast<double*>(reinterpret_cast<char*>(ctx->pilot_part.p) +
                                            gbm3d::pilot_wgrad_partial_floats(wg_grid) * sizeof(float));
  CHECK(pilot_forward(ctx, noisy, B, H, W, sigma, nullptr, pil, st));
  HIP_TRY(ctx, timed(ctx, "pilot_loss", st, [&] {
            return gbm3d::launch_pilot_loss(pil, target, weight, static_cast<size_t>(H) * W, npix, gbuf[0], lpart,
                                            loss_blocks, loss, st);
          }),
          "pilot loss");
  const PilotWeights pw = pilot_weights(ctx);
  const int cap = 4 * ctx->n_cu;
  int cur = 0;
  for (int l = gbm3d::kPilotLayers - 1; l >= 0; --l) {
    HIP_TRY(ctx, timed(ctx, "pilot_wgrad", st, [&] {
              return gbm3d::launch_pilot_wgrad(x(l), gbuf[cur], B, H, W, wg_grid, wpart, l,
                                               grad + gbm3d::pilot_layer_offset(l), st);
            }),
            "pilot weight gradient");
    if (l > 0) {
      const uint16_t* w = pw.wb + static_cast<size_t>(l) * 9 * kPilotC * kPilotC;
      HIP_TRY(ctx, timed(ctx, "pilot_dgrad", st, [&] {
                return gbm3d::launch_pilot_conv(2, gbuf[cur], w, nullptr, x(l), gbuf[cur ^ 1], nullptr, nullptr,
                                                nullptr, B, H, W, cap, st);
              }),
              "pilot input gradient");
      cur ^= 1;
    }
  }
  return GBM3D_OK;
}

int gbm3d_pilot_adam(gbm3d_ctx* ctx, float* master, float* m, float* v, const float* grad, int step, float lr,
                     float beta1, float beta2, float eps, void* stream) {
  if (!ctx) return fail(nullptr, GBM3D_EINVAL, "ctx is NULL");
  if (!master || !m || !v || !grad) return fail(ctx, GBM3D_EINVAL, "NULL argument");
  if (step < 1 || !(lr >= 0.0f) || !(beta1 >= 0.0f && beta1 < 1.0f) || !(beta2 >= 0.0f && beta2 < 1.0f) ||
      !(eps > 0.0f))
    return fail(ctx, GBM3D_EINVAL, "bad Adam hyper-parameters");
  DeviceGuard g(ctx->device);
  if (!g.ok) return fail(ctx, GBM3D_EHIP, "hipSetDevice(%d) failed", ctx->device);
  hipStream_t st = static_cast<hipStream_t>(stream);
  HIP_TRY(ctx, gbm3d::launch_pilot_adam(master, m, v, grad, gbm3d::kPilotParams, lr, beta1, beta2, eps, step, st),
          "adam");
  return gbm3d_pilot_load(ctx, master, stream);
}

int gbm3d_timing_enable(gbm3d_ctx* ctx, int on) {
  if (!ctx) return fail(nullptr, GBM3D_EINVAL, "ctx is NULL");
  ctx->timing = on != 0;
  return GBM3D_OK;
}

int gbm3d_timing_read(gbm3d_ctx* ctx, const char* kernel, double* total_ms, int64_t* launches) {
  if (!ctx || !kernel || !total_ms || !launches) return fail(ctx, GBM3D_EINVAL, "NULL argument");
  DeviceGuard g(ctx->device);
  for (auto& r : ctx->pending) {
    HIP_TRY(ctx, hipEventSynchronize(r.stop), "hipEventSynchronize");
    float ms = 0.0f;
    HIP_TRY(ctx, hipEventElapsedTime(&ms, r.start, r.stop), "hipEventElapsedTime");
    auto& t = ctx->totals[r.name];
    t.first += ms;
    t.second += 1;
    ctx->event_pool.push_back(r.start);
    ctx->event_pool.push_back(r.stop);
  }
  ctx->pending.clear();
  auto it = ctx->totals.find(kernel);
  *total_ms = it == ctx->totals.end() ? 0.0 : it->second.first;
  *launches = it == ctx->totals.end() ? 0 : it->second.second;
  return GBM3D_OK;
}

int gbm3d_timing_reset(gbm3d_ctx* ctx) {
  if (!ctx) return fail(nullptr, GBM3D_EINVAL, "ctx is NULL");
  double ms;
  int64_t n;
  CHECK(gbm3d_timing_read(ctx, "", &ms, &n));
  ctx->totals.clear();
  return GBM3D_OK;
}

int gbm3d_check_args(int H, int W, float sigma, const gbm3d_params* params) {
  const gbm3d_params p = resolve(params);
  CHECK(check_shape(nullptr, H, W, p));
  CHECK(check_k(nullptr, p.k_ht, p, "k_ht"));
  CHECK(check_k(nullptr, p.k_wiener, p, "k_wiener"));
  CHECK(check_sigma(nullptr, sigma));
  CHECK(check_ht(nullptr, p));
  return GBM3D_OK;
}

}  // extern "C"
