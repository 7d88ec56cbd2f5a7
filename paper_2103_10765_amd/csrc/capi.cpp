// C ABI of the G-BM3D library: argument validation, device workspace and the
// stage pipelines.  Every compute step runs in the library's HIP kernels.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <string>
#include <vector>

#include "../../include/gbm3d.h"
#include "kernels.h"

namespace {

struct Buffer {
  void* p = nullptr;
  size_t bytes = 0;
};

thread_local std::string g_thread_error;

}  // namespace

struct TimingRecord {
  const char* name;
  hipEvent_t start, stop;
};

struct gbm3d_ctx {
  int device = 0;
  std::string err;
  Buffer stack_a, stack_b, idx, partials, basic, q;
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

#define HIP_TRY(ctx, expr, what)                 \
  do {                                           \
    hipError_t e_ = (expr);                      \
    if (e_ != hipSuccess) return hip_fail(ctx, e_, what); \
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
int check_shape(gbm3d_ctx* ctx, int H, int W, const gbm3d_params& p) {
  if (p.struct_size != sizeof(gbm3d_params))
    return fail(ctx, GBM3D_EINVAL, "params.struct_size %u != %zu", p.struct_size, sizeof(gbm3d_params));
  if (p.patch != 8) return fail(ctx, GBM3D_EUNSUPPORTED, "patch %d unsupported (only 8)", p.patch);
  if (p.step != 3) return fail(ctx, GBM3D_EUNSUPPORTED, "step %d unsupported (only 3)", p.step);
  if (p.search < 1 || p.search > 39 || p.search % 2 == 0)
    return fail(ctx, GBM3D_EINVAL, "search %d must be odd and in [1, 39]", p.search);
  if (p.bm_split != 0 && p.bm_split != 1 && p.bm_split != 2 && p.bm_split != 4)
    return fail(ctx, GBM3D_EINVAL, "bm_split %d must be 0, 1, 2 or 4", p.bm_split);
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
  if (!(sigma > 0.0f) || !std::isfinite(sigma)) return fail(ctx, GBM3D_EINVAL, "sigma %g must be > 0 and finite", sigma);
  return GBM3D_OK;
}

int check_ht(gbm3d_ctx* ctx, const gbm3d_params& p) {
  if (!std::isfinite(p.ht_a) || !std::isfinite(p.ht_b)) return fail(ctx, GBM3D_EINVAL, "ht_a/ht_b must be finite");
  if (p.ht_weight < GBM3D_W_TV || p.ht_weight > GBM3D_W_UNIT)
    return fail(ctx, GBM3D_EINVAL, "ht_weight %d unknown", p.ht_weight);
  if (!(p.tv_eps_rel > 0.0f) || !std::isfinite(p.tv_eps_rel))
    return fail(ctx, GBM3D_EINVAL, "tv_eps_rel must be > 0 and finite");
  return GBM3D_OK;
}

gbm3d_params resolve(const gbm3d_params* p) {
  gbm3d_params d;
  gbm3d_default_params(&d);
  return p ? *p : d;
}

#define CHECK(expr)               \
  do {                            \
    int s_ = (expr);              \
    if (s_ != GBM3D_OK) return s_; \
  } while (0)

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

size_t stack_bytes(int H, int W) { return static_cast<size_t>(H) * W * 64 * sizeof(float); }
size_t n_refs(int H, int W) { return static_cast<size_t>((H + 2) / 3) * ((W + 2) / 3); }

// Stage 1 into `basic` (and optionally its quantisation into q).
int run_basic(gbm3d_ctx* ctx, const uint16_t* noisy, int H, int W, float sigma, const gbm3d_params& p,
              float* basic, uint16_t* q, hipStream_t st) {
  const int R = p.search / 2;
  CHECK(ensure(ctx, ctx->stack_a, stack_bytes(H, W), "stack"));
  CHECK(ensure(ctx, ctx->idx, n_refs(H, W) * p.k_ht * sizeof(int16_t), "idx"));
  CHECK(ensure(ctx, ctx->partials, gbm3d::partials_bytes(H, W, R), "partials"));
  int16_t* idx = static_cast<int16_t*>(ctx->idx.p);
  float* stack = static_cast<float*>(ctx->stack_a.p);
  void* part = ctx->partials.p;
  const float eps = p.tv_eps_rel * sigma * 64.0f * static_cast<float>(p.k_ht);
  HIP_TRY(ctx, timed(ctx, "bm", st, [&] { return gbm3d::launch_bm(noisy, H, W, R, p.k_ht, idx, st, p.bm_split); }),
          "block matching launch");
  HIP_TRY(ctx, timed(ctx, "stack_bior", st, [&] { return gbm3d::launch_stack(noisy, H, W, GBM3D_STACK_BIOR15, stack, st); }),
          "stack launch");
  HIP_TRY(ctx, timed(ctx, "group_ht", st, [&] {
            return gbm3d::launch_group_ht(stack, idx, H, W, R, p.k_ht, sigma, p.ht_a, p.ht_b, p.ht_weight, eps,
                                          p.keep_dc, part, st);
          }),
          "hard-threshold group launch");
  HIP_TRY(ctx, timed(ctx, "reduce", st, [&] { return gbm3d::launch_reduce(part, H, W, R, basic, q, st); }),
          "aggregation launch");
  return GBM3D_OK;
}

int run_wiener(gbm3d_ctx* ctx, const uint16_t* noisy, const uint16_t* pilot, int H, int W, float sigma,
               const gbm3d_params& p, float* out, hipStream_t st) {
  const int R = p.search / 2;
  CHECK(ensure(ctx, ctx->stack_a, stack_bytes(H, W), "stack"));
  CHECK(ensure(ctx, ctx->stack_b, stack_bytes(H, W), "pilot stack"));
  CHECK(ensure(ctx, ctx->idx, n_refs(H, W) * p.k_wiener * sizeof(int16_t), "idx"));
  CHECK(ensure(ctx, ctx->partials, gbm3d::partials_bytes(H, W, R), "partials"));
  int16_t* idx = static_cast<int16_t*>(ctx->idx.p);
  float* sn = static_cast<float*>(ctx->stack_a.p);
  float* sp = static_cast<float*>(ctx->stack_b.p);
  void* part = ctx->partials.p;
  HIP_TRY(ctx, timed(ctx, "bm", st, [&] { return gbm3d::launch_bm(pilot, H, W, R, p.k_wiener, idx, st, p.bm_split); }),
          "block matching launch");
  HIP_TRY(ctx, timed(ctx, "stack_dct", st, [&] { return gbm3d::launch_stack(noisy, H, W, GBM3D_STACK_DCT, sn, st); }),
          "stack launch");
  HIP_TRY(ctx, timed(ctx, "stack_dct", st, [&] { return gbm3d::launch_stack(pilot, H, W, GBM3D_STACK_DCT, sp, st); }),
          "pilot stack launch");
  HIP_TRY(ctx, timed(ctx, "group_wiener", st, [&] {
            return gbm3d::launch_group_wiener(sn, sp, idx, H, W, R, p.k_wiener, sigma, part, st);
          }),
          "Wiener group launch");
  HIP_TRY(ctx, timed(ctx, "reduce", st, [&] { return gbm3d::launch_reduce(part, H, W, R, out, nullptr, st); }),
          "aggregation launch");
  return GBM3D_OK;
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
  gbm3d_ctx* ctx = new gbm3d_ctx();
  ctx->device = dev;
  *out = ctx;
  return GBM3D_OK;
}

void gbm3d_destroy(gbm3d_ctx* ctx) {
  if (!ctx) return;
  {
    DeviceGuard g(ctx->device);
    (void)hipDeviceSynchronize();
    for (Buffer* b : {&ctx->stack_a, &ctx->stack_b, &ctx->idx, &ctx->partials, &ctx->basic, &ctx->q})
      if (b->p) (void)hipFree(b->p);
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

const char* gbm3d_version(void) { return "gbm3d-mi355x 0.1 (gfx950)"; }

int gbm3d_match(gbm3d_ctx* ctx, const uint16_t* img, int H, int W, int K, const gbm3d_params* params, int16_t* idx,
                void* stream) {
  const gbm3d_params p = resolve(params);
  if (!ctx) return fail(nullptr, GBM3D_EINVAL, "ctx is NULL");
  if (!img || !idx) return fail(ctx, GBM3D_EINVAL, "NULL image or idx pointer");
  CHECK(check_shape(ctx, H, W, p));
  CHECK(check_k(ctx, K, p, "K"));
  DeviceGuard g(ctx->device);
  if (!g.ok) return fail(ctx, GBM3D_EHIP, "hipSetDevice(%d) failed", ctx->device);
  HIP_TRY(ctx, gbm3d::launch_bm(img, H, W, p.search / 2, K, idx, static_cast<hipStream_t>(stream), p.bm_split),
          "block matching launch");
  return GBM3D_OK;
}

int gbm3d_stack(gbm3d_ctx* ctx, const uint16_t* img, int H, int W, int kind, float* out, void* stream) {
  gbm3d_params p;
  gbm3d_default_params(&p);
  p.search = 1;
  if (!ctx) return fail(nullptr, GBM3D_EINVAL, "ctx is NULL");
  if (!img || !out) return fail(ctx, GBM3D_EINVAL, "NULL image or output pointer");
  if (kind != GBM3D_STACK_BIOR15 && kind != GBM3D_STACK_DCT) return fail(ctx, GBM3D_EINVAL, "stack kind %d", kind);
  CHECK(check_shape(ctx, H, W, p));
  DeviceGuard g(ctx->device);
  if (!g.ok) return fail(ctx, GBM3D_EHIP, "hipSetDevice(%d) failed", ctx->device);
  HIP_TRY(ctx, gbm3d::launch_stack(img, H, W, kind, out, static_cast<hipStream_t>(stream)), "stack launch");
  return GBM3D_OK;
}

int gbm3d_basic(gbm3d_ctx* ctx, const uint16_t* noisy, int H, int W, float sigma, const gbm3d_params* params,
                float* basic, void* stream) {
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

int gbm3d_wiener(gbm3d_ctx* ctx, const uint16_t* noisy, const uint16_t* pilot, int H, int W, float sigma,
                 const gbm3d_params* params, float* out, void* stream) {
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

int gbm3d_quantize(gbm3d_ctx* ctx, const float* in, uint16_t* out, size_t n, void* stream) {
  if (!ctx) return fail(nullptr, GBM3D_EINVAL, "ctx is NULL");
  if (n == 0) return GBM3D_OK;
  if (!in || !out) return fail(ctx, GBM3D_EINVAL, "NULL input or output pointer");
  DeviceGuard g(ctx->device);
  if (!g.ok) return fail(ctx, GBM3D_EHIP, "hipSetDevice(%d) failed", ctx->device);
  HIP_TRY(ctx, gbm3d::launch_quantize(in, out, n, static_cast<hipStream_t>(stream)), "quantize launch");
  return GBM3D_OK;
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
  (void)gbm3d_timing_read(ctx, "", &ms, &n);
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
