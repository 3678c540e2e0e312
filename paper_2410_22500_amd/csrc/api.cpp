// Context lifetime, error reporting and workspace management.
#include "common.hpp"

#include <algorithm>

namespace hsn {

hsn_status fail(hsn_ctx *ctx, hsn_status st, const char *fmt, ...) {
  if (ctx) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    ctx->err = buf;
  }
  return st;
}

hsn_status ensure_ws(hsn_ctx *ctx, size_t bytes) {
  if (bytes <= ctx->ws_bytes) return HSN_OK;
  if (ctx->ws) {
    // The old workspace may still be in use by queued work.
    HSN_HIP(ctx, hipDeviceSynchronize());
    HSN_HIP(ctx, hipFree(ctx->ws));
    ctx->ws = nullptr;
    ctx->ws_bytes = 0;
  }
  size_t want = bytes + bytes / 4;
  if (hipMalloc(&ctx->ws, want) != hipSuccess) {
    (void)hipGetLastError();
    ctx->ws = nullptr;
    return fail(ctx, HSN_ERR_OOM, "workspace allocation of %zu bytes failed", want);
  }
  ctx->ws_bytes = want;
  return HSN_OK;
}

hsn_status ensure_host_stage(hsn_ctx *ctx, size_t bytes) {
  if (bytes <= ctx->host_stage_bytes) return HSN_OK;
  HSN_HIP(ctx, hipDeviceSynchronize());
  if (ctx->host_stage) (void)hipHostFree(ctx->host_stage);
  ctx->host_stage = nullptr;
  ctx->host_stage_bytes = 0;
  const size_t n = std::max<size_t>(bytes, 1 << 16);
  if (hipHostMalloc(&ctx->host_stage, n, hipHostMallocDefault) != hipSuccess) {
    (void)hipGetLastError();
    ctx->host_stage = nullptr;
    return fail(ctx, HSN_ERR_OOM, "cannot allocate %zu bytes of pinned host memory", n);
  }
  ctx->host_stage_bytes = n;
  return HSN_OK;
}

void prof_begin(hsn_ctx *ctx, int kind, hipStream_t st) {
  if (!ctx->prof) return;
  auto &pool = ctx->prof_ev[kind];
  const size_t u = ctx->prof_used[kind];
  while (pool.size() < 2 * (u + 1)) {
    hipEvent_t e;
    if (hipEventCreate(&e) != hipSuccess) return;
    pool.push_back(e);
  }
  (void)hipEventRecord(pool[2 * u], st);
}

void prof_end(hsn_ctx *ctx, int kind, hipStream_t st) {
  if (!ctx->prof) return;
  auto &pool = ctx->prof_ev[kind];
  const size_t u = ctx->prof_used[kind];
  if (pool.size() < 2 * (u + 1)) return;
  (void)hipEventRecord(pool[2 * u + 1], st);
  ctx->prof_used[kind] = u + 1;
}

}  // namespace hsn

extern "C" {

hsn_status hsn_profile_enable(hsn_ctx *ctx, int on) {
  if (!ctx) return HSN_ERR_INVALID_ARG;
  ctx->prof = on != 0;
  return HSN_OK;
}

hsn_status hsn_profile_read(hsn_ctx *ctx, int kernel, double *total_ms, int64_t *launches, int reset) {
  if (!ctx) return HSN_ERR_INVALID_ARG;
  if (kernel < 0 || kernel >= HSN_KERN_COUNT) return hsn::fail(ctx, HSN_ERR_INVALID_ARG, "profile: bad kernel id");
  hsn::DeviceGuard g(ctx->device);
  double sum = 0.0;
  const size_t n = ctx->prof_used[kernel];
  auto &pool = ctx->prof_ev[kernel];
  for (size_t i = 0; i < n; ++i) {
    HSN_HIP(ctx, hipEventSynchronize(pool[2 * i + 1]));
    float ms = 0.f;
    HSN_HIP(ctx, hipEventElapsedTime(&ms, pool[2 * i], pool[2 * i + 1]));
    sum += ms;
  }
  if (total_ms) *total_ms = sum;
  if (launches) *launches = int64_t(n);
  if (reset) ctx->prof_used[kernel] = 0;
  return HSN_OK;
}

int hsn_version(void) { return 200; }

hsn_status hsn_create(hsn_ctx **out, int device) {
  if (!out) return HSN_ERR_INVALID_ARG;
  *out = nullptr;
  int n = 0;
  if (hipGetDeviceCount(&n) != hipSuccess || device < 0 || device >= n) {
    (void)hipGetLastError();
    return HSN_ERR_DEVICE;
  }
  hsn_ctx *ctx = new hsn_ctx();
  ctx->device = device;
  hsn::DeviceGuard g(device);
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, device) == hipSuccess) ctx->num_cu = prop.multiProcessorCount;
  if (hipEventCreate(&ctx->ev0) != hipSuccess || hipEventCreate(&ctx->ev1) != hipSuccess ||
      hipMalloc(&ctx->dscalars, 64 * sizeof(double)) != hipSuccess) {
    (void)hipGetLastError();
    hsn_destroy(ctx);
    return HSN_ERR_DEVICE;
  }
  *out = ctx;
  return HSN_OK;
}

void hsn_destroy(hsn_ctx *ctx) {
  if (!ctx) return;
  hsn::DeviceGuard g(ctx->device);
  (void)hipDeviceSynchronize();
  for (hsn::Owned *o : ctx->plans) delete o;
  if (ctx->host_stage) (void)hipHostFree(ctx->host_stage);
  if (ctx->cap_stream) (void)hipStreamDestroy(ctx->cap_stream);
  if (ctx->ws) (void)hipFree(ctx->ws);
  if (ctx->geom) (void)hipFree(ctx->geom);
  if (ctx->dscalars) (void)hipFree(ctx->dscalars);
  if (ctx->ev0) (void)hipEventDestroy(ctx->ev0);
  if (ctx->ev1) (void)hipEventDestroy(ctx->ev1);
  for (auto &pool : ctx->prof_ev)
    for (hipEvent_t e : pool) (void)hipEventDestroy(e);
  delete ctx;
}

const char *hsn_last_error(const hsn_ctx *ctx) { return ctx ? ctx->err.c_str() : "null context"; }

}  // extern "C"
