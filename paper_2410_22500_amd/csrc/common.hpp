// Shared host/device helpers of the hsn library (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdarg>
#include <cstdint>
#include <type_traits>
#include <cstdio>
#include <string>
#include <vector>

#include "../../include/hsn.h"

// ---------------------------------------------------------------------------
// Context
// ---------------------------------------------------------------------------
namespace hsn {
// Device state a context keeps across calls (cached plans); released by hsn_destroy.
struct Owned {
  virtual ~Owned() {}
};
}  // namespace hsn

struct hsn_ctx {
  int device = 0;
  int num_cu = 256;
  std::string err;
  // Device workspace, grown on demand (never shrunk until hsn_destroy).
  void *ws = nullptr;
  size_t ws_bytes = 0;
  // Per-view geometry table cache (device copy of the last angle set).
  double *geom = nullptr;
  size_t geom_cap = 0;
  std::vector<double> geom_host;
  // Projector launch shape (hsn_projector_set_launch; 0 = chosen from the
  // geometry, -1 = the gather kernels).
  int proj_views = 0, proj_split = 0, proj_voxels = 0, proj_threads = 0;
  // ANLS round form of hsn_subspace_nmf (hsn_nmf_set_launch): 1 = one fused
  // pass (the default), 2 = N_V pass, row solves, N_D pass.
  int nmf_anls_passes = 1;
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  // Optional kernel timing: event pairs per kernel kind.
  bool prof = false;
  std::vector<hipEvent_t> prof_ev[HSN_KERN_COUNT];
  size_t prof_used[HSN_KERN_COUNT] = {};
  // Cached batched-decomposition plans (descriptors, workspace, captured graphs).
  std::vector<hsn::Owned *> plans;
  // Stream used only to capture graphs (capture is not allowed on the null stream).
  hipStream_t cap_stream = nullptr;
  std::string last_plan_note;  // description of the last batched plan used
  // Small device scalars owned by the context (hsn_fhr_step's bfloat16 bias).
  double *dscalars = nullptr;
  // Pinned host staging for small device-to-host reads (control block, history).
  void *host_stage = nullptr;
  size_t host_stage_bytes = 0;
};

namespace hsn {

hsn_status fail(hsn_ctx *ctx, hsn_status st, const char *fmt, ...);
hsn_status ensure_ws(hsn_ctx *ctx, size_t bytes);
// Pinned host staging buffer of at least `bytes` (grown on demand; the
// stream is synchronised before it is replaced).
hsn_status ensure_host_stage(hsn_ctx *ctx, size_t bytes);
// Bracket one kernel launch with timing events when profiling is on.
void prof_begin(hsn_ctx *ctx, int kind, hipStream_t st);
void prof_end(hsn_ctx *ctx, int kind, hipStream_t st);

// Bump allocator over the workspace: every carve is 256-byte aligned.
struct Carver {
  char *base;
  size_t off = 0;
  explicit Carver(void *b) : base(static_cast<char *>(b)) {}
  template <typename T>
  T *take(size_t n) {
    off = (off + 255) & ~size_t(255);
    T *p = reinterpret_cast<T *>(base + off);
    off += n * sizeof(T);
    return p;
  }
  static size_t need(std::initializer_list<size_t> bytes) {
    size_t o = 0;
    for (size_t b : bytes) o = ((o + 255) & ~size_t(255)) + b;
    return o + 256;
  }
};

// Restores the caller's current device on scope exit.
struct DeviceGuard {
  int prev = -1;
  explicit DeviceGuard(int dev) {
    if (hipGetDevice(&prev) != hipSuccess) prev = -1;
    if (prev != dev) (void)hipSetDevice(dev);
  }
  ~DeviceGuard() {
    int cur = -1;
    if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
  }
};

}  // namespace hsn

#define HSN_HIP(ctx, call)                                                                    \
  do {                                                                                        \
    hipError_t e_ = (call);                                                                   \
    if (e_ != hipSuccess)                                                                     \
      return hsn::fail((ctx), HSN_ERR_DEVICE, "%s failed: %s", #call, hipGetErrorString(e_)); \
  } while (0)

#define HSN_LAUNCHED(ctx)                                                                      \
  do {                                                                                         \
    hipError_t e_ = hipGetLastError();                                                         \
    if (e_ != hipSuccess)                                                                      \
      return hsn::fail((ctx), HSN_ERR_DEVICE, "kernel launch failed: %s", hipGetErrorString(e_)); \
  } while (0)

// ---------------------------------------------------------------------------
// Device helpers
// ---------------------------------------------------------------------------
namespace hsn {

// Sum over the 64 lanes of a wave with DPP row operations; the total ends in
// lane 63 (other lanes hold partial sums).
__device__ __forceinline__ float wave_sum_to_lane63(float v) {
  v += __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), 0xB1, 0xF, 0xF, true));
  v += __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), 0x4E, 0xF, 0xF, true));
  v += __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), 0x141, 0xF, 0xF, true));
  v += __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), 0x140, 0xF, 0xF, true));
  v += __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), 0x142, 0xA, 0xF, false));
  v += __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), 0x143, 0xC, 0xF, false));
  return v;
}

// Full wave sum of a double via lane shuffles (result in every lane).
__device__ __forceinline__ double wave_sum_all(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Round-to-nearest-even float32 -> bfloat16 bits (finite inputs).
__device__ __forceinline__ uint16_t f32_to_bf16_bits(float f) {
  uint32_t u = __builtin_bit_cast(uint32_t, f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return static_cast<uint16_t>(u >> 16);
}
__device__ __forceinline__ float bf16_bits_to_f32(uint16_t b) {
  return __builtin_bit_cast(float, static_cast<uint32_t>(b) << 16);
}

}  // namespace hsn
