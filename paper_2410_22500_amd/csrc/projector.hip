// K-channel parallel-beam projector A, its adjoint A^T, and per-channel CGLS.
//
// A is the linear projection operator of eq. (3)/(5).  Its entries are
// Joseph's interpolation written as a closed-form footprint:
//   a_{(v,c),(j,i)} = (1/w_v) max(0, 1 - |d|/w_v),
//   d = s_c - (x_i cos t_v + y_j sin t_v),  w_v = max(|cos t_v|, |sin t_v|),
// with s_c = c - h, x_i = i - h, y_j = j - h, h = (N-1)/2, image size N = N_c.
//
// Forward = ray gather: one thread per (view, slice, detector column) steps
// along the dominant image axis and reads the two pixels that straddle the
// ray (weights (1-f)/w and f/w, f the fractional crossing position).
// Adjoint = voxel gather: one thread per voxel loops over the views and
// reads the two detector bins that straddle the voxel centre.  Both
// evaluate the same entries, so A^T is the exact adjoint up to float32
// rounding.  Crossing positions are evaluated in float64 (|x| reaches
// ~N/sqrt(2) pixels, where a float32 position would carry ~1e-5 px error);
// weights and channel sums are float32.  All K channels of a pixel or bin
// are contiguous, so each tap is one vector load.
#include "common.hpp"

#include <cmath>

namespace {

struct ViewGeom {
  double cs, sn, w, inv_w;
};

template <int K>
struct Vec {
  float v[K];
};

template <int K>
__device__ __forceinline__ void load_k(const float *__restrict__ p, float (&out)[K]) {
  if constexpr (K == 4) {
    const float4 a = *reinterpret_cast<const float4 *>(p);
    out[0] = a.x; out[1] = a.y; out[2] = a.z; out[3] = a.w;
  } else if constexpr (K == 8) {
    const float4 a = *reinterpret_cast<const float4 *>(p);
    const float4 b = *reinterpret_cast<const float4 *>(p + 4);
    out[0] = a.x; out[1] = a.y; out[2] = a.z; out[3] = a.w;
    out[4] = b.x; out[5] = b.y; out[6] = b.z; out[7] = b.w;
  } else if constexpr (K == 2) {
    const float2 a = *reinterpret_cast<const float2 *>(p);
    out[0] = a.x; out[1] = a.y;
  } else {
#pragma unroll
    for (int c = 0; c < K; ++c) out[c] = p[c];
  }
}

constexpr int kRayThreads = 128;

// s[v][r][c][:] = alpha * sum_taps a * x[r][j][i][:] + beta * s[v][r][c][:]
template <int K>
__global__ __launch_bounds__(kRayThreads) void project_kernel(const float *__restrict__ x, float *__restrict__ s,
                                                              const ViewGeom *__restrict__ geom, int n_slices,
                                                              int n, float alpha, float beta) {
  const int c = blockIdx.x * kRayThreads + threadIdx.x;
  const int r = blockIdx.y;
  const int v = blockIdx.z;
  if (c >= n) return;
  const ViewGeom g = geom[v];
  const double h = 0.5 * double(n - 1);
  const double sc = double(c) - h;
  const float inv_w = float(g.inv_w);
  float acc[K];
#pragma unroll
  for (int q = 0; q < K; ++q) acc[q] = 0.0f;
  const float *xs = x + size_t(r) * n * n * K;
  if (fabs(g.cs) >= fabs(g.sn)) {
    // Step along image rows j; the ray crosses row j at column position u_j.
    const double u0 = (sc + h * g.sn) / g.cs + h;
    const double du = -g.sn / g.cs;
    for (int j = 0; j < n; ++j) {
      const double u = fma(double(j), du, u0);
      const double fl = floor(u);
      const int i0 = int(fl);
      const float f = float(u - fl);
      if (i0 < -1 || i0 >= n) continue;
      const float w0 = (1.0f - f) * inv_w, w1 = f * inv_w;
      const float *row = xs + size_t(j) * n * K;
      float a[K];
      if (i0 >= 0) {
        load_k<K>(row + size_t(i0) * K, a);
#pragma unroll
        for (int q = 0; q < K; ++q) acc[q] = fmaf(w0, a[q], acc[q]);
      }
      if (i0 + 1 < n) {
        load_k<K>(row + size_t(i0 + 1) * K, a);
#pragma unroll
        for (int q = 0; q < K; ++q) acc[q] = fmaf(w1, a[q], acc[q]);
      }
    }
  } else {
    // Step along image columns i; the ray crosses column i at row position u_i.
    const double u0 = (sc + h * g.cs) / g.sn + h;
    const double du = -g.cs / g.sn;
    for (int i = 0; i < n; ++i) {
      const double u = fma(double(i), du, u0);
      const double fl = floor(u);
      const int j0 = int(fl);
      const float f = float(u - fl);
      if (j0 < -1 || j0 >= n) continue;
      const float w0 = (1.0f - f) * inv_w, w1 = f * inv_w;
      float a[K];
      if (j0 >= 0) {
        load_k<K>(xs + (size_t(j0) * n + i) * K, a);
#pragma unroll
        for (int q = 0; q < K; ++q) acc[q] = fmaf(w0, a[q], acc[q]);
      }
      if (j0 + 1 < n) {
        load_k<K>(xs + (size_t(j0 + 1) * n + i) * K, a);
#pragma unroll
        for (int q = 0; q < K; ++q) acc[q] = fmaf(w1, a[q], acc[q]);
      }
    }
  }
  float *out = s + ((size_t(v) * n_slices + r) * n + c) * K;
#pragma unroll
  for (int q = 0; q < K; ++q) out[q] = (beta == 0.0f) ? alpha * acc[q] : fmaf(alpha, acc[q], beta * out[q]);
}

constexpr int kVoxThreads = 128;

// x[r][j][i][:] = alpha * sum_v sum_taps a * s[v][r][c][:] + beta * x[r][j][i][:]
template <int K>
__global__ __launch_bounds__(kVoxThreads) void backproject_kernel(const float *__restrict__ s, float *__restrict__ x,
                                                                  const ViewGeom *__restrict__ geom, int n_views,
                                                                  int n_slices, int n, float alpha, float beta) {
  const int i = blockIdx.x * kVoxThreads + threadIdx.x;
  const int j = blockIdx.y;
  const int r = blockIdx.z;
  if (i >= n) return;
  const double h = 0.5 * double(n - 1);
  const double xi = double(i) - h, yj = double(j) - h;
  float acc[K];
#pragma unroll
  for (int q = 0; q < K; ++q) acc[q] = 0.0f;
  const size_t view_stride = size_t(n_slices) * n * K;
  const float *sr = s + size_t(r) * n * K;
  for (int v = 0; v < n_views; ++v) {
    const ViewGeom g = geom[v];
    const double u = fma(xi, g.cs, fma(yj, g.sn, h));   // detector position of the voxel centre
    const double fl = floor(u);
    const int c0 = int(fl);
    const float f = float(u - fl);                      // |d| of tap c0; tap c0+1 has |d| = 1 - f
    const float inv_w = float(g.inv_w);
    const float w0 = fmaxf(0.0f, 1.0f - f * inv_w) * inv_w;
    const float w1 = fmaxf(0.0f, 1.0f - (1.0f - f) * inv_w) * inv_w;
    const float *sv = sr + size_t(v) * view_stride;
    float a[K];
    if (c0 >= 0 && c0 < n && w0 > 0.0f) {
      load_k<K>(sv + size_t(c0) * K, a);
#pragma unroll
      for (int q = 0; q < K; ++q) acc[q] = fmaf(w0, a[q], acc[q]);
    }
    if (c0 + 1 >= 0 && c0 + 1 < n && w1 > 0.0f) {
      load_k<K>(sv + size_t(c0 + 1) * K, a);
#pragma unroll
      for (int q = 0; q < K; ++q) acc[q] = fmaf(w1, a[q], acc[q]);
    }
  }
  float *out = x + ((size_t(r) * n + j) * n + i) * K;
#pragma unroll
  for (int q = 0; q < K; ++q) out[q] = (beta == 0.0f) ? alpha * acc[q] : fmaf(alpha, acc[q], beta * out[q]);
}

// ---------------------------------------------------------------------------
// CGLS helpers: per-channel dot products (deterministic two-stage sums) and
// axpy updates that read their per-channel scalars from device memory.
// ---------------------------------------------------------------------------
constexpr int kDotBlocks = 512;
constexpr int kDotThreads = 256;

template <int K>
__global__ __launch_bounds__(kDotThreads) void chan_dot_kernel(const float *__restrict__ a, const float *__restrict__ b,
                                                               int64_t n_items, double *__restrict__ partial) {
  double acc[K];
#pragma unroll
  for (int q = 0; q < K; ++q) acc[q] = 0.0;
  for (int64_t it = int64_t(blockIdx.x) * kDotThreads + threadIdx.x; it < n_items;
       it += int64_t(gridDim.x) * kDotThreads) {
#pragma unroll
    for (int q = 0; q < K; ++q) acc[q] += double(a[it * K + q]) * double(b[it * K + q]);
  }
  __shared__ double red[kDotThreads / 64][K];
#pragma unroll
  for (int q = 0; q < K; ++q) {
    const double t = hsn::wave_sum_all(acc[q]);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6][q] = t;
  }
  __syncthreads();
  if (threadIdx.x < K) {
    double t = 0.0;
    for (int w = 0; w < kDotThreads / 64; ++w) t += red[w][threadIdx.x];
    partial[size_t(blockIdx.x) * K + threadIdx.x] = t;
  }
}

// st layout: gamma[8], alpha[8], beta[8]
enum { kSetGamma = 0, kAlpha = 1, kBeta = 2, kResid = 3 };
__global__ __launch_bounds__(256) void cgls_scalar_kernel(const double *__restrict__ partial, int nblk, int K,
                                                          int mode, double *__restrict__ st,
                                                          double *__restrict__ out) {
  // 256 threads = K channels x groups; each group sums every G-th block partial.
  __shared__ double red[256];
  __shared__ double tot[8];
  const int t = threadIdx.x;
  const int G = 256 / K;
  if (t < G * K) {
    const int q = t % K, g = t / K;
    double a[4] = {0.0, 0.0, 0.0, 0.0};
    int b = g;
    for (; b + 3 * G < nblk; b += 4 * G) {
      double v[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) v[u] = partial[size_t(b + u * G) * K + q];
#pragma unroll
      for (int u = 0; u < 4; ++u) a[u] += v[u];
    }
    for (int u = 0; b < nblk; b += G, ++u) a[u & 3] += partial[size_t(b) * K + q];
    red[t] = (a[0] + a[1]) + (a[2] + a[3]);
  }
  __syncthreads();
  if (t < K) {
    double s = 0.0;
    for (int g = 0; g < G; ++g) s += red[g * K + t];
    tot[t] = s;
  }
  __syncthreads();
  const int q = t;
  if (q >= K) return;
  const double tq = tot[q];
  double *gamma = st, *alpha = st + 8, *beta = st + 16;
  if (mode == kSetGamma) {
    gamma[q] = tq;
  } else if (mode == kAlpha) {
    alpha[q] = (tq > 0.0) ? gamma[q] / tq : 0.0;
  } else if (mode == kBeta) {
    beta[q] = (gamma[q] > 0.0) ? tq / gamma[q] : 0.0;
    gamma[q] = tq;
  } else if (out) {
    out[q] = sqrt(tq);
  }
}

// y += sign * coef[ch] * x over n_items K-vectors.
__global__ void chan_axpy_kernel(float *__restrict__ y, const float *__restrict__ xv, const double *__restrict__ coef,
                                 float sign, int K, int64_t n) {
  for (int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; e < n; e += int64_t(gridDim.x) * blockDim.x)
    y[e] = fmaf(sign * float(coef[e % K]), xv[e], y[e]);
}

__global__ void fill_zero_kernel(float *__restrict__ y, int64_t n) {
  for (int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; e < n; e += int64_t(gridDim.x) * blockDim.x)
    y[e] = 0.0f;
}

// p = s + coef[ch] * p
__global__ void chan_xpby_kernel(float *__restrict__ p, const float *__restrict__ s, const double *__restrict__ coef,
                                 int K, int64_t n) {
  for (int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; e < n; e += int64_t(gridDim.x) * blockDim.x)
    p[e] = fmaf(float(coef[e % K]), p[e], s[e]);
}

hsn_status check_geom(hsn_ctx *ctx, const hsn_geom *g) {
  if (!g) return hsn::fail(ctx, HSN_ERR_INVALID_ARG, "geometry is NULL");
  if (g->n_views <= 0 || g->n_slices <= 0 || g->n_cols <= 0)
    return hsn::fail(ctx, HSN_ERR_SHAPE, "geometry sizes must be positive");
  if (g->k < 1 || g->k > 8) return hsn::fail(ctx, HSN_ERR_SHAPE, "k must be in 1..8 (got %d)", g->k);
  if (g->n_cols > 8192 || g->n_views > 65535 || g->n_slices > 65535)
    return hsn::fail(ctx, HSN_ERR_SHAPE, "geometry too large (n_cols <= 8192, n_views, n_slices <= 65535)");
  return HSN_OK;
}

// Per-view constants in float64 on the host; uploaded only when they change.
hsn_status upload_geom(hsn_ctx *ctx, const hsn_geom *g, hipStream_t st, const ViewGeom **out) {
  const int nv = int(g->n_views);
  std::vector<double> tab(size_t(nv) * 4);
  for (int v = 0; v < nv; ++v) {
    const double t = g->angles ? g->angles[v] : double(v) * M_PI / double(nv);
    const double cs = std::cos(t), sn = std::sin(t);
    const double w = std::fmax(std::fabs(cs), std::fabs(sn));
    tab[4 * v + 0] = cs;
    tab[4 * v + 1] = sn;
    tab[4 * v + 2] = w;
    tab[4 * v + 3] = 1.0 / w;
  }
  if (tab != ctx->geom_host) {
    if (ctx->geom_cap < tab.size()) {
      if (ctx->geom) {
        HSN_HIP(ctx, hipStreamSynchronize(st));
        HSN_HIP(ctx, hipFree(ctx->geom));
        ctx->geom = nullptr;
      }
      if (hipMalloc(&ctx->geom, tab.size() * sizeof(double)) != hipSuccess) {
        (void)hipGetLastError();
        ctx->geom_cap = 0;
        ctx->geom_host.clear();
        return hsn::fail(ctx, HSN_ERR_OOM, "geometry table allocation failed");
      }
      ctx->geom_cap = tab.size();
    }
    // Synchronous copy: queued kernels may still read the previous table.
    HSN_HIP(ctx, hipStreamSynchronize(st));
    HSN_HIP(ctx, hipMemcpy(ctx->geom, tab.data(), tab.size() * sizeof(double), hipMemcpyHostToDevice));
    ctx->geom_host = tab;
  }
  *out = reinterpret_cast<const ViewGeom *>(ctx->geom);
  return HSN_OK;
}

template <int K>
void launch_project(const float *x, float *s, const ViewGeom *geom, const hsn_geom *g, float alpha, float beta,
                    hipStream_t st) {
  const int n = int(g->n_cols);
  dim3 grid(unsigned((n + kRayThreads - 1) / kRayThreads), unsigned(g->n_slices), unsigned(g->n_views));
  project_kernel<K><<<grid, kRayThreads, 0, st>>>(x, s, geom, int(g->n_slices), n, alpha, beta);
}

template <int K>
void launch_backproject(const float *s, float *x, const ViewGeom *geom, const hsn_geom *g, float alpha, float beta,
                        hipStream_t st) {
  const int n = int(g->n_cols);
  dim3 grid(unsigned((n + kVoxThreads - 1) / kVoxThreads), unsigned(n), unsigned(g->n_slices));
  backproject_kernel<K><<<grid, kVoxThreads, 0, st>>>(s, x, geom, int(g->n_views), int(g->n_slices), n, alpha, beta);
}

#define HSN_DISPATCH_K(k, F, ...)   \
  switch (k) {                      \
    case 1: F<1>(__VA_ARGS__); break; \
    case 2: F<2>(__VA_ARGS__); break; \
    case 3: F<3>(__VA_ARGS__); break; \
    case 4: F<4>(__VA_ARGS__); break; \
    case 5: F<5>(__VA_ARGS__); break; \
    case 6: F<6>(__VA_ARGS__); break; \
    case 7: F<7>(__VA_ARGS__); break; \
    default: F<8>(__VA_ARGS__); break; \
  }

template <int K>
void launch_dot(const float *a, const float *b, int64_t n_items, double *partial, hipStream_t st) {
  chan_dot_kernel<K><<<kDotBlocks, kDotThreads, 0, st>>>(a, b, n_items, partial);
}

hsn_status check_align(hsn_ctx *ctx, const void *p, int k, const char *what) {
  const uintptr_t a = reinterpret_cast<uintptr_t>(p);
  const uintptr_t need = (k == 4 || k == 8) ? 16 : (k == 2 ? 8 : 4);
  if (a % need) return hsn::fail(ctx, HSN_ERR_INVALID_ARG, "%s must be %u-byte aligned for k=%d", what, unsigned(need), k);
  return HSN_OK;
}

}  // namespace

extern "C" hsn_status hsn_project(hsn_ctx *ctx, const hsn_geom *g, const float *x, float *s, float alpha, float beta,
                                  void *stream) {
  if (!ctx) return HSN_ERR_INVALID_ARG;
  hsn_status rc = check_geom(ctx, g);
  if (rc != HSN_OK) return rc;
  if (!x || !s) return hsn::fail(ctx, HSN_ERR_INVALID_ARG, "project: x and s are required");
  if ((rc = check_align(ctx, x, g->k, "x")) != HSN_OK || (rc = check_align(ctx, s, g->k, "s")) != HSN_OK) return rc;
  hsn::DeviceGuard dg(ctx->device);
  hipStream_t st = static_cast<hipStream_t>(stream);
  const ViewGeom *geom = nullptr;
  if ((rc = upload_geom(ctx, g, st, &geom)) != HSN_OK) return rc;
  hsn::prof_begin(ctx, HSN_KERN_PROJECT, st);
  HSN_DISPATCH_K(g->k, launch_project, x, s, geom, g, alpha, beta, st);
  hsn::prof_end(ctx, HSN_KERN_PROJECT, st);
  HSN_LAUNCHED(ctx);
  return HSN_OK;
}

extern "C" hsn_status hsn_backproject(hsn_ctx *ctx, const hsn_geom *g, const float *s, float *x, float alpha,
                                      float beta, void *stream) {
  if (!ctx) return HSN_ERR_INVALID_ARG;
  hsn_status rc = check_geom(ctx, g);
  if (rc != HSN_OK) return rc;
  if (!x || !s) return hsn::fail(ctx, HSN_ERR_INVALID_ARG, "backproject: x and s are required");
  if ((rc = check_align(ctx, x, g->k, "x")) != HSN_OK || (rc = check_align(ctx, s, g->k, "s")) != HSN_OK) return rc;
  hsn::DeviceGuard dg(ctx->device);
  hipStream_t st = static_cast<hipStream_t>(stream);
  const ViewGeom *geom = nullptr;
  if ((rc = upload_geom(ctx, g, st, &geom)) != HSN_OK) return rc;
  hsn::prof_begin(ctx, HSN_KERN_BACKPROJECT, st);
  HSN_DISPATCH_K(g->k, launch_backproject, s, x, geom, g, alpha, beta, st);
  hsn::prof_end(ctx, HSN_KERN_BACKPROJECT, st);
  HSN_LAUNCHED(ctx);
  return HSN_OK;
}

extern "C" hsn_status hsn_cgls(hsn_ctx *ctx, const hsn_geom *g, const float *sino, float *x, int n_iter,
                               double *resid, void *stream) {
  if (!ctx) return HSN_ERR_INVALID_ARG;
  hsn_status rc = check_geom(ctx, g);
  if (rc != HSN_OK) return rc;
  if (!sino || !x) return hsn::fail(ctx, HSN_ERR_INVALID_ARG, "cgls: sino and x are required");
  if (n_iter < 0) return hsn::fail(ctx, HSN_ERR_INVALID_ARG, "cgls: n_iter must be >= 0");
  if ((rc = check_align(ctx, x, g->k, "x")) != HSN_OK || (rc = check_align(ctx, sino, g->k, "sino")) != HSN_OK)
    return rc;
  hsn::DeviceGuard dg(ctx->device);
  hipStream_t st = static_cast<hipStream_t>(stream);
  const int K = g->k;
  const int64_t n = g->n_cols;
  const int64_t nx = g->n_slices * n * n;          // voxels
  const int64_t ns = g->n_views * g->n_slices * n; // rays
  const size_t need = hsn::Carver::need({sizeof(float) * ns * K, sizeof(float) * ns * K, sizeof(float) * nx * K,
                                         sizeof(float) * nx * K, sizeof(double) * kDotBlocks * 8,
                                         sizeof(double) * 24});
  if ((rc = hsn::ensure_ws(ctx, need)) != HSN_OK) return rc;
  const ViewGeom *geom = nullptr;
  if ((rc = upload_geom(ctx, g, st, &geom)) != HSN_OK) return rc;
  hsn::Carver cv(ctx->ws);
  float *r = cv.take<float>(ns * K), *q = cv.take<float>(ns * K);
  float *sv = cv.take<float>(nx * K), *p = cv.take<float>(nx * K);
  double *partial = cv.take<double>(kDotBlocks * 8), *scal = cv.take<double>(24);
  const int eb = 256;
  auto blocks = [&](int64_t m) { return unsigned(std::min<int64_t>((m + eb - 1) / eb, 4096)); };

  fill_zero_kernel<<<blocks(nx * K), eb, 0, st>>>(x, nx * K);
  HSN_HIP(ctx, hipMemcpyAsync(r, sino, sizeof(float) * ns * K, hipMemcpyDeviceToDevice, st));
  HSN_DISPATCH_K(K, launch_backproject, r, sv, geom, g, 1.0f, 0.0f, st);
  HSN_HIP(ctx, hipMemcpyAsync(p, sv, sizeof(float) * nx * K, hipMemcpyDeviceToDevice, st));
  HSN_DISPATCH_K(K, launch_dot, sv, sv, nx, partial, st);
  cgls_scalar_kernel<<<1, 256, 0, st>>>(partial, kDotBlocks, K, kSetGamma, scal, nullptr);
  if (resid) {
    HSN_DISPATCH_K(K, launch_dot, r, r, ns, partial, st);
    cgls_scalar_kernel<<<1, 256, 0, st>>>(partial, kDotBlocks, K, kResid, scal, resid);
  }
  for (int it = 0; it < n_iter; ++it) {
    hsn::prof_begin(ctx, HSN_KERN_PROJECT, st);
    HSN_DISPATCH_K(K, launch_project, p, q, geom, g, 1.0f, 0.0f, st);
    hsn::prof_end(ctx, HSN_KERN_PROJECT, st);
    HSN_DISPATCH_K(K, launch_dot, q, q, ns, partial, st);
    cgls_scalar_kernel<<<1, 256, 0, st>>>(partial, kDotBlocks, K, kAlpha, scal, nullptr);
    chan_axpy_kernel<<<blocks(nx * K), eb, 0, st>>>(x, p, scal + 8, 1.0f, K, nx * K);
    chan_axpy_kernel<<<blocks(ns * K), eb, 0, st>>>(r, q, scal + 8, -1.0f, K, ns * K);
    hsn::prof_begin(ctx, HSN_KERN_BACKPROJECT, st);
    HSN_DISPATCH_K(K, launch_backproject, r, sv, geom, g, 1.0f, 0.0f, st);
    hsn::prof_end(ctx, HSN_KERN_BACKPROJECT, st);
    HSN_DISPATCH_K(K, launch_dot, sv, sv, nx, partial, st);
    cgls_scalar_kernel<<<1, 256, 0, st>>>(partial, kDotBlocks, K, kBeta, scal, nullptr);
    chan_xpby_kernel<<<blocks(nx * K), eb, 0, st>>>(p, sv, scal + 16, K, nx * K);
    if (resid) {
      HSN_DISPATCH_K(K, launch_dot, r, r, ns, partial, st);
      cgls_scalar_kernel<<<1, 256, 0, st>>>(partial, kDotBlocks, K, kResid, scal, resid + size_t(it + 1) * K);
    }
  }
  HSN_LAUNCHED(ctx);
  return HSN_OK;
}
