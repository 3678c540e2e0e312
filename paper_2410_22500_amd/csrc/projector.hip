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

#include <algorithm>
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
constexpr int kXcds = 8;  // MI355X: 8 XCDs, each with its own L2; workgroups go round-robin over them

// XCD-aware block order: with >= 8 slices, block id b runs on XCD b % 8 and
// every block of a slice lands on the same XCD (slice = xcd + 8 q), so the
// slice's image (or sinogram) is read from one L2 by all of its views or
// rows.  The grid is padded to a multiple of 8 slices; blocks of padding
// slices exit at once.  Fewer than 8 slices: plain slice-major order.
struct BlockSlot {
  int slice, rest;
};
__device__ __forceinline__ BlockSlot block_slot(unsigned id, int n_slices, int per_slice) {
  BlockSlot b;
  if (n_slices >= kXcds) {
    const unsigned xcd = id % kXcds, local = id / kXcds;
    b.slice = int(xcd + kXcds * (local / unsigned(per_slice)));
    b.rest = int(local % unsigned(per_slice));
  } else {
    b.slice = int(id / unsigned(per_slice));
    b.rest = int(id % unsigned(per_slice));
  }
  return b;
}
inline unsigned slot_grid(int64_t n_slices, int64_t per_slice) {
  const int64_t s = n_slices >= kXcds ? (n_slices + kXcds - 1) / kXcds * kXcds : n_slices;
  return unsigned(s * per_slice);
}

// Block partial of per-channel sums of squares of the values each thread
// wrote (fused CGLS dot products): partial[block][q].
template <int K, int NT>
__device__ __forceinline__ void block_sumsq(const float (&v)[K], bool valid, double *__restrict__ partial,
                                            size_t block) {
  __shared__ double red[NT / 64][K];
#pragma unroll
  for (int q = 0; q < K; ++q) {
    const double t = hsn::wave_sum_all(valid ? double(v[q]) * double(v[q]) : 0.0);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6][q] = t;
  }
  __syncthreads();
  if (threadIdx.x < K) {
    double t = 0.0;
#pragma unroll
    for (int w = 0; w < NT / 64; ++w) t += red[w][threadIdx.x];
    partial[block * K + threadIdx.x] = t;
  }
}

// s[v][r][c][:] = alpha * sum_taps a * x[r][j][i][:] + beta * s[v][r][c][:]
//
// The ray steps along the image axis closer to its direction: rows j for
// flat views (|cos| >= |sin|), columns i for steep ones.  Steep views read
// the transposed image xT[r][i][j][:] (= x[r][j][i][:]), so for every view
// the taps of neighbouring detector columns are neighbouring pixels of one
// image row and a wave's loads are contiguous.  Steps where the ray is
// outside the image are skipped by a conservative step range; at the image
// edge a tap index is clamped and its weight set to 0, which keeps the loop
// free of branches.  Optional: per-block sums of squares of the outputs.
template <int K>
__global__ __launch_bounds__(kRayThreads) void project_kernel(const float *__restrict__ x,
                                                              const float *__restrict__ xT, float *__restrict__ s,
                                                              const ViewGeom *__restrict__ geom, int n_slices,
                                                              int n_views, int n, float alpha, float beta,
                                                              double *__restrict__ sumsq) {
  const int nx = (n + kRayThreads - 1) / kRayThreads;
  const BlockSlot bs = block_slot(blockIdx.x, n_slices, n_views * nx);
  if (bs.slice >= n_slices) return;
  const int v = bs.rest / nx, cx = bs.rest % nx;
  const int r = bs.slice;
  const int c = cx * kRayThreads + threadIdx.x;
  const ViewGeom g = geom[v];
  const double h = 0.5 * double(n - 1);
  const double sc = double(c) - h;
  const float inv_w = float(g.inv_w);
  const bool steep = fabs(g.sn) > fabs(g.cs);
  const double a = steep ? g.sn : g.cs, b = steep ? g.cs : g.sn;
  // crossing position along the other axis at step m: u(m) = u0 + m du
  const double u0 = (sc + h * b) / a + h;
  const double du = -b / a;
  int m_lo = 0, m_hi = n - 1;
  if (du != 0.0) {
    const double ma = (-1.0 - u0) / du, mb = (double(n) - u0) / du;
    // clamped in float64 before the conversion (|du| may be ~1e-16)
    m_lo = int(fmax(0.0, floor(fmin(ma, mb)) - 1.0));
    m_hi = int(fmin(double(n - 1), ceil(fmax(ma, mb)) + 1.0));
  } else if (u0 < -1.0 || u0 >= double(n)) {
    m_hi = -1;
  }
  float acc[K];
#pragma unroll
  for (int q = 0; q < K; ++q) acc[q] = 0.0f;
  const float *img = (steep ? xT : x) + size_t(r) * n * n * K;
  if (c < n) {
#pragma unroll 4
    for (int m = m_lo; m <= m_hi; ++m) {
      const double u = fma(double(m), du, u0);
      const double fl = floor(u);
      const int t0 = int(fl);
      const float f = float(u - fl);
      const float w0 = (t0 >= 0 && t0 < n) ? (1.0f - f) * inv_w : 0.0f;
      const float w1 = (t0 + 1 >= 0 && t0 + 1 < n) ? f * inv_w : 0.0f;
      const int i0 = min(max(t0, 0), n - 1), i1 = min(max(t0 + 1, 0), n - 1);
      const float *row = img + size_t(m) * n * K;
      float p0[K], p1[K];
      load_k<K>(row + size_t(i0) * K, p0);
      load_k<K>(row + size_t(i1) * K, p1);
#pragma unroll
      for (int q = 0; q < K; ++q) acc[q] = fmaf(w1, p1[q], fmaf(w0, p0[q], acc[q]));
    }
  }
  float res[K];
  if (c < n) {
    float *out = s + ((size_t(v) * n_slices + r) * n + c) * K;
#pragma unroll
    for (int q = 0; q < K; ++q) {
      res[q] = (beta == 0.0f) ? alpha * acc[q] : fmaf(alpha, acc[q], beta * out[q]);
      out[q] = res[q];
    }
  }
  if (sumsq) block_sumsq<K, kRayThreads>(res, c < n, sumsq, (size_t(v) * n_slices + r) * nx + cx);
}

constexpr int kVoxThreads = 128;

// x[r][j][i][:] = alpha * sum_v sum_taps a * s[v][r][c][:] + beta * x[r][j][i][:]
// Views are unrolled by 4 with branch-free taps (clamped index, weight 0
// outside the detector) so that several loads are in flight.  Optional:
// per-block sums of squares of the outputs.
template <int K>
__global__ __launch_bounds__(kVoxThreads) void backproject_kernel(const float *__restrict__ s, float *__restrict__ x,
                                                                  const ViewGeom *__restrict__ geom, int n_views,
                                                                  int n_slices, int n, float alpha, float beta,
                                                                  double *__restrict__ sumsq) {
  const int nx = (n + kVoxThreads - 1) / kVoxThreads;
  const BlockSlot bs = block_slot(blockIdx.x, n_slices, n * nx);
  if (bs.slice >= n_slices) return;
  const int j = bs.rest / nx, cx = bs.rest % nx;
  const int r = bs.slice;
  const int i = cx * kVoxThreads + threadIdx.x;
  const bool ok = i < n;
  const double h = 0.5 * double(n - 1);
  const double xi = double(ok ? i : 0) - h, yj = double(j) - h;
  float acc[K];
#pragma unroll
  for (int q = 0; q < K; ++q) acc[q] = 0.0f;
  const size_t view_stride = size_t(n_slices) * n * K;
  const float *sr = s + size_t(r) * n * K;
#pragma unroll 4
  for (int v = 0; v < n_views; ++v) {
    const ViewGeom g = geom[v];
    const double u = fma(xi, g.cs, fma(yj, g.sn, h));   // detector position of the voxel centre
    const double fl = floor(u);
    const int c0 = int(fl);
    const float f = float(u - fl);                      // |d| of tap c0; tap c0+1 has |d| = 1 - f
    const float inv_w = float(g.inv_w);
    const float w0 = (c0 >= 0 && c0 < n) ? fmaxf(0.0f, 1.0f - f * inv_w) * inv_w : 0.0f;
    const float w1 = (c0 + 1 >= 0 && c0 + 1 < n) ? fmaxf(0.0f, 1.0f - (1.0f - f) * inv_w) * inv_w : 0.0f;
    const int k0 = min(max(c0, 0), n - 1), k1 = min(max(c0 + 1, 0), n - 1);
    const float *sv = sr + size_t(v) * view_stride;
    float p0[K], p1[K];
    load_k<K>(sv + size_t(k0) * K, p0);
    load_k<K>(sv + size_t(k1) * K, p1);
#pragma unroll
    for (int q = 0; q < K; ++q) acc[q] = fmaf(w1, p1[q], fmaf(w0, p0[q], acc[q]));
  }
  float res[K];
  if (ok) {
    float *out = x + ((size_t(r) * n + j) * n + i) * K;
#pragma unroll
    for (int q = 0; q < K; ++q) {
      res[q] = (beta == 0.0f) ? alpha * acc[q] : fmaf(alpha, acc[q], beta * out[q]);
      out[q] = res[q];
    }
  }
  if (sumsq) block_sumsq<K, kVoxThreads>(res, ok, sumsq, (size_t(r) * n + j) * nx + cx);
}

constexpr int kTile = 32;

// Per slice: xT[r][i][j][:] = x[r][j][i][:] through a 32 x 32 LDS tile.
// With coef (CGLS direction update), first p = sv + coef[q] * p is formed
// and written back (coef == NULL: p = sv), then transposed into pT.
template <int K>
__global__ __launch_bounds__(256) void xpby_transpose_kernel(float *__restrict__ p, float *__restrict__ pT,
                                                             const float *__restrict__ sv,
                                                             const double *__restrict__ coef, int n, int mode) {
  __shared__ float tile[kTile][kTile + 1][K];
  const int r = blockIdx.z;
  const int j0 = blockIdx.y * kTile, i0 = blockIdx.x * kTile;
  const size_t base = size_t(r) * n * n * K;
  float cf[K];
#pragma unroll
  for (int q = 0; q < K; ++q) cf[q] = (mode == 1) ? float(coef[q]) : 0.0f;
  for (int e = threadIdx.x; e < kTile * kTile; e += 256) {
    const int jj = e / kTile, ii = e % kTile;
    const int j = j0 + jj, i = i0 + ii;
    if (j < n && i < n) {
      const size_t o = base + (size_t(j) * n + i) * K;
      float val[K];
      if (mode == 0) {  // plain transpose of p
        load_k<K>(p + o, val);
      } else {          // p = sv + coef * p (mode 1), p = sv (mode 2)
        float a[K], b[K];
        load_k<K>(sv + o, a);
        if (mode == 1) load_k<K>(p + o, b);
#pragma unroll
        for (int q = 0; q < K; ++q) {
          val[q] = (mode == 1) ? fmaf(cf[q], b[q], a[q]) : a[q];
          p[o + q] = val[q];
        }
      }
#pragma unroll
      for (int q = 0; q < K; ++q) tile[jj][ii][q] = val[q];
    }
  }
  __syncthreads();
  for (int e = threadIdx.x; e < kTile * kTile; e += 256) {
    const int ii = e / kTile, jj = e % kTile;
    const int j = j0 + jj, i = i0 + ii;
    if (j < n && i < n) {
      float *o = pT + base + (size_t(i) * n + j) * K;
#pragma unroll
      for (int q = 0; q < K; ++q) o[q] = tile[jj][ii][q];
    }
  }
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

__global__ void fill_zero_kernel(float *__restrict__ y, int64_t n) {
  for (int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; e < n; e += int64_t(gridDim.x) * blockDim.x)
    y[e] = 0.0f;
}

// x += coef[ch] * p over nx values, then r -= coef[ch] * q over nr values (one launch).
__global__ void chan_axpy2_kernel(float *__restrict__ x, const float *__restrict__ p, int64_t nx,
                                  float *__restrict__ r, const float *__restrict__ q, int64_t nr,
                                  const double *__restrict__ coef, int K) {
  for (int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; e < nx + nr; e += int64_t(gridDim.x) * blockDim.x) {
    if (e < nx) {
      x[e] = fmaf(float(coef[e % K]), p[e], x[e]);
    } else {
      const int64_t f = e - nx;
      r[f] = fmaf(-float(coef[f % K]), q[f], r[f]);
    }
  }
}

hsn_status check_geom(hsn_ctx *ctx, const hsn_geom *g) {
  if (!g) return hsn::fail(ctx, HSN_ERR_INVALID_ARG, "geometry is NULL");
  if (g->n_views <= 0 || g->n_slices <= 0 || g->n_cols <= 0)
    return hsn::fail(ctx, HSN_ERR_SHAPE, "geometry sizes must be positive");
  if (g->k < 1 || g->k > 8) return hsn::fail(ctx, HSN_ERR_SHAPE, "k must be in 1..8 (got %d)", g->k);
  if (g->n_cols > 8192 || g->n_views > 65535 || g->n_slices > 65535)
    return hsn::fail(ctx, HSN_ERR_SHAPE, "geometry too large (n_cols <= 8192, n_views, n_slices <= 65535)");
  // 1-D launch grids: threads per launch must stay below 2^31.
  const int64_t sp = (g->n_slices + 7) / 8 * 8, nxc = (g->n_cols + 127) / 128 * 128;
  if (sp * g->n_views * nxc >= (int64_t(1) << 31) || sp * g->n_cols * nxc >= (int64_t(1) << 31))
    return hsn::fail(ctx, HSN_ERR_SHAPE, "geometry too large for one launch");
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

// Launch grids (1-D, padded, see block_slot) and the number of partials the
// fused sums of squares write (one per real block).
unsigned project_grid(const hsn_geom *g) {
  return slot_grid(g->n_slices, g->n_views * ((g->n_cols + kRayThreads - 1) / kRayThreads));
}
unsigned backproject_grid(const hsn_geom *g) {
  return slot_grid(g->n_slices, g->n_cols * ((g->n_cols + kVoxThreads - 1) / kVoxThreads));
}
size_t project_partials(const hsn_geom *g) {
  return size_t(g->n_slices) * g->n_views * ((g->n_cols + kRayThreads - 1) / kRayThreads);
}
size_t backproject_partials(const hsn_geom *g) {
  return size_t(g->n_slices) * g->n_cols * ((g->n_cols + kVoxThreads - 1) / kVoxThreads);
}

template <int K>
void launch_project(const float *x, const float *xT, float *s, const ViewGeom *geom, const hsn_geom *g, float alpha,
                    float beta, double *sumsq, hipStream_t st) {
  project_kernel<K><<<project_grid(g), kRayThreads, 0, st>>>(x, xT, s, geom, int(g->n_slices), int(g->n_views),
                                                             int(g->n_cols), alpha, beta, sumsq);
}

template <int K>
void launch_backproject(const float *s, float *x, const ViewGeom *geom, const hsn_geom *g, float alpha, float beta,
                        double *sumsq, hipStream_t st) {
  backproject_kernel<K><<<backproject_grid(g), kVoxThreads, 0, st>>>(s, x, geom, int(g->n_views),
                                                                     int(g->n_slices), int(g->n_cols), alpha, beta,
                                                                     sumsq);
}

// mode 0: pT = p^T; mode 1: p = sv + coef p, pT = p^T; mode 2: p = sv, pT = p^T.
template <int K>
void launch_xpby_t(float *p, float *pT, const float *sv, const double *coef, const hsn_geom *g, int mode,
                   hipStream_t st) {
  const unsigned t = unsigned((g->n_cols + kTile - 1) / kTile);
  xpby_transpose_kernel<K><<<dim3(t, t, unsigned(g->n_slices)), 256, 0, st>>>(p, pT, sv, coef, int(g->n_cols), mode);
}

bool has_steep_view(const hsn_geom *g) {
  const int nv = int(g->n_views);
  for (int v = 0; v < nv; ++v) {
    const double t = g->angles ? g->angles[v] : double(v) * M_PI / double(nv);
    if (std::fabs(std::sin(t)) > std::fabs(std::cos(t))) return true;
  }
  return false;
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
  // Steep views read a transposed copy of x (workspace).
  float *xT = nullptr;
  if (has_steep_view(g)) {
    const size_t nxk = size_t(g->n_slices) * g->n_cols * g->n_cols * g->k;
    if ((rc = hsn::ensure_ws(ctx, sizeof(float) * nxk)) != HSN_OK) return rc;
    xT = static_cast<float *>(ctx->ws);
  }
  if ((rc = upload_geom(ctx, g, st, &geom)) != HSN_OK) return rc;
  if (xT) HSN_DISPATCH_K(g->k, launch_xpby_t, const_cast<float *>(x), xT, nullptr, nullptr, g, 0, st);
  hsn::prof_begin(ctx, HSN_KERN_PROJECT, st);
  HSN_DISPATCH_K(g->k, launch_project, x, xT, s, geom, g, alpha, beta, nullptr, st);
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
  HSN_DISPATCH_K(g->k, launch_backproject, s, x, geom, g, alpha, beta, nullptr, st);
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
  // The sums of squares of A p and A^T r come from the projector epilogues
  // (one partial per block); ||r|| for the optional residual history from
  // the dot kernel.
  const size_t nb_proj = project_partials(g), nb_back = backproject_partials(g);
  const size_t n_part = std::max<size_t>({nb_proj, nb_back, size_t(kDotBlocks)});
  const size_t need = hsn::Carver::need({sizeof(float) * ns * K, sizeof(float) * ns * K, sizeof(float) * nx * K,
                                         sizeof(float) * nx * K, sizeof(float) * nx * K,
                                         sizeof(double) * n_part * K, sizeof(double) * 24});
  if ((rc = hsn::ensure_ws(ctx, need)) != HSN_OK) return rc;
  const ViewGeom *geom = nullptr;
  if ((rc = upload_geom(ctx, g, st, &geom)) != HSN_OK) return rc;
  hsn::Carver cv(ctx->ws);
  float *r = cv.take<float>(ns * K), *q = cv.take<float>(ns * K);
  float *sv = cv.take<float>(nx * K), *p = cv.take<float>(nx * K), *pT = cv.take<float>(nx * K);
  double *partial = cv.take<double>(n_part * K), *scal = cv.take<double>(24);
  const int eb = 256;
  auto blocks = [&](int64_t m) { return unsigned(std::min<int64_t>((m + eb - 1) / eb, 4096)); };

  fill_zero_kernel<<<blocks(nx * K), eb, 0, st>>>(x, nx * K);
  HSN_HIP(ctx, hipMemcpyAsync(r, sino, sizeof(float) * ns * K, hipMemcpyDeviceToDevice, st));
  hsn::prof_begin(ctx, HSN_KERN_BACKPROJECT, st);
  HSN_DISPATCH_K(K, launch_backproject, r, sv, geom, g, 1.0f, 0.0f, partial, st);
  hsn::prof_end(ctx, HSN_KERN_BACKPROJECT, st);
  cgls_scalar_kernel<<<1, 256, 0, st>>>(partial, int(nb_back), K, kSetGamma, scal, nullptr);
  HSN_DISPATCH_K(K, launch_xpby_t, p, pT, sv, nullptr, g, 2, st);
  if (resid) {
    HSN_DISPATCH_K(K, launch_dot, r, r, ns, partial, st);
    cgls_scalar_kernel<<<1, 256, 0, st>>>(partial, kDotBlocks, K, kResid, scal, resid);
  }
  for (int it = 0; it < n_iter; ++it) {
    hsn::prof_begin(ctx, HSN_KERN_PROJECT, st);
    HSN_DISPATCH_K(K, launch_project, p, pT, q, geom, g, 1.0f, 0.0f, partial, st);
    hsn::prof_end(ctx, HSN_KERN_PROJECT, st);
    cgls_scalar_kernel<<<1, 256, 0, st>>>(partial, int(nb_proj), K, kAlpha, scal, nullptr);
    chan_axpy2_kernel<<<blocks(nx * K + ns * K), eb, 0, st>>>(x, p, nx * K, r, q, ns * K, scal + 8, K);
    hsn::prof_begin(ctx, HSN_KERN_BACKPROJECT, st);
    HSN_DISPATCH_K(K, launch_backproject, r, sv, geom, g, 1.0f, 0.0f, partial, st);
    hsn::prof_end(ctx, HSN_KERN_BACKPROJECT, st);
    cgls_scalar_kernel<<<1, 256, 0, st>>>(partial, int(nb_back), K, kBeta, scal, nullptr);
    HSN_DISPATCH_K(K, launch_xpby_t, p, pT, sv, scal + 16, g, 1, st);
    if (resid) {
      HSN_DISPATCH_K(K, launch_dot, r, r, ns, partial, st);
      cgls_scalar_kernel<<<1, 256, 0, st>>>(partial, kDotBlocks, K, kResid, scal, resid + size_t(it + 1) * K);
    }
  }
  HSN_LAUNCHED(ctx);
  return HSN_OK;
}
