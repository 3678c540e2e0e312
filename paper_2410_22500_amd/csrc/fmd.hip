// hsn_fmd: the semi-supervised tail of fast material decomposition (Alg. 2).
//
//   T[i][j]  = mean over the voxels n of region i of x^s[n][j]          eq. (7)
//   x^m[n]   = argmin_{x >= 0} || x^s[n] - x T ||^2, row by row         eq. (8)
//   D^m      = D^s T^T                                                  eq. (9)
//
// Regions come as one label per voxel (the paper's masks M_i; the
// clustering that would produce them without labels is not part of this
// path).  The region sums are per-block partials added in a fixed order, so
// T is deterministic; every row solve uses the exact active-set NNLS of the
// ANLS polish with FP64 Cholesky factors of the principal submatrices of
// G = T T^T.
#include "nmf_common.hpp"

#include <algorithm>

namespace hsn {
namespace {

constexpr int kFmdThreads = 256;
constexpr int kFmdBlocks = 512;  // fixed partial count: fixed summation order

// partial[block][i][0..K-1] = sum of x^s rows of region i; [i][K] = count.
template <int M>
__global__ __launch_bounds__(kFmdThreads) void fmd_region_sums_kernel(const float *__restrict__ xs, int64_t n_x,
                                                                      int K, const int32_t *__restrict__ labels,
                                                                      double *__restrict__ partial) {
  double acc[M][9];
#pragma unroll
  for (int i = 0; i < M; ++i)
#pragma unroll
    for (int j = 0; j < 9; ++j) acc[i][j] = 0.0;
  for (int64_t n = int64_t(blockIdx.x) * kFmdThreads + threadIdx.x; n < n_x; n += int64_t(gridDim.x) * kFmdThreads) {
    const int l = labels[n];
#pragma unroll
    for (int i = 0; i < M; ++i) {
      if (l != i) continue;
      for (int j = 0; j < K; ++j) acc[i][j] += double(xs[n * K + j]);
      acc[i][8] += 1.0;
    }
  }
  __shared__ double red[kFmdThreads / 64][M * 9];
#pragma unroll
  for (int i = 0; i < M; ++i)
#pragma unroll
    for (int j = 0; j < 9; ++j) {
      const double s = wave_sum_all(acc[i][j]);
      if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6][i * 9 + j] = s;
    }
  __syncthreads();
  for (int e = threadIdx.x; e < M * 9; e += kFmdThreads) {
    double s = 0.0;
    for (int w = 0; w < kFmdThreads / 64; ++w) s += red[w][e];
    partial[size_t(blockIdx.x) * M * 9 + e] = s;
  }
}

// One block: T (float32 out, float64 in ws), G = T T^T and its factors.
template <int M>
__global__ __launch_bounds__(256) void fmd_transform_kernel(const double *__restrict__ partial, int nblk, int K,
                                                            float *__restrict__ T_out, double *__restrict__ Td,
                                                            double *__restrict__ G, double *__restrict__ chol) {
  __shared__ double tot[M * 9];
  __shared__ double g_s[M * M];
  __shared__ double t_s[M * 8];
  const int t = threadIdx.x;
  if (t < M * 9) {
    double s = 0.0;
    for (int b = 0; b < nblk; ++b) s += partial[size_t(b) * M * 9 + t];
    tot[t] = s;
  }
  __syncthreads();
  if (t < M * 8) {
    const int i = t / 8, j = t % 8;
    const double cnt = tot[i * 9 + 8];
    const double v = (j < K && cnt > 0.0) ? tot[i * 9 + j] / cnt : 0.0;  // empty region: zero row
    t_s[t] = v;
    Td[t] = v;
    if (j < K) T_out[i * K + j] = float(v);
  }
  __syncthreads();
  if (t < M * M) {
    const int a = t / M, b = t % M;
    double s = 0.0;
    for (int j = 0; j < K; ++j) s += t_s[a * 8 + j] * t_s[b * 8 + j];
    g_s[t] = s;
    G[t] = s;
  }
  __syncthreads();
  for (int m = t; m < (1 << M); m += blockDim.x) {
    if (m == 0) continue;
    double L[kCholStride];
    if (!chol_sub(g_s, M, unsigned(m), L)) L[0] = NAN;
    for (int e = 0; e < kCholStride; ++e) chol[size_t(m) * kCholStride + e] = L[e];
  }
}

// x^m[n][:] = NNLS with Gram G and right side h_i = sum_j T[i][j] x^s[n][j].
template <int M>
__global__ __launch_bounds__(256) void fmd_volumes_kernel(const float *__restrict__ xs, int64_t n_x, int K,
                                                          const double *__restrict__ Td, const double *__restrict__ G,
                                                          const double *__restrict__ chol, float *__restrict__ xm) {
  __shared__ double g_s[M * M];
  __shared__ double t_s[M * 8];
  if (threadIdx.x < M * M) g_s[threadIdx.x] = G[threadIdx.x];
  if (threadIdx.x < M * 8) t_s[threadIdx.x] = Td[threadIdx.x];
  __syncthreads();
  for (int64_t n = int64_t(blockIdx.x) * 256 + threadIdx.x; n < n_x; n += int64_t(gridDim.x) * 256) {
    double v[8];
    for (int j = 0; j < 8; ++j) v[j] = j < K ? double(xs[n * K + j]) : 0.0;
    double h[M], x[M];
#pragma unroll
    for (int i = 0; i < M; ++i) {
      double s = 0.0;
      for (int j = 0; j < K; ++j) s += t_s[i * 8 + j] * v[j];
      h[i] = s;
    }
    nnls_gram_row<M>(g_s, chol, h, x);
#pragma unroll
    for (int i = 0; i < M; ++i) xm[n * M + i] = float(x[i]);
  }
}

// D^m[b][i] = sum_j D^s[b][j] T[i][j]
template <int M>
__global__ __launch_bounds__(256) void fmd_spectra_kernel(const float *__restrict__ Ds, int64_t n_k, int K,
                                                          const double *__restrict__ Td, float *__restrict__ Dm) {
  __shared__ double t_s[M * 8];
  if (threadIdx.x < M * 8) t_s[threadIdx.x] = Td[threadIdx.x];
  __syncthreads();
  for (int64_t b = int64_t(blockIdx.x) * 256 + threadIdx.x; b < n_k; b += int64_t(gridDim.x) * 256) {
    double d[8];
    for (int j = 0; j < 8; ++j) d[j] = j < K ? double(Ds[b * K + j]) : 0.0;
#pragma unroll
    for (int i = 0; i < M; ++i) {
      double s = 0.0;
      for (int j = 0; j < K; ++j) s += d[j] * t_s[i * 8 + j];
      Dm[b * M + i] = float(s);
    }
  }
}

template <int M>
void launch_fmd(hipStream_t st, int num_cu, const float *xs, int64_t n_x, int K, const int32_t *labels,
                const float *Ds, int64_t n_k, float *T, float *xm, float *Dm, double *partial, double *Td, double *G,
                double *chol) {
  fmd_region_sums_kernel<M><<<kFmdBlocks, kFmdThreads, 0, st>>>(xs, n_x, K, labels, partial);
  fmd_transform_kernel<M><<<1, 256, 0, st>>>(partial, kFmdBlocks, K, T, Td, G, chol);
  const int nbv = int(std::max<int64_t>(1, std::min<int64_t>((n_x + 255) / 256, 8 * int64_t(num_cu))));
  fmd_volumes_kernel<M><<<nbv, 256, 0, st>>>(xs, n_x, K, Td, G, chol, xm);
  const int nbs = int(std::max<int64_t>(1, std::min<int64_t>((n_k + 255) / 256, int64_t(num_cu))));
  fmd_spectra_kernel<M><<<nbs, 256, 0, st>>>(Ds, n_k, K, Td, Dm);
}

}  // namespace
}  // namespace hsn

extern "C" hsn_status hsn_fmd(hsn_ctx *ctx, const float *xs, int64_t n_x, int k, const int32_t *labels, int n_m,
                              const float *Ds, int64_t n_k, float *T, float *xm, float *Dm, void *stream) {
  using namespace hsn;
  if (!ctx) return HSN_ERR_INVALID_ARG;
  if (!xs || !labels || !Ds || !T || !xm || !Dm) return fail(ctx, HSN_ERR_INVALID_ARG, "fmd: NULL pointer");
  if (k < 1 || k > 8 || n_m < 1 || n_m > 8) return fail(ctx, HSN_ERR_SHAPE, "fmd: k and n_m must be in 1..8");
  if (n_x < 1 || n_k < 1) return fail(ctx, HSN_ERR_SHAPE, "fmd: need n_x >= 1 and n_k >= 1");
  DeviceGuard dg(ctx->device);
  const size_t need = Carver::need({sizeof(double) * kFmdBlocks * 8 * 9, sizeof(double) * 64,
                                    sizeof(double) * 64, sizeof(double) * 256 * kCholStride});
  hsn_status rc = ensure_ws(ctx, need);
  if (rc != HSN_OK) return rc;
  Carver cv(ctx->ws);
  double *partial = cv.take<double>(size_t(kFmdBlocks) * 8 * 9);
  double *Td = cv.take<double>(64), *G = cv.take<double>(64);
  double *chol = cv.take<double>(256 * kCholStride);
  hipStream_t st = static_cast<hipStream_t>(stream);
  switch (n_m) {
#define HSN_M(MM) \
  case MM: launch_fmd<MM>(st, ctx->num_cu, xs, n_x, k, labels, Ds, n_k, T, xm, Dm, partial, Td, G, chol); break;
    HSN_M(1) HSN_M(2) HSN_M(3) HSN_M(4) HSN_M(5) HSN_M(6) HSN_M(7) HSN_M(8)
#undef HSN_M
  }
  HSN_LAUNCHED(ctx);
  return HSN_OK;
}
