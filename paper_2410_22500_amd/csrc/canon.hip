// hsn_canonicalize: the canonical form of an NMF pair p ~ V D^T (eq. 4).
// The factorisation is unique only up to positive column scaling and column
// permutation; the canonical form fixes both: D's columns get unit l2 norm
// (V's columns take the inverse scale) and the columns are ordered to match a
// reference library of spectra (the permutation with the largest summed
// cosine, first in lexicographic order on ties) or, without one, by
// descending norm of the scaled V columns.  Used to build the coefficient
// targets of the warm-start network.
//
// A one-block plan kernel computes the norms, cosines and the permutation
// (K! <= 40320 candidates spread over the threads) in float64; a grid-wide
// kernel then rewrites the rows of V and D in place.
#include "common.hpp"

#include <algorithm>

namespace hsn {
namespace {

constexpr int kPlanThreads = 256;

template <int K>
__global__ __launch_bounds__(kPlanThreads) void canon_plan_kernel(const float *__restrict__ V, int64_t n_p,
                                                                  const float *__restrict__ D, int64_t n_k,
                                                                  const float *__restrict__ lib, int *__restrict__ perm,
                                                                  float *__restrict__ scale) {
  constexpr int NS = K + K + K * K + K;  // |D_j|^2, |L_j|^2, D_a.L_b, |V_j|^2
  __shared__ double red[kPlanThreads / 64][NS];
  __shared__ double tot[NS];
  __shared__ double best_s[kPlanThreads];
  __shared__ int best_i[kPlanThreads];
  const int t = threadIdx.x;
  double acc[NS];
#pragma unroll
  for (int e = 0; e < NS; ++e) acc[e] = 0.0;
  for (int64_t r = t; r < n_k; r += kPlanThreads) {
    double d[K], l[K];
#pragma unroll
    for (int j = 0; j < K; ++j) {
      d[j] = D[r * K + j];
      l[j] = lib ? double(lib[r * K + j]) : 0.0;
      acc[j] += d[j] * d[j];
      acc[K + j] += l[j] * l[j];
    }
#pragma unroll
    for (int a = 0; a < K; ++a)
#pragma unroll
      for (int b = 0; b < K; ++b) acc[2 * K + a * K + b] += d[a] * l[b];
  }
  if (!lib) {
    for (int64_t r = t; r < n_p; r += kPlanThreads)
#pragma unroll
      for (int j = 0; j < K; ++j) {
        const double v = V[r * K + j];
        acc[2 * K + K * K + j] += v * v;
      }
  }
#pragma unroll
  for (int e = 0; e < NS; ++e) {
    const double s = wave_sum_all(acc[e]);
    if ((t & 63) == 0) red[t >> 6][e] = s;
  }
  __syncthreads();
  for (int e = t; e < NS; e += kPlanThreads) {
    double s = 0.0;
    for (int w = 0; w < kPlanThreads / 64; ++w) s += red[w][e];
    tot[e] = s;
  }
  __syncthreads();
  if (lib) {
    int fact = 1;
    for (int i = 2; i <= K; ++i) fact *= i;
    double bs = -1e300;
    int bi = INT_MAX;
    for (int idx = t; idx < fact; idx += kPlanThreads) {
      // Lehmer decoding of the lexicographic rank idx.
      int avail[K], pm[K];
#pragma unroll
      for (int i = 0; i < K; ++i) avail[i] = i;
      int rem = idx, f = fact;
      for (int m = 0; m < K; ++m) {
        f /= (K - m);
        const int q = rem / f;
        rem -= q * f;
        pm[m] = avail[q];
        for (int i = q; i < K - 1 - m; ++i) avail[i] = avail[i + 1];
      }
      double s = 0.0;
      for (int m = 0; m < K; ++m) {
        const double dn = tot[pm[m]] > 0.0 ? sqrt(tot[pm[m]]) : 1.0;
        const double ln = sqrt(tot[K + m]);
        s += tot[2 * K + pm[m] * K + m] / (dn * ln);
      }
      if (s > bs) {  // idx increases, so ties keep the earlier rank
        bs = s;
        bi = idx;
      }
    }
    best_s[t] = bs;
    best_i[t] = bi;
    __syncthreads();
    if (t == 0) {
      double s = best_s[0];
      int b = best_i[0];
      for (int i = 1; i < kPlanThreads; ++i)
        if (best_s[i] > s || (best_s[i] == s && best_i[i] < b)) {
          s = best_s[i];
          b = best_i[i];
        }
      int avail[K];
      for (int i = 0; i < K; ++i) avail[i] = i;
      int rem = b, f = fact;
      for (int m = 0; m < K; ++m) {
        f /= (K - m);
        const int q = rem / f;
        rem -= q * f;
        perm[m] = avail[q];
        for (int i = q; i < K - 1 - m; ++i) avail[i] = avail[i + 1];
      }
    }
  } else if (t == 0) {
    // Stable sort by descending |V_j| * |D_j| (the norm of the scaled column).
    double key[K];
    int ord[K];
    for (int j = 0; j < K; ++j) {
      const double dn = tot[j] > 0.0 ? sqrt(tot[j]) : 1.0;
      key[j] = sqrt(tot[2 * K + K * K + j]) * dn;
      ord[j] = j;
    }
    for (int i = 1; i < K; ++i) {
      const int o = ord[i];
      int j = i - 1;
      while (j >= 0 && key[ord[j]] < key[o]) {
        ord[j + 1] = ord[j];
        --j;
      }
      ord[j + 1] = o;
    }
    for (int m = 0; m < K; ++m) perm[m] = ord[m];
  }
  if (t < K) scale[t] = tot[t] > 0.0 ? float(sqrt(tot[t])) : 1.0f;
}

// Row m of the output is column perm[m] of the input, scaled.
template <int K>
__global__ __launch_bounds__(256) void canon_apply_kernel(float *__restrict__ V, int64_t n_p, float *__restrict__ D,
                                                          int64_t n_k, const int *__restrict__ perm,
                                                          const float *__restrict__ scale) {
  int pm[K];
  float s[K];
#pragma unroll
  for (int j = 0; j < K; ++j) {
    pm[j] = perm[j];
    s[j] = scale[pm[j]];
  }
  for (int64_t r = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; r < n_p + n_k;
       r += int64_t(gridDim.x) * blockDim.x) {
    const bool is_v = r < n_p;
    float *row = is_v ? V + r * K : D + (r - n_p) * K;
    float in[K];
#pragma unroll
    for (int j = 0; j < K; ++j) in[j] = row[j];
#pragma unroll
    for (int m = 0; m < K; ++m) {
      float x = in[0];
#pragma unroll
      for (int j = 1; j < K; ++j)
        if (pm[m] == j) x = in[j];
      row[m] = is_v ? x * s[m] : x / s[m];
    }
  }
}

}  // namespace
}  // namespace hsn

extern "C" hsn_status hsn_canonicalize(hsn_ctx *ctx, float *V, int64_t n_p, float *D, int64_t n_k, int k,
                                       const float *library, void *stream) {
  using namespace hsn;
  if (!ctx) return HSN_ERR_INVALID_ARG;
  if (!V || !D) return fail(ctx, HSN_ERR_INVALID_ARG, "canonicalize: V and D are required");
  if (k < 1 || k > 8) return fail(ctx, HSN_ERR_SHAPE, "canonicalize: k must be in 1..8 (got %d)", k);
  if (n_p < 0 || n_k < 1) return fail(ctx, HSN_ERR_SHAPE, "canonicalize: need n_p >= 0, n_k >= 1");
  DeviceGuard dg(ctx->device);
  hsn_status rc = ensure_ws(ctx, 1024);
  if (rc != HSN_OK) return rc;
  hipStream_t st = static_cast<hipStream_t>(stream);
  int *perm = static_cast<int *>(ctx->ws);
  float *scale = reinterpret_cast<float *>(static_cast<char *>(ctx->ws) + 256);
  const int nb = int(std::min<int64_t>((n_p + n_k + 255) / 256, 4 * int64_t(ctx->num_cu)));
#define HSN_CANON(KK)                                                                                    \
  case KK:                                                                                              \
    canon_plan_kernel<KK><<<1, kPlanThreads, 0, st>>>(V, n_p, D, n_k, library, perm, scale);            \
    canon_apply_kernel<KK><<<nb, 256, 0, st>>>(V, n_p, D, n_k, perm, scale);                            \
    break;
  switch (k) {
    HSN_CANON(1) HSN_CANON(2) HSN_CANON(3) HSN_CANON(4) HSN_CANON(5) HSN_CANON(6) HSN_CANON(7) HSN_CANON(8)
  }
#undef HSN_CANON
  HSN_LAUNCHED(ctx);
  return HSN_OK;
}
