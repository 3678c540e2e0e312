// Float32 NMF pass over p (eq. 4) on the vector ALUs, and the small kernels
// that close every iteration: G = F^T F with its principal Cholesky factors,
// the deterministic reduction of per-workgroup partials, and the D update.
//
// Pass layout: a persistent grid of 256-thread workgroups walks tiles of
// kRows rows of p.  Thread t owns the bins k = 1024 q + 4 t + e (q < NQ,
// e < 4), keeps D[k][:] and the N_D = P^T V partial for those bins in
// registers for the whole pass, and reads its bins of each row with one
// 16-byte load per q.  N_V = P D needs a sum over all bins of a row: per-lane
// partials are summed across the wave with DPP and across the four waves in
// LDS (fixed order, so the result is deterministic).
#include "nmf_common.hpp"

namespace hsn {

constexpr int kPassThreads = 256;
constexpr int kRows = 8;

template <int K, int NQ, int MODE, bool OBJ>
__global__ __launch_bounds__(kPassThreads) void pass_f32_kernel(
    const float *__restrict__ P, int64_t ldp, int64_t n_p, int n_k, float *__restrict__ V, float *__restrict__ NV,
    const float *__restrict__ D, const double *__restrict__ GD, float *__restrict__ part_nd,
    double *__restrict__ part_gv, double *__restrict__ part_obj) {
  const int t = threadIdx.x;
  const int lane = t & 63, wave = t >> 6;
  __shared__ float red[kPassThreads / 64][kRows * K];
  __shared__ float vnew[kRows][K];
  __shared__ double gd_s[K * K];
  __shared__ double obj_s[kPassThreads / 64];

  float d[NQ][4][K];
#pragma unroll
  for (int q = 0; q < NQ; ++q)
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int k = 1024 * q + 4 * t + e;
#pragma unroll
      for (int j = 0; j < K; ++j) d[q][e][j] = (k < n_k) ? D[k * K + j] : 0.0f;
    }
  float nd[NQ][4][K];
#pragma unroll
  for (int q = 0; q < NQ; ++q)
#pragma unroll
    for (int e = 0; e < 4; ++e)
#pragma unroll
      for (int j = 0; j < K; ++j) nd[q][e][j] = 0.0f;
  double gv = 0.0;
  double obj = 0.0;
  if ((MODE == kModeMU || MODE == kModeHALS) && t < K * K) gd_s[t] = GD[t];
  __syncthreads();

  const int64_t n_tiles = (n_p + kRows - 1) / kRows;
  for (int64_t tile = blockIdx.x; tile < n_tiles; tile += gridDim.x) {
    const int64_t row0 = tile * kRows;
    float p[kRows][NQ][4];
#pragma unroll
    for (int r = 0; r < kRows; ++r)
#pragma unroll
      for (int q = 0; q < NQ; ++q) {
        const int k = 1024 * q + 4 * t;
        float4 v4 = make_float4(0.f, 0.f, 0.f, 0.f);
        if (row0 + r < n_p && k < n_k) v4 = *reinterpret_cast<const float4 *>(P + (row0 + r) * ldp + k);
        p[r][q][0] = v4.x;
        p[r][q][1] = (k + 1 < n_k) ? v4.y : 0.0f;
        p[r][q][2] = (k + 2 < n_k) ? v4.z : 0.0f;
        p[r][q][3] = (k + 3 < n_k) ? v4.w : 0.0f;
      }

    if (MODE != kModeND) {
      // N_V partials of this thread's bins, summed over the workgroup.
#pragma unroll
      for (int r = 0; r < kRows; ++r)
#pragma unroll
        for (int j = 0; j < K; ++j) {
          float s = 0.0f;
#pragma unroll
          for (int q = 0; q < NQ; ++q)
#pragma unroll
            for (int e = 0; e < 4; ++e) s = fmaf(p[r][q][e], d[q][e][j], s);
          s = wave_sum_to_lane63(s);
          if (lane == 63) red[wave][r * K + j] = s;
        }
      __syncthreads();
      if (MODE == kModeHALS) {
        if (t < kRows) {
          const int r = t;
          const int64_t row = row0 + r;
          double h[K], x[K];
#pragma unroll
          for (int j = 0; j < K; ++j) {
            float s = 0.0f;
#pragma unroll
            for (int w = 0; w < kPassThreads / 64; ++w) s += red[w][r * K + j];
            h[j] = s;
            x[j] = (row < n_p) ? double(V[row * K + j]) : 0.0;
          }
          hals_row<K>(gd_s, h, x);
#pragma unroll
          for (int j = 0; j < K; ++j) {
            const float vn = (row < n_p) ? float(x[j]) : 0.0f;
            if (row < n_p) V[row * K + j] = vn;
            vnew[r][j] = vn;
          }
        }
      } else if (t < kRows * K) {
        const int r = t / K, j = t - (t / K) * K;
        const int64_t row = row0 + r;
        float s = 0.0f;
#pragma unroll
        for (int w = 0; w < kPassThreads / 64; ++w) s += red[w][t];
        if (MODE == kModeNV) {
          if (row < n_p) NV[row * K + j] = s;
        } else {
          // Lee-Seung: V <- V * N_V / (V G_D), denominator guarded only against 0.
          float vn = 0.0f;
          if (row < n_p) {
            float vr[K];
#pragma unroll
            for (int i = 0; i < K; ++i) vr[i] = V[row * K + i];
            double den = 0.0;
#pragma unroll
            for (int i = 0; i < K; ++i) den += double(vr[i]) * gd_s[i * K + j];
            vn = float(double(vr[j]) * double(s) / fmax(den, 1e-300));
            V[row * K + j] = vn;
          }
          vnew[r][j] = vn;
        }
      }
    } else {
      if (t < kRows * K) {
        const int r = t / K, j = t - (t / K) * K;
        vnew[r][j] = (row0 + r < n_p) ? V[(row0 + r) * K + j] : 0.0f;
      }
    }
    __syncthreads();

    if (MODE != kModeNV) {
      // N_D += P^T V_new for this thread's bins.
#pragma unroll
      for (int r = 0; r < kRows; ++r) {
        float vr[K];
#pragma unroll
        for (int j = 0; j < K; ++j) vr[j] = vnew[r][j];
#pragma unroll
        for (int q = 0; q < NQ; ++q)
#pragma unroll
          for (int e = 0; e < 4; ++e)
#pragma unroll
            for (int j = 0; j < K; ++j) nd[q][e][j] = fmaf(p[r][q][e], vr[j], nd[q][e][j]);
      }
      if (t < K * K) {
        const int i = t / K, j = t - (t / K) * K;
        float s = 0.0f;
#pragma unroll
        for (int r = 0; r < kRows; ++r) s = fmaf(vnew[r][i], vnew[r][j], s);
        gv += double(s);
      }
      if (OBJ) {
        // ||P - V_new D^T||^2 over this thread's bins of the tile.
        float acc = 0.0f;
#pragma unroll
        for (int r = 0; r < kRows; ++r) {
          float vr[K];
#pragma unroll
          for (int j = 0; j < K; ++j) vr[j] = vnew[r][j];
#pragma unroll
          for (int q = 0; q < NQ; ++q)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
              float rec = 0.0f;
#pragma unroll
              for (int j = 0; j < K; ++j) rec = fmaf(vr[j], d[q][e][j], rec);
              const float df = p[r][q][e] - rec;
              acc = fmaf(df, df, acc);
            }
        }
        obj += double(acc);
      }
    }
    __syncthreads();
  }

  if (MODE != kModeNV) {
    float *dst = part_nd + size_t(blockIdx.x) * n_k * K;
#pragma unroll
    for (int q = 0; q < NQ; ++q)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int k = 1024 * q + 4 * t + e;
        if (k < n_k) {
#pragma unroll
          for (int j = 0; j < K; ++j) dst[k * K + j] = nd[q][e][j];
        }
      }
    if (t < K * K) part_gv[size_t(blockIdx.x) * K * K + t] = gv;
    if (OBJ) {
      obj = wave_sum_all(obj);
      if (lane == 0) obj_s[wave] = obj;
      __syncthreads();
      if (t == 0) {
        double s = 0.0;
        for (int w = 0; w < kPassThreads / 64; ++w) s += obj_s[w];
        part_obj[blockIdx.x] = s;
      }
    }
  }
}

// G = F^T F (float64) for F [n][K] float32, and (if want_chol) the packed
// Cholesky factors of all 2^K - 1 principal submatrices.  One workgroup.
template <int K>
__global__ __launch_bounds__(256) void gram_kernel(const float *__restrict__ F, int64_t n, double *__restrict__ G,
                                                   double *__restrict__ chol, int want_chol) {
  const int t = threadIdx.x;
  __shared__ double red[4][K * K];
  __shared__ double g_s[K * K];
  double acc[K * K];
#pragma unroll
  for (int i = 0; i < K * K; ++i) acc[i] = 0.0;
  for (int64_t k = t; k < n; k += 256) {
    double f[K];
#pragma unroll
    for (int j = 0; j < K; ++j) f[j] = F[k * K + j];
#pragma unroll
    for (int i = 0; i < K; ++i)
#pragma unroll
      for (int j = 0; j < K; ++j) acc[i * K + j] += f[i] * f[j];
  }
#pragma unroll
  for (int i = 0; i < K * K; ++i) {
    const double s = wave_sum_all(acc[i]);
    if ((t & 63) == 0) red[t >> 6][i] = s;
  }
  __syncthreads();
  if (t < K * K) {
    const double s = red[0][t] + red[1][t] + red[2][t] + red[3][t];
    g_s[t] = s;
    G[t] = s;
  }
  __syncthreads();
  if (want_chol && t >= 1 && t < (1 << K)) {
    double L[kCholStride];
    if (!chol_sub(g_s, K, unsigned(t), L)) L[0] = NAN;
    for (int i = 0; i < kCholStride; ++i) chol[size_t(t) * kCholStride + i] = L[i];
  }
}

// First-level reduction of the per-workgroup partials (fixed order).
// Grid (ceil(n_k*K / 256), kSplit).
template <int K>
__global__ __launch_bounds__(256) void reduce_kernel(const float *__restrict__ part_nd,
                                                     const double *__restrict__ part_gv,
                                                     const double *__restrict__ part_obj, int n_wg, int n_k,
                                                     int with_obj, double *__restrict__ red_nd,
                                                     double *__restrict__ red_gv, double *__restrict__ red_obj) {
  const int s = blockIdx.y;
  const int w0 = int((int64_t(n_wg) * s) / kSplit), w1 = int((int64_t(n_wg) * (s + 1)) / kSplit);
  const int64_t e = int64_t(blockIdx.x) * 256 + threadIdx.x;
  const int64_t n_e = int64_t(n_k) * K;
  if (e < n_e) {
    double acc = 0.0;
    for (int w = w0; w < w1; ++w) acc += part_nd[size_t(w) * n_e + e];
    red_nd[size_t(s) * n_e + e] = acc;
  }
  if (blockIdx.x == 0) {
    if (threadIdx.x < K * K) {
      double acc = 0.0;
      for (int w = w0; w < w1; ++w) acc += part_gv[size_t(w) * K * K + threadIdx.x];
      red_gv[s * K * K + threadIdx.x] = acc;
    } else if (threadIdx.x == K * K) {
      double acc = 0.0;
      if (with_obj)
        for (int w = w0; w < w1; ++w) acc += part_obj[w];
      red_obj[s] = acc;
    }
  }
}

// G_V = sum of the first-level sums; its factors when the D rows are solved
// exactly; the objective into the history.  One workgroup.
template <int K>
__global__ __launch_bounds__(256) void finish_gv_kernel(const double *__restrict__ red_gv,
                                                        const double *__restrict__ red_obj, double *__restrict__ GV,
                                                        double *__restrict__ chol, int want_chol,
                                                        double *__restrict__ hist_slot) {
  const int t = threadIdx.x;
  __shared__ double g_s[K * K];
  if (t < K * K) {
    double acc = 0.0;
    for (int s = 0; s < kSplit; ++s) acc += red_gv[s * K * K + t];
    g_s[t] = acc;
    GV[t] = acc;
  }
  if (t == 255 && hist_slot) {
    double acc = 0.0;
    for (int s = 0; s < kSplit; ++s) acc += red_obj[s];
    *hist_slot = acc;
  }
  __syncthreads();
  if (want_chol && t >= 1 && t < (1 << K)) {
    double L[kCholStride];
    if (!chol_sub(g_s, K, unsigned(t), L)) L[0] = NAN;
    for (int i = 0; i < kCholStride; ++i) chol[size_t(t) * kCholStride + i] = L[i];
  }
}

// D update, one thread per bin row k: MU (D <- D * N_D / (D G_V)) or the
// exact non-negative row solve with G_V.
template <int K, int MODE>
__global__ __launch_bounds__(256) void update_d_kernel(float *__restrict__ D, const double *__restrict__ red_nd,
                                                       const double *__restrict__ GV, const double *__restrict__ chol,
                                                       int n_k) {
  __shared__ double g_s[K * K];
  if (threadIdx.x < K * K) g_s[threadIdx.x] = GV[threadIdx.x];
  __syncthreads();
  const int k = blockIdx.x * 256 + threadIdx.x;
  if (k >= n_k) return;
  const size_t n_e = size_t(n_k) * K;
  double nd[K];
#pragma unroll
  for (int j = 0; j < K; ++j) {
    double acc = 0.0;
    for (int s = 0; s < kSplit; ++s) acc += red_nd[s * n_e + size_t(k) * K + j];
    nd[j] = acc;
  }
  if (MODE == kModeMU) {
    double dr[K];
#pragma unroll
    for (int j = 0; j < K; ++j) dr[j] = D[k * K + j];
#pragma unroll
    for (int j = 0; j < K; ++j) {
      double den = 0.0;
#pragma unroll
      for (int i = 0; i < K; ++i) den += dr[i] * g_s[i * K + j];
      D[k * K + j] = float(dr[j] * nd[j] / fmax(den, 1e-300));
    }
  } else if (MODE == kModeHALS) {
    double x[K];
#pragma unroll
    for (int j = 0; j < K; ++j) x[j] = D[k * K + j];
    hals_row<K>(g_s, nd, x);
#pragma unroll
    for (int j = 0; j < K; ++j) D[k * K + j] = float(x[j]);
  } else {
    double x[K];
    nnls_gram_row<K>(g_s, chol, nd, x);
#pragma unroll
    for (int j = 0; j < K; ++j) D[k * K + j] = float(x[j]);
  }
}

// Exact non-negative solve of every V row from N_V and the factors of G_D.
template <int K>
__global__ __launch_bounds__(256) void nnls_rows_kernel(const float *__restrict__ NV, const double *__restrict__ GD,
                                                        const double *__restrict__ chol, float *__restrict__ V,
                                                        int64_t n_p) {
  __shared__ double g_s[K * K];
  if (threadIdx.x < K * K) g_s[threadIdx.x] = GD[threadIdx.x];
  __syncthreads();
  for (int64_t row = int64_t(blockIdx.x) * 256 + threadIdx.x; row < n_p; row += int64_t(gridDim.x) * 256) {
    double h[K], x[K];
#pragma unroll
    for (int j = 0; j < K; ++j) h[j] = NV[row * K + j];
    nnls_gram_row<K>(g_s, chol, h, x);
#pragma unroll
    for (int j = 0; j < K; ++j) V[row * K + j] = float(x[j]);
  }
}

// ---------------------------------------------------------------------------
// Host-side launchers (called by the driver for a runtime K).
// ---------------------------------------------------------------------------
template <int K>
void launch_pass_f32_k(int mode, bool obj, int nq, int n_wg, hipStream_t st, const float *P, int64_t ldp, int64_t n_p,
                       int n_k, float *V, float *NV, const float *D, const double *GD, float *part_nd,
                       double *part_gv, double *part_obj) {
#define HSN_PASS(NQ_, M_, O_)                                                                                   \
  pass_f32_kernel<K, NQ_, M_, O_><<<n_wg, kPassThreads, 0, st>>>(P, ldp, n_p, n_k, V, NV, D, GD, part_nd, part_gv, \
                                                                 part_obj)
  if (nq == 1) {
    if (mode == kModeMU) {
      if (obj) HSN_PASS(1, kModeMU, true); else HSN_PASS(1, kModeMU, false);
    } else if (mode == kModeHALS) {
      if (obj) HSN_PASS(1, kModeHALS, true); else HSN_PASS(1, kModeHALS, false);
    } else if (mode == kModeNV) {
      HSN_PASS(1, kModeNV, false);
    } else {
      HSN_PASS(1, kModeND, true);
    }
  } else {
    if (mode == kModeMU) {
      if (obj) HSN_PASS(2, kModeMU, true); else HSN_PASS(2, kModeMU, false);
    } else if (mode == kModeHALS) {
      if (obj) HSN_PASS(2, kModeHALS, true); else HSN_PASS(2, kModeHALS, false);
    } else if (mode == kModeNV) {
      HSN_PASS(2, kModeNV, false);
    } else {
      HSN_PASS(2, kModeND, true);
    }
  }
#undef HSN_PASS
}

void launch_pass_f32(int K, int mode, bool obj, int nq, int n_wg, hipStream_t st, const float *P, int64_t ldp,
                     int64_t n_p, int n_k, float *V, float *NV, const float *D, const double *GD, float *part_nd,
                     double *part_gv, double *part_obj) {
  switch (K) {
#define HSN_K(KK) \
  case KK: launch_pass_f32_k<KK>(mode, obj, nq, n_wg, st, P, ldp, n_p, n_k, V, NV, D, GD, part_nd, part_gv, part_obj); break;
    HSN_K(1) HSN_K(2) HSN_K(3) HSN_K(4) HSN_K(5) HSN_K(6) HSN_K(7) HSN_K(8)
#undef HSN_K
  }
}

void launch_gram(int K, hipStream_t st, const float *F, int64_t n, double *G, double *chol, int want_chol) {
  switch (K) {
#define HSN_K(KK) case KK: gram_kernel<KK><<<1, 256, 0, st>>>(F, n, G, chol, want_chol); break;
    HSN_K(1) HSN_K(2) HSN_K(3) HSN_K(4) HSN_K(5) HSN_K(6) HSN_K(7) HSN_K(8)
#undef HSN_K
  }
}

void launch_reduce_update(int K, int mode_d, bool obj, hipStream_t st, const NmfWork &w, int n_wg, int n_k, float *D,
                          double *hist_slot) {
  const dim3 grid(unsigned((int64_t(n_k) * K + 255) / 256), kSplit);
  const unsigned ub = unsigned((n_k + 255) / 256);
  switch (K) {
#define HSN_K(KK)                                                                                             \
  case KK:                                                                                                    \
    reduce_kernel<KK><<<grid, 256, 0, st>>>(w.part_nd, w.part_gv, w.part_obj, n_wg, n_k, obj ? 1 : 0,         \
                                            w.red_nd, w.red_gv, w.red_obj);                                   \
    finish_gv_kernel<KK><<<1, 256, 0, st>>>(w.red_gv, w.red_obj, w.gv, w.chol, mode_d == kModeNV ? 1 : 0,     \
                                            obj ? hist_slot : nullptr);                                       \
    if (mode_d == kModeMU)                                                                                    \
      update_d_kernel<KK, kModeMU><<<ub, 256, 0, st>>>(D, w.red_nd, w.gv, w.chol, n_k);                       \
    else if (mode_d == kModeHALS)                                                                             \
      update_d_kernel<KK, kModeHALS><<<ub, 256, 0, st>>>(D, w.red_nd, w.gv, w.chol, n_k);                     \
    else                                                                                                      \
      update_d_kernel<KK, kModeNV><<<ub, 256, 0, st>>>(D, w.red_nd, w.gv, w.chol, n_k);                       \
    break;
    HSN_K(1) HSN_K(2) HSN_K(3) HSN_K(4) HSN_K(5) HSN_K(6) HSN_K(7) HSN_K(8)
#undef HSN_K
  }
}

void launch_nnls_rows(int K, hipStream_t st, const float *NV, const double *GD, const double *chol, float *V,
                      int64_t n_p, int n_blocks) {
  switch (K) {
#define HSN_K(KK) case KK: nnls_rows_kernel<KK><<<n_blocks, 256, 0, st>>>(NV, GD, chol, V, n_p); break;
    HSN_K(1) HSN_K(2) HSN_K(3) HSN_K(4) HSN_K(5) HSN_K(6) HSN_K(7) HSN_K(8)
#undef HSN_K
  }
}

}  // namespace hsn
