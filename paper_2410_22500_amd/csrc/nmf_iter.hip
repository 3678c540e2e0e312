// The kernels that close every NMF iteration (eq. 4) around the streaming
// passes, with all loop control kept on the device:
//
//   init      once per call: G_D = D^T D (float64), the Cholesky factors of its
//             principal submatrices when the first step solves rows exactly,
//             the bfloat16 operand images of D for the MFMA pass, control reset.
//   update_d  after every pass that accumulates N_D = P^T V_new:
//             - every block sums the per-workgroup partials of G_V and of the
//               objective (fixed order) and the N_D partials of its 16 bin rows;
//             - applies the D row rule (Lee-Seung MU, HALS sweep, or the exact
//               non-negative row solve with G_V's factors);
//             - block 0 appends the objective to the history and, when it
//               meets the tolerance, lowers stop_at to this iteration + 1;
//             - the last block to finish (arrival counter) sums the blocks'
//               D_new^T D_new partials into G_D for the next pass, plus its
//               factors when the next step solves rows exactly;
//             - rewrites the bfloat16 images of its rows for the MFMA pass.
//   nnls_rows the exact non-negative solve of every V row (ANLS), from N_V and
//             the factors of G_D.
// All sums run in a fixed order, so results are bitwise reproducible.
#include "nmf_common.hpp"

#include <climits>

namespace hsn {

constexpr int kUpdThreads = 1024;
constexpr int kUpdRows = 16;  // D rows per update block

// Row k of D -> its entries in the two bfloat16 operand images.
//   image 1 [k-step s][lane][8]: column n = lane % 16, bins 32 s + 8 (lane/16) + e;
//            n < 8 -> hi(D[k][n]), n >= 8 -> lo(D[k][n-8]).
//   image 3 [block b][lane][8]: bin 16 b + lane % 16; group g = lane / 16:
//            g 0,1 -> hi(D[bin][e]), g 2 -> lo(D[bin][e]), g 3 -> 0.
template <int K>
__device__ inline void write_images_row(uint16_t *__restrict__ img, int64_t ldb, int64_t k, const float (&d)[K],
                                        bool zero) {
  uint16_t *im1 = img;
  uint16_t *im3 = img + (ldb / 32) * 64 * 8;
  const int64_t s = k / 32, g = (k % 32) / 8, e = k % 8;
  for (int n = 0; n < 16; ++n) {
    const int j = n & 7;
    const float v = (!zero && j < K) ? d[j < K ? j : 0] : 0.0f;
    im1[((s * 64) + 16 * g + n) * 8 + e] = (n < 8) ? bf_hi(v) : bf_lo(v);
  }
  const int64_t b = k / 16, l16 = k % 16;
  for (int gg = 0; gg < 4; ++gg)
    for (int ee = 0; ee < 8; ++ee) {
      const float v = (!zero && ee < K && gg < 3) ? d[ee < K ? ee : 0] : 0.0f;
      im3[((b * 64) + 16 * gg + l16) * 8 + ee] = (gg == 2) ? bf_lo(v) : bf_hi(v);
    }
}

// D' entry of a float32 D entry: the bfloat16 hi + lo split that the MFMA
// pass multiplies with (exact in float32: 8 + 8 significand bits).
__device__ __forceinline__ float split_value(float v) {
  return bf16_bits_to_f32(bf_hi(v)) + bf16_bits_to_f32(bf_lo(v));
}

// Factors of all principal submatrices G[S,S] of G (K x K, in LDS) -> chol
// (packed lower, compact index order); with ginv, also their inverses
// G[S,S]^-1 = L^-T L^-1, embedded in a packed symmetric K x K matrix with
// zeros outside S, entry-major with stride kInvStride (the operand of
// nnls_enum_group).  A singular G[S,S] gets NaN as the first entry of both.
// chol may be null (inverses only).
template <int K>
__device__ inline void factor_all(const double *G, double *__restrict__ chol, double *__restrict__ ginv = nullptr) {
  for (int m = threadIdx.x; m < (1 << K); m += blockDim.x) {
    if (m == 0) continue;
    double L[kCholStride];
    const bool ok = chol_sub(G, K, unsigned(m), L);
    if (!ok) L[0] = NAN;
    if (chol)
      for (int i = 0; i < kCholStride; ++i) chol[size_t(m) * kCholStride + i] = L[i];
    if (!ginv) continue;
    double *out = ginv + m;  // entry e at out[e * kInvStride]
    if (!ok) {
      out[0] = NAN;
      for (int e = 1; e < tri(K); ++e) out[e * kInvStride] = 0.0;
      continue;
    }
    int idx[8];
    int s = 0;
    for (int i = 0; i < K; ++i)
      if (m & (1 << i)) idx[s++] = i;
    // M = L^-1 (lower), by forward substitution column by column
    double M[kCholStride];
    for (int c = 0; c < s; ++c) {
      for (int a = c; a < s; ++a) {
        double v = (a == c) ? 1.0 : 0.0;
        for (int b = c; b < a; ++b) v -= L[tri(a) + b] * M[tri(b) + c];
        M[tri(a) + c] = v / L[tri(a) + a];
      }
    }
    for (int e = 0; e < tri(K); ++e) out[e * kInvStride] = 0.0;
    // (M^T M)[a][b] = sum over c >= max(a, b) of M[c][a] M[c][b]
    for (int a = 0; a < s; ++a)
      for (int b = 0; b <= a; ++b) {
        double v = 0.0;
        for (int c = a; c < s; ++c) v += M[tri(c) + a] * M[tri(c) + b];
        out[sym(idx[a], idx[b]) * kInvStride] = v;
      }
  }
}

// G = D^T D over the n_k rows of D (split: of D', the bfloat16 hi + lo
// split of D) by one block, fixed order; g_s (LDS, K*K) holds it on return.
template <int K>
__device__ __forceinline__ void block_gram_d(const float *__restrict__ D, int n_k, bool split,
                                             double (*red)[K * K], double *__restrict__ g_s) {
  const int t = threadIdx.x;
  double acc[K * K];
#pragma unroll
  for (int i = 0; i < K * K; ++i) acc[i] = 0.0;
  for (int k = t; k < n_k; k += kUpdThreads) {
    float d[K];
#pragma unroll
    for (int j = 0; j < K; ++j) d[j] = split ? split_value(D[size_t(k) * K + j]) : D[size_t(k) * K + j];
#pragma unroll
    for (int i = 0; i < K; ++i)
#pragma unroll
      for (int j = 0; j < K; ++j) acc[i * K + j] += double(d[i]) * double(d[j]);
  }
#pragma unroll
  for (int i = 0; i < K * K; ++i) {
    const double v = wave_sum_all(acc[i]);
    if ((t & 63) == 0) red[t >> 6][i] = v;
  }
  __syncthreads();
  if (t < K * K) {
    double v = 0.0;
    for (int w = 0; w < kUpdThreads / 64; ++w) v += red[w][t];
    g_s[t] = v;
  }
  __syncthreads();
}

template <int K>
__device__ __forceinline__ void nmf_init_body(const float *__restrict__ D, int n_k, double *__restrict__ GD,
                                              double *__restrict__ chol, int want_chol, uint16_t *__restrict__ img,
                                              int64_t ldb, NmfCtrl *__restrict__ ctrl,
                                              double *__restrict__ ginv = nullptr,
                                              double *__restrict__ ginv16 = nullptr,
                                              float *__restrict__ dprev = nullptr) {
  const int t = threadIdx.x;
  __shared__ double red[kUpdThreads / 64][K * K];
  __shared__ double g_s[K * K];
  if (dprev)
    for (int e = t; e < n_k * K; e += kUpdThreads) dprev[e] = D[e];
  if (img) {
    for (int64_t k = t; k < ldb; k += kUpdThreads) {
      float d[K];
#pragma unroll
      for (int j = 0; j < K; ++j) d[j] = (k < n_k) ? D[k * K + j] : 0.0f;
      write_images_row<K>(img, ldb, k, d, k >= n_k);
    }
  }
  if (t == 0) {
    ctrl->stop_at = INT_MAX;
    ctrl->upd_ticket = 0;
    ctrl->hist_len = 0;
    ctrl->iter_base = 0;
    ctrl->numeric = 0;
    ctrl->last16 = 0.0;
    ctrl->adj = 0.0;
    ctrl->last_est = 0.0;
    ctrl->beta = kExtrapBeta0;
    ctrl->beta_bar = 1.0;
    ctrl->e_prev = INFINITY;
    ctrl->beta_use = 0.0;
    ctrl->e_prev_bf16 = -1;
  }
  block_gram_d<K>(D, n_k, false, red, g_s);
  if (t < K * K) GD[t] = g_s[t];
  if (want_chol) factor_all<K>(g_s, chol, ginv);
  if (ginv16 && want_chol) {
    __syncthreads();
    block_gram_d<K>(D, n_k, true, red, g_s);
    factor_all<K>(g_s, nullptr, ginv16);
  }
}

template <int K>
__global__ __launch_bounds__(kUpdThreads) void nmf_init_kernel(const float *__restrict__ D, int n_k, double *__restrict__ GD,
                                                               double *__restrict__ chol, int want_chol,
                                                               uint16_t *__restrict__ img, int64_t ldb,
                                                               NmfCtrl *__restrict__ ctrl, double *__restrict__ ginv,
                                                               double *__restrict__ ginv16, float *__restrict__ dprev) {
  nmf_init_body<K>(D, n_k, GD, chol, want_chol, img, ldb, ctrl, ginv, ginv16, dprev);
}

// RULE: kModeMU (Lee-Seung), kModeHALS (column sweep), kModeNV (exact NNLS rows)
// G_V = sum of the workgroups' partials of V_new^T V_new, and the objective,
// reduced once per pass (the D update reads them from ctrl->gvo): thread
// group g sums every G-th partial (8 loads in flight), then the groups are
// summed in order.  red: LDS of kUpdThreads doubles.
template <int K>
__device__ __forceinline__ void reduce_gv_body(const double *__restrict__ part_gv, const double *__restrict__ part_obj,
                                               int n_wg, int has_obj, NmfCtrl *__restrict__ ctrl, int iter,
                                               double *__restrict__ red) {
  if (iter >= ctrl->stop_at) return;
  constexpr int E = K * K + 1;
  constexpr int G = kUpdThreads / E;
  const int t = threadIdx.x;
  if (t < G * E) {
    const int e = t % E, g = t / E;
    double acc = 0.0;
    if (e < K * K)
      acc = strided_sum(g, G, n_wg, [&](int w) { return part_gv[size_t(w) * K * K + e]; });
    else if (has_obj)
      acc = strided_sum(g, G, n_wg, [&](int w) { return part_obj[w]; });
    red[g * E + e] = acc;
  }
  __syncthreads();
  if (t < E) {
    double s = 0.0;
    for (int g = 0; g < G; ++g) s += red[g * E + t];
    ctrl->gvo[t] = s;
  }
}

template <int K>
__global__ __launch_bounds__(kUpdThreads) void reduce_gv_kernel(const double *__restrict__ part_gv,
                                                                const double *__restrict__ part_obj, int n_wg,
                                                                int has_obj, NmfCtrl *__restrict__ ctrl, int iter) {
  __shared__ double red[kUpdThreads];
  reduce_gv_body<K>(part_gv, part_obj, n_wg, has_obj, ctrl, iter, red);
}

// LDS of one update block (all float64 unless noted).
template <int K, int RULE>
struct UpdLds {
  static constexpr int EB = kUpdRows * K;      // N_D entries of a block
  static constexpr int G2 = kUpdThreads / EB;
  static constexpr int NCH = (1 << K) * kCholStride / ((RULE == kModeNV) ? 1 : (1 << K));
  static constexpr int red2 = 0;
  static constexpr int gv = red2 + G2 * EB * 8;
  static constexpr int gd = gv + K * K * 8;
  static constexpr int nd = gd + K * K * 8;
  static constexpr int obj = nd + EB * 8;
  static constexpr int chol = obj + 8;
  static constexpr int dn = chol + NCH * 8;           // float [kUpdRows][K]
  static constexpr int bytes = (dn + kUpdRows * K * 4 + 15) / 16 * 16;
};

// One block `blk` of `n_blk` of the D update.
template <int K, int RULE>
__device__ __forceinline__ void update_d_body(
    float *__restrict__ D, const float *__restrict__ part_nd, int n_wg, int n_k, NmfCtrl *__restrict__ ctrl, int iter,
    int has_obj,
    double f_ref, double tol, double *__restrict__ hist, double *__restrict__ GD, double *__restrict__ chol,
    int next_chol, double *__restrict__ part_gd, uint16_t *__restrict__ img, int64_t ldb, int blk, int n_blk,
    char *__restrict__ lds, int bf16 = 0, const double *__restrict__ bias = nullptr,
    double *__restrict__ part_gd16 = nullptr, int no_stop = 0, float *__restrict__ dprev = nullptr) {
  if (iter >= ctrl->stop_at) return;
  const int t = threadIdx.x;
  using L = UpdLds<K, RULE>;
  constexpr int EB = L::EB, G2 = L::G2;
  double(*red2)[EB] = reinterpret_cast<double(*)[EB]>(lds + L::red2);
  double *gv_s = reinterpret_cast<double *>(lds + L::gv);
  double *gd_s = reinterpret_cast<double *>(lds + L::gd);
  double *nd_s = reinterpret_cast<double *>(lds + L::nd);
  float(*dn_s)[K] = reinterpret_cast<float(*)[K]>(lds + L::dn);
  double &obj_s = *reinterpret_cast<double *>(lds + L::obj);
  double *chol_s = reinterpret_cast<double *>(lds + L::chol);

  const int k0 = blk * kUpdRows;
  // G_V and the objective were reduced by the pass's last workgroup.
  if (t < K * K) gv_s[t] = ctrl->gvo[t];
  else if (t == K * K) obj_s = has_obj ? ctrl->gvo[K * K] : 0.0;
  // N_D of this block's rows.
  if (t < G2 * EB) {
    const int e = t % EB, g = t / EB;
    const int row = k0 + e / K;
    double acc = 0.0;
    if (row < n_k) {
      const size_t base = size_t(k0) * K + e;
      const size_t stride = size_t(n_k) * K;
      acc = strided_sum(g, G2, n_wg, [&](int w) { return double(part_nd[size_t(w) * stride + base]); });
    }
    red2[g][e] = acc;
  }
  __syncthreads();
  if (t >= 64 && t < 64 + EB) {
    const int e = t - 64;
    double s = 0.0;
    for (int g = 0; g < G2; ++g) s += red2[g][e];
    nd_s[e] = s;
  }
  __syncthreads();
  if (RULE == kModeNV) factor_all<K>(gv_s, chol_s);
  if (blk == 0 && t == 0 && has_obj) {
    const int h = ctrl->hist_len;
    hist[h] = obj_s;
    ctrl->hist_len = h + 1;
    // a step on the bfloat16 p (bf16 != 0) compares obj + bias + adj, an
    // estimate of the float32 objective (bias: the normalisation's
    // -||p - p_bf16||^2 or null; adj: the calibration against a float32 round)
    double ob = obj_s;
    if (bf16) {
      ctrl->last16 = obj_s;
      ob = obj_s + (bias ? *bias : 0.0) + ctrl->adj;
    }
    ctrl->last_est = ob;
    if (!isfinite(obj_s)) {
      // a non-finite objective (NaN or Inf in p or in the factors) ends the run
      ctrl->numeric = 1;
      ctrl->stop_at = iter + 1;
    } else if (!no_stop && f_ref > 0.0 && (ob - f_ref) / f_ref <= tol) {
      ctrl->stop_at = iter + 1;
    }
  }
  __syncthreads();

  // Row rule, one thread per bin row.
  if (t < kUpdRows) {
    const int k = k0 + t;
    float dn[K];
    if (k < n_k) {
      double nd[K], x[K];
#pragma unroll
      for (int j = 0; j < K; ++j) {
        nd[j] = nd_s[t * K + j];
        x[j] = D[size_t(k) * K + j];
      }
      if (RULE == kModeMU) {
        double y[K];
#pragma unroll
        for (int j = 0; j < K; ++j) {
          double den = 0.0;
#pragma unroll
          for (int i = 0; i < K; ++i) den += x[i] * gv_s[i * K + j];
          y[j] = x[j] * nd[j] / fmax(den, 1e-300);
        }
#pragma unroll
        for (int j = 0; j < K; ++j) x[j] = y[j];
      } else if (RULE == kModeHALS) {
        hals_row<K>(gv_s, nd, x);
      } else {
        nnls_gram_row<K>(gv_s, chol_s, nd, x);
      }
      if (RULE == kModeNV && dprev) {
        // extrapolated ANLS: D_hat = max(0, D_new + beta (D_new - D_prev)),
        // D_prev <- D_new; the next round solves V for D_hat
        const double bu = ctrl->beta_use;
#pragma unroll
        for (int j = 0; j < K; ++j) {
          const float dnew = float(x[j]);
          const double dp = dprev[size_t(k) * K + j];
          dprev[size_t(k) * K + j] = dnew;
          if (bu > 0.0) x[j] = fmax(0.0, double(dnew) + bu * (double(dnew) - dp));
        }
      }
#pragma unroll
      for (int j = 0; j < K; ++j) {
        dn[j] = float(x[j]);
        D[size_t(k) * K + j] = dn[j];
      }
      if (img) write_images_row<K>(img, ldb, k, dn, false);
    } else {
#pragma unroll
      for (int j = 0; j < K; ++j) dn[j] = 0.0f;
    }
#pragma unroll
    for (int j = 0; j < K; ++j) dn_s[t][j] = dn[j];
  }
  __syncthreads();
  // This block's share of G_D for the next pass (summed by the finish kernel),
  // and of G_D' (the split D of the MFMA pass) when asked for.
  if (t < K * K) {
    const int i = t / K, j = t % K;
    double s = 0.0;
    for (int r = 0; r < kUpdRows; ++r) s += double(dn_s[r][i]) * double(dn_s[r][j]);
    part_gd[size_t(blk) * K * K + t] = s;
  } else if (part_gd16 && t >= 64 && t < 64 + K * K) {
    const int e = t - 64, i = e / K, j = e % K;
    double s = 0.0;
    for (int r = 0; r < kUpdRows; ++r) s += double(split_value(dn_s[r][i])) * double(split_value(dn_s[r][j]));
    part_gd16[size_t(blk) * K * K + e] = s;
  }
}

// After the D update: G_D = sum of the update blocks' partials (thread group
// g sums every G-th block, then the groups in order) and, when the next step
// solves rows exactly, the factors of its principal submatrices.  A kernel of
// its own: the update's blocks would otherwise need device-scope fences to
// hand their partials to a last block, which on this GPU flushes the L2.
template <int K>
__device__ __forceinline__ void finish_gd_body(const double *__restrict__ part_gd, int n_blk, double *__restrict__ GD,
                                               double *__restrict__ chol, int next_chol,
                                               const NmfCtrl *__restrict__ ctrl, int iter, double *__restrict__ red,
                                               double *__restrict__ gd_s, double *__restrict__ ginv = nullptr,
                                               const double *__restrict__ part_gd16 = nullptr,
                                               double *__restrict__ ginv16 = nullptr) {
  if (iter >= ctrl->stop_at) return;
  constexpr int G = kUpdThreads / (K * K);
  const int t = threadIdx.x;
  for (int pass = 0; pass < ((part_gd16 && ginv16 && next_chol) ? 2 : 1); ++pass) {
    const double *src = pass == 0 ? part_gd : part_gd16;
    if (t < G * K * K) {
      const int e = t % (K * K), g = t / (K * K);
      red[g * K * K + e] = strided_sum(g, G, n_blk, [&](int b) { return src[size_t(b) * K * K + e]; });
    }
    __syncthreads();
    if (t < K * K) {
      double s = 0.0;
      for (int g = 0; g < G; ++g) s += red[g * K * K + t];
      gd_s[t] = s;
      if (pass == 0) GD[t] = s;
    }
    __syncthreads();
    // G_D -> chol, ginv; G_D' -> ginv16 (inverses only)
    if (next_chol) factor_all<K>(gd_s, pass == 0 ? chol : nullptr, pass == 0 ? ginv : ginv16);
    __syncthreads();
  }
}

template <int K>
__global__ __launch_bounds__(kUpdThreads) void finish_gd_kernel(const double *__restrict__ part_gd, int n_blk,
                                                                double *__restrict__ GD, double *__restrict__ chol,
                                                                int next_chol, const NmfCtrl *__restrict__ ctrl,
                                                                int iter, double *__restrict__ ginv,
                                                                const double *__restrict__ part_gd16,
                                                                double *__restrict__ ginv16) {
  __shared__ double red[kUpdThreads];
  __shared__ double gd_s[K * K];
  finish_gd_body<K>(part_gd, n_blk, GD, chol, next_chol, ctrl, iter, red, gd_s, ginv, part_gd16, ginv16);
}

template <int K, int RULE>
__global__ __launch_bounds__(kUpdThreads) void update_d_kernel(
    float *__restrict__ D, const float *__restrict__ part_nd, int n_wg, int n_k, NmfCtrl *__restrict__ ctrl, int iter,
    int has_obj,
    double f_ref, double tol, double *__restrict__ hist, double *__restrict__ GD, double *__restrict__ chol,
    int next_chol, double *__restrict__ part_gd, uint16_t *__restrict__ img, int64_t ldb, int bf16,
    const double *__restrict__ bias, double *__restrict__ part_gd16, float *__restrict__ dprev) {
  __shared__ __attribute__((aligned(16))) char lds[UpdLds<K, RULE>::bytes];
  update_d_body<K, RULE>(D, part_nd, n_wg, n_k, ctrl, iter, has_obj, f_ref, tol, hist, GD, chol, next_chol, part_gd,
                         img, ldb, int(blockIdx.x), int(gridDim.x), lds, bf16, bias, part_gd16, 0, dprev);
}

template <int K>
__device__ __forceinline__ void nnls_rows_body(const float *__restrict__ NV, const double *__restrict__ GD,
                                               const double *__restrict__ chol, float *__restrict__ V, int64_t n_p,
                                               const NmfCtrl *__restrict__ ctrl, int iter, int blk, int n_blk) {
  if (iter >= ctrl->stop_at) return;
  __shared__ double g_s[K * K];
  if (threadIdx.x < K * K) g_s[threadIdx.x] = GD[threadIdx.x];
  __syncthreads();
  for (int64_t row = int64_t(blk) * 256 + threadIdx.x; row < n_p; row += int64_t(n_blk) * 256) {
    double h[K], x[K];
#pragma unroll
    for (int j = 0; j < K; ++j) h[j] = NV[row * K + j];
    nnls_gram_row<K>(g_s, chol, h, x);
#pragma unroll
    for (int j = 0; j < K; ++j) V[row * K + j] = float(x[j]);
  }
}

template <int K>
__global__ __launch_bounds__(256) void nnls_rows_kernel(const float *__restrict__ NV, const double *__restrict__ GD,
                                                        const double *__restrict__ chol, float *__restrict__ V,
                                                        int64_t n_p, const NmfCtrl *__restrict__ ctrl, int iter) {
  nnls_rows_body<K>(NV, GD, chol, V, n_p, ctrl, iter, int(blockIdx.x), int(gridDim.x));
}

// ---------------------------------------------------------------------------
// Batched forms: one launch covers the blocks of many decompositions (block
// ranges per instance in BatchInst); iteration = the instance's iter_base +
// the step's position in the replayed chunk.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kUpdThreads) void batched_init_kernel(const BatchInst *__restrict__ d, int want_chol) {
  const BatchInst &b = d[blockIdx.x];
  switch (b.K) {
#define HSN_K(KK) \
  case KK: nmf_init_body<KK>(b.D, b.n_k, b.gd, b.chol, want_chol, b.img, b.img ? b.ldb_img : 0, b.ctrl); break;
    HSN_K(1) HSN_K(2) HSN_K(3) HSN_K(4) HSN_K(5) HSN_K(6) HSN_K(7) HSN_K(8)
#undef HSN_K
    default: break;
  }
}

// One block per instance.
__global__ __launch_bounds__(kUpdThreads) void batched_reduce_gv_kernel(const BatchInst *__restrict__ d, int iter_local,
                                                                        int has_obj, int bf16) {
  __shared__ double red[kUpdThreads];
  const BatchInst &b = d[blockIdx.x];
  const int iter = b.ctrl->iter_base + iter_local;
  const int n_wg = bf16 ? b.n_wgb : b.n_wg;  // partials of the pass that ran
  switch (b.K) {
#define HSN_K(KK) \
  case KK: reduce_gv_body<KK>(b.part_gv, b.part_obj, n_wg, has_obj, b.ctrl, iter, red); break;
    HSN_K(1) HSN_K(2) HSN_K(3) HSN_K(4) HSN_K(5) HSN_K(6) HSN_K(7) HSN_K(8)
#undef HSN_K
    default: break;
  }
}

// One block per instance.
__global__ __launch_bounds__(kUpdThreads) void batched_finish_gd_kernel(const BatchInst *__restrict__ d, int iter_local,
                                                                        int next_chol) {
  __shared__ double red[kUpdThreads];
  __shared__ double gd_s[64];
  const BatchInst &b = d[blockIdx.x];
  const int iter = b.ctrl->iter_base + iter_local;
  switch (b.K) {
#define HSN_K(KK) \
  case KK: finish_gd_body<KK>(b.part_gd, b.n_ub, b.gd, b.chol, next_chol, b.ctrl, iter, red, gd_s); break;
    HSN_K(1) HSN_K(2) HSN_K(3) HSN_K(4) HSN_K(5) HSN_K(6) HSN_K(7) HSN_K(8)
#undef HSN_K
    default: break;
  }
}

template <int RULE>
__global__ __launch_bounds__(kUpdThreads) void batched_update_kernel(const BatchInst *__restrict__ d, int n_inst,
                                                                     int iter_local, int has_obj, int next_chol,
                                                                     int bf16) {
  extern __shared__ __attribute__((aligned(16))) char lds[];
  const int i = batch_find(n_inst, int(blockIdx.x), [&](int j) { return d[j].ub0; });
  const BatchInst &b = d[i];
  const int blk = int(blockIdx.x) - b.ub0;
  if (blk >= b.n_ub) return;
  const int iter = b.ctrl->iter_base + iter_local;
  const int n_wg = bf16 ? b.n_wgb : b.n_wg;
  switch (b.K) {
#define HSN_K(KK)                                                                                                 \
  case KK:                                                                                                        \
    update_d_body<KK, RULE>(b.D, b.part_nd, n_wg, b.n_k, b.ctrl, iter, has_obj, b.f_ref, b.tol, b.hist, b.gd,   \
                            b.chol, next_chol, b.part_gd, b.img, b.img ? b.ldb_img : 0, blk, b.n_ub, lds, bf16, \
                            nullptr, nullptr, bf16);                                                             \
    break;
    HSN_K(1) HSN_K(2) HSN_K(3) HSN_K(4) HSN_K(5) HSN_K(6) HSN_K(7) HSN_K(8)
#undef HSN_K
    default: break;
  }
}

template <int K>
__global__ __launch_bounds__(256) void batched_rows_kernel(const BatchInst *__restrict__ d, int n_inst, int iter_local) {
  const int i = batch_find(n_inst, int(blockIdx.x), [&](int j) { return d[j].rb0; });
  const BatchInst &b = d[i];
  const int blk = int(blockIdx.x) - b.rb0;
  if (blk >= b.n_rb) return;
  const int iter = b.ctrl->iter_base + iter_local;
  nnls_rows_body<K>(b.NV, b.gd, b.chol, b.V, b.n_p, b.ctrl, iter, blk, b.n_rb);
}

__global__ void batched_advance_kernel(const BatchInst *__restrict__ d, int n_inst, int steps) {
  const int i = int(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n_inst) d[i].ctrl->iter_base += steps;
}

// Extrapolated ANLS: this round's weight, from the objective the pass just
// reduced (the stop estimate on p_bf16 steps).  A round whose estimate meets
// the stop test takes its exact D (the returned factors are then at least
// as good as the reported objective).  One thread; runs between the G_V
// reduction and the D update, so every update block reads the same weight.
__global__ void anls_beta_kernel(NmfCtrl *__restrict__ ctrl, int iter, int obj_index, double f_ref, double tol,
                                 int bf16, const double *__restrict__ bias) {
  if (iter >= ctrl->stop_at) return;
  double ob = ctrl->gvo[obj_index];
  if (bf16) ob += (bias ? *bias : 0.0) + ctrl->adj;
  const bool stop = !isfinite(ob) || (f_ref > 0.0 && (ob - f_ref) / f_ref <= tol);
  double use = 0.0;
  if (!stop) {
    if (ctrl->e_prev_bf16 >= 0 && ctrl->e_prev_bf16 != (bf16 ? 1 : 0)) {
      // the previous objective was measured on the other copy of p: not
      // comparable, so the weight stays and is used
      use = ctrl->beta;
    } else if (ob <= ctrl->e_prev) {
      ctrl->beta = fmin(ctrl->beta_bar, kExtrapGrow * ctrl->beta);
      ctrl->beta_bar = fmin(1.0, kExtrapCapGrow * ctrl->beta_bar);
      use = ctrl->beta;
    } else {
      ctrl->beta_bar = ctrl->beta;
      ctrl->beta = ctrl->beta / kExtrapShrink;
    }
  }
  ctrl->e_prev = ob;
  ctrl->e_prev_bf16 = bf16 ? 1 : 0;
  ctrl->beta_use = use;
}

// ---------------------------------------------------------------------------
// Launchers for a runtime K.
// ---------------------------------------------------------------------------
void launch_nmf_init(int K, hipStream_t st, const float *D, int n_k, const NmfWork &w, int want_chol, int64_t ldb) {
  switch (K) {
#define HSN_K(KK) \
  case KK: nmf_init_kernel<KK><<<1, kUpdThreads, 0, st>>>(D, n_k, w.gd, w.chol, want_chol, w.img, ldb, w.ctrl, w.ginv, \
                                                          w.ginv16, w.dprev); break;
    HSN_K(1) HSN_K(2) HSN_K(3) HSN_K(4) HSN_K(5) HSN_K(6) HSN_K(7) HSN_K(8)
#undef HSN_K
  }
}

int update_d_blocks(int n_k) { return (n_k + kUpdRows - 1) / kUpdRows; }

void launch_update_d(int K, int rule, hipStream_t st, float *D, const NmfWork &w, int n_wg, int n_k, int iter,
                     bool has_obj, double f_ref, double tol, bool next_chol, int64_t ldb_img, int bf16,
                     const double *bias, bool extrap) {
  const int nb = update_d_blocks(n_k);
  uint16_t *img = ldb_img > 0 ? w.img : nullptr;
  switch (K) {
#define HSN_K(KK) \
  case KK: reduce_gv_kernel<KK><<<1, kUpdThreads, 0, st>>>(w.part_gv, w.part_obj, n_wg, has_obj, w.ctrl, iter); break;
    HSN_K(1) HSN_K(2) HSN_K(3) HSN_K(4) HSN_K(5) HSN_K(6) HSN_K(7) HSN_K(8)
#undef HSN_K
  }
  const bool ex = extrap && rule == kModeNV && has_obj && w.dprev;
  if (ex) anls_beta_kernel<<<1, 1, 0, st>>>(w.ctrl, iter, K * K, f_ref, tol, bf16, bias);
  switch (K) {
#define HSN_K(KK)                                                                                                 \
  case KK:                                                                                                        \
    if (rule == kModeMU)                                                                                          \
      update_d_kernel<KK, kModeMU><<<nb, kUpdThreads, 0, st>>>(D, w.part_nd, n_wg, n_k,                            \
                                                               w.ctrl, iter, has_obj, f_ref, tol, w.hist, w.gd,   \
                                                               w.chol, next_chol, w.part_gd, img, ldb_img, bf16, bias, w.part_gd16, \
                                                               ex ? w.dprev : nullptr); \
    else if (rule == kModeHALS)                                                                                   \
      update_d_kernel<KK, kModeHALS><<<nb, kUpdThreads, 0, st>>>(D, w.part_nd, n_wg, n_k,                          \
                                                                 w.ctrl, iter, has_obj, f_ref, tol, w.hist, w.gd, \
                                                                 w.chol, next_chol, w.part_gd, img, ldb_img, bf16, bias, w.part_gd16, \
                                                               ex ? w.dprev : nullptr); \
    else                                                                                                          \
      update_d_kernel<KK, kModeNV><<<nb, kUpdThreads, 0, st>>>(D, w.part_nd, n_wg, n_k,                            \
                                                               w.ctrl, iter, has_obj, f_ref, tol, w.hist, w.gd,   \
                                                               w.chol, next_chol, w.part_gd, img, ldb_img, bf16, bias, w.part_gd16, \
                                                               ex ? w.dprev : nullptr); \
    break;
    HSN_K(1) HSN_K(2) HSN_K(3) HSN_K(4) HSN_K(5) HSN_K(6) HSN_K(7) HSN_K(8)
#undef HSN_K
  }
  switch (K) {
#define HSN_K(KK)                                                                                                  \
  case KK:                                                                                                         \
    finish_gd_kernel<KK><<<1, kUpdThreads, 0, st>>>(w.part_gd, nb, w.gd, w.chol, next_chol, w.ctrl, iter, w.ginv, \
                                                    w.part_gd16, w.ginv16);                                            \
    break;
    HSN_K(1) HSN_K(2) HSN_K(3) HSN_K(4) HSN_K(5) HSN_K(6) HSN_K(7) HSN_K(8)
#undef HSN_K
  }
}

void launch_nnls_rows(int K, hipStream_t st, const NmfWork &w, float *V, int64_t n_p, int n_blocks, int iter) {
  switch (K) {
#define HSN_K(KK) \
  case KK: nnls_rows_kernel<KK><<<n_blocks, 256, 0, st>>>(w.nv, w.gd, w.chol, V, n_p, w.ctrl, iter); break;
    HSN_K(1) HSN_K(2) HSN_K(3) HSN_K(4) HSN_K(5) HSN_K(6) HSN_K(7) HSN_K(8)
#undef HSN_K
  }
}

size_t batched_update_lds(int max_k, int rule) {
  switch (max_k) {
#define HSN_K(KK) \
  case KK: return rule == kModeNV ? UpdLds<KK, kModeNV>::bytes : UpdLds<KK, kModeMU>::bytes;
    HSN_K(1) HSN_K(2) HSN_K(3) HSN_K(4) HSN_K(5) HSN_K(6) HSN_K(7)
#undef HSN_K
    default: return rule == kModeNV ? UpdLds<8, kModeNV>::bytes : UpdLds<8, kModeMU>::bytes;
  }
}

hipError_t batched_kernel_setup(size_t pass_lds, size_t upd_lds) {
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(&batched_update_kernel<kModeMU>),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, int(upd_lds));
  if (e == hipSuccess)
    e = hipFuncSetAttribute(reinterpret_cast<const void *>(&batched_update_kernel<kModeNV>),
                            hipFuncAttributeMaxDynamicSharedMemorySize, int(upd_lds));
  (void)pass_lds;
  return e;
}

void launch_batched_init(int n_inst, int want_chol, hipStream_t st, const BatchInst *d) {
  batched_init_kernel<<<n_inst, kUpdThreads, 0, st>>>(d, want_chol);
}

void launch_batched_update(int rule, int n_blocks, size_t lds, hipStream_t st, const BatchInst *d, int n_inst,
                           int iter_local, bool has_obj, bool next_chol, bool bf16) {
  batched_reduce_gv_kernel<<<n_inst, kUpdThreads, 0, st>>>(d, iter_local, has_obj, bf16 ? 1 : 0);
  if (rule == kModeNV)
    batched_update_kernel<kModeNV><<<n_blocks, kUpdThreads, lds, st>>>(d, n_inst, iter_local, has_obj, next_chol,
                                                                        bf16 ? 1 : 0);
  else
    batched_update_kernel<kModeMU><<<n_blocks, kUpdThreads, lds, st>>>(d, n_inst, iter_local, has_obj, next_chol,
                                                                        bf16 ? 1 : 0);
  batched_finish_gd_kernel<<<n_inst, kUpdThreads, 0, st>>>(d, iter_local, next_chol);
}

// Over the instances d[0 .. n_inst) of one K group (rb0 counted from the group's first instance).
void launch_batched_rows(int K, int n_blocks, hipStream_t st, const BatchInst *d, int n_inst, int iter_local) {
  switch (K) {
#define HSN_K(KK) \
  case KK: batched_rows_kernel<KK><<<n_blocks, 256, 0, st>>>(d, n_inst, iter_local); break;
    HSN_K(1) HSN_K(2) HSN_K(3) HSN_K(4) HSN_K(5) HSN_K(6) HSN_K(7) HSN_K(8)
#undef HSN_K
  }
}

// Re-opens a decomposition whose stop test fired (stop_at back to "never"):
// the driver's switch from the bfloat16 polish rounds to the float32 ones.
__global__ void nmf_resume_kernel(NmfCtrl *__restrict__ ctrl) { ctrl->stop_at = INT_MAX; }

void launch_nmf_resume(hipStream_t st, NmfCtrl *ctrl) { nmf_resume_kernel<<<1, 1, 0, st>>>(ctrl); }



// After a float32 round that confirms a stop of the bfloat16 rounds: the
// calibration that makes the estimate of the last bfloat16 objective equal
// to the float32 objective just measured (the last history entry).  That
// round is one round further on, so the calibrated estimate errs low by one
// round's decrease (adding the last bfloat16 round's decrease instead was
// measured to err high: 28 rounds to the tolerance at the full size against
// 22).
__global__ void nmf_calibrate_kernel(NmfCtrl *__restrict__ ctrl, const double *__restrict__ hist,
                                     const double *__restrict__ bias) {
  const int h = ctrl->hist_len;
  if (h > 0) ctrl->adj = hist[h - 1] - (ctrl->last16 + (bias ? *bias : 0.0));
}

void launch_nmf_calibrate(hipStream_t st, NmfCtrl *ctrl, const double *hist, const double *bias) {
  nmf_calibrate_kernel<<<1, 1, 0, st>>>(ctrl, hist, bias);
}

void launch_batched_advance(int n_inst, int steps, hipStream_t st, const BatchInst *d) {
  batched_advance_kernel<<<(n_inst + 63) / 64, 64, 0, st>>>(d, n_inst, steps);
}

}  // namespace hsn
