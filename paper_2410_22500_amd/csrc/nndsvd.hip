// NNDSVD cold start of the NMF (eq. 4), 'a' variant (Boutsidis & Gallopoulos,
// the initialisation the paper names), all on the GPU:
//
//   1. G = P^T P (N_k x N_k) on MFMA from a bfloat16 view of p (16x16x32
//      bf16, float32 accumulation), split over row ranges, the split partials
//      summed in a fixed order in float64;
//   2. the K leading eigenpairs (sigma_j^2, v_j) of G by float64 subspace
//      iteration (L = K + 4 columns, Cholesky-QR each step) and a final
//      Rayleigh-Ritz step solved by cyclic Jacobi;
//   3. u_j = P v_j / sigma_j by the float32 N_V pass of the NMF;
//   4. per pair j >= 2 the positive or negative parts with the larger product
//      of norms (ties: positive), scaled by sqrt(sigma_j m); exact zeros are
//      replaced by mean(p).
// The Gram's bfloat16 inputs make the start accurate to ~1e-3 relative, which
// is all an initial point needs; every later step is exact.
#include "nmf_common.hpp"

#include <climits>
#include <vector>

namespace hsn {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kGT = 128;     // output tile of the Gram
constexpr int kGR = 32;      // rows per contraction step

// Partial Gram of rows [r0, r1) for output tile (bi, bj), bi <= bj.  p is
// either bfloat16 bits (ldb pitch) or float32 (rounded to bfloat16 here).
template <bool F32>
__global__ __launch_bounds__(256) void gram_tile_kernel(const void *__restrict__ pv, int64_t ld, int64_t n_p, int n_k,
                                                        int n_tb, int n_split, float *__restrict__ part) {
  // blockIdx.x -> (bi, bj) with bi <= bj over n_tb tiles; blockIdx.y -> row split
  int pair = blockIdx.x, bi = 0;
  while (pair >= n_tb - bi) {
    pair -= n_tb - bi;
    ++bi;
  }
  const int bj = bi + pair;
  const int64_t r_begin = (n_p * blockIdx.y) / n_split, r_end = (n_p * (blockIdx.y + 1)) / n_split;
  __shared__ __attribute__((aligned(16))) uint16_t At[kGT][kGR + 8];  // transposed tiles, padded rows
  __shared__ __attribute__((aligned(16))) uint16_t Bt[kGT][kGR + 8];
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int wm = (w >> 1) * 64, wn = (w & 1) * 64;
  f32x4 acc[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[a][b] = f32x4{0.f, 0.f, 0.f, 0.f};

  for (int64_t r0 = r_begin; r0 < r_end; r0 += kGR) {
    // 32 rows x 128 columns of each tile: 512 chunks of 8 columns, 2 per thread
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int c = t + 256 * h;
      const int rr = c >> 4, cc = (c & 15) * 8;
      const int64_t row = r0 + rr;
#pragma unroll
      for (int side = 0; side < 2; ++side) {
        const int col0 = (side == 0 ? bi : bj) * kGT + cc;
        uint16_t v[8];
#pragma unroll
        for (int e = 0; e < 8; ++e) {
          const int col = col0 + e;
          uint16_t b = 0;
          if (row < r_end && col < n_k) {
            if (F32)
              b = f32_to_bf16_bits(static_cast<const float *>(pv)[row * ld + col]);
            else
              b = static_cast<const uint16_t *>(pv)[row * ld + col];
          }
          v[e] = b;
        }
        uint16_t(*T)[kGR + 8] = side == 0 ? At : Bt;
#pragma unroll
        for (int e = 0; e < 8; ++e) T[cc + e][rr] = v[e];
      }
    }
    __syncthreads();
#pragma unroll
    for (int a = 0; a < 4; ++a) {
      const uint4 av = *reinterpret_cast<const uint4 *>(&At[wm + 16 * a + (lane & 15)][8 * (lane >> 4)]);
#pragma unroll
      for (int b = 0; b < 4; ++b) {
        const uint4 bv = *reinterpret_cast<const uint4 *>(&Bt[wn + 16 * b + (lane & 15)][8 * (lane >> 4)]);
        acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, av),
                                                            __builtin_bit_cast(bf16x8, bv), acc[a][b], 0, 0, 0);
      }
    }
    __syncthreads();
  }
  // part[split][bi*128 + m][bj*128 + n] (only tiles with bi <= bj are written)
  const int64_t npad = int64_t(n_tb) * kGT;
  float *dst = part + size_t(blockIdx.y) * npad * npad;
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int64_t m = int64_t(bi) * kGT + wm + 16 * a + 4 * (lane >> 4) + q;
        const int64_t nn = int64_t(bj) * kGT + wn + 16 * b + (lane & 15);
        dst[m * npad + nn] = acc[a][b][q];
      }
}

// G[m][n] (float64, full symmetric N_k x N_k) = sum over splits, fixed order.
__global__ void gram_sum_kernel(const float *__restrict__ part, int n_split, int n_tb, int n_k,
                                double *__restrict__ G) {
  const int64_t npad = int64_t(n_tb) * kGT;
  const int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (e >= int64_t(n_k) * n_k) return;
  int64_t m = e / n_k, n = e % n_k;
  if ((m / kGT) > (n / kGT)) {  // lower tiles were not computed: use the mirror
    const int64_t tmp = m;
    m = n;
    n = tmp;
  }
  double s = 0.0;
  for (int sp = 0; sp < n_split; ++sp) s += double(part[size_t(sp) * npad * npad + m * npad + n]);
  G[e] = s;
}

constexpr int kL = 12;              // subspace width (>= K + 4)
constexpr int kSubspaceIters = 40;  // convergence ~ (lambda_{L+1} / lambda_K)^iters

// Z = G Q, Q and Z [n_k][L] float64.
__global__ void gq_kernel(const double *__restrict__ G, const double *__restrict__ Q, int n_k, int L,
                          double *__restrict__ Z) {
  const int row = blockIdx.x;
  const int t = threadIdx.x;
  __shared__ double red[4][kL];
  double acc[kL];
#pragma unroll
  for (int l = 0; l < kL; ++l) acc[l] = 0.0;
  for (int k = t; k < n_k; k += 256) {
    const double g = G[size_t(row) * n_k + k];
#pragma unroll
    for (int l = 0; l < kL; ++l)
      if (l < L) acc[l] += g * Q[size_t(k) * L + l];
  }
#pragma unroll
  for (int l = 0; l < kL; ++l) {
    const double s = wave_sum_all(acc[l]);
    if ((t & 63) == 0) red[t >> 6][l] = s;
  }
  __syncthreads();
  if (t < L) Z[size_t(row) * L + t] = red[0][t] + red[1][t] + red[2][t] + red[3][t];
}

// Q = Z R^{-1} with R^T R = Z^T Z (Cholesky-QR), one workgroup.
__global__ __launch_bounds__(1024) void cholqr_kernel(const double *__restrict__ Z, int n_k, int L,
                                                      double *__restrict__ Q) {
  __shared__ double R[kL][kL];
  __shared__ double red[1024];
  __shared__ int pi[kL * (kL + 1) / 2], pj[kL * (kL + 1) / 2];
  const int t = threadIdx.x;
  const int E = L * (L + 1) / 2;
  const int G = 1024 / E;
  if (t == 0) {
    int q = 0;
    for (int i = 0; i < L; ++i)
      for (int j = i; j < L; ++j, ++q) {
        pi[q] = i;
        pj[q] = j;
      }
  }
  __syncthreads();
  if (t < G * E) {
    const int e = t % E, g = t / E;
    const int i = pi[e], j = pj[e];
    red[g * E + e] = strided_sum(g, G, n_k, [&](int k) { return Z[size_t(k) * L + i] * Z[size_t(k) * L + j]; });
  }
  __syncthreads();
  if (t == 0) {
    double S[kL][kL];
    for (int e = 0; e < E; ++e) {
      double s = 0.0;
      for (int g = 0; g < G; ++g) s += red[g * E + e];
      S[pi[e]][pj[e]] = s;
      S[pj[e]][pi[e]] = s;
    }
    // Cholesky S = R^T R (R upper); a vanishing pivot is clamped (rank loss)
    for (int i = 0; i < L; ++i)
      for (int j = 0; j < L; ++j) R[i][j] = 0.0;
    for (int j = 0; j < L; ++j) {
      double d = S[j][j];
      for (int k = 0; k < j; ++k) d -= R[k][j] * R[k][j];
      R[j][j] = sqrt(fmax(d, 1e-300 + 1e-14 * S[j][j]));
      for (int i = j + 1; i < L; ++i) {
        double v = S[j][i];
        for (int k = 0; k < j; ++k) v -= R[k][j] * R[k][i];
        R[j][i] = v / R[j][j];
      }
    }
  }
  __syncthreads();
  for (int k = t; k < n_k; k += 1024) {
    double z[kL], q[kL];
    for (int l = 0; l < L; ++l) z[l] = Z[size_t(k) * L + l];
    // q R = z (row vector), forward substitution over columns
    for (int j = 0; j < L; ++j) {
      double v = z[j];
      for (int i = 0; i < j; ++i) v -= q[i] * R[i][j];
      q[j] = v / R[j][j];
    }
    for (int l = 0; l < L; ++l) Q[size_t(k) * L + l] = q[l];
  }
}

// Rayleigh-Ritz: H = Q^T Z (Z = G Q), cyclic Jacobi eigen-decomposition of H,
// the K leading Ritz pairs: sigma_j = sqrt(lambda_j), vK[k][j] = (Q y_j)[k] / sigma_j
// (the right singular vector scaled for u_j = P vK_j), vs[k][j] = (Q y_j)[k].
__global__ __launch_bounds__(1024) void ritz_kernel(const double *__restrict__ Q, const double *__restrict__ Z,
                                                    int n_k, int L, int K, double *__restrict__ sigma,
                                                    float *__restrict__ vK, double *__restrict__ vs) {
  __shared__ double H[kL][kL];
  __shared__ double Y[kL][kL];
  __shared__ double red[1024];
  __shared__ int order[kL];
  const int t = threadIdx.x;
  const int E = L * L;
  const int G = 1024 / E;
  if (t < G * E) {
    const int e = t % E, g = t / E;
    const int i = e / L, j = e % L;
    red[g * E + e] = strided_sum(g, G, n_k, [&](int k) { return Q[size_t(k) * L + i] * Z[size_t(k) * L + j]; });
  }
  __syncthreads();
  if (t == 0) {
    for (int i = 0; i < L; ++i)
      for (int j = 0; j < L; ++j) {
        double s = 0.0, s2 = 0.0;
        for (int g = 0; g < G; ++g) {
          s += red[g * E + i * L + j];
          s2 += red[g * E + j * L + i];
        }
        H[i][j] = 0.5 * (s + s2);  // symmetrise
        Y[i][j] = (i == j) ? 1.0 : 0.0;
      }
    for (int sweep = 0; sweep < 60; ++sweep) {
      double off = 0.0, tot = 0.0;
      for (int i = 0; i < L; ++i)
        for (int j = 0; j < L; ++j) {
          tot += H[i][j] * H[i][j];
          if (i != j) off += H[i][j] * H[i][j];
        }
      if (off <= 1e-30 * tot) break;
      for (int p = 0; p < L - 1; ++p)
        for (int q = p + 1; q < L; ++q) {
          if (H[p][q] == 0.0) continue;
          const double th = (H[q][q] - H[p][p]) / (2.0 * H[p][q]);
          const double tt = (th >= 0 ? 1.0 : -1.0) / (fabs(th) + sqrt(th * th + 1.0));
          const double c = 1.0 / sqrt(tt * tt + 1.0), s = tt * c;
          for (int k = 0; k < L; ++k) {
            const double hkp = H[k][p], hkq = H[k][q];
            H[k][p] = c * hkp - s * hkq;
            H[k][q] = s * hkp + c * hkq;
          }
          for (int k = 0; k < L; ++k) {
            const double hpk = H[p][k], hqk = H[q][k];
            H[p][k] = c * hpk - s * hqk;
            H[q][k] = s * hpk + c * hqk;
          }
          for (int k = 0; k < L; ++k) {
            const double ykp = Y[k][p], ykq = Y[k][q];
            Y[k][p] = c * ykp - s * ykq;
            Y[k][q] = s * ykp + c * ykq;
          }
        }
    }
    // order by descending eigenvalue
    for (int i = 0; i < L; ++i) order[i] = i;
    for (int i = 0; i < L; ++i)
      for (int j = i + 1; j < L; ++j)
        if (H[order[j]][order[j]] > H[order[i]][order[i]]) {
          const int tmp = order[i];
          order[i] = order[j];
          order[j] = tmp;
        }
    for (int j = 0; j < K; ++j) sigma[j] = sqrt(fmax(H[order[j]][order[j]], 0.0));
  }
  __syncthreads();
  for (int k = t; k < n_k; k += 1024) {
    double a[kL];
    for (int l = 0; l < L; ++l) a[l] = Q[size_t(k) * L + l];
    for (int j = 0; j < K; ++j) {
      double v = 0.0;
      for (int l = 0; l < L; ++l) v += a[l] * Y[l][order[j]];
      vs[size_t(k) * K + j] = v;
      vK[size_t(k) * K + j] = float(sigma[j] > 0.0 ? v / sigma[j] : 0.0);
    }
  }
}

// Column sums of squares of the positive and negative parts of X [n][K]
// (float32 or float64), plus the sum of the row sums of p when given: per
// block partials, summed in a fixed order by nndsvd_finish.
template <typename T>
__global__ void split_norms_kernel(const T *__restrict__ X, int64_t n, int K, double *__restrict__ part) {
  double acc[16];
  for (int i = 0; i < 16; ++i) acc[i] = 0.0;
  for (int64_t r = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; r < n; r += int64_t(gridDim.x) * blockDim.x)
    for (int j = 0; j < K; ++j) {
      const double x = double(X[r * K + j]);
      if (x > 0) acc[j] += x * x;
      else acc[8 + j] += x * x;
    }
  __shared__ double red[4][16];
  for (int i = 0; i < 16; ++i) {
    const double s = wave_sum_all(acc[i]);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6][i] = s;
  }
  __syncthreads();
  if (threadIdx.x < 16)
    part[size_t(blockIdx.x) * 16 + threadIdx.x] =
        red[0][threadIdx.x] + red[1][threadIdx.x] + red[2][threadIdx.x] + red[3][threadIdx.x];
}

// sum of p (for mean(p)) over rows, per-block partials
__global__ void psum_kernel(const float *__restrict__ p, int64_t ldp, int64_t n_p, int n_k, double *__restrict__ part) {
  double acc = 0.0;
  for (int64_t r = blockIdx.x; r < n_p; r += gridDim.x)
    for (int k = threadIdx.x; k < n_k; k += 256) acc += p[r * ldp + k];
  __shared__ double red[4];
  acc = wave_sum_all(acc);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) part[blockIdx.x] = red[0] + red[1] + red[2] + red[3];
}

// coef[j]: scale and sign for column j; info layout: [0..K) scale_u, [K..2K) scale_v,
// [2K..3K) sign (+1 positive part, -1 negative part), [3K] mean(p).
__global__ void nndsvd_coef_kernel(const double *__restrict__ part_u, int nbu, const double *__restrict__ part_v,
                                   int nbv, const double *__restrict__ part_p, int nbp, double n_elems,
                                   const double *__restrict__ sigma, int K, double *__restrict__ info) {
  if (threadIdx.x != 0) return;
  double su[16] = {}, sv[16] = {};
  for (int b = 0; b < nbu; ++b)
    for (int i = 0; i < 16; ++i) su[i] += part_u[size_t(b) * 16 + i];
  for (int b = 0; b < nbv; ++b)
    for (int i = 0; i < 16; ++i) sv[i] += part_v[size_t(b) * 16 + i];
  double ps = 0.0;
  for (int b = 0; b < nbp; ++b) ps += part_p[b];
  for (int j = 0; j < K; ++j) {
    const double up = sqrt(su[j]), un = sqrt(su[8 + j]), vp = sqrt(sv[j]), vn = sqrt(sv[8 + j]);
    double sgn, nu, nv, m;
    if (j == 0) {
      // first pair: |u_1|, |v_1| with unit norms
      sgn = 0.0;
      nu = sqrt(su[j] + su[8 + j]);
      nv = sqrt(sv[j] + sv[8 + j]);
      m = 1.0;
    } else if (up * vp >= un * vn) {
      sgn = 1.0;
      nu = up;
      nv = vp;
      m = up * vp;
    } else {
      sgn = -1.0;
      nu = un;
      nv = vn;
      m = un * vn;
    }
    const double c = sqrt(sigma[j] * m);
    info[j] = (nu > 0.0) ? c / nu : 0.0;
    info[K + j] = (nv > 0.0) ? c / nv : 0.0;
    info[2 * K + j] = sgn;
  }
  info[3 * K] = ps / n_elems;
}

// X[r][j] <- scale_j * part_j(X[r][j]) with part = |x| (j = 0), max(x,0)
// (sign +1) or max(-x,0) (sign -1); with fill, exact zeros become mean(p)
// (NNDSVDa), else they stay (plain NNDSVD).
template <typename T>
__global__ void nndsvd_apply_kernel(const T *__restrict__ X, int64_t n, int K, const double *__restrict__ info,
                                    int which, int fill, float *__restrict__ out) {
  for (int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; e < n * K; e += int64_t(gridDim.x) * blockDim.x) {
    const int j = int(e % K);
    const double x = double(X[e]);
    const double sg = info[2 * K + j];
    const double part = (sg == 0.0) ? fabs(x) : (sg > 0.0 ? fmax(x, 0.0) : fmax(-x, 0.0));
    const double v = info[which * K + j] * part;
    out[e] = (v == 0.0 && fill) ? float(info[3 * K]) : float(v);
  }
}

__global__ void ctrl_open_kernel(NmfCtrl *c) {
  c->stop_at = INT_MAX;
  c->upd_ticket = 0;
  c->hist_len = 0;
}

// Deterministic start block of the subspace iteration: a fixed +-1 pattern
// from an integer hash of (k, l).
__global__ void qinit_kernel(double *__restrict__ Q, int n_k, int L) {
  const int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (e >= int64_t(n_k) * L) return;
  uint32_t h = uint32_t(e) * 2654435761u;
  h ^= h >> 15;
  h *= 2246822519u;
  h ^= h >> 13;
  Q[e] = (h & 1u) ? 1.0 : -1.0;
}

void launch_pass_f32(int K, int mode, bool obj, int nq, int n_wg, hipStream_t st, const float *P, int64_t ldp,
                     int64_t n_p, int n_k, float *V, float *NV, const float *D, const double *GD, const double *chol,
                     float *part_nd, double *part_gv, double *part_obj, NmfCtrl *ctrl, int iter,
                     const double *ginv);

size_t nndsvd_ws_bytes(int64_t n_p, int n_k, int K, int n_split) {
  const int n_tb = (n_k + kGT - 1) / kGT;
  const size_t npad = size_t(n_tb) * kGT;
  return Carver::need({sizeof(float) * n_split * npad * npad, sizeof(double) * size_t(n_k) * n_k,
                       3 * sizeof(double) * size_t(n_k) * kL, sizeof(double) * 16, sizeof(float) * size_t(n_k) * K,
                       sizeof(double) * size_t(n_k) * K, sizeof(float) * size_t(n_p) * K, sizeof(double) * 1024 * 16,
                       sizeof(double) * 1024 * 16, sizeof(double) * 1024, sizeof(double) * 64, sizeof(NmfCtrl)});
}

// Writes V0 [n_p][K] and D0 [n_k][K].  ws: nndsvd_ws_bytes of device memory.
hsn_status nndsvd_init(hsn_ctx *ctx, hipStream_t st, const float *p, int64_t ldp, const uint16_t *pb, int64_t ldb,
                       int64_t n_p, int n_k, int K, float *V, float *D, void *ws, int n_split, bool fill) {
  const int n_tb = (n_k + kGT - 1) / kGT;
  const size_t npad = size_t(n_tb) * kGT;
  const int L = std::min(kL, n_k);
  if (K > L) return fail(ctx, HSN_ERR_SHAPE, "nndsvd: k exceeds the number of bins");
  Carver cv(ws);
  float *part = cv.take<float>(n_split * npad * npad);
  double *G = cv.take<double>(size_t(n_k) * n_k);
  double *Q = cv.take<double>(size_t(n_k) * kL);
  double *Z = cv.take<double>(size_t(n_k) * kL);
  double *Z2 = cv.take<double>(size_t(n_k) * kL);
  double *sigma = cv.take<double>(16);
  float *vK = cv.take<float>(size_t(n_k) * K);
  double *vs = cv.take<double>(size_t(n_k) * K);
  float *U = cv.take<float>(size_t(n_p) * K);
  double *part_u = cv.take<double>(1024 * 16);
  double *part_v = cv.take<double>(1024 * 16);
  double *part_p = cv.take<double>(1024);
  double *info = cv.take<double>(64);
  NmfCtrl *ctrl = cv.take<NmfCtrl>(1);

  const dim3 g1(unsigned(n_tb * (n_tb + 1) / 2), unsigned(n_split));
  prof_begin(ctx, HSN_KERN_NNDSVD_GRAM, st);
  if (pb)
    gram_tile_kernel<false><<<g1, 256, 0, st>>>(pb, ldb, n_p, n_k, n_tb, n_split, part);
  else
    gram_tile_kernel<true><<<g1, 256, 0, st>>>(p, ldp, n_p, n_k, n_tb, n_split, part);
  prof_end(ctx, HSN_KERN_NNDSVD_GRAM, st);
  gram_sum_kernel<<<unsigned((int64_t(n_k) * n_k + 255) / 256), 256, 0, st>>>(part, n_split, n_tb, n_k, G);
  qinit_kernel<<<unsigned((n_k * L + 255) / 256), 256, 0, st>>>(Q, n_k, L);
  for (int it = 0; it < kSubspaceIters; ++it) {
    gq_kernel<<<n_k, 256, 0, st>>>(G, Q, n_k, L, Z);
    cholqr_kernel<<<1, 1024, 0, st>>>(Z, n_k, L, Q);
  }
  gq_kernel<<<n_k, 256, 0, st>>>(G, Q, n_k, L, Z2);
  ritz_kernel<<<1, 1024, 0, st>>>(Q, Z2, n_k, L, K, sigma, vK, vs);
  // u_j = P v_j / sigma_j with the N_V pass (control block: never stopped)
  ctrl_open_kernel<<<1, 1, 0, st>>>(ctrl);
  const int64_t n_tiles = (n_p + 7) / 8;
  const int wg = int(std::min<int64_t>(n_tiles, 2 * int64_t(ctx->num_cu)));
  launch_pass_f32(K, kModeNV, false, n_k > 1024 ? 2 : 1, wg, st, p, ldp, n_p, n_k, nullptr, U, vK, nullptr, nullptr,
                  nullptr, nullptr, nullptr, ctrl, 0, nullptr);
  const int nbu = 1024, nbv = 64, nbp = 1024;
  split_norms_kernel<float><<<nbu, 256, 0, st>>>(U, n_p, K, part_u);
  split_norms_kernel<double><<<nbv, 256, 0, st>>>(vs, n_k, K, part_v);
  psum_kernel<<<nbp, 256, 0, st>>>(p, ldp, n_p, n_k, part_p);
  nndsvd_coef_kernel<<<1, 64, 0, st>>>(part_u, nbu, part_v, nbv, part_p, nbp, double(n_p) * n_k, sigma, K, info);
  nndsvd_apply_kernel<float><<<2048, 256, 0, st>>>(U, n_p, K, info, 0, fill ? 1 : 0, V);
  nndsvd_apply_kernel<double><<<64, 256, 0, st>>>(vs, n_k, K, info, 1, fill ? 1 : 0, D);
  HSN_LAUNCHED(ctx);
  return HSN_OK;
}

}  // namespace hsn
