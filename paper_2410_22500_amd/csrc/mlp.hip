// Learned warm start of the NMF of eq. (4): a 256-128-128-K perceptron that
// maps a ray's pooled spectrum to its K coefficients (a row of V).  The
// paper starts from NNDSVD and has no learned component; the network, loss
// and optimiser are this library's, trained on decompositions the NMF itself
// produces.
//
// Kernels, templated on T = bfloat16 bits (uint16_t, MFMA 16x16x32 bf16) or
// float (MFMA 16x16x4 f32), the network's precision, always with float32
// accumulation:
//   pool    average pooling of bfloat16 p rows to 256 bins, one wave per row
//   rows    per 64-row tile (16 rows per wave): the three layers, activations
//           staged through LDS between layers; for training also the loss,
//           dL/dz3 and the row-local backward pass down to dL/dz1; writes
//           h1, h2, dz1, dz2, dz3 and per-block bias-gradient / loss partials
//   wgrad   dW = A^T dZ (A = x, h1, h2), contraction over the batch rows:
//           64x64 output tiles x row splits, LDS-transposed operands
//   update  sums the partials in a fixed order (so training is deterministic)
//           and stores the gradient, or applies Adam and republishes the
//           transposed compute copies of the weights
#include "nmf_common.hpp"

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <numeric>
#include <random>
#include <type_traits>
#include <vector>

namespace hsn {

void launch_pass_f32(int K, int mode, bool obj, int nq, int n_wg, hipStream_t st, const float *P, int64_t ldp,
                     int64_t n_p, int n_k, float *V, float *NV, const float *D, const double *GD, const double *chol,
                     float *part_nd, double *part_gv, double *part_obj, NmfCtrl *ctrl, int iter,
                     const double *ginv);
void launch_update_d(int K, int rule, hipStream_t st, float *D, const NmfWork &w, int n_wg, int n_k, int iter,
                     bool has_obj, double f_ref, double tol, bool next_chol, int64_t ldb_img, int bf16 = 0,
                     const double *bias = nullptr, bool extrap = false);
bool launch_pass_bf16(int K, int mode, bool obj, int n_wg, hipStream_t st, const uint16_t *Pb, int64_t ldb,
                      int64_t n_p, int n_k, float *V, const double *GD, const double *chol, const uint16_t *img,
                      float *part_nd, double *part_gv, double *part_obj, NmfCtrl *ctrl, int iter,
                      const double *ginv);

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kIn = HSN_MLP_IN, kHid = HSN_MLP_HIDDEN;
constexpr int kOutPad = 16;                  // output layer padded to one MFMA tile
constexpr int kWaves = 4, kRowsW = 16, kRowsB = kWaves * kRowsW;
constexpr int kBiasCols = 2 * kHid + kOutPad;  // b1 | b2 | b3 partial columns
constexpr int kChunk = 32;                   // rows per contraction step of wgrad
constexpr int kTiles = 14;                   // wgrad output tiles: 8 (W1) + 4 (W2) + 2 (W3)

struct Layout {
  int64_t w1, b1, w2, b2, w3, b3, n;
};
__host__ __device__ inline Layout layout(int k) {
  Layout L;
  L.w1 = 0;
  L.b1 = L.w1 + int64_t(kIn) * kHid;
  L.w2 = L.b1 + kHid;
  L.b2 = L.w2 + int64_t(kHid) * kHid;
  L.w3 = L.b2 + kHid;
  L.b3 = L.w3 + int64_t(kHid) * k;
  L.n = L.b3 + k;
  return L;
}

// Compute copies of the weights ("published" after each update), element T:
//   w1t [128][256] = W1^T   w2t [128][128] = W2^T   w2n [128][128] = W2
//   w3t [16][128]  = W3^T (rows >= K zero)   w3n [128][16] = W3 (cols >= K zero)
constexpr int64_t kPubW1t = 0, kPubW2t = kPubW1t + int64_t(kHid) * kIn, kPubW2n = kPubW2t + kHid * kHid,
                  kPubW3t = kPubW2n + kHid * kHid, kPubW3n = kPubW3t + kOutPad * kHid,
                  kPubElems = kPubW3n + kHid * kOutPad;

template <class T>
struct Mma;
template <>
struct Mma<uint16_t> {
  static constexpr int E = 8;    // consecutive k values per lane
  static constexpr int KS = 32;  // k per instruction
  typedef bf16x8 frag;
  __device__ static frag load(const uint16_t *p) { return __builtin_bit_cast(frag, *reinterpret_cast<const uint4 *>(p)); }
  __device__ static frag zero() { return __builtin_bit_cast(frag, uint4{0u, 0u, 0u, 0u}); }
  __device__ static f32x4 mma(frag a, frag b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
  }
  __host__ __device__ static uint16_t cvt(float x) {
    uint32_t u = __builtin_bit_cast(uint32_t, x);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return static_cast<uint16_t>(u >> 16);
  }
};
template <>
struct Mma<float> {
  static constexpr int E = 1, KS = 4;
  typedef float frag;
  __device__ static frag load(const float *p) { return *p; }
  __device__ static frag zero() { return 0.0f; }
  __device__ static f32x4 mma(frag a, frag b, f32x4 c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }
  __host__ __device__ static float cvt(float x) { return x; }
};

// Copies 16 rows x cols elements from an LDS tile (row pitch lp) to global
// rows [r0, r0+16) of a [.][cols] array, rows >= n skipped; 16-byte chunks.
template <class T, int COLS, int LP>
__device__ inline void tile_to_global(const T (*src)[LP], T *dst, int64_t r0, int64_t n, int lane) {
  constexpr int PER = 16 / sizeof(T);
  constexpr int CH = kRowsW * COLS / PER;
  for (int c = lane; c < CH; c += 64) {
    const int r = c / (COLS / PER), col = (c % (COLS / PER)) * PER;
    if (r0 + r < n)
      *reinterpret_cast<uint4 *>(dst + (r0 + r) * COLS + col) = *reinterpret_cast<const uint4 *>(&src[r][col]);
  }
}

__device__ inline float gelu(float z) { return 0.5f * z * (1.0f + erff(z * 0.70710678118654752f)); }
__device__ inline float gelu_grad(float z) {
  return 0.5f * (1.0f + erff(z * 0.70710678118654752f)) + z * 0.39894228040143268f * expf(-0.5f * z * z);
}
__device__ inline float softplus(float z) { return fmaxf(z, 0.0f) + log1pf(expf(-fabsf(z))); }
__device__ inline float sigmoid(float z) { return 1.0f / (1.0f + expf(-z)); }

// Column sums over a wave's 16 rows of a C-layout tile column (lane & 15):
// the 4 in-lane rows, then the 4 lane groups.
__device__ inline float col_sum16(float s) {
  s += __shfl_xor(s, 16, 64);
  s += __shfl_xor(s, 32, 64);
  return s;
}

struct RowsArgs {
  const void *x;
  int64_t ldx;
  const int32_t *idx;  // optional row permutation: sample of batch row r = idx[row0 + r]
  int64_t row0, n;     // batch = rows [0, n)
  const void *pub;     // published weights
  const float *theta;  // biases are read from the float32 master copy
  float *y;            // inference output [n][ldy]
  int64_t ldy;
  const float *target;  // [.][K] by sample
  float scale;          // dL/dy = scale * (y - t)  (2 / (n K))
  void *h1, *h2, *dz1, *dz2, *dz3;
  float *part_b;
  double *part_loss;
};

template <class T, int K, bool TRAIN>
__global__ __launch_bounds__(256) void mlp_rows_kernel(RowsArgs a) {
  using M = Mma<T>;
  constexpr int E = M::E, KS = M::KS;
  constexpr int LP = kHid + 16 / int(sizeof(T)) * 1;  // row pitch: +16 bytes
  constexpr int DP = kOutPad + 16 / int(sizeof(T));
  __shared__ __attribute__((aligned(16))) T buf[kWaves][2][kRowsW][LP];
  __shared__ __attribute__((aligned(16))) T dzb[kWaves][kRowsW][DP];
  __shared__ float red[kWaves][kBiasCols];
  __shared__ double redl[kWaves];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int lr = lane & 15, lg = lane >> 4;
  const int64_t rbase = int64_t(blockIdx.x) * kRowsB + w * kRowsW;
  const T *pub = static_cast<const T *>(a.pub);
  const T *w1t = pub + kPubW1t, *w2t = pub + kPubW2t, *w2n = pub + kPubW2n, *w3t = pub + kPubW3t,
          *w3n = pub + kPubW3n;
  const Layout L = layout(K);
  const float *b1 = a.theta + L.b1, *b2 = a.theta + L.b2, *b3 = a.theta + L.b3;

  f32x4 acc[8];
  float g1[8][4], g2[8][4];
  // ---- layer 1: z1 = x W1 + b1 (A operand straight from global x)
  {
    const int64_t row = rbase + lr;
    const bool ok = row < a.n;
    const int64_t smp = ok ? (a.idx ? int64_t(a.idx[a.row0 + row]) : a.row0 + row) : 0;
    const T *xr = static_cast<const T *>(a.x) + smp * a.ldx + E * lg;
#pragma unroll
    for (int j = 0; j < 8; ++j) acc[j] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll 2
    for (int s = 0; s < kIn / KS; ++s) {
      const typename M::frag fa = ok ? M::load(xr + s * KS) : M::zero();
#pragma unroll
      for (int j = 0; j < 8; ++j) acc[j] = M::mma(fa, M::load(w1t + (16 * j + lr) * kIn + s * KS + E * lg), acc[j]);
    }
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const float bb = b1[16 * j + lr];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const float z = acc[j][i] + bb;
        if (TRAIN) g1[j][i] = gelu_grad(z);
        buf[w][0][4 * lg + i][16 * j + lr] = M::cvt(gelu(z));
      }
    }
  }
  __syncthreads();
  // ---- layer 2: z2 = h1 W2 + b2
  {
#pragma unroll
    for (int j = 0; j < 8; ++j) acc[j] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll 2
    for (int s = 0; s < kHid / KS; ++s) {
      const typename M::frag fa = M::load(&buf[w][0][lr][s * KS + E * lg]);
#pragma unroll
      for (int j = 0; j < 8; ++j) acc[j] = M::mma(fa, M::load(w2t + (16 * j + lr) * kHid + s * KS + E * lg), acc[j]);
    }
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const float bb = b2[16 * j + lr];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const float z = acc[j][i] + bb;
        if (TRAIN) g2[j][i] = gelu_grad(z);
        buf[w][1][4 * lg + i][16 * j + lr] = M::cvt(gelu(z));
      }
    }
  }
  __syncthreads();
  if (TRAIN) {
    tile_to_global<T, kHid, LP>(buf[w][0], static_cast<T *>(a.h1), rbase, a.n, lane);
    tile_to_global<T, kHid, LP>(buf[w][1], static_cast<T *>(a.h2), rbase, a.n, lane);
  }
  // ---- layer 3: z3 = h2 W3 + b3, y = softplus(z3)
  f32x4 c3 = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll 4
  for (int s = 0; s < kHid / KS; ++s)
    c3 = M::mma(M::load(&buf[w][1][lr][s * KS + E * lg]), M::load(w3t + lr * kHid + s * KS + E * lg), c3);
  const int col = lr;
  const float bb3 = col < K ? b3[col] : 0.0f;
  if (!TRAIN) {
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int64_t row = rbase + 4 * lg + i;
      if (col < K && row < a.n) a.y[(a.row0 + row) * a.ldy + col] = softplus(c3[i] + bb3);
    }
    return;
  }
  // ---- training: loss, dL/dz3
  double lsum = 0.0;
  float bs = 0.0f;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int64_t row = rbase + 4 * lg + i;
    float dz = 0.0f;
    if (col < K && row < a.n) {
      const int64_t smp = a.idx ? int64_t(a.idx[a.row0 + row]) : a.row0 + row;
      const float z = c3[i] + bb3;
      const float d = softplus(z) - a.target[smp * K + col];
      lsum += double(d) * double(d);
      dz = a.scale * d * sigmoid(z);
    }
    bs += dz;
    dzb[w][4 * lg + i][col] = M::cvt(dz);
    if (row < a.n) static_cast<T *>(a.dz3)[row * kOutPad + col] = M::cvt(dz);
  }
  bs = col_sum16(bs);
  if (lg == 0) red[w][2 * kHid + col] = bs;
  __syncthreads();
  // ---- dh2 = dz3 W3^T (contraction over the K <= 16 outputs), dz2 = dh2 * gelu'(z2)
#pragma unroll
  for (int j = 0; j < 8; ++j) acc[j] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int s = 0; s < (kOutPad + KS - 1) / KS; ++s) {
    const int kk = s * KS + E * lg;
    const typename M::frag fa = kk < kOutPad ? M::load(&dzb[w][lr][kk]) : M::zero();
#pragma unroll
    for (int j = 0; j < 8; ++j)
      acc[j] = M::mma(fa, kk < kOutPad ? M::load(w3n + (16 * j + lr) * kOutPad + kk) : M::zero(), acc[j]);
  }
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    float cs = 0.0f;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const float dz = acc[j][i] * g2[j][i];
      cs += dz;
      buf[w][0][4 * lg + i][16 * j + lr] = M::cvt(dz);
    }
    cs = col_sum16(cs);
    if (lg == 0) red[w][kHid + 16 * j + lr] = cs;
  }
  __syncthreads();
  tile_to_global<T, kHid, LP>(buf[w][0], static_cast<T *>(a.dz2), rbase, a.n, lane);
  // ---- dh1 = dz2 W2^T, dz1 = dh1 * gelu'(z1)
#pragma unroll
  for (int j = 0; j < 8; ++j) acc[j] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll 2
  for (int s = 0; s < kHid / KS; ++s) {
    const typename M::frag fa = M::load(&buf[w][0][lr][s * KS + E * lg]);
#pragma unroll
    for (int j = 0; j < 8; ++j) acc[j] = M::mma(fa, M::load(w2n + (16 * j + lr) * kHid + s * KS + E * lg), acc[j]);
  }
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    float cs = 0.0f;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const float dz = acc[j][i] * g1[j][i];
      cs += dz;
      buf[w][1][4 * lg + i][16 * j + lr] = M::cvt(dz);
    }
    cs = col_sum16(cs);
    if (lg == 0) red[w][16 * j + lr] = cs;
  }
  lsum = wave_sum_all(lsum);
  if (lane == 0) redl[w] = lsum;
  __syncthreads();
  tile_to_global<T, kHid, LP>(buf[w][1], static_cast<T *>(a.dz1), rbase, a.n, lane);
  for (int c = threadIdx.x; c < kBiasCols; c += 256) {
    float s = 0.0f;
#pragma unroll
    for (int ww = 0; ww < kWaves; ++ww) s += red[ww][c];
    a.part_b[size_t(blockIdx.x) * kBiasCols + c] = s;
  }
  if (threadIdx.x == 0) a.part_loss[blockIdx.x] = redl[0] + redl[1] + redl[2] + redl[3];
}

// Inference of the bfloat16 network with three 16-row tiles per wave: every
// weight fragment read from L2 feeds three MFMAs (a third of the weight
// traffic of mlp_rows_kernel, which reads all weights for every 16 rows).  Per row the
// arithmetic and the MFMA order are those of mlp_rows_kernel<uint16_t, K,
// false>, so both give the same outputs.  A wave's h1 and then h2 share one
// LDS tile pair (a wave's LDS accesses are performed in order).
constexpr int kTilesW = 3;
constexpr int kRowsB2 = kWaves * kTilesW * kRowsW;

// Three waves per SIMD (at most 168 registers, no spills; 51 KB of LDS per
// workgroup): a CU holds three workgroups.
template <int K>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3))) void mlp_infer2_kernel(RowsArgs a) {
  using T = uint16_t;
  using M = Mma<T>;
  constexpr int E = M::E, KS = M::KS;
  constexpr int LP = kHid + 16 / int(sizeof(T));
  __shared__ __attribute__((aligned(16))) T buf[kWaves][kTilesW][kRowsW][LP];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int lr = lane & 15, lg = lane >> 4;
  const int64_t wbase = int64_t(blockIdx.x) * kRowsB2 + w * (kTilesW * kRowsW);
  const T *pub = static_cast<const T *>(a.pub);
  const T *w1t = pub + kPubW1t, *w2t = pub + kPubW2t, *w3t = pub + kPubW3t;
  const Layout L = layout(K);
  const float *b1 = a.theta + L.b1, *b2 = a.theta + L.b2, *b3 = a.theta + L.b3;

  f32x4 acc[kTilesW][8];
  // ---- layer 1: z1 = x W1 + b1
  {
    const T *xr[kTilesW];
    bool ok[kTilesW];
#pragma unroll
    for (int t = 0; t < kTilesW; ++t) {
      const int64_t row = wbase + 16 * t + lr;
      ok[t] = row < a.n;
      const int64_t smp = ok[t] ? (a.idx ? int64_t(a.idx[a.row0 + row]) : a.row0 + row) : 0;
      xr[t] = static_cast<const T *>(a.x) + smp * a.ldx + E * lg;
#pragma unroll
      for (int j = 0; j < 8; ++j) acc[t][j] = f32x4{0.f, 0.f, 0.f, 0.f};
    }
#pragma unroll 2
    for (int s = 0; s < kIn / KS; ++s) {
      typename M::frag fa[kTilesW];
#pragma unroll
      for (int t = 0; t < kTilesW; ++t) fa[t] = ok[t] ? M::load(xr[t] + s * KS) : M::zero();
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const typename M::frag fb = M::load(w1t + (16 * j + lr) * kIn + s * KS + E * lg);
#pragma unroll
        for (int t = 0; t < kTilesW; ++t) acc[t][j] = M::mma(fa[t], fb, acc[t][j]);
      }
    }
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const float bb = b1[16 * j + lr];
#pragma unroll
      for (int t = 0; t < kTilesW; ++t)
#pragma unroll
        for (int i = 0; i < 4; ++i) buf[w][t][4 * lg + i][16 * j + lr] = M::cvt(gelu(acc[t][j][i] + bb));
    }
  }
  __syncthreads();
  // ---- layer 2: z2 = h1 W2 + b2
  {
#pragma unroll
    for (int t = 0; t < kTilesW; ++t)
#pragma unroll
      for (int j = 0; j < 8; ++j) acc[t][j] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll 2
    for (int s = 0; s < kHid / KS; ++s) {
      typename M::frag fa[kTilesW];
#pragma unroll
      for (int t = 0; t < kTilesW; ++t) fa[t] = M::load(&buf[w][t][lr][s * KS + E * lg]);
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const typename M::frag fb = M::load(w2t + (16 * j + lr) * kHid + s * KS + E * lg);
#pragma unroll
        for (int t = 0; t < kTilesW; ++t) acc[t][j] = M::mma(fa[t], fb, acc[t][j]);
      }
    }
    __syncthreads();  // every h1 read is done before h2 overwrites the tiles
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const float bb = b2[16 * j + lr];
#pragma unroll
      for (int t = 0; t < kTilesW; ++t)
#pragma unroll
        for (int i = 0; i < 4; ++i) buf[w][t][4 * lg + i][16 * j + lr] = M::cvt(gelu(acc[t][j][i] + bb));
    }
  }
  __syncthreads();
  // ---- layer 3: z3 = h2 W3 + b3, y = softplus(z3)
  f32x4 c3[kTilesW];
#pragma unroll
  for (int t = 0; t < kTilesW; ++t) c3[t] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll 4
  for (int s = 0; s < kHid / KS; ++s) {
    const typename M::frag fb = M::load(w3t + lr * kHid + s * KS + E * lg);
#pragma unroll
    for (int t = 0; t < kTilesW; ++t) c3[t] = M::mma(M::load(&buf[w][t][lr][s * KS + E * lg]), fb, c3[t]);
  }
  const int col = lr;
  const float bb3 = col < K ? b3[col] : 0.0f;
#pragma unroll
  for (int t = 0; t < kTilesW; ++t)
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int64_t row = wbase + 16 * t + 4 * lg + i;
      if (col < K && row < a.n) a.y[(a.row0 + row) * a.ldy + col] = softplus(c3[t][i] + bb3);
    }
}

struct WgradArgs {
  const void *x;
  int64_t ldx;
  const int32_t *idx;
  int64_t row0, n;
  const void *h1, *h2, *dz1, *dz2, *dz3;
  float *part_w;  // [n_split][n_params]
  int64_t n_params;
};

// Loads 8 consecutive elements of one row into v (zeros when !ok).
template <class T>
__device__ inline void load8(const T *p, bool ok, T (&v)[8]) {
  if (sizeof(T) == 2) {
    uint4 q = ok ? *reinterpret_cast<const uint4 *>(p) : uint4{0u, 0u, 0u, 0u};
    __builtin_memcpy(v, &q, 16);
  } else {
    uint4 q0 = ok ? *reinterpret_cast<const uint4 *>(p) : uint4{0u, 0u, 0u, 0u};
    uint4 q1 = ok ? *reinterpret_cast<const uint4 *>(p + 4) : uint4{0u, 0u, 0u, 0u};
    __builtin_memcpy(v, &q0, 16);
    __builtin_memcpy(reinterpret_cast<char *>(v) + 16, &q1, 16);
  }
}

template <class T, int K>
__global__ __launch_bounds__(256) void mlp_wgrad_kernel(WgradArgs a) {
  using M = Mma<T>;
  constexpr int E = M::E, KS = M::KS;
  constexpr int TP = kChunk + 16 / int(sizeof(T));
  __shared__ __attribute__((aligned(16))) T At[64][TP];
  __shared__ __attribute__((aligned(16))) T Bt[64][TP];
  const int task = blockIdx.x, split = blockIdx.y, n_split = gridDim.y;
  const Layout L = layout(K);
  // task -> operands and output tile
  const T *A, *B;
  int64_t lda, ldb_, out0, out_ld;
  int mi, ni, bw, nvalid;
  bool gather = false;
  if (task < 8) {
    A = static_cast<const T *>(a.x);
    lda = a.ldx;
    gather = true;
    B = static_cast<const T *>(a.dz1);
    ldb_ = kHid;
    mi = task >> 1;
    ni = task & 1;
    bw = kHid;
    out0 = L.w1;
    out_ld = kHid;
    nvalid = kHid;
  } else if (task < 12) {
    A = static_cast<const T *>(a.h1);
    lda = kHid;
    B = static_cast<const T *>(a.dz2);
    ldb_ = kHid;
    mi = (task - 8) >> 1;
    ni = (task - 8) & 1;
    bw = kHid;
    out0 = L.w2;
    out_ld = kHid;
    nvalid = kHid;
  } else {
    A = static_cast<const T *>(a.h2);
    lda = kHid;
    B = static_cast<const T *>(a.dz3);
    ldb_ = kOutPad;
    mi = task - 12;
    ni = 0;
    bw = kOutPad;
    out0 = L.w3;
    out_ld = K;
    nvalid = K;
  }
  const int64_t r_begin = (a.n * split) / n_split, r_end = (a.n * (split + 1)) / n_split;
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int lr = lane & 15, lg = lane >> 4;
  const int wm = (w >> 1) * 32, wn = (w & 1) * 32;
  f32x4 acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
  const int rr = t >> 3, cc = (t & 7) * 8;
  for (int64_t r0 = r_begin; r0 < r_end; r0 += kChunk) {
    const int64_t row = r0 + rr;
    const bool rok = row < r_end;
    {
      const int64_t src = rok ? (gather ? (a.idx ? int64_t(a.idx[a.row0 + row]) : a.row0 + row) : row) : 0;
      T v[8];
      load8<T>(A + src * lda + 64 * mi + cc, rok, v);
#pragma unroll
      for (int e = 0; e < 8; ++e) At[cc + e][rr] = v[e];
    }
    {
      const int bc = 64 * ni + cc;
      T v[8];
      load8<T>(B + (rok ? row : 0) * ldb_ + bc, rok && bc < bw, v);
#pragma unroll
      for (int e = 0; e < 8; ++e) Bt[cc + e][rr] = v[e];
    }
    __syncthreads();
#pragma unroll
    for (int ks = 0; ks < kChunk / KS; ++ks) {
      typename M::frag fa[2], fb[2];
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        fa[i] = M::load(&At[wm + 16 * i + lr][ks * KS + E * lg]);
        fb[i] = M::load(&Bt[wn + 16 * i + lr][ks * KS + E * lg]);
      }
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = M::mma(fa[i], fb[j], acc[i][j]);
    }
    __syncthreads();
  }
  float *dst = a.part_w + size_t(split) * a.n_params + out0;
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int nn = 64 * ni + wn + 16 * j + lr;
      if (nn < nvalid) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int m = 64 * mi + wm + 16 * i + 4 * lg + q;
          dst[int64_t(m) * out_ld + nn] = acc[i][j][q];
        }
      }
    }
}

// Writes the compute copies that depend on parameter q.
template <class T, int K>
__device__ inline void publish(T *pub, int64_t q, float v) {
  const Layout L = layout(K);
  const T c = Mma<T>::cvt(v);
  if (q < L.b1) {
    const int64_t i = q / kHid, o = q % kHid;
    pub[kPubW1t + o * kIn + i] = c;
  } else if (q >= L.w2 && q < L.b2) {
    const int64_t i = (q - L.w2) / kHid, o = (q - L.w2) % kHid;
    pub[kPubW2t + o * kHid + i] = c;
    pub[kPubW2n + i * kHid + o] = c;
  } else if (q >= L.w3 && q < L.b3) {
    const int64_t i = (q - L.w3) / K, o = (q - L.w3) % K;
    pub[kPubW3t + o * kHid + i] = c;
    pub[kPubW3n + i * kOutPad + o] = c;
  }
}

template <class T, int K>
__global__ void mlp_publish_kernel(const float *__restrict__ theta, T *__restrict__ pub) {
  const int64_t q = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (q < layout(K).n) publish<T, K>(pub, q, theta[q]);
}

struct UpdateArgs {
  float *theta, *m, *v;
  void *pub;
  const float *part_w;
  int n_split;
  const float *part_b;
  int n_blk;
  const double *part_loss;
  double loss_scale;  // 1 / (n K)
  float *grad;        // gradient output (mode without Adam)
  double *loss;       // optional: mean loss of the batch
  double *loss_acc;   // optional: += mean loss of the batch
  int adam;
  float lr, beta1, beta2, eps, c1, c2;  // c1 = 1 - beta1^t, c2 = 1 - beta2^t
};

template <class T, int K>
__global__ __launch_bounds__(256) void mlp_update_kernel(UpdateArgs a) {
  const Layout L = layout(K);
  const int64_t q = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (q == 0 && (a.loss || a.loss_acc)) {
    double s = 0.0;
    for (int b = 0; b < a.n_blk; ++b) s += a.part_loss[b];
    s *= a.loss_scale;
    if (a.loss) *a.loss = s;
    if (a.loss_acc) *a.loss_acc += s;
  }
  if (q >= L.n) return;
  float g = 0.0f;
  int bias_col = -1;
  if (q >= L.b1 && q < L.w2) bias_col = int(q - L.b1);
  else if (q >= L.b2 && q < L.w3) bias_col = kHid + int(q - L.b2);
  else if (q >= L.b3) bias_col = 2 * kHid + int(q - L.b3);
  if (bias_col >= 0) {
    for (int b = 0; b < a.n_blk; ++b) g += a.part_b[size_t(b) * kBiasCols + bias_col];
  } else {
    for (int s = 0; s < a.n_split; ++s) g += a.part_w[size_t(s) * L.n + q];
  }
  if (!a.adam) {
    a.grad[q] = g;
    return;
  }
  const float m = a.beta1 * a.m[q] + (1.0f - a.beta1) * g;
  const float v = a.beta2 * a.v[q] + (1.0f - a.beta2) * g * g;
  const float mh = m / a.c1, vh = v / a.c2;
  const float th = a.theta[q] - a.lr * mh / (sqrtf(vh) + a.eps);
  a.m[q] = m;
  a.v[q] = v;
  a.theta[q] = th;
  publish<T, K>(static_cast<T *>(a.pub), q, th);
}

// x[r][i] = mean of p[r][lo_i .. hi_i), one wave per row.
template <class T>
__global__ __launch_bounds__(256) void pool_kernel(const uint16_t *__restrict__ p, int64_t ldb, int64_t n_p, int n_k,
                                                   T *__restrict__ x) {
  __shared__ float row[kWaves][2048];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  for (int64_t base = int64_t(blockIdx.x) * kWaves; base < n_p; base += int64_t(gridDim.x) * kWaves) {
    const int64_t r = base + w;
    if (r < n_p) {
      for (int c8 = lane * 8; c8 < n_k; c8 += 512) {
        const uint4 q = *reinterpret_cast<const uint4 *>(p + r * ldb + c8);
        const uint32_t u[4] = {q.x, q.y, q.z, q.w};
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          row[w][c8 + 2 * e] = bf16_bits_to_f32(uint16_t(u[e] & 0xFFFFu));
          row[w][c8 + 2 * e + 1] = bf16_bits_to_f32(uint16_t(u[e] >> 16));
        }
      }
    }
    __syncthreads();
    if (r < n_p) {
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int i = lane + 64 * q;
        const int lo = (i * n_k) / kIn, hi = ((i + 1) * n_k + kIn - 1) / kIn;
        float s = 0.0f;
        for (int c = lo; c < hi; ++c) s += row[w][c];
        x[r * kIn + i] = Mma<T>::cvt(s / float(hi - lo));
      }
    }
    __syncthreads();
  }
}

// Exact zeros of D := frac * mean(D) (one block).
__global__ __launch_bounds__(256) void fill_zeros_kernel(float *__restrict__ D, int64_t n, float frac) {
  __shared__ double red[4];
  double s = 0.0;
  for (int64_t e = threadIdx.x; e < n; e += 256) s += double(D[e]);
  s = wave_sum_all(s);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  const float fill = float(frac * (red[0] + red[1] + red[2] + red[3]) / double(n));
  for (int64_t e = threadIdx.x; e < n; e += 256)
    if (D[e] == 0.0f) D[e] = fill;
}

__global__ void ctrl_reset_kernel(NmfCtrl *c) {
  c->stop_at = INT_MAX;
  c->upd_ticket = 0;
  c->hist_len = 0;
}

}  // namespace
}  // namespace hsn

struct hsn_mlp {
  int k = 0, prec = HSN_PREC_BF16, device = 0;
  int64_t n = 0;
  float *theta = nullptr, *m = nullptr, *v = nullptr;  // one allocation
  void *pub = nullptr;
  int64_t step = 0;
  void *scr = nullptr;  // training scratch, grown on demand
  size_t scr_bytes = 0;
};

namespace hsn {
namespace {

size_t elem_size(const hsn_mlp *m) { return m->prec == HSN_PREC_BF16 ? 2 : 4; }

#define HSN_MLP_K(KK, X) \
  case KK: X; break;
#define HSN_MLP_DISPATCH(K, BODY)                                                                         \
  switch (K) {                                                                                           \
    HSN_MLP_K(1, BODY(1)) HSN_MLP_K(2, BODY(2)) HSN_MLP_K(3, BODY(3)) HSN_MLP_K(4, BODY(4))                 \
    HSN_MLP_K(5, BODY(5)) HSN_MLP_K(6, BODY(6)) HSN_MLP_K(7, BODY(7)) HSN_MLP_K(8, BODY(8)) default: break; \
  }

hsn_status publish_all(hsn_ctx *ctx, hsn_mlp *m, hipStream_t st) {
  const int nb = int((m->n + 255) / 256);
  if (m->prec == HSN_PREC_BF16) {
#define B(KK) mlp_publish_kernel<uint16_t, KK><<<nb, 256, 0, st>>>(m->theta, static_cast<uint16_t *>(m->pub))
    HSN_MLP_DISPATCH(m->k, B)
#undef B
  } else {
#define B(KK) mlp_publish_kernel<float, KK><<<nb, 256, 0, st>>>(m->theta, static_cast<float *>(m->pub))
    HSN_MLP_DISPATCH(m->k, B)
#undef B
  }
  HSN_LAUNCHED(ctx);
  return HSN_OK;
}

template <class T>
void launch_rows(int K, bool train, int n_blk, hipStream_t st, const RowsArgs &a) {
  if (train) {
#define B(KK) mlp_rows_kernel<T, KK, true><<<n_blk, 256, 0, st>>>(a)
    HSN_MLP_DISPATCH(K, B)
#undef B
  } else if (std::is_same<T, uint16_t>::value) {
    const unsigned nb2 = unsigned((a.n + kRowsB2 - 1) / kRowsB2);
#define B(KK) mlp_infer2_kernel<KK><<<nb2, 256, 0, st>>>(a)
    HSN_MLP_DISPATCH(K, B)
#undef B
  } else {
#define B(KK) mlp_rows_kernel<T, KK, false><<<n_blk, 256, 0, st>>>(a)
    HSN_MLP_DISPATCH(K, B)
#undef B
  }
}

// Training / gradient scratch for batches of up to `batch` rows.
struct Scratch {
  void *h1, *h2, *dz1, *dz2, *dz3;
  float *part_b, *part_w;
  double *part_loss, *loss_acc;
  int32_t *perm;
  int n_split;
};

int wgrad_splits(int64_t batch) { return int(std::max<int64_t>(1, std::min<int64_t>(16, batch / 256))); }

size_t scratch_bytes(const hsn_mlp *m, int64_t batch, int64_t n_perm, Scratch *s, void *base) {
  const int64_t bp = (batch + kRowsB - 1) / kRowsB * kRowsB;
  const int64_t nblk = bp / kRowsB;
  const int ns = wgrad_splits(batch);
  const size_t es = elem_size(m);
  const size_t sizes[] = {bp * kHid * es,          bp * kHid * es, bp * kHid * es, bp * kHid * es, bp * kOutPad * es,
                          nblk * kBiasCols * 4ull, ns * m->n * 4ull, nblk * 8ull,  8ull, size_t(n_perm) * 4};
  size_t off = 0;
  void *ptr[10];
  for (int i = 0; i < 10; ++i) {
    off = (off + 255) & ~size_t(255);
    ptr[i] = base ? static_cast<char *>(base) + off : nullptr;
    off += sizes[i];
  }
  if (s) {
    s->h1 = ptr[0];
    s->h2 = ptr[1];
    s->dz1 = ptr[2];
    s->dz2 = ptr[3];
    s->dz3 = ptr[4];
    s->part_b = static_cast<float *>(ptr[5]);
    s->part_w = static_cast<float *>(ptr[6]);
    s->part_loss = static_cast<double *>(ptr[7]);
    s->loss_acc = static_cast<double *>(ptr[8]);
    s->perm = static_cast<int32_t *>(ptr[9]);
    s->n_split = ns;
  }
  return off + 256;
}

hsn_status ensure_scratch(hsn_ctx *ctx, hsn_mlp *m, int64_t batch, int64_t n_perm, Scratch *s) {
  const size_t need = scratch_bytes(m, batch, n_perm, nullptr, nullptr);
  if (need > m->scr_bytes) {
    HSN_HIP(ctx, hipDeviceSynchronize());
    if (m->scr) (void)hipFree(m->scr);
    m->scr = nullptr;
    m->scr_bytes = 0;
    if (hipMalloc(&m->scr, need) != hipSuccess) {
      (void)hipGetLastError();
      m->scr = nullptr;
      return fail(ctx, HSN_ERR_OOM, "mlp: cannot allocate %zu bytes of training scratch", need);
    }
    m->scr_bytes = need;
  }
  scratch_bytes(m, batch, n_perm, s, m->scr);
  return HSN_OK;
}

// One batch: rows (train) -> wgrad -> update.  adam == false stores the gradient.
template <class T>
void queue_batch(hsn_ctx *ctx, hsn_mlp *m, hipStream_t st, const void *x, const int32_t *idx, int64_t row0,
                 int64_t nb, const float *target, const Scratch &s, bool adam, float *grad, double *loss,
                 const hsn_train_opts *o) {
  const int K = m->k;
  const int n_blk = int((nb + kRowsB - 1) / kRowsB);
  RowsArgs ra{};
  ra.x = x;
  ra.ldx = kIn;
  ra.idx = idx;
  ra.row0 = row0;
  ra.n = nb;
  ra.pub = m->pub;
  ra.theta = m->theta;
  ra.target = target;
  ra.scale = float(2.0 / (double(nb) * K));
  ra.h1 = s.h1;
  ra.h2 = s.h2;
  ra.dz1 = s.dz1;
  ra.dz2 = s.dz2;
  ra.dz3 = s.dz3;
  ra.part_b = s.part_b;
  ra.part_loss = s.part_loss;
  prof_begin(ctx, HSN_KERN_MLP_ROWS, st);
  launch_rows<T>(K, true, n_blk, st, ra);
  prof_end(ctx, HSN_KERN_MLP_ROWS, st);
  WgradArgs wa{x, kIn, idx, row0, nb, s.h1, s.h2, s.dz1, s.dz2, s.dz3, s.part_w, m->n};
  const dim3 grid(kTiles, s.n_split);
  prof_begin(ctx, HSN_KERN_MLP_WGRAD, st);
#define B(KK) mlp_wgrad_kernel<T, KK><<<grid, 256, 0, st>>>(wa)
  HSN_MLP_DISPATCH(K, B)
#undef B
  prof_end(ctx, HSN_KERN_MLP_WGRAD, st);
  UpdateArgs ua{};
  ua.theta = m->theta;
  ua.m = m->m;
  ua.v = m->v;
  ua.pub = m->pub;
  ua.part_w = s.part_w;
  ua.n_split = s.n_split;
  ua.part_b = s.part_b;
  ua.n_blk = n_blk;
  ua.part_loss = s.part_loss;
  ua.loss_scale = 1.0 / (double(nb) * K);
  ua.grad = grad;
  ua.loss = loss;
  ua.loss_acc = adam ? s.loss_acc : nullptr;
  ua.adam = adam ? 1 : 0;
  if (adam) {
    ++m->step;
    ua.lr = o->lr;
    ua.beta1 = o->beta1;
    ua.beta2 = o->beta2;
    ua.eps = o->eps;
    ua.c1 = float(1.0 - std::pow(double(o->beta1), double(m->step)));
    ua.c2 = float(1.0 - std::pow(double(o->beta2), double(m->step)));
  }
  const int nbu = int((m->n + 255) / 256);
#define B(KK) mlp_update_kernel<T, KK><<<nbu, 256, 0, st>>>(ua)
  HSN_MLP_DISPATCH(K, B)
#undef B
}

hsn_status check_mlp(hsn_ctx *ctx, const hsn_mlp *m) {
  if (!m) return fail(ctx, HSN_ERR_INVALID_ARG, "mlp: network is NULL");
  if (m->device != ctx->device) return fail(ctx, HSN_ERR_INVALID_ARG, "mlp: network lives on another device");
  return HSN_OK;
}

}  // namespace

// V0 = network(pool(p_bf16)) with the pooled rows in xbuf (n_p x 256 of the
// network's precision).
// V0 = network(pooled rows): the rows are pooled from pb into xbuf here,
// or come already pooled (pooled != NULL, [n_p][256] in the network's
// precision).
hsn_status mlp_infer_into(hsn_ctx *ctx, const hsn_mlp *m, const uint16_t *pb, int64_t ldb, int64_t n_p, int n_k,
                          float *V0, void *xbuf, const void *pooled, hipStream_t st) {
  if (!pooled) {
    const int nbp = int(std::min<int64_t>((n_p + kWaves - 1) / kWaves, 16 * int64_t(ctx->num_cu)));
    prof_begin(ctx, HSN_KERN_MLP_POOL, st);
    if (m->prec == HSN_PREC_BF16)
      pool_kernel<uint16_t><<<nbp, 256, 0, st>>>(pb, ldb, n_p, n_k, static_cast<uint16_t *>(xbuf));
    else
      pool_kernel<float><<<nbp, 256, 0, st>>>(pb, ldb, n_p, n_k, static_cast<float *>(xbuf));
    prof_end(ctx, HSN_KERN_MLP_POOL, st);
  }
  RowsArgs ra{};
  ra.x = pooled ? const_cast<void *>(pooled) : xbuf;
  ra.ldx = kIn;
  ra.n = n_p;
  ra.pub = m->pub;
  ra.theta = m->theta;
  ra.y = V0;
  ra.ldy = m->k;
  const int n_blk = int((n_p + kRowsB - 1) / kRowsB);
  prof_begin(ctx, HSN_KERN_MLP_ROWS, st);
  if (m->prec == HSN_PREC_BF16)
    launch_rows<uint16_t>(m->k, false, n_blk, st, ra);
  else
    launch_rows<float>(m->k, false, n_blk, st, ra);
  prof_end(ctx, HSN_KERN_MLP_ROWS, st);
  HSN_LAUNCHED(ctx);
  return HSN_OK;
}

size_t mlp_pool_bytes(const hsn_mlp *m, int64_t n_p) { return size_t(n_p) * kIn * elem_size(m); }
int mlp_k(const hsn_mlp *m) { return m->k; }
int mlp_device(const hsn_mlp *m) { return m->device; }

// The learned start of the NMF: V0 from the network, then D0 by exact
// row-wise NNLS against V0 (one N_D pass and the NNLS row rule), exact zeros
// of D0 set to 1e-6 mean(D0) so that multiplicative updates can move them.
// The N_D pass reads the float32 p, or the bfloat16 copy when wg_bf16 > 0
// (its grid; the decomposition's first rounds then run on that copy too).
// Leaves the control block open for the run.
hsn_status mlp_nmf_start(hsn_ctx *ctx, hipStream_t st, const hsn_mlp *m, const float *p, int64_t ldp,
                         const uint16_t *pb, int64_t ldb, int64_t n_p, int n_k, float *V, float *D, void *xbuf,
                         const void *pooled, const NmfWork &w, int n_wg, int wg_bf16) {
  hsn_status rc = mlp_infer_into(ctx, m, pb, ldb, n_p, n_k, V, xbuf, pooled, st);
  if (rc != HSN_OK) return rc;
  const int K = m->k;
  ctrl_reset_kernel<<<1, 1, 0, st>>>(w.ctrl);
  if (wg_bf16 > 0) {
    prof_begin(ctx, HSN_KERN_NMF_PASS_BF16, st);
    const bool ok = launch_pass_bf16(K, kModeND, false, wg_bf16, st, pb, ldb, n_p, n_k, V, w.gd, w.chol, w.img,
                                     w.part_nd, w.part_gv, w.part_obj, w.ctrl, 0, nullptr);
    prof_end(ctx, HSN_KERN_NMF_PASS_BF16, st);
    if (!ok) return fail(ctx, HSN_ERR_UNSUPPORTED, "learned start: bf16 N_D pass unsupported for this shape");
    n_wg = wg_bf16;
  } else {
    prof_begin(ctx, HSN_KERN_NMF_PASS, st);
    launch_pass_f32(K, kModeND, false, n_k > 1024 ? 2 : 1, n_wg, st, p, ldp, n_p, n_k, V, nullptr, D, w.gd, w.chol,
                    w.part_nd, w.part_gv, w.part_obj, w.ctrl, 0, nullptr);
    prof_end(ctx, HSN_KERN_NMF_PASS, st);
  }
  launch_update_d(K, kModeNV, st, D, w, n_wg, n_k, 0, false, 0.0, 0.0, false, 0);
  fill_zeros_kernel<<<1, 256, 0, st>>>(D, int64_t(n_k) * K, 1e-6f);
  HSN_LAUNCHED(ctx);
  return HSN_OK;
}

}  // namespace hsn

using namespace hsn;

extern "C" int64_t hsn_mlp_n_params(int k) { return (k < 1 || k > 8) ? -1 : layout(k).n; }

extern "C" hsn_status hsn_mlp_create(hsn_ctx *ctx, hsn_mlp **out, int k, int precision, const float *params_host) {
  if (!ctx) return HSN_ERR_INVALID_ARG;
  if (!out) return fail(ctx, HSN_ERR_INVALID_ARG, "mlp_create: out is NULL");
  *out = nullptr;
  if (k < 1 || k > 8) return fail(ctx, HSN_ERR_SHAPE, "mlp_create: k must be in 1..8 (got %d)", k);
  if (precision != HSN_PREC_BF16 && precision != HSN_PREC_FP32)
    return fail(ctx, HSN_ERR_INVALID_ARG, "mlp_create: bad precision");
  DeviceGuard dg(ctx->device);
  hsn_mlp *m = new hsn_mlp;
  m->k = k;
  m->prec = precision;
  m->device = ctx->device;
  m->n = layout(k).n;
  const size_t pb = size_t(kPubElems) * elem_size(m);
  float *state = nullptr;
  void *pub = nullptr;
  if (hipMalloc(&state, sizeof(float) * 3 * m->n) != hipSuccess || hipMalloc(&pub, pb) != hipSuccess) {
    (void)hipGetLastError();
    if (state) (void)hipFree(state);
    delete m;
    return fail(ctx, HSN_ERR_OOM, "mlp_create: out of device memory");
  }
  m->theta = state;
  m->m = state + m->n;
  m->v = state + 2 * m->n;
  m->pub = pub;
  hsn_status rc = HSN_OK;
  if (hipMemset(state, 0, sizeof(float) * 3 * m->n) != hipSuccess || hipMemset(pub, 0, pb) != hipSuccess)
    rc = fail(ctx, HSN_ERR_DEVICE, "mlp_create: hipMemset failed");
  if (rc == HSN_OK && params_host &&
      hipMemcpy(m->theta, params_host, sizeof(float) * m->n, hipMemcpyHostToDevice) != hipSuccess)
    rc = fail(ctx, HSN_ERR_DEVICE, "mlp_create: parameter upload failed");
  if (rc == HSN_OK) rc = publish_all(ctx, m, nullptr);
  if (rc == HSN_OK && hipDeviceSynchronize() != hipSuccess) rc = fail(ctx, HSN_ERR_DEVICE, "mlp_create: sync failed");
  if (rc != HSN_OK) {
    hsn_mlp_destroy(m);
    return rc;
  }
  *out = m;
  return HSN_OK;
}

extern "C" void hsn_mlp_destroy(hsn_mlp *m) {
  if (!m) return;
  DeviceGuard dg(m->device);
  (void)hipDeviceSynchronize();
  if (m->theta) (void)hipFree(m->theta);
  if (m->pub) (void)hipFree(m->pub);
  if (m->scr) (void)hipFree(m->scr);
  delete m;
}

extern "C" int hsn_mlp_k(const hsn_mlp *m) { return m ? m->k : -1; }
extern "C" int hsn_mlp_precision(const hsn_mlp *m) { return m ? m->prec : -1; }

extern "C" hsn_status hsn_mlp_get_params(hsn_ctx *ctx, const hsn_mlp *m, float *params_host) {
  if (!ctx) return HSN_ERR_INVALID_ARG;
  hsn_status rc = check_mlp(ctx, m);
  if (rc != HSN_OK) return rc;
  if (!params_host) return fail(ctx, HSN_ERR_INVALID_ARG, "mlp_get_params: params_host is NULL");
  DeviceGuard dg(ctx->device);
  HSN_HIP(ctx, hipDeviceSynchronize());
  HSN_HIP(ctx, hipMemcpy(params_host, m->theta, sizeof(float) * m->n, hipMemcpyDeviceToHost));
  return HSN_OK;
}

extern "C" hsn_status hsn_mlp_set_params(hsn_ctx *ctx, hsn_mlp *m, const float *params_host) {
  if (!ctx) return HSN_ERR_INVALID_ARG;
  hsn_status rc = check_mlp(ctx, m);
  if (rc != HSN_OK) return rc;
  if (!params_host) return fail(ctx, HSN_ERR_INVALID_ARG, "mlp_set_params: params_host is NULL");
  DeviceGuard dg(ctx->device);
  HSN_HIP(ctx, hipDeviceSynchronize());
  HSN_HIP(ctx, hipMemcpy(m->theta, params_host, sizeof(float) * m->n, hipMemcpyHostToDevice));
  HSN_HIP(ctx, hipMemset(m->m, 0, sizeof(float) * 2 * m->n));
  m->step = 0;
  if ((rc = publish_all(ctx, m, nullptr)) != HSN_OK) return rc;
  HSN_HIP(ctx, hipDeviceSynchronize());
  return HSN_OK;
}

extern "C" hsn_status hsn_mlp_pool(hsn_ctx *ctx, const uint16_t *p_bf16, int64_t ldb, int64_t n_p, int64_t n_k,
                                   int x_dtype, void *x, void *stream) {
  if (!ctx) return HSN_ERR_INVALID_ARG;
  if (!p_bf16 || !x) return fail(ctx, HSN_ERR_INVALID_ARG, "mlp_pool: NULL pointer");
  if (n_p < 0 || n_k < 1 || n_k > 2048) return fail(ctx, HSN_ERR_SHAPE, "mlp_pool: need 1 <= n_k <= 2048");
  if (ldb < n_k || ldb % 8 != 0 || reinterpret_cast<uintptr_t>(p_bf16) % 16 != 0)
    return fail(ctx, HSN_ERR_INVALID_ARG, "mlp_pool: ldb must be >= n_k and a multiple of 8, p_bf16 16-byte aligned");
  if (x_dtype != HSN_PREC_BF16 && x_dtype != HSN_PREC_FP32)
    return fail(ctx, HSN_ERR_INVALID_ARG, "mlp_pool: bad x_dtype");
  if (n_p == 0) return HSN_OK;
  DeviceGuard dg(ctx->device);
  hipStream_t st = static_cast<hipStream_t>(stream);
  const int nbp = int(std::min<int64_t>((n_p + kWaves - 1) / kWaves, 16 * int64_t(ctx->num_cu)));
  if (x_dtype == HSN_PREC_BF16)
    pool_kernel<uint16_t><<<nbp, 256, 0, st>>>(p_bf16, ldb, n_p, int(n_k), static_cast<uint16_t *>(x));
  else
    pool_kernel<float><<<nbp, 256, 0, st>>>(p_bf16, ldb, n_p, int(n_k), static_cast<float *>(x));
  HSN_LAUNCHED(ctx);
  return HSN_OK;
}

extern "C" hsn_status hsn_mlp_forward(hsn_ctx *ctx, const hsn_mlp *m, const void *x, int64_t n, float *y,
                                      void *stream) {
  if (!ctx) return HSN_ERR_INVALID_ARG;
  hsn_status rc = check_mlp(ctx, m);
  if (rc != HSN_OK) return rc;
  if (!x || !y) return fail(ctx, HSN_ERR_INVALID_ARG, "mlp_forward: NULL pointer");
  if (n < 0 || n > (int64_t(1) << 40)) return fail(ctx, HSN_ERR_SHAPE, "mlp_forward: bad n");
  if (reinterpret_cast<uintptr_t>(x) % 16 != 0) return fail(ctx, HSN_ERR_INVALID_ARG, "mlp_forward: x must be 16-byte aligned");
  if (n == 0) return HSN_OK;
  DeviceGuard dg(ctx->device);
  hipStream_t st = static_cast<hipStream_t>(stream);
  RowsArgs ra{};
  ra.x = x;
  ra.ldx = kIn;
  ra.n = n;
  ra.pub = m->pub;
  ra.theta = m->theta;
  ra.y = y;
  ra.ldy = m->k;
  const int n_blk = int((n + kRowsB - 1) / kRowsB);
  prof_begin(ctx, HSN_KERN_MLP_ROWS, st);
  if (m->prec == HSN_PREC_BF16)
    launch_rows<uint16_t>(m->k, false, n_blk, st, ra);
  else
    launch_rows<float>(m->k, false, n_blk, st, ra);
  prof_end(ctx, HSN_KERN_MLP_ROWS, st);
  HSN_LAUNCHED(ctx);
  return HSN_OK;
}

extern "C" hsn_status hsn_mlp_loss_grad(hsn_ctx *ctx, const hsn_mlp *mc, const void *x, const float *target,
                                        int64_t n, float *grad, double *loss, void *stream) {
  if (!ctx) return HSN_ERR_INVALID_ARG;
  hsn_status rc = check_mlp(ctx, mc);
  if (rc != HSN_OK) return rc;
  if (!x || !target || !grad) return fail(ctx, HSN_ERR_INVALID_ARG, "mlp_loss_grad: NULL pointer");
  if (n < 1 || n > (int64_t(1) << 24)) return fail(ctx, HSN_ERR_SHAPE, "mlp_loss_grad: need 1 <= n <= 2^24");
  if (reinterpret_cast<uintptr_t>(x) % 16 != 0)
    return fail(ctx, HSN_ERR_INVALID_ARG, "mlp_loss_grad: x must be 16-byte aligned");
  hsn_mlp *m = const_cast<hsn_mlp *>(mc);  // only the scratch changes
  DeviceGuard dg(ctx->device);
  hipStream_t st = static_cast<hipStream_t>(stream);
  Scratch s;
  if ((rc = ensure_scratch(ctx, m, n, 0, &s)) != HSN_OK) return rc;
  if (m->prec == HSN_PREC_BF16)
    queue_batch<uint16_t>(ctx, m, st, x, nullptr, 0, n, target, s, false, grad, loss, nullptr);
  else
    queue_batch<float>(ctx, m, st, x, nullptr, 0, n, target, s, false, grad, loss, nullptr);
  HSN_LAUNCHED(ctx);
  return HSN_OK;
}

extern "C" hsn_status hsn_mlp_train(hsn_ctx *ctx, hsn_mlp *m, const void *x, const float *target, int64_t n,
                                    const hsn_train_opts *o, double *loss_hist, void *stream) {
  if (!ctx) return HSN_ERR_INVALID_ARG;
  hsn_status rc = check_mlp(ctx, m);
  if (rc != HSN_OK) return rc;
  if (!x || !target || !o) return fail(ctx, HSN_ERR_INVALID_ARG, "mlp_train: NULL pointer");
  if (n < 1 || n > INT32_MAX) return fail(ctx, HSN_ERR_SHAPE, "mlp_train: need 1 <= n < 2^31");
  if (o->epochs < 0 || o->batch < 1 || o->batch > 65536)
    return fail(ctx, HSN_ERR_INVALID_ARG, "mlp_train: epochs >= 0 and 1 <= batch <= 65536 required");
  if (!(o->lr > 0.0f) || !(o->beta1 >= 0.0f && o->beta1 < 1.0f) || !(o->beta2 >= 0.0f && o->beta2 < 1.0f) ||
      !(o->eps > 0.0f))
    return fail(ctx, HSN_ERR_INVALID_ARG, "mlp_train: bad Adam parameters");
  if (reinterpret_cast<uintptr_t>(x) % 16 != 0) return fail(ctx, HSN_ERR_INVALID_ARG, "mlp_train: x must be 16-byte aligned");
  DeviceGuard dg(ctx->device);
  hipStream_t st = static_cast<hipStream_t>(stream);
  const int64_t batch = std::min<int64_t>(o->batch, n);
  Scratch s;
  if ((rc = ensure_scratch(ctx, m, batch, n, &s)) != HSN_OK) return rc;
  std::vector<int32_t> perm(n);
  const int64_t n_batches = (n + batch - 1) / batch;
  for (int e = 0; e < o->epochs; ++e) {
    // Seeded shuffle of the epoch (Fisher-Yates over a 64-bit Mersenne twister).
    std::iota(perm.begin(), perm.end(), 0);
    std::mt19937_64 rng(o->seed * 0x9E3779B97F4A7C15ull + uint64_t(e) + 1);
    for (int64_t i = n - 1; i > 0; --i) {
      const int64_t j = int64_t(rng() % uint64_t(i + 1));
      std::swap(perm[i], perm[j]);
    }
    HSN_HIP(ctx, hipMemcpyAsync(s.perm, perm.data(), sizeof(int32_t) * n, hipMemcpyHostToDevice, st));
    HSN_HIP(ctx, hipMemsetAsync(s.loss_acc, 0, sizeof(double), st));
    for (int64_t b = 0; b < n_batches; ++b) {
      const int64_t row0 = b * batch, nb = std::min<int64_t>(batch, n - row0);
      if (m->prec == HSN_PREC_BF16)
        queue_batch<uint16_t>(ctx, m, st, x, s.perm, row0, nb, target, s, true, nullptr, nullptr, o);
      else
        queue_batch<float>(ctx, m, st, x, s.perm, row0, nb, target, s, true, nullptr, nullptr, o);
    }
    HSN_LAUNCHED(ctx);
    double acc = 0.0;
    HSN_HIP(ctx, hipMemcpyAsync(&acc, s.loss_acc, sizeof(double), hipMemcpyDeviceToHost, st));
    HSN_HIP(ctx, hipStreamSynchronize(st));  // also keeps perm alive until its copy is done
    if (loss_hist) loss_hist[e] = acc / double(n_batches);
  }
  return HSN_OK;
}

extern "C" hsn_status hsn_mlp_infer(hsn_ctx *ctx, const hsn_mlp *m, const uint16_t *p_bf16, int64_t ldb, int64_t n_p,
                                    int64_t n_k, float *V0, void *stream) {
  if (!ctx) return HSN_ERR_INVALID_ARG;
  hsn_status rc = check_mlp(ctx, m);
  if (rc != HSN_OK) return rc;
  if (!p_bf16 || !V0) return fail(ctx, HSN_ERR_INVALID_ARG, "mlp_infer: NULL pointer");
  if (n_p < 0 || n_k < 1 || n_k > 2048) return fail(ctx, HSN_ERR_SHAPE, "mlp_infer: need 1 <= n_k <= 2048");
  if (ldb < n_k || ldb % 8 != 0 || reinterpret_cast<uintptr_t>(p_bf16) % 16 != 0)
    return fail(ctx, HSN_ERR_INVALID_ARG, "mlp_infer: ldb must be >= n_k and a multiple of 8, p_bf16 16-byte aligned");
  if (n_p == 0) return HSN_OK;
  DeviceGuard dg(ctx->device);
  if ((rc = ensure_ws(ctx, mlp_pool_bytes(m, n_p) + 256)) != HSN_OK) return rc;
  return mlp_infer_into(ctx, m, p_bf16, ldb, n_p, int(n_k), V0, ctx->ws, nullptr, static_cast<hipStream_t>(stream));
}

extern "C" hsn_status hsn_mlp_save(hsn_ctx *ctx, const hsn_mlp *m, const char *path) {
  if (!ctx) return HSN_ERR_INVALID_ARG;
  hsn_status rc = check_mlp(ctx, m);
  if (rc != HSN_OK) return rc;
  if (!path) return fail(ctx, HSN_ERR_INVALID_ARG, "mlp_save: path is NULL");
  std::vector<float> th(3 * m->n);  // parameters, then Adam's two moments
  DeviceGuard dg(ctx->device);
  HSN_HIP(ctx, hipDeviceSynchronize());
  HSN_HIP(ctx, hipMemcpy(th.data(), m->theta, sizeof(float) * 3 * m->n, hipMemcpyDeviceToHost));
  FILE *f = std::fopen(path, "wb");
  if (!f) return fail(ctx, HSN_ERR_INVALID_ARG, "mlp_save: cannot open %s", path);
  const int32_t hdr[2] = {m->k, m->prec};
  const int64_t step = m->step;
  bool ok = std::fwrite("HSNMLP01", 1, 8, f) == 8 && std::fwrite(hdr, 4, 2, f) == 2 &&
            std::fwrite(&step, 8, 1, f) == 1 && std::fwrite(th.data(), 4, th.size(), f) == th.size();
  ok = (std::fclose(f) == 0) && ok;
  return ok ? HSN_OK : fail(ctx, HSN_ERR_INVALID_ARG, "mlp_save: write to %s failed", path);
}

extern "C" hsn_status hsn_mlp_load(hsn_ctx *ctx, hsn_mlp **out, const char *path) {
  if (!ctx) return HSN_ERR_INVALID_ARG;
  if (!out || !path) return fail(ctx, HSN_ERR_INVALID_ARG, "mlp_load: NULL pointer");
  *out = nullptr;
  FILE *f = std::fopen(path, "rb");
  if (!f) return fail(ctx, HSN_ERR_INVALID_ARG, "mlp_load: cannot open %s", path);
  char magic[8];
  int32_t hdr[2];
  int64_t step = 0;
  bool ok = std::fread(magic, 1, 8, f) == 8 && std::memcmp(magic, "HSNMLP01", 8) == 0 &&
            std::fread(hdr, 4, 2, f) == 2 && std::fread(&step, 8, 1, f) == 1 && hdr[0] >= 1 && hdr[0] <= 8 &&
            (hdr[1] == HSN_PREC_BF16 || hdr[1] == HSN_PREC_FP32);
  std::vector<float> th;
  int64_t n = 0;
  if (ok) {
    n = layout(hdr[0]).n;
    th.resize(3 * n);
    ok = std::fread(th.data(), 4, th.size(), f) == th.size();
  }
  std::fclose(f);
  if (!ok) return fail(ctx, HSN_ERR_INVALID_ARG, "mlp_load: %s is not a network file", path);
  hsn_status rc = hsn_mlp_create(ctx, out, hdr[0], hdr[1], th.data());
  if (rc != HSN_OK) return rc;
  DeviceGuard dg(ctx->device);
  if (hipMemcpy((*out)->m, th.data() + n, sizeof(float) * 2 * n, hipMemcpyHostToDevice) != hipSuccess) {
    hsn_mlp_destroy(*out);
    *out = nullptr;
    return fail(ctx, HSN_ERR_DEVICE, "mlp_load: upload failed");
  }
  (*out)->step = step;
  return HSN_OK;
}
