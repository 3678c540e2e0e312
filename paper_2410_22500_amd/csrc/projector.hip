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
// rounding.  Positions carry far more than float32 precision (|x| reaches
// ~N/sqrt(2) pixels, where a float32 position would carry ~1e-5 px error):
// the adjoint evaluates them in float64; the forward ray starts in float64
// and steps in 32.32 fixed point, integer steps that are exact, so a
// position is off by less than (m + 1) 2^-33 px after m steps.  Weights
// and channel sums are float32.  In global memory all K channels of a pixel
// or bin are contiguous, so a gather kernel's tap is one vector load.
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
constexpr int kViewGroup = 4;  // views per orientation group of the LDS projector
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

// One ray (view g, detector column c): it steps along the image axis
// closer to its direction (rows for flat views, |cos| >= |sin|; columns for
// steep ones) and crosses the other axis at u(m) = u0 + m du, held as
// U = u 2^32 in 32.32 fixed point.  [m_lo, m_hi] is a conservative range of
// the steps at which a tap can fall inside the image.
struct Ray {
  int64_t U0, dU;
  int m_lo, m_hi;
  float inv_w, s1;  // 1/w and 2^-32 / w
};
__device__ __forceinline__ Ray ray_setup(const ViewGeom &g, int c, int n) {
  Ray ry;
  const double h = 0.5 * double(n - 1);
  const double sc = double(c) - h;
  const bool steep = fabs(g.sn) > fabs(g.cs);
  const double a = steep ? g.sn : g.cs, b = steep ? g.cs : g.sn;
  const double u0 = (sc + h * b) / a + h;
  const double du = -b / a;
  ry.U0 = __double2ll_rn(u0 * 4294967296.0);
  ry.dU = __double2ll_rn(du * 4294967296.0);
  ry.m_lo = 0;
  ry.m_hi = n - 1;
  if (du != 0.0) {
    const double ma = (-1.0 - u0) / du, mb = (double(n) - u0) / du;
    // clamped in float64 before the conversion (|du| may be ~1e-16)
    ry.m_lo = int(fmax(0.0, floor(fmin(ma, mb)) - 1.0));
    ry.m_hi = int(fmin(double(n - 1), ceil(fmax(ma, mb)) + 1.0));
  } else if (u0 < -1.0 || u0 >= double(n)) {
    ry.m_hi = -1;
  }
  ry.inv_w = float(g.inv_w);
  ry.s1 = ry.inv_w * 2.3283064365386963e-10f;  // exact: a power of two
  return ry;
}

// s[v][r][c][:] = alpha * sum_taps a * x[r][j][i][:] + beta * s[v][r][c][:]
//
// One thread per ray.  Steep views read the transposed image
// xT[r][i][j][:] (= x[r][j][i][:]), so for every view the taps of
// neighbouring detector columns are neighbouring pixels of one image row
// and a wave's loads are contiguous.  Tap t0 = floor(u) has weight
// (1 - f)/w and tap t0 + 1 weight f/w (f = u - t0); at the image edge a tap
// index is clamped and its weight set to 0, which keeps the loop free of
// branches.  Optional: per-block sums of squares of the outputs.
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
  const Ray ry = ray_setup(g, c, n);
  float acc[K];
#pragma unroll
  for (int q = 0; q < K; ++q) acc[q] = 0.0f;
  const float *img = ((fabs(g.sn) > fabs(g.cs)) ? xT : x) + size_t(r) * n * n * K;
  if (c < n) {
    int64_t U = ry.U0 + int64_t(ry.m_lo) * ry.dU;
#pragma unroll 4
    for (int m = ry.m_lo; m <= ry.m_hi; ++m, U += ry.dU) {
      const int t0 = int(U >> 32);
      const float w1f = float(uint32_t(U)) * ry.s1;
      const float w0 = (t0 >= 0 && t0 < n) ? ry.inv_w - w1f : 0.0f;
      const float w1 = (t0 + 1 >= 0 && t0 + 1 < n) ? w1f : 0.0f;
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

// Detector position of voxel (i, j) in view g: u = x_i cos + y_j sin + h,
// held as U = u 2^32 = a_i C + b_j S + (n - 1) 2^31 with the odd integers
// a_i = 2i - n + 1, b_j = 2j - n + 1 (x_i = a_i / 2, y_j = b_j / 2) and
// C = cos 2^31, S = sin 2^31 rounded to int32: integer arithmetic, exact
// given C and S, whose rounding moves u by at most n 2^-33 px.  Tap
// c0 = floor(u) = U >> 32 at |d| = f = (U mod 2^32) 2^-32, tap c0 + 1 at
// 1 - f; footprint weights max(0, 1 - |d|/w)/w with 1/w = iw:
//   w0 = max(0, iw - f iw^2),  w1 = max(0, iw - iw^2 + f iw^2).
struct VoxView {
  int C, S;
  float iw2, c1, iw;  // iw^2 2^-32, iw - iw^2, iw
};
__device__ __forceinline__ VoxView vox_view(const ViewGeom &g) {
  VoxView vv;
  vv.C = __double2int_rn(fmin(fmax(g.cs * 2147483648.0, -2147483647.0), 2147483647.0));
  vv.S = __double2int_rn(fmin(fmax(g.sn * 2147483648.0, -2147483647.0), 2147483647.0));
  vv.iw = float(g.inv_w);
  vv.iw2 = (vv.iw * vv.iw) * 2.3283064365386963e-10f;  // exact scaling by 2^-32
  vv.c1 = vv.iw - vv.iw * vv.iw;
  return vv;
}
__device__ __forceinline__ void vox_weights(uint32_t lo, float iw, float iw2, float c1, float &w0, float &w1) {
  const float lf = float(lo);
  w0 = fmaxf(0.0f, fmaf(-lf, iw2, iw));
  w1 = fmaxf(0.0f, fmaf(lf, iw2, c1));
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
  const int a = 2 * (ok ? i : 0) - n + 1, b = 2 * j - n + 1;
  const int64_t H = int64_t(n - 1) << 31;
  float acc[K];
#pragma unroll
  for (int q = 0; q < K; ++q) acc[q] = 0.0f;
  const size_t view_stride = size_t(n_slices) * n * K;
  const float *sr = s + size_t(r) * n * K;
#pragma unroll 4
  for (int v = 0; v < n_views; ++v) {
    const VoxView vv = vox_view(geom[v]);
    const int64_t U = int64_t(a) * vv.C + (int64_t(b) * vv.S + H);
    const int c0 = int(U >> 32);
    float w0, w1;
    vox_weights(uint32_t(U), vv.iw, vv.iw2, vv.c1, w0, w1);
    w0 = (c0 >= 0 && c0 < n) ? w0 : 0.0f;
    w1 = (c0 + 1 >= 0 && c0 + 1 < n) ? w1 : 0.0f;
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

// ---------------------------------------------------------------------------
// LDS-staged projector.  The kernels above take every tap from L1/L2 with
// a dependent gather per step.  Here a block copies the rows it shares (the
// slice image for A, the slice's sinogram rows for A^T) into LDS in bands
// and takes the taps from there, while the next band's global loads are in
// flight.  The staged layout (stage_* below) keeps a tap pair's channels
// (pixels t0, t0 + 1) at one or two addresses with immediate offsets, and
// band copies as 16-byte loads and stores.  Pad zero pixels (bins) on both
// sides and a tap index clamped into them: no bounds tests or weight masks
// in the inner loops.  A clamped tap reads 0 where the gather kernels apply
// weight 0, so with one thread per ray (split 1) both paths give the same
// values bit for bit.
// ---------------------------------------------------------------------------
constexpr int kLdsMaxThreads = 1024;
constexpr int kStageFloats = 15360;  // 60 KB of staged rows
constexpr int kCopyFloats = 16;      // floats each thread copies per band (K <= 4)

// Staged layout of a row of n pixels (A: image pixels; A^T: detector bins)
// with K channels, pad zero pixels on both sides.
//  K <= 4: pixel t's channels at (pad + t) K, one run per row.
//  K >= 5: two parts: channels 0..3 of pixel t at (pad + t) 4 (16-byte
//   aligned, so the first four channels of a tap pair are two 16-byte
//   reads), channels 4..K-1 at b0 + (pad + t) (K - 4), b0 = (n + 2 pad) 4.
//   With a pitch of K words a tap pair's 2 K words need 2 K / 2 paired
//   4-byte reads, and for even K two pixels 16 apart share a bank.
// pad: 2 (K = 2, 4) or 4 pixels, which keeps each part's data 16-byte
// aligned.
template <int K>
__host__ __device__ constexpr int stage_ka() { return K >= 5 ? 4 : K; }
template <int K>
__host__ __device__ constexpr int stage_kb() { return K >= 5 ? K - 4 : 0; }
template <int K>
__host__ __device__ constexpr int stage_pad() { return (K <= 4 && (2 * K) % 4 == 0) ? 2 : 4; }
// Row pitch: K >= 5 rounds it up to whole 16-byte units, so every staged
// row (and both its parts) starts 16-byte aligned whatever n is.
template <int K>
__host__ __device__ constexpr int stage_rp(int n) {
  return K >= 5 ? ((n + 2 * stage_pad<K>()) * K + 3) / 4 * 4 : (n + 2 * stage_pad<K>()) * K;
}
template <int K>
__host__ __device__ constexpr int stage_b0(int n) { return (n + 2 * stage_pad<K>()) * stage_ka<K>(); }
// Floats each thread copies per band: a group of four pixels (K >= 5) or kCopyFloats.
template <int K>
__host__ __device__ constexpr int copy_floats() { return K >= 5 ? 4 * K : kCopyFloats; }
// Staged offset (within its row) of float c of a source row of n K floats.
template <int K>
__device__ __forceinline__ int stage_pos(int c, int n) {
  constexpr int PAD = stage_pad<K>();
  if constexpr (K <= 4) {
    return PAD * K + c;
  } else {
    const int t = c / K, q = c - t * K;
    return q < 4 ? (PAD + t) * 4 + q : stage_b0<K>(n) + (PAD + t) * (K - 4) + (q - 4);
  }
}

// One thread's part of a band copy of `rows` source rows of n K floats
// (row i at src + i * src_ld) into staged rows of pitch rp.  Scalar: the
// floats t + u * nt of the band, u < copy_floats.  VEC, K <= 4: the
// float4s t + u * nt.  VEC, K >= 5: the group of pixels 4 t .. 4 t + 3 of
// the band (K float4 loads; its four 4-channel runs and its (K - 4)-channel
// runs, contiguous, as K float4 stores).  load() issues the global loads
// into registers; store() writes them to the staged rows, so a band's loads
// can be in flight while the previous band is used.
template <int K, bool VEC>
struct BandCopy {
  static constexpr int CF = copy_floats<K>();
  static constexpr bool SPLIT = K >= 5;
  static constexpr int U4 = SPLIT ? 1 : CF / 4;
  int n, width, rp;
  int row4[U4], col4[U4];  // SPLIT: the group's row and first pixel
  float buf[CF];

  __device__ __forceinline__ void init(int npix, int rpitch) {
    n = npix;
    width = npix * K;
    rp = rpitch;
    if constexpr (VEC) {
      if constexpr (SPLIT) {
        const int g = int(threadIdx.x), gpr = npix / 4;
        row4[0] = g / gpr;
        col4[0] = 4 * (g - row4[0] * gpr);
      } else {
        const int w4 = width / 4;
#pragma unroll
        for (int u = 0; u < U4; ++u) {
          const int f = int(threadIdx.x) + u * int(blockDim.x);
          row4[u] = f / w4;
          col4[u] = 4 * (f - row4[u] * w4);
        }
      }
    }
  }
  __device__ __forceinline__ void load(const float *__restrict__ src, size_t src_ld, int rows) {
    if constexpr (VEC) {
#pragma unroll
      for (int u = 0; u < U4; ++u) {
        if (row4[u] < rows) {
          const float *p = src + size_t(row4[u]) * src_ld + (SPLIT ? col4[u] * K : col4[u]);
#pragma unroll
          for (int i = 0; i < (SPLIT ? K : 1); ++i) {
            const float4 v = *reinterpret_cast<const float4 *>(p + 4 * i);
            buf[4 * (u + i)] = v.x;
            buf[4 * (u + i) + 1] = v.y;
            buf[4 * (u + i) + 2] = v.z;
            buf[4 * (u + i) + 3] = v.w;
          }
        }
      }
    } else {
#pragma unroll
      for (int u = 0; u < CF; ++u) {
        const int e = int(threadIdx.x) + u * int(blockDim.x);
        const int r = e / width, c = e - r * width;
        if (r < rows) buf[u] = src[size_t(r) * src_ld + c];
      }
    }
  }
  __device__ __forceinline__ void store(float *__restrict__ rows_lds, int rows) const {
    constexpr int PAD = stage_pad<K>();
    if constexpr (VEC && SPLIT) {
      constexpr int KB = K - 4;
      if (row4[0] < rows) {
        float *d = rows_lds + row4[0] * rp;
#pragma unroll
        for (int p = 0; p < 4; ++p)
          *reinterpret_cast<float4 *>(d + (PAD + col4[0] + p) * 4) =
              make_float4(buf[p * K], buf[p * K + 1], buf[p * K + 2], buf[p * K + 3]);
        float bv[4 * KB];
#pragma unroll
        for (int p = 0; p < 4; ++p)
#pragma unroll
          for (int j = 0; j < KB; ++j) bv[p * KB + j] = buf[p * K + 4 + j];
        float *db = d + stage_b0<K>(n) + (PAD + col4[0]) * KB;
#pragma unroll
        for (int i = 0; i < KB; ++i)
          *reinterpret_cast<float4 *>(db + 4 * i) = make_float4(bv[4 * i], bv[4 * i + 1], bv[4 * i + 2], bv[4 * i + 3]);
      }
    } else if constexpr (VEC) {
#pragma unroll
      for (int u = 0; u < U4; ++u) {
        if (row4[u] < rows)
          *reinterpret_cast<float4 *>(rows_lds + row4[u] * rp + PAD * K + col4[u]) =
              make_float4(buf[4 * u], buf[4 * u + 1], buf[4 * u + 2], buf[4 * u + 3]);
      }
    } else {
#pragma unroll
      for (int u = 0; u < CF; ++u) {
        const int e = int(threadIdx.x) + u * int(blockDim.x);
        const int r = e / width, c = e - r * width;
        if (r < rows) rows_lds[r * rp + stage_pos<K>(c, n)] = buf[u];
      }
    }
  }
};

// Both taps of every channel at staged pixel index tp (t0 + pad) of the
// staged row at `row`: a[q] = channel q of pixel tp, b[q] of pixel tp + 1.
template <int K>
__device__ __forceinline__ void pixel_taps(const float *row, unsigned tp, unsigned b0, float (&a)[K], float (&b)[K]) {
  if constexpr (K <= 4) {
    const float *p = row + __umul24(tp, unsigned(K));
#pragma unroll
    for (int q = 0; q < K; ++q) {
      a[q] = p[q];
      b[q] = p[K + q];
    }
  } else {
    constexpr int KB = K - 4;
    const float4 *pa = static_cast<const float4 *>(__builtin_assume_aligned(row + 4 * tp, 16));
    const float4 x = pa[0], y = pa[1];
    a[0] = x.x; a[1] = x.y; a[2] = x.z; a[3] = x.w;
    b[0] = y.x; b[1] = y.y; b[2] = y.z; b[3] = y.w;
    const float *pb = row + (b0 + tp * unsigned(KB));
    if constexpr (KB == 4) {
      const float4 *p4 = static_cast<const float4 *>(__builtin_assume_aligned(pb, 16));
      const float4 u = p4[0], v = p4[1];
      a[4] = u.x; a[5] = u.y; a[6] = u.z; a[7] = u.w;
      b[4] = v.x; b[5] = v.y; b[6] = v.z; b[7] = v.w;
    } else if constexpr (KB == 2) {
      const float2 *p2 = static_cast<const float2 *>(__builtin_assume_aligned(pb, 8));
      const float2 u = p2[0], v = p2[1];
      a[4] = u.x; a[5] = u.y;
      b[4] = v.x; b[5] = v.y;
    } else {
#pragma unroll
      for (int j = 0; j < KB; ++j) {
        a[4 + j] = pb[j];
        b[4 + j] = pb[KB + j];
      }
    }
  }
}

// Zeroes the pad pixels of `rows` staged rows (n data pixels each).
template <int K>
__device__ __forceinline__ void zero_pads(float *__restrict__ rows_lds, int rp, int n, int rows) {
  constexpr int PAD = stage_pad<K>(), KA = stage_ka<K>(), KB = stage_kb<K>();
  constexpr int PWA = PAD * KA, PWB = PAD * KB;  // floats of one side's pad, each part
  constexpr int PW = 2 * (PWA + PWB);
  const int b0 = stage_b0<K>(n);
  for (int e = threadIdx.x; e < rows * PW; e += blockDim.x) {
    const int row = e / PW, k = e - row * PW;
    int off;
    if (k < 2 * PWA) {
      off = k < PWA ? k : n * KA + k;
    } else {
      const int k2 = k - 2 * PWA;
      off = b0 + (k2 < PWB ? k2 : n * KB + k2);
    }
    rows_lds[row * rp + off] = 0.0f;
  }
}

// Block sum of squares of up to S values per thread (rows of v), any block
// size up to kLdsMaxThreads: partial[block][q].
template <int K, int S>
__device__ __forceinline__ void block_sumsq_n(const float (&v)[S][K], const bool (&valid)[S],
                                              double *__restrict__ partial, size_t block) {
  __shared__ double red[kLdsMaxThreads / 64][K];
  const int nw = int(blockDim.x) >> 6;
#pragma unroll
  for (int q = 0; q < K; ++q) {
    double a = 0.0;
#pragma unroll
    for (int e = 0; e < S; ++e) a += valid[e] ? double(v[e][q]) * double(v[e][q]) : 0.0;
    const double t = hsn::wave_sum_all(a);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6][q] = t;
  }
  __syncthreads();
  if (threadIdx.x < K) {
    double t = 0.0;
    for (int w = 0; w < nw; ++w) t += red[w][threadIdx.x];
    partial[block * K + threadIdx.x] = t;
  }
}

// A: one block = one slice and vb views of one orientation (a view group,
// or a half or quarter of one).  The slice image (x for flat views, xT for
// steep ones) passes through LDS in bands of band_rows rows.  Ray slot
// (view vi, column c) = vi * n + c; `split` copies of the ray set share the
// block (thread = copy * t1 + slot, t1 = blockDim.x / split), copy sp takes
// the band rows m with (m - m0) % split == sp, and the copies' sums are
// added in copy order at the end.
// Occupancy: K <= 5 (not 4) with float4 staging fits 64 VGPRs with a few
// spills outside the tap loop, so two 1024-thread blocks share a CU and one
// block's band copy and barriers overlap the other's taps (K = 5 at full
// size: 1.95 -> 1.56 ms); K = 4 and K >= 6 would spill inside the loop.
template <int K, bool VEC>
__global__ __launch_bounds__(kLdsMaxThreads) __attribute__((amdgpu_waves_per_eu((VEC && K <= 5 && K != 4) ? 8 : 4)))
void project_lds_kernel(
    const float *__restrict__ x, const float *__restrict__ xT, float *__restrict__ s,
    const ViewGeom *__restrict__ geom, const double *__restrict__ groups, int n_groups, int vb, int split,
    int n_slices, int n, int band_rows, float alpha, float beta, double *__restrict__ sumsq) {
  extern __shared__ __align__(16) float stage[];  // band_rows staged rows; then the copies' sums
  constexpr int PAD = stage_pad<K>();
  const int per_group = kViewGroup / vb;
  const BlockSlot bs = block_slot(blockIdx.x, n_slices, n_groups * per_group);
  if (bs.slice >= n_slices) return;
  const int r = bs.slice;
  const int gi = bs.rest / per_group, sub = bs.rest % per_group;
  const size_t part = size_t(r) * (n_groups * per_group) + bs.rest;
  // Views of a group share their orientation; padding (-1) sits at the end
  // of a group, so a sub-group whose first entry is padding is empty.
  const int v_first = int(groups[gi * kViewGroup + sub * vb]);
  if (v_first < 0) {
    if (sumsq && int(threadIdx.x) < K) sumsq[part * K + threadIdx.x] = 0.0;
    return;
  }
  const bool steep = fabs(geom[v_first].sn) > fabs(geom[v_first].cs);
  const int rp = stage_rp<K>(n);
  const int t1 = int(blockDim.x) / split;
  const int sp = int(threadIdx.x) / t1, slot = int(threadIdx.x) - sp * t1;
  // Ray slot -> (view vi, column c).  Neighbouring rays of one view are
  // 1/max(|cos|, |sin|) in [1, 1.41] pixels apart, so 32 of them (a
  // half-wave, one LDS pass) span up to 45 pixels and pixels 32 apart meet
  // in one of the 32 banks.  With an even vb and n % 16 == 0 a half-wave
  // instead takes 16 rays of each of two views of the group: their taps lie
  // within about 30 pixels (the views are close in angle), and for odd K
  // the pitch of K floats per pixel puts distinct pixels of such a window
  // in distinct banks.  Each ray's arithmetic is the same either way.
  int vi, c;
  if ((vb & 1) == 0 && (n & 15) == 0) {
    const int pi = slot / (2 * n), rr = slot - pi * (2 * n);
    vi = 2 * pi + ((rr >> 4) & 1);
    c = ((rr >> 5) << 4) + (rr & 15);
  } else {
    vi = slot / n;
    c = slot - vi * n;
  }
  int view = -1;
  Ray ry{0, 0, 0, -1, 0.0f, 0.0f};
  if (vi < vb) {
    view = int(groups[gi * kViewGroup + sub * vb + vi]);
    if (view >= 0) ry = ray_setup(geom[view], c, n);
  }
  zero_pads<K>(stage, rp, n, band_rows);
  const float *img = (steep ? xT : x) + size_t(r) * n * n * K;
  const unsigned sb0 = unsigned(stage_b0<K>(n));
  BandCopy<K, VEC> cp;
  cp.init(n, rp);
  int rows = min(band_rows, n);
  cp.load(img, size_t(n) * K, rows);
  float acc[K];
#pragma unroll
  for (int q = 0; q < K; ++q) acc[q] = 0.0f;
  const int64_t dUs = ry.dU * split;
  const int bstep = rp * split;
  for (int m0 = 0; m0 < n; m0 += band_rows) {
    __syncthreads();  // the previous band is no longer read
    cp.store(stage, rows);
    __syncthreads();
    const int rows_next = min(band_rows, n - m0 - band_rows);
    if (rows_next > 0) cp.load(img + size_t(m0 + band_rows) * n * K, size_t(n) * K, rows_next);
    const int mb = max(ry.m_lo, m0), me = min(ry.m_hi, m0 + rows - 1);
    int m = m0 + sp + ((max(mb - m0 - sp, 0) + split - 1) / split) * split;  // first own row >= mb
    // U carries PAD in its integer part: the high word is the staged pixel
    // index of tap t0 (t0 + PAD), clamped into the pads; the LDS offset is
    // a 24-bit multiply-add.
    int64_t U = ry.U0 + int64_t(m) * ry.dU + (int64_t(PAD) << 32);
    unsigned base = unsigned((m - m0) * rp);
    for (; m <= me; m += split, U += dUs, base += unsigned(bstep)) {
      const int tp = min(max(int(U >> 32), 0), n + 2 * PAD - 2);
      float a0[K], a1[K];
      pixel_taps<K>(stage + base, unsigned(tp), sb0, a0, a1);
      const float w1 = float(uint32_t(U)) * ry.s1;
      const float w0 = ry.inv_w - w1;
#pragma unroll
      for (int q = 0; q < K; ++q) acc[q] = fmaf(w1, a1[q], fmaf(w0, a0[q], acc[q]));
    }
    rows = rows_next;
  }
  if (split > 1) {
    __syncthreads();
#pragma unroll
    for (int q = 0; q < K; ++q) stage[int(threadIdx.x) * K + q] = acc[q];
    __syncthreads();
    if (sp == 0) {
      for (int c2 = 1; c2 < split; ++c2)
#pragma unroll
        for (int q = 0; q < K; ++q) acc[q] += stage[(c2 * t1 + slot) * K + q];
    }
  }
  float res[1][K];
  bool ok[1] = {sp == 0 && view >= 0};
#pragma unroll
  for (int q = 0; q < K; ++q) res[0][q] = 0.0f;
  if (ok[0]) {
    float *out = s + ((size_t(view) * n_slices + r) * n + c) * K;
#pragma unroll
    for (int q = 0; q < K; ++q) {
      res[0][q] = (beta == 0.0f) ? alpha * acc[q] : fmaf(alpha, acc[q], beta * out[q]);
      out[q] = res[0][q];
    }
  }
  if (sumsq) block_sumsq_n<K, 1>(res, ok, sumsq, part);
}

// Per-view geometry staged by backproject_lds_kernel ahead of the channel
// planes: C, S (int32), the step D = (b_{j + dj} - b_j) S between a
// thread's voxels (int64), iw^2 2^-32, iw - iw^2 and iw (float32).
struct StagedView {
  int64_t D;
  int C, S;
  float iw2, c1, iw, pad;
};
__host__ __device__ inline int geom_stage_bytes(int views) { return views * int(sizeof(StagedView)); }
constexpr int kMaxViewChunk = 64;

// A^T: one block = one slice and VPT * blockDim.x consecutive voxels of it
// (row-major j, i); voxel w of the block is taken by thread w % blockDim.x.
// With VPT > 1, blockDim.x is a multiple of n, so a thread's voxels share
// the column i and lie blockDim.x / n rows apart: their positions differ by
// the integer step D.  The slice's sinogram rows pass through LDS in chunks
// of view_chunk views, with the chunk's geometry.
// Occupancy: K = 5, 4 voxels per thread, float4 staging fits 76 VGPRs
// without spills, so three 512-thread blocks (each 42 KB of LDS at the full
// shape) share a CU (K = 5 at full size: 1.35 ms with one 1024-thread block,
// 1.27 ms with three of 512; plan_backproject picks 512 threads for K = 5).
template <int K, int VPT, bool VEC>
__global__ __launch_bounds__(kLdsMaxThreads) __attribute__((amdgpu_waves_per_eu((VEC && VPT == 4 && K == 5) ? 6 : 4)))
void backproject_lds_kernel(
    const float *__restrict__ s, float *__restrict__ x, const ViewGeom *__restrict__ geom, int n_views,
    int n_slices, int n, int view_chunk, float alpha, float beta, double *__restrict__ sumsq) {
  extern __shared__ __align__(16) float stage[];
  const int nt = blockDim.x;
  const int per_block = VPT * nt;
  const int n_blk = (n * n + per_block - 1) / per_block;
  const BlockSlot bs = block_slot(blockIdx.x, n_slices, n_blk);
  if (bs.slice >= n_slices) return;
  const int r = bs.slice;
  StagedView *gv = reinterpret_cast<StagedView *>(stage);
  float *planes = stage + geom_stage_bytes(view_chunk) / 4;
  constexpr int PAD = stage_pad<K>();
  const int rp = stage_rp<K>(n);
  const int64_t H = (int64_t(n - 1) << 31) + (int64_t(PAD) << 32);
  const int db = 2 * (nt / n);  // b_j step between a thread's voxels (VPT > 1)
  int vox[VPT];
  const int w0i = bs.rest * per_block + int(threadIdx.x);
  const int j0 = w0i / n, i0 = w0i - j0 * n;
  const int a = 2 * i0 - n + 1, b0 = 2 * j0 - n + 1;
#pragma unroll
  for (int e = 0; e < VPT; ++e) {
    const int w = w0i + e * nt;
    vox[e] = w < n * n ? w : -1;
  }
  zero_pads<K>(planes, rp, n, view_chunk);
  const unsigned sb0 = unsigned(stage_b0<K>(n));
  float acc[VPT][K];
#pragma unroll
  for (int e = 0; e < VPT; ++e)
#pragma unroll
    for (int q = 0; q < K; ++q) acc[e][q] = 0.0f;
  const size_t view_stride = size_t(n_slices) * n * K;
  const float *sr = s + size_t(r) * n * K;
  BandCopy<K, VEC> cp;
  cp.init(n, rp);
  int nv = min(view_chunk, n_views);
  cp.load(sr, view_stride, nv);
  ViewGeom gn{};
  if (int(threadIdx.x) < nv) gn = geom[threadIdx.x];
  for (int v0 = 0; v0 < n_views; v0 += view_chunk) {
    __syncthreads();  // the previous chunk is no longer read
    cp.store(planes, nv);
    if (int(threadIdx.x) < nv) {
      const VoxView vv = vox_view(gn);
      StagedView sv;
      sv.C = vv.C;
      sv.S = vv.S;
      sv.D = int64_t(db) * vv.S;
      sv.iw2 = vv.iw2;
      sv.c1 = vv.c1;
      sv.iw = vv.iw;
      sv.pad = 0.0f;
      gv[threadIdx.x] = sv;
    }
    __syncthreads();
    const int nv_next = min(view_chunk, n_views - v0 - view_chunk);
    if (nv_next > 0) {
      cp.load(sr + size_t(v0 + view_chunk) * view_stride, view_stride, nv_next);
      if (int(threadIdx.x) < nv_next) gn = geom[v0 + view_chunk + threadIdx.x];
    }
    // H carries PAD in its integer part: the high word of U is the staged
    // bin index of tap c0 (c0 + PAD), clamped into the pads.
    unsigned base = 0;
    for (int vl = 0; vl < nv; ++vl, base += unsigned(rp)) {
      const StagedView sv = gv[vl];
      int64_t U = int64_t(a) * sv.C + (int64_t(b0) * sv.S + H);
#pragma unroll
      for (int e = 0; e < VPT; ++e, U += sv.D) {
        const int cp0 = min(max(int(U >> 32), 0), n + 2 * PAD - 2);
        float a0[K], a1[K];
        pixel_taps<K>(planes + base, unsigned(cp0), sb0, a0, a1);
        float w0, w1;
        vox_weights(uint32_t(U), sv.iw, sv.iw2, sv.c1, w0, w1);
#pragma unroll
        for (int q = 0; q < K; ++q) acc[e][q] = fmaf(w1, a1[q], fmaf(w0, a0[q], acc[e][q]));
      }
    }
    nv = nv_next;
  }
  float res[VPT][K];
  bool ok[VPT];
#pragma unroll
  for (int e = 0; e < VPT; ++e) {
    ok[e] = vox[e] >= 0;
#pragma unroll
    for (int q = 0; q < K; ++q) res[e][q] = 0.0f;
    if (ok[e]) {
      float *out = x + (size_t(r) * n * n + size_t(vox[e])) * K;
#pragma unroll
      for (int q = 0; q < K; ++q) {
        res[e][q] = (beta == 0.0f) ? alpha * acc[e][q] : fmaf(alpha, acc[e][q], beta * out[q]);
        out[q] = res[e][q];
      }
    }
  }
  if (sumsq) block_sumsq_n<K, VPT>(res, ok, sumsq, size_t(r) * n_blk + bs.rest);
}

constexpr int kTile = 16;  // 16 x 16 pixels: one per thread of a 256-thread block

// tot[q] = sum over b < nblk of partial[b][q], q < K, by a block of 256
// threads in a fixed order, so that every block that calls it gets the same
// bits.  tot is visible to the whole block on return.
__device__ __forceinline__ void sum_partials(const double *__restrict__ partial, int nblk, int K,
                                             double *__restrict__ tot) {
  __shared__ double red[256];
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
    double sum = 0.0;
    for (int g = 0; g < G; ++g) sum += red[g * K + t];
    tot[t] = sum;
  }
  __syncthreads();
}

// CGLS scalars on the device: gamma[2][8] (double-buffered ||A^T r||^2),
// alpha[8], beta[8].
constexpr int kScal = 32;
enum { kGamma = 0, kAlphaOff = 16, kBetaOff = 24 };

// Per slice: xT[r][i][j][:] = x[r][j][i][:] through a 16 x 16 LDS tile.
// mode 0: pT = p^T.  mode 2: p = sv, pT = p^T.  mode 1: p = sv + coef[q] p,
// pT = p^T.  mode 3 (CGLS step, one launch): beta = ||A^T r||^2 / gamma
// from the A^T partial sums (gamma = st[gsel], the new value goes to
// st[1 - gsel]), x += alpha p with the old p, then p = sv + beta p, pT = p^T.
// mode 4: mode 3 without the x update (the MBIR direction step, whose
// partials are <r, r> of the CG step kernel).  mode 5: mode 3 with alpha
// and beta already formed in st (by the scalar kernel, when the partials
// are too many for every block to sum).
template <int K>
__global__ __launch_bounds__(256) void xpby_transpose_kernel(float *__restrict__ p, float *__restrict__ pT,
                                                             const float *__restrict__ sv,
                                                             const double *__restrict__ coef, int n, int mode,
                                                             float *__restrict__ x, const double *__restrict__ partial,
                                                             int nblk, double *__restrict__ st, int gsel) {
  __shared__ float tile[kTile][kTile + 1][K];
  __shared__ double tot[8];
  const int r = blockIdx.z;
  const int j0 = blockIdx.y * kTile, i0 = blockIdx.x * kTile;
  const size_t base = size_t(r) * n * n * K;
  float cf[K], al[K];
  if (mode == 3 || mode == 4) {
    sum_partials(partial, nblk, K, tot);
    const double *gamma = st + kGamma + 8 * gsel;
#pragma unroll
    for (int q = 0; q < K; ++q) {
      cf[q] = float(gamma[q] > 0.0 ? tot[q] / gamma[q] : 0.0);
      al[q] = float(st[kAlphaOff + q]);
    }
    if (blockIdx.x == 0 && blockIdx.y == 0 && blockIdx.z == 0 && int(threadIdx.x) < K)
      st[kGamma + 8 * (1 - gsel) + threadIdx.x] = tot[threadIdx.x];
  } else if (mode == 5) {
#pragma unroll
    for (int q = 0; q < K; ++q) {
      cf[q] = float(st[kBetaOff + q]);
      al[q] = float(st[kAlphaOff + q]);
    }
  } else {
#pragma unroll
    for (int q = 0; q < K; ++q) {
      cf[q] = (mode == 1) ? float(coef[q]) : 0.0f;
      al[q] = 0.0f;
    }
  }
  for (int e = threadIdx.x; e < kTile * kTile; e += 256) {
    const int jj = e / kTile, ii = e % kTile;
    const int j = j0 + jj, i = i0 + ii;
    if (j < n && i < n) {
      const size_t o = base + (size_t(j) * n + i) * K;
      float val[K];
      if (mode == 0) {  // plain transpose of p
        load_k<K>(p + o, val);
      } else {          // p = sv + coef * p (modes 1, 3, 4, 5), p = sv (mode 2)
        float a[K], b[K];
        load_k<K>(sv + o, a);
        if (mode != 2) load_k<K>(p + o, b);
        if (mode == 3 || mode == 5) {
          float xv[K];
          load_k<K>(x + o, xv);
#pragma unroll
          for (int q = 0; q < K; ++q) x[o + q] = fmaf(al[q], b[q], xv[q]);
        }
#pragma unroll
        for (int q = 0; q < K; ++q) {
          val[q] = (mode == 2) ? a[q] : fmaf(cf[q], b[q], a[q]);
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

// One block of 256 threads, from partial sums tot[q] (see sum_partials):
//   kSetGamma: gamma[gsel] = tot          kAlpha: alpha = gamma[gsel] / tot
//   kBeta: beta = tot / gamma[gsel], gamma[1 - gsel] = tot
//   kResid: out = sqrt(tot)
// A zero denominator gives 0 (the iteration has converged).
enum { kSetGamma = 0, kAlpha = 1, kBeta = 2, kResid = 3 };
__global__ __launch_bounds__(256) void cgls_scalar_kernel(const double *__restrict__ partial, int nblk, int K,
                                                          int mode, double *__restrict__ st, int gsel,
                                                          double *__restrict__ out) {
  __shared__ double tot[8];
  sum_partials(partial, nblk, K, tot);
  const int q = threadIdx.x;
  if (q >= K) return;
  const double tq = tot[q];
  double *gamma = st + kGamma + 8 * gsel, *gamma_next = st + kGamma + 8 * (1 - gsel);
  if (mode == kSetGamma) {
    gamma[q] = tq;
  } else if (mode == kAlpha) {
    st[kAlphaOff + q] = (tq > 0.0) ? gamma[q] / tq : 0.0;
  } else if (mode == kBeta) {
    st[kBetaOff + q] = (gamma[q] > 0.0) ? tq / gamma[q] : 0.0;
    gamma_next[q] = tq;
  } else if (out) {
    out[q] = sqrt(tq);
  }
}

// CGLS start in one launch: x = 0 over nx values, r = b over nr values (a
// kernel rather than a runtime copy, which leaves a gap before the next
// kernel on the stream).
__global__ void cgls_start_kernel(float *__restrict__ x, int64_t nx, float *__restrict__ r,
                                  const float *__restrict__ b, int64_t nr) {
  for (int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; e < nx + nr; e += int64_t(gridDim.x) * blockDim.x) {
    if (e < nx)
      x[e] = 0.0f;
    else
      r[e - nx] = b[e - nx];
  }
}

// Two device copies in one launch (a = a_src over na values, b = b_src over nb).
__global__ void copy2_kernel(float *__restrict__ a, const float *__restrict__ a_src, int64_t na,
                             float *__restrict__ b, const float *__restrict__ b_src, int64_t nb) {
  for (int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; e < na + nb; e += int64_t(gridDim.x) * blockDim.x) {
    if (e < na)
      a[e] = a_src[e];
    else
      b[e - na] = b_src[e - na];
  }
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

// CGLS residual step in one launch (256 threads per block): alpha =
// gamma[gsel] / ||A p||^2 from the A partial sums, stored by block 0 for
// the direction update; r -= alpha q over nr values.
__global__ __launch_bounds__(256) void cgls_rstep_kernel(float *__restrict__ r, const float *__restrict__ q, int64_t nr,
                                                         int K, const double *__restrict__ partial, int nblk,
                                                         double *__restrict__ st, int gsel) {
  __shared__ double tot[8];
  sum_partials(partial, nblk, K, tot);
  float al[8];
  const double *gamma = st + kGamma + 8 * gsel;
#pragma unroll
  for (int c = 0; c < 8; ++c) al[c] = (c < K && tot[c] > 0.0) ? float(gamma[c] / tot[c]) : 0.0f;
  if (blockIdx.x == 0 && int(threadIdx.x) < K)
    st[kAlphaOff + threadIdx.x] = tot[threadIdx.x] > 0.0 ? gamma[threadIdx.x] / tot[threadIdx.x] : 0.0;
  for (int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; e < nr; e += int64_t(gridDim.x) * blockDim.x) {
    const int c = int(e % K);
    float a = al[0];
#pragma unroll
    for (int cc = 1; cc < 8; ++cc) a = (c == cc) ? al[cc] : a;
    r[e] = fmaf(-a, q[e], r[e]);
  }
}

// ---------------------------------------------------------------------------
// qGGMRF prior of eq. (5) (q = 2): h(x) = sum over 8-neighbour pairs {s, r}
// inside a slice of b_sr rho(x_s - x_r), b = w1 (nearest), w1 / sqrt(2)
// (diagonal), w1 = 1 / (4 + 2 sqrt(2));
//   rho(d) = |d|^p / (p sx^p) u / (1 + u),  u = |d / (T sx)|^(2 - p).
// The majorisation-minimisation solver uses its symmetric-bound quadratic
// surrogate with a(d) = rho'(|d|) / (2 |d|) = c0 / (1 + u) (1 + ((2 - p) / p) / (1 + u)),
// c0 = 1 / (2 sx^2 T^(2-p)), and the surrogate Hessian
//   (L v)_s = 2 sum_r b_sr a(x'_s - x'_r) (v_s - v_r)   (x' the anchor).
// ---------------------------------------------------------------------------
struct PriorArgs {
  float c0[8];       // 1 / (2 sigma_x^2 T^(2-p)) per channel
  float inv_tsx[8];  // 1 / (T sigma_x)
  float s2[8];       // sigma_v^2
  float e;           // 2 - p
  float rq;          // (2 - p) / p
};

constexpr float kPriorW1 = 0.14644660940672624f;   // 1 / (4 + 2 sqrt(2))
constexpr float kPriorW2 = 0.10355339059327377f;   // w1 / sqrt(2)
constexpr int kPriorBlocks = 1024;

// u = 2^(e log2 t) and 1 / (1 + u) on the hardware exp2, log2 and reciprocal
// (about 1 ulp each); t = 0 gives log2 = -inf and u = 0.  Both ends of an
// edge evaluate the same |d| with the same instructions, so L stays
// symmetric bit for bit.
__device__ __forceinline__ float prior_coef(float d, float c0, float inv_tsx, float e, float rq) {
  const float u = (e == 0.0f) ? 1.0f : __builtin_amdgcn_exp2f(e * __builtin_amdgcn_logf(fabsf(d) * inv_tsx));
  const float iu = __builtin_amdgcn_rcpf(1.0f + u);
  return c0 * iu * fmaf(rq, iu, 1.0f);
}

// w_s += sign sigma_v^2 (L v)_s for every voxel, L with the weights of the
// anchor xa; per-block float64 partials of <v, w_new> (dot_self = 0) or
// <w_new, w_new> (dot_self = 1) per channel.  A block takes 16 x 16 tiles of
// a slice in turn (fixed grid, so the sums have a fixed order) and stages
// the tile of xa and v with a one-pixel halo in LDS, so every operand is
// read from HBM about once.
constexpr int kPriorTile = 16, kPriorHalo = kPriorTile + 2;

template <int K>
__global__ __launch_bounds__(256) void prior_apply_kernel(const float *__restrict__ xa, const float *__restrict__ v,
                                                          float *__restrict__ w, int n, int n_slices, PriorArgs pa,
                                                          float sign, int dot_self, double *__restrict__ partial) {
  __shared__ float sa[kPriorHalo * kPriorHalo * K], sv[kPriorHalo * kPriorHalo * K];
  double dot[K];
#pragma unroll
  for (int q = 0; q < K; ++q) dot[q] = 0.0;
  const int t = threadIdx.x, tx = t % kPriorTile, ty = t / kPriorTile;
  const int tn = (n + kPriorTile - 1) / kPriorTile;
  const int64_t n_tiles = int64_t(n_slices) * tn * tn;
  const int64_t nn = int64_t(n) * n;
  for (int64_t tile = blockIdx.x; tile < n_tiles; tile += gridDim.x) {
    const int64_t r = tile / (int64_t(tn) * tn);
    const int rem = int(tile - r * tn * tn);
    const int j0 = (rem / tn) * kPriorTile, i0 = (rem % tn) * kPriorTile;
    __syncthreads();  // the previous tile's LDS reads are done
    for (int e = t; e < kPriorHalo * kPriorHalo; e += 256) {
      const int hy = e / kPriorHalo, hx = e - hy * kPriorHalo;
      const int jj = j0 + hy - 1, ii = i0 + hx - 1;
      float a[K], b[K];
      if (jj >= 0 && jj < n && ii >= 0 && ii < n) {
        const int64_t o = (r * nn + int64_t(jj) * n + ii) * K;
        load_k<K>(xa + o, a);
        load_k<K>(v + o, b);
      } else {
#pragma unroll
        for (int q = 0; q < K; ++q) a[q] = b[q] = 0.0f;
      }
#pragma unroll
      for (int q = 0; q < K; ++q) {
        sa[e * K + q] = a[q];
        sv[e * K + q] = b[q];
      }
    }
    __syncthreads();
    const int j = j0 + ty, i = i0 + tx;
    if (j < n && i < n) {
      const int c = (ty + 1) * kPriorHalo + tx + 1;
      float as[K], vs[K], acc[K];
#pragma unroll
      for (int q = 0; q < K; ++q) {
        as[q] = sa[c * K + q];
        vs[q] = sv[c * K + q];
        acc[q] = 0.0f;
      }
#pragma unroll
      for (int nb = 0; nb < 8; ++nb) {
        const int dj = (nb < 3) ? -1 : (nb < 5 ? 0 : 1);                 // rows above, same row, below
        const int di = (nb < 3) ? nb - 1 : (nb < 5 ? 2 * nb - 7 : nb - 6);  // -1 0 1 | -1 1 | -1 0 1
        const int jj = j + dj, ii = i + di;
        if (jj < 0 || jj >= n || ii < 0 || ii >= n) continue;
        const float b = (dj == 0 || di == 0) ? kPriorW1 : kPriorW2;
        const int cn = c + dj * kPriorHalo + di;
#pragma unroll
        for (int q = 0; q < K; ++q)
          acc[q] = fmaf(b * prior_coef(as[q] - sa[cn * K + q], pa.c0[q], pa.inv_tsx[q], pa.e, pa.rq),
                        vs[q] - sv[cn * K + q], acc[q]);
      }
      const int64_t vox = r * nn + int64_t(j) * n + i;
#pragma unroll
      for (int q = 0; q < K; ++q) {
        const float res = fmaf(sign * pa.s2[q], 2.0f * acc[q], w[vox * K + q]);
        w[vox * K + q] = res;
        dot[q] += double(dot_self ? res : vs[q]) * double(res);
      }
    }
  }
  __shared__ double red[4][K];
#pragma unroll
  for (int q = 0; q < K; ++q) {
    const double tt = hsn::wave_sum_all(dot[q]);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6][q] = tt;
  }
  __syncthreads();
  if (int(threadIdx.x) < K) {
    const int q = threadIdx.x;
    partial[size_t(blockIdx.x) * K + q] = ((red[0][q] + red[1][q]) + red[2][q]) + red[3][q];
  }
}

// CG step of the surrogate solve: alpha = gamma[gsel] / <d, w> per channel,
// every block summing the prior kernel's partials of <d, w> itself in one
// fixed order (the scalars of cgls_scalar_kernel, without its launch); then
// x += alpha d, r -= alpha w, and per-block partials of <r, r> into
// partial_out (a buffer of its own: other blocks still read the inputs).
// Fixed grid.
template <int K>
__global__ __launch_bounds__(kDotThreads) void mbir_step_kernel(float *__restrict__ x, const float *__restrict__ d,
                                                                float *__restrict__ r, const float *__restrict__ w,
                                                                int64_t n_vox, const double *__restrict__ st, int gsel,
                                                                const double *__restrict__ partial_dw, int nblk_dw,
                                                                double *__restrict__ partial_out) {
  __shared__ double tot[8];
  sum_partials(partial_dw, nblk_dw, K, tot);
  const double *gamma = st + kGamma + 8 * gsel;
  float al[K];
  double dot[K];
#pragma unroll
  for (int q = 0; q < K; ++q) {
    al[q] = float(tot[q] > 0.0 ? gamma[q] / tot[q] : 0.0);
    dot[q] = 0.0;
  }
  for (int64_t vox = int64_t(blockIdx.x) * kDotThreads + threadIdx.x; vox < n_vox;
       vox += int64_t(gridDim.x) * kDotThreads) {
#pragma unroll
    for (int q = 0; q < K; ++q) {
      const int64_t e = vox * K + q;
      x[e] = fmaf(al[q], d[e], x[e]);
      const float rn = fmaf(-al[q], w[e], r[e]);
      r[e] = rn;
      dot[q] += double(rn) * double(rn);
    }
  }
  __shared__ double red[kDotThreads / 64][K];
#pragma unroll
  for (int q = 0; q < K; ++q) {
    const double t = hsn::wave_sum_all(dot[q]);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6][q] = t;
  }
  __syncthreads();
  if (int(threadIdx.x) < K) {
    double t = 0.0;
    for (int wv = 0; wv < kDotThreads / 64; ++wv) t += red[wv][threadIdx.x];
    partial_out[size_t(blockIdx.x) * K + threadIdx.x] = t;
  }
}

// ---------------------------------------------------------------------------
// FBP ramp filter (band-limited ramp sampled at the detector pitch:
// h[0] = 1/4, h[d] = -1/(pi^2 d^2) for odd d, 0 for even d != 0):
//   q[row][c][:] = sum_{c'} h[c - c'] s[row][c'][:]   (zero-padded, not circular)
// One workgroup per detector row (view, slice), the row staged in LDS; each
// output sums the centre tap, then the odd taps d = 1, 3, ... (left before
// right), in float32.
// ---------------------------------------------------------------------------
constexpr int kFbpMaxFloats = 8192;

template <int K>
__global__ __launch_bounds__(256) void ramp_filter_kernel(const float *__restrict__ s, int64_t ld, int n,
                                                          float *__restrict__ q) {
  __shared__ float row[kFbpMaxFloats];
  __shared__ float hodd[kFbpMaxFloats / 2 + 1];  // h[2m + 1]
  const int64_t rr = blockIdx.x;
  const float *src = s + rr * n * ld;
  for (int e = threadIdx.x; e < n * K; e += blockDim.x) {
    const int c = e / K, k = e - (e / K) * K;
    row[e] = src[int64_t(c) * ld + k];
  }
  for (int m = threadIdx.x; 2 * m + 1 < n; m += blockDim.x) {
    const double d = double(2 * m + 1);
    hodd[m] = float(-1.0 / (M_PI * M_PI * d * d));
  }
  __syncthreads();
  for (int c = threadIdx.x; c < n; c += blockDim.x) {
    float acc[K];
#pragma unroll
    for (int k = 0; k < K; ++k) acc[k] = 0.25f * row[c * K + k];
    for (int m = 0; 2 * m + 1 < n; ++m) {
      const int d = 2 * m + 1;
      const float h = hodd[m];
      if (c - d >= 0) {
#pragma unroll
        for (int k = 0; k < K; ++k) acc[k] = fmaf(h, row[(c - d) * K + k], acc[k]);
      }
      if (c + d < n) {
#pragma unroll
        for (int k = 0; k < K; ++k) acc[k] = fmaf(h, row[(c + d) * K + k], acc[k]);
      }
    }
    float *dst = q + (rr * n + c) * K;
#pragma unroll
    for (int k = 0; k < K; ++k) dst[k] = acc[k];
  }
}

template <int K>
void launch_ramp(const float *s, int64_t ld, const hsn_geom *g, float *q, hipStream_t st) {
  ramp_filter_kernel<K><<<unsigned(g->n_views * g->n_slices), 256, 0, st>>>(s, ld, int(g->n_cols), q);
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
// Views of one orientation in groups of kViewGroup for the LDS projector:
// flat views (|cos| >= |sin|) in order, then steep ones; -1 pads a group.
struct GeomTab {
  const ViewGeom *views;
  const double *groups;  // [n_groups][kViewGroup] view index (as double), -1 = none
  int n_groups;
};

// Per-view constants in float64 on the host, and the view groups; uploaded
// only when they change.
hsn_status upload_geom(hsn_ctx *ctx, const hsn_geom *g, hipStream_t st, GeomTab *out) {
  const int nv = int(g->n_views);
  std::vector<double> tab(size_t(nv) * 4);
  std::vector<int> flat, steep;
  for (int v = 0; v < nv; ++v) {
    const double t = g->angles ? g->angles[v] : double(v) * M_PI / double(nv);
    const double cs = std::cos(t), sn = std::sin(t);
    const double w = std::fmax(std::fabs(cs), std::fabs(sn));
    tab[4 * v + 0] = cs;
    tab[4 * v + 1] = sn;
    tab[4 * v + 2] = w;
    tab[4 * v + 3] = 1.0 / w;
    (std::fabs(sn) > std::fabs(cs) ? steep : flat).push_back(v);
  }
  int n_groups = 0;
  for (const auto *list : {&flat, &steep})
    for (size_t a = 0; a < list->size(); a += kViewGroup) {
      for (int e = 0; e < kViewGroup; ++e)
        tab.push_back(a + e < list->size() ? double((*list)[a + e]) : -1.0);
      ++n_groups;
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
  out->views = reinterpret_cast<const ViewGeom *>(ctx->geom);
  out->groups = ctx->geom + size_t(nv) * 4;
  out->n_groups = n_groups;
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

// Launch shape of one projector application: the LDS-staged kernel or,
// where a staged row does not fit or the caller asked for it, the gather
// kernel.
struct ProjLaunch {
  bool lds = false;
  int vb = 0, split = 0;    // A: views per block, copies of the ray set per block
  int vpt = 0;              // A^T: voxels per thread
  int threads = 0;
  int rows = 0;             // A: image rows per band; A^T: views per chunk
  unsigned grid = 0;
  size_t partials = 0;      // sum-of-squares partials (one per real block)
  size_t lds_bytes = 0;
};

int round64(int64_t v) { return int((v + 63) / 64 * 64); }
// Floats each thread copies per band (copy_floats for the geometry's K).
int64_t copy_floats_k(int64_t k) { return k >= 5 ? 4 * k : kCopyFloats; }
// The band copy moves float4s: whole source rows of n K floats (K <= 4),
// groups of four pixels (K >= 5).
bool copy_vec(int64_t k, int64_t n) { return k >= 5 ? n % 4 == 0 : (n * k) % 4 == 0; }
// Row pitch (floats) of the staged rows for the geometry's K.
int64_t staged_rp(const hsn_geom *g) {
  const int n = int(g->n_cols);
  switch (g->k) {
    case 1: return stage_rp<1>(n);
    case 2: return stage_rp<2>(n);
    case 3: return stage_rp<3>(n);
    case 4: return stage_rp<4>(n);
    case 5: return stage_rp<5>(n);
    case 6: return stage_rp<6>(n);
    case 7: return stage_rp<7>(n);
    default: return stage_rp<8>(n);
  }
}

ProjLaunch plan_project(const hsn_ctx *ctx, const hsn_geom *g, int n_groups) {
  ProjLaunch L;
  const int64_t n = g->n_cols, K = g->k, rp = staged_rp(g);
  if (ctx->proj_views < 0 || rp > kStageFloats || n > kLdsMaxThreads) {
    L.threads = kRayThreads;
    L.grid = project_grid(g);
    L.partials = size_t(g->n_slices) * g->n_views * ((n + kRayThreads - 1) / kRayThreads);
    return L;
  }
  auto blocks = [&](int vb) { return int64_t(g->n_slices) * n_groups * (kViewGroup / vb); };
  int vb = ctx->proj_views;
  if (vb > 0) {
    while (vb > 1 && int64_t(vb) * n > kLdsMaxThreads) vb /= 2;
  } else {
    // Most views per block (least staging) that still gives every CU a block.
    vb = 1;
    for (int c : {4, 2}) {
      if (int64_t(c) * n <= kLdsMaxThreads && blocks(c) >= int64_t(ctx->num_cu)) {
        vb = c;
        break;
      }
    }
  }
  const int t1 = round64(int64_t(vb) * n);
  int split = ctx->proj_split;
  if (split <= 0) {
    // Copies of the ray set up to 1024 threads per block.
    split = 1;
    while (2 * split * t1 <= kLdsMaxThreads) split *= 2;
  }
  while (split > 1 && split * t1 > kLdsMaxThreads) split /= 2;
  const int nt = split * t1;
  const int64_t band =
      std::max<int64_t>(1, std::min<int64_t>({n, kStageFloats / rp, copy_floats_k(K) * nt / (n * K)}));
  L.lds = true;
  L.vb = vb;
  L.split = split;
  L.threads = nt;
  L.rows = int(band);
  L.grid = slot_grid(g->n_slices, int64_t(n_groups) * (kViewGroup / vb));
  L.partials = size_t(blocks(vb));
  L.lds_bytes = sizeof(float) * size_t(std::max<int64_t>(band * rp, split > 1 ? int64_t(nt) * K : 0));
  return L;
}

ProjLaunch plan_backproject(const hsn_ctx *ctx, const hsn_geom *g) {
  ProjLaunch L;
  const int64_t n = g->n_cols, K = g->k, rp = staged_rp(g);
  if (ctx->proj_voxels < 0 || rp > kStageFloats || n * K > copy_floats_k(K) * kLdsMaxThreads) {
    L.threads = kVoxThreads;
    L.grid = backproject_grid(g);
    L.partials = size_t(g->n_slices) * n * ((n + kVoxThreads - 1) / kVoxThreads);
    return L;
  }
  // default block: 512 threads for K = 5 (three blocks per CU, see
  // backproject_lds_kernel), else the largest
  int nt = ctx->proj_threads > 0 ? ctx->proj_threads : (K == 5 ? 512 : kLdsMaxThreads);
  nt = std::max<int>({64, round64((n * K + copy_floats_k(K) - 1) / copy_floats_k(K)), std::min<int>(nt, round64(n * n))});
  nt = std::min(nt, kLdsMaxThreads);
  auto per_slice = [&](int vpt) { return (n * n + int64_t(vpt) * nt - 1) / (int64_t(vpt) * nt); };
  int vpt = ctx->proj_voxels;
  if (vpt <= 0) {
    // Most voxels per thread (fewest sinogram stagings) that still give
    // every CU a block.
    vpt = 1;
    for (int c : {4, 2}) {
      if (int64_t(g->n_slices) * per_slice(c) >= int64_t(ctx->num_cu)) {
        vpt = c;
        break;
      }
    }
  }
  // Several voxels per thread step between rows of one column: the block
  // must span whole image rows.
  if (nt % n != 0) vpt = 1;
  const int64_t vc = std::max<int64_t>(
      1, std::min<int64_t>({int64_t(g->n_views), kStageFloats / rp, int64_t(kMaxViewChunk), int64_t(nt),
                            copy_floats_k(K) * nt / (n * K)}));
  L.lds = true;
  L.vpt = vpt;
  L.threads = nt;
  L.rows = int(vc);
  L.grid = slot_grid(g->n_slices, per_slice(vpt));
  L.partials = size_t(g->n_slices) * per_slice(vpt);
  L.lds_bytes = size_t(geom_stage_bytes(int(vc))) + sizeof(float) * size_t(vc * rp);
  return L;
}

bool aligned16(const void *p) { return reinterpret_cast<uintptr_t>(p) % 16 == 0; }

template <int K>
void launch_project(const ProjLaunch &L, const float *x, const float *xT, float *s, const GeomTab &gt,
                    const hsn_geom *g, float alpha, float beta, double *sumsq, hipStream_t st) {
  const int n = int(g->n_cols);
  if (!L.lds) {
    project_kernel<K><<<L.grid, kRayThreads, 0, st>>>(x, xT, s, gt.views, int(g->n_slices), int(g->n_views), n,
                                                      alpha, beta, sumsq);
    return;
  }
  const bool vec4 = copy_vec(K, n) && aligned16(x) && (!xT || aligned16(xT));
  if (vec4)
    project_lds_kernel<K, true><<<L.grid, L.threads, L.lds_bytes, st>>>(
        x, xT, s, gt.views, gt.groups, gt.n_groups, L.vb, L.split, int(g->n_slices), n, L.rows, alpha, beta, sumsq);
  else
    project_lds_kernel<K, false><<<L.grid, L.threads, L.lds_bytes, st>>>(
        x, xT, s, gt.views, gt.groups, gt.n_groups, L.vb, L.split, int(g->n_slices), n, L.rows, alpha, beta, sumsq);
}

template <int K, int VPT>
void launch_backproject_lds(const ProjLaunch &L, const float *s, float *x, const GeomTab &gt, const hsn_geom *g,
                            float alpha, float beta, double *sumsq, hipStream_t st) {
  const int n = int(g->n_cols);
  const bool vec4 = copy_vec(K, n) && aligned16(s);
  if (vec4)
    backproject_lds_kernel<K, VPT, true><<<L.grid, L.threads, L.lds_bytes, st>>>(
        s, x, gt.views, int(g->n_views), int(g->n_slices), n, L.rows, alpha, beta, sumsq);
  else
    backproject_lds_kernel<K, VPT, false><<<L.grid, L.threads, L.lds_bytes, st>>>(
        s, x, gt.views, int(g->n_views), int(g->n_slices), n, L.rows, alpha, beta, sumsq);
}

template <int K>
void launch_backproject(const ProjLaunch &L, const float *s, float *x, const GeomTab &gt, const hsn_geom *g,
                        float alpha, float beta, double *sumsq, hipStream_t st) {
  if (!L.lds) {
    backproject_kernel<K><<<L.grid, kVoxThreads, 0, st>>>(s, x, gt.views, int(g->n_views), int(g->n_slices),
                                                          int(g->n_cols), alpha, beta, sumsq);
    return;
  }
  switch (L.vpt) {
    case 1: launch_backproject_lds<K, 1>(L, s, x, gt, g, alpha, beta, sumsq, st); break;
    case 2: launch_backproject_lds<K, 2>(L, s, x, gt, g, alpha, beta, sumsq, st); break;
    default: launch_backproject_lds<K, 4>(L, s, x, gt, g, alpha, beta, sumsq, st); break;
  }
}

// mode 0: pT = p^T; mode 1: p = sv + coef p, pT = p^T; mode 2: p = sv, pT = p^T;
// mode 3: the fused CGLS direction step, mode 4: the MBIR one, mode 5: the CGLS one with formed
// scalars (see xpby_transpose_kernel).
template <int K>
void launch_xpby_t(float *p, float *pT, const float *sv, const double *coef, const hsn_geom *g, int mode,
                   hipStream_t st, float *x = nullptr, const double *partial = nullptr, int nblk = 0,
                   double *scal = nullptr, int gsel = 0) {
  const unsigned t = unsigned((g->n_cols + kTile - 1) / kTile);
  xpby_transpose_kernel<K><<<dim3(t, t, unsigned(g->n_slices)), 256, 0, st>>>(p, pT, sv, coef, int(g->n_cols), mode,
                                                                              x, partial, nblk, scal, gsel);
}

// Number of view groups upload_geom forms for g.
int count_groups(const hsn_geom *g) {
  const int nv = int(g->n_views);
  int steep = 0;
  for (int v = 0; v < nv; ++v) {
    const double t = g->angles ? g->angles[v] : double(v) * M_PI / double(nv);
    steep += std::fabs(std::sin(t)) > std::fabs(std::cos(t));
  }
  return (nv - steep + kViewGroup - 1) / kViewGroup + (steep + kViewGroup - 1) / kViewGroup;
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

template <int K>
void launch_prior_apply(const float *xa, const float *v, float *w, const hsn_geom *g, const PriorArgs &pa, float sign,
                        int dot_self, double *partial, hipStream_t st) {
  prior_apply_kernel<K><<<kPriorBlocks, 256, 0, st>>>(xa, v, w, int(g->n_cols), int(g->n_slices), pa, sign, dot_self,
                                                       partial);
}

template <int K>
void launch_mbir_step(float *x, const float *d, float *r, const float *w, const hsn_geom *g, const double *scal,
                      int gsel, const double *partial_dw, double *partial_out, hipStream_t st) {
  const int64_t n_vox = int64_t(g->n_slices) * g->n_cols * g->n_cols;
  mbir_step_kernel<K><<<kDotBlocks, kDotThreads, 0, st>>>(x, d, r, w, n_vox, scal, gsel, partial_dw, kPriorBlocks,
                                                          partial_out);
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
  GeomTab gt{};
  // Steep views read a transposed copy of x (workspace).
  float *xT = nullptr;
  if (has_steep_view(g)) {
    const size_t nxk = size_t(g->n_slices) * g->n_cols * g->n_cols * g->k;
    if ((rc = hsn::ensure_ws(ctx, sizeof(float) * nxk)) != HSN_OK) return rc;
    xT = static_cast<float *>(ctx->ws);
  }
  if ((rc = upload_geom(ctx, g, st, &gt)) != HSN_OK) return rc;
  const ProjLaunch L = plan_project(ctx, g, gt.n_groups);
  if (xT) HSN_DISPATCH_K(g->k, launch_xpby_t, const_cast<float *>(x), xT, nullptr, nullptr, g, 0, st);
  hsn::prof_begin(ctx, HSN_KERN_PROJECT, st);
  HSN_DISPATCH_K(g->k, launch_project, L, x, xT, s, gt, g, alpha, beta, nullptr, st);
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
  GeomTab gt{};
  if ((rc = upload_geom(ctx, g, st, &gt)) != HSN_OK) return rc;
  const ProjLaunch L = plan_backproject(ctx, g);
  hsn::prof_begin(ctx, HSN_KERN_BACKPROJECT, st);
  HSN_DISPATCH_K(g->k, launch_backproject, L, s, x, gt, g, alpha, beta, nullptr, st);
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
  GeomTab gt{};
  if ((rc = upload_geom(ctx, g, st, &gt)) != HSN_OK) return rc;
  const ProjLaunch LA = plan_project(ctx, g, gt.n_groups), LB = plan_backproject(ctx, g);
  const size_t nb_proj = LA.partials, nb_back = LB.partials;
  if (nb_proj >= size_t(INT32_MAX) || nb_back >= size_t(INT32_MAX))
    return hsn::fail(ctx, HSN_ERR_SHAPE, "cgls: geometry too large for one launch");
  const size_t n_part = std::max<size_t>({nb_proj, nb_back, size_t(kDotBlocks)});
  const size_t need = hsn::Carver::need({sizeof(float) * ns * K, sizeof(float) * ns * K, sizeof(float) * nx * K,
                                         sizeof(float) * nx * K, sizeof(float) * nx * K,
                                         sizeof(double) * n_part * K, sizeof(double) * kScal});
  if ((rc = hsn::ensure_ws(ctx, need)) != HSN_OK) return rc;
  hsn::Carver cv(ctx->ws);
  float *r = cv.take<float>(ns * K), *q = cv.take<float>(ns * K);
  float *sv = cv.take<float>(nx * K), *p = cv.take<float>(nx * K), *pT = cv.take<float>(nx * K);
  double *partial = cv.take<double>(n_part * K), *scal = cv.take<double>(kScal);
  const int eb = 256;
  auto blocks = [&](int64_t m) { return unsigned(std::min<int64_t>((m + eb - 1) / eb, 4096)); };
  // With few projector partials every block of the update kernels sums them
  // itself (4 launches per iteration); otherwise one block does and the
  // updates read the scalars (6 launches).
  const bool fused = std::max(nb_proj, nb_back) <= 1024;

  cgls_start_kernel<<<blocks(nx * K + ns * K), eb, 0, st>>>(x, nx * K, r, sino, ns * K);
  hsn::prof_begin(ctx, HSN_KERN_BACKPROJECT, st);
  HSN_DISPATCH_K(K, launch_backproject, LB, r, sv, gt, g, 1.0f, 0.0f, partial, st);
  hsn::prof_end(ctx, HSN_KERN_BACKPROJECT, st);
  cgls_scalar_kernel<<<1, 256, 0, st>>>(partial, int(nb_back), K, kSetGamma, scal, 0, nullptr);
  HSN_DISPATCH_K(K, launch_xpby_t, p, pT, sv, nullptr, g, 2, st);
  if (resid) {
    HSN_DISPATCH_K(K, launch_dot, r, r, ns, partial, st);
    cgls_scalar_kernel<<<1, 256, 0, st>>>(partial, kDotBlocks, K, kResid, scal, 0, resid);
  }
  for (int it = 0; it < n_iter; ++it) {
    const int gsel = it & 1;
    hsn::prof_begin(ctx, HSN_KERN_PROJECT, st);
    HSN_DISPATCH_K(K, launch_project, LA, p, pT, q, gt, g, 1.0f, 0.0f, partial, st);
    hsn::prof_end(ctx, HSN_KERN_PROJECT, st);
    if (fused) {
      cgls_rstep_kernel<<<std::min(blocks(ns * K), 512u), 256, 0, st>>>(r, q, ns * K, K, partial, int(nb_proj), scal,
                                                                        gsel);
    } else {
      cgls_scalar_kernel<<<1, 256, 0, st>>>(partial, int(nb_proj), K, kAlpha, scal, gsel, nullptr);
      // r -= alpha q here; x += alpha p goes with the direction step (mode 5),
      // which reads p anyway
      chan_axpy2_kernel<<<blocks(ns * K), eb, 0, st>>>(x, p, 0, r, q, ns * K, scal + kAlphaOff, K);
    }
    hsn::prof_begin(ctx, HSN_KERN_BACKPROJECT, st);
    HSN_DISPATCH_K(K, launch_backproject, LB, r, sv, gt, g, 1.0f, 0.0f, partial, st);
    hsn::prof_end(ctx, HSN_KERN_BACKPROJECT, st);
    if (fused) {
      HSN_DISPATCH_K(K, launch_xpby_t, p, pT, sv, nullptr, g, 3, st, x, partial, int(nb_back), scal, gsel);
    } else {
      cgls_scalar_kernel<<<1, 256, 0, st>>>(partial, int(nb_back), K, kBeta, scal, gsel, nullptr);
      HSN_DISPATCH_K(K, launch_xpby_t, p, pT, sv, nullptr, g, 5, st, x, nullptr, 0, scal, gsel);
    }
    if (resid) {
      HSN_DISPATCH_K(K, launch_dot, r, r, ns, partial, st);
      cgls_scalar_kernel<<<1, 256, 0, st>>>(partial, kDotBlocks, K, kResid, scal, 0, resid + size_t(it + 1) * K);
    }
  }
  // Both paths add alpha p to x in the direction step, which the last
  // iteration still runs; nothing is left to add here.
  HSN_LAUNCHED(ctx);
  return HSN_OK;
}

extern "C" hsn_status hsn_mbir(hsn_ctx *ctx, const hsn_geom *g, const float *sino, float *x, const double *sigma_v,
                               const double *sigma_x, double p, double T, int n_outer, int n_inner, void *stream) {
  if (!ctx) return HSN_ERR_INVALID_ARG;
  hsn_status rc = check_geom(ctx, g);
  if (rc != HSN_OK) return rc;
  if (!sino || !x || !sigma_v || !sigma_x)
    return hsn::fail(ctx, HSN_ERR_INVALID_ARG, "mbir: sino, x, sigma_v and sigma_x are required");
  if (n_outer < 0 || n_inner < 0) return hsn::fail(ctx, HSN_ERR_INVALID_ARG, "mbir: iteration counts must be >= 0");
  if (!(p >= 1.0 && p <= 2.0)) return hsn::fail(ctx, HSN_ERR_INVALID_ARG, "mbir: p must be in [1, 2] (got %g)", p);
  if (!(T > 0.0) || !std::isfinite(T)) return hsn::fail(ctx, HSN_ERR_INVALID_ARG, "mbir: T must be > 0");
  const int K = g->k;
  PriorArgs pa{};
  for (int q = 0; q < K; ++q) {
    if (!(sigma_v[q] > 0.0) || !(sigma_x[q] > 0.0) || !std::isfinite(sigma_v[q]) || !std::isfinite(sigma_x[q]))
      return hsn::fail(ctx, HSN_ERR_INVALID_ARG, "mbir: sigma_v[%d] and sigma_x[%d] must be finite and > 0", q, q);
    pa.c0[q] = float(1.0 / (2.0 * sigma_x[q] * sigma_x[q] * std::pow(T, 2.0 - p)));
    pa.inv_tsx[q] = float(1.0 / (T * sigma_x[q]));
    pa.s2[q] = float(sigma_v[q] * sigma_v[q]);
  }
  pa.e = float(2.0 - p);
  pa.rq = float((2.0 - p) / p);
  if ((rc = check_align(ctx, x, K, "x")) != HSN_OK || (rc = check_align(ctx, sino, K, "sino")) != HSN_OK) return rc;
  hsn::DeviceGuard dg(ctx->device);
  hipStream_t st = static_cast<hipStream_t>(stream);
  const int64_t n = g->n_cols;
  const int64_t nx = g->n_slices * n * n;           // voxels
  const int64_t ns = g->n_views * g->n_slices * n;  // rays
  GeomTab gt{};
  if ((rc = upload_geom(ctx, g, st, &gt)) != HSN_OK) return rc;
  const ProjLaunch LA = plan_project(ctx, g, gt.n_groups), LB = plan_backproject(ctx, g);
  const size_t n_part = std::max<size_t>(kPriorBlocks, kDotBlocks);
  const size_t need = hsn::Carver::need({sizeof(float) * ns * K, sizeof(float) * nx * K, sizeof(float) * nx * K,
                                         sizeof(float) * nx * K, sizeof(float) * nx * K, sizeof(float) * nx * K,
                                         sizeof(float) * nx * K, sizeof(double) * n_part * K,
                                         sizeof(double) * kDotBlocks * K, sizeof(double) * kScal});
  if ((rc = hsn::ensure_ws(ctx, need)) != HSN_OK) return rc;
  hsn::Carver cv(ctx->ws);
  float *s = cv.take<float>(ns * K);
  float *xa = cv.take<float>(nx * K), *xT = cv.take<float>(nx * K), *r = cv.take<float>(nx * K);
  float *d = cv.take<float>(nx * K), *dT = cv.take<float>(nx * K), *w = cv.take<float>(nx * K);
  double *partial = cv.take<double>(n_part * K), *partial_rr = cv.take<double>(kDotBlocks * K);
  double *scal = cv.take<double>(kScal);

  for (int outer = 0; outer < n_outer; ++outer) {
    // Anchor x' = x; r = A^T (V - A x) - sigma_v^2 L x; d = r; gamma = <r, r>.
    copy2_kernel<<<unsigned(std::min<int64_t>((nx * K + ns * K + 255) / 256, 4096)), 256, 0, st>>>(
        xa, x, nx * K, s, sino, ns * K);
    HSN_DISPATCH_K(K, launch_xpby_t, x, xT, nullptr, nullptr, g, 0, st);
    hsn::prof_begin(ctx, HSN_KERN_PROJECT, st);
    HSN_DISPATCH_K(K, launch_project, LA, x, xT, s, gt, g, -1.0f, 1.0f, nullptr, st);
    hsn::prof_end(ctx, HSN_KERN_PROJECT, st);
    hsn::prof_begin(ctx, HSN_KERN_BACKPROJECT, st);
    HSN_DISPATCH_K(K, launch_backproject, LB, s, r, gt, g, 1.0f, 0.0f, nullptr, st);
    hsn::prof_end(ctx, HSN_KERN_BACKPROJECT, st);
    HSN_DISPATCH_K(K, launch_prior_apply, xa, x, r, g, pa, -1.0f, 1, partial, st);
    cgls_scalar_kernel<<<1, 256, 0, st>>>(partial, kPriorBlocks, K, kSetGamma, scal, 0, nullptr);
    HSN_DISPATCH_K(K, launch_xpby_t, d, dT, r, nullptr, g, 2, st);
    for (int it = 0; it < n_inner; ++it) {
      const int gsel = it & 1;
      // w = (A^T A + sigma_v^2 L) d; alpha = gamma / <d, w>
      hsn::prof_begin(ctx, HSN_KERN_PROJECT, st);
      HSN_DISPATCH_K(K, launch_project, LA, d, dT, s, gt, g, 1.0f, 0.0f, nullptr, st);
      hsn::prof_end(ctx, HSN_KERN_PROJECT, st);
      hsn::prof_begin(ctx, HSN_KERN_BACKPROJECT, st);
      HSN_DISPATCH_K(K, launch_backproject, LB, s, w, gt, g, 1.0f, 0.0f, nullptr, st);
      hsn::prof_end(ctx, HSN_KERN_BACKPROJECT, st);
      HSN_DISPATCH_K(K, launch_prior_apply, xa, d, w, g, pa, 1.0f, 0, partial, st);
      // x += alpha d; r -= alpha w (alpha from the <d, w> partials); then
      // beta = <r, r> / gamma and d = r + beta d (from the <r, r> partials)
      HSN_DISPATCH_K(K, launch_mbir_step, x, d, r, w, g, scal, gsel, partial, partial_rr, st);
      HSN_DISPATCH_K(K, launch_xpby_t, d, dT, r, nullptr, g, 4, st, nullptr, partial_rr, kDotBlocks, scal, gsel);
    }
  }
  HSN_LAUNCHED(ctx);
  return HSN_OK;
}

extern "C" hsn_status hsn_projector_set_launch(hsn_ctx *ctx, int views, int split, int voxels, int threads) {
  if (!ctx) return HSN_ERR_INVALID_ARG;
  if (!(views == -1 || views == 0 || views == 1 || views == 2 || views == 4))
    return hsn::fail(ctx, HSN_ERR_INVALID_ARG, "projector launch: views must be -1, 0, 1, 2 or 4 (got %d)", views);
  if (!(split == 0 || split == 1 || split == 2 || split == 4 || split == 8 || split == 16))
    return hsn::fail(ctx, HSN_ERR_INVALID_ARG, "projector launch: split must be 0, 1, 2, 4, 8 or 16 (got %d)", split);
  if (!(voxels == -1 || voxels == 0 || voxels == 1 || voxels == 2 || voxels == 4))
    return hsn::fail(ctx, HSN_ERR_INVALID_ARG, "projector launch: voxels must be -1, 0, 1, 2 or 4 (got %d)", voxels);
  if (!(threads == 0 || threads == 64 || threads == 128 || threads == 256 || threads == 512 || threads == 1024))
    return hsn::fail(ctx, HSN_ERR_INVALID_ARG, "projector launch: threads must be 0 or 64..1024, a power of 2 (got %d)",
                     threads);
  ctx->proj_views = views;
  ctx->proj_split = split;
  ctx->proj_voxels = voxels;
  ctx->proj_threads = threads;
  return HSN_OK;
}

extern "C" hsn_status hsn_projector_launch_info(hsn_ctx *ctx, const hsn_geom *g, int *shape) {
  if (!ctx) return HSN_ERR_INVALID_ARG;
  hsn_status rc = check_geom(ctx, g);
  if (rc != HSN_OK) return rc;
  if (!shape) return hsn::fail(ctx, HSN_ERR_INVALID_ARG, "projector launch info: shape is NULL");
  const ProjLaunch LA = plan_project(ctx, g, count_groups(g)), LB = plan_backproject(ctx, g);
  shape[0] = LA.lds ? LA.vb : 0;
  shape[1] = LA.lds ? LA.split : 0;
  shape[2] = LB.lds ? LB.vpt : 0;
  shape[3] = LB.lds ? LB.threads : 0;
  return HSN_OK;
}

extern "C" hsn_status hsn_fbp(hsn_ctx *ctx, const hsn_geom *g, const float *sino, int64_t ld, float *x, void *stream) {
  if (!ctx) return HSN_ERR_INVALID_ARG;
  hsn_status rc = check_geom(ctx, g);
  if (rc != HSN_OK) return rc;
  if (!sino || !x) return hsn::fail(ctx, HSN_ERR_INVALID_ARG, "fbp: sino and x are required");
  if (ld < g->k) return hsn::fail(ctx, HSN_ERR_INVALID_ARG, "fbp: ld must be >= k");
  if (g->n_cols * g->k > kFbpMaxFloats)
    return hsn::fail(ctx, HSN_ERR_SHAPE, "fbp: n_cols * k must be <= %d", kFbpMaxFloats);
  if (reinterpret_cast<uintptr_t>(sino) % 4 != 0) return hsn::fail(ctx, HSN_ERR_INVALID_ARG, "fbp: sino not 4-byte aligned");
  if ((rc = check_align(ctx, x, g->k, "x")) != HSN_OK) return rc;
  hsn::DeviceGuard dg(ctx->device);
  hipStream_t st = static_cast<hipStream_t>(stream);
  const int64_t ns = g->n_views * g->n_slices * g->n_cols;
  if ((rc = hsn::ensure_ws(ctx, sizeof(float) * size_t(ns) * g->k)) != HSN_OK) return rc;
  float *q = static_cast<float *>(ctx->ws);
  GeomTab gt{};
  if ((rc = upload_geom(ctx, g, st, &gt)) != HSN_OK) return rc;
  const ProjLaunch LB = plan_backproject(ctx, g);
  hsn::prof_begin(ctx, HSN_KERN_FBP_FILTER, st);
  HSN_DISPATCH_K(g->k, launch_ramp, sino, ld, g, q, st);
  hsn::prof_end(ctx, HSN_KERN_FBP_FILTER, st);
  const float scale = float(M_PI / double(g->n_views));
  hsn::prof_begin(ctx, HSN_KERN_BACKPROJECT, st);
  HSN_DISPATCH_K(g->k, launch_backproject, LB, q, x, gt, g, scale, 0.0f, nullptr, st);
  hsn::prof_end(ctx, HSN_KERN_BACKPROJECT, st);
  HSN_LAUNCHED(ctx);
  return HSN_OK;
}
