// -log normalisation (eq. 2) with the Appendix A offset correction.
//
//   p = -ln( max(y, f) / max(y^o, f) ) - b[v][k],  optionally clipped at 0,
//   b[v][k] = mean over background pixels B of the unclipped -ln(y / y^o).
//
// One HBM stream: counts in, float32 p and (optionally) its bfloat16 copy
// out, with per-block float64 partials of sum(p^2) (and, with the bfloat16
// copy, of -sum((p - bf16(p))^2)) reduced in a fixed order.
#include "common.hpp"

#include <mutex>

namespace {

constexpr int kThreads = 256;
constexpr int kSumBlocks = 2048;  // fixed grid so that the sum(p^2) order is fixed

template <typename T>
__device__ __forceinline__ float ld_count(const T *a, int64_t i);
template <>
__device__ __forceinline__ float ld_count<uint16_t>(const uint16_t *a, int64_t i) { return float(a[i]); }
template <>
__device__ __forceinline__ float ld_count<float>(const float *a, int64_t i) { return a[i]; }

// -ln(y/y^o) evaluated as ln(y^o/y) = log2(y^o / y) ln 2 with the hardware
// reciprocal and log2, each within about 1 ulp: a few 1e-7 relative.  A
// ratio below the float32 normal range (2^-126, counts ratios no detector
// produces; never for uint16 counts with f >= 1) would flush to -inf.
__device__ __forceinline__ float neglog(float y, float yo, float floor_) {
  const float ratio = fmaxf(yo, floor_) * __builtin_amdgcn_rcpf(fmaxf(y, floor_));
  return __builtin_amdgcn_logf(ratio) * 0.69314718055994531f;
}

// p - b rounded on its own, never fused with the log's scaling, so that
// every kernel gives the same bits.
__device__ __forceinline__ float sub_offset(float pv, float bv) {
#pragma clang fp contract(off)
  return pv - bv;
}

// b[v][k] = (1/|B|) sum_{(r,c) in B} -ln(y/y^o).  Grid (k-blocks, N_v);
// each thread walks the pixels in order, so the sum is deterministic.
template <typename TY, typename TO>
__global__ __launch_bounds__(kThreads) void offset_kernel(const TY *__restrict__ y, const TO *__restrict__ yo,
                                                          const uint8_t *__restrict__ mask, int64_t n_pix,
                                                          int64_t nk, float floor_, float *__restrict__ b) {
  const int64_t k = int64_t(blockIdx.x) * kThreads + threadIdx.x;
  const int64_t v = blockIdx.y;
  if (k >= nk) return;
  double acc = 0.0;
  int64_t cnt = 0;
  for (int64_t px = 0; px < n_pix; ++px) {
    if (!mask[px]) continue;
    const float pv = neglog(ld_count(y, (v * n_pix + px) * nk + k), ld_count(yo, px * nk + k), floor_);
    acc += double(pv);
    ++cnt;
  }
  b[v * nk + k] = float(acc / double(cnt > 0 ? cnt : 1));
}

// Average pooling of a row to the 256 network inputs: input i covers bins
// [floor(i N_k / 256), ceil((i + 1) N_k / 256)) of the bfloat16-rounded p,
// summed in bin order in float32 and divided by the bin count (the
// arithmetic of the learned start's own pooling of p_bf16).
constexpr int kPoolIn = 256;
constexpr int kPoolMaxBins = 2048;

// Main stream.  A group is R = max(1, 256 / cpr) consecutive detector
// pixels of one view, cpr = ceil(width / 8) chunks of 8 bins per row;
// thread t takes pixel t / cpr of the group and chunk t % cpr (rows longer
// than 2048 bins: one row per group, chunks t, t + 256, ...).  A block walks
// units u = blockIdx.x, + gridDim.x, ...: unit u is pixel group u / n_ch and
// views [vc c, vc c + vc) with c = u % n_ch, taken view by view, so that
// the open-beam row y^o of a pixel is read once per unit instead of once per
// view.  POOL (1: bfloat16 out, 2: float32 out) also writes the pooled rows,
// from a copy of the group's bfloat16-rounded rows in LDS (R * N_k <= 2048
// floats).
template <typename TY, typename TO, bool VEC, int POOL>
__global__ __launch_bounds__(kThreads) void normalize_kernel(
    const TY *__restrict__ y, const TO *__restrict__ yo, int64_t n_v, int64_t vc, int64_t n_pix, int64_t nk,
    const float *__restrict__ b, float floor_, int clip, float *__restrict__ p, int64_t ldp,
    uint16_t *__restrict__ pb, int64_t ldb, void *__restrict__ pooled, double *__restrict__ partial) {
  __shared__ float rowbuf[POOL ? kPoolMaxBins : 1];
  const int width = int((pb && ldb > nk) ? ldb : nk);
  const int cpr = (width + 7) / 8;
  const int R = cpr <= kThreads ? kThreads / cpr : 1;
  const int t = threadIdx.x;
  const int rr = cpr <= kThreads ? t / cpr : 0;
  const int ch0 = cpr <= kThreads ? t - rr * cpr : t;
  const int nki = int(nk);
  double ss = 0.0, sb = 0.0;
  const int64_t n_pg = (n_pix + R - 1) / R, n_ch = (n_v + vc - 1) / vc;
  for (int64_t u = blockIdx.x; u < n_pg * n_ch; u += gridDim.x) {
   const int64_t pg = u / n_ch, v0 = (u - pg * n_ch) * vc;
   const int64_t v1 = v0 + vc < n_v ? v0 + vc : n_v;
   const int64_t px = pg * R + rr;
   const bool row_ok = rr < R && px < n_pix;
   for (int64_t v = v0; v < v1; ++v) {
    const int64_t row = v * n_pix + px;
    for (int ch = ch0; row_ok && ch < cpr; ch += kThreads) {
      const int k0 = ch * 8;
      float out[8];
      if (VEC && k0 + 8 <= nki) {
        // 16-byte loads of 8 uint16 counts (alignment checked on the host).
        const uint4 yv = *reinterpret_cast<const uint4 *>(reinterpret_cast<const uint16_t *>(y) + row * nk + k0);
        const uint4 ov = *reinterpret_cast<const uint4 *>(reinterpret_cast<const uint16_t *>(yo) + px * nk + k0);
        const uint32_t yw[4] = {yv.x, yv.y, yv.z, yv.w};
        const uint32_t ow[4] = {ov.x, ov.y, ov.z, ov.w};
#pragma unroll
        for (int e = 0; e < 8; ++e) {
          const float yc = float((yw[e >> 1] >> (16 * (e & 1))) & 0xFFFFu);
          const float oc = float((ow[e >> 1] >> (16 * (e & 1))) & 0xFFFFu);
          out[e] = neglog(yc, oc, floor_);
        }
      } else {
#pragma unroll
        for (int e = 0; e < 8; ++e) {
          const int k = k0 + e;
          out[e] = (k < nki) ? neglog(ld_count(y, row * nk + k), ld_count(yo, px * nk + k), floor_) : 0.0f;
        }
      }
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const int k = k0 + e;
        float pv = out[e];
        if (k < nki) {
          if (b) pv = sub_offset(pv, b[v * nk + k]);
          if (clip) pv = fmaxf(pv, 0.0f);
        } else {
          pv = 0.0f;
        }
        out[e] = pv;
        ss += double(pv) * double(pv);
        if (pb) {
          const double e = double(pv) - double(hsn::bf16_bits_to_f32(hsn::f32_to_bf16_bits(pv)));
          sb -= e * e;
        }
      }
      if (p) {
        if (VEC && k0 + 8 <= nki) {
          float4 *dst = reinterpret_cast<float4 *>(p + row * ldp + k0);
          dst[0] = make_float4(out[0], out[1], out[2], out[3]);
          dst[1] = make_float4(out[4], out[5], out[6], out[7]);
        } else {
          for (int e = 0; e < 8; ++e)
            if (k0 + e < nki) p[row * ldp + k0 + e] = out[e];
        }
      }
      if (pb) {
        if (VEC && k0 + 8 <= ldb) {
          uint32_t w[4];
#pragma unroll
          for (int e = 0; e < 4; ++e)
            w[e] = uint32_t(hsn::f32_to_bf16_bits(out[2 * e])) | (uint32_t(hsn::f32_to_bf16_bits(out[2 * e + 1])) << 16);
          *reinterpret_cast<uint4 *>(pb + row * ldb + k0) = make_uint4(w[0], w[1], w[2], w[3]);
        } else {
          for (int e = 0; e < 8; ++e)
            if (k0 + e < ldb) pb[row * ldb + k0 + e] = hsn::f32_to_bf16_bits(out[e]);
        }
      }
      if constexpr (POOL != 0) {
#pragma unroll
        for (int e = 0; e < 8; ++e)
          if (k0 + e < nki) rowbuf[rr * nki + k0 + e] = hsn::bf16_bits_to_f32(hsn::f32_to_bf16_bits(out[e]));
      }
    }
    if constexpr (POOL != 0) {
      __syncthreads();
      for (int o = t; o < R * kPoolIn; o += kThreads) {
        const int orow = o / kPoolIn, i = o - orow * kPoolIn;
        if (pg * R + orow >= n_pix) continue;
        const int64_t prow = v * n_pix + pg * R + orow;
        const int lo = (i * nki) / kPoolIn, hi = ((i + 1) * nki + kPoolIn - 1) / kPoolIn;
        float sum = 0.0f;
        for (int c = lo; c < hi; ++c) sum += rowbuf[orow * nki + c];
        const float val = sum / float(hi - lo);
        if constexpr (POOL == 1)
          static_cast<uint16_t *>(pooled)[prow * kPoolIn + i] = hsn::f32_to_bf16_bits(val);
        else
          static_cast<float *>(pooled)[prow * kPoolIn + i] = val;
      }
      __syncthreads();
    }
   }
  }
  // Block reduction of the float64 sum of squares, fixed order.
  __shared__ double red[2][kThreads / 64];
  ss = hsn::wave_sum_all(ss);
  sb = hsn::wave_sum_all(sb);
  if ((threadIdx.x & 63) == 0) {
    red[0][threadIdx.x >> 6] = ss;
    red[1][threadIdx.x >> 6] = sb;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double tt = 0.0, tb = 0.0;
    for (int w = 0; w < kThreads / 64; ++w) {
      tt += red[0][w];
      tb += red[1][w];
    }
    partial[blockIdx.x] = tt;
    partial[kSumBlocks + blockIdx.x] = tb;
  }
}

// Fast path for uint16 counts whose rows split into whole 8-bin chunks
// (n_k % 8 == 0, n_k <= 2048, 16-byte aligned rows, p present, p_bf16 absent
// or 16-byte aligned, its row at most 2048 wide): one chunk per thread per
// row, straight-line code with the options fixed at compile time, and the
// open-beam chunk kept in registers across the unit's views.  Same values,
// the same units per block and the same summation order as normalize_kernel
// (bitwise equal outputs).
template <int POOL, bool HAS_B, bool HAS_PB>
__global__ __launch_bounds__(kThreads) void normalize_u16_kernel(
    const uint16_t *__restrict__ y, const uint16_t *__restrict__ yo, int64_t n_v, int64_t vc, int64_t n_pix, int nk,
    const float *__restrict__ b, float floor_, int clip, float *__restrict__ p, int64_t ldp,
    uint16_t *__restrict__ pb, int64_t ldb, void *__restrict__ pooled, double *__restrict__ partial) {
  __shared__ __attribute__((aligned(16))) float rowbuf[POOL ? kPoolMaxBins : 4];
  // Thread t takes chunk t % cpw of row t / cpw of the group, cpw = the
  // chunks of the widest output row (the padded bfloat16 row when there is
  // one), as normalize_kernel does; chunks past the bins only zero the pad.
  const int cpr = nk >> 3;
  const int cpw = HAS_PB ? int(ldb >> 3) : cpr;
  const int R = kThreads / cpw;
  const int t = threadIdx.x;
  const int rr = t / cpw, k0 = (t - rr * cpw) * 8;
  double ss = 0.0, sb = 0.0;
  const int64_t n_pg = (n_pix + R - 1) / R, n_ch = (n_v + vc - 1) / vc;
  for (int64_t u = blockIdx.x; u < n_pg * n_ch; u += gridDim.x) {
   const int64_t pg = u / n_ch, v0 = (u - pg * n_ch) * vc;
   const int64_t v1 = v0 + vc < n_v ? v0 + vc : n_v;
   const int64_t px = pg * R + rr;
   const bool ok = rr < R && px < n_pix;
   uint4 ov = make_uint4(0, 0, 0, 0);
   if (ok && k0 < nk) ov = *reinterpret_cast<const uint4 *>(yo + px * nk + k0);
   for (int64_t v = v0; v < v1; ++v) {
    const int64_t row = v * n_pix + px;
    if (HAS_PB && ok && k0 >= nk)
      *reinterpret_cast<uint4 *>(pb + row * ldb + k0) = make_uint4(0, 0, 0, 0);
    if (ok && k0 < nk) {
      const uint4 yv = *reinterpret_cast<const uint4 *>(y + row * nk + k0);
      const uint32_t yw[4] = {yv.x, yv.y, yv.z, yv.w};
      const uint32_t ow[4] = {ov.x, ov.y, ov.z, ov.w};
      float out[8];
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const float yc = float((yw[e >> 1] >> (16 * (e & 1))) & 0xFFFFu);
        const float oc = float((ow[e >> 1] >> (16 * (e & 1))) & 0xFFFFu);
        float pv = neglog(yc, oc, floor_);
        if constexpr (HAS_B) pv = sub_offset(pv, b[v * nk + k0 + e]);
        if (clip) pv = fmaxf(pv, 0.0f);
        out[e] = pv;
        ss += double(pv) * double(pv);
        if constexpr (HAS_PB) {
          const double e = double(pv) - double(hsn::bf16_bits_to_f32(hsn::f32_to_bf16_bits(pv)));
          sb -= e * e;
        }
      }
      float4 *dst = reinterpret_cast<float4 *>(p + row * ldp + k0);
      dst[0] = make_float4(out[0], out[1], out[2], out[3]);
      dst[1] = make_float4(out[4], out[5], out[6], out[7]);
      if constexpr (HAS_PB) {
        uint32_t w[4];
#pragma unroll
        for (int e = 0; e < 4; ++e)
          w[e] = uint32_t(hsn::f32_to_bf16_bits(out[2 * e])) | (uint32_t(hsn::f32_to_bf16_bits(out[2 * e + 1])) << 16);
        *reinterpret_cast<uint4 *>(pb + row * ldb + k0) = make_uint4(w[0], w[1], w[2], w[3]);
      }
      if constexpr (POOL != 0) {
#pragma unroll
        for (int e = 0; e < 8; ++e) out[e] = hsn::bf16_bits_to_f32(hsn::f32_to_bf16_bits(out[e]));
        // two 16-byte stores per chunk (eight 4-byte stores 32 bytes apart
        // across the lanes fall on the same banks)
        float4 *rb = reinterpret_cast<float4 *>(rowbuf + rr * nk + k0);
        rb[0] = make_float4(out[0], out[1], out[2], out[3]);
        rb[1] = make_float4(out[4], out[5], out[6], out[7]);
      }
    }
    if constexpr (POOL != 0) {
      __syncthreads();
      for (int o = t; o < R * kPoolIn; o += kThreads) {
        const int orow = o / kPoolIn, i = o - orow * kPoolIn;
        if (pg * R + orow >= n_pix) continue;
        const int64_t prow = v * n_pix + pg * R + orow;
        const int lo = (i * nk) / kPoolIn, hi = ((i + 1) * nk + kPoolIn - 1) / kPoolIn;
        float sum = 0.0f;
        for (int c = lo; c < hi; ++c) sum += rowbuf[orow * nk + c];
        const float val = sum / float(hi - lo);
        if constexpr (POOL == 1)
          static_cast<uint16_t *>(pooled)[prow * kPoolIn + i] = hsn::f32_to_bf16_bits(val);
        else
          static_cast<float *>(pooled)[prow * kPoolIn + i] = val;
      }
      __syncthreads();
    }
   }
  }
  __shared__ double red[2][kThreads / 64];
  ss = hsn::wave_sum_all(ss);
  sb = hsn::wave_sum_all(sb);
  if ((threadIdx.x & 63) == 0) {
    red[0][threadIdx.x >> 6] = ss;
    red[1][threadIdx.x >> 6] = sb;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double tt = 0.0, tb = 0.0;
    for (int w = 0; w < kThreads / 64; ++w) {
      tt += red[0][w];
      tb += red[1][w];
    }
    partial[blockIdx.x] = tt;
    partial[kSumBlocks + blockIdx.x] = tb;
  }
}

template <int POOL>
void launch_norm_u16(int64_t n_v, int64_t vc, int64_t n_pix, int64_t nk, const uint16_t *y, const uint16_t *yo, const float *b,
                     float floor_, int clip, float *p, int64_t ldp, uint16_t *pb, int64_t ldb, void *pooled,
                     double *partial, hipStream_t st) {
#define HSN_NORM16(B, PB)                                                                                    \
  normalize_u16_kernel<POOL, B, PB><<<kSumBlocks, kThreads, 0, st>>>(y, yo, n_v, vc, n_pix, int(nk), b, floor_, \
                                                                     clip, p, ldp, pb, ldb, pooled, partial)
  if (b) {
    if (pb) HSN_NORM16(true, true); else HSN_NORM16(true, false);
  } else {
    if (pb) HSN_NORM16(false, true); else HSN_NORM16(false, false);
  }
#undef HSN_NORM16
}

__global__ void sum_partials_kernel(const double *__restrict__ partial, int n, double *__restrict__ out) {
  __shared__ double red[kThreads / 64];
  double t = 0.0;
  for (int i = threadIdx.x; i < n; i += kThreads) t += partial[i];
  t = hsn::wave_sum_all(t);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = t;
  __syncthreads();
  if (threadIdx.x == 0) {
    double s = 0.0;
    for (int w = 0; w < kThreads / 64; ++w) s += red[w];
    *out = s;
  }
}

template <typename TY, typename TO, bool VEC, int POOL>
void launch_norm(int64_t n_v, int64_t vc, int64_t n_pix, int64_t nk, const TY *y, const TO *yo, const float *b, float floor_,
                 int clip, float *p, int64_t ldp, uint16_t *pb, int64_t ldb, void *pooled, double *partial,
                 hipStream_t st) {
  normalize_kernel<TY, TO, VEC, POOL><<<kSumBlocks, kThreads, 0, st>>>(y, yo, n_v, vc, n_pix, nk, b, floor_, clip, p,
                                                                       ldp, pb, ldb, pooled, partial);
}

// scratch: 2 kSumBlocks doubles of per-block partials, and (when the offset
// is computed but not returned) N_v N_k floats for b; null: taken from the
// context's workspace.  With scratch given nothing is allocated and no
// profiling events are recorded.
template <typename TY, typename TO>
hsn_status launch_all(hsn_ctx *ctx, const hsn_dims *d, const TY *y, const TO *yo, const uint8_t *mask,
                      float floor_, int clip, float *p, int64_t ldp, uint16_t *pb, int64_t ldb,
                      float *offset_b, double *sumsq, double *bf16_bias, void *pooled, int pool_mode,
                      hipStream_t st, double *scratch = nullptr) {
  const int64_t n_pix = d->n_rows * d->n_cols;
  const int64_t n_v = d->n_views;
  // Views per unit: all of them while the pixel groups alone give every
  // block at least 8 units, else fewer (the units' count is n_pg n_ch).
  const int64_t width = (pb && ldb > d->n_bins) ? ldb : d->n_bins;
  const int64_t cpr = (width + 7) / 8;
  const int64_t R = cpr <= kThreads ? kThreads / cpr : 1;
  const int64_t n_pg = (n_pix + R - 1) / R;
  const int64_t want_ch = (8 * int64_t(kSumBlocks) + n_pg - 1) / n_pg;
  const int64_t n_ch = want_ch < 1 ? 1 : (want_ch > n_v ? n_v : want_ch);
  const int64_t vc = (n_v + n_ch - 1) / n_ch;
  const int64_t nk = d->n_bins;
  double *partial = scratch;
  float *b = nullptr;
  float *b_scratch = nullptr;
  if (!scratch) {
    size_t need = hsn::Carver::need({sizeof(double) * 2 * kSumBlocks, mask ? sizeof(float) * d->n_views * nk : 0});
    hsn_status s = hsn::ensure_ws(ctx, need);
    if (s != HSN_OK) return s;
    hsn::Carver cv(ctx->ws);
    partial = cv.take<double>(2 * kSumBlocks);
    if (mask && !offset_b) b_scratch = cv.take<float>(d->n_views * nk);
  }
  if (mask) {
    b = offset_b ? offset_b : b_scratch;
    dim3 grid(unsigned((nk + kThreads - 1) / kThreads), unsigned(d->n_views));
    offset_kernel<TY, TO><<<grid, kThreads, 0, st>>>(y, yo, mask, n_pix, nk, floor_, b);
    HSN_LAUNCHED(ctx);
  }
  const bool vec = std::is_same<TY, uint16_t>::value && std::is_same<TO, uint16_t>::value && nk % 8 == 0 &&
                   (reinterpret_cast<uintptr_t>(y) % 16 == 0) && (reinterpret_cast<uintptr_t>(yo) % 16 == 0) &&
                   (!p || (ldp % 4 == 0 && reinterpret_cast<uintptr_t>(p) % 16 == 0)) &&
                   (!pb || reinterpret_cast<uintptr_t>(pb) % 16 == 0);
  if (!scratch) hsn::prof_begin(ctx, HSN_KERN_NORMALIZE, st);
#define HSN_NORM(V, P) launch_norm<TY, TO, V, P>(n_v, vc, n_pix, nk, y, yo, b, floor_, clip, p, ldp, pb, ldb, pooled, partial, st)
  bool fast = false;
  if constexpr (std::is_same<TY, uint16_t>::value && std::is_same<TO, uint16_t>::value) {
    fast = vec && p && nk <= kPoolMaxBins && (!pb || ldb <= 8 * kThreads);
    if (fast) {
      if (pool_mode == 0)
        launch_norm_u16<0>(n_v, vc, n_pix, nk, y, yo, b, floor_, clip, p, ldp, pb, ldb, pooled, partial, st);
      else if (pool_mode == 1)
        launch_norm_u16<1>(n_v, vc, n_pix, nk, y, yo, b, floor_, clip, p, ldp, pb, ldb, pooled, partial, st);
      else
        launch_norm_u16<2>(n_v, vc, n_pix, nk, y, yo, b, floor_, clip, p, ldp, pb, ldb, pooled, partial, st);
    }
  }
  if (!fast && vec) {
    if (pool_mode == 0) HSN_NORM(true, 0); else if (pool_mode == 1) HSN_NORM(true, 1); else HSN_NORM(true, 2);
  } else if (!fast) {
    if (pool_mode == 0) HSN_NORM(false, 0); else if (pool_mode == 1) HSN_NORM(false, 1); else HSN_NORM(false, 2);
  }
#undef HSN_NORM
  if (!scratch) hsn::prof_end(ctx, HSN_KERN_NORMALIZE, st);
  HSN_LAUNCHED(ctx);
  if (sumsq) {
    sum_partials_kernel<<<1, kThreads, 0, st>>>(partial, kSumBlocks, sumsq);
    HSN_LAUNCHED(ctx);
  }
  if (bf16_bias) {
    sum_partials_kernel<<<1, kThreads, 0, st>>>(partial + kSumBlocks, kSumBlocks, bf16_bias);
    HSN_LAUNCHED(ctx);
  }
  return HSN_OK;
}

}  // namespace

static hsn_status normalize_impl(hsn_ctx *ctx, const hsn_dims *d, const void *y, int y_dtype, const void *y_open,
                          int y_open_dtype, const uint8_t *bg_mask, float count_floor, int clip_nonneg, float *p,
                          int64_t ldp, uint16_t *p_bf16, int64_t ldb, float *offset_b, double *sumsq,
                          double *bf16_bias, void *pooled, int pool_mode, void *stream,
                          double *(*scratch_of)(hsn_ctx *) = nullptr) {
  if (!ctx) return HSN_ERR_INVALID_ARG;
  if (!d || !y || !y_open) return hsn::fail(ctx, HSN_ERR_INVALID_ARG, "normalize: dims, y and y_open are required");
  if (!p && !p_bf16 && !pooled)
    return hsn::fail(ctx, HSN_ERR_INVALID_ARG, "normalize: at least one of p, p_bf16, pooled is required");
  if (pooled && d && d->n_bins > kPoolMaxBins)
    return hsn::fail(ctx, HSN_ERR_SHAPE, "normalize: pooled output needs n_bins <= %d", kPoolMaxBins);
  if (d->n_views <= 0 || d->n_rows <= 0 || d->n_cols <= 0 || d->n_bins <= 0)
    return hsn::fail(ctx, HSN_ERR_SHAPE, "normalize: all dimensions must be positive");
  if ((y_dtype != HSN_U16 && y_dtype != HSN_F32) || (y_open_dtype != HSN_U16 && y_open_dtype != HSN_F32))
    return hsn::fail(ctx, HSN_ERR_INVALID_ARG, "normalize: dtype must be HSN_U16 or HSN_F32");
  if (p && ldp < d->n_bins) return hsn::fail(ctx, HSN_ERR_INVALID_ARG, "normalize: ldp < n_bins");
  if (p_bf16 && (ldb < d->n_bins || ldb % 32 != 0 || reinterpret_cast<uintptr_t>(p_bf16) % 16 != 0))
    return hsn::fail(ctx, HSN_ERR_INVALID_ARG, "normalize: ldb must be >= n_bins, a multiple of 32, 16-byte aligned");
  if (offset_b && !bg_mask) return hsn::fail(ctx, HSN_ERR_INVALID_ARG, "normalize: offset_b requires bg_mask");
  if (bf16_bias && !p_bf16) return hsn::fail(ctx, HSN_ERR_INVALID_ARG, "normalize: bf16_bias requires p_bf16");
  if (!(count_floor >= 0.0f)) return hsn::fail(ctx, HSN_ERR_INVALID_ARG, "normalize: count_floor must be >= 0");
  hsn::DeviceGuard g(ctx->device);
  double *scratch = nullptr;
  if (scratch_of && !(scratch = scratch_of(ctx))) return HSN_ERR_DEVICE;
  hipStream_t st = static_cast<hipStream_t>(stream);
  const bool yu = y_dtype == HSN_U16, ou = y_open_dtype == HSN_U16;
  if (yu && ou)
    return launch_all(ctx, d, (const uint16_t *)y, (const uint16_t *)y_open, bg_mask, count_floor, clip_nonneg, p,
                      ldp, p_bf16, ldb, offset_b, sumsq, bf16_bias, pooled, pool_mode, st, scratch);
  if (yu && !ou)
    return launch_all(ctx, d, (const uint16_t *)y, (const float *)y_open, bg_mask, count_floor, clip_nonneg, p, ldp,
                      p_bf16, ldb, offset_b, sumsq, bf16_bias, pooled, pool_mode, st, scratch);
  if (!yu && ou)
    return launch_all(ctx, d, (const float *)y, (const uint16_t *)y_open, bg_mask, count_floor, clip_nonneg, p, ldp,
                      p_bf16, ldb, offset_b, sumsq, bf16_bias, pooled, pool_mode, st, scratch);
  return launch_all(ctx, d, (const float *)y, (const float *)y_open, bg_mask, count_floor, clip_nonneg, p, ldp,
                    p_bf16, ldb, offset_b, sumsq, bf16_bias, pooled, pool_mode, st, scratch);
}

// ---------------------------------------------------------------------------
// No-allocation form: the per-block partials live in a file-scope device
// array (each GPU holds its own copy, at its own address).  Its address is
// looked up once per device, with that device current, and only that
// address is handed to kernels: in host code the array's name is a host
// stand-in, not a device address.
// ---------------------------------------------------------------------------
// Every call rewrites all 2 kSumBlocks slots (the grid is fixed), so nothing
// needs clearing between calls; calls that overlap on one GPU race on it.
static __device__ __align__(256) double scratch[2 * kSumBlocks];  // 32 KB per GPU, kept until the process ends
namespace {
constexpr int kNoAllocMaxDevices = 64;
double *g_scratch_ptr[kNoAllocMaxDevices] = {};
std::mutex g_scratch_mu;

double *noalloc_scratch(hsn_ctx *ctx) {
  if (ctx->device < 0 || ctx->device >= kNoAllocMaxDevices) {
    hsn::fail(ctx, HSN_ERR_DEVICE, "normalize_noalloc: device index %d beyond %d", ctx->device, kNoAllocMaxDevices);
    return nullptr;
  }
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[ctx->device]) {
    void *ptr = nullptr;  // the caller's DeviceGuard made ctx->device current
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr) {
      (void)hipGetLastError();
      hsn::fail(ctx, HSN_ERR_DEVICE, "normalize_noalloc: hipGetSymbolAddress failed: %s", hipGetErrorString(e));
      return nullptr;
    }
    g_scratch_ptr[ctx->device] = static_cast<double *>(ptr);
  }
  return g_scratch_ptr[ctx->device];
}
}  // namespace

extern "C" hsn_status hsn_normalize(hsn_ctx *ctx, const hsn_dims *d, const void *y, int y_dtype,
                                    const void *y_open, int y_open_dtype, const uint8_t *bg_mask,
                                    float count_floor, int clip_nonneg, float *p, int64_t ldp, uint16_t *p_bf16,
                                    int64_t ldb, float *offset_b, double *sumsq, double *bf16_bias,
                                    void *stream) {
  return normalize_impl(ctx, d, y, y_dtype, y_open, y_open_dtype, bg_mask, count_floor, clip_nonneg, p, ldp, p_bf16,
                        ldb, offset_b, sumsq, bf16_bias, nullptr, 0, stream);
}

extern "C" hsn_status hsn_normalize_pooled(hsn_ctx *ctx, const hsn_dims *d, const void *y, int y_dtype,
                                           const void *y_open, int y_open_dtype, const uint8_t *bg_mask,
                                           float count_floor, int clip_nonneg, float *p, int64_t ldp,
                                           uint16_t *p_bf16, int64_t ldb, float *offset_b, double *sumsq,
                                           double *bf16_bias, void *pooled, int pooled_precision, void *stream) {
  if (!ctx) return HSN_ERR_INVALID_ARG;
  if (!pooled) return hsn::fail(ctx, HSN_ERR_INVALID_ARG, "normalize_pooled: pooled is required");
  if (pooled_precision != HSN_PREC_BF16 && pooled_precision != HSN_PREC_FP32)
    return hsn::fail(ctx, HSN_ERR_INVALID_ARG, "normalize_pooled: pooled_precision must be HSN_PREC_BF16 or HSN_PREC_FP32");
  if (reinterpret_cast<uintptr_t>(pooled) % 4 != 0)
    return hsn::fail(ctx, HSN_ERR_INVALID_ARG, "normalize_pooled: pooled must be 4-byte aligned");
  return normalize_impl(ctx, d, y, y_dtype, y_open, y_open_dtype, bg_mask, count_floor, clip_nonneg, p, ldp, p_bf16,
                        ldb, offset_b, sumsq, bf16_bias, pooled, pooled_precision == HSN_PREC_BF16 ? 1 : 2, stream);
}

extern "C" hsn_status hsn_normalize_noalloc(hsn_ctx *ctx, const hsn_dims *d, const void *y, int y_dtype,
                                            const void *y_open, int y_open_dtype, const uint8_t *bg_mask,
                                            float count_floor, int clip_nonneg, float *p, int64_t ldp,
                                            uint16_t *p_bf16, int64_t ldb, float *offset_b, double *sumsq,
                                            double *bf16_bias, void *stream) {
  if (!ctx) return HSN_ERR_INVALID_ARG;
  if (bg_mask && !offset_b)
    return hsn::fail(ctx, HSN_ERR_INVALID_ARG, "normalize_noalloc: bg_mask needs the caller's offset_b buffer");
  return normalize_impl(ctx, d, y, y_dtype, y_open, y_open_dtype, bg_mask, count_floor, clip_nonneg, p, ldp, p_bf16,
                        ldb, offset_b, sumsq, bf16_bias, nullptr, 0, stream, noalloc_scratch);
}
