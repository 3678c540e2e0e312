// Float32 NMF pass over p (eq. 4) on the vector ALUs.
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

// LDS of one pass workgroup: red [4][kRows*K] f32 | vnew, vold [kRows][K] f32 |
// gd_s [K*K] f64 | obj_s [4] f64 | (fused ANLS) hrow [kRows][K] f32 and, for
// K <= 6, the inverses of G_D's principal submatrices [2^K][36] f64.
template <int K>
constexpr bool kInvInLds = K <= 6;

template <int K, int MODE>
struct PassLds {
  static constexpr int red = 0;
  static constexpr int vnew = red + (kPassThreads / 64) * kRows * K * 4;
  static constexpr int vold = vnew + kRows * K * 4;
  static constexpr int gd = (vold + kRows * K * 4 + 7) / 8 * 8;
  static constexpr int obj = gd + K * K * 8;
  static constexpr int hrow = obj + (kPassThreads / 64) * 8;
  static constexpr int ginv = (hrow + (MODE == kModeANLS ? kRows * K * 4 : 0) + 15) / 16 * 16;
  static constexpr int bytes = ginv + ((MODE == kModeANLS && kInvInLds<K>) ? (1 << K) * tri(K) * 8 : 0);
};

// One workgroup `wg` of `n_wg` of the pass (the kernels below supply the
// index, the count and the LDS block).
template <int K, int NQ, int MODE, bool OBJ>
__device__ __forceinline__ void pass_f32_body(
    const float *__restrict__ P, int64_t ldp, int64_t n_p, int n_k, float *__restrict__ V, float *__restrict__ NV,
    const float *__restrict__ D, const double *__restrict__ GD, const double *__restrict__ chol,
    float *__restrict__ part_nd, double *__restrict__ part_gv, double *__restrict__ part_obj,
    NmfCtrl *__restrict__ ctrl, int iter, int wg, int n_wg, char *__restrict__ lds,
    const double *__restrict__ ginv = nullptr) {
  if (iter >= ctrl->stop_at) return;
  const int t = threadIdx.x;
  const int lane = t & 63, wave = t >> 6;
  using L = PassLds<K, MODE>;
  float(*red)[kRows * K] = reinterpret_cast<float(*)[kRows * K]>(lds + L::red);
  float(*vnew)[K] = reinterpret_cast<float(*)[K]>(lds + L::vnew);
  float(*vold)[K] = reinterpret_cast<float(*)[K]>(lds + L::vold);
  double *gd_s = reinterpret_cast<double *>(lds + L::gd);
  double *obj_s = reinterpret_cast<double *>(lds + L::obj);

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
  if ((MODE == kModeMU || MODE == kModeHALS || MODE == kModeANLS) && t < K * K) gd_s[t] = GD[t];
  float *hrow = reinterpret_cast<float *>(lds + L::hrow);
  const double *ginv_s = ginv;
  if constexpr (MODE == kModeANLS && kInvInLds<K>) {
    // entry-major, stride 2^K
    double *g = reinterpret_cast<double *>(lds + L::ginv);
    for (int i = t; i < (1 << K) * tri(K); i += kPassThreads) g[i] = ginv[(i >> K) * kInvStride + (i & ((1 << K) - 1))];
    ginv_s = g;
  }
  __syncthreads();

  const int64_t n_tiles = (n_p + kRows - 1) / kRows;
  for (int64_t tile = wg; tile < n_tiles; tile += n_wg) {
    const int64_t row0 = tile * kRows;
    // The tile's V values (one per thread t < kRows*K) are loaded with the
    // tile, so the row rule does not wait on a global load.
    float vcur = 0.0f;
    if (MODE != kModeNV && MODE != kModeANLS && t < kRows * K && row0 * K + t < n_p * K) vcur = V[row0 * K + t];
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
      if (t < kRows * K) vold[t / K][t % K] = vcur;
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
      if (MODE == kModeANLS) {
        // Exact NNLS of the tile's rows: 32 lanes per row enumerate the supports.
        if (t < kRows * K) {
          float s = 0.0f;
#pragma unroll
          for (int w = 0; w < kPassThreads / 64; ++w) s += red[w][t];
          hrow[t] = s;
        }
        __syncthreads();
        const int r = t >> 5, l = t & 31;
        const int64_t row = row0 + r;
        float h[K];
#pragma unroll
        for (int j = 0; j < K; ++j) h[j] = hrow[r * K + j];
        const double xl = nnls_enum_group<K, kInvInLds<K> ? (1 << K) : kInvStride>(ginv_s, h, l);
        if (l < K) {
          float vn = float(xl);
          if (row >= n_p) vn = 0.0f;
          if (row < n_p) V[row * K + l] = vn;
          vnew[r][l] = vn;
        }
      } else if (MODE == kModeHALS) {
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
            x[j] = (row < n_p) ? double(vold[r][j]) : 0.0;
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
            for (int i = 0; i < K; ++i) vr[i] = vold[r][i];
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
      if (t < kRows * K) vnew[t / K][t % K] = vcur;
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
    float *dst = part_nd + size_t(wg) * n_k * K;
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
    if (t < K * K) part_gv[size_t(wg) * K * K + t] = gv;
    if (OBJ) {
      obj = wave_sum_all(obj);
      if (lane == 0) obj_s[wave] = obj;
      __syncthreads();
      if (t == 0) {
        double s = 0.0;
        for (int w = 0; w < kPassThreads / 64; ++w) s += obj_s[w];
        part_obj[wg] = s;
      }
    }
  }
}

template <int K, int NQ, int MODE, bool OBJ>
__global__ __launch_bounds__(kPassThreads) void pass_f32_kernel(
    const float *__restrict__ P, int64_t ldp, int64_t n_p, int n_k, float *__restrict__ V, float *__restrict__ NV,
    const float *__restrict__ D, const double *__restrict__ GD, const double *__restrict__ chol,
    float *__restrict__ part_nd, double *__restrict__ part_gv, double *__restrict__ part_obj,
    NmfCtrl *__restrict__ ctrl, int iter, const double *__restrict__ ginv) {
  __shared__ __attribute__((aligned(16))) char lds[PassLds<K, MODE>::bytes];
  pass_f32_body<K, NQ, MODE, OBJ>(P, ldp, n_p, n_k, V, NV, D, GD, chol, part_nd, part_gv, part_obj, ctrl, iter,
                                  int(blockIdx.x), int(gridDim.x), lds, ginv);
}

// ---------------------------------------------------------------------------
// Batched pass: one launch over the workgroups of many decompositions.  Block
// b belongs to the instance whose range [wg0, wg0 + n_wg) holds it; the
// instance's K and bin count pick the body.  The iteration index is the
// instance's iter_base (advanced on the device between graph replays) plus
// the step's position inside the replayed chunk.
// ---------------------------------------------------------------------------
template <int K, int NQ, int MODE, bool OBJ>
__global__ __launch_bounds__(kPassThreads) void batched_pass_kernel(const BatchInst *__restrict__ d, int n_inst,
                                                                    int iter_local) {
  __shared__ __attribute__((aligned(16))) char lds[PassLds<K, MODE>::bytes];
  const int i = batch_find(n_inst, int(blockIdx.x), [&](int j) { return d[j].wg0; });
  const BatchInst &b = d[i];
  const int wg = int(blockIdx.x) - b.wg0;
  if (wg >= b.n_wg) return;
  const int iter = b.ctrl->iter_base + iter_local;
  pass_f32_body<K, NQ, MODE, OBJ>(b.P, b.ldp, b.n_p, b.n_k, b.V, b.NV, b.D, b.gd, b.chol, b.part_nd, b.part_gv,
                                  b.part_obj, b.ctrl, iter, wg, b.n_wg, lds);
}

// One launch over the instances d[0 .. n_inst) of one (K, bin class) group
// (wg0 counted from the group's first instance).  mode: kModeMU (objective
// or not), kModeNV, kModeND (objective always).
template <int K, int NQ>
void launch_batched_pass_kq(int mode, bool obj, int n_blocks, hipStream_t st, const BatchInst *d, int n_inst,
                            int iter_local) {
  if (mode == kModeMU) {
    if (obj)
      batched_pass_kernel<K, NQ, kModeMU, true><<<n_blocks, kPassThreads, 0, st>>>(d, n_inst, iter_local);
    else
      batched_pass_kernel<K, NQ, kModeMU, false><<<n_blocks, kPassThreads, 0, st>>>(d, n_inst, iter_local);
  } else if (mode == kModeNV) {
    batched_pass_kernel<K, NQ, kModeNV, false><<<n_blocks, kPassThreads, 0, st>>>(d, n_inst, iter_local);
  } else {
    batched_pass_kernel<K, NQ, kModeND, true><<<n_blocks, kPassThreads, 0, st>>>(d, n_inst, iter_local);
  }
}

void launch_batched_pass(int K, int nq, int mode, bool obj, int n_blocks, hipStream_t st, const BatchInst *d,
                         int n_inst, int iter_local) {
  switch (K * 4 + nq) {
#define HSN_B(KK, NQ_) \
  case KK * 4 + NQ_: launch_batched_pass_kq<KK, NQ_>(mode, obj, n_blocks, st, d, n_inst, iter_local); break;
    HSN_B(1, 1) HSN_B(2, 1) HSN_B(3, 1) HSN_B(4, 1) HSN_B(5, 1) HSN_B(6, 1) HSN_B(7, 1) HSN_B(8, 1)
    HSN_B(1, 2) HSN_B(2, 2) HSN_B(3, 2) HSN_B(4, 2) HSN_B(5, 2) HSN_B(6, 2) HSN_B(7, 2) HSN_B(8, 2)
#undef HSN_B
    default: break;
  }
}

// ---------------------------------------------------------------------------
// Host-side launchers (called by the driver for a runtime K).
// ---------------------------------------------------------------------------
template <int K>
void launch_pass_f32_k(int mode, bool obj, int nq, int n_wg, hipStream_t st, const float *P, int64_t ldp, int64_t n_p,
                       int n_k, float *V, float *NV, const float *D, const double *GD, const double *chol,
                       float *part_nd, double *part_gv, double *part_obj, NmfCtrl *ctrl, int iter,
                       const double *ginv) {
#define HSN_PASS(NQ_, M_, O_)                                                                                   \
  pass_f32_kernel<K, NQ_, M_, O_><<<n_wg, kPassThreads, 0, st>>>(P, ldp, n_p, n_k, V, NV, D, GD, chol, part_nd,    \
                                                                 part_gv, part_obj, ctrl, iter, ginv)
  if (nq == 1) {
    if (mode == kModeANLS) {
      HSN_PASS(1, kModeANLS, true);
    } else if (mode == kModeMU) {
      if (obj) HSN_PASS(1, kModeMU, true); else HSN_PASS(1, kModeMU, false);
    } else if (mode == kModeHALS) {
      if (obj) HSN_PASS(1, kModeHALS, true); else HSN_PASS(1, kModeHALS, false);
    } else if (mode == kModeNV) {
      HSN_PASS(1, kModeNV, false);
    } else {
      HSN_PASS(1, kModeND, true);
    }
  } else {
    if (mode == kModeANLS) {
      HSN_PASS(2, kModeANLS, true);
    } else if (mode == kModeMU) {
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
                     int64_t n_p, int n_k, float *V, float *NV, const float *D, const double *GD, const double *chol,
                     float *part_nd, double *part_gv, double *part_obj, NmfCtrl *ctrl, int iter,
                     const double *ginv) {
  switch (K) {
#define HSN_K(KK)                                                                                                  \
  case KK:                                                                                                         \
    launch_pass_f32_k<KK>(mode, obj, nq, n_wg, st, P, ldp, n_p, n_k, V, NV, D, GD, chol, part_nd, part_gv,      \
                          part_obj, ctrl, iter, ginv);                                                             \
    break;
    HSN_K(1) HSN_K(2) HSN_K(3) HSN_K(4) HSN_K(5) HSN_K(6) HSN_K(7) HSN_K(8)
#undef HSN_K
  }
}

}  // namespace hsn
