// Pieces shared by the NMF passes (float32 VALU pass, bfloat16 MFMA pass)
// and the per-iteration reduction / factor-update kernels.
#pragma once

#include "common.hpp"

namespace hsn {

// Row-local update rules of one NMF half-step.
enum PassMode {
  kModeMU = 0,  // fused: N_V = P D, Lee-Seung V update, then N_D += P^T V_new
  kModeNV = 1,  // N_V = P D only (written out; the rows are solved separately)
  kModeND = 2,  // N_D += P^T V_new only (V_new given)
  kModeHALS = 3,  // fused: N_V = P D, HALS column sweep of V, then N_D += P^T V_new
  kModeANLS = 4,  // ANLS round.  As a pass mode: fused, N_V = P D, exact NNLS of every V row
                  // (nnls_enum_group), then N_D += P^T V_new.  As a driver step: that pass or
                  // the two-pass form (N_V pass, row solves, N_D pass), then the D row solves
};

// One HALS sweep of a row x given its right-hand side h and Gram G: for each
// column j in order, x_j <- max(0, x_j + (h_j - sum_i x_i G_ij) / G_jj), using
// the already updated x_i (Cichocki-Phan).  Columns with G_jj = 0 are skipped.
template <int K>
__device__ __forceinline__ void hals_row(const double *__restrict__ G, const double (&h)[K], double (&x)[K]) {
#pragma unroll
  for (int j = 0; j < K; ++j) {
    const double gjj = G[j * K + j];
    if (gjj > 0.0) {
      double g = h[j];
#pragma unroll
      for (int i = 0; i < K; ++i) g -= x[i] * G[i * K + j];
      x[j] = fmax(0.0, x[j] + g / gjj);
    }
  }
}

// Device-resident loop control of one decomposition.  Every iteration has a
// global index; kernels of iteration i return at once when i >= stop_at, so
// the host can queue many iterations and synchronise rarely.  stop_at is
// lowered only by the D-update kernel of the iteration whose objective meets
// the tolerance (to i + 1), so no kernel of a running iteration is skipped.
struct NmfCtrl {
  int stop_at;
  int upd_ticket;   // arrival counter of the D-update blocks (last block finishes G_D)
  int hist_len;     // objective values written so far
  int iter_base;    // batched runs: index of the first step of the replayed chunk
  int numeric;      // set (with a stop) when an evaluated objective is NaN or infinite
  int pad[3];
  double last16;    // objective of the last step on p_bf16 that evaluated one
  double adj;       // calibration added to the bfloat16 stop estimate (objective + bias + adj)
  double last_est;  // the value the last stop test compared (the estimate on p_bf16 steps)
  // extrapolated ANLS (hsn_nmf_opts.anls_extrapolate): the extrapolation
  // weight, its cap, the previous round's objective and the weight this
  // round's D update applies (0: no extrapolation)
  double beta, beta_bar, e_prev, beta_use;
  int e_prev_bf16;  // e_prev came from a step on p_bf16 (1), on p (0), none yet (-1)
  int pad2;
  double gvo[65];   // G_V = V^T V (K*K) and the objective of the last pass, reduced
};

// Workspace of one decomposition (all device pointers).
struct NmfWork {
  NmfCtrl *ctrl;
  double *gd;        // [8*8]   G_D = D^T D of the current D
  double *chol;      // [256][36] packed Cholesky factors of principal submatrices of G_D
  float *part_nd;    // [n_wg][n_k][K] per-workgroup partials of P^T V
  double *part_gv;   // [n_wg][K*K]
  double *part_obj;  // [n_wg]
  double *part_gd;   // [update blocks][K*K]
  float *nv;         // [n_p][K] N_V for the row-wise NNLS
  double *ginv;      // [36][kInvStride] inverses of the principal submatrices of G_D (entry-major)
  double *part_gd16; // [update blocks][K*K] partials of G_D' (or null), D' = the bfloat16 hi + lo split of D
  double *ginv16;    // [36][kInvStride] inverses of the principal submatrices of G_D' (or null)
  double *hist;      // [hist_cap] objective history (device)
  uint16_t *img;     // bfloat16 operand images of D for the MFMA pass (or null)
  float *dprev;      // [n_k][K] extrapolated ANLS: the previous round's exact D (or null)
  int n_wg;
};

// One decomposition of a batch (device copy read by the batched kernels):
// its operands, its workspace and its ranges in the shared launch grids.
struct BatchInst {
  const float *P;
  int64_t ldp, n_p;
  int n_k, K, nq;
  float *V, *D, *NV;
  double *gd, *chol;
  float *part_nd;
  double *part_gv, *part_obj, *part_gd, *hist;
  NmfCtrl *ctrl;
  int wg0, n_wg;   // pass workgroups
  int ub0, n_ub;   // D-update blocks
  int rb0, n_rb;   // row-solve blocks
  double f_ref, tol;
  // bfloat16 MU bulk (or null Pb): the bfloat16 p, its pitch, the operand
  // images of D (ldb_img = their padded width) and the MFMA pass's workgroups
  const uint16_t *Pb;
  int64_t ldb, ldb_img;
  uint16_t *img;
  int wg0b, n_wgb;
};

// Instance of a batch that owns grid block b: the last i with first(i) <= b
// (first = the instances' ascending range starts).
template <class F>
__device__ __forceinline__ int batch_find(int n, int b, F first) {
  int lo = 0, hi = n - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (first(mid) <= b) lo = mid; else hi = mid - 1;
  }
  return lo;
}

constexpr int kCholStride = 36;  // packed lower triangle of an 8x8 matrix

// Extrapolated ANLS (Ang & Gillis, Neural Computation 2019): the weight
// starts at kExtrapBeta0 with cap 1; after a round whose objective did not
// rise it grows by kExtrapGrow (capped) and the cap by kExtrapCapGrow (at
// most 1); after a rise the cap becomes the weight, the weight shrinks by
// kExtrapShrink and that round's D is taken without extrapolation.
constexpr double kExtrapBeta0 = 0.5, kExtrapGrow = 1.05, kExtrapCapGrow = 1.01, kExtrapShrink = 1.5;

__host__ __device__ constexpr int tri(int a) { return a * (a + 1) / 2; }

// Cholesky factor (packed lower, compact index order) of G[S,S], S = bits of
// mask.  Returns false if G[S,S] is not numerically positive definite.
__device__ inline bool chol_sub(const double *G, int K, unsigned mask, double *L) {
  int idx[8];
  int s = 0;
  for (int i = 0; i < K; ++i)
    if (mask & (1u << i)) idx[s++] = i;
  for (int a = 0; a < s; ++a) {
    for (int b = 0; b <= a; ++b) {
      double v = G[idx[a] * K + idx[b]];
      for (int c = 0; c < b; ++c) v -= L[tri(a) + c] * L[tri(b) + c];
      if (a == b) {
        if (!(v > 0.0)) return false;
        L[tri(a) + a] = sqrt(v);
      } else {
        L[tri(a) + b] = v / L[tri(b) + b];
      }
    }
  }
  return true;
}

// Non-negative least squares in Gram form, min_{x >= 0} 1/2 x'Gx - h'x, by
// the Lawson-Hanson active-set method with the float64 Cholesky factor of
// the passive set taken from `chol` (indexed by the passive-set bit mask; a
// factor whose first entry is NaN marks a singular set, which is never
// entered).  Same steps, tie breaks and tolerances as the float64 oracle.
template <int K>
__device__ inline void nnls_gram_row(const double *__restrict__ G, const double *__restrict__ chol, const double (&h)[K],
                                     double (&x)[K]) {
  constexpr double tol = 1e-12;
  double scale = 1e-300;
#pragma unroll
  for (int i = 0; i < K; ++i) {
    x[i] = 0.0;
    scale = fmax(scale, fabs(h[i]));
  }
  unsigned passive = 0;
  double w[K];
#pragma unroll
  for (int i = 0; i < K; ++i) w[i] = h[i];
  for (int outer = 0; outer < 4 * K + 8; ++outer) {
    int jmax = -1;
    double wmax = -INFINITY;
#pragma unroll
    for (int i = 0; i < K; ++i)
      if (!(passive & (1u << i)) && w[i] > wmax) {
        wmax = w[i];
        jmax = i;
      }
    if (jmax < 0 || !(wmax > tol * scale)) break;
    if (isnan(chol[(passive | (1u << jmax)) * kCholStride])) break;  // singular: stop at the current point
    passive |= 1u << jmax;
    for (int inner = 0; inner <= K; ++inner) {
      // z = solve on the passive set
      double z[K];
      {
        const double *L = chol + size_t(passive) * kCholStride;
        double t[K];
        int a = 0;
#pragma unroll
        for (int i = 0; i < K; ++i) {
          z[i] = 0.0;
          if (passive & (1u << i)) {
            double v = h[i];
            for (int c = 0; c < a; ++c) v -= L[tri(a) + c] * t[c];
            t[a] = v / L[tri(a) + a];
            ++a;
          }
        }
        const int s = a;
        // back substitution L^T y = t, written into z at the compact positions
        double y[K];
        for (int aa = s - 1; aa >= 0; --aa) {
          double v = t[aa];
          for (int c = aa + 1; c < s; ++c) v -= L[tri(c) + aa] * y[c];
          y[aa] = v / L[tri(aa) + aa];
        }
        a = 0;
#pragma unroll
        for (int i = 0; i < K; ++i)
          if (passive & (1u << i)) z[i] = y[a++];
      }
      bool feasible = true;
#pragma unroll
      for (int i = 0; i < K; ++i)
        if ((passive & (1u << i)) && !(z[i] > 0.0)) feasible = false;
      if (feasible) {
#pragma unroll
        for (int i = 0; i < K; ++i) x[i] = z[i];
        break;
      }
      double alpha = INFINITY;
#pragma unroll
      for (int i = 0; i < K; ++i)
        if ((passive & (1u << i)) && !(z[i] > 0.0)) alpha = fmin(alpha, x[i] / (x[i] - z[i]));
      double xmax = 0.0;
#pragma unroll
      for (int i = 0; i < K; ++i) {
        x[i] = x[i] + alpha * (z[i] - x[i]);
        xmax = fmax(xmax, fabs(x[i]));
      }
      const double thr = tol * fmax(1.0, xmax);
#pragma unroll
      for (int i = 0; i < K; ++i)
        if ((passive & (1u << i)) && !(x[i] > thr)) passive &= ~(1u << i);
#pragma unroll
      for (int i = 0; i < K; ++i)
        if (!(passive & (1u << i))) x[i] = 0.0;
    }
#pragma unroll
    for (int i = 0; i < K; ++i) {
      double v = h[i];
#pragma unroll
      for (int c = 0; c < K; ++c) v -= G[i * K + c] * x[c];
      w[i] = v;
    }
  }
}

// Entry (i, j) of a packed symmetric K x K matrix (lower triangle, row order).
__host__ __device__ constexpr int sym(int i, int j) { return i >= j ? tri(i) + j : tri(j) + i; }

// Inverses of the principal submatrices of a K x K Gram, entry-major: entry
// e (the packed symmetric index sym(i, j) of a K x K matrix) of mask m at
// [e * stride + m].  Per mask, G[S,S]^-1 is embedded in a K x K matrix with
// zeros outside S; a NaN entry 0 marks a singular G[S,S].  The NMF workspace
// holds them with stride kInvStride; the passes stage the tri(K) entries of
// the 2^K masks in LDS with stride 2^K (consecutive masks in consecutive
// words: the lanes of a group read them without bank conflicts).
constexpr int kInvStride = 256;

// Exact non-negative least squares of one row, min_{x >= 0} 1/2 x'Gx - h'x,
// by enumeration of the supports S (bit masks), spread over a group of 32
// lanes (lane l of the group takes masks l, l + 32, ...).  For every S whose
// principal submatrix is positive definite, z_S = G[S,S]^-1 h_S.  Each z
// with all entries on S positive is a feasible point, of cost
// q = -1/2 h_S' z_S; the NNLS minimiser is such a point (its support's
// face-restricted stationary point), so the feasible z of least cost is the
// minimiser (unique when G is positive definite).  Ties in q go to the lower
// mask, x = 0 (empty support, q = 0) is always a candidate.  Lane l < K of
// the group then forms x_l = z_l of the winning support itself and returns
// it (the other lanes return 0), so no lane keeps a z; q_min (optional)
// receives the least cost in every lane.  The 32 lanes must be converged.
// ginv: entry-major inverses with stride STRIDE (see above).
// One exchange of the (cost, mask) minimum with the partner lane that DPP
// control CTRL names (a permutation within each row of 16 lanes).
template <int CTRL>
__device__ __forceinline__ void enum_min_step(double &q, int &m) {
  const uint64_t u = __builtin_bit_cast(uint64_t, q);
  const int lo = __builtin_amdgcn_update_dpp(0, int(uint32_t(u)), CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, int(uint32_t(u >> 32)), CTRL, 0xF, 0xF, false);
  const int om = __builtin_amdgcn_update_dpp(0, m, CTRL, 0xF, 0xF, false);
  const double oq = __builtin_bit_cast(double, (uint64_t(uint32_t(hi)) << 32) | uint32_t(lo));
  if (oq < q || (oq == q && om < m)) {
    q = oq;
    m = om;
  }
}

template <int K, int STRIDE>
__device__ __forceinline__ double nnls_enum_group(const double *__restrict__ ginv, const float (&h)[K], int l,
                                                  double *__restrict__ q_min = nullptr) {
  double best_q = 0.0;
  int best_m = 0;
  for (int m = l; m < (1 << K); m += 32) {
    // no branch before the loads: the empty support (the default) and a
    // singular G[S,S] (NaN first entry) are simply never feasible
    bool feasible = m != 0 && !isnan(ginv[m]);
    double q = 0.0;
    // all rows of z at once for K <= 6 (the tri(K) inverse entries are
    // loaded together, one latency); one row at a time (rolled) beyond,
    // where they would take too many registers beside the pass's own
    constexpr int kRowUnroll = K <= 6 ? K : 1;
#pragma unroll kRowUnroll
    for (int i = 0; i < K; ++i) {
      double s = 0.0, hi = 0.0;
#pragma unroll
      for (int j = 0; j < K; ++j) {
        s = fma(ginv[sym(i, j) * STRIDE + m], double(h[j]), s);
        hi = (j == i) ? double(h[j]) : hi;
      }
      // z_i = s; outside S the embedded inverse gives s = 0 and no cost
      feasible = feasible && (!((m >> i) & 1) || s > 0.0);
      q = fma(-0.5 * hi, s, q);
    }
    if (feasible && (q < best_q || (q == best_q && m < best_m))) {
      best_q = q;
      best_m = m;
    }
  }
  // (q, m) minimum over the 32 lanes: four in-row DPP exchanges (partner
  // lane xor 1, xor 2, mirrored in 8, mirrored in 16), then a swizzle with
  // the lane 16 apart; the combine is order-free, every lane ends with the
  // group's minimum.
  enum_min_step<0xB1>(best_q, best_m);   // quad_perm [1, 0, 3, 2]
  enum_min_step<0x4E>(best_q, best_m);   // quad_perm [2, 3, 0, 1]
  enum_min_step<0x141>(best_q, best_m);  // row_half_mirror
  enum_min_step<0x140>(best_q, best_m);  // row_mirror
  {
    constexpr int kXor16 = 0x1F | (0x10 << 10);  // ds_swizzle bit mode: and 0x1F, xor 0x10
    const double oq = __builtin_bit_cast(
        double, (uint64_t(uint32_t(__builtin_amdgcn_ds_swizzle(int(__builtin_bit_cast(uint64_t, best_q) >> 32),
                                                                kXor16)))
                 << 32) |
                    uint32_t(__builtin_amdgcn_ds_swizzle(int(__builtin_bit_cast(uint64_t, best_q)), kXor16)));
    const int om = __builtin_amdgcn_ds_swizzle(best_m, kXor16);
    if (oq < best_q || (oq == best_q && om < best_m)) {
      best_q = oq;
      best_m = om;
    }
  }
  if (q_min) *q_min = best_q;  // the row's least cost: its objective is ||p_row||^2 + 2 q_min
  double x = 0.0;
  if (l < K && best_m != 0) {
#pragma unroll
    for (int j = 0; j < K; ++j) x = fma(ginv[sym(l, j) * STRIDE + best_m], double(h[j]), x);
  }
  return x;
}

// Sum of f(w) for w = g, g + G, g + 2G, ... < n in a fixed order, with eight
// independent loads in flight per round (the partial sums live in HBM/L2 and
// a dependent chain of loads would be latency bound).
template <typename F>
__device__ __forceinline__ double strided_sum(int g, int G, int n, F f) {
  double a[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  int w = g;
  for (; w + 7 * G < n; w += 8 * G) {
    double v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u] = f(w + u * G);
#pragma unroll
    for (int u = 0; u < 8; ++u) a[u] += v[u];
  }
  for (int u = 0; w < n; w += G, ++u) a[u & 7] += f(w);
  return ((a[0] + a[1]) + (a[2] + a[3])) + ((a[4] + a[5]) + (a[6] + a[7]));
}

// bfloat16 hi/lo split of a float32 value (hi = RNE(x), lo = RNE(x - hi)).
__device__ __forceinline__ uint16_t bf_hi(float f) { return f32_to_bf16_bits(f); }
__device__ __forceinline__ uint16_t bf_lo(float f) { return f32_to_bf16_bits(f - bf16_bits_to_f32(f32_to_bf16_bits(f))); }

}  // namespace hsn
