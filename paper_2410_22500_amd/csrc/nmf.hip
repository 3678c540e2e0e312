// hsn_subspace_nmf: the NMF of eq. (4), (V, D) = argmin_{V,D>=0} ||p - V D^T||^2.
//
// Every iteration is a short fixed sequence of launches on the caller's
// stream, with no host synchronisation except when an objective value is
// read for the stop test:
//   multiplicative updates (Lee-Seung; V first, then D with the new V):
//     gram(D) -> fused pass [N_V = P D, V update, N_D += P^T V_new,
//     G_V += V_new^T V_new, optional ||P - V_new D^T||^2] -> reduce -> D update
//   ANLS round (exact row-wise non-negative least squares, V then D):
//     gram(D)+factors -> pass N_V -> row solves -> pass N_D (+objective)
//     -> reduce -> G_V factors -> row solves of D
// The float32 pass reads p once per MU iteration.  The bfloat16 bulk runs the
// same sequence with the MFMA pass over the bfloat16 copy of p.
#include "nmf_common.hpp"

#include <algorithm>
#include <cmath>

namespace hsn {

void launch_pass_f32(int K, int mode, bool obj, int nq, int n_wg, hipStream_t st, const float *P, int64_t ldp,
                     int64_t n_p, int n_k, float *V, float *NV, const float *D, const double *GD, float *part_nd,
                     double *part_gv, double *part_obj);
void launch_gram(int K, hipStream_t st, const float *F, int64_t n, double *G, double *chol, int want_chol);
void launch_reduce_update(int K, int mode_d, bool obj, hipStream_t st, const NmfWork &w, int n_wg, int n_k, float *D,
                          double *hist_slot);
void launch_nnls_rows(int K, hipStream_t st, const float *NV, const double *GD, const double *chol, float *V,
                      int64_t n_p, int n_blocks);
// bfloat16 MFMA pass (nmf_bf16.hip); returns false if the shape is unsupported.
bool launch_pass_bf16(int K, int mode, bool obj, int n_wg, hipStream_t st, const uint16_t *Pb, int64_t ldb,
                      int64_t n_p, int n_k, float *V, const float *D, const double *GD, uint4 *scratch,
                      float *part_nd, double *part_gv, double *part_obj);
int pass_bf16_wgs(hsn_ctx *ctx, int64_t n_p);
size_t bf16_scratch_bytes(int64_t ldb);

namespace {

struct Run {
  hsn_ctx *ctx;
  hipStream_t st;
  int K;
  int64_t n_p;
  int n_k;
  NmfWork w;
  int hist_len = 0;
  int wg_f32 = 0, wg_bf16 = 0;  // persistent grid sizes of the two passes
  uint4 *bf16_scratch = nullptr;
};

// One fused iteration (MU or HALS row rule): a single streaming read of p.
hsn_status fused_iteration(Run &R, int mode, bool bf16, const float *p, int64_t ldp, const uint16_t *pb, int64_t ldb,
                           float *V, float *D, bool obj) {
  launch_gram(R.K, R.st, D, R.n_k, R.w.gd, R.w.chol, 0);
  const int n_wg = bf16 ? R.wg_bf16 : R.wg_f32;
  prof_begin(R.ctx, HSN_KERN_NMF_PASS, R.st);
  if (bf16) {
    if (!launch_pass_bf16(R.K, mode, obj, n_wg, R.st, pb, ldb, R.n_p, R.n_k, V, D, R.w.gd, R.bf16_scratch,
                          R.w.part_nd, R.w.part_gv, R.w.part_obj))
      return fail(R.ctx, HSN_ERR_UNSUPPORTED, "bf16 pass: unsupported shape (ldb <= 2048, k <= 8)");
  } else {
    launch_pass_f32(R.K, mode, obj, R.n_k > 1024 ? 2 : 1, n_wg, R.st, p, ldp, R.n_p, R.n_k, V, nullptr, D, R.w.gd,
                    R.w.part_nd, R.w.part_gv, R.w.part_obj);
  }
  prof_end(R.ctx, HSN_KERN_NMF_PASS, R.st);
  launch_reduce_update(R.K, mode, obj, R.st, R.w, n_wg, R.n_k, D, obj ? R.w.hist + R.hist_len : nullptr);
  if (obj) ++R.hist_len;
  HSN_LAUNCHED(R.ctx);
  return HSN_OK;
}

hsn_status anls_round(Run &R, const float *p, int64_t ldp, float *V, float *D) {
  const int nq = R.n_k > 1024 ? 2 : 1;
  launch_gram(R.K, R.st, D, R.n_k, R.w.gd, R.w.chol, 1);
  prof_begin(R.ctx, HSN_KERN_NMF_PASS, R.st);
  launch_pass_f32(R.K, kModeNV, false, nq, R.wg_f32, R.st, p, ldp, R.n_p, R.n_k, V, R.w.nv, D, R.w.gd, R.w.part_nd,
                  R.w.part_gv, R.w.part_obj);
  prof_end(R.ctx, HSN_KERN_NMF_PASS, R.st);
  const int nb = int(std::min<int64_t>((R.n_p + 255) / 256, 8 * int64_t(R.ctx->num_cu)));
  launch_nnls_rows(R.K, R.st, R.w.nv, R.w.gd, R.w.chol, V, R.n_p, nb);
  prof_begin(R.ctx, HSN_KERN_NMF_PASS, R.st);
  launch_pass_f32(R.K, kModeND, true, nq, R.wg_f32, R.st, p, ldp, R.n_p, R.n_k, V, nullptr, D, R.w.gd, R.w.part_nd,
                  R.w.part_gv, R.w.part_obj);
  prof_end(R.ctx, HSN_KERN_NMF_PASS, R.st);
  launch_reduce_update(R.K, kModeNV, true, R.st, R.w, R.wg_f32, R.n_k, D, R.w.hist + R.hist_len);
  ++R.hist_len;
  HSN_LAUNCHED(R.ctx);
  return HSN_OK;
}

hsn_status read_last(Run &R, double *out) {
  HSN_HIP(R.ctx, hipMemcpyAsync(out, R.w.hist + (R.hist_len - 1), sizeof(double), hipMemcpyDeviceToHost, R.st));
  HSN_HIP(R.ctx, hipStreamSynchronize(R.st));
  return HSN_OK;
}

}  // namespace
}  // namespace hsn

extern "C" hsn_status hsn_subspace_nmf(hsn_ctx *ctx, const float *p, int64_t ldp, const uint16_t *p_bf16,
                                       int64_t ldb, int64_t n_p, int64_t n_k, float *V, float *D,
                                       const hsn_nmf_opts *o, hsn_nmf_stats *stats, void *stream) {
  using namespace hsn;
  if (!ctx) return HSN_ERR_INVALID_ARG;
  if (!o) return fail(ctx, HSN_ERR_INVALID_ARG, "nmf: opts is NULL");
  if (o->k < 1 || o->k > 8) return fail(ctx, HSN_ERR_SHAPE, "nmf: k must be in 1..8 (got %d)", o->k);
  if (n_p < 1 || n_k < 1 || n_k > 2048) return fail(ctx, HSN_ERR_SHAPE, "nmf: need n_p >= 1 and 1 <= n_k <= 2048");
  if (o->algo != HSN_ALGO_MU && o->algo != HSN_ALGO_ANLS && o->algo != HSN_ALGO_HALS)
    return fail(ctx, HSN_ERR_INVALID_ARG, "nmf: bad algo");
  if (o->polish_rounds > 0 && o->polish_algo != HSN_ALGO_ANLS && o->polish_algo != HSN_ALGO_HALS)
    return fail(ctx, HSN_ERR_INVALID_ARG, "nmf: polish_algo must be HSN_ALGO_ANLS or HSN_ALGO_HALS");
  if (o->precision != HSN_PREC_FP32 && o->precision != HSN_PREC_BF16)
    return fail(ctx, HSN_ERR_INVALID_ARG, "nmf: bad precision");
  if (o->init != HSN_INIT_USER) return fail(ctx, HSN_ERR_UNSUPPORTED, "nmf: only HSN_INIT_USER is available");
  if (o->max_iter < 0 || o->check_every < 1 || o->polish_rounds < 0)
    return fail(ctx, HSN_ERR_INVALID_ARG, "nmf: max_iter >= 0, check_every >= 1, polish_rounds >= 0 required");
  if (!V || !D) return fail(ctx, HSN_ERR_INVALID_ARG, "nmf: V and D are required");
  const bool bf16 = o->precision == HSN_PREC_BF16;
  if (bf16 && o->algo == HSN_ALGO_ANLS)
    return fail(ctx, HSN_ERR_UNSUPPORTED, "nmf: the bfloat16 bulk runs MU or HALS");
  const bool need_f32 = (!bf16 && o->max_iter > 0) || o->polish_rounds > 0;
  if (need_f32) {
    if (!p) return fail(ctx, HSN_ERR_INVALID_ARG, "nmf: float32 p is required");
    if (ldp < n_k || ldp % 4 != 0 || reinterpret_cast<uintptr_t>(p) % 16 != 0)
      return fail(ctx, HSN_ERR_INVALID_ARG, "nmf: ldp must be >= n_k and a multiple of 4, p 16-byte aligned");
  }
  if (bf16 && o->max_iter > 0) {
    if (!p_bf16) return fail(ctx, HSN_ERR_INVALID_ARG, "nmf: p_bf16 is required for the bfloat16 bulk");
    if (ldb < n_k || ldb % 32 != 0 || reinterpret_cast<uintptr_t>(p_bf16) % 16 != 0)
      return fail(ctx, HSN_ERR_INVALID_ARG, "nmf: ldb must be >= n_k and a multiple of 32, p_bf16 16-byte aligned");
  }
  if (stats && stats->history_cap > 0 && !stats->history)
    return fail(ctx, HSN_ERR_INVALID_ARG, "nmf: stats.history is NULL but history_cap > 0");

  DeviceGuard dg(ctx->device);
  hipStream_t st = static_cast<hipStream_t>(stream);
  const int K = o->k;
  const int64_t n_tiles = (n_p + 7) / 8;
  const int wg_f32 = int(std::min<int64_t>(n_tiles, 2 * int64_t(ctx->num_cu)));
  const int wg_bf16 = bf16 ? pass_bf16_wgs(ctx, n_p) : 0;
  const int n_wg = std::max(wg_f32, wg_bf16);
  const int hist_cap = o->max_iter + o->polish_rounds + 2;
  const bool need_nv = o->algo == HSN_ALGO_ANLS || (o->polish_rounds > 0 && o->polish_algo == HSN_ALGO_ANLS);
  const size_t need = Carver::need({sizeof(double) * 64, sizeof(double) * 64, sizeof(double) * 256 * kCholStride,
                                    sizeof(float) * size_t(n_wg) * n_k * K, sizeof(double) * size_t(n_wg) * K * K,
                                    sizeof(double) * n_wg, sizeof(double) * kSplit * size_t(n_k) * K,
                                    sizeof(double) * kSplit * K * K, sizeof(double) * kSplit,
                                    need_nv ? sizeof(float) * n_p * K : 0,
                                    sizeof(double) * hist_cap, bf16 ? bf16_scratch_bytes(ldb) : 0});
  hsn_status rc = ensure_ws(ctx, need);
  if (rc != HSN_OK) return rc;
  Carver cv(ctx->ws);
  Run R{ctx, st, K, n_p, int(n_k), {}};
  R.w.gd = cv.take<double>(64);
  R.w.gv = cv.take<double>(64);
  R.w.chol = cv.take<double>(256 * kCholStride);
  R.w.part_nd = cv.take<float>(size_t(n_wg) * n_k * K);
  R.w.part_gv = cv.take<double>(size_t(n_wg) * K * K);
  R.w.part_obj = cv.take<double>(n_wg);
  R.w.red_nd = cv.take<double>(kSplit * size_t(n_k) * K);
  R.w.red_gv = cv.take<double>(kSplit * K * K);
  R.w.red_obj = cv.take<double>(kSplit);
  R.w.nv = need_nv ? cv.take<float>(n_p * K) : nullptr;
  R.w.hist = cv.take<double>(hist_cap);
  R.w.n_wg = n_wg;
  R.wg_f32 = wg_f32;
  R.wg_bf16 = wg_bf16;
  if (bf16) R.bf16_scratch = cv.take<uint4>(bf16_scratch_bytes(ldb) / sizeof(uint4));

  if (stats) HSN_HIP(ctx, hipEventRecord(ctx->ev0, st));
  const bool stop_test = o->f_ref > 0.0;
  double last = NAN;
  int it = 0;
  bool reached = false;
  for (; it < o->max_iter && !reached; ++it) {
    const bool obj = ((it + 1) % o->check_every == 0) || (it + 1 == o->max_iter);
    if (o->algo == HSN_ALGO_ANLS)
      rc = anls_round(R, p, ldp, V, D);
    else
      rc = fused_iteration(R, o->algo == HSN_ALGO_MU ? kModeMU : kModeHALS, bf16, p, ldp, p_bf16, ldb, V, D, obj);
    if (rc != HSN_OK) return rc;
    if (obj && stop_test) {
      if ((rc = read_last(R, &last)) != HSN_OK) return rc;
      if ((last - o->f_ref) / o->f_ref <= o->rel_obj_tol) reached = true;
    }
  }
  int polished = 0;
  for (; polished < o->polish_rounds; ++polished) {
    rc = (o->polish_algo == HSN_ALGO_ANLS) ? anls_round(R, p, ldp, V, D)
                                           : fused_iteration(R, kModeHALS, false, p, ldp, nullptr, 0, V, D, true);
    if (rc != HSN_OK) return rc;
    if (stop_test) {
      if ((rc = read_last(R, &last)) != HSN_OK) return rc;
      if ((last - o->f_ref) / o->f_ref <= o->rel_obj_tol) {
        ++polished;
        break;
      }
    }
  }
  if (stats) {
    HSN_HIP(ctx, hipEventRecord(ctx->ev1, st));
    HSN_HIP(ctx, hipEventSynchronize(ctx->ev1));
    float ms = 0.f;
    HSN_HIP(ctx, hipEventElapsedTime(&ms, ctx->ev0, ctx->ev1));
    stats->ms = ms;
    stats->iters = it;
    stats->polish_done = polished;
    stats->history_len = 0;
    if (R.hist_len > 0) {
      std::vector<double> h(R.hist_len);
      HSN_HIP(ctx, hipMemcpy(h.data(), R.w.hist, sizeof(double) * R.hist_len, hipMemcpyDeviceToHost));
      last = h.back();
      const int n_copy = std::min(R.hist_len, stats->history_cap);
      for (int i = 0; i < n_copy; ++i) stats->history[i] = h[i];
      stats->history_len = n_copy;
    }
    stats->objective = last;
    stats->rel_obj = stop_test ? (last - o->f_ref) / o->f_ref : NAN;
    if (std::isnan(last) && R.hist_len > 0) return fail(ctx, HSN_ERR_NUMERIC, "nmf: objective is NaN");
  }
  return HSN_OK;
}
