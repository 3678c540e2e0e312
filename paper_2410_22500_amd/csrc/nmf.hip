// hsn_subspace_nmf: the NMF of eq. (4), (V, D) = argmin_{V,D>=0} ||p - V D^T||^2.
//
// Every iteration is a short fixed sequence of launches on the caller's
// stream:
//   MU / HALS iteration (V first, then D with the new V):
//     fused pass [N_V = P D, row rule for V, N_D += P^T V_new, G_V, optional
//     ||P - V_new D^T||^2]  ->  update_d [reductions, D row rule, G_D of D_new]
//   ANLS round (exact row-wise non-negative least squares, V then D):
//     fused pass [N_V = P D, exact NNLS of every V row by support enumeration
//     with the FP64 inverses of G_D's principal submatrices, N_D += P^T V_new,
//     objective] -> update_d (row solves of D); or, in the two-pass form,
//     pass N_V -> row solves of V -> pass N_D -> update_d
// The stop test runs on the device (update_d lowers stop_at), so the host
// queues iterations in chunks and reads the control block once per chunk.
// The float32 pass reads p once per iteration or fused ANLS round; the
// bfloat16 steps run the same sequence with the MFMA pass over the bfloat16
// copy of p.  Polish rounds on the bfloat16 p end when the objective, plus
// the bias -||p - p_bf16||^2 when given and a calibration, meets the
// tolerance; one float32 round confirms such a stop or calibrates the
// estimate (the bfloat16 rounds then resume), and the float32 rounds decide
// the stop on the float32 objective.
#include "nmf_common.hpp"

#include <algorithm>
#include <climits>
#include <cmath>
#include <vector>

namespace hsn {

void launch_pass_f32(int K, int mode, bool obj, int nq, int n_wg, hipStream_t st, const float *P, int64_t ldp,
                     int64_t n_p, int n_k, float *V, float *NV, const float *D, const double *GD, const double *chol,
                     float *part_nd, double *part_gv, double *part_obj, NmfCtrl *ctrl, int iter,
                     const double *ginv);
bool launch_pass_bf16(int K, int mode, bool obj, int n_wg, hipStream_t st, const uint16_t *Pb, int64_t ldb,
                      int64_t n_p, int n_k, float *V, const double *GD, const double *chol, const uint16_t *img,
                      float *part_nd, double *part_gv, double *part_obj, NmfCtrl *ctrl, int iter,
                      const double *ginv);
int pass_bf16_wgs(hsn_ctx *ctx, int64_t n_p);
size_t bf16_image_elems(int64_t ldb);
int64_t bf16_image_ldb(int64_t ldb);
void launch_nmf_init(int K, hipStream_t st, const float *D, int n_k, const NmfWork &w, int want_chol, int64_t ldb);
int update_d_blocks(int n_k);
void launch_update_d(int K, int rule, hipStream_t st, float *D, const NmfWork &w, int n_wg, int n_k, int iter,
                     bool has_obj, double f_ref, double tol, bool next_chol, int64_t ldb_img, int bf16,
                     const double *bias, bool extrap);
void launch_nmf_resume(hipStream_t st, NmfCtrl *ctrl);
void launch_nmf_calibrate(hipStream_t st, NmfCtrl *ctrl, const double *hist, const double *bias);
void launch_nnls_rows(int K, hipStream_t st, const NmfWork &w, float *V, int64_t n_p, int n_blocks, int iter);
size_t nndsvd_ws_bytes(int64_t n_p, int n_k, int K, int n_split);
size_t mlp_pool_bytes(const hsn_mlp *m, int64_t n_p);
int mlp_k(const hsn_mlp *m);
int mlp_device(const hsn_mlp *m);
hsn_status mlp_nmf_start(hsn_ctx *ctx, hipStream_t st, const hsn_mlp *m, const float *p, int64_t ldp,
                         const uint16_t *pb, int64_t ldb, int64_t n_p, int n_k, float *V, float *D, void *xbuf,
                         const void *pooled, const NmfWork &w, int n_wg, int wg_bf16);
hsn_status nndsvd_init(hsn_ctx *ctx, hipStream_t st, const float *p, int64_t ldp, const uint16_t *pb, int64_t ldb,
                       int64_t n_p, int n_k, int K, float *V, float *D, void *ws, int n_split, bool fill);

namespace {

constexpr int kBf16PolishCheck = 4;
constexpr int kBf16Calibrations = 2;

// One step of the schedule, in issue order.
struct Step {
  int rule;     // kModeMU, kModeHALS or kModeANLS (exact row-wise NNLS for V, then for D)
  bool bf16;    // pass over the bfloat16 copy of p
  bool obj;     // objective evaluated (and stop test applied)
};

struct Run {
  hsn_ctx *ctx;
  hipStream_t st;
  int K;
  int64_t n_p;
  int n_k;
  NmfWork w;
  int wg_f32 = 0, wg_bf16 = 0;  // persistent grid sizes of the two passes
  double f_ref = 0.0, tol = 0.0;
  const double *bias = nullptr;  // device -||p - p_bf16||^2 for the bfloat16 stop test, or null
  bool fused_anls = true;        // ANLS rounds as one fused pass (else N_V pass, row solves, N_D pass)
};

// Queue iteration `iter`.  MU / HALS: one streaming pass over p (row rule for
// V, N_D and G_V partials, optional objective) and the D update.  ANLS: the
// fused pass (exact NNLS of the V rows inside the pass) or a pass for
// N_V = P D, the exact row solves of V on all rows in parallel and a pass for
// N_D = P^T V_new (+ objective); then the exact row solves of D.
// next_exact: the following step solves V rows exactly (the update then also
// factors G_D).
hsn_status queue_step(Run &R, const Step &s, int iter, bool next_exact, const float *p, int64_t ldp,
                      const uint16_t *pb, int64_t ldb, float *V, float *D) {
  const int nq = R.n_k > 1024 ? 2 : 1;
  const int n_wg = s.bf16 ? R.wg_bf16 : R.wg_f32;
  const bool obj = s.obj;
  if (s.rule == kModeANLS && !s.bf16 && R.fused_anls) {
    prof_begin(R.ctx, HSN_KERN_NMF_PASS, R.st);
    launch_pass_f32(R.K, kModeANLS, true, nq, n_wg, R.st, p, ldp, R.n_p, R.n_k, V, nullptr, D, R.w.gd, R.w.chol,
                    R.w.part_nd, R.w.part_gv, R.w.part_obj, R.w.ctrl, iter, R.w.ginv);
    prof_end(R.ctx, HSN_KERN_NMF_PASS, R.st);
  } else if (s.rule == kModeANLS && !s.bf16) {
    prof_begin(R.ctx, HSN_KERN_NMF_PASS, R.st);
    // The N_V pass writes no per-workgroup partials, so it takes up to 8
    // workgroups per CU for latency hiding (same rows per workgroup rule,
    // same results): 98 -> 86 us at mid.
    const int wg_nv = int(std::min<int64_t>((R.n_p + 7) / 8, 8 * int64_t(R.ctx->num_cu)));
    launch_pass_f32(R.K, kModeNV, false, nq, wg_nv, R.st, p, ldp, R.n_p, R.n_k, V, R.w.nv, D, R.w.gd, R.w.chol,
                    R.w.part_nd, R.w.part_gv, R.w.part_obj, R.w.ctrl, iter, nullptr);
    prof_end(R.ctx, HSN_KERN_NMF_PASS, R.st);
    const int nb = int(std::min<int64_t>((R.n_p + 255) / 256, 8 * int64_t(R.ctx->num_cu)));
    launch_nnls_rows(R.K, R.st, R.w, V, R.n_p, nb, iter);
    prof_begin(R.ctx, HSN_KERN_NMF_PASS, R.st);
    launch_pass_f32(R.K, kModeND, true, nq, n_wg, R.st, p, ldp, R.n_p, R.n_k, V, nullptr, D, R.w.gd, R.w.chol,
                    R.w.part_nd, R.w.part_gv, R.w.part_obj, R.w.ctrl, iter, nullptr);
    prof_end(R.ctx, HSN_KERN_NMF_PASS, R.st);
  } else {
    prof_begin(R.ctx, s.bf16 ? HSN_KERN_NMF_PASS_BF16 : HSN_KERN_NMF_PASS, R.st);
    if (s.bf16) {
      const bool ok = launch_pass_bf16(R.K, s.rule, obj, n_wg, R.st, pb, ldb, R.n_p, R.n_k, V, R.w.gd, R.w.chol,
                                       R.w.img, R.w.part_nd, R.w.part_gv, R.w.part_obj, R.w.ctrl, iter,
                                       R.w.ginv16 ? R.w.ginv16 : R.w.ginv);
      prof_end(R.ctx, HSN_KERN_NMF_PASS_BF16, R.st);
      if (!ok) return fail(R.ctx, HSN_ERR_UNSUPPORTED, "bf16 pass: unsupported shape (ldb <= 2048, k <= 8)");
    } else {
      launch_pass_f32(R.K, s.rule, obj, nq, n_wg, R.st, p, ldp, R.n_p, R.n_k, V, nullptr, D, R.w.gd, R.w.chol,
                      R.w.part_nd, R.w.part_gv, R.w.part_obj, R.w.ctrl, iter, nullptr);
      prof_end(R.ctx, HSN_KERN_NMF_PASS, R.st);
    }
  }
  launch_update_d(R.K, s.rule == kModeANLS ? kModeNV : s.rule, R.st, D, R.w, n_wg, R.n_k, iter, obj, R.f_ref,
                  R.tol, next_exact, R.w.img ? bf16_image_ldb(ldb) : 0, s.bf16 ? 1 : 0, s.bf16 ? R.bias : nullptr,
                  s.rule == kModeANLS && R.w.dprev != nullptr);
  HSN_LAUNCHED(R.ctx);
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
  if (o->init != HSN_INIT_USER && o->init != HSN_INIT_NNDSVDA && o->init != HSN_INIT_MLP &&
      o->init != HSN_INIT_NNDSVD)
    return fail(ctx, HSN_ERR_INVALID_ARG, "nmf: bad init");
  const bool nndsvd = o->init == HSN_INIT_NNDSVDA || o->init == HSN_INIT_NNDSVD;
  if (o->init == HSN_INIT_MLP) {
    if (!o->mlp) return fail(ctx, HSN_ERR_INVALID_ARG, "nmf: HSN_INIT_MLP needs opts.mlp");
    if (mlp_k(o->mlp) != o->k) return fail(ctx, HSN_ERR_SHAPE, "nmf: the network's k differs from opts.k");
    if (mlp_device(o->mlp) != ctx->device) return fail(ctx, HSN_ERR_INVALID_ARG, "nmf: network on another device");
  }
  if (o->max_iter < 0 || o->check_every < 1 || o->polish_rounds < 0)
    return fail(ctx, HSN_ERR_INVALID_ARG, "nmf: max_iter >= 0, check_every >= 1, polish_rounds >= 0 required");
  if (!V || !D) return fail(ctx, HSN_ERR_INVALID_ARG, "nmf: V and D are required");
  const bool bf16 = o->precision == HSN_PREC_BF16;
  if (o->polish_bf16_rounds < 0) return fail(ctx, HSN_ERR_INVALID_ARG, "nmf: polish_bf16_rounds must be >= 0");
  if (o->anls_extrapolate != 0 && o->anls_extrapolate != 1)
    return fail(ctx, HSN_ERR_INVALID_ARG, "nmf: anls_extrapolate must be 0 or 1");
  // The first polish_bf16_rounds polish rounds (ANLS or HALS) read the bfloat16 p.
  const int pol_bf16 = std::min(o->polish_bf16_rounds, o->polish_rounds);
  const bool need_f32 = (!bf16 && o->max_iter > 0) || o->polish_rounds > pol_bf16 || o->init != HSN_INIT_USER;
  if (need_f32) {
    if (!p) return fail(ctx, HSN_ERR_INVALID_ARG, "nmf: float32 p is required");
    if (ldp < n_k || ldp % 4 != 0 || reinterpret_cast<uintptr_t>(p) % 16 != 0)
      return fail(ctx, HSN_ERR_INVALID_ARG, "nmf: ldp must be >= n_k and a multiple of 4, p 16-byte aligned");
  }
  const bool mlp_pools = o->init == HSN_INIT_MLP && !o->mlp_pooled;
  if ((bf16 && o->max_iter > 0) || pol_bf16 > 0 || mlp_pools) {
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
  const bool any_bf16 = (bf16 && o->max_iter > 0) || pol_bf16 > 0;
  const int wg_bf16 = any_bf16 ? pass_bf16_wgs(ctx, n_p) : 0;
  const int n_wg = std::max(wg_f32, wg_bf16);
  const int hist_cap = o->max_iter + o->polish_rounds + 2;
  const bool two_pass = ctx->nmf_anls_passes == 2;
  const bool need_nv = two_pass && (o->algo == HSN_ALGO_ANLS || (o->polish_rounds > 0 && o->polish_algo == HSN_ALGO_ANLS));
  const int n_upd = update_d_blocks(int(n_k));
  const size_t need = Carver::need({sizeof(NmfCtrl), sizeof(double) * 64, sizeof(double) * 256 * kCholStride,
                                    sizeof(double) * kCholStride * kInvStride,
                                    sizeof(float) * size_t(n_wg) * n_k * K, sizeof(double) * size_t(n_wg) * K * K,
                                    sizeof(double) * n_wg, sizeof(double) * size_t(n_upd) * K * K,
                                    need_nv ? sizeof(float) * n_p * K : 0, sizeof(double) * hist_cap,
                                    any_bf16 ? sizeof(uint16_t) * bf16_image_elems(ldb) : 0,
                                    any_bf16 ? sizeof(double) * size_t(n_upd) * K * K : 0,
                                    any_bf16 ? sizeof(double) * kCholStride * kInvStride : 0,
                                    o->anls_extrapolate ? sizeof(float) * size_t(n_k) * K : 0});
  // NNDSVD runs before any NMF kernel on the same stream, so its scratch can
  // share the workspace with the decomposition's.
  int n_split = 1;
  size_t need_init = 0;
  // A learned start may be replaced by NNDSVDa after its first stop test.
  const bool fallback = o->init == HSN_INIT_MLP && o->mlp_fallback_rel > 0.0 && o->f_ref > 0.0;
  if (nndsvd || fallback) {
    const int64_t n_tb = (n_k + 127) / 128;
    n_split = int(std::max<int64_t>(1, std::min<int64_t>(1024 / (n_tb * (n_tb + 1) / 2), n_p / 32)));
    need_init = nndsvd_ws_bytes(n_p, int(n_k), K, n_split);
  }
  // The learned start pools p into a scratch block placed after the NMF's
  // arrays (its kernels run before the first NMF kernel reads them).
  const size_t need_pool = mlp_pools ? mlp_pool_bytes(o->mlp, n_p) + 256 : 0;
  hsn_status rc = ensure_ws(ctx, std::max(need + need_pool, need_init));
  if (rc != HSN_OK) return rc;
  Carver cv(ctx->ws);
  Run R{ctx, st, K, n_p, int(n_k), {}};
  R.w.ctrl = cv.take<NmfCtrl>(1);
  R.w.gd = cv.take<double>(64);
  R.w.chol = cv.take<double>(256 * kCholStride);
  R.w.ginv = cv.take<double>(size_t(kCholStride) * kInvStride);
  R.w.part_nd = cv.take<float>(size_t(n_wg) * n_k * K);
  R.w.part_gv = cv.take<double>(size_t(n_wg) * K * K);
  R.w.part_obj = cv.take<double>(n_wg);
  R.w.part_gd = cv.take<double>(size_t(n_upd) * K * K);
  R.w.nv = need_nv ? cv.take<float>(n_p * K) : nullptr;
  R.w.hist = cv.take<double>(hist_cap);
  R.w.img = any_bf16 ? cv.take<uint16_t>(bf16_image_elems(ldb)) : nullptr;
  // The steps on p_bf16 solve V rows with G_D' (the Gram of the bfloat16
  // split of D that their products use), so that a row's least cost gives
  // its objective exactly.
  R.w.part_gd16 = any_bf16 ? cv.take<double>(size_t(n_upd) * K * K) : nullptr;
  R.w.ginv16 = any_bf16 ? cv.take<double>(size_t(kCholStride) * kInvStride) : nullptr;
  // Extrapolated ANLS keeps the previous round's exact D.
  R.w.dprev = o->anls_extrapolate ? cv.take<float>(size_t(n_k) * K) : nullptr;
  void *pool_buf = need_pool ? cv.take<char>(need_pool - 256) : nullptr;
  R.w.n_wg = n_wg;
  R.wg_f32 = wg_f32;
  R.wg_bf16 = wg_bf16;
  const bool stop_test = o->f_ref > 0.0;
  R.f_ref = stop_test ? o->f_ref : 0.0;
  R.tol = o->rel_obj_tol;
  R.bias = o->bf16_bias;
  R.fused_anls = !two_pass;

  // The schedule: bulk iterations, then polish rounds (global indices 0..n-1).
  std::vector<Step> steps;
  steps.reserve(size_t(o->max_iter) + o->polish_rounds);
  for (int it = 0; it < o->max_iter; ++it) {
    const int rule = o->algo == HSN_ALGO_MU ? kModeMU : (o->algo == HSN_ALGO_HALS ? kModeHALS : kModeANLS);
    // float32 ANLS steps always evaluate the objective (the pass has it for free)
    const bool obj = ((it + 1) % o->check_every == 0) || (it + 1 == o->max_iter) || (rule == kModeANLS && !bf16);
    steps.push_back({rule, bf16, obj});
  }
  for (int r = 0; r < o->polish_rounds; ++r) {
    const int rule = o->polish_algo == HSN_ALGO_ANLS ? kModeANLS : kModeHALS;
    // HALS polish rounds on p_bf16 evaluate the objective every
    // kBf16PolishCheck-th round and on the last one (its reconstruction costs
    // the bfloat16 pass a third of its time); ANLS rounds have it from their
    // row solves and float32 rounds from their residual: every round.
    const bool on_bf16 = r < pol_bf16;
    const bool obj = !on_bf16 || rule == kModeANLS || (r + 1) % kBf16PolishCheck == 0 || r + 1 == pol_bf16;
    steps.push_back({rule, on_bf16, obj});
  }
  // The steps on p_bf16 form one run [bf16_lo, first_f32): the bulk when its
  // precision is BF16, then the first pol_bf16 polish rounds.  A stop fired
  // inside that run only ends it when float32 polish rounds follow; they
  // then decide the stop on the float32 objective.
  const int bf16_lo = (bf16 && o->max_iter > 0) ? 0 : o->max_iter;
  const int bf16_hi = o->max_iter + pol_bf16;
  const int first_f32_polish = (bf16_hi > bf16_lo && o->polish_rounds > pol_bf16) ? bf16_hi : -1;

  if (stats) HSN_HIP(ctx, hipEventRecord(ctx->ev0, st));
  if (nndsvd && (rc = nndsvd_init(ctx, st, p, ldp, p_bf16, ldb, n_p, int(n_k), K, V, D, ctx->ws, n_split,
                                 o->init == HSN_INIT_NNDSVDA)) != HSN_OK)
    return rc;
  if (o->init == HSN_INIT_MLP &&
      (rc = mlp_nmf_start(ctx, st, o->mlp, p, ldp, p_bf16, ldb, n_p, int(n_k), V, D, pool_buf, o->mlp_pooled, R.w,
                          wg_f32, (!steps.empty() && steps[0].bf16) ? wg_bf16 : 0)) != HSN_OK)
    return rc;
  launch_nmf_init(K, st, D, int(n_k), R.w, !steps.empty() && steps[0].rule == kModeANLS ? 1 : 0,
                  any_bf16 ? bf16_image_ldb(ldb) : 0);
  HSN_LAUNCHED(ctx);
  // Queue in chunks; between chunks read stop_at once (only when a stop test
  // is on).  The stop can only fire at a step that evaluates the objective, so
  // a chunk ends after a number of such steps that starts at 1 and doubles up
  // to 32: a run that converges at once (a learned start) queues no launches
  // past its stop, a long run pays few host round trips.
  int issued = 0, chunk_obj = 1;
  NmfCtrl hc{};
  hc.stop_at = INT32_MAX;
  // With stats requested, each stop-test read-back also brings the history
  // (one round trip); when the loop ends on such a read-back, the stats need
  // no second one.
  NmfCtrl *hcp = nullptr;
  double *hh = nullptr;
  if (stats) {
    if ((rc = ensure_host_stage(ctx, sizeof(NmfCtrl) + sizeof(double) * hist_cap)) != HSN_OK) return rc;
    hcp = static_cast<NmfCtrl *>(ctx->host_stage);
    hh = reinterpret_cast<double *>(static_cast<char *>(ctx->host_stage) + sizeof(NmfCtrl));
  }
  bool staged = false;
  // Host counts of the steps that ran: every step queued since the last
  // read-back whose index is below the stop index then read.
  std::vector<std::pair<int, int>> pending;  // queued index ranges [a, b)
  int ran_bulk = 0, ran_bf16 = 0, ran_f32 = 0;
  auto settle = [&](int stop_at) {
    for (const auto &r : pending)
      for (int i = r.first; i < std::min(r.second, stop_at); ++i) {
        if (i < o->max_iter) ++ran_bulk;
        else if (steps[i].bf16) ++ran_bf16;
        else ++ran_f32;
      }
    pending.clear();
  };
  auto read_back = [&]() -> hsn_status {
    if (stats) {
      HSN_HIP(ctx, hipEventRecord(ctx->ev1, st));
      HSN_HIP(ctx, hipMemcpyAsync(hcp, R.w.ctrl, sizeof(NmfCtrl), hipMemcpyDeviceToHost, st));
      HSN_HIP(ctx, hipMemcpyAsync(hh, R.w.hist, sizeof(double) * hist_cap, hipMemcpyDeviceToHost, st));
      HSN_HIP(ctx, hipStreamSynchronize(st));
      hc = *hcp;
      staged = true;
    } else {
      HSN_HIP(ctx, hipMemcpyAsync(&hc, R.w.ctrl, sizeof(NmfCtrl), hipMemcpyDeviceToHost, st));
      HSN_HIP(ctx, hipStreamSynchronize(st));
    }
    settle(hc.stop_at);
    return HSN_OK;
  };
  // A stop inside the bfloat16 steps [bf16_lo, bf16_hi) is confirmed by one
  // float32 round (the next unused one, f32_next) followed by a calibration
  // of the bfloat16 estimate against it; when that round misses the
  // tolerance, the bfloat16 polish rounds resume (up to kBf16Calibrations
  // times; a stop inside a bfloat16 bulk goes on with the float32 rounds),
  // then the float32 rounds run to the end.
  int f32_next = first_f32_polish;
  int cal_left = kBf16Calibrations;
  bool fell_back = false, first_test = true;
  while (issued < int(steps.size())) {
    int end = issued, n_obj = 0;
    while (end < int(steps.size()) && n_obj < chunk_obj) {
      if (steps[end].obj) ++n_obj;
      ++end;
      if (end == bf16_hi && f32_next > bf16_hi) break;  // the float32 rounds continue at f32_next
    }
    chunk_obj = std::min(2 * chunk_obj, 32);
    for (int i = issued; i < end; ++i) {
      const bool next_exact = (i + 1 < int(steps.size())) && steps[i + 1].rule == kModeANLS;
      if ((rc = queue_step(R, steps[i], i, next_exact, p, ldp, p_bf16, ldb, V, D)) != HSN_OK) return rc;
    }
    pending.push_back({issued, end});
    issued = end;
    if (issued == bf16_hi && f32_next > bf16_hi) issued = f32_next;
    staged = false;
    const bool confirm_possible = f32_next >= 0 && f32_next < int(steps.size());
    if (!stop_test || (issued >= int(steps.size()) && !confirm_possible)) continue;
    if ((rc = read_back()) != HSN_OK) return rc;
    if (fallback && first_test && hc.hist_len > 0 &&
        (hc.numeric || !std::isfinite(hc.last_est) || (hc.last_est - R.f_ref) / R.f_ref > o->mlp_fallback_rel)) {
      // The learned start is off: restart from NNDSVDa with the same
      // schedule (its scratch shares the workspace, whose NMF arrays the
      // initialisation below sets up again; the stream has drained).
      if ((rc = nndsvd_init(ctx, st, p, ldp, p_bf16, ldb, n_p, int(n_k), K, V, D, ctx->ws, n_split, true)) != HSN_OK)
        return rc;
      launch_nmf_init(K, st, D, int(n_k), R.w, !steps.empty() && steps[0].rule == kModeANLS ? 1 : 0,
                      any_bf16 ? bf16_image_ldb(ldb) : 0);
      HSN_LAUNCHED(ctx);
      fell_back = true;
      first_test = false;
      issued = 0;
      chunk_obj = 1;
      f32_next = first_f32_polish;
      cal_left = kBf16Calibrations;
      hc = NmfCtrl{};
      hc.stop_at = INT32_MAX;
      pending.clear();
      ran_bulk = ran_bf16 = ran_f32 = 0;
      staged = false;
      continue;
    }
    if (hc.hist_len > 0) first_test = false;
    if (hc.stop_at == INT32_MAX) continue;
    const int s = hc.stop_at - 1;  // the step whose objective met the tolerance
    if (hc.numeric || !(s >= bf16_lo && s < bf16_hi) || !confirm_possible) break;
    // confirm on p: one float32 round, then the calibration of the estimate
    launch_nmf_resume(st, R.w.ctrl);
    const int f = f32_next++;
    const bool next_exact = (f + 1 < int(steps.size())) && steps[f + 1].rule == kModeANLS;
    if ((rc = queue_step(R, steps[f], f, next_exact, p, ldp, p_bf16, ldb, V, D)) != HSN_OK) return rc;
    launch_nmf_calibrate(st, R.w.ctrl, R.w.hist, R.bias);
    HSN_LAUNCHED(ctx);
    pending.push_back({f, f + 1});
    if ((rc = read_back()) != HSN_OK) return rc;
    if (hc.stop_at != INT32_MAX) break;  // met on p (or numeric)
    chunk_obj = 1;
    if (cal_left > 0 && s >= o->max_iter && s + 1 < bf16_hi) {
      --cal_left;
      issued = s + 1;  // the bfloat16 rounds resume with the calibrated estimate
    } else {
      issued = f32_next;
    }
  }
  if (stats) {
    // One round trip (control block and the whole history into pinned
    // memory), unless the last stop test already brought them.
    if (!staged) {
      HSN_HIP(ctx, hipEventRecord(ctx->ev1, st));
      HSN_HIP(ctx, hipMemcpyAsync(hcp, R.w.ctrl, sizeof(NmfCtrl), hipMemcpyDeviceToHost, st));
      HSN_HIP(ctx, hipMemcpyAsync(hh, R.w.hist, sizeof(double) * hist_cap, hipMemcpyDeviceToHost, st));
      HSN_HIP(ctx, hipStreamSynchronize(st));
      hc = *hcp;
    }
    settle(hc.stop_at);
    float ms = 0.f;
    HSN_HIP(ctx, hipEventElapsedTime(&ms, ctx->ev0, ctx->ev1));
    stats->ms = ms;
    stats->iters = ran_bulk;
    stats->polish_bf16_done = ran_bf16;
    stats->polish_done = ran_bf16 + ran_f32;
    stats->fell_back = fell_back ? 1 : 0;
    stats->history_len = 0;
    double last = NAN;
    const int len = std::min(hc.hist_len, hist_cap);
    if (len > 0) {
      last = hh[len - 1];
      const int n_copy = std::min(len, stats->history_cap);
      for (int i = 0; i < n_copy; ++i) stats->history[i] = hh[i];
      stats->history_len = n_copy;
    }
    stats->objective = last;
    stats->rel_obj = stop_test ? (last - o->f_ref) / o->f_ref : NAN;
  }
  if ((stats || stop_test) && (hc.numeric || (stats && hc.hist_len > 0 && !std::isfinite(stats->objective))))
    return fail(ctx, HSN_ERR_NUMERIC, "nmf: the objective became %s at step %d (NaN or Inf in p or the factors)",
                std::isnan(stats ? stats->objective : NAN) ? "NaN" : "non-finite", hc.stop_at - 1);
  return HSN_OK;
}

extern "C" hsn_status hsn_nmf_set_launch(hsn_ctx *ctx, int anls_passes) {
  if (!ctx) return HSN_ERR_INVALID_ARG;
  if (anls_passes < 0 || anls_passes > 2)
    return hsn::fail(ctx, HSN_ERR_INVALID_ARG, "nmf launch: anls_passes must be 0, 1 or 2 (got %d)", anls_passes);
  ctx->nmf_anls_passes = anls_passes == 2 ? 2 : 1;
  return HSN_OK;
}
