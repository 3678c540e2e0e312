// The FHR hot path of one scan in one call (Alg. 1 with the h = 0
// reconstruction): eq. (2) normalisation, eq. (4) subspace NMF, eq. (5)
// per-channel CGLS on the K subspace sinograms, eq. (6) expansion of a
// voxel x bin range.  It composes the entry points of the other files on
// one stream; its only purpose is to keep the host's turn-around after the
// NMF's convergence read-back (the one synchronisation of the path) in C.
#include "common.hpp"

extern "C" hsn_status hsn_fhr_step(hsn_ctx *ctx, const hsn_dims *dims, const void *y, int y_dtype,
                                   const void *y_open, int y_open_dtype, float count_floor, float *p, int64_t ldp,
                                   uint16_t *p_bf16, int64_t ldb, void *pooled, float *V, float *D,
                                   const hsn_nmf_opts *opts, hsn_nmf_stats *stats, const double *angles,
                                   int cgls_iters, float *x, int64_t vox_begin, int64_t vox_end, int64_t bin_begin,
                                   int64_t bin_end, float *xh, int64_t ldh, void *stream) {
  if (!ctx) return HSN_ERR_INVALID_ARG;
  if (!dims || !opts || !p || !V || !D || !x)
    return hsn::fail(ctx, HSN_ERR_INVALID_ARG, "fhr_step: dims, opts, p, V, D and x are required");
  if (cgls_iters < 0) return hsn::fail(ctx, HSN_ERR_INVALID_ARG, "fhr_step: cgls_iters must be >= 0");
  const bool learned = opts->init == HSN_INIT_MLP;
  if (learned && (!opts->mlp || !pooled))
    return hsn::fail(ctx, HSN_ERR_INVALID_ARG, "fhr_step: the learned start needs opts.mlp and a pooled buffer");
  const bool uses_bf16 = opts->polish_bf16_rounds > 0 || (opts->precision == HSN_PREC_BF16 && opts->max_iter > 0);
  if (uses_bf16 && !p_bf16)
    return hsn::fail(ctx, HSN_ERR_INVALID_ARG, "fhr_step: steps on the bfloat16 p need a p_bf16 buffer");
  const int64_t n_p = dims->n_views * dims->n_rows * dims->n_cols;
  const int64_t n_x = dims->n_rows * dims->n_cols * dims->n_cols;
  // -||p - p_bf16||^2 for the stop test of the bfloat16 rounds
  double *bias = p_bf16 ? ctx->dscalars : nullptr;
  hsn_status rc;
  if (learned) {
    rc = hsn_normalize_pooled(ctx, dims, y, y_dtype, y_open, y_open_dtype, nullptr, count_floor, 1, p, ldp, p_bf16,
                              ldb, nullptr, nullptr, bias, pooled, hsn_mlp_precision(opts->mlp), stream);
  } else {
    rc = hsn_normalize(ctx, dims, y, y_dtype, y_open, y_open_dtype, nullptr, count_floor, 1, p, ldp, p_bf16, ldb,
                       nullptr, nullptr, bias, stream);
  }
  if (rc != HSN_OK) return rc;
  hsn_nmf_opts o = *opts;
  if (learned) o.mlp_pooled = pooled;
  if (bias) o.bf16_bias = bias;
  if ((rc = hsn_subspace_nmf(ctx, p, ldp, p_bf16, ldb, n_p, dims->n_bins, V, D, &o, stats, stream)) != HSN_OK)
    return rc;
  const hsn_geom g{dims->n_views, dims->n_rows, dims->n_cols, opts->k, angles};
  if ((rc = hsn_cgls(ctx, &g, V, x, cgls_iters, nullptr, stream)) != HSN_OK) return rc;
  if (xh)
    rc = hsn_rehydrate(ctx, x, D, n_x, dims->n_bins, opts->k, vox_begin, vox_end, bin_begin, bin_end, xh, ldh, stream);
  return rc;
}
