/*
 * hsn.h -- C ABI of the MI355X (gfx950) library for the data-parallel hot
 * path of fast hyperspectral neutron tomography (arXiv 2410.22500):
 *
 *   -log normalisation (eq. 2, Appendix A)
 *   -> NMF subspace decomposition p ~ V D^T (eq. 4)
 *   -> K-channel parallel-beam projector A and adjoint A^T (eq. 3, eq. 5)
 *   -> per-channel least-squares reconstruction (eq. 5 with h = 0)
 *   -> subspace expansion x^h = x^s D^T (eq. 6)
 *
 * Conventions for every entry point
 *   - Array arguments are DEVICE pointers owned by the caller unless the
 *     comment says "host".  The library never frees, retains or reallocates
 *     a caller buffer past the call.
 *   - `stream` is a hipStream_t (NULL = the default stream).  All device work
 *     is ordered on it; outputs are valid once the stream has synchronised.
 *     Calls that return host-side statistics synchronise the stream.
 *   - Every call validates its arguments on the host before any launch and
 *     returns an hsn_status; on error nothing has been written and
 *     hsn_last_error(ctx) holds a message.  The library never aborts or prints.
 *   - Matrices are row-major with the last index fastest.  Pitches are in
 *     elements.  p rows are ordered (view, detector row, detector column), the
 *     paper's index order v, r, c; p columns are wavelength bins k.
 *   - Concurrent calls on one context must be serialised by the caller.
 */
#ifndef HSN_H
#define HSN_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  HSN_OK = 0,
  HSN_ERR_INVALID_ARG = 1,  /* NULL where required, bad enum, bad pitch/alignment */
  HSN_ERR_SHAPE = 2,        /* sizes out of the supported range */
  HSN_ERR_UNSUPPORTED = 3,  /* valid request the library does not implement */
  HSN_ERR_OOM = 4,          /* workspace allocation failed */
  HSN_ERR_DEVICE = 5,       /* a HIP runtime call failed */
  HSN_ERR_NUMERIC = 6       /* NaN/Inf detected in a result */
} hsn_status;

typedef struct hsn_ctx hsn_ctx;

/* Create a context bound to HIP device `device`; it owns the workspace. */
hsn_status hsn_create(hsn_ctx **ctx, int device);
void hsn_destroy(hsn_ctx *ctx);
/* Message of the last failed call on ctx ("" if none).  Valid until the next call. */
const char *hsn_last_error(const hsn_ctx *ctx);
/* Library ABI version (major*100 + minor). */
int hsn_version(void);

/* ------------------------------------------------------------------ */
/* Normalisation: eq. (2) p = -ln(y / y^o), with the Appendix A offset.  */
/* ------------------------------------------------------------------ */

typedef struct {
  int64_t n_views; /* N_v */
  int64_t n_rows;  /* N_r detector rows (= slices) */
  int64_t n_cols;  /* N_c detector columns */
  int64_t n_bins;  /* N_k wavelength bins */
} hsn_dims;

enum { HSN_U16 = 0, HSN_F32 = 1 };

/*
 * p[(v*N_r + r)*N_c + c][k] = -ln( max(y, f) / max(y^o, f) ) - b[v][k], then
 * clipped at 0 when clip_nonneg != 0.  (eq. 2; offset b from Appendix A.)
 *
 *   y       [N_v][N_r][N_c][N_k] counts, dtype y_dtype (HSN_U16 or HSN_F32)
 *   y_open  [N_r][N_c][N_k] open-beam counts, dtype y_open_dtype
 *   bg_mask optional [N_r][N_c] uint8, non-zero on background pixels B.  When
 *           given, b[v][k] = mean over B of the unclipped -ln(y/y^o)
 *           (Appendix A); when NULL, b = 0.  B must be non-empty.
 *   count_floor  f >= 0 applied to both counts (the log of 0 is undefined).
 *   p       [N_p][ldp] float32 output, ldp >= N_k.  May be NULL if p_bf16 is given.
 *   p_bf16  optional [N_p][ldb] bfloat16 (bits, round-to-nearest-even) copy
 *           for the BF16 NMF path; ldb >= N_k, ldb % 32 == 0; columns
 *           N_k..ldb-1 are written with zeros.  16-byte aligned.
 *   offset_b optional [N_v][N_k] float32 output of b (requires bg_mask).
 *   sumsq   optional device double: sum of p^2 over the float32 p values.
 *   bf16_bias optional device double (requires p_bf16): -||p - p_bf16||^2.
 *           For any V, D: ||p - V D^T||^2 = ||p_bf16 - V D^T||^2
 *           - ||p - p_bf16||^2 + 2 <p - p_bf16, p - V D^T>, and the last
 *           term is small when the rounding error is uncorrelated with the
 *           float32 residual, so an objective measured on p_bf16 plus this
 *           bias estimates the objective on p; hsn_nmf_opts.bf16_bias takes
 *           it (the NMF calibrates what is left against a float32 round).
 */
hsn_status hsn_normalize(hsn_ctx *ctx, const hsn_dims *dims,
                         const void *y, int y_dtype, const void *y_open, int y_open_dtype,
                         const uint8_t *bg_mask, float count_floor, int clip_nonneg,
                         float *p, int64_t ldp, uint16_t *p_bf16, int64_t ldb,
                         float *offset_b, double *sumsq, double *bf16_bias, void *stream);

/*
 * hsn_normalize for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * same arguments, same kernels and results, but no workspace is allocated.
 * The only scratch, 2 x 2048 doubles (32 KB) of per-block partial sums,
 * lives in a static device array of the library that each GPU holds until
 * the process ends; it is independent of the input size.  With bg_mask the
 * caller must pass offset_b (the offset is not kept in scratch), else
 * HSN_ERR_INVALID_ARG.  Calls on one GPU share that array: calls whose work
 * overlaps on one GPU (different streams or threads) race; calls ordered on
 * one stream do not.  No profiling events are recorded.
 */
hsn_status hsn_normalize_noalloc(hsn_ctx *ctx, const hsn_dims *dims,
                                 const void *y, int y_dtype, const void *y_open, int y_open_dtype,
                                 const uint8_t *bg_mask, float count_floor, int clip_nonneg,
                                 float *p, int64_t ldp, uint16_t *p_bf16, int64_t ldb,
                                 float *offset_b, double *sumsq, double *bf16_bias, void *stream);

/*
 * hsn_normalize plus the input of the learned warm start in the same pass:
 * pooled [N_p][256], row i of p average-pooled to 256 values exactly as
 * hsn_mlp_pool pools p_bf16 (bfloat16-rounded p, bin j covering
 * [floor(j N_k/256), ceil((j+1) N_k/256)), summed in bin order in float32),
 * stored as bfloat16 bits (pooled_precision HSN_PREC_BF16) or float32
 * (HSN_PREC_FP32): the precision of the network that will read it (see
 * hsn_nmf_opts.mlp_pooled).  p and p_bf16 may both be NULL.  Requires
 * N_k <= 2048; pooled 4-byte aligned.  Other arguments as hsn_normalize.
 */
hsn_status hsn_normalize_pooled(hsn_ctx *ctx, const hsn_dims *dims,
                                const void *y, int y_dtype, const void *y_open, int y_open_dtype,
                                const uint8_t *bg_mask, float count_floor, int clip_nonneg,
                                float *p, int64_t ldp, uint16_t *p_bf16, int64_t ldb,
                                float *offset_b, double *sumsq, double *bf16_bias, void *pooled,
                                int pooled_precision, void *stream);

/* ------------------------------------------------------------------ */
/* Subspace extraction: eq. (4) (V, D) = argmin_{V,D>=0} ||p - V D^T||^2 */
/* ------------------------------------------------------------------ */

enum { HSN_ALGO_MU = 0,    /* Lee-Seung multiplicative updates, V then D      */
       HSN_ALGO_ANLS = 1,  /* exact row-wise NNLS for V, then for D            */
       HSN_ALGO_HALS = 2 };/* HALS column sweeps (the paper's Fast HALS), V then D */
enum { HSN_PREC_FP32 = 0,  /* float32 p, float32 arithmetic               */
       HSN_PREC_BF16 = 1 };/* bfloat16 p on MFMA, float32 accumulation   */
enum { HSN_INIT_USER = 0,  /* V and D hold the start on entry                    */
       HSN_INIT_NNDSVDA = 1,  /* NNDSVD with zeros filled by mean(p) (Boutsidis &
                                 Gallopoulos; the paper's initialisation); needs p,
                                 uses p_bf16 for the Gram P^T P when given      */
       HSN_INIT_MLP = 2,      /* learned warm start: V0 = opts.mlp(pooled p_bf16),
                                 D0 = argmin_{D>=0} ||p - V0 D^T|| row by row, exact
                                 zeros of D0 set to 1e-6 mean(D0); needs p, and
                                 p_bf16 unless opts.mlp_pooled is given */
       HSN_INIT_NNDSVD = 3 }; /* plain NNDSVD (the paper's start with its exact zeros
                                 kept), for HALS and ANLS; MU keeps zero entries zero */

typedef struct hsn_mlp hsn_mlp;

typedef struct {
  int k;              /* K = N_s, 1..8 */
  int algo;           /* HSN_ALGO_* for the bulk iterations */
  int precision;      /* HSN_PREC_* for the bulk iterations */
  int init;           /* HSN_INIT_* */
  int max_iter;       /* bulk iterations, >= 0 */
  int check_every;    /* objective evaluated every this many iterations (>= 1) */
  int polish_rounds;  /* rounds after the bulk (>= 0) */
  int polish_algo;    /* HSN_ALGO_ANLS or HSN_ALGO_HALS for the polish rounds */
  int polish_bf16_rounds; /* at most this many polish rounds run first on p_bf16 (needs p_bf16),
                             the remaining ones on the float32 p (see the stop test below) */
  double rel_obj_tol; /* stop when (f - f_ref)/f_ref <= tol; ignored if f_ref <= 0 */
  double f_ref;       /* reference objective f* (> 0 enables the stop test) */
  const hsn_mlp *mlp; /* network for HSN_INIT_MLP (its k must equal k), else NULL */
  const void *mlp_pooled; /* optional for HSN_INIT_MLP: the network input already pooled
                             (hsn_normalize_pooled, in the network's precision, [N_p][256]);
                             NULL: pooled here from p_bf16 */
  const double *bf16_bias; /* optional device double -||p - p_bf16||^2 (hsn_normalize's
                              bf16_bias) for the stop test of steps on p_bf16; NULL = 0 */
  double mlp_fallback_rel; /* HSN_INIT_MLP with the stop test on: when the first evaluated
                              objective of the learned start has (f - f_ref)/f_ref above this
                              (or is NaN/Inf), the run restarts from NNDSVDa with the same
                              schedule (stats.fell_back = 1); <= 0: off */
  int anls_extrapolate;    /* 1: ANLS rounds (polish, or an ANLS bulk) extrapolate D between
                              rounds (Ang & Gillis 2019): D_hat = max(0, D_new + beta
                              (D_new - D_prev)) feeds the next round's V solve, with beta
                              adapted from the round objectives (a rise resets the round to its
                              exact D); needs the objective every round.  0: plain ANLS */
} hsn_nmf_opts;

typedef struct {
  int iters;          /* bulk iterations done */
  int polish_done;    /* polish rounds done */
  double objective;   /* last evaluated objective (see below) */
  double rel_obj;     /* (objective - f_ref)/f_ref, or NaN without f_ref */
  double *history;    /* host, optional: evaluated objectives in order */
  int history_cap;    /* capacity of history */
  int history_len;    /* entries written */
  float ms;           /* device time of the call */
  int polish_bf16_done; /* of polish_done, the rounds run on p_bf16 */
  int fell_back;      /* 1 when a learned start was replaced by NNDSVDa (the counts and the
                         history are those of the restarted run) */
} hsn_nmf_stats;

/*
 * Runs the bulk iterations, then the polish rounds, on V [N_p][K] and
 * D [N_k][K] (float32, in/out, both strictly positive on entry for MU).
 * Each evaluated objective is f(V_{t+1}, D_t) = ||p - V_{t+1} D_t^T||_F^2 over
 * the float32 p (steps on p_bf16: over the bfloat16 p), computed from the
 * residual inside the pass, i.e. the objective after the V half-step; for
 * every algorithm it is non-increasing in exact arithmetic.  An ANLS round
 * solves every row of V exactly inside one streaming pass (the NNLS of a
 * row by enumeration of its supports with the inverses of the principal
 * submatrices of D^T D in float64), then every row of D (Lawson-Hanson with
 * float64 Cholesky factors).  The stop test fires on a step whose objective
 * meets (f - f_ref)/f_ref <= rel_obj_tol.  On a step over p_bf16 (a BF16
 * bulk iteration or one of the first polish_bf16_rounds polish rounds) f is
 * the bfloat16 objective plus *bf16_bias plus a calibration (0 at first).
 * When float32 polish rounds follow, such a stop is confirmed by one float32
 * round; if that round misses the tolerance, the calibration is set to the
 * float32 objective minus the last bfloat16 estimate and the bfloat16 rounds
 * resume (at most twice; then the float32 rounds run).  The float32 rounds
 * decide the stop on the float32 objective (stats count only the steps run).
 *   p      [N_p][ldp] float32, ldp % 4 == 0, 16-byte aligned (needed for FP32
 *          steps and for the NNDSVDa and learned starts; may be NULL otherwise)
 *   p_bf16 [N_p][ldb] bfloat16 with zero padding, ldb % 32 == 0, ldb <= 2048
 *          (steps on the bfloat16 p)
 * Returns HSN_OK also when max_iter is reached before the tolerance.  stats
 * (host) may be NULL; filling it synchronises the stream.  An evaluated
 * objective that is NaN or infinite (NaN or Inf in p, overflowing factors)
 * stops the run at that step; the call then returns HSN_ERR_NUMERIC when
 * stats are requested or a stop test is on (otherwise the host never reads
 * the device state, and the caller finds the non-finite values in V or D).
 */
hsn_status hsn_subspace_nmf(hsn_ctx *ctx, const float *p, int64_t ldp,
                            const uint16_t *p_bf16, int64_t ldb,
                            int64_t n_p, int64_t n_k, float *V, float *D,
                            const hsn_nmf_opts *opts, hsn_nmf_stats *stats, void *stream);

/*
 * Form of the ANLS rounds of hsn_subspace_nmf on ctx (a tuning knob; both
 * forms compute the same exact block minimisation of eq. (4)):
 *   anls_passes 1 (default, also 0): one fused streaming pass per round;
 *   anls_passes 2: a pass for N_V = P D, a kernel solving the V rows
 *     (Lawson-Hanson), a pass for N_D = P^T V (float32 p only; rounds on
 *     p_bf16 are always fused).
 * Other values: HSN_ERR_INVALID_ARG.
 */
hsn_status hsn_nmf_set_launch(hsn_ctx *ctx, int anls_passes);

/*
 * Many independent decompositions (eq. 4) of uneven size in one go: every
 * phase of an iteration is ONE launch per kernel shape over the workgroups
 * of all its instances (per-instance descriptors and block ranges), and with
 * HSN_BATCH_GRAPH the iteration chunks are captured once into hipGraphs and
 * replayed.  Schedule (from opts; opts.k is ignored, each problem has its
 * own k): opts.max_iter MU iterations (objective every check_every) on the
 * float32 p (precision HSN_PREC_FP32) or on the bfloat16 p on the matrix
 * cores (HSN_PREC_BF16: each problem's p_bf16), then up to
 * opts.polish_rounds float32 ANLS rounds (N_V pass, row solves, N_D pass);
 * algo must be HSN_ALGO_MU, init HSN_INIT_USER, polish_algo HSN_ALGO_ANLS,
 * polish_bf16_rounds 0.  Instance i stops on its own when f_ref > 0 and its
 * relative objective reaches opts.rel_obj_tol; its kernels then return at
 * once.  Bulk iterations on the bfloat16 p record their objective (on
 * p_bf16) but never stop an instance: the float32 rounds decide.
 * Flags: HSN_BATCH_GRAPH captures and replays graphs (cached in ctx per batch
 * shape); HSN_BATCH_AUTOTUNE, on the first call for a batch shape, times the
 * candidate partitions and keeps the fastest: workgroup budgets of the
 * float32 pass (rows of p per workgroup) and, for the bfloat16 bulk, 1, 2, 4
 * or 8 16-row tiles per MFMA-pass workgroup.  With the environment variable
 * HSN_TUNE_CACHE naming a file, tuned choices are kept there (a JSON object
 * keyed by device and batch shape) and reused by later processes.
 * Without AUTOTUNE every instance is partitioned exactly as hsn_subspace_nmf
 * would partition it alone (ANLS rounds in the two-pass form,
 * hsn_nmf_set_launch(ctx, 2)), so its results are bitwise those of that call.
 * stats: optional host array [n]; ms is the device time of the whole batch.
 */
typedef struct {
  const float *p;   /* [n_p][ldp] float32, ldp >= n_k, ldp % 4 == 0, 16-byte aligned */
  int64_t ldp;
  int64_t n_p, n_k; /* 1 <= n_k <= 2048 */
  int k;            /* 1..8 */
  float *V;         /* [n_p][k] in/out */
  float *D;         /* [n_k][k] in/out */
  double f_ref;     /* > 0 enables this instance's stop test */
  const uint16_t *p_bf16; /* HSN_PREC_BF16: [n_p][ldb] bfloat16 p with zero padding, 16-byte
                             aligned, n_k <= ldb <= 2048, ldb % 32 == 0; else ignored */
  int64_t ldb;
} hsn_nmf_problem;

enum { HSN_BATCH_GRAPH = 1, HSN_BATCH_AUTOTUNE = 2 };

hsn_status hsn_subspace_nmf_batched(hsn_ctx *ctx, int n, const hsn_nmf_problem *probs,
                                    const hsn_nmf_opts *opts, int flags, hsn_nmf_stats *stats,
                                    void *stream);
/* Text description of the plan the last batched call on ctx used (groups,
 * workgroups, tuning timings); valid until the next call. */
const char *hsn_batched_plan_info(const hsn_ctx *ctx);

/* ------------------------------------------------------------------ */
/* Projector A (eq. 3 / eq. 5), K channels, all slices in one launch.   */
/* ------------------------------------------------------------------ */

/*
 * Parallel beam, detector row r sees image slice r (N_c x N_c pixels, pitch
 * 1, centres at index - (N_c-1)/2).  Matrix entries (Joseph interpolation
 * written as a footprint, identical in A and A^T):
 *   a_{(v,c),(j,i)} = (1/w_v) max(0, 1 - |d|/w_v),
 *   d = s_c - (x_i cos t_v + y_j sin t_v),  w_v = max(|cos t_v|, |sin t_v|).
 * Volume x [N_r][N_c][N_c][K] (slice, image row j, column i, channel);
 * sinogram s [N_v][N_r][N_c][K] (the V layout of hsn_subspace_nmf).
 */
typedef struct {
  int64_t n_views;       /* N_v */
  int64_t n_slices;      /* N_r */
  int64_t n_cols;        /* N_c (= image size) */
  int k;                 /* channels, 1..8 */
  const double *angles;  /* host [N_v] radians, or NULL for t_v = v*pi/N_v */
} hsn_geom;

/* s = alpha * A x + beta * s  (beta == 0: s is not read). */
hsn_status hsn_project(hsn_ctx *ctx, const hsn_geom *g, const float *x, float *s,
                       float alpha, float beta, void *stream);
/* x = alpha * A^T s + beta * x  (beta == 0: x is not read). */
hsn_status hsn_backproject(hsn_ctx *ctx, const hsn_geom *g, const float *s, float *x,
                           float alpha, float beta, void *stream);

/*
 * Launch shape of hsn_project, hsn_backproject and hsn_cgls: a tuning knob
 * for the operators of eq. (3)/(5); every shape computes the same entries.
 *   views   A stages the slice image through LDS for `views` views of one
 *           orientation per workgroup: 1, 2 or 4.
 *   split   A runs `split` copies of those rays per workgroup, each over
 *           every split-th image row, summed in copy order: 1, 2, 4, 8, 16
 *           (reduced until the workgroup fits 1024 threads).
 *   voxels  A^T stages the slice's sinogram rows through LDS for `voxels`
 *           voxels per thread: 1, 2 or 4.
 *   threads A^T workgroup size: 64, 128, 256, 512 or 1024.
 * 0 = chosen from the geometry and the CU count (the default); views or
 * voxels -1 = the gather kernel for that operator, which reads every tap
 * from the caches.  Other values: HSN_ERR_INVALID_ARG.  With split 1 (and
 * for A^T always) the staged and gather kernels give the same float32
 * values bit for bit; split > 1 changes the order of the sums per ray.
 * Geometries whose staged row does not fit 60 KB of LDS ((n_cols + 2 pad) k
 * floats, pad = 2 pixels for k = 2 or 4 and 4 otherwise, rounded up to a
 * multiple of 4 for k >= 5), or n_cols > 1024 for A, use the gather
 * kernels whatever is set.
 */
hsn_status hsn_projector_set_launch(hsn_ctx *ctx, int views, int split, int voxels, int threads);
/* The shape the next call would use for g: shape[0..3] = views, split,
 * voxels, threads as above, 0 where that operator runs the gather kernel. */
hsn_status hsn_projector_launch_info(hsn_ctx *ctx, const hsn_geom *g, int *shape);

/*
 * eq. (5) with h = 0: x_j = argmin ||V_j - A x_j||^2 for every channel j by
 * CGLS from x = 0, n_iter iterations (one A and one A^T each), all channels
 * at once with per-channel scalars kept on the device (no host sync).
 *   sino [N_v][N_r][N_c][K] in, x [N_r][N_c][N_c][K] out,
 *   resid optional [n_iter+1][K] float64: ||b - A x_i|| per channel.
 */
hsn_status hsn_cgls(hsn_ctx *ctx, const hsn_geom *g, const float *sino, float *x,
                    int n_iter, double *resid, void *stream);

/*
 * eq. (5) with the qGGMRF prior h (the paper's MBIR), every channel j:
 *   x_j = argmin 1/(2 sigma_v[j]^2) ||V_j - A x_j||^2 + h(x_j),
 *   h(x) = sum over 8-neighbour pairs {s, r} inside a slice of
 *          b_sr rho(x_s - x_r),  b = w1 (nearest), w1/sqrt(2) (diagonal),
 *          w1 = 1/(4 + 2 sqrt(2)), pixels outside the image omitted;
 *   rho(d) = |d|^p / (p sx^p) u / (1 + u),  u = |d / (T sx)|^(2-p),  sx = sigma_x[j]
 * (q = 2; the paper gives no prior parameters: these are the standard
 * qGGMRF form and a stated reading).  Majorisation-minimisation: each of
 * n_outer iterations takes the symmetric-bound quadratic surrogate of h at
 * the current x and runs n_inner conjugate-gradient iterations on
 * (A^T A + sigma_v^2 L) x = A^T V from the current x (the cost never
 * increases in exact arithmetic).  Per inner iteration: one A, one A^T, one
 * prior stencil and two small kernels; per outer iteration one more A,
 * A^T and stencil.  No positivity constraint.
 *   sino [N_v][N_r][N_c][K] float32 in (device);
 *   x [N_r][N_c][N_c][K] float32 in/out (device): the start on entry
 *     (zeros for a cold start), the estimate on return;
 *   sigma_v, sigma_x: host arrays of K doubles, each finite and > 0;
 *   1 <= p <= 2, T > 0.
 * Errors (nothing launched): HSN_ERR_INVALID_ARG for NULL pointers, bad
 * parameters, misaligned x or sino; HSN_ERR_SHAPE for bad geometry;
 * HSN_ERR_OOM if the workspace (6 volumes + 1 sinogram) cannot be allocated.
 */
hsn_status hsn_mbir(hsn_ctx *ctx, const hsn_geom *g, const float *sino, float *x, const double *sigma_v,
                    const double *sigma_x, double p, double T, int n_outer, int n_inner, void *stream);

/*
 * Filtered backprojection, the per-channel reconstruction the paper uses
 * for its DHR baseline (one FBP per wavelength bin) and for "FHR with FBP"
 * (FBP of the K subspace sinograms); Section V, Tables II and IV.  The
 * filter is the band-limited ramp sampled at the detector pitch (Ram-Lak:
 * h[0] = 1/4, h[d] = -1/(pi^2 d^2) for odd d, 0 for even d != 0), applied
 * to every detector row as a zero-padded linear convolution over the N_c
 * columns; then x = (pi / N_v) A^T q with the adjoint of hsn_backproject.
 *   sino [N_v][N_r][N_c] rays of k floats each, ray i at sino + i * ld
 *        (ld >= k floats; ld = k: contiguous [N_v][N_r][N_c][k]; ld > k
 *        reads k consecutive bins of a wider row, e.g. 8 bins of p),
 *        4-byte aligned;
 *   x    [N_r][N_c][N_c][k] out (alignment as hsn_backproject).
 * Requires N_c * k <= 8192.  Workspace: N_v N_r N_c k floats.
 */
hsn_status hsn_fbp(hsn_ctx *ctx, const hsn_geom *g, const float *sino, int64_t ld, float *x, void *stream);

/*
 * The FHR hot path of one scan in one call, in the order of Alg. 1 with the
 * h = 0 reconstruction: eq. (2) (hsn_normalize, or hsn_normalize_pooled for
 * a learned start, floor count_floor, clipped at 0, no offset), eq. (4)
 * (hsn_subspace_nmf with *opts; for HSN_INIT_MLP its mlp_pooled is set to
 * `pooled`), eq. (5) (hsn_cgls, cgls_iters iterations, on V read as the
 * sinogram [N_v][N_r][N_c][K], angles as hsn_geom.angles), and eq. (6)
 * (hsn_rehydrate of [vox_begin, vox_end) x [bin_begin, bin_end) into xh,
 * skipped when xh is NULL).  Same kernels, same results as those calls in
 * sequence; the host's turn-around after the NMF's convergence read-back
 * stays in C.
 *   p [N_p][ldp] float32 and pooled [N_p][256] (learned start only, in the
 *   network's precision): caller-owned intermediates (device);
 *   p_bf16 [N_p][ldb] (optional, device): also written by the normalisation
 *   when given, with -||p - p_bf16||^2 into a context scratch double
 *   that the NMF's opts.bf16_bias then points to (required when
 *   opts.polish_bf16_rounds > 0 or opts.precision is HSN_PREC_BF16);
 *   V [N_p][K], D [N_k][K]: in/out as for hsn_subspace_nmf;
 *   x [N_r][N_c][N_c][K] float32 out; stats as for hsn_subspace_nmf.
 * Errors: those of the composed calls (the first failing one returns; the
 * earlier ones have been queued); HSN_ERR_INVALID_ARG for NULL required
 * pointers or a learned start without opts.mlp or pooled.
 */
hsn_status hsn_fhr_step(hsn_ctx *ctx, const hsn_dims *dims, const void *y, int y_dtype, const void *y_open,
                        int y_open_dtype, float count_floor, float *p, int64_t ldp, uint16_t *p_bf16,
                        int64_t ldb, void *pooled, float *V, float *D, const hsn_nmf_opts *opts,
                        hsn_nmf_stats *stats, const double *angles, int cgls_iters, float *x, int64_t vox_begin,
                        int64_t vox_end, int64_t bin_begin, int64_t bin_end, float *xh, int64_t ldh,
                        void *stream);

/* ------------------------------------------------------------------ */
/* Subspace expansion: eq. (6) x^h = x^s D^T over a voxel x bin range.   */
/* ------------------------------------------------------------------ */

/*
 * xh[v - vox_begin][b - bin_begin] = sum_j xs[v][j] * D[b][j]
 * for v in [vox_begin, vox_end), b in [bin_begin, bin_end).
 *   xs [n_x][K], D [n_k][K] float32; xh [vox_end-vox_begin][ldh] float32,
 *   ldh >= bin_end - bin_begin.
 */
hsn_status hsn_rehydrate(hsn_ctx *ctx, const float *xs, const float *D, int64_t n_x, int64_t n_k,
                         int k, int64_t vox_begin, int64_t vox_end, int64_t bin_begin,
                         int64_t bin_end, float *xh, int64_t ldh, void *stream);

/* ------------------------------------------------------------------ */
/* Fast material decomposition tail (Alg. 2, eq. 7-9), semi-supervised.  */
/* ------------------------------------------------------------------ */

/*
 * From the reconstructed subspace volume x^s [n_x][k] (hsn_cgls output), the
 * subspace spectra D^s [n_k][k] (hsn_subspace_nmf's D) and one region label
 * per voxel (labels[n] in 0..n_m-1, or -1 for a voxel in no region; the
 * paper's masks M_i):
 *   T  [n_m][k]   T[i][j] = mean of x^s[n][j] over the voxels of region i   eq. (7)
 *                 (a region without voxels gives a zero row)
 *   xm [n_x][n_m] xm[n] = argmin_{x >= 0} ||x^s[n] - x T||^2, per voxel       eq. (8)
 *   Dm [n_k][n_m] Dm = D^s T^T, the material spectra                         eq. (9)
 * All outputs float32 (device); sums and solves in float64.  k, n_m in 1..8.
 */
hsn_status hsn_fmd(hsn_ctx *ctx, const float *xs, int64_t n_x, int k, const int32_t *labels, int n_m,
                   const float *Ds, int64_t n_k, float *T, float *xm, float *Dm, void *stream);

/* ------------------------------------------------------------------ */
/* Learned warm start of eq. (4): spectrum -> K coefficients.            */
/* ------------------------------------------------------------------ */

/*
 * The paper starts its NMF from NNDSVD; this network replaces that start
 * with a prediction of the rows of V.  A ray's spectrum is average-pooled to
 * 256 bins (bin i covers [floor(i N_k/256), ceil((i+1) N_k/256))), then
 *   h1 = GELU(x W1 + b1), h2 = GELU(h1 W2 + b2), v = softplus(h2 W3 + b3),
 * GELU(z) = z Phi(z) (erf form), softplus(z) = log(1 + e^z).  Parameters,
 * flat float32 in this order (row-major): W1[256][128], b1[128],
 * W2[128][128], b2[128], W3[128][K], b3[K]; n = 49408 + 129 K.
 * Precision HSN_PREC_BF16: bfloat16 weights and activations on MFMA with
 * float32 accumulation (float32 master weights and Adam state);
 * HSN_PREC_FP32: the same network in float32 throughout.  Inputs x of a
 * network are [n][256] in its precision: bfloat16 bits for BF16, float32
 * for FP32.  Training minimises the mean squared error over the batch and
 * the K outputs with Adam.
 */
enum { HSN_MLP_IN = 256, HSN_MLP_HIDDEN = 128 };

int64_t hsn_mlp_n_params(int k);
/* Creates a network on ctx's device; params_host (host, n floats) or NULL for
 * all-zero parameters.  The network belongs to the caller (hsn_mlp_destroy). */
hsn_status hsn_mlp_create(hsn_ctx *ctx, hsn_mlp **mlp, int k, int precision, const float *params_host);
void hsn_mlp_destroy(hsn_mlp *mlp);
/* Host copies of the float32 master parameters (synchronous). */
hsn_status hsn_mlp_get_params(hsn_ctx *ctx, const hsn_mlp *mlp, float *params_host);
hsn_status hsn_mlp_set_params(hsn_ctx *ctx, hsn_mlp *mlp, const float *params_host);
int hsn_mlp_k(const hsn_mlp *mlp);
int hsn_mlp_precision(const hsn_mlp *mlp);

/* x[i][.] = the 256-bin average pooling of row i of p_bf16 [n_p][ldb]
 * (n_k bins), written as x_dtype: HSN_PREC_BF16 (bits, round to nearest even)
 * or HSN_PREC_FP32. */
hsn_status hsn_mlp_pool(hsn_ctx *ctx, const uint16_t *p_bf16, int64_t ldb, int64_t n_p, int64_t n_k,
                        int x_dtype, void *x, void *stream);
/* y [n][K] float32 = network(x [n][256]). */
hsn_status hsn_mlp_forward(hsn_ctx *ctx, const hsn_mlp *mlp, const void *x, int64_t n, float *y, void *stream);
/* Mean squared error of network(x) against target [n][K] float32 over all n
 * rows as one batch: *loss (device double) and its gradient grad (device,
 * n_params float32, parameter order above). */
hsn_status hsn_mlp_loss_grad(hsn_ctx *ctx, const hsn_mlp *mlp, const void *x, const float *target, int64_t n,
                             float *grad, double *loss, void *stream);

typedef struct {
  int epochs;          /* passes over the data */
  int batch;           /* rows per Adam step (the last batch of an epoch may be short), 1..65536 */
  float lr, beta1, beta2, eps;  /* Adam */
  uint64_t seed;       /* shuffle seed: epoch e visits the rows in a seeded permutation */
} hsn_train_opts;

/* Adam on the mean squared error over shuffled mini-batches of (x, target).
 * loss_hist (host, optional, [epochs]): mean loss of the batches of each
 * epoch.  Adam's step counter persists in the network across calls.  Synchronises
 * the stream once per epoch. */
hsn_status hsn_mlp_train(hsn_ctx *ctx, hsn_mlp *mlp, const void *x, const float *target, int64_t n,
                         const hsn_train_opts *opts, double *loss_hist, void *stream);
/* V0 [n_p][K] float32 = network(pool(p_bf16)): the pooled inputs go through
 * the context's workspace. */
hsn_status hsn_mlp_infer(hsn_ctx *ctx, const hsn_mlp *mlp, const uint16_t *p_bf16, int64_t ldb, int64_t n_p,
                         int64_t n_k, float *V0, void *stream);
/* Binary file: magic "HSNMLP01", int32 k, int32 precision, int64 Adam step,
 * then float32 [n] parameters, [n] Adam first and [n] second moments (little
 * endian), so training can resume. */
hsn_status hsn_mlp_save(hsn_ctx *ctx, const hsn_mlp *mlp, const char *path);
hsn_status hsn_mlp_load(hsn_ctx *ctx, hsn_mlp **mlp, const char *path);

/*
 * Canonical form of an NMF pair (the factorisation is unique only up to
 * column scaling and permutation): D's columns scaled to unit l2 norm, V's
 * scaled inversely (zero columns keep scale 1), then columns reordered, in
 * place.  With library [n_k][K] float32 (device) the order maximises the sum
 * of cosines between the reordered D columns and the library columns (first
 * such permutation in lexicographic order); without it, columns are sorted
 * by descending l2 norm of the scaled V (stable).  These are the coefficient
 * targets of the warm-start network.
 */
hsn_status hsn_canonicalize(hsn_ctx *ctx, float *V, int64_t n_p, float *D, int64_t n_k, int k,
                            const float *library, void *stream);

/* ------------------------------------------------------------------ */
/* Kernel timing for roofline reports.                                   */
/* ------------------------------------------------------------------ */

enum {
  HSN_KERN_NMF_PASS = 0,    /* float32 streaming passes over p inside hsn_subspace_nmf */
  HSN_KERN_PROJECT = 1,     /* the forward projector kernel */
  HSN_KERN_BACKPROJECT = 2, /* the adjoint projector kernel */
  HSN_KERN_NORMALIZE = 3,   /* the normalisation stream kernel */
  HSN_KERN_NMF_PASS_BF16 = 4, /* bfloat16 (MFMA) streaming passes over p */
  HSN_KERN_MLP_ROWS = 5,    /* warm-start network: per-row layers (inference; training forward+backward) */
  HSN_KERN_MLP_WGRAD = 6,   /* warm-start network: weight-gradient contraction over the batch */
  HSN_KERN_NNDSVD_GRAM = 7, /* NNDSVD start: the Gram P^T P on MFMA */
  HSN_KERN_MLP_POOL = 8,    /* warm-start network: pooling of p_bf16 rows to 256 bins */
  HSN_KERN_FBP_FILTER = 9,  /* FBP: the ramp filter of the detector rows */
  HSN_KERN_COUNT = 10
};

/* When on != 0, every launch of the kernels above is bracketed by a pair of
 * hipEvents recorded on the launch's stream (small overhead per launch). */
hsn_status hsn_profile_enable(hsn_ctx *ctx, int on);
/* Synchronises the recorded events of `kernel` and returns the summed device
 * time (ms) and launch count since the last reset; reset != 0 clears them. */
hsn_status hsn_profile_read(hsn_ctx *ctx, int kernel, double *total_ms, int64_t *launches, int reset);

#ifdef __cplusplus
}
#endif

#endif /* HSN_H */
