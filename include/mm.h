/*
 * mm.h -- C ABI of the MI355X maximum-likelihood map-maker (libmm.so).
 *
 * The library solves the map-making normal equations of the MADmap paper
 * (Cantalupo et al., arXiv:0906.1775, Algorithm section, eq. pcgSystem):
 *
 *     H m = b,   H = P^T N^-1 P,   b = P^T N^-1 d,
 *
 * by preconditioned conjugate gradients (Implementation section).  P is the
 * sparse pointing matrix of the Formalism section (the paper calls it A):
 * one unit weight per sample for temperature, or the three weights
 * (1/2, sin(2a_t)/2, cos(2a_t)/2) of (I, Q, U) for an ideal polarimeter.
 * N^-1 is block diagonal with one banded Toeplitz block per stationary
 * interval, (N^-1)_{t,t'} = f(|t - t'|) for |t - t'| < n_c (Weighting
 * section), applied by overlap-save FFTs.  The preconditioner is the
 * white-noise block inverse (P^T W^-1 P)^-1 with W^-1 = diag(N^-1), or the
 * point-Jacobi diag(P^T P)^-1 (Implementation section).
 *
 * Templates ("Using MADmap" section, eqs. eDSN1 and PmatExt): a plan may
 * append template columns B to the pointing matrix, P -> [P B], and the
 * template amplitudes y to the unknowns, m -> [m; y].  Supported B: one-hot
 * columns (a signal synchronous with a binned parameter, or destriping
 * offsets: B[t, idx_t] = 1) and the 32-column half-wave-plate block of
 * eq. HWPmat per segment of samples.  Every operator and solve below then
 * acts on the extended system.
 *
 * Conventions for every entry point:
 *   - Pointers named d_* are device (HBM) pointers on the current HIP device;
 *     all others are host pointers.  The caller owns every buffer it passes.
 *     A plan's device memory is one workspace: the caller's (mm_plan, sized by
 *     mm_plan_workspace_size) or one block mm_plan_create allocates; the plan
 *     allocates no other device memory in any later call.
 *   - `stream` is a hipStream_t (passed as void*); NULL means the default
 *     stream.  Work is enqueued on it.  Plan construction returns once its work
 *     is queued (it waits only for the counts it needs on the host); every later
 *     call on the plan orders its work after that build, whatever its stream.
 *     Entry points that read results on the host (mm_filter_lags, mm_solve,
 *     mm_solve_rhs, mm_noise_gradient) return with their results complete.
 *     Calls on one plan share its work buffers: the caller must not let them
 *     overlap in time (one stream per plan, or its own synchronisation).
 *   - Maps cross the boundary in global pixel layout, float64,
 *     [n_rhs][n_pix][n_stokes] (Stokes fastest).  Pixels never observed are
 *     written as 0.  With templates every map-shaped buffer is the extended
 *     vector: per RHS, the n_pix * n_stokes map values followed by the
 *     n_tmpl template amplitudes (mm_plan_info_t.n_tmpl), templates in
 *     descriptor order; amplitudes no sample touches are written as 0.
 *   - Time-ordered data (TOD) cross the boundary as [n_rhs][n_samples] of
 *     float32 (MM_F32) or float64 (MM_F64).
 *   - Every entry point returns an mm_status_t and never throws; on failure
 *     mm_last_error() gives a message for the calling thread.
 */
#ifndef MM_H
#define MM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct mm_plan_s* mm_plan_t;

typedef enum {
  MM_OK = 0,
  MM_EINVAL = 1,        /* invalid argument or descriptor */
  MM_ENOMEM = 2,        /* device allocation failed */
  MM_EDEVICE = 3,       /* HIP runtime or kernel error */
  MM_ENOTCONV = 4,      /* solve ended at max_iter above tol (best iterate still written) */
  MM_ESINGULAR = 5,     /* a preconditioner block is singular or ill-conditioned */
  MM_EUNSUPPORTED = 6   /* valid request this build does not implement */
} mm_status_t;

/* precision of the CG iterations */
enum { MM_FP64 = 0,     /* gather, filter and scatter in float64 */
       MM_MIXED = 1 };  /* TOD filtering and scatter in float32 with compensated pixel
                           sums; dot products, scalars, preconditioner in float64 */

/* preconditioner */
enum { MM_PRECOND_BLOCK = 0,   /* (P^T W^-1 P)^-1, 1x1 or 3x3 per pixel */
       MM_PRECOND_JACOBI = 1,  /* diag(P^T P)^-1 */
       MM_PRECOND_NONE = 2 };

/* element type of a TOD buffer */
enum { MM_F32 = 0, MM_F64 = 1 };

/* template kinds */
enum { MM_TMPL_ONEHOT = 1,   /* B[t, idx_t] = 1: synchronous bins, destriping offsets */
       MM_TMPL_HWP = 2 };    /* half-wave-plate parametric block, 32 columns per segment */

/*
 * One block of template columns (section "Using MADmap").
 *   MM_TMPL_ONEHOT: n_amp amplitudes; d_idx (device int32 [n_samples]) holds
 *     the amplitude of each sample in [0, n_amp), or -1 for none.
 *   MM_TMPL_HWP: for each segment g of seg_start (host int64 [n_seg + 1],
 *     seg_start[0] = 0, non-decreasing, seg_start[n_seg] = n_samples) the 32
 *     columns of eq. HWPmat, in this order for k = 1..8: cos(k w_t), then
 *     tau_t cos(k w_t), then sin(k w_t), then tau_t sin(k w_t), where w_t is
 *     d_omega[t] (device float32 [n_samples], radians) and
 *     tau_t = (2 (t - s_g) - (L_g - 1)) / L_g is the sample index centred on
 *     the segment [s_g, s_g + L_g) and scaled to (-1, 1) (an affine change of
 *     the paper's time factor: same column span, so the same fitted signal
 *     and map).  Amplitudes: 32 per segment, segment-major.
 * Template rows do not depend on the pointing index: a sample with pixel -1
 * still carries its template columns.  d_idx and d_omega are read by every
 * operator and must stay allocated and unchanged until mm_destroy.
 * Amplitude preconditioner: diag(B^T W^-1 B)^-1 (MM_PRECOND_BLOCK),
 * diag(B^T B)^-1 (MM_PRECOND_JACOBI) or 1, with 0 for an all-zero column.
 */
typedef struct {
  int32_t kind;                 /* MM_TMPL_ONEHOT or MM_TMPL_HWP */
  int32_t n_seg;                /* HWP: number of segments, >= 1 */
  int64_t n_amp;                /* ONEHOT: number of amplitudes, 1 .. 2^31 - 2 */
  const int32_t* d_idx;         /* ONEHOT: device [n_samples] */
  const float* d_omega;         /* HWP: device [n_samples] */
  const int64_t* seg_start;     /* HWP: host [n_seg + 1] */
} mm_template_t;

typedef struct {
  int32_t n_stokes;             /* 1 (T) or 3 (I, Q, U) */
  int64_t n_pix;                /* global pixel count; pointing indices lie in [-1, n_pix) */
  int64_t n_samples;            /* n_t, at most 2^31 - 1 */
  int32_t n_intervals;          /* stationary intervals n_b >= 1 */
  const int64_t* iv_start;      /* host [n_intervals + 1]: iv_start[0] = 0, non-decreasing,
                                   iv_start[n_intervals] = n_samples */
  const int32_t* iv_filter;     /* host [n_intervals]: noise filter of each interval */
  int32_t n_filters;            /* >= 1 */
  const double* filter_params;  /* host [n_filters][3] = (sigma, f_knee, alpha) of
                                   p(f) = sigma^2 (1 + (f_knee/f)^alpha); may be NULL
                                   when filter_lags is given */
  const double* filter_lags;    /* host [n_filters][n_c] explicit f(tau), or NULL */
  double f_samp;                /* sampling frequency in Hz (used with filter_params) */
  int32_t n_c;                  /* correlation length: f(tau) = 0 for tau >= n_c; >= 1 */
  int32_t n_f;                  /* overlap-save FFT length: 0 = library default (the
                                   paper's rule capped at 2^14, or the smallest power of
                                   two above 2 n_c when that is longer; in float32 with the
                                   default shape, twice that, 2^16, where the chunks of the
                                   2^15-point transform take fewer full rounds of one
                                   workgroup per compute unit at 2.25 times the work each),
                                   -1 = autotune
                                   (time every length with a transform on the plan's
                                   intervals and keep the fastest), > 0 = forced power of
                                   two with n_f > 2 n_c.  Transforms exist on chip (one
                                   workgroup) up to 2^16 in float32 and 2^15 in float64,
                                   and as a batched four-step transform through device
                                   memory at 2^17 and 2^18 (the paper's length for
                                   n_c = 8192) in both precisions */
  int32_t lag_dft_len;          /* L_K, frequencies on which 1/p is sampled to build f
                                   from filter_params; 0 = 2^20; power of two >= 4 n_c */
  int32_t precision;            /* MM_FP64 or MM_MIXED */
  int32_t precond;              /* MM_PRECOND_* */
  int32_t n_rhs;                /* right-hand sides solved together, 1 .. 64 */
  int32_t n_templates;          /* template blocks appended to P, 0 .. 16 */
  const mm_template_t* templates;  /* host [n_templates], or NULL when n_templates = 0 */
  int32_t fft_shape;            /* workgroup shape of the overlap-save transform (n_f / 2 complex
                                   points): 0 = library default (for 2^14 and 2^15 points shape
                                   10 in float32, for 2^14 shape 3 in float64; else 1);
                                   1 = 16 points per thread,
                                   radix-16 passes (32 points per
                                   thread for 2^15 points); 2 = radix-32 passes, 32 points per
                                   thread (64 for 2^15); 3 = 512 threads x 32 points, radix-16
                                   passes, conjugate pairs of the real-to-complex step in
                                   registers; 4 = shape 3 with the LDS exchanges split into real
                                   and imaginary halves so two workgroups share a CU; 5 = 256
                                   threads x 64 points, radix-32, split exchanges, two
                                   workgroups per CU; 6 = 1024 threads x 16 points, radix-8
                                   passes, pairs in registers; 7 = shape 6 with split exchanges,
                                   two workgroups per CU; 8 = 512 threads x 32 points, radix-8
                                   passes, pairs in registers; 9 = shape 6 with each exchange
                                   made in two halves of the index space through half the LDS,
                                   two workgroups per CU; 10 = 1024 threads x 16 points, a
                                   four-step transform (16 x 1024) whose 1024-point stages
                                   stay inside one wavefront (exchanges without workgroup
                                   barriers), float32 only; for 2^15 points 1024 threads x 32
                                   points (32 x 1024, two 1024-point rows per wavefront,
                                   workgroup exchanges in two halves).  For 2^15 points shape
                                   3 is 1024 threads x 32 points, radix-8 passes, pairs in
                                   registers.  Shape 2 exists for float32 transforms of
                                   2^13 .. 2^15 points, shapes 3 and 10 for 2^14 and 2^15
                                   points, shapes 4 .. 9 for 2^14 points (3, 6 and 8 also in
                                   float64); elsewhere shape 1 is used.  Ignored with n_f = -1 (the autotuner tries every
                                   shape). */
} mm_desc_t;

typedef struct {
  int64_t n_obs;                /* observed pixels (the unknowns are n_obs * n_stokes per RHS) */
  int64_t n_valid;              /* samples with a pixel (pointing index >= 0) */
  int32_t n_f;                  /* FFT length the iterations use */
  int32_t n_chunks;             /* overlap-save transforms per TOD pass and RHS */
  int32_t n_singular;           /* preconditioner blocks flagged singular */
  int64_t device_bytes;         /* bytes of the workspace in use (at most the bound) */
  int64_t n_sliced;             /* entries of the scatter's pixel-major pointing: n_valid when
                                   it is read as is (128 or more hits per observed pixel on
                                   average and at most 256 MiB of TOD per scatter pass), else
                                   the sliced copy's (a multiple of 64, >= n_valid; the excess
                                   is padding to the widest pixel of each slice) */
  int64_t n_tmpl;               /* template amplitudes per RHS in map-shaped buffers (0 = none) */
  int32_t fft_shape;            /* transform shape the iterations use (1 .. 10, see mm_desc_t) */
} mm_plan_info_t;

/*
 * Device bytes a plan of this descriptor needs in its workspace (an upper bound
 * computed from the descriptor alone: it holds for any pointing the descriptor
 * admits).  The plan holds the time-major observed index and the pixel-major
 * (or sliced) pointing of the pixel-indexing scheme (Implementation section),
 * the lags and overlap-save spectra of N^-1 (Weighting section), the block
 * preconditioner (Implementation section), and the TOD and CG work vectors of
 * the PCG iteration (Algorithm section, eq. pcgSystem).  Host-only.
 * Errors: MM_EINVAL (descriptor), MM_EUNSUPPORTED (forced n_f with no transform).
 */
mm_status_t mm_plan_workspace_size(const mm_desc_t* desc, size_t* bytes);

/*
 * Build a plan in the caller's workspace: validate the descriptor, range-check
 * the pointing, compact the observed pixels (Implementation section, observed
 * index scheme), sort samples by pixel for the pixel-major scatter, build the
 * noise filters (lags f(tau) and overlap-save spectra, Weighting section) and
 * the preconditioner (Implementation section).
 *   d_pix:  device int32 [n_samples], pixel of each sample, -1 = no pixel
 *           (excised sample; its row of P is zero).  Read during the build.
 *   d_w:    device float32 [n_samples][2] = (sin 2a_t, cos 2a_t); required
 *           when n_stokes == 3, ignored (may be NULL) when n_stokes == 1.
 *           d_w must stay allocated and unchanged until mm_destroy.
 *   d_ws:   device workspace of ws_bytes >= mm_plan_workspace_size(desc),
 *           256-byte aligned, owned by the caller; the plan uses it until
 *           mm_destroy and never frees it.  Its contents on entry do not matter.
 * With n_c = 1 (white noise) N^-1 is applied as the diagonal f_b(0) without
 * transforms (the destriping case of the "Using MADmap" section).
 * Errors: MM_EINVAL (descriptor, pixel or template index out of range, NULL or
 * misaligned workspace, ws_bytes below the bound), MM_EDEVICE, MM_EUNSUPPORTED
 * (forced n_f with no transform).  A singular preconditioner
 * block does not fail the plan; it is counted in mm_plan_info_t.n_singular and
 * makes mm_solve return MM_ESINGULAR.
 */
mm_status_t mm_plan(const mm_desc_t* desc, const int32_t* d_pix, const float* d_w, void* d_ws,
                    size_t ws_bytes, void* stream, mm_plan_t* out_plan);

/* mm_plan in a workspace the library allocates (hipMalloc of the bound) and
 * mm_destroy frees.  Errors as mm_plan, and MM_ENOMEM. */
mm_status_t mm_plan_create(const mm_desc_t* desc, const int32_t* d_pix, const float* d_w,
                           void* stream, mm_plan_t* out_plan);

/* Destroy a plan: waits for the device to be idle, so that the caller may free or
 * reuse its workspace at once.  NULL is a no-op.  mm_plan_destroy is the same call. */
mm_status_t mm_destroy(mm_plan_t plan);
mm_status_t mm_plan_destroy(mm_plan_t plan);

/* Sizes the plan found: observed pixels and pointed samples (pixel-indexing
 * scheme, Implementation section), FFT length and transforms per TOD pass of the
 * overlap-save N^-1 (Weighting section, eq. FFTcomplexityFunction), singular
 * preconditioner blocks (Implementation section), workspace bytes in use.  Waits
 * for the preconditioner's singular-block count when first called. */
mm_status_t mm_plan_get_info(mm_plan_t plan, mm_plan_info_t* info);

/* Hit count of every global pixel, the number of samples pointing at it (the
 * pixel-indexing scheme of the Implementation section; for temperature the
 * diagonal of P^T P): device int32 [n_pix], exact integers, unobserved pixels 0. */
mm_status_t mm_hits(mm_plan_t plan, int32_t* d_hits, void* stream);

/* The lags f(tau), tau = 0 .. n_c - 1, of each filter's banded Toeplitz block of
 * N^-1 (Weighting section; built from p(f) of the Algorithm section when the plan
 * has filter_params): host float64 [n_filters][n_c].  Copies on `stream` after
 * the plan's build and synchronises that stream. */
mm_status_t mm_filter_lags(mm_plan_t plan, double* lags_out, void* stream);

/* y = P x: device map [n_rhs][n_pix][n_stokes] float64 -> TOD [n_rhs][n_samples]
 * of tod_dtype (unpointing, Formalism section). */
mm_status_t mm_unpoint(mm_plan_t plan, const double* d_x, void* d_y, int32_t tod_dtype,
                       void* stream);

/* x = P^T y: TOD [n_rhs][n_samples] of tod_dtype -> map (pointing / scatter-add). */
mm_status_t mm_point(mm_plan_t plan, const void* d_y, int32_t tod_dtype, double* d_x,
                     void* stream);

/* y_out = N^-1 y_in per interval (Weighting section), in the plan's precision
 * (float64 for MM_FP64, float32 arithmetic for MM_MIXED).  TOD buffers
 * [n_rhs][n_samples] of tod_dtype; y_out must not overlap y_in. */
mm_status_t mm_weight(mm_plan_t plan, const void* d_y_in, void* d_y_out, int32_t tod_dtype,
                      void* stream);

/* y = H x = P^T N^-1 P x for maps [n_rhs][n_pix][n_stokes] (one CG operator application). */
mm_status_t mm_apply_A(mm_plan_t plan, const double* d_x, double* d_y, void* stream);

/* b = P^T N^-1 d (right-hand side, one pass over the TOD). */
mm_status_t mm_rhs(mm_plan_t plan, const void* d_tod, int32_t tod_dtype, double* d_b,
                   void* stream);

typedef struct {
  double tol;                   /* stop when ||r||_2 / ||b||_2 <= tol (paper default 1e-6) */
  int32_t max_iter;             /* at most this many H applications (paper default 50) */
  int32_t fixed_iters;          /* > 0: run exactly this many iterations, ignore tol */
  int32_t check_every;          /* iterations between host convergence checks (1 .. 256; larger
                                   values are taken as 256); a block
                                   is shortened when every active RHS is predicted (from its
                                   residual rate since the last check) to reach tol sooner */
  int32_t use_graph;            /* replay each full block of check_every iterations as a hipGraph,
                                   captured once per plan from its second solve on (a plan's first
                                   solve launches directly: capture costs more than it saves then);
                                   a reliable-update solve keeps a second graph for its iterations
                                   with the float32 increment of x (see refine) */
  int32_t true_residual;        /* recompute ||b - H x_best|| / ||b|| in float64 at exit */
  const double* d_x0;           /* optional initial map [n_rhs][n_pix][n_stokes]; NULL = 0 */
  int32_t refine;               /* MM_MIXED only: 1 = reliable updates: H is applied in float32,
                                   the iterate, r, b and the dots are float64 (without templates
                                   q, z and p are float32, and once every RHS's float64 residual
                                   is below 1e-5 x moves by a float32 increment folded into the
                                   float64 iterate at each replacement); at the host's
                                   check points each RHS whose recurrence residual fell a
                                   thousandfold since its last replacement (or reached tol) gets
                                   its residual replaced by the float64 true residual b - H x
                                   (float64 filter) and CG continues along the same direction;
                                   blocks between checks are at most min(check_every, 8)
                                   iterations until the convergence rate is known, then up to
                                   2 check_every while the residual is predicted to stay within
                                   4.5 decades of the last float64 one; tol is tested on
                                   those true residuals and the iterate with the lowest one is
                                   returned, so the map reaches float64 accuracy.  0 = plain
                                   mixed iterations.  Ignored with fixed_iters. */
  int32_t map_error;            /* 1 = estimate each returned map's distance to the exact
                                   float64 solution (mm_solve_info_t.map_error): the residual
                                   b - H x is formed in float64 and H e = b - H x is solved by
                                   PCG with the plan's operator to 1e-2 of its right-hand
                                   side (at most 50 iterations); costs those iterations */
} mm_solve_opts_t;

typedef struct {
  int32_t* iters;               /* [n_rhs] H applications performed per RHS */
  int32_t* best_iter;           /* [n_rhs] iteration of the returned iterate (0 = x0) */
  double* best_rel_res;         /* [n_rhs] its relative residual (recurrence; true with refine) */
  double* true_rel_res;         /* [n_rhs] float64 ||b - H x||/||b|| of the returned map, or NaN
                                   (always set with refine; with true_residual otherwise) */
  double* history;              /* [n_rhs][n + 1], n = fixed_iters if > 0 else max_iter:
                                   relative residual per iteration (entry 0 = start, NaN after
                                   the last iteration); with refine, the recurrence residual
                                   between replacements and the float64 true residual at each
                                   replacement; may be NULL */
  double* map_error;            /* [n_rhs] with opts.map_error: ||x - x*|| / ||x|| for the returned
                                   map x and the exact float64 solution x* of H x* = b (map
                                   error against float64, estimated to about two digits); NaN
                                   otherwise; may be NULL */
} mm_solve_info_t;

/* Fill opts with the paper's defaults (tol 1e-6, max_iter 50) and check_every 8, graph on,
 * refine on. */
void mm_solve_opts_default(mm_solve_opts_t* opts);

/*
 * Solve H m = b for every RHS with PCG; writes to d_x the iterate with the
 * lowest relative residual seen (Implementation section).  best_rel_res
 * (and the tol test) use the recurrence residual, or with refine the float64
 * residual of the accumulated map.  Each RHS stops at
 * its own tol.  Returns MM_ENOTCONV (with the best iterate written) if any RHS
 * ends at max_iter above tol, MM_ESINGULAR if the plan flagged a singular
 * preconditioner block.  info may be NULL; its arrays are optional.
 */
mm_status_t mm_solve(mm_plan_t plan, const void* d_tod, int32_t tod_dtype, double* d_x,
                     const mm_solve_opts_t* opts, mm_solve_info_t* info, void* stream);

/*
 * Same solve with the right-hand side given as a map: H m = b for
 * d_b [n_rhs][n_pix][n_stokes] float64 (unobserved pixels ignored).  H is
 * symmetric (Algorithm section), so this is also the adjoint solve of a map
 * loss: lambda = H^-1 dL/dm.
 */
mm_status_t mm_solve_rhs(mm_plan_t plan, const double* d_b, double* d_x,
                         const mm_solve_opts_t* opts, mm_solve_info_t* info, void* stream);

/*
 * Gradient of a map loss with respect to the noise parameters theta = (sigma,
 * f_knee, alpha) of p(f) (Algorithm section).  The map m = H^-1 P^T N^-1 d
 * (eq. eMLM) depends on theta only through N^-1; with lambda = H^-1 dL/dm (the
 * adjoint solve: H is symmetric, Algorithm section, so mm_solve_rhs gives it),
 *     dL/dtheta = sum over RHS r of (P lambda_r)^T (dN^-1/dtheta) (d_r - P m_r),
 * where dN^-1/dtheta is the banded Toeplitz operator (Weighting section) whose
 * lags are the theta-derivative of f(tau) (the plan's lag construction
 * differentiated under the inverse DFT), restricted to the intervals of each
 * filter.  The parameters are shared by the RHS, so their terms are summed.
 *   d_tod:    TOD d [n_rhs][n_samples] of tod_dtype (the solve's data).
 *   d_m:      the map m [n_rhs][n_pix][n_stokes] float64 (map-shaped; with
 *             templates the extended vector).
 *   d_lambda: the adjoint lambda, same layout as d_m.
 *   grad_out: host float64 [n_filters][3] = dL/d(sigma, f_knee, alpha).
 * P m, P lambda, d - P m and the filtered products are formed on the device in
 * float64 whatever the plan's precision; synchronises.  Returns MM_EUNSUPPORTED
 * for plans built from explicit lags.
 */
mm_status_t mm_noise_gradient(mm_plan_t plan, const void* d_tod, int32_t tod_dtype, const double* d_m,
                              const double* d_lambda, double* grad_out, void* stream);

/*
 * The lags of the inverse-noise filter from the noise parameters, without a plan:
 * f(tau), tau = 0 .. n_c - 1, of the banded Toeplitz N^-1 (Weighting section) for
 * p(f) = sigma^2 (1 + (f_knee/f)^alpha) (Algorithm section): the inverse DFT of
 * 1/p(nu_j) on lag_dft_len frequencies nu_j = j f_samp / lag_dft_len (1/p at nu = 0
 * being its limit), tapered by (1 - tau/n_c); with deriv = 1, 2, 3 the same
 * construction applied to the derivative of 1/p with respect to sigma, f_knee,
 * alpha.  The plan builds its lags the same way (filter_params).
 *   d_params: device float64 [n_filters][3] = (sigma, f_knee, alpha), sigma > 0,
 *             f_knee >= 0, alpha > 0 (other values give non-finite lags).
 *   d_lags:   device float64 [n_filters][n_c], written.
 *   d_ws:     device scratch of ws_bytes >= mm_noise_lags_workspace_size(n_c,
 *             lag_dft_len), 256-byte aligned, the caller's; a larger one lets more
 *             filters share a launch.  Its contents on entry do not matter.
 * n_c <= 2^14; lag_dft_len a power of two in [4 n_c, 2^30].  Asynchronous on
 * `stream`.  Errors: MM_EINVAL (arguments, workspace), MM_EUNSUPPORTED (n_c),
 * MM_EDEVICE.
 */
mm_status_t mm_noise_lags_workspace_size(int32_t n_c, int64_t lag_dft_len, size_t* bytes);
mm_status_t mm_noise_lags(const double* d_params, int32_t n_filters, double f_samp, int32_t n_c,
                          int64_t lag_dft_len, int32_t deriv, double* d_lags, void* d_ws, size_t ws_bytes,
                          void* stream);

/*
 * mm_noise_lags for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * lags, with no workspace argument and no allocation.  Its scratch is a static
 * device array of 64 MiB that each device the library runs on holds until the
 * process ends; arguments whose scratch need (mm_noise_lags_workspace_size)
 * exceeds 64 MiB are rejected with MM_EINVAL (for n_c = 8192 the 2^20-point
 * construction needs 16 MiB per filter).  Every call on a device uses that
 * device's one array: calls that overlap in time on one device race, so the
 * caller serialises them (one stream, or its own synchronisation).  Nothing in
 * the array needs to start at zero.  Arguments and errors as mm_noise_lags.
 */
mm_status_t mm_noise_lags_noalloc(const double* d_params, int32_t n_filters, double f_samp, int32_t n_c,
                                  int64_t lag_dft_len, int32_t deriv, double* d_lags, void* stream);

/* FFT length by the paper's halving rule (Weighting section, eq. FFTcomplexityFunction):
 * start at the smallest power of two >= longest, halve while h'(n_f/2) >= 0 and
 * n_f/2 > 2 n_c.  Returns 0 for invalid arguments. */
int32_t mm_fft_length_rule(int32_t n_c, int64_t longest);

/* Message describing the last failure on the calling thread ("" if none). */
const char* mm_last_error(void);

/* Library version string. */
const char* mm_version(void);

#ifdef __cplusplus
}
#endif
#endif /* MM_H */
