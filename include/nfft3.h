/*
 * nfft3.h -- C ABI of the MI355X (gfx950) three-dimensional nonequispaced FFT.
 *
 * The library evaluates the truncated Fourier series of Sec. 2.2.1 of
 * Caliari & Zuccher, "INFFTM: Fast evaluation of 3d Fourier series in MATLAB
 * with an application to quantum vortex reconnections" (arXiv:1605.01244),
 * in the NFFT form the paper hands to the NFFT library:
 *
 *     f_j = sum_{k in I_N} fhat_k exp(-2 pi i k . x_j),   j = 0 .. M-1,
 *     I_N = prod_d {-N_d/2, ..., N_d/2 - 1},  N_d even  (Sec. 2, set I_N),
 *
 * at points x_j in [-1/2, 1/2)^3 (any finite x is folded periodically).
 * The result is the windowed approximation of the NFFT literature the paper
 * cites (Kaiser-Bessel window of half-width m cells on the grid n_d = sigma N_d):
 * (a) deconvolution by the window transform and zero-padding, (b) a 3-D FFT
 * of size n, (c) a window sum over the (2m)^3 nearest grid points.  The error
 * falls like exp(-2 pi m sqrt(1 - 1/sigma)) (the M |log eps|^3 term of the
 * cost quoted in Sec. 1).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Pointers named *_dev are DEVICE pointers (HBM of the GPU the plan lives
 *    on); pointers without the suffix are host pointers.
 *  - Complex data are interleaved (re, im) pairs of float (NFFT3_C64) or
 *    double (NFFT3_C128), i.e. the layout of torch.complex64 / complex128.
 *  - Coefficients are a C-order (N0, N1, N2) array, the last axis contiguous;
 *    array index i_d corresponds to frequency k_d = i_d - N_d/2.  (The paper
 *    stores the same array column-major in MATLAB with index k_d - 1 - N_d/2;
 *    here axis d of the array is paired with column d of the points.)
 *  - Points are an (M, 3) row-major FP64 array in both precisions.
 *  - The plan owns every buffer it allocates (grid, tables, sorted points,
 *    bins); the caller owns the arrays it passes and must keep them alive
 *    until the work enqueued on the plan's stream has finished.
 *  - All work is enqueued on the plan's HIP stream.  nfft3_trafo,
 *    nfft3_adjoint, nfft3_grad_points and the stage calls never synchronise
 *    the host; nfft3_set_points synchronises once (to report non-finite
 *    points and to size the launches).
 *  - Every call returns an int status (NFFT3_OK = 0 or a negative code);
 *    nothing is thrown across the ABI and nothing calls exit().  After
 *    NFFT3_ERR_HIP, nfft3_last_hip_error() describes the runtime failure.
 *  - A plan is bound to one stream and is not thread-safe.
 */
#ifndef NFFT3_H
#define NFFT3_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct nfft3_plan_s *nfft3_plan_t;

/* Precision of coefficients, grid, FFT and window sums.  Point coordinates,
 * their fold into [-1/2, 1/2) and the split into grid cell + fraction are
 * always FP64. */
enum nfft3_dtype { NFFT3_C64 = 0, NFFT3_C128 = 1 };

enum nfft3_status {
    NFFT3_OK = 0,
    NFFT3_ERR_INVALID_ARG = -1, /* bad size, sigma, m or count (see nfft3_plan) */
    NFFT3_ERR_DTYPE = -2,       /* dtype not NFFT3_C64 / NFFT3_C128, or plans mixed */
    NFFT3_ERR_OOM = -3,         /* device allocation failed                      */
    NFFT3_ERR_NO_POINTS = -4,   /* trafo/adjoint/grad before nfft3_set_points    */
    NFFT3_ERR_NONFINITE = -5,   /* a point coordinate is NaN or infinite         */
    NFFT3_ERR_HIP = -6,         /* HIP runtime error (see nfft3_last_hip_error)  */
    NFFT3_ERR_NULL = -7,        /* NULL plan or NULL required pointer            */
    NFFT3_ERR_CAPACITY = -8,    /* batch too large for nfft3_batch_trafo_noalloc */
    NFFT3_ERR_TIMEOUT = -9      /* a nfft3_batch_trafo_queue wait hit its limit  */
};

/* Create a plan for coefficient sizes N[0..2] (host array).
 *   N_d    even, 2 <= N_d (the set I_N of Sec. 2 needs N_d even); or
 *          N_0 = 1, or N_0 = N_1 = 1: leading unit axes, whose only frequency
 *          is 0, so the sum over them is exact (no oversampling, no window:
 *          n_d = 1).  Such a plan is the two- or one-dimensional transform
 *          with points still (M, 3) (unit coordinates are ignored); see
 *          nfft3_plan_nd for the same with (M, d) points.
 *   sigma  oversampling factor > 1; n_d = sigma * N_d must be an even integer
 *          whose prime factors are 2, 3, 5 and 7, with n_d <= 2048.
 *   m      window half-width in oversampled cells, 1 <= m <= 10, 2m <= n_d.
 *          Typical: m = 4 (about 1e-7 relative error at sigma = 2),
 *          m = 6 (1e-11), m = 8 (1e-14).
 *   dtype  NFFT3_C64 or NFFT3_C128.
 *   stream hipStream_t to enqueue on (NULL = the default stream).
 * Arguments are validated on the host before any HIP call; invalid ones give
 * NFFT3_ERR_INVALID_ARG / NFFT3_ERR_DTYPE / NFFT3_ERR_NULL and *out = NULL.
 * Allocates the n0 n1 n2 complex grid and the window tables on the current
 * device. */
int nfft3_plan(nfft3_plan_t *out, const int64_t N[3], double sigma, int m, int dtype,
               void *stream);

/* Plan of d = 1, 2 or 3 axes (the one- and two-dimensional series the paper
 * evaluates with infft and infft2, Appendix B): N[0..d-1] (host array), each
 * even and >= 2, is the coefficient array's shape; the plan is the 3-D plan
 * of nfft3_plan with 3 - d leading unit axes, so the other arguments,
 * limits and errors are those of nfft3_plan.  On such a plan
 *   - points are (M, d) FP64 arrays (nfft3_set_points,
 *     nfft3_points_unchanged; widened on the device into a plan buffer),
 *   - nfft3_grad_points writes (M, d) components,
 *   - bit i of a derivative mask (nfft3_trafo_fields) is the plan's axis i,
 *   - nfft3_infft3 takes a[d], b[d] and (M, d) points,
 *   - nfft3_tube_refine and nfft3_batch_trafo return NFFT3_ERR_INVALID_ARG
 *     (three-dimensional plans only). */
int nfft3_plan_nd(nfft3_plan_t *out, int d, const int64_t *N, double sigma, int m, int dtype,
                  void *stream);

/* Rebind the plan to another stream of the same device. */
int nfft3_set_stream(nfft3_plan_t p, void *stream);

/* Set the M points, x_dev = (M, 3) FP64 device array.  Folds them into
 * [-1/2, 1/2) (Euclidean remainder, as the mod of Sec. 2.2.1), splits
 * n_d x into cell and fraction in FP64, bins and sorts them on the device
 * (counting sort by grid tile) and keeps the sorted copy; x_dev is not
 * referenced afterwards.  M = 0 is allowed (trafo then writes nothing).
 * Returns NFFT3_ERR_NONFINITE (and leaves the plan without points) if any
 * coordinate is NaN or infinite. */
int nfft3_set_points(nfft3_plan_t p, int64_t M, const double *x_dev);

/* Are the plan's sorted points still those of x_dev ((M, 3) FP64 device
 * array)?  *unchanged (host int) = 1 when the plan holds M points and, for
 * every point, the folded coordinates kept by the last nfft3_set_points equal
 * the fold of x_dev's current coordinates bit for bit (so a new
 * nfft3_set_points would produce the same sorted state); 0 otherwise (also
 * when the plan has no points or another M).  A caller that re-evaluates at
 * possibly unchanged points (an autograd forward) uses it to skip the sort,
 * the precomputation of Sec. 2.2.1's method.  One pass over the points;
 * synchronises the plan's stream. */
int nfft3_points_unchanged(nfft3_plan_t p, int64_t M, const double *x_dev, int *unchanged);

/* Type-2 transform (the evaluation of Sec. 2.2.1):
 * f_dev[j] ~ sum_k fhat_k exp(-2 pi i k.x_j), j in the caller's point order.
 * fhat_dev: N0*N1*N2 complex, f_dev: M complex (dtype of the plan).
 * Uses the plan's grid as workspace. */
int nfft3_trafo(nfft3_plan_t p, const void *fhat_dev, void *f_dev);

/* Adjoint (type-1) transform, the conjugate transpose of nfft3_trafo's
 * discrete operator: fhat_dev[k] = sum_j f_j exp(+2 pi i k.x_j) (windowed).
 * The paper only evaluates series; this is the map a gradient with respect
 * to the coefficients needs. */
int nfft3_adjoint(nfft3_plan_t p, const void *f_dev, void *fhat_dev);

/* Gradient with respect to the points for a real loss L(f):
 *   grad_x_dev[j, d] = Re( conj(G_j) * d f_j / d x_{j,d} ),
 *   d f_j / d x_{j,d} = sum_k (-2 pi i k_d) fhat_k exp(-2 pi i k.x_j)
 * (the derivative multipliers of eq. (Lambda) on the unit period), computed
 * through the window derivative.  G_dev holds dL/dRe f + i dL/dIm f (M
 * complex, plan dtype); grad_x_dev is (M, 3) FP64.  Recomputes the grid from
 * fhat_dev. */
int nfft3_grad_points(nfft3_plan_t p, const void *fhat_dev, const void *G_dev, double *grad_x_dev);

/* Evaluate the coefficient field and, for each bit d set in deriv_mask
 * (bit 0,1,2 = axis 0,1,2), the derivative field sum_k (-2 pi i k_d) fhat_k
 * exp(-2 pi i k.x) at the plan's points.  out_dev holds (1 + popcount(mask))
 * consecutive blocks of M complex values: the field first, then the
 * derivative fields in axis order.  NFFT3_C128: one grid; the window sums
 * form the derivative fields through the window derivative (its error stays
 * within the FP64 accuracy of the transform).  NFFT3_C64: one grid and
 * transform per field (the spectral multiplier), since the derivative of
 * the windowed sum amplifies FP32 rounding about n_d-fold. */
int nfft3_trafo_fields(nfft3_plan_t p, const void *fhat_dev, void *out_dev, int deriv_mask);

/* Batched type-2 evaluation of T independent plans (own N, own points, same
 * dtype, sigma and m, with m <= 8): the time snapshots and derivative fields
 * of a vortex-tracking workload evaluated together.  For plan t, fhat_dev[t]
 * holds its coefficients and out_dev[t] receives (1 + popcount(deriv_mask))
 * blocks of M_t values as in nfft3_trafo_fields.  fhat_dev / out_dev are host
 * arrays of T device pointers; plans is a host array of T distinct plans.
 * Each FFT stage (row pass, column pass axis 1, column pass axis 0) runs as
 * one kernel launch per distinct transform length along its axis, the window
 * sums as one launch; each launch covers the work items of every (plan,
 * field) pair in its group, and the results equal the sequential
 * nfft3_trafo_fields results bit for bit.  NFFT3_C64 plans keep one grid per
 * evaluated field, allocated on their first batched call with a given mask;
 * NFFT3_C128 plans use their one grid (derivative fields from the window
 * derivative, as nfft3_trafo_fields).
 * Work is enqueued on plans[0]'s stream; the call returns after it finished
 * (the launch descriptors are staged from host memory). */
int nfft3_batch_trafo(int T, const nfft3_plan_t *plans, const void *const *fhat_dev,
                      void *const *out_dev, int deriv_mask);

/* nfft3_batch_trafo as ONE launch: persistent workgroups take tickets over
 * (transform, stage, tile) from a device counter, the tickets laid out
 * stage-major, and a task waits (spinning on a device counter) only for the
 * previous stage of its own transform; the stages' bodies are those of
 * nfft3_batch_trafo (the column passes in 256-thread tiles of fewer columns,
 * each line's arithmetic unchanged), so the results equal it bit for bit.
 * Same arguments; additionally every plan's three oversampled lengths must
 * be ones the library's compile-time FFT engine covers (64, 80, 96, 128,
 * 160, 192, 256, 320, 384, 512), else NFFT3_ERR_INVALID_ARG before any work.
 * Each wait is bounded by NFFT3_QUEUE_WAIT_US microseconds of wall clock
 * (environment, read per call; default 2000000, at most 3.6e9): a wait past it abandons the
 * batch (the outputs are then incomplete) and returns NFFT3_ERR_TIMEOUT.
 * Allocates its descriptor buffer as nfft3_batch_trafo does (shared with it,
 * under the same per-GPU lock); synchronises before it returns. */
int nfft3_batch_trafo_queue(int T, const nfft3_plan_t *plans, const void *const *fhat_dev,
                            void *const *out_dev, int deriv_mask);

/* nfft3_batch_trafo without device allocation, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc).  Same arguments, kernels and results
 * (bit for bit) as nfft3_batch_trafo; it calls no hipMalloc, hipFree or
 * allocating library routine.  The launch descriptors go to a static device
 * array of NFFT3_BATCH_SCRATCH_BYTES per GPU (held until the process ends)
 * instead of a library-allocated buffer: about 560 bytes per (plan, field)
 * transform, so roughly 450 transforms per call; a larger batch returns
 * NFFT3_ERR_CAPACITY before any work is enqueued.  Every plan must already
 * hold the grids its fields need: NFFT3_C128 plans and deriv_mask = 0 use
 * the plan's own grid; NFFT3_C64 plans with derivative fields one grid per
 * evaluated field (made by an earlier nfft3_batch_trafo call with at least
 * these fields); else NFFT3_ERR_INVALID_ARG.  All calls on one GPU
 * share the array, which keeps the last call's descriptors; calls (of either
 * batch entry point) on one GPU are serialised by a lock in the library,
 * each holding it until its work has finished (the call synchronises before
 * it returns), so host threads overlapping their calls do not race on it. */
#define NFFT3_BATCH_SCRATCH_BYTES (256 * 1024)
int nfft3_batch_trafo_noalloc(int T, const nfft3_plan_t *plans, const void *const *fhat_dev,
                              void *const *out_dev, int deriv_mask);

/* ---- The series on a physical domain (Sec. 2.2.1) and vortex tubes (Sec. 4.3)
 * The paper's own form of the series, eq. (fs), on Omega = prod [a_d, b_d):
 *
 *     psi(xi) = sum_k psihat_k prod_d exp(+2 pi i k_d (xi_d - a_d)/(b_d - a_d)) / sqrt(b_d - a_d),
 *
 * k_d = i_d - N_d/2 for array index i_d (the paper's k_d - 1 - N_d/2 with
 * 1-based k_d), psihat C-order (N0, N1, N2) with axis d paired with point
 * column d.  As Sec. 2.2.1 does, it is evaluated as the NFFT problem at
 * zeta_d = mod((xi_d - a_d)/(a_d - b_d), 1) - 1/2 with coefficients
 * psihat_k (-1)^(k_0 + k_1 + k_2) / prod sqrt(b_d - a_d); both maps run on
 * the device. */

/* psi_dev[j] = psi(xi_j) for the M points xi_dev ((M, 3) FP64, physical
 * coordinates; any finite values, the series being periodic on Omega) and
 * coefficients psihat_dev (plan dtype); a_d < b_d (host arrays).  On a plan
 * of d < 3 axes (nfft3_plan_nd) a and b hold d entries and xi_dev is (M, d):
 * the one- and two-dimensional series of the paper's infft / infft2
 * (Appendix B).  Sets the
 * plan's points to the mapped xi (as nfft3_set_points, including its
 * synchronisation and NFFT3_ERR_NONFINITE) and leaves them set; the mapped
 * points and coefficients live in plan-owned scratch (allocated on first
 * use, grown as needed). */
int nfft3_infft3(nfft3_plan_t p, const double a[3], const double b[3], const void *psihat_dev, int64_t M,
                 const double *xi_dev, void *psi_dev);

/* Evaluation within vortex tubes (Sec. 4.3): start from the regular grid
 * X_N of Omega (x_{d,n} = a_d + n h_d, h_d = (b_d - a_d)/N_d, n_d = 0 ..
 * N_d - 1, in C order) and rho = |psi|^2 there; for l = 0 .. levels-1 keep
 * the current points with rho <= rhobar[l] (host array) and replace each by
 * the 27 points of the regular grid of step h_d / 3^(l+1) centred on it
 * (neighbour (o0, o1, o2) in {-1, 0, 1}^3 at index 9(o0+1) + 3(o1+1) + o2+1,
 * kept points in their order), evaluating rho there with nfft3_infft3.
 * On return *count holds the number of points of the last set; they and
 * their rho are copied to pts_dev ((cap, 3) FP64) and rho_dev (cap FP64)
 * when count <= cap, else NFFT3_ERR_CAPACITY (nothing copied).  The plan's
 * points are those of the last set afterwards.  Synchronises once per
 * level (to size the next). */
int nfft3_tube_refine(nfft3_plan_t p, const double a[3], const double b[3], const void *psihat_dev, int levels,
                      const double *rhobar, int64_t cap, double *pts_dev, double *rho_dev, int64_t *count);

/* ---- Gross-Pitaevskii time splitting (Sec. 3.1) ----------------------------
 * d psi/dt = (i/2) Lap psi + (i/2)(1 - |psi|^2) psi on the regular grid X_N
 * of the periodic domain prod [a_d, b_d) (x_{d,n} = a_d + n h_d), by Strang
 * splitting: half a step of the potential part (exact: it keeps |psi|), a
 * full step of the kinetic part (exact in Fourier space: mode k times
 * exp(-i tau |kappa_k|^2 / 2), kappa_{k,d} = 2 pi k_d / (b_d - a_d)), half a
 * step of the potential part; consecutive half steps are merged.  The
 * Fourier transforms are the library's Stockham passes, in place. */
typedef struct nfft3_gpe_s *nfft3_gpe_t;

/* N_d even, 16 <= N_d <= 2048, prime factors 2, 3, 5, 7 (e.g. the paper's
 * 80); a_d < b_d (host arrays).  Allocates the state and one scratch of
 * N0 N1 N2 complex values. */
int nfft3_gpe_create(nfft3_gpe_t *out, const int64_t N[3], const double a[3], const double b[3], int dtype,
                     void *stream);
int nfft3_gpe_set_stream(nfft3_gpe_t g, void *stream);
/* Copy the state from / to psi_dev (N0 N1 N2 complex, C order of (n0, n1, n2)). */
int nfft3_gpe_set_state(nfft3_gpe_t g, const void *psi_dev);
int nfft3_gpe_get_state(nfft3_gpe_t g, void *psi_dev);
/* nsteps Strang steps of size tau (any sign: the scheme is time
 * reversible).  Does not synchronise. */
int nfft3_gpe_step(nfft3_gpe_t g, double tau, int nsteps);
/* The state's coefficients by the trapezoidal rule of Sec. 2,
 * psihat = fftshift(fftn(psi)) prod sqrt(b_d - a_d) / N_d, in the layout of
 * nfft3_infft3 (C order, index i_d <-> frequency i_d - N_d/2): a time
 * snapshot ready for nfft3_infft3 / nfft3_tube_refine / the batched form. */
int nfft3_gpe_coeffs(nfft3_gpe_t g, void *psihat_dev);
int nfft3_gpe_destroy(nfft3_gpe_t g);

/* ---- Evaluation at a rectilinear grid (Sec. 2.1) ---------------------------
 * The series at every point of a grid y0 x y1 x y2 with arbitrary (not
 * necessarily equispaced) coordinates per axis:
 *
 *     F[i0][i1][i2] = sum_{k in I_N} fhat_k exp(-2 pi i (k0 y0[i0] + k1 y1[i1] + k2 y2[i2]))
 *
 * (the NFFT sign on the unit period, as nfft3_trafo; the paper's E^d matrices
 * and nested sums of Sec. 2.1).  Exact up to rounding (no window): three
 * dense complex matrix products, one per axis, on the matrix cores (FP64 or
 * FP32 MFMA), with the E^d tables formed on the device from the coordinates.
 * Cost 8 (N0 N1 N2 M2 + N0 N1 M1 M2 + N0 M0 M1 M2) real flops counted as
 * four real products per complex one; the matrix cores issue three (Gauss's
 * form), 6/8 of that. */
typedef struct nfft3_rgrid_s *nfft3_rgrid_t;

/* Plan for N[3] coefficients (N_d even, 2 <= N_d <= 16384) and M[3] grid
 * points per axis (1 <= M_d <= 2^20), dtype NFFT3_C64 / NFFT3_C128, on the
 * current device and the given stream (NULL = default).  Leading unit axes,
 * N_0 = M_0 = 1 (or also N_1 = M_1 = 1), give the two-dimensional form (the
 * double matrix product of the paper's igridft2, Appendix B) and the
 * one-dimensional one (the matrix-vector product E psihat of Appendix B):
 * their products are skipped and their coordinate pointers may be NULL.  Allocates the E^d
 * tables and two intermediates of N0 N1 M2 and N0 M1 M2 complex values. */
int nfft3_rgrid_plan(nfft3_rgrid_t *out, const int64_t N[3], const int64_t M[3], int dtype, void *stream);
int nfft3_rgrid_set_stream(nfft3_rgrid_t g, void *stream);
/* Grid coordinates: y_d_dev holds M_d FP64 values (device; any finite
 * reals, the series being 1-periodic).  Forms the E^d tables; synchronises
 * once to report NFFT3_ERR_NONFINITE. */
int nfft3_rgrid_set_axes(nfft3_rgrid_t g, const double *y0_dev, const double *y1_dev, const double *y2_dev);
/* out_dev[i0][i1][i2] (C order, M0 x M1 x M2 complex) = F at the grid;
 * fhat_dev: C-order (N0, N1, N2) complex, index i_d <-> k_d = i_d - N_d/2.
 * NFFT3_ERR_NO_POINTS before nfft3_rgrid_set_axes.  Does not synchronise. */
int nfft3_rgrid_eval(nfft3_rgrid_t g, const void *fhat_dev, void *out_dev);
/* Release the plan (NULL is a no-op). */
int nfft3_rgrid_destroy(nfft3_rgrid_t g);

/* ---- Tuning of the point binning (not in the paper; the window sums of
 * Sec. 2.2.1 at the plan's points are computed the same way for every
 * setting, only faster or slower) ---------------------------------------- */

/* tile: edge, in grid cells, of the (y, x) tiles the points are binned into
 * (a multiple of 4 from 8 to 32; the plane a work group stages in LDS is the
 * tile plus the 2m-1 halo).  items: points per work item of the window-sum kernels (256
 * or 512).  0 keeps the current value.  Defaults: tile 32, items 512.  A changed setting drops the plan's
 * points: call nfft3_set_points again.  INVALID_ARG for other values. */
int nfft3_set_tuning(nfft3_plan_t p, int tile, int items);
int nfft3_get_tuning(nfft3_plan_t p, int *tile, int *items);

/* Autotuner: times nfft3_trafo for every (tile, items) candidate on the
 * caller's points and coefficients (each candidate re-runs
 * nfft3_set_points on x_dev), keeps the fastest and leaves the points set
 * with it.  f_dev (M values) receives the transform outputs; reps >= 1
 * timed transforms per candidate (median).  Synchronizes the plan's
 * stream.  *tile_out / *items_out (may be NULL) receive the choice. */
int nfft3_autotune(nfft3_plan_t p, int64_t M, const double *x_dev, const void *fhat_dev, void *f_dev,
                   int reps, int *tile_out, int *items_out);

/* Release every buffer of the plan.  NULL is a no-op. */
int nfft3_destroy(nfft3_plan_t p);

/* Human-readable text for a status code (static storage). */
const char *nfft3_strerror(int code);
/* Text of the last HIP error seen by the library on this thread. */
const char *nfft3_last_hip_error(void);

/* ---- Introspection and stage access (diagnostics, tests, benchmarks) ---- */

/* n_out[3] = oversampled grid sizes; *M_out = points set (0 if none). */
int nfft3_get_info(nfft3_plan_t p, int64_t n_out[3], int64_t *M_out);

/* Stage (a)+(b): deconvolve fhat_dev (times -2 pi i k_d when deriv_axis is
 * 0, 1 or 2; plain when -1), zero-pad and FFT into the plan's grid. */
int nfft3_stage_grid(nfft3_plan_t p, const void *fhat_dev, int deriv_axis);
/* Stage (c): window sum of the plan's current grid at the points -> f_dev. */
int nfft3_stage_interp(nfft3_plan_t p, void *f_dev);
/* Adjoint stage (c^T): spread f_dev onto the plan's (zeroed) grid. */
int nfft3_stage_spread(nfft3_plan_t p, const void *f_dev);
/* Copy the plan's grid (n0 n1 n2 complex, C order, index l_d in [0, n_d))
 * to dst_dev (to_plan = 0) or from src into the plan (to_plan = 1). */
int nfft3_grid_copy(nfft3_plan_t p, void *buf_dev, int to_plan);

/* ---- Host-only helpers (no GPU needed) --------------------------------- */

/* Deconvolution factors of one axis: c[i] = phi(0) / I0(m sqrt(b^2 - (2 pi k/n)^2)),
 * k = i - Nd/2, b = pi (2 - 1/sigma); the factor that multiplies fhat_k before
 * the FFT when the window is normalised to phi(0) = 1.  c: Nd doubles. */
int nfft3_deconv_factors(int64_t Nd, double sigma, int m, double *c);

/* Window polynomials used on the device.  For stencil offset index
 * r = 0 .. 2m-1 (grid index u + r - m + 1 for a point in cell u with
 * fraction f in [0,1)), the normalised window phi(f - (r - m + 1)) / phi(0)
 * is sum_q coef[r*(deg+1) + q] * y^q with y = 2f - 1.  Writes the degree to
 * *deg (capacity: 2m*(cap_deg+1) doubles at coef) for the target accuracy of
 * dtype. */
int nfft3_window_poly(int m, double sigma, int dtype, int cap_deg, double *coef, int *deg);

#ifdef __cplusplus
}
#endif
#endif /* NFFT3_H */
