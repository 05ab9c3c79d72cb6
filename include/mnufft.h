/*
 * mnufft: 1D/2D/3D nonuniform FFTs of type 1 and type 2 (and type 3) on AMD Instinct MI355X
 * (gfx950), following the three-step method of cuFINUFFT (arXiv 2102.08463):
 * exponential-of-semicircle spreading / interpolation on an upsampled grid,
 * a fine-grid FFT, and deconvolution by the kernel's Fourier transform.
 *
 * C ABI.  Every entry point returns an int status (MNUFFT_OK = 0, a positive
 * value is a warning, a negative value an error) and never throws.  Pointers
 * to array data are device pointers unless a comment says otherwise.  Complex
 * data are interleaved (re, im) of the plan precision: float2 for
 * MNUFFT_F32, double2 for MNUFFT_F64.  A plan is not re-entrant: calls on
 * one plan must not overlap.
 *
 * Problem statement (Sec. I, eqs. 2d1 / 2d2 and their 3D analogue; 1D, which
 * the paper leaves out (Sec. I-B), is the same with one coordinate):
 *   type 1:  f_k = sum_{j<M} c_j exp(iflag * i * k.x_j),   k in I_N1 x I_N2 (x I_N3)
 *   type 2:  c_j = sum_k f_k exp(iflag * i * k.x_j),       j < M
 * with I_N = {k integer : -N/2 <= k < N/2} (eq. I) and points x_j in
 * [-pi, pi)^d.  The paper uses iflag = -1 for type 1 and +1 for type 2;
 * either sign is accepted here.  No normalisation is applied.
 *
 * Mode arrays f are stored with k1 fastest, each k_i ascending from
 * -floor(N_i/2); point arrays c are in the caller's point order.  With
 * ntransf > 1 the transforms are stacked: c is ntransf x M, f is
 * ntransf x (N1 N2 N3), all sharing the same points.
 */
#ifndef MNUFFT_H
#define MNUFFT_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ---------------------------------------------------- */
#define MNUFFT_OK                 0
#define MNUFFT_WARN_EPS_CLAMPED   1   /* eps below the precision floor; plan valid, width capped */
#define MNUFFT_ERR_ARG          (-1)  /* invalid argument; nothing was done */
#define MNUFFT_ERR_ALLOC        (-2)  /* device or host allocation failed */
#define MNUFFT_ERR_HIP          (-3)  /* a HIP runtime call failed */
#define MNUFFT_ERR_FFT          (-4)  /* rocFFT plan creation or execution failed */
#define MNUFFT_ERR_STATE        (-5)  /* call out of order (e.g. execute before setpts) */
#define MNUFFT_ERR_PTS          (-6)  /* a point is non-finite or outside [-3pi, 3pi) (validate_pts) */
#define MNUFFT_ERR_UNSUPPORTED  (-7)  /* valid request the library does not provide */

/* ---- precisions and methods ------------------------------------------ */
#define MNUFFT_F32 0
#define MNUFFT_F64 1

/* Spreading / interpolation methods (Sec. III-A, III-B).
 *   GM      one thread per point in user order, global-memory atomics
 *   GMSORT  one thread per point in bin-sorted order, global-memory atomics
 *   SM      bin-sorted subproblems of at most msub points, each accumulated
 *           in an LDS copy of its padded bin and added back to the grid
 *           (type 1); for type 2 the padded bin is staged through LDS and
 *           the points read it there
 *   AUTO    SM (the library's default) */
#define MNUFFT_METHOD_AUTO   0
#define MNUFFT_METHOD_GM     1
#define MNUFFT_METHOD_GMSORT 2
#define MNUFFT_METHOD_SM     3

typedef struct mnufft_opts {
    int   method;       /* MNUFFT_METHOD_*; default AUTO */
    int   binsize[3];   /* bin extents m_i in fine-grid cells; 0 selects the default,
                           64 in 1D, 32 x 32 in 2D and 16 x 8 x 8 in 3D (measured on gfx950; the
                           paper's V100 choice was 32 x 32 and 16 x 16 x 2, Sec. III-A,
                           first remark), halved along the longest side while the
                           padded bins of method SM do not fit in 160 KB of LDS */
    int   msub;         /* max points per subproblem, > 0; 0 selects 4096 (the paper
                           used 1024, same remark).  Default bins are also halved
                           along their longest side, down to 8 cells, while the fine
                           grid holds fewer than 1024 of them (small grids would
                           leave most compute units idle) */
    int   validate_pts; /* nonzero: setpts checks that every coordinate is finite and
                           in [-3pi, 3pi) and returns MNUFFT_ERR_PTS otherwise (this
                           synchronises the stream) */
    int   device;       /* HIP device ordinal, -1 = the current device */
    void *stream;       /* hipStream_t all work is ordered on; NULL = the null stream */
    double upsampfac;   /* fine-grid upsampling factor sigma: 0 or 2 selects the paper's
                           2 (Sec. II); values in [1.25, 2) use smaller fine grids with
                           wider kernels (see mnufft_choose_params_sigma) */
    int   tune;         /* MNUFFT_TUNE_*: OFF (default) keeps method, bins and msub as
                           given (or their defaults); AUTOTUNE or LEARNED make every
                           mnufft_setpts choose them for its points with mnufft_select
                           (types 1 and 2 in 2D / 3D; method must be AUTO and binsize,
                           msub 0); the plan re-plans its bin tables when the choice
                           changes, which never changes results beyond rounding */
    int   reserved[5];  /* must be zero */
} mnufft_opts;

/* Parameter selection modes (mnufft_opts.tune, mnufft_select). */
#define MNUFFT_TUNE_OFF      0
#define MNUFFT_TUNE_AUTOTUNE 1  /* time every autotuner candidate on the points (cached per class) */
#define MNUFFT_TUNE_LEARNED  2  /* the registered learned selector; the autotuner when none fits */

typedef struct mnufft_plan_s *mnufft_plan;

/* Read-only description of a plan (host memory). */
typedef struct mnufft_info {
    int     type, dim, prec, iflag;
    int64_t nmodes[3];     /* N_i (1 for unused dimensions) */
    int64_t nfine[3];      /* fine grid n_i: smallest 2^a 3^b 5^c >= max(2 N_i, 2w) (Sec. II) */
    int64_t ntransf;
    int64_t M;             /* points set by the last setpts, -1 before */
    int     w;             /* kernel width ceil(log10(1/eps)) + 1 (Sec. II), after clamping */
    double  beta;          /* 2.30 w (Sec. II) */
    int     method;        /* resolved method (never AUTO) */
    int     binsize[3];
    int     msub;
    int64_t nbins;         /* prod ceil(n_i / m_i) */
    int64_t nsub_max;      /* capacity of the subproblem list: nbins + ceil(M / msub) */
    int64_t device_bytes;  /* device memory owned by the plan */
    double  upsampfac;     /* sigma */
    int64_t ntargets;      /* type 3: frequencies K of the last setpts3 (-1 before); else 0.
                              For type 3, nmodes is the spreading grid nf (the inner type 2's
                              modes), nfine that type 2's fine grid and binsize / nbins /
                              method those of the spreading plan; all valid after setpts3 */
} mnufft_info;

/* Fill *o with the defaults listed in mnufft_opts.  Errors: ERR_ARG if o is NULL. */
int mnufft_default_opts(mnufft_opts *o);

/* Create a plan (Sec. I-A: plan, set up, execute, destroy).
 *   type     1 or 2; or 3 (see mnufft_setpts3)
 *   dim      1, 2 or 3
 *   nmodes   host array of dim entries N_i >= 1 (the rest ignored); unused and
 *            may be NULL for type 3
 *   iflag    +1 or -1, the sign in the exponent
 *   ntransf  >= 1 transforms sharing one set of points
 *   eps      requested relative l2 tolerance in (0, 1); sets w and beta (Sec. II)
 *   prec     MNUFFT_F32 or MNUFFT_F64
 *   opts     NULL for defaults
 *   out      receives the plan handle, owned by the caller until mnufft_destroy
 * Picks w, beta and the fine grid, computes the correction factors
 * p_k = (2/w) / phi_hat(alpha k) (Sec. II-A step 3) once, creates the rocFFT
 * plan and allocates the fine grid.  All arguments are validated before any
 * device call.  Returns MNUFFT_WARN_EPS_CLAMPED if eps needs w > 8 in F32 or
 * w > 16 in F64 (the plan then runs at the capped width).  Errors: ERR_ARG,
 * ERR_ALLOC, ERR_HIP, ERR_FFT; *out is NULL on error. */
int mnufft_makeplan(int type, int dim, const int64_t *nmodes, int iflag,
                    int64_t ntransf, double eps, int prec,
                    const mnufft_opts *opts, mnufft_plan *out);

/* Set the M nonuniform points (Sec. III-A bin-sort; the paper's setup stage).
 *   x, y, z  device arrays of M reals of the plan precision (z = NULL in 2D,
 *            y = z = NULL in 1D);
 *            coordinates in [-pi, pi); values in [-3pi, 3pi) are folded by
 *            whole periods, exactly.
 * Bins the points on the fine grid, builds the stable bin-sort permutation
 * (within a bin, points keep their input order) and the subproblem list, and
 * keeps its own sorted copy of the coordinates, so the caller may reuse x/y/z
 * once the stream has passed this call.  Stream-ordered, no host
 * synchronisation unless validate_pts is set.  M = 0 is allowed.
 * Errors: ERR_ARG (M < 0, M > 2^31 - 1, NULL x, or y / z given for an absent
 * dimension or missing for a present one), ERR_PTS, ERR_ALLOC, ERR_HIP. */
int mnufft_setpts(mnufft_plan p, int64_t M, const void *x, const void *y,
                  const void *z);

/* Type 3: nonuniform points to nonuniform frequencies (named as outside the
 * paper's scope in Sec. I-B and Sec. VI), by the published reduction of the
 * FINUFFT paper (Barnett, Magland, af Klinteberg, SIAM J. Sci. Comput. 2019):
 *   f_k = sum_{j<M} c_j exp(iflag * i * s_k.x_j),   k < K,
 * for real points x_j and real frequencies s_k of any range.  With C, X the
 * centre and half-width of the points and D, S those of the frequencies
 * (per dimension), the strengths are multiplied by exp(iflag i D.(x_j - C)),
 * spread at (x_j - C) / gamma onto nf cells of spacing h = 2 pi / nf
 * (nf = smallest even 2^a 3^b 5^c >= max(ceil(2 sigma S X / pi) + w + 1, 2w),
 * gamma = nf / (2 sigma S); S = 0 is read as 1/X, or 1 when X = 0 too), the
 * grid is transformed by a type 2 plan (modes -nf/2 .. nf/2 - 1) at
 * t_k = h gamma (s_k - D), and the result is multiplied by
 * exp(iflag i s_k.C) prod_d (2/w) / phi_hat(w t_kd / 2).
 *   x, y, z  device arrays of M reals of the plan precision (y from 2D, z only in 3D)
 *   s, t, u  device arrays of K reals (t from 2D, u only in 3D)
 * Reads the bounds of both sets back to the host (synchronises the stream),
 * then makes the spreading and type 2 plans (again only when nf changes)
 * and bin-sorts both rescaled sets.  mnufft_execute then takes c (ntransf x M)
 * and writes f (ntransf x K); the adjoint, spread / interp, gradient and
 * sort introspection calls return ERR_UNSUPPORTED on a type 3 plan.
 * M = 0 or K = 0 is allowed.  Errors: ERR_ARG (not a type 3 plan, sizes out
 * of range, a needed pointer NULL or a pointer given for an absent dimension, nf above 2^24 in some
 * dimension), ERR_PTS (a non-finite coordinate), ERR_ALLOC, ERR_HIP, ERR_FFT. */
int mnufft_setpts3(mnufft_plan p, int64_t M, const void *x, const void *y, const void *z,
                   int64_t K, const void *s, const void *t, const void *u);

/* Run the transform (Sec. II-A for type 1, Sec. II-B for type 2).
 *   type 1: c is input (ntransf x M complex), f is output (ntransf x N1 N2 N3)
 *   type 2: f is input, c is output
 * The output is overwritten.  Asynchronous on the plan's stream.
 * Errors: ERR_STATE (no setpts), ERR_ARG (NULL pointer with M > 0), ERR_HIP, ERR_FFT. */
int mnufft_execute(mnufft_plan p, void *c, void *f);

/* mnufft_execute with the point-indexed array c in bin-sorted order instead
 * of the caller's point order: c[t][i] belongs to the point at sorted
 * position i, i.e. to input point perm[i] (mnufft_get_sort).  Spreading then
 * reads, and interpolation writes, c contiguously instead of through the
 * permutation, which is what bounds those kernels for random points; a
 * caller that applies the transform many times to the same points (an
 * iterative solver) can keep its vectors in this order.  Results equal
 * mnufft_execute's bit for bit after the permutation.  Errors as
 * mnufft_execute; ERR_UNSUPPORTED for type 3 and method GM (no sort). */
int mnufft_execute_sorted(mnufft_plan p, void *c, void *f);

/* Apply the adjoint of the plan's operator on the same sorted points: the
 * other type with the opposite sign (type 2 is the adjoint of type 1, Sec. I).
 * Same array roles as mnufft_execute with the directions swapped: for a
 * type 1 plan, f is input and c is output; for a type 2 plan, c is input and
 * f is output.  Errors as mnufft_execute. */
int mnufft_execute_adjoint(mnufft_plan p, void *c, void *f);

/* Position gradient by ES-derivative interpolation (for the backward pass
 * of a type 1 or type 2 transform).  Let v(x) be the type 2 sum of `modes`
 * with the sign of the plan's type 2 direction (iflag for a type 2 plan,
 * -iflag for a type 1 plan), computed by the plan's method on its points,
 * i.e. precorrection, FFT and interpolation (Sec. II-B) with the kernel
 * replaced by its derivative phi'(z) = -beta z (1 - z^2)^(-1/2) phi(z) in one
 * dimension.  Then, for every point j and dimension i,
 *   gx_i[j] = sum over transforms t of Re(conj(wts[t][j]) * d v_t(x_j) / dx_i).
 * For a type 2 plan (c = A f): modes = f and wts = dL/dRe c + i dL/dIm c give
 * dL/dx.  For a type 1 plan (f = A c): modes = dL/dRe f + i dL/dIm f and
 * wts = c give dL/dx.
 *   modes   ntransf x N1 N2 (N3) complex, k1 fastest
 *   wts     ntransf x M complex, input point order
 *   gx, gy, gz   M reals each (gy from 2D, gz only in 3D), input order, overwritten
 * Errors: ERR_STATE, ERR_ARG, ERR_HIP, ERR_FFT. */
int mnufft_interp_grad(mnufft_plan p, const void *modes, const void *wts, void *gx, void *gy,
                       void *gz);

/* Step 1 of type 1 alone (Sec. II-A): grid = sum_j c_j psi_per(l h - pi - x_j)
 * for the first transform, with the plan's method.  grid is caller-owned,
 * n1 n2 (n3) complex, first coordinate fastest, overwritten.  Grid point l
 * sits at l h - pi (the lattice that bins points in Sec. III-A).
 * Errors: ERR_STATE, ERR_ARG, ERR_HIP. */
int mnufft_spread(mnufft_plan p, const void *c, void *grid);

/* Step 3 of type 2 alone (Sec. II-B): c_j = sum_l grid_l psi_per(l h - pi - x_j)
 * for one vector, with the plan's method.  Same grid layout as mnufft_spread;
 * c (M complex) is overwritten.  Errors as mnufft_spread. */
int mnufft_interp(mnufft_plan p, const void *grid, void *c);

/* Copy the bin-sort result into caller-owned device buffers (stream-ordered):
 *   perm      M int32: perm[i] = input index of the point at sorted position i
 *   binstart  nbins + 1 int32: first sorted position of each bin, binstart[nbins] = M
 * Either pointer may be NULL.  Errors: ERR_STATE, ERR_HIP. */
int mnufft_get_sort(mnufft_plan p, int32_t *perm, int32_t *binstart);

/* Copy the subproblem list (Sec. III-A, SM step 1) into caller-owned device
 * buffers: sub holds nsub_max records of 4 int32 (bin, first sorted position,
 * number of points, 0) in bin order, and *nsub (device int32) the number of
 * records in use.  Errors: ERR_STATE, ERR_HIP. */
int mnufft_get_subproblems(mnufft_plan p, int32_t *sub, int32_t *nsub);

/* Move the plan to another stream (hipStream_t; NULL = the null stream): every
 * later call is ordered on it; ordering against work already enqueued on the
 * old stream is the caller's.  The call also creates the FFT plan of the
 * direction not used so far, so that afterwards mnufft_execute and
 * mnufft_execute_adjoint enqueue kernels only (no allocation, no host
 * synchronisation) and can be captured into a HIP graph once each has run
 * eagerly.  A type 3 plan moves its inner plans too; mnufft_setpts3 itself
 * synchronises and is not capturable.  Errors: ERR_ARG, ERR_ALLOC, ERR_FFT. */
int mnufft_set_stream(mnufft_plan p, void *stream);

/* Describe the plan (host memory).  Errors: ERR_ARG. */
int mnufft_get_info(mnufft_plan p, mnufft_info *info);

/* Synchronise the plan's stream, free everything the plan owns and the plan
 * itself.  NULL is accepted and ignored.  Errors: ERR_HIP. */
int mnufft_destroy(mnufft_plan p);

/* Stage timers.  When enabled, the library brackets each stage it enqueues
 * with a pair of HIP events on the plan's stream, so the figures are device
 * durations of exactly that stage's kernels (one kernel launch per stage and
 * transform for SPREAD, INTERP, DECONV and PRECORRECT; two for ADDBACK).  Reading them
 * synchronises the stream. */
#define MNUFFT_STAGE_SETPTS     0  /* the whole bin-sort of mnufft_setpts */
#define MNUFFT_STAGE_ZERO       1  /* clearing the fine grid before spreading */
#define MNUFFT_STAGE_SPREAD     2  /* type 1 step 1 (Sec. II-A); for SM the LDS tile kernel */
#define MNUFFT_STAGE_FFT        3  /* rocFFT of the fine grid (either sign) */
#define MNUFFT_STAGE_DECONV     4  /* type 1 step 3 (Sec. II-A) */
#define MNUFFT_STAGE_PRECORRECT 5  /* type 2 step 1 (Sec. II-B) */
#define MNUFFT_STAGE_INTERP     6  /* type 2 step 3 (Sec. II-B) */
#define MNUFFT_STAGE_ADDBACK    7  /* SM only: adding the padded-bin tiles into the grid
                                      (Sec. III-A, SM step 3) */
#define MNUFFT_STAGE_SCALE      8  /* SM only: max |c| pre-pass fixing the fixed-point scale */
#define MNUFFT_NSTAGES          9

/* Turn the stage timers on (nonzero) or off.  Errors: ERR_ARG. */
int mnufft_set_timing(mnufft_plan p, int enable);

/* Sum of the recorded durations per stage in milliseconds (ms[MNUFFT_NSTAGES],
 * host) and the number of recorded intervals (count[MNUFFT_NSTAGES], host,
 * may be NULL) since the last reset; reset != 0 clears them afterwards.
 * Synchronises the plan's stream.  Errors: ERR_ARG, ERR_HIP. */
int mnufft_get_timing(mnufft_plan p, double *ms, int64_t *count, int reset);

/* Host-only helpers (no device call; usable without a GPU). */

/* Parameters of Sec. II for one dimension: kernel width w = ceil(log10(1/eps)) + 1
 * (at least 2; capped at 8 in F32 and 16 in F64), beta = 2.30 w, and the fine
 * grid n = smallest 2^a 3^b 5^c >= max(2N, 2w).  Outputs are host pointers.
 * Returns MNUFFT_WARN_EPS_CLAMPED when the cap applied.  Errors: ERR_ARG. */
int mnufft_choose_params(double eps, int prec, int64_t N, int *w, double *beta, int64_t *n);

/* The same for an upsampling factor sigma: sigma = 2 gives exactly the rule
 * above; sigma in [1.25, 2), which the paper names as future work (Sec. VI),
 * uses the published rule of the FINUFFT paper (Barnett, Magland and
 * af Klinteberg, SIAM J. Sci. Comput. 2019): w = ceil(ln(1/eps) / (pi
 * sqrt(1 - 1/sigma))), beta = 0.97 pi w (1 - 1/(2 sigma)), and n = smallest
 * 2^a 3^b 5^c >= max(ceil(sigma N), 2w).  In F32 eps is first raised to 1e-7
 * (the rule above's cap of w = 8 at sigma = 2); w is capped at 16.  Returns
 * MNUFFT_WARN_EPS_CLAMPED when a cap applied.  Errors: ERR_ARG (also for sigma
 * outside [1.25, 2]). */
int mnufft_choose_params_sigma(double eps, int prec, int64_t N, double sigma, int *w,
                               double *beta, int64_t *n);

/* The N per-dimension correction factors of Sec. II-A step 3, as the library
 * computes them at plan time (host array out, double):
 *   out[i] = (2/w) / phi_hat(alpha k) * (-1)^k,  k = i - floor(N/2),  alpha = w pi / n,
 * with phi_hat(xi) = int_{-1}^{1} exp(beta (sqrt(1-z^2) - 1)) exp(-i xi z) dz
 * evaluated by tanh-sinh quadrature.  The factor (-1)^k comes from placing
 * grid point l at l h - pi.  Errors: ERR_ARG (N < 1, n < 2N, w outside 2..16,
 * beta <= 0, out NULL). */
int mnufft_correction_factors(int64_t N, int64_t n, int w, double beta, double *out);

/* Grid of the type 3 reduction for one dimension (see mnufft_setpts3): from
 * the half-width X of the points and S of the frequencies, *nf = smallest even
 * 2^a 3^b 5^c >= max(ceil(2 sigma S X / pi) + w + 1, 2w) and
 * *gamma = nf / (2 sigma S), with S = 0 read as 1/X (1 if X = 0 too).  Host
 * only; outputs are host pointers.  Errors: ERR_ARG (X or S negative or not a
 * number, sigma outside [1.25, 2], w outside 2..16, nf above 2^24). */
int mnufft_type3_grid(double X, double S, double sigma, int w, int64_t *nf, double *gamma);

/* ---- autotuning ------------------------------------------------------- */

/* The parameter sets the autotuner searches for a dimension, precision and
 * tolerance: method SM with several bin shapes (those whose padded bins fit
 * in LDS; in 2D every m_1 >= m_2 from {8, 16, 32, 64, 128}) times msub (2D:
 * {1024, 4096}; 3D: {256, 1024, 4096, 16384}), then GMSORT and GM, in this
 * fixed order.  Writes min(count, cap) default-initialised options with
 * method, binsize and msub set (host array, may be NULL when cap = 0) and
 * returns the count (>= 0).  Host only.  Errors: ERR_ARG.  (The paper tuned
 * bins and msub by hand on its GPU: Sec. III-A, first remark.) */
int mnufft_tune_candidates(int dim, int prec, double eps, mnufft_opts *list, int cap);

/* Time setpts + execute of one transform for each candidate (one plan is
 * made, untimed, and given each candidate's method, bins and msub in turn;
 * stream, device and upsampfac come from the first candidate), in
 * milliseconds of device time measured with HIP events on that stream: the median of `reps` runs after
 * one warm-up run; a candidate whose warm-up takes more than cutoff (> 1)
 * times the best median so far keeps that single time.  Candidates that are
 * invalid for the problem get -1.  x, y, z, c, f are device arrays as for
 * mnufft_setpts / mnufft_execute (c and f both needed: input and output);
 * ms is a host array of ncand entries.  Synchronises.  Errors: ERR_ARG,
 * ERR_HIP. */
int mnufft_tune_time(int type, int dim, const int64_t *nmodes, int iflag, double eps, int prec,
                     int64_t M, const void *x, const void *y, const void *z, void *c, void *f,
                     const mnufft_opts *cands, int ncand, int reps, double cutoff, double *ms);

/* ---- learned parameter selector --------------------------------------- */

/* Point-density features: the points' (x, y) are counted on a 16 x 16
 * periodic grid over [-pi, pi)^2 (cell = floor of the folded coordinate
 * (x + pi) 16 / (2 pi), the bin-sort's recipe on 16 cells) and
 * feat[cx + 16 cy] = log(1 + 256 count / M) (0 when M = 0).  x, y: device
 * arrays of M reals of precision prec; feat: device array of 256 floats;
 * work: device scratch of MNUFFT_DENSITY_WORK_BYTES bytes.  Stream-ordered.
 * Errors: ERR_ARG, ERR_HIP. */
#define MNUFFT_DENSITY_WORK_BYTES (512 * 256 * 4)
int mnufft_density_features(int prec, int64_t M, const void *x, const void *y, float *feat,
                            void *work, void *stream);

/* The same features for T point sets stored back to back: set t is points
 * off[t] .. off[t+1]-1 of x, y (off: device array of T + 1 nondecreasing
 * int64, off[0] = 0); its 256 features go to feat + t * ldf (ldf >= 256).
 * work: device scratch of T * MNUFFT_DENSITY_BATCH_WORK_BYTES bytes (cleared
 * by the call itself).  Three kernel launches whatever T; the points are
 * split evenly over the GPU whatever the set sizes.  Errors: ERR_ARG (T < 1 or above 65535, NULL
 * pointers, ldf < 256), ERR_HIP. */
#define MNUFFT_DENSITY_BATCH_WORK_BYTES (32 * 256 * 4)
int mnufft_density_features_batch(int prec, int T, const int64_t *off, const void *x,
                                  const void *y, float *feat, int ldf, void *work, void *stream);

/* mnufft_density_features_batch without a workspace argument, for callers
 * that cannot allocate device memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid allocation): the partial histograms
 * go to a workspace of MNUFFT_DENSITY_NOALLOC_MAX_SETS *
 * MNUFFT_DENSITY_BATCH_WORK_BYTES bytes (2 MiB) that the library holds in
 * static device memory, one copy per GPU for the life of the process (its
 * address is looked up on the first call on each device; the call allocates
 * nothing).  All calls on one GPU share that workspace, so calls that
 * overlap on one GPU (on different streams or host threads) race and must
 * be ordered by the caller.  Same arguments and results as
 * mnufft_density_features_batch otherwise.  Errors: ERR_ARG (also for
 * T > MNUFFT_DENSITY_NOALLOC_MAX_SETS), ERR_HIP. */
#define MNUFFT_DENSITY_NOALLOC_MAX_SETS 64
int mnufft_density_features_batch_noalloc(int prec, int T, const int64_t *off, const void *x,
                                          const void *y, float *feat, int ldf, void *stream);

/* A multilayer perceptron F -> H -> H -> K with ReLU after the two hidden
 * layers, in single precision, all arrays on the device, all calls ordered on
 * `stream` (a hipStream_t).  Parameters are one flat array laid out as
 * W1 (F x H, row i holds input i's weights), b1 (H), W2 (H x H), b2 (H),
 * W3 (H x K), b3 (K); gradients use the same layout.  Errors: ERR_ARG, ERR_HIP. */
int64_t mnufft_mlp_nparams(int F, int H, int K);

/* H1 = relu(X W1 + b1), H2 = relu(H1 W2 + b2), Y = H2 W3 + b3 for a batch of
 * B rows (X: B x F, H1, H2: B x H, Y: B x K, row-major). */
int mnufft_mlp_forward(int F, int H, int K, const float *params, int B, const float *X, float *H1,
                       float *H2, float *Y, void *stream);

/* Masked mean squared error over the B x K entries:
 * *loss = sum mask (Y - T)^2 / max(1, sum mask), dY = 2 mask (Y - T) / max(1, sum mask). */
int mnufft_mlp_loss_grad(int K, int B, const float *Y, const float *T, const float *mask, float *dY,
                         float *loss, void *stream);

/* Gradient of the loss w.r.t. the parameters given dY and the forward
 * activations; work holds 2 B H floats. */
int mnufft_mlp_backward(int F, int H, int K, const float *params, int B, const float *X,
                        const float *H1, const float *H2, const float *dY, float *work,
                        float *grads, void *stream);

/* One Adam step (step >= 1) over n parameters with moments m, v. */
int mnufft_mlp_adam(int64_t n, float *params, const float *grads, float *m, float *v, float lr,
                    float beta1, float beta2, float eps, int step, void *stream);

/* Register a learned selector from a file (host path), replacing one of the
 * same dimension, precision and tolerance.  Format (little-endian): the 8
 * bytes "MNSEL001"; int32 dim, prec; double eps; int32 F, H, K; double
 * margin; K records of int32 (method, binsize[0..2], msub) that must equal
 * mnufft_tune_candidates(dim, prec, eps) in order; then the
 * mnufft_mlp_nparams(F, H, K) float32 parameters of the network, and
 * nothing after them.  1 <= H <= 256.  F must be 262: the 256 density features of
 * mnufft_density_features followed by log2 M / 24, log2 n_i / 12 (i = 1..3,
 * 0 for an absent dimension; n_i the sigma = 2 fine grid), w / 16 and the
 * type minus one.  The network predicts each candidate's log run time
 * relative to the fastest; a prediction whose runner-up is less than
 * `margin` behind is left to the autotuner.  Errors: ERR_ARG (unreadable
 * file, bad format, candidate list mismatch). */
int mnufft_selector_load(const char *path);

/* Forget every registered selector and the autotuner's cached choices. */
int mnufft_selector_clear(void);

/* Choose method, bins and msub for one type 1 / 2 problem on its points.
 *   mode    MNUFFT_TUNE_AUTOTUNE: time every candidate of mnufft_tune_candidates
 *           (setpts + execute, mnufft_tune_time) on these points and take the
 *           fastest; the choice is cached per problem class (type, dimension,
 *           precision, tolerance, rounded log2 of N_i and M, and the points'
 *           clustering level from the density features) for later calls.
 *           MNUFFT_TUNE_LEARNED: the registered selector's argmin over all
 *           candidates from the density features, or the autotuner when no
 *           selector is registered for (dim, prec, eps) or its margin is not met.
 *   base    NULL or options whose stream, device and upsampfac are used
 *   out     receives the chosen options (the base's stream, device, upsampfac)
 *   source  NULL, or receives 0 (learned prediction) or 1 (autotuner)
 * x, y, z as for mnufft_setpts.  Synchronises the stream.  Errors: ERR_ARG,
 * ERR_ALLOC, ERR_HIP, ERR_FFT. */
int mnufft_select(int type, int dim, const int64_t *nmodes, int iflag, double eps, int prec,
                  int64_t M, const void *x, const void *y, const void *z, int mode,
                  const mnufft_opts *base, mnufft_opts *out, int *source);

/* Choose bins and msub (method SM) for each transform of a batch from its
 * points, for mnufft_batch_makeplan: arguments as mnufft_batch_makeplan and
 * mnufft_batch_setpts; binsize (ntr x 3) and msub (ntr) are host arrays that
 * receive the choices, source (ntr, may be NULL) 0 for a learned prediction
 * and 1 for the autotuner.  With MNUFFT_TUNE_LEARNED and a registered
 * selector, all transforms are scored by one batched density-histogram pass,
 * one forward pass of the network and one argmin launch on the device (the
 * scalar features are computed on the host and copied once); transforms
 * whose margin is not met, or all of them with MNUFFT_TUNE_AUTOTUNE, are
 * timed by the autotuner on their own points.  Synchronises the stream.
 * Errors: ERR_ARG, ERR_ALLOC, ERR_HIP, ERR_FFT. */
int mnufft_batch_select(int type, int dim, int ntr, const int64_t *nmodes, const int64_t *npts,
                        const void *x, const void *y, const void *z, double eps, int prec,
                        int mode, const mnufft_opts *base, int32_t *binsize, int32_t *msub,
                        int32_t *source);

/* ---- batches of transforms of uneven size ---------------------------- */

/* A batch runs ntr independent transforms of one type, dimension, sign,
 * tolerance and precision, each with its own modes and points, as one
 * workload: one bin-sort over all points (the transforms' bins numbered
 * consecutively), one subproblem list, and one persistent launch each for
 * spreading, the add-back of the padded bins, interpolation and the
 * corrections (method SM, Sec. III-A); only the fine-grid FFTs run per
 * transform.  Inputs and outputs are concatenated in transform order. */
typedef struct mnufft_batch_s *mnufft_batch;

/* Create a batch.
 *   type, dim, iflag, eps, prec   as in mnufft_makeplan, shared by all transforms
 *   ntr       number of transforms, >= 1
 *   nmodes    host array ntr x 3: N_1, N_2 (, N_3) of transform t at 3t ..
 *   npts      host array ntr: points of each transform (>= 0, total <= 2^31 - 1)
 *   binsize   host array ntr x 3 of bin extents, or NULL; 0 entries take
 *             opts->binsize or the plan default
 *   msub      host array ntr of subproblem sizes, or NULL; 0 entries take
 *             opts->msub or the plan default
 *   opts      NULL or options; method must be AUTO or SM
 * The padded bins of the largest bin extents must fit in LDS.  Errors:
 * ERR_ARG, ERR_UNSUPPORTED (method GM / GMSORT), ERR_ALLOC, ERR_HIP, ERR_FFT;
 * returns MNUFFT_WARN_EPS_CLAMPED like mnufft_makeplan. */
int mnufft_batch_makeplan(int type, int dim, int ntr, const int64_t *nmodes,
                          const int64_t *npts, int iflag, double eps, int prec,
                          const int32_t *binsize, const int32_t *msub,
                          const mnufft_opts *opts, mnufft_batch *out);

/* Set all points: x, y (, z) device arrays of sum(npts) reals of the batch
 * precision, transform 0's points first.  Stream-ordered.  Errors: ERR_ARG,
 * ERR_HIP. */
int mnufft_batch_setpts(mnufft_batch b, const void *x, const void *y, const void *z);

/* Execute all transforms.  c: sum(npts) complex (concatenated per transform);
 * f: sum over t of N_1 N_2 (N_3) complex (concatenated, k1 fastest).  Type 1
 * reads c and overwrites f; type 2 reads f and overwrites c.  Errors:
 * ERR_STATE, ERR_ARG, ERR_HIP, ERR_FFT. */
int mnufft_batch_execute(mnufft_batch b, void *c, void *f);

/* Stage timers of a batch (same stages and semantics as for plans). */
int mnufft_batch_set_timing(mnufft_batch b, int enable);
int mnufft_batch_get_timing(mnufft_batch b, double *ms, int64_t *count, int reset);

/* totals[6] (host): points, modes, fine-grid cells, bins, subproblem
 * capacity, device bytes owned.  Errors: ERR_ARG. */
int mnufft_batch_get_totals(mnufft_batch b, int64_t *totals);

/* Synchronise and free; NULL is ignored.  Errors: ERR_HIP. */
int mnufft_batch_destroy(mnufft_batch b);

/* Human-readable name of a status code (static storage, never NULL). */
const char *mnufft_strerror(int status);

#ifdef __cplusplus
}
#endif

#endif /* MNUFFT_H */
