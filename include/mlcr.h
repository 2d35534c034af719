/*
 * mlcr.h -- C ABI of the multi-level constrained-realization (CR) library
 * for AMD MI355X (gfx950).
 *
 * The library applies the CR system operator of Seljebotn, Mardal, Jewell,
 * Eriksen & Bull (2013), "A multi-level solver for Gaussian constrained CMB
 * realizations":
 *
 *     A   = S^-1 + B Y^T N^-1 Y B                 (Sec. 2.3, eq. system-explicit)
 *     A_h = D_h + B_h Y^T N^-1 Y B_h              (Sec. 3.2, eq. A_h)
 *
 * and solves A x = b with the multi-level cycle of Fig. code:mg.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - Harmonic vectors are "real packed, m-major", float64, length
 *   (lmax+1)^2 per right-hand side: first x_l0 for l = 0..lmax, then for
 *   m = 1..lmax a cosine block (l = m..lmax) followed by a sine block
 *   (l = m..lmax).  The basis is real and orthonormal on the sphere:
 *       f = sum_l x_l0 L_l0 + sum_{m>=1} sqrt(2) L_lm (x^c_lm cos m phi + x^s_lm sin m phi),
 *   L_lm the normalized associated Legendre function of Sec. 3.2 (the
 *   formula beside eq. Ni-dense), Condon-Shortley phase included.
 * - Maps are float64 HEALPix RING order (Gorski et al. 2005; Sec. 2.1),
 *   12 nside^2 pixels per right-hand side.
 * - Batches are contiguous: right-hand side r starts at r * (lmax+1)^2
 *   (harmonic) or r * 12 nside^2 (pixel).
 * - Pointers named dev_* are device pointers owned by the caller (maps and
 *   N^-1 must be 16-byte aligned, as every torch/hipMalloc allocation is); the
 *   library never frees them.  Pointers named host_* are host memory read
 *   during the call only.  `stream` is a hipStream_t (NULL = default
 *   stream); all device work of a call is enqueued on it.
 * - prec selects the arithmetic of the Legendre contraction and the ring
 *   FFTs only (MLCR_FP64, MLCR_FP32 or MLCR_BF16X3, below); inputs and
 *   outputs are always float64.
 * - Return value: 0 on success, a negative MLCR_E* code otherwise; a
 *   description is available from mlcr_last_error() (thread-local).
 *   Argument errors are detected before any device work is enqueued.
 */
#ifndef MLCR_H
#define MLCR_H

#ifdef __cplusplus
extern "C" {
#endif

enum {
    MLCR_OK = 0,
    MLCR_EINVAL = -1,       /* bad argument (null pointer, size out of range, ...) */
    MLCR_ENOMEM = -2,       /* device or host allocation failed                    */
    MLCR_EHIP = -3,         /* HIP runtime error                                   */
    MLCR_ENOTPD = -4,       /* Cholesky of a matrix that is not positive definite  */
    MLCR_ENOCONV = -5,      /* solver did not reach the tolerance                  */
    MLCR_EUNSUPPORTED = -6  /* valid request the library does not implement      */
};

/* Arithmetic of the Legendre contraction:
 *   MLCR_FP64   float64 throughout;
 *   MLCR_FP32   lambda and coefficients rounded to float32, float32 products
 *               and accumulation on the matrix cores;
 *   MLCR_BF16X3 each float32 operand split into bfloat16 hi + lo, products
 *               hi*hi + hi*lo + lo*hi with float32 accumulation (about
 *               3 * 2^-18 relative per product).
 * On both mixed paths the adjoint's sums over the ring-pair blocks of one
 * workgroup are float32 too; its per-workgroup partial sums are added in
 * float64.  The recurrence, its seeds and range scaling are float64 in every
 * mode.  On the FP32 and BF16X3 paths the per-ring FFTs (and, in apply_A,
 * the N^-1 product between them) run in float32 as well; the ring fold and
 * unfold with their phases, and every input and output, stay float64. */
enum { MLCR_FP64 = 0, MLCR_FP32 = 1, MLCR_BF16X3 = 2 };

typedef struct mlcr_geom mlcr_geom;
typedef struct mlcr_op mlcr_op;
typedef struct mlcr_solver mlcr_solver;

/* Thread-local text of the last error of this thread ("" if none). */
const char *mlcr_last_error(void);

/* Library version string. */
const char *mlcr_version(void);

/* Per-kernel timing (measurement support, Sec. 4.1 reports per-step cost):
 * when enabled, every kernel launch of the library is bracketed by a pair
 * of HIP events on its stream; totals accumulate per kernel name.
 * mlcr_timing_get synchronizes on the recorded events.  Not thread-safe. */
int mlcr_timing_enable(int on);
int mlcr_timing_reset(void);
int mlcr_timing_count(void);
int mlcr_timing_get(int i, char *name, int name_len, double *total_ms, long long *calls);

/* ------------------------------------------------------------------------
 * Geometry: HEALPix RING grid of resolution nside (Sec. 2.1) together with
 * the tables of the Legendre recurrence up to lmax and of the per-ring
 * FFTs.  1 <= nside <= 2048 (a power of two is not required; the largest
 * ring FFT must fit in one workgroup's LDS);
 * 0 <= lmax <= 16384.  Allocates device memory for the tables
 * (about 16 (lmax+1)^2 / 2 + 48 * 12 nside^2 bytes) and a workspace that
 * grows on demand.  The handle may be used from one host thread at a time.
 * ---------------------------------------------------------------------- */
int mlcr_geom_create(int nside, int lmax, mlcr_geom **out);
/* Gauss-Legendre grid (Sec. 3.4): nrings rings at the nodes z_k of the
 * Legendre polynomial P_nrings, ordered north to south, each with nphi
 * equispaced pixels from phi = 0 (pixel index k nphi + j).  The quadrature
 * sum_k W_k sum_j f(theta_k, phi_j) (mlcr_geom_weights) is exact for
 * polynomials in cos theta of degree < 2 nrings with frequencies |m| < nphi.
 * nphi: multiple of 4, at most 16384, whose ring FFT fits 8192 points
 * (nphi/2 a power of two, or nphi <= 4096).  The same transforms apply. */
int mlcr_geom_create_gl(int lmax, int nrings, int nphi, mlcr_geom **out);
void mlcr_geom_destroy(mlcr_geom *g);
/* nside (0 for a Gauss-Legendre grid), lmax, pixel count and ring count of a
 * geometry; any out pointer may be NULL. */
int mlcr_geom_info(const mlcr_geom *g, int *nside, int *lmax, long long *npix, int *nrings);
/* Quadrature weight of one pixel of each ring, host_w[nrings]: 4 pi / N_pix
 * for HEALPix (equal area), W_k = w_k 2 pi / nphi for Gauss-Legendre. */
int mlcr_geom_weights(const mlcr_geom *g, double *host_w);
/* Launch shapes of the transform kernels on this geometry for one arithmetic
 * path (prec = MLCR_FP64 / FP32 / BF16X3), as chosen by an autotuner (the
 * Python package's autotune module times every choice on the workload):
 *   adjoint_waves  4 or 8: ring-pair blocks of 64 per matrix-core adjoint
 *                  workgroup (the split-K chunk count is blocks / waves);
 *   synth_chains   2 or 4: recurrence chains per lane of the matrix-core
 *                  synthesis (16 x chains ring pairs per wave);
 *   ring_threads   512 or 1024: threads per ring workgroup for FFT sizes
 *                  above 4096 (smaller FFTs always use 512).
 * Defaults 8, 4, 1024.  Results agree between choices up to rounding order.
 * Host-side only; applies to launches made after the call (a solver's
 * captured cycle graph keeps the shapes it was captured with) and only to
 * this geometry (not to the Gauss-Legendre geometries of an operator's
 * lower levels).  Errors: MLCR_EINVAL for another value or precision. */
int mlcr_geom_set_tuning(mlcr_geom *g, int prec, int adjoint_waves, int synth_chains,
                         int ring_threads);
/* The current launch shapes of one path; any out pointer may be NULL. */
int mlcr_geom_get_tuning(const mlcr_geom *g, int prec, int *adjoint_waves, int *synth_chains,
                         int *ring_threads);

/* Spherical harmonic synthesis map = Y alm (Sec. 2.1, eq. sh-synthesis),
 * evaluated exactly at the pixel centres (no quadrature, any lmax <= the
 * geometry's lmax, including lmax > 3 nside).
 *   dev_alm: [nrhs][(lmax+1)^2] float64;  dev_map: [nrhs][12 nside^2] float64.
 * nrhs >= 1.  EINVAL on null pointers or lmax out of range. */
int sht_synth(mlcr_geom *g, int lmax, int nrhs, const double *dev_alm, double *dev_map,
              int prec, void *stream);

/* sht_synth with prec = MLCR_FP64 for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc): it calls no hipMalloc, hipFree or allocating routine.
 * Its workspaces (packed input and ring-major Fourier coefficients,
 * 8 nrhs (lmax+1)(lmax+2) + 16 nrhs nrings (lmax+1) bytes, rounded) live in
 * one fixed 64 MiB device array per GPU, held until the process ends;
 * requests that need more return MLCR_EINVAL (use sht_synth).  Every call on
 * a GPU shares that array: calls that overlap on one GPU race.  Runs the
 * float64 vector Legendre kernels for any nrhs; results equal sht_synth's
 * float64 path up to rounding order.  Arguments and layouts as sht_synth. */
int sht_synth_noalloc(mlcr_geom *g, int lmax, int nrhs, const double *dev_alm, double *dev_map,
                      void *stream);

/* Adjoint synthesis alm = Y^T map (Sec. 2.1: the transpose of Y, with no
 * quadrature weights; used in place of analysis throughout the method).
 * Same layouts as sht_synth. */
int sht_adjoint(mlcr_geom *g, int lmax, int nrhs, const double *dev_map, double *dev_alm,
                int prec, void *stream);

/* ------------------------------------------------------------------------
 * Operator A = S^-1 + B Y^T N^-1 Y B on the observation grid g
 * (Sec. 2.3, eq. system-explicit).
 *   host_cl[lmax+1]:  prior power spectrum C_l >= 0; C_l = 0 removes all
 *                     modes of that l from the unknowns (their inputs are
 *                     ignored and their outputs are 0).
 *   host_bl[lmax+1]:  beam times pixel window b_l p_l (Sec. 2.2).
 *   dev_ninv[12 nside^2]: inverse noise variance per pixel, 0 in the mask
 *                     (Sec. 2.3), must stay valid while the operator lives.
 *   lmax: band limit of the unknowns (<= the geometry's lmax).
 *   max_nrhs: largest batch later passed to apply_A / wcycle_solve.
 * The operator keeps a reference to g (which must outlive it) and copies
 * host_cl and host_bl.  EINVAL on negative C_l or sizes out of range. */
int mlcr_op_create(mlcr_geom *g, int lmax, const double *host_cl, const double *host_bl,
                   const double *dev_ninv, int max_nrhs, mlcr_op **out);
void mlcr_op_destroy(mlcr_op *op);

/* y = A_h x for a batch (Sec. 3.2, eq. A_h).  level 0 is the top level
 * (f_l = 1, so A_0 = A); level h >= 1 exists after mlcr_op_set_level().
 *   dev_x, dev_y: [nrhs][(lmax_h+1)^2] float64 packed vectors (x != y).
 * 1 <= nrhs <= max_nrhs. */
int apply_A(mlcr_op *op, int level, int nrhs, const double *dev_x, double *dev_y,
            int prec, void *stream);

/* Top-level applies of a mixed batch of independent problems (each with its
 * own operator, grid and band limit; Sec. 2.3 per problem): y_p = A_p x_p,
 * p < nprob.  host_nrhs[nprob]: RHS per problem (NULL: 1 each);
 * host_x / host_y[nprob]: device pointers laid out as for apply_A.  The
 * problems run concurrently on library-owned streams (problems on the same
 * grid in call order on one of them), forked from and joined back into
 * `stream`, so the call is ordered on `stream` like apply_A.  Results equal
 * the single applies.  EINVAL on a NULL entry or nrhs out of range. */
int apply_A_grouped(int nprob, mlcr_op *const *ops, const int *host_nrhs,
                    const double *const *host_x, double *const *host_y, int prec, void *stream);

/* Define level h >= 1 of the operator: band limit lmax_h and the
 * cumulative low-pass filter f^h_l (host_fl[lmax_h+1], f^h_l = 0 allowed),
 * so that A_h = D_h + B_h Y^T N^-1 Y B_h with D_h = diag(f^2 / C_l) and
 * B_h = diag(f b_l p_l) (Sec. 3.2, eq. A_h).  1 <= h < 16. */
int mlcr_op_set_level(mlcr_op *op, int h, int lmax_h, const double *host_fl);

/* Replace the operator's prior spectrum (every defined level follows, with
 * its own filter): host_cl[lmax+1] must be finite and > 0 exactly where the
 * current C_l is (the set of unknowns stays the same).  Solvers built on op
 * then solve the new system: their residuals, stopping norms and
 * certificates use the new C_l, while their smoothers, top diagonal and
 * dense bottom factor keep the values of the C_l they were built with and
 * act as an approximate cycle (as when a C_l sampler reuses the hierarchy
 * across nearby spectra).  Synchronous. */
int mlcr_op_set_prior(mlcr_op *op, const double *host_cl);

/* Gradient of a quadratic loss with respect to binned prior amplitudes
 * (the differentiation form: C_l = q_beta C_fid_l for l in band beta, b
 * held fixed).  With lam = A^-1 dL/dx and dA/dq_beta = -S^-1 / q_beta on the
 * band,
 *     host_out[beta] = sum_r sum_{l in beta, m} lam_lm x_lm / (q_beta C_l)
 * over the operator's active modes, C_l the operator's current spectrum.
 *   dev_lam, dev_x: [nrhs][(lmax+1)^2]; host_band[lmax+1]: band of each l
 *   (-1: none, else 0..nbands-1); host_q[nbands] (NULL: all 1).
 * Float64 throughout; synchronizes on `stream`. */
int mlcr_prior_band_grad(mlcr_op *op, int nrhs, const double *dev_lam, const double *dev_x,
                         const int *host_band, int nbands, const double *host_q,
                         double *host_out, void *stream);

/* Level h like mlcr_op_set_level, with Y^T N^-1 Y evaluated on a
 * Gauss-Legendre grid (Sec. 3.4, eqs. Ni-rewrite and Xi): xi = Y_obs^T N^-1
 * truncated at 2 lmax_h is synthesized on 2 lmax_h + 1 Gauss-Legendre rings
 * of nphi = the smallest power of two >= 4 lmax_h + 1 pixels and weighted
 * by the quadrature, which reproduces every coupling of Y_obs^T N^-1 Y_obs
 * between modes l, l' <= lmax_h exactly (up to rounding) at a cost set by
 * lmax_h rather than by the observation grid.  Needs 2 lmax_h <= the
 * geometry's lmax.  The operator owns the grid; mlcr_op_set_level on the
 * same h returns the level to the observation grid. */
int mlcr_op_set_level_gl(mlcr_op *op, int h, int lmax_h, const double *host_fl);
/* Band limit of level h (0 = top), or a negative error code. */
int mlcr_op_level_lmax(const mlcr_op *op, int h);

/* ------------------------------------------------------------------------
 * Multi-level solver (Sec. 3.2, Fig. code:mg; Sec. 4.1 for the cycle shape).
 *
 * Levels: the top spherical-harmonic level (lmax of the operator) with a
 * high-pass filtered diagonal smoother diag(A)^-1; pixel levels h = 1..H,
 * each a band-limited level operator A_h (Sec. 3.2, eq. A_h) with a sibling
 * HEALPix grid of resolution N_side/2, N_side/4, ... and an error smoother
 * on k x k pixel tiles (k = 8, Sec. 3.5); and a dense bottom level solved
 * exactly for l <= 40.  Default ladder (Sec. 3.2-3.4): pixel level 1 keeps
 * lmax; levels with N_side^h >= 512 are limited to 4 N_side^h and use the q_l
 * filter of eq. fourth-power-beam (q = 0.1 at 2570/3000 of the band limit on
 * the first level, 1536/2048 on the second); levels with N_side^h <= 256 use
 * Gaussians of FWHM two pixels and 6 N_side^h, down to N_side^h = 32.
 * A multi-level ladder needs C_l > 0 for every l (the paper's wide prior
 * C_0 = C_1 = C_2, Sec. 4.1; EINVAL otherwise); an operator small enough for
 * the dense bottom alone also accepts C_l = 0 (modes removed).  The pixel
 * smoothers are one symmetric multicolour block Gauss-Seidel sweep over the
 * k x k tiles and their neighbour couplings (Sec. 3.5's block pattern).
 * Recursion counts: the top and the finest pixel level run once down and
 * once up, the others
 * twice (partial W-cycle, Sec. 4.1), the last pixel level once into the
 * dense bottom.
 * ---------------------------------------------------------------------- */
typedef struct {
    int cycles;         /* outer cycles performed for this RHS until it converged     */
    int converged;      /* 1 if rho <= rtol                                            */
    double rho0;        /* sqrt(r^T S^-1 r / b^T S^-1 b) for the start vector          */
    double rho;         /* the same ratio at return                                    */
    double s_half_res;  /* ||S^{1/2} (b - A x)||_2; times sigma_prior = sqrt(sum_l      */
                        /* (2l+1) C_l / 4 pi) it bounds the max pixel error of x       */
} mlcr_solve_info;

/* The level ladder of a solver (Sec. 3.2 level structure, Sec. 3.3 filters,
 * Sec. 3.4 band limits; Table cycle-cost for a worked example).
 *   nlevels      pixel levels H, 0..8.  0: no pixel level; the dense solve
 *                at lmax_dense = the operator's lmax (<= 64) is the solver.
 *   nside[h]     N_side^h of pixel level h (finest first), a multiple of 8,
 *                8 <= N_side^h <= 2048 (tiles are 8 x 8 nested pixels).
 *   lmax[h]      band limit of level h: 1 <= lmax[0] <= the operator's lmax,
 *                lmax[h] <= lmax[h-1].
 *   nrec[h]      recursion count n_rec^h of level h into the next coarser
 *                level (1 = V, 2 = W; 1..3).  nrec_top: the same for the top
 *                level into pixel level 0 (1..3).
 *   lmax_dense   band limit of the dense bottom level, 0 <= lmax_dense <=
 *                lmax[H-1] and <= 64; the bottom solves A restricted to
 *                l <= lmax_dense with the last pixel level's filter.
 *   filter[h]    host [lmax[h]+1]: cumulative low-pass filter f~^h_l of
 *                level h (eq. A_h; finite, and > 0 for l <= the next coarser
 *                band limit, since restriction divides by it, eq. f_l).
 *   highpass     host [lmax+1] high-pass h_l applied to the top level's
 *                diagonal correction, or NULL for 1 - f~^0_l (0 above lmax[0]
 *                taken as f~ = 0).
 *   gl_levels    1: a coarse level evaluates Y^T N^-1 Y on a Gauss-Legendre
 *                grid (Sec. 3.4) when 2 lmax_h <= lmax, the grid's rings
 *                are at most 16384 pixels long, and it has fewer rings and at
 *                most twice the pixels of the observation grid; 0: always on
 *                the observation grid.
 *   smoother     the pixel levels' error smoother (Sec. 3.5), on the pattern of
 *                8 x 8 tiles and their neighbour tiles:
 *                0  the blocks of Y_h A_h Y_h^T read off the operator by
 *                   probing, one multicolour block symmetric Gauss-Seidel sweep;
 *                1  the paper's construction: blocks of D_hat_h (eq. Dhat) and
 *                   B_hat_h (eq. Bhat) from addition-theorem sums (eq.
 *                   addition-theorem), B_hat^T N^-1 B_hat by block products
 *                   without fill-in over the observation pixels, a block
 *                   incomplete Cholesky with no fill-in in the sweep-colour
 *                   order with the smallest ridge alpha (bisection, then
 *                   1.5 alpha, relative to the largest diagonal entry) that
 *                   succeeds, but at least ridge_min; applied by the two
 *                   triangular solves.  Needs N_side_obs / N_side^h a power
 *                   of two.
 *   ridge_min    (smoother 1) the smallest ridge used, relative to the largest
 *                diagonal entry (default 1e-4, the low end of the ridges the
 *                paper reports in Sec. 3.5).  The zero-fill factor can leave
 *                (L L^T)^-1 A_hat with eigenvalues above 2 when the ridge is
 *                only just large enough for the factorization to succeed, and
 *                then the smoothing step amplifies those error components;
 *                0 gives the paper's rule alone.
 *   ridge_max    (smoother 1) the largest ridge alpha the search may use
 *                (>= ridge_min); MLCR_ENOTPD if the factorization fails even
 *                with it.
 *   keep_blocks  (smoother 1) 1: keep the assembled blocks for
 *                mlcr_solver_level_blocks (memory: as large as the factor).
 * The descriptor is read during mlcr_solver_create only. */
typedef struct {
    int nlevels;
    int nside[8];
    int lmax[8];
    int nrec[8];
    int nrec_top;
    int lmax_dense;
    const double *filter[8];
    const double *highpass;
    int gl_levels;
    int smoother;
    double ridge_min;
    double ridge_max;
    int keep_blocks;
} mlcr_ladder_desc;

/* The ladder mlcr_solver_create uses when given NULL, for an observation
 * grid nside and band limit lmax: levels N_side/2, N_side/4, ... down to 32;
 * band limits lmax on the first, 4 N_side^h on levels N_side^h >= 512 and
 * 6 N_side^h below (Sec. 3.4), capped by the previous level; the q_l filter
 * of eq. fourth-power-beam with q = 0.1 at 2570/3000 of the band limit on the
 * first level and 1536/2048 on the second when N_side^h >= 512, else a
 * Gaussian of FWHM two level pixels (Sec. 3.3); recursion 1 on the top and
 * the last pixel level, 2 elsewhere (Sec. 4.1); dense bottom at l <= 40.
 * host_filters [8 (lmax+1)] receives the filters; out->filter[h] points
 * into it.  Host only. */
int mlcr_ladder_default(int nside, int lmax, mlcr_ladder_desc *out, double *host_filters);
/* Validate a ladder for an observation grid nside and an operator band
 * limit lmax with the rules above (0 or MLCR_EINVAL with the reason).  Host
 * only; mlcr_solver_create runs the same check. */
int mlcr_ladder_check(int nside, int lmax, const mlcr_ladder_desc *ladder);

/* Build the solver for op on a ladder (NULL = mlcr_ladder_default): level
 * geometries and operators, smoothers, the top-level diagonal and the dense
 * bottom factor (all computed on the GPU, in float64; smoothers stored in
 * float32, Sec. 3.5).  The operator and its geometry must outlive the
 * solver.  EINVAL for a ladder that fails mlcr_ladder_check, or C_l = 0 for
 * some l with pixel levels; ENOTPD if the bottom matrix or a tile cannot be
 * factored even with a ridge. */
int mlcr_solver_create(mlcr_op *op, const mlcr_ladder_desc *ladder, int max_nrhs,
                       mlcr_solver **out);
void mlcr_solver_destroy(mlcr_solver *s);
/* Pixel level count, bottom band limit, bottom unknowns and the largest tile
 * ridge alpha used (relative to the largest diagonal element of the block). */
int mlcr_solver_info(const mlcr_solver *s, int *nlevels, int *lmax_bottom, int *n_bottom,
                     float *max_ridge);

/* Per-level account of the cycles (Sec. 4.1, Table cycle-cost): with
 * profiling on, wcycle_solve and pcg_solve bracket every step of every cycle
 * with HIP events on their stream (graph mode is then not used) and add the
 * times per level and kind of work.  Levels: 0 = top, 1..H pixel levels,
 * H + 1 = dense bottom.  Kinds: 0 = applications of A_h (the residuals),
 * 1 = level transforms Y_h and Y_h^T of the pixel smoother, 2 = the error
 * smoother itself (top diagonal, pixel-domain M_h, or the dense solve),
 * 3 = restriction, interpolation and vector updates.
 * mlcr_solver_set_profile(on) also clears the totals.
 * mlcr_solver_profile fills host_ms[4 L] and host_calls[4 L] (either may be
 * NULL) for L = min(nlevels_max, H + 2) levels and returns H + 2. */
int mlcr_solver_set_profile(mlcr_solver *s, int on);
int mlcr_solver_profile(const mlcr_solver *s, int nlevels_max, double *host_ms,
                        long long *host_calls);

/* The smoother blocks of pixel level `level` (1..H) of a solver built with
 * the incomplete-Cholesky smoother: ntiles, nslots (neighbour pairs, the CSR
 * slots of mlcr_tile_graph's ascending neighbour lists), and float32 64 x 64
 * column-major blocks (entry (i, j) at j 64 + i, i and j the nested pixel
 * index within the tile):
 *   which 0: the assembled approximant, dev_diag[ntiles] = A_tt, dev_off[slot
 *            t -> u] = A_tu (needs keep_blocks);
 *   which 1: the factor, dev_diag[t] = L_tt^-1, dev_off[t -> u] = L_tu when u
 *            comes earlier in the sweep colours, L_ut^T when later.
 * Any output may be NULL.  Synchronous. */
int mlcr_solver_level_blocks(const mlcr_solver *s, int level, int which, int *ntiles,
                             long long *nslots, float *dev_diag, float *dev_off);

/* The dense bottom level (Sec. 3.2): the number n of its active modes, the
 * assembled matrix A_B (dev_A: [n][n] float64, row-major, before factoring;
 * entries from the ring Fourier sums of eq. Ni-dense on the level's grid,
 * the Gauss-Legendre grid of Sec. 3.4 when the level uses one) and the
 * packed positions of the modes in a vector of band limit lmax_bottom
 * (host_idx[n]).  Any output may be NULL.  Synchronous. */
int mlcr_solver_bottom(const mlcr_solver *s, int *n, double *dev_A, int *host_idx);

/* Copy of the top-level smoother's diagonal, 1 / diag(A) on active modes and
 * 0 elsewhere (dev_out: [(lmax+1)^2]); diag(Y^T N^-1 Y) comes from the ring
 * sums of eq. Ni-dense at frequencies 0 and 2m.  EINVAL for a dense-only solver. */
int mlcr_solver_top_dinv(const mlcr_solver *s, double *dev_out, void *stream);

/* CR-Solve (Fig. code:mg) in correction form: r = b - A x in float64, one
 * CR-Cycle from zero on r, x += correction, repeat until
 *     rho = sqrt(r^T S^-1 r / b^T S^-1 b) <= rtol        (Sec. 3.2)
 * for every RHS or max_cycles cycles are done.  prec selects the arithmetic
 * of the cycle's transforms; the residual and the update stay float64, so a
 * float32 cycle is iterative refinement.
 *   dev_b, dev_x: [nrhs][(lmax+1)^2] packed; dev_x holds the start vector
 *   on entry (zeros allowed) and the solution on return.  Excluded modes of
 *   x are set to 0.  When the start vector is zero for every RHS the start
 *   residual is b itself and no operator application is made for it.
 *   host_info: [nrhs] or NULL.
 * Returns MLCR_ENOCONV (x and info still valid) if rtol is not reached. */
int wcycle_solve(mlcr_solver *s, int nrhs, const double *dev_b, double *dev_x, double rtol,
                 int max_cycles, int prec, mlcr_solve_info *host_info, void *stream);

/* Graph mode for wcycle_solve / wcycle_solve_grouped (default off): each
 * solve runs its first cycle with direct launches, captures its second cycle
 * (every kernel and device copy of the CR-Cycle plus the float64 residual)
 * into a HIP graph and replays it for the cycles after; results are
 * identical to direct launches.  The solve runs on a library-owned stream
 * forked from and joined back into the caller's stream; a capture that fails
 * falls back to direct launches.  The graph lives for one solve call. */
int mlcr_solver_set_graph(mlcr_solver *s, int on);
/* Cycles launched from a graph so far, and graph captures that fell back to
 * direct launches, over the solver's lifetime (NULL outputs are skipped). */
int mlcr_solver_graph_stats(const mlcr_solver *s, long long *replays, long long *fallbacks);

/* CR-Solve by flexible preconditioned conjugate gradients in float64 with
 * one CR-Cycle from zero as the preconditioner, the alternative named in the
 * caption of Fig. code:mg: alpha = <r, z> / <p, A p>, x += alpha p,
 * r -= alpha A p, z = CR-Cycle(r) in `prec`, beta = <r, z - z_old> /
 * <r_old, z_old>, p = z + beta p, per RHS, until rho <= rtol (as for
 * wcycle_solve) or max_iter iterations (one cycle and one float64 apply
 * each).  Arguments, layouts, info (cycles = iterations) and errors as for
 * wcycle_solve. */
int pcg_solve(mlcr_solver *s, int nrhs, const double *dev_b, double *dev_x, double rtol,
              int max_iter, int prec, mlcr_solve_info *host_info, void *stream);

/* Right-hand side of the CR system (Sec. 2.3, eq. cr-system and the
 * fluctuation terms that turn its solution into a posterior sample):
 *     b = B Y^T (N^-1 d + N^-1/2 w2) + S^-1/2 w1
 * on the active modes of op (0 on excluded ones).
 *   dev_d:  [nrhs][12 nside^2] data maps (RING);
 *   dev_w1: [nrhs][(lmax+1)^2] white noise, or NULL;
 *   dev_w2: [nrhs][12 nside^2] white noise, or NULL;
 *   dev_b:  [nrhs][(lmax+1)^2] output.
 * With dev_w1 = dev_w2 = NULL the solution of A x = b is the Wiener-filtered
 * (maximum-likelihood) map.  float64 throughout; 1 <= nrhs <= max_nrhs. */
int mlcr_cr_rhs(mlcr_op *op, int nrhs, const double *dev_d, const double *dev_w1,
                const double *dev_w2, double *dev_b, void *stream);

/* wcycle_solve for a mixed batch of independent problems (one solver each,
 * every solver at most once): the cycles of all unfinished problems are
 * issued on library-owned streams (forked from and joined back into
 * `stream`, problems on the same grid sharing one) before any residual is
 * read back, so small problems overlap on the GPU.  host_nrhs[nprob] (NULL:
 * 1 each); host_b / host_x[nprob]: device pointers as for wcycle_solve;
 * host_info: sum of nrhs entries in problem order, or NULL.  Each problem
 * stops at its own convergence; results equal the single solves.
 * MLCR_ENOCONV if any problem misses rtol (x and info still valid). */
int wcycle_solve_grouped(int nprob, mlcr_solver *const *s, const int *host_nrhs,
                         const double *const *host_b, double *const *host_x, double rtol,
                         int max_cycles, int prec, mlcr_solve_info *host_info, void *stream);

/* ---- host-only helpers (no GPU needed) ---- */
/* HEALPix NESTED to RING pixel index (Gorski et al. 2005); the tiles of the
 * pixel-level smoothers are nested blocks of k^2 pixels. */
int mlcr_nest2ring(int nside, long long n, const long long *host_nest, long long *host_ring);
/* Tile graph of the pixel-level smoothers (Sec. 3.5): tiles are the 8 x 8
 * nested blocks, tile t = nested pixels [64 t, 64 t + 64), 12 (nside/8)^2 of
 * them (nside % 8 == 0).  Distances are between pixel centres in pixel widths
 * sqrt(4 pi / N_pix).
 *   host_nb [ntiles][max_nb]: the tiles nearer than 4 pixel widths (the
 *     smoother keeps couplings inside a tile and with these), ascending,
 *     padded with -1; EINVAL if a tile has more than max_nb.
 *   host_sweep_color [ntiles]: neighbours have different colours (the block
 *     Gauss-Seidel sweep runs one colour at a time).
 *   host_probe_color [ntiles]: for tiles u != u' of one colour, no tile of
 *     {u} + neighbours(u) comes within 6 pixel widths of u' (the blocks are
 *     probed one colour at a time).
 *   n_sweep, n_probe: colour counts. */
int mlcr_tile_graph(int nside, int max_nb, int *host_nb, int *host_sweep_color,
                    int *host_probe_color, int *n_sweep, int *n_probe);
/* The default ladder for an observation grid nside and band limit lmax:
 * level count, and per pixel level N_side^h, lmax^h and recursion count
 * (arrays of 8), the top recursion count and the bottom band limit. */
int mlcr_ladder_plan(int nside, int lmax, int *nlevels, int *nsides, int *lmaxs, int *nrec,
                     int *nrec_top, int *lmax_bottom);
/* Operation counts of ncycles CR-Solve cycles with the given recursion
 * counts, walking the same recursion as wcycle_solve.  counts[4 * level +
 * {0,1,2,3}] = visits, applications of A_h, level-transfer SHTs (Y_h) and
 * smoother (or dense-solve) applications; level 0 = top, 1..nlevels pixel
 * levels, nlevels + 1 = bottom.  The top count includes the float64
 * residual of each cycle.  counts must hold 4 (nlevels + 2) entries. */
int mlcr_cycle_counts(int nlevels, const int *nrec, int nrec_top, int ncycles, long long *counts);

#ifdef __cplusplus
}
#endif

#endif /* MLCR_H */
