/*
 * psfm.h -- C interface of the MI355X (gfx950) PSF-matching library.
 *
 * The library computes the data-parallel hot path of Alard-Lupton-style PSF
 * matching as formulated by Price & Magnier, "Pan-STARRS PSF-Matching for
 * Subtraction and Stacking":
 *   1. convolve reference-image stamps with every kernel basis function and
 *      accumulate the variance-weighted normal equations of each stamp
 *      (psfm_fit_stamps; Section 2, Eqs. 3-6),
 *   2. assemble the equations with the spatial polynomial terms evaluated at
 *      the stamp centres, solve them, reject discrepant stamps and re-solve
 *      (psfm_solve; Section 2 and Sections 3.3, 3.5, 3.6),
 *   3. apply the spatially varying kernel to the whole image in constant-
 *      kernel patches, with BAD/POOR mask propagation (psfm_convolve_image;
 *      Sections 3.4, 3.5, Section 4.2 Eq. 12),
 *   4. propagate the variance map and the covariance pseudo-matrix
 *      (psfm_propagate_variance; Section 4.2 Eq. 13, Sections 4.2-4.3),
 *   5. form the difference image with its variance, mask and pseudo-matrix
 *      (psfm_subtract; Section 4.3).
 *
 * Conventions shared by every call
 *   - Images are row-major float32: pixel (x, y) of a W x H image is element
 *     y * pitch + x (pitch >= W, in elements).  Masks are uint8 planes with
 *     the same pitch (in bytes); a non-zero input mask value means "masked".
 *   - Every pixel, stamp, matrix and coefficient pointer is a DEVICE pointer
 *     owned by the caller; the library never allocates, frees or retains them.
 *     psfm_fit_stats pointers are device pointers as well.
 *   - Every call is asynchronous and ordered on `stream` (a hipStream_t; NULL
 *     is the default stream).  Host-detectable argument errors are returned
 *     before anything is launched.  Numerical failures found on the device
 *     (too few stamps, a matrix that is not positive definite) are written to
 *     psfm_fit_stats.info; the call itself still returns PSFM_OK (unless the
 *     config's flags hold PSFM_SYNC, see there).
 *   - Calls allocate nothing: scratch memory is the caller's workspace `ws`
 *     (device memory of at least psfm_workspace_bytes() bytes, 256-byte
 *     aligned).  Concurrent calls need separate workspaces.  A context is
 *     read-only after psfm_create and may be shared by concurrent calls.
 *   - Masked pixels, and pixels outside the image, never contribute a value
 *     (not even a NaN) to a convolution.
 *
 * Unknowns.  With nb kernel basis terms and ns = (S+1)(S+2)/2 spatial terms
 * the coefficient vector has N = nb * ns + 1 float64 entries: kernel term i
 * with spatial term s at index i * ns + s, the constant background last.
 * Term 0 carries the flux (unit sum); every other term sums to zero, so the
 * kernel sum at a point is the local coefficient of term 0 there.
 */
#ifndef PSFM_H
#define PSFM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define PSFM_MAX_GAUSS 8

/* Return codes. */
typedef enum {
    PSFM_OK = 0,
    PSFM_ERR_INVALID_ARG = -1,   /* NULL pointer, negative size, bad config value */
    PSFM_ERR_SHAPE = -2,         /* image too small for the kernel, pitch < W, ... */
    PSFM_ERR_TOO_FEW_STAMPS = -3,/* (device, in stats.info) fewer than min_stamps usable */
    PSFM_ERR_NOT_PD = -4,        /* (device) normal matrix not positive definite */
    PSFM_ERR_HIP = -5,           /* a HIP runtime call failed */
    PSFM_ERR_WORKSPACE = -6,     /* workspace missing or smaller than required */
    PSFM_ERR_UNSUPPORTED = -7,   /* configuration outside what the kernels support */
    PSFM_ERR_NORM_SINGULAR = -8  /* (device) stamp totals do not determine b0 and d0 */
} psfm_status;

/* Stamp flag bits (stamp_flags). */
#define PSFM_STAMP_INVALID   1   /* footprint leaves the image or touches a masked pixel */
#define PSFM_STAMP_REJECTED  2   /* removed by the rejection iterations of psfm_solve */
#define PSFM_STAMP_NONFINITE 4   /* non-finite pixel, or variance not finite and > 0 */
#define PSFM_STAMP_EXCLUDED  8   /* excluded by the caller before psfm_solve */
#define PSFM_STAMP_PRIOR    16   /* excluded before the first solution by the learned prior */
#define PSFM_STAMP_RESERVE  32   /* held back to replace a rejected stamp (psfm_solve_norm) */

/* Output mask bits. */
#define PSFM_MASK_BAD       1    /* masked in the input (difference image: image 2) */
#define PSFM_MASK_CONV_BAD  2    /* masked input within the BAD radius of the kernel */
#define PSFM_MASK_CONV_POOR 4    /* masked input within the kernel footprint only */

/* Arithmetic of the stamp fit (the normal equations of Section 2, Eq. 6).
   FP32: FP32 basis convolution, the Gram of the FP32 weighted block on FP64
   MFMA (exact products, FP64 sums).
   BF16 / FP16: the same FP32 design rounded to 16 bits for a 16-bit MFMA
   Gram (FP32 accumulation, per-row FP64 sums); psfm_solve then refines each
   FP64 Cholesky solution `refine` times against residuals recomputed in
   FP64 from the FP32 design (iterative refinement), and takes every chi2_s
   from those pixel residuals. */
#define PSFM_PREC_FP32 0
#define PSFM_PREC_BF16 1
#define PSFM_PREC_FP16 2

/*
 * Method parameters.
 *   Kernel basis (Section 2, Eq. 7; Section 3.1): n_gauss Gaussians of width
 *   sigma[j] (pixels) times the monomials u^p v^q with p + q <= degree[j];
 *   terms are ordered by Gaussian, then total degree d, then p from d down
 *   to 0.  Term 0 (the narrowest Gaussian, unit sum) carries the flux; the
 *   other terms are made zero-sum (Section 2): even terms as
 *   raw/sum(raw) - k_0, odd terms as raw/sum(|raw|).
 *   The kernel is (2 half_width + 1)^2 pixels.
 *   Spatial variation (Section 2): ordinary polynomials x^l y^m, l + m <=
 *   spatial_order, in coordinates scaled to [-1, 1] over the image, ordered by
 *   degree then l descending; evaluated at stamp centres for the fit and at
 *   patch centres for the application.
 *   Stamps are (2 stamp_half + 1)^2 pixels; the weights are 1 / V2, or
 *   1 / (V1 + V2) (weight_mode).
 *   Rejection (Sections 3.3, 3.6): after each solution the used stamps with
 *   chi2_s / npix_s > mean + clip_sigma * std (population, over used stamps)
 *   are rejected and the equations re-solved, at most max_iter solutions; a
 *   clip that would leave fewer than min_stamps stamps is not applied.
 *   Application (Section 3.5): constant kernels on patch x patch squares
 *   anchored at (0, 0), realised at each (clipped) patch centre.
 *   BAD/POOR (Section 3.4): the BAD box radius is the smallest r with
 *   sum_{max(|u|,|v|) > r} k^2 < bad_frac * sum k^2.
 */
typedef struct psfm_config {
    int n_gauss;
    double sigma[PSFM_MAX_GAUSS];
    int degree[PSFM_MAX_GAUSS];
    int half_width;        /* h: kernel taps u, v in [-h, h]; 1 <= h <= 16 */
    int spatial_order;     /* S: 0..6 */
    int stamp_half;        /* r: stamp is (2r+1)^2; 1 <= r <= 32 */
    int patch;             /* P: side of the constant-kernel patches, >= 1 */
    double clip_sigma;     /* rejection threshold (default 3) */
    int max_iter;          /* maximum number of solutions (default 3) */
    int min_stamps;        /* minimum usable stamps (default 3) */
    double bad_frac;       /* BAD/POOR fraction (default 0.2) */
    int precision;         /* PSFM_PREC_* */
    int refine;            /* refinement steps of the 16-bit modes (0..4, default 1) */
    int weight_mode;       /* PSFM_WEIGHT_*: fit weights 1 / V2 (default) or 1 / (V1 + V2) */
    int ortho_basis;       /* 1: psfm_solve works in the orthonormalised basis (FP32 only) */
    int flags;             /* PSFM_SYNC or 0 */
    int fit_band_rows;     /* stamp rows per fit workgroup: 0 = chosen from r, or 7, 9 or 11 */
} psfm_config;

/* weight_mode.  The fit's pixel weights are the inverse variance of the
   target image alone (PSFM_WEIGHT_V2, Section 2's sigma^2 = V2), or of the
   two images' variances added (PSFM_WEIGHT_V1V2: the convolved image's noise
   counted with unit kernel weight); the second needs V1 in the fit calls. */
#define PSFM_WEIGHT_V2   0
#define PSFM_WEIGHT_V1V2 1

/* ortho_basis.  The normal equations are ill-conditioned because the basis
   terms overlap (Section 3.1's Gaussians share their centre).  With
   ortho_basis = 1, psfm_solve and psfm_solve_prior map each stamp's sums to
   the basis whose taps are orthonormal (k' = k R^-1, R the upper Cholesky
   factor of the taps' Gram matrix; background unchanged), solve there, and
   map the coefficients back (a = R^-1 c per spatial term) before the
   residuals, the clip and the statistics, which are basis-independent.  FP32
   precision only; the other solves and the batch return PSFM_ERR_UNSUPPORTED. */

/* flags.  PSFM_SYNC: psfm_solve, psfm_solve_prior, psfm_solve_norm and
   psfm_solve_dual wait for the stream after their launches and return the
   device-detected status (PSFM_ERR_TOO_FEW_STAMPS, PSFM_ERR_NOT_PD,
   PSFM_ERR_NORM_SINGULAR) besides writing it to stats->info.  Such calls
   synchronise the stream and cannot be captured into a graph. */
#define PSFM_SYNC 1

/* Quality record of a fit (device memory, written by the library). */
typedef struct psfm_fit_stats {
    double chi2;               /* sum of chi2_s over used stamps */
    double dof;                /* sum of npix_s over used stamps - N */
    double chi2_dof;           /* chi2 / dof */
    double kernel_sum_centre;  /* kernel sum realised at the image centre */
    double cov_discarded_frac; /* share of sum|C| cut off by the pseudo-matrix crop */
    int n_used;                /* stamps in the final solution */
    int n_rejected;            /* stamps rejected by this solve */
    int n_iter;                /* solutions computed */
    int info;                  /* 0 ok; k > 0: pivot k not positive; -3: too few stamps */
    double chi2_dof_prior;     /* psfm_solve_prior: chi2/dof of the kept stamps at the warm start */
    int n_prior;               /* psfm_solve_prior: stamps left excluded by the prior in the answer */
    int n_restored;            /* psfm_solve_prior: excluded stamps the solution found within the clip */
    int n_trusted;             /* psfm_solve_prior: predictions kept by the 1.05x rule */
    int prior_fallback;        /* psfm_solve_prior: 1 if the full method was rerun (prior void) */
    int n_replaced;            /* psfm_solve_norm: reserve stamps brought in for rejected ones */
} psfm_fit_stats;

typedef struct psfm_context psfm_context;

/* Fills *cfg with the defaults: 3 Gaussians (0.7, 1.5, 3.0 px) x degrees
   (6, 4, 2) = 49 terms, h = 10, S = 0, r = 20, P = 64, clip 3, 3 solutions,
   3 stamps, bad_frac 0.2, FP32, 1 refinement step (16-bit modes only),
   weights 1 / V2, the basis as defined, no flags, fit band rows from r. */
void psfm_config_default(psfm_config* cfg);

/* Validates cfg, builds the basis tables (FP64 on the host) and uploads them
   to the current HIP device.  *out receives a context the caller destroys
   with psfm_destroy.  This is the only call that allocates device memory. */
int psfm_create(const psfm_config* cfg, psfm_context** out);
int psfm_destroy(psfm_context* ctx);

int psfm_n_basis(const psfm_context* ctx);      /* nb */
int psfm_n_spatial(const psfm_context* ctx);    /* ns */
int psfm_n_unknowns(const psfm_context* ctx);   /* N = nb * ns + 1 */
int psfm_stamp_dim(const psfm_context* ctx);    /* L = nb + 1: per-stamp matrix side */

/* Bytes of workspace that every call below needs for a W x H image and
   n_stamps stamps (the maximum over the calls); 0 on invalid arguments. */
size_t psfm_workspace_bytes(const psfm_context* ctx, int W, int H, int n_stamps);

/* Floats of the stamp design that psfm_fit_stamps writes and psfm_solve
   reads in the 16-bit modes: n_stamps * (nb + 2) * (2r + 1)^2 (0 in FP32). */
size_t psfm_stamp_design_floats(const psfm_context* ctx, int n_stamps);

/*
 * Per-stamp normal equations (Section 2, Eqs. 3-6 with c = 0, p = 0).
 * For stamp s centred on (x, y) = stamp_xy[2s], stamp_xy[2s+1] and every
 * pixel of its (2r+1)^2 square: A_i = k_i (x) I1 (true convolution, Eq. 12),
 * A_nb = 1 (background), w = 1 / V2, d = I2;
 *   stamp_M[s] = sum w A A^T   (L x L, row-major, symmetric),
 *   stamp_b[s] = sum w A d     (L),   stamp_e[s] = sum w d^2,
 *   stamp_npix[s] = (2r+1)^2,  stamp_flags[s] = 0,
 * or, for a stamp failing the validity test of Section 3.3 (footprint
 * [x-r-h, x+r+h]^2 outside the image or masked in M1; stamp masked in M2;
 * non-finite or non-positive data), the flag bits and zero sums.
 * Arithmetic: FP32 separable basis convolution, the Gram of the FP32
 * weighted block on FP64 MFMA, per-band partial sums added in FP64 (16-bit
 * Gram in the BF16 / FP16 modes, see PSFM_PREC_*).  Inputs: I1, M1 (convolved
 * image), I2, V2, M2 (target), all W x H with `pitch`; V1 (the convolved
 * image's variance) is read only with weight_mode PSFM_WEIGHT_V1V2 (then the
 * weight is 1 / (V1 + V2), added in FP32, and a stamp whose sum is not finite
 * and positive is NONFINITE), else it may be NULL.  Outputs are float64/int32 device arrays of n_stamps
 * entries (stamp_M n*L*L, stamp_b n*L).  stamp_design (16-bit modes only,
 * else may be NULL; psfm_stamp_design_floats floats): per stamp the FP32
 * weighted design, column-major [term 0..nb-1, sqrt(w), sqrt(w) I2][pixel].
 */
int psfm_fit_stamps(const psfm_context* ctx, const float* I1, const float* V1, const uint8_t* M1,
                    const float* I2, const float* V2, const uint8_t* M2, int W, int H, int64_t pitch,
                    const int32_t* stamp_xy, int n_stamps, double* stamp_M, double* stamp_b,
                    double* stamp_e, int32_t* stamp_npix, int32_t* stamp_flags,
                    float* stamp_design, void* ws, size_t ws_bytes, void* stream);

/*
 * Assembly, solution and rejection (Section 2; Sections 3.3, 3.5, 3.6).
 * Stamps with any stamp_flags bit set on entry are not used.  The equations
 *   M[(i,s),(j,t)] = sum_used g_s(c) g_t(c) M_s[i][j], background last,
 * are solved in FP64 (equilibrated Cholesky); each solution is followed by
 * the per-stamp residual chi2_s = e_s - 2 alpha^T b_s + alpha^T M_s alpha
 * (alpha: local coefficients at the stamp centre) and the sigma-clip.
 * Outputs: coeffs (N float64), stamp_chi2 (n float64, 0 for stamps flagged on
 * entry), stamp_flags gains PSFM_STAMP_REJECTED, *stats (device).  On a
 * device-detected failure stats->info is set (-3 or the failing pivot) and
 * coeffs hold zeros.  In the 16-bit modes stamp_design (from
 * psfm_fit_stamps) is required: each solution is refined against residuals
 * from it and chi2_s is taken from those residuals.
 */
int psfm_solve(const psfm_context* ctx, int W, int H, const int32_t* stamp_xy, int n_stamps,
               const double* stamp_M, const double* stamp_b, const double* stamp_e,
               const int32_t* stamp_npix, int32_t* stamp_flags, const float* stamp_design,
               double* coeffs, double* stamp_chi2, psfm_fit_stats* stats, void* ws,
               size_t ws_bytes, void* stream);

/*
 * The paper's normalisation and quality mode (Sections 3.2, 3.3, 3.6, 3.7).
 *
 * psfm_fit_norm: the unweighted sums of each stamp for the separate
 * normalisation (Section 3.2, sigma(x, y) = 1): with A0 = k_0 (x) I1 the
 * flux-carrying column,
 *   stamp_norm[5 s + 0..4] = npix, sum A0, sum I2, sum A0^2, sum A0 I2
 * over the stamp's (2r+1)^2 pixels (FP64).  Stamps whose flags hold any bit
 * other than PSFM_STAMP_RESERVE get zeros (reserves keep their sums for a
 * later replacement).  stamp_flags: psfm_fit_stamps' flags (plus
 * PSFM_STAMP_RESERVE set by the caller on the reserves).  Stamp footprints
 * must lie inside the image (psfm_fit_stamps flags those that do not).
 */
int psfm_fit_norm(const psfm_context* ctx, const float* I1, const float* I2, int W, int H,
                  int64_t pitch, const int32_t* stamp_xy, int n_stamps,
                  const int32_t* stamp_flags, double* stamp_norm, void* stream);

/*
 * psfm_solve in the paper's normalisation mode (Section 3.2): at every
 * solution b0 and d0 are found first, spatially constant and unweighted,
 * from the stamp totals of the stamps in use (only they add flux; the other
 * terms move flux within a stamp): the least-squares fit of
 * sum I2 = b0 sum A0 + d0 npix over the stamps.  The weighted equations of
 * the other unknowns are then solved with them held (term 0 = b0 at spatial
 * term 0 and 0 at the others, background = d0).  Rejection as psfm_solve;
 * replacement (Section 3.3): with stamp_group (n int32, nullable; group id
 * >= 0 per stamp, e.g. the subregion the stamp was chosen in), each stamp
 * rejected in a round is replaced by the lowest-index stamp of its group
 * whose flags are exactly PSFM_STAMP_RESERVE (stats->n_replaced counts
 * them).  stats->dof = sum npix - (free unknowns + 2); kernel_sum_centre =
 * b0; info PSFM_ERR_NORM_SINGULAR if the totals cannot separate b0 from d0.
 * FP32 stamp fits only.  Workspace: psfm_workspace_bytes().
 */
int psfm_solve_norm(const psfm_context* ctx, int W, int H, const int32_t* stamp_xy, int n_stamps,
                    const double* stamp_M, const double* stamp_b, const double* stamp_e,
                    const int32_t* stamp_npix, const double* stamp_norm,
                    const int32_t* stamp_group, int32_t* stamp_flags, double* coeffs,
                    double* stamp_chi2, psfm_fit_stats* stats, void* ws, size_t ws_bytes,
                    void* stream);

/* Quality record of a solution (device memory, written by psfm_quality). */
typedef struct psfm_quality {
    double dev_mean;     /* normalised mean deviation: mean of dev_s over used stamps, minus 1 */
    double dev_rms;      /* normalised r.m.s. deviation: population std of dev_s */
    double kernel_sum;   /* kernel realised at the image centre: sum, */
    double mom_x, mom_y; /* first moments (pixels), */
    double mom_xx, mom_yy; /* second central moments, */
    double deconv_max;   /* maximum deconvolution fraction */
    int n_used;          /* stamps used */
    int cut_flags;       /* PSFM_CUT_* bits raised */
} psfm_quality;

/* The bad-subtraction cuts the paper recommends (Section 3.7). */
#define PSFM_CUT_FEW_STAMPS 1    /* stamps used < 3 */
#define PSFM_CUT_MEAN_DEV   2    /* normalised mean deviation > 0.5 */
#define PSFM_CUT_RMS_DEV    4    /* normalised r.m.s. deviation > 0.3 */
#define PSFM_CUT_MOMENT1    8    /* |first moment| (x or y) > 0.5 */
#define PSFM_CUT_MOMENT2   16    /* second moment (xx or yy) < 0 */
#define PSFM_CUT_DECONV    32    /* maximum deconvolution fraction > 1.03 */

/*
 * Quality of a solution (Section 3.6).  For each stamp with stamp_flags 0,
 * the residual of the solution applied at the stamp (the kernel realised at
 * its centre convolved with I1, plus the background d0) divided by the
 * variance softened with a scaled flux:
 *   stamp_dev[s] = (1/npix) sum (I2 - m)^2 / (V2 + soft |m|),  m the model,
 * (0 for the other stamps; soft = 0 gives chi2_s / npix_s).  Over the used
 * stamps, *quality gets the normalised mean and r.m.s. deviations; for the
 * kernel realised at the image centre its sum, first moments sum u K / sum K
 * and sum v K / sum K, second central moments, and the maximum over radii
 * rho = 0 .. ceil(h sqrt 2) of the deconvolution fraction
 * sum_{u^2 + v^2 <= rho^2} K / sum K; and the PSFM_CUT_* bits.  coeffs:
 * N float64 (any mode).  stamp_dev: n float64 (device); quality: device.
 * Used stamps' footprints must lie inside the image (as psfm_fit_stamps'
 * valid stamps do); others are skipped.
 */
int psfm_quality_eval(const psfm_context* ctx, const double* coeffs, const float* I1,
                      const float* I2, const float* V2, int W, int H, int64_t pitch,
                      const int32_t* stamp_xy, int n_stamps, const int32_t* stamp_flags,
                      double soft, double* stamp_dev, psfm_quality* quality, void* stream);

/*
 * The dense solve of psfm_solve on its own (Section 2: the normal equations
 * M a = b are symmetric positive definite): symmetric equilibration
 * D = diag(M)^-1/2, FP64 Cholesky of D M D in one workgroup (32-column
 * panels in LDS, FP64 MFMA trailing updates), forward and back substitution.
 * M: n x n float64 row-major (only the lower triangle is read; not
 * modified), b, x: n float64, info (device int): 0, or the 1-based pivot
 * that was not positive (x then undefined).  n <= 496.
 */
size_t psfm_cholesky_workspace_bytes(int n);
int psfm_cholesky_solve(int n, const double* M, const double* b, double* x, int* info, void* ws,
                        size_t ws_bytes, void* stream);

/*
 * Each stamp's own least-squares kernel (no spatial terms): M_s a = b_s
 * solved in FP64 (equilibrated Cholesky) for every stamp; local (n x L
 * float64) receives a, stamp_chi2 receives e_s - 2 a^T b_s + a^T M_s a.
 * Flagged stamps and non-positive pivots give zeros and chi2 = -1.  Used to
 * make training targets for the learned prior.  Needs L <= 64.
 */
int psfm_solve_stamps(const psfm_context* ctx, int n_stamps, const double* stamp_M,
                      const double* stamp_b, const double* stamp_e, const int32_t* stamp_flags,
                      double* local, double* stamp_chi2, void* stream);

/*
 * psfm_solve with a learned prior: stamp_pred (n x L float64, kernel terms;
 * the background slot is ignored) holds per-stamp predicted local kernel
 * coefficients.  Before the first solution
 *   - each prediction is completed with its best background and its residual
 *     chi2 compared with that of the stamp's own least-squares kernel (the
 *     solved value, an L x L FP64 Cholesky per stamp): where the prediction's
 *     chi2 exceeds 1.05x the solved value, the least-squares kernel replaces
 *     it (stats->n_trusted: predictions kept);
 *   - warm start a0: the spatial polynomial of each term fitted to these
 *     per-stamp kernels;
 *   - rejection prior: a variable source shows as a per-stamp kernel sum (its
 *     own flux ratio) far from a0's kernel sum at the stamp, on a stamp that
 *     a0 does not fit; a stamp whose departure d = k_s / k_a0 - 1 lies beyond
 *     max(5 robust sigma, 20%) about the median departure (robust sigma = 1.4826 x
 *     median absolute deviation) and whose chi2_s / npix_s at a0 exceeds the
 *     method's clip threshold there gets PSFM_STAMP_PRIOR and is left out of
 *     the equations; a0 is refitted and the clip repeated (at most
 *     max_iter + 1 rounds, no solve needed);
 *   - stats->chi2_dof_prior: chi2/dof of the kept stamps at a0.
 * The solve and rejection loop of psfm_solve then runs on the kept stamps.
 * The least-squares solution is the judge: if any excluded stamp's
 * chi2_s / npix_s at the final solution lies within the method's clip
 * threshold, or the prior path failed, the exclusions are void and
 * psfm_solve's loop reruns from the complete stamp set with a fresh budget
 * (stats->prior_fallback = 1): the answer is then psfm_solve's.  Needs
 * L <= 64.  Same arguments as psfm_solve.
 */
int psfm_solve_prior(const psfm_context* ctx, int W, int H, const int32_t* stamp_xy, int n_stamps,
                     const double* stamp_M, const double* stamp_b, const double* stamp_e,
                     const int32_t* stamp_npix, int32_t* stamp_flags, const float* stamp_design,
                     const double* stamp_pred, double* coeffs, double* stamp_chi2,
                     psfm_fit_stats* stats, void* ws, size_t ws_bytes, void* stream);

/*
 * Image convolution with the spatially varying kernel (Section 4.2, Eq. 12;
 * Section 3.5) and BAD/POOR masking (Section 3.4):
 *   out(x, y) = sum_{u,v} K_p(u, v) I~(x - u, y - v),  p the patch of (x, y),
 * with I~ = I where inside the image and M == 0, else 0; out_mask(x, y) is
 * PSFM_MASK_CONV_BAD if a masked or outside input lies within the BAD box
 * radius of K_p, else PSFM_MASK_CONV_POOR if one lies within h, else 0.
 * coeffs: N float64 (device).  out, out_mask: W x H with `pitch`.
 */
int psfm_convolve_image(const psfm_context* ctx, const double* coeffs, const float* I,
                        const uint8_t* M, int W, int H, int64_t pitch, float* out,
                        uint8_t* out_mask, void* ws, size_t ws_bytes, void* stream);

/*
 * Variance and covariance propagation (Section 4.2, Eq. 13 and the
 * covariance factor; Section 4.3):
 *   var_out(x, y) = f_p * sum_{u,v} K_p(u, v)^2 V~(x - u, y - v),
 * f_p = raw_p(0) / sum K_p^2 the covariance factor of the patch kernel, with
 *   raw(delta) = sum_{u,u'} K(u) K(u') C_in(delta + u - u').
 * cov_out ((2 cov_out_half + 1)^2 float64, centre = zero offset) is the mean
 * of raw / sum K^2 over the kernels realised at the centres of a 3 x 3
 * partition of the image, divided by its centre value, cropped or
 * zero-padded.  cov_in ((2 cov_in_half + 1)^2 float64) may be NULL: the
 * uncorrelated input.  If stats is not NULL, stats->cov_discarded_frac
 * receives the share of sum|C| cut off by the crop.
 */
int psfm_propagate_variance(const psfm_context* ctx, const double* coeffs, const float* V,
                            const uint8_t* M, int W, int H, int64_t pitch, const double* cov_in,
                            int cov_in_half, float* var_out, double* cov_out, int cov_out_half,
                            psfm_fit_stats* stats, void* ws, size_t ws_bytes, void* stream);

/*
 * psfm_convolve_image and psfm_propagate_variance of the same pair in one
 * call (Section 4.2, Eqs. 12-13; Sections 3.4, 3.5, 4.3): every output tile
 * realises its patch kernel once and forms both I' (with out_mask) and V'.
 * Arguments, layouts and results are those of the two calls (I and V share
 * the mask M and the pitch); the outputs are bit-identical to theirs.  The
 * workspace is psfm_propagate_variance's.
 */
int psfm_convolve_pair(const psfm_context* ctx, const double* coeffs, const float* I,
                       const float* V, const uint8_t* M, int W, int H, int64_t pitch,
                       const double* cov_in, int cov_in_half, float* out, uint8_t* out_mask,
                       float* var_out, double* cov_out, int cov_out_half, psfm_fit_stats* stats,
                       void* ws, size_t ws_bytes, void* stream);

/*
 * Difference image (Section 4.3; sign: science minus matched reference):
 *   diff = I2 - conv - d0, diff_var = V2 + conv_var,
 *   diff_mask = (M2 != 0 ? PSFM_MASK_BAD : 0) | conv_mask,
 * with diff = diff_var = 0 where M2 != 0; d0 = coeffs[N-1] the background.
 * cov_diff ((2 cov_diff_half + 1)^2 float64) = (v2 C2 + vc Cc) / (v2 + vc),
 * v2 and vc the mean of V2 over M2 == 0 and of conv_var over conv_mask == 0;
 * cov2 NULL is the uncorrelated pseudo-matrix; inputs are zero-padded or
 * cropped to the output size.
 */
int psfm_subtract(const psfm_context* ctx, const double* coeffs, const float* I2, const float* V2,
                  const uint8_t* M2, const float* conv, const float* conv_var,
                  const uint8_t* conv_mask, int W, int H, int64_t pitch, const double* cov2,
                  int cov2_half, const double* cov_conv, int cov_conv_half, float* diff,
                  float* diff_var, uint8_t* diff_mask, double* cov_diff, int cov_diff_half,
                  void* ws, size_t ws_bytes, void* stream);

/*
 * psfm_convolve_pair and psfm_subtract of one pair in one pass (Section 4.2,
 * Eqs. 12-13; Sections 3.4, 3.5, 4.3): every output tile realises its patch
 * kernel once, forms I' and V' in registers and writes the difference image
 * (diff, diff_var, diff_mask as psfm_subtract defines them, bit-identical to
 * that call) without storing and reading back the convolved planes.
 * I1, V1 share the mask M1; all planes share W, H and pitch.  conv and
 * conv_mask (both or neither) and conv_var are optional (NULL: not written).
 * cov1 / cov1_half are psfm_propagate_variance's cov_in, cov_conv its
 * cov_out (always written: C_D needs it), cov2 / cov_diff as in
 * psfm_subtract; the variance means of C_D are summed per 64 x 64 tile
 * (equal to psfm_subtract's up to summation order).  Workspace:
 * psfm_workspace_bytes().  Errors as the two calls.
 */
int psfm_match_pair(const psfm_context* ctx, const double* coeffs, const float* I1,
                    const float* V1, const uint8_t* M1, const float* I2, const float* V2,
                    const uint8_t* M2, int W, int H, int64_t pitch, const double* cov1,
                    int cov1_half, const double* cov2, int cov2_half, float* conv,
                    uint8_t* conv_mask, float* conv_var, double* cov_conv, int cov_conv_half,
                    float* diff, float* diff_var, uint8_t* diff_mask, double* cov_diff,
                    int cov_diff_half, psfm_fit_stats* stats, void* ws, size_t ws_bytes,
                    void* stream);

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc):
 * psfm_match_pair without a workspace argument.  Its scratch (covariance
 * samples, per-tile variance sums and the patch taps) lives in a static
 * device array of
 * PSFM_STATIC_SCRATCH_BYTES on each device, held until the process ends;
 * the call allocates nothing.  Arguments, results and errors are those of
 * psfm_match_pair (bit-identical outputs, same kernels), plus
 * PSFM_ERR_WORKSPACE, returned before anything is launched, when the image
 * needs more scratch than the array holds: about 1 MB of covariance samples
 * at h = 10 (1.6 MB at h = 16) plus the FP32 taps of every patch (3.5 KB at
 * h = 10) and 32 bytes per 64 x 64 output tile, i.e. images up to about
 * 8500 x 8500 px at h = 10 with 64-px patches (smaller patches mean more
 * patches and tiles).  Every call on a device shares that device's
 * array and leaves its contents behind: calls that overlap on one device
 * (several streams or host threads) race and must be serialised by the
 * caller.
 */
#define PSFM_STATIC_SCRATCH_BYTES ((size_t)64 << 20)
int psfm_match_pair_static(const psfm_context* ctx, const double* coeffs, const float* I1,
                           const float* V1, const uint8_t* M1, const float* I2, const float* V2,
                           const uint8_t* M2, int W, int H, int64_t pitch, const double* cov1,
                           int cov1_half, const double* cov2, int cov2_half, float* conv,
                           uint8_t* conv_mask, float* conv_var, double* cov_conv,
                           int cov_conv_half, float* diff, float* diff_var, uint8_t* diff_mask,
                           double* cov_diff, int cov_diff_half, psfm_fit_stats* stats,
                           void* stream);

/*
 * Noise-model operations beyond convolution (Section 4.3).  These need no
 * context.  Pseudo-matrices are (2c + 1)^2 float64 arrays centred on zero
 * offset, NULL meaning the uncorrelated (unit centre) one.
 *
 * psfm_bin_image: binning by an integer factor B (1..64) as a convolution
 * with a constant B x B kernel followed by a change of scale.  Output pixel
 * (X, Y) of the (W / B) x (H / B) planes (partial blocks at the right and
 * bottom edges dropped; pitch_b in elements) holds the sum of the block's
 * unmasked pixels, Mb = 1 if any pixel of the block is masked, and
 *   Vb = f * (sum of the block's unmasked variances),  f = raw(0) / B^2,
 *   raw(D) = sum_{u, u' in block} C_in(D + u - u'),
 * the covariance factor of the block sum moved into the variance map; the
 * pseudo-matrix of the binned image is raw sampled at multiples of B,
 * cov_out(D) = raw(B D) / raw(0), cropped or zero-padded to cov_out_half
 * (*discarded, device, nullable: share of its sum |.| cut off).
 */
int psfm_bin_image(const float* I, const float* V, const uint8_t* M, int W, int H, int64_t pitch,
                   int B, const double* cov_in, int cov_in_half, float* Ib, float* Vb, uint8_t* Mb,
                   int64_t pitch_b, double* cov_out, int cov_out_half, double* discarded,
                   void* stream);

/*
 * psfm_resample_cov: a pseudo-matrix carried to a new pixel scale (an output
 * pixel spans `scale` input pixels, scale > 0): output offset D takes the
 * bilinear interpolation of cov_in at scale * D (zero beyond its extent);
 * the centre stays cov_in's (1), and the off-centre entries are scaled
 * together so that their sum -- the total covariance excluding the variance
 * -- equals cov_in's.  Both device arrays, half-sizes up to 256.
 */
int psfm_resample_cov(const double* cov_in, int cov_in_half, double scale, double* cov_out,
                      int cov_out_half, void* stream);

/*
 * psfm_add_images: S = alpha Ia + beta Ib (adding or subtracting images),
 * V_S = alpha^2 Va + beta^2 Vb, MS = Ma | Mb (S = V_S = 0 where it is
 * non-zero), and cov_s = (wa cov_a + wb cov_b) / (wa + wb) with the weights
 * wa = alpha^2 mean(Va), wb = beta^2 mean(Vb), each mean over that input's
 * unmasked pixels; inputs zero-padded or cropped to cov_s_half.  All planes
 * W x H with `pitch`.  ws: device scratch of PSFM_ADD_WORKSPACE_BYTES.
 */
#define PSFM_ADD_WORKSPACE_BYTES 32768
int psfm_add_images(double alpha, const float* Ia, const float* Va, const uint8_t* Ma,
                    const double* cov_a, int cov_a_half, double beta, const float* Ib,
                    const float* Vb, const uint8_t* Mb, const double* cov_b, int cov_b_half, int W,
                    int H, int64_t pitch, float* S, float* VS, uint8_t* MS, double* cov_s,
                    int cov_s_half, void* ws, size_t ws_bytes, void* stream);

/*
 * Matching both images to a common PSF (Section 2, Eqs. 1-4, with the
 * penalty of Eq. 9): I2 is modelled as K1 (x) I1 plus sum c_i g_i k_i (x) I2
 * plus the background, so that K1 (x) I1 + d0 = K2 (x) I2 with
 * K2 = delta - sum_{i>=1} c_i g_i k_i (unit sum: every k_i with i >= 1 sums
 * to zero); neither image has to be deconvolved, e.g. when their PSFs are
 * elongated along different axes.  The context's basis, h, r, patch, spatial
 * order and rejection settings apply; its precision does not (FP32 design,
 * FP64 Gram).
 *
 * Unknowns (psfm_dual_unknowns, N2 = (2 nb - 1) ns + 1, float64): the b-terms
 * b[i * ns + s] (i < nb, the single form's kernel unknowns), the c-terms of
 * basis i = 1..nb-1 at offset nb ns, c[(i - 1) * ns + s], and d0 last.  Stamp
 * matrices are L2 = 2 nb wide: columns k_i (x) I1 (i < nb), k_i (x) I2
 * (1 <= i < nb), then the background.  Supported while 2 nb + 1 <= 128 and
 * N2 <= 496 (the 49-term basis: spatial order 0 or 1).
 *
 * psfm_dual_workspace_bytes: device scratch for either call below (0 for
 * invalid arguments).
 */
size_t psfm_dual_workspace_bytes(const psfm_context* ctx, int width, int height, int n_stamps);
int psfm_dual_unknowns(const psfm_context* ctx);

/*
 * psfm_fit_dual: per-stamp sums of the two-kernel form, weights 1 / V2 (or
 * 1 / (V1 + V2) with weight_mode PSFM_WEIGHT_V1V2, V1 then required):
 * stamp_M (n x L2 x L2), stamp_b (n x L2), stamp_e, stamp_npix, stamp_flags,
 * as psfm_fit_stamps.  Validity as there, plus I2 and M2 over the whole
 * convolution footprint (I2 is convolved): a masked pixel there makes the
 * stamp INVALID, a non-finite one NONFINITE.
 */
int psfm_fit_dual(const psfm_context* ctx, const float* I1, const float* V1, const uint8_t* M1,
                  const float* I2, const float* V2, const uint8_t* M2, int W, int H, int64_t pitch,
                  const int32_t* stamp_xy, int n_stamps, double* stamp_M, double* stamp_b,
                  double* stamp_e, int32_t* stamp_npix, int32_t* stamp_flags, void* ws,
                  size_t ws_bytes, void* stream);

/*
 * psfm_solve_dual: the solution with rejection (as psfm_solve) of the
 * two-kernel form, with the penalty P = Phi Q_i, Q_i = sum (u^2 + v^2)^2
 * k_i(u, v)^2, on the diagonal of every b-term i >= 1 and every c-term (not
 * b_0, the normalisation, nor d0).  Phi is unspecified in the paper beyond
 * "neither negligible nor dominant": here Phi = phi (sum of the penalised
 * unknowns' diagonal) / (sum of their Q_i), recomputed at each assembly, so
 * the penalties add the fraction phi (>= 0) to that diagonal.  The stamp
 * chi2 (rejection, chi2/dof) is the data term alone; kernel_sum_centre is
 * K1's sum at the image centre.  coeffs: N2 float64.
 */
int psfm_solve_dual(const psfm_context* ctx, int W, int H, const int32_t* stamp_xy, int n_stamps,
                    const double* stamp_M, const double* stamp_b, const double* stamp_e,
                    const int32_t* stamp_npix, int32_t* stamp_flags, double phi, double* coeffs,
                    double* stamp_chi2, psfm_fit_stats* stats, void* ws, size_t ws_bytes,
                    void* stream);

/*
 * psfm_dual_subtract: the difference image of the two-kernel form, kernels
 * realised at each patch centre: D = K2 (x) I2 - K1 (x) I1 - d0,
 * V_D = K1^2 (x) V1 + K2^2 (x) V2 (inputs taken as uncorrelated), masked or
 * outside pixels read as 0; diff_mask CONV_BAD within K1's BAD radius of a
 * masked or outside I1 pixel or within K2's of one of I2, else CONV_POOR
 * within h of either.  D and V_D are written everywhere.
 */
int psfm_dual_subtract(const psfm_context* ctx, const double* coeffs, const float* I1,
                       const float* V1, const uint8_t* M1, const float* I2, const float* V2,
                       const uint8_t* M2, int W, int H, int64_t pitch, float* diff,
                       float* diff_var, uint8_t* diff_mask, void* stream);

/*
 * PSF homogenisation for stacking (Section 5.1): every input is matched to a
 * fake target image with one common PSF, the envelope of the inputs' PSFs,
 * so that all inputs share that PSF; outliers among the homogenised inputs
 * are traced back to pixels of the originals; the inputs are then combined
 * (Section 5.2).  Up to PSFM_STACK_MAX_INPUTS inputs; n planes of one array
 * start at multiples of `plane` elements (bytes for masks), each W x H with
 * `pitch`.  No context is needed except by psfm_trace_mask.
 *
 * psfm_envelope_psf: params (device) holds n elliptical Gaussian PSFs as
 * (sigma_major, sigma_minor, angle) triples.  Each is taken in its circular
 * version of peak 1 and width sigma_major (containing the input PSF); env
 * (device, (2 half + 1)^2 float64, row-major, offsets -half..half, half
 * 1..64) receives their pixel-wise maximum, and *sigma (device) the width of
 * the circular peak-1 Gaussian fitted to it by least squares (golden-section
 * search over [0.1, 2 max sigma_major] to a bracket of 1e-10 px).
 */
#define PSFM_STACK_MAX_INPUTS 64
int psfm_envelope_psf(const double* params, int n, int half, double* env, double* sigma,
                      void* stream);

/*
 * psfm_render_target: the fake target image, a circular Gaussian of width
 * sigma (host, 0 < sigma <= 1000) and unit flux sampled at pixel centres,
 * placed at each source of src (device, n (x, y, flux) float64 triples,
 * pixel coordinates) with its flux, over the box of half-width
 * ceil(6 sigma) + 1 around (floor(x), floor(y)); every pixel sums its
 * sources in index order in float64 and stores float32 in out (device,
 * W x H with pitch).  Sources with |x| or |y| >= 1e9 (or NaN) are skipped.
 * ws: device scratch of psfm_render_workspace_bytes(n, W, H, sigma) bytes
 * (0 for invalid arguments).
 */
size_t psfm_render_workspace_bytes(int n, int W, int H, double sigma);
int psfm_render_target(const double* src, int n, double sigma, int W, int H, int64_t pitch,
                       float* out, void* ws, size_t ws_bytes, void* stream);

/*
 * psfm_stack_reject: outlier pixels among n homogenised inputs (1..64).  At
 * each pixel the inputs with M = 0 there are compared with their median (the
 * mean of the two middle values for an even count, in float64); input k is
 * an outlier if |I_k - median| > nsigma sqrt(V_k).  out[k] (device, n planes
 * like I) = 1 for outliers, else 0 (always 0 where fewer than 3 inputs are
 * unmasked, and for masked inputs).
 */
int psfm_stack_reject(int n, const float* I, const float* V, const uint8_t* M, int64_t plane, int W,
                      int H, int64_t pitch, double nsigma, uint8_t* out, void* stream);

/*
 * psfm_trace_mask: outliers found on an image convolved with the context's
 * kernel (coeffs: the solution, device) traced back to the pixels of the
 * input that produced them.  In patch p, pixel x collects |K_p(u)| over the
 * outlier pixels x + u it contributes to (the matched filter of the
 * convolution; outside the image counts as no outlier) and bad = 1 where
 * that sum is positive and at least frac (>= 0) times sum |K_p|, else 0.
 * outliers and bad: device W x H bytes with pitch.
 */
int psfm_trace_mask(const psfm_context* ctx, const double* coeffs, const uint8_t* outliers, int W,
                    int H, int64_t pitch, double frac, uint8_t* bad, void* stream);

/*
 * psfm_stack_combine (Section 5.2): weights w_k = 1 / mean(V_k) over each
 * input's pixels with M = 0 (0 if it has none); at each pixel, over the
 * inputs unmasked there,
 *   S = sum w_k I_k / sum w_k,   V_S = sum w_k^2 V_k / (sum w_k)^2,
 * MS = 0; where none is unmasked S = V_S = 0 and MS = 1.  cov (device,
 * nullable if cov_s is NULL) holds the n inputs' pseudo-matrices, each
 * (2 cov_half + 1)^2; cov_s (device, nullable) receives their average with
 * weights w_k^2 mean(V_k).  weights (device, nullable) receives the w_k.
 * ws: device scratch of PSFM_STACK_WORKSPACE_BYTES.
 */
#define PSFM_STACK_WORKSPACE_BYTES 262656
int psfm_stack_combine(int n, const float* I, const float* V, const uint8_t* M, int64_t plane, int W,
                       int H, int64_t pitch, const double* cov, int cov_half, float* S, float* VS,
                       uint8_t* MS, double* cov_s, double* weights, void* ws, size_t ws_bytes,
                       void* stream);

/*
 * Batched matching of many independent image pairs: the whole path of the
 * calls above (fit, solve with rejection, image and variance convolution,
 * covariance pseudo-matrix, difference) for every pair of a batch, with each
 * stage covering all pairs in one launch (Sections 2-4 per pair; the pairs
 * share nothing but the context's basis, h, r, patch and rejection settings).
 *
 * Per pair the results equal those of the single-pair calls, except that
 * the difference image is formed in the same pass as the convolutions (the
 * convolved image and its variance are written only if requested) and the
 * variance means of C_D are summed per tile instead of per row block.
 */
typedef struct psfm_pair {
    /* inputs (device); image 1 is convolved to match image 2 */
    const float* I1;
    const float* V1;
    const uint8_t* M1;
    const float* I2;
    const float* V2;
    const uint8_t* M2;
    int width, height;
    int64_t pitch;              /* elements (bytes for the masks) */
    const int32_t* stamp_xy;    /* n_stamps (x, y) centres */
    int n_stamps;
    int spatial_order;          /* S of this pair (0..6, N = nb ns + 1 <= 496) */
    const double* cov1;         /* input pseudo-matrix of image 1, NULL: uncorrelated */
    int cov1_half;              /* 0..32 */
    const double* cov2;         /* input pseudo-matrix of image 2, NULL: uncorrelated */
    int cov2_half;
    /* outputs (device) */
    double* coeffs;             /* N(S) float64 */
    psfm_fit_stats* stats;
    float* diff;
    float* diff_var;
    uint8_t* diff_mask;
    double* cov_conv;           /* (2 cov_conv_half + 1)^2: pseudo-matrix of the convolved image */
    int cov_conv_half;
    double* cov_diff;           /* (2 cov_diff_half + 1)^2: pseudo-matrix of the difference */
    int cov_diff_half;
    /* optional outputs (device, NULL: not written) */
    float* conv;                /* I' */
    float* conv_var;            /* V' */
    uint8_t* conv_mask;         /* BAD/POOR of I' (required if conv is given) */
    int32_t* stamp_flags;       /* n_stamps */
    double* stamp_chi2;         /* n_stamps */
} psfm_pair;

/* Launch shape of a batch.  apply_grid: workgroups of the fused apply kernel,
   which visits the 64 x 64 tiles of all pairs in a grid-stride loop (0: one
   workgroup per tile).  order: order of the pairs in the tile list
   (0 as given, 1 smallest first, 2 largest first). */
typedef struct psfm_batch_tuning {
    int apply_grid;
    int order;
} psfm_batch_tuning;

typedef struct psfm_batch psfm_batch;

/* Workspace bytes of a batch (0 on invalid arguments). */
size_t psfm_batch_workspace_bytes(const psfm_context* ctx, const psfm_pair* pairs, int n_pairs);

/*
 * Validates the pairs (host array of n_pairs descriptors, copied), lays out
 * the workspace and uploads the pair descriptors and work lists into it
 * (ordered on `stream`; the call waits for the upload).  times (device,
 * n_pairs + 1 uint64, nullable) receives at each run the start time (entry
 * 0) and each pair's completion time (entry 1 + p) in wall-clock ticks
 * (psfm_wall_clock_hz per second).  *out receives a host-side plan freed by
 * psfm_batch_destroy; no device memory is allocated.  The workspace and the
 * pair buffers must outlive the plan.
 */
int psfm_batch_plan(const psfm_context* ctx, const psfm_pair* pairs, int n_pairs,
                    const psfm_batch_tuning* tuning, void* ws, size_t ws_bytes, uint64_t* times,
                    void* stream, psfm_batch** out);

/* Launches every stage of the batch on `stream` (about 10 + 8 max_iter
   kernels); capturable into a HIP graph.  Runs of one plan must not overlap. */
int psfm_batch_run(psfm_batch* batch, void* stream);

/* One stage of psfm_batch_run: 0 = start time and stamp fits, 1 = solve
   loop, 2 = the patch kernels of every pair (FP32 taps and BAD radii kept in
   the workspace) and the pseudo-matrices of the convolved images, 3 = the
   fused convolution / difference pass (one launch, reading the taps of
   stage 2).  Running stages 0, 1, 2, 3 in order is psfm_batch_run (for
   timing stages). */
int psfm_batch_run_stage(psfm_batch* batch, int stage, void* stream);

/* Changes the apply grid of a plan (tuning->order is fixed at plan time).
   Drops a captured graph. */
int psfm_batch_set_tuning(psfm_batch* batch, const psfm_batch_tuning* tuning);

/* Captures psfm_batch_run on `stream` (not the NULL stream) into a HIP graph
   kept by the plan; psfm_batch_graph_launch replays it on `stream`. */
int psfm_batch_graph_capture(psfm_batch* batch, void* stream);
int psfm_batch_graph_launch(psfm_batch* batch, void* stream);

int psfm_batch_destroy(psfm_batch* batch);

/*
 * Several plans run side by side (a scheduling of the same work, Section 2's
 * fits and solves and Section 3.5's convolutions per pair unchanged): one HIP
 * graph in which each plan's psfm_batch_run is a branch of its own, forked
 * from and joined back to `stream` (not the NULL stream) during the capture.
 * Plans whose pairs differ in unknown count (spatial order) finish their
 * latency-bound solves at different times, so one plan's tile pass fills the
 * device while another still solves.  batches: host array of n (1..16)
 * plans that share no workspace or outputs; the group keeps the pointers,
 * so the plans must outlive it and must not run while it runs.  The capture
 * creates one stream and one event per plan and releases them before it
 * returns; no device memory is allocated.  *out receives a host-side object
 * freed by psfm_batch_group_destroy.  Each plan's time stamps (times of
 * psfm_batch_plan) count from that plan's own start.
 */
typedef struct psfm_batch_group psfm_batch_group;
int psfm_batch_group_capture(psfm_batch* const* batches, int n, void* stream,
                             psfm_batch_group** out);
/* Replays the group's graph on `stream`. */
int psfm_batch_group_launch(psfm_batch_group* group, void* stream);
int psfm_batch_group_destroy(psfm_batch_group* group);

/* Tick rate of the device wall clock used by the batch time stamps. */
double psfm_wall_clock_hz(void);

/*
 * Learned prior: a small CNN that predicts a stamp's kernel from the stamp
 * pair.  Input per stamp: 2 x 41 x 41 FP16 (the reference and target
 * windows); output: PSFM_CNN_OUT FP32 coefficients of the kernel in an
 * orthonormal basis of the kernel-basis span (c = R a with G = R^T R the
 * Gram matrix of the basis taps, so |c| is the kernel-image L2 norm).
 *   conv1 3x3 2->32 stride 1, conv2..conv4 3x3 32->32 stride 2 (zero
 *   padding 1, ReLU; 41 -> 41 -> 21 -> 11 -> 6), fc1 1152 -> 128 ReLU,
 *   fc2 128 -> 49.  Convolutions are cross-correlations.
 * Parameters: one flat vector, for conv1..conv4, fc1, fc2 the weight
 * (row-major [out][in][3][3] or [out][in]) then the bias; FP32 master copy
 * and FP16 working copy (uint16_t bit patterns).  All pointers device.
 */
#define PSFM_CNN_SIDE 41
#define PSFM_CNN_OUT 49

size_t psfm_cnn_param_count(void);
size_t psfm_cnn_workspace_bytes(int batch);

/* out (batch x 49 FP32) = net(x); x: batch x 2 x 41 x 41 FP16. */
int psfm_cnn_forward(const uint16_t* w16, const uint16_t* x, int batch, float* out, void* ws,
                     size_t ws_bytes, void* stream);

/* Forward, loss and its gradient in the parameters (grad, FP32, overwritten).
   loss (device float, may be NULL) = sum_b r_b^T W_b r_b / (batch * 49),
   r_b = out_b - target_b, with W_b = weight[b] (49 x 49 FP32, symmetric) or
   the identity if weight is NULL (plain mean squared error). */
int psfm_cnn_loss_grad(const uint16_t* w16, const uint16_t* x, const float* target,
                       const float* weight, int batch, float* grad, float* loss, void* ws,
                       size_t ws_bytes, void* stream);

/* Loss weights of n stamps (n x 49 x 49 FP32): W = R^-T Mh R^-1 / npix with
   Mh the stamp matrix with the background eliminated, so that r^T W r is the
   chi2/dof excess of a kernel whose orthonormal coefficients are off by r
   (background re-fitted).  Flagged stamps get zeros.  Needs nb = 49. */
int psfm_cnn_loss_weights(const psfm_context* ctx, const double* stamp_M, const int32_t* stamp_npix,
                          const int32_t* stamp_flags, int n_stamps, float* weight, void* stream);

/* One Adam step (bias-corrected, step >= 1) on the FP32 master weights; the
   FP16 copy is refreshed.  m, v: FP32 moments, n = psfm_cnn_param_count(). */
int psfm_cnn_adam(float* w32, uint16_t* w16, float* m, float* v, const float* grad, size_t n,
                  int step, float lr, float beta1, float beta2, float eps, void* stream);

/* Network inputs of n stamps: the 41 x 41 windows of I1 and I2 around each
   centre, minus the mean of each window's unmasked border, divided by the
   reference window's flux F (summed window minus its sky) floored at
   3 sigma_b sqrt(n) (sigma_b: scatter of the reference border, n: valid
   pixels), times 100, clamped to +-60000 (masked / outside pixels 0).
   x: n x 2 x 41 x 41 FP16; flux (nullable): F. */
int psfm_cnn_stamp_inputs(const float* I1, const uint8_t* M1, const float* I2, const uint8_t* M2,
                          int W, int H, int64_t pitch, const int32_t* stamp_xy, int n_stamps,
                          uint16_t* x, float* flux, void* stream);

/* Orthonormal-basis coefficients from local coefficients (n x L, the first
   nb used): ortho = R a (n x 49 FP32); and back: local = R^-1 ortho (the
   background slot set to 0).  Need nb = 49. */
int psfm_cnn_targets(const psfm_context* ctx, const double* local, int n_stamps, float* ortho,
                     void* stream);
int psfm_cnn_local_coeffs(const psfm_context* ctx, const float* ortho, int n_stamps,
                          double* local, void* stream);

/* Training-set standardisation of the prior's targets.  Per component c,
   mu[c] and sd[c] (the unbiased standard deviation, floored at 1e-12) over
   the first n_stats rows of target (n x 49 FP32); then for all n rows
   z = (target - mu) / sd, and the loss weights carried into z coordinates,
   wz = diag(sd) W diag(sd) divided by its mean diagonal (trace / 49, the
   trace floored at 1e-30), so that every stamp counts alike in the loss.
   weight, wz: n x 49 x 49 FP32.  Requires 2 <= n_stats <= n. */
int psfm_cnn_standardize(const float* target, const float* weight, int n, int n_stats,
                         float* mu, float* sd, float* z, float* wz, void* stream);

/* Folds the standardisation into the network: fc2's weight rows times sd,
   its bias sd * b + mu (FP32 master and FP16 copy), so that the network
   returns the coefficients themselves. */
int psfm_cnn_fold_output(float* w32, uint16_t* w16, const float* mu, const float* sd, void* stream);

/* Per-sample excess r^T W r, r = pred - target (n x 49 FP32), W = weight[s]
   (49 x 49): with the weights of psfm_cnn_loss_weights, the chi2/dof excess
   of the predicted kernel.  pred rows pred_stride (49, or 0: the same row,
   e.g. a constant predictor, for every sample) apart.  exc: n FP32. */
int psfm_cnn_excess(const float* pred, int pred_stride, const float* target, const float* weight,
                    int n, float* exc, void* stream);

/* Human-readable text of a psfm_status value (static storage). */
const char* psfm_status_string(int status);

#ifdef __cplusplus
}
#endif

#endif /* PSFM_H */
