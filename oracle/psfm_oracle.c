/*
 * psfm_oracle.c -- plain FP64 CPU reference for the PSF-matching hot path of
 * Price & Magnier, "Pan-STARRS PSF-Matching for Subtraction and Stacking".
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
 * benchmark's CPU-baseline leg load this library.  The product path (the HIP
 * library) never links, calls or includes anything from here, and this file
 * shares no code, header, table or helper with it.
 *
 * Every function computes the paper's definition directly, in double
 * precision, without blocking, separability or reordering beyond what the
 * definition states:
 *   - basis kernels: Section 2, Eq. 7 with the zero-sum requirement of
 *     Section 2 (flux conservation) -- each k_i (i >= 1) sums to zero;
 *   - design matrix, normal equations: Section 2, Eqs. 3-6 with c = 0, p = 0;
 *   - spatial variation evaluated at the stamp centre: Section 2;
 *   - stamp validity: Section 3.3 (masked pixels in the footprint);
 *   - rejection of discrepant stamps: Sections 3.3 and 3.6;
 *   - patch-wise constant kernels: Section 3.5;
 *   - BAD/POOR masking: Section 3.4;
 *   - image and variance convolution: Section 4.2, Eqs. 12-13;
 *   - covariance pseudo-matrix: Section 4.2 (Eqs. 10-11 applied to a kernel),
 *     covariance factor and Section 4.3 (sample average, factor removal);
 *   - image subtraction noise: Section 4.3.
 * Readings of points the paper leaves open are stated where they are used.
 *
 * Conventions: images are row-major, element (x, y) at [y * pitch + x];
 * kernels are (2h+1)^2 arrays indexed [(v + h) * (2h+1) + (u + h)] with u the
 * column (x) offset and v the row (y) offset; masks are uint8, non-zero means
 * masked.  OpenMP threads run over stamps and over patches, as the paper's
 * implementation threads over stamps and patches (Section 3.5).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_MAX_GAUSS 8

typedef struct {
    int n_gauss;
    double sigma[ORC_MAX_GAUSS];
    int degree[ORC_MAX_GAUSS];
    int h;              /* kernel half width: u, v in [-h, h] */
    int S;              /* spatial polynomial order */
    int r;              /* stamp half width: stamp is (2r+1)^2 pixels */
    int P;              /* side of the constant-kernel patches */
    double clip_sigma;  /* rejection threshold in standard deviations */
    int max_iter;       /* maximum number of solutions */
    int min_stamps;     /* fewer usable stamps is an error */
    double bad_frac;    /* BAD/POOR fraction of sum(k^2) */
} orc_config;

typedef struct {
    double chi2, dof, chi2_dof, kernel_sum_centre, cov_discarded_frac;
    int n_used, n_rejected, n_iter, info;
} orc_stats;

/* stamp flag bits */
#define ORC_STAMP_INVALID   1   /* footprint leaves the image or touches a mask */
#define ORC_STAMP_REJECTED  2   /* removed by the rejection iterations */
#define ORC_STAMP_NONFINITE 4   /* non-finite pixel or non-positive variance */
/* output mask bits */
#define ORC_MASK_BAD       1
#define ORC_MASK_CONV_BAD  2
#define ORC_MASK_CONV_POOR 4

static double ipow(double x, int n) {
    double r = 1.0;
    for (int k = 0; k < n; k++) r *= x;
    return r;
}

int orc_n_basis(const orc_config* c) {
    int n = 0;
    for (int j = 0; j < c->n_gauss; j++) n += (c->degree[j] + 1) * (c->degree[j] + 2) / 2;
    return n;
}

int orc_n_spatial(const orc_config* c) { return (c->S + 1) * (c->S + 2) / 2; }

int orc_n_unknowns(const orc_config* c) { return orc_n_basis(c) * orc_n_spatial(c) + 1; }

/*
 * Kernel basis (Section 2, Eq. 7; Section 3.1).  For Gaussian j of width
 * sigma_j and each polynomial term u^p v^q with p + q <= degree_j (terms
 * ordered by total degree d, then p from d down to 0):
 *     raw(u, v) = u^p v^q exp(-(u^2 + v^2) / (2 sigma_j^2)).
 * Reading of the printed exponent: its sign is lost in the source; a Gaussian
 * that decays away from the centre is meant.
 * The first term carries the flux: k_0 = raw_0 / sum(raw_0) (unit sum).
 * The zero-sum requirement of Section 2 is met by subtracting k_0 from each
 * other term that has a non-zero sum (p and q both even):
 *     k_i = raw_i / sum(raw_i) - k_0,
 * while terms odd in u or v already sum to zero and are scaled to unit L1
 * norm: k_i = raw_i / sum(|raw_i|).
 */
void orc_basis(const orc_config* c, double* k) {
    const int K = 2 * c->h + 1, T = K * K, h = c->h;
    double* raw = (double*)malloc(sizeof(double) * T);
    int i = 0;
    for (int j = 0; j < c->n_gauss; j++) {
        const double s2 = 2.0 * c->sigma[j] * c->sigma[j];
        for (int d = 0; d <= c->degree[j]; d++) {
            for (int p = d; p >= 0; p--) {
                const int q = d - p;
                double sum = 0.0, sabs = 0.0;
                for (int v = -h; v <= h; v++)
                    for (int u = -h; u <= h; u++) {
                        double val = ipow(u, p) * ipow(v, q) * exp(-(double)(u * u + v * v) / s2);
                        raw[(v + h) * K + (u + h)] = val;
                        sum += val;
                        sabs += fabs(val);
                    }
                double* ki = k + (size_t)i * T;
                if (i == 0) {
                    for (int t = 0; t < T; t++) ki[t] = raw[t] / sum;
                } else if (p % 2 == 0 && q % 2 == 0) {
                    for (int t = 0; t < T; t++) ki[t] = raw[t] / sum - k[t];
                } else {
                    for (int t = 0; t < T; t++) ki[t] = raw[t] / sabs;
                }
                i++;
            }
        }
    }
    free(raw);
}

/*
 * Spatial polynomial terms g_s(x, y) (Section 2: ordinary polynomials x^l y^m).
 * Reading: coordinates are scaled to [-1, 1] over the image,
 *     xt = (2x - (W-1)) / (W-1),  yt = (2y - (H-1)) / (H-1),
 * and the terms x^l y^m with l + m <= S are ordered by degree, then l
 * descending: 1, x, y, x^2, xy, y^2, ...
 */
void orc_spatial(int S, double x, double y, int W, int H, double* g) {
    const double xt = W > 1 ? (2.0 * x - (W - 1)) / (double)(W - 1) : 0.0;
    const double yt = H > 1 ? (2.0 * y - (H - 1)) / (double)(H - 1) : 0.0;
    int s = 0;
    for (int d = 0; d <= S; d++)
        for (int l = d; l >= 0; l--) g[s++] = ipow(xt, l) * ipow(yt, d - l);
}

/*
 * Local kernel coefficients at a point: alpha_i(x, y) = sum_s a[i*ns + s] g_s(x, y)
 * for the nb kernel terms, plus the background coefficient (last unknown) in
 * alpha[nb].  Unknown ordering: kernel term i, spatial term s at i*ns + s;
 * the constant background last.
 */
void orc_local_coeffs(const orc_config* c, const double* a, double x, double y, int W, int H,
                      double* alpha) {
    const int nb = orc_n_basis(c), ns = orc_n_spatial(c), N = nb * ns + 1;
    double g[64];
    orc_spatial(c->S, x, y, W, H, g);
    for (int i = 0; i < nb; i++) {
        double s = 0.0;
        for (int t = 0; t < ns; t++) s += a[i * ns + t] * g[t];
        alpha[i] = s;
    }
    alpha[nb] = a[N - 1];
}

/* The kernel realised at a point: K(u, v) = sum_i alpha_i(x, y) k_i(u, v). */
void orc_kernel_at(const orc_config* c, const double* kb, const double* a, double x, double y,
                   int W, int H, double* K) {
    const int nb = orc_n_basis(c), T = (2 * c->h + 1) * (2 * c->h + 1);
    double* alpha = (double*)malloc(sizeof(double) * (nb + 1));
    orc_local_coeffs(c, a, x, y, W, H, alpha);
    for (int t = 0; t < T; t++) {
        double s = 0.0;
        for (int i = 0; i < nb; i++) s += alpha[i] * kb[(size_t)i * T + t];
        K[t] = s;
    }
    free(alpha);
}

/*
 * Per-stamp normal equations (Section 2, Eqs. 3-6 with c_i = 0 and P = 0).
 * For every stamp pixel (x, y), with the true convolution of Section 4.2,
 *     A_i(x, y) = sum_{u,v} k_i(u, v) I1(x - u, y - v)     (i < nb)
 *     A_nb      = 1                                        (constant background)
 *     w = 1 / V2(x, y),  d = I2(x, y)
 * (or w = 1 / (V1 + V2) when V1 is given: the variance of the convolved
 * image counted as well, the sum taken in float as the images are stored)
 * and the stamp accumulates M_s = sum w A A^T (L x L, L = nb + 1),
 * b_s = sum w A d and e_s = sum w d^2.
 * Validity (Section 3.3): a stamp whose convolution footprint
 * [x-r-h, x+r+h]^2 leaves the image or holds a masked I1 pixel, or whose
 * stamp [x-r, x+r]^2 holds a masked I2 pixel, is flagged INVALID; a stamp
 * holding a non-finite I1/I2 value or a weight variance that is not finite
 * and positive is flagged NONFINITE.  Flagged stamps get zero sums.
 */
static float weight_var(const float* V1, const float* V2, int64_t o) {
    return V1 ? V2[o] + V1[o] : V2[o];
}

void orc_fit_stamps(const orc_config* c, const double* kb, const float* I1, const uint8_t* M1,
                    const float* I2, const float* V2, const uint8_t* M2, int W, int H,
                    int64_t pitch, const int32_t* xy, int n, double* Ms, double* bs, double* es,
                    int32_t* npix, int32_t* flags, const float* V1) {
    const int nb = orc_n_basis(c), L = nb + 1, h = c->h, r = c->r, K = 2 * h + 1,
              T = K * K;
#pragma omp parallel for schedule(dynamic)
    for (int s = 0; s < n; s++) {
        const int xc = xy[2 * s], yc = xy[2 * s + 1], R = r + h;
        double* M = Ms + (size_t)s * L * L;
        double* b = bs + (size_t)s * L;
        int flag = 0;
        memset(M, 0, sizeof(double) * L * L);
        memset(b, 0, sizeof(double) * L);
        es[s] = 0.0;
        npix[s] = 0;
        if (xc - R < 0 || yc - R < 0 || xc + R >= W || yc + R >= H) {
            flag |= ORC_STAMP_INVALID;
        } else {
            for (int y = yc - R; y <= yc + R; y++)
                for (int x = xc - R; x <= xc + R; x++)
                    if (M1[y * pitch + x]) flag |= ORC_STAMP_INVALID;
            for (int y = yc - r; y <= yc + r; y++)
                for (int x = xc - r; x <= xc + r; x++)
                    if (M2[y * pitch + x]) flag |= ORC_STAMP_INVALID;
            if (!flag) {
                for (int y = yc - R; y <= yc + R; y++)
                    for (int x = xc - R; x <= xc + R; x++)
                        if (!isfinite(I1[y * pitch + x])) flag |= ORC_STAMP_NONFINITE;
                for (int y = yc - r; y <= yc + r; y++)
                    for (int x = xc - r; x <= xc + r; x++) {
                        const float v2 = weight_var(V1, V2, y * pitch + x);
                        if (!isfinite(I2[y * pitch + x]) || !isfinite(v2) || !(v2 > 0.0f))
                            flag |= ORC_STAMP_NONFINITE;
                    }
            }
        }
        flags[s] = flag;
        if (flag) continue;
        double* A = (double*)malloc(sizeof(double) * L);
        double* win = (double*)malloc(sizeof(double) * T);
        for (int y = yc - r; y <= yc + r; y++) {
            for (int x = xc - r; x <= xc + r; x++) {
                for (int v = -h; v <= h; v++)
                    for (int u = -h; u <= h; u++)
                        win[(v + h) * K + (u + h)] = I1[(int64_t)(y - v) * pitch + (x - u)];
                for (int i = 0; i < nb; i++) {
                    const double* ki = kb + (size_t)i * T;
                    double acc = 0.0;
                    for (int t = 0; t < T; t++) acc += ki[t] * win[t];
                    A[i] = acc;
                }
                A[nb] = 1.0;
                const double w = 1.0 / (double)weight_var(V1, V2, y * pitch + x);
                const double d = (double)I2[y * pitch + x];
                for (int i = 0; i < L; i++) {
                    for (int j = 0; j < L; j++) M[i * L + j] += w * A[i] * A[j];
                    b[i] += w * A[i] * d;
                }
                es[s] += w * d * d;
            }
        }
        npix[s] = (2 * r + 1) * (2 * r + 1);
        free(A);
        free(win);
    }
}

/*
 * Assembly of the full normal equations from the per-stamp sums, with the
 * spatial terms evaluated at the stamp centres (Section 2):
 *     M[(i,s),(j,t)] = sum_stamps g_s g_t M_s[i][j]
 *     M[(i,s),bg]    = sum_stamps g_s M_s[i][nb]
 *     M[bg,bg]       = sum_stamps M_s[nb][nb]
 * and likewise for the right-hand side.  Only stamps with used[s] != 0 count.
 */
void orc_assemble(const orc_config* c, int W, int H, const int32_t* xy, int n, const double* Ms,
                  const double* bs, const uint8_t* used, double* M, double* b) {
    const int nb = orc_n_basis(c), ns = orc_n_spatial(c), N = nb * ns + 1, L = nb + 1;
    double g[64];
    memset(M, 0, sizeof(double) * N * N);
    memset(b, 0, sizeof(double) * N);
    for (int s = 0; s < n; s++) {
        if (!used[s]) continue;
        orc_spatial(c->S, xy[2 * s], xy[2 * s + 1], W, H, g);
        const double* Mss = Ms + (size_t)s * L * L;
        const double* bss = bs + (size_t)s * L;
        for (int i = 0; i < nb; i++)
            for (int sa = 0; sa < ns; sa++) {
                const int row = i * ns + sa;
                for (int j = 0; j < nb; j++)
                    for (int t = 0; t < ns; t++)
                        M[(size_t)row * N + j * ns + t] += g[sa] * g[t] * Mss[i * L + j];
                M[(size_t)row * N + N - 1] += g[sa] * Mss[i * L + nb];
                M[(size_t)(N - 1) * N + row] += g[sa] * Mss[nb * L + i];
                b[row] += g[sa] * bss[i];
            }
        M[(size_t)(N - 1) * N + N - 1] += Mss[nb * L + nb];
        b[N - 1] += bss[nb];
    }
}

/*
 * Solution of M a = b "by regular matrix methods" (Section 2): symmetric
 * equilibration D = diag(M)^(-1/2), Cholesky factorisation of D M D, forward
 * and back substitution, a = D y.  Returns 0, or k > 0 when the k-th pivot
 * (1-based) is not positive.
 */
int orc_cholesky_solve(int N, const double* M, const double* b, double* a) {
    double* D = (double*)malloc(sizeof(double) * N);
    double* Lm = (double*)malloc(sizeof(double) * (size_t)N * N);
    double* y = (double*)malloc(sizeof(double) * N);
    int info = 0;
    for (int i = 0; i < N; i++) {
        if (!(M[(size_t)i * N + i] > 0.0)) { info = i + 1; goto done; }
        D[i] = 1.0 / sqrt(M[(size_t)i * N + i]);
    }
    for (int i = 0; i < N; i++)
        for (int j = 0; j < N; j++) Lm[(size_t)i * N + j] = D[i] * M[(size_t)i * N + j] * D[j];
    for (int k = 0; k < N; k++) {
        double s = Lm[(size_t)k * N + k];
        for (int p = 0; p < k; p++) s -= Lm[(size_t)k * N + p] * Lm[(size_t)k * N + p];
        if (!(s > 0.0)) { info = k + 1; goto done; }
        const double lkk = sqrt(s);
        Lm[(size_t)k * N + k] = lkk;
        for (int i = k + 1; i < N; i++) {
            double t = Lm[(size_t)i * N + k];
            for (int p = 0; p < k; p++) t -= Lm[(size_t)i * N + p] * Lm[(size_t)k * N + p];
            Lm[(size_t)i * N + k] = t / lkk;
        }
    }
    for (int i = 0; i < N; i++) {          /* L z = D b */
        double t = D[i] * b[i];
        for (int p = 0; p < i; p++) t -= Lm[(size_t)i * N + p] * y[p];
        y[i] = t / Lm[(size_t)i * N + i];
    }
    for (int i = N - 1; i >= 0; i--) {     /* L^T y = z */
        double t = y[i];
        for (int p = i + 1; p < N; p++) t -= Lm[(size_t)p * N + i] * y[p];
        y[i] = t / Lm[(size_t)i * N + i];
    }
    for (int i = 0; i < N; i++) a[i] = D[i] * y[i];
done:
    free(D);
    free(Lm);
    free(y);
    return info;
}

/*
 * Residual chi^2 of one stamp for a solution a, from its sums:
 *     chi2_s = e_s - 2 alpha^T b_s + alpha^T M_s alpha,
 * alpha the local coefficients at the stamp centre (kernel terms and
 * background).  This equals sum w (A alpha - d)^2 over the stamp pixels.
 */
double orc_stamp_chi2(const orc_config* c, const double* a, int W, int H, int xc, int yc,
                      const double* Mss, const double* bss, double es) {
    const int nb = orc_n_basis(c), L = nb + 1;
    double alpha[512];
    orc_local_coeffs(c, a, xc, yc, W, H, alpha);
    double q = 0.0, lin = 0.0;
    for (int i = 0; i < L; i++) {
        double t = 0.0;
        for (int j = 0; j < L; j++) t += Mss[i * L + j] * alpha[j];
        q += alpha[i] * t;
        lin += alpha[i] * bss[i];
    }
    return es - 2.0 * lin + q;
}

/*
 * Solution with rejection of discrepant stamps (Sections 3.3, 3.5, 3.6).
 * Readings: the per-stamp statistic is q_s = chi2_s / npix_s (the mean
 * squared normalised residual, with no flux softening); after each solution
 * the used stamps with q_s > mean + clip_sigma * std (population standard
 * deviation over the used stamps) are rejected and the equations are
 * re-assembled and re-solved, up to max_iter solutions or until nothing
 * changes.  Rejected stamps are not replaced.  A clip that would leave fewer
 * than min_stamps stamps is not applied.  Stamps flagged on input (any bit)
 * are not used.  Returns 0, -3 (fewer than min_stamps usable stamps) or -4
 * (matrix not positive definite; stats->info holds the pivot).
 * Output flags gain ORC_STAMP_REJECTED for rejected stamps; chi2[s] holds
 * the residual of every unflagged-on-input stamp under the final solution
 * (0 for the others).
 */
int orc_solve(const orc_config* c, int W, int H, const int32_t* xy, int n, const double* Ms,
              const double* bs, const double* es, const int32_t* npix, int32_t* flags,
              double* coeffs, double* chi2, orc_stats* st) {
    const int nb = orc_n_basis(c), ns = orc_n_spatial(c), N = nb * ns + 1, L = nb + 1;
    uint8_t* used = (uint8_t*)calloc(n > 0 ? n : 1, 1);
    uint8_t* fitted = (uint8_t*)calloc(n > 0 ? n : 1, 1);
    double* M = (double*)malloc(sizeof(double) * (size_t)N * N);
    double* b = (double*)malloc(sizeof(double) * N);
    int ret = 0, iter = 0, n_rej = 0;
    memset(st, 0, sizeof(*st));
    for (int s = 0; s < n; s++) {
        used[s] = flags[s] == 0;
        fitted[s] = used[s];
        chi2[s] = 0.0;
    }
    for (int i = 0; i < N; i++) coeffs[i] = 0.0;
    for (;;) {
        int n_used = 0;
        for (int s = 0; s < n; s++) n_used += used[s];
        if (n_used < c->min_stamps) { ret = -3; st->info = -3; break; }
        orc_assemble(c, W, H, xy, n, Ms, bs, used, M, b);
        int info = orc_cholesky_solve(N, M, b, coeffs);
        if (info) { ret = -4; st->info = info; break; }
        iter++;
        for (int s = 0; s < n; s++)
            chi2[s] = fitted[s] ? orc_stamp_chi2(c, coeffs, W, H, xy[2 * s], xy[2 * s + 1],
                                                  Ms + (size_t)s * L * L, bs + (size_t)s * L, es[s])
                                : 0.0;
        if (iter >= c->max_iter) break;
        double mean = 0.0, var = 0.0;
        for (int s = 0; s < n; s++)
            if (used[s]) mean += chi2[s] / npix[s];
        mean /= n_used;
        for (int s = 0; s < n; s++)
            if (used[s]) {
                const double dq = chi2[s] / npix[s] - mean;
                var += dq * dq;
            }
        const double thr = mean + c->clip_sigma * sqrt(var / n_used);
        int n_new = 0;
        for (int s = 0; s < n; s++)
            if (used[s] && chi2[s] / npix[s] > thr) n_new++;
        if (n_new == 0 || n_used - n_new < c->min_stamps) break;
        for (int s = 0; s < n; s++)
            if (used[s] && chi2[s] / npix[s] > thr) {
                used[s] = 0;
                flags[s] |= ORC_STAMP_REJECTED;
                n_rej++;
            }
    }
    st->n_iter = iter;
    st->n_rejected = n_rej;
    if (ret != 0)
        for (int i = 0; i < N; i++) coeffs[i] = 0.0;   /* no solution on failure */
    if (ret == 0) {
        double c2 = 0.0, np = 0.0;
        int nu = 0;
        for (int s = 0; s < n; s++)
            if (used[s]) { c2 += chi2[s]; np += npix[s]; nu++; }
        st->chi2 = c2;
        st->dof = np - N;
        st->chi2_dof = c2 / (np - N);
        st->n_used = nu;
        double alpha[512];
        orc_local_coeffs(c, coeffs, 0.5 * (W - 1), 0.5 * (H - 1), W, H, alpha);
        st->kernel_sum_centre = alpha[0];   /* the other terms sum to zero */
    }
    free(used);
    free(fitted);
    free(M);
    free(b);
    return ret;
}

/*
 * BAD/POOR radius (Section 3.4).  Reading: the smallest box radius r in
 * [0, h] such that the kernel's squared weight outside the box
 * max(|u|,|v|) <= r is below bad_frac of the total; h if none is.
 */
int orc_bad_radius(const double* K, int h, double frac) {
    const int Kw = 2 * h + 1;
    double tot = 0.0;
    for (int t = 0; t < Kw * Kw; t++) tot += K[t] * K[t];
    for (int r = 0; r <= h; r++) {
        double out = 0.0;
        for (int v = -h; v <= h; v++)
            for (int u = -h; u <= h; u++)
                if (abs(u) > r || abs(v) > r) out += K[(v + h) * Kw + (u + h)] * K[(v + h) * Kw + (u + h)];
        if (out < frac * tot) return r;
    }
    return h;
}

/*
 * Covariance pseudo-matrix of a kernel (Section 4.2, Eqs. 10-11 applied to a
 * convolution): the covariance between a pixel and the pixel displaced by
 * delta, relative to the input variance, is
 *     raw(delta) = sum_{u,u'} k(u) k(u') C_in(delta + u - u'),
 * for |delta| <= 2h + c_in (per axis), an array of side 4h + 2c_in + 1.
 * cov_in is (2c_in+1)^2 with its centre at zero offset; NULL means the
 * uncorrelated input (a single unit centre value).
 */
void orc_cov_raw(const double* K, int h, const double* cov_in, int c_in, double* raw) {
    const int Kw = 2 * h + 1, Cw = 2 * c_in + 1, R = 2 * h + c_in, Rw = 2 * R + 1;
    for (int dy = -R; dy <= R; dy++)
        for (int dx = -R; dx <= R; dx++) {
            double s = 0.0;
            for (int v = -h; v <= h; v++)
                for (int u = -h; u <= h; u++) {
                    const double ku = K[(v + h) * Kw + (u + h)];
                    if (ku == 0.0) continue;
                    for (int wy = -c_in; wy <= c_in; wy++)
                        for (int wx = -c_in; wx <= c_in; wx++) {
                            /* C_in(delta + u - u') is needed at w = delta + u - u' */
                            const int u2 = dx + u - wx, v2 = dy + v - wy;
                            if (u2 < -h || u2 > h || v2 < -h || v2 > h) continue;
                            const double cw = cov_in ? cov_in[(wy + c_in) * Cw + (wx + c_in)]
                                                     : (wx == 0 && wy == 0 ? 1.0 : 0.0);
                            s += ku * K[(v2 + h) * Kw + (u2 + h)] * cw;
                        }
                }
            raw[(dy + R) * Rw + (dx + R)] = s;
        }
}

/*
 * Covariance factor of a kernel (Section 4.2): with K = [sum k^2]^-1 absorbed
 * into the pseudo-matrix, C'(delta) = K raw(delta) and the factor is its
 * centre value C'(0) = raw(0) / sum k^2.
 */
double orc_cov_factor(const double* Kk, int h, const double* cov_in, int c_in) {
    const int Kw = 2 * h + 1, Cw = 2 * c_in + 1;
    double s2 = 0.0, raw0 = 0.0;
    for (int t = 0; t < Kw * Kw; t++) s2 += Kk[t] * Kk[t];
    for (int v = -h; v <= h; v++)
        for (int u = -h; u <= h; u++)
            for (int v2 = -h; v2 <= h; v2++)
                for (int u2 = -h; u2 <= h; u2++) {
                    const int wx = u - u2, wy = v - v2;
                    if (wx < -c_in || wx > c_in || wy < -c_in || wy > c_in) continue;
                    const double cw = cov_in ? cov_in[(wy + c_in) * Cw + (wx + c_in)]
                                             : (wx == 0 && wy == 0 ? 1.0 : 0.0);
                    raw0 += Kk[(v + h) * Kw + (u + h)] * Kk[(v2 + h) * Kw + (u2 + h)] * cw;
                }
    return s2 > 0.0 ? raw0 / s2 : 0.0;
}

/* Patch p of the P x P grid anchored at (0, 0); edge patches are clipped and
   the kernel is realised at the clipped patch's centre (Section 3.5). */
static void patch_bounds(int W, int H, int P, int p, int* x0, int* x1, int* y0, int* y1) {
    const int npx = (W + P - 1) / P;
    const int px = p % npx, py = p / npx;
    *x0 = px * P;
    *x1 = *x0 + P < W ? *x0 + P : W;
    *y0 = py * P;
    *y1 = *y0 + P < H ? *y0 + P : H;
}

int orc_n_patches(const orc_config* c, int W, int H) {
    return ((W + c->P - 1) / c->P) * ((H + c->P - 1) / c->P);
}

void orc_patch_kernel(const orc_config* c, const double* kb, const double* a, int W, int H, int p,
                      double* K) {
    int x0, x1, y0, y1;
    patch_bounds(W, H, c->P, p, &x0, &x1, &y0, &y1);
    orc_kernel_at(c, kb, a, 0.5 * (x0 + x1 - 1), 0.5 * (y0 + y1 - 1), W, H, K);
}

/*
 * Image convolution with the spatially varying kernel (Section 4.2, Eq. 12;
 * Section 3.5): in each patch, I'(x, y) = sum_{u,v} K_p(u, v) I~(x-u, y-v)
 * where I~ is I inside the image and unmasked, and 0 otherwise (masked pixels
 * do not contribute, Section 3.4).  Output mask (Section 3.4): CONV_BAD if a
 * masked or out-of-image input pixel lies within box radius r_bad(p) of the
 * output pixel, else CONV_POOR if one lies within the kernel's box radius h.
 */
void orc_convolve_image(const orc_config* c, const double* kb, const double* a, const float* I,
                        const uint8_t* Mk, int W, int H, int64_t pitch, float* out,
                        uint8_t* out_mask) {
    const int h = c->h, Kw = 2 * h + 1, T = Kw * Kw, np = orc_n_patches(c, W, H);
#pragma omp parallel for schedule(dynamic)
    for (int p = 0; p < np; p++) {
        int x0, x1, y0, y1;
        double* K = (double*)malloc(sizeof(double) * T);
        patch_bounds(W, H, c->P, p, &x0, &x1, &y0, &y1);
        orc_patch_kernel(c, kb, a, W, H, p, K);
        const int rb = orc_bad_radius(K, h, c->bad_frac);
        for (int y = y0; y < y1; y++)
            for (int x = x0; x < x1; x++) {
                double s = 0.0;
                int dmin = h + 1;
                for (int v = -h; v <= h; v++)
                    for (int u = -h; u <= h; u++) {
                        const int xx = x - u, yy = y - v;
                        if (xx >= 0 && xx < W && yy >= 0 && yy < H && !Mk[(int64_t)yy * pitch + xx]) {
                            s += K[(v + h) * Kw + (u + h)] * (double)I[(int64_t)yy * pitch + xx];
                        } else {
                            const int dd = abs(u) > abs(v) ? abs(u) : abs(v);
                            if (dd < dmin) dmin = dd;
                        }
                    }
                out[(int64_t)y * pitch + x] = (float)s;
                out_mask[(int64_t)y * pitch + x] =
                    dmin <= rb ? ORC_MASK_CONV_BAD : (dmin <= h ? ORC_MASK_CONV_POOR : 0);
            }
        free(K);
    }
}

/*
 * The same two convolutions (Eqs. 12-13 with the BAD/POOR mask and the
 * covariance factor) restricted to the output rectangle [rx0, rx1) x
 * [ry0, ry1) of the full image: every output pixel is computed exactly as
 * by orc_convolve_image / orc_propagate_variance (same patch grid, same
 * spatial coordinates), so large images can be checked on samples.
 * out, out_mask and var_out are (rx1-rx0) x (ry1-ry0), row-major; NULL
 * outputs are skipped.
 */
void orc_convolve_region(const orc_config* c, const double* kb, const double* a, const float* I,
                         const float* V, const uint8_t* Mk, int W, int H, int64_t pitch,
                         const double* cov_in, int c_in, int rx0, int ry0, int rx1, int ry1,
                         float* out, uint8_t* out_mask, float* var_out) {
    const int h = c->h, Kw = 2 * h + 1, T = Kw * Kw, np = orc_n_patches(c, W, H);
    const int rw = rx1 - rx0;
#pragma omp parallel for schedule(dynamic)
    for (int p = 0; p < np; p++) {
        int x0, x1, y0, y1;
        patch_bounds(W, H, c->P, p, &x0, &x1, &y0, &y1);
        if (x1 <= rx0 || x0 >= rx1 || y1 <= ry0 || y0 >= ry1) continue;
        double* K = (double*)malloc(sizeof(double) * T);
        orc_patch_kernel(c, kb, a, W, H, p, K);
        const int rb = orc_bad_radius(K, h, c->bad_frac);
        const double f = orc_cov_factor(K, h, cov_in, c_in);
        for (int y = y0 > ry0 ? y0 : ry0; y < (y1 < ry1 ? y1 : ry1); y++)
            for (int x = x0 > rx0 ? x0 : rx0; x < (x1 < rx1 ? x1 : rx1); x++) {
                double s = 0.0, sv = 0.0;
                int dmin = h + 1;
                for (int v = -h; v <= h; v++)
                    for (int u = -h; u <= h; u++) {
                        const int xx = x - u, yy = y - v;
                        if (xx >= 0 && xx < W && yy >= 0 && yy < H && !Mk[(int64_t)yy * pitch + xx]) {
                            const double kk = K[(v + h) * Kw + (u + h)];
                            if (I) s += kk * (double)I[(int64_t)yy * pitch + xx];
                            if (V) sv += kk * kk * (double)V[(int64_t)yy * pitch + xx];
                        } else {
                            const int dd = abs(u) > abs(v) ? abs(u) : abs(v);
                            if (dd < dmin) dmin = dd;
                        }
                    }
                const int64_t o = (int64_t)(y - ry0) * rw + (x - rx0);
                if (out) out[o] = (float)s;
                if (out_mask)
                    out_mask[o] = dmin <= rb ? ORC_MASK_CONV_BAD : (dmin <= h ? ORC_MASK_CONV_POOR : 0);
                if (var_out) var_out[o] = (float)(f * sv);
            }
        free(K);
    }
}

/*
 * Variance propagation (Section 4.2, Eq. 13, and Section 4.3):
 *     V'(x, y) = f_p * sum_{u,v} K_p(u, v)^2 V~(x-u, y-v)
 * with V~ zero where masked or outside the image and f_p the covariance
 * factor of the patch kernel, moved into the variance map.
 * Image pseudo-matrix (Section 4.3): the mean of C' = raw / sum k^2 over the
 * kernels realised at the centres of a 3 x 3 partition of the image (reading
 * of "a much smaller array of kernels"), divided by its centre value (the
 * factor already applied to the variance), then cropped (or zero-padded) to
 * (2 c_out + 1)^2.  *discarded receives the fraction of sum |C| cut off.
 */
void orc_propagate_variance(const orc_config* c, const double* kb, const double* a, const float* V,
                            const uint8_t* Mk, int W, int H, int64_t pitch, const double* cov_in,
                            int c_in, float* var_out, double* cov_out, int c_out,
                            double* discarded) {
    const int h = c->h, Kw = 2 * h + 1, T = Kw * Kw, np = orc_n_patches(c, W, H);
#pragma omp parallel for schedule(dynamic)
    for (int p = 0; p < np; p++) {
        int x0, x1, y0, y1;
        double* K = (double*)malloc(sizeof(double) * T);
        patch_bounds(W, H, c->P, p, &x0, &x1, &y0, &y1);
        orc_patch_kernel(c, kb, a, W, H, p, K);
        const double f = orc_cov_factor(K, h, cov_in, c_in);
        for (int y = y0; y < y1; y++)
            for (int x = x0; x < x1; x++) {
                double s = 0.0;
                for (int v = -h; v <= h; v++)
                    for (int u = -h; u <= h; u++) {
                        const int xx = x - u, yy = y - v;
                        if (xx >= 0 && xx < W && yy >= 0 && yy < H && !Mk[(int64_t)yy * pitch + xx]) {
                            const double kk = K[(v + h) * Kw + (u + h)];
                            s += kk * kk * (double)V[(int64_t)yy * pitch + xx];
                        }
                    }
                var_out[(int64_t)y * pitch + x] = (float)(f * s);
            }
        free(K);
    }
    /* pseudo-matrix from a 3 x 3 sample of kernels */
    const int R = 2 * h + c_in, Rw = 2 * R + 1, Ow = 2 * c_out + 1;
    double* avg = (double*)calloc((size_t)Rw * Rw, sizeof(double));
    double* raw = (double*)malloc(sizeof(double) * Rw * Rw);
    double* K = (double*)malloc(sizeof(double) * T);
    for (int jy = 0; jy < 3; jy++)
        for (int jx = 0; jx < 3; jx++) {
            const int cx0 = jx * W / 3, cx1 = (jx + 1) * W / 3;
            const int cy0 = jy * H / 3, cy1 = (jy + 1) * H / 3;
            orc_kernel_at(c, kb, a, 0.5 * (cx0 + cx1 - 1), 0.5 * (cy0 + cy1 - 1), W, H, K);
            double s2 = 0.0;
            for (int t = 0; t < T; t++) s2 += K[t] * K[t];
            orc_cov_raw(K, h, cov_in, c_in, raw);
            for (int t = 0; t < Rw * Rw; t++) avg[t] += (s2 > 0.0 ? raw[t] / s2 : 0.0) / 9.0;
        }
    const double centre = avg[R * Rw + R];
    double tot = 0.0, kept = 0.0;
    for (int t = 0; t < Rw * Rw; t++) {
        avg[t] = centre != 0.0 ? avg[t] / centre : 0.0;
        tot += fabs(avg[t]);
    }
    for (int dy = -c_out; dy <= c_out; dy++)
        for (int dx = -c_out; dx <= c_out; dx++) {
            double val = 0.0;
            if (dx >= -R && dx <= R && dy >= -R && dy <= R) val = avg[(dy + R) * Rw + (dx + R)];
            cov_out[(dy + c_out) * Ow + (dx + c_out)] = val;
            kept += fabs(val);
        }
    if (discarded) *discarded = tot > 0.0 ? (tot - kept) / tot : 0.0;
    free(avg);
    free(raw);
    free(K);
}

/*
 * Difference image (Section 2 sign convention read as science minus model,
 * so new flux is positive; Section 4.3 for the noise):
 *     D = I2 - I1' - d0,  V_D = V2 + V1',
 *     mask_D = (M2 != 0 ? BAD : 0) | mask1';
 * at pixels masked in image 2 the difference and its variance are set to 0.
 * The pseudo-matrices are averaged with weights equal to the mean variance
 * of each input over its unmasked pixels (mask 0):
 *     C_D = (v2 C2 + v1' C1') / (v2 + v1'),
 * each zero-padded or cropped to (2 c_d + 1)^2; cov2 NULL is the
 * uncorrelated (unit centre) pseudo-matrix.
 */
void orc_subtract(const orc_config* c, const double* a, const float* I2, const float* V2,
                  const uint8_t* M2, const float* conv, const float* conv_var,
                  const uint8_t* conv_mask, int W, int H, int64_t pitch, const double* cov2,
                  int c2, const double* cov_conv, int cc, float* diff, float* diff_var,
                  uint8_t* diff_mask, double* cov_diff, int cd) {
    const int N = orc_n_unknowns(c);
    const double d0 = a[N - 1];
    double s2 = 0.0, sc = 0.0;
    long n2 = 0, nc = 0;
    for (int y = 0; y < H; y++)
        for (int x = 0; x < W; x++) {
            const int64_t o = (int64_t)y * pitch + x;
            if (M2[o]) {
                diff[o] = 0.0f;
                diff_var[o] = 0.0f;
                diff_mask[o] = ORC_MASK_BAD | conv_mask[o];
            } else {
                diff[o] = (float)((double)I2[o] - (double)conv[o] - d0);
                diff_var[o] = (float)((double)V2[o] + (double)conv_var[o]);
                diff_mask[o] = conv_mask[o];
                s2 += V2[o];
                n2++;
            }
            if (!conv_mask[o]) {
                sc += conv_var[o];
                nc++;
            }
        }
    const double v2 = n2 ? s2 / n2 : 0.0, vc = nc ? sc / nc : 0.0;
    const int Dw = 2 * cd + 1;
    for (int dy = -cd; dy <= cd; dy++)
        for (int dx = -cd; dx <= cd; dx++) {
            double a2 = 0.0, ac = 0.0;
            if (cov2) {
                if (abs(dx) <= c2 && abs(dy) <= c2) a2 = cov2[(dy + c2) * (2 * c2 + 1) + (dx + c2)];
            } else {
                a2 = (dx == 0 && dy == 0) ? 1.0 : 0.0;
            }
            if (abs(dx) <= cc && abs(dy) <= cc) ac = cov_conv[(dy + cc) * (2 * cc + 1) + (dx + cc)];
            cov_diff[(dy + cd) * Dw + (dx + cd)] = (v2 + vc) > 0.0 ? (v2 * a2 + vc * ac) / (v2 + vc) : 0.0;
        }
}

/* ------------------------------------------------------------------------
 * The paper's normalisation and quality mode (Sections 3.2, 3.3, 3.6, 3.7).
 */

#define ORC_STAMP_RESERVE 32   /* candidate held back to replace a rejected stamp */

/*
 * Unweighted sums of one stamp for the separate normalisation (Section 3.2,
 * sigma(x, y) = 1).  With A0 = k0 (x) I1 the flux-carrying column (the
 * unit-sum term the other terms were made zero-sum against):
 *   norm[5 s + 0] = npix,  [1] = sum A0,  [2] = sum I2,
 *   [3] = sum A0^2,        [4] = sum A0 I2
 * over the stamp pixels; zeros for stamps flagged on input (any bit except
 * ORC_STAMP_RESERVE, whose sums are kept for a later replacement).
 */
void orc_fit_norm(const orc_config* c, const double* kb, const float* I1, const float* I2, int W,
                  int H, int64_t pitch, const int32_t* xy, int n, const int32_t* flags,
                  double* norm) {
    const int h = c->h, r = c->r, K = 2 * h + 1;
    (void)W;
    (void)H;
#pragma omp parallel for schedule(dynamic)
    for (int s = 0; s < n; s++) {
        double* o = norm + 5 * (size_t)s;
        for (int k = 0; k < 5; k++) o[k] = 0.0;
        if (flags[s] & ~ORC_STAMP_RESERVE) continue;
        const int xc = xy[2 * s], yc = xy[2 * s + 1];
        for (int y = yc - r; y <= yc + r; y++)
            for (int x = xc - r; x <= xc + r; x++) {
                double a0 = 0.0;
                for (int v = -h; v <= h; v++)
                    for (int u = -h; u <= h; u++)
                        a0 += kb[(v + h) * K + (u + h)] * (double)I1[(int64_t)(y - v) * pitch + (x - u)];
                const double d = (double)I2[(int64_t)y * pitch + x];
                o[0] += 1.0;
                o[1] += a0;
                o[2] += d;
                o[3] += a0 * a0;
                o[4] += a0 * d;
            }
    }
}

/*
 * Normalisation b0 and background difference d0, spatially constant, from
 * the stamps in use (Section 3.2).  Reading: only b0 and d0 add flux, the
 * zero-sum terms move flux within a stamp, so over each stamp's aperture
 * the totals obey T2_s = b0 T1_s + d0 npix_s; b0 and d0 are the unweighted
 * least-squares fit of that relation over the stamps (sigma = 1, as in
 * aperture photometry).  Returns 0, or 1 if the 2 x 2 system is singular.
 */
int orc_norm_solve(int n, const double* norm, const uint8_t* used, double* b0, double* d0) {
    double saa = 0.0, san = 0.0, snn = 0.0, sad = 0.0, snd = 0.0;
    for (int s = 0; s < n; s++) {
        if (!used[s]) continue;
        const double np = norm[5 * s], t1 = norm[5 * s + 1], t2 = norm[5 * s + 2];
        saa += t1 * t1;
        san += t1 * np;
        snn += np * np;
        sad += t1 * t2;
        snd += np * t2;
    }
    const double det = saa * snn - san * san;
    if (!(det > 1e-12 * saa * snn)) {
        *b0 = 0.0;
        *d0 = 0.0;
        return 1;
    }
    *b0 = (sad * snn - san * snd) / det;
    *d0 = (saa * snd - san * sad) / det;
    return 0;
}

/*
 * Solution in the paper's normalisation mode (Sections 3.2, 3.3): at each
 * iteration b0 and d0 come from orc_norm_solve over the stamps in use; the
 * weighted equations of the other unknowns are then solved with b0 and d0
 * held: unknown 0 (term 0, spatial term 0) = b0, the higher spatial terms of
 * term 0 = 0 (the normalisation is spatially constant), the background =
 * d0, and for the free unknowns f
 *     M_ff a_f = b_f - M_fc a_c
 * (c the held unknowns), solved by orc_cholesky_solve.  The rejection is
 * orc_solve's.  Replacement (Section 3.3, "removed (and replaced, if
 * possible)"): with group non-NULL, each stamp rejected in a round is
 * replaced by the lowest-index stamp of the same group (group >= 0) that is
 * held in reserve (flags == ORC_STAMP_RESERVE on input); it enters the next
 * solution.  stats as orc_solve, with dof = sum npix - (free unknowns + 2);
 * *n_replaced counts replacements.  Returns 0, -3, -4, or -8 (singular
 * normalisation).
 */
int orc_solve_norm(const orc_config* c, int W, int H, const int32_t* xy, int n, const double* Ms,
                   const double* bs, const double* es, const int32_t* npix, const double* norm,
                   const int32_t* group, int32_t* flags, double* coeffs, double* chi2,
                   orc_stats* st, int* n_replaced) {
    const int nb = orc_n_basis(c), ns = orc_n_spatial(c), N = nb * ns + 1, L = nb + 1;
    uint8_t* used = (uint8_t*)calloc(n > 0 ? n : 1, 1);
    uint8_t* fitted = (uint8_t*)calloc(n > 0 ? n : 1, 1);
    uint8_t* held = (uint8_t*)calloc(N, 1);
    int* fidx = (int*)malloc(sizeof(int) * N);
    double* M = (double*)malloc(sizeof(double) * (size_t)N * N);
    double* b = (double*)malloc(sizeof(double) * N);
    double* Mf = (double*)malloc(sizeof(double) * (size_t)N * N);
    double* bf = (double*)malloc(sizeof(double) * N);
    double* af = (double*)malloc(sizeof(double) * N);
    int ret = 0, iter = 0, n_rej = 0, n_rep = 0;
    memset(st, 0, sizeof(*st));
    for (int s = 0; s < n; s++) {
        used[s] = flags[s] == 0;
        fitted[s] = used[s];
        chi2[s] = 0.0;
    }
    for (int t = 0; t < ns; t++) held[0 * ns + t] = 1;
    held[N - 1] = 1;
    int nf = 0;
    for (int i = 0; i < N; i++)
        if (!held[i]) fidx[nf++] = i;
    for (int i = 0; i < N; i++) coeffs[i] = 0.0;
    for (;;) {
        int n_used = 0;
        for (int s = 0; s < n; s++) n_used += used[s];
        if (n_used < c->min_stamps) { ret = -3; st->info = -3; break; }
        double b0, d0;
        if (orc_norm_solve(n, norm, used, &b0, &d0)) { ret = -8; st->info = -8; break; }
        orc_assemble(c, W, H, xy, n, Ms, bs, used, M, b);
        for (int i = 0; i < N; i++) coeffs[i] = 0.0;
        coeffs[0] = b0;
        coeffs[N - 1] = d0;
        for (int p = 0; p < nf; p++) {
            const int i = fidx[p];
            double t = b[i];
            for (int j = 0; j < N; j++)
                if (held[j]) t -= M[(size_t)i * N + j] * coeffs[j];
            bf[p] = t;
            for (int q = 0; q < nf; q++) Mf[(size_t)p * nf + q] = M[(size_t)i * N + fidx[q]];
        }
        int info = orc_cholesky_solve(nf, Mf, bf, af);
        if (info) { ret = -4; st->info = fidx[info - 1] + 1; break; }
        for (int p = 0; p < nf; p++) coeffs[fidx[p]] = af[p];
        iter++;
        for (int s = 0; s < n; s++)
            chi2[s] = fitted[s] ? orc_stamp_chi2(c, coeffs, W, H, xy[2 * s], xy[2 * s + 1],
                                                  Ms + (size_t)s * L * L, bs + (size_t)s * L, es[s])
                                : 0.0;
        if (iter >= c->max_iter) break;
        double mean = 0.0, var = 0.0;
        for (int s = 0; s < n; s++)
            if (used[s]) mean += chi2[s] / npix[s];
        mean /= n_used;
        for (int s = 0; s < n; s++)
            if (used[s]) {
                const double dq = chi2[s] / npix[s] - mean;
                var += dq * dq;
            }
        const double thr = mean + c->clip_sigma * sqrt(var / n_used);
        int n_new = 0;
        for (int s = 0; s < n; s++)
            if (used[s] && chi2[s] / npix[s] > thr) n_new++;
        if (n_new == 0 || n_used - n_new < c->min_stamps) break;
        for (int s = 0; s < n; s++)
            if (used[s] && chi2[s] / npix[s] > thr) {
                used[s] = 0;
                flags[s] |= ORC_STAMP_REJECTED;
                n_rej++;
                if (group && group[s] >= 0)
                    for (int q = 0; q < n; q++)
                        if (group[q] == group[s] && flags[q] == ORC_STAMP_RESERVE) {
                            flags[q] = 0;
                            used[q] = 1;
                            fitted[q] = 1;
                            n_rep++;
                            break;
                        }
            }
    }
    st->n_iter = iter;
    st->n_rejected = n_rej;
    *n_replaced = n_rep;
    if (ret != 0)
        for (int i = 0; i < N; i++) coeffs[i] = 0.0;
    if (ret == 0) {
        double c2 = 0.0, np = 0.0;
        int nu = 0;
        for (int s = 0; s < n; s++)
            if (used[s]) { c2 += chi2[s]; np += npix[s]; nu++; }
        st->chi2 = c2;
        st->dof = np - (nf + 2);
        st->chi2_dof = c2 / (np - (nf + 2));
        st->n_used = nu;
        st->kernel_sum_centre = coeffs[0];
    }
    free(used); free(fitted); free(held); free(fidx); free(M); free(b); free(Mf); free(bf);
    free(af);
    return ret;
}

/* Quality record of a subtraction (Sections 3.6 and 3.7). */
typedef struct {
    double dev_mean, dev_rms;         /* normalised mean deviation, r.m.s. deviation */
    double kernel_sum, mom_x, mom_y, mom_xx, mom_yy, deconv_max;
    int n_used, cut_flags;
} orc_quality;

/* cut bits (Section 3.7's recommended cuts) */
#define ORC_CUT_FEW_STAMPS 1     /* number of stamps used < 3 */
#define ORC_CUT_MEAN_DEV   2     /* normalised mean deviation > 0.5 */
#define ORC_CUT_RMS_DEV    4     /* normalised r.m.s. deviation > 0.3 */
#define ORC_CUT_MOMENT1    8     /* a first moment (x, y) of the kernel > 0.5 in size */
#define ORC_CUT_MOMENT2   16     /* a second moment (xx, yy) of the kernel < 0 */
#define ORC_CUT_DECONV    32     /* maximum deconvolution fraction > 1.03 */

/*
 * Quality of a solution (Section 3.6).
 * Per used stamp (flags == 0), the residual of the solution applied there --
 * the kernel realised at the stamp centre convolved with I1 plus the
 * background, subtracted from I2 -- divided by the variance softened with a
 * scaled flux:  dev_s = (1/npix) sum (I2 - m)^2 / (V2 + soft |m|),
 * m = K_s (x) I1 + d0 (reading: "a scaled version of the flux" is soft
 * times the model flux of the pixel; soft = 0 gives chi2_s / npix_s).
 * dev[s] receives dev_s (0 for unused stamps).  Over the used stamps:
 * dev_mean = mean(dev_s) - 1 (excess over pure noise) and dev_rms =
 * population std of dev_s (readings of the "normalised" mean and r.m.s.
 * deviations).  At the image centre: the kernel sum, first moments
 * (sum u K / sum K, sum v K / sum K), second central moments, and the
 * maximum over radii rho = 0 .. ceil(h sqrt 2) of the deconvolution
 * fraction sum_{u^2 + v^2 <= rho^2} K / sum K.  cut_flags: the bits above.
 */
void orc_quality_eval(const orc_config* c, const double* kb, const double* a, const float* I1,
                      const float* I2, const float* V2, int W, int H, int64_t pitch,
                      const int32_t* xy, int n, const int32_t* flags, double soft, double* dev,
                      orc_quality* q) {
    const int h = c->h, r = c->r, Kw = 2 * h + 1, T = Kw * Kw, N = orc_n_unknowns(c);
    const double d0 = a[N - 1];
#pragma omp parallel for schedule(dynamic)
    for (int s = 0; s < n; s++) {
        dev[s] = 0.0;
        if (flags[s]) continue;
        const int xc = xy[2 * s], yc = xy[2 * s + 1];
        double* K = (double*)malloc(sizeof(double) * T);
        orc_kernel_at(c, kb, a, xc, yc, W, H, K);
        double acc = 0.0;
        int np = 0;
        for (int y = yc - r; y <= yc + r; y++)
            for (int x = xc - r; x <= xc + r; x++) {
                double m = d0;
                for (int v = -h; v <= h; v++)
                    for (int u = -h; u <= h; u++)
                        m += K[(v + h) * Kw + (u + h)] * (double)I1[(int64_t)(y - v) * pitch + (x - u)];
                const double res = (double)I2[(int64_t)y * pitch + x] - m;
                acc += res * res / ((double)V2[(int64_t)y * pitch + x] + soft * fabs(m));
                np++;
            }
        dev[s] = acc / np;
        free(K);
    }
    double sm = 0.0, sv = 0.0;
    int nu = 0;
    for (int s = 0; s < n; s++)
        if (!flags[s]) { sm += dev[s]; nu++; }
    const double mean = nu ? sm / nu : 0.0;
    for (int s = 0; s < n; s++)
        if (!flags[s]) sv += (dev[s] - mean) * (dev[s] - mean);
    q->n_used = nu;
    q->dev_mean = nu ? mean - 1.0 : 0.0;
    q->dev_rms = nu ? sqrt(sv / nu) : 0.0;
    double* K = (double*)malloc(sizeof(double) * T);
    orc_kernel_at(c, kb, a, 0.5 * (W - 1), 0.5 * (H - 1), W, H, K);
    double s0 = 0.0, su = 0.0, sv1 = 0.0;
    for (int v = -h; v <= h; v++)
        for (int u = -h; u <= h; u++) {
            const double k = K[(v + h) * Kw + (u + h)];
            s0 += k;
            su += u * k;
            sv1 += v * k;
        }
    q->kernel_sum = s0;
    q->mom_x = su / s0;
    q->mom_y = sv1 / s0;
    double sxx = 0.0, syy = 0.0;
    for (int v = -h; v <= h; v++)
        for (int u = -h; u <= h; u++) {
            const double k = K[(v + h) * Kw + (u + h)];
            sxx += (u - q->mom_x) * (u - q->mom_x) * k;
            syy += (v - q->mom_y) * (v - q->mom_y) * k;
        }
    q->mom_xx = sxx / s0;
    q->mom_yy = syy / s0;
    const int rmax = (int)ceil(h * sqrt(2.0));
    double best = -1e300;
    for (int rho = 0; rho <= rmax; rho++) {
        double e = 0.0;
        for (int v = -h; v <= h; v++)
            for (int u = -h; u <= h; u++)
                if (u * u + v * v <= rho * rho) e += K[(v + h) * Kw + (u + h)];
        if (e / s0 > best) best = e / s0;
    }
    q->deconv_max = best;
    free(K);
    int f = 0;
    if (q->n_used < 3) f |= ORC_CUT_FEW_STAMPS;
    if (q->dev_mean > 0.5) f |= ORC_CUT_MEAN_DEV;
    if (q->dev_rms > 0.3) f |= ORC_CUT_RMS_DEV;
    if (fabs(q->mom_x) > 0.5 || fabs(q->mom_y) > 0.5) f |= ORC_CUT_MOMENT1;
    if (q->mom_xx < 0.0 || q->mom_yy < 0.0) f |= ORC_CUT_MOMENT2;
    if (q->deconv_max > 1.03) f |= ORC_CUT_DECONV;
    q->cut_flags = f;
}

/* ------------------------------------------------------------------------
 * Noise-model operations beyond convolution (Section 4.3, "Use in practise").
 */

/*
 * Binning by an integer factor B (Section 4.3): a convolution with a
 * constant B x B kernel followed by a change of scale.  Output pixel (X, Y)
 * of the (W / B) x (H / B) image (partial blocks at the right and bottom
 * edges dropped) is the sum over its block; pixels masked in the input
 * contribute nothing and set the output mask (OR of the block's masks).
 * With the box kernel k = 1 the convolution rules give
 *     raw(D) = sum_{u,u' in block} C_in(D + u - u')  (pseudo-matrix of the sum),
 *     V_b = f * sum_block V,   f = raw(0) / B^2  (covariance factor moved in),
 * and the change of scale samples the pseudo-matrix at multiples of B:
 *     C_b(D) = raw(B D) / raw(0),  |D| <= c_out per axis.
 * cov_in: (2 c_in + 1)^2, NULL = uncorrelated.  Output planes have pitch
 * W / B.  *discarded: share of sum |raw(B D) / raw(0)| cut off by the crop.
 */
void orc_bin(const float* I, const float* V, const uint8_t* Mk, int W, int H, int64_t pitch, int B,
             const double* cov_in, int c_in, float* Ib, float* Vb, uint8_t* Mb, double* cov_out,
             int c_out, double* discarded) {
    const int Wb = W / B, Hb = H / B, Cw = 2 * c_in + 1;
    /* raw pseudo-matrix of the block sum at fine offsets |D| <= (B-1) + c_in */
    const int R = B - 1 + c_in, Rw = 2 * R + 1;
    double* raw = (double*)calloc((size_t)Rw * Rw, sizeof(double));
    for (int dy = -R; dy <= R; dy++)
        for (int dx = -R; dx <= R; dx++) {
            double s = 0.0;
            for (int v = 0; v < B; v++)
                for (int u = 0; u < B; u++)
                    for (int v2 = 0; v2 < B; v2++)
                        for (int u2 = 0; u2 < B; u2++) {
                            const int wx = dx + u - u2, wy = dy + v - v2;
                            if (wx < -c_in || wx > c_in || wy < -c_in || wy > c_in) continue;
                            s += cov_in ? cov_in[(wy + c_in) * Cw + (wx + c_in)]
                                        : (wx == 0 && wy == 0 ? 1.0 : 0.0);
                        }
            raw[(dy + R) * Rw + (dx + R)] = s;
        }
    const double raw0 = raw[R * Rw + R];
    const double f = raw0 / ((double)B * B);
    for (int Y = 0; Y < Hb; Y++)
        for (int X = 0; X < Wb; X++) {
            double si = 0.0, sv = 0.0;
            uint8_t m = 0;
            for (int v = 0; v < B; v++)
                for (int u = 0; u < B; u++) {
                    const int64_t o = (int64_t)(B * Y + v) * pitch + (B * X + u);
                    if (Mk[o]) {
                        m = 1;
                    } else {
                        si += I[o];
                        sv += V[o];
                    }
                }
            Ib[(int64_t)Y * Wb + X] = (float)si;
            Vb[(int64_t)Y * Wb + X] = (float)(f * sv);
            Mb[(int64_t)Y * Wb + X] = m;
        }
    /* coarse pseudo-matrix: raw at multiples of B, normalised to the centre */
    const int Rc = R / B, Ow = 2 * c_out + 1;
    double tot = 0.0, kept = 0.0;
    for (int DY = -Rc; DY <= Rc; DY++)
        for (int DX = -Rc; DX <= Rc; DX++) tot += fabs(raw[(B * DY + R) * Rw + (B * DX + R)] / raw0);
    for (int DY = -c_out; DY <= c_out; DY++)
        for (int DX = -c_out; DX <= c_out; DX++) {
            double val = 0.0;
            if (abs(DX) <= Rc && abs(DY) <= Rc) val = raw[(B * DY + R) * Rw + (B * DX + R)] / raw0;
            cov_out[(DY + c_out) * Ow + (DX + c_out)] = val;
            kept += fabs(val);
        }
    if (discarded) *discarded = tot > 0.0 ? (tot - kept) / tot : 0.0;
    free(raw);
}

/*
 * Resampling of a pseudo-matrix to a new pixel scale (Section 4.3): an
 * output pixel spans `scale` input pixels, so output offset D samples the
 * input pseudo-matrix at scale * D by bilinear interpolation (zero beyond
 * its extent).  The centre stays 1 (zero offset is a grid point); the
 * off-centre entries are then scaled together so that their sum -- the
 * total covariance excluding the variance -- equals the input's.
 * cov_in (2 c_in + 1)^2 with centre 1; cov_out (2 c_out + 1)^2.
 */
void orc_resample_cov(const double* cov_in, int c_in, double scale, double* cov_out, int c_out) {
    const int Cw = 2 * c_in + 1, Ow = 2 * c_out + 1;
    double tin = 0.0, tout = 0.0;
    for (int t = 0; t < Cw * Cw; t++)
        if (t != c_in * Cw + c_in) tin += cov_in[t];
    for (int DY = -c_out; DY <= c_out; DY++)
        for (int DX = -c_out; DX <= c_out; DX++) {
            const double x = scale * DX, y = scale * DY;
            const double fx = floor(x), fy = floor(y);
            const double tx = x - fx, ty = y - fy;
            double val = 0.0;
            for (int j = 0; j < 2; j++)
                for (int i = 0; i < 2; i++) {
                    const int px = (int)fx + i, py = (int)fy + j;
                    if (px < -c_in || px > c_in || py < -c_in || py > c_in) continue;
                    const double w = (i ? tx : 1.0 - tx) * (j ? ty : 1.0 - ty);
                    val += w * cov_in[(py + c_in) * Cw + (px + c_in)];
                }
            cov_out[(DY + c_out) * Ow + (DX + c_out)] = val;
            if (DX != 0 || DY != 0) tout += val;
        }
    const double a = tout != 0.0 ? tin / tout : 0.0;
    for (int DY = -c_out; DY <= c_out; DY++)
        for (int DX = -c_out; DX <= c_out; DX++)
            if (DX != 0 || DY != 0) cov_out[(DY + c_out) * Ow + (DX + c_out)] *= a;
}

/*
 * Weighted sum of two images (Section 4.3, adding or subtracting images):
 *     S = alpha Ia + beta Ib,  V_S = alpha^2 Va + beta^2 Vb,
 *     mask_S = mask_a | mask_b (S and V_S are 0 where it is set),
 *     C_S = (wa Ca + wb Cb) / (wa + wb),  wa = alpha^2 mean(Va),
 *     wb = beta^2 mean(Vb)
 * with the means over each image's unmasked pixels (the weights of the
 * weighted average are the average variances of the two terms).  Ca, Cb
 * ((2 ca + 1)^2, (2 cb + 1)^2; NULL = uncorrelated) are zero-padded or
 * cropped to (2 cs + 1)^2.
 */
void orc_add_images(double alpha, const float* Ia, const float* Va, const uint8_t* Ma,
                    const double* Ca, int ca, double beta, const float* Ib, const float* Vb,
                    const uint8_t* Mb, const double* Cb, int cb, int W, int H, int64_t pitch,
                    float* S, float* VS, uint8_t* MS, double* CS, int cs) {
    double sa = 0.0, sb = 0.0;
    long na = 0, nbp = 0;
    for (int y = 0; y < H; y++)
        for (int x = 0; x < W; x++) {
            const int64_t o = (int64_t)y * pitch + x;
            if (!Ma[o]) { sa += Va[o]; na++; }
            if (!Mb[o]) { sb += Vb[o]; nbp++; }
            const uint8_t m = (uint8_t)(Ma[o] | Mb[o]);
            MS[o] = m;
            if (m) {
                S[o] = 0.0f;
                VS[o] = 0.0f;
            } else {
                S[o] = (float)(alpha * (double)Ia[o] + beta * (double)Ib[o]);
                VS[o] = (float)(alpha * alpha * (double)Va[o] + beta * beta * (double)Vb[o]);
            }
        }
    const double wa = alpha * alpha * (na ? sa / na : 0.0), wb = beta * beta * (nbp ? sb / nbp : 0.0);
    const int Sw = 2 * cs + 1;
    for (int dy = -cs; dy <= cs; dy++)
        for (int dx = -cs; dx <= cs; dx++) {
            double va, vb;
            if (Ca) va = (abs(dx) <= ca && abs(dy) <= ca) ? Ca[(dy + ca) * (2 * ca + 1) + (dx + ca)] : 0.0;
            else va = (dx == 0 && dy == 0) ? 1.0 : 0.0;
            if (Cb) vb = (abs(dx) <= cb && abs(dy) <= cb) ? Cb[(dy + cb) * (2 * cb + 1) + (dx + cb)] : 0.0;
            else vb = (dx == 0 && dy == 0) ? 1.0 : 0.0;
            CS[(dy + cs) * Sw + (dx + cs)] = (wa + wb) > 0.0 ? (wa * va + wb * vb) / (wa + wb) : 0.0;
        }
}

/* ------------------------------------------------------------------------
 * PSF homogenisation for stacking (Section 5.1).
 */

/*
 * Envelope PSF (Section 5.1): each input PSF, an elliptical Gaussian
 * (params[3 k + 0..2] = sigma_major, sigma_minor, angle), is realised in a
 * circular version with a common peak of 1 -- reading: the circular Gaussian
 * of the major-axis width, so that it contains the input PSF -- on the grid
 * |u|, |v| <= half; env[] receives the pixel-by-pixel maximum over the
 * inputs, and the envelope model is the circular Gaussian of peak 1 fitted
 * to it by least squares over its width: golden-section search of
 * sum (env - exp(-r^2 / 2 s^2))^2 over s in [0.1, 2 max sigma_major] to a
 * bracket of 1e-10 px.  Returns the fitted width.
 */
static double env_misfit(const double* env, int half, double s) {
    const int Ew = 2 * half + 1;
    double q = 0.0;
    for (int v = -half; v <= half; v++)
        for (int u = -half; u <= half; u++) {
            const double d = env[(v + half) * Ew + (u + half)] - exp(-(double)(u * u + v * v) / (2.0 * s * s));
            q += d * d;
        }
    return q;
}

double orc_envelope_psf(const double* params, int n, int half, double* env) {
    const int Ew = 2 * half + 1;
    double smax = 0.0;
    for (int k = 0; k < n; k++)
        if (params[3 * k] > smax) smax = params[3 * k];
    for (int v = -half; v <= half; v++)
        for (int u = -half; u <= half; u++) {
            double m = 0.0;
            for (int k = 0; k < n; k++) {
                const double s = params[3 * k];
                const double g = exp(-(double)(u * u + v * v) / (2.0 * s * s));
                if (g > m) m = g;
            }
            env[(v + half) * Ew + (u + half)] = m;
        }
    const double gr = 0.5 * (sqrt(5.0) - 1.0);
    double a = 0.1, b = 2.0 * smax;
    double c = b - gr * (b - a), d = a + gr * (b - a);
    double fc = env_misfit(env, half, c), fd = env_misfit(env, half, d);
    while (b - a > 1e-10) {
        if (fc < fd) {
            b = d; d = c; fd = fc;
            c = b - gr * (b - a);
            fc = env_misfit(env, half, c);
        } else {
            a = c; c = d; fc = fd;
            d = a + gr * (b - a);
            fd = env_misfit(env, half, d);
        }
    }
    return 0.5 * (a + b);
}

/*
 * Fake target image (Section 5.1): the envelope PSF, a circular Gaussian of
 * width sigma and unit flux sampled at pixel centres, placed at the known
 * source positions with their fluxes (src[3 s + 0..2] = x, y, flux), each
 * within a box of half-width ceil(6 sigma) + 1 around floor(x), floor(y);
 * sums in source order.
 */
void orc_render_target(const double* src, int n, double sigma, int W, int H, int64_t pitch,
                       float* out) {
    const int rad = (int)ceil(6.0 * sigma) + 1;
    double* acc = (double*)calloc((size_t)W * H, sizeof(double));
    const double norm = 1.0 / (2.0 * 3.14159265358979323846 * sigma * sigma);
    for (int s = 0; s < n; s++) {
        const double x0 = src[3 * s], y0 = src[3 * s + 1], f = src[3 * s + 2];
        const int xi = (int)floor(x0), yi = (int)floor(y0);
        for (int y = yi - rad; y <= yi + rad; y++)
            for (int x = xi - rad; x <= xi + rad; x++) {
                if (x < 0 || x >= W || y < 0 || y >= H) continue;
                const double dx = x - x0, dy = y - y0;
                acc[(size_t)y * W + x] += f * norm * exp(-(dx * dx + dy * dy) / (2.0 * sigma * sigma));
            }
    }
    for (int y = 0; y < H; y++)
        for (int x = 0; x < W; x++) out[(int64_t)y * pitch + x] = (float)acc[(size_t)y * W + x];
    free(acc);
}

/*
 * Outlier pixels across n PSF-homogenised inputs (Section 5.1); plane k of
 * each array starts at k * plane (elements).  At each pixel the inputs not
 * masked there are compared with their median (the mean of the two middle
 * values for an even count); input k is an outlier if
 * |I_k - median| > nsigma sqrt(V_k).  Fewer than 3 unmasked inputs: none is.
 * out[k] = 1 for outliers, else 0.
 */
static int cmp_double(const void* a, const void* b) {
    const double x = *(const double*)a, y = *(const double*)b;
    return (x > y) - (x < y);
}

void orc_stack_reject(int n, const float* I, const float* V, const uint8_t* Mk, int64_t plane,
                      int W, int H, int64_t pitch, double nsigma, uint8_t* out) {
    double vals[64];
    for (int y = 0; y < H; y++)
        for (int x = 0; x < W; x++) {
            const int64_t o = (int64_t)y * pitch + x;
            int m = 0;
            for (int k = 0; k < n; k++) {
                out[k * plane + o] = 0;
                if (!Mk[k * plane + o]) vals[m++] = I[k * plane + o];
            }
            if (m < 3) continue;
            qsort(vals, m, sizeof(double), cmp_double);
            const double med = (m % 2) ? vals[m / 2] : 0.5 * (vals[m / 2 - 1] + vals[m / 2]);
            for (int k = 0; k < n; k++) {
                const int64_t q = k * plane + o;
                if (Mk[q]) continue;
                if (fabs((double)I[q] - med) > nsigma * sqrt((double)V[q])) out[q] = 1;
            }
        }
}

/*
 * Back from outliers on a convolved image to bad pixels of the original
 * (Section 5.1): the outlier mask is correlated with the magnitude of the
 * kernel applied there -- the matched filter, the adjoint of the
 * convolution, so pixel x collects the outlier flags of the convolved pixels
 * x + u it contributed to with weight |K_p(u)| -- and x is bad if that
 * collects at least frac of sum |K_p|; K_p is the patch kernel of x's
 * patch.  Outside the image counts as no outlier.
 */
void orc_trace_mask(const orc_config* c, const double* kb, const double* a, const uint8_t* outl,
                    int W, int H, int64_t pitch, double frac, uint8_t* bad) {
    const int h = c->h, Kw = 2 * h + 1, T = Kw * Kw, np = orc_n_patches(c, W, H);
#pragma omp parallel for schedule(dynamic)
    for (int p = 0; p < np; p++) {
        int x0, x1, y0, y1;
        patch_bounds(W, H, c->P, p, &x0, &x1, &y0, &y1);
        double* K = (double*)malloc(sizeof(double) * T);
        orc_patch_kernel(c, kb, a, W, H, p, K);
        double tot = 0.0;
        for (int t = 0; t < T; t++) tot += fabs(K[t]);
        for (int y = y0; y < y1; y++)
            for (int x = x0; x < x1; x++) {
                double s = 0.0;
                for (int v = -h; v <= h; v++)
                    for (int u = -h; u <= h; u++) {
                        const int xx = x + u, yy = y + v;
                        if (xx < 0 || xx >= W || yy < 0 || yy >= H) continue;
                        if (outl[(int64_t)yy * pitch + xx]) s += fabs(K[(v + h) * Kw + (u + h)]);
                    }
                bad[(int64_t)y * pitch + x] = s >= frac * tot && s > 0.0;
            }
        free(K);
    }
}

/*
 * Weighted combination of n homogenised inputs (Section 5.2): weights
 * w_k = 1 / mean(V_k) over each input's pixels with mask 0 (reading of
 * "weights set to the mean variance": inverse-variance weights);
 *     S = sum_k w_k I_k / sum_k w_k,  V_S = sum_k w_k^2 V_k / (sum_k w_k)^2
 * over the inputs with mask 0 at the pixel; none: S = V_S = 0, MS = 1.
 * Pseudo-matrix: the variance-weighted average of the inputs' (each
 * (2 ck + 1)^2, all the same size, in one array of n (2 ck + 1)^2 values)
 * with weights w_k^2 mean(V_k).  weights_out (nullable) receives the w_k.
 */
void orc_stack_combine(int n, const float* I, const float* V, const uint8_t* Mk, int64_t plane,
                       int W, int H, int64_t pitch, const double* C, int ck, float* S, float* VS,
                       uint8_t* MS, double* CS, double* weights_out) {
    double w[64], vbar[64];
    for (int k = 0; k < n; k++) {
        double sv = 0.0;
        long cnt = 0;
        for (int y = 0; y < H; y++)
            for (int x = 0; x < W; x++) {
                const int64_t q = k * plane + (int64_t)y * pitch + x;
                if (!Mk[q]) { sv += V[q]; cnt++; }
            }
        vbar[k] = cnt ? sv / cnt : 0.0;
        w[k] = vbar[k] > 0.0 ? 1.0 / vbar[k] : 0.0;
        if (weights_out) weights_out[k] = w[k];
    }
    for (int y = 0; y < H; y++)
        for (int x = 0; x < W; x++) {
            const int64_t o = (int64_t)y * pitch + x;
            double sw = 0.0, si = 0.0, sv = 0.0;
            for (int k = 0; k < n; k++) {
                const int64_t q = k * plane + o;
                if (Mk[q]) continue;
                sw += w[k];
                si += w[k] * (double)I[q];
                sv += w[k] * w[k] * (double)V[q];
            }
            if (sw > 0.0) {
                S[o] = (float)(si / sw);
                VS[o] = (float)(sv / (sw * sw));
                MS[o] = 0;
            } else {
                S[o] = 0.0f;
                VS[o] = 0.0f;
                MS[o] = 1;
            }
        }
    const int Cw = 2 * ck + 1;
    double tw = 0.0;
    for (int k = 0; k < n; k++) tw += w[k] * w[k] * vbar[k];
    for (int t = 0; t < Cw * Cw; t++) {
        double s = 0.0;
        for (int k = 0; k < n; k++) s += w[k] * w[k] * vbar[k] * C[(size_t)k * Cw * Cw + t];
        CS[t] = tw > 0.0 ? s / tw : 0.0;
    }
}

/* ------------------------------------------------------------------------
 * Matching both images to a common PSF (Section 2, Eqs. 1-4 with the
 * penalty of Eq. 9).
 *
 * Unknowns a = (b, c, d0): b the nb kernel terms of K1 with their spatial
 * polynomials (b[i * ns + s], exactly the single form's kernel unknowns),
 * c the zero-sum terms i = 1..nb-1 of the kernel applied to I2, with the
 * same spatial polynomials (c[(i - 1) * ns + s] at offset nb ns), and the
 * constant background d0 last: N2 = (2 nb - 1) ns + 1.  Model of I2:
 *     sum_i b_i g k_i (x) I1 + sum_{i>=1} c_i g k_i (x) I2 + d0,
 * so that K1 (x) I1 + d0 = K2 (x) I2 with K2 = delta - sum_{i>=1} c_i g k_i
 * (unit sum, as every k_i with i >= 1 sums to zero).
 */

int orc_dual_unknowns(const orc_config* c) {
    return (2 * orc_n_basis(c) - 1) * orc_n_spatial(c) + 1;
}

/*
 * Per-stamp sums of the two-kernel form: columns A = (k_i (x) I1 for
 * i = 0..nb-1, k_i (x) I2 for i = 1..nb-1, 1), L2 = 2 nb, weights 1 / V2
 * (1 / (V1 + V2) when V1 is given, as in orc_fit_stamps):
 * M_s = A^T W A (L2 x L2), b_s = A^T W I2, e_s = I2^T W I2 over the stamp
 * pixels.  Validity as for the single form, with I2 (and its mask) now
 * also required over the convolution footprint [x-r-h, x+r+h]^2.
 */
void orc_fit_dual(const orc_config* c, const double* kb, const float* I1, const uint8_t* M1,
                  const float* I2, const float* V2, const uint8_t* M2, int W, int H,
                  int64_t pitch, const int32_t* xy, int n, double* Ms, double* bs, double* es,
                  int32_t* npix, int32_t* flags, const float* V1) {
    const int nb = orc_n_basis(c), L = 2 * nb, h = c->h, r = c->r, K = 2 * h + 1, T = K * K;
#pragma omp parallel for schedule(dynamic)
    for (int s = 0; s < n; s++) {
        const int xc = xy[2 * s], yc = xy[2 * s + 1], R = r + h;
        double* M = Ms + (size_t)s * L * L;
        double* b = bs + (size_t)s * L;
        int flag = 0;
        memset(M, 0, sizeof(double) * L * L);
        memset(b, 0, sizeof(double) * L);
        es[s] = 0.0;
        npix[s] = 0;
        if (xc - R < 0 || yc - R < 0 || xc + R >= W || yc + R >= H) {
            flag |= ORC_STAMP_INVALID;
        } else {
            for (int y = yc - R; y <= yc + R; y++)
                for (int x = xc - R; x <= xc + R; x++)
                    if (M1[y * pitch + x] || M2[y * pitch + x]) flag |= ORC_STAMP_INVALID;
            if (!flag) {
                for (int y = yc - R; y <= yc + R; y++)
                    for (int x = xc - R; x <= xc + R; x++)
                        if (!isfinite(I1[y * pitch + x]) || !isfinite(I2[y * pitch + x]))
                            flag |= ORC_STAMP_NONFINITE;
                for (int y = yc - r; y <= yc + r; y++)
                    for (int x = xc - r; x <= xc + r; x++) {
                        const float v2 = weight_var(V1, V2, y * pitch + x);
                        if (!isfinite(v2) || !(v2 > 0.0f)) flag |= ORC_STAMP_NONFINITE;
                    }
            }
        }
        flags[s] = flag;
        if (flag) continue;
        double* A = (double*)malloc(sizeof(double) * L);
        for (int y = yc - r; y <= yc + r; y++) {
            for (int x = xc - r; x <= xc + r; x++) {
                for (int i = 0; i < nb; i++) {
                    const double* ki = kb + (size_t)i * T;
                    double a1 = 0.0, a2 = 0.0;
                    for (int v = -h; v <= h; v++)
                        for (int u = -h; u <= h; u++) {
                            const int64_t o = (int64_t)(y - v) * pitch + (x - u);
                            const double k = ki[(v + h) * K + (u + h)];
                            a1 += k * (double)I1[o];
                            a2 += k * (double)I2[o];
                        }
                    A[i] = a1;
                    if (i >= 1) A[nb + i - 1] = a2;
                }
                A[L - 1] = 1.0;
                const double w = 1.0 / (double)weight_var(V1, V2, y * pitch + x);
                const double d = (double)I2[y * pitch + x];
                for (int i = 0; i < L; i++) {
                    for (int j = 0; j < L; j++) M[i * L + j] += w * A[i] * A[j];
                    b[i] += w * A[i] * d;
                }
                es[s] += w * d * d;
            }
        }
        npix[s] = (2 * r + 1) * (2 * r + 1);
        free(A);
    }
}

/*
 * Penalty weights of the basis (Eq. 9 without Phi): Q_i = sum_{u,v}
 * (u^2 + v^2)^2 k_i(u, v)^2, i = 0..nb-1.
 */
void orc_penalty_q(const orc_config* c, const double* kb, double* Q) {
    const int nb = orc_n_basis(c), h = c->h, K = 2 * h + 1;
    for (int i = 0; i < nb; i++) {
        double q = 0.0;
        for (int v = -h; v <= h; v++)
            for (int u = -h; u <= h; u++) {
                const double r2 = (double)(u * u + v * v);
                const double k = kb[(size_t)i * K * K + (v + h) * K + (u + h)];
                q += r2 * r2 * k * k;
            }
        Q[i] = q;
    }
}

/* Local coefficients of the two-kernel form at (x, y): alpha[0..nb-1] the
   b-terms, alpha[nb + i - 1] the c-term of basis i, alpha[2 nb - 1] = d0. */
static void dual_local(const orc_config* c, const double* a, double x, double y, int W, int H,
                       double* alpha) {
    const int nb = orc_n_basis(c), ns = orc_n_spatial(c), nt = 2 * nb - 1;
    double g[64];
    orc_spatial(c->S, x, y, W, H, g);
    for (int i = 0; i < nt; i++) {
        double v = 0.0;
        for (int s = 0; s < ns; s++) v += a[i * ns + s] * g[s];
        alpha[i] = v;
    }
    alpha[nt] = a[nt * ns];
}

/*
 * Solution of the two-kernel form with rejection (the single form's loop
 * and readings), the assembly over the 2 nb - 1 spatially varying columns,
 * and the penalty of Eq. 9 on the diagonal: unknown j of basis term i
 * (b-terms i >= 1 and every c-term; not b_0, the normalisation, nor d0)
 * gets P_j = Phi Q_i.  Reading of "neither negligible nor dominant":
 * Phi = phi * (sum over penalised j of M_jj) / (sum over penalised j of
 * Q_i(j)), recomputed at every assembly, so that the penalties add the
 * fraction phi (>= 0) to the total diagonal of the penalised unknowns.
 * The per-stamp chi2 (rejection, chi2/dof) is the data term alone.
 * kernel_sum_centre is K1's sum at the image centre (b_0 there).
 */
int orc_solve_dual(const orc_config* c, const double* kb, int W, int H, const int32_t* xy, int n,
                   const double* Ms, const double* bs, const double* es, const int32_t* npix,
                   int32_t* flags, double phi, double* coeffs, double* chi2, orc_stats* st) {
    const int nb = orc_n_basis(c), ns = orc_n_spatial(c), nt = 2 * nb - 1, N = nt * ns + 1,
              L = 2 * nb;
    uint8_t* used = (uint8_t*)calloc(n > 0 ? n : 1, 1);
    uint8_t* fitted = (uint8_t*)calloc(n > 0 ? n : 1, 1);
    double* M = (double*)malloc(sizeof(double) * (size_t)N * N);
    double* b = (double*)malloc(sizeof(double) * N);
    double* Q = (double*)malloc(sizeof(double) * nb);
    double* alpha = (double*)malloc(sizeof(double) * L);
    double g[64];
    orc_penalty_q(c, kb, Q);
    int ret = 0, iter = 0, n_rej = 0;
    memset(st, 0, sizeof(*st));
    for (int s = 0; s < n; s++) {
        used[s] = flags[s] == 0;
        fitted[s] = used[s];
        chi2[s] = 0.0;
    }
    for (int i = 0; i < N; i++) coeffs[i] = 0.0;
    for (;;) {
        int n_used = 0;
        for (int s = 0; s < n; s++) n_used += used[s];
        if (n_used < c->min_stamps) { ret = -3; st->info = -3; break; }
        /* assembly: M[(i,s),(j,t)] = sum g_s g_t M_s[i][j], the background unexpanded */
        memset(M, 0, sizeof(double) * (size_t)N * N);
        memset(b, 0, sizeof(double) * N);
        for (int k = 0; k < n; k++) {
            if (!used[k]) continue;
            orc_spatial(c->S, xy[2 * k], xy[2 * k + 1], W, H, g);
            const double* Mk = Ms + (size_t)k * L * L;
            const double* bk = bs + (size_t)k * L;
            for (int i = 0; i < nt; i++)
                for (int sa = 0; sa < ns; sa++) {
                    const int row = i * ns + sa;
                    for (int j = 0; j < nt; j++)
                        for (int t = 0; t < ns; t++)
                            M[(size_t)row * N + j * ns + t] += g[sa] * g[t] * Mk[i * L + j];
                    M[(size_t)row * N + N - 1] += g[sa] * Mk[i * L + nt];
                    M[(size_t)(N - 1) * N + row] += g[sa] * Mk[nt * L + i];
                    b[row] += g[sa] * bk[i];
                }
            M[(size_t)(N - 1) * N + N - 1] += Mk[nt * L + nt];
            b[N - 1] += bk[nt];
        }
        /* penalty */
        double dsum = 0.0, qsum = 0.0;
        for (int i = 1; i < nt; i++) {
            const double qi = Q[i < nb ? i : i - nb + 1];
            for (int sa = 0; sa < ns; sa++) {
                dsum += M[(size_t)(i * ns + sa) * N + i * ns + sa];
                qsum += qi;
            }
        }
        const double Phi = qsum > 0.0 ? phi * dsum / qsum : 0.0;
        for (int i = 1; i < nt; i++) {
            const double qi = Q[i < nb ? i : i - nb + 1];
            for (int sa = 0; sa < ns; sa++) M[(size_t)(i * ns + sa) * N + i * ns + sa] += Phi * qi;
        }
        int info = orc_cholesky_solve(N, M, b, coeffs);
        if (info) { ret = -4; st->info = info; break; }
        iter++;
        for (int k = 0; k < n; k++) {
            chi2[k] = 0.0;
            if (!fitted[k]) continue;
            dual_local(c, coeffs, xy[2 * k], xy[2 * k + 1], W, H, alpha);
            const double* Mk = Ms + (size_t)k * L * L;
            const double* bk = bs + (size_t)k * L;
            double q = 0.0, lin = 0.0;
            for (int i = 0; i < L; i++) {
                double t = 0.0;
                for (int j = 0; j < L; j++) t += Mk[i * L + j] * alpha[j];
                q += alpha[i] * t;
                lin += alpha[i] * bk[i];
            }
            chi2[k] = es[k] - 2.0 * lin + q;
        }
        if (iter >= c->max_iter) break;
        double mean = 0.0, var = 0.0;
        for (int k = 0; k < n; k++)
            if (used[k]) mean += chi2[k] / npix[k];
        mean /= n_used;
        for (int k = 0; k < n; k++)
            if (used[k]) {
                const double dq = chi2[k] / npix[k] - mean;
                var += dq * dq;
            }
        const double thr = mean + c->clip_sigma * sqrt(var / n_used);
        int n_new = 0;
        for (int k = 0; k < n; k++)
            if (used[k] && chi2[k] / npix[k] > thr) n_new++;
        if (n_new == 0 || n_used - n_new < c->min_stamps) break;
        for (int k = 0; k < n; k++)
            if (used[k] && chi2[k] / npix[k] > thr) {
                used[k] = 0;
                flags[k] |= ORC_STAMP_REJECTED;
                n_rej++;
            }
    }
    st->n_iter = iter;
    st->n_rejected = n_rej;
    if (ret != 0)
        for (int i = 0; i < N; i++) coeffs[i] = 0.0;
    if (ret == 0) {
        double c2 = 0.0, np = 0.0;
        int nu = 0;
        for (int k = 0; k < n; k++)
            if (used[k]) { c2 += chi2[k]; np += npix[k]; nu++; }
        st->chi2 = c2;
        st->dof = np - N;
        st->chi2_dof = c2 / (np - N);
        st->n_used = nu;
        dual_local(c, coeffs, 0.5 * (W - 1), 0.5 * (H - 1), W, H, alpha);
        st->kernel_sum_centre = alpha[0];
    }
    free(used);
    free(fitted);
    free(M);
    free(b);
    free(Q);
    free(alpha);
    return ret;
}

/* K1 = sum_i b_i(x, y) k_i and K2 = delta - sum_{i>=1} c_i(x, y) k_i at
   (x, y), each (2h+1)^2 in the basis layout. */
void orc_dual_kernels(const orc_config* c, const double* kb, const double* a, double x, double y,
                      int W, int H, double* K1, double* K2) {
    const int nb = orc_n_basis(c), h = c->h, Kw = 2 * h + 1, T = Kw * Kw;
    double* alpha = (double*)malloc(sizeof(double) * 2 * nb);
    dual_local(c, a, x, y, W, H, alpha);
    for (int t = 0; t < T; t++) {
        double k1 = 0.0, k2 = 0.0;
        for (int i = 0; i < nb; i++) k1 += alpha[i] * kb[(size_t)i * T + t];
        for (int i = 1; i < nb; i++) k2 += alpha[nb + i - 1] * kb[(size_t)i * T + t];
        K1[t] = k1;
        K2[t] = (t == h * Kw + h ? 1.0 : 0.0) - k2;
    }
    free(alpha);
}

/*
 * The two-kernel difference image: in each patch (kernels realised at the
 * patch centre, Section 3.5),
 *     D = K2 (x) I2~ - K1 (x) I1~ - d0,   V_D = K1^2 (x) V1~ + K2^2 (x) V2~,
 * with ~ meaning zero where masked or outside the image (the inputs are
 * taken as uncorrelated); mask: CONV_BAD if a masked or outside pixel of
 * I1 lies within K1's BAD radius or one of I2 within K2's, else CONV_POOR
 * if one of either lies within h (Section 3.4).
 */
void orc_dual_apply(const orc_config* c, const double* kb, const double* a, const float* I1,
                    const float* V1, const uint8_t* M1, const float* I2, const float* V2,
                    const uint8_t* M2, int W, int H, int64_t pitch, float* D, float* VD,
                    uint8_t* MD) {
    const int h = c->h, Kw = 2 * h + 1, T = Kw * Kw, np = orc_n_patches(c, W, H);
    const double d0 = a[orc_dual_unknowns(c) - 1];
#pragma omp parallel for schedule(dynamic)
    for (int p = 0; p < np; p++) {
        int x0, x1, y0, y1;
        double* K1 = (double*)malloc(sizeof(double) * T);
        double* K2 = (double*)malloc(sizeof(double) * T);
        patch_bounds(W, H, c->P, p, &x0, &x1, &y0, &y1);
        orc_dual_kernels(c, kb, a, 0.5 * (x0 + x1 - 1), 0.5 * (y0 + y1 - 1), W, H, K1, K2);
        const int rb1 = orc_bad_radius(K1, h, c->bad_frac), rb2 = orc_bad_radius(K2, h, c->bad_frac);
        for (int y = y0; y < y1; y++)
            for (int x = x0; x < x1; x++) {
                double s1 = 0.0, s2 = 0.0, v1 = 0.0, v2 = 0.0;
                int dm1 = h + 1, dm2 = h + 1;
                for (int v = -h; v <= h; v++)
                    for (int u = -h; u <= h; u++) {
                        const int xx = x - u, yy = y - v;
                        const int t = (v + h) * Kw + (u + h);
                        const int dd = abs(u) > abs(v) ? abs(u) : abs(v);
                        const int in = xx >= 0 && xx < W && yy >= 0 && yy < H;
                        const int64_t o = (int64_t)yy * pitch + xx;
                        if (in && !M1[o]) {
                            s1 += K1[t] * (double)I1[o];
                            v1 += K1[t] * K1[t] * (double)V1[o];
                        } else if (dd < dm1) {
                            dm1 = dd;
                        }
                        if (in && !M2[o]) {
                            s2 += K2[t] * (double)I2[o];
                            v2 += K2[t] * K2[t] * (double)V2[o];
                        } else if (dd < dm2) {
                            dm2 = dd;
                        }
                    }
                const int64_t o = (int64_t)y * pitch + x;
                D[o] = (float)(s2 - s1 - d0);
                VD[o] = (float)(v1 + v2);
                MD[o] = (dm1 <= rb1 || dm2 <= rb2) ? ORC_MASK_CONV_BAD
                        : (dm1 <= h || dm2 <= h) ? ORC_MASK_CONV_POOR : 0;
            }
        free(K1);
        free(K2);
    }
}
