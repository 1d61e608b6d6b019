// Assembly, solution and rejection (Section 2; Sections 3.3, 3.5, 3.6).
//
// Stream-ordered loop of at most max_iter rounds, each made of
//   k_assemble  - M[(i,s),(j,t)] = sum_used g_s g_t M_s[i][j] (FP64, many
//                 workgroups, one thread per (i, j, s));
//   k_cholesky  - one 1024-thread workgroup: symmetric equilibration,
//                 blocked right-looking Cholesky (32-column panels in LDS,
//                 trailing update read-modify-write in L2-resident
//                 workspace), forward and back substitution;
//   k_chi2_clip - per-stamp chi2 from the stamp sums and the sigma-clip.
// A device-side state word ends the loop early (converged, or failed);
// later kernels of the unrolled loop then return at once, so the host never
// waits on the device.
#include "internal.h"

namespace {

struct SolveState {
    int done;
    int info;
    int n_iter;
    int n_rej;
    int n_used;
    int pad[3];
};

constexpr int CH_NB = 32;        // Cholesky panel width
constexpr int CH_PS = 33;        // LDS row stride of the panel (doubles)
constexpr int CH_THREADS = 512;
constexpr int CH_NMAX = 496;     // largest system the one-workgroup solver holds

__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}


__global__ void k_solve_init(int n, int N, int ns, int S, int W, int H, int min_stamps,
                             const int32_t* __restrict__ xy, const int32_t* __restrict__ flags,
                             uint8_t* __restrict__ used, uint8_t* __restrict__ fitted,
                             double* __restrict__ G, double* __restrict__ chi2,
                             double* __restrict__ coeffs, SolveState* st) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) {
        const int u = flags[t] == 0;
        used[t] = u;
        fitted[t] = u;
        chi2[t] = 0.0;
        double g[64];
        psfm_spatial_terms(S, xy[2 * t], xy[2 * t + 1], W, H, g);
        for (int s = 0; s < ns; s++) G[(size_t)t * ns + s] = g[s];
    }
    if (t < N) coeffs[t] = 0.0;
    if (blockIdx.x == 0) {
        __shared__ int cnt;
        if (threadIdx.x == 0) cnt = 0;
        __syncthreads();
        int c = 0;
        for (int s = threadIdx.x; s < n; s += blockDim.x) c += flags[s] == 0;
        atomicAdd(&cnt, c);
        __syncthreads();
        if (threadIdx.x == 0) {
            st->n_used = cnt;
            st->n_iter = 0;
            st->n_rej = 0;
            st->info = cnt < min_stamps ? PSFM_ERR_TOO_FEW_STAMPS : 0;
            st->done = cnt < min_stamps;
        }
    }
}

// One thread per (i, j, s) of the per-stamp index space; loops over stamps
// (the stamp's weight used_k * g_k is uniform across the workgroup, so it
// comes through the scalar cache; the loop has no data-dependent branch so
// the per-stamp loads pipeline).
template <int NS>
__global__ __launch_bounds__(256) void k_assemble(int n, int nb, int N, const double* __restrict__ Ms,
                                                  const double* __restrict__ bs,
                                                  const double* __restrict__ GU,
                                                  double* __restrict__ M, double* __restrict__ b,
                                                  const SolveState* st) {
    if (st->done) return;
    const int L = nb + 1;
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    const int nm = L * L * NS;
    if (t < nm) {
        const int s = t % NS;
        const int ij = t / NS;
        const int i = ij / L, j = ij - i * L;
        if (i == nb && s != 0) return;
        double acc[NS];
#pragma unroll
        for (int q = 0; q < NS; q++) acc[q] = 0.0;
#pragma unroll 4
        for (int k = 0; k < n; k++) {
            const double m = Ms[(size_t)k * L * L + ij];
            const double* g = GU + (size_t)k * (NS + 1);     // g_k[0..NS), used_k
            const double gm = ((i == nb) ? g[NS] : g[NS] * g[s]) * m;
            if (j == nb) {
                acc[0] += gm;
            } else {
#pragma unroll
                for (int q = 0; q < NS; q++) acc[q] += g[q] * gm;
            }
        }
        const int row = (i == nb) ? N - 1 : i * NS + s;
        if (j == nb) {
            M[(size_t)row * N + N - 1] = acc[0];
        } else {
#pragma unroll
            for (int q = 0; q < NS; q++) M[(size_t)row * N + j * NS + q] = acc[q];
        }
    } else if (t < nm + L * NS) {
        const int e = t - nm;
        const int i = e / NS, s = e - i * NS;
        if (i == nb && s != 0) return;
        double acc = 0.0;
        for (int k = 0; k < n; k++) {
            const double* g = GU + (size_t)k * (NS + 1);
            const double gs = (i == nb) ? g[NS] : g[NS] * g[s];
            acc += gs * bs[(size_t)k * L + i];
        }
        b[(i == nb) ? N - 1 : i * NS + s] = acc;
    }
}

// Stamp weights for the assembly: GU[k] = (g_k[0..ns), used_k).
__global__ void k_weights(int n, int ns, const double* __restrict__ G,
                          const uint8_t* __restrict__ used, double* __restrict__ GU,
                          const SolveState* st) {
    if (st->done) return;
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    for (int q = 0; q < ns; q++) GU[(size_t)t * (ns + 1) + q] = G[(size_t)t * ns + q];
    GU[(size_t)t * (ns + 1) + ns] = used[t] ? 1.0 : 0.0;
}

__device__ __forceinline__ double block_sum(double v, double* red) { return psfm_block_sum(v, red); }

// Equilibrated Cholesky and solve of the N x N system in A (lower triangle
// overwritten by the factor); x receives the solution.  One workgroup.
// Per 32-column panel (staged in LDS):
//   * wave 0 factors the 32 x 32 diagonal block, rows in registers, the
//     pivot column broadcast through LDS, 1/sqrt by v_rsq_f64 + 2 Newton
//     steps (no workgroup barrier per column);
//   * every other panel row is solved against it by its own thread
//     (right-looking, independent FMAs per step);
//   * the forward substitution L z = D b advances by the same 32 unknowns
//     while the panel is in LDS;
//   * the trailing lower triangle is updated with v_mfma_f64_16x16x4f64 on
//     16 x 16 tiles (read-modify-write of the L2-resident workspace).
// The back substitution L^T w = z then walks the panels in reverse, each
// staged in LDS by a coalesced bulk load.
typedef double double4v __attribute__((ext_vector_type(4)));

__device__ __forceinline__ double rsqrt_nr(double d) {
    double r = __builtin_amdgcn_rsq(d);
    r = r * (1.5 - 0.5 * d * r * r);
    r = r * (1.5 - 0.5 * d * r * r);
    return r;
}

__global__ __launch_bounds__(CH_THREADS) void k_cholesky(int N, double* __restrict__ A,
                                                         const double* __restrict__ b,
                                                         double* __restrict__ x,
                                                         double* __restrict__ y, SolveState* st) {
    if (st->done) return;
    extern __shared__ double P[];        // panel [N + 16][CH_PS]
    __shared__ double Dq[CH_NMAX];
    __shared__ double zb[CH_NMAX];
    __shared__ double dinv[CH_NMAX];
    __shared__ double part[CH_NB * (CH_THREADS / 32)];
    __shared__ double cb[64];
    __shared__ int s_bad;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    constexpr int NW = CH_THREADS / 64;
    constexpr int NPART = CH_THREADS / 32;
    (void)y;
    if (tid == 0) s_bad = 0;
    __syncthreads();
    for (int i = tid; i < N; i += CH_THREADS) {
        const double d = A[(size_t)i * N + i];
        if (!(d > 0.0)) atomicOr(&s_bad, 1);
        Dq[i] = d > 0.0 ? 1.0 / sqrt(d) : 0.0;
    }
    __syncthreads();
    if (s_bad) {
        if (tid == 0) {
            int first = N + 1;
            for (int i = 0; i < N; i++)
                if (Dq[i] == 0.0) { first = i + 1; break; }
            st->info = first;
            st->done = 1;
        }
        return;
    }
    for (int i = tid; i < N; i += CH_THREADS) zb[i] = Dq[i] * b[i];
    const int tr = tid >> 5, tc = tid & 31, TR = CH_THREADS / 32;
    for (int i = tr; i < N; i += TR)
        for (int j = tc; j <= i; j += 32) A[(size_t)i * N + j] *= Dq[i] * Dq[j];
    __syncthreads();
    for (int k0 = 0; k0 < N; k0 += CH_NB) {
        const int nk = min(CH_NB, N - k0);
        const int rows = N - k0;
        for (int i = tr; i < rows + 16; i += TR)
            P[i * CH_PS + tc] = (i < rows && tc < nk && (i >= nk || tc <= i))
                                    ? A[(size_t)(k0 + i) * N + k0 + tc] : 0.0;
        __syncthreads();
        // ---- diagonal block (wave 0)
        if (wave == 0) {
            double r[CH_NB];
#pragma unroll
            for (int c = 0; c < CH_NB; c++) r[c] = lane < nk ? P[lane * CH_PS + c] : 0.0;
            int bad = 0;
#pragma unroll
            for (int c = 0; c < CH_NB; c++) {
                if (c < nk && !bad) {
                    if (lane < CH_NB) cb[lane] = r[c];
                    wave_sync();
                    const double d = cb[c];
                    if (!(d > 0.0)) {
                        bad = c + 1;
                    } else {
                        const double inv = rsqrt_nr(d);
                        const double t = (lane > c && lane < nk) ? r[c] * inv * inv : 0.0;
#pragma unroll
                        for (int j = c + 1; j < CH_NB; j++) r[j] -= t * cb[j];
                        r[c] = lane == c ? d * inv : (lane > c ? r[c] * inv : r[c]);
                        if (lane == 0) dinv[k0 + c] = inv;
                    }
                    wave_sync();
                }
            }
            if (lane < nk) {
#pragma unroll
                for (int c = 0; c < CH_NB; c++) P[lane * CH_PS + c] = c <= lane ? r[c] : 0.0;
            }
            if (lane == 0) s_bad = bad;
        }
        __syncthreads();
        if (s_bad) {
            if (tid == 0) {
                st->info = k0 + s_bad;
                st->done = 1;
            }
            return;
        }
        // ---- panel rows below the diagonal block: a L_diag^T = row
        for (int i = nk + tid; i < rows; i += CH_THREADS) {
            double a[CH_NB];
#pragma unroll
            for (int c = 0; c < CH_NB; c++) a[c] = P[i * CH_PS + c];
#pragma unroll
            for (int c = 0; c < CH_NB; c++) {
                if (c < nk) {
                    a[c] *= dinv[k0 + c];
#pragma unroll
                    for (int q = c + 1; q < CH_NB; q++) a[q] -= a[c] * P[q * CH_PS + c];
                }
            }
#pragma unroll
            for (int c = 0; c < CH_NB; c++) P[i * CH_PS + c] = a[c];
        }
        // ---- forward substitution for this block of unknowns (wave 0)
        if (wave == 0) {
            double v = lane < nk ? zb[k0 + lane] : 0.0;
            for (int c = 0; c < nk; c++) {
                const double vc = __shfl(v, c) * dinv[k0 + c];
                if (lane == c) v = vc;
                if (lane > c && lane < nk) v -= P[lane * CH_PS + c] * vc;
            }
            if (lane < nk) zb[k0 + lane] = v;
        }
        __syncthreads();
        for (int i = nk + tid; i < rows; i += CH_THREADS) {
            double acc = 0.0;
            for (int c = 0; c < nk; c++) acc += P[i * CH_PS + c] * zb[k0 + c];
            zb[k0 + i] -= acc;
        }
        for (int i = tr; i < rows; i += TR)
            if (tc < nk && (i >= nk || tc <= i)) A[(size_t)(k0 + i) * N + k0 + tc] = P[i * CH_PS + tc];
        // ---- trailing update on FP64 MFMA: 16 x 16 tiles of the lower triangle
        const int m = rows - nk;
        if (m > 0) {
            const int mt = (m + 15) / 16;
            const int ntile = mt * (mt + 1) / 2;
            for (int tI = wave; tI < ntile; tI += NW) {
                int ti = (int)((sqrt(8.0 * tI + 1.0) - 1.0) * 0.5);
                while ((ti + 1) * (ti + 2) / 2 <= tI) ti++;
                while (ti * (ti + 1) / 2 > tI) ti--;
                const int tj = tI - ti * (ti + 1) / 2;
                const int i0 = nk + 16 * ti, j0 = nk + 16 * tj;
                const int jj = j0 + (lane & 15);
                double4v c;
#pragma unroll
                for (int e = 0; e < 4; e++) {
                    const int ii = i0 + (lane >> 4) + 4 * e;   // f64 MFMA D layout
                    c[e] = (ii < rows && jj <= ii) ? A[(size_t)(k0 + ii) * N + k0 + jj] : 0.0;
                }
                const double* pa = P + (i0 + (lane & 15)) * CH_PS + (lane >> 4);
                const double* pb = P + (j0 + (lane & 15)) * CH_PS + (lane >> 4);
#pragma unroll
                for (int cc = 0; cc < CH_NB; cc += 4)
                    c = __builtin_amdgcn_mfma_f64_16x16x4f64(-pa[cc], pb[cc], c, 0, 0, 0);
#pragma unroll
                for (int e = 0; e < 4; e++) {
                    const int ii = i0 + (lane >> 4) + 4 * e;   // f64 MFMA D layout
                    if (ii < rows && jj <= ii) A[(size_t)(k0 + ii) * N + k0 + jj] = c[e];
                }
            }
        }
        __syncthreads();
    }
    // ---- back substitution L^T w = z, panels in reverse
    for (int k0 = ((N - 1) / CH_NB) * CH_NB; k0 >= 0; k0 -= CH_NB) {
        const int nk = min(CH_NB, N - k0);
        const int rows = N - k0;
        for (int i = tr; i < rows; i += TR)
            P[i * CH_PS + tc] = (tc < nk && (i >= nk || tc <= i)) ? A[(size_t)(k0 + i) * N + k0 + tc] : 0.0;
        __syncthreads();
        {
            const int c = tid & 31, w = tid >> 5;
            double acc = 0.0;
            if (c < nk)
                for (int i = nk + w; i < rows; i += NPART) acc += P[i * CH_PS + c] * zb[k0 + i];
            part[c * NPART + w] = acc;
        }
        __syncthreads();
        if (wave == 0) {
            double v = 0.0;
            if (lane < nk) {
                v = zb[k0 + lane];
                for (int w = 0; w < NPART; w++) v -= part[lane * NPART + w];
            }
            for (int c = nk - 1; c >= 0; c--) {
                const double vc = __shfl(v, c) * dinv[k0 + c];
                if (lane == c) v = vc;
                if (lane < c) v -= P[c * CH_PS + lane] * vc;
            }
            if (lane < nk) zb[k0 + lane] = v;
        }
        __syncthreads();
    }
    for (int i = tid; i < N; i += CH_THREADS) x[i] = Dq[i] * zb[i];
}

// chi2_s = e_s - 2 alpha^T b_s + alpha^T M_s alpha for every fitted stamp,
// then the sigma-clip over the used stamps.
__global__ __launch_bounds__(1024) void k_chi2_clip(
    int n, int nb, int ns, int N, int max_iter, int min_stamps, double clip_sigma,
    const double* __restrict__ Ms, const double* __restrict__ bs, const double* __restrict__ es,
    const int32_t* __restrict__ npix, const double* __restrict__ G, const double* __restrict__ a,
    uint8_t* __restrict__ used, const uint8_t* __restrict__ fitted, int32_t* __restrict__ flags,
    double* __restrict__ chi2, SolveState* st) {
    if (st->done) return;
    __shared__ double alpha[16][64];
    __shared__ double red[16];
    __shared__ double s_thr;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int L = nb + 1;
    for (int s = wave; s < n; s += 16) {
        if (!fitted[s]) continue;               // wave-uniform
        if (lane < L) {
            double al;
            if (lane < nb) {
                al = 0.0;
                for (int q = 0; q < ns; q++) al += a[lane * ns + q] * G[(size_t)s * ns + q];
            } else {
                al = a[N - 1];
            }
            alpha[wave][lane] = al;
        }
        wave_sync();
        // lane j: u_j = sum_i alpha_i M_s[i][j] (row-wise coalesced reads)
        double part = 0.0;
        if (lane < L) {
            const double* Mc = Ms + (size_t)s * L * L + lane;
            double u = 0.0;
#pragma unroll 8
            for (int i = 0; i < L; i++) u += alpha[wave][i] * Mc[(size_t)i * L];
            const double al = alpha[wave][lane];
            part = al * u - 2.0 * al * bs[(size_t)s * L + lane];
        }
        for (int o = 32; o > 0; o >>= 1) part += __shfl_down(part, o);
        if (lane == 0) chi2[s] = es[s] + part;
        wave_sync();
    }
    __syncthreads();
    if (tid == 0) st->n_iter += 1;
    __syncthreads();
    if (st->n_iter >= max_iter) {
        if (tid == 0) st->done = 1;
        return;
    }
    // mean and population std of q_s = chi2_s / npix_s over used stamps
    double sq = 0.0, cnt = 0.0;
    for (int s = tid; s < n; s += 1024)
        if (used[s]) {
            sq += chi2[s] / npix[s];
            cnt += 1.0;
        }
    const double tot = block_sum(sq, red);
    const double nu = block_sum(cnt, red);
    const double mean = tot / nu;
    double dv = 0.0;
    for (int s = tid; s < n; s += 1024)
        if (used[s]) {
            const double d = chi2[s] / npix[s] - mean;
            dv += d * d;
        }
    const double var = block_sum(dv, red) / nu;
    if (tid == 0) s_thr = mean + clip_sigma * sqrt(var);
    __syncthreads();
    const double thr = s_thr;
    double nnew = 0.0;
    for (int s = tid; s < n; s += 1024)
        if (used[s] && chi2[s] / npix[s] > thr) nnew += 1.0;
    const double tnew = block_sum(nnew, red);
    if (tnew == 0.0 || nu - tnew < (double)min_stamps) {
        if (tid == 0) st->done = 1;
        return;
    }
    for (int s = tid; s < n; s += 1024)
        if (used[s] && chi2[s] / npix[s] > thr) {
            used[s] = 0;
            flags[s] |= PSFM_STAMP_REJECTED;
        }
    if (tid == 0) {
        st->n_rej += (int)tnew;
        st->n_used -= (int)tnew;
    }
}

__global__ void k_solve_finish(int n, int nb, int ns, int N, int S, int W, int H,
                               const int32_t* __restrict__ npix, const uint8_t* __restrict__ used,
                               const double* __restrict__ chi2, double* __restrict__ coeffs,
                               const SolveState* st, psfm_fit_stats* stats) {
    __shared__ double red[16];
    const int tid = threadIdx.x;
    double c2 = 0.0, np = 0.0, nu = 0.0;
    for (int s = tid; s < n; s += blockDim.x)
        if (used[s]) {
            c2 += chi2[s];
            np += npix[s];
            nu += 1.0;
        }
    c2 = block_sum(c2, red);
    np = block_sum(np, red);
    nu = block_sum(nu, red);
    const int info = st->info;
    if (info != 0)
        for (int i = tid; i < N; i += blockDim.x) coeffs[i] = 0.0;
    __syncthreads();
    if (tid == 0 && stats) {
        stats->n_iter = st->n_iter;
        stats->n_rejected = st->n_rej;
        stats->info = info;
        if (info == 0) {
            stats->chi2 = c2;
            stats->dof = np - N;
            stats->chi2_dof = c2 / (np - N);
            stats->n_used = (int)nu;
            double g[64];
            psfm_spatial_terms(S, 0.5 * (W - 1), 0.5 * (H - 1), W, H, g);
            double k = 0.0;
            for (int q = 0; q < ns; q++) k += coeffs[q] * g[q];
            stats->kernel_sum_centre = k;
        } else {
            stats->chi2 = 0.0;
            stats->dof = 0.0;
            stats->chi2_dof = 0.0;
            stats->n_used = 0;
            stats->kernel_sum_centre = 0.0;
        }
    }
}

}  // namespace

namespace psfm {

size_t solve_workspace(const psfm_context* ctx, int n) {
    Carver c(nullptr);
    c.take<SolveState>(1);
    c.take<uint8_t>(n + 1);
    c.take<uint8_t>(n + 1);
    c.take<double>((size_t)n * ctx->ns + 1);
    c.take<double>((size_t)n * (ctx->ns + 1) + 1);
    c.take<double>((size_t)ctx->N * ctx->N);
    c.take<double>(ctx->N);
    c.take<double>(ctx->N);
    return c.off;
}

}  // namespace psfm

extern "C" int psfm_solve(const psfm_context* ctx, int W, int H, const int32_t* stamp_xy,
                          int n_stamps, const double* stamp_M, const double* stamp_b,
                          const double* stamp_e, const int32_t* stamp_npix, int32_t* stamp_flags,
                          double* coeffs, double* stamp_chi2, psfm_fit_stats* stats, void* ws,
                          size_t ws_bytes, void* stream) {
    if (!ctx || n_stamps < 0 || !coeffs || !stats) return PSFM_ERR_INVALID_ARG;
    if (W < 1 || H < 1) return PSFM_ERR_SHAPE;
    if (n_stamps > 0 && (!stamp_xy || !stamp_M || !stamp_b || !stamp_e || !stamp_npix ||
                         !stamp_flags || !stamp_chi2))
        return PSFM_ERR_INVALID_ARG;
    if (ctx->N > CH_NMAX) return PSFM_ERR_UNSUPPORTED;
    const size_t need = psfm::solve_workspace(ctx, n_stamps);
    if (!ws || ws_bytes < need) return PSFM_ERR_WORKSPACE;
    const size_t lds = (size_t)(ctx->N + 16) * CH_PS * sizeof(double);
    if (lds > 140 * 1024) return PSFM_ERR_UNSUPPORTED;
    hipStream_t st = (hipStream_t)stream;
    psfm::Carver c(ws);
    SolveState* state = c.take<SolveState>(1);
    uint8_t* used = c.take<uint8_t>(n_stamps + 1);
    uint8_t* fitted = c.take<uint8_t>(n_stamps + 1);
    double* G = c.take<double>((size_t)n_stamps * ctx->ns + 1);
    double* GU = c.take<double>((size_t)n_stamps * (ctx->ns + 1) + 1);
    double* M = c.take<double>((size_t)ctx->N * ctx->N);
    double* b = c.take<double>(ctx->N);
    double* y = c.take<double>(ctx->N);
    const int nb = ctx->nb, ns = ctx->ns, N = ctx->N, L = ctx->L;
    const psfm_config& cf = ctx->cfg;
    static size_t attr_set = 0;      // dynamic LDS granted so far
    if (lds > attr_set) {
        PSFM_HIP_CHECK(hipFuncSetAttribute((const void*)k_cholesky,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
        attr_set = lds;
    }
    const int nt = std::max(n_stamps, N);
    hipLaunchKernelGGL(k_solve_init, dim3((nt + 255) / 256), dim3(256), 0, st, n_stamps, N, ns,
                       cf.spatial_order, W, H, cf.min_stamps, stamp_xy, stamp_flags, used, fitted,
                       G, stamp_chi2, coeffs, state);
    PSFM_HIP_CHECK(hipGetLastError());
    const int nthreads_asm = L * L * ns + L * ns;
    for (int it = 0; it < cf.max_iter; it++) {
        hipLaunchKernelGGL(k_weights, dim3((n_stamps + 255) / 256 + 1), dim3(256), 0, st, n_stamps, ns,
                           G, used, GU, state);
        const dim3 ag((nthreads_asm + 255) / 256);
        switch (ns) {
#define PSFM_ASM_CASE(NSV) \
    case NSV: hipLaunchKernelGGL(k_assemble<NSV>, ag, dim3(256), 0, st, n_stamps, nb, N, stamp_M, stamp_b, GU, M, b, state); break;
            PSFM_ASM_CASE(1) PSFM_ASM_CASE(3) PSFM_ASM_CASE(6) PSFM_ASM_CASE(10) PSFM_ASM_CASE(15)
            PSFM_ASM_CASE(21) PSFM_ASM_CASE(28)
#undef PSFM_ASM_CASE
            default: return PSFM_ERR_UNSUPPORTED;
        }
        hipLaunchKernelGGL(k_cholesky, dim3(1), dim3(CH_THREADS), lds, st, N, M, b, coeffs, y, state);
        hipLaunchKernelGGL(k_chi2_clip, dim3(1), dim3(1024), 0, st, n_stamps, nb, ns, N, cf.max_iter,
                           cf.min_stamps, cf.clip_sigma, stamp_M, stamp_b, stamp_e, stamp_npix, G,
                           coeffs, used, fitted, stamp_flags, stamp_chi2, state);
    }
    hipLaunchKernelGGL(k_solve_finish, dim3(1), dim3(1024), 0, st, n_stamps, nb, ns, N,
                       cf.spatial_order, W, H, stamp_npix, used, stamp_chi2, coeffs, state, stats);
    PSFM_HIP_CHECK(hipGetLastError());
    return PSFM_OK;
}
