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
constexpr int CH_THREADS = 1024;

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

// One thread per (i, j, s) of the per-stamp index space; loops over stamps.
__global__ void k_assemble(int n, int nb, int ns, int N, const double* __restrict__ Ms,
                           const double* __restrict__ bs, const uint8_t* __restrict__ used,
                           const double* __restrict__ G, double* __restrict__ M,
                           double* __restrict__ b, const SolveState* st) {
    if (st->done) return;
    const int L = nb + 1;
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    const int nm = L * L * ns;
    if (t < nm) {
        const int s = t % ns;
        const int ij = t / ns;
        const int i = ij / L, j = ij - i * L;
        if (i == nb && s != 0) return;
        double acc[28];
        const int nt = (j == nb) ? 1 : ns;
#pragma unroll
        for (int q = 0; q < 28; q++) acc[q] = 0.0;
        for (int k = 0; k < n; k++) {
            if (!used[k]) continue;
            const double m = Ms[(size_t)k * L * L + ij];
            const double* g = G + (size_t)k * ns;
            const double gm = ((i == nb) ? 1.0 : g[s]) * m;
            if (j == nb) {
                acc[0] += gm;
            } else {
#pragma unroll
                for (int q = 0; q < 28; q++)
                    if (q < nt) acc[q] += g[q] * gm;
            }
        }
        const int row = (i == nb) ? N - 1 : i * ns + s;
        if (j == nb) {
            M[(size_t)row * N + N - 1] = acc[0];
        } else {
#pragma unroll
            for (int q = 0; q < 28; q++)
                if (q < nt) M[(size_t)row * N + j * ns + q] = acc[q];
        }
    } else if (t < nm + L * ns) {
        const int e = t - nm;
        const int i = e / ns, s = e - i * ns;
        if (i == nb && s != 0) return;
        double acc = 0.0;
        for (int k = 0; k < n; k++) {
            if (!used[k]) continue;
            const double gs = (i == nb) ? 1.0 : G[(size_t)k * ns + s];
            acc += gs * bs[(size_t)k * L + i];
        }
        b[(i == nb) ? N - 1 : i * ns + s] = acc;
    }
}

__device__ __forceinline__ double block_sum(double v, double* red) { return psfm_block_sum(v, red); }

// Equilibrated Cholesky and solve of the N x N system in A (overwritten by
// its factor); x receives the solution.  One workgroup.
__global__ __launch_bounds__(CH_THREADS) void k_cholesky(int N, double* __restrict__ A,
                                                         const double* __restrict__ b,
                                                         double* __restrict__ x,
                                                         double* __restrict__ y, SolveState* st) {
    if (st->done) return;
    extern __shared__ double P[];        // panel [N][CH_NB]
    __shared__ double Dq[512];
    __shared__ int s_bad;
    const int tid = threadIdx.x;
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
    // equilibrate the lower triangle
    for (size_t e = tid; e < (size_t)N * N; e += CH_THREADS) {
        const int i = (int)(e / N), j = (int)(e - (size_t)i * N);
        if (j <= i) A[e] *= Dq[i] * Dq[j];
    }
    __syncthreads();
    for (int k0 = 0; k0 < N; k0 += CH_NB) {
        const int nk = min(CH_NB, N - k0);
        const int rows = N - k0;
        for (int e = tid; e < rows * CH_NB; e += CH_THREADS) {
            const int i = e / CH_NB, c = e - i * CH_NB;
            P[e] = (c < nk && c <= i) ? A[(size_t)(k0 + i) * N + k0 + c] : 0.0;
        }
        __syncthreads();
        for (int c = 0; c < nk; c++) {
            const double piv = P[c * CH_NB + c];
            __syncthreads();
            if (!(piv > 0.0)) {
                if (tid == 0) {
                    st->info = k0 + c + 1;
                    st->done = 1;
                }
                return;
            }
            const double lkk = sqrt(piv);
            const double inv = 1.0 / lkk;
            for (int i = c + 1 + tid; i < rows; i += CH_THREADS) P[i * CH_NB + c] *= inv;
            if (tid == 0) P[c * CH_NB + c] = lkk;
            __syncthreads();
            const int nr = nk - c - 1;
            if (nr > 0) {
                for (int e = tid; e < (rows - c - 1) * nr; e += CH_THREADS) {
                    const int i = c + 1 + e / nr, j = c + 1 + e % nr;
                    if (j <= i) P[i * CH_NB + j] -= P[i * CH_NB + c] * P[j * CH_NB + c];
                }
            }
            __syncthreads();
        }
        for (int e = tid; e < rows * nk; e += CH_THREADS) {
            const int i = e / nk, c = e - i * nk;
            if (c <= i) A[(size_t)(k0 + i) * N + k0 + c] = P[i * CH_NB + c];
        }
        // trailing update, 4x4 register tiles over the lower triangle of the
        // remaining (rows - nk) x (rows - nk) block
        const int m = rows - nk;
        if (m > 0) {
            const int tb = (m + 3) / 4;
            const int ntiles = tb * (tb + 1) / 2;
            for (int tI = tid; tI < ntiles; tI += CH_THREADS) {
                // decode lower-triangular tile index (ti >= tj)
                int ti = (int)((sqrt(8.0 * tI + 1.0) - 1.0) * 0.5);
                while ((ti + 1) * (ti + 2) / 2 <= tI) ti++;
                while (ti * (ti + 1) / 2 > tI) ti--;
                const int tj = tI - ti * (ti + 1) / 2;
                double acc[4][4];
#pragma unroll
                for (int a = 0; a < 4; a++)
#pragma unroll
                    for (int q = 0; q < 4; q++) acc[a][q] = 0.0;
                const int i0 = nk + 4 * ti, j0 = nk + 4 * tj;
                for (int c = 0; c < nk; c++) {
                    double pi[4], pj[4];
#pragma unroll
                    for (int a = 0; a < 4; a++) {
                        pi[a] = (i0 + a < rows) ? P[(i0 + a) * CH_NB + c] : 0.0;
                        pj[a] = (j0 + a < rows) ? P[(j0 + a) * CH_NB + c] : 0.0;
                    }
#pragma unroll
                    for (int a = 0; a < 4; a++)
#pragma unroll
                        for (int q = 0; q < 4; q++) acc[a][q] += pi[a] * pj[q];
                }
#pragma unroll
                for (int a = 0; a < 4; a++)
#pragma unroll
                    for (int q = 0; q < 4; q++) {
                        const int i = i0 + a, j = j0 + q;
                        if (i < rows && j <= i) A[(size_t)(k0 + i) * N + (k0 + j)] -= acc[a][q];
                    }
            }
        }
        __syncthreads();
    }
    // Forward substitution L z = D b, then back substitution L^T w = z, in
    // blocks of 32 unknowns: the off-diagonal part of each block is a
    // parallel (coalesced) matrix-vector product, the 32 x 32 diagonal
    // system is solved by one wave from LDS.
    double* zb = P;                       // [N] right-hand side / solution
    double* Dg = P + 512;                 // [32][33] diagonal block
    double* part = P + 512 + 32 * 33;     // [32][32] partial dot products
    for (int i = tid; i < N; i += CH_THREADS) zb[i] = Dq[i] * b[i];
    __syncthreads();
    const int lane = tid & 63, wave = tid >> 6;
    for (int k0 = 0; k0 < N; k0 += 32) {
        const int nk = min(32, N - k0);
        // part[r][w] = sum_{p in chunk w} L[k0+r][p] z[p], p < k0
        {
            const int r = tid >> 5, w = tid & 31;      // 32 rows x 32 chunks
            double acc = 0.0;
            if (r < nk)
                for (int p = w; p < k0; p += 32) acc += A[(size_t)(k0 + r) * N + p] * zb[p];
            part[r * 32 + w] = acc;
            for (int e = tid; e < nk * nk; e += CH_THREADS) {
                const int i = e / nk, c = e - i * nk;
                Dg[i * 33 + c] = c <= i ? A[(size_t)(k0 + i) * N + k0 + c] : 0.0;
            }
        }
        __syncthreads();
        if (wave == 0) {
            double v = 0.0;
            if (lane < nk) {
                v = zb[k0 + lane];
                for (int w = 0; w < 32; w++) v -= part[lane * 32 + w];
            }
            for (int c = 0; c < nk; c++) {
                const double vc = __shfl(v, c) / Dg[c * 33 + c];
                if (lane == c) v = vc;
                if (lane > c && lane < nk) v -= Dg[lane * 33 + c] * vc;
            }
            if (lane < nk) zb[k0 + lane] = v;
        }
        __syncthreads();
    }
    for (int k1 = N; k1 > 0; k1 -= 32) {
        const int k0 = k1 >= 32 ? k1 - 32 : 0;
        const int nk = k1 - k0;
        // part[c][w] = sum_{p >= k1, p in chunk w} L[p][k0+c] w[p]
        {
            const int c = tid & 31, w = tid >> 5;
            double acc = 0.0;
            if (c < nk)
                for (int p = k1 + w; p < N; p += 32) acc += A[(size_t)p * N + k0 + c] * zb[p];
            part[c * 32 + w] = acc;
            for (int e = tid; e < nk * nk; e += CH_THREADS) {
                const int i = e / nk, cc = e - i * nk;
                Dg[i * 33 + cc] = cc <= i ? A[(size_t)(k0 + i) * N + k0 + cc] : 0.0;
            }
        }
        __syncthreads();
        if (wave == 0) {
            double v = 0.0;
            if (lane < nk) {
                v = zb[k0 + lane];
                for (int w = 0; w < 32; w++) v -= part[lane * 32 + w];
            }
            for (int c = nk - 1; c >= 0; c--) {
                const double vc = __shfl(v, c) / Dg[c * 33 + c];
                if (lane == c) v = vc;
                if (lane < c) v -= Dg[c * 33 + lane] * vc;
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
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        double part = 0.0;
        if (lane < L) {
            const double* Mr = Ms + (size_t)s * L * L + (size_t)lane * L;
            double tq = 0.0;
            for (int j = 0; j < L; j++) tq += Mr[j] * alpha[wave][j];
            const double al = alpha[wave][lane];
            part = al * tq - 2.0 * al * bs[(size_t)s * L + lane];
        }
        for (int o = 32; o > 0; o >>= 1) part += __shfl_down(part, o);
        if (lane == 0) chi2[s] = es[s] + part;
        __builtin_amdgcn_wave_barrier();
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
    if (ctx->N > 512) return PSFM_ERR_UNSUPPORTED;
    const size_t need = psfm::solve_workspace(ctx, n_stamps);
    if (!ws || ws_bytes < need) return PSFM_ERR_WORKSPACE;
    const size_t lds = (size_t)std::max(ctx->N * CH_NB, 2600) * sizeof(double);
    if (lds > 150 * 1024) return PSFM_ERR_UNSUPPORTED;
    hipStream_t st = (hipStream_t)stream;
    psfm::Carver c(ws);
    SolveState* state = c.take<SolveState>(1);
    uint8_t* used = c.take<uint8_t>(n_stamps + 1);
    uint8_t* fitted = c.take<uint8_t>(n_stamps + 1);
    double* G = c.take<double>((size_t)n_stamps * ctx->ns + 1);
    double* M = c.take<double>((size_t)ctx->N * ctx->N);
    double* b = c.take<double>(ctx->N);
    double* y = c.take<double>(ctx->N);
    const int nb = ctx->nb, ns = ctx->ns, N = ctx->N, L = ctx->L;
    const psfm_config& cf = ctx->cfg;
    static bool attr_set = false;
    if (!attr_set) {
        PSFM_HIP_CHECK(hipFuncSetAttribute((const void*)k_cholesky,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, 150 * 1024));
        attr_set = true;
    }
    const int nt = std::max(n_stamps, N);
    hipLaunchKernelGGL(k_solve_init, dim3((nt + 255) / 256), dim3(256), 0, st, n_stamps, N, ns,
                       cf.spatial_order, W, H, cf.min_stamps, stamp_xy, stamp_flags, used, fitted,
                       G, stamp_chi2, coeffs, state);
    PSFM_HIP_CHECK(hipGetLastError());
    const int nthreads_asm = L * L * ns + L * ns;
    for (int it = 0; it < cf.max_iter; it++) {
        hipLaunchKernelGGL(k_assemble, dim3((nthreads_asm + 255) / 256), dim3(256), 0, st, n_stamps,
                           nb, ns, N, stamp_M, stamp_b, used, G, M, b, state);
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
