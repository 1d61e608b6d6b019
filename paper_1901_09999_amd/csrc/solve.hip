// Assembly, solution and rejection (Section 2; Sections 3.3, 3.5, 3.6).
//
// Stream-ordered loop of at most max_iter rounds, each made of
//   k_assemble  - M[(i,s),(j,t)] = sum_used g_s g_t M_s[i][j]
//                 (FP64, stamp-major sums, one item per (i, j, s));
//   k_cholesky  - one 512-thread workgroup: symmetric equilibration,
//                 blocked right-looking Cholesky (32-column panels in LDS,
//                 FP64 MFMA trailing update read-modify-write in the
//                 L2-resident workspace), forward and back substitution;
//   16-bit modes: k_resid / k_assemble_vec / k_resolve refinement steps;
//   k_chi2 + k_clip - per-stamp chi2 (from the stamp sums, or from pixels
//                 in the 16-bit modes) and the sigma-clip.
// A device-side state word ends the loop early (converged, or failed);
// later kernels of the unrolled loop then return at once, so the host never
// waits on the device.  Also here: the batched forms (one workgroup per pair
// for the Cholesky), the per-stamp solves and the learned-prior kernels.
#include "internal.h"

namespace {

constexpr int CH_NB = 32;        // Cholesky panel width
constexpr int CH_PS = 33;        // LDS row stride of the panel (doubles)
constexpr int CH_THREADS = 512;
constexpr int CH_NMAX = 496;     // largest system the one-workgroup solver holds

__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}


__device__ void solve_init_body(int n, int N, int ns, int S, int W, int H, int min_stamps,
                                const int32_t* __restrict__ xy, const int32_t* __restrict__ flags,
                                uint8_t* __restrict__ used, uint8_t* __restrict__ fitted,
                                double* __restrict__ G, double* __restrict__ chi2,
                                double* __restrict__ coeffs, SolveState* st, const int bid) {
    const int t = bid * blockDim.x + threadIdx.x;
    if (t < n) {
        const int u = flags[t] == 0;
        used[t] = u;
        fitted[t] = u;
        chi2[t] = 0.0;
        psfm_spatial_terms(S, xy[2 * t], xy[2 * t + 1], W, H, G + (size_t)t * ns);   // no local array
    }
    if (t < N) coeffs[t] = 0.0;
    if (bid == 0) {
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
            st->n_rep = 0;
            st->prior_done = 0;
            st->n_iter_base = 0;
            st->chi2_done = 0;
            st->info = cnt < min_stamps ? PSFM_ERR_TOO_FEW_STAMPS : 0;
            st->done = cnt < min_stamps;
        }
    }
}

// Set-up of a solve: the state, the spatial terms and the stamp masks.
__global__ __launch_bounds__(256) void k_solve_prep(int n, int N, int ns, int S, int W, int H,
                                                    int min_stamps, const int32_t* __restrict__ xy,
                                                    const int32_t* __restrict__ flags,
                                                    uint8_t* __restrict__ used, uint8_t* __restrict__ fitted,
                                                    double* __restrict__ G, double* __restrict__ chi2,
                                                    double* __restrict__ coeffs, SolveState* st) {
    solve_init_body(n, N, ns, S, W, H, min_stamps, xy, flags, used, fitted, G, chi2, coeffs, st, blockIdx.x);
}

__global__ __launch_bounds__(256) void k_solve_prep_b(const PairDesc* __restrict__ pairs, int min_stamps) {
    const PairDesc& p = pairs[blockIdx.y];
    if ((int)blockIdx.x * (int)blockDim.x >= max(max(p.n, p.N), 1)) return;
    solve_init_body(p.n, p.N, p.ns, p.S, p.W, p.H, min_stamps, p.xy, p.flags, p.used, p.fitted, p.G,
                    p.chi2, p.coeffs, p.st, blockIdx.x);
}

// Assembly of the normal equations (Section 2): row (i, p) of M (the
// background row last) is sum over the used stamps s of
// g_s[p] M_s[i][(j, q)] g_s[q].  The rows (i, p) of one term i all read the
// same M_s[i][.], so one workgroup forms a group of PB of them (the
// background row alone in the last group).  Its ASM_WAVES waves each take a
// fixed share of the stamps, in order; lane j keeps the group's entries
// (j, q) for every q in registers, reading M_s[i][j] (consecutive lanes,
// consecutive words); the values every lane needs (the stamps' spatial
// terms and masks) are loaded one per lane for ASM_UNROLL stamps at a time
// and passed through the wave's own LDS slots (read back as broadcasts).
// b's entries are summed per lane (lane r: stamp k0 + r) and reduced at the
// end.  Each stamp sum is read once per group and no transposed copy is
// needed.  The waves' partial sums are added in wave order, so the result
// does not depend on the launch.  JC: columns per lane (L <= 64 JC).
constexpr int ASM_WAVES = 4;
constexpr int ASM_UNROLL = 8;

// rows per group (a divisor of NS).  One: groups of several rows share the
// loads of M_s[i][.], but their accumulators overflow the registers of a
// lane at the occupancy that hides the loads' latency.
template <int NS>
struct AsmRows {
    static constexpr int value = 1;
    static_assert(NS % value == 0, "a group holds whole rows");
};

template <int NS>
__host__ __device__ constexpr int asm_groups(int nb) { return nb * (NS / AsmRows<NS>::value) + 1; }

template <int NS, int JC>
__device__ void assemble_group(int n, int nb, int N, const double* __restrict__ Ms,
                               const double* __restrict__ bs, const double* __restrict__ G,
                               const uint8_t* __restrict__ used, double* __restrict__ M,
                               double* __restrict__ b, const SolveState* st, int grp) {
    constexpr int PB = AsmRows<NS>::value;
    const int NG = asm_groups<NS>(nb);
    if (st->done || grp >= NG) return;                 // uniform over the workgroup
    const int L = nb + 1, j = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const bool bg = grp == NG - 1;
    const int i = bg ? nb : grp / (NS / PB), p0 = bg ? 0 : (grp % (NS / PB)) * PB;
    const size_t LL = (size_t)L * L;
    const double* mrow = Ms + (size_t)i * L;
    constexpr int GV = (ASM_UNROLL * NS + 63) / 64;
    const int k_lo = (int)((long long)n * wave / ASM_WAVES);
    const int k_hi = (int)((long long)n * (wave + 1) / ASM_WAVES);
    __shared__ double bcast[ASM_WAVES][ASM_UNROLL * (NS + PB)];   // per wave: g_s, then g_s[p] u_s
    double* gsh = bcast[wave];
    double acc[PB][JC][NS];
    double bacc[PB];
#pragma unroll
    for (int t = 0; t < PB; t++) {
        bacc[t] = 0.0;
#pragma unroll
        for (int c = 0; c < JC; c++)
#pragma unroll
            for (int q = 0; q < NS; q++) acc[t][c][q] = 0.0;
    }
    for (int k0 = k_lo; k0 < k_hi; k0 += ASM_UNROLL) {
        // lane e < ASM_UNROLL NS: spatial term e % NS of stamp k0 + e / NS;
        // lane r < ASM_UNROLL: stamp k0 + r's mask, b_s[i] and g_s[p0 + t]
        double gv[GV];
#pragma unroll
        for (int t = 0; t < GV; t++) {
            const int e = j + 64 * t;
            gv[t] = (e < ASM_UNROLL * NS && k0 * NS + e < k_hi * NS) ? G[(size_t)k0 * NS + e] : 0.0;
        }
        const int kr = min(k0 + min(j, ASM_UNROLL - 1), k_hi - 1);
        const double uv = (j < ASM_UNROLL && k0 + j < k_hi && used[kr]) ? 1.0 : 0.0;
        const double bvv = bs[(size_t)kr * L + i];
        double gpv[PB];
#pragma unroll
        for (int t = 0; t < PB; t++) {
            gpv[t] = bg ? (t == 0 ? uv : 0.0) : uv * G[(size_t)kr * NS + p0 + t];
            bacc[t] = fma(gpv[t], bvv, bacc[t]);
        }
        double mv[JC][ASM_UNROLL];
#pragma unroll
        for (int c = 0; c < JC; c++)
#pragma unroll
            for (int r = 0; r < ASM_UNROLL; r++)
                mv[c][r] = mrow[(size_t)min(k0 + r, k_hi - 1) * LL + min(j + 64 * c, L - 1)];
        wave_sync();                                  // the previous chunk's reads are done
#pragma unroll
        for (int t = 0; t < GV; t++)
            if (j + 64 * t < ASM_UNROLL * NS) gsh[j + 64 * t] = gv[t];
        if (j < ASM_UNROLL) {
#pragma unroll
            for (int t = 0; t < PB; t++) gsh[ASM_UNROLL * NS + j * PB + t] = gpv[t];
        }
        wave_sync();
#pragma unroll
        for (int r = 0; r < ASM_UNROLL; r++) {
            double g[NS], gp[PB];
#pragma unroll
            for (int q = 0; q < NS; q++) g[q] = gsh[r * NS + q];
#pragma unroll
            for (int t = 0; t < PB; t++) gp[t] = gsh[ASM_UNROLL * NS + r * PB + t];   // 0: unused, k >= k_hi
#pragma unroll
            for (int c = 0; c < JC; c++) {
#pragma unroll
                for (int t = 0; t < PB; t++) {
                    const double w = gp[t] * mv[c][r];
                    if (j + 64 * c < nb) {
#pragma unroll
                        for (int q = 0; q < NS; q++) acc[t][c][q] = fma(g[q], w, acc[t][c][q]);
                    } else {
                        acc[t][c][0] += w;
                    }
                }
            }
        }
    }
    // b's entries: the lanes' sums in a fixed butterfly order
#pragma unroll
    for (int t = 0; t < PB; t++)
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) bacc[t] += __shfl_xor(bacc[t], o);
    // the waves' partial sums, added in wave order by wave 0, one row at a time
    __shared__ double part[ASM_WAVES - 1][JC * NS][64];
#pragma unroll
    for (int t = 0; t < PB; t++) {
        if (wave > 0) {
#pragma unroll
            for (int c = 0; c < JC; c++)
#pragma unroll
                for (int q = 0; q < NS; q++) part[wave - 1][c * NS + q][j] = acc[t][c][q];
        }
        __syncthreads();
        if (wave == 0) {
#pragma unroll
            for (int w = 0; w < ASM_WAVES - 1; w++)
#pragma unroll
                for (int c = 0; c < JC; c++)
#pragma unroll
                    for (int q = 0; q < NS; q++) acc[t][c][q] += part[w][c * NS + q][j];
        }
        __syncthreads();
    }
    __shared__ double bpart[ASM_WAVES][PB];
    if (j == 0) {
#pragma unroll
        for (int t = 0; t < PB; t++) bpart[wave][t] = bacc[t];
    }
    __syncthreads();
    if (wave > 0) return;
#pragma unroll
    for (int t = 0; t < PB; t++) {
        if (bg && t > 0) continue;                    // the background group has one row
        const int row = bg ? N - 1 : i * NS + p0 + t;
#pragma unroll
        for (int c = 0; c < JC; c++) {
            const int jc = j + 64 * c;
            if (jc < nb) {
#pragma unroll
                for (int q = 0; q < NS; q++) M[(size_t)row * N + jc * NS + q] = acc[t][c][q];
            } else if (jc == nb) {
                M[(size_t)row * N + N - 1] = acc[t][c][0];
            }
        }
        if (j == 0) {
            double bsum = bpart[0][t];
#pragma unroll
            for (int w = 1; w < ASM_WAVES; w++) bsum += bpart[w][t];
            b[row] = bsum;
        }
    }
}

// The groups that share a term i (and so read the same M_s[i][.] of every
// stamp) are kept together on one XCD, whose L2 then serves the repeated
// reads: workgroup slot x of a launch whose width is a multiple of 8 runs on
// XCD x % 8, and XCD c takes the c-th of eight contiguous runs of groups.
// -1 for the slots beyond the groups.
__device__ __forceinline__ int xcd_item(int x, int n_items) {
    const int c = x & 7, k = x >> 3, q = n_items >> 3, r = n_items & 7;
    return k < q + (c < r) ? c * q + min(c, r) + k : -1;
}

template <int NS, int JC>
__global__ __launch_bounds__(64 * ASM_WAVES) void k_assemble(int n, int nb, int N,
                                                             const double* __restrict__ Ms,
                                                             const double* __restrict__ bs,
                                                             const double* __restrict__ G,
                                                             const uint8_t* __restrict__ used,
                                                             double* __restrict__ M, double* __restrict__ b,
                                                             const SolveState* st) {
    const int grp = xcd_item(blockIdx.x, asm_groups<NS>(nb));
    if (grp >= 0) assemble_group<NS, JC>(n, nb, N, Ms, bs, G, used, M, b, st, grp);
}

// Batched: the launch covers the pairs with NS spatial terms, listed in plist.
template <int NS>
__global__ __launch_bounds__(64 * ASM_WAVES) void k_assemble_b(const PairDesc* __restrict__ pairs,
                                                               const int* __restrict__ plist, int nb) {
    const PairDesc& p = pairs[plist[blockIdx.y]];
    const int grp = xcd_item(blockIdx.x, asm_groups<NS>(nb));
    if (p.ns != NS || grp < 0) return;
    assemble_group<NS, 1>(p.n, nb, p.N, p.Ms, p.bs, p.G, p.used, p.A, p.b, p.st, grp);
}

// Launch width of an assembly: the groups, rounded up to a multiple of 8 (see xcd_item).
template <int NS>
int asm_width(int nb) { return (asm_groups<NS>(nb) + 7) / 8 * 8; }


__device__ __forceinline__ double block_sum(double v, double* red) { return psfm_block_sum(v, red); }

typedef double double4v __attribute__((ext_vector_type(4)));

__device__ __forceinline__ double rsqrt_nr(double d) {
    double r = __builtin_amdgcn_rsq(d);
    r = r * (1.5 - 0.5 * d * r * r);
    r = r * (1.5 - 0.5 * d * r * r);
    return r;
}

// 1/d: v_rcp_f64 (relative error e, |e| < 2^-23), then the third-order
// correction 1/d = r / (1 - e) ~ r (1 + e + e^2), truncation e^3: three
// dependent operations after the estimate, where two Newton steps take four.
__device__ __forceinline__ double rcp_nr(double d) {
    const double r = __builtin_amdgcn_rcp(d);
    const double e = fma(-d, r, 1.0);
    return fma(r, fma(e, e, e), r);
}

// Value of v in lane l of the wave (l a compile-time constant after unrolling).
__device__ __forceinline__ double readlane_d(double v, int l) {
    const long long u = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)(u & 0xffffffffll), l);
    const int hi = __builtin_amdgcn_readlane((int)(u >> 32), l);
    return __hiloint2double(hi, lo);
}

constexpr int PL_CHUNK = 8;      // panel rows in flight per thread
constexpr int IV_DOUBLES = CH_NB * CH_NB;   // stored inverse of one 32 x 32 diagonal block

// Rows [r_lo, r_hi) (relative to k0) of the 32 panel columns k0 .. k0 + 31:
// the lower triangle of S (row stride N) for rows below r_end and columns
// below nk, zeros elsewhere, into P[(r) * CH_PS + c].  With Dq given, each
// element is equilibrated on the way (S d_i d_j).  Loads are unconditional
// from clamped addresses, PL_CHUNK per thread in flight before the first
// store.
__device__ __forceinline__ void load_panel(int N, const double* __restrict__ S, int k0, int nk,
                                           int r_lo, int r_hi, int r_end, double* P,
                                           const double* Dq) {
    const int tr = threadIdx.x >> 5, tc = threadIdx.x & 31, TR = CH_THREADS / 32;
    for (int base = r_lo + tr; base < r_hi; base += TR * PL_CHUNK) {
        double v[PL_CHUNK];
#pragma unroll
        for (int u = 0; u < PL_CHUNK; u++) {
            const int i = base + TR * u;
            const bool in = i < r_end && tc < nk && (i >= nk || tc <= i);
            v[u] = S[in ? (k0 + i) * N + k0 + tc : 0];
        }
#pragma unroll
        for (int u = 0; u < PL_CHUNK; u++) {
            const int i = base + TR * u;
            const bool in = i < r_end && tc < nk && (i >= nk || tc <= i);
            if (i < r_hi) P[i * CH_PS + tc] = !in ? 0.0 : Dq ? v[u] * (Dq[k0 + i] * Dq[k0 + tc]) : v[u];
        }
    }
}

// z <- Iv z over the panel's unknowns (forward substitution through the
// diagonal block), by the first 32 lanes of wave 0.
__device__ __forceinline__ void diag_forward(int k0, int nk, const double* Iv, double* zb) {
    const int lane = threadIdx.x & 63;
    double z = 0.0;
    if (lane < CH_NB) {
        double s4[4] = {0.0, 0.0, 0.0, 0.0};      // FP64 latency: four independent chains
#pragma unroll
        for (int k = 0; k < CH_NB; k++) s4[k & 3] += Iv[lane * CH_PS + k] * zb[k0 + k];
        z = (s4[0] + s4[1]) + (s4[2] + s4[3]);
    }
    wave_sync();
    if (lane < nk) zb[k0 + lane] = z;
}

// The stored diagonal-block inverses of an N-unknown factor into P when
// they fit there (returns whether they did).
__device__ __forceinline__ bool stage_inverses(int N, const double* __restrict__ ILg, double* P) {
    const int np = (N + CH_NB - 1) / CH_NB;
    const bool staged = np * IV_DOUBLES <= (max(N, CH_NB) + 16) * CH_PS;
    if (staged) {
        constexpr int CHUNK = 8;        // loads in flight per thread
        const int total = np * IV_DOUBLES;
        for (int e0 = threadIdx.x; e0 < total; e0 += CH_THREADS * CHUNK) {
            double v[CHUNK];
#pragma unroll
            for (int u = 0; u < CHUNK; u++) v[u] = ILg[min(e0 + CH_THREADS * u, total - 1)];
#pragma unroll
            for (int u = 0; u < CHUNK; u++)
                if (e0 + CH_THREADS * u < total) P[e0 + CH_THREADS * u] = v[u];
        }
    }
    __syncthreads();
    return staged;
}

// The LDS copy of panel q's stored inverse: in place when all of them were
// staged, else loaded into the head of P (which always holds one).  Every
// thread of the workgroup calls it, after a barrier that follows the
// previous step's reads.
__device__ __forceinline__ const double* step_inverse(int q, bool staged, const double* __restrict__ ILg,
                                                      double* P) {
    if (staged) return P + q * IV_DOUBLES;
    for (int e = threadIdx.x; e < IV_DOUBLES; e += CH_THREADS) P[e] = ILg[(size_t)q * IV_DOUBLES + e];
    __syncthreads();
    return P;
}

// Row (TRANS = false) or column (TRANS = true) `lane` of a 32 x 32 inverse
// in LDS times z[0..31]; four independent FP64 chains.
template <bool TRANS>
__device__ __forceinline__ double iv_dot(const double* __restrict__ iv, const double* z, int lane) {
    double s4[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int k = 0; k < CH_NB; k++) s4[k & 3] += iv[TRANS ? k * CH_NB + lane : lane * CH_NB + k] * z[k];
    return (s4[0] + s4[1]) + (s4[2] + s4[3]);
}

// Forward substitution L z = z (z in LDS, overwritten) with a stored factor
// (its entries below the diagonal blocks from the transposed copy LT),
// right-looking: z_q = Iv_q z_q (wave 0), then every row below the panel
// takes it out, z_i -= sum_t L(i, q0 + t) z_(q0 + t) (one thread per row).
// The rows of the next panel are loaded during this panel's update (two
// register sets, the step loop unrolled by two so that they swap without a
// copy), so that no load stands in front of wave 0's z_q, the serial chain.
// Inverses as in back_subst.
__device__ __forceinline__ void forward_subst(int N, const double* __restrict__ LT,
                                              const double* __restrict__ ILg, double* zb, double* P,
                                              bool staged, double* wq) {
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int np = (N + CH_NB - 1) / CH_NB;
    // row q0 + nk + tid's nk entries of panel q from the transposed factor
    // (LT[c][i] = L(i, c): consecutive rows are consecutive words, so a load
    // instruction touches a few cache lines, not one per lane; zeros beyond
    // nk); a wave with no row below the panel issues no loads (the vector
    // memory pipeline, not the bytes, bounds these steps)
    auto load_row = [&](int q, double* lv) {
        const int q0 = q * CH_NB, nk = min(CH_NB, N - q0);
        const bool need = wave * 64 < N - q0 - nk;
        const double* col = LT + (size_t)q0 * N + min(q0 + nk + tid, N - 1);
#pragma unroll
        for (int t = 0; t < CH_NB; t++) {
            if (need && t < nk) lv[t] = col[(size_t)t * N];
            else lv[t] = 0.0;
        }
    };
    auto step = [&](int q, const double* lv, double* ln) {
        const int q0 = q * CH_NB, nk = min(CH_NB, N - q0);
        const int i = q0 + nk + tid;
        const double* iv = step_inverse(q, staged, ILg, P);
        if (wave == 0) {
            double z = 0.0;
            if (lane < CH_NB) {
                z = iv_dot<false>(iv, zb + q0, lane);
                wq[lane] = z;
            }
            wave_sync();
            if (lane < nk) zb[q0 + lane] = z;
        }
        __syncthreads();
        if (q + 1 < np) load_row(q + 1, ln);
        if (i < N) {
            double s4[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
            for (int t = 0; t < CH_NB; t++) s4[t & 3] += lv[t] * wq[t];
            zb[i] -= (s4[0] + s4[1]) + (s4[2] + s4[3]);
        }
        __syncthreads();
    };
    double la[CH_NB], lb[CH_NB];
    load_row(0, la);
    for (int q = 0; q < np; q += 2) {
        step(q, la, lb);
        if (q + 1 < np) step(q + 1, lb, la);
    }
}

// Back substitution L^T w = z with the factor in the lower triangle of A and
// the stored diagonal-block inverses; z (LDS) is overwritten by w.  Panels in
// reverse, right-looking: w_q = Iv_q^T z_q (wave 0), then the block row of L
// left of the diagonal block takes w_q out of every earlier unknown,
// z_c -= sum_t L(q0 + t, c) w_t (one thread per column c).  The block row
// of the next panel is loaded during this panel's update, as in
// forward_subst.  The inverses are read from P (staged there by
// stage_inverses, or one per step).  wq (>= CH_NB doubles) is LDS scratch of
// the caller.
static_assert(CH_NMAX <= CH_THREADS, "one thread per unknown left of a panel");
__device__ __forceinline__ void back_subst(int N, const double* __restrict__ A, const double* __restrict__ ILg,
                           double* zb, double* P, bool staged, double* wq) {
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int np = (N + CH_NB - 1) / CH_NB;
    // column tid of panel q's block row (zeros in rows beyond nk); a wave
    // with no column left of the panel issues no loads
    auto load_col = [&](int q, double* lv) {
        const int q0 = q * CH_NB, nk = min(CH_NB, N - q0);
        const bool need = wave * 64 < q0;
        const double* col = A + (size_t)q0 * N + min(tid, max(q0 - 1, 0));
#pragma unroll
        for (int t = 0; t < CH_NB; t++) {
            if (need && t < nk) lv[t] = col[(size_t)t * N];
            else lv[t] = 0.0;
        }
    };
    auto step = [&](int q, const double* lv, double* ln) {
        const int q0 = q * CH_NB, nk = min(CH_NB, N - q0);
        const double* iv = step_inverse(q, staged, ILg, P);
        if (wave == 0) {
            double wv = 0.0;
            if (lane < CH_NB) {
                wv = iv_dot<true>(iv, zb + q0, lane);
                wq[lane] = wv;
            }
            wave_sync();
            if (lane < nk) zb[q0 + lane] = wv;
        }
        __syncthreads();
        if (q > 0) load_col(q - 1, ln);
        if (tid < q0) {
            double s4[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
            for (int t = 0; t < CH_NB; t++) s4[t & 3] += lv[t] * wq[t];
            zb[tid] -= (s4[0] + s4[1]) + (s4[2] + s4[3]);
        }
        __syncthreads();
    };
    double la[CH_NB], lb[CH_NB];
    load_col(np - 1, la);
    for (int q = np - 1; q >= 0; q -= 2) {
        step(q, la, lb);
        if (q - 1 >= 0) step(q - 1, lb, la);
    }
}

// Cholesky of the nk x nk diagonal block in rows 0 .. nk - 1 of Q (row
// stride CH_PS, lower triangle, zeros above and beyond nk), by one wave,
// delivered as the inverse of its factor: L^(-1) (32 x 32, zeros above the
// diagonal and in the rows beyond nk) into Iv (LDS, row stride CH_PS) and
// ivg.  Q is not modified.
//   Lanes 0-31 hold the rows of the block in registers, lanes 32-63 the
//   columns of X = L_unit^(-1), starting from the identity.  Step c of the
//   right-looking L D L^T elimination is one instruction stream for both
//   halves:  v_u -= (v_c / d_c) col_u  for u > c,  col = column c of the
//   partly reduced block.  On a block row this is the rank-one update; on a
//   column of X it is forward substitution with the unit factor
//   (X_uk -= L_uc X_ck), so the inverse costs no instructions of its own.
//   The pivot chain d_(c+1) = A_(c+1,c+1) - A_(c+1,c)^2 / d_c reads its
//   operands from the pivot row's lane; each column reaches all lanes
//   through a double-buffered LDS column (cb), read at the end of the step
//   that finishes it, so that the read overlaps the next reciprocal.  The
//   32 steps are straight-line code (LDS accesses of one wave are ordered).
//   Finally L^(-1) = D^(-1/2) X.
// dd, ds: LDS [32] scratch.  Returns 0, or the 1-based column of the first
// non-positive pivot.
__device__ __forceinline__ int factor_diag(int nk, const double* Q, double* Iv, double* __restrict__ ivg,
                                           double (*cb)[64], double* dd, double* ds) {
    const int lane = threadIdx.x & 63, row = lane & 31;
    const bool xl = lane >= 32;
    double r[CH_NB], col[CH_NB];
    {
        // every lane loads (clamped row), then v * keep + identity: no
        // branches.  Rows beyond nk are identity rows, so that their pivots
        // are 1 and the pivot chain needs no select.  self is made opaque so
        // that the identity is formed here, not hoisted out of the caller's
        // loop and kept in registers.
        const int qr = xl || row >= nk ? 0 : row;
        const double keep = xl || row >= nk ? 0.0 : 1.0;
        int self = xl || row >= nk ? row : -1;
        asm volatile("" : "+v"(self));
#pragma unroll
        for (int c = 0; c < CH_NB; c++)
            r[c] = fma(Q[qr * CH_PS + c], keep, c == self ? 1.0 : 0.0);
    }
    cb[0][lane] = r[0];
#pragma unroll
    for (int u = 1; u < CH_NB; u++) col[u] = cb[0][u];
    // The pivot of step c + 1 and its reciprocal (rcp_nr's stages) are
    // formed during step c, one stage between consecutive batches of the
    // step's updates, so that the chain's latency is covered by them (the
    // wave issues in order).  Empty asm statements fix that order: a stage's
    // result and the multiplier pass through one before the next batch, and
    // each batch's rows through one before the next stage.  The chain has no
    // select: a non-positive pivot is recorded (bad) and the factorization
    // is then abandoned by the caller.
    int bad = 0;
    double rc;
    {
        const double d = readlane_d(r[0], 0);
        bad = 0 < nk && !(d > 0.0) ? 1 : 0;
        if (lane == 0) dd[0] = d;
        rc = rcp_nr(d);
    }
#pragma unroll
    for (int c = 0; c < CH_NB; c++) {
        const int n = CH_NB - 1 - c, s1 = n / 3, s2 = (2 * n) / 3;
        // finished rows (and the pivot row) are left alone
        double t = (xl || row > c) ? r[c] * rc : 0.0;
        double d = 1.0, y = 1.0;
        if (c + 1 < CH_NB) {
            const double a = readlane_d(r[c + 1], c + 1), q = readlane_d(r[c], c + 1);
            d = fma(-q * q, rc, a);
            bad = (bad == 0 && c + 1 < nk && !(d > 0.0)) ? c + 2 : bad;
            if (lane == 0) dd[c + 1] = d;
            y = __builtin_amdgcn_rcp(d);
        }
        asm volatile("" : "+v"(t), "+v"(y));
        auto batch = [&](int k0, int k1) {
#pragma unroll
            for (int k = k0; k < k1; k++) {
                r[c + 1 + k] -= t * col[c + 1 + k];
                if (k == 0) cb[(c + 1) & 1][lane] = r[c + 1];
            }
#pragma unroll
            for (int k = k0; k < k1; k++) asm volatile("" : "+v"(r[c + 1 + k]));
        };
        batch(0, s1);
        double e = fma(-d, y, 1.0);
        asm volatile("" : "+v"(t), "+v"(e));
        batch(s1, s2);
        e = fma(e, e, e);
        asm volatile("" : "+v"(t), "+v"(e));
        batch(s2, n);
        const double rcn = fma(y, e, y);      // 1/d (1 + e + e^2), as rcp_nr
        // column c + 1, for the next step
#pragma unroll
        for (int u = c + 2; u < CH_NB; u++) col[u] = cb[(c + 1) & 1][u];
        rc = rcn;
    }
    if (bad) return bad;
    if (lane < CH_NB) ds[lane] = lane < nk ? rsqrt_nr(dd[lane]) : 0.0;
    wave_sync();
    if (xl) {
#pragma unroll
        for (int i = 0; i < CH_NB; i++) {
            const double v = r[i] * ds[i];
            Iv[i * CH_PS + row] = v;
            ivg[i * CH_NB + row] = v;
        }
    }
    wave_sync();
    return 0;
}

// Trailing update of one 32 x 32 block (block row a2 >= block column b2 of
// the lower triangle below the panel):  C <- C - L_a L_b^T  with L_a, L_b
// the panel rows (in P) of the block's rows and columns, as four 16 x 16
// tiles on v_mfma_f64_16x16x4f64 (three on a diagonal block).  C comes from
// S, equilibrated by Dq when given (the first touch of that element); the
// product runs from zero while the C loads are in flight.  Results go to A,
// or, with Dn given (the block that is the next diagonal block), to Dn with
// zeros above the diagonal and beyond the matrix.  Blocks wholly inside the
// lower triangle take a path without per-element predicates.
__device__ __forceinline__ void trail_block(int N, int k0, int nk, int rows, int a2, int b2,
                                            const double* __restrict__ S, double* __restrict__ A,
                                            const double* Dq, const double* P, double* Dn) {
    const int lane = threadIdx.x & 63, l16 = lane & 15, l4 = lane >> 4;
    const int r0 = nk + 32 * a2, c0 = nk + 32 * b2;      // relative to k0
    const bool diag = a2 == b2;
    const bool full = !diag && r0 + 32 <= rows && !Dq && !Dn;
    const int base = (k0 + r0 + l4) * N + k0 + c0 + l16;  // element (r0 + l4, c0 + l16)
    double4v c[4], acc[4];
    // sub-tile s = 2 sr + sc: rows r0 + 16 sr + l4 + 4 e, columns c0 + 16 sc + l16
    if (full) {
#pragma unroll
        for (int s = 0; s < 4; s++)
#pragma unroll
            for (int e = 0; e < 4; e++) c[s][e] = S[base + (16 * (s >> 1) + 4 * e) * N + 16 * (s & 1)];
    } else {
#pragma unroll
        for (int s = 0; s < 4; s++)
#pragma unroll
            for (int e = 0; e < 4; e++) {
                const int ii = r0 + 16 * (s >> 1) + l4 + 4 * e, jj = c0 + 16 * (s & 1) + l16;
                const bool in = ii < rows && jj <= ii;
                c[s][e] = S[in ? base + (16 * (s >> 1) + 4 * e) * N + 16 * (s & 1) : 0];
            }
    }
#pragma unroll
    for (int s = 0; s < 4; s++) acc[s] = double4v{0.0, 0.0, 0.0, 0.0};
    // operand rows beyond the panel buffer are clamped (their outputs are discarded)
    const int rmax = rows + 15;
    const double* pa0 = P + (r0 + l16) * CH_PS + l4;
    const double* pa1 = P + min(r0 + 16 + l16, rmax) * CH_PS + l4;
    const double* pb0 = P + (c0 + l16) * CH_PS + l4;
    const double* pb1 = P + min(c0 + 16 + l16, rmax) * CH_PS + l4;
    if (diag) {
#pragma unroll
        for (int cc = 0; cc < CH_NB; cc += 4) {
            const double a0 = pa0[cc], a1 = pa1[cc], b0 = pb0[cc], b1 = pb1[cc];
            acc[0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b0, acc[0], 0, 0, 0);
            acc[2] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b0, acc[2], 0, 0, 0);
            acc[3] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b1, acc[3], 0, 0, 0);
        }
    } else {
#pragma unroll
        for (int cc = 0; cc < CH_NB; cc += 4) {
            const double a0 = pa0[cc], a1 = pa1[cc], b0 = pb0[cc], b1 = pb1[cc];
            acc[0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b0, acc[0], 0, 0, 0);
            acc[1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b1, acc[1], 0, 0, 0);
            acc[2] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b0, acc[2], 0, 0, 0);
            acc[3] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b1, acc[3], 0, 0, 0);
        }
    }
    if (full) {
#pragma unroll
        for (int s = 0; s < 4; s++)
#pragma unroll
            for (int e = 0; e < 4; e++)
                A[base + (16 * (s >> 1) + 4 * e) * N + 16 * (s & 1)] = c[s][e] - acc[s][e];
        return;
    }
#pragma unroll
    for (int s = 0; s < 4; s++)
#pragma unroll
        for (int e = 0; e < 4; e++) {
            const int ii = r0 + 16 * (s >> 1) + l4 + 4 * e, jj = c0 + 16 * (s & 1) + l16;
            const bool in = ii < rows && jj <= ii;
            const double cv = Dq && in ? c[s][e] * (Dq[k0 + ii] * Dq[k0 + jj]) : c[s][e];
            const double v = cv - acc[s][e];
            if (Dn) Dn[(ii - nk) * CH_PS + (jj - nk)] = in ? v : 0.0;
            else if (in) A[base + (16 * (s >> 1) + 4 * e) * N + 16 * (s & 1)] = v;
        }
}

// Equilibrated blocked right-looking Cholesky and solve of the N x N system
// M x = b; M's lower triangle is read from S (M itself, or a separate copy).
// Of the factor L of D M D (D = diag(M)^(-1/2)) the blocks below the
// diagonal are left in the lower triangle of A and the 32 x 32 diagonal
// blocks as their inverses in ILg (A's diagonal blocks are not written);
// x receives the solution.  One workgroup.  Per 32-column panel (in LDS):
//   * the panel rows below the diagonal block are multiplied by the inverse
//     of its factor (FP64 MFMA, 16-row tiles, one wave each);
//   * the forward substitution L z = D b advances by the panel's unknowns;
//   * the trailing lower triangle is updated on FP64 MFMA in 32 x 32 blocks
//     handed out to the waves from an LDS counter.  Wave 0 first forms the
//     block that is the next diagonal block, in LDS, and factors and inverts
//     it (look-ahead), so the serial pivot chain of the next panel overlaps
//     the update of the rest of the matrix.
// Equilibration happens on each element's first read (the first panel and
// the first trailing update), so M is read once.  The back substitution
// L^T w = z walks the panels in reverse with the stored inverses (IV_DOUBLES
// per panel in ILg).
__device__ __forceinline__ void cholesky_body(int N, double* __restrict__ A, const double* __restrict__ S,
                              const double* __restrict__ b,
                              double* __restrict__ x, double* __restrict__ ILg,
                              double* __restrict__ Dg, SolveState* st,
                              double* __restrict__ LT = nullptr) {
    if (st->done) return;
    extern __shared__ double P[];        // panel [max(N, 32) + 16][CH_PS]
    __shared__ double Dq[CH_NMAX];
    __shared__ double zb[CH_NMAX + 32];
    __shared__ double Iv[CH_NB * CH_PS];  // inverse of the current diagonal block
    __shared__ double Dn[CH_NB * CH_PS];  // next diagonal block; back substitution partials
    __shared__ double cb[2][64];
    __shared__ double dd[CH_NB], ds[CH_NB];
    __shared__ int s_bad, s_next, s_d0;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    constexpr int NW = CH_THREADS / 64;
    if (tid == 0) s_bad = 0;
    __syncthreads();
    for (int i = tid; i < N; i += CH_THREADS) {
        const double d = S[i * N + i];
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
    for (int i = tid; i < N + 32; i += CH_THREADS) {
        zb[i] = i < N ? Dq[i] * b[i] : 0.0;
        if (Dg && i < N) Dg[i] = Dq[i];
    }
    // first panel: read (equilibrated) and factor its diagonal block
    {
        const int nk = min(CH_NB, N);
        load_panel(N, S, 0, nk, 0, N + 16, N, P, Dq);
        if (tid == 0) {
            s_next = 1;
            s_d0 = 0;
        }
        __syncthreads();
        if (wave == 0) {
            const int bad = factor_diag(nk, P, Iv, ILg, cb, dd, ds);
            if (lane == 0) s_bad = bad;
        }
        __syncthreads();
    }
    const int l16 = lane & 15, l4 = lane >> 4;
    for (int k0 = 0; k0 < N; k0 += CH_NB) {
        const int nk = min(CH_NB, N - k0);
        const int rows = N - k0;
        if (k0 > 0) {
            // diagonal block: factored by the look-ahead; rows below from A
            load_panel(N, A, k0, nk, nk, rows + 16, rows, P, nullptr);
            if (tid == 0) {
                s_next = 1;
                s_d0 = 0;
            }
            __syncthreads();
        }
        if (s_bad) {
            if (tid == 0) {
                st->info = k0 + s_bad;
                st->done = 1;
            }
            return;
        }
        // ---- panel rows below the diagonal block: X = A_below Iv^T, 16-row
        //      tiles on MFMA (the tile's operands are read before it is written)
        const int m = rows - nk;
        if (m > 0) {
            const int nt = (m + 15) / 16;
            for (int t = wave; t < nt; t += NW) {
                const int r0 = nk + 16 * t;
                double a[CH_NB / 4];
#pragma unroll
                for (int q = 0; q < CH_NB / 4; q++) a[q] = P[(r0 + l16) * CH_PS + 4 * q + l4];
                double4v x0 = {0.0, 0.0, 0.0, 0.0}, x1 = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
                for (int q = 0; q < 4; q++)
                    x0 = __builtin_amdgcn_mfma_f64_16x16x4f64(a[q], Iv[l16 * CH_PS + 4 * q + l4], x0, 0, 0, 0);
#pragma unroll
                for (int q = 0; q < CH_NB / 4; q++)
                    x1 = __builtin_amdgcn_mfma_f64_16x16x4f64(a[q], Iv[(16 + l16) * CH_PS + 4 * q + l4], x1, 0, 0, 0);
                wave_sync();
#pragma unroll
                for (int e = 0; e < 4; e++) {
                    P[(r0 + l4 + 4 * e) * CH_PS + l16] = x0[e];
                    P[(r0 + l4 + 4 * e) * CH_PS + 16 + l16] = x1[e];
                }
            }
        }
        // ---- forward substitution for the panel's unknowns (wave 0)
        if (wave == 0) diag_forward(k0, nk, Iv, zb);
        __syncthreads();
        for (int i = nk + tid; i < rows; i += CH_THREADS) {
            double s4[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
            for (int c = 0; c < CH_NB; c++) s4[c & 3] += P[i * CH_PS + c] * zb[k0 + c];
            zb[k0 + i] -= (s4[0] + s4[1]) + (s4[2] + s4[3]);
        }
        {
            const int tr = tid >> 5, tc = tid & 31, TR = CH_THREADS / 32;
            for (int i = nk + tr; i < rows; i += TR)
                if (tc < nk) A[(k0 + i) * N + k0 + tc] = P[i * CH_PS + tc];
        }
        if (LT) {
            // the same entries transposed, LT[c][i] = L(i, c), for the
            // refinement's forward substitution (coalesced reads there)
            const int ti = tid & 63;
            for (int c = tid >> 6; c < nk; c += CH_THREADS / 64)
                for (int i = nk + ti; i < rows; i += 64)
                    LT[(size_t)(k0 + c) * N + k0 + i] = P[i * CH_PS + c];
        }
        // ---- trailing update, with the next diagonal block first (wave 0)
        if (m > 0) {
            const int mt = (m + 31) / 32;
            const int nblk = mt * (mt + 1) / 2;
            const double* src = k0 == 0 ? S : A;
            const double* dq = k0 == 0 ? Dq : nullptr;
            if (wave == 0) {
                // the serial chain of the next panel: first in issue order on its SIMD
                __builtin_amdgcn_s_setprio(3);
                trail_block(N, k0, nk, rows, 0, 0, src, A, dq, P, Dn);
                wave_sync();
                if (lane == 0) __hip_atomic_store(&s_d0, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
                const int bad = factor_diag(min(CH_NB, m), Dn, Iv,
                                            ILg + (size_t)((k0 + nk) / CH_NB) * IV_DOUBLES, cb, dd, ds);
                if (lane == 0) s_bad = bad;
                __builtin_amdgcn_s_setprio(0);
            }
            if (wave == NW / 2) {
                // the wave that shares wave 0's SIMD keeps off the matrix unit
                // until the next diagonal block is formed (bounded wait)
                for (int spin = 0; spin < 4096; spin++) {
                    if (__hip_atomic_load(&s_d0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP)) break;
                    __builtin_amdgcn_s_sleep(1);
                }
            }
            for (;;) {
                int g = 0;
                if (lane == 0) g = atomicAdd(&s_next, 1);
                g = __shfl(g, 0);
                if (g >= nblk) break;
                int a2 = (int)((sqrtf(8.0f * g + 1.0f) - 1.0f) * 0.5f);
                while ((a2 + 1) * (a2 + 2) / 2 <= g) a2++;
                while (a2 * (a2 + 1) / 2 > g) a2--;
                trail_block(N, k0, nk, rows, a2, g - a2 * (a2 + 1) / 2, src, A, dq, P, nullptr);
            }
        }
        __syncthreads();
    }
    {
        const bool staged = stage_inverses(N, ILg, P);
        back_subst(N, A, ILg, zb, P, staged, Dn);
    }
    for (int i = tid; i < N; i += CH_THREADS) x[i] = Dq[i] * zb[i];
}

// OWN: the standalone solve (psfm_cholesky_solve) reads M from a separate
// matrix (left untouched) and reports the pivot status; a separate
// instantiation, so that profiles tell the two uses apart.
template <bool OWN>
__global__ __launch_bounds__(CH_THREADS) void k_cholesky(int N, double* __restrict__ A,
                                                         const double* __restrict__ b,
                                                         double* __restrict__ x,
                                                         double* __restrict__ ILg,
                                                         double* __restrict__ Dg, SolveState* st,
                                                         const double* __restrict__ Msrc,
                                                         int* __restrict__ info,
                                                         double* __restrict__ LT) {
    if (OWN) {
        if (threadIdx.x == 0) {
            st->done = 0;
            st->info = 0;
        }
        __syncthreads();
    }
    cholesky_body(N, A, OWN ? Msrc : A, b, x, ILg, Dg, st, LT);
    if (OWN) {
        __syncthreads();
        if (threadIdx.x == 0) *info = st->info;
    }
}

// Batched: one workgroup per pair, all solved concurrently.
__global__ __launch_bounds__(CH_THREADS) void k_cholesky_b(const PairDesc* __restrict__ pairs) {
    const PairDesc& p = pairs[blockIdx.x];
    cholesky_body(p.N, p.A, p.A, p.b, p.coeffs, p.ILg, nullptr, p.st);
}

// Solution of M d = g with the factor left by cholesky_body (equilibrated
// lower triangle in A, 1/sqrt(diag M) in Dg, the diagonal-block inverses in
// ILg); x += d.  One workgroup.  This is the correction step of the
// iterative refinement of the 16-bit modes.
__device__ __forceinline__ void resolve_body(int N, const double* __restrict__ A, const double* __restrict__ LT,
                             const double* __restrict__ ILg,
                             const double* __restrict__ Dg, const double* __restrict__ g,
                             double* __restrict__ x, const SolveState* st) {
    if (st->done) return;
    extern __shared__ double P[];
    __shared__ double zb[CH_NMAX + 32];
    __shared__ double Dq[CH_NMAX];
    __shared__ double wq[CH_NB];
    const int tid = threadIdx.x;
    for (int i = tid; i < N + 32; i += CH_THREADS) {
        zb[i] = i < N ? Dg[i] * g[i] : 0.0;
        if (i < N) Dq[i] = Dg[i];
    }
    const bool staged = stage_inverses(N, ILg, P);    // (its barrier also orders zb)
    forward_subst(N, LT, ILg, zb, P, staged, wq);     // L z = D g
    back_subst(N, A, ILg, zb, P, staged, wq);
    for (int i = tid; i < N; i += CH_THREADS) x[i] += Dq[i] * zb[i];
}

__global__ __launch_bounds__(CH_THREADS) void k_resolve(int N, const double* __restrict__ A,
                                                        const double* __restrict__ LT,
                                                        const double* __restrict__ ILg,
                                                        const double* __restrict__ Dg,
                                                        const double* __restrict__ g,
                                                        double* __restrict__ x, const SolveState* st) {
    resolve_body(N, A, LT, ILg, Dg, g, x, st);
}

// Pixel residuals of every fitted stamp at the current coefficients, from
// the FP32 stamp design [nb + 2][npix] (terms, sqrt(w), d~) left by the fit:
//   e = d~ - sum_c design_c alpha_c,  chi2_s = e^T e,  g_s = design^T e
// with FP64 accumulation; g_s goes stamp-major to gt[c * n + s].
// Phase 1: one pixel per thread, e kept in LDS; phase 2: one wave per column,
// the lanes striding over the pixels (coalesced), then a wave sum.
constexpr int RES_MAXPIX = (2 * PSFM_RMAX + 1) * (2 * PSFM_RMAX + 1);
constexpr int RES_T = 1024;        // threads of k_resid (one workgroup per stamp)

__global__ __launch_bounds__(RES_T) void k_resid(int n, int nb, int ns, int N, int npix,
                                                 const float* __restrict__ design,
                                                 const double* __restrict__ G,
                                                 const double* __restrict__ a,
                                                 const uint8_t* __restrict__ fitted,
                                                 double* __restrict__ gt, double* __restrict__ chi2,
                                                 const SolveState* st) {
    if (st->done) return;
    const int s = blockIdx.x, tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    constexpr int NWV = RES_T / 64, CPW = (64 + NWV - 1) / NWV;   // columns per wave, max
    const int L = nb + 1;
    __shared__ double alpha[64];
    __shared__ float ebuf[RES_MAXPIX];
    __shared__ double red[16];
    if (!fitted[s]) {
        if (tid < L) gt[(size_t)tid * n + s] = 0.0;
        return;
    }
    if (tid < L) {
        double al;
        if (tid < nb) {
            al = 0.0;
            for (int q = 0; q < ns; q++) al += a[tid * ns + q] * G[(size_t)s * ns + q];
        } else {
            al = a[N - 1];
        }
        alpha[tid] = al;
    }
    __syncthreads();
    const float* D = design + (size_t)s * (nb + 2) * npix;
    // 1. residual per pixel, e = d~ - sum_c alpha_c A~_c: four partial sums,
    //    the columns' loads of a group of eight issued together
    double chi = 0.0;
    for (int p = tid; p < npix; p += RES_T) {
        double e4[4] = {(double)D[(size_t)(nb + 1) * npix + p], 0.0, 0.0, 0.0};
        int c = 0;
        for (; c + 8 <= L; c += 8) {
            float dv[8];
#pragma unroll
            for (int k = 0; k < 8; k++) dv[k] = D[(size_t)(c + k) * npix + p];
#pragma unroll
            for (int k = 0; k < 8; k++) e4[k & 3] -= alpha[c + k] * (double)dv[k];
        }
        for (; c < L; c++) e4[c & 3] -= alpha[c] * (double)D[(size_t)c * npix + p];
        const double e = (e4[0] + e4[1]) + (e4[2] + e4[3]);
        chi += e * e;
        ebuf[p] = (float)e;
    }
    chi = psfm_block_sum(chi, red);     // also orders ebuf before phase 2
    // 2. g_c = sum_p A~_c(p) e(p): wave w takes the columns w, w + NWV, ...,
    //    every lane one pixel of each at a time (all the wave's column loads
    //    for a pixel issued together)
    double acc[CPW];
#pragma unroll
    for (int k = 0; k < CPW; k++) acc[k] = 0.0;
#pragma unroll 4
    for (int p = lane; p < npix; p += 64) {
        const double e = (double)ebuf[p];
        float dv[CPW];
#pragma unroll
        for (int k = 0; k < CPW; k++) {
            const int c = wave + NWV * k;
            dv[k] = D[(size_t)(c < L ? c : 0) * npix + p];
        }
#pragma unroll
        for (int k = 0; k < CPW; k++) acc[k] += (double)dv[k] * e;
    }
#pragma unroll
    for (int k = 0; k < CPW; k++) {
        double v = acc[k];
        for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
        const int c = wave + NWV * k;
        if (lane == 0 && c < L) gt[(size_t)c * n + s] = v;
    }
    if (tid == 0) chi2[s] = chi;
}

// g[(i,q)] = sum_used g_q(c_k) g_k[i], g[N-1] = sum_used g_k[nb]: the
// right-hand side of the correction, assembled like b.
__global__ __launch_bounds__(64) void k_assemble_vec(int n, int nb, int ns, int N,
                                                    const double* __restrict__ gt,
                                                    const double* __restrict__ G,
                                                    const uint8_t* __restrict__ used,
                                                    double* __restrict__ gv, const SolveState* st) {
    // one wave per unknown t, its lanes over the stamps, fixed-order wave sum
    if (st->done) return;
    const int t = blockIdx.x, lane = threadIdx.x;
    const int i = (t == N - 1) ? nb : t / ns;
    const int q = (t == N - 1) ? -1 : t - (t / ns) * ns;
    double acc = 0.0;
    for (int k = lane; k < n; k += 64) {
        const double u = used[k] ? 1.0 : 0.0;
        const double w = q < 0 ? u : u * G[(size_t)k * ns + q];
        acc += w * gt[(size_t)i * n + k];
    }
    for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o);
    if (lane == 0) gv[t] = acc;
}

// chi2_s = e_s - 2 alpha^T b_s + alpha^T M_s alpha for every fitted stamp
// (one wave per stamp; alpha = local coefficients at the stamp centre).
__device__ void chi2_body(int nb, int ns, int N, const double* __restrict__ Ms,
                          const double* __restrict__ bs, const double* __restrict__ es,
                          const double* __restrict__ G, const double* __restrict__ a,
                          const uint8_t* __restrict__ fitted, double* __restrict__ chi2,
                          const SolveState* st, const int s) {
    if (st->done) return;
    const int lane = threadIdx.x;
    if (!fitted[s]) return;
    __shared__ double alpha[128];
    const int L = nb + 1;     // up to 128 (the two-kernel form); rows lane and lane + 64
    for (int r = lane; r < L; r += 64) {
        double al;
        if (r < nb) {
            al = 0.0;
            for (int q = 0; q < ns; q++) al += a[r * ns + q] * G[(size_t)s * ns + q];
        } else {
            al = a[N - 1];
        }
        alpha[r] = al;
    }
    wave_sync();
    double part = 0.0;
    for (int r = lane; r < L; r += 64) {
        const double* Mc = Ms + (size_t)s * L * L + r;
        double u0 = 0.0, u1 = 0.0, u2 = 0.0, u3 = 0.0;
        int i = 0;
        for (; i + 3 < L; i += 4) {
            u0 += alpha[i] * Mc[(size_t)i * L];
            u1 += alpha[i + 1] * Mc[(size_t)(i + 1) * L];
            u2 += alpha[i + 2] * Mc[(size_t)(i + 2) * L];
            u3 += alpha[i + 3] * Mc[(size_t)(i + 3) * L];
        }
        for (; i < L; i++) u0 += alpha[i] * Mc[(size_t)i * L];
        const double al = alpha[r];
        part += al * ((u0 + u1) + (u2 + u3)) - 2.0 * al * bs[(size_t)s * L + r];
    }
    for (int o = 32; o > 0; o >>= 1) part += __shfl_down(part, o);
    if (lane == 0) chi2[s] = es[s] + part;
}

__global__ __launch_bounds__(64) void k_chi2(int nb, int ns, int N, const double* __restrict__ Ms,
                                             const double* __restrict__ bs,
                                             const double* __restrict__ es,
                                             const double* __restrict__ G,
                                             const double* __restrict__ a,
                                             const uint8_t* __restrict__ fitted,
                                             double* __restrict__ chi2, const SolveState* st) {
    chi2_body(nb, ns, N, Ms, bs, es, G, a, fitted, chi2, st, blockIdx.x);
}

// Batched: one wave per stamp of every pair (stamp_pair maps the flat index).
__global__ __launch_bounds__(64) void k_chi2_b(const PairDesc* __restrict__ pairs,
                                               const int* __restrict__ stamp_pair, int nb) {
    const PairDesc& p = pairs[stamp_pair[blockIdx.x]];
    chi2_body(nb, p.ns, p.N, p.Ms, p.bs, p.es, p.G, p.coeffs, p.fitted, p.chi2, p.st,
              blockIdx.x - p.stamp_off);
}

// Sigma-clip over the used stamps after a solution (one workgroup, any size).
__device__ void clip_body(int n, int max_iter, int min_stamps, double clip_sigma,
                          const int32_t* __restrict__ npix, uint8_t* __restrict__ used,
                          int32_t* __restrict__ flags, const double* __restrict__ chi2,
                          SolveState* st) {
    if (st->done) return;
    __shared__ double red[16];
    __shared__ double s_thr;
    const int tid = threadIdx.x;
    __syncthreads();
    if (tid == 0) st->n_iter += 1;
    __syncthreads();
    if (st->n_iter - st->n_iter_base >= max_iter) {
        if (tid == 0) st->done = 1;
        return;
    }
    // mean and population std of q_s = chi2_s / npix_s over used stamps
    double sq = 0.0, cnt = 0.0;
    for (int s = tid; s < n; s += blockDim.x)
        if (used[s]) {
            sq += chi2[s] / npix[s];
            cnt += 1.0;
        }
    const double tot = block_sum(sq, red);
    const double nu = block_sum(cnt, red);
    const double mean = tot / nu;
    double dv = 0.0;
    for (int s = tid; s < n; s += blockDim.x)
        if (used[s]) {
            const double d = chi2[s] / npix[s] - mean;
            dv += d * d;
        }
    const double var = block_sum(dv, red) / nu;
    if (tid == 0) s_thr = mean + clip_sigma * sqrt(var);
    __syncthreads();
    const double thr = s_thr;
    double nnew = 0.0;
    for (int s = tid; s < n; s += blockDim.x)
        if (used[s] && chi2[s] / npix[s] > thr) nnew += 1.0;
    const double tnew = block_sum(nnew, red);
    if (tnew == 0.0 || nu - tnew < (double)min_stamps) {
        if (tid == 0) st->done = 1;
        return;
    }
    for (int s = tid; s < n; s += blockDim.x)
        if (used[s] && chi2[s] / npix[s] > thr) {
            used[s] = 0;
            flags[s] |= PSFM_STAMP_REJECTED;
        }
    if (tid == 0) {
        st->n_rej += (int)tnew;
        st->n_used -= (int)tnew;
    }
}

__global__ __launch_bounds__(1024) void k_clip(int n, int max_iter, int min_stamps,
                                               double clip_sigma,
                                               const int32_t* __restrict__ npix,
                                               uint8_t* __restrict__ used,
                                               int32_t* __restrict__ flags,
                                               const double* __restrict__ chi2, SolveState* st) {
    clip_body(n, max_iter, min_stamps, clip_sigma, npix, used, flags, chi2, st);
}

__global__ __launch_bounds__(1024) void k_clip_b(const PairDesc* __restrict__ pairs, int max_iter,
                                                 int min_stamps, double clip_sigma) {
    const PairDesc& p = pairs[blockIdx.x];
    clip_body(p.n, max_iter, min_stamps, clip_sigma, p.npix, p.used, p.flags, p.chi2, p.st);
}

// chi2 of every stamp (one wave each), then the clip, in one launch: the
// workgroup that finishes last (a device-scope counter in the state,
// acquire-release) runs clip_body and clears the counter for the next
// round.  No workgroup waits on another.
__global__ __launch_bounds__(64) void k_chi2_clip(int n, int nb, int ns, int N,
                                                  const double* __restrict__ Ms,
                                                  const double* __restrict__ bs,
                                                  const double* __restrict__ es,
                                                  const double* __restrict__ G,
                                                  const double* __restrict__ a,
                                                  const uint8_t* __restrict__ fitted,
                                                  double* __restrict__ chi2, int max_iter,
                                                  int min_stamps, double clip_sigma,
                                                  const int32_t* __restrict__ npix,
                                                  uint8_t* __restrict__ used,
                                                  int32_t* __restrict__ flags, SolveState* st) {
    if (st->done) return;                 // uniform: no workgroup of this launch changes it first
    chi2_body(nb, ns, N, Ms, bs, es, G, a, fitted, chi2, st, blockIdx.x);
    __shared__ int s_last;
    if (threadIdx.x == 0) {
        const int prev = __hip_atomic_fetch_add(&st->chi2_done, 1, __ATOMIC_ACQ_REL,
                                                __HIP_MEMORY_SCOPE_AGENT);
        s_last = prev == n - 1;
    }
    __syncthreads();
    if (!s_last) return;
    if (threadIdx.x == 0)
        __hip_atomic_store(&st->chi2_done, 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    clip_body(n, max_iter, min_stamps, clip_sigma, npix, used, flags, chi2, st);
}

// Penalty of the two-kernel form (Eq. 9): unknowns of the spatially varying
// columns i = 1 .. nt - 1 (b-terms i < nb, c-terms of basis i - nb + 1 above),
// every spatial term, get Phi Q_i on the diagonal, with
// Phi = phi (sum of their diagonal) / (sum of their Q_i), summed in a fixed
// order over the workgroup.
__global__ __launch_bounds__(1024) void k_penalty(int N, int ns, int nt, int nb,
                                                  const double* __restrict__ Q, double phi,
                                                  double* __restrict__ M, const SolveState* st) {
    __shared__ double red[16];
    if (st->done) return;
    const int np = (nt - 1) * ns;
    double dsum = 0.0, qsum = 0.0;
    for (int e = threadIdx.x; e < np; e += blockDim.x) {
        const int j = ns + e, i = j / ns;
        dsum += M[(size_t)j * N + j];
        qsum += Q[i < nb ? i : i - nb + 1];
    }
    dsum = block_sum(dsum, red);
    qsum = block_sum(qsum, red);
    const double Phi = qsum > 0.0 ? phi * dsum / qsum : 0.0;
    for (int e = threadIdx.x; e < np; e += blockDim.x) {
        const int j = ns + e, i = j / ns;
        M[(size_t)j * N + j] += Phi * Q[i < nb ? i : i - nb + 1];
    }
}

__device__ void solve_finish_body(int n, int ns, int N, int n_par, int S, int W, int H,
                                  const int32_t* __restrict__ npix,
                                  const uint8_t* __restrict__ used,
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
            stats->dof = np - n_par;
            stats->chi2_dof = c2 / (np - n_par);
            stats->n_used = (int)nu;
            // term 0's spatial polynomial at the image centre
            stats->kernel_sum_centre = psfm_spatial_dot(S, 0.5 * (W - 1), 0.5 * (H - 1), W, H, coeffs);
        } else {
            stats->chi2 = 0.0;
            stats->dof = 0.0;
            stats->chi2_dof = 0.0;
            stats->n_used = 0;
            stats->kernel_sum_centre = 0.0;
        }
        stats->chi2_dof_prior = 0.0;
        stats->n_prior = 0;
        stats->n_restored = 0;
        stats->n_trusted = 0;
        stats->prior_fallback = 0;
        stats->n_replaced = st->n_rep;
    }
}

__global__ void k_prior_finish(const double* __restrict__ pdof, const int* __restrict__ counts,
                               psfm_fit_stats* stats) {
    if (threadIdx.x == 0 && stats) {
        stats->chi2_dof_prior = *pdof;
        stats->n_prior = counts[0];
        stats->n_restored = counts[1];
        stats->n_trusted = counts[2];
        stats->prior_fallback = counts[3];
    }
}

__global__ void k_solve_finish(int n, int ns, int N, int n_par, int S, int W, int H,
                               const int32_t* __restrict__ npix, const uint8_t* __restrict__ used,
                               const double* __restrict__ chi2, double* __restrict__ coeffs,
                               const SolveState* st, psfm_fit_stats* stats) {
    solve_finish_body(n, ns, N, n_par, S, W, H, npix, used, chi2, coeffs, st, stats);
}

__global__ void k_solve_finish_b(const PairDesc* __restrict__ pairs) {
    const PairDesc& p = pairs[blockIdx.x];
    solve_finish_body(p.n, p.ns, p.N, p.N, p.S, p.W, p.H, p.npix, p.used, p.chi2, p.coeffs, p.st,
                      p.stats);
}

// Each stamp's own least-squares problem M_s a = b_s (L x L, FP64): one
// wave per stamp, equilibrated Cholesky in LDS; the local coefficients and
// chi2_s = e_s - 2 a^T b_s + a^T M_s a at that solution.  Flagged stamps and
// non-positive pivots give zeros and chi2 = -1.
constexpr int PS_LD = 65;

__global__ __launch_bounds__(64) void k_solve_stamps(int L, const double* __restrict__ Ms,
                                                     const double* __restrict__ bs,
                                                     const double* __restrict__ es,
                                                     const int32_t* __restrict__ flags,
                                                     double* __restrict__ local,
                                                     double* __restrict__ chi2) {
    __shared__ double A[64 * PS_LD];
    __shared__ double dq[64], x[64];
    __shared__ int s_bad;
    const int s = blockIdx.x, lane = threadIdx.x;
    const double* M = Ms + (size_t)s * L * L;
    const double* b = bs + (size_t)s * L;
    if (lane == 0) s_bad = flags[s] != 0;
    wave_sync();
    if (lane < L) {
        const double d = M[lane * L + lane];
        if (!(d > 0.0)) s_bad = 1;
        dq[lane] = d > 0.0 ? 1.0 / sqrt(d) : 0.0;
    }
    wave_sync();
    if (!s_bad) {
        if (lane < L) {
            for (int j = 0; j <= lane; j++) A[lane * PS_LD + j] = M[lane * L + j] * dq[lane] * dq[j];
            x[lane] = dq[lane] * b[lane];
        }
        wave_sync();
        for (int k = 0; k < L; k++) {
            const double piv = A[k * PS_LD + k];
            if (!(piv > 0.0)) {
                if (lane == 0) s_bad = 1;
                break;
            }
            const double lkk = sqrt(piv);
            wave_sync();
            if (lane == k) A[k * PS_LD + k] = lkk;
            if (lane > k && lane < L) A[lane * PS_LD + k] /= lkk;
            wave_sync();
            if (lane > k && lane < L) {
                const double lik = A[lane * PS_LD + k];
                for (int j = k + 1; j <= lane; j++) A[lane * PS_LD + j] -= lik * A[j * PS_LD + k];
            }
            wave_sync();
        }
        wave_sync();
    }
    if (s_bad) {
        if (lane < L) local[(size_t)s * L + lane] = 0.0;
        if (lane == 0) chi2[s] = -1.0;
        return;
    }
    for (int k = 0; k < L; k++) {                    // L z = x
        if (lane == k) x[k] /= A[k * PS_LD + k];
        wave_sync();
        if (lane > k && lane < L) x[lane] -= A[lane * PS_LD + k] * x[k];
        wave_sync();
    }
    for (int k = L - 1; k >= 0; k--) {               // L^T w = z
        if (lane == k) x[k] /= A[k * PS_LD + k];
        wave_sync();
        if (lane < k) x[lane] -= A[k * PS_LD + lane] * x[k];
        wave_sync();
    }
    double part = 0.0;
    if (lane < L) {
        const double a = dq[lane] * x[lane];
        local[(size_t)s * L + lane] = a;
        x[lane] = a;
    }
    wave_sync();
    if (lane < L) {
        double u = 0.0;
        for (int j = 0; j < L; j++) u += M[lane * L + j] * x[j];
        part = x[lane] * (u - 2.0 * b[lane]);
    }
    for (int o = 32; o > 0; o >>= 1) part += __shfl_xor(part, o);
    if (lane == 0) chi2[s] = es[s] + part;
}

// Prior: each stamp's predicted local kernel coefficients (pred, n x L; the
// background slot is replaced by the best constant for that kernel,
// bg = (b[nb] - sum_i M[nb][i] alpha_i) / M[nb][nb]) and the chi2 of the
// stamp under that prediction, chi2 = e - 2 alpha^T b + alpha^T M alpha.
__global__ __launch_bounds__(64) void k_prior_chi2(int nb, const double* __restrict__ Ms,
                                                   const double* __restrict__ bs,
                                                   const double* __restrict__ es,
                                                   const int32_t* __restrict__ flags,
                                                   const double* __restrict__ pred,
                                                   double* __restrict__ alpha_out,
                                                   double* __restrict__ chi2p) {
    __shared__ double al[64];
    __shared__ double s_bg;
    const int s = blockIdx.x, lane = threadIdx.x, L = nb + 1;
    const double* M = Ms + (size_t)s * L * L;
    const double* b = bs + (size_t)s * L;
    if (flags[s]) {
        if (lane < L) alpha_out[(size_t)s * L + lane] = 0.0;
        if (lane == 0) chi2p[s] = 0.0;
        return;
    }
    if (lane < nb) al[lane] = pred[(size_t)s * L + lane];
    wave_sync();
    double t = 0.0;
    if (lane < nb) t = M[nb * L + lane] * al[lane];
    for (int o = 32; o > 0; o >>= 1) t += __shfl_xor(t, o);
    if (lane == 0) s_bg = M[nb * L + nb] > 0.0 ? (b[nb] - t) / M[nb * L + nb] : 0.0;
    wave_sync();
    if (lane == 0) al[nb] = s_bg;
    wave_sync();
    double part = 0.0;
    if (lane < L) {
        double u = 0.0;
        for (int j = 0; j < L; j++) u += M[lane * L + j] * al[j];
        part = al[lane] * (u - 2.0 * b[lane]);
        alpha_out[(size_t)s * L + lane] = al[lane];
    }
    for (int o = 32; o > 0; o >>= 1) part += __shfl_xor(part, o);
    if (lane == 0) chi2p[s] = es[s] + part;
}

// The 1.05x rule, per stamp: a stamp's predicted kernel is kept only if its
// residual chi2 (background re-fitted) is within PRIOR_TRUST of the residual
// of the stamp's own least-squares kernel (the solved value, from
// k_solve_stamps); otherwise the least-squares kernel replaces the
// prediction.  has[s] = 1 for every stamp with a kernel estimate (usable and
// a positive definite own system), counts[2] = predictions kept.
constexpr double PRIOR_TRUST = 1.05;

__global__ __launch_bounds__(1024) void k_prior_trust(int n, int L, const int32_t* __restrict__ flags,
                                                      double* __restrict__ alpha,
                                                      double* __restrict__ chi2_pred,
                                                      const double* __restrict__ local_ls,
                                                      const double* __restrict__ chi2_ls,
                                                      uint8_t* __restrict__ has,
                                                      int* __restrict__ counts) {
    __shared__ double red[16];
    double kept = 0.0;
    for (int s = threadIdx.x; s < n; s += blockDim.x) {
        const bool ok = flags[s] == 0 && chi2_ls[s] >= 0.0;
        const bool keep = ok && chi2_pred[s] <= PRIOR_TRUST * chi2_ls[s];
        if (ok && !keep) {
            for (int i = 0; i < L; i++) alpha[(size_t)s * L + i] = local_ls[(size_t)s * L + i];
            chi2_pred[s] = chi2_ls[s];
        }
        has[s] = ok;
        kept += keep ? 1.0 : 0.0;
    }
    kept = psfm_block_sum(kept, red);
    if (threadIdx.x == 0) counts[2] = (int)kept;
}

// Warm start a0 of the prior: per kernel term, the spatial polynomial
// fitted (least squares, FP64) to the completed per-stamp predictions of
// the stamps in use; the background as their mean.  One workgroup.
constexpr int PRIOR_T = 1024;

__global__ __launch_bounds__(PRIOR_T) void k_prior_warm(
    int n, int nb, int ns, int N, const double* __restrict__ G,
    const double* __restrict__ alpha, const uint8_t* __restrict__ used,
    const uint8_t* __restrict__ trust, double* __restrict__ a0, const SolveState* st, int force) {
    __shared__ double Gm[28 * 28];
    __shared__ double rhs[64 * 28];
    __shared__ int s_ok;
    const int tid = threadIdx.x, L = nb + 1;
    if (st->done || (st->prior_done && !force)) return;
    for (int t = tid; t < ns * ns + L * ns; t += PRIOR_T) {
        const bool isG = t < ns * ns;
        const int e = isG ? t : t - ns * ns;
        const int r0 = e / ns, q = e % ns;
        // sum over the used stamps: branch-free, four accumulators (loads of
        // successive stamps in flight together)
        double a4[4] = {0.0, 0.0, 0.0, 0.0};
        int s = 0;
        for (; s + 3 < n; s += 4) {
#pragma unroll
            for (int u = 0; u < 4; u++) {
                const int ss = s + u;
                const double* g = G + (size_t)ss * ns;    // spatial terms at the stamp centre
                const double v = isG ? g[r0] : alpha[(size_t)ss * L + r0];
                a4[u] += (used[ss] && trust[ss]) ? v * g[q] : 0.0;
            }
        }
        for (; s < n; s++) {
            const double* g = G + (size_t)s * ns;
            const double v = isG ? g[r0] : alpha[(size_t)s * L + r0];
            a4[0] += (used[s] && trust[s]) ? v * g[q] : 0.0;
        }
        const double acc = (a4[0] + a4[1]) + (a4[2] + a4[3]);
        if (isG) Gm[e] = acc;
        else rhs[e] = acc;
    }
    __syncthreads();
    if (tid == 0) {                           // G = C C^T in place (ns <= 28)
        int ok = 1;
        for (int j = 0; j < ns && ok; j++) {
            double d = Gm[j * ns + j];
            for (int k = 0; k < j; k++) d -= Gm[j * ns + k] * Gm[j * ns + k];
            if (!(d > 0.0)) {
                ok = 0;
                break;
            }
            const double ljj = sqrt(d);
            Gm[j * ns + j] = ljj;
            for (int i = j + 1; i < ns; i++) {
                double v = Gm[i * ns + j];
                for (int k = 0; k < j; k++) v -= Gm[i * ns + k] * Gm[j * ns + k];
                Gm[i * ns + j] = v / ljj;
            }
        }
        s_ok = ok;
    }
    __syncthreads();
    if (tid < nb) {
        double z[28];
        for (int q = 0; q < ns; q++) {
            double v = rhs[tid * ns + q];
            for (int k = 0; k < q; k++) v -= Gm[q * ns + k] * z[k];
            z[q] = s_ok ? v / Gm[q * ns + q] : 0.0;
        }
        for (int q = ns - 1; q >= 0; q--) {
            double v = z[q];
            for (int k = q + 1; k < ns; k++) v -= Gm[k * ns + q] * z[k];
            z[q] = s_ok ? v / Gm[q * ns + q] : 0.0;
        }
        for (int q = 0; q < ns; q++) a0[tid * ns + q] = z[q];
    }
    // background: mean of the used stamps' predictions (block sums)
    __shared__ double red[16];
    double sbg = 0.0, c = 0.0;
    for (int s = tid; s < n; s += PRIOR_T)
        if (used[s] && trust[s]) {
            sbg += alpha[(size_t)s * L + nb];
            c += 1.0;
        }
    sbg = block_sum(sbg, red);
    c = block_sum(c, red);
    if (tid == 0) a0[N - 1] = c > 0.0 ? sbg / c : 0.0;
}

// Rejection prior: a variable source shows up as a stamp whose kernel
// estimate (the prediction, or its own least-squares kernel where the 1.05x
// rule dropped the prediction) has a kernel sum -- its own flux ratio --
// departing from the warm start's kernel sum at that stamp (the consensus),
// and which the warm start does not fit.  The departures d_s = k_s / k_a0 - 1
// of the stamps in use are summarised robustly (median m and 1.4826 x median
// |d - m|, by ranking in LDS); a stamp gets PSFM_STAMP_PRIOR and leaves the
// equations when
// |d_s - m| > max(5 robust sigma, PRIOR_FLOOR) and its chi2_s / npix_s at the
// warm start exceeds the method's clip threshold there (mean + clip_sigma
// std over the stamps in use): the departure must be the stamp's own, not
// the noise of a faint stamp's prediction.  It stays fitted, so its chi2 is
// evaluated at every solution for the final judgement.  A round that excludes
// nothing, or would leave fewer than min_stamps, ends the prior.
constexpr double PRIOR_FLOOR = 0.2;    // flux-ratio departures below 20% never exclude
constexpr int PRIOR_RANK_MAX = 2048;   // robust statistics up to this many stamps

__device__ double block_kth(const double* v, int m, int k, int* s_idx) {
    // value of rank k (0-based) among v[0..m): each thread ranks its entries
    if (threadIdx.x == 0) *s_idx = 0;
    __syncthreads();
    for (int i = threadIdx.x; i < m; i += blockDim.x) {
        const double x = v[i];
        int lt = 0, eq = 0;
        for (int j = 0; j < m; j++) {
            lt += v[j] < x;
            eq += (v[j] == x) && (j < i);
        }
        if (lt + eq == k) *s_idx = i;
    }
    __syncthreads();
    return v[*s_idx];
}

__global__ __launch_bounds__(1024) void k_prior_clip(int n, int ns, int L, int min_stamps,
                                                     double clip_sigma,
                                                     const double* __restrict__ G,
                                                     const double* __restrict__ alpha,
                                                     const double* __restrict__ a0,
                                                     const uint8_t* __restrict__ trust,
                                                     const double* __restrict__ chi2w,
                                                     const int32_t* __restrict__ npix,
                                                     uint8_t* __restrict__ used,
                                                     int32_t* __restrict__ flags, SolveState* st) {
    __shared__ double vals[PRIOR_RANK_MAX];
    __shared__ double red[16];
    __shared__ int s_cnt, s_idx, s_n;
    __shared__ double s_med, s_thr, s_qthr;
    const int tid = threadIdx.x;
    if (st->done || st->prior_done) return;
    // the method's clip threshold at the warm start, over the stamps in use
    {
        double sq = 0.0, cnt = 0.0;
        for (int s = tid; s < n; s += 1024)
            if (used[s]) {
                sq += chi2w[s] / npix[s];
                cnt += 1.0;
            }
        const double tot = psfm_block_sum(sq, red);
        const double nu = psfm_block_sum(cnt, red);
        const double mean = nu > 0.0 ? tot / nu : 0.0;
        double dv = 0.0;
        for (int s = tid; s < n; s += 1024)
            if (used[s]) {
                const double d = chi2w[s] / npix[s] - mean;
                dv += d * d;
            }
        const double var = nu > 0.0 ? psfm_block_sum(dv, red) / nu : 0.0;
        if (tid == 0) s_qthr = mean + clip_sigma * sqrt(var);
    }
    auto dev = [&](int s) {
        double kc = 0.0;
        for (int q = 0; q < ns; q++) kc += a0[q] * G[(size_t)s * ns + q];
        return kc > 0.0 ? alpha[(size_t)s * L] / kc - 1.0 : 0.0;
    };
    if (tid == 0) {
        s_cnt = 0;
        s_n = 0;
    }
    __syncthreads();
    for (int s = tid; s < n; s += 1024)
        if (used[s] && trust[s]) {
            const int k = atomicAdd(&s_cnt, 1);
            if (k < PRIOR_RANK_MAX) vals[k] = dev(s);
        }
    __syncthreads();
    const int m = min(s_cnt, PRIOR_RANK_MAX);
    if (m < 3) {
        if (tid == 0) st->prior_done = 1;
        return;
    }
    const double med = block_kth(vals, m, m / 2, &s_idx);
    if (tid == 0) s_med = med;
    __syncthreads();
    for (int i = tid; i < m; i += 1024) vals[i] = fabs(vals[i] - s_med);
    __syncthreads();
    const double mad = block_kth(vals, m, m / 2, &s_idx);
    if (tid == 0) s_thr = fmax(5.0 * 1.4826 * mad, PRIOR_FLOOR);
    __syncthreads();
    const double thr = s_thr, mm = s_med, qthr = s_qthr;
    auto out = [&](int s) {
        return used[s] && trust[s] && fabs(dev(s) - mm) > thr && chi2w[s] / npix[s] > qthr;
    };
    int nnew = 0;
    for (int s = tid; s < n; s += 1024)
        if (out(s)) nnew++;
    atomicAdd(&s_n, nnew);
    __syncthreads();
    const int tn = s_n;
    if (tn == 0 || st->n_used - tn < min_stamps) {
        if (tid == 0) st->prior_done = 1;
        return;
    }
    for (int s = tid; s < n; s += 1024)
        if (out(s)) {
            used[s] = 0;
            flags[s] |= PSFM_STAMP_PRIOR;
        }
    if (tid == 0) st->n_used -= tn;
}

// chi2/dof of the kept stamps at the warm start (chi2 from the stamp sums).
__global__ __launch_bounds__(1024) void k_prior_dof(int n, int N, const int32_t* __restrict__ npix,
                                                    const uint8_t* __restrict__ used,
                                                    const double* __restrict__ chi2w,
                                                    double* __restrict__ out, const SolveState* st) {
    __shared__ double red[16];
    if (st->info != 0) {
        if (threadIdx.x == 0) *out = 0.0;
        return;
    }
    double c2 = 0.0, np = 0.0;
    for (int s = threadIdx.x; s < n; s += 1024)
        if (used[s]) {
            c2 += chi2w[s];
            np += npix[s];
        }
    c2 = psfm_block_sum(c2, red);
    np = psfm_block_sum(np, red);
    if (threadIdx.x == 0) *out = np > N ? c2 / (np - N) : 0.0;
}

// The least-squares solution judges the prior: at the prior path's final
// solution the method's own clip threshold (mean + clip_sigma std of
// chi2_s / npix_s over the stamps in use) is formed; if any stamp the prior
// excluded lies within it (the method would have kept that stamp), or the
// prior path failed, the exclusions are void and the full method runs again
// from the complete stamp set with a fresh solution budget (the rounds that
// follow), which is psfm_solve's own path.  Otherwise the prior path's answer
// stands.  counts[0]: stamps left excluded, counts[1]: excluded stamps found
// within the threshold, counts[3]: 1 if the full method was rerun.
__global__ __launch_bounds__(1024) void k_prior_fallback(int n, double clip_sigma,
                                                         const int32_t* __restrict__ npix,
                                                         const uint8_t* __restrict__ fitted,
                                                         uint8_t* __restrict__ used,
                                                         int32_t* __restrict__ flags,
                                                         const double* __restrict__ chi2,
                                                         SolveState* st, int* __restrict__ counts) {
    __shared__ double red[16];
    __shared__ double s_thr;
    const int tid = threadIdx.x;
    const bool failed = st->info != 0;
    double sq = 0.0, cnt = 0.0;
    for (int s = tid; s < n; s += 1024)
        if (used[s]) {
            sq += chi2[s] / npix[s];
            cnt += 1.0;
        }
    const double tot = psfm_block_sum(sq, red);
    const double nu = psfm_block_sum(cnt, red);
    const double mean = nu > 0.0 ? tot / nu : 0.0;
    double dv = 0.0;
    for (int s = tid; s < n; s += 1024)
        if (used[s]) {
            const double d = chi2[s] / npix[s] - mean;
            dv += d * d;
        }
    const double var = nu > 0.0 ? psfm_block_sum(dv, red) / nu : 0.0;
    if (tid == 0) s_thr = mean + clip_sigma * sqrt(var);
    __syncthreads();
    const double thr = s_thr;
    double back = 0.0, still = 0.0;
    for (int s = tid; s < n; s += 1024)
        if (flags[s] & PSFM_STAMP_PRIOR) {
            if (failed || chi2[s] / npix[s] <= thr) back += 1.0;
            else still += 1.0;
        }
    const double nback = psfm_block_sum(back, red);
    const double nstill = psfm_block_sum(still, red);
    const bool rerun = failed || nback > 0.0;
    double nfit = 0.0;
    if (rerun)
        for (int s = tid; s < n; s += 1024)
            if (fitted[s]) {
                flags[s] &= ~(PSFM_STAMP_PRIOR | PSFM_STAMP_REJECTED);
                used[s] = 1;
                nfit += 1.0;
            }
    nfit = psfm_block_sum(nfit, red);
    if (tid == 0) {
        counts[0] = rerun ? 0 : (int)nstill;
        counts[1] = (int)nback;
        counts[3] = rerun ? 1 : 0;
        if (rerun) {            // psfm_solve's loop from the complete set, fresh budget
            st->n_used = (int)nfit;
            st->n_rej = 0;
            st->info = 0;
            st->done = 0;
            st->n_iter_base = st->n_iter;
        }
    }
}

// ---- the paper's normalisation mode (Sections 3.2, 3.3)

// b0 and d0, spatially constant, from the stamps in use: the unweighted
// least-squares fit of the stamp totals T2_s = b0 T1_s + d0 npix_s (only the
// normalisation and the background add flux; the zero-sum terms move it
// within a stamp).  hv[0] = b0, hv[1] = d0; a singular 2 x 2 system fails the
// solve with info PSFM_ERR_NORM_SINGULAR.  One workgroup.
__global__ __launch_bounds__(1024) void k_norm_solve(int n, const double* __restrict__ norm,
                                                     const uint8_t* __restrict__ used,
                                                     double* __restrict__ hv, SolveState* st) {
    if (st->done) return;
    __shared__ double red[16];
    double saa = 0.0, san = 0.0, snn = 0.0, sad = 0.0, snd = 0.0;
    for (int s = threadIdx.x; s < n; s += blockDim.x)
        if (used[s]) {
            const double np = norm[5 * (size_t)s], t1 = norm[5 * (size_t)s + 1],
                         t2 = norm[5 * (size_t)s + 2];
            saa += t1 * t1;
            san += t1 * np;
            snn += np * np;
            sad += t1 * t2;
            snd += np * t2;
        }
    saa = block_sum(saa, red);
    san = block_sum(san, red);
    snn = block_sum(snn, red);
    sad = block_sum(sad, red);
    snd = block_sum(snd, red);
    if (threadIdx.x == 0) {
        const double det = saa * snn - san * san;
        if (!(det > 1e-12 * saa * snn)) {
            hv[0] = hv[1] = 0.0;
            st->info = PSFM_ERR_NORM_SINGULAR;
            st->done = 1;
        } else {
            hv[0] = (sad * snn - san * snd) / det;
            hv[1] = (saa * snd - san * sad) / det;
        }
    }
}

// Holds the normalisation (term 0: b0 at spatial term 0, zero at the others)
// and the background (d0) in the assembled equations: their columns move to
// the right-hand side with their values, their rows and columns become those
// of the identity, so the factorisation returns them unchanged and solves
// M_ff a_f = b_f - M_fc a_c for the free unknowns.  One workgroup.
__global__ __launch_bounds__(1024) void k_hold(int N, int ns, double* __restrict__ M,
                                               double* __restrict__ b,
                                               const double* __restrict__ hv,
                                               const SolveState* st) {
    if (st->done) return;
    const double b0 = hv[0], d0 = hv[1];
    auto held = [&](int i) { return i < ns || i == N - 1; };
    for (int i = threadIdx.x; i < N; i += blockDim.x)
        if (!held(i)) b[i] -= M[(size_t)i * N] * b0 + M[(size_t)i * N + N - 1] * d0;
    __syncthreads();
    for (int e = threadIdx.x; e < N * N; e += blockDim.x) {
        const int i = e / N, j = e - i * N;
        if (held(i) || held(j)) M[e] = i == j ? 1.0 : 0.0;
    }
    for (int i = threadIdx.x; i < N; i += blockDim.x)
        if (held(i)) b[i] = i == 0 ? b0 : (i == N - 1 ? d0 : 0.0);
}

// The method's sigma-clip (as clip_body) with replacement (Section 3.3): each
// stamp rejected in this round is replaced by a reserve of its group (a stamp
// whose flags are exactly PSFM_STAMP_RESERVE with the same group id >= 0),
// the group's reserves taken in index order.  newrej / act: scratch flags.
__global__ __launch_bounds__(1024) void k_clip_replace(int n, int max_iter, int min_stamps,
                                                       double clip_sigma,
                                                       const int32_t* __restrict__ npix,
                                                       const int32_t* __restrict__ group,
                                                       uint8_t* __restrict__ used,
                                                       uint8_t* __restrict__ fitted,
                                                       int32_t* __restrict__ flags,
                                                       const double* __restrict__ chi2,
                                                       uint8_t* __restrict__ newrej,
                                                       uint8_t* __restrict__ act, SolveState* st) {
    if (st->done) return;
    __shared__ double red[16];
    __shared__ double s_thr;
    const int tid = threadIdx.x;
    for (int s = tid; s < n; s += blockDim.x) newrej[s] = 0;
    __syncthreads();
    if (tid == 0) st->n_iter += 1;
    __syncthreads();
    if (st->n_iter - st->n_iter_base >= max_iter) {
        if (tid == 0) st->done = 1;
        return;
    }
    double sq = 0.0, cnt = 0.0;
    for (int s = tid; s < n; s += blockDim.x)
        if (used[s]) {
            sq += chi2[s] / npix[s];
            cnt += 1.0;
        }
    const double tot = block_sum(sq, red);
    const double nu = block_sum(cnt, red);
    const double mean = tot / nu;
    double dv = 0.0;
    for (int s = tid; s < n; s += blockDim.x)
        if (used[s]) {
            const double d = chi2[s] / npix[s] - mean;
            dv += d * d;
        }
    const double var = block_sum(dv, red) / nu;
    if (tid == 0) s_thr = mean + clip_sigma * sqrt(var);
    __syncthreads();
    const double thr = s_thr;
    double nnew = 0.0;
    for (int s = tid; s < n; s += blockDim.x)
        if (used[s] && chi2[s] / npix[s] > thr) nnew += 1.0;
    const double tnew = block_sum(nnew, red);
    if (tnew == 0.0 || nu - tnew < (double)min_stamps) {
        if (tid == 0) st->done = 1;
        return;
    }
    for (int s = tid; s < n; s += blockDim.x)
        if (used[s] && chi2[s] / npix[s] > thr) {
            used[s] = 0;
            flags[s] |= PSFM_STAMP_REJECTED;
            newrej[s] = 1;
        }
    __syncthreads();
    double nact = 0.0;
    if (group) {
        // reserve q of group g comes in if fewer of g's reserves precede it
        // than g lost stamps in this round
        for (int q = tid; q < n; q += blockDim.x) {
            act[q] = 0;
            const int g = group[q];
            if (flags[q] != PSFM_STAMP_RESERVE || g < 0) continue;
            int lost = 0, before = 0;
            for (int s = 0; s < n; s++) {
                lost += newrej[s] && group[s] == g;
                before += s < q && flags[s] == PSFM_STAMP_RESERVE && group[s] == g;
            }
            act[q] = before < lost;
        }
        __syncthreads();
        for (int q = tid; q < n; q += blockDim.x)
            if (act[q]) {
                flags[q] = 0;
                used[q] = 1;
                fitted[q] = 1;
                nact += 1.0;
            }
    }
    nact = block_sum(nact, red);
    if (tid == 0) {
        st->n_rej += (int)tnew;
        st->n_used += (int)nact - (int)tnew;
        st->n_rep += (int)nact;
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
    c.take<double>(psfm::solve_il_doubles(ctx->N));
    c.take<double>(ctx->N);                          // 1 / sqrt(diag M)
    c.take<double>((size_t)n * ctx->L + 1);          // residual gradients, stamp-major
    c.take<double>(ctx->N);                          // assembled correction right-hand side
    c.take<double>((size_t)n * ctx->L + 1);          // prior: completed predictions
    c.take<double>(n + 1);                           // prior: predicted chi2
    c.take<double>(n + 1);                           // prior: chi2 at the warm start
    c.take<double>(ctx->N);                          // prior: warm start
    c.take<double>(1);
    c.take<int>(4);
    c.take<double>((size_t)n * ctx->L + 1);          // prior: each stamp's own least-squares kernel
    c.take<double>(n + 1);                           // prior: its chi2 (the solved value)
    c.take<uint8_t>(n + 1);                          // prior: stamps with a kernel estimate
    c.take<double>(2);                               // normalisation mode: b0, d0
    c.take<uint8_t>(n + 1);                          // normalisation mode: rejected this round
    c.take<uint8_t>(n + 1);                          // normalisation mode: reserves to bring in
    if (ctx->cfg.precision != PSFM_PREC_FP32)
        c.take<double>((size_t)ctx->N * ctx->N);     // transposed factor (refinement)
    if (ctx->cfg.ortho_basis) {
        c.take<double>((size_t)n * ctx->L * ctx->L + 1);   // stamp sums in the orthonormal basis
        c.take<double>((size_t)n * ctx->L + 1);
    }
    return c.off;
}

int solve_lds_grant(size_t lds) {
    static size_t granted = 0;      // dynamic LDS granted so far (both forms)
    if (lds > granted) {
        PSFM_HIP_CHECK(hipFuncSetAttribute((const void*)k_cholesky<false>,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
        PSFM_HIP_CHECK(hipFuncSetAttribute((const void*)k_cholesky<true>,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
        PSFM_HIP_CHECK(hipFuncSetAttribute((const void*)k_cholesky_b,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
        PSFM_HIP_CHECK(hipFuncSetAttribute((const void*)k_resolve,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
        granted = lds;
    }
    return PSFM_OK;
}

// panel buffer: N + 16 rows (16-row tiles overrun the panel), at least 48
// (the diagonal-block routines address all 32 rows of the block)
size_t solve_lds_bytes(int N) { return (size_t)(max(N, CH_NB) + 16) * CH_PS * sizeof(double); }
int solve_max_unknowns() { return CH_NMAX; }
size_t solve_il_doubles(int N) { return (size_t)IV_DOUBLES * ((N + CH_NB - 1) / CH_NB); }

// The whole solve loop for every pair of a batch: each launch covers all
// pairs (blockIdx.y or one workgroup per pair); pairs that converged or
// failed idle through the remaining rounds.
int batch_solve(const psfm_context* ctx, const PairDesc* pairs, const int* stamp_pair, int n_pairs,
                int n_stamps_total, int max_n, int max_N, const int* ns_pairs, const int* ns_off,
                const int* ns_cnt, hipStream_t st) {
    if (n_pairs == 0) return PSFM_OK;
    const psfm_config& cf = ctx->cfg;
    const int nb = ctx->nb;
    const size_t lds = solve_lds_bytes(max_N);
    int rc = solve_lds_grant(lds);
    if (rc) return rc;
    const int nt = std::max(std::max(max_n, max_N), 1);
    const int n_init = (nt + 255) / 256;
    hipLaunchKernelGGL(k_solve_prep_b, dim3(n_init, n_pairs), dim3(256), 0, st, pairs, cf.min_stamps);
    PSFM_HIP_CHECK(hipGetLastError());
    for (int it = 0; it < cf.max_iter; it++) {
#define PSFM_ASM_B(NSV)                                                                          \
        if (ns_cnt[NSV] > 0)                                                                     \
            hipLaunchKernelGGL(k_assemble_b<NSV>, dim3(asm_width<NSV>(nb), ns_cnt[NSV]),          \
                               dim3(64 * ASM_WAVES), 0, st, pairs, ns_pairs + ns_off[NSV], nb);
        PSFM_ASM_B(1) PSFM_ASM_B(3) PSFM_ASM_B(6) PSFM_ASM_B(10) PSFM_ASM_B(15) PSFM_ASM_B(21)
        PSFM_ASM_B(28)
#undef PSFM_ASM_B
        hipLaunchKernelGGL(k_cholesky_b, dim3(n_pairs), dim3(CH_THREADS), lds, st, pairs);
        if (n_stamps_total > 0)
            hipLaunchKernelGGL(k_chi2_b, dim3(n_stamps_total), dim3(64), 0, st, pairs, stamp_pair, nb);
        hipLaunchKernelGGL(k_clip_b, dim3(n_pairs), dim3(1024), 0, st, pairs, cf.max_iter,
                           cf.min_stamps, cf.clip_sigma);
        PSFM_HIP_CHECK(hipGetLastError());
    }
    hipLaunchKernelGGL(k_solve_finish_b, dim3(n_pairs), dim3(1024), 0, st, pairs);
    PSFM_HIP_CHECK(hipGetLastError());
    return PSFM_OK;
}

}  // namespace psfm

// Shared launch sequence of psfm_solve and psfm_solve_prior (prior: the
// per-stamp predicted local coefficients, or null).
// penq (nullable): penalty weights of the two-kernel form, whose view of the
// context (nb = 2 nb - 1 spatially varying columns) ctx then is; pen_nb is
// the basis size they index.
// ---- orthonormalised basis (ortho_basis)
// The taps of the basis terms, as columns of B, have the Gram B^T B = R^T R
// (R upper, from the context); the terms k' = k R^-1 are orthonormal.  With
// T = blockdiag(R^-1, 1) (background unchanged) a stamp's sums become
// M' = T^T M T and b' = T^T b.  One wave per stamp: lane j first takes column
// j of [M | b] through the forward substitution with R^T (X = R^-T [M | b]),
// then lane i takes row i of X through the substitution with R from the
// right (M' = X R^-1).  L <= 63, so the L + 1 columns fit one wave.
__global__ __launch_bounds__(64) void k_ortho_stamps(const double* __restrict__ Rm, int nb, int L,
                                                     const double* __restrict__ Ms,
                                                     const double* __restrict__ bs,
                                                     double* __restrict__ Mo,
                                                     double* __restrict__ bo) {
    __shared__ double X[64 * 65];                 // X[i * 65 + j]: row i, column j (b at j = L)
    const int s = blockIdx.x, t = threadIdx.x;
    const double* M = Ms + (size_t)s * L * L;
    if (t <= L) {
        const int j = t;
        auto src = [&](int i) { return j < L ? M[(size_t)i * L + j] : bs[(size_t)s * L + i]; };
        for (int i = 0; i < nb; i++) {
            double v = src(i);
            for (int k = 0; k < i; k++) v -= Rm[k * nb + i] * X[k * 65 + j];
            X[i * 65 + j] = v / Rm[i * nb + i];
        }
        for (int i = nb; i < L; i++) X[i * 65 + j] = src(i);
    }
    __syncthreads();
    if (t < L) {
        const int i = t;
        double* Y = X + i * 65;                   // row i, overwritten left to right
        for (int j = 0; j < nb; j++) {
            double v = Y[j];
            for (int k = 0; k < j; k++) v -= Y[k] * Rm[k * nb + j];
            Y[j] = v / Rm[j * nb + j];
        }
        double* out = Mo + (size_t)s * L * L + (size_t)i * L;
        for (int j = 0; j < L; j++) out[j] = Y[j];
        bo[(size_t)s * L + i] = Y[L];
    }
}

// Coefficients back from the orthonormalised basis after a solution:
// a_(i, p) = sum_j (R^-1)_ij c_(j, p) for each spatial term p (back
// substitution R a = c, in place from the last term up), the background
// unchanged.  Skipped when this round's factorization did not run or failed
// (the state is then done), so that the coefficients are mapped once per
// solution.  One thread per spatial term.
__global__ __launch_bounds__(64) void k_ortho_coeffs(const double* __restrict__ Rm, int nb, int ns,
                                                     double* __restrict__ x,
                                                     const SolveState* __restrict__ st) {
    if (st->done) return;
    const int p = threadIdx.x;
    if (p >= ns) return;
    for (int i = nb - 1; i >= 0; i--) {
        double v = x[i * ns + p];
        for (int k = i + 1; k < nb; k++) v -= Rm[i * nb + k] * x[k * ns + p];
        x[i * ns + p] = v / Rm[i * nb + i];
    }
}

// PSFM_SYNC: wait for the stream, then return the status the device wrote.
static int sync_status(const psfm_context* ctx, const psfm_fit_stats* stats, hipStream_t st) {
    if (!(ctx->cfg.flags & PSFM_SYNC)) return PSFM_OK;
    int info = 0;
    PSFM_HIP_CHECK(hipMemcpyAsync(&info, &stats->info, sizeof(int), hipMemcpyDeviceToHost, st));
    PSFM_HIP_CHECK(hipStreamSynchronize(st));
    if (info > 0) return PSFM_ERR_NOT_PD;
    return info;   // 0, PSFM_ERR_TOO_FEW_STAMPS or PSFM_ERR_NORM_SINGULAR
}

static int solve_impl(const psfm_context* ctx, int W, int H, const int32_t* stamp_xy, int n_stamps,
                      const double* stamp_M, const double* stamp_b, const double* stamp_e,
                      const int32_t* stamp_npix, int32_t* stamp_flags, const float* stamp_design,
                      const double* prior, double* coeffs, double* stamp_chi2,
                      psfm_fit_stats* stats, void* ws, size_t ws_bytes, hipStream_t st,
                      const double* penq = nullptr, double phi = 0.0, int pen_nb = 0) {
    if (!ctx || n_stamps < 0 || !coeffs || !stats) return PSFM_ERR_INVALID_ARG;
    const bool mixed = ctx->cfg.precision != PSFM_PREC_FP32;
    if (mixed && n_stamps > 0 && !stamp_design) return PSFM_ERR_INVALID_ARG;
    if (W < 1 || H < 1) return PSFM_ERR_SHAPE;
    if (n_stamps > 0 && (!stamp_xy || !stamp_M || !stamp_b || !stamp_e || !stamp_npix ||
                         !stamp_flags || !stamp_chi2))
        return PSFM_ERR_INVALID_ARG;
    if (ctx->N > CH_NMAX) return PSFM_ERR_UNSUPPORTED;
    if (prior && ctx->L > 64) return PSFM_ERR_UNSUPPORTED;
    const bool ortho = ctx->cfg.ortho_basis != 0;
    if (ortho && (mixed || penq || ctx->L > 63)) return PSFM_ERR_UNSUPPORTED;
    const size_t need = psfm::solve_workspace(ctx, n_stamps);
    if (!ws || ws_bytes < need) return PSFM_ERR_WORKSPACE;
    const size_t lds = psfm::solve_lds_bytes(ctx->N);
    psfm::Carver c(ws);
    SolveState* state = c.take<SolveState>(1);
    uint8_t* used = c.take<uint8_t>(n_stamps + 1);
    uint8_t* fitted = c.take<uint8_t>(n_stamps + 1);
    double* G = c.take<double>((size_t)n_stamps * ctx->ns + 1);
    double* M = c.take<double>((size_t)ctx->N * ctx->N);
    double* b = c.take<double>(ctx->N);
    double* ILg = c.take<double>(psfm::solve_il_doubles(ctx->N));
    double* Dg = c.take<double>(ctx->N);
    double* gt = c.take<double>((size_t)n_stamps * ctx->L + 1);
    double* gv = c.take<double>(ctx->N);
    double* palpha = c.take<double>((size_t)n_stamps * ctx->L + 1);
    double* pchi2 = c.take<double>(n_stamps + 1);
    double* wchi2 = c.take<double>(n_stamps + 1);
    double* a0 = c.take<double>(ctx->N);
    double* pdof = c.take<double>(1);
    int* pcounts = c.take<int>(4);
    double* pls = c.take<double>((size_t)n_stamps * ctx->L + 1);
    double* pchi2ls = c.take<double>(n_stamps + 1);
    uint8_t* ptrust = c.take<uint8_t>(n_stamps + 1);
    c.take<double>(2);
    c.take<uint8_t>(n_stamps + 1);
    c.take<uint8_t>(n_stamps + 1);
    double* LT = mixed ? c.take<double>((size_t)ctx->N * ctx->N) : nullptr;   // transposed factor
    double* Mo = ortho ? c.take<double>((size_t)n_stamps * ctx->L * ctx->L + 1) : nullptr;
    double* bo = ortho ? c.take<double>((size_t)n_stamps * ctx->L + 1) : nullptr;
    const int nb = ctx->nb, ns = ctx->ns, N = ctx->N, L = ctx->L;
    const int npix = (2 * ctx->r + 1) * (2 * ctx->r + 1);
    const psfm_config& cf = ctx->cfg;
    int rc = psfm::solve_lds_grant(lds);
    if (rc) return rc;
    const int nt = std::max(n_stamps, N);
    const int n_init = (nt + 255) / 256;
    if (ortho && n_stamps > 0)
        hipLaunchKernelGGL(k_ortho_stamps, dim3(n_stamps), dim3(64), 0, st, ctx->kgram_R, nb, L, stamp_M,
                           stamp_b, Mo, bo);
    // the assembly reads the (mapped) sums; the residuals read the originals
    const double* Ma = ortho ? Mo : stamp_M;
    const double* ba = ortho ? bo : stamp_b;
    hipLaunchKernelGGL(k_solve_prep, dim3(n_init), dim3(256), 0, st, n_stamps, N, ns, cf.spatial_order, W,
                       H, cf.min_stamps, stamp_xy, stamp_flags, used, fitted, G, stamp_chi2, coeffs, state);
    PSFM_HIP_CHECK(hipGetLastError());
    if (prior && n_stamps > 0) {
        // completed predictions, the 1.05x rule against each stamp's own
        // least-squares kernel, then (warm start -> kernel-sum clip) rounds
        hipLaunchKernelGGL(k_prior_chi2, dim3(n_stamps), dim3(64), 0, st, nb, stamp_M, stamp_b, stamp_e,
                           stamp_flags, prior, palpha, pchi2);
        hipLaunchKernelGGL(k_solve_stamps, dim3(n_stamps), dim3(64), 0, st, L, stamp_M, stamp_b,
                           stamp_e, stamp_flags, pls, pchi2ls);
        hipLaunchKernelGGL(k_prior_trust, dim3(1), dim3(1024), 0, st, n_stamps, L, stamp_flags, palpha,
                           pchi2, pls, pchi2ls, ptrust, pcounts);
        for (int it = 0; it < cf.max_iter + 1; it++) {
            hipLaunchKernelGGL(k_prior_warm, dim3(1), dim3(PRIOR_T), 0, st, n_stamps, nb, ns, N, G,
                               palpha, used, ptrust, a0, state, 0);
            hipLaunchKernelGGL(k_chi2, dim3(n_stamps), dim3(64), 0, st, nb, ns, N, stamp_M, stamp_b,
                               stamp_e, G, a0, fitted, wchi2, state);
            hipLaunchKernelGGL(k_prior_clip, dim3(1), dim3(1024), 0, st, n_stamps, ns, L, cf.min_stamps,
                               cf.clip_sigma, G, palpha, a0, ptrust, wchi2, stamp_npix, used, stamp_flags,
                               state);
        }
        hipLaunchKernelGGL(k_prior_warm, dim3(1), dim3(PRIOR_T), 0, st, n_stamps, nb, ns, N, G, palpha,
                           used, ptrust, a0, state, 1);
        hipLaunchKernelGGL(k_chi2, dim3(n_stamps), dim3(64), 0, st, nb, ns, N, stamp_M, stamp_b,
                           stamp_e, G, a0, fitted, wchi2, state);
        hipLaunchKernelGGL(k_prior_dof, dim3(1), dim3(1024), 0, st, n_stamps, N, stamp_npix, used, wchi2,
                           pdof, state);
        PSFM_HIP_CHECK(hipGetLastError());
    }
    // one round: assembly, solution (+ refinement), chi2, clip
    auto round = [&]() -> int {
        if (L > 64) {            // the two-kernel form's stamp matrices (up to 128 wide)
            switch (ns) {
#define PSFM_ASM_CASE(NSV) \
    case NSV: hipLaunchKernelGGL((k_assemble<NSV, 2>), dim3(asm_width<NSV>(nb)), dim3(64 * ASM_WAVES), 0, st, n_stamps, nb, N, Ma, ba, G, used, M, b, state); break;
                PSFM_ASM_CASE(1) PSFM_ASM_CASE(3) PSFM_ASM_CASE(6)
#undef PSFM_ASM_CASE
                default: return PSFM_ERR_UNSUPPORTED;
            }
        } else {
            switch (ns) {
#define PSFM_ASM_CASE(NSV) \
    case NSV: hipLaunchKernelGGL((k_assemble<NSV, 1>), dim3(asm_width<NSV>(nb)), dim3(64 * ASM_WAVES), 0, st, n_stamps, nb, N, Ma, ba, G, used, M, b, state); break;
                PSFM_ASM_CASE(1) PSFM_ASM_CASE(3) PSFM_ASM_CASE(6) PSFM_ASM_CASE(10) PSFM_ASM_CASE(15)
                PSFM_ASM_CASE(21) PSFM_ASM_CASE(28)
#undef PSFM_ASM_CASE
                default: return PSFM_ERR_UNSUPPORTED;
            }
        }
        if (penq)
            hipLaunchKernelGGL(k_penalty, dim3(1), dim3(1024), 0, st, N, ns, nb, pen_nb, penq, phi, M,
                               state);
        hipLaunchKernelGGL(k_cholesky<false>, dim3(1), dim3(CH_THREADS), lds, st, N, M, b, coeffs, ILg,
                           mixed ? Dg : nullptr, state, nullptr, nullptr,
                           mixed && n_stamps > 0 ? LT : nullptr);
        if (ortho)
            hipLaunchKernelGGL(k_ortho_coeffs, dim3(1), dim3(64), 0, st, ctx->kgram_R, nb, ns, coeffs, state);
        if (mixed && n_stamps > 0) {
            // 16-bit sums: refine against FP32 pixel residuals, then chi2 from pixels
            for (int k = 0; k < cf.refine; k++) {
                hipLaunchKernelGGL(k_resid, dim3(n_stamps), dim3(RES_T), 0, st, n_stamps, nb, ns, N,
                                   npix, stamp_design, G, coeffs, fitted, gt, stamp_chi2, state);
                hipLaunchKernelGGL(k_assemble_vec, dim3(N), dim3(64), 0, st, n_stamps,
                                   nb, ns, N, gt, G, used, gv, state);
                hipLaunchKernelGGL(k_resolve, dim3(1), dim3(CH_THREADS), lds, st, N, M, LT, ILg, Dg,
                                   gv, coeffs, state);
            }
            hipLaunchKernelGGL(k_resid, dim3(n_stamps), dim3(RES_T), 0, st, n_stamps, nb, ns, N, npix,
                               stamp_design, G, coeffs, fitted, gt, stamp_chi2, state);
        } else if (n_stamps > 0) {
            hipLaunchKernelGGL(k_chi2_clip, dim3(n_stamps), dim3(64), 0, st, n_stamps, nb, ns, N,
                               stamp_M, stamp_b, stamp_e, G, coeffs, fitted, stamp_chi2, cf.max_iter,
                               cf.min_stamps, cf.clip_sigma, stamp_npix, used, stamp_flags, state);
            return PSFM_OK;
        }
        hipLaunchKernelGGL(k_clip, dim3(1), dim3(1024), 0, st, n_stamps, cf.max_iter, cf.min_stamps,
                           cf.clip_sigma, stamp_npix, used, stamp_flags, stamp_chi2, state);
        return PSFM_OK;
    };
    for (int it = 0; it < cf.max_iter; it++) {
        rc = round();
        if (rc) return rc;
    }
    if (prior && n_stamps > 0) {
        // the least-squares solution judges the prior; on a fallback the full
        // method reruns from the complete stamp set
        hipLaunchKernelGGL(k_prior_fallback, dim3(1), dim3(1024), 0, st, n_stamps, cf.clip_sigma,
                           stamp_npix, fitted, used, stamp_flags, stamp_chi2, state, pcounts);
        for (int it = 0; it < cf.max_iter; it++) {   // idle unless the full method reruns
            rc = round();
            if (rc) return rc;
        }
    }
    hipLaunchKernelGGL(k_solve_finish, dim3(1), dim3(1024), 0, st, n_stamps, ns, N, N,
                       cf.spatial_order, W, H, stamp_npix, used, stamp_chi2, coeffs, state, stats);
    if (prior && n_stamps > 0)
        hipLaunchKernelGGL(k_prior_finish, dim3(1), dim3(64), 0, st, pdof, pcounts, stats);
    PSFM_HIP_CHECK(hipGetLastError());
    return sync_status(ctx, stats, st);
}

extern "C" int psfm_solve(const psfm_context* ctx, int W, int H, const int32_t* stamp_xy,
                          int n_stamps, const double* stamp_M, const double* stamp_b,
                          const double* stamp_e, const int32_t* stamp_npix, int32_t* stamp_flags,
                          const float* stamp_design, double* coeffs, double* stamp_chi2,
                          psfm_fit_stats* stats, void* ws, size_t ws_bytes, void* stream) {
    return solve_impl(ctx, W, H, stamp_xy, n_stamps, stamp_M, stamp_b, stamp_e, stamp_npix,
                      stamp_flags, stamp_design, nullptr, coeffs, stamp_chi2, stats, ws, ws_bytes,
                      (hipStream_t)stream);
}

extern "C" int psfm_solve_prior(const psfm_context* ctx, int W, int H, const int32_t* stamp_xy,
                                int n_stamps, const double* stamp_M, const double* stamp_b,
                                const double* stamp_e, const int32_t* stamp_npix,
                                int32_t* stamp_flags, const float* stamp_design,
                                const double* stamp_pred, double* coeffs, double* stamp_chi2,
                                psfm_fit_stats* stats, void* ws, size_t ws_bytes, void* stream) {
    if (n_stamps > 0 && !stamp_pred) return PSFM_ERR_INVALID_ARG;
    return solve_impl(ctx, W, H, stamp_xy, n_stamps, stamp_M, stamp_b, stamp_e, stamp_npix,
                      stamp_flags, stamp_design, stamp_pred, coeffs, stamp_chi2, stats, ws, ws_bytes,
                      (hipStream_t)stream);
}

extern "C" size_t psfm_cholesky_workspace_bytes(int n) {
    if (n < 1) return 0;
    psfm::Carver c(nullptr);
    c.take<SolveState>(1);
    c.take<double>((size_t)n * n);
    c.take<double>(psfm::solve_il_doubles(n));
    return c.off + 256;
}

extern "C" int psfm_cholesky_solve(int n, const double* M, const double* b, double* x, int* info,
                                   void* ws, size_t ws_bytes, void* stream) {
    if (n < 1 || !M || !b || !x || !info) return PSFM_ERR_INVALID_ARG;
    if (n > CH_NMAX) return PSFM_ERR_UNSUPPORTED;
    if (!ws || ws_bytes < psfm_cholesky_workspace_bytes(n)) return PSFM_ERR_WORKSPACE;
    const size_t lds = psfm::solve_lds_bytes(n);
    int rc = psfm::solve_lds_grant(lds);
    if (rc) return rc;
    hipStream_t st = (hipStream_t)stream;
    psfm::Carver c(ws);
    SolveState* state = c.take<SolveState>(1);
    double* A = c.take<double>((size_t)n * n);
    double* ILg = c.take<double>(psfm::solve_il_doubles(n));
    hipLaunchKernelGGL(k_cholesky<true>, dim3(1), dim3(CH_THREADS), lds, st, n, A, b, x, ILg, nullptr,
                       state, M, info, nullptr);
    PSFM_HIP_CHECK(hipGetLastError());
    return PSFM_OK;
}

extern "C" int psfm_solve_stamps(const psfm_context* ctx, int n_stamps, const double* stamp_M,
                                 const double* stamp_b, const double* stamp_e,
                                 const int32_t* stamp_flags, double* local, double* stamp_chi2,
                                 void* stream) {
    if (!ctx || n_stamps < 0) return PSFM_ERR_INVALID_ARG;
    if (n_stamps == 0) return PSFM_OK;
    if (!stamp_M || !stamp_b || !stamp_e || !stamp_flags || !local || !stamp_chi2)
        return PSFM_ERR_INVALID_ARG;
    if (ctx->L > 64) return PSFM_ERR_UNSUPPORTED;
    hipLaunchKernelGGL(k_solve_stamps, dim3(n_stamps), dim3(64), 0, (hipStream_t)stream, ctx->L,
                       stamp_M, stamp_b, stamp_e, stamp_flags, local, stamp_chi2);
    PSFM_HIP_CHECK(hipGetLastError());
    return PSFM_OK;
}

extern "C" int psfm_solve_norm(const psfm_context* ctx, int W, int H, const int32_t* stamp_xy,
                               int n_stamps, const double* stamp_M, const double* stamp_b,
                               const double* stamp_e, const int32_t* stamp_npix,
                               const double* stamp_norm, const int32_t* stamp_group,
                               int32_t* stamp_flags, double* coeffs, double* stamp_chi2,
                               psfm_fit_stats* stats, void* ws, size_t ws_bytes, void* stream) {
    if (!ctx || n_stamps < 0 || !coeffs || !stats) return PSFM_ERR_INVALID_ARG;
    if (ctx->cfg.precision != PSFM_PREC_FP32 || ctx->cfg.ortho_basis) return PSFM_ERR_UNSUPPORTED;
    if (W < 1 || H < 1) return PSFM_ERR_SHAPE;
    if (n_stamps > 0 && (!stamp_xy || !stamp_M || !stamp_b || !stamp_e || !stamp_npix ||
                         !stamp_norm || !stamp_flags || !stamp_chi2))
        return PSFM_ERR_INVALID_ARG;
    if (ctx->N > CH_NMAX) return PSFM_ERR_UNSUPPORTED;
    const size_t need = psfm::solve_workspace(ctx, n_stamps);
    if (!ws || ws_bytes < need) return PSFM_ERR_WORKSPACE;
    hipStream_t st = (hipStream_t)stream;
    const size_t lds = psfm::solve_lds_bytes(ctx->N);
    const int nb = ctx->nb, ns = ctx->ns, N = ctx->N, L = ctx->L;
    psfm::Carver c(ws);
    SolveState* state = c.take<SolveState>(1);
    uint8_t* used = c.take<uint8_t>(n_stamps + 1);
    uint8_t* fitted = c.take<uint8_t>(n_stamps + 1);
    double* G = c.take<double>((size_t)n_stamps * ns + 1);
    double* M = c.take<double>((size_t)N * N);
    double* b = c.take<double>(N);
    double* ILg = c.take<double>(psfm::solve_il_doubles(N));
    c.take<double>(N);
    c.take<double>((size_t)n_stamps * L + 1);
    c.take<double>(N);
    c.take<double>((size_t)n_stamps * L + 1);
    c.take<double>(n_stamps + 1);
    c.take<double>(n_stamps + 1);
    c.take<double>(N);
    c.take<double>(1);
    c.take<int>(4);
    c.take<double>((size_t)n_stamps * L + 1);
    c.take<double>(n_stamps + 1);
    c.take<uint8_t>(n_stamps + 1);
    double* hv = c.take<double>(2);
    uint8_t* newrej = c.take<uint8_t>(n_stamps + 1);
    uint8_t* act = c.take<uint8_t>(n_stamps + 1);
    const psfm_config& cf = ctx->cfg;
    int rc = psfm::solve_lds_grant(lds);
    if (rc) return rc;
    const int nt = std::max(n_stamps, N);
    const int n_init = (nt + 255) / 256;
    hipLaunchKernelGGL(k_solve_prep, dim3(n_init), dim3(256), 0, st, n_stamps, N, ns, cf.spatial_order, W,
                       H, cf.min_stamps, stamp_xy, stamp_flags, used, fitted, G, stamp_chi2, coeffs, state);
    PSFM_HIP_CHECK(hipGetLastError());
    for (int it = 0; it < cf.max_iter; it++) {
        hipLaunchKernelGGL(k_norm_solve, dim3(1), dim3(1024), 0, st, n_stamps, stamp_norm, used, hv, state);
        switch (ns) {
#define PSFM_ASM_CASE(NSV) \
    case NSV: hipLaunchKernelGGL((k_assemble<NSV, 1>), dim3(asm_width<NSV>(nb)), dim3(64 * ASM_WAVES), 0, st, n_stamps, nb, N, stamp_M, stamp_b, G, used, M, b, state); break;
            PSFM_ASM_CASE(1) PSFM_ASM_CASE(3) PSFM_ASM_CASE(6) PSFM_ASM_CASE(10) PSFM_ASM_CASE(15)
            PSFM_ASM_CASE(21) PSFM_ASM_CASE(28)
#undef PSFM_ASM_CASE
            default: return PSFM_ERR_UNSUPPORTED;
        }
        hipLaunchKernelGGL(k_hold, dim3(1), dim3(1024), 0, st, N, ns, M, b, hv, state);
        hipLaunchKernelGGL(k_cholesky<false>, dim3(1), dim3(CH_THREADS), lds, st, N, M, b, coeffs, ILg,
                           nullptr, state, nullptr, nullptr, nullptr);
        if (n_stamps > 0) {
            hipLaunchKernelGGL(k_chi2, dim3(n_stamps), dim3(64), 0, st, nb, ns, N, stamp_M, stamp_b,
                               stamp_e, G, coeffs, fitted, stamp_chi2, state);
            hipLaunchKernelGGL(k_clip_replace, dim3(1), dim3(1024), 0, st, n_stamps, cf.max_iter,
                               cf.min_stamps, cf.clip_sigma, stamp_npix, stamp_group, used, fitted,
                               stamp_flags, stamp_chi2, newrej, act, state);
        }
        PSFM_HIP_CHECK(hipGetLastError());
    }
    // fitted parameters: the free unknowns plus b0 and d0
    hipLaunchKernelGGL(k_solve_finish, dim3(1), dim3(1024), 0, st, n_stamps, ns, N, N - ns + 1,
                       cf.spatial_order, W, H, stamp_npix, used, stamp_chi2, coeffs, state, stats);
    PSFM_HIP_CHECK(hipGetLastError());
    return sync_status(ctx, stats, st);
}

// The two-kernel form's view of the context: its 2 nb - 1 spatially varying
// columns take the place of the nb basis terms (stamp matrices 2 nb wide).
static psfm_context dual_view(const psfm_context* ctx) {
    psfm_context d = *ctx;
    d.nb = 2 * ctx->nb - 1;
    d.L = 2 * ctx->nb;
    d.N = d.nb * ctx->ns + 1;
    d.cfg.precision = PSFM_PREC_FP32;
    return d;
}

namespace psfm {
size_t dual_solve_workspace(const psfm_context* ctx, int n_stamps) {
    const psfm_context d = dual_view(ctx);
    return solve_workspace(&d, n_stamps);
}
int dual_unknowns(const psfm_context* ctx) { return (2 * ctx->nb - 1) * ctx->ns + 1; }
}  // namespace psfm

extern "C" int psfm_solve_dual(const psfm_context* ctx, int W, int H, const int32_t* stamp_xy,
                               int n_stamps, const double* stamp_M, const double* stamp_b,
                               const double* stamp_e, const int32_t* stamp_npix, int32_t* stamp_flags,
                               double phi, double* coeffs, double* stamp_chi2, psfm_fit_stats* stats,
                               void* ws, size_t ws_bytes, void* stream) {
    if (!ctx || !(phi >= 0.0)) return PSFM_ERR_INVALID_ARG;
    if (ctx->cfg.ortho_basis) return PSFM_ERR_UNSUPPORTED;
    const psfm_context d = dual_view(ctx);
    if (d.L > 128) return PSFM_ERR_UNSUPPORTED;
    return solve_impl(&d, W, H, stamp_xy, n_stamps, stamp_M, stamp_b, stamp_e, stamp_npix, stamp_flags,
                      nullptr, nullptr, coeffs, stamp_chi2, stats, ws, ws_bytes, (hipStream_t)stream,
                      ctx->penq, phi, ctx->nb);
}
