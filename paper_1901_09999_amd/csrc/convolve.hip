// Application of the solution to the whole image (Sections 3.4, 3.5, 4.2, 4.3).
//
//   k_conv_tile      one workgroup per 64 x 64 output tile inside a
//                    constant-kernel patch.  Prologue: local coefficients at
//                    the patch centre, K_p = sum alpha_i k_i in FP64 through
//                    the separable factors, the BAD box radius and the
//                    covariance factor; FP32 taps (K_p, or f_p K_p^2 for the
//                    variance) kept column-major in LDS.  Body: halo tile of
//                    the (masked -> 0) input in LDS, direct (2h+1)^2-tap
//                    convolution on the FP32 VALU with 16 outputs per thread
//                    in registers and the taps broadcast from LDS; for images
//                    also the BAD/POOR mask from a bit-packed halo mask.
//   k_cov_auto /     covariance pseudo-matrix of the kernels realised at the
//   k_cov_mix /      centres of a 3 x 3 partition: each kernel's normalised
//   k_cov_finish     autocorrelation (one row of offsets per wave), folded
//                    with a correlated input's pseudo-matrix when there is
//                    one, then averaged, normalised to the centre, cropped.
//   k_subtract /     difference image, its variance and mask, per-block
//   k_subtract_cov   variance sums and the weighted pseudo-matrix.
#include "internal.h"

namespace {

constexpr int TILE = PSFM_TILE;

struct PatchGeom {
    int npx, npy, tpp;
};

__host__ __device__ inline PatchGeom patch_geom(int W, int H, int P) {
    PatchGeom g;
    g.npx = (W + P - 1) / P;
    g.npy = (H + P - 1) / P;
    g.tpp = (P + TILE - 1) / TILE;
    return g;
}

// Orders a wave's LDS writes before its other lanes' reads.
__device__ __forceinline__ void wave_sync_lds() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Basis tables as kernel arguments.
struct BasisArgs {
    const double* fac64;   // [nf][KW]
    const double* psi64;   // [nb]
    const float* z;        // [nb]
    const int* rowf;       // [nb]
    const int* colf;       // [nb]
    const int* rorder;     // [nb] terms grouped by row factor (increasing i within one)
    const int* rstart;     // [nf + 1] group starts in rorder
    int nb, nf, ns, S, h;
};

// LDS scratch of the kernel realisation.
struct RealiseLds {
    double F[32 * (2 * PSFM_HMAX + 1)];
    double gam[64];
    int rf[64], cf[64];
    int ro[64], rs[33];
};

// Taps per thread of the regrouped realisation (a 256-thread workgroup, up to 33 x 33 taps).
constexpr int RK_MAX = ((2 * PSFM_HMAX + 1) * (2 * PSFM_HMAX + 1) + 255) / 256;

// K(u, v) = sum_i alpha_i(x, y) k_i(u, v) in FP64, evaluated through the
// separable factors: with k_i = psi_i f_{rowf}(u) f_{colf}(v) - z_i k_0,
//   K = sum_i gamma_i f_{rowf_i}(u) f_{colf_i}(v),
//   gamma_i = alpha_i psi_i (i >= 1),  gamma_0 = psi_0 (alpha_0 - sum_i z_i alpha_i).
// When the factors are no more than the kernel side (nf <= 2h + 1), the
// terms are regrouped by row factor first:
//   C_r(v) = sum over the terms i with f_{rowf_i} = f_r (increasing i) of gamma_i f_{colf_i}(v),
//   K(u, v) = sum_r f_r(u) C_r(v)  (increasing r),
// each sum an FMA chain from zero (the table C sits in Kd's space until the
// taps are stored), which is nf instead of nb products per tap.
// Kd receives [(v+h)*KW + (u+h)].  All threads of the block (256) call it.
// skip0: term 0 takes no coefficient (the sum over the zero-sum terms only,
// as in the kernel applied to I2 in the two-kernel form; a then points
// ns coefficients before that kernel's first term).
__device__ void realise_kernel(const BasisArgs& B, const double* __restrict__ a, double x, double y,
                               int W, int H, RealiseLds& sh, double* Kd, bool skip0 = false) {
    const int KW = 2 * B.h + 1, T = KW * KW, tid = threadIdx.x, nb = B.nb, ns = B.ns;
    for (int e = tid; e < B.nf * KW; e += blockDim.x) sh.F[e] = B.fac64[e];
    for (int e = tid; e < nb; e += blockDim.x) sh.ro[e] = B.rorder[e];
    for (int e = tid; e <= B.nf; e += blockDim.x) sh.rs[e] = B.rstart[e];
    if (tid < 64) {
        // wave 0, lane i: alpha_i(x, y) from the term's ns spatial
        // coefficients (all loads issued before the first use), the spatial
        // terms in the order of psfm_spatial_dot
        const int i = tid < nb ? tid : 0;
        double cv[28];
#pragma unroll
        for (int q = 0; q < 28; q++) cv[q] = a[i * ns + (q < ns ? q : 0)];
        const double zi = (double)B.z[i], ps = B.psi64[i];
        const int rf = B.rowf[i], cf = B.colf[i];
        const double xt = W > 1 ? (2.0 * x - (W - 1)) / (double)(W - 1) : 0.0;
        const double yt = H > 1 ? (2.0 * y - (H - 1)) / (double)(H - 1) : 0.0;
        double al = 0.0;
#pragma unroll
        for (int d = 0; d <= 6; d++) {
            if (d <= B.S) {
#pragma unroll
                for (int l = d; l >= 0; l--) {
                    double v = 1.0;
#pragma unroll
                    for (int k = 0; k < l; k++) v *= xt;
#pragma unroll
                    for (int k = 0; k < d - l; k++) v *= yt;
                    al += cv[d * (d + 1) / 2 + (d - l)] * v;
                }
            }
        }
        if (skip0 && tid == 0) al = 0.0;
        // c0 = sum_(i >= 1) z_i alpha_i: fixed-order butterfly over the wave
        double c0 = tid >= 1 && tid < nb ? zi * al : 0.0;
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) c0 += __shfl_xor(c0, o);
        if (tid < nb) {
            sh.gam[tid] = (tid == 0 ? al - c0 : al) * ps;
            sh.rf[tid] = rf;
            sh.cf[tid] = cf;
        }
    }
    __syncthreads();
    const int nf = B.nf;
    if (nf <= KW) {
        double* C = Kd;                                // nf * KW <= T entries
        for (int e = tid; e < nf * KW; e += blockDim.x) {
            const int r = e / KW, v = e - r * KW;
            double c = 0.0;
            for (int m = sh.rs[r]; m < sh.rs[r + 1]; m++) {
                const int i = sh.ro[m];
                c = fma(sh.gam[i], sh.F[sh.cf[i] * KW + v], c);
            }
            C[e] = c;
        }
        __syncthreads();
        double kv[RK_MAX];
#pragma unroll
        for (int k = 0; k < RK_MAX; k++) {
            const int t = tid + 256 * k;
            kv[k] = 0.0;
            if (t < T) {
                const int v = t / KW, u = t - v * KW;
                for (int r = 0; r < nf; r++) kv[k] = fma(sh.F[r * KW + u], C[r * KW + v], kv[k]);
            }
        }
        __syncthreads();                               // C is read; Kd takes the taps
#pragma unroll
        for (int k = 0; k < RK_MAX; k++)
            if (tid + 256 * k < T) Kd[tid + 256 * k] = kv[k];
    } else {
        for (int t = tid; t < T; t += blockDim.x) {
            const int v = t / KW, u = t - v * KW;
            double k4[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll 4
            for (int i = 0; i < nb; i++)
                k4[i & 3] += sh.gam[i] * sh.F[sh.rf[i] * KW + u] * sh.F[sh.cf[i] * KW + v];
            Kd[t] = (k4[0] + k4[1]) + (k4[2] + k4[3]);
        }
    }
    __syncthreads();
}

// Squared-weight ring sums, BAD radius and covariance factor of the kernel
// in Kd (FP64, LDS).  All threads call it; results in *rb_out / *f_out (LDS).
__device__ void kernel_stats(const double* Kd, int h, double bad_frac, const double* __restrict__ cov_in,
                             int c_in, double* ring, double* red, int* rb_out, double* f_out) {
    const int KW = 2 * h + 1, T = KW * KW, tid = threadIdx.x;
    // the sums over the taps are formed by wave 0 alone (lane l: taps l,
    // l + 64, ...), so that they do not depend on the workgroup size
    double s2 = 0.0;
    if (tid < 64)
        for (int t = tid; t < T; t += 64) s2 += Kd[t] * Kd[t];
    const double sumk2 = psfm_block_sum(s2, red);
    if (tid <= h) {   // squared weight on the ring max(|u|,|v|) = tid
        const int rr = tid;
        double s = 0.0;
        for (int v = -rr; v <= rr; v++) {
            const int step = (v == -rr || v == rr || rr == 0) ? 1 : 2 * rr;
            for (int u = -rr; u <= rr; u += step) {
                const double k = Kd[(v + h) * KW + (u + h)];
                s += k * k;
            }
        }
        ring[rr] = s;
    }
    double f = 1.0;
    if (cov_in) {
        const int Cw = 2 * c_in + 1;
        double r0 = 0.0;
        for (int t = tid; tid < 64 && t < T; t += 64) {
            const int v = t / KW - h, u = t % KW - h;
            double q = 0.0;
            for (int wy = -c_in; wy <= c_in; wy++)
                for (int wx = -c_in; wx <= c_in; wx++) {
                    const int u2 = u - wx, v2 = v - wy;
                    if (u2 < -h || u2 > h || v2 < -h || v2 > h) continue;
                    q += cov_in[(wy + c_in) * Cw + (wx + c_in)] * Kd[(v2 + h) * KW + (u2 + h)];
                }
            r0 += Kd[t] * q;
        }
        const double raw0 = psfm_block_sum(r0, red);
        f = sumk2 > 0.0 ? raw0 / sumk2 : 0.0;
    }
    __syncthreads();
    if (tid == 0) {
        int rb = h;
        double outside = 0.0;
        for (int rr = 0; rr <= h; rr++) outside += ring[rr];
        const double tot = outside;
        for (int rr = 0; rr <= h; rr++) {
            outside -= ring[rr];
            if (outside < bad_frac * tot) {
                rb = rr;
                break;
            }
        }
        *rb_out = rb;
        *f_out = f;
    }
    __syncthreads();
}

// Halo tile [HW x HW] of the input around the output tile at (X0, Y0):
// masked and out-of-image pixels read as 0; with BITS, their positions are
// also set in the bit-packed mask badw.  Returns (block-wide) whether any
// halo pixel was masked or outside.
template <int H_, bool BITS>
__device__ int load_halo(const float* __restrict__ src, const uint8_t* __restrict__ M, int W, int H,
                         int64_t pitch, int X0, int Y0, float* __restrict__ halo,
                         uint32_t (*badw)[(TILE + 2 * H_ + 31) / 32 + 1]) {
    constexpr int HW = TILE + 2 * H_;
    constexpr int NWB = (HW + 31) / 32 + 1;
    const int tid = threadIdx.x;
    if (BITS) {
        for (int e = tid; e < HW * NWB; e += 256) (&badw[0][0])[e] = 0u;
        __syncthreads();
    }
    // HALO_CHUNK pixels per thread in flight: the mask and value loads are
    // unconditional (from a clamped in-image address) so none waits on another
    constexpr int HALO_CHUNK = 8;
    int anybad = 0;
    for (int e0 = tid; e0 < HW * HW; e0 += 256 * HALO_CHUNK) {
        uint8_t m[HALO_CHUNK];
        float v[HALO_CHUNK];
        bool in[HALO_CHUNK];
#pragma unroll
        for (int u = 0; u < HALO_CHUNK; u++) {
            const int e = e0 + 256 * u;
            const int hy = e / HW, hx = e - hy * HW;
            const int gy = Y0 - H_ + hy, gx = X0 - H_ + hx;
            in[u] = e < HW * HW && gx >= 0 && gx < W && gy >= 0 && gy < H;
            const int64_t o = in[u] ? (int64_t)gy * pitch + gx : 0;
            m[u] = M[o];
            v[u] = src[o];
        }
#pragma unroll
        for (int u = 0; u < HALO_CHUNK; u++) {
            const int e = e0 + 256 * u;
            if (e >= HW * HW) continue;
            const bool ok = in[u] && m[u] == 0;
            halo[e] = ok ? v[u] : 0.0f;
            if (!ok) {
                anybad = 1;
                if (BITS) {
                    const int hy = e / HW, hx = e - hy * HW;
                    atomicOr(&badw[hy][hx >> 5], 1u << (hx & 31));
                }
            }
        }
    }
    return __syncthreads_or(anybad);
}

// Direct (2h+1)^2-tap convolution of 16 consecutive output rows of column lx
// (rows r0 .. r0+15 of the tile) from the LDS halo; taps column-major in LDS.
template <int H_>
__device__ __forceinline__ void conv16(const float* __restrict__ halo, const float* __restrict__ taps,
                                       int lx, int r0, float acc[16]) {
    constexpr int KW = 2 * H_ + 1;
    constexpr int HW = TILE + 2 * H_;
#pragma unroll
    for (int j = 0; j < 16; j++) acc[j] = 0.0f;
    for (int uu = 0; uu < KW; uu++) {
        float kc[KW];
#pragma unroll
        for (int vv = 0; vv < KW; vv++) kc[vv] = taps[uu * KW + vv];
        const float* col = halo + r0 * HW + lx + 2 * H_ - uu;
#pragma unroll
        for (int hr = 0; hr < 16 + 2 * H_; hr++) {
            const float val = col[hr * HW];
#pragma unroll
            for (int j = 0; j < 16; j++) {
                const int vv = j + 2 * H_ - hr;
                if (vv >= 0 && vv < KW) acc[j] = fmaf(kc[vv], val, acc[j]);
            }
        }
    }
}

// BAD / POOR flags of the 16 outputs from the bit-packed halo mask: POOR if
// a masked input lies within the kernel footprint, BAD if within box
// radius rb.  Bit j of the results is output row r0 + j.
template <int H_>
__device__ __forceinline__ void mask16(const uint32_t (*badw)[(TILE + 2 * H_ + 31) / 32 + 1],
                                       int rb, int lx, int r0, uint32_t* bad16, uint32_t* poor16) {
    constexpr int KW = 2 * H_ + 1;
    const uint64_t kmask = (KW >= 64) ? ~0ull : ((1ull << KW) - 1ull);
    const uint64_t bmask = (1ull << (2 * rb + 1)) - 1ull;
    const int w = lx >> 5, sh = lx & 31;
    uint64_t poorv = 0, badv = 0;
#pragma unroll
    for (int hr = 0; hr < 16 + 2 * H_; hr++) {
        const uint32_t* bw = badw[r0 + hr];
        const uint64_t bits = ((uint64_t)bw[w] | ((uint64_t)bw[w + 1] << 32)) >> sh;
        const uint64_t win = bits & kmask;      // halo columns [lx, lx + 2h]
        if (win) poorv |= 1ull << hr;
        if ((win >> (H_ - rb)) & bmask) badv |= 1ull << hr;
    }
    uint32_t b = 0, q = 0;
#pragma unroll
    for (int j = 0; j < 16; j++) {
        if ((badv >> (j + H_ - rb)) & bmask) b |= 1u << j;
        if ((poorv >> j) & kmask) q |= 1u << j;
    }
    *bad16 = b;
    *poor16 = q;
}

// Realises the patch kernel of patch (px, py) in FP64 in the LDS scratch
// (overlaid on the halo buffer) and stores its FP32 taps column-major:
// tapsK = K (if non-null), tapsV = f K^2 (if non-null).  Returns rb in *rb.
template <int H_>
__device__ void patch_taps(const BasisArgs& B, const double* __restrict__ a, int W, int H, int P,
                           int px, int py, double bad_frac, const double* __restrict__ cov_in,
                           int c_in, float* __restrict__ scratch, float* tapsK, float* tapsV,
                           double* ring, double* red, int* s_rb, double* s_f) {
    constexpr int KW = 2 * H_ + 1;
    constexpr int T = KW * KW;
    RealiseLds& sh = *reinterpret_cast<RealiseLds*>(scratch);
    double* Kd = reinterpret_cast<double*>(reinterpret_cast<char*>(scratch) + sizeof(RealiseLds));
    const int x0 = px * P, x1 = min(x0 + P, W), y0 = py * P, y1 = min(y0 + P, H);
    realise_kernel(B, a, 0.5 * (x0 + x1 - 1), 0.5 * (y0 + y1 - 1), W, H, sh, Kd);
    kernel_stats(Kd, H_, bad_frac, tapsV ? cov_in : nullptr, c_in, ring, red, s_rb, s_f);
    const double f = *s_f;
    for (int t = threadIdx.x; t < T; t += 256) {
        const int uu = t / KW, vv = t - uu * KW;     // column-major
        const double k = Kd[vv * KW + uu];
        if (tapsK) tapsK[t] = (float)k;
        if (tapsV) tapsV[t] = (float)(f * k * k);
    }
    __syncthreads();
}

// One workgroup per 64 x 64 output tile inside a constant-kernel patch.
// MODE 0: image I' (and the BAD/POOR mask); MODE 1: variance V' = f K^2 (x) V.
template <int H_, int MODE>
__global__ __launch_bounds__(256) void k_conv_tile(
    const float* __restrict__ src, const uint8_t* __restrict__ M, int W, int H, int64_t pitch,
    int P, const double* __restrict__ a, BasisArgs B, double bad_frac,
    const double* __restrict__ cov_in, int c_in, float* __restrict__ out,
    uint8_t* __restrict__ out_mask) {
    constexpr int KW = 2 * H_ + 1;
    constexpr int T = KW * KW;
    constexpr int HW = TILE + 2 * H_;
    constexpr int NWB = (HW + 31) / 32 + 1;
    static_assert(sizeof(float) * HW * HW >= sizeof(RealiseLds) + sizeof(double) * T,
                  "kernel scratch must fit in the halo buffer");
    __shared__ __align__(16) float halo[HW * HW];
    __shared__ __align__(16) float taps[T + 4];
    __shared__ uint32_t badw[HW][NWB];
    __shared__ double ring[H_ + 1];
    __shared__ double red[16];
    __shared__ int s_rb;
    __shared__ double s_f;
    const int tid = threadIdx.x;
    const PatchGeom g = patch_geom(W, H, P);
    // tiles XCD by XCD (workgroup L of the launch runs on XCD L mod 8): XCD x
    // takes the x-th contiguous eighth of the tiles in row-major order, whose
    // halos overlap in that XCD's L2
    const int ngx = gridDim.x, nt = ngx * gridDim.y, L = blockIdx.y * ngx + blockIdx.x;
    const int xq = L & 7, kq = L >> 3, qq = nt >> 3, rq = nt & 7;
    const int tl = xq * qq + (xq < rq ? xq : rq) + kq, tx = tl % ngx, ty = tl / ngx;
    const int px = tx / g.tpp, sx = tx % g.tpp;
    const int py = ty / g.tpp, sy = ty % g.tpp;
    const int X0 = px * P + sx * TILE, Y0 = py * P + sy * TILE;
    const int X1 = min(min(X0 + TILE, (px + 1) * P), W);
    const int Y1 = min(min(Y0 + TILE, (py + 1) * P), H);
    if (X0 >= X1 || Y0 >= Y1) return;

    patch_taps<H_>(B, a, W, H, P, px, py, bad_frac, cov_in, c_in, halo, MODE == 0 ? taps : nullptr,
                   MODE == 1 ? taps : nullptr, ring, red, &s_rb, &s_f);
    const int anybad = load_halo<H_, MODE == 0>(src, M, W, H, pitch, X0, Y0, halo, badw);

    const int lx = tid & 63;
    const int r0 = (tid >> 6) * 16;
    float acc[16];
    conv16<H_>(halo, taps, lx, r0, acc);
    const int gx = X0 + lx;
    if (gx < X1) {
#pragma unroll
        for (int j = 0; j < 16; j++) {
            const int gy = Y0 + r0 + j;
            if (gy < Y1) out[(int64_t)gy * pitch + gx] = acc[j];
        }
    }
    if (MODE == 0) {
        uint32_t bad16 = 0, poor16 = 0;
        if (anybad) mask16<H_>(badw, s_rb, lx, r0, &bad16, &poor16);
        if (gx < X1) {
#pragma unroll
            for (int j = 0; j < 16; j++) {
                const int gy = Y0 + r0 + j;
                if (gy < Y1) {
                    const uint8_t m = ((bad16 >> j) & 1u) ? PSFM_MASK_CONV_BAD
                                      : ((poor16 >> j) & 1u) ? PSFM_MASK_CONV_POOR : 0;
                    out_mask[(int64_t)gy * pitch + gx] = m;
                }
            }
        }
    }
}

template <int H_, int MODE>
int launch_conv(const float* src, const uint8_t* M, int W, int H, int64_t pitch, int P,
                const double* a, const BasisArgs& B, double bad_frac, const double* cov_in,
                int c_in, float* out, uint8_t* out_mask, hipStream_t st) {
    const PatchGeom g = patch_geom(W, H, P);
    dim3 grid(g.npx * g.tpp, g.npy * g.tpp);
    hipLaunchKernelGGL((k_conv_tile<H_, MODE>), grid, dim3(256), 0, st, src, M, W, H, pitch, P, a, B,
                       bad_frac, cov_in, c_in, out, out_mask);
    PSFM_HIP_CHECK(hipGetLastError());
    return PSFM_OK;
}

template <int MODE>
int dispatch_conv(const float* src, const uint8_t* M, int W, int H, int64_t pitch, int P,
                  const double* a, const BasisArgs& B, double bad_frac, const double* cov_in,
                  int c_in, float* out, uint8_t* out_mask, hipStream_t st) {
    switch (B.h) {
#define PSFM_CONV_CASE(HH) \
    case HH: return launch_conv<HH, MODE>(src, M, W, H, pitch, P, a, B, bad_frac, cov_in, c_in, out, out_mask, st);
        PSFM_CONV_CASE(1) PSFM_CONV_CASE(2) PSFM_CONV_CASE(3) PSFM_CONV_CASE(4) PSFM_CONV_CASE(5)
        PSFM_CONV_CASE(6) PSFM_CONV_CASE(7) PSFM_CONV_CASE(8) PSFM_CONV_CASE(9) PSFM_CONV_CASE(10)
        PSFM_CONV_CASE(11) PSFM_CONV_CASE(12) PSFM_CONV_CASE(13) PSFM_CONV_CASE(14)
        PSFM_CONV_CASE(15) PSFM_CONV_CASE(16)
#undef PSFM_CONV_CASE
        default: return PSFM_ERR_UNSUPPORTED;
    }
}

// Image and variance convolution of one tile in one workgroup: the patch
// kernel and its statistics are realised once (both tap sets), then the
// halo of I (with the mask bits) gives I' and its mask, and the halo of V
// (same buffer, after every wave is done with I) gives V'.  The arithmetic
// of each plane is that of k_conv_tile<H_, 0> and <H_, 1>.
template <int H_>
__global__ __launch_bounds__(256) void k_conv_pair_tile(
    const float* __restrict__ I, const float* __restrict__ V, const uint8_t* __restrict__ M, int W,
    int H, int64_t pitch, int P, const double* __restrict__ a, BasisArgs B, double bad_frac,
    const double* __restrict__ cov_in, int c_in, float* __restrict__ out,
    uint8_t* __restrict__ out_mask, float* __restrict__ var_out) {
    constexpr int KW = 2 * H_ + 1;
    constexpr int T = KW * KW;
    constexpr int HW = TILE + 2 * H_;
    constexpr int NWB = (HW + 31) / 32 + 1;
    static_assert(sizeof(float) * HW * HW >= sizeof(RealiseLds) + sizeof(double) * T,
                  "kernel scratch must fit in the halo buffer");
    __shared__ __align__(16) float halo[HW * HW];
    __shared__ __align__(16) float tapsK[T + 4];
    __shared__ __align__(16) float tapsV[T + 4];
    __shared__ uint32_t badw[HW][NWB];
    __shared__ double ring[H_ + 1];
    __shared__ double red[16];
    __shared__ int s_rb;
    __shared__ double s_f;
    const int tid = threadIdx.x;
    const PatchGeom g = patch_geom(W, H, P);
    // tiles XCD by XCD (workgroup L of the launch runs on XCD L mod 8): XCD x
    // takes the x-th contiguous eighth of the tiles in row-major order, whose
    // halos overlap in that XCD's L2
    const int ngx = gridDim.x, nt = ngx * gridDim.y, L = blockIdx.y * ngx + blockIdx.x;
    const int xq = L & 7, kq = L >> 3, qq = nt >> 3, rq = nt & 7;
    const int tl = xq * qq + (xq < rq ? xq : rq) + kq, tx = tl % ngx, ty = tl / ngx;
    const int px = tx / g.tpp, sx = tx % g.tpp;
    const int py = ty / g.tpp, sy = ty % g.tpp;
    const int X0 = px * P + sx * TILE, Y0 = py * P + sy * TILE;
    const int X1 = min(min(X0 + TILE, (px + 1) * P), W);
    const int Y1 = min(min(Y0 + TILE, (py + 1) * P), H);
    if (X0 >= X1 || Y0 >= Y1) return;

    patch_taps<H_>(B, a, W, H, P, px, py, bad_frac, cov_in, c_in, halo, tapsK, tapsV, ring, red,
                   &s_rb, &s_f);
    const int lx = tid & 63;
    const int r0 = (tid >> 6) * 16;
    const int gx = X0 + lx;
    float acc[16];
    {
        const int anybad = load_halo<H_, true>(I, M, W, H, pitch, X0, Y0, halo, badw);
        conv16<H_>(halo, tapsK, lx, r0, acc);
        uint32_t bad16 = 0, poor16 = 0;
        if (anybad) mask16<H_>(badw, s_rb, lx, r0, &bad16, &poor16);
        if (gx < X1) {
#pragma unroll
            for (int j = 0; j < 16; j++) {
                const int gy = Y0 + r0 + j;
                if (gy < Y1) {
                    out[(int64_t)gy * pitch + gx] = acc[j];
                    out_mask[(int64_t)gy * pitch + gx] = ((bad16 >> j) & 1u) ? PSFM_MASK_CONV_BAD
                                                         : ((poor16 >> j) & 1u) ? PSFM_MASK_CONV_POOR
                                                                                : 0;
                }
            }
        }
    }
    __syncthreads();                       // every wave is done with the image halo
    load_halo<H_, false>(V, M, W, H, pitch, X0, Y0, halo, badw);
    conv16<H_>(halo, tapsV, lx, r0, acc);
    if (gx < X1) {
#pragma unroll
        for (int j = 0; j < 16; j++) {
            const int gy = Y0 + r0 + j;
            if (gy < Y1) var_out[(int64_t)gy * pitch + gx] = acc[j];
        }
    }
}

int dispatch_conv_pair(const float* I, const float* V, const uint8_t* M, int W, int H,
                       int64_t pitch, int P, const double* a, const BasisArgs& B, double bad_frac,
                       const double* cov_in, int c_in, float* out, uint8_t* out_mask,
                       float* var_out, hipStream_t st) {
    const PatchGeom g = patch_geom(W, H, P);
    const dim3 grid(g.npx * g.tpp, g.npy * g.tpp);
    switch (B.h) {
#define PSFM_CP_CASE(HH)                                                                             \
    case HH:                                                                                         \
        hipLaunchKernelGGL((k_conv_pair_tile<HH>), grid, dim3(256), 0, st, I, V, M, W, H, pitch, P,  \
                           a, B, bad_frac, cov_in, c_in, out, out_mask, var_out);                    \
        break;
        PSFM_CP_CASE(1) PSFM_CP_CASE(2) PSFM_CP_CASE(3) PSFM_CP_CASE(4) PSFM_CP_CASE(5)
        PSFM_CP_CASE(6) PSFM_CP_CASE(7) PSFM_CP_CASE(8) PSFM_CP_CASE(9) PSFM_CP_CASE(10)
        PSFM_CP_CASE(11) PSFM_CP_CASE(12) PSFM_CP_CASE(13) PSFM_CP_CASE(14) PSFM_CP_CASE(15)
        PSFM_CP_CASE(16)
#undef PSFM_CP_CASE
        default: return PSFM_ERR_UNSUPPORTED;
    }
    PSFM_HIP_CHECK(hipGetLastError());
    return PSFM_OK;
}

// Normalised autocorrelation of the kernel realised at the centre of cell j
// of the 3 x 3 partition:
//   A(e) = sum_u K(u) K(u + e) / sum_u K(u)^2,   |e_x|, |e_y| <= 2h,
// E = 4h + 1 values a side, row-major at out + j E^2.  Workgroup ry takes
// the row e_y = ry - 2h: its lanes the e_x, its four waves every fourth of
// the kernel rows that overlap (partial sums added in a fixed order).  The
// kernel's rows sit in LDS with 2h zeros either side, so every lane runs
// the same 2h + 1 taps per kernel row.
// Kpre: the cell's kernel realised beforehand (the batch), else realised here.
__device__ void cov_auto_body(const double* __restrict__ a, const BasisArgs& B, int W, int H,
                              double* __restrict__ out, const int j, const int ry,
                              const double* __restrict__ Kpre = nullptr) {
    __shared__ RealiseLds sh;
    __shared__ double Kd[(2 * PSFM_HMAX + 1) * (2 * PSFM_HMAX + 1)];
    __shared__ double Kr[(2 * PSFM_HMAX + 1) * (6 * PSFM_HMAX + 1)];
    __shared__ double part[4][2 * 64];
    __shared__ double red[16];
    const int h = B.h, KW = 2 * h + 1, T = KW * KW, E = 4 * h + 1, RW = 6 * h + 1;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    if (Kpre) {
        for (int t = tid; t < T; t += 256) Kd[t] = Kpre[(size_t)j * T + t];
        __syncthreads();
    } else {
        const int jx = j % 3, jy = j / 3;
        const int cx0 = jx * W / 3, cx1 = (jx + 1) * W / 3, cy0 = jy * H / 3, cy1 = (jy + 1) * H / 3;
        realise_kernel(B, a, 0.5 * (cx0 + cx1 - 1), 0.5 * (cy0 + cy1 - 1), W, H, sh, Kd);
    }
    double s2 = 0.0;
    for (int t = tid; t < T; t += 256) s2 += Kd[t] * Kd[t];
    const double sumk2 = psfm_block_sum(s2, red);
    for (int t = tid; t < KW * RW; t += 256) {
        const int v = t / RW, c = t - v * RW - 2 * h;     // column of K, or padding
        Kr[t] = (c >= 0 && c < KW) ? Kd[v * KW + c] : 0.0;
    }
    __syncthreads();
    const int ey = ry - 2 * h;
    const int v0 = max(-h, -h - ey), v1 = min(h, h - ey);
    for (int q = 0; q < 2; q++) {
        const int xi = lane + 64 * q;                      // xi = e_x + 2h
        double s4[4] = {0.0, 0.0, 0.0, 0.0};
        if (xi < E) {
            for (int v = v0 + wave; v <= v1; v += 4) {
                const double* k1 = Kd + (v + h) * KW;            // K(u, v), uniform over the wave
                const double* k2 = Kr + (v + ey + h) * RW + xi;  // K(u + e_x, v + e_y), u = -h ..
                int u = 0;
                for (; u + 4 <= KW; u += 4) {
                    s4[0] += k1[u] * k2[u];
                    s4[1] += k1[u + 1] * k2[u + 1];
                    s4[2] += k1[u + 2] * k2[u + 2];
                    s4[3] += k1[u + 3] * k2[u + 3];
                }
                for (; u < KW; u++) s4[u & 3] += k1[u] * k2[u];
            }
        }
        part[wave][xi] = (s4[0] + s4[1]) + (s4[2] + s4[3]);
    }
    __syncthreads();
    const double inv = sumk2 > 0.0 ? 1.0 / sumk2 : 0.0;
    if (tid < E)
        out[(size_t)j * E * E + ry * E + tid] =
            (((part[0][tid] + part[1][tid]) + part[2][tid]) + part[3][tid]) * inv;
}

__global__ __launch_bounds__(256) void k_cov_auto(const double* __restrict__ a, BasisArgs B, int W,
                                                  int H, double* __restrict__ out) {
    cov_auto_body(a, B, W, H, out, blockIdx.x, blockIdx.y);
}

// Correlated input: raw(delta) / sum K^2 = sum_w C_in(w) A(delta - w) for
// |delta_x|, |delta_y| <= R = 2h + c_in, from the normalised autocorrelation
// A of cell j (E^2 values, staged in LDS); chunk selects 256 of the offsets.
__device__ void cov_mix_body(const double* __restrict__ A, int h, const double* __restrict__ cov_in,
                             int c_in, double* __restrict__ samples, const int j, const int chunk) {
    __shared__ double As[(4 * PSFM_HMAX + 1) * (4 * PSFM_HMAX + 1)];
    const int E = 4 * h + 1, R = 2 * h + c_in, Rw = 2 * R + 1, Cw = 2 * c_in + 1;
    for (int t = threadIdx.x; t < E * E; t += 256) As[t] = A[(size_t)j * E * E + t];
    __syncthreads();
    const int d = chunk * 256 + threadIdx.x;
    if (d >= Rw * Rw) return;
    const int dy = d / Rw - R, dx = d % Rw - R;
    double s2[2] = {0.0, 0.0};
    for (int wy = -c_in; wy <= c_in; wy++) {
        const int ey = dy - wy;
        if (ey < -2 * h || ey > 2 * h) continue;
        const double* crow = cov_in + (wy + c_in) * Cw + c_in;
        const double* arow = As + (ey + 2 * h) * E + 2 * h;
        for (int wx = -c_in; wx <= c_in; wx++) {
            const int ex = dx - wx;
            const bool in = ex >= -2 * h && ex <= 2 * h;
            const double av = arow[in ? ex : 0];
            s2[wx & 1] += in ? crow[wx] * av : 0.0;
        }
    }
    samples[(size_t)j * Rw * Rw + d] = s2[0] + s2[1];
}

__global__ __launch_bounds__(256) void k_cov_mix(const double* __restrict__ A, int h,
                                                 const double* __restrict__ cov_in, int c_in,
                                                 double* __restrict__ samples) {
    cov_mix_body(A, h, cov_in, c_in, samples, blockIdx.x, blockIdx.y);
}

// Batched: each cell kernel of each pair realised once (the same function,
// so the same values as a workgroup of k_cov_auto realises), then the
// autocorrelation rows read it; they go straight to the samples of a pair
// with an uncorrelated input, else to its cov_auto buffer for k_cov_mix_b.
__global__ __launch_bounds__(256) void k_cell_kernels_b(const PairDesc* __restrict__ pairs, BasisArgs B0) {
    __shared__ RealiseLds sh;
    __shared__ double Kd[(2 * PSFM_HMAX + 1) * (2 * PSFM_HMAX + 1)];
    const PairDesc& p = pairs[blockIdx.y];
    BasisArgs B = B0;
    B.ns = p.ns;
    B.S = p.S;
    const int j = blockIdx.x, W = p.W, H = p.H, T = (2 * B.h + 1) * (2 * B.h + 1);
    const int jx = j % 3, jy = j / 3;
    const int cx0 = jx * W / 3, cx1 = (jx + 1) * W / 3, cy0 = jy * H / 3, cy1 = (jy + 1) * H / 3;
    realise_kernel(B, p.coeffs, 0.5 * (cx0 + cx1 - 1), 0.5 * (cy0 + cy1 - 1), W, H, sh, Kd);
    for (int t = threadIdx.x; t < T; t += 256) p.cellK[(size_t)j * T + t] = Kd[t];
}

__global__ __launch_bounds__(256) void k_cov_auto_b(const PairDesc* __restrict__ pairs, BasisArgs B0) {
    const PairDesc& p = pairs[blockIdx.z];
    BasisArgs B = B0;
    B.ns = p.ns;
    B.S = p.S;
    cov_auto_body(p.coeffs, B, p.W, p.H, p.cov1 ? p.cov_auto : p.cov_samples, blockIdx.x, blockIdx.y,
                  p.cellK);
}

__global__ __launch_bounds__(256) void k_cov_mix_b(const PairDesc* __restrict__ pairs, int h) {
    const PairDesc& p = pairs[blockIdx.z];
    if (!p.cov1) return;
    const int Rw = 2 * (2 * h + p.cov1_half) + 1;
    if ((int)blockIdx.y * 256 >= Rw * Rw) return;
    cov_mix_body(p.cov_auto, h, p.cov1, p.cov1_half, p.cov_samples, blockIdx.x, blockIdx.y);
}

__device__ void cov_finish_body(const double* __restrict__ samples, int R, double* __restrict__ avg,
                                double* __restrict__ cov_out, int c_out, psfm_fit_stats* stats) {
    __shared__ double red[16];
    __shared__ double s_centre;
    const int Rw = 2 * R + 1, n = Rw * Rw, tid = threadIdx.x;
    for (int d = tid; d < n; d += blockDim.x) {
        double s = 0.0;
        for (int j = 0; j < PSFM_COV_SAMPLES; j++) s += samples[(size_t)j * n + d] / 9.0;
        avg[d] = s;
    }
    __syncthreads();
    if (tid == 0) s_centre = avg[R * Rw + R];
    __syncthreads();
    const double centre = s_centre;
    double tot = 0.0;
    for (int d = tid; d < n; d += blockDim.x) {
        const double v = centre != 0.0 ? avg[d] / centre : 0.0;
        avg[d] = v;
        tot += fabs(v);
    }
    tot = psfm_block_sum(tot, red);
    const int Ow = 2 * c_out + 1;
    double kept = 0.0;
    for (int e = tid; e < Ow * Ow; e += blockDim.x) {
        const int dy = e / Ow - c_out, dx = e % Ow - c_out;
        double v = 0.0;
        if (dx >= -R && dx <= R && dy >= -R && dy <= R) v = avg[(dy + R) * Rw + (dx + R)];
        cov_out[e] = v;
        kept += fabs(v);
    }
    kept = psfm_block_sum(kept, red);
    if (tid == 0 && stats) stats->cov_discarded_frac = tot > 0.0 ? (tot - kept) / tot : 0.0;
}

__global__ __launch_bounds__(1024) void k_cov_finish(const double* __restrict__ samples, int R,
                                                    double* __restrict__ avg,
                                                    double* __restrict__ cov_out, int c_out,
                                                    psfm_fit_stats* stats) {
    cov_finish_body(samples, R, avg, cov_out, c_out, stats);
}

__global__ __launch_bounds__(1024) void k_cov_finish_b(const PairDesc* __restrict__ pairs, int h) {
    const PairDesc& p = pairs[blockIdx.x];
    cov_finish_body(p.cov_samples, 2 * h + p.cov1_half, p.cov_avg, p.cov, p.cov_half, p.stats);
}

// VEC: four neighbouring pixels per thread with 16-byte plane and 4-byte
// mask accesses (pitch and W multiples of 4, planes 16-byte aligned).
template <bool VEC>
__global__ __launch_bounds__(256) void k_subtract(
    const float* __restrict__ I2, const float* __restrict__ V2, const uint8_t* __restrict__ M2,
    const float* __restrict__ conv, const float* __restrict__ conv_var,
    const uint8_t* __restrict__ conv_mask, int W, int H, int64_t pitch,
    const double* __restrict__ d0p, float* __restrict__ diff, float* __restrict__ diff_var, uint8_t* __restrict__ diff_mask,
    double* __restrict__ partials) {
    __shared__ double red[16];
    const double d0 = *d0p;
    double s2 = 0.0, n2 = 0.0, sc = 0.0, nc = 0.0;
    auto pixel = [&](uint8_t m2, uint8_t cm, float cv, float v2, float i2, float c1, float& d, float& dv,
                     uint8_t& dm) {
        if (m2) {
            d = 0.0f;
            dv = 0.0f;
            dm = (uint8_t)(PSFM_MASK_BAD | cm);
        } else {
            d = (float)((double)i2 - (double)c1 - d0);
            dv = (float)((double)v2 + (double)cv);
            dm = cm;
            s2 += v2;
            n2 += 1.0;
        }
        if (!cm) {
            sc += cv;
            nc += 1.0;
        }
    };
    for (int y = blockIdx.x; y < H; y += gridDim.x) {
        if constexpr (VEC) {
            for (int x = 4 * threadIdx.x; x < W; x += 4 * 256) {
                const int64_t o = (int64_t)y * pitch + x;
                // all six loads issued before any use
                const uchar4 m2 = *reinterpret_cast<const uchar4*>(M2 + o);
                const uchar4 cm = *reinterpret_cast<const uchar4*>(conv_mask + o);
                const float4 cv = *reinterpret_cast<const float4*>(conv_var + o);
                const float4 v2 = *reinterpret_cast<const float4*>(V2 + o);
                const float4 i2 = *reinterpret_cast<const float4*>(I2 + o);
                const float4 c1 = *reinterpret_cast<const float4*>(conv + o);
                float4 d, dv;
                uchar4 dm;
                pixel(m2.x, cm.x, cv.x, v2.x, i2.x, c1.x, d.x, dv.x, dm.x);
                pixel(m2.y, cm.y, cv.y, v2.y, i2.y, c1.y, d.y, dv.y, dm.y);
                pixel(m2.z, cm.z, cv.z, v2.z, i2.z, c1.z, d.z, dv.z, dm.z);
                pixel(m2.w, cm.w, cv.w, v2.w, i2.w, c1.w, d.w, dv.w, dm.w);
                *reinterpret_cast<float4*>(diff + o) = d;
                *reinterpret_cast<float4*>(diff_var + o) = dv;
                *reinterpret_cast<uchar4*>(diff_mask + o) = dm;
            }
        } else {
            for (int x = threadIdx.x; x < W; x += 256) {
                const int64_t o = (int64_t)y * pitch + x;
                // all six loads unconditional, so that none waits on another
                const uint8_t m2 = M2[o], cm = conv_mask[o];
                const float cv = conv_var[o], v2 = V2[o], i2 = I2[o], c1 = conv[o];
                pixel(m2, cm, cv, v2, i2, c1, diff[o], diff_var[o], diff_mask[o]);
            }
        }
    }
    s2 = psfm_block_sum(s2, red);
    n2 = psfm_block_sum(n2, red);
    sc = psfm_block_sum(sc, red);
    nc = psfm_block_sum(nc, red);
    if (threadIdx.x == 0) {
        double* q = partials + 4 * blockIdx.x;
        q[0] = s2;
        q[1] = n2;
        q[2] = sc;
        q[3] = nc;
    }
}

// C_D = (v2 C_2 + vc C') / (v2 + vc), with v2 and vc the mean variances of
// the unmasked pixels of image 2 and of the convolved image, summed from the
// per-block partials [nparts][4] = (sum V2, n2, sum V', n').
__device__ void cov_diff_body(const double* __restrict__ partials, int nparts,
                              const double* __restrict__ cov2, int c2,
                              const double* __restrict__ covc, int cc, double* __restrict__ covd,
                              int cd) {
    __shared__ double red[16];
    double v[4] = {0.0, 0.0, 0.0, 0.0};
    for (int b = threadIdx.x; b < nparts; b += blockDim.x)
        for (int k = 0; k < 4; k++) v[k] += partials[4 * b + k];
    for (int k = 0; k < 4; k++) v[k] = psfm_block_sum(v[k], red);
    const double v2 = v[1] > 0.0 ? v[0] / v[1] : 0.0;
    const double vc = v[3] > 0.0 ? v[2] / v[3] : 0.0;
    const int Dw = 2 * cd + 1;
    for (int e = threadIdx.x; e < Dw * Dw; e += blockDim.x) {
        const int dy = e / Dw - cd, dx = e % Dw - cd;
        double a2 = 0.0, ac = 0.0;
        if (cov2) {
            if (abs(dx) <= c2 && abs(dy) <= c2) a2 = cov2[(dy + c2) * (2 * c2 + 1) + (dx + c2)];
        } else {
            a2 = (dx == 0 && dy == 0) ? 1.0 : 0.0;
        }
        if (covc && abs(dx) <= cc && abs(dy) <= cc) ac = covc[(dy + cc) * (2 * cc + 1) + (dx + cc)];
        covd[e] = (v2 + vc) > 0.0 ? (v2 * a2 + vc * ac) / (v2 + vc) : 0.0;
    }
}

__global__ __launch_bounds__(256) void k_subtract_cov(const double* __restrict__ partials, int nblk,
                                                      const double* __restrict__ cov2, int c2,
                                                      const double* __restrict__ covc, int cc,
                                                      double* __restrict__ covd, int cd) {
    cov_diff_body(partials, nblk, cov2, c2, covc, cc, covd, cd);
}

// psfm_match_pair's last step: the convolved image's pseudo-matrix C' from
// the samples, then C_D from the tiles' variance sums and C' (one launch).
__global__ __launch_bounds__(1024) void k_cov_finish_diff(const double* __restrict__ samples, int R,
                                                         double* __restrict__ avg,
                                                         double* __restrict__ cov_out, int c_out,
                                                         psfm_fit_stats* stats,
                                                         const double* __restrict__ partials,
                                                         int nparts, const double* __restrict__ cov2,
                                                         int c2, double* __restrict__ covd, int cd) {
    cov_finish_body(samples, R, avg, cov_out, c_out, stats);
    __syncthreads();       // C' (global, this workgroup's writes) before its use
    cov_diff_body(partials, nparts, cov2, c2, cov_out, c_out, covd, cd);
}

// One 64 x 64 tile t of a pair of the fused apply: the patch kernel is
// realised once; I' = K (x) I1 with its BAD/POOR mask, then D = I2 - I' - d0;
// V' = f K^2 (x) V1, then V_D = V2 + V' (I' and V' are stored only where the
// pair asks for them).  The tile's variance sums (sum V2, n2, sum V', n') go
// to p.sub_part[4 t].  All threads of the workgroup call it.
// PRE: the patch taps come from p.ptaps (realised for the whole batch by
// k_realise_b), so the tile kernel carries no realisation code (and its
// registers); otherwise the tile realises its patch kernel itself.
template <int H_, bool PRE>
__device__ __forceinline__ void match_tile(const PairDesc& p, const int t, const BasisArgs& B0, int P,
                                           double bad_frac, float* halo, float* tapsK, float* tapsV,
                                           uint32_t (*badw)[(TILE + 2 * H_ + 31) / 32 + 1],
                                           double* ring, double* red, int* s_rb, double* s_f) {
    const int tid = threadIdx.x;
    const int lx = tid & 63;
    const int r0 = (tid >> 6) * 16;
    const int W = p.W, H = p.H;
    const int64_t pitch = p.pitch;
    const PatchGeom g = patch_geom(W, H, P);
    const int tx = t % p.ntx, ty = t / p.ntx;
    const int px = tx / g.tpp, sx = tx % g.tpp;
    const int py = ty / g.tpp, sy = ty % g.tpp;
    const int X0 = px * P + sx * TILE, Y0 = py * P + sy * TILE;
    const int X1 = min(min(X0 + TILE, (px + 1) * P), W);
    const int Y1 = min(min(Y0 + TILE, (py + 1) * P), H);
    double s2 = 0.0, n2 = 0.0, sc = 0.0, nc = 0.0;
    if (X0 < X1 && Y0 < Y1) {
        // batch: the patch taps (realised by k_realise_b) are loaded into
        // registers first, so that their latency passes under the halo loads
        constexpr int T = (2 * H_ + 1) * (2 * H_ + 1);
        constexpr int NT = (2 * T + 1 + 255) / 256;
        float tk[NT];
        if constexpr (PRE) {
            const float* src = p.ptaps + (size_t)(py * g.npx + px) * psfm::patch_taps_floats(H_);
#pragma unroll
            for (int k = 0; k < NT; k++) tk[k] = src[min(tid + 256 * k, 2 * T)];
        } else {
            BasisArgs B = B0;
            B.ns = p.ns;
            B.S = p.S;
            patch_taps<H_>(B, p.coeffs, W, H, P, px, py, bad_frac, p.cov1, p.cov1_half, halo, tapsK,
                           tapsV, ring, red, s_rb, s_f);
        }
        const int anybad = load_halo<H_, true>(p.I1, p.M1, W, H, pitch, X0, Y0, halo, badw);
        if constexpr (PRE) {
#pragma unroll
            for (int k = 0; k < NT; k++) {
                const int e = tid + 256 * k;
                if (e < T) tapsK[e] = tk[k];
                else if (e < 2 * T) tapsV[e - T] = tk[k];
                else if (e == 2 * T) *s_rb = __float_as_int(tk[k]);
            }
            __syncthreads();
        }
        const int gx = X0 + lx;
        // the target image's mask, values and variance of the 16 outputs,
        // loaded together (clamped addresses outside the tile) and early: their
        // latency passes under the image convolution
        uint32_t m2bits = 0;
        float i2v[16];
#pragma unroll
        for (int j = 0; j < 16; j++) {
            const int gy = Y0 + r0 + j;
            const int64_t o = (gx < X1 && gy < Y1) ? (int64_t)gy * pitch + gx : 0;
            m2bits |= (p.M2[o] != 0 ? 1u : 0u) << j;
            i2v[j] = p.I2[o];
        }
        float acc[16];
        conv16<H_>(halo, tapsK, lx, r0, acc);
        uint32_t bad16 = 0, poor16 = 0;
        if (anybad) mask16<H_>(badw, *s_rb, lx, r0, &bad16, &poor16);
        const double d0 = p.coeffs[p.N - 1];
        if (gx < X1) {
#pragma unroll
            for (int j = 0; j < 16; j++) {
                const int gy = Y0 + r0 + j;
                if (gy < Y1) {
                    const int64_t o = (int64_t)gy * pitch + gx;
                    const uint8_t cm = ((bad16 >> j) & 1u) ? PSFM_MASK_CONV_BAD
                                       : ((poor16 >> j) & 1u) ? PSFM_MASK_CONV_POOR : 0;
                    if (p.conv) {
                        p.conv[o] = acc[j];
                        p.conv_mask[o] = cm;
                    }
                    if ((m2bits >> j) & 1u) {
                        p.diff[o] = 0.0f;
                        p.diff_mask[o] = (uint8_t)(PSFM_MASK_BAD | cm);
                    } else {
                        p.diff[o] = (float)((double)i2v[j] - (double)acc[j] - d0);
                        p.diff_mask[o] = cm;
                    }
                }
            }
        }
        __syncthreads();
        load_halo<H_, false>(p.V1, p.M1, W, H, pitch, X0, Y0, halo, badw);
        float v2v[16];                 // the target's variance, under the variance convolution
#pragma unroll
        for (int j = 0; j < 16; j++) {
            const int gy = Y0 + r0 + j;
            v2v[j] = p.V2[(gx < X1 && gy < Y1) ? (int64_t)gy * pitch + gx : 0];
        }
        conv16<H_>(halo, tapsV, lx, r0, acc);
        if (gx < X1) {
#pragma unroll
            for (int j = 0; j < 16; j++) {
                const int gy = Y0 + r0 + j;
                if (gy < Y1) {
                    const int64_t o = (int64_t)gy * pitch + gx;
                    const float cv = acc[j];
                    if (p.var) p.var[o] = cv;
                    if ((m2bits >> j) & 1u) {
                        p.diff_var[o] = 0.0f;
                    } else {
                        const float v2 = v2v[j];
                        p.diff_var[o] = (float)((double)v2 + (double)cv);
                        s2 += v2;
                        n2 += 1.0;
                    }
                    if (!((bad16 | poor16) >> j & 1u)) {
                        sc += cv;
                        nc += 1.0;
                    }
                }
            }
        }
    }
    double sums[4] = {s2, n2, sc, nc};
    psfm_block_sum4(sums, red);
    if (tid == 0) {
        double* q = p.sub_part + 4 * (size_t)t;
        q[0] = sums[0];
        q[1] = sums[1];
        q[2] = sums[2];
        q[3] = sums[3];
    }
}

// Patch kernels of every pair of a batch, one wave per patch (four per
// workgroup, which share the basis factors in LDS): the arithmetic of
// realise_kernel and kernel_stats for one workgroup (the same operations in
// the same order, their tap sums being wave-0 sums there), then the FP32
// taps K and f K^2 and the BAD radius to p.ptaps for the tile pass.
constexpr int RB_WAVES = 4;

// LDS of the per-wave patch realisation: the basis factors and term tables
// (shared), each wave's coefficients, taps and ring sums.
template <int H_>
struct RealiseWaveLds {
    double F[32 * (2 * H_ + 1)];
    int rf[64], cf[64], ro[64], rs[33];
    double gam[RB_WAVES][64];
    double Kd[RB_WAVES][(2 * H_ + 1) * (2 * H_ + 1)];
    double ring[RB_WAVES][H_ + 1];
};

// All threads: the factors and term tables into L (a barrier follows).
template <int H_>
__device__ void realise_wave_setup(const BasisArgs& B0, RealiseWaveLds<H_>& L) {
    constexpr int KW = 2 * H_ + 1;
    const int tid = threadIdx.x, nb = B0.nb;
    for (int e = tid; e < B0.nf * KW; e += 256) L.F[e] = B0.fac64[e];
    if (tid < nb) {
        L.rf[tid] = B0.rowf[tid];
        L.cf[tid] = B0.colf[tid];
        L.ro[tid] = B0.rorder[tid];
    }
    if (tid <= B0.nf) L.rs[tid] = B0.rstart[tid];
    __syncthreads();
}

// One wave realises patch ql of pair p into p.ptaps (see k_realise_b).
template <int H_>
__device__ void realise_patch_wave(const PairDesc& p, const int ql, const BasisArgs& B0, int P,
                                   double bad_frac, RealiseWaveLds<H_>& L) {
    constexpr int KW = 2 * H_ + 1;
    constexpr int T = KW * KW;
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6, nb = B0.nb;
    const double* F = L.F;
    const int *rf = L.rf, *cf = L.cf, *ro = L.ro, *rs = L.rs;
    double (*gam)[64] = L.gam;
    double (*Kd)[T] = L.Kd;
    double (*ring)[H_ + 1] = L.ring;
    const int W = p.W, H = p.H, ns = p.ns;
    const PatchGeom g = patch_geom(W, H, P);
    const int px = ql % g.npx, py = ql / g.npx;
    const int x0 = px * P, x1 = min(x0 + P, W), y0 = py * P, y1 = min(y0 + P, H);
    const double x = 0.5 * (x0 + x1 - 1), y = 0.5 * (y0 + y1 - 1);
    {
        const int i = lane < nb ? lane : 0;
        double cv[28];
#pragma unroll
        for (int k = 0; k < 28; k++) cv[k] = p.coeffs[i * ns + (k < ns ? k : 0)];
        const double zi = (double)B0.z[i], ps = B0.psi64[i];
        const double xt = W > 1 ? (2.0 * x - (W - 1)) / (double)(W - 1) : 0.0;
        const double yt = H > 1 ? (2.0 * y - (H - 1)) / (double)(H - 1) : 0.0;
        double al = 0.0;
#pragma unroll
        for (int d = 0; d <= 6; d++) {
            if (d <= p.S) {
#pragma unroll
                for (int l = d; l >= 0; l--) {
                    double v = 1.0;
#pragma unroll
                    for (int k = 0; k < l; k++) v *= xt;
#pragma unroll
                    for (int k = 0; k < d - l; k++) v *= yt;
                    al += cv[d * (d + 1) / 2 + (d - l)] * v;
                }
            }
        }
        double c0 = lane >= 1 && lane < nb ? zi * al : 0.0;
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) c0 += __shfl_xor(c0, o);
        if (lane < nb) gam[w][lane] = (lane == 0 ? al - c0 : al) * ps;
    }
    wave_sync_lds();
    double* K = Kd[w];
    const int nf = B0.nf;
    if (nf <= KW) {
        // realise_kernel's regrouped form, the same chains: the table C in
        // this wave's K, then the lane's taps t = lane + 64 k in registers
        constexpr int NT = (T + 63) / 64;
        for (int e = lane; e < nf * KW; e += 64) {
            const int r = e / KW, v = e - r * KW;
            double c = 0.0;
            for (int m = rs[r]; m < rs[r + 1]; m++) {
                const int i = ro[m];
                c = fma(gam[w][i], F[cf[i] * KW + v], c);
            }
            K[e] = c;
        }
        wave_sync_lds();
        double kv[NT];
#pragma unroll
        for (int k = 0; k < NT; k++) {
            const int t = min(lane + 64 * k, T - 1);
            const int v = t / KW, u = t - v * KW;
            kv[k] = 0.0;
            for (int r = 0; r < nf; r++) kv[k] = fma(F[r * KW + u], K[r * KW + v], kv[k]);
        }
        wave_sync_lds();
#pragma unroll
        for (int k = 0; k < NT; k++)
            if (lane + 64 * k < T) K[lane + 64 * k] = kv[k];
    } else {
        // the lane's NT taps t = lane + 64 k at once, the terms in the outer
        // loop (each term's coefficient and factor rows read once for all of
        // them); per tap the same sums in the same order as realise_kernel
        // (term j into k4[j % 4]), so the same values
        constexpr int NT = (T + 63) / 64;
        double k4[NT][4];
        int uo[NT], vo[NT];
#pragma unroll
        for (int k = 0; k < NT; k++) {
            const int t = min(lane + 64 * k, T - 1);
            vo[k] = t / KW;
            uo[k] = t - vo[k] * KW;
            k4[k][0] = k4[k][1] = k4[k][2] = k4[k][3] = 0.0;
        }
        for (int j0 = 0; j0 < nb; j0 += 4) {
#pragma unroll
            for (int r = 0; r < 4; r++) {
                const int j = j0 + r;
                if (j < nb) {
                    const double g = gam[w][j];
                    const double* Fr = F + rf[j] * KW;
                    const double* Fc = F + cf[j] * KW;
#pragma unroll
                    for (int k = 0; k < NT; k++) k4[k][r] += g * Fr[uo[k]] * Fc[vo[k]];
                }
            }
        }
#pragma unroll
        for (int k = 0; k < NT; k++)
            if (lane + 64 * k < T) K[lane + 64 * k] = (k4[k][0] + k4[k][1]) + (k4[k][2] + k4[k][3]);
    }
    wave_sync_lds();
    // kernel_stats' sums: lane partials over taps lane + 64 j, then the
    // workgroup sum's shuffle-down tree (its lane-0 value)
    double s2 = 0.0;
    for (int t = lane; t < T; t += 64) s2 += K[t] * K[t];
    for (int o = 32; o > 0; o >>= 1) s2 += __shfl_down(s2, o);
    const double sumk2 = __shfl(s2, 0);
    if (lane <= H_) {
        const int rr = lane;
        double sr = 0.0;
        for (int v = -rr; v <= rr; v++) {
            const int step = (v == -rr || v == rr || rr == 0) ? 1 : 2 * rr;
            for (int u = -rr; u <= rr; u += step) {
                const double k = K[(v + H_) * KW + (u + H_)];
                sr += k * k;
            }
        }
        ring[w][rr] = sr;
    }
    double f = 1.0;
    if (p.cov1) {
        const int c_in = p.cov1_half, Cw = 2 * c_in + 1;
        const double* cov_in = p.cov1;
        double r0 = 0.0;
        for (int t = lane; t < T; t += 64) {
            const int v = t / KW - H_, u = t % KW - H_;
            double qq = 0.0;
            for (int wy = -c_in; wy <= c_in; wy++)
                for (int wx = -c_in; wx <= c_in; wx++) {
                    const int u2 = u - wx, v2 = v - wy;
                    if (u2 < -H_ || u2 > H_ || v2 < -H_ || v2 > H_) continue;
                    qq += cov_in[(wy + c_in) * Cw + (wx + c_in)] * K[(v2 + H_) * KW + (u2 + H_)];
                }
            r0 += K[t] * qq;
        }
        for (int o = 32; o > 0; o >>= 1) r0 += __shfl_down(r0, o);
        const double raw0 = __shfl(r0, 0);
        f = sumk2 > 0.0 ? raw0 / sumk2 : 0.0;
    }
    wave_sync_lds();
    int rb = H_;
    {
        double outside = 0.0;
        for (int rr = 0; rr <= H_; rr++) outside += ring[w][rr];
        const double tot = outside;
        for (int rr = 0; rr <= H_; rr++) {
            outside -= ring[w][rr];
            if (outside < bad_frac * tot) {
                rb = rr;
                break;
            }
        }
    }
    float* dst = p.ptaps + (size_t)ql * psfm::patch_taps_floats(H_);
    for (int t = lane; t < T; t += 64) {
        const int uu = t / KW, vv = t - uu * KW;     // column-major
        const double k = K[vv * KW + uu];
        dst[t] = (float)k;
        dst[T + t] = (float)(f * k * k);
    }
    if (lane == 0) dst[2 * T] = __int_as_float(rb);
}

template <int H_>
__global__ __launch_bounds__(256) void k_realise_b(const PairDesc* __restrict__ pairs,
                                                   const int* __restrict__ patch_pair, int n_patches,
                                                   BasisArgs B0, int P, double bad_frac) {
    __shared__ RealiseWaveLds<H_> L;
    realise_wave_setup<H_>(B0, L);
    const int q = blockIdx.x * RB_WAVES + (threadIdx.x >> 6);
    if (q >= n_patches) return;                 // the whole wave; no barrier follows
    const PairDesc& p = pairs[patch_pair[q]];
    realise_patch_wave<H_>(p, q - p.patch_off, B0, P, bad_frac, L);
}

// The same for the n_patches patches of one pair (psfm_match_pair).
template <int H_>
__global__ __launch_bounds__(256) void k_realise_1(PairDesc p, int n_patches, BasisArgs B0, int P,
                                                   double bad_frac) {
    __shared__ RealiseWaveLds<H_> L;
    realise_wave_setup<H_>(B0, L);
    const int q = blockIdx.x * RB_WAVES + (threadIdx.x >> 6);
    if (q >= n_patches) return;
    realise_patch_wave<H_>(p, q, B0, P, bad_frac, L);
}

// Fused apply for every pair of a batch: the tiles of all pairs (flattened,
// pair after pair, visited by a grid-stride loop) go through match_tile; the
// workgroup that finishes a pair's last tile forms that pair's C_D and
// stamps its completion time.
template <int H_>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4))) void k_match_tiles_b(const PairDesc* __restrict__ pairs,
                                                       const int* __restrict__ tile_pair,
                                                       int n_tiles, BasisArgs B0, int P,
                                                       double bad_frac) {
    constexpr int KW = 2 * H_ + 1;
    constexpr int T = KW * KW;
    constexpr int HW = TILE + 2 * H_;
    constexpr int NWB = (HW + 31) / 32 + 1;
    static_assert(sizeof(float) * HW * HW >= sizeof(RealiseLds) + sizeof(double) * T,
                  "kernel scratch must fit in the halo buffer");
    __shared__ __align__(16) float halo[HW * HW];
    __shared__ __align__(16) float tapsK[T + 4];
    __shared__ __align__(16) float tapsV[T + 4];
    __shared__ uint32_t badw[HW][NWB];
    __shared__ double ring[H_ + 1];
    __shared__ double red[16];
    __shared__ int s_rb;
    __shared__ double s_f;
    __shared__ int s_last;
    const int tid = threadIdx.x;
    for (int it = blockIdx.x; it < n_tiles; it += gridDim.x) {
        // one workgroup per tile: workgroups go to the 8 XCDs in turn, so
        // XCD x takes the x-th contiguous eighth of the tile list, where
        // neighbouring tiles share their halo rows in that XCD's L2
        int item = it;
        if ((int)gridDim.x == n_tiles) {
            const int x = it & 7, k = it >> 3, q = n_tiles >> 3, r = n_tiles & 7;
            item = x * q + (x < r ? x : r) + k;
        }
        const PairDesc& p = pairs[tile_pair[item]];
        const int t = item - p.tile_off;
        match_tile<H_, true>(p, t, B0, P, bad_frac, halo, tapsK, tapsV, badw, ring, red, &s_rb, &s_f);
        if (tid == 0) {
            __threadfence();
            const unsigned prev = atomicAdd(p.tiles_done, 1u);
            s_last = prev + 1 == (unsigned)(p.ntx * p.nty);
        }
        __syncthreads();
        if (s_last) {
            __threadfence();
            cov_diff_body(p.sub_part, p.ntx * p.nty, p.cov2, p.cov2_half, p.cov, p.cov_half,
                          p.cov_diff, p.cov_diff_half);
            if (tid == 0 && p.t_done) {
                __threadfence();
                *p.t_done = wall_clock64();
            }
        }
        __syncthreads();
    }
}

// The fused apply of one pair (psfm_match_pair): one workgroup per tile, the
// pair's description by value, the patch taps from k_realise_1; C_D follows
// in k_cov_finish_diff.
template <int H_>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4))) void k_match_tile(PairDesc p, BasisArgs B0, int P,
                                                                                          double bad_frac) {
    constexpr int KW = 2 * H_ + 1;
    constexpr int T = KW * KW;
    constexpr int HW = TILE + 2 * H_;
    constexpr int NWB = (HW + 31) / 32 + 1;
    __shared__ __align__(16) float halo[HW * HW];
    __shared__ __align__(16) float tapsK[T + 4];
    __shared__ __align__(16) float tapsV[T + 4];
    __shared__ uint32_t badw[HW][NWB];
    __shared__ double ring[H_ + 1];
    __shared__ double red[16];
    __shared__ int s_rb;
    __shared__ double s_f;
    // one workgroup per tile, XCD by XCD: workgroup b runs on XCD b mod 8, so
    // XCD x takes the x-th contiguous eighth of the tiles, whose halos overlap
    const int n = gridDim.x, x = blockIdx.x & 7, k = blockIdx.x >> 3, q = n >> 3, r = n & 7;
    const int t = x * q + (x < r ? x : r) + k;
    match_tile<H_, true>(p, t, B0, P, bad_frac, halo, tapsK, tapsV, badw, ring, red, &s_rb, &s_f);
}

constexpr int SUB_BLOCKS = 1024;

}  // namespace

namespace psfm {

size_t conv_workspace(const psfm_context* ctx, int, int) {
    const int R = 2 * ctx->h + 32;   // room for cov_in_half up to 32
    const int E = 4 * ctx->h + 1;
    Carver c(nullptr);
    c.take<double>((size_t)PSFM_COV_SAMPLES * (2 * R + 1) * (2 * R + 1));
    c.take<double>((size_t)(2 * R + 1) * (2 * R + 1));
    c.take<double>((size_t)PSFM_COV_SAMPLES * E * E);
    return c.off;
}

size_t subtract_workspace(const psfm_context*, int, int) {
    Carver c(nullptr);
    c.take<double>(4 * SUB_BLOCKS);
    return c.off;
}

// psfm_match_pair: the pseudo-matrix scratch, the tiles' variance sums, then
// the patch taps (FP32 K, f K^2 and the BAD radius of every patch).
static size_t match_sub_bytes(const PatchGeom& g) {
    return sizeof(double) * 4 * (size_t)(g.npx * g.tpp) * (g.npy * g.tpp);
}

size_t match_workspace(const psfm_context* ctx, int W, int H) {
    const PatchGeom g = patch_geom(W, H, ctx->cfg.patch);
    return align_up(conv_workspace(ctx, W, H), 256) + align_up(match_sub_bytes(g), 256) +
           sizeof(float) * (size_t)g.npx * g.npy * patch_taps_floats(ctx->h);
}

int cov_sample_side(const psfm_context* ctx, int c_in) { return 2 * (2 * ctx->h + c_in) + 1; }

static BasisArgs basis_args_of(const psfm_context* ctx) {
    BasisArgs B;
    B.fac64 = ctx->fac64;
    B.psi64 = ctx->psi64;
    B.z = ctx->term_z;
    B.rowf = ctx->term_rowf;
    B.colf = ctx->term_colf;
    B.rorder = ctx->term_rorder;
    B.rstart = ctx->row_start;
    B.nb = ctx->nb;
    B.nf = ctx->nf;
    B.ns = ctx->ns;
    B.S = ctx->cfg.spatial_order;
    B.h = ctx->h;
    return B;
}

template <int H_>
int launch_match_tiles(const psfm_context* ctx, const PairDesc* pairs, const int* tile_pair,
                       int n_tiles, int grid, hipStream_t st) {
    hipLaunchKernelGGL(k_match_tiles_b<H_>, dim3(grid), dim3(256), 0, st, pairs, tile_pair, n_tiles,
                       basis_args_of(ctx), ctx->cfg.patch, ctx->cfg.bad_frac);
    PSFM_HIP_CHECK(hipGetLastError());
    return PSFM_OK;
}

template <int H_>
void launch_realise_b(const psfm_context* ctx, const PairDesc* pairs, const int* patch_pair,
                      int n_patches, hipStream_t st) {
    hipLaunchKernelGGL(k_realise_b<H_>, dim3((n_patches + RB_WAVES - 1) / RB_WAVES), dim3(256), 0, st,
                       pairs, patch_pair, n_patches, basis_args_of(ctx), ctx->cfg.patch, ctx->cfg.bad_frac);
}

int batch_apply(const psfm_context* ctx, const PairDesc* pairs, const int* tile_pair, int n_pairs,
                int n_tiles, const int* patch_pair, int n_patches, int max_cov_in, int conv_grid,
                int parts, hipStream_t st) {
    if (n_pairs == 0) return PSFM_OK;
    if ((parts & 1) && patch_pair && n_patches > 0) {
        switch (ctx->h) {
#define PSFM_RB_CASE(HH) \
    case HH: launch_realise_b<HH>(ctx, pairs, patch_pair, n_patches, st); break;
            PSFM_RB_CASE(1) PSFM_RB_CASE(2) PSFM_RB_CASE(3) PSFM_RB_CASE(4) PSFM_RB_CASE(5)
            PSFM_RB_CASE(6) PSFM_RB_CASE(7) PSFM_RB_CASE(8) PSFM_RB_CASE(9) PSFM_RB_CASE(10)
            PSFM_RB_CASE(11) PSFM_RB_CASE(12) PSFM_RB_CASE(13) PSFM_RB_CASE(14) PSFM_RB_CASE(15)
            PSFM_RB_CASE(16)
#undef PSFM_RB_CASE
            default: return PSFM_ERR_UNSUPPORTED;
        }
        PSFM_HIP_CHECK(hipGetLastError());
    }
    if (parts & 1) {
        const int E = 4 * ctx->h + 1;
        hipLaunchKernelGGL(k_cell_kernels_b, dim3(PSFM_COV_SAMPLES, n_pairs), dim3(256), 0, st, pairs,
                           basis_args_of(ctx));
        hipLaunchKernelGGL(k_cov_auto_b, dim3(PSFM_COV_SAMPLES, E, n_pairs), dim3(256), 0, st,
                           pairs, basis_args_of(ctx));
        if (max_cov_in >= 0) {      // some pair has a correlated input
            const int Rw = cov_sample_side(ctx, max_cov_in);
            hipLaunchKernelGGL(k_cov_mix_b, dim3(PSFM_COV_SAMPLES, (Rw * Rw + 255) / 256, n_pairs),
                               dim3(256), 0, st, pairs, ctx->h);
        }
        hipLaunchKernelGGL(k_cov_finish_b, dim3(n_pairs), dim3(1024), 0, st, pairs, ctx->h);
        PSFM_HIP_CHECK(hipGetLastError());
    }
    if (!(parts & 2) || n_tiles == 0) return PSFM_OK;
    const int grid = (conv_grid > 0 && conv_grid < n_tiles) ? conv_grid : n_tiles;
    switch (ctx->h) {
#define PSFM_MT_CASE(HH) \
    case HH: return launch_match_tiles<HH>(ctx, pairs, tile_pair, n_tiles, grid, st);
        PSFM_MT_CASE(1) PSFM_MT_CASE(2) PSFM_MT_CASE(3) PSFM_MT_CASE(4) PSFM_MT_CASE(5)
        PSFM_MT_CASE(6) PSFM_MT_CASE(7) PSFM_MT_CASE(8) PSFM_MT_CASE(9) PSFM_MT_CASE(10)
        PSFM_MT_CASE(11) PSFM_MT_CASE(12) PSFM_MT_CASE(13) PSFM_MT_CASE(14) PSFM_MT_CASE(15)
        PSFM_MT_CASE(16)
#undef PSFM_MT_CASE
        default: return PSFM_ERR_UNSUPPORTED;
    }
}

}  // namespace psfm

static BasisArgs basis_args(const psfm_context* ctx) { return psfm::basis_args_of(ctx); }


static int check_image_args(const psfm_context* ctx, int W, int H, int64_t pitch) {
    if (!ctx) return PSFM_ERR_INVALID_ARG;
    if (W < 1 || H < 1 || pitch < W) return PSFM_ERR_SHAPE;
    return PSFM_OK;
}

extern "C" int psfm_convolve_image(const psfm_context* ctx, const double* coeffs, const float* I,
                                   const uint8_t* M, int W, int H, int64_t pitch, float* out,
                                   uint8_t* out_mask, void* ws, size_t ws_bytes, void* stream) {
    int rc = check_image_args(ctx, W, H, pitch);
    if (rc) return rc;
    if (!coeffs || !I || !M || !out || !out_mask) return PSFM_ERR_INVALID_ARG;
    (void)ws;
    (void)ws_bytes;
    hipStream_t st = (hipStream_t)stream;
    const psfm_config& cf = ctx->cfg;
    return dispatch_conv<0>(I, M, W, H, pitch, cf.patch, coeffs, basis_args(ctx), cf.bad_frac, nullptr,
                            0, out, out_mask, st);
}

// The covariance pseudo-matrix part of the variance propagation: samples at
// the centres of the 3 x 3 partition, their mean, normalised and cropped.
// With covd given, C_D follows in the same launch as C' (psfm_match_pair):
// from the tiles' variance sums parts[nparts][4] and cov2.
static int cov_pseudo(const psfm_context* ctx, const double* coeffs, int W, int H,
                      const double* cov_in, int cov_in_half, double* cov_out, int cov_out_half,
                      psfm_fit_stats* stats, void* ws, hipStream_t st,
                      const double* parts = nullptr, int nparts = 0, const double* cov2 = nullptr,
                      int c2 = 0, double* covd = nullptr, int cd = 0) {
    psfm::Carver c(ws);
    const int Rmax = 2 * ctx->h + 32;
    double* samples = c.take<double>((size_t)PSFM_COV_SAMPLES * (2 * Rmax + 1) * (2 * Rmax + 1));
    double* avg = c.take<double>((size_t)(2 * Rmax + 1) * (2 * Rmax + 1));
    const int E = 4 * ctx->h + 1;
    double* autoc = c.take<double>((size_t)PSFM_COV_SAMPLES * E * E);
    const int R = 2 * ctx->h + cov_in_half, Rw = 2 * R + 1;
    // uncorrelated input: the samples are the autocorrelation itself
    hipLaunchKernelGGL(k_cov_auto, dim3(PSFM_COV_SAMPLES, E), dim3(256), 0, st, coeffs,
                       basis_args(ctx), W, H, cov_in ? autoc : samples);
    if (cov_in)
        hipLaunchKernelGGL(k_cov_mix, dim3(PSFM_COV_SAMPLES, (Rw * Rw + 255) / 256), dim3(256), 0, st,
                           autoc, ctx->h, cov_in, cov_in_half, samples);
    if (covd)
        hipLaunchKernelGGL(k_cov_finish_diff, dim3(1), dim3(1024), 0, st, samples, R, avg, cov_out,
                           cov_out_half, stats, parts, nparts, cov2, c2, covd, cd);
    else
        hipLaunchKernelGGL(k_cov_finish, dim3(1), dim3(1024), 0, st, samples, R, avg, cov_out,
                           cov_out_half, stats);
    PSFM_HIP_CHECK(hipGetLastError());
    return PSFM_OK;
}

extern "C" int psfm_propagate_variance(const psfm_context* ctx, const double* coeffs,
                                       const float* V, const uint8_t* M, int W, int H,
                                       int64_t pitch, const double* cov_in, int cov_in_half,
                                       float* var_out, double* cov_out, int cov_out_half,
                                       psfm_fit_stats* stats, void* ws, size_t ws_bytes,
                                       void* stream) {
    int rc = check_image_args(ctx, W, H, pitch);
    if (rc) return rc;
    if (!coeffs || !V || !M || !var_out || !cov_out || cov_out_half < 0 || cov_in_half < 0)
        return PSFM_ERR_INVALID_ARG;
    if (cov_in_half > 32 || cov_out_half > 2 * ctx->h + 64) return PSFM_ERR_UNSUPPORTED;
    if (!cov_in) cov_in_half = 0;
    if (!ws || ws_bytes < psfm::conv_workspace(ctx, W, H)) return PSFM_ERR_WORKSPACE;
    hipStream_t st = (hipStream_t)stream;
    const psfm_config& cf = ctx->cfg;
    rc = dispatch_conv<1>(V, M, W, H, pitch, cf.patch, coeffs, basis_args(ctx), cf.bad_frac, cov_in,
                          cov_in_half, var_out, nullptr, st);
    if (rc) return rc;
    return cov_pseudo(ctx, coeffs, W, H, cov_in, cov_in_half, cov_out, cov_out_half, stats, ws, st);
}

extern "C" int psfm_convolve_pair(const psfm_context* ctx, const double* coeffs, const float* I,
                                  const float* V, const uint8_t* M, int W, int H, int64_t pitch,
                                  const double* cov_in, int cov_in_half, float* out,
                                  uint8_t* out_mask, float* var_out, double* cov_out,
                                  int cov_out_half, psfm_fit_stats* stats, void* ws,
                                  size_t ws_bytes, void* stream) {
    int rc = check_image_args(ctx, W, H, pitch);
    if (rc) return rc;
    if (!coeffs || !I || !V || !M || !out || !out_mask || !var_out || !cov_out ||
        cov_out_half < 0 || cov_in_half < 0)
        return PSFM_ERR_INVALID_ARG;
    if (cov_in_half > 32 || cov_out_half > 2 * ctx->h + 64) return PSFM_ERR_UNSUPPORTED;
    if (!cov_in) cov_in_half = 0;
    if (!ws || ws_bytes < psfm::conv_workspace(ctx, W, H)) return PSFM_ERR_WORKSPACE;
    hipStream_t st = (hipStream_t)stream;
    const psfm_config& cf = ctx->cfg;
    rc = dispatch_conv_pair(I, V, M, W, H, pitch, cf.patch, coeffs, basis_args(ctx), cf.bad_frac,
                            cov_in, cov_in_half, out, out_mask, var_out, st);
    if (rc) return rc;
    return cov_pseudo(ctx, coeffs, W, H, cov_in, cov_in_half, cov_out, cov_out_half, stats, ws, st);
}

extern "C" int psfm_subtract(const psfm_context* ctx, const double* coeffs, const float* I2,
                             const float* V2, const uint8_t* M2, const float* conv,
                             const float* conv_var, const uint8_t* conv_mask, int W, int H,
                             int64_t pitch, const double* cov2, int cov2_half,
                             const double* cov_conv, int cov_conv_half, float* diff,
                             float* diff_var, uint8_t* diff_mask, double* cov_diff,
                             int cov_diff_half, void* ws, size_t ws_bytes, void* stream) {
    int rc = check_image_args(ctx, W, H, pitch);
    if (rc) return rc;
    if (!coeffs || !I2 || !V2 || !M2 || !conv || !conv_var || !conv_mask || !diff || !diff_var ||
        !diff_mask || !cov_diff || cov2_half < 0 || cov_conv_half < 0 || cov_diff_half < 0)
        return PSFM_ERR_INVALID_ARG;
    if (!ws || ws_bytes < psfm::subtract_workspace(ctx, W, H)) return PSFM_ERR_WORKSPACE;
    hipStream_t st = (hipStream_t)stream;
    psfm::Carver c(ws);
    double* partials = c.take<double>(4 * SUB_BLOCKS);
    const int nblk = std::min(H, SUB_BLOCKS);
    // the background coefficient is the last unknown, read on the device
    const auto al16 = [](const void* q) { return ((uintptr_t)q & 15) == 0; };
    const bool vec = pitch % 4 == 0 && W % 4 == 0 && al16(I2) && al16(V2) && al16(conv) &&
                     al16(conv_var) && al16(diff) && al16(diff_var) && al16(M2) && al16(conv_mask) &&
                     al16(diff_mask);
    if (vec)
        hipLaunchKernelGGL(k_subtract<true>, dim3(nblk), dim3(256), 0, st, I2, V2, M2, conv, conv_var, conv_mask,
                           W, H, pitch, coeffs + (ctx->N - 1), diff, diff_var, diff_mask, partials);
    else
        hipLaunchKernelGGL(k_subtract<false>, dim3(nblk), dim3(256), 0, st, I2, V2, M2, conv, conv_var, conv_mask,
                           W, H, pitch, coeffs + (ctx->N - 1), diff, diff_var, diff_mask, partials);
    PSFM_HIP_CHECK(hipGetLastError());
    hipLaunchKernelGGL(k_subtract_cov, dim3(1), dim3(256), 0, st, partials, nblk, cov2, cov2_half,
                       cov_conv, cov_conv_half, cov_diff, cov_diff_half);
    PSFM_HIP_CHECK(hipGetLastError());
    return PSFM_OK;
}

template <int H_>
static void launch_match_tile(const PairDesc& p, const BasisArgs& B, int P, double bad_frac, int n_tiles,
                              int n_patches, hipStream_t st) {
    hipLaunchKernelGGL(k_realise_1<H_>, dim3((n_patches + RB_WAVES - 1) / RB_WAVES), dim3(256), 0, st, p,
                       n_patches, B, P, bad_frac);
    hipLaunchKernelGGL(k_match_tile<H_>, dim3(n_tiles), dim3(256), 0, st, p, B, P, bad_frac);
}

// psfm_match_pair with its scratch at `ws` (psfm_match_pair: the caller's
// workspace; psfm_match_pair_static: the library's static device array).
int psfm::match_pair_ws(const psfm_context* ctx, const double* coeffs, const float* I1,
                        const float* V1, const uint8_t* M1, const float* I2, const float* V2,
                        const uint8_t* M2, int W, int H, int64_t pitch, const double* cov1,
                        int cov1_half, const double* cov2, int cov2_half, float* conv,
                        uint8_t* conv_mask, float* conv_var, double* cov_conv, int cov_conv_half,
                        float* diff, float* diff_var, uint8_t* diff_mask, double* cov_diff,
                        int cov_diff_half, psfm_fit_stats* stats, void* ws, size_t ws_bytes,
                        void* stream) {
    int rc = check_image_args(ctx, W, H, pitch);
    if (rc) return rc;
    if (!coeffs || !I1 || !V1 || !M1 || !I2 || !V2 || !M2 || !cov_conv || !diff || !diff_var ||
        !diff_mask || !cov_diff || (conv == nullptr) != (conv_mask == nullptr) || cov1_half < 0 ||
        cov2_half < 0 || cov_conv_half < 0 || cov_diff_half < 0)
        return PSFM_ERR_INVALID_ARG;
    if (cov1_half > 32 || cov_conv_half > 2 * ctx->h + 64) return PSFM_ERR_UNSUPPORTED;
    if (!cov1) cov1_half = 0;
    if (!ws || ws_bytes < psfm::match_workspace(ctx, W, H)) return PSFM_ERR_WORKSPACE;
    hipStream_t st = (hipStream_t)stream;
    const psfm_config& cf = ctx->cfg;
    const PatchGeom g = patch_geom(W, H, cf.patch);
    PairDesc p{};
    p.I1 = I1;
    p.V1 = V1;
    p.M1 = M1;
    p.I2 = I2;
    p.V2 = V2;
    p.M2 = M2;
    p.W = W;
    p.H = H;
    p.pitch = pitch;
    p.N = ctx->N;
    p.ns = ctx->ns;
    p.S = cf.spatial_order;
    p.coeffs = const_cast<double*>(coeffs);
    p.cov1 = cov1;
    p.cov1_half = cov1_half;
    p.conv = conv;
    p.conv_mask = conv_mask;
    p.var = conv_var;
    p.diff = diff;
    p.diff_var = diff_var;
    p.diff_mask = diff_mask;
    p.ntx = g.npx * g.tpp;
    p.nty = g.npy * g.tpp;
    const size_t sub_off = psfm::align_up(psfm::conv_workspace(ctx, W, H), 256);
    p.sub_part = reinterpret_cast<double*>(static_cast<char*>(ws) + sub_off);
    p.ptaps = reinterpret_cast<float*>(static_cast<char*>(ws) + sub_off +
                                       psfm::align_up(psfm::match_sub_bytes(g), 256));
    const int n_tiles = p.ntx * p.nty;
    const int n_patch = g.npx * g.npy;
    const BasisArgs B = basis_args(ctx);
    switch (ctx->h) {
#define PSFM_M1_CASE(HH) \
    case HH: launch_match_tile<HH>(p, B, cf.patch, cf.bad_frac, n_tiles, n_patch, st); break;
        PSFM_M1_CASE(1) PSFM_M1_CASE(2) PSFM_M1_CASE(3) PSFM_M1_CASE(4) PSFM_M1_CASE(5)
        PSFM_M1_CASE(6) PSFM_M1_CASE(7) PSFM_M1_CASE(8) PSFM_M1_CASE(9) PSFM_M1_CASE(10)
        PSFM_M1_CASE(11) PSFM_M1_CASE(12) PSFM_M1_CASE(13) PSFM_M1_CASE(14) PSFM_M1_CASE(15)
        PSFM_M1_CASE(16)
#undef PSFM_M1_CASE
        default: return PSFM_ERR_UNSUPPORTED;
    }
    PSFM_HIP_CHECK(hipGetLastError());
    return cov_pseudo(ctx, coeffs, W, H, cov1, cov1_half, cov_conv, cov_conv_half, stats, ws, st,
                      p.sub_part, n_tiles, cov2, cov2_half, cov_diff, cov_diff_half);
}

extern "C" int psfm_match_pair(const psfm_context* ctx, const double* coeffs, const float* I1,
                               const float* V1, const uint8_t* M1, const float* I2, const float* V2,
                               const uint8_t* M2, int W, int H, int64_t pitch, const double* cov1,
                               int cov1_half, const double* cov2, int cov2_half, float* conv,
                               uint8_t* conv_mask, float* conv_var, double* cov_conv,
                               int cov_conv_half, float* diff, float* diff_var, uint8_t* diff_mask,
                               double* cov_diff, int cov_diff_half, psfm_fit_stats* stats, void* ws,
                               size_t ws_bytes, void* stream) {
    return psfm::match_pair_ws(ctx, coeffs, I1, V1, M1, I2, V2, M2, W, H, pitch, cov1, cov1_half,
                               cov2, cov2_half, conv, conv_mask, conv_var, cov_conv, cov_conv_half,
                               diff, diff_var, diff_mask, cov_diff, cov_diff_half, stats, ws,
                               ws_bytes, stream);
}

// ---------------------------------------------------------------- the paper's
// normalisation and quality mode (Sections 3.2, 3.3, 3.6, 3.7)

namespace {

constexpr int NW_MAX = 2 * PSFM_RMAX + 1 + 2 * PSFM_HMAX;   // window side, stamp + kernel halo
constexpr int NQ_T = 256;

// Loads the (2r+1+2h)^2 window of I1 around stamp centre (xc, yc) into LDS.
__device__ void load_stamp_window(const float* __restrict__ I1, int64_t pitch, int xc, int yc, int r,
                                  int h, float* win) {
    const int R = r + h, WW = 2 * R + 1;
    for (int e = threadIdx.x; e < WW * WW; e += blockDim.x) {
        const int wy = e / WW, wx = e - wy * WW;
        win[e] = I1[(int64_t)(yc - R + wy) * pitch + (xc - R + wx)];
    }
}

__device__ bool stamp_inside(int xc, int yc, int R, int W, int H) {
    return xc - R >= 0 && yc - R >= 0 && xc + R < W && yc + R < H;
}

// Unweighted stamp sums for the separate normalisation: npix, sum A0,
// sum I2, sum A0^2, sum A0 I2 with A0 = k_0 (x) I1 (FP64), one workgroup per
// stamp; stamps flagged with anything but PSFM_STAMP_RESERVE get zeros.
__global__ __launch_bounds__(NQ_T) void k_fit_norm(const double* __restrict__ k0,
                                                   const float* __restrict__ I1,
                                                   const float* __restrict__ I2, int W, int H,
                                                   int64_t pitch, const int32_t* __restrict__ xy,
                                                   const int32_t* __restrict__ flags, int r, int h,
                                                   double* __restrict__ norm) {
    __shared__ float win[NW_MAX * NW_MAX];
    __shared__ double taps[(2 * PSFM_HMAX + 1) * (2 * PSFM_HMAX + 1)];
    __shared__ double red[16];
    const int s = blockIdx.x, tid = threadIdx.x;
    const int xc = xy[2 * s], yc = xy[2 * s + 1];
    const int KW = 2 * h + 1, NPX = 2 * r + 1, WW = NPX + 2 * h;
    double* out = norm + 5 * (size_t)s;
    if ((flags[s] & ~PSFM_STAMP_RESERVE) || !stamp_inside(xc, yc, r + h, W, H)) {
        if (tid < 5) out[tid] = 0.0;
        return;
    }
    for (int t = tid; t < KW * KW; t += NQ_T) taps[t] = k0[t];
    load_stamp_window(I1, pitch, xc, yc, r, h, win);
    __syncthreads();
    double s1 = 0.0, s2 = 0.0, s3 = 0.0, s4 = 0.0, cnt = 0.0;
    for (int p = tid; p < NPX * NPX; p += NQ_T) {
        const int y = p / NPX, x = p - y * NPX;
        double a0 = 0.0;
        for (int v = -h; v <= h; v++) {
            const float* row = win + (size_t)(y + h - v) * WW + (x + h);
            const double* tr = taps + (v + h) * KW + h;
            for (int u = -h; u <= h; u++) a0 += tr[u] * (double)row[-u];
        }
        const double d = (double)I2[(int64_t)(yc - r + y) * pitch + (xc - r + x)];
        s1 += a0;
        s2 += d;
        s3 += a0 * a0;
        s4 += a0 * d;
        cnt += 1.0;
    }
    cnt = psfm_block_sum(cnt, red);
    s1 = psfm_block_sum(s1, red);
    s2 = psfm_block_sum(s2, red);
    s3 = psfm_block_sum(s3, red);
    s4 = psfm_block_sum(s4, red);
    if (tid == 0) {
        out[0] = cnt;
        out[1] = s1;
        out[2] = s2;
        out[3] = s3;
        out[4] = s4;
    }
}

// Softened deviation of each used stamp: the kernel realised at the stamp
// centre (FP64), the model m = K (x) I1 + d0 per stamp pixel, and
// dev_s = (1/npix) sum (I2 - m)^2 / (V2 + soft |m|).  One workgroup per stamp.
__global__ __launch_bounds__(NQ_T) void k_stamp_dev(BasisArgs B, const double* __restrict__ a,
                                                    const float* __restrict__ I1,
                                                    const float* __restrict__ I2,
                                                    const float* __restrict__ V2, int W, int H,
                                                    int64_t pitch, const int32_t* __restrict__ xy,
                                                    const int32_t* __restrict__ flags, int r,
                                                    double soft, double* __restrict__ dev) {
    __shared__ RealiseLds sh;
    __shared__ double Kd[(2 * PSFM_HMAX + 1) * (2 * PSFM_HMAX + 1)];
    __shared__ float win[NW_MAX * NW_MAX];
    __shared__ double red[16];
    const int s = blockIdx.x, tid = threadIdx.x, h = B.h;
    const int xc = xy[2 * s], yc = xy[2 * s + 1];
    const int KW = 2 * h + 1, NPX = 2 * r + 1, WW = NPX + 2 * h;
    if (flags[s] || !stamp_inside(xc, yc, r + h, W, H)) {
        if (tid == 0) dev[s] = 0.0;
        return;
    }
    realise_kernel(B, a, xc, yc, W, H, sh, Kd);
    load_stamp_window(I1, pitch, xc, yc, r, h, win);
    __syncthreads();
    const double d0 = a[B.nb * B.ns];
    double acc = 0.0;
    for (int p = tid; p < NPX * NPX; p += NQ_T) {
        const int y = p / NPX, x = p - y * NPX;
        double m = d0;
        for (int v = -h; v <= h; v++) {
            const float* row = win + (size_t)(y + h - v) * WW + (x + h);
            const double* kr = Kd + (v + h) * KW + h;
            for (int u = -h; u <= h; u++) m += kr[u] * (double)row[-u];
        }
        const int64_t o = (int64_t)(yc - r + y) * pitch + (xc - r + x);
        const double res = (double)I2[o] - m;
        acc += res * res / ((double)V2[o] + soft * fabs(m));
    }
    acc = psfm_block_sum(acc, red);
    if (tid == 0) dev[s] = acc / (double)(NPX * NPX);
}

// Aggregates: normalised mean and r.m.s. deviation over the used stamps; the
// kernel at the image centre (sum, moments, maximum deconvolution fraction
// over circular radii); the cut bits.  One workgroup.
__global__ __launch_bounds__(NQ_T) void k_quality_finish(BasisArgs B, const double* __restrict__ a,
                                                         int W, int H, int n,
                                                         const int32_t* __restrict__ flags,
                                                         const double* __restrict__ dev,
                                                         psfm_quality* __restrict__ q) {
    __shared__ RealiseLds sh;
    __shared__ double Kd[(2 * PSFM_HMAX + 1) * (2 * PSFM_HMAX + 1)];
    __shared__ double red[16];
    __shared__ double enc[64];
    const int tid = threadIdx.x, h = B.h, KW = 2 * h + 1, T = KW * KW;
    double sm = 0.0, cnt = 0.0;
    for (int s = tid; s < n; s += NQ_T)
        if (!flags[s]) {
            sm += dev[s];
            cnt += 1.0;
        }
    sm = psfm_block_sum(sm, red);
    cnt = psfm_block_sum(cnt, red);
    const double mean = cnt > 0.0 ? sm / cnt : 0.0;
    double sv = 0.0;
    for (int s = tid; s < n; s += NQ_T)
        if (!flags[s]) sv += (dev[s] - mean) * (dev[s] - mean);
    sv = psfm_block_sum(sv, red);
    realise_kernel(B, a, 0.5 * (W - 1), 0.5 * (H - 1), W, H, sh, Kd);
    double s0 = 0.0, su = 0.0, sv1 = 0.0;
    for (int t = tid; t < T; t += NQ_T) {
        const int v = t / KW - h, u = t % KW - h;
        s0 += Kd[t];
        su += u * Kd[t];
        sv1 += v * Kd[t];
    }
    s0 = psfm_block_sum(s0, red);
    su = psfm_block_sum(su, red);
    sv1 = psfm_block_sum(sv1, red);
    const double mx = su / s0, my = sv1 / s0;
    double sxx = 0.0, syy = 0.0;
    for (int t = tid; t < T; t += NQ_T) {
        const int v = t / KW - h, u = t % KW - h;
        sxx += (u - mx) * (u - mx) * Kd[t];
        syy += (v - my) * (v - my) * Kd[t];
    }
    sxx = psfm_block_sum(sxx, red);
    syy = psfm_block_sum(syy, red);
    const int rmax = (int)ceil(h * sqrt(2.0));
    if (tid <= rmax) {                 // enclosed sum within radius tid
        double e = 0.0;
        for (int t = 0; t < T; t++) {
            const int v = t / KW - h, u = t % KW - h;
            if (u * u + v * v <= tid * tid) e += Kd[t];
        }
        enc[tid] = e / s0;
    }
    __syncthreads();
    if (tid == 0) {
        double best = enc[0];
        for (int k = 1; k <= rmax; k++) best = fmax(best, enc[k]);
        psfm_quality r;
        r.n_used = (int)cnt;
        r.dev_mean = cnt > 0.0 ? mean - 1.0 : 0.0;
        r.dev_rms = cnt > 0.0 ? sqrt(sv / cnt) : 0.0;
        r.kernel_sum = s0;
        r.mom_x = mx;
        r.mom_y = my;
        r.mom_xx = sxx / s0;
        r.mom_yy = syy / s0;
        r.deconv_max = best;
        int f = 0;
        if (r.n_used < 3) f |= PSFM_CUT_FEW_STAMPS;
        if (r.dev_mean > 0.5) f |= PSFM_CUT_MEAN_DEV;
        if (r.dev_rms > 0.3) f |= PSFM_CUT_RMS_DEV;
        if (fabs(r.mom_x) > 0.5 || fabs(r.mom_y) > 0.5) f |= PSFM_CUT_MOMENT1;
        if (r.mom_xx < 0.0 || r.mom_yy < 0.0) f |= PSFM_CUT_MOMENT2;
        if (r.deconv_max > 1.03) f |= PSFM_CUT_DECONV;
        r.cut_flags = f;
        *q = r;
    }
}

// The two-kernel difference image (Section 2): one workgroup per 64 x 64
// tile of a patch.  K1 (the b-terms) and K2 = delta - sum c_i k_i (the
// c-terms, realised with term 0 left out) are realised in FP64 at the patch
// centre with their BAD radii; FP32 taps of K1, K1^2, K2, K2^2.  The halos of
// I1, I2 (with their mask bits), V1 and V2 go through the tile buffer in
// turn; D = K2 (x) I2 - K1 (x) I1 - d0 and V_D = K1^2 (x) V1 + K2^2 (x) V2
// (uncorrelated inputs), the mask BAD within either kernel's BAD radius of
// its image's masked or outside pixels, else POOR within h of either.
template <int H_>
__global__ __launch_bounds__(256) void k_dual_tile(
    const float* __restrict__ I1, const float* __restrict__ V1, const uint8_t* __restrict__ M1,
    const float* __restrict__ I2, const float* __restrict__ V2, const uint8_t* __restrict__ M2, int W,
    int H, int64_t pitch, int P, const double* __restrict__ a, BasisArgs B, int c_off, int N2,
    double bad_frac, float* __restrict__ D, float* __restrict__ VD, uint8_t* __restrict__ MD) {
    constexpr int KW = 2 * H_ + 1;
    constexpr int T = KW * KW;
    constexpr int HW = TILE + 2 * H_;
    constexpr int NWB = (HW + 31) / 32 + 1;
    static_assert(sizeof(float) * HW * HW >= sizeof(RealiseLds) + sizeof(double) * T,
                  "kernel scratch must fit in the halo buffer");
    __shared__ __align__(16) float halo[HW * HW];
    __shared__ __align__(16) float tK1[T + 4];
    __shared__ __align__(16) float tV1[T + 4];
    __shared__ __align__(16) float tK2[T + 4];
    __shared__ __align__(16) float tV2[T + 4];
    __shared__ uint32_t badw[HW][NWB];
    __shared__ double ring[H_ + 1];
    __shared__ double red[16];
    __shared__ int s_rb1, s_rb2;
    __shared__ double s_f;
    const int tid = threadIdx.x;
    const PatchGeom g = patch_geom(W, H, P);
    const int px = blockIdx.x / g.tpp, sx = blockIdx.x % g.tpp;
    const int py = blockIdx.y / g.tpp, sy = blockIdx.y % g.tpp;
    const int X0 = px * P + sx * TILE, Y0 = py * P + sy * TILE;
    const int X1 = min(min(X0 + TILE, (px + 1) * P), W);
    const int Y1 = min(min(Y0 + TILE, (py + 1) * P), H);
    if (X0 >= X1 || Y0 >= Y1) return;
    {
        RealiseLds& sh = *reinterpret_cast<RealiseLds*>(halo);
        double* Kd = reinterpret_cast<double*>(reinterpret_cast<char*>(halo) + sizeof(RealiseLds));
        const int x0 = px * P, x1 = min(x0 + P, W), y0 = py * P, y1 = min(y0 + P, H);
        const double xc = 0.5 * (x0 + x1 - 1), yc = 0.5 * (y0 + y1 - 1);
        realise_kernel(B, a, xc, yc, W, H, sh, Kd);
        kernel_stats(Kd, H_, bad_frac, nullptr, 0, ring, red, &s_rb1, &s_f);
        for (int t = tid; t < T; t += 256) {
            const int uu = t / KW, vv = t - uu * KW;     // column-major
            const double k = Kd[vv * KW + uu];
            tK1[t] = (float)k;
            tV1[t] = (float)(k * k);
        }
        __syncthreads();
        realise_kernel(B, a + c_off, xc, yc, W, H, sh, Kd, true);
        for (int t = tid; t < T; t += 256) Kd[t] = (t == H_ * KW + H_ ? 1.0 : 0.0) - Kd[t];
        __syncthreads();
        kernel_stats(Kd, H_, bad_frac, nullptr, 0, ring, red, &s_rb2, &s_f);
        for (int t = tid; t < T; t += 256) {
            const int uu = t / KW, vv = t - uu * KW;
            const double k = Kd[vv * KW + uu];
            tK2[t] = (float)k;
            tV2[t] = (float)(k * k);
        }
        __syncthreads();
    }
    const int lx = tid & 63;
    const int r0 = (tid >> 6) * 16;
    float acc1[16], acc2[16], accv[16];
    uint32_t bad = 0, poor = 0;
    {
        const int anybad = load_halo<H_, true>(I1, M1, W, H, pitch, X0, Y0, halo, badw);
        conv16<H_>(halo, tK1, lx, r0, acc1);
        if (anybad) mask16<H_>(badw, s_rb1, lx, r0, &bad, &poor);
    }
    __syncthreads();
    {
        const int anybad = load_halo<H_, true>(I2, M2, W, H, pitch, X0, Y0, halo, badw);
        conv16<H_>(halo, tK2, lx, r0, acc2);
        if (anybad) {
            uint32_t b2 = 0, p2 = 0;
            mask16<H_>(badw, s_rb2, lx, r0, &b2, &p2);
            bad |= b2;
            poor |= p2;
        }
    }
    __syncthreads();
    load_halo<H_, false>(V1, M1, W, H, pitch, X0, Y0, halo, badw);
    conv16<H_>(halo, tV1, lx, r0, accv);
    __syncthreads();
    float accv2[16];
    load_halo<H_, false>(V2, M2, W, H, pitch, X0, Y0, halo, badw);
    conv16<H_>(halo, tV2, lx, r0, accv2);
    const double d0 = a[N2 - 1];
    const int gx = X0 + lx;
    if (gx < X1) {
#pragma unroll
        for (int j = 0; j < 16; j++) {
            const int gy = Y0 + r0 + j;
            if (gy < Y1) {
                const int64_t o = (int64_t)gy * pitch + gx;
                D[o] = (float)((double)acc2[j] - (double)acc1[j] - d0);
                VD[o] = accv[j] + accv2[j];
                MD[o] = ((bad >> j) & 1u) ? PSFM_MASK_CONV_BAD : ((poor >> j) & 1u) ? PSFM_MASK_CONV_POOR : 0;
            }
        }
    }
}

template <int H_>
int launch_dual(const float* I1, const float* V1, const uint8_t* M1, const float* I2, const float* V2,
                const uint8_t* M2, int W, int H, int64_t pitch, int P, const double* a, const BasisArgs& B,
                int c_off, int N2, double bad_frac, float* D, float* VD, uint8_t* MD, hipStream_t st) {
    const PatchGeom g = patch_geom(W, H, P);
    hipLaunchKernelGGL((k_dual_tile<H_>), dim3(g.npx * g.tpp, g.npy * g.tpp), dim3(256), 0, st, I1, V1, M1,
                       I2, V2, M2, W, H, pitch, P, a, B, c_off, N2, bad_frac, D, VD, MD);
    PSFM_HIP_CHECK(hipGetLastError());
    return PSFM_OK;
}

// Outliers on a convolved image traced back to pixels of its input
// (Section 5.1): one workgroup per 64 x 64 tile of a patch.  The outlier
// flags of the tile and its h-halo are bit-packed in LDS; a tile without any
// writes zeros.  Otherwise |K_p| in FP64 (K_p realised at the patch centre)
// with its total summed in tap order, and each pixel x adds |K_p(u, v)| over
// the flagged pixels x + (u, v), rows then columns in increasing order, the
// pixel being marked when the sum is positive and at least frac sum |K_p|.
constexpr int TR_HW = TILE + 2 * PSFM_HMAX;
constexpr int TR_NWB = (TR_HW + 31) / 32 + 1;

__global__ __launch_bounds__(256) void k_trace_tile(const uint8_t* __restrict__ outl, int W, int H,
                                                    int64_t pitch, int P, const double* __restrict__ a,
                                                    BasisArgs B, double frac, uint8_t* __restrict__ bad) {
    __shared__ RealiseLds sh;
    __shared__ double Kd[(2 * PSFM_HMAX + 1) * (2 * PSFM_HMAX + 1)];
    __shared__ uint32_t badw[TR_HW][TR_NWB];
    __shared__ double s_thr;
    const int h = B.h, KW = 2 * h + 1, T = KW * KW, HW = TILE + 2 * h, tid = threadIdx.x;
    const PatchGeom g = patch_geom(W, H, P);
    const int px = blockIdx.x / g.tpp, sx = blockIdx.x % g.tpp;
    const int py = blockIdx.y / g.tpp, sy = blockIdx.y % g.tpp;
    const int X0 = px * P + sx * TILE, Y0 = py * P + sy * TILE;
    const int X1 = min(min(X0 + TILE, (px + 1) * P), W);
    const int Y1 = min(min(Y0 + TILE, (py + 1) * P), H);
    if (X0 >= X1 || Y0 >= Y1) return;
    for (int e = tid; e < TR_HW * TR_NWB; e += 256) (&badw[0][0])[e] = 0u;
    __syncthreads();
    int any = 0;
    for (int e = tid; e < HW * HW; e += 256) {
        const int hy = e / HW, hx = e - hy * HW;
        const int gy = Y0 - h + hy, gx = X0 - h + hx;
        if (gx >= 0 && gx < W && gy >= 0 && gy < H && outl[(int64_t)gy * pitch + gx]) {
            any = 1;
            atomicOr(&badw[hy][hx >> 5], 1u << (hx & 31));
        }
    }
    any = __syncthreads_or(any);
    if (any) {
        const int x0 = px * P, x1 = min(x0 + P, W), y0 = py * P, y1 = min(y0 + P, H);
        realise_kernel(B, a, 0.5 * (x0 + x1 - 1), 0.5 * (y0 + y1 - 1), W, H, sh, Kd);
        for (int t = tid; t < T; t += 256) Kd[t] = fabs(Kd[t]);
        __syncthreads();
        if (tid == 0) {
            double tot = 0.0;
            for (int t = 0; t < T; t++) tot += Kd[t];
            s_thr = frac * tot;
        }
        __syncthreads();
    }
    const double thr = any ? s_thr : 0.0;
    const uint64_t kmask = (1ull << KW) - 1ull;
    for (int e = tid; e < TILE * TILE; e += 256) {
        const int ly = e >> 6, lx = e & 63;
        const int gx = X0 + lx, gy = Y0 + ly;
        if (gx >= X1 || gy >= Y1) continue;
        uint8_t f = 0;
        if (any) {
            double s = 0.0;
            const int w = lx >> 5, shf = lx & 31;
            for (int v = 0; v < KW; v++) {
                const uint32_t* bw = badw[ly + v];
                uint64_t bits = (((uint64_t)bw[w] | ((uint64_t)bw[w + 1] << 32)) >> shf) & kmask;
                while (bits) {
                    const int u = __builtin_ctzll(bits);
                    bits &= bits - 1ull;
                    s += Kd[v * KW + u];
                }
            }
            f = (s >= thr && s > 0.0) ? 1 : 0;
        }
        bad[(int64_t)gy * pitch + gx] = f;
    }
}

}  // namespace

extern "C" int psfm_fit_norm(const psfm_context* ctx, const float* I1, const float* I2, int W, int H,
                             int64_t pitch, const int32_t* stamp_xy, int n_stamps,
                             const int32_t* stamp_flags, double* stamp_norm, void* stream) {
    if (!ctx || n_stamps < 0) return PSFM_ERR_INVALID_ARG;
    if (W < 1 || H < 1 || pitch < W) return PSFM_ERR_SHAPE;
    if (n_stamps == 0) return PSFM_OK;
    if (!I1 || !I2 || !stamp_xy || !stamp_flags || !stamp_norm) return PSFM_ERR_INVALID_ARG;
    hipLaunchKernelGGL(k_fit_norm, dim3(n_stamps), dim3(NQ_T), 0, (hipStream_t)stream, ctx->kb64, I1, I2,
                       W, H, pitch, stamp_xy, stamp_flags, ctx->r, ctx->h, stamp_norm);
    PSFM_HIP_CHECK(hipGetLastError());
    return PSFM_OK;
}

extern "C" int psfm_quality_eval(const psfm_context* ctx, const double* coeffs, const float* I1,
                                 const float* I2, const float* V2, int W, int H, int64_t pitch,
                                 const int32_t* stamp_xy, int n_stamps, const int32_t* stamp_flags,
                                 double soft, double* stamp_dev, psfm_quality* quality, void* stream) {
    if (!ctx || n_stamps < 0 || !coeffs || !quality || !(soft >= 0.0)) return PSFM_ERR_INVALID_ARG;
    if (W < 1 || H < 1 || pitch < W) return PSFM_ERR_SHAPE;
    if (n_stamps > 0 && (!I1 || !I2 || !V2 || !stamp_xy || !stamp_flags || !stamp_dev))
        return PSFM_ERR_INVALID_ARG;
    hipStream_t st = (hipStream_t)stream;
    const BasisArgs B = basis_args(ctx);
    if (n_stamps > 0)
        hipLaunchKernelGGL(k_stamp_dev, dim3(n_stamps), dim3(NQ_T), 0, st, B, coeffs, I1, I2, V2, W, H,
                           pitch, stamp_xy, stamp_flags, ctx->r, soft, stamp_dev);
    hipLaunchKernelGGL(k_quality_finish, dim3(1), dim3(NQ_T), 0, st, B, coeffs, W, H, n_stamps,
                       stamp_flags, stamp_dev, quality);
    PSFM_HIP_CHECK(hipGetLastError());
    return PSFM_OK;
}

extern "C" int psfm_trace_mask(const psfm_context* ctx, const double* coeffs, const uint8_t* outliers,
                               int W, int H, int64_t pitch, double frac, uint8_t* bad, void* stream) {
    int rc = check_image_args(ctx, W, H, pitch);
    if (rc) return rc;
    if (!coeffs || !outliers || !bad || !(frac >= 0.0)) return PSFM_ERR_INVALID_ARG;
    const PatchGeom g = patch_geom(W, H, ctx->cfg.patch);
    hipLaunchKernelGGL(k_trace_tile, dim3(g.npx * g.tpp, g.npy * g.tpp), dim3(256), 0, (hipStream_t)stream,
                       outliers, W, H, pitch, ctx->cfg.patch, coeffs, basis_args(ctx), frac, bad);
    PSFM_HIP_CHECK(hipGetLastError());
    return PSFM_OK;
}

extern "C" int psfm_dual_subtract(const psfm_context* ctx, const double* coeffs, const float* I1,
                                  const float* V1, const uint8_t* M1, const float* I2, const float* V2,
                                  const uint8_t* M2, int W, int H, int64_t pitch, float* diff,
                                  float* diff_var, uint8_t* diff_mask, void* stream) {
    int rc = check_image_args(ctx, W, H, pitch);
    if (rc) return rc;
    if (!coeffs || !I1 || !V1 || !M1 || !I2 || !V2 || !M2 || !diff || !diff_var || !diff_mask)
        return PSFM_ERR_INVALID_ARG;
    hipStream_t st = (hipStream_t)stream;
    const psfm_config& cf = ctx->cfg;
    const BasisArgs B = basis_args(ctx);
    const int c_off = (ctx->nb - 1) * ctx->ns, N2 = psfm::dual_unknowns(ctx);
    switch (ctx->h) {
#define PSFM_DUAL_CASE(HH) \
    case HH: return launch_dual<HH>(I1, V1, M1, I2, V2, M2, W, H, pitch, cf.patch, coeffs, B, c_off, N2, \
                                    cf.bad_frac, diff, diff_var, diff_mask, st);
        PSFM_DUAL_CASE(1) PSFM_DUAL_CASE(2) PSFM_DUAL_CASE(3) PSFM_DUAL_CASE(4) PSFM_DUAL_CASE(5)
        PSFM_DUAL_CASE(6) PSFM_DUAL_CASE(7) PSFM_DUAL_CASE(8) PSFM_DUAL_CASE(9) PSFM_DUAL_CASE(10)
        PSFM_DUAL_CASE(11) PSFM_DUAL_CASE(12) PSFM_DUAL_CASE(13) PSFM_DUAL_CASE(14) PSFM_DUAL_CASE(15)
        PSFM_DUAL_CASE(16)
#undef PSFM_DUAL_CASE
        default: return PSFM_ERR_UNSUPPORTED;
    }
}
