// Noise-model operations beyond convolution (Section 4.3, "Use in
// practise"): integer binning of an image with its variance map, mask and
// covariance pseudo-matrix; bilinear resampling of a pseudo-matrix to a new
// pixel scale; weighted sums of images with their variance maps and
// pseudo-matrices.  All three are HBM-bound streaming passes (the
// pseudo-matrix work is a few thousand operations in one workgroup).
#include "internal.h"

namespace {

constexpr int NB_T = 256;

__device__ __forceinline__ double cov_at(const double* __restrict__ C, int c, int dx, int dy) {
    if (!C) return (dx == 0 && dy == 0) ? 1.0 : 0.0;
    if (dx < -c || dx > c || dy < -c || dy > c) return 0.0;
    return C[(dy + c) * (2 * c + 1) + (dx + c)];
}

// Pseudo-matrix of a B x B block sum at fine offset D:
//   raw(D) = sum_{u, u' in block} C(D + u - u') = sum_{|e| < B} (B - |ex|)(B - |ey|) C(D + e),
// the number of (u, u') pairs with u - u' = e times the input pseudo-matrix.
__device__ double block_raw(const double* __restrict__ C, int c, int B, int dx, int dy) {
    double s = 0.0;
    for (int ey = -(B - 1); ey <= B - 1; ey++) {
        const double wy = (double)(B - abs(ey));
        for (int ex = -(B - 1); ex <= B - 1; ex++)
            s += wy * (double)(B - abs(ex)) * cov_at(C, c, dx + ex, dy + ey);
    }
    return s;
}

// Binned planes: one thread per output pixel; the block's unmasked pixels
// summed in FP64 (rows, then columns, in order), the variance times the
// covariance factor f = raw(0) / B^2 of the block sum.
__global__ __launch_bounds__(NB_T) void k_bin(const float* __restrict__ I, const float* __restrict__ V,
                                              const uint8_t* __restrict__ M, int64_t pitch, int B,
                                              const double* __restrict__ C, int c, int Wb, int Hb,
                                              float* __restrict__ Ib, float* __restrict__ Vb,
                                              uint8_t* __restrict__ Mb, int64_t pitch_b) {
    __shared__ double s_f;
    if (threadIdx.x == 0) s_f = block_raw(C, c, B, 0, 0) / ((double)B * B);
    __syncthreads();
    const int64_t t = (int64_t)blockIdx.x * NB_T + threadIdx.x;
    if (t >= (int64_t)Wb * Hb) return;
    const int Y = (int)(t / Wb), X = (int)(t - (int64_t)Y * Wb);
    double si = 0.0, sv = 0.0;
    uint8_t m = 0;
    for (int v = 0; v < B; v++) {
        const int64_t row = (int64_t)(B * Y + v) * pitch + (int64_t)B * X;
        for (int u = 0; u < B; u++) {
            const int64_t o = row + u;
            if (M[o]) {
                m = 1;
            } else {
                si += I[o];
                sv += V[o];
            }
        }
    }
    const int64_t ob = (int64_t)Y * pitch_b + X;
    Ib[ob] = (float)si;
    Vb[ob] = (float)(s_f * sv);
    Mb[ob] = m;
}

// The binned pseudo-matrix: raw at multiples of B normalised to the centre,
// cropped or zero-padded to (2 c_out + 1)^2; *discarded: share of sum |.|
// cut off.  One workgroup.
__global__ __launch_bounds__(NB_T) void k_bin_cov(const double* __restrict__ C, int c, int B,
                                                  double* __restrict__ out, int c_out,
                                                  double* __restrict__ discarded) {
    __shared__ double red[16];
    __shared__ double s_raw0;
    const int R = B - 1 + c, Rc = R / B, Rw = 2 * Rc + 1, Ow = 2 * c_out + 1;
    if (threadIdx.x == 0) s_raw0 = block_raw(C, c, B, 0, 0);
    __syncthreads();
    const double raw0 = s_raw0;
    double tot = 0.0, kept = 0.0;
    for (int e = threadIdx.x; e < Rw * Rw; e += NB_T) {
        const int DY = e / Rw - Rc, DX = e % Rw - Rc;
        const double v = block_raw(C, c, B, B * DX, B * DY) / raw0;
        tot += fabs(v);
        if (abs(DX) <= c_out && abs(DY) <= c_out) kept += fabs(v);
    }
    for (int e = threadIdx.x; e < Ow * Ow; e += NB_T) {
        const int DY = e / Ow - c_out, DX = e % Ow - c_out;
        out[e] = (abs(DX) <= Rc && abs(DY) <= Rc) ? block_raw(C, c, B, B * DX, B * DY) / raw0 : 0.0;
    }
    tot = psfm_block_sum(tot, red);
    kept = psfm_block_sum(kept, red);
    if (threadIdx.x == 0 && discarded) *discarded = tot > 0.0 ? (tot - kept) / tot : 0.0;
}

// Bilinear resampling of a pseudo-matrix to `scale` input pixels per output
// pixel, the off-centre entries rescaled to keep their input total.  One
// workgroup.
__global__ __launch_bounds__(NB_T) void k_resample_cov(const double* __restrict__ C, int c,
                                                       double scale, double* __restrict__ out,
                                                       int c_out) {
    __shared__ double red[16];
    const int Cw = 2 * c + 1, Ow = 2 * c_out + 1;
    double tin = 0.0, tout = 0.0;
    for (int e = threadIdx.x; e < Cw * Cw; e += NB_T)
        if (e != c * Cw + c) tin += C[e];
    for (int e = threadIdx.x; e < Ow * Ow; e += NB_T) {
        const int DY = e / Ow - c_out, DX = e % Ow - c_out;
        const double x = scale * DX, y = scale * DY;
        const double fx = floor(x), fy = floor(y), tx = x - fx, ty = y - fy;
        const int px = (int)fx, py = (int)fy;
        const double v = (1.0 - tx) * (1.0 - ty) * cov_at(C, c, px, py) +
                         tx * (1.0 - ty) * cov_at(C, c, px + 1, py) +
                         (1.0 - tx) * ty * cov_at(C, c, px, py + 1) + tx * ty * cov_at(C, c, px + 1, py + 1);
        out[e] = v;
        if (DX != 0 || DY != 0) tout += v;
    }
    tin = psfm_block_sum(tin, red);
    tout = psfm_block_sum(tout, red);
    const double a = tout != 0.0 ? tin / tout : 0.0;
    for (int e = threadIdx.x; e < Ow * Ow; e += NB_T)
        if (e != c_out * Ow + c_out) out[e] *= a;
}

constexpr int ADD_BLOCKS = 1024;

// One output pixel of the sum (and its share of the variance means).
__device__ __forceinline__ void add_pixel(double alpha, double beta, float ia, float va, uint8_t ma,
                                          float ib, float vb, uint8_t mb, float& s, float& vs,
                                          uint8_t& ms, double& sa, double& na, double& sb, double& nb) {
    if (!ma) {
        sa += va;
        na += 1.0;
    }
    if (!mb) {
        sb += vb;
        nb += 1.0;
    }
    ms = (uint8_t)(ma | mb);
    if (ms) {
        s = 0.0f;
        vs = 0.0f;
    } else {
        s = (float)(alpha * (double)ia + beta * (double)ib);
        vs = (float)(alpha * alpha * (double)va + beta * beta * (double)vb);
    }
}

// S = alpha Ia + beta Ib, V_S = alpha^2 Va + beta^2 Vb, mask_S = mask_a |
// mask_b (S = V_S = 0 there); per workgroup the unmasked variance sums and
// counts of both inputs (partials[4 b + 0..3], FP64).  Grid-stride over rows;
// with V4 (rows 16-byte aligned) four pixels per thread through 16-byte
// loads and stores (the masks as 4-byte words), the row's remainder one by one.
template <bool V4>
__global__ __launch_bounds__(NB_T) void k_add_images(double alpha, const float* __restrict__ Ia,
                                                     const float* __restrict__ Va,
                                                     const uint8_t* __restrict__ Ma, double beta,
                                                     const float* __restrict__ Ib,
                                                     const float* __restrict__ Vb,
                                                     const uint8_t* __restrict__ Mb, int W, int H,
                                                     int64_t pitch, float* __restrict__ S,
                                                     float* __restrict__ VS, uint8_t* __restrict__ MS,
                                                     double* __restrict__ partials) {
    __shared__ double red[16];
    double sa = 0.0, na = 0.0, sb = 0.0, nb = 0.0;
    const int W4 = V4 ? W / 4 * 4 : 0;
    for (int y = blockIdx.x; y < H; y += gridDim.x) {
        const int64_t row = (int64_t)y * pitch;
        if constexpr (V4) {
            for (int x = 4 * threadIdx.x; x < W4; x += 4 * NB_T) {
                const int64_t o = row + x;
                const float4 ia = *reinterpret_cast<const float4*>(Ia + o);
                const float4 va = *reinterpret_cast<const float4*>(Va + o);
                const float4 ib = *reinterpret_cast<const float4*>(Ib + o);
                const float4 vb = *reinterpret_cast<const float4*>(Vb + o);
                const uchar4 ma = *reinterpret_cast<const uchar4*>(Ma + o);
                const uchar4 mb = *reinterpret_cast<const uchar4*>(Mb + o);
                float4 s, vs;
                uchar4 ms;
                add_pixel(alpha, beta, ia.x, va.x, ma.x, ib.x, vb.x, mb.x, s.x, vs.x, ms.x, sa, na, sb, nb);
                add_pixel(alpha, beta, ia.y, va.y, ma.y, ib.y, vb.y, mb.y, s.y, vs.y, ms.y, sa, na, sb, nb);
                add_pixel(alpha, beta, ia.z, va.z, ma.z, ib.z, vb.z, mb.z, s.z, vs.z, ms.z, sa, na, sb, nb);
                add_pixel(alpha, beta, ia.w, va.w, ma.w, ib.w, vb.w, mb.w, s.w, vs.w, ms.w, sa, na, sb, nb);
                *reinterpret_cast<float4*>(S + o) = s;
                *reinterpret_cast<float4*>(VS + o) = vs;
                *reinterpret_cast<uchar4*>(MS + o) = ms;
            }
        }
        for (int x = W4 + threadIdx.x; x < W; x += NB_T) {
            const int64_t o = row + x;
            add_pixel(alpha, beta, Ia[o], Va[o], Ma[o], Ib[o], Vb[o], Mb[o], S[o], VS[o], MS[o], sa, na,
                      sb, nb);
        }
    }
    sa = psfm_block_sum(sa, red);
    na = psfm_block_sum(na, red);
    sb = psfm_block_sum(sb, red);
    nb = psfm_block_sum(nb, red);
    if (threadIdx.x == 0) {
        double* q = partials + 4 * (size_t)blockIdx.x;
        q[0] = sa;
        q[1] = na;
        q[2] = sb;
        q[3] = nb;
    }
}

// C_S = (wa Ca + wb Cb) / (wa + wb), wa = alpha^2 mean(Va), wb = beta^2
// mean(Vb) over unmasked pixels; the partials summed in block order.
__global__ __launch_bounds__(NB_T) void k_add_cov(double alpha, const double* __restrict__ Ca, int ca,
                                                  double beta, const double* __restrict__ Cb, int cb,
                                                  const double* __restrict__ partials, int nblk,
                                                  double* __restrict__ CS, int cs) {
    __shared__ double s_w[2];
    __shared__ double red[16];
    // thread t: blocks t, t + NB_T, ... (loads independent of each other),
    // then the fixed-order workgroup sums
    double q[4] = {0.0, 0.0, 0.0, 0.0};
    for (int b = threadIdx.x; b < nblk; b += NB_T) {
#pragma unroll
        for (int k = 0; k < 4; k++) q[k] += partials[4 * b + k];
    }
    psfm_block_sum4(q, red);
    if (threadIdx.x == 0) {
        s_w[0] = alpha * alpha * (q[1] > 0.0 ? q[0] / q[1] : 0.0);
        s_w[1] = beta * beta * (q[3] > 0.0 ? q[2] / q[3] : 0.0);
    }
    __syncthreads();
    const double wa = s_w[0], wb = s_w[1];
    const int Sw = 2 * cs + 1;
    for (int e = threadIdx.x; e < Sw * Sw; e += NB_T) {
        const int dy = e / Sw - cs, dx = e % Sw - cs;
        CS[e] = (wa + wb) > 0.0 ? (wa * cov_at(Ca, ca, dx, dy) + wb * cov_at(Cb, cb, dx, dy)) / (wa + wb)
                                : 0.0;
    }
}

}  // namespace

extern "C" int psfm_bin_image(const float* I, const float* V, const uint8_t* M, int W, int H,
                              int64_t pitch, int B, const double* cov_in, int cov_in_half,
                              float* Ib, float* Vb, uint8_t* Mb, int64_t pitch_b, double* cov_out,
                              int cov_out_half, double* discarded, void* stream) {
    if (!I || !V || !M || !Ib || !Vb || !Mb || !cov_out || cov_in_half < 0 || cov_out_half < 0)
        return PSFM_ERR_INVALID_ARG;
    if (B < 1 || B > 64 || cov_in_half > 64 || cov_out_half > 256) return PSFM_ERR_UNSUPPORTED;
    if (W < B || H < B || pitch < W || pitch_b < W / B) return PSFM_ERR_SHAPE;
    if (!cov_in) cov_in_half = 0;
    hipStream_t st = (hipStream_t)stream;
    const int Wb = W / B, Hb = H / B;
    const int64_t n = (int64_t)Wb * Hb;
    hipLaunchKernelGGL(k_bin, dim3((unsigned)((n + NB_T - 1) / NB_T)), dim3(NB_T), 0, st, I, V, M, pitch,
                       B, cov_in, cov_in_half, Wb, Hb, Ib, Vb, Mb, pitch_b);
    hipLaunchKernelGGL(k_bin_cov, dim3(1), dim3(NB_T), 0, st, cov_in, cov_in_half, B, cov_out,
                       cov_out_half, discarded);
    PSFM_HIP_CHECK(hipGetLastError());
    return PSFM_OK;
}

extern "C" int psfm_resample_cov(const double* cov_in, int cov_in_half, double scale, double* cov_out,
                                 int cov_out_half, void* stream) {
    if (!cov_in || !cov_out || cov_in_half < 0 || cov_out_half < 0 || !(scale > 0.0))
        return PSFM_ERR_INVALID_ARG;
    if (cov_in_half > 256 || cov_out_half > 256) return PSFM_ERR_UNSUPPORTED;
    hipLaunchKernelGGL(k_resample_cov, dim3(1), dim3(NB_T), 0, (hipStream_t)stream, cov_in, cov_in_half,
                       scale, cov_out, cov_out_half);
    PSFM_HIP_CHECK(hipGetLastError());
    return PSFM_OK;
}

extern "C" int psfm_add_images(double alpha, const float* Ia, const float* Va, const uint8_t* Ma,
                               const double* cov_a, int cov_a_half, double beta, const float* Ib,
                               const float* Vb, const uint8_t* Mb, const double* cov_b,
                               int cov_b_half, int W, int H, int64_t pitch, float* S, float* VS,
                               uint8_t* MS, double* cov_s, int cov_s_half, void* ws, size_t ws_bytes,
                               void* stream) {
    if (!Ia || !Va || !Ma || !Ib || !Vb || !Mb || !S || !VS || !MS || !cov_s || cov_a_half < 0 ||
        cov_b_half < 0 || cov_s_half < 0)
        return PSFM_ERR_INVALID_ARG;
    if (W < 1 || H < 1 || pitch < W) return PSFM_ERR_SHAPE;
    if (!ws || ws_bytes < PSFM_ADD_WORKSPACE_BYTES) return PSFM_ERR_WORKSPACE;
    hipStream_t st = (hipStream_t)stream;
    double* partials = static_cast<double*>(ws);
    const int nblk = H < ADD_BLOCKS ? H : ADD_BLOCKS;
    auto al16 = [](const void* ptr) { return ((uintptr_t)ptr & 15) == 0; };
    auto al4 = [](const void* ptr) { return ((uintptr_t)ptr & 3) == 0; };
    const bool v4 = (pitch & 3) == 0 && al16(Ia) && al16(Va) && al16(Ib) && al16(Vb) && al16(S) &&
                    al16(VS) && al4(Ma) && al4(Mb) && al4(MS);
    if (v4)
        hipLaunchKernelGGL(k_add_images<true>, dim3(nblk), dim3(NB_T), 0, st, alpha, Ia, Va, Ma, beta, Ib, Vb,
                           Mb, W, H, pitch, S, VS, MS, partials);
    else
        hipLaunchKernelGGL(k_add_images<false>, dim3(nblk), dim3(NB_T), 0, st, alpha, Ia, Va, Ma, beta, Ib,
                           Vb, Mb, W, H, pitch, S, VS, MS, partials);
    hipLaunchKernelGGL(k_add_cov, dim3(1), dim3(NB_T), 0, st, alpha, cov_a, cov_a ? cov_a_half : 0, beta,
                       cov_b, cov_b ? cov_b_half : 0, partials, nblk, cov_s, cov_s_half);
    PSFM_HIP_CHECK(hipGetLastError());
    return PSFM_OK;
}
