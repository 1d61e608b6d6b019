// Per-stamp normal equations (Section 2, Eqs. 3-6 with c = 0, p = 0).
//
// One workgroup handles one band of BR rows of one stamp (BR a template
// constant; the context picks 9 or 11 by stamp size):
//   1. the band's input window of I1 (band rows + 2h halo rows, stamp width
//      + 2h columns) is read from HBM into LDS, masked/non-finite pixels
//      become zeros and raise the stamp flags (validity, Section 3.3);
//   2. column pass: each distinct 1-D factor f_{j,e}(v) is applied along y
//      (FP32 FMA, the window column held in registers);
//   3. for every stamp row of the band: row pass of each basis term
//      (f_{j,p} along x over the column-pass output of f_{j,q}), the
//      zero-sum fix-up A_i = psi_i R_i - z_i A_0, the weighting by sqrt(1/V2)
//      and the extra columns sqrt(w) (background) and sqrt(w) * I2 (target);
//      the 64-column weighted row block is then folded into the Gram
//      G = A~^T A~ with v_mfma_f64_16x16x4f64 on the FP32 values (10 lower
//      16x16 blocks, spread over the 4 waves): exact products, FP64 sums over
//      the band, so the Gram of the FP32 block stays positive semi-definite
//      to FP64 rounding even for the 1e10-condition Grams of bright stars;
//   4. the band's partial Gram is written in FP64; a second kernel adds the
//      bands of each stamp and scatters M_s, b_s, e_s.
// 16-bit modes (PSFM_PREC_FP16 / _BF16): the weighted row block is rounded to
// 16 bits, stored column-major, and folded in with v_mfma_f32_16x16x32_{f16,
// bf16} (FP32 accumulation within a stamp row, rows added in FP64); in BF16 the block is
// split into hi + lo BF16 parts and the Gram is that of hi + lo (four
// products, ~16 significant bits, still positive semi-definite); the FP32
// block itself
// (terms, sqrt(w), d~) is written to the stamp design for the refinement of
// the solution, which recomputes residuals from it.
#include "internal.h"

namespace {

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef double doublex4 __attribute__((ext_vector_type(4)));
typedef _Float16 half8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef unsigned short u16x8 __attribute__((ext_vector_type(8)));

template <int PREC>
__device__ __forceinline__ unsigned short to16(float v) {
    if constexpr (PREC == PSFM_PREC_FP16) return __builtin_bit_cast(unsigned short, (_Float16)v);
    else return __builtin_bit_cast(unsigned short, (__bf16)v);
}

template <int PREC>
__device__ __forceinline__ floatx4 mfma16(u16x8 a, u16x8 b, floatx4 c) {
    if constexpr (PREC == PSFM_PREC_FP16)
        return __builtin_amdgcn_mfma_f32_16x16x32_f16(__builtin_bit_cast(half8, a),
                                                      __builtin_bit_cast(half8, b), c, 0, 0, 0);
    else
        return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, a),
                                                       __builtin_bit_cast(bf16x8, b), c, 0, 0, 0);
}

constexpr int SEG = 12;          // stamp pixels per row-pass item
constexpr int AT_STRIDE = 80;    // LDS row stride of the weighted block (bank spread)
constexpr int GC = PSFM_GRAM_COLS;
constexpr int A16S = 104;        // LDS column stride (halves) of the 16-bit block: up to 96 pixels
// Band mode that only writes the FP32 weighted block to the stamp design (no
// Gram): the two-kernel form's passes over I1 and over I2.
constexpr int PREC_DESIGN = 16;
// Gram entries per lane in rows 48 .. nb+1 (on the VALU): at most 904 for
// nb + 2 = 64 columns, over 4 x 256 lane slots
constexpr int GX_MAX = 4;

struct FitLds {
    int win, col, R, At, sw, dt, psi, z, fac, rf, cf, total;  // float offsets
};

// split: room for two 16-bit blocks (the BF16 mode's hi and lo parts).
__host__ __device__ inline FitLds fit_lds_layout(int h, int r, int nb, int nf, int BR, bool split) {
    const int WC = 2 * r + 1 + 2 * h;
    const int npad = (2 * r + 1 + 3) / 4 * 4;
    FitLds L;
    int o = 0;
    auto a4 = [](int x) { return (x + 3) / 4 * 4; };   // 16-byte aligned regions
    L.col = o;  o += a4(nf * BR * WC + SEG + 2 * h + 4);   // slack for the last row-pass loads
    // The window is dead once the column pass is done, so it shares its
    // space with the row loop's buffers (at seven-row bands, r = 20, h = 10,
    // this keeps a workgroup under a third of the CU's LDS: three per CU).
    const int u0 = o;
    L.win = u0;
    L.R = o;    o += a4(npad * nb);
    const int blk16 = split ? GC * A16S : GC * A16S / 2;     // floats
    L.At = o;   o += a4(npad * AT_STRIDE > blk16 ? npad * AT_STRIDE : blk16);
    if (o < u0 + a4((BR + 2 * h) * WC)) o = u0 + a4((BR + 2 * h) * WC);
    L.sw = o;   o += BR * (2 * r + 1);
    L.dt = o;   o += BR * (2 * r + 1);
    L.psi = o;  o += 64;
    L.z = o;    o += 64;
    L.fac = o;  o += a4(nf * (2 * h + 1));
    L.rf = o;   o += 64;
    L.cf = o;   o += 64;
    L.total = o + 4;
    return L;
}

// Arguments of one stamp fit (one image pair).
struct FitArgs {
    const float* I1;
    const uint8_t* M1;
    const float* I2;
    const float* V2;
    const uint8_t* M2;
    const float* V1;   // weight 1 / (V1 + V2) when wmode is PSFM_WEIGHT_V1V2
    int wmode;
    int W, H;
    int64_t pitch;
    const int32_t* xy;
    int r, nbands;
    const float* fac;
    const int* rowf;
    const int* colf;
    const float* psi;
    const float* zf;
    int nb, nf;
    double* part;
    int* band_flags;
    float* design;     // 16-bit modes: [stamp][nb + 2][(2r+1)^2] FP32 block, column-major
};

// One band of BR rows of one stamp (item = stamp * nbands + band).
template <int H_, int PREC, int BR>
__device__ void fit_band_body(const FitArgs& a, const int item, float* __restrict__ lds) {
    const float* __restrict__ I1 = a.I1;
    const uint8_t* __restrict__ M1 = a.M1;
    const float* __restrict__ I2 = a.I2;
    const float* __restrict__ V2 = a.V2;
    const uint8_t* __restrict__ M2 = a.M2;
    const int W = a.W, H = a.H;
    const int64_t pitch = a.pitch;
    const int32_t* __restrict__ xy = a.xy;
    const int r = a.r, nbands = a.nbands;
    const float* __restrict__ fac = a.fac;
    const int* __restrict__ rowf = a.rowf;
    const int* __restrict__ colf = a.colf;
    const float* __restrict__ psi = a.psi;
    const float* __restrict__ zf = a.zf;
    const int nb = a.nb, nf = a.nf;
    double* __restrict__ part = a.part;
    int* __restrict__ band_flags = a.band_flags;
    constexpr int KW = 2 * H_ + 1;
    __shared__ int s_flags;

    const int tid = threadIdx.x;
    const int s = item / nbands;
    const int band = item % nbands;
    const int xc = xy[2 * s], yc = xy[2 * s + 1];
    const int R = r + H_;
    const int NPX = 2 * r + 1;
    const int WC = NPX + 2 * H_;
    const int npad = (NPX + 3) / 4 * 4;
    const FitLds Lo = fit_lds_layout(H_, r, nb, nf, BR, PREC == PSFM_PREC_BF16);
    float* win = lds + Lo.win;
    float* colb = lds + Lo.col;
    float* Rb = lds + Lo.R;
    float* At = lds + Lo.At;
    float* swb = lds + Lo.sw;
    float* dtb = lds + Lo.dt;
    float* psib = lds + Lo.psi;
    float* zb = lds + Lo.z;
    float* facb = lds + Lo.fac;
    int* rfb = reinterpret_cast<int*>(lds + Lo.rf);
    int* cfb = reinterpret_cast<int*>(lds + Lo.cf);

    if (xc - R < 0 || yc - R < 0 || xc + R >= W || yc + R >= H) {
        if (tid == 0) band_flags[item] = PSFM_STAMP_INVALID;
        return;
    }
    if (tid == 0) s_flags = 0;
    if (tid < 64) {
        psib[tid] = tid < nb ? psi[tid] : 0.0f;
        zb[tid] = tid < nb ? zf[tid] : 0.0f;
        rfb[tid] = tid < nb ? rowf[tid] : 0;
        cfb[tid] = tid < nb ? colf[tid] : 0;
    }
    for (int e = tid; e < nf * KW; e += 256) facb[e] = fac[e];   // the 1-D factors, for the row passes
    __syncthreads();

    const int y_l0 = band * BR;
    const int nbr = min(BR, NPX - y_l0);
    // ---- 1. input window and stamp pixel data
    int fl = 0;
    {
        const int rows = BR + 2 * H_;
        const int gy0 = yc - r + y_l0 - H_;
        const int gx0 = xc - R;
        // WIN_CHUNK pixels per thread in flight (unconditional loads from a
        // clamped address; rows past the band read pixel (gy0, gx0))
        constexpr int WIN_CHUNK = 8;
        for (int e0 = tid; e0 < rows * WC; e0 += 256 * WIN_CHUNK) {
            float xv[WIN_CHUNK];
            uint8_t mv[WIN_CHUNK];
#pragma unroll
            for (int u = 0; u < WIN_CHUNK; u++) {
                const int e = e0 + 256 * u;
                const int wr = e / WC, wc = e - wr * WC;
                const bool in = e < rows * WC && wr < nbr + 2 * H_;
                const int64_t o = (int64_t)(gy0 + (in ? wr : 0)) * pitch + (gx0 + (in ? wc : 0));
                xv[u] = I1[o];
                mv[u] = M1[o];
            }
#pragma unroll
            for (int u = 0; u < WIN_CHUNK; u++) {
                const int e = e0 + 256 * u;
                if (e >= rows * WC) continue;
                const int wr = e / WC;
                float v = 0.0f;
                if (wr < nbr + 2 * H_) {
                    if (mv[u]) fl |= PSFM_STAMP_INVALID;
                    else if (!isfinite(xv[u])) fl |= PSFM_STAMP_NONFINITE;
                    else v = xv[u];
                }
                win[e] = v;
            }
        }
        for (int e = tid; e < nbr * NPX; e += 256) {
            const int br = e / NPX, x = e - br * NPX;
            const int64_t o = (int64_t)(yc - r + y_l0 + br) * pitch + (xc - r + x);
            const float i2 = I2[o];
            const float v2 = a.wmode == PSFM_WEIGHT_V1V2 ? V2[o] + a.V1[o] : V2[o];
            float sw = 0.0f, dt = 0.0f;
            if (M2[o]) {
                fl |= PSFM_STAMP_INVALID;
            } else if (!isfinite(i2) || !isfinite(v2) || !(v2 > 0.0f)) {
                fl |= PSFM_STAMP_NONFINITE;
            } else {
                sw = 1.0f / sqrtf(v2);
                dt = sw * i2;
            }
            swb[e] = sw;
            dtb[e] = dt;
        }
    }
    if (fl) atomicOr(&s_flags, fl);
    // Offset: the window mean c is removed before the basis convolution and
    // added back to term 0 only (every other term sums to zero, so it is
    // blind to a constant).  The FP32 rounding of the zero-sum terms then
    // scales with |I1 - c| instead of |I1| (the sky).
    double wsum = 0.0;
    {
        const int rows = nbr + 2 * H_;
        for (int e = tid; e < rows * WC; e += 256) wsum += win[e];
    }
    __shared__ double red[16];
    const float cshift = (float)(psfm_block_sum(wsum, red) / ((nbr + 2 * H_) * WC));
    const int flags = s_flags;
    if (flags) {
        if (tid == 0) band_flags[item] = flags;
        return;
    }
    for (int e = tid; e < (nbr + 2 * H_) * WC; e += 256) win[e] -= cshift;
    __syncthreads();

    // ---- 2. column pass: colb[f][br][wc] = sum_v f(v) I1(wc, br - v)
    for (int item = tid; item < nf * WC; item += 256) {
        const int f = item / WC, wc = item - f * WC;
        float tap[KW];
#pragma unroll
        for (int vv = 0; vv < KW; vv++) tap[vv] = fac[f * KW + vv];
        float acc[BR];
#pragma unroll
        for (int br = 0; br < BR; br++) acc[br] = 0.0f;
#pragma unroll
        for (int br = 0; br < BR; br++) {
#pragma unroll
            for (int vv = 0; vv < KW; vv++) acc[br] = fmaf(tap[vv], win[(br + 2 * H_ - vv) * WC + wc], acc[br]);
        }
        float* dst = colb + (f * BR) * WC + wc;
#pragma unroll
        for (int br = 0; br < BR; br++) dst[br * WC] = acc[br];
    }
    __syncthreads();

    // ---- 3. rows of the band
    const int lane = tid & 63, wave = tid >> 6;
    floatx4 acc[3];            // 16-bit modes: FP32 MFMA sums of one stamp row
    doublex4 accd[3];          // FP64 sums of the band
#pragma unroll
    for (int q = 0; q < 3; q++) {
        acc[q] = floatx4{0.0f, 0.0f, 0.0f, 0.0f};
        accd[q] = doublex4{0.0, 0.0, 0.0, 0.0};
    }
    // FP32 mode: the Gram rows 48 .. nb+1 on the VALU of waves 2 and 3 --
    // entry e = (tid - 128) + 128 j of the row-major lower triangle of those
    // rows, (er[j], ec[j]), summed in ex[j]
    int er[GX_MAX], ec[GX_MAX], nxl = 0;
    double ex[GX_MAX];
    {
        // entry e = ((tid + 128) % 256) + 256 j of the row-major lower
        // triangle of rows 48 .. nb+1: waves 2 and 3 (one MFMA block each)
        // take the first 128, waves 0 and 1 any beyond
        const int R1 = nb + 1;
        const int E = R1 >= 48 ? (R1 + 1) * (R1 + 2) / 2 - 48 * 49 / 2 : 0;
        const int l2 = (tid + 128) & 255;
#pragma unroll
        for (int j = 0; j < GX_MAX; j++) {
            ex[j] = 0.0;
            er[j] = 0;
            ec[j] = 0;
            const int e = l2 + 256 * j;
            if (PREC == PSFM_PREC_FP32 && e < E) {
                int r = 48, rem = e;
                while (rem >= r + 1) {
                    rem -= r + 1;
                    r++;
                }
                er[j] = r;
                ec[j] = rem;
                nxl = j + 1;
            }
        }
    }
    const int nseg = (NPX + SEG - 1) / SEG;
    // row-pass item of this thread (the usual case: nb * nseg <= 256), its
    // taps held in registers across the rows
    const bool one = nb * nseg <= 256;
    const int i1 = tid < nb * nseg ? tid / nseg : 0, x01 = (tid - i1 * nseg) * SEG;
    float tap1[KW];
#pragma unroll
    for (int uu = 0; uu < KW; uu++) tap1[uu] = facb[rfb[i1] * KW + uu];
    const int src1 = cfb[i1] * BR * WC + x01;
    for (int br = 0; br < nbr; br++) {
        // 3a. row pass: Rb[x][i] = sum_u f_{j,p}(u) colb[f_{j,q}][br][x + 2h - uu]
        auto row_item = [&](const float* tap, const float* src, int i, int x0) {
            float a[SEG];
#pragma unroll
            for (int k = 0; k < SEG; k++) {
                a[k] = 0.0f;
#pragma unroll
                for (int uu = 0; uu < KW; uu++) a[k] = fmaf(tap[uu], src[k + 2 * H_ - uu], a[k]);
            }
#pragma unroll
            for (int k = 0; k < SEG; k++)
                if (x0 + k < NPX) Rb[(x0 + k) * nb + i] = a[k];
        };
        if (one) {
            if (tid < nb * nseg) row_item(tap1, colb + src1 + br * WC, i1, x01);
        } else {
            for (int item = tid; item < nb * nseg; item += 256) {
                const int i = item / nseg, seg = item - i * nseg;
                const int x0 = seg * SEG;
                float tap[KW];
#pragma unroll
                for (int uu = 0; uu < KW; uu++) tap[uu] = facb[rfb[i] * KW + uu];
                row_item(tap, colb + (cfb[i] * BR + br) * WC + x0, i, x0);
            }
        }
        __syncthreads();
        if constexpr (PREC == PSFM_PREC_FP32) {
        // 3b. zero-sum fix-up, weights, extra columns: one column per lane
        //     (its psi and z in registers), the wave's rows four apart
        {
            static_assert(GC == 64, "one Gram column per lane");
            const int c = tid & (GC - 1);
            const float pc = c < nb ? psib[c] : 0.0f, zc = c < nb ? zb[c] : 0.0f, p0 = psib[0];
            const float add = c == 0 ? cshift : 0.0f;
#pragma unroll 4
            for (int x = tid >> 6; x < npad; x += 4) {
                float v = 0.0f;
                if (x < NPX) {
                    const float sw = swb[br * NPX + x];
                    if (c < nb) v = sw * (pc * Rb[x * nb + c] - zc * (p0 * Rb[x * nb]) + add);
                    else if (c == nb) v = sw;
                    else if (c == nb + 1) v = dtb[br * NPX + x];
                }
                At[x * AT_STRIDE + c] = v;
            }
        }
        __syncthreads();
        // 3c. The Gram of the block.  The FP32 values enter
        //     v_mfma_f64_16x16x4f64 as FP64: every product is exact and the
        //     sums run in FP64 over the whole band, so the Gram is that of
        //     the FP32 block to FP64 rounding (and positive semi-definite to
        //     it), whatever its condition.  Rows 0..47 in six 16 x 16 blocks
        //     (bm, bn): w0 (0,0)(1,1); w1 (1,0)(2,2); w2 (2,0); w3 (2,1);
        //     rows 48 .. nb+1 (the last terms, sqrt(w), d~: three rows of the
        //     49-term basis, not worth a block row of MFMA) on the FP64 VALU,
        //     entries (er[j], ec[j]) of each lane.
        for (int ks = 0; ks < npad / 4; ks++) {
            const float* rowp = At + (4 * ks + (lane >> 4)) * AT_STRIDE + (lane & 15);
            if (wave == 0) {
                const double a0 = rowp[0], a1 = rowp[16];
                accd[0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, a0, accd[0], 0, 0, 0);
                accd[1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, a1, accd[1], 0, 0, 0);
            } else if (wave == 1) {
                const double a0 = rowp[0], a1 = rowp[16], a2 = rowp[32];
                accd[0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, a0, accd[0], 0, 0, 0);
                accd[1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a2, a2, accd[1], 0, 0, 0);
            } else {
                const double a2 = rowp[32], ab = rowp[wave == 2 ? 0 : 16];
                accd[0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a2, ab, accd[0], 0, 0, 0);
            }
            const float* xr = At + 4 * ks * AT_STRIDE;
#pragma unroll
            for (int j = 0; j < GX_MAX; j++) {
                if (j < nxl) {
#pragma unroll
                    for (int q = 0; q < 4; q++)
                        ex[j] = fma((double)xr[q * AT_STRIDE + er[j]], (double)xr[q * AT_STRIDE + ec[j]], ex[j]);
                }
            }
        }
        } else {
        // 3b'. the same block, rounded to 16 bits, column-major A16[c][x]
        //      (pixels padded to a multiple of 32); FP32 values to the design
        unsigned short* A16 = reinterpret_cast<unsigned short*>(At);
        unsigned short* A16lo = A16 + GC * A16S;      // BF16: the remainders v - hi
        const int kp = (NPX + 31) / 32 * 32;
        float* dsg = a.design + (size_t)s * (nb + 2) * (NPX * NPX) + (size_t)(y_l0 + br) * NPX;
        for (int e = tid; e < GC * kp; e += 256) {
            const int c = e / kp, x = e - c * kp;
            float v = 0.0f;
            if (x < NPX) {
                const float sw = swb[br * NPX + x];
                if (c < nb) v = sw * (psib[c] * Rb[x * nb + c] - zb[c] * (psib[0] * Rb[x * nb]) +
                                      (c == 0 ? cshift : 0.0f));
                else if (c == nb) v = sw;
                else if (c == nb + 1) v = dtb[br * NPX + x];
                if (c < nb + 2) dsg[(size_t)c * (NPX * NPX) + x] = v;
            }
            if constexpr (PREC != PREC_DESIGN) {
                const unsigned short hi = to16<PREC>(v);
                A16[c * A16S + x] = hi;
                if constexpr (PREC == PSFM_PREC_BF16)
                    A16lo[c * A16S + x] = to16<PREC>(v - (float)__builtin_bit_cast(__bf16, hi));
            }
        }
        __syncthreads();
        if constexpr (PREC != PREC_DESIGN) {
        // 3c'. Gram blocks, K = 32 pixels per instruction (same wave blocks)
        for (int ks = 0; ks < kp / 32; ks++) {
            const unsigned short* colp = A16 + (lane & 15) * A16S + 32 * ks + 8 * (lane >> 4);
            auto ld = [&](int b) { return *reinterpret_cast<const u16x8*>(colp + 16 * b * A16S); };
            if constexpr (PREC == PSFM_PREC_BF16) {
                // x y = (hi_x + lo_x)(hi_y + lo_y), all four BF16 products with FP32
                // sums: the Gram of the 16-bit-significand block hi + lo, so it
                // stays positive semi-definite (dropping lo lo would not)
                auto ll = [&](int b) {
                    return *reinterpret_cast<const u16x8*>(colp + GC * A16S + 16 * b * A16S);
                };
                auto m3 = [&](floatx4 c, int bx, int by) {
                    const u16x8 xh = ld(bx), yh = ld(by), xl = ll(bx), yl = ll(by);
                    c = mfma16<PREC>(xh, yh, c);
                    c = mfma16<PREC>(xh, yl, c);
                    c = mfma16<PREC>(xl, yh, c);
                    return mfma16<PREC>(xl, yl, c);
                };
                if (wave == 0) {
                    acc[0] = m3(acc[0], 0, 0);
                    acc[1] = m3(acc[1], 1, 0);
                    acc[2] = m3(acc[2], 1, 1);
                } else if (wave == 1) {
                    acc[0] = m3(acc[0], 2, 0);
                    acc[1] = m3(acc[1], 2, 1);
                    acc[2] = m3(acc[2], 2, 2);
                } else if (wave == 2) {
                    acc[0] = m3(acc[0], 3, 0);
                    acc[1] = m3(acc[1], 3, 1);
                } else {
                    acc[0] = m3(acc[0], 3, 2);
                    acc[1] = m3(acc[1], 3, 3);
                }
                continue;
            }
            if (wave == 0) {
                const u16x8 a0 = ld(0), a1 = ld(1);
                acc[0] = mfma16<PREC>(a0, a0, acc[0]);
                acc[1] = mfma16<PREC>(a1, a0, acc[1]);
                acc[2] = mfma16<PREC>(a1, a1, acc[2]);
            } else if (wave == 1) {
                const u16x8 a0 = ld(0), a1 = ld(1), a2 = ld(2);
                acc[0] = mfma16<PREC>(a2, a0, acc[0]);
                acc[1] = mfma16<PREC>(a2, a1, acc[1]);
                acc[2] = mfma16<PREC>(a2, a2, acc[2]);
            } else if (wave == 2) {
                const u16x8 a0 = ld(0), a1 = ld(1), a3 = ld(3);
                acc[0] = mfma16<PREC>(a3, a0, acc[0]);
                acc[1] = mfma16<PREC>(a3, a1, acc[1]);
            } else {
                const u16x8 a2 = ld(2), a3 = ld(3);
                acc[0] = mfma16<PREC>(a3, a2, acc[0]);
                acc[1] = mfma16<PREC>(a3, a3, acc[1]);
            }
        }
        }
        }
        // 16-bit modes: the FP32 MFMA sums cover one stamp row; rows are
        // added in FP64.
        if constexpr (PREC != PSFM_PREC_FP32 && PREC != PREC_DESIGN) {
#pragma unroll
            for (int q = 0; q < 3; q++) {
#pragma unroll
                for (int e = 0; e < 4; e++) accd[q][e] += (double)acc[q][e];
                acc[q] = floatx4{0.0f, 0.0f, 0.0f, 0.0f};
            }
        }
        // Rb may be rewritten only after every wave finished 3b (barrier above);
        // At is rewritten after the barrier that follows the next row pass.
    }

    // ---- 4. partial Gram out, column 16 bn + lane % 16; row 16 bm + (lane / 16) + 4 e
    //         from the FP64 MFMA, 16 bm + 4 (lane / 16) + e from the FP32 ones
    if constexpr (PREC == PREC_DESIGN) {
        if (tid == 0) band_flags[item] = 0;
        return;
    }
    double* G = part + (size_t)item * GC * GC;
    // blocks (bm, bn) of each wave: the FP32 mode's six below row 48, the
    // 16-bit modes' ten
    const int bms32[4][3] = {{0, 1, -1}, {1, 2, -1}, {2, -1, -1}, {2, -1, -1}};
    const int bns32[4][3] = {{0, 1, -1}, {0, 2, -1}, {0, -1, -1}, {1, -1, -1}};
    const int bms16[4][3] = {{0, 1, 1}, {2, 2, 2}, {3, 3, -1}, {3, 3, -1}};
    const int bns16[4][3] = {{0, 0, 1}, {0, 1, 2}, {0, 1, -1}, {2, 3, -1}};
    const bool six = PREC == PSFM_PREC_FP32;
    if constexpr (PREC == PSFM_PREC_FP32) {
#pragma unroll
        for (int j = 0; j < GX_MAX; j++)
            if (j < nxl) G[er[j] * GC + ec[j]] = ex[j];
    }
#pragma unroll
    for (int q = 0; q < 3; q++) {
        const int bm = six ? bms32[wave][q] : bms16[wave][q];
        const int bn = six ? bns32[wave][q] : bns16[wave][q];
        if (bm < 0) continue;
        const int col = 16 * bn + (lane & 15);
#pragma unroll
        for (int e = 0; e < 4; e++) {
            const int row = PREC == PSFM_PREC_FP32 ? 16 * bm + (lane >> 4) + 4 * e
                                                   : 16 * bm + 4 * (lane >> 4) + e;
            G[row * GC + col] = accd[q][e];
        }
    }
    if (tid == 0) band_flags[item] = 0;
}

template <int H_, int PREC, int BR>
__global__ __launch_bounds__(256) void k_fit_band(FitArgs a) {
    extern __shared__ float lds[];
    fit_band_body<H_, PREC, BR>(a, blockIdx.x, lds);
}

// All bands of all stamps of all pairs of a batch; item_pair maps the
// flattened band index to its pair.
template <int H_, int BR>
__global__ __launch_bounds__(256) void k_fit_band_b(const PairDesc* __restrict__ pairs,
                                                    const int* __restrict__ item_pair, FitArgs base) {
    extern __shared__ float lds[];
    const PairDesc& pd = pairs[item_pair[blockIdx.x]];
    FitArgs a = base;
    a.I1 = pd.I1;
    a.M1 = pd.M1;
    a.I2 = pd.I2;
    a.V2 = pd.V2;
    a.M2 = pd.M2;
    a.V1 = pd.V1;
    a.W = pd.W;
    a.H = pd.H;
    a.pitch = pd.pitch;
    a.xy = pd.xy;
    a.part = pd.part;
    a.band_flags = pd.bflags;
    fit_band_body<H_, PSFM_PREC_FP32, BR>(a, blockIdx.x - pd.band_off, lds);
}

// Sum of the band partials of each stamp in FP64 and scatter to M_s, b_s, e_s.
// One workgroup per stamp: the stored lower triangle (rows 0 .. nb + 1 of
// the partial Gram, nb + 1 being the weighted target) is read row by row
// (consecutive entries, consecutive lanes), each entry summed over the bands
// in order into LDS; M_s is then written row-major from LDS (its upper part
// mirrored), so both the reads and the writes are contiguous.
constexpr int RED_TRI = (GC + 1) * GC / 2;     // lower-triangle entries of the partial (<= GC rows)

__device__ void fit_reduce_body(const double* __restrict__ part, const int* __restrict__ band_flags,
                                int nbands, int nb, int npix, double* __restrict__ Ms,
                                double* __restrict__ bs, double* __restrict__ es,
                                int32_t* __restrict__ npix_out, int32_t* __restrict__ flags_out,
                                const int s) {
    const int tid = threadIdx.x;
    const int L = nb + 1, R = nb + 2;               // Gram rows: the L unknowns and the target
    __shared__ int s_fl;
    __shared__ double tri[RED_TRI];                  // entry (r, c), c <= r, at r (r + 1) / 2 + c
    if (tid < 64) {     // the bands' flags, one per lane, OR over the wave
        int f = 0;
        for (int b = tid; b < nbands; b += 64) f |= band_flags[s * nbands + b];
        for (int o = 32; o > 0; o >>= 1) f |= __shfl_xor(f, o);
        if (tid == 0) s_fl = (f & PSFM_STAMP_INVALID) ? PSFM_STAMP_INVALID : f;
    }
    __syncthreads();
    const int fl = s_fl;
    const double* P0 = part + (size_t)s * nbands * GC * GC;
    const int ntri = R * (R + 1) / 2;
    // four entries per thread, their band partials loaded together
    for (int e0 = tid; e0 < ntri; e0 += 4 * 256) {
        double v[4] = {0.0, 0.0, 0.0, 0.0};
        int off[4];
#pragma unroll
        for (int u = 0; u < 4; u++) {
            const int e = min(e0 + 256 * u, ntri - 1);
            int r = (int)((sqrtf(8.0f * e + 1.0f) - 1.0f) * 0.5f);
            while ((r + 1) * (r + 2) / 2 <= e) r++;
            while (r * (r + 1) / 2 > e) r--;
            off[u] = r * GC + (e - r * (r + 1) / 2);
        }
        if (!fl) {
            for (int b = 0; b < nbands; b++) {
                const double* Pb = P0 + (size_t)b * GC * GC;
#pragma unroll
                for (int u = 0; u < 4; u++) v[u] += Pb[off[u]];
            }
        }
#pragma unroll
        for (int u = 0; u < 4; u++)
            if (e0 + 256 * u < ntri) tri[e0 + 256 * u] = v[u];
    }
    __syncthreads();
    double* M = Ms + (size_t)s * L * L;
    for (int e = tid; e < L * L; e += 256) {
        const int i = e / L, j = e - i * L;
        const int r = i > j ? i : j, c = i > j ? j : i;
        M[e] = tri[r * (r + 1) / 2 + c];
    }
    for (int i = tid; i <= L; i += 256) {
        const double v = tri[(R - 1) * R / 2 + i];   // row nb + 1: b_i, then e at i = L
        if (i < L) bs[(size_t)s * L + i] = v;
        else es[s] = v;
    }
    if (tid == 0) {
        npix_out[s] = fl ? 0 : npix;
        flags_out[s] = fl;
    }
}

__global__ __launch_bounds__(256) void k_fit_reduce(const double* __restrict__ part,
                                                    const int* __restrict__ band_flags, int nbands,
                                                    int nb, int npix, double* __restrict__ Ms,
                                                    double* __restrict__ bs, double* __restrict__ es,
                                                    int32_t* __restrict__ npix_out,
                                                    int32_t* __restrict__ flags_out) {
    fit_reduce_body(part, band_flags, nbands, nb, npix, Ms, bs, es, npix_out, flags_out, blockIdx.x);
}


__global__ __launch_bounds__(256) void k_fit_reduce_b(const PairDesc* __restrict__ pairs,
                                                      const int* __restrict__ stamp_pair, int nbands,
                                                      int nb, int npix) {
    const PairDesc& pd = pairs[stamp_pair[blockIdx.x]];
    fit_reduce_body(pd.part, pd.bflags, nbands, nb, npix, pd.Ms, pd.bs, pd.es, pd.npix, pd.flags,
                    blockIdx.x - pd.stamp_off);
}

// Per-stamp sums of the two-kernel form (Section 2, Eqs. 3-6 with the I2
// columns): one workgroup per stamp over the two FP32 designs of the
// design-only band passes (over I1, and over I2 in its place).  Columns, in
// the order of the stamp matrix: k_i (x) I1 for i < nb (design 1), k_i (x) I2
// for 1 <= i < nb (design 2), sqrt(w), then sqrt(w) I2 (design 1); chunks of
// GD_KC pixels go through LDS and the lower 16 x 16 blocks of their Gram
// accumulate on v_mfma_f64_16x16x4f64 (exact products of the FP32 values,
// FP64 sums), blocks q = wave + 4 j.
constexpr int GD_KC = 32;               // stamp pixels per LDS chunk
constexpr int GD_COLS = 128;            // 2 nb + 1 <= 125 columns (nb <= 62)
constexpr int GD_STRIDE = GD_COLS + 4;  // LDS row stride (floats)
constexpr int GD_JMAX = 9;              // blocks per wave: 36 lower blocks / 4 waves

__global__ __launch_bounds__(256) void k_gram_dual(const float* __restrict__ d1,
                                                   const float* __restrict__ d2,
                                                   const int* __restrict__ bf1,
                                                   const int* __restrict__ bf2, int nbands, int nb,
                                                   int npix, double* __restrict__ Ms,
                                                   double* __restrict__ bs, double* __restrict__ es,
                                                   int32_t* __restrict__ npix_out,
                                                   int32_t* __restrict__ flags_out) {
    __shared__ float Tb[GD_KC * GD_STRIDE];
    __shared__ int s_fl;
    const int s = blockIdx.x, tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int L = 2 * nb, Lx = L + 1, nblk = (Lx + 15) / 16, ntri = nblk * (nblk + 1) / 2;
    if (tid < 64) {
        int f = 0;
        for (int b = tid; b < nbands; b += 64) f |= bf1[s * nbands + b] | bf2[s * nbands + b];
        for (int o = 32; o > 0; o >>= 1) f |= __shfl_xor(f, o);
        if (tid == 0) s_fl = (f & PSFM_STAMP_INVALID) ? PSFM_STAMP_INVALID : f;
    }
    __syncthreads();
    const int fl = s_fl;
    double* M = Ms + (size_t)s * L * L;
    double* bv = bs + (size_t)s * L;
    if (fl) {
        for (int e = tid; e < L * L; e += 256) M[e] = 0.0;
        for (int e = tid; e < L; e += 256) bv[e] = 0.0;
        if (tid == 0) {
            es[s] = 0.0;
            npix_out[s] = 0;
            flags_out[s] = fl;
        }
        return;
    }
    const size_t dstride = (size_t)(nb + 2) * npix;
    const float* D1 = d1 + (size_t)s * dstride;
    const float* D2 = d2 + (size_t)s * dstride;
    int bmq[GD_JMAX], bnq[GD_JMAX];
    doublex4 acc[GD_JMAX];
#pragma unroll
    for (int j = 0; j < GD_JMAX; j++) {
        const int q = wave + 4 * j;
        int bm = 0;
        while ((bm + 1) * (bm + 2) / 2 <= q) bm++;
        bmq[j] = q < ntri ? bm : -1;
        bnq[j] = q - bm * (bm + 1) / 2;
        acc[j] = doublex4{0.0, 0.0, 0.0, 0.0};
    }
    for (int x0 = 0; x0 < npix; x0 += GD_KC) {
        __syncthreads();
        for (int e = tid; e < GD_COLS * GD_KC; e += 256) {
            const int c = e / GD_KC, x = e - c * GD_KC, px = x0 + x;
            float v = 0.0f;
            if (px < npix && c < Lx) {
                const float* col = c < nb ? D1 + (size_t)c * npix
                                   : c < L - 1 ? D2 + (size_t)(c - nb + 1) * npix
                                   : D1 + (size_t)(nb + c - (L - 1)) * npix;
                v = col[px];
            }
            Tb[x * GD_STRIDE + c] = v;
        }
        __syncthreads();
#pragma unroll 2
        for (int ks = 0; ks < GD_KC / 4; ks++) {
            const float* rowp = Tb + (4 * ks + (lane >> 4)) * GD_STRIDE + (lane & 15);
#pragma unroll
            for (int j = 0; j < GD_JMAX; j++) {
                if (bmq[j] < 0) continue;
                const double av = rowp[16 * bmq[j]], bw = rowp[16 * bnq[j]];
                acc[j] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bw, acc[j], 0, 0, 0);
            }
        }
    }
    // D row 16 bm + (lane / 16) + 4 e, column 16 bn + lane % 16
#pragma unroll
    for (int j = 0; j < GD_JMAX; j++) {
        if (bmq[j] < 0) continue;
#pragma unroll
        for (int e = 0; e < 4; e++) {
            const int i = 16 * bmq[j] + (lane >> 4) + 4 * e, jj = 16 * bnq[j] + (lane & 15);
            if (i >= Lx || jj >= Lx || jj > i) continue;
            const double v = acc[j][e];
            if (i < L) {
                M[(size_t)i * L + jj] = v;
                M[(size_t)jj * L + i] = v;
            } else if (jj < L) {
                bv[jj] = v;
            } else {
                es[s] = v;
            }
        }
    }
    if (tid == 0) {
        npix_out[s] = npix;
        flags_out[s] = 0;
    }
}

FitArgs base_fit_args(const psfm_context* ctx) {
    FitArgs a{};
    a.r = ctx->r;
    a.nbands = psfm::fit_bands(ctx);
    a.fac = ctx->fac;
    a.rowf = ctx->term_rowf;
    a.colf = ctx->term_colf;
    a.psi = ctx->term_psi;
    a.zf = ctx->term_z;
    a.nb = ctx->nb;
    a.nf = ctx->nf;
    a.wmode = ctx->cfg.weight_mode;
    return a;
}

template <int H_, int BR>
int set_fit_lds(size_t lds) {
    static size_t granted = 0;      // dynamic LDS granted so far (all forms)
    if (lds > granted) {
        PSFM_HIP_CHECK(hipFuncSetAttribute((const void*)k_fit_band<H_, PSFM_PREC_FP32, BR>,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
        PSFM_HIP_CHECK(hipFuncSetAttribute((const void*)k_fit_band<H_, PSFM_PREC_FP16, BR>,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
        PSFM_HIP_CHECK(hipFuncSetAttribute((const void*)k_fit_band<H_, PSFM_PREC_BF16, BR>,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
        PSFM_HIP_CHECK(hipFuncSetAttribute((const void*)k_fit_band_b<H_, BR>,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
        PSFM_HIP_CHECK(hipFuncSetAttribute((const void*)k_fit_band<H_, PREC_DESIGN, BR>,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
        granted = lds;
    }
    return PSFM_OK;
}

// The band height is a compile-time constant of the kernels (the column
// pass keeps one accumulator per band row in registers); the context picks
// one of the instantiated heights.
template <int H_>
int set_fit_lds_ctx(const psfm_context* ctx, size_t lds) {
    switch (ctx->fit_br) {
        case PSFM_FIT_BR_SHORT: return set_fit_lds<H_, PSFM_FIT_BR_SHORT>(lds);
        case PSFM_FIT_BR_MID: return set_fit_lds<H_, PSFM_FIT_BR_MID>(lds);
        default: return set_fit_lds<H_, PSFM_FIT_BR_TALL>(lds);
    }
}

template <int H_, int BR>
int launch_fit_br(const psfm_context* ctx, const FitArgs& a, int n_items, const PairDesc* pairs,
                  const int* item_pair, int prec, hipStream_t st) {
    const FitLds Lo = fit_lds_layout(H_, ctx->r, ctx->nb, ctx->nf, BR,
                                     prec == PSFM_PREC_BF16 && !pairs);
    const size_t lds = (size_t)Lo.total * sizeof(float);
    int rc = set_fit_lds<H_, BR>(lds);
    if (rc) return rc;
    if (prec == PREC_DESIGN)
        hipLaunchKernelGGL((k_fit_band<H_, PREC_DESIGN, BR>), dim3(n_items), dim3(256), lds, st, a);
    else if (pairs)
        hipLaunchKernelGGL((k_fit_band_b<H_, BR>), dim3(n_items), dim3(256), lds, st, pairs, item_pair, a);
    else if (prec == PSFM_PREC_FP16)
        hipLaunchKernelGGL((k_fit_band<H_, PSFM_PREC_FP16, BR>), dim3(n_items), dim3(256), lds, st, a);
    else if (prec == PSFM_PREC_BF16)
        hipLaunchKernelGGL((k_fit_band<H_, PSFM_PREC_BF16, BR>), dim3(n_items), dim3(256), lds, st, a);
    else
        hipLaunchKernelGGL((k_fit_band<H_, PSFM_PREC_FP32, BR>), dim3(n_items), dim3(256), lds, st, a);
    PSFM_HIP_CHECK(hipGetLastError());
    return PSFM_OK;
}

template <int H_>
int launch_fit(const psfm_context* ctx, const FitArgs& a, int n_items, const PairDesc* pairs,
               const int* item_pair, int prec, hipStream_t st) {
    switch (ctx->fit_br) {
        case PSFM_FIT_BR_SHORT:
            return launch_fit_br<H_, PSFM_FIT_BR_SHORT>(ctx, a, n_items, pairs, item_pair, prec, st);
        case PSFM_FIT_BR_MID:
            return launch_fit_br<H_, PSFM_FIT_BR_MID>(ctx, a, n_items, pairs, item_pair, prec, st);
        default:
            return launch_fit_br<H_, PSFM_FIT_BR_TALL>(ctx, a, n_items, pairs, item_pair, prec, st);
    }
}

// prec: the context's precision, or PREC_DESIGN for a design-only pass.
int dispatch_fit(const psfm_context* ctx, const FitArgs& a, int n_items, const PairDesc* pairs,
                 const int* item_pair, hipStream_t st, int prec = -1) {
    if (prec < 0) prec = ctx->cfg.precision;
    switch (ctx->h) {
#define PSFM_FIT_CASE(HH) \
    case HH: return launch_fit<HH>(ctx, a, n_items, pairs, item_pair, prec, st);
        PSFM_FIT_CASE(1) PSFM_FIT_CASE(2) PSFM_FIT_CASE(3) PSFM_FIT_CASE(4) PSFM_FIT_CASE(5)
        PSFM_FIT_CASE(6) PSFM_FIT_CASE(7) PSFM_FIT_CASE(8) PSFM_FIT_CASE(9) PSFM_FIT_CASE(10)
        PSFM_FIT_CASE(11) PSFM_FIT_CASE(12) PSFM_FIT_CASE(13) PSFM_FIT_CASE(14) PSFM_FIT_CASE(15)
        PSFM_FIT_CASE(16)
#undef PSFM_FIT_CASE
        default: return PSFM_ERR_UNSUPPORTED;
    }
}

}  // namespace

namespace psfm {

size_t fit_lds_bytes(const psfm_context* ctx) {
    return (size_t)fit_lds_layout(ctx->h, ctx->r, ctx->nb, ctx->nf, ctx->fit_br,
                                  ctx->cfg.precision == PSFM_PREC_BF16).total * sizeof(float);
}

// Grants the fit kernels their dynamic LDS (done ahead of a graph capture).
int fit_prepare(const psfm_context* ctx) {
    const size_t lds = fit_lds_bytes(ctx);
    switch (ctx->h) {
#define PSFM_FIT_PREP(HH) \
    case HH: return set_fit_lds_ctx<HH>(ctx, lds);
        PSFM_FIT_PREP(1) PSFM_FIT_PREP(2) PSFM_FIT_PREP(3) PSFM_FIT_PREP(4) PSFM_FIT_PREP(5)
        PSFM_FIT_PREP(6) PSFM_FIT_PREP(7) PSFM_FIT_PREP(8) PSFM_FIT_PREP(9) PSFM_FIT_PREP(10)
        PSFM_FIT_PREP(11) PSFM_FIT_PREP(12) PSFM_FIT_PREP(13) PSFM_FIT_PREP(14) PSFM_FIT_PREP(15)
        PSFM_FIT_PREP(16)
#undef PSFM_FIT_PREP
        default: return PSFM_ERR_UNSUPPORTED;
    }
}

int batch_fit(const psfm_context* ctx, const PairDesc* pairs, const int* item_pair,
              const int* stamp_pair, int n_items, int n_stamps, hipStream_t st) {
    if (fit_lds_bytes(ctx) > 160 * 1024 - 1024) return PSFM_ERR_UNSUPPORTED;
    if (ctx->cfg.precision != PSFM_PREC_FP32) return PSFM_ERR_UNSUPPORTED;
    if (n_items == 0) return PSFM_OK;
    int rc = dispatch_fit(ctx, base_fit_args(ctx), n_items, pairs, item_pair, st);
    if (rc) return rc;
    const int npix = (2 * ctx->r + 1) * (2 * ctx->r + 1);
    hipLaunchKernelGGL(k_fit_reduce_b, dim3(n_stamps), dim3(256), 0, st, pairs,
                       stamp_pair, fit_bands(ctx), ctx->nb, npix);
    PSFM_HIP_CHECK(hipGetLastError());
    return PSFM_OK;
}

// The two-kernel fit: both designs and both passes' band flags.
size_t dual_fit_workspace(const psfm_context* ctx, int n_stamps) {
    Carver c(nullptr);
    const size_t npix = (size_t)(2 * ctx->r + 1) * (2 * ctx->r + 1);
    const size_t nbl = (size_t)n_stamps * fit_bands(ctx);
    c.take<float>((size_t)n_stamps * (ctx->nb + 2) * npix);
    c.take<float>((size_t)n_stamps * (ctx->nb + 2) * npix);
    c.take<int>(nbl);
    c.take<int>(nbl);
    return c.off;
}

size_t fit_workspace(const psfm_context* ctx, int n_stamps) {
    Carver c(nullptr);
    const size_t nbl = (size_t)n_stamps * fit_bands(ctx);
    c.take<double>(nbl * GC * GC);
    c.take<int>(nbl);
    return c.off;
}

}  // namespace psfm

extern "C" int psfm_fit_stamps(const psfm_context* ctx, const float* I1, const float* V1,
                               const uint8_t* M1, const float* I2, const float* V2,
                               const uint8_t* M2, int W, int H,
                               int64_t pitch, const int32_t* stamp_xy, int n_stamps,
                               double* stamp_M, double* stamp_b, double* stamp_e,
                               int32_t* stamp_npix, int32_t* stamp_flags, float* stamp_design,
                               void* ws, size_t ws_bytes, void* stream) {
    if (!ctx || n_stamps < 0) return PSFM_ERR_INVALID_ARG;
    if (ctx->cfg.precision != PSFM_PREC_FP32 && n_stamps > 0 && !stamp_design)
        return PSFM_ERR_INVALID_ARG;
    if (W < 1 || H < 1 || pitch < W) return PSFM_ERR_SHAPE;
    if (n_stamps == 0) return PSFM_OK;
    if (!I1 || !M1 || !I2 || !V2 || !M2 || !stamp_xy || !stamp_M || !stamp_b || !stamp_e ||
        !stamp_npix || !stamp_flags)
        return PSFM_ERR_INVALID_ARG;
    if (ctx->cfg.weight_mode == PSFM_WEIGHT_V1V2 && !V1) return PSFM_ERR_INVALID_ARG;
    if (psfm::fit_lds_bytes(ctx) > 160 * 1024 - 1024) return PSFM_ERR_UNSUPPORTED;
    const size_t need = psfm::fit_workspace(ctx, n_stamps);
    if (!ws || ws_bytes < need) return PSFM_ERR_WORKSPACE;
    hipStream_t st = (hipStream_t)stream;
    psfm::Carver c(ws);
    const size_t nbl = (size_t)n_stamps * psfm::fit_bands(ctx);
    double* part = c.take<double>(nbl * GC * GC);
    int* bflags = c.take<int>(nbl);
    FitArgs a = base_fit_args(ctx);
    a.I1 = I1;
    a.M1 = M1;
    a.I2 = I2;
    a.V2 = V2;
    a.M2 = M2;
    a.V1 = V1;
    a.W = W;
    a.H = H;
    a.pitch = pitch;
    a.xy = stamp_xy;
    a.part = part;
    a.band_flags = bflags;
    a.design = stamp_design;
    int rc = dispatch_fit(ctx, a, n_stamps * a.nbands, nullptr, nullptr, st);
    if (rc != PSFM_OK) return rc;
    const int npix = (2 * ctx->r + 1) * (2 * ctx->r + 1);
    hipLaunchKernelGGL(k_fit_reduce, dim3(n_stamps), dim3(256), 0, st, part, bflags,
                       psfm::fit_bands(ctx), ctx->nb, npix, stamp_M, stamp_b, stamp_e, stamp_npix,
                       stamp_flags);
    PSFM_HIP_CHECK(hipGetLastError());
    return PSFM_OK;
}

extern "C" int psfm_fit_dual(const psfm_context* ctx, const float* I1, const float* V1,
                             const uint8_t* M1, const float* I2, const float* V2,
                             const uint8_t* M2, int W, int H,
                             int64_t pitch, const int32_t* stamp_xy, int n_stamps, double* stamp_M,
                             double* stamp_b, double* stamp_e, int32_t* stamp_npix,
                             int32_t* stamp_flags, void* ws, size_t ws_bytes, void* stream) {
    if (!ctx || n_stamps < 0) return PSFM_ERR_INVALID_ARG;
    if (W < 1 || H < 1 || pitch < W) return PSFM_ERR_SHAPE;
    if (n_stamps == 0) return PSFM_OK;
    if (!I1 || !M1 || !I2 || !V2 || !M2 || !stamp_xy || !stamp_M || !stamp_b || !stamp_e ||
        !stamp_npix || !stamp_flags)
        return PSFM_ERR_INVALID_ARG;
    if (ctx->cfg.weight_mode == PSFM_WEIGHT_V1V2 && !V1) return PSFM_ERR_INVALID_ARG;
    if (2 * ctx->nb + 1 > GD_COLS) return PSFM_ERR_UNSUPPORTED;
    if (psfm::fit_lds_bytes(ctx) > 160 * 1024 - 1024) return PSFM_ERR_UNSUPPORTED;
    if (!ws || ws_bytes < psfm::dual_fit_workspace(ctx, n_stamps)) return PSFM_ERR_WORKSPACE;
    hipStream_t st = (hipStream_t)stream;
    const int npix = (2 * ctx->r + 1) * (2 * ctx->r + 1);
    const size_t dsz = (size_t)n_stamps * (ctx->nb + 2) * npix;
    psfm::Carver c(ws);
    float* d1 = c.take<float>(dsz);
    float* d2 = c.take<float>(dsz);
    const size_t nbl = (size_t)n_stamps * psfm::fit_bands(ctx);
    int* bf1 = c.take<int>(nbl);
    int* bf2 = c.take<int>(nbl);
    FitArgs a = base_fit_args(ctx);
    a.I1 = I1;
    a.M1 = M1;
    a.I2 = I2;
    a.V2 = V2;
    a.M2 = M2;
    a.V1 = V1;
    a.W = W;
    a.H = H;
    a.pitch = pitch;
    a.xy = stamp_xy;
    a.part = nullptr;
    a.band_flags = bf1;
    a.design = d1;
    int rc = dispatch_fit(ctx, a, n_stamps * a.nbands, nullptr, nullptr, st, PREC_DESIGN);
    if (rc != PSFM_OK) return rc;
    // the I2 columns: the same pass with I2 (and its mask) as the convolved image
    a.I1 = I2;
    a.M1 = M2;
    a.band_flags = bf2;
    a.design = d2;
    rc = dispatch_fit(ctx, a, n_stamps * a.nbands, nullptr, nullptr, st, PREC_DESIGN);
    if (rc != PSFM_OK) return rc;
    hipLaunchKernelGGL(k_gram_dual, dim3(n_stamps), dim3(256), 0, st, d1, d2, bf1, bf2, a.nbands, ctx->nb,
                       npix, stamp_M, stamp_b, stamp_e, stamp_npix, stamp_flags);
    PSFM_HIP_CHECK(hipGetLastError());
    return PSFM_OK;
}
