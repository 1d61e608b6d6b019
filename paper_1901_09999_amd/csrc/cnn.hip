// Stamp-pair CNN: forward, MSE gradient and Adam, FP16 weights and
// activations with FP32 accumulation (the learned warm start / rejection
// prior of the kernel fit).
//
// Network (NCHW, one sample = the reference and target 41 x 41 stamps):
//   conv1 3x3 2->32 s1, conv2..4 3x3 32->32 s2 (zero padding 1, ReLU):
//   41 -> 41 -> 21 -> 11 -> 6;  fc1 1152 -> 128 ReLU;  fc2 128 -> 49.
// A convolution is the cross-correlation
//   y[b,o,i,j] = bias[o] + sum_{c,u,v} w[o,c,u,v] x[b,c, s i+u-1, s j+v-1].
//
// Kernels (FP32 accumulation):
//   k_conv_fwd       first layer (2 input channels): one thread per output
//                    pixel, all 32 output channels in registers, the weights
//                    in LDS ordered [c][uv][o] (8 broadcast 16-byte words per
//                    input value);
//   k_conv_fwd_mfma  the 32 -> 32 layers: implicit GEMM on FP16 MFMA (below);
//   k_conv_bwd_data_mfma  the data gradients of the 32 -> 32 layers per
//                    stride-2 parity class on BF16 MFMA (hi + lo parts, below),
//                    the ReLU mask of the layer below applied on the way out;
//   k_conv_bwd_w_gemm  32 -> 32 layers: the weight gradients as a GEMM over
//                    the pixels, chunks of output gradients and input patches
//                    staged in LDS, 4 x 9 sums per thread, a partial set per
//                    workgroup;
//   k_conv_bwd_w     first layer (2 input channels): one workgroup per (group
//                    of 8 output channels, c) and batch chunk;
//   k_conv_bwd_w_sum adds the partial sets in a fixed order;
//   k_fc_fwd_mfma  the first fully connected layer on FP16 MFMA (below);
//   k_fc_fwd / k_fc_bwd_x / k_fc_bwd_w, k_mse, k_adam.
// The backward pass stores activation gradients in FP32.
#include "internal.h"

#include <hip/hip_fp16.h>

namespace {

constexpr int SIDE0 = PSFM_CNN_SIDE, CH = 32, HID = 128, NOUT = PSFM_CNN_OUT;
constexpr int SIDE1 = 41, SIDE2 = 21, SIDE3 = 11, SIDE4 = 6;
constexpr int FLAT = CH * SIDE4 * SIDE4;

// parameter offsets (elements), in the order conv1.w, conv1.b, ..., fc2.b
constexpr int OFF_C1W = 0, OFF_C1B = OFF_C1W + CH * 2 * 9;
constexpr int OFF_C2W = OFF_C1B + CH, OFF_C2B = OFF_C2W + CH * CH * 9;
constexpr int OFF_C3W = OFF_C2B + CH, OFF_C3B = OFF_C3W + CH * CH * 9;
constexpr int OFF_C4W = OFF_C3B + CH, OFF_C4B = OFF_C4W + CH * CH * 9;
constexpr int OFF_F1W = OFF_C4B + CH, OFF_F1B = OFF_F1W + HID * FLAT;
constexpr int OFF_F2W = OFF_F1B + HID, OFF_F2B = OFF_F2W + NOUT * HID;
constexpr int NPARAM = OFF_F2B + NOUT;

__device__ __forceinline__ float h2f(__half v) { return __half2float(v); }

template <int CIN, int S>
__global__ __launch_bounds__(256) void k_conv_fwd(const __half* __restrict__ x, int Hin,
                                                  const __half* __restrict__ w,
                                                  const __half* __restrict__ bias,
                                                  __half* __restrict__ y, int Hout, int B) {
    __shared__ __align__(16) float ws[CIN * 9 * CH];     // [c][uv][o]
    __shared__ float bs[CH];
    for (int e = threadIdx.x; e < CIN * 9 * CH; e += 256) {
        const int o = e % CH, cuv = e / CH;               // cuv = c * 9 + uv
        ws[e] = h2f(w[o * CIN * 9 + cuv]);
    }
    if (threadIdx.x < CH) bs[threadIdx.x] = h2f(bias[threadIdx.x]);
    __syncthreads();
    const int npix = Hout * Hout;
    for (int t = blockIdx.x * 256 + threadIdx.x; t < B * npix; t += gridDim.x * 256) {
        const int b = t / npix, p = t - b * npix;
        const int i = p / Hout, j = p - i * Hout;
        float acc[CH];
#pragma unroll
        for (int o = 0; o < CH; o++) acc[o] = bs[o];
        for (int c = 0; c < CIN; c++) {
            const __half* xc = x + ((size_t)b * CIN + c) * Hin * Hin;
#pragma unroll
            for (int u = 0; u < 3; u++) {
                const int pi = S * i + u - 1;
#pragma unroll
                for (int v = 0; v < 3; v++) {
                    const int qj = S * j + v - 1;
                    if (pi < 0 || pi >= Hin || qj < 0 || qj >= Hin) continue;
                    const float xv = h2f(xc[pi * Hin + qj]);
                    const float4* wr = reinterpret_cast<const float4*>(ws + (c * 9 + u * 3 + v) * CH);
#pragma unroll
                    for (int q = 0; q < CH / 4; q++) {
                        const float4 ww = wr[q];
                        acc[4 * q] = fmaf(ww.x, xv, acc[4 * q]);
                        acc[4 * q + 1] = fmaf(ww.y, xv, acc[4 * q + 1]);
                        acc[4 * q + 2] = fmaf(ww.z, xv, acc[4 * q + 2]);
                        acc[4 * q + 3] = fmaf(ww.w, xv, acc[4 * q + 3]);
                    }
                }
            }
        }
#pragma unroll
        for (int o = 0; o < CH; o++)
            y[(((size_t)b * CH + o) * Hout + i) * Hout + j] = __float2half(fmaxf(acc[o], 0.0f));
    }
}

typedef _Float16 cnn_half8 __attribute__((ext_vector_type(8)));
typedef float cnn_floatx4 __attribute__((ext_vector_type(4)));

// The 32 -> 32 layers (3 x 3, stride 2, zero padding 1) as the implicit GEMM
// Y[pixel][o] = sum over k = (u, v, c) of X[pixel][k] W[k][o] on
// v_mfma_f32_16x16x32_f16 (FP16 products exact, FP32 sums), k in nine
// chunks of 32 channels, one tap (u, v) each.  One workgroup per (sample,
// band of R output rows): the weights first pass through LDS into registers
// (the B operands of a tile's 18 products: 9 taps x 2 blocks of 16 output
// channels), then the band's 2R + 1 input rows fill the same LDS as
// [row][col][channel] with a zero border (40 halves per pixel: the 16-byte
// reads stay 16-byte aligned, and those of 16 output pixels two columns
// apart meet at most two to a bank); each wave takes tiles of 16 output
// pixels.  y = ReLU(sum + bias) in FP16.
template <int HIN, int HOUT, int R>
__global__ __launch_bounds__(256) void k_conv_fwd_mfma(const __half* __restrict__ x,
                                                       const __half* __restrict__ w,
                                                       const __half* __restrict__ bias,
                                                       __half* __restrict__ y) {
    static_assert(HOUT == (HIN + 1) / 2, "stride 2, padding 1");
    constexpr int WT = HIN + 2;             // tile columns: input columns -1 .. HIN
    constexpr int RT = 2 * R + 1;           // tile rows: input rows 2 i0 - 1 .. 2 i0 + 2 R - 1
    constexpr int PS = 40;                  // halves per tile pixel (80 bytes)
    constexpr int PW = 40;                  // halves per (tap, output channel) of the weights
    constexpr int NBAND = (HOUT + R - 1) / R;
    constexpr int XS = RT * WT * PS, WS = 9 * CH * PW, NSH = XS > WS ? XS : WS;
    static_assert(XS % 8 == 0 && NSH % 8 == 0, "whole 16-byte words");
    __shared__ __align__(16) __half sh[NSH];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int b = blockIdx.x / NBAND, i0 = (blockIdx.x - b * NBAND) * R;
    // weights [o][c][u][v] -> LDS [uv][o][c] -> registers
    for (int e = tid; e < CH * CH * 9; e += 256) {
        const int o = e / (CH * 9), rem = e - o * (CH * 9), c = rem / 9, uv = rem - 9 * c;
        sh[(uv * CH + o) * PW + c] = w[e];
    }
    __syncthreads();
    cnn_half8 bw[9][2];
#pragma unroll
    for (int uv = 0; uv < 9; uv++)
#pragma unroll
        for (int k = 0; k < 2; k++)
            bw[uv][k] = *reinterpret_cast<const cnn_half8*>(sh + (uv * CH + 16 * k + (lane & 15)) * PW +
                                                            8 * (lane >> 4));
    const float b0 = h2f(bias[lane & 15]), b1 = h2f(bias[16 + (lane & 15)]);
    __syncthreads();
    // the band's input rows, zero outside the input
    for (int e = tid; e < XS / 8; e += 256) reinterpret_cast<uint4*>(sh)[e] = make_uint4(0u, 0u, 0u, 0u);
    __syncthreads();
    const int r_lo = 2 * i0 - 1;
    for (int e = tid; e < CH * RT * HIN; e += 256) {
        const int c = e / (RT * HIN), rem = e - c * (RT * HIN), lr = rem / HIN, col = rem - lr * HIN;
        const int gr = r_lo + lr;
        if (gr >= 0 && gr < HIN) sh[(lr * WT + col + 1) * PS + c] = x[(((size_t)b * CH + c) * HIN + gr) * HIN + col];
    }
    __syncthreads();
    const int npx = min(R, HOUT - i0) * HOUT;
    for (int t = wave; 16 * t < npx; t += 4) {
        const int m = 16 * t + (lane & 15);
        const bool valid = m < npx;
        const int mi = valid ? m / HOUT : 0, mj = valid ? m - mi * HOUT : 0;
        cnn_floatx4 acc0 = {0.0f, 0.0f, 0.0f, 0.0f}, acc1 = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
        for (int uv = 0; uv < 9; uv++) {
            const int u = uv / 3, v = uv - 3 * u;
            cnn_half8 a = *reinterpret_cast<const cnn_half8*>(sh + ((2 * mi + u) * WT + 2 * mj + v) * PS +
                                                             8 * (lane >> 4));
            if (!valid) a = cnn_half8{0, 0, 0, 0, 0, 0, 0, 0};
            acc0 = __builtin_amdgcn_mfma_f32_16x16x32_f16(a, bw[uv][0], acc0, 0, 0, 0);
            acc1 = __builtin_amdgcn_mfma_f32_16x16x32_f16(a, bw[uv][1], acc1, 0, 0, 0);
        }
        // lane: output channels lane % 16 and 16 + lane % 16 of pixels 4 (lane / 16) + e
#pragma unroll
        for (int e = 0; e < 4; e++) {
            const int mm = 16 * t + 4 * (lane >> 4) + e;
            if (mm < npx) {
                const int i = i0 + mm / HOUT, j = mm % HOUT;
                const size_t o0 = (((size_t)b * CH + (lane & 15)) * HOUT + i) * HOUT + j;
                y[o0] = __float2half(fmaxf(acc0[e] + b0, 0.0f));
                y[o0 + (size_t)16 * HOUT * HOUT] = __float2half(fmaxf(acc1[e] + b1, 0.0f));
            }
        }
    }
}

// The first fully connected layer, h = ReLU(W x + bias) in FP16, as a GEMM
// on v_mfma_f32_16x16x32_f16 (FP16 products exact, FP32 sums).  One
// workgroup per 16 x 16 tile of (sample, hidden unit); its four waves take
// a quarter of the inputs each, reading the k-contiguous rows of x and W
// straight from global memory in 16-byte pieces (both 16-byte aligned), and
// the four partial tiles are summed in a fixed order through LDS.  Samples
// past B (a ragged last tile) take zero operands and are not written.
template <int K>
__global__ __launch_bounds__(256) void k_fc_fwd_mfma(const __half* __restrict__ x,
                                                     const __half* __restrict__ W,
                                                     const __half* __restrict__ bias, int N, int B,
                                                     __half* __restrict__ y) {
    static_assert(K % 128 == 0, "four waves of 32-wide k steps");
    constexpr int KQ = K / 4;
    __shared__ float part[3][4][64];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int nt = N / 16, tb = blockIdx.x / nt, tn = blockIdx.x - tb * nt;
    const int b = 16 * tb + (lane & 15), n = 16 * tn + (lane & 15);
    const bool bval = b < B;
    const int k0 = wave * KQ + 8 * (lane >> 4);
    const __half* xr = x + (size_t)(bval ? b : 0) * K + k0;
    const __half* wr = W + (size_t)n * K + k0;
    cnn_floatx4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int k = 0; k < KQ; k += 32) {
        const cnn_half8 a = bval ? *reinterpret_cast<const cnn_half8*>(xr + k)
                                 : cnn_half8{0, 0, 0, 0, 0, 0, 0, 0};
        const cnn_half8 w = *reinterpret_cast<const cnn_half8*>(wr + k);
        acc = __builtin_amdgcn_mfma_f32_16x16x32_f16(a, w, acc, 0, 0, 0);
    }
    if (wave > 0)
#pragma unroll
        for (int e = 0; e < 4; e++) part[wave - 1][e][lane] = acc[e];
    __syncthreads();
    if (wave == 0) {
        const float bn = h2f(bias[n]);
        // lane: hidden unit n of samples 16 tb + 4 (lane / 16) + e
#pragma unroll
        for (int e = 0; e < 4; e++) {
            const int bb = 16 * tb + 4 * (lane >> 4) + e;
            const float s = ((acc[e] + part[0][e][lane]) + part[1][e][lane]) + part[2][e][lane];
            if (bb < B) y[(size_t)bb * N + n] = __float2half(fmaxf(s + bn, 0.0f));
        }
    }
}

typedef __bf16 cnn_bf16x8 __attribute__((ext_vector_type(8)));

// The data gradient of a 32 -> 32 layer (3 x 3, stride 2, padding 1, odd
// input side) on v_mfma_f32_16x16x32_bf16.  For an input pixel of parity
// (p mod 2, q mod 2) the taps that reach it are fixed: u = 1 for even p, u in
// {0, 2} for odd p (likewise v), i = (p + 1 - u) / 2, j = (q + 1 - v) / 2, all
// inside the output for an odd side.  So each parity class is a GEMM
// dX[pixel][c] = sum over (tap, o) of dY[i, j][o] W[o][c][tap], K = 32 per
// tap.  The FP32 dY and the FP16 weights enter as BF16 hi + lo parts (the
// weights exactly, dY to 16 bits); the three products hi hi, hi lo, lo hi
// have FP32 sums.  One workgroup per (sample, band of RB input rows): the
// weights ([tap][c][o]) and the band's dY rows ([i][j][o]) in LDS with
// 80-byte rows; each wave takes tiles of 16 pixels of one class and forms both
// 16-channel blocks; dxm = dx * (a > 0).
template <int HIN, int HOUT, int RB>
__global__ __launch_bounds__(256) void k_conv_bwd_data_mfma(const float* __restrict__ dy,
                                                            const __half* __restrict__ w,
                                                            const __half* __restrict__ a,
                                                            float* __restrict__ dxm) {
    static_assert(HIN % 2 == 1 && HOUT == (HIN + 1) / 2, "stride 2, padding 1, odd side");
    constexpr int PW = 40;                                   // halves per LDS row
    constexpr int NRMAX = RB / 2 + 2;                        // dY rows of a band
    constexpr int NBAND = (HIN + RB - 1) / RB;
    constexpr int WSZ = 9 * CH * PW, DSZ = NRMAX * HOUT * PW;
    __shared__ __align__(16) unsigned short wh[WSZ], wl[WSZ], dh[DSZ], dl[DSZ];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int b = blockIdx.x / NBAND, p0 = (blockIdx.x - b * NBAND) * RB, p1 = min(p0 + RB, HIN);
    const int i_lo = max(0, (p0 - 1) >> 1), i_hi = p1 >> 1;   // dY rows the band reaches
    auto hi_lo = [](float v, unsigned short& h, unsigned short& l) {
        const __bf16 bh = (__bf16)v;
        h = __builtin_bit_cast(unsigned short, bh);
        l = __builtin_bit_cast(unsigned short, (__bf16)(v - (float)bh));
    };
    for (int e = tid; e < CH * CH * 9; e += 256) {
        const int o = e / (CH * 9), rem = e - o * (CH * 9), c = rem / 9, uv = rem - 9 * c;
        hi_lo(h2f(w[e]), wh[(uv * CH + c) * PW + o], wl[(uv * CH + c) * PW + o]);
    }
    const int nr = i_hi - i_lo + 1;
    for (int e = tid; e < CH * nr * HOUT; e += 256) {
        const int o = e / (nr * HOUT), rem = e - o * (nr * HOUT), r = rem / HOUT, j = rem - r * HOUT;
        const float v = dy[(((size_t)b * CH + o) * HOUT + i_lo + r) * HOUT + j];
        hi_lo(v, dh[(r * HOUT + j) * PW + o], dl[(r * HOUT + j) * PW + o]);
    }
    __syncthreads();
    // the band's pixels in four parity classes (rp, rq), each row-major
    int cnt[4], first[4], ncol[4];
#pragma unroll
    for (int k = 0; k < 4; k++) {
        const int rp = k >> 1, rq = k & 1;
        first[k] = p0 + (((p0 & 1) != rp) ? 1 : 0);
        const int nrow = first[k] < p1 ? (p1 - 1 - first[k]) / 2 + 1 : 0;
        ncol[k] = (HIN + 1 - rq) / 2;
        cnt[k] = nrow * ncol[k];
    }
    const int t1 = (cnt[0] + 15) / 16, t2 = t1 + (cnt[1] + 15) / 16, t3 = t2 + (cnt[2] + 15) / 16;
    const int ntile = t3 + (cnt[3] + 15) / 16;
    const int n = lane & 15, kq = lane >> 4;
    for (int t = wave; t < ntile; t += 4) {
        const int k = t < t1 ? 0 : t < t2 ? 1 : t < t3 ? 2 : 3;
        const int tl = t - (k == 0 ? 0 : k == 1 ? t1 : k == 2 ? t2 : t3);
        const int rp = k >> 1, rq = k & 1;
        const int m = 16 * tl + n;                       // A row: pixel of the class
        const bool valid = m < cnt[k];
        const int mr = valid ? m / ncol[k] : 0, mc = valid ? m - mr * ncol[k] : 0;
        const int p = first[k] + 2 * mr, q = rq + 2 * mc;
        cnn_floatx4 acc0 = {0.0f, 0.0f, 0.0f, 0.0f}, acc1 = {0.0f, 0.0f, 0.0f, 0.0f};
        for (int su = 0; su < (rp ? 2 : 1); su++) {
            const int u = rp ? 2 * su : 1;
            for (int sv = 0; sv < (rq ? 2 : 1); sv++) {
                const int v = rq ? 2 * sv : 1;
                const int r = (p + 1 - u) / 2 - i_lo, j = (q + 1 - v) / 2;
                const int ao = (r * HOUT + j) * PW + 8 * kq;
                cnn_bf16x8 ah = *reinterpret_cast<const cnn_bf16x8*>(dh + ao);
                cnn_bf16x8 al = *reinterpret_cast<const cnn_bf16x8*>(dl + ao);
                if (!valid) {
                    ah = cnn_bf16x8{};
                    al = cnn_bf16x8{};
                }
                const int uv = u * 3 + v;
                const int bo0 = (uv * CH + n) * PW + 8 * kq, bo1 = bo0 + 16 * PW;
                const cnn_bf16x8 bh0 = *reinterpret_cast<const cnn_bf16x8*>(wh + bo0);
                const cnn_bf16x8 bl0 = *reinterpret_cast<const cnn_bf16x8*>(wl + bo0);
                const cnn_bf16x8 bh1 = *reinterpret_cast<const cnn_bf16x8*>(wh + bo1);
                const cnn_bf16x8 bl1 = *reinterpret_cast<const cnn_bf16x8*>(wl + bo1);
                acc0 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bh0, acc0, 0, 0, 0);
                acc0 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bl0, acc0, 0, 0, 0);
                acc0 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, bh0, acc0, 0, 0, 0);
                acc1 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bh1, acc1, 0, 0, 0);
                acc1 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bl1, acc1, 0, 0, 0);
                acc1 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, bh1, acc1, 0, 0, 0);
            }
        }
        // lane: channels n and 16 + n of the class pixels 16 tl + 4 kq + e
#pragma unroll
        for (int e = 0; e < 4; e++) {
            const int mm = 16 * tl + 4 * kq + e;
            if (mm < cnt[k]) {
                const int rr = mm / ncol[k], cc = mm - rr * ncol[k];
                const int pp = first[k] + 2 * rr, qq = rq + 2 * cc;
                const size_t o0 = (((size_t)b * CH + n) * HIN + pp) * HIN + qq;
                const size_t o1 = o0 + (size_t)16 * HIN * HIN;
                dxm[o0] = h2f(a[o0]) > 0.0f ? acc0[e] : 0.0f;
                dxm[o1] = h2f(a[o1]) > 0.0f ? acc1[e] : 0.0f;
            }
        }
    }
}

__device__ __forceinline__ float block_sum_f(float v, float* red) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) red[wave] = v;
    __syncthreads();
    float s = 0.0f;
    for (int k = 0; k < (int)(blockDim.x >> 6); k++) s += red[k];
    return s;
}

// dw[o,c,u,v] = sum_{b,i,j} dy[b,o,i,j] x[b,c,s i+u-1,s j+v-1]; db[o] = sum dy.
// One workgroup per (group of OG output channels, input channel c) and batch
// chunk: a pixel's nine input values serve OG outputs (OG x 9 sums per
// thread); the sums are reduced per wave by shuffles and then over the four
// waves in a fixed order.
template <int S, int OG>
__global__ __launch_bounds__(256) void k_conv_bwd_w(const float* __restrict__ dy, int Hout,
                                                    const __half* __restrict__ x, int CIN, int Hin,
                                                    int B, float* __restrict__ part) {
    constexpr int NV = OG * 9 + OG;                     // weight sums, then bias sums
    __shared__ float wred[4][NV];
    const int og = blockIdx.x / CIN, c = blockIdx.x % CIN;
    const int nsplit = gridDim.y, split = blockIdx.y;
    const int b0 = split * B / nsplit, b1 = (split + 1) * B / nsplit;
    float acc[NV];
#pragma unroll
    for (int k = 0; k < NV; k++) acc[k] = 0.0f;
    const int npix = Hout * Hout;
    for (int t = b0 * npix + threadIdx.x; t < b1 * npix; t += 256) {
        const int b = t / npix, pp = t - b * npix;
        const int i = pp / Hout, j = pp - i * Hout;
        float g[OG];
#pragma unroll
        for (int q = 0; q < OG; q++) g[q] = dy[((size_t)b * CH + og * OG + q) * npix + pp];
        const __half* xc = x + ((size_t)b * CIN + c) * Hin * Hin;
        // nine input loads, unconditional from clamped addresses (zero outside)
        float xv[9];
#pragma unroll
        for (int u = 0; u < 3; u++)
#pragma unroll
            for (int v = 0; v < 3; v++) {
                const int pi = S * i + u - 1, qj = S * j + v - 1;
                const bool in = pi >= 0 && pi < Hin && qj >= 0 && qj < Hin;
                const float xx = h2f(xc[in ? pi * Hin + qj : 0]);
                xv[u * 3 + v] = in ? xx : 0.0f;
            }
#pragma unroll
        for (int q = 0; q < OG; q++) {
#pragma unroll
            for (int k = 0; k < 9; k++) acc[q * 9 + k] = fmaf(g[q], xv[k], acc[q * 9 + k]);
            acc[OG * 9 + q] += g[q];
        }
    }
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < NV; k++) {
        float v = acc[k];
        for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
        if (lane == 0) wred[wave][k] = v;
    }
    __syncthreads();
    float* pw = part + (size_t)split * (CH * CIN * 9 + CH);
    for (int k = threadIdx.x; k < NV; k += 256) {
        const float sv = ((wred[0][k] + wred[1][k]) + wred[2][k]) + wred[3][k];
        if (k < OG * 9) pw[((og * OG + k / 9) * CIN + c) * 9 + k % 9] = sv;
        else if (c == 0) pw[CH * CIN * 9 + og * OG + (k - OG * 9)] = sv;
    }
}

// Weight and bias gradients of a 32 -> 32 layer as a GEMM over the pixels
// p = (b, i, j):  dW[o][(c,u,v)] = sum_p dy[p][o] X[p][(c,u,v)],  X the
// (zero-padded, strided) input patches.  Workgroup g stages chunks of WG_PIX
// pixels (g, g + G, ...) of dy and X in LDS; thread (ob, c) accumulates the
// 4 x 9 sums of outputs 4 ob .. 4 ob + 3 and input channel c (the bias sums
// ride with c = 0).  Partials per workgroup, (CH * CH * 9 + CH) floats each.
constexpr int WG_PIX = 32;
constexpr int WG_MAXG = 768;
template <int S>
__global__ __launch_bounds__(256) void k_conv_bwd_w_gemm(const float* __restrict__ dy, int Hout,
                                                         const __half* __restrict__ x, int Hin, int B,
                                                         float* __restrict__ part) {
    __shared__ float sdy[WG_PIX][CH + 1];
    __shared__ float sx[WG_PIX][CH * 9 + 1];
    __shared__ int sb[WG_PIX], spp[WG_PIX], si[WG_PIX], sj[WG_PIX];
    const int tid = threadIdx.x, ob = tid >> 5, c = tid & 31;
    const int npix = Hout * Hout, NP = B * npix, nch = (NP + WG_PIX - 1) / WG_PIX;
    float acc[4][9], accb[4];
#pragma unroll
    for (int a = 0; a < 4; a++) {
        accb[a] = 0.0f;
#pragma unroll
        for (int k = 0; k < 9; k++) acc[a][k] = 0.0f;
    }
    for (int q = blockIdx.x; q < nch; q += gridDim.x) {
        const int p0 = q * WG_PIX;
        // the chunk's pixels (b, i, j), decoded once (b = -1 past the end)
        if (tid < WG_PIX) {
            const int pg = p0 + tid, b = pg / npix, pp = pg - b * npix, i = pp / Hout;
            sb[tid] = pg < NP ? b : -1;
            spp[tid] = pp;
            si[tid] = i;
            sj[tid] = pp - i * Hout;
        }
        __syncthreads();
        // stage dy (WG_PIX x CH) and the patches (WG_PIX x CH*9); loads from
        // clamped addresses, zero outside the chunk or the input; the patch
        // values in batches of XB loads in flight (each then stored), which
        // keeps the registers of two waves per SIMD
        constexpr int ND = WG_PIX * CH / 256, NX = WG_PIX * CH * 9 / 256, XB = 12;
        static_assert(NX % XB == 0, "whole batches");
        float dv[ND];
#pragma unroll
        for (int k = 0; k < ND; k++) {
            const int e = tid + 256 * k, pl = e % WG_PIX, o = e / WG_PIX;
            const int b = sb[pl];
            dv[k] = dy[b >= 0 ? ((size_t)b * CH + o) * npix + spp[pl] : 0];
        }
#pragma unroll
        for (int k = 0; k < ND; k++) {
            const int e = tid + 256 * k, pl = e % WG_PIX, o = e / WG_PIX;
            sdy[pl][o] = sb[pl] >= 0 ? dv[k] : 0.0f;
        }
#pragma unroll 1
        for (int k0 = 0; k0 < NX; k0 += XB) {
            __half xh[XB];
#pragma unroll
            for (int kk = 0; kk < XB; kk++) {
                const int e = tid + 256 * (k0 + kk), pl = e % WG_PIX, cuv = e / WG_PIX;
                const int cc = cuv / 9, uv = cuv - 9 * cc, u = uv / 3, v = uv - 3 * u;
                const int b = sb[pl];
                const int pi = S * si[pl] + u - 1, qj = S * sj[pl] + v - 1;
                const bool in = b >= 0 && pi >= 0 && pi < Hin && qj >= 0 && qj < Hin;
                xh[kk] = x[in ? ((size_t)b * CH + cc) * Hin * Hin + pi * Hin + qj : 0];
            }
#pragma unroll
            for (int kk = 0; kk < XB; kk++) {
                const int e = tid + 256 * (k0 + kk), pl = e % WG_PIX, cuv = e / WG_PIX;
                const int cc = cuv / 9, uv = cuv - 9 * cc, u = uv / 3, v = uv - 3 * u;
                const int pi = S * si[pl] + u - 1, qj = S * sj[pl] + v - 1;
                const bool in = sb[pl] >= 0 && pi >= 0 && pi < Hin && qj >= 0 && qj < Hin;
                sx[pl][cuv] = in ? h2f(xh[kk]) : 0.0f;
            }
        }
        __syncthreads();
#pragma unroll 4
        for (int pl = 0; pl < WG_PIX; pl++) {
            float g[4], xv[9];
#pragma unroll
            for (int a = 0; a < 4; a++) g[a] = sdy[pl][4 * ob + a];
#pragma unroll
            for (int k = 0; k < 9; k++) xv[k] = sx[pl][c * 9 + k];
#pragma unroll
            for (int a = 0; a < 4; a++) {
                accb[a] += g[a];
#pragma unroll
                for (int k = 0; k < 9; k++) acc[a][k] = fmaf(g[a], xv[k], acc[a][k]);
            }
        }
        __syncthreads();
    }
    float* pw = part + (size_t)blockIdx.x * (CH * CH * 9 + CH);
#pragma unroll
    for (int a = 0; a < 4; a++) {
        const int o = 4 * ob + a;
#pragma unroll
        for (int k = 0; k < 9; k++) pw[(o * CH + c) * 9 + k] = acc[a][k];
        if (c == 0) pw[CH * CH * 9 + o] = accb[a];
    }
}

// dw = sum of the nsplit partial sets of the weight-gradient kernels: 64
// outputs per workgroup, each summed by WSUM_GROUPS thread groups over fixed
// ranges of the sets (two accumulators each), the group sums added in order.
constexpr int WSUM_GROUPS = 16;

__global__ __launch_bounds__(64 * WSUM_GROUPS) void k_conv_bwd_w_sum(const float* __restrict__ part,
                                                                     int nsplit, int nw,
                                                                     float* __restrict__ dw,
                                                                     float* __restrict__ db) {
    __shared__ float gs[WSUM_GROUPS][64];
    const int l = threadIdx.x & 63, grp = threadIdx.x >> 6;
    const int t = blockIdx.x * 64 + l;
    const int k0 = grp * nsplit / WSUM_GROUPS, k1 = (grp + 1) * nsplit / WSUM_GROUPS;
    float s0 = 0.0f, s1 = 0.0f;
    if (t < nw + CH) {
        int k = k0;
        for (; k + 1 < k1; k += 2) {
            s0 += part[(size_t)k * (nw + CH) + t];
            s1 += part[(size_t)(k + 1) * (nw + CH) + t];
        }
        if (k < k1) s0 += part[(size_t)k * (nw + CH) + t];
    }
    gs[grp][l] = s0 + s1;
    __syncthreads();
    if (grp == 0 && t < nw + CH) {
        float s = gs[0][l];
        for (int g = 1; g < WSUM_GROUPS; g++) s += gs[g][l];
        if (t < nw) dw[t] = s;
        else db[t - nw] = s;
    }
}

// y[b,n] = bias[n] + sum_k W[n,k] x[b,k]  (ReLU -> FP16 out, or FP32 out)
template <bool RELU>
__global__ __launch_bounds__(256) void k_fc_fwd(const __half* __restrict__ x, int K,
                                                const __half* __restrict__ W,
                                                const __half* __restrict__ bias, int N, int B,
                                                __half* __restrict__ y16, float* __restrict__ y32) {
    // one wave per output: the lanes stride over k (coalesced rows of x and
    // W), then a fixed-order shuffle sum
    const int t = blockIdx.x * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
    if (t >= B * N) return;
    const int b = t / N, n = t - b * N;
    const __half* xr = x + (size_t)b * K;
    const __half* wr = W + (size_t)n * K;
    float acc = 0.0f;
    for (int k = lane; k < K; k += 64) acc = fmaf(h2f(wr[k]), h2f(xr[k]), acc);
    for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o);
    acc += h2f(bias[n]);
    if (lane == 0) {
        if (RELU) y16[t] = __float2half(fmaxf(acc, 0.0f));
        else y32[t] = acc;
    }
}

// dxm[b,k] = (sum_n W[n,k] dy[b,n]) * (x[b,k] > 0).  Lane l of a workgroup
// takes output 64 blockIdx.x + l (coalesced rows of W, dy broadcast); its
// four waves take a quarter of the n each (two running sums over alternate
// n), and the quarters are added in a fixed order through LDS.
__global__ __launch_bounds__(256) void k_fc_bwd_x(const float* __restrict__ dy, int N,
                                                  const __half* __restrict__ W,
                                                  const __half* __restrict__ x, int K, int B,
                                                  float* __restrict__ dxm) {
    __shared__ float pd[3][64];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int t = blockIdx.x * 64 + lane;
    const int q = (N + 3) / 4, n0 = min(N, wave * q), n1 = min(N, n0 + q);
    float acc = 0.0f;
    if (t < B * K) {
        const int b = t / K, k = t - b * K;
        const float* dyr = dy + (size_t)b * N;
        float a0 = 0.0f, a1 = 0.0f;
        int n = n0;
#pragma unroll 4
        for (; n + 1 < n1; n += 2) {
            a0 = fmaf(h2f(W[(size_t)n * K + k]), dyr[n], a0);
            a1 = fmaf(h2f(W[(size_t)(n + 1) * K + k]), dyr[n + 1], a1);
        }
        if (n < n1) a0 = fmaf(h2f(W[(size_t)n * K + k]), dyr[n], a0);
        acc = a0 + a1;
    }
    if (wave > 0) pd[wave - 1][lane] = acc;
    __syncthreads();
    if (wave == 0 && t < B * K) {
        const float s = ((acc + pd[0][lane]) + pd[1][lane]) + pd[2][lane];
        dxm[t] = h2f(x[t]) > 0.0f ? s : 0.0f;
    }
}

// dW[n,k] = sum_b dy[b,n] x[b,k];  db[n] = sum_b dy[b,n].  Lane l of a
// workgroup takes output 64 blockIdx.x + l (coalesced rows of x, dy
// broadcast); its four waves take a quarter of the samples each (four running
// sums over every fourth sample, so four loads are in flight), and the
// quarters are added in a fixed order through LDS.
__global__ __launch_bounds__(256) void k_fc_bwd_w(const float* __restrict__ dy, int N,
                                                  const __half* __restrict__ x, int K, int B,
                                                  float* __restrict__ dW, float* __restrict__ db) {
    __shared__ float pw[3][64], pb[3][64];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int t = blockIdx.x * 64 + lane;
    const int q = (B + 3) / 4, b0 = min(B, wave * q), b1 = min(B, b0 + q);
    float w = 0.0f, bsum = 0.0f;
    if (t < N * K) {
        const int n = t / K, k = t - n * K;
        float a4[4] = {0.0f, 0.0f, 0.0f, 0.0f};
        int b = b0;
#pragma unroll 4
        for (; b + 3 < b1; b += 4)
#pragma unroll
            for (int u = 0; u < 4; u++)
                a4[u] = fmaf(dy[(size_t)(b + u) * N + n], h2f(x[(size_t)(b + u) * K + k]), a4[u]);
        for (; b < b1; b++) a4[0] = fmaf(dy[(size_t)b * N + n], h2f(x[(size_t)b * K + k]), a4[0]);
        w = (a4[0] + a4[1]) + (a4[2] + a4[3]);
        if (t < N)
            for (int bb = b0; bb < b1; bb++) bsum += dy[(size_t)bb * N + t];
    }
    if (wave > 0) {
        pw[wave - 1][lane] = w;
        pb[wave - 1][lane] = bsum;
    }
    __syncthreads();
    if (wave == 0 && t < N * K) {
        dW[t] = ((w + pw[0][lane]) + pw[1][lane]) + pw[2][lane];
        if (t < N) db[t] = ((bsum + pb[0][lane]) + pb[1][lane]) + pb[2][lane];
    }
}

// Weighted loss per sample b (one wave): r = out_b - target_b, u = W_b r,
// part_b = r^T u, dout_b = 2 u / count.
__global__ __launch_bounds__(64) void k_wloss(const float* __restrict__ out,
                                              const float* __restrict__ target,
                                              const float* __restrict__ W, int count,
                                              float* __restrict__ dout, float* __restrict__ part) {
    __shared__ float r[64];
    const int b = blockIdx.x, i = threadIdx.x;
    if (i < NOUT) r[i] = out[b * NOUT + i] - target[b * NOUT + i];
    __syncthreads();
    float p = 0.0f;
    if (i < NOUT) {
        const float* Wr = W + ((size_t)b * NOUT + i) * NOUT;
        float u = 0.0f;
        for (int j = 0; j < NOUT; j++) u = fmaf(Wr[j], r[j], u);
        dout[b * NOUT + i] = 2.0f * u / (float)count;
        p = r[i] * u;
    }
    for (int o = 32; o > 0; o >>= 1) p += __shfl_xor(p, o);
    if (i == 0) part[b] = p;
}

__global__ __launch_bounds__(256) void k_sum_parts(const float* __restrict__ part, int B, int count,
                                                   float* __restrict__ loss) {
    __shared__ float red[4];
    float s = 0.0f;
    for (int b = threadIdx.x; b < B; b += 256) s += part[b];
    s = block_sum_f(s, red);
    if (threadIdx.x == 0 && loss) *loss = s / (float)count;
}

// loss = mean (out - target)^2; dout = 2 (out - target) / count.  One workgroup.
__global__ __launch_bounds__(256) void k_mse(const float* __restrict__ out,
                                             const float* __restrict__ target, int count,
                                             float* __restrict__ dout, float* __restrict__ loss) {
    __shared__ float red[4];
    float s = 0.0f;
    for (int e = threadIdx.x; e < count; e += 256) {
        const float r = out[e] - target[e];
        dout[e] = 2.0f * r / (float)count;
        s = fmaf(r, r, s);
    }
    s = block_sum_f(s, red);
    if (threadIdx.x == 0 && loss) *loss = s / (float)count;
}

__global__ __launch_bounds__(256) void k_adam(float* __restrict__ w32, __half* __restrict__ w16,
                                              float* __restrict__ m, float* __restrict__ v,
                                              const float* __restrict__ g, size_t n, float lr,
                                              float b1, float b2, float eps, float c1, float c2) {
    const size_t t = (size_t)blockIdx.x * 256 + threadIdx.x;
    if (t >= n) return;
    const float gt = g[t];
    const float mt = b1 * m[t] + (1.0f - b1) * gt;
    const float vt = b2 * v[t] + (1.0f - b2) * gt * gt;
    m[t] = mt;
    v[t] = vt;
    const float w = w32[t] - lr * (mt / c1) / (sqrtf(vt / c2) + eps);
    w32[t] = w;
    w16[t] = __float2half(w);
}

// Network inputs of stamp s: the 41 x 41 windows of I1 and I2 around the
// stamp centre, each minus the mean of its unmasked border pixels, both
// divided by the reference window's flux F (the summed window minus its sky),
// floored at 3 sigma_b sqrt(n) (sigma_b the reference border scatter, n the
// valid pixels: a faint or empty window cannot blow the scale up), times 100
// and kept within the FP16 range; masked or outside pixels are 0.  One
// workgroup per stamp.
__global__ __launch_bounds__(256) void k_stamp_inputs(const float* __restrict__ I1,
                                                      const uint8_t* __restrict__ M1,
                                                      const float* __restrict__ I2,
                                                      const uint8_t* __restrict__ M2, int W, int H,
                                                      int64_t pitch, const int32_t* __restrict__ xy,
                                                      __half* __restrict__ xo,
                                                      float* __restrict__ flux) {
    __shared__ float red[4];
    constexpr int R = SIDE0 / 2, NP = SIDE0 * SIDE0;
    const int s = blockIdx.x, xc = xy[2 * s], yc = xy[2 * s + 1];
    auto val = [&](const float* I, const uint8_t* M, int e, bool& ok) {
        const int dy = e / SIDE0 - R, dx = e % SIDE0 - R;
        const int gx = xc + dx, gy = yc + dy;
        ok = gx >= 0 && gx < W && gy >= 0 && gy < H;
        if (!ok) return 0.0f;
        const int64_t o = (int64_t)gy * pitch + gx;
        ok = M[o] == 0 && isfinite(I[o]);
        return ok ? I[o] : 0.0f;
    };
    float sky[2], sig1 = 0.0f;
    for (int k = 0; k < 2; k++) {
        const float* I = k ? I2 : I1;
        const uint8_t* M = k ? M2 : M1;
        float sum = 0.0f, sq = 0.0f, cnt = 0.0f;
        for (int e = threadIdx.x; e < NP; e += 256) {
            const int py = e / SIDE0, px = e % SIDE0;
            if (py != 0 && py != SIDE0 - 1 && px != 0 && px != SIDE0 - 1) continue;
            bool ok;
            const float v = val(I, M, e, ok);
            if (ok) {
                sum += v;
                sq = fmaf(v, v, sq);
                cnt += 1.0f;
            }
        }
        sum = block_sum_f(sum, red);
        sq = block_sum_f(sq, red);
        cnt = block_sum_f(cnt, red);
        sky[k] = cnt > 0.0f ? sum / cnt : 0.0f;
        if (k == 0 && cnt > 1.0f) sig1 = sqrtf(fmaxf(sq / cnt - sky[0] * sky[0], 0.0f));
    }
    float f = 0.0f, nv = 0.0f;
    for (int e = threadIdx.x; e < NP; e += 256) {
        bool ok;
        const float v = val(I1, M1, e, ok);
        if (ok) {
            f += v - sky[0];
            nv += 1.0f;
        }
    }
    f = block_sum_f(f, red);
    nv = block_sum_f(nv, red);
    const float den = fmaxf(f, 3.0f * sig1 * sqrtf(nv));
    const float scale = den > 0.0f ? 100.0f / den : 0.0f;
    for (int e = threadIdx.x; e < NP; e += 256) {
        bool ok1, ok2;
        const float v1 = val(I1, M1, e, ok1), v2 = val(I2, M2, e, ok2);
        const float x1 = ok1 ? (v1 - sky[0]) * scale : 0.0f;
        const float x2 = ok2 ? (v2 - sky[1]) * scale : 0.0f;
        xo[((size_t)s * 2 + 0) * NP + e] = __float2half(fminf(fmaxf(x1, -60000.0f), 60000.0f));
        xo[((size_t)s * 2 + 1) * NP + e] = __float2half(fminf(fmaxf(x2, -60000.0f), 60000.0f));
    }
    if (threadIdx.x == 0 && flux) flux[s] = f;
}

// Orthonormal-basis coefficients and local basis coefficients, per stamp:
//   c = R a (targets), a = R^-1 c (predictions), R upper (nb x nb).
__global__ void k_coeff_to_ortho(const double* __restrict__ Rm, int nb, int L,
                                 const double* __restrict__ a, int n, float* __restrict__ c) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n * nb) return;
    const int s = t / nb, i = t - s * nb;
    double acc = 0.0;
    for (int j = i; j < nb; j++) acc += Rm[i * nb + j] * a[(size_t)s * L + j];
    c[t] = (float)acc;
}

__global__ __launch_bounds__(64) void k_ortho_to_coeff(const double* __restrict__ Rm, int nb, int L,
                                                        const float* __restrict__ c,
                                                        double* __restrict__ a) {
    // one wave per stamp; lane i holds row i of the right-hand side, which
    // is reduced column by column (a_k = r_k / R_kk, then r_i -= R_ik a_k)
    const int s = blockIdx.x, i = threadIdx.x;
    double r = i < nb ? (double)c[(size_t)s * nb + i] : 0.0;
    double ai = 0.0;
    for (int k = nb - 1; k >= 0; k--) {
        const double ak = __shfl(r, k) / Rm[k * nb + k];
        if (i == k) ai = ak;
        if (i < k) r -= Rm[i * nb + k] * ak;
    }
    if (i < L) a[(size_t)s * L + i] = i < nb ? ai : 0.0;
}

// Loss weight of stamp s in orthonormal coordinates: the stamp matrix with
// the background eliminated, Mh = M_kk - M_kb M_bb^-1 M_bk (nb x nb), mapped
// by W = R^-T Mh R^-1 and divided by npix, so that r^T W r is the chi2/dof
// excess of a kernel whose orthonormal coefficients are off by r (the
// background re-fitted).  One wave per stamp; flagged stamps get zeros.
__global__ __launch_bounds__(64) void k_loss_weight(const double* __restrict__ Rm, int nb,
                                                    const double* __restrict__ Ms,
                                                    const int32_t* __restrict__ npix,
                                                    const int32_t* __restrict__ flags,
                                                    float* __restrict__ Wout) {
    __shared__ double Y[NOUT * (NOUT + 1)];
    const int s = blockIdx.x, t = threadIdx.x, L = nb + 1, LD = NOUT + 1;
    float* Wo = Wout + (size_t)s * NOUT * NOUT;
    const double* M = Ms + (size_t)s * L * L;
    const bool bad = flags[s] != 0 || !(M[nb * L + nb] > 0.0) || npix[s] <= 0;
    if (bad) {
        for (int e = t; e < NOUT * NOUT; e += 64) Wo[e] = 0.0f;
        return;
    }
    const double mbb = M[nb * L + nb];
    if (t < NOUT)
        for (int i = 0; i < NOUT; i++) Y[i * LD + t] = M[i * L + t] - M[i * L + nb] * M[nb * L + t] / mbb;
    __syncthreads();
    if (t < NOUT) {                 // row t of Mh R^-1: y R = mh
        double* y = Y + t * LD;
        for (int j = 0; j < NOUT; j++) {
            double v = y[j];
            for (int k = 0; k < j; k++) v -= y[k] * Rm[k * nb + j];
            y[j] = v / Rm[j * nb + j];
        }
    }
    __syncthreads();
    if (t < NOUT) {                 // column t of R^-T (Mh R^-1): R^T w = y
        for (int i = 0; i < NOUT; i++) {
            double v = Y[i * LD + t];
            for (int k = 0; k < i; k++) v -= Rm[k * nb + i] * Y[k * LD + t];
            Y[i * LD + t] = v / Rm[i * nb + i];
        }
    }
    __syncthreads();
    const double sc = 1.0 / (double)npix[s];
    for (int e = t; e < NOUT * NOUT; e += 64) {
        const int i = e / NOUT, j = e - i * NOUT;
        Wo[e] = (float)(0.5 * (Y[i * LD + j] + Y[j * LD + i]) * sc);
    }
}

constexpr int WSPLIT_MAX = 128;  // batch chunks of the weight-gradient reduction

// Weight gradient of one convolution layer: (o, c) pairs x batch chunks
// (enough workgroups to fill the chip), then the chunk partials summed in
// a fixed order.
template <int S>
void conv_bwd_w(hipStream_t st, const float* dy, int Hout, const __half* x, int CIN, int Hin, int B,
                float* wpart, float* dw, float* db) {
    if (CIN == CH) {
        const int nch = (B * Hout * Hout + WG_PIX - 1) / WG_PIX;
        int G = (nch + 1) / 2;                    // at least two pixel chunks per workgroup
        G = G < 1 ? 1 : G > WG_MAXG ? WG_MAXG : G;
        hipLaunchKernelGGL((k_conv_bwd_w_gemm<S>), dim3(G), dim3(256), 0, st, dy, Hout, x, Hin, B, wpart);
        const int nw = CH * CH * 9;
        hipLaunchKernelGGL(k_conv_bwd_w_sum, dim3((nw + CH + 63) / 64), dim3(64 * WSUM_GROUPS), 0, st, wpart, G, nw,
                           dw, db);
        return;
    }
    constexpr int OG = 8;                         // output channels per workgroup
    const int groups = (CH / OG) * CIN;
    int nsplit = (1024 + groups - 1) / groups;
    nsplit = nsplit < 1 ? 1 : nsplit > WSPLIT_MAX ? WSPLIT_MAX : nsplit;
    if (nsplit > B) nsplit = B;
    hipLaunchKernelGGL((k_conv_bwd_w<S, OG>), dim3(groups, nsplit), dim3(256), 0, st, dy, Hout, x, CIN, Hin,
                       B, wpart);
    const int nw = CH * CIN * 9;
    hipLaunchKernelGGL(k_conv_bwd_w_sum, dim3((nw + CH + 63) / 64), dim3(64 * WSUM_GROUPS), 0, st, wpart, nsplit, nw,
                       dw, db);
}

struct Acts {
    __half *a1, *a2, *a3, *a4, *h;
    float *out, *dout, *dh, *d4, *d3, *d2, *d1, *part, *wpart;
    size_t bytes;
};

Acts carve(void* base, int B) {
    psfm::Carver c(base);
    Acts A;
    A.a1 = c.take<__half>((size_t)B * CH * SIDE1 * SIDE1);
    A.a2 = c.take<__half>((size_t)B * CH * SIDE2 * SIDE2);
    A.a3 = c.take<__half>((size_t)B * CH * SIDE3 * SIDE3);
    A.a4 = c.take<__half>((size_t)B * FLAT);
    A.h = c.take<__half>((size_t)B * HID);
    A.out = c.take<float>((size_t)B * NOUT);
    A.dout = c.take<float>((size_t)B * NOUT);
    A.dh = c.take<float>((size_t)B * HID);
    A.d4 = c.take<float>((size_t)B * FLAT);
    A.d3 = c.take<float>((size_t)B * CH * SIDE3 * SIDE3);
    A.d2 = c.take<float>((size_t)B * CH * SIDE2 * SIDE2);
    A.d1 = c.take<float>((size_t)B * CH * SIDE1 * SIDE1);
    A.part = c.take<float>((size_t)B);
    A.wpart = c.take<float>((size_t)(WSPLIT_MAX > WG_MAXG ? WSPLIT_MAX : WG_MAXG) * (CH * CH * 9 + CH));
    A.bytes = c.off;
    return A;
}

int grid_for(size_t items) {
    size_t g = (items + 255) / 256;
    return (int)(g < 4096 ? (g ? g : 1) : 4096);
}

int forward_into(const __half* w, const __half* x, int B, const Acts& A, hipStream_t st) {
    hipLaunchKernelGGL((k_conv_fwd<2, 1>), dim3(grid_for((size_t)B * SIDE1 * SIDE1)), dim3(256), 0, st,
                       x, SIDE0, w + OFF_C1W, w + OFF_C1B, A.a1, SIDE1, B);
    constexpr int RB = 3;                       // output rows per workgroup band
    hipLaunchKernelGGL((k_conv_fwd_mfma<SIDE1, SIDE2, RB>), dim3(B * ((SIDE2 + RB - 1) / RB)), dim3(256), 0,
                       st, A.a1, w + OFF_C2W, w + OFF_C2B, A.a2);
    hipLaunchKernelGGL((k_conv_fwd_mfma<SIDE2, SIDE3, RB>), dim3(B * ((SIDE3 + RB - 1) / RB)), dim3(256), 0,
                       st, A.a2, w + OFF_C3W, w + OFF_C3B, A.a3);
    hipLaunchKernelGGL((k_conv_fwd_mfma<SIDE3, SIDE4, RB>), dim3(B * ((SIDE4 + RB - 1) / RB)), dim3(256), 0,
                       st, A.a3, w + OFF_C4W, w + OFF_C4B, A.a4);
    static_assert(HID % 16 == 0 && (FLAT * sizeof(__half)) % 16 == 0 && OFF_F1W % 8 == 0,
                  "16 x 16 tiles, 16-byte aligned rows");
    if ((((uintptr_t)A.a4) | ((uintptr_t)(w + OFF_F1W))) % 16 == 0)
        hipLaunchKernelGGL((k_fc_fwd_mfma<FLAT>), dim3(((B + 15) / 16) * (HID / 16)), dim3(256), 0, st,
                           A.a4, w + OFF_F1W, w + OFF_F1B, HID, B, A.h);
    else  // weights or workspace not 16-byte aligned: one wave per output
        hipLaunchKernelGGL((k_fc_fwd<true>), dim3((B * HID + 3) / 4), dim3(256), 0, st, A.a4, FLAT,
                           w + OFF_F1W, w + OFF_F1B, HID, B, A.h, nullptr);
    hipLaunchKernelGGL((k_fc_fwd<false>), dim3((B * NOUT + 3) / 4), dim3(256), 0, st, A.h, HID,
                       w + OFF_F2W, w + OFF_F2B, NOUT, B, nullptr, A.out);
    PSFM_HIP_CHECK(hipGetLastError());
    return PSFM_OK;
}

// ---- training-set statistics and per-sample transforms of the loss

// Per output component c (one workgroup each): the mean and the unbiased
// standard deviation of target[0..n_stats)[c], two passes with FP64 sums in
// a fixed order; sd floored at 1e-12.
__global__ __launch_bounds__(256) void k_col_stats(const float* __restrict__ target, int n_stats,
                                                   float* __restrict__ mu, float* __restrict__ sd) {
    __shared__ double red[16];
    const int c = blockIdx.x;
    double s = 0.0;
    for (int r = threadIdx.x; r < n_stats; r += blockDim.x) s += target[(size_t)r * NOUT + c];
    const double m = psfm_block_sum(s, red) / n_stats;
    double q = 0.0;
    for (int r = threadIdx.x; r < n_stats; r += blockDim.x) {
        const double d = target[(size_t)r * NOUT + c] - m;
        q += d * d;
    }
    const double var = psfm_block_sum(q, red) / (n_stats - 1);
    if (threadIdx.x == 0) {
        mu[c] = (float)m;
        sd[c] = fmaxf((float)sqrt(var), 1e-12f);
    }
}

// One wave per sample: z = (target - mu) / sd, and the sample's weight
// carried into z coordinates, diag(sd) W diag(sd), divided by its mean
// diagonal (trace / 49, the trace floored at 1e-30).
__global__ __launch_bounds__(64) void k_standardize(const float* __restrict__ target,
                                                    const float* __restrict__ weight,
                                                    const float* __restrict__ mu,
                                                    const float* __restrict__ sd,
                                                    float* __restrict__ z, float* __restrict__ wz) {
    const int s = blockIdx.x, l = threadIdx.x;
    const float* W = weight + (size_t)s * NOUT * NOUT;
    float* Wo = wz + (size_t)s * NOUT * NOUT;
    if (l < NOUT) z[(size_t)s * NOUT + l] = (target[(size_t)s * NOUT + l] - mu[l]) / sd[l];
    double t = l < NOUT ? (double)(W[l * NOUT + l] * sd[l] * sd[l]) : 0.0;
    for (int o = 32; o > 0; o >>= 1) t += __shfl_xor(t, o);
    const float mean_diag = (float)(fmax(t, 1e-30) / NOUT);
    for (int e = l; e < NOUT * NOUT; e += 64) {
        const int i = e / NOUT, j = e - i * NOUT;
        Wo[e] = W[e] * sd[i] * sd[j] / mean_diag;
    }
}

// The output layer rescaled so that the network returns sd * out + mu: fc2's
// weight rows times sd, its bias sd * b + mu; the FP16 copy of those
// parameters refreshed.
__global__ __launch_bounds__(256) void k_fold_output(float* __restrict__ w32, __half* __restrict__ w16,
                                                     const float* __restrict__ mu,
                                                     const float* __restrict__ sd) {
    for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < NOUT * HID + NOUT;
         e += gridDim.x * blockDim.x) {
        float v;
        if (e < NOUT * HID) {
            v = w32[OFF_F2W + e] * sd[e / HID];
            w32[OFF_F2W + e] = v;
            w16[OFF_F2W + e] = __float2half(v);
        } else {
            const int o = e - NOUT * HID;
            v = sd[o] * w32[OFF_F2B + o] + mu[o];
            w32[OFF_F2B + o] = v;
            w16[OFF_F2B + o] = __float2half(v);
        }
    }
}

// One wave per sample: r^T W r with r = pred - target (FP64 sums).
__global__ __launch_bounds__(64) void k_quad_excess(const float* __restrict__ pred, int pred_stride,
                                                    const float* __restrict__ target,
                                                    const float* __restrict__ weight,
                                                    float* __restrict__ exc) {
    const int s = blockIdx.x, l = threadIdx.x;
    const float r = l < NOUT ? pred[(size_t)s * pred_stride + l] - target[(size_t)s * NOUT + l] : 0.0f;
    const float* W = weight + (size_t)s * NOUT * NOUT;
    double wr = 0.0;                                   // (W r)_l
    for (int j = 0; j < NOUT; j++) {
        const float rj = __shfl(r, j);
        if (l < NOUT) wr += (double)W[l * NOUT + j] * rj;
    }
    double q = (double)r * wr;
    for (int o = 32; o > 0; o >>= 1) q += __shfl_xor(q, o);
    if (l == 0) exc[s] = (float)q;
}

}  // namespace

extern "C" size_t psfm_cnn_param_count(void) { return NPARAM; }

extern "C" size_t psfm_cnn_workspace_bytes(int batch) {
    if (batch < 1) return 0;
    return carve(nullptr, batch).bytes + 256;
}

extern "C" int psfm_cnn_forward(const uint16_t* w16, const uint16_t* x, int batch, float* out,
                                void* ws, size_t ws_bytes, void* stream) {
    if (!w16 || !x || !out || batch < 1) return PSFM_ERR_INVALID_ARG;
    if (!ws || ws_bytes < psfm_cnn_workspace_bytes(batch)) return PSFM_ERR_WORKSPACE;
    hipStream_t st = (hipStream_t)stream;
    const Acts A = carve(ws, batch);
    int rc = forward_into(reinterpret_cast<const __half*>(w16), reinterpret_cast<const __half*>(x),
                          batch, A, st);
    if (rc) return rc;
    PSFM_HIP_CHECK(hipMemcpyAsync(out, A.out, sizeof(float) * batch * NOUT, hipMemcpyDeviceToDevice, st));
    return PSFM_OK;
}

extern "C" int psfm_cnn_loss_grad(const uint16_t* w16, const uint16_t* x, const float* target,
                                  const float* weight, int batch, float* grad, float* loss, void* ws,
                                  size_t ws_bytes, void* stream) {
    if (!w16 || !x || !target || !grad || batch < 1) return PSFM_ERR_INVALID_ARG;
    if (!ws || ws_bytes < psfm_cnn_workspace_bytes(batch)) return PSFM_ERR_WORKSPACE;
    hipStream_t st = (hipStream_t)stream;
    const int B = batch;
    const __half* w = reinterpret_cast<const __half*>(w16);
    const __half* x0 = reinterpret_cast<const __half*>(x);
    const Acts A = carve(ws, B);
    int rc = forward_into(w, x0, B, A, st);
    if (rc) return rc;
    if (weight) {
        hipLaunchKernelGGL(k_wloss, dim3(B), dim3(64), 0, st, A.out, target, weight, B * NOUT, A.dout,
                           A.part);
        hipLaunchKernelGGL(k_sum_parts, dim3(1), dim3(256), 0, st, A.part, B, B * NOUT, loss);
    } else {
        hipLaunchKernelGGL(k_mse, dim3(1), dim3(256), 0, st, A.out, target, B * NOUT, A.dout, loss);
    }
    // fc2, fc1
    hipLaunchKernelGGL(k_fc_bwd_w, dim3((NOUT * HID + 63) / 64), dim3(256), 0, st, A.dout, NOUT, A.h,
                       HID, B, grad + OFF_F2W, grad + OFF_F2B);
    hipLaunchKernelGGL(k_fc_bwd_x, dim3((B * HID + 63) / 64), dim3(256), 0, st, A.dout, NOUT,
                       w + OFF_F2W, A.h, HID, B, A.dh);
    hipLaunchKernelGGL(k_fc_bwd_w, dim3((HID * FLAT + 63) / 64), dim3(256), 0, st, A.dh, HID, A.a4,
                       FLAT, B, grad + OFF_F1W, grad + OFF_F1B);
    hipLaunchKernelGGL(k_fc_bwd_x, dim3((B * FLAT + 63) / 64), dim3(256), 0, st, A.dh, HID,
                       w + OFF_F1W, A.a4, FLAT, B, A.d4);
    // conv4 .. conv1 (d_k: gradient at the pre-activation of conv k, ReLU applied)
    conv_bwd_w<2>(st, A.d4, SIDE4, A.a3, CH, SIDE3, B, A.wpart, grad + OFF_C4W, grad + OFF_C4B);
    hipLaunchKernelGGL((k_conv_bwd_data_mfma<SIDE3, SIDE4, SIDE3>), dim3(B), dim3(256), 0, st, A.d4,
                       w + OFF_C4W, A.a3, A.d3);
    conv_bwd_w<2>(st, A.d3, SIDE3, A.a2, CH, SIDE2, B, A.wpart, grad + OFF_C3W, grad + OFF_C3B);
    hipLaunchKernelGGL((k_conv_bwd_data_mfma<SIDE2, SIDE3, 10>), dim3(B * ((SIDE2 + 9) / 10)), dim3(256), 0,
                       st, A.d3, w + OFF_C3W, A.a2, A.d2);
    conv_bwd_w<2>(st, A.d2, SIDE2, A.a1, CH, SIDE1, B, A.wpart, grad + OFF_C2W, grad + OFF_C2B);
    hipLaunchKernelGGL((k_conv_bwd_data_mfma<SIDE1, SIDE2, 6>), dim3(B * ((SIDE1 + 5) / 6)), dim3(256), 0, st,
                       A.d2, w + OFF_C2W, A.a1, A.d1);
    conv_bwd_w<1>(st, A.d1, SIDE1, x0, 2, SIDE0, B, A.wpart, grad + OFF_C1W, grad + OFF_C1B);
    PSFM_HIP_CHECK(hipGetLastError());
    return PSFM_OK;
}

extern "C" int psfm_cnn_adam(float* w32, uint16_t* w16, float* m, float* v, const float* grad,
                             size_t n, int step, float lr, float beta1, float beta2, float eps,
                             void* stream) {
    if (!w32 || !w16 || !m || !v || !grad || step < 1 || n == 0) return PSFM_ERR_INVALID_ARG;
    const float c1 = 1.0f - std::pow(beta1, (float)step);
    const float c2 = 1.0f - std::pow(beta2, (float)step);
    hipLaunchKernelGGL(k_adam, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, (hipStream_t)stream, w32,
                       reinterpret_cast<__half*>(w16), m, v, grad, n, lr, beta1, beta2, eps, c1, c2);
    PSFM_HIP_CHECK(hipGetLastError());
    return PSFM_OK;
}

extern "C" int psfm_cnn_stamp_inputs(const float* I1, const uint8_t* M1, const float* I2,
                                     const uint8_t* M2, int W, int H, int64_t pitch,
                                     const int32_t* stamp_xy, int n_stamps, uint16_t* x,
                                     float* flux, void* stream) {
    if (n_stamps < 0 || W < 1 || H < 1 || pitch < W) return PSFM_ERR_INVALID_ARG;
    if (n_stamps == 0) return PSFM_OK;
    if (!I1 || !M1 || !I2 || !M2 || !stamp_xy || !x) return PSFM_ERR_INVALID_ARG;
    hipLaunchKernelGGL(k_stamp_inputs, dim3(n_stamps), dim3(256), 0, (hipStream_t)stream, I1, M1, I2,
                       M2, W, H, pitch, stamp_xy, reinterpret_cast<__half*>(x), flux);
    PSFM_HIP_CHECK(hipGetLastError());
    return PSFM_OK;
}

extern "C" int psfm_cnn_targets(const psfm_context* ctx, const double* local, int n_stamps,
                                float* ortho, void* stream) {
    if (!ctx || n_stamps < 0 || (n_stamps > 0 && (!local || !ortho))) return PSFM_ERR_INVALID_ARG;
    if (ctx->nb != NOUT || !ctx->kgram_ok) return PSFM_ERR_UNSUPPORTED;
    if (n_stamps == 0) return PSFM_OK;
    hipLaunchKernelGGL(k_coeff_to_ortho, dim3((n_stamps * ctx->nb + 255) / 256), dim3(256), 0,
                       (hipStream_t)stream, ctx->kgram_R, ctx->nb, ctx->L, local, n_stamps, ortho);
    PSFM_HIP_CHECK(hipGetLastError());
    return PSFM_OK;
}

extern "C" int psfm_cnn_loss_weights(const psfm_context* ctx, const double* stamp_M,
                                     const int32_t* stamp_npix, const int32_t* stamp_flags,
                                     int n_stamps, float* weight, void* stream) {
    if (!ctx || n_stamps < 0) return PSFM_ERR_INVALID_ARG;
    if (ctx->nb != NOUT || !ctx->kgram_ok) return PSFM_ERR_UNSUPPORTED;
    if (n_stamps == 0) return PSFM_OK;
    if (!stamp_M || !stamp_npix || !stamp_flags || !weight) return PSFM_ERR_INVALID_ARG;
    hipLaunchKernelGGL(k_loss_weight, dim3(n_stamps), dim3(64), 0, (hipStream_t)stream, ctx->kgram_R,
                       ctx->nb, stamp_M, stamp_npix, stamp_flags, weight);
    PSFM_HIP_CHECK(hipGetLastError());
    return PSFM_OK;
}

extern "C" int psfm_cnn_local_coeffs(const psfm_context* ctx, const float* ortho, int n_stamps,
                                     double* local, void* stream) {
    if (!ctx || n_stamps < 0 || (n_stamps > 0 && (!local || !ortho))) return PSFM_ERR_INVALID_ARG;
    if (ctx->nb != NOUT || !ctx->kgram_ok) return PSFM_ERR_UNSUPPORTED;
    if (n_stamps == 0) return PSFM_OK;
    hipLaunchKernelGGL(k_ortho_to_coeff, dim3(n_stamps), dim3(64), 0, (hipStream_t)stream,
                       ctx->kgram_R, ctx->nb, ctx->L, ortho, local);
    PSFM_HIP_CHECK(hipGetLastError());
    return PSFM_OK;
}

extern "C" int psfm_cnn_standardize(const float* target, const float* weight, int n, int n_stats,
                                    float* mu, float* sd, float* z, float* wz, void* stream) {
    if (!target || !weight || !mu || !sd || !z || !wz || n_stats < 2 || n_stats > n)
        return PSFM_ERR_INVALID_ARG;
    hipStream_t st = (hipStream_t)stream;
    hipLaunchKernelGGL(k_col_stats, dim3(NOUT), dim3(256), 0, st, target, n_stats, mu, sd);
    hipLaunchKernelGGL(k_standardize, dim3(n), dim3(64), 0, st, target, weight, mu, sd, z, wz);
    PSFM_HIP_CHECK(hipGetLastError());
    return PSFM_OK;
}

extern "C" int psfm_cnn_fold_output(float* w32, uint16_t* w16, const float* mu, const float* sd,
                                    void* stream) {
    if (!w32 || !w16 || !mu || !sd) return PSFM_ERR_INVALID_ARG;
    hipLaunchKernelGGL(k_fold_output, dim3((NOUT * HID + NOUT + 255) / 256), dim3(256), 0,
                       (hipStream_t)stream, w32, reinterpret_cast<__half*>(w16), mu, sd);
    PSFM_HIP_CHECK(hipGetLastError());
    return PSFM_OK;
}

extern "C" int psfm_cnn_excess(const float* pred, int pred_stride, const float* target,
                               const float* weight, int n, float* exc, void* stream) {
    if (n < 0 || (pred_stride != 0 && pred_stride != NOUT)) return PSFM_ERR_INVALID_ARG;
    if (n == 0) return PSFM_OK;
    if (!pred || !target || !weight || !exc) return PSFM_ERR_INVALID_ARG;
    hipLaunchKernelGGL(k_quad_excess, dim3(n), dim3(64), 0, (hipStream_t)stream, pred, pred_stride,
                       target, weight, exc);
    PSFM_HIP_CHECK(hipGetLastError());
    return PSFM_OK;
}
