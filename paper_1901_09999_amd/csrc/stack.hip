// PSF homogenisation for stacking (Section 5.1) and the weighted stack of the
// homogenised inputs (Section 5.2).
//
//   k_envelope       one workgroup: the circular (major-axis width, peak 1)
//                    Gaussians of the input PSFs, their pixel-wise maximum,
//                    and the width of the peak-1 circular Gaussian fitted to
//                    it by golden-section search (block-wide FP64 misfits).
//   k_rt_*           the fake target: sources binned to 32 x 32 tiles
//                    (count, scan, fill), then one workgroup per tile puts
//                    its sources back in index order (rank sort in LDS) and
//                    accumulates every pixel's Gaussians in FP64 in that
//                    order; a tile holding more than RT_CAP sources scans the
//                    whole list in order instead.
//   k_stack_reject   one thread per pixel: the unmasked inputs sorted in
//                    registers (bitonic network, masked -> +inf), their
//                    median in FP64 and the per-input outlier flags.
//   k_stack_*        inverse-mean-variance weights (per-block FP64 partials
//                    reduced in a fixed order), the weighted mean, its
//                    variance and mask per pixel, and the weighted mean of
//                    the inputs' pseudo-matrices.
#include "internal.h"

namespace {

constexpr int ST_T = 256;
constexpr int RT_TILE = 32;
constexpr int RT_CAP = 2048;       // sources per tile sorted in LDS
constexpr int ST_BLOCKS = 256;     // row blocks of the mean-variance partials

// ---------------------------------------------------------------- envelope

__device__ double env_misfit(const double* __restrict__ env, int half, double s, double* red) {
    const int Ew = 2 * half + 1;
    double q = 0.0;
    for (int e = threadIdx.x; e < Ew * Ew; e += ST_T) {
        const int v = e / Ew - half, u = e % Ew - half;
        const double d = env[e] - exp(-(double)(u * u + v * v) / (2.0 * s * s));
        q += d * d;
    }
    return psfm_block_sum(q, red);
}

__global__ __launch_bounds__(ST_T) void k_envelope(const double* __restrict__ params, int n, int half,
                                                   double* __restrict__ env, double* __restrict__ sigma) {
    __shared__ double red[16];
    __shared__ double s_max;
    const int Ew = 2 * half + 1;
    if (threadIdx.x == 0) {
        double m = 0.0;
        for (int k = 0; k < n; k++) m = fmax(m, params[3 * k]);
        s_max = m;
    }
    for (int e = threadIdx.x; e < Ew * Ew; e += ST_T) {
        const int v = e / Ew - half, u = e % Ew - half;
        double m = 0.0;
        for (int k = 0; k < n; k++) {
            const double s = params[3 * k];
            m = fmax(m, exp(-(double)(u * u + v * v) / (2.0 * s * s)));
        }
        env[e] = m;
    }
    __syncthreads();
    // every thread runs the same search on block-wide sums
    const double gr = 0.5 * (sqrt(5.0) - 1.0);
    double lo = 0.1, hi = 2.0 * s_max;
    double c = hi - gr * (hi - lo), d = lo + gr * (hi - lo);
    double fc = env_misfit(env, half, c, red), fd = env_misfit(env, half, d, red);
    while (hi - lo > 1e-10) {
        if (fc < fd) {
            hi = d;
            d = c;
            fd = fc;
            c = hi - gr * (hi - lo);
            fc = env_misfit(env, half, c, red);
        } else {
            lo = c;
            c = d;
            fc = fd;
            d = lo + gr * (hi - lo);
            fd = env_misfit(env, half, d, red);
        }
    }
    if (threadIdx.x == 0) *sigma = 0.5 * (lo + hi);
}

// ------------------------------------------------------------ fake target

struct RtGeom {
    int ntx, nty, rad;
};

__host__ __device__ inline int rt_radius(double sigma) { return (int)ceil(6.0 * sigma) + 1; }

// Tile range [*t0, *t1] along one axis covered by a source at coordinate p
// (box floor(p) +- rad, clipped to [0, n)); false if empty.
__device__ inline bool rt_span(double p, int rad, int n, int* t0, int* t1) {
    if (!(p > -1e9 && p < 1e9)) return false;        // also rejects NaN
    const int c = (int)floor(p);
    const int a = max(c - rad, 0), b = min(c + rad, n - 1);
    if (a > b) return false;
    *t0 = a / RT_TILE;
    *t1 = b / RT_TILE;
    return true;
}

__global__ __launch_bounds__(ST_T) void k_rt_zero(int* __restrict__ cnt, int n) {
    const int i = blockIdx.x * ST_T + threadIdx.x;
    if (i < n) cnt[i] = 0;
}

__global__ __launch_bounds__(ST_T) void k_rt_count(const double* __restrict__ src, int n, int W, int H,
                                                   RtGeom g, int* __restrict__ cnt) {
    const int s = blockIdx.x * ST_T + threadIdx.x;
    if (s >= n) return;
    int tx0, tx1, ty0, ty1;
    if (!rt_span(src[3 * s], g.rad, W, &tx0, &tx1) || !rt_span(src[3 * s + 1], g.rad, H, &ty0, &ty1))
        return;
    for (int ty = ty0; ty <= ty1; ty++)
        for (int tx = tx0; tx <= tx1; tx++) atomicAdd(&cnt[ty * g.ntx + tx], 1);
}

// Exclusive scan of cnt[0..n) into off[0..n], copied to cur (fill cursors).
// One workgroup of 1024 threads, chunks of 1024 tiles.
__global__ __launch_bounds__(1024) void k_rt_scan(const int* __restrict__ cnt, int n, int* __restrict__ off,
                                                  int* __restrict__ cur) {
    __shared__ int sh[1024];
    __shared__ int carry;
    if (threadIdx.x == 0) carry = 0;
    __syncthreads();
    for (int base = 0; base < n; base += 1024) {
        const int i = base + threadIdx.x;
        const int v = i < n ? cnt[i] : 0;
        sh[threadIdx.x] = v;
        __syncthreads();
        for (int o = 1; o < 1024; o <<= 1) {
            const int t = threadIdx.x >= o ? sh[threadIdx.x - o] : 0;
            __syncthreads();
            sh[threadIdx.x] += t;
            __syncthreads();
        }
        const int excl = carry + sh[threadIdx.x] - v;
        if (i < n) {
            off[i] = excl;
            cur[i] = excl;
        }
        __syncthreads();
        if (threadIdx.x == 1023) carry += sh[1023];
        __syncthreads();
    }
    if (threadIdx.x == 0) off[n] = carry;
}

__global__ __launch_bounds__(ST_T) void k_rt_fill(const double* __restrict__ src, int n, int W, int H,
                                                  RtGeom g, int* __restrict__ cur, int* __restrict__ list) {
    const int s = blockIdx.x * ST_T + threadIdx.x;
    if (s >= n) return;
    int tx0, tx1, ty0, ty1;
    if (!rt_span(src[3 * s], g.rad, W, &tx0, &tx1) || !rt_span(src[3 * s + 1], g.rad, H, &ty0, &ty1))
        return;
    for (int ty = ty0; ty <= ty1; ty++)
        for (int tx = tx0; tx <= tx1; tx++) list[atomicAdd(&cur[ty * g.ntx + tx], 1)] = s;
}

// Adds source (x0, y0, f) to the 4 pixels of this thread (column lx, rows
// ly0 + 8 j of the tile) that lie in its box.
__device__ __forceinline__ void rt_add(double x0, double y0, double f, int rad, double norm, double s2,
                                       int gx, int gy0, double acc[4]) {
    const int xi = (int)floor(x0), yi = (int)floor(y0);
    if (gx < xi - rad || gx > xi + rad) return;
    const double dx = gx - x0;
#pragma unroll
    for (int j = 0; j < 4; j++) {
        const int gy = gy0 + 8 * j;
        if (gy < yi - rad || gy > yi + rad) continue;
        const double dy = gy - y0;
        acc[j] += f * norm * exp(-(dx * dx + dy * dy) / s2);
    }
}

__global__ __launch_bounds__(ST_T) void k_rt_render(const double* __restrict__ src, int n, double sigma,
                                                    int W, int H, int64_t pitch, RtGeom g,
                                                    const int* __restrict__ off,
                                                    const int* __restrict__ list, float* __restrict__ out) {
    __shared__ int ids[RT_CAP];
    __shared__ int sorted[RT_CAP];
    __shared__ double sp[ST_T][3];
    const int tile = blockIdx.x, tx = tile % g.ntx, ty = tile / g.ntx;
    const int lx = threadIdx.x & 31, ly0 = threadIdx.x >> 5;
    const int gx = tx * RT_TILE + lx, gy0 = ty * RT_TILE + ly0;
    const double norm = 1.0 / (2.0 * 3.14159265358979323846 * sigma * sigma);
    const double s2 = 2.0 * sigma * sigma;
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    const int o0 = off[tile], m = off[tile + 1] - o0;
    if (m <= RT_CAP) {
        for (int i = threadIdx.x; i < m; i += ST_T) ids[i] = list[o0 + i];
        __syncthreads();
        // source indices are distinct within a tile: rank = number smaller
        for (int i = threadIdx.x; i < m; i += ST_T) {
            const int v = ids[i];
            int r = 0;
            for (int j = 0; j < m; j++) r += ids[j] < v;
            sorted[r] = v;
        }
        __syncthreads();
        for (int b = 0; b < m; b += ST_T) {
            const int i = b + threadIdx.x;
            if (i < m) {
                const int s = sorted[i];
                sp[threadIdx.x][0] = src[3 * s];
                sp[threadIdx.x][1] = src[3 * s + 1];
                sp[threadIdx.x][2] = src[3 * s + 2];
            }
            __syncthreads();
            const int e = min(ST_T, m - b);
            for (int k = 0; k < e; k++) rt_add(sp[k][0], sp[k][1], sp[k][2], g.rad, norm, s2, gx, gy0, acc);
            __syncthreads();
        }
    } else {
        // crowded tile: every source, in index order, tested against the tile
        for (int b = 0; b < n; b += ST_T) {
            const int i = b + threadIdx.x;
            if (i < n) {
                sp[threadIdx.x][0] = src[3 * i];
                sp[threadIdx.x][1] = src[3 * i + 1];
                sp[threadIdx.x][2] = src[3 * i + 2];
            }
            __syncthreads();
            const int e = min(ST_T, n - b);
            for (int k = 0; k < e; k++) {
                const double x0 = sp[k][0], y0 = sp[k][1];
                if (!(x0 > -1e9 && x0 < 1e9 && y0 > -1e9 && y0 < 1e9)) continue;
                rt_add(x0, y0, sp[k][2], g.rad, norm, s2, gx, gy0, acc);
            }
            __syncthreads();
        }
    }
    if (gx < W) {
#pragma unroll
        for (int j = 0; j < 4; j++) {
            const int gy = gy0 + 8 * j;
            if (gy < H) out[(int64_t)gy * pitch + gx] = (float)acc[j];
        }
    }
}

struct RtLayout {
    int ntiles;
    size_t off_cnt, off_off, off_cur, off_list, total;
    int64_t list_len;
};

RtLayout rt_layout(int n, int W, int H, double sigma) {
    RtLayout L;
    const int rad = rt_radius(sigma);
    const int64_t span = (2 * (int64_t)rad) / RT_TILE + 2;      // tiles per axis one box can touch
    L.ntiles = ((W + RT_TILE - 1) / RT_TILE) * ((H + RT_TILE - 1) / RT_TILE);
    L.list_len = (int64_t)n * span * span;
    auto al = [](size_t b) { return (b + 255) & ~(size_t)255; };
    L.off_cnt = 0;
    L.off_off = al(L.off_cnt + sizeof(int) * (size_t)L.ntiles);
    L.off_cur = al(L.off_off + sizeof(int) * ((size_t)L.ntiles + 1));
    L.off_list = al(L.off_cur + sizeof(int) * (size_t)L.ntiles);
    L.total = al(L.off_list + sizeof(int) * (size_t)L.list_len);
    return L;
}

// ------------------------------------------------------- outlier rejection

template <int NP>
__device__ __forceinline__ void bitonic(float (&v)[NP]) {
#pragma unroll
    for (int k = 2; k <= NP; k <<= 1) {
#pragma unroll
        for (int j = k >> 1; j > 0; j >>= 1) {
#pragma unroll
            for (int i = 0; i < NP; i++) {
                const int l = i ^ j;
                if (l > i) {
                    const bool up = (i & k) == 0;
                    const float a = v[i], b = v[l];
                    const bool sw = up ? (a > b) : (a < b);
                    v[i] = sw ? b : a;
                    v[l] = sw ? a : b;
                }
            }
        }
    }
}

// One thread per pixel; block 64 x 4 (a wave reads 64 consecutive pixels).
template <int NP>
__global__ __launch_bounds__(ST_T) void k_stack_reject(int n, const float* __restrict__ I,
                                                       const float* __restrict__ V,
                                                       const uint8_t* __restrict__ M, int64_t plane,
                                                       int W, int H, int64_t pitch, double nsigma,
                                                       uint8_t* __restrict__ out) {
    const int x = blockIdx.x * 64 + (threadIdx.x & 63), y = blockIdx.y * 4 + (threadIdx.x >> 6);
    if (x >= W || y >= H) return;
    const int64_t o = (int64_t)y * pitch + x;
    float val[NP], srt[NP];
    int m = 0;
#pragma unroll
    for (int k = 0; k < NP; k++) {
        if (k < n) {
            val[k] = I[k * plane + o];
            const bool mk = M[k * plane + o] != 0;
            srt[k] = mk ? INFINITY : val[k];
            m += mk ? 0 : 1;
        } else {
            val[k] = 0.0f;
            srt[k] = INFINITY;
        }
    }
    if (m < 3) {
        for (int k = 0; k < n; k++) out[k * plane + o] = 0;
        return;
    }
    bitonic<NP>(srt);
    const int i1 = (m - 1) >> 1, i2 = m >> 1;
    float a = 0.0f, b = 0.0f;
#pragma unroll
    for (int k = 0; k < NP; k++) {
        if (k == i1) a = srt[k];
        if (k == i2) b = srt[k];
    }
    const double med = (m & 1) ? (double)b : 0.5 * ((double)a + (double)b);
#pragma unroll
    for (int k = 0; k < NP; k++) {
        if (k < n) {
            const int64_t q = k * plane + o;
            uint8_t f = 0;
            if (M[q] == 0) f = fabs((double)val[k] - med) > nsigma * sqrt((double)V[q]) ? 1 : 0;
            out[q] = f;
        }
    }
}

// ------------------------------------------------------------ weighted stack

// Partial sums of V and counts over the unmasked pixels of input k
// (blockIdx.y) in rows blockIdx.x, + ST_BLOCKS, ...; part[(k * ST_BLOCKS + b) * 2 + {0, 1}].
__global__ __launch_bounds__(ST_T) void k_stack_vsum(const float* __restrict__ V, const uint8_t* __restrict__ M,
                                                     int64_t plane, int W, int H, int64_t pitch,
                                                     double* __restrict__ part) {
    __shared__ double red[16];
    const int k = blockIdx.y;
    double sv = 0.0, cnt = 0.0;
    for (int y = blockIdx.x; y < H; y += ST_BLOCKS) {
        const int64_t row = k * plane + (int64_t)y * pitch;
        for (int x = threadIdx.x; x < W; x += ST_T) {
            if (M[row + x] == 0) {
                sv += V[row + x];
                cnt += 1.0;
            }
        }
    }
    sv = psfm_block_sum(sv, red);
    cnt = psfm_block_sum(cnt, red);
    if (threadIdx.x == 0) {
        part[(k * ST_BLOCKS + blockIdx.x) * 2] = sv;
        part[(k * ST_BLOCKS + blockIdx.x) * 2 + 1] = cnt;
    }
}

// Weights w_k = 1 / mean V_k and the stack pseudo-matrix (one workgroup).
__global__ __launch_bounds__(ST_T) void k_stack_weights(int n, const double* __restrict__ part,
                                                        const double* __restrict__ C, int ck,
                                                        double* __restrict__ wv, double* __restrict__ CS,
                                                        double* __restrict__ weights) {
    __shared__ double sw[64], sv[64];
    if (threadIdx.x < n) {
        const int k = threadIdx.x;
        double s = 0.0, c = 0.0;
        for (int b = 0; b < ST_BLOCKS; b++) {
            s += part[(k * ST_BLOCKS + b) * 2];
            c += part[(k * ST_BLOCKS + b) * 2 + 1];
        }
        const double vbar = c > 0.0 ? s / c : 0.0;
        const double w = vbar > 0.0 ? 1.0 / vbar : 0.0;
        sw[k] = w;
        sv[k] = vbar;
        wv[k] = w;
        if (weights) weights[k] = w;
    }
    __syncthreads();
    if (!CS) return;
    const int Cw = 2 * ck + 1;
    double tw = 0.0;
    for (int k = 0; k < n; k++) tw += sw[k] * sw[k] * sv[k];
    for (int t = threadIdx.x; t < Cw * Cw; t += ST_T) {
        double s = 0.0;
        for (int k = 0; k < n; k++) s += sw[k] * sw[k] * sv[k] * C[(size_t)k * Cw * Cw + t];
        CS[t] = tw > 0.0 ? s / tw : 0.0;
    }
}

__global__ __launch_bounds__(ST_T) void k_stack_combine(int n, const float* __restrict__ I,
                                                        const float* __restrict__ V,
                                                        const uint8_t* __restrict__ M, int64_t plane,
                                                        int W, int H, int64_t pitch,
                                                        const double* __restrict__ wv, float* __restrict__ S,
                                                        float* __restrict__ VS, uint8_t* __restrict__ MS) {
    __shared__ double w[64];
    if (threadIdx.x < n) w[threadIdx.x] = wv[threadIdx.x];
    __syncthreads();
    const int x = blockIdx.x * 64 + (threadIdx.x & 63), y = blockIdx.y * 4 + (threadIdx.x >> 6);
    if (x >= W || y >= H) return;
    const int64_t o = (int64_t)y * pitch + x;
    double swt = 0.0, si = 0.0, sv = 0.0;
    for (int k = 0; k < n; k++) {
        const int64_t q = k * plane + o;
        const float iv = I[q], vv = V[q];
        if (M[q]) continue;
        swt += w[k];
        si += w[k] * (double)iv;
        sv += w[k] * w[k] * (double)vv;
    }
    if (swt > 0.0) {
        S[o] = (float)(si / swt);
        VS[o] = (float)(sv / (swt * swt));
        MS[o] = 0;
    } else {
        S[o] = 0.0f;
        VS[o] = 0.0f;
        MS[o] = 1;
    }
}

template <int NP>
void launch_reject(int n, const float* I, const float* V, const uint8_t* M, int64_t plane, int W, int H,
                   int64_t pitch, double nsigma, uint8_t* out, hipStream_t st) {
    hipLaunchKernelGGL(k_stack_reject<NP>, dim3((W + 63) / 64, (H + 3) / 4), dim3(ST_T), 0, st, n, I, V, M,
                       plane, W, H, pitch, nsigma, out);
}

}  // namespace

extern "C" int psfm_envelope_psf(const double* params, int n, int half, double* env, double* sigma,
                                 void* stream) {
    if (!params || !env || !sigma || n < 1) return PSFM_ERR_INVALID_ARG;
    if (n > PSFM_STACK_MAX_INPUTS || half < 1 || half > 64) return PSFM_ERR_UNSUPPORTED;
    hipLaunchKernelGGL(k_envelope, dim3(1), dim3(ST_T), 0, (hipStream_t)stream, params, n, half, env, sigma);
    PSFM_HIP_CHECK(hipGetLastError());
    return PSFM_OK;
}

extern "C" size_t psfm_render_workspace_bytes(int n, int W, int H, double sigma) {
    if (n < 0 || W < 1 || H < 1 || !(sigma > 0.0) || sigma > 1000.0) return 0;
    return rt_layout(n, W, H, sigma).total;
}

extern "C" int psfm_render_target(const double* src, int n, double sigma, int W, int H, int64_t pitch,
                                  float* out, void* ws, size_t ws_bytes, void* stream) {
    if (!out || n < 0 || (n > 0 && !src) || !(sigma > 0.0)) return PSFM_ERR_INVALID_ARG;
    if (sigma > 1000.0) return PSFM_ERR_UNSUPPORTED;
    if (W < 1 || H < 1 || pitch < W) return PSFM_ERR_SHAPE;
    const RtLayout L = rt_layout(n, W, H, sigma);
    if (!ws || ws_bytes < L.total) return PSFM_ERR_WORKSPACE;
    hipStream_t st = (hipStream_t)stream;
    char* base = static_cast<char*>(ws);
    int* cnt = reinterpret_cast<int*>(base + L.off_cnt);
    int* off = reinterpret_cast<int*>(base + L.off_off);
    int* cur = reinterpret_cast<int*>(base + L.off_cur);
    int* list = reinterpret_cast<int*>(base + L.off_list);
    RtGeom g;
    g.ntx = (W + RT_TILE - 1) / RT_TILE;
    g.nty = (H + RT_TILE - 1) / RT_TILE;
    g.rad = rt_radius(sigma);
    hipLaunchKernelGGL(k_rt_zero, dim3((L.ntiles + ST_T - 1) / ST_T), dim3(ST_T), 0, st, cnt, L.ntiles);
    if (n > 0)
        hipLaunchKernelGGL(k_rt_count, dim3((n + ST_T - 1) / ST_T), dim3(ST_T), 0, st, src, n, W, H, g, cnt);
    hipLaunchKernelGGL(k_rt_scan, dim3(1), dim3(1024), 0, st, cnt, L.ntiles, off, cur);
    if (n > 0)
        hipLaunchKernelGGL(k_rt_fill, dim3((n + ST_T - 1) / ST_T), dim3(ST_T), 0, st, src, n, W, H, g, cur,
                           list);
    hipLaunchKernelGGL(k_rt_render, dim3(L.ntiles), dim3(ST_T), 0, st, src, n, sigma, W, H, pitch, g, off,
                       list, out);
    PSFM_HIP_CHECK(hipGetLastError());
    return PSFM_OK;
}

extern "C" int psfm_stack_reject(int n, const float* I, const float* V, const uint8_t* M, int64_t plane,
                                 int W, int H, int64_t pitch, double nsigma, uint8_t* out, void* stream) {
    if (!I || !V || !M || !out || n < 1 || !(nsigma >= 0.0)) return PSFM_ERR_INVALID_ARG;
    if (n > PSFM_STACK_MAX_INPUTS) return PSFM_ERR_UNSUPPORTED;
    if (W < 1 || H < 1 || pitch < W || plane < pitch * (int64_t)(H - 1) + W) return PSFM_ERR_SHAPE;
    hipStream_t st = (hipStream_t)stream;
    if (n <= 4) launch_reject<4>(n, I, V, M, plane, W, H, pitch, nsigma, out, st);
    else if (n <= 8) launch_reject<8>(n, I, V, M, plane, W, H, pitch, nsigma, out, st);
    else if (n <= 16) launch_reject<16>(n, I, V, M, plane, W, H, pitch, nsigma, out, st);
    else if (n <= 32) launch_reject<32>(n, I, V, M, plane, W, H, pitch, nsigma, out, st);
    else launch_reject<64>(n, I, V, M, plane, W, H, pitch, nsigma, out, st);
    PSFM_HIP_CHECK(hipGetLastError());
    return PSFM_OK;
}

extern "C" int psfm_stack_combine(int n, const float* I, const float* V, const uint8_t* M, int64_t plane,
                                  int W, int H, int64_t pitch, const double* cov, int cov_half, float* S,
                                  float* VS, uint8_t* MS, double* cov_s, double* weights, void* ws,
                                  size_t ws_bytes, void* stream) {
    if (!I || !V || !M || !S || !VS || !MS || n < 1 || cov_half < 0 || (cov_s && !cov))
        return PSFM_ERR_INVALID_ARG;
    if (n > PSFM_STACK_MAX_INPUTS || cov_half > 256) return PSFM_ERR_UNSUPPORTED;
    if (W < 1 || H < 1 || pitch < W || plane < pitch * (int64_t)(H - 1) + W) return PSFM_ERR_SHAPE;
    if (!ws || ws_bytes < PSFM_STACK_WORKSPACE_BYTES) return PSFM_ERR_WORKSPACE;
    hipStream_t st = (hipStream_t)stream;
    double* part = static_cast<double*>(ws);
    double* wv = part + (size_t)PSFM_STACK_MAX_INPUTS * ST_BLOCKS * 2;
    hipLaunchKernelGGL(k_stack_vsum, dim3(ST_BLOCKS, n), dim3(ST_T), 0, st, V, M, plane, W, H, pitch, part);
    hipLaunchKernelGGL(k_stack_weights, dim3(1), dim3(ST_T), 0, st, n, part, cov, cov_half, wv, cov_s,
                       weights);
    hipLaunchKernelGGL(k_stack_combine, dim3((W + 63) / 64, (H + 3) / 4), dim3(ST_T), 0, st, n, I, V, M,
                       plane, W, H, pitch, wv, S, VS, MS);
    PSFM_HIP_CHECK(hipGetLastError());
    return PSFM_OK;
}
