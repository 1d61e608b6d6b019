// Internal declarations of the PSF-matching library (not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>

#include <cstddef>
#include <cstdint>

#include "../../include/psfm.h"

#define PSFM_HMAX 16          // largest supported kernel half width
#define PSFM_RMAX 32          // largest supported stamp half width
#define PSFM_GRAM_COLS 64     // Gram width: nb terms + sqrt(w) + d~ (+ zero padding)
#define PSFM_FIT_BR_SHORT 7   // fit bands (stamp rows per workgroup): the three heights
#define PSFM_FIT_BR_MID 9     // the fit kernels are built for
#define PSFM_FIT_BR_TALL 11
#define PSFM_TILE 64          // output tile side of the image convolution
#define PSFM_COV_SAMPLES 9    // 3 x 3 kernels for the image pseudo-matrix

struct psfm_context {
    psfm_config cfg;
    int nb;     // kernel basis terms
    int ns;     // spatial terms
    int N;      // unknowns
    int L;      // per-stamp matrix side (nb + 1)
    int nf;     // distinct 1-D factors (Gaussian j, power e)
    int h, r, KW, T;
    int fit_br;       // stamp rows per fit workgroup (band): PSFM_FIT_BR_SHORT, _MID or _TALL
    // device tables
    double* kb64;     // [nb][T] full basis taps, FP64 (row v major: [(v+h)*KW + (u+h)])
    float* fac;       // [nf][KW] 1-D factors e-th power x Gaussian j, at offsets -h..h
    int* term_rowf;   // [nb] factor index of the u (row-pass) profile of term i
    int* term_colf;   // [nb] factor index of the v (column-pass) profile of term i
    int* term_rorder; // [nb] the terms ordered by row factor, increasing i within one
    int* row_start;   // [nf + 1] row factor r's terms: term_rorder[row_start[r] .. row_start[r + 1])
    float* term_psi;  // [nb] normalisation of the separable product
    float* term_z;    // [nb] 1 if k_0 is subtracted (even terms i >= 1), else 0
    double* fac64;    // [nf][KW] the 1-D factors in FP64
    double* psi64;    // [nb] normalisations in FP64
    double* kgram_R;  // [nb][nb] upper factor R of B^T B (B = taps as columns): |B a| = |R a|
    bool kgram_ok;    // false if the basis taps are (nearly) dependent: no R
    double* penq;     // [nb] penalty weights sum (u^2 + v^2)^2 k_i^2 (two-kernel form)
    void* dev_block;  // single allocation backing all of the above
};

// Device-side state of one solve (rejection loop).
struct SolveState {
    int done;
    int info;
    int n_iter;
    int n_rej;
    int n_used;
    int prior_done;   // rejection prior converged (psfm_solve_prior)
    int n_iter_base;  // solutions before the current rejection loop (fallback restart)
    int chi2_done;    // stamps whose chi2 is in (k_chi2_clip); zero between launches
    int n_rep;        // stamps brought in from the reserve (psfm_solve_norm)
};

// Everything the kernels need about one image pair: inputs, outputs, the
// pair's share of the workspace and its offsets in the flattened work lists
// of a batch.  Built on the host; single-pair calls pass it by value, batched
// calls read it from a device array.
struct PairDesc {
    const float* I1;
    const float* V1;
    const uint8_t* M1;
    const float* I2;
    const float* V2;
    const uint8_t* M2;
    int W, H;
    int64_t pitch;
    const int32_t* xy;
    int n;                 // stamps
    int S, ns, N;
    // per-stamp results
    double* Ms;
    double* bs;
    double* es;
    int32_t* npix;
    int32_t* flags;
    double* chi2;
    // solution
    double* coeffs;
    psfm_fit_stats* stats;
    // solve scratch
    SolveState* st;
    uint8_t* used;
    uint8_t* fitted;
    double* G;
    double* A;
    double* b;
    double* ILg;
    // fit scratch
    double* part;
    int* bflags;
    // input covariance pseudo-matrices (nullable: uncorrelated)
    const double* cov1;
    int cov1_half;
    const double* cov2;
    int cov2_half;
    // image outputs and their scratch
    float* conv;
    uint8_t* conv_mask;
    float* var;
    double* cov;
    int cov_half;
    float* diff;
    float* diff_var;
    uint8_t* diff_mask;
    double* cov_diff;
    int cov_diff_half;
    double* cov_samples;
    double* cov_auto;                // kernel autocorrelation (correlated input only)
    double* cov_avg;
    double* sub_part;                // [tiles][4] variance sums of the tiles
    float* ptaps;                    // batch: per patch, FP32 taps K, f K^2 and the BAD radius
    double* cellK;                   // batch: the pseudo-matrix cells' kernels, PSFM_COV_SAMPLES x T (FP64)
                                     // (psfm::patch_taps_floats each); null: realised per tile
    unsigned int* tiles_done;        // tiles finished (batch completion counter)
    uint64_t* t_done;                // completion time stamp (nullable)
    // offsets in the flattened work lists of a batch
    int band_off;
    int stamp_off;
    int tile_off;
    int patch_off;         // first patch of the pair in the batch's patch list
    int ntx, nty;
};

namespace psfm {

inline size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

// Carves consecutive 256-byte aligned regions out of a workspace.
struct Carver {
    char* base;
    size_t off = 0;
    explicit Carver(void* b) : base(static_cast<char*>(b)) {}
    // With a null base the returned pointers are the byte offsets (layout mode).
    template <class T>
    T* take(size_t count) {
        off = align_up(off, 256);
        T* p = reinterpret_cast<T*>(reinterpret_cast<uintptr_t>(base) + off);
        off += count * sizeof(T);
        return p;
    }
};

// Per-call workspace needs (bytes).
size_t fit_workspace(const psfm_context* ctx, int n_stamps);
size_t dual_fit_workspace(const psfm_context* ctx, int n_stamps);
size_t solve_workspace(const psfm_context* ctx, int n_stamps);
size_t dual_solve_workspace(const psfm_context* ctx, int n_stamps);
int dual_unknowns(const psfm_context* ctx);
size_t conv_workspace(const psfm_context* ctx, int W, int H);
size_t subtract_workspace(const psfm_context* ctx, int W, int H);
size_t match_workspace(const psfm_context* ctx, int W, int H);

int match_pair_ws(const psfm_context* ctx, const double* coeffs, const float* I1, const float* V1,
                  const uint8_t* M1, const float* I2, const float* V2, const uint8_t* M2, int W,
                  int H, int64_t pitch, const double* cov1, int cov1_half, const double* cov2,
                  int cov2_half, float* conv, uint8_t* conv_mask, float* conv_var,
                  double* cov_conv, int cov_conv_half, float* diff, float* diff_var,
                  uint8_t* diff_mask, double* cov_diff, int cov_diff_half, psfm_fit_stats* stats,
                  void* ws, size_t ws_bytes, void* stream);

int fit_bands(const psfm_context* ctx);
int n_patches(const psfm_context* ctx, int W, int H);

int check_hip(hipError_t e);

// Batched stages (all pairs of a batch per launch); pairs, item/stamp/tile
// maps are device arrays.
int batch_fit(const psfm_context* ctx, const PairDesc* pairs, const int* item_pair,
              const int* stamp_pair, int n_items, int n_stamps, hipStream_t st);
// ns_pairs (device): the pair indices grouped by spatial-term count; the
// pairs with ns terms are ns_pairs[ns_off[ns] .. ns_off[ns] + ns_cnt[ns])
// (host tables indexed by ns, PSFM_BATCH_NS_MAX + 1 entries).
constexpr int PSFM_BATCH_NS_MAX = 28;
int batch_solve(const psfm_context* ctx, const PairDesc* pairs, const int* stamp_pair, int n_pairs,
                int n_stamps_total, int max_n, int max_N, const int* ns_pairs, const int* ns_off,
                const int* ns_cnt, hipStream_t st);
// parts: 1 = the pseudo-matrices, 2 = the fused convolution / difference pass, 3 = both.
int batch_apply(const psfm_context* ctx, const PairDesc* pairs, const int* tile_pair, int n_pairs,
                int n_tiles, const int* patch_pair, int n_patches, int max_cov_in, int conv_grid,
                int parts, hipStream_t st);
// floats per patch in PairDesc::ptaps: K and f K^2 (column-major), the BAD radius
__host__ __device__ inline int patch_taps_floats(int h) { return 2 * (2 * h + 1) * (2 * h + 1) + 4; }
int fit_prepare(const psfm_context* ctx);
size_t fit_lds_bytes(const psfm_context* ctx);
int solve_lds_grant(size_t lds);
size_t solve_lds_bytes(int N);
int solve_max_unknowns();
size_t solve_il_doubles(int N);
int cov_sample_side(const psfm_context* ctx, int c_in);

}  // namespace psfm

#define PSFM_HIP_CHECK(call)                          \
    do {                                              \
        hipError_t e_ = (call);                       \
        if (e_ != hipSuccess) return psfm::check_hip(e_); \
    } while (0)

// ---------------------------------------------------------------- device helpers

// Spatial terms x^l y^m (l + m <= S), degree-major with l descending, in
// coordinates scaled to [-1, 1] over the image.
__device__ __forceinline__ void psfm_spatial_terms(int S, double x, double y, int W, int H,
                                                   double* g) {
    const double xt = W > 1 ? (2.0 * x - (W - 1)) / (double)(W - 1) : 0.0;
    const double yt = H > 1 ? (2.0 * y - (H - 1)) / (double)(H - 1) : 0.0;
    int s = 0;
    for (int d = 0; d <= S; d++) {
        for (int l = d; l >= 0; l--) {
            double v = 1.0;
            for (int k = 0; k < l; k++) v *= xt;
            for (int k = 0; k < d - l; k++) v *= yt;
            g[s++] = v;
        }
    }
}

// sum_s coef[s] g_s(x, y) for the spatial terms above, without a term array.
__device__ __forceinline__ double psfm_spatial_dot(int S, double x, double y, int W, int H,
                                                   const double* __restrict__ coef) {
    const double xt = W > 1 ? (2.0 * x - (W - 1)) / (double)(W - 1) : 0.0;
    const double yt = H > 1 ? (2.0 * y - (H - 1)) / (double)(H - 1) : 0.0;
    double acc = 0.0;
    int s = 0;
    for (int d = 0; d <= S; d++) {
        for (int l = d; l >= 0; l--) {
            double v = 1.0;
            for (int k = 0; k < l; k++) v *= xt;
            for (int k = 0; k < d - l; k++) v *= yt;
            acc += coef[s++] * v;
        }
    }
    return acc;
}

// Four psfm_block_sum's in one pass (the same sums, one set of barriers);
// `red` holds >= 4 * (waves) doubles.  Results in v[0..3] of every thread.
__device__ __forceinline__ void psfm_block_sum4(double v[4], double* red) {
#pragma unroll
    for (int k = 0; k < 4; k++)
        for (int o = 32; o > 0; o >>= 1) v[k] += __shfl_down(v[k], o);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0)
#pragma unroll
        for (int k = 0; k < 4; k++) red[4 * wave + k] = v[k];
    __syncthreads();
    const int nw = (blockDim.x + 63) >> 6;
#pragma unroll
    for (int k = 0; k < 4; k++) {
        double s = 0.0;
        for (int w = 0; w < nw; w++) s += red[4 * w + k];
        v[k] = s;
    }
    __syncthreads();
}

// Fixed-order sum over a workgroup of up to 1024 threads (deterministic).
// Every thread of the block must call it; `red` holds >= 16 doubles in LDS.
__device__ __forceinline__ double psfm_block_sum(double v, double* red) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) red[wave] = v;
    __syncthreads();
    double s = 0.0;
    const int nw = (blockDim.x + 63) >> 6;
    for (int w = 0; w < nw; w++) s += red[w];
    __syncthreads();
    return s;
}
