// psfm_match_pair_static: psfm_match_pair for callers that cannot allocate
// device memory (code under HIP graph capture, tight serving loops).  The
// call's scratch -- the covariance samples of the pseudo-matrix, the
// per-tile variance sums of C_D and the patch taps -- lives in a file-scope
// device array of PSFM_STATIC_SCRATCH_BYTES instead of a caller workspace;
// the kernels are psfm_match_pair's own and take the array's device address
// as their workspace pointer.
//
// Each device holds its own copy of the array (for as long as the library is
// loaded in the process).  Its address is looked up once per device, with
// that device current, on the first call there; host code uses only that
// address, never the array's name.  Every call on a device shares the array:
// calls that overlap on one device race.  Nothing in the array needs to start
// at zero (every word a call reads was written earlier in the same call).
#include <mutex>

#include "internal.h"

static __device__ __align__(256) unsigned char scratch[PSFM_STATIC_SCRATCH_BYTES];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of this device's copy of `scratch` (looked up on first use).
int scratch_address(void** out) {
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return psfm::check_hip(e);
    if (dev < 0 || dev >= kMaxDevices) return PSFM_ERR_UNSUPPORTED;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) return psfm::check_hip(e != hipSuccess ? e : hipErrorUnknown);
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return PSFM_OK;
}

}  // namespace

extern "C" int psfm_match_pair_static(const psfm_context* ctx, const double* coeffs,
                                      const float* I1, const float* V1, const uint8_t* M1,
                                      const float* I2, const float* V2, const uint8_t* M2, int W,
                                      int H, int64_t pitch, const double* cov1, int cov1_half,
                                      const double* cov2, int cov2_half, float* conv,
                                      uint8_t* conv_mask, float* conv_var, double* cov_conv,
                                      int cov_conv_half, float* diff, float* diff_var,
                                      uint8_t* diff_mask, double* cov_diff, int cov_diff_half,
                                      psfm_fit_stats* stats, void* stream) {
    if (!ctx) return PSFM_ERR_INVALID_ARG;
    if (W < 1 || H < 1 || pitch < W) return PSFM_ERR_SHAPE;
    // the size limit is checked before anything else touches the device
    if (psfm::match_workspace(ctx, W, H) > PSFM_STATIC_SCRATCH_BYTES) return PSFM_ERR_WORKSPACE;
    void* ws = nullptr;
    const int rc = scratch_address(&ws);
    if (rc) return rc;
    return psfm::match_pair_ws(ctx, coeffs, I1, V1, M1, I2, V2, M2, W, H, pitch, cov1, cov1_half,
                               cov2, cov2_half, conv, conv_mask, conv_var, cov_conv, cov_conv_half,
                               diff, diff_var, diff_mask, cov_diff, cov_diff_half, stats, ws,
                               PSFM_STATIC_SCRATCH_BYTES, stream);
}
