// Batched matching of many independent image pairs.
//
// A plan lays the workspace out once: per pair the same scratch as the
// single-pair calls, plus a device array of pair descriptors and the
// flattened work lists (fit bands, stamps, 64 x 64 apply tiles) mapping each
// work item to its pair.  A run is then a fixed sequence of launches that
// each cover every pair (Sections 2-4 applied pair by pair):
//   k_batch_init                      clears the tile counters, start time
//   k_fit_band_b / k_fit_reduce_b     stamp normal equations of all pairs
//   solve loop (max_iter rounds)      assembly per spatial order,
//                                     one Cholesky workgroup per pair,
//                                     chi2 of all stamps, clip per pair
//   k_realise_b                       patch kernels of all pairs: FP32 taps and
//                                     BAD radii for the tile pass (stage 2)
//   k_cell_kernels_b / k_cov_auto_b / pseudo-matrices of the convolved images
//   k_cov_mix_b / k_cov_finish_b      (stage 2; each cell kernel realised once)
//   k_match_tiles_b                   (stage 3) fused convolution + difference over the
//                                     tiles of all pairs (grid-stride loop);
//                                     per-pair C_D and completion time
// Nothing in a run allocates or synchronises, so a run can be captured into
// one HIP graph and replayed.
#include <algorithm>
#include <cstdlib>
#include <cstring>
#include <numeric>
#include <vector>

#include "internal.h"

struct psfm_batch {
    const psfm_context* ctx;
    int n_pairs;
    int n_items, n_stamps, n_tiles, n_patches;
    int max_n, max_N, max_cov_in;
    int ns_off[psfm::PSFM_BATCH_NS_MAX + 1], ns_cnt[psfm::PSFM_BATCH_NS_MAX + 1];
    psfm_batch_tuning tuning;
    PairDesc* d_pairs;          // device (in the workspace)
    int* d_item_pair;
    int* d_stamp_pair;
    int* d_tile_pair;
    int* d_patch_pair;
    int* d_ns_pairs;
    unsigned* d_counters;
    uint64_t* times;
    hipGraph_t graph;
    hipGraphExec_t exec;
};

namespace {

__global__ void k_batch_init(unsigned* __restrict__ counters, int n_pairs, uint64_t* times) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n_pairs) counters[t] = 0u;
    if (t == 0 && times) times[0] = wall_clock64();
}

int n_spatial_of(int S) { return (S + 1) * (S + 2) / 2; }

struct PairSizes {
    int nbands, ns, N, L, ntx, nty, npatch, Rw, cov_in;
};

PairSizes sizes_of(const psfm_context* ctx, const psfm_pair& q) {
    PairSizes z;
    z.nbands = psfm::fit_bands(ctx);
    z.ns = n_spatial_of(q.spatial_order);
    z.N = ctx->nb * z.ns + 1;
    z.L = ctx->L;
    const int P = ctx->cfg.patch;
    const int tpp = (P + PSFM_TILE - 1) / PSFM_TILE;
    z.ntx = (q.width + P - 1) / P * tpp;
    z.nty = (q.height + P - 1) / P * tpp;
    z.npatch = ((q.width + P - 1) / P) * ((q.height + P - 1) / P);
    z.cov_in = q.cov1 ? q.cov1_half : 0;
    z.Rw = psfm::cov_sample_side(ctx, z.cov_in);
    return z;
}

int check_pair(const psfm_context* ctx, const psfm_pair& q) {
    if (q.width < 1 || q.height < 1 || q.pitch < q.width) return PSFM_ERR_SHAPE;
    if (q.n_stamps < 0 || q.spatial_order < 0 || q.spatial_order > 6) return PSFM_ERR_INVALID_ARG;
    if (!q.I1 || !q.V1 || !q.M1 || !q.I2 || !q.V2 || !q.M2 || (q.n_stamps > 0 && !q.stamp_xy))
        return PSFM_ERR_INVALID_ARG;
    if (!q.coeffs || !q.stats || !q.diff || !q.diff_var || !q.diff_mask || !q.cov_conv ||
        !q.cov_diff || (q.conv && !q.conv_mask))
        return PSFM_ERR_INVALID_ARG;
    if (q.cov1_half < 0 || q.cov2_half < 0 || q.cov_conv_half < 0 || q.cov_diff_half < 0)
        return PSFM_ERR_INVALID_ARG;
    if (q.cov1_half > 32 || q.cov_conv_half > 2 * ctx->h + 64) return PSFM_ERR_UNSUPPORTED;
    if (ctx->nb * n_spatial_of(q.spatial_order) + 1 > psfm::solve_max_unknowns())
        return PSFM_ERR_UNSUPPORTED;
    return PSFM_OK;
}

// Workspace layout of a batch.  With a null base the pointers are offsets.
struct Layout {
    PairDesc* pairs;
    int* item_pair;
    int* stamp_pair;
    int* tile_pair;
    int* patch_pair;
    int* ns_pairs;
    unsigned* counters;
    std::vector<PairDesc> desc;
    size_t bytes;
    int n_items = 0, n_stamps = 0, n_tiles = 0, n_patches = 0;
};

void lay_out(const psfm_context* ctx, const psfm_pair* q, const int* order, int n, void* base,
             Layout& Lo) {
    psfm::Carver c(base);
    for (int k = 0; k < n; k++) {
        const PairSizes z = sizes_of(ctx, q[k]);
        Lo.n_items += q[k].n_stamps * z.nbands;
        Lo.n_stamps += q[k].n_stamps;
        Lo.n_tiles += z.ntx * z.nty;
        Lo.n_patches += z.npatch;
    }
    Lo.pairs = c.take<PairDesc>(n);
    Lo.item_pair = c.take<int>(Lo.n_items + 1);
    Lo.stamp_pair = c.take<int>(Lo.n_stamps + 1);
    Lo.tile_pair = c.take<int>(Lo.n_tiles + 1);
    Lo.patch_pair = c.take<int>(Lo.n_patches + 1);
    Lo.ns_pairs = c.take<int>(n + 1);
    Lo.counters = c.take<unsigned>(n + 1);
    Lo.desc.assign(n, PairDesc{});
    int band_off = 0, stamp_off = 0, tile_off = 0, patch_off = 0;
    // fit and solve lists follow the given order; tiles follow `order`
    for (int k = 0; k < n; k++) {
        const psfm_pair& p = q[k];
        const PairSizes z = sizes_of(ctx, p);
        PairDesc& d = Lo.desc[k];
        const int ns_st = p.n_stamps;
        d.I1 = p.I1;
        d.V1 = p.V1;
        d.M1 = p.M1;
        d.I2 = p.I2;
        d.V2 = p.V2;
        d.M2 = p.M2;
        d.W = p.width;
        d.H = p.height;
        d.pitch = p.pitch;
        d.xy = p.stamp_xy;
        d.n = ns_st;
        d.S = p.spatial_order;
        d.ns = z.ns;
        d.N = z.N;
        d.Ms = c.take<double>((size_t)ns_st * z.L * z.L + 1);
        d.bs = c.take<double>((size_t)ns_st * z.L + 1);
        d.es = c.take<double>(ns_st + 1);
        d.npix = c.take<int32_t>(ns_st + 1);
        d.flags = p.stamp_flags ? p.stamp_flags : c.take<int32_t>(ns_st + 1);
        d.chi2 = p.stamp_chi2 ? p.stamp_chi2 : c.take<double>(ns_st + 1);
        d.coeffs = p.coeffs;
        d.stats = p.stats;
        d.st = c.take<SolveState>(1);
        d.used = c.take<uint8_t>(ns_st + 1);
        d.fitted = c.take<uint8_t>(ns_st + 1);
        d.G = c.take<double>((size_t)ns_st * z.ns + 1);
        d.A = c.take<double>((size_t)z.N * z.N);
        d.b = c.take<double>(z.N);
        d.ILg = c.take<double>(psfm::solve_il_doubles(z.N));
        d.part = c.take<double>((size_t)ns_st * z.nbands * PSFM_GRAM_COLS * PSFM_GRAM_COLS + 1);
        d.bflags = c.take<int>((size_t)ns_st * z.nbands + 1);
        d.cov1 = p.cov1;
        d.cov1_half = z.cov_in;
        d.cov2 = p.cov2;
        d.cov2_half = p.cov2 ? p.cov2_half : 0;
        d.conv = p.conv;
        d.conv_mask = p.conv_mask;
        d.var = p.conv_var;
        d.cov = p.cov_conv;
        d.cov_half = p.cov_conv_half;
        d.diff = p.diff;
        d.diff_var = p.diff_var;
        d.diff_mask = p.diff_mask;
        d.cov_diff = p.cov_diff;
        d.cov_diff_half = p.cov_diff_half;
        d.cov_samples = c.take<double>((size_t)PSFM_COV_SAMPLES * z.Rw * z.Rw);
        d.cov_auto = p.cov1 ? c.take<double>((size_t)PSFM_COV_SAMPLES * (4 * ctx->h + 1) * (4 * ctx->h + 1))
                            : nullptr;
        d.cov_avg = c.take<double>((size_t)z.Rw * z.Rw);
        d.sub_part = c.take<double>((size_t)4 * z.ntx * z.nty);
        d.ptaps = c.take<float>((size_t)z.npatch * psfm::patch_taps_floats(ctx->h));
        d.cellK = c.take<double>((size_t)PSFM_COV_SAMPLES * (2 * ctx->h + 1) * (2 * ctx->h + 1));
        d.patch_off = patch_off;
        patch_off += z.npatch;
        d.tiles_done = Lo.counters + k;
        d.t_done = nullptr;
        d.band_off = band_off;
        d.stamp_off = stamp_off;
        d.ntx = z.ntx;
        d.nty = z.nty;
        band_off += ns_st * z.nbands;
        stamp_off += ns_st;
    }
    for (int k = 0; k < n; k++) {
        PairDesc& d = Lo.desc[order[k]];
        d.tile_off = tile_off;
        tile_off += d.ntx * d.nty;
    }
    Lo.bytes = c.off;
}

}  // namespace

extern "C" size_t psfm_batch_workspace_bytes(const psfm_context* ctx, const psfm_pair* pairs,
                                             int n_pairs) {
    if (!ctx || n_pairs < 0 || (n_pairs > 0 && !pairs)) return 0;
    for (int k = 0; k < n_pairs; k++)
        if (check_pair(ctx, pairs[k]) != PSFM_OK) return 0;
    std::vector<int> order(n_pairs);
    std::iota(order.begin(), order.end(), 0);
    Layout Lo;
    lay_out(ctx, pairs, order.data(), n_pairs, nullptr, Lo);
    return Lo.bytes;
}

extern "C" int psfm_batch_plan(const psfm_context* ctx, const psfm_pair* pairs, int n_pairs,
                               const psfm_batch_tuning* tuning, void* ws, size_t ws_bytes,
                               uint64_t* times, void* stream, psfm_batch** out) {
    if (!ctx || !out || n_pairs < 1 || !pairs) return PSFM_ERR_INVALID_ARG;
    *out = nullptr;
    for (int k = 0; k < n_pairs; k++) {
        const int rc = check_pair(ctx, pairs[k]);
        if (rc) return rc;
    }
    if (psfm::fit_lds_bytes(ctx) > 160 * 1024 - 1024) return PSFM_ERR_UNSUPPORTED;
    if (ctx->cfg.precision != PSFM_PREC_FP32 || ctx->cfg.ortho_basis) return PSFM_ERR_UNSUPPORTED;
    psfm_batch_tuning tu{0, 0};
    if (tuning) tu = *tuning;
    if (tu.apply_grid < 0 || tu.order < 0 || tu.order > 2) return PSFM_ERR_INVALID_ARG;
    std::vector<int> order(n_pairs);
    std::iota(order.begin(), order.end(), 0);
    auto px = [&](int k) { return (long long)pairs[k].width * pairs[k].height; };
    if (tu.order == 1)
        std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return px(a) < px(b); });
    else if (tu.order == 2)
        std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return px(a) > px(b); });
    Layout probe;
    lay_out(ctx, pairs, order.data(), n_pairs, nullptr, probe);
    if (!ws || ws_bytes < probe.bytes) return PSFM_ERR_WORKSPACE;
    Layout Lo;
    lay_out(ctx, pairs, order.data(), n_pairs, ws, Lo);
    // work lists (host) -> workspace
    std::vector<int> item_pair(Lo.n_items + 1, 0), stamp_pair(Lo.n_stamps + 1, 0),
        tile_pair(Lo.n_tiles + 1, 0), patch_pair(Lo.n_patches + 1, 0);
    int max_n = 0, max_N = 0, max_cov_in = -1;   // -1: no pair has a correlated input
    for (int k = 0; k < n_pairs; k++) {
        const PairDesc& d = Lo.desc[k];
        const int nbands = psfm::fit_bands(ctx);
        for (int i = 0; i < d.n * nbands; i++) item_pair[d.band_off + i] = k;
        for (int i = 0; i < d.n; i++) stamp_pair[d.stamp_off + i] = k;
        for (int i = 0; i < d.ntx * d.nty; i++) tile_pair[d.tile_off + i] = k;
        const PairSizes z = sizes_of(ctx, pairs[k]);
        for (int i = 0; i < z.npatch; i++) patch_pair[d.patch_off + i] = k;
        max_n = std::max(max_n, d.n);
        max_N = std::max(max_N, d.N);
        max_cov_in = std::max(max_cov_in, d.cov1 ? d.cov1_half : -1);
        if (times) Lo.desc[k].t_done = times + 1 + k;
    }
    // the pairs of each spatial-term count, for the assembly launches
    int ns_off[psfm::PSFM_BATCH_NS_MAX + 1] = {}, ns_cnt[psfm::PSFM_BATCH_NS_MAX + 1] = {};
    std::vector<int> ns_pairs(n_pairs + 1, 0);
    for (int k = 0; k < n_pairs; k++) {
        if (Lo.desc[k].ns < 1 || Lo.desc[k].ns > psfm::PSFM_BATCH_NS_MAX) return PSFM_ERR_UNSUPPORTED;
        ns_cnt[Lo.desc[k].ns]++;
    }
    for (int v = 1, o = 0; v <= psfm::PSFM_BATCH_NS_MAX; v++) {
        ns_off[v] = o;
        o += ns_cnt[v];
    }
    {
        int fill[psfm::PSFM_BATCH_NS_MAX + 1] = {};
        for (int k = 0; k < n_pairs; k++) {
            const int v = Lo.desc[k].ns;
            ns_pairs[ns_off[v] + fill[v]++] = k;
        }
    }
    if (psfm::solve_lds_bytes(max_N) > 140 * 1024) return PSFM_ERR_UNSUPPORTED;
    hipStream_t st = (hipStream_t)stream;
    PSFM_HIP_CHECK(hipMemcpyAsync(Lo.pairs, Lo.desc.data(), sizeof(PairDesc) * n_pairs,
                                  hipMemcpyHostToDevice, st));
    PSFM_HIP_CHECK(hipMemcpyAsync(Lo.item_pair, item_pair.data(), sizeof(int) * item_pair.size(),
                                  hipMemcpyHostToDevice, st));
    PSFM_HIP_CHECK(hipMemcpyAsync(Lo.stamp_pair, stamp_pair.data(), sizeof(int) * stamp_pair.size(),
                                  hipMemcpyHostToDevice, st));
    PSFM_HIP_CHECK(hipMemcpyAsync(Lo.tile_pair, tile_pair.data(), sizeof(int) * tile_pair.size(),
                                  hipMemcpyHostToDevice, st));
    PSFM_HIP_CHECK(hipMemcpyAsync(Lo.patch_pair, patch_pair.data(), sizeof(int) * patch_pair.size(),
                                  hipMemcpyHostToDevice, st));
    PSFM_HIP_CHECK(hipMemcpyAsync(Lo.ns_pairs, ns_pairs.data(), sizeof(int) * ns_pairs.size(),
                                  hipMemcpyHostToDevice, st));
    PSFM_HIP_CHECK(hipStreamSynchronize(st));
    // grant dynamic LDS now, so that a later capture launches only kernels
    int rc = psfm::fit_prepare(ctx);
    if (rc) return rc;
    rc = psfm::solve_lds_grant(psfm::solve_lds_bytes(max_N));
    if (rc) return rc;
    psfm_batch* b = static_cast<psfm_batch*>(std::calloc(1, sizeof(psfm_batch)));
    if (!b) return PSFM_ERR_INVALID_ARG;
    b->ctx = ctx;
    b->n_pairs = n_pairs;
    b->n_items = Lo.n_items;
    b->n_stamps = Lo.n_stamps;
    b->n_tiles = Lo.n_tiles;
    b->n_patches = Lo.n_patches;
    b->max_n = max_n;
    b->max_N = max_N;
    b->max_cov_in = max_cov_in;
    std::copy(ns_off, ns_off + psfm::PSFM_BATCH_NS_MAX + 1, b->ns_off);
    std::copy(ns_cnt, ns_cnt + psfm::PSFM_BATCH_NS_MAX + 1, b->ns_cnt);
    b->tuning = tu;
    b->d_pairs = Lo.pairs;
    b->d_item_pair = Lo.item_pair;
    b->d_stamp_pair = Lo.stamp_pair;
    b->d_tile_pair = Lo.tile_pair;
    b->d_patch_pair = Lo.patch_pair;
    b->d_ns_pairs = Lo.ns_pairs;
    b->d_counters = Lo.counters;
    b->times = times;
    *out = b;
    return PSFM_OK;
}

extern "C" int psfm_batch_run_stage(psfm_batch* b, int stage, void* stream) {
    if (!b || stage < 0 || stage > 3) return PSFM_ERR_INVALID_ARG;
    hipStream_t st = (hipStream_t)stream;
    if (stage == 0) {
        hipLaunchKernelGGL(k_batch_init, dim3((b->n_pairs + 255) / 256), dim3(256), 0, st,
                           b->d_counters, b->n_pairs, b->times);
        PSFM_HIP_CHECK(hipGetLastError());
        return psfm::batch_fit(b->ctx, b->d_pairs, b->d_item_pair, b->d_stamp_pair, b->n_items,
                               b->n_stamps, st);
    }
    if (stage == 1)
        return psfm::batch_solve(b->ctx, b->d_pairs, b->d_stamp_pair, b->n_pairs, b->n_stamps,
                                 b->max_n, b->max_N, b->d_ns_pairs, b->ns_off, b->ns_cnt, st);
    return psfm::batch_apply(b->ctx, b->d_pairs, b->d_tile_pair, b->n_pairs, b->n_tiles,
                             b->d_patch_pair, b->n_patches, b->max_cov_in, b->tuning.apply_grid,
                             stage == 2 ? 1 : 2, st);
}

extern "C" int psfm_batch_run(psfm_batch* b, void* stream) {
    if (!b) return PSFM_ERR_INVALID_ARG;
    for (int stage = 0; stage < 4; stage++) {
        const int rc = psfm_batch_run_stage(b, stage, stream);
        if (rc) return rc;
    }
    return PSFM_OK;
}

static void drop_graph(psfm_batch* b) {
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    b->exec = nullptr;
    b->graph = nullptr;
}

extern "C" int psfm_batch_set_tuning(psfm_batch* b, const psfm_batch_tuning* tuning) {
    if (!b || !tuning || tuning->apply_grid < 0) return PSFM_ERR_INVALID_ARG;
    drop_graph(b);
    b->tuning.apply_grid = tuning->apply_grid;
    return PSFM_OK;
}

extern "C" int psfm_batch_graph_capture(psfm_batch* b, void* stream) {
    if (!b || !stream) return PSFM_ERR_INVALID_ARG;
    drop_graph(b);
    hipStream_t st = (hipStream_t)stream;
    PSFM_HIP_CHECK(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
    const int rc = psfm_batch_run(b, stream);
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(st, &g);
    if (rc) {
        if (g) (void)hipGraphDestroy(g);
        return rc;
    }
    PSFM_HIP_CHECK(e);
    b->graph = g;
    PSFM_HIP_CHECK(hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0));
    return PSFM_OK;
}

extern "C" int psfm_batch_graph_launch(psfm_batch* b, void* stream) {
    if (!b || !b->exec) return PSFM_ERR_INVALID_ARG;
    PSFM_HIP_CHECK(hipGraphLaunch(b->exec, (hipStream_t)stream));
    return PSFM_OK;
}

extern "C" int psfm_batch_destroy(psfm_batch* b) {
    if (!b) return PSFM_ERR_INVALID_ARG;
    drop_graph(b);
    std::free(b);
    return PSFM_OK;
}

// ---- several plans as the branches of one graph
struct psfm_batch_group {
    hipGraph_t graph;
    hipGraphExec_t exec;
};

constexpr int PSFM_BATCH_GROUP_MAX = 16;

extern "C" int psfm_batch_group_capture(psfm_batch* const* batches, int n, void* stream,
                                        psfm_batch_group** out) {
    if (!batches || n < 1 || n > PSFM_BATCH_GROUP_MAX || !stream || !out) return PSFM_ERR_INVALID_ARG;
    for (int i = 0; i < n; i++) {
        if (!batches[i]) return PSFM_ERR_INVALID_ARG;
        for (int j = 0; j < i; j++)
            if (batches[j] == batches[i]) return PSFM_ERR_INVALID_ARG;
    }
    hipStream_t st = (hipStream_t)stream;
    hipStream_t br[PSFM_BATCH_GROUP_MAX] = {};
    hipEvent_t ev[PSFM_BATCH_GROUP_MAX + 1] = {};
    int rc = PSFM_OK;
    auto release = [&]() {
        for (int i = 0; i < n; i++)
            if (br[i]) (void)hipStreamDestroy(br[i]);
        for (int i = 0; i <= n; i++)
            if (ev[i]) (void)hipEventDestroy(ev[i]);
    };
    auto ok = [](hipError_t e) { return e == hipSuccess ? PSFM_OK : psfm::check_hip(e); };
    for (int i = 0; i < n && rc == PSFM_OK; i++)
        rc = ok(hipStreamCreateWithFlags(&br[i], hipStreamNonBlocking));
    for (int i = 0; i <= n && rc == PSFM_OK; i++)
        rc = ok(hipEventCreateWithFlags(&ev[i], hipEventDisableTiming));
    if (rc) {
        release();
        return rc;
    }
    hipError_t e = hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) {
        release();
        return psfm::check_hip(e);
    }
    // fork, one branch per plan, join; every forked branch is joined even
    // after an error, so that the capture ends cleanly
    e = hipEventRecord(ev[n], st);
    for (int i = 0; i < n && e == hipSuccess; i++) {
        e = hipStreamWaitEvent(br[i], ev[n], 0);
        if (e != hipSuccess) break;
        if (rc == PSFM_OK) rc = psfm_batch_run(batches[i], br[i]);
        e = hipEventRecord(ev[i], br[i]);
        if (e == hipSuccess) e = hipStreamWaitEvent(st, ev[i], 0);
    }
    hipGraph_t g = nullptr;
    const hipError_t ee = hipStreamEndCapture(st, &g);
    release();
    if (rc == PSFM_OK && e != hipSuccess) rc = psfm::check_hip(e);
    if (rc == PSFM_OK && ee != hipSuccess) rc = psfm::check_hip(ee);
    if (rc) {
        if (g) (void)hipGraphDestroy(g);
        return rc;
    }
    psfm_batch_group* grp = static_cast<psfm_batch_group*>(std::calloc(1, sizeof(psfm_batch_group)));
    if (!grp) {
        (void)hipGraphDestroy(g);
        return PSFM_ERR_INVALID_ARG;
    }
    grp->graph = g;
    e = hipGraphInstantiate(&grp->exec, g, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        (void)hipGraphDestroy(g);
        std::free(grp);
        return psfm::check_hip(e);
    }
    *out = grp;
    return PSFM_OK;
}

extern "C" int psfm_batch_group_launch(psfm_batch_group* grp, void* stream) {
    if (!grp || !grp->exec) return PSFM_ERR_INVALID_ARG;
    PSFM_HIP_CHECK(hipGraphLaunch(grp->exec, (hipStream_t)stream));
    return PSFM_OK;
}

extern "C" int psfm_batch_group_destroy(psfm_batch_group* grp) {
    if (!grp) return PSFM_ERR_INVALID_ARG;
    if (grp->exec) (void)hipGraphExecDestroy(grp->exec);
    if (grp->graph) (void)hipGraphDestroy(grp->graph);
    std::free(grp);
    return PSFM_OK;
}

extern "C" double psfm_wall_clock_hz(void) {
    int dev = 0, khz = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0.0;
    if (hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev) != hipSuccess) return 0.0;
    return 1e3 * (double)khz;
}
