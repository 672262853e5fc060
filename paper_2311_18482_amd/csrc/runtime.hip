// Runtime around the kernels (gfx950): stream capture into HIP graphs, and the
// tile-size / LDS-batch autotuner for a batched multi-view workload.
//
// Graphs: every call after legs_project reads its sizes from device memory
// when legs_bin_sort runs without a host read-back, and the persistent blend
// kernels take tiles from a counter that a kernel (not a memset node) clears,
// so a whole forward + backward step can be captured once and replayed.
//
// Autotuner: the image is bit-identical for every tile size and LDS batch
// size (each pixel evaluates a Gaussian only inside its pixel box), so the
// choice only trades sort work (instances grow as the tile shrinks) against
// blending work (lists grow as the tile grows). It times the full step for
// each of the nine settings and returns the fastest. It is a set-up call: it
// allocates and frees its own buffers and waits on the stream.
#include <string.h>

#include <vector>

#include "legs_internal.h"

struct legs_graph {
    hipGraph_t graph;
    hipGraphExec_t exec;
};

extern "C" {

int32_t legs_capture_begin(legs_ctx *ctx, void *stream)
{
    if (!ctx) return LEGS_ERR_ARG;
    if (!stream) return legs_set_error(ctx, LEGS_ERR_ARG, "the legacy default stream cannot be captured");
    LEGS_CHECK_HIP(ctx, hipStreamBeginCapture((hipStream_t)stream, hipStreamCaptureModeThreadLocal));
    return LEGS_OK;
}

int32_t legs_capture_end(legs_ctx *ctx, void *stream, legs_graph **out)
{
    if (!ctx || !out) return LEGS_ERR_ARG;
    *out = nullptr;
    hipGraph_t g = nullptr;
    LEGS_CHECK_HIP(ctx, hipStreamEndCapture((hipStream_t)stream, &g));
    hipGraphExec_t e = nullptr;
    const hipError_t r = hipGraphInstantiate(&e, g, nullptr, nullptr, 0);
    if (r != hipSuccess) {
        hipGraphDestroy(g);
        return legs_set_error(ctx, LEGS_ERR_HIP, "hipGraphInstantiate: %s", hipGetErrorString(r));
    }
    legs_graph *lg = new legs_graph;
    lg->graph = g;
    lg->exec = e;
    *out = lg;
    return LEGS_OK;
}

int32_t legs_graph_launch(legs_ctx *ctx, legs_graph *graph, void *stream)
{
    if (!ctx || !graph) return LEGS_ERR_ARG;
    LEGS_CHECK_HIP(ctx, hipGraphLaunch(graph->exec, (hipStream_t)stream));
    return LEGS_OK;
}

int32_t legs_graph_destroy(legs_graph *graph)
{
    if (!graph) return LEGS_OK;
    hipGraphExecDestroy(graph->exec);
    hipGraphDestroy(graph->graph);
    delete graph;
    return LEGS_OK;
}

} // extern "C"

namespace {

// Device buffers of one autotuner trial, freed in the destructor.
struct Trial {
    std::vector<void *> ptrs;
    ~Trial()
    {
        for (void *p : ptrs) hipFree(p);
    }
    template <class T> T *alloc(int64_t count)
    {
        void *p = nullptr;
        if (hipMalloc(&p, (size_t)(count > 0 ? count : 1) * sizeof(T)) != hipSuccess) return nullptr;
        ptrs.push_back(p);
        return static_cast<T *>(p);
    }
};

} // namespace

extern "C" int32_t legs_autotune(legs_ctx *ctx, const float *mean, const float *log_scale,
                                 const float *quat, const float *opacity_logit,
                                 const float *channels, int64_t n, int32_t C,
                                 const legs_camera *cams_host, int32_t n_views,
                                 const legs_opts *base, const float *d_out, int32_t reps,
                                 legs_opts *best, float *ms_table, void *stream)
{
    if (!ctx || !best || !base || !cams_host || !mean || !log_scale || !quat || !opacity_logit ||
        !channels)
        return legs_set_error(ctx, LEGS_ERR_ARG, "NULL argument");
    if (n < 1 || C < 1 || C > LEGS_MAX_CHANNELS || n_views < 1 || n_views > LEGS_MAX_VIEWS || reps < 1)
        return legs_set_error(ctx, LEGS_ERR_ARG, "bad sizes");
    hipStream_t s = (hipStream_t)stream;
    const int tiles[3] = {8, 16, 32};
    const int batches[3] = {64, 128, 256};
    float best_ms = 1e30f;
    *best = *base;
    hipEvent_t e0, e1;
    LEGS_CHECK_HIP(ctx, hipEventCreate(&e0));
    LEGS_CHECK_HIP(ctx, hipEventCreate(&e1));
    int32_t rc = LEGS_OK;
    for (int ti = 0; ti < 3 && rc == LEGS_OK; ++ti) {
        legs_opts o = *base;
        o.tile = tiles[ti];
        std::vector<legs_view> vh((size_t)n_views);
        int64_t total_tiles = 0, total_px = 0;
        if (legs_views_build(cams_host, n_views, &o, vh.data(), &total_tiles, &total_px) != LEGS_OK) {
            rc = legs_set_error(ctx, LEGS_ERR_ARG, "invalid cameras");
            break;
        }
        Trial tr;
        legs_view *views = tr.alloc<legs_view>(n_views);
        const int64_t G = n * n_views, nb = legs_projected_blocks(n, n_views);
        legs_projected proj;
        proj.mean2d = tr.alloc<double>(2 * G);
        proj.conic = tr.alloc<float>(4 * G);
        proj.box = tr.alloc<int32_t>(4 * G);
        proj.depth = tr.alloc<float>(G);
        proj.ntiles = tr.alloc<uint32_t>(G);
        proj.block_offsets = tr.alloc<uint64_t>(2 * (nb + 1));
        proj.order = tr.alloc<char>(legs_order_scratch_bytes(n, n_views));
        float *out = tr.alloc<float>(C * total_px), *Tf = tr.alloc<float>(total_px);
        uint32_t *last = tr.alloc<uint32_t>(total_px);
        float *g2 = tr.alloc<float>(8 * G), *dch = tr.alloc<float>(n * C);
        float *dmu = tr.alloc<float>(3 * n), *dls = tr.alloc<float>(3 * n);
        float *dq = tr.alloc<float>(4 * n), *dom = tr.alloc<float>(n);
        if (!views || !proj.block_offsets || !out || !dom) {
            rc = legs_set_error(ctx, LEGS_ERR_HIP, "autotune: out of device memory");
            break;
        }
        if (hipMemcpyAsync(views, vh.data(), sizeof(legs_view) * n_views, hipMemcpyHostToDevice, s) != hipSuccess) {
            rc = legs_set_error(ctx, LEGS_ERR_HIP, "autotune: view table copy failed");
            break;
        }
        rc = legs_project(ctx, mean, log_scale, quat, opacity_logit, n, views, n_views, &o, &proj, stream);
        if (rc != LEGS_OK) break;
        // size the lists from a dry run with a one-element capacity
        legs_bins probe;
        probe.keys = tr.alloc<uint64_t>(1); probe.keys_alt = tr.alloc<uint64_t>(1);
        probe.ids = tr.alloc<uint32_t>(1); probe.ids_alt = tr.alloc<uint32_t>(1);
        probe.ranges = tr.alloc<uint32_t>(2 * total_tiles);
        probe.scratch = tr.alloc<char>(legs_sort_scratch_bytes(1, total_tiles));
        probe.count = tr.alloc<uint64_t>(1);
        probe.capacity = 1;
        int64_t count = 0;
        rc = legs_bin_sort(ctx, &proj, n, views, n_views, total_tiles, &o, &probe, &count, stream);
        if (rc != LEGS_OK && rc != LEGS_ERR_CAPACITY) break;
        rc = LEGS_OK;
        legs_bins bins;
        bins.capacity = count + 1024;
        bins.keys = tr.alloc<uint64_t>(bins.capacity); bins.keys_alt = tr.alloc<uint64_t>(bins.capacity);
        bins.ids = tr.alloc<uint32_t>(bins.capacity); bins.ids_alt = tr.alloc<uint32_t>(bins.capacity);
        bins.ranges = probe.ranges;
        bins.scratch = tr.alloc<char>(legs_sort_scratch_bytes(bins.capacity, total_tiles));
        bins.count = probe.count;
        if (!bins.keys || !bins.ids_alt || !bins.scratch) {
            rc = legs_set_error(ctx, LEGS_ERR_HIP, "autotune: out of device memory for %lld instances",
                                (long long)count);
            break;
        }
        for (int bi = 0; bi < 3 && rc == LEGS_OK; ++bi) {
            o.lds_batch = batches[bi];
            float ms = 0.f;
            for (int r = -1; r < reps && rc == LEGS_OK; ++r) {   // r = -1 is the warm-up
                if (r == 0) hipEventRecord(e0, s);
                rc = legs_project(ctx, mean, log_scale, quat, opacity_logit, n, views, n_views, &o, &proj, stream);
                if (rc == LEGS_OK) rc = legs_bin_sort(ctx, &proj, n, views, n_views, total_tiles, &o, &bins, nullptr, stream);
                if (rc == LEGS_OK) rc = legs_render_forward(ctx, &proj, n, &bins, views, n_views, total_tiles, channels, C, &o, out, Tf, last, stream);
                if (rc == LEGS_OK && d_out) {
                    rc = legs_clear(ctx, g2, (int64_t)sizeof(float) * 8 * G, stream);
                    if (rc == LEGS_OK) rc = legs_clear(ctx, dch, (int64_t)sizeof(float) * n * C, stream);
                    if (rc == LEGS_OK)
                        rc = legs_render_backward(ctx, &proj, n, &bins, views, n_views, total_tiles, channels, C, &o, Tf, last, d_out, g2, dch, stream);
                    if (rc == LEGS_OK)
                        rc = legs_project_backward(ctx, mean, log_scale, quat, opacity_logit, n, views, n_views, &o, &proj, g2, dmu, dls, dq, dom, stream);
                }
            }
            if (rc != LEGS_OK) break;
            hipEventRecord(e1, s);
            hipEventSynchronize(e1);
            hipEventElapsedTime(&ms, e0, e1);
            ms /= (float)reps;
            if (ms_table) ms_table[ti * 3 + bi] = ms;
            if (ms < best_ms) {
                best_ms = ms;
                *best = o;
            }
        }
        hipStreamSynchronize(s);
    }
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    return rc;
}
