// Internal declarations shared by the HIP sources of liblegs.so (gfx950).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "legs.h"

#define LEGS_WAVE 64
#define LEGS_PROJ_BLOCK 256

struct legs_ctx {
    int device;
    int num_cus;
    char err[512];
};

// Error helpers (host side)
int32_t legs_set_error(legs_ctx *ctx, int32_t code, const char *fmt, ...);
#define LEGS_CHECK_HIP(ctx, expr)                                                            \
    do {                                                                                     \
        hipError_t e_ = (expr);                                                              \
        if (e_ != hipSuccess)                                                                \
            return legs_set_error((ctx), LEGS_ERR_HIP, "%s: %s (%s:%d)", #expr,              \
                                  hipGetErrorString(e_), __FILE__, __LINE__);                \
    } while (0)
#define LEGS_CHECK_LAUNCH(ctx) LEGS_CHECK_HIP(ctx, hipGetLastError())

// ---- device helpers ---------------------------------------------------------

__device__ __forceinline__ uint64_t legs_ballot(bool p) { return __builtin_amdgcn_ballot_w64(p); }

__device__ __forceinline__ int legs_lane() { return __lane_id(); }

// Tile -> view lookup over the view table (views sorted by tile_offset).
__device__ __forceinline__ int legs_view_of_tile(const legs_view *views, int n_views, int64_t tile)
{
    int lo = 0, hi = n_views - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (views[mid].tile_offset <= tile) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// Launchers implemented in the .hip files -------------------------------------
int32_t legs_launch_project(legs_ctx *ctx, const float *mean, const float *log_scale,
                            const float *quat, const float *opacity_logit, int64_t n,
                            const legs_view *views, int32_t n_views, const legs_opts *o,
                            legs_projected *out, hipStream_t s);
int32_t legs_launch_project_backward(legs_ctx *ctx, const float *mean, const float *log_scale,
                                     const float *quat, const float *opacity_logit, int64_t n,
                                     const legs_view *views, int32_t n_views, const legs_opts *o,
                                     const legs_projected *proj, const float *grad2d,
                                     float *d_mean, float *d_log_scale, float *d_quat,
                                     float *d_opacity_logit, hipStream_t s);
int32_t legs_launch_bin_sort(legs_ctx *ctx, const legs_projected *proj, int64_t n,
                             const legs_view *views, int32_t n_views, int64_t total_tiles,
                             const legs_opts *o, legs_bins *bins, int64_t *host_count,
                             hipStream_t s);
int32_t legs_launch_blend_forward(legs_ctx *ctx, const legs_projected *proj, int64_t n,
                                  const legs_bins *bins, const legs_view *views, int32_t n_views,
                                  int64_t total_tiles, const float *channels, int32_t C,
                                  const legs_opts *o, float *out, float *T_final, uint32_t *last,
                                  void *zero, int64_t zero_bytes, hipStream_t s);
int32_t legs_launch_blend_backward(legs_ctx *ctx, const legs_projected *proj, int64_t n,
                                   const legs_bins *bins, const legs_view *views, int32_t n_views,
                                   int64_t total_tiles, const float *channels, int32_t C,
                                   const legs_opts *o, const float *T_final, const uint32_t *last,
                                   const float *d_out, float *grad2d, float *d_channels,
                                   hipStream_t s);

int32_t legs_launch_blend_counts(legs_ctx *ctx, const legs_projected *proj, int64_t n,
                                 const legs_bins *bins, const legs_view *views, int32_t n_views,
                                 int64_t total_tiles, const legs_opts *o, uint64_t *counts,
                                 hipStream_t s);

// Sort scratch layout (bytes), shared by the sizing function and the launcher.
struct legs_sort_layout {
    int64_t hist_off;      // uint32 [8][256] digit histograms
    int64_t counter_off;   // uint32 [64] partition counters per pass, blend tile counters
    int64_t status_off;    // uint64 [8][parts][256] look-back status words
    int64_t parts;         // partitions at full capacity
    // depth-first binning only (total_tiles > 0):
    int64_t tcount_off;    // uint32 [total_tiles] per-tile instance counts
    int64_t scount_off;    // uint32 [total_tiles] per-super-tile counts (fewer super-tiles than tiles)
    int64_t cranges_off;   // uint32 [total_tiles][2] super-tile list ranges
    int64_t uoff_off;      // uint32 [total_tiles + 1] first compaction unit of each super-tile
    int64_t desc_off;      // uint32 [32] coarse digit layout, then uint64 [2] capacity cut
    int64_t ccap;          // coarse list capacity: capacity + total_tiles
    int64_t clist_off;     // uint32 [4][ccap] coarse keys and positions, two buffers each
    int64_t ucnt_off;      // uint32 [ccap / unit + total_tiles][32] per-unit tile counts / offsets
    int64_t udesc_off;     // [ccap / unit + total_tiles] 32-byte unit descriptors
    int64_t cpay_off;      // [ccap] 16-byte tile records of the sorted coarse list
    int64_t part_off;      // uint32 [LEGS_TILE_CHUNKS][total_tiles] partial tile-count grids
    int64_t spart_off;     // uint32 [LEGS_TILE_CHUNKS][total_tiles] partial super-tile-count grids
    int64_t seg_off;       // uint32 [2][LEGS_SEG_MAX][256] segment digit counts and starts
    int64_t order_off;     // uint32 [total_tiles] tiles by decreasing list length (persistent blending)
    int64_t total;
};
legs_sort_layout legs_sort_layout_for(int64_t capacity, int64_t total_tiles = 0);

#define LEGS_SORT_THREADS 512
#define LEGS_SORT_ITEMS 8
#define LEGS_SORT_PART (LEGS_SORT_THREADS * LEGS_SORT_ITEMS)
#define LEGS_SORT_MAX_PASSES 8
#define LEGS_TILE_CHUNKS 256
#define LEGS_SEG_MAX 1024
#define LEGS_COMPACT_UNIT 256
// counter slots (u32) in the sort scratch's counter block: 0..15 sort passes
#define LEGS_BLEND_COUNTER_FWD 32
#define LEGS_BLEND_COUNTER_BWD 33
