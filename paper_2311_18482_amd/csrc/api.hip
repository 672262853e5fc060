// C ABI entry points of liblegs.so: argument validation, then the launchers
// in project.hip, sort.hip and blend.hip. See include/legs.h for the contract
// of each call.
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <atomic>
#include <mutex>

#include "legs_internal.h"
#include "legs_decode_internal.h"

// Workspace of legs_semantic_loss_grad_noalloc: LEGS_NOALLOC_MAX_PIXELS rows of
// the decoder-training workspace at the largest K (21,495,808 bytes). Every GPU
// that loads the library holds its own copy until the process ends. In host
// code `scratch` is only a stand-in for the symbol: the device address of a
// GPU's copy comes from hipGetSymbolAddress with that GPU current, once per
// device (in legs_create), and only that address is handed to kernels.
static __device__ __align__(256) float scratch[(size_t)LEGS_NOALLOC_MAX_PIXELS * LEGS_MLP_WS_PER_PIXEL(128)];

namespace {

constexpr int kScratchDevices = 64;
std::mutex g_scratch_mu;
std::atomic<float *> g_scratch[kScratchDevices];

int32_t scratch_setup(legs_ctx *ctx)
{
    if (ctx->device >= kScratchDevices)
        return legs_set_error(ctx, LEGS_ERR_UNSUPPORTED, "device %d beyond the %d with a scratch table",
                              ctx->device, kScratchDevices);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (g_scratch[ctx->device].load()) return LEGS_OK;
    int prev = -1;
    LEGS_CHECK_HIP(ctx, hipGetDevice(&prev));
    LEGS_CHECK_HIP(ctx, hipSetDevice(ctx->device));
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    LEGS_CHECK_HIP(ctx, hipSetDevice(prev));
    if (e != hipSuccess || !p)
        return legs_set_error(ctx, LEGS_ERR_HIP, "hipGetSymbolAddress(scratch) on device %d: %s",
                              ctx->device, hipGetErrorString(e));
    g_scratch[ctx->device].store(static_cast<float *>(p));
    return LEGS_OK;
}

} // namespace

int32_t legs_set_error(legs_ctx *ctx, int32_t code, const char *fmt, ...)
{
    if (ctx) {
        va_list ap;
        va_start(ap, fmt);
        vsnprintf(ctx->err, sizeof ctx->err, fmt, ap);
        va_end(ap);
    }
    return code;
}

namespace {

int32_t check_opts(legs_ctx *ctx, const legs_opts *o)
{
    if (!o) return legs_set_error(ctx, LEGS_ERR_ARG, "opts is NULL");
    if (o->tile != 8 && o->tile != 16 && o->tile != 32)
        return legs_set_error(ctx, LEGS_ERR_ARG, "tile %d not in {8, 16, 32}", o->tile);
    if (o->lds_batch != 64 && o->lds_batch != 128 && o->lds_batch != 256)
        return legs_set_error(ctx, LEGS_ERR_ARG, "lds_batch %d not in {64, 128, 256}", o->lds_batch);
    if (!(o->alpha_max > 0.f && o->alpha_max < 1.f) || !(o->alpha_min >= 0.f) || !(o->t_min > 0.f))
        return legs_set_error(ctx, LEGS_ERR_ARG, "alpha/transmittance thresholds out of range");
    if (!(o->z_near > 0.0) || !(o->guard > 0.0) || !(o->lowpass >= 0.0))
        return legs_set_error(ctx, LEGS_ERR_ARG, "z_near/guard/lowpass out of range");
    return LEGS_OK;
}

int32_t check_views(legs_ctx *ctx, const legs_view *views, int32_t n_views)
{
    if (!views) return legs_set_error(ctx, LEGS_ERR_ARG, "views is NULL");
    if (n_views < 1 || n_views > LEGS_MAX_VIEWS)
        return legs_set_error(ctx, LEGS_ERR_ARG, "n_views %d out of [1, %d]", n_views, LEGS_MAX_VIEWS);
    return LEGS_OK;
}

int32_t use_device(legs_ctx *ctx)
{
    int cur = -1;
    LEGS_CHECK_HIP(ctx, hipGetDevice(&cur));
    if (cur != ctx->device) LEGS_CHECK_HIP(ctx, hipSetDevice(ctx->device));
    return LEGS_OK;
}

bool proj_ok(const legs_projected *p)
{
    return p && p->mean2d && p->conic && p->box && p->depth && p->ntiles && p->block_offsets;
}

bool bins_ok(const legs_bins *b)
{
    return b && b->keys && b->keys_alt && b->ids && b->ids_alt && b->ranges && b->scratch &&
           b->count && b->capacity >= 0;
}

} // namespace

#define LEGS_TRY(expr)                  \
    do {                                \
        int32_t r_ = (expr);            \
        if (r_ != LEGS_OK) return r_;   \
    } while (0)

extern "C" {

int32_t legs_version(void) { return 1; }

void legs_opts_default(legs_opts *o)
{
    if (!o) return;
    memset(o, 0, sizeof *o);
    o->tile = 16;
    o->lds_batch = 256;
    o->alpha_max = 0.99f;
    o->alpha_min = 1.0f / 255.0f;
    o->t_min = 1e-4f;
    o->lowpass = 0.3;
    o->z_near = 0.2;
    o->guard = 1.3;
}

int32_t legs_create(int32_t device, legs_ctx **out)
{
    if (!out) return LEGS_ERR_ARG;
    *out = nullptr;
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || device < 0 || device >= count)
        return LEGS_ERR_ARG;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) != hipSuccess) return LEGS_ERR_HIP;
    if (strncmp(prop.gcnArchName, "gfx950", 6) != 0) return LEGS_ERR_UNSUPPORTED;
    legs_ctx *c = new legs_ctx;
    c->device = device;
    c->num_cus = prop.multiProcessorCount;
    c->err[0] = 0;
    const int32_t rc = scratch_setup(c);
    if (rc != LEGS_OK) {
        fprintf(stderr, "legs_create: %s\n", c->err);
        delete c;
        return rc;
    }
    *out = c;
    return LEGS_OK;
}

int32_t legs_destroy(legs_ctx *ctx)
{
    delete ctx;
    return LEGS_OK;
}

const char *legs_last_error(const legs_ctx *ctx) { return ctx ? ctx->err : "no context"; }

int32_t legs_views_build(const legs_camera *cams, int32_t n_views, const legs_opts *opts,
                         legs_view *out_host, int64_t *total_tiles, int64_t *total_pixels)
{
    if (!cams || !opts || !out_host || n_views < 1 || n_views > LEGS_MAX_VIEWS) return LEGS_ERR_ARG;
    const int T = opts->tile;
    if (T != 8 && T != 16 && T != 32) return LEGS_ERR_ARG;
    int64_t tiles = 0, pix = 0;
    for (int32_t v = 0; v < n_views; ++v) {
        const legs_camera &c = cams[v];
        if (c.width < 1 || c.height < 1 || c.width > 32767 || c.height > 32767) return LEGS_ERR_ARG;
        if (!(c.fx > 0.0) || !(c.fy > 0.0)) return LEGS_ERR_ARG;
        legs_view &w = out_host[v];
        w.cam = c;
        w.tiles_x = (c.width + T - 1) / T;
        w.tiles_y = (c.height + T - 1) / T;
        w.tile_offset = tiles;
        w.pixel_offset = pix;
        tiles += (int64_t)w.tiles_x * w.tiles_y;
        pix += (int64_t)c.width * c.height;
    }
    if (tiles >= (1ll << 32)) return LEGS_ERR_ARG;
    if (total_tiles) *total_tiles = tiles;
    if (total_pixels) *total_pixels = pix;
    return LEGS_OK;
}

int64_t legs_projected_blocks(int64_t n, int32_t n_views)
{
    if (n < 0 || n_views < 1) return -1;
    return ((n + LEGS_PROJ_BLOCK - 1) / LEGS_PROJ_BLOCK) * (int64_t)n_views;
}

int64_t legs_sort_scratch_bytes(int64_t capacity, int64_t total_tiles)
{
    if (capacity < 0 || total_tiles < 0) return -1;
    return legs_sort_layout_for(capacity, total_tiles).total;
}

int32_t legs_sort_passes(int64_t total_tiles)
{
    int bits = 0;
    while (bits < 32 && (1ll << bits) < total_tiles) ++bits;
    return (32 + bits + 7) / 8;
}

int32_t legs_project(legs_ctx *ctx, const float *mean, const float *log_scale, const float *quat,
                     const float *opacity_logit, int64_t n, const legs_view *views_dev,
                     int32_t n_views, const legs_opts *opts, legs_projected *out, void *stream)
{
    if (!ctx) return LEGS_ERR_ARG;
    if (n < 0 || n >= (1ll << 32)) return legs_set_error(ctx, LEGS_ERR_ARG, "n out of range");
    if (n > 0 && (!mean || !log_scale || !quat || !opacity_logit))
        return legs_set_error(ctx, LEGS_ERR_ARG, "NULL Gaussian parameter");
    if (!proj_ok(out)) return legs_set_error(ctx, LEGS_ERR_ARG, "incomplete projected buffers");
    LEGS_TRY(check_opts(ctx, opts));
    LEGS_TRY(check_views(ctx, views_dev, n_views));
    LEGS_TRY(use_device(ctx));
    return legs_launch_project(ctx, mean, log_scale, quat, opacity_logit, n, views_dev, n_views,
                               opts, out, (hipStream_t)stream);
}

int32_t legs_bin_sort(legs_ctx *ctx, const legs_projected *proj, int64_t n,
                      const legs_view *views_dev, int32_t n_views, int64_t total_tiles,
                      const legs_opts *opts, legs_bins *bins, int64_t *host_count, void *stream)
{
    if (!ctx) return LEGS_ERR_ARG;
    if (n < 0 || n >= (1ll << 32)) return legs_set_error(ctx, LEGS_ERR_ARG, "n out of range");
    if (!proj_ok(proj)) return legs_set_error(ctx, LEGS_ERR_ARG, "incomplete projected buffers");
    if (!bins_ok(bins)) return legs_set_error(ctx, LEGS_ERR_ARG, "incomplete bin buffers");
    if (bins->capacity >= (1ll << 32))
        return legs_set_error(ctx, LEGS_ERR_ARG, "capacity must be below 2^32");
    if (total_tiles < 1 || total_tiles >= (1ll << 32))
        return legs_set_error(ctx, LEGS_ERR_ARG, "total_tiles out of range");
    LEGS_TRY(check_opts(ctx, opts));
    LEGS_TRY(check_views(ctx, views_dev, n_views));
    LEGS_TRY(use_device(ctx));
    return legs_launch_bin_sort(ctx, proj, n, views_dev, n_views, total_tiles, opts, bins,
                                host_count, (hipStream_t)stream);
}

int32_t legs_render_forward(legs_ctx *ctx, const legs_projected *proj, int64_t n,
                            const legs_bins *bins, const legs_view *views_dev, int32_t n_views,
                            int64_t total_tiles, const float *channels, int32_t C,
                            const legs_opts *opts, float *out, float *T_final, uint32_t *last,
                            void *stream)
{
    if (!ctx) return LEGS_ERR_ARG;
    if (!proj_ok(proj) || !bins_ok(bins)) return legs_set_error(ctx, LEGS_ERR_ARG, "incomplete buffers");
    if (C < 1 || C > LEGS_MAX_CHANNELS) return legs_set_error(ctx, LEGS_ERR_ARG, "C out of range");
    if ((n > 0 && !channels) || !out || !T_final || !last)
        return legs_set_error(ctx, LEGS_ERR_ARG, "NULL output or channels");
    if (total_tiles < 1 || total_tiles >= (1ll << 32))
        return legs_set_error(ctx, LEGS_ERR_ARG, "total_tiles out of range");
    LEGS_TRY(check_opts(ctx, opts));
    LEGS_TRY(check_views(ctx, views_dev, n_views));
    LEGS_TRY(use_device(ctx));
    return legs_launch_blend_forward(ctx, proj, n, bins, views_dev, n_views, total_tiles, channels,
                                     C, opts, out, T_final, last, nullptr, 0, (hipStream_t)stream);
}

int32_t legs_render_forward_zero(legs_ctx *ctx, const legs_projected *proj, int64_t n,
                                 const legs_bins *bins, const legs_view *views_dev, int32_t n_views,
                                 int64_t total_tiles, const float *channels, int32_t C,
                                 const legs_opts *opts, float *out, float *T_final, uint32_t *last,
                                 void *zero, int64_t zero_bytes, void *stream)
{
    if (!ctx) return LEGS_ERR_ARG;
    if (!proj_ok(proj) || !bins_ok(bins)) return legs_set_error(ctx, LEGS_ERR_ARG, "incomplete buffers");
    if (C < 1 || C > LEGS_MAX_CHANNELS) return legs_set_error(ctx, LEGS_ERR_ARG, "C out of range");
    if ((n > 0 && !channels) || !out || !T_final || !last)
        return legs_set_error(ctx, LEGS_ERR_ARG, "NULL output or channels");
    if (total_tiles < 1 || total_tiles >= (1ll << 32))
        return legs_set_error(ctx, LEGS_ERR_ARG, "total_tiles out of range");
    if (zero_bytes < 0 || zero_bytes % 4 != 0 || (zero_bytes > 0 && !zero) ||
        (reinterpret_cast<uintptr_t>(zero) & 15) != 0)
        return legs_set_error(ctx, LEGS_ERR_ARG,
                              "legs_render_forward_zero: zero must be 16-byte aligned and zero_bytes a "
                              "non-negative multiple of 4");
    LEGS_TRY(check_opts(ctx, opts));
    LEGS_TRY(check_views(ctx, views_dev, n_views));
    LEGS_TRY(use_device(ctx));
    return legs_launch_blend_forward(ctx, proj, n, bins, views_dev, n_views, total_tiles, channels,
                                     C, opts, out, T_final, last, zero, zero_bytes, (hipStream_t)stream);
}

int32_t legs_render_backward(legs_ctx *ctx, const legs_projected *proj, int64_t n,
                             const legs_bins *bins, const legs_view *views_dev, int32_t n_views,
                             int64_t total_tiles, const float *channels, int32_t C,
                             const legs_opts *opts, const float *T_final, const uint32_t *last,
                             const float *d_out, float *grad2d, float *d_channels, void *stream)
{
    if (!ctx) return LEGS_ERR_ARG;
    if (!proj_ok(proj) || !bins_ok(bins)) return legs_set_error(ctx, LEGS_ERR_ARG, "incomplete buffers");
    if (C < 1 || C > LEGS_MAX_CHANNELS) return legs_set_error(ctx, LEGS_ERR_ARG, "C out of range");
    if ((n > 0 && !channels) || !T_final || !last || !d_out || !grad2d || !d_channels)
        return legs_set_error(ctx, LEGS_ERR_ARG, "NULL input or gradient buffer");
    if (total_tiles < 1 || total_tiles >= (1ll << 32))
        return legs_set_error(ctx, LEGS_ERR_ARG, "total_tiles out of range");
    LEGS_TRY(check_opts(ctx, opts));
    LEGS_TRY(check_views(ctx, views_dev, n_views));
    LEGS_TRY(use_device(ctx));
    return legs_launch_blend_backward(ctx, proj, n, bins, views_dev, n_views, total_tiles,
                                      channels, C, opts, T_final, last, d_out, grad2d, d_channels,
                                      (hipStream_t)stream);
}

int32_t legs_render_counts(legs_ctx *ctx, const legs_projected *proj, int64_t n,
                           const legs_bins *bins, const legs_view *views_dev, int32_t n_views,
                           int64_t total_tiles, const legs_opts *opts, uint64_t *counts,
                           void *stream)
{
    if (!ctx) return LEGS_ERR_ARG;
    if (!proj_ok(proj) || !bins_ok(bins) || !counts)
        return legs_set_error(ctx, LEGS_ERR_ARG, "incomplete buffers");
    if (total_tiles < 1 || total_tiles >= (1ll << 32))
        return legs_set_error(ctx, LEGS_ERR_ARG, "total_tiles out of range");
    LEGS_TRY(check_opts(ctx, opts));
    LEGS_TRY(check_views(ctx, views_dev, n_views));
    LEGS_TRY(use_device(ctx));
    return legs_launch_blend_counts(ctx, proj, n, bins, views_dev, n_views, total_tiles, opts,
                                    counts, (hipStream_t)stream);
}

int32_t legs_project_backward(legs_ctx *ctx, const float *mean, const float *log_scale,
                              const float *quat, const float *opacity_logit, int64_t n,
                              const legs_view *views_dev, int32_t n_views, const legs_opts *opts,
                              const legs_projected *proj, const float *grad2d, float *d_mean,
                              float *d_log_scale, float *d_quat, float *d_opacity_logit,
                              void *stream)
{
    if (!ctx) return LEGS_ERR_ARG;
    if (n < 0 || n >= (1ll << 32)) return legs_set_error(ctx, LEGS_ERR_ARG, "n out of range");
    if (n > 0 && (!mean || !log_scale || !quat || !opacity_logit || !grad2d || !d_mean ||
                  !d_log_scale || !d_quat || !d_opacity_logit))
        return legs_set_error(ctx, LEGS_ERR_ARG, "NULL parameter or gradient");
    if (!proj_ok(proj)) return legs_set_error(ctx, LEGS_ERR_ARG, "incomplete projected buffers");
    LEGS_TRY(check_opts(ctx, opts));
    LEGS_TRY(check_views(ctx, views_dev, n_views));
    LEGS_TRY(use_device(ctx));
    return legs_launch_project_backward(ctx, mean, log_scale, quat, opacity_logit, n, views_dev,
                                        n_views, opts, proj, grad2d, d_mean, d_log_scale, d_quat,
                                        d_opacity_logit, (hipStream_t)stream);
}


static int32_t check_feat(legs_ctx *ctx, const float *feat, int64_t P, int64_t cs, int64_t ps,
                          int32_t K, int32_t *top1)
{
    if (P < 0) return legs_set_error(ctx, LEGS_ERR_ARG, "P < 0");
    if (P > 0 && (!feat || !top1)) return legs_set_error(ctx, LEGS_ERR_ARG, "NULL feat or top1");
    if (cs < 0 || ps < 0) return legs_set_error(ctx, LEGS_ERR_ARG, "negative stride");
    if (K != 32 && K != 64 && K != 128) return legs_set_error(ctx, LEGS_ERR_ARG, "K must be 32, 64 or 128");
    return LEGS_OK;
}

int32_t legs_decode_plain(legs_ctx *ctx, const float *feat, int64_t P, int64_t c_stride,
                          int64_t p_stride, const float *proj, int32_t D, const float *codebook,
                          int32_t K, float *probs, int32_t *top1, void *stream)
{
    if (!ctx) return LEGS_ERR_ARG;
    LEGS_TRY(check_feat(ctx, feat, P, c_stride, p_stride, K, top1));
    if (!proj || !codebook) return legs_set_error(ctx, LEGS_ERR_ARG, "NULL proj or codebook");
    if (D < 32 || D > LEGS_DECODE_MAXD || D % 32)
        return legs_set_error(ctx, LEGS_ERR_ARG, "D must be a multiple of 32 in [32, %d]", LEGS_DECODE_MAXD);
    LEGS_TRY(use_device(ctx));
    return legs_launch_decode_plain(ctx, feat, P, c_stride, p_stride, proj, D, codebook, K, probs,
                                    top1, (hipStream_t)stream);
}

int32_t legs_decode_fold(legs_ctx *ctx, const float *proj, int32_t D, const float *codebook,
                         int32_t K, float *folded, void *stream)
{
    if (!ctx) return LEGS_ERR_ARG;
    if (!proj || !codebook || !folded) return legs_set_error(ctx, LEGS_ERR_ARG, "NULL argument");
    if (D < 1 || (K != 32 && K != 64 && K != 128)) return legs_set_error(ctx, LEGS_ERR_ARG, "bad D or K");
    LEGS_TRY(use_device(ctx));
    return legs_launch_decode_fold(ctx, proj, D, codebook, K, folded, (hipStream_t)stream);
}

int32_t legs_decode_folded(legs_ctx *ctx, const float *feat, int64_t P, int64_t c_stride,
                           int64_t p_stride, const float *folded, int32_t K, float *probs,
                           int32_t *top1, void *stream)
{
    if (!ctx) return LEGS_ERR_ARG;
    LEGS_TRY(check_feat(ctx, feat, P, c_stride, p_stride, K, top1));
    if (!folded) return legs_set_error(ctx, LEGS_ERR_ARG, "NULL folded");
    LEGS_TRY(use_device(ctx));
    return legs_launch_decode_folded(ctx, feat, P, c_stride, p_stride, folded, K, probs, top1,
                                     (hipStream_t)stream);
}

int64_t legs_mlp_param_count(int32_t K)
{
    if (K != 32 && K != 64 && K != 128) return -1;
    return LEGS_MLP_NPARAMS(K / 32);
}

static int32_t check_mlp_flags(legs_ctx *ctx, int32_t mlp_flags)
{
    if (mlp_flags & ~LEGS_MLP_NORMALIZE_INPUT) return legs_set_error(ctx, LEGS_ERR_ARG, "unknown mlp_flags bits");
    return LEGS_OK;
}

int32_t legs_decode_mlp(legs_ctx *ctx, const float *feat, int64_t P, int64_t c_stride,
                        int64_t p_stride, const float *params, int32_t K, int32_t mlp_flags,
                        float *probs, int32_t *top1, void *stream)
{
    if (!ctx) return LEGS_ERR_ARG;
    LEGS_TRY(check_feat(ctx, feat, P, c_stride, p_stride, K, top1));
    LEGS_TRY(check_mlp_flags(ctx, mlp_flags));
    if (!params) return legs_set_error(ctx, LEGS_ERR_ARG, "NULL params");
    LEGS_TRY(use_device(ctx));
    return legs_launch_decode_mlp(ctx, feat, P, c_stride, p_stride, params, K, mlp_flags, probs, top1,
                                  (hipStream_t)stream);
}

int64_t legs_mlp_workspace_bytes(int64_t B, int32_t K)
{
    if (B < 0 || (K != 32 && K != 64 && K != 128)) return -1;
    return 4 * legs_mlp_workspace_floats(B, K);
}

int32_t legs_mlp_grad(legs_ctx *ctx, const float *feat, int64_t B, int64_t c_stride,
                      int64_t p_stride, const int32_t *labels, int32_t K, int32_t mlp_flags,
                      const float *params, void *workspace, float *grad, float *loss, void *stream)
{
    if (!ctx) return LEGS_ERR_ARG;
    LEGS_TRY(check_mlp_flags(ctx, mlp_flags));
    if (B < 0 || B > (1ll << 31)) return legs_set_error(ctx, LEGS_ERR_ARG, "B out of range");
    if (K != 32 && K != 64 && K != 128) return legs_set_error(ctx, LEGS_ERR_ARG, "K must be 32, 64 or 128");
    if (!params || !grad || !loss || (B > 0 && (!feat || !labels || !workspace)))
        return legs_set_error(ctx, LEGS_ERR_ARG, "NULL argument");
    if (c_stride < 0 || p_stride < 0) return legs_set_error(ctx, LEGS_ERR_ARG, "negative stride");
    LEGS_TRY(use_device(ctx));
    return legs_launch_mlp_grad(ctx, feat, B, c_stride, p_stride, labels, K, mlp_flags, params,
                                static_cast<float *>(workspace), grad, loss, (hipStream_t)stream);
}

int32_t legs_semantic_loss_grad(legs_ctx *ctx, const float *feat, const float *ru, int64_t P,
                                int64_t c_stride, int64_t p_stride, const int32_t *labels,
                                int32_t K, int32_t mlp_flags, const float *params, float lambda_ce,
                                float lambda_u, float inv_hw, void *workspace, float *grad,
                                float *d_feat, int64_t d_c_stride, int64_t d_p_stride, float *d_ru,
                                float *loss, void *stream)
{
    if (!ctx) return LEGS_ERR_ARG;
    if (P < 0 || P > (1ll << 31)) return legs_set_error(ctx, LEGS_ERR_ARG, "P out of range");
    if (K != 32 && K != 64 && K != 128) return legs_set_error(ctx, LEGS_ERR_ARG, "K must be 32, 64 or 128");
    LEGS_TRY(check_mlp_flags(ctx, mlp_flags));
    if (!params || !grad || !loss ||
        (P > 0 && (!feat || !ru || !labels || !workspace || !d_feat || !d_ru)))
        return legs_set_error(ctx, LEGS_ERR_ARG, "NULL argument");
    if (c_stride < 0 || p_stride < 0 || d_c_stride < 0 || d_p_stride < 0)
        return legs_set_error(ctx, LEGS_ERR_ARG, "negative stride");
    if (!(inv_hw >= 0.0f) || !(lambda_ce >= 0.0f) || !(lambda_u >= 0.0f))
        return legs_set_error(ctx, LEGS_ERR_ARG, "negative or NaN weight");
    LEGS_TRY(use_device(ctx));
    return legs_launch_semantic_loss_grad(ctx, feat, ru, P, c_stride, p_stride, labels, K, mlp_flags,
                                          params, lambda_ce, lambda_u, inv_hw,
                                          static_cast<float *>(workspace), grad, d_feat, d_c_stride,
                                          d_p_stride, d_ru, loss, (hipStream_t)stream);
}

int64_t legs_dmlp_param_count(int32_t N)
{
    return (N == 32 || N == 64 || N == 128) ? (int64_t)LEGS_DMLP_NPARAMS(N / 32) : -1;
}

int32_t legs_decode_dmlp(legs_ctx *ctx, const float *feat, int64_t P, int64_t c_stride, int64_t p_stride,
                         const float *params, int32_t N, int32_t mlp_flags, float *probs, uint16_t *probs_f16,
                         int32_t *top1, void *stream)
{
    if (!ctx) return LEGS_ERR_ARG;
    if (P < 0 || P > (1ll << 40)) return legs_set_error(ctx, LEGS_ERR_ARG, "P out of range");
    if (N != 32 && N != 64 && N != 128) return legs_set_error(ctx, LEGS_ERR_ARG, "N must be 32, 64 or 128");
    LEGS_TRY(check_mlp_flags(ctx, mlp_flags));
    if (!params || (P > 0 && !feat)) return legs_set_error(ctx, LEGS_ERR_ARG, "NULL argument");
    if (!probs && !probs_f16 && !top1) return legs_set_error(ctx, LEGS_ERR_ARG, "no output requested");
    if (c_stride < 0 || p_stride < 0) return legs_set_error(ctx, LEGS_ERR_ARG, "negative stride");
    if ((reinterpret_cast<uintptr_t>(probs) & 15) || (reinterpret_cast<uintptr_t>(probs_f16) & 15))
        return legs_set_error(ctx, LEGS_ERR_ARG, "probs and probs_f16 must be 16-byte aligned");
    LEGS_TRY(use_device(ctx));
    return legs_launch_decode_dmlp(ctx, feat, P, c_stride, p_stride, params, N, mlp_flags, probs, probs_f16,
                                   top1, (hipStream_t)stream);
}

int32_t legs_language_features(legs_ctx *ctx, const uint16_t *probs_f16, int64_t P, int32_t N,
                               const float *S, int32_t d, int32_t out_f16, void *F, void *stream)
{
    if (!ctx) return LEGS_ERR_ARG;
    if (P < 0 || P > (1ll << 40)) return legs_set_error(ctx, LEGS_ERR_ARG, "P out of range");
    if (N != 32 && N != 64 && N != 128) return legs_set_error(ctx, LEGS_ERR_ARG, "N must be 32, 64 or 128");
    if (d < 32 || d > 4096 || d % 32) return legs_set_error(ctx, LEGS_ERR_ARG, "d must be a multiple of 32 in [32, 4096]");
    if (!S || (P > 0 && (!probs_f16 || !F))) return legs_set_error(ctx, LEGS_ERR_ARG, "NULL argument");
    if (reinterpret_cast<uintptr_t>(probs_f16) & 15)
        return legs_set_error(ctx, LEGS_ERR_ARG, "probs_f16 must be 16-byte aligned");
    LEGS_TRY(use_device(ctx));
    return legs_launch_language_features(ctx, probs_f16, P, N, S, d, out_f16, F, (hipStream_t)stream);
}

int32_t legs_quantize(legs_ctx *ctx, const uint16_t *feat, int64_t K, int32_t d, int32_t d_clip,
                      const float *S, int32_t N, float lambda_dino, float lambda_cos, float lambda_lb,
                      void *workspace, int32_t *index, uint32_t *counts, float *prob_mean, float *losses,
                      float *grad, void *stream)
{
    if (!ctx) return LEGS_ERR_ARG;
    if (K < 1 || K > (1ll << 31) - 256) return legs_set_error(ctx, LEGS_ERR_ARG, "K out of [1, 2^31 - 256]");
    if (N != 32 && N != 64 && N != 128) return legs_set_error(ctx, LEGS_ERR_ARG, "N must be 32, 64 or 128");
    if (d < 128 || d > 8192 || d % 128 || d_clip < 0 || d_clip > d || d_clip % 128)
        return legs_set_error(ctx, LEGS_ERR_ARG, "d and d_clip must be multiples of 128, 0 <= d_clip <= d <= 8192");
    if (!S || !workspace || !counts || !feat || !index)
        return legs_set_error(ctx, LEGS_ERR_ARG, "NULL argument");
    if ((reinterpret_cast<uintptr_t>(feat) | reinterpret_cast<uintptr_t>(S) |
         reinterpret_cast<uintptr_t>(workspace)) & 15)
        return legs_set_error(ctx, LEGS_ERR_ARG, "feat, S and workspace must be 16-byte aligned");
    if (!(lambda_dino >= 0.f) || !(lambda_cos >= 0.f) || !(lambda_lb >= 0.f))
        return legs_set_error(ctx, LEGS_ERR_ARG, "negative or NaN weight");
    LEGS_TRY(use_device(ctx));
    return legs_launch_quantize(ctx, feat, K, d, d_clip, S, N, lambda_dino, lambda_cos, lambda_lb, workspace,
                                index, counts, prob_mean, losses, grad, (hipStream_t)stream);
}

int64_t legs_smooth_param_count(void) { return LEGS_SMOOTH_NPARAMS; }

int32_t legs_smooth_loss_grad(legs_ctx *ctx, const float *mean, const float *channels, int32_t C,
                              int32_t sem_channel, int32_t u_channel, int64_t n, const float *params,
                              float w_s, float lambda_smo, void *workspace, float *grad, float *d_channels,
                              float *loss, void *stream)
{
    if (!ctx) return LEGS_ERR_ARG;
    if (n < 0 || n > (1ll << 31) - 64) return legs_set_error(ctx, LEGS_ERR_ARG, "n out of range");
    if (C < 1 || C > LEGS_MAX_CHANNELS || sem_channel < 0 || sem_channel + LEGS_SMOOTH_OUT > C ||
        u_channel < 0 || u_channel >= C)
        return legs_set_error(ctx, LEGS_ERR_ARG, "channel layout out of range");
    if (!params || !grad || !loss || (n > 0 && (!mean || !channels || !workspace || !d_channels)))
        return legs_set_error(ctx, LEGS_ERR_ARG, "NULL argument");
    if (reinterpret_cast<uintptr_t>(workspace) & 15)
        return legs_set_error(ctx, LEGS_ERR_ARG, "workspace must be 16-byte aligned");
    if (!(w_s >= 0.f) || !(lambda_smo >= 0.f)) return legs_set_error(ctx, LEGS_ERR_ARG, "negative or NaN weight");
    LEGS_TRY(use_device(ctx));
    return legs_launch_smooth(ctx, mean, channels, C, sem_channel, u_channel, n, params, w_s, lambda_smo,
                              workspace, grad, d_channels, loss, (hipStream_t)stream);
}

int32_t legs_semantic_loss_grad_noalloc(legs_ctx *ctx, const float *feat, const float *ru, int64_t P,
                                        int64_t c_stride, int64_t p_stride, const int32_t *labels,
                                        int32_t K, int32_t mlp_flags, const float *params,
                                        float lambda_ce, float lambda_u, float inv_hw, float *grad,
                                        float *d_feat, int64_t d_c_stride, int64_t d_p_stride,
                                        float *d_ru, float *loss, void *stream)
{
    if (!ctx) return LEGS_ERR_ARG;
    if (P > LEGS_NOALLOC_MAX_PIXELS)
        return legs_set_error(ctx, LEGS_ERR_ARG,
                              "P = %lld exceeds LEGS_NOALLOC_MAX_PIXELS (%d); process the view in chunks",
                              (long long)P, LEGS_NOALLOC_MAX_PIXELS);
    float *ws = ctx->device < kScratchDevices ? g_scratch[ctx->device].load() : nullptr;
    if (!ws) return legs_set_error(ctx, LEGS_ERR_HIP, "no scratch address for device %d", ctx->device);
    // Every workspace element the kernels read is written earlier in the same
    // call (forward rows, then the hidden-layer gradients), so the array needs
    // no clearing between calls.
    return legs_semantic_loss_grad(ctx, feat, ru, P, c_stride, p_stride, labels, K, mlp_flags, params,
                                   lambda_ce, lambda_u, inv_hw, ws, grad, d_feat, d_c_stride,
                                   d_p_stride, d_ru, loss, stream);
}

int32_t legs_adam(legs_ctx *ctx, const legs_adam_group *groups, int32_t n_groups, int32_t step,
                  float lr, double beta1, double beta2, float eps, void *stream)
{
    if (!ctx) return LEGS_ERR_ARG;
    if (!groups || n_groups < 1 || n_groups > LEGS_ADAM_MAX_GROUPS)
        return legs_set_error(ctx, LEGS_ERR_ARG, "n_groups out of [1, %d]", LEGS_ADAM_MAX_GROUPS);
    if (step < 1) return legs_set_error(ctx, LEGS_ERR_ARG, "step must be >= 1");
    if (!(beta1 >= 0.0 && beta1 < 1.0) || !(beta2 >= 0.0 && beta2 < 1.0) || !(eps >= 0.f))
        return legs_set_error(ctx, LEGS_ERR_ARG, "bad Adam hyper-parameters");
    for (int k = 0; k < n_groups; ++k) {
        const legs_adam_group &g = groups[k];
        if (g.n < 0 || (g.n > 0 && (!g.param || !g.grad || !g.m || !g.v)))
            return legs_set_error(ctx, LEGS_ERR_ARG, "group %d incomplete", k);
        if (g.clamp_every < 0 || (g.clamp_every > 0 && (g.clamp_offset < 0 || g.clamp_offset >= g.clamp_every)))
            return legs_set_error(ctx, LEGS_ERR_ARG, "group %d bad clamp", k);
    }
    LEGS_TRY(use_device(ctx));
    return legs_launch_adam(ctx, groups, n_groups, step, lr, beta1, beta2, eps, (hipStream_t)stream);
}

int32_t legs_mlp_train_step(legs_ctx *ctx, const float *feat, int64_t B, int64_t c_stride,
                            int64_t p_stride, const int32_t *labels, int32_t K, int32_t mlp_flags,
                            float *params, float *m, float *v, float *grad, int32_t step, float lr,
                            double beta1, double beta2, float eps, void *workspace, float *loss,
                            void *stream)
{
    LEGS_TRY(legs_mlp_grad(ctx, feat, B, c_stride, p_stride, labels, K, mlp_flags, params, workspace,
                           grad, loss, stream));
    legs_adam_group g;
    g.param = params;
    g.grad = grad;
    g.m = m;
    g.v = v;
    g.n = legs_mlp_param_count(K);
    g.clamp_every = 0;
    g.clamp_offset = 0;
    g.clamp_lo = 0.f;
    g.clamp_hi = 0.f;
    return legs_adam(ctx, &g, 1, step, lr, beta1, beta2, eps, stream);
}

int32_t legs_l1_loss_grad(legs_ctx *ctx, const float *out, const float *target,
                          const legs_view *views_dev, int32_t n_views, int64_t total_pixels,
                          int32_t C, int32_t n_fit, float lambda_u, float *d_out, float *loss,
                          void *stream)
{
    if (!ctx) return LEGS_ERR_ARG;
    if (!out || !target || !d_out || !loss) return legs_set_error(ctx, LEGS_ERR_ARG, "NULL argument");
    if (C < 1 || C > LEGS_MAX_CHANNELS || n_fit < 0 || n_fit > C || total_pixels < 0)
        return legs_set_error(ctx, LEGS_ERR_ARG, "bad sizes");
    LEGS_TRY(check_views(ctx, views_dev, n_views));
    LEGS_TRY(use_device(ctx));
    return legs_launch_l1_loss_grad(ctx, out, target, views_dev, n_views, total_pixels, C, n_fit,
                                    lambda_u, d_out, loss, (hipStream_t)stream);
}

int32_t legs_clear(legs_ctx *ctx, void *dev, int64_t bytes, void *stream)
{
    if (!ctx) return LEGS_ERR_ARG;
    if (bytes < 0 || (bytes & 3)) return legs_set_error(ctx, LEGS_ERR_ARG, "bytes must be a non-negative multiple of 4");
    if (bytes > 0 && (!dev || (reinterpret_cast<uintptr_t>(dev) & 3)))
        return legs_set_error(ctx, LEGS_ERR_ARG, "NULL or unaligned buffer");
    LEGS_TRY(use_device(ctx));
    return legs_launch_clear(ctx, dev, bytes / 4, (hipStream_t)stream);
}

} // extern "C"
