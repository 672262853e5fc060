// Front-to-back alpha compositing of every channel (RGB, compact semantic
// feature s_G, uncertainty u) and its backward pass (gfx950).
//
// Sec. 3.1 Eq. 1 defines the rendered image as R(p, Sigma, c, alpha; p_cam);
// Sec. 3.4.1 renders s_G into R_s "with rasterization and alpha blending" and
// Sec. 3.4.2 renders u into R_u the same way, so all C channels are blended
// with one set of weights alpha_k T_k.
//
// Work mapping: one workgroup per screen tile (TILE x TILE pixels, TILE in
// {8, 16, 32}); each wave64 owns an 8 x 8 quadrant, one pixel per lane, so a
// Gaussian whose box misses the quadrant is skipped by the whole wave with a
// scalar test. The tile's depth-ordered list is staged through LDS in batches
// (records first, then channels with consecutive lanes reading consecutive
// channel words), and every lane reads the staged entry with broadcast LDS
// loads. Means are staged relative to the tile origin (rounded once from
// float64), which keeps dx, dy accurate to float32 relative precision
// anywhere on a 4K image.
//
// The backward pass replays each pixel back to front from its final
// transmittance and last-contributor position (no per-sample state is
// stored): the same alpha expression (same instructions, same inputs) decides
// box and skip, T_k = T_{k+1} / (1 - alpha_k), and per-Gaussian sums are
// reduced across the wave before one atomic per value.
#include "legs_internal.h"

namespace {

struct BlendParams {
    const double2 *mean2d;
    const float4 *conic;
    const int4 *box;
    const uint32_t *ids;
    const uint32_t *ranges;
    const legs_view *views;
    int n_views;
    int64_t n;
    int64_t total_tiles;
    const float *ch;
    int C;
    int batch;
    float amax, amin, tmin;
};

// The opacity-weighted Gaussian falloff at offset (dx, dy) from the mean.
// Shared by the forward and backward kernels so both take identical decisions.
__device__ __forceinline__ float falloff_alpha(float dx, float dy, float A, float B, float Cc,
                                               float op, float amax, float &ep, bool &clamped)
{
    float power = -0.5f * (A * dx * dx + Cc * dy * dy) - B * dx * dy;
    power = fminf(power, 0.0f);
    ep = __expf(power);
    const float raw = op * ep;
    clamped = raw > amax;
    return clamped ? amax : raw;
}

__device__ __forceinline__ int sext8(uint32_t v, int sh) { return (int)(int8_t)((v >> sh) & 0xffu); }

// Stage list entries [lo, lo + nb) of a tile into LDS.
template <int TILE, int CP>
__device__ __forceinline__ void stage_batch(const BlendParams &P, int v, int tile_x0, int tile_y0,
                                            uint32_t lo, int nb, float4 *s_g1, float4 *s_g2,
                                            uint32_t *s_id, float *s_ch)
{
    constexpr int NT = TILE * TILE;
    const int tid = threadIdx.x;
    for (int k = tid; k < nb; k += NT) {
        const uint32_t gid = P.ids[lo + k];
        const int64_t gv = (int64_t)v * P.n + gid;
        const double2 m = P.mean2d[gv];
        const float4 cn = P.conic[gv];
        const int4 b = P.box[gv];
        const float mxr = (float)(m.x - ((double)tile_x0 + 0.5));
        const float myr = (float)(m.y - ((double)tile_y0 + 0.5));
        const int x0 = min(max(b.x - tile_x0, -1), TILE), x1 = min(max(b.y - tile_x0, -1), TILE);
        const int y0 = min(max(b.z - tile_y0, -1), TILE), y1 = min(max(b.w - tile_y0, -1), TILE);
        const uint32_t pk = (uint32_t)(x0 & 0xff) | ((uint32_t)(x1 & 0xff) << 8) |
                            ((uint32_t)(y0 & 0xff) << 16) | ((uint32_t)(y1 & 0xff) << 24);
        s_g1[k] = make_float4(mxr, myr, cn.x, cn.y);
        s_g2[k] = make_float4(cn.z, cn.w, __uint_as_float(pk), 0.0f);
        s_id[k] = gid;
    }
    __syncthreads();
    const int C = P.C;
    for (int e = tid; e < nb * CP; e += NT) {
        const int k = e / CP, c = e - k * CP;
        s_ch[e] = c < C ? P.ch[(int64_t)s_id[k] * C + c] : 0.0f;
    }
    __syncthreads();
}

template <int TILE>
__device__ __forceinline__ void lane_pixel(int &lx, int &ly, int &qx0, int &qy0)
{
    const int w = threadIdx.x / LEGS_WAVE, l = threadIdx.x % LEGS_WAVE;
    qx0 = (w % (TILE / 8)) * 8;
    qy0 = (w / (TILE / 8)) * 8;
    lx = qx0 + (l & 7);
    ly = qy0 + (l >> 3);
}

template <int TILE, int CP>
__global__ void __launch_bounds__(TILE *TILE)
k_blend_fwd(BlendParams P, float *__restrict__ out, float *__restrict__ Tf,
            uint32_t *__restrict__ last, uint32_t *__restrict__ tile_counter)
{
    extern __shared__ float4 s_dyn[];
    const int B = P.batch;
    float4 *s_g1 = s_dyn;
    float4 *s_g2 = s_g1 + B;
    uint32_t *s_id = reinterpret_cast<uint32_t *>(s_g2 + B);
    float *s_ch = reinterpret_cast<float *>(s_id + B);
    __shared__ int64_t s_tile;

    int lx, ly, qx0, qy0;
    lane_pixel<TILE>(lx, ly, qx0, qy0);
    const float fx = (float)lx, fy = (float)ly;

    for (int64_t it = blockIdx.x;; it += gridDim.x) {
        int64_t tile = it;
        if (tile_counter) {
            if (threadIdx.x == 0) s_tile = (int64_t)atomicAdd(tile_counter, 1u);
            __syncthreads();
            tile = s_tile;
            __syncthreads();
        }
        if (tile >= P.total_tiles) break;
        const int v = legs_view_of_tile(P.views, P.n_views, tile);
        const legs_view &vw = P.views[v];
        const int W = vw.cam.width, H = vw.cam.height;
        const int64_t lt = tile - vw.tile_offset;
        const int tile_x0 = (int)(lt % vw.tiles_x) * TILE, tile_y0 = (int)(lt / vw.tiles_x) * TILE;
        const int px = tile_x0 + lx, py = tile_y0 + ly;
        const bool inside = px < W && py < H;
        const uint32_t rs = P.ranges[2 * tile], re = P.ranges[2 * tile + 1];

        float acc[CP];
#pragma unroll
        for (int c = 0; c < CP; ++c) acc[c] = 0.0f;
        float T = 1.0f;
        uint32_t lastpos = 0;
        bool done = !inside;

        for (uint32_t lo = rs; lo < re; lo += (uint32_t)B) {
            if (__syncthreads_count(!done) == 0) break;
            const int nb = (int)min((uint32_t)B, re - lo);
            stage_batch<TILE, CP>(P, v, tile_x0, tile_y0, lo, nb, s_g1, s_g2, s_id, s_ch);
            for (int j = 0; j < nb; ++j) {
                if (legs_ballot(!done) == 0) break;
                const float4 g2 = s_g2[j];
                const uint32_t pk = __builtin_amdgcn_readfirstlane(__float_as_uint(g2.z));
                const int x0 = sext8(pk, 0), x1 = sext8(pk, 8), y0 = sext8(pk, 16), y1 = sext8(pk, 24);
                if (x1 < qx0 || x0 > qx0 + 7 || y1 < qy0 || y0 > qy0 + 7) continue;
                if (done || lx < x0 || lx > x1 || ly < y0 || ly > y1) continue;
                const float4 g1 = s_g1[j];
                float ep;
                bool clamped;
                const float alpha = falloff_alpha(g1.x - fx, g1.y - fy, g1.z, g1.w, g2.x, g2.y,
                                                  P.amax, ep, clamped);
                if (alpha < P.amin) continue;
                const float Tn = T * (1.0f - alpha);
                if (Tn < P.tmin) { done = true; continue; }
                const float wgt = alpha * T;
                const float *cj = s_ch + j * CP;
#pragma unroll
                for (int c = 0; c < CP; ++c) acc[c] += wgt * cj[c];
                T = Tn;
                lastpos = (lo - rs) + (uint32_t)j + 1u;
            }
        }
        if (inside) {
            const int64_t pix = vw.pixel_offset + (int64_t)py * W + px;
            const int64_t hw = (int64_t)W * H;
            float *o = out + (int64_t)P.C * vw.pixel_offset + (int64_t)py * W + px;
#pragma unroll
            for (int c = 0; c < CP; ++c)
                if (c < P.C) o[c * hw] = acc[c];
            Tf[pix] = T;
            last[pix] = lastpos;
        }
        if (!tile_counter && it + gridDim.x >= P.total_tiles) break;
    }
}

__device__ __forceinline__ float wave_sum(float x)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, LEGS_WAVE);
    return x;
}

template <int TILE, int CP>
__global__ void __launch_bounds__(TILE *TILE)
k_blend_bwd(BlendParams P, const float *__restrict__ Tf, const uint32_t *__restrict__ last,
            const float *__restrict__ d_out, float *__restrict__ grad2d,
            float *__restrict__ d_ch, uint32_t *__restrict__ tile_counter)
{
    extern __shared__ float4 s_dyn[];
    const int B = P.batch;
    float4 *s_g1 = s_dyn;
    float4 *s_g2 = s_g1 + B;
    uint32_t *s_id = reinterpret_cast<uint32_t *>(s_g2 + B);
    float *s_ch = reinterpret_cast<float *>(s_id + B);
    __shared__ int64_t s_tile;
    __shared__ uint32_t s_maxlast;

    int lx, ly, qx0, qy0;
    lane_pixel<TILE>(lx, ly, qx0, qy0);
    const float fx = (float)lx, fy = (float)ly;
    const int lane = legs_lane();

    for (int64_t it = blockIdx.x;; it += gridDim.x) {
        int64_t tile = it;
        if (tile_counter) {
            if (threadIdx.x == 0) s_tile = (int64_t)atomicAdd(tile_counter, 1u);
            __syncthreads();
            tile = s_tile;
            __syncthreads();
        }
        if (tile >= P.total_tiles) break;
        const int v = legs_view_of_tile(P.views, P.n_views, tile);
        const legs_view &vw = P.views[v];
        const int W = vw.cam.width, H = vw.cam.height;
        const int64_t lt = tile - vw.tile_offset;
        const int tile_x0 = (int)(lt % vw.tiles_x) * TILE, tile_y0 = (int)(lt / vw.tiles_x) * TILE;
        const int px = tile_x0 + lx, py = tile_y0 + ly;
        const bool inside = px < W && py < H;
        const uint32_t rs = P.ranges[2 * tile], re = P.ranges[2 * tile + 1];

        float G[CP], Bs[CP];
        float T = 1.0f;
        uint32_t L = 0;
        const int64_t hw = (int64_t)W * H;
        if (inside) {
            const int64_t pix = vw.pixel_offset + (int64_t)py * W + px;
            const float *g = d_out + (int64_t)P.C * vw.pixel_offset + (int64_t)py * W + px;
#pragma unroll
            for (int c = 0; c < CP; ++c) G[c] = c < P.C ? g[c * hw] : 0.0f;
            T = Tf[pix];
            L = last[pix];
        } else {
#pragma unroll
            for (int c = 0; c < CP; ++c) G[c] = 0.0f;
        }
#pragma unroll
        for (int c = 0; c < CP; ++c) Bs[c] = 0.0f;
        if (threadIdx.x == 0) s_maxlast = 0;
        __syncthreads();
        if (L) atomicMax(&s_maxlast, L);
        __syncthreads();
        const uint32_t maxL = min(s_maxlast, re - rs);

        for (uint32_t hi = maxL; hi > 0;) {
            const uint32_t lo_rel = hi > (uint32_t)B ? hi - (uint32_t)B : 0u;
            const int nb = (int)(hi - lo_rel);
            stage_batch<TILE, CP>(P, v, tile_x0, tile_y0, rs + lo_rel, nb, s_g1, s_g2, s_id, s_ch);
            for (int j = nb - 1; j >= 0; --j) {
                const uint32_t pos = lo_rel + (uint32_t)j;  // 0-based list position
                const float4 g2 = s_g2[j];
                const uint32_t pk = __builtin_amdgcn_readfirstlane(__float_as_uint(g2.z));
                const int x0 = sext8(pk, 0), x1 = sext8(pk, 8), y0 = sext8(pk, 16), y1 = sext8(pk, 24);
                if (x1 < qx0 || x0 > qx0 + 7 || y1 < qy0 || y0 > qy0 + 7) continue;
                bool contrib = pos < L && lx >= x0 && lx <= x1 && ly >= y0 && ly <= y1;
                const float4 g1 = s_g1[j];
                const float dx = g1.x - fx, dy = g1.y - fy;
                float ep = 0.0f, alpha = 0.0f;
                bool clamped = false;
                if (contrib) {
                    alpha = falloff_alpha(dx, dy, g1.z, g1.w, g2.x, g2.y, P.amax, ep, clamped);
                    contrib = alpha >= P.amin;
                }
                if (legs_ballot(contrib) == 0) continue;
                const float *cj = s_ch + j * CP;
                float dmx = 0.f, dmy = 0.f, dA = 0.f, dB = 0.f, dC = 0.f, dop = 0.f;
                float dch[CP];
                if (contrib) {
                    const float Tk = T / (1.0f - alpha);
                    const float wgt = alpha * Tk;
                    float dot = 0.0f;
#pragma unroll
                    for (int c = 0; c < CP; ++c) {
                        dch[c] = wgt * G[c];
                        dot += G[c] * (cj[c] - Bs[c]);
                        Bs[c] = alpha * cj[c] + (1.0f - alpha) * Bs[c];
                    }
                    const float dalpha = Tk * dot;
                    T = Tk;
                    if (!clamped) {
                        dop = dalpha * ep;
                        const float dpow = dalpha * alpha;
                        dA = -0.5f * dpow * dx * dx;
                        dB = -dpow * dx * dy;
                        dC = -0.5f * dpow * dy * dy;
                        dmx = -dpow * (g1.z * dx + g1.w * dy);
                        dmy = -dpow * (g1.w * dx + g2.x * dy);
                    }
                } else {
#pragma unroll
                    for (int c = 0; c < CP; ++c) dch[c] = 0.0f;
                }
                dmx = wave_sum(dmx); dmy = wave_sum(dmy); dA = wave_sum(dA);
                dB = wave_sum(dB); dC = wave_sum(dC); dop = wave_sum(dop);
#pragma unroll
                for (int c = 0; c < CP; ++c) dch[c] = wave_sum(dch[c]);
                if (lane == 0) {
                    const uint32_t gid = s_id[j];
                    float *g2d = grad2d + 8 * ((int64_t)v * P.n + gid);
                    atomicAdd(g2d + 0, dmx);
                    atomicAdd(g2d + 1, dmy);
                    atomicAdd(g2d + 2, dA);
                    atomicAdd(g2d + 3, dB);
                    atomicAdd(g2d + 4, dC);
                    atomicAdd(g2d + 5, dop);
                    float *dc = d_ch + (int64_t)gid * P.C;
#pragma unroll
                    for (int c = 0; c < CP; ++c)
                        if (c < P.C) atomicAdd(dc + c, dch[c]);
                }
            }
            hi = lo_rel;
            __syncthreads();
        }
        if (!tile_counter && it + gridDim.x >= P.total_tiles) break;
    }
}

template <int TILE, int CP>
size_t lds_bytes(int batch) { return (size_t)batch * (16 + 16 + 4 + 4 * CP); }

template <int TILE, int CP>
int32_t launch_tile_cp(legs_ctx *ctx, bool fwd, const BlendParams &P, float *out, float *Tf,
                       uint32_t *last, const float *cTf, const uint32_t *clast, const float *d_out,
                       float *grad2d, float *d_ch, hipStream_t s)
{
    const size_t lds = lds_bytes<TILE, CP>(P.batch);
    if (lds > 65536) return legs_set_error(ctx, LEGS_ERR_UNSUPPORTED, "LDS batch too large for C");
    const int64_t grid = P.total_tiles;
    if (grid <= 0) return LEGS_OK;
    if (fwd) {
        hipLaunchKernelGGL((k_blend_fwd<TILE, CP>), dim3((unsigned)grid), dim3(TILE * TILE), lds, s,
                           P, out, Tf, last, (uint32_t *)nullptr);
    } else {
        hipLaunchKernelGGL((k_blend_bwd<TILE, CP>), dim3((unsigned)grid), dim3(TILE * TILE), lds, s,
                           P, cTf, clast, d_out, grad2d, d_ch, (uint32_t *)nullptr);
    }
    LEGS_CHECK_LAUNCH(ctx);
    return LEGS_OK;
}

template <int TILE>
int32_t launch_tile(legs_ctx *ctx, bool fwd, const BlendParams &P, float *out, float *Tf,
                    uint32_t *last, const float *cTf, const uint32_t *clast, const float *d_out,
                    float *grad2d, float *d_ch, hipStream_t s)
{
#define LEGS_CP_CASE(cp)                                                                      \
    if (P.C <= cp)                                                                            \
        return launch_tile_cp<TILE, cp>(ctx, fwd, P, out, Tf, last, cTf, clast, d_out, grad2d, \
                                        d_ch, s);
    LEGS_CP_CASE(4)
    LEGS_CP_CASE(8)
    LEGS_CP_CASE(12)
    LEGS_CP_CASE(16)
    LEGS_CP_CASE(20)
    LEGS_CP_CASE(24)
    LEGS_CP_CASE(32)
    LEGS_CP_CASE(64)
#undef LEGS_CP_CASE
    return legs_set_error(ctx, LEGS_ERR_ARG, "C=%d exceeds %d", P.C, LEGS_MAX_CHANNELS);
}

int32_t launch(legs_ctx *ctx, bool fwd, const BlendParams &P, float *out, float *Tf,
               uint32_t *last, const float *cTf, const uint32_t *clast, const float *d_out,
               float *grad2d, float *d_ch, int tile, hipStream_t s)
{
    switch (tile) {
    case 8: return launch_tile<8>(ctx, fwd, P, out, Tf, last, cTf, clast, d_out, grad2d, d_ch, s);
    case 16: return launch_tile<16>(ctx, fwd, P, out, Tf, last, cTf, clast, d_out, grad2d, d_ch, s);
    case 32: return launch_tile<32>(ctx, fwd, P, out, Tf, last, cTf, clast, d_out, grad2d, d_ch, s);
    default: return legs_set_error(ctx, LEGS_ERR_ARG, "tile must be 8, 16 or 32");
    }
}

BlendParams make_params(const legs_projected *proj, int64_t n, const legs_bins *bins,
                        const legs_view *views, int32_t n_views, int64_t total_tiles,
                        const float *channels, int32_t C, const legs_opts *o)
{
    BlendParams P;
    P.mean2d = reinterpret_cast<const double2 *>(proj->mean2d);
    P.conic = reinterpret_cast<const float4 *>(proj->conic);
    P.box = reinterpret_cast<const int4 *>(proj->box);
    P.ids = bins->ids;
    P.ranges = bins->ranges;
    P.views = views;
    P.n_views = n_views;
    P.n = n;
    P.total_tiles = total_tiles;
    P.ch = channels;
    P.C = C;
    P.batch = o->lds_batch;
    P.amax = o->alpha_max;
    P.amin = o->alpha_min;
    P.tmin = o->t_min;
    return P;
}

} // namespace

int32_t legs_launch_blend_forward(legs_ctx *ctx, const legs_projected *proj, int64_t n,
                                  const legs_bins *bins, const legs_view *views, int32_t n_views,
                                  int64_t total_tiles, const float *channels, int32_t C,
                                  const legs_opts *o, float *out, float *T_final, uint32_t *last,
                                  hipStream_t s)
{
    const BlendParams P = make_params(proj, n, bins, views, n_views, total_tiles, channels, C, o);
    return launch(ctx, true, P, out, T_final, last, nullptr, nullptr, nullptr, nullptr, nullptr,
                  o->tile, s);
}

int32_t legs_launch_blend_backward(legs_ctx *ctx, const legs_projected *proj, int64_t n,
                                   const legs_bins *bins, const legs_view *views, int32_t n_views,
                                   int64_t total_tiles, const float *channels, int32_t C,
                                   const legs_opts *o, const float *T_final, const uint32_t *last,
                                   const float *d_out, float *grad2d, float *d_channels,
                                   hipStream_t s)
{
    const BlendParams P = make_params(proj, n, bins, views, n_views, total_tiles, channels, C, o);
    return launch(ctx, false, P, nullptr, nullptr, nullptr, T_final, last, d_out, grad2d,
                  d_channels, o->tile, s);
}
