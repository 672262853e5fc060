// Front-to-back alpha compositing of every channel (RGB, compact semantic
// feature s_G, uncertainty u) and its backward pass (gfx950).
//
// Sec. 3.1 Eq. 1 defines the rendered image as R(p, Sigma, c, alpha; p_cam);
// Sec. 3.4.1 renders s_G into R_s "with rasterization and alpha blending" and
// Sec. 3.4.2 renders u into R_u the same way, so all C channels are blended
// with one set of weights alpha_k T_k.
//
// One workgroup per screen tile (TILE x TILE pixels, TILE in {8, 16, 32}), or
// a persistent grid taking tiles from an atomic counter. The tile's
// depth-ordered list is staged through LDS in batches (records first, then
// channels with consecutive lanes reading consecutive words); every lane then
// reads the staged entry with broadcast LDS loads.
//
// Means are staged relative to the centre of the first pixel of each 8-pixel
// block column / row (rounded once from float64). Those block origins do not
// depend on the tile size, so every pixel computes the same float32 offset
// (dx, dy) for every tile size and LDS batch size, forward and backward alike:
// images are bit-identical across launch settings and the backward replays the
// forward's decisions exactly. The offsets are also accurate to float32
// relative precision anywhere on a 4K image.
//
// Forward: each wave64 owns an 8 x 8 quadrant, one pixel per lane; a Gaussian
// whose box misses the quadrant is skipped by a scalar test; early exit per
// wave (ballot) and per workgroup (__syncthreads_count).
// Backward: each wave owns a 16 x 16 block with 4 pixels per lane (16 x 8 with
// 2 for 17-32 channels, 8 x 8 with 1 for wider sets or 8-pixel tiles), and
// replays them back to front from (T_final, last): T_k = T_{k+1} / (1 - alpha_k).
// Per Gaussian, a lane first sums its own pixels in registers, then the wave
// sums the 6 + C values with a transpose reduction (lane swaps and DPP moves
// that leave each total in one lane), and one atomic instruction adds all of
// them, one lane per value.
#include "legs_internal.h"
#include "wave_reduce.h"

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
    bool reach;         // skip the pixels outside the reach of alpha_min (reach_box)
    uint32_t *counter;  // non-NULL: persistent launch, tiles taken from this counter
    const uint32_t *order;  // persistent launch: the tiles in decreasing order of list length
    float4 *zero4;      // forward: zero_n4 float4 and then zero_tail floats to set to 0 (NULL: none)
    int64_t zero_n4;
    int zero_tail;
};

// The conic (A, B, C) is staged scaled by (-log2(e)/2, -log2(e), -log2(e)/2),
// so that the falloff exponent in base 2 is
//   power * log2(e) = A' dx^2 + B' dx dy + C' dy^2 = a + dy (b + C' dy),
// with a = A' dx dx and b = B' dx depending on dx only (the backward computes
// them once per Gaussian and pixel column). ep = exp(power).
constexpr float CONIC_SCALE_AC = -0.72134752044448170f;   // -log2(e) / 2
constexpr float CONIC_SCALE_B = -1.44269504088896340f;    // -log2(e)

__device__ __forceinline__ float4 scale_conic(float4 cn)
{
    return make_float4(cn.x * CONIC_SCALE_AC, cn.y * CONIC_SCALE_B, cn.z * CONIC_SCALE_AC, cn.w);
}

// The dx terms of the exponent for a scaled conic.
__device__ __forceinline__ void falloff_dx(float dx, float As, float Bs, float &a, float &b)
{
    a = (As * dx) * dx;
    b = Bs * dx;
}

// The opacity-weighted Gaussian falloff at row offset dy. Shared by the
// forward and backward kernels so both take identical decisions.
__device__ __forceinline__ float falloff_alpha(float a, float b, float dy, float Cs, float op, float amax,
                                               float &ep, bool &clamped)
{
    const float p = fminf(fmaf(dy, fmaf(Cs, dy, b), a), 0.0f);
    ep = __builtin_amdgcn_exp2f(p);
    const float raw = op * ep;   // >= 0: the clamp to [0, amax] is min(raw, amax)
    clamped = raw > amax;
    return __builtin_amdgcn_fmed3f(raw, 0.0f, amax);
}

__device__ __forceinline__ float opaque_zero()
{
    float z;
    asm volatile("v_mov_b32 %0, 0" : "=v"(z));
    return z;
}

// Two opaque zeros from one 64-bit move.
__device__ __forceinline__ void opaque_zero2(float &a, float &b)
{
    double z;
    asm volatile("v_mov_b64 %0, 0" : "=v"(z));
    const uint64_t u = __builtin_bit_cast(uint64_t, z);
    a = __builtin_bit_cast(float, (uint32_t)u);
    b = __builtin_bit_cast(float, (uint32_t)(u >> 32));
}

__device__ __forceinline__ int sext8(uint32_t v, int sh) { return (int)(int8_t)((v >> sh) & 0xffu); }

// The pixels of a Gaussian's 3-sigma box where alpha can reach alpha_min,
// from the staged values the blend kernels compute with: the scaled conic cs
// (exponent in base 2: As dx^2 + Bs dx dy + Cs dy^2, opacity in w) and the
// float32 offset (mx, my) of the mean from the centre of the tile's first
// pixel. The box is cut to the bounding box of the ellipse where the exponent
// is at least log2(alpha_min / opacity); every pixel outside it computes alpha
// < alpha_min, so it neither blends nor stops there and the kernels skip it.
// The ellipse is widened (the bound K by a relative 1e-3, by 1e-3 and by 1e-4
// times kap = (1 + |rho|) / (1 - |rho|), rho the correlation of the form, a
// bound on the sum of the exponent's absolute terms over its value; the half
// widths by 0.5 % and by 0.01 pixel plus 1e-6 of the offset) so that neither
// the few-ulp rounding of the kernels' exponent and exp2 nor the float32
// arithmetic here (within 1e-3 relative while kap <= 1e4) can exclude a pixel
// that reaches alpha_min. Very elongated ellipses (kap > 1e4) keep the whole
// box. (x0, x1, y0, y1): the tile-relative inclusive box, tightened in place;
// an empty result is (TILE, -1, TILE, -1).
template <int TILE>
__device__ __forceinline__ void reach_box(float4 cs, float mx, float my, float amin, int &x0, int &x1,
                                          int &y0, int &y1)
{
    // the form a dx^2 + 2 h dx dy + c dy^2 <= K of the pixels that reach alpha_min
    const float a = -cs.x, h = -0.5f * cs.y, c = -cs.z, op = cs.w;
    if (amin > 0.0f && a > 0.0f && c > 0.0f) {
        if (!(op >= amin)) {   // alpha <= opacity < alpha_min everywhere
            x1 = x0 - 1;
        } else {
            const float r2 = (h * h) / (a * c);
            const float rho = __builtin_sqrtf(r2);
            if (rho < 0.9998f) {   // kap <= 1e4
                const float kap = (1.0f + rho) / (1.0f - rho);
                const float K = (__builtin_amdgcn_logf(op) - __builtin_amdgcn_logf(amin)) * 1.001f + 1e-3f +
                                1e-4f * kap;
                const float u = K / (1.0f - r2);
                const float hw = __builtin_sqrtf(u / a) * 1.005f + 0.01f + 1e-6f * fabsf(mx);
                const float hh = __builtin_sqrtf(u / c) * 1.005f + 0.01f + 1e-6f * fabsf(my);
                // tile-relative pixel x has its centre mx - x from the mean
                const float fx0 = ceilf(mx - hw), fx1 = floorf(mx + hw);
                const float fy0 = ceilf(my - hh), fy1 = floorf(my + hh);
                if (fx0 > (float)x0) x0 = fx0 > (float)x1 ? x1 + 1 : (int)fx0;
                if (fx1 < (float)x1) x1 = fx1 < (float)x0 ? x0 - 1 : (int)fx1;
                if (fy0 > (float)y0) y0 = fy0 > (float)y1 ? y1 + 1 : (int)fy0;
                if (fy1 < (float)y1) y1 = fy1 < (float)y0 ? y0 - 1 : (int)fy1;
            }
        }
    }
    if (x0 > x1 || y0 > y1) {
        x0 = y0 = TILE;
        x1 = y1 = -1;
    }
}

// LDS layout of one staged batch of B entries.
template <int TILE, int CP>
struct Stage {
    static constexpr int NQ = TILE / 8;  // 8-pixel block columns (rows) per tile
    float4 *c;       // [B] (A, B, C, opacity)
    float *ch;       // [B][CP]
    float *qx, *qy;  // [B][NQ] mean minus the centre of the block's first pixel
    uint32_t *box;   // [B] tile-relative box, 4 x int8
    uint32_t *id;    // [B]
    __device__ Stage(void *base, int B)
    {
        c = static_cast<float4 *>(base);
        ch = reinterpret_cast<float *>(c + B);
        qx = ch + (size_t)B * CP;
        qy = qx + (size_t)B * NQ;
        box = reinterpret_cast<uint32_t *>(qy + (size_t)B * NQ);
        id = box + B;
    }
    static size_t bytes(int B) { return (size_t)B * (16 + 4 * CP + 8 * NQ + 4 + 4); }
};

// Stages nb list entries starting at list position lo: each thread takes
// entries tid, tid + NT, ...; their ids are loaded first, then every gather of
// up to two entries is issued before any is stored, so a batch costs two
// dependent memory latencies. Channel sets of up to 16 values travel the same
// way; wider ones are read by consecutive threads after the records.
template <int TILE, int CP, int NT>
__device__ __forceinline__ void stage_batch(const BlendParams &P, int v, int tile_x0, int tile_y0,
                                            uint32_t lo, int nb, Stage<TILE, CP> &S)
{
    constexpr int NQ = TILE / 8;
    constexpr int R = (256 + NT - 1) / NT;       // entries per thread at the largest batch
    constexpr int RC = R > 2 ? 2 : R;            // entries with loads in flight together
    constexpr bool DIRECT = CP <= 16;
    const int tid = threadIdx.x;
    const int C = P.C;
    for (int r0 = 0; r0 < R; r0 += RC) {
        uint32_t gid[RC];
        bool ok[RC];
#pragma unroll
        for (int r = 0; r < RC; ++r) {
            const int k = tid + (r0 + r) * NT;
            ok[r] = k < nb;
            gid[r] = ok[r] ? P.ids[lo + k] : 0u;
        }
        double2 m[RC];
        int4 b[RC];
        float4 cn[RC];
        float ch[RC][DIRECT ? CP : 1];
#pragma unroll
        for (int r = 0; r < RC; ++r) {
            if (!ok[r]) continue;
            const int64_t gv = (int64_t)v * P.n + gid[r];
            m[r] = P.mean2d[gv];
            b[r] = P.box[gv];
            cn[r] = P.conic[gv];
            if constexpr (DIRECT) {
                const float *src = P.ch + (int64_t)gid[r] * C;
#pragma unroll
                for (int c = 0; c < CP; ++c) ch[r][c] = c < C ? src[c] : 0.0f;
            }
        }
#pragma unroll
        for (int r = 0; r < RC; ++r) {
            if (!ok[r]) continue;
            const int k = tid + (r0 + r) * NT;
#pragma unroll
            for (int q = 0; q < NQ; ++q) {
                S.qx[k * NQ + q] = (float)(m[r].x - ((double)(tile_x0 + 8 * q) + 0.5));
                S.qy[k * NQ + q] = (float)(m[r].y - ((double)(tile_y0 + 8 * q) + 0.5));
            }
            const int x0 = min(max(b[r].x - tile_x0, -1), TILE), x1 = min(max(b[r].y - tile_x0, -1), TILE);
            const int y0 = min(max(b[r].z - tile_y0, -1), TILE), y1 = min(max(b[r].w - tile_y0, -1), TILE);
            S.box[k] = (uint32_t)(x0 & 0xff) | ((uint32_t)(x1 & 0xff) << 8) |
                       ((uint32_t)(y0 & 0xff) << 16) | ((uint32_t)(y1 & 0xff) << 24);
            S.c[k] = scale_conic(cn[r]);
            S.id[k] = gid[r];
            if constexpr (DIRECT) {
#pragma unroll
                for (int c = 0; c < CP; ++c) S.ch[k * CP + c] = ch[r][c];
            }
        }
    }
    __syncthreads();
    if (P.reach) {
        // the boxes cut to the reach of alpha_min, from the staged values
        for (int k = tid; k < nb; k += NT) {
            const uint32_t pk = S.box[k];
            int x0 = sext8(pk, 0), x1 = sext8(pk, 8), y0 = sext8(pk, 16), y1 = sext8(pk, 24);
            reach_box<TILE>(S.c[k], S.qx[k * NQ], S.qy[k * NQ], P.amin, x0, x1, y0, y1);
            S.box[k] = (uint32_t)(x0 & 0xff) | ((uint32_t)(x1 & 0xff) << 8) | ((uint32_t)(y0 & 0xff) << 16) |
                       ((uint32_t)(y1 & 0xff) << 24);
        }
        __syncthreads();
    }
    if constexpr (!DIRECT) {
        for (int e = tid; e < nb * CP; e += NT) {
            const int k = e / CP, c = e - k * CP;
            S.ch[e] = c < C ? P.ch[(int64_t)S.id[k] * C + c] : 0.0f;
        }
        __syncthreads();
    }
}

struct TileInfo {
    int v, W, H, tile_x0, tile_y0;
    int64_t pixel_offset;
    uint32_t rs, re;
};

template <int TILE>
__device__ __forceinline__ TileInfo tile_info(const BlendParams &P, int64_t tile)
{
    TileInfo t;
    t.v = legs_view_of_tile(P.views, P.n_views, tile);
    const legs_view &vw = P.views[t.v];
    t.W = vw.cam.width;
    t.H = vw.cam.height;
    const int64_t lt = tile - vw.tile_offset;
    t.tile_x0 = (int)(lt % vw.tiles_x) * TILE;
    t.tile_y0 = (int)(lt / vw.tiles_x) * TILE;
    t.pixel_offset = vw.pixel_offset;
    t.rs = P.ranges[2 * tile];
    t.re = P.ranges[2 * tile + 1];
    return t;
}

// Next tile of this workgroup: one tile per workgroup, or the next entry of
// the heaviest-first tile order from the persistent counter.
__device__ __forceinline__ int64_t next_tile(const BlendParams &P, int64_t prev, int64_t *s_tile)
{
    if (P.counter) {
        if (threadIdx.x == 0) {
            const uint32_t i = atomicAdd(P.counter, 1u);
            *s_tile = (int64_t)i < P.total_tiles ? (int64_t)P.order[i] : P.total_tiles;
        }
        __syncthreads();
        const int64_t t = *s_tile;
        __syncthreads();
        return t;
    }
    return prev < 0 ? (int64_t)blockIdx.x : P.total_tiles;
}

// Next forward work item: one per workgroup, or the next queue position from
// the persistent counter (items / parts of one tile = one queue entry).
__device__ __forceinline__ int64_t next_item(const BlendParams &P, int64_t prev, int64_t items, int64_t *s_item)
{
    if (P.counter) {
        if (threadIdx.x == 0) {
            const uint32_t i = atomicAdd(P.counter, 1u);
            *s_item = (int64_t)i < items ? (int64_t)i : items;
        }
        __syncthreads();
        const int64_t t = *s_item;
        __syncthreads();
        return t;
    }
    return prev < 0 ? (int64_t)blockIdx.x : items;
}

// ---- forward ---------------------------------------------------------------------

// Waves per SIMD the forward asks the register allocator for, with up to 12
// channels and 256-thread workgroups: the LDS limit of a 256-entry batch (7 at
// 16 x 16 tiles, 6 for the 16 x 16 parts of 32 x 32 tiles), which costs at
// most a few spills of loop invariants outside the visit loop; none elsewhere.
template <int TILE, int CP, int SUB>
constexpr int fwd_waves() { return SUB != 16 || CP > 12 ? 1 : (TILE == 16 ? 7 : 6); }

// SUB < TILE: each workgroup composites one SUB x SUB part of a tile over the
// whole tile's list (one workgroup per part, one-per-tile launches only), so
// a part stops as soon as its own pixels are done.
template <int TILE, int CP, int SUB>
__global__ void __launch_bounds__(SUB *SUB) __attribute__((amdgpu_waves_per_eu(fwd_waves<TILE, CP, SUB>())))
k_blend_fwd(BlendParams P, float *__restrict__ out, float *__restrict__ Tf,
            uint32_t *__restrict__ last)
{
    constexpr int NT = SUB * SUB, NQ = TILE / 8, NS = TILE / SUB, QS = SUB / 8;
    static_assert(NS * SUB == TILE, "parts tile the tile");
    extern __shared__ float4 s_dyn[];
    Stage<TILE, CP> S(s_dyn, P.batch);
    __shared__ int64_t s_tile;
    const int B = P.batch;
    const float amax = P.amax;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x / LEGS_WAVE), l = threadIdx.x % LEGS_WAVE;
    if (P.zero4) {
        // the zeroing asked for with the compositing: each workgroup stores its
        // grid-stride share before its first item (the stores drain while the
        // ALU-bound compositing runs)
        for (int64_t i = (int64_t)blockIdx.x * NT + threadIdx.x; i < P.zero_n4; i += (int64_t)gridDim.x * NT)
            P.zero4[i] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
        if (blockIdx.x == 0 && (int)threadIdx.x < P.zero_tail)
            reinterpret_cast<float *>(P.zero4 + P.zero_n4)[threadIdx.x] = 0.0f;
    }
    const float fx = (float)(l & 7), fy = (float)(l >> 3);
    // work items: (tile, part) pairs, the parts of a tile consecutive; one
    // item per workgroup, or the persistent queue (heaviest tiles first)
    constexpr int NP = NS * NS;
    const int64_t items = P.total_tiles * NP;
    for (int64_t item = next_item(P, -1, items, &s_tile); item < items; item = next_item(P, item, items, &s_tile)) {
        const int64_t q = item / NP;
        const int part = (int)(item - q * NP);
        const int64_t tile = P.counter ? (int64_t)P.order[q] : q;
        const int qxi = (part % NS) * QS + w % QS, qyi = (part / NS) * QS + w / QS;   // this wave's 8 x 8 quadrant
        const int qx0 = 8 * qxi, qy0 = 8 * qyi;
        const int lx = qx0 + (l & 7), ly = qy0 + (l >> 3);
        const TileInfo ti = tile_info<TILE>(P, tile);
        const int px = ti.tile_x0 + lx, py = ti.tile_y0 + ly;
        const bool inside = px < ti.W && py < ti.H;
        float acc[CP];
#pragma unroll
        for (int c = 0; c < CP; ++c) acc[c] = 0.0f;
        float T = 1.0f;
        uint32_t lastpos = 0;
        uint64_t donemask = legs_ballot(!inside);   // pixels that stopped (or lie off the image)
        for (uint32_t lo = ti.rs; lo < ti.re; lo += (uint32_t)B) {
            if (__syncthreads_count(l == 0 && ~donemask != 0) == 0) break;
            const int nb = (int)min((uint32_t)B, ti.re - lo);
            stage_batch<TILE, CP, NT>(P, ti.v, ti.tile_x0, ti.tile_y0, lo, nb, S);
            // 64 entries at a time: lane l computes the mask of this wave's 8 x 8
            // block pixels inside entry c0 + l's box; an entry is visited only
            // while it covers a pixel that is not done, and only those lanes work
            for (int c0 = 0; c0 < nb && ~donemask; c0 += LEGS_WAVE) {
                uint32_t mlo = 0, mhi = 0;
                if (c0 + l < nb) {
                    const uint32_t pk = S.box[c0 + l];
                    const int cx0 = max(sext8(pk, 0) - qx0, 0), cx1 = min(sext8(pk, 8) - qx0, 7);
                    const int ry0 = max(sext8(pk, 16) - qy0, 0), ry1 = min(sext8(pk, 24) - qy0, 7);
                    if (cx0 <= cx1 && ry0 <= ry1) {
                        const uint32_t xm = (0xffu << cx0) & (0xffu >> (7 - cx1));
                        const uint32_t xr = xm * 0x01010101u;
                        const uint64_t rows = (~0ull << (8 * ry0)) & (~0ull >> (8 * (7 - ry1)));
                        mlo = (uint32_t)rows & xr;
                        mhi = (uint32_t)(rows >> 32) & xr;
                    }
                }
                uint64_t rel = legs_ballot(((((uint64_t)mhi << 32) | mlo) & ~donemask) != 0);
                while (rel) {
                    const int jl = (int)__builtin_ctzll(rel);
                    rel &= rel - 1;
                    const uint64_t act = (((uint64_t)(uint32_t)__builtin_amdgcn_readlane((int)mhi, jl) << 32) |
                                          (uint32_t)__builtin_amdgcn_readlane((int)mlo, jl)) & ~donemask;
                    if (act == 0) continue;
                    // every lane evaluates (masked lanes would cost the same); only
                    // the pixels of act may blend or stop
                    const int j = c0 + jl;
                    const float4 cn = S.c[j];
                    const float dx = S.qx[j * NQ + qxi] - fx, dy = S.qy[j * NQ + qyi] - fy;
                    float a, b, ep;
                    bool clamped;
                    falloff_dx(dx, cn.x, cn.y, a, b);
                    const float alpha = falloff_alpha(a, b, dy, cn.z, cn.w, amax, ep, clamped);
                    const float Tn = T * (1.0f - alpha);
                    // lane masks straight from the compares (predicates 11 = unordered
                    // or >=, i.e. !(alpha < amin); 4 = ordered <): the pixels of act
                    // that reach alpha_min stop if Tn < t_min and blend otherwise
                    const uint64_t reach = act & __builtin_amdgcn_fcmpf(alpha, P.amin, 11);
                    const uint64_t stop = __builtin_amdgcn_fcmpf(Tn, P.tmin, 4);
                    donemask |= reach & stop;
                    if (__builtin_amdgcn_inverse_ballot_w64(reach & ~stop)) {
                        const float wgt = alpha * T;
                        const float *cj = S.ch + j * CP;
#pragma unroll
                        for (int c = 0; c < CP; ++c) acc[c] = fmaf(wgt, cj[c], acc[c]);
                        T = Tn;
                        lastpos = (lo - ti.rs) + (uint32_t)j + 1u;
                    }
                    if (!~donemask) break;
                }
            }
        }
        if (inside) {
            const int64_t pix = ti.pixel_offset + (int64_t)py * ti.W + px;
            const int64_t hw = (int64_t)ti.W * ti.H;
            float *o = out + (int64_t)P.C * ti.pixel_offset + (int64_t)py * ti.W + px;
#pragma unroll
            for (int c = 0; c < CP; ++c)
                if (c < P.C) o[c * hw] = acc[c];
            Tf[pix] = T;
            last[pix] = lastpos;
        }
    }
}

// ---- backward ----------------------------------------------------------------------

// Per-wave block of the backward: SW x SH pixels, PPL = SW * SH / 64 per lane.
template <int TILE, int CP> struct BwdShape {
    static constexpr int SW = (TILE == 8 || CP > 32) ? 8 : 16;
    static constexpr int SH = (TILE == 8 || CP > 32) ? 8 : (CP <= 16 ? 16 : 8);
    static constexpr int PPL = SW * SH / LEGS_WAVE;
    static constexpr int NT = TILE * TILE / PPL;
    static constexpr int ROWSTEP = LEGS_WAVE / SW;
};

// Backward of Eq. 1 per pixel, back to front from (T_final, last). With
// w_k = alpha_k T_k and g_k = sum_c G_c c_{k,c} (G = dL/dR at the pixel),
//   dL/dc_{k,c}  += w_k G_c
//   dL/dalpha_k  += T_k (g_k - s_k),   s_{k-1} = alpha_k g_k + (1 - alpha_k) s_k,
// where s_k = sum_c G_c (colour composited behind k, renormalised), so the
// recurrence carries one scalar per pixel instead of one per channel; and
// alpha_k = min(alpha_max, o_k exp(power)) gives dL/dpower = alpha dL/dalpha
// and dL/do = exp(power) dL/dalpha when not clamped. The power's derivatives
// (mean offset and conic) are summed per lane as moments of (dx, dy) and
// turned into gradients once per Gaussian (the map is linear).
template <int TILE, int CP>
__global__ void __launch_bounds__((BwdShape<TILE, CP>::NT), 4)
k_blend_bwd(BlendParams P, const float *__restrict__ Tf, const uint32_t *__restrict__ last,
            const float *__restrict__ d_out, float *__restrict__ grad2d, float *__restrict__ d_ch)
{
    using Shp = BwdShape<TILE, CP>;
    constexpr int NT = Shp::NT, PPL = Shp::PPL, NQ = TILE / 8;
    constexpr int NV = 6 + CP;                          // values summed per Gaussian
    constexpr int KF = legs_tr::final_k(NV);
    extern __shared__ float4 s_dyn[];
    Stage<TILE, CP> S(s_dyn, P.batch);
    __shared__ int64_t s_tile;
    __shared__ uint32_t s_maxlast;
    const int B = P.batch;
    const float amax = P.amax;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x / LEGS_WAVE), l = threadIdx.x % LEGS_WAVE;
    constexpr int BX = TILE / Shp::SW;                 // wave blocks per tile row
    const int bx0 = (w % BX) * Shp::SW, by0 = (w / BX) * Shp::SH;
    const int lx = bx0 + (l % Shp::SW);
    const int ly0 = by0 + (l / Shp::SW);               // pixel p of this lane: row ly0 + ROWSTEP p
    const float fx = (float)(lx & 7);
    const int qxi = lx >> 3;
    // which summed value this lane adds to memory after the wave reduction
    int vidx[NV];
    legs_tr::index<NV>(vidx, l);
    bool vgeo[KF], vok[KF];
    int voff[KF];
#pragma unroll
    for (int r = 0; r < KF; ++r) {
        vgeo[r] = vidx[r] >= 0 && vidx[r] < 6;
        voff[r] = vgeo[r] ? vidx[r] : vidx[r] - 6;
        vok[r] = vidx[r] >= 0 && (vgeo[r] || voff[r] < P.C);
    }

    for (int64_t tile = next_tile(P, -1, &s_tile); tile < P.total_tiles; tile = next_tile(P, tile, &s_tile)) {
        const TileInfo ti = tile_info<TILE>(P, tile);
        const int64_t hw = (int64_t)ti.W * ti.H;
        float G[PPL][CP], T[PPL], gs[PPL];
        uint32_t L[PPL];
        uint32_t myL = 0;
#pragma unroll
        for (int p = 0; p < PPL; ++p) {
            const int px = ti.tile_x0 + lx, py = ti.tile_y0 + ly0 + Shp::ROWSTEP * p;
            T[p] = 1.0f;
            L[p] = 0;
            gs[p] = 0.0f;
            if (px < ti.W && py < ti.H) {
                const int64_t pix = ti.pixel_offset + (int64_t)py * ti.W + px;
                const float *g = d_out + (int64_t)P.C * ti.pixel_offset + (int64_t)py * ti.W + px;
#pragma unroll
                for (int c = 0; c < CP; ++c) G[p][c] = c < P.C ? g[c * hw] : 0.0f;
                T[p] = Tf[pix];
                L[p] = last[pix];
            } else {
#pragma unroll
                for (int c = 0; c < CP; ++c) G[p][c] = 0.0f;
            }
            myL = max(myL, L[p]);
        }
        if (threadIdx.x == 0) s_maxlast = 0;
        __syncthreads();
        if (myL) atomicMax(&s_maxlast, myL);
        __syncthreads();
        const uint32_t maxL = min(s_maxlast, ti.re - ti.rs);

        for (uint32_t hi = maxL; hi > 0;) {
            const uint32_t lo_rel = hi > (uint32_t)B ? hi - (uint32_t)B : 0u;
            const int nb = (int)(hi - lo_rel);
            stage_batch<TILE, CP, NT>(P, ti.v, ti.tile_x0, ti.tile_y0, ti.rs + lo_rel, nb, S);
            // 64 entries at a time, back to front: lane l tests entry c1 - 1 - l's
            // box against this wave's block, and only the hits are visited
            for (int c1 = nb; c1 > 0; c1 -= LEGS_WAVE) {
              const int jl = c1 - 1 - l;
              uint32_t pkl = 0;
              bool hit = false;
              if (jl >= 0) {
                  pkl = S.box[jl];
                  const int x0 = sext8(pkl, 0), x1 = sext8(pkl, 8), y0 = sext8(pkl, 16), y1 = sext8(pkl, 24);
                  hit = !(x1 < bx0 || x0 > bx0 + Shp::SW - 1 || y1 < by0 || y0 > by0 + Shp::SH - 1);
              }
              for (uint64_t rel = legs_ballot(hit); rel; rel &= rel - 1) {
                const int hl = (int)__builtin_ctzll(rel);           // the lowest lane: the last entry first
                const int j = c1 - 1 - hl;
                const uint32_t pos = lo_rel + (uint32_t)j;   // 0-based list position
                const uint32_t pk = (uint32_t)__builtin_amdgcn_readlane((int)pkl, hl);
                const int x0 = sext8(pk, 0), x1 = sext8(pk, 8), y0 = sext8(pk, 16), y1 = sext8(pk, 24);
                const float4 cn = S.c[j];
                const float dx = S.qx[j * NQ + qxi] - fx;   // constant over this lane's pixels
                float fa, fb;
                falloff_dx(dx, cn.x, cn.y, fa, fb);
                const bool col_in = lx >= x0 && lx <= x1;
                float cv[CP];
#pragma unroll
                for (int c = 0; c < CP; ++c) cv[c] = S.ch[j * CP + c];
                // zeros the compiler cannot fold into the first band's arithmetic (a
                // folded first band gives the skipped-band paths register copies)
                float s0, sy, syy, sop;
                opaque_zero2(s0, sy);
                opaque_zero2(syy, sop);
                float acc[NV];
#pragma unroll
                for (int c = 0; c + 1 < CP; c += 2) opaque_zero2(acc[6 + c], acc[7 + c]);
                if constexpr (CP & 1) acc[6 + CP - 1] = opaque_zero();
                bool any = false;
#pragma unroll
                for (int p = 0; p < PPL; ++p) {
                    // every band is evaluated (no uniform skips: the branches cost more
                    // than the evaluations they save); the lanes outside the box or past
                    // their pixel's last blended entry do not blend
                    const int ly = ly0 + Shp::ROWSTEP * p;
                    const bool inside = col_in && pos < L[p] && ly >= y0 && ly <= y1;
                    const float dy = S.qy[j * NQ + (ly >> 3)] - (float)(ly & 7);
                    float ep;
                    bool clamped;
                    const float alpha = falloff_alpha(fa, fb, dy, cn.z, cn.w, amax, ep, clamped);
                    if (inside && !(alpha < P.amin)) {   // this pixel blends entry j
                        any = true;
                        const float Tk = T[p] * __builtin_amdgcn_rcpf(1.0f - alpha);
                        const float wgt = alpha * Tk;
                        float g0 = 0.0f, g1 = 0.0f;
#pragma unroll
                        for (int c = 0; c < CP; ++c) {
                            acc[6 + c] = fmaf(wgt, G[p][c], acc[6 + c]);
                            if (c & 1) g1 = fmaf(G[p][c], cv[c], g1);
                            else g0 = fmaf(G[p][c], cv[c], g0);
                        }
                        const float dot = (g0 + g1) - gs[p];
                        gs[p] = fmaf(alpha, dot, gs[p]);
                        T[p] = Tk;
                        if (!clamped) {                      // dL/dalpha below the clamp
                            const float dg = Tk * dot;
                            sop = fmaf(dg, ep, sop);
                            const float dpow = dg * alpha;
                            s0 += dpow;
                            const float ey = dpow * dy;
                            sy += ey;
                            syy = fmaf(ey, dy, syy);
                        }
                    }
                }
                if (legs_ballot(any) == 0) continue;
                // power = -(A dx^2 + 2 B dx dy + C dy^2) / 2 with the unscaled conic:
                // d/dmean = -(conic . (dx, dy)) dpow, d/dA = -dx^2/2 dpow, d/dB = -dx dy dpow, ...
                const float A = cn.x * (1.0f / CONIC_SCALE_AC), Bc = cn.y * (1.0f / CONIC_SCALE_B),
                            Cc = cn.z * (1.0f / CONIC_SCALE_AC);
                const float sx = dx * s0;
                acc[0] = -fmaf(A, sx, Bc * sy);
                acc[1] = -fmaf(Bc, sx, Cc * sy);
                acc[2] = -0.5f * (dx * sx);
                acc[3] = -(dx * sy);
                acc[4] = -0.5f * syy;
                acc[5] = sop;
                legs_tr::reduce<NV>(acc, l);
                const uint32_t gid = (uint32_t)__builtin_amdgcn_readfirstlane((int)S.id[j]);   // scalar addressing
                float *g2d = grad2d + 8 * ((int64_t)ti.v * P.n + gid);
                float *dc = d_ch + (int64_t)gid * P.C;
#pragma unroll
                for (int r = 0; r < KF; ++r)
                    if (vok[r] && acc[r] != 0.0f) atomicAdd((vgeo[r] ? g2d : dc) + voff[r], acc[r]);
              }
            }
            hi = lo_rel;
            __syncthreads();
        }
    }
}

// ---- work counts (a statistics pass, not on the hot path) -------------------------

// Replays the forward decisions of every pixel and counts the algorithmic work
// units of the two blend kernels: counts[0] = alpha evaluations of the forward
// (list entries inside the pixel's box up to and including the stop),
// counts[1] = blended entries, counts[2] = alpha evaluations of the backward
// (entries inside the box before `last`), counts[3] = list positions walked.
template <int TILE>
__global__ void __launch_bounds__(TILE *TILE)
k_blend_count(BlendParams P, unsigned long long *__restrict__ counts)
{
    const int64_t tile = blockIdx.x;
    const TileInfo ti = tile_info<TILE>(P, tile);
    const float amax = P.amax;
    const int lx = threadIdx.x % TILE, ly = threadIdx.x / TILE;
    const int px = ti.tile_x0 + lx, py = ti.tile_y0 + ly;
    uint64_t ef = 0, bl = 0, eb = 0, walked = 0;
    if (px < ti.W && py < ti.H) {
        const int bx = px & ~7, by = py & ~7;
        const float fx = (float)(px & 7), fy = (float)(py & 7);
        float T = 1.0f;
        uint64_t skipped_since_blend = 0;
        for (uint32_t k = ti.rs; k < ti.re; ++k) {
            ++walked;
            const uint32_t gid = P.ids[k];
            const int64_t gv = (int64_t)ti.v * P.n + gid;
            const double2 m = P.mean2d[gv];
            const int4 b = P.box[gv];
            const float4 cn = scale_conic(P.conic[gv]);
            int x0 = min(max(b.x - ti.tile_x0, -1), TILE), x1 = min(max(b.y - ti.tile_x0, -1), TILE);
            int y0 = min(max(b.z - ti.tile_y0, -1), TILE), y1 = min(max(b.w - ti.tile_y0, -1), TILE);
            if (P.reach)
                reach_box<TILE>(cn, (float)(m.x - ((double)ti.tile_x0 + 0.5)), (float)(m.y - ((double)ti.tile_y0 + 0.5)),
                                P.amin, x0, x1, y0, y1);
            if (lx < x0 || lx > x1 || ly < y0 || ly > y1) continue;
            const float dx = (float)(m.x - ((double)bx + 0.5)) - fx;
            const float dy = (float)(m.y - ((double)by + 0.5)) - fy;
            float fa, fb, ep;
            bool clamped;
            falloff_dx(dx, cn.x, cn.y, fa, fb);
            const float alpha = falloff_alpha(fa, fb, dy, cn.z, cn.w, amax, ep, clamped);
            ++ef;
            if (alpha < P.amin) { ++skipped_since_blend; continue; }
            const float Tn = T * (1.0f - alpha);
            if (Tn < P.tmin) break;
            T = Tn;
            ++bl;
            eb += skipped_since_blend + 1;
            skipped_since_blend = 0;
        }
    }
    const uint64_t v[4] = {ef, bl, eb, walked};
    for (int q = 0; q < 4; ++q) {
        uint64_t x = v[q];
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, LEGS_WAVE);
        if (legs_lane() == 0 && x) atomicAdd(counts + q, (unsigned long long)x);
    }
}

__global__ void k_zero_counts(unsigned long long *c) { c[threadIdx.x] = 0ull; }

// Work bucket of a tile list of length n: 0 for an empty list, otherwise
// 1 + 4 floor(log2 n) + the two bits below the leading one (quarter octaves).
__device__ __forceinline__ int length_bucket(uint32_t n)
{
    if (n == 0) return 0;
    const int lz = 31 - __builtin_clz(n);
    const int q = lz >= 2 ? (int)((n >> (lz - 2)) & 3u) : (lz == 1 ? (int)((n & 1u) << 1) : 0);
    return 1 + 4 * lz + q;
}

constexpr int ORDER_BUCKETS = 1 + 4 * 32;

// The persistent blend launches' tile queue: every tile of every view in
// decreasing order of list length (longest-processing-time first, at quarter-
// octave resolution; order inside a bucket is arbitrary), and the queue
// counter reset. One workgroup; a kernel, so it records under graph capture.
__global__ void __launch_bounds__(1024)
k_tile_order(const uint32_t *__restrict__ ranges, int64_t T, uint32_t *__restrict__ order,
             uint32_t *__restrict__ counter)
{
    __shared__ uint32_t cnt[ORDER_BUCKETS];
    for (int b = threadIdx.x; b < ORDER_BUCKETS; b += blockDim.x) cnt[b] = 0u;
    if (threadIdx.x == 0) *counter = 0u;
    __syncthreads();
    for (int64_t t = threadIdx.x; t < T; t += blockDim.x)
        atomicAdd(&cnt[length_bucket(ranges[2 * t + 1] - ranges[2 * t])], 1u);
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t s = 0;
        for (int b = ORDER_BUCKETS - 1; b >= 0; --b) {
            const uint32_t c = cnt[b];
            cnt[b] = s;
            s += c;
        }
    }
    __syncthreads();
    for (int64_t t = threadIdx.x; t < T; t += blockDim.x) {
        const uint32_t pos = atomicAdd(&cnt[length_bucket(ranges[2 * t + 1] - ranges[2 * t])], 1u);
        order[pos] = (uint32_t)t;
    }
}

template <int TILE, int CP>
int32_t launch_tile_cp(legs_ctx *ctx, bool fwd, const BlendParams &P0, float *out, float *Tf,
                       uint32_t *last, const float *cTf, const uint32_t *clast, const float *d_out,
                       float *grad2d, float *d_ch, hipStream_t s)
{
    BlendParams P = P0;
    // single-wave backward workgroups stage at most 128 entries: a 256-entry
    // batch would let LDS, not registers, cap the waves per CU
    if (!fwd && BwdShape<TILE, CP>::NT == LEGS_WAVE && P.batch > 128) P.batch = 128;
    const size_t lds = Stage<TILE, CP>::bytes(P.batch);
    if (lds > 65536) return legs_set_error(ctx, LEGS_ERR_UNSUPPORTED, "LDS batch too large for C");
    int64_t grid = P.total_tiles;
    if (grid <= 0) return LEGS_OK;
    // forward launches at 32-pixel tiles run a workgroup per 16 x 16 part (a
    // part is a work item of its own, persistent or not)
    constexpr int SUB = TILE == 32 ? 16 : TILE;
    const bool parts = fwd && SUB < TILE;
    const int threads = fwd ? (parts ? SUB * SUB : TILE * TILE) : BwdShape<TILE, CP>::NT;
    if (parts) grid *= (TILE / SUB) * (TILE / SUB);
    if (P.counter) {
        // enough workgroups to fill every CU several times; each loops over tiles
        const int64_t per_cu = threads >= 1024 ? 2 : (threads >= 256 ? 6 : 12);
        const int64_t cap = (int64_t)ctx->num_cus * per_cu;
        grid = grid < cap ? grid : cap;
        hipLaunchKernelGGL(k_tile_order, dim3(1), dim3(1024), 0, s, P.ranges, P.total_tiles,
                           const_cast<uint32_t *>(P.order), P.counter);
    }
    if (parts) {
        hipLaunchKernelGGL((k_blend_fwd<TILE, CP, SUB>), dim3((unsigned)grid), dim3(threads), lds, s,
                           P, out, Tf, last);
    } else if (fwd) {
        hipLaunchKernelGGL((k_blend_fwd<TILE, CP, TILE>), dim3((unsigned)grid), dim3(threads), lds, s,
                           P, out, Tf, last);
    } else {
        hipLaunchKernelGGL((k_blend_bwd<TILE, CP>), dim3((unsigned)grid), dim3(threads), lds, s,
                           P, cTf, clast, d_out, grad2d, d_ch);
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
                        const float *channels, int32_t C, const legs_opts *o, int slot)
{
    BlendParams P;
    P.counter = nullptr;
    P.order = nullptr;
    P.zero4 = nullptr;
    P.zero_n4 = 0;
    P.zero_tail = 0;
    if (o->flags & LEGS_FLAG_PERSISTENT) {
        const legs_sort_layout Ls = legs_sort_layout_for(bins->capacity, total_tiles);
        P.counter = reinterpret_cast<uint32_t *>(static_cast<char *>(bins->scratch) + Ls.counter_off) + slot;
        // every persistent launch rebuilds the queue before it starts, so the
        // backward does not depend on a persistent forward having run
        P.order = reinterpret_cast<const uint32_t *>(static_cast<char *>(bins->scratch) + Ls.order_off);
    }
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
    P.reach = (o->flags & LEGS_FLAG_FULL_BOX) == 0;
    return P;
}

} // namespace

int32_t legs_launch_blend_forward(legs_ctx *ctx, const legs_projected *proj, int64_t n,
                                  const legs_bins *bins, const legs_view *views, int32_t n_views,
                                  int64_t total_tiles, const float *channels, int32_t C,
                                  const legs_opts *o, float *out, float *T_final, uint32_t *last,
                                  void *zero, int64_t zero_bytes, hipStream_t s)
{
    BlendParams P = make_params(proj, n, bins, views, n_views, total_tiles, channels, C, o,
                                LEGS_BLEND_COUNTER_FWD);
    if (zero && zero_bytes >= 4) {
        const int64_t words = zero_bytes / 4;
        P.zero4 = static_cast<float4 *>(zero);
        P.zero_n4 = words / 4;
        P.zero_tail = (int)(words % 4);
    }
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
    const BlendParams P = make_params(proj, n, bins, views, n_views, total_tiles, channels, C, o,
                                      LEGS_BLEND_COUNTER_BWD);
    return launch(ctx, false, P, nullptr, nullptr, nullptr, T_final, last, d_out, grad2d,
                  d_channels, o->tile, s);
}

int32_t legs_launch_blend_counts(legs_ctx *ctx, const legs_projected *proj, int64_t n,
                                 const legs_bins *bins, const legs_view *views, int32_t n_views,
                                 int64_t total_tiles, const legs_opts *o, uint64_t *counts,
                                 hipStream_t s)
{
    const BlendParams P = make_params(proj, n, bins, views, n_views, total_tiles, nullptr, 1, o,
                                      LEGS_BLEND_COUNTER_FWD);
    unsigned long long *c = reinterpret_cast<unsigned long long *>(counts);
    hipLaunchKernelGGL(k_zero_counts, dim3(1), dim3(4), 0, s, c);
    if (total_tiles > 0) {
        switch (o->tile) {
        case 8: hipLaunchKernelGGL(k_blend_count<8>, dim3((unsigned)total_tiles), dim3(64), 0, s, P, c); break;
        case 16: hipLaunchKernelGGL(k_blend_count<16>, dim3((unsigned)total_tiles), dim3(256), 0, s, P, c); break;
        case 32: hipLaunchKernelGGL(k_blend_count<32>, dim3((unsigned)total_tiles), dim3(1024), 0, s, P, c); break;
        default: return legs_set_error(ctx, LEGS_ERR_ARG, "tile must be 8, 16 or 32");
        }
    }
    LEGS_CHECK_LAUNCH(ctx);
    return LEGS_OK;
}
