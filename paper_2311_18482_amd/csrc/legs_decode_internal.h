// Internal decoder declarations shared by decode.hip and mlp.hip.
#pragma once

#include "legs_internal.h"

#define LEGS_DECODE_MAXD 512  // largest codebook dimension of the plain decode

// MLP decoder 8 -> 64 -> 64 -> K; float32 master parameters packed as
// W1 [64][8], b1 [64], W2 [64][64], b2 [64], W3 [K][64], b3 [K].
#define LEGS_MLP_IN 8
#define LEGS_MLP_H 64
#define LEGS_MLP_OFF_W1 0
#define LEGS_MLP_OFF_B1 (LEGS_MLP_H * LEGS_MLP_IN)
#define LEGS_MLP_OFF_W2 (LEGS_MLP_OFF_B1 + LEGS_MLP_H)
#define LEGS_MLP_OFF_B2 (LEGS_MLP_OFF_W2 + LEGS_MLP_H * LEGS_MLP_H)
#define LEGS_MLP_OFF_W3 (LEGS_MLP_OFF_B2 + LEGS_MLP_H)
#define LEGS_MLP_OFF_B3(KB) (LEGS_MLP_OFF_W3 + 32 * (KB) * LEGS_MLP_H)
#define LEGS_MLP_NPARAMS(KB) (LEGS_MLP_OFF_B3(KB) + 32 * (KB))
// Decoder of Table 3: 8 -> 128 -> 256 -> N; float32 masters packed as
// W1 [128][8], b1 [128], W2 [256][128], b2 [256], W3 [N][256], b3 [N].
#define LEGS_DMLP_H1 128
#define LEGS_DMLP_H2 256
#define LEGS_DMLP_OFF_W1 0
#define LEGS_DMLP_OFF_B1 (LEGS_DMLP_H1 * LEGS_MLP_IN)
#define LEGS_DMLP_OFF_W2 (LEGS_DMLP_OFF_B1 + LEGS_DMLP_H1)
#define LEGS_DMLP_OFF_B2 (LEGS_DMLP_OFF_W2 + LEGS_DMLP_H2 * LEGS_DMLP_H1)
#define LEGS_DMLP_OFF_W3 (LEGS_DMLP_OFF_B2 + LEGS_DMLP_H2)
#define LEGS_DMLP_OFF_B3(KB) (LEGS_DMLP_OFF_W3 + 32 * (KB) * LEGS_DMLP_H2)
#define LEGS_DMLP_NPARAMS(KB) (LEGS_DMLP_OFF_B3(KB) + 32 * (KB))

// Smoothing MLP of Table 4: 3 -> 128 -> 128 -> 128 -> 8; float32 masters packed
// W1 [128][3], b1 [128], W2 [128][128], b2, W3 [128][128], b3, W4 [8][128], b4 [8].
#define LEGS_SMOOTH_H 128
#define LEGS_SMOOTH_OUT 8
#define LEGS_SMOOTH_OFF_W1 0
#define LEGS_SMOOTH_OFF_B1 (LEGS_SMOOTH_OFF_W1 + LEGS_SMOOTH_H * 3)
#define LEGS_SMOOTH_OFF_W2 (LEGS_SMOOTH_OFF_B1 + LEGS_SMOOTH_H)
#define LEGS_SMOOTH_OFF_B2 (LEGS_SMOOTH_OFF_W2 + LEGS_SMOOTH_H * LEGS_SMOOTH_H)
#define LEGS_SMOOTH_OFF_W3 (LEGS_SMOOTH_OFF_B2 + LEGS_SMOOTH_H)
#define LEGS_SMOOTH_OFF_B3 (LEGS_SMOOTH_OFF_W3 + LEGS_SMOOTH_H * LEGS_SMOOTH_H)
#define LEGS_SMOOTH_OFF_W4 (LEGS_SMOOTH_OFF_B3 + LEGS_SMOOTH_H)
#define LEGS_SMOOTH_OFF_B4 (LEGS_SMOOTH_OFF_W4 + LEGS_SMOOTH_OUT * LEGS_SMOOTH_H)
#define LEGS_SMOOTH_NPARAMS (LEGS_SMOOTH_OFF_B4 + LEGS_SMOOTH_OUT)

// Training workspace per pixel, in floats: X (16 bf16) 8 | H1, H2 (64 bf16) 32 each |
// DZ1, DZ2 (float) 64 each | DZ3 (float) K
#define LEGS_MLP_WS_PER_PIXEL(K) (200 + (K))

typedef __attribute__((ext_vector_type(8))) __bf16 legs_bf16x8;
typedef __attribute__((ext_vector_type(16))) float legs_f32x16;

// Per-lane MFMA fragments of every layer (bf16x8 = 16 bytes per lane), in LDS.
//   w1[mb]        layer 1, block mb: k-slots 0..7 (lower lane half) = W1 row,
//                 k-slots 8..10 (upper half) = the bias b1 split into three
//                 bf16 parts, rest 0
//   w2, w3        layers 2 and 3, [block][k-step]
//   bb2, bb3      the biases of layers 2 and 3 as an A operand: k-slots 8..10
//                 = the three bf16 parts of the bias, rest 0
// The three parts hi = bf16(b), mid = bf16(b - hi), lo = bf16(b - hi - mid)
// sum to b exactly (8 + 8 + 8 significant bits cover float32's 24), so an
// MFMA against the "bias ones" B operand (k-slots 8..10 = 1) yields the
// float32 bias in every accumulator row: the biases cost no registers, no
// VALU work and one 1 KB fragment per block.
struct MlpLds {
    legs_bf16x8 w1[2 * 64];
    legs_bf16x8 w2[2 * 4 * 64];
    legs_bf16x8 w3[4 * 4 * 64];
    legs_bf16x8 bb2[2 * 64];
    legs_bf16x8 bb3[4 * 64];
};

template <int KB>
struct MlpTile {
    legs_bf16x8 x;          // bf16 input (k-slots of the lower half), bias ones (upper half)
    legs_bf16x8 h1[4], h2[4];
    legs_f32x16 z3[KB];     // logits, class 32 b + 8 (r / 4) + 4 (lane / 32) + r % 4
};

typedef __attribute__((ext_vector_type(2))) short legs_i16x2;

// ReLU of 8 accumulator values as a bf16 fragment: rounding keeps the sign, so
// rounding first and then taking the signed 16-bit max with 0 on packed pairs
// gives the same bits as rounding max(z, 0) (-0 becomes +0 either way).
__device__ __forceinline__ legs_bf16x8 relu_bf16x8(const legs_f32x16 &z, int first)
{
    typedef __attribute__((ext_vector_type(2))) float f32x2;
    typedef __attribute__((ext_vector_type(2))) __bf16 bf16x2;
    typedef __attribute__((ext_vector_type(4))) uint32_t u32x4;
    u32x4 w;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        // one v_cvt_pk_bf16_f32 per pair, one v_pk_max_i16 per pair
        const f32x2 v = {z[first + 2 * j], z[first + 2 * j + 1]};
        const legs_i16x2 q = __builtin_bit_cast(legs_i16x2, __builtin_convertvector(v, bf16x2));
        w[j] = __builtin_bit_cast(uint32_t, __builtin_elementwise_max(q, (legs_i16x2){0, 0}));
    }
    return __builtin_bit_cast(legs_bf16x8, w);
}

// accumulator register r of lane half h holds row drow(r, h) of its 32-row block
__device__ __forceinline__ int legs_drow(int r, int h) { return 8 * (r >> 2) + 4 * h + (r & 3); }
// hidden unit fed by k-slot e of k-step ks (lane half h) when a 64-wide
// activation in accumulator layout is reused as the next layer's B operand
__device__ __forceinline__ int legs_khid(int ks, int h, int e)
{
    return 32 * (ks >> 1) + 8 * (2 * (ks & 1) + (e >> 2)) + 4 * h + (e & 3);
}

__device__ __forceinline__ float legs_ldfeat(const float *__restrict__ f, int64_t p, int c,
                                             int64_t cs, int64_t ps)
{
    return f[(int64_t)c * cs + p * ps];
}

// The B operand of the bias MFMAs (and the upper half of layer 1's input):
// k-slots 8..10 = 1 in the upper lane half, 0 elsewhere.
__device__ __forceinline__ legs_bf16x8 mlp_bias_ones(int h)
{
    legs_bf16x8 o = {};
    if (h) {
        o[0] = (__bf16)1.0f;
        o[1] = (__bf16)1.0f;
        o[2] = (__bf16)1.0f;
    }
    return o;
}

__device__ __forceinline__ void legs_split3(float b, __bf16 &hi, __bf16 &mid, __bf16 &lo)
{
    hi = (__bf16)b;
    const float r1 = b - (float)hi;
    mid = (__bf16)r1;
    lo = (__bf16)(r1 - (float)mid);
}

template <int KB>
__device__ __forceinline__ void mlp_stage_weights(const float *__restrict__ params, MlpLds &L)
{
    const float *W1 = params + LEGS_MLP_OFF_W1, *b1 = params + LEGS_MLP_OFF_B1;
    const float *W2 = params + LEGS_MLP_OFF_W2, *b2 = params + LEGS_MLP_OFF_B2;
    const float *W3 = params + LEGS_MLP_OFF_W3, *b3 = params + LEGS_MLP_OFF_B3(KB);
    const int tid = threadIdx.x, nt = blockDim.x;
    __bf16 *w1 = reinterpret_cast<__bf16 *>(L.w1);
    __bf16 *w2 = reinterpret_cast<__bf16 *>(L.w2);
    __bf16 *w3 = reinterpret_cast<__bf16 *>(L.w3);
    // fragment element (block, k-step, lane, e): row 32 block + lane % 32
    for (int i = tid; i < 2 * 64 * 8; i += nt) {
        const int e = i & 7, l = (i >> 3) & 63, mb = i >> 9;
        const int row = 32 * mb + (l & 31), hh = l >> 5;
        if (hh == 0) {
            w1[i] = (__bf16)W1[row * LEGS_MLP_IN + e];
        } else {
            __bf16 p[3];
            legs_split3(b1[row], p[0], p[1], p[2]);
            w1[i] = e < 3 ? p[e] : (__bf16)0.0f;
        }
    }
    for (int i = tid; i < 2 * 4 * 64 * 8; i += nt) {
        const int e = i & 7, l = (i >> 3) & 63, ks = (i >> 9) & 3, mb = i >> 11;
        w2[i] = (__bf16)W2[(32 * mb + (l & 31)) * LEGS_MLP_H + legs_khid(ks, l >> 5, e)];
    }
    for (int i = tid; i < KB * 4 * 64 * 8; i += nt) {
        const int e = i & 7, l = (i >> 3) & 63, ks = (i >> 9) & 3, mb = i >> 11;
        w3[i] = (__bf16)W3[(32 * mb + (l & 31)) * LEGS_MLP_H + legs_khid(ks, l >> 5, e)];
    }
    __bf16 *bb2 = reinterpret_cast<__bf16 *>(L.bb2);
    __bf16 *bb3 = reinterpret_cast<__bf16 *>(L.bb3);
    for (int i = tid; i < (2 + KB) * 64 * 8; i += nt) {
        const int e = i & 7, l = (i >> 3) & 63, mb = i >> 9;
        const bool second = mb < 2;
        const int blk = second ? mb : mb - 2;
        const float b = second ? b2[32 * blk + (l & 31)] : b3[32 * blk + (l & 31)];
        __bf16 p[3];
        legs_split3(b, p[0], p[1], p[2]);
        const __bf16 v = ((l >> 5) == 1 && e < 3) ? p[e] : (__bf16)0.0f;
        if (second) bb2[(blk * 64 + l) * 8 + e] = v;
        else bb3[(blk * 64 + l) * 8 + e] = v;
    }
}

__device__ __forceinline__ legs_f32x16 legs_mfma(legs_bf16x8 a, legs_bf16x8 b, legs_f32x16 c)
{
    return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
}

// Input fragment of one pixel: the feature (NORM: divided by its Euclidean
// norm, a zero feature staying zero), bf16, in the lower lane half; the bias
// ones in the upper half. v: the pixel's 8 features (read by the lower half).
template <bool NORM>
__device__ __forceinline__ legs_bf16x8 mlp_input(const float (&v)[LEGS_MLP_IN], int h)
{
    legs_bf16x8 x = mlp_bias_ones(h);
    if (h == 0) {
        float inv = 1.0f;
        if constexpr (NORM) {
            float ss = 0.0f;
#pragma unroll
            for (int e = 0; e < LEGS_MLP_IN; ++e) ss = fmaf(v[e], v[e], ss);
            const float nrm = sqrtf(ss);
            inv = nrm > 0.0f ? 1.0f / nrm : 0.0f;   // one division, then products
        }
#pragma unroll
        for (int e = 0; e < LEGS_MLP_IN; ++e) x[e] = (__bf16)(NORM ? v[e] * inv : v[e]);
    }
    return x;
}

// Hidden layers of NT 32-pixel tiles at once: every weight fragment read from
// LDS feeds NT independent MFMAs. lds_off is an opaque zero the caller
// refreshes per iteration so that the compiler keeps the fragments in LDS
// rather than in registers.
template <int NT>
__device__ __forceinline__ void mlp_hidden(const MlpLds &L, int lds_off, const legs_bf16x8 (&x)[NT],
                                           legs_bf16x8 (&h2)[NT][4])
{
    const int lane = __lane_id() + lds_off;
    const legs_bf16x8 ones = mlp_bias_ones(__lane_id() >> 5);
    legs_bf16x8 h1[NT][4];
#pragma unroll
    for (int mb = 0; mb < 2; ++mb) {
        const legs_bf16x8 a = L.w1[mb * 64 + lane];
        legs_f32x16 z[NT];
#pragma unroll
        for (int t = 0; t < NT; ++t) z[t] = legs_mfma(a, x[t], (legs_f32x16){});
#pragma unroll
        for (int t = 0; t < NT; ++t) {
            h1[t][2 * mb] = relu_bf16x8(z[t], 0);
            h1[t][2 * mb + 1] = relu_bf16x8(z[t], 8);
        }
    }
#pragma unroll
    for (int mb = 0; mb < 2; ++mb) {
        const legs_f32x16 cb = legs_mfma(L.bb2[mb * 64 + lane], ones, (legs_f32x16){});
        legs_f32x16 z[NT];
#pragma unroll
        for (int ks = 0; ks < 4; ++ks) {
            const legs_bf16x8 a = L.w2[(mb * 4 + ks) * 64 + lane];
#pragma unroll
            for (int t = 0; t < NT; ++t) z[t] = legs_mfma(a, h1[t][ks], ks == 0 ? cb : z[t]);
        }
#pragma unroll
        for (int t = 0; t < NT; ++t) {
            h2[t][2 * mb] = relu_bf16x8(z[t], 0);
            h2[t][2 * mb + 1] = relu_bf16x8(z[t], 8);
        }
    }
}

// Logit block mb (32 classes) of NT tiles.
template <int NT>
__device__ __forceinline__ void mlp_logits_block(const MlpLds &L, int lds_off, int mb, const legs_bf16x8 (&h2)[NT][4],
                                                 legs_f32x16 (&z)[NT])
{
    const int lane = __lane_id() + lds_off;
    const legs_f32x16 cb = legs_mfma(L.bb3[mb * 64 + lane], mlp_bias_ones(__lane_id() >> 5), (legs_f32x16){});
#pragma unroll
    for (int ks = 0; ks < 4; ++ks) {
        const legs_bf16x8 a = L.w3[(mb * 4 + ks) * 64 + lane];
#pragma unroll
        for (int t = 0; t < NT; ++t) z[t] = legs_mfma(a, h2[t][ks], ks == 0 ? cb : z[t]);
    }
}

// Forward of one 32-pixel tile keeping every activation (training, and the
// decode that writes probabilities). pixel p = 32 tile + lane % 32.
template <int KB, bool NORM>
__device__ __forceinline__ void mlp_tile_forward(const MlpLds &L, const float *__restrict__ feat,
                                                 int64_t p, bool valid, int64_t cs, int64_t ps,
                                                 MlpTile<KB> &T, int lds_off = 0)
{
    const int h = __lane_id() >> 5;
    float v[LEGS_MLP_IN];
#pragma unroll
    for (int e = 0; e < LEGS_MLP_IN; ++e) v[e] = (h == 0 && valid) ? legs_ldfeat(feat, p, e, cs, ps) : 0.0f;
    legs_bf16x8 x[1] = {mlp_input<NORM>(v, h)};
    T.x = x[0];
    const int lane = __lane_id() + lds_off;
#pragma unroll
    for (int mb = 0; mb < 2; ++mb) {
        const legs_f32x16 z = legs_mfma(L.w1[mb * 64 + lane], x[0], (legs_f32x16){});
        T.h1[2 * mb] = relu_bf16x8(z, 0);
        T.h1[2 * mb + 1] = relu_bf16x8(z, 8);
    }
    const legs_bf16x8 ones = mlp_bias_ones(h);
#pragma unroll
    for (int mb = 0; mb < 2; ++mb) {
        legs_f32x16 z = legs_mfma(L.bb2[mb * 64 + lane], ones, (legs_f32x16){});
#pragma unroll
        for (int ks = 0; ks < 4; ++ks) z = legs_mfma(L.w2[(mb * 4 + ks) * 64 + lane], T.h1[ks], z);
        T.h2[2 * mb] = relu_bf16x8(z, 0);
        T.h2[2 * mb + 1] = relu_bf16x8(z, 8);
    }
    legs_bf16x8 h2[1][4] = {{T.h2[0], T.h2[1], T.h2[2], T.h2[3]}};
#pragma unroll
    for (int mb = 0; mb < KB; ++mb) {
        legs_f32x16 z[1];
        mlp_logits_block<1>(L, lds_off, mb, h2, z);
        T.z3[mb] = z[0];
    }
}

// launchers
int32_t legs_launch_decode_plain(legs_ctx *ctx, const float *feat, int64_t P, int64_t cs,
                                 int64_t ps, const float *proj, int32_t D, const float *cb,
                                 int32_t K, float *probs, int32_t *top1, hipStream_t s);
int32_t legs_launch_decode_fold(legs_ctx *ctx, const float *proj, int32_t D, const float *cb,
                                int32_t K, float *folded, hipStream_t s);
int32_t legs_launch_decode_folded(legs_ctx *ctx, const float *feat, int64_t P, int64_t cs,
                                  int64_t ps, const float *folded, int32_t K, float *probs,
                                  int32_t *top1, hipStream_t s);
int32_t legs_launch_decode_mlp(legs_ctx *ctx, const float *feat, int64_t P, int64_t cs,
                               int64_t ps, const float *params, int32_t K, int32_t mlp_flags,
                               float *probs, int32_t *top1, hipStream_t s);
int32_t legs_launch_decode_dmlp(legs_ctx *ctx, const float *feat, int64_t P, int64_t cs, int64_t ps,
                                const float *params, int32_t N, int32_t mlp_flags, float *probs,
                                uint16_t *probs16, int32_t *top1, hipStream_t s);
int32_t legs_launch_language_features(legs_ctx *ctx, const uint16_t *probs16, int64_t P, int32_t N,
                                      const float *S, int32_t d, int32_t out_f16, void *F, hipStream_t s);
int64_t legs_smooth_workspace_bytes(int64_t n);
int32_t legs_launch_smooth(legs_ctx *ctx, const float *mean, const float *channels, int32_t C, int32_t sem,
                           int32_t uch, int64_t n, const float *params, float w_s, float lambda_smo,
                           void *workspace, float *grad, float *d_channels, float *loss, hipStream_t s);
int64_t legs_quantize_workspace_bytes(int64_t K, int32_t N, int32_t d);
int32_t legs_launch_quantize(legs_ctx *ctx, const uint16_t *feat, int64_t K, int32_t d, int32_t dC,
                             const float *S, int32_t N, float lam_d, float lam_cos, float lam_lb,
                             void *workspace, int32_t *index, uint32_t *counts, float *prob_mean,
                             float *losses, float *grad, hipStream_t s);
int64_t legs_mlp_workspace_floats(int64_t B, int32_t K);
int32_t legs_launch_mlp_grad(legs_ctx *ctx, const float *feat, int64_t B, int64_t cs, int64_t ps,
                             const int32_t *labels, int32_t K, int32_t mlp_flags, const float *params,
                             float *workspace, float *grad, float *loss, hipStream_t s);
int32_t legs_launch_semantic_loss_grad(legs_ctx *ctx, const float *feat, const float *ru, int64_t P,
                                       int64_t cs, int64_t ps, const int32_t *labels, int32_t K,
                                       int32_t mlp_flags, const float *params, float lambda_ce,
                                       float lambda_u, float inv_hw, float *workspace, float *grad,
                                       float *d_feat, int64_t dcs, int64_t dps, float *d_ru,
                                       float *loss, hipStream_t s);
int32_t legs_launch_adam(legs_ctx *ctx, const legs_adam_group *groups, int32_t n_groups,
                         int32_t step, float lr, double beta1, double beta2, float eps, hipStream_t s);
int32_t legs_launch_clear(legs_ctx *ctx, void *dev, int64_t words, hipStream_t s);
int32_t legs_launch_l1_loss_grad(legs_ctx *ctx, const float *out, const float *target,
                                 const legs_view *views, int32_t n_views, int64_t total_pixels,
                                 int32_t C, int32_t n_fit, float lambda_u, float *d_out,
                                 float *loss, hipStream_t s);
