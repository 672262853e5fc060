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

typedef __attribute__((ext_vector_type(8))) __bf16 legs_bf16x8;
typedef __attribute__((ext_vector_type(16))) float legs_f32x16;

// Per-lane MFMA fragments of every layer (bf16x8 = 16 bytes per lane) and
// the biases in accumulator layout [block][lane half][register].
struct MlpLds {
    legs_bf16x8 w1[2 * 64];
    legs_bf16x8 w2[2 * 4 * 64];
    legs_bf16x8 w3[4 * 4 * 64];
    float b1[2 * 2 * 16];
    float b2[2 * 2 * 16];
    float b3[4 * 2 * 16];
};

template <int KB>
struct MlpTile {
    legs_bf16x8 x;          // bf16 input (k-slots of the lower half)
    legs_f32x16 z1[2], z2[2];
    legs_bf16x8 h1[4], h2[4];
    legs_f32x16 z3[KB];     // logits, class 32 b + 8 (r / 4) + 4 (lane / 32) + r % 4
};

typedef __attribute__((ext_vector_type(2))) short legs_i16x2;

// ReLU of 8 accumulator values as a bf16 fragment: rounding keeps the sign, so
// rounding first and then taking the signed 16-bit max with 0 on packed pairs
// gives the same bits as rounding max(z, 0) (-0 becomes +0 either way).
__device__ __forceinline__ legs_bf16x8 relu_bf16x8(const legs_f32x16 &z, int first)
{
    legs_bf16x8 h;
#pragma unroll
    for (int e = 0; e < 8; ++e) h[e] = (__bf16)z[first + e];
    typedef __attribute__((ext_vector_type(8))) short i16x8;
    i16x8 q = __builtin_bit_cast(i16x8, h);
    q = __builtin_elementwise_max(q, (i16x8){0, 0, 0, 0, 0, 0, 0, 0});
    return __builtin_bit_cast(legs_bf16x8, q);
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
        w1[i] = (__bf16)(hh == 0 ? W1[row * LEGS_MLP_IN + e] : 0.0f);
    }
    for (int i = tid; i < 2 * 4 * 64 * 8; i += nt) {
        const int e = i & 7, l = (i >> 3) & 63, ks = (i >> 9) & 3, mb = i >> 11;
        w2[i] = (__bf16)W2[(32 * mb + (l & 31)) * LEGS_MLP_H + legs_khid(ks, l >> 5, e)];
    }
    for (int i = tid; i < KB * 4 * 64 * 8; i += nt) {
        const int e = i & 7, l = (i >> 3) & 63, ks = (i >> 9) & 3, mb = i >> 11;
        w3[i] = (__bf16)W3[(32 * mb + (l & 31)) * LEGS_MLP_H + legs_khid(ks, l >> 5, e)];
    }
    for (int i = tid; i < 2 * 2 * 16; i += nt) {
        const int r = i & 15, hh = (i >> 4) & 1, mb = i >> 5;
        L.b1[i] = b1[32 * mb + legs_drow(r, hh)];
        L.b2[i] = b2[32 * mb + legs_drow(r, hh)];
    }
    for (int i = tid; i < KB * 2 * 16; i += nt) {
        const int r = i & 15, hh = (i >> 4) & 1, mb = i >> 5;
        L.b3[i] = b3[32 * mb + legs_drow(r, hh)];
    }
}

// Forward of one 32-pixel tile (pixel p = 32 tile + lane % 32).
template <int KB>
__device__ __forceinline__ void mlp_tile_forward(const MlpLds &L, const float *__restrict__ feat,
                                                 int64_t p, bool valid, int64_t cs, int64_t ps,
                                                 MlpTile<KB> &T)
{
    const int lane = __lane_id(), h = lane >> 5;
    legs_bf16x8 x = {};
    if (h == 0 && valid) {
        // the feature divided by its Euclidean norm (zero stays zero)
        float v[LEGS_MLP_IN], ss = 0.0f;
#pragma unroll
        for (int e = 0; e < LEGS_MLP_IN; ++e) {
            v[e] = legs_ldfeat(feat, p, e, cs, ps);
            ss = fmaf(v[e], v[e], ss);
        }
        const float nrm = sqrtf(ss);
        const float inv = nrm > 0.0f ? 1.0f / nrm : 0.0f;   // one division, then products
#pragma unroll
        for (int e = 0; e < LEGS_MLP_IN; ++e) x[e] = (__bf16)(v[e] * inv);
    }
    T.x = x;
#pragma unroll
    for (int mb = 0; mb < 2; ++mb) {
        legs_f32x16 a;
#pragma unroll
        for (int r = 0; r < 16; ++r) a[r] = L.b1[(mb * 2 + h) * 16 + r];
        T.z1[mb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(L.w1[mb * 64 + lane], x, a, 0, 0, 0);
    }
#pragma unroll
    for (int ks = 0; ks < 4; ++ks) T.h1[ks] = relu_bf16x8(T.z1[ks >> 1], 8 * (ks & 1));
#pragma unroll
    for (int mb = 0; mb < 2; ++mb) {
        legs_f32x16 a;
#pragma unroll
        for (int r = 0; r < 16; ++r) a[r] = L.b2[(mb * 2 + h) * 16 + r];
#pragma unroll
        for (int ks = 0; ks < 4; ++ks)
            a = __builtin_amdgcn_mfma_f32_32x32x16_bf16(L.w2[(mb * 4 + ks) * 64 + lane], T.h1[ks], a, 0, 0, 0);
        T.z2[mb] = a;
    }
#pragma unroll
    for (int ks = 0; ks < 4; ++ks) T.h2[ks] = relu_bf16x8(T.z2[ks >> 1], 8 * (ks & 1));
#pragma unroll
    for (int mb = 0; mb < KB; ++mb) {
        legs_f32x16 a;
#pragma unroll
        for (int r = 0; r < 16; ++r) a[r] = L.b3[(mb * 2 + h) * 16 + r];
#pragma unroll
        for (int ks = 0; ks < 4; ++ks)
            a = __builtin_amdgcn_mfma_f32_32x32x16_bf16(L.w3[(mb * 4 + ks) * 64 + lane], T.h2[ks], a, 0, 0, 0);
        T.z3[mb] = a;
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
                               int64_t ps, const float *params, int32_t K, float *probs,
                               int32_t *top1, hipStream_t s);
int64_t legs_mlp_workspace_floats(int64_t B, int32_t K);
int32_t legs_launch_mlp_grad(legs_ctx *ctx, const float *feat, int64_t B, int64_t cs, int64_t ps,
                             const int32_t *labels, int32_t K, const float *params,
                             float *workspace, float *grad, float *loss, hipStream_t s);
int32_t legs_launch_adam(legs_ctx *ctx, const legs_adam_group *groups, int32_t n_groups,
                         int32_t step, float lr, float beta1, float beta2, float eps, hipStream_t s);
int32_t legs_launch_clear(legs_ctx *ctx, void *dev, int64_t words, hipStream_t s);
int32_t legs_launch_l1_loss_grad(legs_ctx *ctx, const float *out, const float *target,
                                 const legs_view *views, int32_t n_views, int64_t total_pixels,
                                 int32_t C, int32_t n_fit, float lambda_u, float *d_out,
                                 float *loss, hipStream_t s);
