// Training of the MLP decoder (gfx950): Eq. 9 cross-entropy against code
// index labels, gradients by the chain rule, and the fused Adam update of
// Sec. 4 (Adam, betas (0.9, 0.999)) used for both the decoder and the
// per-Gaussian parameters.
//
// The forward pass is the inference tile routine (BF16 MFMA, FP32
// accumulation), so training sees exactly the activations inference produces.
// Backward runs in FP32 and passes straight through the bf16 roundings:
//   k_mlp_fwd     logits, softmax, dz3 = (p - onehot) / B, loss; stores the
//                 bf16 input and hidden activations (as floats) per pixel
//   k_mlp_act     dh2 = W3^T dz3, dz2 = dh2 * [z2 > 0], dh1 = W2^T dz2,
//                 dz1 = dh1 * [z1 > 0] (one thread per pixel, weights in LDS)
//   k_mlp_wgrad   dW = dZ^T H and db = sum dZ for each layer: split-K over
//                 pixel chunks, 4x4 register tiles per thread, one float
//                 atomic per weight per chunk
// Workspace per pixel (floats): X 8 | H1 64 | H2 64 | DZ1 64 | DZ2 64 | DZ3 K.
#include "legs_internal.h"
#include "legs_decode_internal.h"

namespace {

constexpr int WS_X = 0, WS_H1 = 8, WS_H2 = 72, WS_DZ1 = 136, WS_DZ2 = 200, WS_DZ3 = 264;
static_assert(WS_DZ3 + 128 == LEGS_MLP_WS_PER_PIXEL(128), "workspace layout");

// Per-pixel weighting of the cross-entropy. ru == NULL: the mean over the
// batch (Eq. 9). Otherwise the uncertainty-weighted loss of Eqs. 10-12:
// pixel p's CE is weighted by lce (1 - ru[p]) inv_hw, the loss gains
// lu ru[p] inv_hw, and d_ru[p] = (lu - lce CE_p) inv_hw.
struct CeWeights {
    const float *ru;
    float *d_ru;
    float lce, lu, inv_hw;
};

template <int KB, bool NORM>
__global__ void __launch_bounds__(256)
k_mlp_fwd(const float *__restrict__ feat, int64_t B, int64_t cs, int64_t ps,
          const int32_t *__restrict__ labels, const float *__restrict__ params,
          float *__restrict__ ws, float *__restrict__ loss, CeWeights cw)
{
    constexpr int K = 32 * KB;
    constexpr int WS = WS_DZ3 + K;
    __shared__ MlpLds L;
    mlp_stage_weights<KB>(params, L);
    __syncthreads();
    const int lane = __lane_id(), wave = threadIdx.x / LEGS_WAVE, h = lane >> 5;
    const int64_t tiles = (B + 31) / 32;
    const int64_t stride = (int64_t)gridDim.x * 4;
    const float invB = 1.0f / (float)B;
    float lsum = 0.0f;
    MlpTile<KB> T;
    for (int64_t tile = (int64_t)blockIdx.x * 4 + wave; tile < tiles; tile += stride) {
        const int64_t p = tile * 32 + (lane & 31);
        const bool valid = p < B;
        mlp_tile_forward<KB, NORM>(L, feat, p, valid, cs, ps, T);
        float mx = -INFINITY;
#pragma unroll
        for (int b = 0; b < KB; ++b)
#pragma unroll
            for (int r = 0; r < 16; ++r) mx = fmaxf(mx, T.z3[b][r]);
        mx = fmaxf(mx, __shfl_xor(mx, 32, LEGS_WAVE));
        float sum = 0.0f;
#pragma unroll
        for (int b = 0; b < KB; ++b)
#pragma unroll
            for (int r = 0; r < 16; ++r) sum += __expf(T.z3[b][r] - mx);
        sum += __shfl_xor(sum, 32, LEGS_WAVE);
        if (!valid) continue;
        const int y = labels[p];
        float *w = ws + p * WS;
        const float inv = 1.0f / sum;
        float wpx = invB;
        if (cw.ru) {
            const float ru = cw.ru[p];
            wpx = cw.lce * (1.0f - ru) * cw.inv_hw;
            if (h == 0) lsum += cw.lu * ru * cw.inv_hw;
        }
#pragma unroll
        for (int b = 0; b < KB; ++b)
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                float4 d;
                float *dv = &d.x;
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const int k = 32 * b + 8 * j + 4 * h + i;
                    const float pr = __expf(T.z3[b][4 * j + i] - mx) * inv;
                    dv[i] = (pr - (k == y ? 1.0f : 0.0f)) * wpx;
                    if (k == y) {
                        const float ce = mx + __logf(sum) - T.z3[b][4 * j + i];
                        lsum += ce * wpx;
                        if (cw.ru) cw.d_ru[p] = (cw.lu - cw.lce * ce) * cw.inv_hw;
                    }
                }
                *reinterpret_cast<float4 *>(w + WS_DZ3 + 32 * b + 8 * j + 4 * h) = d;
            }
        // bf16 activations (as floats) in feature order
#pragma unroll
        for (int ks = 0; ks < 4; ++ks)
#pragma unroll
            for (int q = 0; q < 2; ++q) {
                const int f0 = legs_khid(ks, h, 4 * q);
                float4 a, c;
                a.x = (float)T.h1[ks][4 * q + 0]; a.y = (float)T.h1[ks][4 * q + 1];
                a.z = (float)T.h1[ks][4 * q + 2]; a.w = (float)T.h1[ks][4 * q + 3];
                c.x = (float)T.h2[ks][4 * q + 0]; c.y = (float)T.h2[ks][4 * q + 1];
                c.z = (float)T.h2[ks][4 * q + 2]; c.w = (float)T.h2[ks][4 * q + 3];
                *reinterpret_cast<float4 *>(w + WS_H1 + f0) = a;
                *reinterpret_cast<float4 *>(w + WS_H2 + f0) = c;
            }
        if (h == 0) {
            float4 a, c;
            a.x = (float)T.x[0]; a.y = (float)T.x[1]; a.z = (float)T.x[2]; a.w = (float)T.x[3];
            c.x = (float)T.x[4]; c.y = (float)T.x[5]; c.z = (float)T.x[6]; c.w = (float)T.x[7];
            *reinterpret_cast<float4 *>(w + WS_X) = a;
            *reinterpret_cast<float4 *>(w + WS_X + 4) = c;
        }
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) lsum += __shfl_xor(lsum, off, LEGS_WAVE);
    if (lane == 0 && lsum != 0.0f) atomicAdd(loss, lsum);
}

// dz2 and dz1 per pixel (straight-through the bf16 rounding; ReLU gate from
// the stored activation, which is positive exactly when z > 0).
// Input gradient request: d_feat (NULL: none) receives dL/d(feature) at
// d_feat[c * dcs + p * dps]; with NORM the decoder input was f / |f| and its
// Jacobian (I - u u^T) / |f| (u = f / |f|, from the feature re-read here) is
// applied, straight through the bf16 rounding of the input.
struct InputGrad {
    const float *feat;
    int64_t cs, ps;
    float *d_feat;
    int64_t dcs, dps;
};

template <int KB, bool NORM>
__global__ void __launch_bounds__(256)
k_mlp_act(int64_t B, const float *__restrict__ params, float *__restrict__ ws, InputGrad ig)
{
    constexpr int K = 32 * KB;
    constexpr int WS = WS_DZ3 + K;
    constexpr int H = LEGS_MLP_H;
    __shared__ float s_W3[K * H];
    __shared__ float s_W2[H * H];
    __shared__ float s_W1[H * LEGS_MLP_IN];
    const float *W1 = params + LEGS_MLP_OFF_W1, *W2 = params + LEGS_MLP_OFF_W2, *W3 = params + LEGS_MLP_OFF_W3;
    for (int i = threadIdx.x; i < K * H; i += blockDim.x) s_W3[i] = (float)(__bf16)W3[i];
    for (int i = threadIdx.x; i < H * H; i += blockDim.x) s_W2[i] = (float)(__bf16)W2[i];
    for (int i = threadIdx.x; i < H * LEGS_MLP_IN; i += blockDim.x) s_W1[i] = (float)(__bf16)W1[i];
    __syncthreads();
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < B;
         p += (int64_t)gridDim.x * blockDim.x) {
        float *w = ws + p * WS;
        float d[H];
#pragma unroll
        for (int j = 0; j < H; ++j) d[j] = 0.0f;
        for (int k4 = 0; k4 < K; k4 += 4) {
            const float4 dz = *reinterpret_cast<const float4 *>(w + WS_DZ3 + k4);
            const float *dzv = &dz.x;
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < H; ++j) d[j] += dzv[i] * s_W3[(k4 + i) * H + j];
        }
#pragma unroll
        for (int j4 = 0; j4 < H; j4 += 4) {
            const float4 hv = *reinterpret_cast<const float4 *>(w + WS_H2 + j4);
            d[j4 + 0] = hv.x > 0.0f ? d[j4 + 0] : 0.0f;
            d[j4 + 1] = hv.y > 0.0f ? d[j4 + 1] : 0.0f;
            d[j4 + 2] = hv.z > 0.0f ? d[j4 + 2] : 0.0f;
            d[j4 + 3] = hv.w > 0.0f ? d[j4 + 3] : 0.0f;
            *reinterpret_cast<float4 *>(w + WS_DZ2 + j4) =
                make_float4(d[j4 + 0], d[j4 + 1], d[j4 + 2], d[j4 + 3]);
        }
        float e[H];
#pragma unroll
        for (int i = 0; i < H; ++i) e[i] = 0.0f;
#pragma unroll
        for (int j = 0; j < H; ++j)
#pragma unroll
            for (int i = 0; i < H; ++i) e[i] += d[j] * s_W2[j * H + i];
#pragma unroll
        for (int i4 = 0; i4 < H; i4 += 4) {
            const float4 hv = *reinterpret_cast<const float4 *>(w + WS_H1 + i4);
            e[i4 + 0] = hv.x > 0.0f ? e[i4 + 0] : 0.0f;
            e[i4 + 1] = hv.y > 0.0f ? e[i4 + 1] : 0.0f;
            e[i4 + 2] = hv.z > 0.0f ? e[i4 + 2] : 0.0f;
            e[i4 + 3] = hv.w > 0.0f ? e[i4 + 3] : 0.0f;
            *reinterpret_cast<float4 *>(w + WS_DZ1 + i4) = make_float4(e[i4], e[i4 + 1], e[i4 + 2], e[i4 + 3]);
        }
        if (ig.d_feat) {
            float dx[LEGS_MLP_IN];
#pragma unroll
            for (int c = 0; c < LEGS_MLP_IN; ++c) dx[c] = 0.0f;
#pragma unroll
            for (int i = 0; i < H; ++i)
#pragma unroll
                for (int c = 0; c < LEGS_MLP_IN; ++c) dx[c] += e[i] * s_W1[i * LEGS_MLP_IN + c];
            if constexpr (NORM) {
                float f[LEGS_MLP_IN], ss = 0.0f;
#pragma unroll
                for (int c = 0; c < LEGS_MLP_IN; ++c) {
                    f[c] = legs_ldfeat(ig.feat, p, c, ig.cs, ig.ps);
                    ss = fmaf(f[c], f[c], ss);
                }
                const float nrm = sqrtf(ss);
                const float inv = nrm > 0.0f ? 1.0f / nrm : 0.0f;
                float ud = 0.0f;
#pragma unroll
                for (int c = 0; c < LEGS_MLP_IN; ++c) ud += f[c] * inv * dx[c];
#pragma unroll
                for (int c = 0; c < LEGS_MLP_IN; ++c) dx[c] = (dx[c] - ud * (f[c] * inv)) * inv;
            }
#pragma unroll
            for (int c = 0; c < LEGS_MLP_IN; ++c) ig.d_feat[(int64_t)c * ig.dcs + p * ig.dps] = dx[c];
        }
    }
}

// out[m][n] += sum_p A[p][m] * Bm[p][n] for m < Ma, n < Nb, plus
// bias[m] += sum_p A[p][m] (a virtual column of ones). Grid: x = pixel chunk,
// y = 64 x 64 output tile (the bias tile is the extra column block).
constexpr int WG_CHUNK = 512;
constexpr int WG_SUB = 32;

__global__ void __launch_bounds__(256)
k_mlp_wgrad(int64_t B, const float *__restrict__ ws, int WS, int offA, int Ma, int offB, int Nb,
            float *__restrict__ out, float *__restrict__ bias)
{
    __shared__ float sA[WG_SUB][64];
    __shared__ float sB[WG_SUB][65];
    const int tiles_n = (Nb + 1 + 63) / 64;
    const int tm = blockIdx.y / tiles_n, tn = blockIdx.y % tiles_n;
    const int m0 = tm * 64, n0 = tn * 64;
    const int tid = threadIdx.x, ty = tid / 16, tx = tid % 16;
    float acc[4][4] = {};
    const int64_t p0 = (int64_t)blockIdx.x * WG_CHUNK;
    const int64_t p1 = p0 + WG_CHUNK < B ? p0 + WG_CHUNK : B;
    for (int64_t ps = p0; ps < p1; ps += WG_SUB) {
        for (int i = tid; i < WG_SUB * 64; i += 256) {
            const int q = i / 64, c = i % 64;
            const int64_t p = ps + q;
            const int m = m0 + c, n = n0 + c;
            sA[q][c] = (p < p1 && m < Ma) ? ws[p * WS + offA + m] : 0.0f;
            sB[q][c] = (p < p1) ? (n < Nb ? ws[p * WS + offB + n] : (n == Nb ? 1.0f : 0.0f)) : 0.0f;
        }
        __syncthreads();
#pragma unroll 4
        for (int q = 0; q < WG_SUB; ++q) {
            float a[4], b[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) { a[i] = sA[q][ty * 4 + i]; b[i] = sB[q][tx * 4 + i]; }
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < 4; ++j) acc[i][j] += a[i] * b[j];
        }
        __syncthreads();
    }
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int m = m0 + ty * 4 + i, n = n0 + tx * 4 + j;
            if (m >= Ma || acc[i][j] == 0.0f) continue;
            if (n < Nb) atomicAdd(out + (int64_t)m * Nb + n, acc[i][j]);
            else if (n == Nb) atomicAdd(bias + m, acc[i][j]);
        }
}

__global__ void __launch_bounds__(256)
k_zero_f32(float *__restrict__ p, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
        p[i] = 0.0f;
}

} // namespace

int64_t legs_mlp_workspace_floats(int64_t B, int32_t K) { return B * (WS_DZ3 + (int64_t)K); }

namespace {

// Forward with dz3, hidden-layer backward (and the input gradient), weight
// gradients (accumulated into grad with float atomics).
int32_t mlp_train_kernels(legs_ctx *ctx, const float *feat, int64_t B, int64_t cs, int64_t ps,
                          const int32_t *labels, int32_t K, int32_t mlp_flags, const float *params,
                          float *workspace, float *grad, float *loss, const CeWeights &cw,
                          const InputGrad &ig, hipStream_t s)
{
    const int KB = K / 32;
    if (B == 0) return LEGS_OK;
    int64_t g = (B + 127) / 128;
    const int64_t cap = (int64_t)ctx->num_cus * 8;
    if (g > cap) g = cap;
    const int64_t ga = ((B + 255) / 256) < cap ? (B + 255) / 256 : cap;
    const bool norm = (mlp_flags & LEGS_MLP_NORMALIZE_INPUT) != 0;
#define LEGS_MLP_TRAIN(KBV)                                                                                         \
    if (norm) {                                                                                                     \
        hipLaunchKernelGGL((k_mlp_fwd<KBV, true>), dim3((unsigned)g), dim3(256), 0, s, feat, B, cs, ps, labels, params, workspace, loss, cw); \
        hipLaunchKernelGGL((k_mlp_act<KBV, true>), dim3((unsigned)ga), dim3(256), 0, s, B, params, workspace, ig); \
    } else {                                                                                                        \
        hipLaunchKernelGGL((k_mlp_fwd<KBV, false>), dim3((unsigned)g), dim3(256), 0, s, feat, B, cs, ps, labels, params, workspace, loss, cw); \
        hipLaunchKernelGGL((k_mlp_act<KBV, false>), dim3((unsigned)ga), dim3(256), 0, s, B, params, workspace, ig); \
    }
    switch (KB) {
    case 1: LEGS_MLP_TRAIN(1) break;
    case 2: LEGS_MLP_TRAIN(2) break;
    case 4: LEGS_MLP_TRAIN(4) break;
    default: return legs_set_error(ctx, LEGS_ERR_ARG, "K must be 32, 64 or 128");
    }
#undef LEGS_MLP_TRAIN
    LEGS_CHECK_LAUNCH(ctx);
    const int WS = WS_DZ3 + K;
    const unsigned chunks = (unsigned)((B + WG_CHUNK - 1) / WG_CHUNK);
    const int H = LEGS_MLP_H;
    // layer 3: dW3 [K][64] from DZ3 x H2, db3
    hipLaunchKernelGGL(k_mlp_wgrad, dim3(chunks, (unsigned)(((K + 63) / 64) * ((H + 1 + 63) / 64))), dim3(256), 0, s,
                       B, workspace, WS, WS_DZ3, K, WS_H2, H, grad + LEGS_MLP_OFF_W3, grad + LEGS_MLP_OFF_B3(KB));
    // layer 2: dW2 [64][64] from DZ2 x H1, db2
    hipLaunchKernelGGL(k_mlp_wgrad, dim3(chunks, (unsigned)((H + 1 + 63) / 64)), dim3(256), 0, s,
                       B, workspace, WS, WS_DZ2, H, WS_H1, H, grad + LEGS_MLP_OFF_W2, grad + LEGS_MLP_OFF_B2);
    // layer 1: dW1 [64][8] from DZ1 x X, db1
    hipLaunchKernelGGL(k_mlp_wgrad, dim3(chunks, 1), dim3(256), 0, s,
                       B, workspace, WS, WS_DZ1, H, WS_X, LEGS_MLP_IN, grad + LEGS_MLP_OFF_W1, grad + LEGS_MLP_OFF_B1);
    LEGS_CHECK_LAUNCH(ctx);
    return LEGS_OK;
}

} // namespace

int32_t legs_launch_mlp_grad(legs_ctx *ctx, const float *feat, int64_t B, int64_t cs, int64_t ps,
                             const int32_t *labels, int32_t K, int32_t mlp_flags, const float *params,
                             float *workspace, float *grad, float *loss, hipStream_t s)
{
    const int64_t np = LEGS_MLP_NPARAMS(K / 32);
    hipLaunchKernelGGL(k_zero_f32, dim3(64), dim3(256), 0, s, grad, np);
    hipLaunchKernelGGL(k_zero_f32, dim3(1), dim3(256), 0, s, loss, (int64_t)1);
    LEGS_CHECK_LAUNCH(ctx);
    const CeWeights cw = {nullptr, nullptr, 1.0f, 0.0f, 0.0f};
    const InputGrad ig = {nullptr, 0, 0, nullptr, 0, 0};
    return mlp_train_kernels(ctx, feat, B, cs, ps, labels, K, mlp_flags, params, workspace, grad, loss, cw, ig, s);
}

int32_t legs_launch_semantic_loss_grad(legs_ctx *ctx, const float *feat, const float *ru, int64_t P,
                                       int64_t cs, int64_t ps, const int32_t *labels, int32_t K,
                                       int32_t mlp_flags, const float *params, float lambda_ce,
                                       float lambda_u, float inv_hw, float *workspace, float *grad,
                                       float *d_feat, int64_t dcs, int64_t dps, float *d_ru,
                                       float *loss, hipStream_t s)
{
    const CeWeights cw = {ru, d_ru, lambda_ce, lambda_u, inv_hw};
    const InputGrad ig = {feat, cs, ps, d_feat, dcs, dps};
    return mlp_train_kernels(ctx, feat, P, cs, ps, labels, K, mlp_flags, params, workspace, grad, loss, cw, ig, s);
}

// ---- fused Adam over parameter groups -------------------------------------------

namespace {

struct AdamArgs {
    legs_adam_group g[LEGS_ADAM_MAX_GROUPS];
    int64_t start[LEGS_ADAM_MAX_GROUPS + 1];
    int n_groups;
    // omb = 1 - b rounded once from double (1 - 0.999f would be 1.3e-5 off
    // 0.001); c1 = 1 / (1 - b1^t), c2 = 1 / (1 - b2^t)
    float lr, b1, b2, omb1, omb2, eps, c1, c2;
};

__global__ void __launch_bounds__(256)
k_adam(AdamArgs A)
{
    const int64_t total = A.start[A.n_groups];
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < total; i += (int64_t)gridDim.x * 256) {
        int k = 0;
        while (k + 1 < A.n_groups && i >= A.start[k + 1]) ++k;
        const legs_adam_group &G = A.g[k];
        const int64_t j = i - A.start[k];
        const float g = G.grad[j];
        const float m = A.b1 * G.m[j] + A.omb1 * g;
        const float v = A.b2 * G.v[j] + A.omb2 * g * g;
        G.m[j] = m;
        G.v[j] = v;
        float p = G.param[j] - A.lr * (m * A.c1) / (sqrtf(v * A.c2) + A.eps);
        if (G.clamp_every > 0 && (j % G.clamp_every) == G.clamp_offset)
            p = fminf(fmaxf(p, G.clamp_lo), G.clamp_hi);
        G.param[j] = p;
    }
}

} // namespace

int32_t legs_launch_adam(legs_ctx *ctx, const legs_adam_group *groups, int32_t n_groups,
                         int32_t step, float lr, double beta1, double beta2, float eps, hipStream_t s)
{
    AdamArgs A;
    A.n_groups = n_groups;
    A.start[0] = 0;
    for (int k = 0; k < n_groups; ++k) {
        A.g[k] = groups[k];
        A.start[k + 1] = A.start[k] + groups[k].n;
    }
    A.lr = lr; A.eps = eps;
    A.b1 = (float)beta1; A.b2 = (float)beta2;
    A.omb1 = (float)(1.0 - beta1); A.omb2 = (float)(1.0 - beta2);
    A.c1 = (float)(1.0 / (1.0 - pow(beta1, (double)step)));
    A.c2 = (float)(1.0 / (1.0 - pow(beta2, (double)step)));
    const int64_t total = A.start[n_groups];
    if (total == 0) return LEGS_OK;
    int64_t g = (total + 255) / 256;
    const int64_t cap = (int64_t)ctx->num_cus * 16;
    if (g > cap) g = cap;
    hipLaunchKernelGGL(k_adam, dim3((unsigned)g), dim3(256), 0, s, A);
    LEGS_CHECK_LAUNCH(ctx);
    return LEGS_OK;
}
