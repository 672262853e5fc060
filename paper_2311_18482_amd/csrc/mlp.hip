// Training of the MLP decoder (gfx950): Eq. 9 cross-entropy against code
// index labels (or the uncertainty-weighted loss of Eqs. 10-12), gradients by
// the chain rule, and the fused Adam update of Sec. 4 (Adam, betas (0.9,
// 0.999)) used for both the decoder and the per-Gaussian parameters.
//
// Every contraction runs on v_mfma_f32_32x32x16_bf16 with float32 accumulation:
//   k_mlp_fb     per 32-pixel tile: the inference forward (so training sees
//                exactly the activations inference produces), softmax, CE,
//                dz3 = (p - onehot) w_p, then the backward through the layers
//                (dh2 = W3^T dz3, dz2 = dh2 [h2 > 0], dh1 = W2^T dz2, dz1 =
//                dh1 [h1 > 0], and the input gradient W1^T dz1) with the
//                upstream gradient split into two bf16 parts (hi + lo, 16
//                significant bits) and the W^T fragments in LDS next to the
//                forward ones; straight through the bf16 roundings. Writes
//                the layer inputs (bf16) and the dz (float32) unit-major
//                ([unit][pixel]) into the workspace.
//   k_mlp_wg     dW_l = sum_p dz_l h_(l-1)^T and db_l = sum_p dz_l: the pixels
//                are the MFMA contraction, read straight from the unit-major
//                planes (8 consecutive pixels of one unit = one fragment; dz
//                split into bf16 hi + lo as it is loaded); split over pixel
//                chunks (x) and layers (y), float atomics into the gradient.
// Workspace, Bp = B rounded up to 64 pixels: X [16][Bp] bf16 (the decoder
// input, then a row of ones), H1, H2 [64][Bp] bf16, DZ1, DZ2 [64][Bp] and
// DZ3 [K][Bp] float32: 200 + K floats per pixel.
#include "legs_internal.h"
#include "legs_decode_internal.h"

namespace {

typedef legs_f32x16 f32x16;
typedef legs_bf16x8 bf16x8;

constexpr int MH = LEGS_MLP_H;                     // 64 hidden units
static_assert(LEGS_MLP_WS_PER_PIXEL(0) == 8 + 32 + 32 + 64 + 64, "workspace layout");

// Per-pixel weighting of the cross-entropy. ru == NULL: the mean over the
// batch (Eq. 9). Otherwise the uncertainty-weighted loss of Eqs. 10-12:
// pixel p's CE is weighted by lce (1 - ru[p]) inv_hw, the loss gains
// lu ru[p] inv_hw, and d_ru[p] = (lu - lce CE_p) inv_hw.
struct CeWeights {
    const float *ru;
    float *d_ru;
    float lce, lu, inv_hw;
};

// Input gradient request: d_feat (NULL: none) receives dL/d(feature) at
// d_feat[c * dcs + p * dps]; with NORM the decoder input was f / |f| and its
// Jacobian (I - u u^T) / |f| (u = f / |f|) is applied, straight through the
// bf16 rounding of the input.
struct InputGrad {
    float *d_feat;
    int64_t dcs, dps;
};

struct MlpPlanes {
    int64_t Bp;
    __bf16 *X, *H1, *H2;
    float *D1, *D2, *D3;
};

MlpPlanes mlp_planes(void *ws, int64_t B, int32_t K)
{
    MlpPlanes P;
    P.Bp = (B + 63) / 64 * 64;
    char *c = static_cast<char *>(ws);
    P.X = reinterpret_cast<__bf16 *>(c);                  c += 16 * P.Bp * 2;
    P.H1 = reinterpret_cast<__bf16 *>(c);                 c += MH * P.Bp * 2;
    P.H2 = reinterpret_cast<__bf16 *>(c);                 c += MH * P.Bp * 2;
    P.D1 = reinterpret_cast<float *>(c);                  c += MH * P.Bp * 4;
    P.D2 = reinterpret_cast<float *>(c);                  c += MH * P.Bp * 4;
    P.D3 = reinterpret_cast<float *>(c);
    return P;
}

// W^T fragments of the backward: (block, k-step, lane, e) = row 32 block +
// lane % 32 of W^T (a unit of the layer below), column legs_khid(k-step,
// lane / 32, e) (a unit of the layer above).
template <int KB>
struct MlpBwdLds {
    bf16x8 t3[2 * 2 * KB * 64];     // W3^T: 64 rows x K
    bf16x8 t2[2 * 4 * 64];          // W2^T: 64 x 64
    bf16x8 t1[4 * 64];              // W1^T: 8 rows (block padded to 32) x 64
};

template <int KB>
__device__ __forceinline__ void mlp_stage_bwd(const float *__restrict__ params, MlpBwdLds<KB> &T)
{
    const float *W1 = params + LEGS_MLP_OFF_W1, *W2 = params + LEGS_MLP_OFF_W2, *W3 = params + LEGS_MLP_OFF_W3;
    const int tid = threadIdx.x, nt = blockDim.x;
    constexpr int S3 = 2 * KB;
    for (int i = tid; i < 2 * S3 * 64 * 8; i += nt) {
        const int e = i & 7, l = (i >> 3) & 63, ks = (i >> 9) % S3, mb = (i >> 9) / S3;
        reinterpret_cast<__bf16 *>(T.t3)[i] = (__bf16)W3[legs_khid(ks, l >> 5, e) * MH + 32 * mb + (l & 31)];
    }
    for (int i = tid; i < 2 * 4 * 64 * 8; i += nt) {
        const int e = i & 7, l = (i >> 3) & 63, ks = (i >> 9) & 3, mb = i >> 11;
        reinterpret_cast<__bf16 *>(T.t2)[i] = (__bf16)W2[legs_khid(ks, l >> 5, e) * MH + 32 * mb + (l & 31)];
    }
    for (int i = tid; i < 4 * 64 * 8; i += nt) {
        const int e = i & 7, l = (i >> 3) & 63, ks = i >> 9;
        const int row = l & 31;
        reinterpret_cast<__bf16 *>(T.t1)[i] =
            row < LEGS_MLP_IN ? (__bf16)W1[legs_khid(ks, l >> 5, e) * LEGS_MLP_IN + row] : (__bf16)0.0f;
    }
}

__device__ __forceinline__ void split8(const f32x16 &z, int first, bf16x8 &hi, bf16x8 &lo)
{
#pragma unroll
    for (int e = 0; e < 8; ++e) {
        const __bf16 a = (__bf16)z[first + e];
        hi[e] = a;
        lo[e] = (__bf16)(z[first + e] - (float)a);
    }
}

template <int KB, bool NORM>
__global__ void __launch_bounds__(256)
k_mlp_fb(const float *__restrict__ feat, int64_t B, int64_t cs, int64_t ps, const int32_t *__restrict__ labels,
         const float *__restrict__ params, MlpPlanes W, float *__restrict__ loss, CeWeights cw, InputGrad ig)
{
    constexpr int K = 32 * KB;
    __shared__ MlpLds L;
    __shared__ MlpBwdLds<KB> T;
    mlp_stage_weights<KB>(params, L);
    mlp_stage_bwd<KB>(params, T);
    __syncthreads();
    const int lane = __lane_id(), wave = threadIdx.x / LEGS_WAVE, h = lane >> 5;
    const int64_t tiles = W.Bp / 32;
    const int64_t stride = (int64_t)gridDim.x * 4;
    const float invB = 1.0f / (float)B;
    float lsum = 0.0f;
    MlpTile<KB> F;
    for (int64_t tile = (int64_t)blockIdx.x * 4 + wave; tile < tiles; tile += stride) {
        int off = 0;
        asm volatile("" : "+s"(off));   // fragments are re-read from LDS every tile
        const int ln = lane + off;
        const int64_t p = tile * 32 + (lane & 31);
        const bool valid = p < B;
        mlp_tile_forward<KB, NORM>(L, feat, p, valid, cs, ps, F, off);
        // softmax over the pixel's K logits (this lane and its partner)
        float mx = -INFINITY;
#pragma unroll
        for (int b = 0; b < KB; ++b)
#pragma unroll
            for (int r = 0; r < 16; ++r) mx = fmaxf(mx, F.z3[b][r]);
        mx = fmaxf(mx, __shfl_xor(mx, 32, LEGS_WAVE));
        float sum = 0.0f;
#pragma unroll
        for (int b = 0; b < KB; ++b)
#pragma unroll
            for (int r = 0; r < 16; ++r) sum += __expf(F.z3[b][r] - mx);
        sum += __shfl_xor(sum, 32, LEGS_WAVE);
        const float inv = 1.0f / sum;
        const int y = valid ? labels[p] : -1;
        float wpx = valid ? invB : 0.0f;
        if (cw.ru && valid) {
            const float ru = cw.ru[p];
            wpx = cw.lce * (1.0f - ru) * cw.inv_hw;
            if (h == 0) lsum += cw.lu * ru * cw.inv_hw;
        }
        // dz3 in place of the logits: (p - onehot) w_p; the loss and dL/dR_u
#pragma unroll
        for (int b = 0; b < KB; ++b)
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int k = 32 * b + legs_drow(r, h);
                const float pr = __expf(F.z3[b][r] - mx) * inv;
                if (k == y) {
                    const float ce = mx + __logf(sum) - F.z3[b][r];
                    lsum += ce * wpx;
                    if (cw.ru) cw.d_ru[p] = (cw.lu - cw.lce * ce) * cw.inv_hw;
                }
                F.z3[b][r] = (pr - (k == y ? 1.0f : 0.0f)) * wpx;
            }
        // layer inputs to the workspace (unit-major): X rows 0..7 the bf16
        // input, row 8 ones (the bias column of layer 1), rows 9..15 zero
        if (h == 0) {
            const __bf16 z0 = (__bf16)0.0f;
#pragma unroll
            for (int e = 0; e < 8; ++e) W.X[(int64_t)e * W.Bp + p] = valid ? F.x[e] : z0;
            W.X[8 * W.Bp + p] = valid ? (__bf16)1.0f : z0;
#pragma unroll
            for (int e = 9; e < 16; ++e) W.X[(int64_t)e * W.Bp + p] = z0;
        }
#pragma unroll
        for (int ks = 0; ks < 4; ++ks)
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                const int64_t o = (int64_t)legs_khid(ks, h, e) * W.Bp + p;
                W.H1[o] = valid ? F.h1[ks][e] : (__bf16)0.0f;
                W.H2[o] = valid ? F.h2[ks][e] : (__bf16)0.0f;
            }
#pragma unroll
        for (int b = 0; b < KB; ++b)
#pragma unroll
            for (int r = 0; r < 16; ++r) W.D3[(int64_t)(32 * b + legs_drow(r, h)) * W.Bp + p] = F.z3[b][r];
        // dh2 = W3^T dz3 (two blocks of 32 hidden units), gated by h2 > 0
        bf16x8 bh[2 * KB], bl[2 * KB];
#pragma unroll
        for (int b = 0; b < KB; ++b) {
            split8(F.z3[b], 0, bh[2 * b], bl[2 * b]);
            split8(F.z3[b], 8, bh[2 * b + 1], bl[2 * b + 1]);
        }
        f32x16 dz[2];
#pragma unroll
        for (int mb = 0; mb < 2; ++mb) {
            f32x16 acc = {};
#pragma unroll
            for (int ks = 0; ks < 2 * KB; ++ks) {
                const bf16x8 a = T.t3[(mb * 2 * KB + ks) * 64 + ln];
                acc = legs_mfma(a, bl[ks], legs_mfma(a, bh[ks], acc));
            }
#pragma unroll
            for (int r = 0; r < 16; ++r)
                if (!((float)F.h2[2 * mb + (r >> 3)][r & 7] > 0.0f)) acc[r] = 0.0f;
            dz[mb] = acc;
        }
        // dz2 stored; dh1 = W2^T dz2 gated by h1 > 0
        bf16x8 ch[4], cl[4];
#pragma unroll
        for (int mb = 0; mb < 2; ++mb) {
#pragma unroll
            for (int r = 0; r < 16; ++r) W.D2[(int64_t)(32 * mb + legs_drow(r, h)) * W.Bp + p] = dz[mb][r];
            split8(dz[mb], 0, ch[2 * mb], cl[2 * mb]);
            split8(dz[mb], 8, ch[2 * mb + 1], cl[2 * mb + 1]);
        }
#pragma unroll
        for (int mb = 0; mb < 2; ++mb) {
            f32x16 acc = {};
#pragma unroll
            for (int ks = 0; ks < 4; ++ks) {
                const bf16x8 a = T.t2[(mb * 4 + ks) * 64 + ln];
                acc = legs_mfma(a, cl[ks], legs_mfma(a, ch[ks], acc));
            }
#pragma unroll
            for (int r = 0; r < 16; ++r)
                if (!((float)F.h1[2 * mb + (r >> 3)][r & 7] > 0.0f)) acc[r] = 0.0f;
            dz[mb] = acc;
        }
#pragma unroll
        for (int mb = 0; mb < 2; ++mb) {
#pragma unroll
            for (int r = 0; r < 16; ++r) W.D1[(int64_t)(32 * mb + legs_drow(r, h)) * W.Bp + p] = dz[mb][r];
        }
        if (ig.d_feat) {
            // dx = W1^T dz1: inputs 4 h + r in registers r = 0..3
#pragma unroll
            for (int mb = 0; mb < 2; ++mb) {
                split8(dz[mb], 0, ch[2 * mb], cl[2 * mb]);
                split8(dz[mb], 8, ch[2 * mb + 1], cl[2 * mb + 1]);
            }
            f32x16 acc = {};
#pragma unroll
            for (int ks = 0; ks < 4; ++ks) {
                const bf16x8 a = T.t1[ks * 64 + ln];
                acc = legs_mfma(a, cl[ks], legs_mfma(a, ch[ks], acc));
            }
            float dx[4] = {acc[0], acc[1], acc[2], acc[3]};
            if constexpr (NORM) {
                float f[4], ss = 0.0f;
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    f[r] = valid ? legs_ldfeat(feat, p, 4 * h + r, cs, ps) : 0.0f;
                    ss = fmaf(f[r], f[r], ss);
                }
                ss += __shfl_xor(ss, 32, LEGS_WAVE);
                const float nrm = sqrtf(ss);
                const float iv = nrm > 0.0f ? 1.0f / nrm : 0.0f;
                float ud = 0.0f;
#pragma unroll
                for (int r = 0; r < 4; ++r) ud += f[r] * iv * dx[r];
                ud += __shfl_xor(ud, 32, LEGS_WAVE);
#pragma unroll
                for (int r = 0; r < 4; ++r) dx[r] = (dx[r] - ud * (f[r] * iv)) * iv;
            }
            if (valid) {
#pragma unroll
                for (int r = 0; r < 4; ++r) ig.d_feat[(int64_t)(4 * h + r) * ig.dcs + p * ig.dps] = dx[r];
            }
        }
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) lsum += __shfl_xor(lsum, o, LEGS_WAVE);
    if (lane == 0 && lsum != 0.0f) atomicAdd(loss, lsum);
}

// dW[m][k] += sum_p (dz_hi + dz_lo)[m][p] B[k][p] over the pixels of this
// workgroup's chunk, db[m] += sum_p dz[m][p]. Layer (blockIdx.y): 0: DZ1 x X
// (rows 0..7 the input, row 8 ones -> b1), 1: DZ2 x H1, 2: DZ3 x H2. Wave w
// owns the 32 rows of block w of dz against every block of B.
__global__ void __launch_bounds__(256)
k_mlp_wg(MlpPlanes W, int K, int64_t chunk, float *__restrict__ grad)
{
    const int layer = blockIdx.y;
    const int lane = __lane_id(), wave = threadIdx.x / LEGS_WAVE, h = lane >> 5;
    const float *Dp = layer == 0 ? W.D1 : layer == 1 ? W.D2 : W.D3;
    const __bf16 *Bp = layer == 0 ? W.X : layer == 1 ? W.H1 : W.H2;
    const int M = layer == 2 ? K : MH;
    const int Kb = layer == 0 ? 16 : MH;
    const int MB = M / 32, NB = (Kb + 31) / 32;
    if (wave >= MB) return;
    const int mb = wave, m = 32 * mb + (lane & 31);
    const int64_t g0 = (int64_t)blockIdx.x * chunk;
    const int64_t g1 = min(g0 + chunk, W.Bp);
    const float *Drow = Dp + (int64_t)m * W.Bp + 8 * h;
    const __bf16 *Bq0 = Bp + (int64_t)(lane & 31) * W.Bp + 8 * h;
    const __bf16 *Bq1 = Bp + (int64_t)(32 + (lane & 31)) * W.Bp + 8 * h;
    const bool k0 = (lane & 31) < Kb, k1 = NB > 1;
    f32x16 acc[2] = {};
    float dbs = 0.0f;
#pragma unroll 2
    for (int64_t g = g0; g < g1; g += 16) {
        const float4 v0 = *reinterpret_cast<const float4 *>(Drow + g);
        const float4 v1 = *reinterpret_cast<const float4 *>(Drow + g + 4);
        const float v[8] = {v0.x, v0.y, v0.z, v0.w, v1.x, v1.y, v1.z, v1.w};
        bf16x8 ah, al;
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            ah[e] = (__bf16)v[e];
            al[e] = (__bf16)(v[e] - (float)ah[e]);
            dbs += v[e];
        }
        const bf16x8 b0 = k0 ? *reinterpret_cast<const bf16x8 *>(Bq0 + g) : (bf16x8){};
        acc[0] = legs_mfma(al, b0, legs_mfma(ah, b0, acc[0]));
        if (k1) {
            const bf16x8 b1 = *reinterpret_cast<const bf16x8 *>(Bq1 + g);
            acc[1] = legs_mfma(al, b1, legs_mfma(ah, b1, acc[1]));
        }
    }
    const int KB = K / 32;
    if (layer != 0) {                                   // row sums: the bias gradient
        dbs += __shfl_xor(dbs, 32, LEGS_WAVE);
        float *db = grad + (layer == 1 ? LEGS_MLP_OFF_B2 : LEGS_MLP_OFF_B3(KB));
        if (h == 0 && dbs != 0.0f) atomicAdd(db + m, dbs);
    }
#pragma unroll
    for (int nb = 0; nb < 2; ++nb) {
        if (nb >= NB) continue;
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const int row = 32 * mb + legs_drow(r, h);
            const int col = 32 * nb + (lane & 31);
            const float x = acc[nb][r];
            if (col >= Kb || x == 0.0f) continue;
            if (layer == 0) {
                if (col < LEGS_MLP_IN) atomicAdd(grad + LEGS_MLP_OFF_W1 + row * LEGS_MLP_IN + col, x);
                else if (col == LEGS_MLP_IN) atomicAdd(grad + LEGS_MLP_OFF_B1 + row, x);
            } else {
                const int o = layer == 1 ? LEGS_MLP_OFF_W2 : LEGS_MLP_OFF_W3;
                atomicAdd(grad + o + row * MH + col, x);
            }
        }
    }
}

__global__ void __launch_bounds__(256)
k_zero_f32(float *__restrict__ p, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
        p[i] = 0.0f;
}

} // namespace

int64_t legs_mlp_workspace_floats(int64_t B, int32_t K)
{
    return (B + 63) / 64 * 64 * (int64_t)LEGS_MLP_WS_PER_PIXEL(K);
}

namespace {

// Forward and backward through the layers, then the weight gradients
// (accumulated into grad with float atomics).
int32_t mlp_train_kernels(legs_ctx *ctx, const float *feat, int64_t B, int64_t cs, int64_t ps,
                          const int32_t *labels, int32_t K, int32_t mlp_flags, const float *params,
                          float *workspace, float *grad, float *loss, const CeWeights &cw,
                          const InputGrad &ig, hipStream_t s)
{
    const int KB = K / 32;
    if (B == 0) return LEGS_OK;
    const MlpPlanes W = mlp_planes(workspace, B, K);
    int64_t g = (W.Bp / 32 + 3) / 4;
    const int64_t cap = (int64_t)ctx->num_cus * 2;
    if (g > cap) g = cap;
    const bool norm = (mlp_flags & LEGS_MLP_NORMALIZE_INPUT) != 0;
#define LEGS_MLP_TRAIN(KBV)                                                                                         \
    if (norm) hipLaunchKernelGGL((k_mlp_fb<KBV, true>), dim3((unsigned)g), dim3(256), 0, s, feat, B, cs, ps, labels, \
                                 params, W, loss, cw, ig);                                                           \
    else hipLaunchKernelGGL((k_mlp_fb<KBV, false>), dim3((unsigned)g), dim3(256), 0, s, feat, B, cs, ps, labels,    \
                            params, W, loss, cw, ig);
    switch (KB) {
    case 1: LEGS_MLP_TRAIN(1) break;
    case 2: LEGS_MLP_TRAIN(2) break;
    case 4: LEGS_MLP_TRAIN(4) break;
    default: return legs_set_error(ctx, LEGS_ERR_ARG, "K must be 32, 64 or 128");
    }
#undef LEGS_MLP_TRAIN
    LEGS_CHECK_LAUNCH(ctx);
    // pixel chunks of 256 to 4096 (a multiple of 64), about 256 per layer
    int64_t chunk = (W.Bp / 256 + 63) / 64 * 64;
    chunk = chunk < 256 ? 256 : (chunk > 4096 ? 4096 : chunk);
    const dim3 gw((unsigned)((W.Bp + chunk - 1) / chunk), 3);
    hipLaunchKernelGGL(k_mlp_wg, gw, dim3(256), 0, s, W, K, chunk, grad);
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
    const InputGrad ig = {nullptr, 0, 0};
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
    const InputGrad ig = {d_feat, dcs, dps};
    return mlp_train_kernels(ctx, feat, P, cs, ps, labels, K, mlp_flags, params, workspace, grad, loss, cw, ig, s);
}

// ---- fused Adam over parameter groups -------------------------------------------

namespace {

// Elements per workgroup of k_adam: four neighbouring floats per thread, four times.
constexpr int ADAM_CHUNK = 256 * 4 * 4;

struct AdamArgs {
    legs_adam_group g[LEGS_ADAM_MAX_GROUPS];
    int64_t bstart[LEGS_ADAM_MAX_GROUPS + 1];   // first workgroup of each group
    int vec[LEGS_ADAM_MAX_GROUPS];              // the group's four arrays are 16-byte aligned
    int n_groups;
    // omb = 1 - b rounded once from double (1 - 0.999f would be 1.3e-5 off
    // 0.001); c1 = 1 / (1 - b1^t), c2 = 1 / (1 - b2^t)
    float lr, b1, b2, omb1, omb2, eps, c1, c2;
};

__device__ __forceinline__ float adam_one(const AdamArgs &A, float p, float g, float &m, float &v)
{
    m = A.b1 * m + A.omb1 * g;
    v = A.b2 * v + A.omb2 * g * g;
    return p - A.lr * (m * A.c1) / (sqrtf(v * A.c2) + A.eps);
}

// Each workgroup updates one ADAM_CHUNK of one group, the group found by a
// wave-uniform walk over the workgroup counts (so its pointers are scalars);
// float4 access where the group is aligned, and the clamp test takes one
// remainder per four elements.
__global__ void __launch_bounds__(256)
k_adam(AdamArgs A)
{
    int k = 0;
    while (k + 1 < A.n_groups && (int64_t)blockIdx.x >= A.bstart[k + 1]) ++k;
    const legs_adam_group &G = A.g[k];
    const int64_t c0 = ((int64_t)blockIdx.x - A.bstart[k]) * ADAM_CHUNK;
    const int64_t c1 = c0 + ADAM_CHUNK < G.n ? c0 + ADAM_CHUNK : G.n;
    const int64_t ce = G.clamp_every;
    int64_t j0 = c0;
    if (A.vec[k]) {
        const int64_t q1 = c1 / 4;
        for (int64_t q = c0 / 4 + threadIdx.x; q < q1; q += 256) {
            float4 p = reinterpret_cast<const float4 *>(G.param)[q];
            const float4 g = reinterpret_cast<const float4 *>(G.grad)[q];
            float4 m = reinterpret_cast<const float4 *>(G.m)[q];
            float4 v = reinterpret_cast<const float4 *>(G.v)[q];
            p.x = adam_one(A, p.x, g.x, m.x, v.x);
            p.y = adam_one(A, p.y, g.y, m.y, v.y);
            p.z = adam_one(A, p.z, g.z, m.z, v.z);
            p.w = adam_one(A, p.w, g.w, m.w, v.w);
            if (ce > 0) {
                const int64_t r0 = (4 * q) % ce;
                const int64_t r1 = r0 + 1 == ce ? 0 : r0 + 1, r2 = r1 + 1 == ce ? 0 : r1 + 1,
                              r3 = r2 + 1 == ce ? 0 : r2 + 1;
                const float lo = G.clamp_lo, hi = G.clamp_hi;
                const int64_t off = G.clamp_offset;
                if (r0 == off) p.x = fminf(fmaxf(p.x, lo), hi);
                if (r1 == off) p.y = fminf(fmaxf(p.y, lo), hi);
                if (r2 == off) p.z = fminf(fmaxf(p.z, lo), hi);
                if (r3 == off) p.w = fminf(fmaxf(p.w, lo), hi);
            }
            reinterpret_cast<float4 *>(G.m)[q] = m;
            reinterpret_cast<float4 *>(G.v)[q] = v;
            reinterpret_cast<float4 *>(G.param)[q] = p;
        }
        j0 = 4 * q1;
    }
    for (int64_t j = j0 + threadIdx.x; j < c1; j += 256) {
        float m = G.m[j], v = G.v[j];
        float p = adam_one(A, G.param[j], G.grad[j], m, v);
        G.m[j] = m;
        G.v[j] = v;
        if (ce > 0 && (j % ce) == G.clamp_offset) p = fminf(fmaxf(p, G.clamp_lo), G.clamp_hi);
        G.param[j] = p;
    }
}

} // namespace

int32_t legs_launch_adam(legs_ctx *ctx, const legs_adam_group *groups, int32_t n_groups,
                         int32_t step, float lr, double beta1, double beta2, float eps, hipStream_t s)
{
    AdamArgs A;
    A.n_groups = n_groups;
    A.bstart[0] = 0;
    for (int k = 0; k < n_groups; ++k) {
        const legs_adam_group &G = groups[k];
        A.g[k] = G;
        A.bstart[k + 1] = A.bstart[k] + (G.n + ADAM_CHUNK - 1) / ADAM_CHUNK;
        A.vec[k] = ((reinterpret_cast<uintptr_t>(G.param) | reinterpret_cast<uintptr_t>(G.grad) |
                     reinterpret_cast<uintptr_t>(G.m) | reinterpret_cast<uintptr_t>(G.v)) & 15) == 0;
    }
    A.lr = lr; A.eps = eps;
    A.b1 = (float)beta1; A.b2 = (float)beta2;
    A.omb1 = (float)(1.0 - beta1); A.omb2 = (float)(1.0 - beta2);
    A.c1 = (float)(1.0 / (1.0 - pow(beta1, (double)step)));
    A.c2 = (float)(1.0 / (1.0 - pow(beta2, (double)step)));
    const int64_t blocks = A.bstart[n_groups];
    if (blocks == 0) return LEGS_OK;
    hipLaunchKernelGGL(k_adam, dim3((unsigned)blocks), dim3(256), 0, s, A);
    LEGS_CHECK_LAUNCH(ctx);
    return LEGS_OK;
}
