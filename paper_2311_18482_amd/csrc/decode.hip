// Decoding rendered compact semantic features into a distribution over the
// discrete feature space S (gfx950).
//
//  plain   Sec. 3.3 Eq. 4: cosine max-similarity search of a feature against
//          every basis f_i of S. The rendered 8-d feature is first lifted to
//          the codebook dimension D by a fixed projection P (z = P f); scores
//          s_k = <c_k, z> / (|c_k| |z|), softmax over k, top-1 = argmax.
//          Both contractions (8 -> D, then D -> K) run on FP32 MFMA.
//  folded  the same scores from the exact identities <c_k, P f> = (C P f)_k
//          and |P f|^2 = f^T (P^T P) f: a K x 8 map and an 8 x 8 Gram matrix
//          (built once, float64 accumulation), one FP32 MFMA contraction.
//  mlp     Sec. 3.4.1 Eq. 8 and the supplementary inference equation:
//          softmax(D_MLP(R_s)), D_MLP = 1x1 convolutions, i.e. per-pixel
//          linear layers 8 -> 64 -> 64 -> K with ReLU (the layer pattern of
//          Table 3 at the widths used here). BF16 weights and activations,
//          FP32 accumulation on v_mfma_f32_32x32x16_bf16.
//
// MFMA layout used throughout (32x32 blocks, wave64): operand A holds row
// (lane % 32) and operand B column (lane % 32), each lane carrying the k-slots
// of its half (lane / 32); accumulator register r of lane l holds row
// 8 (r / 4) + 4 (l / 32) + r % 4, column l % 32. Every layer is computed
// transposed (features x pixels), so a layer's accumulators are already the
// next layer's B operand: k-slot e of k-step s is accumulator register
// 8 s + e, and the weights of the next layer are loaded with the matching
// column permutation. No data moves between layers.
#include "legs_internal.h"
#include "legs_decode_internal.h"

namespace {

typedef legs_f32x16 f32x16;

__device__ __forceinline__ int drow(int r, int h) { return legs_drow(r, h); }

__device__ __forceinline__ float ldfeat(const float *__restrict__ f, int64_t p, int c, int64_t cs,
                                        int64_t ps)
{
    return legs_ldfeat(f, p, c, cs, ps);
}

// Running argmax with lowest-index tie-break, then combined with the partner
// lane (lane ^ 32) that holds the other half of the same pixel's scores.
__device__ __forceinline__ void argmax_pair(float &best, int &bidx)
{
    const float ob = __shfl_xor(best, 32, LEGS_WAVE);
    const int oi = __shfl_xor(bidx, 32, LEGS_WAVE);
    if (ob > best || (ob == best && oi < bidx)) { best = ob; bidx = oi; }
}

// Staged row of write_softmax: 32 codes of one pixel plus 4 floats of padding
// (the 16-byte stores of one lane half then fall on distinct banks).
constexpr int SROW = 36;

// Softmax over the pixel's K scores held as KB blocks of 16 registers in this
// lane and its partner (exp taken once per score, in place); writes
// probs[p][K] for the wave's 32 pixels p0 .. p0 + 31 (those below P). Each
// block of 32 codes goes through this wave's LDS tile stage[32][SROW] and
// leaves as runs of 128 contiguous bytes per pixel (8 pixels per store
// instruction) instead of 32-byte pieces of 32 rows. Called by the whole wave.
template <int KB>
__device__ __forceinline__ void write_softmax(f32x16 (&s)[KB], float mx, int h, int64_t p0, int64_t P,
                                              float *__restrict__ probs, float *stage)
{
    float sum = 0.0f;
#pragma unroll
    for (int b = 0; b < KB; ++b)
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            s[b][r] = __expf(s[b][r] - mx);
            sum += s[b][r];
        }
    sum += __shfl_xor(sum, 32, LEGS_WAVE);
    const float inv = 1.0f / sum;
    const int lane = legs_lane(), px = lane & 31;
    const int rr = lane >> 3, c4 = (lane & 7) * 4;      // read-back: row rr + 8 q, codes c4 .. c4 + 3
#pragma unroll
    for (int b = 0; b < KB; ++b) {
#pragma unroll
        for (int j = 0; j < 4; ++j)
            *reinterpret_cast<float4 *>(stage + px * SROW + 8 * j + 4 * h) =
                make_float4(s[b][4 * j] * inv, s[b][4 * j + 1] * inv, s[b][4 * j + 2] * inv, s[b][4 * j + 3] * inv);
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int row = rr + 8 * q;
            const float4 v = *reinterpret_cast<const float4 *>(stage + row * SROW + c4);
            if (p0 + row < P) *reinterpret_cast<float4 *>(probs + (p0 + row) * (int64_t)(32 * KB) + 32 * b + c4) = v;
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();   // the tile's reads are done before the next block is staged
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
}

// ---- plain decode (direct) --------------------------------------------------------

constexpr int PLAIN_THREADS = 256;

template <int KB>
__global__ void __launch_bounds__(PLAIN_THREADS)
k_decode_plain(const float *__restrict__ feat, int64_t P, int64_t cs, int64_t ps,
               const float *__restrict__ proj, int D, const float *__restrict__ cb,
               float *__restrict__ probs, int32_t *__restrict__ top1)
{
    constexpr int K = 32 * KB;
    constexpr int NW = PLAIN_THREADS / LEGS_WAVE;
    constexpr int CPAD = 33;                       // padded codebook chunk row (bank spread)
    __shared__ float s_P[LEGS_DECODE_MAXD * LEGS_DECODE_DIN];
    __shared__ float s_cb[K * CPAD];
    __shared__ float s_inv[K];
    __shared__ __align__(16) float s_stage[NW][32 * SROW];
    const int tid = threadIdx.x, lane = legs_lane(), wave = tid / LEGS_WAVE, h = lane >> 5;
    for (int i = tid; i < D * LEGS_DECODE_DIN; i += PLAIN_THREADS) s_P[i] = proj[i];
    // inverse code norms
    for (int k = tid; k < K; k += PLAIN_THREADS) {
        float acc = 0.0f;
        for (int d = 0; d < D; ++d) { const float c = cb[(int64_t)k * D + d]; acc += c * c; }
        s_inv[k] = acc > 0.0f ? 1.0f / sqrtf(acc) : 0.0f;
    }
    __syncthreads();
    const int64_t tiles = (P + 31) / 32;
    const int64_t rounds = (tiles + NW - 1) / NW;
    for (int64_t rd = blockIdx.x; rd < rounds; rd += gridDim.x) {
        const int64_t tile = rd * NW + wave;
        const int64_t p = tile * 32 + (lane & 31);
        const bool valid = tile < tiles && p < P;
        // B operand of the lift: lane holds f[p][2 s + h]
        float fb[LEGS_DECODE_DIN / 2];
#pragma unroll
        for (int s = 0; s < LEGS_DECODE_DIN / 2; ++s) fb[s] = valid ? ldfeat(feat, p, 2 * s + h, cs, ps) : 0.0f;
        f32x16 S[KB];
#pragma unroll
        for (int b = 0; b < KB; ++b) S[b] = (f32x16){};
        float zz = 0.0f;
        for (int db = 0; db < D / 32; ++db) {
            __syncthreads();
            for (int i = tid; i < K * 32; i += PLAIN_THREADS) {
                const int k = i >> 5, c = i & 31;
                s_cb[k * CPAD + c] = cb[(int64_t)k * D + 32 * db + c];
            }
            __syncthreads();
            // Z^T block (32 dims x 32 px) = P[32 dims][8] x F^T[8][32 px]
            f32x16 Z = (f32x16){};
#pragma unroll
            for (int s = 0; s < LEGS_DECODE_DIN / 2; ++s) {
                const float a = s_P[(32 * db + (lane & 31)) * LEGS_DECODE_DIN + 2 * s + h];
                Z = __builtin_amdgcn_mfma_f32_32x32x2f32(a, fb[s], Z, 0, 0, 0);
            }
#pragma unroll
            for (int r = 0; r < 16; ++r) zz += Z[r] * Z[r];
            // S^T (K codes x 32 px) += C[:, block] x Z^T: k-step r pairs dim
            // drow(r, 0) (lower lanes) with drow(r, 1) (upper lanes)
#pragma unroll
            for (int r = 0; r < 16; ++r) {
#pragma unroll
                for (int b = 0; b < KB; ++b) {
                    const float a = s_cb[(32 * b + (lane & 31)) * CPAD + drow(r, h)];
                    S[b] = __builtin_amdgcn_mfma_f32_32x32x2f32(a, Z[r], S[b], 0, 0, 0);
                }
            }
        }
        zz += __shfl_xor(zz, 32, LEGS_WAVE);
        const float inz = zz > 0.0f ? 1.0f / sqrtf(zz) : 0.0f;
        float best = -INFINITY;
        int bidx = 0x7fffffff;
#pragma unroll
        for (int b = 0; b < KB; ++b)
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int k = 32 * b + drow(r, h);
                const float sc = S[b][r] * s_inv[k] * inz;
                S[b][r] = sc;
                if (sc > best) { best = sc; bidx = k; }   // k increases along the loop: first wins ties
            }
        argmax_pair(best, bidx);
        if (valid && h == 0) top1[p] = bidx;
        if (probs) write_softmax<KB>(S, best, h, tile * 32, P, probs, s_stage[wave]);
    }
}

// ---- folded plain decode ------------------------------------------------------

// folded = [K][8] rows (C_k P) / |C_k|, followed by the Gram matrix P^T P [8][8].
__global__ void __launch_bounds__(256)
k_decode_fold(const float *__restrict__ proj, int D, const float *__restrict__ cb, int K,
              float *__restrict__ folded)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    constexpr int DI = LEGS_DECODE_DIN;
    if (i < K * DI) {
        const int k = i / DI, j = i % DI;
        double acc = 0.0, nn = 0.0;
        for (int d = 0; d < D; ++d) {
            const double c = cb[(int64_t)k * D + d];
            acc += c * (double)proj[d * DI + j];
            nn += c * c;
        }
        folded[i] = nn > 0.0 ? (float)(acc / sqrt(nn)) : 0.0f;
    } else if (i < K * DI + DI * DI) {
        const int q = i - K * DI, a = q / DI, b = q % DI;
        double acc = 0.0;
        for (int d = 0; d < D; ++d) acc += (double)proj[d * DI + a] * (double)proj[d * DI + b];
        folded[i] = (float)acc;
    }
}

template <int KB>
__global__ void __launch_bounds__(256)
k_decode_folded(const float *__restrict__ feat, int64_t P, int64_t cs, int64_t ps,
                const float *__restrict__ folded, float *__restrict__ probs,
                int32_t *__restrict__ top1)
{
    constexpr int K = 32 * KB;
    constexpr int DI = LEGS_DECODE_DIN;
    __shared__ float s_M[K * DI];
    __shared__ float s_Q[DI * DI];
    __shared__ __align__(16) float s_stage[4][32 * SROW];
    const int tid = threadIdx.x, lane = legs_lane(), wave = tid / LEGS_WAVE, h = lane >> 5;
    for (int i = tid; i < K * DI; i += 256) s_M[i] = folded[i];
    if (tid < DI * DI) s_Q[tid] = folded[K * DI + tid];
    __syncthreads();
    // A operands of the K x 8 map are loop invariant: lane holds M[32 b + l%32][2 s + h]
    float am[KB][DI / 2];
#pragma unroll
    for (int b = 0; b < KB; ++b)
#pragma unroll
        for (int s = 0; s < DI / 2; ++s) am[b][s] = s_M[(32 * b + (lane & 31)) * DI + 2 * s + h];
    const int64_t tiles = (P + 31) / 32;
    const int64_t stride = (int64_t)gridDim.x * 4;
    for (int64_t tile = (int64_t)blockIdx.x * 4 + wave; tile < tiles; tile += stride) {
        const int64_t p = tile * 32 + (lane & 31);
        const bool valid = p < P;
        float f[DI];
#pragma unroll
        for (int j = 0; j < DI; ++j) f[j] = valid ? ldfeat(feat, p, j, cs, ps) : 0.0f;
        // |P f|^2 = f^T Q f (each lane of the pair computes it)
        float zz = 0.0f;
#pragma unroll
        for (int a = 0; a < DI; ++a) {
            float t = 0.0f;
#pragma unroll
            for (int b = 0; b < DI; ++b) t += s_Q[a * DI + b] * f[b];
            zz += f[a] * t;
        }
        const float inz = zz > 0.0f ? 1.0f / sqrtf(zz) : 0.0f;
        f32x16 S[KB];
#pragma unroll
        for (int b = 0; b < KB; ++b) {
            S[b] = (f32x16){};
#pragma unroll
            for (int s = 0; s < DI / 2; ++s)
                S[b] = __builtin_amdgcn_mfma_f32_32x32x2f32(am[b][s], f[2 * s + h], S[b], 0, 0, 0);
        }
        float best = -INFINITY;
        int bidx = 0x7fffffff;
#pragma unroll
        for (int b = 0; b < KB; ++b)
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int k = 32 * b + drow(r, h);
                const float sc = S[b][r] * inz;
                S[b][r] = sc;
                if (sc > best) { best = sc; bidx = k; }   // k increases along the loop: first wins ties
            }
        argmax_pair(best, bidx);
        if (valid && h == 0) top1[p] = bidx;
        if (probs) write_softmax<KB>(S, best, h, tile * 32, P, probs, s_stage[wave]);
    }
}

} // namespace

namespace {

template <int KB, bool NORM>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3)))
k_decode_mlp(const float *__restrict__ feat, int64_t P, int64_t cs, int64_t ps,
             const float *__restrict__ params, float *__restrict__ probs,
             int32_t *__restrict__ top1)
{
    __shared__ MlpLds L;
    __shared__ __align__(16) float s_stage[4][32 * SROW];
    mlp_stage_weights<KB>(params, L);
    __syncthreads();
    const int lane = legs_lane(), wave = threadIdx.x / LEGS_WAVE, h = lane >> 5;
    const int64_t tiles = (P + 31) / 32;
    const int64_t stride = (int64_t)gridDim.x * 4;
    MlpTile<KB> T;
    for (int64_t tile = (int64_t)blockIdx.x * 4 + wave; tile < tiles; tile += stride) {
        const int64_t p = tile * 32 + (lane & 31);
        const bool valid = p < P;
        int off = 0;
        asm volatile("" : "+s"(off));   // fragments are re-read from LDS every tile
        mlp_tile_forward<KB, NORM>(L, feat, p, valid, cs, ps, T, off);
        float best = -INFINITY;
        int bidx = 0x7fffffff;
        f32x16 S[KB];
#pragma unroll
        for (int b = 0; b < KB; ++b) {
            S[b] = T.z3[b];
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int k = 32 * b + drow(r, h);
                const float sc = S[b][r];
                if (sc > best) { best = sc; bidx = k; }   // k increases along the loop: first wins ties
            }
        }
        argmax_pair(best, bidx);
        if (valid && h == 0) top1[p] = bidx;
        if (probs) write_softmax<KB>(S, best, h, tile * 32, P, probs, s_stage[wave]);
    }
}

// Top-1 only: NT 32-pixel tiles per wave at once (each weight fragment read
// from LDS feeds NT MFMAs), logits consumed block by block. Per block a lane
// takes the maximum of its 16 logits; when it beats the running maximum, the
// class is the first position of that maximum in the block (KEEP: the
// block's logits are kept and searched once at the end; otherwise the
// position is found per block). Either way the result is the first maximum
// along increasing class index.
template <int KB, int NT, bool VEC8, bool KEEP, bool NORM>
__global__ void __launch_bounds__(256)
k_decode_mlp_top1(const float *__restrict__ feat, int64_t P, int64_t cs, int64_t ps,
                  const float *__restrict__ params, int32_t *__restrict__ top1)
{
    __shared__ MlpLds L;
    mlp_stage_weights<KB>(params, L);
    __syncthreads();
    const int lane = legs_lane(), wave = threadIdx.x / LEGS_WAVE, h = lane >> 5;
    const int64_t groups = (P + 32 * NT - 1) / (32 * NT);
    const int64_t stride = (int64_t)gridDim.x * 4;
    for (int64_t g = (int64_t)blockIdx.x * 4 + wave; g < groups; g += stride) {
        int off = 0;
        asm volatile("" : "+s"(off));   // fragments are re-read from LDS every group
        legs_bf16x8 x[NT];
#pragma unroll
        for (int t = 0; t < NT; ++t) {
            const int64_t p = (g * NT + t) * 32 + (lane & 31);
            float v[LEGS_MLP_IN];
            if (h == 0 && p < P) {
                if constexpr (VEC8) {
                    const float4 a = reinterpret_cast<const float4 *>(feat)[2 * p];
                    const float4 b = reinterpret_cast<const float4 *>(feat)[2 * p + 1];
                    v[0] = a.x; v[1] = a.y; v[2] = a.z; v[3] = a.w;
                    v[4] = b.x; v[5] = b.y; v[6] = b.z; v[7] = b.w;
                } else {
#pragma unroll
                    for (int e = 0; e < LEGS_MLP_IN; ++e) v[e] = ldfeat(feat, p, e, cs, ps);
                }
            } else {
#pragma unroll
                for (int e = 0; e < LEGS_MLP_IN; ++e) v[e] = 0.0f;
            }
            x[t] = mlp_input<NORM>(v, h);
        }
        legs_bf16x8 h2[NT][4];
        mlp_hidden<NT>(L, off, x, h2);
        float best[NT];
        int sb[NT];                       // KEEP: block of the maximum; else its class
        f32x16 kept[KEEP ? NT : 1];
#pragma unroll
        for (int mb = 0; mb < KB; ++mb) {
            f32x16 z[NT];
            mlp_logits_block<NT>(L, off, mb, h2, z);
#pragma unroll
            for (int t = 0; t < NT; ++t) {
                float m = z[t][0];
#pragma unroll
                for (int r = 1; r < 16; ++r) m = fmaxf(m, z[t][r]);
                const bool upd = mb == 0 || m > best[t];
                best[t] = upd ? m : best[t];
                if constexpr (KEEP) {
                    sb[t] = upd ? mb : sb[t];
#pragma unroll
                    for (int r = 0; r < 16; ++r) kept[t][r] = upd ? z[t][r] : kept[t][r];
                } else {
                    int pos = 15;
#pragma unroll
                    for (int r = 14; r >= 0; --r) pos = z[t][r] == m ? r : pos;
                    sb[t] = upd ? 32 * mb + drow(pos, h) : sb[t];
                }
            }
        }
#pragma unroll
        for (int t = 0; t < NT; ++t) {
            int k = sb[t];
            if constexpr (KEEP) {
                int pos = 15;
#pragma unroll
                for (int r = 14; r >= 0; --r) pos = kept[t][r] == best[t] ? r : pos;
                k = 32 * sb[t] + drow(pos, h);
            }
            float bv = best[t];
            argmax_pair(bv, k);
            const int64_t p = (g * NT + t) * 32 + (lane & 31);
            if (h == 0 && p < P) top1[p] = k;
        }
    }
}

int decode_grid(legs_ctx *ctx, int64_t P, int per_block)
{
    int64_t b = (P + per_block - 1) / per_block;
    const int64_t cap = (int64_t)ctx->num_cus * 8;
    if (b > cap) b = cap;
    return (int)(b < 1 ? 1 : b);
}

} // namespace

int32_t legs_launch_decode_plain(legs_ctx *ctx, const float *feat, int64_t P, int64_t cs,
                                 int64_t ps, const float *proj, int32_t D, const float *cb,
                                 int32_t K, float *probs, int32_t *top1, hipStream_t s)
{
    if (P == 0) return LEGS_OK;
    const int grid = decode_grid(ctx, P, 32 * 4);
    switch (K) {
    case 32: hipLaunchKernelGGL(k_decode_plain<1>, dim3(grid), dim3(PLAIN_THREADS), 0, s, feat, P, cs, ps, proj, D, cb, probs, top1); break;
    case 64: hipLaunchKernelGGL(k_decode_plain<2>, dim3(grid), dim3(PLAIN_THREADS), 0, s, feat, P, cs, ps, proj, D, cb, probs, top1); break;
    case 128: hipLaunchKernelGGL(k_decode_plain<4>, dim3(grid), dim3(PLAIN_THREADS), 0, s, feat, P, cs, ps, proj, D, cb, probs, top1); break;
    default: return legs_set_error(ctx, LEGS_ERR_ARG, "K must be 32, 64 or 128");
    }
    LEGS_CHECK_LAUNCH(ctx);
    return LEGS_OK;
}

int32_t legs_launch_decode_fold(legs_ctx *ctx, const float *proj, int32_t D, const float *cb,
                                int32_t K, float *folded, hipStream_t s)
{
    const int n = K * LEGS_DECODE_DIN + LEGS_DECODE_DIN * LEGS_DECODE_DIN;
    hipLaunchKernelGGL(k_decode_fold, dim3((n + 255) / 256), dim3(256), 0, s, proj, D, cb, K, folded);
    LEGS_CHECK_LAUNCH(ctx);
    return LEGS_OK;
}

int32_t legs_launch_decode_folded(legs_ctx *ctx, const float *feat, int64_t P, int64_t cs,
                                  int64_t ps, const float *folded, int32_t K, float *probs,
                                  int32_t *top1, hipStream_t s)
{
    if (P == 0) return LEGS_OK;
    const int grid = decode_grid(ctx, P, 32 * 4);
    switch (K) {
    case 32: hipLaunchKernelGGL(k_decode_folded<1>, dim3(grid), dim3(256), 0, s, feat, P, cs, ps, folded, probs, top1); break;
    case 64: hipLaunchKernelGGL(k_decode_folded<2>, dim3(grid), dim3(256), 0, s, feat, P, cs, ps, folded, probs, top1); break;
    case 128: hipLaunchKernelGGL(k_decode_folded<4>, dim3(grid), dim3(256), 0, s, feat, P, cs, ps, folded, probs, top1); break;
    default: return legs_set_error(ctx, LEGS_ERR_ARG, "K must be 32, 64 or 128");
    }
    LEGS_CHECK_LAUNCH(ctx);
    return LEGS_OK;
}

int32_t legs_launch_decode_mlp(legs_ctx *ctx, const float *feat, int64_t P, int64_t cs,
                               int64_t ps, const float *params, int32_t K, int32_t mlp_flags,
                               float *probs, int32_t *top1, hipStream_t s)
{
    if (P == 0) return LEGS_OK;
    if (K != 32 && K != 64 && K != 128) return legs_set_error(ctx, LEGS_ERR_ARG, "K must be 32, 64 or 128");
    const bool norm = (mlp_flags & LEGS_MLP_NORMALIZE_INPUT) != 0;
    if (probs) {
        const int grid = decode_grid(ctx, P, 32 * 4);
#define LEGS_MLP_ALL(KB)                                                                                     \
        if (norm) hipLaunchKernelGGL((k_decode_mlp<KB, true>), dim3(grid), dim3(256), 0, s, feat, P, cs, ps, params, probs, top1); \
        else hipLaunchKernelGGL((k_decode_mlp<KB, false>), dim3(grid), dim3(256), 0, s, feat, P, cs, ps, params, probs, top1);
        switch (K) {
        case 32: LEGS_MLP_ALL(1) break;
        case 64: LEGS_MLP_ALL(2) break;
        default: LEGS_MLP_ALL(4) break;
        }
#undef LEGS_MLP_ALL
    } else {
        constexpr int NT = 2;
        constexpr bool KEEP = true;
        const int grid = decode_grid(ctx, P, 32 * NT * 4);
        const bool vec8 = cs == 1 && ps == LEGS_MLP_IN && (reinterpret_cast<uintptr_t>(feat) & 15) == 0;
#define LEGS_MLP_TOP1(KB, NORM)                                                                       \
        if (vec8) hipLaunchKernelGGL((k_decode_mlp_top1<KB, NT, true, KEEP, NORM>), dim3(grid), dim3(256), 0, s, feat, P, cs, ps, params, top1); \
        else hipLaunchKernelGGL((k_decode_mlp_top1<KB, NT, false, KEEP, NORM>), dim3(grid), dim3(256), 0, s, feat, P, cs, ps, params, top1);
#define LEGS_MLP_TOP1N(KB) if (norm) { LEGS_MLP_TOP1(KB, true) } else { LEGS_MLP_TOP1(KB, false) }
        switch (K) {
        case 32: LEGS_MLP_TOP1N(1) break;
        case 64: LEGS_MLP_TOP1N(2) break;
        default: LEGS_MLP_TOP1N(4) break;
        }
#undef LEGS_MLP_TOP1N
#undef LEGS_MLP_TOP1
    }
    LEGS_CHECK_LAUNCH(ctx);
    return LEGS_OK;
}
