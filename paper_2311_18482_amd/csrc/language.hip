// Language feature maps (gfx950): the decoder of Table 3 and F = M_infer S of
// the supplementary inference equations.
//
//  dmlp      D_MLP = 1x1 convolutions 8 -> 128 -> 256 -> N with ReLU (Table 3),
//            M_infer = softmax(D_MLP(R_s)) per pixel, top-1 = argmax.
//            BF16 weights and activations, FP32 accumulation on
//            v_mfma_f32_32x32x16_bf16; every layer is computed transposed
//            (units x pixels) so a layer's accumulators are the next layer's
//            B operand without moving data (the layout of the learned decode
//            of decode.hip); the biases enter through one MFMA per block
//            against "bias ones" (exact bf16 hi/mid/lo split of each bias).
//            All weight fragments live in LDS (144 KB at N = 128): one
//            workgroup per CU, each wave runs NT 32-pixel tiles at once so
//            that every fragment read from LDS feeds NT independent MFMAs.
//  features  F = M S with M the FP16 probabilities [P][N] written by dmlp and
//            S [N][d] the discrete feature space: one FP16 MFMA contraction
//            over N per 32 x 32 (d, pixel) block, S^T staged per workgroup in
//            LDS for a chunk of 256 feature dimensions, F written planar
//            [d][P] so that each accumulator register stores 32 consecutive
//            pixels of one feature dimension (full 128-byte lines).
#include "legs_internal.h"
#include "legs_decode_internal.h"

namespace {

typedef legs_f32x16 f32x16;
typedef __attribute__((ext_vector_type(8))) _Float16 f16x8;
typedef __attribute__((ext_vector_type(4))) _Float16 f16x4;

constexpr int H1 = LEGS_DMLP_H1, H2 = LEGS_DMLP_H2;
constexpr int B1 = H1 / 32, B2 = H2 / 32;        // 32-row blocks of layers 1 and 2
constexpr int S2 = H1 / 16, S3 = H2 / 16;        // k-steps of layers 2 and 3

template <int KB>
struct DmlpLds {
    legs_bf16x8 w1[B1 * 64];          // layer 1: W1 row (lower half), b1 split (upper half)
    legs_bf16x8 w2[B2 * S2 * 64];     // [block][k-step][lane]
    legs_bf16x8 bb2[B2 * 64];
    legs_bf16x8 w3[KB * S3 * 64];
    legs_bf16x8 bb3[KB * 64];
};

template <int KB>
__device__ __forceinline__ void dmlp_stage(const float *__restrict__ params, DmlpLds<KB> &L)
{
    const float *W1 = params + LEGS_DMLP_OFF_W1, *b1 = params + LEGS_DMLP_OFF_B1;
    const float *W2 = params + LEGS_DMLP_OFF_W2, *b2 = params + LEGS_DMLP_OFF_B2;
    const float *W3 = params + LEGS_DMLP_OFF_W3, *b3 = params + LEGS_DMLP_OFF_B3(KB);
    const int tid = threadIdx.x, nt = blockDim.x;
    __bf16 *w1 = reinterpret_cast<__bf16 *>(L.w1);
    __bf16 *w2 = reinterpret_cast<__bf16 *>(L.w2);
    __bf16 *w3 = reinterpret_cast<__bf16 *>(L.w3);
    __bf16 *bb2 = reinterpret_cast<__bf16 *>(L.bb2);
    __bf16 *bb3 = reinterpret_cast<__bf16 *>(L.bb3);
    // element (block, k-step, lane, e) of a fragment: row 32 block + lane % 32,
    // hidden unit legs_khid(k-step, lane / 32, e) of the previous layer
    for (int i = tid; i < B1 * 64 * 8; i += nt) {
        const int e = i & 7, l = (i >> 3) & 63, mb = i >> 9;
        const int row = 32 * mb + (l & 31);
        if ((l >> 5) == 0) {
            w1[i] = (__bf16)W1[row * LEGS_MLP_IN + e];
        } else {
            __bf16 p[3];
            legs_split3(b1[row], p[0], p[1], p[2]);
            w1[i] = e < 3 ? p[e] : (__bf16)0.0f;
        }
    }
    for (int i = tid; i < B2 * S2 * 64 * 8; i += nt) {
        const int e = i & 7, l = (i >> 3) & 63, ks = (i >> 9) % S2, mb = (i >> 9) / S2;
        w2[i] = (__bf16)W2[(32 * mb + (l & 31)) * H1 + legs_khid(ks, l >> 5, e)];
    }
    for (int i = tid; i < KB * S3 * 64 * 8; i += nt) {
        const int e = i & 7, l = (i >> 3) & 63, ks = (i >> 9) % S3, mb = (i >> 9) / S3;
        w3[i] = (__bf16)W3[(32 * mb + (l & 31)) * H2 + legs_khid(ks, l >> 5, e)];
    }
    for (int i = tid; i < (B2 + KB) * 64 * 8; i += nt) {
        const int e = i & 7, l = (i >> 3) & 63, mb = i >> 9;
        const bool second = mb < B2;
        const int blk = second ? mb : mb - B2;
        const float b = second ? b2[32 * blk + (l & 31)] : b3[32 * blk + (l & 31)];
        __bf16 p[3];
        legs_split3(b, p[0], p[1], p[2]);
        const __bf16 v = ((l >> 5) == 1 && e < 3) ? p[e] : (__bf16)0.0f;
        if (second) bb2[(blk * 64 + l) * 8 + e] = v;
        else bb3[(blk * 64 + l) * 8 + e] = v;
    }
}

// Hidden layers of NT tiles: x (inputs) -> h2 (B operand of layer 3).
// lds_off is an opaque zero refreshed per group so the compiler re-reads the
// fragments from LDS instead of holding them in registers.
template <int KB, int NT>
__device__ __forceinline__ void dmlp_hidden(const DmlpLds<KB> &L, int lds_off, const legs_bf16x8 (&x)[NT],
                                            legs_bf16x8 (&h2)[NT][S3])
{
    const int lane = __lane_id() + lds_off;
    const legs_bf16x8 ones = mlp_bias_ones(__lane_id() >> 5);
    legs_bf16x8 h1[NT][S2];
#pragma unroll
    for (int mb = 0; mb < B1; ++mb) {
        const legs_bf16x8 a = L.w1[mb * 64 + lane];
#pragma unroll
        for (int t = 0; t < NT; ++t) {
            const f32x16 z = legs_mfma(a, x[t], (f32x16){});
            h1[t][2 * mb] = relu_bf16x8(z, 0);
            h1[t][2 * mb + 1] = relu_bf16x8(z, 8);
        }
    }
#pragma unroll
    for (int mb = 0; mb < B2; ++mb) {
        const f32x16 cb = legs_mfma(L.bb2[mb * 64 + lane], ones, (f32x16){});
        f32x16 z[NT];
#pragma unroll
        for (int ks = 0; ks < S2; ++ks) {
            const legs_bf16x8 a = L.w2[(mb * S2 + ks) * 64 + lane];
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

template <int KB, int NT>
__device__ __forceinline__ void dmlp_logits_block(const DmlpLds<KB> &L, int lds_off, int mb,
                                                  const legs_bf16x8 (&h2)[NT][S3], f32x16 (&z)[NT])
{
    const int lane = __lane_id() + lds_off;
    const f32x16 cb = legs_mfma(L.bb3[mb * 64 + lane], mlp_bias_ones(__lane_id() >> 5), (f32x16){});
#pragma unroll
    for (int ks = 0; ks < S3; ++ks) {
        const legs_bf16x8 a = L.w3[(mb * S3 + ks) * 64 + lane];
#pragma unroll
        for (int t = 0; t < NT; ++t) z[t] = legs_mfma(a, h2[t][ks], ks == 0 ? cb : z[t]);
    }
}

template <int NT, bool VEC8, bool NORM>
__device__ __forceinline__ void dmlp_inputs(const float *__restrict__ feat, int64_t P, int64_t cs, int64_t ps,
                                            int64_t g, legs_bf16x8 (&x)[NT])
{
    const int lane = __lane_id(), h = lane >> 5;
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
                for (int e = 0; e < LEGS_MLP_IN; ++e) v[e] = legs_ldfeat(feat, p, e, cs, ps);
            }
        } else {
#pragma unroll
            for (int e = 0; e < LEGS_MLP_IN; ++e) v[e] = 0.0f;
        }
        x[t] = mlp_input<NORM>(v, h);
    }
}

__device__ __forceinline__ void argmax_pair(float &best, int &bidx)
{
    const float ob = __shfl_xor(best, 32, LEGS_WAVE);
    const int oi = __shfl_xor(bidx, 32, LEGS_WAVE);
    if (ob > best || (ob == best && oi < bidx)) { best = ob; bidx = oi; }
}

// Top-1 only: logits consumed block by block (each lane keeps the block
// holding its running maximum and searches it once at the end: the first
// maximum along increasing class index).
// Row-major input (VEC8): eight waves per workgroup. The weight fragments fill
// the LDS (one workgroup per CU) and such a wave fits in 256 registers, so two
// waves share each SIMD (MFMAs of one beside the other's conversions and
// argmax). The strided input's addressing would spill there: four waves.
template <int KB, int NT, bool VEC8, bool NORM>
__global__ void __launch_bounds__(VEC8 ? 512 : 256)
k_dmlp_top1(const float *__restrict__ feat, int64_t P, int64_t cs, int64_t ps,
            const float *__restrict__ params, int32_t *__restrict__ top1)
{
    __shared__ DmlpLds<KB> L;
    dmlp_stage<KB>(params, L);
    __syncthreads();
    const int lane = __lane_id(), wave = threadIdx.x / LEGS_WAVE, h = lane >> 5;
    const int nw = blockDim.x / LEGS_WAVE;
    const int64_t groups = (P + 32 * NT - 1) / (32 * NT);
    const int64_t stride = (int64_t)gridDim.x * nw;
    for (int64_t g = (int64_t)blockIdx.x * nw + wave; g < groups; g += stride) {
        int off = 0;
        asm volatile("" : "+s"(off));
        legs_bf16x8 x[NT];
        dmlp_inputs<NT, VEC8, NORM>(feat, P, cs, ps, g, x);
        legs_bf16x8 h2[NT][S3];
        dmlp_hidden<KB, NT>(L, off, x, h2);
        float best[NT];
        int sb[NT];
        f32x16 kept[NT];
#pragma unroll
        for (int mb = 0; mb < KB; ++mb) {
            f32x16 z[NT];
            dmlp_logits_block<KB, NT>(L, off, mb, h2, z);
#pragma unroll
            for (int t = 0; t < NT; ++t) {
                float m = z[t][0];
#pragma unroll
                for (int r = 1; r < 16; ++r) m = fmaxf(m, z[t][r]);
                const bool upd = mb == 0 || m > best[t];
                best[t] = upd ? m : best[t];
                sb[t] = upd ? mb : sb[t];
#pragma unroll
                for (int r = 0; r < 16; ++r) kept[t][r] = upd ? z[t][r] : kept[t][r];
            }
        }
#pragma unroll
        for (int t = 0; t < NT; ++t) {
            int pos = 15;
#pragma unroll
            for (int r = 14; r >= 0; --r) pos = kept[t][r] == best[t] ? r : pos;
            int k = 32 * sb[t] + legs_drow(pos, h);
            float bv = best[t];
            argmax_pair(bv, k);
            const int64_t p = (g * NT + t) * 32 + (lane & 31);
            if (h == 0 && p < P) top1[p] = k;
        }
    }
}

// Full distribution: all N logits of NT tiles kept, softmax, then the
// requested outputs: probs [P][N] float32, probs16 [P][N] float16 (the same
// float32 probability rounded to nearest), top1 [P].
// The distribution leaves through a 2.5 KB LDS tile per wave (the weights fill
// 144 KB): 32 codes x 32 pixels as halves (rows of PROW16), or 16 codes x 32
// pixels as floats (rows of PROW32), stored back as 64-byte runs per pixel
// instead of 8- or 16-byte pieces of 32 rows. The rows are padded so that a
// lane half's stores fall on distinct banks.
constexpr int PROW16 = 40, PROW32 = 20;   // 80-byte rows either way: 32 x 80 = 2560 bytes per wave

// LDS writes of this wave are done before its reads (and reads before the next writes).
__device__ __forceinline__ void stage_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <int KB, int NT, bool VEC8, bool NORM>
__global__ void __launch_bounds__(256)
k_dmlp_probs(const float *__restrict__ feat, int64_t P, int64_t cs, int64_t ps,
             const float *__restrict__ params, float *__restrict__ probs, _Float16 *__restrict__ probs16,
             int32_t *__restrict__ top1)
{
    constexpr int N = 32 * KB;
    __shared__ DmlpLds<KB> L;
    __shared__ __align__(16) float s_stage[4][32 * PROW32];
    dmlp_stage<KB>(params, L);
    __syncthreads();
    const int lane = __lane_id(), wave = threadIdx.x / LEGS_WAVE, h = lane >> 5;
    const int64_t groups = (P + 32 * NT - 1) / (32 * NT);
    const int64_t stride = (int64_t)gridDim.x * 4;
    for (int64_t g = (int64_t)blockIdx.x * 4 + wave; g < groups; g += stride) {
        int off = 0;
        asm volatile("" : "+s"(off));
        legs_bf16x8 x[NT];
        dmlp_inputs<NT, VEC8, NORM>(feat, P, cs, ps, g, x);
        legs_bf16x8 h2[NT][S3];
        dmlp_hidden<KB, NT>(L, off, x, h2);
        f32x16 z[KB][NT];
#pragma unroll
        for (int mb = 0; mb < KB; ++mb) dmlp_logits_block<KB, NT>(L, off, mb, h2, z[mb]);
#pragma unroll
        for (int t = 0; t < NT; ++t) {
            const int64_t p = (g * NT + t) * 32 + (lane & 31);
            float best = -INFINITY;
            int bidx = 0x7fffffff;
#pragma unroll
            for (int b = 0; b < KB; ++b)
#pragma unroll
                for (int r = 0; r < 16; ++r) {
                    const float sc = z[b][t][r];
                    if (sc > best) { best = sc; bidx = 32 * b + legs_drow(r, h); }
                }
            argmax_pair(best, bidx);
            float sum = 0.0f;
#pragma unroll
            for (int b = 0; b < KB; ++b)
#pragma unroll
                for (int r = 0; r < 16; ++r) {
                    z[b][t][r] = __expf(z[b][t][r] - best);
                    sum += z[b][t][r];
                }
            sum += __shfl_xor(sum, 32, LEGS_WAVE);
            const float inv = 1.0f / sum;
            if (top1 && h == 0 && p < P) top1[p] = bidx;
            const int64_t p0 = (g * NT + t) * 32;
            float *st = s_stage[wave];
#pragma unroll
            for (int b = 0; b < KB; ++b) {
                if (probs16) {
                    // 32 codes of 32 pixels as halves: rows of PROW16 halves
                    _Float16 *st16 = reinterpret_cast<_Float16 *>(st);
#pragma unroll
                    for (int j = 0; j < 4; ++j) {
                        const f16x4 q = {(_Float16)(z[b][t][4 * j] * inv), (_Float16)(z[b][t][4 * j + 1] * inv),
                                         (_Float16)(z[b][t][4 * j + 2] * inv), (_Float16)(z[b][t][4 * j + 3] * inv)};
                        *reinterpret_cast<f16x4 *>(st16 + (lane & 31) * PROW16 + 8 * j + 4 * h) = q;
                    }
                    stage_sync();
#pragma unroll
                    for (int q = 0; q < 2; ++q) {
                        const int row = (lane >> 2) + 16 * q, c8 = (lane & 3) * 8;
                        const f16x8 v = *reinterpret_cast<const f16x8 *>(st16 + row * PROW16 + c8);
                        if (p0 + row < P) *reinterpret_cast<f16x8 *>(probs16 + (p0 + row) * N + 32 * b + c8) = v;
                    }
                    stage_sync();
                }
                if (probs) {
                    // two halves of 16 codes as floats: rows of PROW32 floats
#pragma unroll
                    for (int half = 0; half < 2; ++half) {
#pragma unroll
                        for (int jj = 0; jj < 2; ++jj) {
                            const int j = 2 * half + jj;
                            *reinterpret_cast<float4 *>(st + (lane & 31) * PROW32 + 8 * jj + 4 * h) =
                                make_float4(z[b][t][4 * j] * inv, z[b][t][4 * j + 1] * inv, z[b][t][4 * j + 2] * inv,
                                            z[b][t][4 * j + 3] * inv);
                        }
                        stage_sync();
#pragma unroll
                        for (int q = 0; q < 2; ++q) {
                            const int row = (lane >> 2) + 16 * q, c4 = (lane & 3) * 4;
                            const float4 v = *reinterpret_cast<const float4 *>(st + row * PROW32 + c4);
                            if (p0 + row < P)
                                *reinterpret_cast<float4 *>(probs + (p0 + row) * N + 32 * b + 16 * half + c4) = v;
                        }
                        stage_sync();
                    }
                }
            }
        }
    }
}

// ---- F = M S ------------------------------------------------------------------------

constexpr int FCHUNK = 512;               // feature dimensions per workgroup (d = 512: M read once)
constexpr int FBLK = FCHUNK / 32;

template <int KB>
struct FeatLds {
    f16x8 s[FBLK * 2 * KB * 64];          // S^T fragments [d-block][k-step][lane]
};

__device__ __forceinline__ f32x16 mfma16(f16x8 a, f16x8 b, f32x16 c)
{
    return __builtin_amdgcn_mfma_f32_32x32x16_f16(a, b, c, 0, 0, 0);
}

// Grid: x = pixel groups (grid-stride), y = chunk of FCHUNK feature
// dimensions. A group is 32 NT consecutive pixels whose NT tiles interleave:
// column c of tile t is pixel 32 NT g + NT c + t, so each lane ends with NT
// neighbouring pixels of every output row and stores them as one vector (a
// half-wave writes 32 NT contiguous elements of a row of F; with one pixel per
// lane, half F took 2-byte stores and ran 25 % slower). B operand of
// k-step ks for pixel p: classes 16 ks + 8 (lane / 32) + e, one 16-byte load
// from the row M[p]. Sixteen waves per workgroup: the S fragments of 512
// dimensions fill the LDS (one workgroup per CU) and a wave fits in 128
// registers. vec: P % NT == 0 and F 16-byte aligned, else element stores.
template <int KB, int NT, bool OUT16>
__global__ void __launch_bounds__(1024)
k_lang_features(const _Float16 *__restrict__ M, int64_t P, const float *__restrict__ S, int d,
                void *__restrict__ F, int vec)
{
    constexpr int N = 32 * KB, KS = 2 * KB;
    __shared__ FeatLds<KB> L;
    const int d0 = blockIdx.y * FCHUNK;
    const int nblk = min(FBLK, (d - d0) / 32);
    {
        _Float16 *s = reinterpret_cast<_Float16 *>(L.s);
        for (int i = threadIdx.x; i < nblk * KS * 64 * 8; i += blockDim.x) {
            const int e = i & 7, l = (i >> 3) & 63, ks = (i >> 9) % KS, db = (i >> 9) / KS;
            const int dd = d0 + 32 * db + (l & 31);
            const int c = 16 * ks + 8 * (l >> 5) + e;
            s[i] = (_Float16)S[(int64_t)c * d + dd];
        }
    }
    __syncthreads();
    const int lane = __lane_id(), wave = threadIdx.x / LEGS_WAVE, h = lane >> 5;
    const int nw = blockDim.x / LEGS_WAVE;
    const int64_t groups = (P + 32 * NT - 1) / (32 * NT);
    const int64_t stride = (int64_t)gridDim.x * nw;
    for (int64_t g = (int64_t)blockIdx.x * nw + wave; g < groups; g += stride) {
        int off = 0;
        asm volatile("" : "+s"(off));
        f16x8 b[NT][KS];
#pragma unroll
        for (int t = 0; t < NT; ++t) {
            const int64_t p = g * NT * 32 + NT * (lane & 31) + t;
#pragma unroll
            for (int ks = 0; ks < KS; ++ks)
                b[t][ks] = p < P ? *reinterpret_cast<const f16x8 *>(M + p * N + 16 * ks + 8 * h) : (f16x8){};
        }
        for (int db = 0; db < nblk; ++db) {
            f32x16 acc[NT];
#pragma unroll
            for (int ks = 0; ks < KS; ++ks) {
                const f16x8 a = L.s[(db * KS + ks) * 64 + lane + off];
#pragma unroll
                for (int t = 0; t < NT; ++t) acc[t] = mfma16(a, b[t][ks], ks == 0 ? (f32x16){} : acc[t]);
            }
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int64_t p0 = g * NT * 32 + NT * (lane & 31);
                const int64_t o = (int64_t)(d0 + 32 * db + legs_drow(r, h)) * P + p0;
                if (vec) {
                    if (p0 < P) {
                        if constexpr (OUT16) {
                            typedef _Float16 hv __attribute__((ext_vector_type(NT)));
                            hv v;
#pragma unroll
                            for (int t = 0; t < NT; ++t) v[t] = (_Float16)acc[t][r];
                            *reinterpret_cast<hv *>(reinterpret_cast<_Float16 *>(F) + o) = v;
                        } else {
                            typedef float fv __attribute__((ext_vector_type(NT)));
                            fv v;
#pragma unroll
                            for (int t = 0; t < NT; ++t) v[t] = acc[t][r];
                            *reinterpret_cast<fv *>(reinterpret_cast<float *>(F) + o) = v;
                        }
                    }
                } else {
#pragma unroll
                    for (int t = 0; t < NT; ++t) {
                        if (p0 + t >= P) break;
                        if constexpr (OUT16) reinterpret_cast<_Float16 *>(F)[o + t] = (_Float16)acc[t][r];
                        else reinterpret_cast<float *>(F)[o + t] = acc[t][r];
                    }
                }
            }
        }
    }
}

int dmlp_grid(legs_ctx *ctx, int64_t P, int per_block, int per_cu)
{
    int64_t b = (P + per_block - 1) / per_block;
    const int64_t cap = (int64_t)ctx->num_cus * per_cu;
    if (b > cap) b = cap;
    return (int)(b < 1 ? 1 : b);
}

} // namespace

int32_t legs_launch_decode_dmlp(legs_ctx *ctx, const float *feat, int64_t P, int64_t cs, int64_t ps,
                                const float *params, int32_t N, int32_t mlp_flags, float *probs,
                                uint16_t *probs16, int32_t *top1, hipStream_t s)
{
    if (P == 0) return LEGS_OK;
    const bool norm = (mlp_flags & LEGS_MLP_NORMALIZE_INPUT) != 0;
    const bool vec8 = cs == 1 && ps == LEGS_MLP_IN && (reinterpret_cast<uintptr_t>(feat) & 15) == 0;
    _Float16 *p16 = reinterpret_cast<_Float16 *>(probs16);
    if (probs || probs16) {
        constexpr int NT = 2;
        const int grid = dmlp_grid(ctx, P, 32 * NT * 4, 1);
#define LEGS_DMLP_P(KB, V, NM) hipLaunchKernelGGL((k_dmlp_probs<KB, NT, V, NM>), dim3(grid), dim3(256), 0, s, \
                                                   feat, P, cs, ps, params, probs, p16, top1)
#define LEGS_DMLP_PN(KB) if (vec8) { if (norm) LEGS_DMLP_P(KB, true, true); else LEGS_DMLP_P(KB, true, false); } \
                         else { if (norm) LEGS_DMLP_P(KB, false, true); else LEGS_DMLP_P(KB, false, false); }
        switch (N) {
        case 32: LEGS_DMLP_PN(1) break;
        case 64: LEGS_DMLP_PN(2) break;
        default: LEGS_DMLP_PN(4) break;
        }
#undef LEGS_DMLP_PN
#undef LEGS_DMLP_P
    } else {
        constexpr int NT = 2;
        const int threads = vec8 ? 512 : 256;      // k_dmlp_top1's workgroup for each input layout
        const int grid = dmlp_grid(ctx, P, 32 * NT * (threads / LEGS_WAVE), 1);
#define LEGS_DMLP_T(KB, V, NM) hipLaunchKernelGGL((k_dmlp_top1<KB, NT, V, NM>), dim3(grid), dim3(threads), 0, s, \
                                                   feat, P, cs, ps, params, top1)
#define LEGS_DMLP_TN(KB) if (vec8) { if (norm) LEGS_DMLP_T(KB, true, true); else LEGS_DMLP_T(KB, true, false); } \
                         else { if (norm) LEGS_DMLP_T(KB, false, true); else LEGS_DMLP_T(KB, false, false); }
        switch (N) {
        case 32: LEGS_DMLP_TN(1) break;
        case 64: LEGS_DMLP_TN(2) break;
        default: LEGS_DMLP_TN(4) break;
        }
#undef LEGS_DMLP_TN
#undef LEGS_DMLP_T
    }
    LEGS_CHECK_LAUNCH(ctx);
    return LEGS_OK;
}

int32_t legs_launch_language_features(legs_ctx *ctx, const uint16_t *probs16, int64_t P, int32_t N,
                                      const float *S, int32_t d, int32_t out_f16, void *F, hipStream_t s)
{
    if (P == 0) return LEGS_OK;
    constexpr int NT = 2;
    const int gx = dmlp_grid(ctx, P, 32 * NT * 16, 1);
    const dim3 grid((unsigned)gx, (unsigned)((d + FCHUNK - 1) / FCHUNK));
    const _Float16 *M = reinterpret_cast<const _Float16 *>(probs16);
    const int vec = P % NT == 0 && (reinterpret_cast<uintptr_t>(F) & 15) == 0;
#define LEGS_FEAT(KB) if (out_f16) hipLaunchKernelGGL((k_lang_features<KB, NT, true>), grid, dim3(1024), 0, s, M, P, S, d, F, vec); \
                      else hipLaunchKernelGGL((k_lang_features<KB, NT, false>), grid, dim3(1024), 0, s, M, P, S, d, F, vec)
    switch (N) {
    case 32: LEGS_FEAT(1); break;
    case 64: LEGS_FEAT(2); break;
    default: LEGS_FEAT(4); break;
    }
#undef LEGS_FEAT
    LEGS_CHECK_LAUNCH(ctx);
    return LEGS_OK;
}
