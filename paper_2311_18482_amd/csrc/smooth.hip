// Adaptive spatial smoothing (Sec. 3.4.2, Eqs. 13-14; PE and MLP of Table 4),
// gfx950.
//
//   s_MLP = MLP(PE(p)), PE of configuration 0 (the position itself), MLP
//   3 -> 128 -> 128 -> 128 -> 8 with ReLU after the first three layers;
//   L_smo = mean_g [ |s_MLP - s_G*| + max(u_G*, w_s) |s_MLP* - s_G| ]
//   (* = stop gradient): the first term trains the MLP, the second pulls s_G
//   towards the smoothed feature; u and the position receive nothing.
//
// BF16 weights and hidden activations, FP32 accumulation on
// v_mfma_f32_32x32x16_bf16, every layer transposed (units x Gaussians) as in
// the decoders. The position enters the first layer unrounded: each
// coordinate is split into three bf16 parts (hi + mid + lo = the float32
// value exactly), so the first layer computes bf16(W1) p + b1 with p in
// float32. Backward through the layers on the same MFMAs with the upstream
// gradient split into two bf16 parts (hi + lo, 16 significant bits): W^T
// fragments stay in LDS next to the forward ones (153 KB in all).
//
//  k_smooth_fwd_bwd  per 32-Gaussian tile (two per wave): forward, loss,
//                    dL/ds_G (accumulated into the channel gradient), and
//                    dz of every layer; writes the bf16 hidden activations and
//                    dz (as its two bf16 parts) into the workspace planes in
//                    the weight gradient's operand order, each lane's 8 rows
//                    transposed across its group of 8 lanes first so that one
//                    16-byte store is one operand fragment.
//  k_smooth_wgrad    dW_l = sum_g dz_l h_(l-1)^T and db_l = sum_g dz_l: the
//                    Gaussians are the MFMA contraction, each operand one
//                    16-byte load (a wave's load of a 128-row plane is 1 KB
//                    contiguous); split over Gaussian chunks (x) and layers
//                    (y), float atomics into the gradient.
#include "legs_internal.h"
#include "legs_decode_internal.h"
#include "lane_transpose.h"

namespace {

typedef legs_f32x16 f32x16;
typedef legs_bf16x8 bf16x8;

constexpr int SH = LEGS_SMOOTH_H;         // 128 hidden units
constexpr int SB = SH / 32;               // 4 blocks
constexpr int SK = SH / 16;               // 8 k-steps
constexpr int SNT = 2;                    // tiles per wave

struct SmoothLds {
    bf16x8 w1[SB * 64];
    bf16x8 w2[SB * SK * 64], bb2[SB * 64];
    bf16x8 w3[SB * SK * 64], bb3[SB * 64];
    bf16x8 w4[SK * 64], bb4[64];
    bf16x8 t4[SB * 64];                   // W4^T
    bf16x8 t3[SB * SK * 64], t2[SB * SK * 64];
};

__device__ void smooth_stage(const float *__restrict__ P, SmoothLds &L)
{
    const float *W1 = P + LEGS_SMOOTH_OFF_W1, *b1 = P + LEGS_SMOOTH_OFF_B1;
    const float *W2 = P + LEGS_SMOOTH_OFF_W2, *b2 = P + LEGS_SMOOTH_OFF_B2;
    const float *W3 = P + LEGS_SMOOTH_OFF_W3, *b3 = P + LEGS_SMOOTH_OFF_B3;
    const float *W4 = P + LEGS_SMOOTH_OFF_W4, *b4 = P + LEGS_SMOOTH_OFF_B4;
    const int tid = threadIdx.x, nt = blockDim.x;
    // layer 1: lower half [wx wy wz wx wy wz wx wy], upper half [wz b_hi b_mid b_lo 0 0 0 0]
    for (int i = tid; i < SB * 64 * 8; i += nt) {
        const int e = i & 7, l = (i >> 3) & 63, mb = i >> 9;
        const int row = 32 * mb + (l & 31), h = l >> 5;
        __bf16 v;
        if (h == 0) {
            v = (__bf16)W1[row * 3 + e % 3];
        } else if (e == 0) {
            v = (__bf16)W1[row * 3 + 2];
        } else if (e <= 3) {
            __bf16 p[3];
            legs_split3(b1[row], p[0], p[1], p[2]);
            v = p[e - 1];
        } else {
            v = (__bf16)0.0f;
        }
        reinterpret_cast<__bf16 *>(L.w1)[i] = v;
    }
    // hidden layers and their transposes: fragment (block, k-step, lane, e)
    // = row 32 block + lane % 32, column legs_khid(k-step, lane / 32, e)
    for (int i = tid; i < SB * SK * 64 * 8; i += nt) {
        const int e = i & 7, l = (i >> 3) & 63, ks = (i >> 9) % SK, mb = (i >> 9) / SK;
        const int row = 32 * mb + (l & 31), col = legs_khid(ks, l >> 5, e);
        reinterpret_cast<__bf16 *>(L.w2)[i] = (__bf16)W2[row * SH + col];
        reinterpret_cast<__bf16 *>(L.w3)[i] = (__bf16)W3[row * SH + col];
        reinterpret_cast<__bf16 *>(L.t3)[i] = (__bf16)W3[col * SH + row];
        reinterpret_cast<__bf16 *>(L.t2)[i] = (__bf16)W2[col * SH + row];
    }
    for (int i = tid; i < SK * 64 * 8; i += nt) {       // W4: rows 8..31 zero
        const int e = i & 7, l = (i >> 3) & 63, ks = i >> 9;
        const int row = l & 31;
        reinterpret_cast<__bf16 *>(L.w4)[i] =
            row < LEGS_SMOOTH_OUT ? (__bf16)W4[row * SH + legs_khid(ks, l >> 5, e)] : (__bf16)0.0f;
    }
    // W4^T: k-slot e of half h is output legs_khid(0, h, e) (outputs 0..7
    // sit in slots 0..3 of both halves)
    for (int i = tid; i < SB * 64 * 8; i += nt) {
        const int e = i & 7, l = (i >> 3) & 63, mb = i >> 9;
        const int o = legs_khid(0, l >> 5, e);
        reinterpret_cast<__bf16 *>(L.t4)[i] =
            o < LEGS_SMOOTH_OUT ? (__bf16)W4[o * SH + 32 * mb + (l & 31)] : (__bf16)0.0f;
    }
    for (int i = tid; i < (2 * SB + 1) * 64 * 8; i += nt) {
        const int e = i & 7, l = (i >> 3) & 63, mb = i >> 9;
        const int row = 32 * (mb % SB) + (l & 31);
        float b = 0.0f;
        if (mb < SB) b = b2[row];
        else if (mb < 2 * SB) b = b3[row];
        else b = row < LEGS_SMOOTH_OUT ? b4[row] : 0.0f;
        __bf16 p[3];
        legs_split3(b, p[0], p[1], p[2]);
        const __bf16 v = ((l >> 5) == 1 && e < 3) ? p[e] : (__bf16)0.0f;
        __bf16 *dst = mb < SB ? reinterpret_cast<__bf16 *>(L.bb2) + (mb * 64 + l) * 8
                    : mb < 2 * SB ? reinterpret_cast<__bf16 *>(L.bb3) + ((mb - SB) * 64 + l) * 8
                                  : reinterpret_cast<__bf16 *>(L.bb4) + l * 8;
        dst[e] = v;
    }
}

// bf16 split of 8 accumulator values (first .. first + 7): hi = bf16(z),
// lo = bf16(z - hi)
__device__ __forceinline__ void split_bf16x8(const f32x16 &z, int first, bf16x8 &hi, bf16x8 &lo)
{
#pragma unroll
    for (int e = 0; e < 8; ++e) {
        const __bf16 a = (__bf16)z[first + e];
        hi[e] = a;
        lo[e] = (__bf16)(z[first + e] - (float)a);
    }
}

// Workspace planes are kept in the operand order of the weight-gradient
// MFMAs (legs_lt::frag_at with the Gaussians as the columns), so a forward
// store is one 16-byte fragment and a weight-gradient load of a 128-row plane
// is 1 KB contiguous per wave.
using legs_lt::frag_at;

struct SmoothArgs {
    const float *mean, *ch;
    int32_t C, sem, uch;
    int64_t n, Gp;
    const float *params;
    float w_s, inv_n;             // inv_n = lambda_smo / n
    float *d_ch, *loss;
    __bf16 *X, *H1, *H2, *H3;     // 16 and 128 (x 3) rows, fragment order (frag_at)
    __bf16 *D1, *D2, *D3, *D4;    // dz: hi plane then lo plane, 128 (x 3) and 8 rows
};

// Hidden-layer step: acc of block mb from B fragments x[NT][KS] and A
// fragments a(mb, ks) in LDS.
template <int KS>
__device__ __forceinline__ void layer_block(const bf16x8 *__restrict__ wA, const bf16x8 *__restrict__ bias,
                                            int mb, int lane, const bf16x8 (&x)[SNT][KS], f32x16 (&z)[SNT])
{
    const f32x16 cb = bias ? legs_mfma(bias[mb * 64 + lane], mlp_bias_ones(__lane_id() >> 5), (f32x16){}) : (f32x16){};
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) {
        const bf16x8 a = wA[(mb * KS + ks) * 64 + lane];
#pragma unroll
        for (int t = 0; t < SNT; ++t) z[t] = legs_mfma(a, x[t][ks], ks == 0 ? cb : z[t]);
    }
}

// Eight rows (row(e), e = 0..7) of this lane's Gaussian into a plane of R
// rows in fragment order: transposed across the lane's group of 8 (Gaussians
// g0 .. g0 + 7), lane i stores row(i) of those Gaussians, one 16-byte
// fragment; rows at or past R are not stored.
template <typename RowOf>
__device__ __forceinline__ void store_rows8(__bf16 *__restrict__ plane, int R, int64_t g0, bf16x8 v, RowOf row_of,
                                            int i8, bool b1, uint32_t psel)
{
    typedef __attribute__((ext_vector_type(4))) uint32_t u32x4;
    const u32x4 x = __builtin_bit_cast(u32x4, v);
    uint32_t w[4] = {x[0], x[1], x[2], x[3]};
    legs_lt::oct_transpose(w, b1, psel);
    const int row = row_of(i8);
    if (row < R) *reinterpret_cast<uint4 *>(plane + frag_at(g0, R, row)) = make_uint4(w[0], w[1], w[2], w[3]);
}

__global__ void __launch_bounds__(256)
k_smooth_fwd_bwd(SmoothArgs A)
{
    __shared__ SmoothLds L;
    smooth_stage(A.params, L);
    __syncthreads();
    const int lane = __lane_id(), wave = threadIdx.x / LEGS_WAVE, h = lane >> 5;
    // position in the lane's group of 8 for the transposed plane stores
    const int i8 = lane & 7;
    const bool b1 = (lane & 2) != 0;
    const uint32_t psel = (lane & 1) ? 0x03020706u : 0x05040100u;
    const int64_t groups = (A.n + 32 * SNT - 1) / (32 * SNT);
    const int64_t stride = (int64_t)gridDim.x * 4;
    float lsum = 0.0f;
    for (int64_t grp = (int64_t)blockIdx.x * 4 + wave; grp < groups; grp += stride) {
        int off = 0;
        asm volatile("" : "+s"(off));     // fragments are re-read from LDS every group
        const int ln = lane + off;
        int64_t gi[SNT];
        bool valid[SNT];
        bf16x8 x[SNT][1];
#pragma unroll
        for (int t = 0; t < SNT; ++t) {
            gi[t] = (grp * SNT + t) * 32 + (lane & 31);
            valid[t] = gi[t] < A.n;
            float p[3] = {0.0f, 0.0f, 0.0f};
            if (valid[t]) {
                p[0] = A.mean[3 * gi[t] + 0];
                p[1] = A.mean[3 * gi[t] + 1];
                p[2] = A.mean[3 * gi[t] + 2];
            }
            __bf16 s[3][3];
#pragma unroll
            for (int c = 0; c < 3; ++c) legs_split3(p[c], s[c][0], s[c][1], s[c][2]);
            // lower half: x_hi y_hi z_hi x_mid y_mid z_mid x_lo y_lo; upper: z_lo 1 1 1 0...
            bf16x8 v;
            if (h == 0) {
                v[0] = s[0][0]; v[1] = s[1][0]; v[2] = s[2][0];
                v[3] = s[0][1]; v[4] = s[1][1]; v[5] = s[2][1];
                v[6] = s[0][2]; v[7] = s[1][2];
            } else {
                v[0] = s[2][2]; v[1] = (__bf16)1.0f; v[2] = (__bf16)1.0f; v[3] = (__bf16)1.0f;
                v[4] = v[5] = v[6] = v[7] = (__bf16)0.0f;
            }
            x[t][0] = v;
            // layer-1 input plane for the weight gradient: rows 0..8 the split
            // coordinates (part-major), row 9 ones (zero for padding
            // Gaussians), rows 10..15 zero; lane half h holds rows 8 h .. 8 h + 7
            if (h == 1) {
                v[1] = valid[t] ? (__bf16)1.0f : (__bf16)0.0f;
                v[2] = v[3] = (__bf16)0.0f;
            }
            store_rows8(A.X, 16, gi[t] - i8, v, [h](int i) { return 8 * h + i; }, i8, b1, psel);
        }
        // forward
        bf16x8 h1[SNT][SK], h2[SNT][SK], h3[SNT][SK];
#pragma unroll
        for (int mb = 0; mb < SB; ++mb) {
            f32x16 z[SNT];
            layer_block<1>(L.w1, nullptr, mb, ln, x, z);
#pragma unroll
            for (int t = 0; t < SNT; ++t) {
                h1[t][2 * mb] = relu_bf16x8(z[t], 0);
                h1[t][2 * mb + 1] = relu_bf16x8(z[t], 8);
            }
        }
#pragma unroll
        for (int mb = 0; mb < SB; ++mb) {
            f32x16 z[SNT];
            layer_block<SK>(L.w2, L.bb2, mb, ln, h1, z);
#pragma unroll
            for (int t = 0; t < SNT; ++t) {
                h2[t][2 * mb] = relu_bf16x8(z[t], 0);
                h2[t][2 * mb + 1] = relu_bf16x8(z[t], 8);
            }
        }
#pragma unroll
        for (int mb = 0; mb < SB; ++mb) {
            f32x16 z[SNT];
            layer_block<SK>(L.w3, L.bb3, mb, ln, h2, z);
#pragma unroll
            for (int t = 0; t < SNT; ++t) {
                h3[t][2 * mb] = relu_bf16x8(z[t], 0);
                h3[t][2 * mb + 1] = relu_bf16x8(z[t], 8);
            }
        }
        f32x16 s4[SNT];
        layer_block<SK>(L.w4, L.bb4, 0, ln, h3, s4);
        // hidden activations to the workspace (zero for padding Gaussians)
#pragma unroll
        for (int t = 0; t < SNT; ++t) {
#pragma unroll
            for (int ks = 0; ks < SK; ++ks) {
                const auto unit = [ks, h](int i) { return legs_khid(ks, h, i); };
                const bf16x8 z8 = {};
                store_rows8(A.H1, SH, gi[t] - i8, valid[t] ? h1[t][ks] : z8, unit, i8, b1, psel);
                store_rows8(A.H2, SH, gi[t] - i8, valid[t] ? h2[t][ks] : z8, unit, i8, b1, psel);
                store_rows8(A.H3, SH, gi[t] - i8, valid[t] ? h3[t][ks] : z8, unit, i8, b1, psel);
            }
        }
        // loss and dz4: outputs 4 h + r in registers r = 0..3
        f32x16 dz4[SNT];
#pragma unroll
        for (int t = 0; t < SNT; ++t) {
            dz4[t] = (f32x16){};
            float sg[4] = {0.0f, 0.0f, 0.0f, 0.0f}, u = 0.0f;
            if (valid[t]) {
                const float *row = A.ch + gi[t] * A.C;
#pragma unroll
                for (int r = 0; r < 4; ++r) sg[r] = row[A.sem + 4 * h + r];
                u = row[A.uch];
            }
            float diff[4], ss = 0.0f;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                diff[r] = s4[t][r] - sg[r];
                ss = fmaf(diff[r], diff[r], ss);
            }
            ss += __shfl_xor(ss, 32, LEGS_WAVE);
            const float nrm = sqrtf(ss);
            const float wgt = fmaxf(u, A.w_s);
            if (!valid[t] || !(nrm > 0.0f)) continue;
            if (h == 0) lsum += nrm * (1.0f + wgt) * A.inv_n;
            const float inv = A.inv_n / nrm;
            float *drow = A.d_ch + gi[t] * A.C + A.sem + 4 * h;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                dz4[t][r] = diff[r] * inv;
                drow[r] += -wgt * diff[r] * inv;
            }
        }
        // backward through the layers: dz_l split into hi and lo bf16 parts,
        // which are also what the planes keep (hi plane, then lo plane). dz is
        // exactly zero for padding Gaussians (dz4 is, and every lower dz is a
        // product with it), so the planes hold zeros there.
        // dh3 = W4^T dz4 (one k-step: outputs 0..7 in slots 0..3 of both halves)
        bf16x8 bh[SNT][SK], bl[SNT][SK];
#pragma unroll
        for (int t = 0; t < SNT; ++t) {
            split_bf16x8(dz4[t], 0, bh[t][0], bl[t][0]);
            const auto out = [h](int i) { return legs_khid(0, h, i); };   // outputs 4 h + i for i < 4
            store_rows8(A.D4, LEGS_SMOOTH_OUT, gi[t] - i8, bh[t][0], out, i8, b1, psel);
            store_rows8(A.D4 + LEGS_SMOOTH_OUT * A.Gp, LEGS_SMOOTH_OUT, gi[t] - i8, bl[t][0], out, i8, b1, psel);
        }
        f32x16 dz[SNT][SB];
#pragma unroll
        for (int mb = 0; mb < SB; ++mb) {
            const bf16x8 a = L.t4[mb * 64 + ln];
#pragma unroll
            for (int t = 0; t < SNT; ++t)
                dz[t][mb] = legs_mfma(a, bl[t][0], legs_mfma(a, bh[t][0], (f32x16){}));
        }
        // ReLU gates from the stored activations (positive exactly where z > 0)
        auto gate = [&](const bf16x8 (&hf)[SNT][SK]) {
#pragma unroll
            for (int t = 0; t < SNT; ++t)
#pragma unroll
                for (int mb = 0; mb < SB; ++mb)
#pragma unroll
                    for (int r = 0; r < 16; ++r)
                        if (!((float)hf[t][2 * mb + (r >> 3)][r & 7] > 0.0f)) dz[t][mb][r] = 0.0f;
        };
        auto back = [&](const bf16x8 *__restrict__ T, __bf16 *plane) {
#pragma unroll
            for (int t = 0; t < SNT; ++t)
#pragma unroll
                for (int mb = 0; mb < SB; ++mb) {
                    split_bf16x8(dz[t][mb], 0, bh[t][2 * mb], bl[t][2 * mb]);
                    split_bf16x8(dz[t][mb], 8, bh[t][2 * mb + 1], bl[t][2 * mb + 1]);
#pragma unroll
                    for (int k = 0; k < 2; ++k) {   // rows legs_khid(2 mb + k, h, .)
                        const int ks = 2 * mb + k;
                        const auto row = [ks, h](int i) { return legs_khid(ks, h, i); };
                        store_rows8(plane, SH, gi[t] - i8, bh[t][ks], row, i8, b1, psel);
                        store_rows8(plane + SH * A.Gp, SH, gi[t] - i8, bl[t][ks], row, i8, b1, psel);
                    }
                }
            if (!T) return;
#pragma unroll
            for (int mb = 0; mb < SB; ++mb) {
                f32x16 acc[SNT];
#pragma unroll
                for (int t = 0; t < SNT; ++t) acc[t] = (f32x16){};
#pragma unroll
                for (int ks = 0; ks < SK; ++ks) {
                    const bf16x8 a = T[(mb * SK + ks) * 64 + ln];
#pragma unroll
                    for (int t = 0; t < SNT; ++t) acc[t] = legs_mfma(a, bl[t][ks], legs_mfma(a, bh[t][ks], acc[t]));
                }
#pragma unroll
                for (int t = 0; t < SNT; ++t) dz[t][mb] = acc[t];
            }
        };
        gate(h3);
        back(L.t3, A.D3);     // dz3 stored; dh2 = W3^T dz3
        gate(h2);
        back(L.t2, A.D2);     // dz2 stored; dh1 = W2^T dz2
        gate(h1);
        back(nullptr, A.D1);  // dz1 stored
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) lsum += __shfl_xor(lsum, o, LEGS_WAVE);
    if (lane == 0 && lsum != 0.0f) atomicAdd(A.loss, lsum);
}

// dW[m][k] += sum_g (Dhi + Dlo)[m][g] B[k][g] over the Gaussians of this
// workgroup's chunk, db[m] += sum_g (Dhi + Dlo)[m][g]. Layer (blockIdx.y):
// 0: D1 x X (rows 0..8 = split coordinates, row 9 = ones) -> W1 [128][3], b1
// 1: D2 x H1 -> W2, b2;  2: D3 x H2 -> W3, b3;  3: D4 (8 rows) x H3 -> W4, b4.
constexpr int WG_CHUNK_G = 4096;

__global__ void __launch_bounds__(256)
k_smooth_wgrad(SmoothArgs A, float *__restrict__ grad)
{
    const int layer = blockIdx.y;
    const int lane = __lane_id(), wave = threadIdx.x / LEGS_WAVE, h = lane >> 5;
    const __bf16 *Dh = layer == 0 ? A.D1 : layer == 1 ? A.D2 : layer == 2 ? A.D3 : A.D4;
    const __bf16 *Bp = layer == 0 ? A.X : layer == 1 ? A.H1 : layer == 2 ? A.H2 : A.H3;
    const int M = layer == 3 ? LEGS_SMOOTH_OUT : SH;          // rows of D
    const int Kb = layer == 0 ? 16 : SH;                      // rows of B
    const int MB = (M + 31) / 32, NB = (Kb + 31) / 32;
    const __bf16 *Dl = Dh + (int64_t)M * A.Gp;                 // lo parts after the hi plane
    // wave w owns the 32 rows of block w of D against every block of B, so
    // each fragment of D is loaded once and each of B once per wave
    if (wave >= MB) return;
    const int mb = wave, m = 32 * mb + (lane & 31);
    const int64_t g0 = (int64_t)blockIdx.x * WG_CHUNK_G;
    const int64_t g1 = min(g0 + (int64_t)WG_CHUNK_G, A.Gp);
    const bool mrow = m < M;
    bool krow[4];
#pragma unroll
    for (int nb = 0; nb < 4; ++nb) krow[nb] = nb < NB && 32 * nb + (lane & 31) < Kb;
    f32x16 acc[4] = {};
    float dbs = 0.0f;
#pragma unroll 2
    for (int64_t g = g0; g < g1; g += 16) {
        // this lane's operands: Gaussians g + 8 h .. + 7 (16-byte fragments)
        const int64_t gl = g + 8 * h;
        bf16x8 ah = {}, al = {}, b[4];
        if (mrow) {                 // dz as hi + lo bf16 parts (16 significant bits)
            ah = *reinterpret_cast<const bf16x8 *>(Dh + frag_at(gl, M, m));
            al = *reinterpret_cast<const bf16x8 *>(Dl + frag_at(gl, M, m));
        }
#pragma unroll
        for (int nb = 0; nb < 4; ++nb)
            b[nb] = krow[nb] ? *reinterpret_cast<const bf16x8 *>(Bp + frag_at(gl, Kb, 32 * nb + (lane & 31)))
                             : (bf16x8){};
#pragma unroll
        for (int nb = 0; nb < 4; ++nb)
            if (nb < NB) acc[nb] = legs_mfma(al, b[nb], legs_mfma(ah, b[nb], acc[nb]));
#pragma unroll
        for (int e = 0; e < 8; ++e) dbs += (float)ah[e] + (float)al[e];
    }
    if (layer != 0) {                                           // bias gradient of rows m
        dbs += __shfl_xor(dbs, 32, LEGS_WAVE);
        float *db = grad + (layer == 1 ? LEGS_SMOOTH_OFF_B2 : layer == 2 ? LEGS_SMOOTH_OFF_B3 : LEGS_SMOOTH_OFF_B4);
        if (h == 0 && mrow && dbs != 0.0f) atomicAdd(db + m, dbs);
    }
#pragma unroll
    for (int nb = 0; nb < 4; ++nb) {
        if (nb >= NB) continue;
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const int row = 32 * mb + legs_drow(r, h);
            const int col = 32 * nb + (lane & 31);
            const float v = acc[nb][r];
            if (row >= M || col >= Kb || v == 0.0f) continue;
            if (layer == 0) {
                if (col < 9) atomicAdd(grad + LEGS_SMOOTH_OFF_W1 + row * 3 + col % 3, v);
                else if (col == 9) atomicAdd(grad + LEGS_SMOOTH_OFF_B1 + row, v);
            } else {
                const int off = layer == 1 ? LEGS_SMOOTH_OFF_W2 : layer == 2 ? LEGS_SMOOTH_OFF_W3 : LEGS_SMOOTH_OFF_W4;
                atomicAdd(grad + off + row * SH + col, v);
            }
        }
    }
}

struct SmoothLayout {
    int64_t Gp, X, H1, H2, H3, D1, D2, D3, D4, total;
};

SmoothLayout smooth_layout(int64_t n)
{
    SmoothLayout L;
    L.Gp = (n + 63) / 64 * 64;
    const int64_t plane = L.Gp * 2;       // one bf16 row
    int64_t o = 0;
    L.X = o;  o += 16 * plane;
    L.H1 = o; o += SH * plane;
    L.H2 = o; o += SH * plane;
    L.H3 = o; o += SH * plane;
    L.D1 = o; o += 2 * SH * plane;            // hi and lo bf16 planes
    L.D2 = o; o += 2 * SH * plane;
    L.D3 = o; o += 2 * SH * plane;
    L.D4 = o; o += 2 * LEGS_SMOOTH_OUT * plane;
    L.total = o;
    return L;
}

} // namespace

int64_t legs_smooth_workspace_bytes(int64_t n) { return smooth_layout(n).total; }

int32_t legs_launch_smooth(legs_ctx *ctx, const float *mean, const float *channels, int32_t C, int32_t sem,
                           int32_t uch, int64_t n, const float *params, float w_s, float lambda_smo,
                           void *workspace, float *grad, float *d_channels, float *loss, hipStream_t s)
{
    if (n == 0) return LEGS_OK;
    const SmoothLayout Lw = smooth_layout(n);
    char *ws = static_cast<char *>(workspace);
    SmoothArgs A;
    A.mean = mean;
    A.ch = channels;
    A.C = C;
    A.sem = sem;
    A.uch = uch;
    A.n = n;
    A.Gp = Lw.Gp;
    A.params = params;
    A.w_s = w_s;
    A.inv_n = lambda_smo / (float)n;
    A.d_ch = d_channels;
    A.loss = loss;
    A.X = reinterpret_cast<__bf16 *>(ws + Lw.X);
    A.H1 = reinterpret_cast<__bf16 *>(ws + Lw.H1);
    A.H2 = reinterpret_cast<__bf16 *>(ws + Lw.H2);
    A.H3 = reinterpret_cast<__bf16 *>(ws + Lw.H3);
    A.D1 = reinterpret_cast<__bf16 *>(ws + Lw.D1);
    A.D2 = reinterpret_cast<__bf16 *>(ws + Lw.D2);
    A.D3 = reinterpret_cast<__bf16 *>(ws + Lw.D3);
    A.D4 = reinterpret_cast<__bf16 *>(ws + Lw.D4);
    int64_t blocks = (Lw.Gp + 32 * SNT * 4 - 1) / (32 * SNT * 4);
    if (blocks > ctx->num_cus) blocks = ctx->num_cus;
    hipLaunchKernelGGL(k_smooth_fwd_bwd, dim3((unsigned)blocks), dim3(256), 0, s, A);
    const dim3 gw((unsigned)((Lw.Gp + WG_CHUNK_G - 1) / WG_CHUNK_G), 4);
    hipLaunchKernelGGL(k_smooth_wgrad, gw, dim3(256), 0, s, A, grad);
    LEGS_CHECK_LAUNCH(ctx);
    return LEGS_OK;
}
