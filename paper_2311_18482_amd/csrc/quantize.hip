// Quantisation of hybrid language features into the discrete feature space
// (Sec. 3.3, Eqs. 4-7, and the supplementary load-balancing loss), gfx950.
//
// Features F [K][d] are IEEE half (CLIP dimensions [0, d_clip), DINO the
// rest), the feature space S [N][d] float32, rounded to half for every use
// (dot products and norms), so the cosines are those of the half-precision
// vectors; products are exact in float32 and accumulate in float32 on
// v_mfma_f32_32x32x16_f16.
//
//  k_quant_prep      S once per call into the LDS image of each 128-dimension
//                    chunk (A-operand fragments, code rows x dimensions), and
//                    1 / |S_j| of both parts.
//  k_quant_pass      one workgroup of 4 waves per CU, 32-feature tiles (two
//                    per wave at N = 32, sharing every codebook fragment read
//                    from LDS): the codebook image of each chunk and every
//                    wave's feature fragments stream straight into one of two
//                    LDS buffers (global_load_lds, no registers) while the
//                    other feeds the MFMAs;
//                    the 32 x N dot products of each part stay in registers
//                    (transposed: codes x features), the feature norms are
//                    summed from the same B fragments. Then per feature the
//                    distance D_j = cos^C_j + lambda cos^D_j, its argmax (first
//                    maximum) and its softmax. ASSIGN: index, histogram of the
//                    indices, sum of the softmax (the mean selection
//                    probability), cosine loss. GRAD: dL_q/dD_j with the final
//                    histogram, written (scaled by 2^10 K) as half weights
//                    W^C, W^D (N x Kp, in the weight gradient's MFMA operand
//                    order: one 16-byte fragment per lane after an 8 x 8 lane
//                    transpose) with 1 / |F_i| of both parts, and the column
//                    sums sum_i dL/dD_ij cos_ij per part. Column sums over the 32
//                    features of a wave go through a transpose reduction
//                    (five lane-bit stages) before the LDS and global atomics.
//  k_quant_wgrad     sum_i W_ij F_ic / |F_i| for every code j and dimension c:
//                    FP16 MFMA with the features as the contraction (the
//                    weight fragments 1 KB contiguous per wave), the unit
//                    feature rows staged through LDS transposed
//                    (dimension-major) in steps of 64, split over feature
//                    ranges (x) and 128-dimension chunks (y), float atomics
//                    into the gradient.
//  k_quant_finish    the gradient's second term, the losses, r and p.
#include "legs_internal.h"
#include "legs_decode_internal.h"
#include "wave_reduce.h"
#include "lane_transpose.h"

namespace {

typedef legs_f32x16 f32x16;
typedef __attribute__((ext_vector_type(8))) _Float16 f16x8;

constexpr int QCH = 128;           // dimensions per chunk
// The gradient's half weights are 2^10 K dL/dD (at most 2^10 (lambda_cos +
// lambda_lb) in magnitude): the scale keeps the small terms of the
// load-balancing loss out of the half-precision subnormal range.
constexpr float WSCALE = 1024.0f;
constexpr int QTHREADS = 256;      // 4 waves, one per SIMD
constexpr int QGROUP = 256;        // feature padding of the half weights W^C, W^D
// 32-feature tiles per wave (every codebook fragment read from LDS feeds QNT
// MFMAs): two at N = 32, one from N = 64 (the LDS holds two chunks of the
// codebook image and of every wave's feature fragments)
template <int KB> constexpr int qnt() { return KB == 1 ? 2 : 1; }

// s_waitcnt vmcnt(N) (expcnt and lgkmcnt not waited for).
template <int N>
__device__ __forceinline__ void vm_wait()
{
    static_assert(N >= 0 && N < 64, "vmcnt range");
    __builtin_amdgcn_s_waitcnt((N & 15) | (7 << 4) | (15 << 8) | ((N >> 4) << 14));
}

// Workgroup barrier for the double-buffered chunks: this wave's LDS reads
// are complete (lgkmcnt 0) and the compiler keeps memory operations on their
// side of it, but the next chunk's loads in flight are not waited for (the
// fence of a __syncthreads() would wait for every load). Each wave waits for
// its own loads of a buffer (vm_wait) before the barrier that precedes the
// buffer's reads.
__device__ __forceinline__ void ring_barrier()
{
    __builtin_amdgcn_s_waitcnt(0xC07F);       // lgkmcnt(0); vmcnt, expcnt not waited for
    asm volatile("" ::: "memory");
    __builtin_amdgcn_s_barrier();
    asm volatile("" ::: "memory");
}

// 16 bytes per lane from global memory straight into LDS (gfx950
// global_load_lds_dwordx4): lane l's bytes land at lds + 16 l; lds is the
// same for the whole wave. Completion: s_waitcnt vmcnt(0) of this wave, then
// a barrier for the other waves' reads.
__device__ __forceinline__ void global_to_lds(const void *src, void *lds)
{
    __builtin_amdgcn_global_load_lds(src, (__attribute__((address_space(3))) void *)lds, 16, 0, 0);
}

// Two floats as a word of halves (round to nearest), a in the low half.
__device__ __forceinline__ uint32_t pack_half2(float a, float b)
{
    typedef __attribute__((ext_vector_type(2))) _Float16 f16x2;
    const f16x2 v = {(_Float16)a, (_Float16)b};
    return __builtin_bit_cast(uint32_t, v);
}

__device__ __forceinline__ f32x16 mfma16(f16x8 a, f16x8 b, f32x16 c)
{
    return __builtin_amdgcn_mfma_f32_32x32x16_f16(a, b, c, 0, 0, 0);
}

// Image of chunk ch: fragment (mb, ks, lane) holds code 32 mb + lane % 32,
// dimensions 128 ch + 16 ks + 8 (lane / 32) + [0, 8).
template <int KB>
__global__ void __launch_bounds__(256)
k_quant_prep(const float *__restrict__ S, int d, int dC, f16x8 *__restrict__ img, float *__restrict__ invS)
{
    constexpr int NF = KB * 8 * 64;
    const int nch = d / QCH;
    for (int q = blockIdx.x * 256 + threadIdx.x; q < nch * NF; q += gridDim.x * 256) {
        const int ch = q / NF, f = q % NF;
        const int l = f & 63, ks = (f >> 6) & 7, mb = f >> 9;
        const float *row = S + (int64_t)(32 * mb + (l & 31)) * d + ch * QCH + 16 * ks + 8 * (l >> 5);
        f16x8 v;
#pragma unroll
        for (int e = 0; e < 8; ++e) v[e] = (_Float16)row[e];
        img[q] = v;
    }
    // 1 / |S_j| per part (0 for a zero part): one wave per code
    constexpr int N = 32 * KB;
    const int wave = (blockIdx.x * 256 + threadIdx.x) / LEGS_WAVE, lane = __lane_id();
    for (int j = wave; j < N; j += gridDim.x * 4) {
        float sc = 0.0f, sd = 0.0f;
        for (int c = lane; c < d; c += LEGS_WAVE) {
            const float v = (float)(_Float16)S[(int64_t)j * d + c];
            if (c < dC) sc = fmaf(v, v, sc);
            else sd = fmaf(v, v, sd);
        }
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
            sc += __shfl_xor(sc, o, LEGS_WAVE);
            sd += __shfl_xor(sd, o, LEGS_WAVE);
        }
        if (lane == 0) {
            invS[j] = sc > 0.0f ? 1.0f / sqrtf(sc) : 0.0f;
            invS[N + j] = sd > 0.0f ? 1.0f / sqrtf(sd) : 0.0f;
        }
    }
}

struct QuantArgs {
    const _Float16 *F;
    int64_t K, Kp;
    int d, dC;
    const f16x8 *img;
    const float *invS;          // [2][N]
    float lam_d, lam_cos, lam_lb;
    int32_t *index;             // [K]
    uint32_t *counts;           // [N]
    float *psum;                // [N] sum of softmax over features
    float *lsum;                // [1] cosine-loss sum
    _Float16 *Wc, *Wd;          // N x Kp half weights 2^10 K dL/dD (lambda_dino K dL/dD for DINO) in
                                // MFMA operand order (legs_lt::frag_at, codes as rows, features as columns)
    float *invF;                // [2][Kp] 1 / |F_i| of both parts (0 past K)
    float *col;                 // [2][N]
};

// Sums over the 32 features of each lane half of V values per lane, then LDS
// atomics: value v of a lane is code code_of(v) (lane half fixed).
template <int V, typename CodeOf>
__device__ __forceinline__ void half_wave_sums(float (&v)[V], float *dst, CodeOf code_of)
{
    const int lane = __lane_id();
    legs_tr::run<4, V, V>(v, lane);
    constexpr int R = legs_tr::final_k(V, 5);
#pragma unroll
    for (int k = 0; k < R; ++k) {
        const int ix = legs_tr::src_index<4, V>(k, lane);
        if (ix >= 0 && v[k] != 0.0f) atomicAdd(dst + code_of(ix), v[k]);
    }
}

template <int KB, bool GRAD>
__global__ void __launch_bounds__(QTHREADS)
k_quant_pass(QuantArgs A)
{
    constexpr int N = 32 * KB, NF = KB * 8 * 64, PER = NF / QTHREADS;
    constexpr int QNT = qnt<KB>(), ROUND = QTHREADS / LEGS_WAVE * 32 * QNT;   // features per round
    static_assert(NF % QTHREADS == 0, "fragments per thread");
    // two LDS buffers, each the codebook image of a chunk and every wave's
    // feature fragments; distinct arrays, so that the compiler can tell the
    // reads of one buffer from the loads still landing in the other
    constexpr int FEF = QTHREADS / LEGS_WAVE * QNT * 8 * LEGS_WAVE;
    __shared__ f16x8 frag0[NF], frag1[NF];
    __shared__ f16x8 feat0[FEF], feat1[FEF];
    __shared__ float s_inv[2][N];
    __shared__ float s_ab[2 * N];         // psum | col^C then col^D
    __shared__ uint32_t s_cnt[N];
    __shared__ float s_r[N];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, h = lane >> 5;
    // position in the lane's group of 8 for the transposed weight stores
    const int i8 = lane & 7;
    const bool b1 = (lane & 2) != 0;
    const uint32_t psel = (lane & 1) ? 0x03020706u : 0x05040100u;
    const float invK = 1.0f / (float)A.K;
    for (int j = tid; j < N; j += QTHREADS) {
        s_inv[0][j] = A.invS[j];
        s_inv[1][j] = A.invS[N + j];
        s_ab[j] = 0.0f;
        s_ab[N + j] = 0.0f;
        s_cnt[j] = 0u;
        if (GRAD) s_r[j] = (float)A.counts[j] * invK;
    }
    float lcos = 0.0f;
    const int nch = A.d / QCH, nchC = A.dC / QCH;
    // the gradient pass writes every column of W^C, W^D below Kp (zeros past
    // K: the weight-gradient kernel reads whole 16-byte fragments)
    const int64_t groups = ((GRAD ? A.Kp : A.K) + ROUND - 1) / ROUND;
    for (int64_t g = blockIdx.x; g < groups; g += gridDim.x) {
        int64_t ii[QNT];
        bool valid[QNT];
        const _Float16 *frow[QNT];
#pragma unroll
        for (int t = 0; t < QNT; ++t) {
            ii[t] = g * ROUND + (wave * QNT + t) * 32 + (lane & 31);
            valid[t] = ii[t] < A.K;
            frow[t] = A.F + (valid[t] ? ii[t] : 0) * (int64_t)A.d + 8 * h;
        }
        f32x16 ac[QNT][KB], ad[QNT][KB];
#pragma unroll
        for (int t = 0; t < QNT; ++t)
#pragma unroll
            for (int mb = 0; mb < KB; ++mb) { ac[t][mb] = (f32x16){}; ad[t][mb] = (f32x16){}; }
        float ssc[QNT] = {}, ssd[QNT] = {};
        // the fragments of chunk ch into LDS buffer ch & 1: the codebook image
        // in 1 KB pieces (wave w copies pieces w, w + 4, ...) and this wave's
        // feature fragments (lane l of k-step ks: feature l % 32, dimensions
        // 128 ch + 16 ks + 8 (l / 32) .. + 7; padding features read row 0 and
        // are zeroed when read back)
        auto issue = [&](int ch, f16x8 *fg, f16x8 *fe) {
            for (int p = wave; p < NF / LEGS_WAVE; p += QTHREADS / LEGS_WAVE)
                global_to_lds(A.img + (int64_t)ch * NF + p * LEGS_WAVE + lane, fg + p * LEGS_WAVE);
#pragma unroll
            for (int t = 0; t < QNT; ++t)
#pragma unroll
                for (int ks = 0; ks < 8; ++ks)
                    global_to_lds(frow[t] + ch * QCH + 16 * ks, fe + ((wave * QNT + t) * 8 + ks) * LEGS_WAVE);
        };
        auto chunk = [&](const f16x8 *fr, const f16x8 *fe, f32x16 (&acc)[QNT][KB], float (&ss)[QNT]) {
            const f16x8(*fb)[8 * LEGS_WAVE] = reinterpret_cast<const f16x8(*)[8 * LEGS_WAVE]>(fe + wave * QNT * 8 * LEGS_WAVE);
            // software pipeline: the fragments of k-step ks + 1 are read while
            // the MFMAs of ks run; a scheduling barrier per k-step keeps the
            // compiler from hoisting every read of the chunk (registers)
            f16x8 a[KB], b[QNT];
#pragma unroll
            for (int mb = 0; mb < KB; ++mb) a[mb] = fr[mb * 8 * 64 + lane];
#pragma unroll
            for (int t = 0; t < QNT; ++t) b[t] = valid[t] ? fb[t][lane] : (f16x8){};
#pragma unroll
            for (int ks = 0; ks < 8; ++ks) {
                f16x8 an[KB], bn[QNT];
                if (ks + 1 < 8) {
#pragma unroll
                    for (int mb = 0; mb < KB; ++mb) an[mb] = fr[(mb * 8 + ks + 1) * 64 + lane];
#pragma unroll
                    for (int t = 0; t < QNT; ++t) bn[t] = valid[t] ? fb[t][(ks + 1) * 64 + lane] : (f16x8){};
                }
#pragma unroll
                for (int mb = 0; mb < KB; ++mb)
#pragma unroll
                    for (int t = 0; t < QNT; ++t) acc[t][mb] = mfma16(a[mb], b[t], acc[t][mb]);
#pragma unroll
                for (int t = 0; t < QNT; ++t)
#pragma unroll
                    for (int e = 0; e < 8; ++e) ss[t] = fmaf((float)b[t][e], (float)b[t][e], ss[t]);
                __builtin_amdgcn_sched_barrier(0);
                if (ks + 1 < 8) {
#pragma unroll
                    for (int mb = 0; mb < KB; ++mb) a[mb] = an[mb];
#pragma unroll
                    for (int t = 0; t < QNT; ++t) b[t] = bn[t];
                }
            }
        };
        // chunk ch + 1 loads while chunk ch computes: the wait for this wave's
        // loads and the barrier before each chunk make its fragments visible
        // and free the other buffer (read by chunk ch - 1) for the next loads.
        // The loop takes two chunks per iteration, even ones in buffer 0 and
        // odd ones in buffer 1, so that every read and every load has its
        // buffer fixed at compile time. In the gradient pass the last chunk
        // reloads itself into the other buffer: there a conditional load made
        // the compiler wait before the reads (and spill); the assign pass
        // loads only what it reads. One set of accumulators serves the part
        // being summed: at chunk nchC the CLIP sums move to ac.
        f32x16 acc[QNT][KB];
        float ss[QNT];
#pragma unroll
        for (int t = 0; t < QNT; ++t) {
            ss[t] = 0.0f;
#pragma unroll
            for (int mb = 0; mb < KB; ++mb) acc[t][mb] = (f32x16){};
        }
        auto part_switch = [&](int ch) {
            if (ch != nchC) return;
#pragma unroll
            for (int t = 0; t < QNT; ++t) {
                ssc[t] = ss[t];
                ss[t] = 0.0f;
#pragma unroll
                for (int mb = 0; mb < KB; ++mb) {
                    ac[t][mb] = acc[t][mb];
                    acc[t][mb] = (f32x16){};
                }
            }
        };
        vm_wait<0>();                                 // the previous round's stores
        __syncthreads();                              // the previous round's readers are done
        issue(0, frag0, feat0);
#pragma unroll 1
        for (int ch = 0; ch < nch; ch += 2) {
            part_switch(ch);
            vm_wait<0>();
            ring_barrier();
            if (GRAD || ch + 1 < nch) issue(ch + 1 < nch ? ch + 1 : ch, frag1, feat1);
            chunk(frag0, feat0, acc, ss);
            if (ch + 1 < nch) {
                part_switch(ch + 1);
                vm_wait<0>();
                ring_barrier();
                if (GRAD || ch + 2 < nch) issue(ch + 2 < nch ? ch + 2 : ch + 1, frag0, feat0);
                chunk(frag1, feat1, acc, ss);
            }
        }
        if (nchC == nch) part_switch(nch);             // no DINO chunks: ad stays zero
#pragma unroll
        for (int t = 0; t < QNT; ++t) {
            ssd[t] = ss[t];
#pragma unroll
            for (int mb = 0; mb < KB; ++mb) ad[t][mb] = acc[t][mb];
        }
#pragma unroll
        for (int t = 0; t < QNT; ++t) {
            const int64_t i = ii[t];
            const bool vt = valid[t];
            const float sc2 = ssc[t] + __shfl_xor(ssc[t], 32, LEGS_WAVE);
            const float sd2 = ssd[t] + __shfl_xor(ssd[t], 32, LEGS_WAVE);
            const float ifc = sc2 > 0.0f ? 1.0f / sqrtf(sc2) : 0.0f;
            const float ifd = sd2 > 0.0f ? 1.0f / sqrtf(sd2) : 0.0f;
            if (GRAD && h == 0) {
                A.invF[i] = vt ? ifc : 0.0f;
                A.invF[A.Kp + i] = vt ? ifd : 0.0f;
            }
            // cosines of both parts in place, distance, argmax (first maximum)
            float best = -INFINITY;
            int bidx = 0x7fffffff;
#pragma unroll
            for (int mb = 0; mb < KB; ++mb)
#pragma unroll
                for (int r = 0; r < 16; ++r) {
                    const int j = 32 * mb + legs_drow(r, h);
                    ac[t][mb][r] = ac[t][mb][r] * ifc * s_inv[0][j];
                    ad[t][mb][r] = ad[t][mb][r] * ifd * s_inv[1][j];
                    const float Dv = ac[t][mb][r] + A.lam_d * ad[t][mb][r];
                    if (Dv > best) { best = Dv; bidx = j; }
                }
            {
                const float ob = __shfl_xor(best, 32, LEGS_WAVE);
                const int oi = __shfl_xor(bidx, 32, LEGS_WAVE);
                if (ob > best || (ob == best && oi < bidx)) { best = ob; bidx = oi; }
                if (bidx >= N) bidx = 0;                  // no comparison held (NaN input)
            }
            float sum = 0.0f;
#pragma unroll
            for (int mb = 0; mb < KB; ++mb)
#pragma unroll
                for (int r = 0; r < 16; ++r) sum += __expf(ac[t][mb][r] + A.lam_d * ad[t][mb][r] - best);
            sum += __shfl_xor(sum, 32, LEGS_WAVE);
            const float isum = 1.0f / sum;
            if constexpr (!GRAD) {
                float sv[KB * 16];
#pragma unroll
                for (int mb = 0; mb < KB; ++mb)
#pragma unroll
                    for (int r = 0; r < 16; ++r) {
                        const float c = ac[t][mb][r], e = ad[t][mb][r];
                        sv[mb * 16 + r] = vt ? __expf(c + A.lam_d * e - best) * isum : 0.0f;
                    }
                // the cosine loss of the assigned code: (1 - cos^C) + lambda (1 - cos^D)
                // = (1 + lambda) - D at the maximum, which is best
                if (vt && h == 0) lcos += (1.0f + A.lam_d) - best;
                half_wave_sums<KB * 16>(sv, s_ab, [h](int v) { return 32 * (v >> 4) + legs_drow(v & 15, h); });
                if (vt && h == 0) {
                    A.index[i] = bidx;
                    atomicAdd(&s_cnt[bidx], 1u);
                }
            } else {
                const int m = vt ? A.index[i] : -1;
                float rs = 0.0f;
#pragma unroll
                for (int mb = 0; mb < KB; ++mb)
#pragma unroll
                    for (int r = 0; r < 16; ++r)
                        rs += s_r[32 * mb + legs_drow(r, h)] * __expf(ac[t][mb][r] + A.lam_d * ad[t][mb][r] - best);
                rs += __shfl_xor(rs, 32, LEGS_WAVE);
                rs *= isum;
                const float scale = (float)A.K * WSCALE;
                // W^C, W^D in the weight gradient's operand order: the 8 codes
                // r = 8 k .. 8 k + 7 of block mb of this lane's feature,
                // transposed across its group of 8 lanes (8 consecutive
                // features), are one 16-byte fragment per lane
                const int64_t i0 = i - i8;
#pragma unroll
                for (int mb = 0; mb < KB; ++mb)
#pragma unroll
                    for (int k = 0; k < 2; ++k) {
                        uint32_t wc[4], wd[4];
#pragma unroll
                        for (int q = 0; q < 4; ++q) {
                            float gv[2];
#pragma unroll
                            for (int u = 0; u < 2; ++u) {
                                const int r = 8 * k + 2 * q + u;
                                const int j = 32 * mb + legs_drow(r, h);
                                const float c = ac[t][mb][r], e = ad[t][mb][r];
                                const float s = __expf(c + A.lam_d * e - best) * isum;
                                float gj = A.lam_lb * invK * s * (s_r[j] - rs);
                                if (j == m) gj -= A.lam_cos * invK;
                                if (!vt) gj = 0.0f;
                                ac[t][mb][r] = gj * c;         // column-sum terms, in place
                                ad[t][mb][r] = A.lam_d * gj * e;
                                gv[u] = gj;
                            }
                            wc[q] = pack_half2(scale * gv[0], scale * gv[1]);
                            wd[q] = pack_half2(scale * A.lam_d * gv[0], scale * A.lam_d * gv[1]);
                        }
                        legs_lt::oct_transpose(wc, b1, psel);
                        legs_lt::oct_transpose(wd, b1, psel);
                        // lane i8 now holds code 32 mb + drow(8 k + i8, h) of features i0 .. i0 + 7
                        const int row = 32 * mb + 16 * k + 8 * (i8 >> 2) + 4 * h + (i8 & 3);
                        const int64_t off = legs_lt::frag_at(i0, N, row);
                        *reinterpret_cast<uint4 *>(A.Wc + off) = make_uint4(wc[0], wc[1], wc[2], wc[3]);
                        *reinterpret_cast<uint4 *>(A.Wd + off) = make_uint4(wd[0], wd[1], wd[2], wd[3]);
                    }
                auto code = [h](int v) { return 32 * (v >> 4) + legs_drow(v & 15, h); };
                {
                    float v[KB * 16];
#pragma unroll
                    for (int k = 0; k < KB * 16; ++k) v[k] = ac[t][k >> 4][k & 15];
                    half_wave_sums<KB * 16>(v, s_ab, code);
                }
                {
                    float v[KB * 16];
#pragma unroll
                    for (int k = 0; k < KB * 16; ++k) v[k] = ad[t][k >> 4][k & 15];
                    half_wave_sums<KB * 16>(v, s_ab + N, code);
                }
            }
        }
    }
    // cosine-loss partial: one wave sum, one atomic
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) lcos += __shfl_xor(lcos, o, LEGS_WAVE);
    __syncthreads();
    if (!GRAD && lane == 0 && lcos != 0.0f) atomicAdd(A.lsum, lcos);
    for (int j = tid; j < N; j += QTHREADS) {
        if (!GRAD) {
            if (s_ab[j] != 0.0f) atomicAdd(A.psum + j, s_ab[j]);
            if (s_cnt[j]) atomicAdd(A.counts + j, s_cnt[j]);
        } else {
            if (s_ab[j] != 0.0f) atomicAdd(A.col + j, s_ab[j]);
            if (s_ab[N + j] != 0.0f) atomicAdd(A.col + N + j, s_ab[N + j]);
        }
    }
}

// sum_i W_ij F_ic over the features [x0, x1) of this workgroup, for the 128
// dimensions of chunk blockIdx.y; wave w computes code block w % KB and
// 4 / (4 / KB) dimension blocks.
constexpr int WG_FEAT = 64;          // features per LDS step

template <int KB>
__global__ void __launch_bounds__(256)
k_quant_wgrad(const _Float16 *__restrict__ F, int64_t K, int64_t Kp, int d, int dC, int64_t per_block,
              const _Float16 *__restrict__ Wc, const _Float16 *__restrict__ Wd, const float *__restrict__ invF,
              const float *__restrict__ invS, float *__restrict__ grad)
{
    constexpr int N = 32 * KB, WPB = 4 / KB, DB = 4 / WPB;   // waves per code block, dim blocks per wave
    __shared__ f16x8 tile[WG_FEAT / 16][QCH / 32][64];   // B fragments of a step: [k-step][dim block][lane]
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, h = lane >> 5;
    const int i8 = lane & 7;
    const bool b1 = (lane & 2) != 0;
    const uint32_t psel = (lane & 1) ? 0x03020706u : 0x05040100u;
    const int mb = wave % KB, db0 = (wave / KB) * DB;
    const int c0 = blockIdx.y * QCH;
    const bool clip = c0 < dC;
    const _Float16 *W = clip ? Wc : Wd;
    const float *iF = invF + (clip ? 0 : Kp);
    const int64_t x0 = (int64_t)blockIdx.x * per_block;
    const int64_t x1 = min(x0 + per_block, Kp);
    f32x16 acc[DB];
#pragma unroll
    for (int q = 0; q < DB; ++q) acc[q] = (f32x16){};
    // the next step's feature rows, their norms and this wave's weight
    // fragments are loaded into registers while the current step computes
    f16x8 fv[4], wa[WG_FEAT / 16];
    float fsc[4];
    auto load_step = [&](int64_t s0) {
#pragma unroll
        for (int it = 0; it < 4; ++it) {
            const int u = 4 * wave + it;
            const int64_t ii = s0 + 8 * (u >> 1) + i8;
            const int c8 = 64 * (u & 1) + 8 * (lane >> 3);
            fv[it] = ii < K ? *reinterpret_cast<const f16x8 *>(F + ii * d + c0 + c8) : (f16x8){};
            fsc[it] = ii < K ? iF[ii] : 0.0f;               // unit feature rows of this part
        }
#pragma unroll
        for (int ks = 0; ks < WG_FEAT / 16; ++ks) {
            // operand order: the wave's fragments of (code block mb, features
            // s0 + 16 ks ..) are 1 KB contiguous
            const int64_t ia = s0 + 16 * ks + 8 * h;
            wa[ks] = ia < x1 ? *reinterpret_cast<const f16x8 *>(W + legs_lt::frag_at(ia, N, 32 * mb + (lane & 31)))
                             : (f16x8){};
        }
    };
    if (x0 < x1) load_step(x0);
    for (int64_t s0 = x0; s0 < x1; s0 += WG_FEAT) {
        ring_barrier();                                    // the previous step's readers are done
        // stage features [s0, s0 + 64) x dimensions [c0, c0 + 128) as B
        // fragments: 16 units of 8 features x 64 dimensions, four per wave;
        // lane l holds dimensions 8 (l / 8) .. + 7 (of the unit's half) of
        // feature l % 8 (of the unit's block of 8), scales the row to unit
        // length, and the transpose across its group of 8 lanes leaves it
        // dimension 8 (l / 8) + l % 8 of the 8 features: one fragment
#pragma unroll
        for (int it = 0; it < 4; ++it) {
            const int u = 4 * wave + it, fb = u >> 1;
            uint32_t w[4];
#pragma unroll
            for (int q = 0; q < 4; ++q)
                w[q] = pack_half2((float)fv[it][2 * q] * fsc[it], (float)fv[it][2 * q + 1] * fsc[it]);
            legs_lt::oct_transpose(w, b1, psel);
            const int c = 64 * (u & 1) + 8 * (lane >> 3) + i8;   // the dimension this lane now holds
            tile[fb >> 1][c >> 5][(c & 31) + 32 * (fb & 1)] =
                __builtin_bit_cast(f16x8, make_uint4(w[0], w[1], w[2], w[3]));
        }
        f16x8 a[WG_FEAT / 16];
#pragma unroll
        for (int ks = 0; ks < WG_FEAT / 16; ++ks) a[ks] = wa[ks];
        if (s0 + WG_FEAT < x1) load_step(s0 + WG_FEAT);
        ring_barrier();                                    // the staged fragments (LDS only: the
                                                           // loads just issued stay in flight)
#pragma unroll
        for (int ks = 0; ks < WG_FEAT / 16; ++ks)
#pragma unroll
            for (int q = 0; q < DB; ++q) {
                const f16x8 b = tile[ks][db0 + q][lane];     // dimension 32 (db0 + q) + lane % 32
                acc[q] = mfma16(a[ks], b, acc[q]);
            }
    }
    const float invK = 1.0f / ((float)K * WSCALE);
    const float *is = invS + (clip ? 0 : N);
#pragma unroll
    for (int q = 0; q < DB; ++q)
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const int j = 32 * mb + legs_drow(r, h);
            const int c = c0 + 32 * (db0 + q) + (lane & 31);
            const float v = acc[q][r] * invK * is[j];
            if (v != 0.0f) atomicAdd(grad + (int64_t)j * d + c, v);
        }
}

// grad[j][c] -= col^part_j S16_jc / |S16_j^part|^2; losses; r and p.
template <int KB>
__global__ void __launch_bounds__(256)
k_quant_finish(const float *__restrict__ S, int d, int dC, int64_t K, const float *__restrict__ invS,
               const float *__restrict__ col, float *__restrict__ grad, const uint32_t *__restrict__ counts,
               const float *__restrict__ psum, const float *__restrict__ lsum, float lam_cos, float lam_lb,
               float *__restrict__ prob_mean, float *__restrict__ losses)
{
    constexpr int N = 32 * KB;
    if (grad) {
        for (int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x; q < (int64_t)N * d; q += (int64_t)gridDim.x * 256) {
            const int j = (int)(q / d), c = (int)(q % d);
            const int part = c >= dC;
            const float iv = invS[part * N + j];
            grad[q] -= col[part * N + j] * (float)(_Float16)S[q] * iv * iv;
        }
    }
    if (blockIdx.x == 0 && threadIdx.x < LEGS_WAVE) {
        const float invK = 1.0f / (float)K;
        float lb = 0.0f;
        for (int j = threadIdx.x; j < N; j += LEGS_WAVE) {
            const float p = psum[j] * invK;
            if (prob_mean) prob_mean[j] = p;
            lb += (float)counts[j] * invK * p;
        }
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) lb += __shfl_xor(lb, o, LEGS_WAVE);
        if (threadIdx.x == 0 && losses) {
            const float lc = lsum[0] * invK;
            losses[0] = lc;
            losses[1] = lb;
            losses[2] = lam_cos * lc + lam_lb * lb;
        }
    }
}

__global__ void __launch_bounds__(256)
k_quant_zero(uint32_t *__restrict__ a, int64_t na, uint32_t *__restrict__ b, int64_t nb)
{
    for (int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x; q < na + nb; q += (int64_t)gridDim.x * 256) {
        if (q < na) a[q] = 0u;
        else b[q - na] = 0u;
    }
}

struct QuantLayout {
    int64_t img, invS, psum, col, lsum, wc, wd, invF, total, Kp;
};

QuantLayout quant_layout(int64_t K, int32_t N, int32_t d)
{
    QuantLayout L;
    auto up = [](int64_t x) { return (x + 255) & ~(int64_t)255; };
    L.Kp = (K + QGROUP - 1) / QGROUP * QGROUP;
    int64_t o = 0;
    L.img = o;  o = up(o + (int64_t)N * d * 2);
    L.invS = o; o = up(o + 2 * (int64_t)N * 4);
    L.psum = o; o = up(o + (int64_t)N * 4);
    L.col = o;  o = up(o + 2 * (int64_t)N * 4);
    L.lsum = o; o = up(o + 4);
    L.wc = o;   o = up(o + (int64_t)N * L.Kp * 2);
    L.wd = o;   o = up(o + (int64_t)N * L.Kp * 2);
    L.invF = o; o = up(o + 2 * L.Kp * 4);
    L.total = o;
    return L;
}

} // namespace

int64_t legs_quantize_workspace_bytes(int64_t K, int32_t N, int32_t d) { return quant_layout(K, N, d).total; }

int32_t legs_launch_quantize(legs_ctx *ctx, const uint16_t *feat, int64_t K, int32_t d, int32_t dC,
                             const float *S, int32_t N, float lam_d, float lam_cos, float lam_lb,
                             void *workspace, int32_t *index, uint32_t *counts, float *prob_mean,
                             float *losses, float *grad, hipStream_t s)
{
    const QuantLayout Lw = quant_layout(K, N, d);
    char *ws = static_cast<char *>(workspace);
    QuantArgs A;
    A.F = reinterpret_cast<const _Float16 *>(feat);
    A.K = K;
    A.Kp = Lw.Kp;
    A.d = d;
    A.dC = dC;
    A.img = reinterpret_cast<const f16x8 *>(ws + Lw.img);
    A.invS = reinterpret_cast<const float *>(ws + Lw.invS);
    A.lam_d = lam_d;
    A.lam_cos = lam_cos;
    A.lam_lb = lam_lb;
    A.index = index;
    A.counts = counts;
    A.psum = reinterpret_cast<float *>(ws + Lw.psum);
    A.lsum = reinterpret_cast<float *>(ws + Lw.lsum);
    A.Wc = reinterpret_cast<_Float16 *>(ws + Lw.wc);
    A.Wd = reinterpret_cast<_Float16 *>(ws + Lw.wd);
    A.col = reinterpret_cast<float *>(ws + Lw.col);
    A.invF = reinterpret_cast<float *>(ws + Lw.invF);
    // psum, col and lsum are contiguous (up to padding) in the workspace
    hipLaunchKernelGGL(k_quant_zero, dim3(1), dim3(256), 0, s, counts, (int64_t)N,
                       reinterpret_cast<uint32_t *>(ws + Lw.psum), (Lw.wc - Lw.psum) / 4);
    const int KB = N / 32;
    const int64_t rounds = (K + QGROUP - 1) / QGROUP;
    const int gq = (int)(rounds < ctx->num_cus ? (rounds < 1 ? 1 : rounds) : ctx->num_cus);
    const int64_t per_block = 4096;
    const dim3 gw((unsigned)((Lw.Kp + per_block - 1) / per_block), (unsigned)(d / QCH));
    const int gz = (int)((((int64_t)N * d + 255) / 256) < 1024 ? ((int64_t)N * d + 255) / 256 : 1024);
#define LEGS_QUANT(KBV)                                                                                              \
    hipLaunchKernelGGL(k_quant_prep<KBV>, dim3(64), dim3(256), 0, s, S, d, dC,                                     \
                       reinterpret_cast<f16x8 *>(ws + Lw.img), reinterpret_cast<float *>(ws + Lw.invS));           \
    if (K > 0) hipLaunchKernelGGL((k_quant_pass<KBV, false>), dim3(gq), dim3(QTHREADS), 0, s, A);                  \
    if (grad) {                                                                                                      \
        hipLaunchKernelGGL(k_quant_zero, dim3(gz), dim3(256), 0, s, reinterpret_cast<uint32_t *>(grad),            \
                           (int64_t)N * d, (uint32_t *)nullptr, (int64_t)0);                                        \
        if (K > 0) {                                                                                                 \
            hipLaunchKernelGGL((k_quant_pass<KBV, true>), dim3(gq), dim3(QTHREADS), 0, s, A);                      \
            hipLaunchKernelGGL(k_quant_wgrad<KBV>, gw, dim3(256), 0, s, A.F, K, Lw.Kp, d, dC, per_block, A.Wc,      \
                               A.Wd, A.invF, A.invS, grad);                                                                 \
        }                                                                                                            \
    }                                                                                                                \
    hipLaunchKernelGGL(k_quant_finish<KBV>, dim3(grad ? gz : 1), dim3(256), 0, s, S, d, dC, K, A.invS, A.col,      \
                       grad, counts, A.psum, A.lsum, lam_cos, lam_lb, prob_mean, losses);
    switch (KB) {
    case 1: LEGS_QUANT(1) break;
    case 2: LEGS_QUANT(2) break;
    case 4: LEGS_QUANT(4) break;
    default: return legs_set_error(ctx, LEGS_ERR_ARG, "N must be 32, 64 or 128");
    }
#undef LEGS_QUANT
    LEGS_CHECK_LAUNCH(ctx);
    return LEGS_OK;
}
