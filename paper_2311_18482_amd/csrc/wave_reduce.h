// Sums of N per-lane values over the 64 lanes of a wave, with the N totals
// left spread over the lanes ("transpose reduction", gfx950).
//
// Six stages, one per lane-id bit b = 5..0. A stage takes K registers and
// returns ceil(K / 2): register i is paired with register i + K/2, and a lane
// whose bit b is 0 keeps (its own + its partner's) copy of register i while a
// lane whose bit b is 1 keeps register i + K/2. An odd register left over is
// summed over bit b in place. One pair costs two instructions (a lane-swap and
// an add) where a plain butterfly would cost one add per value per stage.
//
//   bit 5: v_permlane32_swap (lanes 32-63 of the first operand <-> lanes 0-31
//          of the second)
//   bit 4: v_permlane16_swap (odd rows of the first <-> even rows of the second)
//   bit 3: DPP row_mirror (lane l <-> 15 - l in its row), bank-masked moves
//   bit 2: DPP row_half_mirror (l <-> 7 - l in its half row), bank-masked moves
//   bit 1: DPP quad_perm [2,3,0,1] with selects
//   bit 0: DPP quad_perm [1,0,3,2] with selects
//
// The mirrors also flip lower lane bits, which is harmless: the value a
// register holds depends only on the lane bits of the stages already done.
// legs_tr::index() replays the stages on value indices; it returns, per final
// register, the value whose total this lane holds, or -1 where the lane holds
// a zero or a duplicate (each total is held by exactly one lane).
#pragma once

#include <hip/hip_runtime.h>

namespace legs_tr {

constexpr int next_k(int K) { return K / 2 + (K & 1); }

constexpr int final_k(int K, int stages = 6) { return stages == 0 ? K : final_k(next_k(K), stages - 1); }

__device__ __forceinline__ unsigned fbits(float x) { return __builtin_bit_cast(unsigned, x); }
__device__ __forceinline__ float bitsf(unsigned x) { return __builtin_bit_cast(float, x); }

// DPP move: lanes enabled by BANK read src from the lane CTRL names; the others keep old.
template <int CTRL, int BANK>
__device__ __forceinline__ float dpp_mov(float old, float src)
{
    return bitsf((unsigned)__builtin_amdgcn_update_dpp((int)fbits(old), (int)fbits(src), CTRL, 0xF,
                                                       BANK, false));
}

// One stage over lane bit S: K registers in v[0..K), next_k(K) out.
template <int S, int K, int N>
__device__ __forceinline__ void stage(float (&v)[N], int lane)
{
    constexpr int H = K / 2;
    if constexpr (S == 5 || S == 4) {
#pragma unroll
        for (int i = 0; i < H; ++i) {
            if constexpr (S == 5) {
                auto r = __builtin_amdgcn_permlane32_swap(fbits(v[i]), fbits(v[i + H]), false, false);
                v[i] = bitsf(r[0]) + bitsf(r[1]);
            } else {
                auto r = __builtin_amdgcn_permlane16_swap(fbits(v[i]), fbits(v[i + H]), false, false);
                v[i] = bitsf(r[0]) + bitsf(r[1]);
            }
        }
        if constexpr (K & 1) {   // the total lands in the bit-0 lanes, zero in the others
            if constexpr (S == 5) {
                auto r = __builtin_amdgcn_permlane32_swap(fbits(v[K - 1]), 0u, false, false);
                v[H] = bitsf(r[0]) + bitsf(r[1]);
            } else {
                auto r = __builtin_amdgcn_permlane16_swap(fbits(v[K - 1]), 0u, false, false);
                v[H] = bitsf(r[0]) + bitsf(r[1]);
            }
        }
    } else if constexpr (S == 3 || S == 2) {
        constexpr int CTRL = S == 3 ? 0x140 : 0x141;      // row_mirror / row_half_mirror
        constexpr int LO = S == 3 ? 0x3 : 0x5;            // banks of 4 lanes whose bit S is 0
        constexpr int HI = S == 3 ? 0xC : 0xA;
#pragma unroll
        for (int i = 0; i < H; ++i) {
            const float t = dpp_mov<CTRL, LO>(v[i + H], v[i]);   // bit 0: partner's v[i]; bit 1: own v[i+H]
            const float u = dpp_mov<CTRL, HI>(v[i], v[i + H]);   // bit 1: partner's v[i+H]; bit 0: own v[i]
            v[i] = t + u;
        }
        if constexpr (K & 1) v[H] = v[K - 1] + dpp_mov<CTRL, 0xF>(0.0f, v[K - 1]);
    } else {
        constexpr int CTRL = S == 1 ? 0x4E : 0xB1;         // quad_perm [2,3,0,1] / [1,0,3,2]
        const bool hi = (lane >> S) & 1;
#pragma unroll
        for (int i = 0; i < H; ++i) {
            const float keep = hi ? v[i + H] : v[i];
            const float send = hi ? v[i] : v[i + H];
            v[i] = keep + dpp_mov<CTRL, 0xF>(0.0f, send);
        }
        if constexpr (K & 1) v[H] = v[K - 1] + dpp_mov<CTRL, 0xF>(0.0f, v[K - 1]);
    }
}

template <int S, int K, int N>
__device__ __forceinline__ void run(float (&v)[N], int lane)
{
    if constexpr (S >= 0) {
        stage<S, K, N>(v, lane);
        run<S - 1, next_k(K), N>(v, lane);
    }
}

// In place: on return v[0 .. final_k(N)) hold the totals this lane owns.
template <int N>
__device__ __forceinline__ void reduce(float (&v)[N], int lane)
{
    run<5, N, N>(v, lane);
}

template <int S, int K, int N>
__device__ __forceinline__ void index_run(int (&idx)[N], int lane)
{
    if constexpr (S >= 0) {
        constexpr int H = K / 2;
        const bool hi = (lane >> S) & 1;
#pragma unroll
        for (int i = 0; i < H; ++i) idx[i] = hi ? idx[i + H] : idx[i];
        if constexpr (K & 1) idx[H] = hi ? -1 : idx[K - 1];
        index_run<S - 1, next_k(K), N>(idx, lane);
    }
}

// The value index that slot q of the final registers holds after the stages
// S .. 0 over K values (-1: none), walking the stages backwards from the
// last: the closed form of index_run for one slot, with no array of indices.
template <int S, int K>
__device__ __forceinline__ int src_index(int q, int lane)
{
    if constexpr (S < 0) {
        return q;
    } else {
        const int p = src_index<S - 1, next_k(K)>(q, lane);   // slot after stage S
        constexpr int H = K / 2;
        const bool hi = (lane >> S) & 1;
        if (p < 0) return -1;
        if constexpr (K & 1) {
            if (p == H) return hi ? -1 : K - 1;
        }
        return p + (hi ? H : 0);
    }
}

// Value index of each final register in this lane (-1: a zero or a duplicate).
template <int N>
__device__ __forceinline__ void index(int (&idx)[N], int lane)
{
#pragma unroll
    for (int i = 0; i < N; ++i) idx[i] = i;
    index_run<5, N, N>(idx, lane);
}

} // namespace legs_tr
