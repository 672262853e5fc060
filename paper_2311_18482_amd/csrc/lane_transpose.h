// Cross-lane transposes of 16-bit values for MFMA operand layouts, gfx950.
#pragma once

#include <stdint.h>

namespace legs_lt {

// DPP moves: lanes enabled by BANK (banks of 4 lanes in each row of 16)
// read src from the lane CTRL names, the others keep old.
template <int CTRL, int BANK>
__device__ __forceinline__ uint32_t dpp_move(uint32_t old, uint32_t src)
{
    return (uint32_t)__builtin_amdgcn_update_dpp((int)old, (int)src, CTRL, 0xF, BANK, false);
}

// A DPP move that writes every lane (its source lane always exists): no old
// value to keep, so no register to initialise first.
template <int CTRL>
__device__ __forceinline__ uint32_t dpp_all(uint32_t src)
{
    return (uint32_t)__builtin_amdgcn_mov_dpp((int)src, CTRL, 0xF, 0xF, false);
}

// 8 x 8 transpose of 16-bit values (bf16 or half) across each group of 8
// lanes (i = lane & 7):
// lane i holds 8 values of one row, element e in half e % 2 of word e / 2;
// afterwards lane i holds element i of the 8 lanes' rows, in lane order.
// Three rounds, each keeping one half of the current chunk size and taking
// the partner's other half: words 0-1 / 2-3 across lanes i ^ 4 (DPP row
// shifts by 4 into the banks that need them), words across i ^ 2, halves of
// each word across i ^ 1 (v_perm with psel = 0x05040100 on even lanes: own
// low, partner's low; 0x03020706 on odd lanes: partner's high, own high).
__device__ __forceinline__ void oct_transpose(uint32_t (&w)[4], bool b1, uint32_t psel)
{
    const uint32_t n0 = dpp_move<0x114, 0xA>(w[0], w[2]);   // lanes 4-7: lane i - 4's words 2, 3
    const uint32_t n1 = dpp_move<0x114, 0xA>(w[1], w[3]);
    const uint32_t n2 = dpp_move<0x104, 0x5>(w[2], w[0]);   // lanes 0-3: lane i + 4's words 0, 1
    const uint32_t n3 = dpp_move<0x104, 0x5>(w[3], w[1]);
    // every exchange runs on all lanes before the selects: a DPP move inside
    // one arm of a conditional would run under a partial exec mask and read
    // lanes that are switched off
    const uint32_t p0 = dpp_all<0x4E>(n0), p1 = dpp_all<0x4E>(n1);
    const uint32_t p2 = dpp_all<0x4E>(n2), p3 = dpp_all<0x4E>(n3);
    w[0] = b1 ? p1 : n0;
    w[1] = b1 ? n1 : p0;
    w[2] = b1 ? p3 : n2;
    w[3] = b1 ? n3 : p2;
#pragma unroll
    for (int k = 0; k < 4; ++k) w[k] = __builtin_amdgcn_perm(dpp_all<0xB1>(w[k]), w[k], psel);
}

// Operand order of a [R rows][columns] matrix of 16-bit values for a
// 32 x 32 x 16 MFMA that contracts over the columns: columns in steps of 16,
// rows in blocks of RW = min(R, 32) (R = 8, 16 or a multiple of 32); in the
// chunk of (step, block), slot j = row % 32 + RW ((g % 16) / 8) holds columns
// 16 step + 8 ((g % 16) / 8) .. + 7 of that row, 16 bytes, which is what lane
// j of the MFMA takes. A 32-row chunk is 64 slots in lane order (1 KB).
// Element offset of the fragment of (row, columns g .. g + 7), g a multiple
// of 8:
__device__ __forceinline__ int64_t frag_at(int64_t g, int R, int row)
{
    const int RW = R < 32 ? R : 32, RB = (R + 31) / 32;
    return ((((g >> 4) * RB + row / 32) * (2 * RW)) + row % 32 + RW * ((g >> 3) & 1)) * 8;
}

} // namespace legs_lt
