// aes_col_round.hpp -- one block's rounds with one column word per lane.
//
// Four lanes of a quad share one block, lane 4q + j holding column word W_j,
// so a lane issues four lookups per round instead of sixteen.  The round is
// eq 26: output column j needs byte t of W_{j+t} (W_{j-t} for decryption),
// and DPP quad permutations (one VALU move each) bring those three neighbour
// words to the lane.  Used by the one-column-per-lane ECB kernel and by the
// four-lanes-per-message CBC encryption kernel.  A quad is always wholly
// active or wholly idle, so the permutations read only active lanes.
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>

#include "aes_device.hpp"

namespace aesgpu {

// Word of quad lane (lane + D) mod 4, D = 1..3, by a DPP quad permutation.
template <int D>
__device__ __forceinline__ uint32_t quad_rot(uint32_t w)
{
    constexpr int ctrl = ((0 + D) & 3) | (((1 + D) & 3) << 2) | (((2 + D) & 3) << 4) | (((3 + D) & 3) << 6);
    return static_cast<uint32_t>(__builtin_amdgcn_mov_dpp(static_cast<int>(w), ctrl, 0xf, 0xf, true));
}

// Column j of one block through every round.  kc[r] is round key word
// 4r + j; x1..x3 are W_{j+1..3} (encryption) or W_{j-1..3} (decryption).
template <int NR, bool kDecrypt, int PL>
__device__ __forceinline__ uint32_t col_block(uint32_t w, const uint32_t* lds, const LaneBases<PL, kDecrypt>& lb,
                                              const uint32_t (&kc)[NR + 1])
{
    constexpr int S = PL == kPlace1 ? 128 : 256;
    w ^= kc[0];
#pragma unroll
    for (int round = 1; round < NR; ++round) {
        const uint32_t x1 = kDecrypt ? quad_rot<3>(w) : quad_rot<1>(w);
        const uint32_t x2 = quad_rot<2>(w);
        const uint32_t x3 = kDecrypt ? quad_rot<1>(w) : quad_rot<3>(w);
        wave_priority<2>();
        const uint32_t a = lds_word(lds, addr_of<S, 0>(w, lb.m7, lb.b[0]));
        const uint32_t b = lds_word(lds, addr_of<S, 1>(x1, lb.m7, lb.b[1]));
        const uint32_t c = lds_word(lds, addr_of<S, 2>(x2, lb.m7, lb.b[2]));
        const uint32_t d = lds_word(lds, addr_of<S, 3>(x3, lb.m7, lb.b[3]));
        wave_priority<1>();
        const uint32_t k = kc[round];
        if (PL == kPlace4)
            w = xor3_key(xor3(a, b, c), d, k);
        else if (PL == kPlace2)
            w = xor3(a, c, rotl8(xor3_key(b, d, k)));  // k turned right by 8 bits on the host
        else
            w = xor3_key(xor3(a, rotl8(b), rotl16(c)), rotl24(d), k);
    }
    wave_priority<0>();
    const uint32_t x1 = kDecrypt ? quad_rot<3>(w) : quad_rot<1>(w);
    const uint32_t x2 = quad_rot<2>(w);
    const uint32_t x3 = kDecrypt ? quad_rot<1>(w) : quad_rot<3>(w);
    if (!kDecrypt) {
        const uint32_t f0 = lds_word(lds, addr_of<S, 0>(w, lb.m7, lb.f[0]));
        const uint32_t f1 = lds_word(lds, addr_of<S, 1>(x1, lb.m7, lb.f[1]));
        const uint32_t f2 = lds_word(lds, addr_of<S, 2>(x2, lb.m7, lb.f[2]));
        const uint32_t f3 = lds_word(lds, addr_of<S, 3>(x3, lb.m7, lb.f[3]));
        if (PL == kPlace1)
            return merge4(f0, f1, 0x0c0c0501u, f2, f3, 0x06020c0cu, kc[NR]);
        return merge4(f0, f1, 0x0c0c0500u, f2, f3, 0x07020c0cu, kc[NR]);
    } else if (PL == kPlace4) {
        const uint32_t f0 = lds_word(lds, addr_of<128, 0>(w, lb.m7, lb.bs));
        const uint32_t f1 = lds_word(lds, addr_of<128, 1>(x1, lb.m7, lb.bs));
        const uint32_t f2 = lds_word(lds, addr_of<128, 2>(x2, lb.m7, lb.bs));
        const uint32_t f3 = lds_word(lds, addr_of<128, 3>(x3, lb.m7, lb.bs));
        return merge4(f0, f1, 0x0c0c0500u, f2, f3, 0x07020c0cu, kc[NR]);
    } else {
        const uint32_t g0 = lds_byte(lds, packed_addr<0>(w, lb.m3, lb.m1f80, lb.bs));
        const uint32_t g1 = lds_byte(lds, packed_addr<1>(x1, lb.m3, lb.m1f80, lb.bs));
        const uint32_t g2 = lds_byte(lds, packed_addr<2>(x2, lb.m3, lb.m1f80, lb.bs));
        const uint32_t g3 = lds_byte(lds, packed_addr<3>(x3, lb.m3, lb.m1f80, lb.bs));
        return merge4(g0, g1, 0x0c0c0400u, g2, g3, 0x04000c0cu, kc[NR]);
    }
}

}  // namespace aesgpu
