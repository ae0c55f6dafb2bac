// aes_bitslice.hip -- the bitsliced placement: AES with no tables.
//
// Each lane holds 32 blocks as 128 bit slices: slice 8p + i is a 32-bit
// word whose bit j is bit i of byte p of the lane's block j.  In this form
// the round of section 3.2.2 (Algorithm 1, read as the standard Cipher) is
// plain Boolean algebra on whole registers:
//   SubBytes    the S-box as a network of 3-input LUTs (aes_sbox_circuit.hpp,
//               about 105 v_bitop3_b32 per 32 bytes), no lookups at all;
//   ShiftRows   a renaming of slices (eq 19);
//   MixColumns  an XOR network per column (eq 20), with xtime on slices;
//   AddRoundKey the key bits are uniform, so each slice is XORed with an
//               all-ones or all-zeros mask held in a scalar register.
// Decryption is the equivalent inverse cipher with the decryption schedule
// (the same key form the table placements use), with InvMixColumns written
// as MixColumns after a step that adds {04}(a0 + a2) and {04}(a1 + a3).
// The lane's 32 blocks are loaded as 32 coalesced 1 KiB wave rows (block
// unit + 64 j + lane) and moved into slice form by 32x32 bit transposes, and
// back the same way before the store.  The round loop is not unrolled, so
// the kernel's code stays within the instruction cache.
#include "aes_ecb_kernel.hpp"
#include "aes_sbox_circuit.hpp"

namespace aesgpu {

constexpr int kSlicedBlocks = 32;  // blocks per lane

// Masks of the bit-level transpose stages, kept in VGPRs so that every
// v_bitop3_b32 operand is a VGPR (the full-rate form).
struct TransposeMasks {
    uint32_t m4, m2, m1;
    __device__ __forceinline__ TransposeMasks()
    {
        asm volatile("v_mov_b32 %0, 0x0f0f0f0f" : "=v"(m4));
        asm volatile("v_mov_b32 %0, 0x33333333" : "=v"(m2));
        asm volatile("v_mov_b32 %0, 0x55555555" : "=v"(m1));
    }
};

// In place: afterwards bit c of a[r] is the former bit r of a[c].  Five
// stages exchange the off-diagonal sub-blocks of 16, 8, 4, 2 and 1 bits
// between rows k and k + s.  The 16- and 8-bit stages move whole halves or
// bytes, one v_perm_b32 per result row; the bit stages are a shift and a
// select, (m ? x : y) being the bitop3 table 0xca.
__device__ __forceinline__ void transpose32(uint32_t a[32], const TransposeMasks& tm)
{
#pragma unroll
    for (int k = 0; k < 16; ++k) {  // rows k, k + 16: [a0 a1 b0 b1], [a2 a3 b2 b3] in 16-bit halves
        const uint32_t x = a[k], y = a[k + 16];
        a[k] = __builtin_amdgcn_perm(y, x, 0x05040100u);
        a[k + 16] = __builtin_amdgcn_perm(y, x, 0x07060302u);
    }
#pragma unroll
    for (int g = 0; g < 32; g += 16) {
#pragma unroll
        for (int k = g; k < g + 8; ++k) {  // bytes: [x0 y0 x2 y2], [x1 y1 x3 y3]
            const uint32_t x = a[k], y = a[k + 8];
            a[k] = __builtin_amdgcn_perm(y, x, 0x06020400u);
            a[k + 8] = __builtin_amdgcn_perm(y, x, 0x07030501u);
        }
    }
#pragma unroll
    for (int lvl = 0; lvl < 3; ++lvl) {
        const int s = 4 >> lvl;
        const uint32_t m = lvl == 0 ? tm.m4 : lvl == 1 ? tm.m2 : tm.m1;
#pragma unroll
        for (int g = 0; g < 32; g += 2 * s) {
#pragma unroll
            for (int k = g; k < g + s; ++k) {
                const uint32_t x = a[k], y = a[k + s];
                const uint32_t ys = s == 1 ? y + y : y << s;
                a[k + s] = __builtin_amdgcn_bitop3_b32(m, x >> s, y, 0xca);
                a[k] = __builtin_amdgcn_bitop3_b32(m, x, ys, 0xca);
            }
        }
    }
}

__device__ __forceinline__ uint32_t comp(const uint4& v, int c)
{
    return c == 0 ? v.x : c == 1 ? v.y : c == 2 ? v.z : v.w;
}

__device__ __forceinline__ void set_comp(uint4& v, int c, uint32_t x)
{
    if (c == 0) v.x = x;
    else if (c == 1) v.y = x;
    else if (c == 2) v.z = x;
    else v.w = x;
}

// Blocks first + 64 j (j < 32) of the lane into slices; missing blocks are zero.
template <bool kGuard>
__device__ __forceinline__ void load_slices(const uint4* __restrict__ in, uint64_t first, uint64_t nblocks,
                                            uint32_t s[128], const TransposeMasks& tm)
{
    uint4 v[kSlicedBlocks];
#pragma unroll
    for (int j = 0; j < kSlicedBlocks; ++j) {
        const uint64_t b = first + 64u * j;
        v[j] = (!kGuard || b < nblocks) ? in[b] : make_uint4(0u, 0u, 0u, 0u);
    }
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        uint32_t w[32];
#pragma unroll
        for (int j = 0; j < 32; ++j)
            w[j] = comp(v[j], c);
        transpose32(w, tm);
#pragma unroll
        for (int b = 0; b < 32; ++b)
            s[32 * c + b] = w[b];
    }
}

template <bool kGuard>
__device__ __forceinline__ void store_slices(uint4* __restrict__ out, uint64_t first, uint64_t nblocks,
                                             const uint32_t s[128], const TransposeMasks& tm)
{
    uint4 v[kSlicedBlocks];
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        uint32_t w[32];
#pragma unroll
        for (int b = 0; b < 32; ++b)
            w[b] = s[32 * c + b];
        transpose32(w, tm);
#pragma unroll
        for (int j = 0; j < 32; ++j)
            set_comp(v[j], c, w[j]);
    }
#pragma unroll
    for (int j = 0; j < kSlicedBlocks; ++j) {
        const uint64_t b = first + 64u * j;
        if (!kGuard || b < nblocks)
            out[b] = v[j];
    }
}

// state ^= round key: byte p = 4c + r of the key is bits 8r..8r+7 of word c
__device__ __forceinline__ void add_round_key(uint32_t s[128], const uint32_t k[4])
{
#pragma unroll
    for (int p = 0; p < 16; ++p) {
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            const uint32_t mask = 0u - ((k[p >> 2] >> (8 * (p & 3) + i)) & 1u);
            s[8 * p + i] ^= mask;
        }
    }
}

template <bool kDecrypt>
__device__ __forceinline__ void sub_bytes(uint32_t s[128])
{
#pragma unroll
    for (int p = 0; p < 16; ++p) {
        uint32_t x[8], y[8];
#pragma unroll
        for (int i = 0; i < 8; ++i)
            x[i] = s[8 * p + i];
        if (kDecrypt)
            inv_sbox_slices(x, y);
        else
            sbox_slices(x, y);
#pragma unroll
        for (int i = 0; i < 8; ++i)
            s[8 * p + i] = y[i];
    }
}

// t = ShiftRows(s) (row r rotated left by r columns) or its inverse
template <bool kDecrypt>
__device__ __forceinline__ void shift_rows(const uint32_t s[128], uint32_t t[128])
{
#pragma unroll
    for (int c = 0; c < 4; ++c) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int src = kDecrypt ? (c - r + 4) & 3 : (c + r) & 3;
#pragma unroll
            for (int i = 0; i < 8; ++i)
                t[8 * (r + 4 * c) + i] = s[8 * (r + 4 * src) + i];
        }
    }
}

// multiplication by {02} of one byte in slice form
__device__ __forceinline__ void xtime_slices(const uint32_t u[8], uint32_t x[8])
{
    x[0] = u[7];
    x[1] = u[0] ^ u[7];
    x[2] = u[1];
    x[3] = u[2] ^ u[7];
    x[4] = u[3] ^ u[7];
    x[5] = u[4];
    x[6] = u[5];
    x[7] = u[6];
}

// MixColumns of the column whose byte r, bit i is col[8 r + i]
__device__ __forceinline__ void mix_column(uint32_t col[32])
{
    uint32_t t[8], o[32];
#pragma unroll
    for (int i = 0; i < 8; ++i)
        t[i] = xor3(col[i], col[8 + i], col[16 + i]) ^ col[24 + i];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        uint32_t u[8], x[8];
        const int n = (r + 1) & 3;
#pragma unroll
        for (int i = 0; i < 8; ++i)
            u[i] = col[8 * r + i] ^ col[8 * n + i];
        xtime_slices(u, x);
#pragma unroll
        for (int i = 0; i < 8; ++i)
            o[8 * r + i] = xor3(col[8 * r + i], t[i], x[i]);  // {02}a_r + {03}a_{r+1} + a_{r+2} + a_{r+3}
    }
#pragma unroll
    for (int k = 0; k < 32; ++k)
        col[k] = o[k];
}

// InvMixColumns = MixColumns after a_0,2 += {04}(a0 + a2), a_1,3 += {04}(a1 + a3)
__device__ __forceinline__ void inv_mix_column(uint32_t col[32])
{
    uint32_t u[8], v[8], x[8], y[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        u[i] = col[i] ^ col[16 + i];
        v[i] = col[8 + i] ^ col[24 + i];
    }
    xtime_slices(u, x);
    xtime_slices(x, u);
    xtime_slices(v, y);
    xtime_slices(y, v);
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        col[i] ^= u[i];
        col[16 + i] ^= u[i];
        col[8 + i] ^= v[i];
        col[24 + i] ^= v[i];
    }
    mix_column(col);
}

template <int NR, bool kDecrypt>
__device__ __forceinline__ void crypt_slices(uint32_t s[128], const RoundKeys& rk)
{
    {
        const uint32_t k0[4] = {rk.w[0], rk.w[1], rk.w[2], rk.w[3]};
        add_round_key(s, k0);
    }
#pragma unroll 1
    for (int round = 1; round < NR; ++round) {
        uint32_t t[128];
        sub_bytes<kDecrypt>(s);
        shift_rows<kDecrypt>(s, t);
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            if (kDecrypt)
                inv_mix_column(t + 32 * c);
            else
                mix_column(t + 32 * c);
        }
        const uint32_t k[4] = {rk.w[4 * round], rk.w[4 * round + 1], rk.w[4 * round + 2], rk.w[4 * round + 3]};
        add_round_key(t, k);
#pragma unroll
        for (int q = 0; q < 128; ++q)
            s[q] = t[q];
    }
    uint32_t t[128];
    sub_bytes<kDecrypt>(s);
    shift_rows<kDecrypt>(s, t);
    const uint32_t k[4] = {rk.w[4 * NR], rk.w[4 * NR + 1], rk.w[4 * NR + 2], rk.w[4 * NR + 3]};
    add_round_key(t, k);
#pragma unroll
    for (int q = 0; q < 128; ++q)
        s[q] = t[q];
}

template <int NR, bool kDecrypt>
__global__ __launch_bounds__(256, 2) void bitslice_kernel(const uint4* __restrict__ in, uint4* __restrict__ out,
                                                        uint64_t nblocks, RoundKeys rk)
{
    const uint32_t lane = threadIdx.x & 63u;
    const uint64_t waves_per_grid = (uint64_t)gridDim.x * (blockDim.x >> 6);
    constexpr uint64_t span = 64u * kSlicedBlocks;
    const TransposeMasks tm;
    for (uint64_t wv = (uint64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6); wv * span < nblocks;
         wv += waves_per_grid) {
        const uint64_t first = wv * span + lane;
        uint32_t s[128];
        const bool full = (wv + 1) * span <= nblocks;  // uniform across the wave
        if (full)
            load_slices<false>(in, first, nblocks, s, tm);
        else
            load_slices<true>(in, first, nblocks, s, tm);
        crypt_slices<NR, kDecrypt>(s, rk);
        if (full)
            store_slices<false>(out, first, nblocks, s, tm);
        else
            store_slices<true>(out, first, nblocks, s, tm);
    }
}

template <int NR, bool kDecrypt>
hipError_t launch_bs_one(const void* in, void* out, uint64_t nblocks, const RoundKeys& rk, int wg, int grid_req,
                         int cus, hipStream_t stream)
{
    auto kern = bitslice_kernel<NR, kDecrypt>;
    const LaunchShape shape{kSlicedBlocks, wg, grid_req};
    int grid = 0;
    hipError_t e = grid_for(reinterpret_cast<const void*>(kern), shape, cus, nblocks, &grid);
    if (e != hipSuccess)
        return e;
    hipLaunchKernelGGL(kern, dim3(grid), dim3(wg), 0, stream, static_cast<const uint4*>(in), static_cast<uint4*>(out),
                       nblocks, rk);
    return hipGetLastError();
}

hipError_t launch_bitslice(const LaunchShape& shape, int nr, bool decrypt, const void* in, void* out,
                           uint64_t nblocks, const RoundKeys& rk, int cus, hipStream_t stream)
{
    if (shape.wg > kBitsliceMaxWg)
        return hipErrorInvalidValue;
    switch (nr * 2 + (decrypt ? 1 : 0)) {
    case 20: return launch_bs_one<10, false>(in, out, nblocks, rk, shape.wg, shape.grid, cus, stream);
    case 21: return launch_bs_one<10, true>(in, out, nblocks, rk, shape.wg, shape.grid, cus, stream);
    case 24: return launch_bs_one<12, false>(in, out, nblocks, rk, shape.wg, shape.grid, cus, stream);
    case 25: return launch_bs_one<12, true>(in, out, nblocks, rk, shape.wg, shape.grid, cus, stream);
    case 28: return launch_bs_one<14, false>(in, out, nblocks, rk, shape.wg, shape.grid, cus, stream);
    case 29: return launch_bs_one<14, true>(in, out, nblocks, rk, shape.wg, shape.grid, cus, stream);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace aesgpu
