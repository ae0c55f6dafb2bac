// aes_device.hpp -- T-table AES round core for gfx950 (device side).
//
// One 16-byte AES state per lane, held as four little-endian column words
// W0..W3 (row r of column c in bits 8r..8r+7 of Wc), as in the paper's
// one-state-per-thread granularity (section 4.1).
//
// Inner round (section 3.2.3, eq 26), column j, indices mod 4:
//   enc: e_j = T0[b0(W_j)]   ^ T1[b1(W_{j+1})] ^ T2[b2(W_{j+2})] ^ T3[b3(W_{j+3})] ^ k_j
//   dec: e_j = Td0[b0(W_j)]  ^ Td1[b1(W_{j-1})] ^ Td2[b2(W_{j-2})] ^ Td3[b3(W_{j-3})] ^ k_j
// (decryption is the equivalent inverse cipher of FIPS-197 5.3.5: the round
// keys of rounds 1..Nr-1 have InvMixColumns applied, see aes_expand_key.)
// Final round has no MixColumns: enc takes the S-box byte from the T-table
// whose byte t is {01}s (T2 row 0, T3 row 1, T0 row 2, T1 row 3); dec uses Si4.
//
// LDS layout (gfx950 LDS: 32 banks of 4 bytes; a wave64 ds_read_b32 is served
// 32 lanes per clock, so 32 replicas make any lookup pattern conflict free):
//   table t, entry e, replica r at byte  (t & 1) * 65536 + e * 256 + (t >> 1) * 128 + r * 4
//   Si4 (decryption only), entry e, replica r at byte  131072 + e * 128 + r * 4
// Lane l reads replica r = l mod 32, so every access of one instruction falls
// in bank l mod 32.  With the entry index in address bits 8..15, an address is
// (byte of W shifted to bits 8..15) | base_t, built with one or two of the
// instructions gfx950 issues at full rate (v_bitop3_b32 with VGPR operands,
// v_lshlrev_b16, v_lshrrev_b32, v_or_b32).  v_perm_b32, v_bfe_u32, SDWA forms
// and any VALU form with an SGPR operand issue at about half that rate.
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>

#include "aes_tables.hpp"

namespace aesgpu {

constexpr uint32_t kTableBytes = 131072;        // four 1 KiB tables x 32 replicas
constexpr uint32_t kSi4Offset = 131072;
constexpr uint32_t kSi4Bytes = 32768;           // 256 entries x 32 replicas x 4 B
constexpr uint32_t kEncLdsWords = kTableBytes / 4;
constexpr uint32_t kDecLdsWords = (kTableBytes + kSi4Bytes) / 4;

// Source tables in constant memory (one copy per translation unit).
static __constant__ TableSet c_tables = make_tables();

// Full-rate gfx950 VALU forms (all operands in VGPRs).
__device__ __forceinline__ uint32_t and_or(uint32_t a, uint32_t m, uint32_t b)
{
    uint32_t d;  // (a & m) | b
    asm("v_bitop3_b32 %0, %1, %2, %3 bitop3:0xea" : "=v"(d) : "v"(a), "v"(m), "v"(b));
    return d;
}

__device__ __forceinline__ uint32_t xor3(uint32_t a, uint32_t b, uint32_t c)
{
    uint32_t d;
    asm("v_bitop3_b32 %0, %1, %2, %3 bitop3:0x96" : "=v"(d) : "v"(a), "v"(b), "v"(c));
    return d;
}

__device__ __forceinline__ uint32_t shl16_by8(uint32_t a)
{
    uint32_t d;  // (a << 8) & 0xffff: byte 0 moved to bits 8..15
    asm("v_lshlrev_b16 %0, 8, %1" : "=v"(d) : "v"(a));
    return d;
}

__device__ __forceinline__ uint32_t shl16_by7(uint32_t a)
{
    uint32_t d;  // (a << 7) & 0xffff
    asm("v_lshlrev_b16 %0, 7, %1" : "=v"(d) : "v"(a));
    return d;
}

__device__ __forceinline__ uint32_t lds_word(const uint32_t* lds, uint32_t byte_addr)
{
    return *reinterpret_cast<const uint32_t*>(reinterpret_cast<const char*>(lds) + byte_addr);
}

// Per-lane constants of the lookup addresses.
struct LaneBases {
    uint32_t b[4];   // base of table t for this lane's replica
    uint32_t bs;     // base of Si4 for this lane's replica
    uint32_t m8;     // 0x0000ff00
    uint32_t m7;     // 0x00007f80
    uint32_t m16;    // 0x00ff0000
    uint32_t m24;    // 0xff000000

    __device__ __forceinline__ explicit LaneBases(uint32_t lane)
    {
        uint32_t r4 = (lane & 31u) << 2;
        for (int t = 0; t < 4; ++t)
            b[t] = ((uint32_t(t) & 1u) << 16) | ((uint32_t(t) >> 1) << 7) | r4;
        bs = kSi4Offset | r4;
        // opaque copies keep these in VGPRs so every bitop3 operand is a VGPR
        asm volatile("v_mov_b32 %0, 0xff00" : "=v"(m8));
        asm volatile("v_mov_b32 %0, 0x7f80" : "=v"(m7));
        asm volatile("v_mov_b32 %0, 0xff0000" : "=v"(m16));
        asm volatile("v_mov_b32 %0, 0xff000000" : "=v"(m24));
    }
};

// Fill the replicated tables of one direction into LDS (whole workgroup).
template <bool kDecrypt>
__device__ __forceinline__ void fill_tables(uint32_t* lds, const TableSet* __restrict__ tabs)
{
    const uint32_t* src = kDecrypt ? tabs->td0 : tabs->te0;
    for (uint32_t w = threadIdx.x; w < kEncLdsWords; w += blockDim.x) {
        uint32_t region = w >> 14, e = (w >> 6) & 255u, half = (w >> 5) & 1u;
        uint32_t t = region | (half << 1);
        uint32_t v = src[e];
        lds[w] = t ? ((v << (8 * t)) | (v >> (32 - 8 * t))) : v;
    }
    if (kDecrypt) {
        for (uint32_t w = threadIdx.x; w < kSi4Bytes / 4; w += blockDim.x)
            lds[kSi4Offset / 4 + w] = tabs->si4[w >> 5];
    }
}

// The four lookup addresses of one state word (byte t -> table t).
struct WordAddr {
    uint32_t a[4];
};

__device__ __forceinline__ WordAddr round_addr(uint32_t w, const LaneBases& lb, const uint32_t base[4])
{
    WordAddr r;
    r.a[0] = shl16_by8(w) | base[0];
    r.a[1] = and_or(w, lb.m8, base[1]);
    r.a[2] = and_or(w >> 8, lb.m8, base[2]);
    r.a[3] = and_or(w >> 16, lb.m8, base[3]);
    return r;
}

// One block through all rounds. K(i) returns round-key word i (uniform).
template <int NR, bool kDecrypt, class K>
__device__ __forceinline__ uint4 crypt_block(uint4 in, const uint32_t* lds, const LaneBases& lb, const K& key)
{
    uint32_t w[4] = {in.x ^ key(0), in.y ^ key(1), in.z ^ key(2), in.w ^ key(3)};
#pragma unroll
    for (int round = 1; round < NR; ++round) {
        uint32_t v[4][4];  // v[t][j]: table t looked up with byte t of word j
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            WordAddr a = round_addr(w[j], lb, lb.b);
#pragma unroll
            for (int t = 0; t < 4; ++t)
                v[t][j] = lds_word(lds, a.a[t]);
        }
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int s = kDecrypt ? 3 : 1;  // j+1 (enc) or j-1 (dec), mod 4
            uint32_t x = xor3(v[0][j], v[1][(j + s) & 3], v[2][(j + 2 * s) & 3]);
            w[j] = xor3(x, v[3][(j + 3 * s) & 3], key(4 * round + j));
        }
    }
    uint32_t f[4][4];
    if (!kDecrypt) {
        // byte t of the result row comes from table T_{t+2}, where byte t is {01}s
        const uint32_t fb[4] = {lb.b[2], lb.b[3], lb.b[0], lb.b[1]};
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            WordAddr a = round_addr(w[j], lb, fb);
#pragma unroll
            for (int t = 0; t < 4; ++t)
                f[t][j] = lds_word(lds, a.a[t]);
        }
    } else {
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            f[0][j] = lds_word(lds, and_or(shl16_by7(w[j]), lb.m7, lb.bs));
            f[1][j] = lds_word(lds, and_or(w[j] >> 1, lb.m7, lb.bs));
            f[2][j] = lds_word(lds, and_or(w[j] >> 9, lb.m7, lb.bs));
            f[3][j] = lds_word(lds, and_or(w[j] >> 17, lb.m7, lb.bs));
        }
    }
    uint32_t o[4];
    const int s = kDecrypt ? 3 : 1;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        uint32_t m = f[0][j] & 0xffu;
        m = and_or(f[1][(j + s) & 3], lb.m8, m);
        m = and_or(f[2][(j + 2 * s) & 3], lb.m16, m);
        m = and_or(f[3][(j + 3 * s) & 3], lb.m24, m);
        o[j] = m ^ key(4 * NR + j);
    }
    return make_uint4(o[0], o[1], o[2], o[3]);
}

}  // namespace aesgpu
