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
// With little-endian column words T_k = rotl(T_0, 8k).  The final round has
// no MixColumns: encryption takes the S-box byte from a T-table whose byte t
// is {01}s (T0 has it in bytes 1 and 2, T2 in bytes 0 and 3); decryption
// reads a replicated InvS table.
//
// gfx950 LDS has 32 banks of 4 bytes and serves a wave64 ds_read_b32 32 lanes
// per clock, so a table replicated 32 times, with lane l reading replica
// l mod 32, is conflict free for any data.  Three placements of the tables in
// LDS trade LDS size (and so workgroups per CU) against VALU work:
//
//   4 tables  T0..T3, 32 replicas each: 128 KiB.  Table t, entry e, replica r
//             at byte (t & 1) * 65536 + e * 256 + (t >> 1) * 128 + r * 4.
//   2 tables  T0 and T2 = rotl(T0, 16): 64 KiB, at e * 256 + h * 128 + r * 4
//             (h = 0 for T0, 1 for T2); T1/T3 terms are summed and rotated
//             by 8 once per column.
//   1 table   T0 only: 32 KiB at e * 128 + r * 4; three rotations per column.
//
// InvS for the last decryption round follows the tables: word-wide (InvS in
// all four bytes, e * 128 + r * 4, 32 KiB) with 4 tables, byte-packed
// ((e >> 2) * 128 + r * 4 + (e & 3), 8 KiB) with 1 or 2 tables.
//
// Lookup addresses put the state byte into bits 8..15 (stride 256) or 7..14
// (stride 128) and combine it with the lane's base.  With stride 256 that is
// one v_perm_b32 per lookup, and the last round merges its four bytes with
// two more.  A byte permute issues at about half the rate of a plain
// v_bitop3_b32, so in instruction slots it costs what the two-instruction
// shift-and-OR form costs; but under this load the engine clock drops well
// below its peak, and fewer instructions (and fewer VGPR reads: the
// selectors stay in SGPRs) measured a higher clock and a higher rate.
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>

#include "aes_tables.hpp"

namespace aesgpu {

constexpr int kPlace4 = 0;  // values match AES_PLACEMENT_* in aesgpu.h
constexpr int kPlace2 = 1;
constexpr int kPlace1 = 2;

template <int PL, bool kDecrypt>
struct Layout {
    static constexpr uint32_t table_bytes = PL == kPlace4 ? 131072u : PL == kPlace2 ? 65536u : 32768u;
    static constexpr uint32_t si_offset = table_bytes;
    static constexpr uint32_t si_bytes = !kDecrypt ? 0u : PL == kPlace4 ? 32768u : 8192u;
    static constexpr uint32_t words = (table_bytes + si_bytes) / 4;
};

// Source tables in constant memory (one copy per translation unit).
static __constant__ TableSet c_tables = make_tables();

// Full-rate gfx950 VALU forms (all operands in VGPRs).
// v_bitop3_b32 computes any function of three inputs given as an 8-entry
// truth table indexed by (src0 << 2) | (src1 << 1) | src2.
__device__ __forceinline__ uint32_t and_or(uint32_t a, uint32_t m, uint32_t b)
{
    return __builtin_amdgcn_bitop3_b32(a, m, b, 0xea);  // (a & m) | b
}

__device__ __forceinline__ uint32_t or_xor(uint32_t a, uint32_t b, uint32_t c)
{
    return __builtin_amdgcn_bitop3_b32(a, b, c, 0x56);  // (a | b) ^ c
}

__device__ __forceinline__ uint32_t xor3(uint32_t a, uint32_t b, uint32_t c)
{
    return __builtin_amdgcn_bitop3_b32(a, b, c, 0x96);  // a ^ b ^ c
}

// a ^ b ^ k with k uniform: k stays in an SGPR.  This is the half-rate form,
// but it keeps the round keys out of VGPRs (44-60 of them otherwise), which
// leaves room for more resident waves; the cost is 4 instructions per round.
__device__ __forceinline__ uint32_t xor3_key(uint32_t a, uint32_t b, uint32_t k)
{
    return __builtin_amdgcn_bitop3_b32(a, b, k, 0x96);
}

template <int N>
__device__ __forceinline__ uint32_t shl16(uint32_t a)
{
    uint32_t d;  // (a << N) & 0xffff
    asm("v_lshlrev_b16 %0, %2, %1" : "=v"(d) : "v"(a), "i"(N));
    return d;
}

__device__ __forceinline__ uint32_t rotl8(uint32_t y) { return (y << 8) | (y >> 24); }
__device__ __forceinline__ uint32_t rotl16(uint32_t y) { return (y << 16) | (y >> 16); }
__device__ __forceinline__ uint32_t rotl24(uint32_t y) { return (y << 24) | (y >> 8); }

__device__ __forceinline__ uint32_t lds_word(const uint32_t* lds, uint32_t byte_addr)
{
    return *reinterpret_cast<const uint32_t*>(reinterpret_cast<const char*>(lds) + byte_addr);
}

__device__ __forceinline__ uint32_t lds_byte(const uint32_t* lds, uint32_t byte_addr)
{
    return *(reinterpret_cast<const uint8_t*>(lds) + byte_addr);
}

// Per-lane constants of the lookup addresses.
template <int PL, bool kDecrypt>
struct LaneBases {
    uint32_t b[4];   // base used for state byte t in an inner round
    uint32_t f[4];   // base used for state byte t in the last (encryption) round
    uint32_t bs;     // InvS base
    uint32_t m7, m3, m1f80;

    __device__ __forceinline__ explicit LaneBases(uint32_t lane)
    {
        const uint32_t r4 = (lane & 31u) << 2;
        if (PL == kPlace4) {
            for (int t = 0; t < 4; ++t)
                b[t] = ((uint32_t(t) & 1u) << 16) | ((uint32_t(t) >> 1) << 7) | r4;
            // byte t of the last-round result comes from T_{t+2}
            f[0] = b[2], f[1] = b[3], f[2] = b[0], f[3] = b[1];
        } else if (PL == kPlace2) {
            b[0] = b[1] = r4;                // T0
            b[2] = b[3] = 128u | r4;         // T2
            f[0] = f[3] = 128u | r4;         // T2 has {01}s in bytes 0 and 3
            f[1] = f[2] = r4;                // T0 has {01}s in bytes 1 and 2
        } else {
            for (int t = 0; t < 4; ++t)
                b[t] = f[t] = r4;
        }
        bs = Layout<PL, kDecrypt>::si_offset | r4;
        // opaque copies keep the masks in VGPRs so every bitop3 operand is a VGPR
        asm volatile("v_mov_b32 %0, 0x7f80" : "=v"(m7));
        asm volatile("v_mov_b32 %0, 3" : "=v"(m3));
        asm volatile("v_mov_b32 %0, 0x1f80" : "=v"(m1f80));
    }
};

// Fill the replicated tables of one direction into LDS (whole workgroup).
// The fill is a list of jobs of 8 entries x 32 replicas: 32 jobs for the
// T-table entries, then (decryption) 32 jobs for the word-wide InvS or 8 for
// the byte-packed one (64 packed words).  In a job, lane l stores replicas
// 4(l & 7) .. 4(l & 7) + 3 of entry 8 * job + (l >> 3) with one ds_write_b128
// per stored table, the T-tables as rotations of the one loaded word
// (T_t = rotl(T_0, 8t)); every 8 lanes store 128 consecutive bytes, so the
// stores are conflict free.  A wave loads the source words of up to
// kFillBatch jobs (one per lane per job) before its first store, so the
// whole fill costs one memory round trip with workgroups of 256 threads or
// more (512 or more for decryption) and holds few registers.
constexpr uint32_t kFillBatch = 8;

__device__ __forceinline__ void store4(uint32_t* lds, uint32_t word, uint32_t v)
{
    *reinterpret_cast<uint4*>(lds + word) = make_uint4(v, v, v, v);
}

template <int PL, bool kDecrypt>
__device__ __forceinline__ void fill_tables(uint32_t* lds, const TableSet* __restrict__ tabs)
{
    using L = Layout<PL, kDecrypt>;
    constexpr uint32_t kTJobs = 32;
    constexpr uint32_t kJobs = kTJobs + (!kDecrypt ? 0u : PL == kPlace4 ? 32u : 8u);
    constexpr uint32_t kStride = PL == kPlace1 ? 32u : 64u;  // words from one T-table entry to the next
    const uint32_t* src = kDecrypt ? tabs->td0 : tabs->te0;
    const uint32_t* si = PL == kPlace4 ? tabs->si4 : tabs->si_packed;
    const uint32_t lane = threadIdx.x & 63u;
    const uint32_t sub = lane >> 3;         // entry of the job
    const uint32_t rep = (lane & 7u) * 4u;  // first of the lane's replicas
    const uint32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const uint32_t nwaves = blockDim.x >> 6;
    for (uint32_t j0 = wave; j0 < kJobs; j0 += kFillBatch * nwaves) {
        uint32_t v[kFillBatch];
#pragma unroll
        for (uint32_t k = 0; k < kFillBatch; ++k) {
            const uint32_t job = j0 + k * nwaves;  // uniform
            if (job < kTJobs)
                v[k] = src[job * 8u + sub];
            else if (job < kJobs)
                v[k] = si[(job - kTJobs) * 8u + sub];
        }
#pragma unroll
        for (uint32_t k = 0; k < kFillBatch; ++k) {
            const uint32_t job = j0 + k * nwaves;
            if (job < kTJobs) {
                const uint32_t w = (job * 8u + sub) * kStride + rep;
                store4(lds, w, v[k]);                                      // T0
                if (PL == kPlace4) {
                    store4(lds, 16384u + w, (v[k] << 8) | (v[k] >> 24));   // T1
                    store4(lds, 32u + w, (v[k] << 16) | (v[k] >> 16));     // T2
                    store4(lds, 16416u + w, (v[k] << 24) | (v[k] >> 8));   // T3
                } else if (PL == kPlace2) {
                    store4(lds, 32u + w, (v[k] << 16) | (v[k] >> 16));     // T2
                }
            } else if (job < kJobs) {
                store4(lds, L::si_offset / 4 + ((job - kTJobs) * 8u + sub) * 32u + rep, v[k]);
            }
        }
    }
}

// Store of one finished 16-byte block, marked non-temporal: output blocks are
// written once and not read again by the kernel, and with the hint the L2
// does not keep them as dirty lines that the end of the launch must write
// back.  That write-back otherwise adds about 3 us to every launch from
// 16 MiB up (a third of a 16 MiB launch's time beyond its kernel work).
__device__ __forceinline__ void store_block(uint4* p, uint4 v)
{
    typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
    const u32x4 x = {v.x, v.y, v.z, v.w};
    __builtin_nontemporal_store(x, reinterpret_cast<u32x4*>(p));
}

// Address of byte t of w in a table with entry stride 256 or 128.  Stride
// 256: one v_perm_b32 writes byte t of w into bits 8..15 and copies bytes 0
// and 2 of the lane's base (bytes 1 and 3 of every base are zero).  The
// selector is uniform and stays in an SGPR.  Stride 128 needs a 7-bit shift,
// which a byte permute cannot do.
template <int STRIDE, int T>
__device__ __forceinline__ uint32_t addr_of(uint32_t w, uint32_t m7, uint32_t base)
{
    if (STRIDE == 256) {
        return __builtin_amdgcn_perm(w, base, 0x0c020000u | ((4u + T) << 8));
    } else {
        if (T == 0) return and_or(shl16<7>(w), m7, base);
        if (T == 1) return and_or(w >> 1, m7, base);
        if (T == 2) return and_or(w >> 9, m7, base);
        return and_or(w >> 17, m7, base);
    }
}

// Wave priority (s_setprio) inside the rounds.  The issue arbiter of a SIMD
// serves ready waves by priority before age, so: a wave issuing an inner
// round's lookups runs at 2, one combining an inner round's results at 1,
// and one in the last round, storing or loading blocks at 0.  Waves with
// lookups to issue refill the LDS queue first, and the waves that are
// leaving a unit take the slots left over.  Measured under sustained load
// against no priorities: AES-128 +3 % (encrypt) and +5 % (decrypt).  The
// levels only order this kernel's waves; no wave is ever blocked by them.
template <int LEVEL>
__device__ __forceinline__ void wave_priority()
{
    __builtin_amdgcn_s_setprio(LEVEL);
}

// Bytes 0 and 1 of the result from (a, b), bytes 2 and 3 from (c, d): one
// v_perm_b32 per pair, selectors chosen by the caller; then XOR the key.
__device__ __forceinline__ uint32_t merge4(uint32_t a, uint32_t b, uint32_t sel_ab, uint32_t c, uint32_t d,
                                           uint32_t sel_cd, uint32_t k)
{
    return or_xor(__builtin_amdgcn_perm(b, a, sel_ab), __builtin_amdgcn_perm(d, c, sel_cd), k);
}

// Address of byte t of w in the byte-packed InvS table.
template <int T>
__device__ __forceinline__ uint32_t packed_addr(uint32_t w, uint32_t m3, uint32_t m1f80, uint32_t base)
{
    const uint32_t x = T ? w >> (8 * T) : w;
    return and_or(shl16<5>(x), m1f80, and_or(x, m3, base));
}

// Inner rounds FIRST .. NR-1 and the final round of one block whose state
// after round FIRST-1 is `in`.  K(i) returns round-key word i (uniform).
template <int NR, bool kDecrypt, int PL, int FIRST, class K>
__device__ __forceinline__ uint4 crypt_rounds(uint4 in, const uint32_t* lds, const LaneBases<PL, kDecrypt>& lb,
                                              const K& key)
{
    constexpr int s = kDecrypt ? 3 : 1;  // neighbour column: j+1 (enc) or j-1 (dec), mod 4
    uint32_t w[4] = {in.x, in.y, in.z, in.w};
#pragma unroll
    for (int round = FIRST; round < NR; ++round) {
        // v[j][t]: the lookup with byte t that output column j needs, issued
        // column by column, so column j can be combined once its four lookups
        // are back while the later columns' lookups are still in flight
        uint32_t v[4][4];
        constexpr int S = PL == kPlace1 ? 128 : 256;
        wave_priority<2>();
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            v[j][0] = lds_word(lds, addr_of<S, 0>(w[j], lb.m7, lb.b[0]));
            v[j][1] = lds_word(lds, addr_of<S, 1>(w[(j + s) & 3], lb.m7, lb.b[1]));
            v[j][2] = lds_word(lds, addr_of<S, 2>(w[(j + 2 * s) & 3], lb.m7, lb.b[2]));
            v[j][3] = lds_word(lds, addr_of<S, 3>(w[(j + 3 * s) & 3], lb.m7, lb.b[3]));
        }
        wave_priority<1>();
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const uint32_t a = v[j][0], b = v[j][1], c = v[j][2], d = v[j][3];
            const uint32_t k = key(4 * round + j);
            if (PL == kPlace4) {
                w[j] = xor3_key(xor3(a, b, c), d, k);
            } else if (PL == kPlace2) {
                // a: T0, c: T2 as stored; b, d need T1 = rotl8(T0), T3 = rotl8(T2).
                // The key joins b and d before the rotate, so these kernels take
                // each inner-round key word turned right by 8 bits
                // (inner_keys_rotr8): three VALU instructions per column.
                w[j] = xor3(a, c, rotl8(xor3_key(b, d, k)));
            } else {
                // all from T0: a ^ rotl8(b) ^ rotl16(c) ^ rotl24(d), three
                // independent rotates and two XOR3s (five VALU per column)
                w[j] = xor3_key(xor3(a, rotl8(b), rotl16(c)), rotl24(d), k);
            }
        }
    }
    uint32_t o[4];
    wave_priority<0>();
    if (!kDecrypt) {
        uint32_t f[4][4];  // column by column, as in the inner rounds
        constexpr int S = PL == kPlace1 ? 128 : 256;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            f[j][0] = lds_word(lds, addr_of<S, 0>(w[j], lb.m7, lb.f[0]));
            f[j][1] = lds_word(lds, addr_of<S, 1>(w[(j + s) & 3], lb.m7, lb.f[1]));
            f[j][2] = lds_word(lds, addr_of<S, 2>(w[(j + 2 * s) & 3], lb.m7, lb.f[2]));
            f[j][3] = lds_word(lds, addr_of<S, 3>(w[(j + 3 * s) & 3], lb.m7, lb.f[3]));
        }
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            // byte t of the output is byte t of f[j][t] (PL1: byte 1 for
            // rows 0 and 1, byte 2 for rows 2 and 3, T0 being ({02}s, s, s, {03}s))
            if (PL == kPlace1)
                o[j] = merge4(f[j][0], f[j][1], 0x0c0c0501u, f[j][2], f[j][3], 0x06020c0cu, key(4 * NR + j));
            else
                o[j] = merge4(f[j][0], f[j][1], 0x0c0c0500u, f[j][2], f[j][3], 0x07020c0cu, key(4 * NR + j));
        }
    } else if (PL == kPlace4) {
        uint32_t f[4][4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const uint32_t bs[4] = {lb.bs, lb.bs, lb.bs, lb.bs};
            f[j][0] = lds_word(lds, addr_of<128, 0>(w[j], lb.m7, bs[0]));
            f[j][1] = lds_word(lds, addr_of<128, 1>(w[j], lb.m7, bs[1]));
            f[j][2] = lds_word(lds, addr_of<128, 2>(w[j], lb.m7, bs[2]));
            f[j][3] = lds_word(lds, addr_of<128, 3>(w[j], lb.m7, bs[3]));
        }
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            o[j] = merge4(f[j][0], f[(j + s) & 3][1], 0x0c0c0500u, f[(j + 2 * s) & 3][2], f[(j + 3 * s) & 3][3],
                          0x07020c0cu, key(4 * NR + j));
        }
    } else {
        uint32_t g[4][4];  // InvS bytes, zero-extended
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            g[j][0] = lds_byte(lds, packed_addr<0>(w[j], lb.m3, lb.m1f80, lb.bs));
            g[j][1] = lds_byte(lds, packed_addr<1>(w[j], lb.m3, lb.m1f80, lb.bs));
            g[j][2] = lds_byte(lds, packed_addr<2>(w[j], lb.m3, lb.m1f80, lb.bs));
            g[j][3] = lds_byte(lds, packed_addr<3>(w[j], lb.m3, lb.m1f80, lb.bs));
        }
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            o[j] = merge4(g[j][0], g[(j + s) & 3][1], 0x0c0c0400u, g[(j + 2 * s) & 3][2], g[(j + 3 * s) & 3][3],
                          0x04000c0cu, key(4 * NR + j));
        }
    }
    return make_uint4(o[0], o[1], o[2], o[3]);
}

// One block through all rounds: the first AddRoundKey, then rounds 1 .. NR.
template <int NR, bool kDecrypt, int PL, class K>
__device__ __forceinline__ uint4 crypt_block(uint4 in, const uint32_t* lds, const LaneBases<PL, kDecrypt>& lb,
                                             const K& key)
{
    return crypt_rounds<NR, kDecrypt, PL, 1>(
        make_uint4(in.x ^ key(0), in.y ^ key(1), in.z ^ key(2), in.w ^ key(3)), lds, lb, key);
}

}  // namespace aesgpu
