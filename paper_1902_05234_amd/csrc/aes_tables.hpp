// aes_tables.hpp -- compile-time AES tables for the GPU library (host and device).
//
// Built from exponent/logarithm tables of GF(2^8) with generator {03}; this is
// deliberately a different construction from the byte-wise test oracle.
//
//   S-box (SubBytes, section 3.2.2 Def. 4): s = A(b) with b = inverse of x in
//   GF(2^8) and A the AES affine map, written in the rotation form
//   s = b ^ rotl(b,1) ^ rotl(b,2) ^ rotl(b,3) ^ rotl(b,4) ^ 0x63.
//
//   T-tables (section 3.2.3, eqs 22-25): column word of T0 for input w is
//   ({02}s, s, s, {03}s) for rows 0..3.  A column word keeps row r in bits
//   8r..8r+7 (little-endian), so T_k = rotl(T0, 8k).
//
//   Decryption tables (the paper measures decryption but gives no tables):
//   Td0 for input w is ({0e}t, {09}t, {0d}t, {0b}t) with t = InvS(w), the
//   columns of the inverse MixColumns matrix; Td_k = rotl(Td0, 8k).
//   Si4 holds InvS(w) in all four bytes for the last decryption round, and
//   si_packed four consecutive InvS bytes per word (the byte-packed table).
#pragma once
#include <cstdint>

namespace aesgpu {

struct TableSet {
    uint8_t exp[256];
    uint8_t log[256];
    uint8_t sbox[256];
    uint8_t inv_sbox[256];
    uint32_t te0[256];
    uint32_t td0[256];
    uint32_t si4[256];
    uint32_t si_packed[64];  // InvS bytes 4q..4q+3 in one little-endian word
};

constexpr uint8_t rotl8(uint8_t v, int n) { return static_cast<uint8_t>((v << n) | (v >> (8 - n))); }

constexpr uint8_t gf_mul_log(const TableSet& t, uint8_t a, uint8_t b)
{
    if (a == 0 || b == 0)
        return 0;
    return t.exp[(t.log[a] + t.log[b]) % 255];
}

constexpr TableSet make_tables()
{
    TableSet t{};
    // powers of the generator {03} = x + 1: p <- p ^ xtime(p)
    uint8_t p = 1;
    for (int i = 0; i < 255; ++i) {
        t.exp[i] = p;
        t.log[p] = static_cast<uint8_t>(i);
        uint8_t x2 = static_cast<uint8_t>((p << 1) ^ ((p & 0x80) ? 0x1B : 0));
        p = static_cast<uint8_t>(p ^ x2);
    }
    t.exp[255] = t.exp[0];
    for (int x = 0; x < 256; ++x) {
        uint8_t b = (x == 0) ? 0 : t.exp[(255 - t.log[x]) % 255];
        uint8_t s = static_cast<uint8_t>(b ^ rotl8(b, 1) ^ rotl8(b, 2) ^ rotl8(b, 3) ^ rotl8(b, 4) ^ 0x63);
        t.sbox[x] = s;
        t.inv_sbox[s] = static_cast<uint8_t>(x);
    }
    for (int x = 0; x < 256; ++x) {
        uint8_t s = t.sbox[x];
        uint32_t s2 = gf_mul_log(t, s, 0x02), s3 = gf_mul_log(t, s, 0x03);
        t.te0[x] = s2 | (uint32_t(s) << 8) | (uint32_t(s) << 16) | (s3 << 24);
        uint8_t v = t.inv_sbox[x];
        t.td0[x] = uint32_t(gf_mul_log(t, v, 0x0e)) | (uint32_t(gf_mul_log(t, v, 0x09)) << 8) |
                   (uint32_t(gf_mul_log(t, v, 0x0d)) << 16) | (uint32_t(gf_mul_log(t, v, 0x0b)) << 24);
        t.si4[x] = uint32_t(v) * 0x01010101u;
    }
    for (int q = 0; q < 64; ++q)
        t.si_packed[q] = uint32_t(t.inv_sbox[4 * q]) | (uint32_t(t.inv_sbox[4 * q + 1]) << 8) |
                         (uint32_t(t.inv_sbox[4 * q + 2]) << 16) | (uint32_t(t.inv_sbox[4 * q + 3]) << 24);
    return t;
}

constexpr uint32_t rotl32(uint32_t v, int n) { return n == 0 ? v : ((v << n) | (v >> (32 - n))); }

}  // namespace aesgpu
