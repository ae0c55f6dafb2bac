// aes_ctr.hip -- counter mode on the same round core as ECB.
//
// CTR (section 3.1.5, eq 5; marked parallel in Table 1): data block j is
// XORed with the cipher of a counter block, and counter blocks of successive
// data blocks are successive 128-bit big-endian integers c0 + j (mod 2^128),
// so every block is independent, as in ECB.  Each lane builds its counter
// block from the block index (no memory read), runs the encryption rounds
// and XORs the result into the data it loaded: the same 32 bytes of HBM per
// block as an ECB encryption, and fewer LDS lookups (counter-mode caching,
// below).  Decryption is the same operation.  A partial last block is read and written byte by byte and
// uses the leading bytes of its key-stream block.
#include "aes_ecb_kernel.hpp"

namespace aesgpu {

// State words of counter block c0 + b: byte 0 of the block is the most
// significant byte, and state word c holds bytes 4c..4c+3 little-endian.
__device__ __forceinline__ uint4 counter_state(const Counter128& c0, uint64_t b)
{
    const uint64_t lo = c0.lo + b;
    const uint64_t hi = c0.hi + (lo < c0.lo ? 1u : 0u);
    return make_uint4(__builtin_bswap32(static_cast<uint32_t>(hi >> 32)), __builtin_bswap32(static_cast<uint32_t>(hi)),
                      __builtin_bswap32(static_cast<uint32_t>(lo >> 32)), __builtin_bswap32(static_cast<uint32_t>(lo)));
}

__device__ __forceinline__ uint4 xor4(uint4 a, uint4 b) { return make_uint4(a.x ^ b.x, a.y ^ b.y, a.z ^ b.z, a.w ^ b.w); }

// Counter-mode caching (rounds 1 and 2).  The kernel walks the counters in
// units of span = 64 * BPT consecutive values that start at a multiple of
// span, so within a unit bytes 0..14 of the counter block are the same for
// every lane and only byte 15 (the top byte of state word 3) differs.  In
// round 1 (eq 26) byte 15 feeds one lookup, T3 of output column 0; the
// other 15 lookups and output columns 1..3 are the same for the whole unit.
// In round 2 every output column then has exactly one lookup that depends
// on the lane (a byte of column 0) and three that do not.  So a unit
// computes the 27 shared lookups once, as uniform values from the source
// table in memory (scalar loads: no LDS work), and each lane does 1 + 4
// lookups in rounds 1-2 instead of 32: 16 Nr - 27 per block, 133 for
// AES-128 instead of 160.

// T_t[byte t of w] for a uniform w, from the source table (scalar load).
template <int T>
__device__ __forceinline__ uint32_t shared_lookup(uint32_t w)
{
    const uint32_t v = c_tables.te0[(w >> (8 * T)) & 255u];
    return T == 0 ? v : (v << (8 * T)) | (v >> (32 - 8 * T));
}

// T_t[byte t of w] for a per-lane w, from the tables of placement PL in LDS.
template <int PL, int T>
__device__ __forceinline__ uint32_t lane_lookup(const uint32_t* lds, const LaneBases<PL, false>& lb, uint32_t w)
{
    if (PL == kPlace4)
        return lds_word(lds, addr_of<256, T>(w, lb.m7, lb.b[T]));
    if (PL == kPlace2) {
        const uint32_t v = lds_word(lds, addr_of<256, T>(w, lb.m7, lb.b[T]));  // T0 or T2 as stored
        return (T & 1) ? rotl8(v) : v;
    }
    const uint32_t v = lds_word(lds, addr_of<128, T>(w, lb.m7, lb.b[T]));      // T0
    return T == 0 ? v : T == 1 ? rotl8(v) : T == 2 ? rotl16(v) : rotl24(v);
}

// Rounds 1-2 of a unit, shared part: s = counter words 0..2 and word 3 of
// the unit's first counter; rk(i) = round-key word i as used in eq 26.
struct CtrShared {
    uint32_t u0, v0, v1, v2, v3;  // round 1 column 0 without its lane lookup; round 2 without theirs
};

template <class K>
__device__ __forceinline__ CtrShared ctr_shared(uint32_t w0, uint32_t w1, uint32_t w2, uint32_t w3, const K& rk)
{
    const uint32_t x0 = w0 ^ rk(0), x1 = w1 ^ rk(1), x2 = w2 ^ rk(2), x3 = w3 ^ rk(3);  // byte 15 of x3 unused
    CtrShared c;
    c.u0 = shared_lookup<0>(x0) ^ shared_lookup<1>(x1) ^ shared_lookup<2>(x2) ^ rk(4);
    const uint32_t u1 = shared_lookup<0>(x1) ^ shared_lookup<1>(x2) ^ shared_lookup<2>(x3) ^ shared_lookup<3>(x0) ^ rk(5);
    const uint32_t u2 = shared_lookup<0>(x2) ^ shared_lookup<1>(x3) ^ shared_lookup<2>(x0) ^ shared_lookup<3>(x1) ^ rk(6);
    const uint32_t u3 = shared_lookup<0>(x3) ^ shared_lookup<1>(x0) ^ shared_lookup<2>(x1) ^ shared_lookup<3>(x2) ^ rk(7);
    c.v0 = shared_lookup<1>(u1) ^ shared_lookup<2>(u2) ^ shared_lookup<3>(u3) ^ rk(8);
    c.v1 = shared_lookup<0>(u1) ^ shared_lookup<1>(u2) ^ shared_lookup<2>(u3) ^ rk(9);
    c.v2 = shared_lookup<0>(u2) ^ shared_lookup<1>(u3) ^ shared_lookup<3>(u1) ^ rk(10);
    c.v3 = shared_lookup<0>(u3) ^ shared_lookup<2>(u1) ^ shared_lookup<3>(u2) ^ rk(11);
    return c;
}

// Key-stream block of the lane whose counter has bytes 0..14 of the unit
// and top byte of word 3 equal to that of w3 (w3: the lane's state word 3).
template <int NR, int PL, class K>
__device__ __forceinline__ uint4 ctr_keystream(const CtrShared& c, uint32_t w3, const uint32_t* lds,
                                               const LaneBases<PL, false>& lb, uint32_t k3, const K& key)
{
    const uint32_t a = c.u0 ^ lane_lookup<PL, 3>(lds, lb, w3 ^ k3);  // round 1, column 0
    const uint4 s = make_uint4(c.v0 ^ lane_lookup<PL, 0>(lds, lb, a), c.v1 ^ lane_lookup<PL, 3>(lds, lb, a),
                               c.v2 ^ lane_lookup<PL, 2>(lds, lb, a), c.v3 ^ lane_lookup<PL, 1>(lds, lb, a));
    return crypt_rounds<NR, false, PL, 3>(s, lds, lb, key);
}

// One unit the fast path cannot take (the first, when the counters start
// inside a unit, and the last, partial one): lane by lane, with the whole
// cipher on each counter; a partial last block is read and written byte by
// byte and uses the leading bytes of its key-stream block.
template <int NR, int BPT, int PL, class K>
__device__ __forceinline__ void ctr_edge_unit(const uint4* __restrict__ in, uint4* __restrict__ out, uint64_t nbytes,
                                              const Counter128& c0, uint64_t u, uint32_t d, const uint32_t* lds,
                                              const LaneBases<PL, false>& lb, const K& key)
{
    const uint64_t span = 64u * BPT;
    const uint64_t nfull = nbytes / 16u, nblocks = (nbytes + 15u) / 16u;
    const uint32_t lane = threadIdx.x & 63u;
#pragma unroll
    for (int k = 0; k < BPT; ++k) {
        const uint64_t i = u * span + lane + 64u * k;  // counter offset from c0 - d
        if (i < d)
            continue;
        const uint64_t b = i - d;
        if (b < nfull) {
            store_block(out + b, xor4(in[b], crypt_block<NR, false, PL>(counter_state(c0, b), lds, lb, key)));
        } else if (b < nblocks) {
            const uint4 ks = crypt_block<NR, false, PL>(counter_state(c0, b), lds, lb, key);
            const uint32_t kw[4] = {ks.x, ks.y, ks.z, ks.w};
            const uint8_t* src = reinterpret_cast<const uint8_t*>(in) + 16u * b;
            uint8_t* dst = reinterpret_cast<uint8_t*>(out) + 16u * b;
            const uint32_t rem = static_cast<uint32_t>(nbytes - 16u * b);  // 1..15
            for (uint32_t t = 0; t < rem; ++t)
                dst[t] = static_cast<uint8_t>(src[t] ^ (kw[t >> 2] >> (8u * (t & 3u))));
        }
    }
}

// CTR over nbytes.  Counter of data block b: c0 + b.  With d = c0 mod span
// (span a power of two), block b belongs to unit (b + d) / span, and unit u
// holds the counters c0 - d + u * span + i, i < span, whose bytes 0..14 do
// not change.  Units 1 .. end_full - 1 (and unit 0 when d = 0) hold whole
// blocks only and take the cached path; the first unit (d > 0) and the last
// one (partial blocks) take ctr_edge_unit.
template <int NR, int BPT, int PL>
__global__ __launch_bounds__(1024) void ctr_kernel(const uint4* __restrict__ in, uint4* __restrict__ out,
                                                   uint64_t nbytes, Counter128 c0, RoundKeys rk)
{
    __shared__ __align__(16) uint32_t lds[Layout<PL, false>::words];
    const uint32_t lane = threadIdx.x & 63u;
    const uint64_t waves_per_grid = (uint64_t)gridDim.x * (blockDim.x >> 6);
    // uniform across the wave (made explicit, so the unit's counter and the
    // shared lookups live in scalar registers)
    const uint64_t wave_id =
        (uint64_t)blockIdx.x * (blockDim.x >> 6) + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    constexpr uint64_t span = 64u * BPT;
    const uint64_t nfull = nbytes / 16u;                  // whole blocks
    const uint64_t nblocks = (nbytes + 15u) / 16u;        // including a partial last block
    const uint32_t d = static_cast<uint32_t>(c0.lo & (span - 1u));
    const uint64_t first_full = d ? 1u : 0u;
    const uint64_t end_full = (nfull + d) / span;          // units [first_full, end_full) are whole
    const uint64_t n_units = (nblocks + d + span - 1u) / span;
    const uint64_t base_lo = c0.lo - d;                    // counter of unit 0, slot 0 (no borrow)
    uint64_t u = first_full + wave_id;
    // the data of the first unit is requested before the table fill
    uint4 cur[BPT];
    if (u < end_full) {
#pragma unroll
        for (int k = 0; k < BPT; ++k)
            cur[k] = in[u * span - d + lane + 64u * k];
    }
    fill_tables<PL, false>(lds, &c_tables);
    __syncthreads();
    const LaneBases<PL, false> lb(threadIdx.x);
    auto key = [&](int i) { return rk.w[i]; };
    // rounds 1-2 of the shared part need eq 26's keys as they are (the
    // 2-table kernels receive the inner-round words turned right by 8)
    auto key12 = [&](int i) { return (PL == kPlace2 && i >= 4) ? rotl8(rk.w[i]) : rk.w[i]; };
    for (; u < end_full; u += waves_per_grid) {
        const uint64_t first = u * span - d + lane;
        const uint64_t un = u + waves_per_grid;
        uint4 nxt[BPT];
        if (un < end_full) {
#pragma unroll
            for (int k = 0; k < BPT; ++k)
                nxt[k] = in[un * span - d + lane + 64u * k];
        }
        // counter of the unit's slot 0 (its low byte is a multiple of span)
        const uint64_t lo = base_lo + u * span;
        const uint64_t hi = c0.hi + (lo < base_lo ? 1u : 0u);
        const uint32_t w3 = __builtin_bswap32(static_cast<uint32_t>(lo));
        const CtrShared c = ctr_shared(__builtin_bswap32(static_cast<uint32_t>(hi >> 32)),
                                       __builtin_bswap32(static_cast<uint32_t>(hi)),
                                       __builtin_bswap32(static_cast<uint32_t>(lo >> 32)), w3, key12);
#pragma unroll
        for (int k = 0; k < BPT; ++k) {
            // slot lane + 64k: only byte 15 (bits 24..31 of word 3) moves, with no carry
            const uint32_t w3k = w3 + ((lane + 64u * k) << 24);
            store_block(out + first + 64u * k, xor4(cur[k], ctr_keystream<NR, PL>(c, w3k, lds, lb, rk.w[3], key)));
        }
#pragma unroll
        for (int k = 0; k < BPT; ++k)
            cur[k] = nxt[k];
    }
    // the edge units: the first (counters start inside it) on wave 0, the
    // last (holds the end of the data) on the grid's last wave
    if (d && wave_id == 0)
        ctr_edge_unit<NR, BPT, PL>(in, out, nbytes, c0, 0, d, lds, lb, key);
    const uint64_t back = first_full > end_full ? first_full : end_full;
    if (back < n_units && !(d && back == 0) && wave_id == waves_per_grid - 1)
        ctr_edge_unit<NR, BPT, PL>(in, out, nbytes, c0, back, d, lds, lb, key);
}

template <int NR, int BPT, int PL>
hipError_t launch_ctr_one(const void* in, void* out, uint64_t nbytes, const Counter128& c0, const RoundKeys& rk,
                          const LaunchShape& shape, int cus, hipStream_t stream)
{
    auto kern = ctr_kernel<NR, BPT, PL>;
    int grid = 0;
    hipError_t e = grid_for(reinterpret_cast<const void*>(kern), shape, cus, (nbytes + 15u) / 16u, &grid);
    if (e != hipSuccess)
        return e;
    hipLaunchKernelGGL(kern, dim3(grid), dim3(shape.wg), 0, stream, static_cast<const uint4*>(in),
                       static_cast<uint4*>(out), nbytes, c0, rk);
    return hipGetLastError();
}

template <int BPT, int PL>
hipError_t launch_ctr_nr(int nr, const void* in, void* out, uint64_t nbytes, const Counter128& c0,
                         const RoundKeys& rk, const LaunchShape& shape, int cus, hipStream_t stream)
{
    switch (nr) {
    case 10: return launch_ctr_one<10, BPT, PL>(in, out, nbytes, c0, rk, shape, cus, stream);
    case 12: return launch_ctr_one<12, BPT, PL>(in, out, nbytes, c0, rk, shape, cus, stream);
    case 14: return launch_ctr_one<14, BPT, PL>(in, out, nbytes, c0, rk, shape, cus, stream);
    default: return hipErrorInvalidValue;
    }
}

template <int PL>
hipError_t launch_ctr_bpt(int nr, const void* in, void* out, uint64_t nbytes, const Counter128& c0,
                          const RoundKeys& rk, const LaunchShape& shape, int cus, hipStream_t stream)
{
    switch (shape.bpt) {
    case 1: return launch_ctr_nr<1, PL>(nr, in, out, nbytes, c0, rk, shape, cus, stream);
    case 2: return launch_ctr_nr<2, PL>(nr, in, out, nbytes, c0, rk, shape, cus, stream);
    case 4: return launch_ctr_nr<4, PL>(nr, in, out, nbytes, c0, rk, shape, cus, stream);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_ctr(const LaunchShape& shape, int placement, int nr, const void* in, void* out, uint64_t nbytes,
                      const Counter128& c0, const RoundKeys& rk, int cus, hipStream_t stream)
{
    switch (placement) {
    case kPlace4: return launch_ctr_bpt<kPlace4>(nr, in, out, nbytes, c0, rk, shape, cus, stream);
    case kPlace2: return launch_ctr_bpt<kPlace2>(nr, in, out, nbytes, c0, inner_keys_rotr8(rk, nr), shape, cus, stream);
    case kPlace1: return launch_ctr_bpt<kPlace1>(nr, in, out, nbytes, c0, rk, shape, cus, stream);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace aesgpu
