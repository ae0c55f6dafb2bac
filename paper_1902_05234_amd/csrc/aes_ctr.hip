// aes_ctr.hip -- counter mode on the same round core as ECB.
//
// CTR (section 3.1.5, eq 5; marked parallel in Table 1): data block j is
// XORed with the cipher of a counter block, and counter blocks of successive
// data blocks are successive 128-bit big-endian integers c0 + j (mod 2^128),
// so every block is independent, as in ECB.  Each lane builds its counter
// block from the block index (no memory read), runs the encryption rounds
// and XORs the result into the data it loaded: the same 32 bytes of HBM per
// block and the same LDS lookups as an ECB encryption.  Decryption is the
// same operation.  A partial last block is read and written byte by byte and
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

template <int NR, int BPT, int PL>
__global__ __launch_bounds__(1024) void ctr_kernel(const uint4* __restrict__ in, uint4* __restrict__ out,
                                                   uint64_t nbytes, Counter128 c0, RoundKeys rk)
{
    __shared__ uint32_t lds[Layout<PL, false>::words];
    fill_tables<PL, false>(lds, &c_tables);
    __syncthreads();
    const LaneBases<PL, false> lb(threadIdx.x);
    auto key = [&](int i) { return rk.w[i]; };

    const uint32_t lane = threadIdx.x & 63u;
    const uint64_t waves_per_grid = (uint64_t)gridDim.x * (blockDim.x >> 6);
    const uint64_t span = 64u * BPT;
    const uint64_t nfull = nbytes / 16u;                 // whole blocks
    const uint64_t nblocks = (nbytes + 15u) / 16u;       // including a partial last block
    const uint64_t full_units = nfull / span;
    uint64_t wv = (uint64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    // Same walk as the ECB kernel: full units with the next unit's data
    // loaded ahead, then one ragged unit.
    uint4 cur[BPT];
    if (wv < full_units) {
#pragma unroll
        for (int k = 0; k < BPT; ++k)
            cur[k] = in[wv * span + lane + 64u * k];
    }
    for (; wv < full_units; wv += waves_per_grid) {
        const uint64_t first = wv * span + lane;
        const uint64_t wn = wv + waves_per_grid;
        uint4 nxt[BPT];
        if (wn < full_units) {
#pragma unroll
            for (int k = 0; k < BPT; ++k)
                nxt[k] = in[wn * span + lane + 64u * k];
        }
#pragma unroll
        for (int k = 0; k < BPT; ++k)
            out[first + 64u * k] = xor4(cur[k], crypt_block<NR, false, PL>(counter_state(c0, first + 64u * k), lds, lb, key));
#pragma unroll
        for (int k = 0; k < BPT; ++k)
            cur[k] = nxt[k];
    }
    if (wv == full_units && full_units * span < nblocks) {
#pragma unroll
        for (int k = 0; k < BPT; ++k) {
            const uint64_t b = wv * span + lane + 64u * k;
            if (b < nfull) {
                out[b] = xor4(in[b], crypt_block<NR, false, PL>(counter_state(c0, b), lds, lb, key));
            } else if (b < nblocks) {
                const uint4 ks = crypt_block<NR, false, PL>(counter_state(c0, b), lds, lb, key);
                const uint32_t kw[4] = {ks.x, ks.y, ks.z, ks.w};
                const uint8_t* src = reinterpret_cast<const uint8_t*>(in) + 16u * b;
                uint8_t* dst = reinterpret_cast<uint8_t*>(out) + 16u * b;
                const uint32_t rem = static_cast<uint32_t>(nbytes - 16u * b);  // 1..15
                for (uint32_t i = 0; i < rem; ++i)
                    dst[i] = static_cast<uint8_t>(src[i] ^ (kw[i >> 2] >> (8u * (i & 3u))));
            }
        }
    }
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
