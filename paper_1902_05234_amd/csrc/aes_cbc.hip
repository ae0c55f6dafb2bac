// aes_cbc.hip -- CBC decryption on the ECB decryption core.
//
// CBC (section 3.1.2, eq 2, read with the block cipher: C_i = cipher(P_i
// XOR C_{i-1}), C_0 the initialisation vector) chains encryption, which the
// paper's Table 1 marks unsuitable for parallel work, but its inverse
// P_i = invcipher(C_i) XOR C_{i-1} needs only two ciphertext blocks per
// output block, so every block is independent again.  Each lane decrypts its
// block as in ECB and XORs the preceding ciphertext block, which it loads
// itself: that block is the neighbouring lane's input, so the second load
// hits the cache and HBM traffic stays 32 bytes per block.  Output may not
// alias the input (a lane would overwrite a block that another still reads).
#include "aes_ecb_kernel.hpp"

namespace aesgpu {

__device__ __forceinline__ uint4 xor4c(uint4 a, uint4 b) { return make_uint4(a.x ^ b.x, a.y ^ b.y, a.z ^ b.z, a.w ^ b.w); }

template <int NR, int BPT, int PL>
__global__ __launch_bounds__(1024) void cbc_dec_kernel(const uint4* __restrict__ in, uint4* __restrict__ out,
                                                       uint64_t nblocks, uint4 iv, RoundKeys rk)
{
    __shared__ __align__(16) uint32_t lds[Layout<PL, true>::words];
    fill_tables<PL, true>(lds, &c_tables);
    __syncthreads();
    const LaneBases<PL, true> lb(threadIdx.x);
    auto key = [&](int i) { return rk.w[i]; };
    // ciphertext block b - 1, or the initialisation vector for block 0 (the
    // load then reads block 0, which always exists, and is discarded)
    auto prev = [&](uint64_t b) {
        const uint4 c = in[b ? b - 1 : 0];
        return b ? c : iv;
    };

    const uint32_t lane = threadIdx.x & 63u;
    const uint64_t waves_per_grid = (uint64_t)gridDim.x * (blockDim.x >> 6);
    const uint64_t span = 64u * BPT;
    const uint64_t full_units = nblocks / span;
    uint64_t wv = (uint64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    uint4 cur[BPT], prv[BPT];
    if (wv < full_units) {
#pragma unroll
        for (int k = 0; k < BPT; ++k) {
            cur[k] = in[wv * span + lane + 64u * k];
            prv[k] = prev(wv * span + lane + 64u * k);
        }
    }
    for (; wv < full_units; wv += waves_per_grid) {
        const uint64_t first = wv * span + lane;
        const uint64_t wn = wv + waves_per_grid;
        uint4 nxt[BPT], nxp[BPT];
        if (wn < full_units) {
#pragma unroll
            for (int k = 0; k < BPT; ++k) {
                nxt[k] = in[wn * span + lane + 64u * k];
                nxp[k] = prev(wn * span + lane + 64u * k);
            }
        }
#pragma unroll
        for (int k = 0; k < BPT; ++k)
            store_block(out + first + 64u * k, xor4c(crypt_block<NR, true, PL>(cur[k], lds, lb, key), prv[k]));
#pragma unroll
        for (int k = 0; k < BPT; ++k) {
            cur[k] = nxt[k];
            prv[k] = nxp[k];
        }
    }
    if (wv == full_units && full_units * span < nblocks) {
#pragma unroll
        for (int k = 0; k < BPT; ++k) {
            const uint64_t b = wv * span + lane + 64u * k;
            if (b < nblocks)
                store_block(out + b, xor4c(crypt_block<NR, true, PL>(in[b], lds, lb, key), prev(b)));
        }
    }
}

template <int NR, int BPT, int PL>
hipError_t launch_cbc_one(const void* in, void* out, uint64_t nblocks, const uint4& iv, const RoundKeys& rk,
                          const LaunchShape& shape, int cus, hipStream_t stream)
{
    auto kern = cbc_dec_kernel<NR, BPT, PL>;
    int grid = 0;
    hipError_t e = grid_for(reinterpret_cast<const void*>(kern), shape, cus, nblocks, &grid);
    if (e != hipSuccess)
        return e;
    hipLaunchKernelGGL(kern, dim3(grid), dim3(shape.wg), 0, stream, static_cast<const uint4*>(in),
                       static_cast<uint4*>(out), nblocks, iv, rk);
    return hipGetLastError();
}

template <int BPT, int PL>
hipError_t launch_cbc_nr(int nr, const void* in, void* out, uint64_t nblocks, const uint4& iv, const RoundKeys& rk,
                         const LaunchShape& shape, int cus, hipStream_t stream)
{
    switch (nr) {
    case 10: return launch_cbc_one<10, BPT, PL>(in, out, nblocks, iv, rk, shape, cus, stream);
    case 12: return launch_cbc_one<12, BPT, PL>(in, out, nblocks, iv, rk, shape, cus, stream);
    case 14: return launch_cbc_one<14, BPT, PL>(in, out, nblocks, iv, rk, shape, cus, stream);
    default: return hipErrorInvalidValue;
    }
}

template <int PL>
hipError_t launch_cbc_bpt(int nr, const void* in, void* out, uint64_t nblocks, const uint4& iv, const RoundKeys& rk,
                          const LaunchShape& shape, int cus, hipStream_t stream)
{
    switch (shape.bpt) {
    case 1: return launch_cbc_nr<1, PL>(nr, in, out, nblocks, iv, rk, shape, cus, stream);
    case 2: return launch_cbc_nr<2, PL>(nr, in, out, nblocks, iv, rk, shape, cus, stream);
    case 4: return launch_cbc_nr<4, PL>(nr, in, out, nblocks, iv, rk, shape, cus, stream);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_cbc_decrypt(const LaunchShape& shape, int placement, int nr, const void* in, void* out,
                              uint64_t nblocks, const uint8_t iv_bytes[16], const RoundKeys& rk, int cus,
                              hipStream_t stream)
{
    uint32_t w[4];
    for (int c = 0; c < 4; ++c)
        w[c] = uint32_t(iv_bytes[4 * c]) | (uint32_t(iv_bytes[4 * c + 1]) << 8) |
               (uint32_t(iv_bytes[4 * c + 2]) << 16) | (uint32_t(iv_bytes[4 * c + 3]) << 24);
    const uint4 iv = make_uint4(w[0], w[1], w[2], w[3]);
    switch (placement) {
    case kPlace4: return launch_cbc_bpt<kPlace4>(nr, in, out, nblocks, iv, rk, shape, cus, stream);
    case kPlace2: return launch_cbc_bpt<kPlace2>(nr, in, out, nblocks, iv, inner_keys_rotr8(rk, nr), shape, cus, stream);
    case kPlace1: return launch_cbc_bpt<kPlace1>(nr, in, out, nblocks, iv, rk, shape, cus, stream);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace aesgpu
