// aes_ecb_kernel.hpp -- the plain bulk ECB kernel template and its launcher.
//
// ECB (section 3.1.1, eq 1) encrypts every 16-byte block independently, so a
// buffer is one flat grid of independent states.  The grid is persistent:
// each workgroup fills the replicated T-tables into LDS once and then walks
// the buffer by wave units, so the table fill is paid once per workgroup.
//
// Template parameters:
//   NR   10 / 12 / 14 rounds (128- / 192- / 256-bit keys)
//   DEC  decryption (equivalent inverse cipher) instead of encryption
//   BPT  blocks per thread per unit: 1, 2, 4 (16, 32, 64 bytes per thread);
//        a wave covers 64*BPT consecutive blocks, lane l takes blocks l + 64k,
//        so every global_load/store_dwordx4 of a wave is one contiguous 1 KiB
//   PL   table placement in LDS (4, 2 or 1 tables; see aes_device.hpp)
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>

#include "aes_device.hpp"
#include "aes_internal.hpp"

namespace aesgpu {

template <int NR, bool kDecrypt, int BPT, int PL>
__global__ __launch_bounds__(1024) void ecb_kernel(const uint4* __restrict__ in, uint4* __restrict__ out,
                                                   uint64_t nblocks, RoundKeys rk)
{
    __shared__ __align__(16) uint32_t lds[Layout<PL, kDecrypt>::words];
    const uint32_t lane = threadIdx.x & 63u;
    const uint64_t waves_per_grid = (uint64_t)gridDim.x * (blockDim.x >> 6);
    const uint64_t span = 64u * BPT;
    const uint64_t full_units = nblocks / span;  // units whose BPT blocks all exist
    uint64_t wv = (uint64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    // Full units: the next unit's blocks are loaded before the current
    // unit's rounds, so HBM latency hides behind them; the first unit's
    // blocks are requested before the table fill, so their round trip
    // overlaps the fill's.  wv is uniform across the wave, so these branches
    // are scalar and the loads unpredicated.
    uint4 cur[BPT];
    if (wv < full_units) {
#pragma unroll
        for (int k = 0; k < BPT; ++k)
            cur[k] = in[wv * span + lane + 64u * k];
    }
    fill_tables<PL, kDecrypt>(lds, &c_tables);
    __syncthreads();
    const LaneBases<PL, kDecrypt> lb(threadIdx.x);
    auto key = [&](int i) { return rk.w[i]; };
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
            cur[k] = crypt_block<NR, kDecrypt, PL>(cur[k], lds, lb, key);
#pragma unroll
        for (int k = 0; k < BPT; ++k)
            store_block(out + first + 64u * k, cur[k]);
#pragma unroll
        for (int k = 0; k < BPT; ++k)
            cur[k] = nxt[k];
    }
    // The one ragged unit at the end (if any) belongs to the wave whose
    // sequence reaches index full_units; its missing blocks are skipped.
    if (wv == full_units && full_units * span < nblocks) {
#pragma unroll
        for (int k = 0; k < BPT; ++k) {
            const uint64_t b = wv * span + lane + 64u * k;
            if (b < nblocks)
                store_block(out + b, crypt_block<NR, kDecrypt, PL>(in[b], lds, lb, key));
        }
    }
}

// Workgroups of a launch of kern over nblocks: shape.grid if set, else
// persistent (as many as fit on every CU at once, given LDS and registers),
// never more than the blocks can keep busy.
inline hipError_t grid_for(const void* kern, const LaunchShape& shape, int cus, uint64_t nblocks, int* grid_out)
{
    int grid = shape.grid;
    if (grid <= 0) {
        int per_cu = 0;
        hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, shape.wg, 0);
        if (e != hipSuccess)
            return e;
        grid = cus * (per_cu > 0 ? per_cu : 1);
    }
    const uint64_t per_group = (uint64_t)shape.wg * shape.bpt;
    const uint64_t needed = (nblocks + per_group - 1) / per_group;
    if ((uint64_t)grid > needed)
        grid = (int)needed;
    *grid_out = grid;
    return hipSuccess;
}

template <int NR, bool kDecrypt, int BPT, int PL>
hipError_t launch_one(const void* in, void* out, uint64_t nblocks, const RoundKeys& rk, const LaunchShape& shape,
                      int cus, hipStream_t stream)
{
    auto kern = ecb_kernel<NR, kDecrypt, BPT, PL>;
    int grid = 0;
    hipError_t e = grid_for(reinterpret_cast<const void*>(kern), shape, cus, nblocks, &grid);
    if (e != hipSuccess)
        return e;
    hipLaunchKernelGGL(kern, dim3(grid), dim3(shape.wg), 0, stream, static_cast<const uint4*>(in),
                       static_cast<uint4*>(out), nblocks, rk);
    return hipGetLastError();
}

template <bool kDecrypt, int BPT, int PL>
hipError_t launch_nr(int nr, const void* in, void* out, uint64_t nblocks, const RoundKeys& rk,
                     const LaunchShape& shape, int cus, hipStream_t stream)
{
    switch (nr) {
    case 10: return launch_one<10, kDecrypt, BPT, PL>(in, out, nblocks, rk, shape, cus, stream);
    case 12: return launch_one<12, kDecrypt, BPT, PL>(in, out, nblocks, rk, shape, cus, stream);
    case 14: return launch_one<14, kDecrypt, BPT, PL>(in, out, nblocks, rk, shape, cus, stream);
    default: return hipErrorInvalidValue;
    }
}

template <bool kDecrypt, int PL>
hipError_t launch_bpt(int nr, const void* in, void* out, uint64_t nblocks, const RoundKeys& rk,
                      const LaunchShape& shape, int cus, hipStream_t stream)
{
    switch (shape.bpt) {
    case 1: return launch_nr<kDecrypt, 1, PL>(nr, in, out, nblocks, rk, shape, cus, stream);
    case 2: return launch_nr<kDecrypt, 2, PL>(nr, in, out, nblocks, rk, shape, cus, stream);
    case 4: return launch_nr<kDecrypt, 4, PL>(nr, in, out, nblocks, rk, shape, cus, stream);
    default: return hipErrorInvalidValue;
    }
}

template <int PL>
hipError_t launch_placement(const LaunchShape& shape, int nr, bool decrypt, const void* in, void* out,
                            uint64_t nblocks, const RoundKeys& rk, int cus, hipStream_t stream)
{
    const RoundKeys k = PL == kPlace2 ? inner_keys_rotr8(rk, nr) : rk;
    if (decrypt)
        return launch_bpt<true, PL>(nr, in, out, nblocks, k, shape, cus, stream);
    return launch_bpt<false, PL>(nr, in, out, nblocks, k, shape, cus, stream);
}

}  // namespace aesgpu
