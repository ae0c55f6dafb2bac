// aes_ecb.hip -- plain bulk ECB kernels for gfx950.
//
// ECB (section 3.1.1, eq 1) encrypts every 16-byte block independently, so a
// buffer is one flat grid of independent states.  The grid is persistent:
// one workgroup per CU fills the replicated T-tables into LDS once (about
// 128-160 KiB) and then strides over the buffer, so the table fill is paid
// 256 times per launch rather than once per block group.
//
// Variants (template parameters):
//   NR   10 / 12 / 14 rounds (128- / 192- / 256-bit keys)
//   BPT  blocks per thread per iteration: 1, 2, 4 (16, 32, 64 bytes per thread);
//        a wave covers 64*BPT consecutive blocks, lane l takes blocks l + 64k,
//        so every global_load/store_dwordx4 of a wave is one contiguous 1 KiB.
#include <hip/hip_runtime.h>
#include <cstdint>

#include "aes_device.hpp"
#include "aes_internal.hpp"

namespace aesgpu {

template <int NR, bool kDecrypt, int BPT>
__global__ __launch_bounds__(1024) void ecb_kernel(const uint4* __restrict__ in, uint4* __restrict__ out,
                                                   uint64_t nblocks, RoundKeys rk)
{
    __shared__ uint32_t lds[kDecrypt ? kDecLdsWords : kEncLdsWords];
    fill_tables<kDecrypt>(lds, &c_tables);
    __syncthreads();
    const LaneBases lb(threadIdx.x);
    auto key = [&](int i) { return rk.w[i]; };

    const uint32_t lane = threadIdx.x & 63u;
    const uint64_t waves_per_grid = (uint64_t)gridDim.x * (blockDim.x >> 6);
    const uint64_t span = 64u * BPT;
    uint64_t wv = (uint64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    // The next unit's blocks are loaded before the current unit is
    // encrypted, so the HBM latency of one unit hides behind the rounds of
    // the previous one.  Blocks past the end are neither loaded nor stored.
    uint4 cur[BPT];
#pragma unroll
    for (int k = 0; k < BPT; ++k) {
        const uint64_t b = wv * span + lane + 64u * k;
        cur[k] = b < nblocks ? in[b] : make_uint4(0, 0, 0, 0);
    }
    while (wv * span < nblocks) {
        const uint64_t first = wv * span + lane;
        const uint64_t wn = wv + waves_per_grid;
        uint4 nxt[BPT];
#pragma unroll
        for (int k = 0; k < BPT; ++k) {
            const uint64_t b = wn * span + lane + 64u * k;
            nxt[k] = b < nblocks ? in[b] : make_uint4(0, 0, 0, 0);
        }
#pragma unroll
        for (int k = 0; k < BPT; ++k)
            cur[k] = crypt_block<NR, kDecrypt>(cur[k], lds, lb, key);
#pragma unroll
        for (int k = 0; k < BPT; ++k)
            if (first + 64u * k < nblocks)
                out[first + 64u * k] = cur[k];
#pragma unroll
        for (int k = 0; k < BPT; ++k)
            cur[k] = nxt[k];
        wv = wn;
    }
}

// Plain device copy, used to calibrate HBM traffic counters and as the
// memory roof of the same launch shape.
__global__ __launch_bounds__(256) void copy_kernel(const uint4* __restrict__ in, uint4* __restrict__ out, uint64_t n)
{
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
        out[i] = in[i];
}

template <int NR, bool kDecrypt, int BPT>
static hipError_t launch_one(const void* in, void* out, uint64_t nblocks, const RoundKeys& rk, int grid, int wg,
                             hipStream_t stream)
{
    hipLaunchKernelGGL((ecb_kernel<NR, kDecrypt, BPT>), dim3(grid), dim3(wg), 0, stream,
                       static_cast<const uint4*>(in), static_cast<uint4*>(out), nblocks, rk);
    return hipGetLastError();
}

template <bool kDecrypt, int BPT>
static hipError_t launch_nr(int nr, const void* in, void* out, uint64_t nblocks, const RoundKeys& rk, int grid,
                            int wg, hipStream_t stream)
{
    switch (nr) {
    case 10: return launch_one<10, kDecrypt, BPT>(in, out, nblocks, rk, grid, wg, stream);
    case 12: return launch_one<12, kDecrypt, BPT>(in, out, nblocks, rk, grid, wg, stream);
    case 14: return launch_one<14, kDecrypt, BPT>(in, out, nblocks, rk, grid, wg, stream);
    default: return hipErrorInvalidValue;
    }
}

template <bool kDecrypt>
static hipError_t launch_bpt(int bpt, int nr, const void* in, void* out, uint64_t nblocks, const RoundKeys& rk,
                             int grid, int wg, hipStream_t stream)
{
    switch (bpt) {
    case 1: return launch_nr<kDecrypt, 1>(nr, in, out, nblocks, rk, grid, wg, stream);
    case 2: return launch_nr<kDecrypt, 2>(nr, in, out, nblocks, rk, grid, wg, stream);
    case 4: return launch_nr<kDecrypt, 4>(nr, in, out, nblocks, rk, grid, wg, stream);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_ecb(const LaunchShape& shape, int nr, bool decrypt, const void* in, void* out, uint64_t nblocks,
                      const RoundKeys& rk, hipStream_t stream)
{
    if (decrypt)
        return launch_bpt<true>(shape.bpt, nr, in, out, nblocks, rk, shape.grid, shape.wg, stream);
    return launch_bpt<false>(shape.bpt, nr, in, out, nblocks, rk, shape.grid, shape.wg, stream);
}

hipError_t launch_copy(const void* in, void* out, uint64_t n16, int grid, hipStream_t stream)
{
    hipLaunchKernelGGL(copy_kernel, dim3(grid), dim3(256), 0, stream, static_cast<const uint4*>(in),
                       static_cast<uint4*>(out), n16);
    return hipGetLastError();
}

}  // namespace aesgpu
