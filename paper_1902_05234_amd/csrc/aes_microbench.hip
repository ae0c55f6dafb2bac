// aes_microbench.hip -- the roofs the cipher kernels are measured against.
//
// Two probes complete the copy kernel (aes_ecb.hip):
//   lds_probe   conflict-free ds_read_b32 lookups with per-lane pseudo-random
//               entries in a 32-replica table laid out like the T-tables
//               (entry e, half h, replica r at e*256 + h*128 + r*4), 16
//               independent lookups per wave between waits, two 1024-thread
//               workgroups (32 waves) per CU: the lookup rate the cipher's
//               binding unit can deliver.
//   valu_probe  16 independent chains of full-rate v_bitop3_b32 per lane,
//               32 waves per CU: the integer VALU rate.
// Both write one word per thread so that nothing is optimised away.
#include <hip/hip_runtime.h>
#include <cstdint>

#include "aes_internal.hpp"

namespace aesgpu {

constexpr uint32_t kProbeLdsWords = 16384;  // 64 KiB

__device__ __forceinline__ uint32_t probe_hash(uint32_t x)
{
    x ^= x >> 16;
    x *= 0x7feb352du;
    x ^= x >> 15;
    x *= 0x846ca68bu;
    x ^= x >> 16;
    return x;
}

__global__ __launch_bounds__(1024) void lds_probe(uint32_t* __restrict__ out, uint32_t iters)
{
    __shared__ uint32_t lds[kProbeLdsWords];
    for (uint32_t i = threadIdx.x; i < kProbeLdsWords; i += blockDim.x)
        lds[i] = probe_hash(i);
    __syncthreads();
    const uint32_t lane = threadIdx.x & 63u;
    const uint32_t salt = blockIdx.x * 977u + (threadIdx.x >> 6) * 31u;
    uint32_t a[16];
#pragma unroll
    for (int k = 0; k < 16; ++k) {
        const uint32_t e = probe_hash(lane * 131u + k * 7919u + salt) & 255u;
        a[k] = e * 256u + ((uint32_t)k & 1u) * 128u + (lane & 31u) * 4u;  // < 64 KiB
    }
    uint32_t acc = 0;
    for (uint32_t it = 0; it < iters; ++it) {
        uint32_t r[16];
#pragma unroll
        for (int k = 0; k < 16; ++k)
            asm volatile("ds_read_b32 %0, %1" : "=v"(r[k]) : "v"(a[k]));
        // the results are tied to the wait, so no use of them can move above it
        asm volatile("s_waitcnt lgkmcnt(0)"
                     : "+v"(r[0]), "+v"(r[1]), "+v"(r[2]), "+v"(r[3]), "+v"(r[4]), "+v"(r[5]), "+v"(r[6]),
                       "+v"(r[7]), "+v"(r[8]), "+v"(r[9]), "+v"(r[10]), "+v"(r[11]), "+v"(r[12]), "+v"(r[13]),
                       "+v"(r[14]), "+v"(r[15])
                     :
                     : "memory");
#pragma unroll
        for (int k = 0; k < 16; k += 2)
            acc = __builtin_amdgcn_bitop3_b32(acc, r[k], r[k + 1], 0x96);
    }
    out[blockIdx.x * blockDim.x + threadIdx.x] = acc;
}

__global__ __launch_bounds__(1024) void valu_probe(uint32_t* __restrict__ out, uint32_t iters)
{
    uint32_t x[16];
#pragma unroll
    for (int k = 0; k < 16; ++k)
        x[k] = threadIdx.x * (k + 1) + blockIdx.x;
    uint32_t m = 0x5a5a5a5au ^ threadIdx.x;
    for (uint32_t it = 0; it < iters; ++it) {
#pragma unroll
        for (int k = 0; k < 16; ++k)
            asm volatile("v_bitop3_b32 %0, %0, %1, %2 bitop3:0x96" : "+v"(x[k]) : "v"(x[(k + 1) & 15]), "v"(m));
    }
    uint32_t acc = 0;
#pragma unroll
    for (int k = 0; k < 16; ++k)
        acc ^= x[k];
    out[blockIdx.x * blockDim.x + threadIdx.x] = acc;
}

// grid = cus * 2 workgroups of 1024 threads; out holds one word per thread
hipError_t launch_probe(int which, uint32_t* out, uint32_t iters, int cus, hipStream_t stream)
{
    const dim3 grid(cus * 2), block(1024);
    if (which == 0)
        hipLaunchKernelGGL(lds_probe, grid, block, 0, stream, out, iters);
    else
        hipLaunchKernelGGL(valu_probe, grid, block, 0, stream, out, iters);
    return hipGetLastError();
}

}  // namespace aesgpu
