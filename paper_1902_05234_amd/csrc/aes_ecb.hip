// aes_ecb.hip -- dispatch of the plain ECB kernels by table placement, and
// the plain device copy used as the memory reference.
#include <hip/hip_runtime.h>
#include <cstdint>

#include "aes_internal.hpp"

namespace aesgpu {

hipError_t launch_ecb_p4(const LaunchShape&, int, bool, const void*, void*, uint64_t, const RoundKeys&, int,
                         hipStream_t);
hipError_t launch_ecb_p2(const LaunchShape&, int, bool, const void*, void*, uint64_t, const RoundKeys&, int,
                         hipStream_t);
hipError_t launch_ecb_p1(const LaunchShape&, int, bool, const void*, void*, uint64_t, const RoundKeys&, int,
                         hipStream_t);

hipError_t launch_ecb_col(const LaunchShape&, int, int, bool, const void*, void*, uint64_t, const RoundKeys&, int,
                          hipStream_t);

hipError_t launch_ecb(const LaunchShape& shape, int placement, int nr, bool decrypt, const void* in, void* out,
                      uint64_t nblocks, const RoundKeys& rk, int cus, hipStream_t stream)
{
    if (shape.bpt == AES_BPT_COLUMN)
        return launch_ecb_col(shape, placement, nr, decrypt, in, out, nblocks, rk, cus, stream);
    switch (placement) {
    case 0: return launch_ecb_p4(shape, nr, decrypt, in, out, nblocks, rk, cus, stream);
    case 1: return launch_ecb_p2(shape, nr, decrypt, in, out, nblocks, rk, cus, stream);
    case 2: return launch_ecb_p1(shape, nr, decrypt, in, out, nblocks, rk, cus, stream);
    case 3: return launch_bitslice(shape, nr, decrypt, in, out, nblocks, rk, cus, stream);
    default: return hipErrorInvalidValue;
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

hipError_t launch_copy(const void* in, void* out, uint64_t n16, int grid, hipStream_t stream)
{
    hipLaunchKernelGGL(copy_kernel, dim3(grid), dim3(256), 0, stream, static_cast<const uint4*>(in),
                       static_cast<uint4*>(out), n16);
    return hipGetLastError();
}

}  // namespace aesgpu
