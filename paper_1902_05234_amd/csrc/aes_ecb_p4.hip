// aes_ecb_p4.hip -- plain ECB kernels with the 4-table LDS placement.
#include "aes_ecb_kernel.hpp"

namespace aesgpu {

hipError_t launch_ecb_p4(const LaunchShape& shape, int nr, bool decrypt, const void* in, void* out,
                          uint64_t nblocks, const RoundKeys& rk, int cus, hipStream_t stream)
{
    return launch_placement<kPlace4>(shape, nr, decrypt, in, out, nblocks, rk, cus, stream);
}

}  // namespace aesgpu
