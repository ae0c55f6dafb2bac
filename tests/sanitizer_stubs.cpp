// sanitizer_stubs.cpp -- stand-ins for the kernel launchers, so that the
// library's host-side sources (argument checks, key schedule, batch planner,
// serving engine, host pipeline) link into a host-only build with the
// address and undefined-behaviour sanitizers.  Every launch reports an error;
// the tests that run against that build never reach the device.
#include <hip/hip_runtime.h>

#include "aes_batch_signal.hpp"
#include "aes_cbc_msgs.hpp"
#include "aes_host_word.hpp"
#include "aes_internal.hpp"

namespace aesgpu {

hipError_t launch_ecb(const LaunchShape&, int, int, bool, const void*, void*, uint64_t, const RoundKeys&, int,
                      hipStream_t)
{
    return hipErrorInvalidValue;
}

hipError_t launch_copy(const void*, void*, uint64_t, int, hipStream_t) { return hipErrorInvalidValue; }

hipError_t launch_probe(int, uint32_t*, uint32_t, int, hipStream_t) { return hipErrorInvalidValue; }

hipError_t launch_bitslice(const LaunchShape&, int, bool, const void*, void*, uint64_t, const RoundKeys&, int,
                           hipStream_t)
{
    return hipErrorInvalidValue;
}

hipError_t launch_ctr(const LaunchShape&, int, int, const void*, void*, uint64_t, const Counter128&,
                      const RoundKeys&, int, hipStream_t)
{
    return hipErrorInvalidValue;
}

hipError_t launch_cbc_decrypt(const LaunchShape&, int, int, const void*, void*, uint64_t, const uint8_t*,
                              const RoundKeys&, int, hipStream_t)
{
    return hipErrorInvalidValue;
}

hipError_t launch_cbc_encrypt_msgs(const LaunchShape&, int, int, const void*, uint64_t, const void*, uint64_t, void*,
                                   uint64_t, uint32_t*, const RoundKeys&, int, hipStream_t)
{
    return hipErrorInvalidValue;
}

hipError_t launch_cbc_decrypt_msgs(const LaunchShape&, int, int, const void*, uint64_t, const void*, uint64_t, void*,
                                   uint64_t, uint32_t*, const RoundKeys&, int, hipStream_t)
{
    return hipErrorInvalidValue;
}

hipError_t launch_host_word(uint32_t*, uint32_t, hipStream_t) { return hipErrorInvalidValue; }

hipError_t launch_batch(const BatchArgs&, int, int, int, int, hipStream_t) { return hipErrorInvalidValue; }

hipError_t launch_batch_signal(const BatchArgs&, int, int, int, int, uint32_t*, uint32_t, hipStream_t)
{
    return hipErrorInvalidValue;
}

hipError_t batch_groups_per_cu(int, int, int, int*) { return hipErrorInvalidValue; }

hipError_t launch_batch_noalloc(BatchArgs, int, int, int, int, hipStream_t) { return hipErrorInvalidValue; }

void batch_grid(uint64_t, uint64_t, uint64_t, uint64_t, int, int max_grid, int, int* grid, int* enc_groups)
{
    *grid = max_grid;
    *enc_groups = 0;
}

}  // namespace aesgpu
