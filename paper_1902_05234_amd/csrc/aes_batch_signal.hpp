// aes_batch_signal.hpp -- the batched launch that reports its own completion
// (used by the serving engine).
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>

#include "aes_internal.hpp"

namespace aesgpu {

// launch_batch, and the launch's last workgroup to finish then stores `seq`
// into *done_word (host memory the device maps) with a system-scope release,
// after every workgroup's output stores are released at agent scope: a
// caller that polls the word sees the batch finished without an event query
// or a stream write behind the kernel.
hipError_t launch_batch_signal(const BatchArgs& args, int bpt, int placement, int grid, int wg, uint32_t* done_word,
                               uint32_t seq, hipStream_t stream);

}  // namespace aesgpu
