// aes_host_word.hpp -- a one-thread kernel that stores a sequence number into
// host memory the device maps (aes_host_word.hip), used by the host pipeline
// to see a launch finish without the runtime's completion wait.
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>

namespace aesgpu {

// Enqueue on `stream` a kernel whose one thread stores `seq` into *word with a
// system-scope release.  Stream order puts it after the work enqueued before
// it, so a host thread that reads `seq` from *word knows that work finished.
hipError_t launch_host_word(uint32_t* word, uint32_t seq, hipStream_t stream);

}  // namespace aesgpu
