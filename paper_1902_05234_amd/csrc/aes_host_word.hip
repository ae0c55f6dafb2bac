// aes_host_word.hip -- completion word for the host pipeline.
//
// A host thread that waits for a launch through the runtime (an event or a
// stream synchronisation) sees it end about 5 us later than a word the
// device writes into mapped host memory right after it (measured on MI355X:
// a launch followed by a wait, 11.3 us; followed by polling a word written
// by the next kernel on the stream, 5.9 us).  The preceding kernel's own end
// of launch makes its stores visible before this kernel starts, and this
// kernel's store is a system-scope release, so the word is seen after them.
#include "aes_host_word.hpp"

namespace aesgpu {

namespace {

__global__ void host_word_kernel(uint32_t* word, uint32_t seq)
{
    if (threadIdx.x == 0)
        __hip_atomic_store(word, seq, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
}

}  // namespace

hipError_t launch_host_word(uint32_t* word, uint32_t seq, hipStream_t stream)
{
    if (word == nullptr)
        return hipErrorInvalidValue;
    hipLaunchKernelGGL(host_word_kernel, dim3(1), dim3(64), 0, stream, word, seq);
    return hipGetLastError();
}

}  // namespace aesgpu
