// aes_cbc_msgs.hpp -- launchers of CBC encryption and decryption across
// independent messages (aes_cbc_msgs.hip), used by aes_cbc_encrypt_msgs and
// aes_cbc_decrypt_msgs.
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>

#include "aes_internal.hpp"

namespace aesgpu {

// CBC encryption of nmsgs independent messages (msgs: device array of
// aes_cbc_msg), one chain per lane; rk is the encryption schedule.  Messages
// whose ranges leave their arena (or whose reserved field is nonzero) are
// skipped and counted in *rejected if it is not null.  shape.bpt is the
// number of blocks a lane loads and stores at once (1, 2, 4, 8).
hipError_t launch_cbc_encrypt_msgs(const LaunchShape& shape, int placement, int nr, const void* msgs, uint64_t nmsgs,
                                   const void* in, uint64_t in_blocks, void* out, uint64_t out_blocks,
                                   uint32_t* rejected, const RoundKeys& rk, int cus, hipStream_t stream);

// CBC decryption of the same message sets: rk is the decryption schedule,
// shape.bpt the blocks a lane loads, decrypts and stores at once (1, 2, 4).
hipError_t launch_cbc_decrypt_msgs(const LaunchShape& shape, int placement, int nr, const void* msgs, uint64_t nmsgs,
                                   const void* in, uint64_t in_blocks, void* out, uint64_t out_blocks,
                                   uint32_t* rejected, const RoundKeys& rk, int cus, hipStream_t stream);

}  // namespace aesgpu
