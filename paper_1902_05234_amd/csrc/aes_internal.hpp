// aes_internal.hpp -- declarations shared by the library's translation units.
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>
#include <exception>
#include <new>

#include "../../include/aesgpu.h"

namespace aesgpu {

// Round keys passed by value in the kernel argument block; the kernels read
// them as uniform values (scalar registers).
struct RoundKeys {
    uint32_t w[60];
};

// The 2-table kernels add an inner round's key to the two lookups that are
// rotated left by 8 bits afterwards, so they take words 4 .. 4*nr-1 of the
// schedule rotated right by 8 bits; the first and last round keys are as is.
inline RoundKeys inner_keys_rotr8(const RoundKeys& rk, int nr)
{
    RoundKeys r = rk;
    for (int i = 4; i < 4 * nr && i < 60; ++i)
        r.w[i] = (r.w[i] >> 8) | (r.w[i] << 24);
    return r;
}

struct LaunchShape {
    int bpt;   // blocks per thread per iteration: 1, 2, 4
    int wg;    // workgroup size (multiple of 64, at most 1024)
    int grid;  // number of workgroups; 0 = persistent (CUs x workgroups that fit per CU)
};

// placement: 0 = four tables, 1 = two tables, 2 = one table (aes_device.hpp)
hipError_t launch_ecb(const LaunchShape& shape, int placement, int nr, bool decrypt, const void* in, void* out,
                      uint64_t nblocks, const RoundKeys& rk, int cus, hipStream_t stream);

hipError_t launch_copy(const void* in, void* out, uint64_t n16, int grid, hipStream_t stream);

// Roofline probes (aes_microbench.hip): which 0 = LDS lookups, 1 = VALU;
// cus * 2 workgroups of 1024 threads, one output word per thread.
hipError_t launch_probe(int which, uint32_t* out, uint32_t iters, int cus, hipStream_t stream);

// Bitsliced placement (no tables): 32 blocks per lane, workgroups of at most
// kBitsliceMaxWg threads (the slices take most of the register file).
constexpr int kBitsliceMaxWg = 256;
hipError_t launch_bitslice(const LaunchShape& shape, int nr, bool decrypt, const void* in, void* out,
                           uint64_t nblocks, const RoundKeys& rk, int cus, hipStream_t stream);

// A 128-bit big-endian counter block as two host integers (hi = bytes 0..7).
struct Counter128 {
    uint64_t hi;
    uint64_t lo;
};

// CTR over nbytes (any length): data block j is XORed with the cipher of
// counter c0 + j (mod 2^128).  rk is the encryption schedule.
hipError_t launch_ctr(const LaunchShape& shape, int placement, int nr, const void* in, void* out, uint64_t nbytes,
                      const Counter128& c0, const RoundKeys& rk, int cus, hipStream_t stream);

// CBC decryption of nblocks: block b is invcipher(in[b]) XOR in[b - 1]
// (iv for block 0).  rk is the decryption schedule; out must not alias in.
hipError_t launch_cbc_decrypt(const LaunchShape& shape, int placement, int nr, const void* in, void* out,
                              uint64_t nblocks, const uint8_t iv[16], const RoundKeys& rk, int cus,
                              hipStream_t stream);

// Work item of the batched kernel: one wave-sized chunk of one message.
struct WorkItem {
    uint64_t in_block;
    uint64_t out_block;
    uint32_t nblocks;
    uint32_t key_slot;
};

struct BatchArgs {
    const WorkItem* items;
    uint32_t n_enc;        // items [0, n_enc) encrypt
    uint32_t n_dec;        // items [n_enc, n_enc + n_dec) decrypt
    const uint32_t* key_table;
    uint32_t n_slots;
    const void* in_base;
    void* out_base;
    uint64_t in_blocks;    // arena sizes, for the per-item bounds check
    uint64_t out_blocks;
    uint32_t* counters;    // [0] next enc item, [1] next dec item, [2] finished groups, [3] rejected items
    uint32_t enc_groups;   // workgroups that start on the encryption list
};

// placement: kPlace4 / kPlace2 / kPlace1 (the table placements of the plain kernel)
hipError_t launch_batch(const BatchArgs& args, int bpt, int placement, int grid, int wg, hipStream_t stream);

// launch_batch with the claim counters in the library's per-device scratch
// array (args.counters is ignored), zeroed by a kernel on `stream` first.
hipError_t launch_batch_noalloc(BatchArgs args, int bpt, int placement, int grid, int wg, hipStream_t stream);

// Device address of the per-device scratch array (hipGetSymbolAddress on the
// current device's first call).
hipError_t noalloc_scratch(uint32_t** out);

// Workgroups of the batch kernel variant (bpt, placement, wg) that fit on one
// CU at once (LDS and registers); cached per variant after the first query.
hipError_t batch_groups_per_cu(int bpt, int placement, int wg, int* per_cu);

// Grid of a batch launch: at most max_grid workgroups, no more than the
// items can keep busy, at least one per non-empty direction; enc_groups is
// the requested split (< 0: by block share) clamped to that.
void batch_grid(uint64_t n_enc, uint64_t n_dec, uint64_t enc_blocks, uint64_t total_blocks, int wg, int max_grid,
                int requested_enc_groups, int* grid, int* enc_groups);

// [p, p + n) lies inside one page-locked host allocation that the current
// device maps at the same address, so kernels may read and write it
// (aes_pipe.cpp).
bool host_range_device_mapped(const void* p, uint64_t n);

// Number of compute units of the current device (cached per device).
int device_cu_count();

// Record the message of a failure for aes_last_error() (calling thread) and
// return code; fail_hip formats a HIP error.
int fail(int code, const char* fmt, ...);
int fail_hip(hipError_t e, const char* what);

// Run an entry point's body and turn a C++ exception (a failed host
// allocation, a thread that cannot be started) into a status code, so that
// no exception crosses the C boundary.
template <class F>
int guarded(F&& body) noexcept
{
    try {
        return body();
    } catch (const std::bad_alloc&) {
        return fail(AES_ENOMEM, "out of host memory");
    } catch (const std::exception& e) {
        return fail(AES_EHIP, "internal error: %s", e.what());
    } catch (...) {
        return fail(AES_EHIP, "internal error");
    }
}

}  // namespace aesgpu
