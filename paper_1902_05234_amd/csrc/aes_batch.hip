// aes_batch.hip -- one persistent launch over many independent ECB messages.
//
// The host splits every message into work items of at most `chunk` blocks
// (aes_batch_plan) and lists all encryption items before all decryption
// items.  Each wave claims one item at a time with an atomic counter, loads
// that item's round keys as uniform values, and runs the same round core as
// the plain kernel for the item's key size.
//
// LDS holds the tables of one direction only (4 tables: 128 KiB + 32 KiB of
// InvS; 2 tables: 64 + 8 KiB; 1 table: 32 + 8 KiB), so the workgroups are
// split by role: the first `enc_groups` start on the encryption list, the
// others on the decryption list; when a list runs dry a workgroup reloads
// LDS with the other direction's tables and helps drain the other list.  The
// last workgroup to finish resets the claim counters, so a captured graph can
// replay the launch with no separate reset node.  The table placement and the
// workgroup size are the same design axes as in the plain kernel (section
// 4.2 keeps the tables in shared memory; the placements trade LDS size, and
// so resident waves, against VALU work).
//
// Every item is checked against the arena sizes, the key-table size and the
// largest item size before use; a bad item is skipped and counted in
// counters[3].  For the serving engine the last workgroup also writes a
// completion word in host memory (launch_batch_signal).
#include <hip/hip_runtime.h>
#include <algorithm>
#include <atomic>
#include <cstdint>
#include <mutex>

#include "aes_batch_signal.hpp"
#include "aes_device.hpp"
#include "aes_internal.hpp"

namespace aesgpu {

constexpr int kSlotWords = 128;  // rk_enc at 0, rk_dec at 64, Nr at 124
constexpr int kSlotNr = 124;

template <int NR, bool kDecrypt, int BPT, int PL>
__device__ __forceinline__ void run_item(const uint4* __restrict__ in, uint4* __restrict__ out, uint32_t nblocks,
                                         const uint32_t* lds, const LaneBases<PL, kDecrypt>& lb,
                                         const uint32_t* __restrict__ kp)
{
    uint32_t k[4 * (NR + 1)];
#pragma unroll
    for (int i = 0; i < 4 * (NR + 1); ++i) {
        k[i] = __builtin_amdgcn_readfirstlane(kp[i]);
        // the 2-table round takes inner-round key words turned right by 8
        // bits (see crypt_rounds); taken back to a scalar register, else the
        // turned words stay in VGPRs and the 64-VGPR build spills
        if (PL == kPlace2 && i >= 4 && i < 4 * NR)
            k[i] = __builtin_amdgcn_readfirstlane((k[i] >> 8) | (k[i] << 24));
    }
    auto key = [&](int i) { return k[i]; };
    const uint32_t lane = threadIdx.x & 63u;
    // Whole units first, then the ragged one: every index stays below
    // nblocks + 64*BPT, so no 32-bit sum wraps.
    const uint32_t span = 64u * BPT;
    const uint32_t full = nblocks / span;
    for (uint32_t u = 0; u < full; ++u) {
        const uint32_t first = u * span + lane;
        uint4 x[BPT];
#pragma unroll
        for (int j = 0; j < BPT; ++j)
            x[j] = in[first + 64u * j];
#pragma unroll
        for (int j = 0; j < BPT; ++j)
            x[j] = crypt_block<NR, kDecrypt, PL>(x[j], lds, lb, key);
#pragma unroll
        for (int j = 0; j < BPT; ++j)
            store_block(out + first + 64u * j, x[j]);
    }
    const uint32_t b0 = full * span;
    if (b0 < nblocks) {
#pragma unroll
        for (int j = 0; j < BPT; ++j) {
            const uint32_t b = b0 + lane + 64u * j;
            if (b < nblocks)
                store_block(out + b, crypt_block<NR, kDecrypt, PL>(in[b], lds, lb, key));
        }
    }
}

template <bool kDecrypt, int BPT, int PL>
__device__ __forceinline__ void drain(const WorkItem* __restrict__ items, uint32_t first_item, uint32_t n_items,
                                      const uint32_t* __restrict__ key_table, uint32_t n_slots,
                                      const uint4* __restrict__ in_base, uint4* __restrict__ out_base,
                                      uint64_t in_blocks, uint64_t out_blocks, uint32_t* counters,
                                      const uint32_t* lds)
{
    const uint32_t lane = threadIdx.x & 63u;
    const LaneBases<PL, kDecrypt> lb(threadIdx.x);
    for (;;) {
        uint32_t idx = 0;
        if (lane == 0)
            idx = atomicAdd(&counters[kDecrypt ? 1 : 0], 1u);
        idx = __builtin_amdgcn_readfirstlane(idx);
        if (idx >= n_items)
            break;
        const WorkItem it = items[first_item + idx];
        const uint64_t in_b = __builtin_amdgcn_readfirstlane((uint32_t)it.in_block) |
                              ((uint64_t)__builtin_amdgcn_readfirstlane((uint32_t)(it.in_block >> 32)) << 32);
        const uint64_t out_b = __builtin_amdgcn_readfirstlane((uint32_t)it.out_block) |
                               ((uint64_t)__builtin_amdgcn_readfirstlane((uint32_t)(it.out_block >> 32)) << 32);
        const uint32_t nb = __builtin_amdgcn_readfirstlane(it.nblocks);
        const uint32_t slot = __builtin_amdgcn_readfirstlane(it.key_slot);
        const bool ok = slot < n_slots && nb <= AES_MAX_ITEM_BLOCKS && in_b <= in_blocks && nb <= in_blocks - in_b &&
                        out_b <= out_blocks && nb <= out_blocks - out_b;
        const uint32_t* kp = key_table + (uint64_t)(ok ? slot : 0u) * kSlotWords;
        const int nr = ok ? (int)__builtin_amdgcn_readfirstlane(kp[kSlotNr]) : 0;
        const uint32_t* kd = kp + (kDecrypt ? 64 : 0);
        switch (nr) {
        case 10: run_item<10, kDecrypt, BPT, PL>(in_base + in_b, out_base + out_b, nb, lds, lb, kd); break;
        case 12: run_item<12, kDecrypt, BPT, PL>(in_base + in_b, out_base + out_b, nb, lds, lb, kd); break;
        case 14: run_item<14, kDecrypt, BPT, PL>(in_base + in_b, out_base + out_b, nb, lds, lb, kd); break;
        default:
            if (lane == 0)
                atomicAdd(&counters[3], 1u);
            break;
        }
    }
}

// The 2- and 1-table kernels are built for 8 waves per SIMD (at most 64
// VGPRs), so two 1024-thread workgroups share a CU, as in the plain kernel.
template <int BPT, int PL>
__global__ __launch_bounds__(1024) __attribute__((amdgpu_waves_per_eu(PL == kPlace4 ? 4 : 8))) void batch_kernel(const WorkItem* __restrict__ items, uint32_t n_enc,
                                                     uint32_t n_dec, const uint32_t* __restrict__ key_table,
                                                     uint32_t n_slots, const uint4* __restrict__ in_base,
                                                     uint4* __restrict__ out_base, uint64_t in_blocks,
                                                     uint64_t out_blocks, uint32_t* counters, uint32_t enc_groups,
                                                     uint32_t* done_word, uint32_t done_seq)
{
    __shared__ __align__(16) uint32_t lds[Layout<PL, true>::words];  // the larger of the two directions
    bool dec = blockIdx.x >= enc_groups;
    for (int pass = 0; pass < 2; ++pass, dec = !dec) {
        if ((dec ? n_dec : n_enc) == 0)
            continue;  // uniform across the grid: no tables to load, no barrier to meet
        if (dec)
            fill_tables<PL, true>(lds, &c_tables);
        else
            fill_tables<PL, false>(lds, &c_tables);
        __syncthreads();
        if (dec)
            drain<true, BPT, PL>(items, n_enc, n_dec, key_table, n_slots, in_base, out_base, in_blocks, out_blocks,
                             counters, lds);
        else
            drain<false, BPT, PL>(items, 0, n_enc, key_table, n_slots, in_base, out_base, in_blocks, out_blocks,
                              counters, lds);
        __syncthreads();  // every wave is done with these tables before LDS is refilled
    }
    if (threadIdx.x == 0) {
        __threadfence();
        if (atomicAdd(&counters[2], 1u) == gridDim.x - 1) {
            atomicExch(&counters[0], 0u);
            atomicExch(&counters[1], 0u);
            atomicExch(&counters[2], 0u);
            __threadfence();
            // every workgroup released its stores before counting itself
            if (done_word != nullptr)
                __hip_atomic_store(done_word, done_seq, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
        }
    }
}

void batch_grid(uint64_t n_enc, uint64_t n_dec, uint64_t enc_blocks, uint64_t total_blocks, int wg, int max_grid,
                int requested_enc_groups, int* grid, int* enc_groups)
{
    // one wave claims one item at a time: no point in more workgroups than
    // (items / waves per workgroup) per direction
    const uint64_t wpw = (uint64_t)(wg / 64);
    const uint64_t need_e = (n_enc + wpw - 1) / wpw, need_d = (n_dec + wpw - 1) / wpw;
    uint64_t g = std::min<uint64_t>((uint64_t)max_grid, std::max<uint64_t>(1, need_e + need_d));
    if (n_enc && n_dec && g < 2)
        g = 2;
    int64_t e;
    if (n_enc == 0)
        e = 0;
    else if (n_dec == 0)
        e = (int64_t)g;
    else if (requested_enc_groups >= 0)
        e = requested_enc_groups;
    else
        e = (int64_t)((g * enc_blocks + total_blocks / 2) / std::max<uint64_t>(1, total_blocks));
    if (n_enc && e < 1)
        e = 1;
    if (n_dec && e > (int64_t)g - 1)
        e = (int64_t)g - 1;
    *grid = (int)g;
    *enc_groups = (int)e;
}

namespace {

template <int PL>
const void* batch_kernel_bpt(int bpt)
{
    switch (bpt) {
    case 1: return reinterpret_cast<const void*>(batch_kernel<1, PL>);
    case 2: return reinterpret_cast<const void*>(batch_kernel<2, PL>);
    case 4: return reinterpret_cast<const void*>(batch_kernel<4, PL>);
    default: return nullptr;
    }
}

const void* batch_kernel_for(int bpt, int placement)
{
    switch (placement) {
    case kPlace4: return batch_kernel_bpt<kPlace4>(bpt);
    case kPlace2: return batch_kernel_bpt<kPlace2>(bpt);
    case kPlace1: return batch_kernel_bpt<kPlace1>(bpt);
    default: return nullptr;
    }
}

// Workgroups per CU of each (bpt, placement, workgroup size), from the
// occupancy query on first use; 0 = not asked yet.
std::atomic<int> g_groups_per_cu[3][3][16];

int bpt_index(int bpt) { return bpt == 1 ? 0 : bpt == 2 ? 1 : bpt == 4 ? 2 : -1; }

}  // namespace

hipError_t batch_groups_per_cu(int bpt, int placement, int wg, int* per_cu)
{
    const void* k = batch_kernel_for(bpt, placement);
    const int bi = bpt_index(bpt);
    if (k == nullptr || bi < 0 || wg < 64 || wg > 1024 || wg % 64)
        return hipErrorInvalidValue;
    std::atomic<int>& slot = g_groups_per_cu[bi][placement][wg / 64 - 1];
    int n = slot.load(std::memory_order_relaxed);
    if (n <= 0) {
        hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k, wg, 0);
        if (e != hipSuccess)
            return e;
        n = n > 0 ? n : 1;
        slot.store(n, std::memory_order_relaxed);
    }
    *per_cu = n;
    return hipSuccess;
}

namespace {

hipError_t launch_batch_impl(const BatchArgs& a, int bpt, int placement, int grid, int wg, uint32_t* done_word,
                             uint32_t seq, hipStream_t stream)
{
#define AESGPU_BATCH_LAUNCH(B, P)                                                                                  \
    hipLaunchKernelGGL((batch_kernel<B, P>), dim3(grid), dim3(wg), 0, stream, a.items, a.n_enc, a.n_dec,           \
                       a.key_table, a.n_slots, static_cast<const uint4*>(a.in_base), static_cast<uint4*>(a.out_base), \
                       a.in_blocks, a.out_blocks, a.counters, a.enc_groups, done_word, seq)
#define AESGPU_BATCH_PLACEMENT(P)                   \
    switch (bpt) {                                  \
    case 1: AESGPU_BATCH_LAUNCH(1, P); break;       \
    case 2: AESGPU_BATCH_LAUNCH(2, P); break;       \
    case 4: AESGPU_BATCH_LAUNCH(4, P); break;       \
    default: return hipErrorInvalidValue;           \
    }
    switch (placement) {
    case kPlace4: AESGPU_BATCH_PLACEMENT(kPlace4); break;
    case kPlace2: AESGPU_BATCH_PLACEMENT(kPlace2); break;
    case kPlace1: AESGPU_BATCH_PLACEMENT(kPlace1); break;
    default: return hipErrorInvalidValue;
    }
#undef AESGPU_BATCH_PLACEMENT
#undef AESGPU_BATCH_LAUNCH
    return hipGetLastError();
}

}  // namespace

hipError_t launch_batch(const BatchArgs& a, int bpt, int placement, int grid, int wg, hipStream_t stream)
{
    return launch_batch_impl(a, bpt, placement, grid, wg, nullptr, 0u, stream);
}

hipError_t launch_batch_signal(const BatchArgs& a, int bpt, int placement, int grid, int wg, uint32_t* done_word,
                               uint32_t seq, hipStream_t stream)
{
    if (done_word == nullptr)
        return hipErrorInvalidValue;
    return launch_batch_impl(a, bpt, placement, grid, wg, done_word, seq, stream);
}

// Claim counters of the allocation-free batched launch
// (aes_ecb_batch_noalloc).  One copy per device, held until the process
// ends; kScratchWords words, of which a launch uses the first four, laid out
// as the counters of aes_ecb_batch.  Host code never passes this array's
// name to a kernel: it takes the device address from hipGetSymbolAddress,
// once per device, with that device current.
constexpr uint32_t kScratchWords = AES_NOALLOC_SCRATCH_BYTES / 4;
static __device__ __align__(256) uint32_t scratch[kScratchWords];

namespace {

std::mutex g_scratch_mu;
std::atomic<uint32_t*> g_scratch[64];  // device address of `scratch`, per device

// Zero n words with one small kernel (a kernel node, not a memset node, when
// a caller captures the launch in a graph).
__global__ __launch_bounds__(64) void zero_words(uint32_t* p, uint32_t n)
{
    for (uint32_t i = threadIdx.x; i < n; i += blockDim.x)
        p[i] = 0u;
}

}  // namespace

hipError_t noalloc_scratch(uint32_t** out)
{
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess)
        return e;
    if (dev < 0 || dev >= 64)
        return hipErrorInvalidDevice;
    uint32_t* p = g_scratch[dev].load(std::memory_order_acquire);
    if (p == nullptr) {
        std::lock_guard<std::mutex> lk(g_scratch_mu);
        p = g_scratch[dev].load(std::memory_order_relaxed);
        if (p == nullptr) {
            void* addr = nullptr;
            e = hipGetSymbolAddress(&addr, HIP_SYMBOL(scratch));
            if (e != hipSuccess)
                return e;
            p = static_cast<uint32_t*>(addr);
            g_scratch[dev].store(p, std::memory_order_release);
        }
    }
    *out = p;
    return hipSuccess;
}

hipError_t launch_batch_noalloc(BatchArgs a, int bpt, int placement, int grid, int wg, hipStream_t stream)
{
    uint32_t* p = nullptr;
    hipError_t e = noalloc_scratch(&p);
    if (e != hipSuccess)
        return e;
    // the counters start at zero whatever an earlier launch left
    hipLaunchKernelGGL(zero_words, dim3(1), dim3(64), 0, stream, p, 4u);
    e = hipGetLastError();
    if (e != hipSuccess)
        return e;
    a.counters = p;
    return launch_batch(a, bpt, placement, grid, wg, stream);
}

}  // namespace aesgpu
