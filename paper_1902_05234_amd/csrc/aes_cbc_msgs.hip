// aes_cbc_msgs.hip -- CBC encryption of many independent messages.
//
// CBC encryption (section 3.1.2, eq 2, read with the block cipher: C_i =
// cipher(P_i XOR C_{i-1}), C_0 the initialisation vector) is a chain: block i
// needs the ciphertext of block i - 1, which is why the paper's Table 1 marks
// the mode unsuitable for parallel work within one message.  Separate
// messages are separate chains, so this kernel gives each message one lane:
// a wave walks 64 messages side by side, block by block, with the replicated
// T-tables in LDS as in ECB and the one key in scalar registers.
//
// A lane loads G consecutive blocks of its message at once (16G contiguous
// bytes; G = 8 is one 128-byte line), one group ahead of the rounds, and
// stores a group's G ciphertext blocks together.  The 64 lanes of a wave
// touch 64 different lines per access, so the stores are plain, not
// non-temporal as in ECB: the L2 then merges a lane's 16-byte blocks into
// whole lines before they leave it, where non-temporal 16-byte stores to
// scattered lines went out one by one (about 4x slower: 330 against 1400 GB/s
// for 2^18 messages of 4 KiB).  A chain has one block in the rounds at a
// time, so the LDS is kept busy only when enough waves walk chains at once
// (16 per CU with the 4-table placement: 2^18 messages on 256 CUs); with
// fewer messages a launch is bound by the latency of one block's rounds.  A
// wave lasts as long as the longest of its 64 messages.
//
// For that latency-bound regime a second kernel gives each message a quad of
// lanes, one column word per lane (the round of aes_col_round.hpp: four
// lookups per lane per round and three quad exchanges), 16 messages per
// wave: a block's rounds take about half as long, at some more VALU work per
// block (2^16 messages of 16 KiB: 1172 against 847 GB/s; from 2^17 messages
// on the one-lane kernel is faster).
#include "aes_cbc_msgs.hpp"
#include "aes_col_round.hpp"
#include "aes_ecb_kernel.hpp"

namespace aesgpu {

namespace {

// Layout of aes_cbc_msg (aesgpu.h), read as three 16-byte loads.
struct CbcMsg {
    uint64_t in_block;
    uint64_t out_block;
    uint64_t nblocks;
    uint64_t reserved;
    uint4 iv;
};
static_assert(sizeof(CbcMsg) == 48, "aes_cbc_msg layout");

__device__ __forceinline__ uint4 xor4m(uint4 a, uint4 b) { return make_uint4(a.x ^ b.x, a.y ^ b.y, a.z ^ b.z, a.w ^ b.w); }

template <int G>
__device__ __forceinline__ void load_group(uint4 (&v)[G], const uint4* src, uint64_t first, uint64_t nb)
{
#pragma unroll
    for (int k = 0; k < G; ++k)
        if (first + k < nb)
            v[k] = src[first + k];
}

// Variant bpt of the one-wave-per-message decryption kernel: kWaveMsg plus
// the blocks per lane per unit (AES_BPT_WAVE_MSG in aesgpu.h).
constexpr int kWaveMsg = AES_BPT_WAVE_MSG;

// Message ranges inside their arenas (written so that no sum can wrap) and
// the reserved field zero.
__device__ __forceinline__ bool msg_ok(const CbcMsg& d, uint64_t in_blocks, uint64_t out_blocks)
{
    return d.reserved == 0 && d.in_block <= in_blocks && d.nblocks <= in_blocks - d.in_block &&
           d.out_block <= out_blocks && d.nblocks <= out_blocks - d.out_block;
}

template <int NR, int G, int PL>
__global__ __launch_bounds__(1024) void cbc_enc_msgs_kernel(const CbcMsg* __restrict__ msgs, uint64_t nmsgs,
                                                            const uint4* in, uint64_t in_blocks, uint4* out,
                                                            uint64_t out_blocks, uint32_t* rejected, RoundKeys rk)
{
    __shared__ __align__(16) uint32_t lds[Layout<PL, false>::words];
    fill_tables<PL, false>(lds, &c_tables);
    __syncthreads();
    const LaneBases<PL, false> lb(threadIdx.x);
    auto key = [&](int i) { return rk.w[i]; };

    const uint32_t lane = threadIdx.x & 63u;
    const uint64_t waves_per_grid = (uint64_t)gridDim.x * (blockDim.x >> 6);
    const uint64_t units = (nmsgs + 63u) / 64u;
    for (uint64_t wv = (uint64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6); wv < units;
         wv += waves_per_grid) {
        const uint64_t m = wv * 64u + lane;
        uint64_t nb = 0;
        const uint4* src = in;
        uint4* dst = out;
        uint4 chain = make_uint4(0u, 0u, 0u, 0u);
        if (m < nmsgs) {
            const CbcMsg d = msgs[m];
            if (msg_ok(d, in_blocks, out_blocks)) {
                nb = d.nblocks;
                src = in + d.in_block;
                dst = out + d.out_block;
                chain = d.iv;
            } else if (rejected != nullptr) {
                atomicAdd(rejected, 1u);
            }
        }
        uint4 cur[G];
        load_group<G>(cur, src, 0, nb);
        // each lane walks its own chain; lanes whose message has ended idle
        // until the wave's longest message is done
        for (uint64_t g = 0; g < nb; g += G) {
            uint4 nxt[G];
            load_group<G>(nxt, src, g + G, nb);
#pragma unroll
            for (int k = 0; k < G; ++k) {
                if (k == 0 || g + k < nb) {
                    chain = crypt_block<NR, false, PL>(xor4m(cur[k], chain), lds, lb, key);
                    cur[k] = chain;
                }
            }
#pragma unroll
            for (int k = 0; k < G; ++k)
                if (k == 0 || g + k < nb)
                    dst[g + k] = cur[k];
#pragma unroll
            for (int k = 0; k < G; ++k)
                cur[k] = nxt[k];
        }
    }
}

// One message per quad: lane 4q + j walks column word j of message 16u + q,
// loading and storing word j of kColGroup blocks (one 128-byte line per
// message) at a time.
constexpr int kColGroup = 8;

template <int NR, int PL>
__global__ __launch_bounds__(1024) void cbc_enc_msgs_col_kernel(const CbcMsg* __restrict__ msgs, uint64_t nmsgs,
                                                                const uint32_t* in, uint64_t in_blocks,
                                                                uint32_t* out, uint64_t out_blocks,
                                                                uint32_t* rejected, RoundKeys rk)
{
    __shared__ __align__(16) uint32_t lds[Layout<PL, false>::words];
    fill_tables<PL, false>(lds, &c_tables);
    const uint32_t lane = threadIdx.x & 63u;
    const uint32_t j = lane & 3u;
    uint32_t kc[NR + 1];
#pragma unroll
    for (int r = 0; r <= NR; ++r)
        kc[r] = j == 0 ? rk.w[4 * r] : j == 1 ? rk.w[4 * r + 1] : j == 2 ? rk.w[4 * r + 2] : rk.w[4 * r + 3];
    __syncthreads();
    const LaneBases<PL, false> lb(threadIdx.x);

    const uint64_t waves_per_grid = (uint64_t)gridDim.x * (blockDim.x >> 6);
    const uint64_t units = (nmsgs + 15u) / 16u;
    for (uint64_t wv = (uint64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6); wv < units;
         wv += waves_per_grid) {
        const uint64_t m = wv * 16u + (lane >> 2);
        uint64_t nb = 0;
        const uint32_t* src = in;
        uint32_t* dst = out;
        uint32_t chain = 0;
        if (m < nmsgs) {
            const CbcMsg d = msgs[m];  // the four lanes of a quad read the same record
            if (msg_ok(d, in_blocks, out_blocks)) {
                nb = d.nblocks;
                src = in + 4u * d.in_block + j;
                dst = out + 4u * d.out_block + j;
                chain = j == 0 ? d.iv.x : j == 1 ? d.iv.y : j == 2 ? d.iv.z : d.iv.w;
            } else if (rejected != nullptr && j == 0) {
                atomicAdd(rejected, 1u);
            }
        }
        // a quad's lanes share nb, so a quad is wholly active or wholly idle
        uint32_t cur[kColGroup];
#pragma unroll
        for (int k = 0; k < kColGroup; ++k)
            if ((uint64_t)k < nb)
                cur[k] = src[4u * k];
        for (uint64_t g = 0; g < nb; g += kColGroup) {
            uint32_t nxt[kColGroup];
#pragma unroll
            for (int k = 0; k < kColGroup; ++k)
                if (g + kColGroup + k < nb)
                    nxt[k] = src[4u * (g + kColGroup + k)];
#pragma unroll
            for (int k = 0; k < kColGroup; ++k) {
                if (k == 0 || g + k < nb) {
                    chain = col_block<NR, false, PL>(cur[k] ^ chain, lds, lb, kc);
                    cur[k] = chain;
                }
            }
#pragma unroll
            for (int k = 0; k < kColGroup; ++k)
                if (k == 0 || g + k < nb)
                    dst[4u * (g + k)] = cur[k];
#pragma unroll
            for (int k = 0; k < kColGroup; ++k)
                cur[k] = nxt[k];
        }
    }
}

// CBC decryption of a message set: P_i = invcipher(C_i) XOR C_{i-1}, so a
// lane's G blocks are independent (instruction-level parallelism within the
// lane) and only the XOR needs the preceding ciphertext block, which the lane
// still holds.  Same walk as the one-lane encryption kernel: one message per
// lane, G blocks loaded one group ahead; in place is safe because a lane
// reads every block before it writes it.
template <int NR, int G, int PL>
__global__ __launch_bounds__(1024) void cbc_dec_msgs_kernel(const CbcMsg* __restrict__ msgs, uint64_t nmsgs,
                                                            const uint4* in, uint64_t in_blocks, uint4* out,
                                                            uint64_t out_blocks, uint32_t* rejected, RoundKeys rk)
{
    __shared__ __align__(16) uint32_t lds[Layout<PL, true>::words];
    fill_tables<PL, true>(lds, &c_tables);
    __syncthreads();
    const LaneBases<PL, true> lb(threadIdx.x);
    auto key = [&](int i) { return rk.w[i]; };

    const uint32_t lane = threadIdx.x & 63u;
    const uint64_t waves_per_grid = (uint64_t)gridDim.x * (blockDim.x >> 6);
    const uint64_t units = (nmsgs + 63u) / 64u;
    for (uint64_t wv = (uint64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6); wv < units;
         wv += waves_per_grid) {
        const uint64_t m = wv * 64u + lane;
        uint64_t nb = 0;
        const uint4* src = in;
        uint4* dst = out;
        uint4 prev = make_uint4(0u, 0u, 0u, 0u);  // C_{i-1}: the IV, then the last ciphertext block read
        if (m < nmsgs) {
            const CbcMsg d = msgs[m];
            if (msg_ok(d, in_blocks, out_blocks)) {
                nb = d.nblocks;
                src = in + d.in_block;
                dst = out + d.out_block;
                prev = d.iv;
            } else if (rejected != nullptr) {
                atomicAdd(rejected, 1u);
            }
        }
        uint4 cur[G];
        load_group<G>(cur, src, 0, nb);
        for (uint64_t g = 0; g < nb; g += G) {
            uint4 nxt[G];
            load_group<G>(nxt, src, g + G, nb);
            uint4 pt[G];
#pragma unroll
            for (int k = 0; k < G; ++k)
                if (k == 0 || g + k < nb)
                    pt[k] = crypt_block<NR, true, PL>(cur[k], lds, lb, key);
#pragma unroll
            for (int k = 0; k < G; ++k)
                if (k == 0 || g + k < nb)
                    dst[g + k] = xor4m(pt[k], k == 0 ? prev : cur[k - 1]);
            prev = cur[G - 1];  // only read again if the next group exists, so this group was whole
#pragma unroll
            for (int k = 0; k < G; ++k)
                cur[k] = nxt[k];
        }
    }
}

// CBC decryption of a message set with one wave per message: the wave walks
// its message by units of 64*BPT consecutive blocks (lane l takes blocks
// l + 64k, every access of the wave one contiguous run), as the one-message
// decryption kernel does.  For messages of 64 blocks or more this keeps every
// lane busy however few the messages are.  The next unit's blocks, and the
// ciphertext blocks before them, are loaded before the current unit is
// stored, and no other wave touches the message, so in place is safe.
template <int NR, int BPT, int PL>
__global__ __launch_bounds__(1024) void cbc_dec_msgs_wave_kernel(const CbcMsg* __restrict__ msgs, uint64_t nmsgs,
                                                                 const uint4* in, uint64_t in_blocks, uint4* out,
                                                                 uint64_t out_blocks, uint32_t* rejected,
                                                                 RoundKeys rk)
{
    __shared__ __align__(16) uint32_t lds[Layout<PL, true>::words];
    fill_tables<PL, true>(lds, &c_tables);
    __syncthreads();
    const LaneBases<PL, true> lb(threadIdx.x);
    auto key = [&](int i) { return rk.w[i]; };

    const uint32_t lane = threadIdx.x & 63u;
    const uint64_t waves_per_grid = (uint64_t)gridDim.x * (blockDim.x >> 6);
    constexpr uint64_t span = 64u * BPT;
    // the message index is wave-uniform, so the record comes in through scalar loads
    const uint32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    for (uint64_t m = (uint64_t)blockIdx.x * (blockDim.x >> 6) + wave; m < nmsgs; m += waves_per_grid) {
        const CbcMsg d = msgs[m];  // one record for the whole wave
        if (!msg_ok(d, in_blocks, out_blocks)) {
            if (rejected != nullptr && lane == 0)
                atomicAdd(rejected, 1u);
            continue;
        }
        const uint4* src = in + d.in_block;
        uint4* dst = out + d.out_block;
        const uint64_t nb = d.nblocks;
        // block b and the ciphertext before it (the IV for block 0; the load
        // then reads block 0 and is discarded, so it never leaves the message)
        auto load = [&](uint64_t b, uint4& c, uint4& p) {
            c = src[b];
            const uint4 t = src[b ? b - 1 : 0];
            p = b ? t : d.iv;
        };
        uint4 cur[BPT], prv[BPT];
#pragma unroll
        for (int k = 0; k < BPT; ++k)
            if (lane + 64u * k < nb)
                load(lane + 64u * k, cur[k], prv[k]);
        for (uint64_t u0 = 0; u0 < nb; u0 += span) {
            uint4 nxt[BPT], nxp[BPT];
#pragma unroll
            for (int k = 0; k < BPT; ++k)
                if (u0 + span + lane + 64u * k < nb)
                    load(u0 + span + lane + 64u * k, nxt[k], nxp[k]);
#pragma unroll
            for (int k = 0; k < BPT; ++k) {
                const uint64_t b = u0 + lane + 64u * k;
                if (b < nb)
                    store_block(dst + b, xor4m(crypt_block<NR, true, PL>(cur[k], lds, lb, key), prv[k]));
            }
#pragma unroll
            for (int k = 0; k < BPT; ++k) {
                cur[k] = nxt[k];
                prv[k] = nxp[k];
            }
        }
    }
}

template <int NR, int BPT, int PL>
hipError_t launch_one_cbc_dec_msgs_wave(const CbcMsg* msgs, uint64_t nmsgs, const void* in, uint64_t in_blocks,
                                        void* out, uint64_t out_blocks, uint32_t* rejected, const RoundKeys& rk,
                                        const LaunchShape& shape, int cus, hipStream_t stream)
{
    auto kern = cbc_dec_msgs_wave_kernel<NR, BPT, PL>;
    int grid = shape.grid;
    if (grid <= 0) {
        int per_cu = 0;
        hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, reinterpret_cast<const void*>(kern),
                                                                    shape.wg, 0);
        if (e != hipSuccess)
            return e;
        grid = cus * (per_cu > 0 ? per_cu : 1);
    }
    const uint64_t per_group = (uint64_t)shape.wg / 64u;  // messages per workgroup at a time
    const uint64_t needed = (nmsgs + per_group - 1) / per_group;
    if ((uint64_t)grid > needed)
        grid = (int)needed;
    hipLaunchKernelGGL(kern, dim3(grid), dim3(shape.wg), 0, stream, msgs, nmsgs, static_cast<const uint4*>(in),
                       in_blocks, static_cast<uint4*>(out), out_blocks, rejected, rk);
    return hipGetLastError();
}

template <int NR, int G, int PL>
hipError_t launch_one_cbc_dec_msgs(const CbcMsg* msgs, uint64_t nmsgs, const void* in, uint64_t in_blocks, void* out,
                                   uint64_t out_blocks, uint32_t* rejected, const RoundKeys& rk,
                                   const LaunchShape& shape, int cus, hipStream_t stream)
{
    auto kern = cbc_dec_msgs_kernel<NR, G, PL>;
    int grid = shape.grid;
    if (grid <= 0) {
        int per_cu = 0;
        hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, reinterpret_cast<const void*>(kern),
                                                                    shape.wg, 0);
        if (e != hipSuccess)
            return e;
        grid = cus * (per_cu > 0 ? per_cu : 1);
    }
    const uint64_t waves = (nmsgs + 63u) / 64u;
    const uint64_t per_group = (uint64_t)shape.wg / 64u;
    const uint64_t needed = (waves + per_group - 1) / per_group;
    if ((uint64_t)grid > needed)
        grid = (int)needed;
    hipLaunchKernelGGL(kern, dim3(grid), dim3(shape.wg), 0, stream, msgs, nmsgs, static_cast<const uint4*>(in),
                       in_blocks, static_cast<uint4*>(out), out_blocks, rejected, rk);
    return hipGetLastError();
}

template <int G, int PL>
hipError_t launch_cbc_dec_msgs_nr(int nr, const CbcMsg* msgs, uint64_t nmsgs, const void* in, uint64_t in_blocks,
                                  void* out, uint64_t out_blocks, uint32_t* rejected, const RoundKeys& rk,
                                  const LaunchShape& shape, int cus, hipStream_t stream)
{
    if constexpr (G > kWaveMsg) {  // one wave per message, G - kWaveMsg (1 or 2) blocks per lane per unit
        constexpr int B = G - kWaveMsg;
        switch (nr) {
        case 10: return launch_one_cbc_dec_msgs_wave<10, B, PL>(msgs, nmsgs, in, in_blocks, out, out_blocks, rejected, rk, shape, cus, stream);
        case 12: return launch_one_cbc_dec_msgs_wave<12, B, PL>(msgs, nmsgs, in, in_blocks, out, out_blocks, rejected, rk, shape, cus, stream);
        case 14: return launch_one_cbc_dec_msgs_wave<14, B, PL>(msgs, nmsgs, in, in_blocks, out, out_blocks, rejected, rk, shape, cus, stream);
        default: return hipErrorInvalidValue;
        }
    } else {
        switch (nr) {
        case 10: return launch_one_cbc_dec_msgs<10, G, PL>(msgs, nmsgs, in, in_blocks, out, out_blocks, rejected, rk, shape, cus, stream);
        case 12: return launch_one_cbc_dec_msgs<12, G, PL>(msgs, nmsgs, in, in_blocks, out, out_blocks, rejected, rk, shape, cus, stream);
        case 14: return launch_one_cbc_dec_msgs<14, G, PL>(msgs, nmsgs, in, in_blocks, out, out_blocks, rejected, rk, shape, cus, stream);
        default: return hipErrorInvalidValue;
        }
    }
}

template <int PL>
hipError_t launch_cbc_dec_msgs_g(int nr, const CbcMsg* msgs, uint64_t nmsgs, const void* in, uint64_t in_blocks,
                                 void* out, uint64_t out_blocks, uint32_t* rejected, const RoundKeys& rk,
                                 const LaunchShape& shape, int cus, hipStream_t stream)
{
    switch (shape.bpt) {
    case 1: return launch_cbc_dec_msgs_nr<1, PL>(nr, msgs, nmsgs, in, in_blocks, out, out_blocks, rejected, rk, shape, cus, stream);
    case 2: return launch_cbc_dec_msgs_nr<2, PL>(nr, msgs, nmsgs, in, in_blocks, out, out_blocks, rejected, rk, shape, cus, stream);
    case 4: return launch_cbc_dec_msgs_nr<4, PL>(nr, msgs, nmsgs, in, in_blocks, out, out_blocks, rejected, rk, shape, cus, stream);
    case kWaveMsg + 1: return launch_cbc_dec_msgs_nr<kWaveMsg + 1, PL>(nr, msgs, nmsgs, in, in_blocks, out, out_blocks, rejected, rk, shape, cus, stream);
    case kWaveMsg + 2: return launch_cbc_dec_msgs_nr<kWaveMsg + 2, PL>(nr, msgs, nmsgs, in, in_blocks, out, out_blocks, rejected, rk, shape, cus, stream);
    default: return hipErrorInvalidValue;
    }
}

template <int NR, int PL>
hipError_t launch_one_cbc_msgs_col(const CbcMsg* msgs, uint64_t nmsgs, const void* in, uint64_t in_blocks, void* out,
                                   uint64_t out_blocks, uint32_t* rejected, const RoundKeys& rk,
                                   const LaunchShape& shape, int cus, hipStream_t stream)
{
    auto kern = cbc_enc_msgs_col_kernel<NR, PL>;
    int grid = shape.grid;
    if (grid <= 0) {
        int per_cu = 0;
        hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, reinterpret_cast<const void*>(kern),
                                                                    shape.wg, 0);
        if (e != hipSuccess)
            return e;
        grid = cus * (per_cu > 0 ? per_cu : 1);
    }
    // no more workgroups than the 16-message wave units can keep busy
    const uint64_t waves = (nmsgs + 15u) / 16u;
    const uint64_t per_group = (uint64_t)shape.wg / 64u;
    const uint64_t needed = (waves + per_group - 1) / per_group;
    if ((uint64_t)grid > needed)
        grid = (int)needed;
    hipLaunchKernelGGL(kern, dim3(grid), dim3(shape.wg), 0, stream, msgs, nmsgs, static_cast<const uint32_t*>(in),
                       in_blocks, static_cast<uint32_t*>(out), out_blocks, rejected, rk);
    return hipGetLastError();
}

template <int NR, int G, int PL>
hipError_t launch_one_cbc_msgs(const CbcMsg* msgs, uint64_t nmsgs, const void* in, uint64_t in_blocks, void* out,
                               uint64_t out_blocks, uint32_t* rejected, const RoundKeys& rk, const LaunchShape& shape,
                               int cus, hipStream_t stream)
{
    auto kern = cbc_enc_msgs_kernel<NR, G, PL>;
    int grid = shape.grid;
    if (grid <= 0) {
        int per_cu = 0;
        hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, reinterpret_cast<const void*>(kern),
                                                                    shape.wg, 0);
        if (e != hipSuccess)
            return e;
        grid = cus * (per_cu > 0 ? per_cu : 1);
    }
    // no more workgroups than the 64-message wave units can keep busy
    const uint64_t waves = (nmsgs + 63u) / 64u;
    const uint64_t per_group = (uint64_t)shape.wg / 64u;
    const uint64_t needed = (waves + per_group - 1) / per_group;
    if ((uint64_t)grid > needed)
        grid = (int)needed;
    hipLaunchKernelGGL(kern, dim3(grid), dim3(shape.wg), 0, stream, msgs, nmsgs, static_cast<const uint4*>(in),
                       in_blocks, static_cast<uint4*>(out), out_blocks, rejected, rk);
    return hipGetLastError();
}

template <int G, int PL>
hipError_t launch_cbc_msgs_nr(int nr, const CbcMsg* msgs, uint64_t nmsgs, const void* in, uint64_t in_blocks,
                              void* out, uint64_t out_blocks, uint32_t* rejected, const RoundKeys& rk,
                              const LaunchShape& shape, int cus, hipStream_t stream)
{
    if constexpr (G == 0) {  // one column per lane (AES_BPT_COLUMN)
        switch (nr) {
        case 10: return launch_one_cbc_msgs_col<10, PL>(msgs, nmsgs, in, in_blocks, out, out_blocks, rejected, rk, shape, cus, stream);
        case 12: return launch_one_cbc_msgs_col<12, PL>(msgs, nmsgs, in, in_blocks, out, out_blocks, rejected, rk, shape, cus, stream);
        case 14: return launch_one_cbc_msgs_col<14, PL>(msgs, nmsgs, in, in_blocks, out, out_blocks, rejected, rk, shape, cus, stream);
        default: return hipErrorInvalidValue;
        }
    } else {
        switch (nr) {
        case 10: return launch_one_cbc_msgs<10, G, PL>(msgs, nmsgs, in, in_blocks, out, out_blocks, rejected, rk, shape, cus, stream);
        case 12: return launch_one_cbc_msgs<12, G, PL>(msgs, nmsgs, in, in_blocks, out, out_blocks, rejected, rk, shape, cus, stream);
        case 14: return launch_one_cbc_msgs<14, G, PL>(msgs, nmsgs, in, in_blocks, out, out_blocks, rejected, rk, shape, cus, stream);
        default: return hipErrorInvalidValue;
        }
    }
}

template <int PL>
hipError_t launch_cbc_msgs_g(int nr, const CbcMsg* msgs, uint64_t nmsgs, const void* in, uint64_t in_blocks,
                             void* out, uint64_t out_blocks, uint32_t* rejected, const RoundKeys& rk,
                             const LaunchShape& shape, int cus, hipStream_t stream)
{
    switch (shape.bpt) {
    case 0: return launch_cbc_msgs_nr<0, PL>(nr, msgs, nmsgs, in, in_blocks, out, out_blocks, rejected, rk, shape, cus, stream);
    case 1: return launch_cbc_msgs_nr<1, PL>(nr, msgs, nmsgs, in, in_blocks, out, out_blocks, rejected, rk, shape, cus, stream);
    case 2: return launch_cbc_msgs_nr<2, PL>(nr, msgs, nmsgs, in, in_blocks, out, out_blocks, rejected, rk, shape, cus, stream);
    case 4: return launch_cbc_msgs_nr<4, PL>(nr, msgs, nmsgs, in, in_blocks, out, out_blocks, rejected, rk, shape, cus, stream);
    case 8: return launch_cbc_msgs_nr<8, PL>(nr, msgs, nmsgs, in, in_blocks, out, out_blocks, rejected, rk, shape, cus, stream);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace

hipError_t launch_cbc_decrypt_msgs(const LaunchShape& shape, int placement, int nr, const void* msgs, uint64_t nmsgs,
                                   const void* in, uint64_t in_blocks, void* out, uint64_t out_blocks,
                                   uint32_t* rejected, const RoundKeys& rk, int cus, hipStream_t stream)
{
    const CbcMsg* m = static_cast<const CbcMsg*>(msgs);
    switch (placement) {
    case kPlace4:
        return launch_cbc_dec_msgs_g<kPlace4>(nr, m, nmsgs, in, in_blocks, out, out_blocks, rejected, rk, shape, cus, stream);
    case kPlace2:
        return launch_cbc_dec_msgs_g<kPlace2>(nr, m, nmsgs, in, in_blocks, out, out_blocks, rejected,
                                              inner_keys_rotr8(rk, nr), shape, cus, stream);
    case kPlace1:
        return launch_cbc_dec_msgs_g<kPlace1>(nr, m, nmsgs, in, in_blocks, out, out_blocks, rejected, rk, shape, cus, stream);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_cbc_encrypt_msgs(const LaunchShape& shape, int placement, int nr, const void* msgs, uint64_t nmsgs,
                                   const void* in, uint64_t in_blocks, void* out, uint64_t out_blocks,
                                   uint32_t* rejected, const RoundKeys& rk, int cus, hipStream_t stream)
{
    const CbcMsg* m = static_cast<const CbcMsg*>(msgs);
    switch (placement) {
    case kPlace4:
        return launch_cbc_msgs_g<kPlace4>(nr, m, nmsgs, in, in_blocks, out, out_blocks, rejected, rk, shape, cus, stream);
    case kPlace2:
        return launch_cbc_msgs_g<kPlace2>(nr, m, nmsgs, in, in_blocks, out, out_blocks, rejected,
                                          inner_keys_rotr8(rk, nr), shape, cus, stream);
    case kPlace1:
        return launch_cbc_msgs_g<kPlace1>(nr, m, nmsgs, in, in_blocks, out, out_blocks, rejected, rk, shape, cus, stream);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace aesgpu
