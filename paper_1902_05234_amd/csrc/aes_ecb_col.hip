// aes_ecb_col.hip -- ECB with one column word per lane (4 bytes per thread).
//
// The paper gives each thread one whole 16-byte state (section 4.1).  At
// small sizes a launch is bound by the latency of one block's ten to
// fourteen dependent rounds, and a lane issues all sixteen lookups of a
// round one after the other.  Here four lanes of a quad share one block,
// lane 4q + j holding column word W_j of block q, so a lane issues four
// lookups per round: the round's critical path is about a quarter of the
// lookups plus three quad exchanges.  The round is still eq 26: the output
// column j needs byte t of W_{j+t} (W_{j-t} for decryption), and the quad
// exchanges (DPP quad permutations, one VALU move each) bring those three
// neighbour words to the lane.  Per block this costs more VALU work than the
// whole-state form (the exchanges, and per-lane round keys), so it is a
// variant for the latency-bound sizes; the tables and their placements are
// those of the whole-state kernels.
//
// A wave covers 16 consecutive blocks (256 bytes) per unit: lane l loads
// and stores word l of the unit, so each global_load/store_dword of a wave is
// one contiguous 256-byte access.  The blocks of the last, partial unit are
// whole quads, so a quad is either fully active or fully idle.
#include "aes_col_round.hpp"
#include "aes_ecb_kernel.hpp"

namespace aesgpu {

__device__ __forceinline__ void store_word(uint32_t* p, uint32_t v) { __builtin_nontemporal_store(v, p); }

template <int NR, bool kDecrypt, int PL>
__global__ __launch_bounds__(1024) void ecb_col_kernel(const uint32_t* __restrict__ in, uint32_t* __restrict__ out,
                                                       uint64_t nblocks, RoundKeys rk)
{
    __shared__ __align__(16) uint32_t lds[Layout<PL, kDecrypt>::words];
    const uint32_t lane = threadIdx.x & 63u;
    const uint64_t waves_per_grid = (uint64_t)gridDim.x * (blockDim.x >> 6);
    const uint64_t nwords = nblocks * 4u;
    const uint64_t full_units = nwords / 64u;  // 16 blocks each
    uint64_t wv = (uint64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    uint32_t cur = 0;
    if (wv < full_units)
        cur = in[wv * 64u + lane];
    fill_tables<PL, kDecrypt>(lds, &c_tables);
    // round key words of this lane's column
    const uint32_t j = lane & 3u;
    uint32_t kc[NR + 1];
#pragma unroll
    for (int r = 0; r <= NR; ++r)
        kc[r] = j == 0 ? rk.w[4 * r] : j == 1 ? rk.w[4 * r + 1] : j == 2 ? rk.w[4 * r + 2] : rk.w[4 * r + 3];
    __syncthreads();
    const LaneBases<PL, kDecrypt> lb(threadIdx.x);
    for (; wv < full_units; wv += waves_per_grid) {
        const uint64_t wn = wv + waves_per_grid;
        uint32_t nxt = 0;
        if (wn < full_units)
            nxt = in[wn * 64u + lane];
        store_word(out + wv * 64u + lane, col_block<NR, kDecrypt, PL>(cur, lds, lb, kc));
        cur = nxt;
    }
    // the ragged unit: whole quads of the blocks that exist
    if (wv == full_units && full_units * 64u < nwords) {
        const uint64_t i = wv * 64u + lane;
        if (i < nwords)
            store_word(out + i, col_block<NR, kDecrypt, PL>(in[i], lds, lb, kc));
    }
}

template <int NR, bool kDecrypt, int PL>
hipError_t launch_col_one(const void* in, void* out, uint64_t nblocks, const RoundKeys& rk, const LaunchShape& shape,
                          int cus, hipStream_t stream)
{
    auto kern = ecb_col_kernel<NR, kDecrypt, PL>;
    int grid = shape.grid;
    if (grid <= 0) {
        int per_cu = 0;
        hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, reinterpret_cast<const void*>(kern),
                                                                    shape.wg, 0);
        if (e != hipSuccess)
            return e;
        grid = cus * (per_cu > 0 ? per_cu : 1);
    }
    const uint64_t per_group = (uint64_t)shape.wg / 4u;  // blocks per workgroup per unit
    const uint64_t needed = (nblocks + per_group - 1) / per_group;
    if ((uint64_t)grid > needed)
        grid = (int)needed;
    hipLaunchKernelGGL(kern, dim3(grid), dim3(shape.wg), 0, stream, static_cast<const uint32_t*>(in),
                       static_cast<uint32_t*>(out), nblocks, rk);
    return hipGetLastError();
}

template <bool kDecrypt, int PL>
hipError_t launch_col_nr(int nr, const void* in, void* out, uint64_t nblocks, const RoundKeys& rk,
                         const LaunchShape& shape, int cus, hipStream_t stream)
{
    switch (nr) {
    case 10: return launch_col_one<10, kDecrypt, PL>(in, out, nblocks, rk, shape, cus, stream);
    case 12: return launch_col_one<12, kDecrypt, PL>(in, out, nblocks, rk, shape, cus, stream);
    case 14: return launch_col_one<14, kDecrypt, PL>(in, out, nblocks, rk, shape, cus, stream);
    default: return hipErrorInvalidValue;
    }
}

template <int PL>
hipError_t launch_col_placement(const LaunchShape& shape, int nr, bool decrypt, const void* in, void* out,
                                uint64_t nblocks, const RoundKeys& rk, int cus, hipStream_t stream)
{
    const RoundKeys k = PL == kPlace2 ? inner_keys_rotr8(rk, nr) : rk;
    if (decrypt)
        return launch_col_nr<true, PL>(nr, in, out, nblocks, k, shape, cus, stream);
    return launch_col_nr<false, PL>(nr, in, out, nblocks, k, shape, cus, stream);
}

hipError_t launch_ecb_col(const LaunchShape& shape, int placement, int nr, bool decrypt, const void* in, void* out,
                          uint64_t nblocks, const RoundKeys& rk, int cus, hipStream_t stream)
{
    switch (placement) {
    case kPlace4: return launch_col_placement<kPlace4>(shape, nr, decrypt, in, out, nblocks, rk, cus, stream);
    case kPlace2: return launch_col_placement<kPlace2>(shape, nr, decrypt, in, out, nblocks, rk, cus, stream);
    case kPlace1: return launch_col_placement<kPlace1>(shape, nr, decrypt, in, out, nblocks, rk, cus, stream);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace aesgpu
