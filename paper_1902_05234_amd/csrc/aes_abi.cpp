// aes_abi.cpp -- the extern "C" boundary of libaesgpu (declared in include/aesgpu.h).
//
// Host side only: argument checks, the key schedule, the batch planner and
// the launch of the kernels in aes_ecb.hip / aes_batch.hip.  No entry point
// allocates device memory, and none aborts: every failure is a status code
// with a message available from aes_last_error().
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cstdarg>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <mutex>

#include "../../include/aesgpu.h"
#include "aes_cbc_msgs.hpp"
#include "aes_internal.hpp"
#include "aes_tables.hpp"

namespace aesgpu {

thread_local char g_err[512] = "";

int fail(int code, const char* fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
    return code;
}

int fail_hip(hipError_t e, const char* what)
{
    return fail(AES_EHIP, "%s: %s", what, hipGetErrorString(e));
}

namespace {

constexpr TableSet kHostTables = make_tables();

int rounds_for_bits(int keybits)
{
    switch (keybits) {
    case 128: return 10;
    case 192: return 12;
    case 256: return 14;
    default: return -1;
    }
}

bool valid_nr(int nr) { return nr == 10 || nr == 12 || nr == 14; }

uint32_t sub_word(uint32_t x)
{
    return uint32_t(kHostTables.sbox[x & 0xff]) | (uint32_t(kHostTables.sbox[(x >> 8) & 0xff]) << 8) |
           (uint32_t(kHostTables.sbox[(x >> 16) & 0xff]) << 16) | (uint32_t(kHostTables.sbox[x >> 24]) << 24);
}

// InvMixColumns of one column word: Td0[S[x]] is column 0 of the inverse
// matrix times x, and column r is that word rotated by 8r bits.
uint32_t inv_mix_column(uint32_t x)
{
    uint32_t r = 0;
    for (int t = 0; t < 4; ++t)
        r ^= rotl32(kHostTables.td0[kHostTables.sbox[(x >> (8 * t)) & 0xff]], 8 * t);
    return r;
}

// Size buckets of the tuning table: <=4 KiB, <=64 KiB, <=512 KiB, <=2 MiB,
// <=8 MiB, <=32 MiB, larger.
int size_bucket(uint64_t nblocks)
{
    if (nblocks <= 256) return 0;
    if (nblocks <= 4096) return 1;
    if (nblocks <= 32768) return 2;
    if (nblocks <= 131072) return 3;
    if (nblocks <= 524288) return 4;
    if (nblocks <= 2097152) return 5;
    return 6;
}

struct TuneEntry {
    std::atomic<int> bpt{1}, wg{1024}, placement{AES_PLACEMENT_TTABLE4};
};
TuneEntry g_tune[3][2][AES_SIZE_BUCKETS];  // [nr index][decrypt][bucket]

// Compiled-in defaults: the winners of the MI355X autotune record
// (paper_1902_05234_amd/tuning/mi355x_sweep.json), written into
// aes_tune_defaults.inc by `python -m paper_1902_05234_amd.autotune
// --emit-defaults`; a CPU test checks that the two agree.
struct TuneDefault {
    int bpt, wg, placement;
};
#include "aes_tune_defaults.inc"

struct TuneDefaults {
    TuneDefaults()
    {
        for (int n = 0; n < 3; ++n)
            for (int d = 0; d < 2; ++d)
                for (int b = 0; b < AES_SIZE_BUCKETS; ++b) {
                    const TuneDefault& t = kTuneDefaults[n][d][b];
                    g_tune[n][d][b].bpt.store(t.bpt);
                    g_tune[n][d][b].wg.store(t.wg);
                    g_tune[n][d][b].placement.store(t.placement);
                }
    }
} g_tune_defaults;

int nr_index(int nr) { return (nr - 10) / 2; }

std::atomic<int> g_cu_count[64];

bool ranges_partially_overlap(const void* a, const void* b, uint64_t bytes)
{
    uintptr_t x = reinterpret_cast<uintptr_t>(a), y = reinterpret_cast<uintptr_t>(b);
    if (x == y)
        return false;
    return x < y + bytes && y < x + bytes;
}

int check_buffers(const void* in, void* out, size_t nblocks)
{
    if (in == nullptr || out == nullptr)
        return fail(AES_EINVAL, "null buffer pointer with nblocks=%zu", nblocks);
    if (nblocks > (SIZE_MAX >> 5))
        return fail(AES_EINVAL, "nblocks=%zu too large", nblocks);
    if ((reinterpret_cast<uintptr_t>(in) | reinterpret_cast<uintptr_t>(out)) & 15u)
        return fail(AES_EALIGN, "in/out must be 16-byte aligned");
    if (ranges_partially_overlap(in, out, (uint64_t)nblocks * 16u))
        return fail(AES_EINVAL, "in and out overlap without being the same buffer");
    return AES_OK;
}

int check_variant(const aes_variant* v)
{
    if (v->bpt != AES_BPT_COLUMN && v->bpt != 1 && v->bpt != 2 && v->bpt != 4)
        return fail(AES_EINVAL, "bpt must be 1, 2 or 4 (16, 32 or 64 bytes per thread) or AES_BPT_COLUMN, got %d",
                    v->bpt);
    if (v->bpt == AES_BPT_COLUMN && v->placement == AES_PLACEMENT_BITSLICED)
        return fail(AES_EINVAL, "one column per lane (AES_BPT_COLUMN) runs on the table placements only");
    if (v->wg < 64 || v->wg > 1024 || (v->wg % 64) != 0)
        return fail(AES_EINVAL, "workgroup size must be a multiple of 64 in [64, 1024], got %d", v->wg);
    if (v->placement != AES_PLACEMENT_TTABLE4 && v->placement != AES_PLACEMENT_TTABLE2 &&
        v->placement != AES_PLACEMENT_TTABLE1 && v->placement != AES_PLACEMENT_BITSLICED)
        return fail(AES_EINVAL, "placement %d is not built in this library", v->placement);
    if (v->placement == AES_PLACEMENT_BITSLICED && v->wg > kBitsliceMaxWg)
        return fail(AES_EINVAL, "the bitsliced placement takes workgroups of at most %d threads, got %d",
                    kBitsliceMaxWg, v->wg);
    if (v->grid < 0)
        return fail(AES_EINVAL, "grid must be >= 0 (0 = persistent default), got %d", v->grid);
    return AES_OK;
}

int run_ecb(const uint32_t* rk, int nr, bool decrypt, const void* in, void* out, size_t nblocks,
            const aes_variant* v, void* stream)
{
    if (!valid_nr(nr))
        return fail(AES_EINVAL, "nr must be 10, 12 or 14, got %d", nr);
    if (rk == nullptr)
        return fail(AES_EINVAL, "null round-key pointer");
    if (nblocks == 0)
        return AES_OK;
    int rc = check_buffers(in, out, nblocks);
    if (rc != AES_OK)
        return rc;
    rc = check_variant(v);
    if (rc != AES_OK)
        return rc;
    RoundKeys keys{};
    std::memcpy(keys.w, rk, sizeof(uint32_t) * 4 * (nr + 1));
    int cus = device_cu_count();
    if (cus <= 0)
        return fail(AES_EHIP, "cannot query the current HIP device");
    LaunchShape shape{v->bpt, v->wg, v->grid};
    hipError_t e =
        launch_ecb(shape, v->placement, nr, decrypt, in, out, nblocks, keys, cus, static_cast<hipStream_t>(stream));
    if (e != hipSuccess)
        return fail_hip(e, "ECB kernel launch");
    return AES_OK;
}

// CTR and CBC run on the whole-state table kernels; a bitsliced tuning entry
// (ECB only) is replaced by the 2-table kernel with 32 bytes per thread, and
// a one-column-per-lane entry (ECB only) by the same placement with one
// block per thread.
void table_variant(aes_variant* v)
{
    if (v->placement == AES_PLACEMENT_BITSLICED) {
        v->placement = AES_PLACEMENT_TTABLE2;
        v->bpt = 2;
        v->wg = 1024;
    }
    if (v->bpt == AES_BPT_COLUMN)
        v->bpt = 1;
}

int run_ctr(const uint32_t* rk, int nr, const uint8_t* iv, uint64_t block_offset, const void* in, void* out,
            size_t nbytes, const aes_variant* v, void* stream)
{
    if (!valid_nr(nr))
        return fail(AES_EINVAL, "nr must be 10, 12 or 14, got %d", nr);
    if (rk == nullptr || iv == nullptr)
        return fail(AES_EINVAL, "null round-key or counter pointer");
    if (nbytes == 0)
        return AES_OK;
    if (in == nullptr || out == nullptr)
        return fail(AES_EINVAL, "null buffer pointer with nbytes=%zu", nbytes);
    if (nbytes > (SIZE_MAX >> 1))
        return fail(AES_EINVAL, "nbytes=%zu too large", nbytes);
    if ((reinterpret_cast<uintptr_t>(in) | reinterpret_cast<uintptr_t>(out)) & 15u)
        return fail(AES_EALIGN, "in/out must be 16-byte aligned");
    if (ranges_partially_overlap(in, out, (uint64_t)nbytes))
        return fail(AES_EINVAL, "in and out overlap without being the same buffer");
    int rc = check_variant(v);
    if (rc != AES_OK)
        return rc;
    if (v->placement == AES_PLACEMENT_BITSLICED || v->bpt == AES_BPT_COLUMN)
        return fail(AES_EINVAL, "CTR runs on the whole-state table kernels only (no bitsliced or column variant)");
    // c0 = iv + block_offset as a 128-bit big-endian sum
    Counter128 c0{0, 0};
    for (int i = 0; i < 8; ++i) {
        c0.hi = (c0.hi << 8) | iv[i];
        c0.lo = (c0.lo << 8) | iv[8 + i];
    }
    const uint64_t lo = c0.lo + block_offset;
    c0.hi += lo < c0.lo ? 1u : 0u;
    c0.lo = lo;
    RoundKeys keys{};
    std::memcpy(keys.w, rk, sizeof(uint32_t) * 4 * (nr + 1));
    int cus = device_cu_count();
    if (cus <= 0)
        return fail(AES_EHIP, "cannot query the current HIP device");
    LaunchShape shape{v->bpt, v->wg, v->grid};
    hipError_t e = launch_ctr(shape, v->placement, nr, in, out, nbytes, c0, keys, cus, static_cast<hipStream_t>(stream));
    if (e != hipSuccess)
        return fail_hip(e, "CTR kernel launch");
    return AES_OK;
}

int run_cbc_decrypt(const uint32_t* rk, int nr, const uint8_t* iv, const void* in, void* out, size_t nblocks,
                    const aes_variant* v, void* stream)
{
    if (!valid_nr(nr))
        return fail(AES_EINVAL, "nr must be 10, 12 or 14, got %d", nr);
    if (rk == nullptr || iv == nullptr)
        return fail(AES_EINVAL, "null round-key or initialisation-vector pointer");
    if (nblocks == 0)
        return AES_OK;
    int rc = check_buffers(in, out, nblocks);
    if (rc != AES_OK)
        return rc;
    if (in == out)
        return fail(AES_EINVAL, "CBC decryption cannot run in place (block b reads ciphertext block b - 1)");
    rc = check_variant(v);
    if (rc != AES_OK)
        return rc;
    if (v->placement == AES_PLACEMENT_BITSLICED || v->bpt == AES_BPT_COLUMN)
        return fail(AES_EINVAL,
                    "CBC decryption runs on the whole-state table kernels only (no bitsliced or column variant)");
    RoundKeys keys{};
    std::memcpy(keys.w, rk, sizeof(uint32_t) * 4 * (nr + 1));
    int cus = device_cu_count();
    if (cus <= 0)
        return fail(AES_EHIP, "cannot query the current HIP device");
    LaunchShape shape{v->bpt, v->wg, v->grid};
    hipError_t e = launch_cbc_decrypt(shape, v->placement, nr, in, out, nblocks, iv, keys, cus,
                                      static_cast<hipStream_t>(stream));
    if (e != hipSuccess)
        return fail_hip(e, "CBC kernel launch");
    return AES_OK;
}

// Shape of aes_cbc_encrypt_msgs when the caller names none, on the 4-table
// placement (one workgroup per CU).  With at least 8 one-lane-per-message
// waves per CU (64 messages each) the lanes walk whole states, 8 blocks (one
// 128-byte line) per load and store; with fewer, a block's rounds are the
// bound and four lanes share a message (AES_BPT_COLUMN, 16 messages per
// wave), which shortens them.  Workgroups are just large enough to give
// every CU the same number of waves, up to 1024 threads, so a short list
// still spreads over all CUs instead of filling a few.
aes_variant cbc_msgs_default(size_t nmsgs, int cus)
{
    const uint64_t c = cus > 0 ? (uint64_t)cus : 256u;
    const bool quads = (nmsgs + 63u) / 64u < 8u * c;
    const uint64_t waves = quads ? (nmsgs + 15u) / 16u : (nmsgs + 63u) / 64u;
    const uint64_t per_cu = (waves + c - 1) / c;
    const int wg = (int)std::min<uint64_t>(1024u, 64u * std::max<uint64_t>(per_cu, 1u));
    return aes_variant{quads ? AES_BPT_COLUMN : 8, wg, AES_PLACEMENT_TTABLE4, 0};
}

// Shape of aes_cbc_decrypt_msgs when the caller names none, on 4 tables: one
// wave per message (2 blocks per lane per unit) when the input arena averages
// at least 64 blocks per message, so that a wave's lanes all have blocks,
// else one message per lane with 4 independent blocks at a time; workgroups
// just large enough to give every CU the same number of waves, up to 1024.
aes_variant cbc_dec_msgs_default(size_t nmsgs, size_t in_blocks, int cus)
{
    const uint64_t c = cus > 0 ? (uint64_t)cus : 256u;
    const bool wave = nmsgs > 0 && in_blocks / nmsgs >= 64u;
    const uint64_t waves = wave ? nmsgs : (nmsgs + 63u) / 64u;
    const uint64_t per_cu = (waves + c - 1) / c;
    const int wg = (int)std::min<uint64_t>(1024u, 64u * std::max<uint64_t>(per_cu, 1u));
    return aes_variant{wave ? AES_BPT_WAVE_MSG + 2 : 4, wg, AES_PLACEMENT_TTABLE4, 0};
}

// Encryption (decrypt == false) or decryption of a CBC message set; v ==
// nullptr: the default shape for this many messages.
int run_cbc_msgs(bool decrypt, const uint32_t* rk, int nr, const aes_cbc_msg* msgs_dev, size_t nmsgs,
                 const void* in_base, size_t in_blocks, void* out_base, size_t out_blocks, uint32_t* rejected_dev,
                 const aes_variant* v, void* stream)
{
    if (!valid_nr(nr))
        return fail(AES_EINVAL, "nr must be 10, 12 or 14, got %d", nr);
    if (rk == nullptr)
        return fail(AES_EINVAL, "null round-key pointer");
    if (nmsgs == 0)
        return AES_OK;
    if (msgs_dev == nullptr || in_base == nullptr || out_base == nullptr)
        return fail(AES_EINVAL, "null message list or arena with nmsgs=%zu", nmsgs);
    if (nmsgs > (SIZE_MAX / sizeof(aes_cbc_msg)))
        return fail(AES_EINVAL, "nmsgs=%zu too large", nmsgs);
    if ((reinterpret_cast<uintptr_t>(msgs_dev) | reinterpret_cast<uintptr_t>(in_base) |
         reinterpret_cast<uintptr_t>(out_base)) & 15u)
        return fail(AES_EALIGN, "message list and arenas must be 16-byte aligned");
    if (reinterpret_cast<uintptr_t>(rejected_dev) & 3u)
        return fail(AES_EALIGN, "the rejected counter must be 4-byte aligned");
    if (in_blocks > (SIZE_MAX >> 5) || out_blocks > (SIZE_MAX >> 5))
        return fail(AES_EINVAL, "arena sizes too large (%zu / %zu blocks)", in_blocks, out_blocks);
    // each arena with its own length: only the very same arena may be shared
    const uintptr_t ib = reinterpret_cast<uintptr_t>(in_base), ob = reinterpret_cast<uintptr_t>(out_base);
    if (ib != ob && ib < ob + (uint64_t)out_blocks * 16u && ob < ib + (uint64_t)in_blocks * 16u)
        return fail(AES_EINVAL, "in and out arenas overlap without being the same buffer");
    if (v != nullptr) {
        if (decrypt && v->bpt != 1 && v->bpt != 2 && v->bpt != 4 && v->bpt != AES_BPT_WAVE_MSG + 1 &&
            v->bpt != AES_BPT_WAVE_MSG + 2)
            return fail(AES_EINVAL, "bpt must be 1, 2 or 4 (one message per lane) or AES_BPT_WAVE_MSG + 1 or 2 "
                                    "(one wave per message), got %d", v->bpt);
        if (!decrypt && v->bpt != AES_BPT_COLUMN && v->bpt != 1 && v->bpt != 2 && v->bpt != 4 && v->bpt != 8)
            return fail(AES_EINVAL,
                        "bpt (blocks a lane loads at once) must be 1, 2, 4 or 8, or AES_BPT_COLUMN, got %d", v->bpt);
        aes_variant shape_only = *v;
        shape_only.bpt = 1;
        int rc = check_variant(&shape_only);
        if (rc != AES_OK)
            return rc;
        if (v->placement == AES_PLACEMENT_BITSLICED)
            return fail(AES_EINVAL, "CBC message sets run on the table placements only (not bitsliced)");
    }
    RoundKeys keys{};
    std::memcpy(keys.w, rk, sizeof(uint32_t) * 4 * (nr + 1));
    int cus = device_cu_count();
    if (cus <= 0)
        return fail(AES_EHIP, "cannot query the current HIP device");
    const aes_variant chosen =
        v != nullptr ? *v : decrypt ? cbc_dec_msgs_default(nmsgs, in_blocks, cus) : cbc_msgs_default(nmsgs, cus);
    v = &chosen;
    LaunchShape shape{v->bpt, v->wg, v->grid};
    hipError_t e =
        decrypt ? launch_cbc_decrypt_msgs(shape, v->placement, nr, msgs_dev, nmsgs, in_base, in_blocks, out_base,
                                          out_blocks, rejected_dev, keys, cus, static_cast<hipStream_t>(stream))
                : launch_cbc_encrypt_msgs(shape, v->placement, nr, msgs_dev, nmsgs, in_base, in_blocks, out_base,
                                          out_blocks, rejected_dev, keys, cus, static_cast<hipStream_t>(stream));
    if (e != hipSuccess)
        return fail_hip(e, decrypt ? "CBC decryption kernel launch" : "CBC encryption kernel launch");
    return AES_OK;
}

// Workgroups of a batch launch at most: cfg.grid, or as many as fit on every
// CU at once for the configured variant.
int batch_max_grid(const aes_batch_config& c, int* out)
{
    if (c.bpt != 1 && c.bpt != 2 && c.bpt != 4)
        return fail(AES_EINVAL, "bpt must be 1, 2 or 4, got %d", c.bpt);
    if (c.wg < 64 || c.wg > 1024 || c.wg % 64)
        return fail(AES_EINVAL, "workgroup size must be a multiple of 64 in [64, 1024], got %d", c.wg);
    if (c.placement != AES_PLACEMENT_TTABLE4 && c.placement != AES_PLACEMENT_TTABLE2 &&
        c.placement != AES_PLACEMENT_TTABLE1)
        return fail(AES_EINVAL, "the batch kernel takes the table placements 0, 1 or 2, got %d", c.placement);
    if (c.grid < 0)
        return fail(AES_EINVAL, "grid must be >= 0 (0 = as many workgroups as fit at once), got %d", c.grid);
    if (c.grid > 0) {
        *out = c.grid;
        return AES_OK;
    }
    int cus = device_cu_count();
    if (cus <= 0)
        return fail(AES_EHIP, "cannot query the current HIP device");
    int per_cu = 0;
    hipError_t e = batch_groups_per_cu(c.bpt, c.placement, c.wg, &per_cu);
    if (e != hipSuccess)
        return fail_hip(e, "batch kernel occupancy query");
    *out = cus * per_cu;
    return AES_OK;
}

// Arguments of one batch launch, checked; the caller supplies the counters.
struct BatchLaunch {
    BatchArgs args;
    int bpt, wg, grid, placement;
};

int check_batch(const aes_work_item* items_dev, size_t n_enc, size_t n_dec, const uint32_t* key_table_dev,
                size_t n_slots, const void* in_base, size_t in_blocks, void* out_base, size_t out_blocks,
                const aes_batch_config* cfg, BatchLaunch* out)
{
    if (n_enc > UINT32_MAX || n_dec > UINT32_MAX - n_enc || n_slots > UINT32_MAX)
        return fail(AES_ERANGE, "work list or key table too large");
    if (items_dev == nullptr || key_table_dev == nullptr || in_base == nullptr || out_base == nullptr)
        return fail(AES_EINVAL, "null pointer argument");
    if ((reinterpret_cast<uintptr_t>(in_base) | reinterpret_cast<uintptr_t>(out_base)) & 15u)
        return fail(AES_EALIGN, "in/out arenas must be 16-byte aligned");
    if ((reinterpret_cast<uintptr_t>(items_dev) & 7u) || (reinterpret_cast<uintptr_t>(key_table_dev) & 3u))
        return fail(AES_EALIGN, "work list / key table / counters misaligned");
    if (in_blocks > (SIZE_MAX >> 5) || out_blocks > (SIZE_MAX >> 5))
        return fail(AES_EINVAL, "arena sizes too large (%zu / %zu blocks)", in_blocks, out_blocks);
    // Each arena with its own length: only the very same arena (in place) may
    // be shared; any other overlap would let items read blocks others write.
    const uintptr_t ib = reinterpret_cast<uintptr_t>(in_base), ob = reinterpret_cast<uintptr_t>(out_base);
    if (ib != ob && ib < ob + (uint64_t)out_blocks * 16u && ob < ib + (uint64_t)in_blocks * 16u)
        return fail(AES_EINVAL, "in and out arenas overlap without being the same buffer");
    aes_batch_config c{1, 1024, 0, -1, AES_PLACEMENT_TTABLE4};
    if (cfg)
        c = *cfg;
    int max_grid = 0;
    int rc = batch_max_grid(c, &max_grid);
    if (rc != AES_OK)
        return rc;
    int grid = 0, enc_groups = 0;
    // the item counts stand in for the byte shares (the items live on the device)
    batch_grid(n_enc, n_dec, n_enc, n_enc + n_dec, c.wg, max_grid, c.enc_groups, &grid, &enc_groups);
    out->args = BatchArgs{reinterpret_cast<const WorkItem*>(items_dev), (uint32_t)n_enc, (uint32_t)n_dec,
                          key_table_dev, (uint32_t)n_slots, in_base, out_base, (uint64_t)in_blocks,
                          (uint64_t)out_blocks, nullptr, (uint32_t)enc_groups};
    out->bpt = c.bpt;
    out->wg = c.wg;
    out->grid = grid;
    out->placement = c.placement;
    return AES_OK;
}

}  // namespace

int device_cu_count()
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64)
        return -1;
    int v = g_cu_count[dev].load(std::memory_order_relaxed);
    if (v > 0)
        return v;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || v <= 0)
        return -1;
    g_cu_count[dev].store(v, std::memory_order_relaxed);
    return v;
}

}  // namespace aesgpu

using namespace aesgpu;

static_assert(sizeof(aes_work_item) == sizeof(WorkItem), "work item layout");
static_assert(sizeof(aes_cbc_msg) == 48 && offsetof(aes_cbc_msg, iv) == 32, "CBC message layout");
static_assert(offsetof(aes_work_item, nblocks) == offsetof(WorkItem, nblocks), "work item layout");
static_assert(offsetof(aes_work_item, key_slot) == offsetof(WorkItem, key_slot), "work item layout");

extern "C" {

const char* aes_last_error(void) { return g_err; }

int aes_expand_key(const uint8_t* key, int keybits, uint32_t* rk_enc, uint32_t* rk_dec, int* nr_out)
{
    const int nr = rounds_for_bits(keybits);
    if (nr < 0)
        return fail(AES_EINVAL, "keybits must be 128, 192 or 256, got %d", keybits);
    if (key == nullptr)
        return fail(AES_EINVAL, "null key pointer");
    const int nk = keybits / 32, total = 4 * (nr + 1);
    uint32_t w[AES_MAX_ROUND_KEY_WORDS];
    for (int i = 0; i < nk; ++i)
        w[i] = uint32_t(key[4 * i]) | (uint32_t(key[4 * i + 1]) << 8) | (uint32_t(key[4 * i + 2]) << 16) |
               (uint32_t(key[4 * i + 3]) << 24);
    uint32_t rcon = 1;
    for (int i = nk; i < total; ++i) {
        uint32_t t = w[i - 1];
        if (i % nk == 0) {
            t = sub_word((t >> 8) | (t << 24)) ^ rcon;  // RotWord on a little-endian word is a right rotation
            rcon = ((rcon << 1) ^ ((rcon & 0x80) ? 0x1b : 0)) & 0xff;
        } else if (nk == 8 && i % nk == 4) {
            t = sub_word(t);
        }
        w[i] = w[i - nk] ^ t;
    }
    if (rk_enc)
        std::memcpy(rk_enc, w, sizeof(uint32_t) * total);
    if (rk_dec) {
        // equivalent inverse cipher: round order reversed, InvMixColumns on rounds 1..Nr-1
        for (int j = 0; j < 4; ++j) {
            rk_dec[j] = w[4 * nr + j];
            rk_dec[4 * nr + j] = w[j];
        }
        for (int r = 1; r < nr; ++r)
            for (int j = 0; j < 4; ++j)
                rk_dec[4 * r + j] = inv_mix_column(w[4 * (nr - r) + j]);
    }
    if (nr_out)
        *nr_out = nr;
    return AES_OK;
}

int aes_key_slot(const uint8_t* key, int keybits, uint32_t* slot)
{
    if (slot == nullptr)
        return fail(AES_EINVAL, "null slot pointer");
    std::memset(slot, 0, sizeof(uint32_t) * AES_KEY_SLOT_WORDS);
    int nr = 0;
    int rc = aes_expand_key(key, keybits, slot + AES_KEY_SLOT_ENC, slot + AES_KEY_SLOT_DEC, &nr);
    if (rc != AES_OK)
        return rc;
    slot[AES_KEY_SLOT_NR] = (uint32_t)nr;
    return AES_OK;
}

int aes_ecb_encrypt(const uint32_t* rk, int nr, const void* in, void* out, size_t nblocks, void* stream)
{
    aes_variant v;
    if (!valid_nr(nr))
        return fail(AES_EINVAL, "nr must be 10, 12 or 14, got %d", nr);
    aes_tune_get(nr, 0, nblocks, &v);
    return run_ecb(rk, nr, false, in, out, nblocks, &v, stream);
}

int aes_ecb_decrypt(const uint32_t* rk, int nr, const void* in, void* out, size_t nblocks, void* stream)
{
    aes_variant v;
    if (!valid_nr(nr))
        return fail(AES_EINVAL, "nr must be 10, 12 or 14, got %d", nr);
    aes_tune_get(nr, 1, nblocks, &v);
    return run_ecb(rk, nr, true, in, out, nblocks, &v, stream);
}

int aes_ecb_crypt_variant(const uint32_t* rk, int nr, int decrypt, const void* in, void* out, size_t nblocks,
                          const aes_variant* variant, void* stream)
{
    if (variant == nullptr)
        return fail(AES_EINVAL, "null variant");
    return run_ecb(rk, nr, decrypt != 0, in, out, nblocks, variant, stream);
}

int aes_ctr_crypt(const uint32_t* rk, int nr, const uint8_t* iv, uint64_t block_offset, const void* in, void* out,
                  size_t nbytes, void* stream)
{
    aes_variant v;
    if (!valid_nr(nr))
        return fail(AES_EINVAL, "nr must be 10, 12 or 14, got %d", nr);
    aes_tune_get(nr, 0, (nbytes + 15u) / 16u, &v);
    table_variant(&v);
    return run_ctr(rk, nr, iv, block_offset, in, out, nbytes, &v, stream);
}

int aes_ctr_crypt_variant(const uint32_t* rk, int nr, const uint8_t* iv, uint64_t block_offset, const void* in,
                          void* out, size_t nbytes, const aes_variant* variant, void* stream)
{
    if (variant == nullptr)
        return fail(AES_EINVAL, "null variant");
    return run_ctr(rk, nr, iv, block_offset, in, out, nbytes, variant, stream);
}

int aes_cbc_decrypt(const uint32_t* rk, int nr, const uint8_t* iv, const void* in, void* out, size_t nblocks,
                    void* stream)
{
    aes_variant v;
    if (!valid_nr(nr))
        return fail(AES_EINVAL, "nr must be 10, 12 or 14, got %d", nr);
    aes_tune_get(nr, 1, nblocks, &v);
    table_variant(&v);
    return run_cbc_decrypt(rk, nr, iv, in, out, nblocks, &v, stream);
}

int aes_cbc_decrypt_variant(const uint32_t* rk, int nr, const uint8_t* iv, const void* in, void* out, size_t nblocks,
                            const aes_variant* variant, void* stream)
{
    if (variant == nullptr)
        return fail(AES_EINVAL, "null variant");
    return run_cbc_decrypt(rk, nr, iv, in, out, nblocks, variant, stream);
}

int aes_cbc_encrypt_msgs(const uint32_t* rk, int nr, const aes_cbc_msg* msgs_dev, size_t nmsgs, const void* in_base,
                         size_t in_blocks, void* out_base, size_t out_blocks, uint32_t* rejected_dev, void* stream)
{
    return run_cbc_msgs(false, rk, nr, msgs_dev, nmsgs, in_base, in_blocks, out_base, out_blocks, rejected_dev,
                        nullptr, stream);
}

int aes_cbc_encrypt_msgs_variant(const uint32_t* rk, int nr, const aes_cbc_msg* msgs_dev, size_t nmsgs,
                                 const void* in_base, size_t in_blocks, void* out_base, size_t out_blocks,
                                 uint32_t* rejected_dev, const aes_variant* variant, void* stream)
{
    if (variant == nullptr)
        return fail(AES_EINVAL, "null variant");
    return run_cbc_msgs(false, rk, nr, msgs_dev, nmsgs, in_base, in_blocks, out_base, out_blocks, rejected_dev,
                        variant, stream);
}

int aes_cbc_decrypt_msgs(const uint32_t* rk, int nr, const aes_cbc_msg* msgs_dev, size_t nmsgs, const void* in_base,
                         size_t in_blocks, void* out_base, size_t out_blocks, uint32_t* rejected_dev, void* stream)
{
    return run_cbc_msgs(true, rk, nr, msgs_dev, nmsgs, in_base, in_blocks, out_base, out_blocks, rejected_dev,
                        nullptr, stream);
}

int aes_cbc_decrypt_msgs_variant(const uint32_t* rk, int nr, const aes_cbc_msg* msgs_dev, size_t nmsgs,
                                 const void* in_base, size_t in_blocks, void* out_base, size_t out_blocks,
                                 uint32_t* rejected_dev, const aes_variant* variant, void* stream)
{
    if (variant == nullptr)
        return fail(AES_EINVAL, "null variant");
    return run_cbc_msgs(true, rk, nr, msgs_dev, nmsgs, in_base, in_blocks, out_base, out_blocks, rejected_dev,
                        variant, stream);
}

int aes_tune_set(int nr, int decrypt, size_t nblocks, const aes_variant* v)
{
    if (!valid_nr(nr))
        return fail(AES_EINVAL, "nr must be 10, 12 or 14, got %d", nr);
    if (v == nullptr)
        return fail(AES_EINVAL, "null variant");
    int rc = check_variant(v);
    if (rc != AES_OK)
        return rc;
    TuneEntry& t = g_tune[nr_index(nr)][decrypt ? 1 : 0][size_bucket(nblocks)];
    t.bpt.store(v->bpt);
    t.wg.store(v->wg);
    t.placement.store(v->placement);
    return AES_OK;
}

int aes_tune_get(int nr, int decrypt, size_t nblocks, aes_variant* v)
{
    if (!valid_nr(nr))
        return fail(AES_EINVAL, "nr must be 10, 12 or 14, got %d", nr);
    if (v == nullptr)
        return fail(AES_EINVAL, "null variant");
    const TuneEntry& t = g_tune[nr_index(nr)][decrypt ? 1 : 0][size_bucket(nblocks)];
    v->bpt = t.bpt.load();
    v->wg = t.wg.load();
    v->placement = t.placement.load();
    v->grid = 0;
    return AES_OK;
}

int aes_size_bucket(size_t nblocks) { return size_bucket(nblocks); }

int aes_batch_plan(const aes_msg* msgs, size_t nmsgs, uint32_t chunk_blocks, aes_work_item* items, size_t cap,
                   size_t* n_enc, size_t* n_dec)
{
    if (n_enc == nullptr || n_dec == nullptr)
        return fail(AES_EINVAL, "null count pointer");
    *n_enc = *n_dec = 0;
    if (nmsgs > 0 && msgs == nullptr)
        return fail(AES_EINVAL, "null message array with nmsgs=%zu", nmsgs);
    if (chunk_blocks == 0 || chunk_blocks > AES_MAX_ITEM_BLOCKS)
        return fail(AES_EINVAL, "chunk_blocks must be in [1, %u], got %u", AES_MAX_ITEM_BLOCKS, chunk_blocks);
    // Count first (the counts are returned even when cap is too small); every
    // sum is checked, so the fill below writes exactly the counted items.
    uint64_t ne = 0, nd = 0;
    for (size_t i = 0; i < nmsgs; ++i) {
        const aes_msg& m = msgs[i];
        if (m.in_block > UINT64_MAX - m.nblocks || m.out_block > UINT64_MAX - m.nblocks)
            return fail(AES_EINVAL, "message %zu: block range passes 2^64", i);
        const uint64_t c = m.nblocks / chunk_blocks + (m.nblocks % chunk_blocks != 0);
        if (c > UINT32_MAX - (ne + nd))
            return fail(AES_ERANGE, "more than 2^32 - 1 work items");
        (m.decrypt ? nd : ne) += c;
    }
    *n_enc = (size_t)ne;
    *n_dec = (size_t)nd;
    if (ne + nd > cap || (ne + nd > 0 && items == nullptr))
        return fail(AES_ERANGE, "work list needs %llu items, capacity is %zu", (unsigned long long)(ne + nd), cap);
    size_t ie = 0, id = (size_t)ne;
    for (size_t i = 0; i < nmsgs; ++i) {
        const aes_msg& m = msgs[i];
        const uint64_t c = m.nblocks / chunk_blocks + (m.nblocks % chunk_blocks != 0);
        for (uint64_t k = 0; k < c; ++k) {
            const uint64_t off = k * chunk_blocks;  // < nblocks: no overflow
            aes_work_item& it = items[m.decrypt ? id++ : ie++];
            it.in_block = m.in_block + off;
            it.out_block = m.out_block + off;
            it.nblocks = (uint32_t)std::min<uint64_t>(chunk_blocks, m.nblocks - off);
            it.key_slot = m.key_slot;
        }
    }
    return AES_OK;
}

int aes_ecb_batch(const aes_work_item* items_dev, size_t n_enc, size_t n_dec, const uint32_t* key_table_dev,
                  size_t n_slots, const void* in_base, size_t in_blocks, void* out_base, size_t out_blocks,
                  uint32_t* counters_dev, const aes_batch_config* cfg, void* stream)
{
    if (n_enc + n_dec == 0)
        return AES_OK;
    if (counters_dev == nullptr)
        return fail(AES_EINVAL, "null pointer argument");
    if (reinterpret_cast<uintptr_t>(counters_dev) & 3u)
        return fail(AES_EALIGN, "work list / key table / counters misaligned");
    BatchLaunch b;
    int rc = check_batch(items_dev, n_enc, n_dec, key_table_dev, n_slots, in_base, in_blocks, out_base, out_blocks,
                         cfg, &b);
    if (rc != AES_OK)
        return rc;
    b.args.counters = counters_dev;
    hipError_t e = launch_batch(b.args, b.bpt, b.placement, b.grid, b.wg, static_cast<hipStream_t>(stream));
    if (e != hipSuccess)
        return fail_hip(e, "batch kernel launch");
    return AES_OK;
}

int aes_ecb_batch_noalloc(const aes_work_item* items_dev, size_t n_enc, size_t n_dec, const uint32_t* key_table_dev,
                          size_t n_slots, const void* in_base, size_t in_blocks, void* out_base, size_t out_blocks,
                          const aes_batch_config* cfg, void* stream)
{
    if (n_enc + n_dec == 0)
        return AES_OK;
    BatchLaunch b;
    int rc = check_batch(items_dev, n_enc, n_dec, key_table_dev, n_slots, in_base, in_blocks, out_base, out_blocks,
                         cfg, &b);
    if (rc != AES_OK)
        return rc;
    hipError_t e = launch_batch_noalloc(b.args, b.bpt, b.placement, b.grid, b.wg, static_cast<hipStream_t>(stream));
    if (e != hipSuccess)
        return fail_hip(e, "batch kernel launch (no-allocation form)");
    return AES_OK;
}

int aes_batch_max_grid(const aes_batch_config* cfg, int* grid)
{
    if (grid == nullptr)
        return fail(AES_EINVAL, "null grid pointer");
    aes_batch_config c{1, 1024, 0, -1, AES_PLACEMENT_TTABLE4};
    if (cfg)
        c = *cfg;
    return batch_max_grid(c, grid);
}

int aes_host_tables(uint8_t* sbox, uint8_t* inv_sbox, uint32_t* te0, uint32_t* td0)
{
    if (sbox)
        std::memcpy(sbox, kHostTables.sbox, 256);
    if (inv_sbox)
        std::memcpy(inv_sbox, kHostTables.inv_sbox, 256);
    if (te0)
        std::memcpy(te0, kHostTables.te0, sizeof(kHostTables.te0));
    if (td0)
        std::memcpy(td0, kHostTables.td0, sizeof(kHostTables.td0));
    return AES_OK;
}

int aes_roof_probe(int which, uint32_t iters, void* out_dev, size_t out_bytes, uint64_t* work, void* stream)
{
    if (which != AES_PROBE_LDS && which != AES_PROBE_VALU)
        return fail(AES_EINVAL, "unknown probe %d", which);
    if (iters == 0 || iters > (1u << 24))
        return fail(AES_EINVAL, "iters must be in [1, 2^24], got %u", iters);
    if (out_dev == nullptr)
        return fail(AES_EINVAL, "null probe output");
    int cus = device_cu_count();
    if (cus <= 0)
        return fail(AES_EHIP, "cannot query the current HIP device");
    const uint64_t threads = (uint64_t)cus * 2u * 1024u;
    if (out_dev == nullptr || out_bytes < threads * 4u)
        return fail(AES_EINVAL, "out_dev must hold %llu bytes (one word per probe thread)",
                    (unsigned long long)(threads * 4u));
    if (reinterpret_cast<uintptr_t>(out_dev) & 3u)
        return fail(AES_EALIGN, "out_dev must be 4-byte aligned");
    if (work != nullptr)
        *work = threads * 16u * iters;  // lookups or VALU lane-operations
    hipError_t e = launch_probe(which, static_cast<uint32_t*>(out_dev), iters, cus, static_cast<hipStream_t>(stream));
    if (e != hipSuccess)
        return fail_hip(e, "probe launch");
    return AES_OK;
}

int aes_device_copy(const void* in, void* out, size_t nbytes, void* stream)
{
    if (nbytes == 0)
        return AES_OK;
    if (in == nullptr || out == nullptr)
        return fail(AES_EINVAL, "null buffer pointer");
    if (nbytes % 16 || ((reinterpret_cast<uintptr_t>(in) | reinterpret_cast<uintptr_t>(out)) & 15u))
        return fail(AES_EALIGN, "copy needs 16-byte aligned buffers and a multiple of 16 bytes");
    int cus = device_cu_count();
    if (cus <= 0)
        return fail(AES_EHIP, "cannot query the current HIP device");
    hipError_t e = launch_copy(in, out, nbytes / 16, cus * 4, static_cast<hipStream_t>(stream));
    if (e != hipSuccess)
        return fail_hip(e, "copy kernel launch");
    return AES_OK;
}

}  // extern "C"
