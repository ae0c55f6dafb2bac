// aes_pipe.cpp -- host-inclusive path (aes_pipe_*): host buffer in, host
// buffer out.
//
// The paper times files in host memory (section 5, Tables 4-5), so its GPU
// figures include the copies over the host link.  This path runs the same
// kernels on host buffers: the buffer is cut into pieces of at most a chunk
// (smaller when that gives every slot two pieces), and piece i goes through
// slot i mod N (one stream, one device chunk, one pinned staging chunk per
// slot): host -> device copy, the kernel in place on the device chunk,
// device -> host copy, an event.  Pieces on different slots overlap, so
// copies in both directions and kernels run at once.  Pageable buffers go
// through the slot's pinned chunk (a CPU copy on each side); buffers the
// caller allocated pinned (AES_PIPE_HOST_PINNED) are copied directly.  The
// caller provides the device workspace and the pinned staging; the pipe
// creates its streams and events and one small pinned page for a completion
// word.
//
// A buffer of at most one chunk (and kDirectMax) skips the copies over the
// host link: the kernel runs on host memory the device maps, the caller's
// pinned buffers themselves (if 16-byte aligned) or the slot's pinned chunk.  That takes one
// launch instead of two copies and a launch (from 1 KB to 150 KB about 19 us
// against 24-46 us when both waited through the runtime).  A host range
// qualifies only if it lies inside one
// page-locked allocation that the device maps at the same address
// (hipPointerGetAttributes, hipMemGetAddressRange); anything else takes the
// copy path.  The direct path learns that its launch finished from a word
// that a one-thread kernel behind it writes into a pinned page of the pipe
// (aes_host_word.hip), which the calling thread polls: the runtime's own
// completion wait arrives about 5 us later.  A launch not seen finished
// within kWordWaitSeconds is waited for through the runtime, which also
// reports a failed kernel.  A pageable buffer of 512 KiB or more on this path
// goes through the staging in pieces (run_staged_pieces), so the CPU copies
// of one piece overlap the kernel of another.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>

#include <cstdint>
#include <cstring>
#include <mutex>
#include <new>
#include <vector>

#include "../../include/aesgpu.h"
#include "aes_host_word.hpp"
#include "aes_internal.hpp"

namespace aesgpu {
namespace {

struct Slot {
    hipStream_t stream = nullptr;
    hipEvent_t event = nullptr;
    uint8_t* dev = nullptr;
    uint8_t* pin = nullptr;
    // chunk in flight on this slot, whose output still has to leave the pinned chunk
    bool pending = false;
    uint64_t off = 0, len = 0;
};

}  // namespace
}  // namespace aesgpu

struct aes_pipe {
    int device = 0;
    uint64_t chunk = 0;
    bool has_pinned = false;
    bool staging_mapped = false;  // the pinned staging is addressable by the kernels
    uint32_t* word = nullptr;     // pinned page of the pipe: the direct path's completion word
    uint32_t* word_dev = nullptr; // its device address
    uint32_t seq = 0;             // last value a completion kernel was asked to store
    std::vector<aesgpu::Slot> slots;
    std::mutex mu;  // one run at a time per pipe
};

namespace aesgpu {

// [p, p + n) lies inside one page-locked host allocation that the device maps
// at the same address, so a kernel may read and write it.  A failed query
// leaves no error behind for the next launch's hipGetLastError.
bool host_range_device_mapped(const void* p, uint64_t n)
{
    hipPointerAttribute_t a{};
    if (hipPointerGetAttributes(&a, p) != hipSuccess) {
        (void)hipGetLastError();
        return false;
    }
    if (a.type != hipMemoryTypeHost || a.devicePointer != p)
        return false;
    hipDeviceptr_t base = nullptr;
    size_t size = 0;
    if (hipMemGetAddressRange(&base, &size, const_cast<void*>(p)) != hipSuccess) {
        (void)hipGetLastError();
        return false;
    }
    const uintptr_t b = reinterpret_cast<uintptr_t>(base), q = reinterpret_cast<uintptr_t>(p);
    return q >= b && n <= size && q - b <= size - n;
}

}  // namespace aesgpu

using namespace aesgpu;

namespace {

void destroy_slots(aes_pipe* p)
{
    for (auto& s : p->slots) {
        if (s.event)
            hipEventDestroy(s.event);
        if (s.stream)
            hipStreamDestroy(s.stream);
    }
    p->slots.clear();
    if (p->word != nullptr)
        hipHostFree(p->word);
    p->word = p->word_dev = nullptr;
}

// Longest the direct path polls its completion word before it waits through
// the runtime (a kernel that failed never writes the word).
constexpr double kWordWaitSeconds = 2e-3;

// Wait for the work enqueued on `stream` up to and including a completion
// kernel that stores `seq` into *word: poll the word, then the runtime.  The
// pipe's sequence numbers only grow (modulo 2^32) along the stream, so a
// word at or past `seq` means that kernel has run.
hipError_t wait_word(const volatile uint32_t* word, uint32_t seq, hipStream_t stream)
{
    const auto t0 = std::chrono::steady_clock::now();
    for (uint32_t spins = 1;; ++spins) {
        if (static_cast<int32_t>(__atomic_load_n(const_cast<const uint32_t*>(word), __ATOMIC_ACQUIRE) - seq) >= 0)
            return hipSuccess;
        if ((spins & 1023u) == 0 &&
            std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count() > kWordWaitSeconds)
            return hipStreamSynchronize(stream);
    }
}

bool overlap_partial(const void* a, const void* b, uint64_t n)
{
    const uintptr_t x = reinterpret_cast<uintptr_t>(a), y = reinterpret_cast<uintptr_t>(b);
    return x != y && x < y + n && y < x + n;
}

constexpr uint64_t kDirectMax = 4ull << 20;
constexpr uint64_t kMinPiece = 1ull << 20;  // smallest piece a pipelined buffer is cut into

// The kernel for the bytes [off, off + len) of the message, in -> out on stream.
hipError_t launch_piece(int op, int nr, const RoundKeys& keys, const Counter128& c0, uint64_t off, const void* in,
                        void* out, uint64_t len, int cus, hipStream_t stream)
{
    const uint64_t blocks = (len + 15u) / 16u;
    aes_variant v;
    aes_tune_get(nr, op == AES_PIPE_ECB_DECRYPT ? 1 : 0, blocks, &v);
    if (op == AES_PIPE_CTR && v.placement == AES_PLACEMENT_BITSLICED) {
        v.placement = AES_PLACEMENT_TTABLE2;  // CTR runs on the whole-state table kernels
        v.bpt = 2;
        v.wg = 1024;
    }
    if (op == AES_PIPE_CTR && v.bpt == AES_BPT_COLUMN)
        v.bpt = 1;  // the one-column-per-lane variant is ECB only
    const LaunchShape shape{v.bpt, v.wg, 0};
    if (op == AES_PIPE_CTR) {
        Counter128 c = c0;
        const uint64_t lo = c.lo + off / 16u;
        c.hi += lo < c.lo ? 1u : 0u;
        c.lo = lo;
        return launch_ctr(shape, v.placement, nr, in, out, len, c, keys, cus, stream);
    }
    return launch_ecb(shape, v.placement, nr, op == AES_PIPE_ECB_DECRYPT, in, out, blocks, keys, cus, stream);
}

// A staged single-launch buffer is cut into pieces of at least kStagedPiece
// bytes (at most kStagedPieces of them): each is copied into the staging,
// run there, and copied out as soon as its completion word arrives, so the
// CPU copies of one piece overlap the kernel of another.
constexpr uint64_t kStagedPiece = 256u << 10;
constexpr uint64_t kStagedPieces = 4;

hipError_t run_staged_pieces(aes_pipe* p, Slot& s, int op, int nr, const RoundKeys& keys, const Counter128& c0,
                             const uint8_t* src, uint8_t* dst, uint64_t nbytes, int cus)
{
    const uint64_t np = std::min<uint64_t>(kStagedPieces, std::max<uint64_t>(1, nbytes / kStagedPiece));
    const uint64_t plen = ((nbytes + np - 1) / np + 15u) & ~(uint64_t)15u;  // whole blocks: CTR pieces stay aligned
    const uint32_t base = p->seq;
    uint64_t launched = 0, done = 0;
    auto len_of = [&](uint64_t i) { return std::min<uint64_t>(plen, nbytes - i * plen); };
    auto finish_piece = [&](uint64_t i) {
        hipError_t w = wait_word(p->word, base + (uint32_t)(i + 1), s.stream);
        if (w == hipSuccess)
            std::memcpy(dst + i * plen, s.pin + i * plen, len_of(i));
        return w;
    };
    hipError_t e = hipSuccess;
    for (uint64_t i = 0; i * plen < nbytes && e == hipSuccess; ++i) {
        const uint64_t off = i * plen, len = len_of(i);
        std::memcpy(s.pin + off, src + off, len);
        e = launch_piece(op, nr, keys, c0, off, s.pin + off, s.pin + off, len, cus, s.stream);
        if (e != hipSuccess)
            break;
        ++launched;  // in flight from here on: drained below if anything fails
        e = launch_host_word(p->word_dev, ++p->seq, s.stream);
        if (e == hipSuccess && i > 0 && (e = finish_piece(i - 1)) == hipSuccess)
            ++done;
    }
    while (e == hipSuccess && done < launched)
        if ((e = finish_piece(done)) == hipSuccess)
            ++done;
    if (e != hipSuccess && launched > 0)
        (void)hipStreamSynchronize(s.stream);  // nothing of this call still runs on the staging
    return e;
}

// copy the finished chunk of slot s from its pinned chunk to the caller's buffer
int finish(Slot& s, uint8_t* host_out, bool staged)
{
    if (!s.pending)
        return AES_OK;
    hipError_t e = hipEventSynchronize(s.event);
    if (e != hipSuccess)
        return fail_hip(e, "pipe: waiting for a chunk");
    if (staged)
        std::memcpy(host_out + s.off, s.pin, s.len);
    s.pending = false;
    return AES_OK;
}

}  // namespace

static int pipe_create(const aes_pipe_config* cfg, aes_pipe** out)
{
    if (out == nullptr || cfg == nullptr)
        return fail(AES_EINVAL, "null config or output pointer");
    *out = nullptr;
    if (cfg->chunk_bytes == 0 || cfg->chunk_bytes % 16u)
        return fail(AES_EINVAL, "chunk_bytes must be a positive multiple of 16, got %llu",
                    (unsigned long long)cfg->chunk_bytes);
    if (cfg->nslots < 1 || cfg->nslots > AES_PIPE_MAX_SLOTS)
        return fail(AES_EINVAL, "nslots must be in [1, %d], got %d", AES_PIPE_MAX_SLOTS, cfg->nslots);
    if (cfg->chunk_bytes > UINT64_MAX / (uint64_t)cfg->nslots)
        return fail(AES_EINVAL, "nslots * chunk_bytes passes 2^64");
    const uint64_t need = cfg->chunk_bytes * (uint64_t)cfg->nslots;
    if (cfg->dev == nullptr || cfg->dev_bytes < need)
        return fail(AES_EINVAL, "device workspace must hold nslots * chunk_bytes = %llu bytes",
                    (unsigned long long)need);
    if ((reinterpret_cast<uintptr_t>(cfg->dev) & 15u) || (cfg->chunk_bytes & 15u))
        return fail(AES_EALIGN, "device workspace must be 16-byte aligned");
    if (cfg->pinned != nullptr && cfg->pinned_bytes < need)
        return fail(AES_EINVAL, "pinned staging must hold nslots * chunk_bytes = %llu bytes (or be NULL)",
                    (unsigned long long)need);
    aes_pipe* p = new (std::nothrow) aes_pipe;
    if (p == nullptr)
        return fail(AES_ENOMEM, "pipe: out of host memory");
    hipError_t e = hipGetDevice(&p->device);
    if (e != hipSuccess) {
        delete p;
        return fail_hip(e, "pipe: current device");
    }
    p->chunk = cfg->chunk_bytes;
    p->has_pinned = cfg->pinned != nullptr;
    p->staging_mapped = p->has_pinned && host_range_device_mapped(cfg->pinned, need);
    try {
        p->slots.resize((size_t)cfg->nslots);
    } catch (...) {
        delete p;
        throw;
    }
    for (int i = 0; i < cfg->nslots; ++i) {
        Slot& s = p->slots[(size_t)i];
        s.dev = static_cast<uint8_t*>(cfg->dev) + (uint64_t)i * cfg->chunk_bytes;
        s.pin = p->has_pinned ? static_cast<uint8_t*>(cfg->pinned) + (uint64_t)i * cfg->chunk_bytes : nullptr;
        if ((e = hipStreamCreateWithFlags(&s.stream, hipStreamNonBlocking)) != hipSuccess ||
            (e = hipEventCreateWithFlags(&s.event, hipEventDisableTiming)) != hipSuccess) {
            destroy_slots(p);
            delete p;
            return fail_hip(e, "pipe: stream or event creation");
        }
    }
    // the completion word: without a mapped page the direct path waits on an event
    void* page = nullptr;
    if (hipHostMalloc(&page, 256, hipHostMallocMapped | hipHostMallocCoherent) == hipSuccess) {
        void* dev = nullptr;
        if (hipHostGetDevicePointer(&dev, page, 0) == hipSuccess && dev != nullptr) {
            p->word = static_cast<uint32_t*>(page);
            p->word_dev = static_cast<uint32_t*>(dev);
            __atomic_store_n(p->word, 0u, __ATOMIC_RELEASE);
        } else {
            hipHostFree(page);
        }
    }
    (void)hipGetLastError();  // a refused page leaves no error for the next launch
    *out = p;
    return AES_OK;
}

static int pipe_destroy(aes_pipe* p)
{
    if (p == nullptr)
        return AES_OK;
    {
        std::lock_guard<std::mutex> lk(p->mu);
        for (auto& s : p->slots)
            if (s.stream)
                hipStreamSynchronize(s.stream);
        destroy_slots(p);
    }
    delete p;
    return AES_OK;
}

static int pipe_run(aes_pipe* p, int op, const uint32_t* rk, int nr, const uint8_t* iv, const void* host_in,
                    void* host_out, size_t nbytes, int flags)
{
    if (p == nullptr)
        return fail(AES_EINVAL, "null pipe");
    if (op != AES_PIPE_ECB_ENCRYPT && op != AES_PIPE_ECB_DECRYPT && op != AES_PIPE_CTR)
        return fail(AES_EINVAL, "unknown pipe operation %d", op);
    if (nr != 10 && nr != 12 && nr != 14)
        return fail(AES_EINVAL, "nr must be 10, 12 or 14, got %d", nr);
    if (rk == nullptr || (op == AES_PIPE_CTR && iv == nullptr))
        return fail(AES_EINVAL, "null round-key or counter pointer");
    if (op != AES_PIPE_CTR && nbytes % 16u)
        return fail(AES_EINVAL, "ECB takes whole 16-byte blocks, got %zu bytes", nbytes);
    if (nbytes == 0)
        return AES_OK;
    if (host_in == nullptr || host_out == nullptr)
        return fail(AES_EINVAL, "null host buffer with nbytes=%zu", nbytes);
    if (overlap_partial(host_in, host_out, nbytes))
        return fail(AES_EINVAL, "host in and out overlap without being the same buffer");
    const bool staged = !(flags & AES_PIPE_HOST_PINNED);
    if (staged && !p->has_pinned)
        return fail(AES_EINVAL, "pageable host buffers need pinned staging in the pipe config");

    std::lock_guard<std::mutex> lk(p->mu);
    int prev_dev = 0;
    hipGetDevice(&prev_dev);
    if (prev_dev != p->device)
        hipSetDevice(p->device);
    int cus = device_cu_count();
    if (cus <= 0) {
        if (prev_dev != p->device)
            hipSetDevice(prev_dev);
        return fail(AES_EHIP, "cannot query the pipe's device");
    }
    RoundKeys keys{};
    std::memcpy(keys.w, rk, sizeof(uint32_t) * 4 * (nr + 1));
    Counter128 c0{0, 0};
    if (op == AES_PIPE_CTR)
        for (int i = 0; i < 8; ++i) {
            c0.hi = (c0.hi << 8) | iv[i];
            c0.lo = (c0.lo << 8) | iv[8 + i];
        }
    const uint8_t* src = static_cast<const uint8_t*>(host_in);
    uint8_t* dst = static_cast<uint8_t*>(host_out);
    if (nbytes <= p->chunk && nbytes <= kDirectMax) {
        Slot& s = p->slots[0];
        const void* kin = nullptr;
        void* kout = nullptr;
        const bool aligned = ((reinterpret_cast<uintptr_t>(host_in) | reinterpret_cast<uintptr_t>(host_out)) & 15u) == 0;
        if (!staged && aligned && host_range_device_mapped(host_in, nbytes) &&
            host_range_device_mapped(host_out, nbytes)) {
            kin = host_in;
            kout = host_out;
        } else if (staged && p->staging_mapped) {
            kin = kout = s.pin;
        }
        if (kin != nullptr && staged && p->word != nullptr) {
            hipError_t e = run_staged_pieces(p, s, op, nr, keys, c0, src, dst, nbytes, cus);
            const int rc = e == hipSuccess ? AES_OK : fail_hip(e, "pipe: kernel on host memory");
            if (prev_dev != p->device)
                hipSetDevice(prev_dev);
            return rc;
        }
        if (kin != nullptr) {
            int rc = AES_OK;
            if (staged)
                std::memcpy(s.pin, src, nbytes);
            hipError_t e = launch_piece(op, nr, keys, c0, 0, kin, kout, nbytes, cus, s.stream);
            if (e == hipSuccess && p->word != nullptr) {
                const uint32_t seq = ++p->seq;
                e = launch_host_word(p->word_dev, seq, s.stream);
                if (e == hipSuccess)
                    e = wait_word(p->word, seq, s.stream);
            } else if (e == hipSuccess) {
                e = hipEventRecord(s.event, s.stream);
                if (e == hipSuccess)
                    e = hipEventSynchronize(s.event);
            }
            if (e != hipSuccess)
                rc = fail_hip(e, "pipe: kernel on host memory");
            else if (staged)
                std::memcpy(dst, s.pin, nbytes);
            if (prev_dev != p->device)
                hipSetDevice(prev_dev);
            return rc;
        }
    }
    const size_t ns = p->slots.size();
    int rc = AES_OK;
    // Pieces of at most one chunk, and small enough that every slot gets two
    // (1 MiB at least, whole blocks): a buffer of a few chunks still overlaps
    // its copies in and out.
    const uint64_t spread = ((nbytes + 2 * ns - 1) / (2 * ns) + 15u) & ~(uint64_t)15u;
    const uint64_t piece = std::min<uint64_t>(p->chunk, std::max<uint64_t>(spread, kMinPiece));
    const uint64_t npieces = nbytes / piece + (nbytes % piece != 0);
    for (uint64_t index = 0; index < npieces && rc == AES_OK; ++index) {
        const uint64_t off = index * piece;  // < nbytes: no overflow
        Slot& s = p->slots[index % ns];
        rc = finish(s, dst, staged);
        if (rc != AES_OK)
            break;
        const uint64_t len = nbytes - off < piece ? nbytes - off : piece;
        const void* h2d_src = src + off;
        if (staged) {
            std::memcpy(s.pin, src + off, len);
            h2d_src = s.pin;
        }
        hipError_t e = hipMemcpyAsync(s.dev, h2d_src, len, hipMemcpyHostToDevice, s.stream);
        if (e != hipSuccess) {
            rc = fail_hip(e, "pipe: host to device copy");
            break;
        }
        e = launch_piece(op, nr, keys, c0, off, s.dev, s.dev, len, cus, s.stream);
        if (e != hipSuccess) {
            rc = fail_hip(e, "pipe: kernel launch");
            break;
        }
        e = hipMemcpyAsync(staged ? static_cast<void*>(s.pin) : static_cast<void*>(dst + off), s.dev, len,
                           hipMemcpyDeviceToHost, s.stream);
        if (e == hipSuccess)
            e = hipEventRecord(s.event, s.stream);
        if (e != hipSuccess) {
            rc = fail_hip(e, "pipe: device to host copy");
            break;
        }
        s.off = off;
        s.len = len;
        s.pending = true;
    }
    // drain every slot (also after an error, so no copy into the caller's
    // buffers is still running when the call returns)
    for (auto& s : p->slots) {
        const int r = finish(s, dst, staged && rc == AES_OK);
        if (rc == AES_OK)
            rc = r;
        s.pending = false;
    }
    if (prev_dev != p->device)
        hipSetDevice(prev_dev);
    return rc;
}

extern "C" {

int aes_pipe_create(const aes_pipe_config* cfg, aes_pipe** out)
{
    return guarded([&] { return pipe_create(cfg, out); });
}

int aes_pipe_destroy(aes_pipe* p)
{
    return guarded([&] { return pipe_destroy(p); });
}

int aes_pipe_run(aes_pipe* p, int op, const uint32_t* rk, int nr, const uint8_t* iv, const void* host_in,
                 void* host_out, size_t nbytes, int flags)
{
    return guarded([&] { return pipe_run(p, op, rk, nr, iv, host_in, host_out, nbytes, flags); });
}

}  // extern "C"
