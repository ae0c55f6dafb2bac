// aes_serve.cpp -- native continuous-batching request engine (aes_server_*).
//
// A worker thread owns the policy: requests submitted from any thread are
// admitted in arrival order while the device budget (input + output bytes of
// every admitted, unfinished request) and the output arena allow; whenever
// one of the stream slots is free, everything admitted so far is planned into
// work items (same planner as aes_batch_plan), copied to that slot's device
// work list from pinned staging, and run as one persistent batch launch.  A
// work list of at most kDirectItems items is not copied: when the staging is
// host memory the device maps (checked once at creation), the kernel reads
// the items from it, which saves a copy over the host link per light batch.
// Slots are polled with events; a finished request releases its budget at
// once and its output space when the caller releases it (or immediately with
// auto_release).  All device memory (work lists, counters, arenas) comes
// from the caller; the engine creates only streams and events.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstdint>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <new>
#include <thread>
#include <vector>

#include "../../include/aesgpu.h"
#include "aes_batch_signal.hpp"
#include "aes_internal.hpp"

namespace aesgpu {

int device_cu_count();

constexpr size_t kDirectItems = 4096;
// A batch still not seen complete after this long is checked with the runtime
// (which also reports a failure) on every pass of the worker.
constexpr double kStreamCheckSeconds = 0.002;

namespace {

using Clock = std::chrono::steady_clock;

struct Req {
    uint64_t id;
    aes_request r;
    double arrival = 0, admitted = 0, done = 0;
    uint64_t out_block = 0;
    int status = 0;
    int batch = -1;
};

// First-fit allocator over [0, n) blocks with coalescing frees.
class Arena {
public:
    explicit Arena(uint64_t n) : n_(n) { free_[0] = n; }
    bool alloc(uint64_t len, uint64_t* start)
    {
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= len) {
                *start = it->first;
                const uint64_t rest = it->second - len, s = it->first + len;
                free_.erase(it);
                if (rest)
                    free_[s] = rest;
                used_ += len;
                return true;
            }
        }
        return false;
    }
    void release(uint64_t start, uint64_t len)
    {
        used_ -= len;
        auto it = free_.emplace(start, len).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }
    uint64_t used() const { return used_; }
    uint64_t size() const { return n_; }

private:
    uint64_t n_, used_ = 0;
    std::map<uint64_t, uint64_t> free_;
};

struct Slot {
    hipStream_t stream = nullptr;
    hipEvent_t event = nullptr;
    // Completion word in the pinned staging: the batch kernel's last
    // workgroup writes `seq` into it (launch_batch_signal), and the worker
    // sees completion with a plain load instead of an event query.
    uint32_t* done_word = nullptr;
    uint32_t seq = 0;
    double launched = 0;
    aes_work_item* items_dev = nullptr;
    uint32_t* counters_dev = nullptr;
    aes_work_item* staging = nullptr;
    std::vector<Req*> reqs;
    bool busy = false;
    double dry_done = 0;  // dry run: completion time
};

}  // namespace
}  // namespace aesgpu

struct aes_server {
    aes_serve_config cfg{};
    int device = 0;
    int cus = 0;
    int max_grid = 0;  // workgroups per batch launch at most (cfg.grid, or all that fit at once)
    const uint32_t* key_table = nullptr;
    size_t n_slots = 0;
    const void* in_pool = nullptr;
    size_t in_blocks = 0;
    void* out_arena = nullptr;
    size_t out_blocks = 0;
    std::vector<aesgpu::Slot> slots;
    bool staging_mapped = false;  // kernels may read the work items from the pinned staging
    bool use_done_word = false;   // completion seen through the slots' completion words
    aesgpu::Arena arena{0};
    aesgpu::Clock::time_point t0;

    std::mutex mu;                         // guards incoming, completed, counters below
    std::condition_variable cv;
    std::deque<aesgpu::Req*> incoming;
    std::vector<aesgpu::Req*> completed;
    std::vector<std::pair<uint64_t, uint64_t>> releases;  // (out_block, nblocks) released by the caller
    std::map<uint64_t, uint64_t> outstanding;  // manual release: finished outputs not yet released (start -> blocks)
    uint64_t next_id = 0;
    bool stop = false;

    // worker-only state
    std::deque<aesgpu::Req*> pending;
    uint64_t in_use = 0;
    std::atomic<uint64_t> batches{0};      // written by the worker, read by aes_server_stats
    std::atomic<uint64_t> direct_batches{0};
    std::atomic<uint64_t> launch_ns{0};    // worker time inside the launch calls of all batches
    std::atomic<uint64_t> max_in_use{0};
    std::atomic<int> last_error{AES_OK};
    std::atomic<bool> broken{false};       // the worker stopped on an internal failure
    std::atomic<uint64_t> arena_used_pub{0}, pending_pub{0};  // published by the worker for aes_server_stats
    std::atomic<uint64_t> submitted{0};                         // bumped by every submit and release
    std::thread worker;

    double now() const { return std::chrono::duration<double>(aesgpu::Clock::now() - t0).count(); }
};

namespace aesgpu {
namespace {

void finish(aes_server* s, Slot& sl, int status, double t)
{
    std::vector<Req*> done;
    done.swap(sl.reqs);
    for (Req* q : done) {
        q->done = t;
        q->status = status;
        s->in_use -= 2 * 16 * q->r.nblocks;
        if (s->cfg.auto_release || status != AES_SERVED_DONE)
            s->arena.release(q->out_block, q->r.nblocks);
    }
    sl.busy = false;
    std::lock_guard<std::mutex> g(s->mu);
    if (!s->cfg.auto_release && status == AES_SERVED_DONE)
        for (Req* q : done)
            s->outstanding.emplace(q->out_block, q->r.nblocks);
    s->completed.insert(s->completed.end(), done.begin(), done.end());
}

// Work items of a request of n blocks.
uint64_t items_of(uint64_t n, uint32_t chunk) { return n / chunk + (n % chunk != 0); }

// Work-item size for a request of n blocks : a request of at
// most chunk_blocks blocks is spread over items of small_item_blocks (when
// set), so that several waves share it instead of one wave walking it
// alone; larger requests use chunk_blocks, so that a large request keeps to
// a few CUs and leaves the others to the batches of other slots.
uint32_t chunk_for(const aes_serve_config& c, uint64_t n)
{
    return (c.small_item_blocks > 0 && n <= c.chunk_blocks) ? c.small_item_blocks : c.chunk_blocks;
}

uint64_t request_items(const aes_serve_config& c, uint64_t n) { return items_of(n, chunk_for(c, n)); }

bool valid(const aes_server* s, const aes_request& r)
{
    // the arena bounds come first and the budget is divided, so no product
    // wraps; a request must fit one batch, else it would hold the FIFO forever
    return r.nblocks > 0 && r.nblocks <= s->out_blocks && r.in_block <= s->in_blocks &&
           r.nblocks <= s->in_blocks - r.in_block && r.nblocks <= s->cfg.budget_bytes / 32 &&
           request_items(s->cfg, r.nblocks) <= s->cfg.max_batch_items && r.key_slot < s->n_slots;
}

bool launch(aes_server* s, Slot& sl, std::vector<Req*>& batch)
{
    size_t ne = 0, nd = 0;
    uint64_t enc_b = 0, tot_b = 0;
    for (Req* q : batch) {
        const uint64_t c = request_items(s->cfg, q->r.nblocks);
        (q->r.decrypt ? nd : ne) += c;
        tot_b += q->r.nblocks;
        if (!q->r.decrypt)
            enc_b += q->r.nblocks;
    }
    size_t ie = 0, id = ne;
    for (Req* q : batch) {
        const uint32_t chunk = chunk_for(s->cfg, q->r.nblocks);
        const uint64_t c = items_of(q->r.nblocks, chunk);
        for (uint64_t k = 0; k < c; ++k) {
            const uint64_t off = k * chunk;
            aes_work_item& it = sl.staging[q->r.decrypt ? id++ : ie++];
            it.in_block = q->r.in_block + off;
            it.out_block = q->out_block + off;
            it.nblocks = (uint32_t)std::min<uint64_t>(chunk, q->r.nblocks - off);
            it.key_slot = q->r.key_slot;
        }
    }
    sl.reqs = batch;
    sl.busy = true;
    s->batches.fetch_add(1, std::memory_order_relaxed);
    if (s->cfg.dry_run) {
        sl.dry_done = s->now() + s->cfg.dry_run_seconds;
        return true;
    }
    const size_t n = ne + nd;
    const auto t_launch = Clock::now();
    const bool direct = s->staging_mapped && n <= kDirectItems;
    if (direct)
        s->direct_batches.fetch_add(1, std::memory_order_relaxed);
    hipError_t e = direct ? hipSuccess
                          : hipMemcpyAsync(sl.items_dev, sl.staging, n * sizeof(aes_work_item),
                                           hipMemcpyHostToDevice, sl.stream);
    if (e == hipSuccess) {
        int grid = 0, enc_groups = 0;
        batch_grid(ne, nd, enc_b, tot_b, s->cfg.wg, s->max_grid, -1, &grid, &enc_groups);
        const void* items = direct ? static_cast<const void*>(sl.staging) : static_cast<const void*>(sl.items_dev);
        BatchArgs a{static_cast<const WorkItem*>(items), (uint32_t)ne, (uint32_t)nd, s->key_table,
                    (uint32_t)s->n_slots, s->in_pool, s->out_arena, (uint64_t)s->in_blocks, (uint64_t)s->out_blocks,
                    sl.counters_dev, (uint32_t)enc_groups};
        // with completion words the kernel's last workgroup writes the word
        e = s->use_done_word
                ? launch_batch_signal(a, s->cfg.bpt, s->cfg.placement, grid, s->cfg.wg, sl.done_word, sl.seq + 1,
                                      sl.stream)
                : launch_batch(a, s->cfg.bpt, s->cfg.placement, grid, s->cfg.wg, sl.stream);
    }
    if (e == hipSuccess) {
        sl.launched = s->now();
        if (s->use_done_word)
            ++sl.seq;
        else
            e = hipEventRecord(sl.event, sl.stream);
    }
    s->launch_ns.fetch_add(
        (uint64_t)std::chrono::duration_cast<std::chrono::nanoseconds>(Clock::now() - t_launch).count(),
        std::memory_order_relaxed);
    if (e != hipSuccess) {
        s->last_error.store(AES_EHIP);
        finish(s, sl, AES_SERVED_FAILED, s->now());
        return false;
    }
    return true;
}

void worker_loop(aes_server* s);

// The worker thread: an exception (a failed host allocation) stops it and
// marks the engine broken; submit and poll then report the failure.
void worker_main(aes_server* s)
{
    try {
        worker_loop(s);
    } catch (const std::bad_alloc&) {
        s->last_error.store(AES_ENOMEM);
        s->broken.store(true);
    } catch (...) {
        s->last_error.store(AES_EHIP);
        s->broken.store(true);
    }
}

void worker_loop(aes_server* s)
{
    if (!s->cfg.dry_run)
        hipSetDevice(s->device);
    uint64_t seen = 0;
    // The head of the queue could not be admitted while no slot was busy:
    // only a release by the caller (or a stop) can change that, so the
    // worker sleeps until one arrives instead of retrying.
    bool blocked = false;
    for (;;) {
        bool stopping;
        const bool idle = (s->pending.empty() || blocked) &&
                          std::none_of(s->slots.begin(), s->slots.end(), [](const Slot& x) { return x.busy; });
        if (idle && !blocked) {
            // spin briefly before sleeping: a request arriving within ~50 us
            // is picked up without a thread wake-up
            const auto until = Clock::now() + std::chrono::microseconds(50);
            while (s->submitted.load(std::memory_order_acquire) == seen && Clock::now() < until)
                std::this_thread::yield();
        }
        {
            std::unique_lock<std::mutex> g(s->mu);
            if (idle && s->incoming.empty() && s->releases.empty() && !s->stop)
                s->cv.wait_for(g, std::chrono::microseconds(blocked ? 2000 : 200));
            seen = s->submitted.load(std::memory_order_acquire);
            while (!s->incoming.empty()) {
                s->pending.push_back(s->incoming.front());
                s->incoming.pop_front();
            }
            for (auto& rl : s->releases)
                s->arena.release(rl.first, rl.second);
            s->releases.clear();
            stopping = s->stop;
        }
        // completions
        for (Slot& sl : s->slots) {
            if (!sl.busy)
                continue;
            if (s->cfg.dry_run) {
                if (s->now() >= sl.dry_done)
                    finish(s, sl, AES_SERVED_DONE, s->now());
            } else if (s->use_done_word &&
                       __atomic_load_n(sl.done_word, __ATOMIC_ACQUIRE) == sl.seq) {
                finish(s, sl, AES_SERVED_DONE, s->now());
            } else if (!s->use_done_word || s->now() - sl.launched > kStreamCheckSeconds) {
                // events, or a batch that has run long: ask the runtime, which
                // also reports a failed launch or kernel
                hipError_t q = s->use_done_word ? hipStreamQuery(sl.stream) : hipEventQuery(sl.event);
                if (q == hipSuccess)
                    finish(s, sl, AES_SERVED_DONE, s->now());
                else if (q != hipErrorNotReady) {
                    s->last_error.store(AES_EHIP);
                    finish(s, sl, AES_SERVED_FAILED, s->now());
                }
            }
        }
        // admission into a free slot
        for (Slot& sl : s->slots) {
            if (sl.busy || s->pending.empty())
                continue;
            // Requests join in arrival order until one does not fit.  With
            // size classes the queue's head sets the batch's class (at most
            // chunk_blocks blocks, or more) and requests of the other class
            // keep their place for the next slot, so a small request never
            // waits for a large one that shares its batch.
            std::vector<Req*> batch;
            std::deque<Req*> rest;
            uint64_t items = 0;
            bool have_class = false, small_class = false, untouched = true;
            for (auto it = s->pending.begin(); it != s->pending.end(); ++it) {
                Req* q = *it;
                if (!valid(s, q->r)) {  // can never run: report at once
                    untouched = false;
                    q->status = AES_SERVED_REJECTED;
                    q->done = s->now();
                    std::lock_guard<std::mutex> g(s->mu);
                    s->completed.push_back(q);
                    continue;
                }
                const bool small = q->r.nblocks <= s->cfg.chunk_blocks;
                if (s->cfg.size_classes && have_class && small != small_class) {
                    untouched = false;
                    rest.push_back(q);
                    continue;
                }
                have_class = true;
                small_class = small;
                const uint64_t need = request_items(s->cfg, q->r.nblocks);
                const uint64_t bytes = 2 * 16 * q->r.nblocks;  // valid(): at most the budget
                uint64_t start = 0;
                if (items + need > s->cfg.max_batch_items || bytes > s->cfg.budget_bytes - s->in_use ||
                    !s->arena.alloc(q->r.nblocks, &start)) {
                    if (!untouched)  // the batch is full: the rest keeps its order
                        rest.insert(rest.end(), it, s->pending.end());
                    break;
                }
                untouched = false;
                q->out_block = start;
                q->admitted = s->now();
                q->batch = (int)s->batches.load(std::memory_order_relaxed);
                s->in_use += bytes;
                items += need;
                batch.push_back(q);
            }
            if (!untouched)
                s->pending.swap(rest);
            if (batch.empty())
                break;
            if (s->in_use > s->max_in_use.load(std::memory_order_relaxed))
                s->max_in_use.store(s->in_use, std::memory_order_relaxed);
            launch(s, sl, batch);
        }
        const bool none_busy =
            std::none_of(s->slots.begin(), s->slots.end(), [](const Slot& x) { return x.busy; });
        blocked = !s->pending.empty() && none_busy;
        if (stopping && blocked) {
            // Nothing is running, so the budget is free and the head waits
            // for output space that the caller still holds (manual release);
            // the caller is inside aes_server_destroy and releases nothing
            // more, so the queued requests are finished as rejected.
            std::lock_guard<std::mutex> g(s->mu);
            for (Req* q : s->pending) {
                q->status = AES_SERVED_REJECTED;
                q->done = s->now();
                s->completed.push_back(q);
            }
            s->pending.clear();
            blocked = false;
        }
        s->arena_used_pub.store(s->arena.used(), std::memory_order_relaxed);
        s->pending_pub.store(s->pending.size(), std::memory_order_relaxed);
        if (stopping && s->pending.empty() &&
            std::none_of(s->slots.begin(), s->slots.end(), [](const Slot& x) { return x.busy; })) {
            std::lock_guard<std::mutex> g(s->mu);
            if (s->incoming.empty())
                break;
        }
    }
}

}  // namespace
}  // namespace aesgpu

using namespace aesgpu;

// Byte offset of the completion words in the staging (after the work items, 64-byte aligned).
static size_t staging_words_offset(const aes_serve_config* cfg)
{
    return ((size_t)cfg->nslots * cfg->max_batch_items * sizeof(aes_work_item) + 63) & ~(size_t)63;
}

extern "C" {

size_t aes_server_workspace_bytes(const aes_serve_config* cfg)
{
    if (cfg == nullptr || cfg->nslots <= 0)
        return 0;
    const size_t items = ((size_t)cfg->max_batch_items * sizeof(aes_work_item) + 255) & ~(size_t)255;
    return (size_t)cfg->nslots * (items + 256);
}

size_t aes_server_staging_bytes(const aes_serve_config* cfg)
{
    if (cfg == nullptr || cfg->nslots <= 0)
        return 0;
    // the slots' work items, then one 64-byte line per slot for its completion word
    return staging_words_offset(cfg) + (size_t)cfg->nslots * 64;
}

static int server_create_impl(const aes_serve_config* cfg, const uint32_t* key_table_dev, size_t n_slots,
                      const void* in_pool, size_t in_blocks, void* out_arena, size_t out_blocks,
                      void* workspace_dev, size_t workspace_bytes, void* staging_host, size_t staging_bytes,
                      aes_server** out)
{
    if (out == nullptr || cfg == nullptr)
        return fail(AES_EINVAL, "null config or output pointer");
    *out = nullptr;
    const aes_serve_config& c = *cfg;
    if (c.nslots < 1 || c.nslots > 16 || c.chunk_blocks == 0 || c.chunk_blocks > AES_MAX_ITEM_BLOCKS ||
        c.max_batch_items == 0 || c.budget_bytes == 0 || (c.bpt != 1 && c.bpt != 2 && c.bpt != 4) || c.wg < 64 ||
        c.wg > 1024 || c.wg % 64 || c.grid < 0 || c.small_item_blocks > c.chunk_blocks ||
        (c.completion != AES_SERVE_COMPLETION_AUTO && c.completion != AES_SERVE_COMPLETION_EVENTS) ||
        (c.placement != AES_PLACEMENT_TTABLE4 && c.placement != AES_PLACEMENT_TTABLE2 &&
         c.placement != AES_PLACEMENT_TTABLE1))
        return fail(AES_EINVAL, "serve config out of range (nslots 1..16, chunk 1..AES_MAX_ITEM_BLOCKS, "
                                "items/budget > 0, bpt 1/2/4, wg multiple of 64 in [64, 1024], grid >= 0, "
                                "placement 0/1/2, completion 0/1, small items at most chunk)");
    if (!c.dry_run && (key_table_dev == nullptr || in_pool == nullptr || out_arena == nullptr ||
                       workspace_dev == nullptr || staging_host == nullptr))
        return fail(AES_EINVAL, "null key table, input pool, output arena, workspace or staging");
    if (workspace_bytes < aes_server_workspace_bytes(cfg) || staging_bytes < aes_server_staging_bytes(cfg))
        return fail(AES_ERANGE, "workspace or staging smaller than aes_server_workspace_bytes/staging_bytes");
    if (n_slots == 0 || out_blocks == 0)
        return fail(AES_EINVAL, "empty key table or output arena");
    aes_server* s = new (std::nothrow) aes_server();
    if (!s)
        return fail(AES_ENOMEM, "out of host memory");
    s->cfg = c;
    s->key_table = key_table_dev;
    s->n_slots = n_slots;
    s->in_pool = in_pool;
    s->in_blocks = in_blocks;
    s->out_arena = out_arena;
    s->out_blocks = out_blocks;
    try {
        s->arena = Arena(out_blocks);
        s->slots.resize(c.nslots);
    } catch (...) {
        delete s;
        throw;
    }
    const size_t items_bytes = ((size_t)c.max_batch_items * sizeof(aes_work_item) + 255) & ~(size_t)255;
    int rc = AES_OK;
    if (!c.dry_run) {
        if (hipGetDevice(&s->device) != hipSuccess)
            rc = AES_EHIP;
        s->cus = device_cu_count();
        if (s->cus <= 0)
            rc = AES_EHIP;
        int per_cu = 0;
        if (rc == AES_OK && c.grid == 0 && batch_groups_per_cu(c.bpt, c.placement, c.wg, &per_cu) != hipSuccess)
            rc = AES_EHIP;
        s->max_grid = c.grid > 0 ? c.grid : s->cus * per_cu;
    }
    for (int i = 0; i < c.nslots && rc == AES_OK; ++i) {
        Slot& sl = s->slots[i];
        char* base = static_cast<char*>(workspace_dev) + (size_t)i * (items_bytes + 256);
        sl.items_dev = reinterpret_cast<aes_work_item*>(base);
        sl.counters_dev = reinterpret_cast<uint32_t*>(base + items_bytes);
        sl.staging = reinterpret_cast<aes_work_item*>(static_cast<char*>(staging_host) +
                                                      (size_t)i * c.max_batch_items * sizeof(aes_work_item));
        sl.done_word = reinterpret_cast<uint32_t*>(static_cast<char*>(staging_host) + staging_words_offset(cfg) +
                                                   (size_t)i * 64);
        __atomic_store_n(sl.done_word, 0u, __ATOMIC_RELEASE);
        if (c.dry_run)
            continue;
        if (hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking) != hipSuccess ||
            hipEventCreateWithFlags(&sl.event, hipEventDisableTiming) != hipSuccess ||
            hipMemsetAsync(sl.counters_dev, 0, 16, sl.stream) != hipSuccess)
            rc = AES_EHIP;
    }
    if (rc == AES_OK && !c.dry_run) {
        for (Slot& sl : s->slots)
            if (hipStreamSynchronize(sl.stream) != hipSuccess)
                rc = AES_EHIP;
    }
    if (rc != AES_OK) {
        for (Slot& sl : s->slots) {
            if (sl.event) hipEventDestroy(sl.event);
            if (sl.stream) hipStreamDestroy(sl.stream);
        }
        delete s;
        return rc;
    }
    if (!c.dry_run) {
        s->staging_mapped = host_range_device_mapped(staging_host, aes_server_staging_bytes(cfg));
        s->use_done_word = s->staging_mapped && c.completion == AES_SERVE_COMPLETION_AUTO;
    }
    s->t0 = Clock::now();
    try {
        s->worker = std::thread(worker_main, s);
    } catch (...) {
        for (Slot& sl : s->slots) {
            if (sl.event) hipEventDestroy(sl.event);
            if (sl.stream) hipStreamDestroy(sl.stream);
        }
        delete s;
        throw;
    }
    *out = s;
    return AES_OK;
}

static int server_submit_impl(aes_server* s, const aes_request* reqs, size_t n, uint64_t* first_id)
{
    if (s == nullptr || (n > 0 && reqs == nullptr))
        return AES_EINVAL;
    if (s->broken.load())
        return AES_EHIP;
    std::vector<Req*> made;
    made.reserve(n);
    const double t = s->now();
    for (size_t i = 0; i < n; ++i) {
        Req* q = new (std::nothrow) Req();
        if (!q) {
            for (Req* m : made)
                delete m;
            return AES_ENOMEM;
        }
        q->r = reqs[i];
        q->arrival = t;
        made.push_back(q);
    }
    {
        std::lock_guard<std::mutex> g(s->mu);
        if (s->stop) {
            for (Req* m : made)
                delete m;
            return AES_EBUSY;
        }
        if (first_id)
            *first_id = s->next_id;
        for (Req* q : made) {
            q->id = s->next_id++;
            s->incoming.push_back(q);
        }
        s->submitted.fetch_add(1, std::memory_order_release);
    }
    s->cv.notify_one();
    return AES_OK;
}

static int server_poll_impl(aes_server* s, aes_served* out, size_t cap, size_t* n)
{
    if (s == nullptr || n == nullptr || (cap > 0 && out == nullptr))
        return AES_EINVAL;
    std::vector<Req*> take;
    {
        std::lock_guard<std::mutex> g(s->mu);
        const size_t k = std::min(cap, s->completed.size());
        take.assign(s->completed.begin(), s->completed.begin() + k);
        s->completed.erase(s->completed.begin(), s->completed.begin() + k);
    }
    for (size_t i = 0; i < take.size(); ++i) {
        const Req* q = take[i];
        out[i].id = q->id;
        out[i].arrival_s = q->arrival;
        out[i].admitted_s = q->admitted;
        out[i].done_s = q->done;
        out[i].out_block = q->out_block;
        out[i].nblocks = q->r.nblocks;
        out[i].status = q->status;
        out[i].batch = q->batch;
        delete q;
    }
    *n = take.size();
    if (s->broken.load())
        return s->last_error.load() == AES_ENOMEM ? AES_ENOMEM : AES_EHIP;
    return s->last_error.exchange(AES_OK) == AES_OK ? AES_OK : AES_EHIP;
}

static int server_release_impl(aes_server* s, const aes_served* done, size_t n)
{
    if (s == nullptr || (n > 0 && done == nullptr))
        return AES_EINVAL;
    if (s->cfg.auto_release)
        return AES_OK;
    int rc = AES_OK;
    {
        // only ranges the engine handed out and that are still held go back to
        // the arena: a repeated or made-up release would corrupt its free list
        std::lock_guard<std::mutex> g(s->mu);
        for (size_t i = 0; i < n; ++i) {
            if (done[i].status != AES_SERVED_DONE)
                continue;
            auto it = s->outstanding.find(done[i].out_block);
            if (it == s->outstanding.end() || it->second != done[i].nblocks) {
                rc = fail(AES_EINVAL, "release of blocks [%llu, +%llu) that are not held",
                          (unsigned long long)done[i].out_block, (unsigned long long)done[i].nblocks);
                continue;
            }
            s->outstanding.erase(it);
            s->releases.emplace_back(done[i].out_block, done[i].nblocks);
        }
        s->submitted.fetch_add(1, std::memory_order_release);
    }
    s->cv.notify_one();
    return rc;
}

static int server_stats_impl(aes_server* s, aes_serve_stats* st)
{
    if (s == nullptr || st == nullptr)
        return AES_EINVAL;
    std::lock_guard<std::mutex> g(s->mu);
    st->batches = s->batches.load(std::memory_order_relaxed);
    st->max_device_bytes_in_use = s->max_in_use.load(std::memory_order_relaxed);
    st->arena_blocks_in_use = s->arena_used_pub.load(std::memory_order_relaxed);
    st->pending = s->pending_pub.load(std::memory_order_relaxed) + s->incoming.size();
    st->direct_batches = s->direct_batches.load(std::memory_order_relaxed);
    st->launch_ns = s->launch_ns.load(std::memory_order_relaxed);
    return AES_OK;
}

static int server_destroy_impl(aes_server* s)
{
    if (s == nullptr)
        return AES_OK;
    {
        std::lock_guard<std::mutex> g(s->mu);
        s->stop = true;
    }
    s->cv.notify_one();
    s->worker.join();
    for (Slot& sl : s->slots) {
        if (sl.stream)
            hipStreamSynchronize(sl.stream);
        if (sl.event)
            hipEventDestroy(sl.event);
        if (sl.stream)
            hipStreamDestroy(sl.stream);
    }
    for (Req* q : s->completed)
        delete q;
    for (Req* q : s->incoming)  // non-empty only if the worker stopped on a failure
        delete q;
    for (Req* q : s->pending)
        delete q;
    delete s;
    return AES_OK;
}

static int serve_replay_impl(aes_server* s, const aes_request* reqs, const double* arrival_s, size_t n, aes_served* results)
{
    if (s == nullptr || (n > 0 && (reqs == nullptr || arrival_s == nullptr || results == nullptr)))
        return AES_EINVAL;
    if (!s->cfg.auto_release)
        return AES_EINVAL;
    const double base = s->now();
    std::vector<aes_served> buf(4096);
    size_t got = 0, next = 0;
    uint64_t id0 = 0;
    bool have_id0 = false;
    int rc = AES_OK;
    while (got < n) {
        const double t = s->now() - base;
        size_t k = next;
        while (k < n && arrival_s[k] <= t)
            ++k;
        if (k > next) {
            uint64_t fid;
            int r = server_submit_impl(s, reqs + next, k - next, &fid);
            if (r != AES_OK)
                return r;
            if (!have_id0) {
                id0 = fid;
                have_id0 = true;
            }
            next = k;
        }
        size_t m = 0;
        int pr = server_poll_impl(s, buf.data(), buf.size(), &m);
        if (pr != AES_OK)
            rc = pr;
        if (s->broken.load())
            return rc;
        for (size_t i = 0; i < m; ++i) {
            const size_t idx = (size_t)(buf[i].id - id0);
            if (idx < n) {
                results[idx] = buf[i];
                // open loop: latency is measured from the scheduled arrival
                results[idx].arrival_s = base + arrival_s[idx];
                ++got;
            }
        }
        if (m == 0 && next < n) {
            const double wait = arrival_s[next] - (s->now() - base);
            if (wait > 200e-6)
                std::this_thread::sleep_for(std::chrono::duration<double>(wait - 100e-6));
        }
    }
    return rc;
}

int aes_server_create(const aes_serve_config* cfg, const uint32_t* key_table_dev, size_t n_slots,
                      const void* in_pool, size_t in_blocks, void* out_arena, size_t out_blocks,
                      void* workspace_dev, size_t workspace_bytes, void* staging_host, size_t staging_bytes,
                      aes_server** out)
{
    return guarded([&] {
        return server_create_impl(cfg, key_table_dev, n_slots, in_pool, in_blocks, out_arena, out_blocks,
                                  workspace_dev, workspace_bytes, staging_host, staging_bytes, out);
    });
}

int aes_server_submit(aes_server* s, const aes_request* reqs, size_t n, uint64_t* first_id)
{
    return guarded([&] { return server_submit_impl(s, reqs, n, first_id); });
}

int aes_server_poll(aes_server* s, aes_served* out, size_t cap, size_t* n)
{
    return guarded([&] { return server_poll_impl(s, out, cap, n); });
}

int aes_server_release(aes_server* s, const aes_served* done, size_t n)
{
    return guarded([&] { return server_release_impl(s, done, n); });
}

int aes_server_stats(aes_server* s, aes_serve_stats* st)
{
    return guarded([&] { return server_stats_impl(s, st); });
}

int aes_server_destroy(aes_server* s)
{
    return guarded([&] { return server_destroy_impl(s); });
}

int aes_serve_replay(aes_server* s, const aes_request* reqs, const double* arrival_s, size_t n, aes_served* results)
{
    return guarded([&] { return serve_replay_impl(s, reqs, arrival_s, n, results); });
}

}  // extern "C"
