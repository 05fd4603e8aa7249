// Serving engine: continuous batching of offload-region requests.
//
// A request is one operation of a data region (the paper's data directive,
// section 1.3: arrays copied in at region entry stay on the device for every
// kernel of the region and are copied out at its exit).  The engine keeps a
// FIFO of submitted requests and a fixed number of slots (HIP streams).  On
// every progress step it:
//  - retires requests whose completion event has fired (frees the slot; a
//    region's last request also frees its device arrays and returns their
//    bytes to the budget);
//  - admits queued requests while a slot is free.  A region's first request
//    needs its footprint (arrays + workspace) within the HBM budget; first
//    requests are admitted in arrival order, but requests of regions already
//    open need no memory and pass a first request that waits for budget.
// Requests of different regions run concurrently on different streams; the
// requests of one region keep their order through an event wait on the
// region's previous request.  Region memory comes from the server's own
// block cache: a region's blocks go back to the cache only once the
// completion event of its last request has fired, so a new region can never
// be handed memory that a closing region's queued work still touches, and
// steady-state admission makes no allocation call.  Timestamps are host
// seconds since the server was created.
#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <chrono>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <new>
#include <set>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "../../include/accx.h"
#include "runtime_internal.h"

namespace {

using accx::rt::fail;
using accx::rt::fail_hip;

size_t al256(size_t x) { return (x + 255) & ~(size_t)255; }

struct Region {
    int op = 0, dtype = 0;
    int64_t n = 0;
    uint32_t flags = 0;
    void *mem = nullptr;  // A|B|C or x|result, then workspace
    size_t bytes = 0;     // footprint charged to the budget
    char *a = nullptr, *b = nullptr, *c = nullptr, *work = nullptr;
    size_t work_bytes = 0;
    void *host_c = nullptr;  // matmul: copied out at the last request
    hipEvent_t last = nullptr;  // completion event of the newest admitted request
    int inflight = 0;
    bool closing = false;       // its last request has been admitted (or failed)
    bool close_on_idle = false; // failed last request: close once nothing is in flight
    acc_status err = ACC_OK;
};

// Device block cache: a cached block serves a request when it is at most
// twice the request's size; otherwise a block is allocated (hipMalloc, or the
// caller's allocator when one is set).
// `held` counts every byte the cache holds, in use or free.  Under a budget
// the server charges each region the size of the block it was given and
// frees cached blocks before an allocation would take `held` past the
// budget, so the device memory the engine holds never exceeds it.
struct BlockCache {
    std::multimap<size_t, void *> free;  // block size -> block
    std::unordered_map<void *, size_t> size;
    uint64_t held = 0;

    static size_t round(size_t b)
    {
        const size_t mb = (size_t)1 << 20;
        return b <= mb ? (b + 4095) & ~(size_t)4095 : (b + mb - 1) & ~(mb - 1);
    }
    // The size of the block take(bytes) would hand out, and whether it is a
    // cached one (else a new allocation of that size).
    size_t fit(size_t bytes, bool *cached) const
    {
        const size_t want = round(bytes);
        auto it = free.lower_bound(want);
        *cached = it != free.end() && it->first <= 2 * want;
        return *cached ? it->first : want;
    }
    // Free cached blocks, largest first, until held <= limit (or none is left).
    void trim(uint64_t limit)
    {
        while (held > limit && !free.empty()) {
            auto it = std::prev(free.end());
            accx::rt::device_free(it->second);
            held -= it->first;
            size.erase(it->second);
            free.erase(it);
        }
    }
    // allow_cached = false: a new block of round(bytes) bytes
    void *take(size_t bytes, bool allow_cached = true)
    {
        const size_t want = round(bytes);
        auto it = free.lower_bound(want);
        if (allow_cached && it != free.end() && it->first <= 2 * want) {
            void *p = it->second;
            free.erase(it);
            return p;
        }
        void *p = nullptr;
        if (accx::rt::device_alloc(&p, want) != ACC_OK) {
            trim(0);  // drop every cached block and retry once
            if (accx::rt::device_alloc(&p, want) != ACC_OK) return nullptr;
        }
        size[p] = want;
        held += want;
        return p;
    }
    size_t block_size(void *p) const
    {
        auto it = size.find(p);
        return it == size.end() ? 0 : it->second;
    }
    void give(void *p)
    {
        if (p) free.emplace(size[p], p);
    }
    void release_all()
    {
        for (auto &kv : size) accx::rt::device_free(kv.first);
        free.clear();
        size.clear();
        held = 0;
    }
};

struct Queued {
    accx_request r;
    double t_submit;
};

struct Flight {
    int slot;
    hipEvent_t done;
    accx_request r;
    double t_submit, t_start;
    acc_status status;
};

}  // namespace

struct accx_server_s {
    std::mutex mu;
    std::chrono::steady_clock::time_point t0;
    std::vector<hipStream_t> streams;
    std::vector<bool> busy;
    uint64_t *staging = nullptr;  // pinned: one 8-byte reduction result per slot
    std::deque<Queued> queue;
    std::vector<Flight> flights;
    std::deque<accx_completion> done;
    std::unordered_map<int64_t, Region> regions;
    std::vector<hipEvent_t> events;  // free pool
    BlockCache blocks;
    uint64_t budget = 0, used = 0;
    accx_server_stats_t st{};

    double now() const
    {
        return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    }
};

namespace {

std::set<accx_server_s *> &servers()
{
    static auto *s = new std::set<accx_server_s *>();
    return *s;
}

size_t footprint(const accx_request &r, size_t *work)
{
    if (r.op == ACC_SERVE_MATMUL) {
        *work = accx::rt::matmul_workspace(r.dtype, r.n, r.flags);
        return 3 * al256((size_t)r.n * (size_t)r.n * 4) + al256(*work);
    }
    *work = accx::rt::reduce_workspace(r.n, r.flags);
    return al256((size_t)r.n * 4) + 256 + al256(*work);
}

acc_status validate(const accx_request &r)
{
    if (r.op != ACC_SERVE_MATMUL && r.op != ACC_SERVE_REDUCE) return fail(ACC_ERR_INVALID_ARG, "unknown op");
    if (r.dtype != ACC_FLOAT32 && r.dtype != ACC_INT32) return fail(ACC_ERR_INVALID_ARG, "unknown dtype");
    if (r.op == ACC_SERVE_MATMUL) {
        if (r.flags & ACC_ASYNC) return fail(ACC_ERR_INVALID_ARG, "ACC_ASYNC does not apply");
        acc_status s = accx::rt::check_matmul(r.dtype, r.n, r.flags);
        if (s != ACC_OK) return s;
        if (r.first && (!r.a || !r.b)) return fail(ACC_ERR_INVALID_ARG, "first request needs host a and b");
        if (r.last && !r.c) return fail(ACC_ERR_INVALID_ARG, "last request needs host c");
    } else {
        if (r.flags & ACC_ASYNC) return fail(ACC_ERR_INVALID_ARG, "ACC_ASYNC does not apply");
        acc_status s = accx::rt::check_reduce(r.dtype, r.n, r.flags);
        if (s != ACC_OK) return s;
        if (r.first && r.n > 0 && !r.a) return fail(ACC_ERR_INVALID_ARG, "first request needs host x");
        if (!r.c) return fail(ACC_ERR_INVALID_ARG, "reduction request needs a host result pointer");
    }
    return ACC_OK;
}

hipEvent_t take_event(accx_server_s *sv)
{
    if (!sv->events.empty()) {
        hipEvent_t e = sv->events.back();
        sv->events.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) return nullptr;
    return e;
}

void complete(accx_server_s *sv, const accx_request &r, acc_status status, double t_submit, double t_start)
{
    accx_completion c{};
    c.tag = r.tag;
    c.status = status;
    c.t_submit = t_submit;
    c.t_start = t_start;
    c.t_done = sv->now();
    sv->done.push_back(c);
    if (status == ACC_OK)
        sv->st.completed++;
    else
        sv->st.rejected++;
}

// Open the region of first request r on stream s: allocate and copy in.
acc_status open_region(accx_server_s *sv, const accx_request &r, size_t bytes, size_t work, bool use_cached,
                       hipStream_t s, Region &g)
{
    g.op = r.op;
    g.dtype = r.dtype;
    g.n = r.n;
    g.flags = r.flags;
    g.work_bytes = work;
    g.mem = sv->blocks.take(bytes, use_cached);
    if (!g.mem) return fail(ACC_ERR_OUT_OF_MEMORY, "device allocation failed");
    g.bytes = sv->blocks.block_size(g.mem);  // the block's size is what the region holds
    hipError_t e = hipSuccess;
    char *p = static_cast<char *>(g.mem);
    if (r.op == ACC_SERVE_MATMUL) {
        const size_t m = al256((size_t)r.n * (size_t)r.n * 4);
        g.a = p;
        g.b = p + m;
        g.c = p + 2 * m;
        g.work = p + 3 * m;
        e = hipMemcpyAsync(g.a, r.a, (size_t)r.n * r.n * 4, hipMemcpyHostToDevice, s);
        if (e == hipSuccess) e = hipMemcpyAsync(g.b, r.b, (size_t)r.n * r.n * 4, hipMemcpyHostToDevice, s);
    } else {
        const size_t m = al256((size_t)r.n * 4);
        g.a = p;
        g.c = p + m;  // device result
        g.work = p + m + 256;
        // the reduction's workspace needs no clearing: every call
        // overwrites the partial sums it reads
        if (r.n > 0) e = hipMemcpyAsync(g.a, r.a, (size_t)r.n * 4, hipMemcpyHostToDevice, s);
    }
    if (e != hipSuccess) return fail_hip(e, "region copy-in");
    sv->used += g.bytes;
    sv->st.budget_used = sv->used;
    sv->st.budget_peak = std::max<uint64_t>(sv->st.budget_peak, sv->used);
    sv->st.blocks_held = sv->blocks.held;
    sv->st.blocks_held_peak = std::max<uint64_t>(sv->st.blocks_held_peak, sv->blocks.held);
    return ACC_OK;
}

// Enqueue request r of region g on slot `slot`.
acc_status enqueue(accx_server_s *sv, const accx_request &r, Region &g, int slot, hipEvent_t done)
{
    hipStream_t s = sv->streams[(size_t)slot];
    hipError_t e = hipSuccess;
    if (g.last) e = hipStreamWaitEvent(s, g.last, 0);
    if (e != hipSuccess) return fail_hip(e, "hipStreamWaitEvent");
    acc_status st;
    {
        std::lock_guard<std::recursive_mutex> lk(accx::rt::lock());
        if (r.op == ACC_SERVE_MATMUL) {
            st = accx::rt::matmul(r.dtype, g.a, g.b, g.c, r.n, r.flags, g.work, g.work_bytes, s);
        } else {
            uint32_t init_bits;
            if (r.dtype == ACC_FLOAT32) {
                const float f = (float)r.init;
                std::memcpy(&init_bits, &f, 4);
            } else {
                const int32_t v = (int32_t)r.init;
                std::memcpy(&init_bits, &v, 4);
            }
            st = accx::rt::reduce(r.dtype, g.a, r.n, &init_bits, g.c, r.flags, g.work, s);
        }
    }
    if (st != ACC_OK) return st;
    if (r.op == ACC_SERVE_REDUCE)
        e = hipMemcpyAsync(sv->staging + slot, g.c, 4, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess && r.last && r.op == ACC_SERVE_MATMUL)
        e = hipMemcpyAsync(r.c, g.c, (size_t)r.n * r.n * 4, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipEventRecord(done, s);
    if (e != hipSuccess) return fail_hip(e, "request enqueue");
    return ACC_OK;
}

int free_slot(accx_server_s *sv)
{
    for (size_t k = 0; k < sv->busy.size(); ++k)
        if (!sv->busy[k]) return (int)k;
    return -1;
}

void retire(accx_server_s *sv)
{
    for (size_t k = 0; k < sv->flights.size();) {
        Flight &f = sv->flights[k];
        const hipError_t q = hipEventQuery(f.done);
        if (q == hipErrorNotReady) {
            ++k;
            continue;
        }
        acc_status status = f.status;
        if (q != hipSuccess && status == ACC_OK) status = fail_hip(q, "request");
        // The result first, whatever became of the region: the flights are
        // scanned in no particular order, so the region's last request may
        // have retired (and closed it) earlier in this same pass.
        if (status == ACC_OK && f.r.op == ACC_SERVE_REDUCE) std::memcpy(f.r.c, sv->staging + f.slot, 4);
        auto it = sv->regions.find(f.r.region);
        if (it != sv->regions.end()) {
            Region &g = it->second;
            if (g.last == f.done) g.last = nullptr;
            g.inflight--;
            if (f.r.last || (g.close_on_idle && g.inflight == 0)) {
                // the last request's event has fired: nothing queued touches
                // the region's memory any more
                sv->blocks.give(g.mem);
                sv->used -= std::min<uint64_t>(sv->used, g.bytes);
                sv->st.budget_used = sv->used;
                sv->regions.erase(it);
                sv->st.regions_open = (int64_t)sv->regions.size();
            }
        }
        sv->busy[(size_t)f.slot] = false;
        sv->events.push_back(f.done);
        complete(sv, f.r, status, f.t_submit, f.t_start);
        sv->flights[k] = sv->flights.back();
        sv->flights.pop_back();
    }
}

bool first_queued(accx_server_s *sv, int64_t key, const Queued *before)
{
    for (const Queued &q : sv->queue) {
        if (&q == before) return false;
        if (q.r.region == key && q.r.first) return true;
    }
    return false;
}

void admit(accx_server_s *sv)
{
    bool first_blocked = false;
    for (auto it = sv->queue.begin(); it != sv->queue.end();) {
        const int slot = free_slot(sv);
        if (slot < 0) break;
        const accx_request r = it->r;
        const double t_submit = it->t_submit;
        auto rit = sv->regions.find(r.region);
        if (r.first) {
            if (rit != sv->regions.end()) {
                fail(ACC_ERR_ALREADY_PRESENT, "region key already open");
                complete(sv, r, ACC_ERR_ALREADY_PRESENT, t_submit, sv->now());
                it = sv->queue.erase(it);
                continue;
            }
            if (first_blocked) {
                ++it;
                continue;
            }
            size_t work = 0;
            const size_t bytes = footprint(r, &work);
            if (sv->budget && BlockCache::round(bytes) > sv->budget) {
                complete(sv, r, ACC_ERR_OUT_OF_MEMORY, t_submit, sv->now());
                it = sv->queue.erase(it);
                continue;
            }
            // charged: the block it would get (a cached one, or a new one,
            // for which cached free blocks make room first)
            bool cached = false;
            size_t charge = sv->blocks.fit(bytes, &cached);
            if (sv->budget && sv->used + charge > sv->budget && cached) {
                cached = false;  // the cached block is too large to fit: allocate an exact one
                charge = BlockCache::round(bytes);
            }
            if (sv->budget && sv->used + charge > sv->budget) {
                first_blocked = true;  // first requests keep their order
                ++it;
                continue;
            }
            if (sv->budget && !cached) sv->blocks.trim(sv->budget - charge);
            Region g;
            acc_status s = open_region(sv, r, bytes, work, cached || !sv->budget, sv->streams[(size_t)slot], g);
            if (s != ACC_OK) {
                if (g.mem) {
                    // its copy-in may be queued: park the block behind the stream
                    (void)hipStreamSynchronize(sv->streams[(size_t)slot]);
                    sv->blocks.give(g.mem);  // never charged to the budget
                }
                complete(sv, r, s, t_submit, sv->now());
                it = sv->queue.erase(it);
                continue;
            }
            rit = sv->regions.emplace(r.region, g).first;
            sv->st.regions_open = (int64_t)sv->regions.size();
            sv->st.max_regions_open = std::max<int64_t>(sv->st.max_regions_open, sv->st.regions_open);
        } else if (rit == sv->regions.end()) {
            if (first_queued(sv, r.region, &*it)) {
                ++it;  // its region opens later
                continue;
            }
            fail(ACC_ERR_NOT_PRESENT, "region not open");
            complete(sv, r, ACC_ERR_NOT_PRESENT, t_submit, sv->now());
            it = sv->queue.erase(it);
            continue;
        }
        Region &g = rit->second;
        if (g.closing) {
            complete(sv, r, ACC_ERR_INVALID_ARG, t_submit, sv->now());
            it = sv->queue.erase(it);
            continue;
        }
        hipEvent_t done = take_event(sv);
        acc_status s = done ? (g.err != ACC_OK ? g.err : enqueue(sv, r, g, slot, done))
                            : fail(ACC_ERR_DEVICE, "event pool");
        if (s != ACC_OK) {
            if (g.err == ACC_OK) g.err = s;
            if (done) sv->events.push_back(done);
            if (r.last && g.inflight == 0) {
                // nothing of the region is in flight: its memory is idle once
                // the copy-in of its first request has drained
                (void)hipDeviceSynchronize();
                sv->blocks.give(g.mem);
                sv->used -= std::min<uint64_t>(sv->used, g.bytes);
                sv->regions.erase(rit);
                sv->st.regions_open = (int64_t)sv->regions.size();
            } else if (r.last) {
                g.closing = true;
                g.close_on_idle = true;  // retire() closes it after its last flight
            }
            complete(sv, r, s, t_submit, sv->now());
            it = sv->queue.erase(it);
            continue;
        }
        if (r.last) g.closing = true;
        g.last = done;
        g.inflight++;
        sv->busy[(size_t)slot] = true;
        sv->flights.push_back(Flight{slot, done, r, t_submit, sv->now(), ACC_OK});
        sv->st.admitted++;
        sv->st.max_inflight = std::max<int64_t>(sv->st.max_inflight, (int64_t)sv->flights.size());
        it = sv->queue.erase(it);
    }
}

void progress(accx_server_s *sv)
{
    retire(sv);
    admit(sv);
}

}  // namespace

extern "C" {

acc_status accx_server_create(int slots, uint64_t hbm_budget_bytes, accx_server *out)
{
    if (!out) return fail(ACC_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    acc_status s = accx::rt::ready();
    if (s != ACC_OK) return s;
    if (slots < 1 || slots > 64) return fail(ACC_ERR_INVALID_ARG, "slots must be in [1, 64]");
    accx_server_s *sv = new (std::nothrow) accx_server_s();
    if (!sv) return fail(ACC_ERR_OUT_OF_MEMORY, "host allocation failed");
    sv->t0 = std::chrono::steady_clock::now();
    sv->budget = hbm_budget_bytes;
    hipError_t e = hipHostMalloc(reinterpret_cast<void **>(&sv->staging), sizeof(uint64_t) * (size_t)slots);
    for (int k = 0; k < slots && e == hipSuccess; ++k) {
        hipStream_t st = nullptr;
        e = hipStreamCreateWithFlags(&st, hipStreamNonBlocking);
        if (e == hipSuccess) sv->streams.push_back(st);
    }
    if (e != hipSuccess) {
        for (hipStream_t st : sv->streams) (void)hipStreamDestroy(st);
        if (sv->staging) (void)hipHostFree(sv->staging);
        delete sv;
        return fail_hip(e, "server setup");
    }
    sv->busy.assign((size_t)slots, false);
    servers().insert(sv);
    *out = sv;
    return ACC_OK;
}

acc_status accx_server_submit(accx_server sv, const accx_request *r)
{
    if (!sv || !servers().count(sv) || !r) return fail(ACC_ERR_INVALID_ARG, "unknown server or NULL request");
    std::lock_guard<std::mutex> lk(sv->mu);
    acc_status s = validate(*r);
    if (s != ACC_OK) return s;
    sv->queue.push_back(Queued{*r, sv->now()});
    sv->st.submitted++;
    progress(sv);
    return ACC_OK;
}

acc_status accx_server_poll(accx_server sv, accx_completion *out, int cap, int *n_out)
{
    if (!sv || !servers().count(sv) || !n_out || cap < 0 || (cap > 0 && !out))
        return fail(ACC_ERR_INVALID_ARG, "unknown server or bad output buffer");
    std::lock_guard<std::mutex> lk(sv->mu);
    progress(sv);
    int n = 0;
    while (n < cap && !sv->done.empty()) {
        out[n++] = sv->done.front();
        sv->done.pop_front();
    }
    *n_out = n;
    return ACC_OK;
}

acc_status accx_server_drain(accx_server sv)
{
    if (!sv || !servers().count(sv)) return fail(ACC_ERR_INVALID_ARG, "unknown server");
    for (;;) {
        {
            std::lock_guard<std::mutex> lk(sv->mu);
            progress(sv);
            if (sv->queue.empty() && sv->flights.empty()) return ACC_OK;
            if (sv->flights.empty() && !sv->queue.empty()) {
                // nothing running and nothing admissible: the queue waits on
                // regions that never open
                for (const Queued &q : sv->queue) complete(sv, q.r, ACC_ERR_NOT_PRESENT, q.t_submit, sv->now());
                sv->queue.clear();
                return ACC_OK;
            }
        }
        std::this_thread::yield();
    }
}

acc_status accx_server_now(accx_server sv, double *t)
{
    if (!sv || !servers().count(sv) || !t) return fail(ACC_ERR_INVALID_ARG, "unknown server or NULL output");
    *t = sv->now();
    return ACC_OK;
}

acc_status accx_server_stats(accx_server sv, accx_server_stats_t *out)
{
    if (!sv || !servers().count(sv) || !out) return fail(ACC_ERR_INVALID_ARG, "unknown server or NULL output");
    std::lock_guard<std::mutex> lk(sv->mu);
    sv->st.blocks_held = sv->blocks.held;
    *out = sv->st;
    return ACC_OK;
}

acc_status accx_server_destroy(accx_server sv)
{
    if (!sv || !servers().count(sv)) return fail(ACC_ERR_INVALID_ARG, "unknown server");
    acc_status s = accx_server_drain(sv);
    {
        std::lock_guard<std::mutex> lk(sv->mu);
        for (hipStream_t st : sv->streams) (void)hipStreamSynchronize(st);
        sv->regions.clear();
        sv->blocks.release_all();
        for (hipEvent_t e : sv->events) (void)hipEventDestroy(e);
        for (hipStream_t st : sv->streams) (void)hipStreamDestroy(st);
        if (sv->staging) (void)hipHostFree(sv->staging);
    }
    servers().erase(sv);
    delete sv;
    return s;
}

}  // extern "C"
