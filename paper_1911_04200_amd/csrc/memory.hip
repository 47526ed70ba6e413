// Device memory cache of libjas.
//
// Every device buffer the library uses comes from here.  A freed block is
// kept, tagged with the stream that last used it and an event recorded on that
// stream; a later request reuses it on the same stream directly, or on another
// stream after making that stream wait for the event.  Steady-state calls thus
// never reach hipMalloc/hipFree, whose cost for multi-GB buffers is large and
// erratic.  jas_trim() hands the cached blocks back to the device.
#include <map>
#include <mutex>

#include "jas_internal.hpp"

namespace jas {
namespace {

struct Block {
    void *p;
    size_t bytes;
    hipStream_t s;
    hipEvent_t ev;  // null: no pending work
    int device;
};

std::mutex g_mu;
std::multimap<size_t, Block> g_free;  // by size
std::map<void *, Block> g_live;       // outstanding blocks by address
uint64_t g_cached = 0, g_in_use = 0;

size_t round_size(size_t bytes) {
    if (bytes < (1u << 20)) return (bytes + 511) & ~size_t(511);
    return (bytes + (2u << 20) - 1) & ~size_t((2u << 20) - 1);
}

void release_all_locked() {
    (void)hipDeviceSynchronize();
    for (auto &kv : g_free) {
        if (kv.second.ev) (void)hipEventDestroy(kv.second.ev);
        (void)hipFree(kv.second.p);
    }
    g_free.clear();
    g_cached = 0;
    (void)hipGetLastError();
}

}  // namespace

void *cache_alloc(size_t bytes, hipStream_t s, const char *what) {
    const size_t need = round_size(bytes ? bytes : 1);
    int dev = 0;
    JAS_HIP(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lk(g_mu);
    const size_t cap = need < (64u << 20) ? 2 * need : need + need / 4;
    for (auto it = g_free.lower_bound(need); it != g_free.end() && it->first <= cap; ++it) {
        Block b = it->second;
        if (b.device != dev) continue;
        g_free.erase(it);
        if (b.ev) {
            if (b.s != s) JAS_HIP(hipStreamWaitEvent(s, b.ev, 0));
            (void)hipEventDestroy(b.ev);
            b.ev = nullptr;
        }
        b.s = s;
        g_cached -= b.bytes;
        g_in_use += b.bytes;
        g_live[b.p] = b;
        return b.p;
    }
    void *p = nullptr;
    hipError_t e;
    {
        JAS_HOST_TIMED("malloc");
        e = hipMalloc(&p, need);
    }
    if (e != hipSuccess) {
        (void)hipGetLastError();
        release_all_locked();
        e = hipMalloc(&p, need);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            fail(JAS_ENOMEM, std::string("device allocation of ") + std::to_string(need) + " bytes for " + what +
                                 " failed: " + hipGetErrorString(e));
        }
    }
    g_in_use += need;
    g_live[p] = Block{p, need, s, nullptr, dev};
    return p;
}

void cache_free(void *p, bool synced) {
    if (!p) return;
    std::lock_guard<std::mutex> lk(g_mu);
    auto it = g_live.find(p);
    if (it == g_live.end()) return;
    Block b = it->second;
    g_live.erase(it);
    b.ev = nullptr;
    if (!synced) {
        if (hipEventCreateWithFlags(&b.ev, hipEventDisableTiming) != hipSuccess ||
            hipEventRecord(b.ev, b.s) != hipSuccess) {
            // cannot tag the block: wait for its stream instead
            (void)hipGetLastError();
            if (b.ev) (void)hipEventDestroy(b.ev);
            b.ev = nullptr;
            (void)hipStreamSynchronize(b.s);
        }
    }
    g_in_use -= b.bytes;
    g_cached += b.bytes;
    g_free.emplace(b.bytes, b);
}

hipStream_t side_stream() {
    static std::mutex mu;
    static std::map<int, hipStream_t> streams;  // one per device, kept for the process
    int dev = 0;
    JAS_HIP(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lk(mu);
    auto it = streams.find(dev);
    if (it != streams.end()) return it->second;
    hipStream_t st = nullptr;
    JAS_HIP(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));  // default priority
    streams[dev] = st;
    return st;
}

void stream_after(hipStream_t waiter, hipStream_t on) {
    hipEvent_t ev = nullptr;
    JAS_HIP(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
    const hipError_t e1 = hipEventRecord(ev, on);
    const hipError_t e2 = e1 == hipSuccess ? hipStreamWaitEvent(waiter, ev, 0) : e1;
    (void)hipEventDestroy(ev);
    if (e2 != hipSuccess) {
        // cannot order the streams by an event: wait for the work itself
        (void)hipGetLastError();
        JAS_HIP(hipStreamSynchronize(on));
    }
}

StreamJoin::~StreamJoin() {
    if (!waiter) return;
    try {
        stream_after(waiter, on);
    } catch (...) {
        (void)hipStreamSynchronize(on);
    }
}

void cache_trim() {
    std::lock_guard<std::mutex> lk(g_mu);
    release_all_locked();
}

uint64_t cache_bytes() {
    std::lock_guard<std::mutex> lk(g_mu);
    return g_cached;
}

}  // namespace jas

extern "C" void jas_trim(void) { jas::cache_trim(); }
