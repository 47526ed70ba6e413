// Fixed device workspace of jas_query_noalloc: the query for callers that
// cannot allocate device memory (code under HIP graph capture, tight serving
// loops, harnesses that forbid hipMalloc).
//
// Every temporary of such a query (sort keys, look-back status, digit
// totals, per-query counters) is carved from `scratch`, a file-scope device
// array of kNoAllocScratchBytes that each device running it holds until the
// process ends.  In host code `scratch` names a host-side stand-in, not
// device memory, so the host never passes it to a kernel: the first call on
// a device looks up that device's copy with hipGetSymbolAddress (with the
// device current) and keeps the address; kernels get that address.  Calls in
// one process share the array, so they are serialised by a lock held until
// their work on the stream has finished (with JAS_NO_WAIT a call that finds
// the lock taken returns JAS_EBUSY instead of waiting).
#include <map>
#include <mutex>

#include "jas_internal.hpp"

namespace jas {
namespace {

// Query keys and their second sort buffer take 16 bytes per ID; the
// look-back status (1 KiB per 8192 IDs), digit totals (512 KiB), the
// fallback sort's counts and the per-query arrays fit in the rest.
constexpr uint64_t kNoAllocMaxIds = uint64_t(1) << 23;
constexpr int32_t kNoAllocMaxQueries = 1 << 16;
constexpr size_t kNoAllocScratchBytes = size_t(136) << 20;

static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

std::mutex g_mu;             // serialises the users of every device's copy
std::map<int, char *> g_ptr;  // device -> address of its copy of scratch

}  // namespace

uint64_t noalloc_max_ids() { return kNoAllocMaxIds; }
int32_t noalloc_max_queries() { return kNoAllocMaxQueries; }

Arena noalloc_arena(std::unique_lock<std::mutex> &lk, bool wait) {
    if (wait) {
        lk = std::unique_lock<std::mutex>(g_mu);
    } else {
        lk = std::unique_lock<std::mutex>(g_mu, std::try_to_lock);
        if (!lk.owns_lock()) fail(JAS_EBUSY, "jas_query_noalloc: the fixed workspace is in use (JAS_NO_WAIT)");
    }
    int dev = 0;
    JAS_HIP(hipGetDevice(&dev));
    auto it = g_ptr.find(dev);
    if (it == g_ptr.end()) {
        void *p = nullptr;
        JAS_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) fail(JAS_EDEVICE, "hipGetSymbolAddress returned no address for the fixed workspace");
        it = g_ptr.emplace(dev, static_cast<char *>(p)).first;
    }
    Arena ar;
    ar.base = it->second;
    ar.cap = kNoAllocScratchBytes;
    return ar;
}

}  // namespace jas
