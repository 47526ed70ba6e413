// Internal declarations of libjas (HIP, gfx950).  Not part of the ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <mutex>
#include <string>
#include <utility>
#include <vector>

#include "jas.h"

namespace jas {

// ---------------------------------------------------------------------------
// Errors: every failure inside the library throws jas::Error; the C entry
// points catch it and turn it into a status plus a thread-local message.
struct Error {
    jas_status status;
    std::string msg;
};

[[noreturn]] void fail(jas_status st, const std::string &msg);
// The thread's last error message (jas_last_error).
void set_last_error(const std::string &msg);
// Runs f, turning any failure into a status and the thread's message.
template <class F>
jas_status guarded(F &&f) {
    set_last_error("");
    try {
        f();
        return JAS_OK;
    } catch (const Error &e) {
        set_last_error(e.msg);
        return e.status;
    } catch (const std::bad_alloc &) {
        set_last_error("host allocation failed");
        return JAS_ENOMEM;
    } catch (const std::exception &e) {
        set_last_error(e.what());
        return JAS_EDEVICE;
    } catch (...) {
        set_last_error("unknown error");
        return JAS_EDEVICE;
    }
}
void check_hip(hipError_t e, const char *what);
#define JAS_HIP(call) ::jas::check_hip((call), #call)

// Kernel launch check (launch errors surface on the next runtime call).
void check_launch(const char *what);

// Scoped per-kernel timer: while timing is enabled (jas_timing_enable), records
// HIP events around the launch made in its scope.  Use via JAS_TIMED.
class KernelTimer {
   public:
    KernelTimer(const char *name, hipStream_t s);
    ~KernelTimer();

   private:
    const char *name_;
    hipStream_t s_;
    hipEvent_t a_ = nullptr, b_ = nullptr;
};
bool timing_on();
// Scoped host-side timer (wall clock), reported as "host:<name>" beside the kernels.
class HostTimer {
   public:
    explicit HostTimer(const char *name);
    ~HostTimer();

   private:
    const char *name_;
    double t0_ = -1.0;
};
#define JAS_HOST_TIMED(name) ::jas::HostTimer JAS_CAT(jas_htimer_, __LINE__)(name)
#define JAS_CAT2(a, b) a##b
#define JAS_CAT(a, b) JAS_CAT2(a, b)
#define JAS_TIMED(name, stream) ::jas::KernelTimer JAS_CAT(jas_timer_, __LINE__)(name, stream)

// ---------------------------------------------------------------------------
// Device memory.  Every buffer comes from the library's cache (memory.hip):
// blocks are reused across calls and streams (ordered by events), so steady
// state calls make no hipMalloc/hipFree.  Budget accounting is per call.
void *cache_alloc(size_t bytes, hipStream_t s, const char *what);
// synced: the caller has synchronised every stream that used the block.
void cache_free(void *p, bool synced);
void cache_trim();
uint64_t cache_bytes();

struct Budget {
    uint64_t limit = 0;  // 0 = none
    uint64_t held = 0;
    uint64_t peak = 0;
    Budget *other = nullptr;  // a second account that shares the limit
    void take(uint64_t bytes, const char *what);
    void give(uint64_t bytes) { held -= bytes; }
};

template <class T>
struct DevBuf {
    T *p = nullptr;
    size_t n = 0;
    Budget *budget = nullptr;
    bool owned_by_db = false;  // freed by jas_db_free after a device synchronisation
    bool external = false;     // memory owned elsewhere (an Arena): never freed here
    DevBuf() = default;
    DevBuf(const DevBuf &) = delete;
    DevBuf &operator=(const DevBuf &) = delete;
    DevBuf(DevBuf &&o) noexcept { *this = std::move(o); }
    DevBuf &operator=(DevBuf &&o) noexcept {
        if (this != &o) {
            release();
            p = o.p; n = o.n; budget = o.budget; owned_by_db = o.owned_by_db; external = o.external;
            o.p = nullptr; o.n = 0; o.external = false;
        }
        return *this;
    }
    // view of count elements at ptr (not owned)
    void wrap(T *ptr, size_t count) {
        release();
        p = ptr; n = count; budget = nullptr; owned_by_db = false; external = true;
    }
    ~DevBuf() { release(); }
    // db_owned = false: a temporary of the call (stream-ordered reuse);
    // db_owned = true: part of a jas_db.
    void alloc(size_t count, hipStream_t stream, Budget *b, bool temporary, const char *what) {
        release();
        const size_t bytes = (count ? count : 1) * sizeof(T);
        if (b) b->take(bytes, what);
        try {
            p = static_cast<T *>(cache_alloc(bytes, stream, what));
        } catch (...) {
            if (b) b->give(bytes);
            throw;
        }
        n = count;
        budget = b;
        owned_by_db = !temporary;
    }
    void release() {
        if (p && !external) {
            cache_free(p, owned_by_db);
            if (budget) budget->give((n ? n : 1) * sizeof(T));
        }
        p = nullptr; n = 0; external = false;
    }
    size_t bytes() const { return n * sizeof(T); }
};

// Exchange two buffers of one kind (the two halves of a ping-pong sort).
template <class T>
void swap_bufs(DevBuf<T> &a, DevBuf<T> &b) {
    std::swap(a.p, b.p);
    std::swap(a.n, b.n);
    std::swap(a.external, b.external);
}

// A fixed region of device memory handed out front to back (256-byte
// aligned pieces); used instead of the cache by calls that must not
// allocate.  Exceeding it fails with JAS_ENOMEM before the piece is used.
struct Arena {
    char *base = nullptr;
    size_t cap = 0, used = 0;
    template <class T>
    void take(DevBuf<T> &b, size_t count, const char *what) {
        const size_t bytes = (((count ? count : 1) * sizeof(T)) + 255) & ~size_t(255);
        if (used + bytes > cap)
            fail(JAS_ENOMEM, std::string("fixed workspace of ") + std::to_string(cap) + " bytes too small for " + what);
        b.wrap(reinterpret_cast<T *>(base + used), count);
        used += bytes;
    }
};

// A temporary of a call: from the arena when one is given, else from the cache.
template <class T>
void temp_buf(DevBuf<T> &b, size_t count, hipStream_t s, Budget *budget, Arena *ar, const char *what) {
    if (ar) ar->take(b, count, what);
    else b.alloc(count, s, budget, true, what);
}



// ---------------------------------------------------------------------------
// The encoded database (jas_db).
}  // namespace jas

namespace jas {
// What one eager encode decided and how large its intermediate arrays were:
// a plan (plan.hip) repeats the same decisions with buffers of these sizes
// plus headroom.
// The packed Gram's work units of an encoding: (stored word row, 128-column
// tile pair I <= J), and the word pairs they multiply.
inline void set_tile_stats(jas_encode_stats &o, uint64_t n) {
    const uint64_t t = (n + 127) / 128;
    o.dense_tiles = o.w_rows * (t * (t + 1) / 2);
    o.word_pairs_W = o.dense_tiles * 128 * 128;
}

// A stream of the library's own on the current device (default priority, one
// per device for the process), for work that overlaps the caller's stream
// inside one call.
hipStream_t side_stream();
// Makes `waiter` wait for the work enqueued on `on` so far.
void stream_after(hipStream_t waiter, hipStream_t on);
// While armed (waiter set), makes waiter wait for on when it goes out of
// scope: declared after the buffers the work on `on` uses, so that on an
// error the buffers' stream-ordered release comes after that work.
struct StreamJoin {
    hipStream_t waiter = nullptr, on = nullptr;
    StreamJoin() = default;
    StreamJoin(const StreamJoin &) = delete;
    StreamJoin &operator=(const StreamJoin &) = delete;
    ~StreamJoin();
};

struct EncodeTrace {
    bool onesweep = false;    // the global sort ran as single-pass scatters
    bool local = false;       // ranges finished in LDS (no global classification)
    bool wide = false;        // 64-bit keys in LDS
    bool pairs = false;       // row lists as sorted pair words
    uint64_t stride = 0;      // range stride used
    uint32_t lcap = 0;        // most keys per range of the LDS kernel used
    uint64_t N = 0, nlc = 0, ND = 0, NS = 0, R = 0, QD = 0, QL = 0, nb = 0, Hw = 0, H = 0, P = 0;
};
}  // namespace jas

struct jas_db {
    int device = 0;
    int32_t n = 0;
    uint32_t U = 0, sbits = 0, batch_bits = 0, dmin = 0, flags = 0;
    uint32_t word_bits = 64;  // b: rows per bitmask word (32 or 64)
    jas_encode_stats stats{};
    jas::Budget budget;  // db-owned memory
    // |X_i|
    jas::DevBuf<int64_t> card;
    // packed part: W[H][ldw] 64-bit elements; with b = 64 element row w is
    // word row w (up to 64 rows), with b = 32 it holds word rows 2w and 2w + 1
    // in its low and high halves
    uint64_t H = 0;
    jas::DevBuf<uint64_t> W;
    // row-list part: rows of degree 2..dmin-1, CSR over samples (ascending)
    uint64_t n_list = 0, list_nnz = 0;
    jas::DevBuf<uint64_t> list_ptr;   // n_list + 1
    jas::DevBuf<uint32_t> list_smp;   // list_nnz
    // the rows' pairs (a << 16) | b, a < b, sorted by a (built when
    // n <= kSampleMajorMaxN; else n_pairs = 0 and the Gram step walks the rows)
    uint64_t n_lpairs = 0;
    jas::DevBuf<uint32_t> pairs;
    // query index (JAS_KEEP_IDS): distinct keys (id << sbits | sample) in ascending
    // order and a table of their start by the top `ibits` bits of the ID.
    uint64_t n_keys = 0;
    uint32_t ibits = 0;
    jas::DevBuf<uint64_t> keys;
    jas::DevBuf<uint64_t> bucket;     // (1 << ibits) + 1 entries
    jas::EncodeTrace trace;
    // a plan's db: device sizes (PlanSize) of its last encode; W has H rows of
    // which the ones past the encoded count are zero, and the row-list pair
    // count is dsz[PZ_P] (n_lpairs is the capacity).  Null for jas_encode's dbs.
    const uint64_t *dsz = nullptr;
};

namespace jas {

// ---------------------------------------------------------------------------
// Device primitives (each in its own translation unit).

// out[i] = sum_{k<i} in[k] for i in [0, len]; out has len + 1 entries (out[len] = total).
// tmp: scratch from scan_tmp_elems(len).
size_t scan_tmp_elems(size_t len);
void scan_excl_u32(const uint32_t *in, uint64_t *out, size_t len, uint64_t *tmp, hipStream_t s);
void scan_excl_u64(const uint64_t *in, uint64_t *out, size_t len, uint64_t *tmp, hipStream_t s);

// LSD radix sort of 64-bit keys on bits [lo_bit, hi_bit), stable.  Result in
// *keys (buffers may be swapped with alt).  Each pass: histogram, scan, scatter.
struct RadixWork {
    DevBuf<uint32_t> counts;
    DevBuf<uint64_t> offs, tmp;
};
void radix_sort_u64(DevBuf<uint64_t> &keys, DevBuf<uint64_t> &alt, uint64_t N, uint32_t lo_bit, uint32_t hi_bit,
                    RadixWork &w, hipStream_t s, Budget *b, Arena *ar = nullptr);

// Single-pass-per-digit sort (decoupled look-back) of keys whose digit totals
// are known: ghist = kGhistReplicas copies of [kMaxPasses][256] totals; pass q
// sorts on bits [lo_bit + width*q, min(lo_bit + width*(q+1), hi_bit)),
// width <= 8.  Returns false (and does nothing) when a digit total reaches
// 2^30, where the caller uses radix_sort_u64.  A look-back that waits too long
// sets bit 1 of err[0] (the result is then invalid).
constexpr uint32_t kMaxPasses = 8;
constexpr uint32_t kGhistReplicas = 32;
// Where a sort's first pass takes its keys from when it forms them from CSR
// sets itself (key = id << sbits | sample): the IDs and offsets of the n >= 1
// sets, and a device buffer of 2 words per 8192-key tile (the samples holding
// the tile's first and last entries), which the sort fills first.  The eager
// sort allocates tinfo itself.
struct KeySource {
    const uint64_t *ids = nullptr, *off = nullptr;
    int32_t n = 0;
    uint32_t sbits = 0;
    uint32_t *tinfo = nullptr;
    uint64_t tinfo_words = 0;
};
uint64_t onesweep_tile_keys_u64();  // entries per tile of the 64-bit sort
// With src, keys.p is not read: the first pass forms the keys from src.
bool radix_sort_onesweep(DevBuf<uint64_t> &keys, DevBuf<uint64_t> &alt, uint64_t N, uint32_t lo_bit,
                         uint32_t hi_bit, uint32_t width, const unsigned long long *ghist, uint32_t *err,
                         hipStream_t s, Budget *b, Arena *ar = nullptr, const KeySource *src = nullptr);
bool radix_sort_onesweep_u32(DevBuf<uint32_t> &keys, DevBuf<uint32_t> &alt, uint64_t N, uint32_t lo_bit,
                             uint32_t hi_bit, uint32_t width, const unsigned long long *ghist, uint32_t *err,
                             hipStream_t s, Budget *b, Arena *ar = nullptr);
// Buffers of a planned single-pass sort (see plan.hip): digit starts
// [kMaxPasses][256], maxima [kMaxPasses], look-back status, ticket.
struct OnesweepBufs {
    uint64_t *gstart = nullptr, *maxima = nullptr;
    uint32_t *status = nullptr, *ticket = nullptr;
    uint64_t status_words = 0;
};
uint64_t onesweep_status_words(uint64_t N, bool u32);
// Planned sorts: the key count is *dN (at most Ncap); keys/alt are swapped
// as the passes go; no readback, no allocation.  err |= 4 when a digit total
// is too large, err |= 2 when a look-back gave up.
void radix_sort_onesweep_planned(uint64_t *&keys, uint64_t *&alt, const uint64_t *dN, uint64_t Ncap,
                                 uint32_t lo_bit, uint32_t hi_bit, uint32_t width, const unsigned long long *ghist,
                                 uint32_t *err, const OnesweepBufs &b, hipStream_t s,
                                 const KeySource *src = nullptr);
void radix_sort_onesweep_u32_planned(uint32_t *&keys, uint32_t *&alt, const uint64_t *dN, uint64_t Ncap,
                                     uint32_t lo_bit, uint32_t hi_bit, uint32_t width,
                                     const unsigned long long *ghist, uint32_t *err, const OnesweepBufs &b,
                                     hipStream_t s);
// Allocates w for N keys; returns the number of chunks (counts is [256][chunks]).
uint64_t radix_prepare(RadixWork &w, uint64_t N, hipStream_t s, Budget *b, Arena *ar = nullptr);
uint64_t radix_work_bytes(uint64_t N);

// How the ID bits are sorted.  Only the top `top_bits` of the U ID bits are
// sorted globally (npass passes of `width` bits); that makes every bucket of
// equal top bits contiguous, with about kBucketKeys keys per bucket for
// uniformly spread IDs, and the encoder finishes each run of whole buckets in
// LDS.  Buckets of about 2 kBucketKeys keys (one sorted bit fewer) are taken
// when a range's keys then still fit 32 bits in LDS: the ID bits below the
// buckets, a few bits for the buckets a range spans (kSpanBits) and the
// sample bits.
struct SortPlan {
    uint32_t top_bits = 0, npass = 0, width = 8;
};
constexpr uint64_t kBucketKeys = 512;
constexpr uint32_t kSpanBits = 4;
constexpr int32_t kSampleMajorMaxN = 10240;  // LDS row of per-sample counters (6 bytes each); < 2^16
constexpr uint32_t kLocalCapKeys = 6144;   // most keys one LDS range can hold
constexpr uint32_t kLocalShortCap = 4096;  // ranges no longer than this run four blocks per CU (else three)
// Range strides the encoder tries in turn until no range exceeds
// kLocalCapKeys; shorter ones leave room for larger buckets.
constexpr uint64_t kLocalStrides[2] = {3072, 2048};
constexpr uint64_t kLocalWideStride = 4096;  // tried first when the ranges need no LDS sort passes
SortPlan sort_plan(uint64_t N, uint32_t U, uint32_t sbits);

// Keys (id << sbits) | sample from CSR sets; err[0] |= 1 for an ID >= 2^U;
// ghist: totals of every digit of the plan's passes (kGhistReplicas copies).
// With keys == nullptr only the IDs are checked and the digits counted (the
// sort then forms the keys from the IDs in its first pass).
void build_keys(const uint64_t *ids, const uint64_t *offsets, int32_t n, uint64_t N, uint32_t sbits, uint32_t U,
                const SortPlan &plan, uint64_t *keys, uint32_t *err, unsigned long long *ghist, hipStream_t s);

// Encoding after the global sort (see encode.hip).  keys holds the N keys
// ordered by their top plan.top_bits ID bits; alt (N + 2 entries) is free and
// is used as scratch; offsets are the device CSR offsets.
void encode_sorted(jas_db *db, DevBuf<uint64_t> &keys, DevBuf<uint64_t> &alt, uint64_t N, const SortPlan &plan,
                   const uint64_t *offsets, hipStream_t s, Budget *tmpb);

// A planned encode (plan.hip creates it, encode.hip runs it): the decisions
// of one eager encode and buffers sized for them with headroom, so a like
// collection encodes with no host synchronisation and no allocation.
struct PlanState {
    int32_t n = 0;
    uint32_t U = 0, sbits = 0, batch_bits = 0, word_bits = 64, dmin = 2;
    SortPlan sort;
    uint64_t stride = 4096;
    uint32_t lcap = kLocalCapKeys;
    bool wide = false;
    // capacities
    uint64_t Ncap = 0, nlc_cap = 0, Rcap = 0, QDcap = 0, QLcap = 0, Hwcap = 0, Hcap = 0, Pcap = 0, tile_cap = 0,
             gcap = 0, ldw = 0;
    uint32_t pair_npass = 0, pair_width = 8, pair_bits = 0;
    // device buffers (owned by the plan)
    DevBuf<uint64_t> keys, alt, rs, offD, offS, offR, stmp, rid_g, rid, rptr, toff, Drow, Lrow, bpos, bq, nw, wbase,
        wq0, wq1, npo, np, dsz;
    DevBuf<uint32_t> err, cnt, rdeg, tcnt, bs, pk, palt;
    DevBuf<unsigned long long> ghist, gh, dupc, lprep, st;
    DevBuf<uint64_t> os_gstart, os_maxima, os2_gstart, os2_maxima;
    DevBuf<uint32_t> os_status, os_ticket, os2_status, os2_ticket, os_tinfo;
    DevBuf<int64_t> card;
    DevBuf<uint64_t> W;
    uint32_t *pairs_final = nullptr;  // the buffer holding the sorted pair words after the pair sort
};
void encode_planned(PlanState &p, const uint64_t *ids, const uint64_t *offsets, hipStream_t s);
enum { ST_PAIRS_ = 0, ST_ROWS_, ST_NNZW_, ST_F_, ST_LISTPAIRS_, ST_N_ };  // encode counters (encode.hip)
constexpr uint32_t kStatReplicasPub = 64;
constexpr uint64_t kSplitTilePub = 256 * 8;  // rows per row-split tile

// Degree threshold: rows of degree >= the result are bit-packed, 2..result-1
// kept as row lists; minimises the modelled Gram time (see tune.hip).
uint32_t choose_dense_min_degree(const std::vector<uint64_t> &deg_hist, uint32_t n, uint64_t nbatches,
                                 uint64_t max_packed_bytes);

// Gram and finalize (see gram.hip).
void gram(const jas_db *db, uint32_t flags, hipStream_t s, int32_t *B, int64_t *card, int64_t *den, double *J);
void finalize(uint32_t n, bool upper, hipStream_t s, int32_t *B, const int64_t *card, int64_t *den, double *J);
// Fails with JAS_EOVERFLOW when some card[i] >= card_limit() (one device
// flag, read back: synchronises s).
void check_card_limit(const int64_t *card, uint32_t n, hipStream_t s);
uint64_t kmer_starts(const uint64_t *seq_off, int64_t n_seq, uint32_t k, std::vector<uint64_t> &kbase);
void kmers(const uint64_t *seq, const uint64_t *seq_off, int64_t n_seq, uint32_t k, bool canonical, hipStream_t s,
           uint64_t *ids);
int32_t gram_variants();

// Exact relabelling (see relabel.hip): out[i] = rank of ids[i] among the
// distinct IDs (each < 2^U); returns their number D.  Synchronises s.
uint64_t relabel(const uint64_t *ids, uint64_t N, uint32_t U, hipStream_t s, uint64_t *out);

// Query (see query.hip).
// ar: take every temporary from this region instead of the cache (nothing is allocated).
void query(const jas_db *db, const uint64_t *q_ids, const uint64_t *q_offsets, int32_t nq, uint64_t NQ,
           hipStream_t s, int32_t *B, int64_t *q_card, int64_t *den, double *J, Arena *ar = nullptr);
uint64_t query_workspace_bytes(const jas_db *db, int32_t nq, uint64_t n_q_ids);

// The fixed workspace of jas_query_noalloc (noalloc.hip): the largest query
// it takes, and an arena over the current device's copy, returned with the
// lock that serialises its users held in lk.
uint64_t noalloc_max_ids();
int32_t noalloc_max_queries();
Arena noalloc_arena(std::unique_lock<std::mutex> &lk, bool wait);  // wait = false: JAS_EBUSY if taken

// Sizes of a planned encode, in device memory (plan.hip): kernels read them
// instead of host values, and every kernel returns at once when PZ_ABORT is
// set (a size exceeded its buffer's capacity; nothing is written past a
// buffer, the result is invalid and reported afterwards).
enum PlanSize { PZ_N = 0, PZ_R, PZ_QD, PZ_QL, PZ_NB, PZ_HW, PZ_H, PZ_P, PZ_ABORT, PZ_OVER, PZ_OVER_VALUE, PZ_COUNT };
__device__ __forceinline__ bool plan_aborted(const uint64_t *dsz) { return dsz && dsz[PZ_ABORT]; }

// Largest |X_i| (distinct IDs of one set) the int32 intersections allow:
// 2^31 - 1.  The environment variable JAS_TEST_CARD_LIMIT (a positive
// integer below 2^31, read on the host at every check) lowers the bound so
// tests can reach the overflow error with small inputs.
uint64_t card_limit();
// Largest digit total the eager single-pass sort takes (larger ones exceed
// its 30-bit look-back counts and the sort declines, for the reduce-then-scan
// passes).  JAS_TEST_SCATTER_LIMIT (a positive integer, read on the host at
// every sort) lowers it so tests reach the declined path with small inputs.
uint64_t scatter_count_limit();

inline uint32_t ceil_log2_u64(uint64_t v) {
    uint32_t b = 0;
    while (b < 64 && (uint64_t(1) << b) < v) ++b;
    return b;
}
inline uint64_t div_up(uint64_t a, uint64_t b) { return (a + b - 1) / b; }

}  // namespace jas
