// The C entry points of libjas (include/jas.h): argument checks on the host,
// error capture, host staging for JAS_HOST_PTRS, and the call sequence of
// each operation.  No exception crosses the ABI.
#include <cstdlib>
#include <cstring>
#include <memory>
#include <mutex>
#include <set>

#include "jas_internal.hpp"
#include "onesweep_index.hpp"

namespace jas {

namespace {
thread_local std::string g_err;

template <class F>
jas_status guard(F &&f) {
    g_err.clear();
    try {
        f();
        return JAS_OK;
    } catch (const Error &e) {
        g_err = e.msg;
        return e.status;
    } catch (const std::bad_alloc &) {
        g_err = "host allocation failed";
        return JAS_ENOMEM;
    } catch (const std::exception &e) {
        g_err = e.what();
        return JAS_EDEVICE;
    } catch (...) {
        g_err = "unknown error";
        return JAS_EDEVICE;
    }
}

__global__ void k_zero_u32(uint32_t *p) { *p = 0; }
__global__ void k_zero_u64(unsigned long long *p, uint64_t len) {
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < len; i += (uint64_t)gridDim.x * blockDim.x)
        p[i] = 0;
}

// Offsets to the host and validated: offsets[0] = 0, non-decreasing.
std::vector<uint64_t> host_offsets(const uint64_t *offsets, int32_t n, bool host, hipStream_t s, const char *what) {
    std::vector<uint64_t> h((size_t)n + 1);
    if (host) std::memcpy(h.data(), offsets, sizeof(uint64_t) * (n + 1));
    else {
        JAS_HIP(hipMemcpyAsync(h.data(), offsets, sizeof(uint64_t) * (n + 1), hipMemcpyDeviceToHost, s));
        JAS_HIP(hipStreamSynchronize(s));
    }
    if (h[0] != 0) fail(JAS_EINVAL, std::string(what) + ": offsets[0] must be 0");
    for (int32_t i = 0; i < n; ++i)
        if (h[i + 1] < h[i])
            fail(JAS_EINVAL, std::string(what) + ": offsets decrease at set " + std::to_string(i));
    return h;
}

}  // namespace

void fail(jas_status st, const std::string &msg) { throw Error{st, msg}; }

void set_last_error(const std::string &msg) { g_err = msg; }

void check_hip(hipError_t e, const char *what) {
    if (e != hipSuccess) {
        (void)hipGetLastError();
        fail(e == hipErrorOutOfMemory ? JAS_ENOMEM : JAS_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
    }
}

uint64_t card_limit() {
    constexpr uint64_t kLimit = uint64_t(1) << 31;
    const char *e = std::getenv("JAS_TEST_CARD_LIMIT");
    if (!e || !*e) return kLimit;
    char *end = nullptr;
    const unsigned long long v = std::strtoull(e, &end, 10);
    return (end && *end == 0 && v > 0 && v < kLimit) ? (uint64_t)v : kLimit;
}

uint64_t scatter_count_limit() {
    constexpr uint64_t kLimit = onesweep::kValMask;
    const char *e = std::getenv("JAS_TEST_SCATTER_LIMIT");
    if (!e || !*e) return kLimit;
    char *end = nullptr;
    const unsigned long long v = std::strtoull(e, &end, 10);
    return (end && *end == 0 && v > 0 && v < kLimit) ? (uint64_t)v : kLimit;
}

void check_launch(const char *what) {
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) fail(JAS_EDEVICE, std::string("launch of ") + what + ": " + hipGetErrorString(e));
}

void Budget::take(uint64_t bytes, const char *what) {
    const uint64_t all = held + (other ? other->held : 0);
    if (limit && all + bytes > limit)
        fail(JAS_ENOMEM, std::string("HBM budget of ") + std::to_string(limit) + " bytes exceeded by " + what +
                             " (" + std::to_string(bytes) + " bytes, " + std::to_string(all) + " held)");
    held += bytes;
    if (held > peak) peak = held;
}

}  // namespace jas

using namespace jas;

extern "C" {

const char *jas_last_error(void) { return g_err.c_str(); }

const char *jas_version(void) { return "jas 0.1 (gfx950)"; }

int32_t jas_db_size(const jas_db *db) { return db ? db->n : -1; }

int32_t jas_gram_variants(void) { return jas::gram_variants(); }

uint64_t jas_card_limit(void) { return jas::card_limit(); }

jas_status jas_db_stats(const jas_db *db, jas_encode_stats *stats) {
    return guard([&] {
        if (!db || !stats) fail(JAS_EINVAL, "jas_db_stats: null argument");
        *stats = db->stats;
    });
}

uint64_t jas_db_part_size(const jas_db *db, int32_t part) {
    if (!db) return 0;
    switch (part) {
        case JAS_DB_CARD: return (uint64_t)db->n;
        case JAS_DB_WORDS: return db->H * db->stats.w_stride;
        case JAS_DB_LIST_PAIRS: return db->n_lpairs;
        case JAS_DB_LIST_PTR: return db->n_lpairs || db->n_list == 0 ? 0 : db->n_list + 1;
        case JAS_DB_LIST_SAMPLES: return db->n_lpairs ? 0 : db->list_nnz;
        case JAS_DB_KEYS: return (db->flags & JAS_KEEP_IDS) ? db->n_keys : 0;
        default: return 0;
    }
}

jas_status jas_db_read(const jas_db *db, int32_t part, uint64_t first, uint64_t count, void *host_out) {
    return guard([&] {
        if (!db) fail(JAS_EINVAL, "jas_db_read: db is NULL");
        if (part < JAS_DB_CARD || part > JAS_DB_KEYS) fail(JAS_EINVAL, "jas_db_read: unknown part");
        const uint64_t size = jas_db_part_size(db, part);
        if (first > size || count > size - first) fail(JAS_EINVAL, "jas_db_read: range outside the part");
        if (count == 0) return;
        if (!host_out) fail(JAS_EINVAL, "jas_db_read: host_out is NULL");
        const void *src = nullptr;
        size_t elem = 8;
        switch (part) {
            case JAS_DB_CARD: src = db->card.p; break;
            case JAS_DB_WORDS: src = db->W.p; break;
            case JAS_DB_LIST_PAIRS: src = db->pairs.p; elem = 4; break;
            case JAS_DB_LIST_PTR: src = db->list_ptr.p; break;
            case JAS_DB_LIST_SAMPLES: src = db->list_smp.p; elem = 4; break;
            default: src = db->keys.p; break;
        }
        int cur = 0;
        JAS_HIP(hipGetDevice(&cur));
        if (cur != db->device) JAS_HIP(hipSetDevice(db->device));
        const hipError_t e = hipMemcpy(host_out, static_cast<const char *>(src) + first * elem, count * elem,
                                       hipMemcpyDeviceToHost);
        if (cur != db->device) (void)hipSetDevice(cur);
        check_hip(e, "jas_db_read: hipMemcpy");
    });
}

void jas_db_free(jas_db *db) {
    if (!db) return;
    int cur = 0;
    const int dev = db->device;
    (void)hipGetDevice(&cur);
    if (cur != dev) (void)hipSetDevice(dev);
    {
        JAS_HOST_TIMED("db_free_sync");
        (void)hipDeviceSynchronize();
    }
    {
        JAS_HOST_TIMED("db_free");
        delete db;
    }
    if (cur != dev) (void)hipSetDevice(cur);
}

jas_status jas_encode(const uint64_t *ids, const uint64_t *offsets, int32_t n, const jas_encode_opts *opts,
                      void *hip_stream, jas_db **db_out, jas_encode_stats *stats) {
    JAS_HOST_TIMED("jas_encode");
    return guard([&] {
        if (!db_out) fail(JAS_EINVAL, "jas_encode: db_out is NULL");
        *db_out = nullptr;
        if (!opts) fail(JAS_EINVAL, "jas_encode: opts is NULL");
        if (n < 0) fail(JAS_EINVAL, "jas_encode: n < 0");
        if (n > 0 && !offsets) fail(JAS_EINVAL, "jas_encode: offsets is NULL");
        const uint32_t U = opts->universe_bits;
        if (U < 1 || U > 63) fail(JAS_EINVAL, "jas_encode: universe_bits must be in 1..63");
        if (opts->word_bits != 0 && opts->word_bits != 32 && opts->word_bits != 64)
            fail(JAS_EINVAL, "jas_encode: word_bits must be 32, 64 or 0 (= 64)");
        const uint32_t sbits = ceil_log2_u64((uint64_t)std::max<int32_t>(n, 1));
        if (U + sbits > 64) fail(JAS_EINVAL, "jas_encode: universe_bits + ceil(log2 n) exceeds 64");
        if ((opts->flags & JAS_QUERY_ONLY) && !(opts->flags & JAS_KEEP_IDS))
            fail(JAS_EINVAL, "jas_encode: JAS_QUERY_ONLY needs JAS_KEEP_IDS");
        const bool host = opts->flags & JAS_HOST_PTRS;
        hipStream_t s = (hipStream_t)hip_stream;
        // host arrays are validated before the device is touched
        std::vector<uint64_t> hoff{0};
        if (host && n > 0) hoff = host_offsets(offsets, n, true, s, "jas_encode");
        if (host && hoff[n] > 0 && !ids) fail(JAS_EINVAL, "jas_encode: ids is NULL");
        int dev = 0;
        JAS_HIP(hipGetDevice(&dev));
        if (!host && n > 0) hoff = host_offsets(offsets, n, false, s, "jas_encode");
        const uint64_t N = hoff[n];
        if (N > 0 && !ids) fail(JAS_EINVAL, "jas_encode: ids is NULL");

        std::unique_ptr<jas_db> db(new jas_db());
        db->device = dev;
        db->n = n;
        db->U = U;
        db->sbits = sbits;
        db->batch_bits = (opts->batch_bits == 0 || opts->batch_bits >= U) ? U : opts->batch_bits;
        db->dmin = opts->dense_min_degree == 0 ? 0u : std::max<uint32_t>(2u, opts->dense_min_degree);
        db->flags = opts->flags;
        db->word_bits = opts->word_bits == 32 ? 32 : 64;
        // one budget for the call: temporaries (tb) and the db's own buffers
        Budget tb;
        tb.limit = opts->hbm_budget_bytes;
        tb.other = &db->budget;
        db->budget.limit = opts->hbm_budget_bytes;
        db->budget.other = &tb;

        // inputs on the device
        DevBuf<uint64_t> ids_d, off_d;
        const uint64_t *dids = ids, *doff = offsets;
        if (host) {
            off_d.alloc(n + 1, s, &tb, true, "offsets copy");
            JAS_HIP(hipMemcpyAsync(off_d.p, hoff.data(), sizeof(uint64_t) * (n + 1), hipMemcpyHostToDevice, s));
            doff = off_d.p;
            if (N > 0) {
                ids_d.alloc(N, s, &tb, true, "ids copy");
                JAS_HIP(hipMemcpyAsync(ids_d.p, ids, sizeof(uint64_t) * N, hipMemcpyHostToDevice, s));
                dids = ids_d.p;
            }
        }
        // Sort the keys on their top ID bits (the rest is finished per bucket
        // range in LDS by encode_sorted).  Both buffers get two spare entries:
        // after the sort the free one holds the shared pairs and row pointers.
        DevBuf<uint64_t> keys, alt;
        const SortPlan plan = sort_plan(N, U, sbits);
        if (N > 0) {
            DevBuf<uint32_t> err;
            keys.alloc(N + 2, s, &tb, true, "sort keys");
            alt.alloc(N + 2, s, &tb, true, "sort keys (second buffer)");
            err.alloc(1, s, &tb, true, "error flag");
            {
                JAS_TIMED("zero_u32", s);
                k_zero_u32<<<1, 1, 0, s>>>(err.p);
            }
            DevBuf<unsigned long long> ghist;
            ghist.alloc((uint64_t)kGhistReplicas * kMaxPasses * 256, s, &tb, true, "digit totals");
            {
                JAS_TIMED("zero_u32", s);
                k_zero_u64<<<64, 256, 0, s>>>(ghist.p, (uint64_t)kGhistReplicas * kMaxPasses * 256);
            }
            // with a global sort its first pass forms the keys from the IDs
            const bool from_ids = plan.top_bits > 0 && N > 1;
            build_keys(dids, doff, n, N, sbits, U, plan, from_ids ? nullptr : keys.p, err.p, ghist.p, s);
            uint32_t herr = 0;
            JAS_HIP(hipMemcpyAsync(&herr, err.p, 4, hipMemcpyDeviceToHost, s));
            JAS_HIP(hipStreamSynchronize(s));
            if (herr) fail(JAS_EINVAL, "jas_encode: an ID is >= 2^universe_bits");
            JAS_HOST_TIMED("sort_enqueue");
            const uint32_t lo = sbits + U - plan.top_bits, hi = sbits + U;
            KeySource src;
            src.ids = dids;
            src.off = doff;
            src.n = n;
            src.sbits = sbits;
            db->trace.onesweep = !from_ids || radix_sort_onesweep(keys, alt, N, lo, hi, plan.width, ghist.p, err.p,
                                                                  s, &tb, nullptr, &src);
            if (!db->trace.onesweep) {
                // the single-pass sort declined before any pass: form the keys, then sort them
                build_keys(dids, doff, n, N, sbits, U, plan, keys.p, err.p, ghist.p, s);
                RadixWork rw;
                radix_sort_u64(keys, alt, N, lo, hi, rw, s, &tb);
            }
            ids_d.release();
            JAS_HIP(hipMemcpyAsync(&herr, err.p, 4, hipMemcpyDeviceToHost, s));
            JAS_HIP(hipStreamSynchronize(s));
            if (herr) fail(JAS_EDEVICE, "jas_encode: the radix sort's look-back waited too long (result discarded)");
        }
        try {
            encode_sorted(db.get(), keys, alt, N, plan, doff, s, &tb);
        } catch (...) {
            // the db's buffers return to the cache as idle: let their kernels finish first
            (void)hipStreamSynchronize(s);
            throw;
        }
        alt.release();
        off_d.release();
        keys.release();
        db->budget.limit = 0;
        db->budget.other = nullptr;
        JAS_HIP(hipStreamSynchronize(s));
        db->stats.device_bytes = db->budget.held;
        if (stats) *stats = db->stats;
        *db_out = db.release();
    });
}

jas_status jas_gram(const jas_db *db, uint32_t flags, void *hip_stream, int32_t *B, int64_t *card, int64_t *den,
                    double *J) {
    return guard([&] {
        if (!db) fail(JAS_EINVAL, "jas_gram: db is NULL");
        if (db->flags & JAS_QUERY_ONLY) fail(JAS_EINVAL, "jas_gram: the db was encoded with JAS_QUERY_ONLY");
        if (!B && db->n > 0) fail(JAS_EINVAL, "jas_gram: B is NULL");
        if ((flags & JAS_FORCE_POPCOUNT) && (flags & JAS_FORCE_MFMA))
            fail(JAS_EINVAL, "jas_gram: JAS_FORCE_POPCOUNT and JAS_FORCE_MFMA are exclusive");
        const uint32_t var = (flags >> 16) & 0xFFu;
        if (var && (var > (uint32_t)gram_variants() || (flags & (JAS_TUNE | JAS_FORCE_POPCOUNT))))
            fail(JAS_EINVAL, "jas_gram: bad JAS_GRAM_VARIANT");
        if (flags & JAS_ACCUMULATE) {
            if (!card && db->n > 0) fail(JAS_EINVAL, "jas_gram: JAS_ACCUMULATE needs card");
            if (den || J) fail(JAS_EINVAL, "jas_gram: JAS_ACCUMULATE writes no den or J (see jas_finalize)");
            if (flags & (JAS_TUNE | JAS_HOST_PTRS)) fail(JAS_EINVAL, "jas_gram: JAS_ACCUMULATE with JAS_TUNE or JAS_HOST_PTRS");
        }
        hipStream_t s = (hipStream_t)hip_stream;
        const uint64_t n = (uint64_t)db->n;
        const uint64_t len = (flags & JAS_UPPER) ? n * (n + 1) / 2 : n * n;
        if (!(flags & JAS_HOST_PTRS)) {
            JAS_HOST_TIMED("jas_gram");
            gram(db, flags, s, B, card, den, J);
            return;
        }
        DevBuf<int32_t> dB;
        DevBuf<int64_t> dC, dD;
        DevBuf<double> dJ;
        dB.alloc(len, s, nullptr, true, "B staging");
        if (card) dC.alloc(n, s, nullptr, true, "card staging");
        if (den) dD.alloc(len, s, nullptr, true, "den staging");
        if (J) dJ.alloc(len, s, nullptr, true, "J staging");
        gram(db, flags & ~JAS_HOST_PTRS, s, dB.p, card ? dC.p : nullptr, den ? dD.p : nullptr, J ? dJ.p : nullptr);
        JAS_HIP(hipMemcpyAsync(B, dB.p, len * 4, hipMemcpyDeviceToHost, s));
        if (card) JAS_HIP(hipMemcpyAsync(card, dC.p, n * 8, hipMemcpyDeviceToHost, s));
        if (den) JAS_HIP(hipMemcpyAsync(den, dD.p, len * 8, hipMemcpyDeviceToHost, s));
        if (J) JAS_HIP(hipMemcpyAsync(J, dJ.p, len * 8, hipMemcpyDeviceToHost, s));
        JAS_HIP(hipStreamSynchronize(s));
    });
}

jas_status jas_finalize(int32_t n, uint32_t flags, void *hip_stream, int32_t *B, const int64_t *card, int64_t *den,
                        double *J) {
    return guard([&] {
        if (n < 0) fail(JAS_EINVAL, "jas_finalize: n < 0");
        if (flags & ~(uint32_t)JAS_UPPER) fail(JAS_EINVAL, "jas_finalize: only JAS_UPPER is accepted");
        if (n > 0 && (!B || !card)) fail(JAS_EINVAL, "jas_finalize: B or card is NULL");
        JAS_HOST_TIMED("jas_finalize");
        // int32 sums over batches are exact while every summed |X_i| is below
        // the limit (B_ij <= min(|X_i|, |X_j|)); checked before anything is written
        check_card_limit(card, (uint32_t)n, (hipStream_t)hip_stream);
        finalize((uint32_t)n, flags & JAS_UPPER, (hipStream_t)hip_stream, B, card, den, J);
    });
}

jas_status jas_relabel(const uint64_t *ids, uint64_t n_ids, uint32_t universe_bits, void *hip_stream, uint64_t *out,
                       uint64_t *n_distinct, uint32_t *new_universe_bits) {
    return guard([&] {
        if (universe_bits < 1 || universe_bits > 64) fail(JAS_EINVAL, "jas_relabel: universe_bits must be in 1..64");
        if (n_ids > 0 && (!ids || !out)) fail(JAS_EINVAL, "jas_relabel: ids or out is NULL");
        JAS_HOST_TIMED("jas_relabel");
        const uint64_t D = relabel(ids, n_ids, universe_bits, (hipStream_t)hip_stream, out);
        if (n_distinct) *n_distinct = D;
        if (new_universe_bits) *new_universe_bits = std::max<uint32_t>(1, ceil_log2_u64(D));
    });
}

namespace {
void check_seq_off(const uint64_t *seq_off, int64_t n_seq, uint32_t k, const char *what) {
    if (n_seq < 0) fail(JAS_EINVAL, std::string(what) + ": n_seq < 0");
    if (!seq_off) fail(JAS_EINVAL, std::string(what) + ": seq_off is NULL");
    if (k < 1 || k > 31) fail(JAS_EINVAL, std::string(what) + ": k must be 1..31");
    if (seq_off[0] != 0) fail(JAS_EINVAL, std::string(what) + ": seq_off[0] must be 0");
    for (int64_t s = 0; s < n_seq; ++s)
        if (seq_off[s + 1] < seq_off[s])
            fail(JAS_EINVAL, std::string(what) + ": seq_off decreases at sequence " + std::to_string(s));
}
}  // namespace

jas_status jas_kmer_offsets(const uint64_t *seq_off, int64_t n_seq, const uint64_t *smp_off, int32_t n, uint32_t k,
                            uint64_t *ids_off) {
    return guard([&] {
        check_seq_off(seq_off, n_seq, k, "jas_kmer_offsets");
        if (n < 0 || !smp_off || !ids_off) fail(JAS_EINVAL, "jas_kmer_offsets: n < 0 or NULL smp_off / ids_off");
        if (smp_off[0] != 0 || smp_off[n] != (uint64_t)n_seq)
            fail(JAS_EINVAL, "jas_kmer_offsets: smp_off must run from 0 to n_seq");
        for (int32_t i = 0; i < n; ++i)
            if (smp_off[i + 1] < smp_off[i]) fail(JAS_EINVAL, "jas_kmer_offsets: smp_off decreases");
        std::vector<uint64_t> kb;
        kmer_starts(seq_off, n_seq, k, kb);
        for (int32_t i = 0; i <= n; ++i) ids_off[i] = kb[smp_off[i]];
    });
}

jas_status jas_kmers(const uint64_t *seq, const uint64_t *seq_off, int64_t n_seq, uint32_t k, uint32_t flags,
                     void *hip_stream, uint64_t *ids) {
    return guard([&] {
        check_seq_off(seq_off, n_seq, k, "jas_kmers");
        if (flags & ~(uint32_t)JAS_CANONICAL) fail(JAS_EINVAL, "jas_kmers: only JAS_CANONICAL is accepted");
        std::vector<uint64_t> kb;
        if (kmer_starts(seq_off, n_seq, k, kb) == 0) return;
        if (!seq || !ids) fail(JAS_EINVAL, "jas_kmers: seq or ids is NULL");
        JAS_HOST_TIMED("jas_kmers");
        kmers(seq, seq_off, n_seq, k, flags & JAS_CANONICAL, (hipStream_t)hip_stream, ids);
    });
}

jas_status jas_query(const jas_db *db, const uint64_t *q_ids, const uint64_t *q_offsets, int32_t nq, uint32_t flags,
                     void *hip_stream, int32_t *B, int64_t *q_card, int64_t *den, double *J) {
    return guard([&] {
        if (!db) fail(JAS_EINVAL, "jas_query: db is NULL");
        if (!(db->flags & JAS_KEEP_IDS)) fail(JAS_EINVAL, "jas_query: db was encoded without JAS_KEEP_IDS");
        if (nq < 0) fail(JAS_EINVAL, "jas_query: nq < 0");
        if (nq > 0 && !q_offsets) fail(JAS_EINVAL, "jas_query: q_offsets is NULL");
        if (nq > 0 && db->n > 0 && !B) fail(JAS_EINVAL, "jas_query: B is NULL");
        const uint32_t qbits = ceil_log2_u64((uint64_t)std::max<int32_t>(nq, 1));
        if (db->U + qbits > 64) fail(JAS_EINVAL, "jas_query: universe_bits + ceil(log2 nq) exceeds 64");
        hipStream_t s = (hipStream_t)hip_stream;
        const bool host = flags & JAS_HOST_PTRS;
        if (nq == 0) return;
        std::vector<uint64_t> hoff = host_offsets(q_offsets, nq, host, s, "jas_query");
        const uint64_t NQ = hoff[nq];
        if (NQ > 0 && !q_ids) fail(JAS_EINVAL, "jas_query: q_ids is NULL");
        const uint64_t n = (uint64_t)db->n;
        const uint64_t len = (uint64_t)nq * n;
        if (!host) {
            query(db, q_ids, q_offsets, nq, NQ, s, B, q_card, den, J);
            return;
        }
        DevBuf<uint64_t> di, doff;
        DevBuf<int32_t> dB;
        DevBuf<int64_t> dC, dD;
        DevBuf<double> dJ;
        doff.alloc(nq + 1, s, nullptr, true, "query offsets staging");
        JAS_HIP(hipMemcpyAsync(doff.p, hoff.data(), 8 * (nq + 1), hipMemcpyHostToDevice, s));
        di.alloc(std::max<uint64_t>(NQ, 1), s, nullptr, true, "query ids staging");
        if (NQ) JAS_HIP(hipMemcpyAsync(di.p, q_ids, 8 * NQ, hipMemcpyHostToDevice, s));
        dB.alloc(std::max<uint64_t>(len, 1), s, nullptr, true, "B staging");
        if (q_card) dC.alloc(nq, s, nullptr, true, "q_card staging");
        if (den) dD.alloc(std::max<uint64_t>(len, 1), s, nullptr, true, "den staging");
        if (J) dJ.alloc(std::max<uint64_t>(len, 1), s, nullptr, true, "J staging");
        query(db, di.p, doff.p, nq, NQ, s, dB.p, q_card ? dC.p : nullptr, den ? dD.p : nullptr, J ? dJ.p : nullptr);
        if (len) JAS_HIP(hipMemcpyAsync(B, dB.p, len * 4, hipMemcpyDeviceToHost, s));
        if (q_card) JAS_HIP(hipMemcpyAsync(q_card, dC.p, 8 * (uint64_t)nq, hipMemcpyDeviceToHost, s));
        if (den && len) JAS_HIP(hipMemcpyAsync(den, dD.p, len * 8, hipMemcpyDeviceToHost, s));
        if (J && len) JAS_HIP(hipMemcpyAsync(J, dJ.p, len * 8, hipMemcpyDeviceToHost, s));
        JAS_HIP(hipStreamSynchronize(s));
    });
}

jas_status jas_query_noalloc(const jas_db *db, const uint64_t *q_ids, const uint64_t *q_offsets, int32_t nq,
                             uint32_t flags, void *hip_stream, int32_t *B, int64_t *q_card, int64_t *den,
                             double *J) {
    return guard([&] {
        if (!db) fail(JAS_EINVAL, "jas_query_noalloc: db is NULL");
        if (!(db->flags & JAS_KEEP_IDS)) fail(JAS_EINVAL, "jas_query_noalloc: db was encoded without JAS_KEEP_IDS");
        if (flags & ~(uint32_t)JAS_NO_WAIT)
            fail(JAS_EINVAL, "jas_query_noalloc: takes no flag but JAS_NO_WAIT (device pointers only)");
        if (nq < 0) fail(JAS_EINVAL, "jas_query_noalloc: nq < 0");
        if (nq > 0 && !q_offsets) fail(JAS_EINVAL, "jas_query_noalloc: q_offsets is NULL");
        if (nq > 0 && db->n > 0 && !B) fail(JAS_EINVAL, "jas_query_noalloc: B is NULL");
        const uint32_t qbits = ceil_log2_u64((uint64_t)std::max<int32_t>(nq, 1));
        if (db->U + qbits > 64) fail(JAS_EINVAL, "jas_query_noalloc: universe_bits + ceil(log2 nq) exceeds 64");
        if (nq > noalloc_max_queries())
            fail(JAS_ENOMEM, "jas_query_noalloc: " + std::to_string(nq) + " query sets exceed the fixed workspace (at most " +
                                 std::to_string(noalloc_max_queries()) + ")");
        if (nq == 0) return;
        hipStream_t s = (hipStream_t)hip_stream;
        // the workspace first: with JAS_NO_WAIT a refused call has touched nothing
        std::unique_lock<std::mutex> lk;
        Arena ar = noalloc_arena(lk, !(flags & JAS_NO_WAIT));
        const std::vector<uint64_t> hoff = host_offsets(q_offsets, nq, false, s, "jas_query_noalloc");
        const uint64_t NQ = hoff[nq];
        if (NQ > noalloc_max_ids())
            fail(JAS_ENOMEM, "jas_query_noalloc: " + std::to_string(NQ) + " query IDs exceed the fixed workspace (at most " +
                                 std::to_string(noalloc_max_ids()) + ")");
        if (NQ > 0 && !q_ids) fail(JAS_EINVAL, "jas_query_noalloc: q_ids is NULL");
        try {
            query(db, q_ids, q_offsets, nq, NQ, s, B, q_card, den, J, &ar);
        } catch (...) {
            (void)hipStreamSynchronize(s);  // the workspace is free again only when its kernels are done
            throw;
        }
        JAS_HIP(hipStreamSynchronize(s));
    });
}

uint64_t jas_query_workspace_bytes(const jas_db *db, int32_t nq, uint64_t n_q_ids) {
    if (!db || nq < 0) return 0;
    return query_workspace_bytes(db, nq, n_q_ids);
}

}  // extern "C"
