// Encode plans: the batching form as one capturable launch sequence.
//
// jas_plan_create encodes a collection once, the usual way, and keeps what
// that encode decided (the global sort's bits, the range stride, the key
// width in LDS, the row degree threshold) and how large every intermediate
// array was.  It allocates every buffer the encode needs at those sizes plus
// headroom.  jas_plan_encode then encodes a like collection (same n; sizes
// within the capacities) with those buffers: every size is computed and read
// on the device, nothing is read back and nothing allocated, so the caller
// can capture jas_plan_encode, jas_gram and everything else of a step in one
// HIP graph and replay it for each new collection.  What the eager encode
// would have handled differently (a fallback, a buffer too small) is flagged
// on the device and reported by jas_plan_check after the stream completes.
//
// With JAS_TUNE in the options and no fixed threshold, the threshold is
// chosen by timing: each candidate (the cost model's choice, half and twice
// it, every shared row packed, none packed) runs encode + Gram on the
// device, and the fastest is kept.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <memory>

#include "jas_internal.hpp"

struct jas_plan {
    int device = 0;
    jas_db db;  // views the plan's buffers (W, card, pair words); its budget counts them
    jas::PlanState st;  // destroyed before db (members go in reverse order)
    uint32_t tuned_dmin = 0;
    std::vector<std::pair<uint32_t, double>> tuning;  // (threshold, ms) when tuned
};

namespace jas {
namespace {

uint64_t grow(uint64_t v, double headroom, uint64_t extra) {
    return (uint64_t)std::ceil((double)v * (1.0 + headroom)) + extra;
}

template <class T>
void plan_buf(DevBuf<T> &b, uint64_t count, hipStream_t s, Budget *budget, const char *what) {
    b.alloc(std::max<uint64_t>(count, 1), s, budget, false, what);
}

// encode + Gram of the collection with threshold t, timed on the device (ms)
double time_threshold(const uint64_t *ids, const uint64_t *offsets, int32_t n, const jas_encode_opts &o0, uint32_t t,
                      hipStream_t s, int32_t *B) {
    jas_encode_opts o = o0;
    o.dense_min_degree = t;
    o.flags &= ~(uint32_t)JAS_TUNE;
    jas_db *db = nullptr;
    const auto t0 = std::chrono::steady_clock::now();
    jas_status st = jas_encode(ids, offsets, n, &o, s, &db, nullptr);
    if (st != JAS_OK) fail(st, std::string("plan tuning: ") + jas_last_error());
    st = jas_gram(db, JAS_UPPER, s, B, nullptr, nullptr, nullptr);
    if (st != JAS_OK) {
        jas_db_free(db);
        fail(st, std::string("plan tuning: ") + jas_last_error());
    }
    JAS_HIP(hipStreamSynchronize(s));
    const double ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    jas_db_free(db);
    return ms;
}

}  // namespace
}  // namespace jas

using namespace jas;

extern "C" {

jas_status jas_plan_create(const uint64_t *ids, const uint64_t *offsets, int32_t n, const jas_encode_opts *opts,
                           double headroom, void *hip_stream, jas_plan **plan_out) {
    return guarded([&] {
        if (!plan_out) fail(JAS_EINVAL, "jas_plan_create: plan_out is NULL");
        *plan_out = nullptr;
        if (!opts) fail(JAS_EINVAL, "jas_plan_create: opts is NULL");
        if (opts->flags & (JAS_HOST_PTRS | JAS_KEEP_IDS))
            fail(JAS_EINVAL, "jas_plan_create: device pointers only, and no JAS_KEEP_IDS (plans are for all pairs)");
        if (n < 1 || n > kSampleMajorMaxN)
            fail(JAS_EINVAL, "jas_plan_create: n must be in 1.." + std::to_string(kSampleMajorMaxN));
        if (!(headroom >= 0.0 && headroom <= 4.0)) fail(JAS_EINVAL, "jas_plan_create: headroom must be in [0, 4]");
        hipStream_t s = (hipStream_t)hip_stream;
        std::unique_ptr<jas_plan> plan(new jas_plan());
        JAS_HIP(hipGetDevice(&plan->device));
        jas_encode_opts o = *opts;
        o.flags &= ~(uint32_t)JAS_TUNE;
        // the threshold: fixed, the cost model's, or the fastest candidate timed on the device
        if (opts->dense_min_degree == 0 && (opts->flags & JAS_TUNE)) {
            jas_db *db0 = nullptr;
            jas_encode_stats st0{};
            jas_status e = jas_encode(ids, offsets, n, &o, s, &db0, &st0);
            if (e != JAS_OK) fail(e, std::string("jas_plan_create: ") + jas_last_error());
            jas_db_free(db0);
            const uint32_t t = (uint32_t)st0.dense_min_degree, top = (uint32_t)n + 1;
            std::vector<uint32_t> cand = {t, std::max<uint32_t>(2, t / 2), std::min(top, 2 * t), 2u, top};
            std::sort(cand.begin(), cand.end());
            cand.erase(std::unique(cand.begin(), cand.end()), cand.end());
            DevBuf<int32_t> B;
            B.alloc((uint64_t)n * (n + 1) / 2, s, nullptr, true, "plan tuning output");
            double best = INFINITY;
            for (uint32_t c : cand) {
                (void)time_threshold(ids, offsets, n, o, c, s, B.p);  // warm (the encode's cache)
                const double ms = time_threshold(ids, offsets, n, o, c, s, B.p);
                plan->tuning.emplace_back(c, ms);
                if (ms < best) {
                    best = ms;
                    plan->tuned_dmin = c;
                }
            }
            o.dense_min_degree = plan->tuned_dmin;
        }
        // one eager encode: its decisions and sizes
        jas_db *db0 = nullptr;
        jas_status e = jas_encode(ids, offsets, n, &o, s, &db0, nullptr);
        if (e != JAS_OK) fail(e, std::string("jas_plan_create: ") + jas_last_error());
        const EncodeTrace tr = db0->trace;
        const uint32_t dmin = db0->dmin ? db0->dmin : 2;
        const uint32_t U = db0->U, sbits = db0->sbits, bb = db0->batch_bits, wb = db0->word_bits;
        jas_db_free(db0);
        if (!tr.onesweep || (tr.N > kLocalCapKeys && !tr.local))
            fail(JAS_EUNSUPPORTED, "jas_plan_create: this collection needs the encoder's fallback paths");
        if (tr.QL > 0 && !tr.pairs) fail(JAS_EUNSUPPORTED, "jas_plan_create: row lists need the pair form");
        PlanState &p = plan->st;
        p.n = n;
        p.U = U;
        p.sbits = sbits;
        p.batch_bits = bb;
        p.word_bits = wb;
        p.dmin = dmin;
        p.sort = sort_plan(tr.N, U, sbits);
        p.stride = tr.stride ? tr.stride : kLocalStrides[0];
        p.lcap = tr.lcap ? tr.lcap : kLocalShortCap;
        p.wide = tr.wide;
        p.ldw = div_up((uint64_t)n, 128) * 128;
        p.Ncap = std::max<uint64_t>(grow(tr.N, headroom, 64), kLocalCapKeys + 1);
        p.nlc_cap = div_up(p.Ncap, p.stride);
        p.Rcap = grow(tr.R, headroom, 64);
        // each form gets room whenever the threshold admits it, also where the
        // planning collection had none of its rows (a like collection may)
        const bool can_pack = dmin <= (uint32_t)n, can_list = dmin > 2;
        p.QDcap = can_pack ? std::min(p.Rcap, grow(tr.QD, headroom, 64)) : 0;
        p.QLcap = can_list ? std::min(p.Rcap, grow(tr.QL, headroom, 64)) : 0;
        p.Hwcap = p.QDcap ? grow(tr.Hw, headroom, 64) : 0;
        p.Hcap = wb == 64 ? p.Hwcap : div_up(p.Hwcap, 2);
        p.Pcap = p.QLcap ? grow(tr.P, headroom, 1024) : 0;
        p.tile_cap = div_up(p.Rcap, kSplitTilePub);
        p.gcap = div_up(p.QLcap, (uint64_t)64);
        p.pair_bits = std::max<uint32_t>(1, ceil_log2_u64((uint64_t)n));
        p.pair_npass = (p.pair_bits + 7) / 8;
        p.pair_width = (p.pair_bits + p.pair_npass - 1) / p.pair_npass;
        if (p.nlc_cap > 0xFFFFFFFFull || div_up(p.Ncap, 65536) > 0xFFFFFFFFull || p.tile_cap > 0xFFFFFFFFull)
            fail(JAS_EUNSUPPORTED, "jas_plan_create: collection too large for a plan");
        // every buffer, within the HBM budget
        Budget &bud = plan->db.budget;
        bud.limit = opts->hbm_budget_bytes;
        plan_buf(p.keys, p.Ncap + 2, s, &bud, "plan keys");
        plan_buf(p.alt, p.Ncap + 2, s, &bud, "plan keys (second buffer)");
        plan_buf(p.dsz, PZ_COUNT, s, &bud, "plan sizes");
        plan_buf(p.err, 4, s, &bud, "plan flags");
        plan_buf(p.st, ST_N_, s, &bud, "plan counters");
        plan_buf(p.ghist, (uint64_t)kGhistReplicas * kMaxPasses * 256, s, &bud, "plan digit totals");
        plan_buf(p.os_gstart, (uint64_t)kMaxPasses * 256, s, &bud, "plan digit starts");
        plan_buf(p.os_maxima, kMaxPasses, s, &bud, "plan digit maxima");
        plan_buf(p.os_status, onesweep_status_words(p.Ncap, false), s, &bud, "plan look-back status");
        plan_buf(p.os_ticket, 1, s, &bud, "plan tile ticket");
        if (p.sort.top_bits > 0)
            plan_buf(p.os_tinfo, 2 * div_up(p.Ncap, onesweep_tile_keys_u64()), s, &bud, "plan tile samples");
        plan_buf(p.rs, p.nlc_cap + 1, s, &bud, "plan range starts");
        plan_buf(p.dupc, (uint64_t)n + kStatReplicasPub, s, &bud, "plan repeat counts");
        plan_buf(p.cnt, 3 * p.nlc_cap, s, &bud, "plan range counts");
        plan_buf(p.rid_g, p.Ncap / 2 + 1, s, &bud, "plan row ids (by range)");
        plan_buf(p.offD, p.nlc_cap + 1, s, &bud, "plan range offsets");
        plan_buf(p.offS, p.nlc_cap + 1, s, &bud, "plan range offsets");
        plan_buf(p.offR, p.nlc_cap + 1, s, &bud, "plan range offsets");
        const uint64_t scan_len = std::max({p.nlc_cap, p.tile_cap, p.QDcap, p.gcap, (uint64_t)1});
        plan_buf(p.stmp, scan_tmp_elems(scan_len), s, &bud, "plan scan scratch");
        plan_buf(p.rid, p.Rcap + 1, s, &bud, "plan row ids");
        plan_buf(p.rptr, p.Rcap + 1, s, &bud, "plan row pointers");
        plan_buf(p.rdeg, p.Rcap + 1, s, &bud, "plan row degrees");
        plan_buf(p.card, (uint64_t)n, s, &bud, "plan card");
        plan_buf(p.tcnt, p.tile_cap, s, &bud, "plan row tile counts");
        plan_buf(p.toff, p.tile_cap + 1, s, &bud, "plan row tile offsets");
        plan_buf(p.lprep, kStatReplicasPub, s, &bud, "plan list pair counters");
        plan_buf(p.Drow, p.QDcap, s, &bud, "plan packed rows");
        plan_buf(p.Lrow, p.QLcap, s, &bud, "plan list rows");
        if (p.QDcap) {
            plan_buf(p.bs, p.QDcap, s, &bud, "plan batch flags");
            plan_buf(p.bpos, p.QDcap + 1, s, &bud, "plan batch scan");
            plan_buf(p.bq, p.QDcap + 1, s, &bud, "plan batch starts");
            plan_buf(p.nw, p.QDcap, s, &bud, "plan batch words");
            plan_buf(p.wbase, p.QDcap + 1, s, &bud, "plan word bases");
            plan_buf(p.wq0, p.Hwcap, s, &bud, "plan word rows");
            plan_buf(p.wq1, p.Hwcap, s, &bud, "plan word rows");
            plan_buf(p.W, p.Hcap * p.ldw, s, &bud, "plan packed words");
        }
        if (p.QLcap) {
            plan_buf(p.np, p.gcap, s, &bud, "plan row group pair counts");
            plan_buf(p.npo, p.gcap + 1, s, &bud, "plan row group pair offsets");
            plan_buf(p.pk, p.Pcap + 2, s, &bud, "plan row-list pairs");
            plan_buf(p.palt, p.Pcap + 2, s, &bud, "plan row-list pairs (second buffer)");
            plan_buf(p.gh, (uint64_t)kGhistReplicas * kMaxPasses * 256, s, &bud, "plan pair digit totals");
            plan_buf(p.os2_gstart, (uint64_t)kMaxPasses * 256, s, &bud, "plan pair digit starts");
            plan_buf(p.os2_maxima, kMaxPasses, s, &bud, "plan pair digit maxima");
            plan_buf(p.os2_status, onesweep_status_words(p.Pcap, true), s, &bud, "plan pair look-back status");
            plan_buf(p.os2_ticket, 1, s, &bud, "plan pair tile ticket");
            p.pairs_final = (p.pair_npass % 2) ? p.palt.p : p.pk.p;
        }
        // the plan's db: views of the plan's buffers
        jas_db &db = plan->db;
        db.device = plan->device;
        db.n = n;
        db.U = U;
        db.sbits = sbits;
        db.batch_bits = bb;
        db.word_bits = wb;
        db.dmin = dmin;
        db.flags = 0;
        db.card.wrap(p.card.p, (uint64_t)n);
        db.H = p.QDcap ? p.Hcap : 0;
        if (p.QDcap) db.W.wrap(p.W.p, p.W.n);
        db.n_list = p.QLcap;
        db.n_lpairs = p.QLcap ? p.Pcap : 0;
        if (p.QLcap) db.pairs.wrap(p.pairs_final, p.Pcap + 2);
        db.dsz = p.dsz.p;
        db.stats.dense_min_degree = dmin;
        db.stats.word_bits = wb;
        db.stats.w_rows = db.H;
        db.stats.w_stride = p.ldw;
        bud.limit = 0;
        db.stats.device_bytes = bud.held;
        JAS_HIP(hipStreamSynchronize(s));
        *plan_out = plan.release();
    });
}

jas_status jas_plan_encode(jas_plan *plan, const uint64_t *ids, const uint64_t *offsets, void *hip_stream) {
    return guarded([&] {
        if (!plan) fail(JAS_EINVAL, "jas_plan_encode: plan is NULL");
        if (!offsets || !ids) fail(JAS_EINVAL, "jas_plan_encode: ids or offsets is NULL");
        int dev = 0;
        JAS_HIP(hipGetDevice(&dev));
        if (dev != plan->device) fail(JAS_EINVAL, "jas_plan_encode: the current device is not the plan's");
        encode_planned(plan->st, ids, offsets, (hipStream_t)hip_stream);
    });
}

const jas_db *jas_plan_db(const jas_plan *plan) { return plan ? &plan->db : nullptr; }

uint32_t jas_plan_threshold(const jas_plan *plan) { return plan ? plan->st.dmin : 0; }

jas_status jas_plan_check(jas_plan *plan, void *hip_stream, jas_encode_stats *stats) {
    return guarded([&] {
        if (!plan) fail(JAS_EINVAL, "jas_plan_check: plan is NULL");
        hipStream_t s = (hipStream_t)hip_stream;
        PlanState &p = plan->st;
        uint32_t err[4] = {0, 0, 0, 0};
        uint64_t sz[PZ_COUNT];
        unsigned long long cnt[ST_N_];
        JAS_HIP(hipMemcpyAsync(err, p.err.p, sizeof(err), hipMemcpyDeviceToHost, s));
        JAS_HIP(hipMemcpyAsync(sz, p.dsz.p, sizeof(sz), hipMemcpyDeviceToHost, s));
        JAS_HIP(hipMemcpyAsync(cnt, p.st.p, sizeof(cnt), hipMemcpyDeviceToHost, s));
        JAS_HIP(hipStreamSynchronize(s));
        jas_encode_stats &o = plan->db.stats;
        o.n_ids = sz[PZ_N];
        o.n_rows = cnt[ST_ROWS_];
        o.n_shared_rows = sz[PZ_R];
        o.n_packed_rows = sz[PZ_QD];
        o.n_list_rows = sz[PZ_QL];
        o.n_batches = sz[PZ_NB];
        o.n_word_rows = sz[PZ_HW];
        o.nnz_words = cnt[ST_NNZW_];
        o.word_pairs_F = cnt[ST_F_];
        o.list_pairs = cnt[ST_LISTPAIRS_];
        o.n_list_pairs = sz[PZ_P];
        o.w_rows = sz[PZ_H];
        set_tile_stats(o, (uint64_t)p.n);
        if (stats) *stats = o;
        const uint32_t e = err[0] & ~(p.wide ? 16u : 0u);
        if (e & 1u) fail(JAS_EINVAL, "jas_plan_encode: an ID is >= 2^universe_bits");
        if (e & 32u) {
            static const char *names[] = {"IDs", "shared rows", "packed rows", "list rows", "batches", "word rows",
                                          "W rows", "list pairs"};
            const uint64_t k = sz[PZ_OVER];
            const uint64_t caps[] = {p.Ncap, p.Rcap, p.QDcap, p.QLcap, p.QDcap, p.Hwcap, p.Hcap, p.Pcap};
            std::string what = "a size";
            if (k >= 1 && k <= 8)
                what = std::to_string(sz[PZ_OVER_VALUE]) + " " + names[k - 1] + " (capacity " +
                       std::to_string(caps[k - 1]) + ")";
            fail(JAS_ENOMEM, "jas_plan_encode: " + what + " exceeded the plan (plan with more headroom)");
        }
        if (e & 8u) fail(JAS_EUNSUPPORTED, "jas_plan_encode: a range of buckets exceeds the LDS capacity at the "
                                           "planned stride (plan on this collection)");
        if (e & 16u) fail(JAS_EUNSUPPORTED, "jas_plan_encode: keys need 64 bits in LDS (plan on this collection)");
        if (e & 4u) fail(JAS_EUNSUPPORTED, "jas_plan_encode: a digit total is too large for the single-pass sort");
        if (e & 2u) fail(JAS_EDEVICE, "jas_plan_encode: the radix sort's look-back waited too long");
        if (e & 64u) fail(JAS_EOVERFLOW, "jas_plan_encode: a set has " + std::to_string(card_limit()) +
                                             " or more distinct IDs");
    });
}

int32_t jas_plan_tuning(const jas_plan *plan, uint32_t *thresholds, double *ms, int32_t cap) {
    if (!plan) return 0;
    const int32_t k = (int32_t)plan->tuning.size();
    for (int32_t i = 0; i < std::min(k, cap); ++i) {
        if (thresholds) thresholds[i] = plan->tuning[i].first;
        if (ms) ms[i] = plan->tuning[i].second;
    }
    return k;
}

void jas_plan_free(jas_plan *plan) {
    if (!plan) return;
    int cur = 0;
    const int dev = plan->device;
    (void)hipGetDevice(&cur);
    if (cur != dev) (void)hipSetDevice(dev);
    (void)hipDeviceSynchronize();
    delete plan;
    if (cur != dev) (void)hipSetDevice(cur);
}

}  // extern "C"
