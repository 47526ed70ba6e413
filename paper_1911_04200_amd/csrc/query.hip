// Query x database similarity: Eq. (1) with i over query sets, j over the
// encoded samples.
//
// The query block of B is B_qj = sum_k q_k a_kj over rows k of A.  Query sets
// are made sets like the database (keys (q << U) | id, stable radix sort,
// repeats dropped); each distinct query ID is looked up in the database's
// sorted distinct keys (a table of start positions by the ID's top bits,
// then a binary search), and every database sample holding that ID gains 1.
// One block works on one query's slice of IDs and accumulates its row of B in
// LDS before adding it to global memory.
#include <algorithm>

#include "device_util.hpp"
#include "jas_internal.hpp"

namespace jas {
namespace {

constexpr int kNT = 256;
constexpr uint64_t kQChunk = 2048;  // query entries per block (more blocks than CUs for typical requests)
constexpr int32_t kHistMax = 16384;

// Keys (q << U) | id of 4096 entries per block, and the totals of every
// 8-bit digit of the keys (kGhistReplicas copies) for the single-pass sort.
__global__ __launch_bounds__(kNT) void k_qkeys(const uint64_t *__restrict__ ids, const uint64_t *__restrict__ off,
                                                int32_t nq, uint64_t N, uint32_t U, uint64_t *__restrict__ keys,
                                                uint32_t *err, uint32_t npass, unsigned long long *__restrict__ ghist) {
    __shared__ int32_t s_lo, s_hi;
    __shared__ uint32_t gh[kMaxPasses][256];
    const uint64_t b0 = (uint64_t)blockIdx.x * 4096;
    const uint64_t b1 = min(N, b0 + 4096);
#pragma unroll
    for (int k = 0; k < kMaxPasses; ++k) gh[k][threadIdx.x] = 0;
    if (threadIdx.x == 0) {
        s_lo = find_sample(off, 0, nq - 1, b0);
        s_hi = find_sample(off, s_lo, nq - 1, b1 - 1);
    }
    __syncthreads();
    const uint64_t hi_mask = ~((uint64_t(1) << U) - 1);
    uint32_t bad = 0;
    for (uint64_t t = b0 + threadIdx.x; t < b1; t += kNT) {
        const int32_t q = find_sample(off, s_lo, s_hi, t);
        const uint64_t id = ids[t];
        bad |= (id & hi_mask) != 0;
        const uint64_t key = ((uint64_t)q << U) | (id & ~hi_mask);
        keys[t] = key;
        for (uint32_t p = 0; p < npass; ++p) atomicAdd(&gh[p][(uint32_t)(key >> (8 * p)) & 255u], 1u);
    }
    if (__ballot(bad) && lane_id() == 0) atomicOr(err, 1u);
    __syncthreads();
    if (ghist) {
        unsigned long long *g = ghist + (uint64_t)(blockIdx.x % kGhistReplicas) * kMaxPasses * 256;
        for (uint32_t p = 0; p < npass; ++p)
            if (gh[p][threadIdx.x]) atomicAdd(&g[p * 256 + threadIdx.x], (unsigned long long)gh[p][threadIdx.x]);
    }
}

__global__ void k_qblocks(const uint64_t *off, int32_t nq, uint64_t *nb) {
    for (int32_t q = blockIdx.x * blockDim.x + threadIdx.x; q < nq; q += gridDim.x * blockDim.x)
        nb[q] = (off[q + 1] - off[q] + kQChunk - 1) / kQChunk;
}

__global__ void k_fill_i32(int32_t *p, uint64_t len, int32_t v) {
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < len; i += (uint64_t)gridDim.x * blockDim.x)
        p[i] = v;
}
__global__ void k_fill_u32(uint32_t *p, uint64_t len) {
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < len; i += (uint64_t)gridDim.x * blockDim.x)
        p[i] = 0;
}
__global__ void k_fill_u64(unsigned long long *p, uint64_t len) {
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < len; i += (uint64_t)gridDim.x * blockDim.x)
        p[i] = 0;
}

__global__ __launch_bounds__(kNT) void k_qlookup(const uint64_t *__restrict__ K, const uint64_t *__restrict__ qoff,
                                                  int32_t nq, const uint64_t *__restrict__ bo, uint32_t U,
                                                  const uint64_t *__restrict__ Dk, uint64_t ND,
                                                  const uint64_t *__restrict__ bucket, uint32_t ibits,
                                                  uint32_t sbits, uint32_t n, int lds, int32_t *__restrict__ B,
                                                  unsigned long long *__restrict__ qcard) {
    extern __shared__ uint32_t hist[];
    __shared__ uint64_t sh[kNT / kWave];
    const uint32_t tid = threadIdx.x;
    // block -> (query, slice)
    int32_t lo = 0, hi = nq - 1;
    while (lo < hi) {
        const int32_t mid = (lo + hi + 1) >> 1;
        if (bo[mid] <= blockIdx.x) lo = mid;
        else hi = mid - 1;
    }
    const int32_t q = lo;
    const uint64_t qs = qoff[q];
    const uint64_t t0 = qs + (blockIdx.x - bo[q]) * kQChunk;
    const uint64_t t1 = min(qoff[q + 1], t0 + kQChunk);
    if (lds)
        for (uint32_t i = tid; i < n; i += kNT) hist[i] = 0;
    __syncthreads();
    const uint64_t umask = (uint64_t(1) << U) - 1;
    const uint64_t smask = sbits ? (uint64_t(1) << sbits) - 1 : 0;
    const uint32_t shift = U - ibits;
    uint32_t cnt = 0;
    for (uint64_t t = t0 + tid; t < t1; t += kNT) {
        const uint64_t key = K[t];
        if (t > qs && K[t - 1] == key) continue;  // repeat inside this query set
        ++cnt;
        const uint64_t id = key & umask;
        const uint64_t bk = id >> shift;
        uint64_t a = bucket[bk], b = bucket[bk + 1];
        const uint64_t target = id << sbits;
        while (a < b) {
            const uint64_t m = (a + b) >> 1;
            if (Dk[m] < target) a = m + 1;
            else b = m;
        }
        for (uint64_t u = a; u < ND; ++u) {
            const uint64_t d = Dk[u];
            if ((d >> sbits) != id) break;
            const uint32_t s = (uint32_t)(d & smask);
            if (lds) atomicAdd(&hist[s], 1u);
            else atomicAdd(&B[(uint64_t)q * n + s], 1);
        }
    }
    uint64_t tot;
    block_excl_scan<kNT>(cnt, sh, &tot);
    if (tid == 0 && tot) atomicAdd(&qcard[q], (unsigned long long)tot);
    if (lds)
        for (uint32_t i = tid; i < n; i += kNT)
            if (hist[i]) atomicAdd(&B[(uint64_t)q * n + i], (int32_t)hist[i]);
}

__global__ void k_qfinalize(const int32_t *__restrict__ B, const unsigned long long *__restrict__ qcard,
                            const int64_t *__restrict__ card, int32_t nq, uint32_t n, int64_t *__restrict__ q_card,
                            int64_t *__restrict__ den, double *__restrict__ J) {
    const uint64_t total = (uint64_t)nq * n;
    for (uint64_t p = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; p < total; p += (uint64_t)gridDim.x * blockDim.x) {
        const uint64_t q = p / n, j = p % n;
        const int64_t b = B[p];
        const int64_t c = (int64_t)qcard[q] + card[j] - b;
        if (den) den[p] = c;
        if (J) J[p] = c == 0 ? 1.0 : (double)b / (double)c;
        if (q_card && j == 0) q_card[q] = (int64_t)qcard[q];
    }
}

}  // namespace

uint64_t query_workspace_bytes(const jas_db *db, int32_t nq, uint64_t n_q_ids) {
    (void)db;
    // keys and second buffer, the per-pass fallback's counts, look-back status
    // (1 KiB per 8192 keys), digit totals and starts, per-query blocks
    const uint64_t nk = std::max<uint64_t>(n_q_ids, 1);
    return 2 * 8 * nk + radix_work_bytes(n_q_ids) + (nk / 8192 + 1) * 1024 + 4 + 2 * (uint64_t)kGhistReplicas * 8 * 256 * 8 +
           8 * (uint64_t)(nq + 1) * 4 + scan_tmp_elems(nq) * 8 + 4096;
}

void query(const jas_db *db, const uint64_t *q_ids, const uint64_t *q_offsets, int32_t nq, uint64_t NQ,
           hipStream_t s, int32_t *B, int64_t *q_card, int64_t *den, double *J, Arena *ar) {
    const uint32_t n = (uint32_t)db->n;
    const uint32_t U = db->U;
    const uint32_t qbits = ceil_log2_u64((uint64_t)std::max<int32_t>(nq, 1));
    if (U + qbits > 64) fail(JAS_EINVAL, "universe_bits + ceil(log2 nq) exceeds 64");
    if (nq == 0) return;
    const uint64_t len = (uint64_t)nq * n;
    if (n > 0) {
        {
            JAS_TIMED("fill_i32", s);
            k_fill_i32<<<(uint32_t)std::min<uint64_t>(div_up(len, 256), 65536), 256, 0, s>>>(B, len, 0);
        }
        check_launch("zero B");
    }
    DevBuf<unsigned long long> qc;
    temp_buf(qc, nq, s, nullptr, ar, "query card");
    {
        JAS_TIMED("fill_u64", s);
        k_fill_u64<<<(uint32_t)div_up(nq, 256), 256, 0, s>>>(qc.p, nq);
    }
    check_launch("zero query card");
    if (NQ > 0) {
        DevBuf<uint64_t> keys, alt;
        DevBuf<uint32_t> err;
        temp_buf(keys, NQ, s, nullptr, ar, "query keys");
        temp_buf(alt, NQ, s, nullptr, ar, "query keys");
        temp_buf(err, 1, s, nullptr, ar, "query error flag");
        {
            JAS_TIMED("fill_u32", s);
            k_fill_u32<<<1, 64, 0, s>>>(err.p, 1);
        }
        const uint64_t kb = div_up(NQ, 4096);
        const uint32_t kbits = U + qbits, npass = (kbits + 7) / 8;
        DevBuf<unsigned long long> ghist;
        temp_buf(ghist, (uint64_t)kGhistReplicas * kMaxPasses * 256, s, nullptr, ar, "query digit totals");
        {
            JAS_TIMED("fill_u64", s);
            k_fill_u64<<<64, 256, 0, s>>>(ghist.p, (uint64_t)kGhistReplicas * kMaxPasses * 256);
        }
        {
            JAS_TIMED("qkeys", s);
            k_qkeys<<<(uint32_t)kb, kNT, 0, s>>>(q_ids, q_offsets, nq, NQ, U, keys.p, err.p, npass, ghist.p);
        }
        check_launch("query keys");
        uint32_t herr = 0;
        JAS_HIP(hipMemcpyAsync(&herr, err.p, 4, hipMemcpyDeviceToHost, s));
        JAS_HIP(hipStreamSynchronize(s));
        if (herr) fail(JAS_EINVAL, "a query ID is >= 2^universe_bits");
        // single-pass scatters; if one cannot run (or its look-back gave up),
        // the keys are rebuilt and sorted with per-pass histograms instead
        bool sorted = radix_sort_onesweep(keys, alt, NQ, 0, kbits, 8, ghist.p, err.p, s, nullptr, ar);
        if (sorted) {
            JAS_HIP(hipMemcpyAsync(&herr, err.p, 4, hipMemcpyDeviceToHost, s));
            JAS_HIP(hipStreamSynchronize(s));
            sorted = herr == 0;
        }
        if (!sorted) {
            {
                JAS_TIMED("fill_u32", s);
                k_fill_u32<<<1, 64, 0, s>>>(err.p, 1);
            }
            k_qkeys<<<(uint32_t)kb, kNT, 0, s>>>(q_ids, q_offsets, nq, NQ, U, keys.p, err.p, 0, nullptr);
            check_launch("query keys");
            RadixWork rw;
            radix_sort_u64(keys, alt, NQ, 0, kbits, rw, s, nullptr, ar);
        }
        alt.release();
        DevBuf<uint64_t> nb, bo, tmp;
        temp_buf(nb, nq, s, nullptr, ar, "query blocks");
        temp_buf(bo, nq + 1, s, nullptr, ar, "query blocks");
        temp_buf(tmp, scan_tmp_elems(nq), s, nullptr, ar, "scan scratch");
        {
            JAS_TIMED("qblocks", s);
            k_qblocks<<<(uint32_t)div_up(nq, 256), 256, 0, s>>>(q_offsets, nq, nb.p);
        }
        scan_excl_u64(nb.p, bo.p, nq, tmp.p, s);
        const uint64_t total_blocks = div_up(NQ, kQChunk) + (uint64_t)nq;  // upper bound
        uint64_t hb = 0;
        JAS_HIP(hipMemcpyAsync(&hb, bo.p + nq, 8, hipMemcpyDeviceToHost, s));
        JAS_HIP(hipStreamSynchronize(s));
        if (hb > total_blocks || hb > 0xFFFFFFFFull) fail(JAS_EDEVICE, "query block count");
        if (hb > 0 && n > 0 && db->n_keys > 0) {
            const int lds = (int32_t)n <= kHistMax;
            {
                JAS_TIMED("qlookup", s);
                k_qlookup<<<(uint32_t)hb, kNT, lds ? n * sizeof(uint32_t) : 0, s>>>(
                    keys.p, q_offsets, nq, bo.p, U, db->keys.p, db->n_keys, db->bucket.p, db->ibits, db->sbits, n, lds,
                    B, qc.p);
            }
            check_launch("query lookup");
        } else if (hb > 0) {
            // empty database side: only |Q| is needed
            {
                JAS_TIMED("qlookup", s);
                k_qlookup<<<(uint32_t)hb, kNT, 0, s>>>(keys.p, q_offsets, nq, bo.p, U, db->keys.p, 0, db->bucket.p,
                                                       db->ibits, db->sbits, 0, 0, B, qc.p);
            }
            check_launch("query lookup");
        }
    }
    const uint64_t blocks = std::max<uint64_t>(1, std::min<uint64_t>(div_up(std::max<uint64_t>(len, nq), 256), 65536));
    if (n > 0) {
        {
            JAS_TIMED("qfinalize", s);
            k_qfinalize<<<(uint32_t)blocks, 256, 0, s>>>(B, qc.p, db->card.p, nq, n, q_card, den, J);
        }
        check_launch("query finalize");
    } else if (q_card) {
        JAS_HIP(hipMemcpyAsync(q_card, qc.p, sizeof(int64_t) * nq, hipMemcpyDeviceToDevice, s));
    }
}

}  // namespace jas
