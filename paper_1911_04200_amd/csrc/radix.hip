// Stable LSD radix sort of 64-bit keys on a bit range (8-bit digits).
//
// Used to group equal IDs (the zero-row filter f of Eq. (5) and the
// compaction of Eq. (6) need every nonzero row's entries together).
// Each pass is reduce-then-scan with no inter-block waiting:
//   1. k_radix_hist:    per-chunk digit histograms (digit-major counts[d][chunk]);
//   2. exclusive scan:  global start of every (digit, chunk) bucket;
//   3. k_radix_scatter: per 4096-key tile, a wave64 ballot multisplit ranks
//      keys by digit (stable: waves own consecutive quarters of the tile,
//      rounds go in order), the tile is reordered in LDS, and each digit run
//      is written out contiguously (coalesced).
#include <algorithm>

#include "device_util.hpp"
#include "jas_internal.hpp"

namespace jas {
namespace {

constexpr int kNT = 256;                     // 4 waves
constexpr int kWaves = kNT / kWave;
constexpr int kRounds = 16;                  // keys per lane per tile
constexpr uint32_t kTile = kNT * kRounds;    // 4096 keys
constexpr uint32_t kTilesPerChunk = 16;
constexpr uint64_t kChunk = (uint64_t)kTile * kTilesPerChunk;  // 65536 keys per block
constexpr int kRadix = 256;

__global__ __launch_bounds__(kNT) void k_radix_hist(const uint64_t *__restrict__ keys, uint64_t N, uint32_t shift,
                                                     uint32_t mask, uint32_t *__restrict__ counts,
                                                     uint32_t nchunks) {
    __shared__ uint32_t h[kWaves][kRadix];
    const uint32_t tid = threadIdx.x, w = tid / kWave;
#pragma unroll
    for (int k = 0; k < kWaves; ++k) h[k][tid] = 0;
    __syncthreads();
    const uint64_t c0 = (uint64_t)blockIdx.x * kChunk;
    const uint64_t c1 = min(N, c0 + kChunk);
    for (uint64_t t0 = c0; t0 < c1; t0 += kTile) {
        uint64_t k[kRounds];
#pragma unroll
        for (int j = 0; j < kRounds; ++j) {
            const uint64_t t = t0 + (uint64_t)j * kNT + tid;
            k[j] = t < c1 ? keys[t] : 0;
        }
#pragma unroll
        for (int j = 0; j < kRounds; ++j) {
            const uint64_t t = t0 + (uint64_t)j * kNT + tid;
            if (t < c1) atomicAdd(&h[w][(uint32_t)(k[j] >> shift) & mask], 1u);
        }
    }
    __syncthreads();
    uint32_t c = 0;
#pragma unroll
    for (int k = 0; k < kWaves; ++k) c += h[k][tid];
    counts[(uint64_t)tid * nchunks + blockIdx.x] = c;
}

__global__ __launch_bounds__(kNT) void k_radix_scatter(const uint64_t *__restrict__ in, uint64_t *__restrict__ out,
                                                        uint64_t N, uint32_t shift, uint32_t nbits,
                                                        const uint64_t *__restrict__ offs, uint32_t nchunks) {
    __shared__ uint64_t stage[kTile];
    __shared__ uint32_t wcnt[kWaves][kRadix];
    __shared__ uint32_t tdp[kRadix];
    __shared__ uint64_t base[kRadix];
    __shared__ uint64_t sh[kWaves];
    const uint32_t tid = threadIdx.x, lane = lane_id(), w = tid / kWave;
    const uint32_t mask = (1u << nbits) - 1u;
    const uint64_t c0 = (uint64_t)blockIdx.x * kChunk;
    const uint64_t c1 = min(N, c0 + kChunk);
    const uint64_t lt = lanemask_lt();
    base[tid] = offs[(uint64_t)tid * nchunks + blockIdx.x];

    for (uint64_t t0 = c0; t0 < c1; t0 += kTile) {
#pragma unroll
        for (int k = 0; k < kWaves; ++k) wcnt[k][tid] = 0;
        __syncthreads();
        // wave w owns positions [t0 + w*1024, t0 + (w+1)*1024), 64 per round
        const uint64_t wb = t0 + (uint64_t)w * (kTile / kWaves);
        uint64_t key[kRounds];
        uint32_t rank[kRounds];
#pragma unroll
        for (int j = 0; j < kRounds; ++j) {
            const uint64_t t = wb + (uint64_t)j * kWave + lane;
            key[j] = t < c1 ? in[t] : 0;
        }
#pragma unroll
        for (int j = 0; j < kRounds; ++j) {
            const uint64_t t = wb + (uint64_t)j * kWave + lane;
            const bool valid = t < c1;
            const uint32_t d = (uint32_t)(key[j] >> shift) & mask;
            uint64_t peers = __ballot(valid);
            for (uint32_t b = 0; b < nbits; ++b) {
                const bool bit = (d >> b) & 1u;
                const uint64_t vote = __ballot(valid && bit);
                peers &= bit ? vote : ~vote;
            }
            const uint32_t before = __popcll(peers & lt);
            const uint32_t cnt = __popcll(peers);
            uint32_t b0 = 0;
            if (valid) b0 = wcnt[w][d];
            if (valid && before == 0) wcnt[w][d] = b0 + cnt;
            rank[j] = b0 + before;
        }
        __syncthreads();
        // per digit: tile count, exclusive prefix over digits, prefix over waves
        uint32_t c[kWaves];
        uint32_t tc = 0;
#pragma unroll
        for (int k = 0; k < kWaves; ++k) {
            c[k] = wcnt[k][tid];
            tc += c[k];
        }
        uint64_t tot;
        const uint32_t ex = (uint32_t)block_excl_scan<kNT>(tc, sh, &tot);
        tdp[tid] = ex;
        uint32_t run = 0;
#pragma unroll
        for (int k = 0; k < kWaves; ++k) {
            wcnt[k][tid] = run;
            run += c[k];
        }
        __syncthreads();
#pragma unroll
        for (int j = 0; j < kRounds; ++j) {
            const uint64_t t = wb + (uint64_t)j * kWave + lane;
            if (t < c1) {
                const uint32_t d = (uint32_t)(key[j] >> shift) & mask;
                stage[tdp[d] + wcnt[w][d] + rank[j]] = key[j];
            }
        }
        __syncthreads();
        const uint32_t cnt_tile = (uint32_t)min((uint64_t)kTile, c1 - t0);
        for (uint32_t i = tid; i < cnt_tile; i += kNT) {
            const uint64_t k = stage[i];
            const uint32_t d = (uint32_t)(k >> shift) & mask;
            out[base[d] + (i - tdp[d])] = k;
        }
        __syncthreads();
        base[tid] += tc;
        __syncthreads();
    }
}

}  // namespace

uint64_t radix_work_bytes(uint64_t N) {
    const uint64_t nchunks = div_up(N, kChunk);
    const uint64_t len = (uint64_t)kRadix * nchunks;
    return len * 4 + (len + 1) * 8 + scan_tmp_elems(len) * 8;
}

uint64_t radix_prepare(RadixWork &w, uint64_t N, hipStream_t s, Budget *b) {
    const uint64_t nchunks = div_up(std::max<uint64_t>(N, 1), kChunk);
    if (nchunks > 0xFFFFFFFFull) fail(JAS_EUNSUPPORTED, "radix sort: too many keys");
    const uint64_t len = (uint64_t)kRadix * nchunks;
    if (w.counts.n < len) w.counts.alloc(len, s, b, true, "radix counts");
    if (w.offs.n < len + 1) w.offs.alloc(len + 1, s, b, true, "radix offsets");
    const size_t tl = scan_tmp_elems(len);
    if (w.tmp.n < tl) w.tmp.alloc(tl, s, b, true, "radix scan scratch");
    return nchunks;
}

void radix_sort_u64(DevBuf<uint64_t> &keys, DevBuf<uint64_t> &alt, uint64_t N, uint32_t lo_bit, uint32_t hi_bit,
                    RadixWork &w, hipStream_t s, Budget *b, bool first_counts_ready) {
    if (N <= 1 || hi_bit <= lo_bit) return;
    const uint64_t nchunks = radix_prepare(w, N, s, b);
    const uint64_t len = (uint64_t)kRadix * nchunks;
    for (uint32_t bit = lo_bit; bit < hi_bit; bit += 8) {
        const uint32_t nbits = min(8u, hi_bit - bit);
        const uint32_t mask = (1u << nbits) - 1u;
        if (!(first_counts_ready && bit == lo_bit)) {
            JAS_TIMED("radix_hist", s);
            k_radix_hist<<<(uint32_t)nchunks, kNT, 0, s>>>(keys.p, N, bit, mask, w.counts.p, (uint32_t)nchunks);
        }
        check_launch("radix histogram");
        scan_excl_u32(w.counts.p, w.offs.p, len, w.tmp.p, s);
        {
            JAS_TIMED("radix_scatter", s);
            k_radix_scatter<<<(uint32_t)nchunks, kNT, 0, s>>>(keys.p, alt.p, N, bit, nbits, w.offs.p,
                                                             (uint32_t)nchunks);
        }
        check_launch("radix scatter");
        std::swap(keys.p, alt.p);
        std::swap(keys.n, alt.n);
    }
}

}  // namespace jas
