// Stable LSD radix sorts of keys on a bit range.
//
// Used to group equal IDs (the zero-row filter f of Eq. (5) and the
// compaction of Eq. (6) need every nonzero row's entries together).
// radix_sort_u64 (the path for inputs the single-pass scatter below cannot
// take): each pass is reduce-then-scan with no inter-block waiting:
//   1. k_radix_hist:    per-chunk digit histograms (digit-major counts[d][chunk]);
//   2. exclusive scan:  global start of every (digit, chunk) bucket;
//   3. k_radix_scatter: per 4096-key tile, a wave64 ballot multisplit ranks
//      keys by digit (stable: waves own consecutive quarters of the tile,
//      rounds go in order), the tile is reordered in LDS, and each digit run
//      is written out contiguously (coalesced).
#include <algorithm>

#include "device_util.hpp"
#include "jas_internal.hpp"
#include "onesweep_index.hpp"

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

// ---------------------------------------------------------------------------
// Single-pass scatter with decoupled look-back (chained scan: Merrill &
// Garland, "Single-pass parallel prefix scan with decoupled look-back",
// 2016; as in Adinets & Merrill's Onesweep, 2022).  Persistent blocks take
// 8192-key tiles by ticket from an atomic counter in launch order, so every
// tile a block waits for already belongs to a running block.  Per tile and
// digit a 32-bit status word holds a flag (aggregate / inclusive prefix) and
// a 30-bit count; the caller guarantees every digit total is < 2^30.  The
// same kernel sorts 64-bit keys (the encoder and the query path) and 32-bit
// row-list pair words.
// A load the compiler may issue through the scalar cache: the data stays
// unchanged while the kernel runs (written by an earlier launch) and the
// address is the same across the wave.
template <class T>
__device__ __forceinline__ T const_load(const T *p) {
    return *(const __attribute__((address_space(4))) T *)(p);
}

using onesweep::kFlagA;
using onesweep::kFlagP;
using onesweep::kValMask;
using onesweep::kLookWindow;  // 4 measured best of 4, 8, 16
constexpr uint32_t kMaxSpin = 1u << 20;  // bounded wait (~0.1 s of polls), then give up and flag

__device__ __forceinline__ void status_store(uint32_t *p, uint32_t v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint32_t status_load(const uint32_t *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// One tile = kOsNT threads x R keys; threads tid < kRadix also own digit tid.
constexpr int kOsNT = 512;  // 512 x 16 keys measured best of 512 x 8/12/16 and 1024 x 16 (one block per CU)
constexpr int kOsWaves = kOsNT / kWave;

// With kFromIds the pass reads CSR IDs and forms each key id << src.sbits |
// sample itself.  Its digit is ID bits only (shift >= src.sbits), so the IDs
// are ranked as loaded (each rank starts as soon as its load arrives) and the
// sample joins a key when it is placed in LDS: src.tinfo holds the samples of
// the tile's first and last entries (k_tile_samples), and an entry's sample is
// the first one plus the sample starts inside the tile at or before it (a
// uniform loop of scalar loads, run only by tiles that span several samples).
template <class K, int R, bool kTable, bool kFromIds = false>
__global__ __launch_bounds__(kOsNT) __attribute__((amdgpu_waves_per_eu(4))) void k_radix_onesweep(
    const K *__restrict__ in, K *__restrict__ out, uint64_t N, uint32_t shift, uint32_t nbits,
    const uint64_t *__restrict__ gstart, uint32_t *__restrict__ status, uint32_t *__restrict__ ticket,
    uint32_t ntiles, uint32_t *__restrict__ err, const uint64_t *__restrict__ dN, KeySource src) {
    __shared__ K stage[kOsNT * R];
    __shared__ uint32_t wcnt[kOsWaves][kRadix];
    __shared__ uint32_t tdp[kRadix];
    __shared__ uint64_t base[kRadix];
    __shared__ uint64_t sh[kOsWaves];
    __shared__ uint32_t tile_sh;
    const uint32_t tid = threadIdx.x, lane = lane_id(), w = tid / kWave;
    if (dN) {  // key count from device memory (planned encode): at most the buffers' N
        N = min(N, *dN);
        ntiles = (uint32_t)onesweep::num_tiles(N, kOsNT * R);
    }
    const bool digit = tid < kRadix;  // this thread owns digit tid
    const uint32_t mask = (1u << nbits) - 1u;
    const uint32_t dshift = kFromIds ? shift - src.sbits : shift;  // digit position in a loaded value
    const uint64_t lt = lanemask_lt();
    const uint64_t gs = digit ? gstart[tid] : 0;
    // while ranking, the first kOsWaves*256 words of stage are per-wave tables
    // of the lanes of the current round that have digit d
    static_assert(!kTable || kOsWaves * kRadix * sizeof(uint64_t) <= (kOsNT * R) * sizeof(K),
                  "match tables fit the stage");
    uint64_t *T = reinterpret_cast<uint64_t *>(stage) + w * kRadix;
    // persistent: take tiles in ticket order until none is left
    for (;;) {
        if (tid == 0) tile_sh = atomicAdd(ticket, 1u);
        for (uint32_t i = tid; i < kOsWaves * kRadix; i += kOsNT) {
            (&wcnt[0][0])[i] = 0;
            if constexpr (kTable) reinterpret_cast<uint64_t *>(stage)[i] = 0;
        }
        __syncthreads();
        const uint32_t tile = __builtin_amdgcn_readfirstlane(tile_sh);  // uniform: every thread reads the same ticket
        if (tile >= ntiles) break;  // uniform: every thread read the same ticket
        const uint64_t t0 = onesweep::tile_first(tile, kOsNT * R);
        const uint64_t c1 = onesweep::tile_end(tile, kOsNT * R, N);
        const uint64_t wb = t0 + (uint64_t)w * ((kOsNT * R) / kOsWaves);
        K key[R];
        uint32_t rank[R];
        static_assert(!kFromIds || sizeof(K) == 8, "keys formed from IDs are 64-bit");
        uint64_t tsmp = 0;  // samples of the tile's first and last entries (low, high half), loaded ahead
        if constexpr (kFromIds) tsmp = const_load(reinterpret_cast<const uint64_t *>(src.tinfo) + tile);
#pragma unroll
        for (int j = 0; j < R; ++j) {
            const uint64_t t = wb + (uint64_t)j * kWave + lane;
            key[j] = t < c1 ? in[t] : 0;
        }
        if constexpr (kTable) {
            // Rank within the wave: lanes of a round with the same digit find each
            // other through T[d] (each ORs in its lane bit, reads the set back and
            // clears it; one wave's LDS operations run in order), take consecutive
            // slots after the digit's count so far, and the lowest of them adds the
            // group to the count with an LDS atomic whose return its peers fetch
            // afterwards (in two halves, which keeps fewer registers live).
    #pragma unroll
            for (int h = 0; h < 2; ++h) {
                uint32_t info[R / 2];
    #pragma unroll
                for (int j = h * (R / 2); j < (h + 1) * (R / 2); ++j) {
                    const uint64_t t = wb + (uint64_t)j * kWave + lane;
                    const bool valid = t < c1;
                    const uint32_t d = (uint32_t)(key[j] >> dshift) & mask;
                    uint64_t peers = 0;
                    if (valid) {
                        atomicOr((unsigned long long *)&T[d], 1ull << lane);
                        peers = __hip_atomic_load(&T[d], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
                        __hip_atomic_store(&T[d], 0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
                    }
                    const uint32_t before = __popcll(peers & lt);
                    const uint32_t leader = peers ? (uint32_t)__builtin_ctzll(peers) : lane;
                    uint32_t old = 0;
                    if (valid && before == 0) old = atomicAdd(&wcnt[w][d], (uint32_t)__popcll(peers));
                    rank[j] = old;
                    info[j - h * (R / 2)] = (leader << 8) | before;
                }
    #pragma unroll
                for (int j = h * (R / 2); j < (h + 1) * (R / 2); ++j) {
                    const uint32_t f = info[j - h * (R / 2)];
                    rank[j] = (uint32_t)__shfl((int)rank[j], (int)(f >> 8), kWave) + (f & 255u);
                }
            }
        } else {
            // 64-bit keys: rank by one ballot per digit bit (fewer registers
            // than the table form, which spills with 64-bit keys)
    #pragma unroll
            for (int j = 0; j < R; ++j) {
                const uint64_t t = wb + (uint64_t)j * kWave + lane;
                const bool valid = t < c1;
                const uint32_t d = (uint32_t)(key[j] >> dshift) & mask;
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
        }
        __syncthreads();
        uint32_t tc = 0;
        if (digit) {
#pragma unroll
            for (int k = 0; k < kOsWaves; ++k) tc += wcnt[k][tid];
            // publish the tile's count of digit tid at once
            status_store(status + onesweep::status_index(tile, tid), (tile == 0 ? kFlagP : kFlagA) | tc);
        }
        // reorder the tile in LDS by digit (local offsets only)
        uint64_t tot;
        const uint32_t ex = (uint32_t)block_excl_scan<kOsNT>(tc, sh, &tot);
        if (digit) {  // wcnt[w][d] becomes where wave w's keys of digit d start in the tile
            tdp[tid] = ex;
            uint32_t run = ex;
#pragma unroll
            for (int k = 0; k < kOsWaves; ++k) {
                const uint32_t v = wcnt[k][tid];
                wcnt[k][tid] = run;
                run += v;
            }
        }
        __syncthreads();
        if constexpr (kFromIds) {
            // the sample starts inside the tile lie in (t0, c1), so tile-relative
            // positions compare in 32 bits
            const uint32_t s0 = (uint32_t)tsmp, s1 = (uint32_t)(tsmp >> 32);
            const uint32_t cnt = (uint32_t)(c1 - t0), wl = (uint32_t)(wb - t0) + lane;
#pragma unroll
            for (int j = 0; j < R; ++j) {
                const uint32_t li = wl + j * kWave;  // position in the tile
                if (li < cnt) {
                    const uint32_t d = (uint32_t)(key[j] >> dshift) & mask;
                    uint32_t smp = s0;
                    for (uint32_t k = s0 + 1; k <= s1; ++k) smp += li >= (uint32_t)(const_load(src.off + k) - t0);
                    stage[wcnt[w][d] + rank[j]] = (key[j] << src.sbits) | smp;
                }
            }
        } else {
#pragma unroll
            for (int j = 0; j < R; ++j) {
                const uint64_t t = wb + (uint64_t)j * kWave + lane;
                if (t < c1) {
                    const uint32_t d = (uint32_t)(key[j] >> shift) & mask;
                    stage[wcnt[w][d] + rank[j]] = key[j];
                }
            }
        }
        // then look back for the digit's global offset: kLookWindow
        // predecessor tiles per step, loaded together (one memory round trip)
        // and taken nearest first
        if (digit) {
            uint32_t excl = 0;
            if (tile > 0) {
                bool found = false;
                for (int64_t j0 = (int64_t)tile - 1; j0 >= 0 && !found; j0 -= kLookWindow) {
                    uint32_t v[kLookWindow];
#pragma unroll
                    for (int k = 0; k < kLookWindow; ++k)
                        v[k] = j0 - k >= 0 ? status_load(status + onesweep::status_index(j0 - k, tid)) : kFlagP;
#pragma unroll
                    for (int k = 0; k < kLookWindow; ++k) {
                        if (found) break;
                        uint32_t spins = 0;
                        while ((v[k] & ~kValMask) == 0) {
                            // give up after kMaxSpin polls, or at once when any tile has given up
                            if (++spins > kMaxSpin || (status_load(err) & 2u)) {
                                atomicOr(err, 2u);
                                v[k] = kFlagP;
                                break;
                            }
                            __builtin_amdgcn_s_sleep(1);
                            v[k] = status_load(status + onesweep::status_index(j0 - k, tid));
                        }
                        excl += v[k] & kValMask;
                        found = (v[k] & ~kValMask) == kFlagP;
                    }
                }
                status_store(status + onesweep::status_index(tile, tid), kFlagP | ((excl + tc) & kValMask));
            }
            base[tid] = gs + excl;
        }
        __syncthreads();
        const uint32_t cnt_tile = (uint32_t)(c1 - t0);
        for (uint32_t i = tid; i < cnt_tile; i += kOsNT) {
            const K k = stage[i];
            const uint32_t d = (uint32_t)(k >> shift) & mask;
            out[onesweep::out_index(base[d], i, tdp[d])] = k;
        }
        __syncthreads();  // stage, tdp, base and tile_sh are reused by the next tile
    }
}

// gstart[q][d] = exclusive scan over digits of the summed replicas; maxima[q] = largest digit total.
__global__ __launch_bounds__(kNT) void k_digit_starts(const unsigned long long *__restrict__ ghist, uint32_t npass,
                                                       uint64_t *__restrict__ gstart, uint64_t *__restrict__ maxima,
                                                       uint32_t *__restrict__ err) {
    __shared__ uint64_t sh[kWaves];
    __shared__ uint64_t tot_sh[kRadix];
    const uint32_t tid = threadIdx.x;
    for (uint32_t q = 0; q < npass; ++q) {
        uint64_t t = 0;
        for (uint32_t r = 0; r < kGhistReplicas; ++r) t += ghist[((uint64_t)r * kMaxPasses + q) * kRadix + tid];
        uint64_t all;
        gstart[q * kRadix + tid] = block_excl_scan<kNT>(t, sh, &all);
        tot_sh[tid] = t;
        __syncthreads();
        if (tid == 0) {
            uint64_t m = 0;
            for (int d = 0; d < kRadix; ++d) m = m > tot_sh[d] ? m : tot_sh[d];
            maxima[q] = m;
            if (err && m >= kValMask) atomicOr(err, 4u);  // planned sort: cannot run single-pass
        }
        __syncthreads();
    }
}

__global__ void k_fill32(uint32_t *p, uint64_t len) {
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < len; i += (uint64_t)gridDim.x * blockDim.x)
        p[i] = 0;
}

// Per tile of tile_keys entries: tinfo[2 t] and tinfo[2 t + 1] = the samples
// holding the tile's first and last entries.
__global__ void k_tile_samples(const uint64_t *__restrict__ off, int32_t n, uint64_t N, uint32_t tile_keys,
                               uint32_t *__restrict__ tinfo, const uint64_t *__restrict__ dN) {
    if (dN) N = min(N, *dN);
    const uint64_t ntiles = onesweep::num_tiles(N, tile_keys);
    for (uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; t < ntiles;
         t += (uint64_t)gridDim.x * blockDim.x) {
        const int32_t s0 = find_sample(off, 0, n - 1, onesweep::tile_first(t, tile_keys));
        tinfo[2 * t] = (uint32_t)s0;
        tinfo[2 * t + 1] = (uint32_t)find_sample(off, s0, n - 1, onesweep::tile_end(t, tile_keys, N) - 1);
    }
}

}  // namespace

SortPlan sort_plan(uint64_t N, uint32_t U, uint32_t sbits) {
    SortPlan p;
    if (N <= kLocalCapKeys) return p;  // one LDS range holds everything
    p.top_bits = std::min<uint32_t>(U, ceil_log2_u64(div_up(N, kBucketKeys)));
    const uint32_t fewer = std::min<uint32_t>(U, ceil_log2_u64(div_up(N, 2 * kBucketKeys)));
    if (fewer > 0 && (U - fewer) + kSpanBits + sbits <= 32) p.top_bits = fewer;
    p.npass = (p.top_bits + 7) / 8;
    p.width = p.npass ? (p.top_bits + p.npass - 1) / p.npass : 8;
    return p;
}

uint64_t radix_work_bytes(uint64_t N) {
    const uint64_t nchunks = div_up(N, kChunk);
    const uint64_t len = (uint64_t)kRadix * nchunks;
    return len * 4 + (len + 1) * 8 + scan_tmp_elems(len) * 8;
}

uint64_t radix_prepare(RadixWork &w, uint64_t N, hipStream_t s, Budget *b, Arena *ar) {
    const uint64_t nchunks = div_up(std::max<uint64_t>(N, 1), kChunk);
    if (nchunks > 0xFFFFFFFFull) fail(JAS_EUNSUPPORTED, "radix sort: too many keys");
    const uint64_t len = (uint64_t)kRadix * nchunks;
    if (w.counts.n < len) temp_buf(w.counts, len, s, b, ar, "radix counts");
    if (w.offs.n < len + 1) temp_buf(w.offs, len + 1, s, b, ar, "radix offsets");
    const size_t tl = scan_tmp_elems(len);
    if (w.tmp.n < tl) temp_buf(w.tmp, tl, s, b, ar, "radix scan scratch");
    return nchunks;
}

void radix_sort_u64(DevBuf<uint64_t> &keys, DevBuf<uint64_t> &alt, uint64_t N, uint32_t lo_bit, uint32_t hi_bit,
                    RadixWork &w, hipStream_t s, Budget *b, Arena *ar) {
    if (N <= 1 || hi_bit <= lo_bit) return;
    const uint64_t nchunks = radix_prepare(w, N, s, b, ar);
    const uint64_t len = (uint64_t)kRadix * nchunks;
    for (uint32_t bit = lo_bit; bit < hi_bit; bit += 8) {
        const uint32_t nbits = min(8u, hi_bit - bit);
        const uint32_t mask = (1u << nbits) - 1u;
        {
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
        swap_bufs(keys, alt);
    }
}

}  // namespace jas

namespace jas {

namespace {
// Fills src.tinfo for tiles of tile_keys entries (after checking its size).
void tile_samples(const KeySource &src, uint64_t Ncap, uint32_t tile_keys, const uint64_t *dN, hipStream_t s) {
    const uint64_t ntiles = onesweep::num_tiles(Ncap, tile_keys);
    if (!src.ids || !src.off || !src.tinfo || src.n < 1 || src.tinfo_words < 2 * ntiles)
        fail(JAS_EDEVICE, "sort from IDs: tile sample buffer does not cover the tiles");
    {
        JAS_TIMED("tile_samples", s);
        k_tile_samples<<<(uint32_t)std::max<uint64_t>(1, std::min<uint64_t>(div_up(ntiles, 256), 4096)), 256, 0, s>>>(
            src.off, src.n, Ncap, tile_keys, src.tinfo, dN);
    }
    check_launch("tile samples");
}

// Launches one pass; the first reads src.ids when the keys are formed from IDs.
template <class K, int Rounds, bool Table>
void onesweep_pass(bool from_ids, const K *in, K *out, uint64_t N, uint32_t bit, uint32_t nbits,
                   const uint64_t *gstart, uint32_t *status, uint32_t *ticket, uint32_t ntiles, uint32_t *err,
                   const uint64_t *dN, const KeySource *src, uint32_t grid, hipStream_t s) {
    if (from_ids && bit < src->sbits) fail(JAS_EDEVICE, "sort from IDs: a digit below the ID bits");
    if constexpr (sizeof(K) == 8) {
        if (from_ids) {
            k_radix_onesweep<K, Rounds, Table, true><<<grid, kOsNT, 0, s>>>(
                reinterpret_cast<const K *>(src->ids), out, N, bit, nbits, gstart, status, ticket, ntiles, err, dN,
                *src);
            return;
        }
    }
    if (from_ids) fail(JAS_EDEVICE, "sort from IDs: 64-bit keys only");
    k_radix_onesweep<K, Rounds, Table><<<grid, kOsNT, 0, s>>>(in, out, N, bit, nbits, gstart, status, ticket, ntiles,
                                                             err, dN, KeySource{});
}

// With src the keys are formed from CSR sets by the first pass (keys.p is
// not read); otherwise keys holds them.
template <class K, int Rounds, bool Table>
bool onesweep_sort(DevBuf<K> &keys, DevBuf<K> &alt, uint64_t N, uint32_t lo_bit, uint32_t hi_bit, uint32_t width,
                   const unsigned long long *ghist, uint32_t *err, hipStream_t s, Budget *b, Arena *ar,
                   const char *name, const KeySource *src = nullptr) {
    if (N <= 1 || hi_bit <= lo_bit) return true;
    if (width < 1 || width > 8) return false;
    const uint32_t npass = (hi_bit - lo_bit + width - 1) / width;
    if (npass > kMaxPasses) return false;
    DevBuf<uint64_t> gstart, maxima;
    temp_buf(gstart, (uint64_t)kMaxPasses * kRadix, s, b, ar, "digit starts");
    temp_buf(maxima, kMaxPasses, s, b, ar, "digit maxima");
    {
        JAS_TIMED("digit_starts", s);
        k_digit_starts<<<1, kNT, 0, s>>>(ghist, npass, gstart.p, maxima.p, nullptr);
    }
    check_launch("digit starts");
    uint64_t hm[kMaxPasses];
    JAS_HIP(hipMemcpyAsync(hm, maxima.p, sizeof(uint64_t) * npass, hipMemcpyDeviceToHost, s));
    JAS_HIP(hipStreamSynchronize(s));
    for (uint32_t q = 0; q < npass; ++q)
        if (hm[q] >= std::min<uint64_t>(kValMask, scatter_count_limit())) return false;
    const uint64_t ntiles = onesweep::num_tiles(N, (uint32_t)kOsNT * Rounds);
    if (ntiles > 0xFFFFFFFFull) return false;
    // persistent blocks: two per CU (256 CUs) fit, never more than there are tiles
    const uint32_t grid = (uint32_t)std::min<uint64_t>(ntiles, 256 * 2);
    DevBuf<uint32_t> status, ticket;
    temp_buf(status, onesweep::status_words(ntiles), s, b, ar, "look-back status");
    temp_buf(ticket, 1, s, b, ar, "tile ticket");
    // What the kernel's indexing relies on (see onesweep_index.hpp): the key
    // buffers hold N keys, the tiles cover exactly [0, N), the status array
    // has a word for every (tile, digit), every pass has a row of digit
    // starts, and no 30-bit status count can wrap.
    if (keys.n < N || alt.n < N || ntiles * (uint64_t)kOsNT * Rounds < N ||
        onesweep::tile_first(ntiles - 1, kOsNT * Rounds) >= N ||
        status.n < onesweep::status_words(ntiles) || gstart.n < (uint64_t)npass * kRadix || grid > ntiles ||
        N > 0xFFFFFFFFull * (uint64_t)kOsNT * Rounds)
        fail(JAS_EDEVICE, "single-pass scatter: buffer sizes do not cover its indexing");
    for (uint32_t q = 0; q < npass; ++q)
        if (hm[q] > kValMask) fail(JAS_EDEVICE, "single-pass scatter: a digit total exceeds the status count");
    KeySource ks;
    DevBuf<uint32_t> tinfo;
    if (src) {
        ks = *src;
        temp_buf(tinfo, 2 * ntiles, s, b, ar, "tile samples");
        ks.tinfo = tinfo.p;
        ks.tinfo_words = tinfo.n;
        tile_samples(ks, N, (uint32_t)kOsNT * Rounds, nullptr, s);
        src = &ks;
    }
    for (uint32_t q = 0; q < npass; ++q) {
        const uint32_t bit = lo_bit + width * q;
        const uint32_t nbits = min(width, hi_bit - bit);
        {
            JAS_TIMED("fill_status", s);
            k_fill32<<<(uint32_t)std::min<uint64_t>(div_up(ntiles * kRadix + 1, 256), 65536), 256, 0, s>>>(
                status.p, ntiles * kRadix + 1);
            k_fill32<<<1, 64, 0, s>>>(ticket.p, 1);
        }
        check_launch("look-back reset");
        {
            JAS_TIMED(name, s);
            onesweep_pass<K, Rounds, Table>(src && q == 0, keys.p, alt.p, N, bit, nbits, gstart.p + q * kRadix,
                                            status.p, ticket.p, (uint32_t)ntiles, err, nullptr, src, grid, s);
        }
        check_launch("radix scatter (look-back)");
        swap_bufs(keys, alt);
    }
    return true;
}
// The same passes for a planned encode: the key count is read from *dN
// (at most Ncap, the buffers' size) inside the kernels, every buffer is
// given, nothing is read back and nothing allocated.  A digit total too large
// for the 30-bit status counts sets bit 2 of err[0] (the result is then
// invalid; the caller reports it after the stream completes).
template <class K, int Rounds, bool Table>
void onesweep_sort_planned(K *&keys, K *&alt, const uint64_t *dN, uint64_t Ncap, uint32_t lo_bit, uint32_t hi_bit,
                           uint32_t width, const unsigned long long *ghist, uint32_t *err, const OnesweepBufs &b,
                           hipStream_t s, const char *name, const KeySource *src = nullptr) {
    if (Ncap <= 1 || hi_bit <= lo_bit) return;
    const uint32_t npass = (hi_bit - lo_bit + width - 1) / width;
    if (npass > kMaxPasses || width < 1 || width > 8) fail(JAS_EUNSUPPORTED, "planned sort: bad digit plan");
    const uint64_t ntiles = onesweep::num_tiles(Ncap, (uint32_t)kOsNT * Rounds);
    if (b.status_words < onesweep::status_words(ntiles) || ntiles > 0xFFFFFFFFull)
        fail(JAS_EDEVICE, "planned sort: status buffer too small");
    {
        JAS_TIMED("digit_starts", s);
        k_digit_starts<<<1, kNT, 0, s>>>(ghist, npass, b.gstart, b.maxima, err);
    }
    check_launch("digit starts");
    if (src) tile_samples(*src, Ncap, (uint32_t)kOsNT * Rounds, dN, s);
    const uint32_t grid = (uint32_t)std::min<uint64_t>(ntiles, 256 * 2);
    for (uint32_t q = 0; q < npass; ++q) {
        const uint32_t bit = lo_bit + width * q;
        const uint32_t nbits = min(width, hi_bit - bit);
        {
            JAS_TIMED("fill_status", s);
            k_fill32<<<(uint32_t)std::min<uint64_t>(div_up(onesweep::status_words(ntiles), 256), 65536), 256, 0, s>>>(
                b.status, onesweep::status_words(ntiles));
            k_fill32<<<1, 64, 0, s>>>(b.ticket, 1);
        }
        check_launch("look-back reset");
        {
            JAS_TIMED(name, s);
            onesweep_pass<K, Rounds, Table>(src && q == 0, keys, alt, Ncap, bit, nbits, b.gstart + q * kRadix,
                                            b.status, b.ticket, (uint32_t)ntiles, err, dN, src, grid, s);
        }
        check_launch("radix scatter (planned)");
        std::swap(keys, alt);
    }
}

}  // namespace

uint64_t onesweep_status_words(uint64_t N, bool u32) {
    (void)u32;  // both key widths take 16 keys per lane
    return onesweep::status_words(onesweep::num_tiles(N, (uint32_t)kOsNT * 16));
}

void radix_sort_onesweep_planned(uint64_t *&keys, uint64_t *&alt, const uint64_t *dN, uint64_t Ncap,
                                 uint32_t lo_bit, uint32_t hi_bit, uint32_t width, const unsigned long long *ghist,
                                 uint32_t *err, const OnesweepBufs &b, hipStream_t s, const KeySource *src) {
    onesweep_sort_planned<uint64_t, 16, false>(keys, alt, dN, Ncap, lo_bit, hi_bit, width, ghist, err, b, s,
                                               "radix_onesweep", src);
}

void radix_sort_onesweep_u32_planned(uint32_t *&keys, uint32_t *&alt, const uint64_t *dN, uint64_t Ncap,
                                     uint32_t lo_bit, uint32_t hi_bit, uint32_t width,
                                     const unsigned long long *ghist, uint32_t *err, const OnesweepBufs &b,
                                     hipStream_t s) {
    onesweep_sort_planned<uint32_t, 16, true>(keys, alt, dN, Ncap, lo_bit, hi_bit, width, ghist, err, b, s,
                                              "pair_sort");
}

// 64-bit keys: 16 keys per lane, ballot ranking (the table form is no faster
// for them and needs more registers); 32-bit pair words: table ranking.
constexpr int kU64Rounds = 16;
constexpr bool kU64Table = false;

uint64_t onesweep_tile_keys_u64() { return (uint64_t)kOsNT * kU64Rounds; }

bool radix_sort_onesweep(DevBuf<uint64_t> &keys, DevBuf<uint64_t> &alt, uint64_t N, uint32_t lo_bit,
                         uint32_t hi_bit, uint32_t width, const unsigned long long *ghist, uint32_t *err,
                         hipStream_t s, Budget *b, Arena *ar, const KeySource *src) {
    return onesweep_sort<uint64_t, kU64Rounds, kU64Table>(keys, alt, N, lo_bit, hi_bit, width, ghist, err, s, b, ar,
                                                          "radix_onesweep", src);
}

bool radix_sort_onesweep_u32(DevBuf<uint32_t> &keys, DevBuf<uint32_t> &alt, uint64_t N, uint32_t lo_bit,
                             uint32_t hi_bit, uint32_t width, const unsigned long long *ghist, uint32_t *err,
                             hipStream_t s, Budget *b, Arena *ar) {
    return onesweep_sort<uint32_t, 16, true>(keys, alt, N, lo_bit, hi_bit, width, ghist, err, s, b, ar, "pair_sort");
}

}  // namespace jas
