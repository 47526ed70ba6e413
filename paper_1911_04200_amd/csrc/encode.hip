// Encoding of the indicator matrix A (Sec. III-B).
//
// Input: CSR sets.  Keys (id << sbits) | sample are built in CSR order, which
// is already ascending in `sample`, so a stable sort on the ID bits alone
// leaves every ID's entries together with samples ascending.  The global sort
// (radix.hip) orders the keys by their top ID bits only; each range of whole
// buckets is finished here, in LDS (k_local_cls).
//
// After the sort (encode_sorted):
//   classify   first occurrence of a key = a distinct (ID, sample) pair, i.e. a
//              nonzero of A (repeats dropped: the (max, x) write of Sec. IV-A);
//              |X_i| = entries of sample i minus its repeats (column sums,
//              Eq. (4)); an ID's run of distinct pairs is one nonzero row of A
//              (the filter of Eq. (5)); rows with >= 2 pairs ("shared") are the
//              only rows off-diagonal B depends on, because a row with one
//              nonzero adds only to B_ii = |X_i|.
//   compaction shared rows are numbered in ID order by a prefix sum (Eq. (6)).
//   split      rows of degree >= dmin are bit-packed; rows of degree 2..dmin-1
//              are kept as row lists: their pairs, sorted by the smaller
//              sample, are counted per sample in the Gram step.
//   batches    packed rows are grouped by batch l = id >> batch_bits (Eq. (3));
//              inside a batch, row p (in ID order) is bit p % 64 of word row
//              p / 64, so words never straddle batches.
//   pack       one block per word row ORs the bits of its <= 64 rows into an
//              LDS row of n words and writes it out: W[w][i] is the word of
//              column i (the bitmask compression preceding Eq. (7)).
#include <algorithm>
#include <utility>

#include "device_util.hpp"
#include "jas_internal.hpp"

namespace jas {
namespace {

constexpr int kNT = 256;
constexpr int kWaves = kNT / kWave;
constexpr int kRounds = 16;
constexpr uint32_t kTile = kNT * kRounds;  // 4096
constexpr uint64_t kChunk = 65536;         // elements per classify block
constexpr int32_t kHistMax = 16384;        // LDS column histogram up to this n
constexpr uint32_t kPackCols = 8192;       // LDS words per pack pass, at most
constexpr uint32_t kPackLoads = 8;         // sample loads in flight per lane in k_pack
constexpr uint32_t kPackFlat = 4096;       // k_pack: word rows with at most this many entries spread them over the block

enum { ST_PAIRS = 0, ST_ROWS, ST_NNZW, ST_F, ST_LISTPAIRS, ST_N };
static_assert(ST_N == ST_N_ && ST_ROWS == ST_ROWS_ && ST_NNZW == ST_NNZW_ && ST_F == ST_F_ &&
                  ST_LISTPAIRS == ST_LISTPAIRS_,
              "encode counters");
// Counters that many blocks add to are spread over kStatReplicas slots (one
// counter would serialise an atomic from every block) and summed into st by
// k_sum_replicas.
constexpr uint32_t kStatReplicas = 64;
static_assert(kStatReplicas == kStatReplicasPub, "counter replicas");

// ---------------------------------------------------------------------------
// Keys of one chunk (kChunk entries) per block, and the totals of every digit
// of every global sort pass (ghist, kGhistReplicas copies summed later), which
// the single-pass scatter needs.  Pass q's digit is ID bits
// [idlo + width*q, idlo + width*(q+1)).  k_count_digits only counts (and
// checks the IDs): the sort's first pass then forms the keys itself.
template <bool kWrite>
__device__ __forceinline__ void build_keys_chunk(const uint64_t *__restrict__ ids, const uint64_t *__restrict__ off,
                                                 int32_t n, uint64_t N, uint32_t sbits, uint64_t hi_mask,
                                                 uint64_t *__restrict__ keys, uint32_t *err, uint32_t npass,
                                                 uint32_t idlo, uint32_t width,
                                                 unsigned long long *__restrict__ ghist,
                                                 const uint64_t *__restrict__ dsz) {
    __shared__ int32_t s_lo, s_hi;
    __shared__ uint32_t gh[kMaxPasses][256];
    const uint32_t tid = threadIdx.x;
    if (plan_aborted(dsz)) return;
    if (dsz) N = dsz[PZ_N];
    const uint64_t b0 = (uint64_t)blockIdx.x * kChunk;
    if (b0 >= N) return;  // a planned launch covers the largest N
    const uint64_t b1 = min(N, b0 + kChunk);
    const uint32_t dmask = (1u << width) - 1u;
#pragma unroll
    for (int k = 0; k < kMaxPasses; ++k) gh[k][tid] = 0;
    if (kWrite && tid == 0) {
        s_lo = find_sample(off, 0, n - 1, b0);
        s_hi = find_sample(off, s_lo, n - 1, b1 - 1);
    }
    __syncthreads();
    // A wave whose entries share a digit above the lowest (sets of ascending,
    // dense IDs) adds them with one atomic instead of 64 on one LDS word.  Each
    // wave decides once, from the top digit of its first 64 entries, whether
    // to look for such runs (IDs in no particular order never share it).
    bool agg = false;
    if (npass > 1) {
        const uint64_t t = b0 + tid;
        const uint32_t d = t < b1 ? (uint32_t)(ids[t] >> (idlo + width * (npass - 1))) & dmask : 0u;
        agg = __ballot(t < b1 && d == (uint32_t)__builtin_amdgcn_readfirstlane(d)) == __ballot(t < b1);
    }
    uint32_t bad = 0;
    int32_t lo = kWrite ? s_lo : 0;
    for (uint64_t t = b0 + tid; t < b1; t += kNT) {
        const uint64_t id = ids[t];
        bad |= (id & hi_mask) != 0;
        if constexpr (kWrite) {
            lo = find_sample(off, lo, s_hi, t);  // t only grows, so the search range only shrinks
            keys[t] = (id << sbits) | (uint64_t)lo;
        }
        if (agg) {  // wave-uniform
            const uint64_t active = __ballot(true);
            for (uint32_t q = 0; q < npass; ++q) {
                const uint32_t d = (uint32_t)(id >> (idlo + width * q)) & dmask;
                if (q > 0 && __ballot(d == (uint32_t)__builtin_amdgcn_readfirstlane(d)) == active) {
                    if (lane_id() == (uint32_t)__builtin_ctzll(active))
                        atomicAdd(&gh[q][d], (uint32_t)__popcll(active));
                } else {
                    atomicAdd(&gh[q][d], 1u);
                }
            }
        } else {
            for (uint32_t q = 0; q < npass; ++q)
                atomicAdd(&gh[q][(uint32_t)(id >> (idlo + width * q)) & dmask], 1u);
        }
    }
    if (__ballot(bad) && lane_id() == 0) atomicOr(err, 1u);
    __syncthreads();
    unsigned long long *g = ghist + (uint64_t)(blockIdx.x % kGhistReplicas) * kMaxPasses * 256;
    for (uint32_t q = 0; q < npass; ++q)
        if (gh[q][tid]) atomicAdd(&g[q * 256 + tid], (unsigned long long)gh[q][tid]);
}

__global__ __launch_bounds__(kNT) void k_build_keys(const uint64_t *__restrict__ ids,
                                                     const uint64_t *__restrict__ off, int32_t n, uint64_t N,
                                                     uint32_t sbits, uint64_t hi_mask, uint64_t *__restrict__ keys,
                                                     uint32_t *err, uint32_t npass, uint32_t idlo, uint32_t width,
                                                     unsigned long long *__restrict__ ghist,
                                                     const uint64_t *__restrict__ dsz) {
    build_keys_chunk<true>(ids, off, n, N, sbits, hi_mask, keys, err, npass, idlo, width, ghist, dsz);
}

__global__ __launch_bounds__(kNT) void k_count_digits(const uint64_t *__restrict__ ids, uint64_t N, uint64_t hi_mask,
                                                       uint32_t *err, uint32_t npass, uint32_t idlo, uint32_t width,
                                                       unsigned long long *__restrict__ ghist,
                                                       const uint64_t *__restrict__ dsz) {
    build_keys_chunk<false>(ids, nullptr, 0, N, 0, hi_mask, nullptr, err, npass, idlo, width, ghist, dsz);
}

__global__ void k_fill_u64(uint64_t *p, uint64_t len, uint64_t v) {
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < len; i += (uint64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

// ---------------------------------------------------------------------------
// Classification of the sorted keys.  A block owns a chunk of kChunk keys and
// walks it in tiles of kTile; each tile is staged in LDS with one key of halo
// on each side, so the neighbours that decide an element come from LDS.
//   first    K[t] != K[t-1]: the first copy of a distinct (ID, sample) pair;
//   left     the previous distinct pair has the same ID (not the row's first);
//   right    the next distinct pair (after any copies of K[t]) has the same ID;
//   shared   first && (left || right): the row has >= 2 distinct pairs;
//   rowstart shared && !left;  newid = first && !left (one per nonzero row).
struct Cls {
    bool first, shared, rowstart, newid;
};

// L[0..cnt+1] = K[t0-1 .. t0+cnt] (out-of-range ends are complements of their
// neighbour so they compare unequal).  Element t0+i is L[i+1].
__device__ __forceinline__ void stage_tile(const uint64_t *__restrict__ K, uint64_t N, uint64_t t0, uint32_t cnt,
                                           uint64_t *L) {
    for (uint32_t i = threadIdx.x; i < cnt; i += kNT) L[i + 1] = K[t0 + i];
    if (threadIdx.x == 0) L[0] = t0 > 0 ? K[t0 - 1] : ~K[t0];
    if (threadIdx.x == 1) L[cnt + 1] = (t0 + cnt < N) ? K[t0 + cnt] : ~K[t0 + cnt - 1];
}

__device__ __forceinline__ Cls classify_lds(const uint64_t *__restrict__ K, uint64_t N, uint64_t t0, uint32_t cnt,
                                            const uint64_t *L, uint32_t i, uint32_t sbits) {
    Cls c;
    const uint64_t key = L[i + 1], prev = L[i];
    const uint64_t id = key >> sbits;
    const uint64_t t = t0 + i;
    c.first = (t == 0) || prev != key;
    const bool left = c.first && t > 0 && (prev >> sbits) == id;
    bool right = false;
    if (c.first) {
        // next distinct key: in the tile (or its halo), else (long runs of copies) in global memory
        uint32_t j = i + 2;
        while (j <= cnt + 1 && L[j] == key) ++j;
        uint64_t nxt;
        bool have = true;
        if (j <= cnt + 1) {
            nxt = L[j];
            have = t0 + (j - 1) < N;
        } else {
            uint64_t u = t0 + cnt + 1;
            while (u < N && K[u] == key) ++u;
            have = u < N;
            nxt = have ? K[u] : 0;
        }
        right = have && (nxt >> sbits) == id;
    }
    c.shared = c.first && (left || right);
    c.rowstart = c.shared && !left;
    c.newid = c.first && !left;
    return c;
}

__global__ __launch_bounds__(kNT) void k_cls_count(const uint64_t *__restrict__ K, uint64_t N, uint32_t sbits,
                                                    uint64_t smask, int32_t n, int lds_hist, uint32_t *cD,
                                                    uint32_t *cS, uint32_t *cR, unsigned long long *card,
                                                    unsigned long long *st) {
    extern __shared__ uint32_t hist[];
    __shared__ uint64_t L[kTile + 2];
    __shared__ uint64_t sh[kWaves];
    const uint32_t tid = threadIdx.x;
    if (lds_hist)
        for (int32_t i = tid; i < n; i += kNT) hist[i] = 0;
    const uint64_t c0 = (uint64_t)blockIdx.x * kChunk;
    const uint64_t c1 = min(N, c0 + kChunk);
    uint32_t nD = 0, nS = 0, nR = 0, nI = 0;
    for (uint64_t t0 = c0; t0 < c1; t0 += kTile) {
        const uint32_t cnt = (uint32_t)min((uint64_t)kTile, c1 - t0);
        __syncthreads();
        stage_tile(K, N, t0, cnt, L);
        __syncthreads();
        for (uint32_t i = tid; i < cnt; i += kNT) {
            const Cls c = classify_lds(K, N, t0, cnt, L, i, sbits);
            if (c.first) {
                ++nD;
                const uint32_t s = (uint32_t)(L[i + 1] & smask);
                if (s < (uint32_t)n) {
                    if (lds_hist) atomicAdd(&hist[s], 1u);
                    else atomicAdd(&card[s], 1ull);
                }
            }
            nS += c.shared;
            nR += c.rowstart;
            nI += c.newid;
        }
    }
    uint64_t tD, tS, tR, tI;
    block_excl_scan<kNT>(nD, sh, &tD);
    block_excl_scan<kNT>(nS, sh, &tS);
    block_excl_scan<kNT>(nR, sh, &tR);
    block_excl_scan<kNT>(nI, sh, &tI);
    if (tid == 0) {
        cD[blockIdx.x] = (uint32_t)tD;
        cS[blockIdx.x] = (uint32_t)tS;
        cR[blockIdx.x] = (uint32_t)tR;
        atomicAdd(&st[ST_PAIRS], (unsigned long long)tD);
        atomicAdd(&st[ST_ROWS], (unsigned long long)tI);
    }
    if (lds_hist)
        for (int32_t i = tid; i < n; i += kNT)
            if (hist[i]) atomicAdd(&card[i], (unsigned long long)hist[i]);
}

// Ordered compaction of the classified elements of one chunk: wave w of a
// tile owns its elements [w*1024, (w+1)*1024), 64 per round, in order.
__global__ __launch_bounds__(kNT) void k_cls_write(const uint64_t *__restrict__ K, uint64_t N, uint32_t sbits,
                                                    uint64_t smask, const uint64_t *oD, const uint64_t *oS,
                                                    const uint64_t *oR, uint64_t *Dout, uint32_t *Sout,
                                                    uint64_t *row_id, uint64_t *row_ptr) {
    __shared__ uint64_t L[kTile + 2];
    __shared__ uint32_t wc[3][kWaves];
    __shared__ uint64_t run[3];
    const uint32_t tid = threadIdx.x, lane = lane_id(), w = tid / kWave;
    const uint64_t lt = lanemask_lt();
    const uint64_t c0 = (uint64_t)blockIdx.x * kChunk;
    const uint64_t c1 = min(N, c0 + kChunk);
    if (tid == 0) {
        run[0] = oD[blockIdx.x];
        run[1] = oS[blockIdx.x];
        run[2] = oR[blockIdx.x];
    }
    for (uint64_t t0 = c0; t0 < c1; t0 += kTile) {
        const uint32_t cnt = (uint32_t)min((uint64_t)kTile, c1 - t0);
        __syncthreads();
        stage_tile(K, N, t0, cnt, L);
        __syncthreads();
        const uint32_t wb = w * (kTile / kWaves);
        uint32_t fD = 0, fS = 0, fR = 0;
        uint32_t nD = 0, nS = 0, nR = 0;
#pragma unroll 2
        for (int j = 0; j < kRounds; ++j) {
            const uint32_t i = wb + j * kWave + lane;
            bool d = false, s = false, r = false;
            if (i < cnt) {
                const Cls c = classify_lds(K, N, t0, cnt, L, i, sbits);
                d = c.first;
                s = c.shared;
                r = c.rowstart;
            }
            fD |= (uint32_t)d << j;
            fS |= (uint32_t)s << j;
            fR |= (uint32_t)r << j;
            nD += __popcll(__ballot(d));
            nS += __popcll(__ballot(s));
            nR += __popcll(__ballot(r));
        }
        if (lane == 0) {
            wc[0][w] = nD;
            wc[1][w] = nS;
            wc[2][w] = nR;
        }
        __syncthreads();
        uint64_t pD = run[0], pS = run[1], pR = run[2];
        for (uint32_t k = 0; k < w; ++k) {
            pD += wc[0][k];
            pS += wc[1][k];
            pR += wc[2][k];
        }
#pragma unroll
        for (int j = 0; j < kRounds; ++j) {
            const bool d = (fD >> j) & 1u, s = (fS >> j) & 1u, r = (fR >> j) & 1u;
            const uint64_t bd = __ballot(d), bs = __ballot(s), br = __ballot(r);
            const uint64_t posD = pD + __popcll(bd & lt);
            const uint64_t posS = pS + __popcll(bs & lt);
            const uint64_t posR = pR + __popcll(br & lt);
            if (d | s) {
                const uint64_t key = L[wb + j * kWave + lane + 1];
                if (d && Dout) Dout[posD] = key;
                if (s) Sout[posS] = (uint32_t)(key & smask);
                if (r) {
                    row_id[posR] = key >> sbits;
                    row_ptr[posR] = posS;
                }
            }
            pD += __popcll(bd);
            pS += __popcll(bs);
            pR += __popcll(br);
        }
        __syncthreads();
        if (tid == 0) {
            for (int k = 0; k < kWaves; ++k) {
                run[0] += wc[0][k];
                run[1] += wc[1][k];
                run[2] += wc[2][k];
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Classification in LDS after a sort of the top ID bits only.
//
// The keys are ordered by bucket = key >> bsh (the top ID bits) and, inside a
// bucket, still in input order (every pass was stable, so entries of one ID
// are in ascending sample order).  Range c runs from the first bucket edge at
// or after c*stride to the first at or after (c+1)*stride (k_range_starts);
// the encoder tries the strides of kLocalStrides in turn until no range
// exceeds kLocalCapKeys, and launches the kernel built for kLocalShortCap keys
// when every range fits it, else the one for kLocalCapKeys.
// A range is made of whole buckets, so it holds whole rows of A and needs no
// halo.  One block loads a range (<= Cap keys) into LDS, finishes
// the sort there (stable LSD passes over the ID bits below the range's first
// bucket), classifies as k_cls_count/k_cls_write do, and writes its results
// at the range's own position (distinct keys in place over the range, shared
// pairs at the range start, rows at half the range start) with its counts;
// k_local_move then packs them after a scan of the counts.  A range longer
// than the cap (a bucket with very many keys) sets err bit 8 before any
// block writes; when it does at every try the caller sorts every ID bit
// and uses k_cls_count/k_cls_write.
constexpr int kLNT = 512;
constexpr int kLWaves = kLNT / kWave;

__device__ __forceinline__ uint64_t bucket_of(uint64_t key, uint32_t bsh) { return bsh >= 64 ? 0 : key >> bsh; }
__device__ __forceinline__ uint64_t div_up_dev(uint64_t a, uint64_t b) { return (a + b - 1) / b; }
__device__ __forceinline__ uint32_t dev_ceil_log2(uint64_t v) { return v <= 1 ? 0u : 64u - (uint32_t)__clzll(v - 1); }

// rs[c] = first bucket edge at or after c*stride, c in [0, nlc]; positions
// 0 and N are edges.  One wave per c, 256 keys per step.  An edge more than
// cap keys away is not looked for: rs[c] = ~0 and err |= 8.
__global__ __launch_bounds__(256) void k_range_starts(const uint64_t *__restrict__ K, uint64_t N, uint32_t bsh,
                                                       uint64_t stride, uint64_t nlc, uint64_t *__restrict__ rs,
                                                       uint32_t *err, const uint64_t *__restrict__ dsz,
                                                       uint32_t cap) {
    if (plan_aborted(dsz)) return;
    if (dsz) {
        N = dsz[PZ_N];
        nlc = div_up_dev(N, stride);
    }
    const uint64_t c = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
    const uint32_t lane = lane_id();
    if (c > nlc) return;  // whole waves
    const uint64_t x = c * stride;
    if (x == 0 || x >= N) {
        if (lane == 0) rs[c] = min(x, N);
        return;
    }
    const uint64_t b0 = bucket_of(K[x - 1], bsh);
    for (uint64_t y = x; y < x + cap; y += 4 * kWave) {
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const uint64_t t = y + k * kWave + lane;
            const uint64_t m = __ballot(t >= N || bucket_of(K[t], bsh) != b0);
            if (m) {
                if (lane == 0) rs[c] = y + k * kWave + (uint64_t)__builtin_ctzll(m);
                return;
            }
        }
    }
    if (lane == 0) {
        rs[c] = ~0ull;
        atomicOr(err, 8u);
    }
}

// Checks every range (err |= 8 as above), whether it is longer than
// kLocalShortCap (err |= 128) and whether its keys fit 32 bits once made
// relative to the range's first bucket: ((id - rbase) << sbits) | sample, with
// rbase = first bucket << lowbits, needs lowbits + ceil_log2(the number of
// bucket values spanned) + sbits bits; err |= 16 where that exceeds 32.
// The flags of a thread's ranges are gathered first and set with one atomic
// per wave (every range may set bits 16 and 128).
__global__ void k_range_check(const uint64_t *__restrict__ K, const uint64_t *rs, uint64_t nlc, uint32_t bsh,
                              uint32_t lowbits, uint32_t sbits, uint32_t *err, const uint64_t *__restrict__ dsz,
                              uint64_t stride, uint32_t cap) {
    if (plan_aborted(dsz)) return;
    if (dsz) nlc = div_up_dev(dsz[PZ_N], stride);
    uint32_t f = 0;
    for (uint64_t c = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; c < nlc; c += (uint64_t)gridDim.x * blockDim.x) {
        const uint64_t a = rs[c], b = rs[c + 1];
        if (a == ~0ull || b == ~0ull || b < a || b - a > cap) {
            f |= 8u;
        } else if (b > a) {
            if (b - a > kLocalShortCap) f |= 128u;
            const uint64_t bf = bucket_of(K[a], bsh), bl = bucket_of(K[b - 1], bsh);
            if (lowbits + dev_ceil_log2(bl - bf + 1) + sbits > 32) f |= 16u;
        }
    }
    const uint64_t m8 = __ballot((f & 8u) != 0), m16 = __ballot((f & 16u) != 0), m128 = __ballot((f & 128u) != 0);
    if (lane_id() == 0 && (m8 | m16 | m128))
        atomicOr(err, (m8 ? 8u : 0u) | (m16 ? 16u : 0u) | (m128 ? 128u : 0u));
}

// KT is the LDS form of a key, relative to the range's first bucket:
// uint32_t when every range fits 32 bits (k_range_check), else uint64_t.
// Cap is the most keys of a range.  Blocks per CU (by LDS): 4 for 32-bit keys
// and Cap 4096, 3 for 32-bit keys and Cap 6144 or 64-bit keys and Cap 4096,
// 2 for 64-bit keys and Cap 6144; the register budget matches.
constexpr int local_cls_waves(size_t kt, uint32_t cap) { return kt == 4 ? (cap <= 4096 ? 8 : 6) : (cap <= 4096 ? 6 : 4); }
template <class KT, uint32_t Cap>
__global__ __launch_bounds__(kLNT) __attribute__((amdgpu_waves_per_eu(local_cls_waves(sizeof(KT), Cap)))) void k_local_cls(
    uint64_t *__restrict__ K, uint32_t sbits, uint64_t smask, uint32_t bsh, uint32_t lowbits,
    const uint64_t *__restrict__ rs, uint32_t nlc, uint32_t *__restrict__ cnt, int keep, uint32_t *__restrict__ Sg,
    uint64_t *__restrict__ rid_g, uint64_t *__restrict__ rptr_g, unsigned long long *__restrict__ dupc,
    unsigned long long *__restrict__ rows_rep, const uint64_t *__restrict__ dsz, uint64_t stride, uint32_t *err) {
    static_assert(Cap <= kLocalCapKeys && Cap % kLNT == 0, "range cap");
    constexpr uint32_t kLRounds = Cap / kLNT;  // keys per thread
    __shared__ KT A[Cap];
    // per wave and digit d: a 16-bit count (then start) in half d & 1 of word d >> 1
    // (positions < 2^16; counts per wave <= Cap / kLWaves rounded up to 64 < 2^10)
    __shared__ uint32_t wcnt[kLWaves][128];
    __shared__ uint64_t T[kLWaves][256];  // per wave: lanes of the current round with digit d
    __shared__ uint64_t sh[kLWaves];
    __shared__ uint32_t wc[3][kLWaves];
    const uint32_t tid = threadIdx.x, lane = lane_id(), w = tid / kWave;
    const uint64_t lt = lanemask_lt();
    const uint32_t c = blockIdx.x;
    if (plan_aborted(dsz)) return;
    {
        // a planned launch covers the most ranges; the others count nothing,
        // and a range this kernel cannot hold is flagged and skipped
        const bool beyond = dsz && c >= div_up_dev(dsz[PZ_N], stride);
        const bool bad = !beyond && (rs[c] == ~0ull || rs[c + 1] == ~0ull || rs[c + 1] < rs[c] ||
                                     rs[c + 1] - rs[c] > Cap);
        if (beyond || bad) {
            if (tid == 0) {
                cnt[c] = 0;
                cnt[nlc + c] = 0;
                cnt[2 * (uint64_t)nlc + c] = 0;
                if (bad) atomicOr(err, 8u);
            }
            return;
        }
    }
    for (uint32_t i = tid; i < kLWaves * 256; i += kLNT) (&T[0][0])[i] = 0;
    const uint64_t s0 = rs[c], s1 = rs[c + 1];
    const uint32_t L = (uint32_t)(s1 - s0);  // <= Cap (k_range_check)
    // relative keys: key - kbase = ((id - rbase) << sbits) | sample < 2^(nb + sbits)
    uint64_t kbase = 0;
    uint32_t nb = 0;
    if (L > 0) {
        const uint64_t bf = bucket_of(K[s0], bsh), bl = bucket_of(K[s1 - 1], bsh);
        kbase = (bf << lowbits) << sbits;  // bf > 0 only when lowbits < U <= 63
        // with no ID bits below the buckets (every ID bit sorted globally)
        // the range is sorted already: a bucket is one ID, its keys in sample order
        nb = lowbits == 0 ? 0u : lowbits + dev_ceil_log2(bl - bf + 1);
    }
    {
        // every load of the range in flight at once, then the LDS stores
        uint64_t v[kLRounds];
#pragma unroll
        for (uint32_t j = 0; j < kLRounds; ++j) {
            const uint32_t i = tid + j * kLNT;
            v[j] = i < L ? K[s0 + i] : 0;
        }
#pragma unroll
        for (uint32_t j = 0; j < kLRounds; ++j) {
            const uint32_t i = tid + j * kLNT;
            if (i < L) A[i] = (KT)(v[j] - kbase);
        }
    }
    // wave w owns positions [w*seg, (w+1)*seg), 64 per round, in order
    const uint32_t seg = ((L + kLWaves - 1) / kLWaves + kWave - 1) / kWave * kWave;
    const uint32_t rounds = seg / kWave;
    const uint32_t wb = w * seg;
    __syncthreads();

    // --- finish the sort: stable LSD passes (8-bit digits) over the relative ID
    if (L > 1) {
        for (uint32_t p = 0; p < nb; p += 8) {
            const uint32_t dsh = sbits + p;
            for (uint32_t i = tid; i < kLWaves * 128; i += kLNT) (&wcnt[0][0])[i] = 0;
            KT key[kLRounds];
            uint32_t rank[kLRounds];
#pragma unroll
            for (uint32_t j = 0; j < kLRounds; ++j) {
                const uint32_t t = wb + j * kWave + lane;
                key[j] = (j < rounds && t < L) ? A[t] : 0;
            }
            __syncthreads();
            // Rank within the wave: the lanes of a round with the same digit
            // find each other through T[w][d] (each ORs in its lane bit, reads
            // the set back, and clears it; one wave's LDS operations run in
            // order, so the rounds of a half are issued back to back and
            // their sets read afterwards), take consecutive slots after the
            // digit's count so far, and the lowest of them adds the group to
            // the count with one LDS atomic (in round order) whose return its
            // peers fetch later.  rank[j] = that return | leader << 10 |
            // lanes before << 16 until the fetch (counts per wave < 2^10).
            constexpr uint32_t kHalf = (kLRounds + 1) / 2;
#pragma unroll
            for (uint32_t h = 0; h < 2; ++h) {
                uint64_t peers[kHalf];
#pragma unroll
                for (uint32_t jj = 0; jj < kHalf; ++jj) {
                    const uint32_t j = h * kHalf + jj;
                    peers[jj] = 0;
                    if (j < kLRounds && j < rounds && wb + j * kWave + lane < L) {
                        const uint32_t d = (uint32_t)(key[j] >> dsh) & 255u;
                        atomicOr((unsigned long long *)&T[w][d], 1ull << lane);
                        peers[jj] = __hip_atomic_load(&T[w][d], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
                        __hip_atomic_store(&T[w][d], 0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
                    }
                }
#pragma unroll
                for (uint32_t jj = 0; jj < kHalf; ++jj) {
                    const uint32_t j = h * kHalf + jj;
                    if (j < kLRounds && j < rounds) {
                        const uint64_t pr = peers[jj];
                        const uint32_t before = __popcll(pr & lt);
                        const uint32_t leader = pr ? (uint32_t)__builtin_ctzll(pr) : lane;
                        uint32_t old = 0;
                        if (pr && before == 0) {
                            const uint32_t d = (uint32_t)(key[j] >> dsh) & 255u, hs = (d & 1u) * 16u;
                            old = (atomicAdd(&wcnt[w][d >> 1], (uint32_t)__popcll(pr) << hs) >> hs) & 0xFFFFu;
                        }
                        rank[j] = old | (leader << 10) | (before << 16);
                    }
                }
            }
#pragma unroll
            for (uint32_t j = 0; j < kLRounds; ++j)
                if (j < rounds) {
                    const uint32_t f = rank[j];
                    rank[j] = ((uint32_t)__shfl((int)f, (int)((f >> 10) & 63u), kWave) & 1023u) + (f >> 16);
                }
            __syncthreads();
            // thread tid < 128 owns digits 2 tid and 2 tid + 1
            uint32_t tlo = 0, thi = 0;
            if (tid < 128)
                for (int k = 0; k < kLWaves; ++k) {
                    const uint32_t v = wcnt[k][tid];
                    tlo += v & 0xFFFFu;
                    thi += v >> 16;
                }
            uint64_t all;
            const uint32_t ex = (uint32_t)block_excl_scan<kLNT>(tlo + thi, sh, &all);
            if (tid < 128) {  // the halves become where wave k's keys of each digit start in the range
                uint32_t rlo = ex, rhi = ex + tlo;
                for (int k = 0; k < kLWaves; ++k) {
                    const uint32_t v = wcnt[k][tid];
                    wcnt[k][tid] = rlo | (rhi << 16);
                    rlo += v & 0xFFFFu;
                    rhi += v >> 16;
                }
            }
            __syncthreads();
#pragma unroll
            for (uint32_t j = 0; j < kLRounds; ++j)
                if (j < rounds && wb + j * kWave + lane < L) {
                    const uint32_t d = (uint32_t)(key[j] >> dsh) & 255u;
                    A[((wcnt[w][d >> 1] >> ((d & 1u) * 16u)) & 0xFFFFu) + rank[j]] = key[j];
                }
            __syncthreads();
        }
    }

    // --- classify (as classify_lds, with the whole row in LDS)
    uint32_t fD = 0, fS = 0, fR = 0;
    uint32_t nD = 0, nS = 0, nR = 0;
    uint64_t rows = 0;  // nonzero rows of A (distinct IDs) seen by this thread
    for (uint32_t j = 0; j < rounds; ++j) {
        const uint32_t t = wb + j * kWave + lane;
        bool d = false, sh_ = false, r = false;
        if (t < L) {
            const KT key = A[t], id = key >> sbits;
            const bool first = t == 0 || A[t - 1] != key;
            const bool left = first && t > 0 && (A[t - 1] >> sbits) == id;
            bool right = false;
            if (first) {
                uint32_t u = t + 1;
                while (u < L && A[u] == key) ++u;
                right = u < L && (A[u] >> sbits) == id;
            }
            d = first;
            sh_ = first && (left || right);
            r = sh_ && !left;
            rows += first && !left;
            if (!first) atomicAdd(&dupc[key & smask], 1ull);
        }
        fD |= (uint32_t)d << j;
        fS |= (uint32_t)sh_ << j;
        fR |= (uint32_t)r << j;
        nD += __popcll(__ballot(d));
        nS += __popcll(__ballot(sh_));
        nR += __popcll(__ballot(r));
    }
    if (lane == 0) {
        wc[0][w] = nD;
        wc[1][w] = nS;
        wc[2][w] = nR;
    }
    uint64_t all_rows;
    block_excl_scan<kLNT>(rows, sh, &all_rows);  // synchronises: wc is complete after it
    if (tid == 0) {
        uint32_t tD = 0, tS = 0, tR = 0;
        for (int k = 0; k < kLWaves; ++k) {
            tD += wc[0][k];
            tS += wc[1][k];
            tR += wc[2][k];
        }
        cnt[c] = tD;
        cnt[nlc + c] = tS;
        cnt[2 * (uint64_t)nlc + c] = tR;
        if (all_rows) atomicAdd(&rows_rep[c % kStatReplicas], (unsigned long long)all_rows);
    }

    // --- ordered writes at the range's own position (every read of the range is done)
    uint32_t pD = 0, pS = 0, pR = 0;
    for (uint32_t k = 0; k < w; ++k) {
        pD += wc[0][k];
        pS += wc[1][k];
        pR += wc[2][k];
    }
    const uint64_t r0 = s0 / 2;
    for (uint32_t j = 0; j < rounds; ++j) {
        const bool d = (fD >> j) & 1u, sh_ = (fS >> j) & 1u, r = (fR >> j) & 1u;
        const uint64_t bd = __ballot(d), bs = __ballot(sh_), br = __ballot(r);
        if (d | sh_) {
            const uint64_t key = kbase + (uint64_t)A[wb + j * kWave + lane];
            const uint32_t posS = pS + __popcll(bs & lt);
            if (d && keep) K[s0 + pD + __popcll(bd & lt)] = key;
            if (sh_) Sg[s0 + posS] = (uint32_t)(key & smask);
            if (r) {
                const uint64_t posR = r0 + pR + __popcll(br & lt);
                rid_g[posR] = key >> sbits;
                rptr_g[posR] = posS;
            }
        }
        pD += __popcll(bd);
        pS += __popcll(bs);
        pR += __popcll(br);
    }
}

// Launches the k_local_cls built for the key width and the range cap.
template <class... Args>
void launch_local_cls(bool wide, uint32_t cap, uint32_t grid, hipStream_t s, Args... args) {
    if (cap != kLocalShortCap && cap != kLocalCapKeys) fail(JAS_EDEVICE, "local classify: no kernel for this range cap");
    if (wide) {
        if (cap == kLocalShortCap) k_local_cls<uint64_t, kLocalShortCap><<<grid, kLNT, 0, s>>>(args...);
        else k_local_cls<uint64_t, kLocalCapKeys><<<grid, kLNT, 0, s>>>(args...);
    } else {
        if (cap == kLocalShortCap) k_local_cls<uint32_t, kLocalShortCap><<<grid, kLNT, 0, s>>>(args...);
        else k_local_cls<uint32_t, kLocalCapKeys><<<grid, kLNT, 0, s>>>(args...);
    }
}

// Packs the rows k_local_cls wrote per range (and, for the query index, the
// distinct keys): one block per range (grid-stride).  The shared pairs stay
// where the range wrote them (from its start, with gaps between ranges), so
// a row is row_deg entries of that array from row_ptr.
__global__ __launch_bounds__(256) void k_local_move(const uint64_t *__restrict__ rs, uint64_t nlc,
                                                     const uint64_t *__restrict__ oD, const uint64_t *__restrict__ oS,
                                                     const uint64_t *__restrict__ oR, const uint64_t *__restrict__ K,
                                                     const uint64_t *__restrict__ rid_g,
                                                     const uint64_t *__restrict__ rptr_g, uint64_t *__restrict__ Dk,
                                                     uint64_t *__restrict__ row_id, uint64_t *__restrict__ row_ptr,
                                                     uint32_t *__restrict__ row_deg, const uint64_t *__restrict__ dsz,
                                                     uint64_t stride) {
    if (plan_aborted(dsz)) return;
    if (dsz) nlc = div_up_dev(dsz[PZ_N], stride);
    for (uint64_t c = blockIdx.x; c < nlc; c += gridDim.x) {
        const uint64_t s0 = rs[c], r0 = s0 / 2;
        const uint64_t d0 = oD[c], nd = oD[c + 1] - d0;
        const uint64_t ns = oS[c + 1] - oS[c];
        const uint64_t w0 = oR[c], nr = oR[c + 1] - w0;
        for (uint64_t i = threadIdx.x; i < nr; i += blockDim.x) {
            row_id[w0 + i] = rid_g[r0 + i];
            const uint64_t a = rptr_g[r0 + i];
            row_ptr[w0 + i] = s0 + a;
            row_deg[w0 + i] = (uint32_t)((i + 1 < nr ? rptr_g[r0 + i + 1] : ns) - a);
        }
        if (Dk)
            for (uint64_t i = threadIdx.x; i < nd; i += blockDim.x) Dk[d0 + i] = K[s0 + i];
    }
}

// Degrees of contiguous rows: row_deg[r] = row_ptr[r + 1] - row_ptr[r].
__global__ void k_row_deg(const uint64_t *row_ptr, uint64_t R, uint32_t *row_deg) {
    for (uint64_t r = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; r < R; r += (uint64_t)gridDim.x * blockDim.x)
        row_deg[r] = (uint32_t)(row_ptr[r + 1] - row_ptr[r]);
}

// |X_i| = entries of sample i minus its repeated (ID, sample) entries.
__global__ void k_card_from_dups(const uint64_t *off, const unsigned long long *dupc, int32_t n,
                                 unsigned long long *card) {
    for (int32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
        card[i] = (off[i + 1] - off[i]) - dupc[i];
}

// Row degree histogram (degrees are <= n): input of the degree threshold choice.
__global__ __launch_bounds__(kNT) void k_deg_hist(const uint32_t *row_deg, uint64_t R, uint32_t nb,
                                                   int lds, unsigned long long *hist) {
    extern __shared__ uint32_t h[];
    if (lds)
        for (uint32_t i = threadIdx.x; i < nb; i += kNT) h[i] = 0;
    __syncthreads();
    for (uint64_t r = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; r < R; r += (uint64_t)gridDim.x * blockDim.x) {
        const uint64_t d = min((uint64_t)row_deg[r], (uint64_t)(nb - 1));
        if (lds) atomicAdd(&h[d], 1u);
        else atomicAdd(&hist[d], 1ull);
    }
    __syncthreads();
    if (lds)
        for (uint32_t i = threadIdx.x; i < nb; i += kNT)
            if (h[i]) atomicAdd(&hist[i], (unsigned long long)h[i]);
}

// Rows: degree split.
// Row split by degree in two passes over tiles of kSplitTile rows (8
// consecutive rows per thread): k_row_count counts each tile's packed rows
// (degree >= dmin) and the list rows' pairs; after a scan of the tile counts
// k_row_split places every row: packed row r at its tile's offset plus the
// packed rows before it in the tile, list row r at r minus the packed rows
// before it.
constexpr uint32_t kSplitPer = 8;
constexpr uint64_t kSplitTile = (uint64_t)kNT * kSplitPer;
static_assert(kSplitTile == kSplitTilePub, "row split tile");

// The 8 degrees of rows [r0, r0 + 8) (two 16-byte loads when all exist; r0 is a
// multiple of 8, so they are aligned); rows past R read as degree 0.
__device__ __forceinline__ void load_degrees(const uint32_t *__restrict__ row_deg, uint64_t r0, uint64_t R,
                                             uint32_t (&d)[kSplitPer]) {
    if (r0 + kSplitPer <= R) {
        const uint4 a = *reinterpret_cast<const uint4 *>(row_deg + r0);
        const uint4 b = *reinterpret_cast<const uint4 *>(row_deg + r0 + 4);
        d[0] = a.x; d[1] = a.y; d[2] = a.z; d[3] = a.w;
        d[4] = b.x; d[5] = b.y; d[6] = b.z; d[7] = b.w;
    } else {
#pragma unroll
        for (uint32_t k = 0; k < kSplitPer; ++k) d[k] = r0 + k < R ? row_deg[r0 + k] : 0u;
    }
}

__global__ __launch_bounds__(kNT) void k_row_count(const uint32_t *__restrict__ row_deg, uint64_t R, uint32_t dmin,
                                                    uint32_t *__restrict__ tcnt, unsigned long long *lp_rep,
                                                    const uint64_t *__restrict__ dsz) {
    __shared__ uint64_t sh[kWaves], sh2[kWaves];
    if (plan_aborted(dsz)) return;
    if (dsz) R = dsz[PZ_R];  // tiles past R count nothing
    const uint64_t r0 = (uint64_t)blockIdx.x * kSplitTile + (uint64_t)threadIdx.x * kSplitPer;
    uint64_t nd = 0, lp = 0;
    uint32_t dg[kSplitPer];
    load_degrees(row_deg, r0, R, dg);
#pragma unroll
    for (uint32_t k = 0; k < kSplitPer; ++k) {
        if (r0 + k < R) {
            const uint64_t d = dg[k];
            if (d >= dmin) ++nd;
            else lp += d * (d - 1) / 2;
        }
    }
    // block sums of both (one pass: wave sums, then thread 0)
    const uint64_t wd = wave_incl_scan(nd), wp = wave_incl_scan(lp);
    if (lane_id() == kWave - 1) {
        sh[threadIdx.x / kWave] = wd;
        sh2[threadIdx.x / kWave] = wp;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        uint64_t tot_d = 0, tot_p = 0;
#pragma unroll
        for (int k = 0; k < kWaves; ++k) {
            tot_d += sh[k];
            tot_p += sh2[k];
        }
        tcnt[blockIdx.x] = (uint32_t)tot_d;
        if (tot_p) atomicAdd(&lp_rep[blockIdx.x % kStatReplicas], (unsigned long long)tot_p);
    }
}

__global__ void k_sum_replicas(const unsigned long long *rep, uint32_t nrep, unsigned long long *dst) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        unsigned long long t = 0;
        for (uint32_t k = 0; k < nrep; ++k) t += rep[k];
        *dst += t;
    }
}

__global__ __launch_bounds__(kNT) void k_row_split(const uint32_t *__restrict__ row_deg, uint64_t R, uint32_t dmin,
                                                    const uint64_t *__restrict__ toff, uint64_t *__restrict__ Drow,
                                                    uint64_t *__restrict__ Lrow, const uint64_t *__restrict__ dsz) {
    __shared__ uint64_t sh[kWaves];
    if (plan_aborted(dsz)) return;
    // planned: with every shared row of one form the maps are the identity
    // (the kernels that read them check the same sizes)
    if (dsz && (dsz[PZ_QD] == 0 || dsz[PZ_QL] == 0)) return;
    if (dsz) R = dsz[PZ_R];
    const uint64_t r0 = (uint64_t)blockIdx.x * kSplitTile + (uint64_t)threadIdx.x * kSplitPer;
    uint32_t flags = 0, nd = 0;
    uint32_t dg[kSplitPer];
    load_degrees(row_deg, r0, R, dg);
#pragma unroll
    for (uint32_t k = 0; k < kSplitPer; ++k) {
        if (r0 + k < R && dg[k] >= dmin) {
            flags |= 1u << k;
            ++nd;
        }
    }
    uint64_t tot;
    uint64_t pd = toff[blockIdx.x] + block_excl_scan<kNT>(nd, sh, &tot);  // packed rows before r0
#pragma unroll
    for (uint32_t k = 0; k < kSplitPer; ++k) {
        const uint64_t r = r0 + k;
        if (r < R) {
            if ((flags >> k) & 1u) Drow[pd++] = r;
            else Lrow[r - pd] = r;
        }
    }
}

// Whether the packed-row map Drow / the list-row map Lrow is read: a null map,
// or (planned) every shared row of that form, is the identity.
__device__ __forceinline__ bool packed_map_used(const uint64_t *Drow, const uint64_t *dsz) {
    return Drow && !(dsz && dsz[PZ_QL] == 0);
}
__device__ __forceinline__ bool list_map_used(const uint64_t *Lrow, const uint64_t *dsz) {
    return Lrow && !(dsz && dsz[PZ_QD] == 0);
}

// Batches of packed rows.  Drow maps packed row q to its shared row; null
// when every shared row is packed (q itself), here and in k_pack.
// (planned: flags for q < QD, zeros up to the capacity QDcap = the host QD)
__global__ void k_batch_flag(const uint64_t *Drow, const uint64_t *row_id, uint64_t QD, uint32_t bbits,
                             uint32_t *bs, const uint64_t *__restrict__ dsz) {
    if (plan_aborted(dsz)) return;
    const uint64_t qd = dsz ? dsz[PZ_QD] : QD;
    if (!packed_map_used(Drow, dsz)) Drow = nullptr;
    for (uint64_t q = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; q < QD; q += (uint64_t)gridDim.x * blockDim.x) {
        if (q >= qd) {
            bs[q] = 0;
            continue;
        }
        const uint64_t b = row_id[Drow ? Drow[q] : q] >> bbits;
        bs[q] = (q == 0) || b != (row_id[Drow ? Drow[q - 1] : q - 1] >> bbits);
    }
}

__global__ void k_batch_start(const uint32_t *bs, const uint64_t *bpos, uint64_t QD, uint64_t *bq,
                              const uint64_t *__restrict__ dsz) {
    if (plan_aborted(dsz)) return;
    if (dsz) QD = dsz[PZ_QD];
    for (uint64_t q = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; q < QD; q += (uint64_t)gridDim.x * blockDim.x)
        if (bs[q]) bq[bpos[q]] = q;
}

// Word rows of b = wb bits (32 or 64) per batch: ceil(rows / b).
// (planned: nb batches, zeros up to the capacity nbcap = the host nb)
__global__ void k_batch_words(const uint64_t *bq, uint64_t nb, uint32_t wb, uint64_t *nw,
                              const uint64_t *__restrict__ dsz) {
    if (plan_aborted(dsz)) return;
    const uint64_t nbv = dsz ? dsz[PZ_NB] : nb;
    for (uint64_t b = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; b < nb; b += (uint64_t)gridDim.x * blockDim.x)
        nw[b] = b < nbv ? (bq[b + 1] - bq[b] + wb - 1) / wb : 0;
}

// Word row w (of wb bits) holds packed rows [wq0[w], wq1[w]): bit p % wb of
// row p / wb of its batch.
__global__ void k_word_rows(uint64_t QD, const uint64_t *bpos, const uint64_t *bq, const uint64_t *wbase, uint32_t wb,
                            uint64_t *wq0, uint64_t *wq1, const uint64_t *__restrict__ dsz) {
    if (plan_aborted(dsz)) return;
    if (dsz) QD = dsz[PZ_QD];
    for (uint64_t q = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; q < QD; q += (uint64_t)gridDim.x * blockDim.x) {
        const uint64_t b = bpos[q + 1] - 1;  // batch of packed row q
        const uint64_t p = q - bq[b];        // position inside the batch
        if (p % wb == 0) {
            const uint64_t w = wbase[b] + p / wb;
            wq0[w] = q;
            wq1[w] = min(q + wb, bq[b + 1]);
        }
    }
}

// One block per 64-bit row of W: OR the bits of its <= 64 rows into an LDS
// row of words and write it out.  With b = 64 a row of W is one word row;
// with b = 32 it holds word rows 2w (bits 0..31) and 2w + 1 (bits 32..63),
// each a 32-bit word per column, so the Gram kernels read both as one 64-bit
// step (the AND + popcount, or the dot product, of a 64-bit element is the
// sum over its two halves).  Wave 0 loads the rows' list starts and degrees
// (lane t: the row of bit t) and scans them, then all threads walk the rows'
// (row, sample) pairs in parallel (consecutive threads read consecutive
// samples of a row).  Hw = word rows of b bits.
__global__ __launch_bounds__(kNT) void k_pack(uint64_t *__restrict__ W, uint64_t ldw, uint64_t H, uint64_t Hw,
                                               uint32_t wb, const uint64_t *__restrict__ wq0,
                                               const uint64_t *__restrict__ wq1,
                                               const uint64_t *__restrict__ Drow,
                                               const uint64_t *__restrict__ row_ptr,
                                               const uint32_t *__restrict__ row_deg,
                                               const uint32_t *__restrict__ S, uint32_t cols,
                                               unsigned long long *st, const uint64_t *__restrict__ dsz) {
    extern __shared__ unsigned long long lw[];
    __shared__ uint64_t rstart[kWave + 1];  // exclusive prefix of the rows' degrees
    __shared__ uint64_t rbase[kWave];       // first pair of each row in S
    __shared__ uint8_t prow[kPackFlat];  // up to kPackFlat entries: the row of each entry
    __shared__ uint32_t zsh[2];  // nonzero words of the row (b = 32: of each half)
    const uint32_t tid = threadIdx.x, lane = lane_id();
    if (plan_aborted(dsz)) return;
    // planned: H is the capacity; rows from the actual count on are written as
    // zeros (they add nothing to the Gram product)
    const uint64_t Hv = dsz ? dsz[PZ_H] : H;
    if (!packed_map_used(Drow, dsz)) Drow = nullptr;
    if (dsz) Hw = dsz[PZ_HW];
    unsigned long long nnz_acc = 0, f_acc = 0;  // this block's totals (thread 0)
    for (uint64_t w = blockIdx.x; w < H; w += gridDim.x) {
        if (w >= Hv) {
            for (uint64_t i = tid; i < ldw; i += kNT) W[w * ldw + i] = 0;
            continue;
        }
        if (tid < kWave) {
            uint64_t q0 = 0, q1 = 0, qi = 0;  // this lane's row: qi, if below q1
            if (wb == 64) {
                q0 = wq0[w];
                q1 = wq1[w];
                qi = q0 + lane;
            } else {
                const uint64_t ww = 2 * w + (lane >> 5);
                if (ww < Hw) {
                    q0 = wq0[ww];
                    q1 = wq1[ww];
                }
                qi = q0 + (lane & 31);
            }
            uint64_t base = 0, deg = 0;
            if (qi < q1) {
                const uint64_t r = Drow ? Drow[qi] : qi;
                base = row_ptr[r];
                deg = row_deg[r];
            }
            const uint64_t inc = wave_incl_scan(deg);
            rstart[lane + 1] = inc;
            if (lane == 0) rstart[0] = 0;
            rbase[lane] = base;
        }
        if (tid < 2) zsh[tid] = 0;
        for (uint64_t c0 = 0; c0 < ldw; c0 += cols) {
            const uint32_t cn = (uint32_t)min((uint64_t)cols, ldw - c0);
            for (uint32_t i = tid; i < cn; i += kNT) lw[i] = 0;
            __syncthreads();
            const uint64_t P = rstart[kWave];
            if (P > kPackFlat) {
                // long rows (more than kPackFlat entries in all): the lanes of
                // a wave walk one row at a time
                // (kPackLoads loads in flight per lane before their ORs; a
                // sample of ~0u lies past every chunk)
                const uint32_t wv = tid / kWave;
                for (uint32_t t = wv; t < kWave; t += kNT / kWave) {
                    const uint64_t rb = rbase[t], dg = rstart[t + 1] - rstart[t];
                    for (uint64_t e0 = lane; e0 < dg; e0 += (uint64_t)kWave * kPackLoads) {
                        uint32_t v[kPackLoads];
#pragma unroll
                        for (uint32_t u = 0; u < kPackLoads; ++u) {
                            const uint64_t e = e0 + (uint64_t)u * kWave;
                            v[u] = e < dg ? S[rb + e] : ~0u;
                        }
#pragma unroll
                        for (uint32_t u = 0; u < kPackLoads; ++u)
                            if (v[u] >= c0 && v[u] < c0 + cn) atomicOr(&lw[v[u] - c0], 1ull << t);
                    }
                }
            } else {
                // up to kPackFlat entries: one thread per entry, its row read from prow
                // (filled by the waves a row at a time, once per word row);
                // kPackLoads entries per thread in flight
                if (c0 == 0) {
                    for (uint32_t t = tid / kWave; t < kWave; t += kNT / kWave)
                        for (uint32_t e = (uint32_t)rstart[t] + lane; e < (uint32_t)rstart[t + 1]; e += kWave)
                            prow[e] = (uint8_t)t;
                    __syncthreads();
                }
                for (uint64_t p0 = tid; p0 < P; p0 += (uint64_t)kNT * kPackLoads) {
                    uint32_t v[kPackLoads], row[kPackLoads];
#pragma unroll
                    for (uint32_t u = 0; u < kPackLoads; ++u) {
                        const uint64_t p = p0 + (uint64_t)u * kNT;
                        const uint32_t lo = p < P ? prow[p] : 0u;
                        row[u] = lo;
                        v[u] = p < P ? S[rbase[lo] + (p - rstart[lo])] : ~0u;
                    }
#pragma unroll
                    for (uint32_t u = 0; u < kPackLoads; ++u)
                        if (v[u] >= c0 && v[u] < c0 + cn) atomicOr(&lw[v[u] - c0], 1ull << row[u]);
                }
            }
            __syncthreads();
            uint32_t zl = 0, zh = 0;
            for (uint32_t i = tid; i < cn; i += kNT) {
                const unsigned long long v = lw[i];
                W[w * ldw + c0 + i] = v;
                if (wb == 64) {
                    zl += v != 0;
                } else {
                    zl += (uint32_t)v != 0;
                    zh += (v >> 32) != 0;
                }
            }
            if (zl) atomicAdd(&zsh[0], zl);
            if (zh) atomicAdd(&zsh[1], zh);
            __syncthreads();
        }
        if (tid == 0) {
            const unsigned long long z0 = zsh[0], z1 = zsh[1];
            nnz_acc += z0 + z1;
            f_acc += z0 * (z0 + 1) / 2 + z1 * (z1 + 1) / 2;
        }
        __syncthreads();
    }
    if (tid == 0 && nnz_acc) {
        atomicAdd(&st[ST_NNZW], nnz_acc);
        atomicAdd(&st[ST_F], f_acc);
    }
}

// Row lists: CSR of the rows of degree 2..dmin-1.  Lrow maps list row j to
// its shared row; null when every shared row is a list row (j itself), here
// and in k_list_wave_pairs and k_pair_emit.
__global__ void k_list_deg(const uint64_t *Lrow, const uint32_t *row_deg, uint64_t QL, uint64_t *deg) {
    for (uint64_t j = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; j < QL; j += (uint64_t)gridDim.x * blockDim.x) {
        const uint64_t r = Lrow ? Lrow[j] : j;
        deg[j] = row_deg[r];
    }
}

__global__ void k_list_gather(const uint64_t *Lrow, const uint64_t *row_ptr, const uint32_t *row_deg, const uint32_t *S,
                              const uint64_t *lptr, uint64_t QL, uint32_t *lsmp) {
    for (uint64_t j = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; j < QL; j += (uint64_t)gridDim.x * blockDim.x) {
        const uint64_t r = Lrow ? Lrow[j] : j;
        const uint64_t a0 = row_ptr[r], d = row_deg[r], o = lptr[j];
        for (uint64_t k = 0; k < d; ++k) lsmp[o + k] = S[a0 + k];
    }
}

// Row lists as pairs for the Gram step: every pair (a, b), a < b, of every
// list row as the 32-bit word (a << 16) | b, then sorted by a (single-pass
// scatters over the bits of a), so that the Gram step reads each sample's
// pairs as one contiguous run (the row-by-row form of B = A^T A over the row
// lists).  wnp[g] = pairs of list rows [64g, 64g + 64): one wave per group,
// which is also one wave's share of the emission below.
__global__ void k_list_wave_pairs(const uint64_t *Lrow, const uint32_t *row_deg, uint64_t QL, uint64_t *wnp,
                                  const uint64_t *__restrict__ dsz) {
    if (plan_aborted(dsz)) return;
    // planned: QL is the capacity; groups past the actual rows count nothing
    const uint64_t nw = (QL + kWave - 1) / kWave;
    if (dsz) QL = dsz[PZ_QL];
    if (!list_map_used(Lrow, dsz)) Lrow = nullptr;
    const uint32_t lane = lane_id();
    for (uint64_t g = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave; g < nw;
         g += ((uint64_t)gridDim.x * blockDim.x) / kWave) {
        const uint64_t j = g * kWave + lane;
        uint64_t np = 0;
        if (j < QL) {
            const uint64_t r = Lrow ? Lrow[j] : j;
            const uint64_t d = row_deg[r];
            np = d * (d - 1) / 2;
        }
        const uint64_t inc = wave_incl_scan(np);
        if (lane == kWave - 1) wnp[g] = inc;
    }
}

// A wave takes 64 consecutive rows; their pairs fill one contiguous stretch
// of the output (the rows' pair counts scanned).  When the stretch fits an
// LDS stage, each lane writes its own row's pairs there and the wave copies
// the stage out coalesced.  Otherwise each lane produces output words
// o = lane, lane + 64, ...: the row that holds o comes from a binary search
// over the wave's row starts, the pair (i, j) inside the row from the inverse
// of the triangular count P(i) = i (2d - i - 1) / 2 of the pairs whose smaller
// entry comes before i, so consecutive lanes write consecutive words whatever
// the row lengths (one lane per row would leave most lanes idle behind the
// longest row and scatter the stores).  The rows' samples are one span of the
// sample array (the rows ascend), read into LDS with coalesced loads first
// when it fits (else only the rows' own entries, packed, when those fit), so
// the pair loops read LDS rather than memory.  Per-block LDS totals of the
// sort digits (digit q = bits [16 + width*q, 16 + width*(q+1)) of the word)
// come from one pass over each row's entries.
// Stage sizes measured best of 256..3072 for one-lane-per-row emission.
constexpr uint32_t kEmitStage = 1024;  // output words per wave
constexpr uint32_t kEmitIn = 512;      // sample entries per wave
constexpr uint32_t kPairPasses = 2;   // 16 sample bits, 8-bit digits

// Largest i in [0, d-2] with P(i) <= k, for 0 <= k < d(d-1)/2 and 2 <= d <= 2^14:
// the smaller root of i^2 - (2d-1) i + 2k = 0 in float, then corrected by
// exact integer steps (the estimate is off by at most one).
__device__ __forceinline__ uint32_t pair_first(uint32_t d, uint32_t k) {
    const uint32_t b = 2 * d - 1;
    const float disc = (float)(b * b - 8u * k);
    int32_t i = (int32_t)(((float)b - sqrtf(disc)) * 0.5f);
    i = max(0, min(i, (int32_t)d - 2));
    const auto P = [d](int32_t x) { return (uint32_t)x * (2 * d - (uint32_t)x - 1) / 2; };
    while (i + 1 <= (int32_t)d - 2 && P(i + 1) <= k) ++i;
    while (i > 0 && P(i) > k) --i;
    return (uint32_t)i;
}

// Digit totals of one row: entry i is the smaller sample of deg - 1 - i pairs.
template <class Src>
__device__ __forceinline__ void row_digit_totals(Src src, uint64_t sb, uint32_t deg, uint32_t (*gh)[256],
                                                 uint32_t npass, uint32_t width, uint32_t dmask) {
    for (uint32_t i = 0; i + 1 < deg; ++i) {
        const uint32_t a = src[sb + i];
        for (uint32_t q = 0; q < npass; ++q) atomicAdd(&gh[q][(a >> (width * q)) & dmask], deg - 1 - i);
    }
}

// A wave whose pairs fit the stage: this lane's row's pairs, in order, at
// stage word o onwards.
template <class Src>
__device__ __forceinline__ void stage_row_pairs(Src src, uint64_t sb, uint32_t deg, uint32_t o, uint32_t *st) {
    for (uint32_t i = 0; i + 1 < deg; ++i) {
        const uint32_t a = src[sb + i] << 16;
        for (uint32_t j = i + 1; j < deg; ++j) st[o++] = a | src[sb + j];
    }
}

// The wave's pairs from its rows' entries src[sb + i] (LDS or global), one
// output word per lane at a time.  rst[0..64] are the rows' first words
// (rst[64] = total); a lane's words ascend, so its row only moves forward.
template <class Src>
__device__ __forceinline__ void emit_wave_pairs(Src src, uint32_t total, uint32_t lane, const uint32_t *rst,
                                                const uint32_t *rdg, const uint64_t *rsb,
                                                uint32_t *__restrict__ out) {
    uint32_t t = 0, d = rdg[0], k0 = 0;
    uint64_t s0 = rsb[0];
    for (uint32_t o = lane; o < total; o += kWave) {
        // row t: the largest with rst[t] <= o (a row without pairs shares its
        // successor's start, so it is never the largest)
        if (rst[t + 1] <= o) {
            do {
                ++t;
            } while (rst[t + 1] <= o);
            d = rdg[t];
            k0 = rst[t];
            s0 = rsb[t];
        }
        const uint32_t k = o - k0;
        const uint32_t i = pair_first(d, k);
        const uint32_t j = i + 1 + (k - i * (2 * d - i - 1) / 2);
        out[o] = (src[s0 + i] << 16) | src[s0 + j];
    }
}

__global__ __launch_bounds__(256) void k_pair_emit(const uint64_t *__restrict__ Lrow,
                                                    const uint64_t *__restrict__ row_ptr,
                                                    const uint32_t *__restrict__ row_deg,
                                                    const uint32_t *__restrict__ ls, uint64_t QL,
                                                    const uint64_t *__restrict__ wpo,
                                                    uint32_t *__restrict__ pairs, uint32_t npass, uint32_t width,
                                                    unsigned long long *__restrict__ ghist,
                                                    const uint64_t *__restrict__ dsz) {
    __shared__ uint32_t gh[kPairPasses][256];
    if (plan_aborted(dsz)) return;
    if (dsz) QL = dsz[PZ_QL];
    if (!list_map_used(Lrow, dsz)) Lrow = nullptr;
    // per wave: the output stage, or (for waves whose pairs do not fit it)
    // the rows' first output words, degrees and first entries
    __shared__ uint64_t stgb[256 / kWave][kEmitStage / 2];
    __shared__ uint32_t sinb[256 / kWave][kEmitIn];
    static_assert(2 * kWave + (kWave + 2) + kWave <= kEmitStage, "row tables exceed the stage");  // 32-bit words
    const uint32_t tid = threadIdx.x, lane = lane_id(), w = tid / kWave;
    const uint32_t dmask = (1u << width) - 1u;
#pragma unroll
    for (int k = 0; k < kPairPasses; ++k) gh[k][tid] = 0;
    __syncthreads();
    uint32_t *sin = sinb[w];
    uint32_t *stg = reinterpret_cast<uint32_t *>(stgb[w]);
    uint64_t *rsb = stgb[w];                                  // kWave entries
    uint32_t *rst = reinterpret_cast<uint32_t *>(rsb + kWave);  // kWave + 1 entries
    uint32_t *rdg = rst + kWave + 2;                          // kWave entries
    for (uint64_t r0 = ((uint64_t)blockIdx.x * (256 / kWave) + w) * kWave; r0 < QL;
         r0 += (uint64_t)gridDim.x * 256) {
        const uint64_t r = r0 + lane;
        const uint32_t last = (uint32_t)(min(r0 + kWave, QL) - 1 - r0);  // lane of the wave's last row
        uint64_t e0 = 0, e1 = 0;
        if (r < QL) {
            const uint64_t rr = Lrow ? Lrow[r] : r;
            e0 = row_ptr[rr];
            e1 = e0 + row_deg[rr];
        }
        // the wave's first pair (wpo: scan of the 64-row groups' pair counts)
        // and this row's pairs before it within the group; a list row has at
        // most n <= kSampleMajorMaxN entries, so a wave's 64 rows hold fewer
        // than 2^32 pairs
        const uint64_t base = wpo[r0 / kWave];
        const uint32_t deg = (uint32_t)(e1 - e0);
        const uint32_t np = deg * (deg - (deg ? 1u : 0u)) / 2;
        const uint32_t incl = (uint32_t)wave_incl_scan((uint64_t)np);
        const uint32_t total = __shfl(incl, kWave - 1, kWave);
        // the rows' samples in LDS: the whole span of the sample array when it
        // fits (coalesced), else only the rows' own entries packed one after
        // another (when the span has gaps: rows of other kinds or the ends of
        // LDS ranges)
        const uint64_t dincl = wave_incl_scan((uint64_t)deg);
        const uint64_t dtot = __shfl(dincl, kWave - 1, kWave);
        const uint64_t span0 = __shfl(e0, 0, kWave);
        const uint64_t span1 = __shfl(e1, (int)last, kWave);
        const bool whole = span1 - span0 <= kEmitIn;       // wave-uniform
        const bool staged_in = whole || dtot <= kEmitIn;  // wave-uniform
        uint64_t sb = e0;                                  // entry i of this row: src[sb + i]
        if (whole) {
            for (uint64_t k = lane; k < span1 - span0; k += kWave) sin[k] = ls[span0 + k];
            sb = e0 - span0;
        } else if (staged_in) {
            const uint64_t off = dincl - deg;
            for (uint32_t k = 0; k < deg; k += 4) {
                uint32_t v[4];
#pragma unroll
                for (int u = 0; u < 4; ++u) v[u] = k + u < deg ? ls[e0 + k + u] : 0u;
#pragma unroll
                for (int u = 0; u < 4; ++u)
                    if (k + u < deg) sin[off + k + u] = v[u];
            }
            sb = off;
        }
        const bool fits = total <= kEmitStage;  // wave-uniform
        if (!fits) {
            rsb[lane] = sb;
            rst[lane] = incl - np;
            rdg[lane] = deg;
            if (lane == 0) rst[kWave] = total;
        }
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        __builtin_amdgcn_wave_barrier();
        if (staged_in) row_digit_totals(sin, sb, deg, gh, npass, width, dmask);
        else row_digit_totals(ls, sb, deg, gh, npass, width, dmask);
        if (fits) {
            if (staged_in) stage_row_pairs(sin, sb, deg, incl - np, stg);
            else stage_row_pairs(ls, sb, deg, incl - np, stg);
            __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
            __builtin_amdgcn_wave_barrier();
            for (uint32_t k = lane; k < total; k += kWave) pairs[base + k] = stg[k];
        } else if (staged_in) {
            emit_wave_pairs(sin, total, lane, rst, rdg, rsb, pairs + base);
        } else {
            emit_wave_pairs(ls, total, lane, rst, rdg, rsb, pairs + base);
        }
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        __builtin_amdgcn_wave_barrier();
    }
    __syncthreads();
    unsigned long long *g = ghist + (uint64_t)(blockIdx.x % kGhistReplicas) * kMaxPasses * 256;
    for (uint32_t q = 0; q < npass; ++q)
        if (gh[q][tid]) atomicAdd(&g[q * 256 + tid], (unsigned long long)gh[q][tid]);
}

// Query index: bucket[b] = first distinct key whose ID has top bits >= b.
__global__ void k_bucket(const uint64_t *D, uint64_t ND, uint32_t sbits, uint32_t shift, uint64_t nbk,
                         uint64_t *bucket) {
    for (uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; t <= ND; t += (uint64_t)gridDim.x * blockDim.x) {
        const uint64_t bk = t < ND ? ((D[t] >> sbits) >> shift) : nbk;
        const int64_t prev = t == 0 ? -1 : (int64_t)((D[t - 1] >> sbits) >> shift);
        for (int64_t b = prev + 1; b <= (int64_t)bk; ++b) bucket[b] = t;
    }
}

// --- planned encode: sizes after each scan, checked against the capacities.
// One thread each; a size above its capacity sets PZ_ABORT (every later
// kernel of the encode then returns at once) and err bit 32.
__global__ void k_plan_begin(const uint64_t *off, int32_t n, uint64_t Ncap, uint64_t *dsz, uint32_t *err) {
    uint64_t N = n > 0 ? off[n] : 0;
    for (int k = 0; k < PZ_COUNT; ++k) dsz[k] = 0;
    err[0] = 0;
    if (N > Ncap) {  // nothing is encoded (the sort sees no keys either)
        dsz[PZ_ABORT] = 1;
        dsz[PZ_OVER] = PZ_N + 1;
        dsz[PZ_OVER_VALUE] = N;
        err[0] = 32u;
        N = 0;
    }
    dsz[PZ_N] = N;
}

__global__ void k_plan_rows(const uint64_t *offR, const uint64_t *offS, uint64_t nlc_cap, uint64_t Rcap,
                            uint64_t *rptr, uint64_t *dsz, uint32_t *err) {
    if (dsz[PZ_ABORT]) return;
    const uint64_t R = offR[nlc_cap], NS = offS[nlc_cap];
    if (R > Rcap) {
        dsz[PZ_ABORT] = 1;
        dsz[PZ_OVER] = PZ_R + 1;
        dsz[PZ_OVER_VALUE] = R;
        atomicOr(err, 32u);
        return;
    }
    dsz[PZ_R] = R;
    rptr[R] = NS;
}

__global__ void k_plan_split(const uint64_t *toff, uint64_t tile_cap, uint64_t QDcap, uint64_t QLcap, uint64_t *dsz,
                             uint32_t *err) {
    if (dsz[PZ_ABORT]) return;
    const uint64_t QD = toff[tile_cap], QL = dsz[PZ_R] - QD;
    if (QD > QDcap || QL > QLcap) {
        dsz[PZ_ABORT] = 1;
        dsz[PZ_OVER] = QD > QDcap ? PZ_QD + 1 : PZ_QL + 1;
        dsz[PZ_OVER_VALUE] = QD > QDcap ? QD : QL;
        atomicOr(err, 32u);
        return;
    }
    dsz[PZ_QD] = QD;
    dsz[PZ_QL] = QL;
}

__global__ void k_plan_batches(const uint64_t *bpos, uint64_t QDcap, uint64_t *bq, uint64_t *dsz) {
    if (dsz[PZ_ABORT]) return;
    const uint64_t nb = bpos[QDcap];  // the flags past QD are zero
    dsz[PZ_NB] = nb;
    bq[nb] = dsz[PZ_QD];
}

__global__ void k_plan_words(const uint64_t *wbase, uint64_t QDcap, uint32_t wb, uint64_t Hwcap, uint64_t Hcap,
                             uint64_t *dsz, uint32_t *err) {
    if (dsz[PZ_ABORT]) return;
    const uint64_t Hw = wbase[QDcap], H = wb == 64 ? Hw : (Hw + 1) / 2;
    if (Hw > Hwcap || H > Hcap) {
        dsz[PZ_ABORT] = 1;
        dsz[PZ_OVER] = PZ_HW + 1;
        dsz[PZ_OVER_VALUE] = Hw;
        atomicOr(err, 32u);
        return;
    }
    dsz[PZ_HW] = Hw;
    dsz[PZ_H] = H;
}

__global__ void k_plan_pairs(const uint64_t *npo, uint64_t gcap, uint64_t Pcap, uint64_t *dsz, uint32_t *err) {
    if (dsz[PZ_ABORT]) return;
    const uint64_t P = npo[gcap];
    if (P > Pcap) {
        dsz[PZ_ABORT] = 1;
        dsz[PZ_OVER] = PZ_P + 1;
        dsz[PZ_OVER_VALUE] = P;
        atomicOr(err, 32u);
        return;
    }
    dsz[PZ_P] = P;
}

// err bit 64: a set reaches the int32 bound (|X_i| >= limit)
__global__ void k_plan_card(const int64_t *card, int32_t n, int64_t limit, uint32_t *err) {
    bool over = false;
    for (int32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) over |= card[i] >= limit;
    if (__ballot(over) && lane_id() == 0) atomicOr(err, 64u);
}

template <class F>
void launch_1d(uint64_t work, hipStream_t s, F f) {
    const uint64_t blocks = std::min<uint64_t>(std::max<uint64_t>(div_up(work, 256), 1), 65536);
    f((uint32_t)blocks, s);
}

uint64_t to_host_u64(const uint64_t *dptr, hipStream_t s) {
    JAS_HOST_TIMED("readback_sync");
    uint64_t v = 0;
    JAS_HIP(hipMemcpyAsync(&v, dptr, sizeof(v), hipMemcpyDeviceToHost, s));
    JAS_HIP(hipStreamSynchronize(s));
    return v;
}

}  // namespace

void build_keys(const uint64_t *ids, const uint64_t *offsets, int32_t n, uint64_t N, uint32_t sbits, uint32_t U,
                const SortPlan &plan, uint64_t *keys, uint32_t *err, unsigned long long *ghist, hipStream_t s) {
    if (N == 0) return;
    const uint64_t hi_mask = U >= 64 ? 0 : ~((uint64_t(1) << U) - 1);
    const uint64_t blocks = div_up(N, kChunk);
    if (blocks > 0xFFFFFFFFull) fail(JAS_EUNSUPPORTED, "too many IDs");
    if (keys) {
        JAS_TIMED("build_keys", s);
        k_build_keys<<<(uint32_t)blocks, kNT, 0, s>>>(ids, offsets, n, N, sbits, hi_mask, keys, err, plan.npass,
                                                      U - plan.top_bits, plan.width, ghist, nullptr);
    } else {
        JAS_TIMED("count_digits", s);
        k_count_digits<<<(uint32_t)blocks, kNT, 0, s>>>(ids, N, hi_mask, err, plan.npass, U - plan.top_bits,
                                                        plan.width, ghist, nullptr);
    }
    check_launch("build keys");
}

void encode_sorted(jas_db *db, DevBuf<uint64_t> &keys, DevBuf<uint64_t> &alt, uint64_t N, const SortPlan &plan,
                   const uint64_t *offsets, hipStream_t s, Budget *tb) {
    const int32_t n = db->n;
    const uint32_t sbits = db->sbits;
    const uint64_t smask = sbits ? ((uint64_t(1) << sbits) - 1) : 0;
    const bool keep = db->flags & JAS_KEEP_IDS;
    const bool query_only = db->flags & JAS_QUERY_ONLY;  // no packed words or row lists

    DevBuf<unsigned long long> st;
    st.alloc(ST_N, s, tb, true, "encode counters");
    {
        JAS_TIMED("fill_u64", s);
        k_fill_u64<<<1, 64, 0, s>>>((uint64_t *)st.p, ST_N, 0);
    }
    DevBuf<unsigned long long> cardc;
    cardc.alloc(std::max<int32_t>(n, 1), s, tb, true, "column sums");
    {
        JAS_TIMED("fill_u64", s);
        k_fill_u64<<<64, 256, 0, s>>>((uint64_t *)cardc.p, (uint64_t)std::max<int32_t>(n, 1), 0);
    }
    check_launch("fill");

    // Outputs of the classification: distinct keys (query index), shared
    // pairs S in row order, and per shared row its ID and first pair.
    uint64_t NDk = 0, NS = 0, R = 0;
    DevBuf<uint64_t> Dk, rid_own, rptr_own;
    DevBuf<uint32_t> rdeg_own;
    DevBuf<uint32_t> S_own;
    uint32_t *Sp = nullptr;
    uint64_t *ridp = nullptr, *rptrp = nullptr;
    uint32_t *rdegp = nullptr;
    bool done = N == 0;

    // --- classify each range of whole buckets in LDS ------------------------
    constexpr uint64_t kMinStride = kLocalStrides[sizeof(kLocalStrides) / sizeof(kLocalStrides[0]) - 1];
    if (!done && div_up(N, kMinStride) <= 0xFFFFFFFFull && alt.n >= N + 2) {
        const uint32_t lowbits = db->U - plan.top_bits;
        const uint32_t bsh = sbits + lowbits;
        DevBuf<uint64_t> rs, flags;
        rs.alloc(div_up(N, kMinStride) + 1, s, tb, true, "range starts");
        flags.alloc(1, s, tb, true, "range error flag");
        uint32_t *errL = reinterpret_cast<uint32_t *>(flags.p);
        uint64_t herr = 8, nlc = 0;
        uint32_t cap = kLocalCapKeys;
        // with every ID bit sorted globally the ranges need no LDS passes, and
        // longer ranges (fewer blocks) pay: 4096 is tried first
        const uint64_t strides[] = {kLocalWideStride, kLocalStrides[0], kLocalStrides[1]};
        for (const uint64_t stride : strides) {
            if (stride == kLocalWideStride && lowbits != 0) continue;
            nlc = div_up(N, stride);
            {
                JAS_TIMED("fill_u64", s);
                k_fill_u64<<<1, 64, 0, s>>>(flags.p, 1, 0);
            }
            {
                JAS_TIMED("range_starts", s);
                k_range_starts<<<(uint32_t)div_up(nlc + 1, 256 / kWave), 256, 0, s>>>(keys.p, N, bsh, stride, nlc,
                                                                                       rs.p, errL, nullptr, cap);
                k_range_check<<<(uint32_t)std::min<uint64_t>(div_up(nlc, 256), 4096), 256, 0, s>>>(
                    keys.p, rs.p, nlc, bsh, lowbits, sbits, errL, nullptr, 0, cap);
            }
            check_launch("range starts");
            JAS_HIP(hipMemcpyAsync(&herr, flags.p, sizeof(uint64_t), hipMemcpyDeviceToHost, s));
            JAS_HIP(hipStreamSynchronize(s));
            if ((herr & 8u) == 0) {
                cap = herr & 128u ? kLocalCapKeys : kLocalShortCap;
                db->trace.stride = stride;
                db->trace.lcap = cap;
                break;
            }
        }
        if ((herr & 8u) == 0) {
            DevBuf<unsigned long long> dupc;
            DevBuf<uint32_t> cnt;
            DevBuf<uint64_t> rid_g, offD, offS, offR, stmp;
            // repeat counts per sample, then the row counters (kStatReplicas)
            const uint64_t ndup = (uint64_t)std::max<int32_t>(n, 1);
            dupc.alloc(ndup + kStatReplicas, s, tb, true, "repeat counts");
            unsigned long long *rowsrep = dupc.p + ndup;
            cnt.alloc(3 * nlc, s, tb, true, "range counts");
            rid_g.alloc(N / 2 + 1, s, tb, true, "row ids (by range)");
            {
                JAS_TIMED("fill_u64", s);
                k_fill_u64<<<64, 256, 0, s>>>((uint64_t *)dupc.p, ndup + kStatReplicas, 0);
            }
            // shared pairs at the range starts in the first half of the free sort
            // buffer, row pointers (relative to the range) after it
            uint32_t *Sg = reinterpret_cast<uint32_t *>(alt.p);
            uint64_t *rptr_g = alt.p + div_up(N, 2);
            {
                JAS_TIMED(herr & 16u ? "local_cls_wide" : "local_cls", s);
                launch_local_cls((herr & 16u) != 0, cap, (uint32_t)nlc, s, keys.p, sbits, smask, bsh, lowbits,
                                 (const uint64_t *)rs.p, (uint32_t)nlc, cnt.p, keep ? 1 : 0, Sg, rid_g.p, rptr_g,
                                 dupc.p, rowsrep, (const uint64_t *)nullptr, (uint64_t)0, errL);
                k_sum_replicas<<<1, 64, 0, s>>>(rowsrep, kStatReplicas, st.p + ST_ROWS);
            }
            check_launch("local classify");
            offD.alloc(nlc + 1, s, tb, true, "range offsets");
            offS.alloc(nlc + 1, s, tb, true, "range offsets");
            offR.alloc(nlc + 1, s, tb, true, "range offsets");
            stmp.alloc(scan_tmp_elems(nlc), s, tb, true, "scan scratch");
            scan_excl_u32(cnt.p, offD.p, nlc, stmp.p, s);
            scan_excl_u32(cnt.p + nlc, offS.p, nlc, stmp.p, s);
            scan_excl_u32(cnt.p + 2 * nlc, offR.p, nlc, stmp.p, s);
            uint64_t t3[3];
            JAS_HIP(hipMemcpyAsync(&t3[0], offD.p + nlc, 8, hipMemcpyDeviceToHost, s));
            JAS_HIP(hipMemcpyAsync(&t3[1], offS.p + nlc, 8, hipMemcpyDeviceToHost, s));
            JAS_HIP(hipMemcpyAsync(&t3[2], offR.p + nlc, 8, hipMemcpyDeviceToHost, s));
            JAS_HIP(hipMemcpyAsync(&herr, flags.p, sizeof(uint64_t), hipMemcpyDeviceToHost, s));
            JAS_HIP(hipStreamSynchronize(s));
            if (herr & 8u) fail(JAS_EDEVICE, "local classify: a range exceeds the kernel's capacity");
            NDk = t3[0];
            NS = t3[1];
            R = t3[2];
            db->trace.local = true;
            db->trace.wide = (herr & 16u) != 0;
            db->trace.nlc = nlc;
            if (keep) Dk.alloc(NDk, s, &db->budget, false, "query index keys");
            rid_own.alloc(R, s, tb, true, "row ids");
            rptr_own.alloc(R + 1, s, tb, true, "row pointers");
            rdeg_own.alloc(R + 1, s, tb, true, "row degrees");
            Sp = Sg;  // the shared pairs stay in the ranges' stretches
            ridp = rid_own.p;
            rptrp = rptr_own.p;
            rdegp = rdeg_own.p;
            {
                JAS_TIMED("local_move", s);
                k_local_move<<<(uint32_t)std::min<uint64_t>(nlc, 65536), 256, 0, s>>>(
                    rs.p, nlc, offD.p, offS.p, offR.p, keys.p, rid_g.p, rptr_g, keep ? Dk.p : nullptr, ridp, rptrp,
                    rdegp, nullptr, 0);
            }
            check_launch("local move");
            {
                JAS_TIMED("card", s);
                k_card_from_dups<<<(uint32_t)std::max<uint64_t>(1, std::min<uint64_t>(div_up(n, 256), 1024)), 256, 0,
                                   s>>>(offsets, dupc.p, n, cardc.p);
            }
            check_launch("column sums");
            done = true;
        }
    }

    // --- otherwise: sort every ID bit, classify with neighbours in global memory
    if (!done) {
        JAS_HOST_TIMED("classify_fallback");
        {
            RadixWork rw;
            radix_sort_u64(keys, alt, N, sbits, sbits + db->U, rw, s, tb);
        }
        const uint64_t *K = keys.p;
        const uint64_t nch = div_up(N, kChunk);
        DevBuf<uint32_t> cnt;
        DevBuf<uint64_t> offD, offS, offR, stmp;
        cnt.alloc(3 * nch, s, tb, true, "classify counts");
        const int lds_hist = n <= kHistMax;
        const size_t shmem = lds_hist ? (size_t)n * sizeof(uint32_t) : 0;
        {
            JAS_TIMED("cls_count", s);
            k_cls_count<<<(uint32_t)nch, kNT, shmem, s>>>(K, N, sbits, smask, n, lds_hist, cnt.p, cnt.p + nch,
                                                          cnt.p + 2 * nch, cardc.p, st.p);
        }
        check_launch("classify count");
        offD.alloc(nch + 1, s, tb, true, "classify offsets");
        offS.alloc(nch + 1, s, tb, true, "classify offsets");
        offR.alloc(nch + 1, s, tb, true, "classify offsets");
        stmp.alloc(scan_tmp_elems(nch), s, tb, true, "scan scratch");
        scan_excl_u32(cnt.p, offD.p, nch, stmp.p, s);
        scan_excl_u32(cnt.p + nch, offS.p, nch, stmp.p, s);
        scan_excl_u32(cnt.p + 2 * nch, offR.p, nch, stmp.p, s);
        uint64_t t3[3];
        JAS_HIP(hipMemcpyAsync(&t3[0], offD.p + nch, 8, hipMemcpyDeviceToHost, s));
        JAS_HIP(hipMemcpyAsync(&t3[1], offS.p + nch, 8, hipMemcpyDeviceToHost, s));
        JAS_HIP(hipMemcpyAsync(&t3[2], offR.p + nch, 8, hipMemcpyDeviceToHost, s));
        JAS_HIP(hipStreamSynchronize(s));
        NDk = t3[0];
        NS = t3[1];
        R = t3[2];
        if (keep) Dk.alloc(NDk, s, &db->budget, false, "query index keys");
        S_own.alloc(NS, s, tb, true, "shared pairs");
        rid_own.alloc(R, s, tb, true, "row ids");
        rptr_own.alloc(R + 1, s, tb, true, "row pointers");
        Sp = S_own.p;
        ridp = rid_own.p;
        rptrp = rptr_own.p;
        {
            JAS_TIMED("cls_write", s);
            k_cls_write<<<(uint32_t)nch, kNT, 0, s>>>(K, N, sbits, smask, offD.p, offS.p, offR.p,
                                                      keep ? Dk.p : nullptr, Sp, ridp, rptrp);
        }
        check_launch("classify write");
    }
    if (N > 0) {
        JAS_TIMED("fill_u64", s);
        k_fill_u64<<<1, 1, 0, s>>>(rptrp + R, 1, NS);
    }
    check_launch("fill");
    if (!rdegp) {  // the global classification wrote the rows contiguously
        rdeg_own.alloc(R + 1, s, tb, true, "row degrees");
        rdegp = rdeg_own.p;
        launch_1d(std::max<uint64_t>(R, 1), s, [&](uint32_t b, hipStream_t st_) {
            JAS_TIMED("row_deg", st_);
            k_row_deg<<<b, 256, 0, st_>>>(rptrp, R, rdegp);
        });
        check_launch("row degrees");
    }

    // column sums -> |X_i| (int32 B needs every |X_i| < 2^31)
    db->card.alloc(std::max<int32_t>(n, 1), s, &db->budget, false, "card");
    if (n > 0) {
        std::vector<uint64_t> hc(n);
        JAS_HIP(hipMemcpyAsync(hc.data(), cardc.p, sizeof(uint64_t) * n, hipMemcpyDeviceToHost, s));
        JAS_HIP(hipStreamSynchronize(s));
        const uint64_t lim = card_limit();
        for (int32_t i = 0; i < n; ++i)
            if (hc[i] >= lim)
                fail(JAS_EOVERFLOW, "sample " + std::to_string(i) + " has " + std::to_string(hc[i]) +
                                        " distinct IDs (limit " + std::to_string(lim - 1) + ")");
        JAS_HIP(hipMemcpyAsync(db->card.p, cardc.p, sizeof(int64_t) * n, hipMemcpyDeviceToDevice, s));
    }
    cardc.release();

    // --- split rows by degree ------------------------------------------------
    uint64_t QD = 0, QL = 0;
    DevBuf<uint64_t> Drow, Lrow;
    if (R > 0 && !query_only && db->dmin == 0) {
        // choose the degree threshold from the row degree histogram
        JAS_HOST_TIMED("choose_dmin");
        const uint32_t nb = (uint32_t)n + 2;
        DevBuf<unsigned long long> hist;
        hist.alloc(nb, s, tb, true, "degree histogram");
        k_fill_u64<<<64, 256, 0, s>>>((uint64_t *)hist.p, nb, 0);
        const int lds = nb <= 16384;
        const uint32_t blocks = (uint32_t)std::min<uint64_t>(div_up(R, 256), 2048);
        {
            JAS_TIMED("deg_hist", s);
            k_deg_hist<<<blocks, kNT, lds ? nb * sizeof(uint32_t) : 0, s>>>(rdegp, R, nb, lds, hist.p);
        }
        check_launch("degree histogram");
        std::vector<uint64_t> hh(nb);
        JAS_HIP(hipMemcpyAsync(hh.data(), hist.p, nb * sizeof(uint64_t), hipMemcpyDeviceToHost, s));
        JAS_HIP(hipStreamSynchronize(s));
        size_t free_b = 0, total_b = 0;
        if (hipMemGetInfo(&free_b, &total_b) != hipSuccess) {
            (void)hipGetLastError();
            free_b = 0;
        }
        uint64_t cap = free_b ? (uint64_t)free_b / 2 : ~0ull;
        if (tb->limit) cap = std::min<uint64_t>(cap, tb->limit / 2);
        const uint32_t bb = db->batch_bits, U = db->U;
        const uint64_t nbatches = (U - bb >= 63) ? ~0ull : (uint64_t(1) << (U - bb));
        db->dmin = choose_dense_min_degree(hh, (uint32_t)n, nbatches, cap);
    }
    db->stats.dense_min_degree = db->dmin;
    if (R > 0 && !query_only) {
        const uint64_t nt = div_up(R, kSplitTile);
        if (nt > 0xFFFFFFFFull) fail(JAS_EUNSUPPORTED, "too many rows");
        DevBuf<uint32_t> tcnt;
        DevBuf<uint64_t> toff, tmp, lprep;
        tcnt.alloc(nt, s, tb, true, "row tile counts");
        lprep.alloc(kStatReplicas, s, tb, true, "list pair counters");
        {
            JAS_TIMED("fill_u64", s);
            k_fill_u64<<<1, 64, 0, s>>>(lprep.p, kStatReplicas, 0);
        }
        toff.alloc(nt + 1, s, tb, true, "row tile offsets");
        tmp.alloc(scan_tmp_elems(nt), s, tb, true, "scan scratch");
        {
            JAS_TIMED("row_count", s);
            k_row_count<<<(uint32_t)nt, kNT, 0, s>>>(rdegp, R, db->dmin, tcnt.p,
                                                      reinterpret_cast<unsigned long long *>(lprep.p), nullptr);
            k_sum_replicas<<<1, 64, 0, s>>>(reinterpret_cast<const unsigned long long *>(lprep.p), kStatReplicas,
                                            st.p + ST_LISTPAIRS);
        }
        check_launch("row count");
        scan_excl_u32(tcnt.p, toff.p, nt, tmp.p, s);
        QD = to_host_u64(toff.p + nt, s);
        QL = R - QD;
        // when every shared row is of one form the split is the identity: the
        // kernels take a null Drow / Lrow as row q = q
        if (QD > 0 && QL > 0) {
            Drow.alloc(QD, s, tb, true, "packed rows");
            Lrow.alloc(QL, s, tb, true, "list rows");
            {
                JAS_TIMED("row_split", s);
                k_row_split<<<(uint32_t)nt, kNT, 0, s>>>(rdegp, R, db->dmin, toff.p, Drow.p, Lrow.p, nullptr);
            }
            check_launch("row split");
        }
    }

    // --- row lists, first part -------------------------------------------------
    // Up to kSampleMajorMaxN samples: the rows' pairs, sorted by their smaller
    // sample, straight from the shared pairs.  Otherwise (or if that sort
    // cannot run) the rows as a CSR of samples, summed pair by pair.  The
    // pairs are emitted and sorted on a side stream while the packed rows are
    // packed on s (the two read the same rows and write different arrays); s
    // waits for the side stream before anything of the pair path is freed or
    // read.
    db->n_list = QL;
    bool pairs_done = false;
    const bool pair_form = QL > 0 && n <= kSampleMajorMaxN;
    DevBuf<uint64_t> npo;
    DevBuf<uint32_t> pk, palt, perr;
    DevBuf<unsigned long long> pgh;
    uint64_t P = 0;
    uint32_t psb = 0, pwidth = 0;
    hipStream_t s2 = nullptr;
    StreamJoin join;  // after the buffers: on an error s waits for s2 before they are freed
    if (pair_form) {
        // pairs per group of 64 list rows (one wave of the emission), scanned
        const uint64_t nw = div_up(QL, (uint64_t)kWave);
        DevBuf<uint64_t> np, tmp2;
        np.alloc(nw, s, tb, true, "row group pair counts");
        launch_1d(QL, s, [&](uint32_t b, hipStream_t st_) {
            {
                JAS_TIMED("list_npairs", st_);
                k_list_wave_pairs<<<b, 256, 0, st_>>>(Lrow.p, rdegp, QL, np.p, nullptr);
            }
        });
        check_launch("row pair counts");
        npo.alloc(nw + 1, s, tb, true, "row group pair offsets");
        tmp2.alloc(scan_tmp_elems(nw), s, tb, true, "scan scratch");
        scan_excl_u64(np.p, npo.p, nw, tmp2.p, s);
        P = to_host_u64(npo.p + nw, s);
        np.release();
        tmp2.release();
        psb = std::max<uint32_t>(1, ceil_log2_u64((uint64_t)n));
        const uint32_t npass = (psb + 7) / 8;
        pwidth = (psb + npass - 1) / npass;
        if (npass > kPairPasses) fail(JAS_EUNSUPPORTED, "row-list pairs: too many sample bits");
        pk.alloc(P + 2, s, &db->budget, false, "row-list pairs");
        palt.alloc(P + 2, s, tb, true, "row-list pairs (second buffer)");
        pgh.alloc((uint64_t)kGhistReplicas * kMaxPasses * 256, s, tb, true, "pair digit totals");
        perr.alloc(2, s, tb, true, "pair sort flag");
        s2 = side_stream();
        stream_after(s2, s);  // everything the pair path reads is on s so far
        join.waiter = s;
        join.on = s2;
        {
            JAS_TIMED("fill_u64", s2);
            k_fill_u64<<<64, 256, 0, s2>>>((uint64_t *)pgh.p, (uint64_t)kGhistReplicas * kMaxPasses * 256, 0);
            k_fill_u64<<<1, 64, 0, s2>>>((uint64_t *)perr.p, 1, 0);
        }
        {
            JAS_TIMED("pair_emit", s2);
            k_pair_emit<<<(uint32_t)std::min<uint64_t>(div_up(QL, 256), 8192), 256, 0, s2>>>(
                Lrow.p, rptrp, rdegp, Sp, QL, npo.p, pk.p, npass, pwidth, pgh.p, nullptr);
        }
        check_launch("pair emit");
    }

    // --- packed rows: batches, word rows, pack -------------------------------
    const uint64_t ldw = div_up((uint64_t)std::max<int32_t>(n, 1), 128) * 128;
    const uint32_t wb = db->word_bits;
    uint64_t nb = 0, H = 0, Hw = 0;  // rows of W (64-bit), word rows of wb bits
    if (QD > 0) {
        DevBuf<uint32_t> bs;
        DevBuf<uint64_t> bpos, bq, nw, wbase, tmp, wq0, wq1;
        bs.alloc(QD, s, tb, true, "batch flags");
        const uint32_t bbits = db->batch_bits;
        launch_1d(QD, s, [&](uint32_t b, hipStream_t st_) {
            {
                JAS_TIMED("batch_flag", st_);
                k_batch_flag<<<b, 256, 0, st_>>>(Drow.p, ridp, QD, bbits, bs.p, nullptr);
            }
        });
        check_launch("batch flags");
        bpos.alloc(QD + 1, s, tb, true, "batch scan");
        tmp.alloc(scan_tmp_elems(QD), s, tb, true, "scan scratch");
        scan_excl_u32(bs.p, bpos.p, QD, tmp.p, s);
        nb = to_host_u64(bpos.p + QD, s);
        bq.alloc(nb + 1, s, tb, true, "batch starts");
        launch_1d(QD, s, [&](uint32_t b, hipStream_t st_) { { JAS_TIMED("batch_start", st_); k_batch_start<<<b, 256, 0, st_>>>(bs.p, bpos.p, QD, bq.p, nullptr); } });
        {
            JAS_TIMED("fill_u64", s);
            k_fill_u64<<<1, 1, 0, s>>>(bq.p + nb, 1, QD);
        }
        check_launch("batch starts");
        nw.alloc(nb, s, tb, true, "batch words");
        launch_1d(nb, s, [&](uint32_t b, hipStream_t st_) { { JAS_TIMED("batch_words", st_); k_batch_words<<<b, 256, 0, st_>>>(bq.p, nb, wb, nw.p, nullptr); } });
        check_launch("batch words");
        wbase.alloc(nb + 1, s, tb, true, "word bases");
        tmp.release();
        tmp.alloc(scan_tmp_elems(nb), s, tb, true, "scan scratch");
        scan_excl_u64(nw.p, wbase.p, nb, tmp.p, s);
        Hw = to_host_u64(wbase.p + nb, s);
        H = wb == 64 ? Hw : div_up(Hw, 2);
        wq0.alloc(Hw, s, tb, true, "word rows");
        wq1.alloc(Hw, s, tb, true, "word rows");
        launch_1d(QD, s, [&](uint32_t b, hipStream_t st_) {
            {
                JAS_TIMED("word_rows", st_);
                k_word_rows<<<b, 256, 0, st_>>>(QD, bpos.p, bq.p, wbase.p, wb, wq0.p, wq1.p, nullptr);
            }
        });
        check_launch("word rows");
        db->W.alloc(H * ldw, s, &db->budget, false, "packed words");
        // column chunks of equal size (multiples of 128): fewer LDS bytes per
        // block than a full kPackCols chunk when ldw is not a multiple of it
        const uint64_t nchunk = div_up(ldw, (uint64_t)kPackCols);
        const uint32_t cols = (uint32_t)(div_up(div_up(ldw, nchunk), 128) * 128);
        const uint32_t grid = (uint32_t)std::min<uint64_t>(H, 4096);
        {
            JAS_TIMED("pack", s);
            k_pack<<<grid, kNT, cols * sizeof(unsigned long long), s>>>(db->W.p, ldw, H, Hw, wb, wq0.p, wq1.p,
                                                                        Drow.p, rptrp, rdegp, Sp, cols, st.p, nullptr);
        }
        check_launch("pack");
    }
    db->H = H;

    // --- row lists, second part: the pair sort (side stream), then s waits --
    if (pair_form) {
        const bool ok = radix_sort_onesweep_u32(pk, palt, P, 16, 16 + psb, pwidth, pgh.p, perr.p, s2, tb);
        uint32_t herr = 0;
        JAS_HIP(hipMemcpyAsync(&herr, perr.p, 4, hipMemcpyDeviceToHost, s2));
        JAS_HIP(hipStreamSynchronize(s2));
        stream_after(s, s2);
        join.waiter = nullptr;
        if (ok && herr == 0) {
            db->n_lpairs = P;
            db->pairs = std::move(pk);
            pairs_done = true;
            db->trace.pairs = true;
            db->trace.P = P;
        }
    }
    if (QL > 0 && !pairs_done) {
        db->list_ptr.alloc(QL + 1, s, &db->budget, false, "row list pointers");
        DevBuf<uint64_t> deg, tmp;
        deg.alloc(QL, s, tb, true, "row list degrees");
        launch_1d(QL, s, [&](uint32_t b, hipStream_t st_) { { JAS_TIMED("list_deg", st_); k_list_deg<<<b, 256, 0, st_>>>(Lrow.p, rdegp, QL, deg.p); } });
        check_launch("list degrees");
        tmp.alloc(scan_tmp_elems(QL), s, tb, true, "scan scratch");
        scan_excl_u64(deg.p, db->list_ptr.p, QL, tmp.p, s);
        db->list_nnz = to_host_u64(db->list_ptr.p + QL, s);
        db->list_smp.alloc(db->list_nnz, s, &db->budget, false, "row list samples");
        launch_1d(QL, s, [&](uint32_t b, hipStream_t st_) {
            {
                JAS_TIMED("list_gather", st_);
                k_list_gather<<<b, 256, 0, st_>>>(Lrow.p, rptrp, rdegp, Sp, db->list_ptr.p, QL, db->list_smp.p);
            }
        });
        check_launch("list gather");
    } else {
        db->list_ptr.alloc(1, s, &db->budget, false, "row list pointers");
        {
            JAS_TIMED("fill_u64", s);
            k_fill_u64<<<1, 1, 0, s>>>(db->list_ptr.p, 1, 0);
        }
        db->list_nnz = 0;
        db->list_smp.alloc(1, s, &db->budget, false, "row list samples");
    }

    // --- query index -----------------------------------------------------------
    if (keep) {
        db->n_keys = NDk;
        uint32_t ib = ceil_log2_u64(div_up(std::max<uint64_t>(NDk, 1), 32));
        ib = std::max<uint32_t>(1, std::min<uint32_t>(ib, std::min<uint32_t>(db->U, 26)));
        db->ibits = ib;
        const uint64_t nbk = uint64_t(1) << ib;
        db->bucket.alloc(nbk + 1, s, &db->budget, false, "query buckets");
        if (NDk == 0) {
            {
                JAS_TIMED("fill_u64", s);
                k_fill_u64<<<64, 256, 0, s>>>(db->bucket.p, nbk + 1, 0);
            }
            db->keys.alloc(1, s, &db->budget, false, "query index keys");
        } else {
            launch_1d(NDk + 1, s, [&](uint32_t b, hipStream_t st_) {
                {
                    JAS_TIMED("bucket", st_);
                    k_bucket<<<b, 256, 0, st_>>>(Dk.p, NDk, sbits, db->U - ib, nbk, db->bucket.p);
                }
            });
            db->keys = std::move(Dk);
        }
        check_launch("query buckets");
    }

    // --- stats -----------------------------------------------------------------
    uint64_t hst[ST_N];
    JAS_HIP(hipMemcpyAsync(hst, st.p, sizeof(hst), hipMemcpyDeviceToHost, s));
    JAS_HIP(hipStreamSynchronize(s));
    jas_encode_stats &o = db->stats;
    db->trace.N = N;
    db->trace.ND = NDk;
    db->trace.NS = NS;
    db->trace.R = R;
    db->trace.QD = QD;
    db->trace.QL = QL;
    db->trace.nb = nb;
    db->trace.Hw = Hw;
    db->trace.H = H;
    o.n_ids = N;
    o.n_pairs = NDk;
    o.n_rows = hst[ST_ROWS];
    o.n_shared_rows = R;
    o.n_packed_rows = QD;
    o.n_list_rows = QL;
    o.n_batches = nb;
    o.n_word_rows = Hw;
    o.word_bits = wb;
    o.w_rows = H;
    o.w_stride = ldw;
    o.n_list_pairs = db->n_lpairs;
    o.nnz_words = hst[ST_NNZW];
    o.word_pairs_F = hst[ST_F];
    o.list_pairs = hst[ST_LISTPAIRS];
    o.device_bytes = db->budget.held;
    set_tile_stats(o, (uint64_t)n);
}

// The encode of a plan: the common path of jas_encode (single-pass scatters
// on the top ID bits, ranges finished in LDS with the planned stride and key
// width, the planned degree threshold, row lists as sorted pair words), every
// size read from device memory and every buffer the plan's own.  Nothing is
// read back and nothing allocated, so the whole sequence can be captured in a
// HIP graph; what the eager path would have done differently (a fallback) or
// a size above its capacity is flagged in p.err and reported afterwards.
void encode_planned(PlanState &p, const uint64_t *ids, const uint64_t *offsets, hipStream_t s) {
    const int32_t n = p.n;
    const uint32_t sbits = p.sbits, U = p.U;
    const uint64_t smask = sbits ? ((uint64_t(1) << sbits) - 1) : 0;
    uint64_t *dsz = p.dsz.p;
    uint32_t *err = p.err.p;
    const uint64_t Ncap = p.Ncap;
    auto fill = [&](void *ptr, uint64_t words) {
        JAS_TIMED("fill_u64", s);
        k_fill_u64<<<(uint32_t)std::max<uint64_t>(1, std::min<uint64_t>(div_up(words, 256), 1024)), 256, 0, s>>>(
            (uint64_t *)ptr, words, 0);
    };
    {
        JAS_TIMED("plan_sizes", s);
        k_plan_begin<<<1, 1, 0, s>>>(offsets, n, Ncap, dsz, err);
    }
    fill(p.ghist.p, (uint64_t)kGhistReplicas * kMaxPasses * 256);
    fill(p.st.p, ST_N);
    fill(p.dupc.p, (uint64_t)std::max<int32_t>(n, 1) + kStatReplicas);
    fill(p.lprep.p, kStatReplicas);
    check_launch("plan begin");
    // keys and the global sort on the top ID bits
    const uint64_t hi_mask = U >= 64 ? 0 : ~((uint64_t(1) << U) - 1);
    if (p.sort.top_bits > 0) {  // the sort's first pass forms the keys
        JAS_TIMED("count_digits", s);
        k_count_digits<<<(uint32_t)div_up(Ncap, kChunk), kNT, 0, s>>>(ids, Ncap, hi_mask, err, p.sort.npass,
                                                                       U - p.sort.top_bits, p.sort.width, p.ghist.p,
                                                                       dsz);
    } else {
        JAS_TIMED("build_keys", s);
        k_build_keys<<<(uint32_t)div_up(Ncap, kChunk), kNT, 0, s>>>(ids, offsets, n, Ncap, sbits, hi_mask, p.keys.p,
                                                                     err, p.sort.npass, U - p.sort.top_bits,
                                                                     p.sort.width, p.ghist.p, dsz);
    }
    check_launch("build keys (planned)");
    uint64_t *K = p.keys.p, *F = p.alt.p;
    if (p.sort.top_bits > 0) {
        OnesweepBufs ob;
        ob.gstart = p.os_gstart.p;
        ob.maxima = p.os_maxima.p;
        ob.status = p.os_status.p;
        ob.ticket = p.os_ticket.p;
        ob.status_words = p.os_status.n;
        KeySource src;
        src.ids = ids;
        src.off = offsets;
        src.n = n;
        src.sbits = sbits;
        src.tinfo = p.os_tinfo.p;
        src.tinfo_words = p.os_tinfo.n;
        const uint32_t lo = sbits + U - p.sort.top_bits, hi = sbits + U;
        radix_sort_onesweep_planned(K, F, dsz + PZ_N, Ncap, lo, hi, p.sort.width, p.ghist.p, err, ob, s, &src);
    }
    // ranges of whole buckets, finished in LDS
    const uint32_t lowbits = U - p.sort.top_bits;
    const uint32_t bsh = sbits + lowbits;
    const uint64_t nlc = p.nlc_cap;
    {
        JAS_TIMED("range_starts", s);
        k_range_starts<<<(uint32_t)div_up(nlc + 1, 256 / kWave), 256, 0, s>>>(K, Ncap, bsh, p.stride, nlc, p.rs.p,
                                                                               err, dsz, p.lcap);
        k_range_check<<<(uint32_t)std::max<uint64_t>(1, std::min<uint64_t>(div_up(nlc, 256), 4096)), 256, 0, s>>>(
            K, p.rs.p, nlc, bsh, lowbits, sbits, err, dsz, p.stride, p.lcap);  // bit 16 matters only to narrow plans
    }
    check_launch("range starts (planned)");
    const uint64_t ndup = (uint64_t)std::max<int32_t>(n, 1);
    unsigned long long *rowsrep = p.dupc.p + ndup;
    uint32_t *Sg = reinterpret_cast<uint32_t *>(F);
    uint64_t *rptr_g = F + div_up(Ncap, 2);
    {
        JAS_TIMED(p.wide ? "local_cls_wide" : "local_cls", s);
        launch_local_cls(p.wide, p.lcap, (uint32_t)nlc, s, K, sbits, smask, bsh, lowbits, (const uint64_t *)p.rs.p,
                         (uint32_t)nlc, p.cnt.p, 0, Sg, p.rid_g.p, rptr_g, p.dupc.p, rowsrep, dsz, p.stride, err);
        k_sum_replicas<<<1, 64, 0, s>>>(rowsrep, kStatReplicas, p.st.p + ST_ROWS);
    }
    check_launch("local classify (planned)");
    scan_excl_u32(p.cnt.p, p.offD.p, nlc, p.stmp.p, s);
    scan_excl_u32(p.cnt.p + nlc, p.offS.p, nlc, p.stmp.p, s);
    scan_excl_u32(p.cnt.p + 2 * nlc, p.offR.p, nlc, p.stmp.p, s);
    {
        JAS_TIMED("plan_sizes", s);
        k_plan_rows<<<1, 1, 0, s>>>(p.offR.p, p.offS.p, nlc, p.Rcap, p.rptr.p, dsz, err);
    }
    {
        JAS_TIMED("local_move", s);
        k_local_move<<<(uint32_t)std::min<uint64_t>(nlc, 65536), 256, 0, s>>>(
            p.rs.p, nlc, p.offD.p, p.offS.p, p.offR.p, K, p.rid_g.p, rptr_g, nullptr, p.rid.p, p.rptr.p, p.rdeg.p, dsz,
            p.stride);
    }
    {
        JAS_TIMED("card", s);
        k_card_from_dups<<<(uint32_t)std::max<uint64_t>(1, std::min<uint64_t>(div_up(n, 256), 1024)), 256, 0, s>>>(
            offsets, p.dupc.p, n, reinterpret_cast<unsigned long long *>(p.card.p));
        k_plan_card<<<(uint32_t)std::max<uint64_t>(1, std::min<uint64_t>(div_up(n, 256), 1024)), 256, 0, s>>>(
            p.card.p, n, (int64_t)card_limit(), err);
    }
    check_launch("local move (planned)");
    // rows by degree
    {
        JAS_TIMED("row_count", s);
        k_row_count<<<(uint32_t)p.tile_cap, kNT, 0, s>>>(p.rdeg.p, p.Rcap, p.dmin, p.tcnt.p, p.lprep.p, dsz);
        k_sum_replicas<<<1, 64, 0, s>>>(p.lprep.p, kStatReplicas, p.st.p + ST_LISTPAIRS);
    }
    scan_excl_u32(p.tcnt.p, p.toff.p, p.tile_cap, p.stmp.p, s);
    {
        JAS_TIMED("plan_sizes", s);
        k_plan_split<<<1, 1, 0, s>>>(p.toff.p, p.tile_cap, p.QDcap, p.QLcap, dsz, err);
    }
    {
        JAS_TIMED("row_split", s);
        k_row_split<<<(uint32_t)p.tile_cap, kNT, 0, s>>>(p.rdeg.p, p.Rcap, p.dmin, p.toff.p, p.Drow.p, p.Lrow.p, dsz);
    }
    check_launch("row split (planned)");
    // packed rows
    if (p.QDcap > 0) {
        const uint64_t QDc = p.QDcap;
        launch_1d(QDc, s, [&](uint32_t b, hipStream_t st_) {
            JAS_TIMED("batch_flag", st_);
            k_batch_flag<<<b, 256, 0, st_>>>(p.Drow.p, p.rid.p, QDc, p.batch_bits, p.bs.p, dsz);
        });
        scan_excl_u32(p.bs.p, p.bpos.p, QDc, p.stmp.p, s);
        {
            JAS_TIMED("plan_sizes", s);
            k_plan_batches<<<1, 1, 0, s>>>(p.bpos.p, QDc, p.bq.p, dsz);
        }
        launch_1d(QDc, s, [&](uint32_t b, hipStream_t st_) {
            JAS_TIMED("batch_start", st_);
            k_batch_start<<<b, 256, 0, st_>>>(p.bs.p, p.bpos.p, QDc, p.bq.p, dsz);
            k_batch_words<<<b, 256, 0, st_>>>(p.bq.p, QDc, p.word_bits, p.nw.p, dsz);
        });
        scan_excl_u64(p.nw.p, p.wbase.p, QDc, p.stmp.p, s);
        {
            JAS_TIMED("plan_sizes", s);
            k_plan_words<<<1, 1, 0, s>>>(p.wbase.p, QDc, p.word_bits, p.Hwcap, p.Hcap, dsz, err);
        }
        launch_1d(QDc, s, [&](uint32_t b, hipStream_t st_) {
            JAS_TIMED("word_rows", st_);
            k_word_rows<<<b, 256, 0, st_>>>(QDc, p.bpos.p, p.bq.p, p.wbase.p, p.word_bits, p.wq0.p, p.wq1.p, dsz);
        });
        const uint64_t nchunk = div_up(p.ldw, (uint64_t)kPackCols);
        const uint32_t cols = (uint32_t)(div_up(div_up(p.ldw, nchunk), 128) * 128);
        {
            JAS_TIMED("pack", s);
            k_pack<<<(uint32_t)std::min<uint64_t>(p.Hcap, 4096), kNT, cols * sizeof(unsigned long long), s>>>(
                p.W.p, p.ldw, p.Hcap, p.Hwcap, p.word_bits, p.wq0.p, p.wq1.p, p.Drow.p, p.rptr.p, p.rdeg.p,
                reinterpret_cast<const uint32_t *>(F), cols, p.st.p, dsz);
        }
        check_launch("pack (planned)");
    }
    // row lists as pair words sorted by the smaller sample
    if (p.QLcap > 0) {
        const uint64_t QLc = p.QLcap;
        launch_1d(QLc, s, [&](uint32_t b, hipStream_t st_) {
            JAS_TIMED("list_npairs", st_);
            k_list_wave_pairs<<<b, 256, 0, st_>>>(p.Lrow.p, p.rdeg.p, QLc, p.np.p, dsz);
        });
        scan_excl_u64(p.np.p, p.npo.p, p.gcap, p.stmp.p, s);
        {
            JAS_TIMED("plan_sizes", s);
            k_plan_pairs<<<1, 1, 0, s>>>(p.npo.p, p.gcap, p.Pcap, dsz, err);
        }
        fill(p.gh.p, (uint64_t)kGhistReplicas * kMaxPasses * 256);
        {
            JAS_TIMED("pair_emit", s);
            k_pair_emit<<<(uint32_t)std::max<uint64_t>(1, std::min<uint64_t>(div_up(QLc, 256), 8192)), 256, 0, s>>>(
                p.Lrow.p, p.rptr.p, p.rdeg.p, reinterpret_cast<const uint32_t *>(F), QLc, p.npo.p, p.pk.p,
                p.pair_npass, p.pair_width, p.gh.p, dsz);
        }
        check_launch("pair emit (planned)");
        OnesweepBufs ob;
        ob.gstart = p.os2_gstart.p;
        ob.maxima = p.os2_maxima.p;
        ob.status = p.os2_status.p;
        ob.ticket = p.os2_ticket.p;
        ob.status_words = p.os2_status.n;
        uint32_t *a = p.pk.p, *b = p.palt.p;
        radix_sort_onesweep_u32_planned(a, b, dsz + PZ_P, p.Pcap, 16, 16 + p.pair_bits, p.pair_width, p.gh.p, err,
                                        ob, s);
        if (a != p.pairs_final) fail(JAS_EDEVICE, "planned pair sort ended in an unexpected buffer");
    }
}

}  // namespace jas
