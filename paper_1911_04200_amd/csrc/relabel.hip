// Exact relabelling of IDs by rank: every ID becomes its position among the
// distinct IDs of the array.  Equal IDs stay equal and distinct ones stay
// distinct, so every |X_i cap X_j| (and with it B, C and J) is unchanged,
// while the universe shrinks from U bits to ceil(log2 D) bits (D distinct
// IDs).  It lets long k-mers (k = 31: IDs below 2^62, Sec. II-B) go through
// the encoder, whose keys (ID << ceil(log2 n)) | sample must fit 64 bits.
//
//   1. digit totals of every 8-bit pass of the IDs;
//   2. the IDs sorted (single-pass scatters, or the per-pass sort);
//   3. the distinct IDs: head flags, a scan, compaction;
//   4. a table of where each value of the top `ibits` ID bits starts among
//      the distinct IDs, then for every input ID a binary search inside its
//      bucket gives its rank.
#include <algorithm>

#include "device_util.hpp"
#include "jas_internal.hpp"

namespace jas {
namespace {

constexpr int kNT = 256;

__global__ void k_zero_u64(uint64_t *p, uint64_t len) {
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < len; i += (uint64_t)gridDim.x * blockDim.x)
        p[i] = 0;
}
__global__ void k_zero_u32(uint32_t *p) { *p = 0; }

__global__ __launch_bounds__(kNT) void k_id_digits(const uint64_t *__restrict__ ids, uint64_t N, uint32_t npass,
                                                    unsigned long long *__restrict__ ghist) {
    __shared__ uint32_t gh[kMaxPasses][256];
#pragma unroll
    for (int k = 0; k < kMaxPasses; ++k) gh[k][threadIdx.x] = 0;
    __syncthreads();
    for (uint64_t i = (uint64_t)blockIdx.x * kNT + threadIdx.x; i < N; i += (uint64_t)gridDim.x * kNT) {
        const uint64_t id = ids[i];
        for (uint32_t q = 0; q < npass; ++q) atomicAdd(&gh[q][(uint32_t)(id >> (8 * q)) & 255u], 1u);
    }
    __syncthreads();
    unsigned long long *g = ghist + (uint64_t)(blockIdx.x % kGhistReplicas) * kMaxPasses * 256;
    for (uint32_t q = 0; q < npass; ++q)
        if (gh[q][threadIdx.x]) atomicAdd(&g[q * 256 + threadIdx.x], (unsigned long long)gh[q][threadIdx.x]);
}

__global__ void k_check_range(const uint64_t *__restrict__ ids, uint64_t N, uint64_t hi_mask, uint32_t *err) {
    bool bad = false;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < N; i += (uint64_t)gridDim.x * blockDim.x)
        bad |= (ids[i] & hi_mask) != 0;
    if (__ballot(bad) && lane_id() == 0) atomicOr(err, 1u);
}

// head[i] = 1 where sorted[i] starts a new value
__global__ void k_heads(const uint64_t *__restrict__ sorted, uint64_t N, uint32_t *__restrict__ head) {
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < N; i += (uint64_t)gridDim.x * blockDim.x)
        head[i] = i == 0 || sorted[i] != sorted[i - 1];
}

__global__ void k_compact_heads(const uint64_t *__restrict__ sorted, uint64_t N, const uint32_t *__restrict__ head,
                                const uint64_t *__restrict__ pos, uint64_t *__restrict__ distinct) {
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < N; i += (uint64_t)gridDim.x * blockDim.x)
        if (head[i]) distinct[pos[i]] = sorted[i];
}

// bucket[b] = first distinct ID whose top bits (id >> shift) are >= b, b in [0, nbk]
__global__ void k_rank_buckets(const uint64_t *__restrict__ distinct, uint64_t D, uint32_t shift, uint64_t nbk,
                               uint64_t *__restrict__ bucket) {
    for (uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; t <= D; t += (uint64_t)gridDim.x * blockDim.x) {
        const uint64_t bk = t < D ? (distinct[t] >> shift) : nbk;
        const int64_t prev = t == 0 ? -1 : (int64_t)(distinct[t - 1] >> shift);
        for (int64_t b = prev + 1; b <= (int64_t)bk; ++b) bucket[b] = t;
    }
}

// out[i] = rank of ids[i] among the distinct IDs (out may be ids)
__global__ void k_rank(const uint64_t *ids, uint64_t N, const uint64_t *__restrict__ distinct,
                       const uint64_t *__restrict__ bucket, uint32_t shift, uint64_t *out) {
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < N; i += (uint64_t)gridDim.x * blockDim.x) {
        const uint64_t id = ids[i];
        uint64_t a = bucket[id >> shift], b = bucket[(id >> shift) + 1];
        while (a < b) {  // first distinct >= id (it is id: every input ID is among them)
            const uint64_t m = (a + b) >> 1;
            if (distinct[m] < id) a = m + 1;
            else b = m;
        }
        out[i] = a;
    }
}

uint32_t grid_for(uint64_t work) {
    return (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>(div_up(work, 256), 65536));
}

}  // namespace

uint64_t relabel(const uint64_t *ids, uint64_t N, uint32_t U, hipStream_t s, uint64_t *out) {
    if (N == 0) return 0;
    const uint64_t hi_mask = U >= 64 ? 0 : ~((uint64_t(1) << U) - 1);
    DevBuf<uint32_t> err;
    err.alloc(1, s, nullptr, true, "relabel error flag");
    DevBuf<unsigned long long> ghist;
    ghist.alloc((uint64_t)kGhistReplicas * kMaxPasses * 256, s, nullptr, true, "relabel digit totals");
    const uint32_t npass = (U + 7) / 8;
    {
        JAS_TIMED("relabel_digits", s);
        k_zero_u64<<<64, 256, 0, s>>>(reinterpret_cast<uint64_t *>(ghist.p), (uint64_t)kGhistReplicas * kMaxPasses * 256);
        k_zero_u32<<<1, 1, 0, s>>>(err.p);
        k_check_range<<<grid_for(N), 256, 0, s>>>(ids, N, hi_mask, err.p);
        k_id_digits<<<(uint32_t)std::min<uint64_t>(div_up(N, 256 * 16), 8192), kNT, 0, s>>>(ids, N, npass, ghist.p);
    }
    check_launch("relabel digits");
    uint32_t herr = 0;
    JAS_HIP(hipMemcpyAsync(&herr, err.p, 4, hipMemcpyDeviceToHost, s));
    JAS_HIP(hipStreamSynchronize(s));
    if (herr) fail(JAS_EINVAL, "jas_relabel: an ID is >= 2^universe_bits");
    // sort a copy of the IDs
    DevBuf<uint64_t> keys, alt;
    keys.alloc(N, s, nullptr, true, "relabel keys");
    alt.alloc(N, s, nullptr, true, "relabel keys (second buffer)");
    JAS_HIP(hipMemcpyAsync(keys.p, ids, N * 8, hipMemcpyDeviceToDevice, s));
    bool sorted = radix_sort_onesweep(keys, alt, N, 0, U, 8, ghist.p, err.p, s, nullptr);
    if (sorted) {
        JAS_HIP(hipMemcpyAsync(&herr, err.p, 4, hipMemcpyDeviceToHost, s));
        JAS_HIP(hipStreamSynchronize(s));
        sorted = herr == 0;
    }
    if (!sorted) {  // digit totals too large for the single-pass form, or its look-back gave up
        JAS_HIP(hipMemcpyAsync(keys.p, ids, N * 8, hipMemcpyDeviceToDevice, s));
        RadixWork rw;
        radix_sort_u64(keys, alt, N, 0, U, rw, s, nullptr);
    }
    // distinct IDs (in the free buffer)
    DevBuf<uint32_t> head;
    DevBuf<uint64_t> pos, tmp;
    head.alloc(N, s, nullptr, true, "relabel heads");
    pos.alloc(N + 1, s, nullptr, true, "relabel positions");
    tmp.alloc(scan_tmp_elems(N), s, nullptr, true, "scan scratch");
    {
        JAS_TIMED("relabel_unique", s);
        k_heads<<<grid_for(N), 256, 0, s>>>(keys.p, N, head.p);
    }
    scan_excl_u32(head.p, pos.p, N, tmp.p, s);
    {
        JAS_TIMED("relabel_unique", s);
        k_compact_heads<<<grid_for(N), 256, 0, s>>>(keys.p, N, head.p, pos.p, alt.p);
    }
    check_launch("relabel unique");
    uint64_t D = 0;
    JAS_HIP(hipMemcpyAsync(&D, pos.p + N, 8, hipMemcpyDeviceToHost, s));
    JAS_HIP(hipStreamSynchronize(s));
    head.release();
    pos.release();
    tmp.release();
    // ranks through a bucket table of the top ID bits (about 32 distinct IDs per bucket)
    uint32_t ib = ceil_log2_u64(div_up(D, 32));
    ib = std::max<uint32_t>(1, std::min<uint32_t>(ib, std::min<uint32_t>(U, 26)));
    const uint32_t shift = U - ib;
    const uint64_t nbk = uint64_t(1) << ib;
    DevBuf<uint64_t> bucket;
    bucket.alloc(nbk + 1, s, nullptr, true, "relabel buckets");
    {
        JAS_TIMED("relabel_rank", s);
        k_rank_buckets<<<grid_for(D + 1), 256, 0, s>>>(alt.p, D, shift, nbk, bucket.p);
        k_rank<<<grid_for(N), 256, 0, s>>>(ids, N, alt.p, bucket.p, shift, out);
    }
    check_launch("relabel rank");
    JAS_HIP(hipStreamSynchronize(s));
    return D;
}

}  // namespace jas
