// Exclusive prefix sums over device arrays (reduce-then-scan, no inter-block
// waiting): each block scans 4096 entries and records its total, the totals
// are scanned recursively, then added back.
#include "device_util.hpp"
#include "jas_internal.hpp"

namespace jas {
namespace {

constexpr int kNT = 256;
constexpr int kItems = 16;
constexpr uint64_t kBlock = (uint64_t)kNT * kItems;

template <class T>
__global__ __launch_bounds__(kNT) void k_scan_block(const T *in, uint64_t *out, uint64_t len, uint64_t *sums) {
    __shared__ uint64_t stage[kBlock];
    __shared__ uint64_t sh[kNT / kWave];
    const uint64_t b0 = (uint64_t)blockIdx.x * kBlock;
    const uint32_t tid = threadIdx.x;
    // coalesced load into LDS
#pragma unroll
    for (int m = 0; m < kItems; ++m) {
        const uint64_t idx = b0 + (uint64_t)m * kNT + tid;
        stage[m * kNT + tid] = idx < len ? (uint64_t)in[idx] : 0;
    }
    __syncthreads();
    // each thread owns kItems consecutive entries
    uint64_t v[kItems];
    uint64_t s = 0;
#pragma unroll
    for (int m = 0; m < kItems; ++m) {
        v[m] = stage[tid * kItems + m];
        s += v[m];
    }
    uint64_t tot;
    uint64_t run = block_excl_scan<kNT>(s, sh, &tot);
#pragma unroll
    for (int m = 0; m < kItems; ++m) {
        stage[tid * kItems + m] = run;
        run += v[m];
    }
    __syncthreads();
#pragma unroll
    for (int m = 0; m < kItems; ++m) {
        const uint64_t idx = b0 + (uint64_t)m * kNT + tid;
        if (idx < len) out[idx] = stage[m * kNT + tid];
    }
    if (tid == 0) sums[blockIdx.x] = tot;
}

__global__ __launch_bounds__(kNT) void k_scan_add(uint64_t *out, uint64_t len, const uint64_t *sums_ex) {
    const uint64_t b0 = (uint64_t)blockIdx.x * kBlock;
    const uint64_t add = sums_ex[blockIdx.x];
    if (add == 0) return;
#pragma unroll
    for (int m = 0; m < kItems; ++m) {
        const uint64_t idx = b0 + (uint64_t)m * kNT + threadIdx.x;
        if (idx < len) out[idx] += add;
    }
}

__global__ void k_scan_total(uint64_t *out, uint64_t len, const uint64_t *sums, const uint64_t *sums_ex,
                             uint64_t nb) {
    // out[len] = total of all blocks (0 for an empty input)
    out[len] = nb == 0 ? 0 : (sums_ex ? sums_ex[nb] : sums[0]);
}

template <class T>
void scan_impl(const T *in, uint64_t *out, size_t len, uint64_t *tmp, hipStream_t s) {
    if (len == 0) {
        // out[0] = 0
        {
            JAS_TIMED("scan_total", s);
            k_scan_total<<<1, 1, 0, s>>>(out, 0, tmp, nullptr, 0);
        }
        return;
    }
    const uint64_t nb = div_up(len, kBlock);
    uint64_t *sums = tmp;            // nb
    uint64_t *sums_ex = tmp + nb;    // nb + 1
    uint64_t *next_tmp = sums_ex + nb + 1;
    {
        JAS_TIMED("scan_block", s);
        k_scan_block<T><<<(uint32_t)nb, kNT, 0, s>>>(in, out, len, sums);
    }
    check_launch("scan block");
    if (nb == 1) {
        {
            JAS_TIMED("scan_total", s);
            k_scan_total<<<1, 1, 0, s>>>(out, len, sums, nullptr, 1);
        }
        check_launch("scan total");
        return;
    }
    scan_impl<uint64_t>(sums, sums_ex, nb, next_tmp, s);
    {
        JAS_TIMED("scan_add", s);
        k_scan_add<<<(uint32_t)nb, kNT, 0, s>>>(out, len, sums_ex);
    }
    check_launch("scan add");
    {
        JAS_TIMED("scan_total", s);
        k_scan_total<<<1, 1, 0, s>>>(out, len, sums, sums_ex, nb);
    }
    check_launch("scan total");
}

}  // namespace

size_t scan_tmp_elems(size_t len) {
    size_t total = 1;
    while (len > 1) {
        const size_t nb = div_up(len, kBlock);
        total += 2 * nb + 1;
        len = nb;
        if (nb == 1) break;
    }
    return total + 1;
}

void scan_excl_u32(const uint32_t *in, uint64_t *out, size_t len, uint64_t *tmp, hipStream_t s) {
    scan_impl<uint32_t>(in, out, len, tmp, s);
}

void scan_excl_u64(const uint64_t *in, uint64_t *out, size_t len, uint64_t *tmp, hipStream_t s) {
    scan_impl<uint64_t>(in, out, len, tmp, s);
}

}  // namespace jas
