// Small device helpers shared by the libjas kernels (wave64, gfx950).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace jas {

constexpr int kWave = 64;

__device__ __forceinline__ uint32_t lane_id() { return threadIdx.x & (kWave - 1); }

__device__ __forceinline__ uint64_t lanemask_lt() {
    const uint32_t l = lane_id();
    return l == 0 ? 0ull : (~0ull >> (64 - l));
}

// Inclusive scan across the 64 lanes of a wave.
__device__ __forceinline__ uint64_t wave_incl_scan(uint64_t v) {
    const uint32_t l = lane_id();
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
        const uint64_t t = __shfl_up(v, d, kWave);
        if (l >= (uint32_t)d) v += t;
    }
    return v;
}

// Exclusive scan of one value per thread across a block of NT threads.
// sh needs NT/64 entries.  Every thread of the block must call it.
template <int NT>
__device__ __forceinline__ uint64_t block_excl_scan(uint64_t v, uint64_t *sh, uint64_t *total) {
    const uint32_t l = lane_id(), w = threadIdx.x / kWave;
    const uint64_t inc = wave_incl_scan(v);
    if (l == kWave - 1) sh[w] = inc;
    __syncthreads();
    uint64_t before = 0, tot = 0;
#pragma unroll
    for (int k = 0; k < NT / kWave; ++k) {
        const uint64_t x = sh[k];
        before += (k < (int)w) ? x : 0;
        tot += x;
    }
    __syncthreads();
    *total = tot;
    return before + inc - v;
}

// Largest s in [lo, hi] with off[s] <= t (CSR sample of entry t).
__device__ __forceinline__ int32_t find_sample(const uint64_t *off, int32_t lo, int32_t hi, uint64_t t) {
    while (lo < hi) {
        const int32_t mid = (lo + hi + 1) >> 1;
        if (off[mid] <= t) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// Position of (i, j), i <= j, in an n x n output: row-major full or packed upper.
__device__ __forceinline__ uint64_t out_index(uint32_t i, uint32_t j, uint32_t n, bool upper) {
    return upper ? (uint64_t)i * n - (uint64_t)i * (i - 1) / 2 + (j - i) : (uint64_t)i * n + j;
}

}  // namespace jas
