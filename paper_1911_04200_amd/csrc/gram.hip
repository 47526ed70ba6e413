// Gram product B = A^T A on the encoding, and the similarity (Sec. III-A/B).
//
// Packed rows (Eq. (7)):  B_ij += sum_w popcount(W[w][i] & W[w][j]), summed
//   over every word row of every batch (Eq. (4)).  The upper triangle of
//   128 x 128 column tiles is computed; word rows are split into K ranges so
//   the grid fills the chip, and each block adds its tile into B with integer
//   atomics (exact and order independent).
// Row lists: a row shared by d = 2..dmin-1 sets adds 1 to B_ij for each of its
//   d(d-1)/2 pairs i < j (its outer product a_k a_k^T, unpacked).
// Diagonal: B_ii = |X_i| (column sums, Eq. (4)).
// Finalize: C_ij = |X_i| + |X_j| - B_ij, J_ij = B_ij / C_ij, J = 1 if C_ij = 0
//   (Sec. II-A, Eq. (2)); IEEE binary64 division, round to nearest.
#include <algorithm>
#include <vector>

#include <cmath>
#include <map>
#include <mutex>
#include <tuple>

#include "device_util.hpp"
#include "jas_internal.hpp"

namespace jas {
namespace {

constexpr int kNT = 256;
constexpr int kT = 128;   // column tile
constexpr int kKC = 16;   // word rows per LDS stage

__global__ void k_fill_i32(int32_t *p, uint64_t len, int32_t v) {
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < len; i += (uint64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

// The chip's 8 XCDs each have their own L2, and workgroups go to them
// round-robin by linear id (x fastest), so consecutive ids land on different
// XCDs.  Renumbered so that XCD x runs the ids x*per, x*per + 1, ... in turn,
// all tile pairs of one K range run on one XCD and read that range's column
// slabs through its L2 once instead of once per XCD.  A bijection of the
// grid (ids past the last multiple of 8 keep their own number).  Used by the
// 128 x 128 kernels (paperlike fp4: 30.2 -> 4.9 GB fetched, same time); the
// 256 x 256 kernels measured 2-4 % slower with it and keep launch order.
constexpr uint64_t kXcds = 8;
__device__ __forceinline__ void xcd_pair_split(uint32_t &pair, uint64_t &split) {
    const uint64_t nx = gridDim.x, total = nx * gridDim.y;
    const uint64_t L = (uint64_t)blockIdx.y * nx + blockIdx.x;
    const uint64_t per = total / kXcds;
    const uint64_t V = L < per * kXcds ? (L % kXcds) * per + L / kXcds : L;
    pair = (uint32_t)(V % nx);
    split = V / nx;
}

// Thread (ty, tx) of a 16 x 16 grid owns rows 32c + 2ty + e and columns
// 32c + 2tx + e (c = 0..3, e = 0..1) of the 128 x 128 tile: every LDS read is
// a 16-byte load, consecutive lanes read consecutive 16-byte pieces.
__global__ __launch_bounds__(kNT) void k_gram_popc(const uint64_t *__restrict__ W, uint64_t ldw, uint64_t H,
                                                    uint64_t kper, uint32_t nt, uint32_t n,
                                                    int32_t *__restrict__ B, int upper) {
    __shared__ ulonglong2 As[kKC][kT / 2];
    __shared__ ulonglong2 Bs[kKC][kT / 2];
    // the (renumbered) block enumerates the tile pairs I <= J row by row, then the K ranges
    uint32_t p, I = 0, rowlen = nt;
    uint64_t split;
    xcd_pair_split(p, split);
    while (p >= rowlen) {
        p -= rowlen;
        ++I;
        --rowlen;
    }
    const uint32_t Jt = I + p;
    const uint32_t I0 = I * kT, J0 = Jt * kT;
    const uint64_t k0 = split * kper;
    const uint64_t k1 = min(H, k0 + kper);
    if (k0 >= k1) return;
    const uint32_t tid = threadIdx.x, ty = tid >> 4, tx = tid & 15;
    const bool diag = I == Jt;

    uint32_t acc[8][8];
#pragma unroll
    for (int x = 0; x < 8; ++x)
#pragma unroll
        for (int y = 0; y < 8; ++y) acc[x][y] = 0;

    // global -> register staging: 4 x 16 B per matrix per thread
    ulonglong2 ra[4], rb[4];
    auto gload = [&](uint64_t kb) {
#pragma unroll
        for (int m = 0; m < 4; ++m) {
            const uint32_t idx = tid + kNT * m;      // 0..1023
            const uint32_t kk = idx >> 6, cp = idx & 63;
            const uint64_t k = kb + kk;
            if (k < k1) {
                ra[m] = *reinterpret_cast<const ulonglong2 *>(W + k * ldw + I0 + 2 * cp);
                rb[m] = diag ? ra[m] : *reinterpret_cast<const ulonglong2 *>(W + k * ldw + J0 + 2 * cp);
            } else {
                ra[m] = make_ulonglong2(0, 0);
                rb[m] = make_ulonglong2(0, 0);
            }
        }
    };
    auto sstore = [&]() {
#pragma unroll
        for (int m = 0; m < 4; ++m) {
            const uint32_t idx = tid + kNT * m;
            As[idx >> 6][idx & 63] = ra[m];
            Bs[idx >> 6][idx & 63] = rb[m];
        }
    };

    gload(k0);
    for (uint64_t kb = k0; kb < k1; kb += kKC) {
        __syncthreads();
        sstore();
        __syncthreads();
        if (kb + kKC < k1) gload(kb + kKC);
#pragma unroll 4
        for (int kk = 0; kk < kKC; ++kk) {
            uint64_t a[8], b[8];
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                const ulonglong2 va = As[kk][16 * c + ty];
                const ulonglong2 vb = Bs[kk][16 * c + tx];
                a[2 * c] = va.x;
                a[2 * c + 1] = va.y;
                b[2 * c] = vb.x;
                b[2 * c + 1] = vb.y;
            }
#pragma unroll
            for (int x = 0; x < 8; ++x)
#pragma unroll
                for (int y = 0; y < 8; ++y) {
                    const uint64_t v = a[x] & b[y];
                    acc[x][y] += __popc((uint32_t)v) + __popc((uint32_t)(v >> 32));
                }
        }
    }
    // epilogue: add the strict upper part of the tile into B
#pragma unroll
    for (int x = 0; x < 8; ++x) {
        const uint32_t i = I0 + 32 * (x >> 1) + 2 * ty + (x & 1);
#pragma unroll
        for (int y = 0; y < 8; ++y) {
            const uint32_t j = J0 + 32 * (y >> 1) + 2 * tx + (y & 1);
            if (acc[x][y] && i < j && j < n) atomicAdd(B + out_index(i, j, n, upper), (int32_t)acc[x][y]);
        }
    }
}

// ---------------------------------------------------------------------------
// int8 MFMA form of the same product.  Each bit of a packed word becomes a
// 0/1 byte in registers (never in memory; through a 256-entry LDS table of
// byte patterns) and V_MFMA_I32_32X32X32_I8 sums the byte products in int32:
// sum_k a_ki a_kj over the 32 bits of a half word, exact (every partial sum
// is a count <= 2^31).  The K order inside the instruction does not matter:
// lane group g (lanes 32g..32g+31) feeds bits 16g..16g+15 of the half word
// for both operands, so every bit pairs with itself.
// Block = 2 waves over a 128 x 128 tile; wave c owns columns 64c..64c+63,
// i.e. 4 x 2 MFMA tiles of 32 x 32 (128 int32 accumulators per lane).
typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v16i __attribute__((ext_vector_type(16)));

constexpr int kMfmaNT = 128;

// 8 bits -> 8 bytes (byte k = bit k), 256 entries: an operand of 16 bits is
// two table reads instead of a dozen VALU operations.
__device__ __forceinline__ void fill_byte_lut(unsigned long long *lut) {
    for (uint32_t i = threadIdx.x; i < 256; i += blockDim.x) {
        const unsigned long long lo = ((i & 0xFu) * 0x00204081u) & 0x01010101u;
        const unsigned long long hi = (((i >> 4) & 0xFu) * 0x00204081u) & 0x01010101u;
        lut[i] = lo | (hi << 32);
    }
}

__device__ __forceinline__ v4i bits16_lut(const unsigned long long *lut, uint32_t x) {
    const unsigned long long lo = lut[__builtin_amdgcn_ubfe(x, 0, 8)];
    const unsigned long long hi = lut[__builtin_amdgcn_ubfe(x, 8, 8)];
    v4i r;
    r[0] = (int)(uint32_t)lo;
    r[1] = (int)(uint32_t)(lo >> 32);
    r[2] = (int)(uint32_t)hi;
    r[3] = (int)(uint32_t)(hi >> 32);
    return r;
}

// STEP word rows per loop iteration; the next STEP rows are loaded while the
// current ones are multiplied.  WPE = waves per SIMD the register budget is
// sized for (2: 256 VGPRs).
template <int WPE, int STEP>
__global__ __launch_bounds__(kMfmaNT) __attribute__((amdgpu_waves_per_eu(WPE, WPE))) void k_gram_mfma(
    const uint64_t *__restrict__ W, uint64_t ldw, uint64_t H, uint64_t kper, uint32_t nt, uint32_t n,
    int32_t *__restrict__ B, int upper) {
    __shared__ unsigned long long lut[256];
    // the (renumbered) block enumerates the tile pairs I <= J row by row, then the K ranges
    uint32_t p, I = 0, rowlen = nt;
    uint64_t split;
    xcd_pair_split(p, split);
    while (p >= rowlen) {
        p -= rowlen;
        ++I;
        --rowlen;
    }
    const uint32_t Jt = I + p;
    const uint64_t k0 = split * kper;
    const uint64_t k1 = min(H, k0 + kper);
    if (k0 >= k1) return;
    fill_byte_lut(lut);
    __syncthreads();
    const uint32_t lane = threadIdx.x & 63, wc = threadIdx.x >> 6;
    const uint32_t lm = lane & 31, lg = lane >> 5;
    const uint32_t I0 = I * kT, J0 = Jt * kT + 64 * wc;
    v16i acc[4][2];
#pragma unroll
    for (int x = 0; x < 4; ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y)
#pragma unroll
            for (int r = 0; r < 16; ++r) acc[x][y][r] = 0;

    const uint64_t *pa = W + I0 + lm;
    const uint64_t *pb = W + J0 + lm;
    // STEP word rows per iteration; the next STEP rows are loaded while these are multiplied
    uint64_t a[STEP][4], b[STEP][2];
#pragma unroll
    for (int u = 0; u < STEP; ++u) {
        const uint64_t ku = min(k0 + u, k1 - 1);
#pragma unroll
        for (int x = 0; x < 4; ++x) a[u][x] = pa[ku * ldw + 32 * x];
#pragma unroll
        for (int y = 0; y < 2; ++y) b[u][y] = pb[ku * ldw + 32 * y];
    }
    for (uint64_t k = k0; k < k1; k += STEP) {
        uint64_t na[STEP][4], nb[STEP][2];
#pragma unroll
        for (int u = 0; u < STEP; ++u) {
            const uint64_t kn = min(k + STEP + u, k1 - 1);
#pragma unroll
            for (int x = 0; x < 4; ++x) na[u][x] = pa[kn * ldw + 32 * x];
#pragma unroll
            for (int y = 0; y < 2; ++y) nb[u][y] = pb[kn * ldw + 32 * y];
        }
#pragma unroll
        for (int u = 0; u < STEP; ++u) {
            if (k + u >= k1) break;  // wave-uniform: the tail of the range
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const uint32_t sh = 32 * h + 16 * lg;
                v4i va[4], vb[2];
#pragma unroll
                for (int x = 0; x < 4; ++x) va[x] = bits16_lut(lut, (uint32_t)(a[u][x] >> sh));
#pragma unroll
                for (int y = 0; y < 2; ++y) vb[y] = bits16_lut(lut, (uint32_t)(b[u][y] >> sh));
#pragma unroll
                for (int x = 0; x < 4; ++x)
#pragma unroll
                    for (int y = 0; y < 2; ++y)
                        acc[x][y] = __builtin_amdgcn_mfma_i32_32x32x32_i8(va[x], vb[y], acc[x][y], 0, 0, 0);
            }
        }
#pragma unroll
        for (int u = 0; u < STEP; ++u) {
#pragma unroll
            for (int x = 0; x < 4; ++x) a[u][x] = na[u][x];
#pragma unroll
            for (int y = 0; y < 2; ++y) b[u][y] = nb[u][y];
        }
    }
    // accumulator r of lane (lg, lm) holds row 8*(r/4) + 4*lg + r%4, column lm of each 32 x 32 tile
#pragma unroll
    for (int x = 0; x < 4; ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y)
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const uint32_t i = I0 + 32 * x + 8 * (r >> 2) + 4 * lg + (r & 3);
                const uint32_t j = J0 + 32 * y + lm;
                const int32_t v = acc[x][y][r];
                if (v && i < j && j < n) atomicAdd(B + out_index(i, j, n, upper), v);
            }
}

// 256 x 256 tiles: four waves (2 x 2), each a 128 x 128 block of 16 MFMA
// tiles with its accumulators in the AGPRs (one wave per SIMD).  Against the
// 128 x 128 kernel this halves the words loaded per multiply (each column
// slab feeds twice the tiles) and expands 8 operands per 16 MFMAs instead of
// 6 per 8.  Columns at or past ldw (n rounded to 128) are clamped to a valid
// column; their products land outside j < n and are dropped.
constexpr int kWideT = 256;
constexpr int kWideNT = 256;

template <int STEP>
__global__ __launch_bounds__(kWideNT) __attribute__((amdgpu_waves_per_eu(1, 1))) void k_gram_mfma_wide(
    const uint64_t *__restrict__ W, uint64_t ldw, uint64_t H, uint64_t kper, uint32_t nt, uint32_t n,
    int32_t *__restrict__ B, int upper) {
    __shared__ unsigned long long lut[256];
    const uint64_t split = blockIdx.y;
    uint32_t p = blockIdx.x, I = 0, rowlen = nt;
    while (p >= rowlen) {
        p -= rowlen;
        ++I;
        --rowlen;
    }
    const uint32_t Jt = I + p;
    const uint64_t k0 = split * kper;
    const uint64_t k1 = min(H, k0 + kper);
    if (k0 >= k1) return;
    fill_byte_lut(lut);
    __syncthreads();
    const uint32_t lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const uint32_t lm = lane & 31, lg = lane >> 5;
    const uint32_t I0 = I * kWideT + 128 * (wv >> 1), J0 = Jt * kWideT + 128 * (wv & 1);
    if (I0 >= J0 + 128) return;  // the wave's block lies below the diagonal (no syncs follow)
    v16i acc[4][4];
#pragma unroll
    for (int x = 0; x < 4; ++x)
#pragma unroll
        for (int y = 0; y < 4; ++y)
#pragma unroll
            for (int r = 0; r < 16; ++r) acc[x][y][r] = 0;
    uint64_t ca[4], cb[4];  // this lane's columns, clamped below ldw
#pragma unroll
    for (int x = 0; x < 4; ++x) {
        ca[x] = min<uint64_t>(I0 + lm + 32 * x, ldw - 1);
        cb[x] = min<uint64_t>(J0 + lm + 32 * x, ldw - 1);
    }
    uint64_t a[STEP][4], b[STEP][4];
#pragma unroll
    for (int u = 0; u < STEP; ++u) {
        const uint64_t ku = min(k0 + u, k1 - 1);
#pragma unroll
        for (int x = 0; x < 4; ++x) {
            a[u][x] = W[ku * ldw + ca[x]];
            b[u][x] = W[ku * ldw + cb[x]];
        }
    }
    for (uint64_t k = k0; k < k1; k += STEP) {
        uint64_t na[STEP][4], nb[STEP][4];
#pragma unroll
        for (int u = 0; u < STEP; ++u) {
            const uint64_t kn = min(k + STEP + u, k1 - 1);
#pragma unroll
            for (int x = 0; x < 4; ++x) {
                na[u][x] = W[kn * ldw + ca[x]];
                nb[u][x] = W[kn * ldw + cb[x]];
            }
        }
#pragma unroll
        for (int u = 0; u < STEP; ++u) {
            if (k + u >= k1) break;  // wave-uniform: the tail of the range
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const uint32_t sh = 32 * h + 16 * lg;
                v4i va[4], vb[4];
#pragma unroll
                for (int x = 0; x < 4; ++x) va[x] = bits16_lut(lut, (uint32_t)(a[u][x] >> sh));
#pragma unroll
                for (int y = 0; y < 4; ++y) vb[y] = bits16_lut(lut, (uint32_t)(b[u][y] >> sh));
#pragma unroll
                for (int x = 0; x < 4; ++x)
#pragma unroll
                    for (int y = 0; y < 4; ++y)
                        acc[x][y] = __builtin_amdgcn_mfma_i32_32x32x32_i8(va[x], vb[y], acc[x][y], 0, 0, 0);
            }
        }
#pragma unroll
        for (int u = 0; u < STEP; ++u)
#pragma unroll
            for (int x = 0; x < 4; ++x) {
                a[u][x] = na[u][x];
                b[u][x] = nb[u][x];
            }
    }
    // accumulator r of lane (lg, lm) holds row 8*(r/4) + 4*lg + r%4, column lm of each 32 x 32 tile
#pragma unroll
    for (int x = 0; x < 4; ++x)
#pragma unroll
        for (int y = 0; y < 4; ++y)
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const uint32_t i = I0 + 32 * x + 8 * (r >> 2) + 4 * lg + (r & 3);
                const uint32_t j = J0 + 32 * y + lm;
                const int32_t v = acc[x][y][r];
                if (v && i < j && j < n) atomicAdd(B + out_index(i, j, n, upper), v);
            }
}

// The same 128 x 128 tiles on the fp4 form of the scaled MFMA
// (V_MFMA_F32_32X32X64_F8F6F4, both operands e2m1): a bit becomes the nibble
// 0b0010 (1.0) or 0, so one 64-bit word is one K = 64 step (32 bits per lane
// group) and a table of 256 dwords turns 8 bits into 8 nibbles.  The lanes'
// k order is the same for both operands, so the dot product is the popcount
// of the AND.  Products are 0 or 1 and the float32 sums stay below 2^24
// (at most kFp4MaxK word rows per block), so every count is exact.
constexpr uint64_t kFp4MaxK = (1u << 24) / 64 - 1;
typedef int v8i __attribute__((ext_vector_type(8)));
typedef float v16f __attribute__((ext_vector_type(16)));

// The table is held in COPIES copies, entry x of copy c at word COPIES x + c.
// With 32 copies lane l reads copy l % 32, so the lanes of one read fall in
// distinct banks whatever bytes they look up (with one copy, data-dependent
// indices collide in the banks on dense words, but the extra address
// arithmetic costs more than it saves on sparse words and in the 256 x 256
// kernel, so both forms are tile variants).
template <uint32_t COPIES>
__device__ __forceinline__ void fill_nibble_lut(uint32_t *lut) {
    for (uint32_t e = threadIdx.x; e < 256 * COPIES; e += blockDim.x) {
        const uint32_t i = e / COPIES;
        uint32_t d = 0;
        for (int b = 0; b < 8; ++b) d |= ((i >> b) & 1u) << (4 * b + 1);
        lut[e] = d;
    }
}

// lutc: the table copy of this lane (lut + lane % 32 with 32 copies, else lut)
template <uint32_t COPIES>
__device__ __forceinline__ v8i bits32_fp4(const uint32_t *lutc, uint32_t x) {
    v8i r = {0, 0, 0, 0, 0, 0, 0, 0};
    r[0] = (int)lutc[(x & 255u) * COPIES];
    r[1] = (int)lutc[((x >> 8) & 255u) * COPIES];
    r[2] = (int)lutc[((x >> 16) & 255u) * COPIES];
    r[3] = (int)lutc[(x >> 24) * COPIES];
    return r;
}

template <int WPE, int STEP, uint32_t COPIES>
__global__ __launch_bounds__(kMfmaNT) __attribute__((amdgpu_waves_per_eu(WPE, WPE))) void k_gram_fp4(
    const uint64_t *__restrict__ W, uint64_t ldw, uint64_t H, uint64_t kper, uint32_t nt, uint32_t n,
    int32_t *__restrict__ B, int upper) {
    __shared__ uint32_t lut[256 * COPIES];
    uint32_t p, I = 0, rowlen = nt;
    uint64_t split;
    xcd_pair_split(p, split);
    while (p >= rowlen) {
        p -= rowlen;
        ++I;
        --rowlen;
    }
    const uint32_t Jt = I + p;
    const uint64_t k0 = split * kper;
    const uint64_t k1 = min(H, k0 + kper);
    if (k0 >= k1) return;
    fill_nibble_lut<COPIES>(lut);
    __syncthreads();
    const uint32_t lane = threadIdx.x & 63, wc = threadIdx.x >> 6;
    const uint32_t lm = lane & 31, lg = lane >> 5;
    const uint32_t *lutc = lut + (COPIES > 1 ? lm : 0);
    const uint32_t I0 = I * kT, J0 = Jt * kT + 64 * wc;
    v16f acc[4][2];
#pragma unroll
    for (int x = 0; x < 4; ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y)
#pragma unroll
            for (int r = 0; r < 16; ++r) acc[x][y][r] = 0.f;
    const uint64_t *pa = W + I0 + lm;
    const uint64_t *pb = W + J0 + lm;
    uint64_t a[STEP][4], b[STEP][2];
#pragma unroll
    for (int u = 0; u < STEP; ++u) {
        const uint64_t ku = min(k0 + u, k1 - 1);
#pragma unroll
        for (int x = 0; x < 4; ++x) a[u][x] = pa[ku * ldw + 32 * x];
#pragma unroll
        for (int y = 0; y < 2; ++y) b[u][y] = pb[ku * ldw + 32 * y];
    }
    const uint32_t sh = 32 * lg;  // this lane group's half of the word
    for (uint64_t k = k0; k < k1; k += STEP) {
        uint64_t na[STEP][4], nb[STEP][2];
#pragma unroll
        for (int u = 0; u < STEP; ++u) {
            const uint64_t kn = min(k + STEP + u, k1 - 1);
#pragma unroll
            for (int x = 0; x < 4; ++x) na[u][x] = pa[kn * ldw + 32 * x];
#pragma unroll
            for (int y = 0; y < 2; ++y) nb[u][y] = pb[kn * ldw + 32 * y];
        }
#pragma unroll
        for (int u = 0; u < STEP; ++u) {
            if (k + u >= k1) break;  // wave-uniform: the tail of the range
            v8i va[4], vb[2];
#pragma unroll
            for (int x = 0; x < 4; ++x) va[x] = bits32_fp4<COPIES>(lutc, (uint32_t)(a[u][x] >> sh));
#pragma unroll
            for (int y = 0; y < 2; ++y) vb[y] = bits32_fp4<COPIES>(lutc, (uint32_t)(b[u][y] >> sh));
#pragma unroll
            for (int x = 0; x < 4; ++x)
#pragma unroll
                for (int y = 0; y < 2; ++y)
                    acc[x][y] = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(va[x], vb[y], acc[x][y], 4, 4, 0, 0,
                                                                              0, 0);
        }
#pragma unroll
        for (int u = 0; u < STEP; ++u) {
#pragma unroll
            for (int x = 0; x < 4; ++x) a[u][x] = na[u][x];
#pragma unroll
            for (int y = 0; y < 2; ++y) b[u][y] = nb[u][y];
        }
    }
    // accumulator r of lane (lg, lm) holds row 8*(r/4) + 4*lg + r%4, column lm of each 32 x 32 tile
#pragma unroll
    for (int x = 0; x < 4; ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y)
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const uint32_t i = I0 + 32 * x + 8 * (r >> 2) + 4 * lg + (r & 3);
                const uint32_t j = J0 + 32 * y + lm;
                const int32_t v = (int32_t)acc[x][y][r];  // an exact integer below 2^24
                if (v && i < j && j < n) atomicAdd(B + out_index(i, j, n, upper), v);
            }
}

// fp4 on 256 x 256 tiles: the four waves of k_gram_mfma_wide, each 128 x
// 128, with the fp4 step of k_gram_fp4 (one word per MFMA).
template <int STEP>
__global__ __launch_bounds__(kWideNT) __attribute__((amdgpu_waves_per_eu(1, 1))) void k_gram_fp4_wide(
    const uint64_t *__restrict__ W, uint64_t ldw, uint64_t H, uint64_t kper, uint32_t nt, uint32_t n,
    int32_t *__restrict__ B, int upper) {
    __shared__ uint32_t lut[256];
    const uint64_t split = blockIdx.y;
    uint32_t p = blockIdx.x, I = 0, rowlen = nt;
    while (p >= rowlen) {
        p -= rowlen;
        ++I;
        --rowlen;
    }
    const uint32_t Jt = I + p;
    const uint64_t k0 = split * kper;
    const uint64_t k1 = min(H, k0 + kper);
    if (k0 >= k1) return;
    fill_nibble_lut<1>(lut);
    __syncthreads();
    const uint32_t lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const uint32_t lm = lane & 31, lg = lane >> 5;
    const uint32_t I0 = I * kWideT + 128 * (wv >> 1), J0 = Jt * kWideT + 128 * (wv & 1);
    if (I0 >= J0 + 128) return;  // the wave's block lies below the diagonal (no syncs follow)
    v16f acc[4][4];
#pragma unroll
    for (int x = 0; x < 4; ++x)
#pragma unroll
        for (int y = 0; y < 4; ++y)
#pragma unroll
            for (int r = 0; r < 16; ++r) acc[x][y][r] = 0.f;
    uint64_t ca[4], cb[4];  // this lane's columns, clamped below ldw
#pragma unroll
    for (int x = 0; x < 4; ++x) {
        ca[x] = min<uint64_t>(I0 + lm + 32 * x, ldw - 1);
        cb[x] = min<uint64_t>(J0 + lm + 32 * x, ldw - 1);
    }
    uint64_t a[STEP][4], b[STEP][4];
#pragma unroll
    for (int u = 0; u < STEP; ++u) {
        const uint64_t ku = min(k0 + u, k1 - 1);
#pragma unroll
        for (int x = 0; x < 4; ++x) {
            a[u][x] = W[ku * ldw + ca[x]];
            b[u][x] = W[ku * ldw + cb[x]];
        }
    }
    const uint32_t sh = 32 * lg;
    for (uint64_t k = k0; k < k1; k += STEP) {
        uint64_t na[STEP][4], nb[STEP][4];
#pragma unroll
        for (int u = 0; u < STEP; ++u) {
            const uint64_t kn = min(k + STEP + u, k1 - 1);
#pragma unroll
            for (int x = 0; x < 4; ++x) {
                na[u][x] = W[kn * ldw + ca[x]];
                nb[u][x] = W[kn * ldw + cb[x]];
            }
        }
#pragma unroll
        for (int u = 0; u < STEP; ++u) {
            if (k + u >= k1) break;  // wave-uniform: the tail of the range
            v8i va[4], vb[4];
#pragma unroll
            for (int x = 0; x < 4; ++x) va[x] = bits32_fp4<1>(lut, (uint32_t)(a[u][x] >> sh));
#pragma unroll
            for (int y = 0; y < 4; ++y) vb[y] = bits32_fp4<1>(lut, (uint32_t)(b[u][y] >> sh));
#pragma unroll
            for (int x = 0; x < 4; ++x)
#pragma unroll
                for (int y = 0; y < 4; ++y)
                    acc[x][y] = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(va[x], vb[y], acc[x][y], 4, 4, 0, 0,
                                                                              0, 0);
        }
#pragma unroll
        for (int u = 0; u < STEP; ++u)
#pragma unroll
            for (int x = 0; x < 4; ++x) {
                a[u][x] = na[u][x];
                b[u][x] = nb[u][x];
            }
    }
#pragma unroll
    for (int x = 0; x < 4; ++x)
#pragma unroll
        for (int y = 0; y < 4; ++y)
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const uint32_t i = I0 + 32 * x + 8 * (r >> 2) + 4 * lg + (r & 3);
                const uint32_t j = J0 + 32 * y + lm;
                const int32_t v = (int32_t)acc[x][y][r];  // an exact integer below 2^24
                if (v && i < j && j < n) atomicAdd(B + out_index(i, j, n, upper), v);
            }
}

// Row lists: one thread per row, every pair of its (ascending) samples.
__global__ void k_list_pairs(const uint64_t *__restrict__ lp, const uint32_t *__restrict__ ls, uint64_t nl,
                             uint32_t n, int32_t *__restrict__ B, int upper) {
    for (uint64_t r = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; r < nl; r += (uint64_t)gridDim.x * blockDim.x) {
        const uint64_t a0 = lp[r], a1 = lp[r + 1];
        for (uint64_t a = a0; a < a1; ++a) {
            const uint32_t i = ls[a];
            for (uint64_t b = a + 1; b < a1; ++b) atomicAdd(B + out_index(i, ls[b], n, upper), 1);
        }
    }
}

// Row-list pairs sorted by their smaller sample a: block g takes pairs
// [g*chunk, ...); for each run of one a in it, an LDS row cnt[b] counts the
// rows holding both a and b, and each touched counter is added to row a of B
// once (one atomic per touched pair and chunk instead of one per row and
// pair).  Chunks of at least kPairChunk words, about kPairBlocks of them:
// longer chunks split a sample's run fewer times, so fewer atomics.
constexpr uint64_t kPairChunk = 16384;
constexpr uint64_t kPairBlocks = 4096;

constexpr int kPairCountNT = 512;  // threads per pair-count block (one LDS row of counters each)
__global__ __launch_bounds__(kPairCountNT) void k_pair_count(const uint32_t *__restrict__ pairs, uint64_t P, uint64_t chunk,
                                                     uint32_t n, int32_t *__restrict__ B, int upper,
                                                     const uint64_t *__restrict__ dsz) {
    extern __shared__ uint32_t lds[];
    uint32_t *cnt = lds;  // n counters
    // the counters a short run touched (n < 2^16): a short run has fewer than
    // n/8 words, so at most n/8 entries
    uint16_t *touched = reinterpret_cast<uint16_t *>(lds + n);
    __shared__ uint32_t ntouched;
    __shared__ uint64_t seg_end;
    if (dsz) P = min(P, dsz[PZ_P]);  // a plan's db: P is the capacity, the count is on the device
    const uint64_t lo = (uint64_t)blockIdx.x * chunk, hi = min(P, lo + chunk);
    if (lo >= hi) return;
    for (uint32_t i = threadIdx.x; i < n; i += blockDim.x) cnt[i] = 0;
    if (threadIdx.x == 0) ntouched = 0;
    __syncthreads();
    for (uint64_t s0 = lo; s0 < hi;) {
        const uint32_t a = pairs[s0] >> 16;
        // end of the run of a inside the chunk (the chunk is sorted by a): the
        // first wave narrows [l, h] by 64 probes per step; positions before l
        // hold samples <= a, positions from h on samples > a
        if (threadIdx.x < kWave) {
            const uint32_t lane = threadIdx.x;
            uint64_t l = s0 + 1, h = hi;
            while (h - l > kWave) {
                const uint64_t step = (h - l) / kWave;  // >= 1; probe 64 is l + 64*step <= h
                const uint64_t m = l + (lane + 1) * step;
                const uint64_t gt = __ballot(m >= h || (pairs[m] >> 16) > a);
                if (gt == 0) {
                    l = l + kWave * step + 1;
                } else {
                    const uint32_t k = (uint32_t)__builtin_ctzll(gt);  // probe k+1 is the first above
                    h = min(h, l + (k + 1) * step);
                    if (k > 0) l = l + k * step + 1;
                }
            }
            const uint64_t m = l + lane;
            const uint64_t gt = __ballot(m < h && (pairs[m] >> 16) > a);
            if (lane == 0) seg_end = gt ? l + __builtin_ctzll(gt) : h;
        }
        __syncthreads();
        const uint64_t s1 = seg_end;
        // A long run (at least n/8 words) counts without return and then
        // scans its whole LDS row; a short one keeps a list of the counters it
        // touched.  Words are read 16 bytes at a time (four per thread in
        // flight); the buffer is 16-byte aligned, the unaligned ends by word.
        const bool long_run = (s1 - s0) * 8 >= n;  // block-uniform
        auto count = [&](uint32_t w) {
            const uint32_t b = w & 0xFFFFu;
            if (long_run) {
                __hip_atomic_fetch_add(&cnt[b], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            } else if (atomicAdd(&cnt[b], 1u) == 0) {
                touched[atomicAdd(&ntouched, 1u)] = (uint16_t)b;
            }
        };
        const uint64_t va = min(s1, (s0 + 3) & ~uint64_t(3));  // first aligned word (or s1)
        const uint64_t vb = max(va, s1 & ~uint64_t(3));        // end of the aligned body
        for (uint64_t p = s0 + threadIdx.x; p < va; p += blockDim.x) count(pairs[p]);
        for (uint64_t p = vb + threadIdx.x; p < s1; p += blockDim.x) count(pairs[p]);
        const uint4 *pv = reinterpret_cast<const uint4 *>(pairs);
        const uint64_t q1 = vb / 4;
        for (uint64_t q0 = va / 4; q0 < q1; q0 += 4 * (uint64_t)blockDim.x) {
            uint4 x[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const uint64_t q = q0 + (uint64_t)u * blockDim.x + threadIdx.x;
                if (q < q1) x[u] = pv[q];
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                if (q0 + (uint64_t)u * blockDim.x + threadIdx.x < q1) {
                    count(x[u].x);
                    count(x[u].y);
                    count(x[u].z);
                    count(x[u].w);
                }
            }
        }
        __syncthreads();
        if (long_run) {
            for (uint32_t b = a + 1 + threadIdx.x; b < n; b += blockDim.x) {
                const uint32_t c = cnt[b];
                if (c) {
                    atomicAdd(B + out_index(a, b, n, upper), (int32_t)c);
                    cnt[b] = 0;
                }
            }
        } else {
            const uint32_t nt = ntouched;
            for (uint32_t k = threadIdx.x; k < nt; k += blockDim.x) {
                const uint32_t b = touched[k];
                atomicAdd(B + out_index(a, b, n, upper), (int32_t)cnt[b]);
                cnt[b] = 0;
            }
        }
        __syncthreads();
        if (threadIdx.x == 0) ntouched = 0;
        s0 = s1;
        __syncthreads();
    }
}

// Diagonal, mirror (full layout), unions and J.
// dst[i] += src[i], i < n (the sample sizes of one row batch into the running sums).
__global__ void k_add_i64(int64_t *__restrict__ dst, const int64_t *__restrict__ src, uint32_t n) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) dst[i] += src[i];
}

// flag[0] = 1 when some card[i] >= limit.
__global__ void k_card_check(const int64_t *__restrict__ card, uint32_t n, int64_t limit, uint32_t *flag) {
    bool over = false;
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
        over |= card[i] >= limit;
    if (__ballot(over) && lane_id() == 0) atomicOr(flag, 1u);
}

__global__ void k_zero_flag(uint32_t *flag) { *flag = 0; }

// Full layout: row i of blocks over its n entries; the lower triangle is
// mirrored from the upper.
__global__ void k_finalize(int32_t *__restrict__ B, const int64_t *__restrict__ card, uint32_t n,
                           uint32_t jblocks, int64_t *__restrict__ den, double *__restrict__ J) {
    const uint32_t i = blockIdx.x / jblocks;
    const uint32_t j = (blockIdx.x % jblocks) * blockDim.x + threadIdx.x;
    if (j >= n) return;
    uint64_t pos;
    int64_t b;
    if (i == j) {
        pos = out_index(i, i, n, false);
        b = card[i];
        B[pos] = (int32_t)b;
    } else if (i < j) {
        pos = out_index(i, j, n, false);
        b = B[pos];
    } else {
        pos = (uint64_t)i * n + j;
        b = B[(uint64_t)j * n + i];
        B[pos] = (int32_t)b;
    }
    const int64_t c = card[i] + card[j] - b;
    if (den) den[pos] = c;
    if (J) J[pos] = c == 0 ? 1.0 : (double)b / (double)c;
}

// Packed upper layout: rows i and n-1-i share a row of blocks over their
// n - i and i + 1 entries (n + 1 in all), so no thread of the grid is idle.
__global__ void k_finalize_upper(int32_t *__restrict__ B, const int64_t *__restrict__ card, uint32_t n,
                                 uint32_t jblocks, int64_t *__restrict__ den, double *__restrict__ J) {
    const uint32_t i0 = blockIdx.x / jblocks, i1 = n - 1 - i0;
    const uint32_t t = (blockIdx.x % jblocks) * blockDim.x + threadIdx.x;
    const uint32_t len0 = n - i0;  // entries of row i0
    if (t >= (i0 == i1 ? len0 : n + 1)) return;
    const uint32_t i = t < len0 ? i0 : i1;
    const uint32_t j = t < len0 ? i0 + t : i1 + (t - len0);
    const uint64_t pos = out_index(i, j, n, true);
    int64_t b;
    if (i == j) {
        b = card[i];
        B[pos] = (int32_t)b;
    } else {
        b = B[pos];
    }
    const int64_t c = card[i] + card[j] - b;
    if (den) den[pos] = c;
    if (J) J[pos] = c == 0 ? 1.0 : (double)b / (double)c;
}

// Tile variants of the MFMA Gram: word rows per step of the K loop, and how
// many blocks the K split aims for.  The autotuner (JAS_TUNE) times each on the
// caller's db and keeps the fastest for dbs of the same shape.
enum GramKind { kInt8 = 0, kInt8Wide = 1, kFp4 = 2, kFp4Wide = 3, kFp4Rep = 4 };
struct GramVariant {
    int step;
    uint64_t want_blocks;
    int kind;  // kInt8: k_gram_mfma; kInt8Wide: 256 x 256 tiles (k_gram_mfma_wide); kFp4: k_gram_fp4;
               // kFp4Wide: k_gram_fp4_wide; kFp4Rep: k_gram_fp4 with 32 copies of the nibble table
};
// (wide variants with 2 word rows per step or at most 2048 blocks measured
// slower on both dense workloads and are not listed)
// (int8 variants aimed at 1024 blocks, or with 2 rows per step at 2048, measured
// slower everywhere and are not listed)
constexpr GramVariant kVariants[] = {{4, 2048, kInt8},     {4, 4096, kInt8},     {2, 4096, kInt8},
                                     {4, 4096, kInt8Wide}, {4, 8192, kInt8Wide}, {4, 2048, kFp4},
                                     {2, 2048, kFp4},      {4, 4096, kFp4},      {2, 4096, kFp4},
                                     {4, 8192, kFp4},      {2, 8192, kFp4},      {4, 4096, kFp4Wide},
                                     {4, 8192, kFp4Wide},  {4, 16384, kFp4Wide}, {4, 4096, kFp4Rep},
                                     {4, 8192, kFp4Rep},   {2, 8192, kFp4Rep}};
constexpr int kNumVariants = sizeof(kVariants) / sizeof(kVariants[0]);
// Untuned choice, from the tuner's timings on MI355X: 128 x 128 fp4 tiles
// below n = 2048 (n = 1024: 6.5 ms against 10.6 for int8 tiles), 256 x 256 fp4
// tiles from there on (n = 4096: 16.7 against 26.9 ms; n = 10000: 0.75 against
// 1.09 s), each aimed at 8192 blocks.
constexpr int kDefaultNarrow = 9, kDefaultWide = 12;
static_assert(kVariants[kDefaultNarrow].kind == kFp4 && kVariants[kDefaultWide].kind == kFp4Wide, "defaults");

std::mutex g_tune_mu;
std::map<std::tuple<int, uint32_t, uint32_t>, int> g_tuned;  // (device, n, ceil(log2 H)) -> variant

void k_split(uint64_t H, uint64_t np, uint64_t want, uint64_t &kper, uint64_t &splits) {
    splits = std::max<uint64_t>(1, div_up(want, np));
    kper = div_up(H, splits);
    kper = std::max<uint64_t>(kper, 64);
    kper = div_up(kper, kKC) * kKC;
    splits = div_up(H, kper);
    if (splits > 65535) {
        splits = 65535;
        kper = div_up(div_up(H, splits), kKC) * kKC;
        splits = div_up(H, kper);
    }
}

void launch_mfma(const jas_db *db, int v, hipStream_t s, int32_t *B, bool upper) {
    const uint32_t n = (uint32_t)db->n;
    if (kVariants[v].kind == kInt8Wide || kVariants[v].kind == kFp4Wide) {
        const uint32_t nt = (uint32_t)div_up(n, kWideT);
        const uint64_t np = (uint64_t)nt * (nt + 1) / 2;
        uint64_t kper, splits;
        k_split(db->H, np, kVariants[v].want_blocks, kper, splits);
        const uint64_t ldw = div_up(n, 128) * 128;
        if (kVariants[v].kind == kFp4Wide && kper > kFp4MaxK) {  // keep every block's float sums below 2^24
            kper = kFp4MaxK / kKC * kKC;
            splits = div_up(db->H, kper);
        }
        if (kVariants[v].kind == kFp4Wide && splits <= 65535) {
            dim3 grid((uint32_t)np, (uint32_t)splits);
            k_gram_fp4_wide<4><<<grid, kWideNT, 0, s>>>(db->W.p, ldw, db->H, kper, nt, n, B, upper);
            return;
        }
        k_split(db->H, np, kVariants[v].want_blocks, kper, splits);
        dim3 grid((uint32_t)np, (uint32_t)splits);
        k_gram_mfma_wide<4><<<grid, kWideNT, 0, s>>>(db->W.p, ldw, db->H, kper, nt, n, B, upper);  // 4 rows per step
        return;
    }
    const uint32_t nt = (uint32_t)div_up(n, kT);
    const uint64_t np = (uint64_t)nt * (nt + 1) / 2;
    uint64_t kper, splits;
    k_split(db->H, np, kVariants[v].want_blocks, kper, splits);
    const uint64_t ldw = div_up(n, 128) * 128;
    if (kVariants[v].kind == kFp4 || kVariants[v].kind == kFp4Rep) {
        const bool rep = kVariants[v].kind == kFp4Rep;
        if (kper > kFp4MaxK) {  // keep every block's float sums below 2^24
            kper = kFp4MaxK / kKC * kKC;
            splits = div_up(db->H, kper);
        }
        if (splits <= 65535) {
            dim3 grid((uint32_t)np, (uint32_t)splits);
            if (kVariants[v].step == 4 && rep)
                k_gram_fp4<2, 4, 32><<<grid, kMfmaNT, 0, s>>>(db->W.p, ldw, db->H, kper, nt, n, B, upper);
            else if (kVariants[v].step == 4)
                k_gram_fp4<2, 4, 1><<<grid, kMfmaNT, 0, s>>>(db->W.p, ldw, db->H, kper, nt, n, B, upper);
            else if (rep)
                k_gram_fp4<2, 2, 32><<<grid, kMfmaNT, 0, s>>>(db->W.p, ldw, db->H, kper, nt, n, B, upper);
            else
                k_gram_fp4<2, 2, 1><<<grid, kMfmaNT, 0, s>>>(db->W.p, ldw, db->H, kper, nt, n, B, upper);
            return;
        }
        k_split(db->H, np, kVariants[v].want_blocks, kper, splits);  // too many blocks: the int8 kernel
    }
    dim3 grid((uint32_t)np, (uint32_t)splits);
    if (kVariants[v].step == 4)
        k_gram_mfma<2, 4><<<grid, kMfmaNT, 0, s>>>(db->W.p, ldw, db->H, kper, nt, n, B, upper);
    else
        k_gram_mfma<2, 2><<<grid, kMfmaNT, 0, s>>>(db->W.p, ldw, db->H, kper, nt, n, B, upper);
}

}  // namespace

int32_t gram_variants() { return kNumVariants; }

void finalize(uint32_t n, bool upper, hipStream_t s, int32_t *B, const int64_t *card, int64_t *den, double *J) {
    if (n == 0) return;
    if (upper) {
        // pairs of rows (i, n-1-i), the middle row alone when n is odd
        const uint32_t jb = (uint32_t)div_up((uint64_t)n + 1, 256);
        const uint64_t fb = div_up((uint64_t)n, 2) * jb;
        if (fb > 0xFFFFFFFFull) fail(JAS_EUNSUPPORTED, "n too large for finalize grid");
        JAS_TIMED("finalize", s);
        k_finalize_upper<<<(uint32_t)fb, 256, 0, s>>>(B, card, n, jb, den, J);
    } else {
        const uint32_t jb = (uint32_t)div_up(n, 256);
        const uint64_t fb = (uint64_t)n * jb;
        if (fb > 0xFFFFFFFFull) fail(JAS_EUNSUPPORTED, "n too large for finalize grid");
        JAS_TIMED("finalize", s);
        k_finalize<<<(uint32_t)fb, 256, 0, s>>>(B, card, n, jb, den, J);
    }
    check_launch("finalize");
}

void check_card_limit(const int64_t *card, uint32_t n, hipStream_t s) {
    if (n == 0) return;
    DevBuf<uint32_t> flag;
    flag.alloc(1, s, nullptr, true, "overflow flag");
    {
        JAS_TIMED("card_check", s);
        k_zero_flag<<<1, 1, 0, s>>>(flag.p);
        k_card_check<<<(uint32_t)std::min<uint64_t>(div_up(n, 256), 1024), 256, 0, s>>>(card, n,
                                                                                        (int64_t)card_limit(), flag.p);
    }
    check_launch("card check");
    uint32_t h = 0;
    JAS_HIP(hipMemcpyAsync(&h, flag.p, sizeof(h), hipMemcpyDeviceToHost, s));
    JAS_HIP(hipStreamSynchronize(s));
    if (h)
        fail(JAS_EOVERFLOW, "a summed |X_i| reaches " + std::to_string(card_limit()) +
                                " distinct IDs: int32 intersections would overflow");
}

void gram(const jas_db *db, uint32_t flags, hipStream_t s, int32_t *B, int64_t *card, int64_t *den, double *J) {
    const uint32_t n = (uint32_t)db->n;
    const bool upper = flags & JAS_UPPER;
    const bool accumulate = flags & JAS_ACCUMULATE;
    const uint64_t len = upper ? (uint64_t)n * (n + 1) / 2 : (uint64_t)n * n;
    if (n == 0) return;
    if (!accumulate) {
        JAS_TIMED("fill_i32", s);
        k_fill_i32<<<(uint32_t)std::min<uint64_t>(div_up(len, 256), 65536), 256, 0, s>>>(B, len, 0);
    }
    check_launch("zero B");
    if (db->H > 0 && n >= 2) {
        if (flags & JAS_FORCE_POPCOUNT) {
            const uint32_t nt = (uint32_t)div_up(n, kT);
            const uint64_t np = (uint64_t)nt * (nt + 1) / 2;
            uint64_t kper, splits;
            k_split(db->H, np, 2048, kper, splits);
            const uint64_t ldw = div_up(n, 128) * 128;
            dim3 grid((uint32_t)np, (uint32_t)splits);
            JAS_TIMED("gram_popc", s);
            k_gram_popc<<<grid, kNT, 0, s>>>(db->W.p, ldw, db->H, kper, nt, n, B, upper);
        } else {
            const auto key = std::make_tuple(db->device, n, ceil_log2_u64(db->H));
            int v = n >= 2048 ? kDefaultWide : kDefaultNarrow;
            const uint32_t forced = (flags >> 16) & 0xFFu;  // JAS_GRAM_VARIANT(v): v + 1
            if (forced) {
                v = (int)forced - 1;
            } else if (flags & JAS_TUNE) {
                // time every variant on this db (each adds into B, which is cleared again after)
                JAS_HOST_TIMED("gram_tune");
                hipEvent_t e0, e1;
                JAS_HIP(hipEventCreate(&e0));
                JAS_HIP(hipEventCreate(&e1));
                float best = INFINITY;
                for (int c = 0; c < kNumVariants; ++c) {
                    JAS_HIP(hipEventRecord(e0, s));
                    launch_mfma(db, c, s, B, upper);
                    check_launch("gram (tuning)");
                    JAS_HIP(hipEventRecord(e1, s));
                    JAS_HIP(hipEventSynchronize(e1));
                    float ms = 0.f;
                    JAS_HIP(hipEventElapsedTime(&ms, e0, e1));
                    if (ms < best) {
                        best = ms;
                        v = c;
                    }
                }
                (void)hipEventDestroy(e0);
                (void)hipEventDestroy(e1);
                {
                    std::lock_guard<std::mutex> lk(g_tune_mu);
                    g_tuned[key] = v;
                }
                k_fill_i32<<<(uint32_t)std::min<uint64_t>(div_up(len, 256), 65536), 256, 0, s>>>(B, len, 0);
                check_launch("zero B");
            } else {
                std::lock_guard<std::mutex> lk(g_tune_mu);
                const auto it = g_tuned.find(key);
                if (it != g_tuned.end()) v = it->second;
            }
            JAS_TIMED(kVariants[v].kind >= kFp4 ? "gram_fp4" : "gram_mfma", s);  // kFp4, kFp4Wide, kFp4Rep
            launch_mfma(db, v, s, B, upper);
        }
        check_launch("gram");
    }
    if (db->n_list > 0 && db->n_lpairs > 0) {
        const uint64_t chunk = std::max<uint64_t>(kPairChunk, div_up(db->n_lpairs, kPairBlocks));
        const uint64_t blocks = div_up(db->n_lpairs, chunk);
        if (blocks > 0xFFFFFFFFull) fail(JAS_EUNSUPPORTED, "row lists too long");
        const size_t lds = (size_t)n * sizeof(uint32_t) + ((size_t)n / 8 + 1) * sizeof(uint16_t);
        {
            JAS_TIMED("pair_count", s);
            k_pair_count<<<(uint32_t)blocks, kPairCountNT, lds, s>>>(db->pairs.p, db->n_lpairs, chunk, n, B, upper, db->dsz);
        }
        check_launch("row-list pairs");
    } else if (db->n_list > 0) {
        const uint64_t blocks = std::min<uint64_t>(div_up(db->n_list, 256), 65536);
        {
            JAS_TIMED("list_pairs", s);
            k_list_pairs<<<(uint32_t)blocks, 256, 0, s>>>(db->list_ptr.p, db->list_smp.p, db->n_list, n, B, upper);
        }
        check_launch("row list pairs");
    }
    if (accumulate) {
        {
            JAS_TIMED("add_card", s);
            k_add_i64<<<(uint32_t)div_up(n, 256), 256, 0, s>>>(card, db->card.p, n);
        }
        check_launch("add card");
        return;
    }
    finalize(n, upper, s, B, db->card.p, den, J);
    if (card) JAS_HIP(hipMemcpyAsync(card, db->card.p, sizeof(int64_t) * n, hipMemcpyDeviceToDevice, s));
}

}  // namespace jas
