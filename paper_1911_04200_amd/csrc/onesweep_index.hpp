// Index arithmetic of the single-pass scatter (k_radix_onesweep in
// radix.hip): which keys a tile holds, where a tile's look-back status word
// for a digit lives, and where a key of the reordered tile is written.  Kept
// in one header so that a host emulation of the kernel's tile, status and
// output indexing (tests/radix_bounds_emul.cpp) uses the same expressions
// and can check every address against its buffer at full size.
#pragma once

#include <cstdint>

#if defined(__HIPCC__)
#define JAS_HD __host__ __device__
#else
#define JAS_HD
#endif

namespace jas {
namespace onesweep {

constexpr uint32_t kRadix = 256;
// status word: flag in the top two bits, a 30-bit count below
constexpr uint32_t kFlagA = 1u << 30;  // the tile's own count is available
constexpr uint32_t kFlagP = 2u << 30;  // the inclusive prefix over tiles 0..t is available
constexpr uint32_t kValMask = (1u << 30) - 1u;
constexpr int kLookWindow = 4;  // predecessor tiles read per look-back step

// Keys of tile t: [tile_first(t), tile_end(t)).
JAS_HD inline uint64_t tile_first(uint64_t tile, uint32_t tile_keys) { return tile * tile_keys; }
JAS_HD inline uint64_t tile_end(uint64_t tile, uint32_t tile_keys, uint64_t N) {
    const uint64_t e = (tile + 1) * tile_keys;
    return e < N ? e : N;
}
JAS_HD inline uint64_t num_tiles(uint64_t N, uint32_t tile_keys) { return (N + tile_keys - 1) / tile_keys; }

// Status words: one per (tile, digit), plus one spare.
JAS_HD inline uint64_t status_words(uint64_t ntiles) { return ntiles * kRadix + 1; }
JAS_HD inline uint64_t status_index(uint64_t tile, uint32_t digit) { return tile * kRadix + digit; }

// Output position of the key at position i of the tile reordered by digit,
// whose digit d starts at tdp_d in the tile and at base_d in the output
// (base_d = the digit's global start + the counts of d in earlier tiles).
JAS_HD inline uint64_t out_index(uint64_t base_d, uint32_t i, uint32_t tdp_d) { return base_d + (i - tdp_d); }

}  // namespace onesweep
}  // namespace jas
