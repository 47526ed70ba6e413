// Host emulation of the indexing of the single-pass radix scatter
// (k_radix_onesweep, paper_1911_04200_amd/csrc/radix.hip), using the same
// index expressions (csrc/onesweep_index.hpp).  It walks every tile of every
// pass in ticket order, models the look-back over predecessor tiles whose
// status words are published or not yet published at random (a wait that
// would time out gives up, as the kernel's bounded wait does, and then every
// later wait gives up at once), and checks that every status word read or
// written, every digit start and every output position lies inside its
// buffer.  Without give-ups it also checks that the output ranges of each
// digit over the tiles are exactly consecutive (a permutation of [0, N)).
//
// usage: radix_bounds_emul N tile_keys nbits,nbits,... dist giveup_per_million seed [exact]
//   dist: "uniform" (every digit equally likely) or "skew" (digit 0 for half
//   the keys); exact: also check the position of every key (slow for large N).
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "onesweep_index.hpp"

using namespace jas::onesweep;

static uint64_t mix(uint64_t x) {  // SplitMix64 finaliser (Steele, Lea, Flood 2014)
    x += 0x9E3779B97F4A7C15ull;
    x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
    x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
    return x ^ (x >> 31);
}

static int fails = 0;
#define CHECK(c, ...)                                  \
    do {                                               \
        if (!(c)) {                                    \
            if (fails < 20) std::printf(__VA_ARGS__);  \
            ++fails;                                   \
        }                                              \
    } while (0)

int main(int argc, char **argv) {
    if (argc < 7) return 2;
    const uint64_t N = std::strtoull(argv[1], nullptr, 10);
    const uint32_t T = (uint32_t)std::strtoul(argv[2], nullptr, 10);
    std::vector<uint32_t> widths;
    for (char *p = argv[3]; *p;) {
        widths.push_back((uint32_t)std::strtoul(p, &p, 10));
        if (*p == ',') ++p;
    }
    const bool skew = std::string(argv[4]) == "skew";
    const uint64_t giveup_ppm = std::strtoull(argv[5], nullptr, 10);
    const uint64_t seed = std::strtoull(argv[6], nullptr, 10);
    const bool exact = argc > 7 && std::string(argv[7]) == "exact";
    constexpr uint32_t kMaxPasses = 8;
    if (widths.size() > kMaxPasses) return 2;

    const uint64_t ntiles = num_tiles(N, T);
    std::vector<uint32_t> status(status_words(ntiles));  // what each tile finally publishes
    std::vector<uint32_t> agg(ntiles * kRadix);            // each tile's own counts
    std::vector<uint64_t> gstart((uint64_t)kMaxPasses * kRadix);
    auto digit_of = [&](uint64_t key, uint32_t q, uint32_t mask) -> uint32_t {
        const uint64_t h = mix(seed * 0x100000001B3ull + key * kMaxPasses + q);
        if (skew && (h >> 63)) return 0;
        return (uint32_t)h & mask;
    };
    uint64_t giveups = 0;
    for (uint32_t q = 0; q < widths.size(); ++q) {
        const uint32_t mask = (1u << widths[q]) - 1u;
        // digit totals (as the key-building kernel counts them) and starts
        std::vector<uint64_t> tot(kRadix, 0);
        for (uint64_t k = 0; k < N; ++k) ++tot[digit_of(k, q, mask)];
        uint64_t run = 0, mx = 0;
        for (uint32_t d = 0; d < kRadix; ++d) {
            const uint64_t gi = (uint64_t)q * kRadix + d;
            CHECK(gi < gstart.size(), "gstart index %llu\n", (unsigned long long)gi);
            gstart[gi] = run;
            run += tot[d];
            mx = tot[d] > mx ? tot[d] : mx;
        }
        if (mx >= kValMask) {  // the host refuses the single-pass scatter here
            std::printf("pass %u: a digit total reaches 2^30: falls back to the per-pass sort\n", q);
            continue;
        }
        std::fill(status.begin(), status.end(), 0u);
        std::vector<uint64_t> next_pos(kRadix);  // expected start of each digit's next range
        for (uint32_t d = 0; d < kRadix; ++d) next_pos[d] = gstart[(uint64_t)q * kRadix + d];
        bool gave_up = false;
        std::vector<uint32_t> tc(kRadix), tdp(kRadix);
        std::vector<uint64_t> base(kRadix);
        for (uint64_t tile = 0; tile < ntiles; ++tile) {  // ticket order
            const uint64_t t0 = tile_first(tile, T), c1 = tile_end(tile, T, N);
            CHECK(t0 < c1 && c1 <= N, "tile %llu keys [%llu, %llu)\n", (unsigned long long)tile,
                  (unsigned long long)t0, (unsigned long long)c1);
            std::fill(tc.begin(), tc.end(), 0u);
            for (uint64_t k = t0; k < c1; ++k) ++tc[digit_of(k, q, mask)];
            uint32_t ex = 0;
            for (uint32_t d = 0; d < kRadix; ++d) {
                tdp[d] = ex;
                ex += tc[d];
                const uint64_t si = status_index(tile, d);
                CHECK(si < status.size(), "status write %llu\n", (unsigned long long)si);
                agg[si] = tc[d];
            }
            CHECK(ex == c1 - t0, "tile count\n");
            for (uint32_t d = 0; d < kRadix; ++d) {
                uint32_t excl = 0;
                if (tile > 0) {
                    bool found = false;
                    for (int64_t j0 = (int64_t)tile - 1; j0 >= 0 && !found; j0 -= kLookWindow) {
                        for (int k = 0; k < kLookWindow && !found; ++k) {
                            const int64_t j = j0 - k;
                            uint32_t v = kFlagP;
                            if (j >= 0) {
                                const uint64_t si = status_index((uint64_t)j, d);
                                CHECK(si < status.size(), "status read %llu\n", (unsigned long long)si);
                                // state of predecessor j when read: 0 not published, 1 own count, 2 prefix
                                const uint64_t h = mix(seed ^ (tile * 0x9E37ull + (uint64_t)j * 131 + d));
                                uint32_t state = (uint32_t)(h % 3);
                                if (state == 0) {  // waits: the tile publishes, or the wait gives up
                                    if (gave_up || (giveup_ppm && (h >> 40) % 1000000 < giveup_ppm)) {
                                        gave_up = true;
                                        ++giveups;
                                        state = 3;  // given up: taken as a prefix of 0
                                    } else {
                                        state = 1 + (uint32_t)((h >> 20) & 1);
                                    }
                                }
                                v = state == 3 ? kFlagP : state == 2 ? status[si] : (kFlagA | agg[si]);
                            }
                            excl += v & kValMask;
                            found = (v & ~kValMask) == kFlagP;
                        }
                    }
                }
                const uint64_t si = status_index(tile, d);
                status[si] = kFlagP | ((excl + tc[d]) & kValMask);
                base[d] = gstart[(uint64_t)q * kRadix + d] + excl;
                if (tc[d] == 0) continue;
                const uint64_t lo = out_index(base[d], tdp[d], tdp[d]);
                const uint64_t hi = out_index(base[d], tdp[d] + tc[d] - 1, tdp[d]);
                CHECK(lo <= hi && hi < N, "pass %u tile %llu digit %u writes [%llu, %llu] outside [0, %llu)\n", q,
                      (unsigned long long)tile, d, (unsigned long long)lo, (unsigned long long)hi,
                      (unsigned long long)N);
                if (!gave_up) {
                    CHECK(lo == next_pos[d], "pass %u tile %llu digit %u starts at %llu, expected %llu\n", q,
                          (unsigned long long)tile, d, (unsigned long long)lo, (unsigned long long)next_pos[d]);
                    next_pos[d] = hi + 1;
                }
            }
            if (exact) {
                for (uint32_t i = 0; i < c1 - t0; ++i) {
                    // the key at position i of the tile reordered by digit: the digit whose
                    // stretch [tdp, tdp + tc) holds i
                    uint32_t d = 0;
                    while (d + 1 < kRadix && tdp[d + 1] <= i) ++d;
                    while (tc[d] == 0) ++d;
                    const uint64_t o = out_index(base[d], i, tdp[d]);
                    CHECK(o < N, "key %u of tile %llu -> %llu\n", i, (unsigned long long)tile, (unsigned long long)o);
                }
            }
        }
        if (!gave_up)
            for (uint32_t d = 0; d < kRadix; ++d) {
                const uint64_t end = gstart[(uint64_t)q * kRadix + d] + tot[d];
                CHECK(next_pos[d] == end, "pass %u digit %u ends at %llu, expected %llu\n", q, d,
                      (unsigned long long)next_pos[d], (unsigned long long)end);
            }
    }
    std::printf("N %llu tiles %llu passes %zu giveups %llu fails %d\n", (unsigned long long)N,
                (unsigned long long)ntiles, widths.size(), (unsigned long long)giveups, fails);
    return fails ? 1 : 0;
}
