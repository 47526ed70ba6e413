// Choice of the degree threshold between the two Gram paths.
//
// A shared row of degree d costs d(d-1)/2 pair counts on the row-list path
// (plus a per-row cost of filing it by sample); bit-packed, it costs a 1/64
// share of a word row, and every word row costs the same tile work whatever
// its density (T = nt(nt+1)/2 tiles of 128 x 128 word pairs,
// nt = ceil(n / 128)).  With h[d] rows of degree d:
//   pairs(t)  = sum_{2 <= d < t} h[d] d(d-1)/2,   rows(t) = sum_{2 <= d < t} h[d]
//   words(t)  = ceil(sum_{d >= t} h[d] / 64) + ragged last words of the batches
//   time(t)   = pairs(t) / r_pair + rows(t) / r_row + words(t) * 128^2 T / r_word
// The threshold t minimising time(t) is taken, among those whose packed matrix
// (words(t) * 8 * ceil(n/128)*128 bytes) fits the memory cap.  The rates were
// fitted on MI355X to the row-list kernels (7.4e10 pairs/s and 1.6e10 rows/s,
// over a sweep of thresholds on the paper-like workload) and to k_pack plus
// the default fp4 Gram tiles (2.4e13 to 3.4e13 word pairs/s on n = 1024, 4096
// and 10000; 2.6e13 taken).
#include <algorithm>
#include <cmath>

#include "jas_internal.hpp"

namespace jas {

namespace {
constexpr double kPairRate = 7.4e10;   // row-list pair counts per second
constexpr double kRowRate = 1.6e10;    // row-list rows filed per second
constexpr double kWordRate = 2.6e13;   // packed 64-bit word pairs per second (pack + MFMA kernel)
}  // namespace

uint32_t choose_dense_min_degree(const std::vector<uint64_t> &h, uint32_t n, uint64_t nbatches,
                                 uint64_t max_packed_bytes) {
    const uint64_t top = h.size();  // degrees 0 .. top-1
    const double nt = std::ceil(n / 128.0);
    const double tile_work = nt * (nt + 1) / 2 * 128.0 * 128.0;
    const double ldw = nt * 128.0;
    // packed rows for threshold t = suffix sum; list pairs = prefix sum
    std::vector<double> suffix(top + 1, 0.0);
    for (uint64_t d = top; d-- > 0;) suffix[d] = suffix[d + 1] + (double)h[d];
    double list = 0.0, rows = 0.0;
    double best = INFINITY;
    uint32_t best_t = (uint32_t)top;  // nothing packed
    for (uint64_t t = 2; t <= top; ++t) {
        if (t > 2) {
            const double d = (double)(t - 1);
            list += (double)h[t - 1] * d * (d - 1) / 2;
            rows += (double)h[t - 1];
        }
        const double packed = suffix[t];
        const double words = std::ceil(packed / 64.0) + std::min<double>((double)nbatches, packed) * 0.5;
        if (words * 8.0 * ldw > (double)max_packed_bytes) continue;
        const double time = list / kPairRate + rows / kRowRate + words * tile_work / kWordRate;
        if (time < best) {
            best = time;
            best_t = (uint32_t)t;
        }
    }
    return std::max<uint32_t>(2, best_t);
}

}  // namespace jas
