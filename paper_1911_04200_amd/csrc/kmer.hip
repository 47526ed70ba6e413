// k-mer sets from 2-bit packed sequences: the step before the encoding.
//
// A k-mer is a length-k substring of a sequence (Sec. II-B); a sample's set is
// the k-mers of its sequences.  Each k-mer becomes one ID: the bases read as a
// base-4 number, first base most significant (A = 0, C = 1, G = 2, T = 3), so
// IDs are below 4^k = 2^(2k).  With JAS_CANONICAL the ID is the smaller of the
// k-mer and its reverse complement (the strand-independent form; odd k has
// no k-mer equal to its own reverse complement, Sec. V-A2).
//
// One thread per output k-mer: the sequence holding it comes from a search
// over the per-sequence k-mer starts, its bases from two 64-bit words of the
// packed array (staged in LDS per tile).  Bases sit least significant first in the words (base b
// at bits 2(b mod 32) of word b / 32), so a window read out of the words has
// the first base in its low bits: the reverse complement is then the
// complement of that window (3 - x per base is ~x on 2 bits), and the
// most-significant-first value is the window with its 2-bit groups reversed.
#include "jas_internal.hpp"

namespace jas {
namespace {

// Reverse the order of the 2-bit groups of a 64-bit word.
__device__ __forceinline__ uint64_t reverse_pairs(uint64_t y) {
    y = __builtin_bitreverse64(y);
    return ((y >> 1) & 0x5555555555555555ull) | ((y & 0x5555555555555555ull) << 1);
}

constexpr uint32_t kKmerNT = 256, kKmerPer = 16;  // a block's tile: kKmerNT * kKmerPer k-mers
constexpr uint32_t kKmerStage = 512;              // packed words a tile stages in LDS, at most

// Largest s with kbase[s] <= t (a sequence without k-mers shares its
// successor's start and is never the largest).
__device__ __forceinline__ uint64_t seq_of(const uint64_t *kbase, uint64_t n_seq, uint64_t t) {
    uint64_t lo = 0, hi = n_seq - 1;
    while (lo < hi) {
        const uint64_t mid = (lo + hi + 1) >> 1;
        if (kbase[mid] <= t) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// The k-mer of the bases held in window `win` (first base in the low bits).
__device__ __forceinline__ uint64_t kmer_id(uint64_t win, uint32_t k, uint64_t mask, int canonical) {
    win &= mask;
    const uint64_t fwd = reverse_pairs(win) >> (64 - 2 * k);  // first base most significant
    if (!canonical) return fwd;
    const uint64_t rc = ~win & mask;  // reverse complement, first base most significant
    return rc < fwd ? rc : fwd;
}

// A block per tile of consecutive k-mers.  Two binary searches over the
// per-sequence k-mer starts find the sequences of the tile's first and last
// k-mers; the packed words between their bases are one stretch of the array,
// staged in LDS with coalesced loads when it fits (a tile of 2048 k-mers over
// sequences much longer than k needs about 65 words).  Each thread walks
// forward from the first sequence (k-mers t, t + kKmerNT, ...) with the
// sequence's bounds in registers and reads its two words from LDS.
__global__ __launch_bounds__(kKmerNT) void k_kmers(const uint64_t *__restrict__ seq,
                                                   const uint64_t *__restrict__ seq_off,
                                                   const uint64_t *__restrict__ kbase, uint64_t n_seq,
                                                   uint64_t total, uint32_t k, int canonical,
                                                   uint64_t *__restrict__ ids) {
    __shared__ uint64_t s0, w0, nw;
    __shared__ uint64_t words[kKmerStage];
    const uint64_t mask = (k == 32) ? ~0ull : ((1ull << (2 * k)) - 1);
    const uint64_t tile = (uint64_t)kKmerNT * kKmerPer;
    for (uint64_t t0 = (uint64_t)blockIdx.x * tile; t0 < total; t0 += (uint64_t)gridDim.x * tile) {
        if (threadIdx.x == 0) {
            const uint64_t t1 = min(total, t0 + tile) - 1;
            const uint64_t a = seq_of(kbase, n_seq, t0), z = seq_of(kbase, n_seq, t1);
            const uint64_t b0 = seq_off[a] + (t0 - kbase[a]);          // first base of the tile
            const uint64_t b1 = seq_off[z] + (t1 - kbase[z]) + k - 1;  // last base of the tile
            s0 = a;
            w0 = b0 >> 5;
            nw = (b1 >> 5) - (b0 >> 5) + 1;
        }
        __syncthreads();
        const uint64_t ws = w0, n_words = nw;
        uint64_t s = s0;
        const bool staged = n_words <= kKmerStage;  // block-uniform
        if (staged)
            for (uint32_t i = threadIdx.x; i < n_words; i += kKmerNT) words[i] = seq[ws + i];
        __syncthreads();
        // this thread's sequence: its k-mers end before `next`, and k-mer t
        // starts at base `shift + t`
        uint64_t next = kbase[s + 1], shift = seq_off[s] - kbase[s];
#pragma unroll
        for (uint32_t u = 0; u < kKmerPer; ++u) {
            const uint64_t t = t0 + (uint64_t)u * kKmerNT + threadIdx.x;
            if (t >= total) break;
            if (next <= t) {
                do {
                    ++s;
                    next = kbase[s + 1];  // kbase[n_seq] = total > t ends the walk
                } while (next <= t);
                shift = seq_off[s] - kbase[s];
            }
            const uint64_t b = shift + t;  // first base of the k-mer
            const uint64_t w = b >> 5, sh = 2 * (b & 31);
            const bool two = sh + 2 * k > 64;  // the k-mer reaches into word w + 1 (at most the tile's last)
            uint64_t win;
            if (staged) {
                win = words[w - ws] >> sh;
                if (two) win |= words[w - ws + 1] << (64 - sh);
            } else {
                win = seq[w] >> sh;
                if (two) win |= seq[w + 1] << (64 - sh);
            }
            ids[t] = kmer_id(win, k, mask, canonical);
        }
        __syncthreads();  // s0, w0, nw and words are rewritten by the next tile
    }
}

}  // namespace

uint64_t kmer_starts(const uint64_t *seq_off, int64_t n_seq, uint32_t k, std::vector<uint64_t> &kbase) {
    kbase.assign((size_t)n_seq + 1, 0);
    for (int64_t s = 0; s < n_seq; ++s) {
        const uint64_t len = seq_off[s + 1] - seq_off[s];
        kbase[s + 1] = kbase[s] + (len >= k ? len - k + 1 : 0);
    }
    return kbase[n_seq];
}

void kmers(const uint64_t *seq, const uint64_t *seq_off, int64_t n_seq, uint32_t k, bool canonical, hipStream_t s,
           uint64_t *ids) {
    std::vector<uint64_t> kb;
    const uint64_t total = kmer_starts(seq_off, n_seq, k, kb);
    if (total == 0) return;
    DevBuf<uint64_t> dkb, doff;
    dkb.alloc(kb.size(), s, nullptr, true, "k-mer starts");
    doff.alloc((size_t)n_seq + 1, s, nullptr, true, "sequence offsets");
    JAS_HIP(hipMemcpyAsync(dkb.p, kb.data(), kb.size() * 8, hipMemcpyHostToDevice, s));
    JAS_HIP(hipMemcpyAsync(doff.p, seq_off, ((size_t)n_seq + 1) * 8, hipMemcpyHostToDevice, s));
    const uint64_t blocks = std::min<uint64_t>(div_up(total, (uint64_t)kKmerNT * kKmerPer), 65536);
    {
        JAS_TIMED("kmers", s);
        k_kmers<<<(uint32_t)blocks, kKmerNT, 0, s>>>(seq, doff.p, dkb.p, (uint64_t)n_seq, total, k, canonical ? 1 : 0,
                                                  ids);
    }
    check_launch("k-mers");
    // the host arrays above are read by the copies before this call returns
    JAS_HIP(hipStreamSynchronize(s));
}

}  // namespace jas
