/*
 * jas.h -- C ABI of libjas: exact all-pairs Jaccard similarity of n sets on
 * one AMD MI355X (gfx950), computed as in SimilarityAtScale (arXiv 1911.04200).
 *
 * Problem (Sec. II-A, Eq. (1)): n samples X_1..X_n, each a set of integer IDs;
 * for every pair, J(X_i, X_j) = |X_i cap X_j| / |X_i cup X_j|, and J = 1 when
 * both sets are empty.  IDs here are 0-based integers in [0, 2^U) (the paper's
 * "positive integers up to m" relabelled).
 *
 * Method (Sec. III-A/B): with the indicator matrix A (a_ki = 1 iff k in X_i),
 * B = A^T A holds the intersection sizes, C_ij = |X_i| + |X_j| - B_ij the union
 * sizes and S = B / C the similarities (Eq. (2)).  A is cut into row batches of
 * m~ = 2^batch_bits IDs (Eq. (3)), zero rows are filtered and the rest compacted
 * (Eqs. (5), (6)), 64 consecutive rows of a column are packed into one bitmask
 * word (Sec. III-B), and B accumulates popcount(word_i AND word_j) over words
 * and batches (Eqs. (4), (7)).
 *
 * Conventions shared by every call:
 *  - Pointers are DEVICE pointers unless a call's flags include JAS_HOST_PTRS.
 *    The caller owns every input and output buffer.
 *  - Work is enqueued on `hip_stream` (a hipStream_t; NULL = the null stream).
 *    Outputs are valid once that stream has completed; inputs must stay alive
 *    until then.  Calls may synchronise `hip_stream` where noted.
 *  - Every call returns a jas_status.  On failure, jas_last_error() gives a
 *    message (thread-local, valid until this thread's next jas_* call) and the
 *    contents of output buffers are unspecified.  Argument errors are detected
 *    on the host before any work is enqueued.  No C++ exception crosses the ABI.
 *  - Row-major outputs: entry (i, j) of an n x n result is at i*n + j.  The
 *    packed upper layout (JAS_UPPER) stores row i's entries j >= i back to back:
 *    (i, j) is at i*n - i*(i-1)/2 + (j - i).
 */
#ifndef JAS_H
#define JAS_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    JAS_OK = 0,
    JAS_EINVAL = -1,       /* bad argument (null pointer, bad offsets, ID >= 2^U, ...) */
    JAS_ENOMEM = -2,       /* device allocation failed or the HBM budget is exceeded */
    JAS_EOVERFLOW = -3,    /* a set has 2^31 or more distinct IDs (int32 B would overflow) */
    JAS_EDEVICE = -4,      /* a HIP runtime call failed (message names it) */
    JAS_EBUSY = -5,        /* a shared resource is in use and the caller asked not to wait (JAS_NO_WAIT) */
    JAS_EUNSUPPORTED = -6  /* valid request the library does not support (message says why) */
} jas_status;

/* ---- flags ---------------------------------------------------------------- */
#define JAS_HOST_PTRS 0x1u      /* set arrays / outputs are host memory */
#define JAS_KEEP_IDS 0x2u       /* jas_encode: keep the row index needed by jas_query */
#define JAS_UPPER 0x10u         /* jas_gram: outputs in the packed upper layout (j >= i) */
#define JAS_FORCE_POPCOUNT 0x20u /* jas_gram: every packed tile on the AND+popcount kernel */
#define JAS_FORCE_MFMA 0x40u    /* jas_gram: every packed tile on an MFMA kernel (int8, or fp4 with exact float sums) */
#define JAS_TUNE 0x80u          /* jas_gram: time the MFMA tile variants on this db first (see jas_gram) */
#define JAS_ACCUMULATE 0x100u   /* jas_gram: add this db's counts into B and card (one row batch of many) */
#define JAS_CANONICAL 0x200u    /* jas_kmers: each k-mer as the smaller of itself and its reverse complement */
#define JAS_NO_WAIT 0x400u      /* jas_query_noalloc: JAS_EBUSY at once, instead of waiting, while another call
                                   holds this process's fixed workspace */
#define JAS_QUERY_ONLY 0x800u   /* jas_encode, with JAS_KEEP_IDS: keep only what jas_query reads (the distinct
                                   keys, their bucket table, |X_i|); no packed words or row lists are built, and
                                   jas_gram refuses the db */
/* jas_gram: run MFMA tile variant v, 0 <= v < jas_gram_variants() (bits 16..23 hold v + 1) */
#define JAS_GRAM_VARIANT(v) ((((uint32_t)(v)) + 1u) << 16)

typedef struct jas_db jas_db; /* opaque, library-owned, device-resident encoding of A */

typedef struct {
    uint32_t universe_bits;    /* U, 1..63: every ID is < 2^U; U + ceil(log2 n) <= 64 */
    uint32_t batch_bits;       /* log2 of the row-batch height m~ (Eq. (3)); 0 or >= U: one batch */
    uint32_t dense_min_degree; /* rows shared by >= this many sets are bit-packed (Sec. III-B);
                                  rows shared by 2..this-1 sets are kept as plain row lists;
                                  0 = chosen by the library from the row degree histogram
                                  (cost model of the two Gram paths); 2 = pack every shared row */
    uint32_t flags;            /* JAS_HOST_PTRS, JAS_KEEP_IDS, JAS_QUERY_ONLY */
    uint64_t hbm_budget_bytes; /* cap on device memory this call may hold at once; 0 = none */
    uint32_t word_bits;        /* b, rows per bitmask word (Sec. III-B): 32 or 64; 0 = 64.  B does
                                  not depend on it (every word's popcount sums its rows) */
    uint32_t reserved;         /* 0 */
} jas_encode_opts;

typedef struct {
    uint64_t n_ids;         /* N: input entries, repeats included */
    uint64_t n_pairs;       /* nnz(A): distinct (ID, sample) pairs */
    uint64_t n_rows;        /* nonzero rows of A (distinct IDs), the filter's support (Eq. (5)) */
    uint64_t n_shared_rows; /* rows in >= 2 sets (the only rows off-diagonal B depends on) */
    uint64_t n_packed_rows; /* rows bit-packed (degree >= dense_min_degree) */
    uint64_t n_list_rows;   /* rows kept as row lists (2 <= degree < dense_min_degree) */
    uint64_t n_batches;     /* row batches holding at least one packed row */
    uint64_t n_word_rows;   /* h: word rows of b rows each (b = word_bits) over all batches */
    uint64_t nnz_words;     /* nonzero packed words */
    uint64_t word_pairs_F;  /* sum over word rows of z(z+1)/2, z = nonzero words in the row */
    uint64_t list_pairs;    /* sum over list rows of d(d-1)/2 (pair increments of the list path) */
    uint64_t device_bytes;  /* device memory the db holds */
    uint64_t dense_min_degree; /* the threshold used (chosen by the library when opts asked for 0) */
    uint64_t word_bits;     /* b used (32 or 64) */
    uint64_t w_rows;        /* rows of the stored word array (JAS_DB_WORDS): h for b = 64, ceil(h/2) for 32 */
    uint64_t w_stride;      /* 64-bit elements per stored row (n rounded up to a multiple of 128) */
    uint64_t n_list_pairs;  /* entries of JAS_DB_LIST_PAIRS */
    uint64_t dense_tiles;   /* work units of the packed Gram: (stored word row, pair I <= J of 128-column
                               tiles), w_rows * T with T = t(t+1)/2, t = ceil(n/128); 0 without packed rows.
                               The row lists have no tiles: their work is list_pairs */
    uint64_t word_pairs_W;  /* 64-bit word pairs those units multiply, dense_tiles * 128^2 (for b = 64 at
                               least word_pairs_F: whole tiles run, zero words included) */
} jas_encode_stats;

/*
 * jas_encode -- build the encoded indicator matrix of n sets (Sec. III-B,
 * Eqs. (3)-(6) and the bitmask compression before Eq. (7)).
 *
 *  ids      uint64[offsets[n]]: the IDs of sample i are ids[offsets[i] .. offsets[i+1]),
 *           any order, repeats allowed (a set: repeats are ignored).
 *  offsets  uint64[n+1]: offsets[0] = 0, non-decreasing.
 *  n        number of samples, >= 0.
 *  opts     see jas_encode_opts (required).
 *  db_out   receives the handle; NULL on failure.  Free with jas_db_free.
 *  stats    optional (NULL allowed).
 * Errors: EINVAL (null pointers, offsets[0] != 0, decreasing offsets, an ID >= 2^U,
 * U out of range), EOVERFLOW (a set with >= 2^31 distinct IDs), ENOMEM, EDEVICE.
 * Synchronises hip_stream (the sizes of the encoding are data-dependent).
 * The input arrays are not modified and may be freed after the call returns.
 */
jas_status jas_encode(const uint64_t *ids, const uint64_t *offsets, int32_t n, const jas_encode_opts *opts,
                      void *hip_stream, jas_db **db_out, jas_encode_stats *stats);

/*
 * jas_gram -- the Gram product and the similarity of every pair of encoded
 * samples: B = A^T A accumulated as in Eqs. (4) and (7), the unions
 * C_ij = |X_i| + |X_j| - B_ij and J_ij = B_ij / C_ij (Sec. III-A, Eq. (2)).
 *
 *  B     int32[n*n] (or n(n+1)/2 with JAS_UPPER): B_ij = |X_i cap X_j|; required.
 *  card  int64[n]: |X_i|; may be NULL.
 *  den   int64, same layout as B: C_ij = |X_i cup X_j|; may be NULL.
 *  J     double, same layout as B: C_ij == 0 ? 1.0 : (double)B_ij / (double)C_ij,
 *        IEEE binary64 round-to-nearest; may be NULL.
 *  flags JAS_UPPER, JAS_FORCE_POPCOUNT / JAS_FORCE_MFMA (at most one), JAS_HOST_PTRS,
 *        JAS_TUNE, JAS_GRAM_VARIANT(v) (not with JAS_TUNE or JAS_FORCE_POPCOUNT).
 * The result does not depend on flags other than the layout: every tile path
 * is exact.  Does not synchronise unless JAS_HOST_PTRS or JAS_TUNE is given.
 * JAS_TUNE (autotuner): before the product, the MFMA Gram runs once in each of
 * its variants (tile, number format: int8 or fp4 (e2m1, each bit 0 or 1.0, the
 * float32 sums of a block kept below 2^24 so they are exact), word rows per
 * step, K split) on this db, timed with HIP
 * events on the stream (synchronising); the fastest is kept, in this process,
 * for every later db on the device with the same n and the same power of two
 * of word rows, and is used by later calls without the flag.  Not capturable
 * in a HIP graph; calls without it are.  JAS_GRAM_VARIANT(v) runs variant v
 * instead of the kept or default choice (EINVAL for v out of range).  The
 * default, with nothing kept, is fp4 with 128 x 128 tiles below n = 2048 and
 * 256 x 256 tiles from there on.
 * JAS_ACCUMULATE (row batches streamed one db at a time, the sum over batches
 * l of Eq. (4)): B_ij (i < j) and card_i are added to instead of written, and
 * nothing else is written: card is required, den and J must be NULL, and
 * JAS_TUNE is refused.  The caller clears B and card before the first batch
 * (torch's zero_() or a fill kernel; hipMemsetAsync where no graph is
 * captured) and calls jas_finalize after the last one; until then the
 * diagonal and, in the full layout, the lower triangle of B are undefined.
 * The db of each batch must hold the same n samples; a row (ID) may appear in
 * only one of them.  The sums are int32: they are exact while every summed
 * |X_i| stays below 2^31 (B_ij <= min(|X_i|, |X_j|), so no sum of B can then
 * overflow); jas_finalize checks that bound.
 */
jas_status jas_gram(const jas_db *db, uint32_t flags, void *hip_stream, int32_t *B, int64_t *card, int64_t *den,
                    double *J);

/*
 * jas_finalize -- the last step of a streamed product: from the summed
 * intersections B (i < j entries, as left by jas_gram with JAS_ACCUMULATE) and
 * the summed sizes card, write the diagonal B_ii = |X_i|, in the full layout
 * the lower triangle B_ji = B_ij, and (where not NULL) the unions
 * C_ij = |X_i| + |X_j| - B_ij and J_ij = B_ij / C_ij (1.0 where C_ij = 0),
 * exactly as jas_gram does for one db (Sec. III-A, Eq. (2)).
 *  n       number of samples, >= 0.
 *  flags   JAS_UPPER (the layout B was accumulated in); device pointers only.
 *  B       int32, device, n*n or n(n+1)/2 entries: read and completed.
 *  card    int64[n], device: |X_i| summed over the batches.
 *  den, J  as in jas_gram; may be NULL.
 * Before writing anything, checks on the device that every summed |X_i| is
 * below jas_card_limit() and reads that one flag back (synchronises
 * hip_stream): EOVERFLOW otherwise, because an int32 sum of B may then have
 * overflowed.  EINVAL for n < 0, NULL B or card, other flags.
 */
jas_status jas_finalize(int32_t n, uint32_t flags, void *hip_stream, int32_t *B, const int64_t *card, int64_t *den,
                        double *J);

/* The bound on set sizes the int32 intersections allow: jas_encode and
 * jas_finalize return EOVERFLOW for a set of jas_card_limit() or more distinct
 * IDs.  2^31, unless the environment variable JAS_TEST_CARD_LIMIT holds a
 * positive integer below 2^31 (a test hook, read at every check, so tests can
 * reach the error with small inputs).  Host only. */
uint64_t jas_card_limit(void);

/*
 * jas_kmer_offsets / jas_kmers -- the k-mer sets of n samples from their
 * sequences: the step before jas_encode.  A k-mer is a length-k substring of
 * a sequence (Sec. II-B); sample i's set is the k-mers of its sequences.
 * The ID of a k-mer is its bases read as a base-4 number, first base most
 * significant (A = 0, C = 1, G = 2, T = 3), so IDs are below 2^(2k) and
 * jas_encode takes universe_bits = 2k (when 2k + ceil(log2 n) exceeds 64, as for k = 31 and n > 4, the
 * IDs go through jas_relabel first).  JAS_CANONICAL replaces each by the
 * smaller of it and its reverse complement (strand-independent k-mers; an
 * odd k has no palindromes, Sec. V-A2).  Repeated k-mers are left in; the
 * encoding removes them.
 *
 *  seq_off  uint64[n_seq+1], host: sequence s is bases seq_off[s] ..
 *           seq_off[s+1]-1 of the packed base array (0 first, non-decreasing).
 *  smp_off  uint64[n+1], host: sample i owns sequences smp_off[i] ..
 *           smp_off[i+1]-1 (0 first, non-decreasing, smp_off[n] = n_seq).
 *  k        1..31.
 *  ids_off  uint64[n+1], host output of jas_kmer_offsets: sample i's k-mers
 *           are ids[ids_off[i] .. ids_off[i+1]) (a sequence of length L
 *           holds L - k + 1 of them, none if L < k); ids_off[n] is the size
 *           of ids.  Host arithmetic only, no device call.
 *  seq      uint64 words, device: every base in 2 bits, base b at bits
 *           2 (b mod 32) of word b / 32; ceil(seq_off[n_seq] / 32) words.
 *  ids      uint64[ids_off[n]], device output of jas_kmers, in sequence and
 *           position order.
 * jas_kmers runs on hip_stream and returns after its work is done (it reads
 * seq_off from the host).  EINVAL for bad offsets, k or flags.
 */
jas_status jas_kmer_offsets(const uint64_t *seq_off, int64_t n_seq, const uint64_t *smp_off, int32_t n, uint32_t k,
                            uint64_t *ids_off);
jas_status jas_kmers(const uint64_t *seq, const uint64_t *seq_off, int64_t n_seq, uint32_t k, uint32_t flags,
                     void *hip_stream, uint64_t *ids);

/*
 * jas_relabel -- an exact relabelling of IDs: every ID becomes its rank among
 * the distinct IDs of the array (0 .. D-1).  Equal IDs stay equal and distinct
 * ones stay distinct, so every intersection and union of sets built from
 * these IDs is unchanged (B, C and J are the same), while the IDs then fit
 * ceil(log2 D) bits.  For k-mers of k > 32 - ceil(log2 n) / 2 (k = 31: IDs
 * below 2^62, Sec. II-B), whose IDs and sample numbers do not fit one 64-bit
 * key of jas_encode together.  Relabel everything that is compared in one
 * call (a database and the queries that will be run against it together).
 *  ids     uint64[n_ids], device, each < 2^universe_bits (else EINVAL).
 *  out     uint64[n_ids], device; may be ids itself.
 *  n_distinct, new_universe_bits  host outputs (may be NULL): D, and
 *          max(1, ceil(log2 D)), the universe_bits to encode the result with.
 * Sorts a copy of the IDs on hip_stream (2 x 8 bytes per ID of temporaries)
 * and synchronises it.
 */
jas_status jas_relabel(const uint64_t *ids, uint64_t n_ids, uint32_t universe_bits, void *hip_stream, uint64_t *out,
                       uint64_t *n_distinct, uint32_t *new_universe_bits);

/* Number of MFMA tile variants jas_gram can run (tile shape, word rows per
 * step, K split); variant indices are stable within one build of the library. */
int32_t jas_gram_variants(void);

/*
 * Encode plans -- the batching form as one capturable launch sequence: the
 * encode of Sec. III-B (Eqs. (3)-(6)) for collections of one shape, with no
 * host synchronisation and no allocation, so that jas_plan_encode, jas_gram
 * and jas_finalize's work can be captured in one HIP graph and replayed for
 * every new collection.
 *
 * jas_plan_create encodes (ids, offsets, n) once as jas_encode does and keeps
 * what that encode decided (the sort's bits, the range stride, the key width
 * in LDS, the row degree threshold) together with buffers for every
 * intermediate array at this collection's sizes times (1 + headroom), plus a
 * floor of 64 rows (1024 list pairs) for each form of row the threshold admits,
 * also where this collection has none (packed and list rows are each capped
 * at the shared-row capacity).  opts as
 * in jas_encode, device pointers only, no JAS_KEEP_IDS, 1 <= n <= 10240;
 * with dense_min_degree = 0 and JAS_TUNE in opts->flags the threshold is
 * chosen by timing encode + Gram on the device for candidate thresholds (the
 * cost model's choice t, t/2, 2t, 2 and n+1; jas_plan_tuning lists them).
 * Synchronises hip_stream.  headroom in [0, 4].
 *
 * jas_plan_encode encodes another collection of the same n into the plan's db
 * (jas_plan_db; owned by the plan, never passed to jas_db_free): everything
 * is enqueued on hip_stream, every size is computed and read on the device.
 * Capturable.  The plan's db is then valid for jas_gram once the stream has
 * run; calls on one plan must not overlap.
 *
 * jas_plan_check (after the stream has run; synchronises it) returns what the
 * last jas_plan_encode found: OK; ENOMEM when a size exceeded its capacity
 * (plan again with more headroom); EUNSUPPORTED when the collection needed
 * what the plan did not prepare (wider LDS keys, a shorter range stride, the
 * per-pass sort); EINVAL for an ID >= 2^U; EOVERFLOW for a set of
 * jas_card_limit() or more IDs; EDEVICE when the sort's look-back gave up.
 * Unless OK, the db's contents are unspecified.  stats (may be NULL) gets the
 * encode's statistics.
 */
typedef struct jas_plan jas_plan;
jas_status jas_plan_create(const uint64_t *ids, const uint64_t *offsets, int32_t n, const jas_encode_opts *opts,
                           double headroom, void *hip_stream, jas_plan **plan_out);
jas_status jas_plan_encode(jas_plan *plan, const uint64_t *ids, const uint64_t *offsets, void *hip_stream);
jas_status jas_plan_check(jas_plan *plan, void *hip_stream, jas_encode_stats *stats);
const jas_db *jas_plan_db(const jas_plan *plan);
/* The plan's row degree threshold (0 for NULL). */
uint32_t jas_plan_threshold(const jas_plan *plan);
/* Up to cap (threshold, encode + Gram ms) pairs of the timing that chose it; returns how many there are. */
int32_t jas_plan_tuning(const jas_plan *plan, uint32_t *thresholds, double *ms, int32_t cap);
/* Frees the plan and its device memory (synchronises the device first).  NULL is a no-op. */
void jas_plan_free(jas_plan *plan);

/*
 * jas_query -- similarity of nq query sets against every encoded sample:
 * Eq. (1) with i ranging over the queries and j over the database.
 *
 *  q_ids, q_offsets  CSR query sets, as in jas_encode (IDs < 2^U, else EINVAL;
 *                    repeats ignored).  An ID absent from the database counts
 *                    toward |Q| only.
 *  B      int32[nq*n]: |Q_q cap X_j|, row-major; required.
 *  q_card int64[nq]: |Q_q| (distinct); may be NULL.
 *  den    int64[nq*n]: |Q_q cup X_j|; may be NULL.
 *  J      double[nq*n]; may be NULL.
 * Requires a db encoded with JAS_KEEP_IDS (else EINVAL).  The db is read only:
 * concurrent jas_query calls on different streams are safe.  Synchronises
 * hip_stream (query sizes and the ID range check are read back).
 */
jas_status jas_query(const jas_db *db, const uint64_t *q_ids, const uint64_t *q_offsets, int32_t nq,
                     uint32_t flags, void *hip_stream, int32_t *B, int64_t *q_card, int64_t *den, double *J);

/*
 * jas_query_noalloc -- jas_query for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc).  Same arguments, results and errors as jas_query, with
 * device pointers only (flags: 0 or JAS_NO_WAIT), but every temporary comes from a
 * fixed workspace of 136 MiB that the library holds on each device it runs
 * on until the process ends: no device memory is allocated or freed.  It
 * takes at most 65,536 query sets and 2^23 query IDs (entries, repeats
 * included) per call; larger requests fail with JAS_ENOMEM before any work
 * is enqueued.  Calls share the workspace, so the library serialises them
 * (a lock per process) and each returns only after its work on hip_stream
 * has finished (synchronises hip_stream); with JAS_NO_WAIT a call that finds
 * the workspace in use returns JAS_EBUSY at once, before any work is
 * enqueued.  The workspace keeps the last call's contents, and everything
 * that must start at zero is cleared by the call itself.
 */
jas_status jas_query_noalloc(const jas_db *db, const uint64_t *q_ids, const uint64_t *q_offsets, int32_t nq,
                             uint32_t flags, void *hip_stream, int32_t *B, int64_t *q_card, int64_t *den, double *J);

/* Device bytes jas_query allocates for nq queries with n_q_ids entries in total
 * (for admission control by an HBM budget). */
uint64_t jas_query_workspace_bytes(const jas_db *db, int32_t nq, uint64_t n_q_ids);

/* Number of samples n of the db (-1 for NULL). */
int32_t jas_db_size(const jas_db *db);

/* Statistics recorded by jas_encode.  Returns EINVAL for NULL arguments. */
jas_status jas_db_stats(const jas_db *db, jas_encode_stats *stats);

/*
 * jas_db_part_size / jas_db_read -- the db's arrays, read back to the host
 * (for checking or keeping an encoding; the layout is that of this library version).
 *  JAS_DB_CARD          int64[n]: |X_i| (the column sums of Eq. (4)).
 *  JAS_DB_WORDS         uint64[w_rows * w_stride]: the bitmask words (Sec. III-B) of
 *                       the rows shared by >= dense_min_degree sets, batch by batch
 *                       (Eq. (3)) and in ID order inside a batch; packed row p of a
 *                       batch is bit p mod b of word row floor(p / b) of that batch,
 *                       and word row r of all batches is element row r (b = 64) or the
 *                       low (r even) / high (r odd) half of element row r/2 (b = 32);
 *                       element (row, i) is at row * w_stride + i; columns >= n are 0.
 *  JAS_DB_LIST_PAIRS    uint32: for every row shared by 2..dense_min_degree-1 sets
 *                       (the row lists) and every pair a < b of its sets, the word
 *                       (a << 16) | b, ordered by a (kept when n <= 10240).
 *  JAS_DB_LIST_PTR, JAS_DB_LIST_SAMPLES  uint64 / uint32: the same rows as a CSR of
 *                       their sets, ascending (kept instead of the pairs when n > 10240).
 *  JAS_DB_KEYS          uint64: with JAS_KEEP_IDS, every distinct (ID, sample) as
 *                       (ID << ceil(log2 n)) | sample, ascending.
 * jas_db_part_size returns the part's element count (0 for an unknown part or a
 * NULL db).  jas_db_read copies count elements from element `first` into
 * host_out (synchronous, on the db's device); EINVAL for a range outside the
 * part.  Rows with a single set are not stored: they add only to |X_i|.
 */
#define JAS_DB_CARD 0
#define JAS_DB_WORDS 1
#define JAS_DB_LIST_PAIRS 2
#define JAS_DB_LIST_PTR 3
#define JAS_DB_LIST_SAMPLES 4
#define JAS_DB_KEYS 5
uint64_t jas_db_part_size(const jas_db *db, int32_t part);
jas_status jas_db_read(const jas_db *db, int32_t part, uint64_t first, uint64_t count, void *host_out);

/* Frees the db and its device memory (synchronises the device first). NULL is a no-op. */
void jas_db_free(jas_db *db);

/* Message of the last failing jas_* call on this thread ("" if none). */
const char *jas_last_error(void);

/* Library version string. */
const char *jas_version(void);

/* Device memory: the library keeps freed device buffers for reuse by later
 * calls (ordered across streams by events), so repeated calls of the same size
 * allocate nothing.  jas_trim synchronises the device and returns every cached
 * buffer to it.  Buffers held by live dbs are not affected. */
void jas_trim(void);

/*
 * Per-kernel timing (tracing).  While enabled, the library records a HIP event
 * before and after every kernel it launches, on the stream it launches the
 * kernel on, and jas_timing_report waits for those events and returns the
 * elapsed time summed by kernel name.  Process-wide; off by default.
 */
typedef struct {
    const char *name;  /* static string, valid for the life of the library */
    uint64_t launches;
    double total_ms;
} jas_kernel_time;

void jas_timing_enable(int32_t on);
/* Fills up to cap entries (largest total first), returns the number of kernels
 * timed since the last reset, and resets the totals.  Synchronises on the
 * recorded events. */
int32_t jas_timing_report(jas_kernel_time *out, int32_t cap);

#ifdef __cplusplus
}
#endif

#endif /* JAS_H */
