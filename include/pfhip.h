/*
 * pfhip.h -- C-ABI of the MI355X (gfx950) adaptive k-NN index after PUFFINN
 * (Aumueller, Christiani, Pagh, Vesterli, ESA 2019).
 *
 * The user supplies only a memory budget for the index and the recall a query must
 * reach (Sec. 1, Sec. 5 "Parameter Choices"); everything else has a default.
 *
 * Conventions for every entry point
 *  - Return value: PF_OK (0) or a negative PF_E* code; on error the outputs are left
 *    untouched and pf_last_error() returns a message (thread-local).
 *  - `mem` says where the caller's buffers live: PF_HOST (ordinary host memory; the
 *    call copies through device memory and returns after the results are on the host)
 *    or PF_DEVICE (device pointers on the current HIP device; the call is ordered on
 *    `stream` and returns after queueing unless stated otherwise).  A call never keeps
 *    a caller pointer after it returns; the caller owns every input and output buffer.
 *  - `stream` is a hipStream_t passed as void* (NULL = the null stream).  Streams must
 *    have the default priority.
 *  - An index is not thread-safe: calls on the same index must not overlap.
 *  - An index keeps the device buffers its searches need, grown on demand, until
 *    pf_free_index: a search allocates device memory only when it is larger (more
 *    queries, larger k, more distinct recalls) than every earlier one on the index.
 *  - Layouts are row-major; "n x d" means n rows of d contiguous FP32 values.
 */
#ifndef PFHIP_H
#define PFHIP_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define PF_OK 0
#define PF_EINVAL (-1)       /* bad argument, zero or non-finite vector row          */
#define PF_EBUDGET (-2)      /* the memory budget holds no table (L < 1)             */
#define PF_ENOMEM (-3)       /* device or host allocation failed                     */
#define PF_EDEVICE (-4)      /* a HIP runtime call failed                            */
#define PF_EUNSUPPORTED (-5) /* outside the implemented limits (see each call)       */

#define PF_HOST 0
#define PF_DEVICE 1

/* stopping rules, see pf_search_opts.rule */
#define PF_RULE_FILTER 0 /* Lemma 1's bound with the sketch filter's misses (default)    */
#define PF_RULE_EXACT 1  /* Lemma 1's bound (1 - p^i)^L <= delta, filter not accounted   */
#define PF_RULE_ALG1 2   /* Algorithm 1's printed test L >= ln(1/delta) / p^i            */
#define PF_RULE_POOL 3   /* Algorithm 3 (pooling, App. B): L p^i >= 2 and m >= 5 i^2 / p;
                            failure probability at most 1/2 whatever the recall; needs an
                            index built with a pool                                       */

/* hashing arithmetic, see pf_build_opts.hash_mode */
#define PF_HASH_BF16X3 0 /* BF16 MFMA (three split products, FP32 accumulate), bits whose
                            |projection| is within the derived error bound recomputed in FP64 */
#define PF_HASH_FP64 1   /* every projection as a sequential FP64 sum */

/* what pf_export copies */
#define PF_EXPORT_POINTS 0      /* n x d FP32, the normalised vectors                  */
#define PF_EXPORT_HYPERPLANES 1 /* (L*K + 64*M) x d FP32; with a pool (m + 64*M) x d:
                                   the pool functions, then the sketch functions        */
#define PF_EXPORT_CODES 2       /* L x n u32, sorted codes of each table (rebuilt from
                                   the prefix table and the stored low K - P bits)     */
#define PF_EXPORT_IDX 3         /* L x n u32, point position of each sorted entry (widened from the stored bytes) */
#define PF_EXPORT_SKETCHES 4    /* L x n u64, table-local sketches                     */
#define PF_EXPORT_OFFSETS 5     /* L x (2^P + 1) u32, P = pf_info.P, prefix table      */
#define PF_EXPORT_POOL_SEL 6    /* L x K int32: pool index of h_{t+1,j} (pooled index) */
#define PF_EXPORT_CP_TABLE 7    /* 41 x (ell + 1) FP64: Monte Carlo collision probability of
                                   b-bit prefixes at similarity -1 + 0.05 g (FHT-CP index) */
#define PF_EXPORT_ROWS8 8       /* n x (8 + dpad) bytes, dpad = 4 ceil(d / 4): the 8-bit
                                   row summaries the re-rank bounds candidates with; row:
                                   FP32 scale s = max_i |x_i| / 127, int32 A = sum_i |c_i|,
                                   then int8 c_i = rint(x_i / s), zero padded (x the
                                   normalised vector; IEEE FP32 division).  Where 8 + dpad
                                   bytes take another 128-byte line than dpad (dpad = 121
                                   .. 128, 249 .. 256, ...) every row has the scale of the
                                   largest |x_i| of all rows, and the search bounds with
                                   the largest A of all rows                              */

/* hash families of the table codes (the sketches are always random-hyperplane bits) */
#define PF_FAMILY_HP 0    /* random hyperplanes (Sec. 2.2), one bit per function          */
#define PF_FAMILY_FHTCP 1 /* cross-polytope with three Hadamard rotations (Sec. 2.2, 4.3),
                             ell = log2(2 d') bits per function, d' the power of two >= d  */

/* limits of this implementation */
#define PF_MAX_TABLES 512
#define PF_MAX_K 256 /* neighbours per query */
#define PF_MAX_DIM 4096

typedef struct pf_index pf_index; /* opaque; owns all of its device memory */

typedef struct {
    uint64_t seed;      /* hyperplane seed (counter-based SplitMix64 + Box-Muller)  */
    int32_t K;          /* bits per table code, 1..32; 0 selects 24                 */
    int32_t M;          /* 64-bit sketches per point, 1..64; 0 selects 32           */
    int32_t hash_mode;  /* PF_HASH_BF16X3 (default) or PF_HASH_FP64                  */
    int32_t L_override; /* > 0: use exactly this many tables, ignore the budget rule  */
    int32_t pool;       /* 0: K independent functions per table (Algorithm 1);
                           m > 0: pooling (Sec. 3.2), every table samples K of m shared
                           functions without replacement; m a multiple of 32 in [K, 65536] */
    int32_t family;     /* PF_FAMILY_HP (default) or PF_FAMILY_FHTCP (no pool)          */
    int32_t pos_bytes;  /* bytes per stored table position: 0 or 4 selects 4; 3 (n <= 2^24,
                           else PF_EINVAL) packs them in 3 bytes, which frees n bytes per
                           table for the budget but makes each position read an unaligned
                           load (slower for queries that scan few entries)               */
    int32_t prefix_bits; /* P, the width of the prefix table: 0 selects the width in
                           [min(13, K), min(24, K)] with the fewest resident bytes per table
                           (see pf_build_index); else a width in that range               */
} pf_build_opts;

/* All-zero options are the defaults. */
typedef struct {
    double eps;        /* filter slack: tau = (1 + eps) * 64 * theta_k / pi; default 0 */
    int32_t B;         /* segment size of every array access; 0 selects 12             */
    int32_t rule;      /* PF_RULE_FILTER (default), PF_RULE_EXACT, PF_RULE_ALG1 or
                          PF_RULE_POOL (pooled index only)                              */
    int32_t no_filter; /* 1: sketch filter off (every retrieved candidate re-ranked)   */
    int32_t timing;    /* 1: record per-kernel durations of this call (pf_last_timing) */
    int32_t no_prefilter; /* 1: compute every re-ranked inner product from both 16-bit
                             planes (the upper-plane bound rules nothing out); results
                             are the same either way, only the bytes read differ       */
    int32_t tile;      /* 0: the default kernel tile shape (pf_search: the library's default;
                          pf_search_batch: the autotuned or cached one, else the default);
                          t + 1: shape t, 0 <= t < pf_tile_count()
                          (results are the same for every shape, only the speed differs);
                          PF_EINVAL beyond the count                                      */
    int32_t groups;    /* G: the L repetitions of a level are taken in G consecutive groups
                          (group g: repetitions floor(g L / G) .. floor((g+1) L / G) - 1)
                          and the stopping test runs after each group, with the
                          repetitions not yet at the level counted at the previous one:
                          1 = once per level (Sec. 4.1), L = after every repetition
                          (Algorithm 1); 0 selects the default, min(L, 16); at most
                          min(L, 64), PF_EINVAL beyond                                    */
    int32_t test_entries; /* T: a group's stopping test is taken only once at least T
                          entries were read since the level's previous test (always after
                          the level's last group; groups without entries that directly
                          follow a tested group are tested with it), so that a query
                          that reads few entries per group tests less often; 0 selects
                          the default, 256; a negative value tests after every group    */
} pf_search_opts;

typedef struct {
    int32_t stop_level; /* prefix length at which the query stopped (0 = linear scan) */
    int32_t wave_us;    /* microseconds the query occupied its wave (from taking it off the
                           queue to writing its results; the device's constant clock; not
                           part of the method) */
    int64_t c_scan;   /* entries taken from the sorted arrays                        */
    int64_t c_pass;   /* entries that passed the sketch filter (with multiplicity)   */
    int64_t c_rerank; /* candidates re-ranked (with multiplicity; + n at a linear scan) */
    int64_t c_exact;  /* of those, the ones whose exact FP32 inner product was needed:
                         the rest were ruled out by an upper bound of the inner product
                         (not part of the method's definition; depends on the order in
                         which the kernel met the candidates)                           */
    int64_t c_upper;  /* re-ranked candidates whose upper 16-bit plane was read        */
    int64_t c_q8;     /* re-ranked candidates bounded from their 8-bit row summary     */
} pf_query_stats;

typedef struct {
    int64_t n;
    int32_t d, L, K, M, P, pool; /* P: prefix-table width (pf_build_opts.prefix_bits);
                                    pool: m of a pooled index, 0 otherwise */
    int32_t family;              /* PF_FAMILY_* of the table codes               */
    uint64_t bytes_budget_rule; /* bytes the budget rule counts for this index (fixed +
                                   L per_table, see pf_build_index)                      */
    uint64_t bytes_device;      /* device bytes the index actually holds (equal to
                                   bytes_budget_rule)                                    */
    double build_ms;            /* device time of the last build, if measured         */
    int32_t pos_bytes;          /* bytes per stored table position (3 or 4)           */
} pf_info;

typedef struct {
    double normalize_ms, hash_ms, ranges_ms, search_ms, total_ms;
    int32_t tile;         /* tile shape the search kernel ran with (batched calls) */
    int32_t waves_per_cu; /* cap on resident query waves per CU (0 = occupancy limit) */
    double order_ms;      /* batched calls: the work queue's order (the learned scheduler's
                             features, network and sort, or the upload of a caller's order)
                             and the autotuner when asked; ranges_ms covers the decision
                             tables and the prefix ranges                                 */
    int64_t slots;        /* query waves the search kernel was launched with             */
    int32_t groups;       /* stopping tests per level the call used (pf_search_opts.groups) */
} pf_timing;

/* Measurement aid (not part of the method): the best read rate, in GB/s (10^9 bytes per
 * second), of a plain read-only streaming kernel (16-byte loads, four in flight per lane,
 * plain or non-temporal, 2, 8 or 32 workgroups of 256 lanes per CU; `reps` timed launches
 * of each after one warm-up) over a device buffer of `bytes` bytes that the call
 * allocates, fills and frees on the current device -- the read bandwidth that the
 * device's memory system delivers to a fully coalesced access pattern, against which the
 * search kernel's rate is also reported.  PF_EINVAL for bytes < 1 MiB, reps < 1 or gbs NULL; PF_ENOMEM, PF_EDEVICE.
 * Synchronises `stream`. */
int pf_read_bandwidth(uint64_t bytes, int32_t reps, double *gbs, void *stream);

/* Measurement aid (not part of the method): the best rate, in loads per second, of a
 * kernel whose every lane issues 64 scattered 4-byte reads (eight in flight; word
 * indices from SplitMix64, masked to the largest power-of-two word count that fits in
 * `bytes`; plain or non-temporal loads; 64 workgroups of 256 lanes per CU; `reps` timed
 * launches of each after one warm-up) over a device buffer the call allocates, fills and
 * frees on the current device.  The streaming read rate of pf_read_bandwidth divided by
 * this rate is the memory traffic one scattered 4-byte read costs, as the search kernel
 * pays it for the point id of each entry that passes the sketch filter.  PF_EINVAL for
 * bytes < 1 MiB, reps < 1 or loads_per_s NULL; PF_ENOMEM, PF_EDEVICE.  Synchronises
 * `stream`. */
int pf_random_read_rate(uint64_t bytes, int32_t reps, double *loads_per_s, void *stream);

/* Number of kernel tile shapes the library is built with, and the name of shape t
 * (a static string; "?" when t is out of range). */
int32_t pf_tile_count(void);
const char *pf_tile_name(int32_t t);

/* pf_search_batch flags */
#define PF_BATCH_LEARNED 1  /* order the work queue longest-predicted-first by the
                               scheduler attached with pf_index_set_scheduler */
#define PF_BATCH_AUTOTUNE 2 /* time the built tile shapes on this batch and keep the fastest
                               (cached per architecture, index shape, kmax and position width;
                               also in the JSON-lines file named by the environment variable
                               PF_TUNE_CACHE) */

/* Normalise n rows to unit length (Sec. 4.2, "Vector storage"): squared norm summed in
 * FP64 in index order, FP64 square root and division, each quotient rounded once to
 * FP32.  x and out are n x d (may alias).  PF_EINVAL when a row has zero or non-finite
 * norm (out is then unspecified). */
int pf_normalize(const float *x, int64_t n, int32_t d, float *out, int32_t mem, void *stream);

/* Build the index of Sec. 4.1-4.2 over n points of dimension d:
 *  L = floor((budget - fixed) / per_table) tables, capped at PF_MAX_TABLES and at
 *  floor((2^32 - 2^16 - 1) / n) (32-bit table positions), where the
 *  budget counts every byte the index keeps on the device (Sec. 1, Sec. 5.2: the data
 *  set and the hash functions are part of the index size): fixed = the vectors (two
 *  16-bit planes, 4 dpad bytes per row up to line padding) and their 8-bit summaries
 *  (PF_EXPORT_ROWS8 layout, whole 128-byte lines per row, + 8 bytes per row when the rows
 *  share one scale), the 64 M sketch hyperplanes and their BF16 GEMM copies, and 8 bytes
 *  of padding after the positions; per_table = the table-local sketches (8n), the
 *  positions (4n, or 3n with pos_bytes = 3), the sorted codes' low K - P bits (n when
 *  K - P <= 8, 2n when K - P <= 16, 4n when larger, none when K <= P: the prefix table
 *  holds the leading P bits of every entry's code), the prefix table (4 (2^P + 1)), the
 *  table's K hyperplanes (4Kd) and their GEMM copy; by default P is the width in
 *  [min(13, K), min(24, K)] that makes the codes' share (prefix table and low bits) the
 *  smallest: P = 16 for K = 24 and n above about 229,000, else 13.  For n = 10^6,
 *  d = 100, 2 GiB this gives L = 121 (the paper's count, with 4-byte codes and positions
 *  and without the summaries, gives 108);
 *  pf_info.bytes_device <= budget always holds;
 *  K random-hyperplane functions per table (Sec. 2.2), M 64-bit sketches per point
 *  (Sec. 4.2), each table sorted by its K-bit code with equal codes by position, and a
 *  table of the positions of every P-bit prefix (Sec. 4.2).
 *  With opts->pool = m (Sec. 3.2 "Pooling"): m shared hyperplanes, each table's K
 *  functions drawn from them without replacement (Fisher-Yates on the SplitMix64 stream
 *  seeded with seed + 1), and the budget counts the m pool hyperplanes (with their GEMM
 *  copies) once and 4K bytes of indices per table instead of 4Kd.
 *  With opts->family = PF_FAMILY_FHTCP: each table's code is the first K bits of c =
 *  ceil(K / ell) cross-polytope values (rotation H D3 H D2 H D1 of the zero-padded point,
 *  FP64; value = sign of the largest coordinate as the top bit, then its index), the
 *  stopping rules read the collision probability of a prefix from a Monte Carlo table
 *  (1,000 functions per similarity -1, -0.95, ..., 1, made non-decreasing, similarity
 *  rounded down; Sec. 4.3), and the budget counts 3 c ceil(d' / 32) 32-bit words of
 *  signs per table and the collision table once.
 * `points` n x d (caller-owned, copied).  Errors: PF_EINVAL (n < 1, n >= 2^31, d < 1,
 * d > PF_MAX_DIM, bad row, K, M or pool out of range), PF_EBUDGET, PF_EUNSUPPORTED
 * (an explicit L_override with L n >= 2^32 - 2^16 table entries), PF_ENOMEM, PF_EDEVICE.
 * Synchronises the stream before returning. */
int pf_build_index(const float *points, int64_t n, int32_t d, uint64_t memory_budget_bytes,
                   const pf_build_opts *opts, int32_t mem, void *stream, pf_index **out);

/* The table count L and the device bytes (fixed + L per_table) that pf_build_index would
 * use for n points of dimension d under `budget` and `opts` (nullable = defaults): the
 * budget rule above, evaluated on the host without touching a device.  L and
 * bytes_device are nullable.  Errors as pf_build_index's argument checks (PF_EINVAL,
 * PF_EBUDGET, PF_EUNSUPPORTED). */
int pf_plan_index(int64_t n, int32_t d, uint64_t budget, const pf_build_opts *opts, int32_t *L,
                  uint64_t *bytes_device);

/* Answer m queries (Algorithm 1, adaptive-kNN(q, k, delta), with delta = 1 - recall,
 * Sec. 2.1), level-synchronously as in Sec. 4.1: in each round every table contributes
 * the new entries sharing the query's i-bit prefix, read in whole segments of B
 * entries (Sec. 4.2, App. C); candidates pass when the Hamming distance of their
 * sketch is at most the threshold of the round (Sec. 4.2, Sec. 5.1); survivors not
 * yet seen are re-ranked by exact FP32 inner product into the top-k; after all tables
 * the stopping bound of Lemma 1 is tested in FP64 -- by default extended by the
 * probability that the filter rejects a true neighbour, so that each returned point
 * is a true k-NN with probability at least 1 - delta with the filter on; at prefix
 * length 0 the query is a linear scan.  `queries` m x d; out_ids m x k (int32, best first: inner product
 * descending, position ascending); out_ips m x k FP32 (nullable); stats m (nullable).
 * Errors: PF_EINVAL (k < 1, k > n, k > PF_MAX_K, recall outside (0, 1], bad row, d
 * mismatch), PF_ENOMEM, PF_EDEVICE.  The call synchronises `stream` before returning, with
 * PF_DEVICE too: the rows are checked for zero and non-finite values first, and the
 * next call on the index reuses its device buffers. */
int pf_search(pf_index *ix, const float *queries, int64_t m, int32_t k, double recall,
              int32_t *out_ids, float *out_ips, pf_query_stats *stats, int32_t mem,
              void *stream);

/* pf_search without any device allocation, for callers that cannot allocate (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * computation and results as pf_search with default options, but every per-call device
 * buffer (normalised and hashed queries, hashing scratch, decision tables, prefix ranges)
 * lives in one static device array of the library, 64 MiB on each device that calls it,
 * held until the process ends.  queries (m x d), out_ids (m x k), out_ips (m x k,
 * nullable) and stats (m, nullable) are device pointers on the index's device; the call is
 * ordered on `stream` and synchronises it before returning.  All calls on one device share
 * that device's array: calls that overlap in time on one device race (one at a time per
 * device).  Errors: as pf_search; PF_EUNSUPPORTED when the m queries' buffers exceed the
 * 64 MiB array (e.g. about 6,500 queries at n = 10^6, d = 100, L = 121: split the batch);
 * PF_EINVAL when the current device is not the index's. */
int pf_search_noalloc(pf_index *ix, const float *queries, int64_t m, int32_t k, double recall,
                      int32_t *out_ids, float *out_ips, pf_query_stats *stats, void *stream);

/* pf_search with explicit options (opts may be NULL for the defaults). */
int pf_search_ex(pf_index *ix, const float *queries, int64_t m, int32_t k, double recall,
                 const pf_search_opts *opts, int32_t *out_ids, float *out_ips,
                 pf_query_stats *stats, int32_t mem, void *stream);

/* Batched search: one persistent launch answers m queries with per-query k (ks[i] in
 * [1, kmax]; NULL = kmax for all) and per-query recall (recalls[i] in (0, 1], required),
 * taking queries from a device work queue so that queries of very different cost share
 * the GPU evenly.  The queue is consumed in the order `order` (a permutation of 0..m-1,
 * nullable = 0..m-1) or, with PF_BATCH_LEARNED, longest-predicted-first by the attached
 * scheduler; termination of every query is still decided by the stopping rule, so the
 * results do not depend on the order.  out_ids / out_ips are m x kmax; a query with
 * k < kmax is padded with id -1 and ip -inf.  Other arguments and errors as pf_search_ex. */
int pf_search_batch(pf_index *ix, const float *queries, int64_t m, const int32_t *ks,
                    const double *recalls, int32_t kmax, const pf_search_opts *opts,
                    const int32_t *order, int32_t *out_ids, float *out_ips, pf_query_stats *stats,
                    int32_t flags, int32_t mem, void *stream);

/* Hash m rows with the index's functions (Sec. 2.2: bit = 1 iff <a, x> >= 0) after
 * normalising them: codes L x m (u32, table-major, h_{1,j} the most significant of the
 * K bits), sketches M x m (u64, bit b from sketch hyperplane b).  Either output may be
 * NULL.  Errors: PF_EINVAL, PF_ENOMEM, PF_EDEVICE.  Synchronises. */
int pf_hash(pf_index *ix, const float *x, int64_t m, uint32_t *codes, uint64_t *sketches,
            int32_t mem, void *stream);

/* Copy one resident structure of the index (PF_EXPORT_*) into dst, which must hold
 * dst_bytes >= the structure's size (PF_EINVAL otherwise).  Synchronises. */
int pf_export(const pf_index *ix, int32_t what, void *dst, int64_t dst_bytes, int32_t mem,
              void *stream);

int pf_index_info(const pf_index *ix, pf_info *info);

/* Per-kernel device durations of the last pf_search* call made with opts.timing = 1,
 * measured with HIP events recorded on the call's stream around each launch. */
int pf_last_timing(const pf_index *ix, pf_timing *t);

void pf_free_index(pf_index *ix);

/* ---------------------------------------------------------------- learned scheduler
 * A small network predicts, for each query, the prefix length at which the plain
 * method stops and log2(1 + entries it scans), from the query's 64 sketch-0 bits (+1/-1),
 * log2(1 + size of its 13-bit prefix bucket) in tables 0..31, log2 k and log2(1/delta)
 * (delta = 1 - recall; 40 when delta < 2^-40).  pf_search_batch with
 * PF_BATCH_LEARNED answers the predicted-costliest queries first (longest processing
 * time first), which shortens the tail of the batch; the stopping rule still decides
 * when each query ends, so results are unchanged.  Network: 98 -> 128 ReLU -> 128 ReLU
 * -> 2, FP32, mean squared error, Adam; parameters in one flat FP32 array
 * W1[98][128], b1[128], W2[128][128], b2[128], W3[128][2], b3[2] (y = x W + b). */
#define PF_SCHED_IN 98
#define PF_SCHED_OUT 2
#define PF_SCHED_PARAMS 29442

typedef struct pf_sched pf_sched;

/* He-uniform weights from the counter-based generator seeded with `seed`, zero biases. */
int pf_sched_create(uint64_t seed, pf_sched **out);
void pf_sched_free(pf_sched *s);
/* copy the PF_SCHED_PARAMS host floats out of (get = 1) or into (get = 0) the network */
int pf_sched_params(pf_sched *s, float *params, int32_t get);
/* features of m queries (m x 98 FP32) under index ix; queries are normalised and hashed;
 * per-query k (ks, nullable: kconst) and recall (recalls, nullable: recall_const) in the
 * same memory as the queries.  PF_EINVAL for k < 1 or recall outside (0, 1]. */
int pf_features(pf_index *ix, const float *queries, int64_t m, const int32_t *ks, const double *recalls,
                int32_t kconst, double recall_const, float *feat, int32_t mem, void *stream);
/* predictions (m x 2: stop level, log2(1 + entries scanned)) */
int pf_sched_predict(pf_sched *s, const float *feat, int64_t m, float *out, int32_t mem, void *stream);
/* loss (mean of the m x 2 squared errors) and its gradient w.r.t. every parameter */
int pf_sched_grad(pf_sched *s, const float *feat, const float *target, int64_t m, float *grad, double *loss,
                  int32_t mem, void *stream);
/* minibatch Adam (beta1 0.9, beta2 0.999, eps 1e-8) over `epochs` shuffled passes of the m
 * traces (feat m x 98, target m x 2); epoch_loss (nullable) receives the mean batch loss of
 * each epoch.  Synchronises. */
int pf_sched_train(pf_sched *s, const float *feat, const float *target, int64_t m, int32_t epochs,
                   int32_t batch, float lr, uint64_t seed, float *epoch_loss, int32_t mem, void *stream);
int pf_sched_save(pf_sched *s, const char *path);
int pf_sched_load(pf_sched *s, const char *path);
/* the scheduler PF_BATCH_LEARNED uses for this index (not owned; NULL detaches) */
int pf_index_set_scheduler(pf_index *ix, pf_sched *s);

const char *pf_last_error(void);
const char *pf_version(void);

#ifdef __cplusplus
}
#endif
#endif /* PFHIP_H */
