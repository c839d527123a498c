// Internal declarations of the gfx950 library: the index object, kernel launchers and
// small device helpers.  Not part of the C-ABI.
#pragma once
#include <hip/hip_runtime.h>

#include <algorithm>
#include <map>
#include <cstdint>
#include <stdexcept>
#include <string>
#include <vector>

#include "../../include/pfhip.h"

namespace pf {

struct Error : std::runtime_error {
    int code;
    Error(int c, const std::string &m) : std::runtime_error(m), code(c) {}
};

#define PF_HIP(call)                                                                     \
    do {                                                                                 \
        hipError_t e_ = (call);                                                          \
        if (e_ != hipSuccess)                                                            \
            throw ::pf::Error(e_ == hipErrorOutOfMemory ? PF_ENOMEM : PF_EDEVICE,        \
                              std::string(#call) + ": " + hipGetErrorString(e_));        \
        } while (0)

#define PF_CHECK(cond, code, msg)                                                        \
    do {                                                                                 \
        if (!(cond)) throw ::pf::Error((code), (msg));                                   \
    } while (0)

// Device allocation held by the index (RAII, freed with hipFree).
struct DevBuf {
    void *p = nullptr;
    size_t bytes = 0;
    DevBuf() = default;
    DevBuf(const DevBuf &) = delete;
    DevBuf &operator=(const DevBuf &) = delete;
    ~DevBuf() { release(); }
    void alloc(size_t b) {
        release();
        if (b == 0) b = 16;
        PF_HIP(hipMalloc(&p, b));
        bytes = b;
    }
    void ensure(size_t b) {
        if (bytes < b) alloc(b);
    }
    // kernels queued on any stream may still use the buffer: wait for them before freeing
    void release() {
        if (p) {
            (void)hipDeviceSynchronize();
            (void)hipFree(p);
        }
        p = nullptr;
        bytes = 0;
    }
    template <class T> T *as() const { return static_cast<T *>(p); }
};

// Hyperplane matrix laid out for the hash GEMM: 32 output columns per 32-bit word.
//   word w < L        : table w's code, column c of the word = code bit c
//                       (c < K: hyperplane h_{K-c, w}; c >= K: zero padding)
//   word L + 2m + h    : sketch m, bits 32h .. 32h+31
// With a pool of m functions the first m / 32 words hold the pool bits (column c of word
// w = pool function 32 w + c) and table codes are gathered from them afterwards.
struct HashPlan {
    int32_t d = 0, dpad = 0, kp = 0; // kp: reduction length padded to the MFMA step
    int32_t L = 0, K = 0, M = 0;
    int32_t cw = 0;     // code words: L, or m / 32 with a pool
    int32_t pool = 0;   // m (0: independent functions)
    int32_t words = 0;  // cw + 2M
    int32_t ncols = 0;  // 32 * words
};

struct Index {
    int64_t n = 0;
    int32_t d = 0, dpad = 0, L = 0, K = 0, M = 0, P = 0;
    int32_t hash_mode = PF_HASH_BF16X3;
    int32_t pool = 0; // m of a pooled index (0: independent functions)
    int32_t family = PF_FAMILY_HP;
    int32_t cp_dp = 0, cp_ell = 0, cp_c = 0; // FHT-CP: padded dimension, bits per value, values per code
    uint64_t seed = 0;
    uint64_t bytes_rule = 0;
    double build_ms = 0.0;
    HashPlan plan;
    int device = 0;
    int num_cus = 0;
    double wall_khz = 0.0; // rate of the device's constant clock (wall_clock64)

    // n x dpad FP32 normalised vectors (zero padded), stored as two 16-bit planes: the
    // upper halves of the bit patterns (the vectors truncated to bfloat16; rows of hs
    // elements, padded to whole lines where the padding holds lower halves) and the
    // remaining lower halves (rows of ls elements); the re-rank reads the upper plane
    // first and the lower halves only where the truncated inner product cannot rule a
    // candidate out
    DevBuf Xh, Xl;
    int32_t hs = 0, ls = 0;
    // 8-bit summary of every row (scale, sum of |codes|, int8 codes; rq bytes per row,
    // codes from byte qco), read first by the re-rank: a candidate whose bound from it is
    // below the current k-th inner product is ruled out without reading either plane.
    // qco = 0: every row has the scale s8, no row's sum of |codes| exceeds a8, and the
    // 8-byte headers sit in Xqh for the export
    DevBuf Xq, Xqh;
    int32_t rq = 0, qco = 0;
    float s8 = 0.0f;
    int32_t a8 = 0;
    DevBuf hp;     // (L*K + 64*M) x d FP32 hyperplanes (paper order); pooled: (m + 64*M) x d
    DevBuf psel;   // pooled: L x K int32, pool index of h_{t+1,j}
    DevBuf cpsign; // FHT-CP: (L c) x 3 x d'/32 u32 sign bits (bit set = -1)
    DevBuf cptab;  // FHT-CP: 41 x (ell + 1) FP64 collision table
    DevBuf hcolrow;// ncols int32: hyperplane row of each GEMM column (-1 = padding)
    DevBuf hbf;    // ncols x kp bf16 hi parts, then ncols x kp bf16 lo parts
    DevBuf hbeta;  // ncols FP32 flag bounds (negative = never flagged)
    DevBuf tsuf;   // L x n low K - P bits of the sorted codes (sufw bytes each; none when K <= P)
    int32_t sufw = 0;
    DevBuf tpos;   // L x n table positions, posb bytes each (little endian), then kPosPad bytes
    int32_t posb = 4;
    DevBuf tsk;    // L x n u64
    DevBuf off;    // L x (2^P + 1) u32

    // search scratch (grown on demand)
    DevBuf qX, qcode, qsk, ranges, qstats, flags, tmp;
    DevBuf rlist; // count, then the (query, table) pairs whose prefix bucket is large
    // per-call buffers of the search (outputs for host callers, per-query k and decision
    // rows, work-queue counter and order), grown on demand and kept
    DevBuf c_ids, c_ips, c_stats, c_ks, c_qtab, c_queue, c_order;
    DevBuf hscratch; // hashing scratch of query rows (pool bits, cross-polytope temporaries)
    // learned queue order scratch: features, per-query parameters (and their host copy,
    // kept until the next call so that its asynchronous upload never reads freed memory),
    // sort keys, sort scratch
    DevBuf sfeat, sqp, skeys, ssort;
    std::vector<float> sqph;
    // decision tables of the last (rule, eps, deltas) searched
    DevBuf rule_tab;
    int32_t rule_key_rule = -1, rule_key_filter = -1, rule_key_groups = -1;
    double rule_key_eps = 0.0;
    std::vector<double> rule_key_lndeltas;
    pf_timing timing{};
    // autotuned tile shapes per (arch, n, d, L, kmax)
    struct Tuned {
        int32_t tile, waves;
        double us;
    };
    std::map<std::string, Tuned> tuned;
    struct Sched *sched = nullptr; // learned scheduler used by PF_BATCH_LEARNED (not owned)
};

// ----------------------------------------------------------------- learned scheduler
// MLP 98 -> 128 (ReLU) -> 128 (ReLU) -> 2, FP32, parameters in one flat array:
// W1 [98][128], b1 [128], W2 [128][128], b2 [128], W3 [128][2], b3 [2]
constexpr int kSchedIn = 98, kSchedHidden = 128, kSchedOut = 2;
constexpr int64_t kOffW1 = 0;
constexpr int64_t kOffB1 = kOffW1 + (int64_t)kSchedIn * kSchedHidden;
constexpr int64_t kOffW2 = kOffB1 + kSchedHidden;
constexpr int64_t kOffB2 = kOffW2 + (int64_t)kSchedHidden * kSchedHidden;
constexpr int64_t kOffW3 = kOffB2 + kSchedHidden;
constexpr int64_t kOffB3 = kOffW3 + (int64_t)kSchedHidden * kSchedOut;
constexpr int64_t kSchedParams = kOffB3 + kSchedOut; // 29,186
// chunk partial sums of the weight gradient: at most kWgradChunks chunks of the largest layer
constexpr int64_t kWgradChunks = 64;
constexpr int64_t kWgradScratch = kWgradChunks * ((int64_t)kSchedHidden * kSchedHidden + kSchedHidden);

struct Index;
// features of m queries; qparam: m x 2 (log2 k, log2(1/delta)) on the device
void launch_features(const Index &ix, const uint32_t *qcode, const uint64_t *qsk, int64_t m,
                     const float *qparam, float *feat, hipStream_t s);
// the two per-query parameter features, FP64 then rounded: log2 k, log2(1/delta) capped at 40
std::vector<float> sched_qparams(int64_t m, const int32_t *ks_host, int32_t kconst, const double *rec_host,
                                 double recall_const);
void mlp_forward(const float *params, const float *x, const int32_t *rows, int64_t B, float *h1, float *h2,
                 float *y, hipStream_t s);
void mlp_backward(const float *params, const float *x, const int32_t *rows, const float *tgt, int64_t B,
                  const float *h1, const float *h2, const float *y, float *dy, float *dh2, float *dh1, float *grad,
                  double *loss_acc, float *wscratch, hipStream_t s);
void mlp_adam(float *params, const float *grad, float *m1, float *m2, float lr, int32_t t, hipStream_t s);
// keys whose ascending order is the descending order of column 1 of y (B x 2); NaN last
void launch_lpt_keys(const float *y, int64_t B, uint32_t *keys, hipStream_t s);

// ----------------------------------------------------------------- launchers
// normalise: out[i][0..d) = x[i]/|x[i]|, zero-filled to dpad; *bad = min bad row (or n)
void launch_normalize(const float *x, int64_t n, int32_t d, int32_t ld_in, float *out,
                      int32_t dpad, unsigned long long *bad, hipStream_t s);

void launch_fill_u32(uint32_t *p, int64_t count, uint32_t v, hipStream_t s);
// X (n x dpad FP32) <-> upper / lower 16-bit planes (layout in k_prep.hip); hs, ls:
// elements per row of the upper and lower plane
void plane_strides(int32_t dpad, int32_t *hs, int32_t *ls);
void launch_split_planes(const float *X, int64_t n, int32_t dpad, uint16_t *hi, uint16_t *lo, hipStream_t s);
void launch_join_planes(const uint16_t *hi, const uint16_t *lo, int64_t n, int32_t dpad, float *X, hipStream_t s);
// 8-bit row summaries (layout in k_prep.hip) of X (n x dpad FP32, normalised): rq bytes
// per row, codes from byte co; co = 0: the 8-byte headers in hdr (n x 8), else unused
void rows8_layout(int32_t dpad, int32_t *rq, int32_t *co);
void launch_rows8(const float *X, int64_t n, int32_t dpad, uint8_t *out, uint8_t *hdr, uint32_t *gmax,
                  hipStream_t s);

// best rate (GB/s) of `reps` launches of a read-only streaming kernel over `bytes` bytes
double read_bandwidth_gbs(uint64_t bytes, int32_t reps, int32_t num_cus, hipStream_t s);
double random_read_rate(uint64_t bytes, int32_t reps, int32_t num_cus, hipStream_t s);

// hashing of rows X (n x dpad) into code words; see k_hash.hip.  hash_rows grows `scratch`
// to hash_scratch_bytes(ix, n); hash_rows_into takes a device scratch of that size
void hash_rows(const Index &ix, const float *X, int64_t n, uint32_t *codes, uint64_t *sketches,
               DevBuf &scratch, hipStream_t s);
size_t hash_scratch_bytes(const Index &ix, int64_t n);
void hash_rows_into(const Index &ix, const float *X, int64_t n, uint32_t *codes, uint64_t *sketches,
                    char *scratch, hipStream_t s);

// sorting and derived tables; see k_sort.hip
void sort_tables(const uint32_t *codes, int64_t n, int32_t L, int32_t K, uint32_t *tcode,
                 uint32_t *tidx, DevBuf &scratch, hipStream_t s);
void prefix_tables(const uint32_t *tcode, int64_t n, int32_t L, int32_t K, int32_t P,
                   uint32_t *off, hipStream_t s);
// resident sorted codes: the low K - P bits of each code (code_suffix_bytes per entry:
// 0 when K <= P, 1 when K - P <= 8, 2 when K - P <= 16, else 4), and the full codes rebuilt
// from them
int32_t code_suffix_bytes(int32_t K, int32_t P);
// prefix widths a table may use: [min(13, K), min(24, K)]; the default is the one with the
// fewest resident bytes for n entries
int32_t prefix_bits_min(int32_t K);
int32_t prefix_bits_max(int32_t K);
int32_t choose_prefix_bits(int64_t n, int32_t K);
void code_suffixes(const uint32_t *tcode, int64_t n, int32_t L, int32_t K, int32_t P, void *suf, hipStream_t s);
void join_codes(const void *suf, const uint32_t *off, int64_t n, int32_t L, int32_t K, int32_t P, uint32_t *out,
                hipStream_t s);
void gather_sketches(const uint32_t *tidx, const uint64_t *sk, int64_t n, int32_t L,
                     int32_t M, uint64_t *tsk, hipStream_t s);
// Table positions stored in posb bytes (3: n <= 2^24, little endian; 4) and widened back
constexpr int64_t kPosPad = 8;
int32_t pos_bytes_for(int64_t n, int32_t want);
// the search kernel for an index with 3-byte positions (row chunks dt, tile, shared-scale rows)
const void *search_kernel_pos3(int dt, int tile, bool shared);
// (pack_positions with posb 4 and in == out only writes the padding)
void pack_positions(const uint32_t *in, int64_t count, int32_t posb, uint8_t *out, hipStream_t s);
void unpack_positions(const uint8_t *in, int64_t count, int32_t posb, uint32_t *out, hipStream_t s);

// search; see k_search.hip
struct SearchArgs {
    const float *Q;        // m x dpad normalised
    const uint32_t *qcode; // L x m
    const uint64_t *qsk;   // M x m
    int64_t m;
    int64_t qstride;       // row stride of qcode / qsk (0 = m)
    const int32_t *ks;     // per-query k (nullable: kconst)
    int32_t kconst, kmax;
    const int32_t *qtab;   // per-query row of stopw (nullable: row 0)
    const float *tauv;     // 65 filter-threshold boundaries (see k_search.hip)
    const float *stopw;    // ndelta x K x groups x 66 stopping thresholds
    int32_t groups;        // groups of repetitions per level, the stopping test after each
    int32_t test_entries;  // ... once at least this many entries were read since the previous test
    int32_t B, filter;
    int32_t prefilter;     // 1: rule candidates out on the upper-plane inner product bound
    unsigned int *queue;   // device work-queue counter (nullable: static assignment)
    const int32_t *order;  // queue position -> query (nullable)
    int32_t tile;          // tile shape index (see search_tile_name)
    int32_t waves_per_cu;  // > 0: cap on resident query waves per CU
    int32_t *out_ids;      // m x kmax
    float *out_ips;        // m x kmax (nullable)
    pf_query_stats *stats; // m (nullable)
};
void launch_ranges(Index &ix, const SearchArgs &a, uint32_t *ranges, hipStream_t s);
// the same with the list of large prefix buckets in rlist (ranges_list_bytes(m, L) bytes)
size_t ranges_list_bytes(int64_t m, int32_t L);
void launch_ranges_into(const Index &ix, const SearchArgs &a, uint32_t *ranges, uint32_t *rlist, hipStream_t s);
void launch_rule_tables(const double *lndeltas_dev, int32_t ndelta, double eps, int32_t rule, int32_t L,
                        int32_t M, int32_t K, int32_t G, int32_t pool, const double *cptab, int32_t ell,
                        float *tauv, float *stopw, hipStream_t s);
// groups of repetitions per level when a call asks for the default (0)
int32_t default_groups(int32_t L);
// entries read between two stopping tests of a level for pf_search_opts.test_entries
// (0: the default, 256; negative: 0, a test after every group)
int32_t test_entries_of(int32_t opt);
// FHT-CP table codes of rows X (n x dpad) into codes (L x n); see k_hash.hip
void cp_codes(const Index &ix, const float *X, int64_t n, uint32_t *codes, hipStream_t s);
int32_t rule_table_cols();
// returns the number of query waves launched
int64_t launch_search(Index &ix, const SearchArgs &a, const uint32_t *ranges, hipStream_t s);
int32_t search_tile_count();
int32_t search_default_tile();
const char *search_tile_name(int32_t t);
int32_t search_waves_per_cu(const Index &ix, int32_t kmax, int32_t tile);

// normalise + hash caller rows into the index's query buffers (pf_api.cpp)
void prepare_rows_for(Index &ix, const float *x, int64_t m, int32_t mem, hipStream_t s, float **qX,
                      uint32_t **qcode, uint64_t **qsk);
// the thread-local message returned by pf_last_error
void set_last_error(const std::string &msg);

} // namespace pf

struct pf_index : public pf::Index {};
