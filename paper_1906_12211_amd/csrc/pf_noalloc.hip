// Allocation-free search: pf_search's computation with every per-call device buffer
// (normalised and hashed queries, hashing scratch, decision tables, prefix ranges and the
// list of large prefix buckets, the bad-row flag) carved from one file-scope device array
// instead of the index's grow-on-demand buffers, so that the call makes no device
// allocation.  For callers that cannot allocate (code under graph capture, tight serving
// loops).  Every call on a device shares that device's array: calls that overlap on one
// device race.
#include <cmath>
#include <cstring>
#include <mutex>
#include <string>

#include "pf_internal.h"

#define PF_API extern "C" __attribute__((visibility("default")))

namespace pf {

constexpr size_t kNoAllocScratch = 64ull << 20; // bytes of the array on each device

// the array itself; host code never passes its name to a kernel (on the host it is only
// a stand-in for the symbol): it uses the device address that hipGetSymbolAddress returns
static __device__ __align__(256) unsigned char scratch[kNoAllocScratch];

constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static void *g_scratch_dev[kMaxDevices];

// device address of `scratch` on the current device, looked up once per device
static unsigned char *scratch_on_current_device() {
    int dev = 0;
    PF_HIP(hipGetDevice(&dev));
    PF_CHECK(dev >= 0 && dev < kMaxDevices, PF_EUNSUPPORTED, "pf_search_noalloc: device index out of range");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_dev[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        PF_CHECK(e == hipSuccess && p, PF_EDEVICE,
                 std::string("pf_search_noalloc: hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
        g_scratch_dev[dev] = p;
    }
    return static_cast<unsigned char *>(g_scratch_dev[dev]);
}

static size_t up256(size_t b) { return (b + 255) / 256 * 256; }

// byte offsets of the per-call buffers of m queries inside the scratch array
struct NoAllocLayout {
    size_t flag, dl, tab, qX, qcode, qsk, hscr, ranges, rlist, total;
};

static NoAllocLayout noalloc_layout(const Index &ix, int64_t m) {
    NoAllocLayout o;
    size_t at = 0;
    auto take = [&](size_t b) {
        const size_t p = at;
        at += up256(b);
        return p;
    };
    o.flag = take(sizeof(unsigned long long));
    o.dl = take(sizeof(double));
    o.tab = take((65 + (size_t)ix.K * default_groups(ix.L) * rule_table_cols()) * sizeof(float));
    o.qX = take((size_t)m * ix.dpad * sizeof(float));
    o.qcode = take((size_t)m * ix.L * sizeof(uint32_t));
    o.qsk = take((size_t)m * ix.M * sizeof(uint64_t));
    o.hscr = take(hash_scratch_bytes(ix, m));
    const int32_t nl = ix.K - ix.P;
    o.ranges = take(nl > 0 ? (size_t)m * ix.L * nl * 2 * sizeof(uint32_t) : 0);
    o.rlist = take(nl > 0 ? ranges_list_bytes(m, ix.L) : 0);
    o.total = at;
    return o;
}

static void noalloc_search(pf_index *ix, const float *queries, int64_t m, int32_t k, double recall,
                           int32_t *out_ids, float *out_ips, pf_query_stats *stats, void *stream) {
    PF_CHECK(ix, PF_EINVAL, "pf_search_noalloc: null index");
    PF_CHECK(m >= 0 && (m == 0 || (queries && out_ids)), PF_EINVAL, "pf_search_noalloc: bad arguments");
    PF_CHECK(k >= 1 && k <= PF_MAX_K && k <= ix->n, PF_EINVAL, "pf_search_noalloc: k must be in [1, min(n, 256)]");
    PF_CHECK(recall > 0.0 && recall <= 1.0, PF_EINVAL, "pf_search_noalloc: recall must be in (0, 1]");
    if (m == 0) return;
    const NoAllocLayout lay = noalloc_layout(*ix, m);
    PF_CHECK(lay.total <= kNoAllocScratch, PF_EUNSUPPORTED,
             "pf_search_noalloc: " + std::to_string(m) + " queries need " + std::to_string(lay.total) +
                 " bytes of scratch, more than the " + std::to_string(kNoAllocScratch) +
                 " bytes the library holds; split the batch or call pf_search");
    int dev = 0;
    PF_HIP(hipGetDevice(&dev));
    PF_CHECK(dev == ix->device, PF_EINVAL, "pf_search_noalloc: the current device is not the index's");
    unsigned char *base = scratch_on_current_device();
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);

    // normalise (bad-row flag starts at all ones: no bad row), then hash
    unsigned long long *flag = reinterpret_cast<unsigned long long *>(base + lay.flag);
    float *qX = reinterpret_cast<float *>(base + lay.qX);
    uint32_t *qcode = reinterpret_cast<uint32_t *>(base + lay.qcode);
    uint64_t *qsk = reinterpret_cast<uint64_t *>(base + lay.qsk);
    launch_fill_u32(reinterpret_cast<uint32_t *>(flag), 2, 0xFFFFFFFFu, s);
    launch_normalize(queries, m, ix->d, ix->d, qX, ix->dpad, flag, s);
    unsigned long long bad = 0;
    PF_HIP(hipMemcpyAsync(&bad, flag, sizeof(bad), hipMemcpyDeviceToHost, s));
    PF_HIP(hipStreamSynchronize(s));
    PF_CHECK(bad == ~0ull, PF_EINVAL, "row " + std::to_string(bad) + " has zero or non-finite norm");
    hash_rows_into(*ix, qX, m, qcode, qsk, reinterpret_cast<char *>(base + lay.hscr), s);

    // decision tables of the default rule for delta = 1 - recall (ln delta written by a fill)
    const double lnd = std::log(1.0 - recall);
    uint64_t lbits;
    std::memcpy(&lbits, &lnd, sizeof lbits);
    uint32_t *dlw = reinterpret_cast<uint32_t *>(base + lay.dl);
    launch_fill_u32(dlw, 1, (uint32_t)(lbits & 0xFFFFFFFFu), s);
    launch_fill_u32(dlw + 1, 1, (uint32_t)(lbits >> 32), s);
    float *tab = reinterpret_cast<float *>(base + lay.tab);
    const int32_t G = default_groups(ix->L);
    launch_rule_tables(reinterpret_cast<const double *>(dlw), 1, 0.0, PF_RULE_FILTER, ix->L, ix->M, ix->K, G,
                       ix->pool, ix->family == PF_FAMILY_FHTCP ? ix->cptab.as<double>() : nullptr, ix->cp_ell, tab,
                       tab + 65, s);

    SearchArgs a;
    a.Q = qX;
    a.qcode = qcode;
    a.qsk = qsk;
    a.m = m;
    a.qstride = m;
    a.ks = nullptr;
    a.kconst = k;
    a.kmax = k;
    a.qtab = nullptr;
    a.tauv = tab;
    a.stopw = tab + 65;
    a.B = 12;
    a.groups = G;
    a.test_entries = test_entries_of(0);
    a.filter = 1;
    a.prefilter = 1;
    a.queue = nullptr;
    a.order = nullptr;
    a.tile = search_default_tile();
    a.waves_per_cu = 0;
    a.out_ids = out_ids;
    a.out_ips = out_ips;
    a.stats = stats;
    uint32_t *rg = ix->K > ix->P ? reinterpret_cast<uint32_t *>(base + lay.ranges) : nullptr;
    launch_ranges_into(*ix, a, rg, reinterpret_cast<uint32_t *>(base + lay.rlist), s);
    launch_search(*ix, a, rg, s);
    // results are complete on return, and the next call may reuse the array
    PF_HIP(hipStreamSynchronize(s));
}

} // namespace pf

PF_API int pf_search_noalloc(pf_index *ix, const float *queries, int64_t m, int32_t k, double recall,
                             int32_t *out_ids, float *out_ips, pf_query_stats *stats, void *stream) {
    try {
        pf::noalloc_search(ix, queries, m, k, recall, out_ids, out_ips, stats, stream);
        return PF_OK;
    } catch (const pf::Error &e) {
        pf::set_last_error(e.what());
        return e.code;
    } catch (const std::exception &e) {
        pf::set_last_error(e.what());
        return PF_EDEVICE;
    }
}
