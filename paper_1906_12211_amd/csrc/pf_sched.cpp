// Learned scheduler (C-ABI part): a small MLP predicts, from a query's sketch bits, the
// sizes of its first-level (13-bit prefix) buckets and its k and delta, the level at which the plain
// method stops and log2(1 + entries it scans).  The batched search orders its work
// queue longest-predicted-first; the stopping rule still ends every query, so results
// do not depend on the prediction.  Trained on the GPU with the kernels of k_mlp.hip.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <memory>
#include <numeric>
#include <string>
#include <vector>

#include "pf_internal.h"

#define PF_API extern "C" __attribute__((visibility("default")))

namespace pf {

struct Sched {
    DevBuf params, grad, m1, m2;
    DevBuf act;   // h1, h2, y, dy, dh2, dh1 for one batch
    DevBuf loss;  // FP64 accumulator
    DevBuf wscr;  // chunk partial sums of the weight gradients
    int64_t act_rows = 0;
    int32_t step = 0;
    uint64_t seed = 0;
    void ensure_act(int64_t B) {
        if (B <= act_rows) return;
        act.alloc((size_t)B * (4 * kSchedHidden + 2 * kSchedOut) * sizeof(float));
        act_rows = B;
    }
    float *h1() { return act.as<float>(); }
    float *h2() { return h1() + act_rows * kSchedHidden; }
    float *dh2() { return h2() + act_rows * kSchedHidden; }
    float *dh1() { return dh2() + act_rows * kSchedHidden; }
    float *y() { return dh1() + act_rows * kSchedHidden; }
    float *dy() { return y() + act_rows * kSchedOut; }
};

static inline uint64_t sm64(uint64_t seed, uint64_t s) {
    uint64_t z = seed + (s + 1u) * 0x9E3779B97F4A7C15ull;
    z ^= z >> 30;
    z *= 0xBF58476D1CE4E5B9ull;
    z ^= z >> 27;
    z *= 0x94D049BB133111EBull;
    z ^= z >> 31;
    return z;
}

// He-uniform initialisation: W ~ U(-sqrt(6/fan_in), sqrt(6/fan_in)), biases 0
static std::vector<float> init_params(uint64_t seed) {
    std::vector<float> p(kSchedParams, 0.0f);
    auto fill = [&](int64_t off, int64_t count, int fan_in) {
        const double lim = std::sqrt(6.0 / fan_in);
        for (int64_t i = 0; i < count; ++i) {
            const double u = (double)(sm64(seed, (uint64_t)(off + i)) >> 11) * 0x1.0p-53;
            p[off + i] = (float)((2.0 * u - 1.0) * lim);
        }
    };
    fill(kOffW1, (int64_t)kSchedIn * kSchedHidden, kSchedIn);
    fill(kOffW2, (int64_t)kSchedHidden * kSchedHidden, kSchedHidden);
    fill(kOffW3, (int64_t)kSchedHidden * kSchedOut, kSchedHidden);
    return p;
}

template <class F> static int sguard(F &&f) {
    try {
        f();
        return PF_OK;
    } catch (const Error &e) {
        set_last_error(e.what());
        return e.code;
    } catch (const std::exception &e) {
        set_last_error(e.what());
        return PF_EDEVICE;
    }
}

// a device copy of caller rows (host or device), row-major
static const float *device_rows(const float *src, int64_t count, int32_t mem, DevBuf &tmp, hipStream_t s) {
    if (mem == PF_DEVICE) return src;
    tmp.alloc((size_t)count * sizeof(float));
    PF_HIP(hipMemcpyAsync(tmp.p, src, (size_t)count * sizeof(float), hipMemcpyHostToDevice, s));
    return tmp.as<float>();
}

// predicted cost of each query: 2^(predicted log2(1 + entries scanned))
static std::vector<float> predict_host(Sched &sc, const float *feat_dev, int64_t m, hipStream_t s) {
    std::vector<float> out((size_t)m * kSchedOut);
    const int64_t chunk = 65536;
    sc.ensure_act(std::min(m, chunk));
    for (int64_t r0 = 0; r0 < m; r0 += chunk) {
        const int64_t B = std::min(chunk, m - r0);
        mlp_forward(sc.params.as<float>(), feat_dev + r0 * kSchedIn, nullptr, B, sc.h1(), sc.h2(), sc.y(), s);
        PF_HIP(hipMemcpyAsync(out.data() + r0 * kSchedOut, sc.y(), (size_t)B * kSchedOut * sizeof(float),
                              hipMemcpyDeviceToHost, s));
    }
    PF_HIP(hipStreamSynchronize(s));
    return out;
}

std::vector<float> sched_qparams(int64_t m, const int32_t *ks_host, int32_t kconst, const double *rec_host,
                                 double recall_const) {
    std::vector<float> v((size_t)m * 2);
    for (int64_t i = 0; i < m; ++i) {
        const double k = ks_host ? (double)ks_host[i] : (double)kconst;
        const double delta = 1.0 - (rec_host ? rec_host[i] : recall_const);
        v[2 * i] = (float)std::log2(k);
        v[2 * i + 1] = delta < 0x1.0p-40 ? 40.0f : (float)(-std::log2(delta));
    }
    return v;
}

void learned_order(Index &ix, const uint32_t *qcode, const uint64_t *qsk, int64_t m, const int32_t *ks_host,
                   int32_t kconst, const double *rec_host, double recall_const, int32_t *order, hipStream_t s) {
    Sched &sc = *ix.sched;
    ix.sqph = sched_qparams(m, ks_host, kconst, rec_host, recall_const);
    ix.sfeat.ensure((size_t)m * kSchedIn * sizeof(float));
    ix.sqp.ensure(ix.sqph.size() * sizeof(float));
    ix.skeys.ensure((size_t)m * 2 * sizeof(uint32_t));
    PF_HIP(hipMemcpyAsync(ix.sqp.p, ix.sqph.data(), ix.sqph.size() * sizeof(float), hipMemcpyHostToDevice, s));
    const float *feat = ix.sfeat.as<float>();
    launch_features(ix, qcode, qsk, m, ix.sqp.as<float>(), ix.sfeat.as<float>(), s);
    uint32_t *k = ix.skeys.as<uint32_t>();
    const int64_t chunk = 65536;
    sc.ensure_act(std::min(m, chunk));
    for (int64_t r0 = 0; r0 < m; r0 += chunk) {
        const int64_t B = std::min(chunk, m - r0);
        mlp_forward(sc.params.as<float>(), feat + r0 * kSchedIn, nullptr, B, sc.h1(), sc.h2(), sc.y(), s);
        launch_lpt_keys(sc.y(), B, k + r0, s);
    }
    // longest predicted first (LPT), ties by query index: the stable radix sort of the
    // table builder, on one table of 32-bit keys
    sort_tables(k, m, 1, 32, k + m, reinterpret_cast<uint32_t *>(order), ix.ssort, s);
}

} // namespace pf

using namespace pf;

struct pf_sched : public pf::Sched {};

PF_API int pf_sched_create(uint64_t seed, pf_sched **out) {
    return sguard([&] {
        PF_CHECK(out, PF_EINVAL, "pf_sched_create: null argument");
        auto sc = std::make_unique<pf_sched>();
        sc->seed = seed;
        const std::vector<float> p = init_params(seed);
        sc->params.alloc(kSchedParams * sizeof(float));
        sc->grad.alloc(kSchedParams * sizeof(float));
        sc->m1.alloc(kSchedParams * sizeof(float));
        sc->m2.alloc(kSchedParams * sizeof(float));
        sc->loss.alloc(sizeof(double));
        sc->wscr.alloc((size_t)kWgradScratch * sizeof(float));
        PF_HIP(hipMemcpy(sc->params.p, p.data(), kSchedParams * sizeof(float), hipMemcpyHostToDevice));
        PF_HIP(hipMemset(sc->m1.p, 0, kSchedParams * sizeof(float)));
        PF_HIP(hipMemset(sc->m2.p, 0, kSchedParams * sizeof(float)));
        *out = sc.release();
    });
}

PF_API void pf_sched_free(pf_sched *s) { delete s; }

PF_API int pf_sched_params(pf_sched *sc, float *params, int32_t get) {
    return sguard([&] {
        PF_CHECK(sc && params, PF_EINVAL, "pf_sched_params: null argument");
        if (get)
            PF_HIP(hipMemcpy(params, sc->params.p, kSchedParams * sizeof(float), hipMemcpyDeviceToHost));
        else
            PF_HIP(hipMemcpy(sc->params.p, params, kSchedParams * sizeof(float), hipMemcpyHostToDevice));
    });
}

PF_API int pf_features(pf_index *ix, const float *queries, int64_t m, const int32_t *ks, const double *recalls,
                       int32_t kconst, double recall_const, float *feat, int32_t mem, void *stream) {
    return sguard([&] {
        PF_CHECK(ix && queries && feat && m >= 0, PF_EINVAL, "pf_features: bad arguments");
        PF_CHECK(mem == PF_HOST || mem == PF_DEVICE, PF_EINVAL, "pf_features: bad mem");
        if (m == 0) return;
        hipStream_t s = reinterpret_cast<hipStream_t>(stream);
        const hipMemcpyKind toh = mem == PF_HOST ? hipMemcpyHostToHost : hipMemcpyDeviceToHost;
        std::vector<int32_t> kh;
        std::vector<double> rh;
        if (ks) {
            kh.resize(m);
            PF_HIP(hipMemcpy(kh.data(), ks, (size_t)m * sizeof(int32_t), toh));
        }
        if (recalls) {
            rh.resize(m);
            PF_HIP(hipMemcpy(rh.data(), recalls, (size_t)m * sizeof(double), toh));
        }
        for (int64_t i = 0; i < m; ++i) {
            const int32_t k = ks ? kh[i] : kconst;
            const double r = recalls ? rh[i] : recall_const;
            PF_CHECK(k >= 1 && r > 0.0 && r <= 1.0, PF_EINVAL, "pf_features: k must be >= 1 and recall in (0, 1]");
        }
        const std::vector<float> qph =
            sched_qparams(m, ks ? kh.data() : nullptr, kconst, recalls ? rh.data() : nullptr, recall_const);
        DevBuf qp;
        qp.alloc(qph.size() * sizeof(float));
        PF_HIP(hipMemcpyAsync(qp.p, qph.data(), qph.size() * sizeof(float), hipMemcpyHostToDevice, s));
        uint32_t *qc;
        uint64_t *qs;
        float *qX;
        prepare_rows_for(*ix, queries, m, mem, s, &qX, &qc, &qs);
        if (mem == PF_DEVICE) {
            launch_features(*ix, qc, qs, m, qp.as<float>(), feat, s);
            PF_HIP(hipStreamSynchronize(s));
        } else {
            DevBuf f;
            f.alloc((size_t)m * kSchedIn * sizeof(float));
            launch_features(*ix, qc, qs, m, qp.as<float>(), f.as<float>(), s);
            PF_HIP(hipMemcpyAsync(feat, f.p, (size_t)m * kSchedIn * sizeof(float), hipMemcpyDeviceToHost, s));
            PF_HIP(hipStreamSynchronize(s));
        }
    });
}

PF_API int pf_sched_predict(pf_sched *sc, const float *feat, int64_t m, float *out, int32_t mem, void *stream) {
    return sguard([&] {
        PF_CHECK(sc && feat && out && m >= 0, PF_EINVAL, "pf_sched_predict: bad arguments");
        if (m == 0) return;
        hipStream_t s = reinterpret_cast<hipStream_t>(stream);
        DevBuf tmp;
        const float *x = device_rows(feat, m * kSchedIn, mem, tmp, s);
        const std::vector<float> y = predict_host(*sc, x, m, s);
        PF_HIP(hipMemcpy(out, y.data(), y.size() * sizeof(float),
                         mem == PF_HOST ? hipMemcpyHostToHost : hipMemcpyHostToDevice));
    });
}

PF_API int pf_sched_grad(pf_sched *sc, const float *feat, const float *target, int64_t m, float *grad, double *loss,
                         int32_t mem, void *stream) {
    return sguard([&] {
        PF_CHECK(sc && feat && target && grad && m >= 1, PF_EINVAL, "pf_sched_grad: bad arguments");
        hipStream_t s = reinterpret_cast<hipStream_t>(stream);
        DevBuf tx, tt;
        const float *x = device_rows(feat, m * kSchedIn, mem, tx, s);
        const float *t = device_rows(target, m * kSchedOut, mem, tt, s);
        sc->ensure_act(m);
        PF_HIP(hipMemsetAsync(sc->loss.p, 0, sizeof(double), s));
        mlp_forward(sc->params.as<float>(), x, nullptr, m, sc->h1(), sc->h2(), sc->y(), s);
        mlp_backward(sc->params.as<float>(), x, nullptr, t, m, sc->h1(), sc->h2(), sc->y(), sc->dy(), sc->dh2(),
                     sc->dh1(), sc->grad.as<float>(), sc->loss.as<double>(), sc->wscr.as<float>(), s);
        PF_HIP(hipMemcpyAsync(grad, sc->grad.p, kSchedParams * sizeof(float),
                              mem == PF_HOST ? hipMemcpyDeviceToHost : hipMemcpyDeviceToDevice, s));
        double l = 0;
        PF_HIP(hipMemcpyAsync(&l, sc->loss.p, sizeof(double), hipMemcpyDeviceToHost, s));
        PF_HIP(hipStreamSynchronize(s));
        if (loss) *loss = l;
    });
}

PF_API int pf_sched_train(pf_sched *sc, const float *feat, const float *target, int64_t m, int32_t epochs,
                          int32_t batch, float lr, uint64_t seed, float *epoch_loss, int32_t mem, void *stream) {
    return sguard([&] {
        PF_CHECK(sc && feat && target && m >= 1 && epochs >= 1 && batch >= 1 && lr > 0.0f, PF_EINVAL,
                 "pf_sched_train: bad arguments");
        hipStream_t s = reinterpret_cast<hipStream_t>(stream);
        DevBuf tx, tt, perm;
        const float *x = device_rows(feat, m * kSchedIn, mem, tx, s);
        const float *t = device_rows(target, m * kSchedOut, mem, tt, s);
        sc->ensure_act(batch);
        perm.alloc((size_t)m * sizeof(int32_t));
        std::vector<int32_t> order(m);
        for (int32_t e = 0; e < epochs; ++e) {
            // minibatches over a fresh permutation (Fisher-Yates, counter-based draws)
            std::iota(order.begin(), order.end(), 0);
            for (int64_t i = m - 1; i > 0; --i) {
                const uint64_t z = sm64(seed + (uint64_t)e * 0x9E3779B97F4A7C15ull, (uint64_t)i);
                const int64_t j = (int64_t)(z % (uint64_t)(i + 1));
                std::swap(order[i], order[j]);
            }
            PF_HIP(hipMemcpyAsync(perm.p, order.data(), (size_t)m * sizeof(int32_t), hipMemcpyHostToDevice, s));
            PF_HIP(hipMemsetAsync(sc->loss.p, 0, sizeof(double), s));
            int64_t nb = 0;
            for (int64_t r0 = 0; r0 < m; r0 += batch, ++nb) {
                const int64_t B = std::min<int64_t>(batch, m - r0);
                const int32_t *rows = perm.as<int32_t>() + r0;
                mlp_forward(sc->params.as<float>(), x, rows, B, sc->h1(), sc->h2(), sc->y(), s);
                mlp_backward(sc->params.as<float>(), x, rows, t, B, sc->h1(), sc->h2(), sc->y(), sc->dy(), sc->dh2(),
                             sc->dh1(), sc->grad.as<float>(), sc->loss.as<double>(), sc->wscr.as<float>(), s);
                mlp_adam(sc->params.as<float>(), sc->grad.as<float>(), sc->m1.as<float>(), sc->m2.as<float>(), lr,
                         ++sc->step, s);
            }
            double l = 0;
            PF_HIP(hipMemcpyAsync(&l, sc->loss.p, sizeof(double), hipMemcpyDeviceToHost, s));
            PF_HIP(hipStreamSynchronize(s));
            if (epoch_loss) epoch_loss[e] = (float)(l / (double)nb);
        }
    });
}

PF_API int pf_sched_save(pf_sched *sc, const char *path) {
    return sguard([&] {
        PF_CHECK(sc && path, PF_EINVAL, "pf_sched_save: null argument");
        std::vector<float> p(kSchedParams);
        PF_HIP(hipMemcpy(p.data(), sc->params.p, kSchedParams * sizeof(float), hipMemcpyDeviceToHost));
        FILE *f = std::fopen(path, "wb");
        PF_CHECK(f, PF_EINVAL, std::string("pf_sched_save: cannot open ") + path);
        const char magic[8] = {'P', 'F', 'S', 'C', 'H', 'D', '1', 0};
        const int32_t dims[3] = {kSchedIn, kSchedHidden, kSchedOut};
        const bool ok = std::fwrite(magic, 1, 8, f) == 8 && std::fwrite(dims, 4, 3, f) == 3 &&
                        std::fwrite(p.data(), 4, p.size(), f) == p.size();
        std::fclose(f);
        PF_CHECK(ok, PF_EINVAL, "pf_sched_save: write failed");
    });
}

PF_API int pf_sched_load(pf_sched *sc, const char *path) {
    return sguard([&] {
        PF_CHECK(sc && path, PF_EINVAL, "pf_sched_load: null argument");
        FILE *f = std::fopen(path, "rb");
        PF_CHECK(f, PF_EINVAL, std::string("pf_sched_load: cannot open ") + path);
        char magic[8];
        int32_t dims[3];
        std::vector<float> p(kSchedParams);
        const bool ok = std::fread(magic, 1, 8, f) == 8 && std::memcmp(magic, "PFSCHD1", 8) == 0 &&
                        std::fread(dims, 4, 3, f) == 3 && dims[0] == kSchedIn && dims[1] == kSchedHidden &&
                        dims[2] == kSchedOut && std::fread(p.data(), 4, p.size(), f) == p.size();
        std::fclose(f);
        PF_CHECK(ok, PF_EINVAL, "pf_sched_load: not a scheduler file of this shape");
        PF_HIP(hipMemcpy(sc->params.p, p.data(), kSchedParams * sizeof(float), hipMemcpyHostToDevice));
    });
}

PF_API int pf_index_set_scheduler(pf_index *ix, pf_sched *sc) {
    return sguard([&] {
        PF_CHECK(ix, PF_EINVAL, "pf_index_set_scheduler: null index");
        ix->sched = sc;
    });
}
