// Autotuner (timed sweep over the candidate tile grid) and the learned cost
// model around the device MLP: features, standardisation, initialisation,
// shuffling, save/load and argmin prediction.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <memory>
#include <string>
#include <vector>

#include "../../include/pcot.h"
#include "kernels.hpp"

using namespace pcot;

struct pcot_model {
    float mu[8], sd[8];  // feature standardisation
    float ymu, ysd;      // target (ln ms) standardisation
    std::vector<float> params;
};

namespace {

#define HIP_TRY(expr)                                                                             \
    do {                                                                                          \
        hipError_t e_ = (expr);                                                                   \
        if (e_ != hipSuccess) return fail(PCOT_ERR_HIP, "%s: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

// SplitMix64 (Steele, Lea and Flood, 2014): x_k = mix(seed + k * golden gamma).
uint64_t mix64(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}
struct SplitMix {
    uint64_t s;
    uint64_t next() { return mix64(s += 0x9E3779B97F4A7C15ULL); }
    double uniform() { return (double)(next() >> 11) * 0x1.0p-53; }
};

int dims_of(int kind) { return kind == PCOT_JACOBI1D_3PT ? 1 : kind == PCOT_JACOBI2D_5PT ? 2 : kind == PCOT_HEAT3D_7PT ? 3 : 0; }
size_t esize(int dtype) { return dtype == PCOT_F64 ? 8 : dtype == PCOT_F32 ? 4 : 2; }

bool valid_problem(const pcot_problem* p) {
    if (!p) return false;
    if (p->kind == PCOT_MATRIX_CHAIN) return p->dims[0] >= 1 && p->T >= 1;
    const int d = dims_of(p->kind);
    if (!d || p->dtype < PCOT_F64 || p->dtype > PCOT_BF16 || p->T < 0) return false;
    for (int i = 0; i < d; ++i)
        if (p->dims[i] < 3) return false;
    return true;
}

uint32_t default_mask(int kind) {
    if (kind == PCOT_MATRIX_CHAIN) return (1u << PCOT_SLT_WAVE) | (1u << PCOT_COT_PAR);
    return (1u << PCOT_SLT_LEX) | (1u << PCOT_SLT_WAVE) | (1u << PCOT_COT_SEQ) | (1u << PCOT_COT_PAR);
}

std::vector<std::pair<pcot_tile, int32_t>> candidates(const pcot_problem* p, uint32_t mask) {
    std::vector<std::pair<pcot_tile, int32_t>> out;
    mask = mask ? mask & default_mask(p->kind) : default_mask(p->kind);
    std::vector<pcot_tile> tiles;
    auto mk = [](int t, int a, int b, int c) {
        pcot_tile x;
        x.t = t;
        x.s[0] = a;
        x.s[1] = b;
        x.s[2] = c;
        return x;
    };
    switch (p->kind) {
        case PCOT_JACOBI1D_3PT:
            for (int bt : {16, 32, 64, 128, 256})
                for (int bx : {64, 128, 256}) tiles.push_back(mk(bt, bx, 0, 0));
            break;
        case PCOT_JACOBI2D_5PT:
            for (int bt : {4, 8, 16, 32, 64})
                for (int by : {16, 32, 64, 128, 256})
                    for (int bx : {64, 128, 256}) tiles.push_back(mk(bt, by, bx, 0));
            break;
        case PCOT_HEAT3D_7PT:
            for (int bt : {2, 3, 4, 6, 8, 12})
                for (int bz : {16, 64, 256})
                    for (int by : {2, 4, 8, 16}) tiles.push_back(mk(bt, bz, by, 64));
            break;
        case PCOT_MATRIX_CHAIN:
            for (int b : {16, 32, 64})
                for (int kc : {16, 32, 64, 128, 256})
                    if (kc >= b || b == 16) tiles.push_back(mk(0, b, b, kc));
            break;
        default: return out;
    }
    for (int s = PCOT_SLT_LEX; s <= PCOT_COT_PAR; ++s) {
        if (!(mask >> s & 1)) continue;
        for (const pcot_tile& t : tiles) {
            if (p->kind == PCOT_MATRIX_CHAIN) {
                if (pcot_dp_workspace(p->dims[0], &t, s) == 0) continue;
            } else if (pcot_stencil_tile_supported(p->kind, p->dtype, &t) != PCOT_OK) {
                continue;
            }
            out.push_back({t, s});
        }
    }
    return out;
}

void features(const pcot_problem* p, const pcot_tile* t, int32_t s, float* f) {
    auto l2 = [](double v) { return (float)std::log2(std::max(v, 1.0)); };
    for (int i = 0; i < 8; ++i) f[i] = 0.f;
    if (p->kind == PCOT_MATRIX_CHAIN) {
        f[0] = l2((double)p->dims[0]);
        f[1] = l2(t->s[0]);
        f[2] = l2(t->s[2]);
        f[3] = l2((double)p->T);
        f[4] = (float)s;
        return;
    }
    const int d = dims_of(p->kind);
    double outer = 1, btile = 1;
    for (int i = 0; i + 1 < d; ++i) {
        outer *= (double)p->dims[i];
        btile *= t->s[i];
    }
    if (d == 1) {
        f[0] = l2((double)p->dims[0]);
        f[1] = 0.f;
    } else {
        f[0] = l2(outer);
        f[1] = l2((double)p->dims[d - 1]);
    }
    f[2] = l2((double)p->T);
    f[3] = l2(t->t);
    f[4] = l2(btile);
    f[5] = l2(t->s[d - 1]);
    f[6] = l2((double)esize(p->dtype));
    f[7] = (float)s;
}

// Device buffers of one tuning session.
struct DevBuf {
    void* p = nullptr;
    ~DevBuf() {
        if (p) (void)hipFree(p);
    }
};

pcot_status run_once(const pcot_problem* p, const pcot_tile* t, int32_t s, void* in, void* out, void* ws,
                     size_t wsb, hipStream_t st) {
    if (p->kind == PCOT_MATRIX_CHAIN)
        return pcot_dp_run((const int64_t*)in, p->dims[0], p->T, t, s, (int64_t*)out, ws, wsb, st);
    return pcot_stencil_run(p->kind, p->dtype, p->dims, p->T, t, s, in, out, ws, wsb, st);
}

// Median time (ms) of `reps` runs after `warm` untimed ones.
pcot_status time_candidate(const pcot_problem* p, const pcot_tile* t, int32_t s, void* in, void* out, void* ws,
                           size_t wsb, int warm, int reps, hipStream_t st, float* ms) {
    for (int i = 0; i < warm; ++i) {
        pcot_status e = run_once(p, t, s, in, out, ws, wsb, st);
        if (e != PCOT_OK) return e;
    }
    hipEvent_t a, b;
    HIP_TRY(hipEventCreate(&a));
    HIP_TRY(hipEventCreate(&b));
    std::vector<float> v;
    pcot_status e = PCOT_OK;
    for (int i = 0; i < reps && e == PCOT_OK; ++i) {
        if (hipEventRecord(a, st) != hipSuccess) { e = fail(PCOT_ERR_HIP, "event record"); break; }
        e = run_once(p, t, s, in, out, ws, wsb, st);
        if (e != PCOT_OK) break;
        if (hipEventRecord(b, st) != hipSuccess || hipEventSynchronize(b) != hipSuccess) {
            e = fail(PCOT_ERR_HIP, "event wait");
            break;
        }
        float x = 0.f;
        (void)hipEventElapsedTime(&x, a, b);
        v.push_back(x);
    }
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    if (e != PCOT_OK) return e;
    e = pcot_stream_status(ws, st);
    if (e != PCOT_OK) return e;
    std::sort(v.begin(), v.end());
    *ms = v[v.size() / 2];
    return PCOT_OK;
}

// Device forward of the model on standardised features; returns ms.
pcot_status model_ms(const pcot_model* m, const std::vector<float>& raw, size_t n, std::vector<float>& ms,
                     hipStream_t st) {
    std::vector<float> X(n * 8);
    for (size_t i = 0; i < n; ++i)
        for (int k = 0; k < 8; ++k) X[i * 8 + k] = (raw[i * 8 + k] - m->mu[k]) / m->sd[k];
    std::vector<float> yh(n);
    pcot_status e = pcot_mlp_forward(m->params.data(), X.data(), (int32_t)n, yh.data(), st);
    if (e != PCOT_OK) return e;
    ms.resize(n);
    for (size_t i = 0; i < n; ++i) ms[i] = std::exp(yh[i] * m->ysd + m->ymu);
    return PCOT_OK;
}

}  // namespace

extern "C" {

int64_t pcot_tune_candidates(const pcot_problem* prob, uint32_t sched_mask, pcot_tile* tiles, int32_t* scheds,
                             int64_t cap) {
    PCOT_TRY
    if (!valid_problem(prob)) {
        fail(PCOT_ERR_INVALID, "invalid problem");
        return -1;
    }
    auto c = candidates(prob, sched_mask);
    for (int64_t i = 0; i < (int64_t)c.size() && i < cap; ++i) {
        if (tiles) tiles[i] = c[i].first;
        if (scheds) scheds[i] = c[i].second;
    }
    return (int64_t)c.size();
    PCOT_CATCH(-1)
}

pcot_status pcot_features(const pcot_problem* prob, const pcot_tile* tile, int32_t schedule, float* feat) {
    PCOT_TRY
    if (!valid_problem(prob) || !tile || !feat) return fail(PCOT_ERR_INVALID, "invalid problem, tile or feat");
    features(prob, tile, schedule, feat);
    return PCOT_OK;
    PCOT_CATCH(PCOT_ERR_HOST)
}

pcot_status pcot_tune(const pcot_problem* prob, const pcot_tune_opts* opts, pcot_tile* best, int32_t* best_sched,
                      double* best_ms, pcot_record* records, size_t cap, size_t* n_records, void* stream) {
    PCOT_TRY
    if (!valid_problem(prob)) return fail(PCOT_ERR_INVALID, "invalid problem");
    pcot_tune_opts o;
    memset(&o, 0, sizeof o);
    if (opts) o = *opts;
    const int reps = o.reps > 0 ? o.reps : 5;
    const int warm = o.warmup >= 0 ? o.warmup : 2;
    const int topk = o.topk > 0 ? o.topk : 3;
    if (o.mode < PCOT_TUNE_SWEEP || o.mode > PCOT_TUNE_MODEL_VERIFY) return fail(PCOT_ERR_INVALID, "mode %d", o.mode);
    if (o.mode != PCOT_TUNE_SWEEP && !o.model) return fail(PCOT_ERR_INVALID, "model modes need a model");
    hipStream_t st = (hipStream_t)stream;
    auto cand = candidates(prob, o.sched_mask);
    if (cand.empty()) return fail(PCOT_ERR_UNSUPPORTED, "no runnable candidate");
    const size_t nc = cand.size();
    std::vector<float> feat(nc * 8), ms(nc, INFINITY);
    for (size_t i = 0; i < nc; ++i) features(prob, &cand[i].first, cand[i].second, &feat[i * 8]);

    std::vector<size_t> timed;
    if (o.mode == PCOT_TUNE_SWEEP) {
        for (size_t i = 0; i < nc; ++i) timed.push_back(i);
    } else {
        pcot_status e = model_ms(o.model, feat, nc, ms, st);
        if (e != PCOT_OK) return e;
        if (o.mode == PCOT_TUNE_MODEL_VERIFY) {
            std::vector<size_t> idx(nc);
            for (size_t i = 0; i < nc; ++i) idx[i] = i;
            std::stable_sort(idx.begin(), idx.end(), [&](size_t a, size_t b) { return ms[a] < ms[b]; });
            for (size_t i = 0; i < nc && (int)i < topk; ++i) timed.push_back(idx[i]);
        }
    }
    if (!timed.empty()) {
        // buffers sized for the problem; workspace for the largest candidate
        size_t in_b, out_b, wsb = 256;
        if (prob->kind == PCOT_MATRIX_CHAIN) {
            in_b = 8 * (size_t)(prob->dims[0] + 1);
            out_b = 8 * (size_t)prob->dims[0] * (size_t)prob->dims[0];
        } else {
            size_t el = 1;
            for (int i = 0; i < dims_of(prob->kind); ++i) el *= (size_t)prob->dims[i];
            in_b = out_b = el * esize(prob->dtype);
        }
        for (size_t i : timed) {
            const size_t w = prob->kind == PCOT_MATRIX_CHAIN
                                 ? pcot_dp_workspace(prob->dims[0], &cand[i].first, cand[i].second)
                                 : pcot_stencil_workspace(prob->kind, prob->dtype, prob->dims, prob->T,
                                                          &cand[i].first, cand[i].second);
            wsb = std::max(wsb, w);
        }
        DevBuf in, out, ws;
        HIP_TRY(hipMalloc(&in.p, in_b));
        HIP_TRY(hipMalloc(&out.p, out_b));
        HIP_TRY(hipMalloc(&ws.p, wsb));
        if (prob->kind == PCOT_MATRIX_CHAIN) {
            HIP_TRY(launch_fill_chain((long long*)in.p, (int)prob->dims[0] + 1, (long long)prob->T, st));
        } else {
            HIP_TRY(launch_fill_u32((unsigned*)in.p, in_b / 4, 0u, st));
        }
        for (size_t i : timed) {
            pcot_status e = time_candidate(prob, &cand[i].first, cand[i].second, in.p, out.p, ws.p, wsb, warm, reps,
                                           st, &ms[i]);
            if (e != PCOT_OK) return e;
        }
    }
    // best: among timed candidates when any were timed, else among predictions
    size_t bi = nc;
    const std::vector<size_t>* pool = &timed;
    std::vector<size_t> all;
    if (timed.empty()) {
        for (size_t i = 0; i < nc; ++i) all.push_back(i);
        pool = &all;
    }
    for (size_t i : *pool)
        if (bi == nc || ms[i] < ms[bi]) bi = i;
    if (best) *best = cand[bi].first;
    if (best_sched) *best_sched = cand[bi].second;
    if (best_ms) *best_ms = ms[bi];
    size_t k = 0;
    if (records) {
        const std::vector<size_t>& src = timed.empty() ? all : timed;
        for (size_t i : src) {
            if (k >= cap) break;
            pcot_record& r = records[k++];
            memcpy(r.feat, &feat[i * 8], sizeof r.feat);
            r.ms = ms[i];
            r.tile = cand[i].first;
            r.schedule = cand[i].second;
        }
    }
    if (n_records) *n_records = records ? k : (timed.empty() ? nc : timed.size());
    return PCOT_OK;
    PCOT_CATCH(PCOT_ERR_HOST)
}

// ------------------------------------------------------------------ MLP ---
pcot_status pcot_mlp_forward(const float* params, const float* X, int32_t n, float* yhat, void* stream) {
    PCOT_TRY
    if (!params || !X || !yhat || n < 0) return fail(PCOT_ERR_INVALID, "NULL argument or n < 0");
    if (n == 0) return PCOT_OK;
    hipStream_t st = (hipStream_t)stream;
    DevBuf dp, dx, dy;
    HIP_TRY(hipMalloc(&dp.p, MLP_NP * sizeof(float)));
    HIP_TRY(hipMalloc(&dx.p, (size_t)n * 8 * sizeof(float)));
    HIP_TRY(hipMalloc(&dy.p, (size_t)n * sizeof(float)));
    HIP_TRY(hipMemcpyAsync(dp.p, params, MLP_NP * sizeof(float), hipMemcpyHostToDevice, st));
    HIP_TRY(hipMemcpyAsync(dx.p, X, (size_t)n * 8 * sizeof(float), hipMemcpyHostToDevice, st));
    HIP_TRY(launch_mlp_forward((const float*)dp.p, (const float*)dx.p, n, (float*)dy.p, st));
    HIP_TRY(hipMemcpyAsync(yhat, dy.p, (size_t)n * sizeof(float), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    return PCOT_OK;
    PCOT_CATCH(PCOT_ERR_HOST)
}

pcot_status pcot_mlp_grad(const float* params, const float* X, const float* y, int32_t n, float* grad, float* loss,
                          void* stream) {
    PCOT_TRY
    if (!params || !X || !y || !grad || n < 1 || n > 256) return fail(PCOT_ERR_INVALID, "bad argument (1 <= n <= 256)");
    hipStream_t st = (hipStream_t)stream;
    std::vector<int> rows(n);
    for (int i = 0; i < n; ++i) rows[i] = i;
    DevBuf dp, dx, dy, dr, ds, dg, dl;
    HIP_TRY(hipMalloc(&dp.p, MLP_NP * sizeof(float)));
    HIP_TRY(hipMalloc(&dx.p, (size_t)n * 8 * sizeof(float)));
    HIP_TRY(hipMalloc(&dy.p, (size_t)n * sizeof(float)));
    HIP_TRY(hipMalloc(&dr.p, (size_t)n * sizeof(int)));
    HIP_TRY(hipMalloc(&ds.p, mlp_scratch_floats() * sizeof(float)));
    HIP_TRY(hipMalloc(&dg.p, MLP_NP * sizeof(float)));
    HIP_TRY(hipMalloc(&dl.p, sizeof(float)));
    HIP_TRY(hipMemcpyAsync(dp.p, params, MLP_NP * sizeof(float), hipMemcpyHostToDevice, st));
    HIP_TRY(hipMemcpyAsync(dx.p, X, (size_t)n * 8 * sizeof(float), hipMemcpyHostToDevice, st));
    HIP_TRY(hipMemcpyAsync(dy.p, y, (size_t)n * sizeof(float), hipMemcpyHostToDevice, st));
    HIP_TRY(hipMemcpyAsync(dr.p, rows.data(), (size_t)n * sizeof(int), hipMemcpyHostToDevice, st));
    HIP_TRY(launch_mlp_grad((const float*)dp.p, (const float*)dx.p, (const float*)dy.p, (const int*)dr.p, n,
                            (float*)ds.p, (float*)dg.p, (float*)dl.p, st));
    HIP_TRY(hipMemcpyAsync(grad, dg.p, MLP_NP * sizeof(float), hipMemcpyDeviceToHost, st));
    float l = 0.f;
    HIP_TRY(hipMemcpyAsync(&l, dl.p, sizeof(float), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    if (loss) *loss = l;
    return PCOT_OK;
    PCOT_CATCH(PCOT_ERR_HOST)
}

pcot_status pcot_mlp_train(float* params, float* m, float* v, const float* X, const float* y, int32_t n,
                           const int32_t* order, int32_t epochs, int32_t batch, int32_t step0, float lr,
                           float* epoch_loss, void* stream) {
    PCOT_TRY
    if (!params || !m || !v || !X || !y || !order || n < 1 || epochs < 0 || batch < 1 || batch > 256 || step0 < 0)
        return fail(PCOT_ERR_INVALID, "bad argument");
    for (int64_t i = 0; i < (int64_t)epochs * n; ++i)
        if (order[i] < 0 || order[i] >= n) return fail(PCOT_ERR_INVALID, "order[%lld] out of range", (long long)i);
    if (epochs == 0) return PCOT_OK;
    hipStream_t st = (hipStream_t)stream;
    DevBuf dp, dm, dv, dx, dy, dor, ds, dl;
    const size_t P = MLP_NP * sizeof(float);
    HIP_TRY(hipMalloc(&dp.p, P));
    HIP_TRY(hipMalloc(&dm.p, P));
    HIP_TRY(hipMalloc(&dv.p, P));
    HIP_TRY(hipMalloc(&dx.p, (size_t)n * 8 * sizeof(float)));
    HIP_TRY(hipMalloc(&dy.p, (size_t)n * sizeof(float)));
    HIP_TRY(hipMalloc(&dor.p, (size_t)epochs * n * sizeof(int)));
    HIP_TRY(hipMalloc(&ds.p, mlp_scratch_floats() * sizeof(float)));
    HIP_TRY(hipMalloc(&dl.p, (size_t)epochs * sizeof(float)));
    HIP_TRY(hipMemcpyAsync(dp.p, params, P, hipMemcpyHostToDevice, st));
    HIP_TRY(hipMemcpyAsync(dm.p, m, P, hipMemcpyHostToDevice, st));
    HIP_TRY(hipMemcpyAsync(dv.p, v, P, hipMemcpyHostToDevice, st));
    HIP_TRY(hipMemcpyAsync(dx.p, X, (size_t)n * 8 * sizeof(float), hipMemcpyHostToDevice, st));
    HIP_TRY(hipMemcpyAsync(dy.p, y, (size_t)n * sizeof(float), hipMemcpyHostToDevice, st));
    HIP_TRY(hipMemcpyAsync(dor.p, order, (size_t)epochs * n * sizeof(int), hipMemcpyHostToDevice, st));
    HIP_TRY(launch_mlp_train((float*)dp.p, (float*)dm.p, (float*)dv.p, (const float*)dx.p, (const float*)dy.p,
                             (const int*)dor.p, n, epochs, batch, step0, lr, 0.9f, 0.999f, 1e-8f, (float*)ds.p,
                             (float*)dl.p, st));
    HIP_TRY(hipMemcpyAsync(params, dp.p, P, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipMemcpyAsync(m, dm.p, P, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipMemcpyAsync(v, dv.p, P, hipMemcpyDeviceToHost, st));
    std::vector<float> el(epochs);
    HIP_TRY(hipMemcpyAsync(el.data(), dl.p, (size_t)epochs * sizeof(float), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    if (epoch_loss) memcpy(epoch_loss, el.data(), (size_t)epochs * sizeof(float));
    return PCOT_OK;
    PCOT_CATCH(PCOT_ERR_HOST)
}

// ---------------------------------------------------------------- model ---
pcot_status pcot_model_train(const pcot_record* records, size_t n, const pcot_train_opts* opts, pcot_model** out,
                             float* final_loss, void* stream) {
    PCOT_TRY
    if (!records || !out || n < 2 || n > (1u << 24)) return fail(PCOT_ERR_INVALID, "need 2 .. 2^24 records");
    pcot_train_opts o;
    memset(&o, 0, sizeof o);
    if (opts) o = *opts;
    const int epochs = o.epochs > 0 ? o.epochs : 300;
    const int batch = o.batch > 0 ? o.batch : 256;
    const float lr = o.lr > 0 ? o.lr : 1e-3f;
    if (batch > 256) return fail(PCOT_ERR_INVALID, "batch %d > 256", batch);
    for (size_t i = 0; i < n; ++i)
        if (!(records[i].ms > 0.f) || !std::isfinite(records[i].ms))
            return fail(PCOT_ERR_INVALID, "record %zu: time %g not positive", i, (double)records[i].ms);
    auto m = std::make_unique<pcot_model>();
    // standardisation from the training set (scale 1 for constant features)
    for (int k = 0; k < 8; ++k) {
        double s = 0, s2 = 0;
        for (size_t i = 0; i < n; ++i) s += records[i].feat[k];
        const double mu = s / n;
        for (size_t i = 0; i < n; ++i) s2 += (records[i].feat[k] - mu) * (records[i].feat[k] - mu);
        const double sd = std::sqrt(s2 / n);
        m->mu[k] = (float)mu;
        m->sd[k] = sd > 1e-6 ? (float)sd : 1.f;
    }
    {
        double s = 0, s2 = 0;
        for (size_t i = 0; i < n; ++i) s += std::log((double)records[i].ms);
        const double mu = s / n;
        for (size_t i = 0; i < n; ++i) {
            const double d = std::log((double)records[i].ms) - mu;
            s2 += d * d;
        }
        const double sd = std::sqrt(s2 / n);
        m->ymu = (float)mu;
        m->ysd = sd > 1e-6 ? (float)sd : 1.f;
    }
    std::vector<float> X(n * 8), y(n);
    for (size_t i = 0; i < n; ++i) {
        for (int k = 0; k < 8; ++k) X[i * 8 + k] = (records[i].feat[k] - m->mu[k]) / m->sd[k];
        y[i] = (float)((std::log((double)records[i].ms) - m->ymu) / m->ysd);
    }
    // He-uniform initialisation (bound sqrt(6 / fan_in)), zero biases
    SplitMix g{o.seed * 0x2545F4914F6CDD1DULL + 1802};
    m->params.assign(MLP_NP, 0.f);
    auto fill = [&](int off, int count, int fan_in) {
        const double a = std::sqrt(6.0 / fan_in);
        for (int i = 0; i < count; ++i) m->params[off + i] = (float)((2.0 * g.uniform() - 1.0) * a);
    };
    fill(0, 64 * 8, 8);
    fill(64 * 8 + 64, 64 * 64, 64);
    fill(64 * 8 + 64 + 64 * 64 + 64, 64, 64);
    // one Fisher-Yates permutation per epoch
    std::vector<int32_t> order((size_t)epochs * n);
    for (int e = 0; e < epochs; ++e) {
        int32_t* p = &order[(size_t)e * n];
        for (size_t i = 0; i < n; ++i) p[i] = (int32_t)i;
        for (size_t i = n - 1; i > 0; --i) {
            const size_t j = (size_t)(g.next() % (uint64_t)(i + 1));
            std::swap(p[i], p[j]);
        }
    }
    std::vector<float> mm(MLP_NP, 0.f), vv(MLP_NP, 0.f), el(epochs);
    pcot_status e = pcot_mlp_train(m->params.data(), mm.data(), vv.data(), X.data(), y.data(), (int32_t)n,
                                   order.data(), epochs, batch, 0, lr, el.data(), stream);
    if (e != PCOT_OK) return e;
    if (final_loss) *final_loss = el.back();
    *out = m.release();
    return PCOT_OK;
    PCOT_CATCH(PCOT_ERR_HOST)
}

pcot_status pcot_model_predict_ms(const pcot_model* model, const pcot_record* records, size_t n, float* ms,
                                  void* stream) {
    PCOT_TRY
    if (!model || !records || !ms) return fail(PCOT_ERR_INVALID, "NULL argument");
    std::vector<float> raw(n * 8), out;
    for (size_t i = 0; i < n; ++i) memcpy(&raw[i * 8], records[i].feat, 8 * sizeof(float));
    pcot_status e = model_ms(model, raw, n, out, (hipStream_t)stream);
    if (e != PCOT_OK) return e;
    memcpy(ms, out.data(), n * sizeof(float));
    return PCOT_OK;
    PCOT_CATCH(PCOT_ERR_HOST)
}

pcot_status pcot_model_predict(const pcot_model* model, const pcot_problem* prob, uint32_t sched_mask,
                               pcot_tile* best, int32_t* best_sched, double* pred_ms, void* stream) {
    PCOT_TRY
    pcot_tune_opts o;
    memset(&o, 0, sizeof o);
    o.mode = PCOT_TUNE_MODEL;
    o.sched_mask = sched_mask;
    o.model = model;
    return pcot_tune(prob, &o, best, best_sched, pred_ms, nullptr, 0, nullptr, stream);
    PCOT_CATCH(PCOT_ERR_HOST)
}

pcot_status pcot_model_save(const pcot_model* m, const char* path) {
    PCOT_TRY
    if (!m || !path) return fail(PCOT_ERR_INVALID, "NULL argument");
    FILE* f = fopen(path, "w");
    if (!f) return fail(PCOT_ERR_INVALID, "cannot write %s", path);
    fprintf(f, "pcot-mlp 1\n");
    for (int k = 0; k < 8; ++k) fprintf(f, "%.9g%c", m->mu[k], k == 7 ? '\n' : ' ');
    for (int k = 0; k < 8; ++k) fprintf(f, "%.9g%c", m->sd[k], k == 7 ? '\n' : ' ');
    fprintf(f, "%.9g %.9g\n", m->ymu, m->ysd);
    for (int i = 0; i < MLP_NP; ++i) fprintf(f, "%.9g\n", m->params[i]);
    const bool ok = fclose(f) == 0;
    return ok ? PCOT_OK : fail(PCOT_ERR_INVALID, "write error on %s", path);
    PCOT_CATCH(PCOT_ERR_HOST)
}

pcot_status pcot_model_load(const char* path, pcot_model** out) {
    PCOT_TRY
    if (!path || !out) return fail(PCOT_ERR_INVALID, "NULL argument");
    FILE* f = fopen(path, "r");
    if (!f) return fail(PCOT_ERR_INVALID, "cannot read %s", path);
    auto m = std::make_unique<pcot_model>();
    char magic[32] = {0};
    int ver = 0;
    bool ok = fscanf(f, "%31s %d", magic, &ver) == 2 && std::string(magic) == "pcot-mlp" && ver == 1;
    for (int k = 0; ok && k < 8; ++k) ok = fscanf(f, "%f", &m->mu[k]) == 1;
    for (int k = 0; ok && k < 8; ++k) ok = fscanf(f, "%f", &m->sd[k]) == 1 && m->sd[k] > 0;
    ok = ok && fscanf(f, "%f %f", &m->ymu, &m->ysd) == 2 && m->ysd > 0;
    m->params.assign(MLP_NP, 0.f);
    for (int i = 0; ok && i < MLP_NP; ++i) ok = fscanf(f, "%f", &m->params[i]) == 1;
    fclose(f);
    if (!ok) return fail(PCOT_ERR_INVALID, "%s is not a pcot model file", path);
    *out = m.release();
    return PCOT_OK;
    PCOT_CATCH(PCOT_ERR_HOST)
}

void pcot_model_free(pcot_model* m) { delete m; }

}  // extern "C"
