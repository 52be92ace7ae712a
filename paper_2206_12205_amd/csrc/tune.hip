// Autotuner: times the candidate kernel configurations of a workload on the
// device and keeps the fastest (the batched mode picks one per length class).
#include "internal.hpp"

#include <vector>

namespace {

std::vector<fdas_config> candidates(const fdas_config &c) {
    std::vector<fdas_config> out;
    std::vector<int32_t> Ls;
    if (c.seg_len != 0) {
        Ls.push_back(c.seg_len);
    } else {
        for (int32_t L = 1024; L <= 16384; L *= 2)
            if (L > c.n_taps) Ls.push_back(L);
    }
    std::vector<int32_t> algos;
    if (c.algo != FDAS_ALGO_AUTO) {
        algos.push_back(c.algo);
    } else {
        algos.push_back(FDAS_ALGO_VALU);
        if (c.compute == FDAS_BF16) algos.push_back(FDAS_ALGO_MFMA);
    }
    std::vector<int32_t> zcs;
    if (c.z_chunk != 0) {
        zcs.push_back(c.z_chunk);
    } else {
        for (int d : {1, 2, 4, 8}) {
            const int32_t zc = (c.n_z + d - 1) / d;
            if (zcs.empty() || zcs.back() != zc) zcs.push_back(zc);
        }
    }
    for (int32_t L : Ls)
        for (int32_t a : algos)
            for (int32_t zc : zcs) {
                fdas_config k = c;
                k.seg_len = L;
                k.algo = a;
                k.z_chunk = zc;
                k.max_jobs = 0;
                out.push_back(k);
            }
    return out;
}

struct PlanGuard {
    fdas_plan_t h = nullptr;
    ~PlanGuard() { fdas_destroy(h); }
};

}  // namespace

extern "C" {

int fdas_tune_workspace(const fdas_config *cfg, size_t *workspace_bytes) {
    if (!cfg || !workspace_bytes) return FDAS_E_INVALID;
    *workspace_bytes = 0;
    size_t need = 0;
    bool any = false;
    for (const fdas_config &k : candidates(*cfg)) {
        PlanGuard g;
        size_t b = 0;
        const int st = fdas_plan(&k, &g.h, &b);
        if (st == FDAS_E_UNSUPPORTED) continue;
        if (st != FDAS_OK) return st;
        any = true;
        if (b > need) need = b;
    }
    if (!any) return FDAS_E_UNSUPPORTED;
    *workspace_bytes = need;
    return FDAS_OK;
}

int fdas_tune(const fdas_config *cfg, const void *spectrum, int64_t n_bins, void *plane, void *workspace,
              size_t workspace_bytes, int32_t reps, fdas_config *best, float *best_ms, void *stream) {
    if (!cfg || !spectrum || !plane || !workspace || !best || !best_ms) return FDAS_E_INVALID;
    if (reps < 1 || reps > 1000 || n_bins < 1 || n_bins > cfg->max_bins) return FDAS_E_INVALID;
    size_t need = 0;
    int st = fdas_tune_workspace(cfg, &need);
    if (st != FDAS_OK) return st;
    if (workspace_bytes < need) return FDAS_E_WORKSPACE;
    hipStream_t s = static_cast<hipStream_t>(stream);
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t he = hipEventCreate(&e0);
    if (he == hipSuccess) he = hipEventCreate(&e1);
    float best_t = -1.f;
    fdas_config best_c{};
    for (const fdas_config &k : candidates(*cfg)) {
        if (he != hipSuccess) break;
        PlanGuard g;
        size_t b = 0;
        st = fdas_plan(&k, &g.h, &b);
        if (st == FDAS_E_UNSUPPORTED) continue;
        if (st == FDAS_OK) st = fdas_set_workspace(g.h, workspace, workspace_bytes);
        if (st == FDAS_OK) st = fdas_make_templates(g.h, stream);
        if (st == FDAS_OK) st = fdas_correlate(g.h, spectrum, n_bins, plane, stream);   // warm-up
        if (st != FDAS_OK) break;
        he = hipEventRecord(e0, s);
        for (int32_t r = 0; r < reps && st == FDAS_OK && he == hipSuccess; ++r)
            st = fdas_correlate(g.h, spectrum, n_bins, plane, stream);
        if (st != FDAS_OK) break;
        if (he == hipSuccess) he = hipEventRecord(e1, s);
        if (he == hipSuccess) he = hipEventSynchronize(e1);
        float ms = 0.f;
        if (he == hipSuccess) he = hipEventElapsedTime(&ms, e0, e1);
        if (he != hipSuccess) break;
        ms /= (float)reps;
        fdas_layout lay;
        fdas_get_layout(g.h, &lay);
        if (best_t < 0.f || ms < best_t) {
            best_t = ms;
            best_c = k;
            best_c.seg_len = lay.seg_len;
            best_c.algo = lay.algo;
            best_c.z_chunk = lay.z_chunk;
            best_c.max_jobs = cfg->max_jobs;
        }
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (he != hipSuccess) return fdas::hip_status_of(he);
    if (st != FDAS_OK && st != FDAS_E_UNSUPPORTED) return st;
    if (best_t < 0.f) return FDAS_E_UNSUPPORTED;
    *best = best_c;
    *best_ms = best_t;
    return FDAS_OK;
}

}  // extern "C"
