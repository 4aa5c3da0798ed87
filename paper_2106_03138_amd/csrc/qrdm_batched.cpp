// Host side of batched QRDM: the plan (size classes, longest-first order per
// class, device copies of the sizes, queue counters) and the launch sequence,
// optionally captured once in a hipGraph and replayed.
#include <hip/hip_runtime.h>
#include <string.h>

#include <algorithm>
#include <map>
#include <new>
#include <tuple>
#include <vector>

#include "qrdm_batched.h"

struct qrdm_batch_plan {
    int device = -1;
    int32_t batch = 0;
    qrdm_params p;
    qrdm_batch_tune tune[QRDM_BATCH_CLASSES];
    int32_t count[QRDM_BATCH_CLASSES] = {0};
    int32_t grid[QRDM_BATCH_CLASSES] = {0};
    int32_t offset[QRDM_BATCH_CLASSES] = {0};
    int32_t *d_m = nullptr, *d_n = nullptr, *d_lda = nullptr, *d_order = nullptr;
    uint32_t *d_counters = nullptr;  // 2 per class
    hipStream_t cap_stream = nullptr;  // captures run here (the legacy default stream cannot be captured)
    std::map<std::tuple<const void *, const void *, const void *, const void *, const void *, const void *,
                        const void *>,
             hipGraphExec_t>
        graphs;
};

namespace {

int size_class(int32_t m) {
    if (m <= 64) return 0;
    if (m <= 128) return 1;
    if (m <= 256) return 2;
    return 3;
}

// algorithmic flops of a full factorization: sum_{s<min(m,n)} 4 (m-s)(n-s)
double flops(int64_t m, int64_t n) {
    const int64_t p = std::min(m, n);
    double f = 0.0;
    for (int64_t s = 0; s < p; ++s) f += 4.0 * (double)(m - s) * (double)(n - s);
    return f;
}

const qrdm_batch_tune kDefaultTune[QRDM_BATCH_CLASSES] = {{0, 0}, {0, 0}, {1, 0}, {1, 0}};

hipError_t enqueue(qrdm_batch_plan *pl, double *const *A, double *const *tau_house, int32_t *const *perm,
                   int64_t *rank, int32_t *status, const qrdm_batch_params *pm, int64_t *info, hipStream_t s,
                   const double *const *pristine = nullptr, double band = 0.0, int32_t *ok = nullptr) {
    for (int c = 0; c < QRDM_BATCH_CLASSES; ++c) {
        if (pl->count[c] == 0) continue;
        QbArgs q;
        q.A = A;
        q.m = pl->d_m;
        q.n = pl->d_n;
        q.lda = pl->d_lda;
        q.tau_house = tau_house;
        q.perm = perm;
        q.rank = rank;
        q.status = status;
        q.pm = pm;
        q.info = info;
        q.order = pl->d_order + pl->offset[c];
        q.count = pl->count[c];
        q.counters = pl->d_counters + 2 * c;
        q.tau = pl->p.tau;
        q.delta = pl->p.delta;
        q.kmax = pl->p.kmax;
        q.stop_rule = pl->p.stop_rule;
        q.eps1_scale = pl->p.eps1_scale;
        q.certified = pl->p.certified;
        q.pristine = pristine;
        q.band = band;
        q.ok = ok;
        hipError_t e = launch_qrdm_batched(q, pl->tune[c].variant, pl->grid[c], s);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace

extern "C" {

int qrdm_batch_plan_create(const int32_t *m, const int32_t *n, const int32_t *lda, int32_t batch,
                           const qrdm_params *p, const qrdm_batch_tune *tune, qrdm_batch_plan **plan) {
    if (!plan) return -7;
    *plan = nullptr;
    if (batch < 0) return -4;
    if (batch > 0 && (!m || !n || !lda)) return -1;
    if (!p) return -5;
    if (!(p->tau >= 0.0 && p->tau <= 1.0) || !(p->delta >= 0.0 && p->delta <= 1.0) || p->kmax < 1 ||
        p->stop_rule < 0 || p->stop_rule > 2 || p->precision != QRDM_PREC_FP64 || p->certified < 0 ||
        p->certified > 1)
        return -5;
    if (p->kmax > QRDM_BATCH_KMAX) return QRDM_ERR_UNSUPPORTED;
    if (tune) {
        for (int c = 0; c < QRDM_BATCH_CLASSES; ++c)
            if (tune[c].variant < 0 || tune[c].variant >= QB_VARIANTS || tune[c].wgs_per_cu < 0) return -6;
    }
    for (int32_t i = 0; i < batch; ++i) {
        if (m[i] < 0) return -1;
        if (n[i] < 0) return -2;
        if (lda[i] < std::max<int32_t>(1, m[i])) return -3;
        if (n[i] > QRDM_BATCH_NMAX) return QRDM_ERR_UNSUPPORTED;
    }
    qrdm_batch_plan *pl = new (std::nothrow) qrdm_batch_plan();
    if (!pl) return QRDM_ERR_NOMEM;
    pl->batch = batch;
    pl->p = *p;
    memcpy(pl->tune, tune ? tune : kDefaultTune, sizeof pl->tune);
    hipError_t e = hipGetDevice(&pl->device);
    int ncu = 0;
    if (e == hipSuccess) e = hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, pl->device);
    if (e != hipSuccess) {
        delete pl;
        return QRDM_ERR_HIP + (int)e;
    }
    // longest first inside each class
    std::vector<std::vector<int32_t>> cls(QRDM_BATCH_CLASSES);
    for (int32_t i = 0; i < batch; ++i) cls[size_class(m[i])].push_back(i);
    std::vector<int32_t> order;
    order.reserve(batch);
    for (int c = 0; c < QRDM_BATCH_CLASSES; ++c) {
        std::stable_sort(cls[c].begin(), cls[c].end(),
                         [&](int32_t a, int32_t b) { return flops(m[a], n[a]) > flops(m[b], n[b]); });
        pl->offset[c] = (int32_t)order.size();
        pl->count[c] = (int32_t)cls[c].size();
        order.insert(order.end(), cls[c].begin(), cls[c].end());
        int occ = 0;
        e = qb_occupancy(pl->tune[c].variant, &occ);
        if (e != hipSuccess) break;
        int per_cu = pl->tune[c].wgs_per_cu > 0 ? std::min(occ, (int)pl->tune[c].wgs_per_cu) : occ;
        per_cu = std::max(per_cu, 1);
        pl->grid[c] = std::min<int64_t>(pl->count[c], (int64_t)ncu * per_cu);
    }
    const size_t nb = (size_t)std::max<int32_t>(batch, 1);
    if (e == hipSuccess) e = hipMalloc((void **)&pl->d_m, nb * sizeof(int32_t));
    if (e == hipSuccess) e = hipMalloc((void **)&pl->d_n, nb * sizeof(int32_t));
    if (e == hipSuccess) e = hipMalloc((void **)&pl->d_lda, nb * sizeof(int32_t));
    if (e == hipSuccess) e = hipMalloc((void **)&pl->d_order, nb * sizeof(int32_t));
    if (e == hipSuccess) e = hipMalloc((void **)&pl->d_counters, 2 * QRDM_BATCH_CLASSES * sizeof(uint32_t));
    if (e == hipSuccess && batch > 0) {
        e = hipMemcpy(pl->d_m, m, batch * sizeof(int32_t), hipMemcpyHostToDevice);
        if (e == hipSuccess) e = hipMemcpy(pl->d_n, n, batch * sizeof(int32_t), hipMemcpyHostToDevice);
        if (e == hipSuccess) e = hipMemcpy(pl->d_lda, lda, batch * sizeof(int32_t), hipMemcpyHostToDevice);
        if (e == hipSuccess) e = hipMemcpy(pl->d_order, order.data(), batch * sizeof(int32_t), hipMemcpyHostToDevice);
    }
    if (e == hipSuccess) e = hipMemset(pl->d_counters, 0, 2 * QRDM_BATCH_CLASSES * sizeof(uint32_t));
    if (e == hipSuccess) e = hipDeviceSynchronize();
    if (e != hipSuccess) {
        qrdm_batch_plan_destroy(pl);
        return e == hipErrorOutOfMemory ? QRDM_ERR_NOMEM : QRDM_ERR_HIP + (int)e;
    }
    *plan = pl;
    return QRDM_OK;
}

int qrdm_batch_factor(qrdm_batch_plan *pl, double *const *A, double *const *tau_house, int32_t *const *perm,
                      int64_t *rank, int32_t *status, const qrdm_batch_params *pm, int64_t *info, int32_t use_graph,
                      void *stream) {
    if (!pl) return -1;
    if (pl->batch > 0 && (!A || !tau_house || !perm || !rank || !status)) return -2;
    if (use_graph < 0 || use_graph > 1) return -9;
    if (pl->batch == 0) return QRDM_OK;
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return QRDM_ERR_HIP + (int)e;
    if (dev != pl->device) return -1;
    hipStream_t s = (hipStream_t)stream;
    if (!use_graph) {
        e = enqueue(pl, A, tau_house, perm, rank, status, pm, info, s);
        return e == hipSuccess ? QRDM_OK : QRDM_ERR_HIP + (int)e;
    }
    auto key = std::make_tuple((const void *)A, (const void *)tau_house, (const void *)perm, (const void *)rank,
                               (const void *)status, (const void *)pm, (const void *)info);
    auto it = pl->graphs.find(key);
    if (it == pl->graphs.end()) {
        if (!pl->cap_stream) {
            e = hipStreamCreateWithFlags(&pl->cap_stream, hipStreamNonBlocking);
            if (e != hipSuccess) return QRDM_ERR_HIP + (int)e;
        }
        hipGraph_t g = nullptr;
        hipGraphExec_t ge = nullptr;
        e = hipStreamBeginCapture(pl->cap_stream, hipStreamCaptureModeThreadLocal);
        if (e != hipSuccess) return QRDM_ERR_HIP + (int)e;
        hipError_t el = enqueue(pl, A, tau_house, perm, rank, status, pm, info, pl->cap_stream);
        e = hipStreamEndCapture(pl->cap_stream, &g);
        if (el != hipSuccess) e = el;
        if (e == hipSuccess) e = hipGraphInstantiate(&ge, g, nullptr, nullptr, 0);
        if (g) (void)hipGraphDestroy(g);
        if (e != hipSuccess) return QRDM_ERR_HIP + (int)e;
        it = pl->graphs.emplace(key, ge).first;
    }
    e = hipGraphLaunch(it->second, s);
    return e == hipSuccess ? QRDM_OK : QRDM_ERR_HIP + (int)e;
}

int qb_plan_sizes(const qrdm_batch_plan *pl, int32_t *batch, const int32_t **m, const int32_t **n,
                  const int32_t **lda, int *device) {
    if (!pl) return -1;
    *batch = pl->batch;
    *m = pl->d_m;
    *n = pl->d_n;
    *lda = pl->d_lda;
    *device = pl->device;
    return 0;
}

int qrdm_batch_factor_checked(qrdm_batch_plan *pl, double *const *A, double *const *tau_house,
                              int32_t *const *perm, int64_t *rank, int32_t *status, const qrdm_batch_params *pm,
                              const double *const *pristine, double band, int32_t *ok, int64_t *info, void *stream) {
    if (!pl) return -1;
    if (pl->batch > 0 && (!A || !tau_house || !perm || !rank || !status || !pm || !pristine || !ok)) return -2;
    if (!(band >= 0.0)) return -9;
    if (pl->batch == 0) return QRDM_OK;
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return QRDM_ERR_HIP + (int)e;
    if (dev != pl->device) return -1;
    e = enqueue(pl, A, tau_house, perm, rank, status, pm, info, (hipStream_t)stream, pristine, band, ok);
    return e == hipSuccess ? QRDM_OK : QRDM_ERR_HIP + (int)e;
}

void qrdm_batch_plan_destroy(qrdm_batch_plan *pl) {
    if (!pl) return;
    (void)hipDeviceSynchronize();
    for (auto &kv : pl->graphs) (void)hipGraphExecDestroy(kv.second);
    if (pl->cap_stream) (void)hipStreamDestroy(pl->cap_stream);
    if (pl->d_m) (void)hipFree(pl->d_m);
    if (pl->d_n) (void)hipFree(pl->d_n);
    if (pl->d_lda) (void)hipFree(pl->d_lda);
    if (pl->d_order) (void)hipFree(pl->d_order);
    if (pl->d_counters) (void)hipFree(pl->d_counters);
    delete pl;
}

}  // extern "C"
