// Host entry points of the learned parameter predictor (C ABI of include/qrdm.h).
#include "qrdm_learned.h"

static int lf_err(hipError_t e) { return e == hipSuccess ? QRDM_OK : QRDM_ERR_HIP + (int)e; }

extern "C" {

int qrdm_batch_features(qrdm_batch_plan *plan, double *const *A, double *features, void *stream) {
    int32_t batch;
    LfArgs q;
    int dev;
    if (qb_plan_sizes(plan, &batch, &q.m, &q.n, &q.lda, &dev) != 0) return -1;
    if (batch > 0 && !A) return -2;
    if (batch > 0 && !features) return -3;
    q.A = A;
    return lf_err(launch_features(q, batch, features, (hipStream_t)stream));
}

int qrdm_mlp_forward(const float *params, const float *norm, const double *features, int32_t batch, float *h1,
                     float *h2, float *y, void *stream) {
    if (!params) return -1;
    if (batch < 0) return -4;
    if (batch > 0 && !features) return -3;
    if (batch > 0 && !y) return -7;
    return lf_err(launch_mlp_forward(params, norm, features, batch, h1, h2, y, (hipStream_t)stream));
}

int qrdm_mlp_gradient(const float *params, const float *norm, const double *features, const float *h1,
                      const float *h2, const float *y, const float *target, int32_t batch, float *work, float *grad,
                      float *sqerr, void *stream) {
    if (!params) return -1;
    if (batch <= 0) return -8;
    if (!features) return -3;
    if (!h1 || !h2) return -4;
    if (!y) return -6;
    if (!target) return -7;
    if (!work) return -9;
    if (!grad) return -10;
    return lf_err(launch_mlp_backward(params, norm, features, h1, h2, y, target, batch, work, grad, sqerr,
                                      (hipStream_t)stream));
}

int qrdm_mlp_adam(float *params, const float *grad, float *m, float *v, int32_t t, float lr, float beta1,
                  float beta2, float eps, void *stream) {
    if (!params) return -1;
    if (!grad) return -2;
    if (!m) return -3;
    if (!v) return -4;
    if (t < 1) return -5;
    if (!(lr > 0.f)) return -6;
    if (!(beta1 >= 0.f && beta1 < 1.f)) return -7;
    if (!(beta2 >= 0.f && beta2 < 1.f)) return -8;
    if (!(eps > 0.f)) return -9;
    return lf_err(launch_adam(params, grad, m, v, t, lr, beta1, beta2, eps, (hipStream_t)stream));
}

int qrdm_mlp_to_params(const float *y, int32_t batch, qrdm_batch_params *out, void *stream) {
    if (batch < 0) return -2;
    if (batch > 0 && !y) return -1;
    if (batch > 0 && !out) return -3;
    return lf_err(launch_predict(y, batch, out, (hipStream_t)stream));
}

int qrdm_batch_check(qrdm_batch_plan *plan, double *const *A, const int64_t *rank, double band, double *est,
                     int32_t *ok, void *stream) {
    int32_t batch;
    LfArgs q;
    int dev;
    if (qb_plan_sizes(plan, &batch, &q.m, &q.n, &q.lda, &dev) != 0) return -1;
    if (batch > 0 && !A) return -2;
    if (batch > 0 && !rank) return -3;
    if (!(band >= 0.0)) return -4;
    if (batch > 0 && !ok) return -6;
    q.A = A;
    return lf_err(launch_ice_check(q, batch, rank, band, est, ok, (hipStream_t)stream));
}

}  // extern "C"
