// Host entry points of the least-squares solve (C ABI of include/qrdm.h).
#include "qrdm_lstsq.h"

static int ls_err(hipError_t e) { return e == hipSuccess ? QRDM_OK : QRDM_ERR_HIP + (int)e; }

extern "C" {

int qrdm_lstsq(const double *A, int64_t m, int64_t n, int64_t lda, const double *tau_house, const int32_t *perm,
               int64_t rank, double *B, int64_t ldb, int64_t nrhs, double *X, int64_t ldx, double *resid,
               void *stream) {
    if (m < 0 || m > INT32_MAX) return -2;
    if (n < 0 || n > INT32_MAX) return -3;
    if (lda < (m > 1 ? m : 1)) return -4;
    if (nrhs < 0 || nrhs > INT32_MAX) return -10;
    if (ldb < (m > 1 ? m : 1)) return -9;
    if (ldx < (n > 1 ? n : 1)) return -12;
    if (nrhs == 0) return QRDM_OK;
    const int64_t p = m < n ? m : n;
    if (p > 0 && !A) return -1;
    if (p > 0 && rank > 0 && !tau_house) return -5;
    if (n > 0 && rank >= 0 && !perm) return -6;
    if (m > 0 && !B) return -8;
    if (n > 0 && !X) return -11;
    return ls_err(launch_lstsq_one(A, (int)m, (int)n, lda, tau_house, perm, rank, B, ldb, X, ldx, (int)nrhs, resid,
                                   (hipStream_t)stream));
}

int qrdm_batch_lstsq(qrdm_batch_plan *plan, double *const *A, double *const *tau_house, int32_t *const *perm,
                     const int64_t *rank, double *const *B, double *const *X, int32_t nrhs, double *resid,
                     void *stream) {
    int32_t batch;
    LsBatchArgs q;
    int dev;
    if (qb_plan_sizes(plan, &batch, &q.m, &q.n, &q.lda, &dev) != 0) return -1;
    if (nrhs < 0) return -8;
    if (batch == 0 || nrhs == 0) return QRDM_OK;
    if (!A) return -2;
    if (!tau_house) return -3;
    if (!perm) return -4;
    if (!rank) return -5;
    if (!B) return -6;
    if (!X) return -7;
    if ((int64_t)batch * nrhs > INT32_MAX) return QRDM_ERR_UNSUPPORTED;
    q.A = A;
    q.tau_house = tau_house;
    q.perm = perm;
    q.rank = rank;
    q.B = B;
    q.X = X;
    q.resid = resid;
    q.nrhs = nrhs;
    return ls_err(launch_lstsq_batched(q, batch, (hipStream_t)stream));
}

int qrdm_truncate_rank(const double *A, int64_t m, int64_t n, int64_t lda, int64_t rank, double eps1_scale,
                       int64_t *rank_out, void *stream) {
    if (m < 0 || m > INT32_MAX) return -2;
    if (n < 0 || n > INT32_MAX) return -3;
    if (lda < (m > 1 ? m : 1)) return -4;
    if (!(eps1_scale == eps1_scale)) return -6;
    if (!rank_out) return -7;
    if (m > 0 && n > 0 && rank > 0 && !A) return -1;
    return ls_err(launch_trunc_one(A, (int)m, (int)n, lda, rank, eps1_scale, rank_out, (hipStream_t)stream));
}

int qrdm_batch_truncate_rank(qrdm_batch_plan *plan, double *const *A, const int64_t *rank_in, double eps1_scale,
                             int64_t *rank_out, void *stream) {
    int32_t batch;
    LsBatchArgs q;
    int dev;
    if (qb_plan_sizes(plan, &batch, &q.m, &q.n, &q.lda, &dev) != 0) return -1;
    if (!(eps1_scale == eps1_scale)) return -4;
    if (batch == 0) return QRDM_OK;
    if (!A) return -2;
    if (!rank_in) return -3;
    if (!rank_out) return -5;
    q.A = A;
    return ls_err(launch_trunc_batched(q, batch, rank_in, eps1_scale, rank_out, (hipStream_t)stream));
}

}  // extern "C"
