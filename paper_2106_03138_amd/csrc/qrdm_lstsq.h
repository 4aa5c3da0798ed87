// Internal declarations of the least-squares solve (not public ABI).
#pragma once
#include "qrdm_batched.h"

struct LsBatchArgs {  // device arrays indexed by matrix id
    double *const *A;
    const int32_t *m, *n, *lda;
    double *const *tau_house;
    int32_t *const *perm;
    const int64_t *rank;
    double *const *B;  // m[i] x nrhs, leading dimension max(1, m[i])
    double *const *X;  // n[i] x nrhs, leading dimension max(1, n[i])
    double *resid;     // nrhs per matrix, or null
    int32_t nrhs;
};

hipError_t launch_lstsq_one(const double *A, int m, int n, int64_t lda, const double *tauh, const int32_t *perm,
                            int64_t rank, double *B, int64_t ldb, double *X, int64_t ldx, int nrhs, double *resid,
                            hipStream_t s);
hipError_t launch_lstsq_batched(const LsBatchArgs &q, int batch, hipStream_t s);
hipError_t launch_trunc_one(const double *A, int m, int n, int64_t lda, int64_t rank, double eps1_scale,
                            int64_t *out, hipStream_t s);
hipError_t launch_trunc_batched(const LsBatchArgs &q, int batch, const int64_t *rank_in, double eps1_scale,
                                int64_t *rank_out, hipStream_t s);
