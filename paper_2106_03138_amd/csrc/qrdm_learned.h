// Internal declarations of the learned parameter predictor (not public ABI).
#pragma once
#include "qrdm_batched.h"

#define LF_NFEAT 16
#define LF_NH 64
#define LF_NOUT 3
#define LF_NPARAM (LF_NH * LF_NFEAT + LF_NH + LF_NH * LF_NH + LF_NH + LF_NOUT * LF_NH + LF_NOUT)
#define LF_NDELTA (LF_NOUT + 2 * LF_NH)  // per-sample errors: dy | dz2 | dz1
#define LF_NTAU 6
#define LF_NDELTA_GRID 4
#define LF_TAU_GRID {0.05, 0.15, 0.3, 0.5, 0.7, 0.9}
#define LF_DELTA_GRID {0.5, 0.7, 0.9, 0.95}

struct LfArgs {  // device arrays indexed by matrix id
    double *const *A;
    const int32_t *m, *n, *lda;
};

hipError_t launch_features(const LfArgs &q, int batch, double *feat, hipStream_t s);
hipError_t launch_mlp_forward(const float *P, const float *norm, const double *feat, int B, float *H1, float *H2,
                              float *Y, hipStream_t s);
hipError_t launch_mlp_backward(const float *P, const float *norm, const double *feat, const float *H1,
                               const float *H2, const float *Y, const float *T, int B, float *D, float *G,
                               float *sqerr, hipStream_t s);
hipError_t launch_adam(float *P, const float *G, float *M, float *V, int t, float lr, float b1, float b2, float eps,
                       hipStream_t s);
hipError_t launch_predict(const float *Y, int B, qrdm_batch_params *out, hipStream_t s);
hipError_t launch_ice_check(const LfArgs &q, int batch, const int64_t *rank, double band, double *est, int32_t *ok,
                            hipStream_t s);
