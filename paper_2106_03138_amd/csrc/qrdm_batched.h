// Internal declarations of the batched QRDM path (not part of the public ABI).
#pragma once
#include "qrdm.h"
#include <float.h>

#include "qrdm_internal.h"

#define QB_NMAX 512  // largest n of a batched matrix (partial norms live in LDS)
#define QB_KM 64     // largest k_DM of a batched factorization
#define QB_VARIANTS 3

// Arguments of one persistent launch (one size class).  All arrays are device
// arrays indexed by the matrix id, except `order` (ids of this class, longest
// first) and `counters` ([0] queue head, [1] workgroups done; zero between launches).
struct QbArgs {
    double *const *A;
    const int32_t *m, *n, *lda;
    double *const *tau_house;
    int32_t *const *perm;
    int64_t *rank;
    int32_t *status;
    int64_t *info;  // [4 per matrix]: outer steps, panel breaks, scalar-pivoting steps, clock ticks; or null
    const qrdm_batch_params *pm;  // per-matrix (tau, delta, kmax) or null
    const int32_t *order;
    int32_t count;
    uint32_t *counters;
    double tau, delta;
    int32_t kmax, stop_rule;
    double eps1_scale;
    int32_t certified;  // delta <= tau^2 / (nL - 1) per step (eq. delta_max)
    // the checked form (qrdm_batch_factor_checked): after a matrix is factored with
    // its per-matrix parameters, the online check; a matrix that fails it is
    // restored from pristine[i] and factored again with the plan's parameters
    const double *const *pristine = nullptr;
    double band = 0.0;
    int32_t *ok = nullptr;  // 1: the per-matrix parameters kept, 0: factored again
};

// Incremental condition estimate (Bischof) of sigma_min(R11), R11 the leading
// r x r block (r >= 1) of the R stored in A (column-major, leading dimension
// lda), on one wavefront; sx: r doubles of LDS for the unit vector x.  Per
// column j: alpha = x . R[0:j, j], then the smallest eigenpair of
// [[est^2 + alpha^2, alpha gamma], [alpha gamma, gamma^2]] (gamma = r_jj), with
// lambda_min = est^2 gamma^2 / lambda_max (the determinant over the larger root).
// Returns est in every lane and the smallest |r_jj| (j < r) in *dmin.  The
// online check and the checked batched factorization both take it from here.
__device__ inline double qb_ice(const double *A, int lda, int r, double *sx, double *dmin) {
    const int lane = threadIdx.x & 63;
    double dm = DBL_MAX;
    for (int i = lane; i < r; i += 64) {
        const double d = fabs(A[(int64_t)i * lda + i]);
        dm = d < dm ? d : dm;
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        const double od = __shfl_xor(dm, o, 64);
        dm = od < dm ? od : dm;
    }
    *dmin = dm;
    double est = fabs(A[0]);
    if (lane == 0) sx[0] = 1.0;
    __builtin_amdgcn_wave_barrier();
    for (int j = 1; j < r; ++j) {
        const double *col = A + (int64_t)j * lda;
        double a = 0.0;
        for (int i = lane; i < j; i += 64) a += sx[i] * col[i];
        const double alpha = wave_sum(a);
        const double gamma = col[j];
        const double pp = est * est + alpha * alpha, qq = alpha * gamma, rr = gamma * gamma;
        const double lmax = 0.5 * (pp + rr) + hypot(0.5 * (pp - rr), qq);
        const double lmin = lmax > 0.0 ? (est * est) * rr / lmax : 0.0;
        const double v1a = -qq, v1b = pp - lmin, v2a = rr - lmin, v2b = -qq;
        const bool first = hypot(v1a, v1b) >= hypot(v2a, v2b);
        double sa = first ? v1a : v2a, cb = first ? v1b : v2b;
        const double nv = hypot(sa, cb);
        if (nv > 0.0) {
            sa /= nv;
            cb /= nv;
        } else {
            sa = 1.0;
            cb = 0.0;
        }
        __builtin_amdgcn_wave_barrier();  // every lane has read sx[0..j) for alpha
        for (int i = lane; i < j; i += 64) sx[i] *= sa;
        if (lane == 0) sx[j] = cb;
        est = sqrt(lmin);
        __builtin_amdgcn_wave_barrier();
    }
    return est;
}

// variant: 0 = 256 threads, 16 columns per wavefront in the trailing update,
//          panel rows in registers; 1 = 32 columns, registers; 2 = 16 columns,
//          panel read from memory
int qb_variant_threads(int variant);
hipError_t launch_qrdm_batched(const QbArgs &q, int variant, int grid, hipStream_t s);
hipError_t qb_occupancy(int variant, int *wgs_per_cu);

// device copies of the plan's sizes (for the learned-predictor kernels)
extern "C" int qb_plan_sizes(const qrdm_batch_plan *pl, int32_t *batch, const int32_t **m, const int32_t **n,
                             const int32_t **lda, int *device);
