// Internal declarations of the batched QRDM path (not part of the public ABI).
#pragma once
#include "qrdm.h"
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
};

// variant: 0 = 256 threads, 16 columns per wavefront in the trailing update,
//          panel rows in registers; 1 = 32 columns, registers; 2 = 16 columns,
//          panel read from memory
int qb_variant_threads(int variant);
hipError_t launch_qrdm_batched(const QbArgs &q, int variant, int grid, hipStream_t s);
hipError_t qb_occupancy(int variant, int *wgs_per_cu);

// device copies of the plan's sizes (for the learned-predictor kernels)
extern "C" int qb_plan_sizes(const qrdm_batch_plan *pl, int32_t *batch, const int32_t **m, const int32_t **n,
                             const int32_t **lda, int *device);
