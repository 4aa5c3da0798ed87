// Column-norm kernels of QRDM/QRP on gfx950.
//
//  k_colnorm   initial column norms u_j = ||a_j|| (Algorithm 4, first step;
//              Algorithm 2 for QRP), one wavefront per column, coalesced
//              512-byte loads, fixed-order reduction; flags NaN/Inf.
//  k_downdate  partial norm update after a block (Section 3.2, the equation
//              after Algorithm 3) with the l new rows of R, made safe against
//              cancellation as Section 3.1 requires (reference DBu08): the norm
//              is recomputed from the data when the downdated value has lost
//              too much accuracy.
#include "qrdm_internal.h"

#define WAVES_PER_WG 4

__global__ void __launch_bounds__(64 * WAVES_PER_WG)
k_colnorm(const double *__restrict__ A, int64_t m, int64_t n, int64_t lda, double *vn1, double *vn2,
          QrdmCtl *ctl) {
    const int lane = threadIdx.x & 63;
    const int64_t j = (int64_t)blockIdx.x * WAVES_PER_WG + (threadIdx.x >> 6);
    if (j >= n) return;
    const double *col = A + j * lda;
    double s = 0.0;
    for (int64_t r = lane; r < m; r += 64) {
        double x = col[r];
        s += x * x;
    }
    s = wave_sum(s);
    if (lane == 0) {
        double v = sqrt(s);
        vn1[j] = v;
        vn2[j] = v;
        if (!isfinite(v)) atomicOr(&ctl->nonfinite, 1);
    }
}

hipError_t launch_colnorm(const double *A, int64_t m, int64_t n, int64_t lda, double *vn1, double *vn2,
                          QrdmCtl *ctl, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    dim3 grid((unsigned)((n + WAVES_PER_WG - 1) / WAVES_PER_WG));
    hipLaunchKernelGGL(k_colnorm, grid, dim3(64 * WAVES_PER_WG), 0, s, A, m, n, lda, vn1, vn2, ctl);
    return hipGetLastError();
}

// perm = identity, tau_house = 0, unless the norm sweep found NaN/Inf (then
// nothing is written).
__global__ void k_init(QrdmArgs a) {
    if (a.ctl->nonfinite) return;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < a.n) a.perm[i] = (int32_t)i;
    if (i < p_of(a)) a.tau_house[i] = 0.0;
}

hipError_t launch_init(QrdmArgs a, hipStream_t s) {
    int64_t cnt = a.n;
    if (cnt <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_init, dim3((unsigned)((cnt + 255) / 256)), dim3(256), 0, s, a);
    return hipGetLastError();
}

// One wavefront per column j >= n_s + l.  s_j = sum of squares of the l new
// rows of R in column j; q = max(0, 1 - s_j / vn1_j^2); q2 = q (vn1_j/vn2_j)^2.
// If q2 <= sqrt(eps_w) the norm of A[n_s+l:m, j] is recomputed (and vn2_j
// reset), else vn1_j <- vn1_j sqrt(q).  eps_w is the unit roundoff of the data
// the new rows were computed in (FP64, or FP32 for mixed-precision updates).
__global__ void __launch_bounds__(64 * WAVES_PER_WG) k_downdate(QrdmArgs a) {
    const QrdmCtl *ctl = a.ctl;
    // the step's state is final here (the next step's selection changes it)
    if (a.snap && blockIdx.x == 0 && threadIdx.x == 0) qrdm_write_snapshot(ctl, a.snap);
    if (qrdm_dm_idle(ctl)) return;
    const int64_t ns = ctl->ns;
    const int l = ctl->l;
    const int lane = threadIdx.x & 63;
    const int64_t j = ns + l + (int64_t)blockIdx.x * WAVES_PER_WG + (threadIdx.x >> 6);
    if (j >= a.n) return;
    const double v1 = a.vn1[j];
    if (v1 == 0.0) return;
    const double *col = a.A + j * a.lda;
    double s = 0.0;
    for (int r = lane; r < l; r += 64) {
        double x = col[ns + r];
        s += x * x;
    }
    s = wave_sum(s);
    double q = 1.0 - s / (v1 * v1);
    if (q < 0.0) q = 0.0;
    const double r12 = v1 / a.vn2[j];
    const double q2 = q * (r12 * r12);
    if (q2 <= a.tol3z) {
        double t = 0.0;
        for (int64_t r = ns + l + lane; r < a.m; r += 64) {
            double x = col[r];
            t += x * x;
        }
        t = wave_sum(t);
        if (lane == 0) {
            double v = sqrt(t);
            a.vn1[j] = v;
            a.vn2[j] = v;
            atomicAdd((unsigned long long *)&a.ctl->nrecompute, 1ull);
        }
    } else if (lane == 0) {
        a.vn1[j] = v1 * sqrt(q);
    }
}

hipError_t launch_downdate(QrdmArgs a, int64_t w_bound, hipStream_t s) {
    if (w_bound <= 0 && !a.snap) return hipSuccess;
    if (w_bound <= 0) w_bound = 1;  // one workgroup still writes the snapshot
    dim3 grid((unsigned)((w_bound + WAVES_PER_WG - 1) / WAVES_PER_WG));
    hipLaunchKernelGGL(k_downdate, grid, dim3(64 * WAVES_PER_WG), 0, s, a);
    return hipGetLastError();
}

// Start of a call: the control block zeroed with rank = -1 (no stopping test
// has held yet), and the n recompute flags of the column-pivoting loop cleared.
__global__ void k_ws_reset(QrdmCtl *ctl, int32_t *flag, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) flag[i] = 0;
    if (blockIdx.x == 0) {
        uint64_t *w = (uint64_t *)ctl;
        const int nw = (int)(sizeof(QrdmCtl) / 8);
        for (int k = threadIdx.x; k < nw; k += blockDim.x) w[k] = 0;
        __syncthreads();
        if (threadIdx.x == 0) ctl->rank = -1;
    }
}

hipError_t launch_ws_reset(QrdmCtl *ctl, int32_t *flag, int64_t n, hipStream_t s) {
    static_assert(sizeof(QrdmCtl) % 8 == 0, "the control block is cleared in 8-byte words");
    const int64_t cnt = n > 1 ? n : 1;
    hipLaunchKernelGGL(k_ws_reset, dim3((unsigned)((cnt + 255) / 256)), dim3(256), 0, s, ctl, flag, n);
    return hipGetLastError();
}

// End of a call: the rank in device memory (the first n_s where the stopping
// test held, else the number of reflectors), or -1 after NaN/Inf or a failed
// grid wait.
__global__ void k_rank_out(const QrdmCtl *ctl, int64_t *rank) {
    if (threadIdx.x != 0) return;
    int64_t r = ctl->rank >= 0 ? ctl->rank : ctl->ns;
    if (ctl->nonfinite || ctl->error) r = -1;
    *rank = r;
}

hipError_t launch_rank_out(const QrdmCtl *ctl, int64_t *rank, hipStream_t s) {
    hipLaunchKernelGGL(k_rank_out, dim3(1), dim3(64), 0, s, ctl, rank);
    return hipGetLastError();
}
