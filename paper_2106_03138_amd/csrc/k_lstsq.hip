// Least squares and post-hoc rank truncation on top of a pivoted QR
// factorization.
//
// With A P = Q [R11 R12; 0 R22] from QRDM or QRP and rank r, column pivoting
// singles out the basic solution of min ||A x - b||, the one with r nonzeros
// (Section 1):  y = Q_r^T b with Q_r = H_0 ... H_{r-1},  R11 x1 = y[0:r),
// x[perm[j]] = x1[j] for j < r and 0 otherwise.  The residual is Q_r [0; y[r:m)]
// exactly (x is zero on the columns of R12 and R22), so ||A x - b|| = ||y[r:m)||.
//
// One workgroup per (matrix, group of up to LS_NRC right-hand sides):
//   1. Q_r^T b in blocks of LS_NB reflectors.  One pass over the rows
//      accumulates w = V^T b and the strict lower triangle of V^T V, a single
//      workgroup reduction sums all of them, the triangular recurrence
//      z_j = tau_j (w_j - sum_{k<j} (v_j . v_k) z_k) (the reflectors applied one
//      after the other) runs on one lane per right-hand side, and a second pass
//      applies b -= V z.
//   2. R11 x1 = y[0:r) by blocks of LS_BS rows from the bottom: the diagonal
//      block is solved from LDS by one lane per right-hand side, then every
//      thread updates its rows above the block (column-oriented substitution).
//   3. Scatter through perm; ||y[r:m)|| per right-hand side.
// Each thread owns the rows tid + LS_NT q of b in every phase, so no thread
// reads a value of b that another thread stored: shared data moves through LDS.
#include "qrdm_lstsq.h"

#define LS_NT 256
#define LS_NB 8    // reflectors per block of phase 1
#define LS_BS 16   // rows per block of phase 2
#define LS_NRC 4   // right-hand sides per workgroup
#define LS_NG (LS_NB * (LS_NB - 1) / 2)  // strict lower V^T V entries
static_assert(LS_NG + LS_NB * LS_NRC <= 64, "one reduced value per lane");

struct LsShared {
    double part[LS_NT / 64][64];
    double z[LS_NB][LS_NRC];
    double ynext[LS_BS][LS_NRC];
    double rt[LS_BS][LS_BS + 1];
    double xs[LS_BS][LS_NRC];
    double rs[LS_NT / 64][LS_NRC];
};

// Halving butterfly over the wavefront: afterwards v[0] of lane L holds the
// wavefront sum of entry L (the half kept is the upper one when the lane's
// offset bit is set), in a fixed order.
template <int O>
__device__ __forceinline__ void ls_rs_stage(double (&v)[64], int lane) {
    const bool up = (lane & O) != 0;
#pragma unroll
    for (int i = 0; i < O; ++i) {
        const double keep = up ? v[O + i] : v[i];
        const double send = up ? v[i] : v[O + i];
        v[i] = keep + __shfl_xor(send, O, 64);
    }
}

__device__ __forceinline__ double ls_reduce_scatter(double (&v)[64], int lane) {
    ls_rs_stage<32>(v, lane);
    ls_rs_stage<16>(v, lane);
    ls_rs_stage<8>(v, lane);
    ls_rs_stage<4>(v, lane);
    ls_rs_stage<2>(v, lane);
    ls_rs_stage<1>(v, lane);
    return v[0];
}

__device__ __forceinline__ double ls_wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// v_j[row] of reflector `col`: 0 above the diagonal, 1 on it, stored below it.
__device__ __forceinline__ double ls_v(const double *A, int64_t lda, int row, int col, bool live) {
    if (!live || row < col) return 0.0;
    return row == col ? 1.0 : A[(int64_t)col * lda + row];
}

__device__ __forceinline__ void ls_core(const double *A, int m, int n, int64_t lda, const double *tauh,
                                        const int32_t *perm, int64_t rank, double *B, int64_t ldb, double *X,
                                        int64_t ldx, int nc, double *resid, LsShared &sh) {
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int p = m < n ? m : n;
    if (rank < 0) {  // the factorization failed (NaN/Inf): no solution
        for (int j = tid; j < n; j += LS_NT)
            for (int c = 0; c < nc; ++c) X[(int64_t)c * ldx + j] = __builtin_nan("");
        if (tid < nc && resid) resid[tid] = __builtin_nan("");
        return;
    }
    const int r = rank > p ? p : (int)rank;

    // ---------------------------------------------------------- 1. Q_r^T b
    for (int k0 = 0; k0 < r; k0 += LS_NB) {
        const int nb = r - k0 < LS_NB ? r - k0 : LS_NB;
        double acc[64];
#pragma unroll
        for (int i = 0; i < 64; ++i) acc[i] = 0.0;
        for (int row = (k0 & ~(LS_NT - 1)) + tid; row < m; row += LS_NT) {
            if (row < k0) continue;
            double v[LS_NB], b[LS_NRC];
#pragma unroll
            for (int j = 0; j < LS_NB; ++j) v[j] = ls_v(A, lda, row, k0 + j, j < nb);
#pragma unroll
            for (int c = 0; c < LS_NRC; ++c) b[c] = c < nc ? B[(int64_t)c * ldb + row] : 0.0;
            int g = 0;
#pragma unroll
            for (int j = 1; j < LS_NB; ++j)
#pragma unroll
                for (int k = 0; k < j; ++k) acc[g++] += v[j] * v[k];
#pragma unroll
            for (int j = 0; j < LS_NB; ++j)
#pragma unroll
                for (int c = 0; c < LS_NRC; ++c) acc[LS_NG + LS_NRC * j + c] += v[j] * b[c];
        }
        sh.part[wv][lane] = ls_reduce_scatter(acc, lane);
        __syncthreads();
        if (wv == 0) {
            double tot = 0.0;
#pragma unroll
            for (int w = 0; w < LS_NT / 64; ++w) tot += sh.part[w][lane];
            // lane c < LS_NRC runs the recurrence of right-hand side c
            const int c = lane & (LS_NRC - 1);
            double z[LS_NB];
#pragma unroll
            for (int j = 0; j < LS_NB; ++j) {
                double s = __shfl(tot, LS_NG + LS_NRC * j + c, 64);
#pragma unroll
                for (int k = 0; k < j; ++k) s -= __shfl(tot, j * (j - 1) / 2 + k, 64) * z[k];
                z[j] = j < nb ? tauh[k0 + j] * s : 0.0;
            }
            if (lane < LS_NRC) {
#pragma unroll
                for (int j = 0; j < LS_NB; ++j) sh.z[j][lane] = z[j];
            }
        }
        __syncthreads();
        double zz[LS_NB][LS_NRC];
#pragma unroll
        for (int j = 0; j < LS_NB; ++j)
#pragma unroll
            for (int c = 0; c < LS_NRC; ++c) zz[j][c] = sh.z[j][c];
        for (int row = (k0 & ~(LS_NT - 1)) + tid; row < m; row += LS_NT) {
            if (row < k0) continue;
            double v[LS_NB];
#pragma unroll
            for (int j = 0; j < LS_NB; ++j) v[j] = ls_v(A, lda, row, k0 + j, j < nb);
#pragma unroll
            for (int c = 0; c < LS_NRC; ++c) {
                if (c >= nc) continue;
                double b = B[(int64_t)c * ldb + row];
#pragma unroll
                for (int j = 0; j < LS_NB; ++j) b -= v[j] * zz[j][c];
                B[(int64_t)c * ldb + row] = b;
            }
        }
    }

    // ------------------------------------------- residual norm and preamble
    {
        double s[LS_NRC];
#pragma unroll
        for (int c = 0; c < LS_NRC; ++c) s[c] = 0.0;
        for (int row = (r & ~(LS_NT - 1)) + tid; row < m; row += LS_NT) {
            if (row < r) continue;
#pragma unroll
            for (int c = 0; c < LS_NRC; ++c) {
                const double y = c < nc ? B[(int64_t)c * ldb + row] : 0.0;
                s[c] += y * y;
            }
        }
#pragma unroll
        for (int c = 0; c < LS_NRC; ++c) {
            const double t = ls_wave_sum(s[c]);
            if (lane == 0) sh.rs[wv][c] = t;
        }
    }
    for (int j = r + tid; j < n; j += LS_NT) {
        const int pj = perm[j];
        if (pj < 0 || pj >= n) continue;  // not a permutation: the entry is skipped
        for (int c = 0; c < nc; ++c) X[(int64_t)c * ldx + pj] = 0.0;
    }
    if (r > 0) {
        const int i0 = ((r - 1) / LS_BS) * LS_BS;
        for (int row = (i0 & ~(LS_NT - 1)) + tid; row < r; row += LS_NT) {
            if (row < i0) continue;
#pragma unroll
            for (int c = 0; c < LS_NRC; ++c) sh.ynext[row - i0][c] = c < nc ? B[(int64_t)c * ldb + row] : 0.0;
        }
        const int a = tid % LS_BS, bcol = tid / LS_BS;  // LS_NT == LS_BS * LS_BS
        sh.rt[a][bcol] = (bcol >= a && i0 + bcol < r) ? A[(int64_t)(i0 + bcol) * lda + i0 + a] : 0.0;
    }
    __syncthreads();
    if (tid < nc && resid) {
        double t = 0.0;
#pragma unroll
        for (int w = 0; w < LS_NT / 64; ++w) t += sh.rs[w][tid];
        resid[tid] = sqrt(t);
    }

    // ------------------------------------------------- 2. back substitution
    for (int i0 = ((r - 1) / LS_BS) * LS_BS; r > 0 && i0 >= 0; i0 -= LS_BS) {
        const int s = r - i0 < LS_BS ? r - i0 : LS_BS;
        if (wv == 0) {
            const int c = lane & (LS_NRC - 1);
            double x[LS_BS];
#pragma unroll
            for (int i = LS_BS - 1; i >= 0; --i) {
                double t = 0.0;
                if (i < s) {
                    t = sh.ynext[i][c];
#pragma unroll
                    for (int k = i + 1; k < LS_BS; ++k) t -= sh.rt[i][k] * x[k];
                    t = t / sh.rt[i][i];
                }
                x[i] = t;
            }
            if (lane < nc) {
#pragma unroll
                for (int i = 0; i < LS_BS; ++i) {
                    if (i >= s) continue;
                    sh.xs[i][lane] = x[i];
                    B[(int64_t)lane * ldb + i0 + i] = x[i];
                    const int pj = perm[i0 + i];
                    if (pj >= 0 && pj < n) X[(int64_t)lane * ldx + pj] = x[i];
                }
            }
        }
        __syncthreads();
        const int n0 = i0 - LS_BS;  // first row of the next block (when i0 > 0)
        for (int row = tid; row < i0; row += LS_NT) {
            double y[LS_NRC];
#pragma unroll
            for (int c = 0; c < LS_NRC; ++c) y[c] = c < nc ? B[(int64_t)c * ldb + row] : 0.0;
            for (int k = 0; k < s; ++k) {
                const double rv = A[(int64_t)(i0 + k) * lda + row];
#pragma unroll
                for (int c = 0; c < LS_NRC; ++c) y[c] -= rv * sh.xs[k][c];
            }
#pragma unroll
            for (int c = 0; c < LS_NRC; ++c)
                if (c < nc) B[(int64_t)c * ldb + row] = y[c];
            if (row >= n0) {
#pragma unroll
                for (int c = 0; c < LS_NRC; ++c) sh.ynext[row - n0][c] = y[c];
            }
        }
        if (i0 > 0) {
            const int a = tid % LS_BS, bcol = tid / LS_BS;
            sh.rt[a][bcol] = bcol >= a ? A[(int64_t)(n0 + bcol) * lda + n0 + a] : 0.0;
        }
        __syncthreads();
    }
}

static_assert(LS_NT == LS_BS * LS_BS, "one thread per entry of a diagonal block");

__global__ void __launch_bounds__(LS_NT) k_lstsq_one(const double *A, int m, int n, int64_t lda, const double *tauh,
                                                     const int32_t *perm, int64_t rank, double *B, int64_t ldb,
                                                     double *X, int64_t ldx, int nrhs, double *resid) {
    __shared__ LsShared sh;
    const int c0 = blockIdx.x * LS_NRC;
    const int nc = nrhs - c0 < LS_NRC ? nrhs - c0 : LS_NRC;
    ls_core(A, m, n, lda, tauh, perm, rank, B + (int64_t)c0 * ldb, ldb, X + (int64_t)c0 * ldx, ldx, nc,
            resid ? resid + c0 : nullptr, sh);
}

__global__ void __launch_bounds__(LS_NT) k_lstsq_batched(LsBatchArgs q) {
    __shared__ LsShared sh;
    const int mi = blockIdx.x;
    const int c0 = blockIdx.y * LS_NRC;
    const int nc = q.nrhs - c0 < LS_NRC ? q.nrhs - c0 : LS_NRC;
    const int m = q.m[mi], n = q.n[mi];
    const int64_t ldb = m > 1 ? m : 1, ldx = n > 1 ? n : 1;
    ls_core(q.A[mi], m, n, q.lda[mi], q.tau_house[mi], q.perm[mi], q.rank[mi], q.B[mi] + (int64_t)c0 * ldb, ldb,
            q.X[mi] + (int64_t)c0 * ldx, ldx, nc, q.resid ? q.resid + (int64_t)mi * q.nrhs + c0 : nullptr, sh);
}

// ------------------------------------------------------ rank truncation
// Post-processing of R (Section 5: the diagonal of R shows the gap of the
// singular values even where the stopping criterion overestimates the rank):
// the first i < rank with |r_ii| <= eps_1 |r_00| (NaN counts as small), else
// rank; eps_1 = scale * 2^-52 with scale = n when eps1_scale <= 0.
__device__ __forceinline__ int64_t tr_core(const double *A, int m, int n, int64_t lda, int64_t rank,
                                           double eps1_scale) {
    __shared__ int sfirst[LS_NT / 64];
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int p = m < n ? m : n;
    if (rank <= 0) return rank < 0 ? rank : 0;
    const int r = rank > p ? p : (int)rank;
    if (r == 0) return 0;
    const double scale = eps1_scale > 0.0 ? eps1_scale : (double)n;
    const double thr = scale * 0x1p-52 * fabs(A[0]);
    int first = r;
    for (int i = tid; i < r; i += LS_NT)
        if (!(fabs(A[(int64_t)i * lda + i]) > thr)) {
            first = i;  // the smallest such i of this thread (i increases)
            break;
        }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        const int other = __shfl_xor(first, o, 64);
        first = other < first ? other : first;
    }
    if (lane == 0) sfirst[wv] = first;
    __syncthreads();
    int best = sfirst[0];
#pragma unroll
    for (int w = 1; w < LS_NT / 64; ++w) best = sfirst[w] < best ? sfirst[w] : best;
    return best;
}

__global__ void __launch_bounds__(LS_NT) k_trunc_one(const double *A, int m, int n, int64_t lda, int64_t rank,
                                                     double eps1_scale, int64_t *out) {
    const int64_t k = tr_core(A, m, n, lda, rank, eps1_scale);
    if (threadIdx.x == 0) *out = k;
}

__global__ void __launch_bounds__(LS_NT) k_trunc_batched(LsBatchArgs q, const int64_t *rank_in, double eps1_scale,
                                                         int64_t *rank_out) {
    const int mi = blockIdx.x;
    const int64_t k = tr_core(q.A[mi], q.m[mi], q.n[mi], q.lda[mi], rank_in[mi], eps1_scale);
    __syncthreads();  // every thread has read rank_in[mi] (rank_out may alias it)
    if (threadIdx.x == 0) rank_out[mi] = k;
}

hipError_t launch_trunc_one(const double *A, int m, int n, int64_t lda, int64_t rank, double eps1_scale,
                            int64_t *out, hipStream_t s) {
    hipLaunchKernelGGL(k_trunc_one, dim3(1), dim3(LS_NT), 0, s, A, m, n, lda, rank, eps1_scale, out);
    return hipGetLastError();
}

hipError_t launch_trunc_batched(const LsBatchArgs &q, int batch, const int64_t *rank_in, double eps1_scale,
                                int64_t *rank_out, hipStream_t s) {
    if (batch <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_trunc_batched, dim3(batch), dim3(LS_NT), 0, s, q, rank_in, eps1_scale, rank_out);
    return hipGetLastError();
}

hipError_t launch_lstsq_one(const double *A, int m, int n, int64_t lda, const double *tauh, const int32_t *perm,
                            int64_t rank, double *B, int64_t ldb, double *X, int64_t ldx, int nrhs, double *resid,
                            hipStream_t s) {
    if (nrhs <= 0) return hipSuccess;
    const int groups = (nrhs + LS_NRC - 1) / LS_NRC;
    hipLaunchKernelGGL(k_lstsq_one, dim3(groups), dim3(LS_NT), 0, s, A, m, n, lda, tauh, perm, rank, B, ldb, X, ldx,
                       nrhs, resid);
    return hipGetLastError();
}

hipError_t launch_lstsq_batched(const LsBatchArgs &q, int batch, hipStream_t s) {
    if (batch <= 0 || q.nrhs <= 0) return hipSuccess;
    const int groups = (q.nrhs + LS_NRC - 1) / LS_NRC;
    hipLaunchKernelGGL(k_lstsq_batched, dim3(batch, groups), dim3(LS_NT), 0, s, q);
    return hipGetLastError();
}
