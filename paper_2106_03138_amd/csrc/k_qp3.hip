// QR with column pivoting (Algorithm 2 of the paper, QRP) in the blocked form
// that LAPACK xgeqp3 uses (Section 3.1 cites it as QP3): one pivot per step,
// with the trailing update deferred and accumulated as A_tr -= V F^T, so each
// step costs one matrix-vector sweep of the trailing matrix (the BLAS-2 part
// whose cost Section 5 identifies) and every nb steps one BLAS-3 update.
// It is the classical baseline and the scalar-pivoting continuation of QRDM
// once the partial norms reach the noise level (eq. column_norm_bound_DM).
//
// One step (column j = n_s, block [k0, k0 + nb), b = j - k0 reflectors done):
//   k_qp_select  advance the step state; arg-max of the partial norms (lowest
//                position on ties); stopping test; swap bookkeeping (vn1, vn2,
//                perm, the F row of both columns).
//   k_qp_column  per row slab: normalize the previous reflector; swap columns;
//                x = A[j:m, j] - V F[j,:]^T (the deferred update of the pivot
//                column); partial sums ||x_below||^2, x_j, V^T x.
//   k_qp_gemv    per trailing column c (one wavefront): reflector scalars from
//                the partials (LAPACK larfg convention); F[c, b] = tau v^T a_c
//                corrected by the earlier reflectors of the block; the pivot
//                row A[j, c] of R; the partial norm update of column c with the
//                cancellation-safe recompute flag.
//   k_gemm2      (mode 1) at block end, A_tr -= V F^T with V read in place.
//   k_qp_close   at block end: recompute flagged norms; at the very end
//                normalize the last reflector.
#include <float.h>

#include "qrdm_internal.h"

#define QP_ROWS 256  // rows per workgroup of the pivot-column pass
#define QP_NBMAX 64

hipError_t launch_gemm2_qp3(QrdmArgs a, const double *Vw, int64_t ldv, const double *Fz, int64_t t_bound,
                            int64_t w_bound, hipStream_t s);

// ------------------------------------------------------------ init / select
__global__ void k_qp_init(QrdmArgs a, int nb) {
    QrdmCtl *c = a.ctl;
    if (!c->done) c->ns += c->l;  // finish the advance of a preceding QRDM step
    c->qp_k0 = c->ns;
    c->qp_b = 0;
    c->qp_pend = 0;
    c->qp_end = 0;
    c->qp_stop = 0;
    c->qp_flag = 0;
    c->qp_nb = nb;
    c->l = 0;
}

hipError_t launch_qp3_init(QrdmArgs a, int nb, hipStream_t s) {
    hipLaunchKernelGGL(k_qp_init, dim3(1), dim3(1), 0, s, a, nb);
    return hipGetLastError();
}

// Does the step at column ns close the current block?  Evaluated identically by
// every kernel after the GEMV pass (the fields it reads are final by then).
__device__ __forceinline__ bool qp_closes(const QrdmCtl *c, int64_t p, int nb, int *kb, int64_t *last) {
    const int b = c->qp_b;
    const bool stop = c->qp_stop != 0;
    const bool end = stop || (b + 1 == nb) || (c->ns + 1 == p) || c->qp_flag;
    const int k = stop ? b : b + 1;  // reflectors in the block
    *kb = k;
    *last = c->qp_k0 + k - 1;
    return end;
}

__device__ __forceinline__ bool qp_better(double va, int ja, double vb, int jb) {
    return va > vb || (va == vb && ja < jb);
}

__global__ void __launch_bounds__(1024) k_qp_select(QrdmArgs a, double *Fz) {
    QrdmCtl *ctl = a.ctl;
    __shared__ double s_v[16];
    __shared__ int s_j[16];
    __shared__ int s_go, s_norm;
    if (ctl->done) return;
    const int tid = threadIdx.x;
    if (tid == 0 && ctl->l == 1) {
        // advance from the previous step, which made the reflector of column ns;
        // that reflector stays pending (normalized by the next column pass)
        int kb;
        int64_t last;
        if (qp_closes(ctl, p_of(a), ctl->qp_nb, &kb, &last)) {
            ctl->qp_k0 = last + 1;
            ctl->qp_b = 0;
            ctl->qp_flag = 0;
        } else {
            ctl->qp_b += 1;
        }
        ctl->qp_pend = 1;
        ctl->ns += 1;
        ctl->l = 0;
    }
    __syncthreads();
    const int64_t j = ctl->ns;
    const int64_t p = p_of(a);
    if (j >= p) {
        if (tid == 0) {
            ctl->done = 1;
            if (ctl->rank < 0) ctl->rank = j;
        }
        return;
    }
    double bv = -1.0;
    int bj = 0x7fffffff;
    for (int64_t c = j + tid; c < a.n; c += 1024) {
        const double v = a.vn1[c];
        if (v > bv) { bv = v; bj = (int)c; }
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        const double ov = __shfl_xor(bv, o, 64);
        const int oj = __shfl_xor(bj, o, 64);
        if (qp_better(ov, oj, bv, bj)) { bv = ov; bj = oj; }
    }
    if ((tid & 63) == 0) { s_v[tid >> 6] = bv; s_j[tid >> 6] = bj; }
    __syncthreads();
    if (tid == 0) {
        s_norm = 0;
        double uv = s_v[0];
        int uj = s_j[0];
        for (int i = 1; i < 16; ++i)
            if (qp_better(s_v[i], s_j[i], uv, uj)) { uv = s_v[i]; uj = s_j[i]; }
        double amax = ctl->amax;
        if (ctl->nblocks == 0 && j == 0) { amax = uv; ctl->amax = amax; }
        int go = 1;
        if (amax == 0.0) {
            ctl->rank = 0;
            ctl->done = 1;
            go = 0;
        } else if (ctl->rank < 0) {
            const double lhs = (a.stop_rule == 1) ? uv : sqrt((double)(a.n - j)) * uv;
            if (lhs <= a.eps1 * amax) {
                ctl->rank = j;
                if (a.stop_rule != 2) {
                    go = 0;
                    if (ctl->qp_b > 0) {  // close the block so the trailing block is up to date
                        ctl->qp_stop = 1;
                    } else {
                        ctl->done = 1;
                        s_norm = ctl->qp_pend;  // the previous block's last reflector
                    }
                }
            }
        }
        if (go) {
            ctl->jmax = uj;
            ctl->umax = uv;
            ctl->nblocks += 1;
            if (uj != j) {
                double t1 = a.vn1[j]; a.vn1[j] = a.vn1[uj]; a.vn1[uj] = t1;
                t1 = a.vn2[j]; a.vn2[j] = a.vn2[uj]; a.vn2[uj] = t1;
                const int32_t pp = a.perm[j]; a.perm[j] = a.perm[uj]; a.perm[uj] = pp;
            }
        }
        s_go = go && (uj != j);
    }
    __syncthreads();
    if (s_norm) {  // stopping right after a block end: normalize reflector j-1 in place
        const double rden = 1.0 / ctl->qp_den;
        for (int64_t r = j + tid; r < a.m; r += 1024) a.A[(j - 1) * a.lda + r] *= rden;
        if (tid == 0) a.A[(j - 1) * a.lda + (j - 1)] = ctl->qp_beta;
        return;
    }
    // swap the F rows of columns j and jmax (F^T stored as Fz[b'][column])
    if (s_go) {
        const int uj = ctl->jmax;
        const int b = ctl->qp_b;
        for (int bb = tid; bb < b; bb += 1024) {
            const double t1 = Fz[(int64_t)bb * a.n + j];
            Fz[(int64_t)bb * a.n + j] = Fz[(int64_t)bb * a.n + uj];
            Fz[(int64_t)bb * a.n + uj] = t1;
        }
    }
}

// ------------------------------------------------------------ pivot column
#define QP_NB_REG 32  // earlier reflectors of the block held in registers per row

// Sum of 32 values over a wavefront by butterfly reduce-scatter (32 shuffles):
// on return lane L holds the sum of value (L >> 1) when L is even.
__device__ __forceinline__ double qp_reduce_scatter32(const double (&v)[QP_NB_REG], int lane) {
    double c16[16], c8[8], c4[4], c2[2];
    const bool b5 = lane & 32, b4 = lane & 16, b3 = lane & 8, b2 = lane & 4, b1 = lane & 2;
#pragma unroll
    for (int k = 0; k < 16; ++k) c16[k] = (b5 ? v[16 + k] : v[k]) + __shfl_xor(b5 ? v[k] : v[16 + k], 32, 64);
#pragma unroll
    for (int k = 0; k < 8; ++k) c8[k] = (b4 ? c16[8 + k] : c16[k]) + __shfl_xor(b4 ? c16[k] : c16[8 + k], 16, 64);
#pragma unroll
    for (int k = 0; k < 4; ++k) c4[k] = (b3 ? c8[4 + k] : c8[k]) + __shfl_xor(b3 ? c8[k] : c8[4 + k], 8, 64);
#pragma unroll
    for (int k = 0; k < 2; ++k) c2[k] = (b2 ? c4[2 + k] : c4[k]) + __shfl_xor(b2 ? c4[k] : c4[2 + k], 4, 64);
    const double c1 = (b1 ? c2[1] : c2[0]) + __shfl_xor(b1 ? c2[0] : c2[1], 2, 64);
    return c1 + __shfl_xor(c1, 1, 64);
}

__global__ void __launch_bounds__(256) k_qp_column(QrdmArgs a, const double *Fz, double *PB2) {
    const QrdmCtl *ctl = a.ctl;
    if (ctl->done || ctl->qp_stop) return;
    const int64_t j = ctl->ns;
    const int64_t k0 = ctl->qp_k0;
    const int b = ctl->qp_b;
    const int64_t jm = ctl->jmax;
    const int64_t r0 = (int64_t)blockIdx.x * QP_ROWS;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    __shared__ double sF[QP_NBMAX];
    __shared__ double red[4][2 + 2 * QP_NBMAX];
    __shared__ double stp[QP_NBMAX];  // V[j][bb], written by the thread that holds row j
    for (int bb = tid; bb < QP_NBMAX; bb += 256) {
        sF[bb] = bb < b ? Fz[(int64_t)bb * a.n + j] : 0.0;
        stp[bb] = 0.0;
    }
    __syncthreads();
    const int64_t r = r0 + tid;
    const bool live = (r < a.m) && (r >= j);
    // per row: normalize the pending reflector (column j-1), swap, update x_r
    if (r < a.m) {
        if (ctl->qp_pend) {
            const int64_t pc = j - 1;
            if (r > pc) a.A[pc * a.lda + r] *= 1.0 / ctl->qp_den;
            else if (r == pc) a.A[pc * a.lda + r] = ctl->qp_beta;
        }
        if (jm != j) {
            const double t1 = a.A[j * a.lda + r];
            a.A[j * a.lda + r] = a.A[jm * a.lda + r];
            a.A[jm * a.lda + r] = t1;
        }
    }
    const bool below = live && (r > j);
    const bool atj = live && (r == j);
    double x = 0.0;
    if (b <= QP_NB_REG) {
        // the row's entries of the block's reflectors, loaded once (all loads issued together)
        double vr[QP_NB_REG];
#pragma unroll
        for (int u = 0; u < QP_NB_REG; ++u) vr[u] = (live && u < b) ? a.A[(k0 + u) * a.lda + r] : 0.0;
        if (live) {
            x = a.A[j * a.lda + r];
#pragma unroll
            for (int u = 0; u < QP_NB_REG; ++u) x -= vr[u] * sF[u];
            a.A[j * a.lda + r] = x;
        }
        if (atj) {
#pragma unroll
            for (int u = 0; u < QP_NB_REG; ++u)
                if (u < b) stp[u] = vr[u];
        }
        double pv[QP_NB_REG];
#pragma unroll
        for (int u = 0; u < QP_NB_REG; ++u) pv[u] = below ? vr[u] * x : 0.0;
        const double d = qp_reduce_scatter32(pv, lane);
        if ((lane & 1) == 0 && (lane >> 1) < b) red[wv][2 + (lane >> 1)] = d;
    } else {
        if (live) {
            x = a.A[j * a.lda + r];
            for (int bb = 0; bb < b; ++bb) x -= a.A[(k0 + bb) * a.lda + r] * sF[bb];
            a.A[j * a.lda + r] = x;
        }
        for (int bb = 0; bb < b; ++bb) {
            const double vb = (below || atj) ? a.A[(k0 + bb) * a.lda + r] : 0.0;
            const double d = wave_sum(below ? vb * x : 0.0);
            if (lane == 0) red[wv][2 + bb] = d;
            if (atj) stp[bb] = vb;
        }
    }
    // [0] sum_{r>j} x^2, [1] x_j, [2+bb] sum_{r>j} v_bb[r] x_r, [2+b+bb] v_bb[j]
    const double s0 = wave_sum(below ? x * x : 0.0);
    const double s1 = wave_sum(atj ? x : 0.0);
    if (lane == 0) { red[wv][0] = s0; red[wv][1] = s1; }
    __syncthreads();
    const int nv = 2 + 2 * b;
    for (int e = tid; e < nv; e += 256) {
        const double v = e < 2 + b ? red[0][e] + red[1][e] + red[2][e] + red[3][e] : stp[e - 2 - b];
        PB2[(int64_t)blockIdx.x * (2 + 2 * QP_NBMAX) + e] = v;
    }
}

// -------------------------------------------------------------------- GEMV
__global__ void __launch_bounds__(256) k_qp_gemv(QrdmArgs a, double *Fz, const double *PB2, int32_t *flag) {
    QrdmCtl *ctl = a.ctl;
    if (ctl->done || ctl->qp_stop) return;
    const int64_t j = ctl->ns;
    const int b = ctl->qp_b;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    __shared__ double sv[2 + 2 * QP_NBMAX];
    __shared__ double s_scal[4];
    __shared__ double auxv[QP_NBMAX];
    const int nv = 2 + 2 * b;
    const int npart = (int)((a.m + QP_ROWS - 1) / QP_ROWS);
    // fixed-order reduction of the pivot-column partials (every workgroup); the
    // row slabs above row j hold no live row and contribute exact zeros, so the
    // sum starts at the slab of row j, with up to 32 loads in flight
    const int wfirst = (int)(j / QP_ROWS);
    for (int e = tid; e < nv; e += 256) {
        double acc = 0.0;
        for (int w0 = wfirst; w0 < npart; w0 += 32) {
            double v[32];
#pragma unroll
            for (int u = 0; u < 32; ++u)
                v[u] = (w0 + u < npart) ? PB2[(int64_t)(w0 + u) * (2 + 2 * QP_NBMAX) + e] : 0.0;
#pragma unroll
            for (int u = 0; u < 32; ++u) acc += v[u];
        }
        sv[e] = acc;
    }
    __syncthreads();
    if (tid == 0) {
        const double sp = sv[0], alpha = sv[1];
        const double nrm = sqrt(alpha * alpha + sp);
        double beta, ti, den;
        if (sp == 0.0) {
            ti = 0.0;
            beta = alpha;
            den = 1.0;
        } else {
            beta = (alpha >= 0.0) ? -nrm : nrm;
            ti = (beta - alpha) / beta;
            den = alpha - beta;
        }
        s_scal[0] = beta;
        s_scal[1] = ti;
        s_scal[2] = den;
        if (blockIdx.x == 0) {
            a.tau_house[j] = ti;
            ctl->qp_beta = beta;
            ctl->qp_den = den;
            ctl->l = 1;
        }
    }
    __syncthreads();
    const double ti = s_scal[1], den = s_scal[2];
    for (int bb = tid; bb < b; bb += 256) auxv[bb] = sv[2 + b + bb] + sv[2 + bb] / den;  // V^T v
    __syncthreads();
    const int64_t c = j + 1 + (int64_t)blockIdx.x * 4 + wv;
    if (c >= a.n) return;
    const double *xc = a.A + j * a.lda;
    const double *ac = a.A + c * a.lda;
    double dd[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};  // eight chains: sixteen loads in flight
    int64_t r = j + 1 + lane;
    for (; r + 448 < a.m; r += 512) {
        double xv[8], av[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            xv[u] = xc[r + 64 * u];
            av[u] = ac[r + 64 * u];
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) dd[u] += xv[u] * av[u];
    }
    for (int u = 0; r < a.m; r += 64, ++u) dd[u & 7] += xc[r] * ac[r];
    const double d = wave_sum(((dd[0] + dd[1]) + (dd[2] + dd[3])) + ((dd[4] + dd[5]) + (dd[6] + dd[7])));
    // the F row of column c, one earlier reflector per lane (b <= 64)
    const double fz = lane < b ? Fz[(int64_t)lane * a.n + c] : 0.0;
    const double corr = wave_sum(lane < b ? fz * auxv[lane] : 0.0);
    const double rcor = wave_sum(lane < b ? fz * sv[2 + b + lane] : 0.0);
    if (lane == 0) {
        // F[c, b] = tau v^T a_c - tau sum_{b'<b} F[c, b'] (V^T v)_{b'}
        double f = ac[j] + d / den;
        f = ti * f - ti * corr;
        Fz[(int64_t)b * a.n + c] = f;
        // pivot row of R: A[j, c] -= sum_{b' <= b} V[j, b'] F[c, b'], V[j, b] = 1
        const double rjc = ac[j] - f - rcor;
        a.A[c * a.lda + j] = rjc;
        // partial norm update with the new row (cancellation-safe rule)
        const double v1 = a.vn1[c];
        if (v1 != 0.0) {
            double q = 1.0 - (rjc * rjc) / (v1 * v1);
            if (q < 0.0) q = 0.0;
            const double r12 = v1 / a.vn2[c];
            const double q2 = q * (r12 * r12);
            if (q2 <= a.tol3z) {
                flag[c] = 1;
                atomicOr(&ctl->qp_flag, 1);
            } else {
                a.vn1[c] = v1 * sqrt(q);
            }
        }
    }
}

// ----------------------------------------------------------------- closing
// After the block's BLAS-3 update (k_gemm2 mode 1, which reads V from A and
// scales the pending reflector by 1/den): recompute the flagged partial norms
// (wave per column) and, when the factorization ends here, normalize the last
// reflector in place.
__global__ void __launch_bounds__(256) k_qp_close(QrdmArgs a, int32_t *flag, int nb) {
    QrdmCtl *ctl = a.ctl;
    if (ctl->done) return;
    int kb;
    int64_t last;
    const int64_t p = p_of(a);
    if (!qp_closes(ctl, p, nb, &kb, &last)) return;
    const int lane = threadIdx.x & 63;
    const int64_t c = last + 1 + (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (c < a.n && flag[c]) {
        const double *col = a.A + c * a.lda;
        double t = 0.0;
        for (int64_t r = last + 1 + lane; r < a.m; r += 64) t += col[r] * col[r];
        t = wave_sum(t);
        if (lane == 0) {
            const double v = sqrt(t);
            a.vn1[c] = v;
            a.vn2[c] = v;
            flag[c] = 0;
            atomicAdd((unsigned long long *)&ctl->nrecompute, 1ull);
        }
    }
    const bool final_step = ctl->qp_stop || last + 1 >= p;
    if (final_step && kb > 0) {
        const double rden = 1.0 / ctl->qp_den;
        const int64_t stride = (int64_t)gridDim.x * blockDim.x;
        for (int64_t r = last + 1 + (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < a.m; r += stride)
            a.A[last * a.lda + r] *= rden;
        if (blockIdx.x == 0 && threadIdx.x == 0) a.A[last * a.lda + last] = ctl->qp_beta;
    }
    if (final_step && blockIdx.x == 0 && threadIdx.x == 0 && ctl->qp_stop) ctl->done = 1;
}

hipError_t launch_qp3_step(QrdmArgs a, Qp3Bufs bf, int nb, int64_t t_bound, int64_t w_bound, hipStream_t s) {
    const unsigned g_rows = (unsigned)((a.m + QP_ROWS - 1) / QP_ROWS);
    const unsigned g_cols = (unsigned)((w_bound + 3) / 4 + 1);
    hipLaunchKernelGGL(k_qp_select, dim3(1), dim3(1024), 0, s, a, bf.Fz);
    hipLaunchKernelGGL(k_qp_column, dim3(g_rows), dim3(256), 0, s, a, bf.Fz, bf.PB2);
    hipLaunchKernelGGL(k_qp_gemv, dim3(g_cols), dim3(256), 0, s, a, bf.Fz, bf.PB2, bf.flag);
    hipError_t e = launch_gemm2_qp3(a, a.A, a.lda, bf.Fz, t_bound, w_bound, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_qp_close, dim3(g_cols), dim3(256), 0, s, a, bf.flag, nb);
    return hipGetLastError();
}
