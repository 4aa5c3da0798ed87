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

// Lane exchanges on the VALU (lane_xu / lane_xd of qrdm_internal.h: DPP row
// operations and the gfx950 lane swaps) instead of LDS permutes, whose latency
// the reductions of these latency-bound kernels would otherwise pay once per
// level: qp_x<K>(v) is v of lane ^ K for K = 32, 16, 8, 2, 1, and qp_x<7> that
// of lane ^ 7 (the mirror within each group of 8 lanes), which takes the place
// of lane ^ 4 in the trees below.  Every kernel of this file reduces through
// them, so all its paths sum in the same order.
template <int K>
__device__ __forceinline__ double qp_x(double v) {
    return lane_xd<K>(v);
}
template <int K>
__device__ __forceinline__ int qp_xi(int v) {
    return (int)lane_xu<K>((uint32_t)v);
}
// Sum over the 64 lanes, the same value in every lane.
__device__ __forceinline__ double qp_wave_sum(double v) {
    v += qp_x<32>(v);
    v += qp_x<16>(v);
    v += qp_x<8>(v);
    v += qp_x<7>(v);
    v += qp_x<2>(v);
    v += qp_x<1>(v);
    return v;
}

hipError_t launch_gemm2_qp3(QrdmArgs a, const double *Vw, int64_t ldv, const double *Fz, int64_t t_bound,
                            int64_t w_bound, hipStream_t s);

// ------------------------------------------------------------ init / select
__global__ void k_qp_init(QrdmArgs a, int nb) {
    QrdmCtl *c = a.ctl;
    if (a.gbar) {  // both counter sets of the block kernel (launches alternate between them)
        gbar_clear(a.gbar);
        gbar_clear(a.gbar + GBAR_GROUPS * GBAR_STRIDE);
    }
    if (c->nonfinite) c->done = 1;  // NaN/Inf in A: nothing is written
    if (!c->done) c->ns += c->l;  // finish the advance of a preceding QRDM step
    c->qp_k0 = c->ns;
    c->qp3_start = c->ns;
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

// Arg-max over the 64 lanes of (v, j) pairs in qp_better's order (a total
// order, so the result does not depend on the tree), in every lane.
template <int K>
__device__ __forceinline__ void qp_argmax_step(double &bv, int &bj) {
    const double ov = qp_x<K>(bv);
    const int oj = qp_xi<K>(bj);
    if (qp_better(ov, oj, bv, bj)) { bv = ov; bj = oj; }
}
__device__ __forceinline__ void qp_argmax_lanes(double &bv, int &bj) {
    qp_argmax_step<32>(bv, bj);
    qp_argmax_step<16>(bv, bj);
    qp_argmax_step<8>(bv, bj);
    qp_argmax_step<7>(bv, bj);
    qp_argmax_step<2>(bv, bj);
    qp_argmax_step<1>(bv, bj);
}

__global__ void __launch_bounds__(1024) k_qp_select(QrdmArgs a, double *Fz) {
    QrdmCtl *ctl = a.ctl;
    __shared__ double s_v[16];
    __shared__ int s_j[16];
    __shared__ int s_go, s_norm;
    if (ctl->done) return;
    const int tid = threadIdx.x;
    if (ctl->qp_stop) {  // the block closed by the stopping test is updated and normalized
        if (tid == 0) ctl->done = 1;
        return;
    }
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
    qp_argmax_lanes(bv, bj);
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

// Sum of 32 values over a wavefront by butterfly reduce-scatter (32 lane
// exchanges): on return lane L holds the sum of value (L >> 1) when L is even.
// At each level a lane keeps the half of its values selected by its own lane
// bit and adds the partner's copy of that half.
__device__ __forceinline__ double qp_reduce_scatter32(const double (&v)[QP_NB_REG], int lane) {
    double c16[16], c8[8], c4[4], c2[2];
    const bool b5 = lane & 32, b4 = lane & 16, b3 = lane & 8, b2 = lane & 4, b1 = lane & 2;
#pragma unroll
    for (int k = 0; k < 16; ++k) c16[k] = (b5 ? v[16 + k] : v[k]) + qp_x<32>(b5 ? v[k] : v[16 + k]);
#pragma unroll
    for (int k = 0; k < 8; ++k) c8[k] = (b4 ? c16[8 + k] : c16[k]) + qp_x<16>(b4 ? c16[k] : c16[8 + k]);
#pragma unroll
    for (int k = 0; k < 4; ++k) c4[k] = (b3 ? c8[4 + k] : c8[k]) + qp_x<8>(b3 ? c8[k] : c8[4 + k]);
#pragma unroll
    for (int k = 0; k < 2; ++k) c2[k] = (b2 ? c4[2 + k] : c4[k]) + qp_x<7>(b2 ? c4[k] : c4[2 + k]);
    const double c1 = (b1 ? c2[1] : c2[0]) + qp_x<2>(b1 ? c2[0] : c2[1]);
    return c1 + qp_x<1>(c1);
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
            const double d = qp_wave_sum(below ? vb * x : 0.0);
            if (lane == 0) red[wv][2 + bb] = d;
            if (atj) stp[bb] = vb;
        }
    }
    // [0] sum_{r>j} x^2, [1] x_j, [2+bb] sum_{r>j} v_bb[r] x_r, [2+b+bb] v_bb[j]
    const double s0 = qp_wave_sum(below ? x * x : 0.0);
    const double s1 = qp_wave_sum(atj ? x : 0.0);
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
    const double d = qp_wave_sum(((dd[0] + dd[1]) + (dd[2] + dd[3])) + ((dd[4] + dd[5]) + (dd[6] + dd[7])));
    // the F row of column c, one earlier reflector per lane (b <= 64)
    const double fz = lane < b ? Fz[(int64_t)lane * a.n + c] : 0.0;
    const double corr = qp_wave_sum(lane < b ? fz * auxv[lane] : 0.0);
    const double rcor = qp_wave_sum(lane < b ? fz * sv[2 + b + lane] : 0.0);
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
        t = qp_wave_sum(t);
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
    // after a stop, `done` is raised by the next k_qp_select / k_qp_run: raised
    // here, it could make a workgroup of this grid that starts late skip its rows
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

// ======================================================= persistent QP3 block
// The steps of one QP3 block (up to nb pivots) in one launch (every workgroup
// resident at once, see launch_resident), with
// the arithmetic of k_qp_select / k_qp_column / k_qp_gemv in the same order.
// Per step:
//   arg-max (from the partials of the previous step) and the stopping test ->
//   pivot-column pass over 256-row slabs -> grid barrier -> GEMV over the
//   trailing columns, which also updates the partial norms and publishes each
//   workgroup's arg-max of them -> grid barrier.
// Every workgroup carries the loop state in registers and takes the same
// decisions from the same exchanged values.  Row slab s belongs to workgroup
// s % G for the whole launch, so the rows of the block's reflectors are only
// ever written and read by one thread; the trailing columns are split evenly
// over the workgroups afresh at each step, and everything that crosses
// workgroups (the pivot column, F, the norms, the partials) goes through
// agent-scope atomic loads and stores.  The swap bookkeeping of a pivot
// (norms, perm, F rows) is done by the workgroup that owns the pivot's old
// column in the GEMV phase; the column pass reads the pivot's F row from that
// old column.  Each workgroup stages the pivot column below the diagonal in LDS
// (m <= QR_XS_MAX + 1).  The launch returns at the block end (or at the stop);
// the deferred update (k_gemm2 mode 1) and k_qp_close follow as separate
// launches.
#define QR_THREADS 256
#define QR_XS_MAX 16384  // rows of the staged pivot column (128 KB of LDS)
#define QR_CACHE_ROWS 2048  // rows of the column cache (the owner's reload is one batch of 8 per thread)
#define QR_LDS_DYN (144 * 1024)  // dynamic LDS of the block kernel (at most)

__device__ __forceinline__ double qr_ld(const double *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void qr_st(double *p, double v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ int32_t qr_ldi(const int32_t *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void qr_sti(int32_t *p, int32_t v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Workgroup arg-max of (v, j) pairs (largest value, lowest index on ties).
__device__ __forceinline__ void qr_wg_argmax(double &bv, int &bj, double *sv, int *sj) {
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    qp_argmax_lanes(bv, bj);
    if (lane == 0) { sv[wv] = bv; sj[wv] = bj; }
    __syncthreads();
    bv = sv[0];
    bj = sj[0];
    for (int w = 1; w < QR_THREADS / 64; ++w)
        if (qp_better(sv[w], sj[w], bv, bj)) { bv = sv[w]; bj = sj[w]; }
    __syncthreads();
}

// Arg-max over the G published partials (the unique largest value with the
// lowest index, whatever the order) and the OR of their recompute flags.
__device__ __forceinline__ void qr_reduce_partials(const double *amx, int G, double &uv, int64_t &uj, int &fl,
                                                   double *sv, int *sj, int *sf) {
    double bv = -1.0;
    int bj = 0x7fffffff, f = 0;
    for (int w = threadIdx.x; w < G; w += QR_THREADS) {
        const double v = qr_ld(amx + 4 * w), jd = qr_ld(amx + 4 * w + 1), fd = qr_ld(amx + 4 * w + 2);
        const int jj = (int)jd;
        if (qp_better(v, jj, bv, bj)) { bv = v; bj = jj; }
        f |= fd != 0.0;
    }
    f = __any(f);
    if ((threadIdx.x & 63) == 0) sf[threadIdx.x >> 6] = f;
    qr_wg_argmax(bv, bj, sv, sj);
    int ff = 0;
    for (int w = 0; w < QR_THREADS / 64; ++w) ff |= sf[w];
    uv = bv;
    uj = bj;
    fl = ff;
}

// One batch of the dots of columns ca and cb (cb < 0: none) with the staged
// pivot column, rows r0 .. r0+1535 (below m), added to the chains of
// k_qp_gemv: row j+1+64k goes to chain k mod 8 (1536 rows = 24 row-groups, a
// multiple of 8), each chain in increasing k.
#define QR_DOT_ROWS 24
__device__ __forceinline__ void qr_dot2_batch(const double *pa, const double *pb, bool two, int64_t m, int64_t j,
                                              int64_t r0, const double *xs, int lane, double (&ea)[8],
                                              double (&eb)[8]) {
    double av[QR_DOT_ROWS], bv[QR_DOT_ROWS];
#pragma unroll
    for (int u = 0; u < QR_DOT_ROWS; ++u) {
        const int64_t r = r0 + lane + 64 * u;
        av[u] = r < m ? qr_ld(pa + r) : 0.0;
        bv[u] = (two && r < m) ? qr_ld(pb + r) : 0.0;
    }
#pragma unroll
    for (int u = 0; u < QR_DOT_ROWS; ++u) {
        const int64_t r = r0 + lane + 64 * u;
        if (r < m) {
            const double x = xs[r - j - 1];
            ea[u & 7] += x * av[u];
            eb[u & 7] += x * bv[u];
        }
    }
}

extern __shared__ double qr_xs[];

__global__ void __launch_bounds__(QR_THREADS)
k_qp_run(QrdmArgs a, double *Fz, double *PB2, int32_t *flag, double *amx, int nb, int cq, int crows, int launch) {
    QrdmCtl *ctl = a.ctl;
    if (ctl->done) {
        if (a.snap && blockIdx.x == 0 && threadIdx.x == 0) qrdm_write_snapshot(ctl, a.snap);
        return;
    }
    const int G = gridDim.x, wg = blockIdx.x;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    // barrier counters: launches alternate between two sets, each clearing the
    // other for the launch after it (the one before has finished)
    uint32_t *gb = a.gbar + (launch & 1) * GBAR_GROUPS * GBAR_STRIDE;
    if (wg == 0 && tid == 0) gbar_clear(a.gbar + ((launch + 1) & 1) * GBAR_GROUPS * GBAR_STRIDE);
    const int64_t p = p_of(a);
    const int npart = (int)((a.m + QP_ROWS - 1) / QP_ROWS);
    if (npart > G) {  // one row slab per workgroup at most (the host's grid ensures it)
        if (wg == 0 && tid == 0) atomicOr(&ctl->error, 4);
        return;
    }
    __shared__ double s_v[QR_THREADS / 64];
    __shared__ int s_j[QR_THREADS / 64];
    __shared__ int s_f[QR_THREADS / 64];
    __shared__ double sF[QP_NBMAX];
    __shared__ double red[4][2 + 2 * QP_NBMAX];
    __shared__ double stp[QP_NBMAX];
    __shared__ double sv[2 + 2 * QP_NBMAX];
    __shared__ double auxv[QP_NBMAX];
    // loop state (identical in every workgroup)
    int64_t ns = ctl->ns, rank = ctl->rank, k0 = ctl->qp_k0, nblocks = ctl->nblocks, jm = ctl->jmax;
    int l = ctl->l, b = ctl->qp_b, pend = ctl->qp_pend, qstop = ctl->qp_stop, qflag = ctl->qp_flag, done = 0;
    double amax = ctl->amax, pbeta = ctl->qp_beta, pden = ctl->qp_den, umax = ctl->umax;
    uint32_t bar = 0;
    bool first = true;
    double uv = 0.0;
    int64_t uj = 0;
    // Column cache (cq > 0): this workgroup's trailing columns are fixed for
    // the launch, [cw0, cw1) from the block's first column j0, and held in LDS
    // from row j0 down with their F entries and partial norms; within a block
    // A changes only in the pivot rows (written through here) and by the pivot
    // swaps (the owner of the pivot's old column reloads it).  Otherwise the
    // columns are split afresh at each step and read from memory.
    const bool cached = cq > 0;
    const int64_t j0 = ns + (l == 1 ? 1 : 0);
    const int64_t q0 = a.n > j0 ? (a.n - j0 + G - 1) / G : 0;
    const int64_t cw0 = j0 + (int64_t)wg * q0;
    const int64_t cw1 = cw0 + q0 < a.n ? cw0 + q0 : a.n;
    const int64_t rows0 = a.m > j0 ? a.m - j0 : 0;
    double *xs = qr_xs;
    double *cc = qr_xs + crows;                    // [cq][crows], rows from j0
    double *fzc = cc + (int64_t)cq * crows;         // [cq][64]: F entries of the block
    double *n1c = fzc + (int64_t)cq * QP_NBMAX;     // [cq]
    double *n2c = n1c + cq;                         // [cq]
    // the row's entries of the block's reflectors (b <= 32) and its pivot-column
    // value of the previous step, kept in registers by the row's owner (one
    // row slab per workgroup at most, for the whole launch)
    double vr[QP_NB_REG];
#pragma unroll
    for (int u = 0; u < QP_NB_REG; ++u) vr[u] = 0.0;
    double xlast = 0.0;
    if (cached) {
        // the host sized the cache from bounds on j0 (cannot fail)
        if (q0 > cq || rows0 > crows || crows > QR_CACHE_ROWS) {
            if (wg == 0 && tid == 0) atomicOr(&ctl->error, 4);
            return;
        }
        const int64_t tot = (cw1 > cw0 ? cw1 - cw0 : 0) * rows0;
        for (int64_t i0 = 0; i0 < tot; i0 += 8 * QR_THREADS) {
            double v[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int64_t i = i0 + tid + QR_THREADS * u;
                v[u] = i < tot ? qr_ld(a.A + (cw0 + i / rows0) * a.lda + j0 + i % rows0) : 0.0;
            }
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int64_t i = i0 + tid + QR_THREADS * u;
                if (i < tot) cc[(i / rows0) * crows + i % rows0] = v[u];
            }
        }
        for (int64_t c = cw0 + tid; c < cw1; c += QR_THREADS) {
            n1c[c - cw0] = qr_ld(a.vn1 + c);
            n2c[c - cw0] = qr_ld(a.vn2 + c);
        }
        __syncthreads();
    }
    // ---- the previous launch's block (closed at its end, its deferred update
    // applied by k_gemm2 mode 1 since): what k_qp_close does after the per-step
    // kernels.  Flagged partial norms of this workgroup's columns are recomputed
    // from the updated rows below the block (one wavefront per column, the sum
    // order of k_qp_close); after the last block the last reflector is
    // normalized in place.
    const bool prev = (l == 1) || qstop;
    if (prev) {
        const int kbp = qstop ? b : b + 1;
        const int64_t last = k0 + kbp - 1;  // = j0 - 1
        for (int64_t c = cw0 + wv; c < cw1; c += 4) {
            if (!qr_ldi(flag + c)) continue;
            double t = 0.0;
            if (cached) {
                const double *col = cc + (c - cw0) * crows - j0;
                for (int64_t r = last + 1 + lane; r < a.m; r += 64) t += col[r] * col[r];
            } else {
                const double *col = a.A + c * a.lda;
                for (int64_t r = last + 1 + lane; r < a.m; r += 64) {
                    const double v = qr_ld(col + r);
                    t += v * v;
                }
            }
            t = qp_wave_sum(t);
            if (lane == 0) {
                const double v = sqrt(t);
                qr_st(a.vn1 + c, v);
                qr_st(a.vn2 + c, v);
                qr_sti(flag + c, 0);
                atomicAdd((unsigned long long *)&ctl->nrecompute, 1ull);
                if (cached) {
                    n1c[c - cw0] = v;
                    n2c[c - cw0] = v;
                }
            }
        }
        const bool final_step = qstop || last + 1 >= p;
        if (final_step && kbp > 0) {
            const double rden = 1.0 / pden;
            for (int64_t r = last + 1 + (int64_t)wg * QR_THREADS + tid; r < a.m; r += (int64_t)G * QR_THREADS)
                a.A[last * a.lda + r] *= rden;
            if (wg == 0 && tid == 0) a.A[last * a.lda + last] = pbeta;
        }
        if (final_step && qstop) done = 1;  // the stopping test closed this block: nothing follows
        __builtin_amdgcn_s_waitcnt(0);
        __syncthreads();
    }
    for (;;) {
        if (done) break;
        // ---- advance past the previous step's reflector (k_qp_select)
        if (l == 1) {
            const bool closes = qstop || (b + 1 == nb) || (ns + 1 == p) || qflag;
            const int kb = qstop ? b : b + 1;
            if (closes) {
                k0 = k0 + kb;
                b = 0;
                qflag = 0;
            } else {
                b += 1;
            }
            pend = 1;
            ns += 1;
            l = 0;
        }
        const int64_t j = ns;
        if (j >= p) {
            done = 1;
            if (rank < 0) rank = j;
            break;
        }
        if (first) {
            // arg-max over this workgroup's columns (from j = j0), then exchange
            double bv = -1.0;
            int bj = 0x7fffffff;
            for (int64_t c = (cw0 > j ? cw0 : j) + tid; c < cw1; c += QR_THREADS) {
                const double v = cached ? n1c[c - cw0] : qr_ld(a.vn1 + c);
                if (qp_better(v, (int)c, bv, bj)) { bv = v; bj = (int)c; }
            }
            qr_wg_argmax(bv, bj, s_v, s_j);
            if (tid == 0) {
                qr_st(amx + 4 * wg, bv);
                qr_st(amx + 4 * wg + 1, (double)bj);
                qr_st(amx + 4 * wg + 2, 0.0);
            }
            gbar_wait(gb, G, ++bar, &ctl->error);
            int fl;
            qr_reduce_partials(amx, G, uv, uj, fl, s_v, s_j, s_f);
            first = false;
        }
        // ---- stopping test (k_qp_select)
        if (nblocks == 0 && j == 0) amax = uv;
        int go = 1, snorm = 0;
        if (amax == 0.0) {
            rank = 0;
            done = 1;
            go = 0;
        } else if (rank < 0) {
            const double lhs = (a.stop_rule == 1) ? uv : sqrt((double)(a.n - j)) * uv;
            if (lhs <= a.eps1 * amax) {
                rank = j;
                if (a.stop_rule != 2) {
                    go = 0;
                    if (b > 0) {
                        qstop = 1;
                    } else {
                        done = 1;
                        snorm = pend;
                    }
                }
            }
        }
        if (!go) {
            if (snorm) {  // stopping right after a block end: normalize reflector j-1 in place
                const double rden = 1.0 / pden;
                for (int64_t r = j + (int64_t)wg * QR_THREADS + tid; r < a.m; r += (int64_t)G * QR_THREADS)
                    a.A[(j - 1) * a.lda + r] *= rden;
                if (wg == 0 && tid == 0) a.A[(j - 1) * a.lda + (j - 1)] = pbeta;
            }
            break;
        }
        jm = uj;
        umax = uv;
        nblocks += 1;
        // ---- pivot-column pass (k_qp_column), row slab wg (npart <= G):
        // every load of the slab first, then arithmetic, then every store
        if (wg < npart) {
            const int s = wg;
            const int64_t r = (int64_t)s * QP_ROWS + tid;
            const bool inm = r < a.m;
            const bool live = inm && (r >= j);
            const bool below = live && (r > j);
            const bool atj = live && (r == j);
            const int64_t pc = j - 1;
            const bool npend = pend && inm && r > pc;  // rows of the pending reflector scaled by 1/den
            const bool big = b > QP_NB_REG;
            // the pending reflector's row: this thread's pivot-column value of
            // the previous step, or from memory at the launch's first step
            double pv = npend ? (b > 0 ? xlast : a.A[pc * a.lda + r]) : 0.0;
            double t1 = 0.0, t2 = 0.0;
            if (inm && (jm != j || live)) t1 = qr_ld(a.A + j * a.lda + r);
            if (inm && jm != j) t2 = qr_ld(a.A + jm * a.lda + r);
            for (int bb = tid; bb < QP_NBMAX; bb += QR_THREADS) {
                sF[bb] = bb < b ? qr_ld(Fz + (int64_t)bb * a.n + jm) : 0.0;  // the pivot's F row, before its swap
                stp[bb] = 0.0;
            }
            __syncthreads();
            if (npend) pv *= 1.0 / pden;
            if (!big && pend) {
#pragma unroll
                for (int u = 0; u < QP_NB_REG; ++u)
                    if (u == b - 1 && live) vr[u] = pv;
            }
            double x = live ? (jm != j ? t2 : t1) : 0.0;
            if (!big) {
                if (live) {
#pragma unroll
                    for (int u = 0; u < QP_NB_REG; ++u) x -= vr[u] * sF[u];
                }
                if (atj) {
#pragma unroll
                    for (int u = 0; u < QP_NB_REG; ++u)
                        if (u < b) stp[u] = vr[u];
                }
                double pvv[QP_NB_REG];
#pragma unroll
                for (int u = 0; u < QP_NB_REG; ++u) pvv[u] = below ? vr[u] * x : 0.0;
                const double d = qp_reduce_scatter32(pvv, lane);
                if ((lane & 1) == 0 && (lane >> 1) < b) red[wv][2 + (lane >> 1)] = d;
            } else {
                // more than 32 reflectors: one wavefront sum per reflector (the
                // pending one, column k0 + b - 1, from the scaled register copy)
                if (live) {
                    for (int bb = 0; bb < b; ++bb)
                        x -= (bb == b - 1 ? pv : a.A[(k0 + bb) * a.lda + r]) * sF[bb];
                }
                for (int bb = 0; bb < b; ++bb) {
                    const double vb = (below || atj) ? (bb == b - 1 ? pv : a.A[(k0 + bb) * a.lda + r]) : 0.0;
                    const double d = qp_wave_sum(below ? vb * x : 0.0);
                    if (lane == 0) red[wv][2 + bb] = d;
                    if (atj) stp[bb] = vb;
                }
            }
            const double s0 = qp_wave_sum(below ? x * x : 0.0);
            const double s1 = qp_wave_sum(atj ? x : 0.0);
            if (lane == 0) { red[wv][0] = s0; red[wv][1] = s1; }
            __syncthreads();
            const int nv = 2 + 2 * b;
            for (int e = tid; e < nv; e += QR_THREADS) {
                const double v = e < 2 + b ? red[0][e] + red[1][e] + red[2][e] + red[3][e] : stp[e - 2 - b];
                qr_st(PB2 + (int64_t)s * (2 + 2 * QP_NBMAX) + e, v);
            }
            if (npend) a.A[pc * a.lda + r] = pv;
            else if (pend && inm && r == pc) a.A[pc * a.lda + r] = pbeta;
            if (inm && jm != j) {
                if (!live) qr_st(a.A + j * a.lda + r, t2);  // rows above j: plain swap
                qr_st(a.A + jm * a.lda + r, t1);
            }
            if (live) qr_st(a.A + j * a.lda + r, x);
            xlast = x;
            __syncthreads();
        }
        gbar_wait(gb, G, ++bar, &ctl->error);
        // ---- GEMV (k_qp_gemv): the pivot column below j into LDS, the
        // reflector scalars from the slab partials (every workgroup)
        const double *xc = a.A + j * a.lda;
        // with the column cache, the workgroup that owns the pivot's old
        // column jm takes over what column j held: its rows (swapped in by
        // the column pass), F entries and norms; its own go to column j
        const bool own_jm = cached && jm != j && jm >= cw0 && jm < cw1;
        const int64_t jmi = jm - cw0;
        double rv[8], rf = 0.0, rn1 = 0.0, rn2 = 0.0, of = 0.0, on1 = 0.0, on2 = 0.0;
        int32_t pj = 0, pm = 0;
        if (own_jm) {
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int64_t i = tid + QR_THREADS * u;
                rv[u] = i < rows0 ? qr_ld(a.A + jm * a.lda + j0 + i) : 0.0;
            }
            if (tid < b) {
                rf = qr_ld(Fz + (int64_t)tid * a.n + j);
                of = fzc[jmi * QP_NBMAX + tid];
            }
            if (tid == 0) {
                rn1 = qr_ld(a.vn1 + j);
                rn2 = qr_ld(a.vn2 + j);
                on1 = n1c[jmi];
                on2 = n2c[jmi];
                pj = qr_ldi(a.perm + j);
                pm = qr_ldi(a.perm + jm);
            }
        }
        {
            // the slab partials (rows from j's slab on: the slabs above hold no
            // live row) and the pivot column below j, loads issued together
            const int nv = 2 + 2 * b;
            const int wfirst = (int)(j / QP_ROWS);
            const int64_t nrow = a.m - j - 1;
            double pvv[32], xv[8];
            const bool mine = tid < nv;
#pragma unroll
            for (int u = 0; u < 32; ++u)
                pvv[u] = (mine && wfirst + u < npart) ? qr_ld(PB2 + (int64_t)(wfirst + u) * (2 + 2 * QP_NBMAX) + tid)
                                                      : 0.0;
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int64_t i = tid + QR_THREADS * u;
                xv[u] = i < nrow ? qr_ld(xc + j + 1 + i) : 0.0;
            }
            double acc = 0.0;
#pragma unroll
            for (int u = 0; u < 32; ++u) acc += pvv[u];
            for (int w0 = wfirst + 32; w0 < npart; w0 += 32) {  // more than 32 live slabs
#pragma unroll
                for (int u = 0; u < 32; ++u)
                    pvv[u] = (mine && w0 + u < npart) ? qr_ld(PB2 + (int64_t)(w0 + u) * (2 + 2 * QP_NBMAX) + tid)
                                                      : 0.0;
#pragma unroll
                for (int u = 0; u < 32; ++u) acc += pvv[u];
            }
            if (mine) sv[tid] = acc;
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int64_t i = tid + QR_THREADS * u;
                if (i < nrow) qr_xs[i] = xv[u];
            }
            for (int64_t i0 = 8 * QR_THREADS; i0 < nrow; i0 += 8 * QR_THREADS) {  // more than 2048 rows
#pragma unroll
                for (int u = 0; u < 8; ++u) {
                    const int64_t i = i0 + tid + QR_THREADS * u;
                    xv[u] = i < nrow ? qr_ld(xc + j + 1 + i) : 0.0;
                }
#pragma unroll
                for (int u = 0; u < 8; ++u) {
                    const int64_t i = i0 + tid + QR_THREADS * u;
                    if (i < nrow) qr_xs[i] = xv[u];
                }
            }
            if (own_jm) {
#pragma unroll
                for (int u = 0; u < 8; ++u) {
                    const int64_t i = tid + QR_THREADS * u;
                    if (i < rows0) cc[jmi * crows + i] = rv[u];
                }
                if (tid < b) {
                    fzc[jmi * QP_NBMAX + tid] = rf;
                    qr_st(Fz + (int64_t)tid * a.n + j, of);
                    qr_st(Fz + (int64_t)tid * a.n + jm, rf);
                }
                if (tid == 0) {
                    n1c[jmi] = rn1;
                    n2c[jmi] = rn2;
                    qr_st(a.vn1 + j, on1);
                    qr_st(a.vn2 + j, on2);
                    qr_st(a.vn2 + jm, rn2);  // vn1[jm] is written once, by the column loop
                    qr_sti(a.perm + j, pm);
                    qr_sti(a.perm + jm, pj);
                }
            }
            __syncthreads();
        }
        const double sp = sv[0], alpha = sv[1];
        double beta, ti, den;
        {
            const double nrm = sqrt(alpha * alpha + sp);
            if (sp == 0.0) {
                ti = 0.0;
                beta = alpha;
                den = 1.0;
            } else {
                beta = (alpha >= 0.0) ? -nrm : nrm;
                ti = (beta - alpha) / beta;
                den = alpha - beta;
            }
        }
        if (wg == 0 && tid == 0) a.tau_house[j] = ti;
        for (int bb = tid; bb < b; bb += QR_THREADS) auxv[bb] = sv[2 + b + bb] + sv[2 + bb] / den;  // V^T v
        __syncthreads();
        double bv = -1.0;
        int bj = 0x7fffffff, fany = 0;
        if (cached) {
            // this workgroup's columns after j, column cs + i to wavefront i % 4,
            // two at a time; every operand from LDS
            const int64_t cs = cw0 > j + 1 ? cw0 : j + 1;
            for (int64_t ca = cs + wv; ca < cw1; ca += 8) {
                const int64_t cb = ca + 4 < cw1 ? ca + 4 : -1;
                const bool two = cb >= 0;
                const double *pa = cc + (ca - cw0) * crows - j0, *pb = cc + ((two ? cb : ca) - cw0) * crows - j0;
                double ea[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0},
                       eb[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
                // row j+1+64k to chain k mod 8, each chain in increasing k
                int64_t r = j + 1 + lane;
                for (; r + 448 < a.m; r += 512) {
                    double xv[8], av[8], bw[8];
#pragma unroll
                    for (int u = 0; u < 8; ++u) {
                        xv[u] = xs[r - j - 1 + 64 * u];
                        av[u] = pa[r + 64 * u];
                        bw[u] = two ? pb[r + 64 * u] : 0.0;
                    }
#pragma unroll
                    for (int u = 0; u < 8; ++u) {
                        ea[u] += xv[u] * av[u];
                        eb[u] += xv[u] * bw[u];
                    }
                }
#pragma unroll
                for (int u = 0; u < 8; ++u) {
                    const int64_t rr = r + 64 * u;
                    if (rr < a.m) {
                        const double x = xs[rr - j - 1];
                        ea[u] += x * pa[rr];
                        eb[u] += x * (two ? pb[rr] : 0.0);
                    }
                }
                double dots[2];
                dots[0] = qp_wave_sum(((ea[0] + ea[1]) + (ea[2] + ea[3])) + ((ea[4] + ea[5]) + (ea[6] + ea[7])));
                dots[1] = qp_wave_sum(((eb[0] + eb[1]) + (eb[2] + eb[3])) + ((eb[4] + eb[5]) + (eb[6] + eb[7])));
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                    const int64_t c = h ? cb : ca;
                    if (c < 0) continue;
                    const int64_t ci = c - cw0;
                    const double fz = lane < b ? fzc[ci * QP_NBMAX + lane] : 0.0;
                    const double corr = qp_wave_sum(lane < b ? fz * auxv[lane] : 0.0);
                    const double rcor = qp_wave_sum(lane < b ? fz * sv[2 + b + lane] : 0.0);
                    if (lane == 0) {
                        const double acj = cc[ci * crows + (j - j0)];
                        double f = acj + dots[h] / den;
                        f = ti * f - ti * corr;
                        const double rjc = acj - f - rcor;
                        double v1 = n1c[ci];
                        int upd = 0, flg = 0;
                        if (v1 != 0.0) {
                            double qq = 1.0 - (rjc * rjc) / (v1 * v1);
                            if (qq < 0.0) qq = 0.0;
                            const double r12 = v1 / n2c[ci];
                            const double q2 = qq * (r12 * r12);
                            if (q2 <= a.tol3z) {
                                flg = 1;
                            } else {
                                v1 = v1 * sqrt(qq);
                                upd = 1;
                            }
                        }
                        fzc[ci * QP_NBMAX + b] = f;
                        cc[ci * crows + (j - j0)] = rjc;
                        qr_st(Fz + (int64_t)b * a.n + c, f);
                        qr_st(a.A + c * a.lda + j, rjc);
                        if (upd) n1c[ci] = v1;
                        if (upd || c == jm) qr_st(a.vn1 + c, v1);
                        if (flg) qr_sti(flag + c, 1);
                        fany |= flg;
                        if (qp_better(v1, (int)c, bv, bj)) { bv = v1; bj = (int)c; }
                    }
                }
            }
        } else {
        // this step's share of the trailing columns: a contiguous range per
        // workgroup, column c_lo + i to wavefront i % 4, two columns at a time
        const int64_t q = (a.n - j - 1 + G - 1) / G;
        const int64_t c_lo = j + 1 + (int64_t)wg * q;
        const int64_t c_hi = c_lo + q < a.n ? c_lo + q : a.n;
        for (int64_t ca = c_lo + wv; ca < c_hi; ca += 8) {
            const int64_t cb = ca + 4 < c_hi ? ca + 4 : -1;
            const bool two = cb >= 0;
            const int hs = (jm != j && ca == jm) ? 0 : ((jm != j && cb == jm) ? 1 : -1);  // holds the pivot's old column
            // loads: F rows, norms and row j of both columns (for the pivot's
            // old column, F and the norms of column j: their values after the
            // swap), the swap's other half, then the first batch of the dots
            double fz[2], acj[2] = {0.0, 0.0}, n1[2] = {0.0, 0.0}, n2[2] = {0.0, 0.0};
            double sw_f = 0.0, sw_n1 = 0.0, sw_n2 = 0.0;
            int32_t sw_p1 = 0, sw_p2 = 0;
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const int64_t c = h ? cb : ca;
                const int64_t cs = (h == hs) ? j : c;
                fz[h] = (lane < b && c >= 0) ? qr_ld(Fz + (int64_t)lane * a.n + cs) : 0.0;
                if (lane == 0 && c >= 0) {
                    acj[h] = qr_ld(a.A + c * a.lda + j);
                    n1[h] = qr_ld(a.vn1 + cs);
                    n2[h] = qr_ld(a.vn2 + cs);
                }
            }
            if (hs >= 0) {
                sw_f = lane < b ? qr_ld(Fz + (int64_t)lane * a.n + jm) : 0.0;
                if (lane == 0) {
                    sw_n1 = qr_ld(a.vn1 + jm);
                    sw_n2 = qr_ld(a.vn2 + jm);
                    sw_p1 = qr_ldi(a.perm + j);
                    sw_p2 = qr_ldi(a.perm + jm);
                }
            }
            const double *pa = a.A + ca * a.lda, *pb = a.A + (two ? cb : ca) * a.lda;
            double ea[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0}, eb[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
            for (int64_t r0 = j + 1; r0 < a.m; r0 += 64 * QR_DOT_ROWS)
                qr_dot2_batch(pa, pb, two, a.m, j, r0, qr_xs, lane, ea, eb);
            double dots[2];
            dots[0] = qp_wave_sum(((ea[0] + ea[1]) + (ea[2] + ea[3])) + ((ea[4] + ea[5]) + (ea[6] + ea[7])));
            dots[1] = qp_wave_sum(((eb[0] + eb[1]) + (eb[2] + eb[3])) + ((eb[4] + eb[5]) + (eb[6] + eb[7])));
            double fnew[2], rjc[2], v1n[2];
            int upd[2] = {0, 0}, flg[2] = {0, 0};
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const int64_t c = h ? cb : ca;
                const double corr = qp_wave_sum(lane < b ? fz[h] * auxv[lane] : 0.0);
                const double rcor = qp_wave_sum(lane < b ? fz[h] * sv[2 + b + lane] : 0.0);
                double f = acj[h] + dots[h] / den;
                f = ti * f - ti * corr;
                fnew[h] = f;
                rjc[h] = acj[h] - f - rcor;
                double v1 = n1[h];
                if (v1 != 0.0) {
                    double qq = 1.0 - (rjc[h] * rjc[h]) / (v1 * v1);
                    if (qq < 0.0) qq = 0.0;
                    const double r12 = v1 / n2[h];
                    const double q2 = qq * (r12 * r12);
                    if (q2 <= a.tol3z) {
                        flg[h] = 1;
                    } else {
                        v1 = v1 * sqrt(qq);
                        upd[h] = 1;
                    }
                }
                v1n[h] = v1;
                if (lane == 0 && c >= 0) {
                    fany |= flg[h];
                    if (qp_better(v1, (int)c, bv, bj)) { bv = v1; bj = (int)c; }
                }
            }
            // stores: the swap of the pivot's old column with column j, then
            // both columns' F entry, pivot row entry and norm
            if (hs >= 0) {
                if (lane < b) {
                    qr_st(Fz + (int64_t)lane * a.n + j, sw_f);
                    qr_st(Fz + (int64_t)lane * a.n + jm, fz[hs]);
                }
                if (lane == 0) {
                    qr_st(a.vn1 + j, sw_n1);
                    qr_st(a.vn2 + j, sw_n2);
                    qr_st(a.vn2 + jm, n2[hs]);
                    qr_sti(a.perm + j, sw_p2);
                    qr_sti(a.perm + jm, sw_p1);
                }
            }
            if (lane == 0) {
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                    const int64_t c = h ? cb : ca;
                    if (c < 0) continue;
                    qr_st(Fz + (int64_t)b * a.n + c, fnew[h]);
                    qr_st(a.A + c * a.lda + j, rjc[h]);
                    if (upd[h] || h == hs) qr_st(a.vn1 + c, v1n[h]);
                    if (flg[h]) qr_sti(flag + c, 1);
                }
            }
        }
        }
        // this workgroup's arg-max of the updated norms, and its recompute flag
        fany = __any(fany);
        if (lane == 0) s_f[wv] = fany;
        qr_wg_argmax(bv, bj, s_v, s_j);
        if (tid == 0) {
            int ff = 0;
            for (int w = 0; w < QR_THREADS / 64; ++w) ff |= s_f[w];
            qr_st(amx + 4 * wg, bv);
            qr_st(amx + 4 * wg + 1, (double)bj);
            qr_st(amx + 4 * wg + 2, (double)ff);
        }
        pbeta = beta;
        pden = den;
        l = 1;
        gbar_wait(gb, G, ++bar, &ctl->error);
        int fl;
        qr_reduce_partials(amx, G, uv, uj, fl, s_v, s_j, s_f);
        qflag = qflag || fl;
        if ((b + 1 == nb) || (j + 1 == p) || qflag) break;  // block end: the deferred update follows
    }
    // every workgroup has read the loop state before it is written back
    if (bar == 0) gbar_wait(gb, G, ++bar, &ctl->error);
    if (wg == 0 && tid == 0) {
        ctl->ns = ns;
        ctl->rank = rank;
        ctl->qp_k0 = k0;
        ctl->nblocks = nblocks;
        ctl->jmax = jm;
        ctl->l = l;
        ctl->qp_b = b;
        ctl->qp_pend = pend;
        ctl->qp_stop = qstop;
        ctl->qp_flag = qflag;
        ctl->amax = amax;
        ctl->qp_beta = pbeta;
        ctl->qp_den = pden;
        ctl->umax = umax;
        if (done) ctl->done = 1;
        if (a.snap) qrdm_write_snapshot(ctl, a.snap);
    }
}

// Dynamic LDS of the uncached mode: the pivot column below the diagonal.
static size_t qr_lds_bytes(int64_t m) {
    const int64_t rows = m > 1 ? m - 1 : 1;
    return sizeof(double) * (size_t)rows;
}

// Column cache of the next launch from bounds on its first column j0 >= n - w_bound:
// at most t_bound rows and ceil(w_bound / grid) columns per workgroup.  0 columns
// when the cache would not fit.
static void qr_cache_shape(int64_t t_bound, int64_t w_bound, int grid, int *cq, int *crows, size_t *bytes) {
    *cq = 0;
    *crows = 0;
    const int64_t rows = t_bound > 1 ? t_bound : 1;
    const int64_t q = (w_bound + grid - 1) / grid;
    const size_t need = sizeof(double) * (size_t)(rows + q * rows + q * QP_NBMAX + 2 * q);
    if (rows <= QR_CACHE_ROWS && q >= 1 && need <= QR_LDS_DYN) {
        *cq = (int)q;
        *crows = (int)rows;
        *bytes = need;
    }
}

// One QP3 block as a persistent launch, then the deferred update.  The grid
// comes from qp3_block_grid (at most one workgroup per compute unit); launch
// numbers the launches of one loop from 0 (it selects the barrier counters).
hipError_t launch_qp3_block(QrdmArgs a, Qp3Bufs bf, int nb, int64_t t_bound, int64_t w_bound, int grid,
                            int launch, hipStream_t s, hipEvent_t *ev) {
    if (grid < 1 || grid > QP_RUN_MAXWG || nb < 1 || nb > QP_NBMAX || a.m > QR_XS_MAX + 1) return hipErrorInvalidValue;
    int cq = 0, crows = 0;
    size_t lds = qr_lds_bytes(a.m);
    qr_cache_shape(t_bound, w_bound, grid, &cq, &crows, &lds);
    void *args[] = {&a, &bf.Fz, &bf.PB2, &bf.flag, &bf.amx, &nb, &cq, &crows, &launch};
    hipError_t e;
    if (ev && (e = hipEventRecord(ev[0], s)) != hipSuccess) return e;
    e = launch_resident((const void *)k_qp_run, dim3(grid), dim3(QR_THREADS), args, (unsigned)lds, s);
    if (e != hipSuccess) return e;
    if (ev && (e = hipEventRecord(ev[1], s)) != hipSuccess) return e;
    // the block end: the deferred update; the next launch recomputes flagged
    // norms and, after the last block, normalizes the last reflector
    return launch_gemm2_qp3(a, a.A, a.lda, bf.Fz, t_bound, w_bound, s);
}

// One workgroup per compute unit (all co-resident: the kernel needs one slot
// per CU with its LDS), capped at QP_RUN_MAXWG; 0 (the per-step kernels) when
// the device cannot hold that grid, the pivot column would not fit in LDS, or
// the row slabs would outnumber the workgroups.
int qp3_block_grid(int64_t m) {
    if (m > QR_XS_MAX + 1) return 0;
    const int64_t npart = (m + QP_ROWS - 1) / QP_ROWS;
    int dev = 0, ncu = 0, per_cu = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
    if (hipFuncSetAttribute((const void *)k_qp_run, hipFuncAttributeMaxDynamicSharedMemorySize, QR_LDS_DYN) !=
        hipSuccess)
        return 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void *)k_qp_run, QR_THREADS, QR_LDS_DYN) !=
            hipSuccess ||
        per_cu < 1)
        return 0;
    const int g = ncu < QP_RUN_MAXWG ? ncu : QP_RUN_MAXWG;
    if (g < 1 || npart > (int64_t)g) return 0;
    return g;
}

// ================================================= register-resident tail
// Column pivoting (Algorithm 2) on a trailing block small enough for the
// registers of the grid: every remaining step in one persistent launch, in the
// unblocked form (each reflector applied at once), with one grid barrier per
// step.
//
// Workgroup w holds the trailing columns c = w + G k (k < QT_QMAX, offsets from
// the first column j0 of the launch) from row j0 down, in registers: thread i
// holds rows j0 + i + QT_THREADS u (u < QT_RPT) of each.  Lane k of every
// wavefront holds column k's two partial norms, its current position and
// whether it is still active (the eight wavefronts keep identical copies).
// Per step j:
//   every workgroup reduces the G published (norm, position) partials to the
//   pivot (largest partial norm, lowest position on ties), reads the pivot's
//   column from its owner's published copy, and forms the reflector (LAPACK
//   larfg convention) from it, all in the same order, so every workgroup
//   holds the same bits; the owner writes the final column j (R above, beta,
//   v below) and tau_j;
//   the swap of positions j and the pivot's: each workgroup moves its slab of
//   the rows above j0 (R12 entries of both columns), workgroup 0 the
//   permutation, and the owner of the column at position j notes its new
//   position;
//   each workgroup applies H_j to its active columns: the dot products of a
//   thread's rows with v are summed over the wavefront for all columns at
//   once and over the eight wavefronts through LDS; lane k downdates column
//   k's partial norm by the cancellation-safe rule (recomputed from the rows
//   below j when the downdate lost too much); the workgroup publishes its
//   largest (norm, position) and, ahead of the barrier, a copy of that column
//   below row j: whichever workgroup wins, its column is already out for the
//   next step;
//   grid barrier.
// The stopping test is applied at every step as in the other QP3 kernels.  At
// the end the columns not pivoted (a stop) are written back to their final
// positions.  A launch that follows a QP3 block launch first finishes what the
// block left: the last reflector's normalization and the flagged norms.
#define QT_THREADS 512
#define QT_WAVES (QT_THREADS / 64)
#define QT_ROWS_MAX 2048                   // largest trailing block height it takes
#define QT_RPT (QT_ROWS_MAX / QT_THREADS)  // rows of each column per thread
#define QT_QMAX 8                          // columns per workgroup (at most)
#define QT_META 4                          // doubles per published partial: norm, position, column, unused
static_assert(QT_WAVES == 8 && QT_QMAX == 8, "the sums below take eight values over eight wavefronts");

// v of lane l (the same l in every lane).
__device__ __forceinline__ double qt_lane(double v, int l) {
    const uint64_t b = (uint64_t)__double_as_longlong(v);
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)b, l);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(b >> 32), l);
    return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}

// The eight per-wavefront partial sums p[0..7] in a fixed order.
__device__ __forceinline__ double qt_waves(const double *p) {
    return ((p[0] + p[1]) + (p[2] + p[3])) + ((p[4] + p[5]) + (p[6] + p[7]));
}

// Column k of the register array c (k the same in every lane), row register u:
// a tree of selects on the bits of k (an equality chain would be folded into an
// indexed access, which puts c in scratch memory).
__device__ __forceinline__ double qt_pick(const double (&c)[QT_QMAX][QT_RPT], int k, int u) {
    const bool b0 = k & 1, b1 = k & 2, b2 = k & 4;
    const double y01 = b0 ? c[1][u] : c[0][u], y23 = b0 ? c[3][u] : c[2][u];
    const double y45 = b0 ? c[5][u] : c[4][u], y67 = b0 ? c[7][u] : c[6][u];
    return b2 ? (b1 ? y67 : y45) : (b1 ? y23 : y01);
}

// A published partial of the tail kernel is two 64-bit words, each with the
// step's tag in its top 16 bits, so that a reader tells this step's words from
// older ones without a barrier: word 0 = tag | position | high half of the
// norm, word 1 = tag | column | low half of the norm (position and column
// 0xffff: none).  Tags start at 1; the launch clears its slots first.
__device__ __forceinline__ void qt_meta_put(uint64_t *me, uint32_t tag, double v, int pos, int col) {
    const uint64_t b = (uint64_t)__double_as_longlong(v), t = (uint64_t)(tag & 0xffff) << 48;
    __hip_atomic_store(me, t | ((uint64_t)(pos & 0xffff) << 32) | (b >> 32), __ATOMIC_RELAXED,
                       __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_store(me + 1, t | ((uint64_t)(col & 0xffff) << 32) | (b & 0xffffffffull), __ATOMIC_RELAXED,
                       __HIP_MEMORY_SCOPE_AGENT);
}

// x + y, where lanes with bit K of the lane index clear take x and the partner
// lane's x (lane ^ K), the others y and the partner's y (K = 32 or 16): the
// gfx950 lane swaps exchange the two halves of x and y in one step.
template <int K>
__device__ __forceinline__ double qt_swapsum(double x, double y) {
    const uint64_t xb = (uint64_t)__double_as_longlong(x), yb = (uint64_t)__double_as_longlong(y);
    const uint32_t xl = (uint32_t)xb, xh = (uint32_t)(xb >> 32), yl = (uint32_t)yb, yh = (uint32_t)(yb >> 32);
    uint32_t a0, a1, b0, b1;
    if constexpr (K == 32) {
        const auto lo = __builtin_amdgcn_permlane32_swap(xl, yl, false, false);
        const auto hi = __builtin_amdgcn_permlane32_swap(xh, yh, false, false);
        a0 = lo[0]; b0 = lo[1]; a1 = hi[0]; b1 = hi[1];
    } else {
        static_assert(K == 16, "lane swap");
        const auto lo = __builtin_amdgcn_permlane16_swap(xl, yl, false, false);
        const auto hi = __builtin_amdgcn_permlane16_swap(xh, yh, false, false);
        a0 = lo[0]; b0 = lo[1]; a1 = hi[0]; b1 = hi[1];
    }
    return __longlong_as_double((long long)(((uint64_t)a1 << 32) | a0)) +
           __longlong_as_double((long long)(((uint64_t)b1 << 32) | b0));
}

// Sums over the 64 lanes of e[0..7] at once: the exchanges with lane ^ 32,
// ^ 16 and ^ 8 each halve the values a lane carries (the lane with the bit
// clear keeps the lower half of its set), the rest sum within groups of eight
// lanes.  Lanes 8g .. 8g + 7 return the total of e[g].
__device__ __forceinline__ double qt_sum8(const double (&e)[QT_QMAX]) {
    const int lane = threadIdx.x & 63;
    const bool h8 = lane & 8;
    double f[4], g[2];
#pragma unroll
    for (int c = 0; c < 4; ++c) f[c] = qt_swapsum<32>(e[c], e[c + 4]);
#pragma unroll
    for (int c = 0; c < 2; ++c) g[c] = qt_swapsum<16>(f[c], f[c + 2]);
    double h = (h8 ? g[1] : g[0]) + qp_x<8>(h8 ? g[0] : g[1]);
    h += qp_x<7>(h);
    h += qp_x<2>(h);
    h += qp_x<1>(h);
    return h;
}

__global__ void __launch_bounds__(QT_THREADS) __attribute__((amdgpu_waves_per_eu(2, 2)))
k_qp_tail(QrdmArgs a, double *pub, int32_t *flag, int crows, int launch) {
    QrdmCtl *ctl = a.ctl;
    if (ctl->done) {
        if (a.snap && blockIdx.x == 0 && threadIdx.x == 0) qrdm_write_snapshot(ctl, a.snap);
        return;
    }
    const int G = gridDim.x, wg = blockIdx.x;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    uint32_t *gb = a.gbar + (launch & 1) * GBAR_GROUPS * GBAR_STRIDE;
    if (wg == 0 && tid == 0) gbar_clear(a.gbar + ((launch + 1) & 1) * GBAR_GROUPS * GBAR_STRIDE);
    const int64_t p = p_of(a);
    __shared__ double s_v[QT_WAVES];
    __shared__ int s_j[QT_WAVES];
    __shared__ int s_k[QT_WAVES];
    __shared__ double s_red[QT_WAVES];
    __shared__ double s_alpha;
    __shared__ double s_dp[QT_QMAX * QT_WAVES];  // per-wavefront sums of v^T c_k
    __shared__ double s_rp[QT_QMAX * QT_WAVES];  // per-wavefront sums of squares (recomputed norms)
    __shared__ double s_c0[QT_QMAX];      // row j of each column before H_j
    __shared__ int s_fail;                // a partial did not arrive within the spin limit
    // loop state (identical in every workgroup)
    int64_t ns = ctl->ns, rank = ctl->rank, nblocks = ctl->nblocks, jm = ctl->jmax;
    const int64_t k0 = ctl->qp_k0;
    const int l = ctl->l, b = ctl->qp_b, qstop = ctl->qp_stop;
    int pend = ctl->qp_pend, done = 0;
    double amax = ctl->amax, umax = ctl->umax;
    const double pbeta = ctl->qp_beta, pden = ctl->qp_den;
    uint32_t bar = 0;
    // ---- what a preceding QP3 block launch left (as k_qp_run's prologue): a
    // block closed at its last step (l = 1) or by the stopping test (qstop)
    if (l == 1 || qstop) {
        const int kbp = qstop ? b : b + 1;
        const int64_t last = k0 + kbp - 1;
        const bool final_step = qstop || last + 1 >= p;
        if (final_step && kbp > 0) {
            const double rden = 1.0 / pden;
            for (int64_t r = last + 1 + (int64_t)wg * QT_THREADS + tid; r < a.m; r += (int64_t)G * QT_THREADS)
                a.A[last * a.lda + r] *= rden;
            if (wg == 0 && tid == 0) a.A[last * a.lda + last] = pbeta;
            pend = 0;
        }
        if (final_step && qstop) done = 1;
    }
    if (l == 1) {  // the advance past the block's last reflector
        ns += 1;
        pend = pend || !(ns >= p);
    }
    if (!done && pend && ns < p) {  // normalize the pending reflector ns - 1
        const int64_t pc = ns - 1;
        const double rden = 1.0 / pden;
        for (int64_t r = ns + (int64_t)wg * QT_THREADS + tid; r < a.m; r += (int64_t)G * QT_THREADS)
            a.A[pc * a.lda + r] *= rden;
        if (wg == 0 && tid == 0) a.A[pc * a.lda + pc] = pbeta;
    }
    const int64_t j0 = ns;
    const int64_t t0 = a.m > j0 ? a.m - j0 : 0, w0 = a.n > j0 ? a.n - j0 : 0;
    const int q = wg < w0 ? (int)((w0 - wg + G - 1) / G) : 0;  // columns of this workgroup
    if ((w0 + G - 1) / G > QT_QMAX || t0 > crows || crows > QT_ROWS_MAX) {  // the host's bounds (cannot fail)
        if (wg == 0 && tid == 0) atomicOr(&ctl->error, 4);
        return;
    }
    uint64_t *meta = (uint64_t *)pub;             // [2][G][QT_META]: tagged partials
    double *pdat = pub + 2 * (size_t)G * QT_META; // [2][G][crows]
    if (tid < 2 * QT_META) {  // this workgroup's partial slots, both parities: no tag
        const int par = tid / QT_META;
        __hip_atomic_store(meta + ((size_t)par * G + wg) * QT_META + tid % QT_META, (uint64_t)0, __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
    }
    if (tid == 0) s_fail = 0;
    // ---- this workgroup's columns, and lane k's column state
    // (every load issued before any is used: clamped addresses, then the selects)
    double c[QT_QMAX][QT_RPT];
    if (t0 > 0 && w0 > 0) {
#pragma unroll
        for (int k = 0; k < QT_QMAX; ++k)
#pragma unroll
            for (int u = 0; u < QT_RPT; ++u) {
                const int64_t r = tid + QT_THREADS * u;
                const int64_t col = k < q ? j0 + wg + (int64_t)G * k : j0;
                c[k][u] = a.A[col * a.lda + j0 + (r < t0 ? r : 0)];
            }
#pragma unroll
        for (int k = 0; k < QT_QMAX; ++k)
#pragma unroll
            for (int u = 0; u < QT_RPT; ++u)
                if (!(k < q && tid + QT_THREADS * u < t0)) c[k][u] = 0.0;
    } else {
#pragma unroll
        for (int k = 0; k < QT_QMAX; ++k)
#pragma unroll
            for (int u = 0; u < QT_RPT; ++u) c[k][u] = 0.0;
    }
    const int kl = lane < QT_QMAX ? lane : 0;
    const int64_t cl = j0 + wg + (int64_t)G * kl;  // lane k's column
    bool actv = lane < q;
    double n1v = actv ? qr_ld(a.vn1 + cl) : 0.0, n2v = actv ? qr_ld(a.vn2 + cl) : 1.0;
    int posv = wg + G * kl;  // current position offset (from j0)
    int64_t nrec = 0;
    // partial norms recomputed from the rows rs .. t0 - 1 (offsets from j0) of
    // the columns in the mask nm, the same in every thread; lane k takes column k's
    auto recompute = [&](uint32_t nm, int64_t rs) {
        double e[QT_QMAX];
#pragma unroll
        for (int k = 0; k < QT_QMAX; ++k) {
            e[k] = 0.0;
            if (nm >> k & 1) {
#pragma unroll
                for (int u = 0; u < QT_RPT; ++u) {
                    const int64_t r = tid + QT_THREADS * u;
                    const double y = r >= rs ? c[k][u] : 0.0;
                    e[k] += y * y;
                }
            }
        }
        const double h = qt_sum8(e);
        if ((lane & 7) == 0) s_rp[(lane >> 3) * QT_WAVES + wv] = h;
        __syncthreads();
        if (lane < QT_QMAX && (nm >> kl & 1)) {
            const double v = sqrt(qt_waves(s_rp + QT_WAVES * kl));
            n1v = v;
            n2v = v;
            if (wv == 0) ++nrec;
        }
    };
    // flagged partial norms (a preceding block launch)
    {
        const bool f = actv && qr_ldi(flag + cl) != 0;
        const uint32_t nm = (uint32_t)__ballot(f);
        if (nm) {
            recompute(nm, 0);
            if (f && wv == 0) qr_sti(flag + cl, 0);
        }
    }
    // this workgroup's largest (norm, position) over its active columns, the
    // same in every thread
    auto local_best = [&](double &bv, int &bp, int &bk) {
        bv = actv ? n1v : -1.0;
        bp = actv ? posv : 0x7fffffff;
        qp_argmax_lanes(bv, bp);  // a total order: one lane holds the winner
        const unsigned long long hold = __ballot(actv && n1v == bv && posv == bp);
        bk = hold ? __ffsll((long long)hold) - 1 : -1;
    };
    // publishes rows rs .. t0 - 1 (offsets from j0) of the local best column
    // and then, once those stores are complete, the partial (norm, position,
    // column) with the step's tag, into parity slot par
    auto publish = [&](int par, int64_t rs, uint32_t tag, double bv, int bp, int bk) {
        if (bk >= 0) {
            double *dst = pdat + ((size_t)par * G + wg) * crows;
#pragma unroll
            for (int u = 0; u < QT_RPT; ++u) {
                const int64_t r = tid + QT_THREADS * u;
                const double y = qt_pick(c, bk, u);
                if (r >= rs && r < t0) qr_st(dst + (r - rs), y);
            }
        }
        __builtin_amdgcn_s_waitcnt(0);
        __syncthreads();
        if (tid == 0) qt_meta_put(meta + ((size_t)par * G + wg) * QT_META, tag, bv, bp, bk >= 0 ? wg + G * bk : -1);
    };
    // the cleared slots are seen by every workgroup before any partial is published
    gbar_wait(gb, G, ++bar, &ctl->error);
    {
        double bv;
        int bp, bk;
        local_best(bv, bp, bk);
        publish(0, 0, 1, bv, bp, bk);
    }
    // the slab of the rows above j0 whose R12 entries this workgroup swaps
    const int64_t ur = (j0 + G - 1) / G;
    const int64_t ur0 = (int64_t)wg * ur, ur1 = ur0 + ur < j0 ? ur0 + ur : j0;
    int64_t j = j0;
    for (int par = 0; !done; par ^= 1) {
        if (j >= p) {
            done = 1;
            if (rank < 0) rank = j;
            break;
        }
        // ---- the pivot: the G partials of this step, each read until it
        // carries this step's tag (s_v, s_j and s_k are written again only a
        // step later, after the barriers below)
        double uv = -1.0;
        int up = 0x7fffffff, uc = -1;
        {
            const uint32_t tag = (uint32_t)(j - j0 + 1);
            double bv = -1.0;
            int bp = 0x7fffffff, bc = -1;
            for (int w = tid; w < G; w += QT_THREADS) {
                const uint64_t *me = meta + ((size_t)par * G + w) * QT_META;
                uint64_t w0, w1;
                for (int spin = 0;; ++spin) {
                    w0 = __hip_atomic_load(me, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    w1 = __hip_atomic_load(me + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    if ((uint32_t)(w0 >> 48) == tag && (uint32_t)(w1 >> 48) == tag) break;
                    if (spin > GBAR_SPIN_LIMIT) {
                        atomicOr(&ctl->error, 2);
                        s_fail = 1;
                        w0 = w1 = 0xffffffffull << 32;  // no column
                        break;
                    }
                    __builtin_amdgcn_s_sleep(1);
                }
                const double v = __longlong_as_double((long long)(((w0 & 0xffffffffull) << 32) | (w1 & 0xffffffffull)));
                const int pd = (int)((w0 >> 32) & 0xffff), cd = (int)((w1 >> 32) & 0xffff);
                const int pv = pd == 0xffff ? 0x7fffffff : pd;
                if (qp_better(v, pv, bv, bp)) { bv = v; bp = pv; bc = cd == 0xffff ? -1 : cd; }
            }
            // (norm, position) is a total order: the winner's column rides along
            double vv = bv;
            int pp = bp;
            qp_argmax_lanes(vv, pp);
            if (lane == 0) { s_v[wv] = vv; s_j[wv] = pp; s_k[wv] = -1; }
            if (bp == pp && bv == vv && bc >= 0) s_k[wv] = bc;  // the one lane that holds it
            __syncthreads();
            uv = s_v[0];
            up = s_j[0];
            int wsel = 0;
            for (int w = 1; w < QT_WAVES; ++w)
                if (qp_better(s_v[w], s_j[w], uv, up)) { uv = s_v[w]; up = s_j[w]; wsel = w; }
            uc = s_k[wsel];
            if (s_fail) {  // the same in every thread
                done = 1;
                break;
            }
        }
        // ---- stopping test (as k_qp_select)
        if (nblocks == 0 && j == 0) amax = uv;
        if (amax == 0.0) {
            rank = 0;
            done = 1;
            break;
        }
        if (rank < 0) {
            const double lhs = (a.stop_rule == 1) ? uv : sqrt((double)(a.n - j)) * uv;
            if (lhs <= a.eps1 * amax) {
                rank = j;
                if (a.stop_rule != 2) {
                    done = 1;
                    break;
                }
            }
        }
        if (uc < 0) {  // no column left (cannot happen before j = p)
            if (wg == 0 && tid == 0) atomicOr(&ctl->error, 4);
            done = 1;
            break;
        }
        jm = j0 + up;
        umax = uv;
        nblocks += 1;
        const int owner = uc % G, kw = uc / G;
        const int rj = (int)(j - j0);  // row j: thread rj % QT_THREADS, register ru
        const int ru = rj / QT_THREADS, tr = (int)t0;
        // ---- the pivot column from its owner's copy (rows j .. m - 1), in the
        // row layout of the columns, zero above row j
        // (all loads issued before any is used)
        double x[QT_RPT];
        {
            const double *src = pdat + ((size_t)par * G + owner) * crows;
#pragma unroll
            for (int u = 0; u < QT_RPT; ++u) {
                const int r = tid + QT_THREADS * u;
                x[u] = qr_ld(src + (r >= rj && r < tr ? r - rj : 0));
            }
#pragma unroll
            for (int u = 0; u < QT_RPT; ++u) {
                const int r = tid + QT_THREADS * u;
                if (!(r >= rj && r < tr)) x[u] = 0.0;
            }
        }
        // ---- lane k: the pivot leaves the active set at position j; the
        // column at position j (when another) takes the pivot's old position
        if (wg == owner && lane == kw) {
            actv = false;
            posv = rj;
        } else if (jm != j && actv && posv == rj) {
            posv = up;
        }
        // ---- the reflector (larfg): alpha is row j, sp the sum of squares below it
        double sp = 0.0, xa = 0.0;
#pragma unroll
        for (int u = 0; u < QT_RPT; ++u) {
            if (tid + QT_THREADS * u == rj) xa = x[u];
            else sp += x[u] * x[u];
        }
        sp = qp_wave_sum(sp);
        if (lane == 0) s_red[wv] = sp;
        if (tid == (int)(rj % QT_THREADS)) s_alpha = xa;
        __syncthreads();
        sp = qt_waves(s_red);
        const double alpha = s_alpha;
        double beta, ti, den;
        if (sp == 0.0) {
            ti = 0.0;
            beta = alpha;
            den = 1.0;
        } else {
            const double nrm = sqrt(alpha * alpha + sp);
            beta = (alpha >= 0.0) ? -nrm : nrm;
            ti = (beta - alpha) / beta;
            den = alpha - beta;
        }
        const double rden = 1.0 / den;
#pragma unroll
        for (int u = 0; u < QT_RPT; ++u) x[u] = (tid + QT_THREADS * u == rj) ? 1.0 : x[u] * rden;
        // ---- the owner: the final column j (rows j0 .. m - 1) and tau_j
        if (wg == owner) {
            double *colj = a.A + j * a.lda + j0;
#pragma unroll
            for (int k = 0; k < QT_QMAX; ++k)
                if (k == kw) {
#pragma unroll
                    for (int u = 0; u < QT_RPT; ++u) {
                        const int r = tid + QT_THREADS * u;
                        if (r < tr) colj[r] = r < rj ? c[k][u] : (r == rj ? beta : x[u]);
                    }
                }
            if (tid == 0) a.tau_house[j] = ti;
        }
        // ---- H_j: v^T c_k over this thread's rows (v is zero above row j, so
        // every register takes part; the sums of columns no longer active are
        // not used), then over the wavefront (all columns at once) and the
        // workgroup
        {
            double e[QT_QMAX];
#pragma unroll
            for (int k = 0; k < QT_QMAX; ++k) {
                e[k] = x[0] * c[k][0];
#pragma unroll
                for (int u = 1; u < QT_RPT; ++u) e[k] += x[u] * c[k][u];
            }
            const double h = qt_sum8(e);
            if ((lane & 7) == 0) s_dp[(lane >> 3) * QT_WAVES + wv] = h;
            if (tid == (int)(rj % QT_THREADS)) {
                static_assert(QT_RPT == 4, "row register ru from its two bits");
                const bool b0 = ru & 1, b1 = ru & 2;
#pragma unroll
                for (int k = 0; k < QT_QMAX; ++k)
                    s_c0[k] = b1 ? (b0 ? c[k][3] : c[k][2]) : (b0 ? c[k][1] : c[k][0]);
            }
        }
        __syncthreads();
        // lane k: w_k = tau_j v^T c_k, and the partial norm downdate by the
        // cancellation-safe rule; row j after H_j is c0 - w_k (v_j = 1)
        double wl = 0.0;
        bool nd = false;
        if (actv) {
            wl = ti * qt_waves(s_dp + QT_WAVES * kl);
            const double rjc = s_c0[kl] - wl;
            if (n1v != 0.0) {
                double qq = 1.0 - (rjc * rjc) / (n1v * n1v);
                if (qq < 0.0) qq = 0.0;
                const double r12 = n1v / n2v;
                const double q2 = qq * (r12 * r12);
                if (q2 <= a.tol3z) nd = true;
                else n1v = n1v * sqrt(qq);
            }
        }
        // the update of this thread's rows (w_k = 0 for the columns no longer
        // active; rows above j, where v is zero, keep their value up to the
        // sign of a zero)
#pragma unroll
        for (int k = 0; k < QT_QMAX; ++k) {
            const double w = qt_lane(wl, k);
#pragma unroll
            for (int u = 0; u < QT_RPT; ++u) c[k][u] -= w * x[u];
        }
        const uint32_t nm = (uint32_t)__ballot(nd);
        if (nm) recompute(nm, rj + 1);  // from the rows below j
        // ---- publish for the step at j + 1
        {
            double bv;
            int bp, bk;
            local_best(bv, bp, bk);
            publish(par ^ 1, rj + 1, (uint32_t)(rj + 2), bv, bp, bk);
        }
        // ---- the swap of positions j and jm in this workgroup's slab of the
        // rows above j0, and in the permutation (workgroup 0), off the path of
        // the next step's pivot
        if (jm != j) {
            for (int64_t r = ur0 + tid; r < ur1; r += QT_THREADS) {
                const double x1 = a.A[j * a.lda + r], x2 = a.A[jm * a.lda + r];
                a.A[j * a.lda + r] = x2;
                a.A[jm * a.lda + r] = x1;
            }
            if (wg == 0 && tid == 0) {
                const int32_t p1 = a.perm[j], p2 = a.perm[jm];
                a.perm[j] = p2;
                a.perm[jm] = p1;
            }
        }
        j += 1;
    }
    // ---- the columns not pivoted (a stop): back to their final positions
    {
        const uint32_t am = (uint32_t)__ballot(actv);
#pragma unroll
        for (int k = 0; k < QT_QMAX; ++k)
            if (am >> k & 1) {
                const int pk = __builtin_amdgcn_readlane(posv, k);
                double *dst = a.A + (j0 + pk) * a.lda + j0;
#pragma unroll
                for (int u = 0; u < QT_RPT; ++u) {
                    const int64_t r = tid + QT_THREADS * u;
                    if (r < t0) dst[r] = c[k][u];
                }
            }
    }
    if (nrec) atomicAdd((unsigned long long *)&ctl->nrecompute, (unsigned long long)nrec);
    // every workgroup has read the loop state (the barrier after the first
    // publish) before workgroup 0 writes it back
    if (wg == 0 && tid == 0) {
        ctl->ns = j;
        ctl->rank = rank;
        ctl->qp_k0 = j;
        ctl->nblocks = nblocks;
        ctl->jmax = jm;
        ctl->l = 0;
        ctl->qp_b = 0;
        ctl->qp_pend = 0;
        ctl->qp_stop = 0;
        ctl->qp_flag = 0;
        ctl->amax = amax;
        ctl->umax = umax;
        ctl->done = 1;
        __builtin_amdgcn_s_waitcnt(0);
        if (a.snap) qrdm_write_snapshot(ctl, a.snap);
    }
}

// Shape of the tail kernel from bounds on its trailing block (t_bound rows,
// w_bound columns) and its grid: columns per workgroup and rows of a published
// column; false when the block does not fit the registers of the grid.  The
// kernel takes no dynamic LDS (bytes = 0).
bool qp3_tail_shape(int64_t t_bound, int64_t w_bound, int grid, int *cq, int *crows, size_t *bytes) {
    if (grid < 1) return false;
    const int64_t rows = t_bound > 1 ? t_bound : 1;
    const int64_t q = w_bound > 0 ? (w_bound + grid - 1) / grid : 1;
    if (rows > QT_ROWS_MAX || q > QT_QMAX) return false;
    *cq = (int)q;
    *crows = (int)rows;
    *bytes = 0;
    return true;
}

// Doubles of the published partials and column copies of the tail kernel for m rows.
size_t qp3_tail_pub_doubles(int64_t m) {
    const int64_t rows = m < QT_ROWS_MAX ? (m > 1 ? m : 1) : QT_ROWS_MAX;
    return 2 * (size_t)QP_RUN_MAXWG * QT_META + 2 * (size_t)QP_RUN_MAXWG * (size_t)rows;
}

// One workgroup per compute unit (at most QP_RUN_MAXWG), all co-resident; 0
// when the device cannot hold that grid.
int qp3_tail_grid() {
    int dev = 0, ncu = 0, per_cu = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void *)k_qp_tail, QT_THREADS, 0) !=
            hipSuccess ||
        per_cu < 1)
        return 0;
    return ncu < QP_RUN_MAXWG ? ncu : QP_RUN_MAXWG;
}

hipError_t launch_qp3_tail(QrdmArgs a, double *pub, int32_t *flag, int64_t t_bound, int64_t w_bound, int grid,
                           int launch, hipStream_t s, hipEvent_t *ev) {
    int cq = 0, crows = 0;
    size_t lds = 0;
    if (grid < 1 || grid > QP_RUN_MAXWG || !qp3_tail_shape(t_bound, w_bound, grid, &cq, &crows, &lds))
        return hipErrorInvalidValue;
    void *args[] = {&a, &pub, &flag, &crows, &launch};
    hipError_t e;
    if (ev && (e = hipEventRecord(ev[0], s)) != hipSuccess) return e;
    e = launch_resident((const void *)k_qp_tail, dim3(grid), dim3(QT_THREADS), args, 0, s);
    if (e != hipSuccess) return e;
    if (ev && (e = hipEventRecord(ev[1], s)) != hipSuccess) return e;
    return hipSuccess;
}
