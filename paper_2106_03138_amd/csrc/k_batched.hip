// Batched QRDM for many small matrices: one persistent kernel per size class,
// one workgroup per matrix at a time, matrices taken from an atomic queue in
// longest-processing-time order (the order array).  Every step of Algorithm 4
// (QRDM2) with Algorithm 1 (DM) runs inside the workgroup:
//
//   norms          initial column norms u_j (Algorithm 4, first step)
//   select         arg-max, the practical stopping criterion (Section 3.4), the
//                  scalar-pivoting switch (eq. column_norm_bound_DM), and the
//                  candidate list of eq. (def_candidate_set) cut to k_DM
//                  (eq. candidate_set_limited_by_kDM), ordered by (norm desc,
//                  position asc)
//   gram/greedy    Theta over the candidates (Algorithm 1) on FP64 MFMA, then
//                  the greedy acceptance |theta_ij| < delta in one wavefront
//   swaps          whole columns, tracking current positions
//   panel          Householder reflectors with the break of eq. (lenght_check)
//   compact WY     T from V^T V (forward, column-wise, Section 3.2)
//   trailing       A_tr -= V T^T V^T A_tr on FP64 MFMA, 16-column groups per
//                  wavefront, operands fed from registers (no LDS for Y or Z)
//   downdate       block partial-norm update with the DBu08 recompute rule
//
// The workgroup's state lives in LDS; the matrix stays in global memory (it is
// reused from L2/the Infinity Cache).  Limits: n <= QB_NMAX, k_DM <= QB_KM.
// The queue counters reset themselves when the last workgroup leaves, so a
// launch can be captured in a graph and replayed.
#include <float.h>

#include "qrdm_batched.h"

typedef double dbl4 __attribute__((ext_vector_type(4)));

#define QB_LD (QB_KM + 1)
#ifndef QB_SW
#define QB_SW 8  // columns of a register sub-panel
#endif

__device__ __forceinline__ dbl4 mfma64(double a, double b, dbl4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// every thread's global stores complete before the barrier
__device__ __forceinline__ void sync_global() {
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
}

template <int NT>
__device__ __forceinline__ double block_sum(double v, double *red) {
    constexpr int NW = NT / 64;
    v = wave_sum(v);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) red[w] = v;
    __syncthreads();
    double s = 0.0;
#pragma unroll
    for (int i = 0; i < NW; ++i) s += red[i];
    return s;
}

__device__ __forceinline__ bool qb_beats(double va, int ja, double vb, int jb) {
    return va > vb || (va == vb && ja < jb);
}

struct QbShared {
    double G[QB_KM * QB_LD];  // Gram of the candidates; later V^T V (lower) and T (upper)
    double vn1[QB_NMAX], vn2[QB_NMAX];
    double red[16];
    double rv[16];
    int rj[16];
    double red16[16 * 16];
    double prow[32], fin[32];  // pivot row and reduced sums of the register panel (two buffers)
    int L[QB_KM];
    int J[QB_KM];
    int swp[2 * QB_KM];
    int swround[QB_KM];
    // scalars of the current step
    double umax, amax, eps_s, beta, tau_i, den;
    int64_t rank;
    int ns, l, ks, nL, nsw, nround, go, fb, idx, ncand, nstep, nbreak, nfb;
    int redo, dflt, okv;  // checked form: factor the same matrix again with the plan's parameters
    int64_t t0;
};

// Gram G[i][j] = sum_r X_i[r] X_j[r] over r < t for i, j < nc, X given by col(r, i).
// One 16x16 output tile per wavefront at a time, K in steps of 4 rows.
template <int NT, class F>
__device__ __forceinline__ void qb_gram(const F &col, int nc, int t, double *G) {
    constexpr int NW = NT / 64;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int nt = (nc + 15) >> 4;
    const int ntile = nt * (nt + 1) / 2;
    const int i = lane & 15, kk = lane >> 4;
    for (int tile = w; tile < ntile; tile += NW) {
        int bi = 0, rem = tile;
        while (rem >= nt - bi) { rem -= nt - bi; ++bi; }
        const int bj = bi + rem;
        const int ci = 16 * bi + i, cj = 16 * bj + i;
        dbl4 acc = {0.0, 0.0, 0.0, 0.0};
        for (int k0 = 0; k0 < t; k0 += 16) {
            double a[4], b[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int r = k0 + 4 * u + kk;
                a[u] = (ci < nc && r < t) ? col(r, ci) : 0.0;
                b[u] = (cj < nc && r < t) ? col(r, cj) : 0.0;
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) acc = mfma64(a[u], b[u], acc);
        }
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int row = 16 * bi + 4 * v + kk, cc = 16 * bj + i;
            // a diagonal tile holds both (row, cc) and (cc, row): each entry is
            // stored once, by the lane with row <= cc
            if (row < nc && cc < nc && row <= cc) {
                G[row * QB_LD + cc] = acc[v];
                if (row < cc) G[cc * QB_LD + row] = acc[v];
            }
        }
    }
}

// Trailing update of columns [c0, n) over rows [ns, m) with the l reflectors of
// the block: A -= V (T^T (V^T A)).  Each wavefront owns WC column tiles of 16.
template <int NT, int WC>
__device__ __forceinline__ void qb_trailing(double *A, int lda, int m, int n, int ns, int l, int c0, const double *G) {
    constexpr int NW = NT / 64;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int i = lane & 15, kk = lane >> 4;
    const int t = m - ns;
    const int lt = (l + 15) >> 4;  // reflector tiles (<= 4)
    double *Ab = A + ns;            // row 0 of the block
    auto vval = [&](int r, int a) -> double {  // V[r][a], unit lower trapezoidal
        if (a >= l || r >= t) return 0.0;
        if (r > a) return Ab[(int64_t)(ns + a) * lda + r];
        return r == a ? 1.0 : 0.0;
    };
    const int ncols = n - c0;
    const int ngroups = (ncols + 16 * WC - 1) / (16 * WC);
    for (int g = w; g < ngroups; g += NW) {
        const int cb = c0 + g * 16 * WC;
        // Y = V^T A_chunk: tiles [yt][wc], D[4v + kk][i] = Y[16 yt + 4v + kk][col i]
        dbl4 y[4][WC];
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int c = 0; c < WC; ++c) y[a][c] = dbl4{0.0, 0.0, 0.0, 0.0};
        int colj[WC];
        bool cok[WC];
#pragma unroll
        for (int c = 0; c < WC; ++c) {
            colj[c] = cb + 16 * c + i;
            cok[c] = colj[c] < n;
        }
        for (int k0 = 0; k0 < t; k0 += 4) {
            const int r = k0 + kk;
            double bv[WC];
#pragma unroll
            for (int c = 0; c < WC; ++c) bv[c] = (cok[c] && r < t) ? Ab[(int64_t)colj[c] * lda + r] : 0.0;
#pragma unroll
            for (int a = 0; a < 4; ++a) {
                if (a < lt) {
                    const double av = vval(r, 16 * a + i);
#pragma unroll
                    for (int c = 0; c < WC; ++c) y[a][c] = mfma64(av, bv[c], y[a][c]);
                }
            }
        }
        // Z = T^T Y: Z[16 zt + i'][j] = sum_b T[b][16 zt + i'] Y[b][j], T upper (b <= a)
        dbl4 z[4][WC];
#pragma unroll
        for (int zt = 0; zt < 4; ++zt) {
#pragma unroll
            for (int c = 0; c < WC; ++c) z[zt][c] = dbl4{0.0, 0.0, 0.0, 0.0};
            if (zt < lt) {
#pragma unroll
                for (int yt = 0; yt < 4; ++yt) {
                    if (yt <= zt) {
#pragma unroll
                        for (int v = 0; v < 4; ++v) {
                            const int b = 16 * yt + 4 * v + kk, a = 16 * zt + i;
                            const double tv = (b <= a && a < l && b < l) ? G[b * QB_LD + a] : 0.0;
#pragma unroll
                            for (int c = 0; c < WC; ++c) z[zt][c] = mfma64(tv, y[yt][c][v], z[zt][c]);
                        }
                    }
                }
            }
        }
        // A_chunk -= V Z, one 16-row tile at a time, accumulator initialized from A
        for (int rt = 0; rt * 16 < t; ++rt) {
            dbl4 acc[WC];
#pragma unroll
            for (int c = 0; c < WC; ++c)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int r = 16 * rt + 4 * v + kk;
                    acc[c][v] = (cok[c] && r < t) ? Ab[(int64_t)colj[c] * lda + r] : 0.0;
                }
#pragma unroll
            for (int zt = 0; zt < 4; ++zt) {
                if (zt < lt) {
#pragma unroll
                    for (int v = 0; v < 4; ++v) {
                        const double av = -vval(16 * rt + i, 16 * zt + 4 * v + kk);
#pragma unroll
                        for (int c = 0; c < WC; ++c) acc[c] = mfma64(av, z[zt][c][v], acc[c]);
                    }
                }
            }
#pragma unroll
            for (int c = 0; c < WC; ++c)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int r = 16 * rt + 4 * v + kk;
                    if (cok[c] && r < t) Ab[(int64_t)colj[c] * lda + r] = acc[c][v];
                }
        }
    }
}

// T (forward, column-wise, Section 3.2) of the l reflectors stored in columns
// [c0, c0 + l) from row c0 down, into the upper triangle of G: first V^T V on
// MFMA into G, then T[a][i] = -tau_i sum_{b=a}^{i-1} T[a][b] (v_b^T v_i); row a
// of T is private to thread a (v^T v is read from the lower triangle).
template <int NT>
__device__ __forceinline__ void qb_build_T(const double *A, int lda, int m, int c0, int l, const double *tau_h, double *G) {
    const int tid = threadIdx.x;
    if (l > 1) {
        const double *Ab = A + c0;
        auto vcol = [&](int r, int a) -> double {
            if (r > a) return Ab[(int64_t)(c0 + a) * lda + r];
            return r == a ? 1.0 : 0.0;
        };
        qb_gram<NT>(vcol, l, m - c0, G);
        __syncthreads();
        if (tid < l) {
            const int a = tid;
            G[a * QB_LD + a] = tau_h[c0 + a];
            for (int i2 = a + 1; i2 < l; ++i2) {
                double s = 0.0;
                for (int b = a; b < i2; ++b) s += G[a * QB_LD + b] * G[i2 * QB_LD + b];
                G[a * QB_LD + i2] = -tau_h[c0 + i2] * s;
            }
        }
    } else if (l == 1 && tid == 0) {
        G[0] = tau_h[c0];
    }
    __syncthreads();
}

// Sum of SW values (SW = 8 or 16) over the workgroup: a butterfly
// reduce-scatter inside each wavefront (SW + 2 shuffles for 16, SW + 2 for 8),
// then the wavefront partials in LDS.  fin[0..SW) holds the sums for every
// thread on return.
template <int NT, int SW>
__device__ __forceinline__ void qb_reduce(const double (&v)[SW], double *red, double *fin) {
    constexpr int NW = NT / 64;
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    double cur[SW];
#pragma unroll
    for (int k = 0; k < SW; ++k) cur[k] = v[k];
    int idx = 0;
    int width = SW;
#pragma unroll
    for (int o = 32; o >= 64 / SW; o >>= 1) {  // halve the values kept per lane
        const bool hi = lane & o;
        const int h = width >> 1;
#pragma unroll
        for (int k = 0; k < SW / 2; ++k) {
            if (k < h) {
                const double mine = hi ? cur[h + k] : cur[k], oth = hi ? cur[k] : cur[h + k];
                cur[k] = mine + __shfl_xor(oth, o, 64);
            }
        }
        idx = 2 * idx + (hi ? 1 : 0);
        width = h;
    }
    double u1 = cur[0];
#pragma unroll
    for (int o = 32 / SW; o > 0; o >>= 1) u1 += __shfl_xor(u1, o, 64);
    if ((lane & (64 / SW - 1)) == 0) red[w * SW + idx] = u1;
    __syncthreads();
    if (tid < SW) {
        double s = 0.0;
#pragma unroll
        for (int i = 0; i < NW; ++i) s += red[i * SW + tid];
        fin[tid] = s;
    }
    __syncthreads();
}

// Householder panel with break (Algorithm 4, eq. lenght_check) for panel rows
// [ns, m) held in registers, RPT rows per thread, in sub-panels of SW columns.
// Each column takes one reduction of SW values (||x_below||^2 and x_below^T a_j
// for the sub-panel's later columns); the pivot row is published in LDS.  After
// a sub-panel its reflectors update the panel's later columns through a small
// compact-WY product.  Returns l, the reflectors kept.
template <int NT, int RPT, int SW>
__device__ __forceinline__ int qb_panel_regs(double *A, int lda, int m, int ns, int ks, double eps_s, double *tau_h,
                             QbShared &S) {
    const int tid = threadIdx.x;
    const int t = m - ns;
    int l = ks;
    for (int s0 = 0; s0 < ks; s0 += SW) {
        const int nsub = ks - s0 < SW ? ks - s0 : SW;
        double a[RPT][SW];
#pragma unroll
        for (int q = 0; q < RPT; ++q) {
            const int r = tid + q * NT;
#pragma unroll
            for (int jj = 0; jj < SW; ++jj)
                a[q][jj] = (r < t && jj < nsub) ? A[(int64_t)(ns + s0 + jj) * lda + ns + r] : 0.0;
        }
        int made = nsub;
        bool brk = false;
#pragma unroll
        for (int ii = 0; ii < SW; ++ii) {
            if (ii >= nsub || brk) continue;  // uniform; keeps the loop free of exits so it unrolls
            const int pr = s0 + ii;  // pivot row (relative to ns) = panel column
            double *prow = S.prow + (ii & 1) * 16;
            double *fin = S.fin + (ii & 1) * 16;
            double v[SW];
#pragma unroll
            for (int jj = 0; jj < SW; ++jj) v[jj] = 0.0;
#pragma unroll
            for (int q = 0; q < RPT; ++q) {
                const int r = tid + q * NT;
                if (r > pr && r < t) {
                    v[0] += a[q][ii] * a[q][ii];
#pragma unroll
                    for (int jj = ii + 1; jj < SW; ++jj) v[jj] += a[q][ii] * a[q][jj];
                }
                if (r == pr) {
#pragma unroll
                    for (int jj = 0; jj < SW; ++jj) prow[jj] = a[q][jj];
                }
            }
            qb_reduce<NT, SW>(v, S.red16, fin);
            const double sp = fin[0], alpha = prow[ii];
            const double nrm = sqrt(alpha * alpha + sp);
            if (pr >= 1 && nrm < eps_s) {  // nearly dependent column: end the block here
                l = pr;
                made = ii;
                brk = true;
                continue;
            }
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
            double wj[SW];
#pragma unroll
            for (int jj = ii + 1; jj < SW; ++jj) wj[jj] = ti * (prow[jj] + fin[jj] / den);
#pragma unroll
            for (int q = 0; q < RPT; ++q) {
                const int r = tid + q * NT;
                if (r > pr && r < t) {
                    const double vr = a[q][ii] / den;
                    a[q][ii] = vr;
#pragma unroll
                    for (int jj = ii + 1; jj < SW; ++jj) a[q][jj] -= wj[jj] * vr;
                } else if (r == pr) {
                    a[q][ii] = beta;
#pragma unroll
                    for (int jj = ii + 1; jj < SW; ++jj) a[q][jj] -= wj[jj];
                }
            }
            if (tid == 0) tau_h[ns + pr] = ti;
        }
        // write the sub-panel back (columns past a break are updated by the kept reflectors)
#pragma unroll
        for (int q = 0; q < RPT; ++q) {
            const int r = tid + q * NT;
            if (r < t) {
#pragma unroll
                for (int jj = 0; jj < SW; ++jj)
                    if (jj < nsub) A[(int64_t)(ns + s0 + jj) * lda + ns + r] = a[q][jj];
            }
        }
        sync_global();
        const int rest = s0 + nsub;
        if (made > 0 && rest < ks) {
            // the later panel columns take this sub-panel's reflectors
            qb_build_T<NT>(A, lda, m, ns + s0, made, tau_h, S.G);
            qb_trailing<NT, 1>(A, lda, m, ns + ks, ns + s0, made, ns + rest, S.G);
            sync_global();
        }
        if (brk) break;
    }
    return l;
}

// The same panel for slabs taller than the registers hold: columns read from
// global memory each step (a group of threads per later panel column).
template <int NT>
__device__ __forceinline__ int qb_panel_global(double *A, int lda, int m, int ns, int ks, double eps_s, double *tau_h,
                               QbShared &S) {
    const int tid = threadIdx.x;
    int l = ks;
    for (int i2 = 0; i2 < ks; ++i2) {
        const int c = ns + i2;
        double *xc = A + (int64_t)c * lda;
        // alpha is read before the reduction's barriers: thread 0 overwrites it
        // with beta further down
        const double alpha = xc[c];
        double part = 0.0;
        for (int r = c + 1 + tid; r < m; r += NT) part += xc[r] * xc[r];
        const double sp = block_sum<NT>(part, S.red);
        const double nrm = sqrt(alpha * alpha + sp);
        if (i2 >= 1 && nrm < eps_s) {
            l = i2;
            break;
        }
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
        for (int r = c + 1 + tid; r < m; r += NT) xc[r] = xc[r] / den;
        if (tid == 0) {
            xc[c] = beta;
            tau_h[c] = ti;
        }
        sync_global();
        const int nj = ks - 1 - i2;
        if (nj > 0) {
            int g = 64;
            while (g > 1 && g * nj > NT) g >>= 1;
            const int gid = tid / g, lig = tid % g;
            const bool act = gid < nj;
            double d = 0.0;
            double *yc = A + (int64_t)(c + 1 + (act ? gid : 0)) * lda;
            if (act) {
                for (int r = c + lig; r < m; r += g) d += (r == c ? 1.0 : xc[r]) * yc[r];
            }
            for (int o = g >> 1; o > 0; o >>= 1) d += __shfl_xor(d, o, 64);
            if (act) {
                const double wj = ti * d;
                for (int r = c + lig; r < m; r += g) yc[r] -= wj * (r == c ? 1.0 : xc[r]);
            }
        }
        sync_global();
    }
    return l;
}

template <int NT, int WC, int PANEL>
__global__ void __launch_bounds__(NT) k_qrdm_batched(QbArgs q) {
    constexpr int NW = NT / 64;
    __shared__ QbShared S;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const double eps_w = DBL_EPSILON;
    const double tol3z = sqrt(eps_w);

    if (tid == 0) S.redo = 0;
    for (;;) {
        if (tid == 0) {
            if (S.redo) {  // the matrix that failed the check, again with the plan's parameters
                S.redo = 0;
                S.dflt = 1;
            } else {
                S.idx = (int)atomicAdd(&q.counters[0], 1u);
                S.dflt = 0;
            }
        }
        __syncthreads();
        const int qi = S.idx;
        const bool dflt = S.dflt != 0;
        if (qi >= q.count) break;
        const int mi = q.order[qi];
        double *A = q.A[mi];
        const int m = q.m[mi], n = q.n[mi], lda = q.lda[mi];
        double *tau_h = q.tau_house[mi];
        int32_t *perm = q.perm[mi];
        double tau = q.tau, delta = q.delta;
        int kmax = q.kmax;
        if (q.pm && !dflt) {
            tau = q.pm[mi].tau;
            delta = q.pm[mi].delta;
            kmax = q.pm[mi].kmax;
            if (kmax == 0) {  // this matrix is left as it is (the same in every thread)
                __syncthreads();  // every thread has read S.idx before thread 0 takes the next
                continue;
            }
        }
        kmax = kmax < 1 ? 1 : (kmax > QB_KM ? QB_KM : kmax);  // the per-block arrays hold QB_KM
        const int p = m < n ? m : n;
        const double eps1 = (q.eps1_scale > 0.0 ? q.eps1_scale : (double)n) * eps_w;
        const double fbeps = (double)n * eps_w;

        // ---------------------------------------------------------- norms
        for (int c = wv; c < n; c += NW) {
            double s = 0.0;
            for (int r = lane; r < m; r += 64) {
                const double x = A[(int64_t)c * lda + r];
                s += x * x;
            }
            s = wave_sum(s);
            if (lane == 0) {
                const double v = sqrt(s);
                S.vn1[c] = v;
                S.vn2[c] = v;
            }
        }
        __syncthreads();
        double am = 0.0;
        bool finite = true;
        for (int c = tid; c < n; c += NT) {
            const double v = S.vn1[c];
            finite = finite && isfinite(v);
            am = v > am ? v : am;
        }
        // max and finiteness through the same reduction slots
        {
            double fm = finite ? 0.0 : 1.0;
#pragma unroll
            for (int o = 32; o > 0; o >>= 1) {
                const double oa = __shfl_xor(am, o, 64);
                const double of = __shfl_xor(fm, o, 64);
                am = oa > am ? oa : am;
                fm = of > fm ? of : fm;
            }
            if (lane == 0) { S.red[wv] = am; S.rv[wv] = fm; }
            __syncthreads();
            if (tid == 0) {
                double a2 = 0.0, f2 = 0.0;
                for (int i2 = 0; i2 < NW; ++i2) {
                    a2 = S.red[i2] > a2 ? S.red[i2] : a2;
                    f2 = S.rv[i2] > f2 ? S.rv[i2] : f2;
                }
                S.amax = a2;
                S.go = (f2 == 0.0);
            }
            __syncthreads();
        }
        if (!S.go) {  // NaN/Inf: nothing written
            if (tid == 0) {
                q.rank[mi] = -1;
                q.status[mi] = 1;
                if (q.info) {
                    int64_t *inf = q.info + 4 * (int64_t)mi;
                    inf[0] = inf[1] = inf[2] = inf[3] = 0;
                }
            }
            __syncthreads();
            continue;
        }
        for (int c = tid; c < n; c += NT) perm[c] = c;
        for (int c = tid; c < p; c += NT) tau_h[c] = 0.0;
        if (tid == 0) {
            S.ns = 0;
            S.rank = -1;
            S.fb = 0;
            S.nstep = S.nbreak = S.nfb = 0;
            S.t0 = wall_clock64();
        }
        sync_global();
        const double amax = S.amax;

        while (amax > 0.0) {
            const int ns = S.ns;
            if (ns >= p) break;
            // ------------------------------------------------- arg-max, tests
            double bv = -1.0;
            int bj = 0x7fffffff;
            for (int c = ns + tid; c < n; c += NT) {
                const double v = S.vn1[c];
                if (v > bv) { bv = v; bj = c; }
            }
#pragma unroll
            for (int o = 32; o > 0; o >>= 1) {
                const double ov = __shfl_xor(bv, o, 64);
                const int oj = __shfl_xor(bj, o, 64);
                if (qb_beats(ov, oj, bv, bj)) { bv = ov; bj = oj; }
            }
            if (lane == 0) { S.rv[wv] = bv; S.rj[wv] = bj; }
            __syncthreads();
            if (tid == 0) {
                double uv = S.rv[0];
                int uj = S.rj[0];
                for (int i2 = 1; i2 < NW; ++i2)
                    if (qb_beats(S.rv[i2], S.rj[i2], uv, uj)) { uv = S.rv[i2]; uj = S.rj[i2]; }
                S.umax = uv;
                S.L[0] = uj;
                S.go = 1;
                if (S.rank < 0) {
                    const double lhs = (q.stop_rule == 1) ? uv : sqrt((double)(n - ns)) * uv;
                    if (lhs <= eps1 * amax) {
                        S.rank = ns;
                        if (q.stop_rule != 2) S.go = 0;
                    }
                }
                S.fb = (uv <= fbeps * amax) ? 1 : 0;
                S.eps_s = tau * uv;
                S.ncand = 0;
            }
            __syncthreads();
            if (!S.go) break;
            const double umax = S.umax;
            const int kcap = kmax < p - ns ? kmax : p - ns;  // no block runs past min(m, n)
            // ------------------------------------------------- candidates
            if (S.fb || kcap == 1) {
                if (tid == 0) S.nL = 1;
            } else {
                const double thr = tau * umax;
                int cnt = 0;
                for (int c = ns + tid; c < n; c += NT) {
                    const double v = S.vn1[c];
                    if (v >= thr) {
                        ++cnt;
                        int rk = 0;
                        for (int o = ns; o < n && rk < kcap; ++o) {
                            const double ov = S.vn1[o];
                            rk += (ov >= thr && qb_beats(ov, o, v, c)) ? 1 : 0;
                        }
                        if (rk < kcap) S.L[rk] = c;
                    }
                }
                if (cnt) atomicAdd(&S.ncand, cnt);
                __syncthreads();
                if (tid == 0) S.nL = S.ncand < kcap ? S.ncand : kcap;
            }
            __syncthreads();
            const int nL = S.nL;
            // ------------------------------------------------- Gram, greedy
            if (nL > 1) {
                const double *Ab = A + ns;
                const int t = m - ns;
                auto ccol = [&](int r, int i2) -> double { return Ab[(int64_t)S.L[i2] * lda + r]; };
                qb_gram<NT>(ccol, nL, t, S.G);
                __syncthreads();
                if (wv == 0) {
                    // certified mode: delta <= tau^2 / (k_max - 1), eq. (delta_max)
                    const double dl = q.certified ? fmin(delta, tau * tau / (double)(nL - 1)) : delta;
                    // lane j keeps whether candidate j is accepted; Theta_ij = G_ij / (d_i d_j)
                    const double dj = lane < nL ? sqrt(S.G[lane * QB_LD + lane]) : 0.0;
                    bool acc = lane == 0;
                    int ks = 1;
                    for (int i2 = 1; i2 < nL; ++i2) {
                        const double di = sqrt(S.G[i2 * QB_LD + i2]);
                        bool bad = false;
                        if (acc && lane < i2) {
                            const double th = S.G[i2 * QB_LD + lane] / (di * dj);
                            bad = !(fabs(th) < dl);
                        }
                        const bool rej = __any(bad);
                        if (!rej) {
                            if (lane == i2) acc = true;
                            ++ks;
                        }
                    }
                    // accepted candidates in list order
                    const unsigned long long msk = __ballot(acc);
                    if (acc) {
                        const int pos = __popcll(msk & ((1ull << lane) - 1ull));
                        S.J[pos] = S.L[lane];
                    }
                    if (lane == 0) S.ks = ks;
                }
            } else if (tid == 0) {
                S.J[0] = S.L[0];
                S.ks = 1;
            }
            __syncthreads();
            const int ks = S.ks;
            // ------------------------------------------------- swap plan
            // swap i brings accepted column J_i (tracked at its current
            // position) to position ns + i; a swap runs one round after the
            // latest earlier swap that touches one of its columns, so the swaps
            // of one round are disjoint and run together
            if (wv == 0) {
                int pos = lane < ks ? S.J[lane] : -1;  // current position of accepted column `lane`
                int nsw = 0, myd = -1, mys = -1, myr = 0;
                for (int i2 = 0; i2 < ks; ++i2) {
                    const int qpos = __shfl(pos, i2, 64);
                    const int dst = ns + i2;
                    if (qpos != dst) {
                        int rr = 0;
                        if (lane < nsw && (myd == dst || myd == qpos || mys == dst || mys == qpos)) rr = myr + 1;
#pragma unroll
                        for (int o = 32; o > 0; o >>= 1) {
                            const int orr = __shfl_xor(rr, o, 64);
                            rr = orr > rr ? orr : rr;
                        }
                        if (lane == nsw) {
                            myd = dst;
                            mys = qpos;
                            myr = rr;
                        }
                        ++nsw;
                        if (lane > i2 && pos == dst) pos = qpos;
                    }
                    if (lane == i2) pos = dst;
                }
                int mr = lane < nsw ? myr : -1;
#pragma unroll
                for (int o = 32; o > 0; o >>= 1) {
                    const int om = __shfl_xor(mr, o, 64);
                    mr = om > mr ? om : mr;
                }
                if (lane < nsw) {
                    S.swp[2 * lane] = myd;
                    S.swp[2 * lane + 1] = mys;
                    S.swround[lane] = myr;
                }
                if (lane == 0) {
                    S.nsw = nsw;
                    S.nround = mr + 1;
                }
            }
            __syncthreads();
            {
                const int nsw = S.nsw, nround = S.nround;
                for (int rnd = 0; rnd < nround; ++rnd) {
                    for (int s2 = 0; s2 < nsw; ++s2) {
                        if (S.swround[s2] != rnd) continue;
                        const int d = S.swp[2 * s2], sc = S.swp[2 * s2 + 1];
                        for (int r = tid; r < m; r += NT) {
                            const double x = A[(int64_t)d * lda + r];
                            A[(int64_t)d * lda + r] = A[(int64_t)sc * lda + r];
                            A[(int64_t)sc * lda + r] = x;
                        }
                        if (tid == 0) {
                            double x = S.vn1[d]; S.vn1[d] = S.vn1[sc]; S.vn1[sc] = x;
                            x = S.vn2[d]; S.vn2[d] = S.vn2[sc]; S.vn2[sc] = x;
                            const int32_t pp = perm[d]; perm[d] = perm[sc]; perm[sc] = pp;
                        }
                    }
                    sync_global();
                }
            }
            // ------------------------------------------------- panel with break
            const double eps_s = S.eps_s;
            const int tpan = m - ns;
            int l;
            if (PANEL == 1 && tpan <= NT) l = qb_panel_regs<NT, 1, QB_SW>(A, lda, m, ns, ks, eps_s, tau_h, S);
            else if (PANEL == 1 && tpan <= 2 * NT) l = qb_panel_regs<NT, 2, QB_SW>(A, lda, m, ns, ks, eps_s, tau_h, S);
            else l = qb_panel_global<NT>(A, lda, m, ns, ks, eps_s, tau_h, S);
            // ------------------------------------------------- compact WY: T
            qb_build_T<NT>(A, lda, m, ns, l, tau_h, S.G);
            // ------------------------------------------------- trailing update
            if (l > 0 && ns + ks < n) qb_trailing<NT, WC>(A, lda, m, n, ns, l, ns + ks, S.G);
            sync_global();
            // ------------------------------------------------- downdate
            for (int j = ns + l + tid; j < n; j += NT) {
                const double v1 = S.vn1[j];
                if (v1 == 0.0) continue;
                const double *col = A + (int64_t)j * lda;
                double s = 0.0;
                for (int r = 0; r < l; ++r) s += col[ns + r] * col[ns + r];
                double qq = 1.0 - s / (v1 * v1);
                if (qq < 0.0) qq = 0.0;
                const double r12 = v1 / S.vn2[j];
                if (qq * (r12 * r12) <= tol3z) {
                    double t2 = 0.0;
                    for (int r = ns + l; r < m; ++r) t2 += col[r] * col[r];
                    S.vn1[j] = sqrt(t2);
                    S.vn2[j] = S.vn1[j];
                } else {
                    S.vn1[j] = v1 * sqrt(qq);
                }
            }
            if (tid == 0) {
                S.ns = ns + l;
                S.nstep += 1;
                S.nbreak += l < ks ? 1 : 0;
                S.nfb += S.fb;
            }
            __syncthreads();
        }
        if (tid == 0) {
            q.rank[mi] = S.rank >= 0 ? S.rank : (amax > 0.0 ? S.ns : 0);
            q.status[mi] = 0;
            if (q.info) {
                int64_t *inf = q.info + 4 * (int64_t)mi;
                inf[0] = S.nstep;
                inf[1] = S.nbreak;
                inf[2] = S.nfb;
                inf[3] = wall_clock64() - S.t0;
            }
        }
        sync_global();
        if (q.pristine && q.pm && !dflt) {
            // the online check (as qrdm_batch_check) on wavefront 0; a failure is
            // restored from its pristine copy and factored again at the loop top
            if (wv == 0) {
                int64_t r = S.rank >= 0 ? S.rank : (amax > 0.0 ? S.ns : 0);
                if (r > p) r = p;
                int okv = 1;
                if (r > 0) {
                    double dmin;
                    const double est = qb_ice(A, lda, (int)r, S.vn1, &dmin);
                    okv = est >= q.band * dmin ? 1 : 0;
                }
                if (lane == 0) S.okv = okv;
            }
            __syncthreads();
            const int okv = S.okv;
            if (tid == 0 && q.ok) q.ok[mi] = okv;
            if (!okv) {
                const double *P = q.pristine[mi];
                for (int c = 0; c < n; ++c)
                    for (int r = tid; r < m; r += NT) A[(int64_t)c * lda + r] = P[(int64_t)c * lda + r];
                sync_global();
                if (tid == 0) S.redo = 1;
            }
            __syncthreads();
        }
    }
    // last workgroup out resets the queue for the next launch
    if (tid == 0) {
        const unsigned done = atomicAdd(&q.counters[1], 1u);
        if (done + 1 == gridDim.x) {
            atomicExch(&q.counters[0], 0u);
            atomicExch(&q.counters[1], 0u);
        }
    }
}

// variant -> (threads, column tiles per wavefront in the trailing update, panel
// kind).  512-thread workgroups are not offered: at that size the kernel has
// half the registers per thread and spills.
#define QB_VARIANT_LIST(X)  \
    X(0, 256, 1, 1)         \
    X(1, 256, 2, 1)         \
    X(2, 256, 1, 0)

int qb_variant_threads(int variant) {
#define QB_NT(v, nt, wc, pn) if (variant == v) return nt;
    QB_VARIANT_LIST(QB_NT)
#undef QB_NT
    return 0;
}

hipError_t launch_qrdm_batched(const QbArgs &q, int variant, int grid, hipStream_t s) {
    if (q.count <= 0 || grid <= 0) return hipSuccess;
#define QB_LAUNCH(v, nt, wc, pn)                                                           \
    if (variant == v) {                                                                    \
        hipLaunchKernelGGL((k_qrdm_batched<nt, wc, pn>), dim3(grid), dim3(nt), 0, s, q); \
        return hipGetLastError();                                                          \
    }
    QB_VARIANT_LIST(QB_LAUNCH)
#undef QB_LAUNCH
    return hipErrorInvalidValue;
}

hipError_t qb_occupancy(int variant, int *wgs_per_cu) {
#define QB_OCC(v, nt, wc, pn) \
    if (variant == v) return hipOccupancyMaxActiveBlocksPerMultiprocessor(wgs_per_cu, (const void *)k_qrdm_batched<nt, wc, pn>, nt, 0);
    QB_VARIANT_LIST(QB_OCC)
#undef QB_OCC
    return hipErrorInvalidValue;
}
