// Householder panel of a QRDM block from the Gram matrix of its columns
// (Algorithm 4, the panel with the length check of eq. lenght_check), for
// blocks of at most 64 columns.  The column-by-column panel (k_panel) needs one
// grid-wide reduction per pair of columns; here the whole block takes five
// short launches:
//
//   k_cpchol    one workgroup: R1 = chol(G_JJ) of the accepted columns, whose
//               Gram matrix the DM step has already formed (Algorithm 1).  In
//               exact arithmetic |r_ii| of the Householder QR of the block is
//               the norm of column i after the first i reflectors, so the
//               length check becomes r_ii < eps_s (i >= 1) on the Cholesky
//               diagonal, and the block keeps l columns.  W1 = R1^{-1}.
//   k_cpanel1   row slabs: Q1 = C W1 (FP64 MFMA) into the V staging buffer, and
//               each slab's Q1^T Q1 (CholeskyQR, first pass).
//   k_cpreduce  the fixed-order sum of the slabs' Q1^T Q1.
//   k_cpanel2   one workgroup: E = Q1^T Q1 - I; R2 = chol(I + E) = I + N to
//               first order (N = triu(E) with the diagonal halved; used only
//               when max|E| <= 1e-9, so the neglected terms are below 1e-18),
//               R = R2 R1 (CholeskyQR2), the top l x l block of Q = Q1 R2^{-1};
//               the Householder vectors follow from Q by an LU factorization of
//               I - Q_top S with the sign of each S_jj chosen so that every
//               pivot is 1 + |q| (Householder reconstruction, Ballard et al.,
//               2015): V_top = L, U, T = U L^{-T}, P = -R2^{-1} S U^{-1}, and
//               R_H = S R, which is the R of the LAPACK larfg convention
//               (beta_i = -sign(alpha_i) ||x_i||), tau_i = T_ii.
//   k_cpanel3   row slabs: V below the top block = Q1 P (FP64 MFMA).
//
// The rejected columns of a block that stopped early are not touched here:
// the trailing update applies the l reflectors to them with the rest
// (c0off = l).  A block the Gram route does not take (more than 64 columns, a
// column whose Cholesky diagonal falls below 1e-4 of its norm, a Cholesky
// breakdown, or max|E| > 1e-9) is left to k_panel, which the host always
// launches after these and which runs only when cpath = 0.
#include "qrdm_internal.h"

#define CP_K 64          // largest block of the Gram route
#define CP_LD 65         // LDS row stride (doubles)
#define CP_ROWS 128      // rows per workgroup of the slab kernels
#define CP_SAFE 1e-4     // r_ii / ||c_i|| below this: the column-by-column panel
#define CP_EMAX 1e-9     // max |Q1^T Q1 - I| above this: the column-by-column panel

typedef double dbl4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ dbl4 cp_mfma(double a, double b, dbl4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ double cp_readlane(double v, int l) {
    const uint64_t b = (uint64_t)__double_as_longlong(v);
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)b, l);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(b >> 32), l);
    return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}

// 1 / x from the hardware reciprocal and two Newton steps (relative error a
// few units in the last place), for the steps whose latency adds up
__device__ __forceinline__ double cp_rcp(double x) {
    double y = __builtin_amdgcn_rcp(x);
    y = fma(y, fma(-x, y, 1.0), y);
    return fma(y, fma(-x, y, 1.0), y);
}

// ------------------------------------------------------------------ k_cpchol
// The sequential factorizations of this file run on all four wavefronts with
// one barrier per step: thread (wavefront w, lane c) keeps the entries (r, c)
// for the rows r = w + 4u (u < 16) of a 64 x 64 matrix in registers, and the
// row (or column) that a step eliminates with reaches every thread through LDS.
#define CP_U 16

__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(1, 1)))
k_cpchol(QrdmArgs a, const double *G, double *cp, int enable) {
    QrdmCtl *ctl = a.ctl;
    if (qrdm_dm_idle(ctl)) return;
    const int tid = threadIdx.x, lane = tid & 63, wv = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int ks = ctl->ks, nL = ctl->nL;
    if (tid == 0) {  // the column-by-column panel unless this kernel takes the block
        ctl->cpath = 0;
        ctl->c0off = ks;
    }
    if (!enable || ks < 2 || ks > CP_K || nL > CP_K || a.kmax > CP_K) return;
    __shared__ double Rl[CP_K * CP_LD];  // row j of S when step j takes it, then R1
    __shared__ double Xl[CP_K * CP_LD];  // the rows of R1^{-1}
    __shared__ double d0[CP_K], mri[CP_K], rdg[CP_K];
    __shared__ int sAi[CP_K];
    for (int i = tid; i < ks; i += 256) sAi[i] = ctl->Ai[i];
    __syncthreads();
    double s[CP_U];  // G_JJ, rows wv + 4u
#pragma unroll
    for (int u = 0; u < CP_U; ++u) {
        const int r = wv + 4 * u;
        s[u] = (r < ks && lane < ks) ? G[sAi[r] * QK_KM + sAi[lane]] : 0.0;
        if (r == lane && r < ks) d0[r] = s[u];
    }
    const double eps2 = ctl->eps_s * ctl->eps_s;
    // right-looking Cholesky G_JJ = R1^T R1 on the rows of S as they are
    // eliminated: step j takes d = S_jj and S_rc -= S_jr S_jc / d for r > j, and
    // R1_j. = S_j. / sqrt(d) is formed afterwards.  The break of eq.
    // (lenght_check): sqrt(d) < eps_s for j >= 1 (the norm of column j after j
    // reflectors); sqrt(d) below CP_SAFE of the column's norm leaves the block to
    // the column-by-column panel.  Every thread takes the same decisions from
    // the same d.
    int l = ks, flag = 0;
    __syncthreads();
#pragma unroll
    for (int j = 0; j < CP_K; ++j) {
        if (j < l) {  // uniform: l drops to j at a break
            if (wv == (j & 3)) Rl[j * CP_LD + lane] = s[j >> 2];
            __syncthreads();
            const double d = Rl[j * CP_LD + j], sjc = Rl[j * CP_LD + lane];
            double sjr[CP_U];
#pragma unroll
            for (int u = 0; u < CP_U; ++u) sjr[u] = Rl[j * CP_LD + wv + 4 * u];
            if (j >= 1 && !(d >= eps2)) flag = 1;
            else if (!(d > 0.0) || !(d >= CP_SAFE * CP_SAFE * d0[j])) flag = 2;
            if (flag) {
                l = j;
            } else {
                // rows r <= j are finished (row j is in Rl): updating them too
                // keeps the step free of branches
                const double t = sjc * cp_rcp(d);
#pragma unroll
                for (int uu = 0; uu < CP_U; ++uu) {
                    const int u = (uu + ((j + 1) >> 2)) & (CP_U - 1);  // the next pivot row first
                    s[u] -= sjr[u] * t;
                }
            }
        }
    }
    if (flag == 2) return;
    if (tid < l) {
        const double r = sqrt(Rl[tid * CP_LD + tid]);
        mri[tid] = 1.0 / r;
        rdg[tid] = r;
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < CP_U; ++u) {
        const int i = wv + 4 * u;
        if (i < l) {
            const double v = Rl[i * CP_LD + lane];
            Rl[i * CP_LD + lane] = lane == i ? rdg[i] : ((lane > i && lane < ks) ? v * mri[i] : 0.0);
        }
    }
    // W1 = R1^{-1} by rows from the bottom: row i = (e_i - sum_{k > i} R1_ik W1_k.) / r_ii,
    // each finished row swept out of the rows above it
    double x[CP_U];
#pragma unroll
    for (int u = 0; u < CP_U; ++u) x[u] = (wv + 4 * u == lane && lane < l) ? 1.0 : 0.0;
#pragma unroll
    for (int i = CP_K - 1; i >= 0; --i) {
        if (i < l) {
            if (wv == (i & 3)) Xl[i * CP_LD + lane] = lane < l ? x[i >> 2] * mri[i] : 0.0;
            __syncthreads();
            const double xic = Xl[i * CP_LD + lane];
            double rri[CP_U];
#pragma unroll
            for (int u = 0; u < CP_U; ++u) rri[u] = Rl[(wv + 4 * u) * CP_LD + i];
#pragma unroll
            for (int uu = 0; uu < CP_U; ++uu) {  // rows >= i are finished; row i - 1 first
                const int u = (uu + ((i + 63) >> 2)) & (CP_U - 1);
                x[u] -= rri[u] * xic;
            }
        }
    }
    __syncthreads();
    {
        double *R1 = cp + CP_OFF_R1, *W1 = cp + CP_OFF_W1;
#pragma unroll
        for (int u = 0; u < CP_U; ++u) {
            const int e = tid + 256 * u, i = e >> 6, c = e & 63;
            const bool in = i <= c && c < l;
            R1[e] = in ? Rl[i * CP_LD + c] : 0.0;
            W1[e] = in ? Xl[i * CP_LD + c] : 0.0;
        }
    }
    if (tid == 0) {
        ctl->cpath = 1;
        ctl->l = l;
    }
}

hipError_t launch_cpchol(QrdmArgs a, const double *G, double *cp, int enable, hipStream_t s) {
    hipLaunchKernelGGL(k_cpchol, dim3(1), dim3(256), 0, s, a, G, cp, enable);
    return hipGetLastError();
}

// ------------------------------------------------------------------ k_cpanel1
// Slab s: rows [128 s, 128 s + 128) of the block (from row n_s); Q1 = C W1
// (32 output tiles of 16 x 16, eight per wavefront) and the slab's Q1^T Q1
// (16 tiles, four per wavefront) to Gp[s] (leading dimension kp).
__global__ void __launch_bounds__(256) k_cpanel1(QrdmArgs a, const double *cp, double *Vw, int64_t ldv, double *Gp,
                                                 int kp) {
    const QrdmCtl *ctl = a.ctl;
    if (qrdm_dm_idle(ctl) || !ctl->cpath) return;
    const int64_t ns = ctl->ns, t = a.m - ns;
    const int l = ctl->l;
    const int64_t r0 = (int64_t)blockIdx.x * CP_ROWS;
    if (r0 >= t) return;
    const int nr = (int)(t - r0 < CP_ROWS ? t - r0 : CP_ROWS);
    __shared__ double Cs[CP_ROWS * CP_LD];
    __shared__ double Ws[CP_K * CP_LD];
    const int tid = threadIdx.x, lane = tid & 63, wv = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int lt = (l + 15) >> 4, lp = 16 * lt;
    {  // the slab (column-major walk: coalesced rows) and W1, all loads before the stores
        double v[32], w[16];
#pragma unroll
        for (int u = 0; u < 32; ++u) {
            const int e = tid + 256 * u, c = e >> 7, r = e & (CP_ROWS - 1);
            v[u] = (c < l && r < nr) ? a.A[(ns + c) * a.lda + ns + r0 + r] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < 16; ++u) w[u] = cp[CP_OFF_W1 + tid + 256 * u];
#pragma unroll
        for (int u = 0; u < 32; ++u) {
            const int e = tid + 256 * u, c = e >> 7, r = e & (CP_ROWS - 1);
            Cs[r * CP_LD + c] = v[u];
        }
#pragma unroll
        for (int u = 0; u < 16; ++u) {
            const int e = tid + 256 * u;
            Ws[(e >> 6) * CP_LD + (e & 63)] = w[u];
        }
    }
    __syncthreads();
    const int i16 = lane & 15, k4 = lane >> 4;
    dbl4 acc[8];
    const int ntile = 8 * lt;  // 8 row tiles x lt column tiles
#pragma unroll
    for (int u = 0; u < 8; ++u) {
        const int tile = wv + 4 * u;
        acc[u] = dbl4{0.0, 0.0, 0.0, 0.0};
        if (tile < ntile) {
            const int rt = tile / lt, ct = tile - rt * lt;
            for (int kb = 0; kb < lp; kb += 4)
                acc[u] = cp_mfma(Cs[(rt * 16 + i16) * CP_LD + kb + k4], Ws[(kb + k4) * CP_LD + ct * 16 + i16], acc[u]);
        }
    }
    __syncthreads();  // every MFMA has read Cs: it now holds Q1
#pragma unroll
    for (int u = 0; u < 8; ++u) {
        const int tile = wv + 4 * u;
        if (tile < ntile) {
            const int rt = tile / lt, ct = tile - rt * lt;
#pragma unroll
            for (int v = 0; v < 4; ++v) Cs[(rt * 16 + 4 * v + k4) * CP_LD + ct * 16 + i16] = acc[u][v];
        }
    }
    __syncthreads();
#pragma unroll 4
    for (int u = 0; u < 32; ++u) {
        const int e = tid + 256 * u, c = e >> 7, r = e & (CP_ROWS - 1);
        if (c < l && r < nr) Vw[(int64_t)c * ldv + r0 + r] = Cs[r * CP_LD + c];
    }
    // the slab's Q1^T Q1 (rows past nr are zero)
    double *out = Gp + (int64_t)blockIdx.x * kp * kp;
    const int gt = lt * lt;
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        const int tile = wv + 4 * u;
        if (tile < gt) {
            const int ti = tile / lt, tj = tile - ti * lt;
            dbl4 g = {0.0, 0.0, 0.0, 0.0};
            for (int kb = 0; kb < CP_ROWS; kb += 4)
                g = cp_mfma(Cs[(kb + k4) * CP_LD + ti * 16 + i16], Cs[(kb + k4) * CP_LD + tj * 16 + i16], g);
#pragma unroll
            for (int v = 0; v < 4; ++v) out[(ti * 16 + 4 * v + k4) * kp + tj * 16 + i16] = g[v];
        }
    }
}

hipError_t launch_cpanel1(QrdmArgs a, const double *cp, double *Vw, int64_t ldv, double *Gp, int kp, int64_t t_bound,
                          hipStream_t s) {
    if (t_bound <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_cpanel1, dim3((unsigned)((t_bound + CP_ROWS - 1) / CP_ROWS)), dim3(256), 0, s, a, cp, Vw,
                       ldv, Gp, kp);
    return hipGetLastError();
}

int cpanel_partials(int64_t m) { return (int)((m + CP_ROWS - 1) / CP_ROWS); }

// ------------------------------------------------------------------ k_cpreduce
__global__ void __launch_bounds__(256) k_cpreduce(QrdmArgs a, const double *Gp, int kp, double *cp) {
    const QrdmCtl *ctl = a.ctl;
    if (qrdm_dm_idle(ctl) || !ctl->cpath) return;
    const int l = ctl->l;
    const int64_t t = a.m - ctl->ns;
    const int np = (int)((t + CP_ROWS - 1) / CP_ROWS);
    const int e = blockIdx.x * 256 + threadIdx.x;
    if (e >= l * l) return;
    const int i = e / l, j = e - i * l;
    double s = 0.0;
    for (int w0 = 0; w0 < np; w0 += 16) {  // fixed order, sixteen loads in flight
        double v[16];
#pragma unroll
        for (int u = 0; u < 16; ++u) v[u] = w0 + u < np ? Gp[(int64_t)(w0 + u) * kp * kp + i * kp + j] : 0.0;
#pragma unroll
        for (int u = 0; u < 16; ++u) s += v[u];
    }
    cp[CP_OFF_G2 + i * CP_K + j] = s;
}

hipError_t launch_cpreduce(QrdmArgs a, const double *Gp, int kp, double *cp, hipStream_t s) {
    hipLaunchKernelGGL(k_cpreduce, dim3((CP_K * CP_K + 255) / 256), dim3(256), 0, s, a, Gp, kp, cp);
    return hipGetLastError();
}

// ------------------------------------------------------------------ k_cpanel2
// C = A B for 64 x 64 operands on FP64 MFMA by the four wavefronts (sixteen
// 16 x 16 output tiles, four per wavefront): fa(i, k) and fb(k, j) give the
// operands (zero outside the block), out(i, j, v) takes each result.  A tile's
// operands are all loaded before its MFMAs.
template <typename FA, typename FB, typename OUT>
__device__ __forceinline__ void cp_mm(FA fa, FB fb, OUT out) {
    const int lane = threadIdx.x & 63, wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int i16 = lane & 15, k4 = lane >> 4;
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        const int tile = wv + 4 * u, rt = tile >> 2, ct = tile & 3;
        double av[16], bv[16];
#pragma unroll
        for (int kb = 0; kb < 16; ++kb) {
            av[kb] = fa(rt * 16 + i16, 4 * kb + k4);
            bv[kb] = fb(4 * kb + k4, ct * 16 + i16);
        }
        dbl4 acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int kb = 0; kb < 16; ++kb) acc = cp_mfma(av[kb], bv[kb], acc);
#pragma unroll
        for (int v = 0; v < 4; ++v) out(rt * 16 + 4 * v + k4, ct * 16 + i16, acc[v]);
    }
}

__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(1, 1)))
k_cpanel2(QrdmArgs a, double *cp, const double *Vw, int64_t ldv, double *Vo,
                                                 float *Vo32) {
    QrdmCtl *ctl = a.ctl;
    if (qrdm_dm_idle(ctl) || !ctl->cpath) return;
    const int64_t ns = ctl->ns;
    const int l = ctl->l, ks = ctl->ks;
    const int tid = threadIdx.x, lane = tid & 63, wv = __builtin_amdgcn_readfirstlane(tid >> 6);
    // A1: R1, then Uinv (upper); A2: N (upper) | Linv (strictly lower);
    // A3: Q1_top, then R (upper); A4: Q_top, then the LU (L below the diagonal,
    // dq on it, Y above)
    extern __shared__ double cp_lds[];
    double *A1 = cp_lds, *A2 = A1 + CP_K * CP_LD, *A3 = A2 + CP_K * CP_LD, *A4 = A3 + CP_K * CP_LD;
    __shared__ double sS[CP_K], sUd[CP_K], sUi[CP_K], s_red[4];
    double *Tg = cp + CP_OFF_T, *Pg = cp + CP_OFF_P;
    for (int e = tid; e < 4 * CP_K * CP_LD; e += 256) cp_lds[e] = 0.0;
    for (int e = tid; e < CP_K * CP_K; e += 256) {
        Tg[e] = 0.0;
        Pg[e] = 0.0;
    }
    __syncthreads();
    // ---- E = Q1^T Q1 - I, its size, and N = triu(E) with the diagonal halved
    double emax = 0.0;
    {  // every load of a thread issued before its stores; Q1_top walked down its columns
        double g[16], r1[16], q[16];
#pragma unroll
        for (int u = 0; u < 16; ++u) {
            const int e = tid + 256 * u, i = e >> 6, c = e & 63;
            g[u] = (i < l && c < l) ? cp[CP_OFF_G2 + e] : 0.0;
            r1[u] = (i <= c && c < l) ? cp[CP_OFF_R1 + e] : 0.0;
            q[u] = (c < l && i < l) ? Vw[(int64_t)i * ldv + c] : 0.0;  // row c, column i of Q1
        }
#pragma unroll
        for (int u = 0; u < 16; ++u) {
            const int e = tid + 256 * u, i = e >> 6, c = e & 63;
            if (i < l && c < l) {
                const double v = g[u] - (i == c ? 1.0 : 0.0);
                emax = fmax(emax, fabs(v));
                if (i <= c) A2[i * CP_LD + c] = (i == c) ? 0.5 * v : v;
                A3[c * CP_LD + i] = q[u];
            }
            if (i <= c && c < l) A1[i * CP_LD + c] = r1[u];
        }
    }
    for (int o = 32; o > 0; o >>= 1) emax = fmax(emax, __shfl_xor(emax, o, 64));
    if (lane == 0) s_red[wv] = emax;
    __syncthreads();
    emax = fmax(fmax(s_red[0], s_red[1]), fmax(s_red[2], s_red[3]));
    if (!(emax <= CP_EMAX)) {  // Q1 not orthonormal enough for the first-order R2
        if (tid == 0) {
            ctl->cpath = 0;
            ctl->l = ks;
        }
        return;
    }
    // ---- Q_top = Q1_top (I - N) (R2^{-1} to first order) into A4; R = (I + N) R1 into A3
    cp_mm([&](int i, int k) { return A3[i * CP_LD + k]; }, [&](int k, int j) { return A2[k * CP_LD + j]; },
          [&](int i, int j, double v) { A4[i * CP_LD + j] = A3[i * CP_LD + j] - v; });
    __syncthreads();
    cp_mm([&](int i, int k) { return A2[i * CP_LD + k]; }, [&](int k, int j) { return A1[k * CP_LD + j]; },
          [&](int i, int j, double v) { A3[i * CP_LD + j] = (i <= j) ? A1[i * CP_LD + j] + v : 0.0; });
    __syncthreads();
    // ---- LU of I - Q_top S, signs chosen on the way: pivot j is 1 + |dq_j| with
    // dq_j = W_jj after j steps, L_rj = -S_j W_rj / U_jj, and W_rc -= L_rj W_jc for
    // r, c > j.  Thread (wavefront w, lane c) holds W_rc for the rows r = w + 4u;
    // row j, final at step j, goes to A4 (which ends as L below the diagonal, dq
    // on it, Y above) and the entries W_rj of a wavefront's rows come from its
    // lane j.
    {
        double w[CP_U];
#pragma unroll
        for (int u = 0; u < CP_U; ++u) w[u] = A4[(wv + 4 * u) * CP_LD + lane];
        __syncthreads();  // Q_top read everywhere before its rows are replaced
        // a loop at run time (the register holding row j is picked by a select)
#pragma unroll 1
        for (int j = 0; j < l; ++j) {
            if (wv == (j & 3)) {
                const int uj = j >> 2;
                double wr = w[0];
#pragma unroll
                for (int u = 1; u < CP_U; ++u) wr = u == uj ? w[u] : wr;
                A4[j * CP_LD + lane] = wr;
            }
            __syncthreads();
            const double dq = A4[j * CP_LD + j];
            const double sj = dq >= 0.0 ? -1.0 : 1.0;
            const double ujj = 1.0 - sj * dq;
            const double f = -sj * cp_rcp(ujj);
            const double wjc = lane > j ? A4[j * CP_LD + lane] : 0.0;
            // rows r <= j are finished (row j is in A4): updating them too keeps
            // the sixteen updates free of branches, so that they overlap
#pragma unroll
            for (int u = 0; u < CP_U; ++u) {
                const double m = f * cp_readlane(w[u], j);
                w[u] = lane == j ? m : w[u] - m * wjc;
            }
        }
    }
    __syncthreads();
    if (tid < l) {  // the signs and pivots, from dq on the diagonal of the LU
        const double dq = A4[tid * CP_LD + tid];
        const double sj = dq >= 0.0 ? -1.0 : 1.0;
        const double ujj = 1.0 - sj * dq;
        sS[tid] = sj;
        sUd[tid] = ujj;
        sUi[tid] = 1.0 / ujj;
    }
    __syncthreads();
    // ---- Linv = L^{-1} into A2 below the diagonal and Uinv = U^{-1} into A1 (upper;
    // U_ik = -S_k Y_ik, U_ii = 1 + |dq_i|), in one sweep: step s finishes row
    // k = s of Linv (forward) and row i = l - 1 - s of Uinv (backward) and
    // sweeps each out of the rows that remain.
    {
        double xl[CP_U], xu[CP_U];
#pragma unroll
        for (int u = 0; u < CP_U; ++u) {
            const int r = wv + 4 * u;
            xl[u] = (r == lane && r < l) ? 1.0 : 0.0;
            xu[u] = xl[u];
        }
#pragma unroll 1
        for (int st = 0; st < l; ++st) {
            const int k = st, i = l - 1 - st;  // the rows finished at this step
            if (wv == (k & 3)) {
                double xk = 0.0;
#pragma unroll
                for (int u = 0; u < CP_U; ++u) xk = wv + 4 * u == k ? xl[u] : xk;
                if (lane < k) A2[k * CP_LD + lane] = xk;
            }
            if (wv == (i & 3)) {
                double xi = 0.0;
#pragma unroll
                for (int u = 0; u < CP_U; ++u) xi = wv + 4 * u == i ? xu[u] : xi;
                A1[i * CP_LD + lane] = lane >= i && lane < l ? xi * sUi[i] : 0.0;
            }
            __syncthreads();
            const double xkc = lane < k ? A2[k * CP_LD + lane] : (lane == k ? 1.0 : 0.0);
            const double xic = A1[i * CP_LD + lane];
            const double nsi = -sS[i];
            const double *a4k = A4 + wv * CP_LD + k, *a4i = A4 + wv * CP_LD + i;
            double lk[CP_U], ui[CP_U];  // every load of the step before its updates
#pragma unroll
            for (int u = 0; u < CP_U; ++u) {
                lk[u] = a4k[4 * u * CP_LD];
                ui[u] = a4i[4 * u * CP_LD];
            }
            // rows <= k of Linv, >= i of Uinv, and >= l are finished or unused:
            // updating them too keeps the step free of branches
#pragma unroll
            for (int u = 0; u < CP_U; ++u) {
                xl[u] -= lk[u] * xkc;
                xu[u] -= (nsi * ui[u]) * xic;
            }
        }
    }
    __syncthreads();
    // ---- T = U Linv^T and P = -(I - N) S Uinv.  A block that reaches the last
    // row (t = l) ends with a column of one row: larfg leaves it alone (tau = 0,
    // beta = alpha), where the reconstruction reflects it (tau = 2, v = e); its
    // column of T and tau are zeroed and its diagonal entry takes the other sign.
    const bool lastrow = (a.m - ns) == (int64_t)l;
    auto uval = [&](int i, int k) -> double {
        const double y = A4[i * CP_LD + k], sk = sS[k], ud = sUd[i];  // loads first, then selects
        return (i >= l || k >= l || k < i) ? 0.0 : (k == i ? ud : -sk * y);
    };
    cp_mm(uval,
          [&](int k, int j) {
              const double v = A2[j * CP_LD + k];
              return (j >= l || k >= l) ? 0.0 : (j == k ? 1.0 : (j > k ? v : 0.0));
          },
          [&](int i, int j, double v) {
              if (i < l && j < l && !(lastrow && j == l - 1)) Tg[i * CP_K + j] = v;
          });
    cp_mm(
          [&](int i, int k) {
              const double n = A2[i * CP_LD + k], sk = sS[k];
              return (i >= l || k >= l || k < i) ? 0.0 : (k == i ? -(1.0 - n) * sk : n * sk);
          },
          [&](int k, int j) { return A1[k * CP_LD + j]; },
          [&](int i, int j, double v) {
              if (i < l && j < l) Pg[i * CP_K + j] = v;
          });
    // ---- the top block of A (R_H = S R above, L below), V_top, tau
    for (int e = tid; e < l * l; e += 256) {
        const int i = e / l, c = e - i * l;
        const double flip = (lastrow && i == l - 1) ? -1.0 : 1.0;
        a.A[(ns + c) * a.lda + ns + i] = (i <= c) ? flip * sS[i] * A3[i * CP_LD + c] : A4[i * CP_LD + c];
        const double v = (i > c) ? A4[i * CP_LD + c] : (i == c ? 1.0 : 0.0);
        Vo[(int64_t)c * ldv + i] = v;
        if (Vo32) Vo32[(int64_t)c * ldv + i] = (float)v;
    }
    if (tid < l) a.tau_house[ns + tid] = (lastrow && tid == l - 1) ? 0.0 : sUd[tid];  // T_ii = U_ii
    if (tid == 0) {
        ctl->c0off = l;
        if (l < ks) ctl->nbreaks += 1;
        const double t = (double)(a.m - ns);
        double fl = 0.0;
        for (int i = 0; i < l; ++i) fl += (t - i) * (2.0 + 4.0 * (double)(ks - 1 - i));
        ctl->flop_panel += fl;
        ctl->bytes_panel += 16.0 * t * (double)ks;
        ctl->npanel += 1;
        ctl->ngram += 1;
    }
}

hipError_t launch_cpanel2(QrdmArgs a, double *cp, const double *Vw, int64_t ldv, double *Vo, float *Vo32,
                          hipStream_t s) {
    const unsigned lds = 4 * CP_K * CP_LD * sizeof(double);
    static bool attr = false;
    if (!attr) {
        hipError_t e = hipFuncSetAttribute((const void *)k_cpanel2, hipFuncAttributeMaxDynamicSharedMemorySize, lds);
        if (e != hipSuccess) return e;
        attr = true;
    }
    hipLaunchKernelGGL(k_cpanel2, dim3(1), dim3(256), lds, s, a, cp, Vw, ldv, Vo, Vo32);
    return hipGetLastError();
}

// ------------------------------------------------------------------ k_cpanel3
// Slab s: rows [128 s, 128 s + 128) of the block past its top l rows:
// V = Q1 P, written to A (below the top block) and, in place of Q1, to the V
// staging buffer (and its FP32 copy in mixed precision).
__global__ void __launch_bounds__(256) k_cpanel3(QrdmArgs a, const double *cp, double *Vw, int64_t ldv, float *Vw32) {
    const QrdmCtl *ctl = a.ctl;
    if (qrdm_dm_idle(ctl) || !ctl->cpath) return;
    const int64_t ns = ctl->ns, t = a.m - ns;
    const int l = ctl->l;
    const int64_t r0 = (int64_t)blockIdx.x * CP_ROWS;
    if (r0 >= t) return;
    const int nr = (int)(t - r0 < CP_ROWS ? t - r0 : CP_ROWS);
    const int rlo = r0 < l ? (int)(l - r0) : 0;  // rows of the top block (written by k_cpanel2)
    if (rlo >= nr) return;
    __shared__ double Qs[CP_ROWS * CP_LD];
    __shared__ double Ps[CP_K * CP_LD];
    const int tid = threadIdx.x, lane = tid & 63, wv = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int lt = (l + 15) >> 4, lp = 16 * lt;
    {
        double v[32], w[16];
#pragma unroll
        for (int u = 0; u < 32; ++u) {
            const int e = tid + 256 * u, c = e >> 7, r = e & (CP_ROWS - 1);
            v[u] = (c < l && r >= rlo && r < nr) ? Vw[(int64_t)c * ldv + r0 + r] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < 16; ++u) w[u] = cp[CP_OFF_P + tid + 256 * u];
#pragma unroll
        for (int u = 0; u < 32; ++u) {
            const int e = tid + 256 * u, c = e >> 7, r = e & (CP_ROWS - 1);
            Qs[r * CP_LD + c] = v[u];
        }
#pragma unroll
        for (int u = 0; u < 16; ++u) {
            const int e = tid + 256 * u;
            Ps[(e >> 6) * CP_LD + (e & 63)] = w[u];
        }
    }
    __syncthreads();
    const int i16 = lane & 15, k4 = lane >> 4;
    dbl4 acc[8];
    const int ntile = 8 * lt;
#pragma unroll
    for (int u = 0; u < 8; ++u) {
        const int tile = wv + 4 * u;
        acc[u] = dbl4{0.0, 0.0, 0.0, 0.0};
        if (tile < ntile) {
            const int rt = tile / lt, ct = tile - rt * lt;
            for (int kb = 0; kb < lp; kb += 4)
                acc[u] = cp_mfma(Qs[(rt * 16 + i16) * CP_LD + kb + k4], Ps[(kb + k4) * CP_LD + ct * 16 + i16], acc[u]);
        }
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < 8; ++u) {
        const int tile = wv + 4 * u;
        if (tile < ntile) {
            const int rt = tile / lt, ct = tile - rt * lt;
#pragma unroll
            for (int v = 0; v < 4; ++v) Qs[(rt * 16 + 4 * v + k4) * CP_LD + ct * 16 + i16] = acc[u][v];
        }
    }
    __syncthreads();
#pragma unroll 4
    for (int u = 0; u < 32; ++u) {
        const int e = tid + 256 * u, c = e >> 7, r = e & (CP_ROWS - 1);
        if (c < l && r >= rlo && r < nr) {
            const double v = Qs[r * CP_LD + c];
            a.A[(ns + c) * a.lda + ns + r0 + r] = v;
            Vw[(int64_t)c * ldv + r0 + r] = v;
            if (Vw32) Vw32[(int64_t)c * ldv + r0 + r] = (float)v;
        }
    }
}

hipError_t launch_cpanel3(QrdmArgs a, const double *cp, double *Vw, int64_t ldv, float *Vw32, int64_t t_bound,
                          hipStream_t s) {
    if (t_bound <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_cpanel3, dim3((unsigned)((t_bound + CP_ROWS - 1) / CP_ROWS)), dim3(256), 0, s, a, cp, Vw,
                       ldv, Vw32);
    return hipGetLastError();
}
