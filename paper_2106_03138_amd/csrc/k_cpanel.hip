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
#include <type_traits>
#include <utility>

#include "qrdm_internal.h"

#define CP_K 64          // largest block of the Gram route
#define CP_LD 65         // LDS row stride (doubles)
#define CP_SR 64         // rows per workgroup of the slab kernels
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

// value of lane 16 (lane / 16) + K in every lane (a DPP row broadcast: one
// move for the 64-bit value, where a read of a lane into scalar registers
// takes two)
template <int K>
__device__ __forceinline__ double cp_rowbcast(double v) {
    return __builtin_amdgcn_update_dpp(0.0, v, 0x150 + K, 0xf, 0xf, true);
}

// f(std::integral_constant<int, i>) for i = 0 .. N-1, unrolled at compile time
template <typename F, int... I>
__device__ __forceinline__ void cp_static_for_seq(F &&f, std::integer_sequence<int, I...>) {
    (f(std::integral_constant<int, I>{}), ...);
}
template <int N, typename F>
__device__ __forceinline__ void cp_static_for(F &&f) {
    cp_static_for_seq(f, std::make_integer_sequence<int, N>{});
}

// 1 / x from the hardware reciprocal and two Newton steps (relative error a
// few units in the last place), for the steps whose latency adds up
__device__ __forceinline__ double cp_rcp(double x) {
    double y = __builtin_amdgcn_rcp(x);
    y = fma(y, fma(-x, y, 1.0), y);
    return fma(y, fma(-x, y, 1.0), y);
}

// 1 / sqrt(x) from the hardware estimate and two Newton steps
__device__ __forceinline__ double cp_rsqrt(double x) {
    double y = __builtin_amdgcn_rsq(x);
    const double h = 0.5 * x;
    y = y * fma(-h * y, y, 1.5);
    return y * fma(-h * y, y, 1.5);
}

// ------------------------------------------------------------------ blocked helpers
// The sequential factorizations of this file are blocked by 16 columns: the
// dependent steps inside a 16-column panel run on one wavefront without
// barriers (values move between lanes by readlane), the solves and updates
// around them on FP64 MFMA over the four wavefronts, one barrier between
// phases.
#define CP_LD16 17  // row stride of the 16 x 16 staging blocks

// acc + A B for one 16 x 16 block on one wavefront (K = 16), fa(i, k) and
// fb(k, j) giving the operands; register v of a lane then holds row
// 4v + lane / 16, column lane % 16.
template <typename FA, typename FB>
__device__ __forceinline__ dbl4 cp_mm16(FA fa, FB fb, dbl4 acc) {
    const int lane = threadIdx.x & 63, i16 = lane & 15, k4 = lane >> 4;
    double av[4], bv[4];
#pragma unroll
    for (int kb = 0; kb < 4; ++kb) {
        av[kb] = fa(i16, 4 * kb + k4);
        bv[kb] = fb(4 * kb + k4, i16);
    }
#pragma unroll
    for (int kb = 0; kb < 4; ++kb) acc = cp_mfma(av[kb], bv[kb], acc);
    return acc;
}

// X = R^{-1} for an upper triangular R of order 64: r(i, k) gives R_ik for
// i < k and rinv(i) = 1 / R_ii (the caller makes R the identity outside its
// leading block).  Wavefront w inverts diagonal block w by back substitution
// (lane c < 16 forms column c), then the blocks above the diagonal follow by
// block diagonals on MFMA, X_ij = -X_ii sum_{i < k <= j} R_ik X_kj, one
// barrier per diagonal.  xr(i, j) reads X (on and above the diagonal blocks
// only), xw(i, j, v) writes it.  With TWO, a second, independent inverse
// (r2, rinv2, xr2, xw2) is formed beside the first, step for step, so that the
// two dependent chains overlap; each is computed exactly as it would be alone.
// Tmp holds four 16 x CP_LD16 blocks per inverse.  Every thread of the
// workgroup calls it.
template <bool TWO, typename RA, typename RI, typename XR, typename XW, typename RA2, typename RI2, typename XR2,
          typename XW2>
__device__ __forceinline__ void cp_trinv_n(RA r, RI rinv, XR xr, XW xw, RA2 r2, RI2 rinv2, XR2 xr2, XW2 xw2,
                                           double *Tmp) {
    const int lane = threadIdx.x & 63, wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int i16 = lane & 15, k4 = lane >> 4;
    {
        // column i16 of the block's inverse, right-looking from the bottom: x_k is
        // final once scaled, then swept out of the rows above it
        const int b0 = 16 * wv;
        double x[16], rin[16], x2[16], rin2[16];
#pragma unroll
        for (int ii = 0; ii < 16; ++ii) {
            x[ii] = ii == i16 ? 1.0 : 0.0;
            rin[ii] = rinv(b0 + ii);
            x2[ii] = x[ii];
            rin2[ii] = TWO ? rinv2(b0 + ii) : 0.0;
        }
#pragma unroll
        for (int kk = 15; kk >= 0; --kk) {
            double rv[16], rv2[16];
#pragma unroll
            for (int ii = 0; ii < kk; ++ii) {
                rv[ii] = r(b0 + ii, b0 + kk);
                rv2[ii] = TWO ? r2(b0 + ii, b0 + kk) : 0.0;
            }
            x[kk] *= rin[kk];
            if (TWO) x2[kk] *= rin2[kk];
#pragma unroll
            for (int ii = 0; ii < kk; ++ii) {
                x[ii] -= rv[ii] * x[kk];
                if (TWO) x2[ii] -= rv2[ii] * x2[kk];
            }
        }
        if (lane < 16) {
#pragma unroll
            for (int ii = 0; ii < 16; ++ii) {
                xw(b0 + ii, b0 + i16, x[ii]);
                if (TWO) xw2(b0 + ii, b0 + i16, x2[ii]);
            }
        }
    }
    __syncthreads();
#pragma unroll 1
    for (int d = 1; d < 4; ++d) {
        const int bi = wv, bj = wv + d;
        if (bj < 4) {
            double *M = Tmp + wv * 16 * CP_LD16, *M2 = Tmp + (4 + wv) * 16 * CP_LD16;
            dbl4 acc = {0.0, 0.0, 0.0, 0.0}, acc2 = {0.0, 0.0, 0.0, 0.0};
            for (int kb = bi + 1; kb <= bj; ++kb) {
                acc = cp_mm16([&](int i, int k) { return r(16 * bi + i, 16 * kb + k); },
                              [&](int k, int j) { return xr(16 * kb + k, 16 * bj + j); }, acc);
                if (TWO)
                    acc2 = cp_mm16([&](int i, int k) { return r2(16 * bi + i, 16 * kb + k); },
                                   [&](int k, int j) { return xr2(16 * kb + k, 16 * bj + j); }, acc2);
            }
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                M[(4 * v + k4) * CP_LD16 + i16] = acc[v];
                if (TWO) M2[(4 * v + k4) * CP_LD16 + i16] = acc2[v];
            }
            __builtin_amdgcn_wave_barrier();  // M is this wavefront's own: LDS keeps its order
            acc = cp_mm16([&](int i, int k) { return xr(16 * bi + i, 16 * bi + k); },
                          [&](int k, int j) { return M[k * CP_LD16 + j]; }, dbl4{0.0, 0.0, 0.0, 0.0});
            if (TWO)
                acc2 = cp_mm16([&](int i, int k) { return xr2(16 * bi + i, 16 * bi + k); },
                               [&](int k, int j) { return M2[k * CP_LD16 + j]; }, dbl4{0.0, 0.0, 0.0, 0.0});
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                xw(16 * bi + 4 * v + k4, 16 * bj + i16, -acc[v]);
                if (TWO) xw2(16 * bi + 4 * v + k4, 16 * bj + i16, -acc2[v]);
            }
        }
        __syncthreads();
    }
}

template <typename RA, typename RI, typename XR, typename XW>
__device__ __forceinline__ void cp_trinv(RA r, RI rinv, XR xr, XW xw, double *Tmp) {
    cp_trinv_n<false>(r, rinv, xr, xw, r, rinv, xr, xw, Tmp);
}

// ------------------------------------------------------------------ k_cpchol
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(1, 1)))
k_cpchol(QrdmArgs a, const double *G, double *cp, int enable) {
    QrdmCtl *ctl = a.ctl;
    if (qrdm_dm_idle(ctl)) return;
    const int tid = threadIdx.x, lane = tid & 63, wv = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int i16 = lane & 15, k4 = lane >> 4;
    const int ks = ctl->ks, nL = ctl->nL;
    if (tid == 0) {  // the column-by-column panel unless this kernel takes the block
        ctl->cpath = 0;
        ctl->c0off = ks;
    }
    if (!enable || ks < 2 || ks > CP_K || nL > CP_K || a.kmax > CP_K) return;
    __shared__ double S[CP_K * CP_LD];   // G_JJ, then R1 on and above the diagonal
    __shared__ double Xl[CP_K * CP_LD];  // R1^{-1}
    __shared__ double Tmp[4 * 16 * CP_LD16];
    __shared__ double d0[CP_K], mri[CP_K];
    __shared__ int sAi[CP_K], mfl[2];
    for (int i = tid; i < CP_K; i += 256) {
        if (i < ks) sAi[i] = ctl->Ai[i];
        mri[i] = 0.0;
    }
    __syncthreads();
    {  // G_JJ, zero outside k_s x k_s; every load of a thread before its stores
        double v[16];
#pragma unroll
        for (int u = 0; u < 16; ++u) {
            const int e = tid + 256 * u, i = e >> 6, c = e & 63;
            v[u] = (i < ks && c < ks) ? G[sAi[i] * QK_KM + sAi[c]] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < 16; ++u) {
            const int e = tid + 256 * u, i = e >> 6, c = e & 63;
            S[i * CP_LD + c] = v[u];
            if (i == c) d0[i] = v[u];
        }
    }
    __syncthreads();
    const double eps2 = ctl->eps_s * ctl->eps_s;
    // Cholesky G_JJ = R1^T R1, right-looking by 16-column panels.  Step j takes
    // d = S_jj, R1_j. = S_j. / sqrt(d) and S_ic -= R1_ji R1_jc (i, c > j).  The
    // break of eq. (lenght_check): sqrt(d) < eps_s for j >= 1 (the norm of
    // column j after j reflectors), l = j; sqrt(d) below CP_SAFE of the
    // column's norm leaves the block to the column-by-column panel.
    int l = ks, flag = 0;
#pragma unroll 1
    for (int kb = 0; kb < 4; ++kb) {
        const int j0 = 16 * kb;
        if (j0 >= l) break;
        // (a) the diagonal block on wavefront 0, lane i16 holding row j0 + i16
        // (each 16-lane row of the wavefront holds the same copy, so row jj is
        // broadcast within the rows).  Row j keeps S_j. as it stood when it was
        // eliminated, and is scaled to R1_j. once the block is done; the rows
        // below take S_ic -= (S_ij / d) S_jc.
        if (wv == 0) {
            double g[16], d0b[16];
#pragma unroll
            for (int c = 0; c < 16; ++c) g[c] = S[(j0 + i16) * CP_LD + j0 + c];
#pragma unroll
            for (int jj = 0; jj < 16; ++jj) d0b[jj] = d0[j0 + jj];
            int f = 0, lb = l;
            double myd = 1.0;  // the pivot d of this lane's row
            // The steps past k_s run too, as no-ops (al = 0, no flag, myd kept):
            // with no branch between them the next pivot's reciprocal overlaps
            // the current step's updates.
            cp_static_for<16>([&](auto jc) {
                constexpr int jj = decltype(jc)::value;
                const int j = j0 + jj;
                const bool valid = j < ks;
                const double d = cp_readlane(g[jj], jj);
                const bool c1 = (j >= 1) & !(d >= eps2);
                const bool c2 = !(d > 0.0) | !(d >= CP_SAFE * CP_SAFE * d0b[jj]);
                const int fj = valid ? (c1 ? 1 : (c2 ? 2 : 0)) : 0;
                const bool first = (f == 0) & (fj != 0);  // the first failing column decides
                lb = first ? j : lb;
                f = first ? fj : f;
                const double rd = cp_rcp(d);
                const double al = (valid & (i16 > jj)) ? g[jj] * rd : 0.0;
#pragma unroll
                for (int c = jj + 1; c < 16; ++c) g[c] -= al * cp_rowbcast<jj>(g[c]);
                myd = (valid & (i16 == jj)) ? d : myd;
            });
            const double ri = cp_rsqrt(myd);
            if (lane < 16) {
#pragma unroll
                for (int c = 0; c < 16; ++c)
                    S[(j0 + i16) * CP_LD + j0 + c] = c > i16 ? g[c] * ri : (c == i16 ? myd * ri : 0.0);
                mri[j0 + i16] = ri;
            }
            if (lane == 0) {
                mfl[0] = f;
                mfl[1] = lb;
            }
        }
        __syncthreads();
        flag = mfl[0];
        l = mfl[1];
        if (flag) break;
        // (b) rows j0 .. j0+15 of R1 right of the block: R1_12 = R1_11^{-T} S_12,
        // lane c - j0 - 16 of wavefront 0 forming column c
        if (wv == 0) {
            const int c = j0 + 16 + lane;
            if (c < ks) {
                double x[16];
#pragma unroll
                for (int ii = 0; ii < 16; ++ii) x[ii] = S[(j0 + ii) * CP_LD + c];
#pragma unroll
                for (int ii = 0; ii < 16; ++ii) {
                    double rv[16];
#pragma unroll
                    for (int jj = 0; jj < ii; ++jj) rv[jj] = S[(j0 + jj) * CP_LD + j0 + ii];
                    double sum = x[ii];
#pragma unroll
                    for (int jj = 0; jj < ii; ++jj) sum -= rv[jj] * x[jj];
                    x[ii] = sum * mri[j0 + ii];
                }
#pragma unroll
                for (int ii = 0; ii < 16; ++ii) S[(j0 + ii) * CP_LD + c] = x[ii];
            }
        }
        __syncthreads();
        // (c) the trailing Gram block: S_22 -= R1_12^T R1_12 on MFMA
        {
            const int nt = 3 - kb;
            for (int tile = wv; tile < nt * nt; tile += 4) {
                const int rt = kb + 1 + tile / nt, ct = kb + 1 + tile % nt;
                const dbl4 acc = cp_mm16([&](int i, int k) { return S[(j0 + k) * CP_LD + 16 * rt + i]; },
                                         [&](int k, int j) { return S[(j0 + k) * CP_LD + 16 * ct + j]; },
                                         dbl4{0.0, 0.0, 0.0, 0.0});
#pragma unroll
                for (int v = 0; v < 4; ++v) S[(16 * rt + 4 * v + k4) * CP_LD + 16 * ct + i16] -= acc[v];
            }
        }
        __syncthreads();
    }
    if (flag == 2) return;
    // W1 = R1^{-1} (l x l; the identity past l)
    // (the accessors load first and select after: their addresses are always in range)
    cp_trinv([&](int i, int k) { const double v = S[i * CP_LD + k]; return k < l ? v : 0.0; },
             [&](int i) { const double v = mri[i]; return i < l ? v : 1.0; },
             [&](int i, int j) { return Xl[i * CP_LD + j]; },
             [&](int i, int j, double v) { Xl[i * CP_LD + j] = v; }, Tmp);
    {
        double *R1 = cp + CP_OFF_R1, *W1 = cp + CP_OFF_W1;
#pragma unroll
        for (int u = 0; u < 16; ++u) {
            const int e = tid + 256 * u, i = e >> 6, c = e & 63;
            const bool in = i <= c && c < l;
            R1[e] = in ? S[i * CP_LD + c] : 0.0;
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

// ------------------------------------------------------------------ slab kernels
// A slab of CP_SR rows (row stride CP_LD in LDS) times an upper triangular
// 64 x 64 matrix on MFMA: row tile w of the slab on wavefront w, output tile
// ct summing the k-tiles up to ct (the rest of the product is zero); the four
// tiles' accumulations are independent.  acc[ct] returns tile (w, ct).
__device__ __forceinline__ void cp_slab_upper(const double *Xs, const double *Us, dbl4 acc[4]) {
    const int lane = threadIdx.x & 63, wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int i16 = lane & 15, k4 = lane >> 4;
    double av[16], bv[4][16];
#pragma unroll
    for (int kk = 0; kk < 16; ++kk) av[kk] = Xs[(16 * wv + i16) * CP_LD + 4 * kk + k4];
#pragma unroll
    for (int ct = 0; ct < 4; ++ct) {
#pragma unroll
        for (int kk = 0; kk < 4 * (ct + 1); ++kk) bv[ct][kk] = Us[(4 * kk + k4) * CP_LD + 16 * ct + i16];
    }
#pragma unroll
    for (int ct = 0; ct < 4; ++ct) acc[ct] = dbl4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int kk = 0; kk < 16; ++kk) {
#pragma unroll
        for (int ct = 0; ct < 4; ++ct)
            if (kk < 4 * (ct + 1)) acc[ct] = cp_mfma(av[kk], bv[ct][kk], acc[ct]);
    }
}

// ------------------------------------------------------------------ k_cpanel1
// Slab s: rows [64 s, 64 s + 64) of the block (from row n_s): Q1 = C W1 into
// the V staging buffer, and the slab's Q1^T Q1 to Gp[s] (leading dimension
// kp): its ten tiles on and above the diagonal, each off-diagonal one also
// stored transposed, so the partial is the full symmetric matrix.
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(1, 1)))
k_cpanel1(QrdmArgs a, const double *cp, double *Vw, int64_t ldv, double *Gp, int kp) {
    const QrdmCtl *ctl = a.ctl;
    if (qrdm_dm_idle(ctl) || !ctl->cpath) return;
    const int64_t ns = ctl->ns, t = a.m - ns;
    const int l = ctl->l;
    const int64_t r0 = (int64_t)blockIdx.x * CP_SR;
    if (r0 >= t) return;
    const int nr = (int)(t - r0 < CP_SR ? t - r0 : CP_SR);
    __shared__ double Cs[CP_SR * CP_LD];
    __shared__ double Ws[CP_K * CP_LD];
    const int tid = threadIdx.x, lane = tid & 63, wv = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int i16 = lane & 15, k4 = lane >> 4;
    {  // the slab (column by column: coalesced rows) and W1, all loads before the stores
        double v[16], w[16];
#pragma unroll
        for (int u = 0; u < 16; ++u) {
            const int e = tid + 256 * u, c = e >> 6, r = e & 63;
            v[u] = (c < l && r < nr) ? a.A[(ns + c) * a.lda + ns + r0 + r] : 0.0;
            w[u] = cp[CP_OFF_W1 + e];
        }
#pragma unroll
        for (int u = 0; u < 16; ++u) {
            const int e = tid + 256 * u, c = e >> 6, r = e & 63;
            Cs[r * CP_LD + c] = v[u];
            Ws[c * CP_LD + r] = w[u];  // W1 row c, column r (W1 is stored by rows)
        }
    }
    __syncthreads();
    dbl4 acc[4];
    cp_slab_upper(Cs, Ws, acc);
    __syncthreads();  // every MFMA has read Cs: it now takes Q1
#pragma unroll
    for (int ct = 0; ct < 4; ++ct) {
#pragma unroll
        for (int v = 0; v < 4; ++v) Cs[(16 * wv + 4 * v + k4) * CP_LD + 16 * ct + i16] = acc[ct][v];
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < 16; ++u) {
        const int e = tid + 256 * u, c = e >> 6, r = e & 63;
        const double q = Cs[r * CP_LD + c];
        if (c < l && r < nr) Vw[(int64_t)c * ldv + r0 + r] = q;
    }
    // the slab's Q1^T Q1 (rows past nr are zero): tile d-th diagonal order,
    // wavefront w taking tiles w, w + 4, w + 8 of (0,0) (1,1) (2,2) (3,3) (0,1)
    // (1,2) (2,3) (0,2) (1,3) (0,3)
    double *out = Gp + (int64_t)blockIdx.x * kp * kp;
#pragma unroll
    for (int u = 0; u < 3; ++u) {
        const int idx = wv + 4 * u;
        if (idx < 10) {
            const int d = idx < 4 ? 0 : (idx < 7 ? 1 : (idx < 9 ? 2 : 3));
            const int ti = idx - (d == 0 ? 0 : (d == 1 ? 4 : (d == 2 ? 7 : 9))), tj = ti + d;
            double av[16], bv[16];
#pragma unroll
            for (int kk = 0; kk < 16; ++kk) {
                av[kk] = Cs[(4 * kk + k4) * CP_LD + 16 * ti + i16];
                bv[kk] = Cs[(4 * kk + k4) * CP_LD + 16 * tj + i16];
            }
            dbl4 g = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
            for (int kk = 0; kk < 16; ++kk) g = cp_mfma(av[kk], bv[kk], g);
            if (16 * tj < kp) {
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    out[(16 * ti + 4 * v + k4) * kp + 16 * tj + i16] = g[v];
                    if (d) out[(16 * tj + i16) * kp + 16 * ti + 4 * v + k4] = g[v];
                }
            }
        }
    }
}

hipError_t launch_cpanel1(QrdmArgs a, const double *cp, double *Vw, int64_t ldv, double *Gp, int kp, int64_t t_bound,
                          hipStream_t s) {
    if (t_bound <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_cpanel1, dim3((unsigned)((t_bound + CP_SR - 1) / CP_SR)), dim3(256), 0, s, a, cp, Vw, ldv,
                       Gp, kp);
    return hipGetLastError();
}

int cpanel_partials(int64_t m) { return (int)((m + CP_SR - 1) / CP_SR); }

// ------------------------------------------------------------------ k_cpreduce
__global__ void __launch_bounds__(256) k_cpreduce(QrdmArgs a, const double *Gp, int kp, double *cp) {
    const QrdmCtl *ctl = a.ctl;
    if (qrdm_dm_idle(ctl) || !ctl->cpath) return;
    const int l = ctl->l;
    const int64_t t = a.m - ctl->ns;
    const int np = (int)((t + CP_SR - 1) / CP_SR);
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
// C = A B for 64 x 64 operands on FP64 MFMA by the four wavefronts, fa(i, k)
// and fb(k, j) giving the operands, out(i, j, v) taking each result.  Only the
// products the triangular shapes leave are formed: MODE 1 (B upper
// triangular): every 16 x 16 tile, tile (rt, ct) summing the k-tiles up to ct,
// row tile rt on wavefront rt; MODE 2 (A and B upper triangular): the ten
// tiles on and above the diagonal, k-tiles rt .. ct, five k-tiles per
// wavefront.  A tile's operands for one k-tile are loaded before its MFMAs.
// With TWO, a second product of the same shape (fa2, fb2, out2) is formed
// beside the first, tile for tile, so that the two accumulation chains
// overlap; each tile is summed exactly as it would be alone.
template <int MODE, bool TWO, typename FA, typename FB, typename OUT, typename FA2, typename FB2, typename OUT2>
__device__ __forceinline__ void cp_mm_n(FA fa, FB fb, OUT out, FA2 fa2, FB2 fb2, OUT2 out2) {
    const int lane = threadIdx.x & 63, wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int i16 = lane & 15, k4 = lane >> 4;
    // MODE 2: the tiles (4 rt + ct, plus one; 0 = none) of each wavefront, five bits each
    const uint32_t pk = wv == 0 ? (4u | 1u << 5) : wv == 1 ? (3u | 2u << 5) : wv == 2 ? (8u | 7u << 5)
                                                                                : (12u | 6u << 5 | 11u << 10 | 16u << 15);
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        const int t = MODE == 1 ? 4 * wv + u : (int)((pk >> (5 * u)) & 31u) - 1;
        if (t < 0) break;
        const int rt = t >> 2, ct = t & 3, k0 = MODE == 2 ? rt : 0;
        dbl4 acc = {0.0, 0.0, 0.0, 0.0}, acc2 = {0.0, 0.0, 0.0, 0.0};
        for (int kt = k0; kt <= ct; ++kt) {
            double av[4], bv[4], av2[4], bv2[4];
#pragma unroll
            for (int kb = 0; kb < 4; ++kb) {
                av[kb] = fa(rt * 16 + i16, kt * 16 + 4 * kb + k4);
                bv[kb] = fb(kt * 16 + 4 * kb + k4, ct * 16 + i16);
                av2[kb] = TWO ? fa2(rt * 16 + i16, kt * 16 + 4 * kb + k4) : 0.0;
                bv2[kb] = TWO ? fb2(kt * 16 + 4 * kb + k4, ct * 16 + i16) : 0.0;
            }
#pragma unroll
            for (int kb = 0; kb < 4; ++kb) {
                acc = cp_mfma(av[kb], bv[kb], acc);
                if (TWO) acc2 = cp_mfma(av2[kb], bv2[kb], acc2);
            }
        }
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            out(rt * 16 + 4 * v + k4, ct * 16 + i16, acc[v]);
            if (TWO) out2(rt * 16 + 4 * v + k4, ct * 16 + i16, acc2[v]);
        }
    }
}

template <int MODE, typename FA, typename FB, typename OUT>
__device__ __forceinline__ void cp_mm(FA fa, FB fb, OUT out) {
    cp_mm_n<MODE, false>(fa, fb, out, fa, fb, out);
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
    double *Tmp = A4 + CP_K * CP_LD;  // eight 16 x CP_LD16 blocks for the two triangular inverses
    const int i16 = lane & 15, k4 = lane >> 4;
    __shared__ double sS[CP_K], sUd[CP_K], sUi[CP_K], s_red[4];
    double *Tg = cp + CP_OFF_T, *Pg = cp + CP_OFF_P;
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
        // every entry of A1, A2 and A3 is written (zero outside the block)
#pragma unroll
        for (int u = 0; u < 16; ++u) {
            const int e = tid + 256 * u, i = e >> 6, c = e & 63;
            const double v = (i < l && c < l) ? g[u] - (i == c ? 1.0 : 0.0) : 0.0;
            emax = fmax(emax, fabs(v));
            A2[i * CP_LD + c] = i < c ? v : (i == c ? 0.5 * v : 0.0);
            A3[c * CP_LD + i] = q[u];
            A1[i * CP_LD + c] = r1[u];
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
    cp_mm<1>([&](int i, int k) { return A3[i * CP_LD + k]; }, [&](int k, int j) { return A2[k * CP_LD + j]; },
          [&](int i, int j, double v) { A4[i * CP_LD + j] = A3[i * CP_LD + j] - v; });
    __syncthreads();
    cp_mm<2>([&](int i, int k) { return A2[i * CP_LD + k]; }, [&](int k, int j) { return A1[k * CP_LD + j]; },
          [&](int i, int j, double v) {
              const double r1 = A1[i * CP_LD + j];
              A3[i * CP_LD + j] = (i <= j) ? r1 + v : 0.0;
          });
    __syncthreads();
    // ---- LU of I - Q_top S, the signs chosen on the way, in W = Q_top: pivot j
    // is U_jj = 1 + |dq_j| with dq_j = W_jj after j steps and S_j = -sign(dq_j),
    // L_rj = -S_j W_rj / U_jj, W_rc -= L_rj W_jc (r, c > j).  Blocked by 16:
    // (a) the panel on wavefront 0, lane r holding W_r,panel; (b) the panel's
    // rows right of it, by forward substitution with the unit L_11; (c) the
    // trailing block, W_22 -= L_21 W_12, on MFMA.  A4 ends as L below the
    // diagonal, dq on it and W (the Y of U_rc = -S_c Y_rc) above.
#pragma unroll 1
    for (int kb = 0; kb < 4; ++kb) {
        const int j0 = 16 * kb;
        if (j0 >= l) break;
        if (wv == 0) {
            double p[16];
#pragma unroll
            for (int c = 0; c < 16; ++c) p[c] = A4[lane * CP_LD + j0 + c];
            // the steps past l run too, as no-ops (m = 0, p kept): no branch
            // between the steps
#pragma unroll
            for (int jj = 0; jj < 16; ++jj) {
                const int j = j0 + jj;
                const bool act = (j < l) & (lane > j);
                const double dq = cp_readlane(p[jj], j);
                const double sj = dq >= 0.0 ? -1.0 : 1.0;
                const double f = -sj * cp_rcp(1.0 - sj * dq);
                const double m = act ? f * p[jj] : 0.0;  // zero on the finished rows
#pragma unroll
                for (int c = jj + 1; c < 16; ++c) p[c] -= m * cp_readlane(p[c], j);
                p[jj] = act ? m : p[jj];
            }
            if (lane >= j0) {
#pragma unroll
                for (int c = 0; c < 16; ++c) A4[lane * CP_LD + j0 + c] = p[c];
            }
        }
        __syncthreads();
        if (wv == 0) {
            const int c = j0 + 16 + lane;
            if (c < CP_K) {
                double x[16];
#pragma unroll
                for (int ii = 0; ii < 16; ++ii) x[ii] = A4[(j0 + ii) * CP_LD + c];
#pragma unroll
                for (int ii = 1; ii < 16; ++ii) {
                    double lv[16];
#pragma unroll
                    for (int jj = 0; jj < ii; ++jj) lv[jj] = A4[(j0 + ii) * CP_LD + j0 + jj];
                    double sum = x[ii];
#pragma unroll
                    for (int jj = 0; jj < ii; ++jj) sum -= lv[jj] * x[jj];
                    x[ii] = sum;
                }
#pragma unroll
                for (int ii = 1; ii < 16; ++ii) A4[(j0 + ii) * CP_LD + c] = x[ii];
            }
        }
        __syncthreads();
        {
            const int nt = 3 - kb;
            for (int tile = wv; tile < nt * nt; tile += 4) {
                const int rt = kb + 1 + tile / nt, ct = kb + 1 + tile % nt;
                const dbl4 acc = cp_mm16([&](int i, int k) { return A4[(16 * rt + i) * CP_LD + j0 + k]; },
                                         [&](int k, int j) { return A4[(j0 + k) * CP_LD + 16 * ct + j]; },
                                         dbl4{0.0, 0.0, 0.0, 0.0});
#pragma unroll
                for (int v = 0; v < 4; ++v) A4[(16 * rt + 4 * v + k4) * CP_LD + 16 * ct + i16] -= acc[v];
            }
        }
        __syncthreads();
    }
    if (tid < l) {  // the signs and pivots, from dq on the diagonal of the LU
        const double dq = A4[tid * CP_LD + tid];
        const double sj = dq >= 0.0 ? -1.0 : 1.0;
        const double ujj = 1.0 - sj * dq;
        sS[tid] = sj;
        sUd[tid] = ujj;
        sUi[tid] = 1.0 / ujj;
    }
    __syncthreads();
    // ---- Uinv = U^{-1} into A1 (U_ik = -S_k Y_ik, U_ii = 1 + |dq_i|; A1's R1 is no
    // longer needed) and Linv = L^{-1} into A2 below the diagonal, as the
    // inverse of the unit upper L^T (A2 keeps N above)
    // (the accessors load first and select after: their addresses are always in range)
    cp_trinv_n<true>(
          [&](int i, int k) { const double y = A4[i * CP_LD + k], sk = sS[k]; return k < l ? -sk * y : 0.0; },
          [&](int i) { const double v = sUi[i]; return i < l ? v : 1.0; },
          [&](int i, int j) { return A1[i * CP_LD + j]; },
          [&](int i, int j, double v) { A1[i * CP_LD + j] = v; },
          [&](int i, int k) { const double v = A4[k * CP_LD + i]; return k < l ? v : 0.0; },
          [&](int) { return 1.0; },
          [&](int i, int j) { const double v = A2[j * CP_LD + i]; return i < j ? v : (i == j ? 1.0 : 0.0); },
          [&](int i, int j, double v) {
              if (i < j) A2[j * CP_LD + i] = v;
          },
          Tmp);
    // ---- T = U Linv^T and P = -(I - N) S Uinv.  A block that reaches the last
    // row (t = l) ends with a column of one row: larfg leaves it alone (tau = 0,
    // beta = alpha), where the reconstruction reflects it (tau = 2, v = e); its
    // column of T and tau are zeroed and its diagonal entry takes the other sign.
    const bool lastrow = (a.m - ns) == (int64_t)l;
    auto uval = [&](int i, int k) -> double {
        const double y = A4[i * CP_LD + k], sk = sS[k], ud = sUd[i];  // loads first, then selects
        return (i >= l || k >= l || k < i) ? 0.0 : (k == i ? ud : -sk * y);
    };
    cp_mm_n<2, true>(
          uval,
          [&](int k, int j) {
              const double v = A2[j * CP_LD + k];
              return (j >= l || k >= l) ? 0.0 : (j == k ? 1.0 : (j > k ? v : 0.0));
          },
          [&](int i, int j, double v) {
              if (i < l && j < l && !(lastrow && j == l - 1)) Tg[i * CP_K + j] = v;
          },
          [&](int i, int k) {
              const double n = A2[i * CP_LD + k], sk = sS[k];
              return (i >= l || k >= l || k < i) ? 0.0 : (k == i ? -(1.0 - n) * sk : n * sk);
          },
          [&](int k, int j) { return A1[k * CP_LD + j]; },
          [&](int i, int j, double v) {
              if (i < l && j < l) Pg[i * CP_K + j] = v;
          });
    // ---- the top block of A (R_H = S R above, L below), V_top, tau
#pragma unroll
    for (int u = 0; u < 16; ++u) {  // row i of column c, i fastest: each column's rows are contiguous
        const int e = tid + 256 * u, c = e >> 6, i = e & 63;
        const double r = A3[i * CP_LD + c], lw = A4[i * CP_LD + c], si = sS[i];
        if (i < l && c < l) {
            const double flip = (lastrow && i == l - 1) ? -1.0 : 1.0;
            a.A[(ns + c) * a.lda + ns + i] = (i <= c) ? flip * si * r : lw;
            const double v = (i > c) ? lw : (i == c ? 1.0 : 0.0);
            Vo[(int64_t)c * ldv + i] = v;
            if (Vo32) Vo32[(int64_t)c * ldv + i] = (float)v;
        }
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
    const unsigned lds = (4 * CP_K * CP_LD + 8 * 16 * CP_LD16) * sizeof(double);
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
// Slab s: rows [64 s, 64 s + 64) of the block past its top l rows: V = Q1 P,
// written to A (below the top block) and, in place of Q1, to the V staging
// buffer (and its FP32 copy in mixed precision).
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(1, 1)))
k_cpanel3(QrdmArgs a, const double *cp, double *Vw, int64_t ldv, float *Vw32) {
    const QrdmCtl *ctl = a.ctl;
    if (qrdm_dm_idle(ctl) || !ctl->cpath) return;
    const int64_t ns = ctl->ns, t = a.m - ns;
    const int l = ctl->l;
    const int64_t r0 = (int64_t)blockIdx.x * CP_SR;
    if (r0 >= t) return;
    const int nr = (int)(t - r0 < CP_SR ? t - r0 : CP_SR);
    const int rlo = r0 < l ? (int)(l - r0) : 0;  // rows of the top block (written by k_cpanel2)
    if (rlo >= nr) return;
    __shared__ double Qs[CP_SR * CP_LD];
    __shared__ double Ps[CP_K * CP_LD];
    const int tid = threadIdx.x, lane = tid & 63, wv = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int i16 = lane & 15, k4 = lane >> 4;
    {
        double v[16], w[16];
#pragma unroll
        for (int u = 0; u < 16; ++u) {
            const int e = tid + 256 * u, c = e >> 6, r = e & 63;
            v[u] = (c < l && r >= rlo && r < nr) ? Vw[(int64_t)c * ldv + r0 + r] : 0.0;
            w[u] = cp[CP_OFF_P + e];
        }
#pragma unroll
        for (int u = 0; u < 16; ++u) {
            const int e = tid + 256 * u, c = e >> 6, r = e & 63;
            Qs[r * CP_LD + c] = v[u];
            Ps[c * CP_LD + r] = w[u];  // P row c, column r (P is stored by rows)
        }
    }
    __syncthreads();
    dbl4 acc[4];
    cp_slab_upper(Qs, Ps, acc);
    __syncthreads();
#pragma unroll
    for (int ct = 0; ct < 4; ++ct) {
#pragma unroll
        for (int v = 0; v < 4; ++v) Qs[(16 * wv + 4 * v + k4) * CP_LD + 16 * ct + i16] = acc[ct][v];
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < 16; ++u) {
        const int e = tid + 256 * u, c = e >> 6, r = e & 63;
        const double v = Qs[r * CP_LD + c];
        if (c < l && r >= rlo && r < nr) {
            a.A[(ns + c) * a.lda + ns + r0 + r] = v;
            Vw[(int64_t)c * ldv + r0 + r] = v;
            if (Vw32) Vw32[(int64_t)c * ldv + r0 + r] = (float)v;
        }
    }
}

hipError_t launch_cpanel3(QrdmArgs a, const double *cp, double *Vw, int64_t ldv, float *Vw32, int64_t t_bound,
                          hipStream_t s) {
    if (t_bound <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_cpanel3, dim3((unsigned)((t_bound + CP_SR - 1) / CP_SR)), dim3(256), 0, s, a, cp, Vw,
                       ldv, Vw32);
    return hipGetLastError();
}
