// Block trailing update of QRDM (Algorithm 4 of the paper, the BLAS-3 step;
// compact WY form of Section 3.2).  With the l kept reflectors written as
// H_0...H_{l-1} = I - V T V^T (forward accumulation),
//     A_tr <- (I - V T V^T)^T A_tr = A_tr - V Z,   Z = T^T (V^T A_tr),
// A_tr = A[n_s:m, n_s+c0:n], c0 = k_s (or l when the panel came from the Gram
// matrix: the rejected columns of the block take the update too).  Three
// kernels on gfx950 MFMA:
//   k_gemm1  Y = V^T A_tr, split over rows, partial products published;
//   k_zsum   per 32 or 64 trailing columns: Y = the sum of the partials in split
//            order, then Z = T^T Y.  For l <= 64, T is formed explicitly (the
//            Gram-matrix panel provides it; otherwise from the v_b^T v_a the
//            column panel records: 16 x 16 diagonal blocks by the larft column
//            recurrence, T_12 = -T_11 (V_1^T V_2) T_22 for the halves) and Z is
//            a product on FP64 MFMA.  For larger blocks, with
//            T^{-1} = diag(1/tau) + strict_upper(V^T V), Z solves the lower
//            recurrence Z_a = tau_a (Y_a - sum_{b<a} (v_b^T v_a) Z_b) (Z_a = 0
//            when tau_a = 0, the identity reflector);
//   k_gemm2  A_tr -= V Z on 128 x 128 tiles, A read once and written once;
//            for FP64 blocks of at most 64 reflectors the persistent k_gemm2p
//            (one workgroup per compute unit, V and Z of a tile whole in LDS,
//            the next tile's A and Z loaded during the current tile's MFMAs).
// Precision: FP64 MFMA (16x16x4 f64) by default; mixed mode runs both products
// on FP32 MFMA with FP32 accumulation while A stays FP64 in memory and Z is
// formed in FP64.
#include "qrdm_internal.h"

#define QK_SPLIT_MAX 16  // row splits of the V^T A product

typedef double dbl4 __attribute__((ext_vector_type(4)));
typedef float flt4 __attribute__((ext_vector_type(4)));

// Operand layouts of both 16x16x4 instructions: A[i][k] in lane i + 16k, B[k][j]
// in lane j + 16k.  Result layouts differ: register v of a lane holds
// D[4v + lane/16][lane%16] for f64 and D[4(lane/16) + v][lane%16] for f32.
template <typename T> struct Mfma;
template <> struct Mfma<double> {
    typedef dbl4 acc_t;
    static __device__ __forceinline__ acc_t op(double a, double b, acc_t c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ int row(int lane, int v) { return 4 * v + (lane >> 4); }
};
template <> struct Mfma<float> {
    typedef flt4 acc_t;
    static __device__ __forceinline__ acc_t op(float a, float b, acc_t c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ int row(int lane, int v) { return 4 * (lane >> 4) + v; }
};

// ------------------------------------------------------------------ GEMM1
#ifndef G1_NT
#define G1_NT 256   // trailing columns per workgroup (V reused across them): 128 or 256
#endif
#ifndef G1_TARGET_WGS
#define G1_TARGET_WGS 512  // split count aims at this many workgroups (two per compute unit)
#endif
#ifndef G1_KC
#define G1_KC 16    // rows staged per step: 16 or 32 (16: 120 VGPRs and 44 KB of LDS, two workgroups per CU)
#endif
#define G1_MINROWS 128  // rows of a split at least
#define G1_TH 512   // threads: 8 wavefronts, G1_NT / 8 columns each
#define G1_CT (G1_NT / 128)  // 16-column tiles per wavefront
#define G1_CPP (G1_TH / G1_KC)          // columns staged per pass (one thread per row of a column)
#define G1_AU (G1_NT / G1_CPP)          // staged A elements per thread per step
#define G1_VU (64 / G1_CPP)             // staged V elements per thread per step
#ifndef G1_PAD
#define G1_PAD 1    // LDS row padding of the staged tiles (doubles)
#endif
#define G1_LD (G1_KC + G1_PAD)

__device__ __forceinline__ void st_coh(double *p, double v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ double ld_coh(const double *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// The split of GEMM1's row range, from the actual trailing sizes (t rows, w
// columns) alone, so that the bits of the result do not depend on the launch
// bounds the host passes: at most G1_TARGET_WGS workgroups (one wave over the
// compute units: one more split past it would start a second wave), at most
// QK_SPLIT_MAX splits of at least G1_MINROWS rows, krows a multiple of G1_KC.  Both
// GEMM1 and the partial sum in k_zsum take it from here.
__device__ __forceinline__ int g1_krows(int64_t t, int64_t w) {
    const int ntile = (int)((w + G1_NT - 1) / G1_NT);
    int ns = G1_TARGET_WGS / ntile;
    if (ns > QK_SPLIT_MAX) ns = QK_SPLIT_MAX;
    const int64_t maxs = (t + G1_MINROWS - 1) / G1_MINROWS;
    if (ns > maxs) ns = (int)maxs;
    if (ns < 1) ns = 1;
    return (int)(((t + ns - 1) / ns + G1_KC - 1) / G1_KC * G1_KC);
}

// Split-K: workgroup (x, y, z) forms rows [64z, 64z+64) of the partial
// Y_y = V^T A_tr over rows [y*krows, (y+1)*krows) of A_tr, for trailing columns
// [256x, 256x+256), and writes it to Yp[y] (k_zsum, the next launch, sums them).
template <typename T>
__global__ void __launch_bounds__(G1_TH)
k_gemm1(QrdmArgs a, const T *__restrict__ V, int64_t ldv, double *Yp, int64_t ldz, int64_t ysplit) {
    QrdmCtl *ctl = a.ctl;
    if (qrdm_dm_idle(ctl)) return;
    const int64_t ns = ctl->ns;
    const int l = ctl->l;
    const int64_t t = a.m - ns;
    const int64_t c0 = ns + ctl->c0off;  // k_s, or l after the Gram-matrix panel
    const int64_t w2 = a.n - c0;
    const int64_t jb = (int64_t)blockIdx.x * G1_NT;
    if (l <= 0 || jb >= w2 || t <= 0) return;
    const int krows = g1_krows(t, w2);
    const int nsplit = (int)((t + krows - 1) / krows);
    const int lt = (l + 15) >> 4;
    const int nz = (lt + 3) >> 2;
    const int sp = blockIdx.y, zg = blockIdx.z;
    if (blockIdx.x == 0 && sp == 0 && zg == 0 && threadIdx.x == 0) {
        ctl->flop_gemm += 2.0 * (double)t * (double)l * (double)w2;
        ctl->bytes_gemm2 += 16.0 * (double)t * (double)w2;
        if (nsplit > (int)gridDim.y) atomicOr(&ctl->error, 4);  // a split without a workgroup
    }
    if (sp >= nsplit || zg >= nz) return;
    const int64_t rb = (int64_t)sp * krows;
    const int64_t re = (rb + krows < t) ? rb + krows : t;
    const int q0 = 64 * zg;                 // first reflector of this row group
    const int ltz = (lt - 4 * zg) < 4 ? (lt - 4 * zg) : 4;
    extern __shared__ double g1_lds[];
    T *Vs = reinterpret_cast<T *>(g1_lds);  // [64][G1_LD]
    T *As = Vs + 64 * G1_LD;                // [G1_NT][G1_LD]
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    typedef typename Mfma<T>::acc_t acc_t;
    acc_t acc[4 * G1_CT];  // 4 row tiles x G1_CT column tiles
#pragma unroll
    for (int u = 0; u < 4 * G1_CT; ++u) acc[u] = acc_t{0, 0, 0, 0};
    const int ncols = (int)((w2 - jb) < G1_NT ? (w2 - jb) : G1_NT);
    const double *Abase = a.A + (c0 + jb) * a.lda + ns;
    // staged element u*512 + tid: row r = tid % G1_KC, column/reflector q = u*G1_CPP + tid/G1_KC
    const int rr = tid % G1_KC, qq = tid / G1_KC;
    // A is staged in registers as loaded (FP64) and rounded to T only when it is
    // written to LDS, so the loads of a chunk stay in flight during the MFMAs
    T vreg[G1_VU];
    double areg[G1_AU];
    auto fetch = [&](int64_t rc) {
        const int64_t row = rc + rr;
        const bool rok = row < re;
#pragma unroll
        for (int u = 0; u < G1_VU; ++u) {
            const int q = q0 + u * G1_CPP + qq;
            vreg[u] = (rok && q < l) ? V[(int64_t)q * ldv + row] : (T)0;
        }
#pragma unroll
        for (int u = 0; u < G1_AU; ++u) {
            const int q = u * G1_CPP + qq;
            areg[u] = (rok && q < ncols) ? Abase[(int64_t)q * a.lda + row] : 0.0;
        }
    };
    fetch(rb);
    for (int64_t rc = rb; rc < re; rc += G1_KC) {
        __syncthreads();
#pragma unroll
        for (int u = 0; u < G1_VU; ++u) Vs[(u * G1_CPP + qq) * G1_LD + rr] = vreg[u];
#pragma unroll
        for (int u = 0; u < G1_AU; ++u) As[(u * G1_CPP + qq) * G1_LD + rr] = (T)areg[u];
        __syncthreads();
        if (rc + G1_KC < re) fetch(rc + G1_KC);
        // wave wv owns columns [16 G1_CT wv, 16 G1_CT (wv + 1)): G1_CT column tiles x ltz row tiles
#pragma unroll
        for (int k = 0; k < G1_KC; k += 4) {
            T bcol[G1_CT];
#pragma unroll
            for (int c = 0; c < G1_CT; ++c)
                bcol[c] = As[(wv * 16 * G1_CT + c * 16 + (lane & 15)) * G1_LD + k + (lane >> 4)];
            // FP32: all four row tiles without a branch per tile (the V rows past
            // l are staged as zeros; only the tiles below ltz are stored), which
            // keeps the FP32 accumulators in place; FP64 skips the empty tiles
#pragma unroll
            for (int ti = 0; ti < 4; ++ti) {
                if (sizeof(T) == 4 || ti < ltz) {
                    const T av = Vs[(ti * 16 + (lane & 15)) * G1_LD + k + (lane >> 4)];
#pragma unroll
                    for (int c = 0; c < G1_CT; ++c)
                        acc[ti * G1_CT + c] = Mfma<T>::op(av, bcol[c], acc[ti * G1_CT + c]);
                }
            }
        }
    }
    // the partial: Yp[sp][q0 + row][jb + col] (double)
    double *yp = Yp + (int64_t)sp * ysplit + (int64_t)q0 * ldz;
#pragma unroll
    for (int ti = 0; ti < 4; ++ti) {
        if (ti < ltz) {
#pragma unroll
            for (int c = 0; c < G1_CT; ++c) {
                const int64_t col = jb + wv * 16 * G1_CT + c * 16 + (lane & 15);
                if (col < w2) {
#pragma unroll
                    for (int v = 0; v < 4; ++v)
                        yp[(ti * 16 + Mfma<T>::row(lane, v)) * ldz + col] = (double)acc[ti * G1_CT + c][v];
                }
            }
        }
    }
}

#define ZS_LDY 72  // row stride of the staged Y: the 8 lanes of a column group and the 8
                   // column groups of a wavefront fall on distinct LDS banks

// One step of the recurrence for the column of lanes g = 0..7: the products
// (v_b^T v_aa) Z_b, b = g, g + 8, ... < aa, loaded together, summed in increasing b.
template <int NU>
__device__ __forceinline__ double zs_step(const double *vc, const double *Ys, int aa, int g, int jl) {
    double x[NU], y[NU];
#pragma unroll
    for (int u = 0; u < NU; ++u) {
        const int b = g + 8 * u;
        const bool in = b < aa;
        x[u] = in ? vc[b] : 0.0;
        y[u] = in ? Ys[b * ZS_LDY + jl] : 0.0;
    }
    double part = 0.0;
#pragma unroll
    for (int u = 0; u < NU; ++u)
        if (g + 8 * u < aa) part += x[u] * y[u];
    return part;
}

#define ZT_LD 80  // row stride of T, V^T V and Y on the explicit-T path: the four K
                  // rows of an MFMA operand fall on distinct LDS bank halves

// Z = T^T Y for l <= 64 reflectors with the forward triangular factor T of
// H_0 ... H_{l-1} = I - V T V^T (Section 3.2), formed blockwise: 16 x 16
// diagonal blocks by the column recurrence T_{r,i} = -tau_i sum_{r<=b<i} T_{r,b}
// (v_b^T v_i), T_ii = tau_i (one lane per row), then
// T_12 = -T_11 (V_1^T V_2) T_22 for 16- and 32-column halves.  Reflectors
// a >= l have tau = 0 and vanish.  Z on FP64 MFMA (16x16x4): A = T^T, B = Y.
__device__ __forceinline__ void zs_tmat(const double *VVf, double *Tm, double *Mt, const double *taus) {
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    // diagonal blocks: wavefront w < 4 forms rows/columns [16w, 16w + 16), lane
    // r holding its row in registers; column i's v_b^T v_i are the same in
    // every lane and are read before the row's recurrence uses them
    if (wv < 4 && lane < 16) {
        const int base = 16 * wv, r = lane;
        double tr[16];
#pragma unroll
        for (int i = 0; i < 16; ++i) tr[i] = 0.0;
#pragma unroll
        for (int i = 0; i < 16; ++i) {
            const int ia = base + i;
            double vc[16];
#pragma unroll
            for (int b = 0; b < 16; ++b) vc[b] = b < i ? VVf[(base + b) * ZT_LD + ia] : 0.0;
            if (r < i) {
                double x = 0.0;
#pragma unroll
                for (int b = 0; b < 16; ++b)
                    if (b >= r && b < i) x += tr[b] * vc[b];
                tr[i] = -taus[ia] * x;
            } else if (r == i) {
                tr[i] = taus[ia];
            }
        }
        double *trow = Tm + (base + r) * ZT_LD + base;
#pragma unroll
        for (int i = 0; i < 16; ++i)
            if (i >= r) trow[i] = tr[i];
    }
    __syncthreads();
    for (int sh = 16; sh < 64; sh *= 2) {
        // pairs (r1, r2) = ([2 sh p, 2 sh p + sh), [2 sh p + sh, 2 sh (p + 1))): M = (V_1^T V_2) T_22
        const int np = 64 / (2 * sh), nout = np * sh * sh;
        for (int e = tid; e < nout; e += G1_TH) {
            const int p = e / (sh * sh), x = (e / sh) % sh, y = e % sh;
            const int r1 = 2 * sh * p, r2 = r1 + sh;
            double m = 0.0;
            for (int z = 0; z < sh; ++z)
                if (z <= y) m += VVf[(r1 + x) * ZT_LD + r2 + z] * Tm[(r2 + z) * ZT_LD + r2 + y];
            Mt[(r1 + x) * ZT_LD + r2 + y] = m;
        }
        __syncthreads();
        // T_12 = -T_11 M
        for (int e = tid; e < nout; e += G1_TH) {
            const int p = e / (sh * sh), x = (e / sh) % sh, y = e % sh;
            const int r1 = 2 * sh * p, r2 = r1 + sh;
            double v = 0.0;
            for (int z = 0; z < sh; ++z)
                if (z >= x) v += Tm[(r1 + x) * ZT_LD + r1 + z] * Mt[(r1 + z) * ZT_LD + r2 + y];
            Tm[(r1 + x) * ZT_LD + r2 + y] = -v;
        }
        __syncthreads();
    }
}

template <typename T, int CW>
__device__ __forceinline__ void zs_apply(const double *Ys, const double *Tm, int l, int ncols, T *__restrict__ Z,
                                         int64_t ldz, int64_t cb) {
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    // Z = T^T Y over 4 x (CW / 16) output tiles: wavefront w takes tiles
    // CW/32 w .. CW/32 w + CW/32 - 1 (two for 64 columns, one for 32)
    constexpr int TW = CW / 16, PER = CW / 32;
#pragma unroll
    for (int h = 0; h < PER; ++h) {
        const int q = PER * wv + h, ta = q / TW, tj = q % TW;
        dbl4 acc = {0.0, 0.0, 0.0, 0.0};
        const int i = lane & 15, k = lane >> 4;
        for (int kb = 0; kb < 16 * ta + 16; kb += 4) {  // T_{b,a} = 0 for b > a
            const double av = Tm[(kb + k) * ZT_LD + 16 * ta + i];
            const double bv = Ys[(kb + k) * ZT_LD + 16 * tj + i];
            acc = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, acc, 0, 0, 0);
        }
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int aa = 16 * ta + 4 * v + k, j = 16 * tj + i;
            if (aa < l && j < ncols) Z[(int64_t)aa * ldz + cb + j] = (T)acc[v];
        }
    }
}

// Z for CW trailing columns per workgroup: Y = the k_gemm1 partials summed in
// split order, then Z = T^T Y (l <= 64, explicit T) or the recurrence
// Z_a = tau_a (Y_a - sum_{b<a} (v_b^T v_a) Z_b) per column (Z_a = 0 when tau_a = 0).
template <typename T, int CW>
__global__ void __launch_bounds__(G1_TH)
k_zsum(QrdmArgs a, const double *__restrict__ VV, const double *__restrict__ cpT, const double *__restrict__ Yp,
       T *__restrict__ Z, int64_t ldz, int64_t ysplit) {
    QrdmCtl *ctl = a.ctl;
    if (qrdm_dm_idle(ctl)) return;
    const int64_t ns = ctl->ns;
    const int l = ctl->l;
    const bool tgiven = ctl->cpath != 0;  // T formed by the Gram-matrix panel
    const int64_t t = a.m - ns;
    const int64_t w2 = a.n - (ns + ctl->c0off);
    const int64_t cb = (int64_t)blockIdx.x * CW;
    if (l <= 0 || cb >= w2 || t <= 0) return;
    const int krows = g1_krows(t, w2);
    const int nsplit = (int)((t + krows - 1) / krows);
    const int ncols = (int)((w2 - cb) < CW ? (w2 - cb) : CW);
    const int tid = threadIdx.x;
    const int lp = ((l + 15) >> 4) * 16;
    const bool xt = l <= 64;  // explicit-T path
    if (CW != 64 && !xt) {    // the recurrence takes 64 columns (the host picks CW from kmax)
        if (blockIdx.x == 0 && tid == 0) atomicOr(&ctl->error, 4);
        return;
    }
    const int ldy = xt ? ZT_LD : ZS_LDY;
    extern __shared__ double zs_lds[];
    double *Ys = zs_lds;                           // [lp][ldy]
    double *VVs = Ys + lp * ldy;                   // recurrence: packed strict upper triangle
    double *taus = VVs + (lp * (lp - 1)) / 2 + 1;  // [lp]
    double *VVf = Ys + 64 * ZT_LD;                 // explicit T: [64][ZT_LD] v_b^T v_a (b < a)
    double *Tm = VVf + 64 * ZT_LD;                 // [64][ZT_LD]
    double *taux = Tm + 64 * ZT_LD;                // [64]
    if (xt && tgiven) {
        for (int e = tid; e < 64 * ZT_LD; e += G1_TH) {
            const int b = e / ZT_LD, aa = e - b * ZT_LD;
            Tm[e] = (b <= aa && aa < l) ? cpT[b * 64 + aa] : 0.0;
        }
        __syncthreads();
    } else if (xt) {
        for (int e = tid; e < 64 * ZT_LD; e += G1_TH) {
            const int b = e / ZT_LD, aa = e - b * ZT_LD;
            VVf[e] = (b < aa && aa < l) ? VV[b * QK_KM + aa] : 0.0;
            Tm[e] = 0.0;
        }
        for (int e = tid; e < 64; e += G1_TH) taux[e] = e < l ? a.tau_house[ns + e] : 0.0;
        __syncthreads();
        zs_tmat(VVf, Tm, Ys, taux);  // the Y area is the product's scratch until the partials are summed
        __syncthreads();
    } else {
        for (int e = tid; e < l * l; e += G1_TH) {
            const int b = e / l, aa = e - b * l;
            if (b < aa) VVs[aa * (aa - 1) / 2 + b] = VV[b * QK_KM + aa];
        }
        for (int e = tid; e < l; e += G1_TH) taus[e] = a.tau_house[ns + e];
    }
    // every split's partial of an element is loaded before any is summed
    // (QK_SPLIT_MAX loads in flight per element), then summed in split order
    constexpr int CS = CW == 64 ? 6 : 5;  // log2 CW
    for (int e0 = 0; e0 < l * CW; e0 += G1_TH * 2) {
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            const int e = e0 + u * G1_TH + tid;
            const int aa = e >> CS, j = e & (CW - 1);
            const bool ok = e < l * CW && j < ncols;
            double v[QK_SPLIT_MAX];
#pragma unroll
            for (int s2 = 0; s2 < QK_SPLIT_MAX; ++s2)
                v[s2] = (ok && s2 < nsplit) ? Yp[(int64_t)s2 * ysplit + (int64_t)aa * ldz + cb + j] : 0.0;
            double sum = 0.0;
#pragma unroll
            for (int s2 = 0; s2 < QK_SPLIT_MAX; ++s2) sum += v[s2];
            if (e < l * CW) Ys[aa * ldy + j] = sum;
        }
    }
    if (xt) {
        for (int e = l * CW + tid; e < 64 * CW; e += G1_TH) Ys[(e >> CS) * ldy + (e & (CW - 1))] = 0.0;  // rows a >= l
        __syncthreads();
        zs_apply<T, CW>(Ys, Tm, l, ncols, Z, ldz, cb);
        return;
    }
    __syncthreads();
    // 8 lanes of one wavefront per column; the products of a step are loaded
    // together and summed in increasing b
    const int jl = tid >> 3, g = tid & 7;
    for (int aa = 0; aa < l; ++aa) {
        const double *vc = VVs + aa * (aa - 1) / 2;
        double part = l <= 64 ? zs_step<8>(vc, Ys, aa, g, jl) : zs_step<QK_KM / 8>(vc, Ys, aa, g, jl);
        part += __shfl_xor(part, 1, 64);
        part += __shfl_xor(part, 2, 64);
        part += __shfl_xor(part, 4, 64);
        if (g == 0) {
            const double ta = taus[aa];
            Ys[aa * ZS_LDY + jl] = (ta == 0.0) ? 0.0 : ta * (Ys[aa * ZS_LDY + jl] - part);
        }
    }
    __syncthreads();
    for (int e = tid; e < l * 64; e += G1_TH) {
        const int aa = e >> 6, j = e & 63;
        if (j < ncols) Z[(int64_t)aa * ldz + cb + j] = (T)Ys[aa * ZS_LDY + j];
    }
}

// ------------------------------------------------------------------ GEMM2
#define G2_MT 128
#define G2_NT 128
#define G2_KC 16

// A_tr -= V Z on a 128 x 128 tile, computed transposed (D = Z^T V^T) so that a
// lane's accumulator registers map to 16 consecutive rows of 4 columns: every
// load and store instruction touches four whole 128-byte column segments.
// FP64: the accumulators start as the A tile and the MFMAs add (-Z)^T V^T.
// FP32 (mixed): the A tile is prefetched into FP64 registers while the FP32
// product accumulates, then A - (double)acc.
// MODE 0: QRDM block (rows from n_s, columns from n_s + k_s, K = l, Z indexed
// from the first trailing column).  MODE 1: closing a QP3 block (rows and
// columns from last + 1, K = kb, Z = F^T indexed by absolute column).
template <typename T, int MODE>
__global__ void __launch_bounds__(512, sizeof(T) == 8 ? 4 : 1)
k_gemm2(QrdmArgs a, const T *__restrict__ V, int64_t ldv, const T *__restrict__ Z, int64_t ldz) {
    const QrdmCtl *ctl = a.ctl;
    // a DM step's update is idle after the switch to column pivoting; the QP3
    // block end runs exactly then
    if (MODE == 0 ? qrdm_dm_idle(ctl) : (bool)ctl->done) return;
    int64_t r0, c0;
    int l;
    double rpend = 1.0;  // mode 1: the block's last reflector is stored unscaled
    int64_t vk0 = 0;     // mode 1: first column of V in A
    if constexpr (MODE == 0) {
        r0 = ctl->ns;
        c0 = ctl->ns + ctl->c0off;  // k_s, or l after the Gram-matrix panel
        l = ctl->l;
    } else {
        // QP3 block end: same predicate as the column-pivoting kernels
        const int b = ctl->qp_b;
        const bool stop = ctl->qp_stop != 0;
        const int64_t pmin = a.m < a.n ? a.m : a.n;
        if (!(stop || (b + 1 == ctl->qp_nb) || (ctl->ns + 1 == pmin) || ctl->qp_flag)) return;
        l = stop ? b : b + 1;
        const int64_t last = ctl->qp_k0 + l - 1;
        r0 = last + 1;
        c0 = r0;
        Z += c0;
        rpend = 1.0 / ctl->qp_den;
        vk0 = ctl->qp_k0;
    }
    const int64_t ns = r0;
    const int64_t t = a.m - r0;
    const int64_t w2 = a.n - c0;
    const int64_t rb = (int64_t)blockIdx.y * G2_MT;
    const int64_t jb = (int64_t)blockIdx.x * G2_NT;
    if (l <= 0 || rb >= t || jb >= w2) return;
    __shared__ T Vs[G2_KC * G2_MT];  // [k][row]
    __shared__ T Zs[G2_KC * G2_NT];  // [k][col]
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int wr = (wv >> 1) * 32, wc = (wv & 1) * 64;  // wave's 32 x 64 block (rows, cols)
    typedef typename Mfma<T>::acc_t acc_t;
    const int nrow = (int)((t - rb) < G2_MT ? (t - rb) : G2_MT);
    const int ncol = (int)((w2 - jb) < G2_NT ? (w2 - jb) : G2_NT);
    double *Ab = a.A + (c0 + jb) * a.lda + ns + rb;
    constexpr bool F64 = sizeof(T) == 8;
    // tile (tc, tr): D[i][j] = A[row wr + 16 tr + j][col wc + 16 tc + i]
    acc_t acc[8];
    double apre[F64 ? 1 : 32];
    const int rj = lane & 15;
#pragma unroll
    for (int tc = 0; tc < 4; ++tc)
#pragma unroll
        for (int tr = 0; tr < 2; ++tr) {
            const int r = wr + tr * 16 + rj;
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int cc = wc + tc * 16 + Mfma<T>::row(lane, v);
                const double x = (r < nrow && cc < ncol) ? Ab[(int64_t)cc * a.lda + r] : 0.0;
                if constexpr (F64) acc[tc * 2 + tr][v] = x;
                else apre[(tc * 2 + tr) * 4 + v] = x;
            }
            if constexpr (!F64) acc[tc * 2 + tr] = acc_t{0, 0, 0, 0};
        }
    // the V and Z chunks go through registers to LDS; the next chunk's loads are
    // issued before this chunk's MFMAs so that their latency overlaps them
    T vr[4], zr[4];
    auto load_chunk = [&](int kc) {
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int e = u * 512 + tid, k = e >> 7, r = e & 127;
            const bool kok = kc + k < l;
            if constexpr (MODE == 0) {
                vr[u] = (kok && r < nrow) ? V[(int64_t)(kc + k) * ldv + rb + r] : (T)0;
            } else {
                const double sc = (kc + k == l - 1) ? rpend : 1.0;
                vr[u] = (kok && r < nrow) ? (T)(V[(vk0 + kc + k) * ldv + ns + rb + r] * sc) : (T)0;
            }
            zr[u] = (kok && r < ncol) ? Z[(int64_t)(kc + k) * ldz + jb + r] : (T)0;
        }
    };
    load_chunk(0);
    for (int kc = 0; kc < l; kc += G2_KC) {
        __syncthreads();
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            Vs[u * 512 + tid] = vr[u];
            Zs[u * 512 + tid] = zr[u];
        }
        __syncthreads();
        if (kc + G2_KC < l) load_chunk(kc + G2_KC);
#pragma unroll 2
        for (int k = 0; k < G2_KC; k += 4) {
            T zo[4], vo[2];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                zo[u] = Zs[(k + (lane >> 4)) * G2_NT + wc + u * 16 + rj];  // A-operand: Z^T[i][k]
                if constexpr (F64) zo[u] = -zo[u];
            }
#pragma unroll
            for (int u = 0; u < 2; ++u) vo[u] = Vs[(k + (lane >> 4)) * G2_MT + wr + u * 16 + rj];  // B: V^T[k][j]
#pragma unroll
            for (int tc = 0; tc < 4; ++tc)
#pragma unroll
                for (int tr = 0; tr < 2; ++tr) acc[tc * 2 + tr] = Mfma<T>::op(zo[tc], vo[tr], acc[tc * 2 + tr]);
        }
    }
#pragma unroll
    for (int tc = 0; tc < 4; ++tc)
#pragma unroll
        for (int tr = 0; tr < 2; ++tr) {
            const int r = wr + tr * 16 + rj;
            if (r < nrow) {
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int cc = wc + tc * 16 + Mfma<T>::row(lane, v);
                    if (cc < ncol) {
                        double y;
                        if constexpr (F64) y = acc[tc * 2 + tr][v];
                        else y = apre[(tc * 2 + tr) * 4 + v] - (double)acc[tc * 2 + tr][v];
                        Ab[(int64_t)cc * a.lda + r] = y;
                    }
                }
            }
        }
}

// A_tr -= V Z for an FP64 QRDM block of at most 64 reflectors, persistent:
// one workgroup of 1024 threads per compute unit takes a run of 128 x 128
// tiles (the tiles in row-major order, split evenly over the grid), so that
// its tiles share a row of tiles.  V's rows of that tile row and Z's columns of
// the tile are staged whole in LDS (all l reflectors), so the MFMA loop reads
// no global memory, and the next tile's A and Z are loaded into registers while
// the current tile's MFMAs run.  Wavefront w takes the 32 x 32 block at rows
// 32 (w / 4), columns 32 (w % 4) of the tile; the products are k_gemm2's
// (D = Z^T V^T, the accumulators starting as the A tile, the same order over k).
// A is read once here, with non-temporal loads, so that its stream does not
// evict the V rows and Z columns that other workgroups of the same L2 read.
#define G2P_KMAX 64
#define G2P_TH 1024
#define G2P_LD (G2_MT + 8)  // LDS row of the staged V and Z (doubles); the 8 spread the banks
#define G2P_LDS ((size_t)2 * G2P_KMAX * G2P_LD * sizeof(double))
__global__ void __launch_bounds__(G2P_TH) __attribute__((amdgpu_waves_per_eu(4, 4)))
k_gemm2p(QrdmArgs a, const double *__restrict__ V, int64_t ldv, const double *__restrict__ Z, int64_t ldz) {
    const QrdmCtl *ctl = a.ctl;
    if (qrdm_dm_idle(ctl)) return;
    const int64_t ns = ctl->ns, c0 = ctl->ns + ctl->c0off;  // c0off: k_s, or l after the Gram-matrix panel
    const int l = ctl->l;
    const int64_t t = a.m - ns, w2 = a.n - c0;
    if (l <= 0 || t <= 0 || w2 <= 0) return;
    if (l > G2P_KMAX) {  // the host takes this kernel for k_DM <= 64 only (cannot happen)
        if (blockIdx.x == 0 && threadIdx.x == 0) atomicOr(&a.ctl->error, 4);
        return;
    }
    const int64_t ntc = (w2 + G2_NT - 1) / G2_NT, ntiles = ((t + G2_MT - 1) / G2_MT) * ntc;
    const int64_t tb = ntiles * blockIdx.x / gridDim.x, te = ntiles * (blockIdx.x + 1) / gridDim.x;
    if (tb >= te) return;
    extern __shared__ double g2p_lds[];
    double *Vs = g2p_lds;                 // [k][row]
    double *Zs = Vs + G2P_KMAX * G2P_LD;  // [k][col]
    const int tid = threadIdx.x, lane = tid & 63;
    const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int wr = (wv >> 2) * 32, wc = (wv & 3) * 32;  // wave's 32 x 32 block (rows, cols)
    const int rj = lane & 15;
    const int lk = (l + 15) & ~15;  // reflectors in whole 16-chunks (zeros past l)
    typedef Mfma<double>::acc_t acc_t;
    // Addresses as a part common to the wavefront plus one 32-bit offset per
    // thread (the host takes this kernel when 128 lda, 64 ldv and 64 ldz fit).
    // A of a tile in the accumulator layout: (tc, tr) register v holds
    // A[row wr + 16 tr + rj][col wc + 16 tc + 4 v + lane / 16] (Mfma::row).
    const int lda = (int)a.lda, ldvi = (int)ldv, ldzi = (int)ldz;
    const int aoff = (lane >> 4) * lda + wr + rj;           // + 16 tr, + (wc + 16 tc + 4 v) lda
    const int koff = (tid >> 7), coff = tid & 127;          // staged element u G2P_TH + tid: (8 u + koff, coff)
    auto a_load = [&](int64_t tile, double (&x)[16]) {
        const int64_t rb = (tile / ntc) * G2_MT, jb = (tile % ntc) * G2_NT;
        const int nrow = (int)((t - rb) < G2_MT ? (t - rb) : G2_MT);
        const int ncol = (int)((w2 - jb) < G2_NT ? (w2 - jb) : G2_NT);
        const double *Ab = a.A + (c0 + jb) * a.lda + ns + rb;
#pragma unroll
        for (int tc = 0; tc < 2; ++tc)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int cu = wc + tc * 16 + 4 * v;
                const double *pc = Ab + (int64_t)cu * lda;
                const bool cok = cu + (lane >> 4) < ncol;
#pragma unroll
                for (int tr = 0; tr < 2; ++tr)
                    x[(tc * 2 + tr) * 4 + v] =
                          (cok && wr + tr * 16 + rj < nrow) ? __builtin_nontemporal_load(pc + aoff + tr * 16) : 0.0;
            }
    };
    auto z_load = [&](int64_t tile, double (&z)[8]) {
        const int64_t jb = (tile % ntc) * G2_NT;
        const int ncol = (int)((w2 - jb) < G2_NT ? (w2 - jb) : G2_NT);
        const double *Zb = Z + jb + koff * ldzi + coff;
#pragma unroll
        for (int u = 0; u < 8; ++u)
            z[u] = (8 * u + koff < l && coff < ncol) ? Zb[8 * u * ldzi] : 0.0;
    };
    double apf[16], zpf[8];
    a_load(tb, apf);
    z_load(tb, zpf);
    int64_t vrow = -1;
    for (int64_t tile = tb; tile < te; ++tile) {
        const int64_t trow = tile / ntc, rb = trow * G2_MT, jb = (tile % ntc) * G2_NT;
        const int nrow = (int)((t - rb) < G2_MT ? (t - rb) : G2_MT);
        const int ncol = (int)((w2 - jb) < G2_NT ? (w2 - jb) : G2_NT);
        if (trow != vrow) {  // V's rows of this tile row (all reflectors), once per row of tiles
            const double *Vb = V + rb + koff * ldvi + coff;
            double vr[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) vr[u] = (8 * u + koff < l && coff < nrow) ? Vb[8 * u * ldvi] : 0.0;
#pragma unroll
            for (int u = 0; u < 8; ++u) Vs[(8 * u + koff) * G2P_LD + coff] = vr[u];
            vrow = trow;
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) Zs[(8 * u + koff) * G2P_LD + coff] = zpf[u];
        acc_t acc[4];
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int v = 0; v < 4; ++v) acc[i][v] = apf[i * 4 + v];
        __syncthreads();
        if (tile + 1 < te) {  // the next tile's operands, in flight during the MFMAs
            a_load(tile + 1, apf);
            z_load(tile + 1, zpf);
        }
        for (int k = 0; k < lk; k += 4) {
            double zo[2], vo[2];
#pragma unroll
            for (int u = 0; u < 2; ++u) zo[u] = -Zs[(k + (lane >> 4)) * G2P_LD + wc + u * 16 + rj];  // A-operand: -Z^T[i][k]
#pragma unroll
            for (int u = 0; u < 2; ++u) vo[u] = Vs[(k + (lane >> 4)) * G2P_LD + wr + u * 16 + rj];  // B: V^T[k][j]
#pragma unroll
            for (int tc = 0; tc < 2; ++tc)
#pragma unroll
                for (int tr = 0; tr < 2; ++tr) acc[tc * 2 + tr] = Mfma<double>::op(zo[tc], vo[tr], acc[tc * 2 + tr]);
        }
        double *Ab = a.A + (c0 + jb) * a.lda + ns + rb;
#pragma unroll
        for (int tc = 0; tc < 2; ++tc)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int cu = wc + tc * 16 + 4 * v;
                double *pc = Ab + (int64_t)cu * lda;
                if (cu + (lane >> 4) < ncol) {
#pragma unroll
                    for (int tr = 0; tr < 2; ++tr)
                        if (wr + tr * 16 + rj < nrow) pc[aoff + tr * 16] = acc[tc * 2 + tr][v];
                }
            }
        __syncthreads();  // Vs and Zs read before the next tile writes them
    }
}

// Rows of the V^T A partials per split (k_DM rounded up to the 16-row MFMA
// tiles) times the n columns: the stride between the splits in Yp.
int64_t trail_ysplit(int kmax, int64_t n) {
    const int kp = ((kmax < QK_KM ? kmax : QK_KM) + 15) & ~15;
    return (int64_t)kp * n;
}
int trail_splits_max() { return QK_SPLIT_MAX; }

hipError_t launch_trail(QrdmArgs a, int precision, const double *VV, const double *cpT, const double *Vw, const float *Vw32,
                        int64_t ldv, void *Z, double *Yp, int64_t t_bound, int64_t w_bound, int64_t w_lo,
                        hipStream_t s, hipEvent_t *ev) {
    if (t_bound <= 0 || w_bound <= 0) return hipSuccess;
    const int64_t ldz = a.n;
    const int64_t ysplit = trail_ysplit(a.kmax, a.n);
    const int ntile = (int)((w_bound + G1_NT - 1) / G1_NT);
    // enough splits for any trailing size within the bounds: g1_krows picks the
    // split on the device (at most 16, at most t/G1_MINROWS, at most G1_TARGET_WGS over
    // the column tiles of the narrowest possible w); workgroups past it return
    int64_t nsplit = (t_bound + G1_MINROWS - 1) / G1_MINROWS;
    if (nsplit > QK_SPLIT_MAX) nsplit = QK_SPLIT_MAX;
    {
        const int64_t wl = w_lo > 1 ? w_lo : 1;
        const int64_t nt_lo = (wl + G1_NT - 1) / G1_NT;
        const int64_t by_wgs = G1_TARGET_WGS / nt_lo;
        if (nsplit > by_wgs) nsplit = by_wgs;
    }
    if (nsplit < 1) nsplit = 1;
    const int kk = a.kmax < QK_KM ? a.kmax : QK_KM;
    dim3 g1((unsigned)ntile, (unsigned)nsplit, (unsigned)((((kk + 15) >> 4) + 3) >> 2));
    dim3 g2((unsigned)((w_bound + G2_NT - 1) / G2_NT), (unsigned)((t_bound + G2_MT - 1) / G2_MT));
    const int kp = ((a.kmax < QK_KM ? a.kmax : QK_KM) + 15) & ~15;
    const size_t tsz = precision == 0 ? sizeof(double) : sizeof(float);
    const size_t main_b = (size_t)(64 + G1_NT) * G1_LD * tsz;
    const size_t epi_rec = ((size_t)kp * ZS_LDY + (size_t)kp * (kp - 1) / 2 + 1 + kp) * sizeof(double);
    const size_t epi_xt = ((size_t)3 * 64 * ZT_LD + 64) * sizeof(double);
    const size_t epi_b = epi_rec > epi_xt ? epi_rec : epi_xt;
    static bool attr = false;
    static int g2p_grid = 0;  // one workgroup per compute unit; 0: the tiled k_gemm2 instead
    if (!attr) {
        int dev = 0, ncu = 0, per_cu = 0;
        if (hipGetDevice(&dev) == hipSuccess &&
            hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess &&
            hipFuncSetAttribute((const void *)k_gemm2p, hipFuncAttributeMaxDynamicSharedMemorySize, (int)G2P_LDS) ==
                hipSuccess &&
            hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void *)k_gemm2p, G2P_TH, G2P_LDS) == hipSuccess &&
            per_cu >= 1)
            g2p_grid = ncu;
        (void)hipGetLastError();
        const void *fs[6] = {(const void *)k_gemm1<double>,     (const void *)k_gemm1<float>,
                             (const void *)k_zsum<double, 32>, (const void *)k_zsum<double, 64>,
                             (const void *)k_zsum<float, 32>,  (const void *)k_zsum<float, 64>};
        for (const void *f : fs) {
            hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, 150 * 1024);
            if (e != hipSuccess) return e;
        }
        attr = true;
    }
    // k_zsum: 32 columns per workgroup on the explicit-T path (l <= kmax <= 64),
    // twice the workgroups for the partial sums; 64 for the recurrence
    const bool z32 = a.kmax <= 64;
    const dim3 gz((unsigned)((w_bound + (z32 ? 31 : 63)) / (z32 ? 32 : 64)));
    if (ev) (void)hipEventRecord(ev[0], s);
    if (precision == 0) {
        hipLaunchKernelGGL(k_gemm1<double>, g1, dim3(G1_TH), main_b, s, a, Vw, ldv, Yp, ldz, ysplit);
        if (ev) (void)hipEventRecord(ev[1], s);
        if (z32) hipLaunchKernelGGL((k_zsum<double, 32>), gz, dim3(G1_TH), epi_b, s, a, VV, cpT, (const double *)Yp, (double *)Z, ldz, ysplit);
        else hipLaunchKernelGGL((k_zsum<double, 64>), gz, dim3(G1_TH), epi_b, s, a, VV, cpT, (const double *)Yp, (double *)Z, ldz, ysplit);
    } else {
        hipLaunchKernelGGL(k_gemm1<float>, g1, dim3(G1_TH), main_b, s, a, Vw32, ldv, Yp, ldz, ysplit);
        if (ev) (void)hipEventRecord(ev[1], s);
        if (z32) hipLaunchKernelGGL((k_zsum<float, 32>), gz, dim3(G1_TH), epi_b, s, a, VV, cpT, (const double *)Yp, (float *)Z, ldz, ysplit);
        else hipLaunchKernelGGL((k_zsum<float, 64>), gz, dim3(G1_TH), epi_b, s, a, VV, cpT, (const double *)Yp, (float *)Z, ldz, ysplit);
    }
    if (ev) (void)hipEventRecord(ev[2], s);
    if (precision == 0 && a.kmax <= G2P_KMAX && g2p_grid > 0 && a.lda <= (INT32_MAX / G2_NT) && ldv <= (INT32_MAX / 64) &&
        ldz <= (INT32_MAX / 64))
        hipLaunchKernelGGL(k_gemm2p, dim3((unsigned)g2p_grid), dim3(G2P_TH), G2P_LDS, s, a, Vw, ldv, (const double *)Z, ldz);
    else if (precision == 0)
        hipLaunchKernelGGL((k_gemm2<double, 0>), g2, dim3(512), 0, s, a, Vw, ldv, (const double *)Z, ldz);
    else
        hipLaunchKernelGGL((k_gemm2<float, 0>), g2, dim3(512), 0, s, a, Vw32, ldv, (const float *)Z, ldz);
    if (ev) (void)hipEventRecord(ev[3], s);
    return hipGetLastError();
}

hipError_t launch_gemm2_qp3(QrdmArgs a, const double *Vw, int64_t ldv, const double *Fz, int64_t t_bound,
                            int64_t w_bound, hipStream_t s) {
    if (t_bound <= 0 || w_bound <= 0) return hipSuccess;
    dim3 g2((unsigned)((w_bound + G2_NT - 1) / G2_NT), (unsigned)((t_bound + G2_MT - 1) / G2_MT));
    hipLaunchKernelGGL((k_gemm2<double, 1>), g2, dim3(512), 0, s, a, Vw, ldv, Fz, a.n);
    return hipGetLastError();
}
