// Block trailing update of QRDM (Algorithm 4 of the paper, the BLAS-3 step;
// compact WY form of Section 3.2): with the l kept reflectors as
// H_0...H_{l-1} = I - V T V^T,
//     A_tr <- (I - V T V^T)^T A_tr = A_tr - V (T^T (V^T A_tr)),
// A_tr = A[n_s:m, n_s+k_s:n].  Three kernels on gfx950 MFMA:
//   k_gemm1   Zp[s] = V^T A_tr over row split s (split-K, K = t rows).
//   k_zreduce Z = T^T sum_s Zp[s] (fixed order; FP64).
//   k_gemm2   A_tr -= V Z (K = l), the update accumulated in registers and
//             subtracted from A in one read-modify-write pass.
// Precision: FP64 MFMA (16x16x4 f64) by default; mixed mode uses FP32 MFMA
// (16x16x4 f32) with FP32 accumulation for the two products while A stays
// FP64 in memory and Z is reduced in FP64.
#include "qrdm_internal.h"

typedef double dbl4 __attribute__((ext_vector_type(4)));
typedef float flt4 __attribute__((ext_vector_type(4)));

template <typename T> struct Mfma;
// Operand layouts of both 16x16x4 instructions: A[i][k] in lane i + 16k, B[k][j]
// in lane j + 16k.  Result layouts differ: register v of a lane holds
// D[4v + lane/16][lane%16] for f64 and D[4(lane/16) + v][lane%16] for f32.
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
#define G1_NT 128   // trailing columns per workgroup
#define G1_KC 32    // rows staged per step
#define G1_LD (G1_KC + 1)

// Zp[s] = V^T A_tr over rows [s*split_rows, (s+1)*split_rows).  The next row
// chunk is loaded into registers while the current one is multiplied out of
// LDS, so the HBM latency overlaps the MFMA work.
template <typename T>
__global__ void __launch_bounds__(256)
k_gemm1(QrdmArgs a, const T *__restrict__ V, int64_t ldv, T *__restrict__ Zp, int split_rows, int64_t ldz) {
    const QrdmCtl *ctl = a.ctl;
    if (ctl->done) return;
    const int64_t ns = ctl->ns;
    const int ks = ctl->ks, l = ctl->l;
    const int64_t t = a.m - ns;
    const int64_t c0 = ns + ks;
    const int64_t w2 = a.n - c0;
    const int64_t jb = (int64_t)blockIdx.x * G1_NT;
    const int64_t rb = (int64_t)blockIdx.y * split_rows;
    if (l <= 0 || jb >= w2 || rb >= t) return;
    const int64_t re = (rb + split_rows < t) ? rb + split_rows : t;
    const int lt = (l + 15) >> 4;  // 16-row tiles of Z
    const int lp = lt * 16;
    __shared__ T Vs[QK_KM * G1_LD];
    __shared__ T As[G1_NT * G1_LD];
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    typedef typename Mfma<T>::acc_t acc_t;
    acc_t acc[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) acc[u] = acc_t{0, 0, 0, 0};
    const int ncols = (int)((w2 - jb) < G1_NT ? (w2 - jb) : G1_NT);
    const double *Abase = a.A + (c0 + jb) * a.lda + ns;
    // element u*256 + tid of a chunk: column q = u*8 + tid/32, row r = tid%32
    const int rr = tid & 31, qq = tid >> 5;
    T vreg[16], areg[16];
    auto fetch = [&](int64_t rc) {
        const int64_t row = rc + rr;
        const bool rok = row < re;
#pragma unroll
        for (int u = 0; u < 16; ++u) {
            const int q = u * 8 + qq;
            vreg[u] = (rok && q < l) ? V[(int64_t)q * ldv + row] : (T)0;
            areg[u] = (rok && q < ncols) ? (T)Abase[(int64_t)q * a.lda + row] : (T)0;
        }
    };
    fetch(rb);
    for (int64_t rc = rb; rc < re; rc += G1_KC) {
        __syncthreads();
#pragma unroll
        for (int u = 0; u < 16; ++u) {
            const int q = u * 8 + qq;
            if (q < lp) Vs[q * G1_LD + rr] = vreg[u];
            As[q * G1_LD + rr] = areg[u];
        }
        __syncthreads();
        if (rc + G1_KC < re) fetch(rc + G1_KC);
        // wave wv owns trailing columns [32 wv, 32 wv + 32): 2 column tiles x lt row tiles
#pragma unroll
        for (int k = 0; k < G1_KC; k += 4) {
            const T b0 = As[(wv * 32 + (lane & 15)) * G1_LD + k + (lane >> 4)];
            const T b1 = As[(wv * 32 + 16 + (lane & 15)) * G1_LD + k + (lane >> 4)];
#pragma unroll
            for (int ti = 0; ti < 8; ++ti) {
                if (ti < lt) {
                    const T av = Vs[(ti * 16 + (lane & 15)) * G1_LD + k + (lane >> 4)];
                    acc[2 * ti] = Mfma<T>::op(av, b0, acc[2 * ti]);
                    acc[2 * ti + 1] = Mfma<T>::op(av, b1, acc[2 * ti + 1]);
                }
            }
        }
    }
    T *out = Zp + (int64_t)blockIdx.y * QK_KM * ldz;
#pragma unroll
    for (int ti = 0; ti < 8; ++ti) {
        if (ti < lt) {
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const int64_t col = jb + wv * 32 + h * 16 + (lane & 15);
                if (col < w2) {
#pragma unroll
                    for (int v = 0; v < 4; ++v) {
                        const int row = ti * 16 + Mfma<T>::row(lane, v);
                        out[row * ldz + col] = acc[2 * ti + h][v];
                    }
                }
            }
        }
    }
}

// ---------------------------------------------------------------- zreduce
#define ZR_NC 32

template <typename T>
__global__ void __launch_bounds__(256)
k_zreduce(QrdmArgs a, const T *__restrict__ Zp, int nsplit_bound, int split_rows, const double *__restrict__ Tm,
          T *__restrict__ Z, int64_t ldz) {
    const QrdmCtl *ctl = a.ctl;
    if (ctl->done) return;
    const int64_t ns = ctl->ns;
    const int ks = ctl->ks, l = ctl->l;
    const int64_t t = a.m - ns;
    const int64_t w2 = a.n - (ns + ks);
    const int64_t jb = (int64_t)blockIdx.x * ZR_NC;
    if (l <= 0 || jb >= w2) return;
    const int nsplit = (int)((t + split_rows - 1) / split_rows);
    (void)nsplit_bound;
    if (blockIdx.x == 0 && threadIdx.x == 0) a.ctl->flop_gemm += 2.0 * (double)t * (double)l * (double)w2;
    __shared__ double Ys[QK_KM * ZR_NC];
    __shared__ double Ts[QK_KM * QK_KM / 2 + QK_KM];
    const int tid = threadIdx.x;
    const int jl = tid & (ZR_NC - 1), ag = tid / ZR_NC;  // 8 groups
    const int64_t j = jb + jl;
    // T (upper triangle, packed by columns: T[b][a] for b <= a at a(a+1)/2 + b)
    for (int e = tid; e < l * l; e += 256) {
        const int b = e / l, aa = e - b * l;
        if (b <= aa) Ts[aa * (aa + 1) / 2 + b] = Tm[b * QK_KM + aa];
    }
    for (int b = ag; b < l; b += 256 / ZR_NC) {
        double s = 0.0;
        if (j < w2) {
            for (int sb = 0; sb < nsplit; sb += 8) {
                double v[8];
#pragma unroll
                for (int u = 0; u < 8; ++u)
                    v[u] = (sb + u < nsplit) ? (double)Zp[((int64_t)(sb + u) * QK_KM + b) * ldz + j] : 0.0;
#pragma unroll
                for (int u = 0; u < 8; ++u) s += v[u];
            }
        }
        Ys[b * ZR_NC + jl] = s;
    }
    __syncthreads();
    if (j < w2) {
        for (int aa = ag; aa < l; aa += 256 / ZR_NC) {
            double s = 0.0;
            const double *tc = Ts + aa * (aa + 1) / 2;
            for (int b = 0; b <= aa; ++b) s += tc[b] * Ys[b * ZR_NC + jl];
            Z[(int64_t)aa * ldz + j] = (T)s;
        }
    }
}

// ------------------------------------------------------------------ GEMM2
#define G2_MT 128
#define G2_NT 128
#define G2_KC 16

// A_tr -= V Z on a 128 x 128 tile.  FP64: the accumulators start as the A tile
// (loaded in the MFMA result layout) and the MFMAs add (-V) Z, so A is read
// once, early, and written once.  FP32 (mixed): the A tile is prefetched into
// FP64 registers while the FP32 product accumulates, then A - (double)acc.
template <typename T>
__global__ void __launch_bounds__(256)
k_gemm2(QrdmArgs a, const T *__restrict__ V, int64_t ldv, const T *__restrict__ Z, int64_t ldz) {
    const QrdmCtl *ctl = a.ctl;
    if (ctl->done) return;
    const int64_t ns = ctl->ns;
    const int ks = ctl->ks, l = ctl->l;
    const int64_t t = a.m - ns;
    const int64_t c0 = ns + ks;
    const int64_t w2 = a.n - c0;
    const int64_t rb = (int64_t)blockIdx.y * G2_MT;
    const int64_t jb = (int64_t)blockIdx.x * G2_NT;
    if (l <= 0 || rb >= t || jb >= w2) return;
    __shared__ T Vs[G2_KC * G2_MT];  // [k][row]
    __shared__ T Zs[G2_KC * G2_NT];  // [k][col]
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int wr = (wv >> 1) * 64, wc = (wv & 1) * 64;  // wave's 64x64 quadrant
    typedef typename Mfma<T>::acc_t acc_t;
    const int nrow = (int)((t - rb) < G2_MT ? (t - rb) : G2_MT);
    const int ncol = (int)((w2 - jb) < G2_NT ? (w2 - jb) : G2_NT);
    double *Ab = a.A + (c0 + jb) * a.lda + ns + rb;
    constexpr bool F64 = sizeof(T) == 8;
    acc_t acc[16];
    double apre[F64 ? 1 : 64];
#pragma unroll
    for (int ti = 0; ti < 4; ++ti)
#pragma unroll
        for (int tj = 0; tj < 4; ++tj) {
            const int cc = wc + tj * 16 + (lane & 15);
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int r = wr + ti * 16 + Mfma<T>::row(lane, v);
                const double x = (r < nrow && cc < ncol) ? Ab[(int64_t)cc * a.lda + r] : 0.0;
                if constexpr (F64) acc[ti * 4 + tj][v] = x;
                else apre[(ti * 4 + tj) * 4 + v] = x;
            }
            if constexpr (!F64) acc[ti * 4 + tj] = acc_t{0, 0, 0, 0};
        }
    // K chunks: element e = u*256 + tid -> (k = e / 128, index e % 128)
    for (int kc = 0; kc < l; kc += G2_KC) {
        T vr[8], zr[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int e = u * 256 + tid, k = e >> 7, r = e & 127;
            const bool kok = kc + k < l;
            vr[u] = (kok && r < nrow) ? V[(int64_t)(kc + k) * ldv + rb + r] : (T)0;
            zr[u] = (kok && r < ncol) ? Z[(int64_t)(kc + k) * ldz + jb + r] : (T)0;
        }
        __syncthreads();
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            Vs[u * 256 + tid] = vr[u];
            Zs[u * 256 + tid] = zr[u];
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < G2_KC; k += 4) {
            T av[4], bv[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                av[u] = Vs[(k + (lane >> 4)) * G2_MT + wr + u * 16 + (lane & 15)];
                bv[u] = Zs[(k + (lane >> 4)) * G2_NT + wc + u * 16 + (lane & 15)];
                if constexpr (F64) av[u] = -av[u];
            }
#pragma unroll
            for (int ti = 0; ti < 4; ++ti)
#pragma unroll
                for (int tj = 0; tj < 4; ++tj) acc[ti * 4 + tj] = Mfma<T>::op(av[ti], bv[tj], acc[ti * 4 + tj]);
        }
    }
#pragma unroll
    for (int ti = 0; ti < 4; ++ti) {
#pragma unroll
        for (int tj = 0; tj < 4; ++tj) {
            const int cc = wc + tj * 16 + (lane & 15);
            if (cc < ncol) {
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int r = wr + ti * 16 + Mfma<T>::row(lane, v);
                    if (r < nrow) {
                        double y;
                        if constexpr (F64) y = acc[ti * 4 + tj][v];
                        else y = apre[(ti * 4 + tj) * 4 + v] - (double)acc[ti * 4 + tj][v];
                        Ab[(int64_t)cc * a.lda + r] = y;
                    }
                }
            }
        }
    }
}

hipError_t launch_trail(QrdmArgs a, int precision, const double *Tm, const double *Vw, const float *Vw32,
                        int64_t ldv, void *Zp, void *Z, int64_t t_bound, int64_t w_bound, int split_rows,
                        hipStream_t s, hipEvent_t *ev) {
    if (t_bound <= 0 || w_bound <= 0) return hipSuccess;
    const int64_t ldz = a.n;
    const int nsplit = (int)((t_bound + split_rows - 1) / split_rows);
    dim3 g1((unsigned)((w_bound + G1_NT - 1) / G1_NT), (unsigned)nsplit);
    dim3 gz((unsigned)((w_bound + ZR_NC - 1) / ZR_NC));
    dim3 g2((unsigned)((w_bound + G2_NT - 1) / G2_NT), (unsigned)((t_bound + G2_MT - 1) / G2_MT));
    if (ev) (void)hipEventRecord(ev[0], s);
    if (precision == 0)
        hipLaunchKernelGGL(k_gemm1<double>, g1, dim3(256), 0, s, a, Vw, ldv, (double *)Zp, split_rows, ldz);
    else
        hipLaunchKernelGGL(k_gemm1<float>, g1, dim3(256), 0, s, a, Vw32, ldv, (float *)Zp, split_rows, ldz);
    if (ev) (void)hipEventRecord(ev[1], s);
    if (precision == 0)
        hipLaunchKernelGGL(k_zreduce<double>, gz, dim3(256), 0, s, a, (const double *)Zp, nsplit, split_rows, Tm,
                           (double *)Z, ldz);
    else
        hipLaunchKernelGGL(k_zreduce<float>, gz, dim3(256), 0, s, a, (const float *)Zp, nsplit, split_rows, Tm,
                           (float *)Z, ldz);
    if (ev) (void)hipEventRecord(ev[2], s);
    if (precision == 0)
        hipLaunchKernelGGL(k_gemm2<double>, g2, dim3(256), 0, s, a, Vw, ldv, (const double *)Z, ldz);
    else
        hipLaunchKernelGGL(k_gemm2<float>, g2, dim3(256), 0, s, a, Vw32, ldv, (const float *)Z, ldz);
    if (ev) (void)hipEventRecord(ev[3], s);
    return hipGetLastError();
}
