// Householder panel of one QRDM block with the early break (Algorithm 4 of
// the paper, inner loop; threshold eps_s of eq. lenght_check), on gfx950.  It
// also records the inner products v_a^T v_i of the reflectors, from which the
// trailing update applies the compact WY form (Section 3.2) without forming
// its triangular factor.
//
// The k_s accepted columns (rows n_s..m-1) are split into row slabs, one per
// workgroup, held in LDS for the whole panel.  Every panel column costs one
// grid-wide reduction round: each workgroup contributes, in one vector,
//   Dall_j = sum_{rows > c} x_r a_{r,j}   for every panel column j
//   Top_j  = a_{c,j}                       (row c of the diagonal)
// where x is the current column.  From the reduced vector every workgroup
// derives, redundantly and identically, ||x|| (and the break decision), the
// reflector (LAPACK larfg convention: beta = -sign(alpha)||x||), the products
// v^T a_j of the in-panel update, and the inner products v_a^T v_i.  Reductions are in fixed order, so the run is bit-reproducible
// and every workgroup takes the same branch.
//
// The launch must be cooperative (all workgroups co-resident): the rounds are
// separated by a counter barrier in the loop-state block.
#include "qrdm_internal.h"

#define PN_THREADS 512
#define PN_WAVES (PN_THREADS / 64)
#define PN_SPIN_LIMIT (1 << 26)

// Grid barrier for the cooperative panel.  Partials are published with
// agent-scope (sc1) stores, which are coherent across XCDs without a write-back
// of the whole L2; waiting for them to complete orders them before the counter
// increment.  The spin is bounded: on timeout the error flag is raised and the
// kernel runs to completion (the host then reports an error).
__device__ __forceinline__ void grid_barrier(uint32_t *bar, uint32_t target, int32_t *err) {
    __builtin_amdgcn_s_waitcnt(0);  // every wave's published stores have completed
    __syncthreads();
    if (threadIdx.x == 0) {
        __hip_atomic_fetch_add(bar, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        int it = 0;
        while (__hip_atomic_load(bar, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
            __builtin_amdgcn_s_sleep(1);
            if (++it > PN_SPIN_LIMIT) {
                atomicOr(err, 2);
                break;
            }
        }
    }
    __syncthreads();
}

__device__ __forceinline__ void st_coherent(double *p, double v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ double ld_coherent(const double *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

extern __shared__ double pn_lds[];

__global__ void __launch_bounds__(PN_THREADS)
k_panel(QrdmArgs a, double *PB, double *VV, double *Vw, float *Vw32, int64_t ldv) {
    QrdmCtl *ctl = a.ctl;
    if (ctl->done) return;
    const int64_t ns = ctl->ns;
    const int ks = ctl->ks;
    const double eps_s = ctl->eps_s;
    const int64_t t = a.m - ns;
    const int P = gridDim.x;
    const int wg = blockIdx.x;
    const int rp = (int)((t + P - 1) / P);
    const int64_t g0 = ns + (int64_t)wg * rp;  // first global row of this slab
    int64_t nr64 = a.m - g0;
    if (nr64 < 0) nr64 = 0;
    const int nrows = (int)(nr64 < rp ? nr64 : rp);
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;

    const int ksp = ks + 1;                  // padded row stride of the slab
    double *S = pn_lds;                      // [rp][ksp] slab, row-major
    double *red = S + (size_t)rp * ksp;      // [PN_WAVES][QK_KM] partial dots; reused for sums
    double *sR = red + PN_WAVES * QK_KM;     // reduced Dall
    double *sTop = sR + QK_KM;               // reduced Top
    double *sW = sTop + QK_KM;               // tau * v^T a_j

    // load the slab: 8 independent loads in flight per thread
    {
        const int total = nrows * ks;
        for (int base = 0; base < total; base += PN_THREADS * 8) {
            double v[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int idx = base + u * PN_THREADS + tid;
                v[u] = 0.0;
                if (idx < total) {
                    const int j = idx / nrows, r = idx - j * nrows;
                    v[u] = a.A[(ns + j) * a.lda + g0 + r];
                }
            }
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int idx = base + u * PN_THREADS + tid;
                if (idx < total) {
                    const int j = idx / nrows, r = idx - j * nrows;
                    S[r * ksp + j] = v[u];
                }
            }
        }
    }
    __syncthreads();

    // reduction layout: value e in [0, 2ks) is summed by `gpv` thread groups
    const int nval = 2 * ks;
    int gpv = PN_THREADS / nval;   // groups per value (red holds 4 x 2 QK_KM sums)
    if (gpv > PN_WAVES / 2) gpv = PN_WAVES / 2;
    if (gpv < 1) gpv = 1;
    const int my_e = tid % nval, my_g = tid / nval;
    const int wper = (P + gpv - 1) / gpv;

    int l = ks;
    uint32_t round = 0;
    for (int i = 0; i < ks; ++i, ++round) {
        const int64_t c = ns + i;
        const int64_t cl64 = c - g0;
        const int cl = (cl64 >= 0 && cl64 < nrows) ? (int)cl64 : -1;  // local row of c
        int rstart = (int)(cl64 + 1);
        if (rstart < 0) rstart = 0;
        // ---- partial dots over rows strictly below c
        for (int jj = lane; jj < ks; jj += 64) {
            double s = 0.0;
            for (int r = rstart + wv; r < nrows; r += PN_WAVES) s += S[r * ksp + i] * S[r * ksp + jj];
            red[wv * QK_KM + jj] = s;
        }
        __syncthreads();
        double *pb = PB + ((size_t)(round & 1) * P + wg) * (2 * QK_KM);
        if (tid < nval) {
            const int jj = (tid < ks) ? tid : tid - ks;
            double v;
            if (tid < ks) {
                v = 0.0;
#pragma unroll
                for (int w = 0; w < PN_WAVES; ++w) v += red[w * QK_KM + jj];
            } else {
                v = (cl >= 0) ? S[cl * ksp + jj] : 0.0;
            }
            st_coherent(pb + ((tid < ks) ? jj : QK_KM + jj), v);
        }
        grid_barrier(&ctl->bar, (uint32_t)P * (round + 1), &ctl->error);
        // ---- fixed-order reduction of all partials (every workgroup, identically)
        const double *pb0 = PB + (size_t)(round & 1) * P * (2 * QK_KM);
        if (my_g < gpv && tid < gpv * nval) {
            const int jj = (my_e < ks) ? my_e : my_e - ks;
            const int o = (my_e < ks) ? jj : QK_KM + jj;
            const int w0 = my_g * wper;
            const int w1 = (w0 + wper < P) ? w0 + wper : P;
            double s = 0.0;
            for (int wb = w0; wb < w1; wb += 16) {
                double v[16];
#pragma unroll
                for (int u = 0; u < 16; ++u) v[u] = (wb + u < w1) ? ld_coherent(pb0 + (size_t)(wb + u) * (2 * QK_KM) + o) : 0.0;
#pragma unroll
                for (int u = 0; u < 16; ++u) s += v[u];
            }
            red[my_g * (2 * QK_KM) + my_e] = s;
        }
        __syncthreads();
        if (tid < nval) {
            double s = 0.0;
            for (int g = 0; g < gpv; ++g) s += red[g * (2 * QK_KM) + tid];
            if (tid < ks) sR[tid] = s; else sTop[tid - ks] = s;
        }
        __syncthreads();
        const double alpha = sTop[i];
        const double sp = sR[i];
        const double nrm = sqrt(alpha * alpha + sp);
        if (i >= 1 && nrm < eps_s) {  // length check: column i depends on the kept ones
            l = i;
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
        for (int jj = i + 1 + tid; jj < ks; jj += PN_THREADS) sW[jj] = ti * (sTop[jj] + sR[jj] / den);
        if (wg == 0) {
            // inner products v_a^T v_i = Top_a + Dall_a / den (a < i) of the
            // compact WY form; the trailing update uses them with tau instead of
            // forming T explicitly
            if (tid < i) VV[tid * QK_KM + i] = sTop[tid] + sR[tid] / den;
            if (tid == 0) a.tau_house[c] = ti;
        }
        __syncthreads();
        // ---- apply H_i to the slab: rows below c, then row c.  v = x / (alpha - beta)
        // is formed with one reciprocal per round, as LAPACK larfg scales by it.
        {
            const double rden = 1.0 / den;
            const int j0 = lane, j1 = lane + 64;
            const double w0 = (j0 > i && j0 < ks) ? sW[j0] : 0.0;
            const double w1 = (j1 > i && j1 < ks) ? sW[j1] : 0.0;
            const bool has1 = j1 < ks;
            const bool own0 = (lane == i), own1 = (lane + 64 == i);
#pragma unroll 4
            for (int r = rstart + wv; r < nrows; r += PN_WAVES) {
                double *row = S + r * ksp;
                const double v = row[i] * rden;
                if (j0 < ks) row[j0] = own0 ? v : row[j0] - v * w0;
                if (has1) row[j1] = own1 ? v : row[j1] - v * w1;
            }
        }
        if (cl >= 0 && wv == (cl % PN_WAVES)) {
            for (int jj = lane; jj < ks; jj += 64)
                if (jj > i) S[cl * ksp + jj] -= sW[jj];
            if (lane == 0) S[cl * ksp + i] = beta;
        }
        __syncthreads();
    }
    // ---- write the slab back; V (explicit unit diagonal and zeros above) for
    // the trailing update, rows indexed from n_s
    for (int idx = tid; idx < nrows * ks; idx += PN_THREADS) {
        const int j = idx / nrows, r = idx - j * nrows;
        const double x = S[r * ksp + j];
        a.A[(ns + j) * a.lda + g0 + r] = x;
        if (j < l) {
            const int64_t g = g0 + r;
            const double v = (g > ns + j) ? x : (g == ns + j ? 1.0 : 0.0);
            const int64_t o = (int64_t)j * ldv + (g - ns);
            Vw[o] = v;
            if (Vw32) Vw32[o] = (float)v;
        }
    }
    if (wg == 0 && tid == 0) {
        ctl->l = l;
        if (l < ks) ctl->nbreaks += 1;
        // reflector i: norm 2(t-i), apply to the ks-1-i panel columns to its right 4(t-i)(ks-1-i)
        double f = 0.0;
        for (int i = 0; i < l; ++i) f += (double)(t - i) * (2.0 + 4.0 * (double)(ks - 1 - i));
        ctl->flop_panel += f;
        ctl->bytes_panel += 16.0 * (double)t * (double)ks;
        ctl->npanel += 1;
    }
}

int panel_lds_bytes(int rows_per_wg, int kmax) {
    return (rows_per_wg * (kmax + 1) + (PN_WAVES + 3) * QK_KM) * (int)sizeof(double);
}

// Tallest slab (multiple of 16 rows, at most 256) whose LDS fits in 150 KB.
int panel_rows_per_wg(int kmax) {
    const int budget = 150 * 1024 / (int)sizeof(double) - (PN_WAVES + 3) * QK_KM;
    int r = budget / (kmax + 1);
    if (r > 256) r = 256;
    r &= ~15;
    return r < 16 ? 16 : r;
}

int panel_max_wgs(int rows_per_wg) {
    (void)rows_per_wg;
    int dev = 0;
    hipGetDevice(&dev);
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, dev) != hipSuccess) return 1;
    return prop.multiProcessorCount;
}

hipError_t launch_panel(QrdmArgs a, double *PB, double *VV, double *Vw, float *Vw32, int64_t ldv,
                        int64_t t_bound, int rows_per_wg, hipStream_t s) {
    if (t_bound <= 0) return hipSuccess;
    int P = (int)((t_bound + rows_per_wg - 1) / rows_per_wg);
    if (P < 1) P = 1;
    const int kk = a.kmax < QK_KM ? a.kmax : QK_KM;
    const int lds = panel_lds_bytes(rows_per_wg, kk);
    static bool attr_set = false;
    if (!attr_set) {
        hipError_t e = hipFuncSetAttribute((const void *)k_panel, hipFuncAttributeMaxDynamicSharedMemorySize, 150 * 1024);
        if (e != hipSuccess) return e;
        attr_set = true;
    }
    void *args[] = {&a, &PB, &VV, &Vw, &Vw32, &ldv};
    return hipLaunchCooperativeKernel((const void *)k_panel, dim3(P), dim3(PN_THREADS), args, (unsigned)lds, s);
}
