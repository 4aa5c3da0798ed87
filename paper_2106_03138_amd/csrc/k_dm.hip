// Deviation Maximization block column selection (Algorithm 1 of the paper,
// with the implementation choices of Section 4) on gfx950.
//
//  k_select       one workgroup: n_s <- n_s + l; max partial norm and its
//                 position; stopping test (eq. practical stopping criterion);
//                 switch to scalar pivoting near the noise level (eq.
//                 column_norm_bound_DM); the candidate list
//                 {j : u_j >= tau max u} (eq. def_candidate_set) in norm order,
//                 cut to k_DM entries (eq. candidate_set_limited_by_kDM) by a
//                 radix select on the IEEE bit patterns of the norms.
//  k_gram         C = A[n_s:m, L] gathered into LDS, partial Gram C^T C on
//                 FP64 MFMA (16x16x4), one partial per row slab.
//  k_gram_reduce  fixed-order sum of the partials.
//  k_dm_finish    cosines Theta = D^-1 G D^-1 with D = sqrt(diag G) (Section 4,
//                 option (ii)), greedy |theta| < delta acceptance in candidate
//                 order, and the column transpositions of Section 4 ("swap
//                 column n_s+i with column j_i"), applied in order by one
//                 wavefront to slot tables in LDS; vn1/vn2/perm are permuted
//                 here.  Lemma 1's record of the step (gamma and the sigma_min
//                 bound) is formed beside it when the step log or certified
//                 mode reads it.
//  k_swap         moves the affected columns of A (all m rows) through
//                 registers, on 32-row bands.
#include <float.h>

#include "qrdm_internal.h"

// ============================================================== k_select
#define SEL_THREADS 1024
#define SEL_WAVES (SEL_THREADS / 64)
#define SEL_KEYS 32  // keys per thread: supports n - n_s <= 32768

__device__ __forceinline__ bool better(double va, int ja, double vb, int jb) {
    return va > vb || (va == vb && ja < jb);
}
template <int K>
__device__ __forceinline__ void sel_argmax_step(double &bv, int &bj) {
    const double ov = lane_xd<K>(bv);
    const int oj = (int)lane_xu<K>((uint32_t)bj);
    if (better(ov, oj, bv, bj)) { bv = ov; bj = oj; }
}

// exclusive prefix sum over the 1024 threads (position order = thread order)
__device__ int block_excl_scan(int v, int *wsum, int *total) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    int incl = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        int y = __shfl_up(incl, o, 64);
        if (lane >= o) incl += y;
    }
    if (lane == 63) wsum[w] = incl;
    __syncthreads();
    if (threadIdx.x == 0) {
        int acc = 0;
        for (int i = 0; i < SEL_WAVES; ++i) {
            int x = wsum[i];
            wsum[i] = acc;
            acc += x;
        }
        *total = acc;
    }
    __syncthreads();
    int r = wsum[w] + incl - v;
    __syncthreads();
    return r;
}

__global__ void __launch_bounds__(SEL_THREADS) k_select(QrdmArgs a) {
    QrdmCtl *ctl = a.ctl;
    __shared__ double s_bv[SEL_WAVES];
    __shared__ int s_bj[SEL_WAVES];
    __shared__ int s_wsum[SEL_WAVES];
    __shared__ int s_total;
    __shared__ int s_hist[256];
    __shared__ unsigned long long s_prefix;
    __shared__ int s_krem;
    __shared__ int s_exact;
    __shared__ double s_cv[QK_KM];
    __shared__ int s_cj[QK_KM];
    __shared__ int s_branch;  // 0 = stop, 1 = single pivot, 2 = DM list
    __shared__ double s_umax;

    const int tid = threadIdx.x;
    if (qrdm_dm_idle(ctl)) return;
    if (ctl->nonfinite) {  // NaN/Inf in A (R15): nothing is written
        if (tid == 0) ctl->done = 1;
        return;
    }
    const int64_t ns = ctl->ns + ctl->l;
    const int64_t nblk = ctl->nblocks;
    const double amax0 = ctl->amax;  // read with the rest of the state, before the keys
    const int64_t rank0 = ctl->rank;
    __syncthreads();
    const int64_t p = p_of(a);
    if (tid == 0) {
        ctl->ns = ns;
        ctl->l = 0;
        ctl->ks = 0;
        ctl->nL = 0;
        ctl->nswap = 0;
    }
    if (ns >= p) {
        if (tid == 0) {
            ctl->done = 1;
            if (ctl->rank < 0) ctl->rank = ns;
        }
        return;
    }
    const int64_t w = a.n - ns;
    const int chunk = (int)((w + SEL_THREADS - 1) / SEL_THREADS);
    const int64_t j0 = ns + (int64_t)tid * chunk;
    double keys[SEL_KEYS];
#pragma unroll
    for (int q = 0; q < SEL_KEYS; ++q) {
        int64_t j = j0 + q;
        keys[q] = (q < chunk && j < a.n) ? a.vn1[j] : -1.0;  // -1 marks "no column"
    }
    // ---- max partial norm, lowest position on ties
    double bv = -1.0;
    int bj = 0x7fffffff;
#pragma unroll
    for (int q = 0; q < SEL_KEYS; ++q)
        if (keys[q] > bv) { bv = keys[q]; bj = (int)(j0 + q); }
    // over the wavefront (a total order: the tree does not matter)
    sel_argmax_step<32>(bv, bj);
    sel_argmax_step<16>(bv, bj);
    sel_argmax_step<8>(bv, bj);
    sel_argmax_step<7>(bv, bj);
    sel_argmax_step<2>(bv, bj);
    sel_argmax_step<1>(bv, bj);
    if ((tid & 63) == 0) { s_bv[tid >> 6] = bv; s_bj[tid >> 6] = bj; }
    __syncthreads();
    if (tid == 0) {
        double uv = s_bv[0];
        int uj = s_bj[0];
        for (int i = 1; i < SEL_WAVES; ++i)
            if (better(s_bv[i], s_bj[i], uv, uj)) { uv = s_bv[i]; uj = s_bj[i]; }
        double amax = amax0;
        if (nblk == 0) { amax = uv; ctl->amax = amax; }
        int branch = 2;
        if (amax == 0.0) {
            ctl->rank = 0;
            branch = 0;
        } else if (rank0 < 0) {
            double lhs = (a.stop_rule == 1) ? uv : sqrt((double)(a.n - ns)) * uv;
            if (lhs <= a.eps1 * amax) {
                ctl->rank = ns;
                if (a.stop_rule != 2) branch = 0;
            }
        }
        int64_t cap = a.kmax < (p - ns) ? a.kmax : (p - ns);
        if (branch == 2) {
            if (uv <= a.fbeps * amax) {
                // the rest is scalar pivoting: this step takes no block, and the
                // column-pivoting kernels start at exactly this n_s
                branch = 3;
                ctl->fallback = 1;
            } else if (cap == 1) {
                branch = 1;
            }
        }
        if (branch == 0) {
            ctl->done = 1;
        } else {
            ctl->umax = uv;
            ctl->jmax = uj;
            ctl->eps_s = a.tau * uv;
            if (branch != 3) ctl->nblocks = nblk + 1;
        }
        if (branch == 1) {
            ctl->L[0] = uj;
            ctl->nL = 1;
        }
        s_branch = branch;
        s_umax = uv;
    }
    __syncthreads();
    if (s_branch != 2) return;
    const double thr = a.tau * s_umax;
    const int cap = (int)(a.kmax < (p - ns) ? a.kmax : (p - ns));
    // ---- count candidates
    int cnt = 0;
#pragma unroll
    for (int q = 0; q < SEL_KEYS; ++q) cnt += (keys[q] >= thr) ? 1 : 0;
    int off = block_excl_scan(cnt, s_wsum, &s_total);
    const int total = s_total;
    int nsel;
    if (total <= cap) {
        int pos = off;
#pragma unroll
        for (int q = 0; q < SEL_KEYS; ++q)
            if (keys[q] >= thr) { s_cv[pos] = keys[q]; s_cj[pos] = (int)(j0 + q); ++pos; }
        nsel = total;
    } else {
        // radix select of the cap-th largest key (bit patterns of non-negative
        // doubles order like the values).  Every candidate lies in [thr, umax],
        // so its bits agree with those of umax down to the first bit where thr
        // and umax differ: the digits start below that common prefix.
        const unsigned long long bthr = (unsigned long long)__double_as_longlong(thr),
                                 bmax = (unsigned long long)__double_as_longlong(s_umax);
        int dec = bthr == bmax ? 64 : __clzll((long long)(bthr ^ bmax));  // bits decided
        unsigned long long pmask = dec == 0 ? 0ull : (dec >= 64 ? ~0ull : (~0ull << (64 - dec)));
        unsigned long long prefix = bmax & pmask;
        if (tid == 0) {
            s_krem = cap;
            s_exact = 0;
        }
        bool fin = dec >= 64;  // the same in every thread
        for (int pass = 0; pass < 8; ++pass) {
            if (fin) continue;
            // the last digit may overlap decided bits, which every key counted shares
            const int shift = 64 - dec - 8 > 0 ? 64 - dec - 8 : 0;
            if (tid < 256) s_hist[tid] = 0;
            __syncthreads();
#pragma unroll
            for (int q = 0; q < SEL_KEYS; ++q) {
                const unsigned long long kb = (unsigned long long)__double_as_longlong(keys[q]);
                const bool in = (keys[q] >= thr) && ((kb & pmask) == prefix);
                const int dg = (int)((kb >> shift) & 255);
                // lanes sharing the first active lane's digit add once (keys cluster
                // in few bins); the others add individually
                const unsigned long long act = __ballot(in);
                if (act) {
                    const int lead = __ffsll((long long)act) - 1;  // the same in every lane
                    const int ld = __builtin_amdgcn_readlane(dg, lead);
                    const unsigned long long same = __ballot(in && dg == ld);
                    if ((threadIdx.x & 63) == lead) atomicAdd(&s_hist[ld], __popcll(same));
                    if (in && dg != ld) atomicAdd(&s_hist[dg], 1);
                }
            }
            __syncthreads();
            if (tid < 64) {
                // bins in descending digit order; lane handles 4 consecutive
                const int krem = s_krem;
                int h[4];
                int ls = 0;
#pragma unroll
                for (int u = 0; u < 4; ++u) { h[u] = s_hist[255 - (4 * tid + u)]; ls += h[u]; }
                int incl = ls;
#pragma unroll
                for (int o = 1; o < 64; o <<= 1) {
                    int y = __shfl_up(incl, o, 64);
                    if (tid >= o) incl += y;
                }
                int excl = incl - ls;
                if (excl < krem && krem <= incl) {
                    int c = excl, found = 0, dig = 0, before = 0;
#pragma unroll
                    for (int u = 0; u < 4; ++u) {
                        const bool hit = !found && (c + h[u] >= krem);
                        if (hit) { found = 1; dig = 255 - (4 * tid + u); before = c; }
                        c += h[u];
                    }
                    s_krem = krem - before;
                    s_prefix = prefix | ((unsigned long long)dig << shift);
                    // every key of the chosen bin is needed: the set is decided
                    if (before + s_hist[dig] == krem) s_exact = 1;
                }
            }
            __syncthreads();
            prefix = s_prefix;
            pmask |= (255ull << shift);
            dec = 64 - shift;
            const int exact = s_exact;
            __syncthreads();
            fin = exact != 0 || dec >= 64;
        }
        // from here keys compare with the chosen bin [lo, hi] of the bits decided
        // so far (one value unless the loop stopped early, when the whole last
        // bin is taken)
        const unsigned long long lo = prefix, hi = prefix | ~pmask;
        const int need_eq = s_krem;  // keys equal to the cut value to take
        const int ngt = cap - need_eq;
        int cgt = 0, ceq = 0;
#pragma unroll
        for (int q = 0; q < SEL_KEYS; ++q) {
            if (keys[q] >= thr) {  // candidates only: a partly decided bin may reach below thr
                unsigned long long kb = (unsigned long long)__double_as_longlong(keys[q]);
                cgt += (kb > hi) ? 1 : 0;
                ceq += (kb >= lo && kb <= hi) ? 1 : 0;
            }
        }
        // one scan for both counts: keys above the cut number fewer than cap <= 128
        const int both = block_excl_scan(cgt | (ceq << 8), s_wsum, &s_total);
        int ogt = both & 0xff;
        int oeq = both >> 8;
#pragma unroll
        for (int q = 0; q < SEL_KEYS; ++q) {
            if (keys[q] >= thr) {  // candidates only: a partly decided bin may reach below thr
                unsigned long long kb = (unsigned long long)__double_as_longlong(keys[q]);
                if (kb > hi) {
                    s_cv[ogt] = keys[q]; s_cj[ogt] = (int)(j0 + q); ++ogt;
                } else if (kb >= lo && kb <= hi) {
                    if (oeq < need_eq) { s_cv[ngt + oeq] = keys[q]; s_cj[ngt + oeq] = (int)(j0 + q); }
                    ++oeq;
                }
            }
        }
        nsel = cap;
    }
    __syncthreads();
    // ---- order the list: norm descending, position ascending
    // rank of candidate i = tid / 8 among the list: eight threads count over
    // sixteen entries each, then sum within their group of eight lanes
    {
        const int i = tid >> 3, part = tid & 7;
        const bool mine = i < nsel;
        const double v = mine ? s_cv[i] : 0.0;
        const int j = mine ? s_cj[i] : 0;
        int r = 0;
        if (mine) {
#pragma unroll
            for (int u = 0; u < QK_KM / 8; ++u) {
                const int e = part * (QK_KM / 8) + u;
                if (e < nsel) r += better(s_cv[e], s_cj[e], v, j) ? 1 : 0;
            }
        }
        r += (int)lane_xu<1>((uint32_t)r);
        r += (int)lane_xu<2>((uint32_t)r);
        r += (int)lane_xu<7>((uint32_t)r);
        if (mine && part == 0) ctl->L[r] = j;
    }
    if (tid == 0) ctl->nL = nsel;
}

hipError_t launch_select(QrdmArgs a, hipStream_t s) {
    hipLaunchKernelGGL(k_select, dim3(1), dim3(SEL_THREADS), 0, s, a);
    return hipGetLastError();
}

// ================================================================ k_gram
#define GR_ROWS 128   // rows of C per workgroup

// Leading dimension of each partial Gram matrix: k_DM rounded up to the
// 16-wide MFMA tiles.
__host__ __device__ __forceinline__ int gram_ld(int kmax) { return ((kmax < QK_KM ? kmax : QK_KM) + 15) & ~15; }
#define GR_CHUNK 64   // rows staged in LDS at a time
#define GR_LD (GR_CHUNK + 1)

typedef double dbl4 __attribute__((ext_vector_type(4)));

__global__ void __launch_bounds__(256) k_gram(QrdmArgs a, double *Gp) {
    const QrdmCtl *ctl = a.ctl;
    if (qrdm_dm_idle(ctl)) return;
    const int nL = ctl->nL;
    if (nL <= 1) return;
    const int64_t ns = ctl->ns;
    const int64_t t = a.m - ns;
    const int64_t r0 = (int64_t)blockIdx.x * GR_ROWS;
    if (r0 >= t) return;
    __shared__ double Cs[QK_KM * GR_LD];
    __shared__ int sL[QK_KM];
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int nt = (nL + 15) >> 4;  // 16-wide tiles per dimension
    const int nLp = nt * 16;
    for (int q = tid; q < nLp; q += 256) sL[q] = (q < nL) ? ctl->L[q] : -1;
    dbl4 acc[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) acc[u] = dbl4{0.0, 0.0, 0.0, 0.0};
    const int ntiles = nt * nt;
    const int64_t rend = (r0 + GR_ROWS < t) ? r0 + GR_ROWS : t;
    __syncthreads();
    // chunk element u*256 + tid -> column q = u*4 + tid/64, row r = tid%64
    const int rr = tid & 63, qq = tid >> 6;
    double creg[32];
    auto fetch = [&](int64_t rc) {
        const int64_t row = rc + rr;
#pragma unroll
        for (int u = 0; u < 32; ++u) {
            const int q = u * 4 + qq;
            const int col = (q < nLp) ? sL[q] : -1;
            creg[u] = (col >= 0 && row < rend) ? a.A[(int64_t)col * a.lda + ns + row] : 0.0;
        }
    };
    fetch(r0);
    for (int64_t rc = r0; rc < rend; rc += GR_CHUNK) {
        __syncthreads();
#pragma unroll
        for (int u = 0; u < 32; ++u) {
            const int q = u * 4 + qq;
            if (q < nLp) Cs[q * GR_LD + rr] = creg[u];
        }
        __syncthreads();
        if (rc + GR_CHUNK < rend) fetch(rc + GR_CHUNK);
#pragma unroll
        for (int u = 0; u < 16; ++u) {
            const int tile = wv + 4 * u;
            if (tile < ntiles) {
                const int ti = tile / nt, tj = tile % nt;
                const double *ca = Cs + (ti * 16 + (lane & 15)) * GR_LD + (lane >> 4);
                const double *cb = Cs + (tj * 16 + (lane & 15)) * GR_LD + (lane >> 4);
#pragma unroll 4
                for (int k = 0; k < GR_CHUNK; k += 4) {
                    acc[u] = __builtin_amdgcn_mfma_f64_16x16x4f64(ca[k], cb[k], acc[u], 0, 0, 0);
                }
            }
        }
    }
    const int kp = gram_ld(a.kmax);
    double *out = Gp + (int64_t)blockIdx.x * kp * kp;
#pragma unroll
    for (int u = 0; u < 16; ++u) {
        const int tile = wv + 4 * u;
        if (tile < ntiles) {
            const int ti = tile / nt, tj = tile % nt;
            const int col = tj * 16 + (lane & 15);
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                // f64 16x16x4 MFMA: register v of lane holds D[4v + lane/16][lane%16]
                const int row = ti * 16 + 4 * v + (lane >> 4);
                out[row * kp + col] = acc[u][v];
            }
        }
    }
}

hipError_t launch_gram(QrdmArgs a, double *Gp, int64_t t_bound, hipStream_t s) {
    if (t_bound <= 0) return hipSuccess;
    dim3 grid((unsigned)((t_bound + GR_ROWS - 1) / GR_ROWS));
    hipLaunchKernelGGL(k_gram, grid, dim3(256), 0, s, a, Gp);
    return hipGetLastError();
}

int gram_partials(int64_t t_bound) { return (int)((t_bound + GR_ROWS - 1) / GR_ROWS); }

__global__ void __launch_bounds__(256) k_gram_reduce(QrdmArgs a, const double *Gp, double *G) {
    const QrdmCtl *ctl = a.ctl;
    if (qrdm_dm_idle(ctl)) return;
    const int nL = ctl->nL;
    if (nL <= 1) return;
    const int64_t t = a.m - ctl->ns;
    const int np = (int)((t + GR_ROWS - 1) / GR_ROWS);
    const int e = blockIdx.x * 256 + threadIdx.x;
    if (e >= nL * nL) return;
    const int i = e / nL, j = e % nL;
    // fixed order over the partials, sixteen loads in flight
    const int kp = gram_ld(a.kmax);
    double s = 0.0;
    for (int w0 = 0; w0 < np; w0 += 16) {
        double v[16];
#pragma unroll
        for (int u = 0; u < 16; ++u) v[u] = w0 + u < np ? Gp[(int64_t)(w0 + u) * kp * kp + i * kp + j] : 0.0;
#pragma unroll
        for (int u = 0; u < 16; ++u) s += v[u];
    }
    G[i * QK_KM + j] = s;
}

hipError_t launch_gram_reduce(QrdmArgs a, const double *Gp, double *G, int64_t t_bound, hipStream_t s) {
    (void)t_bound;
    int kk = a.kmax < QK_KM ? a.kmax : QK_KM;
    dim3 grid((unsigned)((kk * kk + 255) / 256));
    hipLaunchKernelGGL(k_gram_reduce, grid, dim3(256), 0, s, a, Gp, G);
    return hipGetLastError();
}

// ============================================================= k_dm_finish
__device__ __forceinline__ int sel4(int r0, int r1, int r2, int r3, int k) {
    return k == 0 ? r0 : (k == 1 ? r1 : (k == 2 ? r2 : r3));
}

__device__ __forceinline__ unsigned long long dm_readlane64(unsigned long long v, int l) {
    const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)v, l);
    const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(v >> 32), l);
    return ((unsigned long long)hi << 32) | lo;
}

__global__ void __launch_bounds__(256) k_dm_finish(QrdmArgs a, const double *G, double *theta_out) {
    QrdmCtl *ctl = a.ctl;
    if (qrdm_dm_idle(ctl)) return;
    __shared__ double sd[QK_KM];
    __shared__ double sG[QK_KM * QK_KM];
    __shared__ int sJ[QK_KM];
    __shared__ int sAi[QK_KM];  // candidate index (row of G) of each accepted column
    __shared__ unsigned long long sbad[QK_KM][2];  // bit j of row i: candidate j conflicts with i
    __shared__ int s_cont[QK_SWAP_MAX], s_pos[QK_SWAP_MAX];  // transposition bookkeeping (slots)
    __shared__ int soutpos[QK_KM];
    __shared__ double s_v1[QK_SWAP_MAX], s_v2[QK_SWAP_MAX];  // vn1, vn2 and perm by slot
    __shared__ int s_pm[QK_SWAP_MAX];
    __shared__ int s_ks;
    const int tid = threadIdx.x, lane = tid & 63;
    const int nL = ctl->nL;
    const int64_t ns = ctl->ns;
    if (nL > 1) {
        for (int base = 0; base < nL * nL; base += 256 * 8) {
            double v[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int e = base + u * 256 + tid;
                v[u] = (e < nL * nL) ? G[(e / nL) * QK_KM + (e % nL)] : 0.0;
            }
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int e = base + u * 256 + tid;
                if (e < nL * nL) sG[(e / nL) * QK_KM + (e % nL)] = v[u];
            }
        }
        __syncthreads();
        G = sG;
        for (int q = tid; q < nL; q += 256) sd[q] = sqrt(G[q * QK_KM + q]);
        __syncthreads();
        if (theta_out) {
            for (int e = tid; e < nL * nL; e += 256) {
                int i = e / nL, j = e % nL;
                theta_out[e] = G[i * QK_KM + j] / (sd[i] * sd[j]);
            }
        }
        // eq. (delta_max): delta <= tau^2 / (k_max - 1), k_max the candidate
        // count, puts every accepted block under the hypotheses of Lemma 1
        const double delta = a.certified ? fmin(a.delta, a.tau * a.tau / (double)(nL - 1)) : a.delta;
        // conflicts |theta_ij| >= delta (or undefined) of every candidate i with
        // every earlier j, as bit masks, all wavefronts in parallel
        // (four rows per wavefront at a time, every load and quotient issued
        // before the ballots: the divisions overlap; rows past nL are computed
        // on row nL - 1 and not stored)
        const double sdl0 = sd[lane], sdl1 = sd[lane + 64];
        for (int i0 = tid >> 6; i0 < nL; i0 += 16) {
            double q0[4], q1[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int i = min(i0 + 4 * u, nL - 1);
                const double di = sd[i];
                q0[u] = G[i * QK_KM + lane] / (di * sdl0);
                q1[u] = G[i * QK_KM + lane + 64] / (di * sdl1);
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int i = i0 + 4 * u;
                const bool bad0 = lane < i && !(fabs(q0[u]) < delta);
                const bool bad1 = lane + 64 < i && !(fabs(q1[u]) < delta);
                const unsigned long long m0 = __ballot(bad0), m1 = __ballot(bad1);
                if (lane == 0 && i < nL) {
                    sbad[i][0] = m0;
                    sbad[i][1] = m1;
                }
            }
        }
        __syncthreads();
        if (tid < 64) {
            // greedy acceptance in candidate order (Algorithm 1): candidate i joins
            // when it conflicts with no accepted candidate and its norm is nonzero;
            // lane L holds the masks of candidates L and L + 64
            const unsigned long long r00 = lane < nL ? sbad[lane][0] : 0ull;
            const unsigned long long r10 = lane + 64 < nL ? sbad[lane + 64][0] : 0ull;
            const unsigned long long r11 = lane + 64 < nL ? sbad[lane + 64][1] : 0ull;
            const bool pos0 = lane < nL && sd[lane] > 0.0, pos1 = lane + 64 < nL && sd[lane + 64] > 0.0;
            const unsigned long long p0 = __ballot(pos0), p1 = __ballot(pos1);
            unsigned long long A0 = 1ull, A1 = 0ull;
            const int nlo = nL < 64 ? nL : 64;
            for (int i = 1; i < nlo; ++i) {  // candidates 1..63: masks of lane i, first register pair
                const unsigned long long b0 = dm_readlane64(r00, i);
                if (((p0 >> i) & 1ull) && !(b0 & A0)) A0 |= 1ull << i;
            }
            for (int i = 64; i < nL; ++i) {  // candidates 64..: second register pair
                const int L = i - 64;
                const unsigned long long b0 = dm_readlane64(r10, L), b1 = dm_readlane64(r11, L);
                if (((p1 >> L) & 1ull) && !((b0 & A0) | (b1 & A1))) A1 |= 1ull << L;
            }
            const bool acc0 = (A0 >> lane) & 1ull, acc1 = (A1 >> lane) & 1ull;
            // compact accepted candidates in order
            unsigned long long b0 = __ballot(acc0), b1 = __ballot(acc1);
            int c0 = __popcll(b0);
            if (acc0) {
                const int o = __popcll(b0 & ((1ull << lane) - 1));
                sJ[o] = ctl->L[lane];
                sAi[o] = lane;
            }
            if (acc1) {
                const int o = c0 + __popcll(b1 & ((1ull << lane) - 1));
                sJ[o] = ctl->L[lane + 64];
                sAi[o] = lane + 64;
            }
            if (lane == 0) s_ks = c0 + __popcll(b1);
        }
    } else {
        if (tid == 0) { sJ[0] = ctl->L[0]; sAi[0] = 0; s_ks = 1; }
    }
    __syncthreads();
    const int ks = s_ks;
    // ---- Lemma 1 on the accepted columns (second wavefront, beside the swap
    // bookkeeping of the first): gamma = min_i (1 - sum_{j != i} |theta_ij|)
    // over J, tau_J = min_J ||c_j|| / max_J ||c_j||, bound sqrt(gamma + tau_J^2 - 1)
    // max_J ||c_j|| (row sums in the order of J).  Only the step log reads them.
    if (tid >= 64 && tid < 128 && a.lemma) {
        double cmax = 0.0, cmin = INFINITY, gmin = INFINITY;
        if (nL > 1) {
            // lane L holds accepted columns L and L + 64: their candidate index and norm
            const int aiv0 = lane < ks ? sAi[lane] : 0, aiv1 = lane + 64 < ks ? sAi[lane + 64] : 0;
            const double dv0 = sd[aiv0], dv1 = sd[aiv1];
            for (int i = lane; i < ks; i += 64) {
                const int ai = i < 64 ? aiv0 : aiv1;
                const double da = i < 64 ? dv0 : dv1;
                cmax = fmax(cmax, da);
                cmin = fmin(cmin, da);
                double rs = 0.0;
                for (int j0 = 0; j0 < ks; j0 += 8) {
                    double g[8], db[8];
#pragma unroll
                    for (int u = 0; u < 8; ++u) {
                        const int j = j0 + u;
                        const int bj = j < ks ? __builtin_amdgcn_readlane(j < 64 ? aiv0 : aiv1, j & 63) : 0;
                        const double d = __longlong_as_double(
                            ((long long)(unsigned)__builtin_amdgcn_readlane(
                                 (int)((unsigned long long)__double_as_longlong(j < 64 ? dv0 : dv1) >> 32), j & 63)
                             << 32) |
                            (unsigned)__builtin_amdgcn_readlane((int)__double_as_longlong(j < 64 ? dv0 : dv1), j & 63));
                        g[u] = j < ks ? G[ai * QK_KM + bj] : 0.0;
                        db[u] = d;
                    }
#pragma unroll
                    for (int u = 0; u < 8; ++u) {
                        const int j = j0 + u;
                        if (j < ks && j != i) rs += fabs(g[u] / (da * db[u]));
                    }
                }
                gmin = fmin(gmin, 1.0 - rs);
            }
#pragma unroll
            for (int o = 32; o > 0; o >>= 1) {
                cmax = fmax(cmax, __shfl_xor(cmax, o, 64));
                cmin = fmin(cmin, __shfl_xor(cmin, o, 64));
                gmin = fmin(gmin, __shfl_xor(gmin, o, 64));
            }
        } else {
            // one column: gamma = 1 and sigma_min = its norm over rows ns..m-1
            const double *col = a.A + (int64_t)ctl->L[0] * a.lda + ns;
            double s = 0.0;
            for (int64_t r = lane; r < a.m - ns; r += 64) s += col[r] * col[r];
            s = wave_sum(s);
            cmax = cmin = sqrt(s);
            gmin = 1.0;
        }
        if (lane == 0) {
            const double tj = cmax > 0.0 ? cmin / cmax : 0.0;
            const double slack = gmin + tj * tj - 1.0;
            ctl->gamma = gmin;
            ctl->sigma_bound = slack > 0.0 ? sqrt(slack) * cmax : 0.0;
        }
    }
    // ---- transpositions: for i = 0..ks-1 swap position ns+i with the current
    // position of column J_i.  Slots: 0..ks-1 = positions ns..ns+ks-1, then the
    // accepted columns outside that range in list order.
    if (tid < 64) {
        int nout = 0;
        int js0 = 0, js1 = 0;  // the slots of J_lane and J_{lane + 64}
        for (int base = 0; base < ks; base += 64) {
            const int i = base + lane;
            const bool valid = i < ks;
            const int jp = valid ? sJ[i] : 0;
            const bool outside = valid && (jp >= ns + ks);
            unsigned long long bo = __ballot(outside);
            const int oi = nout + __popcll(bo & ((1ull << lane) - 1));
            const int sl = outside ? ks + oi : (int)(jp - ns);
            if (valid && outside) soutpos[oi] = jp;
            if (base == 0) js0 = sl;
            else js1 = sl;
            nout += __popcll(bo);
        }
        const int nslots = ks + nout;
        // vn1, vn2 and perm of every slot, loaded before the transpositions so
        // that their latency overlaps them (every load before any store below)
        double pv1[4], pv2[4];
        int ppm[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int sl = lane + 64 * u;
            const int pos = (sl < ks) ? (int)(ns + sl) : (sl < nslots ? soutpos[sl - ks] : 0);
            if (sl < nslots) {
                pv1[u] = a.vn1[pos];
                pv2[u] = a.vn2[pos];
                ppm[u] = a.perm[pos];
            }
        }
        // cont[s]: slot whose original column sits in slot s; posof[c]: slot of
        // column c.  The transpositions are applied in order by the whole
        // wavefront on the same LDS words (same addresses, same values in every
        // lane): one LDS round trip per transposition.
        for (int u = 0; u < 4; ++u) {
            s_cont[lane + 64 * u] = lane + 64 * u;
            s_pos[lane + 64 * u] = lane + 64 * u;
        }
        for (int i = 0; i < ks; ++i) {
            const int js = __builtin_amdgcn_readlane(i < 64 ? js0 : js1, i & 63);
            const int q = s_pos[js];
            const int c = s_cont[i];
            s_cont[i] = js;
            s_cont[q] = c;
            s_pos[c] = q;
            s_pos[js] = i;
        }
        // the loaded values by slot
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int sl = lane + 64 * u;
            if (sl < nslots) {
                s_v1[sl] = pv1[u];
                s_v2[sl] = pv2[u];
                s_pm[sl] = ppm[u];
            }
        }
        // moves: slot s receives the column that was at slot cont[s] (one
        // wavefront: its LDS accesses complete in order)
        int nmv = 0;
        double ov1[4], ov2[4];
        int opm[4], dpos[4], spos[4];
        bool mv[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int sl = lane + 64 * u;
            const int cs = s_cont[sl];
            mv[u] = (sl < nslots) && (cs != sl);
            dpos[u] = (sl < ks) ? (int)(ns + sl) : (sl < nslots ? soutpos[sl - ks] : 0);
            spos[u] = (cs < ks) ? (int)(ns + cs) : (cs < nslots ? soutpos[cs - ks] : 0);
            if (mv[u]) {
                ov1[u] = s_v1[cs];
                ov2[u] = s_v2[cs];
                opm[u] = s_pm[cs];
            }
        }
        __builtin_amdgcn_s_barrier();  // single wave: orders the reads above before the writes
        __threadfence_block();
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            unsigned long long bm = __ballot(mv[u]);
            const int o = nmv + __popcll(bm & ((1ull << lane) - 1));
            if (mv[u]) {
                a.vn1[dpos[u]] = ov1[u];
                a.vn2[dpos[u]] = ov2[u];
                a.perm[dpos[u]] = opm[u];
                ctl->swp_dst[o] = dpos[u];
                ctl->swp_src[o] = spos[u];
            }
            nmv += __popcll(bm);
        }
        if (lane == 0) {
            ctl->nswap = nmv;
            ctl->ks = ks;
        }
        for (int i = lane; i < ks; i += 64) {
            ctl->J[i] = sJ[i];
            ctl->Ai[i] = sAi[i];
        }
    }
}

hipError_t launch_dm_finish(QrdmArgs a, const double *G, double *theta_out, hipStream_t s) {
    hipLaunchKernelGGL(k_dm_finish, dim3(1), dim3(256), 0, s, a, G, theta_out);
    return hipGetLastError();
}

// ================================================================= k_swap
// Column moves of a DM block on a 32-row band per workgroup (so that a
// factorization of 8192 rows fills 256 compute units): the eight 32-lane
// halves of the wavefronts move columns h, h+8, ... with one row per lane;
// every source is read into registers before any destination is written (a
// destination is often another move's source).  The bands are disjoint, so no
// two workgroups touch the same element.
#define SW_ROWS 32
#define SW_PER (QK_SWAP_MAX / 8)

__global__ void __launch_bounds__(256) k_swap(QrdmArgs a) {
    const QrdmCtl *ctl = a.ctl;
    if (blockIdx.x == 0 && threadIdx.x == 0) gbar_clear(a.gbar);  // for the panel launched next
    if (qrdm_dm_idle(ctl)) return;
    const int nsw = ctl->nswap;
    if (nsw == 0) return;
    const int64_t r0 = (int64_t)blockIdx.x * SW_ROWS;
    if (r0 >= a.m) return;
    __shared__ int sdst[QK_SWAP_MAX], ssrc[QK_SWAP_MAX];
    const int tid = threadIdx.x, rl = tid & 31, h = tid >> 5;
    for (int e = tid; e < nsw; e += 256) { sdst[e] = ctl->swp_dst[e]; ssrc[e] = ctl->swp_src[e]; }
    __syncthreads();
    const bool in = r0 + rl < a.m;
    double v[SW_PER];
#pragma unroll
    for (int u = 0; u < SW_PER; ++u) {
        const int e = h + 8 * u;
        v[u] = (e < nsw && in) ? a.A[(int64_t)ssrc[e] * a.lda + r0 + rl] : 0.0;
    }
    __builtin_amdgcn_s_waitcnt(0);  // every read has returned before any write
    __syncthreads();
#pragma unroll
    for (int u = 0; u < SW_PER; ++u) {
        const int e = h + 8 * u;
        if (e < nsw && in) a.A[(int64_t)sdst[e] * a.lda + r0 + rl] = v[u];
    }
}

hipError_t launch_swap(QrdmArgs a, hipStream_t s) {
    dim3 grid((unsigned)((a.m + SW_ROWS - 1) / SW_ROWS));
    hipLaunchKernelGGL(k_swap, grid, dim3(256), 0, s, a);
    return hipGetLastError();
}
