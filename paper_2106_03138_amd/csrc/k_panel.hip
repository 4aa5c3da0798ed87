// Householder panel of one QRDM block with the early break (Algorithm 4 of
// the paper, inner loop; threshold eps_s of eq. lenght_check), on gfx950.  It
// also records the inner products v_a^T v_i of the reflectors, from which the
// trailing update applies the compact WY form (Section 3.2) without forming
// its triangular factor.
//
// The k_s accepted columns (rows n_s..m-1) are split into row slabs, one per
// workgroup, held in LDS for the whole panel.  Every round of two panel
// columns (i, i+1) costs one grid-wide reduction: each workgroup contributes,
// in one vector,
//   Dall_j  = sum_{rows > c} x_r a_{r,j}            for every panel column j
//   Top_j   = a_{c,j}                               (row c of the diagonal)
//   Dall2_j = sum_{rows > c+1} a_{r,i+1} a_{r,j}
//   Top2_j  = a_{c+1,j}
// where x is column i.  From the reduced vector every workgroup derives,
// redundantly and identically, ||x|| (and the break decision), the reflector
// (LAPACK larfg convention: beta = -sign(alpha)||x||), the products v^T a_j of
// the in-panel update and the inner products v_a^T v_i; and the same for
// column i+1 after H_i, in closed form (see the round loop).  Reductions are
// in fixed order, so the run is bit-reproducible and every workgroup takes the
// same branch.
//
// All workgroups must be resident at once (launch_resident): the rounds are
// separated by the grid barrier gbar_wait.
#include "qrdm_internal.h"

#define PN_THREADS 512
#define PN_RB 4  // slab rows whose LDS loads are issued together in the row loops
#define PN_FLAGS 4096  // reserved words at the head of the partials buffer
#ifndef PN_MAX_ROWS
#define PN_MAX_ROWS 256  // tallest slab per workgroup
#endif
#ifndef PN_PREF_ROWS
#define PN_PREF_ROWS 128  // preferred slab height
#endif
#define PN_WAVES (PN_THREADS / 64)


__device__ __forceinline__ void st_coherent(double *p, double v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ double ld_coherent(const double *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

extern __shared__ double pn_lds[];

// Partial dots of one panel round for the lane's column jj: s = sum over rows
// >= r_a of S[r][i] S[r][jj], s2 = sum over rows >= r_b of S[r][i+1] S[r][jj]
// (PAIR), the rows of this wave taken in increasing order.  r0 is
// wave-uniform; PN_RB rows have their loads issued together.
template <bool PAIR>
__device__ __forceinline__ void pn_dots(const double *S, int ksp, int r0, int rb, int nrows, int i, int jj,
                                        double &s_out, double &s2_out) {
    double s = 0.0, s2 = 0.0;
    int r = r0;
    for (; r + (PN_RB - 1) * PN_WAVES < nrows; r += PN_RB * PN_WAVES) {
        double xa[PN_RB], xb[PN_RB], xj[PN_RB];
#pragma unroll
        for (int u = 0; u < PN_RB; ++u) {
            const double *row = S + (r + u * PN_WAVES) * ksp;
            xa[u] = row[i];
            xj[u] = row[jj];
            if (PAIR) xb[u] = row[i + 1];
        }
#pragma unroll
        for (int u = 0; u < PN_RB; ++u) {
            s += xa[u] * xj[u];
            if (PAIR && r + u * PN_WAVES >= rb) s2 += xb[u] * xj[u];
        }
    }
    for (; r < nrows; r += PN_WAVES) {
        const double *row = S + r * ksp;
        const double xj = row[jj];
        s += row[i] * xj;
        if (PAIR && r >= rb) s2 += row[i + 1] * xj;
    }
    s_out = s;
    s2_out = s2;
}

// Rank-one (H_i) or rank-two (H_i then H_{i+1}) update of the slab rows r0,
// r0 + PN_WAVES, ... (wave-uniform r0) in the lane's columns j0 = lane and, when
// TWO, j1 = lane + 64 (stored only if j1 < ks): v = x_r / den,
// vp = (a_{r,i+1} - v W_{i+1}) / den2; column i receives v, column i+1 vp,
// columns to the right a - v W_j - vp W2_j.  Both columns of a row are updated in
// the same pass (column i is rewritten), and all loads of PN_RB rows come before
// their stores.
template <bool PAIR, bool TWO>
__device__ __forceinline__ void pn_update(double *S, int ksp, int r0, int nrows, int i, int j0, int ks,
                                          double rden, double wn, double rden2, double wa0, double wb0, double wa1,
                                          double wb1) {
    const int j1 = j0 + 64;
    const bool st1 = TWO && j1 < ks;
    auto upd = [&](double x, double xn, double y, int j, double wa, double wb) -> double {
        const double v = x * rden;
        if (PAIR) {
            const double vp = (xn - v * wn) * rden2;
            return j == i ? v : (j == i + 1 ? vp : y - v * wa - vp * wb);
        }
        return j == i ? v : y - v * wa;
    };
    int r = r0;
    for (; r + (PN_RB - 1) * PN_WAVES < nrows; r += PN_RB * PN_WAVES) {
        double xa[PN_RB], xb[PN_RB], y0[PN_RB], y1[PN_RB];
#pragma unroll
        for (int u = 0; u < PN_RB; ++u) {
            const double *row = S + (r + u * PN_WAVES) * ksp;
            xa[u] = row[i];
            xb[u] = PAIR ? row[i + 1] : 0.0;
            y0[u] = row[j0];
            y1[u] = st1 ? row[j1] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < PN_RB; ++u) {
            double *row = S + (r + u * PN_WAVES) * ksp;
            row[j0] = upd(xa[u], xb[u], y0[u], j0, wa0, wb0);
            if (st1) row[j1] = upd(xa[u], xb[u], y1[u], j1, wa1, wb1);
        }
    }
    for (; r < nrows; r += PN_WAVES) {
        double *row = S + r * ksp;
        const double xa = row[i], xb = PAIR ? row[i + 1] : 0.0;
        const double y0 = row[j0], y1 = st1 ? row[j1] : 0.0;
        row[j0] = upd(xa, xb, y0, j0, wa0, wb0);
        if (st1) row[j1] = upd(xa, xb, y1, j1, wa1, wb1);
    }
}

__global__ void __launch_bounds__(PN_THREADS)
k_panel(QrdmArgs a, double *PB, double *VV, double *Vw, float *Vw32, int64_t ldv, int rows) {
    QrdmCtl *ctl = a.ctl;
    if (qrdm_dm_idle(ctl) || ctl->cpath) return;  // the Gram-matrix panel took the block
    const int64_t ns = ctl->ns;
    const int ks = ctl->ks;
    const double eps_s = ctl->eps_s;
    // PB: [PN_FLAGS] (unused) | [2][2 QK_KM] rows c, c+1 of the round |
    // [2][P][2 QK_KM] partial dots (double-buffered by round parity)
    double *topb = PB + PN_FLAGS / 2;
    double *part = topb + 4 * QK_KM;
    const int64_t t = a.m - ns;
    const int P = gridDim.x;
    const int wg = blockIdx.x;
    // the slabs depend on the trailing size t alone, whatever the grid, and so do
    // the partial dots and the bits of the result: ceil(t / rows) slabs of equal
    // height (the host sizes the grid from a bound on t; workgroups past the
    // last slab hold no rows)
    const int pact = (int)((t + rows - 1) / rows);  // slabs holding rows (<= P)
    const int rp = (int)((t + pact - 1) / pact);    // <= rows
    const int64_t g0 = ns + (int64_t)wg * rp;  // first global row of this slab
    int64_t nr64 = a.m - g0;
    if (nr64 < 0) nr64 = 0;
    const int nrows = (int)(nr64 < rp ? nr64 : rp);
    const int tid = threadIdx.x, lane = tid & 63;
    const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);  // wave-uniform

    const int ksp = ks + 1;                  // padded row stride of the slab
    double *S = pn_lds;                      // [rp][ksp] slab, row-major
    double *red = S + (size_t)rp * ksp;      // [PN_WAVES][QK_KM] partial dots of column i; reused for sums
    double *red2 = red + PN_WAVES * QK_KM;   // [PN_WAVES][QK_KM] partial dots of column i+1
    double *sR = red2 + PN_WAVES * QK_KM;    // reduced Dall of column i (rows > c)
    double *sTop = sR + QK_KM;               // reduced row c
    double *sG2 = sTop + QK_KM;              // reduced Dall of column i+1 (rows > c+1)
    double *sTop2 = sG2 + QK_KM;             // reduced row c+1
    double *sW = sTop2 + QK_KM;              // tau_i v_i^T a_j
    double *sW2 = sW + QK_KM;                // tau_{i+1} v_{i+1}^T (H_i a_j)

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

    // Rounds take two columns (i, i+1) while both remain: the reduced vector
    // then also holds Dall2_j = sum_{rows > c+1} a_{r,i+1} a_{r,j} and row c+1,
    // from which column i+1 after H_i, its reflector and v_{i+1}^T (H_i a_j)
    // follow in closed form (v_i is a combination of column i and e_c).  When
    // that closed form loses more than a factor 20 to cancellation, the round
    // applies H_i only and the next round starts from the updated column.
    int l = ks;
    uint32_t round = 0;
    for (int i = 0; i < ks;) {
        const bool pair = i + 1 < ks;
        const int nval = (pair ? 2 : 1) * ks;  // reduced values: Dall (and Dall2)
        int gpv = PN_THREADS / nval;  // thread groups per reduced value
        if (gpv > PN_WAVES / 2) gpv = PN_WAVES / 2;
        if (gpv < 1) gpv = 1;
        const int64_t c = ns + i;
        const int64_t cl64 = c - g0;
        const int cl = (cl64 >= 0 && cl64 < nrows) ? (int)cl64 : -1;          // local row of c
        const int cl2 = (cl64 + 1 >= 0 && cl64 + 1 < nrows) ? (int)(cl64 + 1) : -1;  // local row of c+1
        int rstart = (int)(cl64 + 1);
        if (rstart < 0) rstart = 0;
        int rstart2 = (int)(cl64 + 2);
        if (rstart2 < 0) rstart2 = 0;
        // ---- partial dots over rows strictly below c (column i) and below c+1
        // (column i+1)
        for (int jj = lane; jj < ks; jj += 64) {
            double s, s2 = 0.0;
            if (pair) pn_dots<true>(S, ksp, rstart + wv, rstart2, nrows, i, jj, s, s2);
            else pn_dots<false>(S, ksp, rstart + wv, rstart2, nrows, i, jj, s, s2);
            red[wv * QK_KM + jj] = s;
            red2[wv * QK_KM + jj] = s2;
        }
        __syncthreads();
        double *pb = part + ((size_t)(round & 1) * P + wg) * (2 * QK_KM);
        double *tb = topb + (size_t)(round & 1) * (2 * QK_KM);
        if (tid < nval) {
            const int seg = tid / ks, jj = tid - seg * ks;
            const double *rr = seg == 0 ? red : red2;
            double v = 0.0;
#pragma unroll
            for (int w = 0; w < PN_WAVES; ++w) v += rr[w * QK_KM + jj];
            st_coherent(pb + seg * QK_KM + jj, v);
        }
        // rows c and c+1 come from the one workgroup that holds each
        if (cl >= 0 && tid < ks) st_coherent(tb + tid, S[cl * ksp + tid]);
        if (pair && cl2 >= 0 && tid < ks) st_coherent(tb + QK_KM + tid, S[cl2 * ksp + tid]);
        gbar_wait(a.gbar, P, (uint32_t)round + 1u, &ctl->error);
        // ---- fixed-order reduction of all partials (every workgroup, identically)
        const double *pb0 = part + (size_t)(round & 1) * P * (2 * QK_KM);
        {
            const int my_e = tid % nval, my_g = tid / nval;
            const int wper = (pact + gpv - 1) / gpv;
            if (my_g < gpv) {
                const int seg = my_e / ks, jj = my_e - seg * ks;
                const int o = seg * QK_KM + jj;
                const int w0 = my_g * wper;
                const int w1 = (w0 + wper < pact) ? w0 + wper : pact;
                double s = 0.0;
                for (int wb = w0; wb < w1; wb += 16) {
                    double v[16];
#pragma unroll
                    for (int u = 0; u < 16; ++u)
                        v[u] = (wb + u < w1) ? ld_coherent(pb0 + (size_t)(wb + u) * (2 * QK_KM) + o) : 0.0;
#pragma unroll
                    for (int u = 0; u < 16; ++u) s += v[u];
                }
                red[my_g * nval + my_e] = s;
            }
            if (tid < ks) {
                sTop[tid] = ld_coherent(tb + tid);
                if (pair) sTop2[tid] = ld_coherent(tb + QK_KM + tid);
            }
        }
        __syncthreads();
        if (tid < nval) {
            double s = 0.0;
            for (int g = 0; g < gpv; ++g) s += red[g * nval + tid];
            const int seg = tid / ks, jj = tid - seg * ks;
            (seg == 0 ? sR : sG2)[jj] = s;
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
        const double rden = 1.0 / den;  // one reciprocal per reflector (larfg scales by it)
        // ---- column i+1 after H_i, from the reduced sums (every workgroup identically):
        //   v_i[c+1] = Top2_i / den,  Q = sum_{r>c+1} v_i[r]^2,  P_j = sum_{r>c+1} v_i[r] a_{r,j}
        //   alpha2 = Top2_{i+1} - v_i[c+1] W_{i+1},  sp2 = Dall2_{i+1} - 2 W_{i+1} P_{i+1} + W_{i+1}^2 Q
        int npiv = 1;
        bool brk2 = false;
        double vc1 = 0.0, q2 = 0.0, p1 = 0.0, beta2 = 0.0, ti2 = 0.0, den2 = 1.0;
        const double wn = pair ? ti * (sTop[i + 1] + sR[i + 1] * rden) : 0.0;  // W_{i+1} = tau_i v_i^T a_{i+1}
        if (pair) {
            vc1 = sTop2[i] * rden;
            q2 = (sR[i] - sTop2[i] * sTop2[i]) * (rden * rden);
            p1 = (sR[i + 1] - sTop2[i] * sTop2[i + 1]) * rden;
            const double alpha2 = sTop2[i + 1] - vc1 * wn;
            // a column i+1 whose top is the last row has nothing below it: larfg
            // leaves it alone (tau = 0, beta = alpha), so its sum of squares is
            // zero exactly, not the rounding residue of the closed form
            const bool last = c + 2 >= a.m;
            const double sp2 = last ? 0.0 : sG2[i + 1] - 2.0 * wn * p1 + wn * wn * q2;
            const double mag = last ? 0.0 : sG2[i + 1] + 2.0 * fabs(wn * p1) + wn * wn * q2;
            if (sp2 >= 0.05 * mag) {
                const double nrm2 = sqrt(alpha2 * alpha2 + sp2);
                if (nrm2 < eps_s) {
                    brk2 = true;  // column i+1 fails the length check after H_i
                } else {
                    npiv = 2;
                    if (sp2 == 0.0) {
                        ti2 = 0.0;
                        beta2 = alpha2;
                        den2 = 1.0;
                    } else {
                        beta2 = (alpha2 >= 0.0) ? -nrm2 : nrm2;
                        ti2 = (beta2 - alpha2) / beta2;
                        den2 = alpha2 - beta2;
                    }
                }
            }
        }
        const double rden2 = 1.0 / den2;
        for (int jj = i + 1 + tid; jj < ks; jj += PN_THREADS) {
            const double wj = ti * (sTop[jj] + sR[jj] * rden);
            sW[jj] = wj;
            if (npiv == 2 && jj > i + 1) {
                const double pj = (sR[jj] - sTop2[i] * sTop2[jj]) * rden;
                const double topp = sTop2[jj] - vc1 * wj;                              // (H_i a_j) at row c+1
                const double dp = sG2[jj] - wj * p1 - wn * pj + wn * wj * q2;        // sum_{r>c+1} x'_r (H_i a_j)_r
                sW2[jj] = ti2 * (topp + dp * rden2);
            }
        }
        if (wg == 0) {
            // inner products v_a^T v_i = Top_a + Dall_a / den (a < i) of the
            // compact WY form; the trailing update uses them with tau instead of
            // forming T explicitly
            if (tid < i) VV[tid * QK_KM + i] = sTop[tid] + sR[tid] * rden;
            if (tid == 0) a.tau_house[c] = ti;
            if (npiv == 2) {
                // v_a^T v_{i+1} = v_a[c+1] + (sum_{r>c+1} v_a[r] a_{r,i+1} - W_{i+1} sum_{r>c+1} v_a[r] v_i[r]) / den2
                if (tid < i) {
                    const double pa = (sR[tid] - sTop2[i] * sTop2[tid]) * rden;
                    VV[tid * QK_KM + i + 1] = sTop2[tid] + (sG2[tid] - wn * pa) * rden2;
                }
                if (tid == i) VV[i * QK_KM + i + 1] = vc1 + (p1 - wn * q2) * rden2;
                if (tid == 0) a.tau_house[c + 1] = ti2;
            }
        }
        __syncthreads();
        // ---- apply H_i (and H_{i+1}) to the slab.  v = x / (alpha - beta) is
        // formed with one reciprocal per round, as LAPACK larfg scales by it.
        // Rows below c (H_i alone) or below c+1 (both), then the diagonal rows.
        if (lane < ks) {  // lanes past the panel's columns store nothing
            const int rfirst = (npiv == 2 ? rstart2 : rstart) + wv;
            const int j0 = lane, j1 = lane + 64;
            const double wa0 = j0 > i ? sW[j0] : 0.0;
            const double wb0 = (npiv == 2 && j0 > i + 1) ? sW2[j0] : 0.0;
            const double wa1 = (j1 < ks && j1 > i) ? sW[j1] : 0.0;
            const double wb1 = (npiv == 2 && j1 < ks && j1 > i + 1) ? sW2[j1] : 0.0;
            if (ks > 64) {
                if (npiv == 2) pn_update<true, true>(S, ksp, rfirst, nrows, i, j0, ks, rden, wn, rden2, wa0, wb0, wa1, wb1);
                else pn_update<false, true>(S, ksp, rfirst, nrows, i, j0, ks, rden, wn, rden2, wa0, wb0, wa1, wb1);
            } else {
                if (npiv == 2) pn_update<true, false>(S, ksp, rfirst, nrows, i, j0, ks, rden, wn, rden2, wa0, wb0, wa1, wb1);
                else pn_update<false, false>(S, ksp, rfirst, nrows, i, j0, ks, rden, wn, rden2, wa0, wb0, wa1, wb1);
            }
        }
        if (npiv == 2 && cl2 >= 0 && wv == (cl2 % PN_WAVES)) {
            // row c+1: H_i, then H_{i+1} with this row as its diagonal row
            double *row = S + cl2 * ksp;
            const double v = row[i] * rden;
            for (int jj = lane; jj < ks; jj += 64) {
                const double y = row[jj];
                const double nv = jj == i ? v : (jj == i + 1 ? beta2 : y - (jj > i ? v * sW[jj] : 0.0) -
                                                                       (jj > i + 1 ? sW2[jj] : 0.0));
                row[jj] = nv;
            }
        }
        if (cl >= 0 && wv == (cl % PN_WAVES)) {
            for (int jj = lane; jj < ks; jj += 64)
                if (jj > i) S[cl * ksp + jj] -= sW[jj];
            if (lane == 0) S[cl * ksp + i] = beta;
        }
        __syncthreads();
        i += npiv;
        ++round;
        if (brk2) {
            l = i;  // H_i applied; column i+1 is the break
            break;
        }
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

#define PN_LDS_BUDGET (156 * 1024)
#define PN_LDS_FIXED ((2 * PN_WAVES + 6) * QK_KM)  // doubles besides the slab

int panel_lds_bytes(int rows_per_wg, int kmax) {
    return (rows_per_wg * (kmax + 1) + PN_LDS_FIXED) * (int)sizeof(double);
}

// Tallest slab (multiple of 16 rows, at most PN_MAX_ROWS) whose LDS fits in the budget.
int panel_rows_per_wg(int kmax) {
    const int budget = PN_LDS_BUDGET / (int)sizeof(double) - PN_LDS_FIXED;
    int r = budget / (kmax + 1);
    if (r > PN_MAX_ROWS) r = PN_MAX_ROWS;
    r &= ~15;
    return r < 16 ? 16 : r;
}

int panel_max_wgs(int rows_per_wg) {
    (void)rows_per_wg;
    static int cus[64] = {0};  // per device, queried once
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 1;
    if (cus[dev] == 0) {
        hipDeviceProp_t prop;
        if (hipGetDeviceProperties(&prop, dev) != hipSuccess) return 1;
        cus[dev] = prop.multiProcessorCount;
    }
    return cus[dev];
}

// Slab height for an m-row panel: PN_PREF_ROWS (shorter slabs mean less LDS work
// per round for more partials to gather; 128 measured fastest at 8192 rows),
// taller when that many workgroups would not all be co-resident (one per CU),
// never above the LDS budget.
int panel_rows_for(int64_t m, int kmax) {
    const int cap = panel_rows_per_wg(kmax);
    int r = PN_PREF_ROWS < cap ? PN_PREF_ROWS : cap;
    const int ncu = panel_max_wgs(r);
    while (r < cap && (m + r - 1) / r > ncu) r += 16;
    return r;
}

hipError_t launch_panel(QrdmArgs a, double *PB, double *VV, double *Vw, float *Vw32, int64_t ldv,
                        int64_t t_bound, int rows_per_wg, hipStream_t s) {
    if (t_bound <= 0) return hipSuccess;
    int P = (int)((t_bound + rows_per_wg - 1) / rows_per_wg);
    if (P < 1) P = 1;
    if (P > PN_THREADS || P > PN_FLAGS) return hipErrorInvalidValue;  // one polling thread per workgroup
    const int kk = a.kmax < QK_KM ? a.kmax : QK_KM;
    const int lds = panel_lds_bytes(rows_per_wg, kk);
    static bool attr_set = false;
    if (!attr_set) {
        hipError_t e = hipFuncSetAttribute((const void *)k_panel, hipFuncAttributeMaxDynamicSharedMemorySize, PN_LDS_BUDGET);
        if (e != hipSuccess) return e;
        attr_set = true;
    }
    void *args[] = {&a, &PB, &VV, &Vw, &Vw32, &ldv, &rows_per_wg};
    return launch_resident((const void *)k_panel, dim3(P), dim3(PN_THREADS), args, (unsigned)lds, s);
}
