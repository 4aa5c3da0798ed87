/*
 * Plain FP64 CPU oracle for QRDM (QR with Deviation Maximization pivoting,
 * Dessole & Marcuzzi, arXiv 2106.03138) and for QRP (QR with column pivoting).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, obviously-correct
 * reference that the GPU library is checked against.  Only the test suite,
 * the smoke check and the CPU-baseline leg of the benchmark may load it.  It
 * shares no code, header, table or constant with the GPU library.
 *
 * Every function follows the paper's steps in the paper's order:
 *   - Algorithm 1 (Deviation Maximization, DM) for the block column choice,
 *     with the candidate set of eq. (def_candidate_set) truncated to the block
 *     size k_DM as in eq. (candidate_set_limited_by_kDM), Section 4;
 *   - Algorithm 4 (QRDM2, the modified QRDM of Section 4) for the outer loop,
 *     with the Householder-panel break of its check step and the threshold
 *     eps_s of eq. (lenght_check);
 *   - Algorithm 2 (QRP) is the same loop with one pivot per step;
 *   - the compact WY form (Section 3.2, Schreiber & Van Loan) for the block
 *     trailing update;
 *   - the block partial-norm update of Section 3.2 (the equation after
 *     Algorithm 3), made cancellation-safe as the paper requires (reference
 *     DBu08 cited in Section 3.1): downdate, and recompute the norm from the
 *     data when the downdate has lost too much accuracy;
 *   - the practical stopping criterion eq. (practical stopping criterion)
 *     with eps_1 = eps*n, eq. (..._choice1), Section 3.4;
 *   - the switch to scalar pivoting when max ||c_i|| = O(eps), eq.
 *     (column_norm_bound_DM), Section 4.
 *
 * Readings where the paper is silent or garbled (listed with reasons in the
 * design notes of the repository):
 *   R1  u holds column norms (not squared norms);
 *   R2  arg-max ties go to the lowest current position;
 *   R3  candidates are visited in order (norm desc, position asc);
 *   R4  the block size k_DM caps the candidate list INCLUDING the arg-max;
 *   R5  Theta is formed over the candidate list (arg-max included), with the
 *       exact column norms d_i = sqrt(G_ii);
 *   R6  u_i >= tau*max u is non-strict; |theta| < delta and the break test
 *       ||x|| < eps_s are strict;
 *   R7  the downdate sums the l new rows of R, and uses the DBu08 rule:
 *       q = max(0, 1 - s/vn1^2), q2 = q*(vn1/vn2)^2, recompute if q2 <= sqrt(eps);
 *   R8  swaps track current positions; whole columns move;
 *   R9  LAPACK larfg sign convention, beta = -sign(alpha)*||x||, sign(0) = +;
 *   R10 in-panel update covers only the k_s panel columns; the WY update
 *       covers the columns from n_s+k_s on;
 *   R11 the break test applies to every panel column after the first;
 *   R12 eps_s = tau * max_i u_i (same value as the candidate threshold);
 *   R13 fall back to scalar pivoting when umax <= eps*n*amax;
 *   R14 stop rule tested at the top of every outer step; eps = 2^-52;
 *   R15 amax == 0 -> rank 0; NaN/Inf -> error, nothing written.
 *
 * Build: gcc -O2 -fPIC -shared -ffp-contract=off -fopenmp (see build_oracle.py).
 */
#include <float.h>
#ifdef _OPENMP
#include <omp.h>
#endif
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define O_EPS DBL_EPSILON /* 2^-52 (R14) */

#define O_STOP_PAPER 0   /* sqrt(n-ns)*umax <= eps1*amax, then stop          */
#define O_STOP_MAXNORM 1 /* umax <= eps1*amax, then stop                      */
#define O_STOP_NONE 2    /* full factorization; rank from the PAPER test      */

#define O_ERR_ARG (-100) /* generic argument error base: -1..-99 = arg index */
#define O_ERR_NONFINITE 1
#define O_ERR_NOMEM 2

/* One record per outer step (block).  Margins are relative distances of the
 * quantity that decided a branch from its threshold (large = robust). */
typedef struct {
    int64_t ns;        /* columns factored before this block               */
    int32_t ncand;     /* #{j >= ns : vn1_j >= tau*umax}                    */
    int32_t nL;        /* candidate list length after truncation           */
    int32_t ks;        /* accepted columns (|J|)                            */
    int32_t l;         /* reflectors kept (after the break)                */
    int32_t fallback;  /* 1 = scalar pivoting step                          */
    int32_t jmax;      /* arg-max position                                 */
    double umax;       /* max partial norm                                 */
    double eps_s;      /* break threshold tau*umax                          */
    double m_order;    /* order decisions: arg-max and candidate sort/cut  */
    double m_thr;      /* candidate threshold                              */
    double m_cos;      /* greedy |theta| vs delta                           */
    double m_break;    /* panel break test                                 */
    double m_stop;     /* stop test (while rank undecided)                 */
    double m_fb;       /* fallback test                                    */
    double m_recomp;   /* DBu08 recompute decisions                        */
    double gamma;      /* Lemma 1: min_i (1 - sum_{j != i} |theta_ij|) over J */
    double sigma_bound;/* Lemma 1: sqrt(gamma + tau_J^2 - 1) max_J ||c_j||,
                          tau_J = min_J ||c_j|| / max_J ||c_j||; 0 when
                          gamma <= 1 - tau_J^2 (the lemma does not apply)   */
} oracle_block;

typedef struct {
    double tau, delta;
    int32_t kmax;
    int32_t stop_rule;
    double eps1_scale; /* eps_1 = eps1_scale * eps; <= 0 means n */
    int64_t max_ns;    /* stop after ns >= max_ns (bounded runs); <0 = off */
    int32_t certified; /* 1 = delta <= tau^2 / (|L| - 1) per block, eq. (delta_max) */
    int32_t plant;     /* 0 in every real use.  The tests set one of the O_PLANT_*
                          mistakes below to show that their checks catch it.      */
} oracle_params;

/* Deliberate mistakes, for the tests of the checks only (never a reading):   */
#define O_PLANT_SINGLE 1   /* every DM step keeps only the arg-max column         */
#define O_PLANT_TRUNC 2    /* the panel stops after half of the accepted columns  */
#define O_PLANT_ACCEPT 3   /* greedy acceptance skips the |theta| < delta test    */
#define O_PLANT_NOBREAK 4  /* the panel never breaks (eq. lenght_check ignored)   */
#define O_PLANT_FBSCALE 5  /* scalar-pivoting switch at eps*amax, without the n   */
#define O_PLANT_DNORM 6    /* cosines scaled by the downdated norms, not sqrt(G_ii) */
#define O_PLANT_REJECT 7   /* the last candidate that passes the test is dropped  */

static double sq(double x) { return x * x; }

static double rel_margin(double a, double b) {
    double s = fabs(b);
    if (s == 0.0) return (a == b) ? 0.0 : INFINITY;
    return fabs(a - b) / s;
}

/* Margin of a decision between a and b when both carry an absolute rounding
 * noise of about nu: 0 if |a - b| <= nu (a noise-level decision, which two
 * correct implementations may take differently), else the relative margin. */
static double noise_margin(double a, double b, double nu) {
    if (fabs(a - b) <= nu) return 0.0;
    return rel_margin(a, b);
}

/* Column 2-norm of x[0..len): plain sum of squares (R9). */
static double norm2(const double *x, int64_t len) {
    double s = 0.0;
    for (int64_t i = 0; i < len; ++i) s += x[i] * x[i];
    return sqrt(s);
}

/* Sort helper for the candidate list: norm descending, position ascending (R3). */
typedef struct { double v; int64_t j; } cand_t;
static int cand_cmp(const void *pa, const void *pb) {
    const cand_t *a = (const cand_t *)pa, *b = (const cand_t *)pb;
    if (a->v > b->v) return -1;
    if (a->v < b->v) return 1;
    return (a->j < b->j) ? -1 : (a->j > b->j);
}

/*
 * Deviation Maximization, Algorithm 1, on the trailing matrix
 * [A]_{ns:m, ns:n} with partial norms vn1 (Section 2; Section 4 for the
 * truncation to k_DM and the Gram-then-scale way of forming Theta, option (ii)).
 *
 * Writes the ordered candidate list L (|L| = *nL <= cap), the cosine matrix
 * theta (nL x nL, row-major, may be NULL), and the accepted list J (*ks).
 * Margins of the decisions are written into rec when it is not NULL.
 */
static void dm_select(const double *A, int64_t m, int64_t n, int64_t lda, int64_t ns,
                      const double *vn1, double tau, double delta, int64_t cap, int certified,
                      int64_t *L, int *nL, double *theta, int64_t *J, int *ks,
                      oracle_block *rec, cand_t *work, double *G, double nu, int plant) {
    int64_t t = m - ns;
    /* step 1: J = { argmax u }, lowest position on ties (R2) */
    int64_t jmax = ns;
    double umax = vn1[ns];
    for (int64_t j = ns + 1; j < n; ++j)
        if (vn1[j] > umax) { umax = vn1[j]; jmax = j; }
    /* step 2: candidate set u_j >= tau*max u, eq. (def_candidate_set), R6 */
    double thr = tau * umax;
    int64_t nc = 0;
    double mthr = INFINITY;
    for (int64_t j = ns; j < n; ++j) {
        mthr = fmin(mthr, noise_margin(vn1[j], thr, nu));
        if (vn1[j] >= thr) { work[nc].v = vn1[j]; work[nc].j = j; ++nc; }
    }
    /* Section 4: order by norm (sort), keep the first min(k, k_DM) (R3, R4) */
    qsort(work, (size_t)nc, sizeof(cand_t), cand_cmp);
    int64_t nl = nc < cap ? nc : cap;
    double morder = INFINITY;
    int64_t nchk = nc < cap + 1 ? nc : cap + 1;
    for (int64_t a = 0; a + 1 < nchk; ++a) morder = fmin(morder, noise_margin(work[a + 1].v, work[a].v, nu));
    for (int64_t a = 0; a < nl; ++a) L[a] = work[a].j;
    *nL = (int)nl;
    /* step 4: cosine matrix, Theta = D^-1 (C^T C) D^-1 with C = [A]_{ns:m, L} (R5) */
    for (int64_t a = 0; a < nl; ++a) {
        for (int64_t b = 0; b < nl; ++b) {
            const double *ca = A + L[a] * lda + ns;
            const double *cb = A + L[b] * lda + ns;
            double s = 0.0;
            for (int64_t r = 0; r < t; ++r) s += ca[r] * cb[r];
            G[a * nl + b] = s;
        }
    }
    if (plant == O_PLANT_DNORM) {
        /* the planted mistake: D from the partial-norm estimates */
        for (int64_t a = 0; a < nl; ++a)
            for (int64_t b = 0; b < nl; ++b)
                if (a != b) G[a * nl + b] *= sqrt(G[a * nl + a] * G[b * nl + b]) / (vn1[L[a]] * vn1[L[b]]);
    }
    for (int64_t a = 0; a < nl; ++a) {
        for (int64_t b = 0; b < nl; ++b) {
            double da = sqrt(G[a * nl + a]), db = sqrt(G[b * nl + b]);
            double th = (da > 0.0 && db > 0.0) ? G[a * nl + b] / (da * db) : NAN;
            if (theta) theta[a * nl + b] = th;
        }
    }
    /* eq. (delta_max): with delta <= tau^2 / (k_max - 1), k_max the candidate
     * count, every accepted block meets the hypotheses of Lemma 1 */
    if (certified && nl > 1) {
        double dmax = tau * tau / (double)(nl - 1);
        if (dmax < delta) delta = dmax;
    }
    /* steps 5-7: greedy acceptance |theta_ij| < delta for all j in J (R6) */
    J[0] = L[0];
    int k = 1;
    double mcos = INFINITY;
    int64_t last_ok = -1; /* O_PLANT_REJECT: list index of the last accepted candidate */
    for (int64_t a = 1; a < nl; ++a) {
        double worst = 0.0;
        int ok = 1;
        double da = sqrt(G[a * nl + a]);
        if (!(da > 0.0)) ok = 0;
        for (int b = 0; b < k && ok; ++b) {
            /* index of J[b] inside L */
            int64_t bi = 0;
            while (L[bi] != J[b]) ++bi;
            double db = sqrt(G[bi * nl + bi]);
            double th = fabs(G[a * nl + bi] / (da * db));
            if (th > worst) worst = th;
            if (!(th < delta)) ok = 0;
        }
        if (da > 0.0) {
            /* a cosine of columns of norm d carries an error of about nu/d */
            double dmin = da;
            for (int b = 0; b < k; ++b) {
                int64_t bi = 0;
                while (L[bi] != J[b]) ++bi;
                dmin = fmin(dmin, sqrt(G[bi * nl + bi]));
            }
            double mc = fabs(worst - delta);
            mcos = fmin(mcos, (mc <= nu / dmin) ? 0.0 : mc);
        }
        if (plant == O_PLANT_ACCEPT && da > 0.0) ok = 1;
        if (ok) { J[k++] = L[a]; last_ok = a; }
    }
    if (plant == O_PLANT_REJECT && last_ok > 0) --k; /* drop the last accepted candidate */
    if (plant == O_PLANT_SINGLE) k = 1;
    *ks = k;
    /* Lemma 1 on C = [A]_{ns:m, J}: gamma of the cosine matrix of J and the
     * lower bound of sigma_min(C), with tau_J the actual norm ratio inside J */
    double cmax = 0.0, cmin = INFINITY, gam = INFINITY;
    for (int a = 0; a < k; ++a) {
        int64_t ai = 0;
        while (L[ai] != J[a]) ++ai;
        double da = sqrt(G[ai * nl + ai]);
        cmax = fmax(cmax, da);
        cmin = fmin(cmin, da);
        double rs = 0.0;
        for (int b = 0; b < k; ++b) {
            if (b == a) continue;
            int64_t bi = 0;
            while (L[bi] != J[b]) ++bi;
            rs += fabs(G[ai * nl + bi] / (da * sqrt(G[bi * nl + bi])));
        }
        gam = fmin(gam, 1.0 - rs);
    }
    double tj = cmax > 0.0 ? cmin / cmax : 0.0;
    double slack = gam + tj * tj - 1.0;
    if (rec) {
        rec->gamma = gam;
        rec->sigma_bound = slack > 0.0 ? sqrt(slack) * cmax : 0.0;
    }
    if (rec) {
        rec->ncand = (int32_t)nc;
        rec->nL = (int32_t)nl;
        rec->jmax = (int32_t)jmax;
        rec->umax = umax;
        rec->m_order = morder;
        rec->m_thr = mthr;
        rec->m_cos = (nl > 1) ? mcos : INFINITY;
    }
}

/* Swap whole columns a and b of A (all m rows), and the bookkeeping (R8). */
static void swap_cols(double *A, int64_t m, int64_t lda, double *vn1, double *vn2, int32_t *perm,
                      int64_t a, int64_t b) {
    if (a == b) return;
    double *ca = A + a * lda, *cb = A + b * lda;
    for (int64_t r = 0; r < m; ++r) { double x = ca[r]; ca[r] = cb[r]; cb[r] = x; }
    double x = vn1[a]; vn1[a] = vn1[b]; vn1[b] = x;
    x = vn2[a]; vn2[a] = vn2[b]; vn2[b] = x;
    int32_t p = perm[a]; perm[a] = perm[b]; perm[b] = p;
}

/*
 * QRDM2 (Algorithm 4) with DM (Algorithm 1).  kmax == 1 is QRP (Algorithm 2).
 *
 * A is m x n column-major (lda >= m), overwritten with R on and above the
 * diagonal and the Householder vectors (unit leading entry implicit) below it.
 * tau_house[min(m,n)], perm[n] (0-based, A_in[:, perm] = Q R), *rank.
 * log (may be NULL) receives up to log_cap block records; *nblocks the count.
 * Returns 0, a negative argument index, or a positive error code.
 */
int oracle_qrdm(double *A, int64_t m, int64_t n, int64_t lda, const oracle_params *prm,
                double *tau_house, int32_t *perm, int64_t *rank_out,
                oracle_block *log, int64_t log_cap, int64_t *nblocks) {
    if (m < 0) return -2;
    if (n < 0) return -3;
    if (lda < (m > 1 ? m : 1)) return -4;
    if (!prm) return -5;
    /* tau = 0 (a corner of the grid study of Section 5) admits every column */
    if (!(prm->tau >= 0.0 && prm->tau <= 1.0)) return -5;
    if (!(prm->delta >= 0.0 && prm->delta <= 1.0)) return -5;
    if (prm->kmax < 1) return -5;
    if (prm->stop_rule < 0 || prm->stop_rule > 2) return -5;
    if (n > 0 && m > 0 && (!A || !perm || !tau_house)) return -1;
    if (!rank_out) return -8;

    const int64_t p = m < n ? m : n;
    const double eps1 = (prm->eps1_scale > 0.0 ? prm->eps1_scale : (double)n) * O_EPS;
    const double tol3z = sqrt(O_EPS);
    int64_t nb = 0;

    /* NaN/Inf check before any write (R15) */
    for (int64_t j = 0; j < n; ++j)
        for (int64_t r = 0; r < m; ++r)
            if (!isfinite(A[j * lda + r])) return O_ERR_NONFINITE;

    for (int64_t j = 0; j < n; ++j) perm[j] = (int32_t)j;
    for (int64_t i = 0; i < p; ++i) tau_house[i] = 0.0;
    if (nblocks) *nblocks = 0;
    if (p == 0) { *rank_out = 0; return 0; }

    int64_t kcap = prm->kmax;
    double *vn1 = malloc(sizeof(double) * (size_t)n);
    double *vn2 = malloc(sizeof(double) * (size_t)n);
    int64_t *L = malloc(sizeof(int64_t) * (size_t)kcap);
    int64_t *J = malloc(sizeof(int64_t) * (size_t)kcap);
    double *G = malloc(sizeof(double) * (size_t)(kcap * kcap));
    double *T = malloc(sizeof(double) * (size_t)(kcap * kcap));
    double *VV = malloc(sizeof(double) * (size_t)(kcap * kcap));
    double *Y = malloc(sizeof(double) * (size_t)kcap * (size_t)(n > 0 ? n : 1));
    cand_t *work = malloc(sizeof(cand_t) * (size_t)n);
    int32_t *want = malloc(sizeof(int32_t) * (size_t)kcap);
    if (!vn1 || !vn2 || !L || !J || !G || !T || !VV || !Y || !work || !want) {
        free(vn1); free(vn2); free(L); free(J); free(G); free(T); free(VV); free(Y); free(work); free(want);
        return O_ERR_NOMEM;
    }

    /* Algorithm 4, first line: initial column norms (R1) */
    double amax = 0.0;
    for (int64_t j = 0; j < n; ++j) {
        vn1[j] = norm2(A + j * lda, m);
        vn2[j] = vn1[j];
        if (vn1[j] > amax) amax = vn1[j];
    }
    /* absolute rounding-noise scale of partial norms, for the margins only */
    double fro2 = 0.0;
    for (int64_t j = 0; j < n; ++j) fro2 += vn1[j] * vn1[j];
    const double nu = 4.0 * O_EPS * sqrt(fro2);
    int64_t rank = -1;
    if (amax == 0.0) { /* R15 */
        *rank_out = 0;
        free(vn1); free(vn2); free(L); free(J); free(G); free(T); free(VV); free(Y); free(work); free(want);
        return 0;
    }

    int64_t ns = 0;
    while (ns < p) {
        if (prm->max_ns >= 0 && ns >= prm->max_ns) break;
        oracle_block rec;
        memset(&rec, 0, sizeof rec);
        rec.ns = ns;
        rec.m_order = rec.m_thr = rec.m_cos = rec.m_break = rec.m_stop = rec.m_fb = rec.m_recomp = INFINITY;

        /* umax, jmax (R2) */
        int64_t jmax = ns;
        double umax = vn1[ns];
        for (int64_t j = ns + 1; j < n; ++j)
            if (vn1[j] > umax) { umax = vn1[j]; jmax = j; }
        /* stop test, eq. (practical stopping criterion) with eps_1 = eps*n (R14) */
        if (rank < 0) {
            double lhs = (prm->stop_rule == O_STOP_MAXNORM) ? umax : sqrt((double)(n - ns)) * umax;
            double rhs = eps1 * amax;
            double nu_l = (prm->stop_rule == O_STOP_MAXNORM) ? nu : sqrt((double)(n - ns)) * nu;
            rec.m_stop = (fabs(lhs - rhs) <= nu_l) ? 0.0 : rel_margin(lhs, rhs);
            if (lhs <= rhs) {
                rank = ns;
                if (prm->stop_rule != O_STOP_NONE) {
                    if (log && nb < log_cap) log[nb] = rec;
                    ++nb;
                    break;
                }
            }
        }
        /* eq. (column_norm_bound_DM): scalar pivoting near the noise level (R13) */
        double fb_thr = O_EPS * (double)n * amax;
        if (prm->plant == O_PLANT_FBSCALE) fb_thr = O_EPS * amax;
        rec.m_fb = noise_margin(umax, fb_thr, nu);
        int64_t cap = kcap < (p - ns) ? kcap : (p - ns);
        int ks = 1, nl = 1;
        if (umax <= fb_thr || cap == 1) {
            rec.fallback = (umax <= fb_thr);
            J[0] = jmax;
            L[0] = jmax;
            /* order margin of the single arg-max choice */
            double second = -1.0;
            for (int64_t j = ns; j < n; ++j)
                if (j != jmax && vn1[j] > second) second = vn1[j];
            rec.m_order = (second >= 0.0) ? noise_margin(second, umax, nu) : INFINITY;
            rec.ncand = 1; rec.nL = 1; rec.jmax = (int32_t)jmax; rec.umax = umax;
            /* a single column: gamma = 1 and sigma_min(C) = ||c|| (Lemma 1, k = 1) */
            rec.gamma = 1.0;
            rec.sigma_bound = norm2(A + jmax * lda + ns, m - ns);
        } else {
            dm_select(A, m, n, lda, ns, vn1, prm->tau, prm->delta, cap, prm->certified, L, &nl, NULL, J, &ks, &rec,
                      work, G, nu, prm->plant);
        }
        /* eq. (lenght_check): eps_s = tau * max u (R12) */
        double eps_s = prm->tau * umax;
        rec.eps_s = eps_s;

        /* move J to the leading positions by transpositions (Section 4, R8):
         * for i = 0..ks-1 swap position ns+i with the CURRENT position of J_i */
        for (int i = 0; i < ks; ++i) want[i] = perm[J[i]];
        for (int i = 0; i < ks; ++i) {
            int64_t pos = ns + i;
            for (int64_t j = ns + i; j < n; ++j)
                if (perm[j] == want[i]) { pos = j; break; }
            swap_cols(A, m, lda, vn1, vn2, perm, ns + i, pos);
        }

        /* Householder panel with break (Algorithm 4 inner loop, R9-R11) */
        int l = 0;
        double mbreak = INFINITY;
        for (int i = 0; i < ks; ++i) {
            int64_t c = ns + i;
            double *x = A + c * lda + c;
            int64_t len = m - c;
            double alpha = x[0];
            double sp = 0.0;
            for (int64_t r = 1; r < len; ++r) sp += x[r] * x[r];
            double nrm = sqrt(alpha * alpha + sp);
            if (i >= 1) {
                mbreak = fmin(mbreak, noise_margin(nrm, eps_s, nu));
                if (nrm < eps_s && prm->plant != O_PLANT_NOBREAK) break;
                if (prm->plant == O_PLANT_TRUNC && 2 * i >= ks) break;
            }
            double beta, ti;
            if (sp == 0.0) {
                ti = 0.0;
                beta = alpha;
            } else {
                beta = (alpha >= 0.0) ? -nrm : nrm;
                ti = (beta - alpha) / beta;
                double den = alpha - beta;
                for (int64_t r = 1; r < len; ++r) x[r] = x[r] / den;
            }
            x[0] = beta;
            tau_house[c] = ti;
            /* apply H = I - ti v v^T to the remaining panel columns only (R10) */
            for (int64_t j = c + 1; j < ns + ks; ++j) {
                double *y = A + j * lda + c;
                double w = y[0];
                for (int64_t r = 1; r < len; ++r) w += x[r] * y[r];
                w *= ti;
                y[0] -= w;
                for (int64_t r = 1; r < len; ++r) y[r] -= x[r] * w;
            }
            l = i + 1;
        }
        rec.m_break = mbreak;
        /* after a break the rejected panel columns keep the l reflectors
         * already applied to them inside the panel (Section 4) */

        /* compact WY: H_0 ... H_{l-1} = I - V T V^T, forward column-wise */
        /* V_{:,a} = e_a + below-diagonal part of column ns+a (rows ns..m-1) */
        for (int a = 0; a < l; ++a) {
            for (int b = a; b < l; ++b) {
                /* VV[a][b] = V_a^T V_b, rows r >= ns+b (V_a is 0 above ns+a) */
                const double *va = A + (ns + a) * lda;
                const double *vb = A + (ns + b) * lda;
                int64_t rb = ns + b;
                double s = (a == b) ? 1.0 : va[rb]; /* row rb: v_b = 1 */
                for (int64_t r = rb + 1; r < m; ++r) s += va[r] * vb[r];
                VV[a * kcap + b] = s;
            }
        }
        for (int i = 0; i < l; ++i) {
            double ti = tau_house[ns + i];
            for (int a = 0; a < i; ++a) {
                double s = 0.0;
                for (int b = a; b < i; ++b) s += T[a * kcap + b] * VV[b * kcap + i];
                T[a * kcap + i] = -ti * s;
            }
            T[i * kcap + i] = ti;
            for (int a = i + 1; a < l; ++a) T[a * kcap + i] = 0.0;
        }

        /* block trailing update A[ns:m, ns+ks:n] -= V T^T V^T A[ns:m, ns+ks:n] */
        int64_t w0 = ns + ks;
#pragma omp parallel for schedule(static)
        for (int64_t j = w0; j < n; ++j) {
            double *y = A + j * lda;
            double *zz = Y + (j - w0) * kcap;
            /* z = V^T y */
            for (int a = 0; a < l; ++a) {
                const double *va = A + (ns + a) * lda;
                int64_t ra = ns + a;
                double s = y[ra];
                for (int64_t r = ra + 1; r < m; ++r) s += va[r] * y[r];
                zz[a] = s;
            }
            /* z = T^T z (T upper triangular, so T^T lower triangular) */
            for (int a = l - 1; a >= 0; --a) {
                double s = 0.0;
                for (int b = 0; b <= a; ++b) s += T[b * kcap + a] * zz[b];
                zz[a] = s;
            }
            /* y -= V z */
            for (int a = 0; a < l; ++a) {
                const double *va = A + (ns + a) * lda;
                int64_t ra = ns + a;
                y[ra] -= zz[a];
                for (int64_t r = ra + 1; r < m; ++r) y[r] -= va[r] * zz[a];
            }
        }

        /* partial norm update with the l new rows of R (R7) */
        double mrec = INFINITY;
#pragma omp parallel for schedule(static) reduction(min : mrec)
        for (int64_t j = ns + l; j < n; ++j) {
            if (vn1[j] == 0.0) continue;
            const double *y = A + j * lda;
            double s = 0.0;
            for (int64_t r = ns; r < ns + l; ++r) s += y[r] * y[r];
            double q = 1.0 - s / (vn1[j] * vn1[j]);
            if (q < 0.0) q = 0.0;
            double q2 = q * sq(vn1[j] / vn2[j]);
            mrec = fmin(mrec, rel_margin(q2, tol3z));
            if (q2 <= tol3z) {
                vn1[j] = norm2(y + ns + l, m - (ns + l));
                vn2[j] = vn1[j];
            } else {
                vn1[j] = vn1[j] * sqrt(q);
            }
        }
        rec.m_recomp = mrec;
        rec.ks = ks;
        rec.l = l;
        if (log && nb < log_cap) log[nb] = rec;
        ++nb;
        ns += l;
    }
    if (rank < 0) rank = ns;
    *rank_out = rank;
    if (nblocks) *nblocks = nb;
    free(vn1); free(vn2); free(L); free(J); free(G); free(T); free(VV); free(Y); free(work); free(want);
    return 0;
}

/* QRP, Algorithm 2: the same loop with a single pivot (the arg-max) per step. */
int oracle_qrp(double *A, int64_t m, int64_t n, int64_t lda, int32_t stop_rule, double eps1_scale,
               double *tau_house, int32_t *perm, int64_t *rank_out,
               oracle_block *log, int64_t log_cap, int64_t *nblocks) {
    oracle_params p;
    p.tau = 1.0;
    p.delta = 0.0;
    p.kmax = 1;
    p.stop_rule = stop_rule;
    p.eps1_scale = eps1_scale;
    p.max_ns = -1;
    return oracle_qrdm(A, m, n, lda, &p, tau_house, perm, rank_out, log, log_cap, nblocks);
}

/*
 * One DM step (Algorithm 1) on the trailing part [A]_{ns:m, ns:n} with given
 * partial norms vn1[0..n) (only entries >= ns are read).  Exposed for unit
 * tests of the selection alone.  L, J: int64[cap]; theta: double[cap*cap];
 * plant: 0, or an O_PLANT_* mistake (tests of the checks only).
 */
int oracle_dm_step(const double *A, int64_t m, int64_t n, int64_t lda, int64_t ns,
                   const double *vn1, double tau, double delta, int64_t cap,
                   int64_t *L, int32_t *nL, double *theta, int64_t *J, int32_t *ks, int32_t plant) {
    if (ns < 0 || ns >= n || ns >= m || cap < 1) return -5;
    cand_t *work = malloc(sizeof(cand_t) * (size_t)n);
    double *G = malloc(sizeof(double) * (size_t)(cap * cap));
    if (!work || !G) { free(work); free(G); return O_ERR_NOMEM; }
    int nl = 0, k = 0;
    dm_select(A, m, n, lda, ns, vn1, tau, delta, cap, 0, L, &nl, theta, J, &k, NULL, work, G, 0.0, plant);
    *nL = nl;
    *ks = k;
    free(work);
    free(G);
    return 0;
}

size_t oracle_block_size(void) { return sizeof(oracle_block); }

/* Threads the OpenMP loops of the trailing update use (for reporting timings). */
int oracle_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
