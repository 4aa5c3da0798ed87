// Internal declarations shared by the HIP kernels and the host driver of
// libqrdm.so (gfx950).  Not part of the public ABI (include/qrdm.h).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#define QK_KM 128          // capacity of every per-block array (k_DM <= 128)
#define QK_SWAP_MAX (2 * QK_KM)

// Loop state of one factorization, resident in device memory.  Every kernel of
// an outer step reads it; only the single-workgroup kernels write it.
struct QrdmCtl {
    int64_t ns;      // columns factored (n_s)
    int64_t rank;    // -1 until the stopping test first holds
    int32_t l;       // reflectors kept by the current step's panel
    int32_t ks;      // accepted columns of the current step (k_s)
    int32_t nL;      // candidate list length (0 when done)
    int32_t done;    // 1 = no further step
    int32_t fallback;  // 1 = the partial norms reached the noise level (eq.
                       // column_norm_bound_DM): the selection that found it took no
                       // block, and every kernel of the DM loop is idle from then
                       // on; the column-pivoting kernels continue from n_s (sticky)
    int32_t jmax;
    double gamma;        // Lemma 1 on the current step's accepted columns: diagonal-dominance gap
    double sigma_bound;  // and the lower bound of their sigma_min (0 if the lemma does not apply)
    double umax;       // max partial norm of the current step
    int32_t nonfinite; // set by the norm sweep: the loop ends before writing anything
    int32_t error;     // 2: a grid barrier wait timed out; 4: a launch grid smaller
                       // than the kernel's partition (host sizing); either fails the call
    int32_t nswap;     // column moves of the current step
    int32_t pad0;
    double amax;       // max initial column norm
    double eps_s;      // panel break threshold tau*umax
    // statistics
    int64_t nblocks, nbreaks, nfallback, nrecompute;
    double flop_gemm;  // algorithmic flops of one trailing GEMM (2 t l w), summed over blocks
    double flop_panel;   // algorithmic flops of the Householder panels, summed over blocks
    double bytes_panel;  // algorithmic bytes of the panels (slab read + written: 16 t k_s)
    int64_t npanel;      // panels that factored a block
    int32_t L[QK_KM];
    int32_t J[QK_KM];
    int32_t swp_dst[QK_SWAP_MAX];
    int32_t swp_src[QK_SWAP_MAX];
    // column pivoting with deferred trailing update (QRP baseline and the
    // scalar-pivoting continuation of QRDM)
    int64_t qp_k0;      // first column of the current block
    int64_t qp_last;    // last reflector of the block being closed
    int32_t qp_b;       // reflectors completed in the current block
    int32_t qp_kb;      // reflectors in the block being closed
    int32_t qp_pend;    // 1 = reflector ns-1 still awaits its normalization
    int32_t qp_end;     // the block closes at this step
    int32_t qp_stop;    // the stopping test fired at this step
    int32_t qp_flag;    // a partial norm needs recomputation
    int32_t qp_nb;      // block size
    int32_t qp_pad;
    double qp_beta, qp_den;  // scalars of the pending reflector
    int64_t qp3_start;       // first column of the column-pivoting loop
    // the panel of the current DM step
    int32_t cpath;           // 1 = formed from the Gram matrix (k_cpanel.hip), 0 = column by column
    int32_t c0off;           // first column of the trailing update, from n_s: k_s, or l when cpath
    int32_t Ai[QK_KM];       // candidate index (row of the Gram matrix) of each accepted column
    int64_t ngram;           // panels formed from the Gram matrix
    double bytes_gemm2;      // algorithmic bytes of GEMM2 (A read and written once: 16 t w), summed over blocks
};

// Region of the workspace for the Gram-matrix panel (doubles, 64 x 64 each):
// R1, W1 = R1^{-1}, Q1^T Q1, T, P.
#define CP_OFF_R1 0
#define CP_OFF_W1 4096
#define CP_OFF_G2 8192
#define CP_OFF_T 12288
#define CP_OFF_P 16384
#define CP_DOUBLES 20480

struct QrdmArgs {
    double *A;
    int64_t m, n, lda;
    double tau, delta;
    int32_t kmax;
    int32_t stop_rule;
    int32_t certified = 0;  // delta <= tau^2 / (nL - 1) per step (eq. delta_max)
    int32_t lemma = 1;      // form Lemma 1's gamma and sigma bound of each step (read by the step log only)
    double eps1;    // eps_1 * (applied as eps1 * amax) of the stopping test
    double fbeps;   // eps_w * n: scalar pivoting when max partial norm <= fbeps * amax
    double tol3z;   // sqrt(eps_w): recompute a partial norm when the downdate lost this much
    double *vn1, *vn2;
    int32_t *perm;
    double *tau_house;
    QrdmCtl *ctl;
    uint32_t *gbar = nullptr;  // [GBAR_GROUPS * GBAR_STRIDE]: counters of the persistent kernels' grid barrier
    uint64_t *snap = nullptr;  // host-mapped slot for the polled prefix of the control block (or none)
};

// ------------------------------------------------------------------ helpers
// The host polls the first QRDM_SNAP_WORDS 8-byte words of QrdmCtl (n_s, rank,
// l, k_s, |L|, done, fallback, arg-max, gamma, bound, max partial norm, the
// non-finite and error flags).  The last kernel of a step writes them into a
// slot of pinned host memory, so no copy is queued.
#define QRDM_SNAP_WORDS 9
__device__ __forceinline__ void qrdm_write_snapshot(const QrdmCtl *c, uint64_t *dst) {
    const uint64_t *src = (const uint64_t *)c;
    for (int i = 0; i < QRDM_SNAP_WORDS; ++i) dst[i] = src[i];
}
__device__ __forceinline__ double wave_sum(double v) {
    // fixed-order butterfly over the 64 lanes of a wavefront
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

__device__ __forceinline__ int64_t p_of(const QrdmArgs &a) { return a.m < a.n ? a.m : a.n; }

// The kernels of a DM step (Algorithm 4) have nothing to do once the loop is
// done or has passed to the column-pivoting kernels.
__device__ __forceinline__ bool qrdm_dm_idle(const QrdmCtl *c) { return c->done || c->fallback; }

// Grid barrier of the persistent kernels (all G workgroups resident): workgroup
// w adds one to counter w % 16 (one counter per group of workgroups, 256 B
// apart, so the atomics spread), and sixteen threads of every workgroup poll
// the counters until each holds its group's count times k, for the k-th
// barrier of the launch (1.3 us at 256 workgroups; 1.4 with 8 counters, 2.9
// with one flag per workgroup polled by 256 threads).  The counters start at zero for each launch (cleared
// by the kernel launched before it).  A workgroup's stores before the barrier
// complete before its increment.  The wait is bounded: on timeout error bit 2
// is raised, the kernel runs on, and later barriers no longer wait.
#define GBAR_STRIDE 64
#define GBAR_GROUPS 16
#define GBAR_SPIN_LIMIT (1 << 26)
__device__ __forceinline__ void gbar_wait(uint32_t *gbar, int G, uint32_t k, int32_t *err) {
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    if (threadIdx.x == 0)
        __hip_atomic_fetch_add(gbar + GBAR_STRIDE * (blockIdx.x % GBAR_GROUPS), 1u, __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
    if (threadIdx.x < GBAR_GROUPS && !(__hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) & 2)) {
        const uint32_t target = (uint32_t)((G - (int)threadIdx.x + GBAR_GROUPS - 1) / GBAR_GROUPS) * k;
        int it = 0;
        while (__hip_atomic_load(gbar + GBAR_STRIDE * threadIdx.x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) <
               target) {
            __builtin_amdgcn_s_sleep(1);
            if (++it > GBAR_SPIN_LIMIT) {
                atomicOr(err, 2);
                break;
            }
        }
    }
    __syncthreads();
}
// Clears the counters (the calling thread).
__device__ __forceinline__ void gbar_clear(uint32_t *gbar) {
    if (gbar)
        for (int x = 0; x < GBAR_GROUPS; ++x)
            __hip_atomic_store(gbar + GBAR_STRIDE * x, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Lane exchanges on the VALU (DPP and the gfx950 lane swaps): lane_xu<K>(v) is
// v of lane ^ K for K = 32, 16, 8, 2, 1, and of lane ^ 7 (the mirror within
// each group of 8) for K = 7.
template <int K>
__device__ __forceinline__ uint32_t lane_xu(uint32_t v) {
    if constexpr (K == 32) {
        const auto r = __builtin_amdgcn_permlane32_swap(v, v, false, false);
        return (threadIdx.x & 32) ? r[0] : r[1];
    } else if constexpr (K == 16) {
        const auto r = __builtin_amdgcn_permlane16_swap(v, v, false, false);
        return (threadIdx.x & 16) ? r[0] : r[1];
    } else {
        static_assert(K == 8 || K == 7 || K == 2 || K == 1, "lane exchange");
        constexpr int ctrl = K == 8 ? 0x128 : K == 7 ? 0x141 : K == 2 ? 0x4e : 0xb1;  // row_ror:8, row_half_mirror, quad_perm
        return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, ctrl, 0xf, 0xf, false);
    }
}
template <int K>
__device__ __forceinline__ double lane_xd(double v) {
    const uint64_t b = (uint64_t)__double_as_longlong(v);
    const uint64_t lo = lane_xu<K>((uint32_t)b), hi = lane_xu<K>((uint32_t)(b >> 32));
    return __longlong_as_double((long long)((hi << 32) | lo));
}

// ------------------------------------------------------------ launchers
// Launch of a kernel whose workgroups wait on each other through memory (the
// panel, the QP3 block kernel): every workgroup must be resident at once.  The
// callers size the grid to at most one workgroup per compute unit, with the
// occupancy of their largest LDS request checked, so a regular dispatch on an
// otherwise idle device places them all at once, without the extra dispatch
// time of hipLaunchCooperativeKernel.  QRDM_COOPERATIVE=1 in the environment
// selects the cooperative launch (the runtime's co-residency guarantee), for
// devices shared with other work.  Either way the kernels' waits are bounded:
// a wait that times out raises error bit 2 and the call fails.
hipError_t launch_resident(const void *kernel, dim3 grid, dim3 block, void **args, unsigned lds, hipStream_t s);
// Each returns hipGetLastError() of its launch.
hipError_t launch_colnorm(const double *A, int64_t m, int64_t n, int64_t lda, double *vn1, double *vn2,
                          QrdmCtl *ctl, hipStream_t s);
hipError_t launch_init(QrdmArgs a, hipStream_t s);
hipError_t launch_ws_reset(QrdmCtl *ctl, int32_t *flag, int64_t n, hipStream_t s);
hipError_t launch_rank_out(const QrdmCtl *ctl, int64_t *rank, hipStream_t s);
hipError_t launch_select(QrdmArgs a, hipStream_t s);
hipError_t launch_gram(QrdmArgs a, double *Gp, int64_t t_bound, hipStream_t s);
hipError_t launch_gram_reduce(QrdmArgs a, const double *Gp, double *G, int64_t t_bound, hipStream_t s);
hipError_t launch_dm_finish(QrdmArgs a, const double *G, double *theta_out, hipStream_t s);
hipError_t launch_swap(QrdmArgs a, hipStream_t s);
// The Gram-matrix panel (k_cpanel.hip): cp is the CP_DOUBLES region; Gp the Gram
// partials of the DM step (free once k_dm_finish has run); kp their leading
// dimension.
hipError_t launch_cpchol(QrdmArgs a, const double *G, double *cp, int enable, hipStream_t s);
hipError_t launch_cpanel1(QrdmArgs a, const double *cp, double *Vw, int64_t ldv, double *Gp, int kp, int64_t t_bound,
                          hipStream_t s);
hipError_t launch_cpreduce(QrdmArgs a, const double *Gp, int kp, double *cp, hipStream_t s);
hipError_t launch_cpanel2(QrdmArgs a, double *cp, const double *Vw, int64_t ldv, double *Vo, float *Vo32,
                          hipStream_t s);
hipError_t launch_cpanel3(QrdmArgs a, const double *cp, double *Vw, int64_t ldv, float *Vw32, int64_t t_bound,
                          hipStream_t s);
int cpanel_partials(int64_t m);
hipError_t launch_panel(QrdmArgs a, double *PB, double *VV, double *Vw, float *Vw32, int64_t ldv,
                        int64_t t_bound, int rows_per_wg, hipStream_t s);
// VV: v_a^T v_i (a < i) at VV[a * QK_KM + i], from the panel.
// ev (may be null): 4 events recorded before GEMM1, after GEMM1, before GEMM2, after GEMM2
// Yp: QK_SPLIT_MAX x QK_KM x n partials of V^T A (k_gemm1), summed by k_zsum
// t_bound, w_bound: upper bounds on the trailing rows and columns; w_lo: a lower
// bound on the trailing columns (sizes GEMM1's split grid)
// cpT: T of the Gram-matrix panel (used when ctl->cpath; k_zsum forms T from VV otherwise)
hipError_t launch_trail(QrdmArgs a, int precision, const double *VV, const double *cpT, const double *Vw,
                        const float *Vw32, int64_t ldv, void *Z, double *Yp, int64_t t_bound, int64_t w_bound,
                        int64_t w_lo, hipStream_t s, hipEvent_t *ev);
hipError_t launch_downdate(QrdmArgs a, int64_t w_bound, hipStream_t s);

// QP3 (LAPACK xgeqp3-style) column loop: either one block of up to nb steps
// per cooperative launch, or one step per group of launches
#define QP_RUN_MAXWG 256  // workgroups of the persistent block kernel (at most)
struct Qp3Bufs {
    double *PB2;      // [ceil(m/256)][2 + 2 * 64] partials of the pivot column pass
    double *Fz;       // [nb][n]: F^T of the deferred update, absolute column index
    int32_t *flag;    // [n]: partial norm needs recomputation
    double *amx;      // [QP_RUN_MAXWG][4]: per-workgroup arg-max partials of the block kernel
    double *pub;      // [qp3_tail_pub_doubles(m)]: the tail kernel's published partials and columns
};
hipError_t launch_qp3_init(QrdmArgs a, int nb, hipStream_t s);
hipError_t launch_gemm2_qp3(QrdmArgs a, const double *Vw, int64_t ldv, const double *Fz, int64_t t_bound,
                            int64_t w_bound, hipStream_t s);
hipError_t launch_qp3_step(QrdmArgs a, Qp3Bufs b, int nb, int64_t t_bound, int64_t w_bound, hipStream_t s);
// Grid of the block kernel for m rows (0: use the per-step kernels).
int qp3_block_grid(int64_t m);
hipError_t launch_qp3_block(QrdmArgs a, Qp3Bufs b, int nb, int64_t t_bound, int64_t w_bound, int grid,
                            int launch, hipStream_t s, hipEvent_t *ev = nullptr);  // ev[0], ev[1] around k_qp_run
// Register-resident tail of the column-pivoting loop: every remaining step in
// one launch once the trailing block fits in the registers of the grid (at most
// 2048 rows and 8 columns per workgroup: qp3_tail_shape).
int qp3_tail_grid();
bool qp3_tail_shape(int64_t t_bound, int64_t w_bound, int grid, int *cq, int *crows, size_t *bytes);
size_t qp3_tail_pub_doubles(int64_t m);
hipError_t launch_qp3_tail(QrdmArgs a, double *pub, int32_t *flag, int64_t t_bound, int64_t w_bound, int grid,
                           int launch, hipStream_t s, hipEvent_t *ev = nullptr);  // ev[0], ev[1] around k_qp_tail
int panel_max_wgs(int rows_per_wg);
int panel_rows_per_wg(int kmax);
int panel_rows_for(int64_t m, int kmax);
