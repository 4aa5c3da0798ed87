// Host driver and C ABI of libqrdm.so (declared in include/qrdm.h).
//
// The outer loop of Algorithm 4 (QRDM2) is a fixed sequence of kernel
// launches per block; the loop state (n_s, k_s, l, the stop decision, the
// candidate and accepted lists) lives in a device control block and never
// crosses to the host during the loop.  Grids are sized from a lower bound on
// n_s that the host learns by polling a small snapshot of the control block
// `poll_lag` blocks behind the launch front; kernels of blocks enqueued after
// the loop has finished exit at once.
#include <hip/hip_runtime.h>

#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <vector>

#include "../../include/qrdm.h"
#include "qrdm_internal.h"

int gram_partials(int64_t t_bound);
int panel_lds_bytes(int rows_per_wg, int kmax);

namespace {

struct Snapshot {  // first bytes of QrdmCtl copied back for polling
    int64_t ns;
    int64_t rank;
    int32_t l, ks, nL, done, fallback, jmax;
    double gamma, sigma_bound;
};
static_assert(sizeof(Snapshot) == 8 * QRDM_SNAP_WORDS, "the snapshot is the words the kernels write");
static_assert(offsetof(Snapshot, jmax) == offsetof(QrdmCtl, jmax) &&
                  offsetof(Snapshot, gamma) == offsetof(QrdmCtl, gamma) &&
                  offsetof(Snapshot, sigma_bound) == offsetof(QrdmCtl, sigma_bound),
              "the polled snapshot is a prefix of the control block");

struct Workspace {
    int device = -1;
    size_t bytes = 0;
    char *base = nullptr;
    Snapshot *host_snap = nullptr;  // pinned ring
    uint64_t *dev_snap = nullptr;   // its device address (written by the kernels)
    int ring = 0;
    std::vector<hipEvent_t> events;
};

Workspace g_ws;

// timing events of the profiling mode (grown on demand, kept for reuse)
std::vector<hipEvent_t> g_prof_ev;
std::vector<hipEvent_t> g_qp_ev;  // around each QP3 block-kernel launch
int grow_events(std::vector<hipEvent_t> &v, size_t count) {
    while (v.size() < count) {
        hipEvent_t e;
        if (hipEventCreate(&e) != hipSuccess) return -1;
        v.push_back(e);
    }
    return 0;
}
int prof_events(size_t count) { return grow_events(g_prof_ev, count); }

// Timing of the QP3 loop's block-kernel launches (profile mode).
struct Qp3Prof {
    bool on = false;
    int64_t launches = 0;
};

// Algorithmic bytes of the pivot steps j0 .. j1-1: 8 (m-j)(n-j) each.
double qp3_bytes(int64_t m, int64_t n, int64_t j0, int64_t j1) {
    double b = 0.0;
    for (int64_t j = j0; j < j1; ++j) b += 8.0 * (double)(m - j) * (double)(n - j);
    return b;
}

double qp3_run_ms(int64_t launches) {
    double t = 0.0;
    for (int64_t i = 0; i < launches; ++i) {
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, g_qp_ev[2 * i], g_qp_ev[2 * i + 1]) == hipSuccess) t += ms;
    }
    return t;
}

struct Layout {
    size_t ctl, vn1, vn2, gp, g, theta, pb, tm, vw, vw32, z, yp, pb2, fz, flag, qrb, gbar, perm_dbg, total;
};

const int kMinRowsPerWg = 16;   // smallest panel slab (bounds the partial buffer)

size_t align_up(size_t x) { return (x + 255) & ~(size_t)255; }

Layout make_layout(int64_t m, int64_t n) {
    Layout L;
    size_t off = 0;
    auto take = [&](size_t bytes) { size_t o = off; off = align_up(off + bytes); return o; };
    const int64_t mm = std::max<int64_t>(m, 1), nn = std::max<int64_t>(n, 1);
    L.ctl = take(sizeof(QrdmCtl));
    L.vn1 = take(sizeof(double) * nn);
    L.vn2 = take(sizeof(double) * nn);
    L.gp = take(sizeof(double) * (size_t)gram_partials(mm) * QK_KM * QK_KM);
    L.g = take(sizeof(double) * QK_KM * QK_KM);
    L.theta = take(sizeof(double) * QK_KM * QK_KM);
    const int64_t pmax = (mm + kMinRowsPerWg - 1) / kMinRowsPerWg;
    // panel: 4096 arrival flags (16 KB), rows c and c+1 (2 x 2 QK_KM), partial dots (2 x pmax x 2 QK_KM)
    L.pb = take(16384 + sizeof(double) * (4 * QK_KM + 2 * (size_t)pmax * 2 * QK_KM));
    L.tm = take(sizeof(double) * QK_KM * QK_KM);
    L.vw = take(sizeof(double) * (size_t)QK_KM * mm);
    L.vw32 = take(sizeof(float) * (size_t)QK_KM * mm);
    L.z = take(sizeof(double) * (size_t)QK_KM * nn);
    L.yp = take(sizeof(double) * 16 * (size_t)QK_KM * nn);
    L.pb2 = take(sizeof(double) * (size_t)((mm + 255) / 256) * (2 + 2 * 64));
    L.fz = take(sizeof(double) * 64 * (size_t)nn);
    L.flag = take(sizeof(int32_t) * (size_t)nn);
    // QP3 block kernel: 4 doubles of arg-max partials per workgroup
    L.qrb = take(sizeof(double) * 4 * QP_RUN_MAXWG);
    L.gbar = take(2 * sizeof(uint32_t) * GBAR_GROUPS * GBAR_STRIDE);  // grid-barrier counters: panel, QP3 block kernel (2 sets)
    L.perm_dbg = take(sizeof(int32_t) * nn);
    L.total = off;
    return L;
}

int hip_err(hipError_t e) { return e == hipSuccess ? 0 : QRDM_ERR_HIP + (int)e; }

}  // namespace

hipError_t launch_resident(const void *kernel, dim3 grid, dim3 block, void **args, unsigned lds, hipStream_t s) {
    static int coop = -1;
    if (coop < 0) {
        const char *e = getenv("QRDM_COOPERATIVE");
        coop = (e && strcmp(e, "1") == 0) ? 1 : 0;
    }
    if (coop) return hipLaunchCooperativeKernel(kernel, grid, block, args, lds, s);
    return hipLaunchKernel(kernel, grid, block, args, lds, s);
}

namespace {

#define HIP_TRY(x)                                  \
    do {                                            \
        hipError_t _e = (x);                        \
        if (_e != hipSuccess) return hip_err(_e);   \
    } while (0)

int ensure_workspace(size_t bytes, int ring) {
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    if (g_ws.base && g_ws.device == dev && g_ws.bytes >= bytes && g_ws.ring >= ring) return 0;
    if (g_ws.base) {
        (void)hipDeviceSynchronize();
        (void)hipFree(g_ws.base);
        g_ws.base = nullptr;
    }
    if (g_ws.host_snap) {
        (void)hipHostFree(g_ws.host_snap);
        g_ws.host_snap = nullptr;
    }
    for (auto e : g_ws.events) (void)hipEventDestroy(e);
    g_ws.events.clear();
    const char *fault = getenv("QRDM_FAULT");
    if (fault && strcmp(fault, "alloc") == 0) return QRDM_ERR_NOMEM;
    size_t want = std::max(bytes, g_ws.bytes);
    if (hipMalloc((void **)&g_ws.base, want) != hipSuccess) {
        g_ws.base = nullptr;
        g_ws.bytes = 0;
        (void)hipGetLastError();
        return QRDM_ERR_NOMEM;
    }
    int r = std::max(ring, 8);
    if (hipHostMalloc((void **)&g_ws.host_snap, sizeof(Snapshot) * r, hipHostMallocDefault) != hipSuccess ||
        hipHostGetDevicePointer((void **)&g_ws.dev_snap, g_ws.host_snap, 0) != hipSuccess) {
        if (g_ws.host_snap) (void)hipHostFree(g_ws.host_snap);
        g_ws.host_snap = nullptr;
        (void)hipFree(g_ws.base);
        g_ws.base = nullptr;
        return QRDM_ERR_NOMEM;
    }
    if (hipMemset(g_ws.base, 0, want) != hipSuccess) return QRDM_ERR_NOMEM;
    g_ws.events.resize(r);
    for (int i = 0; i < r; ++i) HIP_TRY(hipEventCreateWithFlags(&g_ws.events[i], hipEventDisableTiming));
    g_ws.bytes = want;
    g_ws.device = dev;
    g_ws.ring = r;
    return 0;
}

int check_common(const double *A, int64_t m, int64_t n, int64_t lda, const qrdm_params *p) {
    if (m < 0) return -2;
    if (n < 0) return -3;
    if (lda < std::max<int64_t>(1, m)) return -4;
    if (p) {
        if (!(p->tau >= 0.0 && p->tau <= 1.0)) return -5;
        if (!(p->delta >= 0.0 && p->delta <= 1.0)) return -5;
        if (p->kmax < 1 || p->kmax > QRDM_KMAX_LIMIT) return -5;
        if (p->stop_rule < 0 || p->stop_rule > 2) return -5;
        if (p->precision < 0 || p->precision > 1) return -5;
        if (p->poll_lag < 0) return -5;
        if (p->profile < 0 || p->profile > 1) return -5;
        if (p->certified < 0 || p->certified > 1) return -5;
    }
    if (m > 0 && n > 0 && !A) return -1;
    return 0;
}

QrdmCtl initial_ctl() {
    QrdmCtl c;
    memset(&c, 0, sizeof c);
    c.rank = -1;
    return c;
}

const int kQp3Nb = 32;  // block size of the column-pivoting update

// Column pivoting steps from the device's current n_s until the loop is done.
int run_qp3(const QrdmArgs &a, char *ws, const Layout &L, int nb, int lag, int64_t ns_known, hipStream_t s,
            Qp3Prof *prof) {
    Qp3Bufs bf;
    bf.PB2 = (double *)(ws + L.pb2);
    bf.Fz = (double *)(ws + L.fz);
    bf.flag = (int32_t *)(ws + L.flag);
    bf.amx = (double *)(ws + L.qrb);
    HIP_TRY(launch_qp3_init(a, nb, s));
    const int ring = g_ws.ring;
    const int64_t pmin = std::min(a.m, a.n);
    const char *mode = getenv("QRDM_QP3_STEPS");  // "1": the per-step kernels (comparison runs)
    const int grid = (mode && strcmp(mode, "1") == 0) ? 0 : qp3_block_grid(a.m);
    if (grid > 0) {
        // one block of up to nb steps per launch; a snapshot after each, the
        // host waiting on the one `lag` launches back
        for (int64_t iter = 0;; ++iter) {
            const int64_t tb = a.m - ns_known, wb = a.n - ns_known;
            hipEvent_t *ev = nullptr;
            if (prof && prof->on) {
                if (grow_events(g_qp_ev, 2 * (size_t)(iter + 1)) != 0) return QRDM_ERR_NOMEM;
                ev = g_qp_ev.data() + 2 * iter;
                prof->launches = iter + 1;
            }
            QrdmArgs al = a;
            al.snap = g_ws.dev_snap + (iter % ring) * QRDM_SNAP_WORDS;  // written by the block kernel
            HIP_TRY(launch_qp3_block(al, bf, nb, tb, wb, grid, (int)iter, s, ev));
            HIP_TRY(hipEventRecord(g_ws.events[iter % ring], s));
            if (iter >= lag) {
                const int64_t k = iter - lag;
                HIP_TRY(hipEventSynchronize(g_ws.events[k % ring]));
                const Snapshot sn = g_ws.host_snap[k % ring];
                if (sn.ns > ns_known) ns_known = sn.ns;
                if (sn.done) break;
            }
            if (iter > pmin + lag + 4) break;  // cannot happen: every launch takes at least one step
        }
        return 0;
    }
    // snapshots every kStride steps; the host waits on the one `lag` snapshots back
    const int kStride = 4;
    int64_t nsnap = 0;
    for (int64_t iter = 0;; ++iter) {
        const int64_t tb = a.m - ns_known, wb = a.n - ns_known;
        HIP_TRY(launch_qp3_step(a, bf, nb, tb, wb, s));
        if ((iter + 1) % kStride != 0) continue;
        Snapshot *hs = g_ws.host_snap + (nsnap % ring);
        HIP_TRY(hipMemcpyAsync(hs, a.ctl, sizeof(Snapshot), hipMemcpyDeviceToHost, s));
        HIP_TRY(hipEventRecord(g_ws.events[nsnap % ring], s));
        if (nsnap >= lag) {
            const int64_t k = nsnap - lag;
            HIP_TRY(hipEventSynchronize(g_ws.events[k % ring]));
            const Snapshot sn = g_ws.host_snap[k % ring];
            if (sn.ns > ns_known) ns_known = sn.ns;
            if (sn.done) break;
        }
        ++nsnap;
        if (iter > 2 * pmin + kStride * (lag + 4)) break;  // cannot happen: every step advances n_s
    }
    return 0;
}

}  // namespace

extern "C" {

void qrdm_default_params(qrdm_params *p) {
    if (!p) return;
    p->tau = 0.15;
    p->delta = 0.9;
    p->kmax = 64;
    p->stop_rule = QRDM_STOP_PAPER;
    p->eps1_scale = 0.0;
    p->precision = QRDM_PREC_FP64;
    p->poll_lag = 4;
    p->profile = 0;
    p->certified = 0;
}

const char *qrdm_strerror(int code) {
    if (code == QRDM_OK) return "success";
    if (code < 0) return "invalid argument";
    if (code == QRDM_ERR_NONFINITE) return "matrix contains NaN or Inf";
    if (code == QRDM_ERR_NOMEM) return "workspace allocation failed";
    if (code == QRDM_ERR_UNSUPPORTED) return "size not supported by the kernels";
    if (code >= QRDM_ERR_HIP) return hipGetErrorString((hipError_t)(code - QRDM_ERR_HIP));
    return "unknown error";
}

void qrdm_release(void) {
    if (g_ws.base) {
        (void)hipDeviceSynchronize();
        (void)hipFree(g_ws.base);
    }
    if (g_ws.host_snap) (void)hipHostFree(g_ws.host_snap);
    for (auto e : g_ws.events) (void)hipEventDestroy(e);
    g_ws = Workspace();
}

int qrdm_colnorms(const double *A, int64_t m, int64_t n, int64_t lda, double *out, void *stream) {
    int rc = check_common(A, m, n, lda, nullptr);
    if (rc) return rc;
    if (n > 0 && !out) return -5;
    if (n == 0) return 0;
    hipStream_t s = (hipStream_t)stream;
    Layout L = make_layout(m, n);
    rc = ensure_workspace(L.total, 8);
    if (rc) return rc;
    QrdmCtl *ctl = (QrdmCtl *)(g_ws.base + L.ctl);
    double *vn2 = (double *)(g_ws.base + L.vn2);
    QrdmCtl c0 = initial_ctl();
    HIP_TRY(hipMemcpyAsync(ctl, &c0, sizeof c0, hipMemcpyHostToDevice, s));
    HIP_TRY(launch_colnorm(A, m, n, lda, out, vn2, ctl, s));
    int32_t nf = 0;
    HIP_TRY(hipMemcpyAsync(&nf, &ctl->nonfinite, sizeof nf, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    return nf ? QRDM_ERR_NONFINITE : 0;
}

int qrdm_factor_ex(double *A, int64_t m, int64_t n, int64_t lda, const qrdm_params *pin, double *tau_house,
                   int32_t *perm, int64_t *rank, qrdm_stats *stats, qrdm_block *log, int64_t log_cap,
                   int64_t *nlog, void *stream) {
    qrdm_params p;
    if (pin) p = *pin; else qrdm_default_params(&p);
    int rc = check_common(A, m, n, lda, &p);
    if (rc) return rc;
    const int64_t pmin = std::min(m, n);
    if (pmin > 0 && !tau_house) return -6;
    if (n > 0 && !perm) return -7;
    if (!rank) return -8;
    if (log && log_cap < 0) return -11;
    if (n > 32768 || m > 65536) return QRDM_ERR_UNSUPPORTED;
    hipStream_t s = (hipStream_t)stream;
    if (stats) memset(stats, 0, sizeof *stats);
    if (nlog) *nlog = 0;
    if (pmin == 0) {
        if (n > 0) {
            std::vector<int32_t> id(n);
            for (int64_t j = 0; j < n; ++j) id[j] = (int32_t)j;
            HIP_TRY(hipMemcpyAsync(perm, id.data(), sizeof(int32_t) * n, hipMemcpyHostToDevice, s));
            HIP_TRY(hipStreamSynchronize(s));
        }
        *rank = 0;
        return 0;
    }
    const int lag = log ? 0 : p.poll_lag;
    Layout L = make_layout(m, n);
    rc = ensure_workspace(L.total, lag + 2);
    if (rc) return rc;
    char *ws = g_ws.base;
    QrdmArgs a;
    a.A = A;
    a.m = m;
    a.n = n;
    a.lda = lda;
    a.tau = p.tau;
    a.delta = p.delta;
    a.kmax = p.kmax;
    a.stop_rule = p.stop_rule;
    a.certified = p.certified;
    // working precision of the trailing data: 2^-52 (FP64) or 2^-23 (FP32 updates)
    const double eps_w = (p.precision == QRDM_PREC_MIXED) ? 1.1920928955078125e-07 : 2.220446049250313e-16;
    a.eps1 = (p.eps1_scale > 0.0 ? p.eps1_scale : (double)n) * eps_w;
    a.fbeps = (double)n * eps_w;
    a.tol3z = sqrt(eps_w);
    a.vn1 = (double *)(ws + L.vn1);
    a.vn2 = (double *)(ws + L.vn2);
    a.perm = perm;
    a.tau_house = tau_house;
    a.gbar = (uint32_t *)(ws + L.gbar);
    a.ctl = (QrdmCtl *)(ws + L.ctl);
    double *Gp = (double *)(ws + L.gp), *G = (double *)(ws + L.g), *PB = (double *)(ws + L.pb);
    double *VVb = (double *)(ws + L.tm), *Vw = (double *)(ws + L.vw);
    float *Vw32 = (float *)(ws + L.vw32);
    void *Z = ws + L.z;
    const int64_t ldv = m;

    QrdmCtl c0 = initial_ctl();
    HIP_TRY(hipMemcpyAsync(a.ctl, &c0, sizeof c0, hipMemcpyHostToDevice, s));
    // the GEMM tile counters self-reset, but their place in the cached workspace
    // depends on (m, n): clear them for this call
    HIP_TRY(launch_colnorm(A, m, n, lda, a.vn1, a.vn2, a.ctl, s));
    int32_t nf = 0;
    HIP_TRY(hipMemcpyAsync(&nf, &a.ctl->nonfinite, sizeof nf, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    if (nf) return QRDM_ERR_NONFINITE;
    HIP_TRY(launch_init(a, s));

    if (p.profile) {
        if (prof_events(3) != 0) return QRDM_ERR_NOMEM;
        HIP_TRY(hipEventRecord(g_prof_ev[0], s));
    }
    const int rows_per_wg = panel_rows_for(m, std::min<int>(p.kmax, QK_KM));
    bool switch_qp3 = false;
    HIP_TRY(hipMemsetAsync(ws + L.flag, 0, sizeof(int32_t) * (size_t)n, s));
    int64_t ns_known = 0;
    int64_t nrec = 0;
    int64_t iter = 0;
    bool finished = false;
    const int ring = g_ws.ring;
    const int64_t max_iter = pmin + 2;
    // profile events per block: [0] select, [1] panel, [2] panel end, [3..6] the two
    // GEMMs (start/end each), [7] downdate end; g_prof_ev[0..2] = loop start, QP3
    // start, loop end
    const int kEv = 8;
    while (!finished) {
        const int64_t tb = m - ns_known, wb = n - ns_known;
        hipEvent_t *ev = nullptr;
        if (p.profile) {
            if (prof_events(kEv * (size_t)(iter + 1) + 3) != 0) return QRDM_ERR_NOMEM;
            ev = g_prof_ev.data() + 3 + kEv * iter;
            HIP_TRY(hipEventRecord(ev[0], s));
        }
        HIP_TRY(launch_select(a, s));
        HIP_TRY(launch_gram(a, Gp, tb, s));
        HIP_TRY(launch_gram_reduce(a, Gp, G, tb, s));
        HIP_TRY(launch_dm_finish(a, G, nullptr, s));
        HIP_TRY(launch_swap(a, s));
        if (ev) HIP_TRY(hipEventRecord(ev[1], s));
        HIP_TRY(launch_panel(a, PB, VVb, Vw, p.precision == 1 ? Vw32 : nullptr, ldv, tb, rows_per_wg, s));
        if (ev) HIP_TRY(hipEventRecord(ev[2], s));
        // the device is at most lag + 1 blocks of at most kmax columns ahead of
        // ns_known, and the block's own k_s <= kmax columns leave the trailing
        // part (one block more of slack; k_gemm1 flags a grid that is too small)
        const int64_t wlo = wb - (int64_t)(lag + 3) * p.kmax;
        HIP_TRY(launch_trail(a, p.precision, VVb, Vw, Vw32, ldv, Z, (double *)(ws + L.yp), tb, wb, wlo, s,
                             ev ? ev + 3 : nullptr));
        {
            QrdmArgs al = a;
            al.snap = g_ws.dev_snap + (iter % ring) * QRDM_SNAP_WORDS;  // written by the downdate kernel
            HIP_TRY(launch_downdate(al, wb, s));
        }
        if (ev) HIP_TRY(hipEventRecord(ev[7], s));
        HIP_TRY(hipEventRecord(g_ws.events[iter % ring], s));
        if (iter >= lag) {
            const int64_t k = iter - lag;
            HIP_TRY(hipEventSynchronize(g_ws.events[k % ring]));
            const Snapshot sn = g_ws.host_snap[k % ring];
            if (sn.ns > ns_known) ns_known = sn.ns;
            if (log && !sn.done) {
                if (nrec < log_cap) {
                    qrdm_block b;
                    b.ns = sn.ns;
                    b.nL = sn.nL;
                    b.ks = sn.ks;
                    b.l = sn.l;
                    b.fallback = sn.fallback;
                    b.umax = 0.0;
                    b.gamma = sn.gamma;
                    b.sigma_bound = sn.sigma_bound;
                    log[nrec] = b;
                }
                ++nrec;
            }
            if (sn.done) finished = true;
            if (sn.fallback && !sn.done) switch_qp3 = true;
        }
        ++iter;
        if (switch_qp3) break;
        if (iter > max_iter + lag + 1) break;  // cannot happen: every block advances n_s
    }
    if (p.profile) HIP_TRY(hipEventRecord(g_prof_ev[1], s));
    Qp3Prof qprof;
    qprof.on = p.profile != 0;
    if (switch_qp3 && !finished) {
        // the partial norms reached the noise level: the rest is scalar pivoting,
        // run in the blocked column-pivoting form (deferred trailing update)
        rc = run_qp3(a, ws, L, kQp3Nb, lag, ns_known, s, &qprof);
        if (rc) return rc;
    }
    if (p.profile) HIP_TRY(hipEventRecord(g_prof_ev[2], s));
    HIP_TRY(hipStreamSynchronize(s));
    QrdmCtl cf;
    HIP_TRY(hipMemcpy(&cf, a.ctl, sizeof cf, hipMemcpyDeviceToHost));
    if (stats && p.profile) {
        // intervals (e, e+1): 0 DM selection, 1 panel, 3 GEMM1 (with the fused
        // recurrence), 5 GEMM2, 6 downdate; 2 and 4 are empty gaps
        double t[kEv - 1] = {0};
        for (int64_t k = 0; k < iter; ++k) {
            hipEvent_t *ev = g_prof_ev.data() + 3 + kEv * k;
            for (int e = 0; e + 1 < kEv; ++e) {
                float ms = 0.f;
                if (hipEventElapsedTime(&ms, ev[e], ev[e + 1]) == hipSuccess) t[e] += ms;
            }
        }
        stats->dm_ms = t[0];
        stats->panel_ms = t[1];
        stats->gemm1_ms = t[3];
        stats->gemm2_ms = t[5];
        stats->downdate_ms = t[6];
        stats->gemm_flop = cf.flop_gemm;
        stats->panel_flop = cf.flop_panel;
        stats->panel_bytes = cf.bytes_panel;
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, g_prof_ev[1], g_prof_ev[2]) == hipSuccess) stats->qp3_ms = ms;
        if (hipEventElapsedTime(&ms, g_prof_ev[0], g_prof_ev[2]) == hipSuccess) stats->total_ms = ms;
        stats->nqp3_launch = qprof.launches;
        stats->qp3_run_ms = qp3_run_ms(qprof.launches);
        stats->qp3_bytes = qprof.launches > 0 ? qp3_bytes(m, n, cf.qp3_start, cf.ns) : 0.0;
    }
    if (cf.error) return QRDM_ERR_HIP + (int)hipErrorLaunchTimeOut;
    *rank = cf.rank >= 0 ? cf.rank : cf.ns;
    if (stats) {
        stats->nblocks = cf.nblocks;
        stats->nbreaks = cf.nbreaks;
        stats->nfallback = cf.nfallback;
        stats->nrecompute = cf.nrecompute;
        stats->ncols_factored = cf.ns;
        stats->npanel = cf.npanel;
    }
    if (nlog) *nlog = nrec;
    if (log && lag == 0) {
        // umax of every logged block is not in the snapshot; leave 0
    }
    return 0;
}

int qrdm_factor(double *A, int64_t m, int64_t n, int64_t lda, double tau, double delta, int32_t kmax,
                double *tau_house, int32_t *perm, int64_t *rank, void *stream) {
    qrdm_params p;
    qrdm_default_params(&p);
    p.tau = tau;
    p.delta = delta;
    p.kmax = kmax;
    return qrdm_factor_ex(A, m, n, lda, &p, tau_house, perm, rank, nullptr, nullptr, 0, nullptr, stream);
}

int qrdm_dm_step(const double *A, int64_t m, int64_t n, int64_t lda, int64_t ns, const double *vn1, double tau,
                 double delta, int32_t kmax, int32_t *L, int32_t *nL, double *theta, int32_t *J, int32_t *ks,
                 void *stream) {
    qrdm_params p;
    qrdm_default_params(&p);
    p.tau = tau;
    p.delta = delta;
    p.kmax = kmax;
    int rc = check_common(A, m, n, lda, &p);
    if (rc) return rc;
    if (ns < 0 || ns >= std::min(m, n)) return -5;
    if (!vn1) return -6;
    if (!L || !nL || !J || !ks) return -10;
    if (n > 32768) return QRDM_ERR_UNSUPPORTED;
    hipStream_t s = (hipStream_t)stream;
    Layout Ly = make_layout(m, n);
    rc = ensure_workspace(Ly.total, 8);
    if (rc) return rc;
    char *ws = g_ws.base;
    QrdmArgs a;
    a.A = (double *)A;
    a.m = m;
    a.n = n;
    a.lda = lda;
    a.tau = tau;
    a.delta = delta;
    a.kmax = kmax;
    a.stop_rule = QRDM_STOP_NONE;
    a.eps1 = 0.0;
    a.fbeps = (double)n * 2.220446049250313e-16;
    a.tol3z = 1.4901161193847656e-08;
    a.vn1 = (double *)(ws + Ly.vn1);
    a.vn2 = (double *)(ws + Ly.vn2);
    a.perm = (int32_t *)(ws + Ly.perm_dbg);
    a.tau_house = nullptr;
    a.ctl = (QrdmCtl *)(ws + Ly.ctl);
    HIP_TRY(hipMemcpyAsync(a.vn1, vn1, sizeof(double) * n, hipMemcpyDeviceToDevice, s));
    HIP_TRY(hipMemcpyAsync(a.vn2, vn1, sizeof(double) * n, hipMemcpyDeviceToDevice, s));
    std::vector<int32_t> id(n);
    for (int64_t j = 0; j < n; ++j) id[j] = (int32_t)j;
    HIP_TRY(hipMemcpyAsync(a.perm, id.data(), sizeof(int32_t) * n, hipMemcpyHostToDevice, s));
    QrdmCtl c0 = initial_ctl();
    c0.ns = ns;
    c0.rank = 0;        // stopping test already decided: not applied here
    c0.nblocks = 1;     // keep amax as given
    c0.amax = 2.2250738585072014e-308;  // fallback test never fires for a non-zero trailing block
    HIP_TRY(hipMemcpyAsync(a.ctl, &c0, sizeof c0, hipMemcpyHostToDevice, s));
    double *Gp = (double *)(ws + Ly.gp), *G = (double *)(ws + Ly.g), *th = (double *)(ws + Ly.theta);
    HIP_TRY(launch_select(a, s));
    HIP_TRY(launch_gram(a, Gp, m - ns, s));
    HIP_TRY(launch_gram_reduce(a, Gp, G, m - ns, s));
    HIP_TRY(launch_dm_finish(a, G, th, s));
    QrdmCtl cf;
    HIP_TRY(hipMemcpyAsync(&cf, a.ctl, sizeof cf, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    *nL = cf.nL;
    *ks = cf.ks;
    for (int i = 0; i < cf.nL; ++i) L[i] = cf.L[i];
    for (int i = 0; i < cf.ks; ++i) J[i] = cf.J[i];
    if (theta && cf.nL > 1) {
        std::vector<double> h((size_t)cf.nL * cf.nL);
        HIP_TRY(hipMemcpy(h.data(), th, sizeof(double) * h.size(), hipMemcpyDeviceToHost));
        for (size_t e = 0; e < h.size(); ++e) theta[e] = h[e];
    } else if (theta && cf.nL == 1) {
        theta[0] = 1.0;
    }
    return 0;
}

int qrp_factor_ex(double *A, int64_t m, int64_t n, int64_t lda, const qrdm_params *pin, int32_t nb,
                  double *tau_house, int32_t *perm, int64_t *rank, qrdm_stats *stats, void *stream) {
    qrdm_params p;
    if (pin) p = *pin; else qrdm_default_params(&p);
    p.kmax = 1;
    p.tau = 1.0;
    p.delta = 0.0;
    p.precision = QRDM_PREC_FP64;
    int rc = check_common(A, m, n, lda, &p);
    if (rc) return rc;
    if (nb < 1 || nb > 64) return -6;
    const int64_t pmin = std::min(m, n);
    if (pmin > 0 && !tau_house) return -7;
    if (n > 0 && !perm) return -8;
    if (!rank) return -9;
    if (m > 65536) return QRDM_ERR_UNSUPPORTED;
    hipStream_t s = (hipStream_t)stream;
    if (stats) memset(stats, 0, sizeof *stats);
    if (pmin == 0) {
        if (n > 0) {
            std::vector<int32_t> id(n);
            for (int64_t j = 0; j < n; ++j) id[j] = (int32_t)j;
            HIP_TRY(hipMemcpyAsync(perm, id.data(), sizeof(int32_t) * n, hipMemcpyHostToDevice, s));
            HIP_TRY(hipStreamSynchronize(s));
        }
        *rank = 0;
        return 0;
    }
    Layout L = make_layout(m, n);
    rc = ensure_workspace(L.total, p.poll_lag + 2);
    if (rc) return rc;
    char *ws = g_ws.base;
    QrdmArgs a;
    memset(&a, 0, sizeof a);
    a.A = A;
    a.m = m;
    a.n = n;
    a.lda = lda;
    a.tau = 1.0;
    a.delta = 0.0;
    a.kmax = 1;
    a.stop_rule = p.stop_rule;
    a.eps1 = (p.eps1_scale > 0.0 ? p.eps1_scale : (double)n) * 2.220446049250313e-16;
    a.fbeps = (double)n * 2.220446049250313e-16;
    a.tol3z = 1.4901161193847656e-08;
    a.vn1 = (double *)(ws + L.vn1);
    a.vn2 = (double *)(ws + L.vn2);
    a.perm = perm;
    a.tau_house = tau_house;
    a.gbar = (uint32_t *)(ws + L.gbar);
    a.ctl = (QrdmCtl *)(ws + L.ctl);
    QrdmCtl c0 = initial_ctl();
    HIP_TRY(hipMemcpyAsync(a.ctl, &c0, sizeof c0, hipMemcpyHostToDevice, s));
    HIP_TRY(hipMemsetAsync(ws + L.flag, 0, sizeof(int32_t) * (size_t)n, s));
    HIP_TRY(launch_colnorm(A, m, n, lda, a.vn1, a.vn2, a.ctl, s));
    int32_t nf = 0;
    HIP_TRY(hipMemcpyAsync(&nf, &a.ctl->nonfinite, sizeof nf, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    if (nf) return QRDM_ERR_NONFINITE;
    HIP_TRY(launch_init(a, s));
    Qp3Prof qprof;
    qprof.on = p.profile != 0;
    if (p.profile) {
        if (prof_events(2) != 0) return QRDM_ERR_NOMEM;
        HIP_TRY(hipEventRecord(g_prof_ev[0], s));
    }
    rc = run_qp3(a, ws, L, nb, p.poll_lag, 0, s, &qprof);
    if (rc) return rc;
    if (p.profile) HIP_TRY(hipEventRecord(g_prof_ev[1], s));
    HIP_TRY(hipStreamSynchronize(s));
    QrdmCtl cf;
    HIP_TRY(hipMemcpy(&cf, a.ctl, sizeof cf, hipMemcpyDeviceToHost));
    if (cf.error) return QRDM_ERR_HIP + (int)hipErrorLaunchTimeOut;
    *rank = cf.rank >= 0 ? cf.rank : cf.ns;
    if (stats) {
        stats->nblocks = cf.nblocks;
        stats->nrecompute = cf.nrecompute;
        stats->ncols_factored = cf.ns;
        if (p.profile) {
            float ms = 0.f;
            if (hipEventElapsedTime(&ms, g_prof_ev[0], g_prof_ev[1]) == hipSuccess) stats->qp3_ms = stats->total_ms = ms;
            stats->nqp3_launch = qprof.launches;
            stats->qp3_run_ms = qp3_run_ms(qprof.launches);
            stats->qp3_bytes = qprof.launches > 0 ? qp3_bytes(m, n, cf.qp3_start, cf.ns) : 0.0;
        }
    }
    return 0;
}

int qrp_factor(double *A, int64_t m, int64_t n, int64_t lda, double *tau_house, int32_t *perm, int64_t *rank,
               void *stream) {
    return qrp_factor_ex(A, m, n, lda, nullptr, 32, tau_house, perm, rank, nullptr, stream);
}

}  // extern "C"
