// Host driver and C ABI of libqrdm.so (declared in include/qrdm.h).
//
// The outer loop of Algorithm 4 (QRDM2) is a fixed sequence of kernel
// launches per block; the loop state (n_s, k_s, l, the stop decision, the
// candidate and accepted lists) lives in a device control block and never
// crosses to the host during the loop.  Grids are sized from a lower bound on
// n_s that the host learns by polling a small snapshot of the control block
// `poll_lag` blocks behind the launch front; kernels of blocks enqueued after
// the loop has finished exit at once.
//
// Device state of one call lives in a workspace (the layout below): either the
// library's cache for the current device (qrdm_factor, qrdm_factor_ex, ...;
// calls on it are serialized by a lock) or the caller's (qrdm_factor_ws).
// Host state of one call (the pinned snapshot ring and its events) comes from
// a pool, one entry per call in flight, so calls with their own workspaces run
// concurrently.
#include <hip/hip_runtime.h>

#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <vector>

#include "../../include/qrdm.h"
#include "qrdm_internal.h"

int gram_partials(int64_t t_bound);
int64_t trail_ysplit(int kmax, int64_t n);
int trail_splits_max();

namespace {

struct Snapshot {  // the first QRDM_SNAP_WORDS words of QrdmCtl, polled by the host
    int64_t ns;
    int64_t rank;
    int32_t l, ks, nL, done, fallback, jmax;
    double gamma, sigma_bound, umax;
    int32_t nonfinite, error;
};
static_assert(sizeof(Snapshot) == 8 * QRDM_SNAP_WORDS, "the snapshot is the words the kernels write");
static_assert(offsetof(Snapshot, jmax) == offsetof(QrdmCtl, jmax) &&
                  offsetof(Snapshot, gamma) == offsetof(QrdmCtl, gamma) &&
                  offsetof(Snapshot, umax) == offsetof(QrdmCtl, umax) &&
                  offsetof(Snapshot, error) == offsetof(QrdmCtl, error),
              "the polled snapshot is a prefix of the control block");

// ------------------------------------------------------------ host polling
// Host resources of one call: a ring of snapshot slots in pinned host memory
// (the kernels write them through their device address) with one event per
// slot, and the timing events of the profiling mode.
struct PollCtx {
    int device = -1;
    int ring = 0;
    // copy mode (qrdm_factor_noalloc, which may not allocate pinned memory or
    // events): ring = 1, dev_snap is a slot in device memory and the host reads
    // it with a copy after synchronizing the stream, so the poll lag is 0
    bool copy = false;
    Snapshot *host_snap = nullptr;
    uint64_t *dev_snap = nullptr;
    std::vector<hipEvent_t> events;
    std::vector<hipEvent_t> prof_ev;  // profile mode: loop events and 8 per block
    std::vector<hipEvent_t> qp_ev;    // profile mode: around each QP3 block-kernel launch
    // recorded after the last launch of the call that used the context: kernels
    // launched ahead of the loop's end still write snapshots into the ring, so
    // the context is reused only once this event has completed
    hipEvent_t release_ev = nullptr;
};

std::mutex g_poll_mu;
std::vector<PollCtx *> g_poll_free;

void poll_destroy(PollCtx *pc) {
    if (pc->release_ev) {
        (void)hipEventSynchronize(pc->release_ev);
        (void)hipEventDestroy(pc->release_ev);
    }
    if (pc->host_snap) (void)hipHostFree(pc->host_snap);
    for (auto e : pc->events) (void)hipEventDestroy(e);
    for (auto e : pc->prof_ev) (void)hipEventDestroy(e);
    for (auto e : pc->qp_ev) (void)hipEventDestroy(e);
    delete pc;
}

// A context of the current device with at least `ring` slots (taken from the
// pool, or made).  Returns 0 or QRDM_ERR_NOMEM.
int poll_acquire(int ring, PollCtx **out) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return QRDM_ERR_NOMEM;
    {
        std::lock_guard<std::mutex> g(g_poll_mu);
        for (size_t i = 0; i < g_poll_free.size(); ++i) {
            PollCtx *pc = g_poll_free[i];
            if (pc->device == dev && pc->ring >= ring && hipEventQuery(pc->release_ev) == hipSuccess) {
                g_poll_free.erase(g_poll_free.begin() + (long)i);
                *out = pc;
                return 0;
            }
        }
    }
    PollCtx *pc = new PollCtx();
    pc->device = dev;
    pc->ring = std::max(ring, 8);
    if (hipHostMalloc((void **)&pc->host_snap, sizeof(Snapshot) * pc->ring, hipHostMallocDefault) != hipSuccess ||
        hipHostGetDevicePointer((void **)&pc->dev_snap, pc->host_snap, 0) != hipSuccess) {
        (void)hipGetLastError();
        poll_destroy(pc);
        return QRDM_ERR_NOMEM;
    }
    if (hipEventCreateWithFlags(&pc->release_ev, hipEventDisableTiming) != hipSuccess) {
        pc->release_ev = nullptr;
        poll_destroy(pc);
        return QRDM_ERR_NOMEM;
    }
    pc->events.resize(pc->ring);
    for (int i = 0; i < pc->ring; ++i) {
        if (hipEventCreateWithFlags(&pc->events[i], hipEventDisableTiming) != hipSuccess) {
            pc->events.resize(i);
            poll_destroy(pc);
            return QRDM_ERR_NOMEM;
        }
    }
    *out = pc;
    return 0;
}

void poll_release(PollCtx *pc, hipStream_t s) {
    if (hipEventRecord(pc->release_ev, s) != hipSuccess) {
        // the stream is unusable: wait for the device before the ring is reused
        (void)hipGetLastError();
        (void)hipDeviceSynchronize();
        (void)hipEventRecord(pc->release_ev, nullptr);
    }
    std::lock_guard<std::mutex> g(g_poll_mu);
    g_poll_free.push_back(pc);
}

struct PollGuard {  // returns the context to the pool on every exit path
    PollCtx *pc = nullptr;
    hipStream_t s = nullptr;
    ~PollGuard() {
        if (pc) poll_release(pc, s);
    }
};

int grow_events(std::vector<hipEvent_t> &v, size_t count) {
    while (v.size() < count) {
        hipEvent_t e;
        if (hipEventCreate(&e) != hipSuccess) return -1;
        v.push_back(e);
    }
    return 0;
}

// ------------------------------------------------------------ workspace
struct Layout {
    size_t ctl, vn1, vn2, gp, g, theta, pb, tm, vw, vw32, z, yp, pb2, fz, flag, qrb, gbar, perm_dbg, cp, total;
};

const int kMinRowsPerWg = 16;  // smallest panel slab (bounds the partial buffer)
const int kQp3NbMax = 64;      // largest block of the column-pivoting update

size_t align_up(size_t x) { return (x + 255) & ~(size_t)255; }

// Device workspace of one call for an m x n matrix and block size kmax.
Layout make_layout(int64_t m, int64_t n, int kmax) {
    Layout L;
    size_t off = 0;
    auto take = [&](size_t bytes) { size_t o = off; off = align_up(off + bytes); return o; };
    const int64_t mm = std::max<int64_t>(m, 1), nn = std::max<int64_t>(n, 1);
    const size_t kp = (size_t)((std::min(std::max(kmax, 1), QK_KM) + 15) & ~15);  // k_DM in 16-wide tiles
    L.ctl = take(sizeof(QrdmCtl));
    L.vn1 = take(sizeof(double) * nn);
    L.vn2 = take(sizeof(double) * nn);
    L.gp = take(sizeof(double) * (size_t)std::max(gram_partials(mm), cpanel_partials(mm)) * kp * kp);
    L.g = take(sizeof(double) * QK_KM * QK_KM);
    L.theta = take(sizeof(double) * QK_KM * QK_KM);
    const int64_t pmax = (mm + kMinRowsPerWg - 1) / kMinRowsPerWg;
    // panel: 4096 reserved words (16 KB), rows c and c+1 (2 x 2 QK_KM), partial dots (2 x pmax x 2 QK_KM)
    L.pb = take(16384 + sizeof(double) * (4 * QK_KM + 2 * (size_t)pmax * 2 * QK_KM));
    L.tm = take(sizeof(double) * QK_KM * QK_KM);
    L.vw = take(sizeof(double) * kp * (size_t)mm);
    L.vw32 = take(sizeof(float) * kp * (size_t)mm);
    L.z = take(sizeof(double) * kp * (size_t)nn);
    // split-K partials of V^T A; the column-pivoting tail kernel, which runs after
    // the DM loop, publishes its partials and column copies in the same region
    L.yp = take(sizeof(double) * std::max((size_t)trail_splits_max() * (size_t)trail_ysplit((int)kp, nn),
                                          qp3_tail_pub_doubles(mm)));
    L.pb2 = take(sizeof(double) * (size_t)((mm + 255) / 256) * (2 + 2 * 64));
    L.fz = take(sizeof(double) * kQp3NbMax * (size_t)nn);
    L.flag = take(sizeof(int32_t) * (size_t)nn);
    // QP3 block kernel: 4 doubles of arg-max partials per workgroup
    L.qrb = take(sizeof(double) * 4 * QP_RUN_MAXWG);
    L.gbar = take(2 * sizeof(uint32_t) * GBAR_GROUPS * GBAR_STRIDE);  // grid-barrier counters: panel, QP3 block kernel (2 sets)
    L.perm_dbg = take(sizeof(int32_t) * nn);
    L.cp = take(sizeof(double) * CP_DOUBLES);  // the Gram-matrix panel's small matrices
    L.total = off;
    return L;
}

// The library's workspace for the current device (entry points without a
// workspace argument).  Held under g_ws_mu for the whole call.
struct CachedWs {
    int device = -1;
    size_t bytes = 0;
    char *base = nullptr;
};
std::mutex g_ws_mu;
CachedWs g_ws;

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

// Marks snapshot `slot` as launched (an event after the launch that writes it).
int poll_mark(PollCtx &pc, int64_t slot, hipStream_t s) {
    if (pc.copy) return 0;
    HIP_TRY(hipEventRecord(pc.events[slot % pc.ring], s));
    return 0;
}

// Waits for snapshot `slot` and returns it.  src: the device words the slot's
// snapshot is read from in copy mode (the ring slot, or the control block
// itself when the kernels write no snapshot).
int poll_read(PollCtx &pc, int64_t slot, const void *src, hipStream_t s, Snapshot *out) {
    if (pc.copy) {
        HIP_TRY(hipMemcpyAsync(out, src, sizeof(Snapshot), hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        return 0;
    }
    HIP_TRY(hipEventSynchronize(pc.events[slot % pc.ring]));
    *out = pc.host_snap[slot % pc.ring];
    return 0;
}

// Caller holds g_ws_mu.
int ensure_workspace(size_t bytes) {
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    if (g_ws.base && g_ws.device == dev && g_ws.bytes >= bytes) return 0;
    if (g_ws.base) {
        (void)hipDeviceSynchronize();
        (void)hipFree(g_ws.base);
        g_ws.base = nullptr;
        g_ws.bytes = 0;
    }
    const char *fault = getenv("QRDM_FAULT");
    if (fault && strcmp(fault, "alloc") == 0) return QRDM_ERR_NOMEM;
    size_t want = bytes;
    if (hipMalloc((void **)&g_ws.base, want) != hipSuccess) {
        g_ws.base = nullptr;
        g_ws.bytes = 0;
        (void)hipGetLastError();
        return QRDM_ERR_NOMEM;
    }
    g_ws.bytes = want;
    g_ws.device = dev;
    return 0;
}

int check_params(const qrdm_params *p) {
    if (!(p->tau >= 0.0 && p->tau <= 1.0)) return -5;
    if (!(p->delta >= 0.0 && p->delta <= 1.0)) return -5;
    if (p->kmax < 1 || p->kmax > QRDM_KMAX_LIMIT) return -5;
    if (p->stop_rule < 0 || p->stop_rule > 2) return -5;
    if (p->precision < 0 || p->precision > 1) return -5;
    if (p->poll_lag < 0 || p->poll_lag > 1024) return -5;
    if (p->profile < 0 || p->profile > 1) return -5;
    if (p->certified < 0 || p->certified > 1) return -5;
    return 0;
}

int check_common(const double *A, int64_t m, int64_t n, int64_t lda, const qrdm_params *p) {
    if (m < 0) return -2;
    if (n < 0) return -3;
    if (lda < std::max<int64_t>(1, m)) return -4;
    if (p) {
        int rc = check_params(p);
        if (rc) return rc;
    }
    if (m > 0 && n > 0 && !A) return -1;
    return 0;
}

const int kQp3Nb = 32;  // block size of the column-pivoting update
const double kEps64 = 2.220446049250313e-16;
const double kEps32 = 1.1920928955078125e-07;

// Profiling record of one loop (events in the call's PollCtx).
struct ProfRun {
    bool on = false;
    int64_t dm_iters = 0;     // DM steps with 8 events each
    int64_t qp_launches = 0;  // QP3 block- and tail-kernel launches with 2 events each
    int64_t tail_launches = 0;  // of which tail-kernel launches (0 or 1)
};

// The failure a snapshot reports (NaN/Inf in A, a timed-out grid wait), or 0.
int snapshot_code(const Snapshot &sn) {
    if (sn.nonfinite) return QRDM_ERR_NONFINITE;
    if (sn.error) return QRDM_ERR_HIP + (int)hipErrorLaunchTimeOut;
    return 0;
}
const int kEv = 8;  // per DM step: select, panel, panel end, GEMM1/GEMM2 start/end, downdate end

double qp3_bytes(int64_t m, int64_t n, int64_t j0, int64_t j1) {
    double b = 0.0;
    for (int64_t j = j0; j < j1; ++j) b += 8.0 * (double)(m - j) * (double)(n - j);
    return b;
}

// Column pivoting steps from the device's current n_s until the loop is done.
// *last receives the snapshot with done = 1.
int run_qp3(const QrdmArgs &a, char *ws, const Layout &L, int nb, int lag, int64_t ns_known, hipStream_t s,
            PollCtx &pc, ProfRun &prof, Snapshot *last) {
    Qp3Bufs bf;
    bf.PB2 = (double *)(ws + L.pb2);
    bf.Fz = (double *)(ws + L.fz);
    bf.flag = (int32_t *)(ws + L.flag);
    bf.amx = (double *)(ws + L.qrb);
    bf.pub = (double *)(ws + L.yp);
    HIP_TRY(launch_qp3_init(a, nb, s));
    const int ring = pc.ring;
    const int64_t pmin = std::min(a.m, a.n);
    const char *mode = getenv("QRDM_QP3_STEPS");  // "1": the per-step kernels (comparison runs)
    const int grid = (mode && strcmp(mode, "1") == 0) ? 0 : qp3_block_grid(a.m);
    // "0": no register-resident tail (comparison runs of the block kernel)
    const char *tmode = getenv("QRDM_QP3_TAIL");
    const int tgrid = (grid > 0 && !(tmode && strcmp(tmode, "0") == 0)) ? qp3_tail_grid() : 0;
    if (grid > 0) {
        // one block of up to nb steps per launch; a snapshot after each, the
        // host waiting on the one `lag` launches back; once the trailing block
        // fits in LDS (by the host's bound), one tail launch takes every
        // remaining step
        for (int64_t iter = 0;; ++iter) {
            const int64_t tb = a.m - ns_known, wb = a.n - ns_known;
            hipEvent_t *ev = nullptr;
            if (prof.on) {
                if (grow_events(pc.qp_ev, 2 * (size_t)(iter + 1)) != 0) return QRDM_ERR_NOMEM;
                ev = pc.qp_ev.data() + 2 * iter;
                prof.qp_launches = iter + 1;
            }
            QrdmArgs al = a;
            al.snap = pc.dev_snap + (iter % ring) * QRDM_SNAP_WORDS;  // written by the block or tail kernel
            int cq = 0, crows = 0;
            size_t lds = 0;
            if (tgrid > 0 && qp3_tail_shape(tb, wb, tgrid, &cq, &crows, &lds)) {
                HIP_TRY(launch_qp3_tail(al, bf.pub, bf.flag, tb, wb, tgrid, (int)iter, s, ev));
                if (prof.on) prof.tail_launches += 1;
                int rc = poll_mark(pc, iter, s);
                if (rc) return rc;
                // the launches before it are older: this snapshot is the last one
                Snapshot sn;
                rc = poll_read(pc, iter, pc.dev_snap + (iter % ring) * QRDM_SNAP_WORDS, s, &sn);
                if (rc) return rc;
                if (!sn.done) return (sn.error || sn.nonfinite) ? snapshot_code(sn) : QRDM_ERR_INTERNAL;
                *last = sn;
                return 0;
            }
            HIP_TRY(launch_qp3_block(al, bf, nb, tb, wb, grid, (int)iter, s, ev));
            int rc = poll_mark(pc, iter, s);
            if (rc) return rc;
            if (iter >= lag) {
                const int64_t k = iter - lag;
                Snapshot sn;
                rc = poll_read(pc, k, pc.dev_snap + (k % ring) * QRDM_SNAP_WORDS, s, &sn);
                if (rc) return rc;
                if (sn.ns > ns_known) ns_known = sn.ns;
                if (sn.done) {
                    *last = sn;
                    return 0;
                }
            }
            // every launch takes at least one step: more launches than steps is a fault
            if (iter > pmin + lag + 4) return QRDM_ERR_INTERNAL;
        }
    }
    // snapshots every kStride steps; the host waits on the one `lag` snapshots back
    const int kStride = 4;
    int64_t nsnap = 0;
    for (int64_t iter = 0;; ++iter) {
        const int64_t tb = a.m - ns_known, wb = a.n - ns_known;
        HIP_TRY(launch_qp3_step(a, bf, nb, tb, wb, s));
        if ((iter + 1) % kStride != 0) continue;
        if (!pc.copy)
            HIP_TRY(hipMemcpyAsync(pc.host_snap + (nsnap % ring), a.ctl, sizeof(Snapshot), hipMemcpyDeviceToHost, s));
        int rc = poll_mark(pc, nsnap, s);
        if (rc) return rc;
        if (nsnap >= lag) {
            const int64_t k = nsnap - lag;
            Snapshot sn;
            rc = poll_read(pc, k, a.ctl, s, &sn);
            if (rc) return rc;
            if (sn.ns > ns_known) ns_known = sn.ns;
            if (sn.done) {
                *last = sn;
                return 0;
            }
        }
        ++nsnap;
        // every step advances n_s: more steps than columns is a fault
        if (iter > 2 * pmin + kStride * (lag + 4)) return QRDM_ERR_INTERNAL;
    }
}

// What one factorization call needs besides the matrix arguments.
struct CallEnv {
    char *ws;             // device workspace (layout L)
    Layout L;
    PollCtx *pc;
    hipStream_t s;
    qrdm_block *log;      // may be null
    int64_t log_cap;
    int64_t *nlog;        // may be null
    int64_t *rank_dev;    // may be null: the rank is also written to device memory
};

void prof_fill(const ProfRun &prof, PollCtx &pc, const QrdmCtl &cf, int64_t m, int64_t n, qrdm_stats *st) {
    double t[kEv - 1] = {0};
    for (int64_t k = 0; k < prof.dm_iters; ++k) {
        hipEvent_t *ev = pc.prof_ev.data() + 3 + kEv * k;
        for (int e = 0; e + 1 < kEv; ++e) {
            float ms = 0.f;
            if (hipEventElapsedTime(&ms, ev[e], ev[e + 1]) == hipSuccess) t[e] += ms;
        }
    }
    // intervals (e, e+1): 0 DM selection, 1 panel, 3 GEMM1, 4 partial sum and Z,
    // 5 GEMM2, 6 downdate
    st->dm_ms = t[0];
    st->panel_ms = t[1];
    st->gemm1_ms = t[3];
    st->zsum_ms = t[4];
    st->gemm2_ms = t[5];
    st->downdate_ms = t[6];
    st->gemm_flop = cf.flop_gemm;
    st->gemm2_bytes = cf.bytes_gemm2;
    st->panel_flop = cf.flop_panel;
    st->panel_bytes = cf.bytes_panel;
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, pc.prof_ev[1], pc.prof_ev[2]) == hipSuccess) st->qp3_ms = ms;
    if (hipEventElapsedTime(&ms, pc.prof_ev[0], pc.prof_ev[2]) == hipSuccess) st->total_ms = ms;
    st->nqp3_launch = prof.qp_launches;
    st->nqp3_tail = prof.tail_launches;
    double q = 0.0;
    for (int64_t i = 0; i < prof.qp_launches; ++i) {
        float x = 0.f;
        if (hipEventElapsedTime(&x, pc.qp_ev[2 * i], pc.qp_ev[2 * i + 1]) == hipSuccess) q += x;
    }
    st->qp3_run_ms = q;
    st->qp3_bytes = prof.qp_launches > 0 ? qp3_bytes(m, n, cf.qp3_start, cf.ns) : 0.0;
}

void stats_fill(const QrdmCtl &cf, qrdm_stats *st) {
    st->nblocks = cf.nblocks;
    st->nbreaks = cf.nbreaks;
    st->nrecompute = cf.nrecompute;
    st->ncols_factored = cf.ns;
    st->npanel = cf.npanel;
    st->ngram = cf.ngram;
    st->qp3_start = cf.fallback ? cf.qp3_start : -1;
    st->nfallback = cf.fallback ? cf.ns - cf.qp3_start : 0;
}

// The QRDM loop of one call (Algorithm 4 with Algorithm 1), from the
// workspace reset to the last launch.  On success *final holds the snapshot in
// which the device reported the loop done.  Nothing here waits for the whole
// stream: the host waits on the events of its own snapshots.
int qrdm_run(double *A, int64_t m, int64_t n, int64_t lda, const qrdm_params &p, double *tau_house, int32_t *perm,
             const CallEnv &env, ProfRun &prof, Snapshot *final) {
    char *ws = env.ws;
    const Layout &L = env.L;
    PollCtx &pc = *env.pc;
    hipStream_t s = env.s;
    const int lag = (env.log || env.pc->copy) ? 0 : p.poll_lag;
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
    a.lemma = (env.log != nullptr || p.certified) ? 1 : 0;
    // eps_w, the unit roundoff of the trailing data: 2^-52 (FP64) or 2^-23 in
    // mixed mode, where every trailing update rounds to FP32.  The stopping
    // test (eps_1 = n eps_w) and the recompute tolerance sqrt(eps_w) follow the
    // data; the switch to scalar pivoting stays at n 2^-52 max ||a_j||, which
    // the FP32 rounding noise (about 2^-23 ||A||) never reaches, so mixed mode
    // keeps taking DM blocks to the end.
    const double eps_w = (p.precision == QRDM_PREC_MIXED) ? kEps32 : kEps64;
    a.eps1 = (p.eps1_scale > 0.0 ? p.eps1_scale : (double)n) * eps_w;
    a.fbeps = (double)n * kEps64;
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
    double *cp = (double *)(ws + L.cp);
    const int kpg = (std::min(std::max(p.kmax, 1), QK_KM) + 15) & ~15;  // leading dimension of the Gram partials
    void *Z = ws + L.z;
    const int64_t ldv = m;
    const int64_t pmin = std::min(m, n);

    HIP_TRY(launch_ws_reset(a.ctl, (int32_t *)(ws + L.flag), n, s));
    // NaN/Inf raises the control block's flag: the loop then ends at its first
    // selection with nothing written
    HIP_TRY(launch_colnorm(A, m, n, lda, a.vn1, a.vn2, a.ctl, s));
    HIP_TRY(launch_init(a, s));

    if (prof.on) {
        if (grow_events(pc.prof_ev, 3) != 0) return QRDM_ERR_NOMEM;
        HIP_TRY(hipEventRecord(pc.prof_ev[0], s));
    }
    const int rows_per_wg = panel_rows_for(m, std::min<int>(p.kmax, QK_KM));
    // "0": every block on the column-by-column panel (comparison runs)
    const char *gmode = getenv("QRDM_GRAM_PANEL");
    const int gram = !(gmode && strcmp(gmode, "0") == 0);
    bool switch_qp3 = false, finished = false;
    int64_t ns_known = 0, nrec = 0, iter = 0;
    const int ring = pc.ring;
    Snapshot last;
    memset(&last, 0, sizeof last);
    while (!finished) {
        const int64_t tb = m - ns_known, wb = n - ns_known;
        hipEvent_t *ev = nullptr;
        if (prof.on) {
            if (grow_events(pc.prof_ev, kEv * (size_t)(iter + 1) + 3) != 0) return QRDM_ERR_NOMEM;
            ev = pc.prof_ev.data() + 3 + kEv * iter;
            prof.dm_iters = iter + 1;
            HIP_TRY(hipEventRecord(ev[0], s));
        }
        HIP_TRY(launch_select(a, s));
        HIP_TRY(launch_gram(a, Gp, tb, s));
        HIP_TRY(launch_gram_reduce(a, Gp, G, tb, s));
        HIP_TRY(launch_dm_finish(a, G, nullptr, s));
        HIP_TRY(launch_cpchol(a, G, cp, gram, s));
        HIP_TRY(launch_swap(a, s));
        if (ev) HIP_TRY(hipEventRecord(ev[1], s));
        // the panel: from the Gram matrix when the block allows it, else (and
        // then only) column by column
        float *v32 = p.precision == 1 ? Vw32 : nullptr;
        if (gram) {
            HIP_TRY(launch_cpanel1(a, cp, Vw, ldv, Gp, kpg, tb, s));
            HIP_TRY(launch_cpreduce(a, Gp, kpg, cp, s));
            HIP_TRY(launch_cpanel2(a, cp, Vw, ldv, Vw, v32, s));
            HIP_TRY(launch_cpanel3(a, cp, Vw, ldv, v32, tb, s));
        }
        HIP_TRY(launch_panel(a, PB, VVb, Vw, v32, ldv, tb, rows_per_wg, s));
        if (ev) HIP_TRY(hipEventRecord(ev[2], s));
        // the device is at most lag + 1 blocks of at most kmax columns ahead of
        // ns_known, and the block's own k_s <= kmax columns leave the trailing
        // part (one block more of slack; k_gemm1 flags a grid that is too small)
        const int64_t wlo = wb - (int64_t)(lag + 3) * p.kmax;
        HIP_TRY(launch_trail(a, p.precision, VVb, cp + CP_OFF_T, Vw, Vw32, ldv, Z, (double *)(ws + L.yp), tb, wb, wlo, s,
                             ev ? ev + 3 : nullptr));
        {
            QrdmArgs al = a;
            al.snap = pc.dev_snap + (iter % ring) * QRDM_SNAP_WORDS;  // written by the downdate kernel
            HIP_TRY(launch_downdate(al, wb, s));
        }
        if (ev) HIP_TRY(hipEventRecord(ev[7], s));
        {
            int rc = poll_mark(pc, iter, s);
            if (rc) return rc;
        }
        if (iter >= lag) {
            const int64_t k = iter - lag;
            Snapshot sn;
            int rc = poll_read(pc, k, pc.dev_snap + (k % ring) * QRDM_SNAP_WORDS, s, &sn);
            if (rc) return rc;
            if (sn.ns > ns_known) ns_known = sn.ns;
            // a step that took a block (not the one that ended the loop or passed it
            // to the column-pivoting kernels)
            if (env.log && !sn.done && sn.l > 0) {
                if (nrec < env.log_cap) {
                    qrdm_block b;
                    b.ns = sn.ns;
                    b.nL = sn.nL;
                    b.ks = sn.ks;
                    b.l = sn.l;
                    b.fallback = 0;
                    b.umax = sn.umax;
                    b.gamma = sn.gamma;
                    b.sigma_bound = sn.sigma_bound;
                    env.log[nrec] = b;
                }
                ++nrec;
            }
            if (sn.done) {
                finished = true;
                last = sn;
            } else if (sn.fallback) {
                switch_qp3 = true;
                if (env.log) {  // the hand-over: column pivoting from column sn.ns on
                    if (nrec < env.log_cap) {
                        qrdm_block b;
                        memset(&b, 0, sizeof b);
                        b.ns = sn.ns;
                        b.fallback = 1;
                        b.umax = sn.umax;
                        env.log[nrec] = b;
                    }
                    ++nrec;
                }
            }
        }
        ++iter;
        if (switch_qp3) break;
        // every step that neither ends nor hands over takes >= 1 column
        if (iter > pmin + lag + 4) return QRDM_ERR_INTERNAL;
    }
    if (prof.on) HIP_TRY(hipEventRecord(pc.prof_ev[1], s));
    if (switch_qp3) {
        // the partial norms reached the noise level (eq. column_norm_bound_DM):
        // the rest is scalar pivoting, run in the blocked column-pivoting form
        int rc = run_qp3(a, ws, L, kQp3Nb, lag, ns_known, s, pc, prof, &last);
        if (rc) return rc;
    }
    if (prof.on) HIP_TRY(hipEventRecord(pc.prof_ev[2], s));
    if (env.rank_dev) HIP_TRY(launch_rank_out(a.ctl, env.rank_dev, s));
    if (env.nlog) *env.nlog = nrec;
    *final = last;
    return 0;
}

// Trivial shapes (min(m, n) = 0): perm = identity, rank 0.
__global__ void k_trivial(int32_t *perm, int64_t n, int64_t *rank_dev) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) perm[i] = (int32_t)i;
    if (i == 0 && rank_dev) *rank_dev = 0;
}
int trivial(int32_t *perm, int64_t n, int64_t *rank_dev, hipStream_t s) {
    const int64_t cnt = std::max<int64_t>(n, 1);
    hipLaunchKernelGGL(k_trivial, dim3((unsigned)((cnt + 255) / 256)), dim3(256), 0, s, perm, n, rank_dev);
    HIP_TRY(hipGetLastError());
    return 0;
}

// Arguments of the factorization entry points after the parameters: -6..-8.
int check_outputs(int64_t m, int64_t n, const double *tau_house, const int32_t *perm) {
    if (std::min(m, n) > 0 && !tau_house) return -6;
    if (n > 0 && !perm) return -7;
    return 0;
}

}  // namespace

// ------------------------------------------------------------ no-allocation entry point
// qrdm_factor_noalloc runs in this fixed device array instead of an allocated
// workspace: a 256-byte snapshot slot, then the workspace of one call (the
// layout of make_layout, at most QRDM_NOALLOC_WS_MAX bytes).  Each device that
// runs the library holds its own copy until the process ends.  The array's
// name stands for a host-side shadow in host code: only the device address
// from hipGetSymbolAddress (taken once per device, kept in g_scratch_addr) is
// passed to kernels and copies.
#define QRDM_SCRATCH_SNAP_BYTES 256
static __device__ __align__(256) unsigned char scratch[QRDM_SCRATCH_SNAP_BYTES + QRDM_NOALLOC_WS_MAX];

namespace {

const int kScratchDevices = 64;
std::mutex g_scratch_mu;
char *g_scratch_addr[kScratchDevices] = {};

// Device address of the current device's scratch (looked up on the first call
// on that device).
int scratch_base(char **out) {
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    if (dev < 0 || dev >= kScratchDevices) return QRDM_ERR_UNSUPPORTED;
    std::lock_guard<std::mutex> g(g_scratch_mu);
    if (!g_scratch_addr[dev]) {
        void *ptr = nullptr;
        HIP_TRY(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
        if (!ptr || ((uintptr_t)ptr & 255) != 0) return QRDM_ERR_HIP + (int)hipErrorInvalidSymbol;
        g_scratch_addr[dev] = (char *)ptr;
    }
    *out = g_scratch_addr[dev];
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
    if (code == QRDM_ERR_INTERNAL) return "internal error: the host loop exceeded its bound on the steps";
    if (code == QRDM_ERR_WORKSPACE) return "workspace smaller than qrdm_workspace_size";
    if (code == QRDM_ERR_SCRATCH)
        return "qrdm_workspace_size of this shape exceeds the fixed scratch of qrdm_factor_noalloc "
               "(QRDM_NOALLOC_WS_MAX)";
    if (code >= QRDM_ERR_HIP) return hipGetErrorString((hipError_t)(code - QRDM_ERR_HIP));
    return "unknown error";
}

void qrdm_release(void) {
    {
        std::lock_guard<std::mutex> g(g_ws_mu);
        if (g_ws.base) {
            (void)hipDeviceSynchronize();
            (void)hipFree(g_ws.base);
        }
        g_ws = CachedWs();
    }
    std::lock_guard<std::mutex> g(g_poll_mu);
    for (PollCtx *pc : g_poll_free) poll_destroy(pc);
    g_poll_free.clear();
}

size_t qrdm_workspace_size(int64_t m, int64_t n, const qrdm_params *p) {
    if (m < 0 || n < 0) return 0;
    qrdm_params q;
    if (p) q = *p; else qrdm_default_params(&q);
    return make_layout(m, n, q.kmax).total;
}

int qrdm_colnorms(const double *A, int64_t m, int64_t n, int64_t lda, double *out, void *stream) {
    int rc = check_common(A, m, n, lda, nullptr);
    if (rc) return rc;
    if (n > 0 && !out) return -5;
    if (n == 0) return 0;
    hipStream_t s = (hipStream_t)stream;
    std::lock_guard<std::mutex> lk(g_ws_mu);
    Layout L = make_layout(m, n, 1);
    rc = ensure_workspace(L.total);
    if (rc) return rc;
    QrdmCtl *ctl = (QrdmCtl *)(g_ws.base + L.ctl);
    double *vn2 = (double *)(g_ws.base + L.vn2);
    HIP_TRY(launch_ws_reset(ctl, (int32_t *)(g_ws.base + L.flag), n, s));
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
    rc = check_outputs(m, n, tau_house, perm);
    if (rc) return rc;
    if (!rank) return -8;
    if (log && log_cap < 0) return -11;
    if (n > 32768 || m > 65536) return QRDM_ERR_UNSUPPORTED;
    hipStream_t s = (hipStream_t)stream;
    if (stats) memset(stats, 0, sizeof *stats);
    if (nlog) *nlog = 0;
    if (std::min(m, n) == 0) {
        rc = trivial(perm, n, nullptr, s);
        if (rc) return rc;
        HIP_TRY(hipStreamSynchronize(s));
        *rank = 0;
        if (stats) stats->qp3_start = -1;
        return 0;
    }
    std::lock_guard<std::mutex> lk(g_ws_mu);
    CallEnv env;
    env.L = make_layout(m, n, p.kmax);
    rc = ensure_workspace(env.L.total);
    if (rc) return rc;
    PollGuard pg;
    pg.s = s;
    rc = poll_acquire((log ? 0 : p.poll_lag) + 2, &pg.pc);
    if (rc) return rc;
    env.ws = g_ws.base;
    env.pc = pg.pc;
    env.s = s;
    env.log = log;
    env.log_cap = log_cap;
    env.nlog = nlog;
    env.rank_dev = nullptr;
    ProfRun prof;
    prof.on = p.profile != 0;
    Snapshot fin;
    rc = qrdm_run(A, m, n, lda, p, tau_house, perm, env, prof, &fin);
    if (rc) return rc;
    HIP_TRY(hipStreamSynchronize(s));
    QrdmCtl cf;
    HIP_TRY(hipMemcpy(&cf, env.ws + env.L.ctl, sizeof cf, hipMemcpyDeviceToHost));
    if (cf.nonfinite) return QRDM_ERR_NONFINITE;
    if (cf.error) return QRDM_ERR_HIP + (int)hipErrorLaunchTimeOut;
    *rank = cf.rank >= 0 ? cf.rank : cf.ns;
    if (stats) {
        stats_fill(cf, stats);
        if (prof.on) prof_fill(prof, *pg.pc, cf, m, n, stats);
    }
    return 0;
}

int qrdm_factor_ws(double *A, int64_t m, int64_t n, int64_t lda, const qrdm_params *pin, double *tau_house,
                   int32_t *perm, int64_t *rank_dev, qrdm_stats *stats, void *workspace, size_t ws_bytes,
                   void *stream) {
    qrdm_params p;
    if (pin) p = *pin; else qrdm_default_params(&p);
    int rc = check_common(A, m, n, lda, &p);
    if (rc) return rc;
    rc = check_outputs(m, n, tau_house, perm);
    if (rc) return rc;
    if (!rank_dev) return -8;
    if (p.profile) return -5;  // timing events are for qrdm_factor_ex
    if (n > 32768 || m > 65536) return QRDM_ERR_UNSUPPORTED;
    hipStream_t s = (hipStream_t)stream;
    if (stats) memset(stats, 0, sizeof *stats);
    if (std::min(m, n) == 0) {
        if (stats) stats->qp3_start = -1;
        return trivial(perm, n, rank_dev, s);
    }
    CallEnv env;
    env.L = make_layout(m, n, p.kmax);
    if (!workspace) return -10;
    if (ws_bytes < env.L.total) return QRDM_ERR_WORKSPACE;
    if (((uintptr_t)workspace & 255) != 0) return -10;
    PollGuard pg;
    pg.s = s;
    rc = poll_acquire(p.poll_lag + 2, &pg.pc);
    if (rc) return rc;
    env.ws = (char *)workspace;
    env.pc = pg.pc;
    env.s = s;
    env.log = nullptr;
    env.log_cap = 0;
    env.nlog = nullptr;
    env.rank_dev = rank_dev;
    ProfRun prof;
    Snapshot fin;
    rc = qrdm_run(A, m, n, lda, p, tau_house, perm, env, prof, &fin);
    if (rc) return rc;
    rc = snapshot_code(fin);
    if (rc) return rc;
    if (stats) {
        QrdmCtl cf;
        HIP_TRY(hipMemcpyAsync(&cf, env.ws + env.L.ctl, sizeof cf, hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        stats_fill(cf, stats);
    }
    return 0;
}

int qrdm_factor_noalloc(double *A, int64_t m, int64_t n, int64_t lda, const qrdm_params *pin, double *tau_house,
                        int32_t *perm, int64_t *rank_dev, void *stream) {
    qrdm_params p;
    if (pin) p = *pin; else qrdm_default_params(&p);
    int rc = check_common(A, m, n, lda, &p);
    if (rc) return rc;
    rc = check_outputs(m, n, tau_house, perm);
    if (rc) return rc;
    if (!rank_dev) return -8;
    if (p.profile) return -5;  // timing events are for qrdm_factor_ex
    if (n > 32768 || m > 65536) return QRDM_ERR_UNSUPPORTED;
    hipStream_t s = (hipStream_t)stream;
    if (std::min(m, n) == 0) return trivial(perm, n, rank_dev, s);
    CallEnv env;
    env.L = make_layout(m, n, p.kmax);
    if (env.L.total > QRDM_NOALLOC_WS_MAX) return QRDM_ERR_SCRATCH;
    char *base = nullptr;
    rc = scratch_base(&base);
    if (rc) return rc;
    PollCtx pc;  // copy mode: nothing of it is allocated
    pc.copy = true;
    pc.ring = 1;
    pc.dev_snap = (uint64_t *)base;
    env.ws = base + QRDM_SCRATCH_SNAP_BYTES;
    env.pc = &pc;
    env.s = s;
    env.log = nullptr;
    env.log_cap = 0;
    env.nlog = nullptr;
    env.rank_dev = rank_dev;
    ProfRun prof;
    Snapshot fin;
    rc = qrdm_run(A, m, n, lda, p, tau_house, perm, env, prof, &fin);
    if (rc) return rc;
    return snapshot_code(fin);
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
    std::lock_guard<std::mutex> lk(g_ws_mu);
    Layout Ly = make_layout(m, n, kmax);
    rc = ensure_workspace(Ly.total);
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
    a.fbeps = (double)n * kEps64;
    a.tol3z = sqrt(kEps64);
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
    QrdmCtl c0;
    memset(&c0, 0, sizeof c0);
    c0.ns = ns;
    c0.rank = 0;        // stopping test already decided: not applied here
    c0.nblocks = 1;     // keep amax as given
    c0.amax = 2.2250738585072014e-308;  // the switch to scalar pivoting never fires for a non-zero trailing block
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
    if (nb < 1 || nb > kQp3NbMax) return -6;
    const int64_t pmin = std::min(m, n);
    if (pmin > 0 && !tau_house) return -7;
    if (n > 0 && !perm) return -8;
    if (!rank) return -9;
    if (m > 65536) return QRDM_ERR_UNSUPPORTED;
    hipStream_t s = (hipStream_t)stream;
    if (stats) memset(stats, 0, sizeof *stats);
    if (pmin == 0) {
        rc = trivial(perm, n, nullptr, s);
        if (rc) return rc;
        HIP_TRY(hipStreamSynchronize(s));
        *rank = 0;
        if (stats) stats->qp3_start = -1;
        return 0;
    }
    std::lock_guard<std::mutex> lk(g_ws_mu);
    Layout L = make_layout(m, n, 1);
    rc = ensure_workspace(L.total);
    if (rc) return rc;
    PollGuard pg;
    pg.s = s;
    rc = poll_acquire(p.poll_lag + 2, &pg.pc);
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
    a.eps1 = (p.eps1_scale > 0.0 ? p.eps1_scale : (double)n) * kEps64;
    a.fbeps = (double)n * kEps64;
    a.tol3z = sqrt(kEps64);
    a.vn1 = (double *)(ws + L.vn1);
    a.vn2 = (double *)(ws + L.vn2);
    a.perm = perm;
    a.tau_house = tau_house;
    a.gbar = (uint32_t *)(ws + L.gbar);
    a.ctl = (QrdmCtl *)(ws + L.ctl);
    HIP_TRY(launch_ws_reset(a.ctl, (int32_t *)(ws + L.flag), n, s));
    HIP_TRY(launch_colnorm(A, m, n, lda, a.vn1, a.vn2, a.ctl, s));
    HIP_TRY(launch_init(a, s));
    ProfRun prof;
    prof.on = p.profile != 0;
    if (prof.on) {
        if (grow_events(pg.pc->prof_ev, 3) != 0) return QRDM_ERR_NOMEM;
        HIP_TRY(hipEventRecord(pg.pc->prof_ev[0], s));
    }
    Snapshot fin;
    rc = run_qp3(a, ws, L, nb, p.poll_lag, 0, s, *pg.pc, prof, &fin);
    if (rc) return rc;
    if (prof.on) HIP_TRY(hipEventRecord(pg.pc->prof_ev[1], s));
    HIP_TRY(hipStreamSynchronize(s));
    QrdmCtl cf;
    HIP_TRY(hipMemcpy(&cf, a.ctl, sizeof cf, hipMemcpyDeviceToHost));
    if (cf.nonfinite) return QRDM_ERR_NONFINITE;
    if (cf.error) return QRDM_ERR_HIP + (int)hipErrorLaunchTimeOut;
    *rank = cf.rank >= 0 ? cf.rank : cf.ns;
    if (stats) {
        stats->nblocks = cf.nblocks;
        stats->nrecompute = cf.nrecompute;
        stats->ncols_factored = cf.ns;
        stats->qp3_start = 0;
        if (prof.on) {
            float ms = 0.f;
            if (hipEventElapsedTime(&ms, pg.pc->prof_ev[0], pg.pc->prof_ev[1]) == hipSuccess)
                stats->qp3_ms = stats->total_ms = ms;
            stats->nqp3_launch = prof.qp_launches;
            stats->nqp3_tail = prof.tail_launches;
            double q = 0.0;
            for (int64_t i = 0; i < prof.qp_launches; ++i) {
                float x = 0.f;
                if (hipEventElapsedTime(&x, pg.pc->qp_ev[2 * i], pg.pc->qp_ev[2 * i + 1]) == hipSuccess) q += x;
            }
            stats->qp3_run_ms = q;
            stats->qp3_bytes = prof.qp_launches > 0 ? qp3_bytes(m, n, cf.qp3_start, cf.ns) : 0.0;
        }
    }
    return 0;
}

int qrp_factor(double *A, int64_t m, int64_t n, int64_t lda, double *tau_house, int32_t *perm, int64_t *rank,
               void *stream) {
    return qrp_factor_ex(A, m, n, lda, nullptr, 32, tau_house, perm, rank, nullptr, stream);
}

}  // extern "C"
