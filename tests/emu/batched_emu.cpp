// CPU run of the batched QRDM kernel (k_batched.hip) under the host emulation
// of hip/hip_runtime.h in this directory: each workgroup of the persistent
// launch runs as NT host threads, one workgroup after another.
//
//   batched_emu <in> <out>
//
// in:  int32 count, variant, grid; double tau, delta; int32 kmax, stop_rule;
//      double eps1_scale; int32 certified; then per matrix int32 m, n and the
//      m x n column-major float64 data; optionally int32 mode (1: per-matrix
//      parameters; 2: per-matrix parameters and the online check with the
//      re-run of the failures, as qrdm_batch_factor_checked), double band, and
//      per matrix double tau, delta, int32 kmax, pad (qrdm_batch_params).
// out: per matrix int64 rank, int32 status, float64 tau_house[min(m, n)],
//      int32 perm[n], float64 A[m x n] (the factored matrix), int64 info[4],
//      int32 ok (mode 2; -1 otherwise).
// Variants 0-2 are the library's (256 threads); 3 is the 512-thread form
// with one column tile per wavefront and register panels.
#include "hip/hip_runtime.h"

#include "k_batched.hip"

#include <stdio.h>
#include <stdlib.h>

#include <algorithm>
#include <numeric>
#include <thread>
#include <vector>

thread_local EmuIdx threadIdx, blockIdx;
EmuIdx blockDim, gridDim;
EmuWG *emu_wg;

template <int NT, int WC, int PN>
static void run_grid(const QbArgs &q, int grid) {
    for (int b = 0; b < grid; ++b) {
        EmuWG *wg = new EmuWG;
        pthread_barrier_init(&wg->all, nullptr, NT);
        for (int w = 0; w < NT / 64; ++w) pthread_barrier_init(&wg->wave[w], nullptr, 64);
        emu_wg = wg;
        blockDim = EmuIdx{(unsigned)NT, 1, 1};
        gridDim = EmuIdx{(unsigned)grid, 1, 1};
        std::vector<std::thread> th;
        th.reserve(NT);
        for (int t = 0; t < NT; ++t)
            th.emplace_back([t, b, &q] {
                threadIdx = EmuIdx{(unsigned)t, 0, 0};
                blockIdx = EmuIdx{(unsigned)b, 0, 0};
                k_qrdm_batched<NT, WC, PN>(q);
            });
        for (auto &x : th) x.join();
        for (int w = 0; w < NT / 64; ++w) pthread_barrier_destroy(&wg->wave[w]);
        pthread_barrier_destroy(&wg->all);
        delete wg;
    }
}

template <typename T>
static void rd(FILE *f, T *p, size_t n) {
    if (fread(p, sizeof(T), n, f) != n) {
        fprintf(stderr, "short input\n");
        exit(2);
    }
}

int main(int argc, char **argv) {
    if (argc != 3) {
        fprintf(stderr, "usage: %s in out\n", argv[0]);
        return 2;
    }
    FILE *f = fopen(argv[1], "rb");
    if (!f) return 2;
    int32_t count, variant, grid, kmax, stop_rule, certified;
    double tau, delta, eps1_scale;
    rd(f, &count, 1);
    rd(f, &variant, 1);
    rd(f, &grid, 1);
    rd(f, &tau, 1);
    rd(f, &delta, 1);
    rd(f, &kmax, 1);
    rd(f, &stop_rule, 1);
    rd(f, &eps1_scale, 1);
    rd(f, &certified, 1);
    std::vector<int32_t> m(count), n(count), lda(count), order(count), status(count, -7);
    std::vector<std::vector<double>> A(count), th(count);
    std::vector<std::vector<int32_t>> perm(count);
    std::vector<double *> Ap(count), tp(count);
    std::vector<int32_t *> pp(count);
    std::vector<int64_t> rank(count, -7), info(4 * (size_t)count, 0);
    for (int i = 0; i < count; ++i) {
        rd(f, &m[i], 1);
        rd(f, &n[i], 1);
        lda[i] = m[i];
        A[i].resize((size_t)m[i] * n[i]);
        rd(f, A[i].data(), A[i].size());
        th[i].assign(std::min(m[i], n[i]), -7.0);
        perm[i].assign(n[i], -7);
        Ap[i] = A[i].data();
        tp[i] = th[i].data();
        pp[i] = perm[i].data();
    }
    int32_t mode = 0;
    double band = 0.0;
    std::vector<qrdm_batch_params> pmv;
    if (fread(&mode, sizeof mode, 1, f) == 1 && mode > 0) {
        rd(f, &band, 1);
        pmv.resize(count);
        rd(f, pmv.data(), (size_t)count);
    }
    fclose(f);
    std::vector<std::vector<double>> P(A);  // pristine copies
    std::vector<const double *> Pp(count);
    for (int i = 0; i < count; ++i) Pp[i] = P[i].data();
    std::vector<int32_t> ok(count, -1);
    // longest first, as the library orders a size class
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](int x, int y) {
        const double fx = (double)m[x] * n[x] * std::min(m[x], n[x]), fy = (double)m[y] * n[y] * std::min(m[y], n[y]);
        return fx > fy;
    });
    uint32_t counters[2] = {0, 0};
    QbArgs q;
    memset(&q, 0, sizeof q);
    q.A = Ap.data();
    q.m = m.data();
    q.n = n.data();
    q.lda = lda.data();
    q.tau_house = tp.data();
    q.perm = pp.data();
    q.rank = rank.data();
    q.status = status.data();
    q.info = info.data();
    q.pm = mode > 0 ? pmv.data() : nullptr;
    q.pristine = mode == 2 ? Pp.data() : nullptr;
    q.band = band;
    q.ok = mode == 2 ? ok.data() : nullptr;
    q.order = order.data();
    q.count = count;
    q.counters = counters;
    q.tau = tau;
    q.delta = delta;
    q.kmax = kmax;
    q.stop_rule = stop_rule;
    q.eps1_scale = eps1_scale;
    q.certified = certified;
    switch (variant) {
        case 0: run_grid<256, 1, 1>(q, grid); break;
        case 1: run_grid<256, 2, 1>(q, grid); break;
        case 2: run_grid<256, 1, 0>(q, grid); break;
        case 3: run_grid<512, 1, 1>(q, grid); break;
        default: fprintf(stderr, "variant\n"); return 2;
    }
    if (counters[0] != 0 || counters[1] != 0) {
        fprintf(stderr, "queue counters not reset\n");
        return 3;
    }
    FILE *g = fopen(argv[2], "wb");
    if (!g) return 2;
    for (int i = 0; i < count; ++i) {
        fwrite(&rank[i], 8, 1, g);
        fwrite(&status[i], 4, 1, g);
        fwrite(th[i].data(), 8, th[i].size(), g);
        fwrite(perm[i].data(), 4, perm[i].size(), g);
        fwrite(A[i].data(), 8, A[i].size(), g);
        fwrite(&info[4 * (size_t)i], 8, 4, g);
        fwrite(&ok[i], 4, 1, g);
    }
    fclose(g);
    return 0;
}
