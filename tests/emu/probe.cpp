// Checks of the host emulation itself (tests/emu/hip/hip_runtime.h):
//   probe fenced   one thread writes LDS, a barrier, every thread reads: no race
//   probe racy     the same without the barrier: ThreadSanitizer must report it
//   probe lanes    __shfl_xor, __shfl, __ballot and the 16x16x4 FP64 MFMA
//                  against their definitions (prints "lanes ok")
#include "hip/hip_runtime.h"

#include <stdio.h>
#include <string.h>

#include <thread>
#include <vector>

thread_local EmuIdx threadIdx, blockIdx;
EmuIdx blockDim, gridDim;
EmuWG *emu_wg;

static int g_bad = 0;

__global__ void k_handoff(int fenced, double *out) {
    __shared__ double x;
    if (threadIdx.x == 0) x = 42.0;
    if (fenced) __syncthreads();
    out[threadIdx.x] = x;
}

typedef double dbl4 __attribute__((ext_vector_type(4)));

__global__ void k_lanes(double *mfa, double *mfb, double *mfd) {
    const int l = threadIdx.x % 64;
    if (__shfl_xor(l, 5, 64) != (l ^ 5)) __atomic_fetch_add(&g_bad, 1, __ATOMIC_SEQ_CST);
    if (__shfl(l, 17, 64) != 17) __atomic_fetch_add(&g_bad, 1, __ATOMIC_SEQ_CST);
    if (__shfl(l, 3, 16) != (l & ~15) + 3) __atomic_fetch_add(&g_bad, 1, __ATOMIC_SEQ_CST);
    const unsigned long long b = __ballot(l % 3 == 0);
    if (((b >> l) & 1ull) != (l % 3 == 0 ? 1ull : 0ull)) __atomic_fetch_add(&g_bad, 1, __ATOMIC_SEQ_CST);
    // A is 16 x 4 (A[i][k] = mfa[i * 4 + k]) from lane i + 16k, B is 4 x 16 from lane j + 16k
    const int i = l % 16, k = l / 16;
    dbl4 c = {1.0, 2.0, 3.0, 4.0};
    const dbl4 d = __builtin_amdgcn_mfma_f64_16x16x4f64(mfa[i * 4 + k], mfb[k * 16 + i], c, 0, 0, 0);
    for (int v = 0; v < 4; ++v) mfd[(4 * v + l / 16) * 16 + l % 16] = d[v] - c[v];
}

template <typename F>
static void launch(int nt, F f) {
    EmuWG *wg = new EmuWG;
    pthread_barrier_init(&wg->all, nullptr, nt);
    for (int w = 0; w < nt / 64; ++w) pthread_barrier_init(&wg->wave[w], nullptr, 64);
    emu_wg = wg;
    blockDim = EmuIdx{(unsigned)nt, 1, 1};
    gridDim = EmuIdx{1, 1, 1};
    std::vector<std::thread> th;
    for (int t = 0; t < nt; ++t)
        th.emplace_back([t, &f] {
            threadIdx = EmuIdx{(unsigned)t, 0, 0};
            blockIdx = EmuIdx{0, 0, 0};
            f();
        });
    for (auto &x : th) x.join();
    for (int w = 0; w < nt / 64; ++w) pthread_barrier_destroy(&wg->wave[w]);
    pthread_barrier_destroy(&wg->all);
    delete wg;
}

int main(int argc, char **argv) {
    if (argc != 2) return 2;
    if (!strcmp(argv[1], "fenced") || !strcmp(argv[1], "racy")) {
        const int fenced = !strcmp(argv[1], "fenced");
        std::vector<double> out(128, 0.0);
        launch(128, [&] { k_handoff(fenced, out.data()); });
        return 0;
    }
    if (!strcmp(argv[1], "lanes")) {
        double a[64], b[64], d[256];
        for (int x = 0; x < 64; ++x) {
            a[x] = 1.0 + x;
            b[x] = 0.5 - 0.25 * x;
        }
        launch(64, [&] { k_lanes(a, b, d); });
        for (int r = 0; r < 16; ++r)
            for (int c = 0; c < 16; ++c) {
                double s = 0.0;
                for (int k = 0; k < 4; ++k) s += a[r * 4 + k] * b[k * 16 + c];
                if (d[r * 16 + c] != s) ++g_bad;
            }
        if (g_bad) {
            printf("lanes bad %d\n", g_bad);
            return 1;
        }
        printf("lanes ok\n");
        return 0;
    }
    return 2;
}
