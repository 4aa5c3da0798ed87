// Host emulation of the HIP device interface that the batched kernel
// (k_batched.hip) and the internal header use, for the CPU test of that
// kernel.  One host thread runs each GPU thread of a workgroup; __syncthreads
// is a pthread barrier over the workgroup, and every cross-lane operation
// (shuffles, ballot, the 16x16x4 FP64 MFMA) goes through a per-wavefront
// exchange buffer between two pthread barriers over the wavefront's 64
// threads.  Only these barriers order one thread's memory accesses before
// another's, so ThreadSanitizer reports every hand-off (LDS or global) that
// the kernel does not fence with a barrier or a cross-lane operation.
// Workgroups run one after another: __shared__ variables are function statics.
#pragma once
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <string.h>

#define __global__
#define __device__
#define __host__
#define __forceinline__ inline
#define __launch_bounds__(...)
#define __shared__ static
#define __HIP_MEMORY_SCOPE_AGENT 0

typedef int hipError_t;
enum { hipSuccess = 0, hipErrorInvalidValue = 1 };
typedef void *hipStream_t;
typedef void *hipEvent_t;
struct dim3 {
    unsigned x, y, z;
    dim3(unsigned a = 1, unsigned b = 1, unsigned c = 1) : x(a), y(b), z(c) {}
};
struct EmuIdx {
    unsigned x, y, z;
};
extern thread_local EmuIdx threadIdx, blockIdx;
extern EmuIdx blockDim, gridDim;

// the workgroup being run: its barrier, the wavefront barriers and exchange buffers
struct EmuWG {
    pthread_barrier_t all;
    pthread_barrier_t wave[16];
    uint64_t xa[16][64], xb[16][64];
};
extern EmuWG *emu_wg;

inline void __syncthreads() { pthread_barrier_wait(&emu_wg->all); }
inline void emu_wave_sync() { pthread_barrier_wait(&emu_wg->wave[threadIdx.x / 64]); }

template <typename T>
inline T emu_lane_read(T v, int src) {
    static_assert(sizeof(T) <= 8, "64-bit lanes");
    const int w = threadIdx.x / 64, l = threadIdx.x % 64;
    uint64_t b = 0;
    memcpy(&b, &v, sizeof(T));
    emu_wg->xa[w][l] = b;
    emu_wave_sync();
    const uint64_t r = emu_wg->xa[w][src];
    emu_wave_sync();
    T out;
    memcpy(&out, &r, sizeof(T));
    return out;
}
template <typename T>
inline T __shfl_xor(T v, int mask, int width = 64) {
    const int l = threadIdx.x % 64;
    return emu_lane_read(v, (l & ~(width - 1)) | ((l ^ mask) & (width - 1)));
}
template <typename T>
inline T __shfl(T v, int src, int width = 64) {
    const int l = threadIdx.x % 64;
    return emu_lane_read(v, (l & ~(width - 1)) + (src & (width - 1)));
}
inline unsigned long long __ballot(int pred) {
    const int w = threadIdx.x / 64, l = threadIdx.x % 64;
    emu_wg->xa[w][l] = pred ? 1 : 0;
    emu_wave_sync();
    unsigned long long m = 0;
    for (int i = 0; i < 64; ++i) m |= (unsigned long long)emu_wg->xa[w][i] << i;
    emu_wave_sync();
    return m;
}
inline int __any(int pred) { return __ballot(pred) != 0; }
inline int __popcll(unsigned long long x) { return __builtin_popcountll(x); }

// D = A B + C for 16 x 16 x 4: A[i][k] from lane i + 16k, B[k][j] from lane
// j + 16k; register v of a lane returns D[4v + lane/16][lane%16]
typedef double emu_dbl4 __attribute__((ext_vector_type(4)));
inline emu_dbl4 emu_mfma_f64_16x16x4(double a, double b, emu_dbl4 c, int, int, int) {
    const int w = threadIdx.x / 64, l = threadIdx.x % 64;
    memcpy(&emu_wg->xa[w][l], &a, 8);
    memcpy(&emu_wg->xb[w][l], &b, 8);
    emu_wave_sync();
    emu_dbl4 d;
    for (int v = 0; v < 4; ++v) {
        const int row = 4 * v + l / 16, col = l % 16;
        double s = c[v];
        for (int k = 0; k < 4; ++k) {
            double x, y;
            memcpy(&x, &emu_wg->xa[w][row + 16 * k], 8);
            memcpy(&y, &emu_wg->xb[w][col + 16 * k], 8);
            s += x * y;
        }
        d[v] = s;
    }
    emu_wave_sync();
    return d;
}
#define __builtin_amdgcn_mfma_f64_16x16x4f64 emu_mfma_f64_16x16x4
// a scheduling barrier over the wavefront: here a barrier of its 64 threads
#define __builtin_amdgcn_wave_barrier() emu_wave_sync()

// memory operations: host atomics (ThreadSanitizer sees them), waits are no-ops
template <typename T>
inline T atomicAdd(T *p, T v) { return __atomic_fetch_add(p, v, __ATOMIC_SEQ_CST); }
template <typename T>
inline T atomicExch(T *p, T v) { return __atomic_exchange_n(p, v, __ATOMIC_SEQ_CST); }
template <typename T>
inline T atomicOr(T *p, T v) { return __atomic_fetch_or(p, v, __ATOMIC_SEQ_CST); }
#define __hip_atomic_fetch_add(p, v, order, scope) __atomic_fetch_add((p), (v), (order))
#define __hip_atomic_load(p, order, scope) __atomic_load_n((p), (order))
#define __hip_atomic_store(p, v, order, scope) __atomic_store_n((p), (v), (order))
#define __builtin_amdgcn_s_waitcnt(x) ((void)0)
#define __builtin_amdgcn_s_sleep(x) ((void)0)
inline unsigned long long wall_clock64() { return 0; }
inline long long __double_as_longlong(double x) {
    long long r;
    memcpy(&r, &x, 8);
    return r;
}
inline double __longlong_as_double(long long x) {
    double r;
    memcpy(&r, &x, 8);
    return r;
}
// lane swaps of the other kernels (never called by the batched kernel)
struct EmuPair {
    uint32_t r[2];
    uint32_t operator[](int i) const { return r[i]; }
};
inline EmuPair emu_permlane_swap(uint32_t a, uint32_t b, bool, bool) { return EmuPair{{a, b}}; }
#define __builtin_amdgcn_permlane32_swap emu_permlane_swap
#define __builtin_amdgcn_permlane16_swap emu_permlane_swap
inline int emu_mov_dpp(int v, int, int, int, bool) { return v; }
#define __builtin_amdgcn_mov_dpp emu_mov_dpp

// host API used by the launchers of the included sources
#define hipLaunchKernelGGL(...) ((void)0)
inline hipError_t hipGetLastError() { return hipSuccess; }
inline hipError_t hipOccupancyMaxActiveBlocksPerMultiprocessor(int *n, const void *, int, size_t) {
    *n = 1;
    return hipSuccess;
}
