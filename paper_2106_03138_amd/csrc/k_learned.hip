// Learned choice of (tau, delta, k_DM) per matrix for the batched path.
//
// The paper picks the parameters by a grid study (Section 5) and judges the
// result with the factor-10 rule on d_i / sigma_i; here a small multilayer
// perceptron predicts them from cheap per-matrix features, and an online
// condition estimate decides whether a prediction is kept or the matrix is
// factored again with the defaults.
//
//   k_features     per matrix (one workgroup): order statistics of
//                  log10(||a_j|| / max ||a_j||) (exact ranks), log2 m, log2 n,
//                  n/m, and statistics of |theta_ij| (Algorithm 1's cosines)
//                  over a fixed sample of at most 64 columns
//   k_mlp_forward  16 -> 64 -> 64 -> 3 (tanh, tanh, linear), FP32, one
//                  workgroup of 64 threads per sample
//   k_mlp_delta    per-sample back-propagated errors of the squared loss
//   k_mlp_grad     each gradient entry as a fixed-order sum over the samples
//   k_adam         Adam update (Kingma & Ba)
//   k_predict      MLP outputs -> nearest grid values (tau, delta) and k_DM
//   k_ice_check    incremental condition estimate of sigma_min(R11) per matrix;
//                  accept iff it is >= band * min_{i<rank} |r_ii|
#include <float.h>

#include "qrdm_learned.h"

#define LF_NT 256
#define LF_SAMPLE 64
#define LF_LOG_FLOOR (-30.0)
typedef double lf_dbl4 __attribute__((ext_vector_type(4)));
#define LF_PSORT 2048  // power of two >= LF_SAMPLE (LF_SAMPLE - 1) / 2, the cosines' sort
static_assert(LF_PSORT >= LF_SAMPLE * (LF_SAMPLE - 1) / 2, "sort buffer");

// ---------------------------------------------------------------- features
__global__ void __launch_bounds__(LF_NT) k_features(LfArgs q, double *feat) {
    __shared__ double su[QB_NMAX];
    __shared__ double sl[QB_NMAX];
    __shared__ double sc[LF_SAMPLE * 65];  // staged sampled columns, 64 rows at a time
    __shared__ double sg[LF_SAMPLE * LF_SAMPLE];
    __shared__ double sth[LF_PSORT];  // the sampled cosines, then sorted
    __shared__ double sred[LF_NT / 64];
    __shared__ int scnt[LF_NT / 64];
    const int mi = blockIdx.x;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    constexpr int NW = LF_NT / 64;
    const int m = q.m[mi], n = q.n[mi], lda = q.lda[mi];
    const double *A = q.A[mi];
    double *f = feat + (int64_t)mi * LF_NFEAT;
    if (tid < LF_NFEAT) f[tid] = 0.0;
    __syncthreads();
    if (tid == 0) {
        f[9] = log2((double)(m > 1 ? m : 1));
        f[10] = log2((double)(n > 1 ? n : 1));
        f[11] = (double)n / (double)(m > 1 ? m : 1);
    }
    if (n == 0 || m == 0) return;
    // column norms (fixed-order wavefront sums), four columns of a wavefront at
    // a time with every load issued before the sums (m <= QB_NMAX = 8 x 64 rows)
    for (int c0 = 4 * wv; c0 < n; c0 += 4 * NW) {
        double x[4][QB_NMAX / 64];
#pragma unroll
        for (int cb = 0; cb < 4; ++cb)
#pragma unroll
            for (int u = 0; u < QB_NMAX / 64; ++u) {
                const int c = c0 + cb, r = lane + 64 * u;
                x[cb][u] = (c < n && r < m) ? A[(int64_t)c * lda + r] : 0.0;
            }
#pragma unroll
        for (int cb = 0; cb < 4; ++cb) {
            double s = 0.0;
#pragma unroll
            for (int u = 0; u < QB_NMAX / 64; ++u)
                if (lane + 64 * u < m) s += x[cb][u] * x[cb][u];
            s = wave_sum(s);
            if (lane == 0 && c0 + cb < n) su[c0 + cb] = sqrt(s);
        }
    }
    __syncthreads();
    double um = 0.0;
    for (int c = tid; c < n; c += LF_NT) um = su[c] > um ? su[c] : um;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        const double ou = __shfl_xor(um, o, 64);
        um = ou > um ? ou : um;
    }
    if (lane == 0) sred[wv] = um;
    __syncthreads();
    double umax = 0.0;
    for (int i = 0; i < NW; ++i) umax = sred[i] > umax ? sred[i] : umax;
    if (umax == 0.0) return;
    for (int c = tid; c < n; c += LF_NT) {
        double v = LF_LOG_FLOOR;
        if (su[c] > 0.0) {
            v = log10(su[c] / umax);
            v = v > LF_LOG_FLOOR ? v : LF_LOG_FLOOR;
        }
        sl[c] = v;
    }
    __syncthreads();
    // order statistics: index floor(q (n - 1)) of the ascending order, ranks counted exactly
    for (int c = tid; c < n; c += LF_NT) {
        const double v = sl[c];
        int rk = 0;
        for (int o = 0; o < n; ++o) {
            const double w = sl[o];
            rk += (w < v || (w == v && o < c)) ? 1 : 0;
        }
        for (int k = 0; k < 9; ++k) {
            const double qq = (double)(k + 1) / 10.0;
            if (rk == (int)floor(qq * (double)(n - 1))) f[k] = v;
        }
    }
    // Gram of the sampled columns floor(k n / s) on FP64 MFMA (16x16x4), the
    // rows staged in LDS 64 at a time: wavefront w takes the upper 16 x 16 tiles
    // w, w + 4, ... of the (at most) 4 x 4 grid; in a tile, lane (i, kk) holds
    // the A operand X[16 bi + i][r + kk] and the B operand X[16 bj + i][r + kk]
    const int s = n < LF_SAMPLE ? n : LF_SAMPLE;
    const int nt = (s + 15) >> 4, ntile = nt * (nt + 1) / 2;
    const int ti = lane & 15, kk = lane >> 4;
    constexpr int TPW = (LF_SAMPLE / 16 * (LF_SAMPLE / 16 + 1) / 2 + NW - 1) / NW;  // tiles per wavefront
    lf_dbl4 acc[TPW];
#pragma unroll
    for (int u = 0; u < TPW; ++u) acc[u] = lf_dbl4{0.0, 0.0, 0.0, 0.0};
    auto tile_of = [&](int tile, int &bi, int &bj) {
        bi = 0;
        int rem = tile;
        while (rem >= nt - bi) { rem -= nt - bi; ++bi; }
        bj = bi + rem;
    };
    for (int r0 = 0; r0 < m; r0 += 64) {
        __syncthreads();
        {  // every load of the chunk issued before the stores
            double xv[64 * LF_SAMPLE / LF_NT];
#pragma unroll
            for (int u = 0; u < 64 * LF_SAMPLE / LF_NT; ++u) {
                const int e = tid + LF_NT * u, k = e >> 6, r = e & 63;
                const int col = (int)(((int64_t)k * n) / (s > 0 ? s : 1));
                xv[u] = (k < s && r0 + r < m) ? A[(int64_t)col * lda + r0 + r] : 0.0;
            }
#pragma unroll
            for (int u = 0; u < 64 * LF_SAMPLE / LF_NT; ++u) {
                const int e = tid + LF_NT * u;
                // columns past s as zeros too, so that a tile's padding stays finite
                sc[(e >> 6) * 65 + (e & 63)] = (e >> 6) < s ? xv[u] : 0.0;
            }
        }
        __syncthreads();
#pragma unroll
        for (int u = 0; u < TPW; ++u) {
            const int tile = wv + NW * u;
            if (tile < ntile) {
                int bi, bj;
                tile_of(tile, bi, bj);
#pragma unroll
                for (int k = 0; k < 64; k += 4) {
                    const double av = sc[(16 * bi + ti) * 65 + k + kk];
                    const double bv = sc[(16 * bj + ti) * 65 + k + kk];
                    acc[u] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, acc[u], 0, 0, 0);
                }
            }
        }
    }
    // register v of a lane holds G[16 bi + 4 v + kk][16 bj + ti]; a diagonal
    // tile holds both (row, cc) and (cc, row): each is stored once
#pragma unroll
    for (int u = 0; u < TPW; ++u) {
        const int tile = wv + NW * u;
        if (tile < ntile) {
            int bi, bj;
            tile_of(tile, bi, bj);
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int row = 16 * bi + 4 * v + kk, cc = 16 * bj + ti;
                if (row < s && cc < s && row <= cc) {
                    sg[row * LF_SAMPLE + cc] = acc[u][v];
                    if (row < cc) sg[cc * LF_SAMPLE + row] = acc[u][v];
                }
            }
        }
    }
    __syncthreads();
    const int P = s * (s - 1) / 2;
    if (P == 0) return;
    for (int e = tid; e < P; e += LF_NT) {
        int i = 0, rem = e;
        while (rem >= s - 1 - i) { rem -= s - 1 - i; ++i; }
        const int j = i + 1 + rem;
        const double di = sqrt(sg[i * LF_SAMPLE + i]), dj = sqrt(sg[j * LF_SAMPLE + j]);
        sth[e] = (di > 0.0 && dj > 0.0) ? fabs(sg[i * LF_SAMPLE + j] / (di * dj)) : 0.0;
    }
    __syncthreads();
    // mean, max, fraction above 0.5, and the order statistic floor(0.95 (P - 1))
    double sum = 0.0, mx = 0.0;
    int over = 0;
    for (int e = tid; e < P; e += LF_NT) {
        const double v = sth[e];
        sum += v;
        mx = v > mx ? v : mx;
        over += v > 0.5 ? 1 : 0;
    }
    sum = wave_sum(sum);
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        const double om = __shfl_xor(mx, o, 64);
        mx = om > mx ? om : mx;
        over += __shfl_xor(over, o, 64);
    }
    __syncthreads();
    if (lane == 0) {
        sred[wv] = sum;
        scnt[wv] = over;
    }
    __syncthreads();
    if (tid == 0) {
        double ts = 0.0;
        int tc = 0;
        for (int i = 0; i < NW; ++i) {
            ts += sred[i];
            tc += scnt[i];
        }
        f[12] = ts / (double)P;
        f[15] = (double)tc / (double)P;
    }
    __syncthreads();
    if (lane == 0) sred[wv] = mx;
    __syncthreads();
    if (tid == 0) {
        double tm = 0.0;
        for (int i = 0; i < NW; ++i) tm = sred[i] > tm ? sred[i] : tm;
        f[14] = tm;
    }
    // the order statistic: a bitonic sort of the P cosines in LDS (padded with
    // DBL_MAX to the next power of two), then the entry at floor(0.95 (P - 1))
    const int want = (int)floor(0.95 * (double)(P - 1));
    int ns = 1;
    while (ns < P) ns <<= 1;
    for (int i = P + tid; i < ns; i += LF_NT) sth[i] = DBL_MAX;
    __syncthreads();
    for (int k = 2; k <= ns; k <<= 1)
        for (int j = k >> 1; j > 0; j >>= 1) {
            for (int i = tid; i < ns; i += LF_NT) {
                const int l = i ^ j;
                if (l > i) {
                    const double x = sth[i], y = sth[l];
                    if ((x > y) == ((i & k) == 0)) {
                        sth[i] = y;
                        sth[l] = x;
                    }
                }
            }
            __syncthreads();
        }
    if (tid == 0) f[13] = sth[want];
}

// ---------------------------------------------------------------- MLP
// Parameter layout: W1 [64][16], b1 [64], W2 [64][64], b2 [64], W3 [3][64], b3 [3].
#define OFF_W1 0
#define OFF_B1 (OFF_W1 + LF_NH * LF_NFEAT)
#define OFF_W2 (OFF_B1 + LF_NH)
#define OFF_B2 (OFF_W2 + LF_NH * LF_NH)
#define OFF_W3 (OFF_B2 + LF_NH)
#define OFF_B3 (OFF_W3 + LF_NOUT * LF_NH)

// x = (feature - mean) * inv_std when norm is given (norm[0..16) mean, norm[16..32) inv_std)
__global__ void __launch_bounds__(LF_NH) k_mlp_forward(const float *__restrict__ P, const float *__restrict__ norm,
                                                       const double *__restrict__ feat, int B, float *H1, float *H2,
                                                       float *Y) {
    __shared__ float sx[LF_NFEAT];
    __shared__ float sh1[LF_NH];
    __shared__ float sh2[LF_NH];
    const int b = blockIdx.x, t = threadIdx.x;
    if (b >= B) return;
    if (t < LF_NFEAT) {
        float x = (float)feat[(int64_t)b * LF_NFEAT + t];
        if (norm) x = (x - norm[t]) * norm[LF_NFEAT + t];
        sx[t] = x;
    }
    __syncthreads();
    float z = P[OFF_B1 + t];
    for (int k = 0; k < LF_NFEAT; ++k) z += P[OFF_W1 + t * LF_NFEAT + k] * sx[k];
    const float h1 = tanhf(z);
    sh1[t] = h1;
    __syncthreads();
    z = P[OFF_B2 + t];
    for (int k = 0; k < LF_NH; ++k) z += P[OFF_W2 + t * LF_NH + k] * sh1[k];
    const float h2 = tanhf(z);
    sh2[t] = h2;
    if (H1) H1[(int64_t)b * LF_NH + t] = h1;
    if (H2) H2[(int64_t)b * LF_NH + t] = h2;
    __syncthreads();
    if (t < LF_NOUT) {
        float y = P[OFF_B3 + t];
        for (int k = 0; k < LF_NH; ++k) y += P[OFF_W3 + t * LF_NH + k] * sh2[k];
        Y[(int64_t)b * LF_NOUT + t] = y;
    }
}

// Per sample: dy = (y - target) / B, dz2 = (W3^T dy) (1 - h2^2), dz1 = (W2^T dz2) (1 - h1^2);
// D[b] = [dy (3) | dz2 (64) | dz1 (64)]; sqerr[b] = sum_o (y - target)^2.
__global__ void __launch_bounds__(LF_NH) k_mlp_delta(const float *__restrict__ P, const float *__restrict__ H1,
                                                     const float *__restrict__ H2, const float *__restrict__ Y,
                                                     const float *__restrict__ T, int B, float *D, float *sqerr) {
    __shared__ float sdy[LF_NOUT];
    __shared__ float sdz2[LF_NH];
    const int b = blockIdx.x, t = threadIdx.x;
    if (b >= B) return;
    float *Db = D + (int64_t)b * LF_NDELTA;
    if (t < LF_NOUT) {
        const float e = Y[(int64_t)b * LF_NOUT + t] - T[(int64_t)b * LF_NOUT + t];
        sdy[t] = e / (float)B;
        Db[t] = e / (float)B;
    }
    if (t == 0 && sqerr) {
        float s = 0.f;
        for (int o = 0; o < LF_NOUT; ++o) {
            const float e = Y[(int64_t)b * LF_NOUT + o] - T[(int64_t)b * LF_NOUT + o];
            s += e * e;
        }
        sqerr[b] = s;
    }
    __syncthreads();
    float d2 = 0.f;
    for (int o = 0; o < LF_NOUT; ++o) d2 += P[OFF_W3 + o * LF_NH + t] * sdy[o];
    const float h2 = H2[(int64_t)b * LF_NH + t];
    d2 *= 1.f - h2 * h2;
    sdz2[t] = d2;
    Db[LF_NOUT + t] = d2;
    __syncthreads();
    float d1 = 0.f;
    for (int k = 0; k < LF_NH; ++k) d1 += P[OFF_W2 + k * LF_NH + t] * sdz2[k];
    const float h1 = H1[(int64_t)b * LF_NH + t];
    d1 *= 1.f - h1 * h1;
    Db[LF_NOUT + LF_NH + t] = d1;
}

// One thread per parameter: the sum over samples of (delta x activation), in sample order.
__global__ void k_mlp_grad(const float *__restrict__ norm, const double *__restrict__ feat,
                           const float *__restrict__ H1, const float *__restrict__ H2, const float *__restrict__ D,
                           int B, float *G) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= LF_NPARAM) return;
    float s = 0.f;
    if (p < OFF_B1) {  // W1[t][k]: dz1[t] x[k]
        const int t = p / LF_NFEAT, k = p % LF_NFEAT;
        for (int b = 0; b < B; ++b) {
            float x = (float)feat[(int64_t)b * LF_NFEAT + k];
            if (norm) x = (x - norm[k]) * norm[LF_NFEAT + k];
            s += D[(int64_t)b * LF_NDELTA + LF_NOUT + LF_NH + t] * x;
        }
    } else if (p < OFF_W2) {  // b1[t]
        const int t = p - OFF_B1;
        for (int b = 0; b < B; ++b) s += D[(int64_t)b * LF_NDELTA + LF_NOUT + LF_NH + t];
    } else if (p < OFF_B2) {  // W2[t][k]: dz2[t] h1[k]
        const int e = p - OFF_W2, t = e / LF_NH, k = e % LF_NH;
        for (int b = 0; b < B; ++b) s += D[(int64_t)b * LF_NDELTA + LF_NOUT + t] * H1[(int64_t)b * LF_NH + k];
    } else if (p < OFF_W3) {  // b2[t]
        const int t = p - OFF_B2;
        for (int b = 0; b < B; ++b) s += D[(int64_t)b * LF_NDELTA + LF_NOUT + t];
    } else if (p < OFF_B3) {  // W3[o][k]: dy[o] h2[k]
        const int e = p - OFF_W3, o = e / LF_NH, k = e % LF_NH;
        for (int b = 0; b < B; ++b) s += D[(int64_t)b * LF_NDELTA + o] * H2[(int64_t)b * LF_NH + k];
    } else {  // b3[o]
        const int o = p - OFF_B3;
        for (int b = 0; b < B; ++b) s += D[(int64_t)b * LF_NDELTA + o];
    }
    G[p] = s;
}

__global__ void k_adam(float *P, const float *__restrict__ G, float *M, float *V, int n, float lr, float b1, float b2,
                       float eps, float c1, float c2) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    const float g = G[p];
    const float mo = b1 * M[p] + (1.f - b1) * g;
    const float ve = b2 * V[p] + (1.f - b2) * g * g;
    M[p] = mo;
    V[p] = ve;
    // c1 = 1 - b1^t, c2 = 1 - b2^t (bias corrections)
    P[p] -= lr * (mo / c1) / (sqrtf(ve / c2) + eps);
}

// ---------------------------------------------------------------- predict
__device__ __forceinline__ double lf_nearest(double v, const double *grid, int k) {
    double best = grid[0];
    double bd = fabs(v - grid[0]);
    for (int i = 1; i < k; ++i) {
        const double d = fabs(v - grid[i]);
        if (d < bd) { bd = d; best = grid[i]; }
    }
    return best;
}

__global__ void k_predict(const float *__restrict__ Y, int B, qrdm_batch_params *out) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= B) return;
    const double taus[LF_NTAU] = LF_TAU_GRID;
    const double deltas[LF_NDELTA_GRID] = LF_DELTA_GRID;
    const double y0 = Y[(int64_t)b * LF_NOUT], y1 = Y[(int64_t)b * LF_NOUT + 1], y2 = Y[(int64_t)b * LF_NOUT + 2];
    qrdm_batch_params p;
    p.tau = lf_nearest(y0, taus, LF_NTAU);
    p.delta = lf_nearest(y1, deltas, LF_NDELTA_GRID);
    p.kmax = y2 >= 0.5 ? 64 : 32;
    p.pad = 0;
    out[b] = p;
}

// ---------------------------------------------------------------- ICE check
// One wavefront per matrix: qb_ice on the leading rank x rank block of R.
__global__ void __launch_bounds__(64) k_ice_check(LfArgs q, const int64_t *rank, double band, double *est_out,
                                                 int32_t *ok) {
    __shared__ double sx[QB_NMAX];
    const int mi = blockIdx.x, lane = threadIdx.x;
    const int m = q.m[mi], n = q.n[mi], lda = q.lda[mi];
    int64_t r = rank[mi];
    const int p = m < n ? m : n;
    if (r > p) r = p;
    if (r <= 0) {
        if (lane == 0) {
            if (est_out) est_out[mi] = 0.0;
            ok[mi] = 1;
        }
        return;
    }
    double dmin;
    const double est = qb_ice(q.A[mi], lda, (int)r, sx, &dmin);
    if (lane == 0) {
        if (est_out) est_out[mi] = est;
        ok[mi] = est >= band * dmin ? 1 : 0;
    }
}

// ---------------------------------------------------------------- launchers
hipError_t launch_features(const LfArgs &q, int batch, double *feat, hipStream_t s) {
    if (batch <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_features, dim3(batch), dim3(LF_NT), 0, s, q, feat);
    return hipGetLastError();
}

hipError_t launch_mlp_forward(const float *P, const float *norm, const double *feat, int B, float *H1, float *H2,
                              float *Y, hipStream_t s) {
    if (B <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_mlp_forward, dim3(B), dim3(LF_NH), 0, s, P, norm, feat, B, H1, H2, Y);
    return hipGetLastError();
}

hipError_t launch_mlp_backward(const float *P, const float *norm, const double *feat, const float *H1,
                               const float *H2, const float *Y, const float *T, int B, float *D, float *G,
                               float *sqerr, hipStream_t s) {
    if (B <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_mlp_delta, dim3(B), dim3(LF_NH), 0, s, P, H1, H2, Y, T, B, D, sqerr);
    hipLaunchKernelGGL(k_mlp_grad, dim3((LF_NPARAM + 255) / 256), dim3(256), 0, s, norm, feat, H1, H2, D, B, G);
    return hipGetLastError();
}

hipError_t launch_adam(float *P, const float *G, float *M, float *V, int t, float lr, float b1, float b2, float eps,
                       hipStream_t s) {
    const float c1 = 1.f - powf(b1, (float)t), c2 = 1.f - powf(b2, (float)t);
    hipLaunchKernelGGL(k_adam, dim3((LF_NPARAM + 255) / 256), dim3(256), 0, s, P, G, M, V, LF_NPARAM, lr, b1, b2,
                       eps, c1, c2);
    return hipGetLastError();
}

hipError_t launch_predict(const float *Y, int B, qrdm_batch_params *out, hipStream_t s) {
    if (B <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_predict, dim3((B + 255) / 256), dim3(256), 0, s, Y, B, out);
    return hipGetLastError();
}

hipError_t launch_ice_check(const LfArgs &q, int batch, const int64_t *rank, double band, double *est, int32_t *ok,
                            hipStream_t s) {
    if (batch <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_ice_check, dim3(batch), dim3(64), 0, s, q, rank, band, est, ok);
    return hipGetLastError();
}
