"""Oracle for the learned (tau, delta, k_DM) predictor: plain FP64 definitions.

TEST INFRASTRUCTURE ONLY (tests, the smoke check and the benchmark's CPU leg).
It shares no code with the GPU library.

The paper fixes (tau, delta, k_DM) by a grid study (Section 5) and reports
quality with the factor-10 rule on d_i / sigma_i (Section 5).  This module
defines what the GPU predictor computes, each item written out from its
definition:

  features(a)     16 numbers per matrix: nine order statistics of
                  log10(||a_j|| / max ||a_j||), log2 m, log2 n, n/m, and the
                  mean, 95th order statistic, maximum and fraction above 0.5 of
                  |theta_ij| over a fixed sample of at most 64 columns
                  (theta as in Algorithm 1: G_ij / sqrt(G_ii G_jj)).
  mlp_*           the multilayer perceptron 16 -> 64 -> 64 -> 3 with tanh
                  hidden layers and a linear output; loss
                  L = 1/(2B) sum_b sum_o (yhat_bo - y_bo)^2; Adam (Kingma & Ba).
  quality_ok      the factor-10 rule: min_{i < n_r} d_i / sigma_i >= 0.1 with
                  d_i the i-th largest |r_ii| among the first n_r.
  ice_sigma_min   incremental condition estimation (Bischof) of sigma_min of an
                  upper-triangular R: a unit vector x is grown one column at a
                  time so that ||x^T R_k|| stays small; the estimate is that norm.
"""
from __future__ import annotations

import numpy as np

NFEAT, NH, NOUT = 16, 64, 3
LOG_FLOOR = -30.0
SAMPLE = 64

# parameter layout (one flat vector): W1 [NH, NFEAT], b1 [NH], W2 [NH, NH], b2 [NH], W3 [NOUT, NH], b3 [NOUT]
SHAPES = [(NH, NFEAT), (NH,), (NH, NH), (NH,), (NOUT, NH), (NOUT,)]
NPARAM = sum(int(np.prod(s)) for s in SHAPES)  # 5443


def unpack(theta):
    out, off = [], 0
    for s in SHAPES:
        k = int(np.prod(s))
        out.append(np.asarray(theta[off: off + k], dtype=np.float64).reshape(s))
        off += k
    return out


def pack(parts):
    return np.concatenate([np.asarray(p, dtype=np.float64).ravel() for p in parts])


# ------------------------------------------------------------------ features
def sample_columns(n: int) -> np.ndarray:
    """floor(k n / s) for k < s, s = min(64, n): distinct, spread over the columns."""
    s = min(SAMPLE, n)
    return np.array([(k * n) // s for k in range(s)], dtype=np.int64)


def order_stat(sorted_vals: np.ndarray, q: float) -> float:
    """Lower order statistic: the value at index floor(q (N - 1)) of an ascending array."""
    n = len(sorted_vals)
    return float(sorted_vals[int(np.floor(q * (n - 1)))])


def features(a: np.ndarray) -> np.ndarray:
    a = np.asarray(a, dtype=np.float64)
    m, n = a.shape
    f = np.zeros(NFEAT)
    f[9], f[10], f[11] = np.log2(max(m, 1)), np.log2(max(n, 1)), n / max(m, 1)
    if n == 0 or m == 0:
        return f
    u = np.sqrt(np.sum(a * a, axis=0))
    umax = u.max()
    if umax == 0.0:
        return f
    ell = np.full(n, LOG_FLOOR)
    pos = u > 0
    ell[pos] = np.maximum(np.log10(u[pos] / umax), LOG_FLOOR)
    ell = np.sort(ell)
    for k in range(9):
        f[k] = order_stat(ell, (k + 1) / 10.0)
    cols = sample_columns(n)
    c = a[:, cols]
    g = c.T @ c
    d = np.sqrt(np.diag(g))
    s = len(cols)
    th = []
    for i in range(s):
        for j in range(i + 1, s):
            th.append(abs(g[i, j] / (d[i] * d[j])) if d[i] > 0 and d[j] > 0 else 0.0)
    if th:
        th = np.sort(np.array(th))
        f[12] = float(np.mean(th))
        f[13] = order_stat(th, 0.95)
        f[14] = float(th[-1])
        f[15] = float(np.mean(th > 0.5))
    return f


# ----------------------------------------------------------------------- MLP
def mlp_forward(theta, x):
    """x [B, 16] -> (yhat [B, 3], cache)."""
    w1, b1, w2, b2, w3, b3 = unpack(theta)
    h1 = np.tanh(x @ w1.T + b1)
    h2 = np.tanh(h1 @ w2.T + b2)
    y = h2 @ w3.T + b3
    return y, (x, h1, h2)


def mlp_loss(theta, x, y):
    yhat, _ = mlp_forward(theta, x)
    return 0.5 * float(np.sum((yhat - y) ** 2)) / x.shape[0]


def mlp_grad(theta, x, y):
    """Gradient of mlp_loss by the chain rule (backpropagation)."""
    w1, b1, w2, b2, w3, b3 = unpack(theta)
    yhat, (x, h1, h2) = mlp_forward(theta, x)
    bsz = x.shape[0]
    dy = (yhat - y) / bsz                # dL/dyhat
    gw3 = dy.T @ h2
    gb3 = dy.sum(axis=0)
    dh2 = dy @ w3
    dz2 = dh2 * (1.0 - h2 * h2)          # tanh' = 1 - tanh^2
    gw2 = dz2.T @ h1
    gb2 = dz2.sum(axis=0)
    dh1 = dz2 @ w2
    dz1 = dh1 * (1.0 - h1 * h1)
    gw1 = dz1.T @ x
    gb1 = dz1.sum(axis=0)
    return pack([gw1, gb1, gw2, gb2, gw3, gb3])


def adam_step(theta, g, mom, vel, t, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update at step t >= 1; returns (theta, mom, vel)."""
    mom = b1 * mom + (1.0 - b1) * g
    vel = b2 * vel + (1.0 - b2) * g * g
    mhat = mom / (1.0 - b1 ** t)
    vhat = vel / (1.0 - b2 ** t)
    return theta - lr * mhat / (np.sqrt(vhat) + eps), mom, vel


# ------------------------------------------------------------------ quality
def numerical_rank(sigma: np.ndarray, n: int) -> int:
    """n_r = #{sigma_i > eps n sigma_1} (Section 5)."""
    if len(sigma) == 0 or sigma[0] == 0:
        return 0
    return int(np.sum(sigma > np.finfo(np.float64).eps * n * sigma[0]))


def quality_ok(rdiag: np.ndarray, sigma: np.ndarray, n: int, band: float = 0.1) -> bool:
    """Factor-10 rule on the first n_r values: d_i / sigma_i >= band."""
    nr = numerical_rank(sigma, n)
    if nr == 0:
        return True
    d = np.sort(np.abs(np.asarray(rdiag)[:nr]))[::-1]
    return bool(np.min(d / sigma[:nr]) >= band)


def ice_sigma_min(r: np.ndarray) -> float:
    """Incremental condition estimation of sigma_min for upper-triangular r (k x k).

    Keeps a unit vector x_k and the row y_k = x_k^T R_k.  For the next column
    [v; gamma], x_{k+1} = [s x_k; c] with s^2 + c^2 = 1 gives
    ||x_{k+1}^T R_{k+1}||^2 = s^2 ||y_k||^2 + (s alpha + c gamma)^2, alpha = x_k^T v;
    (s, c) is the unit eigenvector of the smallest eigenvalue of
    M = [[p, q], [q, r]] = [[||y||^2 + alpha^2, alpha gamma], [alpha gamma, gamma^2]].
    det M = ||y||^2 gamma^2 exactly, so lambda_min = det M / lambda_max is formed
    without cancellation (lambda_max = (p + r)/2 + sqrt(((p - r)/2)^2 + q^2));
    the eigenvector is the larger of (-q, p - lambda_min) and (r - lambda_min, -q)."""
    r = np.asarray(r, dtype=np.float64)
    k = r.shape[0]
    if k == 0:
        return 0.0
    x = np.array([1.0])
    est = abs(r[0, 0])
    for j in range(1, k):
        v, gamma = r[:j, j], r[j, j]
        alpha = float(x @ v)
        p = est * est + alpha * alpha
        q = alpha * gamma
        rr = gamma * gamma
        lmax = 0.5 * (p + rr) + np.hypot(0.5 * (p - rr), q)
        lmin = (est * est) * rr / lmax if lmax > 0 else 0.0
        v1 = np.array([-q, p - lmin])
        v2 = np.array([rr - lmin, -q])
        vec = v1 if np.hypot(*v1) >= np.hypot(*v2) else v2
        nv = np.hypot(*vec)
        s, c = (vec / nv) if nv > 0 else (1.0, 0.0)
        x = np.concatenate([s * x, [c]])
        est = float(np.sqrt(lmin))
    return est
