"""Seeded synthetic inputs for QRDM / QRP (numpy, host side).

This module only builds matrices: it holds none of the factorization's
arithmetic and is shared by the tests, the benchmark and the oracle side.
All matrices are float64, Fortran (column-major) order.

The paper evaluates on numerically singular matrices of the SJSU Singular
Matrix Database (Section 5), which is not available here; these prescribed
spectrum matrices stand in for it.  Each generator states its recipe.
"""
from __future__ import annotations

import numpy as np

EPS = np.finfo(np.float64).eps


def haar(n: int, rng: np.random.Generator) -> np.ndarray:
    """Haar-distributed orthogonal n x n: QR of a Gaussian, columns x sign(diag R)."""
    g = rng.standard_normal((n, n))
    q, r = np.linalg.qr(g)
    q *= np.sign(np.diag(r))[None, :]
    return np.asfortranarray(q)


def haar_cols(m: int, k: int, rng: np.random.Generator) -> np.ndarray:
    """m x k with Haar-distributed orthonormal columns (k <= m)."""
    g = rng.standard_normal((m, k))
    q, r = np.linalg.qr(g)
    q *= np.sign(np.diag(r))[None, :]
    return np.asfortranarray(q)


def from_spectrum(m: int, n: int, sigma: np.ndarray, seed: int) -> np.ndarray:
    """A = U diag(sigma) V^T with U (m x p), V (n x p) Haar columns, p = len(sigma)."""
    rng = np.random.default_rng(seed)
    p = len(sigma)
    u = haar_cols(m, p, rng)
    v = haar_cols(n, p, rng)
    a = (u * np.asarray(sigma)[None, :]) @ v.T
    return np.asfortranarray(a)


def geometric_rank(n: int, r: int, top: float, bottom: float, tail: float) -> np.ndarray:
    """sigma_1..r geometric top->bottom, sigma_{r+1..n} = tail."""
    s = np.full(n, tail, dtype=np.float64)
    s[:r] = np.geomspace(top, bottom, r)
    return s


def small_rank64(seed: int = 0, n: int = 256) -> np.ndarray:
    """256 x 256, sigma_1..64 geometric 1 -> 1e-3, sigma_65..256 = 1e-15."""
    return from_spectrum(n, n, geometric_rank(n, 64, 1.0, 1e-3, 1e-15), seed)


def half_rank_noise(n: int = 4096, seed: int = 0) -> np.ndarray:
    """n x n, sigma_1..n/2 geometric 1 -> 1e-8, the rest 1e-16*|g_i|, g ~ N(0,1)."""
    rng = np.random.default_rng(seed + 7919)
    r = n // 2
    s = np.empty(n)
    s[:r] = np.geomspace(1.0, 1e-8, r)
    s[r:] = 1e-16 * np.abs(rng.standard_normal(n - r))
    return from_spectrum(n, n, s, seed)


def kahan(n: int = 4096, theta: float = 1.2) -> np.ndarray:
    """Kahan matrix K_n(theta) = diag(s^i) (I - c * strictly-upper ones), c = cos, s = sin."""
    c, s = np.cos(theta), np.sin(theta)
    k = -c * np.triu(np.ones((n, n)), 1) + np.eye(n)
    d = s ** np.arange(n)
    return np.asfortranarray(d[:, None] * k)


def geometric_full(n: int = 8192, seed: int = 0) -> np.ndarray:
    """n x n, sigma geometric 1 -> 1e-16 over all n."""
    return from_spectrum(n, n, np.geomspace(1.0, 1e-16, n), seed)


def devils_stairs(n: int = 8192, step: int = 512, seed: int = 0) -> np.ndarray:
    """n x n, sigma_i = 10^-floor((i-1)/step): steps of `step` values dropping 10x each."""
    s = 10.0 ** (-np.floor(np.arange(n) / step))
    return from_spectrum(n, n, s, seed)


def gaussian(m: int, n: int, seed: int = 0) -> np.ndarray:
    """A_ij ~ N(0, 1) iid."""
    rng = np.random.default_rng(seed)
    return np.asfortranarray(rng.standard_normal((m, n)))


def rank1(m: int, n: int, seed: int = 0) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return np.asfortranarray(np.outer(rng.standard_normal(m), rng.standard_normal(n)))


def orthogonal_columns(m: int, norms: np.ndarray, seed: int = 0) -> tuple[np.ndarray, np.ndarray]:
    """A = Q0 diag(s) Pi0: orthogonal columns with prescribed norms s in a random
    column order.  Returns (A, order) where column j of A has norm norms[order[j]]."""
    rng = np.random.default_rng(seed)
    k = len(norms)
    q = haar_cols(m, k, rng)
    order = rng.permutation(k)
    a = q[:, order] * np.asarray(norms)[order][None, :]
    return np.asfortranarray(a), order


def paired_columns(m: int, npair: int, cos: float, seed: int = 0) -> np.ndarray:
    """2*npair columns in pairs: column 2k is Gaussian, column 2k+1 is a unit
    vector at angle arccos(cos) to it inside the plane of column 2k and a fresh
    Gaussian direction, scaled to 0.999 of its norm.  Pairs are nearly
    orthogonal to each other (m >> npair); the pair's cosine is `cos`, so the DM
    cosine test separates the members of a pair when cos >= delta."""
    rng = np.random.default_rng(seed)
    q = haar_cols(m, 2 * npair, rng)
    norms = np.exp(rng.uniform(-1.0, 1.0, npair))
    a = np.empty((m, 2 * npair))
    sn = np.sqrt(1.0 - cos * cos)
    for k in range(npair):
        a[:, 2 * k] = norms[k] * q[:, 2 * k]
        a[:, 2 * k + 1] = 0.999 * norms[k] * (cos * q[:, 2 * k] + sn * q[:, 2 * k + 1])
    return np.asfortranarray(a)


def angles_in_plane(m: int, angles: np.ndarray, norms: np.ndarray, seed: int = 0) -> np.ndarray:
    """Columns norms[i] * (cos(angles[i]) e + sin(angles[i]) f) for two orthonormal
    vectors e, f of R^m (Haar), so the cosine of columns i and j is exactly
    cos(angles[i] - angles[j])."""
    rng = np.random.default_rng(seed)
    q = haar_cols(m, 2, rng)
    a = q[:, :1] * (norms * np.cos(angles))[None, :] + q[:, 1:2] * (norms * np.sin(angles))[None, :]
    return np.asfortranarray(a)


def three_directions(m: int = 16, seed: int = 0) -> np.ndarray:
    """Three unit columns at 0, 120 and 240 degrees in a random plane of R^m."""
    rng = np.random.default_rng(seed)
    q = haar_cols(m, 2, rng)
    ang = np.array([0.0, 2.0 * np.pi / 3.0, 4.0 * np.pi / 3.0])
    coef = np.stack([np.cos(ang), np.sin(ang)])
    return np.asfortranarray(q @ coef)


def batch_shapes(count: int = 2048, seed: int = 0, mmin: int = 32, mmax: int = 512,
                 nmin: int = 16) -> list[tuple[int, int, int]]:
    """(m, n, r): m ~ U{mmin..mmax}, n ~ U{nmin..m}, r ~ U{ceil(n/4)..n}."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(count):
        m = int(rng.integers(mmin, mmax + 1))
        n = int(rng.integers(nmin, m + 1))
        r = int(rng.integers((n + 3) // 4, n + 1))
        out.append((m, n, r))
    return out


def batch_matrix(m: int, n: int, r: int, seed_seq: np.random.SeedSequence) -> np.ndarray:
    """U[:, :r] diag(sigma) V[:, :r]^T, sigma_j = 10^(-14 (j-1)/(r-1)), zero beyond r."""
    rng = np.random.default_rng(seed_seq)
    sig = np.logspace(0.0, -14.0, r) if r > 1 else np.ones(1)
    u = haar_cols(m, r, rng)
    v = haar_cols(n, r, rng)
    return np.asfortranarray((u * sig[None, :]) @ v.T)


def batch(count: int = 2048, seed: int = 0, mmin: int = 32, mmax: int = 512, nmin: int = 16):
    """The uneven least-squares batch: list of Fortran float64 matrices and their (m, n, r)."""
    shapes = batch_shapes(count, seed, mmin, mmax, nmin)
    seqs = np.random.SeedSequence(seed).spawn(count)
    mats = [batch_matrix(m, n, r, s) for (m, n, r), s in zip(shapes, seqs)]
    return mats, shapes


# ---------------------------------------------------------------- learned predictor
def mlp_init(seed: int = 0) -> np.ndarray:
    """Initial MLP parameters (16 -> 64 -> 64 -> 3, the flat layout W1, b1, W2,
    b2, W3, b3): Glorot-uniform weights, zero biases; float64."""
    rng = np.random.default_rng(seed)
    parts = []
    for fan_out, fan_in in ((64, 16), (64, 64), (3, 64)):
        lim = np.sqrt(6.0 / (fan_in + fan_out))
        parts.append(rng.uniform(-lim, lim, size=fan_out * fan_in))
        parts.append(np.zeros(fan_out))
    return np.concatenate(parts)


def spectrum(kind: str, n: int, r: int, rng: np.random.Generator) -> np.ndarray:
    """Singular values (length min(m, n) = n here) of the training families:
    geom   10^(-14 (j-1)/(r-1)) for j <= r, zero beyond (the uneven batch's law);
    stairs 10^-floor(j / step), step = max(r // 6, 1), for j <= r, zero beyond;
    flat   1 for j <= r, 1e-15 beyond (a clean gap);
    split  two clusters, 1 and 10^-u (u ~ U[2, 10]), half each, zero beyond r."""
    s = np.zeros(n)
    j = np.arange(r)
    if kind == "geom":
        s[:r] = np.logspace(0.0, -14.0, r) if r > 1 else 1.0
    elif kind == "stairs":
        step = max(r // 6, 1)
        s[:r] = 10.0 ** (-np.floor(j / step))
    elif kind == "flat":
        s[:r] = 1.0
        s[r:] = 1e-15
    elif kind == "split":
        s[:r] = np.where(j < (r + 1) // 2, 1.0, 10.0 ** (-rng.uniform(2.0, 10.0)))
    else:
        raise ValueError(kind)
    return s


def training_batch(count: int = 4096, seed: int = 11, mmin: int = 32, mmax: int = 512, nmin: int = 16):
    """Matrices for the predictor's labels: the uneven batch's shapes with the
    four spectrum families above.  Returns (mats, shapes (m, n, r), sigmas, kinds)."""
    rng = np.random.default_rng(seed)
    kinds = ("geom", "stairs", "flat", "split")
    mats, shapes, sigmas, kk = [], [], [], []
    for i in range(count):
        m = int(rng.integers(mmin, mmax + 1))
        n = int(rng.integers(nmin, m + 1))
        r = int(rng.integers((n + 3) // 4, n + 1))
        kind = kinds[i % 4]
        s = spectrum(kind, n, r, rng)
        u = haar_cols(m, n, rng)
        v = haar_cols(n, n, rng)
        mats.append(np.asfortranarray((u * s[None, :]) @ v.T))
        shapes.append((m, n, r))
        sigmas.append(np.sort(s)[::-1])
        kk.append(kind)
    return mats, shapes, sigmas, kk


def lstsq_factors(m: int, n: int, r: int, seed):
    """Synthetic output of a pivoted QR for the least-squares solve, in the
    LAPACK layout: reflector entries N(0, 1/m) below the diagonal, scalars
    uniform in [0.5, 1], an upper triangle with diagonal entries of random sign
    and magnitude in [1, 2] and other entries N(0, 1/r), and a random
    permutation.  Any such arrays define Q_r and R11.  Returns (qr, tau, perm)."""
    rng = np.random.default_rng(seed)
    p = min(m, n)
    qr = np.asfortranarray(rng.standard_normal((m, n)) / np.sqrt(max(m, 1)))
    up = np.triu(rng.standard_normal((m, n)) / np.sqrt(max(r, 1)), 1)
    qr = np.where(np.triu(np.ones((m, n), dtype=bool), 1), up, qr)
    d = rng.uniform(1.0, 2.0, p) * rng.choice([-1.0, 1.0], p)
    qr[np.arange(p), np.arange(p)] = d
    tau = rng.uniform(0.5, 1.0, p)
    perm = rng.permutation(n).astype(np.int32)
    return np.asfortranarray(qr), tau, perm


def device_spectrum(n: int, spectrum: str, seed: int = 0) -> np.ndarray:
    """Singular values (in U diag(s) V^T order) of the device workloads with a
    prescribed spectrum: geometric 1 -> 1e-16; stairs, steps of 512 dropping 10x;
    half_rank, geometric 1 -> 1e-8 over n/2 then 1e-16 |g_i| (the noise drawn
    from its own stream, seed + 7919, as half_rank_noise)."""
    if spectrum == "geometric":
        return np.geomspace(1.0, 1e-16, n)
    if spectrum == "stairs":
        return 10.0 ** (-np.floor(np.arange(n) / 512))
    if spectrum == "half_rank":
        r = n // 2
        s = np.empty(n)
        s[:r] = np.geomspace(1.0, 1e-8, r)
        s[r:] = 1e-16 * np.abs(np.random.default_rng(seed + 7919).standard_normal(n - r))
        return s
    raise ValueError(spectrum)


def device_matrix(n: int, spectrum: str, seed: int, torch):
    """Seeded synthetic n x n matrix on the GPU (column-major float64), the benchmark workload.
    geometric: sigma 1 -> 1e-16; stairs: steps of 512 dropping 10x; half_rank: sigma
    1 -> 1e-8 over n/2, then noise; gaussian: N(0,1); kahan: K_n(1.2).
    U, V are Haar: QR of seeded host Gaussians (signs fixed), formed on the GPU."""
    rng = np.random.default_rng(seed)
    if spectrum == "gaussian":
        a = torch.from_numpy(rng.standard_normal((n, n))).cuda()
        return a.t().contiguous().t()
    if spectrum == "kahan":
        return torch.from_numpy(np.ascontiguousarray(kahan(n, 1.2).T)).cuda().t()
    s = device_spectrum(n, spectrum, seed)

    def haar():
        g = torch.from_numpy(rng.standard_normal((n, n))).cuda()
        q, r = torch.linalg.qr(g)
        return q * torch.sign(torch.diagonal(r))[None, :]

    u, v = haar(), haar()
    a = (u * torch.from_numpy(s).cuda()[None, :]) @ v.t()
    del u, v
    return a.t().contiguous().t()  # column-major (m, n) view
