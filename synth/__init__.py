"""Seeded synthetic inputs shared by the tests, the smoke check and the bench.

This module only draws point sets (numpy ``default_rng``); it holds none of
the method's arithmetic. Shapes and value distributions follow the paper's
workloads (Sec. 4: clustered Gaussian data, image-shaped 784-d data standing
in for MNIST, large low-d clustered data), none of which ships with the paper.

Every generator returns float32 ``X[N, d]`` plus a dict of the parameters the
method runs with (K, rho, delta, max_iters, seed).
"""
from __future__ import annotations

import math

import numpy as np

__all__ = ["workload", "WORKLOADS", "gaussian_mixture", "integer_points", "image_like",
           "lowd_blobs", "anisotropic_clusters", "batched_datasets", "clustered_labels",
           "single_gaussian", "synthetic_gaussian", "audio_like"]


def gaussian_mixture(N: int, d: int, n_centres: int, seed: int, lo: float = -10.0,
                     hi: float = 10.0, sigma: float = 1.0, return_labels: bool = False):
    """Isotropic Gaussian mixture: centres U[lo,hi]^d, uniform labels, x = c + sigma*N(0,I)."""
    rng = np.random.default_rng(seed)
    centres = rng.uniform(lo, hi, (n_centres, d))
    labels = rng.integers(0, n_centres, N)
    X = (centres[labels] + sigma * rng.standard_normal((N, d))).astype(np.float32)
    return (X, labels) if return_labels else X


def single_gaussian(N: int, d: int, seed: int) -> np.ndarray:
    """The paper's Synthetic Single Gaussian Dataset (Sec. 4): every point from
    one Gaussian centred at the origin with covariance 2 I_d."""
    rng = np.random.default_rng(seed)
    return (math.sqrt(2.0) * rng.standard_normal((N, d), dtype=np.float32)).astype(np.float32)


def synthetic_gaussian(N: int, d: int, seed: int) -> np.ndarray:
    """The paper's Synthetic Gaussian Dataset (Sec. 4), non-single variant: one
    Gaussian per dimension i, centred at the canonical basis vector e_i, with
    covariance 2 I_d; each point picks its Gaussian uniformly at random (the
    paper does not give the mixing weights)."""
    rng = np.random.default_rng(seed)
    labels = rng.integers(0, d, N)
    X = math.sqrt(2.0) * rng.standard_normal((N, d))
    X[np.arange(N), labels] += 1.0
    return X.astype(np.float32)


def integer_points(N: int, d: int, hi: int, seed: int) -> np.ndarray:
    """Small non-negative integer coordinates in [0, hi]: every FP32 sum below 2^24
    is exact, so FP32 and FP64 distances agree bit for bit."""
    rng = np.random.default_rng(seed)
    return rng.integers(0, hi + 1, (N, d)).astype(np.float32)


def clustered_labels(N: int, d: int, n_clusters: int, seed: int, spread: float = 0.5):
    """Clustered dataset in the sense of Sec. 3.2 (every point's nearest
    neighbours lie in its own cluster): well separated centres."""
    return gaussian_mixture(N, d, n_clusters, seed, -10.0, 10.0, spread, return_labels=True)


def image_like(N: int = 60000, seed: int = 1, side: int = 28, n_protos: int = 10, on_frac: float = 0.2,
               noise: float = 0.01, jitter: float = 1.0, return_labels: bool = False):
    """784-d image-shaped integers in [0, 255], ~80% zeros (stand-in for MNIST, Sec. 4).

    Each of 10 prototypes is a smooth field, a sum of 3-6 Gaussian bumps. A
    point picks a prototype and deforms it with a few continuous parameters
    (a global shift and stretch, a per-bump jitter of ``jitter`` pixels, per-bump
    amplitudes), so the points lie near a low-dimensional manifold the way
    handwritten digits do. The top ``on_frac`` pixels of the field are kept and
    mapped to intensities 90..255, scaled by U(0.6, 1); each pixel is then set to
    U{1..255} with probability ``noise``; values are rounded and clipped.
    Squared norms stay below 2^23, so all pair distances are exact in FP32.
    """
    rng = np.random.default_rng(seed)
    yy, xx = np.mgrid[0:side, 0:side].astype(np.float32)
    yy, xx = yy.reshape(-1), xx.reshape(-1)
    protos = []
    for _ in range(n_protos):
        nb = int(rng.integers(3, 7))
        protos.append((rng.uniform(7, side - 7, (nb, 2)), rng.uniform(1.5, 4.0, (nb, 2)), rng.uniform(0.6, 1.0, nb)))
    labels = rng.integers(0, n_protos, N)
    d = side * side
    X = np.empty((N, d), np.float32)
    for s in range(0, N, 4096):
        n = min(4096, N - s)
        out = np.zeros((n, d), np.float32)
        for k, (c, sg, a) in enumerate(protos):
            idx = np.nonzero(labels[s:s + n] == k)[0]
            if len(idx) == 0:
                continue
            m, nb = len(idx), len(a)
            shift = rng.normal(0, 1.0, (m, 1, 2)) + rng.normal(0, jitter, (m, nb, 2))
            stretch = np.exp(rng.normal(0, 0.08, (m, 1, 2)))
            amp = a[None, :] * rng.uniform(0.75, 1.0, (m, nb))
            cc = (c[None] + shift).astype(np.float32)
            ss = (sg[None] * stretch).astype(np.float32)
            f = np.zeros((m, d), np.float32)
            for b in range(nb):
                f += amp[:, b:b + 1].astype(np.float32) * np.exp(
                    -0.5 * (((yy[None] - cc[:, b, 0:1]) / ss[:, b, 0:1]) ** 2
                            + ((xx[None] - cc[:, b, 1:2]) / ss[:, b, 1:2]) ** 2))
            f /= f.max(1, keepdims=True)
            thr = np.quantile(f, 1.0 - on_frac, axis=1, keepdims=True)
            v = np.where(f >= thr, 90.0 + 165.0 * (f - thr) / np.maximum(1e-6, 1.0 - thr), 0.0)
            out[idx] = v * rng.uniform(0.6, 1.0, (m, 1))
        nz = rng.random((n, d)) < noise
        out = np.where(nz, rng.integers(1, 256, (n, d)).astype(np.float32), out)
        X[s:s + n] = np.clip(np.rint(out), 0, 255)
    return (X, labels) if return_labels else X


def lowd_blobs(N: int = 4_000_000, seed: int = 2, n_blobs: int = 1000, sigma: float = 0.01,
               background: float = 0.1, return_labels: bool = False):
    """3-d: Gaussian blobs (sigma) around U[0,1]^3 centres plus uniform background,
    rows shuffled into random memory order. Label -1 marks background."""
    rng = np.random.default_rng(seed)
    nb = int(round(N * background))
    nc = N - nb
    centres = rng.uniform(0.0, 1.0, (n_blobs, 3))
    lab = rng.integers(0, n_blobs, nc)
    X = np.empty((N, 3), np.float32)
    X[:nc] = centres[lab] + sigma * rng.standard_normal((nc, 3))
    X[nc:] = rng.uniform(0.0, 1.0, (nb, 3))
    labels = np.concatenate([lab, -np.ones(nb, np.int64)])
    perm = rng.permutation(N)
    X = X[perm]
    labels = labels[perm]
    return (X, labels) if return_labels else X


def anisotropic_clusters(N: int = 200_000, d: int = 960, seed: int = 3, n_clusters: int = 100):
    """Centres U[-1,1]^d; per-cluster per-dimension sigma = 10^U(-1,0); x = c + sigma*N(0,I)."""
    rng = np.random.default_rng(seed)
    centres = rng.uniform(-1.0, 1.0, (n_clusters, d)).astype(np.float32)
    sig = (10.0 ** rng.uniform(-1.0, 0.0, (n_clusters, d))).astype(np.float32)
    lab = rng.integers(0, n_clusters, N)
    X = np.empty((N, d), np.float32)
    for s in range(0, N, 16384):
        n = min(16384, N - s)
        l = lab[s:s + n]
        X[s:s + n] = centres[l] + sig[l] * rng.standard_normal((n, d), dtype=np.float32)
    return X


def audio_like(N: int = 54387, d: int = 192, seed: int = 7, n_speakers: int = 30, rank: int = 16,
               ar: float = 0.9):
    """Stand-in for the shape of the Audio dataset of Sec. 4 (54387 frames of
    192 features from spoken English sentences; the real set is not used).

    Frames come in sentences (lengths 20 + Geometric(1/60)) of one speaker
    each; a speaker has a mean m_s ~ N(0, I) and a rank-16 mixing A_s; within
    a sentence a latent z_t follows an AR(1) walk (coefficient 0.9, unit
    stationary variance) and the frame is (m_s + A_s z_t / 4 + 0.1 N(0, I))
    times per-feature scales 1 / sqrt(1 + j / 24), j = 0..d-1 (feature
    variance falling along the vector, as in spectral features)."""
    from scipy.signal import lfilter
    rng = np.random.default_rng(seed)
    scale = (1.0 / np.sqrt(1.0 + np.arange(d) / 24.0)).astype(np.float64)
    means = rng.standard_normal((n_speakers, d))
    mix = rng.standard_normal((n_speakers, d, rank)) / math.sqrt(rank)
    X = np.empty((N, d), np.float32)
    s = 0
    while s < N:
        L = min(N - s, 20 + int(rng.geometric(1.0 / 60.0)))
        spk = int(rng.integers(0, n_speakers))
        eps = rng.standard_normal((L, rank))
        z = lfilter([math.sqrt(1.0 - ar * ar)], [1.0, -ar], eps, axis=0)
        z[0] = eps[0]
        fr = means[spk] + 0.25 * z @ mix[spk].T + 0.1 * rng.standard_normal((L, d))
        X[s:s + L] = (fr * scale).astype(np.float32)
        s += L
    return X


def batched_datasets(count: int = 512, seed: int = 4, n_lo: int = 500, n_hi: int = 20000,
                     dims=(16, 64, 128)):
    """Independent Gaussian-mixture datasets of uneven N and d.

    N_i = round(exp(U(ln n_lo, ln n_hi))), d_i uniform over ``dims``, 5..20
    components with centres U[-10,10]^d and sigma 1, per-dataset seeds drawn
    from the master generator. Returns a list of (X_i, seed_i)."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(count):
        n = int(round(math.exp(rng.uniform(math.log(n_lo), math.log(n_hi)))))
        d = int(dims[int(rng.integers(0, len(dims)))])
        comps = int(rng.integers(5, 21))
        s = int(rng.integers(0, 2**31 - 1))
        out.append((gaussian_mixture(n, d, comps, s), s))
    return out


# Method parameters per workload. max_iters for the large cases and the seeds
# of blobs4m_d3 and aniso200k_d960 are readings (the workload text leaves
# them open).
WORKLOADS = {
    "gauss2k_d8": dict(name="gauss2k_d8", K=10, rho=1.0, delta=0.001, max_iters=20, seed=0),
    "image60k_d784": dict(name="image60k_d784", K=20, rho=1.0, delta=0.001, max_iters=30, seed=1),
    "blobs4m_d3": dict(name="blobs4m_d3", K=15, rho=0.5, delta=0.001, max_iters=30, seed=2),
    "aniso200k_d960": dict(name="aniso200k_d960", K=20, rho=0.5, delta=0.001, max_iters=30, seed=3),
    "batch512": dict(name="batch512", K=15, rho=1.0, delta=0.001, max_iters=30, seed=4),
}


def workload(name: str, N: int | None = None):
    """(X, params) of a named workload. ``N`` shrinks the point count (tests)."""
    p = dict(WORKLOADS[name])
    if name == "gauss2k_d8":
        X = gaussian_mixture(N or 2000, 8, 10, 0)
    elif name == "image60k_d784":
        X = image_like(N or 60000, 1)
    elif name == "blobs4m_d3":
        X = lowd_blobs(N or 4_000_000, 2)
    elif name == "aniso200k_d960":
        X = anisotropic_clusters(N or 200_000, 960, 3)
    else:
        raise ValueError(f"{name}: a batch of datasets, see batched_datasets()")
    return X, p
