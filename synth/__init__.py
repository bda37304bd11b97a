"""Seeded synthetic inputs for the coprime-blurred-pair (CBP) workloads.

This module is the only code shared by the CPU oracle's tests and the GPU
path's tests and benchmark.  It holds the *forward* model only: scenes,
blur kernels, the full linear convolution B = L (x) K + N_e of the paper's
blur model (Sec. 4, eq. 1) and the coprimality rule used to redraw kernel
pairs (Sec. 3: the two kernels, read as bivariate polynomials, share no
non-constant factor).  No step of the recovery method lives here.

Every generator takes an explicit seed; per-frame / per-stream streams are
derived with ``numpy.random.SeedSequence`` from (seed, key, ...) so that any
frame of a long sequence can be regenerated on its own.

Conventions: images are row-major ``[y][x]``; a kernel of size k is k x k;
a blurred frame of an m x n latent is (m+k-1) x (n+k-1) (full convolution).
"""

from __future__ import annotations

import numpy as np
from scipy import signal

__all__ = [
    "rng_for", "full_conv2d", "sylvester_margin", "is_coprime_pair",
    "uniform_scene", "gaussian_scene", "blob_sequence",
    "uniform_kernel", "gaussian_perturbed_kernel", "draw_coprime_pair",
    "blur_pair", "config1", "config2", "config3_frames"
]


def rng_for(seed: int, *keys: int) -> np.random.Generator:
    """PCG64 generator for (seed, *keys); keys name a frame / stream / role."""
    return np.random.default_rng(np.random.SeedSequence([int(seed), *map(int, keys)]))


# --------------------------------------------------------------------------
# forward model
# --------------------------------------------------------------------------

def full_conv2d(L: np.ndarray, K: np.ndarray) -> np.ndarray:
    """Full linear 2-D convolution (output (m+k-1) x (n+k-1)), eq. 1 without noise.

    Integer inputs are convolved exactly (direct sum in int64 / object);
    floating inputs in float64, directly for small problems and by FFT for
    large ones (rounding ~1e-16 relative, i.e. at the level of the data's own
    float64 representation).
    """
    if L.dtype.kind in "iuO" and K.dtype.kind in "iuO":
        return signal.convolve2d(L, K, mode="full")
    L = np.asarray(L, dtype=np.float64)
    K = np.asarray(K, dtype=np.float64)
    if L.size * K.size <= 4_000_000:
        return signal.convolve2d(L, K, mode="full")
    return signal.fftconvolve(L, K, mode="full")


def _sylvester(p: np.ndarray, q: np.ndarray) -> np.ndarray:
    """Sylvester matrix of two 1-D polynomials given by ascending coefficients."""
    dp, dq = len(p) - 1, len(q) - 1
    n = dp + dq
    S = np.zeros((n, n), dtype=np.complex128)
    for c in range(dq):
        S[c:c + dp + 1, c] = p
    for c in range(dp):
        S[c:c + dq + 1, dq + c] = q
    return S


def sylvester_margin(K1: np.ndarray, K2: np.ndarray, sample_counts=(None,)) -> float:
    """Smallest relative singular value of the 1-D Sylvester matrices of the
    kernel pair restricted to unit-circle samples, along both axes.

    For each S in ``sample_counts`` (None = max kernel size) and each S-th
    root of unity w, the slices k_c(w, .) (rows weighted by w^y) and
    k_c(., w) are 1-D polynomials; they share a root iff their Sylvester
    matrix is singular.  The returned margin is min sigma_min / sigma_max
    over all slices.  A bivariate pair with a common non-constant factor
    has margin ~0 at every sample.
    """
    k1, k2 = K1.shape[0], K2.shape[0]
    margin = np.inf
    for S in sample_counts:
        S = max(k1, k2) if S is None else int(S)
        for j in range(S):
            for axis in (0, 1):
                w1 = np.exp(-2j * np.pi * ((j * np.arange(k1)) % S) / S)
                w2 = np.exp(-2j * np.pi * ((j * np.arange(k2)) % S) / S)
                if axis == 0:
                    p, q = w1 @ K1, w2 @ K2      # evaluate along y, poly in x
                else:
                    p, q = K1 @ w1, K2 @ w2      # evaluate along x, poly in y
                if len(p) == 1 or len(q) == 1:
                    s = np.array([abs(p[0]) if len(p) == 1 else abs(q[0])])
                    margin = min(margin, 1.0 if s[0] > 0 else 0.0)
                    continue
                s = np.linalg.svd(_sylvester(p, q), compute_uv=False)
                margin = min(margin, s[-1] / s[0])
    return float(margin)


def is_coprime_pair(K1, K2, sample_counts=(None,), tol=1e-10) -> bool:
    return sylvester_margin(K1, K2, sample_counts) > tol


# --------------------------------------------------------------------------
# scenes
# --------------------------------------------------------------------------

def uniform_scene(rng: np.random.Generator, m: int, n: int) -> np.ndarray:
    return rng.random((m, n))


def _gaussian_sum(rng, m, n, count, axes_frac=(0.02, 0.2), amp=(0.2, 1.0)):
    yy, xx = np.mgrid[0:m, 0:n].astype(np.float64)
    img = np.zeros((m, n))
    for _ in range(count):
        cy, cx = rng.uniform(0, m), rng.uniform(0, n)
        ay = rng.uniform(*axes_frac) * m
        ax = rng.uniform(*axes_frac) * n
        th = rng.uniform(0, np.pi)
        a = rng.uniform(*amp)
        c, s = np.cos(th), np.sin(th)
        dy, dx = yy - cy, xx - cx
        u = (c * dx + s * dy) / ax
        v = (-s * dx + c * dy) / ay
        img += a * np.exp(-0.5 * (u * u + v * v))
    return img


def gaussian_scene(rng: np.random.Generator, m: int, n: int, count: int = 40,
                   texture: float = 0.1) -> np.ndarray:
    """Smooth scene: a sum of ``count`` random anisotropic Gaussians (centres
    uniform, axes U(0.02, 0.2) x image size, angle U(0, pi), amplitude
    U(0.2, 1)), scaled to [0, 1-texture], plus ``texture`` x U[0,1) noise."""
    g = _gaussian_sum(rng, m, n, count)
    g = g / max(g.max(), 1e-30)
    return (1.0 - texture) * g + texture * rng.random((m, n))


def blob_sequence(seed: int, nframes: int, m: int, n: int, blobs: int = 30,
                  max_shift: int = 4):
    """Generator of frames of a moving-blob surveillance-like scene.

    A static smooth background (``gaussian_scene``) plus ``blobs`` Gaussian
    blobs of radius 8..40 px moving by integer random-walk shifts of at most
    ``max_shift`` px per frame; values clamped to [0, 1].
    """
    r = rng_for(seed, 0)
    bg = gaussian_scene(r, m, n)
    cy = r.uniform(0, m, blobs)
    cx = r.uniform(0, n, blobs)
    rad = r.uniform(8, 40, blobs)
    amp = r.uniform(-0.5, 0.5, blobs)
    yy, xx = np.mgrid[0:m, 0:n].astype(np.float64)
    for f in range(nframes):
        rf = rng_for(seed, 1, f)
        if f:
            cy = np.clip(cy + rf.integers(-max_shift, max_shift + 1, blobs), 0, m - 1)
            cx = np.clip(cx + rf.integers(-max_shift, max_shift + 1, blobs), 0, n - 1)
        img = bg.copy()
        for b in range(blobs):
            img += amp[b] * np.exp(-((yy - cy[b]) ** 2 + (xx - cx[b]) ** 2) / (2 * rad[b] ** 2))
        yield np.clip(img, 0.0, 1.0)


# --------------------------------------------------------------------------
# kernels
# --------------------------------------------------------------------------

def uniform_kernel(rng: np.random.Generator, k: int) -> np.ndarray:
    """k x k kernel with U(0,1) entries, normalised to sum 1."""
    K = rng.random((k, k))
    while np.any(K == 0.0):
        K = rng.random((k, k))
    return K / K.sum()


def gaussian_perturbed_kernel(rng: np.random.Generator, k: int, sigma: float = 2.0,
                              perturb: float = 0.2) -> np.ndarray:
    """Centred Gaussian (std ``sigma``) scaled to peak 1, plus ``perturb`` x
    U[0,1) per entry (additive reading), normalised to sum 1."""
    c = (k - 1) / 2.0
    y, x = np.mgrid[0:k, 0:k].astype(np.float64)
    g = np.exp(-((y - c) ** 2 + (x - c) ** 2) / (2 * sigma * sigma))
    K = g / g.max() + perturb * rng.random((k, k))
    return K / K.sum()


def draw_coprime_pair(rng: np.random.Generator, k1: int, k2: int, kind: str = "uniform",
                      sample_counts=(None,), tol: float = 1e-10, max_tries: int = 100):
    """Draw (K1, K2) until the pair passes the coprimality rule at every
    unit-circle sample that the recovery will use."""
    make = {"uniform": uniform_kernel, "gaussian": gaussian_perturbed_kernel}[kind]
    for _ in range(max_tries):
        K1, K2 = make(rng, k1), make(rng, k2)
        if is_coprime_pair(K1, K2, sample_counts, tol):
            return K1, K2
    raise RuntimeError("could not draw a coprime kernel pair")


def blur_pair(rng: np.random.Generator, L, K1, K2, noise: float = 0.0):
    """B_c = L (x) K_c + N_e with i.i.d. N(0, noise^2) per pixel, independent
    per stream."""
    B1 = full_conv2d(L, K1)
    B2 = full_conv2d(L, K2)
    if noise > 0:
        B1 = B1 + noise * rng.standard_normal(B1.shape)
        B2 = B2 + noise * rng.standard_normal(B2.shape)
    return B1, B2


# --------------------------------------------------------------------------
# named workloads
# --------------------------------------------------------------------------

def config1(seed: int = 1001):
    """64x64 U[0,1] latent, two coprime 5x5 U(0,1) kernels (sum 1), full
    convolution, no noise; float64.  S = 5, lambda = 0."""
    r = rng_for(seed, 0)
    m = n = 64
    L = uniform_scene(r, m, n)
    K1, K2 = draw_coprime_pair(r, 5, 5, "uniform", sample_counts=(None, 10))
    B1, B2 = blur_pair(r, L, K1, K2, 0.0)
    return dict(name="plain-64x64-k5", L=L, K1=K1, K2=K2, B1=B1, B2=B2,
                m=m, n=n, S=5, lam=0.0, noise=0.0, dtype="f64")


def config2(seed: int = 1002, noise: float = 1e-3, k1: int = 9, k2: int = 11,
            m: int = 480, n: int = 640):
    """480x640 smooth scene (40 anisotropic Gaussians + 0.1 texture), coprime
    9x9 / 11x11 kernels (Gaussian sigma=2 + 0.2 U[0,1), sum 1), additive
    N(0, noise^2).  Frames are returned in float64; cast to float32 for the
    mixed form."""
    r = rng_for(seed, 0)
    L = gaussian_scene(r, m, n)
    K1, K2 = draw_coprime_pair(r, k1, k2, "gaussian", sample_counts=(None, 2 * max(k1, k2)))
    B1, B2 = blur_pair(rng_for(seed, 1), L, K1, K2, noise)
    return dict(name=f"plain-{m}x{n}-k{k1}-k{k2}", L=L, K1=K1, K2=K2, B1=B1, B2=B2,
                m=m, n=n, S=max(k1, k2), lam=(1e-4 if noise > 0 else 0.0),
                noise=noise, dtype="f32")


def config3_frames(seed: int = 1003, nframes: int = 64, m: int = 720, n: int = 1280,
                   noise: float = 1e-3):
    """Moving-blob 720p frames, per-frame coprime pairs of distinct odd sizes
    from 7..15 with U(0,1) entries (sum 1), additive N(0, noise^2)."""
    sizes = np.array([7, 9, 11, 13, 15])
    for f, L in enumerate(blob_sequence(seed, nframes, m, n)):
        r = rng_for(seed, 2, f)
        k1, k2 = r.choice(sizes, 2, replace=False)
        K1, K2 = draw_coprime_pair(r, int(k1), int(k2), "uniform")
        B1, B2 = blur_pair(rng_for(seed, 3, f), L, K1, K2, noise)
        yield dict(L=L, K1=K1, K2=K2, B1=B1, B2=B2, m=m, n=n,
                   S=int(max(k1, k2)), lam=1e-4, noise=noise)



def blob_frame(seed: int, f: int, m: int, n: int, blobs: int = 30, max_shift: int = 4):
    """Frame f of ``blob_sequence`` alone (the random walk is advanced without
    rendering the frames before it), so frames can be made independently."""
    r = rng_for(seed, 0)
    bg = gaussian_scene(r, m, n)
    cy = r.uniform(0, m, blobs)
    cx = r.uniform(0, n, blobs)
    rad = r.uniform(8, 40, blobs)
    amp = r.uniform(-0.5, 0.5, blobs)
    for g in range(1, f + 1):
        rf = rng_for(seed, 1, g)
        cy = np.clip(cy + rf.integers(-max_shift, max_shift + 1, blobs), 0, m - 1)
        cx = np.clip(cx + rf.integers(-max_shift, max_shift + 1, blobs), 0, n - 1)
    yy, xx = np.mgrid[0:m, 0:n].astype(np.float64)
    img = bg.copy()
    for b in range(blobs):
        img += amp[b] * np.exp(-((yy - cy[b]) ** 2 + (xx - cx[b]) ** 2) / (2 * rad[b] ** 2))
    return np.clip(img, 0.0, 1.0)


def config5_frame(f: int, seed: int = 1005, m: int = 1080, n: int = 1920, noise: float = 5e-3,
                  k1: int = 15, k2: int = 17):
    """Frame f of the 1080p colour workload, [channel][y][x]: the moving-blob
    scene scaled by a per-channel gain U(0.6, 1.0) plus 0.05 U[0,1) texture
    per channel, one coprime 15x15 / 17x17 pair (U(0,1) entries, sum 1) for
    every frame, additive N(0, noise^2) per channel and stream."""
    K1, K2 = draw_coprime_pair(rng_for(seed, 5), k1, k2, "uniform")
    gains = rng_for(seed, 6).uniform(0.6, 1.0, 3)
    L = blob_frame(seed, f, m, n)
    Ls = np.stack([g * L + 0.05 * rng_for(seed, 7, f, c).random((m, n)) for c, g in enumerate(gains)])
    B = [blur_pair(rng_for(seed, 8, f, c), Ls[c], K1, K2, noise) for c in range(3)]
    return dict(L=Ls, K1=K1, K2=K2, B1=np.stack([b[0] for b in B]), B2=np.stack([b[1] for b in B]),
                m=m, n=n, S=max(k1, k2), lam=1e-4, noise=noise)


def config5_frames(seed: int = 1005, nframes: int = 8, **kw):
    """Frames 0..nframes-1 of the 1080p colour workload (config5_frame)."""
    for f in range(nframes):
        yield config5_frame(f, seed, **kw)
