"""The CBP encoder and the multi-level streams in plain Python / NumPy -- the oracle.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Encoder (Sec. 3, blur kernel selection; Sec. 4 eq. 1 without the sensor
noise): every captured frame L is blurred by two random kernels that are
coprime as bivariate polynomials, a new pair per frame, into the public
stream B1 = L (x) K1 and the private stream B2 = L (x) K2 (full linear
convolution, each channel alike).

Random kernels.  The draws come from the counter-based generator
Philox4x64-10 (Salmon, Moraes, Dror and Shaw, "Parallel random numbers: as
easy as 1, 2, 3", SC 2011): ten rounds of
    (c0, c1, c2, c3) <- (hi(M1 c2) ^ c1 ^ k0, lo(M1 c2), hi(M0 c0) ^ c3 ^ k1, lo(M0 c0))
with M0 = 0xD2E7470EE14C6C93, M1 = 0xCA5A826395121157 and the key bumped by
(0x9E3779B97F4A7C15, 0xBB67AE8584CAA73B) between rounds.  Readings taken
here (the paper only says the kernels are constructed at random, large and
new for every frame):
  * entry e (row-major [y][x]) of kernel s in {1, 2} of frame f, draw
    attempt a, uses word e mod 4 of Philox(counter = (e div 4, s, a, 0),
    key = (seed, f)); u_e = ((word >> 11) + 1/2) 2^-53 in (0, 1);
  * K_s = u / sum(u), the sum taken in entry order;
  * coprimality (Sec. 3): the pair is redrawn (a + 1) while at some sample
    w_j (j < S, both evaluation orders) the Sylvester system of the two
    kernel slices, [C_{k2-1}(p) | -C_{k1-1}(q)] with p = k1(w_j, .) and
    q = k2(w_j, .) (or k1(., w_j), k2(., w_j)), has
    lambda_min / lambda_max of its Gram below SYLV_MIN = 1e-12 (the
    slices then nearly share a root); at most MAX_ATTEMPTS attempts.

Multi-level security (Sec. 3): a level sees the 8-bit streams with its b
least significant bits removed.  Readings: q = clamp(rint(255 B), 0, 255)
in the frame's precision (round half to even), level b keeps
q & (255 << b) & 255, and the receiver reads q / 255.
"""

from __future__ import annotations

import numpy as np

M0 = 0xD2E7470EE14C6C93
M1 = 0xCA5A826395121157
W0 = 0x9E3779B97F4A7C15
W1 = 0xBB67AE8584CAA73B
MASK64 = (1 << 64) - 1
SYLV_MIN = 1e-12
MAX_ATTEMPTS = 64


def philox4x64(counter, key):
    """Philox4x64-10 of a 4-word counter and a 2-word key (Python integers)."""
    c = [int(v) & MASK64 for v in counter]
    k = [int(v) & MASK64 for v in key]
    for r in range(10):
        if r:
            k = [(k[0] + W0) & MASK64, (k[1] + W1) & MASK64]
        p0 = M0 * c[0]
        p1 = M1 * c[2]
        c = [((p1 >> 64) ^ c[1] ^ k[0]) & MASK64, p1 & MASK64, ((p0 >> 64) ^ c[3] ^ k[1]) & MASK64, p0 & MASK64]
    return c


def kernel_draw(seed: int, frame: int, stream: int, attempt: int, k: int) -> np.ndarray:
    """One k x k kernel of entries in (0, 1) normalised to sum 1 (entry order)."""
    u = np.empty(k * k)
    for e in range(k * k):
        w = philox4x64((e // 4, stream, attempt, 0), (seed, frame))[e % 4]
        u[e] = ((w >> 11) + 0.5) * 2.0 ** -53
    s = 0.0
    for e in range(k * k):
        s += u[e]
    return (u / s).reshape(k, k)


def sylvester_ratios(K1: np.ndarray, K2: np.ndarray, S: int) -> np.ndarray:
    """lambda_min / lambda_max of the Sylvester Gram of the kernel slices at
    every sample [pass][j] (1 where a slice pair has no Sylvester matrix)."""
    k1, k2 = K1.shape[0], K2.shape[0]
    out = np.ones((2, S))
    for p in range(2):
        for j in range(S):
            w1 = np.exp(-2j * np.pi * ((j * np.arange(k1)) % S) / S)
            w2 = np.exp(-2j * np.pi * ((j * np.arange(k2)) % S) / S)
            a, b = (w1 @ K1, w2 @ K2) if p == 0 else (K1 @ w1, K2 @ w2)
            n = (k1 - 1) + (k2 - 1)
            if n == 0:
                continue
            A = np.zeros((n, n), dtype=np.complex128)
            for c in range(k2 - 1):          # C_{k2-1}(a): a shifted down by c
                A[c:c + k1, c] = a
            for c in range(k1 - 1):          # -C_{k1-1}(b)
                A[c:c + k2, k2 - 1 + c] = -b
            ev = np.linalg.eigvalsh(A.conj().T @ A)
            out[p, j] = max(ev[0], 0.0) / ev[-1] if ev[-1] > 0 else 0.0
    return out


def draw_pair(seed: int, frame: int, k1: int, k2: int, S: int = 0):
    """(K1, K2, attempt) of frame f: the first attempt whose pair passes the
    coprimality rule; attempt = -1 (and the last draw) when none of
    MAX_ATTEMPTS does."""
    S = S or max(k1, k2)
    for a in range(MAX_ATTEMPTS):
        K1 = kernel_draw(seed, frame, 1, a, k1)
        K2 = kernel_draw(seed, frame, 2, a, k2)
        if np.min(sylvester_ratios(K1, K2, S)) > SYLV_MIN:
            return K1, K2, a
    return K1, K2, -1


def blur(L: np.ndarray, K: np.ndarray) -> np.ndarray:
    """Full linear convolution B[y, x] = sum_{a, b} L[y - a, x - b] K[a, b]
    (eq. 1 without noise), by shifted sums of the whole latent; colour
    frames [channel][y][x] channel by channel."""
    L = np.asarray(L)
    if L.ndim == 3:
        return np.stack([blur(L[c], K) for c in range(L.shape[0])])
    m, n = L.shape
    k = K.shape[0]
    B = np.zeros((m + k - 1, n + k - 1), dtype=np.result_type(L.dtype, np.float64))
    for a in range(k):
        for b in range(k):
            B[a:a + m, b:b + n] += K[a, b] * L
    return B


def quantize(B: np.ndarray, drop_bits: int = 0) -> np.ndarray:
    """8-bit stream of a level that lacks the drop_bits least significant bits:
    clamp(rint(255 B), 0, 255) & (255 << drop_bits), computed in B's precision."""
    B = np.asarray(B)
    q = np.clip(np.rint(B * B.dtype.type(255)), 0, 255).astype(np.uint8)
    return (q & np.uint8((0xFF << drop_bits) & 0xFF)).astype(np.uint8)


def dequantize(q: np.ndarray, dtype=np.float32) -> np.ndarray:
    """The receiver's frame q / 255 in `dtype`."""
    return (np.asarray(q).astype(dtype) / dtype(255)).astype(dtype)
