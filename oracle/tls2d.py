"""Independent route to the kernels: the 2-D null space, by brute force.

TEST INFRASTRUCTURE ONLY.

For coprime kernels of full bidegree, (K2, K1) spans the one-dimensional
null space of the 2-D system  B1 (x) U - B2 (x) V = 0  with supp U = k2 x k2
and supp V = k1 x k1 (eq. 4: b1 k2 = l k1 k2 = b2 k1, and k1 u = k2 v with
k1, k2 coprime forces u = c k2).  This module solves that system directly,
without the per-sample decomposition of Sec. 4, as a cross-check of the
whole method on noiseless inputs.
"""

from __future__ import annotations

import numpy as np
from scipy import signal


def system_matrix(B1: np.ndarray, B2: np.ndarray, k1: int, k2: int) -> np.ndarray:
    """Explicit matrix of (U, V) -> B1 (x) U - B2 (x) V, columns ordered as
    U row-major then V row-major.  Only for small frames."""
    H1, W1 = B1.shape
    Ho, Wo = H1 + k2 - 1, W1 + k2 - 1
    cols = []
    for B, k, sign in ((B1, k2, 1.0), (B2, k1, -1.0)):
        H, W = B.shape
        for p in range(k):
            for q in range(k):
                img = np.zeros((Ho, Wo))
                img[p:p + H, q:q + W] = sign * B
                cols.append(img.ravel())
    return np.stack(cols, axis=1)


def gram_matrix(B1: np.ndarray, B2: np.ndarray, k1: int, k2: int) -> np.ndarray:
    """A^T A of ``system_matrix`` from 2-D auto/cross-correlations, so that
    mid-size frames fit in memory.  Entry for shifts s=(p,q), s'=(p',q'):
    sum_t X[t - s] Y[t - s'] = corr_{X,Y}(s - s')."""
    def corr(X, Y, kx, ky):
        # C[dy, dx] = sum_t X[t] Y[t + d] for d in [-(kx-1), ky-1]^2
        full = signal.correlate(Y, X, mode="full", method="fft")
        cy, cx = X.shape[0] - 1, X.shape[1] - 1
        return full, cy, cx

    blocks = []
    specs = ((B1, k2, 1.0), (B2, k1, -1.0))
    for Xa, ka, sa in specs:
        row = []
        for Xb, kb, sb in specs:
            full, cy, cx = corr(Xa, Xb, ka, kb)
            G = np.zeros((ka * ka, kb * kb))
            for p in range(ka):
                for q in range(ka):
                    for pp in range(kb):
                        for qq in range(kb):
                            # sum_t Xa[t-(p,q)] Xb[t-(pp,qq)] = sum_u Xa[u] Xb[u + (p-pp, q-qq)]
                            G[p * ka + q, pp * kb + qq] = full[cy + p - pp, cx + q - qq]
            row.append(sa * sb * G)
        blocks.append(row)
    return np.block(blocks)


def recover_kernels_2d(B1, B2, k1: int, k2: int, explicit: bool | None = None):
    """(K1, K2) normalised to sum 1 from the smallest singular vector of the
    2-D system (explicit SVD for small frames, Gram eigenvector otherwise)."""
    B1 = np.asarray(B1, dtype=np.float64)
    B2 = np.asarray(B2, dtype=np.float64)
    if explicit is None:
        explicit = B1.size * (k1 * k1 + k2 * k2) <= 4_000_000
    if explicit:
        _, s, Vh = np.linalg.svd(system_matrix(B1, B2, k1, k2), full_matrices=False)
        z = Vh[-1]
        spec = s[::-1] ** 2
    else:
        w, v = np.linalg.eigh(gram_matrix(B1, B2, k1, k2))
        z, spec = v[:, 0], w
    U = z[:k2 * k2].reshape(k2, k2)
    V = z[k2 * k2:].reshape(k1, k1)
    return V / V.sum(), U / U.sum(), spec
