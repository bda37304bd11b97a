"""Paper-faithful variants of the method in plain FP64 NumPy -- the oracle.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The default method (oracle/cbp.py) takes readings where the paper's text is
thin; the paper itself describes, or implies, these narrower steps:

  * single-channel division (Sec. 4: the latent is obtained by dividing the
    blurred frame B1 by the kernel K1 in the Fourier domain; Sec. 5: one frame
    of the pair is deblurred by inverse FFT):
        Lhat = conj(K1hat) B1hat / (|K1hat|^2 + lambda)
    on the same Py x Px grid as the two-channel division (the smallest
    7-smooth sizes covering both frames);
  * the k1-only scale least squares (Sec. 5: the scale factors come from
    the two estimates of k1 alone -- 2t unknowns over t x t equations): the
    scale system of oracle/cbp.py restricted to kernel 1's rows; both kernels
    are then assembled with those scales (the scales belong to the
    per-sample null vectors, which hold both cofactors);
  * the one-axis scale fix (a reading: the per-sample scales of ONE
    evaluation order fixed by the kernel's finite support instead of by the
    second order).  With pass-X null vectors X_j (slices of the kernels at
    sample w_j, each scaled by an unknown c_j) and a_j = 1 / c_j,
        K_c[y, x] = (1/S) sum_j a_j X^c_j[x] w_j^{-y},   y < S,
    must vanish for k_c <= y < S.  These k_c (S - k_c) equations per kernel
    can fix a up to one factor only when there are at least S - 1 of them
    (at S = k1 = k2 there are none; the fix then refuses); a is the smallest
    right singular vector of the stacked
    equations and K_c is the real part of the expression above on its
    support, divided by its complex sum.
"""

from __future__ import annotations

import numpy as np

from . import cbp


def deconvolve_single(B1, B2, K1, m: int, n: int, lam: float = 0.0):
    """L = crop_{m x n} IFFT2( conj(Kh1) Bh1 / (|Kh1|^2 + lam) ) on the grid
    Py = smooth7(max H_c), Px = smooth7(max W_c) (B2 only sizes the grid).
    Colour frames are divided channel by channel."""
    B1 = np.asarray(B1, dtype=np.float64)
    B2 = np.asarray(B2)
    if B1.ndim == 3:
        return np.stack([deconvolve_single(B1[c], B2[c], K1, m, n, lam) for c in range(B1.shape[0])])
    Py = cbp.smooth7(max(B1.shape[0], B2.shape[0]))
    Px = cbp.smooth7(max(B1.shape[1], B2.shape[1]))
    Bh1 = np.fft.fft2(B1, s=(Py, Px))
    Kh1 = np.fft.fft2(K1, s=(Py, Px))
    Lh = np.conj(Kh1) * Bh1 / (np.abs(Kh1) ** 2 + lam)
    return np.real(np.fft.ifft2(Lh))[:m, :n]


def scale_fix_k1(P, Q):
    """(a, b) from kernel 1's rows of the scale system only (Sec. 5)."""
    z, spec = cbp.null_vector(cbp.scale_system(P[:1], Q[:1]))
    S = P[0].shape[0]
    return z[:S], z[S:], spec


def one_axis_system(XU, XV, k1: int, k2: int, S: int) -> np.ndarray:
    """Rows (kernel c, x < k_c, k_c <= y < S) of M a = 0, M[row, j] =
    X^c_j[x] w_j^{-y} (kernel 1: the V parts, kernel 2: the U parts)."""
    rows = []
    for X, k in ((XV, k1), (XU, k2)):
        for x in range(k):
            for y in range(k, S):
                rows.append(X[:, x] * np.exp(2j * np.pi * ((np.arange(S) * y) % S) / S))
    if len(rows) < S - 1:
        raise ValueError("the one-axis scale fix needs at least S - 1 support equations "
                         "(S >= max(k1, k2) + 1 when k1 = k2)")
    return np.array(rows)


def one_axis_kernel(X, a, k: int):
    """K[y, x] = Re( F[y, x] / sum_{y,x<k} F ), F[y, x] = (1/S) sum_j a_j X_j[x] w_j^{-y}
    for y < S, x < k; also the energy fraction of F outside y < k."""
    S = X.shape[0]
    Winv = np.exp(2j * np.pi * (np.outer(np.arange(S), np.arange(S)) % S) / S)   # [y, j] = w_j^{-y}
    F = Winv @ (a[:, None] * X[:, :k]) / S                                      # [y, x]
    Fc = F[:k]
    s = Fc.sum()
    out = (np.sum(np.abs(F) ** 2) - np.sum(np.abs(Fc) ** 2)) / max(np.sum(np.abs(F) ** 2), 1e-300)
    Kn = Fc / s
    return np.real(Kn), dict(outside=float(out),
                             imag=float(np.linalg.norm(Kn.imag) / max(np.linalg.norm(Kn.real), 1e-300)))


def recover_kernels(B1, B2, m: int, n: int, S: int = 0, scale: str = "both"):
    """Kernels by the default steps (O1-O4) with the scale fix `scale`:
    "both" (oracle/cbp.py), "k1" (kernel 1's rows only) or "one_axis"
    (pass X only, fixed by the kernels' support; S >= max k + 1)."""
    if scale == "both":
        return cbp.recover_kernels(B1, B2, m, n, S)
    B1 = np.asarray(B1)
    B2 = np.asarray(B2)
    k1, k2 = cbp.kernel_sizes(B1.shape[-2:], B2.shape[-2:], m, n)
    S = S or max(k1, k2)
    if S < max(k1, k2):
        raise ValueError("S must be >= max kernel size")
    if B1.ndim == 3:
        ev1 = [cbp.unit_circle_eval(B1[c], S) for c in range(B1.shape[0])]
        ev2 = [cbp.unit_circle_eval(B2[c], S) for c in range(B2.shape[0])]
        EX1, EY1 = np.stack([e[0] for e in ev1]), np.stack([e[1] for e in ev1])
        EX2, EY2 = np.stack([e[0] for e in ev2]), np.stack([e[1] for e in ev2])
    else:
        EX1, EY1 = cbp.unit_circle_eval(B1, S)
        EX2, EY2 = cbp.unit_circle_eval(B2, S)
    XU, XV, _ = cbp.sample_cofactors(EX1, EX2, k1, k2)
    if scale == "one_axis":
        a, _ = cbp.null_vector(one_axis_system(XU, XV, k1, k2, S))
        K1, _ = one_axis_kernel(XV, a, k1)
        K2, _ = one_axis_kernel(XU, a, k2)
        return K1, K2
    if scale != "k1":
        raise ValueError(f"unknown scale fix {scale!r}")
    YU, YV, _ = cbp.sample_cofactors(EY1, EY2, k1, k2)
    P, Q = cbp.cofactor_grids(XU, XV, YU, YV, S)
    a, b, _ = scale_fix_k1(P, Q)
    K1, _ = cbp.assemble_kernel(P[0], Q[0], a, b, k1)
    K2, _ = cbp.assemble_kernel(P[1], Q[1], a, b, k2)
    return K1, K2


def deblur(B1, B2, m: int, n: int, S: int = 0, lam: float = 0.0, scale: str = "both",
           division: str = "two"):
    """Latent and kernels with the chosen scale fix and division ("two":
    oracle/cbp.py's two-channel division; "single": B1 / K1)."""
    K1, K2 = recover_kernels(B1, B2, m, n, S, scale)
    if division == "single":
        L = deconvolve_single(B1, B2, K1, m, n, lam)
    elif division == "two":
        L = cbp.deconvolve(B1, B2, K1, K2, m, n, lam)
    else:
        raise ValueError(f"unknown division {division!r}")
    return L, K1, K2
