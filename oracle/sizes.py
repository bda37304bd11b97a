"""Blind kernel-size estimation in plain FP64 NumPy -- the oracle.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper's first stage (Sec. 4, Sec. 5 and the "kernel degree estimation"
row of Table 1) finds the kernel size from the singularity of nested leading
submatrices built from the frames' unit-circle samples (after Barnett: the
rank deficiency of a Bezout matrix is the degree of the GCD).  The paper's
own matrices and its text about them are not recoverable, so this module
takes the equivalent test on the per-sample systems the recovery already
uses.

When the latent size is unknown only the difference d = H1 - H2 = W1 - W2 =
k1 - k2 is known.  For a trial size k (k1' = k, k2' = k - d) and a sample w
of either pass, the 1-D system

    A(k) = [C_{k-d}(e1) | -C_k(e2)],   e_c = b_c evaluated at w,

has a null vector exactly when b1 u = b2 v has a solution with u of k - d
taps and v of k taps.  Since b1 = l k1 and b2 = l k2 with coprime slices,
every solution is (u, v) = (k2 s, k1 s) for a polynomial s, so the nullity
of A(k) is max(0, k - k1 + 1): zero below the true size, one at it, growing
above it.  The test per trial size is the relative smallest eigenvalue of
the Gram matrix,

    s(k) = lambda_min(A(k)^H A(k)) / lambda_max(A(k)^H A(k))
         = (sigma_min(A(k)) / sigma_max(A(k)))^2,

which is non-increasing in k (the Grams are nested principal submatrices of
one Gram, so eigenvalue interlacing applies) and falls to the rounding /
noise level at the true size.  Readings taken here (the paper is silent):

  * both passes, S samples each (w_j = exp(-2 pi i j / S)); colour frames
    stack the channels' matrices, as the recovery does;
  * per candidate, the score L(k) = median over the 2S samples of
    log10(max(s(k), FLOOR)), FLOOR = 1e-13 (above the ~1e-16 rounding level
    of any FP64 Gram, so two valid evaluation orders give the same floored
    score);
  * the estimate is the candidate with the largest drop
    D(k_c) = L(k_{c-1}) - L(k_c), with L(k_{-1}) = 0 (a perfectly
    conditioned system) for the first candidate; the first such candidate
    wins a tie;
  * a largest drop below MIN_DROP = 2 decades means no candidate made the
    system singular (the true size lies above the search range): the
    estimate is then the largest candidate and flag NONE_SINGULAR is set; a
    winning first candidate sets FIRST_SINGULAR (the true size may lie below
    the range);
  * candidates: k = kmin, kmin + step, ..., <= kmax with 1 <= k - d and both
    sizes <= 32.  The paper's own search is odd sizes 9..25 (Sec. 5):
    kmin = 9, kmax = 25, step = 2.
"""

from __future__ import annotations

import numpy as np

from .cbp import MAX_K, sample_matrix, unit_circle_eval

FLOOR = 1e-13
MIN_DROP = 2.0
NONE_SINGULAR = 1
FIRST_SINGULAR = 2


def candidates(d: int, kmin: int, kmax: int, step: int = 1):
    """Trial sizes k1' (k2' = k1' - d) of a search, ascending."""
    out = []
    for k in range(max(1, kmin), kmax + 1, max(1, step)):
        if 1 <= k - d and k <= MAX_K and k - d <= MAX_K:
            out.append(k)
    return out


def size_scores(B1, B2, cands, S: int):
    """s(k) for every candidate, pass and sample: array [cand][pass][sample]."""
    B1 = np.asarray(B1, dtype=np.float64)
    B2 = np.asarray(B2, dtype=np.float64)
    if B1.ndim == 2:
        B1, B2 = B1[None], B2[None]
    d = B1.shape[1] - B2.shape[1]
    if B1.shape[2] - B2.shape[2] != d:
        raise ValueError("H1 - H2 must equal W1 - W2")
    ev1 = [unit_circle_eval(B1[c], S) for c in range(B1.shape[0])]
    ev2 = [unit_circle_eval(B2[c], S) for c in range(B2.shape[0])]
    s = np.zeros((len(cands), 2, S))
    for ci, k in enumerate(cands):
        for p in range(2):
            for j in range(S):
                A = np.vstack([sample_matrix(ev1[c][p][j], ev2[c][p][j], k, k - d) for c in range(len(ev1))])
                sv = np.linalg.svd(A, compute_uv=False)
                s[ci, p, j] = (sv[-1] / sv[0]) ** 2
    return s


def decide(cands, s):
    """Scores L(k), drops D(k) and the decision (k1, flags) from s[cand][pass][sample]."""
    L = np.array([float(np.median(np.log10(np.maximum(s[c].ravel(), FLOOR)))) for c in range(len(cands))])
    prev = np.concatenate([[0.0], L[:-1]])
    D = prev - L
    c = int(np.argmax(D))
    flags = 0
    if D[c] < MIN_DROP:
        c = len(cands) - 1
        flags |= NONE_SINGULAR
    elif c == 0:
        flags |= FIRST_SINGULAR
    return cands[c], flags, L, D


def estimate_sizes(B1, B2, kmin: int = 1, kmax: int = MAX_K, step: int = 1, S: int = 0):
    """Blind (k1, k2) of a blurred pair: the nullity test above over the
    candidate sizes.  S = 0 uses S = the largest candidate.  Returns a dict
    with k1, k2, flags, the candidates, their scores L and drops D, and the
    per-sample ratios s."""
    B1 = np.asarray(B1)
    B2 = np.asarray(B2)
    d = B1.shape[-2] - B2.shape[-2]
    cands = candidates(d, kmin, kmax, step)
    H = min(B1.shape[-2], B2.shape[-2])
    W = min(B1.shape[-1], B2.shape[-1])
    cands = [k for k in cands if k <= H + max(d, 0) and k <= W + max(d, 0)]
    if not cands:
        raise ValueError("no candidate size fits the frames")
    S = S or max(cands)
    s = size_scores(B1, B2, cands, S)
    k1, flags, L, D = decide(cands, s)
    return dict(k1=k1, k2=k1 - d, flags=flags, candidates=cands, scores=L, drops=D, ratios=s, S=S)
