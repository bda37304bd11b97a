"""Pins of the blind kernel-size oracle (oracle/sizes.py; Sec. 4 and Sec. 5:
the kernel degree from the singularity of nested submatrices, after Barnett).

What fixes the expected values here (none comes from the oracle itself):
  * exact arithmetic: at the 4th roots of unity the per-sample system of a
    trial size k has nullity max(0, k - k1 + 1) over Q(i) (SymPy), which is
    the rank statement the test rests on;
  * ground truth: noiseless pairs of known sizes, uneven and even, with the
    default search and the paper's odd 9..25 search;
  * a closed form: a pair sharing a factor f of size kf has cofactors of
    sizes k_c - kf + 1, so the estimate is k1 - kf + 1;
  * invariants: the scores are non-increasing in k (nested Grams,
    eigenvalue interlacing); a range below the truth finds no singular
    candidate, a range above it is singular from its first candidate.
"""

import json
import os

import numpy as np
import pytest

import synth
from oracle import exact, sizes

HERE = os.path.dirname(os.path.abspath(__file__))


def pair(k1, k2, m=40, n=46, noise=0.0, seed=7, kind="uniform"):
    r = synth.rng_for(seed, k1, k2)
    L = synth.uniform_scene(r, m, n)
    K1, K2 = synth.draw_coprime_pair(r, k1, k2, kind)
    return synth.blur_pair(r, L, K1, K2, noise)


def test_exact_nullity_of_trial_sizes():
    """Over Q(i), the trial system of size k at w in {1, -i, -1, i} has nullity
    max(0, k - k1 + 1) (Barnett: rank deficiency = degree of the GCD of the
    cofactor problem), and the oracle's floored score sits at the floor
    exactly where the nullity is positive."""
    g = json.load(open(os.path.join(HERE, "golden", "tiny_integer_case.json")))
    L, K1, K2 = (np.array(g[k], dtype=object) for k in ("L", "K1", "K2"))
    B1, B2 = exact.exact_blur(L, K1), exact.exact_blur(L, K2)
    k1, k2 = K1.shape[0], K2.shape[0]
    d = k1 - k2
    for k in range(1, 5):
        for j in range(4):
            for axis in ("x", "y"):
                ns = exact.sample_null_space(B1, B2, k, k - d, j, axis)
                assert len(ns) == max(0, k - k1 + 1), (k, j, axis)
    cands = sizes.candidates(d, 1, 4)
    s = sizes.size_scores(B1.astype(np.float64), B2.astype(np.float64), cands, 4)
    for ci, k in enumerate(cands):
        at_floor = np.all(s[ci] < sizes.FLOOR)
        assert at_floor == (k >= k1), (k, s[ci])
    e = sizes.estimate_sizes(B1.astype(np.float64), B2.astype(np.float64), 1, 4, 1, 4)
    assert (e["k1"], e["k2"], e["flags"]) == (k1, k2, 0)


@pytest.mark.parametrize("k1,k2", [(5, 5), (7, 5), (4, 9), (3, 3), (12, 11), (2, 1)])
def test_noiseless_sizes_recovered(k1, k2):
    B1, B2 = pair(k1, k2)
    e = sizes.estimate_sizes(B1, B2, 1, 16)
    assert (e["k1"], e["k2"]) == (k1, k2)
    assert e["flags"] == (sizes.FIRST_SINGULAR if k1 == e["candidates"][0] else 0)
    # nested Grams: the scores never increase with the trial size
    assert np.all(np.diff(e["scores"]) <= 1e-9)
    # per sample too, above the rounding floor
    assert np.all(np.diff(np.log10(np.maximum(e["ratios"], sizes.FLOOR)), axis=0) <= 1e-6)


@pytest.mark.parametrize("k", [9, 15, 25])
def test_paper_odd_search(k):
    """The paper's search: odd square sizes 9..25 (Sec. 5)."""
    B1, B2 = pair(k, k, m=30, n=34)
    e = sizes.estimate_sizes(B1, B2, 9, 25, 2)
    assert e["candidates"] == list(range(9, 26, 2))
    assert (e["k1"], e["k2"]) == (k, k)
    assert e["flags"] == (sizes.FIRST_SINGULAR if k == 9 else 0)


def test_shared_factor_gives_the_cofactor_size():
    """K_c = G_c (x) F with a common 3x3 factor F: gcd(b1, b2) = l f, the
    cofactors are G1, G2, so the estimate is k1 - 3 + 1."""
    r = synth.rng_for(3, 1)
    L = synth.uniform_scene(r, 36, 40)
    G1, G2 = synth.draw_coprime_pair(r, 5, 4, "uniform")
    F = synth.uniform_kernel(r, 3)
    K1, K2 = synth.full_conv2d(G1, F), synth.full_conv2d(G2, F)
    B1, B2 = synth.full_conv2d(L, K1), synth.full_conv2d(L, K2)
    e = sizes.estimate_sizes(B1, B2, 1, 12)
    assert (e["k1"], e["k2"]) == (5, 4)


def test_range_without_the_true_size():
    B1, B2 = pair(9, 9, m=30, n=34)
    below = sizes.estimate_sizes(B1, B2, 3, 8)
    assert below["flags"] == sizes.NONE_SINGULAR and below["k1"] == 8
    above = sizes.estimate_sizes(B1, B2, 11, 16)
    assert above["flags"] == sizes.FIRST_SINGULAR and above["k1"] == 11


def test_colour_frames_stack_channels():
    """Three channels with one kernel pair: same sizes; one blank channel does
    not change the decision."""
    r = synth.rng_for(9, 2)
    K1, K2 = synth.draw_coprime_pair(r, 6, 4, "uniform")
    Ls = [synth.uniform_scene(r, 30, 33) for _ in range(3)]
    Ls[1] = np.zeros_like(Ls[1])
    B1 = np.stack([synth.full_conv2d(L, K1) for L in Ls])
    B2 = np.stack([synth.full_conv2d(L, K2) for L in Ls])
    e = sizes.estimate_sizes(B1, B2, 1, 10)
    assert (e["k1"], e["k2"]) == (6, 4)


def test_decision_rule():
    """decide(): largest drop from a virtual 0 before the first candidate,
    first candidate on ties, MIN_DROP threshold and the two flags."""
    c = [3, 4, 5, 6]
    mk = lambda L: np.repeat(10.0 ** np.asarray(L)[:, None, None], 2, axis=1).repeat(3, axis=2)
    k, f, L, D = sizes.decide(c, mk([-1.0, -1.5, -9.0, -9.5]))
    assert (k, f) == (5, 0) and np.allclose(D, [1.0, 0.5, 7.5, 0.5])
    k, f, _, _ = sizes.decide(c, mk([-12.0, -12.5, -13.0, -13.0]))
    assert (k, f) == (3, sizes.FIRST_SINGULAR)
    k, f, _, _ = sizes.decide(c, mk([-0.5, -1.0, -1.5, -2.0]))
    assert (k, f) == (6, sizes.NONE_SINGULAR)
    k, f, _, _ = sizes.decide(c, mk([-1.0, -4.0, -7.0, -7.5]))     # equal drops: the first wins
    assert (k, f) == (4, 0)
    k, f, L, _ = sizes.decide(c, mk([-1.0, -20.0, -30.0, -30.0]))  # scores floor at 1e-13
    assert (k, f) == (4, 0) and L[2] == -13.0
    # the score is the median over samples: one outlier sample does not move it
    s = np.full((3, 2, 3), 0.1)
    s[1] = 10.0 ** -1.5
    s[1, 0, 0] = 1e-13
    s[2] = 1e-4
    k, f, L, D = sizes.decide([3, 4, 5], s)
    assert (k, f) == (5, 0) and np.allclose(L, [-1.0, -1.5, -4.0]) and np.allclose(D, [1.0, 0.5, 2.5])


def test_ratio_is_the_gram_eigenvalue_ratio():
    """s(k) is lambda_min / lambda_max of the Gram A(k)^H A(k), taken here from
    the explicit Gram's eigenvalues (the oracle uses singular values of A)."""
    from oracle import cbp
    B1, B2 = pair(6, 4, m=20, n=24)
    cands = [2, 3, 4, 5]
    S = 5
    s = sizes.size_scores(B1, B2, cands, S)
    E1, E2 = cbp.unit_circle_eval(B1, S), cbp.unit_circle_eval(B2, S)
    for ci, k in enumerate(cands):
        for p in range(2):
            for j in range(S):
                A = cbp.sample_matrix(E1[p][j], E2[p][j], k, k - 2)
                ev = np.linalg.eigvalsh(A.conj().T @ A)
                assert abs(s[ci, p, j] - ev[0] / ev[-1]) <= 1e-12 + 1e-8 * s[ci, p, j]


def test_candidates_and_shape_errors():
    assert sizes.candidates(0, 9, 25, 2) == [9, 11, 13, 15, 17, 19, 21, 23, 25]
    assert sizes.candidates(3, 1, 6) == [4, 5, 6]           # k2 = k - 3 >= 1
    assert sizes.candidates(-2, 30, 40) == [30]             # k2 = k + 2 <= 32
    with pytest.raises(ValueError):
        sizes.size_scores(np.zeros((10, 10)), np.zeros((9, 10)), [2], 4)
