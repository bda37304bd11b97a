"""Pins of the paper-faithful variants (oracle/variants.py).

What fixes the expected values here:
  * ground truth on noiseless pairs: each variant recovers the true kernels
    and the latent exactly (up to rounding) where the paper's method does;
  * library routines and closed forms: the single-channel division at
    lambda = 0 with the true kernel inverts the blur; lambda * L tends to the
    'valid' cross-correlation of B1 with K1 (scipy.signal.correlate2d) as
    lambda grows; the two-channel division of a doubled channel at 2 lambda
    is the single-channel division at lambda;
  * optimality: the k1-only scales minimise kernel 1's scale residual (no
    more than the scales of both kernels do), and are the unit minimiser;
  * the one-axis fix has no equation at S = k1 = k2 (it must refuse) and
    needs only the smaller kernel's support when the sizes differ.
"""

import numpy as np
import pytest
from scipy import signal

import synth
from oracle import cbp, variants


def pair(k1, k2, m=40, n=44, noise=0.0, seed=21, kind="uniform"):
    r = synth.rng_for(seed, k1, k2)
    L = synth.uniform_scene(r, m, n)
    K1, K2 = synth.draw_coprime_pair(r, k1, k2, kind, sample_counts=(None, max(k1, k2) + 1))
    B1, B2 = synth.blur_pair(r, L, K1, K2, noise)
    return L, K1, K2, B1, B2


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def test_single_division_inverts_with_the_true_kernel():
    L, K1, K2, B1, B2 = pair(5, 7)
    Lr = variants.deconvolve_single(B1, B2, K1, 40, 44, 0.0)
    assert np.max(np.abs(Lr - L)) < 1e-8


def test_single_division_limits_and_two_channel_relation():
    L, K1, K2, B1, B2 = pair(5, 5, noise=1e-3)
    lam = 1e9
    Lr = variants.deconvolve_single(B1, B2, K1, 40, 44, lam)
    corr = signal.correlate2d(B1, K1, mode="valid")
    assert corr.shape == (40, 44)
    assert rel(lam * Lr, corr) < 1e-6
    # a doubled channel: (2 conj K B) / (2 |K|^2 + 2 lam) = single(lam)
    for lam in (0.0, 1e-3, 0.5):
        two = cbp.deconvolve(B1, B1, K1, K1, 40, 44, 2 * lam)
        one = variants.deconvolve_single(B1, B1, K1, 40, 44, lam)
        assert np.max(np.abs(two - one)) <= 1e-12 * max(1.0, np.max(np.abs(one)))


@pytest.mark.parametrize("k1,k2", [(5, 5), (7, 4), (3, 6)])
def test_k1_only_scales_recover_the_kernels(k1, k2):
    L, K1, K2, B1, B2 = pair(k1, k2)
    R1, R2 = variants.recover_kernels(B1, B2, 40, 44, 0, "k1")
    assert rel(R1, K1) < 1e-8 and rel(R2, K2) < 1e-8
    Ld, D1, D2 = variants.deblur(B1, B2, 40, 44, 0, 0.0, "k1", "single")
    assert np.max(np.abs(Ld - L)) < 1e-6


def test_k1_only_scales_minimise_kernel_1_rows():
    L, K1, K2, B1, B2 = pair(6, 5, noise=1e-2)
    _, _, full = cbp.recover_kernels(B1, B2, 40, 44, 0, full=True)
    P, Q = full["P"], full["Q"]
    a1, b1, _ = variants.scale_fix_k1(P, Q)
    M1 = cbp.scale_system(P[:1], Q[:1])
    z1 = np.concatenate([a1, b1])
    zb = np.concatenate([full["a"], full["b"]])
    r1 = np.linalg.norm(M1 @ z1)
    assert abs(np.linalg.norm(z1) - 1.0) < 1e-12
    assert r1 <= np.linalg.norm(M1 @ zb) * (1 + 1e-12)
    # the minimiser: its squared residual is the smallest eigenvalue of M1^H M1
    ev = np.linalg.eigvalsh(M1.conj().T @ M1)
    assert abs(r1 ** 2 - ev[0]) <= 1e-9 * ev[-1]


@pytest.mark.parametrize("k1,k2,S", [(5, 5, 6), (4, 4, 8), (7, 5, 7), (5, 7, 7), (6, 3, 7)])
def test_one_axis_scale_fix_recovers_the_kernels(k1, k2, S):
    L, K1, K2, B1, B2 = pair(k1, k2)
    R1, R2 = variants.recover_kernels(B1, B2, 40, 44, S, "one_axis")
    assert rel(R1, K1) < 1e-8 and rel(R2, K2) < 1e-8
    # the equations hold: no energy outside the supports
    EX1, _ = cbp.unit_circle_eval(B1, S)
    EX2, _ = cbp.unit_circle_eval(B2, S)
    XU, XV, _ = cbp.sample_cofactors(EX1, EX2, k1, k2)
    a, _ = cbp.null_vector(variants.one_axis_system(XU, XV, k1, k2, S))
    _, d1 = variants.one_axis_kernel(XV, a, k1)
    _, d2 = variants.one_axis_kernel(XU, a, k2)
    assert d1["outside"] < 1e-20 and d2["outside"] < 1e-20 and d1["imag"] < 1e-8


def test_one_axis_needs_an_extra_sample_for_equal_sizes():
    L, K1, K2, B1, B2 = pair(5, 5)
    with pytest.raises(ValueError):
        variants.recover_kernels(B1, B2, 40, 44, 5, "one_axis")


def test_variants_agree_with_the_default_method_noiselessly():
    L, K1, K2, B1, B2 = pair(6, 4)
    D1, D2 = cbp.recover_kernels(B1, B2, 40, 44, 7)
    for scale in ("k1", "one_axis"):
        R1, R2 = variants.recover_kernels(B1, B2, 40, 44, 7, scale)
        assert rel(R1, D1) < 1e-8 and rel(R2, D2) < 1e-8
    with pytest.raises(ValueError):
        variants.recover_kernels(B1, B2, 40, 44, 7, "nope")


def test_normalisation_on_noisy_frames():
    """Each variant divides by the complex sum over the kernel's support: the
    kernels sum to 1 whatever the noise (Sec. 5: normalisation)."""
    L, K1, K2, B1, B2 = pair(5, 4, noise=1e-2)
    for scale, S in (("k1", 0), ("one_axis", 6)):
        R1, R2 = variants.recover_kernels(B1, B2, 40, 44, S, scale)
        assert abs(R1.sum() - 1.0) < 1e-12 and abs(R2.sum() - 1.0) < 1e-12
