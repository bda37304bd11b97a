"""Pins of the oracle against exact arithmetic on a tiny integer case.

The fixture tests/golden/tiny_integer_case.json holds a 4x5 integer latent
and coprime 2x2 / 3x3 integer kernels.  Expected values come from exact
rational (and Gaussian-rational) arithmetic, never from the oracle:
  * eq. 4: gcd(b1, b2) = l up to a constant; the kernels are the cofactors;
  * Sec. 3: the kernels are coprime (both resultants are non-zero);
  * the 2-D system B1 (x) U = B2 (x) V has the one-dimensional null space
    spanned by (K2, K1);
  * at every 4th root of unity, along both axes, the 1-D system
    [C(b1) | -C(b2)] has the one-dimensional null space spanned by the kernel
    slices (Sec. 4: t 1-D GCD sub-problems at unit-circle samples).
"""

import json
import os

import numpy as np
import pytest
import sympy as sp

from oracle import cbp, exact

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def case():
    with open(os.path.join(HERE, "golden", "tiny_integer_case.json")) as f:
        d = json.load(f)
    L = np.array(d["L"], dtype=np.int64)
    K1 = np.array(d["K1"], dtype=np.int64)
    K2 = np.array(d["K2"], dtype=np.int64)
    B1 = exact.exact_blur(L, K1)
    B2 = exact.exact_blur(L, K2)
    return L, K1, K2, B1, B2


def test_gcd_is_latent_and_kernels_coprime(case):
    L, K1, K2, B1, B2 = case
    g, rx, ry = exact.gcd_and_resultants(B1, B2, K1, K2)
    ratio = sp.cancel(exact.to_poly(L).as_expr() / g.as_expr())
    assert ratio.free_symbols == set(), "gcd(b1, b2) must equal l up to a constant"
    assert sp.expand(rx) != 0 and sp.expand(ry) != 0


def test_exact_blur_matches_integer_convolution(case):
    from scipy import signal
    L, K1, K2, B1, B2 = case
    assert np.array_equal(B1.astype(np.int64), signal.convolve2d(L, K1))
    assert np.array_equal(B2.astype(np.int64), signal.convolve2d(L, K2))


def test_2d_null_space_is_the_kernel_pair(case):
    L, K1, K2, B1, B2 = case
    ns = exact.null_space_2d(B1, B2, K1.shape[0], K2.shape[0])
    assert len(ns) == 1
    v = ns[0]
    truth = list(K2.ravel()) + list(K1.ravel())
    # v must be a rational multiple of truth
    c = v[0] / truth[0]
    assert all(sp.simplify(v[i] - c * truth[i]) == 0 for i in range(len(truth)))


@pytest.mark.parametrize("axis", ["x", "y"])
@pytest.mark.parametrize("j", [0, 1, 2, 3])
def test_sample_null_space_exact(case, axis, j):
    L, K1, K2, B1, B2 = case
    k1, k2 = K1.shape[0], K2.shape[0]
    ns = exact.sample_null_space(B1, B2, k1, k2, j, axis)
    assert len(ns) == 1
    truth = exact.kernel_slice_exact(K2, j, axis) + exact.kernel_slice_exact(K1, j, axis)
    v = ns[0]
    piv = next(i for i, t in enumerate(truth) if sp.simplify(t) != 0)
    c = sp.simplify(v[piv] / truth[piv])
    for i, t in enumerate(truth):
        assert sp.simplify(sp.expand(v[i] - c * t)) == 0


@pytest.mark.parametrize("axis", ["x", "y"])
@pytest.mark.parametrize("j", [0, 1, 2, 3])
def test_oracle_null_vector_matches_exact(case, axis, j):
    """O2 + O3 at S = 4 against the exact null vector (up to a complex scale)."""
    L, K1, K2, B1, B2 = case
    k1, k2 = K1.shape[0], K2.shape[0]
    EX1, EY1 = cbp.unit_circle_eval(B1.astype(np.float64), 4)
    EX2, EY2 = cbp.unit_circle_eval(B2.astype(np.float64), 4)
    E1, E2 = (EX1, EX2) if axis == "x" else (EY1, EY2)
    x, spec = cbp.null_vector(cbp.sample_matrix(E1[j], E2[j], k1, k2))
    ex = exact.to_complex(exact.sample_null_space(B1, B2, k1, k2, j, axis)[0])
    cos = abs(np.vdot(ex, x)) / (np.linalg.norm(ex) * np.linalg.norm(x))
    assert cos == pytest.approx(1.0, abs=1e-13)
    assert spec[0] <= 1e-20 * spec[-1]


@pytest.mark.parametrize("S", [3, 4, 7])
def test_oracle_recovers_integer_kernels(case, S):
    L, K1, K2, B1, B2 = case
    R1, R2 = cbp.recover_kernels(B1.astype(np.float64), B2.astype(np.float64), 4, 5, S)
    np.testing.assert_allclose(R1, K1 / K1.sum(), rtol=0, atol=1e-13)
    np.testing.assert_allclose(R2, K2 / K2.sum(), rtol=0, atol=1e-13)


def test_oracle_deconvolution_exact_with_true_kernels(case):
    L, K1, K2, B1, B2 = case
    # kernels normalised to sum 1 scale the latent by the kernel sums
    out = cbp.deconvolve(B1.astype(float), B2.astype(float), K1.astype(float), K2.astype(float), 4, 5, 0.0)
    np.testing.assert_allclose(out, L, rtol=0, atol=1e-12)
