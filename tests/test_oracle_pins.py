"""Pins of the FP64 oracle against things other than itself.

  * O2 against Horner evaluation (numpy.polynomial.polynomial.polyval) and
    the closed forms at S = 1 and S = 2;
  * C_k(e) u against numpy.convolve;
  * O3 against the smallest eigenvector of the explicit Gram matrix (eigh)
    and against the ground-truth kernel slices;
  * O4-O6 against ground truth: per-sample scales, the scale-fix null
    vector, kernel invariants;
  * O7 against the exact inverse with true kernels, the lambda -> infinity
    limit and the single-channel inverse filter;
  * the whole method against ground truth and against the brute-force 2-D
    null space (oracle.tls2d);
  * the non-coprime case, where every per-sample null space has dimension
    >= 2.
Ground truth comes from the seeded generator (synth), which draws L, K1, K2
and forms B = L (x) K; it holds no step of the method.
"""

import numpy as np
import pytest
from numpy.polynomial import polynomial as npoly

import synth
from oracle import cbp, tls2d


def rel(a, b):
    return np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b))


@pytest.fixture(scope="module")
def c1():
    return synth.config1()


# ---------------------------------------------------------------- O1 / grid

def test_smooth7_is_smallest_7_smooth():
    def smooth(v):
        for p in (2, 3, 5, 7):
            while v % p == 0:
                v //= p
        return v == 1
    for n in range(1, 2200):
        s = cbp.smooth7(n)
        assert s >= n and smooth(s)
        assert not any(smooth(v) for v in range(n, s))


def test_kernel_sizes_and_errors():
    assert cbp.kernel_sizes((68, 70), (70, 72), 64, 66) == (5, 7)
    with pytest.raises(ValueError):
        cbp.kernel_sizes((68, 71), (70, 72), 64, 66)
    with pytest.raises(ValueError):
        cbp.kernel_sizes((64 + 32, 66 + 32), (70, 72), 64, 66)


# ---------------------------------------------------------------- O2

@pytest.mark.parametrize("S", [1, 2, 5, 11, 32])
def test_unit_circle_eval_matches_horner(S):
    r = np.random.default_rng(5)
    B = r.random((23, 17))
    EX, EY = cbp.unit_circle_eval(B, S)
    for j in range(S):
        w = np.exp(-2j * np.pi * j / S)
        for x in range(B.shape[1]):
            assert EX[j, x] == pytest.approx(npoly.polyval(w, B[:, x]), abs=1e-12)
        for y in range(B.shape[0]):
            assert EY[j, y] == pytest.approx(npoly.polyval(w, B[y, :]), abs=1e-12)


def test_unit_circle_eval_closed_forms():
    r = np.random.default_rng(6)
    B = r.random((9, 8))
    EX, EY = cbp.unit_circle_eval(B, 1)
    np.testing.assert_allclose(EX[0], B.sum(axis=0), atol=1e-14)
    np.testing.assert_allclose(EY[0], B.sum(axis=1), atol=1e-14)
    EX, EY = cbp.unit_circle_eval(B, 2)
    sgn = (-1.0) ** np.arange(9)
    np.testing.assert_allclose(EX[1], sgn @ B, atol=1e-13)
    np.testing.assert_allclose(EY[1], B @ ((-1.0) ** np.arange(8)), atol=1e-13)


# ---------------------------------------------------------------- O3

def test_conv_matrix_is_convolution():
    r = np.random.default_rng(7)
    e = r.standard_normal(13) + 1j * r.standard_normal(13)
    u = r.standard_normal(4) + 1j * r.standard_normal(4)
    np.testing.assert_allclose(cbp.conv_matrix(e, 4) @ u, np.convolve(e, u), atol=1e-13)


def test_null_vector_matches_gram_eigh(c1):
    EX1, _ = cbp.unit_circle_eval(c1["B1"], 5)
    EX2, _ = cbp.unit_circle_eval(c1["B2"], 5)
    for j in range(5):
        A = cbp.sample_matrix(EX1[j], EX2[j], 5, 5)
        x, spec = cbp.null_vector(A)
        w, v = np.linalg.eigh(A.conj().T @ A)
        assert abs(np.vdot(v[:, 0], x)) == pytest.approx(1.0, abs=1e-9)
        np.testing.assert_allclose(spec[1:], w[1:], rtol=1e-9)


def _truth_slices(K, S, axis):
    """k(w_j, .) (axis 'x') or k(., w_i) (axis 'y') for all samples, by direct sums."""
    k = K.shape[0]
    out = np.zeros((S, k), dtype=complex)
    for j in range(S):
        w = np.exp(-2j * np.pi * j / S) ** np.arange(k)
        out[j] = (w @ K) if axis == "x" else (K @ w)
    return out


@pytest.mark.parametrize("axis", ["x", "y"])
def test_cofactors_are_kernel_slices_with_one_scale(c1, axis):
    """u_j = c_j k2(w_j, .) and v_j = c_j k1(w_j, .) with the SAME c_j."""
    K1, K2, full = cbp.recover_kernels(c1["B1"], c1["B2"], 64, 64, 5, full=True)
    U, V = (full["XU"], full["XV"]) if axis == "x" else (full["YU"], full["YV"])
    t1 = _truth_slices(c1["K1"], 5, axis)
    t2 = _truth_slices(c1["K2"], 5, axis)
    for j in range(5):
        cu = U[j] / t2[j]
        cv = V[j] / t1[j]
        np.testing.assert_allclose(cu, cu[0], rtol=1e-11)
        np.testing.assert_allclose(cv, cu[0], rtol=1e-11)


def test_non_coprime_pair_has_degenerate_samples():
    r = synth.rng_for(77, 0)
    L = r.random((20, 24))
    K1 = r.random((3, 3))
    f = r.random((2, 2)) + 0.5
    K2 = synth.full_conv2d(K1, f)           # K2 = K1 (x) f shares the factor K1
    B1, B2 = synth.full_conv2d(L, K1), synth.full_conv2d(L, K2)
    EX1, _ = cbp.unit_circle_eval(B1, 4)
    EX2, _ = cbp.unit_circle_eval(B2, 4)
    for j in range(4):
        _, spec = cbp.null_vector(cbp.sample_matrix(EX1[j], EX2[j], 3, 4))
        assert spec[1] <= 1e-20 * spec[-1]        # nullity >= 2 (it is k1 = 3)


# ---------------------------------------------------------------- O4-O6

def test_scale_fix_inverts_per_sample_scales(c1):
    K1, K2, full = cbp.recover_kernels(c1["B1"], c1["B2"], 64, 64, 5, full=True)
    t1x = _truth_slices(c1["K1"], 5, "x")
    t1y = _truth_slices(c1["K1"], 5, "y")
    c = np.array([full["XV"][j, 0] / t1x[j, 0] for j in range(5)])
    d = np.array([full["YV"][i, 0] / t1y[i, 0] for i in range(5)])
    a, b = full["a"], full["b"]
    np.testing.assert_allclose(a * c, (a * c)[0], rtol=1e-11)
    np.testing.assert_allclose(b * d, (a * c)[0], rtol=1e-11)
    assert full["Hspec"][0] <= 1e-20 * full["Hspec"][-1]
    assert full["Hspec"][1] >= 1e-6 * full["Hspec"][-1]


def test_assembly_invariants_noiseless(c1):
    K1, K2, full = cbp.recover_kernels(c1["B1"], c1["B2"], 64, 64, 5, full=True)
    for K, d in zip((K1, K2), full["diag"]):
        assert K.sum() == pytest.approx(1.0, abs=1e-14)
        assert d["imag"] < 1e-12 and d["outside"] < 1e-24


def test_assembly_is_plain_inverse_dft_when_grids_are_exact():
    """With P = c_j Khat and Q = d_i Khat, a = 1/c, b = 1/d, O6 returns the
    kernel exactly (inverse DFT of its own S x S spectrum)."""
    r = np.random.default_rng(3)
    k, S = 4, 6
    K = r.random((k, k))
    Kfull = np.zeros((S, S))
    Kfull[:k, :k] = K
    Khat = np.fft.fft2(Kfull).T                   # [i (x freq), j (y freq)]
    c = r.standard_normal(S) + 1j * r.standard_normal(S)
    d = r.standard_normal(S) + 1j * r.standard_normal(S)
    P = Khat * c[None, :]
    Q = Khat * d[:, None]
    out, diag = cbp.assemble_kernel(P, Q, 1 / c, 1 / d, k)
    np.testing.assert_allclose(out, K / K.sum(), atol=1e-14)


# ---------------------------------------------------------------- O7

def test_deconvolve_exact_inverse_with_true_kernels(c1):
    L = cbp.deconvolve(c1["B1"], c1["B2"], c1["K1"], c1["K2"], 64, 64, 0.0)
    np.testing.assert_allclose(L, c1["L"], atol=1e-11)


def test_deconvolve_single_channel_is_inverse_filter(c1):
    B1, K1 = c1["B1"], c1["K1"]
    Py, Px = cbp.smooth7(B1.shape[0]), cbp.smooth7(B1.shape[1])
    ref = np.real(np.fft.ifft2(np.fft.fft2(B1, s=(Py, Px)) / np.fft.fft2(K1, s=(Py, Px))))[:64, :64]
    np.testing.assert_allclose(cbp.deconvolve(B1, B1, K1, K1, 64, 64, 0.0), ref, atol=1e-11)


def test_deconvolve_large_lambda_limit(c1):
    B1, B2, K1, K2 = c1["B1"], c1["B2"], c1["K1"], c1["K2"]
    lam = 1e12
    Py, Px = cbp.smooth7(B1.shape[0]), cbp.smooth7(B1.shape[1])
    s = (Py, Px)
    num = np.conj(np.fft.fft2(K1, s=s)) * np.fft.fft2(B1, s=s) + np.conj(np.fft.fft2(K2, s=s)) * np.fft.fft2(B2, s=s)
    ref = np.real(np.fft.ifft2(num))[:64, :64]
    np.testing.assert_allclose(lam * cbp.deconvolve(B1, B2, K1, K2, 64, 64, lam), ref, rtol=1e-9, atol=1e-9)


# ---------------------------------------------------------------- whole method

def test_config1_recovers_truth(c1):
    L, K1, K2 = cbp.deblur(c1["B1"], c1["B2"], 64, 64, 5, 0.0)
    assert rel(K1, c1["K1"]) < 1e-12 and rel(K2, c1["K2"]) < 1e-12
    np.testing.assert_allclose(L, c1["L"], atol=1e-10)


def test_tls2d_agrees_with_truth_and_method(c1):
    V, U, spec = tls2d.recover_kernels_2d(c1["B1"], c1["B2"], 5, 5)
    assert rel(V, c1["K1"]) < 1e-12 and rel(U, c1["K2"]) < 1e-12
    G = tls2d.gram_matrix(c1["B1"][:20, :22], c1["B2"][:20, :22], 5, 5)
    A = tls2d.system_matrix(c1["B1"][:20, :22], c1["B2"][:20, :22], 5, 5)
    np.testing.assert_allclose(G, A.T @ A, rtol=1e-12, atol=1e-12 * np.abs(G).max())


@pytest.mark.parametrize("k1,k2,S", [(3, 5, 5), (5, 3, 10), (1, 3, 3), (4, 4, 4), (7, 6, 9)])
def test_uneven_sizes_and_oversampling(k1, k2, S):
    r = synth.rng_for(99, k1, k2, S)
    L = r.random((30, 37))
    K1, K2 = synth.draw_coprime_pair(r, k1, k2, "uniform", sample_counts=(S,))
    B1, B2 = synth.full_conv2d(L, K1), synth.full_conv2d(L, K2)
    R1, R2 = cbp.recover_kernels(B1, B2, 30, 37, S)
    assert rel(R1, K1) < 1e-10 and rel(R2, K2) < 1e-10


def test_config2_noiseless_recovers_truth():
    c = synth.config2(noise=0.0, m=120, n=160)
    K1, K2 = cbp.recover_kernels(c["B1"], c["B2"], 120, 160)
    assert rel(K1, c["K1"]) < 1e-9 and rel(K2, c["K2"]) < 1e-9


# ---------------------------------------------------------------- operand rounding of the matrix-core forms

def test_bf16_rounding_ties_and_library():
    """round_operands('bf16'): FP64 -> FP32 -> bfloat16, each round to nearest
    even.  Pinned by hand-worked ties and by torch's own float32 -> bfloat16
    conversion (a library routine) on random values."""
    r = lambda v: cbp.round_operands(np.array([v], dtype=np.complex128), "bf16")[0].real
    assert r(1.0) == 1.0
    assert r(1.0 + 2.0 ** -8) == 1.0                     # tie -> even (mantissa 0)
    assert r(1.0 + 3 * 2.0 ** -8) == 1.0 + 2.0 ** -6     # tie -> even (mantissa 2)
    assert r(1.0 + 2.0 ** -8 + 2.0 ** -20) == 1.0 + 2.0 ** -7   # above the tie
    assert r(-(1.0 + 3 * 2.0 ** -8)) == -(1.0 + 2.0 ** -6)
    assert r(0.0) == 0.0
    torch = pytest.importorskip("torch")
    x = np.random.default_rng(5).standard_normal(4096) * 10.0 ** np.random.default_rng(6).uniform(-8, 8, 4096)
    want = torch.tensor(x.astype(np.float32)).to(torch.bfloat16).to(torch.float64).numpy()
    got = cbp.round_operands(x + 0j, "bf16").real
    assert np.array_equal(got, want)
    got32 = cbp.round_operands(x + 1j * x, "f32")
    assert np.array_equal(got32.real, x.astype(np.float32).astype(np.float64))
    assert np.array_equal(got32.imag, got32.real)


def test_rounded_gram_reduces_to_plain_and_is_block_toeplitz():
    """fmt None is the plain Gram; any format gives a Hermitian block-Toeplitz
    G whose null vector is the rounded problem's (checked against svd)."""
    r = np.random.default_rng(8)
    e1 = r.standard_normal(40) + 1j * r.standard_normal(40)
    e2 = r.standard_normal(38) + 1j * r.standard_normal(38)   # len(e1) + k2 = len(e2) + k1
    k1, k2 = 5, 3
    A = cbp.sample_matrix(e1, e2, k1, k2)
    assert np.array_equal(cbp.sample_gram(e1, e2, k1, k2), A.conj().T @ A)
    for fmt in ("f32", "bf16"):
        G = cbp.sample_gram(e1, e2, k1, k2, fmt)
        assert np.allclose(G, G.conj().T, rtol=0, atol=1e-12 * np.abs(G).max())
        for p in range(k2 - 1):      # G11 is Toeplitz: G[p + 1, 1] = G[p, 0]
            assert abs(G[p + 1, 1] - G[p, 0]) <= 1e-12 * np.abs(G).max()
        x, _ = cbp.null_vector(cbp.sample_matrix(cbp.round_operands(e1, fmt), cbp.round_operands(e2, fmt), k1, k2))
        w, V = np.linalg.eigh(G)
        assert abs(abs(np.vdot(V[:, 0], x)) - 1.0) <= 1e-8
        assert np.abs(G - cbp.sample_gram(e1, e2, k1, k2)).max() > 0   # the rounding is seen
