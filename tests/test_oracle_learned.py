"""Pins of the learned form's oracle (oracle/learned.py) against things other
than itself: central differences for the MLP gradients, a dense
least-squares solve for the separable weighted assembly, an explicit
weighted row system for the weighted scale fix, closed-form features, and
the reductions to the plain method."""

import numpy as np
import pytest

import synth
from oracle import cbp, learned


def test_features_closed_form():
    f = learned.spectrum_features(np.array([1e-10, 1e-5, 1.0]))
    assert f.shape == (32,)
    assert np.allclose(f[:3], [-1.0, -0.5, 0.0], atol=1e-15)
    assert np.all(f[3:] == learned.PAD)
    g = learned.spectrum_features(np.array([0.0, 1e-20, 2.0]))  # below 1e-14 lambda_max: the floor
    assert np.allclose(g[:2], -1.4) and g[2] == 0.0


def test_mlp_gradients_match_central_differences():
    rng = np.random.default_rng(3)
    p = learned.init_params(rng)
    p = {k: v + 0.05 * rng.standard_normal(v.shape) for k, v in p.items()}
    X = rng.standard_normal((7, 32))
    tw = rng.standard_normal(7)
    tt = rng.standard_normal(7)
    loss, g = learned.loss_and_grad(p, X, tw, tt)
    h = 1e-6
    for name in ("W1", "b1", "W2", "b2", "W3", "b3"):
        idx = [tuple(rng.integers(0, s) for s in p[name].shape) for _ in range(6)]
        for ix in idx:
            q = {k: v.copy() for k, v in p.items()}
            q[name][ix] += h
            lp, _ = learned.loss_and_grad(q, X, tw, tt)
            q[name][ix] -= 2 * h
            lm, _ = learned.loss_and_grad(q, X, tw, tt)
            num = (lp - lm) / (2 * h)
            assert abs(num - g[name][ix]) <= 1e-6 * max(1.0, abs(num)), (name, ix, num, g[name][ix])


def _grids(seed, k1, k2, S, noise=0.0):
    r = synth.rng_for(seed)
    L = r.random((40, 44))
    K1, K2 = synth.draw_coprime_pair(r, k1, k2, "uniform")
    B1, B2 = synth.blur_pair(synth.rng_for(seed, 1), L, K1, K2, noise)
    _, _, f = cbp.recover_kernels(B1, B2, 40, 44, S, full=True)
    return f, K1, K2


def test_weighted_scale_fix_against_row_system():
    f, _, _ = _grids(11, 4, 5, 6, noise=1e-3)
    P, Q = f["P"], f["Q"]
    S = P[0].shape[0]
    rng = np.random.default_rng(4)
    wX, wY = rng.uniform(0.2, 3.0, S), rng.uniform(0.2, 3.0, S)
    a, b, _ = learned.weighted_scale_core(P, Q, wX, wY)
    rows = []
    for Pc, Qc in zip(P, Q):
        for i in range(S):
            for j in range(S):
                r = np.zeros(2 * S, dtype=np.complex128)
                sw = np.sqrt(wX[j] * wY[i])
                r[j] = sw * Pc[i, j]
                r[S + i] = -sw * Qc[i, j]
                rows.append(r)
    _, _, Vh = np.linalg.svd(np.array(rows))
    z = Vh[-1].conj()
    zz = np.concatenate([a, b])
    assert abs(abs(np.vdot(z, zz)) - 1.0) <= 1e-10
    # unit weights through the weighted route equal the plain scale fix
    a1, b1, _ = learned.weighted_scale_core(P, Q, np.ones(S), np.ones(S))
    a0, b0, _ = cbp.scale_fix(P, Q)
    assert abs(abs(np.vdot(np.concatenate([a0, b0]), np.concatenate([a1, b1]))) - 1.0) <= 1e-12


def test_weighted_assembly_against_dense_lstsq_and_plain():
    f, K1, K2 = _grids(12, 4, 3, 5, noise=1e-3)
    P, Q = f["P"], f["Q"]
    S = P[0].shape[0]
    a, b, _ = cbp.scale_fix(P, Q)
    rng = np.random.default_rng(5)
    wX, wY = rng.uniform(0.2, 3.0, S), rng.uniform(0.2, 3.0, S)
    k = 4
    K, _ = learned.weighted_assembly_core(P[0], Q[0], a, b, k, wX, wY, 0.0)
    # dense weighted least squares over the k*k complex unknowns Z[x][y]
    Kh = (wX[None, :] * a[None, :] * P[0] + wY[:, None] * b[:, None] * Q[0]) / (wX[None, :] + wY[:, None])
    F = cbp.unit_roots_matrix(S, k)
    A = np.zeros((S * S, k * k), dtype=np.complex128)
    rhs = np.zeros(S * S, dtype=np.complex128)
    for i in range(S):
        for j in range(S):
            sw = np.sqrt(wY[i] * wX[j])
            A[i * S + j] = sw * np.outer(F[i], F[j]).ravel()     # Z[x][y] coefficient F[i][x] F[j][y]
            rhs[i * S + j] = sw * Kh[i, j]
    Z = np.linalg.lstsq(A, rhs, rcond=None)[0].reshape(k, k)
    Kd = Z.T / Z.sum()
    assert np.abs(K - Kd.real).max() <= 1e-10 * np.abs(Kd).max()
    # unit weights, tau = 0 through the weighted route: the plain assembly
    Ku, _ = learned.weighted_assembly_core(P[0], Q[0], a, b, k, np.ones(S), np.ones(S), 0.0)
    Kp, _ = cbp.assemble_kernel(P[0], Q[0], a, b, k)
    assert np.abs(Ku - Kp).max() <= 1e-12
    # uniform weights: tau only rescales Z, which the normalisation removes
    Kt, _ = learned.weighted_assembly_core(P[0], Q[0], a, b, k, 2 * np.ones(S), 2 * np.ones(S), 3.0)
    assert np.abs(Kt - Kp).max() <= 1e-12
    # tau -> infinity: Z -> C / tau^2, the weighted adjoint of Khat
    Kinf, _ = learned.weighted_assembly_core(P[0], Q[0], a, b, k, wX, wY, 1e9)
    C = F.conj().T @ np.diag(wY) @ Kh @ np.diag(wX) @ F.conj()
    Kc = C.T / C.sum()
    assert np.abs(Kinf - Kc.real).max() <= 1e-6 * np.abs(Kc).max()


def test_constant_network_output_reduces_to_plain():
    """A network with zero last-layer weights outputs constants: constant
    weights and tau ~ e^-30 give the plain kernels."""
    r = synth.rng_for(77)
    L = r.random((48, 50))
    K1, K2 = synth.draw_coprime_pair(r, 5, 4, "uniform")
    B1, B2 = synth.blur_pair(synth.rng_for(77, 1), L, K1, K2, 1e-3)
    p = learned.init_params(np.random.default_rng(1))
    p["W3"][:] = 0.0
    p["b3"][:] = [4.0, -40.0]
    Q1, Q2, info = learned.recover_kernels_learned(B1, B2, 48, 50, p, full=True)
    P1, P2 = info["plain"]
    assert np.allclose(info["wX"], info["wX"][0]) and info["tau"] <= 1e-12
    assert np.abs(Q1 - P1).max() <= 1e-9 and np.abs(Q2 - P2).max() <= 1e-9


def test_bf16_network_emulation_reduces_to_fp64_on_representable_values():
    """With parameters and inputs that bfloat16 holds exactly and activations
    that stay exact, the emulated forward equals the FP64 forward; the
    rounding itself matches the operand rounding of the Gram forms."""
    rng = np.random.default_rng(9)
    p = learned.init_params(rng)
    p = {k: learned.round_bf16(v) for k, v in p.items()}
    X = learned.round_bf16(rng.standard_normal((5, 32)))
    o1, _ = learned.mlp_forward_bf16(p, X)
    o0, _ = learned.mlp_forward(p, X)
    assert np.abs(o1 - o0).max() <= 2e-2 * np.abs(o0).max()     # only the hidden roundings differ
    x = rng.standard_normal(1000)
    assert np.array_equal(learned.round_bf16(x), cbp.round_operands(x + 0j, "bf16").real)
    v = learned.pack(p)
    q = learned.unpack(v)
    assert all(np.array_equal(p[k], q[k]) for k in p) and v.size == 20994


def test_judge_objective_is_zero_on_true_kernels_and_prefers_them():
    """Noiseless: the true kernels' slices are the per-sample null vectors, so
    their objective is ~0 (relative to the Gram scale) and any perturbation
    raises it."""
    r = synth.rng_for(91)
    L = r.random((36, 40))
    K1, K2 = synth.draw_coprime_pair(r, 4, 5, "uniform")
    B1, B2 = synth.full_conv2d(L, K1), synth.full_conv2d(L, K2)
    S = 5
    EX = [cbp.unit_circle_eval(B, S)[0] for B in (B1, B2)]
    EY = [cbp.unit_circle_eval(B, S)[1] for B in (B1, B2)]
    J0 = learned.judge_objective(K1, K2, EX, EY, S)
    scale = sum(np.trace(cbp.sample_gram(EX[0][j], EX[1][j], 4, 5)).real for j in range(S))
    assert J0 <= 1e-20 * scale
    J1 = learned.judge_objective(K1 + 1e-3 * r.random(K1.shape), K2, EX, EY, S)
    assert J1 > 1e6 * max(J0, 1e-300)
    # the slices of a kernel pair at a sample are the ones the oracle's truth pins use
    x = learned.kernel_slices(K1, K2, S, 0, 2)
    w = np.exp(-2j * np.pi * 2 / S)
    assert np.allclose(x[:5], (w ** np.arange(5)) @ K2) and np.allclose(x[5:], (w ** np.arange(4)) @ K1)


def test_noise_gate_separates_noiseless_from_noisy_frames():
    """The learned form's noise gate: a noiseless pair has its per-sample
    lambda_0 at the rounding level (feature f_0 at the 1e-14 floor, -1.4), a
    pair with noise 1e-3 a noise floor far above 1e-10 (f_0 > -1); exactly
    half of the samples above the threshold is not yet noisy."""
    r = synth.rng_for(93)
    L = synth.gaussian_scene(r, 96, 128)
    K1, K2 = synth.draw_coprime_pair(r, 5, 7, "uniform")
    for noise, want in ((0.0, False), (1e-3, True)):
        B1, B2 = synth.blur_pair(synth.rng_for(94), L, K1, K2, noise)
        _, _, f = cbp.recover_kernels(B1, B2, 96, 128, 0, full=True)
        XF, YF = learned.spectrum_features(f["Xspec"]), learned.spectrum_features(f["Yspec"])
        print(noise, np.median(XF[:, 0]), np.median(YF[:, 0]))
        assert learned.frame_is_noisy(XF, YF) == want
    XF = np.full((4, 32), -1.4)
    YF = np.full((4, 32), -1.4)
    XF[:, 0] = -0.5                                   # 4 of 8 samples above: not more than half
    assert not learned.frame_is_noisy(XF, YF)
    YF[0, 0] = -0.99                                  # 5 of 8
    assert learned.frame_is_noisy(XF, YF)


def _exact_case(n=8, seed=23):
    """Parameters, inputs and every activation and back-propagated signal
    exactly representable in bfloat16: sparse {0, +-1} layer weights,
    half-integer inputs and biases, a head in quarters, and targets chosen so
    that dL/do1 = 0 and dL/do2 = 1/4 exactly.  Every sum is then exact in FP64
    whatever its order, so any rounding point of the emulation is the
    identity."""
    rng = np.random.default_rng(seed)

    def sparse(o, i, nnz):
        W = np.zeros((o, i))
        for r in range(o):
            c = rng.choice(i, nnz, replace=False)
            W[r, c] = rng.choice([-1.0, 1.0], nnz)
        return W

    p = dict(W1=sparse(128, 32, 4), b1=0.5 * rng.integers(-2, 3, 128),
             W2=sparse(128, 128, 4), b2=0.5 * rng.integers(-2, 3, 128),
             W3=0.25 * rng.integers(-4, 5, (2, 128)) * (rng.random((2, 128)) < 0.1), b3=np.array([0.5, -1.0]))
    X = 0.5 * rng.integers(-2, 3, (n, 32))
    o, _ = learned.mlp_forward(p, X)
    t1 = np.log(learned.softplus(o[:, 0]))
    t2 = o[:, 1] - n / 8.0
    return p, X, t1, t2


def test_bf16_network_equals_fp64_network_where_bf16_is_exact():
    """Pin of the bf16 emulation against the FP64 network (itself pinned by
    central differences): on a case where bfloat16 holds every operand,
    activation and back-propagated signal exactly, the emulated forward and
    the emulated loss and gradients of every block equal the FP64 ones bit
    for bit -- so the emulation multiplies, transposes and masks the same
    quantities as the exact network and differs from it only by its
    roundings."""
    p, X, t1, t2 = _exact_case()
    for v in (*p.values(), X):
        assert np.array_equal(learned.round_bf16(v), v)
    o0, c0 = learned.mlp_forward(p, X)
    o1, c1 = learned.mlp_forward_bf16(p, X)
    assert np.array_equal(o0, o1)
    assert np.array_equal(learned.round_bf16(c0["h1"]), c0["h1"]) and np.array_equal(c0["h1"], c1["h1"])
    assert np.array_equal(learned.round_bf16(c0["h2"]), c0["h2"]) and np.array_equal(c0["h2"], c1["h2"])
    l0, g0 = learned.loss_and_grad(p, X, t1, t2)
    l1, g1 = learned.loss_and_grad_bf16(p, X, t1, t2)
    assert l0 == l1
    for k in ("W1", "b1", "W2", "b2", "W3", "b3"):
        assert np.array_equal(g0[k], g1[k]), k
        assert np.any(g0[k] != 0.0), k          # the case exercises every block
    # the signals into the hidden layers are exact here too
    dO = np.zeros_like(o0)
    dO[:, 1] = 0.25
    dZ2 = (dO @ p["W3"]) * (c0["z2"] > 0)
    assert np.array_equal(learned.round_bf16(dZ2), dZ2)
    dZ1 = (dZ2 @ p["W2"]) * (c0["z1"] > 0)
    assert np.array_equal(learned.round_bf16(dZ1), dZ1)


def test_bf16_emulation_rounds_at_the_stated_points():
    """Each rounding point of the emulation is live: perturbing one operand
    of the exact case by less than half a bfloat16 unit leaves the emulated
    result unchanged where that operand is rounded (inputs, W1, W2), and
    moves the exact network's result."""
    p, X, t1, t2 = _exact_case()
    l1, g1 = learned.loss_and_grad_bf16(p, X, t1, t2)
    for name in ("W1", "W2"):
        q = {k: v.copy() for k, v in p.items()}
        nz = np.argwhere(q[name] != 0)[0]
        q[name][tuple(nz)] *= 1.0 + 2.0 ** -10          # below half an ulp of a bf16 +-1
        _, gq = learned.loss_and_grad_bf16(q, X, t1, t2)
        _, gx = learned.loss_and_grad(q, X, t1, t2)
        _, g0 = learned.loss_and_grad(p, X, t1, t2)
        assert all(np.array_equal(gq[k], g1[k]) for k in g1), name
        assert any(not np.array_equal(gx[k], g0[k]) for k in g0), name
    Xq = X + (X != 0) * X * 2.0 ** -10
    oq, _ = learned.mlp_forward_bf16(p, Xq)
    o1, _ = learned.mlp_forward_bf16(p, X)
    assert np.array_equal(oq, o1)
