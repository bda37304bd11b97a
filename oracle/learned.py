"""Learned per-sample weights (the learned form; the paper has no counterpart)
in plain FP64 NumPy -- TEST INFRASTRUCTURE ONLY, like the rest of oracle/.

A small MLP reads each sample's Gram spectrum and predicts a confidence
weight w and a Tikhonov strength tau.  The weights enter the scale fix and
the kernel assembly; with w == 1 and tau == 0 every step reduces to the plain
method (scale_fix / assemble_kernel of oracle.cbp), which the functions below
call in that case, so the reduction is exact by construction.

Readings (no paper text covers this form; these are this implementation's
definitions):
  * features: the sample's ascending Gram eigenvalues as
    f_i = log10(max(lambda_i, 1e-14 lambda_max) / lambda_max) / 10 for
    i < N = k1 + k2, and the sentinel +1 for i = N .. 31 (real features are
    <= 0, so the sentinel marks the padding).  The floor 1e-14 sits above the
    rounding level of an FP64 Gram's eigenvalues (about 1e-16 lambda_max), so
    eigenvalues below it, which no FP64 route resolves, all read as -1.4;
  * MLP 32 -> 128 -> 128 -> 2 with ReLU, outputs o = (o1, o2):
    w = clip(softplus(o1), 1e-3, 1e3), tau_j = exp(clip(o2, -30, 5));
    the frame's tau is the median of its samples' tau_j;
  * scale fix: the rows a_j P_c[i,j] - b_i Q_c[i,j] weighted by
    sqrt(wX_j wY_i), smallest eigenvector of the weighted normal matrix;
  * assembly: Khat = (wX_j a_j P + wY_i b_i Q) / (wX_j + wY_i); the kernel Z
    (k x k, [x][y]) minimises the separable weighted fit
        || D_u^(1/2) (Fx Z Fy^T - Khat) D_v^(1/2) ||_F^2
    (u_i = wY_i on the x-samples, v_j = wX_j on the y-samples,
    Fx[i][x] = w_i^x, Fy[j][y] = w_j^y) with per-axis Tikhonov terms, whose
    normal equations are (Ax + tau I) Z (By + tau I) = C,
        Ax = Fx^H D_u Fx,  By = Fy^T D_v conj(Fy),  C = Fx^H D_u Khat D_v conj(Fy);
    then K = Z^T is divided by its complex sum and its real part kept (as
    the plain assembly).  At w == 1, tau == 0: Ax = By = S I and Z is the
    cropped inverse DFT of Khat -- the plain assembly.
"""

from __future__ import annotations

import numpy as np

from . import cbp

FEAT = 32
HIDDEN = 128
PAD = 1.0
LOG_FLOOR = 1e-14


# --------------------------------------------------------------------------
# features
# --------------------------------------------------------------------------

def spectrum_features(spec: np.ndarray) -> np.ndarray:
    """spec: (..., N) ascending Gram eigenvalues -> (..., 32) features."""
    spec = np.asarray(spec, dtype=np.float64)
    N = spec.shape[-1]
    if N > FEAT:
        raise ValueError("at most 32 eigenvalues")
    lmax = spec[..., -1:]
    f = np.log10(np.maximum(spec, LOG_FLOOR * lmax) / lmax) / 10.0
    out = np.full(spec.shape[:-1] + (FEAT,), PAD)
    out[..., :N] = f
    return out


# --------------------------------------------------------------------------
# the MLP (FP64 reference of the BF16 kernels)
# --------------------------------------------------------------------------

def init_params(rng: np.random.Generator):
    """He-normal weights, zero biases; W1 (128 x 32), W2 (128 x 128), W3 (2 x 128)."""
    def he(o, i):
        return rng.standard_normal((o, i)) * np.sqrt(2.0 / i)
    return dict(W1=he(HIDDEN, FEAT), b1=np.zeros(HIDDEN), W2=he(HIDDEN, HIDDEN), b2=np.zeros(HIDDEN),
                W3=he(2, HIDDEN) * 0.1, b3=np.zeros(2))


def mlp_forward(p, X: np.ndarray):
    """X (n, 32) -> outputs (n, 2) and the activations the backward pass needs."""
    z1 = X @ p["W1"].T + p["b1"]
    h1 = np.maximum(z1, 0.0)
    z2 = h1 @ p["W2"].T + p["b2"]
    h2 = np.maximum(z2, 0.0)
    o = h2 @ p["W3"].T + p["b3"]
    return o, dict(X=X, z1=z1, h1=h1, z2=z2, h2=h2)


def mlp_backward(p, cache, dO: np.ndarray):
    """Gradients of sum(dO * o) with respect to every parameter."""
    g = {}
    g["W3"] = dO.T @ cache["h2"]
    g["b3"] = dO.sum(0)
    dh2 = dO @ p["W3"]
    dz2 = dh2 * (cache["z2"] > 0)
    g["W2"] = dz2.T @ cache["h1"]
    g["b2"] = dz2.sum(0)
    dh1 = dz2 @ p["W2"]
    dz1 = dh1 * (cache["z1"] > 0)
    g["W1"] = dz1.T @ cache["X"]
    g["b1"] = dz1.sum(0)
    return g


def softplus(x):
    return np.logaddexp(0.0, x)


def weights_from_outputs(o: np.ndarray):
    """(w, tau_j) per sample from the MLP outputs."""
    w = np.clip(softplus(o[..., 0]), 1e-3, 1e3)
    tau = np.exp(np.clip(o[..., 1], -30.0, 5.0))
    return w, tau


def loss_and_grad(p, X: np.ndarray, logw_target: np.ndarray, logtau_target: np.ndarray):
    """Mean squared error of (log w, log tau) against their targets, and its
    parameter gradients (the training objective)."""
    o, cache = mlp_forward(p, X)
    sp = softplus(o[:, 0])
    lw = np.log(sp)
    n = X.shape[0]
    r1 = lw - logw_target
    r2 = o[:, 1] - logtau_target
    loss = float(np.mean(r1 ** 2 + r2 ** 2))
    dO = np.zeros_like(o)
    sig = 1.0 / (1.0 + np.exp(-o[:, 0]))
    dO[:, 0] = 2.0 * r1 / n * sig / sp
    dO[:, 1] = 2.0 * r2 / n
    return loss, mlp_backward(p, cache, dO)


# --------------------------------------------------------------------------
# weighted scale fix and assembly
# --------------------------------------------------------------------------

def scale_fix_weighted(P, Q, wX: np.ndarray, wY: np.ndarray):
    """(a, b) minimising sum_{c,i,j} wX_j wY_i |a_j P_c[i,j] - b_i Q_c[i,j]|^2,
    ||(a, b)|| = 1: smallest eigenvector of the weighted normal matrix.
    Unit weights take the plain scale fix."""
    wX = np.asarray(wX, dtype=np.float64)
    wY = np.asarray(wY, dtype=np.float64)
    if np.all(wX == 1.0) and np.all(wY == 1.0):
        return cbp.scale_fix(P, Q)
    return weighted_scale_core(P, Q, wX, wY)


def weighted_scale_core(P, Q, wX, wY):
    """The weighted normal matrix and its smallest eigenvector (any weights)."""
    S = P[0].shape[0]
    W = np.outer(wY, wX)                       # [i][j]
    H = np.zeros((2 * S, 2 * S), dtype=np.complex128)
    for Pc, Qc in zip(P, Q):
        H[:S, :S] += np.diag((W * np.abs(Pc) ** 2).sum(0))
        H[S:, S:] += np.diag((W * np.abs(Qc) ** 2).sum(1))
        C = (W * np.conj(Pc) * Qc).T            # [j][i]
        H[:S, S:] -= C
        H[S:, :S] -= C.conj().T
    w, V = np.linalg.eigh(H)
    z = V[:, 0]
    return z[:S], z[S:], w


def assemble_weighted(Pc, Qc, a, b, k: int, wX, wY, tau: float):
    """The weighted, regularised assembly (module docstring).  Unit weights
    with tau = 0 take the plain assembly."""
    wX = np.asarray(wX, dtype=np.float64)
    wY = np.asarray(wY, dtype=np.float64)
    if np.all(wX == 1.0) and np.all(wY == 1.0) and tau == 0.0:
        return cbp.assemble_kernel(Pc, Qc, a, b, k)
    return weighted_assembly_core(Pc, Qc, a, b, k, wX, wY, tau)


def weighted_assembly_core(Pc, Qc, a, b, k, wX, wY, tau):
    """The separable weighted fit with per-axis Tikhonov terms (any weights)."""
    S = Pc.shape[0]
    Kh = (wX[None, :] * a[None, :] * Pc + wY[:, None] * b[:, None] * Qc) / (wX[None, :] + wY[:, None])
    F = cbp.unit_roots_matrix(S, k)            # F[i][x] = w_i^x
    Du, Dv = np.diag(wY), np.diag(wX)
    Ax = F.conj().T @ Du @ F
    By = F.T @ Dv @ F.conj()
    C = F.conj().T @ Du @ Kh @ Dv @ F.conj()
    I = np.eye(k)
    Z = np.linalg.solve(Ax + tau * I, C)
    Z = np.linalg.solve((By + tau * I).T, Z.T).T
    K = Z.T
    s = K.sum()
    Kn = K / s
    return Kn.real, dict(imag=float(np.linalg.norm(Kn.imag) / np.linalg.norm(Kn.real)), sum=s)


def recover_kernels_learned(B1, B2, m: int, n: int, params, S: int = 0, full: bool = False,
                            bf16: bool = False):
    """Kernels with MLP weights (O1-O6 with the weighted O5 / O6).  bf16 runs
    the network with the GPU kernels' roundings (mlp_forward_bf16) and takes
    the features in FP32, as the GPU stores them."""
    K1p, K2p, f = cbp.recover_kernels(B1, B2, m, n, S, full=True)
    k1, k2, S = f["k1"], f["k2"], f["S"]
    XF = spectrum_features(f["Xspec"])
    YF = spectrum_features(f["Yspec"])
    fwd = mlp_forward
    if bf16:
        XF, YF, fwd = _f32(XF), _f32(YF), mlp_forward_bf16
    oX, _ = fwd(params, XF)
    oY, _ = fwd(params, YF)
    wX, tX = weights_from_outputs(oX)
    wY, tY = weights_from_outputs(oY)
    tau = float(np.median(np.concatenate([tX, tY])))
    a, b, _ = scale_fix_weighted(f["P"], f["Q"], wX, wY)
    L1, _ = assemble_weighted(f["P"][0], f["Q"][0], a, b, k1, wX, wY, tau)
    L2, _ = assemble_weighted(f["P"][1], f["Q"][1], a, b, k2, wX, wY, tau)
    # the plain method judges: keep its kernels when their objective is smaller
    Jp = judge_objective(K1p, K2p, f["EX"], f["EY"], S)
    Jl = judge_objective(L1, L2, f["EX"], f["EY"], S)
    noisy = frame_is_noisy(XF, YF)
    # the learned kernels are kept only on a frame without a noise floor and
    # when their objective is a number no larger than the plain one's
    fallback = noisy or not (Jl <= Jp)
    K1, K2 = (K1p, K2p) if fallback else (L1, L2)
    if not full:
        return K1, K2
    return K1, K2, dict(plain=(K1p, K2p), learned=(L1, L2), judge=(Jp, Jl), fallback=fallback, noisy=noisy,
                        wX=wX, wY=wY,
                        tau=tau, features=(XF, YF), base=f)


# The noise gate of the learned form (no counterpart in the paper): a frame
# is noisy when more than half of its 2S samples have a smallest-eigenvalue
# feature f_0 above NOISY_F0 (lambda_0 / lambda_max > 1e-10); there the
# network does not gain on held-out pairs and the plain kernels are kept.
NOISY_F0 = -1.0


def frame_is_noisy(XF: np.ndarray, YF: np.ndarray) -> bool:
    f0 = np.concatenate([np.asarray(XF)[:, 0], np.asarray(YF)[:, 0]])
    return int(np.sum(f0 > NOISY_F0)) > f0.size // 2


def kernel_slices(K1, K2, S: int, pass_: int, j: int) -> np.ndarray:
    """x = (u: K2 slice, v: K1 slice) of the kernels at sample j of a pass:
    pass X (0) evaluates along y at w_j, pass Y (1) along x."""
    w = np.exp(-2j * np.pi * j / S)
    def sl(K):
        p = w ** np.arange(K.shape[0])
        return p @ K if pass_ == 0 else K @ p
    return np.concatenate([sl(K2), sl(K1)])


def judge_objective(K1, K2, EX, EY, S: int) -> float:
    """The plain method's objective for a kernel pair: the sum over both
    passes and all samples of the Rayleigh quotient x^H G x / x^H x of the
    pair's slices in the sample's Gram (the per-sample TLS residual)."""
    k1, k2 = K1.shape[0], K2.shape[0]
    J = 0.0
    for p, (E1, E2) in enumerate((EX, EY)):
        for j in range(S):
            G = cbp.sample_gram(E1[j], E2[j], k1, k2)
            x = kernel_slices(K1, K2, S, p, j)
            J += float(np.real(np.vdot(x, G @ x)) / np.real(np.vdot(x, x)))
    return J


# --------------------------------------------------------------------------
# the network in the kernels' precision (for parity of the GPU network)
# --------------------------------------------------------------------------

def round_bf16(x: np.ndarray) -> np.ndarray:
    """Round to float32 (nearest even), then to bfloat16 (nearest even)."""
    f = np.asarray(x, dtype=np.float64).astype(np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def _f32(x):
    return np.asarray(x, dtype=np.float64).astype(np.float32).astype(np.float64)


def mlp_forward_bf16(p, X: np.ndarray):
    """The forward pass with the roundings the GPU kernels make: inputs, W1,
    W2 and both hidden activations in bfloat16; biases and the head W3 in
    FP32; every sum exact (FP64) here."""
    Xb = round_bf16(X)
    z1 = Xb @ round_bf16(p["W1"]).T + _f32(p["b1"])
    h1 = round_bf16(np.maximum(z1, 0.0))
    z2 = h1 @ round_bf16(p["W2"]).T + _f32(p["b2"])
    h2 = round_bf16(np.maximum(z2, 0.0))
    o = h2 @ _f32(p["W3"]).T + _f32(p["b3"])
    return o, dict(X=Xb, h1=h1, h2=h2)


def loss_and_grad_bf16(p, X, logw_target, logtau_target):
    """loss_and_grad with the GPU's roundings: the backpropagated signals into
    the hidden layers (dZ2, dZ1) are rounded to bfloat16, as the kernels
    store them."""
    o, c = mlp_forward_bf16(p, X)
    n = X.shape[0]
    sp = softplus(o[:, 0])
    r1 = np.log(sp) - logw_target
    r2 = o[:, 1] - logtau_target
    loss = float(np.mean(r1 ** 2 + r2 ** 2))
    dO = np.zeros_like(o)
    sig = 1.0 / (1.0 + np.exp(-o[:, 0]))
    dO[:, 0] = 2.0 * r1 / n * sig / sp
    dO[:, 1] = 2.0 * r2 / n
    g = {}
    g["W3"] = dO.T @ c["h2"]
    g["b3"] = dO.sum(0)
    dZ2 = round_bf16((dO @ _f32(p["W3"])) * (c["h2"] > 0))
    g["W2"] = dZ2.T @ c["h1"]
    g["b2"] = dZ2.sum(0)
    dZ1 = round_bf16((dZ2 @ round_bf16(p["W2"])) * (c["h1"] > 0))
    g["W1"] = dZ1.T @ c["X"]
    g["b1"] = dZ1.sum(0)
    return loss, g


def pack(p) -> np.ndarray:
    """Parameters in the packed order W1, b1, W2, b2, W3, b3 (FP64)."""
    return np.concatenate([p["W1"].ravel(), p["b1"], p["W2"].ravel(), p["b2"], p["W3"].ravel(), p["b3"]])


def unpack(v: np.ndarray):
    v = np.asarray(v, dtype=np.float64)
    o = 0
    out = {}
    for name, shape in (("W1", (HIDDEN, FEAT)), ("b1", (HIDDEN,)), ("W2", (HIDDEN, HIDDEN)), ("b2", (HIDDEN,)),
                        ("W3", (2, HIDDEN)), ("b3", (2,))):
        size = int(np.prod(shape))
        out[name] = v[o:o + size].reshape(shape).copy()
        o += size
    return out
