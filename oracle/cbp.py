"""The CBP recovery method in plain FP64 NumPy -- the oracle.

TEST INFRASTRUCTURE ONLY (see the package docstring).  Nothing here is
blocked, fused or reordered beyond what each step's definition states; every
function cites the passage it follows.  Library primitives used as steps:
``numpy.linalg.svd`` (null vectors), ``numpy.fft.fft2/ifft2`` (the final
Fourier division).

Notation (images row-major [y][x]):
  B_c  blurred frame c in {1,2}, H_c x W_c;  L latent m x n;  K_c k_c x k_c.
  Full convolution: H_c = m + k_c - 1, W_c = n + k_c - 1.
  S    samples per axis (the paper's t);  w_j = exp(-2 pi i j / S).
  Pass X evaluates each frame along y (the z1 / row direction of eq. 3) at
  w_j, leaving a polynomial in x; pass Y evaluates along x at w_i, leaving a
  polynomial in y.

Readings of the paper taken here (where it is silent or garbled):
  * samples are the S-th roots of unity, S = max(k1, k2) by default;
  * the 1-D cofactors at a sample are the null vector of the stacked
    convolution matrix [C_k2(b1) | -C_k1(b2)] (smallest right singular
    vector; equivalently the smallest eigenvector of its Gram matrix);
  * the scale fix minimises sum |a_j P_c[i,j] - b_i Q_c[i,j]|^2 over both
    kernels with ||(a, b)|| = 1;
  * the two scaled estimates are averaged in the Fourier domain, inverse
    transformed, cropped to the kernel support, divided by their (complex)
    sum and the real part kept;
  * the latent is recovered by two-channel Tikhonov-regularised Fourier
    division on the smallest 7-smooth grid covering both frames.

Parity status: every function here is pinned by tests (exact arithmetic on
integer inputs, ground-truth recovery on noiseless inputs, library routines,
brute-force null spaces); see tests/test_oracle_*.py.
"""

from __future__ import annotations

import numpy as np

MAX_K = 32


# --------------------------------------------------------------------------
# O1  shapes (Sec. 4, problem statement around eq. 4; Sec. 6: latent size known)
# --------------------------------------------------------------------------

def kernel_sizes(shape1, shape2, m: int, n: int):
    """Kernel sizes from the blurred and latent shapes under full convolution.

    A blurred frame of an m x n latent with a k x k kernel is
    (m+k-1) x (n+k-1), so k_c = H_c - m + 1 and it must equal W_c - n + 1.
    """
    (H1, W1), (H2, W2) = shape1, shape2
    k1, k2 = H1 - m + 1, H2 - m + 1
    if W1 - n + 1 != k1 or W2 - n + 1 != k2:
        raise ValueError("frames are not full convolutions of one m x n latent")
    if not (1 <= k1 <= MAX_K and 1 <= k2 <= MAX_K):
        raise ValueError("kernel size outside 1..32")
    return k1, k2


def smooth7(n: int) -> int:
    """Smallest integer >= n whose prime factors are all in {2, 3, 5, 7}."""
    v = max(int(n), 1)
    while True:
        r = v
        for p in (2, 3, 5, 7):
            while r % p == 0:
                r //= p
        if r == 1:
            return v
        v += 1


def unit_roots_matrix(S: int, length: int) -> np.ndarray:
    """V[j, t] = w_j^t = exp(-2 pi i (j t mod S) / S), shape S x length."""
    jt = np.outer(np.arange(S), np.arange(length)) % S
    return np.exp(-2j * np.pi * jt / S)


# --------------------------------------------------------------------------
# O2  unit-circle evaluation (Sec. 4 eq. 3; Sec. 5: the evaluations at the
#     S-th roots of unity form a length-S DFT)
# --------------------------------------------------------------------------

def unit_circle_eval(B: np.ndarray, S: int):
    """Evaluate the frame polynomial b(z1, z2) = z1^T B z2 at S roots of unity
    along one axis at a time (eq. 3), by direct Vandermonde products.

    Returns
      EX[j, x] = sum_y B[y, x] w_j^y   (S x W)   -- pass X, polynomial in z2
      EY[i, y] = sum_x B[y, x] w_i^x   (S x H)   -- pass Y, polynomial in z1
    """
    B = np.asarray(B, dtype=np.float64)
    H, W = B.shape
    EX = unit_roots_matrix(S, H) @ B
    EY = unit_roots_matrix(S, W) @ B.T
    return EX, EY


# --------------------------------------------------------------------------
# O3  per-sample 1-D cofactors (Sec. 4: the 2-D GCD is split into t 1-D GCD
#     sub-problems; Sec. 5: one factorisation per sample and direction)
# --------------------------------------------------------------------------

def conv_matrix(e: np.ndarray, k: int) -> np.ndarray:
    """C_k(e)[r, c] = e[r - c]: the (len(e)+k-1) x k matrix with C_k(e) u = e (x) u."""
    Le = len(e)
    C = np.zeros((Le + k - 1, k), dtype=np.complex128)
    for c in range(k):
        C[c:c + Le, c] = e
    return C


def sample_matrix(e1: np.ndarray, e2: np.ndarray, k1: int, k2: int) -> np.ndarray:
    """A = [C_k2(e1) | -C_k1(e2)].  Since b1 k2 = l k1 k2 = b2 k1 (eq. 4), the
    vector (k2-slice, k1-slice) of the kernels at this sample solves A x = 0."""
    if len(e1) + k2 != len(e2) + k1:
        raise ValueError("inconsistent 1-D lengths")
    return np.hstack([conv_matrix(e1, k2), -conv_matrix(e2, k1)])


def null_vector(A: np.ndarray):
    """Smallest right singular vector x of A (unit norm) and the ascending
    spectrum of the Gram matrix A^H A (squared singular values)."""
    _, s, Vh = np.linalg.svd(A, full_matrices=False)
    x = Vh[-1].conj()
    return x, (s[::-1] ** 2)


def round_operands(e: np.ndarray, fmt):
    """The matrix-core operand precision of the MFMA32 / BF16 forms: each real
    and imaginary part of the FP64 evaluation rounded to FP32 (round to
    nearest even), and for "bf16" then to bfloat16 (round to nearest even on
    the 16 dropped bits) -- the two roundings the GPU applies.  fmt None
    leaves e unchanged."""
    if fmt is None:
        return e
    def r(x):
        f = np.asarray(x, dtype=np.float64).astype(np.float32)
        if fmt == "bf16":
            u = f.view(np.uint32).astype(np.uint64)
            u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
            f = u.astype(np.uint32).view(np.float32)
        elif fmt != "f32":
            raise ValueError(fmt)
        return f.astype(np.float64)
    return r(e.real) + 1j * r(e.imag)


def sample_gram(e1: np.ndarray, e2: np.ndarray, k1: int, k2: int, fmt=None) -> np.ndarray:
    """G = A^H A for A = [C_k2(e1) | -C_k1(e2)] built from the (rounded)
    evaluations, accumulated in FP64."""
    A = sample_matrix(round_operands(e1, fmt), round_operands(e2, fmt), k1, k2)
    return A.conj().T @ A


def sample_cofactors(E1: np.ndarray, E2: np.ndarray, k1: int, k2: int, fmt=None):
    """Null vectors for every sample of one pass.

    Returns U (S x k2: cofactor slices of kernel 2), V (S x k1: slices of
    kernel 1), spectra (S x (k1+k2), ascending Gram eigenvalues).  With fmt
    ("f32" / "bf16") the stacked matrix is built from operands rounded as the
    matrix-core forms round them (round_operands); the null vector is then
    exact for those operands.
    """
    E1 = np.asarray(E1)
    E2 = np.asarray(E2)
    if E1.ndim == 2:                       # one channel
        E1, E2 = E1[None], E2[None]
    S = E1.shape[1]
    U = np.zeros((S, k2), dtype=np.complex128)
    V = np.zeros((S, k1), dtype=np.complex128)
    spec = np.zeros((S, k1 + k2))
    for j in range(S):
        # colour frames share one kernel pair: the channels' sample matrices
        # are stacked, so the Gram is the sum of the channels' Grams
        A = np.vstack([sample_matrix(round_operands(E1[c, j], fmt), round_operands(E2[c, j], fmt), k1, k2)
                       for c in range(E1.shape[0])])
        x, sp = null_vector(A)
        U[j], V[j], spec[j] = x[:k2], x[k2:], sp
    return U, V, spec


# --------------------------------------------------------------------------
# O4  cofactors evaluated on the other axis (Sec. 5: evaluating the factored
#     results on the unit circle gives scaled kernel-spectrum coefficients)
# --------------------------------------------------------------------------

def cofactor_grids(XU, XV, YU, YV, S: int):
    """S x S grids of scaled kernel spectra, indexed [i (x-sample), j (y-sample)].

      P_c[i, j] = sum_x Xc_j[x] w_i^x   (pass-X slice j evaluated along x)
      Q_c[i, j] = sum_y Yc_i[y] w_j^y   (pass-Y slice i evaluated along y)

    Kernel 1 uses the V parts, kernel 2 the U parts.  In exact arithmetic
    P_c[i,j] = c_j Khat_c[i,j] and Q_c[i,j] = d_i Khat_c[i,j] with
    Khat_c[i,j] = sum_{y,x} K_c[y,x] w_j^y w_i^x.
    """
    k1, k2 = XV.shape[1], XU.shape[1]
    W1 = unit_roots_matrix(S, k1)
    W2 = unit_roots_matrix(S, k2)
    P1 = W1 @ XV.T
    P2 = W2 @ XU.T
    Q1 = YV @ W1.T
    Q2 = YU @ W2.T
    return (P1, P2), (Q1, Q2)


# --------------------------------------------------------------------------
# O5  scale fix (Sec. 4: run the evaluation in both orders and combine by
#     least squares; Sec. 5: 2t unknowns, t x t equations, solved by SVD)
# --------------------------------------------------------------------------

def scale_system(P, Q) -> np.ndarray:
    """Rows a_j P_c[i,j] - b_i Q_c[i,j] for c in {1,2}, i, j in [0, S): the
    (2 S^2) x (2S) matrix M with unknown z = (a_0..a_{S-1}, b_0..b_{S-1})."""
    S = P[0].shape[0]
    rows = []
    for Pc, Qc in zip(P, Q):
        for i in range(S):
            for j in range(S):
                r = np.zeros(2 * S, dtype=np.complex128)
                r[j] = Pc[i, j]
                r[S + i] = -Qc[i, j]
                rows.append(r)
    return np.array(rows)


def scale_fix(P, Q):
    """(a, b) minimising sum |a_j P - b_i Q|^2 with ||(a,b)|| = 1: the smallest
    right singular vector of the scale system.  Also returns the ascending
    spectrum of its Gram matrix."""
    z, spec = null_vector(scale_system(P, Q))
    S = P[0].shape[0]
    return z[:S], z[S:], spec


# --------------------------------------------------------------------------
# O6  assembly and inverse DFT (Sec. 5: normalise, average the two estimates;
#     abstract: the inverse transform of the kernel matrices gives the kernels)
# --------------------------------------------------------------------------

def assemble_kernel(Pc, Qc, a, b, k: int):
    """Average the two scaled estimates, inverse-DFT, crop, normalise.

    Khat[i,j] = (a_j P[i,j] + b_i Q[i,j]) / 2;
    K_full[y,x] = (1/S^2) sum_{i,j} Khat[i,j] w_j^{-y} w_i^{-x}, y, x < S;
    K = Re( K_full[:k, :k] / sum(K_full[:k, :k]) ).
    Returns K and diagnostics (relative imaginary norm after normalisation,
    fraction of energy outside the k x k support).
    """
    S = Pc.shape[0]
    Khat = 0.5 * (a[None, :] * Pc + b[:, None] * Qc)      # [i, j]
    Winv = np.conj(unit_roots_matrix(S, S))                # [i, t] = w_i^{-t}
    # K_full[y, x] = (1/S^2) sum_j sum_i w_j^{-y} Khat[i, j] w_i^{-x}
    K_full = (Winv.T @ Khat.T @ Winv) / (S * S)
    Kc = K_full[:k, :k]
    s = Kc.sum()
    Kn = Kc / s
    out = np.sum(np.abs(K_full) ** 2) - np.sum(np.abs(Kc) ** 2)
    diag = dict(imag=float(np.linalg.norm(Kn.imag) / max(np.linalg.norm(Kn.real), 1e-300)),
                outside=float(out / max(np.sum(np.abs(K_full) ** 2), 1e-300)),
                khat=Khat)
    return np.real(Kn), diag


# --------------------------------------------------------------------------
# O7  latent recovery (Sec. 4: divide by the kernel in the Fourier domain;
#     here with both channels and a Tikhonov term lambda)
# --------------------------------------------------------------------------

def deconvolve(B1, B2, K1, K2, m: int, n: int, lam: float = 0.0):
    """L = crop_{m x n} IFFT2( (conj Kh1 Bh1 + conj Kh2 Bh2) / (|Kh1|^2+|Kh2|^2+lam) )
    on the Py x Px grid, Py = smooth7(max H_c), Px = smooth7(max W_c).
    Colour frames ([channel][y][x]) are divided channel by channel."""
    B1 = np.asarray(B1, dtype=np.float64)
    B2 = np.asarray(B2, dtype=np.float64)
    if B1.ndim == 3:
        return np.stack([deconvolve(B1[c], B2[c], K1, K2, m, n, lam) for c in range(B1.shape[0])])
    Py = smooth7(max(B1.shape[0], B2.shape[0]))
    Px = smooth7(max(B1.shape[1], B2.shape[1]))
    s = (Py, Px)
    Bh1, Bh2 = np.fft.fft2(B1, s=s), np.fft.fft2(B2, s=s)
    Kh1, Kh2 = np.fft.fft2(K1, s=s), np.fft.fft2(K2, s=s)
    Lh = (np.conj(Kh1) * Bh1 + np.conj(Kh2) * Bh2) / (np.abs(Kh1) ** 2 + np.abs(Kh2) ** 2 + lam)
    return np.real(np.fft.ifft2(Lh))[:m, :n]


# --------------------------------------------------------------------------
# whole method
# --------------------------------------------------------------------------

def recover_kernels(B1, B2, m: int, n: int, S: int = 0, full: bool = False, gram_fmt=None):
    """Kernels K1, K2 from the blurred pair (O1-O6).  With ``full`` also
    returns every intermediate in a dict.  gram_fmt ("f32" / "bf16") rounds
    the per-sample operands as the matrix-core precision forms do."""
    B1 = np.asarray(B1)
    B2 = np.asarray(B2)
    k1, k2 = kernel_sizes(B1.shape[-2:], B2.shape[-2:], m, n)
    S = S or max(k1, k2)
    if S < max(k1, k2):
        raise ValueError("S must be >= max kernel size")
    if B1.ndim == 3:
        # colour frames [channel][y][x]: every channel evaluated; the samples'
        # null vectors come from the channels' stacked sample matrices
        ev1 = [unit_circle_eval(B1[c], S) for c in range(B1.shape[0])]
        ev2 = [unit_circle_eval(B2[c], S) for c in range(B2.shape[0])]
        EX1, EY1 = np.stack([e[0] for e in ev1]), np.stack([e[1] for e in ev1])
        EX2, EY2 = np.stack([e[0] for e in ev2]), np.stack([e[1] for e in ev2])
    else:
        EX1, EY1 = unit_circle_eval(B1, S)
        EX2, EY2 = unit_circle_eval(B2, S)
    XU, XV, Xspec = sample_cofactors(EX1, EX2, k1, k2, gram_fmt)
    YU, YV, Yspec = sample_cofactors(EY1, EY2, k1, k2, gram_fmt)
    P, Q = cofactor_grids(XU, XV, YU, YV, S)
    a, b, Hspec = scale_fix(P, Q)
    K1, d1 = assemble_kernel(P[0], Q[0], a, b, k1)
    K2, d2 = assemble_kernel(P[1], Q[1], a, b, k2)
    if not full:
        return K1, K2
    return K1, K2, dict(k1=k1, k2=k2, S=S, EX=(EX1, EX2), EY=(EY1, EY2),
                        XU=XU, XV=XV, YU=YU, YV=YV, Xspec=Xspec, Yspec=Yspec,
                        P=P, Q=Q, a=a, b=b, Hspec=Hspec, diag=(d1, d2))


def deblur(B1, B2, m: int, n: int, S: int = 0, lam: float = 0.0, gram_fmt=None):
    """Latent frame and kernels from the blurred pair (O1-O7)."""
    K1, K2 = recover_kernels(B1, B2, m, n, S, gram_fmt=gram_fmt)
    return deconvolve(B1, B2, K1, K2, m, n, lam), K1, K2
