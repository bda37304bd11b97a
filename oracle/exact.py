"""Exact arithmetic checks on tiny integer inputs (SymPy over Q and Q(i)).

TEST INFRASTRUCTURE ONLY.

Images are bivariate polynomials (Sec. 4, eq. 2): pixel [y][x] is the
coefficient of y^r x^c.  Blurring is polynomial multiplication, so for
B_c = L (x) K_c the latent is the GCD of b1 and b2 up to a constant (eq. 4)
and the kernels are the cofactors.  These functions compute, exactly:
  * gcd(b1, b2) and the two resultants of k1, k2 (coprimality, Sec. 3);
  * the null space of the 2-D system B1 (x) U = B2 (x) V over Q;
  * the per-sample null spaces of the 1-D systems at the 4th roots of unity
    {1, -i, -1, i}, where all evaluations are Gaussian integers (Sec. 4: the
    2-D problem decomposed into 1-D GCD problems at unit-circle samples).
"""

from __future__ import annotations

import numpy as np
import sympy as sp

X, Y = sp.symbols("x y")


def to_poly(M) -> sp.Poly:
    """b(x, y) = sum_{r,c} M[r][c] y^r x^c."""
    M = np.asarray(M)
    expr = sum(int(M[r, c]) * Y ** r * X ** c
               for r in range(M.shape[0]) for c in range(M.shape[1]))
    return sp.Poly(expr, X, Y, domain="QQ")


def exact_blur(L, K) -> np.ndarray:
    """Full convolution by polynomial multiplication, returned as an int array."""
    p = to_poly(L) * to_poly(K)
    H = L.shape[0] + K.shape[0] - 1
    W = L.shape[1] + K.shape[1] - 1
    out = np.zeros((H, W), dtype=object)
    for (cx, cy), v in p.terms():
        out[cy, cx] = int(v)
    return out


def gcd_and_resultants(B1, B2, K1, K2):
    """(gcd(b1, b2), Res_x(k1, k2), Res_y(k1, k2)) as SymPy expressions."""
    g = sp.gcd(to_poly(B1), to_poly(B2))
    k1, k2 = to_poly(K1).as_expr(), to_poly(K2).as_expr()
    return g, sp.resultant(k1, k2, X), sp.resultant(k1, k2, Y)


def null_space_2d(B1, B2, k1: int, k2: int):
    """Exact basis of {(U, V): B1 (x) U - B2 (x) V = 0}, U k2 x k2, V k1 x k1."""
    H1, W1 = B1.shape
    Ho, Wo = H1 + k2 - 1, W1 + k2 - 1
    cols = []
    for B, k, sign in ((B1, k2, 1), (B2, k1, -1)):
        H, W = B.shape
        for p in range(k):
            for q in range(k):
                img = [[0] * Wo for _ in range(Ho)]
                for r in range(H):
                    for c in range(W):
                        img[p + r][q + c] = sign * int(B[r, c])
                cols.append([v for row in img for v in row])
    A = sp.Matrix(cols).T
    return A.nullspace()


def _root4(j: int):
    """w_j = exp(-2 pi i j / 4) = (-i)^j, exactly."""
    return [sp.Integer(1), -sp.I, sp.Integer(-1), sp.I][j % 4]


def evaluate_exact(B, j: int, axis: str):
    """Pass X (axis='x'): e[x] = sum_y B[y,x] w_j^y;  pass Y: e[y] = sum_x B[y,x] w_j^x."""
    w = _root4(j)
    B = np.asarray(B)
    H, W = B.shape
    if axis == "x":
        return [sp.expand(sum(int(B[y, x]) * w ** y for y in range(H))) for x in range(W)]
    return [sp.expand(sum(int(B[y, x]) * w ** x for x in range(W))) for y in range(H)]


def sample_null_space(B1, B2, k1: int, k2: int, j: int, axis: str):
    """Exact null space over Q(i) of [C_k2(e1) | -C_k1(e2)] at w_j (S = 4)."""
    e1 = evaluate_exact(B1, j, axis)
    e2 = evaluate_exact(B2, j, axis)
    rows = len(e1) + k2 - 1
    A = sp.zeros(rows, k1 + k2)
    for c in range(k2):
        for t, v in enumerate(e1):
            A[t + c, c] = v
    for c in range(k1):
        for t, v in enumerate(e2):
            A[t + c, k2 + c] = -v
    return [sp.Matrix([sp.nsimplify(sp.expand(v)) for v in vec]) for vec in A.nullspace(simplify=True)]


def kernel_slice_exact(K, j: int, axis: str):
    """k(w_j, .) (axis 'x': evaluated along y) or k(., w_j) (axis 'y') exactly."""
    return evaluate_exact(K, j, axis)


def to_complex(vec) -> np.ndarray:
    return np.array([complex(sp.N(v, 30)) for v in vec], dtype=np.complex128)
