"""Slow, plain FP64 CPU oracle for coprime-blurred-pair (CBP) deblurring.

TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
benchmark's CPU-baseline leg may import anything from this package; the
product path (the HIP library and its Python binding) never does, and this
package imports nothing from it.

Modules
  cbp    -- the method, step by step, in the paper's order (Sec. 4 and 5):
            unit-circle evaluation, per-sample cofactor null vectors, the
            two-order scale fix, assembly + inverse DFT, Fourier division.
  tls2d  -- an independent route: the 2-D null space of the full system
            B1 (x) U = B2 (x) V by brute force.
  exact  -- exact rational / Gaussian-rational arithmetic (SymPy) on tiny
            integer inputs: GCD, resultants, exact null spaces.
  learned -- the learned form: spectrum features, the MLP (forward, backward,
            loss), the weighted scale fix and the weighted, regularised
            assembly; it reduces to cbp's steps at unit weights.
  sizes  -- blind kernel-size estimation: the per-sample nullity test over
            trial sizes (the kernel degree stage of Sec. 4 and Sec. 5).
  variants -- the paper's narrower steps: single-channel division B1 / K1,
            the k1-only scale least squares, the one-axis scale fix.
  encoder -- the CBP encoder (Philox4x64-10 kernel draws, the coprimality
            redraw rule, the full-convolution blur) and the multi-level
            8-bit streams with dropped least significant bits (Sec. 3).
"""

from . import cbp, tls2d, exact, learned, sizes, variants, encoder  # noqa: F401
