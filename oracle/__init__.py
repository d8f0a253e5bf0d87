"""FP64 CPU oracle for one-step spectral-CT reconstruction by MOCCA with
diagonal and block-diagonal step preconditioning (arXiv 1801.06263).

TEST INFRASTRUCTURE ONLY.  This package is the plain, slow, obviously correct
reference the GPU library is checked against.  Only the test suite, the
package's ``smoke()`` check and the CPU-baseline leg of the benchmark may
import or run it; the product path never does.  It shares no code with the
HIP library: both sides read inputs from the ``synth`` generator and nothing
else.

Modules
  projector  the discrete projection X of Eq. (fullModel) as an exact
             line-intersection matrix (scipy CSR), plus closed forms.
  model      softexp, the counts model (Eq. finalModel), D_TPL (Eq. DTPL),
             the matrices A(f), B(f), Z and the derivatives of Sec. II.
  spc        step lengths: diagonal SPC and the m-block-diagonal SPC of
             Sec. II, both from dense K and in factorised per-ray form.
  mocca      the CPPD step on the local convex quadratic with negative
             curvature removed (MOCCA), one inner iteration per expansion
             point.

Parity status of each function is stated in its docstring; every function is
pinned by the ``-m "not gpu"`` tests.  The paper prints no iterate values, so
the MOCCA iteration is pinned through properties the mathematics fixes: the
Fejer monotonicity and closed-form limit of the CPPD step on a fixed convex
quadratic, equality with a dense CPPD step written from the definitions, the
fixed point at the truth, rotation equivariance of block SPC and the
block-vs-diagonal claim.  The expansion point fbar_n is a reading of the
paper (it leaves it unstated).
"""
