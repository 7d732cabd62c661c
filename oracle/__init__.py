"""CPU FP64 oracle for the oblique QR factorisation Z = QR, Q^T A Q = I.

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
benchmark's CPU-baseline leg may import anything from this package; the
library (paper_1401_5171_amd) never does, and this package never imports the
library.  The two share no code: the only module both sides use is the seeded
input generator package `workloads`, which holds none of the method's
arithmetic.

Citations are to Lowery & Langou, "Stability Analysis of QR factorization in
an Oblique Inner Product" (arXiv 1401.5171): Section 1 (problem statement and
Theorem 1.1), Section 2 (CHOLQR, Algorithm 1, Theorem 2.1), Section 3
(PRE-CHOLQR, Algorithm 2), Section 4 (CHOL-EQR, Algorithm 3), Section 5
(EQR-SYEV, Algorithm 4), Section 6 (Gram-Schmidt), Section 7 (test cases and
error measures), Section 8 (performance, flop normalisation).

Modules
  reference  the acceptance oracle (CHOL-EQR, EQR-SYEV, stencil DST route)
  variants   per-algorithm FP64 references (CHOLQR, CholQR2, PRE-CHOLQR, CGS,
             MGS row/column, CGS2) and the textbook Cholesky with `info`
  exact      50-digit brute force for tiny inputs (mpmath)
  stencil    the 7-point operator: apply, dense assembly, exact eigenbasis
  metrics    orthogonality loss, residuals, condition diagnostics
  mixed      emulated reduced-precision CholQR pass (expected error level)
"""
from . import reference, variants, exact, stencil, metrics, mixed  # noqa: F401
