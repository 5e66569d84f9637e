"""CPU FP64 oracle for the hybrid Hermite WENO scheme with artificial linear weights
(Zhao & Qiu, arXiv 2002.08816).

TEST INFRASTRUCTURE ONLY.  This package is a plain, slow, direct transcription of the
scheme's definitions (Section 2 of the paper) used to check the GPU path.  Only the test
suite, the smoke check and the CPU-baseline leg of the benchmark may import it.  The
product path (the HIP library and its Python binding) never imports, links or calls it,
and the oracle imports nothing from the product path.

Modules
-------
exact      exact rational derivation of every reconstruction operator from its defining
           moment conditions (Section 2.1 Steps 1-2, Section 2.2 Step 5)
physics    flux functions, wave speeds and characteristic eigenvectors (eqs. euler1, euler2)
weno       smoothness-indicator based nonlinear weights (eqs. GHYZ, tao5, tao4, 99)
kxrcf      troubled-cell indicator (Remarks 1 and 3; Krivodonova et al. form)
scheme1d   one-dimensional semi-discrete operator L(U) (eq. odeH) and TVD-RK3 (eq. RK)
scheme2d   two-dimensional semi-discrete operator L(U) (eq. ode2) and TVD-RK3 (Step 6)

Parity status of every function is listed in its module docstring; the one function
whose constants no external fact fixes (the KXRCF threshold form) says
"parity unpinned" there.
"""
