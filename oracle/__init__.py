"""CPU FP64 oracle for the MLFFT / block-Toeplitz solver path.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path imports, calls or
executes this package: only the test-suite, the smoke check and the benchmark's
CPU-baseline leg do.  It shares no code with the HIP library (no kernels,
headers, helpers or constant tables); the two meet only at the seeded inputs
produced by ``paper_2506_20350_amd.synth``, which the oracle never imports
either (callers pass arrays in).

Everything here is plain NumPy/SciPy in complex128 / float64 and follows the
paper's definitions directly, with no blocking or fusion:

  toeplitz   dense assembly of the two-level block-Toeplitz Z_A (eq. Tblock),
             circulant embedding (eqs. scalarC, cT1, circL1, circL2), the
             blockwise multilevel DFT (eqs. F1, F2, App. A/B semantics) and
             the three matvecs (dense, direct block convolution, FFT form of
             eq. multL).
  direct     dense LU solve and the block Rybicki recursion (Sec. III-D,
             eqs. xmpo, xi, GM1, HM1, HM, GH).
  precond    Kindt self-block preconditioner (Sec. III-B) and the two-level
             Strang block-circulant preconditioner (a reading, see its module).
  krylov     restarted right-preconditioned GMRES / flexible GMRES per RHS
             (Sec. III-C) and the global (vectorised) variant (eq. ZIVvec).
  border     the full matrix with border blocks Z_B, Z_C (eq. Zblock): its
             blockwise product (eq. ZIVblock), the Schur-complement direct
             solve around the block Rybicki recursion (Sec. III-E) and the
             block-diagonal preconditioner P_X (Sec. III-B).
  spectrum   singular values of P^{-1} Z by a randomized range finder with a
             given test matrix (Sec. V; Halko, Martinsson and Tropp).
  net        FP64 3x3 convolution network used as a learned correction of the
             block-circulant preconditioner: forward, backward, loss, Adam and
             bfloat16 round-to-nearest-even emulation.

Every function names the passage of the paper it follows.  Readings of points
where the paper is silent are stated where they are used.
"""
