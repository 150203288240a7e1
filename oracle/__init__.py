"""CPU FP64 oracle for sgn(gamma5 Dw(mu)) b -- TEST INFRASTRUCTURE ONLY.

This package is the checker, not the product.  Only the test suite, the
smoke check and the benchmark's CPU-baseline leg may import it.  It shares no
code with the HIP library: it builds the operator from the hopping formula of
Section 1 (Wilson-Dirac operator at chemical potential), evaluates matrix
functions by the spectral definition, and runs the Krylov methods of
Sections 2-4 step by step in plain numpy/scipy.

Modules:
  dirac     -- gamma matrices, lattice geometry, dense and CSR gamma5*Dw(mu)
  sign      -- spectral sign (eig), Roberts' Newton iteration, Hermitian eigh
  freefield -- closed-form sign for unit links via the lattice Fourier transform
  krylov    -- LR deflation, two-sided Lanczos, Arnoldi, two-pass replay
  eigtrip   -- critical left/right eigentriples
  derivative-- Daleckii-Krein derivative of Re<chi, sgn(A) b>

Every function cites the passage of the paper it follows.  Functions whose
result has no independent pin say "parity unpinned" in their docstring.
"""
