"""FP64 CPU oracle for FLINTS kriging interpolation on HEALPix maps.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path (the HIP library and its
Python binding) imports, calls or links anything in this package; only the test
suite, the smoke check and the CPU-baseline leg of the benchmark do.  The oracle
shares no code with the GPU path: it is a plain, slow, step-by-step restatement of
the method (Lavaux & Wandelt, "Fast and optimal CMB lensing using statistical
interpolation on the sphere"), written in numpy/scipy in double precision.

Modules
  healpix      RING-ordered pixel centres (Gorski et al. 2005 formulas).
  correlation  correlation functions zeta (spin 0) and xi+/xi- (spin 2), evaluated
               exactly per pair by l-recurrences in the variable u = 1 - cos(beta).
  wigner       brute-force Wigner d, spin-weighted harmonics and resummation; used
               only to pin the rest of the oracle.
  kriging      stencil selection, covariance assembly, nugget, Cholesky solve and
               the interpolated value / kriging variance.

Parity status of each function is stated in its docstring; a function with no
independent pin says "parity unpinned".
"""
