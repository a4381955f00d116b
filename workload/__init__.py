"""Seeded synthetic inputs shaped like the paper's lensing workloads.

This package serves both the GPU path's tests/benchmark and the CPU oracle, so it
holds none of the interpolation method's arithmetic: it draws Gaussian a_lm for
the stated spectra, synthesises HEALPix RING maps at pixel centres, builds the
lensing deflection d = grad(phi) and the displaced target directions (paper
Sec. 3.1, vector form of the remap), and picks seeded subsets.  It shares no code
with `oracle/` or with the HIP library.

Seeds: numpy PCG64 from SeedSequence([10034984, cfg, job, stream]) with
stream 0 = a_lm, 1 = lensing potential, 2 = parity subset, 3 = random targets,
4 = arrivals.
"""
from .spectra import (cl_config1, cl_acoustic, cl_phi, deflection_rms_rad)  # noqa: F401
from .seeds import rng  # noqa: F401
