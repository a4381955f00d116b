"""Synthetic angular power spectra standing in for the paper's CAMB spectra.

The paper's spectra come from CAMB (Sec. 3.3), which is not available; these
closed forms reproduce the shape (a damped red spectrum with acoustic-like
oscillations, a weaker partially correlated E mode, no primordial B) at the band
limits the paper uses.
"""
import numpy as np

ARCMIN = np.pi / (180.0 * 60.0)


def cl_config1(lmax, sigma_arcmin=10.0):
    """C_l = 1e3 / (l (l+1)) exp(-l^2 sigma^2), sigma = 10 arcmin taken literally, l >= 2."""
    ell = np.arange(lmax + 1, dtype=np.float64)
    cl = np.zeros(lmax + 1)
    s = sigma_arcmin * ARCMIN
    l2 = ell[2:]
    cl[2:] = 1e3 / (l2 * (l2 + 1.0)) * np.exp(-(l2 * s) ** 2)
    return cl


def cl_acoustic(lmax):
    """(TT, EE, TE, BB) with TT = 1e3 (1 + 0.5 cos(pi l / 300)) / (l (l+1)) e^{-(l/1500)^2},
    EE = 0.05 x TT with the cosine phase-shifted by pi/2, TE = 0.3 sqrt(TT EE), BB = 0; l >= 2."""
    ell = np.arange(lmax + 1, dtype=np.float64)
    tt = np.zeros(lmax + 1)
    ee = np.zeros(lmax + 1)
    l2 = ell[2:]
    env = 1e3 / (l2 * (l2 + 1.0)) * np.exp(-(l2 / 1500.0) ** 2)
    tt[2:] = (1.0 + 0.5 * np.cos(np.pi * l2 / 300.0)) * env
    ee[2:] = 0.05 * (1.0 + 0.5 * np.cos(np.pi * l2 / 300.0 + 0.5 * np.pi)) * env
    te = 0.3 * np.sqrt(tt * ee)
    bb = np.zeros(lmax + 1)
    return tt, ee, te, bb


def deflection_rms_rad(arcmin=2.5):
    return arcmin * ARCMIN


def cl_phi(lmax, rms_arcmin=2.5):
    """C^phiphi_l = A l^-4 for 2 <= l <= lmax, A set so that
    sqrt(sum (2l+1)/(4 pi) l (l+1) C^phiphi_l) = rms deflection."""
    ell = np.arange(lmax + 1, dtype=np.float64)
    shape = np.zeros(lmax + 1)
    shape[2:] = ell[2:] ** -4.0
    var1 = np.sum((2 * ell + 1) / (4 * np.pi) * ell * (ell + 1) * shape)
    return shape * (deflection_rms_rad(rms_arcmin) ** 2 / var1)
