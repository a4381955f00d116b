"""Lensing pipeline steps for the oracle (test infrastructure only).

The paper's lensing pipeline (Sec. 3.1): synthesise the unlensed maps and the
deflection field d = grad(phi) from their harmonic coefficients, move every
pixel centre n to n' = cos|d| n + sin|d| d/|d| (the vector form, which needs no
special case at the poles), and interpolate the unlensed maps at n'.

* synth_points: spin-s synthesis F(n) = sum_{l,m} a_lm sY_lm(n) at arbitrary
  directions by brute force, with sY_lm from wigner.sY (the explicit Wigner-d
  formula of App. A; tiny lmax only).  The coefficients are given for m >= 0 as
  a = e + i b, where e and b are each those of a real-type field,
  e_{l,-m} = (-1)^m conj(e_lm) (likewise b).  Then
    spin 0, e = a^T:                 F = T;
    spin 1, e = -sqrt(l(l+1)) phi_lm: F = d_theta + i d_phi (the gradient of phi);
    spin 2, e = -E, b = -B:           F = Q + i U (P = sum 2a_lm 2Y_lm,
                                       2a_lm = -(E_lm + i B_lm)).
* synth_points_spin0_scipy: spin-0 synthesis with scipy's spherical harmonics
  (a library routine; usable at larger l than the explicit formula).
* lensed_directions: the vector-form displacement.

Pins (tests/test_oracle_lensing.py): spin 1 against the finite-difference
gradient of the resummed potential; spin 0 against scipy's harmonics; spin 2
against wigner.resum_spin2; the displacement preserves |n|, moves n by the
angle |d| along the bearing of d, and is the identity for d = 0.
"""
import numpy as np

from . import wigner


def _coeff(a, l, m):
    """a_{l,m} for any m from the stored m >= 0 half (real-type rule)."""
    if m >= 0:
        return a[l, m]
    return (-1) ** m * np.conj(a[l, -m])


def synth_points(spin, elm, blm, theta, phi):
    """F(theta, phi) = sum_{l, m} (e + i b)_lm sY_lm (complex; tiny lmax)."""
    theta = np.asarray(theta, dtype=np.float64)
    phi = np.asarray(phi, dtype=np.float64)
    lmax = elm.shape[0] - 1
    if blm is None:
        blm = np.zeros_like(elm)
    out = np.zeros(np.broadcast(theta, phi).shape, dtype=np.complex128)
    for l in range(abs(spin), lmax + 1):
        for m in range(-l, l + 1):
            a = _coeff(elm, l, m) + 1j * _coeff(blm, l, m)
            if a != 0:
                out += a * wigner.sY(spin, l, m, theta, phi)
    return out


def synth_points_spin0_scipy(alm, theta, phi):
    """T(theta, phi) = sum_{l,m} a_lm Y_lm with scipy's Y_lm (real field)."""
    from scipy.special import sph_harm_y
    theta = np.asarray(theta, dtype=np.float64)
    phi = np.asarray(phi, dtype=np.float64)
    lmax = alm.shape[0] - 1
    out = np.zeros(np.broadcast(theta, phi).shape, dtype=np.float64)
    for l in range(lmax + 1):
        for m in range(0, l + 1):
            if alm[l, m] == 0:
                continue
            y = sph_harm_y(l, m, theta, phi)
            term = alm[l, m] * y
            out += term.real if m == 0 else 2.0 * term.real
    return out


def lensed_directions(theta, phi, d_theta, d_phi):
    """(theta', phi') of n' = cos|d| n + sin|d| (d_theta e_theta + d_phi e_phi)/|d|."""
    theta = np.asarray(theta, dtype=np.float64)
    phi = np.asarray(phi, dtype=np.float64)
    st, ct = np.sin(theta), np.cos(theta)
    sp, cp = np.sin(phi), np.cos(phi)
    n = np.stack([st * cp, st * sp, ct], axis=-1)
    et = np.stack([ct * cp, ct * sp, -st], axis=-1)
    ep = np.stack([-sp, cp, np.zeros_like(sp)], axis=-1)
    dmod = np.hypot(d_theta, d_phi)
    safe = np.where(dmod > 0, dmod, 1.0)
    dhat = (np.asarray(d_theta)[..., None] * et + np.asarray(d_phi)[..., None] * ep) / safe[..., None]
    npr = np.cos(dmod)[..., None] * n + np.sin(dmod)[..., None] * dhat
    th2 = np.arctan2(np.hypot(npr[..., 0], npr[..., 1]), npr[..., 2])
    ph2 = np.mod(np.arctan2(npr[..., 1], npr[..., 0]), 2 * np.pi)
    return th2, ph2
