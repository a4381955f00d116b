"""Brute-force Wigner d, spin-weighted harmonics and resummation (tiny l only).

Test infrastructure only (see oracle/__init__.py).  These are the independent
pins for the rest of the oracle: nothing here uses a recurrence.

* d^l_{m m'}(beta): the explicit finite-sum (Wigner) formula, in Python floats
  with exact integer factorials.  Valid and accurate for l <= ~30.
* sY(s, l, m, theta, phi) = (-1)^s sqrt((2l+1)/(4 pi)) e^{i m phi} d^l_{m,-s}(theta)
  as written in the paper's App. A (Condon-Shortley phase).
* Resummation of a field from its a_lm at arbitrary directions (paper Sec. 1 and
  Sec. 3.2: the exact method, used there as the precision benchmark).

a_lm storage convention used across the tests: complex array alm[l, m] for
0 <= m <= l (entries with m > l are zero); the field is real, so
a_{l,-m} = (-1)^m conj(a_{lm}).  Polarisation follows P = Q + iU =
sum_{lm} 2a_{lm} 2Y_{lm} with 2a_{lm} = -(E_{lm} + i B_{lm}).
"""
import math
import numpy as np


def wigner_d(l, m, mp, beta):
    """Explicit Wigner formula for d^l_{m, mp}(beta), vectorised over beta."""
    beta = np.asarray(beta, dtype=np.float64)
    if l < abs(m) or l < abs(mp):
        return np.zeros_like(beta)
    c = np.cos(0.5 * beta)
    s = np.sin(0.5 * beta)
    pref = math.sqrt(math.factorial(l + m) * math.factorial(l - m)
                     * math.factorial(l + mp) * math.factorial(l - mp))
    tot = np.zeros_like(beta)
    for k in range(0, 2 * l + 1):
        a, b, c2, d = l + mp - k, k, l - k - m, k - mp + m
        if min(a, b, c2, d) < 0:
            continue
        coef = (-1) ** (k - mp + m) * pref / (math.factorial(a) * math.factorial(b)
                                             * math.factorial(c2) * math.factorial(d))
        tot = tot + coef * c ** (2 * l + mp - m - 2 * k) * s ** (2 * k - mp + m)
    return tot


def sY(s, l, m, theta, phi):
    theta = np.asarray(theta, dtype=np.float64)
    phi = np.asarray(phi, dtype=np.float64)
    if l < abs(s) or l < abs(m):
        return np.zeros(np.broadcast(theta, phi).shape, dtype=np.complex128)
    return ((-1) ** s * math.sqrt((2 * l + 1) / (4 * math.pi))
            * np.exp(1j * m * phi) * wigner_d(l, m, -s, theta))


def resum_spin0(alm, theta, phi):
    """T(theta, phi) = sum_{l,m} a_lm Y_lm, for a real field (tiny lmax)."""
    lmax = alm.shape[0] - 1
    out = np.zeros(np.broadcast(theta, phi).shape, dtype=np.complex128)
    for l in range(lmax + 1):
        for m in range(0, l + 1):
            y = sY(0, l, m, theta, phi)
            if m == 0:
                out += alm[l, 0] * y
            else:
                out += alm[l, m] * y + (-1) ** m * np.conj(alm[l, m]) * sY(0, l, -m, theta, phi)
    return out.real


def resum_spin2(elm, blm, theta, phi):
    """(Q, U) with Q + iU = sum_{l,m} -(E_lm + i B_lm) 2Y_lm (tiny lmax)."""
    lmax = elm.shape[0] - 1
    P = np.zeros(np.broadcast(theta, phi).shape, dtype=np.complex128)
    for l in range(2, lmax + 1):
        for m in range(-l, l + 1):
            if m >= 0:
                e, b = elm[l, m], blm[l, m]
            else:
                e = (-1) ** m * np.conj(elm[l, -m])
                b = (-1) ** m * np.conj(blm[l, -m])
            P += -(e + 1j * b) * sY(2, l, m, theta, phi)
    return P.real, P.imag


def resum_spin1_gradient(plm, theta, phi, h=1e-6):
    """Gradient (d_theta, d_phi / sin theta) of a real spin-0 field by central
    finite differences of the brute-force resummation (pins the generator's
    deflection field; accuracy ~h^2)."""
    f = lambda t, p: resum_spin0(plm, t, p)
    dth = (f(theta + h, phi) - f(theta - h, phi)) / (2 * h)
    dph = (f(theta, phi + h) - f(theta, phi - h)) / (2 * h) / np.sin(theta)
    return dth, dph
