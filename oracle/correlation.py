"""Correlation functions of an isotropic field, evaluated exactly per pair.

Test infrastructure only (see oracle/__init__.py).

Spin 0 (paper Sec. 2.1, Eq. correlation_func):
    zeta(beta) = sum_{l=1}^{lmax} (2l+1)/(4 pi) C_l P_l(cos beta),
    sigma_0^2 = zeta(0).   The monopole is excluded, the dipole kept, as written.

Spin 2 (paper Sec. 2.2, Eq. spins_correl, with the Wigner d functions of App. B):
    xi_+(beta) = sum_{l>=2} (2l+1)/(4 pi) (C^EE_l + C^BB_l) d^l_{2,2}(beta)
    xi_-(beta) = sum_{l>=2} (2l+1)/(4 pi) (C^EE_l - C^BB_l) d^l_{2,-2}(beta)
The paper writes only the Hermitian term (xi_+, with d^l_{-s,-s} = d^l_{s,s}); the
pseudo-covariance xi_- is what an exact Gaussian conditional mean of (Q, U) also
needs; it is computed here for the full spin-2 mode (the paper mode omits it).

All functions take u = 1 - cos(beta) = |n_a - n_b|^2 / 2 rather than cos(beta):
near beta = 0 the covariances differ from their zero-lag value by O(l^2 u), and
a rounded cos(beta) would lose those digits.  The three-term l-recurrences are
rewritten for the deficits q_l = 1 - P_l and e_l = 1 - d^l_{22}, which are small
and carry full relative precision:
    (l+1) q_{l+1} = (2l+1) (u + (1-u) q_l) - l q_{l-1},          q_0 = 0, q_1 = u
    l(l-1)(l+3) e_{l+1} = (2l+1) [ (l(l+1)(1-u) - 4) e_l + l(l+1) u ]
                          - (l+1)(l-2)(l+2) e_{l-1},              e_2 = u - u^2/4
    l(l-1)(l+3) g_{l+1} = (2l+1) (l(l+1)(1-u) + 4) g_l - (l+1)(l-2)(l+2) g_{l-1},
                          g_l = d^l_{2,-2},                        g_2 = u^2/4
These follow from the standard l-recurrence of d^l_{m m'} (m = m' = 0;
m = m' = 2; m = -m' = 2) by substituting d = 1 - deficit; the constant terms
cancel exactly.  Pins: closed forms d^2, d^3, single-l spectra, and the explicit
Wigner formula in oracle/wigner.py (tests/test_oracle_correlation.py).
"""
import numpy as np


def _weights(cl, lmin):
    cl = np.asarray(cl, dtype=np.float64)
    ell = np.arange(cl.shape[-1], dtype=np.float64)
    w = (2.0 * ell + 1.0) / (4.0 * np.pi) * cl
    w[..., :lmin] = 0.0
    return w


def legendre_deficits(u, lmax):
    """Yield (l, q_l = 1 - P_l(1 - u)) for l = 0 .. lmax."""
    u = np.asarray(u, dtype=np.float64)
    q_prev = np.zeros_like(u)
    yield 0, q_prev
    if lmax < 1:
        return
    q = u.copy()
    yield 1, q
    for l in range(1, lmax):
        q_next = ((2 * l + 1) * (u + (1.0 - u) * q) - l * q_prev) / (l + 1)
        q_prev, q = q, q_next
        yield l + 1, q


def zeta(u, cl):
    """zeta(u) and the variogram gamma(u) = zeta(0) - zeta(u), spin 0.

    cl: C^TT_l for l = 0..lmax (l = 0 ignored).  Returns (zeta, gamma).
    """
    w = _weights(cl, 1)
    lmax = w.shape[-1] - 1
    u = np.asarray(u, dtype=np.float64)
    gam = np.zeros_like(u)
    for l, q in legendre_deficits(u, lmax):
        if w[l] != 0.0:
            gam += w[l] * q
    sigma2 = w.sum()
    return sigma2 - gam, gam


def d22_deficits(u, lmax):
    """Yield (l, e_l = 1 - d^l_{22}(beta)) for l = 2 .. lmax."""
    u = np.asarray(u, dtype=np.float64)
    if lmax < 2:
        return
    e_prev = np.ones_like(u)          # d^1_{22} = 0 (unused: its coefficient vanishes at l = 2)
    e = u - 0.25 * u * u
    yield 2, e
    for l in range(2, lmax):
        A = l * (l - 1) * (l + 3)
        B = (2 * l + 1)
        L2 = l * (l + 1)
        C = (l + 1) * (l - 2) * (l + 2)
        e_next = (B * ((L2 * (1.0 - u) - 4.0) * e + L2 * u) - C * e_prev) / A
        e_prev, e = e, e_next
        yield l + 1, e


def d2m2_values(u, lmax):
    """Yield (l, d^l_{2,-2}(beta)) for l = 2 .. lmax."""
    u = np.asarray(u, dtype=np.float64)
    if lmax < 2:
        return
    g_prev = np.zeros_like(u)
    g = 0.25 * u * u
    yield 2, g
    for l in range(2, lmax):
        A = l * (l - 1) * (l + 3)
        L2 = l * (l + 1)
        C = (l + 1) * (l - 2) * (l + 2)
        g_next = ((2 * l + 1) * (L2 * (1.0 - u) + 4.0) * g - C * g_prev) / A
        g_prev, g = g, g_next
        yield l + 1, g


def xi_pm(u, cl_ee, cl_bb):
    """(xi_+(u), xi_-(u), xi_+(0)) for spin 2.

    cl_ee, cl_bb: spectra for l = 0..lmax (l < 2 ignored).
    """
    wp = _weights(np.asarray(cl_ee) + np.asarray(cl_bb), 2)
    wm = _weights(np.asarray(cl_ee) - np.asarray(cl_bb), 2)
    lmax = wp.shape[-1] - 1
    u = np.asarray(u, dtype=np.float64)
    gam = np.zeros_like(u)
    for l, e in d22_deficits(u, lmax):
        if wp[l] != 0.0:
            gam += wp[l] * e
    xim = np.zeros_like(u)
    for l, g in d2m2_values(u, lmax):
        if wm[l] != 0.0:
            xim += wm[l] * g
    xp0 = wp.sum()
    return xp0 - gam, xim, xp0
