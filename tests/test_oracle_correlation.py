"""Pins of the oracle's correlation functions (paper Eq. correlation_func and
Eq. spins_correl; Wigner d of App. B) against closed forms and the explicit
Wigner formula."""
import numpy as np
import pytest

from oracle import correlation, wigner

U = np.array([0.0, 1e-9, 1e-5, 3e-3, 0.1, 0.7, 1.3, 1.99])


@pytest.mark.parametrize("l", range(1, 12))
def test_single_l_spin0(l):
    cl = np.zeros(l + 1)
    cl[l] = 2.5
    z, gam = correlation.zeta(U, cl)
    beta = np.arccos(1 - U)
    ref = (2 * l + 1) / (4 * np.pi) * 2.5 * wigner.wigner_d(l, 0, 0, beta)
    assert np.allclose(z, ref, rtol=0, atol=1e-13)
    # deficit form: gamma = zeta(0) - zeta(u), exactly zero at u = 0
    assert gam[0] == 0.0


@pytest.mark.parametrize("l", range(2, 12))
def test_single_l_spin2(l):
    ee = np.zeros(l + 1)
    bb = np.zeros(l + 1)
    ee[l], bb[l] = 1.7, 0.4
    xp, xm, xp0 = correlation.xi_pm(U, ee, bb)
    beta = np.arccos(1 - U)
    f = (2 * l + 1) / (4 * np.pi)
    assert np.allclose(xp, f * 2.1 * wigner.wigner_d(l, 2, 2, beta), atol=1e-13)
    assert np.allclose(xm, f * 1.3 * wigner.wigner_d(l, 2, -2, beta), atol=1e-13)
    assert xp0 == pytest.approx(f * 2.1, rel=1e-15)
    assert xm[0] == 0.0


def test_l2_closed_forms():
    """d^2_{22} = ((1+cos b)/2)^2 and d^2_{2,-2} = ((1-cos b)/2)^2."""
    cl = np.zeros(3)
    cl[2] = 4 * np.pi / 5
    xp, xm, _ = correlation.xi_pm(U, cl, np.zeros(3))
    x = 1 - U
    assert np.allclose(xp, ((1 + x) / 2) ** 2, atol=1e-15)
    assert np.allclose(xm, ((1 - x) / 2) ** 2, atol=1e-15)


def test_legendre_sum_rule():
    """sum_l (2l+1) P_l(1) = (lmax+1)^2 and the monopole is excluded."""
    lmax = 50
    cl = np.ones(lmax + 1) * 4 * np.pi
    z, _ = correlation.zeta(np.zeros(1), cl)
    assert z[0] == pytest.approx((lmax + 1) ** 2 - 1, rel=1e-14)


def test_deficit_precision_vs_longdouble():
    """The u-form keeps relative precision of zeta(0) - zeta(u) at small u."""
    lmax = 600
    ell = np.arange(lmax + 1)
    cl = np.zeros(lmax + 1)
    cl[1:] = 1.0 / (ell[1:] * (ell[1:] + 1.0))
    u = np.array([1e-12, 1e-9, 1e-7, 1e-5])
    _, gam = correlation.zeta(u, cl)
    ul = u.astype(np.longdouble)
    w = ((2 * ell + 1) / (4 * np.pi) * cl).astype(np.longdouble)
    P_prev = np.ones_like(ul)
    P = 1 - ul
    g = w[1] * (1 - P)
    for l in range(1, lmax):
        Pn = ((2 * l + 1) * (1 - ul) * P - l * P_prev) / (l + 1)
        P_prev, P = P, Pn
        g += w[l + 1] * (1 - P)
    # long double still cancels in 1 - P at u = 1e-12 only to ~1e-19/1e-12; compare
    # where the reference itself is good to better than 1e-6 relative
    ok = u >= 1e-9
    assert np.allclose(gam[ok], g[ok].astype(float), rtol=1e-8)
