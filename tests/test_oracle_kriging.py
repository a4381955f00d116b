"""Pins of the oracle's kriging steps (paper Sec. 2.1 and 2.4)."""
import numpy as np
import pytest

from oracle import correlation, healpix, kriging, wigner


def _cl(lmax, sig=0.02):
    ell = np.arange(lmax + 1, dtype=float)
    cl = np.zeros(lmax + 1)
    cl[2:] = 1e3 / (ell[2:] * (ell[2:] + 1)) * np.exp(-(ell[2:] * sig) ** 2)
    return cl


def test_k1_closed_form():
    """K = 1: w = rho / (1 + n), var = sigma0^2 (1 - rho^2 / (1 + n))."""
    N, cl = 16, _cl(40)
    m = np.random.default_rng(0).normal(size=healpix.npix(N))
    th, ph = np.array([0.7, 2.0]), np.array([1.1, 4.0])
    v, var, st = kriging.interpolate(N, cl, 1, 0, m, th, ph)
    t = healpix.ang2vec(th, ph)
    p = healpix.pix2vec(N, st[:, 0])
    z, _ = correlation.zeta(0.5 * np.sum((t - p) ** 2, -1), cl)
    s2 = correlation.zeta(np.zeros(1), cl)[0][0]
    rho = z / s2
    e = kriging.EPS_F64
    assert np.allclose(v, rho / (1 + e) * m[st[:, 0]], rtol=1e-13)
    assert np.allclose(var, s2 * (1 - rho ** 2 / (1 + e)), rtol=1e-12)


def test_block_inverse_identities():
    """Sec. 2.1: for V = [[1, B^T], [B, S]] the inverse W has
    W_00 = 1 / (1 - B^T S^-1 B) and W_0i = -(S^-1 B)_i / (1 - B^T S^-1 B); the
    oracle's weights and variance are -W_0i / W_00 and sigma0^2 / W_00."""
    N, K, cl = 16, 5, _cl(30)
    th, ph = 1.3, 0.4
    st, _ = kriging.stencil(N, th, ph, K)
    pts = np.concatenate([healpix.ang2vec(th, ph)[None], healpix.pix2vec(N, st)])
    u = 0.5 * np.sum((pts[:, None] - pts[None]) ** 2, -1)
    s2 = correlation.zeta(np.zeros(1), cl)[0][0]
    V = correlation.zeta(u, cl)[0] / s2
    W = np.linalg.inv(V)
    vals = np.random.default_rng(1).normal(size=K)
    v, var, _ = kriging.interpolate(N, cl, K, 0, np.zeros(healpix.npix(N)), [th], [ph],
                                    nugget="on_failure", stencil_idx=st[None])
    m = np.zeros(healpix.npix(N))
    m[st] = vals
    v, var, _ = kriging.interpolate(N, cl, K, 0, m, [th], [ph], nugget="on_failure",
                                    stencil_idx=st[None])
    w_ref = -W[0, 1:] / W[0, 0]
    assert v[0] == pytest.approx(w_ref @ vals, rel=1e-9, abs=1e-12)
    assert var[0] == pytest.approx(s2 / W[0, 0], rel=1e-7)


def test_pixel_centre_reproduction():
    """At a pixel centre the estimate reproduces the pixel (up to the nugget) and
    the variance is at most n sigma0^2."""
    N, K, cl = 32, 12, _cl(60)
    rng = np.random.default_rng(2)
    pix = rng.choice(healpix.npix(N), 20, replace=False)
    th, ph = healpix.pix2ang(N, pix)
    m = rng.normal(size=healpix.npix(N))
    v, var, st = kriging.interpolate(N, cl, K, 0, m, th, ph)
    s2 = correlation.zeta(np.zeros(1), cl)[0][0]
    assert np.all(st[:, 0] == pix)
    # exact arithmetic gives var <= n sigma0^2; 1 - b^T w cancels to ~1e-12 here
    assert np.all(var <= kriging.EPS_F64 * s2 + 1e-12 * s2)
    assert np.all(var >= 0)
    # without a nugget the reproduction is exact up to rounding of a singular-free S
    v0, var0, _ = kriging.interpolate(N, cl, K, 0, m, th, ph, nugget="on_failure", stencil_idx=st)
    assert np.allclose(v0, m[pix], atol=1e-7 * np.abs(m).max())


def test_zero_deflection_identity_and_variance_relation():
    N, K, cl = 16, 9, _cl(40)
    rng = np.random.default_rng(4)
    m = rng.normal(size=healpix.npix(N))
    pix = np.arange(0, healpix.npix(N), 37)
    th, ph = healpix.pix2ang(N, pix)
    v, _, _ = kriging.interpolate(N, cl, K, 0, m, th, ph)
    assert np.allclose(v, m[pix], atol=2e-5 * np.abs(m).max())
    # var_paper - var_mse = sigma0^2 n |w|^2 >= 0 at displaced points
    th2, ph2 = th + 0.01, ph + 0.013
    _, vp, _ = kriging.interpolate(N, cl, K, 0, m, th2, ph2)
    _, vm, _ = kriging.interpolate(N, cl, K, 0, m, th2, ph2, var_kind="mse")
    assert np.all(vp >= vm) and np.all(vm > 0)


def test_exact_recovery_band_limited():
    """K >= number of modes: a field with C_l > 0 only for l <= 2 (8 modes) is
    recovered exactly by a 12-pixel stencil."""
    N, K, lmax = 8, 12, 2
    cl = np.zeros(lmax + 1)
    cl[1:] = [1.0, 0.5]
    rng = np.random.default_rng(5)
    alm = np.zeros((lmax + 1, lmax + 1), complex)
    for l in range(1, lmax + 1):
        alm[l, 0] = rng.normal() * np.sqrt(cl[l])
        for mm in range(1, l + 1):
            alm[l, mm] = (rng.normal() + 1j * rng.normal()) * np.sqrt(cl[l] / 2)
    thp, php = healpix.pix2ang(N, np.arange(healpix.npix(N)))
    m = wigner.resum_spin0(alm, thp, php)
    th, ph = rng.uniform(0.2, 2.9, 10), rng.uniform(0, 6.28, 10)
    truth = wigner.resum_spin0(alm, th, ph)
    v, var, _ = kriging.interpolate(N, cl, K, 0, m, th, ph)
    s0 = np.sqrt(correlation.zeta(np.zeros(1), cl)[0][0])
    assert np.allclose(v, truth, atol=1e-3 * s0)
    assert np.all(var < 1e-6 * s0 ** 2)
