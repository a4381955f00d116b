"""Pins of the oracle's estimator against brute-force harmonic fields.

Exact recovery (spin 2): a field whose a_lm vanish beyond a small l lies in a
finite-dimensional space; once the stencil carries at least that many real
values the Gaussian conditional mean reproduces the field anywhere and the
kriging variance vanishes (up to the nugget).  This fixes every spin-2 phase
sign: a covariance with a wrong parallel-transport sign spans another space and
does not reproduce the field.

Calibration (paper Sec. 3.2: the error divided by the predicted deviation is a
unit normal).  The oracle's estimate is linear in the map, so interpolating
each harmonic basis field once gives the error of every realisation as a
matrix product.  Two checks follow:
  * deterministic: with the MSE variance (var_kind="mse"), the expected squared
    error sum_k sigma_k^2 e_k^2 over the prior of the harmonic coefficients must
    equal the predicted variance at every target;
  * sampled: z over >= 1e4 independent realisations has mean z^2 in [0.95, 1.05].
The truth and the basis fields come from wigner (explicit Wigner-d sums), not
from the oracle's correlation functions or covariance assembly.
"""
import numpy as np
import pytest

from oracle import correlation, healpix, kriging, wigner


def _spin0_basis(lmax, lmin=1):
    """(l, m, unit a_lm value) of the real basis of a real spin-0 field."""
    out = []
    for l in range(lmin, lmax + 1):
        out.append((l, 0, 1.0))
        for m in range(1, l + 1):
            out.append((l, m, 1.0))
            out.append((l, m, 1j))
    return out


def _alm(lmax, l, m, v):
    a = np.zeros((lmax + 1, lmax + 1), complex)
    a[l, m] = v
    return a


def _prior_sd(cl, l, m):
    """Standard deviation of the real coefficient: a_l0 ~ N(0, C_l); for m > 0
    the real and imaginary parts are N(0, C_l / 2)."""
    return np.sqrt(cl[l] if m == 0 else 0.5 * cl[l])


# ------------------------------------------------------------------ exact recovery, spin 2
def _random_elm(rng, cl, lmax):
    a = np.zeros((lmax + 1, lmax + 1), complex)
    for l in range(2, lmax + 1):
        a[l, 0] = rng.normal() * np.sqrt(cl[l])
        for m in range(1, l + 1):
            a[l, m] = (rng.normal() + 1j * rng.normal()) * np.sqrt(0.5 * cl[l])
    return a


@pytest.mark.parametrize("K", [8, 12])
def test_spin2_exact_recovery_full_mode(K):
    """E modes with l in {2, 3}: 5 + 7 = 12 real degrees of freedom, 2K >= 16
    stencil values, so (Q, U) is recovered at arbitrary directions."""
    N, lmax = 4, 3
    ee = np.array([0.0, 0.0, 1.0, 0.6])
    bb = np.zeros(lmax + 1)
    rng = np.random.default_rng(21 + K)
    elm = _random_elm(rng, ee, lmax)
    thp, php = healpix.pix2ang(N, np.arange(healpix.npix(N)))
    q, u = wigner.resum_spin2(elm, 0 * elm, thp, php)
    th, ph = np.arccos(rng.uniform(-1, 1, 25)), rng.uniform(0, 2 * np.pi, 25)
    tq, tu = wigner.resum_spin2(elm, 0 * elm, th, ph)
    v, var, _ = kriging.interpolate(N, (ee, bb), K, 2, (q, u), th, ph, mode="full")
    s = np.sqrt(correlation.xi_pm(np.zeros(1), ee, bb)[2])
    assert np.max(np.abs(v[:, 0] - tq)) < 1e-3 * s
    assert np.max(np.abs(v[:, 1] - tu)) < 1e-3 * s
    assert np.all(var < 1e-6 * s ** 2)


def test_spin2_exact_recovery_paper_mode():
    """C^EE = C^BB makes xi_- vanish, so the paper's Hermitian estimator is the
    exact conditional mean; E and B with l in {2, 3} give 24 real degrees of
    freedom, 2K = 32 values recover them in both modes, and the modes agree."""
    N, lmax, K = 4, 3, 16
    cl = np.array([0.0, 0.0, 1.0, 0.5])
    rng = np.random.default_rng(31)
    elm, blm = _random_elm(rng, cl, lmax), _random_elm(rng, cl, lmax)
    thp, php = healpix.pix2ang(N, np.arange(healpix.npix(N)))
    q, u = wigner.resum_spin2(elm, blm, thp, php)
    th, ph = np.arccos(rng.uniform(-1, 1, 20)), rng.uniform(0, 2 * np.pi, 20)
    tq, tu = wigner.resum_spin2(elm, blm, th, ph)
    s = np.sqrt(correlation.xi_pm(np.zeros(1), cl, cl)[2])
    res = {}
    for mode in ("paper", "full"):
        v, var, _ = kriging.interpolate(N, (cl, cl), K, 2, (q, u), th, ph, mode=mode)
        assert np.max(np.abs(v[:, 0] - tq)) < 1e-3 * s, mode
        assert np.max(np.abs(v[:, 1] - tu)) < 1e-3 * s, mode
        assert np.all(var < 1e-6 * s ** 2), mode
        res[mode] = v
    assert np.allclose(res["paper"], res["full"], atol=1e-9 * s)


def test_spin2_recovery_fails_with_flipped_phase(monkeypatch):
    """The recovery pin above is sensitive to the transport phases: with the
    sign of the bearing difference flipped in <P_a P_b*> the same field is no
    longer reproduced (a planted mistake, on the CPU)."""
    N, lmax, K = 4, 3, 12
    ee = np.array([0.0, 0.0, 1.0, 0.6])
    bb = np.zeros(lmax + 1)
    rng = np.random.default_rng(33)
    elm = _random_elm(rng, ee, lmax)
    thp, php = healpix.pix2ang(N, np.arange(healpix.npix(N)))
    q, u = wigner.resum_spin2(elm, 0 * elm, thp, php)
    th, ph = np.arccos(rng.uniform(-1, 1, 25)), rng.uniform(0, 2 * np.pi, 25)
    tq, tu = wigner.resum_spin2(elm, 0 * elm, th, ph)
    orig = kriging.spin2_gamma_pi

    def flipped(n, et, ep, cl_ee, cl_bb):
        G, P, xp0 = orig(n, et, ep, cl_ee, cl_bb)
        return np.conj(G), P, xp0

    monkeypatch.setattr(kriging, "spin2_gamma_pi", flipped)
    v, _, _ = kriging.interpolate(N, (ee, bb), K, 2, (q, u), th, ph, mode="full")
    s = np.sqrt(correlation.xi_pm(np.zeros(1), ee, bb)[2])
    assert np.max(np.abs(np.concatenate([v[:, 0] - tq, v[:, 1] - tu]))) > 1e-2 * s


# ------------------------------------------------------------------ calibration
def _errors_spin0(N, cl, K, th, ph):
    """Error of the oracle's estimate per target and basis field, the basis
    standard deviations, and the oracle's MSE variance."""
    lmax = len(cl) - 1
    thp, php = healpix.pix2ang(N, np.arange(healpix.npix(N)))
    basis = _spin0_basis(lmax)
    E = np.empty((len(th), len(basis)))
    sd = np.empty(len(basis))
    var = None
    for k, (l, m, v) in enumerate(basis):
        a = _alm(lmax, l, m, v)
        est, var, _ = kriging.interpolate(N, cl, K, 0, wigner.resum_spin0(a, thp, php), th, ph,
                                          var_kind="mse")
        E[:, k] = est - wigner.resum_spin0(a, th, ph)
        sd[k] = _prior_sd(cl, l, m)
    return E, sd, var


def _errors_spin2(N, ee, bb, K, th, ph):
    """As _errors_spin0 for (Q, U): rows are Q errors then U errors."""
    lmax = len(ee) - 1
    thp, php = healpix.pix2ang(N, np.arange(healpix.npix(N)))
    basis = [("E",) + b for b in _spin0_basis(lmax, 2)] + [("B",) + b for b in _spin0_basis(lmax, 2)]
    n = len(th)
    E = np.empty((2 * n, len(basis)))
    sd = np.empty(len(basis))
    var = None
    for k, (kind, l, m, v) in enumerate(basis):
        a = _alm(lmax, l, m, v)
        e, b = (a, 0 * a) if kind == "E" else (0 * a, a)
        q, u = wigner.resum_spin2(e, b, thp, php)
        est, var, _ = kriging.interpolate(N, (ee, bb), K, 2, (q, u), th, ph, mode="full",
                                          var_kind="mse")
        tq, tu = wigner.resum_spin2(e, b, th, ph)
        E[:n, k] = est[:, 0] - tq
        E[n:, k] = est[:, 1] - tu
        sd[k] = _prior_sd(ee if kind == "E" else bb, l, m)
    return E, sd, np.concatenate([var[:, 0], var[:, 1]])


def _check(E, sd, var, seed):
    # deterministic: expected squared error under the prior equals the MSE variance
    expect = (E ** 2) @ (sd ** 2)
    assert np.allclose(expect / var, 1.0, rtol=0, atol=1e-7), np.max(np.abs(expect / var - 1))
    # sampled: 20,000 independent realisations per target
    rng = np.random.default_rng(seed)
    g = rng.normal(size=(len(sd), 20000)) * sd[:, None]
    z = (E @ g) / np.sqrt(var)[:, None]
    assert z.size >= 10000
    assert 0.95 < np.mean(z ** 2) < 1.05
    assert abs(np.mean(z)) < 0.03
    # every target separately (20,000 samples each: sd of mean z^2 is 0.01)
    assert np.all(np.abs(np.mean(z ** 2, axis=1) - 1.0) < 0.06)


def test_calibration_spin0():
    N, K, lmax = 4, 8, 6
    ell = np.arange(lmax + 1, dtype=float)
    cl = np.zeros(lmax + 1)
    cl[1:] = 1.0 / (ell[1:] + 1.0) ** 2
    rng = np.random.default_rng(10)
    th, ph = np.arccos(rng.uniform(-1, 1, 12)), rng.uniform(0, 2 * np.pi, 12)
    _check(*_errors_spin0(N, cl, K, th, ph), seed=100)


def test_calibration_spin2_full():
    """xi_- != 0 (C^BB = 0.3 C^EE): the full-mode estimator and its MSE variance."""
    N, K, lmax = 4, 8, 5
    ell = np.arange(lmax + 1, dtype=float)
    ee = np.zeros(lmax + 1)
    ee[2:] = 1.0 / (ell[2:] + 1.0) ** 2
    bb = 0.3 * ee
    rng = np.random.default_rng(11)
    th, ph = np.arccos(rng.uniform(-1, 1, 8)), rng.uniform(0, 2 * np.pi, 8)
    _check(*_errors_spin2(N, ee, bb, K, th, ph), seed=101)


def test_calibration_detects_dropped_term(monkeypatch):
    """A planted mistake in the oracle (the l = 1 term dropped from the
    correlation function used for the covariance) breaks the deterministic
    calibration."""
    N, K, lmax = 4, 8, 6
    ell = np.arange(lmax + 1, dtype=float)
    cl = np.zeros(lmax + 1)
    cl[1:] = 1.0 / (ell[1:] + 1.0) ** 2
    rng = np.random.default_rng(12)
    th, ph = np.arccos(rng.uniform(-1, 1, 6)), rng.uniform(0, 2 * np.pi, 6)
    orig = kriging.zeta

    def dropped(u, c):
        c = np.array(c, dtype=float)
        c[1] = 0.0
        return orig(u, c)

    monkeypatch.setattr(kriging, "zeta", dropped)
    E, sd, var = _errors_spin0(N, cl, K, th, ph)
    expect = (E ** 2) @ (sd ** 2)
    assert np.max(np.abs(expect / var - 1.0)) > 1e-2
