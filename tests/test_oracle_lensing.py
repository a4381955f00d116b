"""Pins of the oracle's lensing steps (paper Sec. 3.1): spin-s synthesis at
arbitrary directions and the vector-form displacement."""
import numpy as np

from oracle import healpix, lensing, wigner


def _alm(rng, lmax, lmin=0):
    a = np.zeros((lmax + 1, lmax + 1), complex)
    for l in range(lmin, lmax + 1):
        a[l, 0] = rng.normal()
        for m in range(1, l + 1):
            a[l, m] = rng.normal() + 1j * rng.normal()
    return a


def test_spin0_matches_scipy_harmonics():
    rng = np.random.default_rng(1)
    a = _alm(rng, 8)
    th, ph = np.arccos(rng.uniform(-1, 1, 50)), rng.uniform(0, 2 * np.pi, 50)
    f = lensing.synth_points(0, a, None, th, ph)
    assert np.max(np.abs(f.imag)) < 1e-12
    assert np.allclose(f.real, lensing.synth_points_spin0_scipy(a, th, ph), atol=1e-11)
    assert np.allclose(f.real, wigner.resum_spin0(a, th, ph), atol=1e-11)


def test_spin1_is_the_gradient():
    """e = -sqrt(l(l+1)) phi_lm gives d_theta + i d_phi = grad(phi) (checked
    against central differences of the resummed potential)."""
    rng = np.random.default_rng(2)
    lmax = 6
    p = _alm(rng, lmax, 1)
    ell = np.arange(lmax + 1, dtype=float)
    e = -np.sqrt(ell * (ell + 1))[:, None] * p
    th, ph = rng.uniform(0.3, 2.8, 30), rng.uniform(0, 2 * np.pi, 30)
    f = lensing.synth_points(1, e, None, th, ph)
    dth, dph = wigner.resum_spin1_gradient(p, th, ph, h=1e-5)
    assert np.allclose(f.real, dth, atol=1e-6)
    assert np.allclose(f.imag, dph, atol=1e-6)


def test_spin2_matches_resummation_with_b():
    rng = np.random.default_rng(3)
    E, B = _alm(rng, 6, 2), _alm(rng, 6, 2)
    th, ph = np.arccos(rng.uniform(-1, 1, 40)), rng.uniform(0, 2 * np.pi, 40)
    f = lensing.synth_points(2, -E, -B, th, ph)
    q, u = wigner.resum_spin2(E, B, th, ph)
    assert np.allclose(f.real, q, atol=1e-11) and np.allclose(f.imag, u, atol=1e-11)


def test_displacement_geometry():
    rng = np.random.default_rng(4)
    th, ph = np.arccos(rng.uniform(-1, 1, 500)), rng.uniform(0, 2 * np.pi, 500)
    th[:3] = [0.0, np.pi, 1e-12]
    dth, dph = rng.normal(size=500) * 1e-3, rng.normal(size=500) * 1e-3
    t2, p2 = lensing.lensed_directions(th, ph, dth, dph)
    n = healpix.ang2vec(th, ph)
    n2 = healpix.ang2vec(t2, p2)
    ang = np.arctan2(np.linalg.norm(np.cross(n, n2), axis=-1), np.sum(n * n2, -1))
    assert np.allclose(ang, np.hypot(dth, dph), rtol=1e-9, atol=1e-15)
    # the displacement leaves n along d: its components on (e_theta, e_phi) are d / |d| sin|d|
    st, ct = np.sin(th), np.cos(th)
    et = np.stack([ct * np.cos(ph), ct * np.sin(ph), -st], -1)
    ep = np.stack([-np.sin(ph), np.cos(ph), np.zeros_like(ph)], -1)
    dmod = np.hypot(dth, dph)
    assert np.allclose(np.sum((n2 - n) * et, -1), dth / dmod * np.sin(dmod), atol=1e-12)
    assert np.allclose(np.sum((n2 - n) * ep, -1), dph / dmod * np.sin(dmod), atol=1e-12)
    # zero deflection is the identity
    t3, p3 = lensing.lensed_directions(th[3:], ph[3:], 0 * dth[3:], 0 * dph[3:])
    assert np.allclose(t3, th[3:], atol=1e-15) and np.allclose(np.mod(p3 - ph[3:] + 1, 2 * np.pi) - 1, 0, atol=1e-12)


def _edge_points(rng, n):
    th = np.concatenate([[0.0, np.pi, 1e-3, np.pi - 1e-3], np.arccos(rng.uniform(-1, 1, n))])
    return th, rng.uniform(0, 2 * np.pi, th.size)


def test_eth_route_matches_explicit_formula():
    rng = np.random.default_rng(6)
    th, ph = _edge_points(rng, 20)
    th, ph = th[4:], ph[4:]                      # the eth route divides by sin(theta)
    for s in range(3):
        e, b = _alm(rng, 10, s), (_alm(rng, 10, s) if s == 2 else None)
        ref = lensing.synth_points(s, e, b, th, ph)
        assert np.allclose(lensing.synth_points_eth(s, e, b, th, ph), ref, atol=1e-12), s


def test_recurrence_matches_explicit_formula_poles_included():
    rng = np.random.default_rng(7)
    th, ph = _edge_points(rng, 30)
    for s in range(3):
        e, b = _alm(rng, 10, s), (_alm(rng, 10, s) if s == 2 else None)
        ref = lensing.synth_points(s, e, b, th, ph)
        got = lensing.synth_points_recurrence(s, e, b, th, ph)
        assert np.allclose(got, ref, atol=1e-12), (s, np.max(np.abs(got - ref)))


def test_recurrence_matches_eth_route_at_l48():
    rng = np.random.default_rng(8)
    th, ph = _edge_points(rng, 8)
    th, ph = th[4:], ph[4:]
    for s in range(3):
        e, b = _alm(rng, 48, s), (_alm(rng, 48, s) if s == 2 else None)
        ref = lensing.synth_points_eth(s, e, b, th, ph)
        got = lensing.synth_points_recurrence(s, e, b, th, ph)
        assert np.max(np.abs(got - ref)) < 1e-12 * np.max(np.abs(ref)), s


def test_recurrence_unitarity_to_l2048():
    """Rows of the rotation matrix are unit vectors: sum over m of (d^l_{m,s})^2
    = 1, negative orders by d^l_{-m,s} = (-1)^{m+s} d^l_{m,-s}; at every l up to
    2048 and at polar, intermediate and equatorial angles.  The recurrence error
    near the poles grows like l^2 eps."""
    th = np.array([1e-3, 0.02, 0.7, 0.5 * np.pi, 2.9, np.pi - 1e-4, np.pi])
    for sp in (0, 1, 2):
        gp = lensing.wigner_d_by_l(sp, 2048, th)
        gm = lensing.wigner_d_by_l(-sp, 2048, th)
        worst = 0.0
        for (l, dp), (_, dm) in zip(gp, gm):
            if l < sp:
                assert np.all(dp == 0) and np.all(dm == 0)
                continue
            tot = dp[:, 0] ** 2 + np.sum(dp[:, 1:] ** 2 + dm[:, 1:] ** 2, axis=1)
            worst = max(worst, np.max(np.abs(tot - 1.0)))
        assert worst < 5e-10, (sp, worst)


def test_recurrence_m0_is_legendre_to_l4096():
    from scipy.special import eval_legendre
    th = np.array([1e-3, 0.3, 1.2, 0.5 * np.pi, 2.5, np.pi - 1e-3])
    worst = 0.0
    for l, d in lensing.wigner_d_by_l(0, 4096, th):
        if l % 97 == 0 or l >= 4090:
            worst = max(worst, np.max(np.abs(d[:, 0] - eval_legendre(l, np.cos(th)))))
    assert worst < 1e-9, worst
