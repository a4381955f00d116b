"""Pins of the spin-2 covariance phases by the brute-force addition theorem
(paper App. A): sum_m 2Y_lm(n1) 2Y*_lm(n2) and sum_m 2Y_lm(n1) -2Y*_lm(n2)."""
import numpy as np
import pytest

from oracle import healpix, kriging, wigner


def _frames(th, ph):
    return kriging._frames(np.asarray(th, float), np.asarray(ph, float))


@pytest.mark.parametrize("seed", range(6))
def test_addition_theorem_phases(seed):
    rng = np.random.default_rng(seed)
    th = rng.uniform(0.05, np.pi - 0.05, 2)
    ph = rng.uniform(0, 2 * np.pi, 2)
    lmax = 7
    n, et, ep = _frames(th, ph)
    for l in range(2, lmax + 1):
        ee = np.zeros(l + 1)
        ee[l] = 1.0
        G, P, xp0 = kriging.spin2_gamma_pi(n[None], et[None], ep[None], ee, np.zeros(l + 1))
        g_bf = sum(wigner.sY(2, l, m, th[0], ph[0]) * np.conj(wigner.sY(2, l, m, th[1], ph[1]))
                   for m in range(-l, l + 1))
        p_bf = sum(wigner.sY(2, l, m, th[0], ph[0]) * np.conj(wigner.sY(-2, l, m, th[1], ph[1]))
                   for m in range(-l, l + 1))
        assert abs(G[0, 0, 1] - g_bf) < 1e-13
        assert abs(P[0, 0, 1] - p_bf) < 1e-13


def test_phase_trivial_on_meridian_and_equator():
    """Two points on one meridian or both on the equator: transport is trivial."""
    cl = np.zeros(6)
    cl[2:] = 1.0
    for th, ph in [((0.4, 0.9), (1.2, 1.2)), ((np.pi / 2, np.pi / 2), (0.1, 0.5))]:
        n, et, ep = _frames(th, ph)
        G, P, _ = kriging.spin2_gamma_pi(n[None], et[None], ep[None], cl, 0 * cl)
        assert abs(G[0, 0, 1].imag) < 1e-15 and abs(P[0, 0, 1].imag) < 1e-15


def test_paper_mode_equals_real_system_without_pi():
    """The complex Hermitian K x K estimator (paper Eq. major_eq) equals the real
    2K x 2K conditional mean when <P P> is dropped."""
    rng = np.random.default_rng(3)
    N, K = 8, 6
    lmax = 20
    ee = np.zeros(lmax + 1)
    ee[2:] = 1.0 / np.arange(2, lmax + 1) ** 2
    bb = 0.3 * ee
    th, ph = rng.uniform(0.3, 2.8, 5), rng.uniform(0, 6.2, 5)
    st = kriging.stencils(N, th, ph, K)
    nv, et, ep = kriging._pixel_frames(N, st)
    q, u = rng.normal(size=(5, K)), rng.normal(size=(5, K))
    vp, varp, _ = kriging.krige_spin2(th, ph, nv, et, ep, q, u, ee, bb, mode="paper")
    # real system with Pi = 0, built by hand from Gamma only
    t, tet, tep = kriging._frames(th, ph)
    n = np.concatenate([t[:, None], nv], 1)
    e1 = np.concatenate([tet[:, None], et], 1)
    e2 = np.concatenate([tep[:, None], ep], 1)
    G, _, xp0 = kriging.spin2_gamma_pi(n, e1, e2, ee, bb)
    Gn = G / xp0
    C = np.block([[Gn.real[:, 1:, 1:], -Gn.imag[:, 1:, 1:]], [Gn.imag[:, 1:, 1:], Gn.real[:, 1:, 1:]]])
    C = C + kriging.EPS_F64 * np.eye(2 * K)
    cQ = np.concatenate([Gn.real[:, 1:, 0], Gn.imag[:, 1:, 0]], 1)
    cU = np.concatenate([-Gn.imag[:, 1:, 0], Gn.real[:, 1:, 0]], 1)
    x = np.concatenate([q, u], 1)
    wQ = np.linalg.solve(C, cQ[..., None])[..., 0]
    wU = np.linalg.solve(C, cU[..., None])[..., 0]
    assert np.allclose(vp[:, 0], np.einsum("bi,bi->b", wQ, x), atol=1e-9)
    assert np.allclose(vp[:, 1], np.einsum("bi,bi->b", wU, x), atol=1e-9)
    vq = 0.5 * xp0 * (1 - np.einsum("bi,bi->b", wQ, cQ))
    assert np.allclose(varp[:, 0], vq, rtol=1e-7, atol=1e-14)
