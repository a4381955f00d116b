"""Pins of the seeded input generator (shares no code with the oracle; checked
against its brute-force resummation and against scipy's spherical harmonics)."""
import numpy as np
import pytest
import torch

from oracle import healpix, wigner
from workload import configs, seeds, spectra, synth, rings


def _alm(lmax, seed):
    rng = seeds.rng(99, seed, 0)
    cl = np.zeros(lmax + 1)
    cl[1:] = 1.0 / np.arange(1, lmax + 1)
    return synth.draw_alm(rng, cl, lmax)


@pytest.mark.parametrize("nside,lmax", [(2, 4), (4, 9), (8, 12)])
def test_synthesis_matches_resummation(nside, lmax):
    a = _alm(lmax, nside)
    th, ph = healpix.pix2ang(nside, np.arange(healpix.npix(nside)))
    T = synth.synth(a, 0, nside).numpy()
    assert np.allclose(T, wigner.resum_spin0(a, th, ph), atol=1e-12)
    q, u = synth.synth(-a, 2, nside)
    qr, ur = wigner.resum_spin2(a, 0 * a, th, ph)
    assert np.allclose(q.numpy(), qr, atol=1e-12) and np.allclose(u.numpy(), ur, atol=1e-12)
    ell = np.arange(lmax + 1)
    dt, dp = synth.synth(-np.sqrt(ell * (ell + 1.0))[:, None] * a, 1, nside)
    rt, rp = wigner.resum_spin1_gradient(a, th, ph)
    scale = np.abs(rt).max()
    assert np.allclose(dt.numpy(), rt, atol=1e-6 * scale) and np.allclose(dp.numpy(), rp, atol=1e-6 * scale)


def test_high_l_against_scipy():
    from scipy.special import sph_harm_y
    nside, lmax = 64, 180
    rg = rings.ring_geometry(nside)
    for L, M in [(180, 175), (180, 2), (150, 90)]:
        a = np.zeros((lmax + 1, lmax + 1), complex)
        a[L, M] = 0.3 + 0.7j
        T = synth.synth(a, 0, nside).numpy()
        for r in [0, 3, 40, 127, 200, 254]:
            phs = rg["phi0"][r] + rg["dphi"][r] * np.arange(rg["count"][r])
            ref = 2 * np.real(a[L, M] * sph_harm_y(L, M, rg["theta"][r], phs))
            got = T[rg["first"][r]: rg["first"][r] + rg["count"][r]]
            assert np.allclose(got, ref, atol=1e-12)


def test_seeds_deterministic():
    a = seeds.rng(1, 0, 0).standard_normal(5)
    b = seeds.rng(1, 0, 0).standard_normal(5)
    c = seeds.rng(1, 0, 1).standard_normal(5)
    assert np.array_equal(a, b) and not np.array_equal(a, c)


def test_config1_inputs():
    inp = configs.build(1)
    assert inp["maps"]["T"].shape == (49152,)
    th, ph = inp["theta"].numpy(), inp["phi"].numpy()
    th0, ph0 = healpix.pix2ang(64, np.arange(49152))
    d = np.arccos(np.clip(np.sum(healpix.ang2vec(th, ph) * healpix.ang2vec(th0, ph0), -1), -1, 1))
    rms = np.sqrt(np.mean(d ** 2)) / spectra.ARCMIN
    assert 1.5 < rms < 3.5          # 2.5' rms deflection (one realisation)
    assert np.all((th >= 0) & (th <= np.pi)) and np.all((ph >= 0) & (ph < 2 * np.pi))


def test_deflection_normalisation():
    cl = spectra.cl_phi(4096)
    ell = np.arange(4097)
    rms = np.sqrt(np.sum((2 * ell + 1) / (4 * np.pi) * ell * (ell + 1) * cl))
    assert rms == pytest.approx(spectra.deflection_rms_rad(), rel=1e-12)
