"""Pins of the oracle's HEALPix RING geometry (Gorski et al. 2005)."""
import os

import numpy as np
import pytest

from oracle import healpix

GOLD = os.path.join(os.path.dirname(__file__), "golden", "healpix_nside1.txt")


def test_counts():
    for N in (1, 2, 3, 8, 64):
        rt = healpix.ring_table(N)
        assert len(rt["count"]) == 4 * N - 1
        assert rt["count"].sum() == 12 * N * N
        assert np.all(rt["first"][1:] == rt["first"][:-1] + rt["count"][:-1])
    # paper Sec. 3.2: N_side = 64 has 49,152 pixels
    assert healpix.npix(64) == 49152


def test_nside1_golden():
    g = np.loadtxt(GOLD)
    th, ph = healpix.pix2ang(1, g[:, 0].astype(int))
    assert np.allclose(np.cos(th), g[:, 1], atol=1e-15)
    assert np.allclose(ph / np.pi, g[:, 2], atol=1e-15)


@pytest.mark.parametrize("N", [1, 2, 4, 16])
def test_equal_area_monte_carlo(N):
    """Pixels are equal-area: nearest-centre cells are not, so draw uniform points
    and assign them by the RING ang2pix rule derived from the same geometry
    (ring boundaries), checking counts against a multinomial."""
    rng = np.random.default_rng(1)
    M = 400000
    z = rng.uniform(-1, 1, M)
    phi = rng.uniform(0, 2 * np.pi, M)
    pix = _ang2pix_ring(N, z, phi)
    counts = np.bincount(pix, minlength=12 * N * N)
    exp = M / (12 * N * N)
    chi2 = np.sum((counts - exp) ** 2 / exp)
    dof = 12 * N * N - 1
    assert chi2 < dof + 6 * np.sqrt(2 * dof)


def _ang2pix_ring(N, z, phi):
    """Pixel boundaries from the HEALPix construction (Gorski et al. 2005, Sec. 4):
    equatorial zone |z| <= 2/3 uses the two families of boundary lines
    z = 2/3 - 4 nside t / 3 ... expressed through jp, jm; polar caps use
    the sqrt(3 (1 - |z|)) scaling.  Written from the definition, independent of
    the pixel-centre code under test."""
    tt = np.mod(phi, 2 * np.pi) / (0.5 * np.pi)        # in [0, 4)
    za = np.abs(z)
    pix = np.empty(z.shape, dtype=np.int64)
    eq = za <= 2.0 / 3.0
    # equatorial
    t1 = N * (0.5 + tt[eq])
    t2 = N * z[eq] * 0.75
    jp = np.floor(t1 - t2).astype(np.int64)
    jm = np.floor(t1 + t2).astype(np.int64)
    ir = N + 1 + jp - jm                                  # ring 1..2N+1 within the belt
    kshift = 1 - (ir & 1)
    ip = (jp + jm - N + kshift + 1) // 2
    ip = np.mod(ip, 4 * N)
    pix[eq] = 2 * N * (N - 1) + (ir - 1) * 4 * N + ip
    # polar caps
    pc = ~eq
    tp = tt[pc] - np.floor(tt[pc])
    tmp = N * np.sqrt(3 * (1 - za[pc]))
    jp = np.floor(tp * tmp).astype(np.int64)
    jm = np.floor((1.0 - tp) * tmp).astype(np.int64)
    ir = jp + jm + 1
    ip = np.floor(tt[pc] * ir).astype(np.int64)
    ip = np.mod(ip, 4 * ir)
    north = z[pc] > 0
    pix_pc = np.where(north, 2 * ir * (ir - 1) + ip, 12 * N * N - 2 * ir * (ir + 1) + ip)
    pix[pc] = pix_pc
    return pix


@pytest.mark.parametrize("N", [1, 2, 5, 16])
def test_centres_inside_own_pixel(N):
    th, ph = healpix.pix2ang(N, np.arange(12 * N * N))
    assert np.all(_ang2pix_ring(N, np.cos(th), ph) == np.arange(12 * N * N))


def test_north_south_mirror():
    N = 8
    v = healpix.all_vec(N)
    rt = healpix.ring_table(N)
    nr = len(rt["count"])
    for r in range(nr):
        m = nr - 1 - r
        a = v[rt["first"][r]: rt["first"][r] + rt["count"][r]]
        b = v[rt["first"][m]: rt["first"][m] + rt["count"][m]]
        assert np.allclose(a[:, :2], b[:, :2], atol=1e-15)
        assert np.allclose(a[:, 2], -b[:, 2], atol=1e-15)


@pytest.mark.parametrize("N", [1, 2, 4, 8, 32])
def test_ang2pix_centres_round_trip(N):
    pix = np.arange(healpix.npix(N))
    th, ph = healpix.pix2ang(N, pix)
    assert np.array_equal(healpix.ang2pix(N, th, ph), pix)
    # also with phi shifted by whole turns
    assert np.array_equal(healpix.ang2pix(N, th, ph - 4 * np.pi), pix)


@pytest.mark.parametrize("N", [1, 2, 4, 16])
def test_ang2pix_equal_area_and_second_transcription(N):
    rng = np.random.default_rng(2)
    M = 400000
    z = rng.uniform(-1, 1, M)
    phi = rng.uniform(0, 2 * np.pi, M)
    pix = healpix.ang2pix(N, np.arccos(z), phi)
    assert np.array_equal(pix, _ang2pix_ring(N, z, phi))
    counts = np.bincount(pix, minlength=12 * N * N)
    exp = M / (12 * N * N)
    dof = 12 * N * N - 1
    assert np.sum((counts - exp) ** 2 / exp) < dof + 6 * np.sqrt(2 * dof)


def test_ang2pix_contains_near_centre():
    """The containing pixel's centre is one of the four nearest centres and
    closer than the largest pixel radius (< 1.4 x the mean pixel size)."""
    N = 16
    rng = np.random.default_rng(3)
    th, ph = np.arccos(rng.uniform(-1, 1, 3000)), rng.uniform(0, 2 * np.pi, 3000)
    pix = healpix.ang2pix(N, th, ph)
    v = healpix.ang2vec(th, ph)
    allv = healpix.all_vec(N)
    d = np.linalg.norm(allv[None, :, :] - v[:, None, :], axis=-1)
    rank = np.sum(d < d[np.arange(len(pix)), pix][:, None], axis=1)
    assert np.all(rank < 4)
    assert np.max(d[np.arange(len(pix)), pix]) < 1.4 * np.sqrt(4 * np.pi / healpix.npix(N))
