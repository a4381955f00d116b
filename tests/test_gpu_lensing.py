"""The lensing pipeline on the device (paper Sec. 3.1) against the oracle:
spin-s synthesis of RING maps (flints_synthesize), the displaced pixel centres
(flints_lensed_directions) and the whole chain to the interpolated T, Q, U.

Synthesis tolerances, relative to the largest oracle value: 1e-11 up to
lmax ~ 300 (both sides double precision; the recurrence error is ~ l eps in the
oscillatory region); 1e-8 at lmax 4096, where near the poles the three-term
recurrence in l loses ~ l^2 eps on both sides (the oracle's own unitarity pin
sees 1e-10 at l = 2048) and the closed-form seeds carry the ~1e-13 error of
log-gamma at large arguments.  Directions: unit vectors within 1e-14."""
import numpy as np
import pytest
import torch

import paper_1003_4984_amd as fl
from oracle import healpix, kriging, lensing
from workload import seeds, spectra, synth

from _gpu_helpers import dev, compare

pytestmark = pytest.mark.gpu


def _alm(seed, lmax, cl=None, lmin=0):
    r = seeds.rng(43, seed, 0)
    cl = np.ones(lmax + 1) if cl is None else cl
    a = synth.draw_alm(r, cl, lmax)
    a[:lmin] = 0
    return a


def _gpu_synth(nside, lmax, spin, e, b=None):
    am = dev(fl.alm_mmajor(e))
    bm = dev(fl.alm_mmajor(b)) if b is not None else None
    out = torch.full(((1 if spin == 0 else 2) * 12 * nside * nside,), -7.0, dtype=torch.float64, device="cuda")
    fl.synthesize(nside, lmax, spin, am, bm, out=out)
    torch.cuda.synchronize()
    return out


def _as_complex(spin, m, pix=None):
    npix = m.numel() // (1 if spin == 0 else 2)
    if pix is not None:
        idx = torch.as_tensor(pix, device="cuda")
        re = m[:npix][idx].cpu().numpy()
        im = m[npix:][idx].cpu().numpy() if spin else np.zeros_like(re)
    else:
        re = m[:npix].cpu().numpy()
        im = m[npix:].cpu().numpy() if spin else np.zeros_like(re)
    return re + 1j * im


def _check_synth(nside, lmax, spin, seed, pix=None, tol=1e-11, with_b=True):
    e = _alm(seed, lmax, lmin=spin)
    b = _alm(seed + 1000, lmax, lmin=spin) if (spin == 2 and with_b) else None
    m = _gpu_synth(nside, lmax, spin, e, b)
    if pix is None:
        pix = np.arange(12 * nside * nside)
    th, ph = healpix.pix2ang(nside, pix)
    # oracle convention: a = e + i b with the per-spin scaling written out
    ell = np.arange(lmax + 1, dtype=np.float64)
    if spin == 0:
        ea, ba = e, None
    elif spin == 1:
        ea, ba = -np.sqrt(ell * (ell + 1))[:, None] * e, None
    else:
        ea, ba = -e, (-b if b is not None else None)
    ref = lensing.synth_points_recurrence(spin, ea, ba, th, ph)
    got = _as_complex(spin, m, pix)
    scale = np.max(np.abs(ref))
    if scale == 0:                       # lmax below the spin: the sum is empty
        assert np.all(got == 0)
        return 0.0
    err = np.max(np.abs(got - ref)) / scale
    print(f"synth nside {nside} lmax {lmax} spin {spin}: max err / max {err:.2e}", flush=True)
    assert err < tol, err
    if spin == 0:
        assert np.all(got.imag == 0)
    return err


@pytest.mark.parametrize("spin", [0, 1, 2])
def test_synthesis_all_pixels_small(spin):
    """Every pixel of N_side 8 (lmax 20) and N_side 4 (lmax 40: orders far above
    every ring's Nyquist frequency fold onto the ring's DFT)."""
    _check_synth(8, 20, spin, 1)
    _check_synth(4, 40, spin, 2)


@pytest.mark.parametrize("nside,lmax", [(6, 17), (24, 50), (3, 1)])
def test_synthesis_non_power_of_two_nside(nside, lmax):
    """Belt rings of 4 N_side pixels that are not powers of two take the chirp-z
    path too; lmax 1 leaves the spin-2 sum empty and the map is still written (zeros)."""
    for spin in (0, 1, 2):
        _check_synth(nside, lmax, spin, 3 + spin)


def test_synthesis_spin2_without_b_and_lmax0():
    _check_synth(16, 30, 2, 9, with_b=False)
    m = _gpu_synth(2, 0, 0, np.array([[2.0 + 0j]]))
    assert torch.allclose(m, torch.full_like(m, 2.0 * np.sqrt(1 / (4 * np.pi))), rtol=1e-15, atol=0)
    m = _gpu_synth(2, 1, 2, np.ones((2, 2), complex), np.ones((2, 2), complex))
    assert torch.all(m == 0)


def _sample_pixels(nside, rng, per_ring=2):
    rt = healpix.ring_table(nside)
    rings = sorted({1, 2, 3, nside - 1, nside, nside + 1, 2 * nside, 3 * nside - 1, 3 * nside,
                    4 * nside - 2, 4 * nside - 1} | set(rng.integers(1, 4 * nside, 6).tolist()))
    pix = []
    for r in rings:
        if r < 1 or r > 4 * nside - 1:
            continue
        i = r - 1
        first, n = int(rt["first"][i]), int(rt["count"][i])
        pix += [first, first + n - 1] + (first + rng.integers(0, n, per_ring)).tolist()
    return np.unique(np.array(pix, dtype=np.int64))


@pytest.mark.parametrize("spin", [0, 1, 2])
def test_synthesis_nside128_lmax256_sampled(spin):
    rng = np.random.default_rng(10 + spin)
    _check_synth(128, 256, spin, 20 + spin, pix=_sample_pixels(128, rng, 20))


@pytest.mark.parametrize("spin", [0, 2])
def test_synthesis_full_shape_sampled(spin):
    """N_side 4096, lmax 4096 (the headline lensing shape) on sampled pixels of
    the polar, boundary, belt and equator rings."""
    rng = np.random.default_rng(30 + spin)
    lmax = 4096
    tt, ee, _, _ = spectra.cl_acoustic(lmax)
    cl = tt if spin == 0 else ee
    e = _alm(40 + spin, lmax, cl=cl, lmin=spin)
    b = _alm(50 + spin, lmax, cl=0.1 * cl, lmin=spin) if spin == 2 else None
    m = _gpu_synth(4096, lmax, spin, e, b)
    assert torch.isfinite(m).all()
    pix = _sample_pixels(4096, rng, 0)[::2]      # about one pixel per sampled ring (oracle ~1 s per pixel)
    th, ph = healpix.pix2ang(4096, pix)
    ref = lensing.synth_points_recurrence(spin, e if spin == 0 else -e, -b if spin == 2 else None, th, ph)
    got = _as_complex(spin, m, pix)
    err = np.max(np.abs(got - ref)) / np.max(np.abs(ref))
    print(f"full shape spin {spin}: {pix.size} pixels, max err / max {err:.2e}", flush=True)
    assert err < 1e-8, err


def test_lensed_directions():
    nside = 64
    npix = 12 * nside * nside
    rng = np.random.default_rng(60)
    dth = rng.normal(size=npix) * 7e-4
    dph = rng.normal(size=npix) * 7e-4
    dth[:10], dph[:10] = 0.0, 0.0
    dth[10:20] = rng.uniform(-1.5, 1.5, 10)      # large displacements, across the poles
    dth[npix - 5:] = 3.0
    theta, phi = fl.lensed_directions(nside, dev(np.concatenate([dth, dph])))
    torch.cuda.synchronize()
    th0, ph0 = healpix.pix2ang(nside, np.arange(npix))
    to, po = lensing.lensed_directions(th0, ph0, dth, dph)
    tg, pg = theta.cpu().numpy(), phi.cpu().numpy()
    assert np.all((tg >= 0) & (tg <= np.pi) & (pg >= 0) & (pg < 2 * np.pi))
    gap = np.linalg.norm(healpix.ang2vec(tg, pg) - healpix.ang2vec(to, po), axis=-1)
    assert np.max(gap) < 1e-14, np.max(gap)
    # zero deflection: the pixel centres themselves
    assert np.max(np.linalg.norm(healpix.ang2vec(tg[:10], pg[:10]) - healpix.ang2vec(th0[:10], ph0[:10]),
                                 axis=-1)) < 1e-15


def test_lens_pipeline_against_oracle():
    """The whole chain at N_side 32, lmax 64: unlensed T, Q, U and grad(phi) by
    synthesis, displaced centres, then T+Q/U kriging (K 16) there.  Maps and
    directions are checked everywhere; interpolated values and variances on a
    sample of targets against the oracle's kriging of the oracle's maps at the
    oracle's directions."""
    nside, lmax, K = 32, 64, 16
    npix = 12 * nside * nside
    tt, ee, _, bb = spectra.cl_acoustic(lmax)
    cl_phi = spectra.cl_phi(lmax)
    tlm = _alm(70, lmax, cl=tt)
    elm = _alm(71, lmax, cl=ee, lmin=2)
    blm = _alm(72, lmax, cl=0.05 * ee, lmin=2)
    plm = _alm(73, lmax, cl=cl_phi * 400.0, lmin=1)   # deflections of ~ a pixel
    cl_bb = 0.05 * ee
    p0 = fl.Plan(nside, lmax, tt, K, 0)
    p2 = fl.Plan(nside, lmax, np.concatenate([ee, cl_bb]), K, 2)
    res = fl.lens_tqu(p0, p2, lmax, dev(fl.alm_mmajor(tlm)), dev(fl.alm_mmajor(elm)), dev(fl.alm_mmajor(blm)),
                      dev(fl.alm_mmajor(plm)))
    torch.cuda.synchronize()
    out_t, var_t, out_qu, var_qu, th_g, ph_g = [x.cpu().numpy() for x in res]
    # oracle chain
    pix = np.arange(npix)
    th0, ph0 = healpix.pix2ang(nside, pix)
    ell = np.arange(lmax + 1, dtype=np.float64)
    t_map = lensing.synth_points_recurrence(0, tlm, None, th0, ph0).real
    qu = lensing.synth_points_recurrence(2, -elm, -blm, th0, ph0)
    d = lensing.synth_points_recurrence(1, -np.sqrt(ell * (ell + 1))[:, None] * plm, None, th0, ph0)
    to, po = lensing.lensed_directions(th0, ph0, d.real, d.imag)
    gap = np.linalg.norm(healpix.ang2vec(th_g, ph_g) - healpix.ang2vec(to, po), axis=-1)
    assert np.max(gap) < 1e-13, np.max(gap)
    rms_d = np.sqrt(np.mean(np.abs(d) ** 2))
    print(f"deflection rms {rms_d:.2e} rad", flush=True)
    rng = np.random.default_rng(74)
    sel = np.unique(np.concatenate([rng.choice(npix, 400, replace=False), [0, 1, npix - 1]]))
    vo, varo, _ = kriging.interpolate(nside, tt, K, 0, t_map, to[sel], po[sel])
    compare(out_t[sel], var_t[sel], vo, varo, 1e-8, 1e-4, 1e-9 * p0.info()["sigma2"])
    vo2, varo2, _ = kriging.interpolate(nside, (ee, cl_bb), K, 2, (qu.real, qu.imag), to[sel], po[sel])
    g = out_qu.reshape(2, npix).T[sel]
    gv = var_qu.reshape(2, npix).T[sel]
    compare(g, gv, vo2, varo2, 1e-8, 1e-4, 1e-9 * p2.info()["sigma2"])
