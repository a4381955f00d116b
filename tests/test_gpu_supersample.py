"""Supersampling (paper Sec. 2.6, Table 1): a map interpolated at every pixel
centre of a finer RING map, targets generated on the device.  Element by
element against the FP64 oracle at the same directions (the device's pixel
centres, checked against the oracle's to 1e-14, on the GPU's stencils), spin 0
and spin 2; N_side -> N_side reproduces the map (pixel centres,
nugget-limited)."""
import numpy as np
import pytest
import torch

import paper_1003_4984_amd as fl
from oracle import healpix, kriging
from workload import configs, spectra, synth, seeds

from _gpu_helpers import compare, dev, gpu_stencil, reconcile_stencils

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("spin,K", [(0, 9), (0, 36), (2, 9), (2, 16)])
def test_supersample_parity(gpu_ok, spin, K):
    nside, lmax = 32, 64
    nout = 2 * nside
    tt, ee, te, bb = spectra.cl_acoustic(lmax)
    rng = seeds.rng(44, spin * 100 + K, 0)
    if spin == 0:
        maps = synth.synth(synth.draw_alm(rng, tt, lmax), 0, nside).numpy()
        cl, clo, m = tt, tt, dev(maps)
    else:
        q, u = synth.synth(-synth.draw_alm(rng, ee, lmax), 2, nside)
        maps = (q.numpy(), u.numpy())
        cl, clo, m = np.concatenate([ee, 0.2 * ee]), (ee, 0.2 * ee), dev(np.concatenate(maps))
    p = fl.Plan(nside, lmax, cl, K, spin)
    out, var = fl.supersample(p, m, nout)
    torch.cuda.synchronize()
    npo = 12 * nout * nout
    o = out.cpu().numpy()
    v = var.cpu().numpy()
    if spin == 2:
        o, v = o.reshape(2, npo).T, v.reshape(2, npo).T
    assert np.all(np.isfinite(o)) and np.all(v >= 0)
    st = p.stats()
    assert st["bad_inputs"] == 0 and st["search_failures"] == 0
    pick = configs.parity_subset(44, npo, 1500)
    # the directions the call used (child centres often sit at equal distance
    # from two parent centres, so an ulp decides such ties: compare at exactly
    # the GPU's directions); they are the oracle's pixel centres to rounding
    dth, dph = fl.pixel_centres(nout)
    torch.cuda.synchronize()
    th, ph = dth.cpu().numpy()[pick], dph.cpu().numpy()[pick]
    oth, oph = healpix.pix2ang(nout, pick)
    assert np.max(np.abs(th - oth)) < 1e-14 and np.max(np.abs(np.mod(ph - oph + 1, 2 * np.pi) - 1)) < 1e-14
    g = gpu_stencil(p, th, ph)
    reconcile_stencils(nside, th, ph, g, kriging.stencils(nside, th, ph, K))
    vo, varo, _ = kriging.interpolate(nside, clo, K, spin, maps, th, ph, stencil_idx=g)
    compare(o[pick], v[pick], vo, varo, 1e-8, 1e-4, 1e-9 * p.info()["sigma2"])


def test_supersample_same_resolution_reproduces_map(gpu_ok):
    nside, lmax, K = 16, 32, 12
    cl = spectra.cl_config1(lmax, sigma_arcmin=120.0)
    m = synth.synth(synth.draw_alm(seeds.rng(45, 0, 0), cl, lmax), 0, nside).numpy()
    p = fl.Plan(nside, lmax, cl, K, 0)
    out, var = fl.supersample(p, dev(m), nside)
    torch.cuda.synchronize()
    s2 = p.info()["sigma2"]
    assert np.max(np.abs(out.cpu().numpy() - m)) < 1e-5 * np.sqrt(s2)
    assert np.all(var.cpu().numpy() <= p.info()["nugget_eps"] * s2 * (1 + 1e-3) + 1e-12 * s2)
    with pytest.raises(fl.FlintsError):
        fl.supersample(p, dev(m), 0)
