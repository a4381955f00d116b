"""FP32 + iterative refinement path (covariance entries and residuals in FP64,
factorisation and solves in FP32, one refinement step, FP64 recompute of
rejected neighbourhoods).  Tolerance against the FP64 oracle: values within
2e-4 of the rms value, variances within 1e-2 relative (+1e-9 sigma0^2)."""
import numpy as np
import pytest
import torch

import paper_1003_4984_amd as fl
from oracle import kriging
from workload import configs, spectra, synth, seeds

from _gpu_helpers import dev, gpu_stencil, reconcile_stencils, run_gpu, compare

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def cfg1(gpu_ok):
    return configs.build(1)


def _oracle(nside, cl, K, spin, maps, th, ph, g, **kw):
    reconcile_stencils(nside, th, ph, g, kriging.stencils(nside, th, ph, K))
    return kriging.interpolate(nside, cl, K, spin, maps, th, ph, stencil_idx=g, **kw)


def test_fp32ir_parity_cfg1(cfg1):
    sh = cfg1["shape"]
    nside, K = sh["nside"], sh["K"]
    p = fl.Plan(nside, sh["lmax"], cfg1["cl_tt"], K, 0, precision=fl.FP32_IR)
    info = p.info()
    assert info["precision"] == fl.FP32_IR          # the creation probe kept the FP32 path
    T = cfg1["maps"]["T"].numpy()
    th, ph = cfg1["theta"].numpy(), cfg1["phi"].numpy()
    v, var = run_gpu(p, T, th, ph)
    frac = p.stats()["fp64_fallbacks"] / len(th)
    print(f"cfg1 FP32+IR: probe rejection {info['fp32_probe_reject']:.3f}, "
          f"FP64 recompute fraction {frac:.4f}")
    assert frac < 0.05                              # the FP32 path carries the work
    sel = configs.parity_subset(1, len(th), 3000)
    g = gpu_stencil(p, th[sel], ph[sel])
    vo, varo, _ = _oracle(nside, cfg1["cl_tt"], K, 0, T, th[sel], ph[sel], g)
    compare(v[sel], var[sel], vo, varo, 2e-4, 1e-2, 1e-9 * p.info()["sigma2"])


@pytest.mark.parametrize("mode", [fl.S2_FULL, fl.S2_PAPER])
def test_fp32ir_parity_spin2(gpu_ok, mode):
    nside, lmax, K = 64, 160, 16
    tt, ee, te, bb = spectra.cl_acoustic(lmax)
    rng = seeds.rng(7, 0, 0)
    q, u = synth.synth(-synth.draw_alm(rng, ee, lmax), 2, nside)
    q, u = q.numpy(), u.numpy()
    p = fl.Plan(nside, lmax, np.concatenate([ee, bb]), K, 2, precision=fl.FP32_IR, spin2_mode=mode)
    th, ph = np.arccos(rng.uniform(-1, 1, 1500)), rng.uniform(0, 2 * np.pi, 1500)
    v, var = run_gpu(p, (q, u), th, ph)
    g = gpu_stencil(p, th, ph)
    vo, varo, _ = _oracle(nside, (ee, bb), K, 2, (q, u), th, ph, g,
                          mode="paper" if mode == fl.S2_PAPER else "full")
    compare(v, var, vo, varo, 2e-4, 1e-2, 1e-9 * p.info()["sigma2"])


@pytest.mark.parametrize("spin,K", [(0, 16), (2, 16), (0, 40), (2, 32)])
def test_forced_fallback_equals_fp64(gpu_ok, spin, K):
    """Pivot-ratio threshold 1 rejects every FP32 factorisation; the FP64
    recompute must then reproduce the FP64 path bit for bit (row-group sizes
    n <= 32 and tile sizes n > 32)."""
    nside, lmax = 32, 80
    tt, ee, te, bb = spectra.cl_acoustic(lmax)
    rng = seeds.rng(8, spin, 0)
    if spin == 0:
        maps = synth.synth(synth.draw_alm(rng, tt, lmax), 0, nside).numpy()
        cl = tt
    else:
        q, u = synth.synth(-synth.draw_alm(rng, ee, lmax), 2, nside)
        maps, cl = (q.numpy(), u.numpy()), np.concatenate([ee, bb])
    th, ph = np.arccos(rng.uniform(-1, 1, 700)), rng.uniform(0, 2 * np.pi, 700)
    p64 = fl.Plan(nside, lmax, cl, K, spin)
    p32 = fl.Plan(nside, lmax, cl, K, spin, precision=fl.FP32_IR, pivot_ratio_min=1.0, fp32_max_reject=1.0)
    assert p32.info()["precision"] == fl.FP32_IR and p32.info()["fp32_probe_reject"] == 1.0
    v64, var64 = run_gpu(p64, maps, th, ph)
    v32, var32 = run_gpu(p32, maps, th, ph)
    assert p32.stats()["fp64_fallbacks"] == len(th)
    assert np.array_equal(v64, v32) and np.array_equal(var64, var32)


def test_no_fallback_when_tests_disabled(gpu_ok):
    nside, lmax, K = 32, 64, 16
    cl = spectra.cl_config1(lmax, sigma_arcmin=60.0)
    rng = seeds.rng(9, 0, 0)
    m = synth.synth(synth.draw_alm(rng, cl, lmax), 0, nside).numpy()
    p = fl.Plan(nside, lmax, cl, K, 0, precision=fl.FP32_IR, pivot_ratio_min=1e-300,
                refine_tol=1e300)
    th, ph = np.arccos(rng.uniform(-1, 1, 500)), rng.uniform(0, 2 * np.pi, 500)
    v, var = run_gpu(p, m, th, ph)
    assert p.stats()["fp64_fallbacks"] == 0
    g = gpu_stencil(p, th, ph)
    vo, varo, _ = _oracle(nside, cl, K, 0, m, th, ph, g)
    compare(v, var, vo, varo, 2e-4, 1e-2, 1e-9 * p.info()["sigma2"])


def test_probe_routes_unfit_plans_to_fp64(gpu_ok):
    """A plan whose FP32 systems are all rejected (pivot-ratio threshold 1)
    computes in FP64 from the start: no FP32 attempt, no fallbacks, results
    equal to the FP64 plan bit for bit; with the skip disabled the same plan
    runs FP32 and recomputes every point."""
    nside, lmax, K = 32, 80, 16
    cl = spectra.cl_config1(lmax, sigma_arcmin=60.0)
    rng = seeds.rng(10, 0, 0)
    m = synth.synth(synth.draw_alm(rng, cl, lmax), 0, nside).numpy()
    th, ph = np.arccos(rng.uniform(-1, 1, 400)), rng.uniform(0, 2 * np.pi, 400)
    p64 = fl.Plan(nside, lmax, cl, K, 0)
    p32 = fl.Plan(nside, lmax, cl, K, 0, precision=fl.FP32_IR, pivot_ratio_min=1.0)
    assert p32.info()["fp32_probe_reject"] == 1.0 and p32.info()["precision"] == fl.FP64
    assert p64.info()["fp32_probe_reject"] == -1.0
    v64, w64 = run_gpu(p64, m, th, ph)
    v32, w32 = run_gpu(p32, m, th, ph)
    assert p32.stats()["fp64_fallbacks"] == 0
    assert np.array_equal(v64, v32) and np.array_equal(w64, w32)
