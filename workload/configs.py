"""Input builders for the five workload shapes.

cfg 1  T only, N_side 64, lmax 128, K 16: C_l = 1e3/(l(l+1)) exp(-l^2 sigma^2),
       sigma = 10'; one displaced target per pixel.
cfg 2  T+Q+U, N_side 512, lmax 1024, K 24: damped acoustic TT/EE/TE, BB = 0.
cfg 3  T+Q+U, N_side 4096, lmax 4096, K 32: cfg-2 spectral forms.
cfg 4  64 jobs, N_side in {128..2048}, spin in {0,2}, K in {16,24,32,48},
       n ~ log-uniform[1e4, 5e7], uniform targets, lmax = min(2 N_side, 4096).
cfg 5  serving requests: N_side in {256,1024,2048,4096} w.p. {.4,.3,.2,.1}, T or
       T+Q+U w.p. 1/2, K 32, one displaced target per pixel.
Lensing potential: C^phiphi ~ l^-4 (2 <= l <= lmax), 2.5' rms deflection.
"""
import numpy as np
import torch

from . import seeds
from .spectra import cl_config1, cl_acoustic, cl_phi
from .synth import draw_alm, draw_alm_te, synth
from .lens import displaced_pixel_centres

SHAPES = {
    1: dict(nside=64, lmax=128, K=16, fields="T"),
    2: dict(nside=512, lmax=1024, K=24, fields="TQU"),
    3: dict(nside=4096, lmax=4096, K=32, fields="TQU"),
}


def spectra(cfg, lmax):
    if cfg == 1:
        tt = cl_config1(lmax)
        z = np.zeros_like(tt)
        return tt, z, z, z
    return cl_acoustic(lmax)


def lensing_targets(cfg, nside, lmax, device="cpu", job=0):
    """Displaced pixel centres (theta', phi') from a seeded potential."""
    rng = seeds.rng(cfg, job, seeds.STREAM_PHI)
    plm = draw_alm(rng, cl_phi(lmax), lmax)
    ell = np.arange(lmax + 1, dtype=np.float64)
    e = -np.sqrt(ell * (ell + 1.0))[:, None] * plm
    dth, dph = synth(e, 1, nside, device)
    return displaced_pixel_centres(nside, dth, dph, device)


def maps(cfg, nside, lmax, fields, device="cpu", job=0):
    """Seeded T (and Q, U) RING maps at pixel centres, float64 tensors."""
    tt, ee, te, bb = spectra(cfg, lmax)
    rng = seeds.rng(cfg, job, seeds.STREAM_ALM)
    out = {}
    if fields == "T":
        out["T"] = synth(draw_alm(rng, tt, lmax), 0, nside, device)
        return out
    aT, aE = draw_alm_te(rng, tt, ee, te, lmax)
    out["T"] = synth(aT, 0, nside, device)
    q, u = synth(-aE, 2, nside, device)
    out["Q"], out["U"] = q, u
    return out


def build(cfg, device="cpu", job=0, **override):
    """Full input set of a lensing config: maps, targets and spectra."""
    sh = dict(SHAPES[cfg])
    sh.update(override)
    nside, lmax = sh["nside"], sh["lmax"]
    tt, ee, te, bb = spectra(cfg, lmax)
    m = maps(cfg, nside, lmax, sh["fields"], device, job)
    th, ph = lensing_targets(cfg, nside, lmax, device, job)
    return dict(shape=sh, cl_tt=tt, cl_ee=ee, cl_bb=bb, cl_te=te, maps=m, theta=th, phi=ph)


def parity_subset(cfg, n_total, n_sub, job=0):
    """Seeded random subset of target indices (uniform, without replacement)."""
    rng = seeds.rng(cfg, job, seeds.STREAM_SUBSET)
    if n_sub >= n_total:
        return np.arange(n_total)
    return np.sort(rng.choice(n_total, size=n_sub, replace=False))


def batch_jobs(n_jobs=64, total_scale=1.0):
    """Job list of the batched uneven workload (sizes only)."""
    rng = seeds.rng(4, 0, seeds.STREAM_TARGETS)
    jobs = []
    for j in range(n_jobs):
        nside = int(rng.choice([128, 256, 512, 1024, 2048]))
        spin = int(rng.choice([0, 2]))
        K = int(rng.choice([16, 24, 32, 48]))
        n = int(np.exp(rng.uniform(np.log(1e4), np.log(5e7))) * total_scale)
        jobs.append(dict(job=j, nside=nside, spin=spin, K=K, n=max(n, 1),
                         lmax=min(2 * nside, 4096)))
    return jobs


def uniform_targets(cfg, job, n, device="cpu"):
    rng = seeds.rng(cfg, job, seeds.STREAM_TARGETS)
    z = rng.uniform(-1.0, 1.0, n)
    ph = rng.uniform(0.0, 2 * np.pi, n)
    th = np.arccos(z)
    return (torch.as_tensor(th, dtype=torch.float64, device=device),
            torch.as_tensor(ph, dtype=torch.float64, device=device))
