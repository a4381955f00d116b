"""Batched persistent execution (flints_batch_*): every job of a mixed batch
(N_side, K, spin, system-size class, single-plan side path) must reproduce
flints_interpolate bit for bit, also when replayed from a captured HIP graph
and with autotuned tiles; one batched job is also checked against the oracle."""
import numpy as np
import pytest
import torch

import paper_1003_4984_amd as fl
from oracle import kriging
from workload import spectra, synth, seeds

from _gpu_helpers import dev, gpu_stencil, reconcile_stencils, compare

pytestmark = pytest.mark.gpu

# (nside, K, spin, precision, var_kind, points): classes n <= 16, 32, 48, 64 for
# both spins, plus FP32, MSE and 80-row (spin-2 K 40) jobs on the single-plan
# path and an empty job
JOBS = [
    (32, 12, 0, fl.FP64, fl.VAR_PAPER, 9000),
    (64, 16, 2, fl.FP64, fl.VAR_PAPER, 20000),
    (16, 8, 2, fl.FP64, fl.VAR_PAPER, 5000),
    (64, 24, 0, fl.FP64, fl.VAR_PAPER, 30000),
    (32, 24, 2, fl.FP64, fl.VAR_PAPER, 7000),
    (64, 40, 0, fl.FP64, fl.VAR_PAPER, 6000),
    (32, 32, 2, fl.FP64, fl.VAR_PAPER, 12000),
    (64, 64, 0, fl.FP64, fl.VAR_PAPER, 3000),
    (32, 16, 0, fl.FP32_IR, fl.VAR_PAPER, 4000),
    (32, 16, 2, fl.FP64, fl.VAR_MSE, 4000),
    (32, 40, 2, fl.FP64, fl.VAR_PAPER, 1500),
    (16, 16, 0, fl.FP64, fl.VAR_PAPER, 0),
]


def _make(seed=0):
    jobs = []
    for i, (nside, K, spin, prec, vk, npts) in enumerate(JOBS):
        lmax = 2 * nside
        tt, ee, te, bb = spectra.cl_acoustic(lmax)
        rng = seeds.rng(40 + seed, i, 0)
        if spin == 0:
            cl = tt
            m = synth.synth(synth.draw_alm(rng, tt, lmax), 0, nside)
        else:
            cl = np.concatenate([ee, 0.1 * ee])
            q, u = synth.synth(-synth.draw_alm(rng, ee, lmax), 2, nside)
            m = torch.cat([q, u])
        p = fl.Plan(nside, lmax, cl, K, spin, precision=prec, var_kind=vk)
        th = dev(np.arccos(rng.uniform(-1, 1, npts)))
        ph = dev(rng.uniform(0, 2 * np.pi, npts))
        nf = 1 if spin == 0 else 2
        out = torch.full((nf * npts,), 7.0, dtype=torch.float64, device="cuda")
        var = torch.full((nf * npts,), 7.0, dtype=torch.float64, device="cuda")
        jobs.append((p, dev(m.numpy()), th, ph, out, var))
    return jobs


def _single(jobs):
    ref = []
    for p, m, th, ph, _, _ in jobs:
        o, v = fl.interpolate(p, m, th, ph)
        ref.append((o, v))
    torch.cuda.synchronize()
    return ref


def _check_equal(jobs, ref):
    for i, ((_, _, _, _, out, var), (o, v)) in enumerate(zip(jobs, ref)):
        assert torch.equal(out, o), f"job {i}: values differ from flints_interpolate"
        assert torch.equal(var, v), f"job {i}: variances differ from flints_interpolate"


def test_batch_equals_single(gpu_ok):
    jobs = _make()
    ref = _single(jobs)
    b = fl.Batch(jobs)
    info = b.info()
    assert info["njobs"] == len(JOBS) and info["classes"] >= 4
    assert all((t > 0) == (w > 0) for t, w in zip(info["tiles"], info["waves_per_block"]))
    assert info["fused_jobs"] == sum(1 for j in JOBS if j[3] == fl.FP64 and j[4] == fl.VAR_PAPER and j[5] > 0
                                     and (j[1] if j[2] == 0 else 2 * j[1]) <= 64)
    b.run()
    torch.cuda.synchronize()
    _check_equal(jobs, ref)
    # a second run over outputs reset to garbage gives the same result
    for *_, out, var in jobs:
        out.fill_(-3.0)
        var.fill_(-3.0)
    b.run()
    torch.cuda.synchronize()
    _check_equal(jobs, ref)
    b.close()


def test_batch_graph_replays(gpu_ok):
    jobs = _make(1)
    ref = _single(jobs)
    b = fl.Batch(jobs)
    s = torch.cuda.Stream()
    b.capture(s)
    assert b.info()["captured"] == 1
    for rep in range(3):
        for *_, out, var in jobs:
            out.fill_(float(rep) + 0.5)
            var.fill_(float(rep) + 0.5)
        torch.cuda.synchronize()
        b.run(s)
        s.synchronize()
        _check_equal(jobs, ref)
        torch.cuda.synchronize()
    b.close()


def test_batch_autotune(gpu_ok):
    jobs = _make(2)
    ref = _single(jobs)
    b = fl.Batch(jobs, autotune=True)
    info = b.info()
    for c in range(len(info["tiles"])):
        if info["tiles"][c]:
            # launch groups 12.. are the tile engines, whose waves take tiles one by one
            sizes = (64, 128, 256, 1024) if c >= 12 else (256, 1024, 4096, 16384)
            assert info["tile_points"][c] in sizes
            assert 1 <= info["waves_per_block"][c] <= 8
    for *_, out, var in jobs:
        out.fill_(0.0)
        var.fill_(0.0)
    b.run()
    torch.cuda.synchronize()
    _check_equal(jobs, ref)
    b.close()


def test_batched_job_against_oracle(gpu_ok):
    jobs = _make(3)
    b = fl.Batch(jobs)
    b.run()
    torch.cuda.synchronize()
    p, m, th, ph, out, var = jobs[6]          # spin 2, K 32 (tile class n <= 64)
    nside, lmax = p.nside, p.lmax
    tt, ee, te, bb = spectra.cl_acoustic(lmax)
    sel = np.arange(0, th.numel(), 97)
    thn, phn = th.cpu().numpy()[sel], ph.cpu().numpy()[sel]
    g = gpu_stencil(p, thn, phn)
    reconcile_stencils(nside, thn, phn, g, kriging.stencils(nside, thn, phn, p.K))
    mm = m.cpu().numpy()
    npix = 12 * nside * nside
    vo, varo, _ = kriging.interpolate(nside, (ee, 0.1 * ee), p.K, 2, (mm[:npix], mm[npix:]), thn, phn,
                                      stencil_idx=g)
    n = th.numel()
    o = out.cpu().numpy().reshape(2, n).T[sel]
    v = var.cpu().numpy().reshape(2, n).T[sel]
    compare(o, v, vo, varo, 1e-8, 1e-4, 1e-9 * p.info()["sigma2"])
    b.close()
