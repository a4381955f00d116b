"""Benchmark: lensed T/Q/U kriging interpolation at N_side 4096 on one MI355X.

Workload (one step): a full-sky lensing remap at N_side = 4096 (201,326,592
pixels), lmax = 4096, K = 32 nearest pixels -- every displaced pixel centre is
interpolated in T (spin-0 plan) and in Q, U (spin-2 plan, full xi+/xi- mode),
with the kriging variance of each field.  Inputs (seeded Gaussian maps with
damped acoustic spectra, 2.5' rms lensing deflection) are generated on the GPU
before timing and stay resident in HBM.

Prints ONE JSON line.  `value` counts interpolated field samples (T, Q and U
separately) per second.  `roofline` is the dominant kernel's algorithmic FP64
flop rate (the T+Q/U call with shared stencils, or with --tqu separate the
spin-2 launch),
timed with HIP events on the launch stream, against the MI355X FP64 vector
peak.  `cpu_baseline` is the FP64 CPU
oracle on a bounded sample of the same workload, which also serves as a
sampled parity check of this very run.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

FP64_PEAK_TFLOPS = 78.6          # MI355X FP64 vector (and matrix) peak
SHAPES = {
    "nside4096": dict(cfg=3, nside=4096, lmax=4096, K=32),
    "nside512": dict(cfg=2, nside=512, lmax=1024, K=24),
}


def flops_spin0(K):
    """Algorithmic flops per point, spin 0 (LAPACK convention): Cholesky K^3/3
    FMAs, two triangular solves, 20 flops per covariance entry."""
    return 2.0 / 3.0 * K ** 3 + 2 * K ** 2 + 4 * K + 20 * (K * (K + 1) / 2 + K)


def flops_spin2(K):
    """Algorithmic flops per point, spin 2 full mode: Cholesky of 2K x 2K, solves
    for 2 right-hand sides, 60 flops per 2x2 covariance block."""
    return 16.0 / 3.0 * K ** 3 + 16 * K ** 2 + 60 * (K * (K + 1) / 2 + K)


# Counter summaries of the dominant work per T+Q+U mode (shared: all kernels of
# the shared-stencil T+Q/U call; separate: the spin-2 launch).
TRAFFIC_FILES = {
    "shared": os.path.join(ROOT, "profiles", "traffic_interp_tqu_nside4096_K32.md"),
    "separate": os.path.join(ROOT, "profiles", "traffic_interp_tile_nside4096_K32.md"),
}


# Sources outside the measured single-plan and T+Q/U kernels: the batched
# launches, the pixel-tied stencils, supersampling and the synthesis (each a
# translation unit of its own that the measured kernels do not include).
NOT_MEASURED = ("batch.hip", "fixed.hip", "supersample.hip", "sht.hip")


def kernel_source_hash():
    """sha256 of the sources of the measured kernels (all of csrc but the batch
    file) with comments and blank space removed (a change of
    comments does not change the kernels the counters measured)."""
    import glob
    import hashlib
    import re
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_1003_4984_amd", "csrc")
    for f in sorted(glob.glob(os.path.join(csrc, "*.hip")) + glob.glob(os.path.join(csrc, "*.h"))):
        if os.path.basename(f) in NOT_MEASURED:
            continue
        with open(f) as fh:
            text = fh.read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        text = re.sub(r"//[^\n]*", "", text)
        text = re.sub(r"\s+", " ", text)
        h.update(os.path.basename(f).encode())
        h.update(text.encode())
    return h.hexdigest()


def measured_traffic(workload, mode="shared"):
    """HBM bytes per launch of the dominant kernel from the committed counter
    summary (FETCH_SIZE + WRITE_SIZE, copy-calibrated), or None if that summary
    is for other kernel sources or another workload."""
    path = TRAFFIC_FILES[mode]
    if workload != "nside4096" or not os.path.exists(path):
        return None
    vals = {}
    with open(path) as fh:
        for line in fh:
            if ":" in line and line.split(":")[0] in ("traffic_bytes_per_launch", "source_sha256"):
                k, v = line.split(":", 1)
                vals[k] = v.strip()
    if vals.get("source_sha256") != kernel_source_hash():
        return None
    return float(vals["traffic_bytes_per_launch"])


def log(msg):
    print(f"[bench {time.strftime('%H:%M:%S')}] {msg}", file=sys.stderr, flush=True)


def make_inputs(shape, device):
    import torch
    from workload import configs, spectra
    cfg, nside, lmax = shape["cfg"], shape["nside"], shape["lmax"]
    tt, ee, te, bb = spectra.cl_acoustic(lmax)
    log(f"synthesising T, Q, U maps at nside {nside}, lmax {lmax}")
    maps = configs.maps(cfg, nside, lmax, "TQU", device)
    log("synthesising the lensing deflection and displaced targets")
    th, ph = configs.lensing_targets(cfg, nside, lmax, device)
    qu = torch.cat([maps["Q"], maps["U"]])
    torch.cuda.synchronize()
    return dict(T=maps["T"], QU=qu, theta=th, phi=ph, tt=tt, ee=ee, bb=bb)


def host_workers():
    """Worker processes for the oracle baseline: the host cores this process
    may run on, at most 16 (one GPU's share of a shared host)."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    cap = int(os.environ.get("OMP_NUM_THREADS", "16") or 16)
    return max(1, min(n, cap, 16))


def _worker_init():
    from threadpoolctl import threadpool_limits
    global _BLAS_LIMIT
    _BLAS_LIMIT = threadpool_limits(limits=1)   # one BLAS thread per worker process


def _stencil_chunk(args):
    from oracle import kriging
    nside, th, ph, K = args
    return kriging.stencils(nside, th, ph, K)


class _StencilValues:
    """Map lookup pix -> value over the pixels of a chunk's stencils only."""

    def __init__(self, pix, vals):
        self.pix, self.vals = pix, vals

    def __call__(self, p):
        p = np.asarray(p)
        return self.vals[np.searchsorted(self.pix, p.ravel())].reshape(p.shape)


def _krige_chunk(args):
    from oracle import kriging
    nside, K, tt, eebb, th, ph, st, pix, tv, qv, uv = args
    v0, w0, _ = kriging.interpolate(nside, tt, K, 0, _StencilValues(pix, tv), th, ph, stencil_idx=st)
    v2, w2, _ = kriging.interpolate(nside, eebb, K, 2, (_StencilValues(pix, qv), _StencilValues(pix, uv)),
                                    th, ph, stencil_idx=st)
    return v0, w0, v2, w2


# Parity gate of the sampled comparison (the target contract): values within
# 2e-4 of the rms value (L-infinity), variances within 1e-2 relative.
VAL_TOL, VAR_TOL = 2e-4, 1e-2


def oracle_pool():
    """Spawned worker processes for the oracle (started before this process
    touches the GPU, one BLAS thread each) and their count."""
    import multiprocessing as mp
    nw = host_workers()
    pool = mp.get_context("spawn").Pool(nw, initializer=_worker_init)
    pool.map(_worker_init_probe, range(nw))
    return pool, nw


def cpu_baseline(pool, nw, shape, inp, out_t, var_t, out_qu, var_qu, n_sample, seed_cfg):
    """FP64 oracle on a seeded sample of targets, spread over the host cores
    (the worker pool); returns the baseline record and the sampled parity of
    this run's GPU outputs."""
    import torch
    from workload import configs
    nside, K = shape["nside"], shape["K"]
    n = inp["theta"].numel()
    sel = configs.parity_subset(seed_cfg, n, n_sample)
    sel_t = torch.as_tensor(sel, device=inp["theta"].device)
    th = inp["theta"][sel_t].cpu().numpy()
    ph = inp["phi"][sel_t].cpu().numpy()
    npix = 12 * nside * nside
    chunks = np.array_split(np.arange(len(sel)), nw * 4)
    chunks = [c for c in chunks if c.size]
    t0 = time.perf_counter()
    st = np.concatenate(pool.map(_stencil_chunk, [(nside, th[c], ph[c], K) for c in chunks]))
    work = []
    for c in chunks:
        pix = np.unique(st[c])
        pt = torch.as_tensor(pix, device=inp["T"].device)
        tv = inp["T"][pt].cpu().numpy()
        qv = inp["QU"][pt].cpu().numpy()
        uv = inp["QU"][pt + npix].cpu().numpy()
        work.append((nside, K, inp["tt"], (inp["ee"], inp["bb"]), th[c], ph[c], st[c], pix, tv, qv, uv))
    res = pool.map(_krige_chunk, work)
    dt = time.perf_counter() - t0
    v0 = np.concatenate([r[0] for r in res])
    w0 = np.concatenate([r[1] for r in res])
    v2 = np.concatenate([r[2] for r in res])
    w2 = np.concatenate([r[3] for r in res])
    g0 = out_t[sel_t].cpu().numpy()
    gv0 = var_t[sel_t].cpu().numpy()
    gq = out_qu[sel_t].cpu().numpy()
    gu = out_qu[sel_t + n].cpu().numpy()
    gvq = var_qu[sel_t].cpu().numpy()
    gvu = var_qu[sel_t + n].cpu().numpy()

    def rel(g, o):
        return float(np.max(np.abs(g - o)) / np.sqrt(np.mean(o ** 2)))

    def vrel(g, o):
        return float(np.max(np.abs(g - o) / np.abs(o)))

    verr = {"T": rel(g0, v0), "Q": rel(gq, v2[:, 0]), "U": rel(gu, v2[:, 1])}
    werr = {"T": vrel(gv0, w0), "Q": vrel(gvq, w2[:, 0]), "U": vrel(gvu, w2[:, 1])}
    ok = all(np.isfinite(v) and v <= VAL_TOL for v in verr.values()) and \
        all(np.isfinite(v) and v <= VAR_TOL for v in werr.values())
    parity = {"points": int(len(sel)), "value_err_rel_rms": verr, "var_err_rel": werr,
              "tolerance": {"value_rel_rms": VAL_TOL, "var_rel": VAR_TOL}, "parity_ok": bool(ok)}
    base = {"value": 3.0 * len(sel) / dt, "unit": "samples/s", "cores": nw, "kind": "oracle",
            "sample": f"{len(sel)} seeded targets of the same N_side {nside} T+Q+U workload "
                      f"(K={K}, exact per-pair correlation sums to lmax {shape['lmax']}), "
                      f"{dt:.1f} s of numpy over {nw} worker processes (one BLAS thread each)"}
    return base, parity


def _worker_init_probe(_):
    return os.getpid()


# ---------------------------------------------------------------------------- extra legs
def _time_calls(torch, fn, steps, warmup=1):
    """Mean seconds per call of fn() over `steps` calls (HIP events on the
    current stream) after `warmup` untimed calls."""
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    for a, b in evs:
        a.record()
        fn()
        b.record()
    torch.cuda.synchronize()
    return float(np.mean([a.elapsed_time(b) for a, b in evs])) * 1e-3


def leg_nside512(fl, torch, pool, nw):
    """N_side 512, lmax 1024, K 24, T+Q+U: FP64 and FP32 + refinement, each
    with its fallback fraction and a sampled parity check against the oracle."""
    from workload import configs, spectra
    sh = SHAPES["nside512"]
    nside, lmax, K = sh["nside"], sh["lmax"], sh["K"]
    tt, ee, te, bb = spectra.cl_acoustic(lmax)
    m = configs.maps(2, nside, lmax, "TQU", "cuda")
    th, ph = configs.lensing_targets(2, nside, lmax, "cuda")
    inp = dict(T=m["T"], QU=torch.cat([m["Q"], m["U"]]), theta=th, phi=ph, tt=tt, ee=ee, bb=bb)
    n = th.numel()
    res = {"workload": f"lensing remap N_side {nside} lmax {lmax} K {K} T+Q+U, one displaced target per pixel"}
    for prec, code in (("fp64", fl.FP64), ("fp32ir", fl.FP32_IR)):
        p0 = fl.Plan(nside, lmax, tt, K, 0, precision=code)
        p2 = fl.Plan(nside, lmax, np.concatenate([ee, bb]), K, 2, precision=code)
        o = [torch.empty(k * n, dtype=torch.float64, device="cuda") for k in (1, 1, 2, 2)]
        call = lambda: fl.interpolate_tqu(p0, p2, inp["T"], inp["QU"], th, ph, out_t=o[0], var_t=o[1],
                                          out_qu=o[2], var_qu=o[3])
        call()
        torch.cuda.synchronize()
        p0.reset_stats()
        p2.reset_stats()
        t = _time_calls(torch, call, steps=5, warmup=0)
        st0, st2 = p0.stats(), p2.stats()
        r = {"samples_per_s": 3.0 * n / t, "s_per_step": t, "tqu_shared": bool(fl.tqu_shared(p0, p2)),
             "plan_precision_run": {"T": "fp64" if p0.info()["precision"] == fl.FP64 else "fp32ir",
                                    "QU": "fp64" if p2.info()["precision"] == fl.FP64 else "fp32ir"},
             "fp32_probe_reject": {"T": p0.info()["fp32_probe_reject"], "QU": p2.info()["fp32_probe_reject"]},
             "fp64_recompute_fraction": {"T": st0["fp64_fallbacks"] / (5 * n),
                                         "QU": st2["fp64_fallbacks"] / (5 * n)}}
        if pool is not None:
            _, par = cpu_baseline(pool, nw, sh, inp, o[0], o[1], o[2], o[3], 600, 2)
            r["parity_sample"] = par
        res[prec] = r
    res["fp32ir_speedup_over_fp64"] = res["fp64"]["s_per_step"] / res["fp32ir"]["s_per_step"]
    return res


def leg_supersample(fl, torch):
    """The paper's supersampling shape (Table 1): a T map at N_side 2048,
    lmax 4096, interpolated at every pixel centre of N_side 4096, K = 9 and
    36 nearest pixels.  Paper context: 3.3 min (K 9) and 19 min (K 36) on one
    Xeon E5410 core with tabulated S^-1."""
    from workload import configs, spectra
    nside, nout, lmax = 2048, 4096, 4096
    tt, ee, te, bb = spectra.cl_acoustic(lmax)
    m = configs.maps(3, nside, lmax, "T", "cuda")["T"]
    npo = 12 * nout * nout
    out = torch.empty(npo, dtype=torch.float64, device="cuda")
    var = torch.empty(npo, dtype=torch.float64, device="cuda")
    res = {"workload": f"supersampling N_side {nside} -> {nout}, lmax {lmax}, T", "targets": npo}
    paper_s = {9: 3.3 * 60, 36: 19 * 60}
    for K in (9, 36):
        p = fl.Plan(nside, lmax, tt, K, 0)
        t = _time_calls(torch, lambda: fl.supersample(p, m, nout, out=out, var=var), steps=2)
        res[f"K{K}"] = {"samples_per_s": npo / t, "s_per_map": t,
                        "paper_cpu_s_per_map": paper_s[K],
                        "paper_context": "Table 1, one Xeon E5410 2.33 GHz core, tabulated S^-1 stencil"}
    return res


def _oracle_parity_on(pool, nside, K, tt, eebb, inp, th, ph, st, g0, gv0, g2, gv2):
    """Oracle values on the GPU's own stencils st (n, K) at (th, ph) in the
    worker pool, compared with the GPU outputs (g0, gv0: T; g2, gv2: (n, 2))."""
    import torch
    npix = 12 * nside * nside
    chunks = [c for c in np.array_split(np.arange(len(th)), 32) if c.size]
    work = []
    for c in chunks:
        pix = np.unique(st[c])
        pt = torch.as_tensor(pix, device=inp["T"].device)
        work.append((nside, K, tt, eebb, th[c], ph[c], st[c], pix, inp["T"][pt].cpu().numpy(),
                     inp["QU"][pt].cpu().numpy(), inp["QU"][pt + npix].cpu().numpy()))
    res = pool.map(_krige_chunk, work)
    v0 = np.concatenate([r[0] for r in res])
    w0 = np.concatenate([r[1] for r in res])
    v2 = np.concatenate([r[2] for r in res])
    w2 = np.concatenate([r[3] for r in res])
    rel = lambda g, o: float(np.max(np.abs(g - o)) / np.sqrt(np.mean(o ** 2)))
    vrel = lambda g, o: float(np.max(np.abs(g - o) / np.abs(o)))
    verr = {"T": rel(g0, v0), "Q": rel(g2[:, 0], v2[:, 0]), "U": rel(g2[:, 1], v2[:, 1])}
    werr = {"T": vrel(gv0, w0), "Q": vrel(gv2[:, 0], w2[:, 0]), "U": vrel(gv2[:, 1], w2[:, 1])}
    ok = all(v <= VAL_TOL for v in verr.values()) and all(v <= VAR_TOL for v in werr.values())
    return {"points": int(len(th)), "value_err_rel_rms": verr, "var_err_rel": werr, "parity_ok": bool(ok)}


def leg_pixel_stencils(fl, torch, inp_main, pool):
    """The paper's own scheme (stencil tied to the containing pixel, factors
    tabulated per pixel class) at the lensing shape of its Table 2: N_side
    4096, lmax 4096, K 9, T + Q + U at the main workload's lensed pixel centres
    (paper: 22 min of interpolation for N_side 4096); and the supersampling
    shape of its Table 1 (N_side 2048 -> 4096, lmax 4096, T, K 9 and 36;
    paper: 3.3 and 19 min).  Plan times include the class tables."""
    from workload import configs, spectra
    res = {}
    nside, lmax, K = 4096, 4096, 9
    tt, ee, te, bb = spectra.cl_acoustic(lmax)
    t0 = time.perf_counter()
    p0 = fl.Plan(nside, lmax, tt, K, 0, stencil=fl.STENCIL_PIXEL)
    p2 = fl.Plan(nside, lmax, np.concatenate([ee, bb]), K, 2, stencil=fl.STENCIL_PIXEL)
    torch.cuda.synchronize()
    t_plan = time.perf_counter() - t0
    th, ph = inp_main["theta"], inp_main["phi"]
    n = th.numel()
    o0 = torch.empty(n, dtype=torch.float64, device="cuda")
    v0 = torch.empty(n, dtype=torch.float64, device="cuda")
    o2 = torch.empty(2 * n, dtype=torch.float64, device="cuda")
    v2 = torch.empty(2 * n, dtype=torch.float64, device="cuda")

    def call():
        fl.interpolate(p0, inp_main["T"], th, ph, out=o0, var=v0)
        fl.interpolate(p2, inp_main["QU"], th, ph, out=o2, var=v2)
    t = _time_calls(torch, call, steps=3)
    i0, i2 = p0.info(), p2.info()
    r = {"workload": f"lensing remap N_side {nside} lmax {lmax} K {K} T+Q+U, stencil of the containing pixel",
         "samples_per_s": 3.0 * n / t, "s_per_step": t, "plan_s": t_plan,
         "pixel_classes": {"T": i0["pixel_classes"], "QU": i2["pixel_classes"]},
         "table_gib": {"T": i0["table_bytes"] / 2 ** 30, "QU": i2["table_bytes"] / 2 ** 30},
         "paper_cpu_s_per_step": 22 * 60,
         "paper_context": "Table 2 interpolation time, N_side 4096 (hardware not stated)"}
    if pool is not None:
        sel = configs.parity_subset(3, n, 600, job=2)
        sel_t = torch.as_tensor(sel, device="cuda")
        ths, phs = th[sel_t].contiguous(), ph[sel_t].contiguous()
        st = fl.stencil(p0, ths, phs).cpu().numpy()
        g2 = torch.stack([o2[sel_t], o2[sel_t + n]], 1).cpu().numpy()
        gv2 = torch.stack([v2[sel_t], v2[sel_t + n]], 1).cpu().numpy()
        r["parity_sample"] = _oracle_parity_on(pool, nside, K, tt, (ee, bb), inp_main, ths.cpu().numpy(),
                                               phs.cpu().numpy(), st, o0[sel_t].cpu().numpy(),
                                               v0[sel_t].cpu().numpy(), g2, gv2)
    res["lensing_tqu_K9"] = r
    del p0, p2, o0, v0, o2, v2
    torch.cuda.empty_cache()
    # supersampling N_side 2048 -> 4096 (Table 1 shape)
    ns, nout = 2048, 4096
    m = configs.maps(3, ns, lmax, "T", "cuda")["T"]
    npo = 12 * nout * nout
    out = torch.empty(npo, dtype=torch.float64, device="cuda")
    var = torch.empty(npo, dtype=torch.float64, device="cuda")
    paper_s = {9: 3.3 * 60, 36: 19 * 60}
    for Kk in (9, 36):
        t0 = time.perf_counter()
        p = fl.Plan(ns, lmax, tt, Kk, 0, stencil=fl.STENCIL_PIXEL)
        torch.cuda.synchronize()
        t_plan = time.perf_counter() - t0
        t = _time_calls(torch, lambda: fl.supersample(p, m, nout, out=out, var=var), steps=2)
        res[f"supersample_2048_to_4096_K{Kk}"] = {
            "samples_per_s": npo / t, "s_per_map": t, "plan_s": t_plan,
            "pixel_classes": p.info()["pixel_classes"], "table_gib": p.info()["table_bytes"] / 2 ** 30,
            "paper_cpu_s_per_map": paper_s[Kk],
            "paper_context": "Table 1, one Xeon E5410 2.33 GHz core, tabulated S^-1 stencil"}
        del p
        torch.cuda.empty_cache()
    return res


def leg_large_systems(fl, torch, inp_main, pool, stride=48):
    """K 48 at the headline's N_side 4096, lmax 4096 maps, on every 48th target
    of the headline workload: spin 0 (48-row systems, tile engine) and spin 2
    (96-row systems, the LDS elimination), with a sampled parity check against
    the oracle."""
    from workload import configs
    nside, K = 4096, 48
    tt, ee, bb = inp_main["tt"], inp_main["ee"], inp_main["bb"]
    lmax = len(tt) - 1
    th = inp_main["theta"][::stride].contiguous()
    ph = inp_main["phi"][::stride].contiguous()
    n = th.numel()
    p0 = fl.Plan(nside, lmax, tt, K, 0)
    p2 = fl.Plan(nside, lmax, np.concatenate([ee, bb]), K, 2)
    o0 = torch.empty(n, dtype=torch.float64, device="cuda")
    v0 = torch.empty(n, dtype=torch.float64, device="cuda")
    o2 = torch.empty(2 * n, dtype=torch.float64, device="cuda")
    v2 = torch.empty(2 * n, dtype=torch.float64, device="cuda")
    t0 = _time_calls(torch, lambda: fl.interpolate(p0, inp_main["T"], th, ph, out=o0, var=v0), steps=2)
    t2 = _time_calls(torch, lambda: fl.interpolate(p2, inp_main["QU"], th, ph, out=o2, var=v2), steps=2)
    r = {"workload": f"N_side {nside} lmax {lmax} K {K}, every {stride}th headline target",
         "targets": n,
         "T": {"rows": K, "engine": "tile", "samples_per_s": n / t0, "s": t0},
         "QU": {"rows": 2 * K, "engine": "LDS elimination", "samples_per_s": 2.0 * n / t2, "s": t2},
         "stats": {"T": p0.stats(), "QU": p2.stats()}}
    if pool is not None:
        sel = configs.parity_subset(3, n, 200, job=5)
        sel_t = torch.as_tensor(sel, device="cuda")
        ths, phs = th[sel_t].contiguous(), ph[sel_t].contiguous()
        st = fl.stencil(p0, ths, phs).cpu().numpy()
        g2 = torch.stack([o2[sel_t], o2[sel_t + n]], 1).cpu().numpy()
        gv2 = torch.stack([v2[sel_t], v2[sel_t + n]], 1).cpu().numpy()
        r["parity_sample"] = _oracle_parity_on(pool, nside, K, tt, (ee, bb), inp_main, ths.cpu().numpy(),
                                               phs.cpu().numpy(), st, o0[sel_t].cpu().numpy(),
                                               v0[sel_t].cpu().numpy(), g2, gv2)
    return r


_LENS_ALM = None


def _lens_alm():
    """The seeded harmonic coefficients of the headline lensing workload
    (T, E and the lensing potential at lmax 4096; drawn once per process)."""
    global _LENS_ALM
    if _LENS_ALM is None:
        from workload import seeds, spectra
        from workload.synth import draw_alm, draw_alm_te
        lmax = 4096
        tt, ee, te, bb = spectra.cl_acoustic(lmax)
        aT, aE = draw_alm_te(seeds.rng(3, 0, seeds.STREAM_ALM), tt, ee, te, lmax)
        plm = draw_alm(seeds.rng(3, 0, seeds.STREAM_PHI), spectra.cl_phi(lmax), lmax)
        _LENS_ALM = (aT, aE, plm)
    return _LENS_ALM


def _lens_pixel_task(args):
    """Oracle chain at one pixel of N_side 4096: the unlensed T and Q + iU at
    its centre, grad(phi) there, the displaced direction and the exact lensed
    T and Q + iU at it (sums over all l, m)."""
    from oracle import healpix, lensing
    nside, pix = args
    aT, aE, plm = _lens_alm()
    lmax = aT.shape[0] - 1
    th, ph = healpix.pix2ang(nside, np.array([pix]))
    ell = np.arange(lmax + 1, dtype=np.float64)
    t0 = lensing.synth_points_recurrence(0, aT, None, th, ph).real
    p0 = lensing.synth_points_recurrence(2, -aE, None, th, ph)
    d = lensing.synth_points_recurrence(1, -np.sqrt(ell * (ell + 1))[:, None] * plm, None, th, ph)
    t2, p2 = lensing.lensed_directions(th, ph, d.real, d.imag)
    t1 = lensing.synth_points_recurrence(0, aT, None, t2, p2).real
    p1 = lensing.synth_points_recurrence(2, -aE, None, t2, p2)
    return float(t0[0]), complex(p0[0]), complex(d[0]), float(t2[0]), float(p2[0]), float(t1[0]), complex(p1[0])


def leg_lensing_pipeline(fl, torch, inp_main, pool, n_pix=48):
    """The paper's total lensing time (Table 2: interpolation + unlensed map
    synthesis + deflection map, initialisation excluded) on the device at
    N_side 4096, lmax 4096: spin-0 and spin-2 synthesis of the unlensed T and
    Q, U, spin-1 synthesis of grad(phi), the displaced pixel centres and T+Q/U
    interpolation there -- with the K 32 nearest-pixel plans of the headline
    and with the paper's K 9 pixel-tied stencils.  With the oracle pool, the
    synthesised maps, deflections and directions are checked at sampled pixels
    against the oracle's chain from the same coefficients, and the
    interpolated values against the exact lensed sky there (the paper's
    precision measure: error std and max over the map std)."""
    from workload import spectra, configs
    nside, lmax = 4096, 4096
    npix = 12 * nside * nside
    tt, ee, te, bb = spectra.cl_acoustic(lmax)
    aT, aE, plm = _lens_alm()
    tlm = torch.as_tensor(fl.alm_mmajor(aT), device="cuda")
    elm = torch.as_tensor(fl.alm_mmajor(aE), device="cuda")
    ell = np.arange(lmax + 1, dtype=np.float64)
    plm_d = torch.as_tensor(fl.alm_mmajor(plm), device="cuda")
    t_map = torch.empty(npix, dtype=torch.float64, device="cuda")
    qu_map = torch.empty(2 * npix, dtype=torch.float64, device="cuda")
    defl = torch.empty(2 * npix, dtype=torch.float64, device="cuda")
    th = torch.empty(npix, dtype=torch.float64, device="cuda")
    ph = torch.empty(npix, dtype=torch.float64, device="cuda")
    stages = {
        "synth_T_s": lambda: fl.synthesize(nside, lmax, 0, tlm, out=t_map),
        "synth_QU_s": lambda: fl.synthesize(nside, lmax, 2, elm, None, out=qu_map),
        "synth_deflection_s": lambda: fl.synthesize(nside, lmax, 1, plm_d, out=defl),
        "displace_s": lambda: fl.lensed_directions(nside, defl, th, ph),
    }
    res = {"workload": f"lensing pipeline N_side {nside} lmax {lmax}: synthesis of T, Q, U and grad(phi), "
                       "displaced pixel centres, T+Q/U interpolation (all on the device)"}
    for name, fn in stages.items():
        res[name] = _time_calls(torch, fn, steps=2)
    synth_s = res["synth_T_s"] + res["synth_QU_s"]
    res["unlensed_map_s"] = synth_s
    # consistency with the input generator's maps of the same seeds (not a parity claim)
    res["max_diff_vs_input_generator"] = {
        "T": float((t_map - inp_main["T"]).abs().max() / inp_main["T"].abs().max()),
        "QU": float((qu_map - inp_main["QU"]).abs().max() / inp_main["QU"].abs().max())}
    o = [torch.empty(k * npix, dtype=torch.float64, device="cuda") for k in (1, 1, 2, 2)]
    sel = configs.parity_subset(3, npix, n_pix, job=5)
    oracle = None
    if pool is not None:
        log(f"lensing pipeline: oracle chain at {sel.size} pixels")
        oracle = pool.map(_lens_pixel_task, [(nside, int(p)) for p in sel])
        sel_t = torch.as_tensor(sel, device="cuda")
        ot = np.array([r[0] for r in oracle])
        oqu = np.array([r[1] for r in oracle])
        od = np.array([r[2] for r in oracle])
        gt = t_map[sel_t].cpu().numpy()
        gqu = qu_map[sel_t].cpu().numpy() + 1j * qu_map[sel_t + npix].cpu().numpy()
        gd = defl[sel_t].cpu().numpy() + 1j * defl[sel_t + npix].cpu().numpy()
        from oracle import healpix
        gap = np.linalg.norm(healpix.ang2vec(th[sel_t].cpu().numpy(), ph[sel_t].cpu().numpy())
                             - healpix.ang2vec(np.array([r[3] for r in oracle]), np.array([r[4] for r in oracle])),
                             axis=-1)
        res["parity_sample"] = {
            "pixels": int(sel.size),
            "T_max_err_rel": float(np.max(np.abs(gt - ot)) / np.max(np.abs(ot))),
            "QU_max_err_rel": float(np.max(np.abs(gqu - oqu)) / np.max(np.abs(oqu))),
            "deflection_max_err_rel": float(np.max(np.abs(gd - od)) / np.max(np.abs(od))),
            "direction_max_gap_rad": float(np.max(gap)),
            "tolerance": {"maps_rel": 1e-8, "direction_rad": 1e-12}}
        res["parity_sample"]["parity_ok"] = bool(
            max(res["parity_sample"]["T_max_err_rel"], res["parity_sample"]["QU_max_err_rel"],
                res["parity_sample"]["deflection_max_err_rel"]) < 1e-8
            and res["parity_sample"]["direction_max_gap_rad"] < 1e-12)
        # exact lensed sky at the oracle's displaced directions; map std of the unlensed maps
        ex_t = np.array([r[5] for r in oracle])
        ex_qu = np.array([r[6] for r in oracle])
        sd_t = float(inp_main["T"].std())
        sd_p = float(inp_main["QU"].std())
    for label, kw in (("K32_nearest", dict(K=32)), ("K9_pixel_stencil", dict(K=9, stencil=fl.STENCIL_PIXEL))):
        K = kw.pop("K")
        t0 = time.perf_counter()
        p0 = fl.Plan(nside, lmax, tt, K, 0, **kw)
        p2 = fl.Plan(nside, lmax, np.concatenate([ee, bb]), K, 2, **kw)
        torch.cuda.synchronize()
        plan_s = time.perf_counter() - t0
        call = lambda: fl.interpolate_tqu(p0, p2, t_map, qu_map, th, ph, out_t=o[0], var_t=o[1],
                                          out_qu=o[2], var_qu=o[3])
        t_int = _time_calls(torch, call, steps=2)
        total = synth_s + res["synth_deflection_s"] + res["displace_s"] + t_int
        r = {"interp_s": t_int, "plan_init_s": plan_s, "total_s": total,
             "interp_over_unlensed_synthesis": t_int / synth_s,
             "samples_per_s_total": 3.0 * npix / total}
        if oracle is not None:
            gi_t = o[0][sel_t].cpu().numpy()
            gi_q = o[2][sel_t].cpu().numpy()
            gi_u = o[2][sel_t + npix].cpu().numpy()
            e_t, e_q, e_u = gi_t - ex_t, gi_q - ex_qu.real, gi_u - ex_qu.imag
            r["precision_vs_exact_lensed"] = {
                "pixels": int(sel.size),
                "T": {"L2": float(np.sqrt(np.mean(e_t ** 2)) / sd_t), "Linf": float(np.max(np.abs(e_t)) / sd_t)},
                "Q": {"L2": float(np.sqrt(np.mean(e_q ** 2)) / sd_p), "Linf": float(np.max(np.abs(e_q)) / sd_p)},
                "U": {"L2": float(np.sqrt(np.mean(e_u ** 2)) / sd_p), "Linf": float(np.max(np.abs(e_u)) / sd_p)},
                "note": "interpolated minus exact lensed value (all-l, m sum at the displaced direction), "
                        "over the unlensed map std, as the paper's Table 2 precision columns"}
        res[label] = r
        del p0, p2
        torch.cuda.empty_cache()
    res["paper_context"] = {"total_s": 51 * 60, "interp_s": 22 * 60, "K": 9, "L2": 4e-4, "Linf": 3e-3,
                            "note": "Table 2, N_side 4096, lmax 4096, T+Q+U (hardware not stated)"}
    return res


def leg_serving(fl, torch, inp_main, rate=1.0, n_req=16):
    """Serving: Poisson requests (rate per second) with N_side {256, 1024, 2048,
    4096} (weights .4/.3/.2/.1), T or T+Q+U, K 32, lmax = N_side; each request
    takes its maps and targets from a pre-generated pool (one seeded input set
    per N_side; the N_side 4096 set is the main workload's), held in pinned host
    memory and copied to the device at admission; admission by HBM footprint
    over two streams."""
    from paper_1003_4984_amd.serve import DeviceExecutor, PlanCache, Request, Server, report
    from workload import configs, spectra
    from workload.seeds import rng as seeded
    nsides, weights = (256, 1024, 2048, 4096), np.array([0.4, 0.3, 0.2, 0.1])
    pin = lambda x: x.cpu().pin_memory()
    pool_in = {}
    for ns in nsides:
        if ns == 4096:
            mt, mqu, th, ph = inp_main["T"], inp_main["QU"], inp_main["theta"], inp_main["phi"]
        else:
            m = configs.maps(5, ns, ns, "TQU", "cuda", job=ns)
            mt, mqu = m["T"], torch.cat([m["Q"], m["U"]])
            th, ph = configs.lensing_targets(5, ns, ns, "cuda", job=ns)
        pool_in[ns] = {"T": pin(mt), "QU": pin(mqu), "theta": pin(th), "phi": pin(ph)}
    torch.cuda.synchronize()
    g = seeded(5, 0, 4)
    t, reqs = 0.0, []
    for i in range(n_req):
        t += g.exponential(1.0 / rate)
        ns = int(g.choice(nsides, p=weights / weights.sum()))
        fields = "TQU" if g.uniform() < 0.5 else "T"
        tt, ee, te, bb = spectra.cl_acoustic(ns)
        src = pool_in[ns]
        host = {"T": src["T"], "theta": src["theta"], "phi": src["phi"]}
        if fields == "TQU":
            host["QU"] = src["QU"]
        reqs.append(Request(rid=i, arrival=t, nside=ns, lmax=ns, K=32, fields=fields, n=src["theta"].numel(),
                            cl_tt=tt, cl_ee=ee, cl_bb=bb, host=host))
    plans = PlanCache(lambda nside, lmax, cl, K, spin: fl.Plan(nside, lmax, cl, K, spin))
    plans.warm(reqs)
    ex = DeviceExecutor(plans, slots=2, tqu_shared=True)
    srv = Server(ex, hbm_budget=160 * 2 ** 30, slots=2, plans=plans)
    t0 = time.perf_counter()
    done = srv.run(reqs)
    torch.cuda.synchronize()
    rep = report(done, time.perf_counter() - t0)
    rep.update({"rate_per_s": rate, "K": 32, "nsides": list(nsides), "weights": weights.tolist(),
                "slots": 2, "hbm_budget_gib": 160, "peak_admitted_gib": srv.peak / 2 ** 30,
                "inputs": "pinned host memory, copied to the device at admission"})
    del pool_in
    return rep


def _all_parity_ok(d):
    """False if any parity sample nested in the legs' results broke its tolerance
    or a leg failed; the headline's own gate stays parity_ok."""
    if isinstance(d, dict):
        if "error" in d or d.get("parity_ok") is False:
            return False
        return all(_all_parity_ok(v) for v in d.values())
    return True


def run_legs(fl, torch, inp_main, pool, nw, only=None):
    legs = {}
    for name, fn in (("nside512_fp64_vs_fp32ir", lambda: leg_nside512(fl, torch, pool, nw)),
                     ("supersample_2048_to_4096", lambda: leg_supersample(fl, torch)),
                     ("pixel_stencils", lambda: leg_pixel_stencils(fl, torch, inp_main, pool)),
                     ("large_systems_K48", lambda: leg_large_systems(fl, torch, inp_main, pool)),
                     ("lensing_pipeline", lambda: leg_lensing_pipeline(fl, torch, inp_main, pool)),
                     ("serving_cfg5", lambda: leg_serving(fl, torch, inp_main))):
        if only is not None and name not in only:
            continue
        log(f"leg {name}")
        try:
            legs[name] = fn()
        except Exception as e:           # a failed leg is reported, the headline stands
            legs[name] = {"error": f"{type(e).__name__}: {e}"}
        torch.cuda.synchronize()
        torch.cuda.empty_cache()
    return legs


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="nside4096", choices=sorted(SHAPES))
    ap.add_argument("--precision", default="fp64", choices=["fp64", "fp32ir"])
    ap.add_argument("--cpu-sample", type=int, default=6000)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--tqu", default="shared", choices=["shared", "separate"],
                    help="T and Q/U in one call sharing the stencil search (shared), or one "
                         "call per plan (separate)")
    ap.add_argument("--no-legs", action="store_true",
                    help="skip the extra measurements (N_side 512 FP64 and FP32+IR, supersampling, serving)")
    ap.add_argument("--legs", default=None,
                    help="comma-separated names of the extra measurements to run (default: all)")
    ap.add_argument("--copy-probe-mb", type=int, default=0,
                    help="before timing, copy this many MiB device to device once (a plain copy of "
                         "known size that calibrates HBM traffic counters)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)

    pool = nw = None
    if not args.no_cpu and args.cpu_sample > 0:
        pool, nw = oracle_pool()         # before this process initialises the GPU
    import torch
    import paper_1003_4984_amd as fl
    shape = SHAPES[args.workload]
    dev = "cuda:0"
    torch.cuda.set_device(0)
    inp = make_inputs(shape, dev)
    n = inp["theta"].numel()
    if args.copy_probe_mb > 0:
        src = torch.ones(args.copy_probe_mb << 17, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        log(f"copy probe: {args.copy_probe_mb} MiB read + {args.copy_probe_mb} MiB written")
        del src, dst
    prec = fl.FP64 if args.precision == "fp64" else fl.FP32_IR
    log("building plans")
    p0 = fl.Plan(shape["nside"], shape["lmax"], inp["tt"], shape["K"], 0, precision=prec)
    p2 = fl.Plan(shape["nside"], shape["lmax"], np.concatenate([inp["ee"], inp["bb"]]),
                 shape["K"], 2, precision=prec)
    out_t = torch.empty(n, dtype=torch.float64, device=dev)
    var_t = torch.empty(n, dtype=torch.float64, device=dev)
    out_qu = torch.empty(2 * n, dtype=torch.float64, device=dev)
    var_qu = torch.empty(2 * n, dtype=torch.float64, device=dev)
    stream = torch.cuda.current_stream()

    shared = args.tqu == "shared"
    tqu_mode = args.tqu
    if shared and not fl.tqu_shared(p0, p2):
        tqu_mode = "shared call running as two searching calls (plans not shareable)"

    def step(ev=None):
        if ev:
            ev[0].record(stream)
        if shared:
            fl.interpolate_tqu(p0, p2, inp["T"], inp["QU"], inp["theta"], inp["phi"], out_t=out_t,
                               var_t=var_t, out_qu=out_qu, var_qu=var_qu, stream=stream)
            if ev:
                ev[1].record(stream)
                ev[2].record(stream)
            return
        fl.interpolate(p0, inp["T"], inp["theta"], inp["phi"], out=out_t, var=var_t, stream=stream)
        if ev:
            ev[1].record(stream)
        fl.interpolate(p2, inp["QU"], inp["theta"], inp["phi"], out=out_qu, var=var_qu, stream=stream)
        if ev:
            ev[2].record(stream)

    for i in range(args.warmup):
        log(f"warmup step {i + 1}/{args.warmup}")
        step()
    torch.cuda.synchronize()
    p0.reset_stats()
    p2.reset_stats()
    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        step(evs[i])
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    log(f"timed {args.steps} steps in {wall:.2f} s")
    t_spin0 = np.array([e[0].elapsed_time(e[1]) for e in evs]) * 1e-3
    t_spin2 = np.array([e[1].elapsed_time(e[2]) for e in evs]) * 1e-3
    step_t = t_spin0 + t_spin2
    st0, st2 = p0.stats(), p2.stats()

    K = shape["K"]
    if shared:
        fpp = flops_spin0(K) + flops_spin2(K)
        achieved = fpp * n / t_spin0.mean() / 1e12
        kname = ("T+Q/U call with shared stencils (12 x k_interp_tile_st<4> + 12 x k_interp_rs_ld<2> "
                 "+ two fix-up scans)") if tqu_mode == "shared" else "T+Q/U call (" + tqu_mode + ")"
        kernel_s = {"tqu": float(t_spin0.mean())}
        tunit = "HBM bytes per T+Q/U call (rocprofv3 FETCH_SIZE + WRITE_SIZE, all its kernels)"
    else:
        fpp = flops_spin2(K)
        achieved = fpp * n / t_spin2.mean() / 1e12
        kname = "spin-2 interpolation launch (k_interp_tile<4,2> + fix-up scan)"
        kernel_s = {"spin0": float(t_spin0.mean()), "spin2": float(t_spin2.mean())}
        tunit = "HBM bytes per spin-2 launch (rocprofv3 FETCH_SIZE + WRITE_SIZE)"
    result = {
        "metric": "interpolated T/Q/U samples/sec at Nside=4096 within 2e-4 rel err; p50/p99 latency",
        "value": 3.0 * n * args.steps / wall,
        "unit": "samples/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.precision == "fp64" else "f32+f64",
        "data": "synthetic",
        "config": {"workload": f"lensing remap N_side {shape['nside']} lmax {shape['lmax']} "
                               f"K {K} T+Q+U, one displaced target per pixel",
                   "points": n, "precision": args.precision, "spin2_mode": "full", "tqu": tqu_mode,
                   "nugget": "always (eps = 2^-26)",
                   "plan_precision_run": {"T": "fp64" if p0.info()["precision"] == fl.FP64 else "fp32ir",
                                          "QU": "fp64" if p2.info()["precision"] == fl.FP64 else "fp32ir"},
                   "fp32_probe_reject": {"T": p0.info()["fp32_probe_reject"],
                                         "QU": p2.info()["fp32_probe_reject"]}},
        "points_per_s": n * args.steps / wall,
        "latency_s": {"p50": float(np.percentile(step_t, 50)), "p99": float(np.percentile(step_t, 99)),
                      "note": "per full-sky request (T, Q and U), HIP events"},
        "kernel_s": kernel_s,
        "roofline": {"bound": "alu", "achieved": achieved, "peak": FP64_PEAK_TFLOPS,
                     "unit": "TFLOP/s", "frac": achieved / FP64_PEAK_TFLOPS,
                     "traffic": measured_traffic(args.workload, args.tqu),
                     "traffic_unit": tunit, "kernel": kname, "flops_per_point": fpp},
        "stats": {"spin0": st0, "spin2": st2},
    }
    if not args.no_cpu and args.cpu_sample > 0:
        log(f"oracle on {args.cpu_sample} sampled targets")
        base, parity = cpu_baseline(pool, nw, shape, inp, out_t, var_t, out_qu, var_qu, args.cpu_sample,
                                    shape["cfg"])
        result["cpu_baseline"] = base
        result["parity_sample"] = parity
        result["parity_ok"] = parity["parity_ok"]
    if not args.no_legs and args.workload == "nside4096":
        out_t = var_t = out_qu = var_qu = None      # the legs need the memory
        only = None if args.legs is None else set(args.legs.split(","))
        result["legs"] = run_legs(fl, torch, inp, pool, nw, only)
        result["legs_parity_ok"] = _all_parity_ok(result["legs"])
    if pool is not None:
        pool.close()
        pool.join()
    print(json.dumps(result), flush=True)
    if result.get("parity_ok") is False:
        log("parity sample outside the tolerance: " + json.dumps(result["parity_sample"]))
        sys.exit(3)


if __name__ == "__main__":
    main()
