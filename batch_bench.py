"""Batched uneven workload: 64 interpolation jobs in persistent fused launches.

Jobs follow the batched configuration of the workload module (N_side in
{128 .. 2048}, spin 0 or 2, K in {16, 24, 32, 48}, target counts log-uniform in
[1e4, 5e7] times --scale, uniform random directions); spin-2 jobs with K = 48
(96-row systems) run the LDS elimination through the single-plan path inside
the batch.  One map per
(N_side, spin) is shared by the jobs that use it.  Reports samples/s for the
jobs run one after another through flints_interpolate, for one batched run, for
graph replays and for an autotuned batch, and checks that all four agree bit
for bit.  Prints one JSON line.
"""
import argparse
import json
import sys
import time

import numpy as np


def log(msg):
    print(f"[batch_bench {time.strftime('%H:%M:%S')}] {msg}", file=sys.stderr, flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--scale", type=float, default=0.25, help="scale of the target counts")
    ap.add_argument("--jobs", type=int, default=64)
    ap.add_argument("--reps", type=int, default=2)
    ap.add_argument("--precision", default="fp64", choices=["fp64", "fp32ir"],
                    help="plan precision; FP32+IR plans whose creation probe keeps FP32 run outside "
                         "the persistent launches")
    args = ap.parse_args()
    import torch
    import paper_1003_4984_amd as fl
    from workload import configs, spectra, synth
    from workload.seeds import rng as seeded

    t_setup = time.perf_counter()
    specs = configs.batch_jobs(args.jobs, args.scale)
    maps, plans, jobs = {}, {}, []
    for sp in specs:
        nside, spin, K, lmax = sp["nside"], sp["spin"], sp["K"], sp["lmax"]
        tt, ee, te, bb = spectra.cl_acoustic(lmax)
        if (nside, spin) not in maps:
            r = seeded(4, nside, spin)
            if spin == 0:
                maps[(nside, spin)] = synth.synth(synth.draw_alm(r, tt, lmax), 0, nside, "cuda")
            else:
                q, u = synth.synth(-synth.draw_alm(r, ee, lmax), 2, nside, "cuda")
                maps[(nside, spin)] = torch.cat([q, u])
        key = (nside, lmax, K, spin)
        if key not in plans:
            cl = tt if spin == 0 else np.concatenate([ee, bb])
            plans[key] = fl.Plan(nside, lmax, cl, K, spin,
                                 precision=fl.FP64 if args.precision == "fp64" else fl.FP32_IR)
        th, ph = configs.uniform_targets(4, sp["job"], sp["n"], "cuda")
        nf = 1 if spin == 0 else 2
        out = torch.empty(nf * sp["n"], dtype=torch.float64, device="cuda")
        var = torch.empty_like(out)
        jobs.append((plans[key], maps[(nside, spin)], th, ph, out, var))
    torch.cuda.synchronize()
    t_setup = time.perf_counter() - t_setup
    samples = sum(j[4].numel() for j in jobs)
    points = sum(j[2].numel() for j in jobs)

    log(f"set up {len(jobs)} jobs, {points} targets in {t_setup:.1f} s")

    def timed(fn, name):
        best = 1e30
        for r in range(args.reps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            fn()
            torch.cuda.synchronize()
            best = min(best, time.perf_counter() - t0)
            log(f"{name} run {r + 1}/{args.reps}: {time.perf_counter() - t0:.2f} s")
        return best

    def sequential():
        for p, m, th, ph, out, var in jobs:
            fl.interpolate(p, m, th, ph, out=out, var=var)

    t_seq = timed(sequential, "per-job launches")
    ref = [(j[4].clone(), j[5].clone()) for j in jobs]

    def same():
        return all(torch.equal(j[4], r[0]) and torch.equal(j[5], r[1]) for j, r in zip(jobs, ref))

    b = fl.Batch(jobs)
    t_batch = timed(b.run, "batch")
    ok_batch = same()
    s = torch.cuda.Stream()
    b.capture(s)

    def replay():
        b.run(s)
        s.synchronize()

    t_graph = timed(replay, "graph replay")
    ok_graph = same()
    info_plain = b.info()
    b.close()
    log("autotuning")
    t0 = time.perf_counter()
    bt = fl.Batch(jobs, autotune=True)
    t_tune = time.perf_counter() - t0
    log(f"autotuned in {t_tune:.1f} s")
    t_auto = timed(bt.run, "autotuned batch")
    ok_auto = same()
    info_auto = bt.info()
    bt.close()
    res = {
        "metric": "batched uneven workload samples/s", "unit": "samples/s", "jobs": len(jobs),
        "points": int(points), "samples": int(samples), "scale": args.scale,
        "sequential_samples_per_s": samples / t_seq, "batch_samples_per_s": samples / t_batch,
        "graph_samples_per_s": samples / t_graph, "autotuned_samples_per_s": samples / t_auto,
        "autotune_s": t_tune, "setup_s": t_setup, "precision": args.precision,
        "plans_running_fp32": sum(1 for p in plans.values() if p.info()["precision"] == fl.FP32_IR),
        "plans": len(plans),
        "bit_identical": {"batch": ok_batch, "graph": ok_graph, "autotuned": ok_auto},
        "batch_info": info_plain, "autotuned_info": info_auto,
    }
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
