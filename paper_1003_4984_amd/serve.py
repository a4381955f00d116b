"""Serving loop: continuous batching of lensing interpolation requests.

Requests (a map set -- T, or T with Q/U -- plus displaced target directions)
arrive over time with their inputs in host memory.  The server keeps plans, and
with them the device-resident correlation tables, in a cache keyed by (N_side,
lmax, K, spin, spectrum) that is filled before serving starts (the tables of
the served configurations are built once, like the paper's initialisation
step); admits waiting requests first-come first-served while the HBM they need
(maps, targets, outputs, variances, the stencil buffer of a T+Q+U call and any
new plan's table) fits a budget and a launch slot is free; copies the admitted
requests' inputs to the device on the slot's stream and groups them into one
batched launch (flints_batch_*) on that stream, so the work of different
requests overlaps on the device -- except that a T+Q+U request runs through
flints_interpolate_tqu on that stream (one K-nearest search per target serves
both its plans); and releases a request's device memory when its completion
event has fired.  Batch descriptors are destroyed only while no launch is in
flight (freeing device memory waits for the whole device).  Latency is
completion minus arrival; the report gives p50 and p99 next to throughput in
samples per second.

The scheduling logic is independent of the device: `Server` drives an
executor with `launch(requests, slot) -> token` and `done(token) -> bool`;
`DeviceExecutor` is the FLINTS one.  Batching is an addition to the method; the
paper interpolates one map at a time.
"""
import argparse
import hashlib
import json
import time
from collections import deque
from dataclasses import dataclass, field

import numpy as np

BYTES_PER_SAMPLE = 16          # one double of output and one of variance
TABLE_BYTES_BOUND = 256 * 1024  # plan table upper bound used for admission
TQU_CHUNK = 1 << 24            # targets per stencil-buffer chunk of flints_interpolate_tqu
BATCH_BYTES_BOUND = 1 << 20     # device job table, tile lists and queue counters of one batch


@dataclass
class Request:
    rid: int
    arrival: float               # seconds on the server clock
    nside: int
    lmax: int
    K: int
    fields: str                  # "T" or "TQU"
    n: int                       # targets
    cl_tt: object = None
    cl_ee: object = None
    cl_bb: object = None
    maps: dict = field(default_factory=dict)   # "T": tensor, "QU": tensor (device, from admission)
    theta: object = None
    phi: object = None
    host: dict = field(default_factory=dict)   # inputs in host memory: "T", "QU", "theta", "phi"
    out: dict = field(default_factory=dict)    # filled at admission: field set -> (out, var)
    admitted: float = None
    finished: float = None

    @property
    def samples(self):
        return self.n * len(self.fields)

    def footprint(self, new_tables=0, tqu_shared=True):
        """HBM a request holds while admitted: its maps (f fields of 12 N_side^2
        doubles), its target directions (16 B each), outputs and variances
        (16 B per sample), the stencil buffer of a T+Q+U call (K int32 per
        target of one 2^24-target chunk), a batch descriptor, and the tables of
        plans not yet cached."""
        f = len(self.fields)
        stencils = 4 * self.K * min(self.n, TQU_CHUNK) if (self.fields == "TQU" and tqu_shared) else 0
        return (8 * 12 * self.nside * self.nside * f + 16 * self.n + self.samples * BYTES_PER_SAMPLE
                + stencils + BATCH_BYTES_BOUND + new_tables * TABLE_BYTES_BOUND)


class PlanCache:
    """Plans (and their device tables) kept across requests."""

    def __init__(self, make_plan):
        self._make = make_plan
        self._plans = {}

    @staticmethod
    def key(nside, lmax, K, spin, cl):
        h = hashlib.sha1(np.ascontiguousarray(cl, dtype=np.float64).tobytes()).hexdigest()
        return (int(nside), int(lmax), int(K), int(spin), h)

    def missing(self, req):
        keys = [self.key(req.nside, req.lmax, req.K, 0, req.cl_tt)]
        if req.fields == "TQU":
            keys.append(self.key(req.nside, req.lmax, req.K, 2, np.concatenate([req.cl_ee, req.cl_bb])))
        return sum(k not in self._plans for k in keys)

    def get(self, nside, lmax, K, spin, cl):
        k = self.key(nside, lmax, K, spin, cl)
        if k not in self._plans:
            self._plans[k] = self._make(nside, lmax, cl, K, spin)
        return self._plans[k]

    def warm(self, requests):
        """Build the plans (tables) every request needs, before serving."""
        for r in requests:
            self.get(r.nside, r.lmax, r.K, 0, r.cl_tt)
            if r.fields == "TQU":
                self.get(r.nside, r.lmax, r.K, 2, np.concatenate([r.cl_ee, r.cl_bb]))

    def __len__(self):
        return len(self._plans)


class Server:
    """Admission by HBM footprint, FIFO, continuous batching over `slots` streams."""

    def __init__(self, executor, hbm_budget, slots=2, plans=None, clock=time.perf_counter,
                 max_group_samples=1 << 26, sleep=time.sleep, tqu_shared=True):
        self.ex = executor
        self.sleep = sleep
        self.tqu_shared = tqu_shared
        self.budget = int(hbm_budget)
        self.max_group = int(max_group_samples)   # caps one launch so groups finish in turn
        self.slots = int(slots)
        self.plans = plans
        self.clock = clock
        self.in_use = 0
        self.peak = 0

    def run(self, requests, idle=None):
        """Serve `requests` (sorted by arrival, times relative to the start).
        Returns the list of finished requests."""
        t0 = self.clock()
        pending = deque(sorted(requests, key=lambda r: r.arrival))
        waiting = deque()
        running = {}          # slot -> (token, [requests], bytes)
        free = list(range(self.slots))
        done = []
        while pending or waiting or running:
            now = self.clock() - t0
            progress = False
            while pending and pending[0].arrival <= now:
                waiting.append(pending.popleft())
                progress = True
            # completions
            for slot in list(running):
                token, reqs, nbytes = running[slot]
                if self.ex.done(token):
                    t = self.clock() - t0
                    for r in reqs:
                        r.finished = t
                        done.append(r)
                    self.in_use -= nbytes
                    del running[slot]
                    free.append(slot)
                    progress = True
            if not running and hasattr(self.ex, "quiesce"):
                self.ex.quiesce()              # nothing in flight: release retired launches
            # admission: first come first served while memory and a slot allow
            if free and waiting:
                group, nbytes, nsamp = [], 0, 0
                while waiting:
                    r = waiting[0]
                    if group and nsamp + r.samples > self.max_group:
                        break
                    need = r.footprint(self.plans.missing(r) if self.plans is not None else 0,
                                       self.tqu_shared)
                    if need > self.budget:
                        raise ValueError(f"request {r.rid} needs {need} B, more than the budget")
                    if self.in_use + nbytes + need > self.budget:
                        break
                    group.append(waiting.popleft())
                    nbytes += need
                    nsamp += r.samples
                if group:
                    slot = free.pop(0)
                    t = self.clock() - t0
                    for r in group:
                        r.admitted = t
                    token = self.ex.launch(group, slot)
                    running[slot] = (token, group, nbytes)
                    self.in_use += nbytes
                    self.peak = max(self.peak, self.in_use)
                    continue
            if idle is not None:
                idle()
            elif not progress:
                # nothing to do until the next arrival or a completion: yield
                # the host thread instead of spinning
                wait = pending[0].arrival - (self.clock() - t0) if pending else 1e-3
                self.sleep(min(max(wait, 0.0), 2e-4 if running else 1e-3))
        return done


def report(done, wall):
    lat = np.array([r.finished - r.arrival for r in done])
    samples = sum(r.samples for r in done)
    return {"requests": len(done), "samples": int(samples), "wall_s": wall,
            "samples_per_s": samples / wall if wall > 0 else None,
            "latency_p50_s": float(np.percentile(lat, 50)) if len(lat) else None,
            "latency_p99_s": float(np.percentile(lat, 99)) if len(lat) else None}


class DeviceExecutor:
    """FLINTS executor: one flints batch per admitted group, on `slots` streams
    of default priority; the group's inputs are copied from host memory on the
    slot's stream first; completion via a recorded event.  With `tqu_shared`,
    T+Q+U requests run through interpolate_tqu (shared stencil search) on the
    group's stream instead of as two batch jobs.  `keep_inputs` keeps the
    requests' device inputs after completion (for checking results)."""

    def __init__(self, plans, slots, tqu_shared=True, keep_inputs=False):
        import torch
        import paper_1003_4984_amd as fl
        self.fl, self.torch = fl, torch
        self.plans = plans
        self.streams = [torch.cuda.Stream() for _ in range(slots)]
        self.tqu_shared = tqu_shared
        self.keep_inputs = keep_inputs
        self.retired = []             # batches to destroy once nothing is in flight
        self.t_ref = torch.cuda.Event(enable_timing=True)
        self.t_ref.record()
        self.intervals = []           # (start event, end event, request ids) per group

    def jobs_for(self, r):
        torch, fl = self.torch, self.fl
        jobs = []
        p0 = self.plans.get(r.nside, r.lmax, r.K, 0, r.cl_tt)
        o = torch.empty(r.n, dtype=torch.float64, device=r.theta.device)
        v = torch.empty(r.n, dtype=torch.float64, device=r.theta.device)
        r.out["T"] = (o, v)
        jobs.append((p0, r.maps["T"], r.theta, r.phi, o, v))
        if r.fields == "TQU":
            p2 = self.plans.get(r.nside, r.lmax, r.K, 2, np.concatenate([r.cl_ee, r.cl_bb]))
            o2 = torch.empty(2 * r.n, dtype=torch.float64, device=r.theta.device)
            v2 = torch.empty(2 * r.n, dtype=torch.float64, device=r.theta.device)
            r.out["QU"] = (o2, v2)
            jobs.append((p2, r.maps["QU"], r.theta, r.phi, o2, v2))
        return jobs

    def run_tqu(self, r, s):
        fl = self.fl
        p0 = self.plans.get(r.nside, r.lmax, r.K, 0, r.cl_tt)
        p2 = self.plans.get(r.nside, r.lmax, r.K, 2, np.concatenate([r.cl_ee, r.cl_bb]))
        o, v, o2, v2 = fl.interpolate_tqu(p0, p2, r.maps["T"], r.maps["QU"], r.theta, r.phi, stream=s)
        r.out["T"] = (o, v)
        r.out["QU"] = (o2, v2)

    def stage_inputs(self, r):
        """Copy a request's host inputs to the device (on the current stream)."""
        dev = "cuda"
        if r.host:
            r.maps = {k: r.host[k].to(dev, non_blocking=True) for k in ("T", "QU") if k in r.host}
            r.theta = r.host["theta"].to(dev, non_blocking=True)
            r.phi = r.host["phi"].to(dev, non_blocking=True)

    def launch(self, group, slot):
        torch = self.torch
        s = self.streams[slot]
        # device inputs produced on the default stream (if any) come first
        s.wait_stream(torch.cuda.current_stream())
        start = torch.cuda.Event(enable_timing=True)
        with torch.cuda.stream(s):
            start.record(s)
            for r in group:
                self.stage_inputs(r)
            shared = [r for r in group if self.tqu_shared and r.fields == "TQU"]
            ids = {id(r) for r in shared}
            jobs = [j for r in group if id(r) not in ids for j in self.jobs_for(r)]
            b = None
            if jobs:
                b = self.fl.Batch(jobs)
                b.run(s)
            for r in shared:
                self.run_tqu(r, s)
        ev = torch.cuda.Event(enable_timing=True)
        ev.record(s)
        self.intervals.append((start, ev, [r.rid for r in group]))
        return (ev, b, group)

    def done(self, token):
        ev, b, group = token
        if not ev.query():
            return False
        if b is not None:
            self.retired.append(b)
        if not self.keep_inputs:
            for r in group:
                r.maps, r.theta, r.phi = {}, None, None
        return True

    def quiesce(self):
        """Destroy retired batches (called when no launch is in flight)."""
        while self.retired:
            self.retired.pop().close()

    def device_intervals(self):
        """(start s, end s, request ids) of every launched group on the device
        clock (relative to the executor's creation); call after synchronising."""
        return [(self.t_ref.elapsed_time(a) * 1e-3, self.t_ref.elapsed_time(b) * 1e-3, ids)
                for a, b, ids in self.intervals]


def make_requests(n_req, rate, seed=0, nsides=(256, 1024, 2048, 4096), weights=(0.4, 0.3, 0.2, 0.1),
                  tqu_frac=0.5, K=32, device="cuda", max_points=None, host_inputs=True):
    """Poisson stream of lensing requests (rate per second) with fresh seeded
    maps and deflections, lmax = N_side; inputs are synthesised (on `device`)
    before the clock starts and, with host_inputs, moved to pinned host memory
    so that they reach the device only when the request is admitted."""
    import torch
    from workload import configs, spectra
    from workload.seeds import rng as seeded
    g = seeded(5, seed, 0)
    t, reqs = 0.0, []
    p = np.asarray(weights, dtype=np.float64)
    for i in range(n_req):
        t += g.exponential(1.0 / rate)
        nside = int(g.choice(nsides, p=p / p.sum()))
        lmax = nside
        fields = "TQU" if g.uniform() < tqu_frac else "T"
        tt, ee, te, bb = spectra.cl_acoustic(lmax)
        job = seed * 100000 + i
        m = configs.maps(5, nside, lmax, fields, device, job=job)
        maps = {"T": m["T"]}
        if fields == "TQU":
            maps["QU"] = torch.cat([m["Q"], m["U"]])
        del m
        th, ph = configs.lensing_targets(5, nside, lmax, device, job=job)
        if max_points is not None and th.numel() > max_points:
            th, ph = th[:max_points].contiguous(), ph[:max_points].contiguous()
        r = Request(rid=i, arrival=t, nside=nside, lmax=lmax, K=K, fields=fields, n=th.numel(),
                    cl_tt=tt, cl_ee=ee, cl_bb=bb)
        if host_inputs:
            pin = lambda x: x.cpu().pin_memory()
            r.host = {k: pin(v) for k, v in maps.items()}
            r.host["theta"], r.host["phi"] = pin(th), pin(ph)
            del maps, th, ph
        else:
            r.maps, r.theta, r.phi = maps, th, ph
        reqs.append(r)
    return reqs


def main():
    ap = argparse.ArgumentParser(description="FLINTS serving simulation (Poisson request stream)")
    ap.add_argument("--requests", type=int, default=24)
    ap.add_argument("--rate", type=float, default=20.0, help="requests per second")
    ap.add_argument("--slots", type=int, default=2)
    ap.add_argument("--budget-gb", type=float, default=64.0)
    ap.add_argument("--group-msamples", type=float, default=64.0, help="samples per launch cap (millions)")
    ap.add_argument("--nsides", default="256,1024,2048")
    ap.add_argument("--weights", default="0.4,0.3,0.2")
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--no-tqu-shared", action="store_true",
                    help="run T+Q+U requests as two batch jobs instead of interpolate_tqu")
    args = ap.parse_args()
    import torch
    import paper_1003_4984_amd as fl
    nsides = tuple(int(x) for x in args.nsides.split(","))
    weights = tuple(float(x) for x in args.weights.split(","))
    reqs = make_requests(args.requests, args.rate, args.seed, nsides, weights)
    torch.cuda.synchronize()
    plans = PlanCache(lambda nside, lmax, cl, K, spin: fl.Plan(nside, lmax, cl, K, spin))
    plans.warm(reqs)
    ex = DeviceExecutor(plans, args.slots, tqu_shared=not args.no_tqu_shared)
    srv = Server(ex, args.budget_gb * 2 ** 30, args.slots, plans,
                 max_group_samples=int(args.group_msamples * 1e6), tqu_shared=not args.no_tqu_shared)
    t0 = time.perf_counter()
    done = srv.run(reqs)
    torch.cuda.synchronize()
    rep = report(done, time.perf_counter() - t0)
    rep.update({"rate_per_s": args.rate, "slots": args.slots, "plans_cached": len(plans),
                "group_msamples": args.group_msamples, "tqu_shared": not args.no_tqu_shared,
                "peak_admitted_bytes": srv.peak, "nsides": list(nsides), "K": 32})
    print(json.dumps(rep), flush=True)


if __name__ == "__main__":
    main()
