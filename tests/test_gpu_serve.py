"""Serving on the device: requests of several N_side arriving faster than they
are served overlap on two streams in batched launches (T+Q+U requests through
the shared-stencil call, or as two batch jobs), with their inputs copied from
host memory at admission; the device intervals of groups on the two streams
overlap; every result must equal the same request computed alone (bit for
bit), and p50/p99 are reported."""
import pytest
import torch

import paper_1003_4984_amd as fl
from paper_1003_4984_amd.serve import DeviceExecutor, PlanCache, Server, make_requests, report

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("tqu_shared", [True, False])
def test_served_results_equal_alone(gpu_ok, tqu_shared):
    # N_side 256 and 512 requests (5 to 80 ms of device work each) arriving
    # within a few ms: the first runs alone, the next are admitted on the other
    # stream while it is still on the device
    reqs = make_requests(6, rate=2000.0, seed=1, nsides=(256, 512), weights=(0.5, 0.5),
                         tqu_frac=0.5, K=32, device="cuda")
    torch.cuda.synchronize()
    plans = PlanCache(lambda nside, lmax, cl, K, spin: fl.Plan(nside, lmax, cl, K, spin))
    plans.warm(reqs)
    ex = DeviceExecutor(plans, slots=2, tqu_shared=tqu_shared, keep_inputs=True)
    srv = Server(ex, hbm_budget=8 * 2 ** 30, slots=2, plans=plans, tqu_shared=tqu_shared)
    done = srv.run(reqs)
    torch.cuda.synchronize()
    assert len(done) == len(reqs)
    assert all(r.host for r in reqs)              # inputs reached the device at admission
    # groups on the two streams were on the device at the same time
    iv = ex.device_intervals()
    assert len(iv) >= 2
    assert any(a0 < b1 and b0 < a1 for i, (a0, a1, _) in enumerate(iv) for (b0, b1, _) in iv[i + 1:])
    assert any(len(g) > 1 for g in [[r for r in done if r.admitted == a] for a in {r.admitted for r in done}])
    rep = report(done, max(r.finished for r in done))
    assert rep["latency_p50_s"] is not None and rep["latency_p99_s"] >= rep["latency_p50_s"]
    for r in done:
        p0 = plans.get(r.nside, r.lmax, r.K, 0, r.cl_tt)
        o, v = fl.interpolate(p0, r.maps["T"], r.theta, r.phi)
        torch.cuda.synchronize()
        assert torch.equal(o, r.out["T"][0]) and torch.equal(v, r.out["T"][1]), r.rid
        if r.fields == "TQU":
            import numpy as np
            p2 = plans.get(r.nside, r.lmax, r.K, 2, np.concatenate([r.cl_ee, r.cl_bb]))
            o, v = fl.interpolate(p2, r.maps["QU"], r.theta, r.phi)
            torch.cuda.synchronize()
            assert torch.equal(o, r.out["QU"][0]) and torch.equal(v, r.out["QU"][1]), r.rid
