"""Served stream on the GPU: mixed requests (2D forward, 2D gradient, 3D forward) arriving
while others run are admitted, overlap on the device, and every result equals the same job
run alone."""
import numpy as np
import pytest

from paper_2311_02293_amd import inputs as I
from helpers import dev, say

pytestmark = pytest.mark.gpu


def stream_requests():
    from paper_2311_02293_amd.server import Request
    from oracle import oracle as O  # noqa: F401  (not used: dobs comes from the GPU forward)
    jobs = I.stream_config5(njobs=12, rate=400.0, seed=1005, scale=0.12, nt2d=3000, nt3d=1500,
                            ntgrad=4000)
    reqs = []
    for k, sj in enumerate(jobs):
        j = sj.job
        vs = [j.vp] + ([j.extra["vp_true"]] if "vp_true" in j.extra else [])
        j.grid.vpmin = float(min(v.min() for v in vs))
        j.grid.vpmax = float(1.02 * max(v.max() for v in vs))
        kind = {"forward2d": "forward", "grad2d": "grad", "forward3d": "forward"}[sj.kind]
        reqs.append(Request(kind, j, arrival=sj.arrival, model_key=None))
    return reqs


def test_served_results_equal_alone():
    import torch
    from paper_2311_02293_amd.server import HipBackend, ShotServer
    be = HipBackend(0, nstreams=3)
    reqs = stream_requests()
    # observed data for the gradient requests: forward of the true model, run alone
    for r in reqs:
        if r.kind == "grad":
            vp, rho, stf = dev(r.job)
            vt = torch.from_numpy(r.job.extra["vp_true"]).cuda()
            d, _, _ = be.ctx.forward(r.job.grid, r.job.acq, vt, rho, stf)
            r.dobs = d.cpu().numpy()
    srv = ShotServer(be, max_inflight=3)
    out = srv.run(reqs)
    say("served:", len(reqs), "requests, p50", out["p50"], "p99", out["p99"],
        "GPts/s", out["gpts_per_s"], "failed", out["failed"])
    assert out["failed"] == 0
    for r, o in zip(reqs, out["outcomes"]):
        vp, rho, stf = dev(r.job)
        if r.kind == "forward":
            alone, _, _ = be.ctx.forward(r.job.grid, r.job.acq, vp, rho, stf)
            np.testing.assert_array_equal(o.result, alone.cpu().numpy())
        else:
            d = torch.from_numpy(r.dobs).cuda()
            g, J, _ = be.ctx.fwi_grad(r.job.grid, r.job.acq, vp, rho, stf, d)
            np.testing.assert_array_equal(o.result[0], g.cpu().numpy())
            np.testing.assert_array_equal(o.result[1], J.cpu().numpy())


def test_batched_requests_equal_alone():
    """Requests that share grid and model are merged into one multi-shot call."""
    from paper_2311_02293_amd.server import HipBackend, Request, ShotServer
    be = HipBackend(0, nstreams=2)
    base = I.config2(n1=60, n2=180, nt=400, nshot=4)
    base.grid.vpmin = float(base.vp.min())
    base.grid.vpmax = float(base.vp.max())
    reqs = []
    for s in range(4):
        j = I.Job(base.grid, base.vp, base.rho, base.acq.shot(s), base.stf[s:s + 1], name=f"s{s}")
        reqs.append(Request("forward", j, arrival=0.0, model_key="layers"))
    out = ShotServer(be, max_inflight=1).run(reqs)
    assert [o.batch for o in out["outcomes"]] == [4, 4, 4, 4]
    for r, o in zip(reqs, out["outcomes"]):
        vp, rho, stf = dev(r.job)
        alone, _, _ = be.ctx.forward(r.job.grid, r.job.acq, vp, rho, stf)
        k, res = o.result
        n = r.job.grid.nt * r.job.acq.nrec(0)
        np.testing.assert_array_equal(res[k * n:(k + 1) * n], alone.cpu().numpy())
