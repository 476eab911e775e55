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
        np.testing.assert_array_equal(o.result, alone.cpu().numpy())


@pytest.mark.parametrize("kind", ["grad", "rtm"])
def test_merged_gradient_and_image_requests_equal_alone(kind):
    """Gradient and RTM requests on one model, queued together, run as one multi-shot call
    with one shot group per request; each gets its own gradient and misfit (or image and
    illumination), bitwise equal to the request run alone.  Off-grid receivers with
    overlapping operators, requests of one and of two shots."""
    import torch
    from paper_2311_02293_amd.server import HipBackend, Request, ShotServer
    be = HipBackend(0, nstreams=2)
    base = I.config3(n1=60, n2=150, nt=400, nshot=5)
    base.grid.vpmin = float(min(base.vp.min(), base.extra["vp_true"].min()))
    base.grid.vpmax = float(max(base.vp.max(), base.extra["vp_true"].max()))
    xmax = (base.grid.n2 - 1) * base.grid.d2
    base.acq.rec[:, 1] = np.minimum(base.acq.rec[:, 1] + 3.3, xmax)   # off the grid
    base.acq.src[:, 1] += 1.7
    _, rho, stf = dev(base)
    vt = torch.from_numpy(base.extra["vp_true"]).cuda()
    parts = [[0], [1, 2], [3], [4]]
    reqs = []
    for k, shots in enumerate(parts):
        j = I.Job(base.grid, base.vp, base.rho, base.acq.subset(shots), base.stf[shots],
                  name=f"r{k}")
        d, _, _ = be.ctx.forward(j.grid, j.acq, vt, rho, torch.from_numpy(j.stf).cuda())
        reqs.append(Request(kind, j, arrival=0.0, dobs=d.cpu().numpy(), model_key="survey"))
    out = ShotServer(be, max_inflight=1).run(reqs)
    say(kind, "requests per call", [o.batch for o in out["outcomes"]], "calls", out["calls"])
    assert out["failed"] == 0 and out["merged_calls"] >= 1
    assert max(o.batch for o in out["outcomes"]) == len(parts)
    for r, o in zip(reqs, out["outcomes"]):
        vp, rho_r, stf_r = dev(r.job)
        d = torch.from_numpy(r.dobs).cuda()
        if kind == "grad":
            g, J, _ = be.ctx.fwi_grad(r.job.grid, r.job.acq, vp, rho_r, stf_r, d)
            np.testing.assert_array_equal(o.result[0], g.cpu().numpy())
            np.testing.assert_array_equal(o.result[1], J.cpu().numpy())
        else:
            img, il = be.ctx.rtm_image(r.job.grid, r.job.acq, vp, rho_r, stf_r, d)
            np.testing.assert_array_equal(o.result[0], img.cpu().numpy())
            np.testing.assert_array_equal(o.result[1], il.cpu().numpy())


def test_pooled_stream_merges_and_equals_alone():
    """A stream of single-shot requests over a few surveys (models resident in the cache):
    requests queued behind busy slots merge per survey, and every result equals the request
    run alone."""
    import torch
    from paper_2311_02293_amd.server import HipBackend, Request, ShotServer
    jobs = I.stream_config5(njobs=24, rate=2000.0, seed=1005, scale=0.12, pool=2)
    be = HipBackend(0, nstreams=2)
    reqs = []
    for sj in jobs:
        j = sj.job
        vs = [j.vp] + ([j.extra["vp_true"]] if "vp_true" in j.extra else [])
        j.grid.vpmin = float(min(v.min() for v in vs))
        j.grid.vpmax = float(1.02 * max(v.max() for v in vs))
        kind = "grad" if sj.kind == "grad2d" else "forward"
        r = Request(kind, j, arrival=sj.arrival, model_key=sj.model_key)
        if kind == "grad":
            _, rho, stf = dev(j)
            d, _, _ = be.ctx.forward(j.grid, j.acq, torch.from_numpy(j.extra["vp_true"]).cuda(),
                                     rho, stf)
            r.dobs = d.cpu().numpy()
        reqs.append(r)
    out = ShotServer(be, max_inflight=2).run(reqs)
    say("pooled stream: calls", out["calls"], "merged", out["merged_calls"], "requests per call",
        out["requests_per_call"], "cache hits", be.models.hits, "misses", be.models.misses,
        "alg GB/s", out["alg_GBps"])
    assert out["failed"] == 0 and out["merged_calls"] >= 1
    assert be.models.hits >= 1
    for r, o in zip(reqs, out["outcomes"]):
        vp, rho, stf = dev(r.job)
        if r.kind == "forward":
            alone, _, _ = be.ctx.forward(r.job.grid, r.job.acq, vp, rho, stf)
            np.testing.assert_array_equal(o.result, alone.cpu().numpy())
        else:
            g, J, _ = be.ctx.fwi_grad(r.job.grid, r.job.acq, vp, rho, stf,
                                      torch.from_numpy(r.dobs).cuda())
            np.testing.assert_array_equal(o.result[0], g.cpu().numpy())
            np.testing.assert_array_equal(o.result[1], J.cpu().numpy())
