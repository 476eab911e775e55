"""GPU: 2D forward passes run in shot groups (SMI_OPT_FWD_GROUP) give bitwise the results of one
time loop over all shots -- seismograms (receivers sampled inside the v launches, off-grid
operators, free surface), snapshots, and the gradients of jobs whose forward pass saves bands
(every level, and decimated with the final state kept aside) -- as eager launches and as a
replayed graph, with timing samples taken; and the automatic grouping of a forward batch whose
fields exceed the last-level cache agrees with the oracle."""
import numpy as np
import pytest

from paper_2311_02293_amd import inputs as I
from helpers import dev, rel_l2, say, with_bounds

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    from paper_2311_02293_amd import binding as B
    return B.Context(0)


def _with(ctx, opts, fn):
    from paper_2311_02293_amd import binding as B
    for k, v in opts.items():
        ctx.set_option(k, v)
    try:
        return fn()
    finally:
        for k in opts:
            ctx.set_option(k, 0)
        ctx.set_option(B.OPT_FWD_GROUP, 0)


def _equal(name, got, ref):
    for k, (a, b) in enumerate(zip(got, ref)):
        same = np.array_equal(a, b)
        say(f"{name} output {k}: bitwise {same}, rel L2 {rel_l2(a, b):.2e}")
        assert same


def _offgrid(job):
    xmax = (job.grid.n2 - 1) * job.grid.d2
    job.acq.rec[:, 1] = np.minimum(job.acq.rec[:, 1] + 3.3, xmax)
    job.acq.rec[:, 0] += 0.37 * job.grid.d1
    job.acq.src[:, 1] += 1.7
    job.acq.src[:, 0] += 0.45 * job.grid.d1
    return job


@pytest.mark.parametrize("freesurf", [0, 1])
@pytest.mark.parametrize("per", [1, 2])
def test_grouped_forward_equals_one_loop(ctx, freesurf, per):
    """Seismograms and snapshots of a 5-shot forward pass with at most `per` shots per time
    loop, against one loop over the 5 shots."""
    from paper_2311_02293_amd import binding as B
    job = I.config2(n1=96, n2=260, nt=500, nshot=5)
    job.grid.freesurf = freesurf
    job = with_bounds(_offgrid(job))
    vp, rho, stf = dev(job)
    levels = [0, 120, 333, job.grid.nt]

    def run(k):
        def go():
            d, snaps, _ = ctx.forward(job.grid, job.acq, vp, rho, stf, snaps=levels)
            return [d.cpu().numpy(), snaps.cpu().numpy()]
        return _with(ctx, {B.OPT_FWD_GROUP: k}, go)
    ref = run(job.acq.nshot)
    got = run(per)
    ctx.poll_status()
    _equal(f"forward freesurf {freesurf} groups of {per}", got, ref)


@pytest.mark.parametrize("dr", [1, 3])
def test_grouped_forward_of_a_gradient_equals_one_loop(ctx, dr):
    """A gradient whose forward pass saves bands (dr 1: every level on the half steps; dr 3: the
    run past nt with level nt kept aside and restored, and the last saved level) with forward
    groups of 2 and reverse groups of 3, against one loop each way."""
    import torch
    from paper_2311_02293_amd import binding as B
    job = I.config3(n1=70, n2=160, nt=420, nshot=5)
    job.grid.dr = dr
    job = with_bounds(job, [job.extra["vp_true"]])
    vp, rho, stf = dev(job)
    d, _, _ = ctx.forward(job.grid, job.acq, torch.from_numpy(job.extra["vp_true"]).cuda(), rho, stf)

    def run(kf, kr):
        return _with(ctx, {B.OPT_FWD_GROUP: kf, B.OPT_REV_GROUP: kr}, lambda: [
            t.cpu().numpy() for t in ctx.fwi_grad(job.grid, job.acq, vp, rho, stf, d,
                                                  want_dcal=True)])
    ref = run(job.acq.nshot, job.acq.nshot)
    got = run(2, 3)
    _equal(f"gradient dr {dr}", got, ref)


def test_grouped_forward_graph_and_timing(ctx):
    """Forward groups replayed as a HIP graph (three replays with eager work between) equal the
    eager result; with event timing on, every sampled step of every group is timed."""
    import torch
    from paper_2311_02293_amd import binding as B
    job = with_bounds(_offgrid(I.config2(n1=96, n2=260, nt=400, nshot=4)))
    vp, rho, stf = dev(job)

    def call():
        return [ctx.forward(job.grid, job.acq, vp, rho, stf)[0].cpu().numpy()]
    ref = _with(ctx, {B.OPT_FWD_GROUP: 2}, call)
    for rep in range(3):
        got = _with(ctx, {B.OPT_FWD_GROUP: 2, B.OPT_GRAPH: 1}, call)
        torch.cuda.synchronize()
        _equal(f"graph replay {rep}", got, ref)

    def timed():
        ctx.set_option(B.OPT_TIMING, 20)
        out = call()
        torch.cuda.synchronize()
        return out, ctx.kernel_timing(1), ctx.kernel_timing(2)
    out, tv, tp = _with(ctx, {B.OPT_FWD_GROUP: 2}, timed)
    ctx.set_option(B.OPT_TIMING, 0)
    _equal("timed", out, ref)
    say("timing samples", tv, tp)
    assert tv[2] == 2 * (job.grid.nt // 20) and tp[2] == tv[2]
    assert tv[0] > 0 and tv[1] > 0 and tp[0] > 0 and tp[1] > 0


def test_automatic_forward_groups_match_the_oracle(ctx):
    """32 shots of the 500 x 1500 benchmark grid with the computing box off (11.8 MB of fields
    per shot, 378 MB in all) run in automatic forward groups; the seismograms equal one loop's
    bitwise, and one shot's agrees with the oracle."""
    import torch
    from oracle import oracle as O
    from paper_2311_02293_amd import binding as B
    job = with_bounds(I.config2(nt=300, nshot=32, box=0))
    vp, rho, stf = dev(job)
    auto = ctx.forward(job.grid, job.acq, vp, rho, stf)[0].cpu().numpy()
    one = _with(ctx, {B.OPT_FWD_GROUP: job.acq.nshot}, lambda: ctx.forward(
        job.grid, job.acq, vp, rho, stf)[0].cpu().numpy())
    _equal("automatic groups", [auto], [one])
    s = 21
    js = I.Job(job.grid, job.vp, job.rho, job.acq.shot(s), job.stf[s:s + 1], name=f"s{s}")
    want = O.forward_job(js, vmax=float(job.grid.vpmax), box=0)[0]
    got = B.split_dcal(torch.from_numpy(auto), job.acq, job.grid.nt)[s].numpy()
    e = rel_l2(got, want)
    say(f"shot {s} of the grouped batch against the oracle: rel L2 {e:.2e}")
    assert e <= 1e-4
