"""GPU: 2D reverse passes run in shot groups (SMI_OPT_REV_GROUP) give bitwise the results of one
reverse loop over all shots -- gradients (Vp and density, the face sums), misfit, image,
illumination and snapshots of the reconstructed field -- with off-grid sources and receivers
(overlapping operators), decimated bands, a free surface, both reverse-step forms, per-request
shot groups and graph replay; and the automatic grouping of a gradient whose reverse state
exceeds the last-level cache agrees with the oracle."""
import numpy as np
import pytest

from paper_2311_02293_amd import inputs as I
from helpers import dev, rel_l2, say, with_bounds

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    from paper_2311_02293_amd import binding as B
    return B.Context(0)


def _job(nshot=5, dr=1, freesurf=0, offgrid=True):
    job = I.config3(n1=70, n2=160, nt=420, nshot=nshot)
    job.grid.dr = dr
    job.grid.freesurf = freesurf
    if offgrid:
        xmax = (job.grid.n2 - 1) * job.grid.d2
        job.acq.rec[:, 1] = np.minimum(job.acq.rec[:, 1] + 3.3, xmax)
        job.acq.src[:, 1] += 1.7
        job.acq.src[:, 0] += 0.4 * job.grid.d1
    return with_bounds(job, [job.extra["vp_true"]])


def _dobs(ctx, job):
    import torch
    _, rho, stf = dev(job)
    d, _, _ = ctx.forward(job.grid, job.acq, torch.from_numpy(job.extra["vp_true"]).cuda(), rho, stf)
    return d


def _with(ctx, opts, fn):
    from paper_2311_02293_amd import binding as B
    for k, v in opts.items():
        ctx.set_option(k, v)
    try:
        return fn()
    finally:
        for k in opts:
            ctx.set_option(k, 0)
        ctx.set_option(B.OPT_REV_GROUP, 0)


def _equal(name, got, ref):
    for k, (a, b) in enumerate(zip(got, ref)):
        same = np.array_equal(a, b)
        say(f"{name} output {k}: bitwise {same}, rel L2 {rel_l2(a, b):.2e}")
        assert same


CASES = {
    "grad": dict(dr=1),
    "grad-dr3": dict(dr=3),
    "grad-freesurf": dict(dr=1, freesurf=1),
}


@pytest.mark.parametrize("case", list(CASES))
@pytest.mark.parametrize("per", [1, 2, 3])
def test_grouped_gradient_equals_one_loop(ctx, case, per):
    """Vp and density gradients and the misfit of a 5-shot gradient with at most `per` shots
    per reverse loop, against one loop over the 5 shots."""
    from paper_2311_02293_amd import binding as B
    job = _job(**CASES[case])
    vp, rho, stf = dev(job)
    d = _dobs(ctx, job)

    def run(k):
        return _with(ctx, {B.OPT_REV_GROUP: k}, lambda: [
            t.cpu().numpy() for t in ctx.fwi_grad(job.grid, job.acq, vp, rho, stf, d,
                                                  rho_grad=True)[:3]])
    ref = run(job.acq.nshot)
    got = run(per)
    ctx.poll_status()
    _equal(f"{case} groups of {per}", got, ref)


@pytest.mark.parametrize("form", [1, 2])
def test_grouped_image_equals_one_loop(ctx, form):
    """Image and illumination (decimated bands, dr 3) with groups of 2 shots, each reverse-step
    form (two launches, five launches)."""
    from paper_2311_02293_amd import binding as B
    job = _job(dr=3)
    vp, rho, stf = dev(job)
    d = _dobs(ctx, job)

    def run(k):
        return _with(ctx, {B.OPT_REV_GROUP: k, B.OPT_REVERSE: form}, lambda: [
            t.cpu().numpy() for t in ctx.rtm_image(job.grid, job.acq, vp, rho, stf, d)])
    ref = run(job.acq.nshot)
    got = run(2)
    _equal(f"image form {form}", got, ref)


def test_grouped_snapshots_and_request_groups_equal_one_loop(ctx):
    """Snapshots of the reconstructed field taken inside the grouped reverse loops, and outputs
    reduced per request (smi_set_shot_groups over 2 + 3 shots) while the reverse loop runs in
    groups of 2 that straddle the requests."""
    from paper_2311_02293_amd import binding as B
    job = _job()
    vp, rho, stf = dev(job)
    levels = [0, 100, 250, job.grid.nt]

    def rec(k):
        def go():
            _, _, state = ctx.forward(job.grid, job.acq, vp, rho, stf, save=True)
            out = ctx.adjoint_reconstruct(state, None, grad=False, image=False, illum=False,
                                          snaps=levels, nshot=job.acq.nshot, npts=job.vp.size)
            return [out["snaps"].cpu().numpy()]
        return _with(ctx, {B.OPT_REV_GROUP: k}, go)
    _equal("snapshots", rec(2), rec(job.acq.nshot))

    d = _dobs(ctx, job)
    ctx.set_shot_groups([0, 2, 5])
    try:
        def run(k):
            return _with(ctx, {B.OPT_REV_GROUP: k}, lambda: [
                t.cpu().numpy() for t in ctx.fwi_grad(job.grid, job.acq, vp, rho, stf, d)[:2]])
        ref = run(job.acq.nshot)
        got = run(2)
    finally:
        ctx.set_shot_groups(None)
    _equal("per-request gradients", got, ref)


def test_grouped_reverse_as_graph_equals_eager(ctx):
    """The grouped reverse loops captured as a HIP graph and replayed (twice, with eager work
    between) give the eager grouped result."""
    import torch
    from paper_2311_02293_amd import binding as B
    job = _job()
    vp, rho, stf = dev(job)
    d = _dobs(ctx, job)

    def call():
        return [t.cpu().numpy() for t in ctx.fwi_grad(job.grid, job.acq, vp, rho, stf, d)[:2]]
    ref = _with(ctx, {B.OPT_REV_GROUP: 2}, call)
    for rep in range(3):
        got = _with(ctx, {B.OPT_REV_GROUP: 2, B.OPT_GRAPH: 1}, call)
        torch.cuda.synchronize()
        _equal(f"graph replay {rep}", got, ref)


def test_automatic_groups_of_a_large_gradient_match_the_oracle(ctx):
    """A 2D gradient whose reverse state (32 shots of 300 x 900 with the computing box off,
    about 13 MB each) exceeds the 224 MiB group budget runs its reverse loop in automatic
    groups; it equals the one-loop result bitwise, and two of its shots' gradients, run alone,
    agree with the oracle (observed data: 0.9 times the oracle's data of the true model)."""
    import torch
    from oracle import oracle as O
    from paper_2311_02293_amd import binding as B
    job = I.config3(nt=300, nshot=32)
    job.grid.box = 0
    job = with_bounds(job, [job.extra["vp_true"]])
    vp, rho, stf = dev(job)
    d = _dobs(ctx, job)
    auto = [t.cpu().numpy() for t in ctx.fwi_grad(job.grid, job.acq, vp, rho, stf, d)[:2]]
    one = _with(ctx, {B.OPT_REV_GROUP: job.acq.nshot}, lambda: [
        t.cpu().numpy() for t in ctx.fwi_grad(job.grid, job.acq, vp, rho, stf, d)[:2]])
    _equal("automatic groups", auto, one)
    for s in (0, 19):
        js = I.Job(job.grid, job.vp, job.rho, job.acq.shot(s), job.stf[s:s + 1], name=f"s{s}")
        # 300 steps end before the wave meets the anomaly: scaled data keep the residual large
        dobs = [0.9 * x for x in O.forward_job(js, vp=job.extra["vp_true"],
                                               vmax=float(job.grid.vpmax), box=0)]
        ds = torch.from_numpy(np.concatenate([x.ravel() for x in dobs]).astype(np.float32)).cuda()
        _, rho_s, stf_s = dev(js)
        g, _, _ = ctx.fwi_grad(js.grid, js.acq, vp, rho_s, stf_s, ds)
        ref_g, _ = O.fwi_grad(js, dobs, vmax=float(job.grid.vpmax), box=0)
        e = rel_l2(g.cpu().numpy().reshape(job.vp.shape), ref_g)
        say(f"shot {s} alone against the oracle: rel L2 {e:.2e}")
        assert e <= 1e-4
