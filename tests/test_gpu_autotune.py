"""GPU: the autotuner (SMI_OPT_AUTOTUNE) picks kernels by timing them, and the picked kernels
give the default's results: seismograms, gradients and images, on the first call of a plan
shape (which times the forward candidates, and alternates the 2D reverse forms) and on the
calls after it (which run the picks)."""
import re

import numpy as np
import pytest

from paper_2311_02293_amd import inputs as I
from helpers import dev, rel_l2, say, with_bounds

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    from paper_2311_02293_amd import binding as B
    return B.Context(0)


def _same(name, a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    e = rel_l2(a, b)
    say(f"{name}: tuned vs default rel L2 {e:.2e} bitwise {np.array_equal(a, b)}")
    assert e <= 1e-6


@pytest.mark.parametrize("ndim", [2, 3])
def test_tuned_forward_equals_default(ctx, ndim):
    from paper_2311_02293_amd import binding as B
    if ndim == 2:
        job = with_bounds(I.config2(n1=96, n2=260, nt=500, nshot=3))
    else:
        job = with_bounds(I.config4(n=36, nt=160, nshot=2, dr=1, rec_step=4))
    vp, rho, stf = dev(job)
    ref = ctx.forward(job.grid, job.acq, vp, rho, stf)[0].cpu().numpy()
    ctx.set_option(B.OPT_AUTOTUNE, 2)          # no picks carried over from earlier tests
    ctx.set_option(B.OPT_AUTOTUNE, 1)
    try:
        for call in range(3):
            got = ctx.forward(job.grid, job.acq, vp, rho, stf)[0].cpu().numpy()
            ctx.poll_status()
            _same(f"{ndim}D forward call {call}", got, ref)
        rep = ctx.tuning_report()
    finally:
        ctx.set_option(B.OPT_AUTOTUNE, 0)
    say("tuning report:", rep)
    assert rep.startswith("forward ") and re.search(r"pick \S+", rep)
    times = [float(x) for x in re.findall(r"([0-9.]+) us/step", rep)]
    assert times and all(t > 0 for t in times)


def test_tuned_reverse_equals_default(ctx):
    """The first gradient call alternates the 2D reverse forms on sampled iterations, the next
    reads the samples and keeps the faster; both equal the default gradient and image."""
    import torch
    from paper_2311_02293_amd import binding as B
    job = I.config3(n1=70, n2=160, nt=420, nshot=3)
    job = with_bounds(job, [job.extra["vp_true"]])
    vp, rho, stf = dev(job)
    vt = torch.from_numpy(job.extra["vp_true"]).cuda()
    dobs = ctx.forward(job.grid, job.acq, vt, rho, stf)[0]
    g0, J0, _ = ctx.fwi_grad(job.grid, job.acq, vp, rho, stf, dobs)
    i0, l0 = ctx.rtm_image(job.grid, job.acq, vp, rho, stf, dobs)
    ref = [t.cpu().numpy() for t in (g0, J0, i0, l0)]
    ctx.set_option(B.OPT_AUTOTUNE, 2)
    ctx.set_option(B.OPT_AUTOTUNE, 1)
    reports = []
    try:
        for call in range(3):
            g, J, _ = ctx.fwi_grad(job.grid, job.acq, vp, rho, stf, dobs)
            reports.append(ctx.tuning_report())
            im, il = ctx.rtm_image(job.grid, job.acq, vp, rho, stf, dobs)
            ctx.poll_status()
            for name, a, b in zip(("grad", "misfit", "image", "illum"),
                                  (t.cpu().numpy() for t in (g, J, im, il)), ref):
                _same(f"call {call} {name}", a, b)
    finally:
        ctx.set_option(B.OPT_AUTOTUNE, 0)
    say("reports:", reports)
    assert any(r.startswith("reverse ") and "pick" in r for r in reports)
