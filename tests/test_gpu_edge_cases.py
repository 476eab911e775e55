"""Degenerate and boundary inputs through the whole path, GPU against the oracle: a shot with
no receivers between shots that have some, a single time step, fewer steps than the band
decimation, the smallest grids the plan accepts (2D and 3D, one tile or less), and receivers on
the corners of the interior.  Seismograms, both gradients (family 1), the image and the
illumination must match the oracle as in the other parity tests."""
import math

import numpy as np
import pytest

from paper_2311_02293_amd import inputs as I
from helpers import dev, rel_l2, say

pytestmark = pytest.mark.gpu

SUM_ABS = {4: 9 / 8 + 1 / 24, 8: 1225 / 1024 + 245 / 3072 + 49 / 5120 + 5 / 7168}


def layered(shape, lo, hi):
    """Smooth increase with depth (axis -1 is z) plus a lateral ramp, in [lo, hi]."""
    z = np.linspace(0.0, 1.0, shape[-1])
    x = np.linspace(0.0, 1.0, shape[-2])
    f = 0.8 * z[None, :] + 0.2 * x[:, None]
    if len(shape) == 3:
        f = f[None, :, :] * np.ones((shape[0], 1, 1))
    return (lo + (hi - lo) * f).astype(np.float32)


def make_job(ndim, n, order, nt, dr=1, nb=None, recs=None, srcs=None, box=1):
    N = order // 2
    d = 10.0
    n1, n2 = n[0], n[1]
    n3 = n[2] if ndim == 3 else 1
    vmin, vmax = 1800.0, 2600.0
    ppw = 5.0 if order == 4 else 3.0
    fm = 0.9 * min(15.0, vmin / (2.5 * d * ppw))
    dt = math.floor(0.8 * d / (vmax * math.sqrt(ndim) * SUM_ABS[order]) * 1e5) / 1e5
    g = I.Grid(ndim=ndim, n1=n1, n2=n2, n3=n3, d1=d, d2=d, d3=d, nb=nb or N + 2, order=order,
               nt=nt, dt=dt, fm=fm, box=box, dr=dr)
    shape = (n3, n2, n1) if ndim == 3 else (n2, n1)
    vp = layered(shape, vmin, 0.95 * vmax)
    rho = layered(shape, 1200.0, 2300.0)
    vtrue = (vp * 1.03).astype(np.float32)
    g.vpmin, g.vpmax = float(vp.min()), float(vtrue.max())
    src = np.array(srcs, np.float64)
    offs = np.cumsum([0] + [len(r) for r in recs]).astype(np.int32)
    flat = [p for r in recs for p in r]
    rec = np.array(flat, np.float64).reshape(-1, 3)
    stf = np.repeat(I.ricker(nt, dt, fm)[None, :], len(srcs), 0).astype(np.float32)
    job = I.Job(g, vp, rho, I.Acquisition(src, offs, rec), stf)
    job.extra["vp_true"] = vtrue
    return job


def line(n, d, z, step=3, ndim=2):
    return [[z * d, x * d, (n[2] // 2) * d if ndim == 3 else 0.0] for x in range(1, n[1] - 1, step)]


CASES = {
    # the middle shot records nothing: its data block is empty and it adds nothing to the
    # gradient, while it still contributes to the image through its source field alone
    "shot_without_receivers": lambda: make_job(
        2, (40, 60), 8, 220, srcs=[[30.0, 150.0, 0.0], [30.0, 300.0, 0.0], [30.0, 450.0, 0.0]],
        recs=[line((40, 60), 10.0, 3), [], line((40, 60), 10.0, 3)]),
    # one step: the first seismogram row holds the injection at the source node and nothing
    # else; the gradient and the image pair fields of level 0, which vanish, so both are zero
    "single_step": lambda: make_job(
        2, (36, 44), 8, 1, srcs=[[100.0, 200.0, 0.0]],
        recs=[[[100.0, 200.0, 0.0]] + line((36, 44), 10.0, 10, step=1)]),
    "two_steps_order4": lambda: make_job(
        2, (36, 44), 4, 2, srcs=[[100.0, 200.0, 0.0]], recs=[line((36, 44), 10.0, 10, step=1)]),
    "fewer_steps_than_decimation": lambda: make_job(
        2, (40, 48), 8, 7, dr=3, srcs=[[150.0, 230.0, 0.0]], recs=[line((40, 48), 10.0, 15, 1)]),
    "smallest_2d_grid": lambda: make_job(
        2, (8, 8), 8, 60, nb=4, srcs=[[30.0, 40.0, 0.0]], recs=[[[0.0, 0.0, 0.0], [70.0, 70.0, 0.0],
                                                               [0.0, 70.0, 0.0], [70.0, 0.0, 0.0]]]),
    "smallest_3d_grid": lambda: make_job(
        3, (8, 8, 8), 4, 40, nb=2, srcs=[[30.0, 40.0, 30.0]],
        recs=[[[0.0, 0.0, 0.0], [70.0, 70.0, 70.0], [0.0, 70.0, 30.0], [70.0, 0.0, 50.0]]]),
    "corner_receivers_box_off": lambda: make_job(
        2, (30, 70), 8, 150, box=0, srcs=[[0.0, 0.0, 0.0], [290.0, 690.0, 0.0]],
        recs=[[[0.0, 0.0, 0.0], [290.0, 690.0, 0.0], [0.0, 690.0, 0.0], [290.0, 0.0, 0.0]]] * 2),
}


def err(got, ref):
    """Relative L2 error; a reference that vanishes identically must be matched exactly."""
    got = np.asarray(got, np.float64)
    if not np.any(ref):
        return 0.0 if not np.any(got) else float("inf")
    return rel_l2(got, ref)


@pytest.fixture(scope="module")
def ctx():
    from paper_2311_02293_amd import binding as B
    return B.Context(0)


@pytest.mark.parametrize("case", sorted(CASES))
def test_edge_case_matches_oracle(ctx, case):
    from oracle import oracle as O
    from paper_2311_02293_amd import binding as B
    import torch
    job = CASES[case]()
    g = job.grid
    say("edge case", case, g, "nshot", job.acq.nshot, "rec_off", list(job.acq.rec_off))
    vmax = float(g.vpmax)
    vp, rho, stf = dev(job)
    dcal, _, _ = ctx.forward(g, job.acq, vp, rho, stf)
    ctx.poll_status()
    got = [d.cpu().numpy() for d in B.split_dcal(dcal, job.acq, g.nt)]
    ref = O.forward_job(job, vmax=vmax, box=0)
    for s in range(job.acq.nshot):
        assert got[s].shape == ref[s].shape == (g.nt, job.acq.nrec(s))
    ef = max((err(got[s], ref[s]) for s in range(job.acq.nshot) if got[s].size), default=0.0)
    dobs = O.forward_job(job, vp=job.extra["vp_true"], vmax=vmax, box=0)
    dobs_t = torch.from_numpy(np.concatenate([d.ravel() for d in dobs]).astype(np.float32)).cuda()
    r1, r2, rJ = O.fwi_grad_family(job, dobs, 1, vmax=vmax, box=0)
    g1, g2, J, _ = ctx.fwi_grad(g, job.acq, vp, rho, stf, dobs_t, rho_grad=True)
    ctx.poll_status()
    e1 = err(g1.cpu().numpy().reshape(job.vp.shape), r1)
    e2 = err(g2.cpu().numpy().reshape(job.vp.shape), r2)
    ims, ils = O.rtm_image(job, dobs, vmax=vmax, box=0, per_shot=True)
    im, il = ctx.rtm_image(g, job.acq, vp, rho, stf, dobs_t)
    ei = err(im.cpu().numpy().reshape(job.vp.shape), np.sum(ims, 0))
    el = err(il.cpu().numpy().reshape(job.vp.shape), np.sum(ils, 0))
    say("edge case", case, "forward", ef, "J", float(J.cpu()[0]), rJ, "grad", e1, e2, "image", ei, el)
    assert ef <= 1e-4
    # misfit: relative, with a floor at 1e-6 of the data energy for a residual that vanishes
    # (FP32 rounding of data that agree)
    energy = 0.5 * g.dt * sum(float(np.sum(np.asarray(d, np.float64) ** 2)) for d in dobs)
    assert abs(float(J.cpu()[0]) - rJ) <= 1e-4 * rJ + 1e-6 * energy
    assert max(e1, e2, ei, el) <= 1e-4
