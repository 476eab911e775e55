"""GPU: bit-stable reverse passes and per-request results of batched calls.

* The adjoint sources (eq. 8) are injected as a fixed-order gather, so gradients and images
  whose receiver operators overlap (off-grid receivers two cells apart, two receivers on one
  point) are bitwise equal from run to run, and batched equal alone.
* smi_set_shot_groups: one batched call returns, per group of shots, exactly what that group's
  shots give in a call of their own (gradient, misfit, image, illumination).
* A replayed time-loop graph never stands in for a call whose source operators differ.
"""
import numpy as np
import pytest

from paper_2311_02293_amd import inputs as I
from helpers import dev, rel_l2, say, with_bounds

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    from paper_2311_02293_amd import binding as B
    return B.Context(0)


def _overlap_job(ndim, nshot=2):
    """Off-grid receivers two cells apart (operators of half-width 4 overlap) plus one pair of
    receivers on the same point, off-grid sources; small 2D or 3D grid."""
    if ndim == 2:
        job = I.config3(n1=60, n2=120, nt=360, nshot=nshot)
        d = job.grid.d1
        xs = (np.arange(4, 116, 2) + 0.5) * d
        recs = [[2.37 * d, x, 0.0] for x in xs] + [[2.37 * d, xs[7], 0.0]]
        src = np.array([[3.4 * d, (20 + 40 * s + 0.3) * d, 0.0] for s in range(nshot)])
    else:
        job = I.config4(n=28, nt=150, nshot=nshot, dr=1, rec_step=4)
        d = job.grid.d1
        recs = [[2.37 * d, (x + 0.5) * d, (y + 0.25) * d] for y in range(4, 24, 2)
                for x in range(4, 24, 2)]
        recs.append(list(recs[5]))
        src = np.array([[3.4 * d, (6 + 7 * s + 0.3) * d, 14.6 * d] for s in range(nshot)])
    rec = np.concatenate([np.array(recs)] * nshot)
    off = np.arange(nshot + 1, dtype=np.int32) * len(recs)
    job.acq = I.Acquisition(src, off, rec)
    return with_bounds(job, [job.extra["vp_true"]])


def _dobs(job):
    from oracle import oracle as O
    import torch
    d = O.forward_job(job, vp=job.extra["vp_true"], vmax=float(job.grid.vpmax), box=0)
    return d, torch.from_numpy(np.concatenate([x.ravel() for x in d]).astype(np.float32)).cuda()


@pytest.mark.parametrize("ndim", [2, 3])
def test_overlapping_adjoint_sources_are_bitwise_stable(ctx, ndim):
    """Gradient, misfit, image and illumination: two runs give the same bits; against the
    oracle within the parity tolerances."""
    from oracle import oracle as O
    job = _overlap_job(ndim)
    ref, dobs = _dobs(job)
    vp, rho, stf = dev(job)
    runs = []
    for _ in range(2):
        g, J, _ = ctx.fwi_grad(job.grid, job.acq, vp, rho, stf, dobs)
        im, il = ctx.rtm_image(job.grid, job.acq, vp, rho, stf, dobs)
        ctx.poll_status()
        runs.append([t.cpu().numpy() for t in (g, J, im, il)])
    for a, b in zip(*runs):
        np.testing.assert_array_equal(a, b)
    vmax = float(job.grid.vpmax)
    ref_g, ref_J = O.fwi_grad(job, ref, vmax=vmax, box=0)
    ref_i, ref_l = O.rtm_image(job, ref, vmax=vmax, box=0)
    g, J, im, il = runs[0]
    eg = rel_l2(g.reshape(job.vp.shape), ref_g)
    ei = rel_l2(im.reshape(job.vp.shape), ref_i)
    el = rel_l2(il.reshape(job.vp.shape), ref_l)
    say(f"{ndim}D overlapping operators: grad {eg:.2e} image {ei:.2e} illum {el:.2e} "
        f"J {float(J[0]):.6e} / {ref_J:.6e}")
    assert max(eg, ei, el) <= 1e-4
    assert abs(float(J[0]) - ref_J) <= 1e-4 * ref_J


@pytest.mark.parametrize("ndim", [2, 3])
def test_shot_groups_equal_calls_of_their_own(ctx, ndim):
    """Three shots in one call with groups {0} and {1, 2}: each group's gradient, misfit,
    image and illumination are bitwise those of a call on its shots alone."""
    job = _overlap_job(ndim, nshot=3)
    _, dobs = _dobs(job)
    vp, rho, stf = dev(job)
    nrec = int(job.acq.rec_off[1])
    nt = job.grid.nt
    npts = job.vp.size
    try:
        ctx.set_shot_groups([0, 1, 3])
        g, J, _ = ctx.fwi_grad(job.grid, job.acq, vp, rho, stf, dobs)
        im, il = ctx.rtm_image(job.grid, job.acq, vp, rho, stf, dobs)
    finally:
        ctx.set_shot_groups(None)
    g, J, im, il = (t.cpu().numpy() for t in (g, J, im, il))
    assert g.shape == (2 * npts,) and J.shape == (2,)
    for k, (a, b) in enumerate([(0, 1), (1, 3)]):
        sub = I.Job(job.grid, job.vp, job.rho,
                    I.Acquisition(job.acq.src[a:b], job.acq.rec_off[a:b + 1] - job.acq.rec_off[a],
                                  job.acq.rec[a * nrec:b * nrec]),
                    job.stf[a:b].copy())
        svp, srho, sstf = dev(sub)
        sd = dobs[a * nt * nrec:b * nt * nrec].contiguous()
        g1, J1, _ = ctx.fwi_grad(sub.grid, sub.acq, svp, srho, sstf, sd)
        im1, il1 = ctx.rtm_image(sub.grid, sub.acq, svp, srho, sstf, sd)
        ctx.poll_status()
        np.testing.assert_array_equal(g[k * npts:(k + 1) * npts], g1.cpu().numpy())
        np.testing.assert_array_equal(J[k:k + 1], J1.cpu().numpy())
        np.testing.assert_array_equal(im[k * npts:(k + 1) * npts], im1.cpu().numpy())
        np.testing.assert_array_equal(il[k * npts:(k + 1) * npts], il1.cpu().numpy())
        say(f"{ndim}D group {k} (shots {a}..{b - 1}) equals its own call")


def test_shot_groups_must_cover_the_call(ctx):
    from paper_2311_02293_amd import binding as B
    job = _overlap_job(2, nshot=2)
    _, dobs = _dobs(job)
    vp, rho, stf = dev(job)
    try:
        ctx.set_shot_groups([0, 1, 2, 3])
        with pytest.raises(B.SmiError) as e:
            ctx.fwi_grad(job.grid, job.acq, vp, rho, stf, dobs)
        assert "SMI_E_ARG" in str(e.value)
        with pytest.raises(B.SmiError):
            ctx.set_shot_groups([0, 2, 2])
    finally:
        ctx.set_shot_groups(None)


def test_graph_replay_tells_on_and_off_grid_sources_apart(ctx):
    """Graph replay with reused buffers, alternating a source on a node and one 0.3 cells off
    it (both round to the same node, same boxes and receivers): every call equals its eager
    run; the two sources give different data."""
    from paper_2311_02293_amd import binding as B
    import torch
    job = with_bounds(I.config2(n1=64, n2=160, nt=240, nshot=1))
    d = job.grid.d1
    on = job.acq.src.copy()
    on[0, :2] = [4 * d, 80 * d]
    off = on.copy()
    off[0, 1] += 0.3 * d
    vp, rho, stf = dev(job)
    nrec = int(job.acq.rec_off[-1])
    dcal = torch.empty(job.grid.nt * nrec, device="cuda")
    ws = torch.empty(ctx.workspace_bytes(job.grid, job.acq, B.JOB_FORWARD), dtype=torch.uint8,
                     device="cuda")
    eager = {}
    for name, src in (("on", on), ("off", off)):
        job.acq.src = src
        ctx.forward(job.grid, job.acq, vp, rho, stf, dcal=dcal, ws=ws)
        eager[name] = dcal.cpu().numpy().copy()
    assert rel_l2(eager["on"], eager["off"]) > 1e-3
    ctx.set_option(B.OPT_GRAPH, 1)
    try:
        for rep in range(3):
            for name, src in (("on", on), ("off", off)):
                job.acq.src = src
                dcal.zero_()
                ctx.forward(job.grid, job.acq, vp, rho, stf, dcal=dcal, ws=ws)
                torch.cuda.synchronize()
                np.testing.assert_array_equal(dcal.cpu().numpy(), eager[name])
    finally:
        ctx.set_option(B.OPT_GRAPH, 0)
