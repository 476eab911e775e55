"""GPU: the fused 2D steps -- marching (SMI_OPT_KERNEL 6) and tiled (SMI_OPT_KERNEL 7) --
against the half-step kernels and the oracle: seismograms, and gradients / images of reverse
passes whose forward pass ran on them (bands saved by their side work, decimated bands,
off-grid points, every run or tile width)."""
import numpy as np
import pytest

from paper_2311_02293_amd import inputs as I
from helpers import dev, rel_l2, say, with_bounds

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    from paper_2311_02293_amd import binding as B
    return B.Context(0)


def _run(ctx, kernel, chunk, fn):
    from paper_2311_02293_amd import binding as B
    ctx.set_option(B.OPT_KERNEL, kernel)
    ctx.set_option(B.OPT_CHUNK, chunk)
    try:
        return fn()
    finally:
        ctx.set_option(B.OPT_KERNEL, 0)
        ctx.set_option(B.OPT_CHUNK, 0)


def _compare(name, a, b, tol=1e-6):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    same = np.array_equal(a, b)
    e = rel_l2(a, b)
    say(f"{name}: fused vs half steps rel L2 {e:.2e} bitwise {same}")
    assert e <= tol


# (SMI_OPT_KERNEL, SMI_OPT_CHUNK): the marching step's run widths and load depths, the tiled
# step's tile widths
VARIANTS = [(6, 32), (6, 64), (6, 132), (6, 432), (6, 464), (7, 32), (7, 64)]


@pytest.mark.parametrize("kernel,run", VARIANTS)
@pytest.mark.parametrize("case", ["box", "nobox", "offgrid", "order4"])
def test_fused_step_seismograms(ctx, kernel, run, case):
    from oracle import oracle as O
    box = 0 if case == "nobox" else 1
    job = with_bounds(I.config2(n1=96, n2=260, nt=500, nshot=3, box=box))
    if case == "offgrid":
        job.acq.src[:, 1] += 0.3 * job.grid.d2
        job.acq.src[:, 0] += 0.45 * job.grid.d1
        job.acq.rec[:, 0] += 0.37 * job.grid.d1
    if case == "order4":
        job.grid.order = 4
        job.grid.nb = 12
        job.grid.fm = 7.0          # five points per wavelength at order 4
    vp, rho, stf = dev(job)
    ref = ctx.forward(job.grid, job.acq, vp, rho, stf)[0].cpu().numpy()
    got = _run(ctx, kernel, run, lambda: ctx.forward(job.grid, job.acq, vp, rho, stf)[0].cpu().numpy())
    ctx.poll_status()
    _compare(f"kernel {kernel} {case} run {run} seismograms", got, ref)
    want = O.forward_job(job, vmax=float(job.grid.vpmax), box=0)
    from paper_2311_02293_amd import binding as B
    import torch
    got_s = [d.numpy() for d in B.split_dcal(torch.from_numpy(got), job.acq, job.grid.nt)]
    for s in range(job.acq.nshot):
        e = rel_l2(got_s[s], want[s])
        say(f"  shot {s} against the oracle {e:.2e}")
        assert e <= 1e-4


@pytest.mark.parametrize("kernel,dr,run", [(6, 1, 32), (6, 3, 32), (6, 1, 432), (7, 1, 32),
                                           (7, 3, 64)])
def test_fused_forward_then_reverse(ctx, kernel, dr, run):
    """Gradient and image whose forward pass (bands saved by the fused step's side work, and
    with dr > 1 the run past nt) ran on the fused step, against the half-step kernels."""
    import torch
    from oracle import oracle as O
    job = I.config3(n1=70, n2=160, nt=420, nshot=3)
    job.grid.dr = dr
    job = with_bounds(job, [job.extra["vp_true"]])
    dobs = O.forward_job(job, vp=job.extra["vp_true"], vmax=float(job.grid.vpmax), box=0)
    d = torch.from_numpy(np.concatenate([x.ravel() for x in dobs]).astype(np.float32)).cuda()
    vp, rho, stf = dev(job)

    def both():
        g, J, dc = ctx.fwi_grad(job.grid, job.acq, vp, rho, stf, d, want_dcal=True)
        im, il = ctx.rtm_image(job.grid, job.acq, vp, rho, stf, d)
        return [t.cpu().numpy() for t in (g, J, dc, im, il)]

    ref = both()
    got = _run(ctx, kernel, run, both)
    ctx.poll_status()
    for name, a, b in zip(("grad", "misfit", "dcal", "image", "illum"), got, ref):
        _compare(f"kernel {kernel} dr {dr} {name}", a, b)
    if dr == 1:
        ref_g, ref_J = O.fwi_grad(job, dobs, vmax=float(job.grid.vpmax), box=0)
        e = rel_l2(got[0].reshape(job.vp.shape), ref_g)
        say(f"  gradient against the oracle {e:.2e}")
        assert e <= 1e-4
