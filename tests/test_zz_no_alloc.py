"""GPU: smi_forward_static (no workspace argument; the library's static device buffer) against
smi_forward on the same inputs, on two calls in a row, the second with a smaller job, and its
host-side refusal of a job larger than the static buffer."""
import numpy as np
import pytest

from paper_2311_02293_amd import inputs as I
from helpers import dev, rel_l2, say, with_bounds

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    from paper_2311_02293_amd import binding as B
    return B.Context(0)


def _job(n1, n2, nt, nshot, off_grid=False):
    job = with_bounds(I.config2(n1=n1, n2=n2, nt=nt, nshot=nshot))
    if off_grid:
        job.acq.src[:, 1] += 0.3 * job.grid.d2
        job.acq.rec[:, 0] += 0.37 * job.grid.d1
    return job


def test_static_forward_equals_forward_on_two_calls(ctx):
    """First a larger job (3 shots, off-grid points), then a smaller one (1 shot, on-grid): the
    static entry point's seismograms equal smi_forward's bit for bit, and both match the
    oracle within the seismogram tolerance."""
    from paper_2311_02293_amd import binding as B
    from oracle import oracle as O
    for k, (n1, n2, nt, ns, og) in enumerate([(96, 260, 400, 3, True), (40, 90, 150, 1, False)]):
        job = _job(n1, n2, nt, ns, og)
        need = ctx.workspace_bytes(job.grid, job.acq, B.JOB_FORWARD)
        say(f"static forward call {k}: {n1}x{n2} nt {nt} shots {ns} off-grid {og} "
            f"workspace {need} B")
        vp, rho, stf = dev(job)
        ref, _, _ = ctx.forward(job.grid, job.acq, vp, rho, stf)
        got = ctx.forward_static(job.grid, job.acq, vp, rho, stf)
        ctx.poll_status()
        np.testing.assert_array_equal(got.cpu().numpy(), ref.cpu().numpy())
        want = O.forward_job(job, vmax=float(job.grid.vpmax), box=0)
        got = [d.cpu().numpy() for d in B.split_dcal(got, job.acq, nt)]
        for s in range(ns):
            e = rel_l2(got[s], want[s])
            say(f"  shot {s} rel L2 against the oracle {e:.2e}")
            assert e <= 1e-4


def test_static_forward_refuses_a_job_beyond_the_buffer(ctx):
    from paper_2311_02293_amd import binding as B
    job = _job(500, 1500, 40, 16)
    assert ctx.workspace_bytes(job.grid, job.acq, B.JOB_FORWARD) > 64 << 20
    vp, rho, stf = dev(job)
    with pytest.raises(B.SmiError) as e:
        ctx.forward_static(job.grid, job.acq, vp, rho, stf)
    assert "SMI_E_WORKSPACE" in str(e.value)
    # the context stays usable
    small = _job(40, 90, 60, 1)
    vp, rho, stf = dev(small)
    a = ctx.forward_static(small.grid, small.acq, vp, rho, stf)
    b, _, _ = ctx.forward(small.grid, small.acq, vp, rho, stf)
    np.testing.assert_array_equal(a.cpu().numpy(), b.cpu().numpy())
