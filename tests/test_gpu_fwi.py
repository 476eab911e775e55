"""FWI driver on the GPU: a few bounded L-BFGS iterations (Alg. 1) and one SGD epoch (Sec. 5)
on a small 2D problem reduce the misfit and move the model towards the true one."""
import numpy as np
import pytest

from paper_2311_02293_amd import inputs as I
from helpers import rel_l2, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def setup():
    import torch
    from paper_2311_02293_amd import binding as B
    ctx = B.Context(0)
    job = I.config3(n1=50, n2=120, nt=500, nshot=4)
    vt = job.extra["vp_true"]
    rt = job.rho.copy()
    rt[40:80, 15:35] *= 1.1
    job.grid.vpmin, job.grid.vpmax = 1400.0, 4900.0
    dev = "cuda:0"
    vt_t = torch.from_numpy(vt).to(dev)
    rt_t = torch.from_numpy(rt).to(dev)
    stf = torch.from_numpy(job.stf).to(dev)
    dobs, _, _ = ctx.forward(job.grid, job.acq, vt_t, rt_t, stf)
    return ctx, job, dobs, vt, rt


def test_lbfgs_reduces_misfit_and_model_error(setup):
    from paper_2311_02293_amd import fwi as F
    ctx, job, dobs, vt, _ = setup
    b = F.Bounds(vpmin=1400.0, vpmax=4900.0, rhomin=1500.0, rhomax=3000.0)
    vp, rho, h = F.invert(ctx, job, dobs, family=1, npar=1, bounds=b,
                          cfg=F.LbfgsConfig(niter=4, nls=8, first_step=0.02))
    say("lbfgs J", h.J, "fg calls", h.nfg)
    assert len(h.J) >= 3
    assert all(b2 < b1 for b1, b2 in zip(h.J, h.J[1:]))
    assert h.J[-1] < 0.8 * h.J[0]
    v = vp.cpu().numpy().reshape(job.vp.shape)
    assert np.linalg.norm(v - vt) < np.linalg.norm(job.vp - vt)
    assert v.min() >= 1400.0 - 1e-2 and v.max() <= 4900.0 + 1e-2


def test_two_parameter_family2_reduces_misfit(setup):
    from paper_2311_02293_amd import fwi as F
    ctx, job, dobs, _, _ = setup
    b = F.Bounds(vpmin=1400.0, vpmax=4900.0, rhomin=1500.0, rhomax=3000.0)
    vp, rho, h = F.invert(ctx, job, dobs, family=2, npar=2, bounds=b,
                          cfg=F.LbfgsConfig(niter=3, nls=8, first_step=0.02))
    say("family 2 J", h.J)
    assert h.J[-1] < 0.9 * h.J[0]


def test_sgd_epoch_decreases_each_batch(setup):
    from paper_2311_02293_amd import fwi as F
    ctx, job, dobs, _, _ = setup
    b = F.Bounds(vpmin=1400.0, vpmax=4900.0)
    vp, rho, log = F.sgd(ctx, job, dobs, batch=3, epochs=1, seed=5, bounds=b, first_step=0.02)
    say("sgd", [(bb, round(a, 6), round(c, 6)) for bb, a, c in log])
    assert [len(bb) for bb, _, _ in log] == [3, 1]
    assert all(c < a for _, a, c in log)


def _oracle_fg(job, dobs_list, vmax, weights=None):
    """(J, dJ/d ln Vp) of the oracle at x = ln Vp (rho fixed), with optional data weights w:
    J = 1/2 dt sum (w r)^2, adjoint source dt w^2 r -- the same as the GPU problem."""
    import torch
    from oracle import oracle as O

    def fg(x):
        vp = torch.exp(x).float().cpu().numpy().reshape(job.vp.shape)
        if weights is None:
            g, J = O.fwi_grad(job, dobs_list, vp=vp, vmax=vmax)
        else:
            gr = O.og_grid(job.grid, vmax=vmax)
            gk = np.zeros(vp.size)
            J = 0.0
            for s in range(job.acq.nshot):
                src, rec, st, rt = O.shot_ops(job.grid, job.acq, s)
                fw = O.forward(gr, vp, job.rho, src, job.stf[s], rec, bands=True, final=True,
                               st=st, rt=rt)
                w = weights[s]
                r = w * (fw["dcal"] - dobs_list[s])
                J += 0.5 * job.grid.dt * float(np.sum(r * r))
                out = O.adjoint(gr, vp, job.rho, src, job.stf[s], rec, job.grid.dt * w * r,
                                bands=fw["bands"], final=fw["final"], want=("gk",), st=st, rt=rt)
                gk += out["gk"]
            g = (2.0 * job.rho.astype(np.float64).ravel() * vp.astype(np.float64).ravel()
                 * gk).reshape(vp.shape)
        return J, torch.from_numpy((g.astype(np.float64) * vp.astype(np.float64)).ravel())
    return fg


def _two_fixed_iterations(fg, x0, first_step):
    """Two L-BFGS iterations of Alg. 1 with fixed trial steps: a steepest-descent step scaled
    to `first_step`, then the unit step along the two-loop direction of the first pair."""
    from paper_2311_02293_amd import fwi as F
    J0, g0 = fg(x0)
    d0 = -g0
    x1 = x0 + first_step / float(d0.abs().max()) * d0
    J1, g1 = fg(x1)
    d1 = -F.two_loop(g1, [(x1 - x0, g1 - g0)])
    x2 = x1 + d1
    J2, _ = fg(x2)
    return [x0, x1, x2], [J0, J1, J2]


def test_lbfgs_iterations_on_gpu_gradients_match_oracle_ones():
    """Alg. 1 on a small 2D problem (4 shots, rho fixed, log-Vp variables): two iterations
    with fixed trial steps, once on the GPU's misfit and gradient, once on the oracle's; the
    models agree to 1e-4 rel L2 after each iteration, and so do the model updates."""
    import torch
    from oracle import oracle as O
    from paper_2311_02293_amd import binding as B
    from paper_2311_02293_amd import fwi as F
    job = I.config3(n1=50, n2=120, nt=500, nshot=4)
    bounds = F.Bounds(vpmin=1400.0, vpmax=4900.0)
    job.grid.vpmin, job.grid.vpmax = bounds.vpmin, bounds.vpmax
    dobs = O.forward_job(job, vp=job.extra["vp_true"], vmax=bounds.vpmax)
    dt = torch.from_numpy(np.concatenate([d.ravel() for d in dobs]).astype(np.float32)).cuda()
    prob = F.FwiProblem(B.Context(0), job, dt, bounds=bounds)
    x0 = torch.log(torch.from_numpy(job.vp.astype(np.float64)).reshape(-1))

    def gpu_fg(x):
        J, g = prob(x.cuda())
        return J, g.cpu()
    xs_g, Js_g = _two_fixed_iterations(gpu_fg, x0, 0.02)
    xs_o, Js_o = _two_fixed_iterations(_oracle_fg(job, dobs, bounds.vpmax), x0, 0.02)
    for k in range(3):
        vg, vo = torch.exp(xs_g[k]).numpy(), torch.exp(xs_o[k]).numpy()
        e = rel_l2(vg, vo)
        du = rel_l2(xs_g[k] - xs_g[max(k - 1, 0)], xs_o[k] - xs_o[max(k - 1, 0)]) if k else 0.0
        say(f"iteration {k}: J {Js_g[k]:.6e} / {Js_o[k]:.6e}, model rel L2 {e:.2e}, update rel L2 {du:.2e}")
        assert e <= 1e-4
        assert du <= 1e-4
        assert abs(Js_g[k] - Js_o[k]) <= 1e-4 * Js_o[k]
    assert Js_g[2] < Js_g[0]


def test_weighted_and_muted_misfit_gradient_match_oracle():
    """Offset weighting and front muting (Sec. 3.7) on the GPU path: J and dJ/d ln Vp with the
    data weights of both, against the oracle with the same weights."""
    import torch
    from oracle import oracle as O
    from paper_2311_02293_amd import binding as B
    from paper_2311_02293_amd import fwi as F
    job = I.config3(n1=50, n2=120, nt=500, nshot=3)
    bounds = F.Bounds(vpmin=1400.0, vpmax=4900.0)
    job.grid.vpmin, job.grid.vpmax = bounds.vpmin, bounds.vpmax
    nt = job.grid.nt
    dobs = O.forward_job(job, vp=job.extra["vp_true"], vmax=bounds.vpmax)
    w = (F.offset_weights(job.acq, nt, 100.0, [1.0, 0.8, 0.5, 0.3]) *
         F.mute_weights(job.acq, nt, job.grid.dt, [0.0, 1200.0], [0.05, 0.45], 20, 1))
    wl = [w[nt * int(job.acq.rec_off[s]): nt * int(job.acq.rec_off[s + 1])].reshape(nt, -1).astype(np.float64)
          for s in range(job.acq.nshot)]
    dt = torch.from_numpy(np.concatenate([d.ravel() for d in dobs]).astype(np.float32)).cuda()
    prob = F.FwiProblem(B.Context(0), job, dt, bounds=bounds, weights=torch.from_numpy(w).cuda())
    x = torch.log(torch.from_numpy(job.vp.astype(np.float64)).reshape(-1))
    Jg, gg = prob(x.cuda())
    Jo, go = _oracle_fg(job, dobs, bounds.vpmax, weights=wl)(x)
    e = rel_l2(gg.cpu().numpy(), go.numpy())
    say(f"weighted + muted: J {Jg:.6e} / {Jo:.6e}, gradient rel L2 {e:.2e}")
    assert abs(Jg - Jo) <= 1e-4 * Jo
    assert e <= 1e-4
