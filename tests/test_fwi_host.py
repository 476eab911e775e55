"""FWI driver logic on the CPU (no GPU): L-BFGS two-loop recursion, Wolfe line search, bounds,
SGD shot batches, parametrisation transforms."""
import math

import numpy as np
import pytest
import torch

from paper_2311_02293_amd import fwi as F


def quad(A, b):
    A = torch.as_tensor(A, dtype=torch.float64)
    b = torch.as_tensor(b, dtype=torch.float64)

    def fg(x):
        return float(0.5 * x @ A @ x - b @ x), A @ x - b
    return fg


def test_lbfgs_minimises_a_convex_quadratic():
    rng = np.random.default_rng(3)
    Q = rng.standard_normal((12, 12))
    A = Q @ Q.T + 12 * np.eye(12)
    b = rng.standard_normal(12)
    x, h = F.lbfgs(quad(A, b), torch.zeros(12, dtype=torch.float64),
                   F.LbfgsConfig(niter=60, npair=6, first_step=0.5))
    xs = np.linalg.solve(A, b)
    assert np.max(np.abs(x.numpy() - xs)) <= 1e-7 * np.max(np.abs(xs))
    assert all(b <= a + 1e-12 for a, b in zip(h.J, h.J[1:]))       # monotone decrease


def test_lbfgs_minimises_rosenbrock():
    def fg(x):
        a, b = float(x[0]), float(x[1])
        J = (1 - a) ** 2 + 100 * (b - a * a) ** 2
        g = torch.tensor([-2 * (1 - a) - 400 * a * (b - a * a), 200 * (b - a * a)],
                         dtype=torch.float64)
        return J, g
    x, h = F.lbfgs(fg, torch.tensor([-1.2, 1.0], dtype=torch.float64),
                   F.LbfgsConfig(niter=200, npair=5, first_step=0.1))
    assert np.allclose(x.numpy(), [1.0, 1.0], atol=1e-5), x


def test_two_loop_recovers_the_inverse_hessian_of_a_quadratic():
    """With n exact pairs of an n-dimensional quadratic, BFGS's H equals A^-1 on those
    directions: H y_i = s_i (the secant equations) for the newest pair exactly."""
    rng = np.random.default_rng(5)
    Q = rng.standard_normal((6, 6))
    A = torch.as_tensor(Q @ Q.T + 6 * np.eye(6))
    pairs = []
    for _ in range(6):
        s = torch.as_tensor(rng.standard_normal(6))
        pairs.append((s, A @ s))
    for k in range(1, 7):
        s, y = pairs[k - 1]
        np.testing.assert_allclose(F.two_loop(y, pairs[:k]).numpy(), s.numpy(), rtol=1e-10, atol=1e-12)


def test_bounds_are_respected_and_active_at_the_solution():
    A = np.eye(3)
    b = np.array([5.0, -5.0, 0.5])                       # unconstrained minimum (5, -5, 0.5)
    lo = torch.tensor([-1.0, -1.0, -1.0], dtype=torch.float64)
    hi = torch.tensor([1.0, 1.0, 1.0], dtype=torch.float64)
    x, _ = F.lbfgs(quad(A, b), torch.zeros(3, dtype=torch.float64),
                   F.LbfgsConfig(niter=40, first_step=0.5), lo, hi)
    np.testing.assert_allclose(x.numpy(), [1.0, -1.0, 0.5], atol=1e-6)


def test_wolfe_step_satisfies_both_conditions():
    def fg(x):
        return float((x ** 4).sum() - 3 * (x ** 2).sum() + x.sum()), 4 * x ** 3 - 6 * x + 1
    x = torch.tensor([0.3, -0.2], dtype=torch.float64)
    J0, g0 = fg(x)
    d = -g0
    cfg = F.LbfgsConfig()
    a, xn, Jn, gn = F.wolfe_search(fg, x, J0, g0, d, 1e-3, cfg)
    slope = float(g0 @ d)
    assert Jn <= J0 + cfg.c1 * a * slope
    assert float(gn @ d) >= cfg.c2 * slope


@pytest.mark.parametrize("nshot,batch", [(10, 4), (8, 2), (5, 5)])
def test_shot_batches_visit_every_shot_once_per_epoch(nshot, batch):
    b = F.shot_batches(nshot, batch, epochs=3, seed=11)
    per = math.ceil(nshot / batch)
    assert len(b) == 3 * per
    for e in range(3):
        ep = b[e * per:(e + 1) * per]
        assert sorted(i for x in ep for i in x) == list(range(nshot))
        assert [len(x) for x in ep] == [batch] * (per - 1) + [nshot - batch * (per - 1)]
    assert F.shot_batches(nshot, batch, 3, seed=11) == b                 # seeded


def test_family_transforms_round_trip():
    class Job:
        pass
    job = Job()
    job.vp = np.array([[1500.0, 2500.0], [3000.0, 2000.0]], np.float32)
    job.rho = np.array([[1000.0, 2200.0], [2400.0, 1800.0]], np.float32)
    for family in (1, 2):
        p = F.FwiProblem.__new__(F.FwiProblem)
        p.family, p.npar, p.n, p.dev, p.bounds = family, 2, 4, torch.device("cpu"), F.Bounds()
        vp = torch.from_numpy(job.vp).reshape(-1)
        rho = torch.from_numpy(job.rho).reshape(-1)
        x = p.to_x(vp, rho)
        v2, r2 = p.to_model(x)
        np.testing.assert_allclose(v2.numpy(), vp.numpy(), rtol=1e-6)
        np.testing.assert_allclose(r2.numpy(), rho.numpy(), rtol=1e-6)
        if family == 2:
            np.testing.assert_allclose(np.exp(x[4:].numpy()), (vp * rho).numpy(), rtol=1e-6)
        lo, hi = p.x_bounds()
        assert lo.shape == x.shape and bool((lo < hi).all())


def _line_acq():
    from paper_2311_02293_amd import inputs as I
    return I._surface_line(np.array([100.0, 500.0]), 20.0, np.arange(0, 1000, 50.0), 20.0)


def test_offset_weights_follow_the_table():
    acq = _line_acq()
    nt = 7
    w = F.offset_weights(acq, nt, dxw=200.0, xw=[0.0, 0.5, 1.0])
    assert w.shape == (nt * int(acq.rec_off[-1]),)
    s = 0
    a, b = int(acq.rec_off[s]), int(acq.rec_off[s + 1])
    block = w[nt * a: nt * b].reshape(nt, b - a)
    off = np.abs(acq.rec[a:b, 1] - acq.src[s, 1])
    exp = np.clip(off / 200.0 * 0.5, 0.0, 1.0)
    np.testing.assert_allclose(block[3], exp, atol=1e-6)
    assert np.all(block == block[0])                      # constant in time


@pytest.mark.parametrize("mode", [1, 2])
def test_mute_weights_cut_at_the_mute_line(mode):
    acq = _line_acq()
    nt, dt = 200, 0.01
    w = F.mute_weights(acq, nt, dt, xmute=[0.0, 1000.0], tmute=[0.2, 1.2], ntaper=10, mode=mode)
    a, b = int(acq.rec_off[0]), int(acq.rec_off[1])
    block = w[nt * a: nt * b].reshape(nt, b - a)
    for r in range(b - a):
        off = abs(acq.rec[a + r, 1] - acq.src[0, 1])
        tcut = 0.2 + off / 1000.0
        i0 = int(np.floor(tcut / dt + 1e-9))
        before, after = block[: max(i0 - 1, 0), r], block[i0 + 11:, r]
        if mode == 1:
            assert np.all(before == 0) and np.all(after == 1)
        else:
            assert np.all(before == 1) and np.all(after == 0)
        assert np.all((block[:, r] >= 0) & (block[:, r] <= 1))
