"""Pins of the FP64 oracle against what the paper and the mathematics fix (CPU only).

Each test ties one part of the oracle to something other than itself: exact rationals,
closed-form Green's functions, conserved energy, reciprocity, the adjoint dot product,
finite differences, exact invertibility of the leap-frog step.  A plausible slip in the
oracle (a dropped term, a sign, an index shift, a transposed operand) breaks one of them.
"""
import math
from fractions import Fraction

import numpy as np
import pytest

from paper_2311_02293_amd import inputs as I


# ----------------------------------------------------------------------------- helpers

def smooth_random_model(n1, n2, seed, vmin=1800.0, vmax=2600.0, n3=None):
    from scipy.ndimage import gaussian_filter
    rng = np.random.default_rng(seed)
    shape = (n3, n2, n1) if n3 else (n2, n1)
    v = gaussian_filter(rng.standard_normal(shape), 3.0, mode="nearest")
    v = (v - v.min()) / (v.max() - v.min())
    vp = (vmin + (vmax - vmin) * v).astype(np.float32)
    r = gaussian_filter(rng.standard_normal(shape), 3.0, mode="nearest")
    r = (r - r.min()) / (r.max() - r.min())
    rho = (1000.0 + 1500.0 * r).astype(np.float32)
    return vp, rho


def small_grid(order=8, n1=48, n2=64, nt=300, nb=10, dt=1e-3, fm=15.0, ndim=2, n3=1, d=10.0,
               box=0, dr=1):
    return I.Grid(ndim=ndim, n1=n1, n2=n2, n3=n3, d1=d, d2=d, d3=d, nb=nb, order=order, nt=nt,
                  dt=dt, fm=fm, box=box, dr=dr)


def padded_model(vp, rho, nb, ndim):
    """kappa and beta_a on the padded grid, written out for the energy pin."""
    pad = [(nb, nb)] * ndim
    v = np.pad(vp.astype(np.float64), pad, mode="edge")
    r = np.pad(rho.astype(np.float64), pad, mode="edge")
    kap = r * v * v
    bets = []
    # numpy axis order is (.., x, z): paper axis a -> numpy axis ndim-1-a
    for a in range(ndim):
        ax = ndim - 1 - a
        rn = np.concatenate([np.take(r, range(1, r.shape[ax]), axis=ax),
                             np.take(r, [r.shape[ax] - 1], axis=ax)], axis=ax)
        bets.append(2.0 / (r + rn))
    return kap, bets


# ----------------------------------------------------------------------------- P1

@pytest.mark.parametrize("order", [2, 4, 6, 8, 10, 12, 14, 16])
def test_fd_coefficients_solve_the_exactness_system(oracle, order):
    """eq. (4): a_l make the staggered difference exact on polynomials of degree <= 2N-1;
    the oracle's closed form must equal the solution of that linear system, and the stencil
    must miss the first derivative of x^(2N+1) (order exactly 2N)."""
    N = order // 2
    a = oracle.fd_coef(order)
    # sum_l a_l * 2 ((2l-1)/2)^(2k-1) = delta_{k,1}, k = 1..N  (odd monomials; even ones vanish)
    A = [[2 * Fraction(2 * l - 1, 2) ** (2 * k - 1) for l in range(1, N + 1)] + [Fraction(k == 1)]
         for k in range(1, N + 1)]
    for c in range(N):  # exact Gauss-Jordan elimination over the rationals
        piv = next(r for r in range(c, N) if A[r][c] != 0)
        A[c], A[piv] = A[piv], A[c]
        A[c] = [x / A[c][c] for x in A[c]]
        for r in range(N):
            if r != c and A[r][c] != 0:
                A[r] = [x - A[r][c] * y for x, y in zip(A[r], A[c])]
    np.testing.assert_allclose(a, [float(A[k][N]) for k in range(N)], rtol=1e-14, atol=0)
    x0, h = 0.37, 1.0 / N  # f(x) = (x0 + h x)^k keeps every sample below 1
    for k in range(0, 2 * N + 2):
        f = lambda x: (x0 + h * x) ** k
        approx = sum(a[l - 1] * (f((2 * l - 1) / 2.0) - f(-(2 * l - 1) / 2.0)) for l in range(1, N + 1))
        exact = h * k * x0 ** (k - 1) if k > 0 else 0.0
        if k <= 2 * N:
            assert abs(approx - exact) < 1e-13, (k, approx, exact)
        else:
            assert abs(approx - exact) > 1e-13 * 1e3, (k, approx, exact)


def test_fd_coefficients_known_rationals(oracle):
    """Fornberg's staggered weights quoted in the literature the paper cites for eq. (4)
    (fixture tests/golden/fd_coefficients.txt)."""
    import os
    known = {}
    path = os.path.join(os.path.dirname(__file__), "golden", "fd_coefficients.txt")
    for line in open(path):
        if line.strip() and not line.startswith("#"):
            o, l, num, den = map(int, line.split())
            known.setdefault(o, []).append(Fraction(num, den))
    assert sorted(known) == [4, 8]
    for order, fr in known.items():
        np.testing.assert_allclose(oracle.fd_coef(order), [float(x) for x in fr], rtol=1e-15)
    assert abs(np.sum(np.abs(oracle.fd_coef(8))) - 1.2863095238095) < 1e-12


# ----------------------------------------------------------------------------- P2

@pytest.mark.parametrize("factor,stable", [(0.99, True), (1.01, False)])
def test_cfl_bound_is_sharp(oracle, factor, stable):
    """eq. (5) is the leap-frog stability limit: just below it a random field stays bounded,
    just above it grows without bound (homogeneous medium, no absorption)."""
    c, d, order = 2000.0, 10.0, 8
    g = small_grid(order=order, n1=64, n2=64, nt=400, nb=4, d=d)
    coef = np.sum(np.abs(oracle.fd_coef(order)))
    g.dt = factor / (c * math.sqrt(2.0) / d * coef)
    vp, rho = I.homogeneous(2, 64, d, c)
    gr = oracle.og_grid(g, vmax=c, pml=0)
    assert abs(oracle.cfl_number(g, c) - factor) < 1e-12
    P = oracle.padded_size(gr)
    rng = np.random.default_rng(7)
    init = np.zeros((4, P))
    init[0] = rng.standard_normal(P)
    src = np.array([36, 36, 0], np.int32)
    rec = np.array([[20, 20, 0], [36, 50, 0]], np.int32)
    out = oracle.forward(gr, vp, rho, src, np.zeros(g.nt), rec, init=init)
    amp = np.max(np.abs(out["dcal"][-50:]))
    if stable:
        assert amp < 10.0
    else:
        assert amp > 1e6


# ----------------------------------------------------------------------------- P3

def test_energy_is_conserved_without_absorption(oracle):
    """Discrete energy E^n = 1/2 sum p^2/kappa + 1/2 sum_a v_a^{n+1/2} v_a^{n-1/2}/beta_a
    is invariant for the staggered leap-frog with D- = -(D+)^T (PML off, no source)."""
    g = small_grid(order=8, n1=40, n2=56, nt=800, nb=6)
    vp, rho = smooth_random_model(g.n1, g.n2, 11)
    gr = oracle.og_grid(g, vmax=float(vp.max()), pml=0)
    kap, bets = padded_model(vp, rho, g.nb, 2)
    M2, M1 = kap.shape
    z = np.arange(M1)[None, :] - M1 / 2
    x = np.arange(M2)[:, None] - M2 / 2
    init = np.zeros((4, M1 * M2))
    init[0] = np.exp(-(x * x + z * z) / 8.0).ravel()
    out = oracle.forward(gr, vp, rho, np.array([20, 20, 0], np.int32), np.zeros(g.nt),
                         np.array([[20, 30, 0]], np.int32), init=init, hist=True)
    h = out["hist"]
    E = []
    for n in range(g.nt):
        e = 0.5 * np.sum(h[n, 0] ** 2 / kap.ravel())
        for a in range(2):
            e += 0.5 * np.sum(h[n + 1, 1 + a] * h[n, 1 + a] / bets[a].ravel())
        E.append(e)
    E = np.array(E)
    assert np.max(np.abs(E - E[0])) / E[0] < 1e-12
    # the field really moved
    assert np.max(np.abs(h[-1, 0] - h[0, 0])) > 0.1


# ----------------------------------------------------------------------------- P4

def _green_case(oracle, A, order, dt, window=0.6, n=241, nb=20, c=2000.0, fm=10.0):
    nt = int(round(window / dt))
    g = I.Grid(ndim=2, n1=n, n2=n, d1=10.0, d2=10.0, nb=nb, order=order, nt=nt, dt=dt, fm=fm)
    vp, rho = I.homogeneous(2, n, 10.0, c)
    gr = oracle.og_grid(g, vmax=c)
    ctr = nb + n // 2
    src = np.array([ctr, ctr, 0], np.int32)
    rec = np.array([[ctr, ctr + 30, 0], [ctr, ctr + 60, 0]], np.int32)
    out = oracle.forward(gr, vp, rho, src, I.ricker(nt, dt, fm), rec)
    t = (np.arange(nt) + 1) * dt
    errs = []
    for k, r in enumerate([300.0, 600.0]):
        ref = A.green2d_trace(r, c, t, fm, 1.2 / fm, dt, ntau=20000)
        errs.append(np.linalg.norm(out["dcal"][:, k] - ref) / np.linalg.norm(ref))
    return errs


def test_green_function_2d_order4(oracle):
    """Homogeneous 2D medium: seismograms match p = G2 * s' (amplitude, phase, the dt/2
    source timing and the 1/dV source normalisation all enter)."""
    from oracle import analytic as A
    e300, e600 = _green_case(oracle, A, 4, 1e-3)
    assert e300 <= 5e-3 and e600 <= 1e-2, (e300, e600)


def test_green_function_2d_order8_converges_in_dt(oracle):
    """At order 8 the time discretisation dominates: halving dt cuts the error ~4x."""
    from oracle import analytic as A
    e1 = _green_case(oracle, A, 8, 1e-3)[0]
    e2 = _green_case(oracle, A, 8, 0.5e-3)[0]
    assert e1 < 1e-2
    assert 3.5 <= e1 / e2 <= 4.5, (e1, e2)


def test_green_function_3d(oracle):
    """Homogeneous 3D medium: p = s'(t - r/c) / (4 pi c^2 r)."""
    from oracle import analytic as A
    c, d, fm, dt, n, nb = 2000.0, 10.0, 15.0, 1e-3, 61, 10
    nt = 260
    g = I.Grid(ndim=3, n1=n, n2=n, n3=n, d1=d, d2=d, d3=d, nb=nb, order=8, nt=nt, dt=dt, fm=fm)
    vp, rho = I.homogeneous(3, n, d, c)
    gr = oracle.og_grid(g, vmax=c)
    ctr = nb + n // 2
    src = np.array([ctr, ctr, ctr], np.int32)
    rec = np.array([[ctr, ctr + 15, ctr], [ctr + 12, ctr + 12, ctr]], np.int32)
    out = oracle.forward(gr, vp, rho, src, I.ricker(nt, dt, fm), rec)
    t = (np.arange(nt) + 1) * dt
    for k in range(2):
        r = d * math.sqrt(float(np.sum((rec[k] - src) ** 2)))
        ref = A.green3d_trace(r, c, t, fm, 1.2 / fm, dt)
        err = np.linalg.norm(out["dcal"][:, k] - ref) / np.linalg.norm(ref)
        assert err <= 1e-2, (k, err)


# ----------------------------------------------------------------------------- P5

@pytest.mark.parametrize("ndim", [2, 3])
def test_reciprocity(oracle, ndim):
    """Swapping source and receiver: p(x_r; x_s) kappa(x_s) = p(x_s; x_r) kappa(x_r)
    (heterogeneous medium, no absorption: exact to round-off)."""
    if ndim == 2:
        g = small_grid(order=8, n1=40, n2=50, nt=250, nb=6)
        vp, rho = smooth_random_model(g.n1, g.n2, 5)
        A_, B_ = np.array([14, 15, 0], np.int32), np.array([35, 44, 0], np.int32)
    else:
        g = small_grid(order=4, n1=20, n2=22, n3=24, nt=120, nb=4, ndim=3)
        vp, rho = smooth_random_model(g.n1, g.n2, 6, n3=g.n3)
        A_, B_ = np.array([8, 9, 10, 0], np.int32)[:3], np.array([18, 20, 22], np.int32)
    gr = oracle.og_grid(g, vmax=float(vp.max()), pml=0)
    stf = I.ricker(g.nt, g.dt, g.fm)
    d_ab = oracle.forward(gr, vp, rho, A_, stf, B_[None])["dcal"][:, 0]
    d_ba = oracle.forward(gr, vp, rho, B_, stf, A_[None])["dcal"][:, 0]
    kap = lambda p: (rho.astype(np.float64) * vp.astype(np.float64) ** 2)[
        tuple(int(p[a]) - g.nb for a in range(ndim))[::-1]]
    lhs, rhs = d_ab * kap(A_), d_ba * kap(B_)
    assert np.max(np.abs(lhs - rhs)) <= 1e-12 * np.max(np.abs(lhs))
    assert np.max(np.abs(lhs)) > 0


# ----------------------------------------------------------------------------- P6

def _dot_case(oracle, pml, ndim=2, freesurf=0):
    if ndim == 2:
        g = small_grid(order=8, n1=40, n2=48, nt=220, nb=8)
        vp, rho = smooth_random_model(g.n1, g.n2, 3)
    else:
        g = small_grid(order=4, n1=18, n2=20, n3=22, nt=90, nb=4, ndim=3)
        vp, rho = smooth_random_model(g.n1, g.n2, 4, n3=g.n3)
    g.freesurf = freesurf
    gr = oracle.og_grid(g, vmax=float(vp.max()), pml=pml)
    rng = np.random.default_rng(21)
    src = np.array([g.nb + 3, g.nb + g.n2 // 3, g.nb + 5 if ndim == 3 else 0], np.int32)
    rec = np.array([[g.nb + 2, g.nb + j, g.nb + 6 if ndim == 3 else 0] for j in range(1, g.n2 - 1, 3)],
                   np.int32)
    stf = I.ricker(g.nt, g.dt, g.fm)
    dk = np.zeros(vp.shape)
    core = tuple(slice(2, s - 2) for s in vp.shape)
    dk[core] = rng.standard_normal(dk[core].shape)
    dk *= float(np.mean(rho * vp.astype(np.float64) ** 2))
    dd = oracle.born(gr, vp, rho, src, stf, rec, dk)
    G = rng.standard_normal(dd.shape)
    fw = oracle.forward(gr, vp, rho, src, stf, rec, hist=True)
    gk = oracle.adjoint(gr, vp, rho, src, stf, rec, G, hist=fw["hist"], want=("gk",))["gk"]
    lhs = float(np.sum(dd * G))
    rhs = float(np.sum(dk.ravel() * gk))
    return abs(lhs - rhs) / abs(lhs)


@pytest.mark.parametrize("ndim", [2, 3])
def test_dot_product_adjoint_exact_without_pml(oracle, ndim):
    """<L dk, d> = <dk, L* d>: the same-solver adjoint (eq. 8) with the kappa gradient of
    eq. (7) is the exact transpose of the tangent-linear map (no absorption)."""
    assert _dot_case(oracle, 0, ndim) <= 1e-12


def test_dot_product_with_cpml_is_close(oracle):
    """With CPML the same-solver adjoint is not the exact transpose; the mismatch stays at
    the level of the PML's residual reflections."""
    assert _dot_case(oracle, 1) <= 1e-4


def test_born_is_the_derivative_of_the_forward_map(oracle):
    """Central finite differences of the forward map in a kappa direction match og_born."""
    g = small_grid(order=8, n1=36, n2=44, nt=200, nb=8)
    vp, rho = smooth_random_model(g.n1, g.n2, 8)
    gr = oracle.og_grid(g, vmax=3000.0)
    rng = np.random.default_rng(3)
    src = np.array([g.nb + 3, g.nb + 20, 0], np.int32)
    rec = np.array([[g.nb + 2, g.nb + j, 0] for j in range(2, 40, 4)], np.int32)
    stf = I.ricker(g.nt, g.dt, g.fm)
    kap = rho.astype(np.float64) * vp.astype(np.float64) ** 2
    dk = np.zeros(vp.shape)
    dk[3:-3, 3:-3] = rng.standard_normal((g.n2 - 6, g.n1 - 6)) * kap[3:-3, 3:-3]
    eps = 1e-4
    vpp = np.sqrt((kap + eps * dk) / rho)
    vpm = np.sqrt((kap - eps * dk) / rho)
    dp = oracle.forward(gr, vpp, rho, src, stf, rec)["dcal"]
    dm = oracle.forward(gr, vpm, rho, src, stf, rec)["dcal"]
    fd = (dp - dm) / (2 * eps)
    born = oracle.born(gr, vp, rho, src, stf, rec, dk)
    assert np.linalg.norm(fd - born) / np.linalg.norm(born) < 1e-6


# ----------------------------------------------------------------------------- P7

@pytest.mark.parametrize("box", [0, 1])
def test_fwi_gradient_matches_finite_differences(oracle, box):
    """eq. (6)-(8): dJ/dVp from the reverse loop (reconstruction from saved boundaries,
    CPML on) against central differences of J on 20 random cells."""
    g = small_grid(order=8, n1=50, n2=70, nt=420, nb=12, fm=15.0, box=box)
    vp, rho = smooth_random_model(g.n1, g.n2, 9, vmin=1800.0, vmax=2500.0)
    vtrue = vp.astype(np.float64).copy()
    vtrue[20:40, 15:30] *= 1.08
    sx = np.array([15.0, 35.0, 55.0]) * g.d2
    acq = I._surface_line(sx, 3 * g.d1, np.arange(0, g.n2, 2) * g.d2, 2 * g.d1)
    stf = np.repeat(I.ricker(g.nt, g.dt, g.fm)[None], 3, 0)
    job = I.Job(g, vp, rho, acq, stf)
    vmax = 2800.0
    dobs = oracle.forward_job(job, vp=vtrue, vmax=vmax)
    grad, J0 = oracle.fwi_grad(job, dobs, vmax=vmax)
    grad_h, J1 = oracle.fwi_grad(job, dobs, vmax=vmax, use_history=True)
    assert abs(J0 - J1) <= 1e-13 * J0
    # plain definition (stored history) == method (boundary reconstruction)
    assert np.max(np.abs(grad - grad_h)) <= 1e-10 * np.max(np.abs(grad_h))
    rng = np.random.default_rng(1003)
    N = g.order // 2
    cand = [(ix, iz) for ix in range(2 * N, g.n2 - 2 * N) for iz in range(2 * N, g.n1 - 2 * N)
            if abs(grad[ix, iz]) >= 0.01 * np.max(np.abs(grad))]
    pick = rng.choice(len(cand), 20, replace=False)

    def J(v):
        d = oracle.forward_job(job, vp=v, vmax=vmax)
        return sum(oracle.misfit(d[s], dobs[s], g.dt)[0] for s in range(3))

    worst = 0.0
    for k in pick:
        ix, iz = cand[k]
        eps = 1e-4 * float(vp[ix, iz])
        vpl = vp.astype(np.float64).copy()
        vpl[ix, iz] += eps
        vmi = vp.astype(np.float64).copy()
        vmi[ix, iz] -= eps
        fd = (J(vpl) - J(vmi)) / (2 * eps)
        worst = max(worst, abs(fd - grad[ix, iz]) / abs(grad[ix, iz]))
    assert worst <= 1e-4, worst


def _density_case(oracle):
    g = small_grid(order=8, n1=46, n2=64, nt=400, nb=12, fm=15.0)
    vp, rho = smooth_random_model(g.n1, g.n2, 19, vmin=1800.0, vmax=2500.0)
    vtrue = vp.astype(np.float64).copy()
    rtrue = rho.astype(np.float64).copy()
    vtrue[18:36, 14:30] *= 1.06
    rtrue[10:40, 24:40] *= 1.15
    sx = np.array([14.0, 32.0, 50.0]) * g.d2
    acq = I._surface_line(sx, 3 * g.d1, np.arange(0, g.n2, 2) * g.d2, 2 * g.d1)
    stf = np.repeat(I.ricker(g.nt, g.dt, g.fm)[None], 3, 0)
    job = I.Job(g, vp, rho, acq, stf)
    vmax = 2800.0
    dobs = oracle.forward_job(I.Job(g, vtrue, rtrue, acq, stf), vmax=vmax)

    def J(v, r):
        d = oracle.forward_job(I.Job(g, v, r, acq, stf), vmax=vmax)
        return sum(oracle.misfit(d[s], dobs[s], g.dt)[0] for s in range(3))
    return g, job, dobs, vmax, J


def _fd_cells(g, grad, n, seed):
    N = g.order // 2
    cand = [(ix, iz) for ix in range(2 * N, g.n2 - 2 * N) for iz in range(2 * N, g.n1 - 2 * N)
            if abs(grad[ix, iz]) >= 0.02 * np.max(np.abs(grad))]
    rng = np.random.default_rng(seed)
    return [cand[k] for k in rng.choice(len(cand), n, replace=False)]


@pytest.mark.parametrize("family", [1, 2])
def test_density_gradient_matches_finite_differences(oracle, family):
    """eq. (7), density part, and the chain rule of Sec. 2.2: both gradients of family 1
    (Vp, rho) and family 2 (Vp, Ip = rho Vp) from one reverse loop (boundary reconstruction)
    against central differences of J on 12 cells each; the stored-history run agrees."""
    g, job, dobs, vmax, J = _density_case(oracle)
    g1, g2, J0 = oracle.fwi_grad_family(job, dobs, family, vmax=vmax)
    h1, h2, _ = oracle.fwi_grad_family(job, dobs, family, vmax=vmax, use_history=True)
    assert np.max(np.abs(g2 - h2)) <= 1e-10 * np.max(np.abs(h2))
    vp = job.vp.astype(np.float64)
    rho = job.rho.astype(np.float64)
    worst = 0.0
    for which, grad in ((1, g1), (2, g2)):
        for ix, iz in _fd_cells(g, grad, 12, 40 + 2 * family + which):
            if family == 1:
                base = vp if which == 1 else rho
            else:
                base = vp if which == 1 else rho * vp            # Ip
            eps = 1e-4 * float(base[ix, iz])
            vals = []
            for sgn in (1.0, -1.0):
                v, r = vp.copy(), rho.copy()
                if family == 1 and which == 1:
                    v[ix, iz] += sgn * eps
                elif family == 1:
                    r[ix, iz] += sgn * eps
                elif which == 1:                                  # Vp at fixed Ip
                    ip = rho[ix, iz] * vp[ix, iz]
                    v[ix, iz] += sgn * eps
                    r[ix, iz] = ip / v[ix, iz]
                else:                                             # Ip at fixed Vp
                    r[ix, iz] = (rho[ix, iz] * vp[ix, iz] + sgn * eps) / vp[ix, iz]
                vals.append(J(v, r))
            fd = (vals[0] - vals[1]) / (2 * eps)
            worst = max(worst, abs(fd - grad[ix, iz]) / abs(grad[ix, iz]))
    assert worst <= 1e-4, worst


# ----------------------------------------------------------------------------- P8, P9, P10

@pytest.mark.parametrize("ndim,box", [(2, 0), (2, 1), (3, 0), (3, 1)])
def test_reconstruction_from_saved_boundaries_is_exact(oracle, ndim, box):
    """Sec. 4.2 with dr = 1: running the step backwards on the interior with the saved
    bands restored returns the forward wavefield at every level (to round-off)."""
    if ndim == 2:
        g = small_grid(order=8, n1=48, n2=60, nt=300, nb=10, box=box)
        vp, rho = smooth_random_model(g.n1, g.n2, 13)
        src = np.array([g.nb + 4, g.nb + 25, 0], np.int32)
    else:
        g = small_grid(order=8, n1=20, n2=24, n3=22, nt=100, nb=6, ndim=3, box=box)
        vp, rho = smooth_random_model(g.n1, g.n2, 14, n3=g.n3)
        src = np.array([g.nb + 3, g.nb + 10, g.nb + 11], np.int32)
    gr = oracle.og_grid(g, vmax=float(vp.max()))
    stf = I.ricker(g.nt, g.dt, g.fm)
    levels = list(range(0, g.nt + 1, 7)) + [g.nt]
    fw = oracle.forward(gr, vp, rho, src, stf, src[None], bands=True, final=True, snaps=levels)
    rc = oracle.reconstruct(gr, vp, rho, src, stf, fw["bands"], fw["final"], levels)
    err = np.max(np.linalg.norm(rc - fw["snaps"], axis=1)) / np.max(np.linalg.norm(fw["snaps"], axis=1))
    assert err <= 1e-13, err


@pytest.mark.parametrize("bp_off,bv_off,exact", [(-1, 0, True), (0, -1, False)])
def test_minimal_band_width(oracle, bp_off, bv_off, exact):
    """N-1 planes of p and N of the face-normal v per face are the minimum for exact
    reconstruction; dropping one v plane breaks it."""
    g = small_grid(order=8, n1=40, n2=50, nt=250, nb=10)
    vp, rho = smooth_random_model(g.n1, g.n2, 15)
    N = g.order // 2
    gr = oracle.og_grid(g, vmax=float(vp.max()), band_p=N + bp_off, band_v=N + bv_off)
    src = np.array([g.nb + 4, g.nb + 20, 0], np.int32)
    stf = I.ricker(g.nt, g.dt, g.fm)
    levels = list(range(0, g.nt + 1, 10))
    fw = oracle.forward(gr, vp, rho, src, stf, src[None], bands=True, final=True, snaps=levels)
    rc = oracle.reconstruct(gr, vp, rho, src, stf, fw["bands"], fw["final"], levels)
    err = np.max(np.linalg.norm(rc - fw["snaps"], axis=1)) / np.max(np.linalg.norm(fw["snaps"], axis=1))
    if exact:
        assert err <= 1e-13, err
    else:
        assert err >= 1e-6, err


def test_computing_box_changes_nothing(oracle):
    """Sec. 4.1: the evolving box (radius ceil(vmax (it+1) dt / d) + margin around the
    source) reproduces the full-grid seismograms.  What the box cuts off is the leap-frog's
    exponentially small numerical precursor: with the default margin 2N it is far below
    FP32 resolution, with 4N at FP64 round-off, and with no margin it is visible."""
    g = small_grid(order=8, n1=60, n2=90, nt=400, nb=10)
    vp, rho = smooth_random_model(g.n1, g.n2, 16)
    src = np.array([g.nb + 3, g.nb + 30, 0], np.int32)
    rec = np.array([[g.nb + 2, g.nb + j, 0] for j in range(0, g.n2, 3)], np.int32)
    stf = I.ricker(g.nt, g.dt, g.fm)
    ref = oracle.forward(oracle.og_grid(g, vmax=float(vp.max()), box=0), vp, rho, src, stf, rec)["dcal"]
    scale = np.max(np.abs(ref))
    err = {}
    for m in (0, g.order, 2 * g.order):
        g.margin = m
        on = oracle.forward(oracle.og_grid(g, vmax=float(vp.max()), box=1), vp, rho, src, stf, rec)["dcal"]
        err[m] = np.max(np.abs(on - ref)) / scale
    assert err[g.order] <= 1e-10, err
    assert err[2 * g.order] <= 1e-14, err
    assert err[0] > 1e3 * err[g.order], err
    # the box really is smaller than the grid early on
    lo, hi = oracle.fwd_box(oracle.og_grid(g, vmax=float(vp.max()), box=1), src, 10)
    assert hi[1] - lo[1] + 1 < g.n2 + 2 * g.nb


def test_box_schedule_grows_with_wavefront(oracle):
    """Sec. 4.1 figure: the box half-width after it+1 steps is ceil(vmax (it+1) dt / d) + margin."""
    g = small_grid(order=8, n1=200, n2=300, nt=1000, nb=20, box=1)
    g.margin = 8
    gr = oracle.og_grid(g, vmax=2000.0, box=1)
    src = np.array([g.nb + 5, g.nb + 150, 0], np.int32)
    for it, t in [(49, 0.05), (99, 0.1), (149, 0.15), (199, 0.2)]:
        lo, hi = oracle.fwd_box(gr, src, it)
        half = math.ceil(2000.0 * t / g.d2 - 1e-9) + 8
        assert hi[1] - src[1] == half and src[1] - lo[1] == half
        hz = math.ceil(2000.0 * t / g.d1 - 1e-9) + 8
        assert lo[0] == max(0, src[0] - hz)  # clipped at the top of the padded grid
        assert hi[0] == min(g.n1 + 2 * g.nb - 1, src[0] + hz)


# ----------------------------------------------------------------------------- P11

def test_cpml_absorbs(oracle):
    """Sec. 2.1 (CPML, 20 layers): after two crossing times the energy left is < 1e-3 of
    its maximum, and near-boundary traces match a much larger domain to 1e-2."""
    c, n, nb, dt = 2000.0, 121, 20, 1e-3
    g = I.Grid(ndim=2, n1=n, n2=n, d1=10.0, d2=10.0, nb=nb, order=4, nt=1300, dt=dt, fm=10.0)
    vp, rho = I.homogeneous(2, n, 10.0, c)
    gr = oracle.og_grid(g, vmax=c)
    ctr = nb + n // 2
    src = np.array([ctr, ctr, 0], np.int32)
    rec = np.array([[ctr, nb + n - 3, 0], [nb + 2, ctr, 0], [nb + 5, nb + 5, 0]], np.int32)
    levels = list(range(0, g.nt + 1, 50))
    out = oracle.forward(gr, vp, rho, src, I.ricker(g.nt, dt, g.fm), rec, snaps=levels)
    e = np.sum(out["snaps"] ** 2, axis=1)
    assert e[-1] / e.max() < 1e-3
    # large domain: same source, receivers at the same offsets, boundary far away
    n2 = 3 * n
    gb = I.Grid(ndim=2, n1=n2, n2=n2, d1=10.0, d2=10.0, nb=nb, order=4, nt=700, dt=dt, fm=10.0)
    vpb, rhob = I.homogeneous(2, n2, 10.0, c)
    cb = nb + n2 // 2
    shift = cb - ctr
    srcb = src + np.array([shift, shift, 0], np.int32)
    recb = rec + np.array([shift, shift, 0], np.int32)
    outb = oracle.forward(oracle.og_grid(gb, vmax=c), vpb, rhob, srcb, I.ricker(gb.nt, dt, g.fm), recb)
    small = out["dcal"][:700]
    big = outb["dcal"]
    assert np.max(np.abs(small - big)) / np.max(np.abs(big)) < 1e-2


# ----------------------------------------------------------------------------- P15 (decimated bands)

@pytest.mark.parametrize("ndim", [2, 3])
def test_decimated_band_reconstruction(oracle, ndim):
    """Sec. 4.2 with dr > 1: the interpolation kernel is not given by the paper (parity
    unpinned).  Sanity: the error against the true field falls with dr, stays below 2e-3 at
    dr = 10 (3.3 samples per period at 2.5 fm), and every level that is a saved one is exact
    to round-off at dr = 1."""
    errs = []
    for dr in (2, 5, 10):
        if ndim == 2:
            g = small_grid(order=8, n1=60, n2=80, nt=600, nb=10, dr=dr, fm=12)
            vp, rho = smooth_random_model(g.n1, g.n2, 13)
            src = np.array([g.nb + 30, g.nb + 40, 0], np.int32)
        else:
            g = small_grid(order=8, n1=28, n2=28, n3=28, nt=180, nb=8, ndim=3, dr=dr, fm=12, d=12.5)
            vp, rho = smooth_random_model(g.n1, g.n2, 14, n3=g.n3)
            src = np.array([g.nb + 14, g.nb + 14, g.nb + 14], np.int32)
        gr = oracle.og_grid(g, vmax=float(vp.max()))
        stf = I.ricker(g.nt, g.dt, g.fm)
        levels = list(range(0, g.nt + 1, 10))
        fw = oracle.forward(gr, vp, rho, src, stf, src[None], bands=True, final=True, snaps=levels)
        rc = oracle.reconstruct(gr, vp, rho, src, stf, fw["bands"], fw["final"], levels)
        errs.append(np.max(np.linalg.norm(rc - fw["snaps"], axis=1)) / np.max(np.linalg.norm(fw["snaps"], axis=1)))
    assert errs[0] < errs[1] < errs[2] <= 2e-3, errs


def test_decimated_forward_records_the_same_data(oracle):
    """Running the forward pass past nt to save the interpolator's last levels does not
    change the seismograms of steps 0..nt-1."""
    g = small_grid(order=8, n1=40, n2=60, nt=300, nb=10, dr=10)
    vp, rho = smooth_random_model(g.n1, g.n2, 17)
    gr = oracle.og_grid(g, vmax=float(vp.max()))
    src = np.array([g.nb + 5, g.nb + 30, 0], np.int32)
    rec = np.array([[g.nb + 2, g.nb + j, 0] for j in range(0, g.n2, 5)], np.int32)
    stf = I.ricker(g.nt, g.dt, g.fm)
    a = oracle.forward(gr, vp, rho, src, stf, rec, bands=True, final=True)
    b = oracle.forward(gr, vp, rho, src, stf, rec)
    np.testing.assert_array_equal(a["dcal"], b["dcal"])
    assert a["bands"].shape[0] == (g.nt - 1) // g.dr + 4 + 1


# ----------------------------------------------------------------------------- RTM post-processing

@pytest.mark.parametrize("ndim", [2, 3])
def test_laplacian_matches_closed_forms(oracle, ndim):
    """Sec. 2.3 Laplace filter: exact (to round-off) on quadratics inside the image, and the
    discrete eigenvalue -(4/d^2) sin^2(k d / 2) on a sine that vanishes at the padding."""
    n = (7, 6, 5)[:ndim]
    d = (2.0, 3.0, 1.5)[:ndim]
    axes = [np.arange(n[a]) * d[a] for a in range(ndim)]
    grids = np.meshgrid(*axes[::-1], indexing="ij")            # numpy order (y,) x, z
    coords = grids[::-1]                                        # coords[a] for axis a
    coef = (1.0, 2.0, -0.5)[:ndim]
    f = sum(c * q * q for c, q in zip(coef, coords)) + 3.0 * coords[0]
    L = oracle.laplacian(f, d)
    inner = tuple(slice(1, -1) for _ in range(ndim))
    np.testing.assert_allclose(L[inner], 2.0 * sum(coef), rtol=0, atol=1e-9)
    # sine along z that is zero one node outside both ends (so the zero padding is exact)
    m = n[0] + 1
    k = 3 * math.pi / (m * d[0])
    s = np.sin(k * (np.arange(n[0]) + 1) * d[0])
    shape = [1] * ndim
    shape[-1] = n[0]
    g = np.broadcast_to(s.reshape(shape), f.shape).copy()
    Lg = oracle.laplacian(g, (d[0],) + (1e30,) * (ndim - 1))   # other axes: no curvature weight
    lam = -4.0 / d[0] ** 2 * math.sin(k * d[0] / 2) ** 2
    np.testing.assert_allclose(Lg, lam * g, rtol=0, atol=1e-12)


def test_normalized_image_divides_by_source_illumination(oracle):
    """Sec. 2.3 normalised imaging condition: a source twice as strong doubles each shot's
    image and quadruples its illumination (and the stabiliser, a fraction of the peak), so the
    normalised image halves; the plain image doubles.  A receiver-side normalisation would not
    scale this way."""
    g = small_grid(order=4, n1=36, n2=48, nt=260, nb=8, fm=12)
    vp, rho = smooth_random_model(g.n1, g.n2, 21)
    d = g.d1
    acq = I._surface_line(np.array([12.0, 36.0]) * d, 2 * d, np.arange(g.n2) * d, 2 * d)
    stf = np.repeat(I.ricker(g.nt, g.dt, g.fm)[None, :], 2, 0).astype(np.float32)
    vtrue = vp.copy()
    vtrue[:, 24:] *= 1.1                                        # a reflector at depth 24
    job = I.Job(g, vtrue, rho, acq, stf)
    dobs = oracle.forward_job(job)
    job = I.Job(g, vp, rho, acq, stf)
    ims, ils = oracle.rtm_image(job, dobs, per_shot=True)
    a = oracle.normalized_image(ims, ils)
    job.stf = 2.0 * job.stf
    ims2, ils2 = oracle.rtm_image(job, dobs, per_shot=True)
    b = oracle.normalized_image(ims2, ils2)
    assert np.max(np.abs(b - 0.5 * a)) <= 1e-12 * np.max(np.abs(a))
    assert np.max(np.abs(np.sum(ims2, 0) - 2.0 * np.sum(ims, 0))) <= 1e-12 * np.max(np.abs(np.sum(ims, 0)))
    assert np.max(np.abs(a)) > 0


# ----------------------------------------------------------------------------- off-grid operators

@pytest.mark.parametrize("r,tol", [(2, 2.5e-2), (4, 1.5e-3)])
def test_windowed_sinc_interpolates_band_limited_signals(oracle, r, tol):
    """Sec. 2.1 point operators (Kaiser-windowed sinc, half-width r = order/2): cosines up to
    half the Nyquist wavenumber are interpolated at off-grid points to the stated accuracy; a
    point on a node is that node with weight 1."""
    rng = np.random.default_rng(40 + r)
    worst = 0.0
    for _ in range(100):
        u = 30.0 + rng.uniform(0.01, 0.99)
        nodes, w = oracle.hicks_weights_1d(u, r, 100)
        assert len(nodes) == 2 * r
        for kd in np.linspace(0.05, math.pi / 2, 12):
            ph = rng.uniform(0, 2 * math.pi)
            est = sum(wi * math.cos(kd * j + ph) for j, wi in zip(nodes, w))
            worst = max(worst, abs(est - math.cos(kd * u + ph)))
    assert worst <= tol, worst
    assert oracle.hicks_weights_1d(41.0, r, 100) == ([41], [1.0])


@pytest.mark.parametrize("ndim", [2, 3])
def test_reciprocity_with_off_grid_points(oracle, ndim):
    """Homogeneous medium, no absorption: a source at A recorded at B equals a source at B
    recorded at A when both points are off the grid (injection is the transpose of sampling)."""
    if ndim == 2:
        g = small_grid(order=8, n1=40, n2=50, nt=220, nb=6)
        A_, B_ = (62.3, 71.8, 0.0), (251.7, 333.4, 0.0)
    else:
        g = small_grid(order=4, n1=22, n2=22, n3=22, nt=110, nb=4, ndim=3)
        A_, B_ = (61.2, 78.9, 83.3), (151.6, 163.7, 141.1)
    vp, rho = I.homogeneous(ndim, g.n1, g.d1, 2200.0)
    if ndim == 2:
        vp, rho = np.full((g.n2, g.n1), 2200.0, np.float32), np.full((g.n2, g.n1), 1800.0, np.float32)
    gr = oracle.og_grid(g, vmax=2200.0, pml=0)
    stf = I.ricker(g.nt, g.dt, g.fm)

    def run(S, R):
        st = oracle.point_taps(g, [S])
        rt = oracle.point_taps(g, [R])
        assert len(st.w) == (2 * (g.order // 2)) ** ndim
        src = oracle.node(g, S)
        rec = oracle.node(g, R)[None]
        return oracle.forward(gr, vp, rho, src, stf, rec, st=st, rt=rt)["dcal"][:, 0]
    ab, ba = run(A_, B_), run(B_, A_)
    assert np.max(np.abs(ab - ba)) <= 1e-12 * np.max(np.abs(ab))
    assert np.max(np.abs(ab)) > 0


def test_off_grid_source_matches_the_green_function(oracle):
    """2D homogeneous medium, order 8: a source between nodes, recorded 310 m away with the
    windowed-sinc operators, matches the analytic trace at the true distance; rounding source
    and receiver to their nearest nodes (320 m apart) is several times worse."""
    from oracle import analytic as A
    n, nb, c, fm, dt = 181, 20, 2000.0, 10.0, 1e-3
    nt = 450
    g = I.Grid(ndim=2, n1=n, n2=n, d1=10.0, d2=10.0, nb=nb, order=8, nt=nt, dt=dt, fm=fm)
    vp, rho = I.homogeneous(2, n, 10.0, c)
    gr = oracle.og_grid(g, vmax=c)
    S = (903.0, 905.0, 0.0)                 # between nodes in z and x
    R = (903.0, 1215.0, 0.0)                # 310 m along x, off-grid too; the nearest nodes
                                            # are 320 m apart
    st, rt = oracle.point_taps(g, [S]), oracle.point_taps(g, [R])
    t = (np.arange(nt) + 1) * dt
    ref = A.green2d_trace(310.0, c, t, fm, 1.2 / fm, dt, ntau=20000)
    stf = I.ricker(nt, dt, fm)
    d = oracle.forward(gr, vp, rho, oracle.node(g, S), stf, oracle.node(g, R)[None], st=st, rt=rt)["dcal"][:, 0]
    e_op = np.linalg.norm(d - ref) / np.linalg.norm(ref)
    d0 = oracle.forward(gr, vp, rho, oracle.node(g, S), stf, oracle.node(g, R)[None])["dcal"][:, 0]
    e_node = np.linalg.norm(d0 - ref) / np.linalg.norm(ref)
    assert e_op <= 1.5e-2 and e_node >= 3 * e_op, (e_op, e_node)


def test_gradient_with_off_grid_points_matches_finite_differences(oracle):
    """eq. (6)-(8) with sources and receivers off the grid: the adjoint source is injected
    with the transpose of the receivers' sampling operator, so dJ/dVp still matches central
    differences of J (10 cells).  Every operator's nodes lie in the interior: where they
    reach into the CPML the same-solver adjoint is not the exact transpose (the level of the
    dot-product test with CPML, 1e-4)."""
    g = small_grid(order=8, n1=44, n2=60, nt=380, nb=12, fm=15.0)
    vp, rho = smooth_random_model(g.n1, g.n2, 23, vmin=1800.0, vmax=2500.0)
    vtrue = vp.astype(np.float64).copy()
    vtrue[18:36, 14:30] *= 1.08
    sx = (np.array([14.0, 33.0, 47.0]) + 0.37) * g.d2
    acq = I._surface_line(sx, 3.6 * g.d1, (np.arange(6, 54, 2) + 0.5) * g.d2, 4.3 * g.d1)
    stf = np.repeat(I.ricker(g.nt, g.dt, g.fm)[None], 3, 0)
    job = I.Job(g, vp, rho, acq, stf)
    assert oracle.shot_ops(g, acq, 0)[2] is not None and oracle.shot_ops(g, acq, 0)[3] is not None
    vmax = 2800.0
    dobs = oracle.forward_job(job, vp=vtrue, vmax=vmax)
    grad, J0 = oracle.fwi_grad(job, dobs, vmax=vmax)

    def J(v):
        d = oracle.forward_job(job, vp=v, vmax=vmax)
        return sum(oracle.misfit(d[s], dobs[s], g.dt)[0] for s in range(3))
    worst = 0.0
    for ix, iz in _fd_cells(g, grad, 10, 77):
        eps = 1e-4 * float(vp[ix, iz])
        vpl = vp.astype(np.float64).copy()
        vpl[ix, iz] += eps
        vmi = vp.astype(np.float64).copy()
        vmi[ix, iz] -= eps
        fd = (J(vpl) - J(vmi)) / (2 * eps)
        worst = max(worst, abs(fd - grad[ix, iz]) / abs(grad[ix, iz]))
    assert worst <= 1e-4, worst


# ----------------------------------------------------------------------------- free surface

def test_free_surface_matches_the_image_source(oracle):
    """Sec. 2.1 free surface (image method): in a homogeneous half-space the trace is the
    direct wave minus the wave of the image source mirrored above the surface,
    G(r1) - G(r2); the pressure-release sign, the surface position and the v_z symmetry all
    enter.  Without the surface (absorbing top) the ghost is absent and the error is large."""
    from oracle import analytic as A
    n1, n2, nb, c, fm, dt, d = 120, 201, 20, 2000.0, 10.0, 1e-3, 10.0
    nt = 500
    t = (np.arange(nt) + 1) * dt
    zs, zr, off = 100.0, 50.0, 300.0
    r1 = math.hypot(off, zr - zs)
    r2 = math.hypot(off, zr + zs)
    ref = (A.green2d_trace(r1, c, t, fm, 1.2 / fm, dt, ntau=20000)
           - A.green2d_trace(r2, c, t, fm, 1.2 / fm, dt, ntau=20000))
    errs = []
    for fs in (1, 0):
        g = I.Grid(ndim=2, n1=n1, n2=n2, d1=d, d2=d, nb=nb, order=8, nt=nt, dt=dt, fm=fm,
                   freesurf=fs)
        vp = np.full((n2, n1), c, np.float32)
        rho = np.full((n2, n1), 1000.0, np.float32)
        gr = oracle.og_grid(g, vmax=c)
        xs = 60
        src = np.array([nb + int(zs / d), nb + xs, 0], np.int32)
        rec = np.array([[nb + int(zr / d), nb + xs + int(off / d), 0]], np.int32)
        out = oracle.forward(gr, vp, rho, src, I.ricker(nt, dt, fm), rec)["dcal"][:, 0]
        errs.append(np.linalg.norm(out - ref) / np.linalg.norm(ref))
    assert errs[0] <= 1.5e-2 and errs[1] >= 0.3, errs


@pytest.mark.parametrize("ndim", [2, 3])
def test_free_surface_reconstruction_is_exact(oracle, ndim):
    """Sec. 4.2 with a free surface: the bands above the surface are the mirror images and the
    rebuilt p vanishes on the surface, so the reconstruction is still exact."""
    if ndim == 2:
        g = small_grid(order=8, n1=40, n2=50, nt=260, nb=10)
        vp, rho = smooth_random_model(g.n1, g.n2, 51)
        src = np.array([g.nb + 3, g.nb + 25, 0], np.int32)
    else:
        g = small_grid(order=4, n1=18, n2=20, n3=20, nt=100, nb=5, ndim=3)
        vp, rho = smooth_random_model(g.n1, g.n2, 52, n3=g.n3)
        src = np.array([g.nb + 2, g.nb + 10, g.nb + 9], np.int32)
    g.freesurf = 1
    gr = oracle.og_grid(g, vmax=float(vp.max()))
    stf = I.ricker(g.nt, g.dt, g.fm)
    levels = list(range(0, g.nt + 1, 9)) + [g.nt]
    fw = oracle.forward(gr, vp, rho, src, stf, src[None], bands=True, final=True, snaps=levels)
    rc = oracle.reconstruct(gr, vp, rho, src, stf, fw["bands"], fw["final"], levels)
    err = np.max(np.linalg.norm(rc - fw["snaps"], axis=1)) / np.max(np.linalg.norm(fw["snaps"], axis=1))
    assert err <= 1e-13, err
    assert np.max(np.abs(fw["snaps"][-1].reshape(vp.shape)[..., 0])) == 0.0   # p = 0 on the surface


def test_free_surface_gradient_matches_finite_differences(oracle):
    """eq. (6)-(8) with a free surface: the same-solver adjoint with the same mirroring is the
    transpose of the forward map; dJ/dVp against central differences on 10 cells."""
    g = small_grid(order=8, n1=40, n2=56, nt=360, nb=12, fm=15.0)
    g.freesurf = 1
    vp, rho = smooth_random_model(g.n1, g.n2, 53, vmin=1800.0, vmax=2500.0)
    vtrue = vp.astype(np.float64).copy()
    vtrue[14:34, 12:26] *= 1.08
    sx = np.array([12.0, 28.0, 44.0]) * g.d2
    acq = I._surface_line(sx, 3 * g.d1, np.arange(2, g.n2 - 2, 2) * g.d2, 1 * g.d1)
    stf = np.repeat(I.ricker(g.nt, g.dt, g.fm)[None], 3, 0)
    job = I.Job(g, vp, rho, acq, stf)
    vmax = 2800.0
    dobs = oracle.forward_job(job, vp=vtrue, vmax=vmax)
    grad, _ = oracle.fwi_grad(job, dobs, vmax=vmax)
    grad_h, _ = oracle.fwi_grad(job, dobs, vmax=vmax, use_history=True)
    assert np.max(np.abs(grad - grad_h)) <= 1e-10 * np.max(np.abs(grad_h))

    def J(v):
        d = oracle.forward_job(job, vp=v, vmax=vmax)
        return sum(oracle.misfit(d[s], dobs[s], g.dt)[0] for s in range(3))
    worst = 0.0
    for ix, iz in _fd_cells(g, grad, 10, 91):
        eps = 1e-4 * float(vp[ix, iz])
        a = vp.astype(np.float64).copy()
        a[ix, iz] += eps
        b = vp.astype(np.float64).copy()
        b[ix, iz] -= eps
        fd = (J(a) - J(b)) / (2 * eps)
        worst = max(worst, abs(fd - grad[ix, iz]) / abs(grad[ix, iz]))
    assert worst <= 1e-4, worst


@pytest.mark.parametrize("ndim", [2, 3])
def test_dot_product_with_free_surface_is_exact(oracle, ndim):
    """<L dk, d> = <dk, L* d> with the image-method surface (no absorption elsewhere): the
    adjoint sources near the surface receive their images like the forward sources, and the
    same solver is then the exact transpose."""
    assert _dot_case(oracle, 0, ndim, freesurf=1) <= 1e-12


# ----------------------------------------------------------------------------- P16

def test_literal_gradient_position_differs_only_at_receiver_cells(oracle):
    """Reading of the gradient time pairing (Alg. 2 writes the gradient after both updates of
    an iteration): taking it there pairs p~ before the next adjoint injection, and the sum
    over the iterations differs from the exact pairing (p~ right after its own injection) only
    at the receiver cells: bitwise equal everywhere else with the stored history; with the
    reconstruction from bands the literal sum also takes p~^0 times the rebuilt v^{-1/2}, which
    is zero up to the reconstruction's rounding."""
    g = small_grid(order=4, n1=40, n2=56, nt=300, nb=10, fm=15.0)
    vp, rho = smooth_random_model(g.n1, g.n2, 31, vmin=1800.0, vmax=2500.0)
    sx = np.array([28.0]) * g.d2
    acq = I._surface_line(sx, 3 * g.d1, np.arange(4, g.n2 - 4, 3) * g.d2, 5 * g.d1)
    stf = I.ricker(g.nt, g.dt, g.fm)
    gr = oracle.og_grid(g, vmax=2600.0)
    src, rec = oracle.shot_nodes(g, acq, 0)
    fw = oracle.forward(gr, vp, rho, src, stf, rec, hist=True, bands=True, final=True)
    G = g.dt * fw["dcal"] * np.linspace(0.5, 1.5, rec.shape[0])[None, :]
    nb = g.nb
    onrec = np.zeros((g.n2, g.n1), bool)
    onrec[rec[:, 1] - nb, rec[:, 0] - nb] = True
    for kw in ({"hist": fw["hist"]}, {"bands": fw["bands"], "final": fw["final"]}):
        ex = oracle.adjoint(gr, vp, rho, src, stf, rec, G, want=("gk",), **kw)["gk"]
        li = oracle.adjoint(gr, vp, rho, src, stf, rec, G, want=("gk",), literal=True, **kw)["gk"]
        ex, li = ex.reshape(g.n2, g.n1), li.reshape(g.n2, g.n1)
        if "hist" in kw:
            np.testing.assert_array_equal(ex[~onrec], li[~onrec])
        else:
            assert np.max(np.abs(ex[~onrec] - li[~onrec])) <= 1e-12 * np.abs(ex).max()
        d = np.abs(ex[onrec] - li[onrec])
        assert np.all(d > 0) and d.max() > 1e-3 * np.abs(ex).max()


# ----------------------------------------------------------------------------- eq. (10) image

def _image_case(oracle, ndim, pml, box=0, off_grid=False):
    """A small heterogeneous job with a reflector, its forward history, its bands and an
    adjoint source G; returns everything the image pins need."""
    if ndim == 2:
        g = small_grid(order=8, n1=40, n2=48, nt=220, nb=8, box=box)
        vp, rho = smooth_random_model(g.n1, g.n2, 31)
        vp[:, 22:] *= 1.08
    else:
        g = small_grid(order=4, n1=18, n2=20, n3=22, nt=90, nb=4, ndim=3, box=box)
        vp, rho = smooth_random_model(g.n1, g.n2, 32, n3=g.n3)
        vp[..., 10:] *= 1.08
    gr = oracle.og_grid(g, vmax=float(vp.max()), pml=pml)
    src = np.array([g.nb + 3, g.nb + g.n2 // 3, g.nb + 5 if ndim == 3 else 0], np.int32)
    rec = np.array([[g.nb + 2, g.nb + j, g.nb + 6 if ndim == 3 else 0]
                    for j in range(1, g.n2 - 1, 3)], np.int32)
    rt = None
    if off_grid:   # receivers 0.37 / 0.61 of a cell off the nodes (Kaiser-windowed sinc)
        pos = [((r[0] - g.nb + 0.37) * g.d1, (r[1] - g.nb + 0.61) * g.d2, 0.0) for r in rec]
        rt = oracle.point_taps(g, pos)
    stf = I.ricker(g.nt, g.dt, g.fm)
    rng = np.random.default_rng(41 + ndim)
    G = rng.standard_normal((g.nt, len(rec)))
    dm = np.zeros(vp.shape)
    core = tuple(slice(2, s - 2) for s in vp.shape)
    dm[core] = rng.standard_normal(dm[core].shape)
    fw = oracle.forward(gr, vp, rho, src, stf, rec, hist=True, bands=True, final=True, rt=rt)
    return g, gr, vp, rho, src, rec, stf, G, dm, fw, rt


def test_image_map_is_the_derivative_of_the_reaction_forward(oracle):
    """The map of og_react (data of a field driven by dt kappa m p^it before every step) is the
    derivative of the forward run whose steps start with p *= 1 + eps dt kappa m: central
    finite differences of the second match the first."""
    g, gr, vp, rho, src, rec, stf, G, dm, fw, rt = _image_case(oracle, 2, pml=1)
    lin = oracle.react(gr, vp, rho, src, stf, rec, dm, lin=True)
    kmax = float(np.max(rho.astype(np.float64) * vp.astype(np.float64) ** 2))
    eps = 1e-5 / (g.dt * kmax)            # |eps dt kappa m| ~ 1e-5 of p per step
    dp = oracle.react(gr, vp, rho, src, stf, rec, dm, eps=eps, lin=False)
    dn = oracle.react(gr, vp, rho, src, stf, rec, dm, eps=-eps, lin=False)
    fd = (dp - dn) / (2 * eps)
    assert np.linalg.norm(lin) > 0
    assert np.linalg.norm(fd - lin) / np.linalg.norm(lin) < 1e-5
    # eps = 0 is the plain forward run
    d0 = oracle.react(gr, vp, rho, src, stf, rec, dm, eps=0.0, lin=False)
    np.testing.assert_allclose(d0, fw["dcal"], rtol=0, atol=1e-14 * np.max(np.abs(fw["dcal"])))


def _image_dot(oracle, case, planted=0, use_history=True):
    g, gr, vp, rho, src, rec, stf, G, dm, fw, rt = case
    lin = oracle.react(gr, vp, rho, src, stf, rec, dm, lin=True, rt=rt)
    if use_history:
        im = oracle.adjoint(gr, vp, rho, src, stf, rec, G, hist=fw["hist"], want=("image",),
                            rt=rt, planted=planted)["image"]
    else:
        im = oracle.adjoint(gr, vp, rho, src, stf, rec, G, bands=fw["bands"], final=fw["final"],
                            want=("image",), rt=rt, planted=planted)["image"]
    lhs = float(np.sum(lin * G))
    rhs = float(np.sum(dm.ravel() * im))
    return abs(lhs - rhs) / abs(lhs)


@pytest.mark.parametrize("ndim,off_grid", [(2, False), (2, True), (3, False)])
def test_image_is_the_exact_transpose_of_the_reaction_map(oracle, ndim, off_grid):
    """eq. (10) as the oracle pairs it: <L m, G> = <m, I(G)> with L the map of og_react and
    I(G) the image of adjoint source G, exact without absorption, from the stored history and
    from the boundary reconstruction alike."""
    case = _image_case(oracle, ndim, pml=0, off_grid=off_grid)
    assert _image_dot(oracle, case, use_history=True) <= 1e-12
    assert _image_dot(oracle, case, use_history=False) <= 1e-12


@pytest.mark.parametrize("planted", [1, 2])
def test_image_pin_catches_planted_slips(oracle, planted):
    """The transpose identity above fails for the image paired one level early (the adjoint
    field before its step) and for the image without its factor dt."""
    case = _image_case(oracle, 2, pml=0)
    assert _image_dot(oracle, case, planted=planted) > 1e-3


@pytest.mark.parametrize("ndim,box", [(2, 0), (2, 1), (3, 1)])
def test_image_and_illumination_from_history_equal_reconstructed(oracle, ndim, box):
    """With the absorbing layers on, the image and the source illumination from the boundary
    reconstruction equal those from the stored forward history; the illumination equals its
    plain definition dt sum_{it < nt} (p^it)^2 read off that history (p at levels 0..nt-1)."""
    g, gr, vp, rho, src, rec, stf, G, dm, fw, rt = _image_case(oracle, ndim, pml=1, box=box)
    a = oracle.adjoint(gr, vp, rho, src, stf, rec, G, hist=fw["hist"], want=("image", "illum"))
    b = oracle.adjoint(gr, vp, rho, src, stf, rec, G, bands=fw["bands"], final=fw["final"],
                       want=("image", "illum"))
    for key in ("image", "illum"):
        assert np.max(np.abs(a[key])) > 0
        assert np.max(np.abs(a[key] - b[key])) <= 1e-12 * np.max(np.abs(a[key])), key
    shape = [gr.n1 + 2 * gr.nb, gr.n2 + 2 * gr.nb] + ([gr.n3 + 2 * gr.nb] if ndim == 3 else [])
    hist_p = fw["hist"][:, 0, :].reshape([g.nt + 1] + shape[::-1])
    inner = (slice(None),) + tuple(slice(g.nb, s - g.nb) for s in shape[::-1])
    p_int = hist_p[inner].reshape(g.nt + 1, -1)
    plain = g.dt * np.sum(p_int[:g.nt] ** 2, axis=0)
    assert np.max(np.abs(b["illum"] - plain)) <= 1e-12 * np.max(plain)
    late = g.dt * np.sum(p_int[1:] ** 2, axis=0)      # levels 1..nt: a one-level slip
    assert np.max(np.abs(late - plain)) > 1e-6 * np.max(plain)


def test_normalized_image_is_per_shot(oracle):
    """Sec. 2.3 normalisation is per shot: with shot 0's wavelet doubled and shot 1's kept,
    the normalised image is N0 / 2 + N1 (Ns: shot s's own normalised image), which a
    normalisation by the illumination summed over shots does not give."""
    g = small_grid(order=4, n1=36, n2=48, nt=260, nb=8, fm=12)
    vp, rho = smooth_random_model(g.n1, g.n2, 22)
    d = g.d1
    acq = I._surface_line(np.array([12.0, 36.0]) * d, 2 * d, np.arange(g.n2) * d, 2 * d)
    w = I.ricker(g.nt, g.dt, g.fm)
    stf = np.stack([w, w]).astype(np.float32)
    vtrue = vp.copy()
    vtrue[:, 24:] *= 1.1
    dobs = oracle.forward_job(I.Job(g, vtrue, rho, acq, stf))
    job = I.Job(g, vp, rho, acq, stf)
    ims, ils = oracle.rtm_image(job, dobs, per_shot=True)
    n0 = oracle.normalized_image(ims[:1], ils[:1])
    n1 = oracle.normalized_image(ims[1:], ils[1:])
    job.stf = np.stack([2.0 * w, w]).astype(np.float32)
    ims2, ils2 = oracle.rtm_image(job, dobs, per_shot=True)
    got = oracle.normalized_image(ims2, ils2)
    want = 0.5 * n0 + n1
    assert np.max(np.abs(got - want)) <= 1e-12 * np.max(np.abs(want))
    summed = np.sum(ims2, 0) / (np.sum(ils2, 0) + 1e-3 * np.max(np.sum(ils2, 0)))
    assert np.max(np.abs(summed - want)) > 1e-3 * np.max(np.abs(want))


def test_reverse_loop_snapshots_equal_the_reconstruction(oracle):
    """The source field the reverse loop holds at each level (the snapshots of og_adjoint) is
    the field og_reconstruct rebuilds from the same bands, and, with dr = 1, the forward field
    itself to rounding."""
    g, gr, vp, rho, src, rec, stf, G, dm, fw, rt = _image_case(oracle, 2, pml=1, box=1)
    levels = [0, 40, 110, g.nt - 1, g.nt]
    a = oracle.adjoint(gr, vp, rho, src, stf, rec, G, bands=fw["bands"], final=fw["final"],
                       want=("image",), snaps=levels)["snaps"]
    b = oracle.reconstruct(gr, vp, rho, src, stf, fw["bands"], fw["final"], levels)
    np.testing.assert_array_equal(a, b)
    f = oracle.forward(gr, vp, rho, src, stf, rec, snaps=levels)["snaps"]
    assert np.max(np.abs(a - f)) <= 1e-12 * np.max(np.abs(f))
