"""Nonlinear FWI driver (Alg. 1, Sec. 2.2 and 3.7): bounded L-BFGS with a Wolfe line search,
parametrisation families with log-transformed variables, bathymetry mask, data weighting,
and the batchwise stochastic-gradient schedule over shuffled shots (Sec. 5).

The misfit and gradient of every trial model come from one call of the library (forward with
boundary saving, then the reverse loop); the optimiser itself is vector arithmetic on device
tensors.  The optimiser works on any `fg(x) -> (J, grad)` over torch tensors, so its logic is
tested on the CPU with analytic functions.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Callable, List, Optional, Sequence, Tuple

import numpy as np
import torch


# ----------------------------------------------------------------------------- optimiser

@dataclasses.dataclass
class LbfgsConfig:
    niter: int = 20          # nonlinear iterations
    nls: int = 20            # trial steps per line search
    npair: int = 5           # memory length
    c1: float = 1e-4         # sufficient decrease (Armijo)
    c2: float = 0.9          # curvature (weak Wolfe)
    first_step: float = 0.01  # first trial: the largest component of the update, in x units
    gtol: float = 0.0        # stop when |grad|_inf falls below gtol * |grad_0|_inf


@dataclasses.dataclass
class History:
    J: List[float] = dataclasses.field(default_factory=list)
    gnorm: List[float] = dataclasses.field(default_factory=list)
    steps: List[float] = dataclasses.field(default_factory=list)
    nfg: int = 0


def _dot(a: torch.Tensor, b: torch.Tensor) -> float:
    return float(torch.dot(a.reshape(-1).double(), b.reshape(-1).double()))


def two_loop(g: torch.Tensor, pairs: Sequence[Tuple[torch.Tensor, torch.Tensor]]) -> torch.Tensor:
    """L-BFGS two-loop recursion: H g with H built from the stored (s, y) pairs (oldest first)
    and the initial scaling gamma = s'y / y'y of the newest pair."""
    q = g.clone()
    alphas = []
    for s, y in reversed(pairs):
        rho = 1.0 / _dot(y, s)
        a = rho * _dot(s, q)
        q -= a * y
        alphas.append((rho, a))
    if pairs:
        s, y = pairs[-1]
        q *= _dot(s, y) / _dot(y, y)
    for (s, y), (rho, a) in zip(pairs, reversed(alphas)):
        b = rho * _dot(y, q)
        q += (a - b) * s
    return q


def project(x: torch.Tensor, lo: Optional[torch.Tensor], hi: Optional[torch.Tensor]) -> torch.Tensor:
    if lo is not None:
        x = torch.maximum(x, lo)
    if hi is not None:
        x = torch.minimum(x, hi)
    return x


def wolfe_search(fg, x, J0, g0, d, alpha, cfg: LbfgsConfig, lo=None, hi=None, hist=None,
                 armijo_only: bool = False):
    """Line search along d from x for a step satisfying the weak Wolfe conditions (with the
    trial point projected on the bounds): bracketing by doubling, then bisection; with
    armijo_only, the first step of sufficient decrease (halving until found).  Returns
    (alpha, x_new, J_new, g_new) -- the best decreasing trial if the budget runs out -- or None
    when no trial decreased J."""
    slope = _dot(g0, d)
    if slope >= 0:
        return None
    lo_a, hi_a = 0.0, math.inf
    best = None
    for _ in range(cfg.nls):
        xt = project(x + alpha * d, lo, hi)
        Jt, gt = fg(xt)
        if hist is not None:
            hist.nfg += 1
        if Jt < J0 and (best is None or Jt < best[2]):
            best = (alpha, xt, Jt, gt)
        if Jt > J0 + cfg.c1 * alpha * slope:
            hi_a = alpha                       # too long: shrink
        elif not armijo_only and _dot(gt, d) < cfg.c2 * slope:
            lo_a = alpha                       # too short: grow
        else:
            return alpha, xt, Jt, gt
        alpha = 0.5 * (lo_a + hi_a) if math.isfinite(hi_a) else 2.0 * alpha
    return best


def lbfgs(fg: Callable[[torch.Tensor], Tuple[float, torch.Tensor]], x0: torch.Tensor,
          cfg: LbfgsConfig = LbfgsConfig(), lo=None, hi=None, callback=None):
    """Bounded L-BFGS (Alg. 1): descent direction from the two-loop recursion, step from the
    Wolfe line search, update m_k = m_{k-1} + alpha dm (projected on [lo, hi]).  Returns
    (x, history)."""
    hist = History()
    x = project(x0.clone(), lo, hi)
    J, g = fg(x)
    hist.nfg += 1
    hist.J.append(float(J))
    g0n = float(g.abs().max())
    hist.gnorm.append(g0n)
    pairs: List[Tuple[torch.Tensor, torch.Tensor]] = []
    for k in range(cfg.niter):
        d = -two_loop(g, pairs)
        if _dot(d, g) >= 0:                    # not a descent direction: restart
            pairs.clear()
            d = -g
        alpha = 1.0 if pairs else cfg.first_step / max(float(d.abs().max()), 1e-300)
        res = wolfe_search(fg, x, J, g, d, alpha, cfg, lo, hi, hist)
        if res is None:
            break
        alpha, xn, Jn, gn = res
        s, y = xn - x, gn - g
        if _dot(s, y) > 1e-12 * math.sqrt(_dot(s, s) * _dot(y, y)):
            pairs.append((s, y))
            if len(pairs) > cfg.npair:
                pairs.pop(0)
        x, J, g = xn, Jn, gn
        hist.J.append(float(J))
        hist.gnorm.append(float(g.abs().max()))
        hist.steps.append(alpha)
        if callback is not None:
            callback(k, x, J)
        if cfg.gtol > 0 and hist.gnorm[-1] <= cfg.gtol * g0n:
            break
    return x, hist


# ----------------------------------------------------------------------------- FWI problem

@dataclasses.dataclass
class Bounds:
    vpmin: float = 1000.0
    vpmax: float = 7000.0
    rhomin: float = 500.0
    rhomax: float = 3500.0


class FwiProblem:
    """Misfit and gradient of a multi-shot job for a parametrisation family, in the
    log-transformed variables x = ln(m) (Sec. 3.7: bounds act on the transformed variables).

    family 1 inverts (Vp, rho), family 2 (Vp, Ip = rho Vp); npar = 1 inverts Vp alone with the
    second parameter of the family held fixed.  `mask` (n1*n2[*n3], 0 above the seafloor) zeroes
    the gradient where the model must not change (bathymetry); `weights` (layout of the data)
    weights the residual: J = 1/2 dt sum (w (dcal - dobs))^2.
    """

    def __init__(self, ctx, job, dobs: torch.Tensor, *, family: int = 1, npar: int = 1,
                 bounds: Bounds = Bounds(), mask: Optional[torch.Tensor] = None,
                 weights: Optional[torch.Tensor] = None, shots: Optional[Sequence[int]] = None):
        from . import binding as B
        import copy
        self.B = B
        self.ctx = ctx
        self.job = job
        # the model moves between the bounds: the stability checks, the CPML and the
        # computing box use the bounds' speed range
        self.grid = copy.copy(job.grid)
        self.grid.vpmin = float(bounds.vpmin)
        self.grid.vpmax = float(bounds.vpmax)
        self.family = family
        self.npar = npar
        self.bounds = bounds
        self.dev = dobs.device
        self.n = job.vp.size
        self.mask = None if mask is None else mask.reshape(-1).float()
        self.set_shots(shots, dobs, weights)
        self.rho0 = torch.from_numpy(np.ascontiguousarray(job.rho, np.float32)).reshape(-1).to(self.dev)
        self.stf_all = torch.from_numpy(np.ascontiguousarray(job.stf, np.float32)).to(self.dev)

    def set_shots(self, shots, dobs, weights=None):
        """Restrict the problem to a subset of the shots (dobs / weights: full layout)."""
        acq = self.job.acq
        self.all_shots = list(range(acq.nshot))
        self.shots = self.all_shots if shots is None else list(shots)
        nt = self.job.grid.nt
        off = np.asarray(acq.rec_off)
        self.sub = acq.subset(self.shots) if shots is not None else acq
        idx = np.concatenate([np.arange(nt * off[s], nt * off[s + 1]) for s in self.shots])
        ii = torch.from_numpy(idx).to(dobs.device)
        self.dobs = dobs.reshape(-1)[ii].contiguous()
        self.w = None if weights is None else weights.reshape(-1)[ii].contiguous()
        self._dobs_full, self._w_full = dobs, weights

    # model <-> variables
    def to_x(self, vp: torch.Tensor, rho: torch.Tensor) -> torch.Tensor:
        m2 = rho if self.family == 1 else rho * vp
        xs = [torch.log(vp.reshape(-1).double())]
        if self.npar == 2:
            xs.append(torch.log(m2.reshape(-1).double()))
        return torch.cat(xs)

    def to_model(self, x: torch.Tensor) -> Tuple[torch.Tensor, torch.Tensor]:
        vp = torch.exp(x[: self.n]).float()
        if self.npar == 2:
            m2 = torch.exp(x[self.n:]).float()
            rho = m2 if self.family == 1 else m2 / vp
        else:
            rho = self.rho0
        return vp, rho

    def x_bounds(self):
        b = self.bounds
        lo = [torch.full((self.n,), math.log(b.vpmin), dtype=torch.float64, device=self.dev)]
        hi = [torch.full((self.n,), math.log(b.vpmax), dtype=torch.float64, device=self.dev)]
        if self.npar == 2:
            if self.family == 1:
                lo.append(torch.full((self.n,), math.log(b.rhomin), dtype=torch.float64, device=self.dev))
                hi.append(torch.full((self.n,), math.log(b.rhomax), dtype=torch.float64, device=self.dev))
            else:
                lo.append(torch.full((self.n,), math.log(b.rhomin * b.vpmin), dtype=torch.float64, device=self.dev))
                hi.append(torch.full((self.n,), math.log(b.rhomax * b.vpmax), dtype=torch.float64, device=self.dev))
        return torch.cat(lo), torch.cat(hi)

    def __call__(self, x: torch.Tensor):
        """(J, dJ/dx) at x."""
        B = self.B
        vp, rho = self.to_model(x)
        g = self.grid
        stf = self.stf_all[self.shots].contiguous()
        self.ctx.set_option(B.OPT_FAMILY, self.family)
        want2 = self.npar == 2 or self.family == 2
        if self.w is None:
            out = self.ctx.fwi_grad(g, self.sub, vp, rho, stf, self.dobs, rho_grad=want2)
            g1, g2, Jt = (out[0], out[1], out[2]) if want2 else (out[0], None, out[1])
            J = float(Jt.cpu()[0])
        else:
            dcal, _, state = self.ctx.forward(g, self.sub, vp, rho, stf, save=True)
            r = self.w * (dcal - self.dobs)
            J = 0.5 * g.dt * float(torch.sum(r.double() * r.double()))
            G = (g.dt * self.w * r).contiguous()
            res = self.ctx.adjoint_reconstruct(state, G, grad=True, grad_rho=want2, image=False,
                                               illum=False)
            g1, g2 = res["grad"], res["grad_rho"]
        self.ctx.set_option(B.OPT_FAMILY, 1)
        m1 = vp
        gx = [(g1 * m1).double()]                      # dJ/d ln(m) = m dJ/dm
        if self.npar == 2:
            m2 = rho if self.family == 1 else rho * vp
            gx.append((g2 * m2).double())
        if self.mask is not None:
            gx = [q * self.mask.double() for q in gx]
        return J, torch.cat(gx)


def invert(ctx, job, dobs, *, family=1, npar=1, cfg: LbfgsConfig = LbfgsConfig(),
           bounds: Bounds = Bounds(), mask=None, weights=None, vp0=None, rho0=None):
    """Alg. 1 on all shots: returns (vp, rho, history)."""
    prob = FwiProblem(ctx, job, dobs, family=family, npar=npar, bounds=bounds, mask=mask,
                      weights=weights)
    dev = dobs.device
    vp = torch.from_numpy(np.ascontiguousarray(job.vp if vp0 is None else vp0, np.float32)).reshape(-1).to(dev)
    rho = torch.from_numpy(np.ascontiguousarray(job.rho if rho0 is None else rho0, np.float32)).reshape(-1).to(dev)
    lo, hi = prob.x_bounds()
    x, hist = lbfgs(prob, prob.to_x(vp, rho), cfg, lo, hi)
    vp, rho = prob.to_model(x)
    return vp, rho, hist


# ----------------------------------------------------------------------------- SGD batches

def shot_batches(nshot: int, batch: int, epochs: int, seed: int = 0) -> List[List[int]]:
    """Random shuffling of the shot indices, cut into batches (the last batch of an epoch may
    be smaller); each epoch visits every shot once."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(epochs):
        perm = rng.permutation(nshot)
        out += [sorted(int(i) for i in perm[k:k + batch]) for k in range(0, nshot, batch)]
    return out


def sgd(ctx, job, dobs, *, batch: int, epochs: int = 1, seed: int = 0, family=1, npar=1,
        bounds: Bounds = Bounds(), mask=None, first_step: float = 0.01, nls: int = 10):
    """Batchwise stochastic gradient descent (Sec. 5): each batch of shuffled shots makes one
    steepest-descent update of the model with an Armijo line search on that batch; the
    updated model starts the next batch.  Returns (vp, rho, list of (batch, J before, J after))."""
    dev = dobs.device
    prob = FwiProblem(ctx, job, dobs, family=family, npar=npar, bounds=bounds, mask=mask)
    lo, hi = prob.x_bounds()
    vp = torch.from_numpy(np.ascontiguousarray(job.vp, np.float32)).reshape(-1).to(dev)
    rho = torch.from_numpy(np.ascontiguousarray(job.rho, np.float32)).reshape(-1).to(dev)
    x = prob.to_x(vp, rho)
    log = []
    cfg = LbfgsConfig(niter=1, nls=nls, npair=0, first_step=first_step)
    for b in shot_batches(job.acq.nshot, batch, epochs, seed):
        prob.set_shots(b, dobs)
        J0, g0 = prob(x)
        d = -g0
        alpha = first_step / max(float(d.abs().max()), 1e-300)
        res = wolfe_search(prob, x, J0, g0, d, alpha, cfg, lo, hi, armijo_only=True)
        if res is not None:
            x = res[1]
            log.append((b, J0, res[2]))
        else:
            log.append((b, J0, J0))
    vp, rho = prob.to_model(x)
    return vp, rho, log


# ----------------------------------------------------------------------------- data weighting

def offset_weights(acq, nt: int, dxw: float, xw: Sequence[float]) -> np.ndarray:
    """Offset weighting (Sec. 3.7, data weighting): receiver r of shot s gets the weight of its
    offset |x_r - x_s| linearly interpolated in the table xw sampled every dxw metres (the last
    value beyond the table).  Returned in the layout of the data (float32)."""
    xw = np.asarray(xw, np.float64)
    out = np.empty(nt * int(acq.rec_off[-1]), np.float32)
    for s in range(acq.nshot):
        a, b = int(acq.rec_off[s]), int(acq.rec_off[s + 1])
        h = np.hypot(acq.rec[a:b, 1] - acq.src[s, 1], acq.rec[a:b, 2] - acq.src[s, 2])
        w = np.interp(h / dxw, np.arange(len(xw)), xw)
        out[nt * a: nt * b] = np.tile(w.astype(np.float32), nt)
    return out


def mute_weights(acq, nt: int, dt: float, xmute: Sequence[float], tmute: Sequence[float],
                 ntaper: int, mode: int) -> np.ndarray:
    """Front (mode 1) or tail (mode 2) muting (Sec. 3.7): the mute time of a trace is the line
    (xmute, tmute) interpolated at the trace's offset; mode 1 zeroes the samples before it
    (keeping later arrivals, the reflections), mode 2 those after it (keeping the first
    arrivals); ntaper samples of a cosine taper join the muted and kept parts."""
    xm, tm = np.asarray(xmute, np.float64), np.asarray(tmute, np.float64)
    out = np.empty(nt * int(acq.rec_off[-1]), np.float32)
    t = np.arange(nt) * dt
    for s in range(acq.nshot):
        a, b = int(acq.rec_off[s]), int(acq.rec_off[s + 1])
        h = np.hypot(acq.rec[a:b, 1] - acq.src[s, 1], acq.rec[a:b, 2] - acq.src[s, 2])
        tcut = np.interp(h, xm, tm)                            # per receiver
        u = (t[:, None] - tcut[None, :]) / max(ntaper * dt, 1e-30)   # samples past the line
        ramp = np.clip(u, 0.0, 1.0)
        taper = 0.5 - 0.5 * np.cos(np.pi * ramp)               # 0 before, 1 after the taper
        w = taper if mode == 1 else 1.0 - taper
        out[nt * a: nt * b] = w.astype(np.float32).ravel()
    return out
