"""Seeded synthetic inputs: velocity/density models, source wavelets, acquisition.

This module holds no step of the modelling method itself (no stencil, no PML, no
imaging); it only draws the inputs that both the HIP path and the FP64 oracle
consume, so both sides see byte-identical models and geometries.

Conventions (Sec. 3.4-3.6 of the paper: n1 = z is the fastest axis, then x, then y):
  * 2D arrays have shape (n2, n1)  -> index [x, z]
  * 3D arrays have shape (n3, n2, n1) -> index [y, x, z]
  * positions are (z, x, y) in metres measured from interior cell 0.

The paper's own workloads (Marmousi, Overthrust; Sec. 5) are not available, so
seeded layered / perturbed models of the same shapes stand in for them.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional

import numpy as np
from scipy.ndimage import gaussian_filter


@dataclasses.dataclass
class Grid:
    """Simulation parameters; names follow the paper's keywords (Sec. 3.6, 3.8, 4.2)."""
    ndim: int
    n1: int
    n2: int
    n3: int = 1
    d1: float = 10.0
    d2: float = 10.0
    d3: float = 10.0
    nb: int = 20
    order: int = 4
    nt: int = 1000
    dt: float = 1e-3
    fm: float = 10.0
    dr: int = 1
    box: int = 0
    margin: int = -1          # -1: default 2N = order
    freesurf: int = 0
    vpmin: float = 0.0        # 0: let the library reduce the model
    vpmax: float = 0.0

    @property
    def shape(self):
        return (self.n3, self.n2, self.n1) if self.ndim == 3 else (self.n2, self.n1)

    @property
    def npts(self) -> int:
        return self.n1 * self.n2 * (self.n3 if self.ndim == 3 else 1)

    @property
    def padded(self):
        m = [self.n1 + 2 * self.nb, self.n2 + 2 * self.nb]
        if self.ndim == 3:
            m.append(self.n3 + 2 * self.nb)
        return m

    @property
    def padded_npts(self) -> int:
        return int(np.prod(self.padded))


@dataclasses.dataclass
class Acquisition:
    """Sources and their receivers (Sec. 3.4): one source per shot, CSR receiver lists."""
    src: np.ndarray        # (nshot, 3) float64, (z, x, y) metres
    rec_off: np.ndarray    # (nshot+1,) int32
    rec: np.ndarray        # (rec_off[-1], 3) float64, (z, x, y) metres

    @property
    def nshot(self) -> int:
        return int(self.src.shape[0])

    def nrec(self, s: int) -> int:
        return int(self.rec_off[s + 1] - self.rec_off[s])

    def shot(self, s: int) -> "Acquisition":
        a, b = int(self.rec_off[s]), int(self.rec_off[s + 1])
        return Acquisition(self.src[s:s + 1].copy(), np.array([0, b - a], np.int32),
                           self.rec[a:b].copy())

    def subset(self, shots) -> "Acquisition":
        shots = list(shots)
        recs = [self.rec[self.rec_off[s]:self.rec_off[s + 1]] for s in shots]
        off = np.zeros(len(shots) + 1, np.int32)
        off[1:] = np.cumsum([len(r) for r in recs])
        return Acquisition(self.src[shots].copy(), off,
                           np.concatenate(recs).astype(np.float64) if recs else np.zeros((0, 3)))


@dataclasses.dataclass
class Job:
    grid: Grid
    vp: np.ndarray          # float32, grid.shape
    rho: np.ndarray         # float32, grid.shape
    acq: Acquisition
    stf: np.ndarray         # float32 (nshot, nt)
    name: str = ""
    extra: dict = dataclasses.field(default_factory=dict)


def ricker(nt: int, dt: float, fm: float, t0: Optional[float] = None) -> np.ndarray:
    """Ricker wavelet w(t) sampled at t = n*dt, delay t0 = 1.2/fm by default."""
    if t0 is None:
        t0 = 1.2 / fm
    t = np.arange(nt, dtype=np.float64) * dt - t0
    a = (math.pi * fm * t) ** 2
    return (1.0 - 2.0 * a) * np.exp(-a)


def gardner(vp: np.ndarray) -> np.ndarray:
    """Gardner's relation rho = 310 * vp^0.25 (kg/m^3, vp in m/s)."""
    return (310.0 * np.power(vp.astype(np.float64), 0.25)).astype(np.float32)


def _surface_line(nshot_pos_x: np.ndarray, z: float, rec_x: np.ndarray, rec_z: float,
                  y: float = 0.0) -> Acquisition:
    ns = len(nshot_pos_x)
    src = np.zeros((ns, 3))
    src[:, 0] = z
    src[:, 1] = nshot_pos_x
    src[:, 2] = y
    one = np.zeros((len(rec_x), 3))
    one[:, 0] = rec_z
    one[:, 1] = rec_x
    one[:, 2] = y
    rec = np.concatenate([one] * ns) if ns else np.zeros((0, 3))
    off = np.arange(ns + 1, dtype=np.int32) * len(rec_x)
    return Acquisition(src, off, rec)


# --------------------------------------------------------------------------- models

def three_layer_2d(n1=201, n2=201, speeds=(1500.0, 2000.0, 2500.0)) -> np.ndarray:
    """Horizontal layers of equal thickness along z."""
    vp = np.empty((n2, n1), np.float32)
    k = len(speeds)
    for j in range(k):
        z0 = (j * n1) // k
        z1 = ((j + 1) * n1) // k if j < k - 1 else n1
        vp[:, z0:z1] = speeds[j]
    return vp


def dipping_layers_2d(n1: int, n2: int, d: float, nlayer=10, vmin=1500.0, vmax=4500.0,
                      dip_deg=10.0, pert=0.05, sigma_cells=5.0, seed=1002) -> np.ndarray:
    """Dipping layers v_j = vmin + j (vmax-vmin)/(nlayer-1), interfaces at j*H/nlayer
    deepening by tan(dip) per metre of x, times (1 + p) with p a Gaussian-smoothed
    N(0,1) field scaled to max|p| = pert."""
    H = n1 * d
    z = np.arange(n1) * d
    x = np.arange(n2) * d
    zz = z[None, :] - x[:, None] * math.tan(math.radians(dip_deg))
    j = np.clip(np.floor(zz / (H / nlayer)), 0, nlayer - 1).astype(np.int64)
    v = vmin + j * (vmax - vmin) / (nlayer - 1)
    if pert > 0:
        rng = np.random.default_rng(seed)
        g = gaussian_filter(rng.standard_normal((n2, n1)), sigma_cells, mode="nearest")
        g *= pert / np.max(np.abs(g))
        v = v * (1.0 + g)
    return v.astype(np.float32)


def flat_layers_3d(n: int, d: float, speeds=(1500, 2000, 2500, 3000, 3500, 4000)) -> np.ndarray:
    k = len(speeds)
    vp = np.empty((n, n, n), np.float32)
    for j in range(k):
        z0 = (j * n) // k
        z1 = ((j + 1) * n) // k if j < k - 1 else n
        vp[:, :, z0:z1] = speeds[j]
    return vp


def salt_ellipsoid(vp: np.ndarray, seed: int, vsalt=4500.0, edge_cells=2.0) -> np.ndarray:
    """Blend a smooth ellipsoid of speed vsalt into a cube (index [y, x, z])."""
    n3, n2, n1 = vp.shape
    rng = np.random.default_rng(seed)
    L = np.array([n1, n2, n3], np.float64)
    centre = np.array([0.55, 0.5, 0.5]) * L + rng.uniform(-0.05, 0.05, 3) * L
    semi = np.array([0.12, 0.22, 0.18]) * L * rng.uniform(0.8, 1.2, 3)
    iz = (np.arange(n1) - centre[0]) / semi[0]
    ix = (np.arange(n2) - centre[1]) / semi[1]
    iy = (np.arange(n3) - centre[2]) / semi[2]
    r = np.sqrt(iy[:, None, None] ** 2 + ix[None, :, None] ** 2 + iz[None, None, :] ** 2)
    # signed distance along the radius, in cells of the smallest semi-axis
    w = 0.5 * (1.0 - np.tanh((r - 1.0) * semi.min() / edge_cells))
    return (vp * (1.0 - w) + vsalt * w).astype(np.float32)


def gaussian_anomaly(vp: np.ndarray, d: float, centre_zx=(1500.0, 4500.0), sigma=200.0,
                     amp=0.1) -> np.ndarray:
    n2, n1 = vp.shape
    z = np.arange(n1) * d - centre_zx[0]
    x = np.arange(n2) * d - centre_zx[1]
    r2 = x[:, None] ** 2 + z[None, :] ** 2
    return (vp.astype(np.float64) * (1.0 + amp * np.exp(-r2 / (2 * sigma ** 2)))).astype(np.float32)


# --------------------------------------------------------------------------- workloads

def config1(nt=1000) -> Job:
    """2D forward, one shot: 201x201, 10 m, 3 layers, rho 1000, order 4, 20 CPML layers,
    Ricker 10 Hz at grid (10,100), dt 1 ms, 201 receivers at depth index 5."""
    g = Grid(ndim=2, n1=201, n2=201, d1=10.0, d2=10.0, nb=20, order=4, nt=nt, dt=1e-3, fm=10.0)
    vp = three_layer_2d(201, 201)
    rho = np.full_like(vp, 1000.0)
    acq = _surface_line(np.array([100 * 10.0]), 10 * 10.0, np.arange(201) * 10.0, 5 * 10.0)
    stf = ricker(nt, g.dt, g.fm)[None, :].astype(np.float32)
    return Job(g, vp, rho, acq, stf, name="2d-forward-201x201-order4")


def config2(n1=500, n2=1500, nt=4000, nshot=16, box=1, seed=1002) -> Job:
    """2D batched forward: 10 dipping layers 1500-4500 m/s +-5% smoothed noise, Gardner
    density, order 8, 30 CPML layers, Ricker 15 Hz, dt 0.8 ms, shots spread along the
    surface (z index 2), every surface column recorded (z index 2)."""
    d = 10.0
    g = Grid(ndim=2, n1=n1, n2=n2, d1=d, d2=d, nb=30, order=8, nt=nt, dt=0.8e-3, fm=15.0,
             box=box)
    vp = dipping_layers_2d(n1, n2, d, seed=seed)
    rho = gardner(vp)
    sx = np.array([round((k + 0.5) * n2 / nshot) for k in range(nshot)], np.float64) * d
    acq = _surface_line(sx, 2 * d, np.arange(n2) * d, 2 * d)
    stf = np.repeat(ricker(nt, g.dt, g.fm)[None, :], nshot, 0).astype(np.float32)
    return Job(g, vp, rho, acq, stf, name=f"2d-batched-forward-{n1}x{n2}-order8-{nshot}shots")


def config3(n1=300, n2=900, nt=4000, nshot=32, seed=1003) -> Job:
    """2D FWI gradient: config-2 model family at 300x900, 32 shots, true model with a
    +10% Gaussian anomaly (sigma 200 m) at (z, x) = (1500 m, 4500 m); rho held fixed
    (Gardner density of the background model, in both models)."""
    d = 10.0
    g = Grid(ndim=2, n1=n1, n2=n2, d1=d, d2=d, nb=30, order=8, nt=nt, dt=0.8e-3, fm=15.0,
             box=1, dr=1)
    vp0 = dipping_layers_2d(n1, n2, d, seed=seed)
    rho = gardner(vp0)
    centre = (min(1500.0, 0.5 * n1 * d), min(4500.0, 0.5 * n2 * d))
    vtrue = gaussian_anomaly(vp0, d, centre_zx=centre)
    sx = np.array([round((k + 0.5) * n2 / nshot) for k in range(nshot)], np.float64) * d
    acq = _surface_line(sx, 2 * d, np.arange(n2) * d, 2 * d)
    stf = np.repeat(ricker(nt, g.dt, g.fm)[None, :], nshot, 0).astype(np.float32)
    job = Job(g, vp0, rho, acq, stf, name=f"2d-fwi-gradient-{n1}x{n2}-order8-{nshot}shots")
    job.extra["vp_true"] = vtrue
    rng = np.random.default_rng(seed)
    job.extra["rng"] = rng
    return job


def config4(n=400, nt=3000, dr=10, nshot=4, seed=1004, rec_step=2) -> Job:
    """3D RTM: n^3 cells of 12.5 m, 6 flat layers 1500-4000 m/s + seeded salt ellipsoid
    (4500 m/s), Gardner density, order 8, 20 CPML layers, Ricker 12 Hz, dt 1 ms, shots at
    (x, y) in {n/4, 3n/4}^2 at z index 2, receivers on every rec_step-th (x, y) surface cell
    at z index 2. Migration model = true model smoothed with sigma = 8 cells."""
    d = 12.5
    g = Grid(ndim=3, n1=n, n2=n, n3=n, d1=d, d2=d, d3=d, nb=20, order=8, nt=nt, dt=1e-3,
             fm=12.0, dr=dr, box=1)
    vtrue = salt_ellipsoid(flat_layers_3d(n, d), seed)
    vmig = gaussian_filter(vtrue.astype(np.float64), 8.0, mode="nearest").astype(np.float32)
    rho = gardner(vmig)
    q = [n // 4, (3 * n) // 4]
    pos = [(a, b) for a in q for b in q][:nshot]
    src = np.array([[2 * d, x * d, y * d] for (x, y) in pos], np.float64)
    ys, xs = np.meshgrid(np.arange(0, n, rec_step), np.arange(0, n, rec_step), indexing="ij")
    one = np.stack([np.full(xs.size, 2 * d), xs.ravel() * d, ys.ravel() * d], 1)
    rec = np.concatenate([one] * len(pos))
    off = np.arange(len(pos) + 1, dtype=np.int32) * one.shape[0]
    stf = np.repeat(ricker(nt, g.dt, g.fm)[None, :], len(pos), 0).astype(np.float32)
    job = Job(g, vmig, rho, Acquisition(src, off, rec), stf,
              name=f"3d-rtm-{n}^3-order8-{len(pos)}shots-dr{dr}")
    job.extra["vp_true"] = vtrue
    job.extra["rho_true"] = gardner(vtrue)
    return job


def hyperbolic_event(job: "Job", depth: float, v: float, t0: Optional[float] = None) -> List[np.ndarray]:
    """Synthetic observed data: one reflection event per trace, the job's wavelet delayed by
    the two-way time sqrt((2 depth / v)^2 + (offset / v)^2) of a flat reflector under a
    homogeneous overburden, scaled by 1 / (v t) (spherical spreading).  A closed-form stand-in
    for recorded data (no modelling run); list of [nt, nrec_s] float64 arrays per shot."""
    g = job.grid
    fm = g.fm
    t0 = 1.2 / fm if t0 is None else t0
    t = np.arange(g.nt) * g.dt
    out = []
    for s in range(job.acq.nshot):
        a, b = int(job.acq.rec_off[s]), int(job.acq.rec_off[s + 1])
        h = np.sqrt(np.sum((job.acq.rec[a:b, 1:] - job.acq.src[s, 1:]) ** 2, axis=1))
        tr = np.sqrt((2.0 * depth / v) ** 2 + (h / v) ** 2)
        arg = (math.pi * fm * (t[:, None] - tr[None, :] - t0)) ** 2
        out.append((1.0 - 2.0 * arg) * np.exp(-arg) / (v * tr[None, :]))
    return out


def homogeneous(ndim: int, n: int, d: float, c: float, rho: float = 1000.0) -> np.ndarray:
    shape = (n, n, n) if ndim == 3 else (n, n)
    return np.full(shape, c, np.float32), np.full(shape, rho, np.float32)


@dataclasses.dataclass
class StreamJob:
    """One request of the served shot stream."""
    kind: str              # "forward2d" | "grad2d" | "forward3d"
    arrival: float         # seconds after stream start
    job: Job
    model_key: Optional[str] = None   # requests with equal keys share grid, model and wavelet


_CLASSES = ("forward2d", "grad2d", "forward3d")


def _survey(cls: str, k: int, seed: int, scale: float, nt2d: int, nt3d: int, ntgrad: int):
    """Survey k of a job class of the served stream: grid, model, density and wavelet, built
    from its own seeded generator (independent of the arrival draws)."""
    r = np.random.default_rng([seed, _CLASSES.index(cls), k])
    fm = float(r.uniform(10.0, 15.0))
    if cls == "forward2d":
        n1 = max(16, int(r.integers(200, 801) * scale))
        n2 = max(16, int(r.integers(600, 2001) * scale))
        nt = max(20, int(nt2d * scale))
        g = Grid(ndim=2, n1=n1, n2=n2, d1=10.0, d2=10.0, nb=20, order=8, nt=nt, dt=0.8e-3,
                 fm=fm, box=1)
        vp = dipping_layers_2d(n1, n2, 10.0, seed=int(r.integers(1 << 30)))
        return {"grid": g, "vp": vp, "rho": gardner(vp), "extra": {},
                "stf": ricker(nt, g.dt, fm)[None, :].astype(np.float32)}
    if cls == "grad2d":
        n1, n2 = max(16, int(300 * scale)), max(16, int(900 * scale))
        nt = max(20, int(ntgrad * scale))
        j = config3(n1=n1, n2=n2, nt=nt, nshot=1, seed=int(r.integers(1 << 30)))
        j.grid.fm = fm
        return {"grid": j.grid, "vp": j.vp, "rho": j.rho, "extra": {"vp_true": j.extra["vp_true"]},
                "stf": ricker(nt, j.grid.dt, fm)[None, :].astype(np.float32)}
    n = max(12, int(r.integers(200, 351) * scale))
    nt = max(20, int(nt3d * scale))
    g = Grid(ndim=3, n1=n, n2=n, n3=n, d1=12.5, d2=12.5, d3=12.5, nb=20, order=8, nt=nt,
             dt=1e-3, fm=fm, box=1)
    vp = flat_layers_3d(n, 12.5)
    return {"grid": g, "vp": vp, "rho": gardner(vp), "extra": {},
            "stf": ricker(nt, g.dt, fm)[None, :].astype(np.float32)}


def stream_config5(njobs=300, rate=1.0, seed=1005, scale=1.0, nt2d=3000, nt3d=1500,
                   ntgrad=4000, pool=0) -> List[StreamJob]:
    """Served stream: Poisson arrivals; 60% 2D forward (nz~U[200,800], nx~U[600,2000]),
    30% 2D gradient (config-3 sizes, 1 shot), 10% 3D forward (side~U[200,350]); order 8,
    fm~U[10,15], seeded layered models. `scale` shrinks every size for tests.

    pool = 0: every request has its own grid and model.  pool > 0: each class draws its
    requests from `pool` seeded surveys (grid, model and wavelet; model_key "<class>-<k>"),
    and a request is one shot of its survey at a seeded surface position, with the survey's
    receiver spread -- the stream of many shots over few models that a modelling or inversion
    service sees, where requests of one survey can share a launch."""
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    surveys = {}
    for k in range(njobs):
        t += rng.exponential(1.0 / rate)
        u = rng.uniform()
        if pool > 0:
            cls = "forward2d" if u < 0.6 else ("grad2d" if u < 0.9 else "forward3d")
            key = f"{cls}-{int(rng.integers(pool))}"
            if key not in surveys:
                surveys[key] = _survey(cls, int(key.rsplit("-", 1)[1]), seed, scale, nt2d,
                                       nt3d, ntgrad)
            sv = surveys[key]
            g = sv["grid"]
            if g.ndim == 2:
                sx = float(rng.integers(g.n2)) * g.d2
                acq = _surface_line(np.array([sx]), 2 * g.d1, np.arange(g.n2) * g.d2, 2 * g.d1)
            else:
                n = g.n1
                sx, sy = (float(v) * g.d2 for v in rng.integers(n, size=2))
                ys, xs = np.meshgrid(np.arange(0, n, 2), np.arange(0, n, 2), indexing="ij")
                rec = np.stack([np.full(xs.size, 2 * g.d1), xs.ravel() * g.d2, ys.ravel() * g.d3], 1)
                acq = Acquisition(np.array([[2 * g.d1, sx, sy]]),
                                  np.array([0, rec.shape[0]], np.int32), rec)
            j = Job(g, sv["vp"], sv["rho"], acq, sv["stf"], name=f"{cls}-{k}")
            j.extra.update(sv["extra"])
            out.append(StreamJob(cls, t, j, model_key=key))
            continue
        fm = float(rng.uniform(10.0, 15.0))
        if u < 0.6:
            n1 = max(16, int(rng.integers(200, 801) * scale))
            n2 = max(16, int(rng.integers(600, 2001) * scale))
            nt = max(20, int(nt2d * scale))
            d = 10.0
            g = Grid(ndim=2, n1=n1, n2=n2, d1=d, d2=d, nb=20, order=8, nt=nt, dt=0.8e-3, fm=fm,
                     box=1)
            vp = dipping_layers_2d(n1, n2, d, seed=int(rng.integers(1 << 30)))
            acq = _surface_line(np.array([round(n2 / 2) * d]), 2 * d, np.arange(n2) * d, 2 * d)
            stf = ricker(nt, g.dt, fm)[None, :].astype(np.float32)
            out.append(StreamJob("forward2d", t, Job(g, vp, gardner(vp), acq, stf,
                                                      name=f"fwd2d-{k}")))
        elif u < 0.9:
            n1 = max(16, int(300 * scale))
            n2 = max(16, int(900 * scale))
            nt = max(20, int(ntgrad * scale))
            j = config3(n1=n1, n2=n2, nt=nt, nshot=1, seed=int(rng.integers(1 << 30)))
            j.grid.fm = fm
            j.stf = ricker(nt, j.grid.dt, fm)[None, :].astype(np.float32)
            j.name = f"grad2d-{k}"
            out.append(StreamJob("grad2d", t, j))
        else:
            n = max(12, int(rng.integers(200, 351) * scale))
            nt = max(20, int(nt3d * scale))
            d = 12.5
            g = Grid(ndim=3, n1=n, n2=n, n3=n, d1=d, d2=d, d3=d, nb=20, order=8, nt=nt,
                     dt=1e-3, fm=fm, box=1)
            vp = flat_layers_3d(n, d)
            ys, xs = np.meshgrid(np.arange(0, n, 2), np.arange(0, n, 2), indexing="ij")
            rec = np.stack([np.full(xs.size, 2 * d), xs.ravel() * d, ys.ravel() * d], 1)
            acq = Acquisition(np.array([[2 * d, (n // 2) * d, (n // 2) * d]]),
                              np.array([0, rec.shape[0]], np.int32), rec)
            stf = ricker(nt, g.dt, fm)[None, :].astype(np.float32)
            out.append(StreamJob("forward3d", t, Job(g, vp, gardner(vp), acq, stf,
                                                      name=f"fwd3d-{k}")))
    return out
