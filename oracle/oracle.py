"""FP64 CPU oracle for the SMIwiz modelling / imaging path -- TEST INFRASTRUCTURE ONLY.

Only the test suite, the smoke check and the CPU-baseline leg of the benchmark may import
this module.  It wraps the plain C stepper in ``smi_oracle.c`` (built with gcc, loaded
with ctypes) and adds the host-side arithmetic of the method in plain numpy:

  * eq. (5)  CFL number                                    -> :func:`cfl_number`
  * eq. (6)  L2 misfit and residual adjoint source         -> :func:`misfit`
  * eq. (7)  kappa gradient, chain rule to Vp (rho fixed)  -> :func:`fwi_grad`
  * eq. (7)  rho gradient, families (Vp, rho), (Vp, Ip)      -> :func:`fwi_grad_family`
  * eq. (10) cross-correlation image                       -> :func:`rtm_image`
  * eq. (10) the map whose transpose is the image            -> :func:`react`
  * Sec. 2.3 source-normalised image, Laplace filter         -> :func:`normalized_image`,
                                                               :func:`laplacian`
  * Alg. 2   forward loop, adjoint source, reverse loop, sum over shots

Positions in metres are turned into padded grid nodes by rounding (on-grid positions only).
Arrays follow the memory order of the paper's files: n1 = z fastest, i.e. numpy shape
(n2, n1) in 2D and (n3, n2, n1) in 3D.
"""
from __future__ import annotations

import ctypes as C
import math
import os
import subprocess
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "smi_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")


class OgTaps(C.Structure):
    _fields_ = [("n", C.c_int), ("off", C.POINTER(C.c_int)), ("idx", C.POINTER(C.c_int)),
                ("w", C.POINTER(C.c_double))]


class Taps:
    """Point operators (off-grid sources / receivers) and the arrays they point to."""

    def __init__(self, off, idx, w):
        self.off = np.ascontiguousarray(off, np.int32)
        self.idx = np.ascontiguousarray(idx, np.int32).reshape(-1, 3)
        self.w = np.ascontiguousarray(w, np.float64)
        self.c = OgTaps(len(self.off) - 1, self.off.ctypes.data_as(C.POINTER(C.c_int)),
                        self.idx.ctypes.data_as(C.POINTER(C.c_int)),
                        self.w.ctypes.data_as(C.POINTER(C.c_double)))


def _tp(t: Optional["Taps"]):
    return None if t is None else C.byref(t.c)


class OgGrid(C.Structure):
    _fields_ = [("ndim", C.c_int), ("n1", C.c_int), ("n2", C.c_int), ("n3", C.c_int),
                ("d1", C.c_double), ("d2", C.c_double), ("d3", C.c_double),
                ("nb", C.c_int), ("order", C.c_int), ("nt", C.c_int),
                ("dt", C.c_double), ("fm", C.c_double), ("vmax", C.c_double),
                ("pml", C.c_int), ("box", C.c_int), ("margin", C.c_int), ("dr", C.c_int),
                ("band_p", C.c_int), ("band_v", C.c_int), ("freesurf", C.c_int)]


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (FP64, IEEE semantics, OpenMP)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-D_DEFAULT_SOURCE", "-fopenmp",
                               "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        L = C.CDLL(_LIB)
        dp = C.POINTER(C.c_double)
        ip = C.POINTER(C.c_int)
        gp = C.POINTER(OgGrid)
        L.og_fd_coef.argtypes = [C.c_int, dp]
        L.og_cpml_profile.argtypes = [gp, C.c_int, C.c_int, dp, dp]
        L.og_fwd_box.argtypes = [gp, ip, C.c_int, ip, ip]
        L.og_band_size.argtypes = [gp]
        L.og_band_size.restype = C.c_size_t
        L.og_band_levels.argtypes = [gp]
        L.og_band_levels.restype = C.c_size_t
        tp = C.POINTER(OgTaps)
        L.og_forward.argtypes = [gp, dp, dp, ip, dp, C.c_int, ip, dp, dp, dp, dp, dp, C.c_int,
                                 ip, dp, tp, tp]
        L.og_reconstruct.argtypes = [gp, dp, dp, ip, dp, dp, dp, C.c_int, ip, dp, tp]
        L.og_adjoint.argtypes = [gp, dp, dp, ip, dp, C.c_int, ip, dp, dp, dp, dp, dp, dp, dp, dp,
                                 tp, tp, C.c_int, C.c_int, ip, dp]
        L.og_born.argtypes = [gp, dp, dp, ip, dp, C.c_int, ip, dp, dp, tp, tp]
        L.og_react.argtypes = [gp, dp, dp, ip, dp, C.c_int, ip, dp, C.c_double, C.c_int, dp,
                               tp, tp]
        _lib = L
    return _lib


def _d(a: Optional[np.ndarray]):
    if a is None:
        return None
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _i(a: Optional[np.ndarray]):
    if a is None:
        return None
    assert a.dtype == np.int32 and a.flags.c_contiguous
    return a.ctypes.data_as(C.POINTER(C.c_int))


# ------------------------------------------------------------------ grid helpers

def fd_coef(order: int) -> np.ndarray:
    a = np.zeros(order // 2)
    if lib().og_fd_coef(order, _d(a)) != 0:
        raise ValueError("unsupported order")
    return a


def og_grid(g, *, vmax: float, pml: int = 1, box: Optional[int] = None,
            band_p: int = 0, band_v: int = 0) -> OgGrid:
    """Build the C grid record from any object with the paper's keywords."""
    margin = getattr(g, "margin", -1)
    if margin is None or margin < 0:
        margin = g.order
    return OgGrid(g.ndim, g.n1, g.n2, g.n3 if g.ndim == 3 else 1,
                  float(g.d1), float(g.d2), float(g.d3 if g.ndim == 3 else 1.0),
                  g.nb, g.order, g.nt, float(g.dt), float(g.fm), float(vmax), int(pml),
                  int(g.box if box is None else box), int(margin), int(getattr(g, "dr", 1)),
                  int(band_p), int(band_v), int(getattr(g, "freesurf", 0) or 0))


def cfl_number(g, vmax: float) -> float:
    """Left-hand side of eq. (5): dt Vmax sqrt(sum 1/d^2) sum |a_l| (stable iff <= 1)."""
    inv = 1.0 / g.d1 ** 2 + 1.0 / g.d2 ** 2 + (1.0 / g.d3 ** 2 if g.ndim == 3 else 0.0)
    return g.dt * vmax * math.sqrt(inv) * float(np.sum(np.abs(fd_coef(g.order))))


def node(g, pos) -> np.ndarray:
    """Padded node of a position (z, x, y) in metres (nearest node)."""
    ds = [g.d1, g.d2, g.d3]
    out = np.zeros(3, np.int32)
    for a in range(g.ndim):
        out[a] = g.nb + int(round(float(pos[a]) / ds[a]))
    return out


# Kaiser window parameter b of the windowed-sinc point operators for half-width r (Hicks'
# table for a maximum wavenumber of half the Nyquist one); the half-width is order / 2.
KAISER_B = {1: 1.24, 2: 2.94, 3: 4.53, 4: 6.31}
ON_GRID = 1e-3          # positions within this fraction of a spacing of a node are on it


def _i0(x: float) -> float:
    s, t, k = 1.0, 1.0, 1
    while True:
        t *= (x / (2.0 * k)) ** 2
        s += t
        if t < 1e-17 * s:
            return s
        k += 1


def hicks_weights_1d(u: float, r: int, M: int):
    """Nodes and weights of the windowed-sinc operator of a point at fractional padded index
    u along one axis: sinc(j - u) times the Kaiser window I0(b sqrt(1 - ((j-u)/r)^2)) / I0(b)
    on the 2r nodes around u; a point within ON_GRID of a node is that node, weight 1.  Nodes
    outside [0, M) are dropped."""
    j0 = int(round(u))
    if abs(u - j0) <= ON_GRID:
        return [j0], [1.0]
    b = KAISER_B[r]
    nodes, w = [], []
    base = int(math.floor(u))
    for j in range(base - r + 1, base + r + 1):
        x = j - u
        win = _i0(b * math.sqrt(max(0.0, 1.0 - (x / r) ** 2))) / _i0(b)
        if 0 <= j < M:
            nodes.append(j)
            w.append(math.sin(math.pi * x) / (math.pi * x) * win)
    return nodes, w


def point_taps(g, positions) -> Taps:
    """Tensor-product windowed-sinc operators (Sec. 2.1) of a list of positions (z, x, y) in
    metres: padded nodes and weights per point."""
    ds = [g.d1, g.d2, g.d3]
    Ms = [g.n1 + 2 * g.nb, g.n2 + 2 * g.nb, (g.n3 + 2 * g.nb) if g.ndim == 3 else 1]
    r = g.order // 2
    off, idx, w = [0], [], []
    for pos in positions:
        per = []
        for a in range(3):
            if a >= g.ndim:
                per.append(([0], [1.0]))
            else:
                per.append(hicks_weights_1d(g.nb + float(pos[a]) / ds[a], r, Ms[a]))
        for i3, w3 in zip(*per[2]):
            for i2, w2 in zip(*per[1]):
                for i1, w1 in zip(*per[0]):
                    idx.append((i1, i2, i3))
                    w.append(w1 * w2 * w3)
        off.append(len(w))
    return Taps(off, np.array(idx, np.int32).reshape(-1, 3), np.array(w))


def shot_ops(g, acq, s: int):
    """(src node, receiver nodes, source operator, receiver operator) of shot s; the operators
    are None when every point of the kind lies on a node.  The nodes (nearest) centre the
    computing boxes."""
    src, rec = shot_nodes(g, acq, s)
    a, b = int(acq.rec_off[s]), int(acq.rec_off[s + 1])
    st = point_taps(g, [acq.src[s]])
    rt = point_taps(g, acq.rec[a:b])
    return (src, rec, None if len(st.w) == 1 else st,
            None if len(rt.w) == b - a else rt)


def shot_nodes(g, acq, s: int):
    src = node(g, acq.src[s])
    a, b = int(acq.rec_off[s]), int(acq.rec_off[s + 1])
    rec = np.zeros((b - a, 3), np.int32)
    for k in range(b - a):
        rec[k] = node(g, acq.rec[a + k])
    return src, np.ascontiguousarray(rec)


def cpml_profile(gr: OgGrid, axis: int, half: int):
    n = [gr.n1, gr.n2, gr.n3][axis] + 2 * gr.nb
    a = np.zeros(n)
    b = np.zeros(n)
    lib().og_cpml_profile(C.byref(gr), axis, half, _d(a), _d(b))
    return a, b


def fwd_box(gr: OgGrid, src: np.ndarray, it: int):
    lo = np.zeros(3, np.int32)
    hi = np.zeros(3, np.int32)
    lib().og_fwd_box(C.byref(gr), _i(src), it, _i(lo), _i(hi))
    return lo, hi


def band_size(gr: OgGrid) -> int:
    return int(lib().og_band_size(C.byref(gr)))


def padded_size(gr: OgGrid) -> int:
    P = (gr.n1 + 2 * gr.nb) * (gr.n2 + 2 * gr.nb)
    if gr.ndim == 3:
        P *= gr.n3 + 2 * gr.nb
    return P


def interior_size(gr: OgGrid) -> int:
    return gr.n1 * gr.n2 * (gr.n3 if gr.ndim == 3 else 1)


# ------------------------------------------------------------------ single-shot drivers

def forward(gr: OgGrid, vp, rho, src, stf, rec, *, init=None, hist=False, bands=False,
            final=False, snaps: Sequence[int] = (), st: Optional[Taps] = None,
            rt: Optional[Taps] = None):
    """Forward loop of Alg. 2 for one shot.  Returns dict(dcal[nt, nrec], hist, bands,
    final, snaps).  st / rt: off-grid source / receiver operators (None: at the nodes)."""
    vp = np.ascontiguousarray(vp, np.float64)
    rho = np.ascontiguousarray(rho, np.float64)
    stf = np.ascontiguousarray(stf, np.float64)
    src = np.ascontiguousarray(src, np.int32)
    rec = np.ascontiguousarray(np.asarray(rec, np.int32).reshape(-1, 3))
    nrec = rec.shape[0]
    P = padded_size(gr)
    out = {"dcal": np.zeros((gr.nt, nrec))}
    out["hist"] = np.zeros((gr.nt + 1, 4, P)) if hist else None
    out["bands"] = np.zeros((int(lib().og_band_levels(C.byref(gr))), band_size(gr))) if bands else None
    out["final"] = np.zeros((4, P)) if final else None
    snap_it = np.ascontiguousarray(np.asarray(list(snaps), np.int32))
    out["snaps"] = np.zeros((len(snap_it), interior_size(gr)))
    init_a = None if init is None else np.ascontiguousarray(init, np.float64)
    rc = lib().og_forward(C.byref(gr), _d(vp), _d(rho), _i(src), _d(stf), nrec, _i(rec),
                          _d(out["dcal"]), _d(init_a), _d(out["hist"]), _d(out["bands"]),
                          _d(out["final"]), len(snap_it), _i(snap_it) if len(snap_it) else None,
                          _d(out["snaps"]) if len(snap_it) else None, _tp(st), _tp(rt))
    if rc:
        raise RuntimeError("og_forward failed: %d" % rc)
    return out


def reconstruct(gr: OgGrid, vp, rho, src, stf, bands, final, snaps: Sequence[int],
                st: Optional[Taps] = None):
    vp = np.ascontiguousarray(vp, np.float64)
    rho = np.ascontiguousarray(rho, np.float64)
    stf = np.ascontiguousarray(stf, np.float64)
    src = np.ascontiguousarray(src, np.int32)
    snap_it = np.ascontiguousarray(np.asarray(list(snaps), np.int32))
    out = np.zeros((len(snap_it), interior_size(gr)))
    rc = lib().og_reconstruct(C.byref(gr), _d(vp), _d(rho), _i(src), _d(stf),
                              _d(np.ascontiguousarray(bands)), _d(np.ascontiguousarray(final)),
                              len(snap_it), _i(snap_it), _d(out), _tp(st))
    if rc:
        raise RuntimeError("og_reconstruct failed: %d" % rc)
    return out


def adjoint(gr: OgGrid, vp, rho, src, stf, rec, G, *, hist=None, bands=None, final=None,
            want=("gk", "image", "illum"), st: Optional[Taps] = None, rt: Optional[Taps] = None,
            literal: bool = False, planted: int = 0, snaps: Sequence[int] = ()):
    """Reverse loop of Alg. 2 for one shot; returns interior gk (dJ/dkappa), image, illum and,
    when "grk" is wanted, dJ/drho at fixed kappa (the buoyancy part of eq. 7).  `literal` takes
    gk after both updates of each iteration, where Alg. 2 writes it (a comparison only).
    `planted` (tests of the pins only) puts a known mistake into the image: 1 pairs p^it with
    the adjoint field one level early, 2 drops the factor dt.  `snaps`: levels at which the
    source-field p of the interior (as the reverse loop rebuilds it) is returned as "snaps"."""
    vp = np.ascontiguousarray(vp, np.float64)
    rho = np.ascontiguousarray(rho, np.float64)
    stf = np.ascontiguousarray(stf, np.float64)
    src = np.ascontiguousarray(src, np.int32)
    rec = np.ascontiguousarray(np.asarray(rec, np.int32).reshape(-1, 3))
    G = np.ascontiguousarray(G, np.float64)
    I = interior_size(gr)
    gk = np.zeros(I) if "gk" in want else None
    im = np.zeros(I) if "image" in want else None
    il = np.zeros(I) if "illum" in want else None
    grk = np.zeros(I) if "grk" in want else None
    snap_it = np.ascontiguousarray(np.asarray(list(snaps), np.int32))
    sn = np.zeros((len(snap_it), I)) if len(snap_it) else None
    rc = lib().og_adjoint(C.byref(gr), _d(vp), _d(rho), _i(src), _d(stf), rec.shape[0], _i(rec),
                          _d(G), _d(None if hist is None else np.ascontiguousarray(hist)),
                          _d(None if bands is None else np.ascontiguousarray(bands)),
                          _d(None if final is None else np.ascontiguousarray(final)),
                          _d(gk), _d(im), _d(il), _d(grk), _tp(st), _tp(rt),
                          int(literal) | (2 if planted == 1 else 0) | (4 if planted == 2 else 0),
                          len(snap_it), _i(snap_it) if len(snap_it) else None, _d(sn))
    if rc:
        raise RuntimeError("og_adjoint failed: %d" % rc)
    return {"gk": gk, "image": im, "illum": il, "grk": grk, "snaps": sn}


def born(gr: OgGrid, vp, rho, src, stf, rec, dkappa, st: Optional[Taps] = None,
         rt: Optional[Taps] = None):
    vp = np.ascontiguousarray(vp, np.float64)
    rho = np.ascontiguousarray(rho, np.float64)
    stf = np.ascontiguousarray(stf, np.float64)
    src = np.ascontiguousarray(src, np.int32)
    rec = np.ascontiguousarray(np.asarray(rec, np.int32).reshape(-1, 3))
    dk = np.ascontiguousarray(dkappa, np.float64).ravel()
    dd = np.zeros((gr.nt, rec.shape[0]))
    rc = lib().og_born(C.byref(gr), _d(vp), _d(rho), _i(src), _d(stf), rec.shape[0], _i(rec),
                       _d(dk), _d(dd), _tp(st), _tp(rt))
    if rc:
        raise RuntimeError("og_born failed: %d" % rc)
    return dd


def react(gr: OgGrid, vp, rho, src, stf, rec, dm, *, eps: float = 0.0, lin: bool = True,
          st: Optional[Taps] = None, rt: Optional[Taps] = None):
    """The map whose exact transpose is the eq. (10) image (see og_react): with lin, the data
    of a field driven by dt kappa m p^it added before every step; without, the data of the
    forward run whose steps start with p *= 1 + eps dt kappa m (its finite-difference check)."""
    vp = np.ascontiguousarray(vp, np.float64)
    rho = np.ascontiguousarray(rho, np.float64)
    stf = np.ascontiguousarray(stf, np.float64)
    src = np.ascontiguousarray(src, np.int32)
    rec = np.ascontiguousarray(np.asarray(rec, np.int32).reshape(-1, 3))
    m = np.ascontiguousarray(dm, np.float64).ravel()
    out = np.zeros((gr.nt, rec.shape[0]))
    rc = lib().og_react(C.byref(gr), _d(vp), _d(rho), _i(src), _d(stf), rec.shape[0], _i(rec),
                        _d(m), float(eps), int(bool(lin)), _d(out), _tp(st), _tp(rt))
    if rc:
        raise RuntimeError("og_react failed: %d" % rc)
    return out


# ------------------------------------------------------------------ multi-shot jobs

def misfit(dcal: np.ndarray, dobs: np.ndarray, dt: float):
    """eq. (6) with the rectangle rule: J = 1/2 dt sum r^2; adjoint source G = dt r."""
    r = np.asarray(dcal, np.float64) - np.asarray(dobs, np.float64)
    return 0.5 * dt * float(np.sum(r * r)), dt * r


def model_vmax(job) -> float:
    return float(job.grid.vpmax) if getattr(job.grid, "vpmax", 0) else float(np.max(job.vp))


def forward_job(job, shots=None, vp=None, box=None, pml=1, vmax=None):
    """Seismograms of every (or the listed) shot: list of [nt, nrec_s] arrays."""
    vp = job.vp if vp is None else vp
    vmax = model_vmax(job) if vmax is None else vmax
    gr = og_grid(job.grid, vmax=vmax, pml=pml, box=box)
    shots = range(job.acq.nshot) if shots is None else shots
    out = []
    for s in shots:
        src, rec, st, rt = shot_ops(job.grid, job.acq, s)
        out.append(forward(gr, vp, job.rho, src, job.stf[s], rec, st=st, rt=rt)["dcal"])
    return out


def fwi_grad(job, dobs, shots=None, vp=None, box=None, vmax=None, use_history=False):
    """dJ/dVp (rho fixed) summed over shots in order, and J (eq. 6, 7; Alg. 2)."""
    vp = job.vp if vp is None else vp
    vmax = model_vmax(job) if vmax is None else vmax
    gr = og_grid(job.grid, vmax=vmax, box=box)
    shots = list(range(job.acq.nshot)) if shots is None else list(shots)
    gk = np.zeros(interior_size(gr))
    J = 0.0
    for k, s in enumerate(shots):
        src, rec, st, rt = shot_ops(job.grid, job.acq, s)
        fw = forward(gr, vp, job.rho, src, job.stf[s], rec, hist=use_history,
                     bands=not use_history, final=not use_history, st=st, rt=rt)
        Js, G = misfit(fw["dcal"], dobs[k], gr.dt)
        J += Js
        r = adjoint(gr, vp, job.rho, src, job.stf[s], rec, G, hist=fw["hist"],
                    bands=fw["bands"], final=fw["final"], want=("gk",), st=st, rt=rt)
        gk += r["gk"]
    vp64 = np.asarray(vp, np.float64).ravel()
    rho64 = np.asarray(job.rho, np.float64).ravel()
    return (2.0 * rho64 * vp64 * gk).reshape(job.vp.shape), J


def fwi_grad_family(job, dobs, family: int = 1, shots=None, vp=None, rho=None, box=None,
                    vmax=None, use_history=False):
    """eq. (7) with the chain rule of the two parametrisations of Sec. 2.2, summed over shots:
    family 1 -> (dJ/dVp at fixed rho, dJ/drho at fixed Vp); family 2 -> (dJ/dVp at fixed Ip,
    dJ/dIp at fixed Vp) with Ip = rho Vp; and J.  From dJ/dkappa (fixed rho) and dJ/drho (fixed
    kappa): kappa = rho Vp^2 gives dJ/dVp|rho = 2 rho Vp gk, dJ/drho|Vp = Vp^2 gk + grk;
    kappa = Ip Vp, rho = Ip / Vp give dJ/dVp|Ip = rho Vp gk - (rho / Vp) grk and
    dJ/dIp|Vp = Vp gk + grk / Vp."""
    vp = job.vp if vp is None else vp
    rho = job.rho if rho is None else rho
    vmax = model_vmax(job) if vmax is None else vmax
    gr = og_grid(job.grid, vmax=vmax, box=box)
    shots = list(range(job.acq.nshot)) if shots is None else list(shots)
    gk = np.zeros(interior_size(gr))
    grk = np.zeros(interior_size(gr))
    J = 0.0
    for k, s in enumerate(shots):
        src, rec, st, rt = shot_ops(job.grid, job.acq, s)
        fw = forward(gr, vp, rho, src, job.stf[s], rec, hist=use_history,
                     bands=not use_history, final=not use_history, st=st, rt=rt)
        Js, G = misfit(fw["dcal"], dobs[k], gr.dt)
        J += Js
        r = adjoint(gr, vp, rho, src, job.stf[s], rec, G, hist=fw["hist"],
                    bands=fw["bands"], final=fw["final"], want=("gk", "grk"), st=st, rt=rt)
        gk += r["gk"]
        grk += r["grk"]
    v = np.asarray(vp, np.float64).ravel()
    rh = np.asarray(rho, np.float64).ravel()
    if family == 1:
        g1, g2 = 2.0 * rh * v * gk, v * v * gk + grk
    elif family == 2:
        g1, g2 = rh * v * gk - (rh / v) * grk, v * gk + grk / v
    else:
        raise ValueError("family must be 1 or 2")
    return g1.reshape(job.vp.shape), g2.reshape(job.vp.shape), J


def rtm_image(job, dobs, shots=None, box=None, vmax=None, per_shot=False):
    """eq. (10): image and source illumination, summed over shots (G = dt dobs); with
    per_shot, the lists of each shot's image and illumination instead."""
    vmax = model_vmax(job) if vmax is None else vmax
    gr = og_grid(job.grid, vmax=vmax, box=box)
    shots = list(range(job.acq.nshot)) if shots is None else list(shots)
    ims, ils = [], []
    for k, s in enumerate(shots):
        src, rec, st, rt = shot_ops(job.grid, job.acq, s)
        fw = forward(gr, job.vp, job.rho, src, job.stf[s], rec, bands=True, final=True, st=st,
                     rt=rt)
        r = adjoint(gr, job.vp, job.rho, src, job.stf[s], rec, gr.dt * np.asarray(dobs[k]),
                    bands=fw["bands"], final=fw["final"], want=("image", "illum"), st=st,
                    rt=rt)
        ims.append(r["image"].reshape(job.vp.shape))
        ils.append(r["illum"].reshape(job.vp.shape))
    if per_shot:
        return ims, ils
    return np.sum(ims, axis=0), np.sum(ils, axis=0)


# Stabiliser of the source normalisation, as a fraction of each shot's peak illumination.
NORM_EPS = 1e-3


def normalized_image(images, illums, eps_frac: float = NORM_EPS):
    """Sec. 2.3, normalised imaging condition: each shot's image divided by that shot's
    source illumination, then summed over shots.  The paper gives no stabiliser; here the
    division is by illum_s + eps_frac * max(illum_s)."""
    out = np.zeros_like(np.asarray(images[0], np.float64))
    for im, il in zip(images, illums):
        il = np.asarray(il, np.float64)
        out += np.asarray(im, np.float64) / (il + eps_frac * np.max(il))
    return out


def laplacian(img, spacing):
    """Sec. 2.3, Laplace filter of an image: the second-order central-difference Laplacian
    sum_a (f[i+1] - 2 f[i] + f[i-1]) / d_a^2 over the image's axes, with zero outside the
    image.  `img` has numpy shape (n2, n1) or (n3, n2, n1); spacing = (d1, d2[, d3])."""
    f = np.asarray(img, np.float64)
    out = np.zeros_like(f)
    nd = f.ndim
    for a in range(nd):
        ax = nd - 1 - a                     # axis a (z = 0) is the last numpy axis
        d = float(spacing[a])
        pad = [(0, 0)] * nd
        pad[ax] = (1, 1)
        g = np.pad(f, pad)
        sl = lambda o: tuple(slice(1 + o, g.shape[i] - 1 + o) if i == ax else slice(None)
                             for i in range(nd))
        out += (g[sl(1)] - 2.0 * g[sl(0)] + g[sl(-1)]) / (d * d)
    return out
