"""Shot server: continuous batching of modelling / gradient / RTM requests on one GPU.

Requests (forward, FWI gradient or RTM jobs on their own grids and models) arrive over time.
The server keeps a FIFO queue; at every scheduling pass it

  * merges queued requests that share a grid and a model (same `model_key`) and a job kind
    into one multi-shot call (the library runs all shots of a call in one launch per step);
    requests that arrive while a call runs join the next call of their model.  Each member
    of a merged call gets its own result: its traces of the forward data, or its own
    gradient, misfit, image and illumination (the call runs with one shot group per
    request, so the library reduces each request's shots on their own);
  * admits calls while their HBM footprint (workspace from smi_workspace_bytes + data and
    result buffers) fits the remaining budget and a stream is free -- later, smaller calls
    may pass a call that does not fit yet (backfill);
  * launches each admitted call on its own HIP stream, so calls admitted while others run
    overlap on the device;
  * polls completion events, frees the call's memory and records per-request latency
    (completion - arrival) and the call's algorithmic HBM bytes.

Models stay on the device between calls: `HipBackend` keeps the device copies of (vp, rho)
per model_key in a bounded cache (least recently used first out, never while a call uses
them), so a request on a resident model uploads only its wavelet (and observed data).

A failing request (validation error) fails alone; the rest of the stream continues.  The
scheduling logic is independent of the device: `HipBackend` runs calls through the C ABI,
`FakeBackend` simulates durations on a virtual clock for CPU tests.
"""
from __future__ import annotations

import dataclasses
import math
import threading
import time
from collections import OrderedDict, deque
from typing import Any, Dict, List, Optional

import numpy as np

from . import inputs as I


@dataclasses.dataclass(eq=False)
class Request:
    kind: str                     # "forward" | "grad" | "rtm"
    job: I.Job                    # grid, model, acquisition, wavelet (host arrays)
    arrival: float = 0.0          # seconds after the stream start
    dobs: Optional[np.ndarray] = None   # flat observed data (grad, rtm)
    model_key: Optional[str] = None     # requests with equal keys share grid + model
    rid: int = -1


@dataclasses.dataclass
class Outcome:
    rid: int
    kind: str
    ok: bool
    latency: float = float("nan")
    result: Any = None
    error: str = ""
    gpts: float = 0.0
    batch: int = 1


def _grid_sig(g) -> tuple:
    return (g.ndim, g.n1, g.n2, g.n3, g.d1, g.d2, g.d3, g.nb, g.order, g.nt, g.dt, g.fm, g.dr,
            g.box, g.margin)


def merge_requests(reqs: List[Request]) -> I.Job:
    """One multi-shot job from requests that share grid and model."""
    base = reqs[0].job
    src = np.concatenate([r.job.acq.src for r in reqs])
    recs = [r.job.acq.rec for r in reqs]
    off = np.zeros(len(src) + 1, np.int32)
    k = 0
    for r in reqs:
        for s in range(r.job.acq.nshot):
            off[k + 1] = off[k] + r.job.acq.nrec(s)
            k += 1
    acq = I.Acquisition(src, off, np.concatenate(recs) if recs else np.zeros((0, 3)))
    stf = np.concatenate([r.job.stf for r in reqs])
    return I.Job(base.grid, base.vp, base.rho, acq, stf, name="+".join(r.job.name for r in reqs))


class _ModelCache:
    """Device copies of (vp, rho) per model_key within `cap` bytes, least recently used out
    first; an entry that an in-flight call uses is never evicted.  An upload is enqueued on
    the stream of the call that needs it; a call on another stream waits for its event."""

    def __init__(self, cap: int):
        self.cap = cap
        self.used = 0
        self.d: "OrderedDict[str, dict]" = OrderedDict()
        self.lock = threading.Lock()
        self.hits = 0
        self.misses = 0

    def acquire(self, key, job, torch, dev, stream):
        nb = 4 * (job.vp.size + job.rho.size)
        with self.lock:
            e = self.d.get(key)
            if e is not None:
                self.d.move_to_end(key)
                e["users"] += 1
                self.hits += 1
                return e
            self.misses += 1
            for k in [k for k, v in self.d.items() if v["users"] == 0]:
                if self.used + nb <= self.cap:
                    break
                self.used -= self.d.pop(k)["bytes"]
            if self.used + nb > self.cap:
                return None                  # no room: the call uploads a private copy
            with torch.cuda.stream(stream):
                vp = torch.from_numpy(np.ascontiguousarray(job.vp)).to(dev)
                rho = torch.from_numpy(np.ascontiguousarray(job.rho)).to(dev)
                ev = torch.cuda.Event()
                ev.record(stream)
            e = {"vp": vp, "rho": rho, "ready": ev, "users": 1, "bytes": nb}
            self.d[key] = e
            self.used += nb
            return e

    def resident(self, key) -> bool:
        with self.lock:
            return key in self.d

    def release(self, key):
        with self.lock:
            e = self.d.get(key)
            if e is not None:
                e["users"] -= 1


class HipBackend:
    """Runs calls through libsmi on one device: one HIP stream, one library context and one
    host thread per in-flight slot.  Enqueueing a call's time loop costs a few microseconds of
    host time per launch, which for small single-shot calls is as long as the device work, so
    the slots enqueue in parallel (the library call releases the interpreter lock; a context
    is used by one thread at a time).  Models with a model_key stay resident in a bounded
    device cache of `cache_frac` of the free memory."""

    def __init__(self, device: int = 0, nstreams: int = 4, cache_frac: float = 0.1):
        import torch
        from concurrent.futures import ThreadPoolExecutor
        from . import binding as B
        self.torch = torch
        self.B = B
        self.dev = f"cuda:{device}"
        self.ctxs = [B.Context(device) for _ in range(nstreams)]
        self.ctx = self.ctxs[0]
        self.streams = [torch.cuda.Stream(device=self.dev) for _ in range(nstreams)]
        self.pool = ThreadPoolExecutor(max_workers=nstreams)
        free, _ = torch.cuda.mem_get_info(self.dev)
        self.models = _ModelCache(int(cache_frac * free))

    def budget(self, frac: float = 0.85) -> int:
        """Bytes the calls' own buffers may take: a share of the free memory, less what the
        model cache may hold."""
        free, _ = self.torch.cuda.mem_get_info(self.dev)
        return int(frac * (free + self.models.used)) - self.models.cap

    def footprint(self, job: I.Job, kind: str, model_key: Optional[str] = None) -> int:
        B = self.B
        jobtype = {"forward": B.JOB_FORWARD, "grad": B.JOB_GRAD, "rtm": B.JOB_RTM}[kind]
        ws = self.ctx.workspace_bytes(job.grid, job.acq, jobtype)
        nrec = int(job.acq.rec_off[-1])
        data = 4 * job.grid.nt * nrec * (2 if kind != "forward" else 1)
        results = 4 * job.grid.npts * (2 if kind != "forward" else 0) * max(1, job.acq.nshot)
        # the model counts unless it is resident already (an upload into the cache, or a private
        # copy when the cache has no room, both need the bytes)
        model = 0 if model_key is not None and self.models.resident(model_key) else 4 * job.grid.npts * 2
        return ws + data + results + model + 4 * job.stf.size

    def _run(self, job: I.Job, kind: str, dobs: Optional[np.ndarray], slot: int,
             parts: List[int], model_key: Optional[str]):
        torch = self.torch
        st = self.streams[slot]
        ctx = self.ctxs[slot]
        ent = self.models.acquire(model_key, job, torch, self.dev, st) if model_key else None
        with torch.cuda.stream(st):
            if ent is not None:
                st.wait_event(ent["ready"])
                vp, rho = ent["vp"], ent["rho"]
            else:
                vp = torch.from_numpy(np.ascontiguousarray(job.vp)).to(self.dev)
                rho = torch.from_numpy(np.ascontiguousarray(job.rho)).to(self.dev)
            stf = torch.from_numpy(np.ascontiguousarray(job.stf)).to(self.dev)
            jt = {"forward": self.B.JOB_FORWARD, "grad": self.B.JOB_GRAD, "rtm": self.B.JOB_RTM}[kind]
            ws = torch.empty(ctx.workspace_bytes(job.grid, job.acq, jt), dtype=torch.uint8,
                             device=self.dev)
            groups = np.concatenate([[0], np.cumsum(parts)]).astype(np.int32)
            try:
                if kind == "forward":
                    out, _, _ = ctx.forward(job.grid, job.acq, vp, rho, stf, ws=ws, stream=st)
                    keep = (vp, rho, stf, ws, out)
                else:
                    d = torch.from_numpy(np.ascontiguousarray(dobs, np.float32)).to(self.dev)
                    # one shot group per request: each gets its own reduced outputs
                    ctx.set_shot_groups(groups if len(parts) > 1 else None)
                    if kind == "grad":
                        g, J, _ = ctx.fwi_grad(job.grid, job.acq, vp, rho, stf, d, ws=ws, stream=st)
                        out = (g, J)
                    else:
                        out = ctx.rtm_image(job.grid, job.acq, vp, rho, stf, d, ws=ws, stream=st)
                    keep = (vp, rho, stf, ws, d, out)
            finally:
                if kind != "forward" and len(parts) > 1:
                    ctx.set_shot_groups(None)
            ev = torch.cuda.Event()
            ev.record(st)
        return {"ev": ev, "out": out, "keep": keep, "gpts": sum(ctx.last_counts()),
                "bytes": sum(ctx.last_bytes()), "groups": groups, "kind": kind,
                "rec_off": np.asarray(job.acq.rec_off), "nt": job.grid.nt,
                "npts": job.grid.npts}

    def launch(self, job: I.Job, kind: str, dobs: Optional[np.ndarray], slot: int,
               parts: Optional[List[int]] = None, model_key: Optional[str] = None):
        parts = parts or [job.acq.nshot]
        return {"fut": self.pool.submit(self._run, job, kind, dobs, slot, parts, model_key),
                "key": model_key}

    def done(self, h) -> bool:
        f = h["fut"]
        if not f.done():
            return False
        return f.exception() is not None or f.result()["ev"].query()

    def results(self, h) -> list:
        """One result per request of the call, in the order of `parts`: the request's own
        traces (forward), (gradient, misfit) or (image, illumination)."""
        r = h["fut"].result()                   # re-raises an error of the call
        grp, n = r["groups"], len(r["groups"]) - 1
        if r["kind"] == "forward":
            d = r["out"].cpu().numpy()
            off, nt = r["rec_off"], r["nt"]
            return [d[nt * int(off[grp[k]]): nt * int(off[grp[k + 1]])] for k in range(n)]
        host = tuple(None if o is None else o.cpu().numpy() for o in r["out"])
        npts = r["npts"]
        out = []
        for k in range(n):
            if r["kind"] == "grad":
                out.append((host[0][k * npts:(k + 1) * npts], host[1][k:k + 1]))
            else:
                out.append(tuple(None if o is None else o[k * npts:(k + 1) * npts] for o in host))
        return out

    def finish(self, h):
        """The call has ended: its model may leave the cache again."""
        if h.get("key"):
            self.models.release(h["key"])

    def gpts(self, h) -> float:
        f = h["fut"]
        return f.result()["gpts"] if f.exception() is None else 0.0

    def nbytes(self, h) -> float:
        f = h["fut"]
        return f.result()["bytes"] if f.exception() is None else 0.0

    def now(self) -> float:
        return time.perf_counter()

    def idle(self):
        time.sleep(2e-4)


class FakeBackend:
    """Virtual-clock backend for CPU tests: a call takes `cost(job)` seconds once launched,
    calls on different slots overlap; `fail(job)` makes a launch raise."""

    def __init__(self, cost=None, fail=None, footprint=None):
        self.t = 0.0
        self.cost = cost or (lambda job, kind: 1e-3 * job.acq.nshot)
        self.fail = fail or (lambda job, kind: False)
        self.fp = footprint or (lambda job, kind: 1)
        self.running = []
        self.launched = []

    def budget(self, frac: float = 0.85) -> int:
        return 1 << 60

    def footprint(self, job, kind, model_key=None) -> int:
        return self.fp(job, kind)

    def launch(self, job, kind, dobs, slot, parts=None, model_key=None):
        if self.fail(job, kind):
            raise RuntimeError("SMI_E_ARG: injected failure")
        parts = parts or [job.acq.nshot]
        h = {"end": self.t + self.cost(job, kind), "job": job, "slot": slot, "parts": parts}
        self.launched.append((self.t, job.name, slot))
        return h

    def done(self, h) -> bool:
        return self.t >= h["end"] - 1e-15

    def results(self, h):
        """Per request: the call's name and the request's shot range in the call."""
        off = np.concatenate([[0], np.cumsum(h["parts"])])
        return [(h["job"].name, int(off[k]), int(off[k + 1])) for k in range(len(h["parts"]))]

    def finish(self, h):
        pass

    def gpts(self, h) -> float:
        return 0.0

    def nbytes(self, h) -> float:
        return float(self.fp(h["job"], "forward"))

    def now(self) -> float:
        return self.t

    def idle(self, pending_arrivals: Optional[float] = None, ends: Optional[List[float]] = None):
        cands = [e for e in (ends or []) if e > self.t]
        if pending_arrivals is not None and pending_arrivals > self.t:
            cands.append(pending_arrivals)
        self.t = min(cands) if cands else self.t + 1e-3


class ShotServer:
    def __init__(self, backend, budget_bytes: Optional[int] = None, max_inflight: int = 4,
                 max_batch_shots: int = 64, batch: bool = True):
        self.be = backend
        self.budget = budget_bytes if budget_bytes is not None else backend.budget()
        self.max_inflight = max_inflight
        self.max_batch = max_batch_shots
        self.batch = batch
        self.log: List[str] = []

    def _batches(self, queue: deque) -> List[List[Request]]:
        """Group queued requests (FIFO order of first member) into compatible calls."""
        groups: Dict[tuple, List[Request]] = {}
        order = []
        for r in queue:
            if self.batch and r.model_key is not None and r.kind in ("forward", "rtm", "grad"):
                key = (r.kind, r.model_key, _grid_sig(r.job.grid))
            else:
                key = ("solo", r.rid)
            if key not in groups:
                groups[key] = []
                order.append(key)
            g = groups[key]
            if sum(x.job.acq.nshot for x in g) + r.job.acq.nshot <= self.max_batch or not g:
                g.append(r)
        return [groups[k] for k in order]

    def run(self, requests: List[Request]) -> Dict[str, Any]:
        reqs = sorted(requests, key=lambda r: r.arrival)
        for i, r in enumerate(reqs):
            if r.rid < 0:
                r.rid = i
        be = self.be
        t0 = be.now()
        pending = deque(reqs)
        queue: deque = deque()
        inflight = []                 # (handle, [requests], footprint, slot)
        free_slots = list(range(self.max_inflight))
        used = 0
        outcomes: Dict[int, Outcome] = {}
        total_gpts = 0.0
        total_bytes = 0.0
        calls: List[int] = []         # requests per completed call
        while pending or queue or inflight:
            now = be.now() - t0
            while pending and pending[0].arrival <= now:
                queue.append(pending.popleft())
            # completions
            still = []
            for h, rs, fp, slot in inflight:
                if be.done(h):
                    tdone = be.now() - t0
                    be.finish(h)
                    try:
                        res = be.results(h)
                    except Exception as e:      # an error raised while the call ran
                        for r in rs:
                            outcomes[r.rid] = Outcome(r.rid, r.kind, False, error=str(e))
                        used -= fp
                        free_slots.append(slot)
                        continue
                    for k, r in enumerate(rs):
                        outcomes[r.rid] = Outcome(r.rid, r.kind, True, tdone - r.arrival,
                                                  res[k], gpts=be.gpts(h) / len(rs),
                                                  batch=len(rs))
                    total_gpts += be.gpts(h)
                    total_bytes += be.nbytes(h)
                    calls.append(len(rs))
                    used -= fp
                    free_slots.append(slot)
                else:
                    still.append((h, rs, fp, slot))
            inflight = still
            # admissions (FIFO with backfill)
            launched_any = False
            if queue and free_slots:
                for grp in self._batches(queue):
                    if not free_slots:
                        break
                    job = merge_requests(grp) if len(grp) > 1 else grp[0].job
                    kind = grp[0].kind
                    key = grp[0].model_key if len({r.model_key for r in grp}) == 1 else None
                    try:
                        fp = be.footprint(job, kind, key)
                    except Exception as e:      # validation error: this request fails alone
                        for r in grp:
                            outcomes[r.rid] = Outcome(r.rid, r.kind, False, error=str(e))
                            queue.remove(r)
                        continue
                    if fp > self.budget:
                        for r in grp:
                            outcomes[r.rid] = Outcome(r.rid, r.kind, False,
                                                      error=f"footprint {fp} B exceeds the budget")
                            queue.remove(r)
                        continue
                    if used + fp > self.budget:
                        continue                 # waits for memory; smaller calls may pass
                    dobs = None
                    if kind != "forward":
                        dobs = np.concatenate([np.ravel(r.dobs) for r in grp])
                    slot = free_slots.pop()
                    try:
                        h = be.launch(job, kind, dobs, slot, [r.job.acq.nshot for r in grp], key)
                    except Exception as e:
                        free_slots.append(slot)
                        for r in grp:
                            outcomes[r.rid] = Outcome(r.rid, r.kind, False, error=str(e))
                            queue.remove(r)
                        continue
                    used += fp
                    for r in grp:
                        queue.remove(r)
                    inflight.append((h, grp, fp, slot))
                    launched_any = True
            if not launched_any:
                if isinstance(be, FakeBackend):
                    be.idle(pending[0].arrival + t0 if pending else None,
                            [h["end"] for h, _, _, _ in inflight])
                else:
                    be.idle()
        makespan = be.now() - t0
        lat = np.array([o.latency for o in outcomes.values() if o.ok])
        return {"outcomes": [outcomes[r.rid] for r in reqs],
                "p50": float(np.percentile(lat, 50)) if lat.size else math.nan,
                "p99": float(np.percentile(lat, 99)) if lat.size else math.nan,
                "makespan": makespan, "gpts": total_gpts,
                "gpts_per_s": total_gpts / makespan if makespan > 0 else math.nan,
                # algorithmic HBM bytes of every completed call (the library's count of the
                # fields, model and tables a call must move) over the makespan
                "alg_bytes": total_bytes,
                "alg_GBps": total_bytes / makespan / 1e9 if makespan > 0 else math.nan,
                "calls": len(calls), "merged_calls": sum(1 for c in calls if c > 1),
                "requests_per_call": float(np.mean(calls)) if calls else math.nan,
                "failed": sum(1 for o in outcomes.values() if not o.ok)}
