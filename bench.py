"""Throughput benchmark of the batched staggered-grid forward modelling on one MI355X.

Workload (the configuration the headline metric is quoted on): 2D batched forward modelling,
500 x 1500 cells of 10 m, 10 dipping layers 1500-4500 m/s with a +-5% smoothed random
perturbation (seeded), Gardner density, order 8, 30 CPML layers, Ricker 15 Hz, dt 0.8 ms,
nt 4000, 16 shots spread along the surface in one launch, 1500 receivers each, evolving
computing box on.  One bench "step" = one whole job: smi_forward over all 16 shots and all
4000 time steps (model preparation, every time step of every shot, every seismogram sample).

Reported: grid-point updates per second (a GPt = one cell of a shot's computing box advanced
by one time step), p50/p99 of the step time, the plain one-shot-per-launch stepper on the same
GPU, the fraction of the HBM roofline reached by the forward step kernels, and the FP64 oracle
timed on the host cores.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "grid-point updates/s (GPts/s) and % HBM roofline, batched vs plain; p50/p99"
HBM_PEAK_GBS = 8000.0


def percentile(xs, q):
    return float(np.percentile(np.asarray(xs), q))


def cpu_baseline(job, steps: int, one_thread_steps: int = 200):
    """The FP64 oracle on the host cores: one shot, `steps` time steps at full spatial size,
    computing box off (the plain definition); rate in GPts/s of the same cell-step count."""
    from oracle import oracle as O
    import copy
    g = copy.copy(job.grid)
    g.nt = steps
    gr = O.og_grid(g, vmax=float(job.grid.vpmax), box=0)
    src, rec = O.shot_nodes(g, job.acq, 0)
    O.lib()
    t0 = time.perf_counter()
    O.forward(gr, job.vp, job.rho, src, job.stf[0][:steps], rec)
    dt = time.perf_counter() - t0
    cells = O.padded_size(gr) * steps
    threads = int(os.environ.get("OMP_NUM_THREADS", len(os.sched_getaffinity(0))))
    out = {"value": cells / dt / 1e9, "unit": "GPts/s", "cores": threads, "kind": "oracle",
           "sample": f"1 shot x {steps} of {job.grid.nt} steps, full padded grid "
                     f"{g.n1 + 2 * g.nb}x{g.n2 + 2 * g.nb}, FP64, box off; {dt:.1f} s"}
    # the same oracle on one thread (OpenMP runtime of the oracle's library), a shorter sample
    try:
        import ctypes
        gomp = ctypes.CDLL("libgomp.so.1")
        gomp.omp_set_num_threads(1)
        g1 = copy.copy(g)
        g1.nt = one_thread_steps
        gr1 = O.og_grid(g1, vmax=float(job.grid.vpmax), box=0)
        t0 = time.perf_counter()
        O.forward(gr1, job.vp, job.rho, src, job.stf[0][:one_thread_steps], rec)
        d1 = time.perf_counter() - t0
        gomp.omp_set_num_threads(threads)
        out["one_thread"] = {"value": O.padded_size(gr1) * one_thread_steps / d1 / 1e9,
                             "unit": "GPts/s", "cores": 1,
                             "sample": f"1 shot x {one_thread_steps} steps; {d1:.1f} s"}
    except OSError:
        out["one_thread"] = None
    return out


def probe_copy(torch, gib: float = 1.0, reps: int = 20):
    """A plain device-to-device copy of known size: the reference the HBM counters of the
    step kernels are scaled by (bytes read = bytes written = `gib` GiB per copy)."""
    n = int(gib * (1 << 30)) // 4
    a = torch.ones(n, dtype=torch.float32, device="cuda:0")
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    print(json.dumps({"probe": "copy", "bytes_read": 4 * n, "bytes_written": 4 * n,
                      "ms": ms, "GBps": 8 * n / (ms / 1e3) / 1e9}), flush=True)


# HBM traffic of the step kernels from rocprofv3 counter runs, kept with the profiles: valid
# only while the kernel source is the one the counters were taken on.
COUNTERS = os.path.join(ROOT, "profiles", "step_kernels_2d_order8_16shots_counters.txt")
KERNEL_SRC = os.path.join(ROOT, "paper_2311_02293_amd", "csrc", "kernels.hip")
# the library's default step configuration on the batched 2D workload, by the autotuner's name:
# register-blocked marching kernels, 4 cells per lane, tiles dealt round-robin over the XCDs
DEFAULT_CONFIG = "march4-xcd"


def counter_traffic(config: str):
    """HBM bytes per step from the counter file, or None unless the counters were taken on the
    same kernel source and the same step kernel configuration (`config`, the autotuner's name
    of the timed configuration)."""
    import hashlib
    try:
        kv = {}
        with open(COUNTERS) as f:
            for line in f:
                if ":" in line and not line.startswith("#"):
                    k, v = line.split(":", 1)
                    kv[k.strip()] = v.strip()
        with open(KERNEL_SRC, "rb") as f:
            src = hashlib.sha256(f.read()).hexdigest()
        if kv.get("kernel_source_sha256") != src or kv.get("kernel_config") != config:
            return None
        return float(kv["traffic_bytes_per_step"])
    except (OSError, KeyError, ValueError):
        return None


def latency(torch, graph: bool = False, only: str = "", reps_override: int = 0,
            kernel: int = -1, chunk: int = -1, nt: int = 0):
    """Per-call latency of the four fixed workloads: repetitions of the library call after two
    warm-ups, each timed with events on the call's stream; one JSON line per workload.  With
    `graph`, the two forward workloads with their time loops replayed as HIP graphs.  `only`
    keeps the workloads whose name contains it; `reps_override` > 0 replaces the repetitions;
    `kernel` / `chunk` >= 0 set SMI_OPT_KERNEL / SMI_OPT_CHUNK; `nt` > 0 shortens the runs."""
    from paper_2311_02293_amd import binding as B
    from paper_2311_02293_amd import inputs as I

    ctx = B.Context(0)
    if graph:
        ctx.set_option(B.OPT_GRAPH, 1)
    if kernel >= 0:
        ctx.set_option(B.OPT_KERNEL, kernel)
    if chunk >= 0:
        ctx.set_option(B.OPT_CHUNK, chunk)
    stream = torch.cuda.current_stream()
    def full_grid_3d(nt: int = 3000):
        # the 3D RTM's grid, model and shots, forward only, box off: every step updates the
        # whole padded grid (the step's steady state, which the box reaches after ~1000 steps)
        job = I.config4(nt=nt)
        job.grid.box = 0
        return job
    cases = [("2d-forward-201x201-order4-1shot", I.config1, "forward", 20),
             ("2d-batched-forward-500x1500-order8-16shots", I.config2, "forward", 20),
             ("2d-fwi-gradient-300x900-order8-32shots", I.config3, "grad", 20),
             ("3d-rtm-400^3-order8-4shots-dr10", I.config4, "rtm", 2),
             ("3d-full-grid-forward-400^3-order8-4shots", full_grid_3d, "forward", 2)]
    if graph:
        cases = [c for c in cases if c[2] == "forward"]
    # the full-grid 3D forward runs only when named
    cases = [c for c in cases if only in c[0] and (only or not c[0].startswith("3d-full-grid"))]
    if not cases:
        raise SystemExit(f"no latency workload matches {only!r}")
    for name, make, kind, reps in cases:
        job = make(nt=nt) if nt > 0 else make()
        reps = reps_override if reps_override > 0 else reps
        vs = [job.vp] + ([job.extra["vp_true"]] if "vp_true" in job.extra else [])
        job.grid.vpmin = float(min(v.min() for v in vs))
        job.grid.vpmax = float(max(v.max() for v in vs))
        vp, rho, stf = (torch.from_numpy(np.ascontiguousarray(a)).cuda()
                        for a in (job.vp, job.rho, job.stf))
        jt = {"forward": B.JOB_FORWARD, "grad": B.JOB_GRAD, "rtm": B.JOB_RTM}[kind]
        ws = ctx.workspace(ctx.workspace_bytes(job.grid, job.acq, jt))
        dobs = None
        if kind != "forward":
            vt = torch.from_numpy(job.extra["vp_true"]).cuda()
            dobs, _, _ = ctx.forward(job.grid, job.acq, vt, rho, stf)

        # one output buffer for every call (a captured graph is keyed by its buffers)
        dcal = torch.empty(job.grid.nt * int(job.acq.rec_off[-1]), dtype=torch.float32, device="cuda")

        def call():
            if kind == "forward":
                ctx.forward(job.grid, job.acq, vp, rho, stf, dcal=dcal, ws=ws, stream=stream)
            elif kind == "grad":
                ctx.fwi_grad(job.grid, job.acq, vp, rho, stf, dobs, ws=ws, stream=stream)
            else:
                ctx.rtm_image(job.grid, job.acq, vp, rho, stf, dobs, ws=ws, stream=stream)
        print(f"bench: latency {name}", file=sys.stderr, flush=True)
        for w in range(2):
            call()
            torch.cuda.synchronize()
            print(f"bench: {name} warm-up {w} done", file=sys.stderr, flush=True)
        ms = []
        for r in range(reps):
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record(stream)
            call()
            b.record(stream)
            torch.cuda.synchronize()
            ms.append(a.elapsed_time(b))
            print(f"bench: {name} rep {r}: {ms[-1]:.1f} ms", file=sys.stderr, flush=True)
        upd = sum(ctx.last_counts())
        print(json.dumps({"metric": "per-call latency", "workload": name, "call": kind,
                          "nt": job.grid.nt, "kernel_option": kernel, "chunk_option": chunk,
                          "graph_replay": graph, "reps": reps,
                          "warmup": 2, "p50_ms": percentile(ms, 50), "p99_ms": percentile(ms, 99),
                          "GPts_s": upd / (np.median(ms) / 1e3) / 1e9,
                          "data": "synthetic", "dtype": "f32"}), flush=True)
        del ws, dobs


def reverse_leg(torch, reps: int = 5, timing_every: int = 32):
    """The 2D FWI gradient workload (300 x 900, order 8, 32 shots, nt 4000, box on, bands at
    every step): per-call p50 / p99 of smi_fwi_grad, GPts/s of its forward + adjoint +
    reconstruction cell updates, and the reverse iteration's algorithmic GB/s from device-
    stamped events around every `timing_every`-th reverse iteration of one more call.  The
    observed data are the same library's forward data of the true model (synthetic)."""
    from paper_2311_02293_amd import binding as B
    from paper_2311_02293_amd import inputs as I
    job = I.config3()
    vt = job.extra["vp_true"]
    job.grid.vpmin = float(min(job.vp.min(), vt.min()))
    job.grid.vpmax = float(max(job.vp.max(), vt.max()))
    vp, rho, stf = (torch.from_numpy(np.ascontiguousarray(a)).cuda() for a in (job.vp, job.rho, job.stf))
    ctx = B.Context(0)
    stream = torch.cuda.current_stream()
    ws = ctx.workspace(ctx.workspace_bytes(job.grid, job.acq, B.JOB_GRAD))
    dobs, _, _ = ctx.forward(job.grid, job.acq, torch.from_numpy(vt).cuda(), rho, stf)

    def call():
        ctx.fwi_grad(job.grid, job.acq, vp, rho, stf, dobs, ws=ws, stream=stream)
    print("bench: reverse leg warm-up", file=sys.stderr, flush=True)
    call()
    torch.cuda.synchronize()
    ms = []
    for r in range(reps):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        call()
        b.record(stream)
        torch.cuda.synchronize()
        ms.append(a.elapsed_time(b))
        print(f"bench: reverse leg rep {r}: {ms[-1]:.1f} ms", file=sys.stderr, flush=True)
    upd = sum(ctx.last_counts())
    fwd_bytes, rev_bytes = ctx.last_bytes()
    ctx.set_option(B.OPT_TIMING, timing_every)
    call()
    torch.cuda.synchronize()
    rms, rby, rn = ctx.kernel_timing(3)
    fv, fb, _ = ctx.kernel_timing(1)
    fp, _, _ = ctx.kernel_timing(2)
    fs_bytes = ctx.kernel_timing(0)[1]
    ctx.set_option(B.OPT_TIMING, 0)
    rev_GBps = rby / (rms / 1e3) / 1e9 if rms > 0 else None
    fwd_us = (fv + fp) * 1e3
    out = {"workload": job.name, "call": "smi_fwi_grad", "reps": reps, "warmup": 1,
           "p50_ms": percentile(ms, 50), "p99_ms": percentile(ms, 99),
           "value": upd / (np.median(ms) / 1e3) / 1e9, "unit": "GPts/s",
           "gpts_per_call": upd,
           "whole_call_alg_GBps": (fwd_bytes + rev_bytes) / (np.median(ms) / 1e3) / 1e9,
           "reverse_step": {"avg_us": rms * 1e3, "alg_bytes": rby, "samples": rn,
                            "achieved_GBps": rev_GBps, "peak_GBps": HBM_PEAK_GBS,
                            "frac": rev_GBps / HBM_PEAK_GBS if rev_GBps else None,
                            "what": "one reverse iteration of Alg. 2 (adjoint source, source "
                                    "removal, reconstruction with the gradient sum, adjoint "
                                    "step) over one group of the shots, first launch to end of "
                                    "last: the reverse loop runs once per group of shots whose "
                                    "reverse state fits the last-level cache (SMI_OPT_REV_GROUP; "
                                    "two groups of 16 here)"},
           "forward_step": {"avg_us": fwd_us, "alg_bytes": fs_bytes,
                            "achieved_GBps": fs_bytes / (fwd_us / 1e6) / 1e9 if fwd_us > 0 else None}}
    del ws, dobs
    return out


def serve(torch, njobs: int, pool: int = 6):
    """Served stream of mixed requests, one shot each, over `pool` seeded surveys per job class
    (the models stay resident on the device; requests of one survey that queue together share
    a launch): a capacity run (every request queued at t = 0), then the same requests arriving
    as a Poisson stream at 0.7 x that capacity (latency p50 / p99, algorithmic GB/s and its
    fraction of HBM peak), then every request alone on the plain stepper (one shot per launch,
    box off)."""
    from paper_2311_02293_amd import binding as B
    from paper_2311_02293_amd import inputs as I
    from paper_2311_02293_amd.server import HipBackend, Request, ShotServer

    be = HipBackend(0, nstreams=4)
    jobs = I.stream_config5(njobs=njobs, rate=1.0, seed=1005, pool=pool)
    gaps = np.diff([0.0] + [sj.arrival for sj in jobs])     # unit-rate exponential gaps
    reqs = []
    for sj in jobs:
        j = sj.job
        vs = [j.vp] + ([j.extra["vp_true"]] if "vp_true" in j.extra else [])
        j.grid.vpmin = float(min(v.min() for v in vs))
        j.grid.vpmax = float(1.02 * max(v.max() for v in vs))
        kind = "grad" if sj.kind == "grad2d" else "forward"
        r = Request(kind, j, arrival=0.0, model_key=sj.model_key)
        if kind == "grad":          # observed data: forward of the true model, before the stream
            rho = torch.from_numpy(j.rho).cuda()
            stf = torch.from_numpy(j.stf).cuda()
            vt = torch.from_numpy(j.extra["vp_true"]).cuda()
            d, _, _ = be.ctx.forward(j.grid, j.acq, vt, rho, stf)
            r.dobs = d.cpu().numpy()
        reqs.append(r)
    torch.cuda.synchronize()
    counts = {k: sum(1 for r in reqs if (r.kind, r.job.grid.ndim) == k)
              for k in (("forward", 2), ("grad", 2), ("forward", 3))}
    print(f"bench: serve {njobs} requests {counts}", file=sys.stderr, flush=True)
    srv = ShotServer(be, max_inflight=4)
    cap = srv.run(reqs)
    capacity = njobs / cap["makespan"]
    print(f"bench: capacity {capacity:.2f} requests/s", file=sys.stderr, flush=True)
    rate = 0.7 * capacity
    t = 0.0
    for r, gp in zip(reqs, gaps):
        t += gp / rate
        r.arrival = t
    srv = ShotServer(be, max_inflight=4)
    st = srv.run(reqs)
    print("bench: plain stepper, every request alone", file=sys.stderr, flush=True)
    be.ctx.set_option(B.OPT_KERNEL, 1)
    plain_s, plain_gpts = 0.0, 0.0
    for k, r in enumerate(reqs):
        if k % 50 == 0:
            print(f"bench: plain request {k}", file=sys.stderr, flush=True)
        j = r.job
        box = j.grid.box
        j.grid.box = 0
        vp, rho, stf = (torch.from_numpy(np.ascontiguousarray(a)).cuda() for a in (j.vp, j.rho, j.stf))
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        if r.kind == "forward":
            be.ctx.forward(j.grid, j.acq, vp, rho, stf)
        else:
            be.ctx.fwi_grad(j.grid, j.acq, vp, rho, stf, torch.from_numpy(r.dobs).cuda())
        torch.cuda.synchronize()
        plain_s += time.perf_counter() - t0
        plain_gpts += sum(be.ctx.last_counts())
        j.grid.box = box
    be.ctx.set_option(B.OPT_KERNEL, 0)
    print(json.dumps({
        "metric": "served shot stream: requests/s, GPts/s, latency p50/p99",
        "requests": njobs, "mix": {"forward2d": counts[("forward", 2)], "grad2d": counts[("grad", 2)],
                                   "forward3d": counts[("forward", 3)]},
        "surveys_per_class": pool,
        "capacity": {"requests_per_s": capacity, "GPts_s": cap["gpts_per_s"] / 1e9,
                     "makespan_s": cap["makespan"], "failed": cap["failed"],
                     "alg_GBps": cap["alg_GBps"], "hbm_frac": cap["alg_GBps"] / HBM_PEAK_GBS,
                     "calls": cap["calls"], "merged_calls": cap["merged_calls"],
                     "requests_per_call": cap["requests_per_call"]},
        "stream": {"arrival_rate_per_s": rate, "p50_s": st["p50"], "p99_s": st["p99"],
                   "GPts_s": st["gpts_per_s"] / 1e9, "makespan_s": st["makespan"], "failed": st["failed"],
                   "alg_GBps": st["alg_GBps"], "hbm_frac": st["alg_GBps"] / HBM_PEAK_GBS,
                   "calls": st["calls"], "merged_calls": st["merged_calls"],
                   "requests_per_call": st["requests_per_call"]},
        "model_cache": {"hits": be.models.hits, "misses": be.models.misses,
                        "resident_bytes": be.models.used},
        "plain_alone": {"requests_per_s": njobs / plain_s, "GPts_s_full_grid": plain_gpts / plain_s / 1e9,
                        "total_s": plain_s,
                        "what": "each request alone, one shot per launch, separate v and p kernels, box off"},
        "served_vs_plain_requests_per_s": capacity / (njobs / plain_s),
        "data": "synthetic", "dtype": "f32"}), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--nt", type=int, default=4000)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--cpu-steps", type=int, default=4000)
    ap.add_argument("--timing-every", type=int, default=32,
                    help="device-stamp the step kernels of every k-th time step (0: off)")
    ap.add_argument("--probe-copy", action="store_true",
                    help="only run a plain device copy of known size (counter calibration)")
    ap.add_argument("--latency", action="store_true",
                    help="per-call latency p50 / p99 of the four fixed workloads (2D forward one "
                         "shot, 2D batched forward, 2D gradient, 3D RTM) instead of the benchmark")
    ap.add_argument("--latency-graph", action="store_true",
                    help="as --latency for the two forward workloads, with the time loop replayed "
                         "as a HIP graph (SMI_OPT_GRAPH)")
    ap.add_argument("--workload", default="",
                    help="with --latency: only the workloads whose name contains this text")
    ap.add_argument("--reps", type=int, default=0,
                    help="with --latency: repetitions per workload (0: the defaults, 20 or 2)")
    ap.add_argument("--serve", type=int, default=0,
                    help="served-stream mode: N jobs of the mixed request stream (2D forward, "
                         "2D gradient, 3D forward) instead of the batched-forward benchmark")
    ap.add_argument("--pool", type=int, default=6,
                    help="with --serve: seeded surveys (models) per job class of the stream")
    ap.add_argument("--no-autotune", action="store_true",
                    help="run the library's default kernels instead of the autotuner's pick")
    ap.add_argument("--reverse-only", action="store_true",
                    help="only the reverse leg (the 2D FWI gradient workload), its object printed "
                         "as the one JSON line: for traces of the reverse loop")
    ap.add_argument("--no-reverse", action="store_true",
                    help="skip the reverse leg (the 2D FWI gradient workload)")
    ap.add_argument("--kernel", type=int, default=-1,
                    help="SMI_OPT_KERNEL for the timed forward (-1: the library's default)")
    ap.add_argument("--chunk", type=int, default=-1, help="SMI_OPT_CHUNK (-1: default)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "the benchmark runs on one GPU; --gpus above 1 is not provided "
                                   "(shots would shard across GPUs with one gradient all-reduce)"}))
        sys.exit(2)

    import torch
    if args.probe_copy:
        probe_copy(torch)
        return
    if args.serve > 0:
        serve(torch, args.serve, pool=args.pool)
        return
    if args.latency or args.latency_graph:
        latency(torch, graph=args.latency_graph, only=args.workload, reps_override=args.reps,
                kernel=args.kernel, chunk=args.chunk, nt=args.nt if args.nt != 4000 else 0)
        return
    if args.reverse_only:
        print(json.dumps(reverse_leg(torch)), flush=True)
        return
    from paper_2311_02293_amd import binding as B
    from paper_2311_02293_amd import inputs as I

    job = I.config2(nt=args.nt)
    job.grid.vpmin = float(job.vp.min())
    job.grid.vpmax = float(job.vp.max())
    dev = "cuda:0"
    vp = torch.from_numpy(job.vp).to(dev)
    rho = torch.from_numpy(job.rho).to(dev)
    stf = torch.from_numpy(job.stf).to(dev)
    ctx = B.Context(0)
    if args.kernel >= 0:
        ctx.set_option(B.OPT_KERNEL, args.kernel)
    if args.chunk >= 0:
        ctx.set_option(B.OPT_CHUNK, args.chunk)
    # the library picks the step kernels by timing them (first call of the shape: the warm-up)
    tuned = args.kernel < 0 and not args.no_autotune
    if tuned:
        ctx.set_option(B.OPT_AUTOTUNE, 1)
    nrec = int(job.acq.rec_off[-1])
    dcal = torch.empty(job.grid.nt * nrec, dtype=torch.float32, device=dev)
    ws = ctx.workspace(ctx.workspace_bytes(job.grid, job.acq, B.JOB_FORWARD))
    stream = torch.cuda.current_stream()

    def step():
        ctx.forward(job.grid, job.acq, vp, rho, stf, dcal=dcal, ws=ws, stream=stream)

    print(f"bench: warmup {args.warmup}", file=sys.stderr, flush=True)
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    ctx.poll_status()
    gpts = ctx.last_counts()[0]
    alg_bytes = ctx.last_bytes()[0]
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(args.steps)]
    ctx.set_option(B.OPT_TIMING, args.timing_every)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        evs[k][0].record(stream)
        step()
        evs[k][1].record(stream)
        print(f"bench: step {k} enqueued", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = [a.elapsed_time(b) for a, b in evs]
    total_ms = sum(ms)
    value = gpts * args.steps / (total_ms / 1e3) / 1e9
    # the dominant kernel: the forward time step (v kernel + p kernel, every shot of the batch
    # in one launch each), timed on the device at every k-th step of the timed region
    kt = {}
    for which, name in ((0, "step_span"), (1, "v_kernel"), (2, "p_kernel")):
        kms, kby, kn = ctx.kernel_timing(which)
        kt[name] = {"avg_us": kms * 1e3, "alg_bytes": kby, "samples": kn,
                    "GBps": kby / (kms / 1e3) / 1e9 if kms > 0 else None}
    ctx.set_option(B.OPT_TIMING, 0)
    pick = ctx.tuning_report() if tuned else ""
    # the timed step configuration by the autotuner's name for it (the library's default on
    # this workload when nothing was tuned)
    config = pick.rsplit("pick ", 1)[-1].strip() if pick else (
        DEFAULT_CONFIG if args.kernel < 0 and args.chunk < 0 else "")
    # duration of the step = the two kernels' own durations (the span from the start of the v
    # kernel to the end of the p kernel also holds the launch gap between them); a fused step
    # is one kernel (reported as the first, the second reports nothing)
    step_us = kt["v_kernel"]["avg_us"] + kt["p_kernel"]["avg_us"]
    step_bytes = kt["step_span"]["alg_bytes"]
    achieved = step_bytes / (step_us / 1e6) / 1e9 if step_us > 0 else None
    whole_job_GBps = alg_bytes / (np.mean(ms) / 1e3) / 1e9

    out = {"metric": METRIC, "value": value, "unit": "GPts/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": total_ms / args.steps, "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
           "config": {"workload": job.name, "nz": job.grid.n1, "nx": job.grid.n2,
                      "nshot": job.acq.nshot, "nt": job.grid.nt, "order": job.grid.order,
                      "nb": job.grid.nb, "box": job.grid.box,
                      "gpts_per_step": gpts, "wall_s": wall},
           "p50_ms": percentile(ms, 50), "p99_ms": percentile(ms, 99),
           # every padded cell of every shot at every step, over the same time: credits the box
           "full_grid_equiv_GPts_s": (job.grid.n1 + 2 * job.grid.nb) * (job.grid.n2 + 2 * job.grid.nb)
                                     * job.acq.nshot * job.grid.nt / (np.mean(ms) / 1e3) / 1e9,
           "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                        "frac": achieved / HBM_PEAK_GBS if achieved else None,
                        "traffic": counter_traffic(config), "config": config,
                        "kernel": ("forward time step over 16 shots, " +
                                   ("fused v + p kernel (k_step2d)" if kt["p_kernel"]["samples"] == 0
                                    else "v kernel + p kernel (k_march_v, k_march_p)")),
                        "alg_bytes_per_launch": step_bytes, "avg_launch_us": step_us,
                        "kernels": kt, "whole_job_alg_GBps": whole_job_GBps,
                        "whole_job_alg_bytes": alg_bytes}}

    if tuned:
        # the library's default kernels on the same workload, timed the same way (the same
        # number of jobs, with the same device timing samples), for comparison with the pick
        ctx.set_option(B.OPT_AUTOTUNE, 0)
        step()
        ctx.set_option(B.OPT_TIMING, args.timing_every)
        torch.cuda.synchronize()
        dms = []
        for _ in range(args.steps):
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record(stream)
            step()
            b.record(stream)
            torch.cuda.synchronize()
            dms.append(a.elapsed_time(b))
        ctx.set_option(B.OPT_TIMING, 0)
        out["autotune"] = {"pick": pick, "default_config": DEFAULT_CONFIG,
                           "default_kernels_ms_per_step": float(np.mean(dms)),
                           "picked_ms_per_step": total_ms / args.steps}
        print(f"bench: autotuner {pick}", file=sys.stderr, flush=True)

    if not args.no_plain:
        # plain stepper: one shot per launch, separate v and p kernels, box off
        print("bench: plain stepper", file=sys.stderr, flush=True)
        ctx.set_option(B.OPT_KERNEL, 1)
        job.grid.box = 0
        ws_p = ctx.workspace(ctx.workspace_bytes(job.grid, job.acq, B.JOB_FORWARD))
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        ctx.forward(job.grid, job.acq, vp, rho, stf, dcal=dcal, ws=ws_p, stream=stream)
        b.record(stream)
        torch.cuda.synchronize()
        pms = a.elapsed_time(b)
        pg = ctx.last_counts()[0]
        ctx.set_option(B.OPT_KERNEL, max(args.kernel, 0))
        job.grid.box = 1
        out["plain"] = {"value": pg / (pms / 1e3) / 1e9, "unit": "GPts/s", "ms_per_step": pms,
                        "gpts_per_step": pg,
                        "what": "one shot per launch, separate v and p kernels, box off",
                        "batched_speedup_wall": pms / (total_ms / args.steps)}

    if not args.no_reverse:
        print("bench: reverse leg", file=sys.stderr, flush=True)
        del ws
        out["reverse"] = reverse_leg(torch)

    if not args.no_cpu:
        print("bench: cpu baseline", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(job, args.cpu_steps)

    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
