"""Shared helpers of the GPU parity tests: move a seeded job to the device, run the oracle
on the same inputs, and compare."""
from __future__ import annotations

import sys

import numpy as np


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def dev(job, device="cuda:0"):
    import torch
    vp = torch.from_numpy(np.ascontiguousarray(job.vp, np.float32)).to(device)
    rho = torch.from_numpy(np.ascontiguousarray(job.rho, np.float32)).to(device)
    stf = torch.from_numpy(np.ascontiguousarray(job.stf, np.float32)).to(device)
    return vp, rho, stf


def rel_l2(a, b) -> float:
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def oracle_dcal(job, shots=None, box=0, vp=None):
    from oracle import oracle as O
    return O.forward_job(job, shots=shots, box=box, vp=vp, vmax=float(job.grid.vpmax))


def with_bounds(job, extra_models=()):
    """State the model speed range on the grid (used by the CPML, the box and the checks)."""
    vs = [np.asarray(job.vp)] + [np.asarray(m) for m in extra_models]
    job.grid.vpmin = float(min(np.min(v) for v in vs))
    job.grid.vpmax = float(max(np.max(v) for v in vs))
    return job
