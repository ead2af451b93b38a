"""Spread the oracle's per-(particle, shot) work over host cores.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py): used to time the FP64
oracle as the CPU baseline and to produce reference gradients at sizes where
one core would be slow.  Each worker is a single-threaded process running
oracle.fwi on one (particle, shot) pair; results are combined in fixed shot
order, so the outcome does not depend on scheduling.
"""
from __future__ import annotations

import multiprocessing as mp
import os

import numpy as np

from oracle import fwi


def _init_worker():
    for k in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS"):
        os.environ[k] = "1"


def _shot_grad(job):
    vel, grid, geom, s, dobs_s, sigma = job
    v_pad, c = fwi.coefficient(vel, grid)
    g = fwi.sponge(grid)
    w = fwi.ricker(grid.nt, grid.dt, geom.f0, geom.t0)
    return fwi.shot_gradient(c, g, v_pad, grid, geom, s, dobs_s, sigma, w)


def _shot_data(job):
    vel, grid, geom, s = job
    _, c = fwi.coefficient(vel, grid)
    g = fwi.sponge(grid)
    w = fwi.ricker(grid.nt, grid.dt, geom.f0, geom.t0)
    rec = (np.asarray(geom.rec_iz) + grid.nb, np.asarray(geom.rec_ix) + grid.nb)
    src = (geom.src_iz[s] + grid.nb, geom.src_ix[s] + grid.nb)
    return fwi.forward_shot(c, g, grid, src, rec, wavelet=w)[0]


def default_workers(cap: int = 16) -> int:
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(n, cap))


def simulate(vel, grid, geom, workers: int):
    jobs = [(np.asarray(vel, dtype=np.float64), grid, geom, s) for s in range(geom.ns)]
    ctx = mp.get_context("fork")
    with ctx.Pool(workers, initializer=_init_worker) as pool:
        out = pool.map(_shot_data, jobs, chunksize=1)
    return np.stack(out)


def grad_logpost(vels, grid, geom, dobs, sigma, workers: int):
    """(logpost, grad) of every particle (no prior term), like
    oracle.fwi.grad_logpost but with pairs spread over processes."""
    vels = np.asarray(vels, dtype=np.float64)
    npart = vels.shape[0]
    jobs = [(vels[p], grid, geom, s, dobs[s], sigma) for p in range(npart) for s in range(geom.ns)]
    ctx = mp.get_context("fork")
    with ctx.Pool(workers, initializer=_init_worker) as pool:
        res = pool.map(_shot_grad, jobs, chunksize=1)
    logpost = np.zeros(npart)
    grad = np.zeros_like(vels)
    for p in range(npart):
        J = 0.0
        gpad = np.zeros((grid.NZ, grid.NX))
        for s in range(geom.ns):
            Js, gs = res[p * geom.ns + s]
            J += Js
            gpad += gs
        logpost[p] = -J
        grad[p] = -fwi.fold_edge(gpad, grid.nb)
    return logpost, grad
