"""ctypes front end of oracle/cref.c (plain C, FP64) -- TEST INFRASTRUCTURE ONLY.

The C routines implement the same definitions as oracle.fwi / oracle.svgd and
are pinned against them (tests/test_oracle_cref.py).  Calls release the GIL,
so shots and row blocks run in parallel on host threads.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading
from concurrent.futures import ThreadPoolExecutor

import numpy as np

from oracle import fwi

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "cref.c")
LIB = os.path.join(HERE, "libcref.so")

_lib = None
_lock = threading.Lock()
_dp = ctypes.POINTER(ctypes.c_double)
_ip = ctypes.POINTER(ctypes.c_int)


def build() -> str:
    """Compile oracle/libcref.so with gcc (every call recompiles)."""
    tmp = LIB + ".tmp"
    subprocess.run(["gcc", "-O3", "-std=c99", "-fPIC", "-shared", "-o", tmp, SRC, "-lm"],
                   check=True)
    os.replace(tmp, LIB)
    return LIB


def lib():
    global _lib
    with _lock:
        return _load()


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
            build()
        L = ctypes.CDLL(LIB)
        i, d, ll = ctypes.c_int, ctypes.c_double, ctypes.c_longlong
        L.cref_shot_forward.argtypes = [i, i, i, i, d, d, d, d, _dp, i, i, i, _ip, _ip, _dp, _dp]
        L.cref_shot_forward.restype = i
        L.cref_shot_snapshots.argtypes = [i, i, i, i, d, d, d, d, _dp, i, i, i, _ip, _ip, _dp, i,
                                           _ip, _dp, _dp]
        L.cref_shot_snapshots.restype = i
        L.cref_shot_gradient.argtypes = [i, i, i, i, d, d, d, d, _dp, i, i, i, _ip, _ip, _dp, _dp,
                                         d, _dp, _dp]
        L.cref_shot_gradient.restype = i
        L.cref_sqdist_rows.argtypes = [i, ll, _dp, i, i, _dp]
        L.cref_sqdist_rows.restype = None
        _lib = L
    return _lib


def _p(a, t=_dp):
    return a.ctypes.data_as(t)


def _geom_arrays(geom):
    rz = np.ascontiguousarray(geom.rec_iz, dtype=np.int32)
    rx = np.ascontiguousarray(geom.rec_ix, dtype=np.int32)
    return rz, rx


def simulate(vel, grid: fwi.Grid, geom: fwi.Geometry, workers: int = 1):
    """Receiver data [ns][nt][nr] (same as oracle.fwi.simulate)."""
    vel = np.ascontiguousarray(vel, dtype=np.float64)
    w = fwi.ricker(grid.nt, grid.dt, geom.f0, geom.t0)
    rz, rx = _geom_arrays(geom)
    out = np.zeros((geom.ns, grid.nt, geom.nr))

    def one(s):
        st = lib().cref_shot_forward(grid.nz, grid.nx, grid.nb, grid.nt, grid.dx, grid.dz, grid.dt,
                                     grid.alpha, _p(vel), int(geom.src_iz[s]), int(geom.src_ix[s]),
                                     geom.nr, _p(rz, _ip), _p(rx, _ip), _p(w), _p(out[s]))
        assert st == 0

    with ThreadPoolExecutor(max(1, workers)) as ex:
        list(ex.map(one, range(geom.ns)))
    return out


def snapshots(vel, grid: fwi.Grid, geom: fwi.Geometry, shot: int, steps):
    """Wavefields u^n [len(steps)][NZ][NX] of shot `shot` at the ascending
    steps `steps` (the same recurrence as oracle.fwi.forward_shot)."""
    vel = np.ascontiguousarray(vel, dtype=np.float64)
    w = fwi.ricker(grid.nt, grid.dt, geom.f0, geom.t0)
    rz, rx = _geom_arrays(geom)
    steps = np.ascontiguousarray(steps, dtype=np.int32)
    out = np.zeros((len(steps), grid.NZ, grid.NX))
    traces = np.zeros((grid.nt, geom.nr))
    st = lib().cref_shot_snapshots(grid.nz, grid.nx, grid.nb, grid.nt, grid.dx, grid.dz, grid.dt,
                                   grid.alpha, _p(vel), int(geom.src_iz[shot]),
                                   int(geom.src_ix[shot]), geom.nr, _p(rz, _ip), _p(rx, _ip),
                                   _p(w), len(steps), _p(steps, _ip), _p(out), _p(traces))
    assert st == 0, st
    return out


def grad_logpost(vels, grid: fwi.Grid, geom: fwi.Geometry, dobs, sigma, workers: int = 1):
    """(logpost, grad) per particle without prior (as oracle.fwi.grad_logpost);
    (particle, shot) pairs run on `workers` threads, shot sums in fixed order."""
    vels = np.ascontiguousarray(vels, dtype=np.float64)
    dobs = np.ascontiguousarray(dobs, dtype=np.float64)
    npart = vels.shape[0]
    w = fwi.ricker(grid.nt, grid.dt, geom.f0, geom.t0)
    rz, rx = _geom_arrays(geom)
    J = np.zeros((npart, geom.ns))
    gp = np.zeros((npart, geom.ns, grid.NZ, grid.NX))

    def one(job):
        p, s = job
        Jv = ctypes.c_double(0.0)
        st = lib().cref_shot_gradient(grid.nz, grid.nx, grid.nb, grid.nt, grid.dx, grid.dz,
                                      grid.dt, grid.alpha, _p(vels[p]), int(geom.src_iz[s]),
                                      int(geom.src_ix[s]), geom.nr, _p(rz, _ip), _p(rx, _ip),
                                      _p(w), _p(dobs[s]), sigma, ctypes.byref(Jv), _p(gp[p, s]))
        assert st == 0
        J[p, s] = Jv.value

    jobs = [(p, s) for p in range(npart) for s in range(geom.ns)]
    with ThreadPoolExecutor(max(1, workers)) as ex:
        list(ex.map(one, jobs))
    logpost = np.zeros(npart)
    grad = np.zeros_like(vels)
    for p in range(npart):
        Jp = 0.0
        acc = np.zeros((grid.NZ, grid.NX))
        for s in range(geom.ns):
            Jp += J[p, s]
            acc += gp[p, s]
        logpost[p] = -Jp
        grad[p] = -fwi.fold_edge(acc, grid.nb)
    return logpost, grad


def sqdist(X, workers: int = 1, block: int = 16):
    """D_ij = |x_i - x_j|^2 evaluated directly, FP64."""
    X = np.ascontiguousarray(X, dtype=np.float64)
    n, d = X.shape
    D = np.zeros((n, n))

    def rows(i0):
        lib().cref_sqdist_rows(n, d, _p(X), i0, min(n, i0 + block), _p(D))

    with ThreadPoolExecutor(max(1, workers)) as ex:
        list(ex.map(rows, range(0, n, block)))
    return D
