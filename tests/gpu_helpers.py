"""Device-side setup shared by the GPU tests (imports torch and the binding)."""
from __future__ import annotations

import numpy as np
import torch

from paper_2310_13325_amd import binding as vb

_CTX = {}


def ctx(graph_mode=False) -> vb.Context:
    key = bool(graph_mode)
    if key not in _CTX:
        _CTX[key] = vb.Context(0, graph_mode=graph_mode)
    return _CTX[key]


def dev(a, dtype=torch.float32):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device="cuda")


def grid_geom(c, case, src_rows=None, rec_rows=None):
    p = case.prob
    grid = vb.Grid(nx=p.nx, nz=p.nz, nt=p.nt, dx=p.dx, dt=p.dt, vmax=case.vmax, nb=p.nb,
                   sponge_alpha=p.alpha)
    w = vb.vip_ricker(c, p.nt, p.dt, p.f0)
    og = case.ogeom
    geom = vb.Geometry(og.src_iz, og.src_ix, og.rec_iz, og.rec_ix, w)
    return grid, geom


def rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))
