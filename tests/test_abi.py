"""Host-only checks of the C ABI: the header is valid C, the library loads
and exports every declared entry point, and argument validation (which runs
before any device work) returns the documented status codes."""
import ctypes
import os
import re
import subprocess

import numpy as np
import pytest

from paper_2310_13325_amd import binding as vb

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "vip.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(vip_[a-z0-9_]+)\s*\(", text)))


def test_header_is_plain_c():
    r = subprocess.run(["gcc", "-std=c99", "-Wall", "-Werror", "-fsyntax-only", "-x", "c", HEADER],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr


def test_library_exports_every_declared_symbol():
    if not os.path.exists(vb.LIB_PATH):
        pytest.skip("libvip.so not built")
    lib = ctypes.CDLL(vb.LIB_PATH)
    names = declared_functions()
    assert {"vip_forward", "vip_grad_logpost", "vip_svgd_step", "vip_ssvgd_step"} <= set(names)
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing


def _grid(**kw):
    g = dict(nx=64, nz=48, nt=300, dx=10.0, dt=1e-3, vmax=3000.0, nb=20)
    g.update(kw)
    return vb.Grid(**g)


def _geom(nx=64, rec_iz=2, rec_ix=None):
    rec_ix = list(range(nx)) if rec_ix is None else rec_ix
    return vb.Geometry([1, 1], [10, 40], [rec_iz] * len(rec_ix), rec_ix, None)


def _ws(grid, geom, npart=4, k=50, live=0, stored=0):
    lib = vb.lib()
    nbytes = ctypes.c_size_t(0)
    g, ge = grid.c(), geom.c()
    st = lib.vip_grad_logpost_workspace(ctypes.byref(g), ctypes.byref(ge), npart, k, stored,
                                        live, ctypes.byref(nbytes))
    return st, nbytes.value


@pytest.mark.skipif(not os.path.exists(vb.LIB_PATH), reason="libvip.so not built")
def test_workspace_queries_and_validation():
    st, b = _ws(_grid(), _geom())
    assert st == 0 and b > 0
    st2, b2 = _ws(_grid(), _geom(), live=2)
    assert st2 == 0 and b2 < b                       # fewer live pairs, less memory
    # stability limit sqrt(3/8): 3000 m/s * 1 ms / 10 m = 0.3 passes, 6200 fails
    assert _ws(_grid(vmax=6200.0), _geom())[0] == -2
    assert _ws(_grid(), _geom(rec_iz=48))[0] == -1           # receiver row outside
    assert _ws(_grid(), _geom(rec_ix=[3, 3]))[0] == -1       # two receivers, one node
    assert _ws(_grid(nt=1), _geom())[0] == -1
    # minibatch geometry: rows of d_obs must exist
    full = _geom()
    assert _ws(_grid(), full.subset([1]))[0] == 0
    bad = vb.Geometry(full.src_iz[:1], full.src_ix[:1], full.rec_iz, full.rec_ix, None,
                      shot_index=[2], nobs=2)
    assert _ws(_grid(), bad)[0] == -1
    # stored tail segment: valid 0 .. nt-1, one a^n field per stored step and
    # live pair beyond the k-step segment buffer, one checkpoint (2 fields) less
    # per k steps it covers
    g, ge = _grid(), _geom()
    nt, N = g.nt, (g.nx + 2 * g.nb) * (g.nz + 2 * g.nb)
    assert _ws(g, ge, stored=-1)[0] == -1 and _ws(g, ge, stored=nt)[0] == -1
    pairs = 4 * 2
    st0, b0 = _ws(g, ge, k=50)
    st1, b1 = _ws(g, ge, k=50, stored=100)
    assert st0 == 0 and st1 == 0
    nseg0 = -(-(nt - 1) // 50)
    nseg1 = -(-(nt - 1 - 100) // 50) + 1
    assert b1 - b0 == pairs * N * 4 * ((100 - 50) - 2 * (nseg0 - nseg1))
    assert _ws(_grid(), _geom(), k=0)[0] == -1
    assert _ws(_grid(), _geom(), npart=0)[0] == -1
    nb = ctypes.c_size_t(0)
    assert vb.lib().vip_svgd_workspace(128, 24000, ctypes.byref(nb)) == 0 and nb.value > 0
    assert vb.lib().vip_svgd_workspace(0, 10, ctypes.byref(nb)) == -1


@pytest.mark.skipif(not os.path.exists(vb.LIB_PATH), reason="libvip.so not built")
def test_status_strings():
    assert vb.status_string(0) == "VIP_OK"
    assert "CFL" in vb.status_string(-2)
    assert vb.lib().vip_version() >= 10000


@pytest.mark.skipif(not os.path.exists(vb.LIB_PATH), reason="libvip.so not built")
def test_create_without_a_device_fails_cleanly():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a device is visible")
    h = ctypes.c_void_p()
    st = vb.lib().vip_create(ctypes.byref(h), 0, None)
    assert st in (-1, -4) and not h.value
