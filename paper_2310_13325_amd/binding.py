"""ctypes binding of libvip (include/vip.h) over torch device tensors.

Argument marshalling only: every step of the computation runs in the HIP
kernels of libvip.so.  torch provides device memory (inputs, outputs and the
workspaces the library asks for) and the stream the library enqueues on.
There is no fallback: a missing library or a call on a machine without a GPU
raises.

The call names follow the C ABI: vip_forward, vip_grad_logpost,
vip_svgd_step, vip_ssvgd_step (plus the tape, plain-path and batching calls).
"""
from __future__ import annotations

import ctypes
import math
import os
from dataclasses import dataclass
from typing import Optional, Sequence

import numpy as np
import torch

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libvip.so")

VIP_OK = 0
VIP_PRIOR_NONE = 0
VIP_PRIOR_UNIFORM_CLIP = 1
VIP_PRIOR_UNIFORM_TRANSFORM = 2
VIP_PRIOR_GAUSSIAN = 3
VIP_BW_MEDIAN_ALL = 0
VIP_BW_MEDIAN_OFFDIAG = 1
VIP_BW_FIXED = 2
VIP_GRAM_BF16 = 0
VIP_GRAM_FP32 = 1
VIP_FLAG_NONFINITE = 0x1
VIP_FLAG_VMAX = 0x2
VIP_FLAG_NOT_PD = 0x4
VIP_FLAG_JITTER = 0x8
VIP_ADVI_FULL_RANK = 0
VIP_ADVI_MEAN_FIELD = 1
VIP_ADVI_MAX_SAMPLES = 32

_i32p = ctypes.POINTER(ctypes.c_int32)


class VipGrid(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("nz", ctypes.c_int32), ("nb", ctypes.c_int32),
                ("nt", ctypes.c_int32), ("dx", ctypes.c_double), ("dz", ctypes.c_double),
                ("dt", ctypes.c_double), ("sponge_alpha", ctypes.c_double),
                ("vmax", ctypes.c_double)]


class VipGeometry(ctypes.Structure):
    _fields_ = [("ns", ctypes.c_int32), ("src_ix", _i32p), ("src_iz", _i32p),
                ("nr", ctypes.c_int32), ("rec_ix", _i32p), ("rec_iz", _i32p),
                ("wavelet", ctypes.c_void_p), ("shot_index", _i32p), ("nobs", ctypes.c_int32)]


class VipPrior(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("lo", ctypes.c_void_p), ("hi", ctypes.c_void_p),
                ("mean", ctypes.c_void_p), ("std", ctypes.c_void_p)]


class VipSvgdLayout(ctypes.Structure):
    _fields_ = [("D", ctypes.c_size_t), ("K", ctypes.c_size_t), ("h2", ctypes.c_size_t),
                ("L", ctypes.c_size_t), ("phi", ctypes.c_size_t)]


TIMING_KINDS = ("forward", "recompute", "adjoint", "forward_store")


class VipTiming(ctypes.Structure):
    _fields_ = [("launches", ctypes.c_int64 * 4), ("ms", ctypes.c_double * 4),
                ("point_steps", ctypes.c_double * 4)]


class VipOptimizer(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("s1", ctypes.c_void_p), ("s2", ctypes.c_void_p),
                ("t", ctypes.c_int64), ("beta1", ctypes.c_double), ("beta2", ctypes.c_double),
                ("delta", ctypes.c_double)]


VIP_OPT_SGD, VIP_OPT_ADAGRAD, VIP_OPT_ADADELTA, VIP_OPT_ADAM = range(4)
VIP_KERNEL_RBF, VIP_KERNEL_DIAG_VAR = 0, 1


class VipSvgdConfig(ctypes.Structure):
    _fields_ = [("bw_mode", ctypes.c_int32), ("h_fixed", ctypes.c_double),
                ("gram_prec", ctypes.c_int32), ("kernel", ctypes.c_int32),
                ("noise", ctypes.c_int32), ("xi", ctypes.c_void_p), ("seed", ctypes.c_uint64),
                ("stream", ctypes.c_uint64), ("opt", ctypes.POINTER(VipOptimizer))]


class VipError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        super().__init__(f"{where}: {status_string(status)} ({status})")


_lib = None


def lib() -> ctypes.CDLL:
    """Load libvip.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python -m paper_2310_13325_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        vp, sz, i32, i64, u64, dbl = (ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int32,
                                      ctypes.c_int64, ctypes.c_uint64, ctypes.c_double)
        G, GE, PR = ctypes.POINTER(VipGrid), ctypes.POINTER(VipGeometry), ctypes.POINTER(VipPrior)
        szp = ctypes.POINTER(sz)
        sig = {
            "vip_status_string": (ctypes.c_char_p, [ctypes.c_int]),
            "vip_version": (ctypes.c_int, []),
            "vip_create": (ctypes.c_int, [ctypes.POINTER(vp), ctypes.c_int, vp]),
            "vip_destroy": (ctypes.c_int, [vp]),
            "vip_set_stream": (ctypes.c_int, [vp, vp]),
            "vip_set_graph_mode": (ctypes.c_int, [vp, ctypes.c_int]),
            "vip_poll": (ctypes.c_int, [vp, vp, ctypes.POINTER(ctypes.c_uint32)]),
            "vip_ricker": (ctypes.c_int, [vp, i32, dbl, dbl, dbl, vp]),
            "vip_forward_workspace": (ctypes.c_int, [G, GE, i32, szp]),
            "vip_forward": (ctypes.c_int, [vp, G, GE, i32, vp, vp, vp, sz]),
            "vip_grad_logpost_workspace": (ctypes.c_int, [G, GE, i32, i32, i32, i32, szp]),
            "vip_grad_logpost": (ctypes.c_int, [vp, G, GE, PR, i32, vp, vp, dbl, i32, i32, i32, vp,
                                                vp, vp, sz]),
            "vip_grad_logpost_plain_workspace": (ctypes.c_int, [G, GE, i32, szp]),
            "vip_grad_logpost_plain": (ctypes.c_int, [vp, G, GE, PR, i32, vp, vp, dbl, vp, vp, vp,
                                                      sz]),
            "vip_tape_bytes": (ctypes.c_int, [G, GE, i32, i32, szp]),
            "vip_tape_workspace": (ctypes.c_int, [G, GE, i32, i32, szp]),
            "vip_forward_tape": (ctypes.c_int, [vp, G, GE, i32, vp, vp, i32, vp, sz, vp, sz]),
            "vip_adjoint_tape": (ctypes.c_int, [vp, G, GE, i32, vp, i32, vp, sz, vp, vp, vp, sz]),
            "vip_svgd_workspace": (ctypes.c_int, [i32, i64, szp]),
            "vip_svgd_layout_of": (ctypes.c_int, [i32, i64, ctypes.POINTER(VipSvgdLayout)]),
            "vip_svgd_step": (ctypes.c_int, [vp, i32, i64, vp, vp, dbl, i32, dbl, i32, PR, vp, vp,
                                             sz]),
            "vip_ssvgd_step": (ctypes.c_int, [vp, i32, i64, vp, vp, dbl, i32, dbl, i32, PR, vp,
                                              u64, u64, vp, vp, sz]),
            "vip_svgd_step_noalloc": (ctypes.c_int, [vp, i32, i64, vp, vp, dbl, i32, dbl, i32, PR,
                                                     vp, vp]),
            "vip_philox_normals": (ctypes.c_int, [vp, i64, u64, u64, vp]),
            "vip_philox_uint32": (ctypes.c_int, [vp, i64, u64, u64, vp]),
            "vip_set_timing": (ctypes.c_int, [vp, ctypes.c_int]),
            "vip_set_tile": (ctypes.c_int, [vp, ctypes.c_int]),
            "vip_tile_count": (ctypes.c_int, []),
            "vip_prior_transform": (ctypes.c_int, [vp, PR, i32, i64, vp, vp, i32]),
            "vip_svgd_step_opt": (ctypes.c_int, [vp, i32, i64, vp, vp, dbl, i32, dbl, i32, PR,
                                                 ctypes.POINTER(VipOptimizer), vp, vp, sz]),
            "vip_svgd_step_ex": (ctypes.c_int, [vp, i32, i64, vp, vp, dbl,
                                                ctypes.POINTER(VipSvgdConfig), PR, vp, vp, sz]),
            "vip_tile_shape": (ctypes.c_int, [ctypes.c_int, ctypes.POINTER(ctypes.c_int32)]),
            "vip_tile_persistent": (ctypes.c_int, [ctypes.c_int]),
            "vip_tile_for_grid": (ctypes.c_int, [vp, G, ctypes.c_int64, ctypes.POINTER(ctypes.c_int32)]),
            "vip_read_timing": (ctypes.c_int, [vp, ctypes.POINTER(VipTiming)]),
            "vip_advi_sample": (ctypes.c_int, [vp, i32, i64, i32, vp, vp, i64, vp, vp]),
            "vip_advi_step": (ctypes.c_int, [vp, i32, i64, i32, vp, vp, i64, vp, vp, dbl,
                                             ctypes.POINTER(VipOptimizer),
                                             ctypes.POINTER(VipOptimizer), vp, vp, vp, vp]),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name, None)
            if f is None:
                continue
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def status_string(s: int) -> str:
    try:
        return lib().vip_status_string(int(s)).decode()
    except Exception:
        return "unknown"


def _check(status: int, where: str):
    if status != VIP_OK:
        raise VipError(status, where)


def tile_shape(tile: int) -> dict:
    """Extended width/height, rows per thread and steps per launch of a blocked tile."""
    a = (ctypes.c_int32 * 4)()
    _check(lib().vip_tile_shape(int(tile), a), "vip_tile_shape")
    persistent = lib().vip_tile_persistent(int(tile))
    _check(min(persistent, 0), "vip_tile_persistent")
    return {"ex": a[0], "ez": a[1], "rz": a[2], "tmax": a[3], "persistent": bool(persistent)}


# ----------------------------------------------------------------------------
# Plain-python descriptions of a problem, converted to the C structs per call
# ----------------------------------------------------------------------------

@dataclass
class Grid:
    nx: int
    nz: int
    nt: int
    dx: float
    dt: float
    vmax: float
    nb: int = 20
    dz: Optional[float] = None
    sponge_alpha: float = 0.015

    def c(self) -> VipGrid:
        return VipGrid(self.nx, self.nz, self.nb, self.nt, self.dx,
                       self.dx if self.dz is None else self.dz, self.dt, self.sponge_alpha,
                       self.vmax)


class Geometry:
    """Shot / receiver interior indices (host) and the device wavelet."""

    def __init__(self, src_iz: Sequence[int], src_ix: Sequence[int], rec_iz: Sequence[int],
                 rec_ix: Sequence[int], wavelet: torch.Tensor,
                 shot_index: Optional[Sequence[int]] = None, nobs: int = 0):
        self.src_iz = np.ascontiguousarray(src_iz, dtype=np.int32)
        self.src_ix = np.ascontiguousarray(src_ix, dtype=np.int32)
        self.rec_iz = np.ascontiguousarray(rec_iz, dtype=np.int32)
        self.rec_ix = np.ascontiguousarray(rec_ix, dtype=np.int32)
        assert len(self.src_iz) == len(self.src_ix) and len(self.rec_iz) == len(self.rec_ix)
        self.wavelet = wavelet
        self.shot_index = (None if shot_index is None
                           else np.ascontiguousarray(shot_index, dtype=np.int32))
        self.nobs = int(nobs)

    def subset(self, shots: Sequence[int]) -> "Geometry":
        """The shots `shots` of this survey, reading their observed data in place
        (rows `shots` of the full d_obs)."""
        shots = np.asarray(shots, dtype=np.int64)
        rows = shots if self.shot_index is None else self.shot_index[shots]
        return Geometry(self.src_iz[shots], self.src_ix[shots], self.rec_iz, self.rec_ix,
                        self.wavelet, shot_index=rows,
                        nobs=self.nobs if self.shot_index is not None else self.ns)

    @property
    def ns(self):
        return len(self.src_iz)

    @property
    def nr(self):
        return len(self.rec_iz)

    def c(self) -> VipGeometry:
        p = lambda a: a.ctypes.data_as(_i32p)
        w = self.wavelet.data_ptr() if self.wavelet is not None else None
        si = p(self.shot_index) if self.shot_index is not None else None
        return VipGeometry(self.ns, p(self.src_ix), p(self.src_iz), self.nr, p(self.rec_ix),
                           p(self.rec_iz), w, si, self.nobs)


@dataclass
class Prior:
    """A prior of section 3 (device float [d] arrays): uniform on [lo, hi] by
    clipping (strategy 1) or in the transformed space of eq:transform
    (strategy 2), or independent Gaussians N(mean, std^2)."""
    kind: int
    lo: Optional[torch.Tensor] = None
    hi: Optional[torch.Tensor] = None
    mean: Optional[torch.Tensor] = None
    std: Optional[torch.Tensor] = None

    @staticmethod
    def clip(lo, hi):
        return Prior(VIP_PRIOR_UNIFORM_CLIP, lo=lo, hi=hi)

    @staticmethod
    def transform(lo, hi):
        return Prior(VIP_PRIOR_UNIFORM_TRANSFORM, lo=lo, hi=hi)

    @staticmethod
    def gaussian(mean, std):
        return Prior(VIP_PRIOR_GAUSSIAN, mean=mean, std=std)

    def c(self) -> VipPrior:
        f = lambda t: _ptr(t.reshape(-1), torch.float32) if t is not None else None
        return VipPrior(self.kind, f(self.lo), f(self.hi), f(self.mean), f(self.std))


def _prior(lo: Optional[torch.Tensor], hi: Optional[torch.Tensor], prior: Optional[Prior] = None):
    if prior is not None:
        return prior.c()
    if lo is None:
        return None
    return VipPrior(VIP_PRIOR_UNIFORM_CLIP, _ptr(lo, torch.float32), _ptr(hi, torch.float32))


def vip_prior_transform(ctx: "Context", prior: Prior, x: torch.Tensor, to_theta: bool,
                        out: Optional[torch.Tensor] = None) -> torch.Tensor:
    """eq:transform over particles x [n][...]: m -> theta (to_theta) or theta -> m."""
    ctx.sync_stream()
    n = x.shape[0]
    d = x.numel() // n
    out = torch.empty_like(x) if out is None else out
    pr = prior.c()
    _check(lib().vip_prior_transform(ctx.handle, ctypes.byref(pr), n, d, _ptr(x, torch.float32),
                                     _ptr(out, torch.float32), 1 if to_theta else 0),
           "vip_prior_transform")
    return out


def _ptr(t: Optional[torch.Tensor], dtype=None):
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("expected a device tensor")
    if not t.is_contiguous():
        raise ValueError("expected a contiguous tensor")
    if dtype is not None and t.dtype != dtype:
        raise ValueError(f"expected {dtype}, got {t.dtype}")
    return t.data_ptr()


class Context:
    """A libvip context on one device; enqueues on torch's current stream."""

    def __init__(self, device: int = 0, graph_mode: bool = False):
        if not torch.cuda.is_available():
            raise RuntimeError("libvip needs a HIP device; none is visible")
        self.device = torch.device("cuda", device)
        self._h = ctypes.c_void_p()
        _check(lib().vip_create(ctypes.byref(self._h), device,
                                ctypes.c_void_p(torch.cuda.current_stream(self.device).cuda_stream)),
               "vip_create")
        if graph_mode:
            _check(lib().vip_set_graph_mode(self._h, 1), "vip_set_graph_mode")
        self._ws = {}

    def close(self):
        if self._h:
            lib().vip_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def handle(self):
        return self._h

    def sync_stream(self):
        _check(lib().vip_set_stream(
            self._h, ctypes.c_void_p(torch.cuda.current_stream(self.device).cuda_stream)),
            "vip_set_stream")

    def set_graph_mode(self, on: bool):
        _check(lib().vip_set_graph_mode(self._h, 1 if on else 0), "vip_set_graph_mode")

    def workspace(self, tag: str, nbytes: int) -> torch.Tensor:
        """Zero-initialised device workspace reused across calls with the same tag."""
        ws = self._ws.get(tag)
        if ws is None or ws.numel() < nbytes:
            ws = None                       # release the smaller buffer before allocating
            self._ws.pop(tag, None)
            ws = torch.zeros(max(int(nbytes), 256), dtype=torch.uint8, device=self.device)
            self._ws[tag] = ws
        return ws

    def workspace_bytes(self) -> int:
        """Device bytes held by this context's cached workspaces."""
        return sum(int(w.numel()) for w in self._ws.values())

    def set_tile(self, tile: int):
        """-2 automatic, -1 one step per launch, 0.. a temporally blocked shape."""
        _check(lib().vip_set_tile(self._h, int(tile)), "vip_set_tile")

    def tile_for(self, grid: "Grid", pairs: int = 0) -> int:
        """Tile index a single-problem call on `grid` over `pairs` (particle, shot)
        pairs per launch uses (-1: one step per launch; pairs 0: many)."""
        t = ctypes.c_int32(0)
        g = grid.c()
        _check(lib().vip_tile_for_grid(self._h, ctypes.byref(g), int(pairs), ctypes.byref(t)),
               "vip_tile_for_grid")
        return int(t.value)

    def set_timing(self, on: bool):
        _check(lib().vip_set_timing(self._h, 1 if on else 0), "vip_set_timing")

    def read_timing(self) -> dict:
        """Per step-kernel kind (forward, recompute, adjoint): launches, ms, point-steps."""
        t = VipTiming()
        _check(lib().vip_read_timing(self._h, ctypes.byref(t)), "vip_read_timing")
        kinds = TIMING_KINDS
        return {k: {"launches": int(t.launches[i]), "ms": float(t.ms[i]),
                    "point_steps": float(t.point_steps[i])} for i, k in enumerate(kinds)}

    def poll(self, ws: torch.Tensor) -> int:
        flags = ctypes.c_uint32(0)
        _check(lib().vip_poll(self._h, ctypes.c_void_p(ws.data_ptr()), ctypes.byref(flags)),
               "vip_poll")
        return int(flags.value)


# ----------------------------------------------------------------------------
# Calls
# ----------------------------------------------------------------------------

def vip_ricker(ctx: Context, nt: int, dt: float, f0: float, t0: float = 0.0) -> torch.Tensor:
    ctx.sync_stream()
    out = torch.empty(nt, dtype=torch.float32, device=ctx.device)
    _check(lib().vip_ricker(ctx.handle, nt, dt, f0, t0, ctypes.c_void_p(out.data_ptr())),
           "vip_ricker")
    return out


def vip_forward(ctx: Context, grid: Grid, geom: Geometry, vel: torch.Tensor,
                data: Optional[torch.Tensor] = None) -> torch.Tensor:
    ctx.sync_stream()
    npart = vel.shape[0]
    g, ge = grid.c(), geom.c()
    nbytes = ctypes.c_size_t()
    _check(lib().vip_forward_workspace(ctypes.byref(g), ctypes.byref(ge), npart,
                                       ctypes.byref(nbytes)), "vip_forward_workspace")
    ws = ctx.workspace("forward", nbytes.value)
    if data is None:
        data = torch.empty((npart, geom.ns, grid.nt, geom.nr), dtype=torch.float32,
                           device=ctx.device)
    _check(lib().vip_forward(ctx.handle, ctypes.byref(g), ctypes.byref(ge), npart,
                             _ptr(vel, torch.float32), _ptr(data, torch.float32),
                             ctypes.c_void_p(ws.data_ptr()), ws.numel()), "vip_forward")
    return data


def grad_logpost_workspace_bytes(grid: Grid, geom: Geometry, npart: int, ckpt_every: int,
                                 live_pairs: int = 0, stored_steps: int = 0) -> int:
    g, ge = grid.c(), geom.c()
    nbytes = ctypes.c_size_t()
    _check(lib().vip_grad_logpost_workspace(ctypes.byref(g), ctypes.byref(ge), npart,
                                            ckpt_every, stored_steps, live_pairs,
                                            ctypes.byref(nbytes)),
           "vip_grad_logpost_workspace")
    return nbytes.value


def stored_steps_for_budget(grid: Grid, geom: Geometry, npart: int, ckpt_every: int,
                            budget_bytes: int, live_pairs: int = 0) -> int:
    """Largest stored_steps S >= ckpt_every whose vip_grad_logpost workspace fits
    budget_bytes, or 0.  For S >= k the workspace grows with S (one a^n slot per
    stored step against two checkpoint fields per k steps), so bisection applies."""
    k, m = min(ckpt_every, grid.nt - 1), grid.nt - 1
    size = lambda s: grad_logpost_workspace_bytes(grid, geom, npart, ckpt_every, live_pairs, s)
    if size(k) > budget_bytes:
        return 0
    lo, hi = k, m
    if size(hi) <= budget_bytes:
        return hi
    while hi - lo > 1:
        mid = (lo + hi) // 2
        if size(mid) <= budget_bytes:
            lo = mid
        else:
            hi = mid
    return lo


def vip_grad_logpost(ctx: Context, grid: Grid, geom: Geometry, vel: torch.Tensor,
                     dobs: torch.Tensor, sigma: float, ckpt_every: int = 50,
                     lo: Optional[torch.Tensor] = None, hi: Optional[torch.Tensor] = None,
                     live_pairs: int = 0, logpost: Optional[torch.Tensor] = None,
                     grad: Optional[torch.Tensor] = None, ws_tag: str = "grad",
                     stored_steps: int = 0, prior: Optional[Prior] = None):
    ctx.sync_stream()
    npart = vel.shape[0]
    nbytes = grad_logpost_workspace_bytes(grid, geom, npart, ckpt_every, live_pairs,
                                          stored_steps)
    ws = ctx.workspace(ws_tag, nbytes)
    if logpost is None:
        logpost = torch.empty(npart, dtype=torch.float64, device=ctx.device)
    if grad is None:
        grad = torch.empty_like(vel)
    g, ge = grid.c(), geom.c()
    pr = _prior(lo, hi, prior)
    _check(lib().vip_grad_logpost(ctx.handle, ctypes.byref(g), ctypes.byref(ge),
                                  ctypes.byref(pr) if pr is not None else None, npart,
                                  _ptr(vel, torch.float32), _ptr(dobs, torch.float32), sigma,
                                  ckpt_every, stored_steps, live_pairs,
                                  _ptr(logpost, torch.float64),
                                  _ptr(grad, torch.float32), ctypes.c_void_p(ws.data_ptr()),
                                  ws.numel()), "vip_grad_logpost")
    return logpost, grad


def vip_grad_logpost_minibatch(ctx: Context, grid: Grid, geom: Geometry, vel: torch.Tensor,
                               dobs: torch.Tensor, sigma: float, shots: Sequence[int], **kw):
    """Unbiased minibatch estimate (section 2.4) from the shots `shots` of the
    survey `geom` (observed data dobs [ns][nt][nr], read in place); the
    library scales the subset's misfit by ns / len(shots) itself."""
    return vip_grad_logpost(ctx, grid, geom.subset(shots), vel, dobs, sigma, **kw)


def vip_grad_logpost_plain(ctx: Context, grid: Grid, geom: Geometry, vel: torch.Tensor,
                           dobs: torch.Tensor, sigma: float, lo=None, hi=None,
                           prior: Optional[Prior] = None):
    ctx.sync_stream()
    npart = vel.shape[0]
    g, ge = grid.c(), geom.c()
    nbytes = ctypes.c_size_t()
    _check(lib().vip_grad_logpost_plain_workspace(ctypes.byref(g), ctypes.byref(ge), npart,
                                                  ctypes.byref(nbytes)),
           "vip_grad_logpost_plain_workspace")
    ws = ctx.workspace("plain", nbytes.value)
    logpost = torch.empty(npart, dtype=torch.float64, device=ctx.device)
    grad = torch.empty_like(vel)
    pr = _prior(lo, hi, prior)
    _check(lib().vip_grad_logpost_plain(ctx.handle, ctypes.byref(g), ctypes.byref(ge),
                                        ctypes.byref(pr) if pr is not None else None, npart,
                                        _ptr(vel, torch.float32), _ptr(dobs, torch.float32),
                                        sigma, _ptr(logpost, torch.float64),
                                        _ptr(grad, torch.float32),
                                        ctypes.c_void_p(ws.data_ptr()), ws.numel()),
           "vip_grad_logpost_plain")
    return logpost, grad


def tape_sizes(grid: Grid, geom: Geometry, npart: int, ckpt_every: int):
    g, ge = grid.c(), geom.c()
    tb, wb = ctypes.c_size_t(), ctypes.c_size_t()
    _check(lib().vip_tape_bytes(ctypes.byref(g), ctypes.byref(ge), npart, ckpt_every,
                                ctypes.byref(tb)), "vip_tape_bytes")
    _check(lib().vip_tape_workspace(ctypes.byref(g), ctypes.byref(ge), npart, ckpt_every,
                                    ctypes.byref(wb)), "vip_tape_workspace")
    return tb.value, wb.value


def vip_forward_tape(ctx: Context, grid: Grid, geom: Geometry, vel: torch.Tensor,
                     ckpt_every: int, tape: torch.Tensor, ws: torch.Tensor) -> torch.Tensor:
    ctx.sync_stream()
    npart = vel.shape[0]
    data = torch.empty((npart, geom.ns, grid.nt, geom.nr), dtype=torch.float32, device=ctx.device)
    g, ge = grid.c(), geom.c()
    _check(lib().vip_forward_tape(ctx.handle, ctypes.byref(g), ctypes.byref(ge), npart,
                                  _ptr(vel, torch.float32), _ptr(data, torch.float32), ckpt_every,
                                  ctypes.c_void_p(tape.data_ptr()), tape.numel(),
                                  ctypes.c_void_p(ws.data_ptr()), ws.numel()), "vip_forward_tape")
    return data


def vip_adjoint_tape(ctx: Context, grid: Grid, geom: Geometry, vel: torch.Tensor, ckpt_every: int,
                     tape: torch.Tensor, grad_data: torch.Tensor, ws: torch.Tensor) -> torch.Tensor:
    ctx.sync_stream()
    npart = vel.shape[0]
    grad_vel = torch.empty_like(vel)
    g, ge = grid.c(), geom.c()
    _check(lib().vip_adjoint_tape(ctx.handle, ctypes.byref(g), ctypes.byref(ge), npart,
                                  _ptr(vel, torch.float32), ckpt_every,
                                  ctypes.c_void_p(tape.data_ptr()), tape.numel(),
                                  _ptr(grad_data, torch.float32), _ptr(grad_vel, torch.float32),
                                  ctypes.c_void_p(ws.data_ptr()), ws.numel()), "vip_adjoint_tape")
    return grad_vel


def svgd_workspace_bytes(n: int, d: int) -> int:
    nbytes = ctypes.c_size_t()
    _check(lib().vip_svgd_workspace(n, d, ctypes.byref(nbytes)), "vip_svgd_workspace")
    return nbytes.value


def svgd_layout(n: int, d: int) -> VipSvgdLayout:
    lay = VipSvgdLayout()
    _check(lib().vip_svgd_layout_of(n, d, ctypes.byref(lay)), "vip_svgd_layout_of")
    return lay


def vip_svgd_step(ctx: Context, x: torch.Tensor, g: torch.Tensor, eps: float,
                  bw_mode: int = VIP_BW_MEDIAN_ALL, h_fixed: float = 1.0,
                  gram_prec: int = VIP_GRAM_BF16, lo=None, hi=None,
                  h2_out: Optional[torch.Tensor] = None, ws_tag: str = "svgd",
                  prior: Optional[Prior] = None) -> torch.Tensor:
    """In-place SVGD update of x ([n][d] float32); returns the workspace."""
    ctx.sync_stream()
    n = x.shape[0]
    d = x.numel() // n
    ws = ctx.workspace(ws_tag, svgd_workspace_bytes(n, d))
    pr = _prior(lo, hi, prior)
    _check(lib().vip_svgd_step(ctx.handle, n, d, _ptr(x, torch.float32), _ptr(g, torch.float32),
                               eps, bw_mode, h_fixed, gram_prec,
                               ctypes.byref(pr) if pr is not None else None,
                               _ptr(h2_out, torch.float64), ctypes.c_void_p(ws.data_ptr()),
                               ws.numel()), "vip_svgd_step")
    return ws


VIP_NOALLOC_SCRATCH_BYTES = 64 * 1024 * 1024


def vip_svgd_step_noalloc(ctx: Context, x: torch.Tensor, g: torch.Tensor, eps: float,
                          bw_mode: int = VIP_BW_MEDIAN_ALL, h_fixed: float = 1.0,
                          gram_prec: int = VIP_GRAM_BF16, lo=None, hi=None,
                          h2_out: Optional[torch.Tensor] = None,
                          status: Optional[torch.Tensor] = None,
                          prior: Optional[Prior] = None) -> None:
    """In-place SVGD update of x ([n][d] float32) without a workspace: the
    library's fixed per-device array serves instead (status: device int32 [1]
    the step ORs its flags into, or None)."""
    ctx.sync_stream()
    n = x.shape[0]
    d = x.numel() // n
    pr = _prior(lo, hi, prior)
    _check(lib().vip_svgd_step_noalloc(ctx.handle, n, d, _ptr(x, torch.float32),
                                       _ptr(g, torch.float32), eps, bw_mode, h_fixed, gram_prec,
                                       ctypes.byref(pr) if pr is not None else None,
                                       _ptr(h2_out, torch.float64), _ptr(status, torch.int32)),
           "vip_svgd_step_noalloc")


class Optimizer:
    """State of a step rule for vip_svgd_step_opt (zero-initialised, carried
    from step to step)."""

    def __init__(self, kind: int, like: torch.Tensor, beta1: float = 0.9, beta2: float = 0.999,
                 delta: float = 1e-8):
        self.kind, self.beta1, self.beta2, self.delta = kind, beta1, beta2, delta
        self.t = 0
        self.s1 = torch.zeros_like(like) if kind != VIP_OPT_SGD else None
        self.s2 = torch.zeros_like(like) if kind in (VIP_OPT_ADADELTA, VIP_OPT_ADAM) else None

    def c(self) -> VipOptimizer:
        return VipOptimizer(self.kind, _ptr(self.s1, torch.float32), _ptr(self.s2, torch.float32),
                            self.t, self.beta1, self.beta2, self.delta)


def vip_svgd_step_opt(ctx: Context, x: torch.Tensor, g: torch.Tensor, eps: float, opt: Optimizer,
                      bw_mode: int = VIP_BW_MEDIAN_ALL, h_fixed: float = 1.0,
                      gram_prec: int = VIP_GRAM_BF16, lo=None, hi=None,
                      prior: Optional[Prior] = None, h2_out: Optional[torch.Tensor] = None,
                      ws_tag: str = "svgd") -> torch.Tensor:
    """In-place SVGD update of x with the step rule `opt` (its step count advances)."""
    ctx.sync_stream()
    n = x.shape[0]
    d = x.numel() // n
    ws = ctx.workspace(ws_tag, svgd_workspace_bytes(n, d))
    pr = _prior(lo, hi, prior)
    opt.t += 1
    oc = opt.c()
    _check(lib().vip_svgd_step_opt(ctx.handle, n, d, _ptr(x, torch.float32),
                                   _ptr(g, torch.float32), eps, bw_mode, h_fixed, gram_prec,
                                   ctypes.byref(pr) if pr is not None else None, ctypes.byref(oc),
                                   _ptr(h2_out, torch.float64), ctypes.c_void_p(ws.data_ptr()),
                                   ws.numel()), "vip_svgd_step_opt")
    return ws


def vip_svgd_step_ex(ctx: Context, x: torch.Tensor, g: torch.Tensor, eps: float,
                     kernel: int = VIP_KERNEL_RBF, noise: bool = False,
                     xi: Optional[torch.Tensor] = None, seed: int = 0, stream: int = 0,
                     opt: Optional[Optimizer] = None, bw_mode: int = VIP_BW_MEDIAN_ALL,
                     h_fixed: float = 1.0, gram_prec: int = VIP_GRAM_BF16, lo=None, hi=None,
                     prior: Optional[Prior] = None, h2_out: Optional[torch.Tensor] = None,
                     ws_tag: str = "svgd") -> torch.Tensor:
    """In-place SVGD / sSVGD update with every option (kernel, noise, step rule)."""
    ctx.sync_stream()
    n = x.shape[0]
    d = x.numel() // n
    ws = ctx.workspace(ws_tag, svgd_workspace_bytes(n, d))
    pr = _prior(lo, hi, prior)
    oc = None
    if opt is not None:
        opt.t += 1
        oc = opt.c()
    cfg = VipSvgdConfig(bw_mode, h_fixed, gram_prec, kernel, 1 if noise else 0,
                        _ptr(xi, torch.float32), seed, stream,
                        ctypes.pointer(oc) if oc is not None else None)
    _check(lib().vip_svgd_step_ex(ctx.handle, n, d, _ptr(x, torch.float32), _ptr(g, torch.float32),
                                  eps, ctypes.byref(cfg),
                                  ctypes.byref(pr) if pr is not None else None,
                                  _ptr(h2_out, torch.float64), ctypes.c_void_p(ws.data_ptr()),
                                  ws.numel()), "vip_svgd_step_ex")
    return ws


def vip_ssvgd_step(ctx: Context, x: torch.Tensor, g: torch.Tensor, eps: float,
                   xi: Optional[torch.Tensor] = None, seed: int = 0, stream: int = 0,
                   bw_mode: int = VIP_BW_MEDIAN_ALL, h_fixed: float = 1.0,
                   gram_prec: int = VIP_GRAM_BF16, lo=None, hi=None,
                   h2_out: Optional[torch.Tensor] = None, ws_tag: str = "svgd",
                   prior: Optional[Prior] = None) -> torch.Tensor:
    """In-place sSVGD update of x; returns the workspace."""
    ctx.sync_stream()
    n = x.shape[0]
    d = x.numel() // n
    ws = ctx.workspace(ws_tag, svgd_workspace_bytes(n, d))
    pr = _prior(lo, hi, prior)
    _check(lib().vip_ssvgd_step(ctx.handle, n, d, _ptr(x, torch.float32), _ptr(g, torch.float32),
                                eps, bw_mode, h_fixed, gram_prec,
                                ctypes.byref(pr) if pr is not None else None,
                                _ptr(xi, torch.float32), seed, stream,
                                _ptr(h2_out, torch.float64), ctypes.c_void_p(ws.data_ptr()),
                                ws.numel()), "vip_ssvgd_step")
    return ws


def vip_philox_normals(ctx: Context, count: int, seed: int, stream: int) -> torch.Tensor:
    ctx.sync_stream()
    out = torch.empty(count, dtype=torch.float32, device=ctx.device)
    _check(lib().vip_philox_normals(ctx.handle, count, seed, stream,
                                    ctypes.c_void_p(out.data_ptr())), "vip_philox_normals")
    return out


def vip_philox_uint32(ctx: Context, nblocks: int, seed: int, stream: int) -> torch.Tensor:
    ctx.sync_stream()
    out = torch.empty(4 * nblocks, dtype=torch.int32, device=ctx.device)
    _check(lib().vip_philox_uint32(ctx.handle, nblocks, seed, stream,
                                   ctypes.c_void_p(out.data_ptr())), "vip_philox_uint32")
    return out


def workspace_view(ws: torch.Tensor, offset: int, count: int, dtype) -> torch.Tensor:
    """A typed view into a workspace at a byte offset (for inspecting results)."""
    itemsize = torch.tensor([], dtype=dtype).element_size()
    return ws[offset: offset + count * itemsize].view(dtype)


# ----------------------------------------------------------------------------
# Batches of problems / ensembles
# ----------------------------------------------------------------------------

class VipProblem(ctypes.Structure):
    _fields_ = [("grid", VipGrid), ("geom", VipGeometry), ("prior", VipPrior), ("np", ctypes.c_int32),
                ("vel", ctypes.c_void_p), ("dobs", ctypes.c_void_p), ("sigma", ctypes.c_double),
                ("logpost", ctypes.c_void_p), ("grad", ctypes.c_void_p)]


class VipEnsemble(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("d", ctypes.c_int64), ("x", ctypes.c_void_p),
                ("g", ctypes.c_void_p), ("eps", ctypes.c_double), ("prior", VipPrior),
                ("xi", ctypes.c_void_p), ("h2_out", ctypes.c_void_p)]


@dataclass
class Problem:
    """One inversion of a batch; logpost and grad are allocated when None."""
    grid: Grid
    geom: Geometry
    vel: torch.Tensor
    dobs: torch.Tensor
    sigma: float
    lo: Optional[torch.Tensor] = None
    hi: Optional[torch.Tensor] = None
    logpost: Optional[torch.Tensor] = None
    grad: Optional[torch.Tensor] = None
    prior: Optional[Prior] = None

    def c(self) -> VipProblem:
        if self.logpost is None:
            self.logpost = torch.empty(self.vel.shape[0], dtype=torch.float64, device=self.vel.device)
        if self.grad is None:
            self.grad = torch.empty_like(self.vel)
        pr = _prior(self.lo, self.hi, self.prior) or VipPrior(VIP_PRIOR_NONE)
        return VipProblem(self.grid.c(), self.geom.c(), pr, self.vel.shape[0],
                          _ptr(self.vel, torch.float32), _ptr(self.dobs, torch.float32), self.sigma,
                          _ptr(self.logpost, torch.float64), _ptr(self.grad, torch.float32))


def _multi_lib():
    L = lib()
    vp, sz, i32, i64, u64, dbl = (ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int32,
                                  ctypes.c_int64, ctypes.c_uint64, ctypes.c_double)
    PP, EP = ctypes.POINTER(VipProblem), ctypes.POINTER(VipEnsemble)
    L.vip_grad_logpost_multi_workspace.argtypes = [i32, PP, i32, ctypes.POINTER(sz)]
    L.vip_grad_logpost_multi.argtypes = [vp, i32, PP, i32, vp, sz]
    L.vip_svgd_multi_workspace.argtypes = [i32, EP, ctypes.POINTER(sz)]
    L.vip_svgd_step_multi.argtypes = [vp, i32, EP, i32, dbl, i32, vp, sz]
    L.vip_ssvgd_step_multi.argtypes = [vp, i32, EP, i32, dbl, i32, u64, u64, vp, sz]
    for f in (L.vip_grad_logpost_multi_workspace, L.vip_grad_logpost_multi,
              L.vip_svgd_multi_workspace, L.vip_svgd_step_multi, L.vip_ssvgd_step_multi):
        f.restype = ctypes.c_int
    return L


def vip_grad_logpost_multi(ctx: Context, problems, ckpt_every: int = 50, ws_tag: str = "multi"):
    """Gradients of several inversions in merged launches; returns [(logpost, grad)]."""
    ctx.sync_stream()
    L = _multi_lib()
    arr = (VipProblem * len(problems))(*[p.c() for p in problems])
    nbytes = ctypes.c_size_t()
    _check(L.vip_grad_logpost_multi_workspace(len(problems), arr, ckpt_every, ctypes.byref(nbytes)),
           "vip_grad_logpost_multi_workspace")
    ws = ctx.workspace(ws_tag, nbytes.value)
    _check(L.vip_grad_logpost_multi(ctx.handle, len(problems), arr, ckpt_every,
                                    ctypes.c_void_p(ws.data_ptr()), ws.numel()),
           "vip_grad_logpost_multi")
    return [(p.logpost, p.grad) for p in problems]


def _ensembles(xs, gs, eps, lo, hi, xis, h2s):
    out = []
    for k, (x, g) in enumerate(zip(xs, gs)):
        n = x.shape[0]
        pr = _prior(lo[k], hi[k]) if lo is not None else None
        out.append(VipEnsemble(n, x.numel() // n, _ptr(x, torch.float32), _ptr(g, torch.float32),
                               float(eps[k]), pr or VipPrior(VIP_PRIOR_NONE),
                               _ptr(xis[k], torch.float32) if xis is not None else None,
                               _ptr(h2s[k], torch.float64) if h2s is not None else None))
    return (VipEnsemble * len(out))(*out)


def vip_ssvgd_step_multi(ctx: Context, xs, gs, eps, xis=None, seed=0, stream=0, lo=None, hi=None,
                         h2s=None, bw_mode=VIP_BW_MEDIAN_ALL, h_fixed=1.0,
                         gram_prec=VIP_GRAM_BF16, noise=True, ws_tag="svgd_multi"):
    """In-place (s)SVGD update of several independent ensembles; returns the workspace."""
    ctx.sync_stream()
    L = _multi_lib()
    arr = _ensembles(xs, gs, eps, lo, hi, xis, h2s)
    nbytes = ctypes.c_size_t()
    _check(L.vip_svgd_multi_workspace(len(xs), arr, ctypes.byref(nbytes)), "vip_svgd_multi_workspace")
    ws = ctx.workspace(ws_tag, nbytes.value)
    if noise:
        st = L.vip_ssvgd_step_multi(ctx.handle, len(xs), arr, bw_mode, h_fixed, gram_prec, seed,
                                    stream, ctypes.c_void_p(ws.data_ptr()), ws.numel())
    else:
        st = L.vip_svgd_step_multi(ctx.handle, len(xs), arr, bw_mode, h_fixed, gram_prec,
                                   ctypes.c_void_p(ws.data_ptr()), ws.numel())
    _check(st, "vip_(s)svgd_step_multi")
    return ws


class Advi:
    """Variational parameters of the ADVI Gaussian family q = N(mu, L L^T) in
    the unconstrained space (vip_advi_sample / vip_advi_step), with the step
    rules' state.  Full rank: L is a [d][ldl] device array (ldl = d rounded up
    to 4) whose lower triangle L[:, :d] holds the factor; mean field: L is the
    diagonal [d].  Starts from N(mu0, scale^2 I)."""

    def __init__(self, d: int, family: int = VIP_ADVI_FULL_RANK, device=None,
                 kind: int = VIP_OPT_ADAM, beta1: float = 0.9, beta2: float = 0.999,
                 delta: float = 1e-8, mu0: Optional[torch.Tensor] = None, scale: float = 1.0,
                 ldl: Optional[int] = None):
        device = device if device is not None else torch.device("cuda", 0)
        self.d, self.family = int(d), family
        self.mu = (mu0.detach().to(device, torch.float32).reshape(-1).clone() if mu0 is not None
                   else torch.zeros(d, dtype=torch.float32, device=device))
        if family == VIP_ADVI_FULL_RANK:
            self.ldl = int(ldl) if ldl is not None else (d + 3) // 4 * 4
            self.L = torch.zeros(d, self.ldl, dtype=torch.float32, device=device)
            self.L[:, :d].diagonal().fill_(scale)
        else:
            self.ldl = 0
            self.L = torch.full((d,), float(scale), dtype=torch.float32, device=device)
        self.opt_mu = Optimizer(kind, self.mu, beta1, beta2, delta)
        self.opt_L = Optimizer(kind, self.L, beta1, beta2, delta)

    def factor(self) -> torch.Tensor:
        """L as a d x d lower-triangular (or diagonal) matrix."""
        if self.family == VIP_ADVI_FULL_RANK:
            return torch.tril(self.L[:, :self.d])
        return torch.diag(self.L)

    def covariance(self) -> torch.Tensor:
        Lm = self.factor().double()
        return Lm @ Lm.T


def vip_advi_sample(ctx: Context, q: Advi, eta: torch.Tensor,
                    theta: Optional[torch.Tensor] = None) -> torch.Tensor:
    """theta[s] = mu + L eta[s] (eta: [S][d] device float)."""
    ctx.sync_stream()
    S = eta.shape[0]
    if theta is None:
        theta = torch.empty(S, q.d, dtype=torch.float32, device=q.mu.device)
    _check(lib().vip_advi_sample(ctx.handle, q.family, q.d, S, _ptr(q.mu, torch.float32),
                                 _ptr(q.L, torch.float32), q.ldl, _ptr(eta, torch.float32),
                                 _ptr(theta, torch.float32)), "vip_advi_sample")
    return theta


def vip_advi_step(ctx: Context, q: Advi, eta: torch.Tensor, g: torch.Tensor, eps: float,
                  logpost: Optional[torch.Tensor] = None, grads: bool = False):
    """One ascent step of q from the samples' normals eta and gradients g
    ([S][d] each); returns (elbo or None, grad_mu or None, grad_L or None)."""
    ctx.sync_stream()
    S = eta.shape[0]
    dev = q.mu.device
    elbo = torch.empty(1, dtype=torch.float64, device=dev) if logpost is not None else None
    gm = torch.zeros_like(q.mu) if grads else None
    gL = torch.zeros_like(q.L) if grads else None
    q.opt_mu.t += 1
    q.opt_L.t += 1
    om, ol = q.opt_mu.c(), q.opt_L.c()
    _check(lib().vip_advi_step(ctx.handle, q.family, q.d, S, _ptr(q.mu, torch.float32),
                               _ptr(q.L, torch.float32), q.ldl, _ptr(eta, torch.float32),
                               _ptr(g, torch.float32), eps, ctypes.byref(om), ctypes.byref(ol),
                               _ptr(gm, torch.float32), _ptr(gL, torch.float32),
                               _ptr(logpost, torch.float64), _ptr(elbo, torch.float64)),
           "vip_advi_step")
    return elbo, gm, gL


def vip_advi_iteration(ctx: Context, q: Advi, grid: Grid, geom: Geometry, dobs: torch.Tensor,
                       sigma: float, prior: Prior, S: int, eps: float, seed: int, it: int,
                       ckpt_every: int = 50, stored_steps: int = 0, live_pairs: int = 0,
                       ws_tag: str = "advi"):
    """One ADVI iteration on the FWI posterior: Philox normals (key seed,
    stream it), the S samples, their log-posteriors and theta-gradients
    (vip_grad_logpost under `prior`, normally the transform of the uniform
    prior), and the step.  Returns the ELBO estimate (device double [1])."""
    eta = vip_philox_normals(ctx, S * q.d, seed, it).view(S, q.d)
    theta = vip_advi_sample(ctx, q, eta)
    lp, g = vip_grad_logpost(ctx, grid, geom, theta.view(S, grid.nz, grid.nx), dobs, sigma,
                             ckpt_every=ckpt_every, live_pairs=live_pairs,
                             stored_steps=stored_steps, prior=prior, ws_tag=ws_tag)
    elbo, _, _ = vip_advi_step(ctx, q, eta, g.view(S, q.d), eps, logpost=lp)
    return elbo
