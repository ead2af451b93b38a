"""FP64 oracle: 2-D acoustic finite-difference forward modelling, its exact
discrete adjoint, and the adjoint-state gradient of the log-posterior.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).  Written in plain NumPy,
float64 throughout, storing the whole forward history (no checkpointing), so
that it follows a different code path from the library on purpose.

What the paper fixes (VIP, section 4.2 "Full-waveform inversion"):
  * waveforms come from a time-domain finite-difference simulation driven by a
    Ricker wavelet; data noise is Gaussian (eq:likelihood);
  * gradients of the log-posterior with respect to velocity come from the
    adjoint method (section 3, "Code overview");
  * the inversion layer only needs log-posterior values and gradients per
    particle (section 3), i.e. ``grad_logpost`` below.

What it leaves open, and the reading taken here:
  * constant-density acoustic equation (1/v^2) u_tt - lap(u) = f, one velocity
    per cell;
  * second order in time, fourth order in space (central weights
    -1/12, 4/3, -5/2, 4/3, -1/12), u = 0 on two ghost layers outside the
    padded grid;
  * Cerjan absorbing sponge of nb cells on all four sides:
    g = gamma(delta_z) * gamma(delta_x), gamma(delta) = exp(-(alpha delta)^2),
    applied as u^{n+1} = g (2u^n + c (L u^n + f^n) - g u^{n-1});
  * velocity inside the sponge = edge replication of the model (map P), so the
    gradient is folded back with P^T;
  * unit-peak Ricker with t0 = 1.5/f, injected as w(t_n)/(dx dz) at one node;
  * receivers read grid nodes, samples n = 0..nt-1 (d^0 = 0).
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

# Central fourth-order weights of the second derivative at offsets -2..2.
D2_OFFSETS = (-2, -1, 0, 1, 2)
D2_WEIGHTS = (-1.0 / 12.0, 4.0 / 3.0, -5.0 / 2.0, 4.0 / 3.0, -1.0 / 12.0)


@dataclass(frozen=True)
class Grid:
    """Interior nz x nx cells (z = rows = depth, x = columns), sponge width nb."""
    nz: int
    nx: int
    nb: int
    nt: int
    dx: float
    dz: float
    dt: float
    alpha: float = 0.015

    @property
    def NZ(self) -> int:
        return self.nz + 2 * self.nb

    @property
    def NX(self) -> int:
        return self.nx + 2 * self.nb


@dataclass(frozen=True)
class Geometry:
    """Shot and receiver nodes in interior (iz, ix) indices; the same receivers
    record every shot (section 4.2).  f0 is the Ricker peak frequency."""
    src_iz: tuple
    src_ix: tuple
    rec_iz: tuple
    rec_ix: tuple
    f0: float
    t0: float | None = None

    @property
    def ns(self) -> int:
        return len(self.src_iz)

    @property
    def nr(self) -> int:
        return len(self.rec_iz)


# ----------------------------------------------------------------------------
# Grid operators
# ----------------------------------------------------------------------------

def pad_edge(v: np.ndarray, nb: int) -> np.ndarray:
    """P: extend the model into the sponge by replicating its edge cells."""
    return np.pad(np.asarray(v, dtype=np.float64), nb, mode="edge")


def fold_edge(gp: np.ndarray, nb: int) -> np.ndarray:
    """P^T: every padded cell adds into the interior cell it was copied from.

    Written as an explicit sum over padded cells so that it is the transpose of
    pad_edge by construction."""
    NZ, NX = gp.shape
    nz, nx = NZ - 2 * nb, NX - 2 * nb
    out = np.zeros((nz, nx))
    src_row = np.clip(np.arange(NZ) - nb, 0, nz - 1)
    src_col = np.clip(np.arange(NX) - nb, 0, nx - 1)
    for i in range(NZ):
        np.add.at(out[src_row[i]], src_col, gp[i])
    return out


def sponge_profile(n: int, nb: int, alpha: float) -> np.ndarray:
    """gamma(delta(k)) along one padded axis of n interior cells."""
    k = np.arange(n + 2 * nb)
    delta = np.maximum(np.maximum(nb - k, k - (nb + n - 1)), 0)
    return np.exp(-(alpha * delta.astype(np.float64)) ** 2)


def sponge(grid: Grid) -> np.ndarray:
    """Separable Cerjan damping factor g over the padded grid (1 inside)."""
    return np.outer(sponge_profile(grid.nz, grid.nb, grid.alpha),
                    sponge_profile(grid.nx, grid.nb, grid.alpha))


def laplacian(u: np.ndarray, dz: float, dx: float) -> np.ndarray:
    """(L u)_ij = sum_o w_o (u_{i+o,j}/dz^2 + u_{i,j+o}/dx^2), zero ghosts."""
    NZ, NX = u.shape
    p = np.zeros((NZ + 4, NX + 4))
    p[2:2 + NZ, 2:2 + NX] = u
    out = np.zeros((NZ, NX))
    for o, w in zip(D2_OFFSETS, D2_WEIGHTS):
        out += w * (p[2 + o:2 + o + NZ, 2:2 + NX] / dz ** 2
                    + p[2:2 + NZ, 2 + o:2 + o + NX] / dx ** 2)
    return out


def ricker(nt: int, dt: float, f0: float, t0: float | None = None) -> np.ndarray:
    """Unit-peak Ricker wavelet w(t_n), t_n = n dt, centred at t0 (1.5/f0)."""
    if t0 is None:
        t0 = 1.5 / f0
    t = np.arange(nt, dtype=np.float64) * dt
    arg = (np.pi * f0 * (t - t0)) ** 2
    return (1.0 - 2.0 * arg) * np.exp(-arg)


def coefficient(vel: np.ndarray, grid: Grid):
    """Padded velocity and c = v_pad^2 dt^2."""
    v_pad = pad_edge(vel, grid.nb)
    return v_pad, v_pad ** 2 * grid.dt ** 2


def courant(vmax: float, grid: Grid) -> float:
    return vmax * grid.dt / min(grid.dx, grid.dz)


COURANT_LIMIT = float(np.sqrt(3.0 / 8.0))


# ----------------------------------------------------------------------------
# One shot: forward, adjoint
# ----------------------------------------------------------------------------

def _nodes(grid: Grid, iz, ix):
    return (np.asarray(iz, dtype=np.int64) + grid.nb,
            np.asarray(ix, dtype=np.int64) + grid.nb)


def forward_shot(c, g, grid: Grid, src, rec, wavelet=None, source_field=None,
                 keep_history=False, keep_wavefield=False):
    """Leapfrog forward simulation of one shot.

    u^0 = u^{-1} = 0; for n = 0 .. nt-2:
        a^n     = L u^n + f^n
        u^{n+1} = g (2 u^n + c a^n - g u^{n-1})
    with f^n = w(t_n)/(dx dz) at the source node, or an arbitrary space-time
    field ``source_field[n]``.  Traces d^n_r = u^n(x_r), n = 0 .. nt-1.

    Returns (traces [nt][nr], a-history [nt-1][NZ][NX] or None,
    wavefield history [nt][NZ][NX] or None)."""
    nt, NZ, NX = grid.nt, grid.NZ, grid.NX
    rz, rx = rec
    traces = np.zeros((nt, len(rz)))
    hist = np.zeros((nt - 1, NZ, NX)) if keep_history else None
    wave = np.zeros((nt, NZ, NX)) if keep_wavefield else None
    u_prev = np.zeros((NZ, NX))
    u = np.zeros((NZ, NX))
    area = grid.dx * grid.dz
    for n in range(nt - 1):
        a = laplacian(u, grid.dz, grid.dx)
        if source_field is not None:
            a = a + source_field[n]
        else:
            a[src] += wavelet[n] / area
        u_next = g * (2.0 * u + c * a - g * u_prev)
        traces[n + 1] = u_next[rz, rx]
        if hist is not None:
            hist[n] = a
        if wave is not None:
            wave[n + 1] = u_next
        u_prev, u = u, u_next
    return traces, hist, wave


def adjoint_shot(c, g, grid: Grid, rec, rho, a_hist=None, keep_z=False):
    """Exact discrete adjoint of forward_shot, in the scaled variable
    z = g c lambda (lambda = Lagrange multiplier of the step equation), which
    obeys the same recurrence as the forward field:

    z^{nt} = z^{nt+1} = 0; for n = nt-1 .. 1:
        b   = L z^{n+1} + R^T rho^n
        z^n = g (2 z^{n+1} + c b - g z^{n+2})

    (L is symmetric, R^T scatters receiver values onto their nodes.)
    With a-history, returns img = sum_{n=0}^{nt-2} z^{n+1} * a^n, and with
    keep_z the adjoint of the source-field map: zs[n] = z^{n+1}."""
    nt, NZ, NX = grid.nt, grid.NZ, grid.NX
    rz, rx = rec
    z1 = np.zeros((NZ, NX))   # z^{n+1}
    z2 = np.zeros((NZ, NX))   # z^{n+2}
    img = np.zeros((NZ, NX)) if a_hist is not None else None
    zs = np.zeros((nt - 1, NZ, NX)) if keep_z else None
    for n in range(nt - 1, 0, -1):
        b = laplacian(z1, grid.dz, grid.dx)
        np.add.at(b, (rz, rx), rho[n])
        z = g * (2.0 * z1 + c * b - g * z2)
        if img is not None:
            img += z * a_hist[n - 1]
        if zs is not None:
            zs[n - 1] = z
        z2, z1 = z1, z
    return img, zs


# ----------------------------------------------------------------------------
# Whole problem: data, misfit, gradient, log-posterior
# ----------------------------------------------------------------------------

def simulate(vel, grid: Grid, geom: Geometry) -> np.ndarray:
    """Receiver data d[s][n][r] for every shot of one velocity model."""
    _, c = coefficient(vel, grid)
    g = sponge(grid)
    w = ricker(grid.nt, grid.dt, geom.f0, geom.t0)
    rec = _nodes(grid, geom.rec_iz, geom.rec_ix)
    out = np.zeros((geom.ns, grid.nt, geom.nr))
    for s in range(geom.ns):
        src = (geom.src_iz[s] + grid.nb, geom.src_ix[s] + grid.nb)
        out[s] = forward_shot(c, g, grid, src, rec, wavelet=w)[0]
    return out


def misfit(d, dobs, sigma):
    """J = 1/2 sum ((d - dobs)/sigma)^2 (minus log of eq:likelihood, constants
    dropped) and the residual rho = (d - dobs)/sigma^2 = dJ/dd."""
    r = np.asarray(d, dtype=np.float64) - np.asarray(dobs, dtype=np.float64)
    return 0.5 * float(np.sum(r * r)) / sigma ** 2, r / sigma ** 2


def shot_gradient(c, g, v_pad, grid: Grid, geom: Geometry, s: int, dobs_s,
                  sigma: float, wavelet):
    """(J_s, dJ_s/dv_pad) for one shot: forward with history, residual,
    adjoint, imaging dJ/dv_pad = (2/v_pad) sum_n z^{n+1} a^n
    (dc/dv = 2 v dt^2 = 2c/v, and dJ/dc = sum_n g lambda^{n+1} a^n =
    sum_n z^{n+1} a^n / c)."""
    rec = _nodes(grid, geom.rec_iz, geom.rec_ix)
    src = (geom.src_iz[s] + grid.nb, geom.src_ix[s] + grid.nb)
    traces, hist, _ = forward_shot(c, g, grid, src, rec, wavelet=wavelet,
                                   keep_history=True)
    J, rho = misfit(traces, dobs_s, sigma)
    img, _ = adjoint_shot(c, g, grid, rec, rho, a_hist=hist)
    return J, 2.0 / v_pad * img


def data_gradient(vel, grid: Grid, geom: Geometry, dobs, sigma):
    """(J, dJ/dv) for one model: shot sum of padded gradients, then P^T."""
    v_pad, c = coefficient(vel, grid)
    g = sponge(grid)
    w = ricker(grid.nt, grid.dt, geom.f0, geom.t0)
    J = 0.0
    gpad = np.zeros((grid.NZ, grid.NX))
    for s in range(geom.ns):
        Js, gs = shot_gradient(c, g, v_pad, grid, geom, s, dobs[s], sigma, w)
        J += Js
        gpad += gs
    return J, fold_edge(gpad, grid.nb)


def uniform_log_prior(vel, lo, hi):
    """Uniform prior (section 3): log p = 0 inside [lo, hi] (normalising
    constant dropped), -inf outside; gradient 0 inside."""
    inside = np.all((vel >= lo) & (vel <= hi))
    return (0.0 if inside else -np.inf), np.zeros_like(np.asarray(vel, dtype=np.float64))


def grad_logpost(vels, grid: Grid, geom: Geometry, dobs, sigma, lo=None, hi=None):
    """log p(m|d) (up to a constant, eq:Bayes) and its gradient for every
    particle: log-likelihood -J plus log-prior."""
    vels = np.asarray(vels, dtype=np.float64)
    npart = vels.shape[0]
    logpost = np.zeros(npart)
    grad = np.zeros_like(vels)
    for p in range(npart):
        J, dJ = data_gradient(vels[p], grid, geom, dobs, sigma)
        lp, glp = (0.0, 0.0) if lo is None else uniform_log_prior(vels[p], lo, hi)
        logpost[p] = -J + lp
        grad[p] = -dJ + glp
    return logpost, grad


def minibatch_grad_logpost(vels, grid: Grid, geom: Geometry, dobs, sigma, shots, lo=None,
                           hi=None):
    """Section 2.4: the gradient of log p computed from uniformly random data
    subsets -- here a subset of the shots -- is a stochastic approximation; the
    log-likelihood of the subset scaled by ns / |subset| has the full-data value
    as its expectation over subsets, and so has its gradient.  dobs holds every
    shot of the survey; `shots` lists the subset (any order)."""
    vels = np.asarray(vels, dtype=np.float64)
    shots = [int(s) for s in shots]
    scale = geom.ns / len(shots)
    g = sponge(grid)
    w = ricker(grid.nt, grid.dt, geom.f0, geom.t0)
    logpost = np.zeros(vels.shape[0])
    grad = np.zeros_like(vels)
    for p in range(vels.shape[0]):
        v_pad, c = coefficient(vels[p], grid)
        J = 0.0
        gpad = np.zeros((grid.NZ, grid.NX))
        for s in shots:
            Js, gs = shot_gradient(c, g, v_pad, grid, geom, s, dobs[s], sigma, w)
            J += Js
            gpad += gs
        lp, glp = (0.0, 0.0) if lo is None else uniform_log_prior(vels[p], lo, hi)
        logpost[p] = -scale * J + lp
        grad[p] = -scale * fold_edge(gpad, grid.nb) + glp
    return logpost, grad
