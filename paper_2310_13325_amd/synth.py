"""Seeded synthetic inputs shared by the tests, the smoke check and the
benchmark.

Holds none of the method's arithmetic (no wave propagation, no wavelet, no
kernel, no update): only velocity models, prior bounds, initial particles and
standard-normal draws.  The paper's own data (the Marmousi section of its
section 4.2 and the British-Isles travel times of section 4.1) are not
available; these recipes stand in for them:

* "layers_anomalies": 4 flat layers (interfaces at sorted U(0.15, 0.9) x depth,
  velocities sorted U[1500, 3000] m/s with the top layer at 1500) plus two
  Gaussian anomalies of +-U(200, 400) m/s, width 0.08 min(nx, nz) cells,
  centred in the middle half of the grid; clipped to [1500, 3000].
* "faulted" (Marmousi stand-in): water rows at 1500 m/s; below them a
  background rising linearly from 1800 to 4200 m/s, ten dipping interfaces
  (dip U(-10, 10) degrees, contrast +-U(50, 300) m/s) offset by three normal
  faults (dip U(55, 75) degrees, throw U(40, 160) m on the hanging wall);
  clipped to [1500, 4500].
* prior "rowmean_pm500": U(vbar(z) - 500, vbar(z) + 500), vbar the row mean of
  the true model; "background_2kms": U(max(1500, vb - 1000), vb + 1000), vb the
  background, i.e. a 2 km/s interval per depth with a 1.5 km/s floor
  (section 4.2).
* initial particles i.i.d. uniform within the prior (section 4.2).
* every random stream derives from numpy SeedSequence(seed).spawn(7):
  [model, data noise, particles, sSVGD normals, finite-difference cells,
  SVGD-precision fields, minibatch shot subsets] (the i-th child of a
  SeedSequence does not depend on how many are spawned).
"""
from __future__ import annotations

import numpy as np

(STREAM_MODEL, STREAM_NOISE, STREAM_PARTICLES, STREAM_XI, STREAM_FDCELLS, STREAM_C5,
 STREAM_MINIBATCH) = range(7)


def rng(seed: int, stream: int) -> np.random.Generator:
    return np.random.default_rng(np.random.SeedSequence(seed).spawn(7)[stream])


def layers_anomalies(nz: int, nx: int, r: np.random.Generator) -> np.ndarray:
    iface = np.sort(r.uniform(0.15, 0.9, size=3)) * nz
    vlay = np.sort(r.uniform(1500.0, 3000.0, size=4))
    vlay[0] = 1500.0
    z = np.arange(nz)[:, None] + 0.5
    x = np.arange(nx)[None, :] + 0.5
    layer = np.searchsorted(iface, z[:, 0])
    v = np.repeat(vlay[layer][:, None], nx, axis=1).astype(np.float64)
    width = 0.08 * min(nx, nz)
    for _ in range(2):
        amp = r.choice([-1.0, 1.0]) * r.uniform(200.0, 400.0)
        cz = r.uniform(0.25, 0.75) * nz
        cx = r.uniform(0.25, 0.75) * nx
        v += amp * np.exp(-((z - cz) ** 2 + (x - cx) ** 2) / (2.0 * width ** 2))
    return np.clip(v, 1500.0, 3000.0)


def faulted(nz: int, nx: int, dx: float, water_rows: int, r: np.random.Generator):
    """Returns (model, background); both [nz][nx] float64."""
    z = np.arange(nz, dtype=np.float64)[:, None] + 0.5
    x = np.arange(nx, dtype=np.float64)[None, :] + 0.5
    depth_frac = np.clip((z - water_rows) / max(nz - water_rows, 1), 0.0, 1.0)
    vb = 1800.0 + (4200.0 - 1800.0) * depth_frac
    vb = np.where(z < water_rows, 1500.0, vb) * np.ones((1, nx))
    # Normal faults: a point on the hanging-wall side sees the layering shifted
    # down by the throw.
    zs = np.repeat(z, nx, axis=1).copy()
    for _ in range(3):
        x_top = r.uniform(0.2, 0.8) * nx
        dip = np.deg2rad(r.uniform(55.0, 75.0))
        side = r.choice([-1.0, 1.0])
        throw = r.uniform(40.0, 160.0) / dx
        x_plane = x_top + side * (z - water_rows) / np.tan(dip)
        hanging = side * (x - x_plane) > 0.0
        zs = zs - throw * hanging
    pert = np.zeros((nz, nx))
    tops = np.sort(r.uniform(water_rows + 2, nz - 2, size=10))
    for zk in tops:
        dipk = np.deg2rad(r.uniform(-10.0, 10.0))
        contrast = r.choice([-1.0, 1.0]) * r.uniform(50.0, 300.0)
        pert += contrast * (zs > zk + np.tan(dipk) * (x - nx / 2.0))
    v = np.where(z < water_rows, 1500.0, np.clip(vb + pert, 1500.0, 4500.0))
    return v.astype(np.float64), vb.astype(np.float64)


def true_model(prob):
    """(v_true, background) for a Problem."""
    r = rng(prob.seed, STREAM_MODEL)
    if prob.model == "layers_anomalies":
        v = layers_anomalies(prob.nz, prob.nx, r)
        return v, np.repeat(v.mean(axis=1, keepdims=True), prob.nx, axis=1)
    if prob.model == "faulted":
        return faulted(prob.nz, prob.nx, prob.dx, prob.water_rows, r)
    raise ValueError(prob.model)


def prior_bounds(prob, v_true, background):
    if prob.prior == "rowmean_pm500":
        vbar = np.repeat(v_true.mean(axis=1, keepdims=True), prob.nx, axis=1)
        return vbar - 500.0, vbar + 500.0
    if prob.prior == "background_2kms":
        return np.maximum(1500.0, background - 1000.0), background + 1000.0
    raise ValueError(prob.prior)


def initial_particles(prob, lo, hi, count=None):
    r = rng(prob.seed, STREAM_PARTICLES)
    n = prob.np if count is None else count
    return r.uniform(lo[None], hi[None], size=(n,) + lo.shape)


def noise(prob):
    """Standard-normal data noise [ns][nt][nr]; scaled by sigma by the caller."""
    return rng(prob.seed, STREAM_NOISE).standard_normal((prob.ns, prob.nt, prob.nr))


def normals(seed: int, n: int, d: int) -> np.ndarray:
    """Standard-normal [n][d] array for the sSVGD noise (passed to both sides)."""
    return rng(seed, STREAM_XI).standard_normal((n, d))


def fd_cells(prob, count: int = 32):
    """Interior cells for finite-difference gradient checks: a quarter on the
    model edges / corners (where the sponge copies fold back), the rest random."""
    r = rng(prob.seed, STREAM_FDCELLS)
    edge = [(0, 0), (prob.nz - 1, prob.nx - 1), (0, prob.nx // 2), (prob.nz - 1, prob.nx // 3),
            (prob.nz // 2, 0), (prob.nz // 3, prob.nx - 1), (0, prob.nx - 1), (prob.nz - 1, 0)]
    k = count - len(edge)
    iz = r.integers(0, prob.nz, size=k)
    ix = r.integers(0, prob.nx, size=k)
    cells = edge[: min(len(edge), count)] + list(zip(iz.tolist(), ix.tolist()))
    return cells[:count]


def smooth_fields(n: int, nz: int, nx: int, r: np.random.Generator, sigma_cells=2.0):
    """n Gaussian-smoothed N(0,1) fields, rescaled to unit RMS each."""
    from scipy.ndimage import gaussian_filter
    out = np.empty((n, nz, nx))
    for i in range(n):
        f = gaussian_filter(r.standard_normal((nz, nx)), sigma_cells, mode="reflect")
        out[i] = f / np.sqrt(np.mean(f * f))
    return out


def svgd_precision_case(case, v_center):
    """Particles X_i = v + spread zeta_i and gradient-like fields
    G_i = -(X_i - v)/spread^2 + 1e-4 N(0,1), as float64 [n][d]."""
    r = rng(case.seed, STREAM_C5)
    nz, nx = v_center.shape
    zeta = smooth_fields(case.n, nz, nx, r)
    X = v_center[None] + case.spread * zeta
    G = -(X - v_center[None]) / case.spread ** 2 + 1e-4 * r.standard_normal(X.shape)
    return X.reshape(case.n, -1), G.reshape(case.n, -1)


def minibatch_shots(seed: int, ns: int, b: int, iterations: int) -> np.ndarray:
    """[iterations][b] shot subsets, each drawn uniformly without replacement
    (section 2.4's uniformly random data subsets; passed to both sides)."""
    r = rng(seed, STREAM_MINIBATCH)
    return np.stack([r.choice(ns, size=b, replace=False) for _ in range(iterations)])
