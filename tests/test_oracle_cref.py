"""Pins for the C oracle (oracle/cref.c): it must agree with the pinned NumPy
oracle to rounding, and its gradient must match central differences of its
own forward."""
import numpy as np

from oracle import cref, fwi, svgd


def _problem(seed=0):
    r = np.random.default_rng(seed)
    grid = fwi.Grid(nz=14, nx=19, nb=7, nt=130, dx=10.0, dz=12.0, dt=1e-3, alpha=0.08)
    vel = r.uniform(1600.0, 3200.0, size=(14, 19))
    geom = fwi.Geometry(src_iz=(0, 13, 6), src_ix=(0, 18, 9), rec_iz=(1, 1, 5, 13, 0),
                        rec_ix=(0, 7, 18, 3, 10), f0=30.0)
    return r, grid, vel, geom


def test_forward_matches_numpy_oracle():
    _, grid, vel, geom = _problem()
    a = cref.simulate(vel, grid, geom, workers=2)
    b = fwi.simulate(vel, grid, geom)
    assert np.abs(a - b).max() <= 1e-12 * np.abs(b).max()


def test_gradient_matches_numpy_oracle_and_finite_differences():
    r, grid, vel, geom = _problem(1)
    dobs = fwi.simulate(vel * 1.03, grid, geom) + 1e-3 * r.standard_normal((3, 130, 5))
    sigma = 0.01
    lp_c, g_c = cref.grad_logpost(vel[None], grid, geom, dobs, sigma, workers=3)
    lp_n, g_n = fwi.grad_logpost(vel[None], grid, geom, dobs, sigma)
    assert abs(lp_c[0] - lp_n[0]) <= 1e-12 * abs(lp_n[0])
    assert np.abs(g_c - g_n).max() <= 1e-11 * np.abs(g_n).max()
    gmax = np.abs(g_c).max()
    for (i, j) in [(0, 0), (13, 18), (7, 9), (0, 12), (10, 0)]:
        vp = vel.copy(); vp[i, j] += 1e-2
        vm = vel.copy(); vm[i, j] -= 1e-2
        Jp = 0.5 * np.sum((cref.simulate(vp, grid, geom) - dobs) ** 2) / sigma ** 2
        Jm = 0.5 * np.sum((cref.simulate(vm, grid, geom) - dobs) ** 2) / sigma ** 2
        fd = (Jp - Jm) / 2e-2
        assert abs(fd + g_c[0, i, j]) <= 1e-6 * gmax, (i, j, fd, -g_c[0, i, j])


def test_sqdist_matches_numpy_oracle():
    X = np.random.default_rng(2).standard_normal((37, 101)) * 50.0 + 3000.0
    D = cref.sqdist(X, workers=3, block=5)
    assert np.abs(D - svgd.sqdist(X)).max() <= 1e-12 * D.max()
    assert np.all(np.diag(D) == 0.0)


def test_snapshots_match_numpy_oracle_wavefield():
    _, grid, vel, geom = _problem(4)
    _, c = fwi.coefficient(vel, grid)
    g = fwi.sponge(grid)
    w = fwi.ricker(grid.nt, grid.dt, geom.f0)
    rec = (np.asarray(geom.rec_iz) + grid.nb, np.asarray(geom.rec_ix) + grid.nb)
    for s in (0, 2):
        src = (geom.src_iz[s] + grid.nb, geom.src_ix[s] + grid.nb)
        _, _, wave = fwi.forward_shot(c, g, grid, src, rec, wavelet=w, keep_wavefield=True)
        steps = [0, 1, 17, 64, 65, grid.nt - 1]
        snap = cref.snapshots(vel, grid, geom, s, steps)
        for k, n in enumerate(steps):
            assert np.abs(snap[k] - wave[n]).max() <= 1e-12 * max(np.abs(wave[n]).max(), 1e-300), n
        assert np.all(snap[0] == 0.0)
