"""Pins for the FP64 FWI oracle against what mathematics fixes independently of
it: the analytic 2-D Green's function, the adjoint identity, finite differences,
reciprocity, discrete energy conservation, exactness properties of the misfit,
the stability limit, and closed forms of each grid operator."""
import numpy as np
import pytest

from oracle import fwi
from tests.analytic import green2d_ricker, ricker_closed_form


def _homogeneous_trace(dx, dt, n_int, nt, v=2000.0, r=300.0, f0=10.0):
    grid = fwi.Grid(nz=n_int, nx=n_int, nb=20, nt=nt, dx=dx, dz=dx, dt=dt)
    c0 = n_int // 2
    off = int(round(r / dx))
    geom = fwi.Geometry(src_iz=(c0,), src_ix=(c0,), rec_iz=(c0,), rec_ix=(c0 + off,), f0=f0)
    d = fwi.simulate(np.full((n_int, n_int), v), grid, geom)[0, :, 0]
    ref = green2d_ricker(r, v, np.arange(nt) * dt, f0, 1.5 / f0)
    return np.linalg.norm(d - ref) / np.linalg.norm(ref)


def test_green_function_homogeneous():
    # 10 m, 1 ms, 10 Hz, v = 2000 m/s, offset 300 m; the window ends before the
    # first wave that reaches the sponge can return to the receiver.
    err = _homogeneous_trace(10.0, 1e-3, 141, 450)
    assert err <= 3e-3, err


@pytest.mark.slow
def test_green_function_converges():
    e1 = _homogeneous_trace(10.0, 1e-3, 141, 450)
    e2 = _homogeneous_trace(5.0, 5e-4, 281, 900)
    assert e1 / e2 >= 1.8, (e1, e2)


def _random_problem(seed, nz=12, nx=16, nb=6, nt=60, alpha=0.1, dx=10.0):
    r = np.random.default_rng(seed)
    grid = fwi.Grid(nz=nz, nx=nx, nb=nb, nt=nt, dx=dx, dz=dx * 1.25, dt=1e-3, alpha=alpha)
    vel = r.uniform(1500.0, 3500.0, size=(nz, nx))
    _, c = fwi.coefficient(vel, grid)
    return r, grid, vel, c, fwi.sponge(grid)


def test_adjoint_dot_product():
    r, grid, vel, c, g = _random_problem(1)
    NZ, NX = grid.NZ, grid.NX
    rec = (np.array([3, 7, 7, 10, 3]) + grid.nb, np.array([0, 5, 5, 15, 9]) + grid.nb)  # one duplicate
    x = r.standard_normal((grid.nt - 1, NZ, NX))
    y = r.standard_normal((grid.nt, len(rec[0])))
    Fx, _, _ = fwi.forward_shot(c, g, grid, None, rec, source_field=x)
    _, FTy = fwi.adjoint_shot(c, g, grid, rec, y, keep_z=True)
    lhs = float(np.sum(Fx[1:] * y[1:]))          # d^0 = 0 whatever y^0 is
    rhs = float(np.sum(x * FTy))
    assert abs(lhs - rhs) <= 1e-10 * max(abs(lhs), abs(rhs)), (lhs, rhs)


def _fd_setup():
    grid = fwi.Grid(nz=16, nx=20, nb=10, nt=150, dx=10.0, dz=10.0, dt=1e-3, alpha=0.05)
    z = np.arange(16)[:, None]
    x = np.arange(20)[None, :]
    v_true = 1800.0 + 40.0 * z + 150.0 * np.exp(-((z - 9) ** 2 + (x - 11) ** 2) / 12.0)
    v0 = 1800.0 + 38.0 * z + 5.0 * np.sin(0.7 * x)
    geom = fwi.Geometry(src_iz=(1, 2), src_ix=(4, 15), rec_iz=tuple([1] * 20),
                        rec_ix=tuple(range(20)), f0=25.0)
    dobs = fwi.simulate(v_true, grid, geom)
    sigma = 0.05 * float(np.sqrt(np.mean(dobs ** 2)))
    return grid, geom, v0, dobs, sigma


def test_gradient_matches_central_differences():
    grid, geom, v0, dobs, sigma = _fd_setup()
    J0, g = fwi.data_gradient(v0, grid, geom, dobs, sigma)
    cells = [(0, 0), (15, 19), (0, 10), (15, 3), (8, 0), (5, 19), (0, 19), (15, 0)]
    r = np.random.default_rng(3)
    cells += list(zip(r.integers(0, 16, 16).tolist(), r.integers(0, 20, 16).tolist()))
    gmax = np.abs(g).max()
    delta = 1e-2
    for (i, j) in cells:
        vp = v0.copy(); vp[i, j] += delta
        vm = v0.copy(); vm[i, j] -= delta
        Jp, _ = fwi.misfit(fwi.simulate(vp, grid, geom), dobs, sigma)
        Jm, _ = fwi.misfit(fwi.simulate(vm, grid, geom), dobs, sigma)
        fd = (Jp - Jm) / (2 * delta)
        assert abs(fd - g[i, j]) <= 1e-6 * gmax, ((i, j), fd, g[i, j], gmax)


def test_gradient_taylor_remainder_is_quadratic():
    grid, geom, v0, dobs, sigma = _fd_setup()
    J0, g = fwi.data_gradient(v0, grid, geom, dobs, sigma)
    p = np.random.default_rng(4).standard_normal(v0.shape)
    rem = []
    for h in (4.0, 2.0, 1.0):
        J1, _ = fwi.misfit(fwi.simulate(v0 + h * p, grid, geom), dobs, sigma)
        rem.append(abs(J1 - J0 - h * float(np.sum(g * p))))
    assert 3.0 < rem[0] / rem[1] < 5.0 and 3.0 < rem[1] / rem[2] < 5.0, rem


def test_reciprocity_without_sponge():
    # g = 1 and zero walls: M = diag(1/c) and L are symmetric, so the trace from
    # node A to node B equals the trace from B to A, whatever the velocity.
    r, grid, vel, c, _ = _random_problem(5, nz=20, nx=24, nb=4, nt=220, alpha=0.0)
    g = np.ones((grid.NZ, grid.NX))
    w = fwi.ricker(grid.nt, grid.dt, 30.0)
    A = (3 + grid.nb, 4 + grid.nb)
    B = (15 + grid.nb, 19 + grid.nb)
    ab = fwi.forward_shot(c, g, grid, A, (np.array([B[0]]), np.array([B[1]])), wavelet=w)[0][:, 0]
    ba = fwi.forward_shot(c, g, grid, B, (np.array([A[0]]), np.array([A[1]])), wavelet=w)[0][:, 0]
    assert np.linalg.norm(ab - ba) <= 1e-12 * np.linalg.norm(ab)


def test_discrete_energy_is_conserved_after_the_source():
    r, grid, vel, c, _ = _random_problem(6, nz=24, nx=24, nb=4, nt=400, alpha=0.0)
    g = np.ones((grid.NZ, grid.NX))
    f0 = 40.0
    w = fwi.ricker(grid.nt, grid.dt, f0)
    src = (12 + grid.nb, 12 + grid.nb)
    rec = (np.array([src[0]]), np.array([src[1]]))
    _, _, u = fwi.forward_shot(c, g, grid, src, rec, wavelet=w, keep_wavefield=True)
    n_quiet = int((1.5 / f0 + 3.0 / f0) / grid.dt)   # w < 1e-30 afterwards
    E = []
    for n in range(n_quiet, grid.nt - 1):
        du = u[n + 1] - u[n]
        E.append(float(np.sum(du * du / c)) - float(np.sum(u[n + 1] * fwi.laplacian(u[n], grid.dz, grid.dx))))
    E = np.array(E)
    assert E.min() > 0.0
    assert np.abs(E - E[0]).max() <= 1e-12 * abs(E[0])


def test_noise_free_data_give_zero_misfit_and_gradient():
    grid, geom, v0, _, _ = _fd_setup()
    dobs = fwi.simulate(v0, grid, geom)
    J, g = fwi.data_gradient(v0, grid, geom, dobs, 1.0)
    assert J == 0.0 and np.all(g == 0.0)


def test_data_are_linear_in_the_wavelet():
    r, grid, vel, c, g = _random_problem(7, nt=120)
    rec = (np.array([3, 9]) + grid.nb, np.array([2, 13]) + grid.nb)
    src = (5 + grid.nb, 8 + grid.nb)
    w1 = r.standard_normal(grid.nt)
    w2 = r.standard_normal(grid.nt)
    d1 = fwi.forward_shot(c, g, grid, src, rec, wavelet=w1)[0]
    d2 = fwi.forward_shot(c, g, grid, src, rec, wavelet=w2)[0]
    d12 = fwi.forward_shot(c, g, grid, src, rec, wavelet=2.0 * w1 - 3.0 * w2)[0]
    assert np.abs(d12 - (2.0 * d1 - 3.0 * d2)).max() <= 1e-12 * np.abs(d12).max()


def test_stability_limit():
    # sqrt(3/8) is the largest Courant number v dt / dx for which the 2-D
    # fourth-order leapfrog stays bounded (symbol maximum 32 / (3 dx^2)).
    n = 40
    grid_ok = fwi.Grid(nz=n, nx=n, nb=0, nt=1500, dx=10.0, dz=10.0, dt=0.99 * fwi.COURANT_LIMIT * 10.0 / 3000.0)
    grid_bad = fwi.Grid(nz=n, nx=n, nb=0, nt=1500, dx=10.0, dz=10.0, dt=1.03 * fwi.COURANT_LIMIT * 10.0 / 3000.0)
    v = np.full((n, n), 3000.0)
    geom = fwi.Geometry(src_iz=(20,), src_ix=(20,), rec_iz=(5,), rec_ix=(5,), f0=30.0)
    ok = np.abs(fwi.simulate(v, grid_ok, geom)).max()
    bad = np.abs(fwi.simulate(v, grid_bad, geom)).max()
    assert ok < 1.0 and bad > 1e6, (ok, bad)
    assert fwi.courant(3000.0, grid_ok) < fwi.COURANT_LIMIT < fwi.courant(3000.0, grid_bad)


def test_padding_fold_is_the_transpose():
    r = np.random.default_rng(8)
    v = r.standard_normal((7, 9))
    w = r.standard_normal((7 + 8, 9 + 8))
    assert abs(np.sum(fwi.pad_edge(v, 4) * w) - np.sum(v * fwi.fold_edge(w, 4))) < 1e-12
    # corners of the sponge fold into the corner cells: (nb + 1)^2 copies
    assert fwi.fold_edge(np.ones((15, 17)), 4)[0, 0] == 25.0
    assert fwi.fold_edge(np.ones((15, 17)), 4)[3, 4] == 1.0


def test_sponge_profile_values():
    p = fwi.sponge_profile(10, 20, 0.015)
    assert np.all(p[20:30] == 1.0)
    assert abs(p[0] - np.exp(-(0.015 * 20) ** 2)) < 1e-15 and abs(p[0] - 0.9139) < 1e-4
    assert np.allclose(p, p[::-1])


def test_laplacian_is_exact_on_quartics():
    # the fourth-order weights differentiate polynomials up to degree 5 exactly
    NZ, NX = 14, 15
    dz, dx = 2.0, 3.0
    z = (np.arange(NZ) * dz)[:, None]
    x = (np.arange(NX) * dx)[None, :]
    u = z ** 4 - 2 * z ** 2 * x + x ** 3 + 0 * z * x
    lap = 12 * z ** 2 - 4 * x + 6 * x
    L = fwi.laplacian(u, dz, dx)
    assert np.allclose(L[2:-2, 2:-2], lap[2:-2, 2:-2], rtol=1e-12, atol=1e-9)


def test_ricker_closed_form():
    w = fwi.ricker(400, 1e-3, 10.0)
    t = np.arange(400) * 1e-3
    assert np.allclose(w, ricker_closed_form(t, 10.0, 0.15), atol=1e-15)
    assert abs(w[150] - 1.0) < 1e-15                    # unit peak at t0
    # zero crossings at t0 +- 1 / (pi f sqrt 2)
    tz = 0.15 + 1.0 / (np.pi * 10.0 * np.sqrt(2.0))
    assert abs(ricker_closed_form(np.array([tz]), 10.0, 0.15)[0]) < 1e-15


def _minibatch_setup():
    """Four shots on a small grid (two particles) for the minibatch pins."""
    grid = fwi.Grid(nz=12, nx=14, nb=6, nt=90, dx=10.0, dz=10.0, dt=1e-3)
    z = np.arange(12)[:, None]
    x = np.arange(14)[None, :]
    v_true = 1900.0 + 35.0 * z + 120.0 * np.exp(-((z - 6) ** 2 + (x - 7) ** 2) / 8.0)
    geom = fwi.Geometry(src_iz=(1, 1, 2, 1), src_ix=(2, 5, 9, 12), rec_iz=tuple([2] * 14),
                        rec_ix=tuple(range(14)), f0=30.0)
    dobs = fwi.simulate(v_true, grid, geom)
    sigma = 0.05 * float(np.sqrt(np.mean(dobs ** 2)))
    vels = np.stack([1900.0 + 33.0 * z + 4.0 * np.sin(0.5 * x) + 0 * x,
                     1950.0 + 30.0 * z + 0 * x])
    return grid, geom, vels, dobs, sigma


def test_minibatch_estimate_is_unbiased_over_all_subsets():
    """Section 2.4's stochastic gradient from uniformly random shot subsets:
    the average over every subset of b shots reproduces the full-data
    log-likelihood and gradient (a wrong scale, or a wrong shot, breaks it)."""
    import itertools
    grid, geom, vels, dobs, sigma = _minibatch_setup()
    lp_full, g_full = fwi.grad_logpost(vels, grid, geom, dobs, sigma)
    for b in (1, 2, 3):
        subsets = list(itertools.combinations(range(geom.ns), b))
        lps, gs = zip(*[fwi.minibatch_grad_logpost(vels, grid, geom, dobs, sigma, s)
                        for s in subsets])
        lp_avg, g_avg = np.mean(lps, axis=0), np.mean(gs, axis=0)
        assert np.allclose(lp_avg, lp_full, rtol=1e-12, atol=0), b
        assert np.linalg.norm(g_avg - g_full) <= 1e-12 * np.linalg.norm(g_full), b
    # all shots in another order: the full-data value itself
    lp_all, g_all = fwi.minibatch_grad_logpost(vels, grid, geom, dobs, sigma, [2, 0, 3, 1])
    assert np.allclose(lp_all, lp_full, rtol=1e-12, atol=0)
    assert np.linalg.norm(g_all - g_full) <= 1e-12 * np.linalg.norm(g_full)
    # one subset is not the full value (the estimate is stochastic)
    lp_one, _ = fwi.minibatch_grad_logpost(vels, grid, geom, dobs, sigma, [1, 3])
    assert not np.allclose(lp_one, lp_full, rtol=1e-3)
