"""Pins of the prior oracle (section 3, eq:transform) against closed forms,
finite differences and a library density."""
import numpy as np
import pytest
from scipy import stats

from oracle import fwi, prior, svgd


def test_transform_round_trip_and_derivatives():
    r = np.random.default_rng(1)
    a, b = 1500.0 + r.uniform(0, 100, 50), 3000.0 + r.uniform(0, 100, 50)
    m = a + (b - a) * r.uniform(0.01, 0.99, 50)
    th = prior.to_theta(m, a, b)
    assert np.allclose(prior.to_model(th, a, b), m, rtol=1e-13, atol=0)
    h = 1e-5
    fd = (prior.to_model(th + h, a, b) - prior.to_model(th - h, a, b)) / (2 * h)
    assert np.allclose(prior.dm_dtheta(th, a, b), fd, rtol=1e-8)
    # gradient of sum log|dm/dtheta|, one coordinate at a time
    g = prior.grad_log_jacobian(th, a, b)
    for k in range(0, 50, 7):
        e = np.zeros(50)
        e[k] = h
        fdk = (prior.log_jacobian(th + e, a, b) - prior.log_jacobian(th - e, a, b)) / (2 * h)
        assert abs(fdk - g[k]) <= 1e-7 * max(1.0, abs(g[k]))
    # closed forms at theta = 0: the midpoint, slope (b - a)/4, zero log-Jacobian gradient
    mid = prior.to_model(np.zeros(50), a, b)
    assert np.allclose(mid, 0.5 * (a + b), rtol=1e-15)
    assert np.allclose(prior.dm_dtheta(np.zeros(50), a, b), 0.25 * (b - a), rtol=1e-15)
    assert np.allclose(prior.grad_log_jacobian(np.zeros(50), a, b), 0.0, atol=1e-15)


def test_clip_is_idempotent():
    r = np.random.default_rng(2)
    x = r.uniform(1000, 4000, (5, 30))
    lo, hi = np.full(30, 1500.0), np.full(30, 3000.0)
    once = svgd.clip(x, lo, hi)
    assert np.array_equal(svgd.clip(once, lo, hi), once)
    assert once.min() >= 1500.0 and once.max() <= 3000.0


def test_gaussian_prior_matches_scipy_up_to_a_constant():
    r = np.random.default_rng(3)
    mean, std = r.uniform(1500, 3000, 40), r.uniform(50, 400, 40)
    m1, m2 = mean + std * r.standard_normal(40), mean + std * r.standard_normal(40)
    l1, g1 = prior.gaussian_log_prior(m1, mean, std)
    l2, _ = prior.gaussian_log_prior(m2, mean, std)
    s1 = stats.norm.logpdf(m1, mean, std).sum()
    s2 = stats.norm.logpdf(m2, mean, std).sum()
    assert abs((l1 - l2) - (s1 - s2)) <= 1e-10 * max(1.0, abs(s1 - s2))
    h = 1e-4
    for k in (0, 13, 39):
        e = np.zeros(40)
        e[k] = h
        fd = (prior.gaussian_log_prior(m1 + e, mean, std)[0] -
              prior.gaussian_log_prior(m1 - e, mean, std)[0]) / (2 * h)
        assert abs(fd - g1[k]) <= 1e-8 * max(1.0, abs(g1[k]))


def _tiny():
    grid = fwi.Grid(nz=10, nx=12, nb=6, nt=80, dx=10.0, dz=10.0, dt=1e-3)
    z = np.arange(10)[:, None]
    x = np.arange(12)[None, :]
    v_true = 1900.0 + 30.0 * z + 100.0 * np.exp(-((z - 5) ** 2 + (x - 6) ** 2) / 6.0)
    geom = fwi.Geometry(src_iz=(1,), src_ix=(5,), rec_iz=tuple([2] * 12),
                        rec_ix=tuple(range(12)), f0=30.0)
    dobs = fwi.simulate(v_true, grid, geom)
    sigma = 0.05 * float(np.sqrt(np.mean(dobs ** 2)))
    return grid, geom, dobs, sigma


def test_transformed_logpost_gradient_matches_finite_differences():
    grid, geom, dobs, sigma = _tiny()
    a, b = np.full((10, 12), 1600.0), np.full((10, 12), 2600.0)
    th = prior.to_theta(1950.0 + 25.0 * np.arange(10)[:, None] + 0 * np.arange(12)[None, :], a, b)
    lp, g = prior.transformed_grad_logpost(th[None], grid, geom, dobs, sigma, a, b)
    g = g[0]
    h = 1e-4
    cells = [(0, 0), (9, 11), (4, 6), (2, 9), (7, 1)]
    for (i, j) in cells:
        tp, tm = th.copy(), th.copy()
        tp[i, j] += h
        tm[i, j] -= h
        lpp, _ = prior.transformed_grad_logpost(tp[None], grid, geom, dobs, sigma, a, b)
        lpm, _ = prior.transformed_grad_logpost(tm[None], grid, geom, dobs, sigma, a, b)
        fd = (lpp[0] - lpm[0]) / (2 * h)
        assert abs(fd - g[i, j]) <= 1e-6 * np.abs(g).max(), ((i, j), fd, g[i, j])


def test_svgd_on_the_transformed_uniform_prior_reaches_the_logistic_law():
    """With no data the density of theta = log(m - a) - log(b - m) for m
    uniform on (a, b) is the standard logistic, mean 0, variance pi^2 / 3;
    SVGD driven by the log-Jacobian gradient alone reaches both."""
    r = np.random.default_rng(5)
    X = r.normal(0.5, 0.3, (300, 1))
    a, b = np.array([0.0]), np.array([1.0])
    for _ in range(600):
        G = prior.grad_log_jacobian(X, a, b)
        X, _ = svgd.svgd_step(X, G, 2.0)
    assert abs(X.mean()) < 0.02
    # finite-n SVGD with the median bandwidth settles a few percent narrow
    assert abs(X.var() / (np.pi ** 2 / 3.0) - 1.0) < 0.1
