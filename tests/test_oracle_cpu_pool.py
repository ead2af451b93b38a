"""Pins for oracle/cpu_pool.py, which spreads the oracle's (particle, shot)
pairs over processes (the CPU baseline and large references use it): it must
reproduce oracle.fwi, itself pinned by the Green's function, the dot-product
test and central differences (test_oracle_fwi.py), to rounding -- so a wrong
shot sum, edge fold or sign in the pool fails here.  Also the -inf branch of
the uniform log-prior (a particle outside its bounds)."""
import numpy as np

from oracle import cpu_pool, fwi


def _problem(seed=3):
    r = np.random.default_rng(seed)
    grid = fwi.Grid(nz=13, nx=17, nb=6, nt=110, dx=10.0, dz=10.0, dt=1e-3, alpha=0.07)
    geom = fwi.Geometry(src_iz=(0, 12, 5), src_ix=(0, 16, 8), rec_iz=(1, 1, 6, 12),
                        rec_ix=(0, 9, 16, 4), f0=28.0)
    v_true = r.uniform(1700.0, 3000.0, size=(13, 17))
    vels = v_true[None] * r.uniform(0.95, 1.05, size=(3, 13, 17))
    sigma = 0.02
    dobs = fwi.simulate(v_true, grid, geom) + 1e-3 * r.standard_normal((3, 110, 4))
    return grid, geom, vels, dobs, sigma


def test_pool_simulate_matches_oracle():
    grid, geom, vels, _, _ = _problem()
    a = cpu_pool.simulate(vels[1], grid, geom, workers=2)
    b = fwi.simulate(vels[1], grid, geom)
    assert a.shape == b.shape
    assert np.abs(a - b).max() <= 1e-12 * np.abs(b).max()


def test_pool_gradients_match_oracle():
    grid, geom, vels, dobs, sigma = _problem()
    lp_a, g_a = cpu_pool.grad_logpost(vels, grid, geom, dobs, sigma, workers=2)
    lp_b, g_b = fwi.grad_logpost(vels, grid, geom, dobs, sigma)
    assert np.all(np.abs(lp_a - lp_b) <= 1e-12 * np.abs(lp_b))
    for p in range(vels.shape[0]):
        assert np.abs(g_a[p] - g_b[p]).max() <= 1e-12 * np.abs(g_b[p]).max()
    # the edge fold: cells of the first and last rows and columns carry the
    # sponge copies, so they differ from an unfolded interior-only gradient
    assert np.abs(g_a[0, 0, 0]) > 0.0 and np.abs(g_a[0, -1, -1]) > 0.0


def test_uniform_prior_is_minus_infinity_outside_its_bounds():
    grid, geom, vels, dobs, sigma = _problem()
    lo, hi = np.full((13, 17), 1500.0), np.full((13, 17), 3300.0)
    inside = np.clip(vels, lo, hi)
    outside = inside.copy()
    outside[1, 4, 7] = 3300.5
    lp_in, _ = fwi.grad_logpost(inside, grid, geom, dobs, sigma, lo, hi)
    lp_out, g_out = fwi.grad_logpost(outside, grid, geom, dobs, sigma, lo, hi)
    assert np.all(np.isfinite(lp_in))
    assert lp_out[1] == -np.inf and np.isfinite(lp_out[0]) and np.isfinite(lp_out[2])
    # the prior adds no gradient (the clip strategy keeps particles inside)
    assert np.all(np.isfinite(g_out))
