"""Pins for the FP64 SVGD / sSVGD oracle: brute force on tiny ensembles,
closed forms (n = 1, n = 2), invariants, textbook routines, Gaussian targets
with a known mean and covariance, and the published Philox known answers."""
import numpy as np
import pytest

from oracle import philox
from oracle import svgd


def test_vectorised_matches_bruteforce_double_loop():
    r = np.random.default_rng(0)
    X = r.standard_normal((7, 5)) * 3.0
    G = r.standard_normal((7, 5))
    info = svgd.svgd_direction(X, G)
    phi_bf = svgd.svgd_direction_bruteforce(X, G, info["h2"])
    assert np.abs(info["phi"] - phi_bf).max() <= 1e-13 * max(1.0, np.abs(phi_bf).max())
    # D against a literal triple loop
    D = np.array([[sum((X[i, a] - X[j, a]) ** 2 for a in range(5)) for j in range(7)] for i in range(7)])
    assert np.abs(info["D"] - D).max() < 1e-12


def test_single_particle_is_gradient_ascent():
    r = np.random.default_rng(1)
    X = r.standard_normal((1, 6))
    G = r.standard_normal((1, 6))
    info = svgd.svgd_direction(X, G)
    assert info["h2"] == 1.0 and info["K"][0, 0] == 1.0
    assert np.array_equal(info["phi"], G)


def test_two_particles_closed_form():
    r = np.random.default_rng(2)
    X = r.standard_normal((2, 4)) * 5.0
    G = r.standard_normal((2, 4))
    info = svgd.svgd_direction(X, G)
    d = float(np.sum((X[0] - X[1]) ** 2))
    # median of {0, 0, d, d} = d/2, h^2 = d / (4 ln 3)  =>  k12 = exp(-2 ln 3) = 1/9
    assert abs(info["h2"] - d / (4.0 * np.log(3.0))) <= 1e-15 * info["h2"]
    assert abs(info["K"][0, 1] - 1.0 / 9.0) < 1e-15
    h2 = info["h2"]
    phi0 = 0.5 * (G[0] + G[1] / 9.0 + (X[0] - X[1]) / (9.0 * h2))
    assert np.abs(info["phi"][0] - phi0).max() < 1e-14 * np.abs(phi0).max()
    # the off-diagonal median would give k12 = 1/3
    info_off = svgd.svgd_direction(X, G, mode=svgd.BW_MEDIAN_OFFDIAG)
    assert abs(info_off["K"][0, 1] - 1.0 / 3.0) < 1e-15


def test_invariants():
    r = np.random.default_rng(3)
    n, d = 9, 6
    X = r.standard_normal((n, d))
    G = r.standard_normal((n, d))
    info = svgd.svgd_direction(X, G)
    K, s, h2 = info["K"], info["s"], info["h2"]
    rep = (s[:, None] * X - K @ X) / h2
    assert np.abs(rep.sum(axis=0)).max() < 1e-12           # repulsion sums to zero
    perm = r.permutation(n)
    info_p = svgd.svgd_direction(X[perm], G[perm])
    assert np.abs(info_p["phi"] - info["phi"][perm]).max() < 1e-12
    t = r.standard_normal(d) * 100.0
    info_t = svgd.svgd_direction(X + t, G)                   # target translated with X
    assert np.abs(info_t["phi"] - info["phi"]).max() < 1e-9
    assert np.allclose(K, K.T) and np.all(np.diag(K) == 1.0)


def test_median_against_numpy_and_bruteforce():
    r = np.random.default_rng(4)
    for m in (1, 2, 5, 16, 17, 1000):
        v = r.standard_normal(m)
        assert svgd.median_of(v) == pytest.approx(float(np.median(v)), abs=0, rel=1e-15)
    v = [3.0, 1.0, 2.0, 10.0]
    assert svgd.median_of(v) == 2.5
    assert svgd.bandwidth_sq(np.zeros((3, 3))) == 1.0      # identical particles
    D = svgd.sqdist(r.standard_normal((6, 3)))
    assert svgd.bandwidth_sq(D, svgd.BW_FIXED, 2.0) == 4.0


def test_cholesky_properties_and_jitter():
    r = np.random.default_rng(5)
    X = r.standard_normal((12, 4))
    K = svgd.rbf(svgd.sqdist(X), 1.5)
    L, retries = svgd.cholesky_jitter(K / 12.0)
    assert retries == 0
    assert np.allclose(L, np.tril(L)) and np.all(np.diag(L) > 0)
    assert np.abs(L @ L.T - K / 12.0).max() < 1e-15
    # coincident particles: K is all ones (rank one), factorisation needs jitter
    ones = np.ones((5, 5)) / 5.0
    L1, retries1 = svgd.cholesky_jitter(ones)
    assert retries1 >= 1 and np.abs(L1 @ L1.T - ones).max() < 1e-6


def test_clip_is_a_projection():
    r = np.random.default_rng(6)
    lo = np.full(10, -1.0)
    hi = np.full(10, 2.0)
    X = r.standard_normal((4, 10)) * 3.0
    C = svgd.clip(X, lo, hi)
    assert np.array_equal(svgd.clip(C, lo, hi), C)
    assert np.all(C >= lo) and np.all(C <= hi)
    inside = (X >= lo) & (X <= hi)
    assert np.array_equal(C[inside], X[inside])


MU = np.array([1.0, -2.0])
SIGMA = np.array([[2.0, 0.6], [0.6, 0.5]])
PREC = np.linalg.inv(SIGMA)


def _grad_log_gauss(X):
    return -(X - MU) @ PREC


@pytest.mark.slow
def test_svgd_converges_on_a_gaussian_target():
    r = np.random.default_rng(7)
    X = r.standard_normal((200, 2)) * 3.0
    for _ in range(5000):
        X, _ = svgd.svgd_step(X, _grad_log_gauss(X), 0.2)
    mean, _ = svgd.posterior_stats(X)
    cov = np.cov(X.T, ddof=0)
    sd = np.sqrt(np.diag(SIGMA))
    assert np.all(np.abs(mean - MU) <= 1e-3 * sd), mean
    assert np.linalg.norm(cov - SIGMA) <= 0.10 * np.linalg.norm(SIGMA), cov


@pytest.mark.slow
def test_ssvgd_samples_a_gaussian_target():
    r = np.random.default_rng(8)
    n = 20
    X = r.standard_normal((n, 2)) * 3.0
    burn, thin, iters = 5000, 10, 40000
    keep = []
    for it in range(iters):
        xi = r.standard_normal((n, 2))
        X, _ = svgd.ssvgd_step(X, _grad_log_gauss(X), 0.01, xi)
        if it in svgd.retained([it], burn, thin):
            keep.append(X.copy())
    S = np.concatenate(keep)
    mean, _ = svgd.posterior_stats(S)
    cov = np.cov(S.T, ddof=0)
    sd = np.sqrt(np.diag(SIGMA))
    assert np.all(np.abs(mean - MU) <= 0.1 * sd), mean
    assert np.linalg.norm(cov - SIGMA) <= 0.15 * np.linalg.norm(SIGMA), cov


def test_ssvgd_noise_covariance():
    # eq:noise_term: per coordinate, Cov(eta) = 2 eps Kbar / n
    r = np.random.default_rng(9)
    n, draws, eps = 6, 200000, 0.05
    K = svgd.rbf(svgd.sqdist(r.standard_normal((n, 3))), 2.0)
    xi = r.standard_normal((n, draws))
    eta, L, _ = svgd.ssvgd_noise(K, eps, xi)
    emp = eta @ eta.T / draws
    assert np.abs(emp - 2.0 * eps * K / n).max() < 0.02 * (2.0 * eps / n)


def test_retained_iterations():
    assert svgd.retained(range(30), 10, 4) == [10, 14, 18, 22, 26]


def test_philox_known_answers():
    # known-answer vectors of Philox4x32-10 published with the reference
    # implementation of Salmon et al. (SC'11)
    assert philox.philox4x32((0, 0, 0, 0), (0, 0)) == (0x6627E8D5, 0xE169C58D, 0xBC57AC4C, 0x9B00DBD8)
    assert philox.philox4x32((0xFFFFFFFF,) * 4, (0xFFFFFFFF, 0xFFFFFFFF)) == (
        0x408F276D, 0x41C83B0E, 0xA20BC7C6, 0x6D5451FD)
    assert philox.philox4x32((0x243F6A88, 0x85A308D3, 0x13198A2E, 0x03707344), (0xA4093822, 0x299F31D0)) == (
        0xD16CFE09, 0x94FDCCEB, 0x5001E420, 0x24126EA1)


def test_philox_normals_statistics():
    z = philox.normals(40000, seed=123, stream=7)
    assert abs(z.mean()) < 0.02 and abs(z.var() - 1.0) < 0.03
    from scipy import stats
    assert stats.kstest(z, "norm").pvalue > 1e-3
    assert not np.array_equal(philox.normals(16, 123, 7), philox.normals(16, 123, 8))


# ---- diagonal matrix-valued kernel ------------------------------------------

def test_diag_kernel_matches_its_double_loop_and_reduces_to_rbf():
    r = np.random.default_rng(31)
    X = r.normal(0.0, 1.0, (9, 5)) * np.array([1.0, 3.0, 0.2, 10.0, 1.0])
    G = r.standard_normal((9, 5))
    q = svgd.diag_precision(X)
    info = svgd.svgd_direction_diag(X, G, q)
    bf = svgd.svgd_direction_diag_bruteforce(X, G, q, info["h2"])
    assert np.allclose(info["phi"], bf, rtol=1e-12, atol=1e-14)
    # q = 1: the RBF kernel of eq:phi_mean
    one = svgd.svgd_direction_diag(X, G, np.ones(5))
    ref = svgd.svgd_direction(X, G)
    assert np.allclose(one["phi"], ref["phi"], rtol=1e-12, atol=1e-14)
    assert one["h2"] == ref["h2"]


def test_diag_kernel_is_rbf_svgd_in_rescaled_coordinates():
    """With y = sqrt(q) x (fixed q), the matrix-valued kernel direction is the
    RBF direction of y, mapped back: phi_x = phi_y / sqrt(q) with the
    gradient of log p in y, g / sqrt(q)."""
    r = np.random.default_rng(32)
    X = r.normal(0.0, 1.0, (12, 4)) * np.array([0.5, 2.0, 40.0, 1.0])
    G = r.standard_normal((12, 4))
    q = svgd.diag_precision(X)
    sq = np.sqrt(q)
    phi_x = svgd.svgd_direction_diag(X, G, q)["phi"]
    phi_y = svgd.svgd_direction(X * sq, G / sq)["phi"]
    assert np.allclose(phi_x, phi_y / sq, rtol=1e-10, atol=1e-13)


def test_diag_precision_and_zero_variance():
    X = np.array([[1.0, 5.0, 2.0], [3.0, 5.0, 2.0], [5.0, 5.0, 8.0]])
    q = svgd.diag_precision(X)
    assert np.allclose(q, [1.0 / np.var([1, 3, 5]), 1.0, 1.0 / np.var([2, 2, 8])])


def test_diag_kernel_svgd_on_an_anisotropic_gaussian():
    """Target N(mu, diag(s^2)) with scales 0.1 and 100: diag-kernel SVGD reaches
    the mean and the per-coordinate spread."""
    mu, sd = np.array([1.0, -50.0]), np.array([0.1, 100.0])
    r = np.random.default_rng(33)
    X = mu + r.normal(0.0, 1.0, (200, 2)) * np.array([0.5, 300.0]) + np.array([0.3, 200.0])
    for _ in range(300):
        G = -(X - mu) / sd ** 2
        X, _ = svgd.svgd_step_diag(X, G, 0.5)
    assert np.all(np.abs(X.mean(axis=0) - mu) < 0.05 * sd)
    assert np.all(np.abs(X.std(axis=0) / sd - 1.0) < 0.1)


def test_diag_kernel_ssvgd_noise_covariance():
    """eta = sqrt(2 eps) L xi / sqrt(q): covariance 2 eps (K/n) per coordinate
    scaled by 1 / q."""
    r = np.random.default_rng(34)
    X = r.normal(0.0, 1.0, (5, 3)) * np.array([1.0, 4.0, 0.5])
    G = np.zeros((5, 3))
    q = svgd.diag_precision(X)
    K = svgd.svgd_direction_diag(X, G, q)["K"]
    eps = 0.3
    draws = []
    for k in range(4000):
        xi = r.standard_normal((5, 3))
        _, info = svgd.ssvgd_step_diag(X, G, eps, xi)
        draws.append(info["eta"][:, 1])
    C = np.cov(np.array(draws).T, bias=True)
    assert np.allclose(C, 2 * eps * K / 5 / q[1], atol=0.08 * np.abs(2 * eps * K / 5 / q[1]).max())
