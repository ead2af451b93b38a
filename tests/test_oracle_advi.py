"""Pins of the ADVI oracle (section 2.2, eq:gradient_mu, eq:gradient_L; the
mean-field family of section 5) against closed forms for Gaussian targets,
finite differences of the Monte Carlo ELBO, a library entropy and the known
optima of both families."""
import numpy as np
from scipy import stats

from oracle import advi, optim


def _spd(r, d):
    B = r.standard_normal((d, d))
    return B @ B.T / d + 0.5 * np.eye(d)


def _symmetric_normals(d):
    """2d points +-sqrt(d) e_k: mean 0 and second moment I exactly, so the
    Monte Carlo averages of a gradient that is affine in theta are exact."""
    E = np.sqrt(d) * np.eye(d)
    return np.vstack([E, -E])


def test_gradients_match_the_gaussian_closed_form():
    """For log p = -1/2 (theta - m)^T A (theta - m):
    E[g] = -A (mu - m) and E[g eta^T] = -A L, so the exact gradients are
    -A (mu - m) and the lower part of -A L + L^-T, whose lower part is
    -tril(A L) + diag(1 / L_ii)."""
    r = np.random.default_rng(11)
    d = 6
    A, m = _spd(r, d), r.standard_normal(d)
    mu = r.standard_normal(d)
    L = np.tril(r.standard_normal((d, d))) + 2.0 * np.eye(d)
    eta = _symmetric_normals(d)
    th = advi.sample(mu, L, eta)
    g = -(th - m) @ A.T
    gm, gL = advi.gradients(L, eta, g)
    assert np.allclose(gm, -A @ (mu - m), rtol=1e-12, atol=1e-12)
    ref = -np.tril(A @ L) + np.diag(1.0 / np.diag(L))
    assert np.allclose(gL, ref, rtol=1e-12, atol=1e-12)
    # mean field: L = diag(l), the gradient of l is the diagonal of the above
    l = 1.0 + r.uniform(0.0, 1.0, d)
    th = advi.sample(mu, l, eta, advi.MEAN_FIELD)
    g = -(th - m) @ A.T
    gm, gl = advi.gradients(l, eta, g, advi.MEAN_FIELD)
    assert np.allclose(gm, -A @ (mu - m), rtol=1e-12, atol=1e-12)
    assert np.allclose(gl, -np.diag(A) * l + 1.0 / l, rtol=1e-12, atol=1e-12)


def test_elbo_matches_the_gaussian_closed_form_and_scipy_entropy():
    r = np.random.default_rng(12)
    d = 5
    A, m = _spd(r, d), r.standard_normal(d)
    mu = r.standard_normal(d)
    L = np.tril(r.standard_normal((d, d))) + 2.0 * np.eye(d)
    L[2, 2] = -L[2, 2]      # the entropy takes |det L|
    cov = L @ L.T
    assert abs(advi.entropy(L) - stats.multivariate_normal(mu, cov).entropy()) <= 1e-12
    eta = _symmetric_normals(d)
    th = advi.sample(mu, L, eta)
    lp = -0.5 * np.einsum("si,ij,sj->s", th - m, A, th - m)
    exact = -0.5 * ((mu - m) @ A @ (mu - m) + np.trace(A @ cov))
    assert abs(advi.elbo(lp, L) - (exact + stats.multivariate_normal(mu, cov).entropy())) <= 1e-10
    l = r.uniform(0.5, 2.0, d)
    assert abs(advi.entropy(l, advi.MEAN_FIELD) -
               stats.multivariate_normal(mu, np.diag(l * l)).entropy()) <= 1e-12


def _logcosh_target(r, d):
    B = r.standard_normal((d + 2, d))
    c = r.standard_normal(d + 2)

    def f(th):
        th = np.atleast_2d(th)
        z = th @ B.T - c
        lp = -np.sum(np.log(np.cosh(z)), axis=1)
        g = -np.tanh(z) @ B
        return lp, g
    return f


def test_gradients_are_the_derivatives_of_the_monte_carlo_elbo():
    """With eta held fixed the estimates are the exact gradient of the
    Monte Carlo ELBO 1/S sum_s log p(mu + L eta_s) + log|det L| (+ const):
    central differences on a non-Gaussian target, every free entry."""
    r = np.random.default_rng(13)
    d, S = 5, 3
    f = _logcosh_target(r, d)
    mu = r.standard_normal(d)
    L = np.tril(0.3 * r.standard_normal((d, d))) + np.eye(d)
    eta = r.standard_normal((S, d))

    def F(mu_, L_, fam):
        return advi.elbo(f(advi.sample(mu_, L_, eta, fam))[0], L_, fam)

    _, g = f(advi.sample(mu, L, eta))
    gm, gL = advi.gradients(L, eta, g)
    h = 1e-6
    for i in range(d):
        e = np.zeros(d)
        e[i] = h
        fd = (F(mu + e, L, advi.FULL_RANK) - F(mu - e, L, advi.FULL_RANK)) / (2 * h)
        assert abs(fd - gm[i]) <= 1e-7
        for j in range(i + 1):
            E = np.zeros((d, d))
            E[i, j] = h
            fd = (F(mu, L + E, advi.FULL_RANK) - F(mu, L - E, advi.FULL_RANK)) / (2 * h)
            assert abs(fd - gL[i, j]) <= 1e-7, (i, j, fd, gL[i, j])
    assert np.all(np.triu(gL, 1) == 0.0)
    l = r.uniform(0.5, 1.5, d)
    _, g = f(advi.sample(mu, l, eta, advi.MEAN_FIELD))
    _, gl = advi.gradients(l, eta, g, advi.MEAN_FIELD)
    for i in range(d):
        e = np.zeros(d)
        e[i] = h
        fd = (F(mu, l + e, advi.MEAN_FIELD) - F(mu, l - e, advi.MEAN_FIELD)) / (2 * h)
        assert abs(fd - gl[i]) <= 1e-7


def _gaussian(A, m):
    def f(th):
        z = np.atleast_2d(th) - m
        return -0.5 * np.einsum("si,ij,sj->s", z, A, z), -z @ A.T
    return f


def _two_phase(r, f, mu, L, family):
    """Adam with 4 samples per iteration, then a smaller step with 16 samples
    to shrink the Monte Carlo jitter around the optimum."""
    d = mu.shape[0]
    etas = [r.standard_normal((4, d)) for _ in range(3000)]
    mu, L, e1 = advi.run(f, mu, L, etas, 0.01, optim.ADAM, family)
    etas = [r.standard_normal((16, d)) for _ in range(2000)]
    mu, L, e2 = advi.run(f, mu, L, etas, 0.002, optim.ADAM, family)
    return mu, L, np.concatenate([e1, e2])


def test_full_rank_advi_reaches_the_gaussian_target():
    """The ELBO optimum for a Gaussian target N(m, A^-1) is the target itself:
    mu = m, L L^T = A^-1 (the gradient -A L + L^-T vanishes there)."""
    r = np.random.default_rng(14)
    d = 3
    A, m = _spd(r, d), r.standard_normal(d)
    mu, L, elbos = _two_phase(r, _gaussian(A, m), np.zeros(d), np.eye(d), advi.FULL_RANK)
    cov = np.linalg.inv(A)
    assert np.abs(mu - m).max() <= 0.05 * np.sqrt(np.diag(cov)).max()
    assert np.abs(L @ L.T - cov).max() <= 0.1 * np.abs(cov).max()
    assert elbos[-500:].mean() > elbos[:50].mean()


def test_mean_field_advi_reaches_the_mean_field_optimum():
    """For a correlated Gaussian target with precision A the mean-field optimum
    has the target mean and variances 1 / A_ii (Bishop 2006, section 10.1.2),
    smaller than the marginal variances."""
    r = np.random.default_rng(15)
    d = 3
    A, m = _spd(r, d), r.standard_normal(d)
    mu, l, _ = _two_phase(r, _gaussian(A, m), np.zeros(d), np.ones(d), advi.MEAN_FIELD)
    assert np.abs(mu - m).max() <= 0.05 / np.sqrt(np.diag(A)).min()
    assert np.allclose(l * l, 1.0 / np.diag(A), rtol=0.1)
    assert np.all(1.0 / np.diag(A) < np.diag(np.linalg.inv(A)) + 1e-12)


def test_sgd_step_moves_by_eps_times_the_gradient_and_keeps_l_lower():
    r = np.random.default_rng(16)
    d, S = 4, 2
    mu = r.standard_normal(d)
    L = np.tril(r.standard_normal((d, d))) + 3.0 * np.eye(d)
    eta, g = r.standard_normal((S, d)), r.standard_normal((S, d))
    mu2, L2, gm, gL = advi.step(mu, L, eta, g, 0.25)
    assert np.allclose(mu2, mu + 0.25 * g.mean(axis=0), rtol=1e-14)
    assert np.allclose(L2 - L, 0.25 * gL, rtol=1e-12, atol=1e-14)
    assert np.all(np.triu(L2, 1) == 0.0)


def test_inverse_term_keeps_its_structural_zeros_for_ill_conditioned_factors():
    """The lower part of (L^-1)^T is diag(1 / L_ii) however badly L is
    conditioned (a random triangular factor of this size has entries of L^-1
    near 1e13)."""
    r = np.random.default_rng(18)
    d = 400
    L = np.tril(r.normal(0.0, 0.3, (d, d)), -1) + np.diag(r.uniform(0.5, 2.0, d))
    zero = np.zeros((1, d))
    _, gL = advi.gradients(L, zero, zero)
    assert np.array_equal(gL, np.diag(1.0 / np.diag(L)))


def test_row_functions_agree_with_the_full_matrix_functions():
    r = np.random.default_rng(19)
    d, S = 40, 3
    mu = r.standard_normal(d)
    L = np.tril(r.normal(0, 0.3, (d, d))) + np.diag(r.uniform(0.5, 2.0, d))
    eta, g = r.standard_normal((S, d)), r.standard_normal((S, d))
    rows = [0, 7, 39]
    th = advi.sample(mu, L, eta)
    assert np.allclose(advi.sample_rows(mu, L[rows], eta, rows), th[:, rows], rtol=1e-13, atol=1e-13)
    _, gL = advi.gradients(L, eta, g)
    for k, i in enumerate(rows):
        assert np.allclose(advi.gradient_rows(L[rows], eta, g, rows)[k], gL[i, : i + 1],
                           rtol=1e-12, atol=1e-12)
