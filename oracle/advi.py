"""FP64 oracle: automatic differentiation variational inference (section 2.2:
eq:prob_transforma, eq:normal, eq:argmaxELBO_advi, eq:gradient_mu,
eq:gradient_L; the mean-field variant of section 5).

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

The variational family is a Gaussian in the unconstrained space,
q(theta) = N(mu, L L^T), with L lower triangular (full rank) or diagonal
(mean field, a diagonal covariance).  One iteration with S Monte Carlo
samples eta_s ~ N(0, I) (passed in) takes
    theta_s = mu + L eta_s,
    g_s     = grad_theta log p(theta_s, d_obs)     (the bracket of
              eq:gradient_mu: the model-space gradient through dT^-1/dtheta
              plus the gradient of log|det J_T^-1|; with the transform of
              eq:transform it is what oracle.prior.transformed_grad_logpost
              returns),
    grad_mu = 1/S sum_s g_s                                  (eq:gradient_mu)
    grad_L  = 1/S sum_s g_s eta_s^T + (L^-1)^T               (eq:gradient_L)
restricted to the free entries of L: the lower triangle for the full-rank
family, the diagonal for the mean-field one (L = diag(l)).  Then both move
uphill with one of the step rules of oracle.optim, each with its own state.

The ELBO of eq:argmaxELBO_advi is estimated as
    1/S sum_s log p(theta_s, d_obs) + H[q],
    H[q] = d/2 (1 + log 2 pi) + log|det L|      (the Gaussian entropy),
up to whatever constant the caller's log p drops.
"""
from __future__ import annotations

import numpy as np
from scipy.linalg import solve_triangular

from oracle import optim

FULL_RANK, MEAN_FIELD = 0, 1


def _as_L(L, family):
    L = np.asarray(L, dtype=np.float64)
    return np.diag(L) if family == MEAN_FIELD else L


def sample(mu, L, eta, family=FULL_RANK):
    """theta[s] = mu + L eta[s] (eq:normal's reparameterisation).  L is the
    d x d lower-triangular factor, or the vector l of the mean-field family."""
    mu = np.asarray(mu, dtype=np.float64)
    eta = np.atleast_2d(np.asarray(eta, dtype=np.float64))
    Lm = np.tril(_as_L(L, family))
    return mu[None, :] + eta @ Lm.T


def gradients(L, eta, g, family=FULL_RANK):
    """(grad_mu, grad_L) of eq:gradient_mu and eq:gradient_L, the expectations
    replaced by the mean over the S samples (rows of eta and g)."""
    eta = np.atleast_2d(np.asarray(eta, dtype=np.float64))
    g = np.atleast_2d(np.asarray(g, dtype=np.float64))
    S = eta.shape[0]
    Lm = np.tril(_as_L(L, family))
    grad_mu = g.mean(axis=0)
    # L^-1 by triangular solve: it is exactly lower triangular, where a
    # general pivoted inverse leaks rounding into the structural zeros
    Linv = solve_triangular(Lm, np.eye(Lm.shape[0]), lower=True)
    full = g.T @ eta / S + Linv.T
    if family == MEAN_FIELD:
        return grad_mu, np.diag(full).copy()
    return grad_mu, np.tril(full)


def entropy(L, family=FULL_RANK):
    Lm = _as_L(L, family)
    d = Lm.shape[0]
    return 0.5 * d * (1.0 + np.log(2.0 * np.pi)) + float(np.sum(np.log(np.abs(np.diag(Lm)))))


def elbo(logp, L, family=FULL_RANK):
    """Monte Carlo ELBO estimate from the samples' log p(theta_s, d_obs)."""
    return float(np.mean(np.asarray(logp, dtype=np.float64))) + entropy(L, family)


def step(mu, L, eta, g, eps, kind=optim.SGD, state_mu=None, state_L=None,
         family=FULL_RANK, **rule):
    """One ascent step of mu and L; returns (mu, L, grad_mu, grad_L).  The
    state dicts carry each rule's per-entry memory between calls."""
    grad_mu, grad_L = gradients(L, eta, g, family)
    state_mu = {} if state_mu is None else state_mu
    state_L = {} if state_L is None else state_L
    mu = np.asarray(mu, dtype=np.float64) + optim.step(kind, grad_mu, state_mu, eps, **rule)
    L = np.asarray(L, dtype=np.float64) + optim.step(kind, grad_L, state_L, eps, **rule)
    if family == FULL_RANK:
        L = np.tril(L)
    return mu, L, grad_mu, grad_L


def run(grad_logpost, mu, L, etas, eps, kind=optim.ADAM, family=FULL_RANK, **rule):
    """Iterate ADVI with the given per-iteration normals etas[k] ([S][d] each);
    grad_logpost(thetas) -> (logp [S], g [S][d]).  Returns (mu, L, elbos)."""
    state_mu, state_L = {}, {}
    elbos = []
    for eta in etas:
        th = sample(mu, L, eta, family)
        lp, g = grad_logpost(th)
        elbos.append(elbo(lp, L, family))
        mu, L, _, _ = step(mu, L, eta, g, eps, kind, state_mu, state_L, family, **rule)
    return mu, L, np.array(elbos)


def sample_rows(mu, L_rows, eta, rows):
    """theta[s][i] for the listed coordinates only, from those rows of the
    full-rank factor (L_rows[k] = row rows[k] of L, entries past the diagonal
    ignored): the reparameterisation of eq:normal one coordinate at a time."""
    eta = np.atleast_2d(np.asarray(eta, dtype=np.float64))
    out = np.empty((eta.shape[0], len(rows)))
    for k, i in enumerate(rows):
        Li = np.asarray(L_rows[k][: i + 1], dtype=np.float64)
        out[:, k] = float(mu[i]) + eta[:, : i + 1] @ Li
    return out


def gradient_rows(L_rows, eta, g, rows):
    """Rows of grad_L (eq:gradient_L) for the listed coordinates: entry (i, j),
    j <= i, is 1/S sum_s g_s[i] eta_s[j], plus 1 / L_ii on the diagonal (the
    lower part of (L^-1)^T)."""
    eta = np.atleast_2d(np.asarray(eta, dtype=np.float64))
    g = np.atleast_2d(np.asarray(g, dtype=np.float64))
    S = eta.shape[0]
    out = []
    for k, i in enumerate(rows):
        row = g[:, i] @ eta[:, : i + 1] / S
        row[i] += 1.0 / float(L_rows[k][i])
        out.append(row)
    return out
