"""FP64 oracle: the prior strategies of section 3 beyond clipping.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

* Uniform prior, strategy 2 (eq:transform): invert in the unconstrained space
  theta = log(m - a) - log(b - m), m = a + (b - a) / (1 + exp(-theta)).  The
  density of theta is p(m(theta)) |dm/dtheta| with
  dm/dtheta = (m - a)(b - m) / (b - a), so
      log p(theta | d) = log p(m | d) + sum log((m - a)(b - m) / (b - a)),
      grad_theta       = grad_m log p(m | d) * dm/dtheta + (a + b - 2m) / (b - a).
* Gaussian prior: independent N(mean, std^2) per coordinate,
      log p(m) = -1/2 sum ((m - mean) / std)^2 (constants dropped),
      grad     = -(m - mean) / std^2.
"""
from __future__ import annotations

import numpy as np

from oracle import fwi


def to_theta(m, a, b):
    m = np.asarray(m, dtype=np.float64)
    return np.log(m - a) - np.log(b - m)


def to_model(theta, a, b):
    theta = np.asarray(theta, dtype=np.float64)
    return a + (b - a) / (1.0 + np.exp(-theta))


def dm_dtheta(theta, a, b):
    m = to_model(theta, a, b)
    return (m - a) * (b - m) / (b - a)


def log_jacobian(theta, a, b):
    """sum over coordinates of log|dm/dtheta|."""
    return float(np.sum(np.log(dm_dtheta(theta, a, b))))


def grad_log_jacobian(theta, a, b):
    m = to_model(theta, a, b)
    return (a + b - 2.0 * m) / (b - a)


def transformed_grad_logpost(thetas, grid, geom, dobs, sigma, a, b):
    """log p(theta | d) and its theta-gradient for every particle (rows of
    thetas shaped like the model), the misfit from oracle.fwi."""
    thetas = np.asarray(thetas, dtype=np.float64)
    logpost = np.zeros(thetas.shape[0])
    grad = np.zeros_like(thetas)
    for p in range(thetas.shape[0]):
        m = to_model(thetas[p], a, b)
        J, dJ = fwi.data_gradient(m, grid, geom, dobs, sigma)
        logpost[p] = -J + log_jacobian(thetas[p], a, b)
        grad[p] = -dJ * dm_dtheta(thetas[p], a, b) + grad_log_jacobian(thetas[p], a, b)
    return logpost, grad


def gaussian_log_prior(m, mean, std):
    z = (np.asarray(m, dtype=np.float64) - mean) / std
    return -0.5 * float(np.sum(z * z)), -(np.asarray(m, dtype=np.float64) - mean) / std ** 2


def gaussian_grad_logpost(vels, grid, geom, dobs, sigma, mean, std):
    vels = np.asarray(vels, dtype=np.float64)
    logpost = np.zeros(vels.shape[0])
    grad = np.zeros_like(vels)
    for p in range(vels.shape[0]):
        J, dJ = fwi.data_gradient(vels[p], grid, geom, dobs, sigma)
        lp, glp = gaussian_log_prior(vels[p], mean, std)
        logpost[p] = -J + lp
        grad[p] = -dJ + glp
    return logpost, grad
