"""FP64 oracle: RBF kernel, median bandwidth, SVGD and sSVGD particle updates,
uniform-prior clipping and posterior statistics.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Paper basis (VIP, section 2.3-2.4):
  * eq:rbf          k(m, m') = exp(-|m - m'|^2 / (2 h^2)), h a scale factor;
  * eq:phi_mean     phi(m) = 1/n sum_j [k(m_j, m) grad log p(m_j) + grad_{m_j} k(m_j, m)],
                    m_i <- m_i + eps phi(m_i);
  * eq:stochastic_svgd, eq:matrixK, eq:matrixDK, eq:noise_term
                    z <- z + eps [K grad log p + div K] + N(0, 2 eps K), the noise
                    drawn as sqrt(2 eps) P^T L_{D_K} N(0, I), L from the Cholesky
                    factor of the n x n kernel matrix (D_K carries a 1/n);
  * section 3       uniform prior, strategy 1: reset values outside the bounds
                    to the nearest bound;
  * section 4       posterior mean / std over final particles (SVGD) or over
                    retained post-burn-in samples (sSVGD).

  * section 5        diagonal matrix-valued kernel: a positive definite diagonal
                    Q combined with the RBF, Q = inverse per-coordinate variance
                    across particles; read as K(m, m') = Q^-1 k_Q(m, m') with
                    k_Q = exp(-(m - m')^T Q (m - m') / (2 h^2)), whose SVGD
                    direction is 1/n sum_j k_Q(m_j, m_i) [Q^-1 grad log p(m_j)
                    + (m_i - m_j) / h^2] (the divergence of Q^-1 k_Q brings
                    Q^-1 Q = I), and whose sSVGD noise is sqrt(2 eps) L Xi Q^-1/2.

Readings where the paper is silent:
  * bandwidth: median heuristic over all n^2 squared distances (the n zero
    self-distances included; even count -> mean of the two middle values),
    h^2 = med / (2 ln(n + 1)); h^2 = 1 when med = 0;
  * the j = i term of eq:phi_mean is kept (k_ii = 1, its gradient is 0);
  * Cholesky failure: add jitter 1e-12 * trace(A)/n, times 10 per retry, at
    most 6 retries;
  * std uses ddof = 0;
  * Q of the matrix-valued kernel: q_a = 1 / var_a over the current particles
    (ddof = 0), q_a = 1 where var_a = 0; recomputed at every step.
"""
from __future__ import annotations

import numpy as np

BW_MEDIAN_ALL = 0
BW_MEDIAN_OFFDIAG = 1
BW_FIXED = 2


def sqdist(X: np.ndarray) -> np.ndarray:
    """D_ij = sum_a (x_ia - x_ja)^2, evaluated directly (no Gram identity)."""
    X = np.asarray(X, dtype=np.float64)
    n = X.shape[0]
    if n * n * X.shape[1] <= 4_000_000:
        diff = X[:, None, :] - X[None, :, :]
        return np.sum(diff * diff, axis=2)
    D = np.empty((n, n))
    for i in range(n):
        diff = X - X[i]
        D[i] = np.einsum("ja,ja->j", diff, diff)
    return D


def median_of(values: np.ndarray) -> float:
    """Median by sorting: middle value, or mean of the two middle values."""
    v = np.sort(np.asarray(values, dtype=np.float64), axis=None)
    m = v.size
    if m % 2 == 1:
        return float(v[m // 2])
    return 0.5 * (float(v[m // 2 - 1]) + float(v[m // 2]))


def bandwidth_sq(D: np.ndarray, mode: int = BW_MEDIAN_ALL, h_fixed: float = 1.0) -> float:
    n = D.shape[0]
    if mode == BW_FIXED:
        return float(h_fixed) ** 2
    if mode == BW_MEDIAN_ALL:
        med = median_of(D)
    elif mode == BW_MEDIAN_OFFDIAG:
        iu = np.triu_indices(n, 1)
        med = median_of(D[iu]) if n > 1 else 0.0
    else:
        raise ValueError(mode)
    if med == 0.0:
        return 1.0
    return med / (2.0 * np.log(n + 1.0))


def rbf(D: np.ndarray, h2: float) -> np.ndarray:
    """eq:rbf on precomputed squared distances."""
    return np.exp(-D / (2.0 * h2))


def diag_precision(X):
    """q_a = 1 / var_a across the particles (ddof = 0); 1 where var_a = 0."""
    X = np.asarray(X, dtype=np.float64)
    var = X.var(axis=0, ddof=0)
    return np.where(var > 0.0, 1.0 / np.where(var > 0.0, var, 1.0), 1.0)


def sqdist_q(X, q):
    """D_ij = sum_a q_a (x_ia - x_ja)^2, evaluated directly."""
    X = np.asarray(X, dtype=np.float64)
    n = X.shape[0]
    D = np.empty((n, n))
    for i in range(n):
        diff = X - X[i]
        D[i] = (diff * diff) @ q
    return D


def svgd_direction_diag(X, G, q, mode=BW_MEDIAN_ALL, h_fixed=1.0):
    """Diagonal matrix-valued kernel (see the header):
    phi_i = 1/n [ sum_j K_ij g_j / q + (s_i x_i - sum_j K_ij x_j) / h^2 ],
    K_ij = exp(-D^Q_ij / (2 h^2)).  Returns dict(D, h2, K, s, phi)."""
    X = np.asarray(X, dtype=np.float64)
    G = np.asarray(G, dtype=np.float64)
    n = X.shape[0]
    D = sqdist_q(X, q)
    h2 = bandwidth_sq(D, mode, h_fixed)
    K = rbf(D, h2)
    s = K.sum(axis=1)
    phi = (K @ (G / q) + (s[:, None] * X - K @ X) / h2) / n
    return {"D": D, "h2": h2, "K": K, "s": s, "phi": phi}


def svgd_direction_diag_bruteforce(X, G, q, h2):
    """The matrix-valued-kernel direction as a literal double loop."""
    X = np.asarray(X, dtype=np.float64)
    G = np.asarray(G, dtype=np.float64)
    n, d = X.shape
    phi = np.zeros((n, d))
    for i in range(n):
        acc = np.zeros(d)
        for j in range(n):
            diff = X[i] - X[j]
            k = np.exp(-float(diff @ (q * diff)) / (2.0 * h2))
            acc += k * (G[j] / q) + k * diff / h2
        phi[i] = acc / n
    return phi


def svgd_step_diag(X, G, eps, lo=None, hi=None, mode=BW_MEDIAN_ALL, h_fixed=1.0):
    """One SVGD iteration with the diagonal matrix-valued kernel, Q from X."""
    q = diag_precision(X)
    info = svgd_direction_diag(X, G, q, mode, h_fixed)
    info["q"] = q
    return clip(np.asarray(X, dtype=np.float64) + eps * info["phi"], lo, hi), info


def ssvgd_step_diag(X, G, eps, xi, lo=None, hi=None, mode=BW_MEDIAN_ALL, h_fixed=1.0):
    """sSVGD with the diagonal matrix-valued kernel: noise sqrt(2 eps) L Xi / sqrt(q)."""
    q = diag_precision(X)
    info = svgd_direction_diag(X, G, q, mode, h_fixed)
    eta, L, retries = ssvgd_noise(info["K"], eps, xi)
    eta = eta / np.sqrt(q)
    info.update(q=q, eta=eta, L=L, retries=retries)
    return clip(np.asarray(X, dtype=np.float64) + eps * info["phi"] + eta, lo, hi), info


def svgd_direction(X, G, mode=BW_MEDIAN_ALL, h_fixed=1.0, D=None):
    """phi_i = 1/n [ sum_j K_ij G_j + (s_i x_i - sum_j K_ij x_j) / h^2 ],
    s_i = sum_j K_ij; the second term is sum_j grad_{m_j} k(m_j, m_i) with
    grad_{m_j} k(m_j, m_i) = K_ij (m_i - m_j) / h^2.

    D may be passed in when it was computed by another direct evaluation
    (oracle.cref.sqdist for large ensembles).  Returns dict(D, h2, K, s, phi)."""
    X = np.asarray(X, dtype=np.float64)
    G = np.asarray(G, dtype=np.float64)
    n = X.shape[0]
    D = sqdist(X) if D is None else np.asarray(D, dtype=np.float64)
    h2 = bandwidth_sq(D, mode, h_fixed)
    K = rbf(D, h2)
    s = K.sum(axis=1)
    phi = (K @ G + (s[:, None] * X - K @ X) / h2) / n
    return {"D": D, "h2": h2, "K": K, "s": s, "phi": phi}


def svgd_direction_bruteforce(X, G, h2):
    """eq:phi_mean as a literal double loop (for tiny ensembles)."""
    X = np.asarray(X, dtype=np.float64)
    G = np.asarray(G, dtype=np.float64)
    n, d = X.shape
    phi = np.zeros((n, d))
    for i in range(n):
        acc = np.zeros(d)
        for j in range(n):
            diff = X[j] - X[i]
            kji = np.exp(-float(diff @ diff) / (2.0 * h2))
            grad_k = -kji * diff / h2          # d/dm_j of k(m_j, m_i)
            acc += kji * G[j] + grad_k
        phi[i] = acc / n
    return phi


def clip(X, lo, hi):
    """Uniform prior, strategy 1: values outside [lo, hi] go to the nearest bound."""
    if lo is None:
        return np.asarray(X, dtype=np.float64)
    return np.minimum(np.maximum(X, lo), hi)


def svgd_step(X, G, eps, lo=None, hi=None, mode=BW_MEDIAN_ALL, h_fixed=1.0):
    """One SVGD iteration: X' = clip(X + eps phi).  Returns (X', info)."""
    info = svgd_direction(X, G, mode, h_fixed)
    return clip(np.asarray(X, dtype=np.float64) + eps * info["phi"], lo, hi), info


def cholesky_jitter(A, max_retries=6):
    """Lower Cholesky factor of a symmetric positive (semi)definite matrix.

    Uses the library factorisation as one step; on failure adds
    delta = 1e-12 trace(A)/n to the diagonal, x10 per retry.
    Returns (L, retries) or raises numpy.linalg.LinAlgError."""
    A = np.asarray(A, dtype=np.float64)
    n = A.shape[0]
    delta = 1e-12 * np.trace(A) / n
    for r in range(max_retries + 1):
        try:
            Aj = A if r == 0 else A + delta * np.eye(n)
            return np.linalg.cholesky(Aj), r
        except np.linalg.LinAlgError:
            if r > 0:
                delta *= 10.0
    raise np.linalg.LinAlgError("not positive definite after jitter retries")


def ssvgd_noise(K, eps, xi):
    """eq:noise_term with the particle-major layout: the noise of coordinate a
    over the n particles is sqrt(2 eps) L xi[:, a], L L^T = Kbar / n."""
    n = K.shape[0]
    L, retries = cholesky_jitter(K / n)
    return np.sqrt(2.0 * eps) * (L @ np.asarray(xi, dtype=np.float64)), L, retries


def ssvgd_step(X, G, eps, xi, lo=None, hi=None, mode=BW_MEDIAN_ALL, h_fixed=1.0):
    """One sSVGD iteration (eq:stochastic_svgd): K grad log p + div K reduces
    per particle to the SVGD direction phi, plus correlated Gaussian noise.
    Returns (X', info)."""
    info = svgd_direction(X, G, mode, h_fixed)
    eta, L, retries = ssvgd_noise(info["K"], eps, xi)
    info.update(eta=eta, L=L, retries=retries)
    Xn = np.asarray(X, dtype=np.float64) + eps * info["phi"] + eta
    return clip(Xn, lo, hi), info


def posterior_stats(samples):
    """Mean and standard deviation (ddof = 0) over the sample axis 0."""
    s = np.asarray(samples, dtype=np.float64)
    return s.mean(axis=0), s.std(axis=0, ddof=0)


def retained(iterations, burn_in, thin):
    """Iterations l >= burn_in with (l - burn_in) % thin == 0 (sSVGD)."""
    return [l for l in iterations if l >= burn_in and (l - burn_in) % thin == 0]
