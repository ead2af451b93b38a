"""Closed-form references used to pin the oracle (not part of the oracle).

Green's function of the 2-D scalar wave operator (1/v^2) d_tt - lap:
    G(r, t) = H(t - r/v) / (2 pi sqrt(t^2 - r^2/v^2)),
so a point source w(t) delta(x) radiates
    u(r, t) = (1/(2 pi)) int_{-inf}^{t - r/v} w(tau) / sqrt((t - tau)^2 - r^2/v^2) dtau.
With t - tau = r/v + s^2 the inverse-square-root singularity disappears:
    u(r, t) = (1/(2 pi)) int_0^{sqrt(t - r/v)} 2 w(t - r/v - s^2) / sqrt(s^2 + 2 r/v) ds
(w is taken as 0 before t = 0), evaluated here by composite Gauss-Legendre.
"""
from __future__ import annotations

import numpy as np


def ricker_closed_form(t, f0, t0):
    a = (np.pi * f0 * (t - t0)) ** 2
    return (1.0 - 2.0 * a) * np.exp(-a)


def green2d_ricker(r: float, v: float, times, f0: float, t0: float,
                   panels: int = 64, order: int = 16) -> np.ndarray:
    xg, wg = np.polynomial.legendre.leggauss(order)
    out = np.zeros(len(times))
    tau_r = r / v
    for k, t in enumerate(times):
        smax2 = t - tau_r
        if smax2 <= 0.0:
            continue
        smax = np.sqrt(smax2)
        edges = np.linspace(0.0, smax, panels + 1)
        acc = 0.0
        for a, b in zip(edges[:-1], edges[1:]):
            s = 0.5 * (b - a) * xg + 0.5 * (b + a)
            f = 2.0 * ricker_closed_form(t - tau_r - s * s, f0, t0) / np.sqrt(s * s + 2.0 * tau_r)
            acc += 0.5 * (b - a) * np.dot(wg, f)
        out[k] = acc / (2.0 * np.pi)
    return out
