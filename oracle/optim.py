"""FP64 oracle: step rules for gradient ascent named in section 2.2 (SGD,
AdaGrad, AdaDelta, Adam), written from their published definitions (Duchi et
al. 2011; Zeiler 2012; Kingma and Ba 2014) for an ascent direction g; used as
the SVGD update x <- x + step(phi).

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

state: dict of per-coordinate arrays (created zero on first use) and the
1-based step count t.
"""
from __future__ import annotations

import numpy as np

SGD, ADAGRAD, ADADELTA, ADAM = range(4)


def step(kind, g, state, eps, beta1=0.9, beta2=0.999, delta=1e-8):
    """Return the increment for ascent direction g and update `state`."""
    g = np.asarray(g, dtype=np.float64)
    state["t"] = state.get("t", 0) + 1
    if kind == SGD:
        return eps * g
    if kind == ADAGRAD:
        G = state.get("s1", np.zeros_like(g)) + g * g
        state["s1"] = G
        return eps * g / (np.sqrt(G) + delta)
    if kind == ADADELTA:
        rho = beta1
        Eg = rho * state.get("s1", np.zeros_like(g)) + (1.0 - rho) * g * g
        Ed = state.get("s2", np.zeros_like(g))
        u = np.sqrt(Ed + delta) / np.sqrt(Eg + delta) * g
        state["s1"] = Eg
        state["s2"] = rho * Ed + (1.0 - rho) * u * u
        return eps * u
    if kind == ADAM:
        t = state["t"]
        m = beta1 * state.get("s1", np.zeros_like(g)) + (1.0 - beta1) * g
        v = beta2 * state.get("s2", np.zeros_like(g)) + (1.0 - beta2) * g * g
        state["s1"], state["s2"] = m, v
        mh = m / (1.0 - beta1 ** t)
        vh = v / (1.0 - beta2 ** t)
        return eps * mh / (np.sqrt(vh) + delta)
    raise ValueError(kind)
