"""Pins of the step-rule oracle: closed forms under a constant direction, and
convergence of each rule to the maximum of a concave quadratic."""
import numpy as np
import pytest

from oracle import optim, svgd


def test_constant_direction_closed_forms():
    c = np.array([2.0, -0.5, 1e-3])
    eps, delta = 0.1, 1e-8
    st_adam, st_ada, st_dd = {}, {}, {}
    for t in range(1, 8):
        # Adam: bias-corrected moments equal c and c^2 at every step
        s = optim.step(optim.ADAM, c, st_adam, eps, 0.9, 0.999, delta)
        assert np.allclose(s, eps * c / (np.abs(c) + delta), rtol=1e-12)
        # AdaGrad: the accumulator is t c^2
        s = optim.step(optim.ADAGRAD, c, st_ada, eps, delta=delta)
        assert np.allclose(s, eps * c / (np.sqrt(t) * np.abs(c) + delta), rtol=1e-12)
    # AdaDelta, first step: sqrt(delta) / sqrt((1 - rho) c^2 + delta) c
    rho = 0.95
    s = optim.step(optim.ADADELTA, c, st_dd, 1.0, rho, delta=1e-6)
    assert np.allclose(s, np.sqrt(1e-6) / np.sqrt((1 - rho) * c * c + 1e-6) * c, rtol=1e-12)
    assert np.allclose(st_dd["s2"], (1 - rho) * s * s, rtol=1e-12)
    # SGD
    assert np.array_equal(optim.step(optim.SGD, c, {}, eps), eps * c)


@pytest.mark.parametrize("kind,eps,its", [(optim.SGD, 0.1, 300), (optim.ADAGRAD, 0.5, 2000),
                                          (optim.ADADELTA, 1.0, 4000), (optim.ADAM, 0.05, 2000)])
def test_rules_reach_the_maximum_of_a_concave_quadratic(kind, eps, its):
    target = np.array([3.0, -1.0, 0.5])
    x = np.zeros(3)
    st = {}
    beta1 = 0.95 if kind == optim.ADADELTA else 0.9
    for _ in range(its):
        x = x + optim.step(kind, -(x - target), st, eps, beta1, 0.999, 1e-6)
    assert np.allclose(x, target, atol=2e-2), (kind, x)


def test_svgd_with_adam_reaches_a_gaussian_mean():
    r = np.random.default_rng(4)
    X = r.normal(5.0, 0.5, (100, 2))
    st = {}
    for _ in range(400):
        info = svgd.svgd_direction(X, -(X - 1.0))
        X = X + optim.step(optim.ADAM, info["phi"], st, 0.05)
    assert np.allclose(X.mean(axis=0), 1.0, atol=0.05)
