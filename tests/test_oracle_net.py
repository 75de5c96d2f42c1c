"""Pins of the oracle's gauge-covariant network (learned preconditioner)."""
import numpy as np
import pytest

from oracle import lattice as LT
from oracle import net as ON
from paper_2402_00016_amd import inputs


@pytest.fixture(scope="module")
def setup():
    dims = (2, 2, 2, 4)
    U = inputs.gauge_links(dims, 0.5, seed=5)
    return dims, U, ON.Transport(dims, U)


def _rv(rng, shape):
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


def test_sizes():
    assert ON.n_params() == 2304
    assert [s for s in ON.layer_shapes()] == [(9, 8, 4), (9, 8, 8), (9, 4, 8)]


def test_identity_weights(setup):
    dims, U, T = setup
    rng = np.random.default_rng(0)
    X = _rv(rng, (3, 12 * LT.volume(dims)))
    assert np.allclose(ON.apply_net(T, ON.identity_theta(), X), X)


def test_linear_and_gauge_covariant(setup):
    dims, U, T = setup
    rng = np.random.default_rng(1)
    th = rng.standard_normal(ON.n_params()) * 0.3
    n = 12 * LT.volume(dims)
    X, Y = _rv(rng, (1, n)), _rv(rng, (1, n))
    a, b = 0.7 - 0.2j, -1.3j
    assert np.allclose(ON.apply_net(T, th, a * X + b * Y), a * ON.apply_net(T, th, X) + b * ON.apply_net(T, th, Y))
    g = inputs.random_gauge_transform(dims, seed=3)
    Tg = ON.Transport(dims, LT.gauge_rotate(U, g, dims))
    lhs = ON.apply_net(Tg, th, LT.colour_rotate(X, g))
    rhs = LT.colour_rotate(ON.apply_net(T, th, X), g)
    assert np.allclose(lhs, rhs, atol=1e-12)


def test_transport_adjoint(setup):
    dims, U, T = setup
    rng = np.random.default_rng(2)
    V = LT.volume(dims)
    a, g = _rv(rng, (2, V, 2, 4, 3)), _rv(rng, (2, V, 2, 4, 3))
    for p in range(9):
        assert abs(np.vdot(g, T.apply(a, p)) - np.vdot(T.adjoint(g, p), a)) < 1e-11


def test_gradient_matches_finite_differences(setup):
    dims, U, T = setup
    rng = np.random.default_rng(3)
    th = rng.standard_normal(ON.n_params()) * 0.2
    n = 12 * LT.volume(dims)
    R, E = _rv(rng, (2, n)), _rv(rng, (2, n))
    L0, g = ON.loss_and_grad(T, th, R, E)
    h = 1e-6
    for idx in rng.choice(ON.n_params(), 40, replace=False):
        tp, tm = th.copy(), th.copy()
        tp[idx] += h
        tm[idx] -= h
        fd = (ON.loss_and_grad(T, tp, R, E)[0] - ON.loss_and_grad(T, tm, R, E)[0]) / (2 * h)
        assert abs(fd - g[idx]) < 1e-6 * max(1.0, abs(fd))


def test_loss_special_cases(setup):
    dims, U, T = setup
    rng = np.random.default_rng(4)
    R = _rv(rng, (3, 12 * LT.volume(dims)))
    assert ON.loss_and_grad(T, ON.identity_theta(), R, R)[0] < 1e-28
    assert abs(ON.loss_and_grad(T, np.zeros(ON.n_params()), R, 2 * R)[0] - 1.0) < 1e-14
    # identity weights against targets 2r: loss = 1/4 for every pair
    assert abs(ON.loss_and_grad(T, ON.identity_theta(), R, 2 * R)[0] - 0.25) < 1e-14
