"""Pins of the oracle's estimators (Sec. 1-2, Sec. 6-7) against exact traces,
the exact Z(4) variance and the telescoping identity."""
import numpy as np
import pytest

from oracle import estimator as ES
from oracle import krylov, poly
from oracle import lattice as LT
from oracle.philox import z4_noise, z4_noise_batch
from oracle.wilson import WilsonOp
from paper_2402_00016_amd import inputs


@pytest.fixture(scope="module")
def f2222():
    dims = (2, 2, 2, 2)
    U = inputs.gauge_links(dims, 0.5, seed=1)
    op = WilsonOp(dims, 0.115, U)
    M = LT.dense_wilson(dims, 0.115, U)
    return dims, op, M


def test_exact_z4_variance_matches_empirical(f2222):
    dims, op, M = f2222
    A = np.linalg.inv(M)
    eta = z4_noise_batch(3, 0, 0, 4000, op.n)
    X = np.einsum("rn,nm,rm->r", eta.conj(), A, eta)
    m, v = ES.level_stats(X)
    v_exact = ES.exact_z4_variance(A)
    assert abs(m - np.trace(A)) < 5 * np.sqrt(v_exact / len(X))
    assert abs(v / v_exact - 1) < 0.15


@pytest.mark.parametrize("theta", ["I", "g5"])
def test_hutchinson_and_subtracted_unbiased(f2222, theta):
    dims, op, M = f2222
    S = LT.theta_matrix(theta)
    G = np.kron(np.eye(LT.volume(dims)), np.kron(S, np.eye(3)))
    Minv = np.linalg.inv(M)
    exact = np.trace(G @ Minv)
    b = z4_noise(1, 0x100, 0, op.n)
    P, _, _ = krylov.gmres_poly(op, b, 8)
    Pmat = poly.apply_poly(op, P, np.eye(op.n)).T
    N = 300
    X0, T0 = ES.level_samples(op, None, None, None, theta, 5, 0, 0, N, solve_tol=1e-12)
    est, se = ES.combine([(X0, T0)])
    assert abs(est - exact) < 4 * np.sqrt(ES.exact_z4_variance(G @ Minv) / N)
    # eq. 2: subtracted level plus the exact correction Tr(Theta p(M))
    X1, _ = ES.level_samples(op, None, P, None, theta, 5, 1, 0, N, solve_tol=1e-12)
    est1, se1 = ES.combine([(X1, np.trace(G @ Pmat))])
    v1 = ES.exact_z4_variance(G @ (Minv - Pmat))
    assert abs(est1 - exact) < 4 * np.sqrt(v1 / N) + 1e-9
    assert v1 < 0.05 * ES.exact_z4_variance(G @ Minv)
    # Tr(M^-1) and Tr(g5 M^-1) are real by gamma5-hermiticity
    assert abs(exact.imag) < 1e-10


def test_telescoping_with_shared_noise(f2222):
    """With one shared eta, (M^-1 - p1) + (p1 - p2) + (p2 - p3) + p3 = M^-1."""
    dims, op, M = f2222
    b = z4_noise(1, 0x100, 0, op.n)
    P1, _, _ = krylov.gmres_poly(op, b, 17)
    P2, _, _ = krylov.gmres_poly(op, b, 9)
    P3, _, _ = krylov.gmres_poly(op, b, 3)
    eta = z4_noise_batch(11, 0, 0, 4, op.n)
    xs = np.linalg.solve(M, eta.T).T
    parts = [ES.level_samples(op, None, P1, None, "I", 0, 0, 0, 4, eta=eta, X_solved=xs)[0],
             ES.level_samples(op, P1, P2, None, "I", 0, 0, 0, 4, eta=eta)[0],
             ES.level_samples(op, P2, P3, None, "I", 0, 0, 0, 4, eta=eta)[0],
             ES.level_samples(op, P3, None, None, "I", 0, 0, 0, 4, eta=eta)[0]]
    total = np.sum(parts, axis=0)
    ref = np.einsum("rn,rn->r", eta.conj(), xs)
    assert np.allclose(total, ref, atol=1e-10 * np.max(np.abs(ref)))


def test_config_plain_4444_subtracted_vs_dense():
    """4^4, kappa=0.115, eps=0.5: GMRES(16) (degree 15), 32 Z(4) noises with and
    without subtraction, against the dense exact trace."""
    dims = (4, 4, 4, 4)
    U = inputs.gauge_links(dims, 0.5, seed=1)
    op = WilsonOp(dims, 0.115, U)
    M = LT.dense_wilson(dims, 0.115, U)
    Minv = np.linalg.inv(M)
    exact = np.trace(Minv)
    b = z4_noise(1, 0x100, 0, op.n)
    P, d_eff, _ = krylov.gmres_poly(op, b, 16)
    assert P.degree == 15
    N = 32
    eta = z4_noise_batch(1, 0, 0, N, op.n)
    xs = np.linalg.solve(M, eta.T).T
    Xns, _ = ES.level_samples(op, None, None, None, "I", 1, 0, 0, N, eta=eta, X_solved=xs)
    trP = np.trace(poly.apply_poly(op, P, np.eye(op.n)).T)
    Xs, _ = ES.level_samples(op, None, P, None, "I", 1, 0, 0, N, eta=eta, X_solved=xs)
    est_ns, se_ns = ES.combine([(Xns, 0)])
    est_s, se_s = ES.combine([(Xs, trP)])
    assert abs(est_ns - exact) < 4 * se_ns
    assert abs(est_s - exact) < 4 * se_s + 1e-9
    assert se_s < 0.05 * se_ns
