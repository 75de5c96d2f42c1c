"""Pins of the oracle's deflation (Sec. 7, Sec. 8) and main solves."""
import numpy as np
import pytest

from oracle import deflation as DF
from oracle import krylov, poly, solve
from oracle import lattice as LT
from oracle.philox import z4_noise
from oracle.wilson import WilsonOp, gamma5
from paper_2402_00016_amd import inputs


def _nearest_dist(vals, ref):
    return np.array([np.min(np.abs(ref - v)) for v in vals])


def test_free_field_eigenvalues_closed_form():
    dims = (4, 4, 4, 4)
    kappa = 0.12
    op = WilsonOp(dims, kappa, inputs.unit_links(dims))
    b = z4_noise(1, 0x200, 0, op.n)
    P_in, _, _ = krylov.gmres_poly(op, b, 5)
    D, info = DF.pp_arnoldi_eigs(op, P_in.roots, b, m=40, nev=8)
    ref = LT.free_eigenvalues(dims, kappa)
    assert D.k >= 4
    assert np.all(_nearest_dist(D.lam, ref) < 1e-8)
    # the smallest |lambda| of the closed form is found
    assert abs(np.min(np.abs(D.lam)) - np.min(np.abs(ref))) < 1e-8


@pytest.fixture(scope="module")
def small_field():
    dims = (4, 4, 2, 2)
    kappa = 0.2
    U = inputs.gauge_links(dims, 0.5, seed=21)
    op = WilsonOp(dims, kappa, U)
    M = LT.dense_wilson(dims, kappa, U)
    return dims, kappa, op, M


def test_random_links_eigenpairs_vs_dense(small_field):
    dims, kappa, op, M = small_field
    lam_ref, R = np.linalg.eig(M)
    b = z4_noise(2, 0x200, 0, op.n)
    P_in, _, _ = krylov.gmres_poly(op, b, 4)
    D, info = DF.pp_arnoldi_eigs(op, P_in.roots, b, m=120, nev=12)
    assert D.k >= 4
    assert np.all(_nearest_dist(D.lam, lam_ref) < 1e-6)
    # the smallest eigenvalue of M is found
    i0 = np.argmin(np.abs(lam_ref))
    assert np.min(np.abs(D.lam - lam_ref[i0])) < 1e-6
    for i in range(D.k):
        z, u = D.Z[i], D.U[i]
        assert abs(np.vdot(u, z) - 1) < 1e-12
        assert np.linalg.norm(M @ z - D.lam[i] * z) < 1e-3
        # u is a LEFT eigenvector: u^H M = lambda u^H
        un = u / np.linalg.norm(u)
        assert np.linalg.norm(un.conj() @ M - D.lam[i] * un.conj()) < 1e-3


def test_deflated_level_is_unbiased_exactly(small_field):
    """E[eta^H A' eta] + T = Tr(A) for the deflated A' (dense, exact), for good
    and for garbage deflation vectors alike."""
    dims, kappa, op, M = small_field
    b = z4_noise(2, 0x200, 0, op.n)
    Pa, _, _ = krylov.gmres_poly(op, b, 9)
    Pb, _, _ = krylov.gmres_poly(op, b, 3)
    n = op.n
    Ia = poly.apply_poly(op, Pa, np.eye(n)).T      # columns: Pa(M) e_j
    Ib = poly.apply_poly(op, Pb, np.eye(n)).T
    P_in, _, _ = krylov.gmres_poly(op, b, 4)
    D, _ = DF.pp_arnoldi_eigs(op, P_in.roots, b, m=120, nev=12)
    rng = np.random.default_rng(3)
    junk = DF.Deflation(rng.standard_normal(3) + 1j, rng.standard_normal((3, n)) + 0j,
                        rng.standard_normal((3, n)) + 0j)
    for theta in ("I", "g5"):
        S = LT.theta_matrix(theta)
        G = np.kron(np.eye(LT.volume(dims)), np.kron(S, np.eye(3)))
        A = G @ (Ia - Ib)
        for Dx in (D, junk):
            c = poly.eval_poly(Pa, Dx.lam) - poly.eval_poly(Pb, Dx.lam)
            A_defl = A - sum(c[i] * np.outer(G @ Dx.Z[i], Dx.U[i].conj()) for i in range(Dx.k))
            T = DF.exact_correction(Dx, c, S)
            assert abs(np.trace(A_defl) + T - np.trace(A)) < 1e-9 * max(1, abs(np.trace(A)))
            eta = np.stack([z4_noise(4, 1, j, n) for j in range(3)])
            term = DF.deflated_term(Dx, c, eta, S)
            dense_term = np.einsum("rn,nm,rm->r", eta.conj(), A - A_defl, eta)
            assert np.allclose(term, dense_term, atol=1e-9)
        # the deflated solve level: A = Theta (M^-1 - Pa(M)), c = 1/lambda - Pa(lambda)
        Minv = np.linalg.inv(M)
        A0 = G @ (Minv - Ia)
        c0 = 1.0 / D.lam - poly.eval_poly(Pa, D.lam)
        A0_defl = A0 - sum(c0[i] * np.outer(G @ D.Z[i], D.U[i].conj()) for i in range(D.k))
        T0 = DF.exact_correction(D, c0, S)
        assert abs(np.trace(A0_defl) + T0 - np.trace(A0)) < 1e-9 * max(1, abs(np.trace(A0)))
        # Whether deflation lowers the variance is an empirical property of the
        # field and the polynomials (non-normality can raise it, Sec. 7); only
        # the unbiasedness above is an identity.


def test_deflated_solve_level_samples_match_dense(small_field):
    """Per-sample values of the deflated solve level against the dense
    quadratic forms eta^H Theta (M^-1 - p(M) - sum_i c_i z_i u_i^H) eta."""
    dims, kappa, op, M = small_field
    from oracle import estimator as ES
    b = z4_noise(2, 0x200, 0, op.n)
    P, _, _ = krylov.gmres_poly(op, b, 6)
    P_in, _, _ = krylov.gmres_poly(op, b, 4)
    D, _ = DF.pp_arnoldi_eigs(op, P_in.roots, b, m=120, nev=12)
    n = op.n
    Minv = np.linalg.inv(M)
    Pm = poly.apply_poly(op, P, np.eye(n)).T
    c = 1.0 / D.lam - poly.eval_poly(P, D.lam)
    for theta in ("I", "g5"):
        S = LT.theta_matrix(theta)
        G = np.kron(np.eye(LT.volume(dims)), np.kron(S, np.eye(3)))
        A = G @ (Minv - Pm - sum(c[i] * np.outer(D.Z[i], D.U[i].conj()) for i in range(D.k)))
        X, T = ES.level_samples(op, None, P, D, theta, 5, 0, 0, 4, solve_tol=1e-12, deflate_solve=True)
        eta = ES.noise_batch(5, 0, 0, 4, n)
        ref = np.einsum("rn,nm,rm->r", eta.conj(), A, eta)
        assert np.allclose(X, ref, rtol=1e-9, atol=1e-9)
        assert abs(T - DF.exact_correction(D, c, S)) < 1e-12
        X0, T0 = ES.level_samples(op, None, P, D, theta, 5, 0, 0, 4, solve_tol=1e-12)
        assert T0 == 0 and not np.allclose(X0, X)


def test_gmres_solve_true_residual_and_dense(small_field):
    dims, kappa, op, M = small_field
    b = z4_noise(7, 0, 0, op.n)
    x, its, rr = solve.gmres_solve(op, b, m=30, tol=1e-11)
    assert rr <= 1e-11
    assert np.linalg.norm(b - M @ x) <= 1.01e-11 * np.linalg.norm(b)
    assert np.allclose(x, np.linalg.solve(M, b), atol=1e-9)
    # with deflation the same solution, no more iterations
    P_in, _, _ = krylov.gmres_poly(op, b, 4)
    D, _ = DF.pp_arnoldi_eigs(op, P_in.roots, z4_noise(2, 0x200, 0, op.n), m=120, nev=12)
    xd, itsd, rrd = solve.gmres_solve(op, b, m=30, tol=1e-11, D=D)
    assert rrd <= 1e-11 and np.allclose(xd, x, atol=1e-9)
    assert itsd <= its
