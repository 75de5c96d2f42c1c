"""Oracle: eigenpairs for deflation and the deflated level term
(test infrastructure only).

Sec. 7: small eigenvalues lambda_i of M with right and left eigenvectors z_i,
u_i are found with a polynomial-preconditioned Arnoldi method (Arnoldi on
phi_in(M) = M p_in(M)); the polynomial-difference levels then sample

    Tr( Theta (p_a(M) - p_b(M)) - sum_i (p_a(lambda_i) - p_b(lambda_i)) Theta z_i u_i^H )

and add back the exact trace of the removed part, Tr(Theta z_i u_i^H) =
u_i^H Theta z_i.  Sec. 8 gives the acceptance rule: residual norms below 1e-3,
Ritz values whose imaginary part is below 2e-4 treated as real.

Readings (the paper defers details to its references):
* Ritz pairs (mu, s) of the Arnoldi matrix H_m of phi_in; candidates are the
  nev Ritz values of smallest |mu|; z = V_m s normalised; lambda = z^H M z.
* Left vectors from gamma5-hermiticity (M^H = g5 M g5): g5 z_j is a left
  eigenvector for conj(lambda_j), so u_i = g5 z_j with lambda_j closest to
  conj(lambda_i) (j = i when |Im lambda_i| < real_tol).  u_i is scaled so that
  u_i^H z_i = 1.
* Accept when ||M z - lambda z|| and ||M^H u - conj(lambda) u|| / ||u|| are both
  below accept_tol (z unit norm).
The estimator is unbiased for ANY {lambda, z, u} because the correction is
exact; quality only changes the variance.

Pins (tests/test_oracle_deflation.py): free-field eigenvalues against the
closed form a +- i|b|; 4^4 random-link eigenpairs against dense
numpy.linalg.eig; the deflated level's exact expectation equals the
undeflated trace (dense); u^H z = 1.
"""
import numpy as np

from .krylov import arnoldi
from .poly import phi
from .wilson import gamma5


class Deflation:
    def __init__(self, lam, Z, U):
        self.lam = np.asarray(lam, dtype=np.complex128)   # (k,)
        self.Z = np.asarray(Z, dtype=np.complex128)       # (k, n) right vectors
        self.U = np.asarray(U, dtype=np.complex128)       # (k, n) left vectors, u_i^H z_i = 1

    @property
    def k(self):
        return len(self.lam)


def left_vectors(op, lam, Z, real_tol):
    """Pair each eigenvalue with its conjugate partner; u_i = g5 z_j, u_i^H z_i = 1.

    Returns (U, partner index or -1)."""
    k = len(lam)
    U = np.zeros_like(Z)
    partner = np.full(k, -1)
    for i in range(k):
        if abs(lam[i].imag) < real_tol:
            j = i
        else:
            dist = np.abs(lam - np.conj(lam[i]))
            dist[i] = np.inf
            j = int(np.argmin(dist))
        u = gamma5(Z[j])
        ov = np.vdot(u, Z[i])
        if abs(ov) < 1e-300:
            continue
        U[i] = u / np.conj(ov)
        partner[i] = j
    return U, partner


def pp_arnoldi_eigs(op, inner_roots, b, m, nev, accept_tol=1e-3, real_tol=2e-4):
    """Eigenpairs of M from Arnoldi on phi_in(M) (inner_roots None -> on M itself)."""
    A = op if inner_roots is None else phi(op, inner_roots)
    V, H, beta, d_eff = arnoldi(A, b, m)
    mu, S = np.linalg.eig(H[:d_eff, :d_eff])
    idx = np.argsort(np.abs(mu), kind="stable")[:nev]
    Z = (S[:, idx].T @ V[:d_eff])
    Z /= np.linalg.norm(Z, axis=1, keepdims=True)
    MZ = op(Z)
    lam = np.einsum("kn,kn->k", Z.conj(), MZ)
    U, partner = left_vectors(op, lam, Z, real_tol)
    rres = np.linalg.norm(MZ - lam[:, None] * Z, axis=1)
    un = np.linalg.norm(U, axis=1)
    un[un == 0] = 1.0
    Uh = U / un[:, None]
    lres = np.linalg.norm(op.dagger(Uh) - np.conj(lam)[:, None] * Uh, axis=1)
    ok = (partner >= 0) & (rres < accept_tol) & (lres < accept_tol)
    order = np.argsort(np.abs(lam[ok]), kind="stable")
    sel = np.flatnonzero(ok)[order]
    return Deflation(lam[sel], Z[sel], U[sel]), dict(rres=rres, lres=lres, lam_all=lam, mu=mu[idx])


def exact_correction(D, coeff, theta_spin):
    """T = sum_i c_i u_i^H Theta z_i."""
    from .lattice import spin_op
    if D is None or D.k == 0:
        return 0j
    TZ = spin_op(D.Z, theta_spin)
    return complex(np.sum(coeff * np.einsum("kn,kn->k", D.U.conj(), TZ)))


def deflated_term(D, coeff, eta, theta_spin):
    """Per-sample sum_i c_i (eta^H Theta z_i)(u_i^H eta) for eta of shape (N, n)."""
    from .lattice import spin_op
    if D is None or D.k == 0:
        return np.zeros(eta.shape[0], dtype=np.complex128)
    TZ = spin_op(D.Z, theta_spin)            # (k, n)
    a = eta.conj() @ TZ.T                    # (N, k): eta^H Theta z_i
    b = eta @ D.U.conj().T                   # (N, k): u_i^H eta
    return (a * b) @ coeff
