"""Oracle: main solves M x = b (test infrastructure only).

Sec. 1: each Hutchinson sample needs a solve M x_i = eta_i, the main expense.
Sec. 8 uses deflated, polynomial-preconditioned GMRES; its details are
deferred to the paper's references.  Reading used here: restarted GMRES(m) in
FP64 with the deflated initial guess x0 = Z Lambda^-1 U^H b and the same
projection x += Z Lambda^-1 U^H r applied at each restart, iterated until the
TRUE relative residual ||b - M x|| / ||b|| <= tol.  Any correct solver is an
oracle for x = M^-1 b; the pins check the true residual with the oracle's own
operator and compare against a dense LU solve on 4^4.
"""
import numpy as np

from .krylov import arnoldi, gmres_residual


def defl_guess(D, r):
    if D is None or D.k == 0:
        return np.zeros_like(r)
    c = (D.U.conj() @ r) / D.lam
    return D.Z.T @ c


def gmres_solve(op, b, m=50, tol=1e-10, D=None, max_restarts=400):
    """Deflated restarted GMRES(m) for one right-hand side."""
    b = np.asarray(b, dtype=np.complex128)
    bn = np.linalg.norm(b)
    x = defl_guess(D, b)
    its = 0
    for _ in range(max_restarts):
        r = b - op(x)
        if np.linalg.norm(r) <= tol * bn:
            return x, its, np.linalg.norm(r) / bn
        if D is not None and D.k:
            x = x + defl_guess(D, r)
            r = b - op(x)
        V, H, beta, d_eff = arnoldi(op, r, m)
        y, _ = gmres_residual(H, beta)
        x = x + V[:d_eff].T @ y
        its += d_eff
    r = b - op(x)
    return x, its, np.linalg.norm(r) / bn


def solve_many(op, B, **kw):
    X = np.empty_like(B)
    info = []
    for i in range(B.shape[0]):
        X[i], its, rr = gmres_solve(op, B[i], **kw)
        info.append((its, rr))
    return X, info


def dense_solve(M, B):
    """x = M^-1 b by dense LU, B shape (N, n)."""
    return np.linalg.solve(M, np.asarray(B).T).T
