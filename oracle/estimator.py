"""Oracle: level estimators and the multipolynomial combination
(test infrastructure only).

* Hutchinson (Sec. 1):        X = eta^H Theta M^-1 eta.
* Subtracted (Sec. 2 eq. 2):  X = eta^H Theta (M^-1 - p(M)) eta, plus the
                              correction Tr(Theta p(M)).
* Multipolynomial (Sec. 6):   Tr(Theta M^-1) = Tr(Theta(M^-1 - p_1))
                              + sum_l Tr(Theta(p_l - p_{l+1})) + Tr(Theta p_K),
                              each term its own Monte Carlo with independent
                              noise (independent streams).
* Deflated levels (Sec. 7):   on polynomial-difference levels subtract
                              sum_i c_i (eta^H Theta z_i)(u_i^H eta),
                              c_i = p_l(lambda_i) - p_{l+1}(lambda_i), and add
                              back T_l = sum_i c_i u_i^H Theta z_i.
* Deflated solve level:       when p_1 is the deflated double polynomial it
                              does not approximate 1/lambda on the deflated
                              eigenvalues, so the first level M^-1 - p_1 is
                              deflated the same way with c_i = 1/lambda_i -
                              p_1(lambda_i) (Sec. 7's level formula with M^-1
                              in place of the upper polynomial; exact for any
                              eigen-triples, like every deflated level).

Reading of the error bookkeeping (Sec. 8 only gives the total tolerance):
samples are complex; a level's variance is s^2 = sum |X - mean|^2 / (N-1);
the total standard error is sqrt(sum_l s_l^2 / N_l).

Pins (tests/test_oracle_estimator.py): exact traces by dense inversion on
4^4; the exact Z(4) variance ||A||_F^2 - sum |A_jj|^2 against the empirical
variance; the deflated level's expectation equals the undeflated one; with a
shared noise vector the level samples telescope to eta^H Theta M^-1 eta.
"""
import numpy as np

from . import philox
from .deflation import deflated_term, exact_correction
from .lattice import spin_op, theta_matrix
from .poly import apply_poly, eval_poly
from .solve import gmres_solve


def noise_batch(seed, stream, first, N, n):
    return philox.z4_noise_batch(seed, stream, first, N, n)


def quad(eta, theta_spin, y):
    """eta^H Theta y per row."""
    return np.einsum("rn,rn->r", eta.conj(), spin_op(y, theta_spin))


def level_samples(op, upper, lower, D, theta, seed, stream, first, N,
                  solve_tol=1e-10, solve_m=50, eta=None, X_solved=None, deflate_solve=False):
    """Samples of one level and its exact correction T.

    upper: GmresPoly or None (None = M^-1 via a solve); lower: GmresPoly or
    None (None = 0).  Deflation is applied when both are polynomials, and on
    the solve level (upper None, lower a polynomial) when deflate_solve.
    """
    S = theta_matrix(theta)
    if eta is None:
        eta = noise_batch(seed, stream, first, N, op.n)
    if upper is None:
        if X_solved is None:
            X_solved = np.stack([gmres_solve(op, e, m=solve_m, tol=solve_tol)[0] for e in eta])
        up = quad(eta, S, X_solved)
    else:
        up = quad(eta, S, np.stack([apply_poly(op, upper, e) for e in eta]))
    lo = 0 if lower is None else quad(eta, S, np.stack([apply_poly(op, lower, e) for e in eta]))
    X = up - lo
    T = 0j
    if upper is not None and lower is not None and D is not None and D.k:
        c = eval_poly(upper, D.lam) - eval_poly(lower, D.lam)
        X = X - deflated_term(D, c, eta, S)
        T = exact_correction(D, c, S)
    elif deflate_solve and upper is None and lower is not None and D is not None and D.k:
        c = 1.0 / D.lam - eval_poly(lower, D.lam)
        X = X - deflated_term(D, c, eta, S)
        T = exact_correction(D, c, S)
    return X, T


def level_stats(X):
    X = np.asarray(X)
    N = len(X)
    mean = X.mean()
    var = np.sum(np.abs(X - mean) ** 2) / (N - 1) if N > 1 else np.inf
    return mean, var


def combine(levels):
    """levels: list of (samples, T). Returns (estimate, std error)."""
    est = 0j
    var = 0.0
    for X, T in levels:
        m, v = level_stats(X)
        est += m + T
        var += v / len(X)
    return est, float(np.sqrt(var))


def exact_z4_variance(A):
    """E|eta^H A eta - Tr A|^2 for Z(4) noise: ||A||_F^2 - sum |A_jj|^2."""
    return float(np.sum(np.abs(A) ** 2) - np.sum(np.abs(np.diag(A)) ** 2))
