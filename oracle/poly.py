"""Oracle: GMRES polynomials p(M), pi(M) and the double polynomial
(test infrastructure only).

Sec. 3: pi(M) = prod_i (1 - M/theta_i) over the Leja-ordered harmonic Ritz
values, and p(M) of degree d-1 is defined by pi(M) = 1 - M p(M).  The expansion
printed in Sec. 3 carries a leading M in u_k that makes sum_k u_k = 1 - pi(M)
(degree d, contradicting the stated degree d-1).  Reading used here, which
satisfies pi = 1 - M p exactly:

    p(M) = sum_{k=1}^{d} (1/theta_k) prod_{i<k} (1 - M/theta_i),

evaluated by the recurrence w_1 = x, y = sum_k w_k/theta_k,
w_{k+1} = w_k - M w_k/theta_k (d-1 operator applications).

Sec. 5: the double polynomial.  p_in comes from GMRES on M, p_out from GMRES
on phi_in(M) = M p_in(M); p_double(M) = p_in(M) p_out(phi_in(M)), of degree
(d_in)(d_out) - 1 when p_in, p_out come from GMRES(d_in), GMRES(d_out).

Deflated double polynomial (Sec. 7 and the conclusions name it; the
mechanism is deferred to a reference).  Reading: p_in as above (GMRES on M,
not deflated); the outer cycle is GMRES on Q phi_in(M) started from Q b,
Q = I - Z U^H the oblique projector of the deflation set, so every Arnoldi
vector lies in the range of Q and p_out fits phi_in only on the spectrum that
deflation leaves.  p_double(M) = p_in(M) p_out(phi_in(M)) is applied as before
(it is a polynomial of M; the deflated eigen-components are handled by the
deflation of the Monte Carlo levels).

Pins (tests/test_oracle_krylov.py): pi(M) = 1 - M p(M) on random vectors to
1e-12 (two different formulas); pi(M) b equals the GMRES residual; scalar
p(lambda) equals the vector action on free-field plane waves; the double
polynomial's outer residual identity and its matvec count.  Deflated double
polynomial: pi_out(Q phi_in) Q b equals the least-squares residual on an
explicit monomial basis of the projected Krylov space, and with exact
eigenvectors also pi_out(phi_in) Q b; every Arnoldi vector is annihilated by
U^H; with exact eigenvectors deflated, no harmonic Ritz value of the outer
cycle comes near phi_in(lambda_i) of a deflated eigenvalue, which the
undeflated cycle does resolve.
"""
import numpy as np

from .krylov import GmresPoly, gmres_poly


def apply_p(op, roots, x):
    """y = p(M) x by the Leja-product expansion (see module docstring)."""
    roots = np.asarray(roots)
    w = np.array(x, dtype=np.complex128, copy=True)
    y = w / roots[0]
    for k in range(len(roots) - 1):
        w = w - op(w) / roots[k]
        y = y + w / roots[k + 1]
    return y


def apply_pi(op, roots, x):
    """pi(M) x = prod_i (1 - M/theta_i) x (product form, Sec. 3)."""
    w = np.array(x, dtype=np.complex128, copy=True)
    for th in roots:
        w = w - op(w) / th
    return w


def eval_p(roots, lam):
    """Scalar p(lambda) for an array of lambda."""
    lam = np.asarray(lam, dtype=np.complex128)
    w = np.ones_like(lam)
    y = w / roots[0]
    for k in range(len(roots) - 1):
        w = w * (1 - lam / roots[k])
        y = y + w / roots[k + 1]
    return y


def phi(op, inner_roots):
    """Operator phi_in(M) = M p_in(M)."""
    return lambda v: op(apply_p(op, inner_roots, v))


def apply_poly(op, P, x):
    """y = P(M) x for a single (P.inner is None) or double GmresPoly."""
    if P.inner is None:
        return apply_p(op, P.roots, x)
    u = apply_p(phi(op, P.inner.roots), P.roots, x)
    return apply_p(op, P.inner.roots, u)


def eval_poly(P, lam):
    """Scalar P(lambda) for single or double polynomials."""
    if P.inner is None:
        return eval_p(P.roots, lam)
    pin = eval_p(P.inner.roots, lam)
    return pin * eval_p(P.roots, np.asarray(lam) * pin)


def projector(Z, U):
    """Q x = x - sum_i z_i (u_i^H x): the oblique projector of a deflation set
    (Z, U of shape (k, n)), on vectors of shape (n,) or (N, n)."""
    Z = np.asarray(Z, dtype=np.complex128)
    U = np.asarray(U, dtype=np.complex128)

    def Q(x):
        x = np.asarray(x, dtype=np.complex128)
        c = x @ U.conj().T                  # (..., k): u_i^H x
        return x - c @ Z
    return Q


def double_poly(op, b, d_in, d_out, proj=None):
    """GMRES(d_in) on M, then GMRES(d_out) on phi_in(M) from the same b; with
    proj (the deflation projector Q) the outer cycle is the deflated one, on
    Q phi_in(M) from Q b."""
    P_in, din_eff, res_in = gmres_poly(op, b, d_in)
    P_out, dout_eff, res_out = gmres_poly(phi(op, P_in.roots), b, d_out, proj=proj)
    return GmresPoly(P_out.roots, inner=P_in), (din_eff, dout_eff), (res_in, res_out)


def matvec_count(P):
    """Operator applications in one P(M) x: d-1 single, d_in*d_out - 1 double."""
    if P.inner is None:
        return P.d - 1
    return (P.d - 1) * P.inner.d + (P.inner.d - 1)
