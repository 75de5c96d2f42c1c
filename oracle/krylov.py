"""Oracle: Arnoldi / one GMRES(d) cycle, harmonic Ritz values, Leja order
(test infrastructure only).

Sec. 3: the GMRES polynomial is built from the harmonic Ritz values of a
single GMRES(d) cycle, Leja ordered for stability.  The paper cites, but does
not define, harmonic Ritz values and Leja ordering; readings used here:

* Arnoldi with classical Gram-Schmidt applied twice (CGS2), started from the
  normalised vector b.  Breakdown (h_{j+1,j} <= 1e-14 ||H||_F) truncates the
  cycle to d_eff = j+1 steps: the Krylov space is then invariant.
* Deflated cycle (Sec. 7 names a deflated double polynomial, its mechanism is
  left to a reference): with a projector Q = I - Z U^H the start vector is Qb
  and every new vector is Q applied to the operator's output, i.e. Arnoldi on
  Q op from Qb.  The polynomial then fits the spectrum that deflation leaves.
* Harmonic Ritz values: eigenvalues of H_d + |h_{d+1,d}|^2 H_d^{-H} e_d e_d^T,
  which are the roots of the GMRES residual polynomial.
* Leja order: first the value of largest modulus, then repeatedly the value
  maximising sum_i log|theta - theta_i| over those already chosen.  Candidates
  are first sorted by (Re, Im) so that exact ties go to the earlier one; an
  exact duplicate (log = -inf) is placed last.

Pins (tests/test_oracle_krylov.py): the Arnoldi relation; pi(M) b equals the
GMRES residual obtained independently by least squares on an explicit Krylov
basis; Cayley-Hamilton on a 1^4 lattice (n = 12); breakdown at kappa = 0;
the Leja choice rule and permutation property.
"""
import numpy as np


def arnoldi(op, b, d, breakdown_rtol=1e-14, proj=None):
    """d steps of Arnoldi (CGS2) on op from b; with proj (a callable Q), on
    Q op from Q b.

    Returns (V, H, beta, d_eff): V is (d_eff+1, n) with orthonormal rows (the
    last row is zero on breakdown), H is (d_eff+1, d_eff), beta = ||b|| (of
    Q b when projected).
    """
    b = np.asarray(b, dtype=np.complex128)
    if proj is not None:
        b = proj(b)
    n = b.size
    V = np.zeros((d + 1, n), dtype=np.complex128)
    H = np.zeros((d + 1, d), dtype=np.complex128)
    beta = np.linalg.norm(b)
    V[0] = b / beta
    d_eff = d
    for j in range(d):
        w = op(V[j])
        if proj is not None:
            w = proj(w)
        Vj = V[: j + 1]
        h = Vj.conj() @ w
        w = w - Vj.T @ h
        h2 = Vj.conj() @ w
        w = w - Vj.T @ h2
        H[: j + 1, j] = h + h2
        hn = np.linalg.norm(w)
        H[j + 1, j] = hn
        if hn <= breakdown_rtol * np.linalg.norm(H[: j + 2, : j + 1]):
            H[j + 1, j] = 0.0
            d_eff = j + 1
            break
        V[j + 1] = w / hn
    return V[: d_eff + 1], H[: d_eff + 1, :d_eff], beta, d_eff


def harmonic_ritz(H):
    """Harmonic Ritz values from an Arnoldi Hessenberg H of shape (d+1, d)."""
    d = H.shape[1]
    Hd = H[:d, :d]
    h = H[d, d - 1]
    A = Hd.copy()
    if h != 0:
        ed = np.zeros(d, dtype=np.complex128)
        ed[-1] = 1.0
        f = np.linalg.solve(Hd.conj().T, ed)
        A[:, d - 1] += abs(h) ** 2 * f
    return np.linalg.eigvals(A)


def leja_order(theta):
    """Leja ordering of a finite set of complex values (see module docstring)."""
    th = np.asarray(theta, dtype=np.complex128)
    cand = th[np.lexsort((th.imag, th.real))]
    d = len(cand)
    if d == 0:
        return cand
    chosen = [int(np.argmax(np.abs(cand)))]
    taken = np.zeros(d, dtype=bool)
    taken[chosen[0]] = True
    S = np.zeros(d)
    with np.errstate(divide="ignore"):
        for _ in range(d - 1):
            S = S + np.log(np.abs(cand - cand[chosen[-1]]))
            score = np.where(taken, -np.inf, S)
            free = np.flatnonzero(~taken)
            best = free[int(np.argmax(score[free]))]
            chosen.append(int(best))
            taken[best] = True
    return cand[chosen]


def log10_pof(roots):
    """log10 of the product of other factors of each root,
    pof(k) = prod_{i != k} |1 - theta_k / theta_i|, the growth of the GMRES
    residual polynomial with theta_k removed, evaluated at theta_k."""
    th = np.asarray(roots, dtype=np.complex128)
    out = np.zeros(len(th))
    for k in range(len(th)):
        others = np.delete(th, k)
        out[k] = np.sum(np.log10(np.abs(1.0 - th[k] / others)))
    return out


def add_roots(roots, log10_threshold=4.0, digits=14.0):
    """Stabilisation of a high-degree polynomial by added roots (Embree, Loe and
    Morgan's rule for polynomial preconditioners): every root theta_k with
    log10 pof(k) > threshold gets ceil((log10 pof(k) - threshold) / digits)
    extra copies; the extended list is Leja ordered (copies go last, their
    log-distance to an equal chosen root being -inf).  Returns (roots, added)."""
    th = np.asarray(roots, dtype=np.complex128)
    lp = log10_pof(th)
    extra = []
    for k in range(len(th)):
        if lp[k] > log10_threshold:
            extra.extend([th[k]] * int(np.ceil((lp[k] - log10_threshold) / digits)))
    if not extra:
        return leja_order(th), 0
    return leja_order(np.concatenate([th, np.asarray(extra)])), len(extra)


def gmres_residual(H, beta):
    """GMRES least-squares solution y and residual norm from H (d+1, d)."""
    d = H.shape[1]
    rhs = np.zeros(H.shape[0], dtype=np.complex128)
    rhs[0] = beta
    y, *_ = np.linalg.lstsq(H, rhs, rcond=None)
    return y, np.linalg.norm(rhs - H @ y)


class GmresPoly:
    """Leja-ordered roots of one GMRES(d) cycle; degree of p is len(roots) - 1."""

    def __init__(self, roots, inner=None):
        self.roots = np.asarray(roots, dtype=np.complex128)
        self.inner = inner            # GmresPoly of p_in for a double polynomial

    @property
    def d(self):
        return len(self.roots)

    @property
    def degree(self):
        if self.inner is None:
            return self.d - 1
        return self.inner.d * self.d - 1


def gmres_poly(op, b, d, proj=None):
    """One GMRES(d) cycle on op from b -> (GmresPoly, d_eff, relative residual).
    With proj the cycle is the deflated one (on Q op from Q b; the residual is
    relative to ||Q b||)."""
    V, H, beta, d_eff = arnoldi(op, b, d, proj=proj)
    _, res = gmres_residual(H, beta)
    roots = leja_order(harmonic_ritz(H))
    return GmresPoly(roots), d_eff, res / beta
