"""GPU parity at the shapes of the 8^4 three-level estimate (8^4 Wilson
lattice, kappa 0.120, links with eps 0.5 and seed 2; polynomials of degree 128,
32 and 8 from GMRES(129), GMRES(33), GMRES(9); 20 deflated eigenpairs).

The GPU builds the polynomials and the deflation set exactly as the estimate
does; their roots and eigenpairs are imported into the FP64 oracle, which then
evaluates the same quantities with its own arithmetic:

* Sec. 3: with the GPU's GMRES(129), GMRES(33) and GMRES(9) roots, pi(M) b
  under the oracle operator is the residual vector of the oracle's own cycle
  from the same b.
* Sec. 7: every imported eigenpair is an eigenpair of the oracle operator to
  the acceptance threshold, and its left vector has u_i^H z_i = 1.
* Sec. 4 and 7: every term of the estimate, per sample, on 8 noises, in FP64
  (solve term, two deflated polynomial differences, last polynomial).

Tolerances: polynomial terms 1e-10 relative (the FP64 parity bound) plus an
absolute floor of 1e-12 n for the rounding of the forms themselves; the
solve term is limited by the solver tolerance, |eta^H Theta (x - x*)| <=
||eta||^2 ||M^-1|| tol per side, with ||eta||^2 = n and ||M^-1|| <= 1/(1 - 8
kappa) = 25 (the hopping term has norm at most 8 for unitary links).
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from oracle import deflation as ODF  # noqa: E402
from oracle import estimator as OES  # noqa: E402
from oracle import krylov as OK  # noqa: E402
from oracle import poly as OP  # noqa: E402
from oracle import solve as OS  # noqa: E402
from oracle.philox import z4_noise, z4_noise_batch  # noqa: E402
from oracle.wilson import WilsonOp  # noqa: E402
from paper_2402_00016_amd import driver, inputs, mpmc  # noqa: E402

FP64 = mpmc.FP64
DIMS, KAPPA, EPS, SEED = (8, 8, 8, 8), 0.120, 0.5, 2
MINV_BOUND = 1.0 / (1.0 - 8 * KAPPA)


def rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


@pytest.fixture(scope="module")
def f84():
    U = inputs.gauge_links(DIMS, EPS, seed=SEED)
    op, ctx = WilsonOp(DIMS, KAPPA, U), mpmc.Context(DIMS, KAPPA, U)
    plan = driver.Plan(degrees=[128, 32, 8], noises=8, seed=SEED, nev=20, defl_candidates=40, defl_m=112,
                       defl_pin_degree=8)
    polys = driver.build_polys(ctx, plan)
    D = driver.build_deflation(ctx, plan)
    lam, Z, U_ = ctx.defl_vectors(D)
    torch.cuda.synchronize()
    Do = ODF.Deflation(np.asarray(lam)[:D.k], Z.cpu().numpy(), U_.cpu().numpy())
    Po = [OK.GmresPoly(P.roots) for P in polys]
    return op, ctx, plan, polys, D, Po, Do


@pytest.mark.parametrize("j", [0, 1, 2])
def test_gmres_residual_identity(f84, j):
    """pi(M) b with the GPU's roots (129, 33 and 9 of them), under the oracle
    operator, is the residual vector b - M x_d of the oracle's own GMRES(d)
    cycle from the same Z(4) vector (the defining property of the GMRES
    polynomial, Sec. 3).  Both vectors carry rounding of ~1e-15 ||b||, which
    dominates when the residual itself is that small (on this field GMRES(129)
    reaches 2e-15 and GMRES(33) 5e-11), so the bound is 1e-12 ||b|| plus
    1e-9 of the residual."""
    op, ctx, plan, polys, D, Po, Do = f84
    P = polys[j]
    d = plan.degrees[j] + 1
    assert P.d_eff == d
    b = z4_noise(SEED, 0x100 + j, 0, op.n)
    V, H, beta, d_eff = OK.arnoldi(op, b, d)
    assert d_eff == d
    y, res = OK.gmres_residual(H, beta)
    e1 = np.zeros(H.shape[0], dtype=np.complex128)
    e1[0] = beta
    r_or = V.T @ (e1 - H @ y)
    r_gpu = OP.apply_pi(op, P.roots, b)
    print("d %d: relres gpu %.6e oracle %.6e; |r_gpu - r_oracle| / |b| %.3e"
          % (d, P.relres, res / beta, np.linalg.norm(r_gpu - r_or) / beta))
    assert np.linalg.norm(r_gpu - r_or) <= 1e-12 * beta + 1e-9 * np.linalg.norm(r_or)
    assert abs(P.relres - res / beta) <= 1e-12 + 1e-8 * res / beta
    # p itself: b - M p(M) b is the same residual
    r_p = b - op(OP.apply_p(op, P.roots, b))
    assert np.linalg.norm(r_p - r_or) <= 1e-12 * beta + 1e-9 * np.linalg.norm(r_or)


def test_imported_deflation_set_is_eigenpairs(f84):
    op, ctx, plan, polys, D, Po, Do = f84
    assert Do.k >= 8
    for i in range(Do.k):
        z = Do.Z[i]
        # acceptance (Sec. 7 set-up): ||M z - lambda z|| < accept_tol for unit z
        assert np.linalg.norm(op(z) - Do.lam[i] * z) <= plan.accept_tol * np.linalg.norm(z) * 1.01
        # left vector scaled so that u_i^H z_i = 1 (the oblique projector's normalisation)
        assert abs(np.vdot(Do.U[i], z) - 1) < 1e-12


def test_every_term_per_sample_fp64(f84):
    """The four terms of the 8^4 estimate (Theta = I) per sample, FP64 on both
    sides, same Z(4) noises (seed 2, the streams of the estimate's levels)."""
    op, ctx, plan, polys, D, Po, Do = f84
    N = 8
    g = polys
    # solve term M^-1 - p_1 (deflation only as the solver's initial guess)
    eta = z4_noise_batch(SEED, 0, 0, N, op.n)
    Xs = np.stack([OS.gmres_solve(op, e, m=50, tol=1e-12, D=Do)[0] for e in eta])
    res = np.linalg.norm(eta - np.stack([op(x) for x in Xs]), axis=1) / np.linalg.norm(eta, axis=1)
    assert np.all(res <= 1.05e-12)
    X, T, _ = ctx.level(None, g[0], D, mpmc.THETA_I, SEED, 0, 0, N, prec=FP64, solve_tol=1e-12, solve_restart=50)
    Xr, Tr = OES.level_samples(op, None, Po[0], Do, "I", SEED, 0, 0, N, eta=eta, X_solved=Xs)
    bound = 2 * op.n * MINV_BOUND * 1e-12
    print("solve term: max |dX| %.3e (bound %.3e), |X| ~ %.3e" % (np.max(np.abs(X - Xr)), bound,
                                                                 np.max(np.abs(Xr))))
    assert np.max(np.abs(X - Xr)) < bound and T == 0 and Tr == 0
    # polynomial differences with the deflation correction (Sec. 7), then the last term
    for l, (up, lo) in enumerate([(0, 1), (1, 2), (2, None)], start=1):
        X, T, mv = ctx.level(g[up], None if lo is None else g[lo], D, mpmc.THETA_I, SEED, l, 0, N, prec=FP64)
        Xr, Tr = OES.level_samples(op, Po[up], None if lo is None else Po[lo], Do, "I", SEED, l, 0, N)
        print("term %d: max |dX| %.3e, |X| ~ %.3e, T %s vs %s" % (l, np.max(np.abs(X - Xr)), np.max(np.abs(Xr)),
                                                                    T, Tr))
        # the two forms of a difference term are each of size ~n ||M^-1|| and
        # carry FP64 rounding ~1e-14 of that through the recurrence; on this
        # field p_1 and p_2 agree with M^-1 to 1e-11, so the difference samples
        # (~1e-8) sit near that floor: bound 1e-10 relative plus 1e-12 n
        assert np.max(np.abs(X - Xr)) <= 1e-10 * np.max(np.abs(Xr)) + 1e-12 * op.n
        assert abs(T - Tr) < 1e-10 * max(1.0, abs(Tr))
        if lo is not None:
            assert abs(Tr) > 0
