"""GPU parity at the full sizes of the 16^4 and 24^4 configurations, in the
launch configuration bench.py uses (all noise vectors of a term in one
batch), checked against the FP64 oracle on sampled right-hand sides that the
oracle computes one by one, and by properties that hold at any size.

Tolerances: FP32 kernels with FP64 sums -- a level sample is a sum of n terms
|eta_c|^2 p ~ O(1) with FP32 relative rounding ~6e-8 per term, so the sample
error is bounded by ~1e-6 n (bound used: 1e-5 n); FP64 polynomial application
1e-11 relative; solves: the oracle's true relative residual <= 1.05 x the
requested tolerance; network forward 2.5e-2 (BF16 operands, as in
test_gpu_net.py).
"""
import numpy as np
import pytest

pytestmark = [pytest.mark.gpu, pytest.mark.slow]

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from oracle import krylov as OK  # noqa: E402
from oracle import net as ON  # noqa: E402
from oracle import poly as OP  # noqa: E402
from oracle.philox import z4_noise  # noqa: E402
from oracle.wilson import WilsonOp  # noqa: E402
from paper_2402_00016_amd import driver, inputs, mpmc  # noqa: E402

FP64, FP32 = mpmc.FP64, mpmc.FP32


def rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def g5(v):
    w = np.array(v, dtype=np.complex128).reshape(-1, 4, 3)
    w[:, 2:, :] *= -1
    return w.reshape(-1)


@pytest.fixture(scope="module")
def f24():
    dims, kappa = (24, 24, 24, 24), 0.1245
    U = inputs.gauge_links(dims, 0.4, seed=4)
    ctx = mpmc.Context(dims, kappa, U)
    yield dims, kappa, U, WilsonOp(dims, kappa, U), ctx
    ctx.release_workspace()
    torch.cuda.empty_cache()


@pytest.fixture(scope="module")
def f16():
    dims, kappa = (16, 16, 16, 16), 0.124
    U = inputs.gauge_links(dims, 0.4, seed=3)
    ctx = mpmc.Context(dims, kappa, U)
    yield dims, kappa, U, WilsonOp(dims, kappa, U), ctx
    ctx.release_workspace()
    torch.cuda.empty_cache()


def test_24_gmres_roots(f24):
    dims, kappa, U, op, ctx = f24
    P = ctx.gmres_poly(4, 0x103, 9)
    ref, de, rr = OK.gmres_poly(op, z4_noise(4, 0x103, 0, op.n), 9)
    d = np.abs(np.subtract.outer(P.roots, ref.roots)).min(axis=1).max()
    assert P.d_eff == de == 9 and d < 1e-9 * np.abs(ref.roots).max()
    assert abs(P.relres - rr) < 1e-9 * rr


@pytest.mark.parametrize("prec,tol", [(FP64, 1e-9), (FP32, 1e-4)])
def test_24_delayed_gram_schmidt_matches_plain(f24, prec, tol):
    """At 24^4 the delayed Gram-Schmidt's dot pass runs with 8 (FP64) or 4
    (FP32) 16-byte slots per thread: GMRES(33) roots and relres equal plain
    CGS2's to rounding of the storage precision."""
    dims, kappa, U, op, ctx = f24
    ctx.set_setup_precision(prec)
    out = []
    try:
        for cgs2 in (1, 0):
            ctx.set_arnoldi_cgs2(cgs2)
            out.append(ctx.gmres_poly(4, 0x104, 33))
    finally:
        ctx.set_arnoldi_cgs2(-1)
        ctx.set_setup_precision(FP64)
    P1, P0 = out
    assert P0.d_eff == P1.d_eff == 33
    d = np.abs(np.subtract.outer(P0.roots, P1.roots)).min(axis=1).max()
    assert d < tol * np.abs(P1.roots).max()
    assert abs(P0.relres - P1.relres) < tol * P1.relres


@pytest.mark.parametrize("theta", [mpmc.THETA_I, mpmc.THETA_G5])
def test_24_fused_level_step_sampled(f24, theta):
    """Tr(Theta p(M)) samples of 64 noise vectors in one FP32 fused batch; two
    samples recomputed by the oracle with the GPU's roots."""
    dims, kappa, U, op, ctx = f24
    P = ctx.gmres_poly(4, 0x103, 9)
    N = 64
    X, corr, mv = ctx.level(P, None, None, theta, 4, 3, 0, N, prec=FP32)
    for j in (0, 37):
        eta = z4_noise(4, 3, j, op.n)
        y = OP.apply_p(op, P.roots, eta)
        ref = np.vdot(eta, g5(y) if theta == mpmc.THETA_G5 else y)
        assert abs(X[j] - ref) < 1e-5 * op.n


def test_24_column_kernels_agree(f24):
    """At the bench's shape (24^4, 64 right-hand sides) the column kernel with
    2x2x4 tiles and 32-wide chunks (variant 12) gives the 2x2x2 kernel's
    operator bit for bit and its fused level samples up to the grouping of
    the FP64 sums, with the block order alternating between the launches."""
    dims, kappa, U, op, ctx = f24
    N = 64
    x = ctx.noise(4, 5, 0, N, FP32)
    out = {}
    for v in (10, 12):
        ctx.tune_set(N, FP32, v)
        out[v] = ctx.apply_M(x, N, FP32)
    assert torch.equal(out[10], out[12])
    P = ctx.gmres_poly(4, 0x104, 6)
    X = {}
    for v in (10, 12):
        ctx.tune_set(N, FP32, v)
        X[v] = ctx.level(P, None, None, mpmc.THETA_I, 4, 6, 0, N, prec=FP32)[0]
        # five fused launches: the repeat starts with the other block order
        again = ctx.level(P, None, None, mpmc.THETA_I, 4, 6, 0, N, prec=FP32)[0]
        assert np.array_equal(again, X[v])
    ctx.tune_set(N, FP32, -1)
    assert np.max(np.abs(X[12] - X[10])) < 1e-12 * np.max(np.abs(X[10]))


def test_24_double_poly_fp64_sampled(f24):
    dims, kappa, U, op, ctx = f24
    pin = ctx.gmres_poly(4, 0x100, 16)
    P = ctx.gmres_poly(4, 0x100, 16, inner=pin)
    assert P.info["degree"] == 255
    N = 64
    x = ctx.noise(9, 1, 0, N, FP64)
    y = ctx.unpack(ctx.apply_poly(P, x, N, FP64), N, FP64)
    ref = OP.apply_poly(op, OK.GmresPoly(P.roots, inner=OK.GmresPoly(pin.roots)), z4_noise(9, 1, N - 1, op.n))
    assert rel(y[N - 1].cpu().numpy(), ref) < 1e-11
    del x, y
    torch.cuda.empty_cache()


def test_24_solve_true_residual_sampled(f24):
    dims, kappa, U, op, ctx = f24
    N = 64
    b = ctx.noise(5, 2, 0, N, FP64)
    x, its, relres = ctx.solve(b, N, restart=50, tol=1e-8, inner_prec=FP32)
    assert np.all(relres <= 1e-8)
    X = ctx.unpack(x, N, FP64)
    for j in (0, 50):
        bj = z4_noise(5, 2, j, op.n)
        r = bj - op(X[j].cpu().numpy())
        assert np.linalg.norm(r) / np.linalg.norm(bj) <= 1.05e-8
    del b, x, X
    ctx.release_workspace()
    torch.cuda.empty_cache()


def test_24_net_forward_sampled(f24):
    dims, kappa, U, op, ctx = f24
    rng = np.random.default_rng(0)
    theta = 0.3 * rng.standard_normal(ON.n_params())
    N = 16
    x = ctx.noise(7, 0, 0, N, FP32)
    y = ctx.unpack(ctx.net(theta).apply(x, N), N, FP32)
    T = ON.Transport(dims, U)
    for j in (0, 11):
        ref = ON.apply_net(T, theta, z4_noise(7, 0, j, op.n)[None, :])[0]
        assert rel(y[j].cpu().numpy(), ref) < 2.5e-2
    del x, y
    torch.cuda.empty_cache()


def test_16_double_poly_level_sampled(f16):
    """The 16^4 configuration: 16x16 double polynomial, 256 right-hand sides in
    one fused FP32 batch; two samples against the oracle."""
    dims, kappa, U, op, ctx = f16
    pin = ctx.gmres_poly(3, 0x100, 16)
    P = ctx.gmres_poly(3, 0x100, 16, inner=pin)
    N = 256
    X, corr, mv = ctx.level(P, None, None, mpmc.THETA_I, 3, 1, 0, N, prec=FP32)
    Po = OK.GmresPoly(P.roots, inner=OK.GmresPoly(pin.roots))
    for j in (3, 255):
        eta = z4_noise(3, 1, j, op.n)
        ref = np.vdot(eta, OP.apply_poly(op, Po, eta))
        assert abs(X[j] - ref) < 1e-5 * op.n


def test_16_deflation_100_requested(f16):
    """PP-Arnoldi at 16^4 asked for 100 eigenpairs: every accepted pair meets
    the acceptance rule under the oracle operator, u^H z = 1."""
    dims, kappa, U, op, ctx = f16
    plan = driver.Plan(degrees=[(15, 15)], nev=100, defl_candidates=120, defl_m=136, defl_pin_degree=8, seed=3)
    D = driver.build_deflation(ctx, plan)
    assert D.k >= 1
    lam, Z, Uv = ctx.defl_vectors(D)
    for i in sorted({0, D.k // 2, D.k - 1}):
        z, u = Z[i].cpu().numpy(), Uv[i].cpu().numpy()
        assert abs(np.linalg.norm(z) - 1) < 1e-10
        assert abs(np.vdot(u, z) - 1) < 1e-10
        assert np.linalg.norm(op(z) - lam[i] * z) < 1e-3
        un = u / np.linalg.norm(u)
        assert np.linalg.norm(op.dagger(un) - np.conj(lam[i]) * un) < 1e-3
    assert np.all(np.diff(np.abs(lam)) >= -1e-12)     # ordered by |lambda|
