"""Error behaviour of the C ABI on the GPU: every documented argument error
returns its code (EINVAL, ESTATE) with a message naming the call, launches
nothing, and leaves the context usable: the same valid call before and after
the rejected ones gives bit-identical results and the MVP counter does not move
on a rejection.  Marked gpu."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2402_00016_amd import inputs  # noqa: E402
from paper_2402_00016_amd import mpmc  # noqa: E402

FP64, FP32, FP16S = mpmc.FP64, mpmc.FP32, mpmc.FP16S


@pytest.fixture(scope="module")
def ctx():
    dims = (4, 4, 4, 8)
    return mpmc.Context(dims, 0.12, inputs.gauge_links(dims, 0.5, seed=3))


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy().copy()


def rejects(code, word, fn, *args, **kw):
    with pytest.raises(mpmc.MpmcError) as e:
        fn(*args, **kw)
    assert e.value.rc == code, str(e.value)
    assert word in str(e.value), str(e.value)


def test_operator_and_noise_errors_leave_context_usable(ctx):
    h, N = ctx.handle, 8
    x = ctx.noise(5, 1, 0, N, FP32)
    y = ctx.vector(N, FP32)
    before = host(ctx.apply_M(x, N, FP32))
    mv0 = ctx.mvps
    rejects(mpmc.EINVAL, "mpmc_apply_M", mpmc.mpmc_apply_M, h, x, y, 0, FP32)
    rejects(mpmc.EINVAL, "mpmc_apply_M", mpmc.mpmc_apply_M, h, x, y, N, 7)
    rejects(mpmc.EINVAL, "mpmc_apply_M", mpmc.mpmc_apply_M, h, x, y, N, FP32, 0, 9)
    rejects(mpmc.EINVAL, "alias", mpmc.mpmc_apply_M, h, x, x, N, FP32)
    rejects(mpmc.EINVAL, "mpmc_apply_M", mpmc.mpmc_apply_M, h, None, y, N, FP32)
    rejects(mpmc.EINVAL, "mpmc_noise", mpmc.mpmc_noise, h, 1, 0, 0, 0, FP32, y)
    rejects(mpmc.EINVAL, "mpmc_noise", mpmc.mpmc_noise, h, 1, 0, 2 ** 32 - 4, N, FP32, y)
    rejects(mpmc.EINVAL, "mpmc_vector_bytes", ctx.vector, 0, FP32)
    rejects(mpmc.EINVAL, "mpmc_tune_set", mpmc.mpmc_tune_set, h, N, FP32, mpmc.WILSON_VARIANTS)
    assert ctx.mvps == mv0
    after = host(ctx.apply_M(x, N, FP32, out=y))
    assert np.array_equal(before, after)
    assert ctx.mvps == mv0 + N


def test_polynomial_and_estimate_errors(ctx):
    h = ctx.handle
    rejects(mpmc.EINVAL, "mpmc_gmres_poly", ctx.gmres_poly, 1, 0, 0)
    rejects(mpmc.EINVAL, "mpmc_gmres_poly", ctx.gmres_poly, 1, 0, 501)
    rejects(mpmc.EINVAL, "mpmc_poly_create", ctx.poly_from_roots, np.array([1.0, 0.0], dtype=np.complex128))
    rejects(mpmc.EINVAL, "mpmc_poly_create", ctx.poly_from_roots, np.array([np.nan], dtype=np.complex128))
    p = ctx.gmres_poly(1, 0, 4)
    q = ctx.gmres_poly(2, 0, 3, inner=p)
    rejects(mpmc.EINVAL, "single", ctx.gmres_poly, 3, 0, 2, inner=q)
    rejects(mpmc.EINVAL, "mpmc_level_estimate", mpmc.mpmc_level_estimate, h, p, None, None, mpmc.THETA_I,
            1, 0, 0, 0, FP32)
    rejects(mpmc.EINVAL, "mpmc_level_estimate", mpmc.mpmc_level_estimate, h, p, None, None, mpmc.THETA_I,
            1, 0, 0, 4, FP16S)
    rejects(mpmc.EINVAL, "solve level", mpmc.mpmc_level_estimate, h, None, None, None, mpmc.THETA_I,
            1, 0, 0, 4, FP64, solve_tol=0.0)
    other = mpmc.Context((4, 4, 4, 4), 0.12, inputs.gauge_links((4, 4, 4, 4), 0.5, seed=4))
    po = other.gmres_poly(1, 0, 4)
    rejects(mpmc.ESTATE, "another context", mpmc.mpmc_level_estimate, h, po, None, None, mpmc.THETA_I,
            1, 0, 0, 4, FP32)
    # the valid estimate is unchanged by the rejected calls before it
    s1, _, _ = mpmc.mpmc_level_estimate(h, p, None, None, mpmc.THETA_I, 1, 0, 0, 4, FP64)
    rejects(mpmc.EINVAL, "mpmc_level_estimate", mpmc.mpmc_level_estimate, h, p, None, None, 5,
            1, 0, 0, 4, FP64)
    s2, _, _ = mpmc.mpmc_level_estimate(h, p, None, None, mpmc.THETA_I, 1, 0, 0, 4, FP64)
    assert np.array_equal(s1, s2)


def test_solve_errors(ctx):
    h, N = ctx.handle, 4
    b = ctx.noise(9, 0, 0, N, FP64)
    x = ctx.vector(N, FP64)
    for kw in (dict(restart=0), dict(restart=401), dict(tol=0.0), dict(max_outer=0)):
        rejects(mpmc.EINVAL, "mpmc_solve", mpmc.mpmc_solve, h, b, x, N, **kw)
    rejects(mpmc.EINVAL, "alias", mpmc.mpmc_solve, h, b, b, N)
    rejects(mpmc.EINVAL, "inner precision", mpmc.mpmc_solve, h, b, x, N, inner_prec=9)
    its, rel, rc = mpmc.mpmc_solve(h, b, x, N, tol=1e-9, inner_prec=FP32)
    assert rc == mpmc.OK and np.all(rel <= 1e-9)


# ------------------------------------------------ forced failures (host-side) --

def test_nonconvergence_reports_true_residual(ctx):
    """max_outer = 1 with a 1e-12 target: MPMC_ENOCONV, and the reported
    relative residual is the true one of the returned iterate (checked with
    the oracle operator), finite and above the target."""
    from oracle.philox import z4_noise_batch
    from oracle.wilson import WilsonOp
    N = 4
    b = ctx.noise(9, 0, 0, N, FP64)
    x = ctx.vector(N, FP64)
    its, rel, rc = mpmc.mpmc_solve(ctx.handle, b, x, N, restart=4, tol=1e-12, inner_prec=FP32, max_outer=1,
                                   raise_on_noconv=False)
    assert rc == mpmc.ENOCONV and its == 4
    assert "not converged" in mpmc.mpmc_last_error(ctx.handle)
    op = WilsonOp(ctx.dims, ctx.kappa, ctx.links)
    B = z4_noise_batch(9, 0, 0, N, op.n)
    X = host(ctx.unpack(x, N))
    true = np.linalg.norm(B - op(X), axis=1) / np.linalg.norm(B, axis=1)
    assert np.all(np.isfinite(rel)) and np.all(rel > 1e-12)
    assert np.allclose(rel, true, rtol=1e-6)
    with pytest.raises(mpmc.MpmcError) as e:
        ctx.solve(b, N, restart=4, tol=1e-12, inner_prec=FP32, max_outer=1)
    assert e.value.rc == mpmc.ENOCONV


def test_nan_right_hand_side_and_links_are_enumeric(ctx):
    """A NaN in a right-hand side is rejected before any iteration; a NaN link
    makes the first true residual non-finite: both MPMC_ENUMERIC, bounded."""
    N = 2
    canon = torch.zeros((N, ctx.n), dtype=torch.complex128, device="cuda")
    canon[0, 5] = float("nan")
    canon[1, 7] = 1.0
    b = ctx.pack(canon, FP64)
    rejects(mpmc.ENUMERIC, "not finite", ctx.solve, b, N, restart=8, tol=1e-8, max_outer=3)
    U = np.array(ctx.links, copy=True)
    U[3, 1, 0, 0] = np.nan
    bad = mpmc.Context(ctx.dims, ctx.kappa, U)
    bb = bad.noise(1, 0, 0, N, FP64)
    rejects(mpmc.ENUMERIC, "not finite", bad.solve, bb, N, restart=8, tol=1e-8, inner_prec=FP32, max_outer=3)
    # the good context is untouched
    x, its, rel = ctx.solve(ctx.noise(1, 0, 0, N, FP64), N, restart=20, tol=1e-8, inner_prec=FP32)
    assert np.all(rel <= 1e-8)


def test_fp16s_pack_keeps_huge_and_tiny_sites(ctx):
    """FP16 storage with one FP32 scale per (site, rhs): sites whose magnitudes
    span 1e-30 .. 1e+30 keep a relative error below 2^-10 of the site maximum
    (no overflow, no flush), and the FP16S operator on them stays finite."""
    N = 3
    rng = np.random.default_rng(4)
    V = ctx.V
    mag = 10.0 ** rng.uniform(-30, 30, size=(N, V))
    v = (rng.standard_normal((N, V, 12)) + 1j * rng.standard_normal((N, V, 12))) * mag[:, :, None]
    canon = torch.from_numpy(v.reshape(N, ctx.n)).cuda()
    h = ctx.pack(canon, FP16S)
    back = host(ctx.unpack(h, N, FP16S)).reshape(N, V, 12)
    site_max = np.max(np.maximum(np.abs(v.real), np.abs(v.imag)), axis=2)
    err = np.max(np.abs(back - v), axis=2) / site_max
    assert np.all(np.isfinite(back)) and np.max(err) < 2.0 ** -10
    y = host(ctx.unpack(ctx.apply_M(h, N, FP16S), N, FP16S))
    assert np.all(np.isfinite(y))


def test_garbage_deflation_set_keeps_levels_unbiased():
    """A random (garbage) deflation set imported to the GPU: the deflated
    polynomial-difference level still has the dense exact expectation
    Tr(p_a - p_b) (the correction is exact for any triples), per sample equal
    to the oracle's, and the sampled mean is within 3.5 standard errors."""
    from oracle import deflation as ODF
    from oracle import estimator as OES
    from oracle import krylov as OK
    from oracle import poly as OP
    from oracle.philox import z4_noise
    from oracle.wilson import WilsonOp
    dims, kappa = (4, 4, 4, 4), 0.115
    U = inputs.gauge_links(dims, 0.5, seed=1)
    op, c = WilsonOp(dims, kappa, U), mpmc.Context(dims, kappa, U)
    b = z4_noise(1, 0x100, 0, op.n)
    Pa, _, _ = OK.gmres_poly(op, b, 9)
    Pb, _, _ = OK.gmres_poly(op, b, 3)
    rng = np.random.default_rng(11)
    k = 5
    junk = ODF.Deflation(rng.standard_normal(k) + 0.3j * rng.standard_normal(k),
                         rng.standard_normal((k, op.n)) + 1j * rng.standard_normal((k, op.n)),
                         rng.standard_normal((k, op.n)) + 1j * rng.standard_normal((k, op.n)))
    D = c.defl_from_arrays(junk.lam, torch.from_numpy(junk.Z).cuda(), torch.from_numpy(junk.U).cuda())
    ga, gb = c.poly_from_roots(Pa.roots), c.poly_from_roots(Pb.roots)
    N = 256
    X, T, _ = c.level(ga, gb, D, 0, 4, 2, 0, N, prec=FP64)
    Xr, Tr = OES.level_samples(op, Pa, Pb, junk, "I", 4, 2, 0, N)
    assert np.max(np.abs(X - Xr)) < 1e-9 * max(1.0, np.max(np.abs(Xr)))
    assert abs(T - Tr) < 1e-9 * max(1.0, abs(Tr))
    exact = np.trace(OP.apply_poly(op, Pa, np.eye(op.n)).T - OP.apply_poly(op, Pb, np.eye(op.n)).T)
    m, v = OES.level_stats(X)
    assert abs(m + T - exact) < 3.5 * np.sqrt(v / N)
