"""GPU parity: every call of the C ABI against the FP64 oracle on the same
seeded inputs (run on an MI355X; marked gpu).

Tolerances (derived from the arithmetic):
* Z(4) noise, indexing, pack/unpack in FP64: bit-exact.
* FP64 operator: ||y_gpu - y_oracle|| / ||y_oracle|| <= 1e-13 (sums of ~100
  terms in a different order, unit roundoff 1.1e-16).
* FP32 operator: <= 2e-6 (FP32 links and spinors, unit roundoff 6e-8, ~100
  terms per component).
* FP16S operator output: <= 1.5e-3 (half storage, 2^-11 relative to the
  per-(site, rhs) maximum).
* FP64 polynomials / solves / level samples: 1e-10 relative (the FP64-mode parity bound).
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
from oracle import lattice as OLT  # noqa: E402
from oracle import poly as OP  # noqa: E402
from oracle import solve as OS  # noqa: E402
from oracle.philox import z4_noise, z4_noise_batch  # noqa: E402
from oracle.wilson import WilsonOp  # noqa: E402
from paper_2402_00016_amd import inputs  # noqa: E402
from paper_2402_00016_amd import mpmc  # noqa: E402

FP64, FP32, FP16S = mpmc.FP64, mpmc.FP32, mpmc.FP16S


def rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


@pytest.fixture(scope="module")
def f44():
    dims, kappa = (4, 4, 4, 4), 0.115
    U = inputs.gauge_links(dims, 0.5, seed=1)
    return dims, kappa, U, WilsonOp(dims, kappa, U), mpmc.Context(dims, kappa, U)


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


# ------------------------------------------------------------------ noise --

@pytest.mark.parametrize("prec", [FP64, FP32, FP16S])
@pytest.mark.parametrize("N,seed,stream,first", [(1, 1, 0, 0), (5, 7, 3, 11), (64, 2 ** 40 + 5, 0x100, 1000)])
def test_noise_bit_exact(f44, prec, N, seed, stream, first):
    dims, kappa, U, op, ctx = f44
    eta = ctx.noise(seed, stream, first, N, prec)
    got = host(ctx.unpack(eta, N, prec))
    ref = z4_noise_batch(seed, stream, first, N, op.n)
    assert np.array_equal(got, ref)


def test_noise_bit_exact_ragged_lattice():
    dims = (3, 5, 2, 7)
    U = inputs.gauge_links(dims, 0.4, seed=5)
    ctx = mpmc.Context(dims, 0.1, U)
    n = 12 * int(np.prod(dims))
    got = host(ctx.unpack(ctx.noise(9, 2, 3, 3, FP64), 3, FP64))
    assert np.array_equal(got, z4_noise_batch(9, 2, 3, 3, n))


# ----------------------------------------------------------- pack/unpack --

def test_pack_roundtrip(f44):
    dims, kappa, U, op, ctx = f44
    rng = np.random.default_rng(0)
    X = rng.standard_normal((7, op.n)) + 1j * rng.standard_normal((7, op.n))
    Xd = torch.from_numpy(X).cuda()
    assert np.array_equal(host(ctx.unpack(ctx.pack(Xd, FP64), 7, FP64)), X)
    assert rel(host(ctx.unpack(ctx.pack(Xd, FP32), 7, FP32)), X) < 1e-7
    assert rel(host(ctx.unpack(ctx.pack(Xd, FP16S), 7, FP16S)), X) < 1e-3


# -------------------------------------------------------------- operator --

TOL = {FP64: 1e-13, FP32: 2e-6, FP16S: 1.5e-3}


@pytest.mark.parametrize("prec", [FP64, FP32, FP16S])
@pytest.mark.parametrize("N", [1, 3, 64, 65])
@pytest.mark.parametrize("dagger,theta", [(0, 0), (1, 0), (0, 1)])
def test_apply_M_parity(f44, prec, N, dagger, theta):
    dims, kappa, U, op, ctx = f44
    rng = np.random.default_rng(N + 10 * dagger + 100 * theta)
    X = rng.standard_normal((N, op.n)) + 1j * rng.standard_normal((N, op.n))
    x = ctx.pack(torch.from_numpy(X).cuda(), prec)
    y = ctx.apply_M(x, N, prec, dagger=dagger, theta=theta)
    got = host(ctx.unpack(y, N, prec))
    Xin = host(ctx.unpack(x, N, prec))          # what the kernel actually read
    ref = op.dagger(Xin) if dagger else op(Xin)
    if theta:
        ref = OLT.spin_op(ref, OLT.GAMMA5)
    assert rel(got, ref) < TOL[prec]


def test_apply_M_free_field_and_kappa0():
    dims = (4, 4, 4, 6)
    ctx = mpmc.Context(dims, 0.11, inputs.unit_links(dims))
    p = OLT.free_momenta(dims)[77]
    chi = (np.arange(12).reshape(4, 3) + 1j).astype(np.complex128)
    psi = OLT.plane_wave(dims, p, chi)
    y = host(ctx.unpack(ctx.apply_M(ctx.pack(torch.from_numpy(psi[None]).cuda()), 1), 1))[0]
    assert rel(y, OLT.plane_wave(dims, p, OLT.free_symbol(p, 0.11) @ chi)) < 1e-13
    ctx0 = mpmc.Context(dims, 0.0, inputs.gauge_links(dims, 0.5, seed=3))
    e = ctx0.noise(1, 0, 0, 2)
    assert torch.equal(ctx0.apply_M(e, 2), e)


@pytest.mark.parametrize("L,N,prec", [(8, 128, FP32), (16, 64, FP32), (24, 64, FP32), (8, 16, FP64)])
def test_apply_M_full_size_sampled(L, N, prec):
    """Full-size shapes in the bench launch configuration; the oracle checks
    two sampled right-hand sides (first and last) of the Z(4) input."""
    dims = (L, L, L, L)
    U = inputs.gauge_links(dims, 0.4, seed=4)
    ctx = mpmc.Context(dims, 0.1245, U)
    op = WilsonOp(dims, 0.1245, U)
    eta = ctx.noise(3, 0, 0, N, prec)
    y = ctx.apply_M(eta, N, prec)
    full = ctx.unpack(y, N, prec)
    for r in (0, N - 1):
        got = full[r].cpu().numpy()
        ref = op(z4_noise(3, 0, r, op.n))
        assert rel(got, ref) < TOL[prec]
    del y, full, eta
    torch.cuda.empty_cache()


# ------------------------------------------------------------ polynomials --

def _match_sets(a, b):
    """max over a of the distance to the nearest element of b (and vice versa)."""
    a, b = np.asarray(a), np.asarray(b)
    d1 = max(np.min(np.abs(b - x)) for x in a)
    d2 = max(np.min(np.abs(a - x)) for x in b)
    return max(d1, d2)


@pytest.mark.parametrize("d", [4, 9, 16])
def test_gmres_poly_roots_parity(f44, d):
    dims, kappa, U, op, ctx = f44
    P = ctx.gmres_poly(1, 0x100, d)
    ref, de, rr = OK.gmres_poly(op, z4_noise(1, 0x100, 0, op.n), d)
    assert P.d_eff == de == d
    roots = P.roots
    assert _match_sets(roots, ref.roots) < 1e-9 * np.max(np.abs(ref.roots))
    assert abs(abs(roots[0]) - abs(ref.roots[0])) < 1e-9     # Leja starts at the largest modulus
    assert abs(P.relres - rr) < 1e-9 * max(rr, 1e-12) + 1e-13


def test_gmres_poly_roots_parity_high_degree():
    """degree 47 on a slowly converging operator (kappa 0.2): many QR sweeps"""
    dims, kappa = (4, 4, 4, 4), 0.2
    U = inputs.gauge_links(dims, 0.5, seed=21)
    op, ctx = WilsonOp(dims, kappa, U), mpmc.Context(dims, kappa, U)
    P = ctx.gmres_poly(1, 0x100, 48)
    ref, de, rr = OK.gmres_poly(op, z4_noise(1, 0x100, 0, op.n), 48)
    assert P.d_eff == de == 48
    assert _match_sets(P.roots, ref.roots) < 1e-8 * np.max(np.abs(ref.roots))
    assert abs(P.relres - rr) < 1e-8 * rr


@pytest.mark.parametrize("dims,kappa,seed,d", [((4, 4, 4, 4), 0.2, 21, 48), ((8, 8, 8, 8), 0.12, 2, 129),
                                               ((8, 8, 8, 8), 0.12, 2, 33), ((4, 4, 4, 4), 0.115, 1, 300)])
def test_dense_eigensolvers_agree(dims, kappa, seed, d):
    """Harmonic Ritz values by the Aberth-Ehrlich iteration (the default) and by
    the shifted QR agree to rounding, and each set comes out in the oracle's
    Leja order of its own values.  d = 300 (more than 256 rows) takes the QR
    in both settings."""
    U = inputs.gauge_links(dims, 0.5, seed=seed)
    ctx = mpmc.Context(dims, kappa, U)
    P_ab = ctx.gmres_poly(1, 0x100, d)
    ctx.set_dense_method(mpmc.DENSE_QR)
    P_qr = ctx.gmres_poly(1, 0x100, d)
    ctx.set_dense_method(mpmc.DENSE_ABERTH)
    assert P_ab.d_eff == P_qr.d_eff == d
    scale = np.max(np.abs(P_qr.roots))
    assert _match_sets(P_ab.roots, P_qr.roots) < 1e-11 * scale
    assert abs(P_ab.relres - P_qr.relres) <= 1e-12 * P_qr.relres
    for P in (P_ab, P_qr):
        assert np.max(np.abs(OK.leja_order(P.roots) - P.roots)) <= 1e-13 * scale
    with pytest.raises(mpmc.MpmcError):
        ctx.set_dense_method(2)


def test_gmres_poly_breakdown_kappa0():
    dims = (2, 2, 2, 2)
    ctx = mpmc.Context(dims, 0.0, inputs.gauge_links(dims, 0.5, seed=1))
    P = ctx.gmres_poly(1, 0x100, 16)
    assert P.d_eff == 1
    assert np.allclose(P.roots, [1.0])


@pytest.mark.parametrize("N", [1, 5])
@pytest.mark.parametrize("prec,tol", [(FP64, 1e-12), (FP32, 2e-5)])
def test_apply_poly_parity(f44, prec, tol, N):
    """N = 1 is the single-vector kernel, whose first step also starts the
    accumulator at x / theta_1."""
    dims, kappa, U, op, ctx = f44
    ref, _, _ = OK.gmres_poly(op, z4_noise(1, 0x100, 0, op.n), 16)
    P = ctx.poly_from_roots(ref.roots)
    eta = ctx.noise(4, 1, 0, N, prec)
    got = host(ctx.unpack(ctx.apply_poly(P, eta, N, prec), N, prec))
    E = z4_noise_batch(4, 1, 0, N, op.n)
    want = np.stack([OP.apply_p(op, ref.roots, e) for e in E])
    assert rel(got, want) < tol
    assert P.info["degree"] == 15 and P.info["matvecs"] == 15


@pytest.mark.parametrize("variant", [1, 2])
@pytest.mark.parametrize("prec,tol_m,tol_p", [(FP64, 1e-13, 1e-12), (FP32, 2e-6, 2e-5)])
def test_single_vector_site_per_lane(f44, prec, tol_m, tol_p, variant):
    """Single vectors with one site per lane, pinned with mpmc_tune_set(ctx, 1,
    prec, v): v = 2 the single-vector kernel (the default above 12^4 sites),
    v = 1 the generic kernel at one right-hand side.  M, M^H and gamma5 M
    against the oracle, and a polynomial on one vector (its accumulator start
    y = x / theta_1 fused into the first step for v = 2, a separate pass for
    v = 1)."""
    dims, kappa, U, op, ctx = f44
    xh = z4_noise(9, 1, 0, op.n)
    ref, _, _ = OK.gmres_poly(op, z4_noise(1, 0x100, 0, op.n), 16)
    ctx.tune_set(1, prec, variant)
    try:
        x = ctx.noise(9, 1, 0, 1, prec)
        for dagger, theta in ((False, 0), (True, 0), (False, 1)):
            y = host(ctx.unpack(ctx.apply_M(x, 1, prec, dagger=dagger, theta=theta), 1, prec))[0]
            want = op.dagger(xh) if dagger else op(xh)
            if theta:
                want = OLT.spin_op(want[None, :], OLT.theta_matrix("g5"))[0]
            assert rel(y, want) < tol_m, (dagger, theta)
        P = ctx.poly_from_roots(ref.roots)
        got = host(ctx.unpack(ctx.apply_poly(P, x, 1, prec), 1, prec))[0]
        assert rel(got, OP.apply_p(op, ref.roots, xh)) < tol_p
    finally:
        ctx.tune_set(1, prec, -1)


@pytest.mark.parametrize("prec", [FP64, FP32])
@pytest.mark.parametrize("dims", [(4, 4, 4, 4), (3, 5, 4, 6)])
def test_single_vector_kernel_matches_generic(prec, dims):
    """The single-vector kernel computes each hop with the generic kernel's
    arithmetic from coordinate-derived neighbours: M, M^H and gamma5 M equal
    the generic kernel's bit for bit on a lattice with odd extents (every
    boundary wraps, antiperiodic in t), and against the oracle."""
    kappa = 0.12
    U = inputs.gauge_links(dims, 0.5, seed=4)
    op, ctx = WilsonOp(dims, kappa, U), mpmc.Context(dims, kappa, U)
    x = ctx.noise(11, 2, 0, 1, prec)
    xh = z4_noise(11, 2, 0, op.n)
    tol = 1e-13 if prec == FP64 else 2e-6
    for dagger, theta in ((False, 0), (True, 0), (False, 1), (True, 1)):
        out = {}
        for v in (1, 2):
            ctx.tune_set(1, prec, v)
            out[v] = ctx.apply_M(x, 1, prec, dagger=dagger, theta=theta)
        ctx.tune_set(1, prec, -1)
        assert torch.equal(out[1], out[2]), (dagger, theta)
        want = op.dagger(xh) if dagger else op(xh)
        if theta:
            want = OLT.spin_op(want[None, :], OLT.theta_matrix("g5"))[0]
        assert rel(host(ctx.unpack(out[2], 1, prec))[0], want) < tol


def test_pi_equals_one_minus_M_p_on_gpu(f44):
    """pi(M) = 1 - M p(M) with the GPU's own roots: residual of the GMRES cycle."""
    dims, kappa, U, op, ctx = f44
    P = ctx.gmres_poly(1, 0x100, 16)
    b = ctx.noise(1, 0x100, 0, 1)
    Mp = host(ctx.unpack(ctx.apply_M(ctx.apply_poly(P, b, 1), 1), 1))[0]
    bb = z4_noise(1, 0x100, 0, op.n)
    lhs = OP.apply_pi(op, P.roots, bb)
    # b - M p(M) b cancels to ||pi(M) b|| ~ 1e-5 ||b||: FP64 rounding of the
    # O(||b||) terms is amplified by ||b|| / ||pi(M) b||
    amp = np.linalg.norm(bb) / np.linalg.norm(lhs)
    assert rel(bb - Mp, lhs) < 1e-14 * amp
    assert abs(np.linalg.norm(lhs) / np.linalg.norm(bb) - P.relres) < 1e-10


def test_double_poly_parity(f44):
    dims, kappa, U, op, ctx = f44
    b = z4_noise(1, 0x100, 0, op.n)
    Dref, _, _ = OP.double_poly(op, b, 5, 4)
    Pin = ctx.gmres_poly(1, 0x100, 5)
    Pd = ctx.gmres_poly(1, 0x100, 4, inner=Pin)
    assert _match_sets(Pin.roots, Dref.inner.roots) < 1e-9
    assert _match_sets(Pd.roots, Dref.roots) < 1e-8
    assert Pd.info["degree"] == 19 and Pd.info["matvecs"] == 19
    # application with the oracle's roots imported on both levels
    Pi2 = ctx.poly_from_roots(Dref.inner.roots)
    Pd2 = ctx.poly_from_roots(Dref.roots, inner=Pi2)
    eta = ctx.noise(8, 2, 0, 3)
    got = host(ctx.unpack(ctx.apply_poly(Pd2, eta, 3), 3))
    want = np.stack([OP.apply_poly(op, Dref, e) for e in z4_noise_batch(8, 2, 0, 3, op.n)])
    assert rel(got, want) < 1e-12
    lam = np.array([0.3 + 0.2j, 0.9, 1.4 - 0.1j])
    assert np.allclose(Pd2.eval(lam), OP.eval_poly(Dref, lam), rtol=1e-13)


# -------------------------------------------------------------- deflation --

@pytest.mark.parametrize("m,method", [(80, mpmc.DENSE_ABERTH), (150, mpmc.DENSE_ABERTH), (80, mpmc.DENSE_QR),
                                      (150, mpmc.DENSE_QR)])   # QR at 150: from global memory
def test_deflate_parity(m, method):
    dims, kappa = (4, 4, 4, 4), 0.2
    U = inputs.gauge_links(dims, 0.5, seed=21)
    op, ctx = WilsonOp(dims, kappa, U), mpmc.Context(dims, kappa, U)
    ctx.set_dense_method(method)
    Pin_ref, _, _ = OK.gmres_poly(op, z4_noise(1, 0x100, 0, op.n), 4)
    Pin = ctx.poly_from_roots(Pin_ref.roots)
    D = ctx.deflate(Pin, 1, 0x200, m=m, nev=10)
    Dref, info = ODF.pp_arnoldi_eigs(op, Pin_ref.roots, z4_noise(1, 0x200, 0, op.n), m, 10)
    assert D.k >= 1 and abs(D.k - Dref.k) <= 2
    lam, Z, Uv = ctx.defl_vectors(D)
    assert _match_sets(lam, Dref.lam) < 1e-7
    Zh, Uh = Z.cpu().numpy(), Uv.cpu().numpy()
    for i in range(D.k):
        assert abs(np.vdot(Uh[i], Zh[i]) - 1) < 1e-10
        assert np.linalg.norm(op(Zh[i]) - lam[i] * Zh[i]) < 1e-3
        u = Uh[i] / np.linalg.norm(Uh[i])
        assert np.linalg.norm(op.dagger(u) - np.conj(lam[i]) * u) < 1e-3


# ------------------------------------------------------------------ solve --

@pytest.mark.parametrize("inner", [FP64, FP32, FP16S])
def test_solve_true_residual(f44, inner):
    dims, kappa, U, op, ctx = f44
    N = 6
    b = ctx.noise(5, 0, 0, N, FP64)
    x, its, relres = ctx.solve(b, N, restart=20, tol=1e-10, inner_prec=inner)
    X = host(ctx.unpack(x, N))
    B = z4_noise_batch(5, 0, 0, N, op.n)
    R = B - op(X)
    rr = np.linalg.norm(R, axis=1) / np.linalg.norm(B, axis=1)
    assert np.all(rr <= 1.05e-10)
    assert np.allclose(rr, relres, rtol=1e-3, atol=1e-14)


def test_solve_with_imported_deflation(f44):
    dims, kappa, U, op, ctx = f44
    Pin_ref, _, _ = OK.gmres_poly(op, z4_noise(1, 0x100, 0, op.n), 4)
    Dref, _ = ODF.pp_arnoldi_eigs(op, Pin_ref.roots, z4_noise(1, 0x200, 0, op.n), 60, 8)
    D = ctx.defl_from_arrays(Dref.lam, torch.from_numpy(Dref.Z).cuda(), torch.from_numpy(Dref.U).cuda())
    b = ctx.noise(6, 0, 0, 4)
    x, its, relres = ctx.solve(b, 4, defl=D, restart=20, tol=1e-10, inner_prec=FP32)
    X = host(ctx.unpack(x, 4))
    B = z4_noise_batch(6, 0, 0, 4, op.n)
    assert np.all(np.linalg.norm(B - op(X), axis=1) / np.linalg.norm(B, axis=1) <= 1.05e-10)


# ----------------------------------------------------------------- levels --

def test_level_samples_parity(f44):
    """Same noise, same (imported) polynomials and eigenpairs: per-sample
    values of every level kind agree with the oracle to 1e-10."""
    dims, kappa, U, op, ctx = f44
    b = z4_noise(1, 0x100, 0, op.n)
    P1, _, _ = OK.gmres_poly(op, b, 17)
    P2, _, _ = OK.gmres_poly(op, b, 9)
    Pin, _, _ = OK.gmres_poly(op, b, 4)
    Dref, _ = ODF.pp_arnoldi_eigs(op, Pin.roots, z4_noise(1, 0x200, 0, op.n), 60, 8)
    g1, g2 = ctx.poly_from_roots(P1.roots), ctx.poly_from_roots(P2.roots)
    D = ctx.defl_from_arrays(Dref.lam, torch.from_numpy(Dref.Z).cuda(), torch.from_numpy(Dref.U).cuda())
    N = 8
    for theta, th in (("I", 0), ("g5", 1)):
        # polynomial-difference level with deflation
        X, T, mv = ctx.level(g1, g2, D, th, 3, 2, 0, N)
        Xr, Tr = OES.level_samples(op, P1, P2, Dref, theta, 3, 2, 0, N)
        assert rel(X, Xr) < 1e-10 and abs(T - Tr) < 1e-10 * max(1, abs(Tr))
        assert mv == N * (16 + 8)
        # last level
        X, T, _ = ctx.level(g2, None, None, th, 3, 3, 0, N)
        Xr, _ = OES.level_samples(op, P2, None, None, theta, 3, 3, 0, N)
        assert rel(X, Xr) < 1e-10 and T == 0
        # solve level: each side solves to relative residual 1e-12, so a sample
        # can differ by |eta^H (x - x*)| <= ||eta||^2 ||M^-1|| 1e-12 per side
        # (||eta||^2 = n, ||M^-1|| < 10 on this field)
        X, T, _ = ctx.level(None, g1, None, th, 3, 1, 0, N, solve_tol=1e-12, solve_restart=30)
        Xr, _ = OES.level_samples(op, None, P1, None, theta, 3, 1, 0, N, solve_tol=1e-12)
        assert np.max(np.abs(X - Xr)) < 2 * op.n * 10 * 1e-12


@pytest.mark.parametrize("prec,theta", [(FP64, 0), (FP32, 0), (FP32, 1)])
def test_levels_multi_equal_one_at_a_time(f44, prec, theta):
    """mpmc_level_estimate_multi gives the samples, corrections and MVPs of
    mpmc_level_estimate term by term, bit for bit: single polynomials of
    degrees 16, 8, 3 and 0 share launches (the degree-0 one needs no step), a
    double polynomial term falls back to one term at a time, and one term has
    no lower polynomial.  Against the oracle on the first term as well."""
    dims, kappa, U, op, ctx = f44
    b = z4_noise(1, 0x100, 0, op.n)
    P1, _, _ = OK.gmres_poly(op, b, 17)
    P2, _, _ = OK.gmres_poly(op, b, 9)
    P3, _, _ = OK.gmres_poly(op, b, 4)
    Pin, _, _ = OK.gmres_poly(op, b, 4)
    Dref, _ = ODF.pp_arnoldi_eigs(op, Pin.roots, z4_noise(1, 0x200, 0, op.n), 60, 8)
    D = ctx.defl_from_arrays(Dref.lam, torch.from_numpy(Dref.Z).cuda(), torch.from_numpy(Dref.U).cuda())
    g1, g2, g3 = (ctx.poly_from_roots(P.roots) for P in (P1, P2, P3))
    g0 = ctx.poly_from_roots(P1.roots[:1])
    gin = ctx.poly_from_roots(P3.roots)
    gd = ctx.poly_from_roots(P3.roots[:3], inner=gin)
    ups = [g1, g2, g3, gd, g0]
    los = [g2, g3, g0, g3, None]
    streams = [1, 2, 3, 4, 5]
    N = 64
    ctx.tune_set(N, prec, 5)   # the blocked 64-wide traversal of the shared launches, also for the fallbacks
    try:
        Xs, Ts, mv = ctx.levels_multi(ups, los, D, theta, 3, streams, 7, N, prec=prec)
        mv_one = 0
        for t, (u, l) in enumerate(zip(ups, los)):
            X, T, m = ctx.level(u, l, D if l is not None else None, theta, 3, streams[t], 7, N, prec=prec)
            assert np.array_equal(Xs[t], X), t
            assert Ts[t] == T
            mv_one += m
        # any other traversal groups the FP64 partial sums differently: the
        # sample (a difference of two forms of size ~n) moves by ~1e-16 n
        ctx.tune_set(N, prec, -1)
        X, _, _ = ctx.level(ups[0], los[0], D, theta, 3, streams[0], 7, N, prec=prec)
        assert np.max(np.abs(X - Xs[0])) < 1e-12 * op.n
    finally:
        ctx.tune_set(N, prec, -1)
    assert mv == mv_one
    Xr, Tr = OES.level_samples(op, P1, P2, Dref, "g5" if theta else "I", 3, 1, 7, N)
    assert abs(Ts[0] - Tr) < 1e-10 * max(1, abs(Tr))
    if prec == FP64:
        assert rel(Xs[0], Xr) < 1e-10
    # 20 noises: no 64-wide chunks, every term one at a time (same values)
    Xs20, _, _ = ctx.levels_multi(ups[:2], los[:2], D, theta, 3, streams[:2], 7, 20, prec=prec)
    for t in range(2):
        assert np.array_equal(Xs20[t], ctx.level(ups[t], los[t], D, theta, 3, streams[t], 7, 20, prec=prec)[0])
    with pytest.raises(mpmc.MpmcError):
        ctx.levels_multi([None], [g1], D, theta, 3, [1], 0, N, prec=prec)
    with pytest.raises(mpmc.MpmcError):
        ctx.levels_multi(ups[:1], los[:1], D, theta, 3, [1], 0, N, prec=mpmc.FP16S)


def test_plain_4444_estimate_vs_dense_exact(f44):
    """4^4, kappa 0.115: 32 Z(4) noises, Hutchinson and the subtracted level
    against the dense exact traces of M^-1 and M^-1 - p(M)."""
    dims, kappa, U, op, ctx = f44
    M = OLT.dense_wilson(dims, kappa, U)
    Minv = np.linalg.inv(M)
    P = ctx.gmres_poly(1, 0x100, 16)
    Pm = OP.apply_p(op, P.roots, np.eye(op.n)).T
    X, _, _ = ctx.level(None, None, None, 0, 1, 0, 0, 32, solve_tol=1e-10)
    m, v = OES.level_stats(X)
    assert abs(m - np.trace(Minv)) < 3.5 * np.sqrt(v / 32)
    Xs, _, _ = ctx.level(None, P, None, 0, 1, 1, 0, 32, solve_tol=1e-12)
    ms, vs = OES.level_stats(Xs)
    assert abs(ms - np.trace(Minv - Pm)) < 3.5 * np.sqrt(vs / 32) + 1e-9
    assert vs < 1e-3 * v


# ------------------------------------------------- fused level steps --

@pytest.mark.parametrize("N", [64, 128, 256, 512])
def test_fused_level_parity(f44, N):
    """Batches that are multiples of 64 use the fused step (eta^H Theta w
    accumulated inside the Wilson kernel): per-sample parity with the oracle,
    single and double polynomials, Theta = I and g5, FP64."""
    dims, kappa, U, op, ctx = f44
    b = z4_noise(1, 0x100, 0, op.n)
    P1, _, _ = OK.gmres_poly(op, b, 9)
    D, _, _ = OP.double_poly(op, b, 3, 4)
    g1 = ctx.poly_from_roots(P1.roots)
    gi = ctx.poly_from_roots(D.inner.roots)
    gd = ctx.poly_from_roots(D.roots, inner=gi)
    for theta, th in (("I", 0), ("g5", 1)):
        X, _, mv = ctx.level(gd, g1, None, th, 5, 2, 7, N)
        Xr, _ = OES.level_samples(op, D, P1, None, theta, 5, 2, 7, N)
        assert rel(X, Xr) < 1e-10
        assert mv == N * (11 + 8)


def test_fused_level_fp32_bias_bound(f44):
    """FP32 fused steps: per-sample error bounded by the FP32 rounding of the
    recurrence (||eta||^2 * d * 1e-6 relative to the sample scale)."""
    dims, kappa, U, op, ctx = f44
    b = z4_noise(1, 0x100, 0, op.n)
    P1, _, _ = OK.gmres_poly(op, b, 17)
    g1 = ctx.poly_from_roots(P1.roots)
    N = 64
    X, _, _ = ctx.level(g1, None, None, 0, 9, 0, 0, N, prec=FP32)
    Xr, _ = OES.level_samples(op, P1, None, None, "I", 9, 0, 0, N)
    assert np.max(np.abs(X - Xr)) < op.n * 17 * 1e-6


def test_apply_poly_fp32_ignores_garbage_output(f44):
    """Regression: the output buffer's old contents (here NaN) never leak in."""
    dims, kappa, U, op, ctx = f44
    ref, _, _ = OK.gmres_poly(op, z4_noise(1, 0x100, 0, op.n), 9)
    P = ctx.poly_from_roots(ref.roots)
    N = 128
    eta = ctx.noise(4, 1, 0, N, FP32)
    y = ctx.vector(N, FP32)
    y.view(torch.float32).fill_(float("nan"))
    ctx.apply_poly(P, eta, N, FP32, out=y)
    got = host(ctx.unpack(y, N, FP32))
    assert np.all(np.isfinite(got))
    want = np.stack([OP.apply_p(op, ref.roots, e) for e in z4_noise_batch(4, 1, 0, 2, op.n)])
    assert rel(got[:2], want) < 2e-5


@pytest.mark.parametrize("prec,tol", [(FP64, 1e-12), (FP32, 2e-5)])
def test_apply_poly_single_vector_ignores_garbage_output(f44, prec, tol):
    """Regression: a single vector's accumulator starts inside the first Wilson
    launch, which never reads the output's old contents (here NaN); a degree-1
    polynomial (no Wilson launch) still gives x / theta_1."""
    dims, kappa, U, op, ctx = f44
    ref, _, _ = OK.gmres_poly(op, z4_noise(1, 0x100, 0, op.n), 9)
    x = ctx.noise(6, 3, 0, 1, prec)
    xh = z4_noise(6, 3, 0, op.n)
    for roots in (ref.roots, np.array([2.0 + 0.5j])):
        P = ctx.poly_from_roots(roots)
        y = ctx.vector(1, prec)
        y.view(torch.float64 if prec == FP64 else torch.float32).fill_(float("nan"))
        ctx.apply_poly(P, x, 1, prec, out=y)
        got = host(ctx.unpack(y, 1, prec))[0]
        assert np.all(np.isfinite(got))
        assert rel(got, OP.apply_p(op, roots, xh)) < tol


# ---------------------------------------------------------------- probing --

def test_poly_trace_probing_exact(f44):
    """Exact Tr(Theta p(M)) by probing against the oracle's dense trace:
    brute force (every site its own colour) for degree 15, and a 2x2x2x2 block
    colouring for degree 1 (exact since 1 < 2 <= L/2)."""
    dims, kappa, U, op, ctx = f44
    b = z4_noise(1, 0x100, 0, op.n)
    P, _, _ = OK.gmres_poly(op, b, 16)
    Pm = OP.apply_p(op, P.roots, np.eye(op.n)).T
    g = ctx.poly_from_roots(P.roots)
    for theta, th in (("I", 0), ("g5", 1)):
        G = np.kron(np.eye(OLT.volume(dims)), np.kron(OLT.theta_matrix(theta), np.eye(3)))
        tr, exact, mv = ctx.poly_trace(g, theta=th, max_batch=192)
        assert exact and mv == op.n * 15
        assert abs(tr - np.trace(G @ Pm)) < 1e-10 * max(1.0, abs(np.trace(G @ Pm)))
    P2, _, _ = OK.gmres_poly(op, b, 2)
    P2m = OP.apply_p(op, P2.roots, np.eye(op.n)).T
    tr2, exact2, mv2 = ctx.poly_trace(ctx.poly_from_roots(P2.roots), period=(2, 2, 2, 2))
    assert exact2 and mv2 == 16 * 12 * 1
    assert abs(tr2 - np.trace(P2m)) < 1e-10 * abs(np.trace(P2m))
    # a too-coarse colouring is reported as inexact
    _, exact3, _ = ctx.poly_trace(g, period=(2, 2, 2, 2))
    assert not exact3


@pytest.mark.parametrize("d", [4, 9])
def test_poly_trace_distance_colouring_exact(f44, d):
    """Exact Tr(Theta p(M)) with the distance-(deg + 1) colouring (Sec. 6)
    against the oracle's dense trace, FP64 and FP32 (FP64 sums)."""
    dims, kappa, U, op, ctx = f44
    P, _, _ = OK.gmres_poly(op, z4_noise(1, 0x100, 0, op.n), d)
    Pm = OP.apply_p(op, P.roots, np.eye(op.n)).T
    g = ctx.poly_from_roots(P.roots)
    k, m, W, nc = mpmc.mpmc_probe_colouring(dims, d - 1)
    for theta, th in (("I", 0), ("g5", 1)):
        G = np.kron(np.eye(OLT.volume(dims)), np.kron(OLT.theta_matrix(theta), np.eye(3)))
        ref = np.trace(G @ Pm)
        tr, nprobe, mv = ctx.poly_trace_probe(g, theta=th, prec=FP64, max_batch=96)
        assert nprobe == 12 * nc and mv == nprobe * (d - 1)
        assert abs(tr - ref) < 1e-10 * max(1.0, abs(ref))
        tr32, _, _ = ctx.poly_trace_probe(g, theta=th, prec=FP32)
        assert abs(tr32 - ref) < 1e-5 * max(1.0, abs(ref))


@pytest.mark.parametrize("d", [5, 9])
def test_poly_trace_probe_vs_sampled_8x4(d):
    """8^4, degrees 4 and 8: the probed trace agrees with a 256-noise
    Hutchinson estimate of the same term within 3.5 standard errors.  Degree
    4 takes a 64-colour code (768 probes); for degree 8 the 8^4 torus admits
    no code of at most 512 colours, so every site is its own colour."""
    dims, kappa = (8, 8, 8, 8), 0.12
    U = inputs.gauge_links(dims, 0.5, seed=2)
    ctx = mpmc.Context(dims, kappa, U)
    g = ctx.gmres_poly(2, 0x103, d)
    tr, nprobe, mv = ctx.poly_trace_probe(g, prec=FP32)
    X, T, _ = ctx.level(g, None, None, 0, 2, 3, 0, 256, prec=FP64)
    m, v = OES.level_stats(X)
    assert abs(tr - m) < 3.5 * np.sqrt(v / 256)
    k, mods, W, nc = mpmc.mpmc_probe_colouring(dims, d - 1)
    assert nprobe == 12 * nc and mv == nprobe * (d - 1)
    if d == 5:
        assert nc == 64


# ------------------------------------------------------------- autotuner --

@pytest.mark.parametrize("prec", [FP64, FP32, FP16S])
def test_autotune_variants_bit_identical(f44, prec):
    """every kernel variant (occupancy target, traversal order) gives the same
    bits; the autotuner picks one of them and reports a time for each"""
    dims, kappa, U, op, ctx = f44
    N = 128
    x = ctx.noise(4, 1, 0, N, prec)
    outs = []
    for v in range(mpmc.WILSON_VARIANTS):
        ctx.tune_set(N, prec, v)
        outs.append(host(ctx.apply_M(x, N, prec)).copy())
    ctx.tune_set(N, prec, -1)
    for o in outs[1:]:
        assert np.array_equal(o, outs[0])
    v, us = ctx.autotune(N, prec)
    tried = us > 0   # variants that fall back to another one on this shape are not timed
    assert 0 <= v < mpmc.WILSON_VARIANTS and tried[v] and us[v] == us[tried].min()
    assert tried.sum() >= 10 - 2 * (prec != FP32)   # the column kernels are FP32 only
    assert np.array_equal(host(ctx.apply_M(x, N, prec)), outs[0])
    ctx.tune_set(N, prec, -1)
    assert ctx.autotune(20, prec)[0] == -1     # not a multiple of 64: nothing to tune


@pytest.mark.parametrize("prec,variants", [(FP32, (1, 3, 5, 7, 9, 10, 11, 12)), (FP64, (0, 2, 4, 6, 8))])
def test_fused_level_step_traversals(f44, prec, variants):
    """The fused level step under each traversal (site-major, chunk-major,
    4D-blocked with 64-, 16- and 32-wide chunks and their per-chunk
    reductions): per-element arithmetic is the
    same, so the samples differ only by the order of the FP64 sums; two
    samples are recomputed by the oracle."""
    dims, kappa, U, op, ctx = f44
    P1, _, _ = OK.gmres_poly(op, z4_noise(1, 0x100, 0, op.n), 17)
    g1 = ctx.poly_from_roots(P1.roots)
    N = 128
    outs = []
    for v in variants:
        ctx.tune_set(N, prec, v)
        X, T, mv = ctx.level(g1, None, None, 0, 5, 1, 0, N, prec=prec)
        assert T == 0 and mv == N * 16
        outs.append(X)
    ctx.tune_set(N, prec, -1)
    for X in outs[1:]:
        assert rel(X, outs[0]) < 1e-13
    Xr, _ = OES.level_samples(op, P1, None, None, "I", 5, 1, 0, 2)
    for j in range(2):
        if prec == FP64:
            assert abs(outs[-1][j] - Xr[j]) < 1e-10 * abs(Xr[j])
        else:   # FP32 kernels, FP64 sums: ~1e-6 n (bound 1e-5 n)
            assert abs(outs[-1][j] - Xr[j]) < 1e-5 * op.n


@pytest.mark.parametrize("prec", [FP32, FP64])
def test_autotune_level_orders(prec):
    """mpmc_autotune_level times every traversal valid for the shape (the three
    column kernels only in FP32), keeps the fastest, reports a time per order,
    and the level estimate after it gives the default traversal's samples up
    to the grouping of the FP64 sums."""
    dims, kappa = (4, 4, 4, 4), 0.115
    U = inputs.gauge_links(dims, 0.5, seed=1)
    ctx = mpmc.Context(dims, kappa, U)
    N = 128
    P = ctx.poly_from_roots(np.array([1.0 + 0.1j * k for k in range(7)]))
    X0 = ctx.level(P, None, None, 0, 5, 1, 0, N, prec=prec)[0]
    order, us = ctx.autotune_level(N, prec)
    assert us.shape == (8,)
    tried = us > 0
    assert tried[order] and us[order] == us[tried].min()
    expect = {0, 2, 3, 4} | ({5, 6, 7} if prec == FP32 else set())
    assert set(np.flatnonzero(tried)) == expect
    X1 = ctx.level(P, None, None, 0, 5, 1, 0, N, prec=prec)[0]
    assert rel(X1, X0) < 1e-13
    with pytest.raises(mpmc.MpmcError):
        ctx.autotune_level(96, prec)   # not a multiple of 64


@pytest.mark.parametrize("dims", [(8, 12, 8, 6), (6, 4, 12, 4)])
def test_column_pair_kernel_matches_column(dims):
    """The column kernel with 2x2x4 tiles and 32-wide chunks (two sites per
    wavefront, links broadcast within 16-lane rows; variant 12) against the
    2x2x2-tile one (variant 10) on lattices whose block grid is ragged: M, M^H
    and gamma5 M bit for bit; the fused steps of a single and of a double
    polynomial (combining steps) up to the grouping of the FP64 sums; two
    samples against the oracle."""
    kappa = 0.12
    U = inputs.gauge_links(dims, 0.5, seed=6)
    op, ctx = WilsonOp(dims, kappa, U), mpmc.Context(dims, kappa, U)
    N = 128
    x = ctx.noise(7, 1, 0, N, FP32)
    for dagger, theta in ((False, 0), (True, 0), (False, 1)):
        out = {}
        for v in (10, 12):
            ctx.tune_set(N, FP32, v)
            out[v] = ctx.apply_M(x, N, FP32, dagger=dagger, theta=theta)
        ctx.tune_set(N, FP32, -1)
        assert torch.equal(out[10], out[12]), (dagger, theta)
    P1, _, _ = OK.gmres_poly(op, z4_noise(1, 0x100, 0, op.n), 9)
    g1 = ctx.poly_from_roots(P1.roots)
    inner = ctx.gmres_poly(1, 0x101, 3)
    dp = ctx.gmres_poly(1, 0x102, 4, inner=inner)
    for P in (g1, dp):
        X = {}
        for v in (10, 12):
            ctx.tune_set(N, FP32, v)
            X[v], T, mv = ctx.level(P, None, None, 0, 5, 1, 0, N, prec=FP32)
        ctx.tune_set(N, FP32, -1)
        assert rel(X[12], X[10]) < 1e-13
        if P is g1:
            Xr, _ = OES.level_samples(op, P1, None, None, "I", 5, 1, 0, 2)
            for j in range(2):   # FP32 kernels, FP64 sums
                assert abs(X[12][j] - Xr[j]) < 1e-5 * op.n


@pytest.mark.parametrize("prec,variant", [(FP32, 5), (FP64, 4)])
def test_apply_batch_matches_single(prec, variant):
    """Uneven lattices in one batched launch: every lattice's result is
    bit-identical to its own launch of the same traversal, and one of them is
    checked against the oracle operator."""
    shapes = [((4, 4, 4, 4), 0.115, 1), ((4, 4, 4, 8), 0.12, 2), ((6, 6, 6, 6), 0.11, 3), ((2, 4, 6, 8), 0.1, 4)]
    N = 64
    ctxs, xs, refs = [], [], []
    for dims, kappa, seed in shapes:
        U = inputs.gauge_links(dims, 0.5, seed=seed)
        c = mpmc.Context(dims, kappa, U)
        x = c.noise(seed, 3, 0, N, prec)
        c.tune_set(N, prec, variant)
        refs.append(host(c.apply_M(x, N, prec)).copy())
        ctxs.append(c)
        xs.append(x)
    mv0 = [c.mvps for c in ctxs]
    ys = mpmc.Context.apply_M_batch(ctxs, xs, N, prec)
    for c, y, ref, m0 in zip(ctxs, ys, refs, mv0):
        assert np.array_equal(host(y), ref)
        assert c.mvps == m0 + N
    dims, kappa, seed = shapes[2]
    op = WilsonOp(dims, kappa, inputs.gauge_links(dims, 0.5, seed=seed))
    got = host(ctxs[2].unpack(ys[2], N, prec))
    want = op(z4_noise(seed, 3, 17, op.n))
    assert rel(got[17], want) < (1e-13 if prec == FP64 else 1e-6)
    with pytest.raises(mpmc.MpmcError):
        mpmc.Context.apply_M_batch(ctxs, xs, 20, prec)
    with pytest.raises(mpmc.MpmcError):
        mpmc.Context.apply_M_batch(ctxs * 3, xs * 3, N, prec)


def test_timing_counts_single_vectors_without_events(f44):
    """Launch timing: multi-RHS launches carry event times, single-vector
    launches are counted with their algorithmic bytes only."""
    dims, kappa, U, op, ctx = f44
    V = op.n // 12
    x1, x64 = ctx.noise(3, 0, 0, 1, FP64), ctx.noise(3, 0, 0, 64, FP64)
    mpmc.mpmc_timing_enable(ctx.handle, 1)
    ctx.apply_M(x1, 1, FP64)
    ctx.apply_M(x64, 64, FP64)
    n1, ms1, b1 = mpmc.mpmc_timing_read(ctx.handle, FP64 | mpmc.TIMING_SINGLE)
    n64, ms64, b64 = mpmc.mpmc_timing_read(ctx.handle, FP64 | mpmc.TIMING_PLAIN)
    na, msa, ba = mpmc.mpmc_timing_read(ctx.handle, FP64)
    mpmc.mpmc_timing_enable(ctx.handle, 0)
    assert (n1, ms1, b1) == (1, 0.0, V * (2 * 192.0 + 576.0))
    assert n64 == 1 and ms64 > 0 and b64 == V * (64 * 2 * 192.0 + 576.0)
    assert (na, msa, ba) == (2, ms64, b1 + b64)


@pytest.mark.parametrize("N", [64, 20])
def test_solve_fp16_basis_matches_fp32(N):
    """FP16S Krylov basis (FP32 arithmetic, FP64 defect correction): same true
    residual bound and the same solution as the FP32-basis solve."""
    dims, kappa = (8, 8, 8, 8), 0.120
    U = inputs.gauge_links(dims, 0.5, seed=2)
    ctx = mpmc.Context(dims, kappa, U)
    op = WilsonOp(dims, kappa, U)
    b = ctx.noise(6, 0, 0, N, FP64)
    x16, it16, rr16 = ctx.solve(b, N, restart=50, tol=1e-9, inner_prec=FP16S)
    x32, it32, rr32 = ctx.solve(b, N, restart=50, tol=1e-9, inner_prec=FP32)
    assert np.all(rr16 <= 1e-9) and np.all(rr32 <= 1e-9)
    X16, X32 = host(ctx.unpack(x16, N)), host(ctx.unpack(x32, N))
    assert rel(X16, X32) < 5e-9
    j = N - 1
    bj = z4_noise(6, 0, j, op.n)
    assert np.linalg.norm(bj - op(X16[j])) / np.linalg.norm(bj) <= 1.05e-9


@pytest.mark.parametrize("inner", [FP64, FP32, FP16S])
def test_solve_gram_schmidt_passes(inner):
    """One or two classical projections per inner GMRES step: both reach the
    true FP64 residual (checked under the oracle operator on a sampled
    right-hand side) and the same solution; one projection costs at most one
    more 10-step convergence check of inner iterations; the default (0) is one
    projection for FP32/FP16S inner cycles and two for FP64."""
    dims, kappa = (8, 8, 8, 8), 0.120
    U = inputs.gauge_links(dims, 0.5, seed=2)
    ctx = mpmc.Context(dims, kappa, U)
    op = WilsonOp(dims, kappa, U)
    N, tol = 20, 1e-9
    b = ctx.noise(9, 0, 0, N, FP64)
    out = {}
    for passes in (2, 1, 0):
        ctx.set_solve_gs_passes(passes)
        out[passes] = ctx.solve(b, N, restart=50, tol=tol, inner_prec=inner)
    X = {p: host(ctx.unpack(x, N)) for p, (x, _, _) in out.items()}
    for p in (1, 2):
        assert np.all(out[p][2] <= tol)
        bj = z4_noise(9, 0, 11, op.n)
        assert np.linalg.norm(bj - op(X[p][11])) / np.linalg.norm(bj) <= 1.05 * tol
    assert rel(X[1], X[2]) < 5 * tol
    assert out[1][1] <= out[2][1] + 10
    dflt = 2 if inner == FP64 else 1
    assert out[0][1] == out[dflt][1] and torch.equal(out[0][0], out[dflt][0])
    with pytest.raises(mpmc.MpmcError):
        ctx.set_solve_gs_passes(3)


# ------------------------------------------------- PP-GMRES main solves --

@pytest.mark.parametrize("inner", [FP64, FP32, FP16S])
def test_pp_solve_matches_plain_solve(inner):
    """GMRES on M p(M) (right-preconditioned, correction p(M) V y) reaches the
    same true FP64 residual and solution, in fewer inner iterations."""
    dims, kappa = (8, 8, 8, 8), 0.120
    U = inputs.gauge_links(dims, 0.5, seed=2)
    ctx = mpmc.Context(dims, kappa, U)
    op = WilsonOp(dims, kappa, U)
    N = 20
    pp = ctx.gmres_poly(2, 0x1FF, 9)
    b = ctx.noise(8, 0, 0, N, FP64)
    x0, it0, r0 = ctx.solve(b, N, restart=50, tol=1e-9, inner_prec=inner)
    x1, it1, r1 = ctx.solve_pp(b, N, pp, restart=50, tol=1e-9, inner_prec=inner)
    assert np.all(r0 <= 1e-9) and np.all(r1 <= 1e-9)
    X0, X1 = host(ctx.unpack(x0, N)), host(ctx.unpack(x1, N))
    assert rel(X1, X0) < 5e-9
    assert it1 < it0
    bj = z4_noise(8, 0, 7, op.n)
    assert np.linalg.norm(bj - op(X1[7])) / np.linalg.norm(bj) <= 1.05e-9


def test_level_with_pp_solves_unchanged(f44):
    dims, kappa, U, op, ctx = f44
    p = ctx.gmres_poly(1, 0x100, 9)
    pp = ctx.gmres_poly(1, 0x1FF, 5)
    X0, c0, m0 = ctx.level(None, p, None, mpmc.THETA_I, 3, 0, 0, 12, prec=FP64, solve_tol=1e-11)
    ctx.set_level_solve_poly(pp)
    try:
        X1, c1, m1 = ctx.level(None, p, None, mpmc.THETA_I, 3, 0, 0, 12, prec=FP64, solve_tol=1e-11)
    finally:
        ctx.set_level_solve_poly(None)
    assert np.max(np.abs(X1 - X0)) < 1e-9 * op.n


# ---------------------------------------------------------- added roots --

def test_add_roots_matches_oracle_synthetic(f44):
    dims, kappa, U, op, ctx = f44
    ring = 1.0 + 0.5 * np.exp(2j * np.pi * (np.arange(20) + 0.25) / 20)
    th = OK.leja_order(np.concatenate([ring, [50.0, 0.02 + 0.01j]]))
    P = ctx.poly_from_roots(th)
    added = P.add_roots()
    ref, radded = OK.add_roots(th)
    assert added == radded > 0
    assert np.allclose(P.roots, ref, rtol=0, atol=1e-12)
    assert P.info["degree"] == len(ref) - 1


def test_add_roots_high_degree_gmres_poly():
    """A GMRES(200) polynomial on the 8^4 field: the device rule matches the
    oracle's on the same roots, and the stabilised p still satisfies
    pi = 1 - M p on a vector (FP64)."""
    dims, kappa = (8, 8, 8, 8), 0.120
    U = inputs.gauge_links(dims, 0.5, seed=2)
    ctx = mpmc.Context(dims, kappa, U)
    op = WilsonOp(dims, kappa, U)
    P = ctx.gmres_poly(2, 0x105, 200)
    th = P.roots.copy()
    added = P.add_roots()
    ref, radded = OK.add_roots(th)
    assert added == radded
    assert _match_sets(P.roots, ref) < 1e-10 * np.abs(ref).max() and len(P.roots) == len(ref)
    assert np.allclose(P.roots, ref, rtol=0, atol=1e-10 * np.abs(ref).max())
    x = ctx.noise(3, 2, 0, 1, FP64)
    y = host(ctx.unpack(ctx.apply_poly(P, x, 1, FP64), 1))[0]
    xh = z4_noise(3, 2, 0, op.n)
    pi_ref = OP.apply_pi(op, ref, xh)
    assert rel(xh - op(y), pi_ref) < 1e-8 * max(1.0, np.linalg.norm(xh) / max(np.linalg.norm(pi_ref), 1e-300))


# ---------------------------------------------- deflated double polynomial --

@pytest.fixture(scope="module")
def f44c():
    """4^4 field at kappa 0.2 (small eigenvalues) with an oracle deflation set
    imported to the GPU."""
    dims, kappa = (4, 4, 4, 4), 0.2
    U = inputs.gauge_links(dims, 0.5, seed=21)
    op, ctx = WilsonOp(dims, kappa, U), mpmc.Context(dims, kappa, U)
    Pin4, _, _ = OK.gmres_poly(op, z4_noise(1, 0x1FF, 0, op.n), 5)
    Dref, _ = ODF.pp_arnoldi_eigs(op, Pin4.roots, z4_noise(1, 0x200, 0, op.n), 80, 12)
    assert Dref.k >= 6
    D = ctx.defl_from_arrays(Dref.lam, torch.from_numpy(Dref.Z).cuda(), torch.from_numpy(Dref.U).cuda())
    return op, ctx, Dref, D


@pytest.mark.parametrize("cgs2", [-1, 0])
@pytest.mark.parametrize("din,dout", [(5, 4), (16, 16)])
def test_deflated_double_poly_parity(f44c, din, dout, cgs2):
    """mpmc_gmres_poly(inner, defl) (Sec. 7: the deflated double polynomial)
    against the oracle's projected outer cycle on Q phi_in from Q b, with the
    same imported deflation set: inner and outer roots, relres, and the
    GMRES residual identity under the oracle operator with the GPU's roots;
    with the default Gram-Schmidt of this size (plain CGS2) and the delayed one."""
    op, ctx, Dref, D = f44c
    b = z4_noise(1, 0x100, 0, op.n)
    Q = OP.projector(Dref.Z, Dref.U)
    ref, (di, do), (ri, ro) = OP.double_poly(op, b, din, dout, proj=Q)
    ctx.set_arnoldi_cgs2(cgs2)
    try:
        Pin = ctx.gmres_poly(1, 0x100, din)
        Pd = ctx.gmres_poly(1, 0x100, dout, inner=Pin, defl=D)
        Pu = ctx.gmres_poly(1, 0x100, dout, inner=Pin)
    finally:
        ctx.set_arnoldi_cgs2(-1)
    assert Pd.d_eff == do == dout
    scale = np.max(np.abs(ref.roots))
    assert _match_sets(Pin.roots, ref.inner.roots) < 1e-9 * np.max(np.abs(ref.inner.roots))
    assert _match_sets(Pd.roots, ref.roots) < 1e-8 * scale
    assert abs(Pd.relres - ro) < 1e-8 * ro
    assert Pd.info["degree"] == din * dout - 1
    # with the GPU's own roots: ||pi_out(Q phi_in) Q b|| / ||Q b|| is the reported relres
    phi = OP.phi(op, Pin.roots)
    c = Q(b)
    r = OP.apply_pi(lambda v: Q(phi(v)), Pd.roots, c)
    assert abs(np.linalg.norm(r) / np.linalg.norm(c) - Pd.relres) < 1e-9 * Pd.relres
    # the undeflated outer cycle is a different polynomial
    assert _match_sets(Pu.roots, Pd.roots) > 1e-6 * scale


def test_deflated_solve_level_parity(f44c):
    """Solve level with mpmc_set_solve_level_deflation(1): per-sample values
    and the exact correction against the oracle's deflated solve level, for a
    deflated double polynomial p_1 (imported roots), Theta = I and g5."""
    op, ctx, Dref, D = f44c
    b = z4_noise(1, 0x100, 0, op.n)
    ref, _, _ = OP.double_poly(op, b, 5, 4, proj=OP.projector(Dref.Z, Dref.U))
    gi = ctx.poly_from_roots(ref.inner.roots)
    gd = ctx.poly_from_roots(ref.roots, inner=gi)
    N = 6
    ctx.set_solve_level_deflation(1)
    try:
        for theta, th in (("I", 0), ("g5", 1)):
            X, T, _ = ctx.level(None, gd, D, th, 3, 0, 0, N, solve_tol=1e-12, solve_restart=30)
            Xr, Tr = OES.level_samples(op, None, ref, Dref, theta, 3, 0, 0, N, solve_tol=1e-12, deflate_solve=True)
            # solves to 1e-12 on both sides: |eta^H (x - x*)| <= n ||M^-1|| 1e-12 per
            # side, ||M^-1|| = 11.3 on this field (smallest singular value, dense)
            assert np.max(np.abs(X - Xr)) < 2 * op.n * 12 * 1e-12
            assert abs(T - Tr) < 1e-10 * max(1, abs(Tr))
            assert abs(Tr) > 0
    finally:
        ctx.set_solve_level_deflation(0)
    X0, T0, _ = ctx.level(None, gd, D, 0, 3, 0, 0, N, solve_tol=1e-12, solve_restart=30)
    assert T0 == 0
    with pytest.raises(mpmc.MpmcError):
        ctx.set_solve_level_deflation(2)


# ------------------------------------------- set-up Gram-Schmidt variants --

@pytest.mark.parametrize("prec,tol", [(FP64, 1e-9), (FP32, 1e-4)])
def test_delayed_and_plain_cgs2_agree(f44, prec, tol):
    """The set-up Arnoldi with the second projection delayed by one step (the
    default) and with plain CGS2: the same GMRES roots and relres and the same
    deflation eigenvalues, to rounding of the storage precision (both forms are
    held to the oracle by the other tests, which run the default)."""
    dims, kappa, U, op, ctx = f44
    ctx.set_setup_precision(prec)
    out = []
    try:
        for cgs2 in (1, 0):
            ctx.set_arnoldi_cgs2(cgs2)
            P = ctx.gmres_poly(1, 0x100, 16)
            Pin = ctx.gmres_poly(1, 0x1FF, 5)
            D = ctx.deflate(Pin, 1, 0x200, m=60, nev=8)
            lam, _, _ = ctx.defl_vectors(D)
            out.append((P, np.asarray(lam)[:D.k], D.k))
    finally:
        ctx.set_arnoldi_cgs2(-1)
        ctx.set_setup_precision(FP64)
    (P1, l1, k1), (P0, l0, k0) = out
    assert P0.d_eff == P1.d_eff == 16
    assert _match_sets(P0.roots, P1.roots) < tol * np.max(np.abs(P1.roots))
    assert abs(P0.relres - P1.relres) < tol * P1.relres
    assert k0 == k1 >= 1 and _match_sets(l0, l1) < tol * np.max(np.abs(l1))
    with pytest.raises(mpmc.MpmcError):
        ctx.set_arnoldi_cgs2(2)


@pytest.mark.parametrize("cgs2", [0, 1])
@pytest.mark.parametrize("kappa,seed,d", [(0.115, 1, 9), (0.2, 21, 48)])
def test_delayed_cgs2_roots_parity(cgs2, kappa, seed, d):
    """GMRES(d) roots and relres of both Gram-Schmidt forms against the oracle
    (plain CGS2) on the same Z(4) start vector (kappa 0.2: slow convergence,
    many steps); the kappa = 0 breakdown gives d_eff = 1 in both forms."""
    dims = (4, 4, 4, 4)
    U = inputs.gauge_links(dims, 0.5, seed=seed)
    op, ctx = WilsonOp(dims, kappa, U), mpmc.Context(dims, kappa, U)
    ctx.set_arnoldi_cgs2(cgs2)
    P = ctx.gmres_poly(1, 0x100, d)
    ref, de, rr = OK.gmres_poly(op, z4_noise(1, 0x100, 0, op.n), d)
    assert P.d_eff == de == d
    assert _match_sets(P.roots, ref.roots) < 1e-8 * np.max(np.abs(ref.roots))
    assert abs(P.relres - rr) < 1e-8 * rr
    c0 = mpmc.Context((2, 2, 2, 2), 0.0, inputs.gauge_links((2, 2, 2, 2), 0.5, seed=1))
    c0.set_arnoldi_cgs2(cgs2)
    P0 = c0.gmres_poly(1, 0x100, 16)
    assert P0.d_eff == 1 and np.allclose(P0.roots, [1.0])


# ------------------------------------------------- FP32 setup precision --

def test_fp32_setup_polynomials_and_deflation():
    """mpmc_set_setup_precision(FP32): Arnoldi vectors in FP32, every scalar
    in FP64.  The GMRES polynomial's roots stay within FP32 rounding of the
    FP64 ones, its relres is the residual of its own roots under the oracle
    operator, and the deflation set passes the same acceptance test with
    eigenvalues matching the FP64 build."""
    dims, kappa = (4, 4, 4, 4), 0.2
    U = inputs.gauge_links(dims, 0.5, seed=21)
    op, ctx = WilsonOp(dims, kappa, U), mpmc.Context(dims, kappa, U)
    b = z4_noise(1, 0x100, 0, op.n)
    P64 = ctx.gmres_poly(1, 0x100, 12)
    Pin = ctx.gmres_poly(1, 0x100, 5)   # FP64 p_in for both deflation builds
    ctx.set_setup_precision(FP32)
    try:
        P32 = ctx.gmres_poly(1, 0x100, 12)
        assert P32.d_eff == 12
        assert _match_sets(P32.roots, P64.roots) < 1e-4 * np.max(np.abs(P64.roots))
        r = OP.apply_pi(op, P32.roots, b)
        assert abs(np.linalg.norm(r) / np.linalg.norm(b) - P32.relres) < 1e-4 * P32.relres + 1e-7
        # m = 120: ten pairs converged far below the 1e-3 acceptance (oracle: residuals <= 2e-7)
        D32 = ctx.deflate(Pin, 1, 0x200, m=120, nev=10)
        lam32, Z32, U32 = ctx.defl_vectors(D32)
    finally:
        ctx.set_setup_precision(FP64)
    D64 = ctx.deflate(Pin, 1, 0x200, m=120, nev=10)
    lam64, _, _ = ctx.defl_vectors(D64)
    assert D32.k >= 8 and abs(D32.k - D64.k) <= 1
    assert _match_sets(lam32, lam64) < 1e-5
    Zh, Uh = Z32.cpu().numpy(), U32.cpu().numpy()
    for i in range(D32.k):
        assert abs(np.vdot(Uh[i], Zh[i]) - 1) < 1e-10
        assert np.linalg.norm(op(Zh[i]) - lam32[i] * Zh[i]) < 1e-3
    with pytest.raises(mpmc.MpmcError):
        ctx.set_setup_precision(FP16S)


# ------------------------------------------------ captured recurrences --

@pytest.mark.parametrize("prec", [FP64, FP32])
def test_graph_recurrences_bit_identical(prec):
    """mpmc_set_graph_recurrences: the fused recurrences of the polynomial
    levels (single and double polynomials, deflated level) replayed from
    captured hipGraphs give the samples of the launches run one by one, bit
    for bit, on every one of several replays with unrelated eager work and
    synchronisations in between, and again after the workspace is released."""
    dims, kappa = (4, 4, 4, 4), 0.115
    U = inputs.gauge_links(dims, 0.5, seed=1)
    op, ctx = WilsonOp(dims, kappa, U), mpmc.Context(dims, kappa, U)
    b = z4_noise(1, 0x100, 0, op.n)
    P1, _, _ = OK.gmres_poly(op, b, 9)
    Dp, _, _ = OP.double_poly(op, b, 3, 4)
    Pin, _, _ = OK.gmres_poly(op, b, 4)
    Dref, _ = ODF.pp_arnoldi_eigs(op, Pin.roots, z4_noise(1, 0x200, 0, op.n), 60, 8)
    D = ctx.defl_from_arrays(Dref.lam, torch.from_numpy(Dref.Z).cuda(), torch.from_numpy(Dref.U).cuda())
    g1 = ctx.poly_from_roots(P1.roots)
    gd = ctx.poly_from_roots(Dp.roots, inner=ctx.poly_from_roots(Dp.inner.roots))
    N = 64
    cases = [(gd, g1, D), (g1, None, None)]
    want = [ctx.level(u, l, d, 1, 5, 2, 0, N, prec=prec) for u, l, d in cases]
    ctx.set_graph_recurrences(1)
    try:
        for rep in range(4):
            for (u, l, d), (Xw, Tw, mw) in zip(cases, want):
                X, T, mv = ctx.level(u, l, d, 1, 5, 2, 0, N, prec=prec)
                assert np.array_equal(X, Xw) and T == Tw and mv == mw, rep
            y = ctx.apply_M(ctx.noise(3, 0, 0, 8, prec), 8, prec)          # eager work in between
            float(torch.sum(y.view(torch.float32)).item())
            if rep == 1:
                ctx.release_workspace()
                assert mpmc.mpmc_graph_replays(ctx.handle)[1] == 0
        replays, graphs = mpmc.mpmc_graph_replays(ctx.handle)
        assert replays >= 6 and graphs >= 1
    finally:
        ctx.set_graph_recurrences(0)
    X, _, _ = ctx.level(g1, None, None, 1, 5, 2, 0, N, prec=prec)
    assert np.array_equal(X, want[1][0])
