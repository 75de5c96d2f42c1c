"""GPU: solves of several uneven lattices in lockstep (mpmc_solve_batch, one
batched Wilson launch per inner iteration) give, lattice by lattice, the same
iterates and iteration counts as each lattice's own mpmc_solve, with and
without deflation sets and a learned preconditioner; the solutions meet the
tolerance under the oracle operator."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from oracle.philox import z4_noise_batch  # noqa: E402
from oracle.wilson import WilsonOp  # noqa: E402
from paper_2402_00016_amd import driver, inputs, mpmc  # noqa: E402

FP64, FP32 = mpmc.FP64, mpmc.FP32
SPECS = [((4, 4, 4, 4), 0.115, 1), ((4, 4, 6, 6), 0.12, 2), ((8, 8, 8, 8), 0.12, 3)]


@pytest.fixture(scope="module")
def lattices():
    ctxs = [mpmc.Context(d, k, inputs.gauge_links(d, 0.5, seed=s)) for d, k, s in SPECS]
    D = [ctxs[0].deflate(ctxs[0].gmres_poly(1, 0x1FF, 5), 1, 0x200, m=60, nev=8), None, None]
    assert D[0].k >= 1
    return ctxs, D


@pytest.mark.parametrize("prec", [FP64, FP32])
def test_solve_batch_equals_single_solves(lattices, prec):
    ctxs, D = lattices
    N, tol = 64, 1e-9
    bs = [c.noise(5, 1, 0, N, FP64) for c in ctxs]
    single = [c.solve(b, N, defl=d, restart=20, tol=tol, inner_prec=prec) for c, b, d in zip(ctxs, bs, D)]
    xs, its, rel = mpmc.Context.solve_batch(ctxs, bs, N, defls=D, restart=20, tol=tol, inner_prec=prec)
    for i, (x, it, r) in enumerate(single):
        assert its[i] == it, i
        assert torch.equal(xs[i], x), i
        assert np.array_equal(rel[i], r)
        assert np.all(rel[i] <= tol)
    # the first lattice's solutions under the oracle operator
    dims, kappa, seed = SPECS[0]
    op = WilsonOp(dims, kappa, inputs.gauge_links(dims, 0.5, seed=seed))
    X = ctxs[0].unpack(xs[0], N).cpu().numpy()
    B = z4_noise_batch(5, 1, 0, N, op.n)
    assert np.all(np.linalg.norm(B - op(X), axis=1) / np.linalg.norm(B, axis=1) <= 1.05 * tol)


def test_solve_batch_with_network(lattices):
    """A learned preconditioner on one lattice (FP32 inner cycles, flexible
    GMRES): that lattice's iterates equal its own solve with the same network;
    the others are unchanged by its presence."""
    ctxs, D = lattices
    N, tol = 64, 1e-8
    rng = np.random.default_rng(7)
    net = ctxs[2].net(driver.net_identity_weights() + 0.01 * rng.standard_normal(mpmc.mpmc_net_n_params()))
    nets = [None, None, net]
    bs = [c.noise(6, 2, 0, N, FP64) for c in ctxs]
    single = [c.solve(b, N, defl=d, restart=20, tol=tol, inner_prec=FP32, net=t)
              for c, b, d, t in zip(ctxs, bs, D, nets)]
    xs, its, rel = mpmc.Context.solve_batch(ctxs, bs, N, defls=D, nets=nets, restart=20, tol=tol, inner_prec=FP32)
    for i, (x, it, r) in enumerate(single):
        assert its[i] == it and torch.equal(xs[i], x), i


def test_solve_batch_rejects_bad_input(lattices):
    ctxs, D = lattices
    b = ctxs[0].noise(1, 0, 0, 64, FP64)
    with pytest.raises(mpmc.MpmcError):   # the same context twice
        mpmc.Context.solve_batch([ctxs[0], ctxs[0]], [b, b], 64)
    b32 = ctxs[0].noise(1, 0, 0, 32, FP64)
    with pytest.raises(mpmc.MpmcError):   # nrhs not a multiple of 64
        mpmc.Context.solve_batch([ctxs[0]], [b32], 32)
