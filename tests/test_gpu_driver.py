"""GPU: the host driver's estimate is the same whether the setup runs on one
stream or overlapped on side streams (same kernels, same inputs), and the
learned form gives the same estimate as the plain form to solver accuracy."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2402_00016_amd import driver, inputs, mpmc  # noqa: E402


@pytest.fixture(scope="module")
def ctx():
    dims, kappa = (4, 4, 4, 4), 0.115
    return mpmc.Context(dims, kappa, inputs.gauge_links(dims, 0.5, seed=1))


def plan(**kw):
    base = dict(degrees=[24, 8], noises=16, seed=3, nev=6, defl_candidates=12, defl_m=48, defl_pin_degree=4,
                solve_tol=1e-10)
    base.update(kw)
    return driver.Plan(**base)


def test_overlapped_setup_is_identical(ctx):
    e0 = driver.estimate(ctx, plan(overlap_setup=False), torch.cuda.synchronize)
    e1 = driver.estimate(ctx, plan(overlap_setup=True), torch.cuda.synchronize)
    for a, b in zip(e0.polys, e1.polys):
        assert np.array_equal(a.roots, b.roots)
    assert e0.defl_k == e1.defl_k
    for L0, L1 in zip(e0.levels, e1.levels):
        assert np.allclose(L0.samples, L1.samples, rtol=0, atol=1e-9)
    assert e0.mvps == e1.mvps


def test_overlapped_levels_same_samples(ctx):
    """Polynomial terms on a side stream while the solve term runs: every
    sample as with all terms on one stream."""
    e0 = driver.estimate(ctx, plan(overlap_levels=False), torch.cuda.synchronize)
    e1 = driver.estimate(ctx, plan(overlap_levels=True), torch.cuda.synchronize)
    assert [L.name for L in e0.levels] == [L.name for L in e1.levels]
    for L0, L1 in zip(e0.levels, e1.levels):
        assert np.array_equal(L0.samples, L1.samples) and L0.corr == L1.corr and L0.mvps == L1.mvps
    assert e0.value == e1.value and e0.mvps == e1.mvps


def test_batched_levels_same_estimate(ctx):
    """Polynomial terms in shared launches: the same samples bit for bit as the
    terms one at a time with the same (blocked 64-wide) traversal, so the same
    estimate."""
    ctx.tune_set(64, mpmc.FP32, 5)
    try:
        e0 = driver.estimate(ctx, plan(noises=64, batch_levels=False), torch.cuda.synchronize)
        e1 = driver.estimate(ctx, plan(noises=64, batch_levels=True), torch.cuda.synchronize)
    finally:
        ctx.tune_set(64, mpmc.FP32, -1)
    for L0, L1 in zip(e0.levels[1:], e1.levels[1:]):
        assert np.array_equal(L0.samples, L1.samples) and L0.corr == L1.corr
    assert np.allclose(e0.levels[0].samples, e1.levels[0].samples, rtol=0, atol=1e-9)
    assert abs(e0.value - e1.value) < 1e-8 and e0.mvps == e1.mvps


def test_learned_form_same_estimate(ctx):
    p = plan(solve_inner_prec=mpmc.FP32)
    e0 = driver.estimate(ctx, p, torch.cuda.synchronize)
    e1 = driver.estimate(ctx, plan(solve_inner_prec=mpmc.FP32, learned=True, net_batches=2, net_pairs=16,
                                   net_steps=10), torch.cuda.synchronize)
    e2 = driver.estimate(ctx, plan(solve_inner_prec=mpmc.FP32, learned=True, net_source="random", net_batches=2,
                                   net_pairs=16, net_steps=10), torch.cuda.synchronize)
    assert abs(e2.value - e0.value) < 1e-6
    assert "net_loss" in e1.info and e1.info["net_loss"][1] < e1.info["net_loss"][0]
    # same noise, solves to 1e-10: the solve-term samples agree to ~1e-10 n
    assert np.max(np.abs(e1.levels[0].samples - e0.levels[0].samples)) < 1e-7
    assert abs(e1.value - e0.value) < 1e-6


@pytest.mark.parametrize("poly_prec,solve_prec", [(mpmc.FP64, mpmc.FP64), (mpmc.FP32, mpmc.FP32)])
def test_multilevel_estimate_within_3_sigma_of_dense_exact(ctx, poly_prec, solve_prec):
    """The complete multipolynomial estimate (deflation set, two polynomials,
    three Monte Carlo terms, FP64 or mixed precision) against Tr M^-1 from the
    dense FP64 inverse of the oracle: within 3 of its own standard errors.  The
    solve term (M^-1 - p1) carries a tiny variance; the error budget sits in
    the cheap low-degree terms."""
    from oracle import lattice as OLT
    dims, kappa = (4, 4, 4, 4), 0.115
    U = inputs.gauge_links(dims, 0.5, seed=1)
    exact = np.trace(np.linalg.inv(OLT.dense_wilson(dims, kappa, U)))
    e = driver.estimate(ctx, plan(noises=64, seed=11, poly_prec=poly_prec, solve_inner_prec=solve_prec),
                        torch.cuda.synchronize)
    assert 0 < e.stderr < np.inf
    assert abs(e.value - exact) < 3 * e.stderr
    assert e.levels[0].var < 1e-3 * e.levels[-1].var


@pytest.fixture(scope="module")
def dense44():
    from oracle import lattice as OLT
    dims, kappa = (4, 4, 4, 4), 0.115
    U = inputs.gauge_links(dims, 0.5, seed=1)
    return np.linalg.inv(OLT.dense_wilson(dims, kappa, U))


def test_probed_last_term_estimate(ctx, dense44):
    """Sec. 6 with the last term by probing: the probed term equals the dense
    Tr p_K(M) of the GPU's own roots, carries no variance, and the estimate is
    within 3 standard errors of the dense Tr M^-1 with a far smaller error than
    the all-sampled estimate."""
    from oracle import poly as OP
    from oracle.wilson import WilsonOp
    dims, kappa = (4, 4, 4, 4), 0.115
    op = WilsonOp(dims, kappa, inputs.gauge_links(dims, 0.5, seed=1))
    e_s = driver.estimate(ctx, plan(noises=64, seed=11), torch.cuda.synchronize)
    e_p = driver.estimate(ctx, plan(noises=64, seed=11, probe_last=True), torch.cuda.synchronize)
    last = e_p.levels[-1]
    assert last.exact and last.var == 0.0 and "probed" in last.name
    Pm = OP.apply_p(op, e_p.polys[-1].roots, np.eye(op.n)).T
    # the default plan probes in FP32 arithmetic (FP64 sums): FP32 rounding per probe
    assert abs(last.mean - np.trace(Pm)) < 1e-6 * abs(np.trace(Pm))
    exact = np.trace(dense44)
    assert 0 < e_p.stderr < 0.1 * e_s.stderr
    assert abs(e_p.value - exact) < 3 * e_p.stderr + 1e-9 * abs(exact)
    for L0, L1 in zip(e_s.levels[:-1], e_p.levels[:-1]):
        assert np.array_equal(L0.samples, L1.samples)


@pytest.mark.parametrize("probe", [False, True])
def test_estimate_to_error_stops_at_target(ctx, dense44, probe):
    """Sec. 8's adaptive stopping: every sampled term stops once its standard
    error is at most eps / sqrt(#sampled terms) (or at the noise cap), the
    minimum counts 2 / 3 / 6 hold, counts grow in steps of check_every, and the
    estimate is within 3 standard errors of the dense trace."""
    eps = 1.0
    p = plan(seed=5, probe_last=probe)
    e = driver.estimate_to_error(ctx, p, eps, check_every=3, max_noises=4096)
    sampled = [L for L in e.levels if not L.exact]
    target = eps / np.sqrt(len(sampled))
    for l, L in enumerate(sampled):
        assert L.n >= (2, 3, 6)[min(l, 2)]
        assert (L.n - (2, 3, 6)[min(l, 2)]) % 3 == 0
        assert np.sqrt(L.var / L.n) <= target or L.n >= 4096
    assert e.stderr <= eps * 1.0000001
    assert len(e.levels) == 3 and (e.levels[-1].exact == probe)
    assert abs(e.value - np.trace(dense44)) < 3 * max(e.stderr, 1e-9)


class _Stop(Exception):
    pass


@pytest.mark.parametrize("learned", [False, True])
def test_estimate_to_error_resumes_from_checkpoint(ctx, tmp_path, learned):
    """An adaptive estimate interrupted after its fourth batch and resumed from
    its checkpoint directory gives every term's samples, counts and the
    estimate of the same run left uninterrupted (noise i of term l comes from
    (seed, l, i); the set-up is reloaded from its roots, eigenpairs and
    weights)."""
    p = plan(seed=7, degrees=[(3, 3), 24, 8], learned=learned, net_batches=1, net_pairs=16)
    eps = 1.0
    full = driver.estimate_to_error(ctx, p, eps, check_every=3, checkpoint=str(tmp_path / "a"))
    seen = []

    def stop(l, n):
        seen.append((l, n))
        if len(seen) == 4:
            raise _Stop()

    with pytest.raises(_Stop):
        driver.estimate_to_error(ctx, p, eps, check_every=3, checkpoint=str(tmp_path / "b"), on_batch=stop)
    state = driver.load_mc(str(tmp_path / "b" / "mc.npz"), ctx, p)
    assert state[seen[-1][0]][0].n == seen[-1][1] and len(state) == seen[-1][0] + 1
    resumed = driver.estimate_to_error(ctx, p, eps, check_every=3, checkpoint=str(tmp_path / "b"))
    assert [L.name for L in resumed.levels] == [L.name for L in full.levels]
    for L0, L1 in zip(full.levels, resumed.levels):
        assert L0.n == L1.n and np.array_equal(L0.samples, L1.samples) and L0.corr == L1.corr
    assert resumed.value == full.value and resumed.stderr == full.stderr
    # a finished checkpoint resumes to the same result without new samples
    again = driver.estimate_to_error(ctx, p, eps, check_every=3, checkpoint=str(tmp_path / "b"))
    assert again.value == full.value
    with pytest.raises(ValueError):   # another plan on the same directory
        driver.estimate_to_error(ctx, plan(seed=8, degrees=[(3, 3), 24, 8]), eps, checkpoint=str(tmp_path / "b"))
