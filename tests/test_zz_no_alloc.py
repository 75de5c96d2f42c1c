"""GPU: mpmc_apply_poly_noalloc, the variant of mpmc_apply_poly that allocates
nothing (its work vectors live in the library's fixed device scratch array),
gives the same bits as mpmc_apply_poly, on two calls in a row with the second
one smaller, for single and double polynomials in FP32 and FP64; sizes beyond
the array and calls with launch timing on are rejected."""
import ctypes

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2402_00016_amd import inputs, mpmc  # noqa: E402

FP64, FP32 = mpmc.FP64, mpmc.FP32
SCRATCH = 64 << 20


@pytest.fixture(scope="module")
def ctx():
    dims, kappa = (8, 8, 8, 8), 0.12
    return mpmc.Context(dims, kappa, inputs.gauge_links(dims, 0.5, seed=2))


def noalloc(ctx, poly, x, y, nrhs, prec):
    return mpmc._L.mpmc_apply_poly_noalloc(ctx.handle, poly.handle, ctypes.c_void_p(x.data_ptr()),
                                           ctypes.c_void_p(y.data_ptr()), int(nrhs), int(prec))


@pytest.mark.parametrize("kind,prec,sizes", [("single", FP32, (64, 24)), ("single", FP64, (16, 3)),
                                             ("double", FP32, (8, 1)), ("double", FP64, (4, 2))])
def test_noalloc_equals_apply_poly(ctx, kind, prec, sizes):
    P = ctx.gmres_poly(2, 0x100, 9)
    if kind == "double":
        P = ctx.gmres_poly(2, 0x101, 4, inner=ctx.gmres_poly(2, 0x101, 5))
    for call, N in enumerate(sizes):
        x = ctx.noise(7, 3, 100 * call, N, prec)
        want = ctx.apply_poly(P, x, N, prec)
        got = ctx.vector(N, prec)
        got.fill_(0xAB)
        torch.cuda.synchronize()
        assert noalloc(ctx, P, x, got, N, prec) == mpmc.OK, mpmc.mpmc_last_error(ctx.handle)
        torch.cuda.synchronize()
        assert torch.equal(got, want), (kind, prec, N)


def test_noalloc_limits(ctx):
    P = ctx.gmres_poly(2, 0x100, 9)
    vb = mpmc.mpmc_vector_bytes(ctx.handle, 128, FP32)
    assert 2 * vb > SCRATCH                  # two work vectors of 128 FP32 right-hand sides do not fit
    x = ctx.noise(1, 0, 0, 128, FP32)
    y = ctx.vector(128, FP32)
    assert noalloc(ctx, P, x, y, 128, FP32) == mpmc.EINVAL
    assert "limit" in mpmc.mpmc_last_error(ctx.handle)
    x = ctx.noise(1, 0, 0, 8, FP32)
    y = ctx.vector(8, FP32)
    assert noalloc(ctx, P, x, x, 8, FP32) == mpmc.EINVAL          # aliasing
    mpmc.mpmc_timing_enable(ctx.handle, 1)
    try:
        assert noalloc(ctx, P, x, y, 8, FP32) == mpmc.ESTATE      # timing would create events
    finally:
        mpmc.mpmc_timing_enable(ctx.handle, 0)
    assert noalloc(ctx, P, x, y, 8, FP32) == mpmc.OK
