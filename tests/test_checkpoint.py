"""Checkpoint files of the adaptive estimate (host logic, no GPU): the Monte
Carlo state round-trips exactly through its file, a file written for another
lattice, gauge field or plan is refused, and the file is replaced atomically."""
import os
import types

import numpy as np
import pytest

from paper_2402_00016_amd import driver


def fake_ctx(kappa=0.115, seed=0):
    links = np.random.default_rng(seed).standard_normal((4 ** 4, 4, 3, 3, 2))
    return types.SimpleNamespace(dims=(4, 4, 4, 4), kappa=kappa, t_antiperiodic=True, links=links)


def plan(**kw):
    base = dict(degrees=[(3, 3), 24, 8], noises=16, seed=3, nev=6)
    base.update(kw)
    return driver.Plan(**base)


def terms():
    rng = np.random.default_rng(1)
    mk = lambda n: rng.standard_normal(n) + 1j * rng.standard_normal(n)
    return [(driver.LevelResult("term 0", mk(5), 0.25 - 0.5j, 1234, 0.5), True),
            (driver.LevelResult("term 1 (probed, 81 probes)", mk(1), 0j, 99, 0.1, exact=True), True),
            (driver.LevelResult("term 2", mk(9), 1e-300 + 3j, 77, 2.0), False)]


def test_mc_state_round_trip(tmp_path):
    ctx, p = fake_ctx(), plan()
    path = str(tmp_path / "mc.npz")
    driver.save_mc(path, ctx, p, terms())
    assert not os.path.exists(path + ".tmp")
    back = driver.load_mc(path, ctx, p)
    assert len(back) == 3
    for (L0, d0), (L1, d1) in zip(terms(), back):
        assert d0 == d1 and L0.name == L1.name and L0.exact == L1.exact
        assert np.array_equal(L0.samples, L1.samples) and L1.samples.dtype == np.complex128
        assert L0.corr == L1.corr and L0.mvps == L1.mvps and L0.seconds == L1.seconds


@pytest.mark.parametrize("other", ["kappa", "links", "plan", "theta"])
def test_mc_state_refused_for_another_configuration(tmp_path, other):
    ctx, p = fake_ctx(), plan()
    path = str(tmp_path / "mc.npz")
    driver.save_mc(path, ctx, p, terms())
    if other == "kappa":
        ctx = fake_ctx(kappa=0.12)
    elif other == "links":
        ctx = fake_ctx(seed=1)
    elif other == "plan":
        p = plan(degrees=[(3, 3), 24, 9])
    else:
        p = plan(theta=1)
    with pytest.raises(ValueError):
        driver.load_mc(path, ctx, p)


def test_identity_is_stable():
    """The identity text depends on the configuration only (the links digest is
    cached per context and equal for equal links)."""
    a, b = fake_ctx(), fake_ctx()
    assert driver.plan_identity(a, plan()) == driver.plan_identity(b, plan())
    assert driver.plan_identity(a, plan()) != driver.plan_identity(a, plan(seed=4))
