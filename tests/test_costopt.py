"""Cost-optimal noise allocation over the Monte Carlo terms, checked against a
numerical constrained minimisation and against the one-term special case
(CPU only)."""
import numpy as np
import pytest
from scipy.optimize import minimize

from paper_2402_00016_amd import driver


def test_single_term_is_variance_over_eps2():
    N, cost = driver.optimal_noise_counts([4.0], [3.0], 0.1, min_counts=(1,))
    assert N[0] == 400 and cost == 1200.0


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_matches_numerical_minimum(seed):
    rng = np.random.default_rng(seed)
    L = 4
    V = 10.0 ** rng.uniform(-6, 2, L)
    C = 10.0 ** rng.uniform(0, 3, L)
    eps = 0.05
    N, cost = driver.optimal_noise_counts(V, C, eps, min_counts=(1,))
    # continuous optimum by SLSQP in log N, started from the uniform allocation
    # that meets the constraint; objective and constraint scaled to O(1)
    n0 = np.full(L, np.sum(V) / eps ** 2)
    ref = float(np.sum(n0 * C))
    res = minimize(lambda y: float(np.sum(np.exp(y) * C)) / ref, x0=np.log(n0),
                   constraints=[{"type": "ineq", "fun": lambda y: 1.0 - float(np.sum(V * np.exp(-y))) / eps ** 2}],
                   method="SLSQP", options=dict(ftol=1e-14, maxiter=1000))
    assert res.success
    n_opt = np.exp(res.x)
    cont = np.sqrt(V / C) * np.sum(np.sqrt(V * C)) / eps ** 2
    assert np.allclose(cont, n_opt, rtol=1e-3)
    assert np.all(N >= cont) and np.all(N < cont + 1)        # rounded up
    assert np.sum(V / N) <= eps ** 2 * (1 + 1e-12)            # constraint met
    assert cost <= float(np.sum(n_opt * C)) + np.sum(C)       # within one noise per term


def test_minimum_counts_and_errors():
    N, _ = driver.optimal_noise_counts([1e-12, 1e-12, 1.0], [1.0, 1.0, 1.0], 1.0)
    assert list(N[:2]) == [2, 3]
    with pytest.raises(ValueError):
        driver.optimal_noise_counts([1.0], [0.0], 0.1)
    with pytest.raises(ValueError):
        driver.optimal_noise_counts([1.0, 2.0], [1.0], 0.1)
