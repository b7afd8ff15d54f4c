"""Diagnostics against series whose effective sample size is known in closed form."""
import numpy as np
import pytest

from paper_1402_4089_amd import diagnostics as dg


def _ar1(rho, T, d, seed):
    rng = np.random.default_rng(seed)
    e = rng.normal(size=(T, d))
    x = np.empty((T, d))
    x[0] = e[0] / np.sqrt(1 - rho * rho)
    for t in range(1, T):
        x[t] = rho * x[t - 1] + e[t]
    return x


@pytest.mark.parametrize("rho", [0.0, 0.5, 0.9])
def test_ess_ar1_closed_form(rho):
    # AR(1): integrated autocorrelation time (1 + rho) / (1 - rho).
    T = 100_000
    x = _ar1(rho, T, 4, seed=int(rho * 10))
    want = T * (1 - rho) / (1 + rho)
    got = dg.ess(x)
    assert np.all(np.abs(got / want - 1) < 0.08)


def test_ess_antithetic_capped_reasonably():
    x = _ar1(-0.5, 20000, 2, seed=3)
    assert np.all(dg.ess(x) > 20000)


def test_multichain_ess_and_rhat():
    chains = np.stack([_ar1(0.5, 4000, 3, seed=s) for s in range(4)])
    e = dg.multichain_ess(chains)
    want = 4 * 4000 / 3
    assert np.all(np.abs(e / want - 1) < 0.15)
    assert np.all(np.abs(dg.split_rhat(chains) - 1) < 0.01)
    shifted = chains.copy()
    shifted[0] += 3.0
    assert np.all(dg.split_rhat(shifted) > 1.1)
