"""Pins of the oracle's Poisson-regression link (y_i ~ Poisson(exp(x_i^T beta)), one
coefficient column, nothing pinned) against facts fixed by mathematics: closed forms at
beta = 0 and at the maximum-likelihood point of an intercept-only model, scipy's Poisson
log-pmf, finite differences, leapfrog reversibility, and a posterior mean by quadrature."""
import numpy as np
import pytest
from scipy import special, stats

import oracle
from workloads import make_draws

G, C, P = oracle.GAUSS, oracle.CAUCHY, oracle.POISSON


def _toy(n=60, p=5, seed=4, scale=0.3):
    rng = np.random.default_rng(seed)
    X = rng.normal(size=(n, p))
    B = rng.normal(0, scale, size=(p, 1))
    y = rng.poisson(np.exp(X @ B[:, 0])).astype(np.int32)
    return X, y, B


def test_logk_and_gradient_at_zero_closed_form():
    # beta = 0: every rate is 1, so l = sum_i (y_i * 0 - 1) = -n, the Gaussian prior adds 0,
    # and the gradient is X^T (y - 1) exactly (small integers: exact in float64).
    rng = np.random.default_rng(2)
    n, p = 33, 7
    X = rng.integers(-4, 5, size=(n, p)).astype(np.float64)
    y = rng.integers(0, 9, size=n).astype(np.int32)
    B = np.zeros((p, 1))
    assert oracle.log_kernel(X, y, B, G, 1.0, 0, P) == -float(n)
    g = oracle.grad_log_kernel(X, y, B, G, 1.0, 0, P)
    assert np.array_equal(g[:, 0], X.T @ (y.astype(np.float64) - 1.0))


def test_log_likelihood_matches_scipy_logpmf():
    # scipy's log-pmf is y log mu - mu - log y!; the oracle drops the constant log y!.
    X, y, B = _toy()
    mu = np.exp(X @ B[:, 0])
    ref = float(np.sum(stats.poisson.logpmf(y, mu) + special.gammaln(y + 1.0)))
    assert oracle.log_likelihood(X, y, B, P) == pytest.approx(ref, rel=1e-13, abs=1e-11)


def test_intercept_only_gradient_vanishes_at_the_mle():
    # One column of ones: l(b) = S b - n e^b, maximised at b = log(S / n); without prior
    # weight (a very wide Gaussian) the gradient there is zero.
    y = np.array([0, 3, 1, 4, 2, 2, 5, 1], dtype=np.int32)
    X = np.ones((y.size, 1))
    b = np.log(y.sum() / y.size)
    g = oracle.grad_log_kernel(X, y, np.array([[b]]), G, 1e12, 0, P)
    assert abs(g[0, 0]) < 1e-12


def _fd_grad(f, B, h=1e-5):
    g = np.zeros_like(B)
    for idx in np.ndindex(B.shape):
        def d(hh):
            Bp = B.copy(); Bp[idx] += hh
            Bm = B.copy(); Bm[idx] -= hh
            return (f(Bp) - f(Bm)) / (2 * hh)
        g[idx] = (4 * d(h / 2) - d(h)) / 3
    return g


@pytest.mark.parametrize("prior,scale", [(G, 1.0), (C, 0.5)])
def test_gradient_matches_finite_differences(prior, scale):
    X, y, B = _toy(n=80, p=6, seed=9)
    f = lambda BB: oracle.log_kernel(X, y, BB, prior, scale, 0, P)
    g = oracle.grad_log_kernel(X, y, B, prior, scale, 0, P)
    fd = _fd_grad(f, B)
    assert np.max(np.abs(g - fd)) <= 1e-7 * max(1.0, np.max(np.abs(g)))


def test_leapfrog_is_time_reversible():
    X, y, B = _toy(n=40, p=4, seed=12)
    eta = np.random.default_rng(3).normal(size=B.shape)
    G0 = oracle.grad_log_kernel(X, y, B, G, 1.0, 0, P)
    B1, e1, G1, _ = oracle.leapfrog(X, y, B, eta, G0, 0.01, 20, G, 1.0, 0, P)
    B2, e2, _, _ = oracle.leapfrog(X, y, B1, -e1, G1, 0.01, 20, G, 1.0, 0, P)
    assert np.max(np.abs(B2 - B)) <= 1e-12 * max(1.0, np.max(np.abs(B)))
    assert np.max(np.abs(-e2 - eta)) <= 1e-11 * max(1.0, np.max(np.abs(eta)))


@pytest.mark.slow
def test_posterior_mean_matches_quadrature():
    # Intercept-only model, n = 20, Gaussian N(0, 1) prior: the posterior density of b is
    # proportional to exp(S b - n e^b - b^2 / 2); dense 1-D quadrature gives its mean, which
    # the oracle chain must contain within 3 MCSE.
    from paper_1402_4089_amd.diagnostics import ess
    rng = np.random.default_rng(23)
    y = rng.poisson(2.0, size=20).astype(np.int32)
    X = np.ones((20, 1))
    grid = np.linspace(-6, 6, 48001)
    lk = y.sum() * grid - 20 * np.exp(grid) - grid ** 2 / 2
    w = np.exp(lk - lk.max())
    mean_q = np.sum(grid * w) / np.sum(w)
    n_iter = 3000
    d = make_draws(1, 1, n_iter, seed=(98, 1, 0))
    out = oracle.sample(X, y, 1, d.xi, d.u, 0.08, 8, G, 1.0, 0, link=P)
    chain = out["samples"][n_iter // 5:, 0, 0]
    e = ess(chain)[0]
    mcse = chain.std(ddof=1) / np.sqrt(e)
    assert out["accepted"].mean() > 0.6
    assert abs(chain.mean() - mean_q) < 3 * mcse
