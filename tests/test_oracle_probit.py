"""Pins of the oracle's probit link (binary y_i, P(y_i = 1) = Phi(x_i^T beta), one coefficient
column, nothing pinned) against facts fixed by mathematics: closed forms at beta = 0, the
two-branch Bernoulli log-likelihood, the asymptotic series of the normal tail far from the
mean, a symmetry of the model, finite differences, leapfrog reversibility, and a posterior
mean by quadrature."""
import math

import numpy as np
import pytest
from scipy import stats

import oracle
from workloads import make_draws

G, C, PR = oracle.GAUSS, oracle.CAUCHY, oracle.PROBIT


def _toy(n=60, p=5, seed=4, scale=0.5):
    rng = np.random.default_rng(seed)
    X = rng.normal(size=(n, p))
    B = rng.normal(0, scale, size=(p, 1))
    # latent-variable draw: y = 1 iff x^T beta + e > 0 with e ~ N(0, 1)
    y = (X @ B[:, 0] + rng.normal(size=n) > 0).astype(np.int32)
    return X, y, B


def test_logk_and_gradient_at_zero_closed_form():
    # beta = 0: Phi(0) = 1/2 for every row, so l = -n log 2; the residual is s_i phi(0) /
    # Phi(0) = s_i sqrt(2 / pi), so G = sqrt(2 / pi) X^T s.
    rng = np.random.default_rng(2)
    n, p = 33, 7
    X = rng.integers(-4, 5, size=(n, p)).astype(np.float64)
    y = rng.integers(0, 2, size=n).astype(np.int32)
    B = np.zeros((p, 1))
    assert oracle.log_kernel(X, y, B, G, 1.0, 0, PR) == pytest.approx(-n * math.log(2.0), rel=1e-14)
    g = oracle.grad_log_kernel(X, y, B, G, 1.0, 0, PR)
    s = 2.0 * y - 1.0
    np.testing.assert_allclose(g[:, 0], math.sqrt(2.0 / math.pi) * (X.T @ s), rtol=1e-14, atol=1e-13)


def test_log_likelihood_is_the_bernoulli_sum():
    # the two-branch form y log Phi(z) + (1 - y) log(1 - Phi(z)) at moderate z
    X, y, B = _toy()
    z = X @ B[:, 0]
    assert np.max(np.abs(z)) < 6
    ref = float(np.sum(y * np.log(stats.norm.cdf(z)) + (1 - y) * np.log(stats.norm.sf(z))))
    assert oracle.log_likelihood(X, y, B, PR) == pytest.approx(ref, rel=1e-12)


def test_labels_other_than_one_are_failures():
    X, y, B = _toy(seed=8)
    y2 = np.where(y == 1, 1, 7).astype(np.int32)
    assert oracle.log_likelihood(X, y2, B, PR) == oracle.log_likelihood(X, y, B, PR)


@pytest.mark.parametrize("t", [-8.0, -30.0, -300.0])
def test_residual_far_in_the_tail_follows_the_mills_series(t):
    # A success at z = t << 0: r = phi(t) / Phi(t). With Phi(t) = phi(t) / |t| (1 - 1/t^2 +
    # 3/t^4 - 15/t^6 + 105/t^8 - 945/t^10 + ...) (the asymptotic series of the normal tail),
    # r = |t| / (that series). The first omitted term, 10395 / t^12, bounds the truncation
    # error: 1.5e-7 at t = -8, negligible at t = -30 and -300, where phi(t) and Phi(t)
    # themselves underflow or nearly so. The oracle forms the ratio as exp(log phi - log Phi);
    # the two logs are about t^2 / 2 in size, so their difference carries an absolute error
    # of about t^2 eps: 1e-11 at t = -300.
    X = np.array([[t]])
    y = np.array([1], dtype=np.int32)
    r = oracle.residual(X, y, np.array([[1.0]]), PR)[0, 0]
    u = 1.0 / (t * t)
    series = 1 - u + 3 * u**2 - 15 * u**3 + 105 * u**4 - 945 * u**5
    tol = {-8.0: 2e-7, -30.0: 1e-12, -300.0: 1e-10}[t]
    assert r == pytest.approx(abs(t) / series, rel=tol)
    # a failure at z = -t is the mirror image
    r0 = oracle.residual(-X, np.array([0], dtype=np.int32), np.array([[1.0]]), PR)[0, 0]
    assert r0 == pytest.approx(-abs(t) / series, rel=tol)


def test_flipping_labels_and_features_leaves_the_likelihood():
    # Phi(s z) is unchanged when both s and z change sign
    X, y, B = _toy(seed=11)
    assert oracle.log_likelihood(-X, 1 - y, B, PR) == pytest.approx(
        oracle.log_likelihood(X, y, B, PR), rel=1e-15)


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
    f = lambda BB: oracle.log_kernel(X, y, BB, prior, scale, 0, PR)
    g = oracle.grad_log_kernel(X, y, B, prior, scale, 0, PR)
    fd = _fd_grad(f, B)
    assert np.max(np.abs(g - fd)) <= 1e-7 * max(1.0, np.max(np.abs(g)))


def test_leapfrog_is_time_reversible():
    X, y, B = _toy(n=40, p=4, seed=12)
    eta = np.random.default_rng(3).normal(size=B.shape)
    G0 = oracle.grad_log_kernel(X, y, B, G, 1.0, 0, PR)
    B1, e1, G1, _ = oracle.leapfrog(X, y, B, eta, G0, 0.01, 20, G, 1.0, 0, PR)
    B2, e2, _, _ = oracle.leapfrog(X, y, B1, -e1, G1, 0.01, 20, G, 1.0, 0, PR)
    assert np.max(np.abs(B2 - B)) <= 1e-12 * max(1.0, np.max(np.abs(B)))
    assert np.max(np.abs(-e2 - eta)) <= 1e-11 * max(1.0, np.max(np.abs(eta)))


@pytest.mark.slow
def test_posterior_mean_matches_quadrature():
    # Intercept-only model, n = 30, N(0, 1) prior: the posterior density of b is proportional
    # to Phi(b)^S Phi(-b)^(n - S) exp(-b^2 / 2); dense 1-D quadrature gives its mean, which
    # the oracle chain must contain within 3 MCSE.
    from paper_1402_4089_amd.diagnostics import ess
    rng = np.random.default_rng(29)
    n = 30
    y = (rng.random(n) < 0.7).astype(np.int32)
    S = int(y.sum())
    X = np.ones((n, 1))
    grid = np.linspace(-6, 6, 48001)
    lk = S * stats.norm.logcdf(grid) + (n - S) * stats.norm.logcdf(-grid) - grid ** 2 / 2
    w = np.exp(lk - lk.max())
    mean_q = np.sum(grid * w) / np.sum(w)
    n_iter = 3000
    d = make_draws(1, 1, n_iter, seed=(98, 2, 0))
    out = oracle.sample(X, y, 1, d.xi, d.u, 0.1, 8, G, 1.0, 0, link=PR)
    chain = out["samples"][n_iter // 5:, 0, 0]
    e = ess(chain)[0]
    mcse = chain.std(ddof=1) / np.sqrt(e)
    assert out["accepted"].mean() > 0.6
    assert abs(chain.mean() - mean_q) < 3 * mcse
