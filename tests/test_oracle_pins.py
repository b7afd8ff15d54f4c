"""Pins of the FP64 oracle against facts fixed by the paper and by mathematics.

Each test checks the oracle against something other than itself: closed forms,
special cases that reduce to textbook or library routines, finite differences,
hand-worked fixtures and invariants of the leapfrog integrator.
"""
import json
import math
import os
from fractions import Fraction

import numpy as np
import pytest

import oracle
from oracle import loops
from workloads import make_draws

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
G, C = oracle.GAUSS, oracle.CAUCHY


def _toy(n=40, p=5, K=4, seed=3, scale=0.4, pin=1):
    rng = np.random.default_rng(seed)
    X = rng.normal(size=(n, p))
    y = rng.integers(0, K, size=n).astype(np.int32)
    B = rng.normal(0, scale, size=(p, K))
    if pin:
        B[:, K - 1] = 0.0
    return X, y, B


# ---------------------------------------------------------------- log-posterior kernel

@pytest.mark.parametrize("K", [2, 3, 7])
@pytest.mark.parametrize("pin", [0, 1])
@pytest.mark.parametrize("prior", [G, C])
def test_logk_at_zero_coefficients(K, pin, prior):
    # Section 2.1: at B = 0 every psi_ik = 1/K and the prior terms vanish.
    X, y, _ = _toy(n=37, p=6, K=K)
    val = oracle.log_kernel(X, y, np.zeros((6, K)), prior, 0.7, pin)
    assert val == pytest.approx(-37 * math.log(K), rel=1e-14)


@pytest.mark.parametrize("prior,scale", [(G, 1.0), (G, 0.1), (C, 1.0), (C, 2.5)])
def test_logk_at_zero_design_matches_scipy_prior(prior, scale):
    # With X = 0 the likelihood is -n log K; the rest is the prior, checked against
    # scipy's log-densities with their normalising constants removed.
    from scipy import stats
    n, p, K = 11, 4, 3
    X = np.zeros((n, p))
    y = np.arange(n, dtype=np.int32) % K
    rng = np.random.default_rng(0)
    B = rng.normal(size=(p, K))
    B[:, K - 1] = 0.0
    free = B[:, : K - 1]
    if prior == G:
        lp = np.sum(stats.norm.logpdf(free, 0, scale) + 0.5 * np.log(2 * np.pi * scale * scale))
    else:
        lp = np.sum(stats.cauchy.logpdf(free, 0, scale) + np.log(np.pi * scale))
    val = oracle.log_kernel(X, y, B, prior, scale, 1)
    assert val == pytest.approx(-n * math.log(K) + lp, rel=1e-13)


def test_logistic_special_case():
    # K = 2 with the last class pinned is logistic regression on class 0.
    X, y, B = _toy(n=60, p=4, K=2, pin=1)
    z = X @ B[:, 0]
    ll = np.sum(np.where(y == 0, z, 0.0) - np.logaddexp(0.0, z))
    assert oracle.log_likelihood(X, y, B) == pytest.approx(ll, rel=1e-13)


def test_softmax_rows_are_distributions():
    X, y, B = _toy(n=200, p=8, K=6, scale=3.0)
    Z = oracle.logits(X, B)
    P = oracle.softmax_rows(Z)
    assert np.all(P > 0)
    # exp(z - LSE) inherits the absolute rounding of LSE as a relative error
    bound = (6 + np.max(np.abs(oracle.log_sum_exp_rows(Z)))) * 2.3e-16
    assert np.max(np.abs(P.sum(axis=1) - 1.0)) < bound


def test_softmax_large_logits_stable():
    Z = np.array([[1000.0, 999.0, -1000.0], [-800.0, -800.0, -801.0]])
    P = oracle.softmax_rows(Z)
    assert np.all(np.isfinite(P))
    e = math.exp(-1.0)
    assert P[0, 0] == pytest.approx(1 / (1 + e), rel=1e-14)
    assert P[1, 2] == pytest.approx(e / (2 + e), rel=1e-14)


# ---------------------------------------------------------------- gradient

@pytest.mark.parametrize("K", [2, 4, 8])
@pytest.mark.parametrize("pin", [0, 1])
def test_gradient_at_zero_exact(K, pin):
    # At B = 0 the gradient is X^T (Y - 1/K), masked. The expected value is exact
    # rational arithmetic; the oracle's softmax reaches 1/K through exp(-log K), which
    # may be off by an ulp, so allow n * max|x| ulps.
    rng = np.random.default_rng(K + 10 * pin)
    n, p = 23, 5
    Xi = rng.integers(-3, 4, size=(n, p))
    y = rng.integers(0, K, size=n).astype(np.int32)
    expect = np.zeros((p, K))
    for j in range(p):
        for k in range(K):
            if pin and k == K - 1:
                continue
            s = sum(Fraction(int(Xi[i, j])) * (Fraction(int(y[i] == k)) - Fraction(1, K))
                    for i in range(n))
            expect[j, k] = float(s)
    got = oracle.grad_log_kernel(Xi.astype(np.float64), y, np.zeros((p, K)), G, 1.0, pin)
    assert np.max(np.abs(got - expect)) <= n * 3 * 2.3e-16


def _fd_grad(f, B, h=1e-4):
    """Central differences with one Richardson step: O(h^4) truncation."""
    g = np.zeros_like(B)
    for idx in np.ndindex(B.shape):
        def d(hh):
            Bp = B.copy(); Bp[idx] += hh
            Bm = B.copy(); Bm[idx] -= hh
            return (f(Bp) - f(Bm)) / (2 * hh)
        g[idx] = (4 * d(h / 2) - d(h)) / 3
    return g


@pytest.mark.parametrize("prior,scale", [(G, 1.0), (G, 0.3), (C, 1.0), (C, 0.5)])
@pytest.mark.parametrize("pin", [0, 1])
def test_gradient_matches_finite_differences(prior, scale, pin):
    X, y, B = _toy(n=50, p=6, K=4, seed=11, scale=0.8, pin=pin)
    f = lambda BB: oracle.log_kernel(X, y, BB, prior, scale, pin)
    g = oracle.grad_log_kernel(X, y, B, prior, scale, pin)
    fd = _fd_grad(f, B) * oracle.free_mask(6, 4, pin)
    assert np.max(np.abs(g - fd)) <= 1e-7 * max(1.0, np.max(np.abs(g)))


def test_gradient_matches_torch_autograd():
    # Independent library: torch's log_softmax and reverse-mode autodiff in float64.
    torch = pytest.importorskip("torch")
    X, y, B = _toy(n=300, p=12, K=5, seed=5, scale=0.5, pin=1)
    for prior, scale in [(G, 0.7), (C, 1.3)]:
        Bt = torch.tensor(B, dtype=torch.float64, requires_grad=True)
        Xt = torch.tensor(X, dtype=torch.float64)
        yt = torch.tensor(y, dtype=torch.int64)
        ll = torch.log_softmax(Xt @ Bt, dim=1).gather(1, yt[:, None]).sum()
        free = Bt[:, :4]
        if prior == G:
            lp = -(free * free).sum() / (2 * scale * scale)
        else:
            lp = -torch.log1p((free / scale) ** 2).sum()
        (ll + lp).backward()
        tg = Bt.grad.numpy().copy()
        tg[:, 4] = 0.0
        g = oracle.grad_log_kernel(X, y, B, prior, scale, 1)
        assert np.max(np.abs(g - tg)) <= 1e-12 * max(1.0, np.max(np.abs(tg)))
        assert oracle.log_kernel(X, y, B, prior, scale, 1) == pytest.approx(float(ll + lp), rel=1e-13)


@pytest.mark.parametrize("prior", [G, C])
@pytest.mark.parametrize("pin", [0, 1])
def test_loop_definitions_match_vectorised(prior, pin):
    X, y, B = _toy(n=6, p=3, K=3, seed=2, scale=0.6, pin=pin)
    lk = loops.log_kernel_loops(X.tolist(), y.tolist(), B.tolist(), 3, prior, 0.8, pin)
    gl = np.array(loops.grad_loops(X.tolist(), y.tolist(), B.tolist(), 3, prior, 0.8, pin))
    assert oracle.log_kernel(X, y, B, prior, 0.8, pin) == pytest.approx(lk, rel=1e-13)
    assert np.allclose(oracle.grad_log_kernel(X, y, B, prior, 0.8, pin), gl, rtol=1e-12, atol=1e-13)


# ---------------------------------------------------------------- leapfrog integrator

def test_harmonic_oscillator_fixture():
    with open(os.path.join(GOLDEN, "harmonic_leapfrog_step.json")) as f:
        cases = json.load(f)["cases"]
    n, p, K = 9, 1, 2
    X = np.zeros((n, p))
    y = np.zeros(n, dtype=np.int32)
    for c in cases:
        B = np.array([[c["beta"], 0.0]])
        eta = np.array([[c["eta"], 0.0]])
        Gr = oracle.grad_log_kernel(X, y, B, G, c["sigma"], 1)
        B1, e1, _, _ = oracle.leapfrog_step(X, y, B, eta, Gr, c["eps"], G, c["sigma"], 1)
        assert B1[0, 0] == pytest.approx(c["beta_next"], abs=1e-14)
        assert e1[0, 0] == pytest.approx(c["eta_next"], abs=1e-14)
        assert B1[0, 1] == 0.0 and e1[0, 1] == 0.0


def test_leapfrog_is_time_reversible():
    X, y, B = _toy(n=80, p=5, K=4, seed=21, scale=0.3)
    rng = np.random.default_rng(4)
    eta = rng.normal(size=B.shape) * oracle.free_mask(5, 4, 1)
    Gr = oracle.grad_log_kernel(X, y, B, C, 1.0, 1)
    B1, e1, G1, _ = oracle.leapfrog(X, y, B, eta, Gr, 0.02, 25, C, 1.0, 1)
    B2, e2, _, _ = oracle.leapfrog(X, y, B1, -e1, G1, 0.02, 25, C, 1.0, 1)
    assert np.max(np.abs(B2 - B)) <= 1e-12 * max(1.0, np.max(np.abs(B)))
    assert np.max(np.abs(e2 + eta)) <= 1e-12 * max(1.0, np.max(np.abs(eta)))


def test_energy_error_is_second_order():
    X, y, B = _toy(n=120, p=4, K=3, seed=8, scale=0.2)
    rng = np.random.default_rng(9)
    eta = rng.normal(size=B.shape) * oracle.free_mask(4, 3, 1)
    T = 0.4
    errs = []
    for eps in [0.02, 0.01, 0.005, 0.0025]:
        L = int(round(T / eps))
        Gr = oracle.grad_log_kernel(X, y, B, G, 1.0, 1)
        H0 = -oracle.log_kernel(X, y, B, G, 1.0, 1) + oracle.kinetic(eta)
        B1, e1, _, lk1 = oracle.leapfrog(X, y, B, eta, Gr, eps, L, G, 1.0, 1)
        errs.append(abs(-lk1 + oracle.kinetic(e1) - H0))
    slope = np.polyfit(np.log([0.02, 0.01, 0.005, 0.0025]), np.log(errs), 1)[0]
    assert 1.8 < slope < 2.2


def test_leapfrog_preserves_volume():
    X, y, B = _toy(n=30, p=2, K=2, seed=13, scale=0.5)
    eta = np.array([[0.3, 0.0], [-0.4, 0.0]])

    def step(v):
        Bv = np.array([[v[0], 0.0], [v[1], 0.0]])
        ev = np.array([[v[2], 0.0], [v[3], 0.0]])
        Gr = oracle.grad_log_kernel(X, y, Bv, C, 1.0, 1)
        B1, e1, _, _ = oracle.leapfrog_step(X, y, Bv, ev, Gr, 0.3, C, 1.0, 1)
        return np.array([B1[0, 0], B1[1, 0], e1[0, 0], e1[1, 0]])

    v0 = np.array([B[0, 0], B[1, 0], eta[0, 0], eta[1, 0]])
    J = np.zeros((4, 4))
    h = 1e-6
    for a in range(4):
        dv = np.zeros(4); dv[a] = h
        J[:, a] = (step(v0 + dv) - step(v0 - dv)) / (2 * h)
    assert abs(np.linalg.det(J) - 1.0) < 1e-7


# ---------------------------------------------------------------- accept rule and sampler

def test_accept_rule_fixture():
    with open(os.path.join(GOLDEN, "accept_cases.json")) as f:
        cases = json.load(f)["cases"]
    for c in cases:
        H1 = float(c["H1"])
        acc, div = oracle.accept_decision(c["H0"], H1, c["u"], c["inv_temp"])
        assert (acc, div) == (c["accepted"], c["divergent"]), c["note"]


def test_annealing_schedule():
    it = oracle.annealed_inv_temps(100, 1e3, 0.9)
    assert it[0] == pytest.approx(1e-3)
    assert it[1] == pytest.approx(1 / 900.0)
    # 1000 * 0.9**65 = 1.06 > 1, 1000 * 0.9**66 = 0.958 < 1
    assert it[65] < 1.0 and it[66] == 1.0 and np.all(it[66:] == 1.0)


def test_iteration_records_energies():
    X, y, B = _toy(n=40, p=3, K=3, seed=1, scale=0.1)
    Gr = oracle.grad_log_kernel(X, y, B, G, 1.0, 1)
    lk = oracle.log_kernel(X, y, B, G, 1.0, 1)
    xi = np.random.default_rng(2).normal(size=B.shape)
    r = oracle.hmc_iteration(X, y, B, Gr, lk, xi, 0.5, 0.05, 5, G, 1.0, 1)
    eta0 = xi * oracle.free_mask(3, 3, 1)
    assert r["H0"] == pytest.approx(-lk + 0.5 * np.sum(eta0 ** 2), rel=1e-15)
    lk1 = oracle.log_kernel(X, y, r["B_prop"], G, 1.0, 1)
    assert r["H1"] == pytest.approx(-lk1 + 0.5 * np.sum(r["eta_prop"] ** 2), rel=1e-13)


@pytest.mark.slow
def test_posterior_mean_matches_quadrature():
    # One free coefficient (p = 1, K = 2 pinned, n = 20): the posterior mean and variance
    # from dense 1-D quadrature must contain the chain's mean within 3 MCSE.
    from paper_1402_4089_amd.diagnostics import ess
    rng = np.random.default_rng(17)
    n = 20
    X = rng.normal(size=(n, 1))
    y = (rng.random(n) < 1 / (1 + np.exp(-1.5 * X[:, 0]))).astype(np.int32)
    y = 1 - y                                                 # class 0 is the free one
    grid = np.linspace(-12, 12, 48001)
    lk = np.array([oracle.log_kernel(X, y, np.array([[b, 0.0]]), C, 1.0, 1) for b in grid])
    w = np.exp(lk - lk.max())
    mean_q = np.sum(grid * w) / np.sum(w)
    n_iter = 3000
    d = make_draws(1, 2, n_iter, seed=(99, 1, 0))
    out = oracle.sample(X, y, 2, d.xi, d.u, 0.15, 8, C, 1.0, 1)
    chain = out["samples"][n_iter // 5:, 0, 0]
    e = ess(chain)[0]
    mcse = chain.std(ddof=1) / np.sqrt(e)
    assert out["accepted"].mean() > 0.6
    assert abs(chain.mean() - mean_q) < 3 * mcse


def test_posterior_predictive_argmax():
    X = np.array([[1.0, 0.0], [0.0, 1.0], [1.0, 1.0]])
    S = np.zeros((2, 2, 3))
    S[:, 0, 0] = 5.0
    S[:, 1, 1] = 5.0
    pred = oracle.posterior_predictive_class(X, S)
    assert list(pred[:2]) == [0, 1]


# ---------------------------------------------------------------- counter-based draws

def test_philox_known_answers():
    # Known-answer vectors published with the Philox4x32-10 definition (Random123).
    from oracle import philox
    cases = [((0, 0, 0, 0), (0, 0), (0x6627E8D5, 0xE169C58D, 0xBC57AC4C, 0x9B00DBD8)),
             ((0xFFFFFFFF,) * 4, (0xFFFFFFFF,) * 2, (0x408F276D, 0x41C83B0E, 0xA20BC7C6, 0x6D5451FD)),
             ((0x243F6A88, 0x85A308D3, 0x13198A2E, 0x03707344), (0xA4093822, 0x299F31D0),
              (0xD16CFE09, 0x94FDCCEB, 0x5001E420, 0x24126EA1))]
    for ctr, key, want in cases:
        got = tuple(int(v) for v in philox.philox4x32_10(*ctr, *key))
        assert got == want


def test_philox_normals_are_standard_normal():
    from scipy import stats
    from oracle import philox
    z = philox.momentum_normals(12345, 3, 7, 200001)
    assert abs(z.mean()) < 5 / math.sqrt(z.size)
    assert abs(z.var() - 1) < 5 * math.sqrt(2 / z.size)
    assert stats.kstest(z, "norm").pvalue > 1e-3
    u = np.array([philox.accept_uniform(5, 0, t) for t in range(4000)])
    assert np.all((u > 0) & (u < 1)) and stats.kstest(u, "uniform").pvalue > 1e-3
