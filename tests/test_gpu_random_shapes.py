"""Seeded random shapes through every form against the FP64 oracle (GPU tier).

Shapes, formats, priors and pinning are drawn from a fixed seed, so every run checks the same
cases: n, p and K anywhere in their ranges (ragged tiles, row blocks, column chunks and class
blocks), whichever path the built-in rule picks for them, the split-precision planes and
batches of uneven problems with 1, 2 or 4 chains. Each gradient and log K of equations
(logkernel) and (fullgrad) must meet the parity bar of its format.
"""
import numpy as np
import pytest

import oracle
from gradbound import UNIT_ROUNDOFF, assert_elementwise
from oracle import split
from workloads import make_problem, make_random_state

pytestmark = pytest.mark.gpu


def _relL2(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def _plain_cases(count=24, seed=2024):
    rng = np.random.default_rng(seed)
    out = []
    for i in range(count):
        f64 = i % 3 == 2
        n = int(rng.integers(1, 3001 if f64 else 5001))
        p = int(rng.integers(1, 1501 if f64 else 3001))
        K = int(rng.integers(2, 65))
        pin = int(rng.integers(0, 2))
        prior = int(rng.integers(0, 2))
        out.append(("c1_small_f64" if f64 else "c3_widep", n, p, K, pin, prior, 100 + i))
    return out


def _split_cases(count=12, seed=2025):
    rng = np.random.default_rng(seed)
    return [(int(rng.integers(1, 5001)), int(rng.integers(1, 2501)), int(rng.integers(2, 65)),
             bool(rng.integers(0, 2)), int(rng.integers(0, 2)), 200 + i) for i in range(count)]


@pytest.mark.parametrize("name,n,p,K,pin,prior,seed", _plain_cases())
def test_random_plain_shapes(lib, name, n, p, K, pin, prior, seed):
    import torch
    prob = make_problem(name, n=n, p=p, K=K, seed=seed, prior=prior, prior_scale=0.7,
                        pin_last_class=pin)
    dp = lib.Problem(torch.from_numpy(np.ascontiguousarray(prob.X)).cuda(),
                     torch.from_numpy(prob.y).cuda(), K, prior, 0.7, bool(pin))
    Bd = torch.from_numpy(make_random_state(prob, 0.2, seed=seed).astype(prob.state_dtype)).cuda()
    logk, G = lib.logpost_grad(dp, Bd)
    G = G.double().cpu().numpy()
    Bs = Bd.double().cpu().numpy()
    lk_o, G_o = oracle.log_kernel_and_grad(prob.X64, prob.y, Bs, prior, 0.7, pin)
    tol = 1e-12 if prob.xfmt == "f64" else 1e-5
    err = _relL2(G, G_o)
    print(f"[random] {prob.xfmt} n={n} p={p} K={K} pin={pin} prior={prior}: rel-L2 {err:.2e}",
          flush=True)
    assert err <= tol
    assert_elementwise(G, G_o, prob.X64, prob.y, Bs, prior, 0.7, pin, UNIT_ROUNDOFF[prob.xfmt])
    assert abs(float(logk) - lk_o) <= max(tol, 1e-6) * max(abs(lk_o), 1.0)
    if pin:
        assert np.all(G[:, -1] == 0)


@pytest.mark.parametrize("n,p,K,hi_only,prior,seed", _split_cases())
def test_random_split_shapes(lib, n, p, K, hi_only, prior, seed):
    import torch
    prob = make_problem("c4_bf16", n=n, p=p, K=K, seed=seed, prior=prior, prior_scale=0.7)
    hi, lo = lib.split_bf16(torch.from_numpy(np.ascontiguousarray(prob.X64)).cuda(), hi_only=hi_only)
    dp = lib.Problem(hi, torch.from_numpy(prob.y).cuda(), K, prior, 0.7, True, X_lo=lo)
    Bd = torch.from_numpy(make_random_state(prob, 0.05, seed=seed).astype(np.float32)).cuda()
    logk, G = lib.logpost_grad(dp, Bd)
    G = G.double().cpu().numpy()
    Bs = Bd.double().cpu().numpy()
    h, l = split.split_hilo(prob.X64)
    Xe = h if hi_only else h + l
    lk_o, G_o = oracle.log_kernel_and_grad(Xe, prob.y, Bs, prior, 0.7, 1)
    err = _relL2(G, G_o)
    bound = 2.0 ** -14 * float(np.sum(np.max(np.abs(Xe) @ np.abs(Bs), axis=1))) + n * 1e-6
    print(f"[random] bf16 hi_only={hi_only} n={n} p={p} K={K}: rel-L2 {err:.2e}", flush=True)
    assert err <= 6e-5
    assert abs(float(logk) - lk_o) <= bound
    assert np.all(G[:, -1] == 0)


@pytest.mark.parametrize("seed", [31, 32, 33, 34])
def test_random_batches(lib, seed):
    """Five uneven problems, chains and the largest K drawn so that chains x class blocks
    stays within the four blocks a batch can stack."""
    import torch
    rng = np.random.default_rng(seed)
    chains = int(rng.choice([1, 2, 4]))
    kmax = 16 * (4 // chains)
    probs = []
    for b in range(5):
        n, p, K = int(rng.integers(1, 3001)), int(rng.integers(1, 1201)), int(rng.integers(2, kmax + 1))
        probs.append(make_problem("c4_bf16", n=n, p=p, K=K, seed=[seed, 7, b]))
    dev = []
    for pr in probs:
        hi, lo = lib.split_bf16(torch.from_numpy(np.ascontiguousarray(pr.X64)).cuda())
        dev.append(lib.Problem(hi, torch.from_numpy(pr.y).cuda(), pr.K, pr.prior, pr.prior_scale,
                               True, X_lo=lo))
    bt = lib.Batch(dev, chains)
    B, G, logk = bt.zeros_state()
    for b, pr in enumerate(probs):
        for c in range(chains):
            B[b][c].copy_(torch.from_numpy(make_random_state(pr, 0.05, seed=50 * b + c).astype(np.float32)))
    bt.logpost_grad(B, G, logk)
    lk = logk.cpu().numpy()
    worst = 0.0
    for b, pr in enumerate(probs):
        h, l = split.split_hilo(pr.X64)
        for c in range(chains):
            Bc = B[b][c].double().cpu().numpy()
            lk_o, G_o = oracle.log_kernel_and_grad(h + l, pr.y, Bc, pr.prior, pr.prior_scale, 1)
            Gd = G[b][c].double().cpu().numpy()
            err = _relL2(Gd, G_o)
            worst = max(worst, err)
            assert err <= 6e-5, f"problem {b} (n={pr.n}, p={pr.p}, K={pr.K}) chain {c}: {err:.2e}"
            assert abs(lk[b, c] - lk_o) <= 1e-6 * abs(lk_o) + 1e-4
            assert np.all(Gd[:, -1] == 0)
    print(f"[random] batch seed {seed}: {chains} chains, K up to {max(pr.K for pr in probs)}, "
          f"worst rel-L2 {worst:.2e}", flush=True)


def _leapfrog_cases(count=6, seed=2026):
    rng = np.random.default_rng(seed)
    return [(int(rng.integers(1, 2001)), int(rng.integers(1, 1201)), int(rng.integers(2, 41)),
             int(rng.integers(0, 2)), 300 + i) for i in range(count)]


@pytest.mark.parametrize("n,p,K,pin,seed", _leapfrog_cases())
def test_random_leapfrog_f64(lib, n, p, K, pin, seed):
    """Six FP64 leapfrog updates from a random state and momentum (equations (hmc1)-(hmc3)):
    position, momentum, gradient and log K within 1e-12 of the oracle's, on random shapes of
    both the row tile and the wide-p path."""
    import torch
    prob = make_problem("c1_small_f64", n=n, p=p, K=K, seed=seed, pin_last_class=pin)
    mask = oracle.free_mask(p, K, pin)
    B = make_random_state(prob, 0.1, seed=seed)
    eta = np.random.default_rng(seed).normal(size=B.shape) * mask
    eps = 0.2 / (np.sqrt(n) + np.sqrt(p))
    dp = lib.Problem(torch.from_numpy(prob.X).cuda(), torch.from_numpy(prob.y).cuda(), K,
                     prob.prior, prob.prior_scale, bool(pin))
    Bd = torch.from_numpy(B.copy()).cuda()
    logk, Gd = lib.logpost_grad(dp, Bd)
    ed = torch.from_numpy(eta.copy()).cuda()
    lib.leapfrog(dp, Bd, ed, Gd, logk, eps, 6)
    G0 = oracle.grad_log_kernel(prob.X64, prob.y, B, prob.prior, prob.prior_scale, pin)
    B1, e1, G1, lk1 = oracle.leapfrog(prob.X64, prob.y, B, eta, G0, eps, 6, prob.prior,
                                      prob.prior_scale, pin)
    eb = _relL2(Bd.cpu().numpy(), B1)
    ee = _relL2(ed.cpu().numpy(), e1)
    eg = _relL2(Gd.cpu().numpy(), G1)
    print(f"[random] leapfrog f64 n={n} p={p} K={K} pin={pin}: B {eb:.1e} eta {ee:.1e} G {eg:.1e}",
          flush=True)
    assert eb < 1e-12 and ee < 1e-12 and eg < 1e-12
    assert abs(float(logk) - lk1) < 1e-12 * max(abs(lk1), 1.0)
