"""Degenerate shapes of the method against the FP64 oracle (GPU tier).

A single observation (n = 1), a single predictor (p = 1), the two-class case (K = 2, where
the pinned model is logistic regression), and combinations of them, through every form: the
row tile, the wide-p passes (forced, and chosen by the rule for a single long row), the
split-precision planes and a batch whose problems are degenerate. log K and G of equations
(logkernel) and (fullgrad) must match the oracle at each format's parity tolerance, and the
pinned column of G must be exactly zero.
"""
import numpy as np
import pytest

import oracle
from oracle import split
from workloads import make_problem, make_random_state

pytestmark = pytest.mark.gpu

# (config, n, p, K, path): path 0 = the rule's choice, 2 = wide p forced
# (the FP32 shapes use the unstandardised FP32 recipe: one row has no column spread to scale)
PLAIN = [("c3_widep", 1, 1, 2, 0), ("c3_widep", 1, 1000, 10, 0), ("c3_widep", 5, 1, 2, 0),
         ("c3_widep", 16, 1, 64, 0), ("c3_widep", 1, 2001, 3, 0), ("c3_widep", 1, 40, 5, 2),
         ("c1_small_f64", 1, 1, 2, 0), ("c1_small_f64", 2, 1, 64, 0), ("c1_small_f64", 1, 700, 3, 0)]
SPLIT = [(1, 1, 2), (1, 4096, 64), (129, 1, 5), (33, 7, 17)]


def _relL2(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


@pytest.mark.parametrize("name,n,p,K,path", PLAIN)
def test_plain_degenerate_shapes(lib, name, n, p, K, path):
    import torch
    prob = make_problem(name, n=n, p=p, K=K)
    kw = {} if path == 0 else dict(tuning=dict(path=path))
    dp = lib.Problem(torch.from_numpy(np.ascontiguousarray(prob.X)).cuda(),
                     torch.from_numpy(prob.y).cuda(), K, prob.prior, prob.prior_scale, True, **kw)
    # coefficients on the prior's own scale, so the likelihood part of G is not swamped
    B = make_random_state(prob, 0.3 * prob.prior_scale)
    Bd = torch.from_numpy(B.astype(prob.state_dtype)).cuda()
    logk, G = lib.logpost_grad(dp, Bd)
    G = G.double().cpu().numpy()
    Bs = Bd.double().cpu().numpy()
    lk_o, G_o = oracle.log_kernel_and_grad(prob.X64, prob.y, Bs, prob.prior, prob.prior_scale, 1)
    tol = 1e-12 if prob.xfmt == "f64" else 1e-5
    err = _relL2(G, G_o)
    print(f"[degenerate] {name} n={n} p={p} K={K} tuning {dp.tuning}: rel-L2 {err:.2e}", flush=True)
    assert err <= tol
    assert abs(float(logk) - lk_o) <= max(tol, 1e-6) * max(abs(lk_o), 1.0)
    assert np.all(G[:, -1] == 0)


@pytest.mark.parametrize("n,p,K", SPLIT)
def test_split_degenerate_shapes(lib, n, p, K):
    import torch
    prob = make_problem("c4_bf16", n=n, p=p, K=K)
    hi, lo = lib.split_bf16(torch.from_numpy(np.ascontiguousarray(prob.X64)).cuda())
    dp = lib.Problem(hi, torch.from_numpy(prob.y).cuda(), K, prob.prior, prob.prior_scale, True,
                     X_lo=lo)
    Bd = torch.from_numpy(make_random_state(prob, 0.3).astype(np.float32)).cuda()
    logk, G = lib.logpost_grad(dp, Bd)
    G = G.double().cpu().numpy()
    Bs = Bd.double().cpu().numpy()
    h, l = split.split_hilo(prob.X64)
    lk_o, G_o = oracle.log_kernel_and_grad(h + l, prob.y, Bs, prob.prior, prob.prior_scale, 1)
    err = _relL2(G, G_o)
    bound = 2.0 ** -14 * float(np.sum(np.max(np.abs(h + l) @ np.abs(Bs), axis=1))) + n * 1e-6
    print(f"[degenerate] bf16 n={n} p={p} K={K}: rel-L2 {err:.2e}", flush=True)
    assert err <= 6e-5
    assert abs(float(logk) - lk_o) <= bound
    assert np.all(G[:, -1] == 0)


def test_batched_degenerate_problems(lib):
    """A batch of 4 chains per problem whose problems have one row, one predictor or both,
    beside an ordinary one."""
    import torch
    shapes = [(1, 1, 2), (1, 300, 16), (130, 1, 3), (1, 1, 16), (700, 150, 9)]
    probs = [make_problem("c4_bf16", n=n, p=p, K=K, seed=[44, 1, i]) for i, (n, p, K) in enumerate(shapes)]
    dev = []
    for pr in probs:
        hi, lo = lib.split_bf16(torch.from_numpy(np.ascontiguousarray(pr.X64)).cuda())
        dev.append(lib.Problem(hi, torch.from_numpy(pr.y).cuda(), pr.K, pr.prior, pr.prior_scale,
                               True, X_lo=lo))
    bt = lib.Batch(dev, 4)
    B, G, logk = bt.zeros_state()
    for b, pr in enumerate(probs):
        for c in range(4):
            B[b][c].copy_(torch.from_numpy(make_random_state(pr, 0.3, seed=10 * b + c).astype(np.float32)))
    bt.logpost_grad(B, G, logk)
    lk = logk.cpu().numpy()
    for b, pr in enumerate(probs):
        h, l = split.split_hilo(pr.X64)
        for c in range(4):
            Bc = B[b][c].double().cpu().numpy()
            lk_o, G_o = oracle.log_kernel_and_grad(h + l, pr.y, Bc, pr.prior, pr.prior_scale, 1)
            Gd = G[b][c].double().cpu().numpy()
            err = _relL2(Gd, G_o)
            assert err <= 6e-5, f"problem {b} chain {c}: rel-L2 {err:.2e}"
            assert abs(lk[b, c] - lk_o) <= 1e-6 * abs(lk_o) + 1e-4
            assert np.all(Gd[:, -1] == 0)
    print(f"[degenerate] batched: {len(probs)} problems x 4 chains match the oracle", flush=True)
