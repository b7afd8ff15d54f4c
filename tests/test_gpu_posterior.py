"""Posterior means of device chains vs an independent oracle chain (GPU tier).

Chains from different random streams agree only in distribution, so the comparison is
statistical: after discarding the first 20% of iterations, each coordinate's two posterior
means must agree within 3 sqrt(MCSE_dev^2 + MCSE_oracle^2), MCSE = sd / sqrt(ESS)
(Geyer's initial monotone sequence estimator; rank-normalised multi-chain ESS for the
batched chains). Every draw is seeded, so the outcome is deterministic; at most one
coordinate may exceed 3 (each does so with probability 0.27% by chance) and none may
exceed 4.
"""
import numpy as np
import pytest

import oracle
from oracle import philox
from paper_1402_4089_amd import diagnostics
from workloads import make_problem

pytestmark = pytest.mark.gpu


def _oracle_chain(prob, X64, n_iter, eps, L, seed):
    xis, us = philox.draws(seed, 0, n_iter, prob.p, prob.K)
    out = oracle.sample(X64, prob.y, prob.K, xis, us, eps, L, prob.prior, prob.prior_scale, 1)
    return out["samples"].reshape(n_iter, -1)


def _z(dev, dev_se, orc):
    keep = int(0.2 * len(orc))
    o = orc[keep:]
    se_o = o.std(axis=0) / np.sqrt(diagnostics.ess(o))
    return np.abs(dev - o.mean(axis=0)) / np.sqrt(dev_se ** 2 + se_o ** 2)


def _free(prob):
    f = np.ones((prob.p, prob.K), dtype=bool)
    f[:, -1] = False
    return f.reshape(-1)


def test_fp32_chain_posterior_means_match_oracle(lib):
    import torch
    prob = make_problem("c2_f32", n=300, p=4, K=3)
    eps, L, n_iter = 0.05, 10, 3000
    X = torch.from_numpy(prob.X).cuda()
    y = torch.from_numpy(prob.y).cuda()
    dp = lib.Problem(X, y, prob.K, prob.prior, prob.prior_scale, True)
    B = dp.zeros_state()
    logk, G = lib.logpost_grad(dp, B)
    out = lib.sample(dp, B, G, logk, eps, L, n_iter, seed=31, chain=5)
    s = out["samples"].double().cpu().numpy().reshape(n_iter, -1)[int(0.2 * n_iter):]
    free = _free(prob)
    s = s[:, free]
    se = s.std(axis=0) / np.sqrt(diagnostics.ess(s))
    orc = _oracle_chain(prob, prob.X64, n_iter, eps, L, seed=977)[:, free]
    z = _z(s.mean(axis=0), se, orc)
    print(f"[posterior] FP32 chain vs oracle: z = {np.round(z, 2)}, accept {float(out['accepted'].float().mean()):.3f}",
          flush=True)
    assert np.sum(z > 3) <= 1 and np.all(z < 4)


def test_batched_bf16_chains_posterior_means_match_oracle(lib):
    import torch
    from oracle import split
    prob = make_problem("c2_f32", n=300, p=4, K=3)
    eps, L, n_iter, chains = 0.05, 10, 1000, 4
    X = torch.from_numpy(prob.X).cuda()
    hi, lo = lib.split_bf16(X)
    y = torch.from_numpy(prob.y).cuda()
    bt = lib.Batch([lib.Problem(hi, y, prob.K, prob.prior, prob.prior_scale, True, X_lo=lo)], chains)
    B, G, logk = bt.zeros_state()
    bt.logpost_grad(B, G, logk)
    out = bt.sample(B, G, logk, [eps], L, n_iter, seed=44, record_samples=True)
    smp = out["samples"][0].double().cpu().numpy()              # [n_iter, chains, p, K]
    free = _free(prob)
    smp = smp.reshape(n_iter, chains, -1)[int(0.2 * n_iter):, :, free]
    m = smp.mean(axis=(0, 1))
    se = smp.std(axis=(0, 1)) / np.sqrt(diagnostics.multichain_ess(np.transpose(smp, (1, 0, 2))))
    h, l = split.split_hilo(prob.X64)
    orc = _oracle_chain(prob, h + l, 4 * n_iter, eps, L, seed=978)[:, free]
    z = _z(m, se, orc)
    print(f"[posterior] batched bf16 chains vs oracle: z = {np.round(z, 2)}", flush=True)
    assert np.sum(z > 3) <= 1 and np.all(z < 4)
