"""torch.autograd.Function wrapper: backward is the hand-written device gradient."""
import numpy as np
import pytest

import oracle
from workloads import make_problem, make_random_state

pytestmark = pytest.mark.gpu


def _dev(lib, prob, pin):
    import torch
    X = torch.from_numpy(np.asarray(prob.X)).cuda()
    y = torch.from_numpy(prob.y).cuda()
    return lib.Problem(X, y, prob.K, prob.prior, prob.prior_scale, pin)


def test_gradcheck_fp64_unpinned(lib):
    import torch
    prob = make_problem("c1_small_f64", n=60, p=5, K=3, prior=oracle.CAUCHY, pin_last_class=0)
    dp = _dev(lib, prob, False)
    B = torch.from_numpy(make_random_state(prob, 0.3)).cuda().requires_grad_(True)
    f = lambda b: lib.LogPosterior.apply(b, dp)
    assert torch.autograd.gradcheck(f, (B,), eps=1e-6, atol=1e-7, rtol=1e-6)


def test_backward_matches_oracle_and_chain_rule(lib):
    import torch
    prob = make_problem("c1_small_f64", n=200, p=12, K=4)
    dp = _dev(lib, prob, True)
    B0 = make_random_state(prob, 0.2)
    B = torch.from_numpy(B0).cuda().requires_grad_(True)
    out = 3.0 * lib.LogPosterior.apply(B, dp)
    out.backward()
    G_o = oracle.grad_log_kernel(prob.X64, prob.y, B0)
    assert np.allclose(B.grad.cpu().numpy(), 3.0 * G_o, rtol=1e-12, atol=1e-10)
    assert float(out) == pytest.approx(3.0 * oracle.log_kernel(prob.X64, prob.y, B0), rel=1e-13)


def test_fp32_autograd_vs_finite_differences_64_coords(lib):
    """Plain FP32 workload n=20000, p=1000, K=10: autograd gradient vs central differences
    of the FP64 log-posterior on 64 seeded free coordinates."""
    import torch
    prob = make_problem("c2_f32")
    dp = _dev(lib, prob, True)
    B0 = make_random_state(prob, 0.05)
    B = torch.from_numpy(B0.astype(np.float32)).cuda().requires_grad_(True)
    lib.LogPosterior.apply(B, dp).backward()
    G = B.grad.double().cpu().numpy()
    Bs = B0.astype(np.float32).astype(np.float64)
    rng = np.random.default_rng(64)
    scale = np.linalg.norm(G) / np.sqrt(G.size)
    for j, k in zip(rng.integers(0, prob.p, 64), rng.integers(0, prob.K - 1, 64)):
        vals = []
        for h in (1e-4, 5e-5):
            Bp = Bs.copy(); Bp[j, k] += h
            Bm = Bs.copy(); Bm[j, k] -= h
            vals.append((oracle.log_kernel(prob.X64, prob.y, Bp) - oracle.log_kernel(prob.X64, prob.y, Bm)) / (2 * h))
        fd = (4 * vals[1] - vals[0]) / 3
        assert abs(G[j, k] - fd) <= 1e-5 * scale + 1e-4 * abs(fd)
