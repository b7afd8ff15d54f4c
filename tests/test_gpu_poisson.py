"""The Poisson-regression link (y_i ~ Poisson(exp(x_i^T beta)), one coefficient column)
through the same fused and wide-p passes, against the FP64 oracle's Poisson link (GPU tier).
Tolerances are those of the multinomial path: FP64 gradient rel-L2 <= 1e-12, FP32 <= 1e-5,
log K relative to max(1, |log K|) <= 1e-12 / 1e-6; replayed chains decide identically."""
import numpy as np
import pytest

import oracle
from workloads import make_draws, make_poisson

pytestmark = pytest.mark.gpu
P = oracle.POISSON


def _dev(lib, prob):
    import torch
    X = torch.from_numpy(np.asarray(prob.X)).cuda()
    y = torch.from_numpy(prob.y).cuda()
    return lib.Problem(X, y, 1, prob.prior, prob.prior_scale, False, link=lib.HMC_LINK_POISSON)


def _relL2(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


@pytest.mark.parametrize("xfmt,n,p,gtol,ltol", [
    ("f64", 500, 20, 1e-12, 1e-12), ("f64", 1007, 130, 1e-12, 1e-12), ("f64", 33, 3000, 1e-12, 1e-12),
    ("f32", 3001, 1000, 1e-5, 1e-6), ("f32", 2050, 257, 1e-5, 1e-6), ("f32", 300, 5000, 1e-5, 1e-6),
    ("f32", 1, 7, 1e-5, 1e-6)])
@pytest.mark.parametrize("prior", [oracle.GAUSS, oracle.CAUCHY])
def test_poisson_gradient_matches_oracle(lib, xfmt, n, p, gtol, ltol, prior):
    import torch
    prob = make_poisson(n, p, seed=(6, n, p), xfmt=xfmt, prior=prior, prior_scale=0.7)
    dp = _dev(lib, prob)
    B = prob.B_true * 0.8
    Bd = torch.from_numpy(np.ascontiguousarray(B.astype(prob.state_dtype))).cuda()
    Bseen = Bd.double().cpu().numpy()
    logk, G = lib.logpost_grad(dp, Bd)
    lk_o, G_o = oracle.log_kernel_and_grad(prob.X64, prob.y, Bseen, prior, 0.7, 0, P)
    err = _relL2(G.double().cpu().numpy(), G_o)
    lerr = abs(float(logk) - lk_o) / max(1.0, abs(lk_o))
    print(f"[poisson] {xfmt} n={n} p={p}: grad rel-L2 {err:.2e}, log K rel {lerr:.2e}", flush=True)
    assert err <= gtol and lerr <= ltol


def test_poisson_gradient_at_zero_exact(lib):
    # beta = 0: log K = -n and G = X^T (y - 1), exact for small-integer X in FP64
    import torch
    rng = np.random.default_rng(3)
    n, p = 700, 40
    X = rng.integers(-3, 4, size=(n, p)).astype(np.float64)
    y = rng.integers(0, 6, size=n).astype(np.int32)
    dp = lib.Problem(torch.from_numpy(X).cuda(), torch.from_numpy(y).cuda(), 1, 0, 1.0, False,
                     link=lib.HMC_LINK_POISSON)
    logk, G = lib.logpost_grad(dp, torch.zeros(p, 1, dtype=torch.float64, device="cuda"))
    assert float(logk) == -float(n)
    assert np.array_equal(G.cpu().numpy()[:, 0], X.T @ (y - 1.0))


def test_poisson_sampler_replay_matches_oracle(lib):
    import torch
    prob = make_poisson(400, 12, seed=(6, 1), xfmt="f64", eps=0.01, L=10)
    n_iter = 40
    d = make_draws(prob.p, 1, n_iter, seed=(6, 1, 0))
    dp = _dev(lib, prob)
    Bd = torch.zeros(prob.p, 1, dtype=torch.float64, device="cuda")
    logk, Gd = lib.logpost_grad(dp, Bd)
    out = lib.sample(dp, Bd, Gd, logk, prob.eps, prob.L, n_iter,
                     normals=torch.from_numpy(np.ascontiguousarray(d.xi)).cuda(),
                     uniforms=torch.from_numpy(np.ascontiguousarray(d.u)).cuda())
    torch.cuda.synchronize()
    dev = {k: v.cpu().numpy() for k, v in out.items() if v is not None}
    orc = oracle.sample(prob.X64, prob.y, 1, d.xi, d.u, prob.eps, prob.L, prob.prior,
                        prob.prior_scale, 0, link=P)
    assert np.array_equal(dev["accepted"], orc["accepted"])
    assert dev["accepted"].mean() > 0.3
    assert np.max(np.abs(dev["samples"] - orc["samples"])) < 1e-10
    assert np.max(np.abs(dev["H"] - orc["H"])) < 1e-9


def test_poisson_leapfrog_f32_matches_oracle(lib):
    import torch
    prob = make_poisson(5000, 300, seed=(6, 2), xfmt="f32")
    dp = _dev(lib, prob)
    B = (prob.B_true * 0.9).astype(np.float32).astype(np.float64)
    eta = np.random.default_rng(5).normal(size=B.shape).astype(np.float32).astype(np.float64)
    Bd = torch.from_numpy(B.astype(np.float32)).cuda()
    logk, Gd = lib.logpost_grad(dp, Bd)
    ed = torch.from_numpy(eta.astype(np.float32)).cuda()
    lib.leapfrog(dp, Bd, ed, Gd, logk, 0.002, 8)
    G0 = oracle.grad_log_kernel(prob.X64, prob.y, B, prob.prior, prob.prior_scale, 0, P)
    B1, e1, G1, lk1 = oracle.leapfrog(prob.X64, prob.y, B, eta, G0, 0.002, 8, prob.prior,
                                      prob.prior_scale, 0, P)
    assert _relL2(Bd.double().cpu().numpy(), B1) < 1e-6
    assert _relL2(ed.double().cpu().numpy(), e1) < 1e-5
    assert _relL2(Gd.double().cpu().numpy(), G1) < 1e-5
    assert abs(float(logk) - lk1) / max(1.0, abs(lk1)) < 1e-6
