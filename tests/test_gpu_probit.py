"""The probit link (binary y_i, P(y_i = 1) = Phi(x_i^T beta), one coefficient column) through
the same fused and wide-p passes, against the FP64 oracle's probit link (GPU tier).
Tolerances are those of the multinomial path: FP64 gradient rel-L2 <= 1e-12, FP32 <= 1e-5,
log K relative to max(1, |log K|) <= 1e-12 / 1e-6; replayed chains decide identically."""
import math

import numpy as np
import pytest

import oracle
from workloads import make_draws, make_probit

pytestmark = pytest.mark.gpu
PR = oracle.PROBIT


def _dev(lib, prob):
    import torch
    X = torch.from_numpy(np.asarray(prob.X)).cuda()
    y = torch.from_numpy(prob.y).cuda()
    return lib.Problem(X, y, 1, prob.prior, prob.prior_scale, False, link=lib.HMC_LINK_PROBIT)


def _relL2(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


@pytest.mark.parametrize("xfmt,n,p,gtol,ltol", [
    ("f64", 500, 20, 1e-12, 1e-12), ("f64", 1007, 130, 1e-12, 1e-12), ("f64", 33, 3000, 1e-12, 1e-12),
    ("f32", 3001, 1000, 1e-5, 1e-6), ("f32", 2050, 257, 1e-5, 1e-6), ("f32", 300, 5000, 1e-5, 1e-6),
    ("f32", 1, 7, 1e-5, 1e-6)])
@pytest.mark.parametrize("prior", [oracle.GAUSS, oracle.CAUCHY])
def test_probit_gradient_matches_oracle(lib, xfmt, n, p, gtol, ltol, prior):
    import torch
    prob = make_probit(n, p, seed=(7, n, p), xfmt=xfmt, prior=prior, prior_scale=0.7)
    dp = _dev(lib, prob)
    B = prob.B_true * 0.8
    Bd = torch.from_numpy(np.ascontiguousarray(B.astype(prob.state_dtype))).cuda()
    Bseen = Bd.double().cpu().numpy()
    logk, G = lib.logpost_grad(dp, Bd)
    lk_o, G_o = oracle.log_kernel_and_grad(prob.X64, prob.y, Bseen, prior, 0.7, 0, PR)
    err = _relL2(G.double().cpu().numpy(), G_o)
    lerr = abs(float(logk) - lk_o) / max(1.0, abs(lk_o))
    print(f"[probit] {xfmt} n={n} p={p}: grad rel-L2 {err:.2e}, log K rel {lerr:.2e}", flush=True)
    assert err <= gtol and lerr <= ltol


def test_probit_at_zero_closed_form(lib):
    # beta = 0: log K = -n log 2 and G = sqrt(2 / pi) X^T s (s = +1 for a success, -1 else)
    import torch
    rng = np.random.default_rng(3)
    n, p = 700, 40
    X = rng.integers(-3, 4, size=(n, p)).astype(np.float64)
    y = rng.integers(0, 2, size=n).astype(np.int32)
    dp = lib.Problem(torch.from_numpy(X).cuda(), torch.from_numpy(y).cuda(), 1, 0, 1.0, False,
                     link=lib.HMC_LINK_PROBIT)
    logk, G = lib.logpost_grad(dp, torch.zeros(p, 1, dtype=torch.float64, device="cuda"))
    assert float(logk) == pytest.approx(-n * math.log(2.0), rel=1e-14)
    ref = math.sqrt(2.0 / math.pi) * (X.T @ (2.0 * y - 1.0))
    np.testing.assert_allclose(G.cpu().numpy()[:, 0], ref, rtol=1e-14, atol=1e-12)


@pytest.mark.parametrize("xfmt", ["f64", "f32"])
def test_probit_far_tail_rows(lib, xfmt):
    # Rows whose z = x^T beta lies far on either side of the label (to |z| = 35): on the wrong
    # side the residual is about |z| and log Phi(s z) about -z^2 / 2, both finite, in FP32
    # too; on the right side both underflow towards 0. The oracle takes them through logs.
    import torch
    rng = np.random.default_rng(17)
    n, p = 600, 3
    zmax = 35.0
    X = np.zeros((n, p))
    X[:, 0] = np.linspace(-zmax, zmax, n)
    X[:, 1:] = rng.normal(size=(n, p - 1))
    y = rng.integers(0, 2, size=n).astype(np.int32)
    Xs = X.astype(np.float32) if xfmt == "f32" else X
    dt = torch.float32 if xfmt == "f32" else torch.float64
    dp = lib.Problem(torch.from_numpy(np.ascontiguousarray(Xs)).cuda(), torch.from_numpy(y).cuda(),
                     1, 0, 1.0, False, link=lib.HMC_LINK_PROBIT)
    B = np.array([[1.0], [0.0], [0.0]])
    logk, G = lib.logpost_grad(dp, torch.from_numpy(B).to(dt).cuda())
    lk_o, G_o = oracle.log_kernel_and_grad(Xs.astype(np.float64), y, B, 0, 1.0, 0, PR)
    g = G.double().cpu().numpy()
    assert np.all(np.isfinite(g)) and math.isfinite(float(logk))
    gtol, ltol = (1e-12, 1e-12) if xfmt == "f64" else (1e-5, 1e-6)
    assert _relL2(g, G_o) <= gtol
    assert abs(float(logk) - lk_o) / max(1.0, abs(lk_o)) <= ltol


def test_probit_sampler_replay_matches_oracle(lib):
    import torch
    prob = make_probit(400, 12, seed=(7, 1), xfmt="f64", eps=0.02, L=10)
    n_iter = 40
    d = make_draws(prob.p, 1, n_iter, seed=(7, 1, 0))
    dp = _dev(lib, prob)
    Bd = torch.zeros(prob.p, 1, dtype=torch.float64, device="cuda")
    logk, Gd = lib.logpost_grad(dp, Bd)
    out = lib.sample(dp, Bd, Gd, logk, prob.eps, prob.L, n_iter,
                     normals=torch.from_numpy(np.ascontiguousarray(d.xi)).cuda(),
                     uniforms=torch.from_numpy(np.ascontiguousarray(d.u)).cuda())
    torch.cuda.synchronize()
    dev = {k: v.cpu().numpy() for k, v in out.items() if v is not None}
    orc = oracle.sample(prob.X64, prob.y, 1, d.xi, d.u, prob.eps, prob.L, prob.prior,
                        prob.prior_scale, 0, link=PR)
    assert np.array_equal(dev["accepted"], orc["accepted"])
    assert dev["accepted"].mean() > 0.3
    assert np.max(np.abs(dev["samples"] - orc["samples"])) < 1e-10
    assert np.max(np.abs(dev["H"] - orc["H"])) < 1e-9


def test_probit_leapfrog_f32_matches_oracle(lib):
    import torch
    prob = make_probit(5000, 300, seed=(7, 2), xfmt="f32")
    dp = _dev(lib, prob)
    B = (prob.B_true * 0.9).astype(np.float32).astype(np.float64)
    eta = np.random.default_rng(5).normal(size=B.shape).astype(np.float32).astype(np.float64)
    Bd = torch.from_numpy(B.astype(np.float32)).cuda()
    logk, Gd = lib.logpost_grad(dp, Bd)
    ed = torch.from_numpy(eta.astype(np.float32)).cuda()
    lib.leapfrog(dp, Bd, ed, Gd, logk, 0.002, 8)
    G0 = oracle.grad_log_kernel(prob.X64, prob.y, B, prob.prior, prob.prior_scale, 0, PR)
    B1, e1, G1, lk1 = oracle.leapfrog(prob.X64, prob.y, B, eta, G0, 0.002, 8, prob.prior,
                                      prob.prior_scale, 0, PR)
    assert _relL2(Bd.double().cpu().numpy(), B1) < 1e-6
    assert _relL2(ed.double().cpu().numpy(), e1) < 1e-5
    assert _relL2(Gd.double().cpu().numpy(), G1) < 1e-5
    assert abs(float(logk) - lk1) / max(1.0, abs(lk1)) < 1e-6
