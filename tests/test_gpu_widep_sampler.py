"""The wide-p path with one row slice, and graph plans, against the FP64 oracle (GPU tier).

When the wide-p gradient kernel has 512 or more workgroups of 16-column blocks (p > 32,768
in FP64 with one class block, p > 65,536 in FP32), it runs with a single row slice and applies the leapfrog epilogue
itself: the closing and opening half kicks of equations (hmc1)-(hmc3), the position step, the prior and
mask, and the kinetic-energy partials of equation (accept). The autotuner may also choose
one slice for the high-dimensional workload (n=2000, p=50000, K=4, FP32), whose rule gives two
slices and the shared epilogue; both branches run here. These tests drive them in leapfrog
and sampler mode, and check replayed graph plans against the oracle chain itself.
"""
import numpy as np
import pytest

import oracle
from workloads import make_draws, make_problem

pytestmark = pytest.mark.gpu

# n = 40 rows, p = 33000 (2063 blocks of 16 columns, 512 workgroups: one row slice), K = 4, FP64.
WIDE1 = dict(n=40, p=33000, K=4)


def _relL2(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def _dev(lib, prob):
    import torch
    X = torch.from_numpy(np.asarray(prob.X)).cuda()
    y = torch.from_numpy(prob.y).cuda()
    return lib.Problem(X, y, prob.K, prob.prior, prob.prior_scale, bool(prob.pin_last_class))


def _state(prob, B64):
    import torch
    return torch.from_numpy(np.ascontiguousarray(B64.astype(prob.state_dtype))).cuda()


def test_wide_one_slice_leapfrog_f64(lib):
    import torch
    prob = make_problem("c1_small_f64", **WIDE1)
    rng = np.random.default_rng(41)
    B = rng.normal(0.0, 0.02, size=(prob.p, prob.K)) * oracle.free_mask(prob.p, prob.K, 1)
    eta = rng.normal(size=B.shape) * oracle.free_mask(prob.p, prob.K, 1)
    dp = _dev(lib, prob)
    Bd = _state(prob, B)
    logk, Gd = lib.logpost_grad(dp, Bd)
    ed = torch.from_numpy(eta.copy()).cuda()
    lib.leapfrog(dp, Bd, ed, Gd, logk, 0.01, 6)
    G0 = oracle.grad_log_kernel(prob.X64, prob.y, B)
    B1, e1, G1, lk1 = oracle.leapfrog(prob.X64, prob.y, B, eta, G0, 0.01, 6)
    eb, ee, eg = _relL2(Bd.cpu().numpy(), B1), _relL2(ed.cpu().numpy(), e1), _relL2(Gd.cpu().numpy(), G1)
    print(f"[wide1 leapfrog] rel-L2 B {eb:.2e} eta {ee:.2e} G {eg:.2e}", flush=True)
    assert eb < 1e-12 and ee < 1e-12 and eg < 1e-12
    assert abs(float(logk) - lk1) < 1e-12 * abs(lk1)
    assert np.all(Gd.cpu().numpy()[:, -1] == 0) and np.all(Bd.cpu().numpy()[:, -1] == 0)


def test_wide_one_slice_sampler_f64_replay(lib):
    """hmc_sample with replayed draws through the one-slice branch: identical decisions,
    samples within 1e-10, (H0, H1) within 1e-9. eps = 0.01, L = 6 gives a mix of accepts and
    rejects on this shape (the oracle rejects iterations 0 and 17 of 20)."""
    import torch
    prob = make_problem("c1_small_f64", **WIDE1)
    n_iter, eps, L = 20, 0.01, 6
    d = make_draws(prob.p, prob.K, n_iter, seed=(3, 3, 0))
    dp = _dev(lib, prob)
    Bd = _state(prob, np.zeros((prob.p, prob.K)))
    logk, Gd = lib.logpost_grad(dp, Bd)
    out = lib.sample(dp, Bd, Gd, logk, eps, L, n_iter, normals=torch.from_numpy(d.xi).cuda(),
                     uniforms=torch.from_numpy(d.u).cuda())
    torch.cuda.synchronize()
    orc = oracle.sample(prob.X64, prob.y, prob.K, d.xi, d.u, eps, L)
    acc = out["accepted"].cpu().numpy()
    assert np.array_equal(acc, orc["accepted"])
    assert 0 < acc.sum() < n_iter
    assert np.max(np.abs(out["samples"].cpu().numpy() - orc["samples"])) < 1e-10
    assert np.max(np.abs(out["H"].cpu().numpy() - orc["H"])) < 1e-9
    assert abs(float(logk) - orc["logk"]) < 1e-10 * abs(orc["logk"])


def test_c3_fp32_trajectory_decisions(lib):
    """The full high-dimensional workload (n=2000, p=50000, K=4, FP32, N(0, 0.1^2) prior):
    20 independent 10-step trajectories from B = 0, each with its own momentum and uniform,
    on the device and in the oracle. The FP32 energy difference must agree with the oracle's
    within DH_TOL, and decisions must be identical outside that tie band. At eps = 0.001 the
    oracle's H0 - H1 is about -1.6 to -2.1 here, so with uniform u both outcomes occur."""
    import torch
    prob = make_problem("c3_widep")
    X64 = prob.X64
    eps, L, trials = 1e-3, 10, 20
    DH_TOL = 2e-2
    B = np.zeros((prob.p, prob.K))
    G0 = oracle.grad_log_kernel(X64, prob.y, B, prob.prior, prob.prior_scale)
    lk0 = oracle.log_kernel(X64, prob.y, B, prob.prior, prob.prior_scale)
    dp = _dev(lib, prob)
    rng = np.random.default_rng(5003)
    agree = ties = accepted = 0
    worst = 0.0
    for trial in range(trials):
        xi = rng.normal(size=(1, prob.p, prob.K))
        u = rng.random(1) * 0.5 + 0.01
        Bd = _state(prob, B)
        logk, Gd = lib.logpost_grad(dp, Bd)
        out = lib.sample(dp, Bd, Gd, logk, eps, L, 1, normals=torch.from_numpy(xi).cuda(),
                         uniforms=torch.from_numpy(u).cuda(), record_samples=False)
        acc_d = int(out["accepted"].cpu()[0])
        H_d = out["H"].cpu().numpy()[0]
        r = oracle.hmc_iteration(X64, prob.y, B, G0, lk0, xi[0], u[0], eps, L, prob.prior,
                                 prob.prior_scale)
        dH_err = abs((H_d[0] - H_d[1]) - (r["H0"] - r["H1"]))
        worst = max(worst, dH_err)
        assert dH_err < DH_TOL, f"trial {trial}: delta-H differs by {dH_err}"
        if abs(np.log(u[0]) - (r["H0"] - r["H1"])) <= DH_TOL:
            ties += 1
            continue
        agree += int(acc_d == int(r["accepted"]))
        accepted += int(r["accepted"])
    print(f"[c3 trajectories] worst delta-H error {worst:.2e}, ties {ties}, accepted {accepted}",
          flush=True)
    assert agree == trials - ties
    assert 0 < accepted < trials - ties


@pytest.mark.parametrize("shape", ["fused", "wide"])
def test_plan_replay_matches_oracle(lib, shape):
    """A graph plan with replayed draws, launched in two parts (7 + 13 iterations), against
    the oracle chain driven by the same draws: identical decisions, samples within 1e-10."""
    import torch
    if shape == "fused":
        prob = make_problem("c1_small_f64")
        eps, L = prob.eps, prob.L
    else:
        prob = make_problem("c1_small_f64", **WIDE1)
        eps, L = 0.01, 6
    n_iter = 20
    d = make_draws(prob.p, prob.K, n_iter, seed=(3, 3, 0))
    dp = _dev(lib, prob)
    Bd = _state(prob, np.zeros((prob.p, prob.K)))
    logk, Gd = lib.logpost_grad(dp, Bd)
    plan, out = lib.plan(dp, Bd, Gd, logk, eps, L, n_iter, normals=torch.from_numpy(d.xi).cuda(),
                         uniforms=torch.from_numpy(d.u).cuda())
    plan.launch(7)
    torch.cuda.synchronize()
    plan.launch(13)
    torch.cuda.synchronize()
    plan.destroy()
    orc = oracle.sample(prob.X64, prob.y, prob.K, d.xi, d.u, eps, L)
    acc = out["accepted"].cpu().numpy()
    assert np.array_equal(acc, orc["accepted"])
    assert 0 < acc.sum()
    assert np.max(np.abs(out["samples"].cpu().numpy() - orc["samples"])) < 1e-10
    assert np.max(np.abs(out["H"].cpu().numpy() - orc["H"])) < 1e-9
    assert abs(float(logk) - orc["logk"]) < 1e-10 * abs(orc["logk"])
