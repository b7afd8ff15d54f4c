"""Split-precision (bfloat16 hi + lo) form vs the FP64 oracle (GPU tier).

The device encodes X itself (hmc_split_bf16); that encoding must equal the oracle's
definition bit for bit. The oracle then runs in FP64 on the values the device sees,
X_eff = hi + lo (or hi alone for the hi-only form), so the measured error is that of the
device arithmetic: three-term bf16 products of X with the split FP32 operands, FP32
accumulation, FP64 softmax statistics.

Tolerances (derived from the arithmetic): each product hi*A_hi + hi*A_lo + lo*A_hi of an
FP32 operand A = A_hi + A_lo + r drops lo*A_lo and X*r, both at most 2^-16 of |x a|, so a
sum's error is at most 2^-15 of the sum of absolute terms and about 2^-16 of the root sum
of squares when the rounding signs are random. Gradient relative L2 error: <= 6e-5
(about four times 2^-16, to cover the FP32 accumulation over row slices).
log K: |error| <= 2^-14 * sum_i max_k sum_j |x_ij b_jk| + n * 1e-6 (twice the logit bound
per row, plus the FP32 exponentials inside the FP64 log-sum-exp).
"""
import numpy as np
import pytest

import oracle
from oracle import split
from workloads import make_draws, make_problem, make_random_state

pytestmark = pytest.mark.gpu

GTOL = 6e-5


def _planes(lib, prob, hi_only=False):
    import torch
    X = torch.from_numpy(np.ascontiguousarray(prob.X64)).cuda()
    hi, lo = lib.split_bf16(X, hi_only=hi_only)
    del X
    return hi, lo


def _dev(lib, prob, hi_only=False):
    import torch
    hi, lo = _planes(lib, prob, hi_only)
    y = torch.from_numpy(prob.y).cuda()
    return lib.Problem(hi, y, prob.K, prob.prior, prob.prior_scale, bool(prob.pin_last_class), X_lo=lo)


def _x_eff(prob, hi_only=False):
    hi, lo = split.split_hilo(prob.X64)
    return hi if hi_only else hi + lo


def _relL2(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def _logk_bound(Xe, B):
    return 2.0 ** -14 * float(np.sum(np.max(np.abs(Xe) @ np.abs(B), axis=1))) + Xe.shape[0] * 1e-6


def _check(lib, prob, B64, hi_only=False):
    import torch
    dp = _dev(lib, prob, hi_only)
    Bd = torch.from_numpy(np.ascontiguousarray(B64.astype(np.float32))).cuda()
    Bseen = Bd.double().cpu().numpy()
    logk, G = lib.logpost_grad(dp, Bd)
    G = G.double().cpu().numpy()
    Xe = _x_eff(prob, hi_only)
    lk_o, G_o = oracle.log_kernel_and_grad(Xe, prob.y, Bseen, prob.prior, prob.prior_scale,
                                           prob.pin_last_class)
    err = _relL2(G, G_o)
    lerr = abs(float(logk) - lk_o)
    bound = _logk_bound(Xe, Bseen)
    print(f"[bf16] n={prob.n} p={prob.p} K={prob.K} hi_only={hi_only}: grad rel-L2 {err:.3e}, "
          f"|dlogK| {lerr:.3e} (bound {bound:.3e})", flush=True)
    assert err <= GTOL, f"gradient rel-L2 {err:.3e}"
    assert lerr <= bound, f"log K error {lerr:.3e} > {bound:.3e}"
    if prob.pin_last_class:
        assert np.all(G[:, -1] == 0)
    return err, lerr


@pytest.mark.parametrize("src", ["f64", "f32"])
def test_split_matches_oracle_bitwise(lib, src):
    import torch
    rng = np.random.default_rng(11)
    n, p = 37, 45
    X = rng.standard_normal((n, p)) * np.exp(rng.uniform(-30, 30, (n, p)))
    # exact ties of 8 significant bits, a float64-only near-tie, zeros and tiny values
    X[0, :8] = [1 + 2.0 ** -8, 1 + 3 * 2.0 ** -8, -(1 + 2.0 ** -8 + 2.0 ** -40), 0.0, -0.0,
                3 * 2.0 ** -134, 2.0 ** -140, 1e-300]
    if src == "f32":
        X = X.astype(np.float32)
    Xd = torch.from_numpy(X).cuda()
    ldo = 48
    hi = torch.full((n, ldo), 0x5555, dtype=torch.int16, device="cuda")
    lo = torch.full((n, ldo), 0x5555, dtype=torch.int16, device="cuda")
    lib.hmc_split_bf16(Xd, lib.HMC_X_F64 if src == "f64" else lib.HMC_X_F32, n, p, p, hi, lo, ldo)
    hb = hi.cpu().numpy().view(np.uint16)
    lb = lo.cpu().numpy().view(np.uint16)
    ho, lo_ = split.split_hilo(X.astype(np.float64))
    assert np.array_equal(hb[:, :p], split.bf16_bits(ho))
    assert np.array_equal(lb[:, :p], split.bf16_bits(lo_))
    assert np.all(hb[:, p:] == 0) and np.all(lb[:, p:] == 0)


BF16_SHAPES = [(300, 70, 5), (1000, 130, 17), (777, 200, 40), (129, 33, 64), (2050, 256, 64),
               (31, 8, 2), (1, 3, 2), (5000, 1000, 10)]


@pytest.mark.parametrize("shape", BF16_SHAPES)
@pytest.mark.parametrize("prior,pin", [(oracle.GAUSS, 1), (oracle.CAUCHY, 0)])
def test_logpost_grad_bf16_hilo(lib, shape, prior, pin):
    n, p, K = shape
    prob = make_problem("c4_bf16", n=n, p=p, K=K, prior=prior, pin_last_class=pin)
    _check(lib, prob, make_random_state(prob, 0.1))


@pytest.mark.parametrize("n", [100003, 150001])
def test_logpost_grad_bf16_many_row_blocks(lib, n):
    # Some 800 and 1200 logits row blocks (several rounds of the resident workgroups, the
    # last one partly filled), ragged n and p
    prob = make_problem("c4_bf16", n=n, p=70, K=10)
    _check(lib, prob, make_random_state(prob, 0.1))


@pytest.mark.parametrize("shape", [(300, 70, 5), (2050, 256, 64), (1000, 130, 17)])
def test_logpost_grad_bf16_hi_only(lib, shape):
    n, p, K = shape
    prob = make_problem("c4_bf16", n=n, p=p, K=K)
    _check(lib, prob, make_random_state(prob, 0.1), hi_only=True)


def test_bf16_gradient_at_zero_and_determinism(lib):
    """At B = 0 every logit is 0 exactly, so the only error is the residual split."""
    import torch
    prob = make_problem("c4_bf16", n=3000, p=300, K=32)
    dp = _dev(lib, prob)
    Bd = torch.zeros(prob.p, prob.K, dtype=torch.float32, device="cuda")
    l1, G1 = lib.logpost_grad(dp, Bd)
    l2, G2 = lib.logpost_grad(dp, Bd)
    assert torch.equal(G1, G2) and float(l1) == float(l2)
    assert abs(float(l1) - (-prob.n * np.log(prob.K))) <= 1e-9 * prob.n
    lk_o, G_o = oracle.log_kernel_and_grad(_x_eff(prob), prob.y, np.zeros((prob.p, prob.K)))
    assert _relL2(G1.double().cpu().numpy(), G_o) <= GTOL


def test_bf16_leapfrog_matches_oracle(lib):
    import torch
    prob = make_problem("c4_bf16", n=2000, p=200, K=16)
    B = make_random_state(prob, 0.05)
    eta = np.random.default_rng(8).normal(size=B.shape) * oracle.free_mask(prob.p, prob.K, 1)
    eta = eta.astype(np.float32).astype(np.float64)
    dp = _dev(lib, prob)
    Bd = torch.from_numpy(B.astype(np.float32)).cuda()
    logk, Gd = lib.logpost_grad(dp, Bd)
    ed = torch.from_numpy(eta.astype(np.float32)).cuda()
    lib.leapfrog(dp, Bd, ed, Gd, logk, 0.002, 8)
    Xe = _x_eff(prob)
    G0 = oracle.grad_log_kernel(Xe, prob.y, B)
    B1, e1, G1, lk1 = oracle.leapfrog(Xe, prob.y, B, eta, G0, 0.002, 8)
    eB, ee, eG = (_relL2(Bd.double().cpu().numpy(), B1), _relL2(ed.double().cpu().numpy(), e1),
                  _relL2(Gd.double().cpu().numpy(), G1))
    print(f"[bf16] leapfrog rel-L2 B {eB:.2e} eta {ee:.2e} G {eG:.2e}", flush=True)
    assert eB < 1e-6 and ee < GTOL and eG < GTOL
    assert abs(float(logk) - lk1) <= _logk_bound(Xe, B1)


@pytest.mark.parametrize("K,hi_only", [(16, False), (40, False), (9, True)])
def test_bf16_epilogue_packing_equals_the_pack_pass(lib, K, hi_only):
    """Within a leapfrog run the epilogue of each update writes the next pass's packed B
    operand (no pack pass of its own). The gradient and log K the run leaves at its final
    position must equal, bit for bit, those of a fresh evaluation there, which packs B with
    the pack pass."""
    import torch
    prob = make_problem("c4_bf16", n=1500, p=130, K=K)
    B = make_random_state(prob, 0.05)
    eta = np.random.default_rng(9).normal(size=B.shape) * oracle.free_mask(prob.p, prob.K, 1)
    X = torch.from_numpy(prob.X64).cuda()
    hi, lo = lib.split_bf16(X, hi_only=hi_only)
    y = torch.from_numpy(prob.y).cuda()
    dp = lib.Problem(hi, y, prob.K, prob.prior, prob.prior_scale, True, X_lo=lo)
    Bd = torch.from_numpy(B.astype(np.float32)).cuda()
    logk, Gd = lib.logpost_grad(dp, Bd)
    ed = torch.from_numpy(eta.astype(np.float32)).cuda()
    lib.leapfrog(dp, Bd, ed, Gd, logk, 0.002, 6)
    logk2, G2 = lib.logpost_grad(dp, Bd)
    torch.cuda.synchronize()
    assert torch.equal(Gd, G2)
    assert float(logk) == float(logk2)


def test_bf16_accept_decisions_trajectories(lib):
    """60 independent 10-step trajectories from a common oracle state: same decisions
    outside the tie band; the energy change agrees within the band."""
    import torch
    prob = make_problem("c4_bf16", n=4000, p=256, K=16)
    Xe = _x_eff(prob)
    burn = make_draws(prob.p, prob.K, 120, seed=(4, 7, 0))
    base = oracle.sample(Xe, prob.y, prob.K, burn.xi, burn.u, 0.006, 10)["B"]
    B = base.astype(np.float32).astype(np.float64)
    G0 = oracle.grad_log_kernel(Xe, prob.y, B)
    lk0 = oracle.log_kernel(Xe, prob.y, B)
    dp = _dev(lib, prob)
    rng = np.random.default_rng(99)
    eps, L, band = 0.02, 10, 5e-3
    agree = ties = accepted = 0
    for trial in range(60):
        xi = rng.normal(size=(1, prob.p, prob.K))
        u = rng.random(1) * 0.999 + 0.0005
        Bd = torch.from_numpy(B.astype(np.float32)).cuda()
        logk, Gd = lib.logpost_grad(dp, Bd)
        out = lib.sample(dp, Bd, Gd, logk, eps, L, 1,
                         normals=torch.from_numpy(xi).cuda(), uniforms=torch.from_numpy(u).cuda())
        acc_d = int(out["accepted"].cpu()[0])
        H_d = out["H"].cpu().numpy()[0]
        r = oracle.hmc_iteration(Xe, prob.y, B, G0, lk0, xi[0], u[0], eps, L)
        margin = abs(np.log(u[0]) - (r["H0"] - r["H1"]))
        dH_err = abs((H_d[0] - H_d[1]) - (r["H0"] - r["H1"]))
        assert dH_err < band, f"trial {trial}: delta-H differs by {dH_err}"
        if margin <= band:
            ties += 1
            continue
        agree += int(acc_d == int(r["accepted"]))
        accepted += int(r["accepted"])
    assert agree == 60 - ties
    assert 5 < accepted < 57 - ties


@pytest.mark.slow
def test_full_c4_gradient(lib, tmp_path, monkeypatch):
    """Precision form at full size (n=200000, p=4096, K=64, hi + lo) at a random state, in
    the built-in rule's decomposition and in the one the autotuner measures (as the
    benchmark does before timing; a private cache, so it measures here); also reports the
    error against the unsplit float64 X (the encoding's own contribution)."""
    import torch
    from paper_1402_4089_amd import tuning
    monkeypatch.setenv(tuning.ENV, str(tmp_path / "cache.json"))
    prob = make_problem("c4_bf16")
    B = make_random_state(prob, 0.02)
    hi, lo = _planes(lib, prob)
    y = torch.from_numpy(prob.y).cuda()
    Bd = torch.from_numpy(B.astype(np.float32)).cuda()
    results = []
    for tn in (None, "auto"):
        dp = lib.Problem(hi, y, prob.K, prob.prior, prob.prior_scale, True, X_lo=lo, tuning=tn)
        logk, G = lib.logpost_grad(dp, Bd)
        results.append((dp.tuning, float(logk), G.double().cpu().numpy()))
    Xe = _x_eff(prob)
    lk_o, G_o = oracle.log_kernel_and_grad(Xe, prob.y, B)
    bound = _logk_bound(Xe, B)
    del Xe
    lk_x, G_x = oracle.log_kernel_and_grad(prob.X64, prob.y, B)
    for tn, logk, G in results:
        err = _relL2(G, G_o)
        lerr = abs(logk - lk_o)
        print(f"[bf16] full C4 {tn}: grad rel-L2 {err:.3e} vs X_eff, {_relL2(G, G_x):.3e} vs "
              f"float64 X; |dlogK| {lerr:.3e} vs X_eff, {abs(logk - lk_x):.3e} vs float64 X", flush=True)
        assert err <= GTOL
        assert lerr <= bound
