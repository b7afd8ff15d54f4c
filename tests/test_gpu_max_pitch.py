"""Problems at the largest row pitch the boundary accepts, row padding filled with NaN (GPU tier).

The kernels address X through 32-bit byte offsets from the first row of a row group (16 rows
in the row tile, 64 in the wide-p gradient, 128 in the split-precision logits), so the row
pitch is bounded: 2^24 - 1 elements for FP32, 2^23 - 1 for FP64, 2^23 - 8 for the bf16
planes (hmc_max_p reports these). At exactly that pitch the farthest offsets come within a
row of 2^32 bytes, and X itself spans more than 4 GB, so the loads that read past column p
(the tail of the last column chunk or k step) land inside the buffer instead of past its
end. Here every padding element (columns p .. ldx - 1 of every row) is NaN: the gradient
and log K of equations (logkernel) and (fullgrad) must match the FP64 oracle at the parity
tolerance of the format, which also shows that no padding element reaches the result (a
single one would make it NaN). Shapes have a ragged last row group and a ragged last column
block.
"""
import numpy as np
import pytest

import oracle
from gradbound import UNIT_ROUNDOFF, assert_elementwise
from oracle import split
from workloads import make_problem, make_random_state

pytestmark = pytest.mark.gpu

PITCH = {"f32": (1 << 24) - 1, "f64": (1 << 23) - 1, "bf16": (1 << 23) - 8}

# (format, n, p, K, path): path 1 = row tile, 2 = wide p, 0 = the rule's choice
PLAIN = [("f32", 70, 1000, 10, 1), ("f32", 70, 1000, 10, 2), ("f32", 70, 2001, 4, 0),
         ("f64", 70, 300, 7, 1), ("f64", 70, 601, 3, 0)]
# (n, p, K, hi_only): split-precision planes
SPLIT = [(130, 1001, 20, False), (130, 77, 5, True)]


def _relL2(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


@pytest.mark.parametrize("fmt,n,p,K,path", PLAIN)
def test_plain_formats_at_max_pitch(lib, fmt, n, p, K, path):
    import torch
    ldx = PITCH[fmt]
    assert lib.hmc_max_p(lib.HMC_X_F32 if fmt == "f32" else lib.HMC_X_F64, K) == min((1 << 30) // K, ldx)
    prob = make_problem("c2_f32" if fmt == "f32" else "c1_small_f64", n=n, p=p, K=K)
    dt = torch.float32 if fmt == "f32" else torch.float64
    big = torch.full((n, ldx), float("nan"), dtype=dt, device="cuda")
    big[:, :p].copy_(torch.from_numpy(np.ascontiguousarray(prob.X)))
    X = big[:, :p]
    assert X.stride(0) == ldx
    tuning = None if path == 0 else dict(path=path)
    dp = lib.Problem(X, torch.from_numpy(prob.y).cuda(), K, prob.prior, prob.prior_scale, True,
                     **({} if tuning is None else dict(tuning=tuning)))
    B64 = make_random_state(prob, 0.05 if fmt == "f32" else 0.2)
    Bd = torch.from_numpy(B64.astype(prob.state_dtype)).cuda()
    logk, G = lib.logpost_grad(dp, Bd)
    G = G.double().cpu().numpy()
    Bs = Bd.double().cpu().numpy()
    lk_o, G_o = oracle.log_kernel_and_grad(prob.X64, prob.y, Bs, prob.prior, prob.prior_scale, 1)
    tol = 1e-12 if fmt == "f64" else 1e-5
    err = _relL2(G, G_o)
    print(f"[max pitch] {fmt} n={n} p={p} K={K} ldx={ldx} tuning {dp.tuning}: rel-L2 {err:.2e}",
          flush=True)
    assert np.all(np.isfinite(G)) and np.isfinite(float(logk))
    assert err <= tol
    assert abs(float(logk) - lk_o) <= max(tol, 1e-6) * abs(lk_o)
    assert_elementwise(G, G_o, prob.X64, prob.y, Bs, prob.prior, prob.prior_scale, 1,
                       UNIT_ROUNDOFF[fmt])
    del dp, X, big
    torch.cuda.empty_cache()


@pytest.mark.parametrize("n,p,K,hi_only", SPLIT)
def test_split_planes_at_max_pitch(lib, n, p, K, hi_only):
    import torch
    ldx = PITCH["bf16"]
    fmt = lib.HMC_X_BF16 if hi_only else lib.HMC_X_BF16_HILO
    assert lib.hmc_max_p(fmt, K) == min((1 << 30) // K, ldx)
    prob = make_problem("c4_bf16", n=n, p=p, K=K)
    hi = torch.empty((n, ldx), dtype=torch.bfloat16, device="cuda")
    lo = None if hi_only else torch.empty((n, ldx), dtype=torch.bfloat16, device="cuda")
    X64 = torch.from_numpy(np.ascontiguousarray(prob.X64)).cuda()
    lib.hmc_split_bf16(X64, lib.HMC_X_F64, n, p, p, hi, lo, ldx)
    del X64
    hi[:, p:] = float("nan")
    if lo is not None:
        lo[:, p:] = float("nan")
    dp = lib.Problem(hi[:, :p], torch.from_numpy(prob.y).cuda(), K, prob.prior, prob.prior_scale,
                     True, X_lo=None if lo is None else lo[:, :p])
    Bd = torch.from_numpy(make_random_state(prob, 0.05).astype(np.float32)).cuda()
    logk, G = lib.logpost_grad(dp, Bd)
    G = G.double().cpu().numpy()
    Bs = Bd.double().cpu().numpy()
    h, l = split.split_hilo(prob.X64)
    Xe = h if hi_only else h + l
    lk_o, G_o = oracle.log_kernel_and_grad(Xe, prob.y, Bs, prob.prior, prob.prior_scale, 1)
    err = _relL2(G, G_o)
    bound = 2.0 ** -14 * float(np.sum(np.max(np.abs(Xe) @ np.abs(Bs), axis=1))) + n * 1e-6
    print(f"[max pitch] bf16 hi_only={hi_only} n={n} p={p} K={K} ldx={ldx}: rel-L2 {err:.2e}",
          flush=True)
    assert np.all(np.isfinite(G)) and np.isfinite(float(logk))
    assert err <= 6e-5
    assert abs(float(logk) - lk_o) <= bound
    assert np.all(G[:, -1] == 0)
    del dp, hi, lo
    torch.cuda.empty_cache()


def test_batched_split_planes_at_max_pitch(lib):
    """Two problems of a batch (4 chains each) on planes at the largest pitch with NaN
    padding: every chain's gradient and log K against the oracle on X_eff = hi + lo."""
    import torch
    ldx = PITCH["bf16"]
    shapes = [(130, 1001, 5), (70, 300, 9)]
    probs, dev, keep = [], [], []
    for i, (n, p, K) in enumerate(shapes):
        pr = make_problem("c4_bf16", n=n, p=p, K=K)
        hi = torch.empty((n, ldx), dtype=torch.bfloat16, device="cuda")
        lo = torch.empty((n, ldx), dtype=torch.bfloat16, device="cuda")
        X64 = torch.from_numpy(np.ascontiguousarray(pr.X64)).cuda()
        lib.hmc_split_bf16(X64, lib.HMC_X_F64, n, p, p, hi, lo, ldx)
        del X64
        hi[:, p:] = float("nan")
        lo[:, p:] = float("nan")
        keep += [hi, lo]
        probs.append(pr)
        dev.append(lib.Problem(hi[:, :p], torch.from_numpy(pr.y).cuda(), K, pr.prior,
                               pr.prior_scale, True, X_lo=lo[:, :p]))
    bt = lib.Batch(dev, 4)
    B, G, logk = bt.zeros_state()
    for b, pr in enumerate(probs):
        for c in range(4):
            B[b][c].copy_(torch.from_numpy(make_random_state(pr, 0.1, seed=10 * b + c).astype(np.float32)))
    bt.logpost_grad(B, G, logk)
    lk = logk.cpu().numpy()
    for b, pr in enumerate(probs):
        h, l = split.split_hilo(pr.X64)
        for c in range(4):
            Bc = B[b][c].double().cpu().numpy()
            lk_o, G_o = oracle.log_kernel_and_grad(h + l, pr.y, Bc, pr.prior, pr.prior_scale, 1)
            Gd = G[b][c].double().cpu().numpy()
            err = _relL2(Gd, G_o)
            print(f"[max pitch] batched problem {b} chain {c}: rel-L2 {err:.2e}", flush=True)
            assert np.all(np.isfinite(Gd)) and np.isfinite(lk[b, c])
            assert err <= 6e-5
            assert abs(lk[b, c] - lk_o) <= 1e-6 * abs(lk_o) + 1e-4
    del bt, dev, keep
    torch.cuda.empty_cache()
