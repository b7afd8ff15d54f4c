"""hmc_logpost_grad_noalloc (the entry point for callers that cannot allocate) against
hmc_logpost_grad with a caller workspace (GPU tier), called through the C-ABI.

Two calls in a row share the built-in scratch array, the second on a smaller problem:
each must equal the workspace entry point bit for bit (same kernels, same fixed reduction
order) and meet the gradient tolerance against the FP64 oracle (relative L2 <= 1e-5 for
FP32, <= 1e-12 for FP64). A problem whose workspace exceeds the scratch is refused on the
host.
"""
import numpy as np
import pytest

import oracle
from workloads import make_problem, make_random_state

pytestmark = pytest.mark.gpu


def _dev(lib, prob):
    import torch
    X = torch.from_numpy(np.asarray(prob.X)).cuda()
    y = torch.from_numpy(prob.y).cuda()
    return lib.Problem(X, y, prob.K, prob.prior, prob.prior_scale, bool(prob.pin_last_class))


def _both(lib, prob, B64):
    import torch
    dp = _dev(lib, prob)
    B = torch.from_numpy(B64.astype(prob.state_dtype)).cuda()
    lk_ws = torch.empty((), dtype=torch.float64, device="cuda")
    G_ws = torch.empty_like(B)
    lib.hmc_logpost_grad(dp.desc, B, lk_ws, G_ws, dp.ws)
    lk_na = torch.full((), float("nan"), dtype=torch.float64, device="cuda")
    G_na = torch.full_like(B, float("nan"))
    lib.hmc_logpost_grad_noalloc(dp.desc, B, lk_na, G_na)
    torch.cuda.synchronize()
    return B, lk_ws, G_ws, lk_na, G_na


@pytest.mark.parametrize("name,big,small,tol", [
    ("c2_f32", (20000, 1000, 10), (3001, 257, 4), 1e-5),
    ("c1_small_f64", (4099, 250, 5), (500, 20, 3), 1e-12),
])
def test_noalloc_matches_workspace_call_twice(lib, name, big, small, tol):
    for n, p, K in (big, small):
        prob = make_problem(name, n=n, p=p, K=K)
        B64 = make_random_state(prob, 0.05)
        B, lk_ws, G_ws, lk_na, G_na = _both(lib, prob, B64)
        assert float(lk_na) == float(lk_ws)
        assert bool((G_na == G_ws).all())
        lk_o, G_o = oracle.log_kernel_and_grad(prob.X64, prob.y, B.double().cpu().numpy(),
                                               prob.prior, prob.prior_scale, 1)
        G = G_na.double().cpu().numpy()
        assert np.linalg.norm(G - G_o) <= tol * np.linalg.norm(G_o)
        assert abs(float(lk_na) - lk_o) <= max(tol, 1e-6) * abs(lk_o)
        print(f"[noalloc] {name} n={n} p={p} K={K}: identical to the workspace call", flush=True)


def test_noalloc_refuses_a_workspace_beyond_the_scratch(lib):
    import torch
    prob = make_problem("c2_f32", n=64, p=60000, K=4)      # wide-p: ~8 MB of partial logits
    dp = _dev(lib, prob)
    need = lib.hmc_workspace_bytes(dp.desc)
    if need <= 32 << 20:
        # a problem large enough to exceed 32 MiB of workspace without a large X upload:
        # the check runs on the host before anything is enqueued
        d = lib.hmc_problem(n=1 << 20, p=60000, K=4, xfmt=lib.HMC_X_F32, X=dp.X.data_ptr(),
                            X_lo=None, ldx=60000, y=dp.y.data_ptr(), prior=0, prior_scale=1.0,
                            pin_last_class=1)
    else:
        d = dp.desc
    assert lib.hmc_workspace_bytes(d) > 32 << 20
    B = torch.zeros(60000, 4, dtype=torch.float32, device="cuda")
    G = torch.empty_like(B)
    lk = torch.empty((), dtype=torch.float64, device="cuda")
    with pytest.raises(lib.HMCError) as ei:
        lib.hmc_logpost_grad_noalloc(d, B, lk, G)
    assert ei.value.status == -5
