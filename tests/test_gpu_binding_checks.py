"""The Python binding refuses state tensors whose dtype, shape, layout or device do not match
the problem before anything reaches the library (GPU tier: the tensors live on the GPU, but
no kernel is launched by the calls that must fail)."""
import numpy as np
import pytest

from workloads import make_problem

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dp(lib):
    import torch
    prob = make_problem("c1_small_f64", n=64, p=6, K=3)
    return lib.Problem(torch.from_numpy(prob.X).cuda(), torch.from_numpy(prob.y).cuda(), 3)


def _bad_states(torch, p, K):
    return [torch.zeros(p, K, dtype=torch.float32, device="cuda"),       # wrong dtype
            torch.zeros(p + 1, K, dtype=torch.float64, device="cuda"),   # wrong shape
            torch.zeros(K, p, dtype=torch.float64, device="cuda").t(),   # not contiguous
            torch.zeros(p, K, dtype=torch.float64)]                      # host tensor


def test_logpost_grad_rejects_mismatched_state(lib, dp):
    import torch
    for B in _bad_states(torch, dp.p, dp.K):
        with pytest.raises(ValueError):
            lib.logpost_grad(dp, B)


def test_leapfrog_and_sample_reject_mismatched_tensors(lib, dp):
    import torch
    B = dp.zeros_state()
    logk, G = lib.logpost_grad(dp, B)
    eta = torch.zeros_like(B)
    for bad in _bad_states(torch, dp.p, dp.K):
        with pytest.raises(ValueError):
            lib.leapfrog(dp, B, bad, G, logk, 0.01, 2)
        with pytest.raises(ValueError):
            lib.sample(dp, B, bad, logk, 0.01, 2, 3)
    with pytest.raises(ValueError):
        lib.leapfrog(dp, B, eta, G, logk.float(), 0.01, 2)
    with pytest.raises(ValueError):
        lib.sample(dp, B, G, logk, 0.01, 2, 3,
                   normals=torch.zeros(2, dp.p, dp.K, dtype=torch.float64, device="cuda"),
                   uniforms=torch.full((3,), 0.5, dtype=torch.float64, device="cuda"))
    with pytest.raises(ValueError):
        lib.sample(dp, B, G, logk, 0.01, 2, 3,
                   inv_temperature=torch.ones(3, dtype=torch.float32, device="cuda"))
    # the good call still runs after the refusals
    out = lib.sample(dp, B, G, logk, 0.01, 2, 3)
    torch.cuda.synchronize()
    assert np.all(np.isfinite(out["H"].cpu().numpy()))
