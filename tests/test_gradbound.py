"""The element-wise gradient bound of the GPU parity tests, checked on the CPU: it admits a
float32 evaluation of the gradient (the precision of the FP32 device path) and rejects a
gradient with one 16-column block off by 5e-5 relative, a mistake the global rel-L2
tolerance of 1e-5 lets through."""
import numpy as np
import pytest

import oracle
from gradbound import UNIT_ROUNDOFF, assert_elementwise
from workloads import make_problem, make_random_state


def _f32_gradient(prob, B):
    Xf = prob.X.astype(np.float32)
    Z = Xf @ B.astype(np.float32)
    Z = Z - Z.max(axis=1, keepdims=True)
    E = np.exp(Z)
    P = E / E.sum(axis=1, keepdims=True)
    R = oracle.onehot(prob.y, prob.K).astype(np.float32) - P
    G = (Xf.T @ R).astype(np.float64) + oracle.log_prior_grad(B, prob.prior, prob.prior_scale)
    return G * oracle.free_mask(prob.p, prob.K, prob.pin_last_class)


@pytest.fixture(scope="module")
def case():
    prob = make_problem("c2_f32", n=6000, p=600, K=10)
    B = make_random_state(prob, 0.05)
    G_o = oracle.grad_log_kernel(prob.X64, prob.y, B, prob.prior, prob.prior_scale, 1)
    return prob, B, G_o


def test_bound_admits_a_float32_evaluation(case):
    prob, B, G_o = case
    assert_elementwise(_f32_gradient(prob, B), G_o, prob.X64, prob.y, B, prob.prior,
                       prob.prior_scale, 1, UNIT_ROUNDOFF["f32"])


def test_bound_rejects_one_wrong_block(case):
    prob, B, G_o = case
    bad = G_o.copy()
    bad[320:336] *= 1.0 + 5e-5
    rel = np.linalg.norm(bad - G_o) / np.linalg.norm(G_o)
    assert rel < 1e-5                                   # the rel-L2 tolerance would pass it
    with pytest.raises(AssertionError):
        assert_elementwise(bad, G_o, prob.X64, prob.y, B, prob.prior, prob.prior_scale, 1,
                           UNIT_ROUNDOFF["f32"])
