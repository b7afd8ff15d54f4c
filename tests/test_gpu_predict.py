"""Posterior-predictive classification of Section 3.2 on the device (GPU tier), against the
oracle's posterior_predictive_class: the mean over samples of the softmax class
probabilities (float64 sums) and its argmax, on held-out rows of the MNIST-shaped stand-in
(784 U(0,1) pixels + intercept, K = 10) and on a small FP64 problem with K > 16.

The argmax must be identical wherever the two largest oracle mean probabilities differ by
more than a tie band (1e-5 for FP32, whose per-sample probabilities carry about 1e-7
relative error; 1e-12 for FP64); the mean probabilities must agree within 2e-6 (FP32) and
1e-13 (FP64) absolute."""
import numpy as np
import pytest

import oracle
from workloads import make_problem

pytestmark = pytest.mark.gpu


def _run(lib, X, samples, K, pin):
    import torch
    Xd = torch.from_numpy(np.ascontiguousarray(X)).cuda()
    Sd = torch.from_numpy(np.ascontiguousarray(samples.astype(X.dtype))).cuda()
    mean, cls = lib.posterior_predictive(Xd, Sd, K, pin)
    torch.cuda.synchronize()
    return mean.cpu().numpy(), cls.cpu().numpy()


def _oracle_mean(X64, samples):
    acc = np.zeros((X64.shape[0], samples.shape[2]))
    for B in samples:
        acc += oracle.softmax_rows(oracle.logits(X64, B))
    return acc / len(samples)


@pytest.mark.parametrize("name,n,p,K,S,dtype,band,atol", [
    ("c0_mnist_shape", 3001, 785, 10, 40, np.float32, 1e-5, 2e-6),
    ("c1_small_f64", 1003, 60, 23, 17, np.float64, 1e-12, 1e-13),
    ("c2_f32", 517, 300, 64, 5, np.float32, 1e-5, 2e-6),
])
def test_posterior_predictive_matches_oracle(lib, name, n, p, K, S, dtype, band, atol):
    prob = make_problem(name, n=n, p=p, K=K)
    X = np.asarray(prob.X, dtype=dtype)
    rng = np.random.default_rng(17)
    Bt = prob.B_true - prob.B_true[:, -1:]                 # the pinned parametrisation
    samples = Bt[None] + rng.normal(0.0, 0.05, size=(S, p, K))
    samples[:, :, -1] = 0.0
    samples = samples.astype(dtype).astype(np.float64)     # the values the device reads
    mean, cls = _run(lib, X, samples, K, True)
    X64 = X.astype(np.float64)
    mean_o = _oracle_mean(X64, samples)
    cls_o = oracle.posterior_predictive_class(X64, samples)
    assert np.max(np.abs(mean - mean_o)) <= atol
    top2 = np.sort(mean_o, axis=1)[:, -2:]
    clear = (top2[:, 1] - top2[:, 0]) > band
    assert np.array_equal(cls[clear], cls_o[clear])
    assert clear.mean() > 0.9
    print(f"[predict] {name}: {int(clear.sum())} of {n} rows clear of ties, argmax identical; "
          f"max |mean diff| {np.max(np.abs(mean - mean_o)):.2e}", flush=True)


def test_posterior_predictive_reads_pinned_column_as_zero(lib):
    prob = make_problem("c1_small_f64", n=200, p=30, K=5)
    rng = np.random.default_rng(3)
    samples = rng.normal(0.0, 0.3, size=(6, 30, 5))
    dirty = samples.copy()
    samples[:, :, -1] = 0.0
    mean, cls = _run(lib, prob.X64, dirty, 5, True)
    assert np.max(np.abs(mean - _oracle_mean(prob.X64, samples))) <= 1e-13
