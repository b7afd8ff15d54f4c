"""Seeded synthetic workloads shaped like the paper's multinomial-regression problems.

Every array comes from ``numpy.random.default_rng`` with a fixed seed sequence, so the
oracle and the device path see bit-identical inputs. Shapes follow the paper's timing
sweep (Section 3.1, Table 1: N, K and p ranges), its MNIST-scale run (Section 3.2) and
its high-dimensional framing (abstract, Section 1); the dataset itself is not used.

Labels are drawn from the model's categorical distribution with the Gumbel-max rule
(argmax_k of logit plus a standard Gumbel variate), which has exactly the softmax
class probabilities of Section 2.1 while evaluating no softmax here.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

GAUSS = 0
CAUCHY = 1


@dataclass
class Problem:
    name: str
    n: int
    p: int
    K: int
    X: np.ndarray            # n x p, row-major, storage dtype (float64 or float32)
    y: np.ndarray            # int32 labels in [0, K)
    B_true: np.ndarray       # p x K float64 (generating coefficients, all K columns)
    prior: int = GAUSS
    prior_scale: float = 1.0
    pin_last_class: int = 1
    eps: float = 0.01
    L: int = 10
    n_iter: int = 200
    xfmt: str = "f64"        # "f64" | "f32" | "bf16hilo"
    meta: dict = field(default_factory=dict)

    @property
    def X64(self) -> np.ndarray:
        """The exact values the device reads, widened to float64."""
        return np.asarray(self.X, dtype=np.float64)

    @property
    def state_dtype(self):
        return np.float64 if self.xfmt == "f64" else np.float32


@dataclass
class Draws:
    xi: np.ndarray   # n_iter x p x K standard normals (momentum refresh)
    u: np.ndarray    # n_iter uniforms in (0, 1) (accept test)


def _open_uniform(rng, size):
    """Uniforms strictly inside (0, 1): odd multiples of 2**-53, all exactly representable."""
    k = rng.integers(0, 2 ** 52, size=size, dtype=np.int64)
    return (k.astype(np.float64) + 0.5) * 2.0 ** -52


def gumbel_max_labels(rng, X, B_true):
    """y_i ~ Categorical(softmax(x_i B_true)) through argmax(x_i B_true + Gumbel)."""
    n, K = X.shape[0], B_true.shape[1]
    g = -np.log(-np.log(_open_uniform(rng, (n, K))))
    return np.argmax(X @ B_true + g, axis=1).astype(np.int32)


def _sparse_normal(rng, shape, frac, var):
    mask = rng.random(shape) < frac
    return np.where(mask, rng.normal(0.0, np.sqrt(var), size=shape), 0.0)


# name -> (config index used in the seed sequence, defaults)
_CONFIGS = {
    # small FP64 problem: n=500, p=20, K=3, Gaussian N(0,1) prior, eps=0.01, L=10
    "c1_small_f64": dict(idx=1, n=500, p=20, K=3, xfmt="f64", prior=GAUSS, prior_scale=1.0,
                         eps=0.01, L=10, n_iter=200),
    # plain FP32: n=20000, p=1000, K=10, standardised columns, 10% nonzero N(0, var 2) truth
    "c2_f32": dict(idx=2, n=20000, p=1000, K=10, xfmt="f32", prior=GAUSS, prior_scale=1.0,
                   eps=0.002, L=50, n_iter=1000),
    # p >> n: n=2000, p=50000, K=4, 1% nonzero truth, N(0, 0.1^2) prior
    "c3_widep": dict(idx=3, n=2000, p=50000, K=4, xfmt="f32", prior=GAUSS, prior_scale=0.1,
                     eps=5e-4, L=100, n_iter=500),
    # precision form: n=200000, p=4096, K=64, X split into bf16 hi + lo on the device
    "c4_bf16": dict(idx=4, n=200000, p=4096, K=64, xfmt="bf16hilo", prior=GAUSS, prior_scale=1.0,
                    eps=1e-3, L=50, n_iter=100),
    # MNIST-shaped stand-in (Section 3.2): 784 U(0,1) pixels + intercept, K=10, Cauchy(0,1) prior
    "c0_mnist_shape": dict(idx=0, n=60000, p=785, K=10, xfmt="f32", prior=CAUCHY, prior_scale=1.0,
                           eps=7e-5, L=100, n_iter=100),
}


def config_names():
    return list(_CONFIGS)


def standard_configs():
    return {k: dict(v) for k, v in _CONFIGS.items()}


def make_problem(name: str, n: int | None = None, p: int | None = None, K: int | None = None,
                 seed: int | None = None, **overrides) -> Problem:
    """Build a named workload, optionally shrunk (n, p, K) for parity tests.

    The seed sequence is ``[config index, 0]`` (the small FP64 config uses plain seed 0)
    unless ``seed`` is given.
    """
    cfg = dict(_CONFIGS[name])
    idx = cfg.pop("idx")
    n = cfg["n"] if n is None else int(n)
    p = cfg["p"] if p is None else int(p)
    K = cfg["K"] if K is None else int(K)
    cfg.update(n=n, p=p, K=K)
    cfg.update(overrides)
    if seed is None:
        rng = np.random.default_rng(0 if name == "c1_small_f64" else [idx, 0])
    else:
        rng = np.random.default_rng(seed)

    if name == "c0_mnist_shape":
        X = np.empty((n, p))
        X[:, : p - 1] = rng.random((n, p - 1))
        X[:, p - 1] = 1.0                                # intercept column
        B_true = rng.normal(0.0, 0.1, size=(p, K))
    else:
        X = rng.normal(size=(n, p))
        if name == "c2_f32":
            X = (X - X.mean(axis=0)) / X.std(axis=0)     # standardised columns, ddof = 0
            B_true = _sparse_normal(rng, (p, K), 0.10, 2.0)
        elif name == "c3_widep":
            B_true = _sparse_normal(rng, (p, K), 0.01, 1.0)
        elif name == "c4_bf16":
            B_true = rng.normal(0.0, np.sqrt(1.0 / p), size=(p, K))
        else:
            B_true = rng.normal(size=(p, K))
    y = gumbel_max_labels(rng, X, B_true)
    xfmt = cfg["xfmt"]
    Xs = X.astype(np.float32) if xfmt == "f32" else X
    return Problem(name=name, n=n, p=p, K=K, X=np.ascontiguousarray(Xs), y=y, B_true=B_true,
                   prior=cfg["prior"], prior_scale=float(cfg["prior_scale"]),
                   pin_last_class=int(cfg.get("pin_last_class", 1)), eps=float(cfg["eps"]),
                   L=int(cfg["L"]), n_iter=int(cfg["n_iter"]), xfmt=xfmt)


def make_poisson(n: int, p: int, seed=(6, 0), xfmt: str = "f32", prior: int = GAUSS,
                 prior_scale: float = 1.0, eps: float = 0.002, L: int = 50) -> Problem:
    """Count data for the Poisson-regression link: X iid N(0, 1), beta_true iid
    N(0, 0.25 / p) (so x_i^T beta_true ~ N(0, 0.25): rates around 1), y_i ~ Poisson(exp(x_i^T
    beta_true)) drawn with numpy's Poisson sampler. One coefficient column, nothing pinned."""
    rng = np.random.default_rng(list(seed))
    X = rng.normal(size=(n, p))
    B_true = rng.normal(0.0, np.sqrt(0.25 / p), size=(p, 1))
    y = rng.poisson(np.exp(X @ B_true[:, 0])).astype(np.int32)
    Xs = X.astype(np.float32) if xfmt == "f32" else X
    return Problem(name="poisson_" + xfmt, n=n, p=p, K=1, X=np.ascontiguousarray(Xs), y=y,
                   B_true=B_true, prior=prior, prior_scale=float(prior_scale), pin_last_class=0,
                   eps=float(eps), L=int(L), n_iter=100, xfmt=xfmt, meta={"link": "poisson"})


def make_probit(n: int, p: int, seed=(7, 0), xfmt: str = "f32", prior: int = GAUSS,
                prior_scale: float = 1.0, eps: float = 0.002, L: int = 50) -> Problem:
    """Binary data for the probit link: X iid N(0, 1), beta_true iid N(0, 1 / p) (so
    x_i^T beta_true ~ N(0, 1)), y_i = 1 iff x_i^T beta_true + e_i > 0 with e_i iid N(0, 1)
    (the latent-variable form of P(y_i = 1) = Phi(x_i^T beta_true)). One coefficient
    column, nothing pinned."""
    rng = np.random.default_rng(list(seed))
    X = rng.normal(size=(n, p))
    B_true = rng.normal(0.0, np.sqrt(1.0 / p), size=(p, 1))
    y = (X @ B_true[:, 0] + rng.normal(size=n) > 0).astype(np.int32)
    Xs = X.astype(np.float32) if xfmt == "f32" else X
    return Problem(name="probit_" + xfmt, n=n, p=p, K=1, X=np.ascontiguousarray(Xs), y=y,
                   B_true=B_true, prior=prior, prior_scale=float(prior_scale), pin_last_class=0,
                   eps=float(eps), L=int(L), n_iter=100, xfmt=xfmt, meta={"link": "probit"})


def make_draws(p: int, K: int, n_iter: int, seed=(0, 1, 0)) -> Draws:
    """Momentum normals and accept uniforms for ``n_iter`` iterations of one chain."""
    rng = np.random.default_rng(list(seed) if not isinstance(seed, int) else seed)
    xi = rng.standard_normal((n_iter, p, K))
    u = _open_uniform(rng, n_iter)
    return Draws(xi=xi, u=u)


def make_random_state(prob: Problem, scale: float = 0.05, seed: int = 7) -> np.ndarray:
    """A generic (non-zero) coefficient matrix for gradient checks; last column zero if pinned."""
    rng = np.random.default_rng(seed)
    B = rng.normal(0.0, scale, size=(prob.p, prob.K))
    if prob.pin_last_class:
        B[:, prob.K - 1] = 0.0
    return B.astype(prob.state_dtype).astype(np.float64)


def make_batched(n_prob: int = 64, seed: int = 5, n_range=(1000, 50000), p_range=(64, 2048),
                 K_range=(2, 16)) -> list[Problem]:
    """Many uneven problems: n ~ U[1k,50k], p ~ U[64,2048], K ~ U[2,16] (inclusive integers),
    step size eps_b = 0.4 / (sqrt n_b + sqrt p_b)."""
    out = []
    for b in range(n_prob):
        rng = np.random.default_rng([seed, 0, b])
        n = int(rng.integers(n_range[0], n_range[1] + 1))
        p = int(rng.integers(p_range[0], p_range[1] + 1))
        K = int(rng.integers(K_range[0], K_range[1] + 1))
        X = rng.normal(size=(n, p))
        B_true = rng.normal(0.0, np.sqrt(1.0 / p), size=(p, K))
        y = gumbel_max_labels(rng, X, B_true)
        # 1/(sqrt n + sqrt p) leaves the chains of problems with p near n at acceptance 0
        # (checked with the oracle); 0.4 of it lets every problem's chains move
        eps = 0.4 / (np.sqrt(n) + np.sqrt(p))
        out.append(Problem(name=f"batched_{b}", n=n, p=p, K=K, X=X.astype(np.float32), y=y,
                           B_true=B_true, prior=GAUSS, prior_scale=1.0, pin_last_class=1,
                           eps=float(eps), L=20, n_iter=200, xfmt="f32"))
    return out
