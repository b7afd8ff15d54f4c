"""FP64 CPU oracle for Hamiltonian Monte Carlo on Bayesian multinomial regression.

TEST INFRASTRUCTURE ONLY. This module is the slow, plain reference that the device
path is checked against. Only the tests, the smoke check and the benchmark's CPU
baseline leg may import it; the library itself never does.

Everything is NumPy in float64, written step by step from the paper:
  * model and log-posterior kernel: Section 2.1, equations (softmax), (loglike),
    (logkernel) and the matrix form (logkernelGPU);
  * gradient: equation (gradient) and the Appendix derivation, equations (lastline)
    and (fullgrad), with the identifiability mask of the Appendix;
  * leapfrog: Section 1.1, equations (hmc1)-(hmc3);
  * accept rule: Section 1.1, equation (accept);
  * annealed burn-in acceptance: Section 3.2;
  * a second per-row likelihood, the Poisson regression (log link), through the same
    contractions: the Discussion's claim that the approach carries over to any model whose
    likelihood and gradient are matrix products. y_i ~ Poisson(exp(x_i^T beta)), one
    coefficient column (K = 1, nothing pinned); log-likelihood sum_i y_i z_i - exp(z_i)
    (the constant -log y_i! dropped), gradient X^T (y - exp(X beta));
  * a third, the probit regression, under the same claim: binary y_i with
    P(y_i = 1) = Phi(x_i^T beta), Phi the standard normal distribution function, one
    coefficient column; with s_i = 2 y_i - 1 the log-likelihood is sum_i log Phi(s_i z_i)
    and the gradient X^T r with r_i = s_i phi(z_i) / Phi(s_i z_i) (phi the normal density,
    which is even). Labels other than 1 count as failures.

Readings where the paper is silent or misprinted:
  * kinetic energy is one half of eta . eta (equation (accept) prints eta . eta; only the
    half is consistent with the unit-mass position update of the leapfrog);
  * the prior-gradient term is -2 beta / (s^2 + beta^2) (the Appendix prints +2 beta /
    (1 + beta^2), which is the derivative of +log(1 + beta^2));
  * the momentum is eta ~ N(0, I) on the free coordinates, redrawn every iteration;
  * the pinned class is column K-1 (0-based); its coefficients, gradient and momentum
    stay zero, and it still contributes the implicit logit 0 to every row's softmax;
  * the log of the softmax uses the max-shifted log-sum-exp (equal in exact arithmetic);
  * accept iff H1 is finite and log(u) < (H0 - H1) * inv_temp (strict); a non-finite H1,
    or H1 - H0 > 1000, marks the transition divergent;
  * a Gaussian prior N(0, sigma^2) is also supported (additive constants dropped).
"""
from __future__ import annotations

import numpy as np
from scipy import special

GAUSS = 0
CAUCHY = 1
SOFTMAX = 0      # multinomial logit (Section 2.1)
POISSON = 1      # Poisson regression with log link (see the module docstring)
PROBIT = 2       # binary probit regression (see the module docstring)
DIVERGENCE_THRESHOLD = 1000.0


def free_mask(p: int, K: int, pin_last_class: int) -> np.ndarray:
    """M_jk = 1 for a free coefficient, 0 for the pinned class column (Appendix)."""
    M = np.ones((p, K))
    if pin_last_class:
        M[:, K - 1] = 0.0
    return M


def onehot(y: np.ndarray, K: int) -> np.ndarray:
    """Y_ik = 1 iff observation i is in class k (Section 2.1)."""
    Y = np.zeros((y.shape[0], K))
    Y[np.arange(y.shape[0]), y] = 1.0
    return Y


def logits(X: np.ndarray, B: np.ndarray) -> np.ndarray:
    """Z = X B, row i holding x_i^T beta_k for every class k (Section 2.1)."""
    return np.asarray(X, dtype=np.float64) @ np.asarray(B, dtype=np.float64)


def log_sum_exp_rows(Z: np.ndarray) -> np.ndarray:
    """LSE_i = m_i + log sum_k exp(Z_ik - m_i), m_i = max_k Z_ik."""
    m = Z.max(axis=1)
    return m + np.log(np.exp(Z - m[:, None]).sum(axis=1))


def softmax_rows(Z: np.ndarray) -> np.ndarray:
    """psi(x_i, beta_k) for every i, k: equation (softmax)."""
    return np.exp(Z - log_sum_exp_rows(Z)[:, None])


def log_likelihood(X, y, B, link=SOFTMAX) -> float:
    """l(B | X, Y) = sum_i sum_k y_ik log psi_ik: equation (loglike); for the Poisson link
    sum_i y_i z_i - exp(z_i) with z = X beta (constants dropped); for the probit link
    sum_i log Phi(s_i z_i)."""
    Z = logits(X, B)
    if link == POISSON:
        z = Z[:, 0]
        return float(np.sum(np.asarray(y, dtype=np.float64) * z - np.exp(z)))
    if link == PROBIT:
        return float(np.sum(special.log_ndtr(_probit_sign(y) * Z[:, 0])))
    lse = log_sum_exp_rows(Z)
    return float(np.sum(Z[np.arange(Z.shape[0]), y] - lse))


def _probit_sign(y) -> np.ndarray:
    """s_i = +1 for a success (y_i = 1), -1 otherwise."""
    return np.where(np.asarray(y) == 1, 1.0, -1.0)


def residual(X, y, B, link=SOFTMAX) -> np.ndarray:
    """R with X^T R the likelihood part of the gradient: Y - psi(X B) (equation (gradient))
    for the softmax link, y - exp(X beta) (as a column) for the Poisson link,
    s phi(z) / Phi(s z) (as a column) for the probit link."""
    Z = logits(X, B)
    if link == POISSON:
        return (np.asarray(y, dtype=np.float64) - np.exp(Z[:, 0]))[:, None]
    if link == PROBIT:
        s = _probit_sign(y)
        z = Z[:, 0]
        # phi(z) / Phi(s z) through logs: both factors underflow far in the tail
        log_phi = -0.5 * z * z - 0.5 * np.log(2.0 * np.pi)
        return (s * np.exp(log_phi - special.log_ndtr(s * z)))[:, None]
    return onehot(y, Z.shape[1]) - softmax_rows(Z)


def log_prior(B, prior: int, scale: float, mask: np.ndarray) -> float:
    """Sum of the prior log-density over free coefficients, constants dropped.

    Cauchy(0, s): -log(1 + (beta/s)^2), the term of equation (logkernel) (s = 1 there).
    Gaussian N(0, s^2): -beta^2 / (2 s^2).
    """
    B = np.asarray(B, dtype=np.float64)
    if prior == CAUCHY:
        terms = -np.log1p((B / scale) ** 2)
    elif prior == GAUSS:
        terms = -(B * B) / (2.0 * scale * scale)
    else:
        raise ValueError("unknown prior")
    return float(np.sum(terms * mask))


def log_prior_grad(B, prior: int, scale: float) -> np.ndarray:
    """Elementwise derivative of the prior log-density.

    Cauchy: d/dbeta[-log(1 + beta^2/s^2)] = -2 beta / (s^2 + beta^2)  (the Appendix's
    Gamma matrix with its sign corrected).  Gaussian: -beta / s^2.
    """
    B = np.asarray(B, dtype=np.float64)
    if prior == CAUCHY:
        return -2.0 * B / (scale * scale + B * B)
    if prior == GAUSS:
        return -B / (scale * scale)
    raise ValueError("unknown prior")


def log_kernel(X, y, B, prior=GAUSS, scale=1.0, pin_last_class=1, link=SOFTMAX) -> float:
    """log K(B | X, Y): equation (logkernel), i.e. the matrix form (logkernelGPU)."""
    p, K = np.shape(B)
    return (log_likelihood(X, y, B, link)
            + log_prior(B, prior, scale, free_mask(p, K, pin_last_class)))


def grad_log_kernel(X, y, B, prior=GAUSS, scale=1.0, pin_last_class=1, link=SOFTMAX) -> np.ndarray:
    """M * [X^T (Y - psi(X B)) + prior'(B)]: equations (gradient), (fullgrad) and the mask."""
    X = np.asarray(X, dtype=np.float64)
    B = np.asarray(B, dtype=np.float64)
    p, K = B.shape
    G = X.T @ residual(X, y, B, link) + log_prior_grad(B, prior, scale)
    return G * free_mask(p, K, pin_last_class)


def log_kernel_and_grad(X, y, B, prior=GAUSS, scale=1.0, pin_last_class=1, link=SOFTMAX):
    return (log_kernel(X, y, B, prior, scale, pin_last_class, link),
            grad_log_kernel(X, y, B, prior, scale, pin_last_class, link))


def kinetic(eta: np.ndarray) -> float:
    """One half of eta . eta (the kinetic term of equation (accept), half restored)."""
    eta = np.asarray(eta, dtype=np.float64)
    return 0.5 * float(np.sum(eta * eta))


def leapfrog_step(X, y, B, eta, G, eps, prior=GAUSS, scale=1.0, pin_last_class=1, link=SOFTMAX):
    """One leapfrog update, equations (hmc1)-(hmc3), in the printed order.

    ``G`` is the gradient at ``B``.  Returns (B', eta', G', log K(B')).
    """
    eta = eta + (eps / 2.0) * G                                    # (hmc1)
    B = B + eps * eta                                              # position full step
    logk = log_kernel(X, y, B, prior, scale, pin_last_class, link)
    G = grad_log_kernel(X, y, B, prior, scale, pin_last_class, link)
    eta = eta + (eps / 2.0) * G                                    # (hmc3)
    return B, eta, G, logk


def leapfrog(X, y, B, eta, G, eps, L, prior=GAUSS, scale=1.0, pin_last_class=1, link=SOFTMAX):
    """L successive leapfrog updates (Section 1.1); L gradient evaluations."""
    logk = None
    for _ in range(int(L)):
        B, eta, G, logk = leapfrog_step(X, y, B, eta, G, eps, prior, scale, pin_last_class, link)
    return B, eta, G, logk


def accept_decision(H0: float, H1: float, u: float, inv_temp: float = 1.0):
    """Metropolis test of equation (accept) in the log domain.

    exp(-H1)/exp(-H0) is compared with u, i.e. accept iff log u < (H0 - H1); under the
    annealed schedule of Section 3.2 the ratio is raised to 1/T, which multiplies the
    log-ratio by inv_temp = 1/T.  Returns (accepted, divergent).
    """
    finite = bool(np.isfinite(H1))
    accepted = finite and (np.log(u) < (H0 - H1) * inv_temp)
    divergent = (not finite) or (H1 - H0 > DIVERGENCE_THRESHOLD)
    return bool(accepted), bool(divergent)


def hmc_iteration(X, y, B, G, logk, xi, u, eps, L, prior=GAUSS, scale=1.0, pin_last_class=1,
                  inv_temp=1.0, link=SOFTMAX):
    """One HMC transition: momentum draw, L leapfrog updates, accept or reject.

    ``G`` and ``logk`` belong to the current ``B`` (cached from the previous iteration),
    so the transition costs exactly L gradient evaluations.
    """
    p, K = B.shape
    eta0 = free_mask(p, K, pin_last_class) * xi
    H0 = -logk + kinetic(eta0)
    B1, eta1, G1, logk1 = leapfrog(X, y, B, eta0, G, eps, L, prior, scale, pin_last_class, link)
    H1 = -logk1 + kinetic(eta1)
    accepted, divergent = accept_decision(H0, H1, u, inv_temp)
    if accepted:
        B, G, logk = B1, G1, logk1
    return dict(B=B, G=G, logk=logk, accepted=accepted, divergent=divergent, H0=H0, H1=H1,
                B_prop=B1, eta_prop=eta1)


def annealed_inv_temps(n_iter: int, T0: float = 1e3, r: float = 0.9) -> np.ndarray:
    """1/T_t for t = 1..n_iter with T_t = max(1, r T_{t-1}); iteration t uses T_{t-1}."""
    out = np.empty(n_iter)
    T = float(T0)
    for t in range(n_iter):
        out[t] = 1.0 / T
        T = max(1.0, r * T)
    return out


def sample(X, y, K, xis, us, eps, L, prior=GAUSS, scale=1.0, pin_last_class=1, B0=None,
           inv_temps=None, link=SOFTMAX):
    """A full chain from B0 (default zeros) using the supplied draws ``xis`` [n_iter,p,K], ``us``."""
    X = np.asarray(X, dtype=np.float64)
    p = X.shape[1]
    n_iter = len(us)
    B = np.zeros((p, K)) if B0 is None else np.array(B0, dtype=np.float64)
    logk = log_kernel(X, y, B, prior, scale, pin_last_class, link)
    G = grad_log_kernel(X, y, B, prior, scale, pin_last_class, link)
    samples = np.empty((n_iter, p, K))
    acc = np.zeros(n_iter, dtype=np.int32)
    div = np.zeros(n_iter, dtype=np.int32)
    H = np.empty((n_iter, 2))
    for t in range(n_iter):
        it = 1.0 if inv_temps is None else float(inv_temps[t])
        r = hmc_iteration(X, y, B, G, logk, xis[t], us[t], eps, L, prior, scale, pin_last_class, it,
                          link)
        B, G, logk = r["B"], r["G"], r["logk"]
        samples[t] = B
        acc[t], div[t] = r["accepted"], r["divergent"]
        H[t] = (r["H0"], r["H1"])
    return dict(samples=samples, accepted=acc, divergent=div, H=H, B=B, G=G, logk=logk)


def posterior_predictive_class(X, samples) -> np.ndarray:
    """Class with the highest posterior-mean softmax probability (Section 3.2)."""
    X = np.asarray(X, dtype=np.float64)
    acc = np.zeros((X.shape[0], samples.shape[2]))
    for B in samples:
        acc += softmax_rows(logits(X, B))
    return np.argmax(acc / len(samples), axis=1)
