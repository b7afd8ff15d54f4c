"""Loop-level definitions for tiny inputs (test infrastructure only; parity checker).

These follow the paper's scalar equations one term at a time, with no vectorisation and
no max-shift: equation (softmax) for psi, equation (logkernel) for the log-posterior
kernel, and the per-coordinate Appendix derivative x_ij (y_ik - psi_ik) summed over
observations plus the prior term (sign as in the derivative of -log(1 + beta^2)).
They are meant for n, p, K of a handful each.
"""
from __future__ import annotations

import math

GAUSS = 0
CAUCHY = 1


def _psi(x, B, k, K):
    p = len(x)
    num = math.exp(sum(x[j] * B[j][k] for j in range(p)))
    den = 0.0
    for c in range(K):
        den += math.exp(sum(x[j] * B[j][c] for j in range(p)))
    return num / den


def _prior_term(b, prior, s):
    if prior == CAUCHY:
        return -math.log(1.0 + (b / s) ** 2)
    return -(b * b) / (2.0 * s * s)


def _prior_deriv(b, prior, s):
    if prior == CAUCHY:
        return -2.0 * b / (s * s + b * b)
    return -b / (s * s)


def log_kernel_loops(X, y, B, K, prior=GAUSS, scale=1.0, pin_last_class=1):
    n, p = len(X), len(X[0])
    total = 0.0
    for i in range(n):
        for k in range(K):
            yik = 1.0 if int(y[i]) == k else 0.0
            if yik:
                total += yik * math.log(_psi(X[i], B, k, K))
    for k in range(K):
        if pin_last_class and k == K - 1:
            continue
        for j in range(p):
            total += _prior_term(B[j][k], prior, scale)
    return total


def grad_loops(X, y, B, K, prior=GAUSS, scale=1.0, pin_last_class=1):
    n, p = len(X), len(X[0])
    G = [[0.0] * K for _ in range(p)]
    for j in range(p):
        for k in range(K):
            if pin_last_class and k == K - 1:
                continue
            acc = 0.0
            for i in range(n):
                yik = 1.0 if int(y[i]) == k else 0.0
                acc += X[i][j] * (yik - _psi(X[i], B, k, K))
            G[j][k] = acc + _prior_deriv(B[j][k], prior, scale)
    return G
