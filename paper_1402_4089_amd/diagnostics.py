"""Chain diagnostics on recorded samples: effective sample size, MCSE, split R-hat.

Host-side post-processing of samples the device has already produced; nothing here is on
the sampling path.

ESS for one chain uses Geyer's initial monotone sequence estimator (Geyer 1992, Statistical
Science 7): autocorrelations are summed in adjacent pairs, the pair sums are truncated at
the first non-positive one and made non-increasing. Multi-chain ESS and R-hat follow the
rank-normalised split-chain recipe of Vehtari, Gelman, Simpson, Carpenter and Buerkner
(2021, Bayesian Analysis 16).
"""
from __future__ import annotations

import numpy as np


def _autocov(x: np.ndarray) -> np.ndarray:
    """Biased autocovariance of each column of x (T x d) at lags 0..T-1, via FFT."""
    T = x.shape[0]
    xc = x - x.mean(axis=0)
    nfft = 1 << int(np.ceil(np.log2(2 * T)))
    f = np.fft.rfft(xc, n=nfft, axis=0)
    ac = np.fft.irfft(f * np.conj(f), n=nfft, axis=0)[:T]
    return ac / T


def _tau_from_rho(rho: np.ndarray) -> np.ndarray:
    """Integrated autocorrelation time from autocorrelations rho (T x d), Geyer IMSE: the
    pair sums Gamma_m = rho_2m + rho_2m+1 are kept up to (not including) the first
    non-positive one and made non-increasing; tau = -1 + 2 sum Gamma_m."""
    T, d = rho.shape
    npair = T // 2
    pairs = rho[0:2 * npair:2] + rho[1:2 * npair:2]         # Gamma_m = rho_2m + rho_2m+1
    nonpos = pairs <= 0.0
    first = np.where(nonpos.any(axis=0), nonpos.argmax(axis=0), npair)   # per column
    mono = np.minimum.accumulate(pairs, axis=0)
    keep = np.arange(npair)[:, None] < first[None, :]
    tau = -1.0 + 2.0 * np.where(keep, mono, 0.0).sum(axis=0)
    return np.maximum(tau, 1.0 / np.log10(max(T, 10)))


def ess(x: np.ndarray) -> np.ndarray:
    """Effective sample size per coordinate of one chain; x is T x d (or T)."""
    x = np.asarray(x, dtype=np.float64)
    if x.ndim == 1:
        x = x[:, None]
    T = x.shape[0]
    ac = _autocov(x)
    var0 = ac[0]
    const = var0 <= 0.0
    rho = ac / np.where(const, 1.0, var0)
    out = T / _tau_from_rho(rho)
    out[const] = np.nan
    return out


def mcse_mean(x: np.ndarray) -> np.ndarray:
    x = np.asarray(x, dtype=np.float64)
    if x.ndim == 1:
        x = x[:, None]
    return x.std(axis=0, ddof=1) / np.sqrt(ess(x))


def _rank_normalise(chains: np.ndarray) -> np.ndarray:
    from scipy.stats import norm, rankdata
    M, T, d = chains.shape
    flat = chains.reshape(M * T, d)
    r = np.apply_along_axis(rankdata, 0, flat)
    z = norm.ppf((r - 0.375) / (M * T + 0.25))
    return z.reshape(M, T, d)


def multichain_ess(chains: np.ndarray, rank_normalise: bool = True) -> np.ndarray:
    """Bulk ESS over M chains (M x T x d), split-chain, optionally rank-normalised."""
    c = np.asarray(chains, dtype=np.float64)
    M, T, d = c.shape
    h = T // 2
    c = np.concatenate([c[:, :h], c[:, T - h:]], axis=0)     # split chains
    if rank_normalise:
        c = _rank_normalise(c)
    M2 = c.shape[0]
    acov = np.stack([_autocov(c[m]) for m in range(M2)])     # M2 x h x d
    W = acov[:, 0].mean(axis=0) * h / (h - 1)
    mean_c = c.mean(axis=1)
    var_plus = W * (h - 1) / h + mean_c.var(axis=0, ddof=1)
    rho = 1.0 - (W - acov.mean(axis=0)) / np.where(var_plus > 0, var_plus, 1.0)
    rho[0] = 1.0
    return M2 * h / _tau_from_rho(rho)


def split_rhat(chains: np.ndarray) -> np.ndarray:
    c = np.asarray(chains, dtype=np.float64)
    M, T, d = c.shape
    h = T // 2
    c = np.concatenate([c[:, :h], c[:, T - h:]], axis=0)
    W = c.var(axis=1, ddof=1).mean(axis=0)
    B = h * c.mean(axis=1).var(axis=0, ddof=1)
    var_plus = (h - 1) / h * W + B / h
    return np.sqrt(var_plus / W)
