"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle's callers.

This package draws data only. It evaluates none of the sampler's arithmetic (no
log-posterior, gradient, leapfrog or accept step), so the oracle and the device path
can both be fed from it without sharing any of the method's code.
"""
from .synth import (  # noqa: F401
    Problem, Draws, make_problem, make_draws, make_batched, make_random_state, standard_configs,
    config_names, make_poisson, make_probit,
    GAUSS, CAUCHY,
)
