"""Persistent cache of autotuned launch decompositions for the single-problem path.

``tuned(problem)`` returns the hmc_tuning for a Problem: from the cache when an entry for
its key exists, otherwise measured on the device by the library's autotuner
(hmc_autotune) and stored. The key is (X format, 16-class blocks, 16-column blocks,
row-count bucket, link): every tuning in the cache is valid for every problem with that key
(a row-tile variant covers the key's column blocks, and the other fields are counts that fit
any row count). The cache is a JSON file at $HMC_TUNING_CACHE, or
~/.cache/paper_1402_4089_amd/tuning.json when that variable is unset; a cache that cannot
be read or written is ignored (the tuning is then measured in every process).
"""
from __future__ import annotations

import json
import os

ENV = "HMC_TUNING_CACHE"


def cache_path() -> str:
    p = os.environ.get(ENV)
    if p:
        return p
    return os.path.join(os.path.expanduser("~"), ".cache", "paper_1402_4089_amd", "tuning.json")


def key_of(prob) -> str:
    nb = (prob.K + 15) // 16
    nblk = (prob.p + 15) // 16
    nbucket = 1 << max(0, int(prob.n - 1).bit_length())       # n rounded up to a power of two
    return f"xfmt={prob.xfmt}:nb={nb}:nblk={nblk}:n<={nbucket}:link={prob.link}"


def _read(path: str) -> dict:
    try:
        with open(path) as fh:
            d = json.load(fh)
        return d if isinstance(d, dict) else {}
    except (OSError, ValueError):
        return {}


def _write(path: str, d: dict) -> None:
    try:
        os.makedirs(os.path.dirname(path) or ".", exist_ok=True)
        tmp = path + f".tmp{os.getpid()}"
        with open(tmp, "w") as fh:
            json.dump(d, fh, indent=1, sort_keys=True)
        os.replace(tmp, path)
    except OSError:
        pass


def lookup(prob):
    """The cached tuning dict for this problem's key, or None."""
    ent = _read(cache_path()).get(key_of(prob))
    return None if ent is None else ent.get("tuning")


def usable(prob, t) -> bool:
    """Whether the library accepts the tuning dict t for this problem: a cache written by
    another build of the library, or edited by hand, may hold a decomposition this build
    refuses (checked on the host, through the workspace query, without device work)."""
    from . import HMCError, hmc_problem, hmc_tuning, hmc_workspace_bytes
    try:
        t = dict(t)
        if not set(t) <= {name for name, _ in hmc_tuning._fields_}:
            return False
        desc = hmc_problem.from_buffer_copy(prob.desc)
        desc.tuning = hmc_tuning(**t)
        hmc_workspace_bytes(desc)
        return True
    except (HMCError, TypeError, ValueError):
        return False


def tuned(prob):
    """(tuning dict, measured microseconds per gradient evaluation or None if cached). A
    cached entry the library refuses is measured again and replaced."""
    hit = lookup(prob)
    if hit is not None and usable(prob, hit):
        return hit, None
    import torch
    from . import _aligned_workspace, hmc_autotune, hmc_autotune_workspace_bytes
    ws = _aligned_workspace(hmc_autotune_workspace_bytes(prob.desc), prob.X.device)
    B = prob.zeros_state()
    logk = torch.empty((), dtype=torch.float64, device=prob.X.device)
    G = torch.empty_like(B)
    t, us = hmc_autotune(prob.desc, B, logk, G, ws)
    del ws
    d = _read(cache_path())
    d[key_of(prob)] = {"tuning": t.as_dict(), "us_per_gradient": round(us, 3),
                       "measured_on": {"n": prob.n, "p": prob.p, "K": prob.K}}
    _write(cache_path(), d)
    return t.as_dict(), us
