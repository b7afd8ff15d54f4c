"""GPU-resident HMC for Bayesian multinomial regression on MI355X (gfx950).

Thin ctypes binding over ``libhmc.so`` (declared in ``include/hmc.h``). The functions
named like the C entry points only marshal arguments: every step of the sampler runs in
the library's HIP kernels. PyTorch supplies device memory (``data_ptr``) and streams.
The binding has no fallback: if the library is missing it raises.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libhmc.so")

HMC_X_F64, HMC_X_F32, HMC_X_BF16_HILO, HMC_X_BF16 = 0, 1, 2, 3
HMC_PRIOR_GAUSS, HMC_PRIOR_CAUCHY = 0, 1
HMC_LINK_SOFTMAX, HMC_LINK_POISSON, HMC_LINK_PROBIT = 0, 1, 2
STATUS = {0: "HMC_OK", -1: "HMC_ERR_ARG", -2: "HMC_ERR_SHAPE", -3: "HMC_ERR_DTYPE",
          -4: "HMC_ERR_HIP", -5: "HMC_ERR_WORKSPACE", -6: "HMC_ERR_UNSUPPORTED"}


class HMCError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


class hmc_tuning(ctypes.Structure):
    _fields_ = [("path", ctypes.c_int32), ("waves", ctypes.c_int32), ("mb", ctypes.c_int32),
                ("grid", ctypes.c_int32), ("rows_per_slice", ctypes.c_int32)]

    def as_dict(self) -> dict:
        return {k: int(getattr(self, k)) for k, _ in self._fields_}


class hmc_problem(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("p", ctypes.c_int64), ("K", ctypes.c_int32),
                ("xfmt", ctypes.c_int32), ("X", ctypes.c_void_p), ("X_lo", ctypes.c_void_p),
                ("ldx", ctypes.c_int64), ("y", ctypes.c_void_p), ("prior", ctypes.c_int32),
                ("prior_scale", ctypes.c_double), ("pin_last_class", ctypes.c_int32),
                ("link", ctypes.c_int32), ("tuning", hmc_tuning)]


class hmc_sample_args(ctypes.Structure):
    _fields_ = [("eps", ctypes.c_double), ("L", ctypes.c_int32), ("n_iter", ctypes.c_int32),
                ("first_iter", ctypes.c_int32), ("chain", ctypes.c_int32),
                ("seed", ctypes.c_uint64), ("replay_normals", ctypes.c_void_p),
                ("replay_uniforms", ctypes.c_void_p), ("inv_temperature", ctypes.c_void_p),
                ("samples", ctypes.c_void_p), ("accepted", ctypes.c_void_p),
                ("H", ctypes.c_void_p), ("divergent", ctypes.c_void_p)]


class hmc_batch_tuning(ctypes.Structure):
    _fields_ = [("rows_per_slice", ctypes.c_int32), ("grid", ctypes.c_int32)]


class hmc_batch_args(ctypes.Structure):
    _fields_ = [("eps", ctypes.c_void_p), ("L", ctypes.c_int32), ("n_iter", ctypes.c_int32),
                ("first_iter", ctypes.c_int32), ("seed", ctypes.c_uint64),
                ("tuning", hmc_batch_tuning), ("samples", ctypes.c_void_p),
                ("moments", ctypes.c_void_p), ("accepted", ctypes.c_void_p),
                ("H", ctypes.c_void_p), ("divergent", ctypes.c_void_p),
                ("replay_normals", ctypes.c_void_p), ("replay_uniforms", ctypes.c_void_p),
                ("inv_temperature", ctypes.c_void_p)]


_lib = None
_P = ctypes.POINTER


def load(path: str | None = None):
    """Load libhmc.so (built in-tree by ``paper_1402_4089_amd.build``); raise if absent."""
    global _lib
    if _lib is not None:
        return _lib
    path = path or LIB_PATH
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with `python -m paper_1402_4089_amd.build`")
    lib = ctypes.CDLL(path)
    lib.hmc_max_p.argtypes = [ctypes.c_int32, ctypes.c_int32]
    lib.hmc_max_p.restype = ctypes.c_int64
    lib.hmc_workspace_bytes.argtypes = [_P(hmc_problem), _P(ctypes.c_size_t)]
    lib.hmc_autotune_workspace_bytes.argtypes = [_P(hmc_problem), _P(ctypes.c_size_t)]
    lib.hmc_autotune.argtypes = [_P(hmc_problem), ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                 ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p, _P(hmc_tuning),
                                 _P(ctypes.c_double)]
    lib.hmc_autotune_workspace_bytes.restype = ctypes.c_int
    lib.hmc_autotune.restype = ctypes.c_int
    lib.hmc_logpost_grad.argtypes = [_P(hmc_problem), ctypes.c_void_p, ctypes.c_void_p,
                                     ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t,
                                     ctypes.c_void_p]
    lib.hmc_leapfrog.argtypes = [_P(hmc_problem), ctypes.c_void_p, ctypes.c_void_p,
                                 ctypes.c_void_p, ctypes.c_void_p, ctypes.c_double, ctypes.c_int32,
                                 ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p]
    lib.hmc_sample.argtypes = [_P(hmc_problem), ctypes.c_void_p, ctypes.c_void_p,
                               ctypes.c_void_p, _P(hmc_sample_args), ctypes.c_void_p,
                               ctypes.c_size_t, ctypes.c_void_p]
    lib.hmc_logpost_grad_noalloc.argtypes = [_P(hmc_problem), ctypes.c_void_p, ctypes.c_void_p,
                                             ctypes.c_void_p, ctypes.c_void_p]
    for f in ("hmc_workspace_bytes", "hmc_logpost_grad", "hmc_logpost_grad_noalloc", "hmc_leapfrog",
              "hmc_sample"):
        getattr(lib, f).restype = ctypes.c_int
    lib.hmc_split_bf16.argtypes = [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_int64,
                                   ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64,
                                   ctypes.c_void_p]
    lib.hmc_split_bf16.restype = ctypes.c_int
    _VP = ctypes.c_void_p
    lib.hmc_batch_workspace_bytes.argtypes = [_P(hmc_problem), ctypes.c_int32, ctypes.c_int32,
                                              _P(ctypes.c_size_t)]
    lib.hmc_logpost_grad_batched.argtypes = [_P(hmc_problem), ctypes.c_int32, ctypes.c_int32, _VP,
                                             _VP, _VP, _P(hmc_batch_tuning), _VP, ctypes.c_size_t, _VP]
    lib.hmc_sample_batched.argtypes = [_P(hmc_problem), ctypes.c_int32, ctypes.c_int32, _VP, _VP,
                                       _VP, _P(hmc_batch_args), _VP, ctypes.c_size_t, _VP]
    lib.hmc_batch_autotune.argtypes = [_P(hmc_problem), ctypes.c_int32, ctypes.c_int32, _VP, _VP,
                                       _VP, _VP, ctypes.c_size_t, _VP, _P(hmc_batch_tuning)]
    lib.hmc_plan_create.argtypes = [_P(_VP), _P(hmc_problem), _VP, _VP, _VP, _P(hmc_sample_args),
                                    _VP, ctypes.c_size_t, _VP]
    lib.hmc_plan_create_batched.argtypes = [_P(_VP), _P(hmc_problem), ctypes.c_int32, ctypes.c_int32,
                                            _VP, _VP, _VP, _P(hmc_batch_args), _VP, ctypes.c_size_t, _VP]
    lib.hmc_plan_launch.argtypes = [_VP, ctypes.c_int32, _VP]
    lib.hmc_plan_destroy.argtypes = [_VP]
    for fn in ("hmc_batch_workspace_bytes", "hmc_logpost_grad_batched", "hmc_sample_batched",
               "hmc_batch_autotune", "hmc_plan_create", "hmc_plan_create_batched", "hmc_plan_launch",
               "hmc_plan_destroy"):
        getattr(lib, fn).restype = ctypes.c_int
    lib.hmc_posterior_predictive.argtypes = [_P(hmc_problem), _VP, ctypes.c_int32, _VP, _VP, _VP]
    lib.hmc_posterior_predictive.restype = ctypes.c_int
    lib.hmc_stream_read.argtypes = [ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int32, ctypes.c_void_p,
                                    ctypes.c_void_p]
    lib.hmc_stream_read.restype = ctypes.c_int
    lib.hmc_profile_begin.argtypes = [ctypes.c_int32, ctypes.c_int32]
    lib.hmc_profile_end.argtypes = [_P(ctypes.c_int64), _P(ctypes.c_double), _P(ctypes.c_double),
                                    _P(ctypes.c_double)]
    lib.hmc_profile_begin.restype = ctypes.c_int
    lib.hmc_profile_end.restype = ctypes.c_int
    lib.hmc_status_string.argtypes = [ctypes.c_int]
    lib.hmc_status_string.restype = ctypes.c_char_p
    lib.hmc_last_error.argtypes = []
    lib.hmc_last_error.restype = ctypes.c_char_p
    _lib = lib
    return lib


def _check(status: int):
    if status != 0:
        raise HMCError(status, load().hmc_last_error().decode())


def _ptr(t) -> int | None:
    if t is None:
        return None
    return t.data_ptr()


def _need(t, name: str, dtype, shape, device):
    """Raise ValueError unless t is a contiguous tensor of this dtype and shape on the
    problem's device: the library reads and writes exactly that many elements through the
    raw pointer, so a mismatch would reach memory the tensor does not own."""
    if t is None or not hasattr(t, "data_ptr"):
        raise ValueError(f"{name} must be a tensor")
    if t.device != device:
        raise ValueError(f"{name} is on {t.device}, the problem on {device}")
    if t.dtype != dtype:
        raise ValueError(f"{name} must be {dtype}, got {t.dtype}")
    if tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} must have shape {tuple(shape)}, got {tuple(t.shape)}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")


def _need_logk(t, device, count: int = 1):
    import torch
    if t is None or not hasattr(t, "data_ptr") or t.device != device or t.dtype != torch.float64 \
            or t.numel() != count or not t.is_contiguous():
        raise ValueError(f"logpost must be a contiguous float64 tensor of {count} element(s) "
                         f"on {device}")


def _stream(stream) -> int | None:
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return s.cuda_stream


# ---------------------------------------------------------------- C entry points

def hmc_max_p(xfmt: int, K: int) -> int:
    return int(load().hmc_max_p(xfmt, K))


def hmc_workspace_bytes(desc: hmc_problem) -> int:
    out = ctypes.c_size_t(0)
    _check(load().hmc_workspace_bytes(ctypes.byref(desc), ctypes.byref(out)))
    return int(out.value)


def hmc_autotune_workspace_bytes(desc: hmc_problem) -> int:
    out = ctypes.c_size_t(0)
    _check(load().hmc_autotune_workspace_bytes(ctypes.byref(desc), ctypes.byref(out)))
    return int(out.value)


def hmc_autotune(desc, B, logpost, G, ws, stream=None):
    """(fastest hmc_tuning, its microseconds per gradient evaluation)."""
    t = hmc_tuning()
    us = ctypes.c_double(0.0)
    _check(load().hmc_autotune(ctypes.byref(desc), _ptr(B), _ptr(logpost), _ptr(G), _ptr(ws),
                               ws.numel(), _stream(stream), ctypes.byref(t), ctypes.byref(us)))
    return t, us.value


def hmc_logpost_grad(desc, B, logpost, G, ws, stream=None):
    _check(load().hmc_logpost_grad(ctypes.byref(desc), _ptr(B), _ptr(logpost), _ptr(G), _ptr(ws),
                                   ws.numel(), _stream(stream)))


def hmc_logpost_grad_noalloc(desc, B, logpost, G, stream=None):
    _check(load().hmc_logpost_grad_noalloc(ctypes.byref(desc), _ptr(B), _ptr(logpost), _ptr(G),
                                           _stream(stream)))


def hmc_leapfrog(desc, B, eta, G, logpost, eps, L, ws, stream=None):
    _check(load().hmc_leapfrog(ctypes.byref(desc), _ptr(B), _ptr(eta), _ptr(G), _ptr(logpost),
                               float(eps), int(L), _ptr(ws), ws.numel(), _stream(stream)))


def hmc_sample(desc, B, G, logpost, args: hmc_sample_args, ws, stream=None):
    _check(load().hmc_sample(ctypes.byref(desc), _ptr(B), _ptr(G), _ptr(logpost),
                             ctypes.byref(args), _ptr(ws), ws.numel(), _stream(stream)))


def hmc_split_bf16(X, src_fmt, n, p, ldx, X_hi, X_lo, ld_out, stream=None):
    _check(load().hmc_split_bf16(_ptr(X), src_fmt, n, p, ldx, _ptr(X_hi), _ptr(X_lo), ld_out,
                                 _stream(stream)))


def hmc_posterior_predictive(desc, samples, n_samples: int, mean_prob, classes, stream=None):
    _check(load().hmc_posterior_predictive(ctypes.byref(desc), _ptr(samples), int(n_samples),
                                           _ptr(mean_prob), _ptr(classes), _stream(stream)))


def posterior_predictive(X, samples, K: int, pin_last_class: bool = True, stream=None):
    """(mean class probabilities [n, K] float64, predicted classes [n] int32) of the rows of
    X (n x p float32/float64 on the GPU, unit column stride) over coefficient samples
    ([S, p, K] in X's dtype): Section 3.2's posterior-predictive classification."""
    import torch
    if X.dim() != 2 or X.stride(1) != 1 or X.dtype not in (torch.float32, torch.float64):
        raise ValueError("X must be a 2-D float32/float64 tensor with unit column stride")
    n, p = X.shape
    _need(samples, "samples", X.dtype, (samples.shape[0], p, int(K)), X.device)
    desc = hmc_problem(n=n, p=p, K=int(K), xfmt=HMC_X_F64 if X.dtype == torch.float64 else HMC_X_F32,
                       X=X.data_ptr(), X_lo=None, ldx=X.stride(0), y=None, prior=0, prior_scale=1.0,
                       pin_last_class=int(bool(pin_last_class)), link=HMC_LINK_SOFTMAX)
    mean = torch.empty(n, int(K), dtype=torch.float64, device=X.device)
    cls = torch.empty(n, dtype=torch.int32, device=X.device)
    hmc_posterior_predictive(desc, samples, samples.shape[0], mean, cls, stream)
    return mean, cls


def hmc_stream_read(buf, nbytes: int, reps: int = 1, sink=None, stream=None):
    _check(load().hmc_stream_read(_ptr(buf), int(nbytes), int(reps), _ptr(sink), _stream(stream)))


def hmc_profile_begin(capacity: int, repeat: int = 1):
    _check(load().hmc_profile_begin(int(capacity), int(repeat)))


def hmc_profile_end():
    """(timed event pairs, mean, min, max duration of one launch in microseconds) of the
    gradient pass over X."""
    n = ctypes.c_int64(0)
    mean, mn, mx = ctypes.c_double(0), ctypes.c_double(0), ctypes.c_double(0)
    _check(load().hmc_profile_end(ctypes.byref(n), ctypes.byref(mean), ctypes.byref(mn),
                                  ctypes.byref(mx)))
    return int(n.value), mean.value, mn.value, mx.value


# ---------------------------------------------------------------- torch-facing helpers

def split_bf16(X, hi_only: bool = False, stream=None):
    """Split-precision planes of X (n x p float32/float64 on the GPU): (hi, lo) bfloat16
    tensors of shape (n, p) viewed from row-pitch-padded storage; lo is None if hi_only."""
    import torch
    if X.dim() != 2 or X.stride(1) != 1 or X.dtype not in (torch.float32, torch.float64):
        raise ValueError("X must be a 2-D float32/float64 tensor with unit column stride")
    n, p = X.shape
    ldo = (p + 63) // 64 * 64            # rows on 128-byte lines (hmc_split_bf16's ld_out)
    hi = torch.empty(n, ldo, dtype=torch.bfloat16, device=X.device)
    lo = None if hi_only else torch.empty(n, ldo, dtype=torch.bfloat16, device=X.device)
    hmc_split_bf16(X, HMC_X_F64 if X.dtype == torch.float64 else HMC_X_F32, n, p, X.stride(0),
                   hi, lo, ldo, stream)
    return hi[:, :p], (None if lo is None else lo[:, :p])


def _aligned_workspace(nbytes: int, device):
    import torch
    ws = torch.empty(nbytes + 256, dtype=torch.uint8, device=device)
    off = (-ws.data_ptr()) % 256
    return ws[off:off + nbytes]


class Problem:
    """Device-resident problem: X (n x p, unit column stride), labels y.

    X is float32 or float64, or the bfloat16 hi plane of the split-precision form with the
    lo plane in ``X_lo`` (None for the hi-only form); the state dtype is then float32.
    ``link`` selects the per-row likelihood (HMC_LINK_SOFTMAX; HMC_LINK_POISSON with K = 1,
    y the counts and pin_last_class False; HMC_LINK_PROBIT likewise, y = 1 a success). Holds
    the C descriptor and a workspace tensor sized by hmc_workspace_bytes.
    """

    def __init__(self, X, y, K: int, prior: int = HMC_PRIOR_GAUSS, prior_scale: float = 1.0,
                 pin_last_class: bool = True, X_lo=None, link: int = HMC_LINK_SOFTMAX,
                 tuning=None):
        import torch
        if not (X.is_cuda and y.is_cuda):
            raise ValueError("X and y must be GPU tensors")
        if X.dim() != 2 or X.stride(1) != 1:
            raise ValueError("X must be 2-D with unit column stride")
        if X.dtype == torch.bfloat16:
            xfmt = HMC_X_BF16 if X_lo is None else HMC_X_BF16_HILO
            if X_lo is not None and (X_lo.dtype != torch.bfloat16 or X_lo.shape != X.shape
                                     or X_lo.stride() != X.stride()):
                raise ValueError("X_lo must be a bfloat16 plane laid out like X")
            self.dtype = torch.float32
        elif X.dtype in (torch.float32, torch.float64):
            if X_lo is not None:
                raise ValueError("X_lo is only for a bfloat16 X")
            xfmt = HMC_X_F64 if X.dtype == torch.float64 else HMC_X_F32
            self.dtype = X.dtype
        else:
            raise ValueError("X must be float32, float64 or bfloat16")
        if y.dtype != torch.int32 or y.dim() != 1 or y.shape[0] != X.shape[0]:
            raise ValueError("y must be int32 with one label per row of X")
        self.X, self.X_lo, self.y, self.K = X, X_lo, y.contiguous(), int(K)
        self.n, self.p = X.shape
        self.xfmt = xfmt
        self.link = int(link)
        self.desc = hmc_problem(n=self.n, p=self.p, K=self.K, xfmt=xfmt,
                                X=X.data_ptr(), X_lo=None if X_lo is None else X_lo.data_ptr(),
                                ldx=X.stride(0), y=self.y.data_ptr(),
                                prior=int(prior), prior_scale=float(prior_scale),
                                pin_last_class=int(bool(pin_last_class)), link=self.link)
        self.tuned_us = None
        if tuning == "auto":
            from . import tuning as _tuning
            tuning, self.tuned_us = _tuning.tuned(self)
        if tuning is not None:
            t = tuning if isinstance(tuning, hmc_tuning) else hmc_tuning(**dict(tuning))
            self.desc.tuning = t
        self.ws = _aligned_workspace(hmc_workspace_bytes(self.desc), X.device)

    @property
    def tuning(self) -> dict:
        return self.desc.tuning.as_dict()

    def zeros_state(self):
        import torch
        return torch.zeros(self.p, self.K, dtype=self.dtype, device=self.X.device)


def logpost_grad(prob: Problem, B, stream=None):
    """(log K(B) as a 0-d float64 tensor, gradient G) at B."""
    import torch
    _need(B, "B", prob.dtype, (prob.p, prob.K), prob.X.device)
    logk = torch.empty((), dtype=torch.float64, device=B.device)
    G = torch.empty_like(B)
    hmc_logpost_grad(prob.desc, B, logk, G, prob.ws, stream)
    return logk, G


def leapfrog(prob: Problem, B, eta, G, logk, eps: float, L: int, stream=None):
    """L leapfrog updates of (B, eta, G, logk) in place."""
    for t, name in ((B, "B"), (eta, "eta"), (G, "G")):
        _need(t, name, prob.dtype, (prob.p, prob.K), prob.X.device)
    _need_logk(logk, prob.X.device)
    hmc_leapfrog(prob.desc, B, eta, G, logk, eps, L, prob.ws, stream)


def sample(prob: Problem, B, G, logk, eps: float, L: int, n_iter: int, normals=None,
           uniforms=None, seed: int = 0, chain: int = 0, first_iter: int = 0,
           inv_temperature=None, record_samples: bool = True, stream=None):
    """n_iter HMC transitions in place on (B, G, logk); returns the device records."""
    args, out = _sample_args(prob, B, eps, L, n_iter, normals, uniforms, seed, chain, first_iter,
                             inv_temperature, record_samples, G, logk)
    hmc_sample(prob.desc, B, G, logk, args, prob.ws, stream)
    return out


# ---------------------------------------------------------------- plans and batches

class Plan:
    """A captured HIP graph of one HMC iteration (hmc_plan_create / _batched); ``launch(n)``
    replays it n times on the stream. Keeps the objects baked into the graph alive."""

    def __init__(self, handle, keep):
        self._h = handle
        self._keep = keep

    def launch(self, n_iter: int, stream=None):
        _check(load().hmc_plan_launch(self._h, int(n_iter), _stream(stream)))

    def destroy(self):
        if self._h:
            _check(load().hmc_plan_destroy(self._h))
            self._h = None

    def __del__(self):
        try:
            self.destroy()
        except Exception:  # interpreter shutdown: the library may already be gone
            pass


def _sample_args(prob, B, eps, L, n_iter, normals, uniforms, seed, chain, first_iter,
                 inv_temperature, record_samples, G=None, logk=None):
    import torch
    dev = prob.X.device
    _need(B, "B", prob.dtype, (prob.p, prob.K), dev)
    if G is not None:
        _need(G, "G", prob.dtype, (prob.p, prob.K), dev)
    if logk is not None:
        _need_logk(logk, dev)
    if normals is not None:
        _need(normals, "normals", torch.float64, (int(n_iter), prob.p, prob.K), dev)
    if uniforms is not None:
        _need(uniforms, "uniforms", torch.float64, (int(n_iter),), dev)
    if inv_temperature is not None:
        _need(inv_temperature, "inv_temperature", torch.float64, (int(n_iter),), dev)
    out = dict(accepted=torch.empty(n_iter, dtype=torch.int32, device=dev),
               divergent=torch.empty(n_iter, dtype=torch.int32, device=dev),
               H=torch.empty(n_iter, 2, dtype=torch.float64, device=dev))
    out["samples"] = (torch.empty(n_iter, prob.p, prob.K, dtype=prob.dtype, device=dev)
                      if record_samples else None)
    args = hmc_sample_args(eps=float(eps), L=int(L), n_iter=int(n_iter), first_iter=int(first_iter),
                           chain=int(chain), seed=int(seed), replay_normals=_ptr(normals),
                           replay_uniforms=_ptr(uniforms), inv_temperature=_ptr(inv_temperature),
                           samples=_ptr(out["samples"]), accepted=_ptr(out["accepted"]),
                           H=_ptr(out["H"]), divergent=_ptr(out["divergent"]))
    return args, out


def plan(prob: Problem, B, G, logk, eps: float, L: int, n_iter: int, normals=None, uniforms=None,
         seed: int = 0, chain: int = 0, first_iter: int = 0, inv_temperature=None,
         record_samples: bool = True, stream=None):
    """Graph plan of hmc_sample's iteration; returns (Plan, records dict of n_iter slots)."""
    args, out = _sample_args(prob, B, eps, L, n_iter, normals, uniforms, seed, chain, first_iter,
                             inv_temperature, record_samples, G, logk)
    h = ctypes.c_void_p()
    _check(load().hmc_plan_create(ctypes.byref(h), ctypes.byref(prob.desc), _ptr(B), _ptr(G),
                                  _ptr(logk), ctypes.byref(args), _ptr(prob.ws), prob.ws.numel(),
                                  _stream(stream)))
    return Plan(h, (prob, B, G, logk, normals, uniforms, inv_temperature, out, args)), out


class Batch:
    """Many split-precision problems (bf16 planes) with ``chains`` chains each; every chain
    takes ceil(K_max / 16) class blocks of the batch's largest K, chains x blocks <= 4.

    State: ``B[b]``/``G[b]`` are float32 tensors [chains, p_b, K_b]; ``logpost`` is a float64
    tensor [n_prob, chains]. Holds the descriptor array and the batch workspace.
    """

    def __init__(self, problems, chains: int = 4):
        import torch
        self.problems = list(problems)
        self.chains = int(chains)
        self.n_prob = len(self.problems)
        self.descs = (hmc_problem * self.n_prob)(*[pr.desc for pr in self.problems])
        nbytes = ctypes.c_size_t(0)
        _check(load().hmc_batch_workspace_bytes(self.descs, self.n_prob, self.chains, ctypes.byref(nbytes)))
        dev = self.problems[0].X.device
        ws = torch.empty(nbytes.value + 256, dtype=torch.uint8, device=dev)
        off = (-ws.data_ptr()) % 256
        self.ws = ws[off:off + nbytes.value]
        self.tuning = hmc_batch_tuning(0, 0)

    def zeros_state(self):
        import torch
        dev = self.ws.device
        B = [torch.zeros(self.chains, pr.p, pr.K, dtype=torch.float32, device=dev) for pr in self.problems]
        G = [torch.empty_like(b) for b in B]
        logk = torch.empty(self.n_prob, self.chains, dtype=torch.float64, device=dev)
        return B, G, logk

    @staticmethod
    def _ptrs(ts):
        return (ctypes.c_void_p * len(ts))(*[t.data_ptr() for t in ts])

    def _check_state(self, B, G, logk):
        import torch
        dev = self.ws.device
        for name, ts in (("B", B), ("G", G)):
            if len(ts) != self.n_prob:
                raise ValueError(f"{name} must hold one tensor per problem ({self.n_prob})")
            for b, (t, pr) in enumerate(zip(ts, self.problems)):
                _need(t, f"{name}[{b}]", torch.float32, (self.chains, pr.p, pr.K), dev)
        _need_logk(logk, dev, self.n_prob * self.chains)

    def logpost_grad(self, B, G, logk, stream=None):
        """log K and gradient at every chain's B, into G and logk (in place)."""
        self._check_state(B, G, logk)
        self._keep = (self._ptrs(B), self._ptrs(G))
        _check(load().hmc_logpost_grad_batched(self.descs, self.n_prob, self.chains, self._keep[0],
                                               _ptr(logk), self._keep[1], ctypes.byref(self.tuning),
                                               _ptr(self.ws), self.ws.numel(), _stream(stream)))

    def autotune(self, B, G, logk, stream=None):
        """Measure the candidate decompositions; keeps and returns the fastest (rows, grid)."""
        self._check_state(B, G, logk)
        out = hmc_batch_tuning(0, 0)
        bp, gp = self._ptrs(B), self._ptrs(G)
        _check(load().hmc_batch_autotune(self.descs, self.n_prob, self.chains, bp, gp, _ptr(logk),
                                         _ptr(self.ws), self.ws.numel(), _stream(stream),
                                         ctypes.byref(out)))
        self.tuning = out
        return out.rows_per_slice, out.grid

    def _args(self, eps, L, n_iter, seed, first_iter, record_samples, moments, records,
              normals=None, uniforms=None, inv_temperature=None):
        import torch
        dev = self.ws.device
        nch = self.n_prob * self.chains
        if len(eps) != self.n_prob:
            raise ValueError(f"eps must hold one step size per problem ({self.n_prob})")
        eps_arr = (ctypes.c_double * self.n_prob)(*[float(e) for e in eps])
        if (normals is None) != (uniforms is None):
            raise ValueError("normals and uniforms must be given together")
        nrm_arr = uni_arr = None
        if normals is not None:
            if len(normals) != self.n_prob or len(uniforms) != self.n_prob:
                raise ValueError("normals and uniforms must hold one tensor per problem")
            for b, pr in enumerate(self.problems):
                _need(normals[b], f"normals[{b}]", torch.float64,
                      (int(n_iter), self.chains, pr.p, pr.K), dev)
                _need(uniforms[b], f"uniforms[{b}]", torch.float64, (int(n_iter), self.chains), dev)
            nrm_arr, uni_arr = self._ptrs(normals), self._ptrs(uniforms)
        if inv_temperature is not None:
            _need(inv_temperature, "inv_temperature", torch.float64, (int(n_iter),), dev)
        out = {}
        if records:
            out.update(accepted=torch.empty(n_iter, nch, dtype=torch.int32, device=dev),
                       divergent=torch.empty(n_iter, nch, dtype=torch.int32, device=dev),
                       H=torch.empty(n_iter, nch, 2, dtype=torch.float64, device=dev))
        samp_arr = mom_arr = None
        if record_samples is not False and record_samples is not None:
            # True: every problem; a collection of problem indices: those problems only
            pick = set(range(self.n_prob)) if record_samples is True else set(record_samples)
            out["samples"] = [torch.empty(n_iter, self.chains, pr.p, pr.K, dtype=torch.float32, device=dev)
                              if b in pick else None for b, pr in enumerate(self.problems)]
            samp_arr = (ctypes.c_void_p * self.n_prob)(*[None if t is None else t.data_ptr()
                                                         for t in out["samples"]])
        if moments:
            out["moments"] = [torch.zeros(2, self.chains, pr.p, pr.K, dtype=torch.float64, device=dev)
                              for pr in self.problems]
            mom_arr = self._ptrs(out["moments"])
        args = hmc_batch_args(eps=ctypes.cast(eps_arr, ctypes.c_void_p), L=int(L), n_iter=int(n_iter),
                              first_iter=int(first_iter), seed=int(seed), tuning=self.tuning,
                              samples=None if samp_arr is None else ctypes.cast(samp_arr, ctypes.c_void_p),
                              moments=None if mom_arr is None else ctypes.cast(mom_arr, ctypes.c_void_p),
                              accepted=_ptr(out.get("accepted")), H=_ptr(out.get("H")),
                              divergent=_ptr(out.get("divergent")),
                              replay_normals=None if nrm_arr is None else ctypes.cast(nrm_arr, ctypes.c_void_p),
                              replay_uniforms=None if uni_arr is None else ctypes.cast(uni_arr, ctypes.c_void_p),
                              inv_temperature=_ptr(inv_temperature))
        return args, out, (eps_arr, samp_arr, mom_arr, nrm_arr, uni_arr, normals, uniforms,
                           inv_temperature)

    def sample(self, B, G, logk, eps, L: int, n_iter: int, seed: int = 0, first_iter: int = 0,
               record_samples: bool = False, moments: bool = False, records: bool = True,
               normals=None, uniforms=None, inv_temperature=None, stream=None):
        """n_iter transitions of every chain in place; returns the device records.

        normals[b] ([n_iter, chains, p_b, K_b] float64) and uniforms[b] ([n_iter, chains])
        replay the draws of problem b's chains instead of Philox; inv_temperature
        ([n_iter] float64) applies the annealed acceptance to every chain."""
        self._check_state(B, G, logk)
        args, out, keep = self._args(eps, L, n_iter, seed, first_iter, record_samples, moments, records,
                                     normals, uniforms, inv_temperature)
        bp, gp = self._ptrs(B), self._ptrs(G)
        _check(load().hmc_sample_batched(self.descs, self.n_prob, self.chains, bp, gp, _ptr(logk),
                                         ctypes.byref(args), _ptr(self.ws), self.ws.numel(),
                                         _stream(stream)))
        return out

    def plan(self, B, G, logk, eps, L: int, n_iter: int, seed: int = 0, first_iter: int = 0,
             record_samples: bool = False, moments: bool = False, records: bool = True,
             normals=None, uniforms=None, inv_temperature=None, stream=None):
        """Graph plan of one batched iteration; returns (Plan, records of n_iter slots)."""
        self._check_state(B, G, logk)
        args, out, keep = self._args(eps, L, n_iter, seed, first_iter, record_samples, moments, records,
                                     normals, uniforms, inv_temperature)
        bp, gp = self._ptrs(B), self._ptrs(G)
        h = ctypes.c_void_p()
        _check(load().hmc_plan_create_batched(ctypes.byref(h), self.descs, self.n_prob, self.chains,
                                              bp, gp, _ptr(logk), ctypes.byref(args), _ptr(self.ws),
                                              self.ws.numel(), _stream(stream)))
        return Plan(h, (self, B, G, logk, out, args, keep, bp, gp)), out


def _make_logposterior():
    import torch

    class LogPosterior(torch.autograd.Function):
        """log K(B) as a differentiable torch function whose backward is the library gradient.

        forward(B, problem) -> 0-d float64 tensor log K(B) (equation (logkernel)); the fused
        pass also produces the gradient (equation (gradient)), which backward returns scaled
        by the incoming gradient. With the last class pinned the returned gradient is zero in
        column K-1 (that column is a constant of the model, not a parameter).
        """

        @staticmethod
        def forward(ctx, B, problem):
            logk, G = logpost_grad(problem, B.detach().contiguous())
            ctx.save_for_backward(G)
            return logk

        @staticmethod
        def backward(ctx, grad_out):
            (G,) = ctx.saved_tensors
            return grad_out.to(G.dtype) * G, None

    return LogPosterior


def __getattr__(name):
    if name == "LogPosterior":
        cls = _make_logposterior()
        globals()["LogPosterior"] = cls
        return cls
    raise AttributeError(name)
