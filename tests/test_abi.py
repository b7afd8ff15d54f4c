"""The C-ABI library loads on a machine without a GPU, exports every declared entry point
and rejects bad arguments on the host before any device work."""
import ctypes
import os
import re

import pytest

import paper_1402_4089_amd as hmc

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    names = set()
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if fn.endswith(".h"):
            txt = open(os.path.join(ROOT, "include", fn)).read()
            names |= set(re.findall(r"^\s*(?:const\s+)?[\w]+\*?\s+\*?(hmc_\w+)\s*\(", txt, re.M))
    return names


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(hmc.LIB_PATH):
        pytest.fail("libhmc.so is not built: run python -m paper_1402_4089_amd.build")
    return hmc.load()


def test_exports_every_declared_symbol(lib):
    names = _declared()
    assert {"hmc_logpost_grad", "hmc_leapfrog", "hmc_sample", "hmc_workspace_bytes"} <= names
    for nm in names:
        assert hasattr(lib, nm), nm


def test_status_strings(lib):
    for code in [0, -1, -2, -3, -4, -5, -6]:
        assert lib.hmc_status_string(code).decode()


def _desc(**kw):
    d = dict(n=1000, p=100, K=5, xfmt=hmc.HMC_X_F32, X=4096, X_lo=None, ldx=100, y=8192,
             prior=hmc.HMC_PRIOR_GAUSS, prior_scale=1.0, pin_last_class=1)
    d.update(kw)
    return hmc.hmc_problem(**d)


def test_workspace_bytes_valid(lib):
    nb = hmc.hmc_workspace_bytes(_desc())
    # at least the per-workgroup gradient partials: ceil(1000/16) workgroups x p x K floats
    assert nb >= 63 * 100 * 5 * 4


@pytest.mark.parametrize("kw,status", [
    (dict(K=1), -2), (dict(K=65), -2), (dict(n=0), -2), (dict(p=0), -2), (dict(ldx=50), -2),
    (dict(xfmt=7), -3), (dict(prior=5), -3), (dict(prior_scale=0.0), -1),
    (dict(prior_scale=float("nan")), -1), (dict(X=None), -1), (dict(y=None), -1),
    (dict(pin_last_class=2), -1), (dict(X_lo=16), -1), (dict(p=10 ** 9, ldx=10 ** 9), -6),
    (dict(xfmt=2), -1), (dict(xfmt=2, X_lo=8192, ldx=100), -2), (dict(xfmt=2, X_lo=8200, ldx=104), -1),
    (dict(xfmt=3, X=4104, ldx=104), -1), (dict(xfmt=3, X_lo=8192, ldx=104), -1),
    # Poisson link: one coefficient column, nothing pinned, FP64/FP32 X; unknown links
    (dict(link=1), -2), (dict(link=1, K=1), -1), (dict(link=1, K=1, pin_last_class=0, xfmt=3, ldx=104), -6),
    # probit link: the same constraints
    (dict(link=2), -2), (dict(link=2, K=1), -1), (dict(link=2, K=1, pin_last_class=0, xfmt=2, X_lo=8192, ldx=104), -6),
    (dict(link=3), -3), (dict(link=-1), -3),
])
def test_bad_problem_rejected_on_host(lib, kw, status):
    with pytest.raises(hmc.HMCError) as ei:
        hmc.hmc_workspace_bytes(_desc(**kw))
    assert ei.value.status == status
    assert lib.hmc_last_error().decode()


@pytest.mark.parametrize("link", [hmc.HMC_LINK_POISSON, hmc.HMC_LINK_PROBIT])
def test_one_column_links_accepted(lib, link):
    for xfmt in (hmc.HMC_X_F32, hmc.HMC_X_F64):
        for p in (100, 5000):
            assert hmc.hmc_workspace_bytes(_desc(link=link, K=1, pin_last_class=0,
                                                 xfmt=xfmt, p=p, ldx=p)) > 0


def test_bf16_formats_accepted(lib):
    for fmt, lo in [(2, 8192), (3, None)]:
        nb = hmc.hmc_workspace_bytes(_desc(xfmt=fmt, X_lo=lo, ldx=104, K=64, p=100))
        # packed residual operand: 2 planes x 2 bytes x 64 padded classes per row
        assert nb >= 1000 * 64 * 4


@pytest.mark.parametrize("kw,status", [
    (dict(src_fmt=2), -3), (dict(ld_out=50), -2), (dict(ld_out=100), -2), (dict(ldx=10), -2),
    (dict(X=None), -1), (dict(X_hi=4104), -1), (dict(n=0), -2),
])
def test_split_rejects_bad_arguments(lib, kw, status):
    d = dict(X=4096, src_fmt=0, n=10, p=20, ldx=20, X_hi=8192, X_lo=16384, ld_out=24)
    d.update(kw)
    st = lib.hmc_split_bf16(d["X"], d["src_fmt"], d["n"], d["p"], d["ldx"], d["X_hi"], d["X_lo"],
                            d["ld_out"], None)
    assert st == status


def test_max_p_reported(lib):
    assert hmc.hmc_max_p(hmc.HMC_X_F32, 10) >= 1000
    assert hmc.hmc_max_p(hmc.HMC_X_F64, 3) >= 20
    assert hmc.hmc_max_p(9, 3) == 0
    assert hmc.hmc_max_p(hmc.HMC_X_BF16_HILO, 64) >= 4096


def test_calls_reject_bad_workspace_before_launch(lib):
    d = _desc()
    st = lib.hmc_logpost_grad(ctypes.byref(d), ctypes.c_void_p(4096), ctypes.c_void_p(4096),
                              ctypes.c_void_p(4096), None, 0, None)
    assert st == -5
    st = lib.hmc_logpost_grad(ctypes.byref(d), ctypes.c_void_p(4096), ctypes.c_void_p(4096),
                              ctypes.c_void_p(4096), ctypes.c_void_p(4096 + 8), 1 << 30, None)
    assert st == -5
    args = hmc.hmc_sample_args(eps=0.1, L=0, n_iter=1)
    st = lib.hmc_sample(ctypes.byref(d), ctypes.c_void_p(4096), ctypes.c_void_p(4096),
                        ctypes.c_void_p(4096), ctypes.byref(args), ctypes.c_void_p(4096), 1 << 30, None)
    assert st == -1
    st = lib.hmc_leapfrog(ctypes.byref(d), ctypes.c_void_p(4096), ctypes.c_void_p(4096),
                          ctypes.c_void_p(4096), ctypes.c_void_p(4096), float("inf"), 3,
                          ctypes.c_void_p(4096), 1 << 30, None)
    assert st == -1


def test_binding_refuses_missing_library(tmp_path):
    import importlib
    mod = importlib.import_module("paper_1402_4089_amd")
    saved = mod._lib
    try:
        mod._lib = None
        with pytest.raises(RuntimeError):
            mod.load(str(tmp_path / "nope.so"))
    finally:
        mod._lib = saved


def _bdesc(**kw):
    d = dict(n=1000, p=100, K=5, xfmt=hmc.HMC_X_BF16_HILO, X=4096, X_lo=8192, ldx=104, y=16384,
             prior=hmc.HMC_PRIOR_GAUSS, prior_scale=1.0, pin_last_class=1)
    d.update(kw)
    return hmc.hmc_problem(**d)


def _batch_bytes(lib, descs, chains):
    arr = (hmc.hmc_problem * len(descs))(*descs)
    nb = ctypes.c_size_t(0)
    st = lib.hmc_batch_workspace_bytes(arr, len(descs), chains, ctypes.byref(nb))
    return st, nb.value


def test_batch_workspace_and_validation(lib):
    st, nb = _batch_bytes(lib, [_bdesc(), _bdesc(n=50, p=7, K=2)], 4)
    assert st == 0 and nb > 0
    assert _batch_bytes(lib, [_bdesc()], 3)[0] == -2                       # chains must be 1, 2 or 4
    # a chain of K classes takes ceil(K / 16) blocks; chains x blocks <= 4
    assert _batch_bytes(lib, [_bdesc(K=17)], 4)[0] == -2
    assert _batch_bytes(lib, [_bdesc(K=17)], 2)[0] == 0
    assert _batch_bytes(lib, [_bdesc(K=33)], 2)[0] == -2
    assert _batch_bytes(lib, [_bdesc(K=64)], 1)[0] == 0
    assert _batch_bytes(lib, [_bdesc(K=65)], 1)[0] == -2
    assert _batch_bytes(lib, [_bdesc(K=5), _bdesc(K=20)], 4)[0] == -2     # the largest K counts
    assert _batch_bytes(lib, [_bdesc(K=17)], 2)[1] > _batch_bytes(lib, [_bdesc(K=16)], 2)[1]
    assert _batch_bytes(lib, [_bdesc(xfmt=1, X_lo=None, ldx=100)], 4)[0] == -6   # bf16 planes only
    assert _batch_bytes(lib, [_bdesc(), _bdesc(xfmt=3, X_lo=None)], 4)[0] == -3  # one format per batch
    assert _batch_bytes(lib, [], 4)[0] == -2
    # workspace grows with the problem count and is independent of the tuning
    assert _batch_bytes(lib, [_bdesc()] * 3, 4)[1] > _batch_bytes(lib, [_bdesc()] * 2, 4)[1]


def test_batch_calls_reject_bad_arguments_before_launch(lib):
    arr = (hmc.hmc_problem * 1)(_bdesc())
    ptrs = (ctypes.c_void_p * 1)(4096)
    eps = (ctypes.c_double * 1)(float("nan"))
    args = hmc.hmc_batch_args(eps=ctypes.cast(eps, ctypes.c_void_p), L=3, n_iter=2)
    st = lib.hmc_sample_batched(arr, 1, 4, ptrs, ptrs, 4096, ctypes.byref(args), 4096, 1 << 30, None)
    assert st == -1
    eps[0] = 0.01
    st = lib.hmc_sample_batched(arr, 1, 4, ptrs, ptrs, 4096, ctypes.byref(args), 4096, 16, None)
    assert st == -5
    bad = hmc.hmc_batch_tuning(rows_per_slice=1000, grid=0)
    st = lib.hmc_logpost_grad_batched(arr, 1, 4, ptrs, 4096, ptrs, ctypes.byref(bad), 4096, 1 << 30, None)
    assert st == -1
    assert lib.hmc_plan_launch(None, 1, None) == -1
    assert lib.hmc_plan_destroy(None) == 0
    h = ctypes.c_void_p()
    sargs = hmc.hmc_sample_args(eps=0.1, L=0, n_iter=1)
    st = lib.hmc_plan_create(ctypes.byref(h), ctypes.byref(_desc()), 4096, 4096, 4096,
                             ctypes.byref(sargs), 4096, 1 << 30, None)
    assert st == -1 and not h.value


@pytest.mark.parametrize("buf,nbytes,reps,status", [
    (None, 1024, 1, -1), (4104, 1024, 1, -1), (4096, 1000, 1, -1), (4096, 0, 1, -1), (4096, 1024, 0, -1),
])
def test_stream_read_rejects_bad_arguments(lib, buf, nbytes, reps, status):
    assert lib.hmc_stream_read(buf, nbytes, reps, None, None) == status


@pytest.mark.parametrize("capacity,repeat", [(0, 1), (4, 0), (4, 65), (1 << 21, 1)])
def test_profile_begin_rejects_bad_arguments(lib, capacity, repeat):
    assert lib.hmc_profile_begin(capacity, repeat) == -1
    # nothing was started: ending reports that profiling is not active
    assert lib.hmc_profile_end(None, None, None, None) == -1


@pytest.mark.parametrize("xfmt,ok_ldx,lo", [
    (hmc.HMC_X_F32, (1 << 24) - 1, None), (hmc.HMC_X_F64, (1 << 23) - 1, None),
    (hmc.HMC_X_BF16, (1 << 23) - 8, None), (hmc.HMC_X_BF16_HILO, (1 << 23) - 8, 8192)])
def test_row_pitch_limit_of_32bit_offsets(lib, xfmt, ok_ldx, lo):
    """The largest row pitch is the one whose in-kernel 32-bit byte offsets (64 rows of
    FP32/FP64, 128 rows of a bf16 plane) cannot wrap; one element (one 16-byte row step for
    bf16) more is refused as unsupported rather than computed wrongly."""
    step = 8 if xfmt in (hmc.HMC_X_BF16, hmc.HMC_X_BF16_HILO) else 1
    assert hmc.hmc_workspace_bytes(_desc(xfmt=xfmt, X_lo=lo, n=10, p=100, ldx=ok_ldx)) > 0
    with pytest.raises(hmc.HMCError) as ei:
        hmc.hmc_workspace_bytes(_desc(xfmt=xfmt, X_lo=lo, n=10, p=100, ldx=ok_ldx + step))
    assert ei.value.status == -6
    assert hmc.hmc_max_p(xfmt, 4) == ok_ldx


def test_row_count_limits_of_32bit_offsets(lib):
    """Per-row work buffers addressed with 32-bit offsets bound n: the wide-p residuals
    (n * 16 * 4 bytes at K = 4, FP32) and the packed split-precision residuals
    ((n + 128) * 64 bytes at K <= 16)."""
    lim = (2 ** 32 - 1) // 64                                  # wide-p FP32, one class block
    assert hmc.hmc_workspace_bytes(_desc(n=lim, p=2000, ldx=2000, K=4)) > 0
    with pytest.raises(hmc.HMCError) as ei:
        hmc.hmc_workspace_bytes(_desc(n=lim + 1, p=2000, ldx=2000, K=4))
    assert ei.value.status == -6
    # the row tile (p <= 1024) keeps no per-row buffer: the same n is accepted there
    assert hmc.hmc_workspace_bytes(_desc(n=lim + 1, p=1000, ldx=1000, K=4)) > 0
    lim_b = (2 ** 32 - 1) // 64 - 128
    assert hmc.hmc_workspace_bytes(_desc(xfmt=3, n=lim_b, p=100, ldx=104, K=4)) > 0
    with pytest.raises(hmc.HMCError) as ei:
        hmc.hmc_workspace_bytes(_desc(xfmt=3, n=lim_b + 1, p=100, ldx=104, K=4))
    assert ei.value.status == -6
    # batched: the chains of a problem multiply the packed residual's row bytes
    assert _batch_bytes(lib, [_bdesc(n=lim_b // 4 - 96, p=64, ldx=64)], 4)[0] == 0
    assert _batch_bytes(lib, [_bdesc(n=lim_b // 4 + 1, p=64, ldx=64)], 4)[0] == -6


def test_batch_replay_arguments_checked(lib):
    arr = (hmc.hmc_problem * 1)(_bdesc())
    ptrs = (ctypes.c_void_p * 1)(4096)
    eps = (ctypes.c_double * 1)(0.01)
    nrm = (ctypes.c_void_p * 1)(4096)
    args = hmc.hmc_batch_args(eps=ctypes.cast(eps, ctypes.c_void_p), L=3, n_iter=2,
                              replay_normals=ctypes.cast(nrm, ctypes.c_void_p))
    st = lib.hmc_sample_batched(arr, 1, 4, ptrs, ptrs, 4096, ctypes.byref(args), 4096, 1 << 30, None)
    assert st == -1                                      # normals without uniforms
    nul = (ctypes.c_void_p * 1)(None)
    args.replay_uniforms = ctypes.cast(nul, ctypes.c_void_p)
    st = lib.hmc_sample_batched(arr, 1, 4, ptrs, ptrs, 4096, ctypes.byref(args), 4096, 1 << 30, None)
    assert st == -1                                      # a NULL entry in the uniforms array


@pytest.mark.parametrize("tuning,status", [
    (dict(path=4), -1), (dict(path=0, grid=3), -1), (dict(path=1, waves=8, mb=3), -1),
    (dict(path=1, waves=8, mb=1), -1),                        # 128 columns do not cover p = 1000
    (dict(path=3), -1),                                       # split-precision needs bf16 X
    (dict(path=2, rows_per_slice=100), -1), (dict(path=1, grid=5000), -1),
    (dict(path=1, grid=-1), -1),
])
def test_bad_tuning_rejected(lib, tuning, status):
    d = _desc(n=20000, p=1000, ldx=1000, K=10)
    d.tuning = hmc.hmc_tuning(**tuning)
    with pytest.raises(hmc.HMCError) as ei:
        hmc.hmc_workspace_bytes(d)
    assert ei.value.status == status


def test_tuning_sets_the_workspace(lib):
    d = _desc(n=20000, p=1000, ldx=1000, K=10)
    rule = hmc.hmc_workspace_bytes(d)
    d.tuning = hmc.hmc_tuning(path=1, waves=16, mb=4, grid=125)
    half = hmc.hmc_workspace_bytes(d)
    assert rule - half >= 125 * 10048 * 4 - 4096              # 125 fewer partial gradients
    d.tuning = hmc.hmc_tuning(path=2)
    assert hmc.hmc_workspace_bytes(d) > 0                      # the wide-p path takes any p
    d.tuning = hmc.hmc_tuning()
    assert hmc.hmc_autotune_workspace_bytes(d) >= rule
    b = _desc(xfmt=3, n=5000, p=100, ldx=104, K=5)
    b.tuning = hmc.hmc_tuning(path=3, grid=64, rows_per_slice=1024)
    assert hmc.hmc_workspace_bytes(b) > 0
    b.tuning = hmc.hmc_tuning(path=1)
    with pytest.raises(hmc.HMCError):
        hmc.hmc_workspace_bytes(b)
    wide = _desc(n=100, p=5000, ldx=5000, K=4)
    wide.tuning = hmc.hmc_tuning(path=1)
    with pytest.raises(hmc.HMCError) as ei:
        hmc.hmc_workspace_bytes(wide)
    assert ei.value.status == -6


def test_tuning_cache_round_trip(tmp_path, monkeypatch):
    from paper_1402_4089_amd import tuning

    class P:                                     # the fields the cache key reads
        n, p, K, xfmt, link = 20000, 1000, 10, hmc.HMC_X_F32, 0
    path = tmp_path / "t.json"
    monkeypatch.setenv(tuning.ENV, str(path))
    assert tuning.cache_path() == str(path)
    assert tuning.lookup(P) is None
    d = {tuning.key_of(P): {"tuning": {"path": 1, "waves": 16, "mb": 4, "grid": 250,
                                       "rows_per_slice": 0}}}
    tuning._write(str(path), d)
    assert tuning.lookup(P)["grid"] == 250

    class Q(P):                                  # same key: same column blocks and row bucket
        n, p = 17000, 993
    assert tuning.key_of(Q) == tuning.key_of(P)

    class R(P):                                  # another column-block count: another key
        p = 1100
    assert tuning.lookup(R) is None


def test_tuning_cache_entry_the_library_refuses_is_not_used(lib):
    """A cached decomposition is checked against this build before use: a row-tile entry
    for a problem whose row does not fit the row tile, or a malformed entry, is refused
    (the autotuner then measures again); a valid one is accepted."""
    from paper_1402_4089_amd import tuning

    class P:
        desc = _desc(n=100, p=5000, ldx=5000, K=4)
    assert not tuning.usable(P, {"path": 1, "waves": 16, "mb": 4, "grid": 250, "rows_per_slice": 0})
    assert not tuning.usable(P, {"path": 2, "bogus": 1})
    assert tuning.usable(P, {"path": 2, "waves": 0, "mb": 0, "grid": 0, "rows_per_slice": 0})
