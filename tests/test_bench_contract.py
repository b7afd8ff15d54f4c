"""The benchmark's command-line contract: one JSON line with the fields the harness reads, a
refusal of more than one GPU, and the link between the committed counter summary and the
kernel source it was taken on."""
import json
import os
import subprocess
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_counter_summary_matches_its_kernel_source():
    # bench.py reports HBM traffic only from a summary taken on the current fused kernel:
    # a summary of another kernel source gives null, never a stale figure
    sys.path.insert(0, ROOT)
    import bench
    path = os.path.join(ROOT, "profiles", "fused_logpost_grad_c2_f32_pmc.txt")
    text = open(path).read()
    assert "command (fetch):" in text and "rocprofv3 --pmc FETCH_SIZE" in text
    current = f"kernel_source_sha256_16: {bench.kernel_source_hash()}" in text
    traffic = bench.read_traffic("c2_f32")
    if current:
        assert traffic is not None and 80e6 < traffic < 120e6
    else:
        assert traffic is None


@pytest.mark.parametrize("prior,pin", [(0, 1), (1, 0)])
def test_numpy_fp32_timing_twin_computes_the_gradient(prior, pin):
    # the float32 NumPy leg times the same computation as the oracle's gradient
    sys.path.insert(0, ROOT)
    import numpy as np
    import bench
    import oracle
    from workloads import make_problem
    prob = make_problem("c2_f32", n=500, p=60, K=6, prior=prior, pin_last_class=pin)
    B = np.random.default_rng(1).normal(0, 0.1, size=(60, 6))
    if pin:
        B[:, -1] = 0.0
    B = B.astype(np.float32)
    g = bench.numpy_fp32_grad_fn(prob, B)().astype(np.float64)
    g_o = oracle.grad_log_kernel(prob.X64, prob.y, B.astype(np.float64), prior, prob.prior_scale,
                                 pin)
    assert np.linalg.norm(g - g_o) / np.linalg.norm(g_o) < 1e-5


@pytest.mark.gpu
def test_bench_prints_one_contract_line():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--steps", "5", "--warmup", "2",
                        "--forms-iters", "0", "--no-cpu-baseline"],
                       capture_output=True, text=True, timeout=600, cwd=ROOT)
    assert r.returncode == 0, r.stderr[-2000:]
    lines = [l for l in r.stdout.splitlines() if l.strip()]
    assert len(lines) == 1
    d = json.loads(lines[0])
    for k in ("metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step",
              "higher_is_better", "scaling", "vs_baseline", "dtype", "data", "config", "roofline"):
        assert k in d, k
    assert d["n_gpus"] == 1 and d["steps"] == 5 and d["warmup"] == 2
    assert d["value"] > 0 and d["higher_is_better"] is True
    assert "workload" in d["config"]
    rr = d["replay_repeats"]["grad_evals_per_s"]
    assert d["replay_repeats"]["repeats"] == 5 and rr["min"] <= rr["median"] <= rr["max"]
    rf = d["roofline"]
    for k in ("bound", "achieved", "peak", "unit", "frac", "traffic"):
        assert k in rf, k
    assert rf["bound"] == "hbm" and rf["unit"] == "GB/s" and rf["peak"] == 8000.0
    assert abs(rf["frac"] - rf["achieved"] / rf["peak"]) < 1e-3
    print(f"[bench] {d['value']:.0f} {d['unit']}, frac {rf['frac']}", flush=True)


class _FakeSampler:
    """Stands in for the library in tune_eps: the acceptance of a probe is a fixed function
    of the step size (exactly `probe` Bernoulli outcomes at that rate)."""

    def __init__(self, rate):
        self.rate, self.calls = rate, []

    def sample(self, dp, B, G, logk, eps, L, n_iter, seed=0, first_iter=0, record_samples=False):
        import torch
        self.calls.append(eps)
        k = int(round(self.rate(eps) * n_iter))
        return {"accepted": torch.tensor([1] * k + [0] * (n_iter - k), dtype=torch.int32)}


@pytest.mark.parametrize("eps0", [0.002, 0.05])
def test_tune_eps_reaches_the_band(eps0):
    """From a step size that accepts everything or nothing, the probes bracket and bisect
    to one whose acceptance lies in [0.65, 0.75] (acceptance falling smoothly in eps)."""
    import bench

    class P:
        L = 10

    fake = _FakeSampler(lambda e: float(np.clip(1.0 - (e / 0.02) ** 2, 0.0, 1.0)))
    eps, probes = bench.tune_eps(fake, None, P, None, None, None, eps0, 1, 0)
    assert 0.65 <= probes[-1]["accept_rate"] <= 0.75
    assert probes[-1]["eps"] == eps
    assert 0.0098 < eps < 0.0119                      # where 1 - (eps / 0.02)^2 is in the band


def test_tune_eps_reopens_a_closed_bracket():
    """An early probe that rejected at a step size which accepts everything later (a chain
    that had not moved yet) must not pin the bracket: once it closes, growth resumes."""
    import bench

    class P:
        L = 10

    state = {"n": 0}

    def rate(e):
        state["n"] += 1
        if state["n"] == 1:
            return 0.0                                # the first probe, at eps0, rejects all
        return float(np.clip(1.0 - (e / 0.02) ** 2, 0.0, 1.0))

    fake = _FakeSampler(rate)
    eps, probes = bench.tune_eps(fake, None, P, None, None, None, 0.004, 1, 0, max_probes=20)
    assert 0.65 <= probes[-1]["accept_rate"] <= 0.75


def test_tune_eps_returns_a_probed_step_when_the_band_is_missed():
    """With too few probes to reach the band, the step size returned is one that was probed:
    the one whose acceptance came closest to the band's centre."""
    import bench

    class P:
        L = 10

    fake = _FakeSampler(lambda e: float(np.clip(1.0 - (e / 0.02) ** 2, 0.0, 1.0)))
    eps, probes = bench.tune_eps(fake, None, P, None, None, None, 1e-4, 1, 0, max_probes=3)
    assert not any(0.65 <= q["accept_rate"] <= 0.75 for q in probes)
    assert eps in [q["eps"] for q in probes]
    assert eps == min(probes, key=lambda q: abs(q["accept_rate"] - 0.7))["eps"]


def test_config_table_names_every_configuration():
    """The per-configuration timing leg covers every named workload, and its timer averages
    the calls after an untimed first one."""
    import bench
    from workloads.synth import _CONFIGS
    assert set(bench.CONFIG_TABLE) == set(_CONFIGS)
    calls = []
    t = bench._mean_seconds(lambda: calls.append(1), reps=5)
    assert len(calls) == 6 and t >= 0.0


def test_ess_of_a_nearly_stuck_chain_is_capped():
    """A Metropolis chain that moved once, at its last iteration, has two distinct states:
    its ESS is at most 2, although the autocorrelation estimator alone returns the full
    length; a chain that accepts every move keeps the estimator's value."""
    import bench
    from paper_1402_4089_amd import diagnostics
    T = 80
    x = np.zeros((T, 3))
    x[-1] = [0.3, -1.0, 2.0]
    acc = np.zeros(T, dtype=np.int32)
    acc[-1] = 1
    assert np.all(diagnostics.ess(x) > 70)
    assert np.all(bench.capped_ess(x, acc, diagnostics) == 2.0)
    rng = np.random.default_rng(5)
    y = rng.normal(size=(T, 4))
    full = np.ones(T, dtype=np.int32)
    assert np.allclose(bench.capped_ess(y, full, diagnostics), diagnostics.ess(y))
    still = np.zeros((T, 2))
    assert bench.capped_ess(still, np.zeros(T), diagnostics).size == 0
