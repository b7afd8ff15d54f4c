#!/usr/bin/env python
"""Throughput of GPU-resident HMC for Bayesian multinomial regression on one MI355X.

A step is one HMC iteration of the whole device path: Philox momentum draw, L leapfrog
updates (each one fused log-posterior + gradient pass over X plus its epilogue) and the
Metropolis accept, with X, labels and chain state resident in HBM before timing starts.
The default workload is the plain-FP32 problem n=20000, p=1000, K=10 (L=50, eps=0.002,
Gaussian N(0,1) prior, last class pinned) on seeded synthetic data.

Prints one JSON line. ``value`` is leapfrog gradient evaluations per second; the line also
carries effective samples per second, the fused kernel's roofline fraction (its duration
measured with HIP events on its own stream during the timed steps) and the FP64 oracle
timed on the host cores as a reported CPU baseline.
"""
from __future__ import annotations

import argparse
import dataclasses
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
BF16_PEAK_TFLOPS = 2500.0          # dense BF16 MFMA, MI355X
X_BYTES = {"f64": 8, "f32": 4, "bf16hilo": 4, "bf16": 2}
PROFILE_REPEAT = 8      # launches of the gradient pass per timing event pair
DEFAULT_STEPS = {
    "c2_f32": (500, 100), "poisson_f32": (500, 100), "probit_f32": (500, 100),
    "c3_widep": (60, 10), "c4_bf16": (16, 2), "c4_bf16hi": (16, 2), "c1_small_f64": (500, 50),
    "c0_mnist_shape": (100, 20)}
METRIC = "leapfrog grad evals/s + ESS/s, BF16/batched vs plain FP32, at stated grad error"


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_source_hash() -> str:
    """Hash of the fused kernel's source: fused.hip, the device helpers it includes and its
    argument struct (other declarations of internal.h do not change the kernel)."""
    csrc = os.path.join(ROOT, "paper_1402_4089_amd", "csrc")
    h = hashlib.sha256()
    for f in ("fused.hip", "device_common.h"):
        with open(os.path.join(csrc, f), "rb") as fh:
            h.update(fh.read())
    with open(os.path.join(csrc, "internal.h")) as fh:
        txt = fh.read()
    i = txt.index("struct FusedArgs {")
    h.update(txt[i:txt.index("};", i)].encode())
    return h.hexdigest()[:16]


def read_traffic(workload: str):
    """Per-launch HBM bytes of the fused kernel from the committed counter summary, or None
    when the summary is absent or was taken on a different kernel source."""
    path = os.path.join(ROOT, "profiles", f"fused_logpost_grad_{workload}_pmc.txt")
    if not os.path.exists(path):
        return None
    fields = {}
    with open(path) as fh:
        for line in fh:
            if ":" in line:
                k, v = line.split(":", 1)
                fields[k.strip()] = v.strip()
    if fields.get("kernel_source_sha256_16") != kernel_source_hash():
        return None
    try:
        return float(fields["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def oracle_x(prob):
    """The X values the device sees, in float64 (the split-precision sum for bf16 forms)."""
    if prob.xfmt in ("bf16hilo", "bf16"):
        from oracle import split
        hi, lo = split.split_hilo(prob.X64)
        return hi if prob.xfmt == "bf16" else hi + lo
    return prob.X64


def host_info() -> dict:
    """The host the CPU legs run on: CPU model, usable cores, and the BLAS library NumPy
    calls with its thread count."""
    model = None
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    blas = []
    try:
        from threadpoolctl import threadpool_info
        for d in threadpool_info():
            if d.get("user_api") == "blas":
                blas.append({"library": d.get("internal_api"), "version": d.get("version"),
                             "threads": d.get("num_threads"),
                             "architecture": d.get("architecture")})
    except Exception:  # threadpoolctl missing: the BLAS pool stays unreported
        pass
    return {"cpu_model": model, "cores_available": len(os.sched_getaffinity(0)), "blas": blas}


def cpu_baseline(prob, B_dev_final, G_dev_final, seconds: float):
    """Oracle leg: the FP64 NumPy oracle timed on the host cores on a bounded sample of the
    same workload (leapfrog updates from B = 0 with a Philox momentum, one gradient
    evaluation each, until `seconds` have passed), plus the device gradient's error
    against the oracle at the device's final state."""
    import oracle
    from oracle import philox
    try:
        from threadpoolctl import threadpool_info
        cores = max([d.get("num_threads", 1) for d in threadpool_info()] or [1])
    except Exception:  # threadpoolctl missing or no BLAS pool reported
        cores = len(os.sched_getaffinity(0))
    X64 = oracle_x(prob)
    link = {"poisson": oracle.POISSON, "probit": oracle.PROBIT}.get(prob.meta.get("link"),
                                                                   oracle.SOFTMAX)
    B = np.zeros((prob.p, prob.K))
    G = oracle.grad_log_kernel(X64, prob.y, B, prob.prior, prob.prior_scale, prob.pin_last_class,
                               link)
    xi, _ = philox.draws(1234, 0, 1, prob.p, prob.K)
    eta = xi[0] * oracle.free_mask(prob.p, prob.K, prob.pin_last_class)
    t0 = time.perf_counter()
    grads = 0
    with np.errstate(over="ignore", invalid="ignore"):
        while True:
            B, eta, G, lk = oracle.leapfrog_step(X64, prob.y, B, eta, G, prob.eps, prob.prior,
                                                 prob.prior_scale, prob.pin_last_class, link)
            grads += 1
            if not (np.isfinite(lk) and np.all(np.isfinite(G))):
                # an unstable stretch (no Metropolis test here): restart from B = 0
                B = np.zeros((prob.p, prob.K))
                G = oracle.grad_log_kernel(X64, prob.y, B, prob.prior, prob.prior_scale,
                                           prob.pin_last_class, link)
                grads += 1
            if grads % prob.L == 0:                       # momentum refresh, as per iteration
                eta = xi[0] * oracle.free_mask(prob.p, prob.K, prob.pin_last_class)
            if time.perf_counter() - t0 >= seconds:
                break
    dt = time.perf_counter() - t0
    # stated gradient error of the device path at its final state
    Bf = B_dev_final.astype(np.float64)
    G_o = oracle.grad_log_kernel(X64, prob.y, Bf, prob.prior, prob.prior_scale, prob.pin_last_class,
                                 link)
    rel = float(np.linalg.norm(G_dev_final - G_o) / max(np.linalg.norm(G_o), 1e-300))
    if prob.xfmt in ("bf16hilo", "bf16"):
        # the total error of the form: against the unsplit X, bfloat16 quantisation included
        G_x = oracle.grad_log_kernel(prob.X64, prob.y, Bf, prob.prior, prob.prior_scale,
                                     prob.pin_last_class, link)
        rel_x = float(np.linalg.norm(G_dev_final - G_x) / max(np.linalg.norm(G_x), 1e-300))
    else:
        rel_x = None
    base = {"value": grads / dt, "unit": "grad_evals/s", "cores": int(cores), "kind": "oracle",
            "sample": f"{grads} gradient evaluations in leapfrog updates (momentum reset every "
                      f"L = {prob.L} updates) of the same {prob.name} workload from B = 0, "
                      f"FP64 NumPy, {dt:.1f} s",
            "host": host_info()}
    return base, rel, rel_x


def numpy_fp32_grad_fn(prob, B_dev_final):
    """A float32 NumPy/BLAS gradient of the multinomial-logit log-posterior (the kind of CPU
    code Section 3.1 times against its GPU), as a closure over the workload and a state."""
    X = np.ascontiguousarray(prob.X, dtype=np.float32)
    B = np.asarray(B_dev_final, dtype=np.float32)
    Y = np.zeros((prob.n, prob.K), dtype=np.float32)
    Y[np.arange(prob.n), prob.y] = 1.0
    s2 = np.float32(prob.prior_scale ** 2)

    def grad():
        Z = X @ B
        E = np.exp(Z - Z.max(axis=1, keepdims=True))
        P = E / E.sum(axis=1, keepdims=True)
        G = X.T @ (Y - P) + (-B / s2 if prob.prior == 0 else -2.0 * B / (s2 + B * B))
        if prob.pin_last_class:
            G[:, -1] = 0.0
        return G

    return grad


def numpy_fp32_rate(prob, B_dev_final, reps: int = 5) -> dict:
    """The paper's CPU comparison in kind: one gradient evaluation of numpy_fp32_grad_fn on
    the host at the device's final state, mean of `reps` after one warm-up (the paper
    averages 5 runs). A timing leg only; it is not the oracle and checks nothing."""
    grad = numpy_fp32_grad_fn(prob, B_dev_final)
    grad()
    t0 = time.perf_counter()
    for _ in range(reps):
        grad()
    dt = (time.perf_counter() - t0) / reps
    try:
        from threadpoolctl import threadpool_info
        cores = max([d.get("num_threads", 1) for d in threadpool_info()] or [1])
    except Exception:  # threadpoolctl missing or no BLAS pool reported
        cores = len(os.sched_getaffinity(0))
    return {"value": round(1.0 / dt, 2), "unit": "grad_evals/s", "cores": int(cores),
            "kind": "numpy_fp32",
            "sample": f"one gradient evaluation of the same {prob.name} workload in float32 "
                      f"NumPy, mean of {reps} after one warm-up: {dt * 1e3:.2f} ms"}


def rows_sweep(hmc, torch, rows=(20000, 60000, 200000, 1000000), p: int = 1000, K: int = 10,
               L: int = 50, iters: int = 20) -> dict:
    """The plain-FP32 pass of the default workload's width (p = 1000, K = 10, last class
    pinned, Gaussian prior) at growing row counts: how the fixed cost of each gradient
    evaluation (first tile, partial write-out, epilogue) amortises. X and labels are drawn on
    the device (iid N(0, 1), uniform labels); eps scales as 1/sqrt(n) from the default's
    0.002 at n = 20000."""
    dev = torch.device("cuda:0")
    gen = torch.Generator(device=dev)
    gen.manual_seed(1402)
    recs = []
    for n in rows:
        X = torch.randn(n, p, device=dev, generator=gen)
        y = torch.randint(0, K, (n,), device=dev, dtype=torch.int32, generator=gen)
        dp = hmc.Problem(X, y, K, 0, 1.0, True)
        B = dp.zeros_state()
        logk, G = hmc.logpost_grad(dp, B)
        eps = 0.002 * (20000.0 / n) ** 0.5
        hmc.sample(dp, B, G, logk, eps, L, 2, seed=1, record_samples=False)
        hmc.hmc_profile_begin(4 * L, PROFILE_REPEAT)
        hmc.sample(dp, B, G, logk, eps, L, 4, seed=1, first_iter=2, record_samples=False)
        _, pass_us, _, _ = hmc.hmc_profile_end()
        plan, _ = hmc.plan(dp, B, G, logk, eps, L, iters, seed=1, first_iter=6, record_samples=False)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        plan.launch(iters)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        plan.destroy()
        alg = n * p * 4 + 4 * n + 2 * p * K * 4
        grad_us = dt / (iters * L) * 1e6
        recs.append({"n": n, "fused_pass_us": round(pass_us, 2),
                     "pass_frac_of_8tbs": round(alg / (pass_us * 1e-6) / 1e9 / HBM_PEAK_GBS, 4),
                     "grad_eval_us": round(grad_us, 2), "grad_evals_per_s": round(1e6 / grad_us, 1),
                     "step_frac_of_8tbs": round(alg / (grad_us * 1e-6) / 1e9 / HBM_PEAK_GBS, 4)})
        log(f"[bench] rows sweep n={n}: pass {pass_us:.2f} us, gradient evaluation {grad_us:.2f} us")
        del dp, X, y, B, G
        torch.cuda.empty_cache()
    return {"rows_sweep": {"p": p, "K": K, "L": L, "iters": iters, "dtype": "f32",
                           "records": recs,
                           "note": "fused_pass_us: HIP events around the gradient pass; grad_eval_us: "
                                   "graph replay of whole iterations (pass, epilogue, update, accept) "
                                   "divided by the gradient evaluations"}}


def shard_shares(hmc, torch, gpus: int, iters: int = 10) -> dict:
    """One GPU's share of each configuration sharded over `gpus` GPUs, measured on this one
    GPU (no collective runs: this build drives one GPU). Rows shard for the plain-FP32 and
    split-precision workloads (n / gpus rows each), columns for the high-dimensional one
    (p / gpus columns each, all n rows). Each share runs its configuration's L and step size
    as graph replays of whole iterations; reported per gradient evaluation, with the payload
    of the one all-reduce per leapfrog update the sharded form would add (the partial
    gradient and log-likelihood for rows, the partial logits and kinetic energy for columns,
    FP32 plus one FP64 scalar)."""
    from workloads import make_problem
    dev = torch.device("cuda:0")
    recs = []
    for name, axis in (("c2_f32", "rows"), ("c4_bf16", "rows"), ("c3_widep", "columns")):
        cfg_n, cfg_p = {"c2_f32": (20000, 1000), "c4_bf16": (200000, 4096),
                        "c3_widep": (2000, 50000)}[name]
        n, p = (cfg_n // gpus, cfg_p) if axis == "rows" else (cfg_n, cfg_p // gpus)
        prob = make_problem(name, n=n, p=p)
        y = torch.from_numpy(prob.y).to(dev)
        if prob.xfmt == "bf16hilo":
            X64 = torch.from_numpy(prob.X64).to(dev)
            hi, lo = hmc.split_bf16(X64)
            del X64
            dp = hmc.Problem(hi, y, prob.K, prob.prior, prob.prior_scale, True, X_lo=lo)
            xbytes = 4
        else:
            X = torch.from_numpy(np.asarray(prob.X)).to(dev)
            dp = hmc.Problem(X, y, prob.K, prob.prior, prob.prior_scale, bool(prob.pin_last_class))
            xbytes = X.element_size()
        B = dp.zeros_state()
        logk, G = hmc.logpost_grad(dp, B)
        hmc.sample(dp, B, G, logk, prob.eps, prob.L, 1, seed=1, record_samples=False)
        plan, _ = hmc.plan(dp, B, G, logk, prob.eps, prob.L, iters, seed=1, first_iter=1,
                           record_samples=False)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        plan.launch(iters)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        plan.destroy()
        k_eff = prob.K - 1 if prob.pin_last_class else prob.K
        us = dt / (iters * prob.L) * 1e6
        alg = prob.n * prob.p * xbytes + 4 * prob.n + 2 * prob.p * prob.K * 4
        payload = (prob.p * k_eff if axis == "rows" else prob.n * k_eff) * 4 + 8
        recs.append({"workload": name, "split": axis, "n": prob.n, "p": prob.p, "K": prob.K,
                     "L": prob.L, "grad_eval_us": round(us, 2),
                     "frac_of_8tbs": round(alg / (us * 1e-6) / 1e9 / HBM_PEAK_GBS, 4),
                     "allreduce_bytes_per_update": payload})
        log(f"[bench] share of {name} over {gpus} GPUs ({axis}): n={prob.n} p={prob.p}, "
            f"{us:.2f} us per gradient evaluation")
        del dp, B, G, y
        torch.cuda.empty_cache()
    return {"shards": {"gpus": gpus, "records": recs,
                       "note": "one GPU's share, measured alone; the all-reduce is not run"}}


def read_stream_gbs(hmc, torch, nbytes: int) -> float:
    """Measured read bandwidth of this GPU for a buffer of the given size: the library's
    streaming-read kernel (every byte read once per pass, 16-byte loads), 10 timed passes
    between HIP events on the current stream."""
    nbytes = max(nbytes // 16 * 16, 1 << 24)
    x = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda:0")
    sink = torch.zeros(2048, dtype=torch.int32, device="cuda:0")
    stream = torch.cuda.current_stream()
    hmc.hmc_stream_read(x, nbytes, 2, sink, stream)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    hmc.hmc_stream_read(x, nbytes, 10, sink, stream)
    e1.record()
    e1.synchronize()
    gbs = nbytes * 10 / (e0.elapsed_time(e1) * 1e-3) / 1e9
    del x
    torch.cuda.empty_cache()
    return gbs


def cold_warm_pass_us(hmc, torch, dp, B, passes: int = 20):
    """Gradient-pass time with X evicted from the 256 MB memory-side cache before every pass
    (a streaming read of 640 MB in between) and without, one launch per event pair in both,
    so the two figures share the cost of recording the events."""
    flush = torch.ones(160 << 20, dtype=torch.float32, device="cuda:0")
    stream = torch.cuda.current_stream()
    out = {}
    for key, evict in (("warm_us", False), ("cold_us", True)):
        hmc.hmc_profile_begin(passes, 1)
        for _ in range(passes):
            if evict:
                hmc.hmc_stream_read(flush, flush.numel() * 4, 1, None, stream)
            hmc.logpost_grad(dp, B)
        out[key] = round(hmc.hmc_profile_end()[1], 3)
    del flush
    torch.cuda.empty_cache()
    return out


TABLE1_N = (100, 1000, 5000, 10000)
TABLE1_K = (2, 3, 4, 5, 10, 15, 20)
TABLE1_P = (10, 50, 100, 500, 1000, 5000, 10000, 20000)


def table1_sweep(hmc, torch, reps: int = 5, quick: bool = False, log_progress: bool = True):
    """The timing sweep of Section 3.1 (Table 1, Figures 1-4): for every (N, K, p) of Table 1,
    pinned and unpinned, one gradient evaluation and one leapfrog update, each the mean of
    `reps` runs, on the device (FP32) and with the FP64 oracle on the host cores. X and B are
    iid N(0, 1e-3) (variance), y ~ Categorical(softmax(X B)). Reports the oracle/device time
    ratios (the paper's CPU/GPU ratio) and the device gradient's rel-L2 error against the
    oracle for every combination."""
    import oracle
    from workloads.synth import gumbel_max_labels
    Ns = TABLE1_N[:2] if quick else TABLE1_N
    Ps = TABLE1_P[:5] if quick else TABLE1_P
    dev = torch.device("cuda:0")
    recs = []
    t_start = time.perf_counter()
    for n in Ns:
        for p in Ps:
            for K in TABLE1_K:
                rng = np.random.default_rng([31, n, p, K])
                X = rng.normal(0.0, np.sqrt(1e-3), size=(n, p)).astype(np.float32)
                B = rng.normal(0.0, np.sqrt(1e-3), size=(p, K)).astype(np.float32)
                y = gumbel_max_labels(rng, X.astype(np.float64), B.astype(np.float64))
                X64 = X.astype(np.float64)
                Xd = torch.from_numpy(X).to(dev)
                yd = torch.from_numpy(y).to(dev)
                for pin in (1, 0):
                    dp = hmc.Problem(Xd, yd, K, hmc.HMC_PRIOR_GAUSS, 1.0, bool(pin))
                    # pinned: the model's last coefficient column is zero (beta_K = 0)
                    Bm = B.copy()
                    if pin:
                        Bm[:, -1] = 0.0
                    B64 = Bm.astype(np.float64)
                    Bd = torch.from_numpy(Bm).to(dev)
                    logk, G = hmc.logpost_grad(dp, Bd)            # warm-up
                    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                    e0.record()
                    for _ in range(reps):                          # preallocated outputs
                        hmc.hmc_logpost_grad(dp.desc, Bd, logk, G, dp.ws, None)
                    e1.record()
                    e1.synchronize()
                    g_us = e0.elapsed_time(e1) * 1e3 / reps
                    G_d = G.double().cpu().numpy()
                    eta = torch.from_numpy(rng.normal(size=(p, K)).astype(np.float32)).to(dev)
                    hmc.leapfrog(dp, Bd, eta, G, logk, 1e-3, 1)       # warm-up
                    e0.record()
                    for _ in range(reps):
                        hmc.leapfrog(dp, Bd, eta, G, logk, 1e-3, 1)
                    e1.record()
                    e1.synchronize()
                    l_us = e0.elapsed_time(e1) * 1e3 / reps
                    # oracle: the same operations in FP64 NumPy on the host (one untimed call
                    # first, as on the device)
                    oracle.grad_log_kernel(X64, y, B64, oracle.GAUSS, 1.0, pin)
                    t0 = time.perf_counter()
                    for _ in range(reps):
                        G_o = oracle.grad_log_kernel(X64, y, B64, oracle.GAUSS, 1.0, pin)
                    og = (time.perf_counter() - t0) / reps
                    eta_o = np.zeros((p, K))
                    t0 = time.perf_counter()
                    for _ in range(reps):
                        oracle.leapfrog_step(X64, y, B64, eta_o, G_o, 1e-3, oracle.GAUSS, 1.0, pin)
                    ol = (time.perf_counter() - t0) / reps
                    err = float(np.linalg.norm(G_d - G_o) / max(np.linalg.norm(G_o), 1e-300))
                    recs.append({"N": n, "K": K, "p": p, "pinned": pin,
                                 "device_grad_us": round(g_us, 2), "device_leapfrog_us": round(l_us, 2),
                                 "oracle_grad_ms": round(og * 1e3, 3), "oracle_leapfrog_ms": round(ol * 1e3, 3),
                                 "ratio_grad": round(og * 1e6 / g_us, 1),
                                 "ratio_leapfrog": round(ol * 1e6 / l_us, 1), "grad_rel_l2": err})
                    del dp, Bd, G, logk, eta
                del Xd, yd
            if log_progress:
                log(f"[table1] N={n} p={p} done ({len(recs)} records, {time.perf_counter() - t_start:.0f} s)")
    torch.cuda.empty_cache()
    summary = {}
    for n in Ns:
        rg = [r["ratio_grad"] for r in recs if r["N"] == n]
        rl = [r["ratio_leapfrog"] for r in recs if r["N"] == n]
        summary[str(n)] = {"ratio_grad_min": min(rg), "ratio_grad_median": float(np.median(rg)),
                           "ratio_grad_max": max(rg), "ratio_leapfrog_min": min(rl),
                           "ratio_leapfrog_median": float(np.median(rl)), "ratio_leapfrog_max": max(rl),
                           "device_slower": int(sum(1 for v in rg + rl if v < 1.0))}
    try:
        from threadpoolctl import threadpool_info
        cores = max([d.get("num_threads", 1) for d in threadpool_info()] or [1])
    except Exception:  # threadpoolctl missing or no BLAS pool reported
        cores = len(os.sched_getaffinity(0))
    return {"table1": {"combinations": len(recs), "reps": reps, "oracle": "FP64 NumPy",
                       "oracle_cores": cores, "device": "FP32 path of this library, one MI355X",
                       "max_grad_rel_l2": max(r["grad_rel_l2"] for r in recs),
                       "by_N": summary, "records": recs,
                       "paper": "Section 3.1: FP32 NumPy on 2x Xeon E5-2670 vs PyCuda on a Tesla "
                                "K20; the GPU 50-100x faster for large problems, slower only for "
                                "some N = 100 cases"}}


def mnist_protocol(hmc, torch, seed: int = 20140217):
    """The sampling protocol of Section 3.2 on the MNIST-shaped stand-in (the dataset itself is
    absent): 70,000 rows of 784 U(0, 1) "pixels" plus an intercept, K = 10, labels drawn from a
    softmax model; the first 60,000 rows fit the model, the last 10,000 are held out. HMC with
    L = 100: 100 burn-in iterations at eps = 1e-4 with the annealed acceptance (T0 = 1e3,
    r = 0.9), then 100 sampling iterations at eps = 7e-5; Cauchy(0, 1) prior, last class pinned.
    Reports the device wall time of the run, the sampling-phase acceptance rate, and the held-out
    accuracy of the posterior-predictive class (highest mean softmax over the samples), beside
    the accuracy of the generating coefficients on the same rows (synthetic labels: a sanity
    check of the sampler, not a measure of MNIST accuracy)."""
    from workloads import make_problem
    prob = make_problem("c0_mnist_shape", n=70000)
    n_fit = 60000
    X = np.ascontiguousarray(prob.X[:n_fit])
    yt = prob.y[n_fit:]
    dev = torch.device("cuda:0")
    dp = hmc.Problem(torch.from_numpy(X).to(dev), torch.from_numpy(prob.y[:n_fit].copy()).to(dev),
                     prob.K, prob.prior, prob.prior_scale, bool(prob.pin_last_class))
    B = dp.zeros_state()
    logk, G = hmc.logpost_grad(dp, B)
    temps = torch.from_numpy(annealed_inv_temps(100)).to(dev)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    burn = hmc.sample(dp, B, G, logk, 1e-4, 100, 100, seed=seed, record_samples=False,
                      inv_temperature=temps)
    out = hmc.sample(dp, B, G, logk, 7e-5, 100, 100, seed=seed, first_iter=100,
                     record_samples=True)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    # posterior-predictive class of the held-out rows on the device (hmc_posterior_predictive:
    # float64 mean of the softmax over the 100 samples, then its argmax)
    Xt_dev = torch.from_numpy(np.ascontiguousarray(prob.X[n_fit:])).to(dev)
    t1 = time.perf_counter()
    _, cls = hmc.posterior_predictive(Xt_dev, out["samples"], prob.K, True)
    torch.cuda.synchronize()
    pred_s = time.perf_counter() - t1
    acc_post = float(np.mean(cls.cpu().numpy() == yt))
    Bt = prob.B_true - prob.B_true[:, -1:]                    # same classifier, last class pinned
    _, cls_t = hmc.posterior_predictive(Xt_dev, torch.from_numpy(Bt[None].astype(np.float32)).to(dev),
                                        prob.K, True)
    acc_true = float(np.mean(cls_t.cpu().numpy() == yt))
    return {"mnist_protocol": {
        "workload": "MNIST-shaped stand-in: n = 60,000 (+10,000 held out), p = 785 (784 U(0,1) + intercept), K = 10, Cauchy(0,1) prior",
        "iterations": {"burn_in": 100, "sampling": 100, "L": 100, "eps": [1e-4, 7e-5],
                       "annealing": {"T0": 1e3, "r": 0.9}},
        "gradient_evaluations": 20000,
        "device_seconds": round(wall, 3),
        "grad_evals_per_s": round(20000 / wall, 1),
        "accept_rate_burn_in": round(float(burn["accepted"].float().mean()), 3),
        "accept_rate_sampling": round(float(out["accepted"].float().mean()), 3),
        "divergent": int(out["divergent"].sum()) + int(burn["divergent"].sum()),
        "heldout_accuracy_posterior_predictive": round(acc_post, 4),
        "prediction_device_seconds": round(pred_s, 4),
        "heldout_accuracy_generating_coefficients": round(acc_true, 4),
        "paper": "Section 3.2, Table 2: 3 min 54 s (234 s) for this protocol on MNIST, presumably "
                 "on the Tesla K20 of Section 3.1 (other hardware and real data: context only)"}}


def annealed_inv_temps(n: int, T0: float = 1e3, r: float = 0.9) -> np.ndarray:
    """1/T_t for warm-up iteration t: T_t = max(1, T0 r^t) (the annealed burn-in of
    Section 3.2: proposals far from the mode are accepted while T is large)."""
    return 1.0 / np.maximum(1.0, T0 * r ** np.arange(n))


def _pooled_mean_mcse(chains_trace: np.ndarray):
    """Pooled posterior mean over M chains (M x T x d) and its Monte-Carlo standard error
    from within-chain ESS (Geyer): MCSE^2 = sum_c s_c^2 / ESS_c / M^2. A coordinate on
    which some chain never moved has no ESS estimate: its MCSE is NaN (not comparable)."""
    from paper_1402_4089_amd import diagnostics
    M = chains_trace.shape[0]
    means = chains_trace.mean(axis=1)
    var = np.zeros(chains_trace.shape[2])
    for c in range(M):
        e = diagnostics.ess(chains_trace[c])
        s2 = chains_trace[c].var(axis=0, ddof=1)
        var += np.where(np.isfinite(e) & (e > 0) & (s2 > 0), s2 / np.where(e > 0, e, 1.0), np.nan)
    return means.mean(axis=0), np.sqrt(var) / M


def _z_summary(m1, se1, m2, se2):
    se = np.sqrt(se1 ** 2 + se2 ** 2)
    ok = np.isfinite(se) & (se > 0)
    z = np.abs(m1 - m2)[ok] / se[ok]
    return {"coords": int(z.size), "coords_without_mcse": int((~ok).sum()),
            "frac_beyond_3_mcse": round(float(np.mean(z > 3)), 5),
            "median_z": round(float(np.median(z)), 4), "max_z": round(float(z.max()), 3)}


def forms_accuracy(hmc, torch, probs, fp32, bf, seed: int, problems=(37, 14), chains: int = 4,
                   burn: int = 100, kept: int = 200, oracle_chains: int = 2, bf_hi=None) -> dict:
    """Matched posterior-mean accuracy of the two forms on batch problems whose chains mix
    well at the configured step size (the smallest, with p much below n): each form runs
    `chains` chains of every listed problem from B = 0 for `burn` + `kept` iterations on its
    own Philox stream (batched bf16: seed + 10, through the batched kernels on a batch of
    these problems; plain FP32: seed + 11), and the FP64 oracle runs `oracle_chains` chains
    of each (seed + 12). Per free coordinate, the pooled posterior means of two samplers are
    compared within 3 sqrt(MCSE_1^2 + MCSE_2^2), each MCSE from within-chain ESS (Geyer) of
    the kept iterations; independent correct samplers exceed that on about 0.3% of
    coordinates (more when the ESS estimate of short chains runs high)."""
    import oracle
    from oracle import philox
    L = 20
    free = {b: np.arange(probs[b].K) != probs[b].K - 1 for b in problems}
    eps = [probs[b].eps for b in problems]

    def batched_chains(forms, stream):
        # a batched form on a batch of just these problems
        sub = hmc.Batch([forms[b] for b in problems], chains)
        B, G, logk = sub.zeros_state()
        sub.logpost_grad(B, G, logk)
        plan, _ = sub.plan(B, G, logk, eps, L, burn, seed=stream, records=False)
        plan.launch(burn)
        plan.destroy()
        plan, rec = sub.plan(B, G, logk, eps, L, kept, seed=stream, first_iter=burn, record_samples=True)
        plan.launch(kept)
        torch.cuda.synchronize()
        plan.destroy()
        tr = {b: rec["samples"][i].double().cpu().numpy()[:, :, :, free[b]].reshape(kept, chains, -1)
              .transpose(1, 0, 2) for i, b in enumerate(problems)}
        return tr, float(rec["accepted"].float().mean())

    tr_b, acc_b = batched_chains(bf, seed + 10)
    tr_h, acc_h = batched_chains(bf_hi, seed + 13) if bf_hi is not None else (None, None)
    # plain FP32 form, chain by chain
    tr_p, acc_p = {}, []
    for b in problems:
        pr, per = probs[b], []
        for c in range(chains):
            Bc = fp32[b].zeros_state()
            lk, Gc = hmc.logpost_grad(fp32[b], Bc)
            pl, out = hmc.plan(fp32[b], Bc, Gc, lk, pr.eps, L, burn + kept, seed=seed + 11,
                               chain=b * chains + c, record_samples=True)
            pl.launch(burn + kept)
            torch.cuda.synchronize()
            pl.destroy()
            per.append(out["samples"].double().cpu().numpy()[burn:][:, :, free[b]].reshape(kept, -1))
            acc_p.append(float(out["accepted"][burn:].float().mean()))
        tr_p[b] = np.stack(per)
    # FP64 oracle chains
    t0 = time.perf_counter()
    tr_o, acc_o = {}, []
    for b in problems:
        pr, per = probs[b], []
        for c in range(oracle_chains):
            xis, us = philox.draws(seed + 12, b * chains + c, burn + kept, pr.p, pr.K)
            r = oracle.sample(pr.X64, pr.y, pr.K, xis, us, pr.eps, L, pr.prior, pr.prior_scale, 1)
            per.append(r["samples"][burn:][:, :, free[b]].reshape(kept, -1))
            acc_o.append(float(r["accepted"][burn:].mean()))
        tr_o[b] = np.stack(per)
    t_orc = time.perf_counter() - t0
    stat = {name: [_pooled_mean_mcse(tr[b]) for b in problems]
            for name, tr in (("b", tr_b), ("p", tr_p), ("o", tr_o), ("h", tr_h)) if tr is not None}

    def z(u, v):
        return _z_summary(np.concatenate([m for m, _ in stat[u]]), np.concatenate([s for _, s in stat[u]]),
                          np.concatenate([m for m, _ in stat[v]]), np.concatenate([s for _, s in stat[v]]))
    out = {"problems": [{"index": b, "n": probs[b].n, "p": probs[b].p, "K": probs[b].K,
                         "eps": round(probs[b].eps, 6)} for b in problems],
           "iterations": {"burn_in": burn, "kept": kept, "L": L,
                          "chains": {"batched_bf16": chains, "plain_fp32": chains, "oracle_fp64": oracle_chains}},
           "accept_rate": {"batched_bf16": round(acc_b, 4), "plain_fp32": round(float(np.mean(acc_p)), 4),
                           "oracle_fp64": round(float(np.mean(acc_o)), 4)},
           "batched_vs_plain": z("b", "p"), "batched_vs_oracle": z("b", "o"),
           "plain_vs_oracle": z("p", "o"), "oracle_seconds": round(t_orc, 1),
           "rule": "per free coordinate, pooled means within 3 sqrt(MCSE_1^2 + MCSE_2^2), MCSE from "
                   "within-chain ESS of the kept iterations; independent Philox streams per sampler"}
    if tr_h is not None:
        out["accept_rate"]["batched_bf16_hi_only"] = round(acc_h, 4)
        out["hi_only_vs_oracle"] = z("h", "o")
        out["hi_only_vs_plain"] = z("h", "p")
    return out


def _mean_seconds(fn, reps: int = 5) -> float:
    """Mean wall time of `reps` calls of fn after one untimed call (the paper's average of 5)."""
    fn()
    t0 = time.perf_counter()
    for _ in range(reps):
        fn()
    return (time.perf_counter() - t0) / reps


def _device_problem(hmc, torch, prob, tuning="auto"):
    """The device problem of a workload as the benchmark builds it (bf16 planes split on the
    device for the precision form)."""
    dev = torch.device("cuda:0")
    y = torch.from_numpy(prob.y).to(dev)
    if prob.xfmt in ("bf16hilo", "bf16"):
        X64 = torch.from_numpy(prob.X64).to(dev)
        hi, lo = hmc.split_bf16(X64, hi_only=prob.xfmt == "bf16")
        torch.cuda.synchronize()
        del X64
        torch.cuda.empty_cache()
        return hmc.Problem(hi, y, prob.K, prob.prior, prob.prior_scale, bool(prob.pin_last_class),
                           X_lo=lo, tuning=tuning)
    X = torch.from_numpy(np.asarray(prob.X)).to(dev)
    return hmc.Problem(X, y, prob.K, prob.prior, prob.prior_scale, bool(prob.pin_last_class),
                       tuning=tuning)


CONFIG_TABLE = ("c1_small_f64", "c2_f32", "c3_widep", "c4_bf16", "c0_mnist_shape")


def config_timings(hmc, torch, cpu_full_max_s: float = 30.0) -> dict:
    """Every configuration, device against host, in the paper's terms (Section 3.1: one
    gradient evaluation and one leapfrog update, mean of 5 after one warm-up) and as a full
    sampling run (the configuration's iterations x L gradient evaluations).

    Device: single calls of the gradient and of one leapfrog update timed on the host clock
    with a synchronisation after each (launch latency included, as a caller sees it), and the
    full run as replays of one captured iteration (Philox momenta, from B = 0). Host: the FP64
    oracle (and, for the plain-FP32 configurations, a float32 NumPy gradient) on the host's
    cores; its full run is measured where it takes at most `cpu_full_max_s` seconds and
    otherwise extrapolated from the leapfrog update's time (marked). The batched workload
    (64 problems x 4 chains) times one oracle gradient per problem, times 4 chains."""
    import oracle
    from workloads import make_batched, make_draws, make_problem, make_random_state
    recs = []
    for name in CONFIG_TABLE:
        prob = make_problem(name)
        grads_full = prob.n_iter * prob.L
        dp = _device_problem(hmc, torch, prob)
        B = dp.zeros_state()
        logk, G = hmc.logpost_grad(dp, B)
        eta = torch.randn(B.shape, dtype=B.dtype, device=B.device) * 0.01

        def dev_grad():
            hmc.logpost_grad(dp, B)
            torch.cuda.synchronize()

        def dev_step():
            hmc.leapfrog(dp, B, eta, G, logk, prob.eps, 1)
            torch.cuda.synchronize()

        d_grad = _mean_seconds(dev_grad)
        B.zero_()
        logk, G = hmc.logpost_grad(dp, B)
        d_step = _mean_seconds(dev_step)
        B.zero_()
        logk, G = hmc.logpost_grad(dp, B)
        plan, _ = hmc.plan(dp, B, G, logk, prob.eps, prob.L, 2, seed=1, record_samples=False)
        plan.launch(2)
        torch.cuda.synchronize()
        plan.destroy()
        plan, out = hmc.plan(dp, B, G, logk, prob.eps, prob.L, prob.n_iter, seed=1, first_iter=2,
                             record_samples=False)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        plan.launch(prob.n_iter)
        torch.cuda.synchronize()
        d_full = time.perf_counter() - t0
        plan.destroy()
        acc = float(out["accepted"].float().mean())
        del dp, B, G, eta
        torch.cuda.empty_cache()

        # the oracle's cost does not depend on the values: the precision form is timed on
        # the unsplit X (its X_eff = hi + lo would cost two more copies of X to form)
        X64 = prob.X64 if prob.xfmt in ("bf16hilo", "bf16") else oracle_x(prob)
        Bh = make_random_state(prob, 0.01)
        Gh = oracle.grad_log_kernel(X64, prob.y, Bh, prob.prior, prob.prior_scale, prob.pin_last_class)
        eh = np.random.default_rng(3).normal(size=Bh.shape) * oracle.free_mask(prob.p, prob.K, prob.pin_last_class)
        with np.errstate(over="ignore", invalid="ignore"):
            c_grad = _mean_seconds(lambda: oracle.log_kernel_and_grad(
                X64, prob.y, Bh, prob.prior, prob.prior_scale, prob.pin_last_class))
            c_step = _mean_seconds(lambda: oracle.leapfrog_step(
                X64, prob.y, Bh, eh, Gh, prob.eps, prob.prior, prob.prior_scale, prob.pin_last_class))
        rec = {"config": name, "n": prob.n, "p": prob.p, "K": prob.K, "xfmt": prob.xfmt, "L": prob.L,
               "iterations": prob.n_iter,
               "device": {"grad_ms": round(d_grad * 1e3, 4), "leapfrog_ms": round(d_step * 1e3, 4),
                          "full_run_s": round(d_full, 3), "full_run_grad_us": round(d_full / grads_full * 1e6, 2),
                          "accept_rate": round(acc, 4)},
               "oracle_fp64": {"grad_ms": round(c_grad * 1e3, 3), "leapfrog_ms": round(c_step * 1e3, 3)}}
        if c_step * grads_full <= cpu_full_max_s:
            d = make_draws(prob.p, prob.K, prob.n_iter, seed=(9, 0, 0))
            t0 = time.perf_counter()
            with np.errstate(over="ignore", invalid="ignore"):
                oracle.sample(X64, prob.y, prob.K, d.xi, d.u, prob.eps, prob.L, prob.prior,
                              prob.prior_scale, prob.pin_last_class)
            rec["oracle_fp64"]["full_run_s"] = round(time.perf_counter() - t0, 2)
            rec["oracle_fp64"]["full_run"] = "measured"
        else:
            rec["oracle_fp64"]["full_run_s"] = round(c_step * grads_full, 1)
            rec["oracle_fp64"]["full_run"] = "extrapolated"
        rec["grad_ratio_oracle_over_device"] = round(c_grad / d_grad, 1)
        rec["leapfrog_ratio_oracle_over_device"] = round(c_step / d_step, 1)
        rec["full_run_ratio_oracle_over_device"] = round(rec["oracle_fp64"]["full_run_s"] / d_full, 1)
        if prob.xfmt == "f32":
            rec["numpy_fp32"] = {"grad_ms": round(1e3 / numpy_fp32_rate(prob, Bh)["value"], 3)}
        log(f"[bench] configs {name}: device grad {d_grad * 1e3:.3f} ms, leapfrog {d_step * 1e3:.3f} ms, "
            f"full run {d_full:.2f} s; oracle grad {c_grad * 1e3:.1f} ms, leapfrog {c_step * 1e3:.1f} ms, "
            f"full run {rec['oracle_fp64']['full_run_s']} s ({rec['oracle_fp64']['full_run']})")
        recs.append(rec)
        del X64, prob
    # the batched workload: all 256 chains per launch on the device; the oracle runs a chain
    # at a time
    probs = make_batched(64)
    chains, L, iters = 4, 20, probs[0].n_iter
    dev = torch.device("cuda:0")
    bf = []
    for pr in probs:
        X = torch.from_numpy(pr.X).to(dev)
        hi, lo = hmc.split_bf16(X)
        del X
        bf.append(hmc.Problem(hi, torch.from_numpy(pr.y).to(dev), pr.K, pr.prior, pr.prior_scale,
                              True, X_lo=lo))
    bt = hmc.Batch(bf, chains)
    B, G, logk = bt.zeros_state()
    bt.autotune(B, G, logk)
    bt.logpost_grad(B, G, logk)
    eps = [pr.eps for pr in probs]

    def bgrad():
        bt.logpost_grad(B, G, logk)
        torch.cuda.synchronize()

    d_grad = _mean_seconds(bgrad)
    plan, _ = bt.plan(B, G, logk, eps, L, 2, seed=1, records=False)
    plan.launch(2)
    torch.cuda.synchronize()
    plan.destroy()
    plan, rec_b = bt.plan(B, G, logk, eps, L, iters, seed=1, first_iter=2)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    plan.launch(iters)
    torch.cuda.synchronize()
    d_full = time.perf_counter() - t0
    plan.destroy()
    acc = float(rec_b["accepted"].float().mean())
    del bt, bf, B, G, logk
    torch.cuda.empty_cache()
    c_grad = 0.0
    with np.errstate(over="ignore", invalid="ignore"):
        for b, pr in enumerate(probs):
            X64 = np.asarray(pr.X, dtype=np.float64)
            Bh = make_random_state(pr, 0.01)
            if b == 0:
                oracle.log_kernel_and_grad(X64, pr.y, Bh, pr.prior, pr.prior_scale, 1)
            t0 = time.perf_counter()
            oracle.log_kernel_and_grad(X64, pr.y, Bh, pr.prior, pr.prior_scale, 1)
            c_grad += (time.perf_counter() - t0) * chains
            del X64
    grads_full = iters * L
    recs.append({"config": "batched_64x4", "problems": len(probs), "chains": chains, "L": L,
                 "iterations": iters, "xfmt": "bf16hilo",
                 "device": {"grad_ms": round(d_grad * 1e3, 3), "full_run_s": round(d_full, 2),
                            "full_run_grad_us": round(d_full / grads_full * 1e6, 1),
                            "accept_rate": round(acc, 4)},
                 "oracle_fp64": {"grad_ms": round(c_grad * 1e3, 1),
                                 "grad_sample": "one gradient per problem (X in float64), x 4 chains",
                                 "full_run_s": round(c_grad * grads_full, 1), "full_run": "extrapolated"},
                 "grad_ratio_oracle_over_device": round(c_grad / d_grad, 1),
                 "full_run_ratio_oracle_over_device": round(c_grad * grads_full / d_full, 1)})
    log(f"[bench] configs batched: device batched gradient {d_grad * 1e3:.2f} ms, full run {d_full:.2f} s; "
        f"oracle {c_grad * 1e3:.0f} ms per batched gradient")
    return {"config_timings": recs, "host": host_info(),
            "note": "device single calls: host clock with a synchronisation after each call; device full "
                    "run: graph replay of the configuration's iterations from B = 0; oracle: FP64 NumPy "
                    "on the host cores, mean of 5 after one warm-up"}


def _time_batch(hmc, torch, problems, chains, eps, L, burn, iters, seed, check):
    """One batched form on the forms workload: autotuned work split, `burn` untimed and
    `iters` timed iterations from B = 0 as replays of one captured iteration, then the kernel
    time of its gradient pass (HIP events around each pass of a short eager run)."""
    bt = hmc.Batch(problems, chains)
    B, G, logk = bt.zeros_state()
    rows, grid = bt.autotune(B, G, logk)
    bt.logpost_grad(B, G, logk)
    plan, _ = bt.plan(B, G, logk, eps, L, burn, seed=seed, records=False)
    plan.launch(burn)
    torch.cuda.synchronize()
    plan.destroy()
    plan, rec = bt.plan(B, G, logk, eps, L, iters, seed=seed, first_iter=burn)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    plan.launch(iters)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    plan.destroy()
    acc = float(rec["accepted"].float().mean())
    final = {b: (B[b][0].double().cpu().numpy(), G[b][0].double().cpu().numpy()) for b in check}
    Bx = [b.clone() for b in B]
    Gx = [g.clone() for g in G]
    hmc.hmc_profile_begin(2 * L, PROFILE_REPEAT)
    bt.sample(Bx, Gx, logk.clone(), eps, L, 2, seed=seed, first_iter=burn + iters, records=False)
    _, pass_us, _, _ = hmc.hmc_profile_end()
    del Bx, Gx, bt, B, G, logk
    torch.cuda.empty_cache()
    return {"dt": dt, "acc": acc, "rows": rows, "grid": grid, "final": final, "pass_us": pass_us}


def forms_comparison(hmc, torch, iters: int, seed: int, burn: int = 5, accuracy: bool = True):
    """BF16 hi/lo + batched vs plain FP32 on the batched workload: 64 problems with
    n ~ U[1k,50k], p ~ U[64,2048], K ~ U[2,16] (FP32 X), 4 chains each, L = 20.

    Throughput: the batched form runs all 256 chains per launch (chains of a problem share
    each pass over X) as a replayed graph of one iteration, with the autotuned work split;
    the plain form runs the same chains one problem and chain at a time through the FP32
    path, each as a replayed graph of its own iteration. Both start at B = 0, take `burn`
    untimed iterations and then `iters` timed ones, on independent Philox streams. Accuracy
    (forms_accuracy): long converged chains of both forms and the FP64 oracle on small
    problems of the batch, compared within 3 MCSE. Each form's gradient error is measured
    against the FP64 oracle at its final state. A third form runs the batch on the hi planes
    alone (X rounded to bfloat16, 2 bytes per element) through the same batched kernels."""
    import oracle
    from workloads import make_batched
    probs = make_batched(64)
    chains, L = 4, 20
    dev = torch.device("cuda:0")
    fp32, bf, bf_hi = [], [], []
    for pr in probs:
        X = torch.from_numpy(pr.X).to(dev)
        y = torch.from_numpy(pr.y).to(dev)
        fp32.append(hmc.Problem(X, y, pr.K, pr.prior, pr.prior_scale, True))
        hi, lo = hmc.split_bf16(X)
        bf.append(hmc.Problem(hi, y, pr.K, pr.prior, pr.prior_scale, True, X_lo=lo))
        bf_hi.append(hmc.Problem(hi, y, pr.K, pr.prior, pr.prior_scale, True))   # same hi plane
    torch.cuda.synchronize()
    eps = [pr.eps for pr in probs]
    elems = sum(pr.n * pr.p for pr in probs)
    check = (37, 14)                        # small problems whose gradients are checked
    log(f"[bench] forms: 64 problems, {elems / 1e9:.2f} G elements of X, 4 chains each, L={L}, "
        f"{burn} untimed + {iters} timed iterations")

    run_b = _time_batch(hmc, torch, bf, chains, eps, L, burn, iters, seed, check)
    log(f"[bench] batched bf16: {iters} iterations in {run_b['dt']:.3f} s (tuning rows="
        f"{run_b['rows']} grid={run_b['grid']}), pass {run_b['pass_us']:.1f} us")
    # the same batch on the hi planes alone (bf16 X, 2 bytes per element: the data the
    # sampler sees is X rounded to bfloat16), on its own Philox stream
    run_h = _time_batch(hmc, torch, bf_hi, chains, eps, L, burn, iters, seed + 2, check)
    log(f"[bench] batched bf16 hi only: {iters} iterations in {run_h['dt']:.3f} s (tuning rows="
        f"{run_h['rows']} grid={run_h['grid']}), pass {run_h['pass_us']:.1f} us")
    dt_b, acc_b, final_b = run_b["dt"], run_b["acc"], run_b["final"]

    t_plain = 0.0
    acc_p = []
    final_p = {}
    for b, pr in enumerate(probs):
        for c in range(chains):
            Bc = fp32[b].zeros_state()
            lk, Gc = hmc.logpost_grad(fp32[b], Bc)
            pl, _ = hmc.plan(fp32[b], Bc, Gc, lk, pr.eps, L, burn, seed=seed + 1, chain=b * chains + c,
                             record_samples=False)
            pl.launch(burn)
            pl.destroy()
            pl, out = hmc.plan(fp32[b], Bc, Gc, lk, pr.eps, L, iters, seed=seed + 1,
                               chain=b * chains + c, first_iter=burn, record_samples=False)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            pl.launch(iters)
            torch.cuda.synchronize()
            t_plain += time.perf_counter() - t0
            pl.destroy()
            acc_p.append(float(out["accepted"].float().mean()))
            if b in check and c == 0:
                final_p[b] = (Bc.double().cpu().numpy(), Gc.double().cpu().numpy())
    log(f"[bench] plain fp32: {iters} iterations of 256 chains in {t_plain:.3f} s")

    # measured gradient error of each form at its final state (chain 0 of the checked
    # problems) against the FP64 oracle on the unsplit FP32 X
    def grad_err(finals):
        errs = []
        for b, (Bf, Gf) in finals.items():
            pr = probs[b]
            G_o = oracle.grad_log_kernel(pr.X64, pr.y, Bf, pr.prior, pr.prior_scale, 1)
            errs.append(float(np.linalg.norm(Gf - G_o) / np.linalg.norm(G_o)))
        return max(errs)

    grads = 64 * chains * L * iters
    s_x = 4
    res = {
        "workload": f"64 problems n~U[1k,50k] p~U[64,2048] K~U[2,16], X FP32 / bf16 hi+lo / bf16 hi, "
                    f"4 chains each, L={L}, eps_b=0.4/(sqrt n_b + sqrt p_b), N(0,1) prior, "
                    f"{burn} untimed + {iters} timed iterations from B=0, independent Philox "
                    f"streams per form",
        "batched_bf16": {"chain_grad_evals_per_s": round(grads / dt_b, 1), "seconds": round(dt_b, 3),
                         "accept_rate": round(acc_b, 4),
                         "tuning": {"rows_per_slice": run_b["rows"], "grid": run_b["grid"]},
                         "grad_rel_l2_measured": grad_err(final_b),
                         "pass_mean_us": round(run_b["pass_us"], 2),
                         "hbm_gbs_algorithmic": round(elems * s_x / (run_b["pass_us"] * 1e-6) / 1e9, 1),
                         "frac_of_8tbs": round(elems * s_x / (run_b["pass_us"] * 1e-6) / 1e9 / HBM_PEAK_GBS, 4)},
        "batched_bf16_hi_only": {
            "chain_grad_evals_per_s": round(grads / run_h["dt"], 1), "seconds": round(run_h["dt"], 3),
            "accept_rate": round(run_h["acc"], 4),
            "tuning": {"rows_per_slice": run_h["rows"], "grid": run_h["grid"]},
            "grad_rel_l2_measured": grad_err(run_h["final"]),
            "pass_mean_us": round(run_h["pass_us"], 2),
            "hbm_gbs_algorithmic": round(elems * 2 / (run_h["pass_us"] * 1e-6) / 1e9, 1),
            "frac_of_8tbs": round(elems * 2 / (run_h["pass_us"] * 1e-6) / 1e9 / HBM_PEAK_GBS, 4),
            "speedup_vs_plain_fp32": round(t_plain / run_h["dt"], 2),
            "note": "X rounded to bfloat16 once (2 bytes per element): its gradient error against "
                    "the unsplit X is the rounding of the data, not of the arithmetic"},
        "plain_fp32": {"chain_grad_evals_per_s": round(grads / t_plain, 1), "seconds": round(t_plain, 3),
                       "accept_rate": round(float(np.mean(acc_p)), 4),
                       "grad_rel_l2_measured": grad_err(final_p)},
        "grad_error_note": "largest gradient rel-L2 against the FP64 oracle (unsplit FP32 X) at "
                           f"the final state of chain 0 of problems {list(check)}",
        "speedup": round(t_plain / dt_b, 2),
    }
    if accuracy:
        log("[bench] forms: accuracy study")
        res["posterior_means"] = forms_accuracy(hmc, torch, probs, fp32, bf, seed, bf_hi=bf_hi)
        pm = res["posterior_means"]
        log(f"[bench] forms: accuracy study done (oracle {pm['oracle_seconds']} s); beyond 3 MCSE: "
            f"batched vs oracle {pm['batched_vs_oracle']['frac_beyond_3_mcse']}, hi only vs oracle "
            f"{pm['hi_only_vs_oracle']['frac_beyond_3_mcse']}, plain vs oracle "
            f"{pm['plain_vs_oracle']['frac_beyond_3_mcse']}")
    return res


def capped_ess(samples: np.ndarray, accepted: np.ndarray, diagnostics) -> np.ndarray:
    """ESS per coordinate of one Metropolis chain (T x d samples, T accept flags), capped at
    the number of distinct states the chain visited (accepted moves + 1): between accepted
    moves the chain repeats its state, and an autocorrelation estimator applied to a chain
    that moved once or twice can return up to its full length (one move at the last of 80
    iterations gives 80 under Geyer's estimator and the split-chain one alike). Coordinates
    that never moved have no ESS and are dropped."""
    e = diagnostics.ess(samples)
    e = e[np.isfinite(e)]
    return np.minimum(e, float(np.sum(accepted)) + 1.0)


def ess_segment(hmc, torch, dp, prob, B, G, logk, eps, n_iter, seed, first_iter, diagnostics):
    """Effective samples per second at equilibrium: a chain segment of n_iter iterations at
    T = 1 continuing from the current state, run as graph replays outside the timed region.
    The first 20% are discarded as burn-in; ESS (Geyer's initial monotone sequence) is taken
    per free coordinate over the rest and divided by the device time of those kept
    iterations."""
    burn = n_iter // 5
    keep = n_iter - burn
    if burn:
        pl, _ = hmc.plan(dp, B, G, logk, eps, prob.L, burn, seed=seed, first_iter=first_iter,
                         record_samples=False)
        pl.launch(burn)
        torch.cuda.synchronize()
        pl.destroy()
    pl, out = hmc.plan(dp, B, G, logk, eps, prob.L, keep, seed=seed, first_iter=first_iter + burn,
                       record_samples=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    pl.launch(keep)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    pl.destroy()
    free = np.ones((prob.p, prob.K), dtype=bool)
    if prob.pin_last_class:
        free[:, -1] = False
    samples = out["samples"].float().cpu().numpy().reshape(keep, -1)[:, free.reshape(-1)]
    accepted = out["accepted"].cpu().numpy()
    e = capped_ess(samples, accepted, diagnostics)
    acc = float(accepted.mean())
    log(f"[bench] ESS segment eps={eps:g}: {n_iter} iterations ({burn} discarded), accept {acc:.3f}, "
        f"min ESS {e.min() if e.size else float('nan'):.1f} in {dt:.3f} s")
    return {"iterations": n_iter, "discarded": burn, "kept": keep, "eps": eps,
            "seconds_kept": round(dt, 4), "accept_rate": round(acc, 4),
            "divergent": int(out["divergent"].sum()),
            "ess_min": round(float(e.min()), 2) if e.size else None,
            "ess_median": round(float(np.median(e)), 2) if e.size else None,
            "ess_min_per_s": round(float(e.min()) / dt, 2) if e.size else None,
            "ess_median_per_s": round(float(np.median(e)) / dt, 2) if e.size else None,
            "note": "ESS per free coordinate (Geyer initial monotone sequence, capped at the "
                    "distinct states visited: accepted moves + 1) of the kept iterations over "
                    "their device time"}


def tune_eps(hmc, dp, prob, B, G, logk, eps0, seed, first_iter, lo=0.65, hi=0.75, probe=20,
             max_probes=10):
    """A step size whose acceptance falls in [lo, hi] (Section 3.2 tunes its step size to
    0.65-0.75): short probes of `probe` iterations from the current state, halving the step
    while acceptance is below the band and growing it by half while above, then bisecting
    (geometrically) between the last step sizes on either side. Moves the chain state (used
    as further warm-up)."""
    eps, below, above = eps0, None, None
    probes = []
    it = first_iter
    for _ in range(max_probes):
        out = hmc.sample(dp, B, G, logk, eps, prob.L, probe, seed=seed, first_iter=it,
                         record_samples=False)
        it += probe
        a = float(out["accepted"].float().mean())
        probes.append({"eps": eps, "iterations": probe, "accept_rate": round(a, 3)})
        if lo <= a <= hi:
            break
        if a < lo:
            above = eps
        else:
            below = eps
        if above is not None and below is not None and above < 1.02 * below:
            # the bracket has closed without a probe in the band: the acceptance measured at
            # its upper end (early, perhaps before the chain had moved) no longer holds, so
            # grow from the lower end again
            above = None
        if above is not None and below is not None:
            eps = float(np.sqrt(above * below))
        elif above is not None:
            eps = eps * 0.5
        else:
            eps = eps * 1.5
    else:
        # no probe landed in the band: the probed step size closest to its centre
        eps = min(probes, key=lambda q: abs(q["accept_rate"] - 0.5 * (lo + hi)))["eps"]
    log(f"[bench] tuned eps {eps:g} after {len(probes)} probes")
    return eps, probes


def batched_passes(hmc, torch, passes: int, hi_only: bool = False) -> dict:
    """Only the batched split-precision gradient pass of the 64-problem batch (4 chains each,
    bf16 hi + lo planes split on the device, or the hi planes alone, autotuned decomposition),
    `passes` times at B = 0: the short run that profilers and counters are taken on."""
    from workloads import make_batched
    probs = make_batched(64)
    dev = torch.device("cuda:0")
    bf = []
    for pr in probs:
        X = torch.from_numpy(pr.X).to(dev)
        hi, lo = hmc.split_bf16(X, hi_only=hi_only)
        del X
        bf.append(hmc.Problem(hi, torch.from_numpy(pr.y).to(dev), pr.K, pr.prior, pr.prior_scale, True,
                              X_lo=lo))
    bt = hmc.Batch(bf, 4)
    B, G, logk = bt.zeros_state()
    rows, grid = bt.autotune(B, G, logk)
    hmc.hmc_profile_begin(passes, 1)
    for _ in range(passes):
        bt.logpost_grad(B, G, logk)
    _, us, mn, mx = hmc.hmc_profile_end()
    elems = sum(pr.n * pr.p for pr in probs)
    s_x = 2 if hi_only else 4
    return {"batched_passes": {"passes": passes, "planes": "hi" if hi_only else "hi+lo",
                               "tuning": {"rows_per_slice": rows, "grid": grid},
                               "pass_mean_us": round(us, 2), "pass_min_us": round(mn, 2),
                               "algorithmic_bytes": elems * s_x,
                               "frac_of_8tbs": round(elems * s_x / (us * 1e-6) / 1e9 / HBM_PEAK_GBS, 4)}}


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None, help="timed HMC iterations")
    ap.add_argument("--warmup", type=int, default=None, help="untimed HMC iterations")
    ap.add_argument("--workload", default="c2_f32")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-tune", action="store_true",
                    help="use the library's built-in launch rule instead of the autotuned one")
    ap.add_argument("--ess-iters", type=int, default=-1,
                    help="iterations of the equilibrium segment ESS/s is measured on (-1: the "
                         "workload's stated length, e.g. 1000 at n=20000, p=1000, K=10; 0 skips)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 1 GiB device-to-device copy 5 times (the reference "
                         "kernel that scales the FETCH_SIZE / WRITE_SIZE counters) and exit")
    ap.add_argument("--forms-only", action="store_true",
                    help="run only the BF16+batched vs plain FP32 comparison and print it")
    ap.add_argument("--forms-iters", type=int, default=100,
                    help="iterations of the BF16+batched vs plain FP32 comparison (0 skips it)")
    ap.add_argument("--hi-only", action="store_true",
                    help="with --batched-passes: the batch on the bf16 hi planes alone")
    ap.add_argument("--batched-passes", type=int, default=0, metavar="K",
                    help="run only K batched split-precision gradient passes of the 64-problem "
                         "batch (for profilers) and print their time")
    ap.add_argument("--table1", action="store_true",
                    help="run only the timing sweep of Table 1 (224 (N, K, p) combinations, "
                         "pinned and unpinned) and print it")
    ap.add_argument("--table1-quick", action="store_true",
                    help="the sweep on N <= 1000 and p <= 1000 only")
    ap.add_argument("--rows-sweep", type=int, nargs="*", default=None, metavar="N",
                    help="run only the plain-FP32 pass at p=1000, K=10 for the given row counts "
                         "(default 20000 60000 200000 1000000) and print it")
    ap.add_argument("--shards", type=int, default=0, metavar="G",
                    help="run only one GPU's share of each configuration sharded over G GPUs "
                         "(rows, or columns for the high-dimensional one) and print it")
    ap.add_argument("--configs", action="store_true",
                    help="every configuration timed against the FP64 oracle (one gradient, one "
                         "leapfrog update, full sampling run) instead of the benchmark line")
    ap.add_argument("--mnist-protocol", action="store_true",
                    help="run only the sampling protocol of Section 3.2 on the MNIST-shaped "
                         "stand-in and print it")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_1402_4089_amd as hmc
    from paper_1402_4089_amd import diagnostics
    from workloads import make_poisson, make_probit, make_problem

    if not torch.cuda.is_available():
        print("no GPU visible", file=sys.stderr)
        sys.exit(1)
    if args.copy_calibration:
        src = torch.ones(1 << 28, dtype=torch.float32, device="cuda:0")
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        log("[bench] copy calibration: 5 copies of 1 GiB (1048576 KiB read and written each)")
        return
    hmc.load()
    if args.forms_only:
        print(json.dumps(forms_comparison(hmc, torch, max(args.forms_iters, 1), 20140217)), flush=True)
        return
    if args.batched_passes > 0:
        print(json.dumps(batched_passes(hmc, torch, args.batched_passes, args.hi_only)), flush=True)
        return
    if args.mnist_protocol:
        print(json.dumps(mnist_protocol(hmc, torch)), flush=True)
        return
    if args.configs:
        print(json.dumps(config_timings(hmc, torch)), flush=True)
        return
    if args.shards > 0:
        print(json.dumps(shard_shares(hmc, torch, args.shards)), flush=True)
        return
    if args.rows_sweep is not None:
        rows = tuple(args.rows_sweep) or (20000, 60000, 200000, 1000000)
        print(json.dumps(rows_sweep(hmc, torch, rows=rows)), flush=True)
        return
    if args.table1 or args.table1_quick:
        print(json.dumps(table1_sweep(hmc, torch, quick=args.table1_quick)), flush=True)
        return
    d_steps, d_warm = DEFAULT_STEPS.get(args.workload, (100, 10))
    args.steps = d_steps if args.steps is None else args.steps
    args.warmup = d_warm if args.warmup is None else args.warmup
    if args.workload == "poisson_f32":
        # the Poisson-regression link through the same fused pass, at the default shape
        prob = make_poisson(20000, 1000)
    elif args.workload == "probit_f32":
        # the probit link through the same fused pass, at the default shape
        prob = make_probit(20000, 1000)
    elif args.workload == "c4_bf16hi":
        # the precision configuration with the hi plane only (2 bytes per element of X)
        prob = dataclasses.replace(make_problem("c4_bf16", xfmt="bf16"), name="c4_bf16hi")
    else:
        prob = make_problem(args.workload)
    log(f"[bench] workload {prob.name}: n={prob.n} p={prob.p} K={prob.K} xfmt={prob.xfmt} "
        f"L={prob.L} eps={prob.eps}")
    dev = torch.device("cuda:0")
    y = torch.from_numpy(prob.y).to(dev)
    if prob.xfmt in ("bf16hilo", "bf16"):
        # the precision form's one-time preparation: split X into bf16 planes on the device
        X64 = torch.from_numpy(prob.X64).to(dev)
        hi, lo = hmc.split_bf16(X64, hi_only=prob.xfmt == "bf16")
        torch.cuda.synchronize()
        del X64
        torch.cuda.empty_cache()
        dp = hmc.Problem(hi, y, prob.K, prob.prior, prob.prior_scale, bool(prob.pin_last_class),
                         X_lo=lo, tuning=None if args.no_tune else "auto")
    else:
        X = torch.from_numpy(np.asarray(prob.X)).to(dev)
        link = {"poisson": hmc.HMC_LINK_POISSON, "probit": hmc.HMC_LINK_PROBIT}.get(
            prob.meta.get("link"), hmc.HMC_LINK_SOFTMAX)
        dp = hmc.Problem(X, y, prob.K, prob.prior, prob.prior_scale, bool(prob.pin_last_class),
                         link=link, tuning=None if args.no_tune else "auto")
    log(f"[bench] launch decomposition {dp.tuning}"
        + (f" (autotuned: {dp.tuned_us:.2f} us per gradient)" if dp.tuned_us else ""))
    B = dp.zeros_state()
    logk, G = hmc.logpost_grad(dp, B)
    seed = 20140217

    temps = torch.from_numpy(annealed_inv_temps(args.warmup)).to(dev)
    hmc.sample(dp, B, G, logk, prob.eps, prob.L, args.warmup, seed=seed, record_samples=False,
               inv_temperature=temps)
    torch.cuda.synchronize()
    log(f"[bench] warmup {args.warmup} iterations done")

    # eager segment: the same iterations launched kernel by kernel (wall clock)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    hmc.sample(dp, B, G, logk, prob.eps, prob.L, args.steps, seed=seed,
               first_iter=args.warmup, record_samples=False)
    torch.cuda.synchronize()
    dt_eager = time.perf_counter() - t0
    # kernel time of the gradient pass: a short eager run with every pass bracketed by a pair
    # of HIP events on its stream, PROFILE_REPEAT back-to-back launches of the (idempotent)
    # pass per pair
    n_prof = max(1, min(args.steps, 4))
    hmc.hmc_profile_begin(n_prof * prob.L, PROFILE_REPEAT)
    hmc.sample(dp, B, G, logk, prob.eps, prob.L, n_prof, seed=seed,
               first_iter=args.warmup + args.steps, record_samples=False)
    launches, mean_us, min_us, max_us = hmc.hmc_profile_end()
    log(f"[bench] eager: {args.steps} iterations in {dt_eager:.3f} s; gradient pass: {launches} "
        f"event pairs x {PROFILE_REPEAT} launches, mean {mean_us:.2f} us per launch "
        f"(min {min_us:.2f}, max {max_us:.2f})")
    # timed segment: the same iteration captured once as a HIP graph and replayed
    plan, out = hmc.plan(dp, B, G, logk, prob.eps, prob.L, args.steps, seed=seed,
                         first_iter=args.warmup + args.steps + n_prof, record_samples=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    plan.launch(args.steps)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    plan.destroy()
    log(f"[bench] graph: {args.steps} iterations in {dt:.3f} s")

    grads = args.steps * prob.L
    value = grads / dt
    acc = float(out["accepted"].float().mean())
    div = int(out["divergent"].sum())
    del out
    next_iter = args.warmup + 2 * args.steps + n_prof

    # run-to-run spread of the same replay, outside the timed segment: five more replays of
    # a fifth of the timed iterations each (the paper averages 5 runs)
    rep_iters = max(1, args.steps // 5)
    rep_rates = []
    for r in range(5):
        plan, _ = hmc.plan(dp, B, G, logk, prob.eps, prob.L, rep_iters, seed=seed,
                           first_iter=next_iter, record_samples=False)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        plan.launch(rep_iters)
        torch.cuda.synchronize()
        rep_rates.append(rep_iters * prob.L / (time.perf_counter() - t0))
        plan.destroy()
        next_iter += rep_iters
    replay_repeats = {"repeats": 5, "iterations_each": rep_iters,
                      "grad_evals_per_s": {"median": round(float(np.median(rep_rates)), 1),
                                           "mean": round(float(np.mean(rep_rates)), 1),
                                           "min": round(min(rep_rates), 1),
                                           "max": round(max(rep_rates), 1)}}
    log(f"[bench] replay repeats: median {replay_repeats['grad_evals_per_s']['median']:.1f}, "
        f"mean {replay_repeats['grad_evals_per_s']['mean']:.1f} grad evals/s")

    # effective samples per second at equilibrium: a separate segment of the configuration's
    # stated length, outside the timed region
    ess_seg = None
    if args.ess_iters != 0:
        n_seg = args.ess_iters if args.ess_iters > 0 else prob.n_iter
        ess_seg = ess_segment(hmc, torch, dp, prob, B, G, logk, prob.eps, n_seg, seed, next_iter,
                              diagnostics)
        next_iter += n_seg
        if not 0.65 <= ess_seg["accept_rate"] <= 0.75:
            # the configured step size is outside the paper's 0.65-0.75 acceptance band (at
            # n = 200000, p = 4096 it accepts almost nothing; at n = 20000, p = 1000 almost
            # everything, with short moves): a second segment at a step size tuned into the
            # band, labelled as such
            # probes as long as about 0.2 s of iterations allow (20 to 200): the acceptance
            # of a 20-iteration probe has a standard error near 0.1, as wide as the band
            probe = int(min(200, max(20, 0.2 / (dt / args.steps))))
            eps_t, probes = tune_eps(hmc, dp, prob, B, G, logk, prob.eps, seed, next_iter,
                                     probe=probe)
            next_iter += sum(pr["iterations"] for pr in probes)
            tuned = ess_segment(hmc, torch, dp, prob, B, G, logk, eps_t, n_seg, seed, next_iter,
                                diagnostics)
            next_iter += n_seg
            tuned["tuning_probes"] = probes
            ess_seg = {"configured_eps": ess_seg, "tuned_eps": tuned}

    s_x = X_BYTES[prob.xfmt]
    s_state = 8 if prob.xfmt == "f64" else 4
    alg_bytes = prob.n * prob.p * s_x + 4 * prob.n + 2 * prob.p * prob.K * s_state
    achieved = alg_bytes / (mean_us * 1e-6) / 1e9
    kernel = {"bf16hilo": "pack_b+hilo_logits+hilo_grad", "bf16": "pack_b+hilo_logits+hilo_grad"}.get(
        prob.xfmt, "wide_logits+wide_softmax+wide_grad" if prob.name == "c3_widep" else "fused_logpost_grad")
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": read_traffic(prob.name) if kernel == "fused_logpost_grad" else None,
                "kernel": kernel, "kernel_mean_us": round(mean_us, 3),
                "algorithmic_bytes_per_launch": alg_bytes}
    stream = read_stream_gbs(hmc, torch, prob.n * prob.p * s_x)
    roofline["measured_read_stream_gbs"] = round(stream, 1)
    if prob.n * prob.p * s_x < (256 << 20):
        # X fits the memory-side cache: the timed runs reuse it across passes (warm); the
        # cold figure re-reads X from HBM every pass
        cw = cold_warm_pass_us(hmc, torch, dp, B)
        cw["note"] = ("one launch per event pair (so both include the cost of recording the "
                      "events), 20 passes each; cold = a 640 MB streaming read before every pass "
                      "evicts X from the 256 MB memory-side cache")
        cold_us = mean_us + (cw["cold_us"] - cw["warm_us"])
        cw["cold_kernel_us_est"] = round(cold_us, 3)
        cw["cold_frac_est"] = round(alg_bytes / (cold_us * 1e-6) / 1e9 / HBM_PEAK_GBS, 4)
        roofline["cache"] = cw
    roofline["frac_of_measured_stream"] = round(achieved / stream, 4)
    roofline["stream_note"] = ("hmc_stream_read over a buffer of the X size on this GPU (every byte "
                               "read once per pass, 16-byte loads): the attainable read bandwidth")
    if prob.xfmt in ("bf16hilo", "bf16"):
        # the matrix-core side of the split-precision pass: three (hi + lo) or two (hi only)
        # bf16 products per element in each of the two contractions, classes padded to 16 and
        # p to 32, over the dense bf16 peak; useful work is 4 n p K_eff
        k_eff = prob.K - 1 if prob.pin_last_class else prob.K
        useful = 4.0 * prob.n * prob.p * k_eff
        products = 3 if prob.xfmt == "bf16hilo" else 2
        executed = products * 4.0 * prob.n * (32 * ((prob.p + 31) // 32)) * 16 * ((prob.K + 15) // 16)
        t = mean_us * 1e-6
        roofline["mfma"] = {"useful_tflops": round(useful / t / 1e12, 2),
                            "executed_tflops": round(executed / t / 1e12, 2),
                            "peak": BF16_PEAK_TFLOPS, "unit": "TFLOP/s",
                            "frac": round(executed / t / 1e12 / BF16_PEAK_TFLOPS, 4),
                            "useful_frac": round(useful / t / 1e12 / BF16_PEAK_TFLOPS, 4)}

    link_text = {"poisson": "Poisson link", "probit": "probit link"}.get(prob.meta.get("link"),
                                                                        "multinomial logit")
    prior_text = (f"Gaussian N(0,{prob.prior_scale:g}^2)" if prob.prior == 0
                  else f"Cauchy(0,{prob.prior_scale:g})")
    pin_text = "last class pinned" if prob.pin_last_class else "no class pinned"
    result = {
        "metric": METRIC, "value": round(value, 1), "unit": "grad_evals/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(1e3 * dt / args.steps, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": {"f64": "f64", "f32": "f32", "bf16hilo": "bf16x3", "bf16": "bf16x2"}[prob.xfmt],
        "data": "synthetic",
        "config": {"workload": f"{prob.name}: n={prob.n} p={prob.p} K={prob.K} X {prob.xfmt}, "
                               f"{link_text}, L={prob.L}, eps={prob.eps}, {prior_text} prior, "
                               f"{pin_text}, 1 chain, Philox momenta",
                   "n": prob.n, "p": prob.p, "K": prob.K, "L": prob.L, "eps": prob.eps,
                   "chains": 1, "parallelism": "single GPU",
                   "launch": {"tuning": dp.tuning,
                              "source": "built-in rule" if args.no_tune else
                                        ("autotuned in this run" if dp.tuned_us else "tuning cache")}},
        # at the configured step size; the tuned segment, if any, is reported beside it
        "ess_per_s": (ess_seg["configured_eps"] if ess_seg and "tuned_eps" in ess_seg else ess_seg or {}).get("ess_min_per_s"),
        "ess_median_per_s": (ess_seg["configured_eps"] if ess_seg and "tuned_eps" in ess_seg else ess_seg or {}).get("ess_median_per_s"),
        "ess_per_s_tuned_eps": (ess_seg["tuned_eps"].get("ess_min_per_s")
                                if ess_seg and "tuned_eps" in ess_seg else None),
        "ess_segment": ess_seg,
        "accept_rate": round(acc, 4), "divergent": div,
        "eager_grad_evals_per_s": round(args.steps * prob.L / dt_eager, 1),
        "replay_repeats": replay_repeats,
        "timing": "value: HIP-graph replay of one iteration (hmc_plan_launch); kernel time from "
                  "HIP events around every gradient pass of an eager run of the same kernels",
        "roofline": roofline,
    }
    if args.forms_iters > 0 and prob.name == "c2_f32":
        result["forms"] = forms_comparison(hmc, torch, args.forms_iters, seed)
        # the same pass with more rows per launch: the fixed cost per gradient amortised
        result["rows_sweep"] = rows_sweep(hmc, torch, rows=(200000, 1000000))["rows_sweep"]
    result["paper_context"] = {
        "grad_evals_per_s": 85.5, "hardware": "NVIDIA Tesla K20, FP32 (2014)",
        "workload": "MNIST HMC run: n=60000, p=785, K=10, L=100 (20,000 leapfrog steps in 234 s)",
        "note": "context only: a different workload and machine, so vs_baseline stays null"}
    if not args.no_cpu_baseline:
        base, rel, rel_x = cpu_baseline(prob, B.double().cpu().numpy(), G.double().cpu().numpy(),
                                        args.cpu_seconds)
        result["cpu_baseline"] = base
        result["grad_rel_l2_vs_oracle"] = rel
        if rel_x is not None:
            result["grad_rel_l2_vs_unsplit_x"] = rel_x
        if prob.xfmt == "f32" and prob.meta.get("link") is None:
            result["cpu_numpy_fp32"] = numpy_fp32_rate(prob, B.float().cpu().numpy())
        result["device_over_oracle"] = round(value / base["value"], 1)
    else:
        result["cpu_baseline"] = None
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
