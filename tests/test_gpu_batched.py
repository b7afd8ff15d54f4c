"""Batched form (many bf16 problems, several chains each) and graph plans (GPU tier).

Each chain of a batch is an independent HMC chain of its problem, so the oracle runs it
alone: FP64 on the values the device sees (X_eff = hi + lo), driven by the same Philox
draws (chain index b * chains + c). Gradient tolerance as for the single-problem bf16 form
(relative L2 <= 6e-5, from the three-term product error); decisions must agree outside
the tie band. Plans replay a captured graph and must reproduce the eager calls bit for
bit, across separate launches with host synchronisation and other work in between.
"""
import numpy as np
import pytest

import oracle
from oracle import philox, split
from workloads import make_batched, make_draws, make_problem, make_random_state

pytestmark = pytest.mark.gpu

GTOL = 6e-5


def _relL2(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def _x_eff(prob):
    hi, lo = split.split_hilo(prob.X64)
    return hi + lo


def _batch(lib, probs, chains, hi_only=False):
    import torch
    dev = []
    for pr in probs:
        X = torch.from_numpy(np.ascontiguousarray(pr.X)).cuda()
        hi, lo = lib.split_bf16(X, hi_only=hi_only)
        y = torch.from_numpy(pr.y).cuda()
        dev.append(lib.Problem(hi, y, pr.K, pr.prior, pr.prior_scale, bool(pr.pin_last_class), X_lo=lo))
    return lib.Batch(dev, chains)


def _small(n_prob=6, seed=21):
    return make_batched(n_prob, seed=seed, n_range=(40, 2500), p_range=(5, 300), K_range=(2, 16))


@pytest.mark.parametrize("chains", [1, 2, 4])
def test_batched_gradient_matches_oracle(lib, chains):
    import torch
    probs = _small(7, seed=30 + chains)
    bt = _batch(lib, probs, chains)
    B, G, logk = bt.zeros_state()
    states = []
    for b, pr in enumerate(probs):
        for c in range(chains):
            Bc = make_random_state(pr, 0.1, seed=100 * b + c).astype(np.float32)
            B[b][c].copy_(torch.from_numpy(Bc))
            states.append((b, c, Bc.astype(np.float64)))
    bt.logpost_grad(B, G, logk)
    lk = logk.cpu().numpy()
    worst = 0.0
    for b, c, Bc in states:
        pr = probs[b]
        lk_o, G_o = oracle.log_kernel_and_grad(_x_eff(pr), pr.y, Bc, pr.prior, pr.prior_scale, 1)
        err = _relL2(G[b][c].double().cpu().numpy(), G_o)
        worst = max(worst, err)
        assert err <= GTOL, f"problem {b} chain {c}: rel-L2 {err:.3e}"
        assert abs(lk[b, c] - lk_o) <= 1e-6 * abs(lk_o) + 1e-4
        assert np.all(G[b][c][:, -1].cpu().numpy() == 0)
    print(f"[batched] chains={chains}: worst gradient rel-L2 {worst:.3e}", flush=True)


@pytest.mark.parametrize("chains", [1, 2, 4])
def test_batched_hi_only_gradient_matches_oracle(lib, chains):
    """The batched form on hi planes alone (bf16 X, 2 bytes per element: X_eff = hi), every
    chain against the oracle on X_eff at the same bar as the hi + lo form."""
    import torch
    probs = _small(6, seed=60 + chains)
    bt = _batch(lib, probs, chains, hi_only=True)
    B, G, logk = bt.zeros_state()
    for b, pr in enumerate(probs):
        for c in range(chains):
            B[b][c].copy_(torch.from_numpy(make_random_state(pr, 0.1, seed=70 * b + c).astype(np.float32)))
    bt.logpost_grad(B, G, logk)
    lk = logk.cpu().numpy()
    worst = 0.0
    for b, pr in enumerate(probs):
        hi, _ = split.split_hilo(pr.X64)
        for c in range(chains):
            Bc = B[b][c].double().cpu().numpy()
            lk_o, G_o = oracle.log_kernel_and_grad(hi, pr.y, Bc, pr.prior, pr.prior_scale, 1)
            err = _relL2(G[b][c].double().cpu().numpy(), G_o)
            worst = max(worst, err)
            assert err <= GTOL, f"problem {b} chain {c}: rel-L2 {err:.3e}"
            assert abs(lk[b, c] - lk_o) <= 1e-6 * abs(lk_o) + 1e-4
    print(f"[batched] hi only, chains={chains}: worst gradient rel-L2 {worst:.3e}", flush=True)


def test_batched_sampler_matches_oracle_chains(lib):
    probs = _small(5, seed=41)
    chains, n_iter, L, seed = 2, 4, 5, 77
    bt = _batch(lib, probs, chains)
    B, G, logk = bt.zeros_state()
    bt.logpost_grad(B, G, logk)
    eps = [0.5 * pr.eps for pr in probs]
    out = bt.sample(B, G, logk, eps, L, n_iter, seed=seed, record_samples=True)
    acc = out["accepted"].cpu().numpy()
    H = out["H"].cpu().numpy()
    agree = ties = 0
    for b, pr in enumerate(probs):
        Xe = _x_eff(pr)
        for c in range(chains):
            ch = b * chains + c
            xis, us = philox.draws(seed, ch, n_iter, pr.p, pr.K)
            orc = oracle.sample(Xe, pr.y, pr.K, xis, us, eps[b], L, pr.prior, pr.prior_scale, 1)
            dH_o = orc["H"][:, 0] - orc["H"][:, 1]
            margin = np.abs(np.log(us) - dH_o)
            dH = np.abs((H[:, ch, 0] - H[:, ch, 1]) - dH_o)
            for t in range(n_iter):
                assert dH[t] < 5e-3, f"problem {b} chain {c} iteration {t}: delta-H error {dH[t]:.2e}"
                if margin[t] <= 5e-3:
                    ties += 1
                    break                       # the chains may part after a tie
                assert acc[t, ch] == orc["accepted"][t], f"problem {b} chain {c} iteration {t}"
                agree += 1
                err = _relL2(out["samples"][b][t, c].double().cpu().numpy(), orc["samples"][t])
                assert err < 1e-4, f"problem {b} chain {c} iteration {t}: state rel-L2 {err:.2e}"
    assert agree >= 30
    print(f"[batched] sampler: {agree} decisions compared, {ties} tie stops", flush=True)


def test_batched_plan_replays_match_eager(lib):
    import torch
    probs = _small(4, seed=52)
    chains, n_iter, L, seed = 4, 6, 4, 5
    eps = [0.5 * pr.eps for pr in probs]
    bt = _batch(lib, probs, chains)
    B1, G1, l1 = bt.zeros_state()
    bt.logpost_grad(B1, G1, l1)
    B2 = [b.clone() for b in B1]
    G2 = [g.clone() for g in G1]
    l2 = l1.clone()
    eager = bt.sample(B1, G1, l1, eps, L, n_iter, seed=seed, record_samples=True, moments=True)
    torch.cuda.synchronize()
    bt2 = _batch(lib, probs, chains)
    plan, rec = bt2.plan(B2, G2, l2, eps, L, n_iter, seed=seed, record_samples=True, moments=True)
    plan.launch(2)
    torch.cuda.synchronize()
    _ = torch.randn(1000, device="cuda").sum().item()       # unrelated eager work between replays
    plan.launch(3)
    torch.cuda.synchronize()
    plan.launch(1)
    torch.cuda.synchronize()
    for b in range(len(probs)):
        assert torch.equal(B1[b], B2[b]) and torch.equal(G1[b], G2[b])
        assert torch.equal(eager["samples"][b], rec["samples"][b])
        assert torch.equal(eager["moments"][b], rec["moments"][b])
        s = rec["samples"][b].double()
        assert torch.allclose(rec["moments"][b][0], s.sum(0), rtol=1e-12, atol=1e-12)
    assert torch.equal(l1, l2)
    assert torch.equal(eager["accepted"], rec["accepted"]) and torch.equal(eager["H"], rec["H"])
    with pytest.raises(lib.HMCError):
        plan.launch(1)                                      # records hold n_iter iterations
    plan.destroy()


def test_batched_autotune_then_sample(lib):
    probs = _small(6, seed=63)
    bt = _batch(lib, probs, 4)
    B, G, logk = bt.zeros_state()
    rows, grid = bt.autotune(B, G, logk)
    assert rows in (1024, 2048, 4096, 8192) and grid in (1024, 2048, 4096, 8192, 16384)
    for b, pr in enumerate(probs):
        G_o = oracle.grad_log_kernel(_x_eff(pr), pr.y, np.zeros((pr.p, pr.K)))
        for c in range(4):
            assert _relL2(G[b][c].double().cpu().numpy(), G_o) <= GTOL
    out = bt.sample(B, G, logk, [0.5 * pr.eps for pr in probs], 3, 2, seed=1)
    assert out["accepted"].shape == (2, 24)


@pytest.mark.parametrize("name,xfmt", [("c1_small_f64", None), ("c2_f32", None)])
def test_single_plan_replays_match_eager(lib, name, xfmt):
    import torch
    prob = make_problem(name, n=700, p=40, K=5)
    X = torch.from_numpy(np.asarray(prob.X)).cuda()
    y = torch.from_numpy(prob.y).cuda()
    dp = lib.Problem(X, y, prob.K, prob.prior, prob.prior_scale, True)
    B1 = dp.zeros_state()
    l1, G1 = lib.logpost_grad(dp, B1)
    B2, G2, l2 = B1.clone(), G1.clone(), l1.clone()
    eager = lib.sample(dp, B1, G1, l1, 0.01, 5, 7, seed=9, first_iter=3)
    torch.cuda.synchronize()
    dp2 = lib.Problem(X, y, prob.K, prob.prior, prob.prior_scale, True)
    plan, rec = lib.plan(dp2, B2, G2, l2, 0.01, 5, 7, seed=9, first_iter=3)
    plan.launch(4)
    torch.cuda.synchronize()
    _ = torch.ones(10, device="cuda").sum().item()
    plan.launch(3)
    torch.cuda.synchronize()
    assert torch.equal(B1, B2) and torch.equal(G1, G2) and torch.equal(l1, l2)
    for k in ("accepted", "H", "divergent", "samples"):
        assert torch.equal(eager[k], rec[k]), k
    plan.destroy()


def test_single_plan_bf16_and_unbounded(lib):
    """A plan without records may run any number of iterations and continues the chain."""
    import torch
    prob = make_problem("c4_bf16", n=900, p=64, K=8)
    X = torch.from_numpy(prob.X64).cuda()
    hi, lo = lib.split_bf16(X)
    y = torch.from_numpy(prob.y).cuda()
    dp = lib.Problem(hi, y, prob.K, prob.prior, prob.prior_scale, True, X_lo=lo)
    B1 = dp.zeros_state()
    l1, G1 = lib.logpost_grad(dp, B1)
    B2, G2, l2 = B1.clone(), G1.clone(), l1.clone()
    lib.sample(dp, B1, G1, l1, 0.004, 4, 9, seed=2, record_samples=False)
    dp2 = lib.Problem(hi, y, prob.K, prob.prior, prob.prior_scale, True, X_lo=lo)
    args, _ = lib._sample_args(dp2, B2, 0.004, 4, 1, None, None, 2, 0, 0, None, False)
    args.accepted = args.H = args.divergent = None
    import ctypes
    h = ctypes.c_void_p()
    lib._check(lib.load().hmc_plan_create(ctypes.byref(h), ctypes.byref(dp2.desc), B2.data_ptr(),
                                          G2.data_ptr(), l2.data_ptr(), ctypes.byref(args),
                                          dp2.ws.data_ptr(), dp2.ws.numel(), None))
    plan = lib.Plan(h, (dp2, args))
    plan.launch(5)
    plan.launch(4)
    torch.cuda.synchronize()
    assert torch.equal(B1, B2) and torch.equal(l1, l2)
    plan.destroy()


def test_full_batch_gradient_sampled(lib):
    """The benchmark's batch at full size (64 problems, n ~ U[1k,50k], p ~ U[64,2048],
    K ~ U[2,16], 4 chains each) in the autotuned launch configuration the benchmark times:
    every chain at its own random state in one batched gradient, with the chains of the
    problems of largest p, largest n and largest K and one more checked against the oracle
    one by one."""
    import torch
    probs = make_batched(64)
    bt = _batch(lib, probs, 4)
    B, G, logk = bt.zeros_state()
    bt.autotune(B, G, logk)
    for b, pr in enumerate(probs):
        for c in range(4):
            Bc = make_random_state(pr, 0.05, seed=1000 * b + c).astype(np.float32)
            B[b][c].copy_(torch.from_numpy(Bc))
    bt.logpost_grad(B, G, logk)
    torch.cuda.synchronize()
    lk = logk.cpu().numpy()
    picks = {int(np.argmax([pr.p for pr in probs])), int(np.argmax([pr.n for pr in probs])),
             int(np.argmax([pr.K for pr in probs])), 17}
    worst = 0.0
    for b in sorted(picks):
        pr = probs[b]
        xe = _x_eff(pr)
        for c in (0, 3):
            Bc = B[b][c].double().cpu().numpy()
            lk_o, G_o = oracle.log_kernel_and_grad(xe, pr.y, Bc, pr.prior, pr.prior_scale, 1)
            err = _relL2(G[b][c].double().cpu().numpy(), G_o)
            worst = max(worst, err)
            assert err <= GTOL, f"problem {b} (n={pr.n}, p={pr.p}, K={pr.K}) chain {c}: {err:.3e}"
            assert abs(lk[b, c] - lk_o) <= 1e-6 * abs(lk_o) + 1e-4
    print(f"[batched] full batch, problems {sorted(picks)}: worst gradient rel-L2 {worst:.3e}",
          flush=True)


@pytest.mark.parametrize("use_plan", [False, True])
def test_batched_replay_and_annealing_match_oracle(lib, use_plan):
    """Replayed normals and uniforms per chain, with the annealed acceptance of Section 3.2
    (1/T_t shared by every chain), through hmc_sample_batched and through a batched plan:
    every chain equals the oracle chain driven by the same draws and temperatures
    (decisions outside the tie band, delta-H, states)."""
    import torch
    probs = _small(4, seed=88)
    chains, n_iter, L = 2, 6, 5
    eps = [0.5 * pr.eps for pr in probs]
    temps = oracle.annealed_inv_temps(n_iter, 20.0, 0.5)
    bt = _batch(lib, probs, chains)
    B, G, logk = bt.zeros_state()
    bt.logpost_grad(B, G, logk)
    draws = [[make_draws(pr.p, pr.K, n_iter, seed=(9, b, c)) for c in range(chains)]
             for b, pr in enumerate(probs)]
    nrm = [torch.from_numpy(np.ascontiguousarray(np.stack([d.xi for d in ds], axis=1))).cuda()
           for ds in draws]
    uni = [torch.from_numpy(np.ascontiguousarray(np.stack([d.u for d in ds], axis=1))).cuda()
           for ds in draws]
    it = torch.from_numpy(temps).cuda()
    if use_plan:
        plan, out = bt.plan(B, G, logk, eps, L, n_iter, record_samples=True, normals=nrm,
                            uniforms=uni, inv_temperature=it)
        plan.launch(2)
        torch.cuda.synchronize()
        plan.launch(n_iter - 2)
        torch.cuda.synchronize()
        plan.destroy()
    else:
        out = bt.sample(B, G, logk, eps, L, n_iter, record_samples=True, normals=nrm, uniforms=uni,
                        inv_temperature=it)
    torch.cuda.synchronize()
    acc = out["accepted"].cpu().numpy()
    H = out["H"].cpu().numpy()
    agree = 0
    for b, pr in enumerate(probs):
        Xe = _x_eff(pr)
        for c in range(chains):
            ch = b * chains + c
            d = draws[b][c]
            orc = oracle.sample(Xe, pr.y, pr.K, d.xi, d.u, eps[b], L, pr.prior, pr.prior_scale, 1,
                                inv_temps=temps)
            dH_o = orc["H"][:, 0] - orc["H"][:, 1]
            for t in range(n_iter):
                dH = abs((H[t, ch, 0] - H[t, ch, 1]) - dH_o[t])
                assert dH < 5e-3, f"problem {b} chain {c} iteration {t}: delta-H error {dH:.2e}"
                if abs(np.log(d.u[t]) - dH_o[t] * temps[t]) <= 5e-3 * temps[t]:
                    break                       # a tie: the chains may part here
                assert acc[t, ch] == orc["accepted"][t], f"problem {b} chain {c} iteration {t}"
                agree += 1
                err = _relL2(out["samples"][b][t, c].double().cpu().numpy(), orc["samples"][t])
                assert err < 1e-4, f"problem {b} chain {c} iteration {t}: state rel-L2 {err:.2e}"
    assert agree >= 30


def test_batched_epilogue_packing_equals_the_pack_pass(lib):
    """In a batched run the epilogue of each update packs the next pass's B operand; the
    gradient and log K each chain holds at the end (from its last proposal when accepted)
    must equal, bit for bit, a fresh batched evaluation at the final states, which packs B
    with the pack pass. All proposals are accepted here (eps small), so the held gradient is
    the one of the run's last pass."""
    import torch
    probs = _small(4, seed=91)
    bt = _batch(lib, probs, 2)
    B, G, logk = bt.zeros_state()
    bt.logpost_grad(B, G, logk)
    out = bt.sample(B, G, logk, [0.05 * pr.eps for pr in probs], 5, 2, seed=3)
    assert bool(out["accepted"].all())
    G2 = [torch.empty_like(g) for g in G]
    logk2 = torch.empty_like(logk)
    bt.logpost_grad(B, G2, logk2)
    torch.cuda.synchronize()
    for g, g2 in zip(G, G2):
        assert torch.equal(g, g2)
    assert torch.equal(logk, logk2)


# Chains of more than 16 classes take 2 or 4 class blocks each (chains x blocks <= 4): K up to
# 32 with 1 or 2 chains, up to 64 with 1 chain. The batch's block count follows its largest K,
# so its smaller problems are padded.
WIDE_K = [(2, (17, 32)), (1, (17, 32)), (1, (33, 64)), (1, (2, 64))]


@pytest.mark.parametrize("chains,K_range", WIDE_K)
def test_batched_wide_class_gradient_matches_oracle(lib, chains, K_range):
    import torch
    probs = make_batched(5, seed=60 + K_range[1] + chains, n_range=(40, 2000), p_range=(5, 300),
                         K_range=K_range)
    bt = _batch(lib, probs, chains)
    B, G, logk = bt.zeros_state()
    states = []
    for b, pr in enumerate(probs):
        for c in range(chains):
            Bc = make_random_state(pr, 0.1, seed=200 * b + c).astype(np.float32)
            B[b][c].copy_(torch.from_numpy(Bc))
            states.append((b, c, Bc.astype(np.float64)))
    bt.logpost_grad(B, G, logk)
    lk = logk.cpu().numpy()
    for b, c, Bc in states:
        pr = probs[b]
        lk_o, G_o = oracle.log_kernel_and_grad(_x_eff(pr), pr.y, Bc, pr.prior, pr.prior_scale, 1)
        err = _relL2(G[b][c].double().cpu().numpy(), G_o)
        assert err <= GTOL, f"problem {b} (K={pr.K}) chain {c}: rel-L2 {err:.3e}"
        assert abs(lk[b, c] - lk_o) <= 1e-6 * abs(lk_o) + 1e-4
        assert np.all(G[b][c][:, -1].cpu().numpy() == 0)


def test_batched_wide_class_sampler_and_packing(lib):
    """Two chains of K in [17, 32] (two class blocks each): a sampled run whose decisions and
    states follow the oracle chains driven by the same Philox draws, then the epilogue-packed
    B checked against a fresh packed evaluation (bit for bit)."""
    import torch
    probs = make_batched(4, seed=83, n_range=(40, 1500), p_range=(5, 200), K_range=(17, 32))
    chains, n_iter, L, seed = 2, 4, 5, 19
    bt = _batch(lib, probs, chains)
    B, G, logk = bt.zeros_state()
    bt.logpost_grad(B, G, logk)
    eps = [0.5 * pr.eps for pr in probs]
    out = bt.sample(B, G, logk, eps, L, n_iter, seed=seed, record_samples=True)
    acc = out["accepted"].cpu().numpy()
    H = out["H"].cpu().numpy()
    agree = 0
    for b, pr in enumerate(probs):
        Xe = _x_eff(pr)
        for c in range(chains):
            ch = b * chains + c
            xis, us = philox.draws(seed, ch, n_iter, pr.p, pr.K)
            orc = oracle.sample(Xe, pr.y, pr.K, xis, us, eps[b], L, pr.prior, pr.prior_scale, 1)
            dH_o = orc["H"][:, 0] - orc["H"][:, 1]
            margin = np.abs(np.log(us) - dH_o)
            for t in range(n_iter):
                assert abs((H[t, ch, 0] - H[t, ch, 1]) - dH_o[t]) < 5e-3
                if margin[t] <= 5e-3:
                    break                       # the chains may part after a tie
                assert acc[t, ch] == orc["accepted"][t], f"problem {b} chain {c} iteration {t}"
                agree += 1
                err = _relL2(out["samples"][b][t, c].double().cpu().numpy(), orc["samples"][t])
                assert err < 1e-4, f"problem {b} chain {c} iteration {t}: state rel-L2 {err:.2e}"
    assert agree >= 20
    # packing: a short all-accepted run, then the held gradient against a fresh evaluation
    out = bt.sample(B, G, logk, [0.05 * pr.eps for pr in probs], 5, 2, seed=3, first_iter=n_iter)
    assert bool(out["accepted"].all())
    G2 = [torch.empty_like(g) for g in G]
    logk2 = torch.empty_like(logk)
    bt.logpost_grad(B, G2, logk2)
    torch.cuda.synchronize()
    for g, g2 in zip(G, G2):
        assert torch.equal(g, g2)
    assert torch.equal(logk, logk2)
