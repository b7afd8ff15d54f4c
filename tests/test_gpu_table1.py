"""The timing sweep of Section 3.1 (Table 1) as a parity sweep (GPU tier): every (N, K, p)
with N <= 1000 and p <= 1000 of Table 1, pinned and unpinned (140 combinations), one
gradient evaluation on the FP32 device path against the FP64 oracle on the same FP32 inputs.
The bound is the FP32 path's stated gradient tolerance, rel-L2 <= 1e-5."""
import math

import pytest

pytestmark = pytest.mark.gpu


def test_table1_quick_sweep_parity(lib):
    import torch
    import bench
    out = bench.table1_sweep(lib, torch, reps=1, quick=True, log_progress=False)["table1"]
    assert out["combinations"] == 2 * 5 * 7 * 2
    for r in out["records"]:
        assert math.isfinite(r["device_grad_us"]) and r["device_grad_us"] > 0
        assert r["grad_rel_l2"] <= 1e-5, r
    print(f"[table1] {out['combinations']} combinations, max rel-L2 {out['max_grad_rel_l2']:.2e}",
          flush=True)
