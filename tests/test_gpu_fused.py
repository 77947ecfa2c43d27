"""Fused sub-paths (secondary slicing): plans compiled with fuse_rank run
runs of stem steps as one kernel per run. Checked against the brute-force
state vector on reduced circuits (every slice, several batches, all modes),
against the stored oracle amplitudes on the full 30-qubit workload, and
against the same plan run step by step."""
import os

import numpy as np
import pytest

from tests.gpu_util import banner, rel_l2
from tests.test_gpu_amplitudes import GOLDEN, TOL_C64, _reduced, _sv
from workload import make_workload

pytestmark = pytest.mark.gpu
TOL_SPLIT = 5e-4


@pytest.fixture(scope="module")
def torch():
    import torch as t
    assert t.cuda.is_available(), "GPU tests need a GPU"
    return t


@pytest.mark.parametrize("cycles,t,fuse_rank", [(10, 14, 6), (10, 14, 7), (12, 16, 7)])
@pytest.mark.parametrize("batch", [1, 3, 0])
def test_fused_reduced(torch, cycles, t, fuse_rank, batch):
    import paper_2205_00393_amd as P
    w = _reduced(rows=4, cols=5, n_open=6, cycles=cycles, t=t)
    pr = P.prepare(w, alphas=(0.5, 1.0), taus=(0.0, 0.3), n_seeds=3, reconf_k=6)
    plan = P.Plan(pr.net, pr.path, pr.sliced, max_rank=t, fuse_rank=fuse_rank)
    groups = plan.groups()
    assert groups, "no fused sub-path found"
    n = 1 << len(pr.sliced)
    plan.bind(batch=batch, budget_bytes=1 << 30)
    ref = _sv(w)
    for mode in ("c64", "split_f16", "split_bf16"):
        banner(f"fused reduced cycles={cycles} t={t} fuse_rank={fuse_rank} batch={batch} {mode}: "
               f"{len(groups)} groups {groups}")
        out = plan.execute_range(0, n, mode=mode)
        torch.cuda.synchronize()
        err = rel_l2(out.cpu().numpy(), ref)
        banner(f"  rel err {err:.3e}")
        assert err < (TOL_C64 if mode == "c64" else TOL_SPLIT)
    # step by step on the same plan and arena gives the same amplitudes
    plan.set_fusion(False)
    out2 = plan.execute_range(0, n)
    plan.set_fusion(True)
    out1 = plan.execute_range(0, n)
    torch.cuda.synchronize()
    assert rel_l2(out1.cpu().numpy(), out2.cpu().numpy()) < 1e-5


def test_fused_rqc30_full_size(torch):
    """The 30-qubit workload on the reconfigured path with fused sub-paths
    (working rank 11), all slices, every mode, against the stored oracle
    amplitudes; fused and step-by-step times are printed."""
    import time
    import paper_2205_00393_amd as P
    path = os.path.join(GOLDEN, "rqc30_amplitudes.npy")
    if not os.path.exists(path):
        pytest.skip("golden rqc30 amplitudes not generated")
    ref = np.load(path)
    w = make_workload("rqc30")
    pr = P.prepare(w, reconf_k=8)
    plan = P.Plan(pr.net, pr.path, pr.sliced, max_rank=w.max_rank, fuse_rank=11)
    groups = plan.groups()
    assert groups
    n = 1 << len(pr.sliced)
    plan.bind(batch=n)
    for mode in ("c64", "split_f16", "split_bf16"):
        banner(f"rqc30 fused {mode}: {len(groups)} groups")
        plan.autotune(mode)
        out = plan.execute_range(0, n, mode=mode)
        torch.cuda.synchronize()
        err = rel_l2(out.cpu().numpy(), ref)
        times = {}
        for fused in (True, False):
            plan.set_fusion(fused)
            plan.execute_range(0, n, out, mode)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(3):
                plan.execute_range(0, n, out, mode)
            torch.cuda.synchronize()
            times[fused] = (time.perf_counter() - t0) / 3 * 1e3
        plan.set_fusion(True)
        banner(f"rqc30 fused {mode}: rel err {err:.3e}; {times[True]:.2f} ms fused, "
               f"{times[False]:.2f} ms step by step")
        assert err < (TOL_C64 if mode == "c64" else TOL_SPLIT)
