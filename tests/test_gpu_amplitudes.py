"""GPU parity of the forward contraction against the oracle, through the
C ABI: the 12-qubit amplitude, reduced 30-qubit-shaped circuits with
slicing (every slice, ragged batches), per-slice enumeration, both kernel
classes, partitions / determinism, and the full 30-qubit workload."""
import json
import os

import numpy as np
import pytest

from tests.gpu_util import banner, rel_l2
from workload import make_workload, make_rqc, Workload

pytestmark = pytest.mark.gpu

TOL_C64 = 1e-4
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


@pytest.fixture(scope="module")
def torch():
    import torch as t
    assert t.cuda.is_available(), "GPU tests need a GPU"
    return t


def _sv(w):
    from oracle import statevector as sv
    return sv.amplitudes(w.circuit, w.open_qubits, w.closed_bits)


def _reduced(rows=4, cols=5, cycles=10, n_open=6, t=12, seed=0):
    c = make_rqc(rows, cols, cycles, seed=seed)
    n = c.n_qubits
    open_q = tuple(range(n - n_open, n))
    closed = {q: int(b) for q, b in zip(range(n - n_open),
                                         np.random.default_rng(1).integers(0, 2, n - n_open))}
    return Workload(f"rqc{n}_t{t}", c, open_q, closed, t)


def test_rqc12_single_amplitude(torch):
    import paper_2205_00393_amd as P
    banner("rqc12 single amplitude")
    w = make_workload("rqc12")
    pr = P.prepare(w)
    plan = pr.plan()
    plan.bind(batch=1)
    out = plan.execute_range(0, 1 << len(pr.sliced))
    torch.cuda.synchronize()
    got = out.cpu().numpy()
    assert rel_l2(got, _sv(w)) < TOL_C64


@pytest.mark.parametrize("fat", [0, 1, 100])
@pytest.mark.parametrize("batch", [1, 5, 0])
def test_reduced_all_slices(torch, fat, batch):
    """fat = 1: MFMA GEMM wherever a tile fits; 100: generic kernel only."""
    import paper_2205_00393_amd as P
    w = _reduced()
    banner(f"reduced {w.name} fat={fat} batch={batch}")
    pr = P.prepare(w, alphas=(0.5, 1.0), taus=(0.0, 0.3), n_seeds=4)
    assert len(pr.sliced) >= 2
    plan = pr.plan(batch=batch, fat_threshold=fat)
    plan.bind(batch=batch if batch else 0, budget_bytes=1 << 30)
    n = 1 << len(pr.sliced)
    out = plan.execute_range(0, n)
    torch.cuda.synchronize()
    assert rel_l2(out.cpu().numpy(), _sv(w)) < TOL_C64
    if fat == 1:
        kinds = [plan.step_kernel(k)[0] for k in range(plan.info()["n_steps"])]
        assert any(c > 0 for c in kinds), "no step took the MFMA path"


def test_slice_enumeration_matches_oracle(torch):
    """Each slice alone equals the oracle's contraction with S fixed to the
    bits of its id (Sec. 2.1.1 subtasks), placed at the same outputs."""
    import paper_2205_00393_amd as P
    from oracle import network as onw, planner as opl
    w = _reduced(cycles=8, t=10)
    pr = P.prepare(w, alphas=(1.0,), taus=(0.0, 0.3), n_seeds=3)
    onet = onw.absorb_small(onw.circuit_network(w.circuit, w.open_qubits, w.closed_bits))
    opath, oS, _ = opl.path_search(onet.indices, w.max_rank, (), (1.0,), (0.0, 0.3), 3)
    assert (opath, oS) == (pr.path, pr.sliced)
    plan = pr.plan(fat_threshold=1)
    plan.bind(batch=3)
    # some slices are exactly zero (fsim(pi/2, .) is a phased permutation),
    # so each slice's error is measured against the norm of the full output
    scale = np.linalg.norm(_sv(w))
    nonzero = 0
    for s in range(1 << len(oS)):
        banner(f"slice {s}")
        out = plan.execute([s])
        torch.cuda.synchronize()
        ref = np.zeros(1 << len(onet.open_ids), dtype=np.complex128)
        blk = onw.slice_output(onet, opath, oS, s)
        ref[onw.place(onet, oS, s, blk)] += blk
        nonzero += np.linalg.norm(ref) > 1e-3 * scale
        assert np.linalg.norm(out.cpu().numpy() - ref) < TOL_C64 * scale
    assert nonzero >= 2


@pytest.mark.parametrize("batch", [2, 5, 16])
def test_sliced_open_indices_are_placed(torch, batch):
    """Slicing an open index places each slice's block instead of summing.
    Two open and two closed indices are sliced: 16 slices in 4 groups that
    share their sliced open bits (and so their targets). Batches of 5 and 16
    take the one-wave-per-element FP64 sum (equal targets summed in lane
    order, written once per target), batches of 2 the per-element loop."""
    import paper_2205_00393_amd as P
    w = _reduced(rows=3, cols=4, cycles=8, n_open=4, t=-1)
    pr = P.prepare(w, alphas=(1.0,), taus=(0.0,), n_seeds=1)
    net = pr.net
    closed = [x for x in range(net.n_indices) if x not in net.open_ids][:2]
    S = [net.open_ids[1], closed[0], net.open_ids[3], closed[1]] + [x for x in pr.sliced]
    plan = P.Plan(net, pr.path, S)
    plan.bind(batch=batch)
    out = plan.execute_range(0, 1 << len(S))
    torch.cuda.synchronize()
    assert rel_l2(out.cpu().numpy(), _sv(w)) < TOL_C64


def test_partition_and_rerun_determinism(torch):
    import paper_2205_00393_amd as P
    w = _reduced()
    pr = P.prepare(w, alphas=(0.5,), taus=(0.3,), n_seeds=2)
    plan = pr.plan(fat_threshold=1)
    plan.bind(batch=4)
    n = 1 << len(pr.sliced)
    a = plan.execute_range(0, n)
    b = plan.execute_range(0, n)
    ids = np.random.default_rng(0).permutation(n)
    c = plan.new_output()
    plan.execute(ids[: n // 3], c)
    plan.execute(ids[n // 3:], c)
    torch.cuda.synchronize()
    a, b, c = a.cpu().numpy(), b.cpu().numpy(), c.cpu().numpy()
    assert np.array_equal(a, b)                    # fixed reduction order
    assert rel_l2(c, a) < 1e-12                    # any partition, same sum
    # a lost chunk re-run into the same accumulator completes it
    d = plan.new_output()
    plan.execute(ids[: n // 2], d)
    plan.execute(ids[n // 2:], d)
    torch.cuda.synchronize()
    assert rel_l2(d.cpu().numpy(), a) < 1e-12


def test_autotuned_plan_parity(torch, tmp_path):
    import paper_2205_00393_amd as P
    w = _reduced(cycles=12, t=14)
    pr = P.prepare(w, alphas=(0.5, 1.0), taus=(0.0, 0.3), n_seeds=3)
    plan = pr.plan(fat_threshold=1)
    plan.bind(batch=4)
    cache = str(tmp_path / "tune.json")
    plan.autotune("c64", cache)
    assert json.load(open(cache))
    out = plan.execute_range(0, 1 << len(pr.sliced))
    torch.cuda.synchronize()
    assert rel_l2(out.cpu().numpy(), _sv(w)) < TOL_C64
    ms = plan.profile_steps(0)
    assert np.all(ms >= 0)


def test_rqc30_full_size(torch):
    """The 30-qubit workload at full size, all slices, in the benchmark's
    launch configuration (autotuned, largest batch), against the oracle's
    complex128 amplitudes stored by tests/golden/make_rqc30_reference.py."""
    import paper_2205_00393_amd as P
    path = os.path.join(GOLDEN, "rqc30_amplitudes.npy")
    if not os.path.exists(path):
        pytest.skip("golden rqc30 amplitudes not generated")
    ref = np.load(path)
    meta = json.load(open(os.path.join(GOLDEN, "rqc30_amplitudes.json")))
    w = make_workload("rqc30")
    pr = P.prepare(w)
    assert pr.sliced == meta["sliced"]
    plan = pr.plan()
    banner("rqc30 bind")
    plan.bind(batch=1 << len(pr.sliced))
    banner("rqc30 autotune")
    plan.autotune("c64")
    banner("rqc30 execute")
    out = plan.execute_range(0, 1 << len(pr.sliced))
    torch.cuda.synchronize()
    err = rel_l2(out.cpu().numpy(), ref)
    banner(f"rqc30 rel err {err:.3e}")
    assert err < TOL_C64


TOL_SPLIT = 5e-4


@pytest.mark.parametrize("mode", ["c64", "split_f16", "split_bf16"])
@pytest.mark.parametrize("reconf_k", [8, 10])
def test_rqc30_reconfigured_path(torch, mode, reconf_k):
    """The 30-qubit workload on the path improved by subtree reconfiguration
    (different tree, same amplitudes): all slices, autotuned, against the
    stored oracle amplitudes. Window 8 leaves 4 sliced indices; window 10
    finds a tree that needs none (one slice, its root step a split sum)."""
    import paper_2205_00393_amd as P
    path = os.path.join(GOLDEN, "rqc30_amplitudes.npy")
    if not os.path.exists(path):
        pytest.skip("golden rqc30 amplitudes not generated")
    ref = np.load(path)
    w = make_workload("rqc30")
    pr = P.prepare(w, reconf_k=reconf_k)
    plan = pr.plan()
    n = 1 << len(pr.sliced)
    banner(f"rqc30 reconfigured path (k={reconf_k}) |S|={len(pr.sliced)} {mode}")
    plan.bind(batch=n)
    plan.autotune(mode)
    out = plan.execute_range(0, n, mode=mode)
    torch.cuda.synchronize()
    err = rel_l2(out.cpu().numpy(), ref)
    banner(f"rqc30 reconfigured {mode} rel err {err:.3e}")
    assert err < (TOL_C64 if mode == "c64" else TOL_SPLIT)


@pytest.mark.parametrize("mode", ["c64", "split_bf16"])
def test_rqc30_refined_slicing(torch, mode):
    """A slicing set from the refiner (Algorithms 2-4, seeds 0 and 1) on the
    reconfigured 30-qubit path: a different set of sliced indices with no
    larger cost, contracted over all its slices against the stored oracle
    amplitudes."""
    import paper_2205_00393_amd as P
    path = os.path.join(GOLDEN, "rqc30_amplitudes.npy")
    if not os.path.exists(path):
        pytest.skip("golden rqc30 amplitudes not generated")
    ref = np.load(path)
    w = make_workload("rqc30")
    base = P.prepare(w, reconf_k=8)
    pr = P.prepare(w, reconf_k=8, refine_seeds=2)
    assert sorted(pr.sliced) != sorted(base.sliced)
    c0 = P.tree_costs(base.net, base.path, base.sliced).sliced
    c1 = P.tree_costs(pr.net, pr.path, pr.sliced).sliced
    assert c1 <= c0
    plan = pr.plan()
    n = 1 << len(pr.sliced)
    banner(f"rqc30 refined slicing {sorted(pr.sliced)} (was {sorted(base.sliced)}) {mode}")
    plan.bind(batch=n)
    out = plan.execute_range(0, n, mode=mode)
    torch.cuda.synchronize()
    err = rel_l2(out.cpu().numpy(), ref)
    banner(f"rqc30 refined slicing {mode} rel err {err:.3e}")
    assert err < (TOL_C64 if mode == "c64" else TOL_SPLIT)


@pytest.mark.parametrize("mode", ["split_f16", "split_bf16"])
@pytest.mark.parametrize("fat", [1, 0])
def test_reduced_split_precision(torch, mode, fat):
    """Split fp16 / bf16 GEMMs (hi + lo per real part, FP32 accumulate) on
    every MFMA step, FP64 slice sum; relative L2 vs the oracle <= 5e-4."""
    import paper_2205_00393_amd as P
    w = _reduced(cycles=12, t=14)
    banner(f"reduced split {mode} fat={fat}")
    pr = P.prepare(w, alphas=(0.5, 1.0), taus=(0.0, 0.3), n_seeds=3)
    plan = pr.plan(fat_threshold=fat)
    plan.bind(batch=3)
    n = 1 << len(pr.sliced)
    out = plan.execute_range(0, n, mode=mode)
    ref64 = plan.execute_range(0, n, mode="c64")
    torch.cuda.synchronize()
    sv = _sv(w)
    err = rel_l2(out.cpu().numpy(), sv)
    banner(f"{mode} err {err:.3e} (c64 {rel_l2(ref64.cpu().numpy(), sv):.3e})")
    assert err < TOL_SPLIT
    kinds = [plan.step_kernel(k, mode)[0] for k in range(plan.info()["n_steps"])]
    if fat == 1:
        assert 2 in kinds, "no step took the split MFMA path"


@pytest.mark.parametrize("mode", ["split_f16", "split_bf16"])
def test_rqc30_split_full_size(torch, mode):
    import paper_2205_00393_amd as P
    path = os.path.join(GOLDEN, "rqc30_amplitudes.npy")
    if not os.path.exists(path):
        pytest.skip("golden rqc30 amplitudes not generated")
    ref = np.load(path)
    w = make_workload("rqc30")
    pr = P.prepare(w)
    plan = pr.plan()
    plan.bind(batch=1 << len(pr.sliced))
    banner(f"rqc30 {mode} autotune")
    plan.autotune(mode)
    out = plan.execute_range(0, 1 << len(pr.sliced), mode=mode)
    torch.cuda.synchronize()
    err = rel_l2(out.cpu().numpy(), ref)
    banner(f"rqc30 {mode} rel err {err:.3e}")
    assert err < TOL_SPLIT


def test_rqc53_sampled_slice(torch):
    """53-qubit workload at full size (t = 30, |S| = 68): the first two
    slices of the seeded subset (2^20 amplitudes each) in complex64, split
    fp16 and split bf16 against the oracle's complex128 contraction of the
    same slices, stored by tests/golden/make_rqc53_reference.py: element by
    element on 2^16 seeded output positions, and the block's squared norm."""
    import paper_2205_00393_amd as P
    path = os.path.join(GOLDEN, "rqc53_slices.npz")
    if not os.path.exists(path):
        pytest.skip("golden rqc53 slices not generated")
    ref = np.load(path)
    meta = json.load(open(os.path.join(GOLDEN, "rqc53_slices.json")))
    w = make_workload("rqc53")
    banner("rqc53 plan")
    pr = P.prepare(w)
    assert pr.sliced == meta["sliced"]
    assert len(meta["slices"]) >= 2
    plan = pr.plan()
    plan.bind(batch=1)
    for j, rec in enumerate(meta["slices"]):
        s = int(rec["id"])
        for mode, tol in (("c64", TOL_C64), ("split_f16", TOL_SPLIT), ("split_bf16", TOL_SPLIT)):
            banner(f"rqc53 slice {s} {mode}")
            out = plan.execute([s], mode=mode)
            torch.cuda.synchronize()
            got = out.cpu().numpy()
            err = rel_l2(got[ref["positions"]], ref["amplitudes"][j])
            n2 = float(np.sum(np.abs(got) ** 2))
            banner(f"rqc53 slice {s} {mode}: sampled rel err {err:.3e}, norm2 {n2:.6e} vs {rec['norm2']:.6e}")
            assert err < tol
            assert abs(n2 - rec["norm2"]) < 2 * tol * rec["norm2"]


def test_rqc53_reconfigured_sampled_slice(torch):
    """53-qubit workload on the reconfigured path (t = 30): the first two
    slices of the seeded subset in all three modes against the oracle's
    complex128 contraction of the same slices, element by element on the
    stored seeded output positions
    (tests/golden/make_rqc53_reference.py --reconf 8)."""
    import paper_2205_00393_amd as P
    path = os.path.join(GOLDEN, "rqc53_reconf_slices.npz")
    if not os.path.exists(path):
        pytest.skip("golden reconfigured rqc53 slices not generated")
    ref = np.load(path)
    meta = json.load(open(os.path.join(GOLDEN, "rqc53_reconf_slices.json")))
    w = make_workload("rqc53")
    banner("rqc53 reconfigured plan")
    pr = P.prepare(w, reconf_k=8)
    assert pr.sliced == meta["sliced"]
    assert len(meta["slices"]) >= 2
    plan = pr.plan()
    plan.bind(batch=1)
    for j, rec in enumerate(meta["slices"]):
        s = int(rec["id"])
        for mode, tol in (("c64", TOL_C64), ("split_f16", TOL_SPLIT), ("split_bf16", TOL_SPLIT)):
            banner(f"rqc53 reconfigured slice {s} {mode}")
            out = plan.execute([s], mode=mode)
            torch.cuda.synchronize()
            got = out.cpu().numpy()
            err = rel_l2(got[ref["positions"]], ref["amplitudes"][j])
            n2 = float(np.sum(np.abs(got) ** 2))
            banner(f"rqc53 reconfigured slice {s} {mode}: sampled rel err {err:.3e}, norm2 {n2:.6e} vs {rec['norm2']:.6e}")
            assert err < tol
            assert abs(n2 - rec["norm2"]) < 2 * tol * rec["norm2"]
