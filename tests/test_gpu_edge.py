"""Edge cases through the C ABI: empty slice lists and ranges, slice ids out
of range, a plan with no slicing at all, every qubit open (the root is the
whole state vector), a ragged last batch with the largest batch the budget
allows, and outputs accumulated over calls."""
import numpy as np
import pytest

from tests.gpu_util import banner, rel_l2
from tests.test_gpu_amplitudes import _reduced, _sv
from workload import Workload, make_rqc, make_workload

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as t
    assert t.cuda.is_available(), "GPU tests need a GPU"
    return t


def test_empty_inputs_leave_output_untouched(torch):
    import paper_2205_00393_amd as P
    w = _reduced(cycles=8, t=10)
    pr = P.prepare(w, alphas=(1.0,), taus=(0.0,), n_seeds=1)
    plan = pr.plan()
    plan.bind(batch=2, budget_bytes=1 << 30)
    banner("empty slice list / range")
    out = plan.new_output()
    out.fill_(complex(1.5, -2.0))
    plan.execute([], out)
    plan.execute_range(3, 3, out)
    torch.cuda.synchronize()
    assert torch.all(out == complex(1.5, -2.0))


def test_out_of_range_ids_are_rejected(torch):
    import paper_2205_00393_amd as P
    w = _reduced(cycles=8, t=10)
    pr = P.prepare(w, alphas=(1.0,), taus=(0.0,), n_seeds=1)
    n = 1 << len(pr.sliced)
    plan = pr.plan()
    plan.bind(batch=2, budget_bytes=1 << 30)
    banner(f"out-of-range ids (2^|S| = {n})")
    with pytest.raises(P.LtnError):
        plan.execute([0, n])
    with pytest.raises(P.LtnError):
        plan.execute_range(0, n + 1)


def test_no_slicing_and_all_qubits_open(torch):
    """A 10-qubit circuit with every qubit open and no cap: one slice, the
    root tensor is the whole state vector in output order."""
    import paper_2205_00393_amd as P
    c = make_rqc(2, 5, 8, seed=4)
    w = Workload("open10", c, tuple(range(10)), {}, None)
    pr = P.prepare(w, alphas=(1.0,), taus=(0.0,), n_seeds=1)
    assert pr.sliced == []
    plan = pr.plan()
    plan.bind(batch=4, budget_bytes=1 << 30)
    banner("all qubits open, no slicing")
    out = plan.execute_range(0, 1)
    torch.cuda.synchronize()
    got = out.cpu().numpy()
    ref = _sv(w)
    assert got.shape == ref.shape == (1 << 10,)
    assert rel_l2(got, ref) < 1e-4
    assert abs(np.sum(np.abs(got) ** 2) - 1.0) < 1e-5


@pytest.mark.parametrize("mode", ["c64", "split_bf16"])
def test_ragged_batches_and_accumulation(torch, mode):
    """All slices in batches of 3 (the last one ragged), run twice into the
    same output: twice the amplitudes."""
    import paper_2205_00393_amd as P
    w = _reduced(cycles=10, t=12)
    pr = P.prepare(w, alphas=(0.5, 1.0), taus=(0.0, 0.3), n_seeds=3)
    n = 1 << len(pr.sliced)
    assert n % 3 != 0
    plan = pr.plan()
    plan.bind(batch=3, budget_bytes=1 << 30)
    banner(f"ragged batches of 3 over {n} slices, {mode}")
    out = plan.execute_range(0, n, mode=mode)
    plan.execute(list(range(n))[::-1], out, mode)
    torch.cuda.synchronize()
    assert rel_l2(out.cpu().numpy() / 2, _sv(w)) < (1e-4 if mode == "c64" else 5e-4)
