"""The allocation-free entry point, ltn_execute_scratch, against
ltn_execute on the same plans, through the C ABI: two calls in a row, the
second with a smaller input, each checked against ltn_execute's output
and the oracle's state vector at the stated tolerances."""
import numpy as np
import pytest

from tests.gpu_util import banner, rel_l2
from workload import make_workload, make_rqc, Workload

pytestmark = pytest.mark.gpu

TOL = {"c64": 1e-4, "split_f16": 5e-4, "split_bf16": 5e-4}


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


def test_execute_scratch_two_calls(torch):
    import paper_2205_00393_amd as P
    from paper_2205_00393_amd import _lib as L
    # call 1: a sliced 20-qubit circuit, every slice; the scratch holds
    # fewer slices than that, so several batches run (the last ragged)
    w = _reduced(cycles=12)
    pr = P.prepare(w, alphas=(0.5, 1.0), taus=(0.0, 0.3), n_seeds=3)
    plan = pr.plan()
    n = 1 << len(pr.sliced)
    per_slice = plan.workspace_size(2) - plan.workspace_size(1)
    fixed = plan.workspace_size(1) - per_slice
    fit = ((64 << 20) - fixed) // per_slice
    banner(f"scratch call 1: {w.name}, {n} slices, about {fit} per batch in the scratch")
    assert 1 <= fit < n
    plan.bind(batch=n)
    ids = np.arange(n, dtype=np.uint64)
    ref_sv = _sv(w)
    for mode in ("c64", "split_bf16"):
        want = plan.execute(ids, mode=mode)
        got = plan.execute_scratch(ids, mode=mode)
        torch.cuda.synchronize()
        want, got = want.cpu().numpy(), got.cpu().numpy()
        e_api, e_sv = rel_l2(got, want), rel_l2(got, ref_sv)
        banner(f"scratch call 1 {mode}: vs ltn_execute {e_api:.2e}, vs oracle {e_sv:.2e}")
        assert e_api < TOL[mode] and e_sv < TOL[mode]
    # call 2: a smaller input, the 12-qubit plan (one slice, one amplitude),
    # never bound to a workspace of its own
    w2 = make_workload("rqc12")
    pr2 = P.prepare(w2)
    plan2 = pr2.plan()
    banner("scratch call 2: rqc12, 1 slice")
    got2 = plan2.execute_scratch([0]).cpu().numpy()
    plan2.bind(batch=1)
    want2 = plan2.execute([0]).cpu().numpy()
    e_api, e_sv = rel_l2(got2, want2), rel_l2(got2, _sv(w2))
    banner(f"scratch call 2 c64: vs ltn_execute {e_api:.2e}, vs oracle {e_sv:.2e}")
    assert e_api < TOL["c64"] and e_sv < TOL["c64"]
    # the first plan's own binding was left as it was
    again = plan.execute(ids[:5]).cpu().numpy()
    first5 = plan.execute_scratch(ids[:5]).cpu().numpy()
    assert rel_l2(first5, again) < TOL["c64"]
    # a plan whose one slice needs more than the scratch is refused
    big = P.prepare(make_workload("rqc30")).plan()
    out = torch.zeros(64, dtype=torch.complex128, device="cuda")
    one = np.zeros(1, dtype=np.uint64)
    import ctypes as C
    st = L.lib().ltn_execute_scratch(big._h, one.ctypes.data_as(C.POINTER(C.c_uint64)), 1, 0,
                                     C.c_void_p(out.data_ptr()), None)
    assert st == -3 and "scratch" in L.lib().ltn_last_error().decode()
