"""GPU adjoint contraction (torch.autograd.Function over libltn) against
the oracle's gradient references."""
import os

import numpy as np
import pytest

from tests.gpu_util import banner, rel_l2
from workload import make_workload, make_rqc, sample_bitstrings, Workload

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


@pytest.fixture(scope="module")
def torch():
    import torch as t
    assert t.cuda.is_available()
    return t


def _run(torch, w, batch=0, tune_cache=None):
    import paper_2205_00393_amd as P
    from paper_2205_00393_amd.autograd import Amplitudes
    pr = P.prepare(w, alphas=(0.5, 1.0), taus=(0.0, 0.3), n_seeds=3)
    plan = pr.plan()
    plan.bind(batch=batch, grad=True, budget_bytes=8 << 30)
    if tune_cache is not None:
        plan.autotune("c64", tune_cache)
    ids = [pr.slice_of_bitstring(int(x)) for x in w.bitstrings]
    angles = torch.tensor(w.circuit.angles(), dtype=torch.float64, device="cuda",
                          requires_grad=True)
    out = Amplitudes.apply(angles, plan, ids)
    psi = out[torch.as_tensor(np.asarray(w.bitstrings), device="cuda")]
    loss = torch.sum(torch.log(torch.abs(psi) ** 2))
    loss.backward()
    torch.cuda.synchronize()
    return psi.detach().cpu().numpy(), float(loss), angles.grad.cpu().numpy()


def _small_workload():
    c = make_rqc(3, 3, 6, u3_seed=7)
    bs = sample_bitstrings(9, 32, 1)
    return Workload("u3_9", c, tuple(range(9)), {}, None, True, bs)


def test_small_gradient_against_sv_adjoint(torch):
    from oracle import gradients as gr
    w = _small_workload()
    banner("u3 3x3 gradient")
    psi, loss, g = _run(torch, w, batch=5)
    L, gref = gr.sv_adjoint(w.circuit, w.bitstrings)
    from oracle import statevector as sv
    assert rel_l2(psi, sv.bitstring_amplitudes(w.circuit, w.bitstrings)) < 1e-4
    assert abs(loss - L) < 1e-3 * abs(L)
    assert rel_l2(g, gref) < 1e-3


def test_rqc20_gradient(torch):
    path = os.path.join(GOLDEN, "rqc20_grad_reference.npz")
    if not os.path.exists(path):
        pytest.skip("golden gradient reference not generated")
    ref = np.load(path)
    w = make_workload("rqc20_grad")
    assert np.array_equal(ref["bitstrings"], w.bitstrings)
    banner("rqc20 gradient")
    psi, loss, g = _run(torch, w)
    assert rel_l2(psi, ref["amplitudes"]) < 1e-4
    assert rel_l2(g, ref["grad"]) < 1e-3
    sub = ref["subset"]
    assert rel_l2(g[sub], ref["finite_diff"]) < 1e-3
    assert rel_l2(g[sub], ref["param_shift"]) < 1e-3


def test_rqc20_gradient_autotuned(torch, tmp_path):
    """The same gradient after ltn_autotune in complex64 on a plan bound
    for gradients: forward steps and the adjoint products (cache keys
    g0_m_k_n_bB) take their timed tiles; parity against the oracle's
    adjoint gradient is unchanged. A second plan reading the written cache
    reproduces the gradient bit for bit."""
    import json
    path = os.path.join(GOLDEN, "rqc20_grad_reference.npz")
    if not os.path.exists(path):
        pytest.skip("golden gradient reference not generated")
    ref = np.load(path)
    w = make_workload("rqc20_grad")
    cache = str(tmp_path / "tune.json")
    banner("rqc20 gradient, autotuned forward and adjoint tiles")
    psi, loss, g = _run(torch, w, tune_cache=cache)
    keys = json.load(open(cache))
    adj = [k for k in keys if k.startswith("g0_")]
    banner(f"{len(adj)} adjoint product shapes tuned")
    assert adj, "no adjoint product was tuned"
    assert rel_l2(psi, ref["amplitudes"]) < 1e-4
    assert rel_l2(g, ref["grad"]) < 1e-3
    psi2, loss2, g2 = _run(torch, w, tune_cache=cache)
    assert np.array_equal(g, g2)


def _splitk64_fits(cfg, m, k, n):
    """Split-K configuration 6 (64 x 32 tile) or 7 (64 x 64) fits rows m,
    sum k, columns n (sums of 2^10 and more, chunks of at least 2^8 and of
    at most 2^(23 - m - n) per slice, each chunk at least one 16-deep k-tile)."""
    if k < 10:
        return False
    c = min(23 - (m + n), k - 8)
    return c > 0 and m >= 6 and n >= (5 if cfg == 6 else 6) and k - c >= 4


def test_rqc20_gradient_split_k_adjoint(torch, tmp_path):
    """Adjoint products with long sums forced onto the split-K tiles for
    64-row products (a tuning cache whose adjoint entries name split-K
    configuration 6, direct form, or 7, three-product form): the gradient
    still matches the oracle's adjoint gradient."""
    import json
    path = os.path.join(GOLDEN, "rqc20_grad_reference.npz")
    if not os.path.exists(path):
        pytest.skip("golden gradient reference not generated")
    ref = np.load(path)
    w = make_workload("rqc20_grad")
    cache = str(tmp_path / "tune.json")
    _run(torch, w, tune_cache=cache)
    keys = json.load(open(cache))
    for cfg in (6, 7):
        fits = [k for k in keys if k.startswith("g0_") and _splitk64_fits(cfg, *map(int, k.split("_")[1:4]))]
        assert fits, "no adjoint product has a long sum that the 64-row split-K tile fits"
        forced = dict(keys)
        for k in fits:
            forced[k] = [5000 + cfg, 0]
        path2 = str(tmp_path / f"forced{cfg}.json")
        json.dump(forced, open(path2, "w"))
        banner(f"rqc20 gradient, split-K configuration {cfg} on adjoint shapes {fits}")
        psi, loss, g = _run(torch, w, tune_cache=path2)
        assert rel_l2(psi, ref["amplitudes"]) < 1e-4
        assert rel_l2(g, ref["grad"]) < 1e-3


def test_gradient_reuses_one_batch_forward(torch):
    """On a plan bound for gradients with all slices in one batch, the
    autograd forward (ltn_execute) leaves its intermediates in the gradient
    arena and the backward does not recompute them. The amplitudes and the
    gradient must match a plan that recomputes (three batches), and a
    forward on other slices or new parameters in between must drop the kept
    intermediates (the gradient is then that of the slices and parameters
    the backward is asked for)."""
    import paper_2205_00393_amd as P
    from paper_2205_00393_amd.autograd import Amplitudes
    w = _small_workload()
    pr = P.prepare(w, alphas=(0.5, 1.0), taus=(0.0, 0.3), n_seeds=3)
    ids = [pr.slice_of_bitstring(int(x)) for x in w.bitstrings]
    sel = torch.as_tensor(np.asarray(w.bitstrings), device="cuda")
    a0 = torch.tensor(w.circuit.angles(), dtype=torch.float64, device="cuda")
    one, three = pr.plan(), pr.plan()
    assert one.bind(batch=64, grad=True, budget_bytes=1 << 30) >= len(ids)
    assert three.bind(batch=12, grad=True, budget_bytes=1 << 30) == 12

    def grad(plan, angles, between=None):
        a = angles.clone().requires_grad_(True)
        out = Amplitudes.apply(a, plan, ids)
        if between is not None:
            between()
        loss = torch.sum(torch.log(torch.abs(out[sel]) ** 2))
        loss.backward()
        torch.cuda.synchronize()
        return out.detach().cpu().numpy(), a.grad.cpu().numpy()

    o1, g1 = grad(one, a0)
    o3, g3 = grad(three, a0)
    banner(f"one-batch reuse vs three batches: amp {rel_l2(o1, o3):.2e}, grad {rel_l2(g1, g3):.2e}")
    assert rel_l2(o1, o3) < 1e-5 and rel_l2(g1, g3) < 1e-5
    # other work on the same plan between forward and backward
    _, g_other = grad(one, a0, between=lambda: one.execute(ids[:5]))
    assert rel_l2(g_other, g3) < 1e-5
    a1 = a0 + 0.01
    _, g_new3 = grad(three, a1)
    _, g_params = grad(one, a1, between=lambda: one.set_params(a0))
    assert rel_l2(g_params, g_new3) < 1e-5


def test_gradient_graph_replays_match_eager(torch):
    """Full gradient batches run from two captured graphs (recomputed
    forward, adjoint sweep). A plan bound with batch 4 replays them 8 times
    per call on 32 slices; three calls (cotangents a, b, a), with other work
    and synchronisations between them, must each match a plan whose single
    batch of 32 is below its bound size and so runs eagerly (to FP32
    reordering: kernel choices depend on the batch size), and the repeated
    cotangent must give bit-identical gradients."""
    import paper_2205_00393_amd as P
    w = _small_workload()
    pr = P.prepare(w, alphas=(0.5, 1.0), taus=(0.0, 0.3), n_seeds=3)
    ids = [pr.slice_of_bitstring(int(x)) for x in w.bitstrings]
    angles = torch.tensor(w.circuit.angles(), dtype=torch.float64, device="cuda")
    graphed, eager = pr.plan(), pr.plan()
    assert graphed.bind(batch=4, grad=True, budget_bytes=1 << 30) == 4
    assert eager.bind(batch=64, grad=True, budget_bytes=1 << 30) > len(ids)
    graphed.set_params(angles)
    eager.set_params(angles)
    gen = torch.Generator(device="cpu").manual_seed(11)
    n_out = 1 << graphed.info()["n_open"]
    cots = [torch.complex(torch.randn(n_out, generator=gen, dtype=torch.float64),
                          torch.randn(n_out, generator=gen, dtype=torch.float64)).cuda()
            for _ in range(2)]
    first = None
    for call, cot in enumerate([cots[0], cots[1], cots[0]]):
        out_g, out_e = graphed.new_output(), eager.new_output()
        g_graph = graphed.execute_grad(ids, cot, out_g)
        graphed.execute(ids[:3])  # other work on the same plan between replays
        torch.cuda.synchronize()
        g_eager = eager.execute_grad(ids, cot, out_e)
        torch.cuda.synchronize()
        gg = g_graph.cpu().numpy()
        err = rel_l2(gg, g_eager.cpu().numpy())
        err_out = rel_l2(out_g.cpu().numpy(), out_e.cpu().numpy())
        banner(f"gradient graph replay {call}: rel diff {err:.2e} (outputs {err_out:.2e})")
        assert err < 1e-5 and err_out < 1e-5
        if call == 0:
            first = gg
        if call == 2:
            assert np.array_equal(gg, first)
