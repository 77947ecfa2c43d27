"""The native host planner (libltn) against the oracle, bit for bit:
network structure after absorption, greedy paths, Eq. (1)/(4) costs, stems,
Algorithm 1 slicing sets, the path search, and the compiled plan's step
index sets and multiply-add count (Eq. (4) per slice)."""
import numpy as np
import pytest

import paper_2205_00393_amd as P
from oracle import network as onw
from oracle import planner as opl
from tests.netgen import random_network
from workload import make_workload, make_rqc

NAMES = ["rqc12", "rqc30", "rqc20_grad", "rqc53"]


def _both(name, **over):
    w = make_workload(name, **over)
    onet = onw.absorb_small(onw.circuit_network(w.circuit, w.open_qubits, w.closed_bits))
    cnet = P.Network.from_circuit(w.circuit, w.open_qubits, w.closed_bits)
    return w, onet, cnet


@pytest.mark.parametrize("name", NAMES)
def test_network_structure_and_data(name):
    w, onet, cnet = _both(name)
    assert cnet.indices == onet.indices
    assert cnet.open_ids == onet.open_ids
    assert cnet.n_indices == onet.n_indices
    assert cnet.params == onet.param
    for a, b in zip(cnet.leaf_data("c128"), onet.data):
        np.testing.assert_allclose(a, b, rtol=0, atol=1e-14)
    for a, b in zip(cnet.leaf_data("c64"), onet.data):
        np.testing.assert_allclose(a, b, rtol=0, atol=1e-7)


def test_network_without_absorption():
    w = make_workload("rqc12")
    raw = onw.circuit_network(w.circuit, w.open_qubits, w.closed_bits)
    cnet = P.Network.from_circuit(w.circuit, w.open_qubits, w.closed_bits, absorb=False)
    assert cnet.indices == raw.indices


@pytest.mark.parametrize("name", NAMES)
@pytest.mark.parametrize("alpha,tau,seed", [(1.0, 0.0, 0), (0.5, 0.3, 3), (2.0, 1.0, 7)])
def test_greedy_path_bit_exact(name, alpha, tau, seed):
    w, onet, cnet = _both(name)
    ex = onet.open_ids if w.slice_open else []
    po = opl.greedy_path(onet.indices, alpha, tau, seed, exclude=ex)
    pc = P.greedy_path(cnet, alpha, tau, seed, exclude=ex)
    assert pc == po


@pytest.mark.parametrize("seed", range(8))
def test_random_networks_greedy_costs_stem(seed):
    idx, n, opens = random_network(seed, 9, 14, 2)
    data = [np.ones([2] * len(ix), dtype=np.complex64) for ix in idx]
    cnet = P.Network.from_arrays(idx, data, opens, n)
    for alpha, tau in [(1.0, 0.0), (0.5, 0.5)]:
        po = opl.greedy_path(idx, alpha, tau, seed)
        assert P.greedy_path(cnet, alpha, tau, seed) == po
        tree = opl.Tree(idx, po)
        S = [int(x) for x in np.random.default_rng(seed).choice(n, 3, replace=False)]
        c = P.tree_costs(cnet, po, S)
        assert c.cost == tree.cost()
        assert c.sliced == tree.sliced_cost(S)
        assert c.space_log2 == int(np.log2(tree.space(S)))
        assert P.tree_stem(cnet, po) == tree.stem()
        for t in range(1, max(len(s) for s in tree.sets)):
            assert P.slice_finder(cnet, po, t) == opl.slice_finder(tree, t)


@pytest.mark.parametrize("name", ["rqc12", "rqc30", "rqc53"])
def test_stem_profile_matches_oracle_tree(name):
    """ltn_stem_profile: ranks and Eq. (1) node sizes along the stem, with
    and without S, against the oracle's tree."""
    w, onet, cnet = _both(name)
    p = opl.greedy_path(onet.indices, 0.5, 0.3, 1)
    tree = opl.Tree(onet.indices, p)
    S = opl.slice_finder(tree, w.max_rank if w.max_rank is not None else -1)
    rows = P.stem_profile(cnet, p, S)
    assert [r["tensor"] for r in rows] == tree.stem()
    Ss = set(S)
    for r in rows:
        v = r["tensor"]
        assert r["rank"] == len(tree.sets[v]) and r["rank_sliced"] == len(tree.sets[v] - Ss)
        if v < tree.L:
            assert r["log2_node_cost"] is None
        else:
            assert r["log2_node_cost"] == len(tree.node_set(v))
            assert r["log2_node_cost_sliced"] == len(tree.node_set(v) - Ss)


def test_slice_finder_hand_worked_stems():
    """The library's Algorithm 1 on the hand-worked chains of
    tests/golden/alg1_stems.json (Sec. 4.2)."""
    import json
    import os
    fix = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "alg1_stems.json")))
    for case in fix["cases"]:
        idx = case["leaves"]
        n = 1 + max(x for leaf in idx for x in leaf)
        opens = [x for x in range(n) if sum(x in leaf for leaf in idx) == 1]
        data = [np.ones([2] * len(ix), dtype=np.complex64) for ix in idx]
        cnet = P.Network.from_arrays(idx, data, opens, n)
        path = [tuple(p) for p in case["path"]]
        assert P.tree_stem(cnet, path) == [0, 6, 7, 8, 9, 10]
        assert P.slice_finder(cnet, path, case["t"]) == case["S"]


@pytest.mark.parametrize("name,t", [("rqc30", 26), ("rqc30", 22), ("rqc12", 6), ("rqc53", 30)])
def test_slice_finder_bit_exact(name, t):
    w, onet, cnet = _both(name)
    p = opl.greedy_path(onet.indices, 0.5, 0.3, 1)
    tree = opl.Tree(onet.indices, p)
    S = opl.slice_finder(tree, t)
    assert P.slice_finder(cnet, p, t) == S
    c = P.tree_costs(cnet, p, S)
    assert c.sliced == tree.sliced_cost(S) and c.cost == tree.cost()
    assert tree.space(S) <= 2 ** t


def test_slice_finder_with_pre_sliced_open_indices():
    w, onet, cnet = _both("rqc20_grad")
    pre = list(reversed(onet.open_ids))
    p = opl.greedy_path(onet.indices, exclude=pre)
    tree = opl.Tree(onet.indices, p)
    for t in (-1, 10, 8):
        assert P.slice_finder(cnet, p, t, pre) == opl.slice_finder(tree, t, pre)


@pytest.mark.parametrize("name", ["rqc12", "rqc30"])
def test_path_search_bit_exact(name):
    w, onet, cnet = _both(name)
    t = w.max_rank if w.max_rank is not None else -1
    kw = dict(alphas=(0.5, 1.0), taus=(0.0, 0.3), n_seeds=3, seed_base=5)
    po, So, to = opl.path_search(onet.indices, t, (), **kw)
    pc, Sc, tc = P.path_search(cnet, t, (), **kw)
    assert (pc, Sc, tc) == (po, So, to)


@pytest.mark.parametrize("name", ["rqc12", "rqc30", "rqc20_grad"])
def test_compiled_plan_matches_tree(name):
    """Plan compile: every step's operand/output index sets are the tree's
    sets minus S, and sum_steps 2^(m+k+n) * 2^|S| equals Eq. (4) exactly."""
    w, onet, cnet = _both(name)
    pr = P.prepare(w, alphas=(1.0,), taus=(0.0, 0.3), n_seeds=2)
    plan = pr.plan()
    info = plan.info()
    tree = opl.Tree(onet.indices, pr.path)
    S = set(pr.sliced)
    assert info["sliced_ids"] == pr.sliced
    assert info["macs_per_slice"] << len(S) == tree.sliced_cost(pr.sliced)
    for k, st in enumerate(plan.steps()):
        v = tree.L + k
        a, b = tree.children[v]
        assert (st["left"], st["right"], st["out"]) == (a, b, v)
        A = tree.sets[a] - S if st["a_is_left"] else tree.sets[b] - S
        B = tree.sets[b] - S if st["a_is_left"] else tree.sets[a] - S
        assert set(st["a_idx"]) == A and set(st["b_idx"]) == B
        assert set(st["c_idx"]) == tree.sets[v] - S
        assert st["k"] == len(A & B) and st["m"] == len(A - B) and st["n"] == len(B - A)
        # the contracted indices are the lowest bits of both operands, in
        # the same order
        assert st["a_idx"][: st["k"]] == st["b_idx"][: st["k"]]
        # the output is a merge of A's and B's free indices, each in order
        fa = [x for j, x in enumerate(st["c_idx"]) if (st["c_mask_a"] >> j) & 1]
        fb = [x for j, x in enumerate(st["c_idx"]) if not (st["c_mask_a"] >> j) & 1]
        assert fa == st["a_idx"][st["k"]:] and fb == st["b_idx"][st["k"]:]


def test_plan_load_errors():
    w, onet, cnet = _both("rqc12")
    p = P.greedy_path(cnet)
    with pytest.raises(P.LtnError):
        P.Plan(cnet, p[:-1] + [(p[-1][0], p[-1][0])], [])
    with pytest.raises(P.LtnError):
        P.Plan(cnet, p, [0, 0])
    with pytest.raises(P.LtnError) as e:
        P.Plan(cnet, p, [], max_rank=2)
    assert e.value.code == -2
    bad = [list(ix) for ix in onet.indices]
    bad[1] = bad[1] + [bad[0][0]]  # an index in three leaves
    data = [np.ones([2] * len(ix), dtype=np.complex64) for ix in bad]
    with pytest.raises(P.LtnError):
        P.Plan(P.Network.from_arrays(bad, data, onet.open_ids, onet.n_indices), p, [])


@pytest.mark.parametrize("name", ["rqc12", "rqc30", "rqc20_grad"])
def test_arena_liveness_no_overlap(name):
    """Tensors alive at the same time never share arena bytes, and every
    tensor lies inside the per-slice arena (leaves live from the gather at
    time 0, step k runs at time k+1, the slice sum at time L)."""
    w = make_workload(name)
    pr = P.prepare(w, alphas=(1.0,), taus=(0.0,), n_seeds=1)
    plan = pr.plan()
    info = plan.info()
    L = info["n_leaves"]
    steps = plan.steps()
    off, rank, born, dies = {}, {}, {}, {}
    for k, st in enumerate(steps):
        a, b = (st["left"], st["right"]) if st["a_is_left"] else (st["right"], st["left"])
        for v, o, r in ((a, st["arena_off"][0], st["m"] + st["k"]),
                        (b, st["arena_off"][1], st["n"] + st["k"]),
                        (st["out"], st["arena_off"][2], st["m"] + st["n"])):
            off[v], rank[v] = o, r
        dies[a] = dies[b] = k + 1
        born[st["out"]] = k + 1
    for v in off:
        born.setdefault(v, 0)
        dies.setdefault(v, L)
        assert off[v] + (8 << rank[v]) <= info["arena_bytes_per_slice"]
    vs = sorted(off)
    for i, u in enumerate(vs):
        for v in vs[i + 1:]:
            if born[u] <= dies[v] and born[v] <= dies[u]:
                lo = max(off[u], off[v])
                hi = min(off[u] + (8 << rank[u]), off[v] + (8 << rank[v]))
                assert lo >= hi, f"tensors {u} and {v} overlap while both alive"


@pytest.mark.parametrize("seed", range(8))
def test_slice_refiner_and_greedy_slicer_bit_exact_random(seed):
    idx, n, opens = random_network(seed, 10, 16, 2)
    data = [np.ones([2] * len(ix), dtype=np.complex64) for ix in idx]
    cnet = P.Network.from_arrays(idx, data, opens, n)
    p = opl.greedy_path(idx, 1.0, 0.0, seed)
    tree = opl.Tree(idx, p)
    mx = max(len(s) for s in tree.sets)
    for t in range(max(1, mx - 4), mx):
        S = opl.slice_finder(tree, t)
        for kw in ({"seed": seed}, {"seed": seed + 100, "iters_per_temp": 3, "alpha": 0.9},
                   {"seed": seed, "n_fixed": min(1, len(S)), "t0": 0.05, "tf": 1e-2}):
            assert P.slice_refine(cnet, p, t, S, **kw) == opl.slice_refine(tree, t, S, **kw)
        assert P.slice_greedy_overhead(cnet, p, t) == opl.greedy_overhead_slicer(tree, t)
        assert P.slice_greedy_overhead(cnet, p, t, S[:1]) == opl.greedy_overhead_slicer(tree, t, S[:1])


@pytest.mark.parametrize("name,t,kw", [("rqc12", 6, {}), ("rqc30", 22, {"tf": 0.05}),
                                       ("rqc20_grad", 10, {"tf": 0.05})])
def test_slice_refiner_bit_exact_workloads(name, t, kw):
    w, onet, cnet = _both(name)
    pre = list(reversed(onet.open_ids)) if w.slice_open else []
    p = opl.greedy_path(onet.indices, 0.5, 0.3, 1, exclude=pre)
    tree = opl.Tree(onet.indices, p)
    S = opl.slice_finder(tree, t, pre)
    got = P.slice_refine(cnet, p, t, S, n_fixed=len(pre), **kw)
    want = opl.slice_refine(tree, t, S, n_fixed=len(pre), **kw)
    assert got == want
    assert got[0][: len(pre)] == pre
    assert tree.sliced_cost(got[0]) <= tree.sliced_cost(S)


def test_slice_refiner_errors():
    idx, n, opens = random_network(0, 8, 12, 2)
    data = [np.ones([2] * len(ix), dtype=np.complex64) for ix in idx]
    cnet = P.Network.from_arrays(idx, data, opens, n)
    p = opl.greedy_path(idx, 1.0, 0.0, 0)
    with pytest.raises(P.LtnError, match="target rank"):
        P.slice_refine(cnet, p, 1, [])
    with pytest.raises(P.LtnError, match="alpha"):
        P.slice_refine(cnet, p, 99, [], alpha=1.5)
    with pytest.raises(P.LtnError, match="repeated"):
        P.slice_refine(cnet, p, 99, [0, 0])


@pytest.mark.parametrize("seed", range(6))
def test_reconfigure_bit_exact_random(seed):
    idx, n, opens = random_network(seed, 16, 28, 3)
    data = [np.ones([2] * len(ix), dtype=np.complex64) for ix in idx]
    cnet = P.Network.from_arrays(idx, data, opens, n)
    p = opl.greedy_path(idx, 0.5, 1.0, seed)
    for k in (3, 6, 9):
        want = opl.reconfigure(idx, p, k, sweeps=3)
        assert P.tree_reconfigure(cnet, p, k, 3) == want
        tr = opl.Tree(idx, want)
        t = max(1, max(len(s) for s in tr.sets) - 2)
        S = opl.slice_finder(tr, t)
        assert P.tree_reconfigure(cnet, want, k, 2, S, t) == opl.reconfigure(idx, want, k, 2, S, t)


@pytest.mark.parametrize("name", ["rqc12", "rqc30", "rqc20_grad"])
def test_path_search_with_reconfiguration_bit_exact(name):
    w, onet, cnet = _both(name)
    pre = list(reversed(onet.open_ids)) if w.slice_open else []
    t = w.max_rank if w.max_rank is not None else -1
    kw = dict(alphas=(1.0, 0.5), taus=(0.0, 0.3), n_seeds=2, reconf_k=6, reconf_sweeps=2)
    want = opl.path_search(onet.indices, t, pre, **kw)
    got = P.path_search(cnet, t, pre, **kw)
    assert got == (want[0], want[1], want[2])
