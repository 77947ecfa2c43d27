"""Pins of the oracle planner: Eq. (3) worked example, Eq. (1)/(2)/(4),
the halving/doubling rule, lifetime linearity, Algorithm 1 on hand-worked
stems and against brute force, and the no-overhead case of lifetimes
spanning a whole sub-path."""
import collections
import itertools
import json
import os

import numpy as np
import pytest

from oracle import network as nw
from oracle import planner as pl
from tests.netgen import random_network
from workload import make_workload

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _named_tree(fix):
    names = sorted({x for leaf in fix["leaves"] for x in leaf})
    ids = {n: i for i, n in enumerate(names)}
    leaves = [[ids[x] for x in leaf] for leaf in fix["leaves"]]
    tree = pl.Tree(leaves, [tuple(p) for p in fix["path"]])
    return tree, ids


def test_eq3_worked_example():
    """Sec. 3.1, Eq. (3): the contractions involving e and its lifetime."""
    fix = json.load(open(os.path.join(GOLDEN, "eq3_lifetime.json")))
    tree, ids = _named_tree(fix)
    to_set = lambda names: frozenset(ids[x] for x in names)
    for v, (a, b, c) in zip(tree.nodes(), fix["contractions"]):
        ca, cb = tree.children[v]
        assert tree.sets[ca] == to_set(a)
        assert tree.sets[cb] == to_set(b)
        assert tree.sets[v] == to_set(c)
    life = {tree.sets[v] for v in tree.lifetime(ids["e"])}
    assert life == {to_set(t) for t in fix["lifetime_of_e"]}
    corr = [v for v in tree.nodes() if ids["e"] in tree.node_set(v)]
    assert len(corr) == fix["correlated_contractions_of_e"]


def _executed_macs(leaves, path, S):
    """Multiply-adds a sliced contraction really does, from the ranks of
    the tensors it builds, summed over all 2^|S| subtasks."""
    tot = 0
    for s in range(1 << len(S)):
        fixed = set(S)
        tens = {i: [x for x in ix if x not in fixed] for i, ix in enumerate(leaves)}
        L = len(leaves)
        for k, (a, b) in enumerate(path):
            ia, ib = tens.pop(a), tens.pop(b)
            union = set(ia) | set(ib)
            tot += 2 ** len(union)
            tens[L + k] = [x for x in ia if x not in ib] + [x for x in ib if x not in ia]
    return tot


@pytest.mark.parametrize("seed", range(6))
def test_eq4_equals_executed_work(seed):
    idx, n, _ = random_network(seed, 7, 10, 2)
    path = pl.greedy_path(idx)
    tree = pl.Tree(idx, path)
    rng = np.random.default_rng(seed)
    S = [int(x) for x in rng.choice(n, size=3, replace=False)]
    assert tree.sliced_cost(S) == _executed_macs(idx, path, S)
    assert tree.sliced_cost([]) == tree.cost() == _executed_macs(idx, path, [])
    assert tree.overhead(S) >= 1.0


@pytest.mark.parametrize("seed", range(4))
def test_halving_doubling_rule(seed):
    """Sec. 3.1: after slicing e, contractions on e's lifetime keep their
    total complexity, every other contraction doubles."""
    idx, n, _ = random_network(seed + 10, 8, 12, 1)
    tree = pl.Tree(idx, pl.greedy_path(idx))
    for e in range(n):
        on = sum(2 ** len(tree.node_set(v)) for v in tree.nodes() if e in tree.node_set(v))
        off = sum(2 ** len(tree.node_set(v)) for v in tree.nodes() if e not in tree.node_set(v))
        assert tree.sliced_cost([e]) == on + 2 * off


def _edges_form_path(tree, tensors):
    """In the paper's tree a tensor is an edge (from the node that makes it
    to the node that consumes it; the root tensor ends at the final scalar
    node). True if the given tensors' edges form one simple path."""
    TOP = -2
    ends = lambda u: (u, tree.parent[u] if tree.parent[u] >= 0 else TOP)
    verts, deg = set(), {}
    for u in tensors:
        a, b = ends(u)
        for x in (a, b):
            verts.add(x)
            deg[x] = deg.get(x, 0) + 1
    if len(tensors) != len(verts) - 1 or max(deg.values()) > 2:
        return False
    adj = {v: set() for v in verts}
    for u in tensors:
        a, b = ends(u)
        adj[a].add(b)
        adj[b].add(a)
    seen, stack = set(), [next(iter(verts))]
    while stack:
        v = stack.pop()
        if v not in seen:
            seen.add(v)
            stack.extend(adj[v] - seen)
    return seen == verts


@pytest.mark.parametrize("name", ["rqc12", "rqc30"])
def test_lifetime_linearity(name):
    """Supplement, Theorem 'Linearity': an index's tensors form one tree
    path from a leaf to another leaf (closed) or to the root (open)."""
    w = make_workload(name)
    net = nw.absorb_small(nw.circuit_network(w.circuit, w.open_qubits, w.closed_bits))
    tree = pl.Tree(net.indices, pl.greedy_path(net.indices))
    for x in range(net.n_indices):
        life = tree.lifetime(x)
        assert _edges_form_path(tree, life)
        leaves = [v for v in life if v < tree.L]
        corr = {v for v in tree.nodes() if x in tree.node_set(v)}
        if x in net.open_ids:
            assert len(leaves) == 1 and tree.root in life
            assert corr == {tree.parent[u] for u in life if u != tree.root}
        else:
            assert len(leaves) == 2 and tree.root not in life
            # the nodes of the path are the correlated contractions
            assert corr == {tree.parent[u] for u in life}


def test_no_overhead_when_lifetimes_span_the_subpath():
    """Sec. 5.2 (secondary slicing): slicing edges whose lifetimes span the
    whole sub-path costs nothing extra and divides the memory; here 5 such
    edges take the largest tensor from 2^8 to 2^3 with 2^5 subtasks."""
    span = [100, 101, 102, 103, 104]
    # a stem absorbing three small tensors; the 5 spanning indices start in
    # leaf 0 and stay open to the end
    leaves = [span + [0, 1, 2], [0, 10], [1, 2, 11], [10, 11]]
    path = [(0, 1), (4, 2), (5, 3)]
    tree = pl.Tree(leaves, path)
    assert tree.space() == 2 ** 8
    assert tree.space(span) == 2 ** 3
    assert tree.sliced_cost(span) == tree.cost()
    assert tree.overhead(span) == 1.0


def test_plain_greedy_hand_example():
    # chain [a] - [a,b] - [b,c] - [c]: every candidate scores -4, ties go to
    # the smallest (lower id, higher id)
    leaves = [[0], [0, 1], [1, 2], [2]]
    assert pl.greedy_path(leaves) == [(0, 1), (2, 3), (4, 5)]
    # disconnected pieces end with outer products of the two lowest ids
    assert pl.greedy_path([[0], [0], [1], [1]]) == [(0, 1), (2, 3), (4, 5)]


def test_stem_of_caterpillar():
    leaves = [[0, 1, 2, 3], [0, 4], [1, 5], [2, 6], [4, 5, 6], [3]]
    path = [(0, 1), (6, 2), (7, 3), (8, 4), (9, 5)]
    tree = pl.Tree(leaves, path)
    assert tree.stem() == [0, 6, 7, 8, 9, 10]


def _min_slicing(tree, n, t):
    for k in range(n + 1):
        for S in itertools.combinations(range(n), k):
            if tree.space(S) <= 2 ** t:
                return k
    return None


@pytest.mark.parametrize("seed", range(25))
def test_slice_finder_vs_brute_force(seed):
    idx, n, _ = random_network(seed, 6, 9, 1)
    tree = pl.Tree(idx, pl.greedy_path(idx))
    W = max(len(s) for s in tree.sets)
    for t in range(max(1, W - 3), W):
        S = pl.slice_finder(tree, t)
        assert len(set(S)) == len(S)
        assert tree.space(S) <= 2 ** t                 # memory constraint (Sec. 4.1)
        assert len(S) >= _min_slicing(tree, n, t)      # never below the optimum
        assert pl.slice_finder(tree, t) == S           # deterministic


def _alg1_cases():
    return json.load(open(os.path.join(GOLDEN, "alg1_stems.json")))["cases"]


@pytest.mark.parametrize("case", _alg1_cases(), ids=lambda c: c["name"])
def test_slice_finder_hand_worked_stems(case):
    """Sec. 4.2, Algorithm 1 on three chains whose slicing sets were worked
    out by hand (the steps are in tests/golden/alg1_stems.json). In the
    first the leaf-side end of the over-cap stem has the smaller rank and
    is fixed first, in the second the root-side end, in the third the two
    ends tie and the root side goes first. Each one's set depends on which
    end is taken and on preferring the index whose lifetime covers the most
    over-cap stem tensors; each reaches the brute-force minimum."""
    tree = pl.Tree(case["leaves"], [tuple(p) for p in case["path"]])
    assert tree.stem() == [0, 6, 7, 8, 9, 10]
    for v, ix in case["node_sets"].items():
        assert tree.sets[int(v)] == frozenset(ix)
    n = 1 + max(x for leaf in case["leaves"] for x in leaf)
    S = pl.slice_finder(tree, case["t"])
    assert S == case["S"]
    assert tree.space(S) <= 2 ** case["t"]
    assert _min_slicing(tree, n, case["t"]) == case["brute_force_min"] == len(S)


def _gap_histogram():
    """|S| of the slice finder minus the smallest |S| meeting the cap, over
    200 random networks (8 tensors, 13 closed and 2 open indices) on their
    greedy trees, at the three caps just below the largest tensor."""
    hist = collections.Counter()
    for seed in range(200):
        idx, n, _ = random_network(seed, 8, 13, 2)
        tree = pl.Tree(idx, pl.greedy_path(idx))
        W = max(len(s) for s in tree.sets)
        for t in range(max(1, W - 3), W):
            hist[len(pl.slice_finder(tree, t)) - _min_slicing(tree, n, t)] += 1
    return hist


def test_slice_finder_gap_to_brute_force():
    """The paper claims a slicing set "as small as possible", not the
    smallest (Sec. 4.2). Measured here: the set is minimal in 386 of 600
    cases, one index above in 188, two above in 26 (never below, never
    more). The assertions keep that quality; an index ranking that prefers
    short lifetimes reaches the minimum in only 26 % of the cases (see
    test_slice_finder_pins_catch_misreadings)."""
    hist = _gap_histogram()
    total = sum(hist.values())
    print("gap histogram", sorted(hist.items()))
    assert min(hist) >= 0
    assert hist[0] / total >= 0.6
    assert sum(g * c for g, c in hist.items()) / total <= 0.45


def test_slice_finder_pins_catch_misreadings(monkeypatch):
    """Three misreadings of Algorithm 1, planted in the oracle, each change
    the slicing set of at least one hand-worked stem: taking the larger
    end first, taking the leaf-side end on a tie, and preferring indices
    with short lifetimes (which also fails the brute-force gap bound)."""
    cases = _alg1_cases()

    def sets():
        return [pl.slice_finder(pl.Tree(c["leaves"], [tuple(p) for p in c["path"]]), c["t"])
                for c in cases]

    want = [c["S"] for c in cases]
    assert sets() == want
    with monkeypatch.context() as m:
        m.setattr(pl, "pick_end", lambda over, rank: over[-1] if rank(over[0]) < rank(over[-1]) else over[0])
        assert sets() != want
    with monkeypatch.context() as m:
        m.setattr(pl, "pick_end", lambda over, rank: over[0] if rank(over[0]) <= rank(over[-1]) else over[-1])
        got = sets()
        assert got != want and got[:2] == want[:2]
    with monkeypatch.context() as m:
        m.setattr(pl, "lifetime_order",
                  lambda cands, span, whole: sorted(cands, key=lambda x: (span[x], -whole[x], x)))
        assert all(g != w for g, w in zip(sets(), want))
        hist = _gap_histogram()
        assert hist[0] / sum(hist.values()) < 0.3


def test_slice_finder_prefix_and_no_cap():
    idx, n, _ = random_network(3, 6, 9, 2)
    tree = pl.Tree(idx, pl.greedy_path(idx))
    assert pl.slice_finder(tree, -1, pre=[4, 2]) == [4, 2]
    S = pl.slice_finder(tree, 2, pre=[4])
    assert S[0] == 4 and tree.space(S) <= 4


def test_keyed_uniform_reference_values():
    # SplitMix64 from state 0 yields 0xE220A8397B1DCDAF (published first
    # output of the generator seeded with 0)
    assert pl.splitmix64(0) == 0xE220A8397B1DCDAF
    u = [pl.keyed_uniform(7, s, 1, 2) for s in range(1000)]
    assert 0.0 <= min(u) and max(u) < 1.0
    assert abs(np.mean(u) - 0.5) < 0.03


def test_randomised_greedy_improves_rqc30():
    w = make_workload("rqc30")
    net = nw.absorb_small(nw.circuit_network(w.circuit, w.open_qubits, w.closed_bits))
    plain = pl.Tree(net.indices, pl.greedy_path(net.indices))
    S0 = pl.slice_finder(plain, 26)
    p, S, trial = pl.path_search(net.indices, 26, alphas=(0.5, 1.0), taus=(0.0, 0.3), n_seeds=3)
    best = pl.Tree(net.indices, p)
    assert best.sliced_cost(S) <= plain.sliced_cost(S0)
    assert best.space(S) <= 2 ** 26
