"""Pins of the oracle's slice refiner (Sec. 4.3, Algorithms 2-4) and of the
greedy least-overhead slicer, against hand-worked cases and brute force.

Hand-worked chain (leaves T0 {0,1}, T1 {1,2,3}, T2 {3,4,5}, T3 {5,6,7},
T4 {7,8}, contracted left to right; open indices 0, 2, 4, 6, 8):
intermediate tensors n5 {0,2,3}, n6 {0,2,4,5}, n7 {0,2,4,6,7}, n8 {0,2,4,6,8};
Eq. (4) node sets s_v: {0,1,2,3}, {0,2,3,4,5}, {0,2,4,5,6,7}, {0,2,4,6,7,8},
so C(B) = 16 + 32 + 64 + 64 = 176. With t = 4 only n7 and n8 are too large.
  * S = {4}: C = 32 + 32 + 64 + 64 = 192; the lifetime of 4 is T2, n6, n7,
    n8 with ranks 2, 3, 4, 4 after slicing, so the critical tensors are n7
    and n8 and the candidates {0,2,4,6,7} n {0,2,4,6,8} minus S = [0, 2, 6];
    C({0}) = C({2}) = 176, C({6}) = 32 + 64 + 64 + 64 = 224. The refiner's
    first move reaches {0}, the optimum, and keeps it as the best seen.
  * S = {0, 7}: the lifetime of 7 is T3, n7 with ranks 2, 3: no critical
    tensor, so 7 is dropped.
  * The greedy slicer compares the indices of n7, n8: {0} and {2} both give
    176 and lie in both tensors, so it takes the smaller id, 0.
"""
import itertools

import pytest

from oracle import planner as opl
from tests.netgen import random_network

CHAIN = [[0, 1], [1, 2, 3], [3, 4, 5], [5, 6, 7], [7, 8]]
CHAIN_PATH = [(0, 1), (5, 2), (6, 3), (7, 4)]


def _chain():
    return opl.Tree(CHAIN, CHAIN_PATH)


def test_chain_costs_and_algorithms_3_4():
    tr = _chain()
    assert tr.cost() == 176
    assert tr.sliced_cost([4]) == 192
    assert tr.sliced_cost([0]) == tr.sliced_cost([2]) == 176
    assert tr.sliced_cost([6]) == 224
    crit = opl.critical_tensors(tr, [4], 4, 4)
    assert crit == [7, 8]
    assert opl.candidate_indices(tr, crit, [4]) == [0, 2, 6]
    assert opl.critical_tensors(tr, [0, 7], 7, 4) == []


def test_chain_refiner_and_greedy_slicer():
    tr = _chain()
    S, st = opl.slice_refine(tr, 4, [4], seed=0)
    assert S == [0]
    assert st["iterations"] == 342  # 0.98^k >= 1e-3 for k = 0..341
    S2, st2 = opl.slice_refine(tr, 4, [0, 7], seed=0)
    assert len(S2) == 1 and tr.sliced_cost(S2) == 176 and st2["dropped"] == 1
    assert opl.greedy_overhead_slicer(tr, 4) == [0]
    # fixed entries never move: with the only slot fixed nothing happens
    S3, st3 = opl.slice_refine(tr, 4, [4], n_fixed=1)
    assert S3 == [4] and st3["proposals"] == 0


def test_input_must_meet_cap():
    tr = _chain()
    with pytest.raises(ValueError):
        opl.slice_refine(tr, 4, [8])  # n7 keeps rank 5


def _brute_min(tree, t, kmax):
    ids = sorted(set().union(*tree.sets))
    best = None
    for k in range(0, kmax + 1):
        for S in itertools.combinations(ids, k):
            if opl.fits(tree, S, t):
                c = tree.sliced_cost(S)
                best = c if best is None or c < best else best
    return best


@pytest.mark.parametrize("seed", range(10))
def test_candidate_swaps_keep_the_cap(seed):
    """Every Algorithm 4 candidate holds all critical tensors of the index it
    replaces, so the swap keeps every tensor within t; an index without
    critical tensors can be dropped. Checked against the cap directly."""
    idx, n, opens = random_network(seed, 9, 14, 2)
    tr = opl.Tree(idx, opl.greedy_path(idx, 1.0, 0.0, seed))
    mx = max(len(s) for s in tr.sets)
    for t in range(max(1, mx - 3), mx):
        S = opl.slice_finder(tr, t)
        for j, a in enumerate(S):
            crit = opl.critical_tensors(tr, S, a, t)
            if not crit:
                assert opl.fits(tr, S[:j] + S[j + 1:], t)
                continue
            cand = opl.candidate_indices(tr, crit, S)
            for c in cand:
                assert opl.fits(tr, S[:j] + [c] + S[j + 1:], t)
            # candidates = unsliced indices whose lifetime contains every
            # critical tensor (the definition in Sec. 4.3)
            want = [b for b in range(n) if b not in S and set(crit) <= set(tr.lifetime(b))]
            assert cand == want


@pytest.mark.parametrize("seed", range(12))
def test_refiner_invariants_and_brute_force(seed):
    idx, n, opens = random_network(seed, 8, 12, 2)
    tr = opl.Tree(idx, opl.greedy_path(idx, 1.0, 0.0, seed))
    mx = max(len(s) for s in tr.sets)
    for t in range(max(1, mx - 3), mx):
        S = opl.slice_finder(tr, t)
        R, st = opl.slice_refine(tr, t, S, seed=seed)
        assert opl.fits(tr, R, t)
        assert len(R) <= len(S) and len(set(R)) == len(R)
        assert tr.sliced_cost(R) <= tr.sliced_cost(S)
        assert tr.sliced_cost(R) >= _brute_min(tr, t, len(S))
        assert opl.slice_refine(tr, t, S, seed=seed) == (R, st)  # deterministic
        G = opl.greedy_overhead_slicer(tr, t)
        assert opl.fits(tr, G, t)
        assert tr.sliced_cost(G) >= _brute_min(tr, t, len(G))
        # the greedy slicer's first pick is the cheapest single index among
        # those of the tensors above t
        big = [s for s in tr.sets if len(s) > t]
        pool = sorted(set().union(*big))
        assert tr.sliced_cost(G[:1]) == min(tr.sliced_cost([x]) for x in pool)


def test_refiner_reaches_brute_force_optimum_mostly():
    """Over small random trees the annealing finds the best set of at most
    |S| indices in most cases (a refiner that never moves, or that moves at
    random, does far worse)."""
    hits = tot = 0
    for seed in range(16):
        idx, n, opens = random_network(seed, 8, 12, 2)
        tr = opl.Tree(idx, opl.greedy_path(idx, 1.0, 0.0, seed))
        mx = max(len(s) for s in tr.sets)
        for t in range(max(1, mx - 2), mx):
            S = opl.slice_finder(tr, t)
            R, _ = opl.slice_refine(tr, t, S, seed=seed)
            tot += 1
            hits += tr.sliced_cost(R) == _brute_min(tr, t, len(S))
    assert hits >= 0.6 * tot, (hits, tot)


# ---------------------------------------------------------------------------
# Subtree reconfiguration


def _all_tree_costs(sets, Sset):
    """Brute force: the cheapest total node cost 2^|s_v - S| over every way
    of contracting the given tensors pairwise (no subset table)."""
    best = None
    items = [frozenset(s) for s in sets]

    def rec(items, acc):
        nonlocal best
        if best is not None and acc >= best:
            return
        if len(items) == 1:
            best = acc
            return
        for i in range(len(items)):
            for j in range(i + 1, len(items)):
                a, b = items[i], items[j]
                c = 1 << len((a | b) - Sset)
                rest = [items[x] for x in range(len(items)) if x not in (i, j)] + [a ^ b]
                rec(rest, acc + c)

    rec(items, 0)
    return best


def _is_ssa_cover(L, path):
    seen = set()
    for k, (a, b) in enumerate(path):
        v = L + k
        if not (0 <= a < v and 0 <= b < v and a != b) or a in seen or b in seen:
            return False
        seen.update((a, b))
    return len(path) == L - 1


@pytest.mark.parametrize("seed", range(8))
def test_reconfigure_whole_tree_is_optimal_on_tiny_networks(seed):
    """With k >= number of leaves the root's frontier is every leaf, so one
    sweep must reach the cheapest contraction order (brute force over all
    pairwise orders)."""
    idx, n, opens = random_network(seed, 6, 8, 2)
    p = opl.greedy_path(idx, 1.0, 0.0, seed)
    p2 = opl.reconfigure(idx, p, k=6, sweeps=1)
    assert _is_ssa_cover(len(idx), p2)
    assert opl.Tree(idx, p2).cost() == _all_tree_costs(idx, frozenset())
    # with a slicing set the sliced node costs are minimised instead
    S = [0, 3]
    p3 = opl.reconfigure(idx, p, k=6, sweeps=1, S=S)
    assert opl.Tree(idx, p3).sliced_cost(S) == _all_tree_costs(idx, frozenset(S)) * 4


@pytest.mark.parametrize("seed", range(8))
def test_reconfigure_invariants(seed):
    idx, n, opens = random_network(seed, 14, 24, 3)
    p = opl.greedy_path(idx, 0.5, 1.0, seed)
    tr = opl.Tree(idx, p)
    for k in (3, 5, 7):
        p2 = opl.reconfigure(idx, p, k, sweeps=3)
        tr2 = opl.Tree(idx, p2)
        assert _is_ssa_cover(len(idx), p2)
        assert tr2.sets[tr2.root] == tr.sets[tr.root]  # same output indices
        assert tr2.cost() <= tr.cost()
        mx = max(len(s) for s in tr2.sets)
        t = max(1, mx - 2)
        S = opl.slice_finder(tr2, t)
        p3 = opl.reconfigure(idx, p2, k, sweeps=3, S=S, t=t)
        tr3 = opl.Tree(idx, p3)
        assert opl.fits(tr3, S, t)
        assert tr3.sliced_cost(S) <= tr2.sliced_cost(S)
